/*
 * gv_oracle.c -- plain CPU FP64 reference for the general-voting
 * maximum-depth search (Aiger et al., ICCV 2021, Sec. 3.2, Alg. 2).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  It shares no code
 * with the HIP library.  Build: gcc -O2 -ffp-contract=off -fPIC -shared.
 *
 * What it computes (each step cites the paper):
 *   - Surfaces in parametric form x_q = F_q(x_P; t) + f_q in the unit cube
 *     (Sec. 3, Eq. 1).  Families: 2D line fitting by duality (Eq. 2),
 *     hyperplanes in 3-space (Eq. 3), rays in 3-space (Sec. 4.3, the
 *     two-equation line form, generalized to the dominant axis), and the
 *     known-gravity calibrated pose (the 5DoF surface of Sec. 4.2.1 with
 *     focal length 1), the known-gravity pose with unknown focal length
 *     (the 5DoF surface of Sec. 4.2.1 itself, axes x, y, z, kappa, f), and
 *     similarity alignment of planar point sets (Sec. 4.4, the translation
 *     written in terms of scale-rotation).
 *   - Canonization (Sec. 3.2.1): translate to the cell's minimum corner,
 *     round essential parameters to eps'/((l+1) delta) and free parameters
 *     to eps'/(l+1), group equal results and keep their multiplicity.
 *   - Alg. 2: recursive 2^a subdivision, keep the surfaces that meet each
 *     child, stop when every side is at most eps, return the argmax.
 *     Pruning against the best leaf found so far (the Branch&Bound remark at
 *     the end of Sec. 3.3) never changes the result because counts only
 *     shrink down the tree.
 *   - Inliers: the original surfaces whose canonization chain reaches the
 *     chosen leaf (member tracking, Sec. 3.2.1).
 *
 * Parity pins: none of this code is checked against itself; see tests/.
 */
#include "gv_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define MAXD OR_MAXD
#define MAXL 48

typedef struct {
  /* linear: t[q][i] at p[2q+i], f[q] at p[4+q]; pose: W1,W2,W3,xi,eta,0 */
  double p[6];
  int32_t tag;
  uint32_t w;
} rec;

typedef struct {
  const or_problem *prob;
  int fam, d, ell, exact;
  double c;
  double lo[MAXD], E[MAXD], inv[MAXD], epsn[MAXD];
  int L[MAXD], Lstar, B, Bcell;
  int abits[MAXL + 1], rem[MAXL + 2];
  /* linear families */
  double sf[MAXD];
  double pad[MAXL][MAXD];
  /* pose */
  double sW, sW3, sXi, sEta, Rg2, padz, padk, epsk, ce;
  /* 5DoF: the f axis in user units (f > 0) and a bound on f over the box */
  double flo, Ef, Fb;
  /* search state */
  uint64_t best;
  uint64_t *shared_best; /* thread pool: one best key for every worker */
  uint64_t tests, expanded, pruned, merged, budget;
  /* threshold reporting: the best key stays at tau 2^B - 1, so a cell is
   * pruned exactly when its count is below tau; every leaf that reaches
   * tau is recorded instead of raising the best key */
  int report;
  uint64_t *rep_idx;
  uint32_t *rep_cnt;
  int64_t rep_cap, rep_n;
} ctx;

/* Best key so far.  With a thread pool every worker reads and raises one
 * shared value; it only tightens pruning, never changes the result, because
 * a leaf's key is unique (count, then lowest index). */
static uint64_t best_get(const ctx *C) {
  return C->shared_best ? __atomic_load_n(C->shared_best, __ATOMIC_RELAXED) : C->best;
}

static void best_offer(ctx *C, uint64_t key) {
  if (!C->shared_best) {
    if (key > C->best) C->best = key;
    return;
  }
  uint64_t cur = __atomic_load_n(C->shared_best, __ATOMIC_RELAXED);
  while (key > cur &&
         !__atomic_compare_exchange_n(C->shared_best, &cur, key, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
  }
}

const char *or_status_str(int st) {
  switch (st) {
    case OR_OK: return "ok";
    case OR_EINVAL: return "invalid argument";
    case OR_ENOMEM: return "out of memory";
    case OR_EBUFSZ: return "inlier buffer too small";
    case OR_ERANGE: return "lattice too fine for exact binary64 arithmetic";
    case OR_EBUDGET: return "test budget exhausted";
  }
  return "unknown status";
}

/* largest power of two <= x (x > 0, finite) */
static double p2floor(double x) {
  int e;
  (void)frexp(x, &e); /* x = m * 2^e, m in [0.5, 1) */
  return ldexp(1.0, e - 1);
}

static int imin(int a, int b) { return a < b ? a : b; }

/* the two camera-posing families share sectors, lattice and predicate */
static int is_pose(const ctx *C) { return C->fam == OR_POSE4DOF || C->fam == OR_POSE5DOF; }

/* side of axis j at level m in the unit cube: 2^-min(m, L_j) */
static double side(const ctx *C, int j, int m) { return ldexp(1.0, -imin(m, C->L[j])); }

static void lin_axes(const ctx *C, int tag, int *nP, int P[2], int *nQ, int Q[2]) {
  if (C->fam == OR_LINE2D) {
    *nP = 1; P[0] = 0; *nQ = 1; Q[0] = 1;
  } else if (C->fam == OR_PLANE3D) {
    *nP = 2; P[0] = 0; P[1] = 1; *nQ = 1; Q[0] = 2;
  } else if (C->fam == OR_SIM2D) {
    *nP = 2; P[0] = 0; P[1] = 1; *nQ = 2; Q[0] = 2; Q[1] = 3;
  } else { /* RAY3D: parameter axis = tag, dependents ascending */
    int k = 0;
    *nP = 1; P[0] = tag; *nQ = 2;
    for (int j = 0; j < 3; j++)
      if (j != tag) Q[k++] = j;
  }
}

/* ------------------------------------------------------------------ */
/* Set-up: axes, levels, lattice steps, pads (normalization w.l.o.g. to  */
/* the unit cube, Sec. 3; per-coordinate eps, Sec. 3.2).                 */
/* ------------------------------------------------------------------ */
static int ctx_init(ctx *C, const or_problem *p) {
  memset(C, 0, sizeof(*C));
  C->prob = p;
  C->fam = p->family;
  if (p->n < 0 || p->n > 0x7fffffffLL) return OR_EINVAL;
  switch (C->fam) {
    case OR_LINE2D: C->d = 2; C->ell = 1; break;
    case OR_PLANE3D: C->d = 3; C->ell = 2; break;
    case OR_RAY3D: C->d = 3; C->ell = 2; break;
    case OR_POSE4DOF: C->d = 4; C->ell = 4; break;
    case OR_POSE5DOF: C->d = 5; C->ell = 4; break;
    case OR_SIM2D: C->d = 4; C->ell = 2; break;
    default: return OR_EINVAL;
  }
  C->c = p->canon_c == 0.0 ? 1.0 : p->canon_c;
  if (!(C->c > 0.0) || isnan(C->c)) return OR_EINVAL;
  C->exact = isinf(C->c) ? 1 : 0;

  /* axes given in user units: all but kappa for the pose families */
  for (int j = 0; j < C->d; j++) {
    if (is_pose(C) && j == 3) continue;
    if (!isfinite(p->lo[j]) || !isfinite(p->hi[j]) || !(p->hi[j] > p->lo[j])) return OR_EINVAL;
    if (!isfinite(p->eps[j]) || !(p->eps[j] > 0.0)) return OR_EINVAL;
    C->lo[j] = p->lo[j];
    C->E[j] = p->hi[j] - p->lo[j];
    C->inv[j] = 1.0 / C->E[j];
    C->epsn[j] = p->eps[j] * C->inv[j];
  }
  if (is_pose(C)) {
    /* x and y share one scale so that horizontal distances stay Euclidean */
    if (C->E[0] != C->E[1]) return OR_EINVAL;
    if (!isfinite(p->eps[3]) || !(p->eps[3] > 0.0)) return OR_EINVAL;
    /* kappa axis: tan of the yaw offset inside one sector, fixed [-1, 1] */
    C->lo[3] = -1.0; C->E[3] = 2.0; C->inv[3] = 0.5;
    C->epsk = p->eps[3];
    C->epsn[3] = C->epsk * 0.5;
    /* f: the factor of the image coordinates in the direction tangents,
     * positive over the box; 4DoF is the case f = 1 */
    C->flo = 1.0; C->Ef = 0.0; C->Fb = 1.0;
    if (C->fam == OR_POSE5DOF) {
      if (!(p->lo[4] > 0.0)) return OR_EINVAL;
      C->flo = p->lo[4];
      C->Ef = C->E[4];
      C->Fb = p->hi[4] * (1.0 + 0x1p-20);
    }
  }
  /* L_j: smallest L >= 0 with E_j 2^-L <= eps_j (leaf sides at most eps) */
  int Lstar = 0, Bcell = 0;
  for (int j = 0; j < C->d; j++) {
    double ej = (is_pose(C) && j == 3) ? C->epsk : p->eps[j];
    int L = 0;
    while (ldexp(C->E[j], -L) > ej) {
      L++;
      if (L > 40) return OR_EINVAL;
    }
    C->L[j] = L;
    if (L > Lstar) Lstar = L;
    Bcell += L;
  }
  if (Lstar < 1) return OR_EINVAL; /* the root alone would already be a leaf */
  C->Lstar = Lstar;
  C->Bcell = Bcell;
  C->B = Bcell + (is_pose(C) ? 2 : 0);
  if (C->B > 62) return OR_EINVAL;
  /* key = count * 2^B + low bits must fit 64 bits */
  if ((uint64_t)p->n >= (1ULL << (64 - C->B))) return OR_EINVAL;
  for (int m = 0; m < Lstar; m++) {
    int a = 0;
    for (int j = 0; j < C->d; j++)
      if (m < C->L[j]) a++;
    C->abits[m] = a;
  }
  C->rem[Lstar] = 0;
  for (int m = Lstar - 1; m >= 0; m--) C->rem[m] = C->rem[m + 1] + C->abits[m];

  if (!is_pose(C)) {
    /* free step: largest power of two <= eps'/(l+1), eps' = eps/(c(L*+1));
     * essential step at level m: free step * 2^min(m, L_P) = eps'/((l+1) delta) */
    for (int q = 0; q < C->d; q++) {
      if (C->exact) {
        C->sf[q] = ldexp(1.0, -36);
      } else {
        double ep = C->epsn[q] / (C->c * (double)(Lstar + 1));
        C->sf[q] = p2floor(ep / (double)(C->ell + 1));
      }
      if (!(C->sf[q] > 0.0)) return OR_EINVAL;
      for (int m = 0; m < Lstar; m++) {
        /* accumulated canonization deviation after levels 0..m */
        double Em = C->exact ? 0.0 : (double)((m + 1) * (C->ell + 1)) * C->sf[q] * 0.5;
        C->pad[m][q] = ceil((C->epsn[q] + Em) / C->sf[q]) * C->sf[q];
      }
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Front end: observation -> normalized surface parameters (Eq. 1-3,    */
/* Sec. 4.2.1, Sec. 4.3).                                               */
/* ------------------------------------------------------------------ */
static int front(const ctx *C, int64_t i, rec *r) {
  const or_problem *p = C->prob;
  memset(r, 0, sizeof(*r));
  r->w = 1;
  for (int k = 0; k < (C->fam == OR_RAY3D ? 6 : is_pose(C) ? 5 : C->d); k++)
    if (!isfinite(p->col[k][i])) return OR_EINVAL;
  if (C->fam == OR_LINE2D) {
    /* point (x, y) -> dual line b = y - x a (vertical distance preserved) */
    double x = p->col[0][i], y = p->col[1][i];
    r->p[0] = -((x * C->E[0]) * C->inv[1]);
    r->p[4] = ((y - x * C->lo[0]) - C->lo[1]) * C->inv[1];
  } else if (C->fam == OR_PLANE3D) {
    /* point (x, y, z) -> dual plane a0 = z - x a1 - y a2 */
    double x = p->col[0][i], y = p->col[1][i], z = p->col[2][i];
    r->p[0] = -((x * C->E[0]) * C->inv[2]);
    r->p[1] = -((y * C->E[1]) * C->inv[2]);
    r->p[4] = (((z - x * C->lo[0]) - y * C->lo[1]) - C->lo[2]) * C->inv[2];
  } else if (C->fam == OR_SIM2D) {
    /* correspondence p -> q under q_x = a p_x + b p_y + c, q_y = -b p_x +
     * a p_y + d: the translation as a function of (a, b),
     * c = q_x - a p_x - b p_y,  d = q_y + b p_x - a p_y */
    double px = p->col[0][i], py = p->col[1][i], qx = p->col[2][i], qy = p->col[3][i];
    r->p[0] = -((px * C->E[0]) * C->inv[2]);
    r->p[1] = -((py * C->E[1]) * C->inv[2]);
    r->p[4] = (((qx - px * C->lo[0]) - py * C->lo[1]) - C->lo[2]) * C->inv[2];
    r->p[2] = -((py * C->E[0]) * C->inv[3]);
    r->p[3] = (px * C->E[1]) * C->inv[3];
    r->p[5] = (((qy - py * C->lo[0]) + px * C->lo[1]) - C->lo[3]) * C->inv[3];
  } else if (C->fam == OR_RAY3D) {
    /* ray w + s u -> x_q = w_q + (u_q/u_pi)(x_pi - w_pi), pi the dominant axis */
    double w[3], u[3];
    for (int k = 0; k < 3; k++) { w[k] = p->col[k][i]; u[k] = p->col[3 + k][i]; }
    int pi = 0;
    for (int k = 1; k < 3; k++)
      if (fabs(u[k]) > fabs(u[pi])) pi = k;
    if (u[pi] == 0.0) return OR_EINVAL;
    r->tag = pi;
    int qi = 0;
    for (int q = 0; q < 3; q++) {
      if (q == pi) continue;
      double s = u[q] / u[pi];
      r->p[2 * qi] = (s * C->E[pi]) * C->inv[q];
      r->p[4 + qi] = ((w[q] - C->lo[q]) + s * (C->lo[pi] - w[pi])) * C->inv[q];
      qi++;
    }
  } else {
    /* correspondence (w, xi, eta) in normalized units; eta is the elevation
     * tangent so that z = w3 - eta * horizontal distance */
    r->p[0] = (p->col[0][i] - C->lo[0]) * C->inv[0];
    r->p[1] = (p->col[1][i] - C->lo[1]) * C->inv[1];
    r->p[2] = (p->col[2][i] - C->lo[2]) * C->inv[2];
    r->p[3] = p->col[3][i];
    r->p[4] = p->col[4][i] * C->ce;
  }
  return OR_OK;
}

/* Pose lattice: needs data bounds, so it runs after the front end.  The
 * steps are chosen so that rounding one parameter by half a step moves z and
 * kappa by at most eps'/(2(l+1)) anywhere on the box, from bounds on the
 * derivatives of z = W3 - eta' f r and kappa = tan(phi - atan(xi f)):
 * |dz/dW3| = 1, |dz/deta'| <= f R, |dz/dW| <= |eta'| f, |dkappa/dxi| <=
 * (1 + kappa^2) f, |dkappa/dW| <= (1 + kappa^2) / r with r >= R_g. */
static int pose_lattice(ctx *C) {
  const or_problem *p = C->prob;
  C->ce = C->E[0] * C->inv[2];
  double Hmax = 0.0, R2 = 0.0, Xmax = 0.0;
  for (int64_t i = 0; i < p->n; i++) {
    rec r;
    int st = front(C, i, &r);
    if (st) return st;
    double h = fabs(r.p[4]);
    if (h > Hmax) Hmax = h;
    if (fabs(r.p[3]) > Xmax) Xmax = fabs(r.p[3]);
    double a0 = r.p[0] * r.p[0], a1 = (r.p[0] - 1.0) * (r.p[0] - 1.0);
    double b0 = r.p[1] * r.p[1], b1 = (r.p[1] - 1.0) * (r.p[1] - 1.0);
    double r2 = (a0 > a1 ? a0 : a1) + (b0 > b1 ? b0 : b1);
    if (r2 > R2) R2 = r2;
  }
  /* 5DoF: the directions with kappa in a cell's widened interval, over the
   * cell's f interval, form one arc of angle at most 2 atan(1 + padk) +
   * atan(|xi| f_hi), padk <= 2 eps_kappa; the arc test needs it below pi */
  if (C->fam == OR_POSE5DOF && !(2.0 * atan(1.0 + 2.0 * C->epsk) + atan(Xmax * p->hi[4]) < 3.1)) return OR_EINVAL;
  int Lxy = C->L[0] > C->L[1] ? C->L[0] : C->L[1];
  double Rg = ldexp(1.0, -Lxy); /* apex guard: one leaf xy side */
  C->Rg2 = Rg * Rg;
  if (C->exact) {
    C->sW = C->sW3 = C->sXi = C->sEta = ldexp(1.0, -36);
    C->padz = ceil(C->epsn[2] / C->sW3) * C->sW3;
    C->padk = ceil(C->epsk / C->sXi) * C->sXi;
    return OR_OK;
  }
  double l1 = (double)(C->ell + 1);
  double ez = C->epsn[2] / (C->c * (double)(C->Lstar + 1));
  double ek = C->epsk / (C->c * (double)(C->Lstar + 1));
  double Hb = (Hmax > 0x1p-10 ? Hmax : 0x1p-10) * (1.0 + 0x1p-20);
  double Rb = (sqrt(R2) + 0x1p-20) * (1.0 + 0x1p-20);
  double pk0 = C->epsk + ek * 0.5;
  double Bk = 1.0 + (1.0 + pk0) * (1.0 + pk0); /* bound on 1 + kappa^2 */
  C->sW3 = p2floor(ez / l1);
  C->sEta = p2floor(ez / (l1 * Rb * C->Fb));
  double wz = ez / (l1 * Hb * C->Fb), wk = (ek * Rg) / (l1 * Bk);
  C->sW = p2floor(wz < wk ? wz : wk);
  C->sXi = p2floor(ek / (l1 * Bk * C->Fb));
  C->padz = ceil((C->epsn[2] + ez * 0.5) / C->sW3) * C->sW3;
  C->padk = ceil((C->epsk + ek * 0.5) / C->sXi) * C->sXi;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Canonization (Sec. 3.2.1).                                           */
/* ------------------------------------------------------------------ */
static void canon(const ctx *C, rec *r, int m, const int32_t *cc) {
  if (is_pose(C)) {
    /* fixed global lattice, applied once at the root */
    if (m != 0) return;
    r->p[0] = nearbyint(r->p[0] / C->sW) * C->sW;
    r->p[1] = nearbyint(r->p[1] / C->sW) * C->sW;
    r->p[2] = nearbyint(r->p[2] / C->sW3) * C->sW3;
    r->p[3] = nearbyint(r->p[3] / C->sXi) * C->sXi;
    r->p[4] = nearbyint(r->p[4] / C->sEta) * C->sEta;
    r->p[5] = 0.0;
    return;
  }
  if (C->exact && m != 0) return; /* exact mode: quantize once */
  int nP, P[2], nQ, Q[2];
  lin_axes(C, r->tag, &nP, P, &nQ, Q);
  double u[MAXD];
  for (int j = 0; j < C->d; j++) u[j] = (double)cc[j] * side(C, j, m);
  for (int qi = 0; qi < nQ; qi++) {
    int q = Q[qi];
    double sf = C->sf[q];
    /* 1. translate: value at the cell's min corner, relative to its q floor */
    double floc = r->p[4 + qi];
    for (int k = 0; k < nP; k++) floc = floc + r->p[2 * qi + k] * u[P[k]];
    floc = floc - u[q];
    /* 2. round each essential parameter to sf * 2^min(m, L_P) */
    double tn[2];
    for (int k = 0; k < nP; k++) {
      double st = ldexp(sf, imin(m, C->L[P[k]]));
      tn[k] = nearbyint(r->p[2 * qi + k] / st) * st;
    }
    /* 3. round the translated free parameter to sf */
    double fl = nearbyint(floc / sf) * sf;
    /* 4. translate back */
    double fn = fl;
    for (int k = 0; k < nP; k++) fn = fn - tn[k] * u[P[k]];
    fn = fn + u[q];
    for (int k = 0; k < nP; k++) r->p[2 * qi + k] = tn[k];
    r->p[4 + qi] = fn;
  }
}

/* ------------------------------------------------------------------ */
/* Surface / box predicate (Sec. 3.2.1 "two functions"; the subset of   */
/* conditions of the Surface-Box paragraph: one interval test per      */
/* dependent axis).  Surface canonized at level m, cell at level m+1.  */
/* ------------------------------------------------------------------ */
static double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

static int meets_pose(const ctx *C, const rec *r, int m1, int sector, const int32_t *cc) {
  double hx = side(C, 0, m1), hy = side(C, 1, m1), hz = side(C, 2, m1), hk = side(C, 3, m1);
  /* f interval of the cell in user units (4DoF: f = 1) */
  double Fl = 1.0, Fh = 1.0;
  if (C->fam == OR_POSE5DOF) {
    double hf = side(C, 4, m1);
    Fl = C->flo + C->Ef * ((double)cc[4] * hf);
    Fh = C->flo + C->Ef * ((double)(cc[4] + 1) * hf);
  }
  double Xlo = (double)cc[0] * hx, Xhi = (double)(cc[0] + 1) * hx;
  double Ylo = (double)cc[1] * hy, Yhi = (double)(cc[1] + 1) * hy;
  double Zlo = (double)cc[2] * hz, Zhi = (double)(cc[2] + 1) * hz;
  double Klo = 2.0 * ((double)cc[3] * hk) - 1.0, Khi = 2.0 * ((double)(cc[3] + 1) * hk) - 1.0;
  double W1 = r->p[0], W2 = r->p[1], W3 = r->p[2], xi = r->p[3], eta = r->p[4];
  double Alo = W1 - Xhi, Ahi = W1 - Xlo, Blo = W2 - Yhi, Bhi = W2 - Ylo;
  double x0, x1, y0, y1; /* V = Rot_s(box of (W1 - X, W2 - Y)) */
  switch (sector) {
    case 0: x0 = Alo; x1 = Ahi; y0 = Blo; y1 = Bhi; break;
    case 1: x0 = Blo; x1 = Bhi; y0 = -Ahi; y1 = -Alo; break;
    case 2: x0 = -Ahi; x1 = -Alo; y0 = -Bhi; y1 = -Blo; break;
    default: x0 = -Bhi; x1 = -Blo; y0 = Alo; y1 = Ahi; break;
  }
  /* z = W3 - eta f |v| over V and the f interval: |v| spans [r_min, r_max],
   * |eta| f spans [|eta| Fl, |eta| Fh] */
  double dx = x0 > 0.0 ? x0 : (x1 < 0.0 ? -x1 : 0.0);
  double dy = y0 > 0.0 ? y0 : (y1 < 0.0 ? -y1 : 0.0);
  double rmin2 = dx * dx + dy * dy;
  double mx0 = x0 * x0, mx1 = x1 * x1, my0 = y0 * y0, my1 = y1 * y1;
  double rmax2 = (mx0 > mx1 ? mx0 : mx1) + (my0 > my1 ? my0 : my1);
  double Glo = W3 - (Zhi + C->padz), Ghi = W3 - (Zlo - C->padz);
  double Tlo, Thi, a;
  if (eta >= 0.0) { Tlo = Glo; Thi = Ghi; a = eta; }
  else { Tlo = -Ghi; Thi = -Glo; a = -eta; }
  double ah = a * Fh, al = a * Fl;
  int zlo_ok = (Tlo <= 0.0) || ((ah * ah) * rmax2 >= Tlo * Tlo); /* a Fh r_max >= Tlo */
  int zhi_ok = (Thi >= 0.0) && ((al * al) * rmin2 <= Thi * Thi); /* a Fl r_min <= Thi */
  if (!(zlo_ok && zhi_ok)) return 0;
  /* kappa = (v2 - t v1)/(v1 + t v2) with v1 + t v2 > 0 and t = xi f, over V
   * and the f interval: the directions form the arc from the one with kappa
   * = Llo at the smallest t counter-clockwise to the one with kappa = Lhi at
   * the largest t */
  if (rmin2 < C->Rg2) return 1; /* apex guard: kappa unbounded near the apex */
  double Llo = Klo - C->padk, Lhi = Khi + C->padk;
  double t1 = xi * Fl, t2 = xi * Fh;
  double tl = t1 < t2 ? t1 : t2, th = t1 < t2 ? t2 : t1;
  double elx = 1.0 - Llo * tl, ely = Llo + tl; /* direction with kappa = Llo at t = tl */
  double ehx = 1.0 - Lhi * th, ehy = Lhi + th; /* direction with kappa = Lhi at t = th */
  double ax, ay, bx, by; /* silhouette corners: V's angular span from a CCW to b */
  if (x0 > 0.0) {
    if (y0 > 0.0) { ax = x1; ay = y0; bx = x0; by = y1; }
    else if (y1 < 0.0) { ax = x0; ay = y0; bx = x1; by = y1; }
    else { ax = x0; ay = y0; bx = x0; by = y1; }
  } else if (x1 < 0.0) {
    if (y0 > 0.0) { ax = x1; ay = y1; bx = x0; by = y0; }
    else if (y1 < 0.0) { ax = x0; ay = y1; bx = x1; by = y0; }
    else { ax = x1; ay = y1; bx = x1; by = y0; }
  } else {
    if (y0 > 0.0) { ax = x1; ay = y0; bx = x0; by = y0; }
    else if (y1 < 0.0) { ax = x0; ay = y1; bx = x1; by = y1; }
    else return 1; /* apex inside V (not reachable: r_min >= R_g > 0) */
  }
  /* two arcs shorter than pi meet iff one holds an endpoint of the other */
  if (cross2(elx, ely, ax, ay) >= 0.0 && cross2(ax, ay, ehx, ehy) >= 0.0) return 1;
  if (cross2(elx, ely, bx, by) >= 0.0 && cross2(bx, by, ehx, ehy) >= 0.0) return 1;
  if (cross2(ax, ay, elx, ely) >= 0.0 && cross2(elx, ely, bx, by) >= 0.0) return 1;
  if (cross2(ax, ay, ehx, ehy) >= 0.0 && cross2(ehx, ehy, bx, by) >= 0.0) return 1;
  return 0;
}

static int meets(const ctx *C, const rec *r, int m, int sector, const int32_t *cc) {
  int m1 = m + 1;
  if (is_pose(C)) return meets_pose(C, r, m1, sector, cc);
  int nP, P[2], nQ, Q[2];
  lin_axes(C, r->tag, &nP, P, &nQ, Q);
  for (int qi = 0; qi < nQ; qi++) {
    int q = Q[qi];
    double gmin = r->p[4 + qi], gmax = r->p[4 + qi];
    for (int k = 0; k < nP; k++) {
      int j = P[k];
      double h = side(C, j, m1);
      double lo = (double)cc[j] * h, hi = (double)(cc[j] + 1) * h;
      double a = r->p[2 * qi + k] * lo, b = r->p[2 * qi + k] * hi;
      gmin = gmin + (a < b ? a : b);
      gmax = gmax + (a < b ? b : a);
    }
    double h = side(C, q, m1);
    double clo = (double)cc[q] * h, chi = (double)(cc[q] + 1) * h;
    if (gmax < clo - C->pad[m][q]) return 0;
    if (gmin > chi + C->pad[m][q]) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------ */
/* Grouping: equal canonical surfaces merge, multiplicities add.        */
/* ------------------------------------------------------------------ */
static int rec_cmp(const void *a, const void *b) {
  const rec *x = (const rec *)a, *y = (const rec *)b;
  if (x->tag != y->tag) return x->tag < y->tag ? -1 : 1;
  for (int k = 0; k < 6; k++)
    if (x->p[k] != y->p[k]) return x->p[k] < y->p[k] ? -1 : 1;
  return 0;
}

static int64_t group(ctx *C, rec *S, int64_t n) {
  if (C->prob->no_group || n < 2) return n;
  qsort(S, (size_t)n, sizeof(rec), rec_cmp);
  int64_t k = 0;
  for (int64_t i = 1; i < n; i++) {
    if (rec_cmp(&S[k], &S[i]) == 0) {
      S[k].w += S[i].w;
      C->merged++;
    } else {
      S[++k] = S[i];
    }
  }
  return k + 1;
}

/* ------------------------------------------------------------------ */
/* Cell tree: child digits in axis order, MSB first; leaf index =       */
/* [sector] || digits of levels 0..L*-1.                                */
/* ------------------------------------------------------------------ */
static void child_coords(const ctx *C, int m, const int32_t *cc, int digit, int32_t *out) {
  int a = C->abits[m], k = 0;
  for (int j = 0; j < C->d; j++) {
    if (m < C->L[j]) {
      int b = (digit >> (a - 1 - k)) & 1;
      out[j] = 2 * cc[j] + b;
      k++;
    } else {
      out[j] = cc[j];
    }
  }
}

static uint64_t key_of(const ctx *C, uint64_t count, uint64_t idx) {
  uint64_t mask = (C->B == 64) ? ~0ULL : ((1ULL << C->B) - 1ULL);
  return (count << C->B) | (mask - idx);
}

/* filter S against one child; returns count, writes survivors */
static uint64_t filter(ctx *C, const rec *S, int64_t n, int m, int sector, const int32_t *child,
                       rec *out, int64_t *nout) {
  uint64_t cnt = 0;
  int64_t k = 0;
  for (int64_t i = 0; i < n; i++) {
    C->tests++;
    if (meets(C, &S[i], m, sector, child)) {
      cnt += S[i].w;
      if (out) out[k] = S[i];
      k++;
    }
  }
  if (nout) *nout = k;
  return cnt;
}

/* Alg. 2 with pruning: depth-first over children in index order. */
static int expand(ctx *C, int m, int sector, const int32_t *cc, uint64_t prefix, const rec *S,
                  int64_t n) {
  int a = C->abits[m];
  C->expanded++;
  rec *buf = (rec *)malloc(sizeof(rec) * (size_t)(n > 0 ? n : 1));
  if (!buf) return OR_ENOMEM;
  for (int digit = 0; digit < (1 << a); digit++) {
    if (C->budget && C->tests > C->budget) { free(buf); return OR_EBUDGET; }
    int32_t ch[MAXD];
    child_coords(C, m, cc, digit, ch);
    int64_t nc;
    uint64_t cnt = filter(C, S, n, m, sector, ch, buf, &nc);
    uint64_t cpre = (prefix << a) | (uint64_t)digit;
    uint64_t key = key_of(C, cnt, cpre << C->rem[m + 1]);
    if (!C->prob->no_prune && key <= best_get(C)) { C->pruned++; continue; }
    if (m + 1 == C->Lstar) {
      if (C->report) {
        if (C->rep_n < C->rep_cap) {
          C->rep_idx[C->rep_n] = cpre;
          C->rep_cnt[C->rep_n] = (uint32_t)cnt;
        }
        C->rep_n++;
      } else {
        best_offer(C, key);
      }
      continue;
    }
    for (int64_t i = 0; i < nc; i++) canon(C, &buf[i], m + 1, ch);
    nc = group(C, buf, nc);
    int st = expand(C, m + 1, sector, ch, cpre, buf, nc);
    if (st) { free(buf); return st; }
  }
  free(buf);
  return OR_OK;
}

/* Greedy dive: follow the best child (count, then lowest index) to a leaf;
 * its key is an achieved leaf key, hence a valid starting lower bound. */
static int dive(ctx *C, int sector, const rec *S0, int64_t n0) {
  rec *cur = (rec *)malloc(sizeof(rec) * (size_t)(n0 > 0 ? n0 : 1));
  rec *nxt = (rec *)malloc(sizeof(rec) * (size_t)(n0 > 0 ? n0 : 1));
  if (!cur || !nxt) { free(cur); free(nxt); return OR_ENOMEM; }
  memcpy(cur, S0, sizeof(rec) * (size_t)n0);
  int64_t n = n0;
  int32_t cc[MAXD] = {0};
  uint64_t prefix = (uint64_t)sector;
  for (int m = 0; m < C->Lstar; m++) {
    int a = C->abits[m], bestd = 0;
    uint64_t bestc = 0;
    for (int digit = 0; digit < (1 << a); digit++) {
      int32_t ch[MAXD];
      child_coords(C, m, cc, digit, ch);
      uint64_t cnt = filter(C, cur, n, m, sector, ch, NULL, NULL);
      if (digit == 0 || cnt > bestc) { bestc = cnt; bestd = digit; }
    }
    int32_t ch[MAXD];
    child_coords(C, m, cc, bestd, ch);
    int64_t nc;
    filter(C, cur, n, m, sector, ch, nxt, &nc);
    prefix = (prefix << a) | (uint64_t)bestd;
    memcpy(cc, ch, sizeof(cc));
    if (m + 1 < C->Lstar) {
      for (int64_t i = 0; i < nc; i++) canon(C, &nxt[i], m + 1, ch);
      nc = group(C, nxt, nc);
    }
    rec *t = cur; cur = nxt; nxt = t;
    n = nc;
    if (m + 1 == C->Lstar) {
      best_offer(C, key_of(C, bestc, prefix));
    }
  }
  free(cur);
  free(nxt);
  return OR_OK;
}

/* decode a leaf index into the per-level path of cell coordinates */
static int leaf_path(const ctx *C, uint64_t idx, int *sector, int32_t path[][MAXD]) {
  if (C->B < 64 && idx >= (1ULL << C->B)) return OR_EINVAL;
  *sector = is_pose(C) ? (int)(idx >> C->Bcell) : 0;
  for (int j = 0; j < MAXD; j++) path[0][j] = 0;
  for (int m = 0; m < C->Lstar; m++) {
    int a = C->abits[m];
    int digit = (int)((idx >> C->rem[m + 1]) & ((1ULL << a) - 1ULL));
    child_coords(C, m, path[m], digit, path[m + 1]);
  }
  return OR_OK;
}

/* Path of cell coordinates from the root to the level-`level` cell whose
 * index is [sector] || the child digits of levels 0..level-1. */
static void cell_path(const ctx *C, uint64_t idx, int level, int *sector, int32_t path[][MAXD]) {
  int bits = 0;
  for (int m = 0; m < level; m++) bits += C->abits[m];
  *sector = is_pose(C) ? (int)(idx >> bits) : 0;
  for (int j = 0; j < MAXD; j++) path[0][j] = 0;
  int rem = bits;
  for (int m = 0; m < level; m++) {
    int a = C->abits[m];
    rem -= a;
    int digit = (int)((idx >> rem) & ((1ULL << a) - 1ULL));
    child_coords(C, m, path[m], digit, path[m + 1]);
  }
}

/* per-surface chain along a fixed path (member tracking by replay) */
static int chain_passes(const ctx *C, rec r, int sector, int32_t path[][MAXD]) {
  canon(C, &r, 0, path[0]);
  for (int m = 0; m < C->Lstar; m++) {
    if (!meets(C, &r, m, sector, path[m + 1])) return 0;
    if (m + 1 < C->Lstar) canon(C, &r, m + 1, path[m + 1]);
  }
  return 1;
}

static int check_range(ctx *C, const rec *S, int64_t n) {
  if (is_pose(C)) return OR_OK;
  /* every value stays a multiple of sf/2 below 2^52 sf/2: exact in binary64 */
  for (int64_t i = 0; i < n; i++) {
    int nP, P[2], nQ, Q[2];
    lin_axes(C, S[i].tag, &nP, P, &nQ, Q);
    for (int qi = 0; qi < nQ; qi++) {
      double M = fabs(S[i].p[4 + qi]) + 4.0;
      for (int k = 0; k < nP; k++) M += fabs(S[i].p[2 * qi + k]);
      if (!(M < ldexp(C->sf[Q[qi]], 48))) return OR_ERANGE;
    }
  }
  return OR_OK;
}

static int build_root(ctx *C, rec **out, int64_t *nout) {
  const or_problem *p = C->prob;
  if (is_pose(C)) {
    int st = pose_lattice(C);
    if (st) return st;
  }
  rec *S = (rec *)malloc(sizeof(rec) * (size_t)(p->n > 0 ? p->n : 1));
  if (!S) return OR_ENOMEM;
  int32_t zero[MAXD] = {0};
  for (int64_t i = 0; i < p->n; i++) {
    int st = front(C, i, &S[i]);
    if (st) { free(S); return st; }
    canon(C, &S[i], 0, zero);
  }
  int st = check_range(C, S, p->n);
  if (st) { free(S); return st; }
  *out = S;
  *nout = p->n;
  return OR_OK;
}

static void leaf_point(const ctx *C, int sector, const int32_t *lc, double *pt) {
  for (int j = 0; j < C->d; j++) {
    /* centre of the leaf cell: lo + E ((2c+1) 2^-(L+1)) */
    double u = (double)(2 * lc[j] + 1) * ldexp(1.0, -(C->L[j] + 1));
    pt[j] = C->lo[j] + C->E[j] * u;
  }
  if (is_pose(C)) {
    double yaw = (double)sector * (M_PI / 2.0) + atan(pt[3]);
    if (yaw < 0.0) yaw += 2.0 * M_PI;
    if (yaw >= 2.0 * M_PI) yaw -= 2.0 * M_PI;
    pt[3] = yaw;
  }
}

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int replay_inliers(const ctx *C, uint64_t idx, uint64_t *count, int64_t *inl, int64_t cap,
                          int64_t *ninl) {
  int sector;
  int32_t path[MAXL + 1][MAXD];
  int st = leaf_path(C, idx, &sector, path);
  if (st) return st;
  int64_t k = 0;
  for (int64_t i = 0; i < C->prob->n; i++) {
    rec r;
    st = front(C, i, &r);
    if (st) return st;
    if (chain_passes(C, r, sector, path)) {
      if (inl && k < cap) inl[k] = i;
      k++;
    }
  }
  *count = (uint64_t)k;
  if (ninl) *ninl = k;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Optional thread pool: disjoint subtrees of one level, handed out in   */
/* index order; each worker derives its subtree's list from the root by  */
/* the same filter / canonize / group steps and searches it depth-first. */
/* Workers share only the best key, so the result equals the serial one. */
/* ------------------------------------------------------------------ */
typedef struct {
  ctx *base;
  const rec *S;
  int64_t n;
  int level;          /* subtrees are the cells of this level */
  uint64_t ntask;     /* nsec * 2^(digit bits of levels 0..level-1) */
  uint64_t *next;     /* shared task counter */
  int *status;        /* first error of any worker */
  ctx local;          /* this worker's counters */
} worker;

static int subtree(ctx *C, const rec *S, int64_t n, int level, uint64_t task) {
  int sector;
  int32_t path[MAXL + 1][MAXD];
  cell_path(C, task, level, &sector, path);
  rec *cur = (rec *)malloc(sizeof(rec) * (size_t)(n > 0 ? n : 1));
  rec *nxt = (rec *)malloc(sizeof(rec) * (size_t)(n > 0 ? n : 1));
  if (!cur || !nxt) { free(cur); free(nxt); return OR_ENOMEM; }
  memcpy(cur, S, sizeof(rec) * (size_t)n);
  int64_t nc = n;
  uint64_t prefix = (uint64_t)sector;
  int st = OR_OK;
  for (int m = 0; m < level; m++) {
    int a = C->abits[m];
    int digit = (int)((task >> (C->rem[m + 1] - C->rem[level])) & ((1ULL << a) - 1ULL));
    int64_t k;
    uint64_t cnt = filter(C, cur, nc, m, sector, path[m + 1], nxt, &k);
    prefix = (prefix << a) | (uint64_t)digit;
    uint64_t key = key_of(C, cnt, prefix << C->rem[m + 1]);
    if (!C->prob->no_prune && key <= best_get(C)) { C->pruned++; goto out; }
    for (int64_t i = 0; i < k; i++) canon(C, &nxt[i], m + 1, path[m + 1]);
    k = group(C, nxt, k);
    rec *t = cur; cur = nxt; nxt = t;
    nc = k;
  }
  st = expand(C, level, sector, path[level], prefix, cur, nc);
out:
  free(cur);
  free(nxt);
  return st;
}

static void *worker_main(void *arg) {
  worker *W = (worker *)arg;
  for (;;) {
    if (__atomic_load_n(W->status, __ATOMIC_RELAXED)) break;
    uint64_t t = __atomic_fetch_add(W->next, 1, __ATOMIC_RELAXED);
    if (t >= W->ntask) break;
    int st = subtree(&W->local, W->S, W->n, W->level, t);
    if (st) {
      int zero = 0;
      __atomic_compare_exchange_n(W->status, &zero, st, 0, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
      break;
    }
  }
  return NULL;
}

static int search_parallel(ctx *C, const rec *S, int64_t n, int nthreads) {
  int nsec = is_pose(C) ? 4 : 1;
  /* subtrees: the first level with at least 64 cells per worker (or the
   * last level above the leaves) */
  int level = 0;
  uint64_t cells = (uint64_t)nsec;
  while (level < C->Lstar - 1 && cells < 64ULL * (uint64_t)nthreads) cells <<= C->abits[level++];
  if (level == 0) {
    for (int s = 0; s < nsec; s++) {
      int32_t zero[MAXD] = {0};
      int st = expand(C, 0, s, zero, (uint64_t)s, S, n);
      if (st) return st;
    }
    return OR_OK;
  }
  uint64_t shared = C->best, next = 0;
  int status = OR_OK;
  worker *W = (worker *)calloc((size_t)nthreads, sizeof(worker));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!W || !th) { free(W); free(th); return OR_ENOMEM; }
  uint64_t budget = C->budget ? (C->budget + (uint64_t)nthreads - 1) / (uint64_t)nthreads : 0;
  int started = 0;
  for (int i = 0; i < nthreads; i++) {
    W[i].base = C; W[i].S = S; W[i].n = n; W[i].level = level; W[i].ntask = cells;
    W[i].next = &next; W[i].status = &status;
    W[i].local = *C;
    W[i].local.shared_best = &shared;
    W[i].local.tests = W[i].local.expanded = W[i].local.pruned = W[i].local.merged = 0;
    W[i].local.budget = budget;
    if (pthread_create(&th[i], NULL, worker_main, &W[i]) != 0) break;
    started++;
  }
  if (started == 0) worker_main(&W[0]);
  for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
  for (int i = 0; i < (started ? started : 1); i++) {
    C->tests += W[i].local.tests;
    C->expanded += W[i].local.expanded;
    C->pruned += W[i].local.pruned;
    C->merged += W[i].local.merged;
  }
  C->best = shared;
  free(W);
  free(th);
  return status;
}

int or_solve(const or_problem *p, or_result *res, int64_t *inliers, int64_t cap) {
  ctx C;
  memset(res, 0, sizeof(*res));
  int st = ctx_init(&C, p);
  if (st) return st;
  C.budget = p->test_budget;
  rec *S;
  int64_t n;
  st = build_root(&C, &S, &n);
  if (st) return st;
  double t0 = now_s();
  n = group(&C, S, n);
  int nsec = is_pose(&C) ? 4 : 1;
  C.best = 0;
  if (p->has_seed) {
    /* a leaf named by the caller: its count by replay is achieved */
    uint64_t cnt;
    int64_t ninl;
    st = replay_inliers(&C, p->seed_leaf, &cnt, NULL, 0, &ninl);
    if (!st) C.best = key_of(&C, cnt, p->seed_leaf);
  }
  if (!p->no_dive)
    for (int s = 0; s < nsec && !st; s++) st = dive(&C, s, S, n);
  if (!st && p->threads > 1) {
    st = search_parallel(&C, S, n, p->threads);
  } else {
    int32_t zero[MAXD] = {0};
    for (int s = 0; s < nsec && !st; s++) st = expand(&C, 0, s, zero, (uint64_t)s, S, n);
  }
  free(S);
  res->tests = C.tests;
  res->cells_expanded = C.expanded;
  res->cells_pruned = C.pruned;
  res->groups_merged = C.merged;
  res->seconds = now_s() - t0;
  if (st) return st;
  uint64_t mask = (1ULL << C.B) - 1ULL;
  res->key = C.best;
  res->count = C.best >> C.B;
  res->leaf_index = mask - (C.best & mask);
  res->lstar = C.Lstar;
  res->index_bits = C.B;
  for (int j = 0; j < MAXD; j++) res->levels[j] = j < C.d ? C.L[j] : 0;
  int sector;
  int32_t path[MAXL + 1][MAXD];
  leaf_path(&C, res->leaf_index, &sector, path);
  res->sector = sector;
  for (int j = 0; j < MAXD; j++) res->leaf_coords[j] = j < C.d ? path[C.Lstar][j] : 0;
  leaf_point(&C, sector, path[C.Lstar], res->point);
  uint64_t cnt;
  int64_t ninl;
  st = replay_inliers(&C, res->leaf_index, &cnt, inliers, cap, &ninl);
  if (st) return st;
  res->n_inliers = ninl;
  if (cnt != res->count) return OR_EINVAL; /* internal consistency: never expected */
  if (ninl > cap) return OR_EBUFSZ;
  return OR_OK;
}

/* Threshold reporting (the ray-intersection setting of Sec. 4.3: every
 * cell of the leaf grid met by at least tau surfaces): the search of Alg. 2
 * with the cut "count < tau" in place of the best key.  Leaves come out in
 * index order (children are visited in digit order). */
int or_report(const or_problem *p, uint64_t tau, uint64_t *leaves, uint32_t *counts, int64_t cap,
              int64_t *n_out, uint64_t *tests) {
  ctx C;
  *n_out = 0;
  int st = ctx_init(&C, p);
  if (st) return st;
  if (tau < 1 || tau >= (1ULL << (63 - C.B))) return OR_EINVAL;
  rec *S;
  int64_t n;
  st = build_root(&C, &S, &n);
  if (st) return st;
  n = group(&C, S, n);
  C.report = 1;
  C.rep_idx = leaves;
  C.rep_cnt = counts;
  C.rep_cap = cap;
  C.best = (tau << C.B) - 1ULL;
  int nsec = is_pose(&C) ? 4 : 1;
  int32_t zero[MAXD] = {0};
  for (int s = 0; s < nsec && !st; s++) st = expand(&C, 0, s, zero, (uint64_t)s, S, n);
  free(S);
  *n_out = C.rep_n;
  if (tests) *tests = C.tests;
  if (st) return st;
  if (C.rep_n > cap) return OR_EBUFSZ;
  return OR_OK;
}

static void to_tf(const ctx *C, const rec *r, double *t, double *f, int32_t *tag) {
  if (is_pose(C)) {
    t[0] = r->p[0]; t[1] = r->p[1]; t[2] = r->p[3]; t[3] = r->p[4];
    f[0] = r->p[2]; f[1] = r->p[5];
  } else {
    for (int k = 0; k < 4; k++) t[k] = r->p[k];
    f[0] = r->p[4]; f[1] = r->p[5];
  }
  *tag = r->tag;
}

static void from_tf(const ctx *C, const double *t, const double *f, int32_t tag, rec *r) {
  memset(r, 0, sizeof(*r));
  r->w = 1;
  r->tag = tag;
  if (is_pose(C)) {
    r->p[0] = t[0]; r->p[1] = t[1]; r->p[3] = t[2]; r->p[4] = t[3];
    r->p[2] = f[0]; r->p[5] = f[1];
  } else {
    for (int k = 0; k < 4; k++) r->p[k] = t[k];
    r->p[4] = f[0]; r->p[5] = f[1];
  }
}

int or_parametrize(const or_problem *p, double *t, double *f, int32_t *tag) {
  ctx C;
  int st = ctx_init(&C, p);
  if (st) return st;
  if (is_pose(&C)) C.ce = C.E[0] * C.inv[2];
  for (int64_t i = 0; i < p->n; i++) {
    rec r;
    st = front(&C, i, &r);
    if (st) return st;
    to_tf(&C, &r, t + 4 * i, f + 2 * i, tag + i);
  }
  return OR_OK;
}

int or_root_canon(const or_problem *p, double *t, double *f, int32_t *tag) {
  ctx C;
  int st = ctx_init(&C, p);
  if (st) return st;
  rec *S;
  int64_t n;
  st = build_root(&C, &S, &n);
  if (st) return st;
  for (int64_t i = 0; i < n; i++) to_tf(&C, &S[i], t + 4 * i, f + 2 * i, tag + i);
  free(S);
  return OR_OK;
}

int or_leaf_count(const or_problem *p, uint64_t leaf_index, uint64_t *count, int64_t *inliers,
                  int64_t cap) {
  ctx C;
  int st = ctx_init(&C, p);
  if (st) return st;
  if (is_pose(&C)) {
    st = pose_lattice(&C);
    if (st) return st;
  }
  int64_t ninl;
  st = replay_inliers(&C, leaf_index, count, inliers, cap, &ninl);
  if (st) return st;
  if (inliers && ninl > cap) return OR_EBUFSZ;
  return OR_OK;
}

int or_all_leaf_counts(const or_problem *p, uint32_t *out, uint64_t out_len) {
  ctx C;
  int st = ctx_init(&C, p);
  if (st) return st;
  if (C.B > 24 || out_len < (1ULL << C.B)) return OR_EINVAL;
  if (is_pose(&C)) {
    st = pose_lattice(&C);
    if (st) return st;
  }
  rec *S = (rec *)malloc(sizeof(rec) * (size_t)(p->n > 0 ? p->n : 1));
  if (!S) return OR_ENOMEM;
  for (int64_t i = 0; i < p->n; i++) {
    st = front(&C, i, &S[i]);
    if (st) { free(S); return st; }
  }
  for (uint64_t idx = 0; idx < (1ULL << C.B); idx++) {
    int sector;
    int32_t path[MAXL + 1][MAXD];
    leaf_path(&C, idx, &sector, path);
    uint32_t k = 0;
    for (int64_t i = 0; i < p->n; i++) k += (uint32_t)chain_passes(&C, S[i], sector, path);
    out[idx] = k;
  }
  free(S);
  return OR_OK;
}

/* chain of one surface down a path, levels 0..level-1 */
static int chain_upto(const ctx *C, rec r, int sector, int32_t path[][MAXD], int level) {
  canon(C, &r, 0, path[0]);
  for (int m = 0; m < level; m++) {
    if (!meets(C, &r, m, sector, path[m + 1])) return 0;
    if (m + 1 < C->Lstar) canon(C, &r, m + 1, path[m + 1]);
  }
  return 1;
}

static int small_tree(ctx *C, const or_problem *p) {
  int st = ctx_init(C, p);
  if (st) return st;
  if (C->B > 24) return OR_EINVAL;
  if (is_pose(C)) return pose_lattice(C);
  return OR_OK;
}

int or_level_counts(const or_problem *p, int level, uint32_t *out, uint64_t out_len) {
  ctx C;
  int st = small_tree(&C, p);
  if (st) return st;
  if (level < 0 || level > C.Lstar) return OR_EINVAL;
  int bits = is_pose(&C) ? 2 : 0;
  for (int m = 0; m < level; m++) bits += C.abits[m];
  if (out_len < (1ULL << bits)) return OR_EINVAL;
  rec *S = (rec *)malloc(sizeof(rec) * (size_t)(p->n > 0 ? p->n : 1));
  if (!S) return OR_ENOMEM;
  for (int64_t i = 0; i < p->n; i++) {
    st = front(&C, i, &S[i]);
    if (st) { free(S); return st; }
  }
  for (uint64_t idx = 0; idx < (1ULL << bits); idx++) {
    int sector;
    int32_t path[MAXL + 1][MAXD];
    cell_path(&C, idx, level, &sector, path);
    uint32_t k = 0;
    for (int64_t i = 0; i < p->n; i++) k += (uint32_t)chain_upto(&C, S[i], sector, path, level);
    out[idx] = k;
  }
  free(S);
  return OR_OK;
}

int or_leaf_indicator(const or_problem *p, int64_t i, uint8_t *out, uint64_t out_len) {
  ctx C;
  int st = small_tree(&C, p);
  if (st) return st;
  if (i < 0 || i >= p->n || out_len < (1ULL << C.B)) return OR_EINVAL;
  rec r;
  st = front(&C, i, &r);
  if (st) return st;
  for (uint64_t idx = 0; idx < (1ULL << C.B); idx++) {
    int sector;
    int32_t path[MAXL + 1][MAXD];
    leaf_path(&C, idx, &sector, path);
    out[idx] = (uint8_t)chain_passes(&C, r, sector, path);
  }
  return OR_OK;
}

int or_cell_masks(const or_problem *p, int level, int32_t sector, const int32_t *coords, uint32_t *masks) {
  ctx C;
  int st = ctx_init(&C, p);
  if (st) return st;
  if (level < 0 || level >= C.Lstar) return OR_EINVAL;
  if (is_pose(&C)) {
    st = pose_lattice(&C);
    if (st) return st;
  }
  /* the path of cells from the root to the given one */
  int32_t path[MAXL + 1][MAXD];
  for (int m = 0; m <= level; m++)
    for (int j = 0; j < MAXD; j++) {
      int bits = j < C.d ? imin(level, C.L[j]) : 0, mb = j < C.d ? imin(m, C.L[j]) : 0;
      path[m][j] = j < C.d ? (coords[j] >> (bits - mb)) : 0;
    }
  for (int64_t i = 0; i < p->n; i++) {
    rec r;
    st = front(&C, i, &r);
    if (st) return st;
    for (int m = 0; m <= level; m++) canon(&C, &r, m, path[m]);
    uint32_t mask = 0;
    for (int digit = 0; digit < (1 << C.abits[level]); digit++) {
      int32_t ch[MAXD];
      child_coords(&C, level, path[level], digit, ch);
      if (meets(&C, &r, level, sector, ch)) mask |= 1u << digit;
    }
    masks[i] = mask;
  }
  return OR_OK;
}

int or_meets(const or_problem *p, const double *t, const double *f, int32_t tag, int level,
             int32_t sector, const int32_t *coords) {
  ctx C;
  int st = ctx_init(&C, p);
  if (st) return st;
  if (level < 0 || level >= C.Lstar) return OR_EINVAL;
  if (is_pose(&C)) {
    st = pose_lattice(&C);
    if (st) return st;
  }
  rec r;
  from_tf(&C, t, f, tag, &r);
  return meets(&C, &r, level, sector, coords);
}

int or_canon_at(const or_problem *p, const double *t, const double *f, int32_t tag, int level,
                const int32_t *coords, double *t_out, double *f_out) {
  ctx C;
  int st = ctx_init(&C, p);
  if (st) return st;
  if (level < 0 || level > C.Lstar) return OR_EINVAL;
  if (is_pose(&C)) {
    st = pose_lattice(&C);
    if (st) return st;
  }
  rec r;
  from_tf(&C, t, f, tag, &r);
  canon(&C, &r, level, coords);
  int32_t tg;
  to_tf(&C, &r, t_out, f_out, &tg);
  return OR_OK;
}

int or_constants(const or_problem *p, double *out, int out_len) {
  ctx C;
  int st = ctx_init(&C, p);
  if (st) return st;
  if (out_len < 27) return OR_EINVAL;
  if (is_pose(&C)) {
    st = pose_lattice(&C);
    if (st) return st;
  }
  memset(out, 0, sizeof(double) * (size_t)out_len);
  out[0] = C.Lstar;
  out[1] = C.B;
  for (int j = 0; j < 4; j++) out[2 + j] = j < C.d ? C.L[j] : 0;
  if (is_pose(&C)) {
    out[6] = C.sW; out[7] = C.sW3; out[8] = C.sXi; out[9] = C.sEta;
    out[10] = C.padz; out[11] = C.padk;
    out[14] = C.padz; out[15] = C.padk;
  } else {
    for (int j = 0; j < 4; j++) out[6 + j] = j < C.d ? C.sf[j] : 0;
    for (int j = 0; j < 4; j++) out[10 + j] = j < C.d ? C.pad[0][j] : 0;
    for (int j = 0; j < 4; j++) out[14 + j] = j < C.d ? C.pad[C.Lstar - 1][j] : 0;
  }
  out[18] = sqrt(C.Rg2);
  out[19] = C.epsn[0]; out[20] = C.epsn[1]; out[21] = C.epsn[2]; out[22] = C.epsn[3];
  out[23] = C.exact;
  out[24] = C.d > 4 ? C.L[4] : 0;
  out[25] = C.d > 4 ? C.epsn[4] : 0;
  out[26] = is_pose(&C) ? C.Fb : 0;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* After the vote (pose families): verification of the angular error of */
/* the inlier set and refinement of the pose by a more accurate method   */
/* that works on that nearly outlier-free set (Sec. 4.2, opening remark; */
/* Sec. 5, angular verification of the final inlier set).                */
/*                                                                       */
/* Pose q = (x, y, z, kappa[, f]) in user units, within the sector s of  */
/* the vote's leaf: the camera forward direction, turned into the        */
/* sector's frame, is (1, kappa)/sqrt(1 + kappa^2).  In camera axes      */
/* (forward, lateral, up) match i is observed along                      */
/*   o = (1, a, b sqrt(1 + a^2)),  a = xi f, b = eta f  (f = 1 for 4DoF) */
/* and its point w is seen along                                         */
/*   d = ((u1 + kappa u2)/n, (u2 - kappa u1)/n, w3 - z),                 */
/* u = Rot_s(w1 - x, w2 - y), n = sqrt(1 + kappa^2).  Only +, -, *, /    */
/* and sqrt are used, so the verification decision (angle(o, d) <= tau:  */
/* o.d > 0 and |o x d|^2 <= tan^2(tau) (o.d)^2) is exact IEEE binary64.  */
/* The first verification is at the centre of the vote's leaf (the      */
/* minimal cuboid) with a threshold tau0 that covers the leaf.           */
/* Refinement: Gauss-Newton steps with a small fixed damping on the sum  */
/* of squared differences of the unit directions, |d/|d| - o/|o||^2      */
/* (= (2 sin(angle/2))^2), over the verified matches; a fixed number of  */
/* steps per round, then verification again at the new pose.             */
/* ------------------------------------------------------------------ */
#define RF_DAMP 1e-6

static void rf_rot(int s, double a, double b, double *u1, double *u2) {
  switch (s & 3) {
    case 0: *u1 = a; *u2 = b; break;
    case 1: *u1 = b; *u2 = -a; break;
    case 2: *u1 = -a; *u2 = -b; break;
    default: *u1 = -b; *u2 = a; break;
  }
}

/* directions o (observed) and d (predicted) of match i at pose q */
static void rf_dirs(const or_problem *p, int five, int s, const double *q, int64_t i, double o[3], double d[3]) {
  double f = five ? q[4] : 1.0;
  double a = p->col[3][i] * f, b = p->col[4][i] * f;
  o[0] = 1.0;
  o[1] = a;
  o[2] = b * sqrt(1.0 + a * a);
  double u1, u2;
  rf_rot(s, p->col[0][i] - q[0], p->col[1][i] - q[1], &u1, &u2);
  double n = sqrt(1.0 + q[3] * q[3]);
  d[0] = (u1 + q[3] * u2) / n;
  d[1] = (u2 - q[3] * u1) / n;
  d[2] = p->col[2][i] - q[2];
}

static int rf_verified(const double o[3], const double d[3], double T2) {
  double dot = (o[0] * d[0] + o[1] * d[1]) + o[2] * d[2];
  double c0 = o[1] * d[2] - o[2] * d[1], c1 = o[2] * d[0] - o[0] * d[2], c2 = o[0] * d[1] - o[1] * d[0];
  double cr = (c0 * c0 + c1 * c1) + c2 * c2;
  return dot > 0.0 && cr <= T2 * (dot * dot);
}

/* residual r = d/|d| - o/|o| and its Jacobian J (3 x P) w.r.t. q */
static void rf_resid(const or_problem *p, int five, int s, const double *q, int64_t i, double r[3], double J[3][5]) {
  double o[3], d[3];
  rf_dirs(p, five, s, q, i, o, d);
  double nd = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  double no = sqrt((o[0] * o[0] + o[1] * o[1]) + o[2] * o[2]);
  double dh[3] = {d[0] / nd, d[1] / nd, d[2] / nd}, oh[3] = {o[0] / no, o[1] / no, o[2] / no};
  for (int k = 0; k < 3; k++) r[k] = dh[k] - oh[k];
  /* derivatives of d: u depends on x, y through Rot_s; F, L on kappa */
  double n2 = 1.0 + q[3] * q[3], n = sqrt(n2);
  double ux1, ux2, uy1, uy2;
  rf_rot(s, -1.0, 0.0, &ux1, &ux2);
  rf_rot(s, 0.0, -1.0, &uy1, &uy2);
  double dd[5][3];
  dd[0][0] = (ux1 + q[3] * ux2) / n; dd[0][1] = (ux2 - q[3] * ux1) / n; dd[0][2] = 0.0;
  dd[1][0] = (uy1 + q[3] * uy2) / n; dd[1][1] = (uy2 - q[3] * uy1) / n; dd[1][2] = 0.0;
  dd[2][0] = 0.0; dd[2][1] = 0.0; dd[2][2] = -1.0;
  dd[3][0] = d[1] / n2; dd[3][1] = -d[0] / n2; dd[3][2] = 0.0;
  int P = five ? 5 : 4;
  for (int k = 0; k < 4; k++) {
    /* (I - dh dh^T) dd / |d| */
    double pr = (dh[0] * dd[k][0] + dh[1] * dd[k][1]) + dh[2] * dd[k][2];
    for (int c = 0; c < 3; c++) J[c][k] = (dd[k][c] - dh[c] * pr) / nd;
  }
  if (five) {
    /* o depends on f: do/df = (0, xi, eta s + b a xi / s) */
    double xi = p->col[3][i], eta = p->col[4][i];
    double a = xi * q[4], b = eta * q[4];
    double sa = sqrt(1.0 + a * a);
    double dof[3] = {0.0, xi, eta * sa + (b * a) * xi / sa};
    double pr = (oh[0] * dof[0] + oh[1] * dof[1]) + oh[2] * dof[2];
    for (int c = 0; c < 3; c++) J[c][4] = -((dof[c] - oh[c] * pr) / no);
  }
  (void)P;
}

/* Cholesky solve of (A + damping diag(A)) x = -g; x = 0 when not positive
 * definite */
static void rf_solve(int P, double A[5][5], const double *g, double *x) {
  double M[5][5], L[5][5] = {{0}};
  for (int r = 0; r < P; r++)
    for (int c = 0; c < P; c++) M[r][c] = A[r][c] + (r == c ? RF_DAMP * A[r][c] : 0.0);
  for (int j = 0; j < P; j++) {
    double sdiag = M[j][j];
    for (int k = 0; k < j; k++) sdiag -= L[j][k] * L[j][k];
    if (!(sdiag > 0.0) || !isfinite(sdiag)) {
      for (int k = 0; k < P; k++) x[k] = 0.0;
      return;
    }
    L[j][j] = sqrt(sdiag);
    for (int r = j + 1; r < P; r++) {
      double v = M[r][j];
      for (int k = 0; k < j; k++) v -= L[r][k] * L[j][k];
      L[r][j] = v / L[j][j];
    }
  }
  double y[5];
  for (int r = 0; r < P; r++) {
    double v = -g[r];
    for (int k = 0; k < r; k++) v -= L[r][k] * y[k];
    y[r] = v / L[r][r];
  }
  for (int r = P - 1; r >= 0; r--) {
    double v = y[r];
    for (int k = r + 1; k < P; k++) v -= L[k][r] * x[k];
    x[r] = v / L[r][r];
  }
}

int or_refine(const or_problem *p, uint64_t leaf_index, const int64_t *idx, int64_t n_idx, double tau0, double tau,
              int rounds, int iters, double *pose_out, int64_t *verified, int64_t *n_verified, double *rms_out,
              double *rms0_out) {
  ctx C;
  int st = ctx_init(&C, p);
  if (st) return st;
  if (!is_pose(&C)) return OR_EINVAL;
  if (!(tau > 0.0 && tau < 1.5) || !(tau0 > 0.0 && tau0 < 1.5) || rounds < 0 || iters < 0 || n_idx < 0)
    return OR_EINVAL;
  for (int64_t k = 0; k < n_idx; k++)
    if (idx[k] < 0 || idx[k] >= p->n) return OR_EINVAL;
  int five = C.fam == OR_POSE5DOF, P = five ? 5 : 4;
  /* start: the centre of the vote's leaf, kappa at the centre of its
   * interval, in user units */
  int sector;
  int32_t path[MAXL + 1][MAXD];
  st = leaf_path(&C, leaf_index, &sector, path);
  if (st) return st;
  double q[5] = {0};
  for (int j = 0; j < C.d; j++) {
    double u = (double)(2 * path[C.Lstar][j] + 1) * ldexp(1.0, -(C.L[j] + 1));
    q[j] = C.lo[j] + C.E[j] * u;
  }
  /* the first verification, at the leaf centre, takes tau0 (wide enough for
   * the whole leaf); the later ones, at refined poses, take tau */
  double T20 = tan(tau0) * tan(tau0), T2 = tan(tau) * tan(tau);
  uint8_t *ok = (uint8_t *)calloc((size_t)(n_idx > 0 ? n_idx : 1), 1);
  if (!ok) return OR_ENOMEM;
  for (int round = 0; round <= rounds; round++) {
    /* verification at the current pose */
    for (int64_t k = 0; k < n_idx; k++) {
      double o[3], d[3];
      rf_dirs(p, five, sector, q, idx[k], o, d);
      ok[k] = (uint8_t)rf_verified(o, d, round == 0 ? T20 : T2);
    }
    if (round == 0 && rms0_out) {
      double e = 0.0;
      int64_t m = 0;
      for (int64_t k = 0; k < n_idx; k++) {
        if (!ok[k]) continue;
        double r[3], J[3][5];
        rf_resid(p, five, sector, q, idx[k], r, J);
        e += (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
        m++;
      }
      *rms0_out = m ? sqrt(e / (double)m) : 0.0;
    }
    if (round == rounds) break;
    for (int it = 0; it < iters; it++) {
      double A[5][5] = {{0}}, g[5] = {0};
      for (int64_t k = 0; k < n_idx; k++) {
        if (!ok[k]) continue;
        double r[3], J[3][5];
        rf_resid(p, five, sector, q, idx[k], r, J);
        for (int a = 0; a < P; a++) {
          g[a] += (J[0][a] * r[0] + J[1][a] * r[1]) + J[2][a] * r[2];
          for (int b = 0; b <= a; b++) A[a][b] += (J[0][a] * J[0][b] + J[1][a] * J[1][b]) + J[2][a] * J[2][b];
        }
      }
      for (int a = 0; a < P; a++)
        for (int b = a + 1; b < P; b++) A[a][b] = A[b][a];
      double dq[5];
      rf_solve(P, A, g, dq);
      for (int a = 0; a < P; a++) q[a] += dq[a];
    }
  }
  int64_t m = 0;
  double e = 0.0;
  for (int64_t k = 0; k < n_idx; k++) {
    if (!ok[k]) continue;
    if (verified) verified[m] = idx[k];
    m++;
    double r[3], J[3][5];
    rf_resid(p, five, sector, q, idx[k], r, J);
    e += (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
  }
  free(ok);
  *n_verified = m;
  *rms_out = m ? sqrt(e / (double)m) : 0.0;
  double yaw = (double)sector * (M_PI / 2.0) + atan(q[3]);
  if (yaw < 0.0) yaw += 2.0 * M_PI;
  if (yaw >= 2.0 * M_PI) yaw -= 2.0 * M_PI;
  for (int j = 0; j < MAXD; j++) pose_out[j] = j < C.d ? q[j] : 0.0;
  pose_out[3] = yaw;
  return OR_OK;
}
