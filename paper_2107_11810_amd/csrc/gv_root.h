// gv_root.h -- front-end, root-canonization and inlier-replay kernels.
//
// Several problems can share one launch: their originals are concatenated
// (problem p owns global indices [ooff[p], ooff[p+1])) and every per-problem
// constant comes from a device table indexed by p.
#pragma once
#include "gv_device.h"

struct Cols {
  const double* c[6];
};

struct PathC {
  uint8_t digit[GV_MAXL];
  int32_t sector;
};

__device__ inline void atomic_max_f64_pos(unsigned long long* a, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

// problem owning global original index i (ooff has nprob + 1 entries)
__device__ inline uint32_t prob_of(const uint64_t* __restrict__ ooff, uint32_t nprob, uint64_t i) {
  uint32_t lo = 0, hi = nprob;
  while (hi - lo > 1) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (ooff[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void k_front(int fam, const ProbC* __restrict__ Pp, Cols cols, int64_t n, double* __restrict__ t,
                        double* __restrict__ f, int32_t* __restrict__ tag, int* __restrict__ bad) {
  const ProbC& P = *Pp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double tt[4], ff[2];
    int32_t tg;
    if (!front_eval(fam, cols.c, i, P, tt, ff, &tg)) atomicOr(bad, 1);
    for (int k = 0; k < 4; k++) t[4 * i + k] = tt[k];
    f[2 * i] = ff[0];
    f[2 * i + 1] = ff[1];
    tag[i] = tg;
  }
}

// root canonization of a linear surface: translate by the zero corner and
// round every parameter to the free step s_f
template <int FAM>
__device__ inline bool root_lin(const ProbC& P, const double* const* col, int64_t i, LinS& s, int* bad) {
  double t[4], f[2];
  int32_t tag;
  if (!front_eval(FAM, col, i, P, t, f, &tag)) {
    atomicOr(bad, 1);
    return false;
  }
  s.K[0][0] = s.K[0][1] = s.K[1][0] = s.K[1][1] = 0;
  s.F[0] = s.F[1] = 0;
  s.tag = tag;
  s.w = 1;
  bool ok = true;
  for (int qi = 0; qi < nQ<FAM>(); qi++) {
    const int q = Qax<FAM>(s, qi);
    for (int pi = 0; pi < nP<FAM>(); pi++) {
      double k = rint(t[2 * qi + pi] * P.inv_sf[q]);
      ok = ok && fabs(k) < 1073741824.0;
      s.K[qi][pi] = ok ? (int32_t)k : 0;
    }
    double F = rint(f[qi] * P.inv_sf[q]);
    ok = ok && fabs(F) < 1073741824.0;
    s.F[qi] = ok ? (int32_t)F : 0;
  }
  if (!ok) atomicOr(bad, 2);
  return true;
}

template <int FAM>
__global__ void k_root_lin(const ProbC* __restrict__ Pp, Cols cols, int64_t n, typename EntOf<FAM>::T* __restrict__ out,
                           unsigned int* __restrict__ maxabs, int* __restrict__ bad) {
  const ProbC& P = *Pp;
  unsigned mk = 0, mf = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    LinS s;
    if (!root_lin<FAM>(P, cols.c, i, s, bad)) {
      s = LinS{};
      s.w = 1;
    }
    for (int qi = 0; qi < 2; qi++) {
      for (int pi = 0; pi < 2; pi++) mk = max(mk, (unsigned)abs(s.K[qi][pi]));
      mf = max(mf, (unsigned)abs(s.F[qi]));
    }
    out[i] = store_lin<FAM>(s);
  }
  atomicMax(&maxabs[0], mk);
  atomicMax(&maxabs[1], mf);
}

// data bounds of a pose problem: mx[0] = max |eta'|, mx[1] = max squared
// horizontal reach from the box, mx[7] = max |xi|
__global__ void k_pose_bounds(const ProbC* __restrict__ Pp, int fam, Cols cols, int64_t n,
                              unsigned long long* __restrict__ mx, int* __restrict__ bad) {
  const ProbC& P = *Pp;
  double H = 0.0, R2 = 0.0, Xm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double t[4], f[2];
    int32_t tag;
    if (!front_eval(fam, cols.c, i, P, t, f, &tag)) {
      atomicOr(bad, 1);
      continue;
    }
    double h = fabs(t[3]);
    H = h > H ? h : H;
    double x = fabs(t[2]);
    Xm = x > Xm ? x : Xm;
    double a0 = t[0] * t[0], a1 = (t[0] - 1.0) * (t[0] - 1.0);
    double b0 = t[1] * t[1], b1 = (t[1] - 1.0) * (t[1] - 1.0);
    double r2 = (a0 > a1 ? a0 : a1) + (b0 > b1 ? b0 : b1);
    R2 = r2 > R2 ? r2 : R2;
  }
  atomic_max_f64_pos(&mx[0], H);
  atomic_max_f64_pos(&mx[1], R2);
  atomic_max_f64_pos(&mx[7], Xm);
}

// quantize once at the root to the fixed pose lattice; the binary64 master
// is SoA with stride Ntot, entries carry their global index
__global__ void k_root_pose(const ProbC* __restrict__ Pp, int fam, Cols cols, int64_t n, uint64_t base, uint64_t Ntot,
                            double* __restrict__ m64, EntQ32* __restrict__ e32, EntQ64* __restrict__ e64,
                            unsigned long long* __restrict__ mx) {
  const ProbC& P = *Pp;
  double a[5] = {0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double t[4], f[2];
    int32_t tag;
    front_eval(fam, cols.c, i, P, t, f, &tag);
    const double W1 = rint(t[0] * P.inv_sW) * P.sW;
    const double W2 = rint(t[1] * P.inv_sW) * P.sW;
    const double W3 = rint(f[0] * P.inv_sW3) * P.sW3;
    const double xi = rint(t[2] * P.inv_sXi) * P.sXi;
    const double eta = rint(t[3] * P.inv_sEta) * P.sEta;
    const uint64_t g = base + (uint64_t)i;
    m64[g] = W1;
    m64[Ntot + g] = W2;
    m64[2 * Ntot + g] = W3;
    m64[3 * Ntot + g] = xi;
    m64[4 * Ntot + g] = eta;
    e32[g] = EntQ32{(float)W1, (float)W2, (float)W3, (float)xi, (float)eta, 1u, (uint32_t)g, 0u};
    e64[g] = EntQ64{W1, W2, W3, xi, eta, 1u, (uint32_t)g};
    double v[5] = {fabs(W1), fabs(W2), fabs(W3), fabs(xi), fabs(eta)};
    for (int k = 0; k < 5; k++) a[k] = v[k] > a[k] ? v[k] : a[k];
  }
  for (int k = 0; k < 5; k++) atomic_max_f64_pos(&mx[2 + k], a[k]);
}

// ---------------------------------------------------------------------------
// Replay: every original surface's canonization chain along its problem's
// chosen root-to-leaf path; an inlier iff every test on the path passes
// (member tracking, Sec. 3.2.1).
// ---------------------------------------------------------------------------
template <int FAM>
__global__ void k_replay_lin(const ProbC* __restrict__ Ptab, const Cols* __restrict__ ctab,
                             const uint64_t* __restrict__ ooff, uint32_t nprob, uint64_t Ntot,
                             const PathC* __restrict__ paths, uint32_t* __restrict__ flag, int* __restrict__ bad) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Ntot; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t p = prob_of(ooff, nprob, i);
    const ProbC& P = Ptab[p];
    const PathC& path = paths[p];
    LinS s;
    uint32_t ok = 0;
    if (root_lin<FAM>(P, ctab[p].c, (int64_t)(i - ooff[p]), s, bad)) {
      ok = 1;
      for (int m = 0; m < P.Lstar; m++) {
        const LevelC& lv = P.lev[m];
        const uint32_t cb = lv.cbits[path.digit[m]];
        if (!lin_meets<FAM>(s, lv, cb)) { ok = 0; break; }
        if (m + 1 < P.Lstar) s = lin_canon_child<FAM>(s, lv, cb);
      }
    }
    flag[i] = ok;
  }
}

__global__ void k_replay_pose(const ProbC* __restrict__ Ptab, const double* __restrict__ m64, uint64_t Ntot,
                              const uint64_t* __restrict__ ooff, uint32_t nprob, const PathC* __restrict__ paths,
                              uint32_t* __restrict__ flag) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Ntot; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t p = prob_of(ooff, nprob, i);
    const ProbC& P = Ptab[p];
    const PathC& path = paths[p];
    const double W1 = m64[i], W2 = m64[Ntot + i], W3 = m64[2 * Ntot + i], xi = m64[3 * Ntot + i],
                 eta = m64[4 * Ntot + i];
    int32_t cc[4] = {0, 0, 0, 0};
    uint32_t ok = 1;
    for (int m = 0; m < P.Lstar && ok; m++) {
      const LevelC& lv = P.lev[m];
      const uint32_t cb = lv.cbits[path.digit[m]];
      int32_t ch[4];
      for (int a = 0; a < 4; a++) ch[a] = lv.split[a] ? 2 * cc[a] + (int32_t)((cb >> a) & 1u) : cc[a];
      const int m1 = m + 1;
      double h[4];
      for (int j = 0; j < 4; j++) h[j] = ldexp(1.0, -min(m1, P.L[j]));
      const double Xlo = (double)ch[0] * h[0], Xhi = (double)(ch[0] + 1) * h[0];
      const double Ylo = (double)ch[1] * h[1], Yhi = (double)(ch[1] + 1) * h[1];
      const double Zlo = (double)ch[2] * h[2], Zhi = (double)(ch[2] + 1) * h[2];
      const double Klo = 2.0 * ((double)ch[3] * h[3]) - 1.0, Khi = 2.0 * ((double)(ch[3] + 1) * h[3]) - 1.0;
      VBox<double> v = pose_vbox<double>(W1, W2, Xlo, Xhi, Ylo, Yhi, path.sector);
      const double rmin2 = rmin2_of(v), rmax2 = rmax2_of(v);
      ok = zhalf64(W3, eta, rmin2, rmax2, Zhi + P.padz, Zlo - P.padz) &&
           khalf64(v, rmin2, P.Rg2, xi, Klo - P.padk, Khi + P.padk);
      for (int a = 0; a < 4; a++) cc[a] = ch[a];
    }
    flag[i] = ok;
  }
}

// inliers as indices local to their problem, sorted within each problem
__global__ void k_write_inliers(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                const uint64_t* __restrict__ ooff, uint32_t nprob, uint64_t Ntot,
                                int64_t* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Ntot; i += (uint64_t)gridDim.x * blockDim.x)
    if (flag[i]) out[pos[i]] = (int64_t)(i - ooff[prob_of(ooff, nprob, i)]);
}
