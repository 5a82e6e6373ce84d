// gv_device.h -- device-side data layout and per-family arithmetic of the
// MI355X general-voting library (gfx950, wave64).
//
// Linear families (LINE2D, PLANE3D, RAY3D) carry each canonical surface in
// a cell-relative integer lattice form: after the root canonization every
// parameter is a multiple of the free step s_f (Sec. 3.2.1: essential
// parameters rounded to eps'/((l+1) delta), free parameters to eps'/(l+1)),
// so the surface restricted to a cell is fully described by
//   K_i = t_i / s_t,i(m)     (s_t,i(m) = s_f * 2^min(m, L_i), an integer)
//   F_q = (G_q(u) - u_q) / s_f   (its height at the cell's min corner)
// and both the child test and the next canonization are exact small-integer
// arithmetic in units of s_f/2.  The two camera-posing families (POSE4DOF,
// and POSE5DOF with the focal-length factor f as a fifth axis) are quantized
// once at the root and evaluated in binary64 (POSE4DOF also in binary32 with
// a certified bound).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define GV_MAXL 40
#define GV_MAXD 5
#define GV_ITEM 1024  // most entries per work item (one wave)
#define GV_ITEM_LOG 10
static_assert(GV_ITEM == 1 << GV_ITEM_LOG, "item size");

enum { FAM_LINE2D = 1, FAM_PLANE3D = 2, FAM_RAY3D = 3, FAM_POSE4DOF = 4, FAM_SIM2D = 5, FAM_POSE5DOF = 6 };
// Exact mode of a linear family (quantized once at the root to a fixed
// 2^-36 lattice, never re-canonized, tested in binary64): kernel-side family
// code = family + 8.
enum { FAM_XLINE2D = 9, FAM_XPLANE3D = 10, FAM_XRAY3D = 11, FAM_XSIM2D = 13 };
constexpr bool fam_exact(int f) { return f >= 8; }
constexpr int fam_base(int f) { return f >= 8 ? f - 8 : f; }
// families whose count pass stores per-entry pass masks and whose
// compaction copies entries unchanged (the surfaces do not change below the
// root)
constexpr bool fam_pose(int f) { return f == FAM_POSE4DOF || f == FAM_POSE5DOF; }
constexpr bool fam_masked(int f) { return fam_pose(f) || fam_exact(f); }

// Per-level constants for the test from level m to level m+1.
struct LevelC {
  int32_t split[GV_MAXD];  // 1 if axis j splits at level m
  int32_t H[4];            // h_j(m) / s_f,j  (linear families)
  int32_t padu[4];         // 2 pad_j(m) / s_f,j (linear families)
  int32_t abits;           // number of split axes
  int32_t rem_next;        // index bits below level m+1
  uint8_t cbits[32];       // child digit -> bit j set iff b_j = 1
};

struct ProbC {
  int32_t fam, d, Lstar, B, Bcell, nsec;
  int32_t L[GV_MAXD];
  uint64_t idxmask;        // 2^B - 1
  // front end
  double lo[GV_MAXD], E[GV_MAXD], inv[GV_MAXD], ce;
  // POSE5DOF: the f axis in user units, f = flo + Ef u (POSE4DOF: f = 1)
  double flo, Ef;
  // linear lattice
  double sf[4], inv_sf[4];
  // pose lattice
  double sW, sW3, sXi, sEta, Rg2, padz, padk;
  double inv_sW, inv_sW3, inv_sXi, inv_sEta;
  float Rg2f, padzf, padkf, _pf;
  // exact mode: 1 when every surface is quantized once to the 2^-36
  // lattice and never re-canonized; xpad = eps rounded up to that lattice
  int32_t exact, _pe;
  double xpad[4];
  LevelC lev[GV_MAXL];
};

struct Cell {
  int32_t c[GV_MAXD];
  uint64_t prefix;   // index bits of this cell (sector on top for POSE4DOF)
  uint64_t off;      // first entry of its list in the batch
  uint32_t len;      // number of entries
  uint32_t sector;   // POSE4DOF yaw sector, else 0
  uint32_t prob;     // problem of this cell within the batch
  uint32_t _pad;
};

// A work item: entries [off, off + cnt) of one cell's list; cnt <= 2^ilog
// <= GV_ITEM, off - cell offset a multiple of 2^ilog (the batch's item size).
struct Item {
  uint64_t off;
  uint32_t cell, cnt;
};

// Linear-family entries (cell-relative lattice integers + multiplicity).
struct __attribute__((aligned(16))) EntL2 { int32_t K, F, w, _; };                 // LINE2D
struct __attribute__((aligned(16))) EntP3 { int32_t K1, K2, F, w; };               // PLANE3D
struct __attribute__((aligned(8))) EntR3 { int32_t K1, K2, F1, F2, w, tag; };     // RAY3D: K_q over axis tag
// SIM2D: K[q][i] of dependent axes c, d over parameter axes a, b
struct __attribute__((aligned(16))) EntS2 { int32_t K00, K01, K10, K11, F0, F1, w, _; };

// POSE4DOF entries: quantized parameters, weight, index of the root record.
struct __attribute__((aligned(16))) EntQ32 { float W1, W2, W3, xi, eta; uint32_t w, ridx, _; };
// unit-weight POSE4DOF lists below the root: the binary32 values and the
// root index only (24 bytes; every multiplicity is 1)
struct __attribute__((aligned(8))) EntQ24 { float W1, W2, W3, xi, eta; uint32_t ridx; };
static_assert(sizeof(EntQ24) == 24 && offsetof(EntQ24, ridx) == 20 && offsetof(EntQ32, eta) == 16 &&
                  offsetof(EntQ32, ridx) == 24,
              "the compaction copies these entries as words");
template <typename E> __device__ inline uint32_t pose_w(const E& e) { return e.w; }
template <> __device__ inline uint32_t pose_w<EntQ24>(const EntQ24&) { return 1u; }
struct __attribute__((aligned(16))) EntQ64 { double W1, W2, W3, xi, eta; uint32_t w, ridx; };

// Exact-mode linear entry: the root-quantized binary64 parameters t[q][i]
// (slope of dependent axis q over parameter axis i) and f[q].
//   LINE2D  t00 = t,  f0 = f
//   PLANE3D t00 = t1, t01 = t2, f0 = f
//   RAY3D   t00 = t of the first dependent axis, t10 = of the second; tag =
//           parameter axis
//   SIM2D   t00, t01 (axis c over a, b), t10, t11 (axis d), f0, f1
struct __attribute__((aligned(16))) EntX { double t00, t01, t10, t11, f0, f1; uint32_t w; int32_t tag; };
static_assert(sizeof(EntX) == 64, "copied as 16-byte words");

template <int FAM> struct EntOf;
template <> struct EntOf<FAM_LINE2D> { using T = EntL2; };
template <> struct EntOf<FAM_PLANE3D> { using T = EntP3; };
template <> struct EntOf<FAM_RAY3D> { using T = EntR3; };
template <> struct EntOf<FAM_SIM2D> { using T = EntS2; };

// Packed linear entries for the deeper levels, once the host has shown
// that every lattice value of a level fits (8 bytes instead of 16):
//   LINE2D : int16 K, int16 F, u32 w
//   PLANE3D: lo = K1 (13 bits, signed) | K2 (13, signed) | w bits 0..5,
//            hi = F (16, signed) | w bits 6..21
// RAY3D keeps its full entry.
#define GV_P3_KMAX 4095    // |K| limit of a packed PLANE3D entry
#define GV_P3_FMAX 32767   // |F| limit
#define GV_P3_WMAX 4194303 // weight limit (22 bits)
#define GV_L2_MAX 32767    // |K|, |F| limit of a packed LINE2D entry
struct __attribute__((aligned(8))) EntL2p { int16_t K, F; uint32_t w; };
struct __attribute__((aligned(8))) EntP3p { uint32_t lo, hi; };
// PLANE3D unit-weight lists at the deep levels, where the slopes fit 8 bits:
// one word, K1 (8, signed) | K2 (8, signed) << 8 | F (16, signed) << 16, and
// every multiplicity is 1.
#define GV_P3U_KMAX 127
struct __attribute__((aligned(4))) EntP3u { uint32_t v; };
template <int FAM> struct PackOf { using T = void; };  // no packed entry
template <> struct PackOf<FAM_LINE2D> { using T = EntL2p; };
template <> struct PackOf<FAM_PLANE3D> { using T = EntP3p; };

__device__ __host__ inline int32_t sext_field(uint32_t x, int pos, int bits) {
  return (int32_t)(x << (32 - pos - bits)) >> (32 - bits);
}
__device__ __host__ inline EntP3p pack_p3(int32_t K1, int32_t K2, int32_t F, uint32_t w) {
  EntP3p e;
  e.lo = ((uint32_t)K1 & 0x1fffu) | (((uint32_t)K2 & 0x1fffu) << 13) | ((w & 0x3fu) << 26);
  e.hi = ((uint32_t)F & 0xffffu) | ((w >> 6) << 16);
  return e;
}

// round-half-to-even of x/2 for an integer x
__device__ __host__ inline int32_t rne_half(int32_t x) {
  int32_t q = x >> 1;  // floor(x/2)
  return (x & 1) ? (q + (q & 1)) : q;
}

__device__ inline int32_t imin32(int32_t a, int32_t b) { return a < b ? a : b; }
__device__ inline int32_t imax32(int32_t a, int32_t b) { return a < b ? b : a; }

// ---------------------------------------------------------------------------
// Front end (binary64, operation order fixed, no contraction):
// observation -> normalized (t, f, tag).  Returns false on non-finite input
// or a zero ray direction.
// ---------------------------------------------------------------------------
__device__ inline bool front_eval(int fam, const double* const* col, int64_t i, const ProbC& P,
                                  double t[4], double f[2], int32_t* tag) {
  t[0] = t[1] = t[2] = t[3] = 0.0;
  f[0] = f[1] = 0.0;
  *tag = 0;
  if (fam == FAM_LINE2D) {
    double x = col[0][i], y = col[1][i];
    if (!isfinite(x) || !isfinite(y)) return false;
    t[0] = -((x * P.E[0]) * P.inv[1]);
    f[0] = ((y - x * P.lo[0]) - P.lo[1]) * P.inv[1];
  } else if (fam == FAM_PLANE3D) {
    double x = col[0][i], y = col[1][i], z = col[2][i];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return false;
    t[0] = -((x * P.E[0]) * P.inv[2]);
    t[1] = -((y * P.E[1]) * P.inv[2]);
    f[0] = (((z - x * P.lo[0]) - y * P.lo[1]) - P.lo[2]) * P.inv[2];
  } else if (fam == FAM_SIM2D) {
    // q_x = a p_x + b p_y + c, q_y = -b p_x + a p_y + d:
    // c = q_x - a p_x - b p_y, d = q_y + b p_x - a p_y
    double px = col[0][i], py = col[1][i], qx = col[2][i], qy = col[3][i];
    if (!isfinite(px) || !isfinite(py) || !isfinite(qx) || !isfinite(qy)) return false;
    t[0] = -((px * P.E[0]) * P.inv[2]);
    t[1] = -((py * P.E[1]) * P.inv[2]);
    f[0] = (((qx - px * P.lo[0]) - py * P.lo[1]) - P.lo[2]) * P.inv[2];
    t[2] = -((py * P.E[0]) * P.inv[3]);
    t[3] = (px * P.E[1]) * P.inv[3];
    f[1] = (((qy - py * P.lo[0]) + px * P.lo[1]) - P.lo[3]) * P.inv[3];
  } else if (fam == FAM_RAY3D) {
    double w[3], u[3];
    for (int k = 0; k < 3; k++) {
      w[k] = col[k][i];
      u[k] = col[3 + k][i];
      if (!isfinite(w[k]) || !isfinite(u[k])) return false;
    }
    int pi = 0;
    if (fabs(u[1]) > fabs(u[pi])) pi = 1;
    if (fabs(u[2]) > fabs(u[pi])) pi = 2;
    if (u[pi] == 0.0) return false;
    *tag = pi;
    int qi = 0;
    for (int q = 0; q < 3; q++) {
      if (q == pi) continue;
      double s = u[q] / u[pi];
      t[2 * qi] = (s * P.E[pi]) * P.inv[q];
      f[qi] = ((w[q] - P.lo[q]) + s * (P.lo[pi] - w[pi])) * P.inv[q];
      qi++;
    }
  } else {
    double wx = col[0][i], wy = col[1][i], wz = col[2][i], xi = col[3][i], eta = col[4][i];
    if (!isfinite(wx) || !isfinite(wy) || !isfinite(wz) || !isfinite(xi) || !isfinite(eta)) return false;
    t[0] = (wx - P.lo[0]) * P.inv[0];  // W1
    t[1] = (wy - P.lo[1]) * P.inv[1];  // W2
    t[2] = xi;
    t[3] = eta * P.ce;                 // eta' in normalized z units
    f[0] = (wz - P.lo[2]) * P.inv[2];  // W3
  }
  return true;
}

// ---------------------------------------------------------------------------
// Linear families: surface state in registers.
// ---------------------------------------------------------------------------
struct LinS {
  int32_t K[2][2];  // K[qi][pi]
  int32_t F[2];
  int32_t w, tag;
};

template <int FAM> __device__ inline constexpr int nQ() { return FAM == FAM_RAY3D || FAM == FAM_SIM2D ? 2 : 1; }
template <int FAM> __device__ inline constexpr int nP() { return FAM == FAM_PLANE3D || FAM == FAM_SIM2D ? 2 : 1; }

template <int FAM> __device__ inline int Pax(const LinS& s, int pi) {
  if (FAM == FAM_LINE2D) return 0;
  if (FAM == FAM_PLANE3D || FAM == FAM_SIM2D) return pi;
  return s.tag;
}
template <int FAM> __device__ inline int Qax(const LinS& s, int qi) {
  if (FAM == FAM_LINE2D) return 1;
  if (FAM == FAM_PLANE3D) return 2;
  if (FAM == FAM_SIM2D) return 2 + qi;
  // RAY3D: the two non-parameter axes, ascending
  int t = s.tag;
  return qi == 0 ? (t == 0 ? 1 : 0) : (t == 2 ? 1 : 2);
}

template <int FAM> __device__ __host__ inline LinS lin_zero() {
  LinS s;
  s.K[0][0] = s.K[0][1] = s.K[1][0] = s.K[1][1] = 0;
  s.F[0] = s.F[1] = 0;
  s.w = 0;
  s.tag = 0;
  return s;
}

// entry -> register state
template <int FAM> __device__ __host__ inline LinS load_ent(const EntL2& e) {
  LinS s = lin_zero<FAM>();
  s.K[0][0] = e.K; s.F[0] = e.F; s.w = e.w;
  return s;
}
template <int FAM> __device__ __host__ inline LinS load_ent(const EntP3& e) {
  LinS s = lin_zero<FAM>();
  s.K[0][0] = e.K1; s.K[0][1] = e.K2; s.F[0] = e.F; s.w = e.w;
  return s;
}
template <int FAM> __device__ __host__ inline LinS load_ent(const EntR3& e) {
  LinS s = lin_zero<FAM>();
  s.K[0][0] = e.K1; s.K[1][0] = e.K2; s.F[0] = e.F1; s.F[1] = e.F2; s.w = e.w; s.tag = e.tag;
  return s;
}
template <int FAM> __device__ __host__ inline LinS load_ent(const EntS2& e) {
  LinS s = lin_zero<FAM>();
  s.K[0][0] = e.K00; s.K[0][1] = e.K01; s.K[1][0] = e.K10; s.K[1][1] = e.K11;
  s.F[0] = e.F0; s.F[1] = e.F1; s.w = e.w;
  return s;
}
template <int FAM> __device__ __host__ inline LinS load_ent(const EntL2p& e) {
  LinS s = lin_zero<FAM>();
  s.K[0][0] = e.K; s.F[0] = e.F; s.w = (int32_t)e.w;
  return s;
}
template <int FAM> __device__ __host__ inline LinS load_ent(const EntP3p& e) {
  LinS s = lin_zero<FAM>();
  s.K[0][0] = sext_field(e.lo, 0, 13);
  s.K[0][1] = sext_field(e.lo, 13, 13);
  s.F[0] = sext_field(e.hi, 0, 16);
  s.w = (int32_t)(((e.hi >> 16) << 6) | (e.lo >> 26));
  return s;
}

template <int FAM> __device__ __host__ inline LinS load_ent(const EntP3u& e) {
  LinS s = lin_zero<FAM>();
  s.K[0][0] = sext_field(e.v, 0, 8);
  s.K[0][1] = sext_field(e.v, 8, 8);
  s.F[0] = sext_field(e.v, 16, 16);
  s.w = 1;
  return s;
}

// register state -> entry; a packed store clears ok when a value does not fit
template <int FAM, typename E> __device__ __host__ inline E store_ent(const LinS& s, bool& ok);
template <> __device__ __host__ inline EntL2 store_ent<FAM_LINE2D, EntL2>(const LinS& s, bool&) {
  EntL2 e;
  e.K = s.K[0][0]; e.F = s.F[0]; e.w = s.w; e._ = 0;
  return e;
}
template <> __device__ __host__ inline EntP3 store_ent<FAM_PLANE3D, EntP3>(const LinS& s, bool&) {
  EntP3 e;
  e.K1 = s.K[0][0]; e.K2 = s.K[0][1]; e.F = s.F[0]; e.w = s.w;
  return e;
}
template <> __device__ __host__ inline EntR3 store_ent<FAM_RAY3D, EntR3>(const LinS& s, bool&) {
  EntR3 e;
  e.K1 = s.K[0][0]; e.K2 = s.K[1][0]; e.F1 = s.F[0]; e.F2 = s.F[1]; e.w = s.w; e.tag = s.tag;
  return e;
}
template <> __device__ __host__ inline EntS2 store_ent<FAM_SIM2D, EntS2>(const LinS& s, bool&) {
  EntS2 e;
  e.K00 = s.K[0][0]; e.K01 = s.K[0][1]; e.K10 = s.K[1][0]; e.K11 = s.K[1][1];
  e.F0 = s.F[0]; e.F1 = s.F[1]; e.w = s.w; e._ = 0;
  return e;
}
template <> __device__ __host__ inline EntL2p store_ent<FAM_LINE2D, EntL2p>(const LinS& s, bool& ok) {
  ok = ok && abs(s.K[0][0]) <= GV_L2_MAX && abs(s.F[0]) <= GV_L2_MAX;
  EntL2p e;
  e.K = (int16_t)s.K[0][0]; e.F = (int16_t)s.F[0]; e.w = (uint32_t)s.w;
  return e;
}
template <> __device__ __host__ inline EntP3p store_ent<FAM_PLANE3D, EntP3p>(const LinS& s, bool& ok) {
  ok = ok && abs(s.K[0][0]) <= GV_P3_KMAX && abs(s.K[0][1]) <= GV_P3_KMAX && abs(s.F[0]) <= GV_P3_FMAX &&
       (uint32_t)s.w <= GV_P3_WMAX;
  return pack_p3(s.K[0][0], s.K[0][1], s.F[0], (uint32_t)s.w);
}

template <> __device__ __host__ inline EntP3u store_ent<FAM_PLANE3D, EntP3u>(const LinS& s, bool& ok) {
  ok = ok && abs(s.K[0][0]) <= GV_P3U_KMAX && abs(s.K[0][1]) <= GV_P3U_KMAX && abs(s.F[0]) <= GV_P3_FMAX &&
       s.w == 1;
  EntP3u e;
  e.v = ((uint32_t)s.K[0][0] & 0xffu) | (((uint32_t)s.K[0][1] & 0xffu) << 8) | ((uint32_t)s.F[0] << 16);
  return e;
}

template <int FAM> __device__ inline typename EntOf<FAM>::T store_lin(const LinS& s) {
  bool ok = true;
  return store_ent<FAM, typename EntOf<FAM>::T>(s, ok);
}

// per-lane selection from a small uniform array (avoids scratch indexing)
__device__ inline int32_t sel4(const int32_t* a, int j) {
  return j == 0 ? a[0] : (j == 1 ? a[1] : (j == 2 ? a[2] : a[3]));
}

// Test of the surface (canonized at the parent, level m) against child digit
// ch: for every dependent axis q the surface's range over the child's
// parameter box must reach the child's q-interval widened by pad(m).
template <int FAM> __device__ inline bool lin_meets(const LinS& s, const LevelC& lv, uint32_t cb) {
  bool ok = true;
#pragma unroll
  for (int qi = 0; qi < nQ<FAM>(); qi++) {
    int q = Qax<FAM>(s, qi);
    int32_t gmin = 2 * s.F[qi], gmax = gmin;
#pragma unroll
    for (int pi = 0; pi < nP<FAM>(); pi++) {
      int j = Pax<FAM>(s, pi);
      int32_t b = (int32_t)((cb >> j) & 1u);
      int32_t sp = sel4(lv.split, j);
      int32_t lo = sp ? b : 0, hi = sp ? b + 1 : 2;
      int32_t K = s.K[qi][pi];
      int32_t x = K * lo, y = K * hi;
      gmin += imin32(x, y);
      gmax += imax32(x, y);
    }
    int32_t bq = (int32_t)((cb >> q) & 1u);
    int32_t H = sel4(lv.H, q), pad = sel4(lv.padu, q);
    int32_t spq = sel4(lv.split, q);
    int32_t qlo = spq ? bq * H : 0, qhi = spq ? (bq + 1) * H : 2 * H;
    ok = ok && (gmax >= qlo - pad) && (gmin <= qhi + pad);
  }
  return ok;
}

// Canonization of the surface at the child cell (Sec. 3.2.1): translate to
// the child's min corner, round essential and free parameters to the
// child's lattice (half to even).
template <int FAM> __device__ inline LinS lin_canon_child(const LinS& s, const LevelC& lv, uint32_t cb) {
  LinS o = s;
#pragma unroll
  for (int qi = 0; qi < nQ<FAM>(); qi++) {
    int q = Qax<FAM>(s, qi);
    int32_t v = 2 * s.F[qi];
#pragma unroll
    for (int pi = 0; pi < nP<FAM>(); pi++) {
      int j = Pax<FAM>(s, pi);
      int32_t sp = sel4(lv.split, j);
      int32_t b = (int32_t)((cb >> j) & 1u);
      if (sp) v += s.K[qi][pi] * b;
      o.K[qi][pi] = sp ? rne_half(s.K[qi][pi]) : s.K[qi][pi];
    }
    int32_t spq = sel4(lv.split, q);
    int32_t bq = (int32_t)((cb >> q) & 1u);
    if (spq) v -= bq * sel4(lv.H, q);
    o.F[qi] = rne_half(v);
  }
  return o;
}

// ---------------------------------------------------------------------------
// Exact mode (linear families): the surface/box test in binary64 with the
// operation order of the plain definition (per dependent axis q, the range
// of f + sum t_i u_i over the child's parameter box, each term's min and max
// at the two ends, against the child's q-interval widened by the pad).
// lo/hi: the child box per axis.
// ---------------------------------------------------------------------------
__device__ inline bool x_axis(double f, double t0, int j0, double t1, int j1, int q, const double* lo,
                              const double* hi, double pad) {
  double gmin = f, gmax = f;
  {
    const double a = t0 * lo[j0], b = t0 * hi[j0];
    gmin = gmin + (a < b ? a : b);
    gmax = gmax + (a < b ? b : a);
  }
  if (j1 >= 0) {
    const double a = t1 * lo[j1], b = t1 * hi[j1];
    gmin = gmin + (a < b ? a : b);
    gmax = gmax + (a < b ? b : a);
  }
  return !(gmax < lo[q] - pad) && !(gmin > hi[q] + pad);
}

template <int BF>
__device__ inline bool x_meets(const EntX& e, const double* lo, const double* hi, const double* xpad) {
  if constexpr (BF == FAM_LINE2D) {
    return x_axis(e.f0, e.t00, 0, 0.0, -1, 1, lo, hi, xpad[1]);
  } else if constexpr (BF == FAM_PLANE3D) {
    return x_axis(e.f0, e.t00, 0, e.t01, 1, 2, lo, hi, xpad[2]);
  } else if constexpr (BF == FAM_SIM2D) {
    return x_axis(e.f0, e.t00, 0, e.t01, 1, 2, lo, hi, xpad[2]) && x_axis(e.f1, e.t10, 0, e.t11, 1, 3, lo, hi, xpad[3]);
  } else {
    const int t = e.tag;
    const int q0 = t == 0 ? 1 : 0, q1 = t == 2 ? 1 : 2;
    return x_axis(e.f0, e.t00, t, 0.0, -1, q0, lo, hi, xpad[q0]) &&
           x_axis(e.f1, e.t10, t, 0.0, -1, q1, lo, hi, xpad[q1]);
  }
}

// the child box (per axis, in the unit cube) of digit cb of a level-m cell
__device__ inline void x_child_box(const ProbC& P, const LevelC& lv, const int32_t* c, int m, uint32_t cb,
                                   double* lo, double* hi) {
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int32_t cj = lv.split[j] ? 2 * c[j] + (int32_t)((cb >> j) & 1u) : c[j];
    const double h = ldexp(1.0, -min(m + 1, P.L[j]));
    lo[j] = (double)cj * h;
    hi[j] = (double)(cj + 1) * h;
  }
}

// ---------------------------------------------------------------------------
// POSE4DOF predicate halves.  V = Rot_s(box of (W1 - X, W2 - Y)).
// ---------------------------------------------------------------------------
template <typename R> struct VBox { R x0, x1, y0, y1; };

template <typename R>
__device__ inline VBox<R> pose_vbox(R W1, R W2, R Xlo, R Xhi, R Ylo, R Yhi, int sector) {
  R Alo = W1 - Xhi, Ahi = W1 - Xlo, Blo = W2 - Yhi, Bhi = W2 - Ylo;
  VBox<R> v;
  if (sector == 0) { v.x0 = Alo; v.x1 = Ahi; v.y0 = Blo; v.y1 = Bhi; }
  else if (sector == 1) { v.x0 = Blo; v.x1 = Bhi; v.y0 = -Ahi; v.y1 = -Alo; }
  else if (sector == 2) { v.x0 = -Ahi; v.x1 = -Alo; v.y0 = -Bhi; v.y1 = -Blo; }
  else { v.x0 = -Bhi; v.x1 = -Blo; v.y0 = Alo; v.y1 = Ahi; }
  return v;
}

template <typename R> __device__ inline R rmin2_of(const VBox<R>& v) {
  R z = (R)0;
  R dx = v.x0 > z ? v.x0 : (v.x1 < z ? -v.x1 : z);
  R dy = v.y0 > z ? v.y0 : (v.y1 < z ? -v.y1 : z);
  return dx * dx + dy * dy;
}
template <typename R> __device__ inline R rmax2_of(const VBox<R>& v) {
  R a = v.x0 * v.x0, b = v.x1 * v.x1, c = v.y0 * v.y0, d = v.y1 * v.y1;
  return (a > b ? a : b) + (c > d ? c : d);
}

// silhouette corners: V's angular span runs from (ax,ay) counter-clockwise to
// (bx,by); returns false when V holds the apex.  The corner of each case
// (V right of, left of or across the vertical axis, and above, below or
// across the horizontal one) is picked by selects, without branches.
template <typename R>
__device__ inline bool silhouette(const VBox<R>& v, R& ax, R& ay, R& bx, R& by) {
  const R z = (R)0;
  const bool right = v.x0 > z, left = v.x1 < z, up = v.y0 > z, down = v.y1 < z;
  ax = (up || (left && !down)) ? v.x1 : v.x0;
  ay = (left || (!right && down)) ? v.y1 : v.y0;
  bx = (down || (left && !up)) ? v.x1 : v.x0;
  by = (right || (!left && down)) ? v.y1 : v.y0;
  return right || left || up || down;
}

// kappa-half edge directions of one kappa interval [Llo, Lhi] for one
// surface: e_lo = (1 - Llo xi, Llo + xi), e_hi likewise, and (binary32) the
// magnitudes that scale their certified cross-product bounds
template <typename R> struct KEdge { R pl, ph, elx, ely, ehx, ehy; };
template <typename R> __device__ inline KEdge<R> kedge(R xi, R Llo, R Lhi) {
  KEdge<R> e;
  e.pl = Llo * xi;
  e.ph = Lhi * xi;
  e.elx = (R)1 - e.pl;
  e.ely = Llo + xi;
  e.ehx = (R)1 - e.ph;
  e.ehy = Lhi + xi;
  return e;
}

// z-half in binary64: z = W3 - eta r over r in [r_min, r_max] must reach
// [Zlo - pad, Zhi + pad]; ZH = Zhi + pad, ZL = Zlo - pad.
__device__ inline bool zhalf64(double W3, double eta, double rmin2, double rmax2, double ZH, double ZL) {
  double Glo = W3 - ZH, Ghi = W3 - ZL;
  double Tlo, Thi, a;
  if (eta >= 0.0) { Tlo = Glo; Thi = Ghi; a = eta; }
  else { Tlo = -Ghi; Thi = -Glo; a = -eta; }
  double a2 = a * a;
  bool lo_ok = (Tlo <= 0.0) || (a2 * rmax2 >= Tlo * Tlo);
  bool hi_ok = (Thi >= 0.0) && (a2 * rmin2 <= Thi * Thi);
  return lo_ok && hi_ok;
}

// z-half terms that do not depend on the (x, y) part of the child: the
// signed reach of the surface's height range against the child's padded z
// interval, oriented so that the slope a = |eta| is non-negative
template <typename R> struct ZPre { R Tlo, Thi, a2, Ylo, Yhi; };
template <typename R> __device__ inline ZPre<R> zpre(R W3, R eta, R ZH, R ZL) {
  ZPre<R> z;
  const R Glo = W3 - ZH, Ghi = W3 - ZL;
  R a;
  if (eta >= (R)0) { z.Tlo = Glo; z.Thi = Ghi; a = eta; }
  else { z.Tlo = -Ghi; z.Thi = -Glo; a = -eta; }
  z.a2 = a * a;
  z.Ylo = z.Tlo * z.Tlo;
  z.Yhi = z.Thi * z.Thi;
  return z;
}
__device__ inline bool zhalf64p(const ZPre<double>& z, double rmin2, double rmax2) {
  const bool lo_ok = (z.Tlo <= 0.0) || (z.a2 * rmax2 >= z.Ylo);
  const bool hi_ok = (z.Thi >= 0.0) && (z.a2 * rmin2 <= z.Yhi);
  return lo_ok && hi_ok;
}

// kappa-half in binary64: the cone of directions with kappa in [Llo, Lhi]
// (kappa = (v2 - xi v1)/(v1 + xi v2), v1 + xi v2 > 0) meets V.
__device__ inline bool khalf64e(const VBox<double>& v, double rmin2, double Rg2, const KEdge<double>& e) {
  if (rmin2 < Rg2) return true;  // apex guard
  double ax, ay, bx, by;
  if (!silhouette(v, ax, ay, bx, by)) return true;
  double c1 = e.elx * ay - e.ely * ax;  // cross(e_lo, a)
  double c2 = ax * e.ehy - ay * e.ehx;  // cross(a, e_hi)
  double c3 = e.elx * by - e.ely * bx;  // cross(e_lo, b)
  double c4 = bx * e.ehy - by * e.ehx;  // cross(b, e_hi)
  return (c1 >= 0.0 && c2 >= 0.0) || (c3 >= 0.0 && c4 >= 0.0) || (c1 <= 0.0 && c3 >= 0.0) ||
         (c2 >= 0.0 && c4 <= 0.0);
}
__device__ inline bool khalf64(const VBox<double>& v, double rmin2, double Rg2, double xi, double Llo,
                               double Lhi) {
  return khalf64e(v, rmin2, Rg2, kedge<double>(xi, Llo, Lhi));
}

// binary32 filters: each decides meets / misses, or reports the half as
// undecided when a binary32 value lies within its certified error bound of
// the threshold.  Inputs are exact in binary32 (checked per problem on the
// host).  Each certified sign is a pair of comparisons (v > bound: positive,
// v < -bound: negative, neither: undecided), kept as lane masks so that the
// logic combining them runs on the scalar unit.
#define GV_U32 5.9604644775390625e-08f  // 2^-24

// z-half: returns whether it passes; *und = undecided (recheck in binary64).
__device__ inline bool zhalf32m(const ZPre<float>& z, float rmin2, float rmax2, bool& und) {
  const float X = z.a2 * rmax2;
  const float dl = X - z.Ylo, bl = 8.0f * GV_U32 * (X + z.Ylo);
  const bool lo_t = z.Tlo <= 0.0f;
  const bool lp = lo_t || dl > bl, ln = !lo_t && dl < -bl;
  const float X2 = z.a2 * rmin2;
  const float dh = z.Yhi - X2, bh = 8.0f * GV_U32 * (X2 + z.Yhi);
  const bool hneg = z.Thi < 0.0f;
  const bool hp = !hneg && dh > bh, hn = hneg || dh < -bh;
  const bool pass = lp && hp;
  und = !(ln || hn) && !pass;
  return pass;
}

// kappa-half: returns whether it passes; *und = undecided.  kSl, kSh: the
// cross products' bound factors 8u (|p| + |e_x| + |e_y|) of e_lo and e_hi.
__device__ inline bool khalf32m(const VBox<float>& v, float rmin2, float Rg2, const KEdge<float>& e, float kSl,
                                float kSh, bool& und) {
  const float gv = Rg2 - rmin2, gb = 4.0f * GV_U32 * (Rg2 + rmin2);
  const bool gpos = gv > gb, gneg = gv < -gb;  // apex guard certified either way
  float ax, ay, bx, by;
  const bool sil = silhouette(v, ax, ay, bx, by);
  const float Na = fabsf(ax) + fabsf(ay), Nb = fabsf(bx) + fabsf(by);
  const float v1 = e.elx * ay - e.ely * ax, b1 = kSl * Na;  // cross(e_lo, a)
  const float v2 = ax * e.ehy - ay * e.ehx, b2 = kSh * Na;  // cross(a, e_hi)
  const float v3 = e.elx * by - e.ely * bx, b3 = kSl * Nb;  // cross(e_lo, b)
  const float v4 = bx * e.ehy - by * e.ehx, b4 = kSh * Nb;  // cross(b, e_hi)
  const bool p1 = v1 > b1, n1 = v1 < -b1, p2 = v2 > b2, n2 = v2 < -b2;
  const bool p3 = v3 > b3, n3 = v3 < -b3, p4 = v4 > b4, n4 = v4 < -b4;
  const bool und_c = !(p1 || n1) || !(p2 || n2) || !(p3 || n3) || !(p4 || n4);
  const bool r = (p1 && p2) || (p3 && p4) || (n1 && p3) || (p2 && n4);
  und = !gpos && (!gneg || (sil && und_c));
  return gpos || (gneg && (!sil || r));
}
// magnitudes bounding the rounding of the cross products with e_lo, e_hi
__device__ inline float kedge_sl(const KEdge<float>& e) { return fabsf(e.pl) + fabsf(e.elx) + fabsf(e.ely); }
__device__ inline float kedge_sh(const KEdge<float>& e) { return fabsf(e.ph) + fabsf(e.ehx) + fabsf(e.ehy); }
