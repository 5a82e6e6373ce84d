// gvote.hip -- MI355X general-voting library: C ABI, host runtime and the
// root / replay kernels.  See include/gvote.h for the interface.
//
// Pipeline of one solve (Alg. 2 of Aiger et al., ICCV 2021):
//   front end (Eq. 1-3, the posing surface) -> root canonization
//   -> greedy dive (an achieved leaf key seeds the pruning bound)
//   -> depth-first over batches of same-level cells: incidence test + counts,
//      prune against the best key, compaction + canonization into the
//      children's lists, best-key atomic max at the leaves
//   -> inliers by per-surface replay along the chosen leaf's path.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <map>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gvote.h"
#include "gv_device.h"
#include "gv_kernels.h"

// ===========================================================================
// Root kernels
// ===========================================================================
struct Cols {
  const double* c[6];
};

__device__ inline void atomic_max_f64_pos(unsigned long long* a, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
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
    // root: translate by the zero corner, round to the free step s_f
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

__global__ void k_pose_bounds(const ProbC* __restrict__ Pp, Cols cols, int64_t n, unsigned long long* __restrict__ mx,
                              int* __restrict__ bad) {
  const ProbC& P = *Pp;
  double H = 0.0, R2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double t[4], f[2];
    int32_t tag;
    if (!front_eval(FAM_POSE4DOF, cols.c, i, P, t, f, &tag)) {
      atomicOr(bad, 1);
      continue;
    }
    double h = fabs(t[3]);
    H = h > H ? h : H;
    double a0 = t[0] * t[0], a1 = (t[0] - 1.0) * (t[0] - 1.0);
    double b0 = t[1] * t[1], b1 = (t[1] - 1.0) * (t[1] - 1.0);
    double r2 = (a0 > a1 ? a0 : a1) + (b0 > b1 ? b0 : b1);
    R2 = r2 > R2 ? r2 : R2;
  }
  atomic_max_f64_pos(&mx[0], H);
  atomic_max_f64_pos(&mx[1], R2);
}

// quantize once at the root to the fixed pose lattice
__global__ void k_root_pose(const ProbC* __restrict__ Pp, Cols cols, int64_t n, double* __restrict__ m64,
                            EntQ32* __restrict__ e32, EntQ64* __restrict__ e64, unsigned long long* __restrict__ mx) {
  const ProbC& P = *Pp;
  double a[5] = {0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double t[4], f[2];
    int32_t tag;
    front_eval(FAM_POSE4DOF, cols.c, i, P, t, f, &tag);
    double W1 = rint(t[0] * P.inv_sW) * P.sW;
    double W2 = rint(t[1] * P.inv_sW) * P.sW;
    double W3 = rint(f[0] * P.inv_sW3) * P.sW3;
    double xi = rint(t[2] * P.inv_sXi) * P.sXi;
    double eta = rint(t[3] * P.inv_sEta) * P.sEta;
    m64[i] = W1;
    m64[n + i] = W2;
    m64[2 * n + i] = W3;
    m64[3 * n + i] = xi;
    m64[4 * n + i] = eta;
    if (e32) e32[i] = EntQ32{(float)W1, (float)W2, (float)W3, (float)xi, (float)eta, 1u, (uint32_t)i, 0u};
    if (e64) e64[i] = EntQ64{W1, W2, W3, xi, eta, 1u, (uint32_t)i};
    double v[5] = {fabs(W1), fabs(W2), fabs(W3), fabs(xi), fabs(eta)};
    for (int k = 0; k < 5; k++) a[k] = v[k] > a[k] ? v[k] : a[k];
  }
  for (int k = 0; k < 5; k++) atomic_max_f64_pos(&mx[2 + k], a[k]);
}

template <typename E>
__global__ void k_replicate(const E* __restrict__ src, int64_t n, int nsec, E* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * nsec; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i % n];
}

// root cells: one per sector s0 .. s0+ncell-1; lists either back to back
// (shared == 0) or all the same list at offset 0
__global__ void k_root_cells(Cell* cells, int ncell, int s0, uint64_t n, int shared) {
  int k = threadIdx.x;
  if (k < ncell) {
    Cell c;
    c.c[0] = c.c[1] = c.c[2] = c.c[3] = 0;
    c.prefix = (uint64_t)(s0 + k);
    c.off = shared ? 0 : (uint64_t)k * n;
    c.len = (uint32_t)n;
    c.sector = (uint32_t)(s0 + k);
    cells[k] = c;
  }
}

// ===========================================================================
// Replay: every original surface's canonization chain along the chosen
// leaf's root-to-leaf path; it is an inlier iff every test on the path passes
// (member tracking, Sec. 3.2.1).
// ===========================================================================
struct PathC {
  uint8_t digit[GV_MAXL];
  int32_t sector;
};

template <int FAM>
__global__ void k_replay_lin(const ProbC* __restrict__ Pp, Cols cols, int64_t n, PathC path, uint32_t* __restrict__ flag,
                             int* __restrict__ bad) {
  const ProbC& P = *Pp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    LinS s;
    uint32_t ok = 0;
    if (root_lin<FAM>(P, cols.c, i, s, bad)) {
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

__global__ void k_replay_pose(const ProbC* __restrict__ Pp, const double* __restrict__ m64, int64_t n, PathC path,
                              uint32_t* __restrict__ flag) {
  const ProbC& P = *Pp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double W1 = m64[i], W2 = m64[n + i], W3 = m64[2 * n + i], xi = m64[3 * n + i], eta = m64[4 * n + i];
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

__global__ void k_write_inliers(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos, int64_t n,
                                int64_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (flag[i]) out[pos[i]] = i;
}

// ===========================================================================
// Host runtime
// ===========================================================================
// Caching device allocator owned by a context.  All library work on a
// context is ordered on its stream, so a block released after its last use
// was enqueued can be handed to any later allocation on that stream without a
// synchronization.  Sizes are rounded to 8 classes per power of two.
struct DevCache {
  std::multimap<size_t, void*> free_blocks;
  std::map<void*, size_t> live;
  uint64_t cached = 0, in_use = 0, peak = 0;

  static size_t round(size_t b) {
    if (b <= 4096) return 4096;
    int e = 63 - __builtin_clzll((unsigned long long)b);  // 2^e <= b < 2^(e+1)
    size_t step = (size_t)1 << (e >= 3 ? e - 3 : 0);
    return (b + step - 1) / step * step;
  }
  void* get(size_t bytes, hipStream_t st, std::string& err) {
    const size_t r = round(bytes);
    auto it = free_blocks.lower_bound(r);
    if (it != free_blocks.end() && it->first <= r + r / 4) {
      void* p = it->second;
      live[p] = it->first;
      in_use += it->first;
      cached -= it->first;
      free_blocks.erase(it);
      peak = std::max(peak, in_use);
      return p;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim(st);
      e = hipMalloc(&p, r);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        err = std::string("hipMalloc: ") + hipGetErrorString(e);
        return nullptr;
      }
    }
    live[p] = r;
    in_use += r;
    peak = std::max(peak, in_use);
    return p;
  }
  void put(void* p) {
    auto it = live.find(p);
    if (it == live.end()) return;
    free_blocks.emplace(it->second, p);
    cached += it->second;
    in_use -= it->second;
    live.erase(it);
  }
  void trim(hipStream_t st) {
    (void)hipStreamSynchronize(st);
    for (auto& kv : free_blocks) (void)hipFree(kv.second);
    free_blocks.clear();
    cached = 0;
  }
};

struct gv_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t budget = 0;
  std::mutex mu;
  std::string err;
  int n_cu = 256;
  DevCache cache;
  bool kernel_timing = false;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

thread_local std::string tl_err;

struct DevErr {
  gv_status st;
};

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) {                                                            \
      X.ctx->err = std::string(#x) + ": " + hipGetErrorString(e_);                     \
      throw DevErr{GV_EDEVICE};                                                        \
    }                                                                                  \
  } while (0)

struct Setup {
  ProbC P;
  int fam, d, ell;
  double epsn[4];
  double ez, ek;  // pose eps'
  bool filter;    // binary32 filter usable
  int64_t n;
};

// largest power of two <= x
double p2floor(double x) {
  int e;
  (void)std::frexp(x, &e);
  return std::ldexp(1.0, e - 1);
}

gv_status setup_axes(const gv_problem* p, Setup& S, std::string& why) {
  std::memset(&S, 0, sizeof(S));
  ProbC& P = S.P;
  S.fam = (int)p->family;
  S.n = p->n;
  if (p->n < 0 || p->n > 0x7fffffffLL) { why = "n out of range"; return GV_EINVAL; }
  switch (S.fam) {
    case GV_LINE2D: S.d = 2; S.ell = 1; break;
    case GV_PLANE3D: S.d = 3; S.ell = 2; break;
    case GV_RAY3D: S.d = 3; S.ell = 2; break;
    case GV_POSE4DOF: S.d = 4; S.ell = 4; break;
    default: why = "bad family"; return GV_EINVAL;
  }
  P.fam = S.fam;
  P.d = S.d;
  P.nsec = S.fam == GV_POSE4DOF ? 4 : 1;
  double c = p->canon_c == 0.0 ? 1.0 : p->canon_c;
  if (!(c > 0.0) || std::isnan(c)) { why = "canon_c must be > 0"; return GV_EINVAL; }
  if (std::isinf(c)) { why = "exact mode (canon_c = inf) is not available on the device path"; return GV_EINVAL; }
  int nuser = S.fam == GV_POSE4DOF ? 3 : S.d;
  for (int j = 0; j < nuser; j++) {
    if (!std::isfinite(p->lo[j]) || !std::isfinite(p->hi[j]) || !(p->hi[j] > p->lo[j])) { why = "bad box"; return GV_EINVAL; }
    if (!std::isfinite(p->eps[j]) || !(p->eps[j] > 0.0)) { why = "bad eps"; return GV_EINVAL; }
    P.lo[j] = p->lo[j];
    P.E[j] = p->hi[j] - p->lo[j];
    P.inv[j] = 1.0 / P.E[j];
    S.epsn[j] = p->eps[j] * P.inv[j];
  }
  double epsk = 0.0;
  if (S.fam == GV_POSE4DOF) {
    if (P.E[0] != P.E[1]) { why = "POSE4DOF needs hi[0]-lo[0] == hi[1]-lo[1]"; return GV_EINVAL; }
    if (!std::isfinite(p->eps[3]) || !(p->eps[3] > 0.0)) { why = "bad yaw eps"; return GV_EINVAL; }
    epsk = p->eps[3];
    P.lo[3] = -1.0;
    P.E[3] = 2.0;
    P.inv[3] = 0.5;
    S.epsn[3] = epsk * 0.5;
    P.ce = P.E[0] * P.inv[2];
  }
  int Lstar = 0, Bcell = 0;
  for (int j = 0; j < S.d; j++) {
    double ej = (S.fam == GV_POSE4DOF && j == 3) ? epsk : p->eps[j];
    int L = 0;
    while (std::ldexp(P.E[j], -L) > ej) {
      if (++L > 30) { why = "eps too small for the box"; return GV_EINVAL; }
    }
    P.L[j] = L;
    Lstar = std::max(Lstar, L);
    Bcell += L;
  }
  if (Lstar < 1) { why = "eps covers the whole box"; return GV_EINVAL; }
  if (Lstar > GV_MAXL) { why = "too many levels"; return GV_EINVAL; }
  P.Lstar = Lstar;
  P.Bcell = Bcell;
  P.B = Bcell + (S.fam == GV_POSE4DOF ? 2 : 0);
  if (P.B > 62) { why = "leaf index does not fit 62 bits"; return GV_EINVAL; }
  if ((uint64_t)p->n >= (1ULL << (64 - P.B))) { why = "n too large for the key"; return GV_EINVAL; }
  P.idxmask = (1ULL << P.B) - 1ULL;
  int rem[GV_MAXL + 1];
  rem[Lstar] = 0;
  int ab[GV_MAXL];
  for (int m = 0; m < Lstar; m++) {
    int a = 0;
    for (int j = 0; j < S.d; j++)
      if (m < P.L[j]) a++;
    ab[m] = a;
  }
  for (int m = Lstar - 1; m >= 0; m--) rem[m] = rem[m + 1] + ab[m];
  for (int m = 0; m < Lstar; m++) {
    LevelC& lv = P.lev[m];
    std::memset(&lv, 0, sizeof(lv));
    lv.abits = ab[m];
    lv.rem_next = rem[m + 1];
    int splits[4], ns = 0;
    for (int j = 0; j < 4; j++) {
      lv.split[j] = (j < S.d && m < P.L[j]) ? 1 : 0;
      if (lv.split[j]) splits[ns++] = j;
    }
    // child digit: split axes' bits in axis order, most significant first
    for (int dg = 0; dg < (1 << ab[m]); dg++) {
      uint8_t cb = 0;
      for (int k = 0; k < ns; k++)
        if ((dg >> (ns - 1 - k)) & 1) cb |= (uint8_t)(1u << splits[k]);
      lv.cbits[dg] = cb;
    }
  }
  if (S.fam != GV_POSE4DOF) {
    for (int q = 0; q < S.d; q++) {
      double ep = S.epsn[q] / (c * (double)(Lstar + 1));
      P.sf[q] = p2floor(ep / (double)(S.ell + 1));
      P.inv_sf[q] = 1.0 / P.sf[q];
      if (!(P.sf[q] > 0.0) || P.sf[q] < std::ldexp(1.0, -29)) { why = "lattice too fine for 32-bit cells"; return GV_ERANGE; }
      for (int m = 0; m < Lstar; m++) {
        double Em = (double)((m + 1) * (S.ell + 1)) * P.sf[q] * 0.5;
        double padc = std::ceil((S.epsn[q] + Em) / P.sf[q]);  // pad in units of s_f
        double H = std::ldexp(1.0, -std::min(m, P.L[q])) * P.inv_sf[q];
        if (padc * 2.0 > 1e9 || H > 1e9) { why = "lattice too fine for 32-bit cells"; return GV_ERANGE; }
        P.lev[m].padu[q] = (int32_t)(2.0 * padc);
        P.lev[m].H[q] = (int32_t)H;
      }
    }
  } else {
    S.ez = S.epsn[2] / (c * (double)(Lstar + 1));
    S.ek = epsk / (c * (double)(Lstar + 1));
  }
  return GV_OK;
}

// POSE4DOF lattice from the data bounds (same definition as the oracle)
void pose_lattice(Setup& S, double Hmax, double R2, double epsk) {
  ProbC& P = S.P;
  int Lxy = std::max(P.L[0], P.L[1]);
  double Rg = std::ldexp(1.0, -Lxy);
  P.Rg2 = Rg * Rg;
  double l1 = (double)(S.ell + 1);
  double Hb = (Hmax > 0x1p-10 ? Hmax : 0x1p-10) * (1.0 + 0x1p-20);
  double Rb = (std::sqrt(R2) + 0x1p-20) * (1.0 + 0x1p-20);
  double pk0 = epsk + S.ek * 0.5;
  double Bk = 1.0 + (1.0 + pk0) * (1.0 + pk0);
  P.sW3 = p2floor(S.ez / l1);
  P.sEta = p2floor(S.ez / (l1 * Rb));
  double wz = S.ez / (l1 * Hb), wk = (S.ek * Rg) / (l1 * Bk);
  P.sW = p2floor(wz < wk ? wz : wk);
  P.sXi = p2floor(S.ek / (l1 * Bk));
  P.padz = std::ceil((S.epsn[2] + S.ez * 0.5) / P.sW3) * P.sW3;
  P.padk = std::ceil((epsk + S.ek * 0.5) / P.sXi) * P.sXi;
  P.inv_sW = 1.0 / P.sW;
  P.inv_sW3 = 1.0 / P.sW3;
  P.inv_sXi = 1.0 / P.sXi;
  P.inv_sEta = 1.0 / P.sEta;
  P.Rg2f = (float)P.Rg2;
  P.padzf = (float)P.padz;
  P.padkf = (float)P.padk;
}

// binary32 evaluation is exact on the inputs iff every lattice value and
// every difference the filter forms fits 24 significant bits
bool pose_filter_exact(const Setup& S, const double* mx) {
  const ProbC& P = S.P;
  const double T = 16777216.0;  // 2^24
  double W12 = std::max(mx[2], mx[3]);
  if (P.L[0] > 23 || P.L[1] > 23 || P.L[2] > 23 || P.L[3] > 22) return false;
  if (!(W12 + 1.0 < T * P.sW)) return false;
  if (!(mx[4] + 1.0 + P.padz + 1.0 < T * std::min(P.sW3, std::ldexp(1.0, -P.L[2])))) return false;
  if (!(mx[5] < T * P.sXi)) return false;
  if (!(mx[6] < T * P.sEta)) return false;
  if (!(1.0 + P.padk < T * std::min(P.sXi, std::ldexp(1.0, -(P.L[3] - 1))))) return false;
  if (P.sW < 0x1p-40 || P.sEta < 0x1p-40 || P.sXi < 0x1p-40) return false;
  return true;
}

struct Batch {
  int level;
  uint32_t ncell;
  uint64_t nent;
  Cell* cells;
  void* ents;
  bool unit = true;  // every multiplicity is 1
};

struct Run {
  gv_ctx* ctx;
  hipStream_t st;
  Setup S;
  int group_mode = 0;
  double lat_bound[GV_MAXL + 1];  // canonical surfaces a cell of level m can hold (linear)
  ProbC* dP = nullptr;
  unsigned long long* dbest = nullptr;
  unsigned long long* drecheck = nullptr;
  uint64_t* dtot = nullptr;
  uint32_t* dummy = nullptr;    // sink for outputs a leaf-level pass does not need
  unsigned long long* dreads = nullptr;  // parent entries read by compaction passes
  size_t ent_bytes = 0;                  // entry + mask bytes of this run
  uint64_t budget_entries = 0;  // max entries of one materialized chunk
  uint64_t first_cells = 65536;  // cells in the first chunk of every expansion
  bool trace = false;            // GV_TRACE=1: one stderr line per expansion
  bool beam = true;              // progressive chunks until the first leaf level
  // kernel timing: (start, stop, kind 0 test / 1 compact)
  std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>> ev;
  size_t ev_used = 0;
  gv_stats stats{};
  double* m64 = nullptr;  // pose master
  int64_t n = 0;
};

template <typename T>
T* dalloc(Run& X, size_t count) {
  if (count == 0) count = 1;
  void* p = X.ctx->cache.get(count * sizeof(T), X.st, X.ctx->err);
  if (!p) throw DevErr{GV_ENOMEM};
  return (T*)p;
}
void dfree(Run& X, void* p) {
  if (p) X.ctx->cache.put(p);
}

template <typename In, typename Out>
void excl_scan(Run& X, const In* in, Out* out, uint64_t n) {
  if (n == 0) return;
  size_t tb = 0;
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, in, out, (int)n, X.st));
  void* tmp = dalloc<char>(X, tb);
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(tmp, tb, in, out, (int)n, X.st));
  dfree(X, tmp);
}

inline unsigned nblk(uint64_t n, unsigned b = 256) { return (unsigned)std::max<uint64_t>(1, (n + b - 1) / b); }
inline unsigned gs_grid(Run& X, uint64_t n) {
  return (unsigned)std::min<uint64_t>(nblk(n), (uint64_t)X.ctx->n_cu * 16);
}

// Expansion state of a batch whose kept children are materialized later,
// one chunk of the count-sorted order at a time.
struct Parent {
  int level = 0;
  uint32_t ncell = 0;
  uint64_t nent = 0;
  Cell* cells = nullptr;
  void* ents = nullptr;
  bool own_ents = false;
  void* masks = nullptr;
  Item* items = nullptr;
  uint32_t* nitems = nullptr;
  uint64_t max_items = 0;
  uint32_t nkept = 0;
  uint32_t* order = nullptr;    // rank -> child (cell * nch + digit)
  uint32_t* scount = nullptr;   // rank -> count (descending)
  uint32_t* rank_of = nullptr;  // child -> rank (or ~0)
  uint64_t* soff = nullptr;     // rank -> first entry (nkept + 1 values)
  uint32_t* cnent = nullptr;    // child -> entries
  uint32_t* ioff = nullptr;     // cell -> its first item
  uint64_t* itemoff = nullptr;  // child-major exclusive scan of per-item survivors
  uint32_t istride = 0;
  int pending = 0;
  bool sorted = true;           // children in descending count order
  bool unit = true;             // every multiplicity is 1
};

struct Task {
  bool chunk;
  Batch b;
  Parent* par;
  uint32_t r0, r1;
};

void free_parent(Run& X, Parent* pa) {
  dfree(X, pa->cells);
  if (pa->own_ents) dfree(X, pa->ents);
  dfree(X, pa->masks);
  dfree(X, pa->items);
  dfree(X, pa->nitems);
  dfree(X, pa->order);
  dfree(X, pa->scount);
  dfree(X, pa->rank_of);
  dfree(X, pa->soff);
  dfree(X, pa->cnent);
  dfree(X, pa->ioff);
  dfree(X, pa->itemoff);
  delete pa;
}

template <typename T>
uint64_t d2h1(Run& X, const T* p) {
  T v{};
  HIPCHK(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  return (uint64_t)v;
}

std::pair<hipEvent_t, hipEvent_t> ev_begin(Run& X, int kind) {
  gv_ctx* c = X.ctx;
  std::pair<hipEvent_t, hipEvent_t> p{nullptr, nullptr};
  if (!c->kernel_timing) return p;
  while (c->ev_pool.size() < 2 * (X.ev_used + 1)) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  p.first = c->ev_pool[2 * X.ev_used];
  p.second = c->ev_pool[2 * X.ev_used + 1];
  X.ev_used++;
  HIPCHK(hipEventRecord(p.first, X.st));
  X.ev.push_back({p, kind});
  return p;
}
void ev_end(Run& X, std::pair<hipEvent_t, hipEvent_t> p) {
  if (p.second) HIPCHK(hipEventRecord(p.second, X.st));
}

// Grouping of a batch's lists: sort by (cell, tuple hash), merge equal
// tuples, sum multiplicities.  Replaces b.ents (freed if owned) and the
// cells' offsets and lengths.
template <typename E>
void group_batch(Run& X, Batch& b, bool own_ents) {
  const uint64_t n = b.nent;
  if (n < 2) return;
  const int cbits = b.ncell <= 1 ? 0 : 64 - __builtin_clzll((unsigned long long)(b.ncell - 1));
  const int hb = 64 - cbits;
  uint64_t* k0 = dalloc<uint64_t>(X, n);
  uint32_t* i0 = dalloc<uint32_t>(X, n);
  uint64_t* k1 = dalloc<uint64_t>(X, n);
  uint32_t* i1 = dalloc<uint32_t>(X, n);
  k_group_keys<E><<<nblk(n), 256, 0, X.st>>>(b.cells, b.ncell, (const E*)b.ents, n, hb, k0, i0);
  {
    size_t tb = 0;
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k0, k1, i0, i1, (int)n, 0, 64, X.st));
    void* tmp = dalloc<char>(X, tb);
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, k0, k1, i0, i1, (int)n, 0, 64, X.st));
    dfree(X, tmp);
  }
  dfree(X, k0);
  dfree(X, i0);
  uint32_t* head = dalloc<uint32_t>(X, n);
  uint32_t* hscan = dalloc<uint32_t>(X, n);
  k_group_heads<E><<<nblk(n), 256, 0, X.st>>>(k1, i1, (const E*)b.ents, n, head);
  excl_scan(X, head, hscan, n);
  uint32_t last[2];
  HIPCHK(hipMemcpyAsync(&last[0], hscan + n - 1, 4, hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipMemcpyAsync(&last[1], head + n - 1, 4, hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  const uint64_t U = (uint64_t)last[0] + last[1];
  if (U < n) {
    E* out = dalloc<E>(X, U);
    uint32_t* newlen = dalloc<uint32_t>(X, b.ncell);
    uint32_t* newoff = dalloc<uint32_t>(X, b.ncell);
    HIPCHK(hipMemsetAsync(newlen, 0, b.ncell * sizeof(uint32_t), X.st));
    k_group_write<E><<<nblk(n), 256, 0, X.st>>>(k1, i1, (const E*)b.ents, n, head, hscan, hb, out, newlen);
    excl_scan(X, newlen, newoff, b.ncell);
    k_group_cells<<<nblk(b.ncell), 256, 0, X.st>>>(b.cells, b.ncell, newlen, newoff);
    dfree(X, newlen);
    dfree(X, newoff);
    if (own_ents) dfree(X, b.ents);
    b.ents = out;
    b.nent = U;
    b.unit = false;
    X.stats.groups_merged += n - U;
  }
  dfree(X, k1);
  dfree(X, i1);
  dfree(X, head);
  dfree(X, hscan);
}

// merge when the lists outgrow the number of canonical surfaces their cells
// can hold (linear families; POSE4DOF surfaces do not change below the root)
bool want_group(const Run& X, const Batch& b) {
  if (X.group_mode < 0 || b.nent < 2) return false;
  if (X.group_mode > 0) return true;
  if (X.S.fam == GV_POSE4DOF) return false;
  const double avg = (double)b.nent / (double)std::max<uint32_t>(1, b.ncell);
  return avg >= 0.5 * X.lat_bound[b.level];
}

// One expansion: incidence test and per-child counts, pruning against the
// best key (or, for the greedy dive, keeping only the best child), then the
// kept children sorted by count.  Returns nullptr when nothing is kept (or at
// the last level, where the leaf keys went into the best-key reduction).
// The batch's cells/entries are handed over to the Parent (or freed).
template <int FAM, typename E, typename M>
Parent* expand(Run& X, Batch& b, bool own_ents, bool dive) {
  const ProbC& P = X.S.P;
  const int m = b.level;
  const LevelC lv = P.lev[m];
  const uint32_t nch = 1u << lv.abits;
  const bool leaf = (m + 1 == P.Lstar);
  const uint64_t nk = (uint64_t)b.ncell * nch;
  X.stats.tests += b.nent * nch;
  X.stats.cells_expanded += b.ncell;

  Parent* pa = new Parent();
  pa->level = m;
  pa->ncell = b.ncell;
  pa->nent = b.nent;
  pa->cells = b.cells;
  pa->ents = b.ents;
  pa->own_ents = own_ents;
  pa->unit = b.unit;

  // work items: at most GV_ITEM entries of one cell each
  uint32_t* nitem = dalloc<uint32_t>(X, b.ncell);
  pa->ioff = dalloc<uint32_t>(X, b.ncell);
  pa->max_items = b.ncell + b.nent / GV_ITEM + 1;
  pa->items = dalloc<Item>(X, pa->max_items);
  pa->nitems = dalloc<uint32_t>(X, 1);
  HIPCHK(hipMemsetAsync(pa->nitems, 0, sizeof(uint32_t), X.st));
  k_item_counts<<<nblk(b.ncell), 256, 0, X.st>>>(b.cells, b.ncell, nitem);
  excl_scan(X, nitem, pa->ioff, b.ncell);
  k_item_fill<<<nblk(b.ncell), 256, 0, X.st>>>(b.cells, b.ncell, nitem, pa->ioff, pa->items, pa->nitems);
  dfree(X, nitem);
  pa->istride = (uint32_t)pa->max_items;
  uint32_t* itemcnt = leaf ? nullptr : dalloc<uint32_t>(X, (uint64_t)nch * pa->istride);
  if (itemcnt) HIPCHK(hipMemsetAsync(itemcnt, 0, (uint64_t)nch * pa->istride * sizeof(uint32_t), X.st));

  pa->masks = dalloc<M>(X, b.nent);
  uint32_t* ccnt = dalloc<uint32_t>(X, nk);
  pa->cnent = dalloc<uint32_t>(X, nk);
  HIPCHK(hipMemsetAsync(ccnt, 0, nk * sizeof(uint32_t), X.st));
  HIPCHK(hipMemsetAsync(pa->cnent, 0, nk * sizeof(uint32_t), X.st));
  const unsigned grid = (unsigned)std::min<uint64_t>((pa->max_items + 3) / 4, (uint64_t)X.ctx->n_cu * 8);
  auto evp = ev_begin(X, 0);
  X.stats.test_launches++;
  X.stats.test_bytes += b.nent * (sizeof(E) + sizeof(M));
  if constexpr (FAM == FAM_POSE4DOF) {
    k_count_pose<E><<<grid, 256, 0, X.st>>>(X.dP, m, lv, b.cells, pa->items, pa->nitems, (const E*)b.ents, X.m64,
                                             (uint64_t)X.n, (uint16_t*)pa->masks, ccnt, pa->cnent, X.drecheck,
                                             itemcnt ? itemcnt : X.dummy, itemcnt ? pa->istride : 0u);
  } else {
    if (b.unit)
      k_count_lin<FAM, true><<<grid, 256, 0, X.st>>>(lv, b.cells, pa->items, pa->nitems, (const E*)b.ents,
                                                      (uint8_t*)pa->masks, ccnt, pa->cnent,
                                                      itemcnt ? itemcnt : X.dummy, itemcnt ? pa->istride : 0u);
    else
      k_count_lin<FAM, false><<<grid, 256, 0, X.st>>>(lv, b.cells, pa->items, pa->nitems, (const E*)b.ents,
                                                       (uint8_t*)pa->masks, ccnt, pa->cnent,
                                                       itemcnt ? itemcnt : X.dummy, itemcnt ? pa->istride : 0u);
  }
  ev_end(X, evp);
  HIPCHK(hipGetLastError());

  uint32_t* keepf = dalloc<uint32_t>(X, nk);
  uint64_t* keptn = dalloc<uint64_t>(X, nk);
  if (dive) {
    k_pick_best<<<1, 64, 0, X.st>>>(lv, P.B, P.idxmask, leaf ? 1 : 0, b.cells, ccnt, pa->cnent, X.dbest, keepf, keptn);
  } else {
    k_prune<<<nblk(nk), 256, 0, X.st>>>(lv, P.B, P.idxmask, leaf ? 1 : 0, b.cells, b.ncell, ccnt, pa->cnent,
                                        X.dbest, keepf, keptn);
  }
  HIPCHK(hipGetLastError());
  dfree(X, keptn);
  if (leaf) {
    if (!dive) X.beam = false;
    dfree(X, keepf);
    dfree(X, ccnt);
    pa->pending = 0;
    free_parent(X, pa);
    return nullptr;
  }
  uint32_t* keepscan = dalloc<uint32_t>(X, nk);
  excl_scan(X, keepf, keepscan, nk);
  k_kept_total<<<1, 64, 0, X.st>>>(keepf, keepscan, nk, X.dtot);
  const uint64_t nkept = d2h1(X, X.dtot);
  X.stats.cells_pruned += nk - nkept;
  if (X.trace) {
    const uint64_t bst = d2h1(X, X.dbest);
    std::fprintf(stderr, "gv: level %d cells %u entries %llu kept %llu best %llu%s\n", m, b.ncell,
                 (unsigned long long)b.nent, (unsigned long long)nkept, (unsigned long long)(bst >> P.B),
                 dive ? " (dive)" : "");
  }
  if (nkept == 0) {
    dfree(X, keepf);
    dfree(X, keepscan);
    dfree(X, ccnt);
    dfree(X, itemcnt);
    free_parent(X, pa);
    return nullptr;
  }
  pa->itemoff = dalloc<uint64_t>(X, (uint64_t)nch * pa->istride);
  excl_scan(X, itemcnt, pa->itemoff, (uint64_t)nch * pa->istride);
  dfree(X, itemcnt);
  pa->nkept = (uint32_t)nkept;
  uint32_t* kcnt = dalloc<uint32_t>(X, nkept);
  uint32_t* kid = dalloc<uint32_t>(X, nkept);
  k_select_kept<<<nblk(nk), 256, 0, X.st>>>(keepf, keepscan, ccnt, nk, kcnt, kid);
  dfree(X, keepf);
  dfree(X, keepscan);
  dfree(X, ccnt);
  // POSE4DOF keeps count order throughout: its bound keeps improving after
  // the first descent, and its incidence test (not the list traffic) dominates
  pa->sorted = X.beam || dive || FAM == FAM_POSE4DOF;
  if (!pa->sorted) {
    // after the first descent the bound is strong: keep parent order so that
    // a chunk is a contiguous range of parents, each read once
    pa->scount = kcnt;
    pa->order = kid;
    kcnt = kid = nullptr;
  } else {
    pa->scount = dalloc<uint32_t>(X, nkept);
    pa->order = dalloc<uint32_t>(X, nkept);
    size_t tb = 0;
    HIPCHK(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tb, kcnt, pa->scount, kid, pa->order, (int)nkept, 0,
                                                         32, X.st));
    void* tmp = dalloc<char>(X, tb);
    HIPCHK(hipcub::DeviceRadixSort::SortPairsDescending(tmp, tb, kcnt, pa->scount, kid, pa->order, (int)nkept, 0, 32,
                                                         X.st));
    dfree(X, tmp);
  }
  dfree(X, kcnt);
  dfree(X, kid);
  pa->rank_of = dalloc<uint32_t>(X, nk);
  HIPCHK(hipMemsetAsync(pa->rank_of, 0xff, nk * sizeof(uint32_t), X.st));
  uint32_t* sn = dalloc<uint32_t>(X, nkept);
  k_rank<<<nblk(nkept), 256, 0, X.st>>>(pa->order, (uint32_t)nkept, pa->cnent, pa->rank_of, sn);
  pa->soff = dalloc<uint64_t>(X, nkept + 1);
  excl_scan(X, sn, pa->soff, nkept);
  k_soff_last<<<1, 64, 0, X.st>>>(pa->soff, sn, (uint32_t)nkept);
  dfree(X, sn);
  return pa;
}

// Chunk schedule over the sorted children: chunk j holds at most
// first_cells * 4^j cells and at most budget entries, so the first descent
// follows a narrow beam of the highest-count cells.
void plan_chunks(Run& X, Parent* pa, std::vector<std::pair<uint32_t, uint32_t>>& chunks) {
  const uint32_t nk = pa->nkept;
  const uint64_t stride = std::max<uint64_t>(1, (nk + (1u << 20) - 1) >> 20);
  const uint64_t ns = (nk + stride - 1) / stride;  // samples soff[i*stride], plus soff[nk]
  uint64_t* d = dalloc<uint64_t>(X, ns + 1);
  k_gather_u64<<<nblk(ns + 1), 256, 0, X.st>>>(pa->soff, nk, stride, d);
  std::vector<uint64_t> s(ns + 1);
  HIPCHK(hipMemcpyAsync(s.data(), d, (ns + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  dfree(X, d);
  auto at = [&](uint64_t i) { return i >= ns ? s[ns] : s[i]; };  // sample i -> soff[min(i*stride, nk)]
  auto rk = [&](uint64_t i) { return (uint32_t)std::min<uint64_t>(i * stride, nk); };
  uint64_t i0 = 0, cap = X.beam ? X.first_cells : (1ull << 30);
  while (rk(i0) < nk) {
    uint64_t i1 = i0 + 1;
    while (i1 < ns && (rk(i1 + 1) - rk(i0)) <= cap && at(i1 + 1) - at(i0) <= X.budget_entries) i1++;
    chunks.push_back({rk(i0), rk(i1)});
    i0 = i1;
    cap = X.beam ? std::min<uint64_t>(cap * 4, 1ull << 30) : (1ull << 30);
  }
}

// Materialize one chunk [r0, r1) of a parent as a new batch (after cutting it
// against the current best).  Returns false when nothing remains.
template <int FAM, typename E, typename M>
bool materialize(Run& X, Parent* pa, uint32_t r0, uint32_t r1, Batch& nb) {
  const ProbC& P = X.S.P;
  const LevelC lv = P.lev[pa->level];
  k_chunk_cut<<<1, 64, 0, X.st>>>(pa->scount, pa->soff, r0, r1, X.dbest, P.B, pa->sorted ? 1 : 0, X.dtot);
  uint64_t cut[2];
  HIPCHK(hipMemcpyAsync(cut, X.dtot, sizeof(cut), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  const uint32_t rc = (uint32_t)cut[0];
  bool made = false;
  X.stats.cells_pruned += r1 - rc;
  if (rc > r0) {
    nb.level = pa->level + 1;
    nb.ncell = rc - r0;
    nb.nent = cut[1];
    nb.cells = dalloc<Cell>(X, nb.ncell);
    nb.ents = dalloc<E>(X, nb.nent);
    k_emit_ranked<<<nblk(nb.ncell), 256, 0, X.st>>>(lv, pa->cells, pa->order, pa->soff, r0, rc, pa->cnent, nb.cells);
    const unsigned grid = (unsigned)std::min<uint64_t>((pa->max_items + 3) / 4, (uint64_t)X.ctx->n_cu * 8);
    auto evp = ev_begin(X, 1);
    X.stats.compact_launches++;
    X.stats.compact_bytes += nb.nent * sizeof(E);
    if (X.ctx->kernel_timing)
      k_chunk_reads<<<nblk(pa->ncell), 256, 0, X.st>>>(pa->cells, pa->ncell, 1u << lv.abits, pa->rank_of, r0, rc,
                                                       X.dreads);
    k_compact<FAM, E, M, FAM == FAM_POSE4DOF><<<grid, 256, 0, X.st>>>(
        lv, pa->cells, pa->items, pa->nitems, pa->ioff, pa->itemoff, pa->istride, (const E*)pa->ents,
        (const M*)pa->masks, pa->rank_of, r0, rc, pa->soff, (E*)nb.ents);
    ev_end(X, evp);
    HIPCHK(hipGetLastError());
    nb.unit = pa->unit;
    made = true;
  }
  if (--pa->pending == 0) free_parent(X, pa);
  if (made && want_group(X, nb)) group_batch<E>(X, nb, true);
  return made;
}

template <int FAM, typename E, typename M>
void push_children(Run& X, Parent* pa, std::vector<Task>& stack) {
  std::vector<std::pair<uint32_t, uint32_t>> chunks;
  plan_chunks(X, pa, chunks);
  pa->pending = (int)chunks.size();
  for (auto it = chunks.rbegin(); it != chunks.rend(); ++it) {
    Task t{};
    t.chunk = true;
    t.par = pa;
    t.r0 = it->first;
    t.r1 = it->second;
    stack.push_back(t);
  }
}

template <int FAM, typename E, typename M>
void search(Run& X, E* root0, int64_t n0) {
  const ProbC& P = X.S.P;
  X.ent_bytes = sizeof(E) + sizeof(M);
  const int nsec = P.nsec;
  // root canonization is done; group equal root surfaces once for all sectors
  E* root = root0;
  uint64_t n = (uint64_t)n0;
  bool unit = true, own_root = false;
  if (X.group_mode >= 0 && n > 1) {
    Batch rb;
    rb.level = 0;
    rb.ncell = 1;
    rb.nent = n;
    rb.cells = dalloc<Cell>(X, 1);
    k_root_cells<<<1, 64, 0, X.st>>>(rb.cells, 1, 0, n, 1);
    rb.ents = root;
    group_batch<E>(X, rb, false);
    dfree(X, rb.cells);
    if (rb.ents != (void*)root) {
      root = (E*)rb.ents;
      n = rb.nent;
      own_root = true;
    }
    unit = rb.unit;
  }
  // greedy dive per sector: an achieved leaf key is a valid starting bound
  for (int s = 0; s < nsec; s++) {
    Batch b;
    b.level = 0;
    b.ncell = 1;
    b.nent = n;
    b.unit = unit;
    b.cells = dalloc<Cell>(X, 1);
    k_root_cells<<<1, 64, 0, X.st>>>(b.cells, 1, s, n, 1);
    b.ents = root;
    bool own = false;
    while (true) {
      Parent* pa = expand<FAM, E, M>(X, b, own, true);
      if (!pa) break;
      pa->pending = 1;
      if (!materialize<FAM, E, M>(X, pa, 0, pa->nkept, b)) break;
      own = true;
    }
  }
  // depth-first over batches; children of a batch in count order
  std::vector<Task> stack;
  bool root_owned_by_batch = false;
  {
    Task t{};
    t.chunk = false;
    Batch& r = t.b;
    r.level = 0;
    r.ncell = (uint32_t)nsec;
    r.nent = n * nsec;
    r.unit = unit;
    r.cells = dalloc<Cell>(X, nsec);
    k_root_cells<<<1, 64, 0, X.st>>>(r.cells, nsec, 0, n, 0);
    if (nsec == 1) {
      r.ents = root;
      root_owned_by_batch = own_root;
    } else {
      E* rep = dalloc<E>(X, n * nsec);
      k_replicate<E><<<gs_grid(X, n * nsec), 256, 0, X.st>>>(root, (int64_t)n, nsec, rep);
      r.ents = rep;
      root_owned_by_batch = true;
      if (own_root) dfree(X, root);
    }
    stack.push_back(t);
  }
  bool first = true;
  while (!stack.empty()) {
    Task t = stack.back();
    stack.pop_back();
    Batch b;
    bool own = true;
    if (t.chunk) {
      if (!materialize<FAM, E, M>(X, t.par, t.r0, t.r1, b)) continue;
    } else {
      b = t.b;
      own = first ? root_owned_by_batch : true;
    }
    first = false;
    Parent* pa = expand<FAM, E, M>(X, b, own, false);
    if (pa) push_children<FAM, E, M>(X, pa, stack);
  }
}

void check_bad(Run& X, int* dbad) {
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  if (bad & 1) {
    X.ctx->err = "non-finite observation or zero ray direction";
    throw DevErr{GV_EINVAL};
  }
  if (bad & 2) {
    X.ctx->err = "lattice too fine for 32-bit cells";
    throw DevErr{GV_ERANGE};
  }
}

template <int FAM>
void run_linear(Run& X, Cols cols, PathC& path, uint64_t& best) {
  using E = typename EntOf<FAM>::T;
  const int64_t n = X.n;
  E* root = dalloc<E>(X, n);
  unsigned* dmax = dalloc<unsigned>(X, 2);
  int* dbad = dalloc<int>(X, 1);
  HIPCHK(hipMemsetAsync(dmax, 0, 2 * sizeof(unsigned), X.st));
  HIPCHK(hipMemsetAsync(dbad, 0, sizeof(int), X.st));
  if (n > 0) k_root_lin<FAM><<<gs_grid(X, n), 256, 0, X.st>>>(X.dP, cols, n, root, dmax, dbad);
  check_bad(X, dbad);
  unsigned mx[2];
  HIPCHK(hipMemcpyAsync(mx, dmax, sizeof(mx), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  {
    // every intermediate of the integer test stays below 2^30
    const ProbC& P = X.S.P;
    double Hmax = 0, padmax = 0;
    for (int j = 0; j < X.S.d; j++) {
      Hmax = std::max(Hmax, (double)P.lev[0].H[j]);
      padmax = std::max(padmax, (double)P.lev[0].padu[j]);
    }
    const double np = (FAM == FAM_PLANE3D) ? 2.0 : 1.0;
    const double Fb = std::max((double)mx[1], Hmax + padmax + np * mx[0]);
    if (2.0 * Fb + 2.0 * np * mx[0] + 2.0 * Hmax + padmax >= 1073741824.0) {
      X.ctx->err = "lattice too fine for 32-bit cells";
      throw DevErr{GV_ERANGE};
    }
  }
  dfree(X, dmax);
  {
    // canonical surfaces a cell of level m can hold: slopes shrink by 2 per
    // split of their parameter axis, heights span the cell plus its pads
    const ProbC& P = X.S.P;
    X.lat_bound[0] = 1e300;
    for (int m = 1; m <= P.Lstar; m++) {
      double D = (FAM == FAM_RAY3D) ? 3.0 : 1.0;
      const int nq = (FAM == FAM_RAY3D) ? 2 : 1, np = (FAM == FAM_PLANE3D) ? 2 : 1;
      for (int qi = 0; qi < nq; qi++) {
        const int q = (FAM == FAM_LINE2D) ? 1 : 2;
        double ks = 0.0, kprod = 1.0;
        for (int pi = 0; pi < np; pi++) {
          const int pax = (FAM == FAM_PLANE3D) ? pi : 0;
          const double km = std::ceil((double)mx[0] / std::ldexp(1.0, std::min(m, P.L[pax]))) + 1.0;
          ks += km;
          kprod *= 2.0 * km + 1.0;
        }
        const double Hm = std::ldexp(1.0, -std::min(m, P.L[q])) * P.inv_sf[q];
        D *= (Hm + (double)P.lev[m - 1].padu[q] + 4.0 * ks + 2.0) * kprod;
      }
      X.lat_bound[m] = D;
    }
  }
  search<FAM, E, uint8_t>(X, root, n);
  dfree(X, root);
  HIPCHK(hipMemcpyAsync(&best, X.dbest, sizeof(best), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  (void)path;
  dfree(X, dbad);
}

void run_pose(Run& X, Cols cols, double epsk, bool want_filter, uint64_t& best) {
  const int64_t n = X.n;
  unsigned long long* dmx = dalloc<unsigned long long>(X, 8);
  int* dbad = dalloc<int>(X, 1);
  HIPCHK(hipMemsetAsync(dmx, 0, 8 * sizeof(unsigned long long), X.st));
  HIPCHK(hipMemsetAsync(dbad, 0, sizeof(int), X.st));
  if (n > 0) k_pose_bounds<<<gs_grid(X, n), 256, 0, X.st>>>(X.dP, cols, n, dmx, dbad);
  check_bad(X, dbad);
  unsigned long long mxb[8];
  HIPCHK(hipMemcpyAsync(mxb, dmx, sizeof(mxb), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  double mx[8];
  for (int k = 0; k < 8; k++) std::memcpy(&mx[k], &mxb[k], 8);
  pose_lattice(X.S, mx[0], mx[1], epsk);
  HIPCHK(hipMemcpyAsync(X.dP, &X.S.P, sizeof(ProbC), hipMemcpyHostToDevice, X.st));
  X.m64 = dalloc<double>(X, (uint64_t)n * 5);
  EntQ32* e32 = want_filter ? dalloc<EntQ32>(X, n) : nullptr;
  EntQ64* e64 = dalloc<EntQ64>(X, n);
  if (n > 0) k_root_pose<<<gs_grid(X, n), 256, 0, X.st>>>(X.dP, cols, n, X.m64, e32, e64, dmx);
  HIPCHK(hipMemcpyAsync(mxb, dmx, sizeof(mxb), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  for (int k = 0; k < 8; k++) std::memcpy(&mx[k], &mxb[k], 8);
  const bool filt = want_filter && pose_filter_exact(X.S, mx);
  X.S.filter = filt;
  if (filt) {
    dfree(X, e64);
    search<FAM_POSE4DOF, EntQ32, uint16_t>(X, e32, n);
    dfree(X, e32);
  } else {
    if (e32) dfree(X, e32);
    search<FAM_POSE4DOF, EntQ64, uint16_t>(X, e64, n);
    dfree(X, e64);
  }
  HIPCHK(hipMemcpyAsync(&best, X.dbest, sizeof(best), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipStreamSynchronize(X.st));
  dfree(X, dmx);
  dfree(X, dbad);
}

void decode_leaf(const ProbC& P, uint64_t idx, PathC& path, int32_t* coords) {
  path.sector = P.fam == GV_POSE4DOF ? (int32_t)(idx >> P.Bcell) : 0;
  int32_t cc[4] = {0, 0, 0, 0};
  for (int m = 0; m < P.Lstar; m++) {
    const LevelC& lv = P.lev[m];
    const uint32_t dg = (uint32_t)((idx >> lv.rem_next) & ((1ull << lv.abits) - 1ull));
    path.digit[m] = (uint8_t)dg;
    const uint32_t cb = lv.cbits[dg];
    for (int a = 0; a < 4; a++)
      if (lv.split[a]) cc[a] = 2 * cc[a] + (int32_t)((cb >> a) & 1u);
  }
  for (int a = 0; a < 4; a++) coords[a] = cc[a];
}

gv_status solve_impl(gv_ctx* ctx, const gv_problem* p, gv_result* r) {
  auto t0 = std::chrono::steady_clock::now();
  Run X;
  X.ctx = ctx;
  X.st = ctx->stream;
  X.n = p->n;
  X.group_mode = p->group;
  X.trace = std::getenv("GV_TRACE") != nullptr;
  if (const char* fc = std::getenv("GV_FIRST_CELLS")) X.first_cells = std::max<uint64_t>(1, std::strtoull(fc, nullptr, 10));
  std::string why;
  gv_status st = setup_axes(p, X.S, why);
  if (st != GV_OK) {
    ctx->err = why;
    return st;
  }
  const ProbC& P = X.S.P;
  std::vector<void*> owned;
  try {
    HIPCHK(hipSetDevice(ctx->device));
    // one chunk per level can be alive along the depth-first path
    X.budget_entries = std::max<uint64_t>(1ull << 22, ctx->budget / (uint64_t)(P.Lstar + 2) / 64);
    X.dP = dalloc<ProbC>(X, 1);
    X.dbest = dalloc<unsigned long long>(X, 1);
    X.drecheck = dalloc<unsigned long long>(X, 1);
    X.dtot = dalloc<uint64_t>(X, 2);
    X.dummy = dalloc<uint32_t>(X, 64);
    X.dreads = dalloc<unsigned long long>(X, 1);
    HIPCHK(hipMemsetAsync(X.dreads, 0, 8, X.st));
    HIPCHK(hipMemsetAsync(X.dbest, 0, 8, X.st));
    HIPCHK(hipMemsetAsync(X.drecheck, 0, 8, X.st));
    HIPCHK(hipMemcpyAsync(X.dP, &P, sizeof(ProbC), hipMemcpyHostToDevice, X.st));
    const int ncol = p->family == GV_RAY3D ? 6 : (p->family == GV_POSE4DOF ? 5 : X.S.d);
    Cols cols{};
    for (int k = 0; k < ncol; k++) {
      if (!p->col[k] && p->n > 0) {
        ctx->err = "missing column";
        return GV_EINVAL;
      }
      if (p->cols_on_device || p->n == 0) {
        cols.c[k] = p->col[k];
      } else {
        double* d = dalloc<double>(X, p->n);
        HIPCHK(hipMemcpyAsync(d, p->col[k], p->n * sizeof(double), hipMemcpyHostToDevice, X.st));
        owned.push_back(d);
        cols.c[k] = d;
      }
    }
    uint64_t best = 0;
    PathC path{};
    switch (p->family) {
      case GV_LINE2D: run_linear<FAM_LINE2D>(X, cols, path, best); break;
      case GV_PLANE3D: run_linear<FAM_PLANE3D>(X, cols, path, best); break;
      case GV_RAY3D: run_linear<FAM_RAY3D>(X, cols, path, best); break;
      default: run_pose(X, cols, p->eps[3], p->precision == GV_FP32_FILTER, best); break;
    }
    const uint64_t count = best >> P.B;
    const uint64_t leaf = P.idxmask - (best & P.idxmask);
    int32_t coords[4];
    decode_leaf(X.S.P, leaf, path, coords);
    // inliers by replay
    uint32_t* flag = dalloc<uint32_t>(X, X.n);
    uint32_t* pos = dalloc<uint32_t>(X, X.n);
    int* dbad = dalloc<int>(X, 1);
    HIPCHK(hipMemsetAsync(dbad, 0, sizeof(int), X.st));
    if (X.n > 0) {
      switch (p->family) {
        case GV_LINE2D: k_replay_lin<FAM_LINE2D><<<gs_grid(X, X.n), 256, 0, X.st>>>(X.dP, cols, X.n, path, flag, dbad); break;
        case GV_PLANE3D: k_replay_lin<FAM_PLANE3D><<<gs_grid(X, X.n), 256, 0, X.st>>>(X.dP, cols, X.n, path, flag, dbad); break;
        case GV_RAY3D: k_replay_lin<FAM_RAY3D><<<gs_grid(X, X.n), 256, 0, X.st>>>(X.dP, cols, X.n, path, flag, dbad); break;
        default: k_replay_pose<<<gs_grid(X, X.n), 256, 0, X.st>>>(X.dP, X.m64, X.n, path, flag); break;
      }
      HIPCHK(hipGetLastError());
      excl_scan(X, flag, pos, (uint64_t)X.n);
    }
    uint32_t last[2] = {0, 0};
    if (X.n > 0) {
      HIPCHK(hipMemcpyAsync(&last[0], pos + X.n - 1, 4, hipMemcpyDeviceToHost, X.st));
      HIPCHK(hipMemcpyAsync(&last[1], flag + X.n - 1, 4, hipMemcpyDeviceToHost, X.st));
    }
    unsigned long long rech = 0;
    HIPCHK(hipMemcpyAsync(&rech, X.drecheck, 8, hipMemcpyDeviceToHost, X.st));
    HIPCHK(hipStreamSynchronize(X.st));
    const uint64_t ninl = (uint64_t)last[0] + last[1];
    r->count = count;
    r->leaf_index = leaf;
    r->sector = path.sector;
    for (int a = 0; a < 4; a++) r->leaf_coords[a] = a < X.S.d ? coords[a] : 0;
    for (int j = 0; j < 4; j++) r->point[j] = 0.0;
    for (int j = 0; j < X.S.d; j++) {
      double u = (double)(2 * coords[j] + 1) * std::ldexp(1.0, -(P.L[j] + 1));
      r->point[j] = P.lo[j] + P.E[j] * u;
    }
    if (p->family == GV_POSE4DOF) {
      double yaw = (double)path.sector * (M_PI / 2.0) + std::atan(r->point[3]);
      if (yaw < 0.0) yaw += 2.0 * M_PI;
      if (yaw >= 2.0 * M_PI) yaw -= 2.0 * M_PI;
      r->point[3] = yaw;
    }
    for (int j = 0; j < 4; j++) r->bound[j] = 0.0;
    for (int j = 0; j < X.S.d; j++) {
      if (p->family == GV_POSE4DOF) {
        r->bound[j] = j == 2 ? (P.padz + X.S.ez * 0.5) * P.E[2] : (j == 3 ? P.padk + X.S.ek * 0.5 : 0.5 * std::ldexp(P.E[j], -P.L[j]));
      } else {
        const double Em = (double)(P.Lstar * (X.S.ell + 1)) * P.sf[j] * 0.5;
        r->bound[j] = (X.S.epsn[j] + 2.0 * Em + P.sf[j]) * P.E[j];
      }
    }
    r->n_inliers = ninl;
    gv_status out = GV_OK;
    if (ninl != count) {
      ctx->err = "internal: replayed inlier count differs from the leaf count";
      out = GV_EDEVICE;
    } else if (ninl > r->inliers_cap || (!r->inliers && ninl > 0)) {
      out = GV_EBUFSZ;
    } else if (ninl > 0) {
      int64_t* dout = dalloc<int64_t>(X, ninl);
      k_write_inliers<<<gs_grid(X, X.n), 256, 0, X.st>>>(flag, pos, X.n, dout);
      HIPCHK(hipMemcpyAsync(r->inliers, dout, ninl * sizeof(int64_t), hipMemcpyDeviceToHost, X.st));
      HIPCHK(hipStreamSynchronize(X.st));
      dfree(X, dout);
    }
    dfree(X, flag);
    dfree(X, pos);
    dfree(X, dbad);
    if (X.m64) dfree(X, X.m64);
    for (void* q : owned) dfree(X, q);
    dfree(X, X.dP);
    dfree(X, X.dbest);
    dfree(X, X.drecheck);
    dfree(X, X.dtot);
    if (X.ctx->kernel_timing) {
      unsigned long long rd = 0;
      HIPCHK(hipMemcpyAsync(&rd, X.dreads, 8, hipMemcpyDeviceToHost, X.st));
      HIPCHK(hipStreamSynchronize(X.st));
      X.stats.compact_bytes += rd * X.ent_bytes;
    }
    dfree(X, X.dummy);
    dfree(X, X.dreads);
    HIPCHK(hipStreamSynchronize(X.st));
    X.stats.fp64_rechecks = rech;
    X.stats.levels = (uint32_t)P.Lstar;
    for (auto& e : X.ev) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e.first.first, e.first.second));
      (e.second == 0 ? X.stats.test_ms : X.stats.compact_ms) += (double)ms;
    }
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    X.stats.ms_total = ms;
    X.stats.ms_kernels = ms;
    r->stats = X.stats;
    return out;
  } catch (DevErr& e) {
    for (void* q : owned) dfree(X, q);
    (void)hipStreamSynchronize(X.st);
    return e.st;
  }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* gv_status_str(gv_status s) {
  switch (s) {
    case GV_OK: return "ok";
    case GV_EINVAL: return "invalid argument";
    case GV_ENOMEM: return "out of memory";
    case GV_ETOOBIG: return "problem exceeds the memory budget";
    case GV_EBUFSZ: return "inlier buffer too small";
    case GV_EAGAIN: return "not finished";
    case GV_ETIMEDOUT: return "timed out";
    case GV_ECANCELED: return "cancelled";
    case GV_EDEVICE: return "device error";
    case GV_ERANGE: return "lattice too fine for the device arithmetic";
  }
  return "unknown status";
}

const char* gv_last_error(gv_ctx* ctx) {
  if (!ctx) return "";
  std::lock_guard<std::mutex> g(ctx->mu);
  tl_err = ctx->err;
  return tl_err.c_str();
}

gv_status gv_create(gv_ctx** out, const gv_ctx_config* cfg) {
  if (!out) return GV_EINVAL;
  *out = nullptr;
  gv_ctx* c = new (std::nothrow) gv_ctx();
  if (!c) return GV_ENOMEM;
  c->device = cfg ? cfg->device : 0;
  c->kernel_timing = cfg && cfg->kernel_timing;
  if (hipSetDevice(c->device) != hipSuccess) {
    delete c;
    return GV_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  if (cfg && cfg->hip_stream) {
    c->stream = (hipStream_t)cfg->hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return GV_EDEVICE;
    }
    c->own_stream = true;
  }
  size_t fr = 0, tot = 0;
  (void)hipMemGetInfo(&fr, &tot);
  c->budget = (cfg && cfg->mem_budget_bytes) ? cfg->mem_budget_bytes : (uint64_t)(0.6 * (double)fr);
  *out = c;
  return GV_OK;
}

gv_status gv_destroy(gv_ctx* ctx) {
  if (!ctx) return GV_EINVAL;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->cache.trim(ctx->stream);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto& kv : ctx->cache.live) (void)hipFree(kv.first);
  ctx->cache.live.clear();
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return GV_OK;
}

gv_status gv_solve(gv_ctx* ctx, const gv_problem* p, gv_result* r) {
  if (!ctx || !p || !r) return GV_EINVAL;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->err.clear();
  std::memset(&r->stats, 0, sizeof(r->stats));
  return solve_impl(ctx, p, r);
}

gv_status gv_parametrize(gv_ctx* ctx, const gv_problem* p, double* t_out, double* f_out, int32_t* tag_out) {
  if (!ctx || !p || (!t_out && p->n > 0) || (!f_out && p->n > 0)) return GV_EINVAL;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->err.clear();
  Run X;
  X.ctx = ctx;
  X.st = ctx->stream;
  X.n = p->n;
  std::string why;
  gv_status st = setup_axes(p, X.S, why);
  if (st != GV_OK && st != GV_ERANGE) {
    ctx->err = why;
    return st;
  }
  std::vector<void*> owned;
  try {
    HIPCHK(hipSetDevice(ctx->device));
    X.dP = dalloc<ProbC>(X, 1);
    HIPCHK(hipMemcpyAsync(X.dP, &X.S.P, sizeof(ProbC), hipMemcpyHostToDevice, X.st));
    const int ncol = p->family == GV_RAY3D ? 6 : (p->family == GV_POSE4DOF ? 5 : X.S.d);
    Cols cols{};
    for (int k = 0; k < ncol; k++) {
      if (p->cols_on_device || p->n == 0) {
        cols.c[k] = p->col[k];
      } else {
        double* d = dalloc<double>(X, p->n);
        HIPCHK(hipMemcpyAsync(d, p->col[k], p->n * sizeof(double), hipMemcpyHostToDevice, X.st));
        owned.push_back(d);
        cols.c[k] = d;
      }
    }
    if (p->n > 0) {
      double* t = dalloc<double>(X, (uint64_t)p->n * 4);
      double* f = dalloc<double>(X, (uint64_t)p->n * 2);
      int32_t* tg = dalloc<int32_t>(X, p->n);
      int* bad = dalloc<int>(X, 1);
      HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), X.st));
      k_front<<<gs_grid(X, p->n), 256, 0, X.st>>>((int)p->family, X.dP, cols, p->n, t, f, tg, bad);
      HIPCHK(hipMemcpyAsync(t_out, t, p->n * 4 * sizeof(double), hipMemcpyDeviceToHost, X.st));
      HIPCHK(hipMemcpyAsync(f_out, f, p->n * 2 * sizeof(double), hipMemcpyDeviceToHost, X.st));
      if (tag_out) HIPCHK(hipMemcpyAsync(tag_out, tg, p->n * sizeof(int32_t), hipMemcpyDeviceToHost, X.st));
      int hb = 0;
      HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, X.st));
      HIPCHK(hipStreamSynchronize(X.st));
      dfree(X, t);
      dfree(X, f);
      dfree(X, tg);
      dfree(X, bad);
      if (hb) {
        ctx->err = "non-finite observation or zero ray direction";
        st = GV_EINVAL;
      }
    }
    for (void* q : owned) dfree(X, q);
    dfree(X, X.dP);
    HIPCHK(hipStreamSynchronize(X.st));
    return st == GV_ERANGE ? GV_OK : st;
  } catch (DevErr& e) {
    (void)hipStreamSynchronize(X.st);
    return e.st;
  }
}

gv_status gv_submit(gv_ctx* ctx, const gv_problem* p, uint64_t* ticket) {
  (void)p;
  (void)ticket;
  if (ctx) ctx->err = "continuous batching is not built yet";
  return GV_EINVAL;
}
gv_status gv_poll(gv_ctx* ctx, uint64_t ticket, gv_result* r, int timeout_ms) {
  (void)ticket;
  (void)r;
  (void)timeout_ms;
  if (ctx) ctx->err = "continuous batching is not built yet";
  return GV_EINVAL;
}
gv_status gv_cancel(gv_ctx* ctx, uint64_t ticket) {
  (void)ticket;
  if (ctx) ctx->err = "continuous batching is not built yet";
  return GV_EINVAL;
}

}  // extern "C"
