// gv_exact.h -- exact mode of the linear families, and the incidence-only
// kernels behind gv_incidence.
//
// Exact mode (canon_c = +inf) is the plain definition of the problem (Sec.
// 3.1, Alg. 1 with the eps neighbourhood on the leaf grid): every surface is
// quantized once at the root to the fixed 2^-36 lattice and never
// re-canonized, a surface counts at a leaf when on every level of its path it
// passes within eps (rounded up to that lattice) of the child, and the test
// runs in binary64 in the order of the definition.  The surfaces do not
// change below the root, so the count pass stores a pass mask per entry and
// compaction copies entries unchanged (as for the 4-DoF pose family).
#pragma once
#include "gv_kernels.h"
#include "gv_root.h"

// root quantization of one observation: the four canonization steps at the
// root cell (whose minimum corner is the origin) with every step 2^-36
template <int BF>
__device__ inline bool root_x(const ProbC& P, const double* const* col, int64_t i, EntX& e, int* bad) {
  double t[4], f[2];
  int32_t tag;
  e = EntX{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1u, 0};
  if (!front_eval(BF, col, i, P, t, f, &tag)) {
    atomicOr(bad, 1);
    return false;
  }
  const double s = 0x1p-36, inv = 0x1p36, u = 0.0;
  // parameters per dependent axis: (slopes, offset)
  const int nq = BF == FAM_RAY3D || BF == FAM_SIM2D ? 2 : 1, np = BF == FAM_PLANE3D || BF == FAM_SIM2D ? 2 : 1;
  double out_t[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, out_f[2] = {0.0, 0.0};
  double M = 0.0;
  for (int qi = 0; qi < nq; qi++) {
    double floc = f[qi];
    for (int k = 0; k < np; k++) floc = floc + t[2 * qi + k] * u;
    floc = floc - u;
    double tn[2] = {0.0, 0.0};
    for (int k = 0; k < np; k++) tn[k] = rint(t[2 * qi + k] * inv) * s;
    const double fl = rint(floc * inv) * s;
    double fn = fl;
    for (int k = 0; k < np; k++) fn = fn - tn[k] * u;
    fn = fn + u;
    out_f[qi] = fn;
    double mq = fabs(fn) + 4.0;
    for (int k = 0; k < np; k++) {
      out_t[qi][k] = tn[k];
      mq += fabs(tn[k]);
    }
    M = mq > M ? mq : M;
  }
  if (!(M < 0x1p12)) atomicOr(bad, 2);  // beyond the range the definition evaluates exactly
  e = EntX{out_t[0][0], out_t[0][1], out_t[1][0], out_t[1][1], out_f[0], out_f[1], 1u, tag};
  return true;
}

// grouping of exact-mode lists: equal parameter tuples (bit patterns)
template <> struct Tuple<EntX> {
  __device__ static uint64_t hash(const EntX& e) {
    uint64_t h = hcomb(8, (uint32_t)e.tag);
    h = hcomb(h, (uint64_t)__double_as_longlong(e.t00));
    h = hcomb(h, (uint64_t)__double_as_longlong(e.t01));
    h = hcomb(h, (uint64_t)__double_as_longlong(e.t10));
    h = hcomb(h, (uint64_t)__double_as_longlong(e.t11));
    h = hcomb(h, (uint64_t)__double_as_longlong(e.f0));
    return hcomb(h, (uint64_t)__double_as_longlong(e.f1));
  }
  __device__ static bool same(const EntX& x, const EntX& y) {
    return x.tag == y.tag && __double_as_longlong(x.t00) == __double_as_longlong(y.t00) &&
           __double_as_longlong(x.t01) == __double_as_longlong(y.t01) &&
           __double_as_longlong(x.t10) == __double_as_longlong(y.t10) &&
           __double_as_longlong(x.t11) == __double_as_longlong(y.t11) &&
           __double_as_longlong(x.f0) == __double_as_longlong(y.f0) &&
           __double_as_longlong(x.f1) == __double_as_longlong(y.f1);
  }
  __device__ static void setw(EntX& e, uint32_t w) { e.w = w; }
  __device__ static uint32_t w(const EntX& e) { return e.w; }
};

template <int BF>
__global__ void k_root_x(const ProbC* __restrict__ Pp, Cols cols, int64_t n, EntX* __restrict__ out,
                         int* __restrict__ bad) {
  const ProbC& P = *Pp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    EntX e;
    root_x<BF>(P, cols.c, i, e, bad);
    out[i] = e;
  }
}

// Count pass: one wave per item; per entry the pass mask over the cell's
// children (stored for the compaction), per child the summed multiplicities
// (one atomic per item and child) and the item's survivors (for the
// compaction's write offsets).
template <int BF, bool UNIT, typename M>
__global__ void __launch_bounds__(256) k_count_x(const ProbC* __restrict__ Ptab, int m, LevelC lv,
                                                 const Cell* __restrict__ cells, const Item* __restrict__ items,
                                                 const uint32_t* __restrict__ nitems_p, const EntX* __restrict__ ents,
                                                 M* __restrict__ masks, uint32_t* __restrict__ ccnt,
                                                 uint32_t* __restrict__ cnent, uint32_t* __restrict__ itemcnt,
                                                 uint32_t istride) {
  constexpr int NC = 8 * (int)sizeof(M);  // children a mask holds (8, or 16 for four split axes)
  const uint32_t nch = 1u << lv.abits;
  const uint32_t lane = lane_id();
  const uint32_t wave = uniform_u32((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  const uint32_t nitems = *nitems_p;
  for (uint32_t it = wave; it < nitems; it += nwaves) {
    const Item I = items[it];
    const Cell C = cells[I.cell];
    const ProbC& P = Ptab[C.prob];
    uint32_t aw[NC], an[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ch++) { aw[ch] = 0; an[ch] = 0; }
    for (uint32_t k0 = 0; k0 < I.cnt; k0 += 64) {
      const uint32_t k = k0 + lane;
      uint32_t mask = 0, w = 0;
      if (k < I.cnt) {
        const EntX e = ents[I.off + k];
        w = e.w;
        for (uint32_t ch = 0; ch < nch; ch++) {
          double lo[4], hi[4];
          x_child_box(P, lv, C.c, m, lv.cbits[ch], lo, hi);
          if (x_meets<BF>(e, lo, hi, P.xpad)) mask |= 1u << ch;
        }
        masks[I.off + k] = (M)mask;
      }
#pragma unroll
      for (int ch = 0; ch < NC; ch++) {
        const bool p = (mask >> ch) & 1u;
        if constexpr (UNIT) {
          an[ch] += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(p));
        } else {
          aw[ch] += p ? w : 0u;
          an[ch] += p ? 1u : 0u;
        }
      }
    }
#pragma unroll
    for (int ch = 0; ch < NC; ch++) {
      if ((uint32_t)ch < nch) {
        const uint32_t n = UNIT ? an[ch] : wave_sum_u32(an[ch]);
        const uint32_t w = UNIT ? n : wave_sum_u32(aw[ch]);
        if (lane == 0 && n) {
          atomicAdd(&ccnt[I.cell * nch + ch], w);
          atomicAdd(&cnent[I.cell * nch + ch], n);
          if (istride) itemcnt[(uint64_t)ch * istride + it] = n;
        }
      }
    }
  }
}

// Replay along each problem's chosen path (member tracking): an original is
// an inlier iff its quantized surface passes every level's test.
template <int BF>
__global__ void k_replay_x(const ProbC* __restrict__ Ptab, const Cols* __restrict__ ctab,
                           const uint64_t* __restrict__ ooff, uint32_t nprob, uint64_t Ntot,
                           const PathC* __restrict__ paths, uint32_t* __restrict__ flag, int* __restrict__ bad) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Ntot; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t p = prob_of(ooff, nprob, i);
    const ProbC& P = Ptab[p];
    const PathC& path = paths[p];
    EntX e;
    uint32_t ok = 0;
    if (root_x<BF>(P, ctab[p].c, (int64_t)(i - ooff[p]), e, bad)) {
      ok = 1;
      int32_t cc[4] = {0, 0, 0, 0};
      for (int m = 0; m < P.Lstar && ok; m++) {
        const LevelC& lv = P.lev[m];
        const uint32_t cb = lv.cbits[path.digit[m]];
        double lo[4], hi[4];
        x_child_box(P, lv, cc, m, cb, lo, hi);
        ok = x_meets<BF>(e, lo, hi, P.xpad) ? 1u : 0u;
        for (int a = 0; a < 4; a++) cc[a] = lv.split[a] ? 2 * cc[a] + (int32_t)((cb >> a) & 1u) : cc[a];
      }
    }
    flag[i] = ok;
  }
}

// ---------------------------------------------------------------------------
// Incidence only (gv_incidence): every surface of one problem, in its
// canonical form at a given cell (the root canonization, then the child
// canonization of every level on the path to the cell), tested against each
// child of that cell; one pass mask per surface (bit = child digit).
// ---------------------------------------------------------------------------
template <int FAM, typename E, int NCH>
__global__ void k_incidence_lin(const ProbC* __restrict__ Pp, const E* __restrict__ root, int64_t n, PathC path,
                                int m, uint32_t* __restrict__ masks) {
  const ProbC& P = *Pp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    LinS s = load_ent<FAM>(root[i]);
    for (int k = 0; k < m; k++) s = lin_canon_child<FAM>(s, P.lev[k], P.lev[k].cbits[path.digit[k]]);
    bool p[NCH];
    lin_pass<FAM, NCH>(s, P.lev[m], p);
    uint32_t mask = 0;
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) mask |= p[ch] ? 1u << ch : 0u;
    masks[i] = mask;
  }
}

template <int BF>
__global__ void k_incidence_x(const ProbC* __restrict__ Pp, const EntX* __restrict__ root, int64_t n, Cell C, int m,
                              uint32_t* __restrict__ masks) {
  const ProbC& P = *Pp;
  const LevelC& lv = P.lev[m];
  const uint32_t nch = 1u << lv.abits;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const EntX e = root[i];
    uint32_t mask = 0;
    for (uint32_t ch = 0; ch < nch; ch++) {
      double lo[4], hi[4];
      x_child_box(P, lv, C.c, m, lv.cbits[ch], lo, hi);
      if (x_meets<BF>(e, lo, hi, P.xpad)) mask |= 1u << ch;
    }
    masks[i] = mask;
  }
}

// POSE4DOF: binary64 (EntQ64) or the binary32 filter with binary64 recheck
// of undecided halves (EntQ32), exactly as in the count pass
template <typename E>
__global__ void k_incidence_pose(const ProbC* __restrict__ Pp, const E* __restrict__ root, int64_t n,
                                 const double* __restrict__ m64, uint64_t n_root, Cell C, int m,
                                 uint32_t* __restrict__ masks, unsigned long long* __restrict__ rechecks) {
  const ProbC& P = *Pp;
  const LevelC& lv = P.lev[m];
  PoseLevel B;
  pose_level_boxes(P, lv, C, m, B);
  float Bf[16];
  for (int b = 0; b < 2; b++) {
    Bf[0 + b] = (float)B.Xlo[b]; Bf[2 + b] = (float)B.Xhi[b];
    Bf[4 + b] = (float)B.Ylo[b]; Bf[6 + b] = (float)B.Yhi[b];
    Bf[8 + b] = (float)B.ZH[b];  Bf[10 + b] = (float)B.ZL[b];
    Bf[12 + b] = (float)B.Llo[b]; Bf[14 + b] = (float)B.Lhi[b];
  }
  uint32_t nre = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const E e = root[i];
    uint32_t mask;
    if constexpr (sizeof(E) == sizeof(EntQ64)) {
      mask = pose_mask64<false>(P, lv, B, (int)C.sector, e.W1, e.W2, e.W3, e.xi, e.eta);
    } else {
      mask = pose_mask32<false>(P, lv, C, m, Bf, (int)C.sector, e, m64, n_root, nre);
    }
    masks[i] = mask;
  }
  if (nre) atomicAdd(rechecks, (unsigned long long)nre);
}
