// gv_kernels.h -- HIP kernels of the general-voting library (gfx950, wave64).
//
// Work decomposition: a batch holds cells of one level, each with a
// contiguous list of canonical surfaces.  Lists are cut into items of at most
// 2^ilog <= GV_ITEM entries (the batch's item size) that belong to a single
// cell; one wavefront processes one item, so the cell's child boxes are wave-uniform (scalar registers) and the
// per-child counts reduce across the wave before a single atomic per child.
#pragma once
#include "gv_device.h"

#include <type_traits>

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline uint32_t lane_id() { return threadIdx.x & 63u; }
__device__ inline uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint64_t uniform_u64(uint64_t v) {
  return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
         (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}
__device__ inline uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ---------------------------------------------------------------------------
// Items: per cell ceil(len / 2^ilog) work items of 2^ilog entries (the last
// one ragged).
// ---------------------------------------------------------------------------
__device__ inline uint32_t items_of(uint32_t len, uint32_t ilog) { return (len + (1u << ilog) - 1u) >> ilog; }
__global__ void k_item_counts(const Cell* __restrict__ cells, uint32_t ncell, uint32_t ilog,
                              uint32_t* __restrict__ nitem) {
  uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncell) nitem[c] = items_of(cells[c].len, ilog);
}
__global__ void k_item_fill(const Cell* __restrict__ cells, uint32_t ncell, uint32_t ilog,
                            const uint32_t* __restrict__ nitem, const uint32_t* __restrict__ ioff,
                            Item* __restrict__ items, uint32_t* __restrict__ total) {
  uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  uint32_t o = ioff[c], k = nitem[c];
  const uint64_t off = cells[c].off;
  const uint32_t len = cells[c].len, isz = 1u << ilog;
  for (uint32_t j = 0; j < k; j++) items[o + j] = Item{off + (uint64_t)j * isz, c, min(isz, len - j * isz)};
  if (c == ncell - 1) *total = o + k;
}

// ---------------------------------------------------------------------------
// Single-workgroup forms of the frontier bookkeeping for small batches: one
// launch where the general form takes a device-wide scan (two launches) and
// the small kernels around it.  1024 threads; thread t owns the contiguous
// run [t * GV_SMALL_PER, (t + 1) * GV_SMALL_PER) of the array.  Totals that
// the host reads go to host-coherent memory, fenced at system scope.
// ---------------------------------------------------------------------------
#define GV_SMALL_PER 4
#define GV_SMALL_N (1024u * GV_SMALL_PER)

// Exclusive prefix of the per-thread values s over the workgroup (wsum: 16
// slots of LDS); every thread also gets the total.
template <typename T>
__device__ inline T block_excl(T s, T* wsum, T& tot) {
  const uint32_t t = threadIdx.x, l = t & 63u, w = t >> 6;
  T x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (l >= (uint32_t)o) x += y;
  }
  if (l == 63u) wsum[w] = x;
  __syncthreads();
  T pre = 0, all = 0;
  for (uint32_t k = 0; k < (blockDim.x >> 6); k++) {
    const T v = wsum[k];
    if (k < w) pre += v;
    all += v;
  }
  __syncthreads();
  tot = all;
  return pre + x - s;
}

// out = exclusive prefix sums of in[0, n), n <= GV_SMALL_N; *total = the sum
// (when given)
template <typename In, typename Out>
__global__ void __launch_bounds__(1024) k_scan_small(const In* __restrict__ in, Out* __restrict__ out, uint32_t n,
                                                     Out* __restrict__ total) {
  __shared__ Out wsum[16];
  const uint32_t b = threadIdx.x * GV_SMALL_PER;
  Out v[GV_SMALL_PER];
  Out s = 0;
#pragma unroll
  for (int j = 0; j < GV_SMALL_PER; j++) {
    v[j] = b + j < n ? (Out)in[b + j] : (Out)0;
    s += v[j];
  }
  Out tot;
  Out run = block_excl<Out>(s, wsum, tot);
#pragma unroll
  for (int j = 0; j < GV_SMALL_PER; j++) {
    if (b + j < n) out[b + j] = run;
    run += v[j];
  }
  if (total && threadIdx.x == 0) *total = tot;
}

// Work items of a batch of at most GV_SMALL_N cells: per-cell item counts,
// their offsets and the items themselves, in one launch.
__global__ void __launch_bounds__(1024) k_items_small(const Cell* __restrict__ cells, uint32_t ncell,
                                                      uint32_t ilog, uint32_t* __restrict__ ioff,
                                                      Item* __restrict__ items, uint32_t* __restrict__ total) {
  __shared__ uint32_t wsum[16];
  const uint32_t b = threadIdx.x * GV_SMALL_PER;
  uint64_t off[GV_SMALL_PER];
  uint32_t len[GV_SMALL_PER];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < GV_SMALL_PER; j++) {  // every load issued before any is used
    const bool in = b + j < ncell;
    off[j] = in ? cells[b + j].off : 0ull;
    len[j] = in ? cells[b + j].len : 0u;
  }
#pragma unroll
  for (int j = 0; j < GV_SMALL_PER; j++) s += items_of(len[j], ilog);
  uint32_t tot;
  uint32_t o = block_excl<uint32_t>(s, wsum, tot);
#pragma unroll
  for (int j = 0; j < GV_SMALL_PER; j++) {
    if (b + j >= ncell) break;
    const uint32_t k = items_of(len[j], ilog), isz = 1u << ilog;
    ioff[b + j] = o;
    for (uint32_t i = 0; i < k; i++) items[o + i] = Item{off[j] + (uint64_t)i * isz, b + j, min(isz, len[j] - i * isz)};
    o += k;
  }
  if (threadIdx.x == 0) *total = tot;
}

// Prune tail of a small expansion: keepscan = exclusive prefix of keepf,
// tot[0] = kept children, tot[1] = their entries (host-coherent memory).
__global__ void __launch_bounds__(1024) k_keep_small(const uint32_t* __restrict__ keepf,
                                                     const uint64_t* __restrict__ keptn, uint32_t nk,
                                                     uint32_t* __restrict__ keepscan, uint64_t* tot) {
  __shared__ uint32_t wsum[16];
  __shared__ uint64_t wsum64[16];
  const uint32_t b = threadIdx.x * GV_SMALL_PER;
  uint32_t v[GV_SMALL_PER];
  uint32_t s = 0;
  uint64_t e = 0;
#pragma unroll
  for (int j = 0; j < GV_SMALL_PER; j++) {
    v[j] = b + j < nk ? keepf[b + j] : 0u;
    e += b + j < nk ? keptn[b + j] : 0ull;
    s += v[j];
  }
  uint32_t kt;
  uint64_t et;
  uint32_t run = block_excl<uint32_t>(s, wsum, kt);
  (void)block_excl<uint64_t>(e, wsum64, et);
#pragma unroll
  for (int j = 0; j < GV_SMALL_PER; j++) {
    if (b + j < nk) keepscan[b + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) {
    tot[0] = kt;
    tot[1] = et;
    __threadfence_system();
  }
}

// Chunk totals of a small chunk: cidx / coff = exclusive prefixes of keepc /
// csize, tot[0] = kept cells, tot[1] = their entries (host-coherent memory).
__global__ void __launch_bounds__(1024) k_chunk_small(const uint32_t* __restrict__ keepc,
                                                      const uint64_t* __restrict__ csize, uint32_t nr,
                                                      uint32_t* __restrict__ cidx, uint64_t* __restrict__ coff,
                                                      uint64_t* tot) {
  __shared__ uint32_t wsum[16];
  __shared__ uint64_t wsum64[16];
  const uint32_t b = threadIdx.x * GV_SMALL_PER;
  uint32_t v[GV_SMALL_PER];
  uint64_t z[GV_SMALL_PER];
  uint32_t s = 0;
  uint64_t e = 0;
#pragma unroll
  for (int j = 0; j < GV_SMALL_PER; j++) {
    v[j] = b + j < nr ? keepc[b + j] : 0u;
    z[j] = b + j < nr ? csize[b + j] : 0ull;
    s += v[j];
    e += z[j];
  }
  uint32_t kt;
  uint64_t et;
  uint32_t run = block_excl<uint32_t>(s, wsum, kt);
  uint64_t run64 = block_excl<uint64_t>(e, wsum64, et);
#pragma unroll
  for (int j = 0; j < GV_SMALL_PER; j++) {
    if (b + j < nr) {
      cidx[b + j] = run;
      coff[b + j] = run64;
    }
    run += v[j];
    run64 += z[j];
  }
  if (threadIdx.x == 0) {
    tot[0] = kt;
    tot[1] = et;
    __threadfence_system();
  }
}

// one-word unit-weight PLANE3D entries -> 8-byte entries (before grouping)
__global__ void k_unit_to_p3(const EntP3u* __restrict__ in, uint64_t n, EntP3p* __restrict__ out) {
  const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += st) {
    const LinS s = load_ent<FAM_PLANE3D>(in[i]);
    out[i] = pack_p3(s.K[0][0], s.K[0][1], s.F[0], 1u);
  }
}

// zero up to three u32 arrays in one launch
__global__ void k_zero3(uint32_t* __restrict__ a, uint64_t na, uint32_t* __restrict__ b, uint64_t nb,
                        uint32_t* __restrict__ c, uint64_t nc) {
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = i0; i < na; i += st) a[i] = 0;
  for (uint64_t i = i0; i < nb; i += st) b[i] = 0;
  for (uint64_t i = i0; i < nc; i += st) c[i] = 0;
}

// ---------------------------------------------------------------------------
// Linear families: incidence test of every (canonical surface, child) pair
// and per-child counts.  No pass masks are stored: the compaction pass reads
// every entry anyway and repeats the (cheap, integer) test.
// ---------------------------------------------------------------------------
// Pass predicates of one surface for the NCH children of its cell.
// PLANE3D with all three axes splitting (digit = b_a1 b_a2 b_a0): with
// c = max(K, 0), child (b1, b2, b0) is met iff
//   0 <= u - b0 H <= H + 2 pad + |K1| + |K2|,  u = 2F + pad + c1 + c2 + b1 K1 + b2 K2,
// which is the general test (the surface's range over the child reaches the
// child's widened interval) with both bounds in one unsigned comparison.
template <int FAM, int NCH>
__device__ inline void lin_pass(const LinS& s, const LevelC& lv, bool (&p)[NCH]) {
  if constexpr (FAM == FAM_PLANE3D && NCH == 8) {
    const int32_t K1 = s.K[0][0], K2 = s.K[0][1], K12 = K1 + K2;
    const int32_t H = lv.H[2], pad = lv.padu[2];
    const int32_t S = imax32(K1, 0) + imax32(K2, 0);  // |K1| + |K2| = 2 S - K12
    const int32_t u = 2 * s.F[0] + pad + S;
    const uint32_t R = (uint32_t)(2 * S + (H + 2 * pad) - K12);
    const int32_t uu[4] = {u, u + K2, u + K1, u + K12};  // (b1, b2) = 00, 01, 10, 11
#pragma unroll
    for (int q = 0; q < 4; q++) {
      p[2 * q] = (uint32_t)uu[q] <= R;
      p[2 * q + 1] = (uint32_t)(uu[q] - H) <= R;
    }
  } else {
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) p[ch] = lin_meets<FAM>(s, lv, lv.cbits[ch]);
  }
}

// UNIT: every multiplicity is 1 (no merged surfaces), so a child's count is
// the popcount of its ballot, accumulated in scalar registers.  Each item
// writes its per-child entry counts (and, unless UNIT, weights) as one row
// icnt[it * NCH + ch]; k_cell_scan turns the rows into per-cell counts and
// per-item list offsets, so no atomics are needed.
template <int FAM, bool UNIT, typename E, int NCH>
__global__ void __launch_bounds__(256) k_count_lin(LevelC lv, const Item* __restrict__ items,
                                                   const uint32_t* __restrict__ nitems_p, const E* __restrict__ ents,
                                                   uint32_t* __restrict__ icnt, uint32_t* __restrict__ iw) {
  // entries per lane in flight: a whole item for 8-byte entries
  constexpr int NB = sizeof(E) <= 8 ? 16 : (sizeof(E) <= 16 ? 8 : 4);
  const uint32_t lane = lane_id();
  const uint32_t wave = uniform_u32((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  const uint32_t nitems = *nitems_p;
  Item I = wave < nitems ? items[wave] : Item{};
  for (uint32_t it = wave; it < nitems; it += nwaves) {
    const Item In = it + nwaves < nitems ? items[it + nwaves] : Item{};  // next item, fetched early
    const uint32_t cnt = I.cnt;
    uint32_t aw[NCH], an[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) { aw[ch] = 0; an[ch] = 0; }
    for (uint32_t k0 = 0; k0 < cnt; k0 += 64 * NB) {
      E ev[NB];
      if (k0 + 64 * NB <= cnt) {
        // a full block (the common case): no per-entry bounds
#pragma unroll
        for (int j = 0; j < NB; j++) ev[j] = ents[I.off + k0 + 64 * j + lane];
#pragma unroll
        for (int j = 0; j < NB; j++) {
          const LinS s = load_ent<FAM>(ev[j]);
          bool p[NCH];
          lin_pass<FAM, NCH>(s, lv, p);
#pragma unroll
          for (int ch = 0; ch < NCH; ch++) {
            an[ch] += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(p[ch]));
            if constexpr (!UNIT) aw[ch] += p[ch] ? (uint32_t)s.w : 0u;
          }
        }
        continue;
      }
#pragma unroll
      for (int j = 0; j < NB; j++) {
        const uint32_t k = k0 + 64 * j + lane;
        ev[j] = E{};
        if (k < cnt) ev[j] = ents[I.off + k];
      }
#pragma unroll
      for (int j = 0; j < NB; j++) {
        if (k0 + 64 * j >= cnt) break;
        const LinS s = load_ent<FAM>(ev[j]);
        const bool valid = k0 + 64 * j + lane < cnt;  // lanes past the item's end pass nothing
        bool p[NCH];
        lin_pass<FAM, NCH>(s, lv, p);
#pragma unroll
        for (int ch = 0; ch < NCH; ch++) {
          p[ch] = p[ch] && valid;
          an[ch] += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(p[ch]));
          if constexpr (!UNIT) aw[ch] += p[ch] ? (uint32_t)s.w : 0u;
        }
      }
    }
    // lane ch < NCH writes child ch's column of the item's row
    uint32_t vn = 0, vw = 0;
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) {
      const uint32_t w = UNIT ? an[ch] : wave_sum_u32(aw[ch]);
      vn = lane == (uint32_t)ch ? an[ch] : vn;
      vw = lane == (uint32_t)ch ? w : vw;
    }
    if (lane < (uint32_t)NCH) {
      icnt[(uint64_t)it * NCH + lane] = vn;
      if constexpr (!UNIT) iw[(uint64_t)it * NCH + lane] = vw;
    }
    I = In;
  }
}

// Per (cell, child): the cell's count and entries from its items' rows, and
// each item's offset inside the child's list (exclusive, within the cell).
// A cell of length len owns ceil(len / 2^ilog) items from ioff[cell].
template <int NCH, bool UNIT>
__global__ void k_cell_scan(const Cell* __restrict__ cells, uint32_t ncell, uint32_t ilog, const uint32_t* __restrict__ ioff,
                            const uint32_t* __restrict__ icnt, const uint32_t* __restrict__ iw,
                            uint64_t* __restrict__ itemoff, uint32_t* __restrict__ ccnt, uint32_t* __restrict__ cnent) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)ncell * NCH) return;
  const uint32_t c = (uint32_t)(t / NCH), ch = (uint32_t)(t % NCH);
  const uint32_t i0 = ioff[c], ni = items_of(cells[c].len, ilog);
  uint64_t n = 0, w = 0;
  for (uint32_t i = i0; i < i0 + ni; i++) {
    const uint64_t k = (uint64_t)i * NCH + ch;
    if (itemoff) itemoff[k] = n;
    n += icnt[k];
    if constexpr (!UNIT) w += iw[k];
  }
  cnent[t] = (uint32_t)n;
  ccnt[t] = (uint32_t)(UNIT ? n : w);
}

// ---------------------------------------------------------------------------
// POSE4DOF incidence: per (surface, child) the z-half and the kappa-half.
// Children (bx, by, bz, bk) share the V rectangle of their (bx, by) part.
// ---------------------------------------------------------------------------
struct PoseLevel {
  // child boxes of the item's cell, per bit value (wave-uniform)
  double Xlo[2], Xhi[2], Ylo[2], Yhi[2], ZH[2], ZL[2], Llo[2], Lhi[2];
};

__device__ inline void pose_level_boxes(const ProbC& P, const LevelC& lv, const Cell& C, int m, PoseLevel& B) {
  const int m1 = m + 1;
  double h[4];
  for (int j = 0; j < 4; j++) h[j] = ldexp(1.0, -min(m1, P.L[j]));
  for (int b = 0; b < 2; b++) {
    int32_t cx = lv.split[0] ? 2 * C.c[0] + b : C.c[0];
    int32_t cy = lv.split[1] ? 2 * C.c[1] + b : C.c[1];
    int32_t cz = lv.split[2] ? 2 * C.c[2] + b : C.c[2];
    int32_t ck = lv.split[3] ? 2 * C.c[3] + b : C.c[3];
    B.Xlo[b] = (double)cx * h[0];
    B.Xhi[b] = (double)(cx + 1) * h[0];
    B.Ylo[b] = (double)cy * h[1];
    B.Yhi[b] = (double)(cy + 1) * h[1];
    double Zlo = (double)cz * h[2], Zhi = (double)(cz + 1) * h[2];
    B.ZH[b] = Zhi + P.padz;
    B.ZL[b] = Zlo - P.padz;
    double Klo = 2.0 * ((double)ck * h[3]) - 1.0, Khi = 2.0 * ((double)(ck + 1) * h[3]) - 1.0;
    B.Llo[b] = Klo - P.padk;
    B.Lhi[b] = Khi + P.padk;
  }
}

// Pass mask of a cell's children from the half tests of one surface:
// child ch passes iff its z half and its kappa half pass.  Half-test bit
// index: bx | by << 1 | (z or kappa bit) << 2 [| bf << 3 for the f half,
// NAX = 5].  ALL (every axis splits): the digit holds the axis bits in axis
// order, most significant first, so each child's two bit indices are
// compile-time constants; otherwise they come from the level's table.
template <int NAX, bool ALL>
__device__ inline uint32_t pose_children(const LevelC& lv, uint32_t nch, uint32_t zbits, uint32_t kbits) {
  constexpr int NCH = 1 << NAX;
  uint32_t mask = 0;
  if constexpr (ALL) {
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) {
      const int bx = (ch >> (NAX - 1)) & 1, by = (ch >> (NAX - 2)) & 1, bz = (ch >> (NAX - 3)) & 1;
      const int bk = (ch >> (NAX - 4)) & 1, bf = NAX == 5 ? (ch & 1) : 0;
      const int zi = bx | (by << 1) | (bz << 2) | (bf << 3), ki = bx | (by << 1) | (bk << 2) | (bf << 3);
      mask |= (((zbits >> zi) & (kbits >> ki)) & 1u) << ch;
    }
  } else {
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) {
      if ((uint32_t)ch >= nch) break;
      const uint32_t cb = lv.cbits[ch];
      const uint32_t xy = cb & 3u, zb = (cb >> 2) & 1u, kb = (cb >> 3) & 1u, fb = NAX == 5 ? (cb >> 4) & 1u : 0u;
      if (((zbits >> (xy | (zb << 2) | (fb << 3))) & 1u) && ((kbits >> (xy | (kb << 2) | (fb << 3))) & 1u))
        mask |= 1u << ch;
    }
  }
  return mask;
}

// binary64 mask over the children of one cell for one surface.  ALL: every
// axis splits at this level (16 children), so no per-axis checks.
template <bool ALL>
__device__ inline uint32_t pose_mask64(const ProbC& P, const LevelC& lv, const PoseLevel& B, int sector,
                                       double W1, double W2, double W3, double xi, double eta) {
  const uint32_t nch = ALL ? 16u : 1u << lv.abits;
  uint32_t zbits = 0, kbits = 0;  // bit (bx | by<<1 | b<<2)
  // terms shared by the four (x, y) parts
  const ZPre<double> zp[2] = {zpre<double>(W3, eta, B.ZH[0], B.ZL[0]), zpre<double>(W3, eta, B.ZH[1], B.ZL[1])};
  const KEdge<double> ke[2] = {kedge<double>(xi, B.Llo[0], B.Lhi[0]), kedge<double>(xi, B.Llo[1], B.Lhi[1])};
#pragma unroll
  for (int xy = 0; xy < 4; xy++) {
    int bx = xy & 1, by = xy >> 1;
    if (!ALL && ((bx && !lv.split[0]) || (by && !lv.split[1]))) continue;
    VBox<double> v = pose_vbox<double>(W1, W2, B.Xlo[bx], B.Xhi[bx], B.Ylo[by], B.Yhi[by], sector);
    double rmin2 = rmin2_of(v), rmax2 = rmax2_of(v);
#pragma unroll
    for (int b = 0; b < 2; b++) {
      if (!ALL && b && !lv.split[2]) continue;
      if (zhalf64p(zp[b], rmin2, rmax2)) zbits |= 1u << (xy | (b << 2));
    }
#pragma unroll
    for (int b = 0; b < 2; b++) {
      if (!ALL && b && !lv.split[3]) continue;
      if (khalf64e(v, rmin2, P.Rg2, ke[b])) kbits |= 1u << (xy | (b << 2));
    }
  }
  return pose_children<4, ALL>(lv, nch, zbits, kbits);
}

// One child half's bounds in binary64, computed as pose_level_boxes does
// (bit-equal values): x, y by (bx, by), the z or kappa interval by bq.
__device__ inline void pose_half_bounds(const ProbC& P, const LevelC& lv, const Cell& C, int m, int bx, int by,
                                        int bq, bool kap, double& x0, double& x1, double& y0, double& y1,
                                        double& qlo, double& qhi) {
  const int m1 = m + 1;
  const int32_t cx = lv.split[0] ? 2 * C.c[0] + bx : C.c[0];
  const int32_t cy = lv.split[1] ? 2 * C.c[1] + by : C.c[1];
  const double hx = ldexp(1.0, -min(m1, P.L[0])), hy = ldexp(1.0, -min(m1, P.L[1]));
  x0 = (double)cx * hx;
  x1 = (double)(cx + 1) * hx;
  y0 = (double)cy * hy;
  y1 = (double)(cy + 1) * hy;
  if (kap) {
    const int32_t ck = lv.split[3] ? 2 * C.c[3] + bq : C.c[3];
    const double hk = ldexp(1.0, -min(m1, P.L[3]));
    const double Klo = 2.0 * ((double)ck * hk) - 1.0, Khi = 2.0 * ((double)(ck + 1) * hk) - 1.0;
    qlo = Klo - P.padk;
    qhi = Khi + P.padk;
  } else {
    const int32_t cz = lv.split[2] ? 2 * C.c[2] + bq : C.c[2];
    const double hz = ldexp(1.0, -min(m1, P.L[2]));
    const double Zlo = (double)cz * hz, Zhi = (double)(cz + 1) * hz;
    qlo = Zlo - P.padz;  // ZL
    qhi = Zhi + P.padz;  // ZH
  }
}

// binary32 mask; the undecided halves (bit index xy | b << 2 of zund /
// kund) are then recomputed in binary64 one at a time, from the entry's
// binary64 root values and the child's bounds
template <bool ALL, typename EQ>
__device__ inline uint32_t pose_mask32(const ProbC& P, const LevelC& lv, const Cell& C, int m, const float* Bf,
                                       int sector, const EQ& e, const double* __restrict__ m64,
                                       uint64_t n_root, uint32_t& nrecheck) {
  const uint32_t nch = ALL ? 16u : 1u << lv.abits;
  uint32_t zbits = 0, kbits = 0, zund = 0, kund = 0;
  // Bf layout: Xlo[2] Xhi[2] Ylo[2] Yhi[2] ZH[2] ZL[2] Llo[2] Lhi[2]
  // terms shared by the four (x, y) parts
  const ZPre<float> zp[2] = {zpre<float>(e.W3, e.eta, Bf[8], Bf[10]), zpre<float>(e.W3, e.eta, Bf[9], Bf[11])};
  const KEdge<float> ke[2] = {kedge<float>(e.xi, Bf[12], Bf[14]), kedge<float>(e.xi, Bf[13], Bf[15])};
  const float kSl[2] = {8.0f * GV_U32 * kedge_sl(ke[0]), 8.0f * GV_U32 * kedge_sl(ke[1])};
  const float kSh[2] = {8.0f * GV_U32 * kedge_sh(ke[0]), 8.0f * GV_U32 * kedge_sh(ke[1])};
#pragma unroll
  for (int xy = 0; xy < 4; xy++) {
    int bx = xy & 1, by = xy >> 1;
    if (!ALL && ((bx && !lv.split[0]) || (by && !lv.split[1]))) continue;
    VBox<float> v = pose_vbox<float>(e.W1, e.W2, Bf[0 + bx], Bf[2 + bx], Bf[4 + by], Bf[6 + by], sector);
    float rmin2 = rmin2_of(v), rmax2 = rmax2_of(v);
#pragma unroll
    for (int b = 0; b < 2; b++) {
      if (!ALL && b && !lv.split[2]) continue;
      bool u;
      const uint32_t bit = 1u << (xy | (b << 2));
      if (zhalf32m(zp[b], rmin2, rmax2, u)) zbits |= bit;
      if (u) zund |= bit;
    }
#pragma unroll
    for (int b = 0; b < 2; b++) {
      if (!ALL && b && !lv.split[3]) continue;
      bool u;
      const uint32_t bit = 1u << (xy | (b << 2));
      if (khalf32m(v, rmin2, P.Rg2f, ke[b], kSl[b], kSh[b], u)) kbits |= bit;
      if (u) kund |= bit;
    }
  }
  if (zund | kund) {
    const uint64_t r = e.ridx;
    const double W1 = m64[r], W2 = m64[n_root + r], W3 = m64[2 * n_root + r], xi = m64[3 * n_root + r],
                 eta = m64[4 * n_root + r];
    uint32_t und = zund | (kund << 8);
#pragma unroll 1
    while (und) {
      const uint32_t j = (uint32_t)__builtin_ctz(und);
      und &= und - 1u;
      const bool kap = j >= 8;
      const uint32_t i = j & 7u;
      double x0, x1, y0, y1, qlo, qhi;
      pose_half_bounds(P, lv, C, m, (int)(i & 1u), (int)((i >> 1) & 1u), (int)((i >> 2) & 1u), kap, x0, x1, y0,
                       y1, qlo, qhi);
      const VBox<double> vd = pose_vbox<double>(W1, W2, x0, x1, y0, y1, sector);
      const double rmin2d = rmin2_of(vd);
      const bool pass = kap ? khalf64(vd, rmin2d, P.Rg2, xi, qlo, qhi)
                            : zhalf64(W3, eta, rmin2d, rmax2_of(vd), qhi, qlo);
      const uint32_t bm = 1u << i;
      if (kap)
        kbits = pass ? (kbits | bm) : (kbits & ~bm);
      else
        zbits = pass ? (zbits | bm) : (zbits & ~bm);
      nrecheck++;
    }
  }
  return pose_children<4, ALL>(lv, nch, zbits, kbits);
}

// UNIT: every multiplicity is 1, so a child's count is the popcount of its
// ballot (scalar), else per-lane sums reduced across the wave.
template <typename E, bool UNIT, bool ALL>
__global__ void __launch_bounds__(256, 4) k_count_pose(const ProbC* __restrict__ Ptab, int m, LevelC lv,
                                                    const Cell* __restrict__ cells, const Item* __restrict__ items,
                                                    const uint32_t* __restrict__ nitems_p, const E* __restrict__ ents,
                                                    const double* __restrict__ m64, uint64_t n_root,
                                                    uint16_t* __restrict__ masks, uint32_t* __restrict__ ccnt,
                                                    uint32_t* __restrict__ cnent,
                                                    unsigned long long* __restrict__ rechecks,
                                                    uint32_t* __restrict__ itemcnt, uint32_t istride) {
  const uint32_t nch = ALL ? 16u : 1u << lv.abits;
  const uint32_t lane = lane_id();
  const uint32_t wave = uniform_u32((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  const uint32_t nitems = *nitems_p;
  uint32_t nre = 0;
  for (uint32_t it = wave; it < nitems; it += nwaves) {
    const Item I = items[it];
    const Cell C = cells[I.cell];
    const ProbC& P = Ptab[C.prob];
    const uint32_t cnt = I.cnt;
    const int sector = (int)C.sector;
    PoseLevel B;
    pose_level_boxes(P, lv, C, m, B);
    float Bf[16];
    for (int b = 0; b < 2; b++) {
      Bf[0 + b] = (float)B.Xlo[b]; Bf[2 + b] = (float)B.Xhi[b];
      Bf[4 + b] = (float)B.Ylo[b]; Bf[6 + b] = (float)B.Yhi[b];
      Bf[8 + b] = (float)B.ZH[b];  Bf[10 + b] = (float)B.ZL[b];
      Bf[12 + b] = (float)B.Llo[b]; Bf[14 + b] = (float)B.Lhi[b];
    }
    uint32_t aw[16], an[16];
#pragma unroll
    for (int ch = 0; ch < 16; ch++) { aw[ch] = 0; an[ch] = 0; }
    for (uint32_t k0 = 0; k0 < cnt; k0 += 64) {
      const uint32_t k = k0 + lane;
      const uint64_t ei = I.off + k;
      uint32_t mask = 0, w = 0;
      if (k < cnt) {
        const E e = ents[ei];
        w = pose_w(e);
        if constexpr (sizeof(E) == sizeof(EntQ64)) {
          mask = pose_mask64<ALL>(P, lv, B, sector, e.W1, e.W2, e.W3, e.xi, e.eta);
        } else {
          mask = pose_mask32<ALL>(P, lv, C, m, Bf, sector, e, m64, n_root, nre);
        }
        masks[ei] = (uint16_t)mask;
      }
#pragma unroll
      for (int ch = 0; ch < 16; ch++) {
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
    for (int ch = 0; ch < 16; ch++) {
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
  uint32_t tot = wave_sum_u32(nre);
  if (lane_id() == 0 && tot) atomicAdd(rechecks, (unsigned long long)tot);
}

// ---------------------------------------------------------------------------
// Pruning against the best key (counts only shrink down the tree, so a cell
// whose best possible key cannot beat the best leaf found so far is dropped)
// and, at the last level, the best-key reduction (u64 atomic max).
// key = count * 2^B + (2^B - 1 - leaf index): largest count, lowest index.
// ---------------------------------------------------------------------------
// Best-key update of a wave's leaf keys: when every active lane belongs to
// one problem (the usual case) the wave reduces its maximum first and one
// lane issues the atomic; otherwise every lane does.  Every lane of the wave
// must call it (inactive ones with active = false).
__device__ inline void wave_best_max(unsigned long long* __restrict__ best, uint32_t prob, uint64_t key,
                                     bool active) {
  const uint64_t act = __builtin_amdgcn_ballot_w64(active);
  if (!act) return;
  const uint32_t lead = (uint32_t)__builtin_ctzll(act);
  const uint32_t p0 = __shfl(prob, (int)lead, 64);
  if (__builtin_amdgcn_ballot_w64(active && prob != p0) == 0ull) {
    uint64_t k = active ? key : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint64_t y = __shfl_xor(k, o, 64);
      k = y > k ? y : k;
    }
    if (lane_id() == lead && k > best[p0]) atomicMax(&best[p0], (unsigned long long)k);
  } else if (active && key > best[prob]) {
    atomicMax(&best[prob], (unsigned long long)key);
  }
}

__global__ void k_prune(LevelC lv, int B, uint64_t idxmask, int leaf, const Cell* __restrict__ cells, uint32_t ncell,
                        const uint32_t* __restrict__ ccnt, const uint32_t* __restrict__ cnent,
                        unsigned long long* __restrict__ best, uint32_t* __restrict__ keepf,
                        uint64_t* __restrict__ keptn) {
  const uint32_t nch = 1u << lv.abits;
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nk = (uint64_t)ncell * nch;
  if (leaf) {  // (uniform: the whole wave stays for the reduction)
    const bool act = k < nk;
    uint64_t key = 0;
    uint32_t prob = 0;
    if (act) {
      const uint32_t c = (uint32_t)(k / nch), ch = (uint32_t)(k % nch);
      const uint64_t pre = (cells[c].prefix << lv.abits) | ch;
      key = ((uint64_t)ccnt[k] << B) | (idxmask - (pre << lv.rem_next));
      prob = cells[c].prob;
    }
    wave_best_max(best, prob, key, act);
    return;
  }
  if (k >= nk) return;
  const uint32_t c = (uint32_t)(k / nch), ch = (uint32_t)(k % nch);
  const Cell& C = cells[c];
  const uint64_t pre = (C.prefix << lv.abits) | ch;
  const uint64_t idxmin = pre << lv.rem_next;
  const uint64_t key = ((uint64_t)ccnt[k] << B) | (idxmask - idxmin);
  unsigned long long* bp = &best[C.prob];
  {
    const uint32_t keep = key > *bp ? 1u : 0u;
    keepf[k] = keep;
    keptn[k] = keep ? (uint64_t)cnent[k] : 0ull;
  }
}

// Threshold reporting at the last level: every leaf whose key exceeds its
// problem's fixed bound tau 2^B - 1 (count >= tau) is appended to the output
// (up to cap; *n counts them all).  At this level a child's digit completes
// its leaf index.
__global__ void k_report_leaves(LevelC lv, int B, uint64_t idxmask, const Cell* __restrict__ cells, uint32_t ncell,
                                const uint32_t* __restrict__ ccnt, const unsigned long long* __restrict__ best,
                                uint64_t* __restrict__ out_idx, uint32_t* __restrict__ out_cnt,
                                unsigned long long* __restrict__ n, uint64_t cap) {
  const uint32_t nch = 1u << lv.abits;
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (uint64_t)ncell * nch) return;
  const uint32_t c = (uint32_t)(k / nch), ch = (uint32_t)(k % nch);
  const uint64_t idx = ((cells[c].prefix << lv.abits) | ch) << lv.rem_next;
  const uint64_t key = ((uint64_t)ccnt[k] << B) | (idxmask - idx);
  if (key > best[cells[c].prob]) {
    const unsigned long long slot = atomicAdd(n, 1ull);
    if (slot < cap) {
      out_idx[slot] = idx;
      out_cnt[slot] = ccnt[k];
    }
  }
}

// Greedy dive: in every cell keep only the best child (count, then lowest
// digit); at the last level record its key.
__global__ void k_pick_best(LevelC lv, int B, uint64_t idxmask, int leaf, const Cell* __restrict__ cells,
                            uint32_t ncell, const uint32_t* __restrict__ ccnt, const uint32_t* __restrict__ cnent,
                            unsigned long long* __restrict__ best, uint32_t* __restrict__ keepf,
                            uint64_t* __restrict__ keptn) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = c < ncell;
  const uint32_t nch = 1u << lv.abits;
  const uint64_t o = (uint64_t)c * nch;
  uint32_t bc = 0, bd = 0;
  if (act) {
    for (uint32_t ch = 0; ch < nch; ch++)
      if (ch == 0 || ccnt[o + ch] > bc) { bc = ccnt[o + ch]; bd = ch; }
    for (uint32_t ch = 0; ch < nch; ch++) {
      keepf[o + ch] = (ch == bd) ? 1u : 0u;
      keptn[o + ch] = (ch == bd) ? (uint64_t)cnent[o + ch] : 0ull;
    }
  }
  if (leaf) {  // (uniform: the whole wave stays for the reduction)
    uint64_t key = 0;
    uint32_t prob = 0;
    if (act) {
      const uint64_t pre = (cells[c].prefix << lv.abits) | bd;
      key = ((uint64_t)bc << B) | (idxmask - (pre << lv.rem_next));
      prob = cells[c].prob;
    }
    wave_best_max(best, prob, key, act);
  }
}

// Greedy dive above the leaves: every cell keeps its best child, in parent
// order, so rank r is cell r.  Writes the kept list directly: order (child
// index), count, entries, and each child's rank (~0 for the dropped ones).
__global__ void k_pick_kept(LevelC lv, uint32_t ncell, const uint32_t* __restrict__ ccnt,
                            const uint32_t* __restrict__ cnent, uint32_t* __restrict__ order,
                            uint32_t* __restrict__ scount, uint32_t* __restrict__ sn, uint32_t* __restrict__ rank_of) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const uint32_t nch = 1u << lv.abits;
  const uint64_t o = (uint64_t)c * nch;
  uint32_t bc = 0, bd = 0;
  for (uint32_t ch = 0; ch < nch; ch++)
    if (ch == 0 || ccnt[o + ch] > bc) { bc = ccnt[o + ch]; bd = ch; }
  for (uint32_t ch = 0; ch < nch; ch++) rank_of[o + ch] = ch == bd ? c : 0xffffffffu;
  order[c] = (uint32_t)(o + bd);
  scount[c] = bc;
  sn[c] = cnent[o + bd];
}

// the host's totals from a scan's last value: out[0] = n, out[1] = *sum
// (host-coherent memory)
__global__ void k_tot_from(uint64_t n, const uint64_t* __restrict__ sum, uint64_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = n;
    out[1] = *sum;
    __threadfence_system();
  }
}

// ---------------------------------------------------------------------------
// Ordering of kept children: highest count first (radix sort on the host
// side), so the first descent of the depth-first search follows the most
// promising cells like a beam and reaches a strong lower bound early.
// ---------------------------------------------------------------------------
__global__ void k_select_kept(const uint32_t* __restrict__ keepf, const uint32_t* __restrict__ keepscan,
                              const uint32_t* __restrict__ ccnt, uint64_t nk, uint32_t* __restrict__ kcnt,
                              uint32_t* __restrict__ kid, uint32_t* __restrict__ rank_of) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nk) rank_of[k] = 0xffffffffu;  // k_rank fills in the kept children
  if (k < nk && keepf[k]) {
    kcnt[keepscan[k]] = ccnt[k];
    kid[keepscan[k]] = (uint32_t)k;
  }
}

__global__ void k_kept_total(const uint32_t* keepf, const uint32_t* keepscan, uint64_t nk, const uint64_t* esum,
                             uint64_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = nk ? (uint64_t)keepscan[nk - 1] + keepf[nk - 1] : 0;
    out[1] = *esum;
    __threadfence_system();
  }
}

// rank_of[k] = position of child k in the sorted order; sn[r] = its entries
__global__ void k_rank(const uint32_t* __restrict__ order, uint32_t nkept, const uint32_t* __restrict__ cnent,
                       const uint32_t* __restrict__ ccnt, uint32_t* __restrict__ rank_of, uint32_t* __restrict__ sn,
                       uint32_t* __restrict__ scount) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nkept) {
    const uint32_t k = order[r];
    rank_of[k] = r;
    sn[r] = cnent[k];
    scount[r] = ccnt[k];
  }
}

// several problems in a batch: order children by their count relative to
// the largest kept count of their own problem, so the first chunks carry
// the most promising cells of every problem
__global__ void k_prob_max(const uint32_t* __restrict__ kcnt, const uint32_t* __restrict__ kid, uint32_t nkept,
                           const Cell* __restrict__ cells, uint32_t nch, uint32_t* __restrict__ pmax) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nkept) atomicMax(&pmax[cells[kid[r] / nch].prob], kcnt[r]);
}
__global__ void k_prob_norm(const uint32_t* __restrict__ kcnt, const uint32_t* __restrict__ kid, uint32_t nkept,
                            const Cell* __restrict__ cells, uint32_t nch, const uint32_t* __restrict__ pmax,
                            uint32_t* __restrict__ key) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nkept) {
    const uint32_t m = pmax[cells[kid[r] / nch].prob];
    key[r] = m ? (uint32_t)(((uint64_t)kcnt[r] << 30) / m) : 0u;
  }
}
__global__ void k_soff_last(uint64_t* soff, const uint32_t* sn, uint32_t nkept) {
  if (threadIdx.x == 0 && blockIdx.x == 0) soff[nkept] = nkept ? soff[nkept - 1] + sn[nkept - 1] : 0;
}
// out may be host-coherent memory the host reads after the stream wait
__global__ void k_gather_u64(const uint64_t* __restrict__ a, uint64_t n, uint64_t stride, uint64_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t m = (n + stride - 1) / stride;
  if (i < m) out[i] = a[i * stride];
  if (i == 0) out[m] = a[n];
  __threadfence_system();
}

// Re-cut a pending chunk [r0, r1) against the current bounds: a child is
// kept only if its count can still reach the best leaf of its own problem.
// keepc / csize are chunk-local (index r - r0).
// keep_all: no re-cut (a chunk materialized right after its parent's
// pruning, whose bounds cannot have moved; its sizes are then known).
__global__ void k_chunk_keep(const uint32_t* __restrict__ order, const uint32_t* __restrict__ scount,
                             const Cell* __restrict__ cells, uint32_t nch, const unsigned long long* __restrict__ best,
                             int B, uint32_t r0, uint32_t r1, const uint32_t* __restrict__ cnent,
                             uint32_t* __restrict__ keepc, uint64_t* __restrict__ csize, int keep_all) {
  const uint32_t r = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= r1) return;
  const uint32_t k = order[r];
  const uint64_t bc = (uint64_t)(best[cells[k / nch].prob] >> B);
  const uint32_t keep = (keep_all || (uint64_t)scount[r] >= bc) ? 1u : 0u;
  keepc[r - r0] = keep;
  csize[r - r0] = keep ? (uint64_t)cnent[k] : 0ull;
}

__global__ void k_chunk_totals(const uint32_t* keepc, const uint32_t* cidx, const uint64_t* csize,
                               const uint64_t* coff, uint32_t n, uint64_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = n ? (uint64_t)cidx[n - 1] + keepc[n - 1] : 0;
    out[1] = n ? coff[n - 1] + csize[n - 1] : 0;
    __threadfence_system();
  }
}

// entries of the parent cells that have a child in [r0, r1): what one
// compaction pass must read
__global__ void k_chunk_reads(const Cell* __restrict__ cells, uint32_t ncell, uint32_t nch,
                              const uint32_t* __restrict__ rank_of, uint32_t r0, uint32_t r1,
                              const uint32_t* __restrict__ keepc, uint32_t bits_per_entry,
                              unsigned long long* __restrict__ acc) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t v = 0;
  if (c < ncell) {
    bool hit = false;
    for (uint32_t ch = 0; ch < nch; ch++) {
      const uint32_t r = rank_of[(uint64_t)c * nch + ch];
      hit = hit || (r >= r0 && r < r1 && keepc[r - r0]);
    }
    v = hit ? (uint64_t)cells[c].len * bits_per_entry : 0;
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63u) == 0 && v) atomicAdd(acc, (unsigned long long)v);
}

// cells of a materialized chunk, in rank order
__global__ void k_emit_ranked(LevelC lv, const Cell* __restrict__ cells, const uint32_t* __restrict__ order,
                              uint32_t r0, uint32_t r1, const uint32_t* __restrict__ keepc,
                              const uint32_t* __restrict__ cidx, const uint64_t* __restrict__ coff,
                              const uint32_t* __restrict__ cnent, Cell* __restrict__ out) {
  const uint32_t r = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= r1 || !keepc[r - r0]) return;
  const uint32_t nch = 1u << lv.abits;
  const uint32_t k = order[r];
  const uint32_t c = k / nch, ch = k % nch;
  const Cell P = cells[c];
  Cell o;
  const uint32_t cb = lv.cbits[ch];
  for (int a = 0; a < GV_MAXD; a++) o.c[a] = lv.split[a] ? 2 * P.c[a] + (int32_t)((cb >> a) & 1u) : P.c[a];
  o.prefix = (P.prefix << lv.abits) | ch;
  o.off = coff[r - r0];
  o.len = cnent[k];
  o.sector = P.sector;
  o.prob = P.prob;
  o._pad = 0;
  out[cidx[r - r0]] = o;
}

// ---------------------------------------------------------------------------
// Compaction of one chunk: survivors whose child's rank lies in [r0, r1) go
// into that child's list, canonized to it.  Write positions are known in
// advance: the count pass recorded every item's per-child survivors, and
// their exclusive scan (itemoff, child-major) gives each item's offset inside
// the child's list; within an item, a wavefront ballot ranks the lanes.
// ---------------------------------------------------------------------------
// Work list of one linear-family compaction pass: the items whose cell has a
// child in the chunk, each with its kept children and, per kept child, where
// its survivors go (the child's list offset plus the item's offset inside
// that list).  One thread per item; a wave appends its records with one
// atomic.
template <int NCH> struct CWork {
  uint64_t off;
  uint32_t cnt, kmask;
  uint64_t wpos[NCH];
};

// Items a chunk [r0, r1) of a parent's kept children can draw from, written
// to out[0], out[1] (host-coherent memory): in parent order (sorted == 0)
// the chunk's children belong to a contiguous range of parent cells, so
// only those cells' items; in count order every item.  Also clears the work
// list's counter.
__global__ void k_chunk_range(const uint32_t* __restrict__ order, uint32_t r0, uint32_t r1, uint32_t nch,
                              const uint32_t* __restrict__ ioff, uint32_t ncell, const uint32_t* __restrict__ nitems_p,
                              int sorted, uint32_t* __restrict__ nwork, uint64_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *nwork = 0;
    if (sorted || r1 <= r0) {
      out[0] = 0;
      out[1] = *nitems_p;
    } else {
      const uint32_t c0 = order[r0] / nch, c1 = order[r1 - 1] / nch;
      out[0] = ioff[c0];
      out[1] = c1 + 1 < ncell ? ioff[c1 + 1] : *nitems_p;
    }
    __threadfence_system();
  }
}

// One thread per item of [i0, i1); with acc, also the bits of the entries
// the compaction reads (items with a kept child in the chunk).
template <int NCH>
__global__ void k_chunk_work(const Item* __restrict__ items, const uint32_t* __restrict__ nitems_p, uint32_t i0,
                             uint32_t i1,
                             const uint64_t* __restrict__ itemoff, const uint32_t* __restrict__ rank_of, uint32_t r0,
                             uint32_t r1, const uint32_t* __restrict__ keepc, const uint64_t* __restrict__ coff,
                             CWork<NCH>* __restrict__ work, uint32_t* __restrict__ nwork, uint32_t bits_per_entry,
                             unsigned long long* __restrict__ acc) {
  const uint32_t it = i0 + blockIdx.x * blockDim.x + threadIdx.x;
  CWork<NCH> w{};
  if (it < i1 && it < *nitems_p) {
    const Item I = items[it];
    w.off = I.off;
    w.cnt = I.cnt;
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) {
      const uint32_t r = rank_of[(uint64_t)I.cell * NCH + ch];
      if (r >= r0 && r < r1 && keepc[r - r0]) {
        w.kmask |= 1u << ch;
        w.wpos[ch] = coff[r - r0] + itemoff[(uint64_t)it * NCH + ch];
      }
    }
  }
  if (acc) {
    uint64_t v = w.kmask ? (uint64_t)w.cnt * bits_per_entry : 0ull;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63u) == 0 && v) atomicAdd(acc, (unsigned long long)v);
  }
  const uint64_t b = __ballot(w.kmask != 0u);
  if (!b) return;
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(nwork, (uint32_t)__popcll(b));
  base = __shfl(base, 0, 64);
  if (w.kmask) work[base + mbcnt64(b)] = w;
}

// Linear-family compaction over the work list: every entry of a work item is
// re-tested; a kept child's ballot gives the lanes to write and, by its bit
// count below the lane, their order.  The child list may use the packed
// entry; a value that does not fit sets *ovf.
template <int FAM, typename E, typename EO, int NCH>
__global__ void __launch_bounds__(256) k_compact_lin(LevelC lv, const CWork<NCH>* __restrict__ work,
                                                     const uint32_t* __restrict__ nwork_p, const E* __restrict__ ents,
                                                     EO* __restrict__ out, int* __restrict__ ovf) {
  constexpr int GJ = sizeof(E) <= 8 ? 8 : 4;  // entries per lane in flight
  bool fits = true;
  const uint32_t lane = lane_id();
  const uint32_t wave = uniform_u32((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  const uint32_t nwork = *nwork_p;
  if constexpr (FAM == FAM_PLANE3D && NCH == 8 &&
                (std::is_same<EO, EntP3p>::value || std::is_same<EO, EntP3u>::value)) {
    constexpr bool UW = std::is_same<EO, EntP3u>::value;  // one-word unit-weight child entries
    // Every axis splits; child digit = 4 b1 + 2 b2 + b0 (split axes in axis
    // order, most significant first).  The pass test compares
    // t = 2F + pad + S + b1 K1 + b2 K2 - b0 H against [0, R] (unsigned), and
    // the child's canonical height is rne((2F + b1 K1 + b2 K2 - b0 H) / 2) =
    // rne((t - pad - S) / 2), so a child costs a subtraction and a rounding.
    // K1', K2' and the weight (the low word and the top of the high word) are
    // the same in every child.  The written heights' range is checked once
    // at the end; a packed input's K and weight always fit.
    // A wave holds a whole item (16 entries per lane) and writes its
    // survivors child by child, so each child list receives one sequential
    // run per item instead of eight interleaved ones (measured 11% faster
    // than writing all children per entry).
    const int32_t H = lv.H[2], pad = lv.padu[2];
    int32_t flo = 0, fhi = 0;
    for (uint32_t wi = wave; wi < nwork; wi += nwaves) {
      const CWork<8>* Wp = work + wi;
      const uint64_t off = uniform_u64(Wp->off);
      const uint32_t cnt = uniform_u32(Wp->cnt);
      const uint32_t kmask = uniform_u32(Wp->kmask);
      // each kept child's run starts at a wave-uniform address; the
      // position inside the run (< cnt) is a scalar 32-bit count, so a
      // store is a scalar base plus one per-lane offset
      EO* cbase[8];
      uint32_t cpos[8];
      bool kept[8];
#pragma unroll
      for (int ch = 0; ch < 8; ch++) {
        kept[ch] = (kmask >> ch) & 1u;
        cbase[ch] = out + (kept[ch] ? uniform_u64(Wp->wpos[ch]) : 0ull);
        cpos[ch] = 0u;
      }
      constexpr int G = GV_ITEM / 64;
      for (uint32_t k0 = 0; k0 < cnt; k0 += 64 * G) {
        E ev[G];
#pragma unroll
        for (int j = 0; j < G; j++) {
          const uint32_t k = k0 + 64 * j + lane;
          ev[j] = E{};
          if (k < cnt) ev[j] = ents[off + k];
        }
        int32_t U[G], BASE[G], KA[G], KB[G];
        uint32_t RR[G], LO[G], WHI[G];
        bool V[G];  // lanes past the item's end pass nothing
#pragma unroll
        for (int j = 0; j < G; j++) {
          const LinS s = load_ent<FAM>(ev[j]);
          const int32_t K1 = s.K[0][0], K2 = s.K[0][1], K12 = K1 + K2;
          const int32_t S = imax32(K1, 0) + imax32(K2, 0);
          V[j] = k0 + 64 * j + lane < cnt;
          const int32_t F = s.F[0];
          U[j] = 2 * F + pad + S;
          BASE[j] = pad + S;
          KA[j] = K1;
          KB[j] = K2;
          RR[j] = (uint32_t)(2 * S + (H + 2 * pad) - K12);
          const int32_t K1c = rne_half(K1), K2c = rne_half(K2);
          const uint32_t w = (uint32_t)s.w;
          if constexpr (UW) {
            // a one-word input's K and weight always fit
            if constexpr (!std::is_same<E, EntP3u>::value)
              fits = fits && abs(K1c) <= GV_P3U_KMAX && abs(K2c) <= GV_P3U_KMAX && (w == 1u || !V[j]);
            LO[j] = ((uint32_t)K1c & 0xffu) | (((uint32_t)K2c & 0xffu) << 8);
            WHI[j] = 0u;
          } else {
            if constexpr (!std::is_same<E, EntP3p>::value)
              fits = fits && abs(K1c) <= GV_P3_KMAX && abs(K2c) <= GV_P3_KMAX && w <= GV_P3_WMAX;
            LO[j] = ((uint32_t)K1c & 0x1fffu) | (((uint32_t)K2c & 0x1fffu) << 13) | ((w & 0x3fu) << 26);
            WHI[j] = (w >> 6) << 16;
          }
        }
#pragma unroll
        for (int ch = 0; ch < 8; ch++) {
          if (!kept[ch]) continue;
#pragma unroll
          for (int j = 0; j < G; j++) {
            if (k0 + 64 * j >= cnt) break;
            const int32_t uu = U[j] + ((ch & 4) ? KA[j] : 0) + ((ch & 2) ? KB[j] : 0);
            const int32_t t = (ch & 1) ? uu - H : uu;
            const bool c = V[j] && (uint32_t)t <= RR[j];
            const uint64_t b = __builtin_amdgcn_ballot_w64(c);
            if (c) {
              const int32_t Fc = rne_half(t - BASE[j]);
              flo = imin32(flo, Fc);
              fhi = imax32(fhi, Fc);
              EO e;
              if constexpr (UW) {
                e.v = LO[j] | ((uint32_t)Fc << 16);
              } else {
                e.lo = LO[j];
                e.hi = ((uint32_t)Fc & 0xffffu) | WHI[j];
              }
              // 32-bit byte offset (< GV_ITEM entries) from the scalar base
              const uint32_t boff = (cpos[ch] + mbcnt64(b)) * (uint32_t)sizeof(EO);
              *reinterpret_cast<EO*>(reinterpret_cast<char*>(cbase[ch]) + boff) = e;
            }
            cpos[ch] = uniform_u32(cpos[ch] + (uint32_t)__popcll(b));
          }
        }
      }
    }
    fits = fits && flo >= -GV_P3_FMAX && fhi <= GV_P3_FMAX;
    if (!fits) atomicOr(ovf, 1);
    return;
  }
  for (uint32_t wi = wave; wi < nwork; wi += nwaves) {
    const CWork<NCH> W = work[wi];
    const uint32_t kmask = W.kmask;
    const uint32_t cnt = W.cnt;
    uint64_t wpos[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) wpos[ch] = W.wpos[ch];
    for (uint32_t k0 = 0; k0 < cnt; k0 += 64 * GJ) {
      E ev[GJ];
#pragma unroll
      for (int j = 0; j < GJ; j++) {
        const uint32_t k = k0 + 64 * j + lane;
        ev[j] = E{};
        if (k < cnt) ev[j] = ents[W.off + k];
      }
#pragma unroll
      for (int j = 0; j < GJ; j++) {
        if (k0 + 64 * j >= cnt) break;
        const LinS s = load_ent<FAM>(ev[j]);
        const bool valid = k0 + 64 * j + lane < cnt;  // lanes past the item's end pass nothing
        bool p[NCH];
        lin_pass<FAM, NCH>(s, lv, p);
#pragma unroll
        for (int ch = 0; ch < NCH; ch++) {
          if (!((kmask >> ch) & 1u)) continue;
          p[ch] = p[ch] && valid;
          const uint64_t b = __builtin_amdgcn_ballot_w64(p[ch]);
          if (p[ch]) out[wpos[ch] + mbcnt64(b)] = store_ent<FAM, EO>(lin_canon_child<FAM>(s, lv, lv.cbits[ch]), fits);
          wpos[ch] += (uint64_t)__popcll(b);
        }
      }
    }
  }
  if (!fits) atomicOr(ovf, 1);
}

// a copied word as a clang vector, for stores through a global-memory pointer
template <typename W> struct WordVec;
template <> struct WordVec<uint4> {
  using T = uint32_t __attribute__((ext_vector_type(4)));
  __device__ static T of(const uint4& v) { return T{v.x, v.y, v.z, v.w}; }
};
template <> struct WordVec<uint2> {
  using T = uint32_t __attribute__((ext_vector_type(2)));
  __device__ static T of(const uint2& v) { return T{v.x, v.y}; }
};

// Linear families re-encode on the way (the child list may use the packed
// entry); a value that does not fit its encoding sets *ovf.
template <int FAM, typename E, typename EO, typename M, bool POSE>
__global__ void __launch_bounds__(256) k_compact(LevelC lv, const Cell* __restrict__ cells,
                                                 const Item* __restrict__ items, const uint32_t* __restrict__ nitems_p,
                                                 const uint32_t* __restrict__ ioff, const uint64_t* __restrict__ itemoff,
                                                 uint32_t istride, const E* __restrict__ ents,
                                                 const M* __restrict__ masks, const uint32_t* __restrict__ rank_of,
                                                 uint32_t r0, uint32_t r1, const uint32_t* __restrict__ keepc,
                                                 const uint64_t* __restrict__ coff, EO* __restrict__ out,
                                                 int* __restrict__ ovf) {
  bool fits = true;
  // children a cell can have: one bit of the pass mask each
  constexpr uint32_t NCP = POSE ? 8u * (uint32_t)sizeof(M) : 8u;
  const uint32_t nch = 1u << lv.abits;
  const uint32_t lane = lane_id();
  const uint32_t wave = uniform_u32((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  const uint32_t nitems = *nitems_p;
  for (uint32_t it = wave; it < nitems; it += nwaves) {
    const Item I = items[it];
    uint32_t kmask = 0;
    uint64_t wpos[NCP];
    const uint32_t first = ioff[I.cell];
#pragma unroll
    for (uint32_t ch = 0; ch < NCP; ch++) {
      wpos[ch] = 0;
      if (ch >= nch) continue;
      const uint32_t r = rank_of[(uint64_t)I.cell * nch + ch];
      if (r >= r0 && r < r1 && keepc[r - r0]) {
        kmask |= 1u << ch;
        wpos[ch] = coff[r - r0] + (itemoff[(uint64_t)ch * istride + it] - itemoff[(uint64_t)ch * istride + first]);
      }
    }
    kmask = uniform_u32(kmask);
    if (!kmask) continue;
    const uint32_t cnt = I.cnt;
    if constexpr (POSE) {
      // G entries per lane in registers, survivors written child by child:
      // one sequential run per child list instead of one interleaved piece
      // per child and row
      // Entries move as words the copy never looks inside (16-byte words,
      // or 8-byte ones for the 24-byte unit entry).  EntQ32 -> EntQ24 drops
      // the weight (1 in a unit list) and the padding on the way.
      constexpr bool CONV = std::is_same<E, EntQ32>::value && std::is_same<EO, EntQ24>::value;
      static_assert(CONV || std::is_same<E, EO>::value, "pose entries are copied whole");
      using Wd = std::conditional_t<sizeof(EO) % 16 == 0, uint4, uint2>;
      constexpr int NV = sizeof(EO) / sizeof(Wd);
      // (32-child masks: fewer entries per lane, the store loop runs per child)
      constexpr int G = sizeof(EO) <= 32 && NCP <= 16 ? 16 : 8;
      // each child's run continues at a wave-uniform byte address; a lane
      // adds its 32-bit rank offset, so a store is a scalar base plus one
      // per-lane offset
      using gchar = __attribute__((address_space(1))) char;  // global memory
      gchar* cb[NCP];
#pragma unroll
      for (uint32_t ch = 0; ch < NCP; ch++)
        cb[ch] = (gchar*)out + uniform_u64(wpos[ch]) * sizeof(EO);  // address-space cast
      for (uint32_t k0 = 0; k0 < cnt; k0 += 64 * G) {
        uint32_t mk[G];
        Wd ev[G][NV];
#pragma unroll
        for (int j = 0; j < G; j++) {
          const uint32_t k = k0 + 64 * j + lane;
          mk[j] = k < cnt ? (uint32_t)masks[I.off + k] & kmask : 0u;
        }
#pragma unroll
        for (int j = 0; j < G; j++) {
          const uint64_t ei = I.off + k0 + 64 * j + lane;
          if constexpr (CONV) {
            uint4 lo = make_uint4(0u, 0u, 0u, 0u), hi = lo;
            if (mk[j]) {
              lo = reinterpret_cast<const uint4*>(ents + ei)[0];  // W1 W2 W3 xi
              hi = reinterpret_cast<const uint4*>(ents + ei)[1];  // eta w ridx pad
            }
            ev[j][0] = make_uint2(lo.x, lo.y);
            ev[j][1] = make_uint2(lo.z, lo.w);
            ev[j][2] = make_uint2(hi.x, hi.z);
          } else {
#pragma unroll
            for (int q = 0; q < NV; q++) {
              ev[j][q] = Wd{};
              if (mk[j]) ev[j][q] = reinterpret_cast<const Wd*>(ents + ei)[q];
            }
          }
        }
        // Every entry load of the block completes here, once.  Without this
        // wait the loads' lane-dependent branches leave the compiler unsure
        // which of them are outstanding, and it waits for the whole memory
        // counter (stores included) before every store.  Encoding:
        // vmcnt(0), expcnt and lgkmcnt left at their maxima.
        __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
        for (uint32_t ch = 0; ch < NCP; ch++) {
          if (!((kmask >> ch) & 1u)) continue;
#pragma unroll
          for (int j = 0; j < G; j++) {
            if (k0 + 64 * j >= cnt) break;
            const bool p = (mk[j] >> ch) & 1u;
            const uint64_t bal = __ballot(p);
            if (p) {
              using gV = __attribute__((address_space(1))) typename WordVec<Wd>::T;
              gV* d = (gV*)(cb[ch] + mbcnt64(bal) * (uint32_t)sizeof(EO));
#pragma unroll
              for (int q = 0; q < NV; q++) d[q] = WordVec<Wd>::of(ev[j][q]);
            }
            cb[ch] += (uint32_t)__popcll(bal) * (uint32_t)sizeof(EO);
          }
        }
      }
      continue;
    }
    for (uint32_t k0 = 0; k0 < cnt; k0 += 64) {
      const uint32_t k = k0 + lane;
      const bool valid = k < cnt;
      const uint64_t ei = I.off + k;
      uint32_t mask = 0;
      E e;
      if (valid) {
        mask = (uint32_t)masks[ei] & kmask;
        if (mask) e = ents[ei];
      }
#pragma unroll
      for (uint32_t ch = 0; ch < NCP; ch++) {
        if (!((kmask >> ch) & 1u)) continue;
        const bool p = (mask >> ch) & 1u;
        const uint64_t bal = __ballot(p);
        if (p) {
          const uint64_t pos = wpos[ch] + mbcnt64(bal);
          if constexpr (!POSE)  // (POSE4DOF lists take the path above)
            out[pos] = store_ent<FAM, EO>(lin_canon_child<FAM>(load_ent<FAM>(e), lv, lv.cbits[ch]), fits);
        }
        wpos[ch] += (uint64_t)__popcll(bal);
      }
    }
  }
  if (!fits) atomicOr(ovf, 1);
}

// ---------------------------------------------------------------------------
// Grouping (Sec. 3.2.1: surfaces that canonize to the same surface in a cell
// merge, their multiplicities add).  Sort key = (cell, 64-bit hash of the
// canonical tuple); adjacent entries with the same key AND the same tuple
// merge.  A hash collision can only leave duplicates unmerged, which never
// changes a count.
// ---------------------------------------------------------------------------
__device__ inline uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}
__device__ inline uint64_t hcomb(uint64_t h, uint64_t v) { return mix64(h ^ (v + 0x9e3779b97f4a7c15ull + (h << 6))); }

template <typename E> struct Tuple;
template <> struct Tuple<EntL2> {
  __device__ static uint64_t hash(const EntL2& e) { return hcomb(hcomb(1, (uint32_t)e.K), (uint32_t)e.F); }
  __device__ static bool same(const EntL2& a, const EntL2& b) { return a.K == b.K && a.F == b.F; }
  __device__ static void setw(EntL2& e, uint32_t w) { e.w = (int32_t)w; }
  __device__ static uint32_t w(const EntL2& e) { return (uint32_t)e.w; }
};
template <> struct Tuple<EntP3> {
  __device__ static uint64_t hash(const EntP3& e) {
    return hcomb(hcomb(hcomb(2, (uint32_t)e.K1), (uint32_t)e.K2), (uint32_t)e.F);
  }
  __device__ static bool same(const EntP3& a, const EntP3& b) { return a.K1 == b.K1 && a.K2 == b.K2 && a.F == b.F; }
  __device__ static void setw(EntP3& e, uint32_t w) { e.w = (int32_t)w; }
  __device__ static uint32_t w(const EntP3& e) { return (uint32_t)e.w; }
};
template <> struct Tuple<EntL2p> {
  __device__ static uint64_t hash(const EntL2p& e) {
    return hcomb(hcomb(6, (uint32_t)(int32_t)e.K), (uint32_t)(int32_t)e.F);
  }
  __device__ static bool same(const EntL2p& a, const EntL2p& b) { return a.K == b.K && a.F == b.F; }
  __device__ static void setw(EntL2p& e, uint32_t w) { e.w = w; }
  __device__ static uint32_t w(const EntL2p& e) { return e.w; }
};
// a merged PLANE3D weight never exceeds the problem size, below the 22-bit
// limit whenever packed entries are used
template <> struct Tuple<EntP3p> {
  __device__ static uint64_t hash(const EntP3p& e) { return hcomb(hcomb(7, e.lo & 0x3ffffffu), e.hi & 0xffffu); }
  __device__ static bool same(const EntP3p& a, const EntP3p& b) {
    return (a.lo & 0x3ffffffu) == (b.lo & 0x3ffffffu) && (a.hi & 0xffffu) == (b.hi & 0xffffu);
  }
  __device__ static void setw(EntP3p& e, uint32_t w) {
    e.lo = (e.lo & 0x3ffffffu) | ((w & 0x3fu) << 26);
    e.hi = (e.hi & 0xffffu) | ((w >> 6) << 16);
  }
  __device__ static uint32_t w(const EntP3p& e) { return ((e.hi >> 16) << 6) | (e.lo >> 26); }
};
template <> struct Tuple<EntR3> {
  __device__ static uint64_t hash(const EntR3& e) {
    uint64_t h = hcomb(3, (uint32_t)e.tag);
    h = hcomb(h, (uint32_t)e.K1);
    h = hcomb(h, (uint32_t)e.K2);
    h = hcomb(h, (uint32_t)e.F1);
    return hcomb(h, (uint32_t)e.F2);
  }
  __device__ static bool same(const EntR3& a, const EntR3& b) {
    return a.tag == b.tag && a.K1 == b.K1 && a.K2 == b.K2 && a.F1 == b.F1 && a.F2 == b.F2;
  }
  __device__ static void setw(EntR3& e, uint32_t w) { e.w = (int32_t)w; }
  __device__ static uint32_t w(const EntR3& e) { return (uint32_t)e.w; }
};
template <> struct Tuple<EntS2> {
  __device__ static uint64_t hash(const EntS2& e) {
    uint64_t h = hcomb(9, (uint32_t)e.K00);
    h = hcomb(h, (uint32_t)e.K01);
    h = hcomb(h, (uint32_t)e.K10);
    h = hcomb(h, (uint32_t)e.K11);
    h = hcomb(h, (uint32_t)e.F0);
    return hcomb(h, (uint32_t)e.F1);
  }
  __device__ static bool same(const EntS2& a, const EntS2& b) {
    return a.K00 == b.K00 && a.K01 == b.K01 && a.K10 == b.K10 && a.K11 == b.K11 && a.F0 == b.F0 && a.F1 == b.F1;
  }
  __device__ static void setw(EntS2& e, uint32_t w) { e.w = (int32_t)w; }
  __device__ static uint32_t w(const EntS2& e) { return (uint32_t)e.w; }
};
template <> struct Tuple<EntQ32> {
  __device__ static uint64_t hash(const EntQ32& e) {
    uint64_t h = hcomb(4, __float_as_uint(e.W1));
    h = hcomb(h, __float_as_uint(e.W2));
    h = hcomb(h, __float_as_uint(e.W3));
    h = hcomb(h, __float_as_uint(e.xi));
    return hcomb(h, __float_as_uint(e.eta));
  }
  __device__ static bool same(const EntQ32& a, const EntQ32& b) {
    return __float_as_uint(a.W1) == __float_as_uint(b.W1) && __float_as_uint(a.W2) == __float_as_uint(b.W2) &&
           __float_as_uint(a.W3) == __float_as_uint(b.W3) && __float_as_uint(a.xi) == __float_as_uint(b.xi) &&
           __float_as_uint(a.eta) == __float_as_uint(b.eta);
  }
  __device__ static void setw(EntQ32& e, uint32_t w) { e.w = w; }
  __device__ static uint32_t w(const EntQ32& e) { return e.w; }
};
template <> struct Tuple<EntQ64> {
  __device__ static uint64_t hash(const EntQ64& e) {
    uint64_t h = hcomb(5, (uint64_t)__double_as_longlong(e.W1));
    h = hcomb(h, (uint64_t)__double_as_longlong(e.W2));
    h = hcomb(h, (uint64_t)__double_as_longlong(e.W3));
    h = hcomb(h, (uint64_t)__double_as_longlong(e.xi));
    return hcomb(h, (uint64_t)__double_as_longlong(e.eta));
  }
  __device__ static bool same(const EntQ64& a, const EntQ64& b) {
    return __double_as_longlong(a.W1) == __double_as_longlong(b.W1) &&
           __double_as_longlong(a.W2) == __double_as_longlong(b.W2) &&
           __double_as_longlong(a.W3) == __double_as_longlong(b.W3) &&
           __double_as_longlong(a.xi) == __double_as_longlong(b.xi) &&
           __double_as_longlong(a.eta) == __double_as_longlong(b.eta);
  }
  __device__ static void setw(EntQ64& e, uint32_t w) { e.w = w; }
  __device__ static uint32_t w(const EntQ64& e) { return e.w; }
};

// key = cell << hb | top hb bits of the tuple hash (cells ordered by offset)
template <typename E>
__global__ void k_group_keys(const Cell* __restrict__ cells, uint32_t ncell, const E* __restrict__ ents, uint64_t n,
                             int hb, uint64_t* __restrict__ keys, uint32_t* __restrict__ idx) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t lo = 0, hi = ncell;  // last cell with off <= i
  while (hi - lo > 1) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (cells[mid].off <= i) lo = mid;
    else hi = mid;
  }
  const uint64_t h = Tuple<E>::hash(ents[i]);
  keys[i] = hb >= 64 ? h : (((uint64_t)lo << hb) | (h >> (64 - hb)));
  idx[i] = (uint32_t)i;
}

template <typename E>
__global__ void k_group_heads(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ idx,
                              const E* __restrict__ ents, uint64_t n, uint32_t* __restrict__ head) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  head[i] = (i == 0 || keys[i] != keys[i - 1] || !Tuple<E>::same(ents[idx[i]], ents[idx[i - 1]])) ? 1u : 0u;
}

// one thread per run head: the merged entry carries the run's summed weight
template <typename E>
__global__ void k_group_write(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ idx,
                              const E* __restrict__ ents, uint64_t n, const uint32_t* __restrict__ head,
                              const uint32_t* __restrict__ hscan, int hb, E* __restrict__ out,
                              uint32_t* __restrict__ newlen) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !head[i]) return;
  uint32_t w = 0;
  uint64_t j = i;
  do {
    w += Tuple<E>::w(ents[idx[j]]);
    j++;
  } while (j < n && !head[j]);
  E e = ents[idx[i]];
  Tuple<E>::setw(e, w);
  out[hscan[i]] = e;
  const uint32_t c = hb >= 64 ? 0u : (uint32_t)(keys[i] >> hb);
  atomicAdd(&newlen[c], 1u);
}

__global__ void k_group_cells(Cell* __restrict__ cells, uint32_t ncell, const uint32_t* __restrict__ newlen,
                              const uint32_t* __restrict__ newoff) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncell) {
    cells[c].off = newoff[c];
    cells[c].len = newlen[c];
  }
}
