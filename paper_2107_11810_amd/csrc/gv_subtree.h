// gv_subtree.h -- device-side search of small subtrees (pose families).
//
// A persistent kernel over a work queue of (problem, cell) items: every cell
// of a batch whose list is at most GV_SUB_T entries is taken by one
// workgroup, which runs the rest of Alg. 2 below that cell on its own:
// incidence test and counts of the cell's children, pruning against its
// problem's best key (shared by every workgroup through the same u64
// atomic maximum), and depth-first descent into the kept children, highest
// count first, with each child's list compacted into the workgroup's own
// frame buffer.  The surfaces of this family do not change below the root,
// so a child's list is a copy of the parent's survivors.  Cells with longer
// lists are written back for the host-driven path.  The result is that of
// the host-driven search: a leaf's key is unique, so neither the order nor
// the pruning bound changes the maximum.
#pragma once
#include "gv_kernels.h"
#include "gv_pose5.h"

#define GV_SUB_T 2048   // longest list a workgroup takes
#define GV_SUB_WG 256

// a pose family's cell constants and masks: 16 children and 16-bit masks
// (4-DoF) or 32 and 32-bit (5-DoF)
template <int FAM> struct SubFam;
template <> struct SubFam<FAM_POSE4DOF> {
  static constexpr int NCH = 16, NBF = 16;
  using M = uint16_t;
  using Boxes = PoseLevel;
  __device__ static void boxes(const ProbC& P, const LevelC& lv, const Cell& C, int m, Boxes& B, float* Bf) {
    pose_level_boxes(P, lv, C, m, B);
    for (int b = 0; b < 2; b++) {
      Bf[0 + b] = (float)B.Xlo[b]; Bf[2 + b] = (float)B.Xhi[b];
      Bf[4 + b] = (float)B.Ylo[b]; Bf[6 + b] = (float)B.Yhi[b];
      Bf[8 + b] = (float)B.ZH[b];  Bf[10 + b] = (float)B.ZL[b];
      Bf[12 + b] = (float)B.Llo[b]; Bf[14 + b] = (float)B.Lhi[b];
    }
  }
  template <typename E>
  __device__ static uint32_t mask(const ProbC& P, const LevelC& lv, const Cell& C, int m, const Boxes& B,
                                  const float* Bf, const E& e, const double* __restrict__ m64, uint64_t n_root,
                                  uint32_t& nre) {
    if constexpr (sizeof(E) == sizeof(EntQ64)) {
      return lv.abits == 4 ? pose_mask64<true>(P, lv, B, (int)C.sector, e.W1, e.W2, e.W3, e.xi, e.eta)
                           : pose_mask64<false>(P, lv, B, (int)C.sector, e.W1, e.W2, e.W3, e.xi, e.eta);
    } else {
      return lv.abits == 4 ? pose_mask32<true>(P, lv, C, m, Bf, (int)C.sector, e, m64, n_root, nre)
                           : pose_mask32<false>(P, lv, C, m, Bf, (int)C.sector, e, m64, n_root, nre);
    }
  }
};
template <> struct SubFam<FAM_POSE5DOF> {
  static constexpr int NCH = 32, NBF = GV_P5_NBF;
  using M = uint32_t;
  using Boxes = Pose5Level;
  __device__ static void boxes(const ProbC& P, const LevelC& lv, const Cell& C, int m, Boxes& B, float* Bf) {
    pose5_level_boxes(P, lv, C, m, B);
    pose5_boxes32(B, Bf);
  }
  template <typename E>
  __device__ static uint32_t mask(const ProbC& P, const LevelC& lv, const Cell& C, int m, const Boxes& B,
                                  const float* Bf, const E& e, const double* __restrict__ m64, uint64_t n_root,
                                  uint32_t& nre) {
    if (lv.abits == 5) return pose5_mask_of<true>(P, lv, C, m, B, Bf, e, m64, n_root, nre);
    return pose5_mask_of<false>(P, lv, C, m, B, Bf, e, m64, n_root, nre);
  }
};

template <int NCH>
struct SubFrame {
  Cell c;
  int32_t level, nkept, next, _;
  uint32_t cnt[NCH], nent[NCH];
  uint8_t order[NCH];
};

// fbuf: per workgroup (nframes - 1) * GV_SUB_T entries (the lists of frames
// 1..); mbuf: per workgroup nframes * GV_SUB_T pass masks.  nover[0] counts
// the cells written back to over[], nover[1] their entries.
template <int FAM, typename E>
__global__ void __launch_bounds__(GV_SUB_WG) k_subtree_pose(
    const ProbC* __restrict__ Ptab, int m0, const Cell* __restrict__ cells, uint32_t ncell,
    const E* __restrict__ ents, const double* __restrict__ m64, uint64_t n_root, unsigned long long* best,
    unsigned long long* __restrict__ rechecks, unsigned long long* __restrict__ tests,
    uint32_t* __restrict__ next_cell, Cell* __restrict__ over, uint32_t* __restrict__ nover,
    E* __restrict__ fbuf, typename SubFam<FAM>::M* __restrict__ mbuf, int nframes) {
  using F = SubFam<FAM>;
  using M = typename F::M;
  constexpr int NCH = F::NCH;
  __shared__ SubFrame<NCH> fr[GV_MAXL + 1];
  __shared__ uint32_t wcnt[GV_SUB_WG / 64][NCH], wnent[GV_SUB_WG / 64][NCH];
  __shared__ uint32_t wtot[GV_SUB_WG / 64];
  __shared__ uint32_t s_item;
  __shared__ int s_skip;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  E* const myf = fbuf + (uint64_t)blockIdx.x * (uint64_t)(nframes - 1) * GV_SUB_T;
  M* const mym = mbuf + (uint64_t)blockIdx.x * (uint64_t)nframes * GV_SUB_T;
  uint64_t ntests = 0;
  uint32_t nre = 0;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(next_cell, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= ncell) break;
    const Cell C0 = cells[item];
    if (C0.len > GV_SUB_T) {  // too long for one workgroup: back to the host-driven path
      if (tid == 0) {
        over[atomicAdd(nover, 1u)] = C0;
        atomicAdd(nover + 1, C0.len);
      }
      continue;
    }
    if (tid == 0) {
      fr[0].c = C0;
      fr[0].level = m0;
    }
    int d = 0;
    bool expand = true;
    while (d >= 0) {
      if (expand) {
        // ---- incidence test and counts of frame d's children ----
        __syncthreads();
        const Cell C = fr[d].c;
        const int l = fr[d].level;
        const ProbC& P = Ptab[C.prob];
        const LevelC& lv = P.lev[l];
        const uint32_t nch = 1u << lv.abits;
        const uint32_t len = C.len;
        const E* list = d == 0 ? ents + C.off : myf + (uint64_t)(d - 1) * GV_SUB_T;
        M* masks = mym + (uint64_t)d * GV_SUB_T;
        if (tid < NCH) {
          for (uint32_t w = 0; w < GV_SUB_WG / 64; w++) {
            wcnt[w][tid] = 0;
            wnent[w][tid] = 0;
          }
        }
        typename F::Boxes B;
        float Bf[F::NBF];
        F::boxes(P, lv, C, l, B, Bf);
        __syncthreads();
        for (uint32_t base = 0; base < len; base += GV_SUB_WG) {
          const uint32_t j = base + tid;
          uint32_t mask = 0, w = 0;
          if (j < len) {
            const E e = list[j];
            w = pose_w(e);
            mask = F::template mask<E>(P, lv, C, l, B, Bf, e, m64, n_root, nre);
            masks[j] = (M)mask;
          }
#pragma unroll
          for (int ch = 0; ch < NCH; ch++) {
            const bool p = (mask >> ch) & 1u;
            const uint32_t n = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(p));
            uint32_t s = n;  // unit entries: the count is the number of survivors
            if constexpr (!std::is_same<E, EntQ24>::value) s = wave_sum_u32(p ? w : 0u);
            if (lane == 0) {
              wnent[wv][ch] += n;
              wcnt[wv][ch] += s;
            }
          }
        }
        __syncthreads();
        if (tid == 0) {
          ntests += (uint64_t)len * nch;
          const bool leaf = l + 1 == P.Lstar;
          const unsigned long long bst = *(volatile unsigned long long*)&best[C.prob];
          uint64_t kmax = 0;
          int nk = 0;
          for (uint32_t ch = 0; ch < nch; ch++) {
            uint32_t c = 0, ne = 0;
            for (uint32_t w = 0; w < GV_SUB_WG / 64; w++) {
              c += wcnt[w][ch];
              ne += wnent[w][ch];
            }
            fr[d].cnt[ch] = c;
            fr[d].nent[ch] = ne;
            const uint64_t idx = ((C.prefix << lv.abits) | ch) << lv.rem_next;
            const uint64_t key = ((uint64_t)c << P.B) | (P.idxmask - idx);
            if (key <= bst) continue;
            if (leaf) {
              kmax = key > kmax ? key : kmax;
            } else {
              // kept children, highest count first (then lowest digit)
              int pos = nk++;
              while (pos > 0 && fr[d].cnt[fr[d].order[pos - 1]] < c) {
                fr[d].order[pos] = fr[d].order[pos - 1];
                pos--;
              }
              fr[d].order[pos] = (uint8_t)ch;
            }
          }
          if (leaf && kmax) atomicMax(&best[C.prob], (unsigned long long)kmax);
          fr[d].nkept = nk;
          fr[d].next = 0;
        }
        expand = false;
      }
      __syncthreads();
      // ---- next kept child of frame d, or back up ----
      if (tid == 0) {
        s_skip = 1;
        while (fr[d].next < fr[d].nkept) {
          const Cell C = fr[d].c;
          const ProbC& P = Ptab[C.prob];
          const LevelC& lv = P.lev[fr[d].level];
          const uint32_t ch = fr[d].order[fr[d].next++];
          const uint64_t idx = ((C.prefix << lv.abits) | ch) << lv.rem_next;
          const uint64_t key = ((uint64_t)fr[d].cnt[ch] << P.B) | (P.idxmask - idx);
          if (key <= *(volatile unsigned long long*)&best[C.prob]) continue;  // the bound moved
          Cell K = C;
          const uint32_t cb = lv.cbits[ch];
          for (int a = 0; a < GV_MAXD; a++) K.c[a] = lv.split[a] ? 2 * C.c[a] + (int32_t)((cb >> a) & 1u) : C.c[a];
          K.prefix = (C.prefix << lv.abits) | ch;
          K.off = 0;
          K.len = fr[d].nent[ch];
          fr[d + 1].c = K;
          fr[d + 1].level = fr[d].level + 1;
          s_skip = (int)ch;  // a child to descend into
          s_skip = -1 - s_skip;
          break;
        }
      }
      __syncthreads();
      const int sk = s_skip;
      if (sk >= 0) {  // no child left: back up
        d--;
        continue;
      }
      // ---- compaction of the child's survivors into frame d + 1 ----
      const uint32_t ch = (uint32_t)(-1 - sk);
      const uint32_t len = fr[d].c.len;
      const E* src = d == 0 ? ents + fr[d].c.off : myf + (uint64_t)(d - 1) * GV_SUB_T;
      const M* masks = mym + (uint64_t)d * GV_SUB_T;
      E* dst = myf + (uint64_t)d * GV_SUB_T;
      uint32_t run = 0;
      for (uint32_t base = 0; base < len; base += GV_SUB_WG) {
        const uint32_t j = base + tid;
        const bool p = j < len && ((masks[j] >> ch) & 1u);
        const uint64_t bal = __builtin_amdgcn_ballot_w64(p);
        if (lane == 0) wtot[wv] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t off = run, tot = 0;
        for (uint32_t w = 0; w < GV_SUB_WG / 64; w++) {
          off += w < wv ? wtot[w] : 0u;
          tot += wtot[w];
        }
        if (p) dst[off + mbcnt64(bal)] = src[j];
        run += tot;
        __syncthreads();
      }
      d++;
      expand = true;
    }
  }
  if (tid == 0 && ntests) atomicAdd(tests, (unsigned long long)ntests);
  const uint32_t r = wave_sum_u32(nre);
  if (lane == 0 && r) atomicAdd(rechecks, (unsigned long long)r);
}
