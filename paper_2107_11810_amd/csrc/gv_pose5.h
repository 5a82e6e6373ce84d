// gv_pose5.h -- the 5-DoF camera-posing family (Sec. 4.2.1: known gravity
// direction, unknown focal length).  Axes (x, y, z, kappa, f): the camera
// position, the tangent of the yaw offset inside one of four sectors, and
// the factor f that turns image coordinates into direction tangents
// (tangent = xi f).  A match (w, xi, eta) is the 3-surface
//   kappa = ((w2 - y) - xi f (w1 - x)) / ((w1 - x) + xi f (w2 - y)),
//   z     = w3 - eta f sqrt((w1 - x)^2 + (w2 - y)^2),
// i.e. the 4-DoF surface with xi and eta scaled by f.  The surfaces are
// quantized once at the root (the pose lattice, with the f bound in its
// derivative bounds) and tested in binary64; a level has up to 32 children
// (every axis split), so pass masks are 32-bit words.
//
// Over a cell, f runs through [Fl, Fh] (Fl > 0):
//   z-half: |eta| f r spans [|eta| Fl r_min, |eta| Fh r_max], so the
//     4-DoF conditions hold with the slope |eta| Fh on the r_max side and
//     |eta| Fl on the r_min side;
//   kappa-half: the cone of directions with kappa in [Llo, Lhi] at tangent
//     t turns with atan t, so over t in [t_lo, t_hi] (t = xi f) the
//     directions form one arc from (1 - Llo t_lo, Llo + t_lo)
//     counter-clockwise to (1 - Lhi t_hi, Lhi + t_hi); every direction of it
//     has a t at which kappa is in range and v1 + t v2 > 0.
// Both conditions are tested separately, as for every family with two
// dependent axes.
#pragma once
#include "gv_kernels.h"
#include "gv_root.h"

// child boxes of an item's cell per bit value (wave-uniform); f in user units
struct Pose5Level {
  double Xlo[2], Xhi[2], Ylo[2], Yhi[2], ZH[2], ZL[2], Llo[2], Lhi[2], Flo[2], Fhi[2];
};

__device__ inline void pose5_level_boxes(const ProbC& P, const LevelC& lv, const Cell& C, int m, Pose5Level& B) {
  const int m1 = m + 1;
  double h[5];
  for (int j = 0; j < 5; j++) h[j] = ldexp(1.0, -min(m1, P.L[j]));
  for (int b = 0; b < 2; b++) {
    const int32_t cx = lv.split[0] ? 2 * C.c[0] + b : C.c[0];
    const int32_t cy = lv.split[1] ? 2 * C.c[1] + b : C.c[1];
    const int32_t cz = lv.split[2] ? 2 * C.c[2] + b : C.c[2];
    const int32_t ck = lv.split[3] ? 2 * C.c[3] + b : C.c[3];
    const int32_t cf = lv.split[4] ? 2 * C.c[4] + b : C.c[4];
    B.Xlo[b] = (double)cx * h[0];
    B.Xhi[b] = (double)(cx + 1) * h[0];
    B.Ylo[b] = (double)cy * h[1];
    B.Yhi[b] = (double)(cy + 1) * h[1];
    const double Zlo = (double)cz * h[2], Zhi = (double)(cz + 1) * h[2];
    B.ZH[b] = Zhi + P.padz;
    B.ZL[b] = Zlo - P.padz;
    const double Klo = 2.0 * ((double)ck * h[3]) - 1.0, Khi = 2.0 * ((double)(ck + 1) * h[3]) - 1.0;
    B.Llo[b] = Klo - P.padk;
    B.Lhi[b] = Khi + P.padk;
    B.Flo[b] = P.flo + P.Ef * ((double)cf * h[4]);
    B.Fhi[b] = P.flo + P.Ef * ((double)(cf + 1) * h[4]);
  }
}

// z-half over the f interval: zp from zpre (the z bit), ah2 = (|eta| Fh)^2,
// al2 = (|eta| Fl)^2 (the f bit)
__device__ inline bool zhalf5(const ZPre<double>& z, double ah2, double al2, double rmin2, double rmax2) {
  const bool lo_ok = (z.Tlo <= 0.0) || (ah2 * rmax2 >= z.Ylo);
  const bool hi_ok = (z.Thi >= 0.0) && (al2 * rmin2 <= z.Yhi);
  return lo_ok && hi_ok;
}

// kappa-half edge directions over the tangents t = xi f, f in [Fl, Fh]
template <typename R>
__device__ inline KEdge<R> kedge5(R xi, R Llo, R Lhi, R Fl, R Fh) {
  const R t1 = xi * Fl, t2 = xi * Fh;
  const R tl = t1 < t2 ? t1 : t2, th = t1 < t2 ? t2 : t1;
  KEdge<R> e;
  e.pl = Llo * tl;
  e.ph = Lhi * th;
  e.elx = (R)1 - e.pl;
  e.ely = Llo + tl;
  e.ehx = (R)1 - e.ph;
  e.ehy = Lhi + th;
  return e;
}

// Pass mask over the children of one cell for one surface.  ALL: every axis
// splits at this level (32 children), so no per-axis checks.  Half-test bit
// index: bx | by << 1 | (z or kappa bit) << 2 | bf << 3.
template <bool ALL>
__device__ inline uint32_t pose5_mask64(const ProbC& P, const LevelC& lv, const Pose5Level& B, int sector, double W1,
                                        double W2, double W3, double xi, double eta) {
  const uint32_t nch = ALL ? 32u : 1u << lv.abits;
  uint32_t zbits = 0, kbits = 0;
  const ZPre<double> zp[2] = {zpre<double>(W3, eta, B.ZH[0], B.ZL[0]), zpre<double>(W3, eta, B.ZH[1], B.ZL[1])};
  const double a = eta >= 0.0 ? eta : -eta;
#pragma unroll
  for (int bf = 0; bf < 2; bf++) {
    if (!ALL && bf && !lv.split[4]) continue;
    const double ah = a * B.Fhi[bf], al = a * B.Flo[bf];
    const double ah2 = ah * ah, al2 = al * al;
    const KEdge<double> ke[2] = {kedge5<double>(xi, B.Llo[0], B.Lhi[0], B.Flo[bf], B.Fhi[bf]),
                                 kedge5<double>(xi, B.Llo[1], B.Lhi[1], B.Flo[bf], B.Fhi[bf])};
#pragma unroll
    for (int xy = 0; xy < 4; xy++) {
      const int bx = xy & 1, by = xy >> 1;
      if (!ALL && ((bx && !lv.split[0]) || (by && !lv.split[1]))) continue;
      const VBox<double> v = pose_vbox<double>(W1, W2, B.Xlo[bx], B.Xhi[bx], B.Ylo[by], B.Yhi[by], sector);
      const double rmin2 = rmin2_of(v), rmax2 = rmax2_of(v);
#pragma unroll
      for (int b = 0; b < 2; b++) {
        if (!ALL && b && !lv.split[2]) continue;
        if (zhalf5(zp[b], ah2, al2, rmin2, rmax2)) zbits |= 1u << (xy | (b << 2) | (bf << 3));
      }
#pragma unroll
      for (int b = 0; b < 2; b++) {
        if (!ALL && b && !lv.split[3]) continue;
        if (khalf64e(v, rmin2, P.Rg2, ke[b])) kbits |= 1u << (xy | (b << 2) | (bf << 3));
      }
    }
  }
  return pose_children<5, ALL>(lv, nch, zbits, kbits);
}

// ---------------------------------------------------------------------------
// binary32 filter.  W, xi, eta and the x, y, z, kappa child bounds are exact
// in binary32 (lattice values, checked per problem on the host); the f
// bounds are rounded to binary32.  Each half's deciding value is computed in
// binary32 with a bound on its distance from the value the binary64 test
// compares: where the value clears the bound the binary64 test decides the
// same way, else the half is undecided and recomputed in binary64 with the
// plain test's own operations.  Rounding: each operation adds a relative
// error of at most u = 2^-24; the host keeps every nonzero intermediate of
// the kappa half and of the z half's first products in the normal range.
//   z-half, low end: X = (|eta| Fh)^2 rmax2 carries 8u (Fh rounded, the
//     product, its square, the two roundings of rmax2, the last product),
//     Tlo^2 one rounding and the difference one more: at most
//     9u X + 2u Tlo^2 to first order.  The bound 16u (X + Tlo^2) covers the
//     higher orders and the binary64 value's own rounding (below 2^-50
//     relative); the absolute 2^-100 covers the last product's underflow
//     (al^2 rmin2 can fall below the normal range).  The high end likewise
//     with Fl and rmin2.
//   kappa-half: t = xi F carries 2u (F rounded, the product), p = L t 3u,
//     e_x = 1 - p at most 3u|p| + u|e_x|, e_y = L + t at most 2u|t| + u|e_y|;
//     a cross product e_x a_y - e_y a_x with exact corners a then errs by at
//     most 3u (|p| + |t| + |e_x| + |e_y|)(|a_x| + |a_y|); the bound takes 8u
//     with |xi| Fh for |t|.  The apex guard is the 4-DoF one.
// ---------------------------------------------------------------------------
#define GV_TINY32 7.888609052210118e-31f  // 2^-100

__device__ inline bool zhalf5_32m(const ZPre<float>& z, float ah2, float al2, float rmin2, float rmax2, bool& und) {
  const float X = ah2 * rmax2;
  const float dl = X - z.Ylo, bl = 16.0f * GV_U32 * (X + z.Ylo) + GV_TINY32;
  const bool lo_t = z.Tlo <= 0.0f;
  const bool lp = lo_t || dl > bl, ln = !lo_t && dl < -bl;
  const float X2 = al2 * rmin2;
  const float dh = z.Yhi - X2, bh = 16.0f * GV_U32 * (X2 + z.Yhi) + GV_TINY32;
  const bool hneg = z.Thi < 0.0f;
  const bool hp = !hneg && dh > bh, hn = hneg || dh < -bh;
  const bool pass = lp && hp;
  und = !(ln || hn) && !pass;
  return pass;
}

// Bf layout: Xlo[2] Xhi[2] Ylo[2] Yhi[2] ZH[2] ZL[2] Llo[2] Lhi[2] Flo[2] Fhi[2]
#define GV_P5_NBF 20
__device__ inline void pose5_boxes32(const Pose5Level& B, float* Bf) {
  for (int b = 0; b < 2; b++) {
    Bf[0 + b] = (float)B.Xlo[b];
    Bf[2 + b] = (float)B.Xhi[b];
    Bf[4 + b] = (float)B.Ylo[b];
    Bf[6 + b] = (float)B.Yhi[b];
    Bf[8 + b] = (float)B.ZH[b];
    Bf[10 + b] = (float)B.ZL[b];
    Bf[12 + b] = (float)B.Llo[b];
    Bf[14 + b] = (float)B.Lhi[b];
    Bf[16 + b] = (float)B.Flo[b];
    Bf[18 + b] = (float)B.Fhi[b];
  }
}

// One child half's bounds in binary64, computed as pose5_level_boxes does
// (bit-equal values): x, y by (bx, by), the z or kappa interval by bq, f by bf.
__device__ inline void pose5_half_bounds(const ProbC& P, const LevelC& lv, const Cell& C, int m, int bx, int by,
                                         int bq, int bf, bool kap, VBox<double>& xy, double& qlo, double& qhi,
                                         double& Fl, double& Fh) {
  const int m1 = m + 1;
  const int32_t cx = lv.split[0] ? 2 * C.c[0] + bx : C.c[0];
  const int32_t cy = lv.split[1] ? 2 * C.c[1] + by : C.c[1];
  const int32_t cf = lv.split[4] ? 2 * C.c[4] + bf : C.c[4];
  const double hx = ldexp(1.0, -min(m1, P.L[0])), hy = ldexp(1.0, -min(m1, P.L[1]));
  const double hf = ldexp(1.0, -min(m1, P.L[4]));
  xy.x0 = (double)cx * hx;
  xy.x1 = (double)(cx + 1) * hx;
  xy.y0 = (double)cy * hy;
  xy.y1 = (double)(cy + 1) * hy;
  Fl = P.flo + P.Ef * ((double)cf * hf);
  Fh = P.flo + P.Ef * ((double)(cf + 1) * hf);
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

// binary32 mask; the undecided halves (bit index xy | b << 2 | bf << 3 of
// zund / kund) are then recomputed in binary64 one at a time, from the
// entry's binary64 root values and the child's bounds, with the plain test's
// operations
template <bool ALL, typename EQ>
__device__ inline uint32_t pose5_mask32(const ProbC& P, const LevelC& lv, const Cell& C, int m, const float* Bf,
                                        int sector, const EQ& e, const double* __restrict__ m64, uint64_t n_root,
                                        uint32_t& nrecheck) {
  const uint32_t nch = ALL ? 32u : 1u << lv.abits;
  uint32_t zbits = 0, kbits = 0, zund = 0, kund = 0;
  const ZPre<float> zp[2] = {zpre<float>(e.W3, e.eta, Bf[8], Bf[10]), zpre<float>(e.W3, e.eta, Bf[9], Bf[11])};
  const float a = fabsf(e.eta), axi = fabsf(e.xi);
  // the two halves of the f interval in turn (not unrolled: both halves'
  // terms live at once took 156 registers, 142 this way); bounds picked by
  // selects
#pragma unroll 1
  for (int bf = 0; bf < 2; bf++) {
    if (!ALL && bf && !lv.split[4]) continue;
    const float Fl = bf ? Bf[17] : Bf[16], Fh = bf ? Bf[19] : Bf[18];
    const float ah = a * Fh, al = a * Fl;
    const float ah2 = ah * ah, al2 = al * al;
    const KEdge<float> ke[2] = {kedge5<float>(e.xi, Bf[12], Bf[14], Fl, Fh), kedge5<float>(e.xi, Bf[13], Bf[15], Fl, Fh)};
    const float tm = axi * Fh;
    float kSl[2], kSh[2];
#pragma unroll
    for (int b = 0; b < 2; b++) {
      kSl[b] = 8.0f * GV_U32 * (fabsf(ke[b].pl) + tm + fabsf(ke[b].elx) + fabsf(ke[b].ely));
      kSh[b] = 8.0f * GV_U32 * (fabsf(ke[b].ph) + tm + fabsf(ke[b].ehx) + fabsf(ke[b].ehy));
    }
#pragma unroll
    for (int xy = 0; xy < 4; xy++) {
      const int bx = xy & 1, by = xy >> 1;
      if (!ALL && ((bx && !lv.split[0]) || (by && !lv.split[1]))) continue;
      const VBox<float> v = pose_vbox<float>(e.W1, e.W2, Bf[0 + bx], Bf[2 + bx], Bf[4 + by], Bf[6 + by], sector);
      const float rmin2 = rmin2_of(v), rmax2 = rmax2_of(v);
#pragma unroll
      for (int b = 0; b < 2; b++) {
        if (!ALL && b && !lv.split[2]) continue;
        bool u;
        const uint32_t bit = 1u << (xy | (b << 2) | (bf << 3));
        if (zhalf5_32m(zp[b], ah2, al2, rmin2, rmax2, u)) zbits |= bit;
        if (u) zund |= bit;
      }
#pragma unroll
      for (int b = 0; b < 2; b++) {
        if (!ALL && b && !lv.split[3]) continue;
        bool u;
        const uint32_t bit = 1u << (xy | (b << 2) | (bf << 3));
        if (khalf32m(v, rmin2, P.Rg2f, ke[b], kSl[b], kSh[b], u)) kbits |= bit;
        if (u) kund |= bit;
      }
    }
  }
  if (zund | kund) {
    const uint64_t r = e.ridx;
    const double W1 = m64[r], W2 = m64[n_root + r], W3 = m64[2 * n_root + r], xi = m64[3 * n_root + r],
                 eta = m64[4 * n_root + r];
    uint32_t und = zund | (kund << 16);
#pragma unroll 1
    while (und) {
      const uint32_t j = (uint32_t)__builtin_ctz(und);
      und &= und - 1u;
      const bool kap = j >= 16;
      const uint32_t i = j & 15u;
      const int bx = i & 1, by = (i >> 1) & 1, bq = (i >> 2) & 1, bf = (i >> 3) & 1;
      VBox<double> box;
      double qlo, qhi, Fl, Fh;
      pose5_half_bounds(P, lv, C, m, bx, by, bq, bf, kap, box, qlo, qhi, Fl, Fh);
      const VBox<double> vd = pose_vbox<double>(W1, W2, box.x0, box.x1, box.y0, box.y1, sector);
      const double rmin2d = rmin2_of(vd);
      bool pass;
      if (kap) {
        pass = khalf64e(vd, rmin2d, P.Rg2, kedge5<double>(xi, qlo, qhi, Fl, Fh));
      } else {
        const double rmax2d = rmax2_of(vd);
        const ZPre<double> zq = zpre<double>(W3, eta, qhi, qlo);
        const double aa = eta >= 0.0 ? eta : -eta;
        const double ah = aa * Fh, al = aa * Fl;
        pass = zhalf5(zq, ah * ah, al * al, rmin2d, rmax2d);
      }
      const uint32_t bm = 1u << i;
      if (kap)
        kbits = pass ? (kbits | bm) : (kbits & ~bm);
      else
        zbits = pass ? (zbits | bm) : (zbits & ~bm);
      nrecheck++;
    }
  }
  return pose_children<5, ALL>(lv, nch, zbits, kbits);
}

// mask of one entry: the binary64 test on binary64 lists, else the filter
template <bool ALL, typename E>
__device__ inline uint32_t pose5_mask_of(const ProbC& P, const LevelC& lv, const Cell& C, int m, const Pose5Level& B,
                                         const float* Bf, const E& e, const double* __restrict__ m64,
                                         uint64_t n_root, uint32_t& nre) {
  if constexpr (std::is_same<E, EntQ64>::value)
    return pose5_mask64<ALL>(P, lv, B, (int)C.sector, e.W1, e.W2, e.W3, e.xi, e.eta);
  else
    return pose5_mask32<ALL>(P, lv, C, m, Bf, (int)C.sector, e, m64, n_root, nre);
}

// Incidence test and per-child counts of a batch (one wave per item), with
// a 32-bit pass mask stored per entry for the compaction.  UNIT: every
// multiplicity is 1: each lane counts its own passes, four children to a
// word (one byte each: a lane tests at most GV_ITEM/64 = 16 entries of an
// item), the wave sums them once per item in 16-bit halves (at most 1024
// per child).  Thirty-two scalar ballot accumulators, beside the cell's
// binary64 child boxes, overflowed the scalar registers.
static_assert(GV_ITEM / 64 <= 255 && 64 * (GV_ITEM / 64) <= 65535, "per-lane byte counters, 16-bit wave sums");
// E: EntQ64 (binary64 lists) or EntQ32 / EntQ24 (binary32 filter; m64 holds
// the binary64 root values for the recheck, n_root their column stride).
// binary32 lists at 4 waves per SIMD (128 registers, 36 B per lane spilled):
// 1.94-1.96 against 2.02-2.05 ms of count kernel per pose5dof_20k solve at
// the 3 waves of its unconstrained 142 registers; binary64 lists keep theirs
// (capping them spilled 224-448 B per lane and ran slower)
template <typename E> constexpr int pose5_min_blocks() { return std::is_same<E, EntQ64>::value ? 1 : 4; }
template <typename E, bool UNIT, bool ALL>
__global__ void __launch_bounds__(256, pose5_min_blocks<E>()) k_count_pose5(const ProbC* __restrict__ Ptab, int m, LevelC lv,
                                                     const Cell* __restrict__ cells, const Item* __restrict__ items,
                                                     const uint32_t* __restrict__ nitems_p, const E* __restrict__ ents,
                                                     const double* __restrict__ m64, uint64_t n_root,
                                                     uint32_t* __restrict__ masks, uint32_t* __restrict__ ccnt,
                                                     uint32_t* __restrict__ cnent,
                                                     unsigned long long* __restrict__ rechecks,
                                                     uint32_t* __restrict__ itemcnt, uint32_t istride) {
  constexpr bool F64 = std::is_same<E, EntQ64>::value;
  const uint32_t nch = ALL ? 32u : 1u << lv.abits;
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
    Pose5Level B;
    pose5_level_boxes(P, lv, C, m, B);
    float Bf[F64 ? 1 : GV_P5_NBF];
    if constexpr (!F64) pose5_boxes32(B, Bf);
    if constexpr (UNIT) {
      uint32_t pk[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // byte b of pk[g]: passes of child 4g + b
      for (uint32_t k0 = 0; k0 < cnt; k0 += 64) {
        const uint32_t k = k0 + lane;
        const uint64_t ei = I.off + k;
        uint32_t mask = 0;
        if (k < cnt) {
          const E e = ents[ei];
          mask = pose5_mask_of<ALL>(P, lv, C, m, B, Bf, e, m64, n_root, nre);
          masks[ei] = mask;
        }
        // spread each nibble of the mask to the low bits of four bytes
#pragma unroll
        for (int g = 0; g < 8; g++) pk[g] += (((mask >> (4 * g)) & 0xFu) * 0x204081u) & 0x01010101u;
      }
#pragma unroll
      for (int g = 0; g < 8; g++) {
        if ((uint32_t)(4 * g) >= nch) break;
        const uint32_t ev = wave_sum_u32(pk[g] & 0x00FF00FFu);         // children 4g, 4g + 2
        const uint32_t od = wave_sum_u32((pk[g] >> 8) & 0x00FF00FFu);  // children 4g + 1, 4g + 3
        const uint32_t n4[4] = {ev & 0xFFFFu, od & 0xFFFFu, ev >> 16, od >> 16};
#pragma unroll
        for (int b = 0; b < 4; b++) {
          const uint32_t ch = 4 * g + b, n = n4[b];
          if (lane == 0 && ch < nch && n) {
            atomicAdd(&ccnt[I.cell * nch + ch], n);
            atomicAdd(&cnent[I.cell * nch + ch], n);
            if (istride) itemcnt[(uint64_t)ch * istride + it] = n;
          }
        }
      }
    } else {
      uint32_t aw[32], an[32];
#pragma unroll
      for (int ch = 0; ch < 32; ch++) { aw[ch] = 0; an[ch] = 0; }
      for (uint32_t k0 = 0; k0 < cnt; k0 += 64) {
        const uint32_t k = k0 + lane;
        const uint64_t ei = I.off + k;
        uint32_t mask = 0, w = 0;
        if (k < cnt) {
          const E e = ents[ei];
          w = pose_w(e);
          mask = pose5_mask_of<ALL>(P, lv, C, m, B, Bf, e, m64, n_root, nre);
          masks[ei] = mask;
        }
#pragma unroll
        for (int ch = 0; ch < 32; ch++) {
          const bool p = (mask >> ch) & 1u;
          aw[ch] += p ? w : 0u;
          an[ch] += p ? 1u : 0u;
        }
      }
#pragma unroll
      for (int ch = 0; ch < 32; ch++) {
        if ((uint32_t)ch < nch) {
          const uint32_t n = wave_sum_u32(an[ch]);
          const uint32_t w = wave_sum_u32(aw[ch]);
          if (lane == 0 && n) {
            atomicAdd(&ccnt[I.cell * nch + ch], w);
            atomicAdd(&cnent[I.cell * nch + ch], n);
            if (istride) itemcnt[(uint64_t)ch * istride + it] = n;
          }
        }
      }
    }
  }
  if constexpr (!F64) {
    const uint32_t tot = wave_sum_u32(nre);
    if (lane == 0 && tot) atomicAdd(rechecks, (unsigned long long)tot);
  }
}

// Replay of every original match along its problem's chosen path: the
// root-quantized surface passes every cell of the path (member tracking,
// Sec. 3.2.1; the surfaces do not change below the root).
__global__ void k_replay_pose5(const ProbC* __restrict__ Ptab, const double* __restrict__ m64, uint64_t Ntot,
                               const uint64_t* __restrict__ ooff, uint32_t nprob, const PathC* __restrict__ paths,
                               uint32_t* __restrict__ flag) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Ntot; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t p = prob_of(ooff, nprob, i);
    const ProbC& P = Ptab[p];
    const PathC& path = paths[p];
    const double W1 = m64[i], W2 = m64[Ntot + i], W3 = m64[2 * Ntot + i], xi = m64[3 * Ntot + i],
                 eta = m64[4 * Ntot + i];
    const double a = eta >= 0.0 ? eta : -eta;
    int32_t cc[5] = {0, 0, 0, 0, 0};
    uint32_t ok = 1;
    for (int m = 0; m < P.Lstar && ok; m++) {
      const LevelC& lv = P.lev[m];
      const uint32_t cb = lv.cbits[path.digit[m]];
      int32_t ch[5];
      for (int j = 0; j < 5; j++) ch[j] = lv.split[j] ? 2 * cc[j] + (int32_t)((cb >> j) & 1u) : cc[j];
      const int m1 = m + 1;
      double h[5];
      for (int j = 0; j < 5; j++) h[j] = ldexp(1.0, -min(m1, P.L[j]));
      const double Xlo = (double)ch[0] * h[0], Xhi = (double)(ch[0] + 1) * h[0];
      const double Ylo = (double)ch[1] * h[1], Yhi = (double)(ch[1] + 1) * h[1];
      const double Zlo = (double)ch[2] * h[2], Zhi = (double)(ch[2] + 1) * h[2];
      const double Klo = 2.0 * ((double)ch[3] * h[3]) - 1.0, Khi = 2.0 * ((double)(ch[3] + 1) * h[3]) - 1.0;
      const double Fl = P.flo + P.Ef * ((double)ch[4] * h[4]), Fh = P.flo + P.Ef * ((double)(ch[4] + 1) * h[4]);
      const VBox<double> v = pose_vbox<double>(W1, W2, Xlo, Xhi, Ylo, Yhi, path.sector);
      const double rmin2 = rmin2_of(v), rmax2 = rmax2_of(v);
      const double ah = a * Fh, al = a * Fl;
      ok = zhalf5(zpre<double>(W3, eta, Zhi + P.padz, Zlo - P.padz), ah * ah, al * al, rmin2, rmax2) &&
           khalf64e(v, rmin2, P.Rg2, kedge5<double>(xi, Klo - P.padk, Khi + P.padk, Fl, Fh));
      for (int j = 0; j < 5; j++) cc[j] = ch[j];
    }
    flag[i] = ok;
  }
}

// Incidence test only (gv_incidence): every root surface against the
// children of cell C at level m, exactly as in the count pass.
template <typename E>
__global__ void k_incidence_pose5(const ProbC* __restrict__ Pp, const E* __restrict__ root, int64_t n,
                                  const double* __restrict__ m64, uint64_t n_root, Cell C, int m,
                                  uint32_t* __restrict__ masks, unsigned long long* __restrict__ rechecks) {
  const ProbC& P = *Pp;
  const LevelC& lv = P.lev[m];
  Pose5Level B;
  pose5_level_boxes(P, lv, C, m, B);
  float Bf[GV_P5_NBF];
  pose5_boxes32(B, Bf);
  uint32_t nre = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const E e = root[i];
    if constexpr (std::is_same<E, EntQ64>::value)
      masks[i] = pose5_mask64<false>(P, lv, B, (int)C.sector, e.W1, e.W2, e.W3, e.xi, e.eta);
    else
      masks[i] = pose5_mask32<false>(P, lv, C, m, Bf, (int)C.sector, e, m64, n_root, nre);
  }
  if (nre) atomicAdd(rechecks, (unsigned long long)nre);
}
