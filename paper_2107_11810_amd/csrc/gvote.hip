// gvote.hip -- MI355X general-voting library: C ABI and host runtime.
// See include/gvote.h for the interface.
//
// Pipeline (Alg. 2 of Aiger et al., ICCV 2021), for one problem or an epoch
// of compatible problems whose cells share every batch:
//   front end (Eq. 1-3, the posing surface) -> root canonization + grouping
//   -> greedy dive (achieved leaf keys seed the pruning bounds)
//   -> depth-first over batches of same-level cells: incidence test + counts,
//      prune against the best key, count-ordered chunks, compaction +
//      canonization into the children's lists, best-key atomic max at leaves
//   -> inliers by per-surface replay along each problem's chosen path.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gvote.h"
#include "gv_device.h"
#include "gv_kernels.h"
#include "gv_root.h"
#include "gv_exact.h"
#include "gv_subtree.h"
#include "gv_pose5.h"
#include "gv_refine.h"

// Caching device allocator owned by a context.  All library work on a
// context is ordered on its stream, so a block released after its last use
// was enqueued can be handed to any later allocation on that stream without a
// synchronization.  Sizes are rounded to 8 classes per power of two.
struct DevCache {
  std::multimap<size_t, void*> free_blocks;
  std::map<void*, size_t> live;
  uint64_t cached = 0, in_use = 0, peak = 0;
  // Arena mode: every block is carved from one fixed device region
  // [arena, arena + arena_size) (first fit, neighbours coalesce on release);
  // nothing is ever allocated from or returned to the runtime.
  char* arena = nullptr;
  size_t arena_size = 0;
  std::map<size_t, size_t> afree;  // offset -> length of the free runs
  void arena_reset(char* base, size_t size) {
    arena = base;
    arena_size = size;
    afree.clear();
    afree[0] = size;
    live.clear();
    in_use = peak = 0;
  }
  void* arena_get(size_t bytes, std::string& err) {
    const size_t r = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    for (auto it = afree.begin(); it != afree.end(); ++it) {
      if (it->second < r) continue;
      const size_t off = it->first, len = it->second;
      afree.erase(it);
      if (len > r) afree[off + r] = len - r;
      void* p = arena + off;
      live[p] = r;
      in_use += r;
      peak = std::max(peak, in_use);
      return p;
    }
    err = "the search outgrew the library's scratch region";
    return nullptr;
  }
  void arena_put(void* p) {
    auto it = live.find(p);
    if (it == live.end()) return;
    size_t off = (size_t)((char*)p - arena), len = it->second;
    in_use -= len;
    live.erase(it);
    auto nx = afree.lower_bound(off);
    if (nx != afree.end() && off + len == nx->first) {
      len += nx->second;
      nx = afree.erase(nx);
    }
    if (nx != afree.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += len;
        return;
      }
    }
    afree[off] = len;
  }

  static size_t round(size_t b) {
    if (b <= 4096) return 4096;
    int e = 63 - __builtin_clzll((unsigned long long)b);  // 2^e <= b < 2^(e+1)
    size_t step = (size_t)1 << (e >= 3 ? e - 3 : 0);
    return (b + step - 1) / step * step;
  }
  // a cached block serves a request up to 1.25x its size (1.5x from 64 MB
  // on, where sizes vary most and each new block costs the most)
  static size_t slack(size_t r) { return r >= (64ull << 20) ? r / 2 : r / 4; }
  void* take(std::multimap<size_t, void*>::iterator it) {
    void* p = it->second;
    live[p] = it->first;
    in_use += it->first;
    cached -= it->first;
    free_blocks.erase(it);
    peak = std::max(peak, in_use);
    return p;
  }
  void* get(size_t bytes, hipStream_t st, std::string& err) {
    if (arena) return arena_get(bytes, err);
    const size_t r = round(bytes);
    auto it = free_blocks.lower_bound(r);
    if (it != free_blocks.end() && it->first <= r + slack(r)) return take(it);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      // out of device memory: any cached block large enough, else free them all
      if (it != free_blocks.end()) return take(it);
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
  // free the largest cached blocks until at most target bytes stay cached
  void release_to(uint64_t target, hipStream_t st) {
    if (arena || cached <= target) return;
    (void)hipStreamSynchronize(st);
    while (cached > target && !free_blocks.empty()) {
      auto it = std::prev(free_blocks.end());
      (void)hipFree(it->second);
      cached -= it->first;
      free_blocks.erase(it);
    }
  }
  void put(void* p) {
    if (arena) {
      arena_put(p);
      return;
    }
    auto it = live.find(p);
    if (it == live.end()) return;
    free_blocks.emplace(it->second, p);
    cached += it->second;
    in_use -= it->second;
    live.erase(it);
  }
  void trim(hipStream_t st) {
    if (arena) return;
    (void)hipStreamSynchronize(st);
    for (auto& kv : free_blocks) (void)hipFree(kv.second);
    free_blocks.clear();
    cached = 0;
  }
};

namespace gvi {
struct ProbRec;
struct Lane;
}

// Scratch region of the allocation-free solve (gv_solve_noalloc): device
// memory of a fixed size that the library holds on every GPU it runs on
// until the process ends.  In host code this name is not a device address;
// the address comes from hipGetSymbolAddress, once per device, when a context
// is created there, and only that address is used afterwards.
constexpr size_t kScratchBytes = 256ull << 20;
constexpr int64_t kNoAllocMaxN = 1ll << 19;  // observations per allocation-free solve
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per device: the scratch address, and the arena over it (calls on one
// device take the slot's lock, so they run one after the other).
struct ScratchSlot {
  std::mutex mu;
  bool init = false;
  void* ptr = nullptr;
  std::string err;
  DevCache arena;
};
constexpr int kMaxDevices = 64;
static ScratchSlot g_scratch[kMaxDevices];

// Candidate grids of the item-looping kernels, in blocks of four waves per
// CU.  A slot tries them in turn on its large launches and keeps the one with
// the lowest median event time per byte (the entry bytes the launch reads or
// writes, so levels with different entry sizes compare) once each has
// kTuneSamples samples.  The median of 8: with the mean over 4, the levels
// that happened to fall to a candidate decided its figure (compaction at 4
// blocks per CU read 0.32 or 0.53 ps/byte in two runs of the same solve).
constexpr int kTuneCand[] = {2, 4, 8, 16, 32};
constexpr int kNCand = 5;
constexpr int kTuneSamples = 8;
constexpr uint64_t kTuneMinBytes = 256ull << 20;  // smaller launches use the default shape
constexpr int kLastFam = GV_POSE5DOF;               // family codes run 1..kLastFam
constexpr int kGridDefault = 8;
// Entries per work item of a 5-DoF batch: GV_ITEM, halved (down to 256)
// while the batch would give fewer than 16 items per compute unit, so that
// a small batch spreads over the chip instead of leaving a few waves 16
// entries of 32 children each per lane (pose5dof_20k: count kernel 1.67-1.71
// against 1.94-1.96 ms per solve, compaction 0.48 against 0.60).  The other
// families keep GV_ITEM: smaller items gave nothing there or lost a little
// (pose4dof_1m 61-62 against 60.6 ms, the 256-problem set 1.00-1.21 s
// against 1.00 s for items down to 64 or 256 entries, 16 or 64 per CU).
constexpr uint32_t kItemLogMin5 = 8;
constexpr uint64_t kItemsPerCu5 = 16;
// Surface tile of the count pass: log2 of the entries per work item (256,
// 512 or 1024), tuned like the grid on batches of at least kTuneMinBytes
// once the count kernel's grid is chosen, so that every sample runs at that
// grid.  A sample is the count kernel's event time per entry byte of a
// batch whose items were cut at the candidate size.
constexpr int kTileCand[] = {8, 9, 10};
constexpr int kNTile = 3;
constexpr int kTuneKinds = 3;  // 0 count grid, 1 compaction grid, 2 count tile
inline int tune_ncand(int kind) { return kind == 2 ? kNTile : kNCand; }
inline int tune_value(int kind, int k) { return kind == 2 ? kTileCand[k] : kTuneCand[k]; }
struct gvi_tune_slot {
  int chosen = 0;  // blocks per CU (kinds 0, 1) or log2 entries per item (kind 2) once chosen
  int next = 0;    // next candidate to try
  double r[kNCand][kTuneSamples] = {};  // per-sample event time per byte
  int n[kNCand] = {};
};

struct gv_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t budget = 0;
  std::mutex mu;           // serializes all device work of the context
  std::string err;         // error text of the running device operation
  std::mutex emu;
  std::string last_err;    // what gv_last_error reports
  int n_cu = 256;
  DevCache cache;
  uint64_t* hpin = nullptr;      // host-coherent pinned words the kernels write totals to
  uint64_t* hpin_dev = nullptr;  // (device address of the same)
  bool kernel_timing = false;
  std::vector<hipEvent_t> ev_pool;
  // continuous batching
  std::mutex qmu;
  std::condition_variable cv_work, cv_done;
  std::deque<gvi::ProbRec*> queue;
  std::map<uint64_t, gvi::ProbRec*> tickets;
  uint64_t next_ticket = 1;
  uint64_t inflight = 0;   // estimated bytes of admitted problems
  std::vector<gvi::Lane*> lanes;  // serving lanes, started by the first gv_submit
  // one host thread, stream and allocator each; three lanes plus the
  // context's own stream fill the four hardware queues a process gets
  // (measured on 256 pose problems: 3 lanes 1.10 s, 4 lanes 1.24 s)
  int nlanes = 3;
  int running = 0;         // epochs running in the lanes
  bool stop = false;
  size_t max_batch = 1024; // problems per epoch
  // observations an epoch may take beyond its first problem.  Sharing batches
  // between problems measured slower than stepping one-problem epochs
  // round-robin (each problem needs its own first-descent beam), so by
  // default every epoch holds one problem.
  uint64_t batch_n = 0;
  // packed 8-byte list entries where the lattice bounds allow (GV_PACK=0 off)
  bool pack = true;
  // launch-shape autotuner: per family (index 1..kLastFam) and choice
  // (0 count grid, 1 compaction grid, 2 count tile)
  std::mutex tmu;
  gvi_tune_slot tune[kLastFam + 1][kTuneKinds];
  bool autotune = true;
  uint64_t tune_min = kTuneMinBytes;  // launches of fewer entry bytes are not tuning samples
  std::string tune_path;   // autotune cache file ("" = keep choices in memory)
  std::string arch;        // device architecture name, the cache file's key
};

namespace gvi {

thread_local std::string tl_err;

struct DevErr {
  gv_status st;
};

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) {                                                            \
      *X.err = std::string(#x) + ": " + hipGetErrorString(e_);                         \
      throw DevErr{GV_EDEVICE};                                                        \
    }                                                                                  \
  } while (0)

struct Setup {
  ProbC P;
  int fam, d, ell;
  double epsn[4];
  double ez, ek;  // pose eps'
  bool filter;    // binary32 filter usable
  bool exact;     // canon_c = +inf: quantize once to 2^-36, no re-canonization
  double Hmax, R2;  // pose data bounds: max |eta'|, max squared horizontal reach
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
    case GV_SIM2D: S.d = 4; S.ell = 2; break;
    case GV_POSE4DOF: S.d = 4; S.ell = 4; break;
    case GV_POSE5DOF: S.d = 5; S.ell = 4; break;
    default: why = "bad family"; return GV_EINVAL;
  }
  const bool pose = fam_pose(S.fam);
  P.fam = S.fam;
  P.d = S.d;
  P.nsec = pose ? 4 : 1;
  double c = p->canon_c == 0.0 ? 1.0 : p->canon_c;
  if (!(c > 0.0) || std::isnan(c)) { why = "canon_c must be > 0"; return GV_EINVAL; }
  S.exact = std::isinf(c);
  P.exact = S.exact ? 1 : 0;
  for (int j = 0; j < S.d; j++) {
    if (pose && j == 3) continue;  // kappa: fixed [-1, 1] per sector
    if (!std::isfinite(p->lo[j]) || !std::isfinite(p->hi[j]) || !(p->hi[j] > p->lo[j])) { why = "bad box"; return GV_EINVAL; }
    if (!std::isfinite(p->eps[j]) || !(p->eps[j] > 0.0)) { why = "bad eps"; return GV_EINVAL; }
    P.lo[j] = p->lo[j];
    P.E[j] = p->hi[j] - p->lo[j];
    P.inv[j] = 1.0 / P.E[j];
    S.epsn[j] = p->eps[j] * P.inv[j];
  }
  double epsk = 0.0;
  if (pose) {
    if (P.E[0] != P.E[1]) { why = "pose families need hi[0]-lo[0] == hi[1]-lo[1]"; return GV_EINVAL; }
    if (!std::isfinite(p->eps[3]) || !(p->eps[3] > 0.0)) { why = "bad yaw eps"; return GV_EINVAL; }
    epsk = p->eps[3];
    P.lo[3] = -1.0;
    P.E[3] = 2.0;
    P.inv[3] = 0.5;
    S.epsn[3] = epsk * 0.5;
    P.ce = P.E[0] * P.inv[2];
    // f: the factor of the image coordinates in the direction tangents,
    // positive over the box (POSE4DOF: f = 1)
    P.flo = 1.0;
    P.Ef = 0.0;
    if (S.fam == GV_POSE5DOF) {
      if (!(p->lo[4] > 0.0)) { why = "POSE5DOF needs lo[4] > 0 (f)"; return GV_EINVAL; }
      P.flo = p->lo[4];
      P.Ef = P.E[4];
    }
  }
  int Lstar = 0, Bcell = 0;
  for (int j = 0; j < S.d; j++) {
    double ej = (pose && j == 3) ? epsk : p->eps[j];
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
  P.B = Bcell + (pose ? 2 : 0);
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
    int splits[GV_MAXD], ns = 0;
    for (int j = 0; j < GV_MAXD; j++) {
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
  if (!pose && S.exact) {
    // exact mode: one 2^-36 lattice, pads = eps rounded up to it
    for (int q = 0; q < S.d; q++) {
      P.sf[q] = 0x1p-36;
      P.inv_sf[q] = 0x1p36;
      P.xpad[q] = std::ceil((S.epsn[q] + 0.0) / P.sf[q]) * P.sf[q];
    }
  } else if (!pose) {
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
  } else if (!S.exact) {
    S.ez = S.epsn[2] / (c * (double)(Lstar + 1));
    S.ek = epsk / (c * (double)(Lstar + 1));
  }
  return GV_OK;
}

// Pose lattice from the data bounds (same definition as the oracle): rounding
// one parameter by half a step moves z and kappa by at most eps'/(2(l+1))
// anywhere on the box, from the derivative bounds of z = W3 - eta' f r and
// kappa = tan(phi - atan(xi f)) (Fb bounds f; 1 for POSE4DOF).  POSE5DOF:
// false when the directions of one cell could span an arc of pi or more
// (max |xi| f_hi too large), which the arc test does not handle.
bool pose_lattice(Setup& S, double Hmax, double R2, double epsk, double Xmax, const gv_problem* p) {
  ProbC& P = S.P;
  double Fb = 1.0;
  if (S.fam == GV_POSE5DOF) {
    if (!(2.0 * std::atan(1.0 + 2.0 * epsk) + std::atan(Xmax * p->hi[4]) < 3.1)) return false;
    Fb = p->hi[4] * (1.0 + 0x1p-20);
  }
  int Lxy = std::max(P.L[0], P.L[1]);
  double Rg = std::ldexp(1.0, -Lxy);
  P.Rg2 = Rg * Rg;
  S.Hmax = Hmax;
  S.R2 = R2;
  if (S.exact) {
    // exact mode: every parameter on the 2^-36 lattice, pads = eps rounded up
    P.sW = P.sW3 = P.sXi = P.sEta = 0x1p-36;
    P.padz = std::ceil(S.epsn[2] / P.sW3) * P.sW3;
    P.padk = std::ceil(epsk / P.sXi) * P.sXi;
  } else {
  double l1 = (double)(S.ell + 1);
  double Hb = (Hmax > 0x1p-10 ? Hmax : 0x1p-10) * (1.0 + 0x1p-20);
  double Rb = (std::sqrt(R2) + 0x1p-20) * (1.0 + 0x1p-20);
  double pk0 = epsk + S.ek * 0.5;
  double Bk = 1.0 + (1.0 + pk0) * (1.0 + pk0);
  P.sW3 = p2floor(S.ez / l1);
  P.sEta = p2floor(S.ez / (l1 * Rb * Fb));
  double wz = S.ez / (l1 * Hb * Fb), wk = (S.ek * Rg) / (l1 * Bk);
  P.sW = p2floor(wz < wk ? wz : wk);
  P.sXi = p2floor(S.ek / (l1 * Bk * Fb));
  P.padz = std::ceil((S.epsn[2] + S.ez * 0.5) / P.sW3) * P.sW3;
  P.padk = std::ceil((epsk + S.ek * 0.5) / P.sXi) * P.sXi;
  }
  P.inv_sW = 1.0 / P.sW;
  P.inv_sW3 = 1.0 / P.sW3;
  P.inv_sXi = 1.0 / P.sXi;
  P.inv_sEta = 1.0 / P.sEta;
  P.Rg2f = (float)P.Rg2;
  P.padzf = (float)P.padz;
  P.padkf = (float)P.padk;
  return true;
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

// POSE5DOF: the 4-DoF conditions on x, y, z, kappa and the lattice values,
// every step at least 2^-30 and f within [2^-10, 2^10], so that the kappa
// half's products and the z half's first products stay in binary32's normal
// range, and the z half's products below 2^100 (the f bounds are rounded to
// binary32; the filter's bounds include that rounding)
bool pose5_filter_exact(const Setup& S, const double* mx) {
  const ProbC& P = S.P;
  if (!pose_filter_exact(S, mx)) return false;
  if (std::min(std::min(P.sW, P.sW3), std::min(P.sXi, P.sEta)) < 0x1p-30) return false;
  const double fmax = P.flo + P.Ef;
  if (!(P.flo >= 0x1p-10 && fmax <= 0x1p10)) return false;
  const double r = std::max(mx[2], mx[3]) + 1.0, a = mx[6] * fmax;
  if (!(a * a * 2.0 * r * r < 0x1p100 && mx[5] * fmax < 0x1p20)) return false;
  return true;
}

// ---------------------------------------------------------------------------
// One problem inside an epoch (also the record behind a ticket).
// ---------------------------------------------------------------------------
struct ProbRec {
  gv_problem p{};
  Setup S{};
  Cols cols{};
  std::vector<double> host_cols[6];  // submitted host columns (copied at submit)
  std::vector<void*> dev_owned;      // device copies of host columns
  int64_t n = 0;
  double epsk = 0.0;
  bool filter_ok = false;
  unsigned maxK = 0, maxF = 0;
  uint64_t est_bytes = 0;
  // outcome
  gv_status st = GV_OK;
  std::string err;
  uint64_t count = 0, leaf = 0;
  PathC path{};
  int32_t coords[GV_MAXD] = {0, 0, 0, 0, 0};
  std::vector<int64_t> inliers;
  gv_stats stats{};
  // serving
  uint64_t ticket = 0;
  bool done = false, canceled = false;
  std::chrono::steady_clock::time_point t_submit{};
  double ms_queued = 0.0;  // submission to admission
};

struct Batch {
  int level;
  uint32_t ncell;
  uint64_t nent;     // entries of the list buffer
  Cell* cells;
  void* ents;
  bool unit = true;  // every multiplicity is 1
  uint64_t nlive = ~0ull;  // entries the cells hold, when fewer than nent
};

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
  uint32_t* scount = nullptr;   // rank -> count
  uint32_t* rank_of = nullptr;  // child -> rank (or ~0)
  uint64_t* soff = nullptr;     // rank -> first entry (nkept + 1 values)
  uint32_t* cnent = nullptr;    // child -> entries
  uint32_t* ioff = nullptr;     // cell -> its first item
  uint64_t* itemoff = nullptr;  // child-major exclusive scan of per-item survivors
  uint32_t istride = 0;
  int pending = 0;
  bool sorted = true;  // children in descending count order
  uint64_t kept_entries = 0;  // entries of all kept children
  bool unit = true;    // every multiplicity is 1
  bool fresh = false;  // its one chunk comes next, right after its pruning
};

struct Task {
  bool chunk;
  Batch b;
  Parent* par;
  uint32_t r0, r1;
};

// An epoch: a set of problems of one family and one level structure whose
// cells share every batch.  Per-problem constants, best keys and paths live
// in device tables indexed by the cell's problem id.
struct Run {
  gv_ctx* ctx = nullptr;
  hipStream_t st = nullptr;                 // every device operation of the epoch is ordered on it
  DevCache* cache = nullptr;                // allocator of that stream
  std::vector<hipEvent_t>* ev_pool = nullptr;
  uint64_t* hpin = nullptr;      // host-coherent totals (host and device address), else dtot is device memory
  uint64_t* hpin_dev = nullptr;
  std::string* err = nullptr;               // text of the failing HIP call
  uint64_t budget = 0;                      // device bytes the epoch may plan with
  std::vector<ProbRec*> probs;
  int fam = 0;
  ProbC P0{};  // level structure shared by the epoch (first problem's constants)
  int group_mode = 0;
  double lat_bound[GV_MAXL + 1];
  ProbC* dP = nullptr;                    // [nprob]
  unsigned long long* dbest = nullptr;    // [nprob]
  unsigned long long* drecheck = nullptr;
  uint64_t* dtot = nullptr;
  uint32_t* dummy = nullptr;              // sink for outputs a leaf-level pass does not need
  unsigned long long* dreads = nullptr;   // parent bytes read by compaction passes
  int* dovf = nullptr;                    // set when a packed entry could not hold a value
  int pack_from = 1 << 30;                // lists of this level and deeper use the packed entry
  int unit_from = 1 << 30;                // PLANE3D unit-weight lists of this level and deeper: one word
  bool q24 = false;                       // POSE4DOF unit-weight lists below the root: 24-byte entries
  size_t ent_bytes = 0;
  uint64_t chunk_bytes = 0;               // device bytes one materialized chunk may need
  uint64_t first_cells = 262144;          // cells in the first chunk of every expansion
  uint64_t dive_cells = 4096;             // cells from which the diversified dive goes greedy
  bool reuse = true;                      // the main search starts at the dive's greedy level (GV_REUSE=0: off)
  bool root_dive = false;                 // greedy dive from the root cells first (the diversified dive subsumes it)
  int grid_env[2] = {0, 0};               // GV_GRID_COUNT / GV_GRID_COMPACT: fixed blocks per CU (experiments)
  uint32_t tile_env = 0;                  // GV_ITEM_ENTRIES: fixed entries per work item (256, 512 or 1024)
  uint64_t waits = 0;                     // host waits for the stream, and their time
  double wait_ms = 0.0;
  bool trace = false;                     // GV_TRACE=1: one stderr line per expansion
  bool beam = true;                       // progressive chunks until the first leaf level
  bool root_only = false;                 // build the root entries only (gv_incidence)
  bool fixed = false;                     // no tuning samples, no events (allocation-free solve)
  // POSE4DOF: cells of this level and deeper whose lists hold at most
  // GV_SUB_T entries are searched to the leaves on the device
  // (k_subtree_pose), one workgroup per cell (GV_SUBTREE=0: off).  Measured
  // on the 256-problem set: from two levels above the leaves it matches the
  // host-driven path (1.03 against 1.02 s batched) with one host wait for
  // the last two levels; from four levels above the leaves a workgroup's
  // depth-first walk of a large subtree becomes the critical path (1.51 s),
  // from seven levels above 2.64 s.
  bool subtree = true;
  int subtree_from = -2;  // < 0: relative to the leaf level
  unsigned long long* dtests = nullptr;   // tests counted on the device
  // threshold reporting: the best key stays at tau 2^B - 1 (cells below tau
  // are cut) and every leaf reaching tau is appended to rep_idx / rep_cnt
  bool report = false;
  uint64_t tau = 0, rep_cap = 0;
  uint64_t* rep_idx = nullptr;
  uint32_t* rep_cnt = nullptr;
  unsigned long long* rep_n = nullptr;
  struct EvRec {
    std::pair<hipEvent_t, hipEvent_t> e;
    int kind;        // 0 count, 1 compaction
    int cand;        // autotuner candidate index, -1 when not a tuning sample
    uint64_t units;  // entry bytes the launch read (count) or wrote (compaction)
    int tcand;       // count tile candidate index, -1 when not a tile sample
  };
  std::vector<EvRec> ev;
  size_t ev_used = 0;
  gv_stats stats{};
  // originals and roots
  uint64_t Ntot = 0;
  std::vector<uint64_t> ooff;             // [nprob + 1]
  uint64_t* dooff = nullptr;
  double* m64 = nullptr;                  // POSE4DOF binary64 master, SoA stride Ntot
  void* root = nullptr;                   // root entries (grouped), owned
  // search state
  std::vector<Task> stack;
  bool own_first = true;
  std::chrono::steady_clock::time_point t0;
};

// Two host-coherent pinned words that kernels write totals to, so the host
// reads them after a stream wait without a copy.  Null pointers (and device
// memory plus a copy) when the allocation fails.
// Layout: 8 words of totals, then kStageN + 1 words that the chunk planner's
// samples are gathered into.
constexpr uint64_t kStageN = 65536;
void alloc_hpin(uint64_t*& h, uint64_t*& d) {
  h = d = nullptr;
  void* p = nullptr;
  if (hipHostMalloc(&p, (8 + kStageN + 1) * sizeof(uint64_t), hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess)
    return;
  void* q = nullptr;
  if (hipHostGetDevicePointer(&q, p, 0) != hipSuccess) {
    (void)hipHostFree(p);
    return;
  }
  h = (uint64_t*)p;
  d = (uint64_t*)q;
}
void free_hpin(uint64_t*& h, uint64_t*& d) {
  if (h) (void)hipHostFree(h);
  h = d = nullptr;
}

// the host waits for the epoch's stream (counted for the trace line)
void host_wait(Run& X) {
  const auto t = std::chrono::steady_clock::now();
  HIPCHK(hipStreamSynchronize(X.st));
  X.waits++;
  X.wait_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

// epochs of gv_solve / gv_parametrize use the context's stream and allocator
void bind_ctx(Run& X, gv_ctx* c) {
  X.ctx = c;
  X.st = c->stream;
  X.cache = &c->cache;
  X.ev_pool = &c->ev_pool;
  X.hpin = c->hpin;
  X.hpin_dev = c->hpin_dev;
  X.err = &c->err;
  X.budget = c->budget;
}

template <typename T>
T* dalloc(Run& X, size_t count) {
  if (count == 0) count = 1;
  void* p = X.cache->get(count * sizeof(T), X.st, *X.err);
  if (!p) throw DevErr{GV_ENOMEM};
  return (T*)p;
}
void dfree(Run& X, void* p) {
  if (p) X.cache->put(p);
}

template <typename In, typename Out>
void excl_scan(Run& X, const In* in, Out* out, uint64_t n) {
  if (n == 0) return;
  if (n <= GV_SMALL_N) {
    k_scan_small<In, Out><<<1, 1024, 0, X.st>>>(in, out, (uint32_t)n, nullptr);
    return;
  }
  size_t tb = 0;
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, in, out, (int)n, X.st));
  void* tmp = dalloc<char>(X, tb);
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(tmp, tb, in, out, (int)n, X.st));
  dfree(X, tmp);
}

// Stable descending sort of at most GV_SMALL_N (key, value) pairs in one
// workgroup (a block radix sort over the key's low end_bit bits): one launch
// where the device-wide sort takes several.  Padding keys are 0 and sort
// after every real key of 0, because the sort is stable.
__global__ void __launch_bounds__(1024) k_sort_desc_small(const uint32_t* __restrict__ key,
                                                          const uint32_t* __restrict__ val, uint32_t n, int end_bit,
                                                          uint32_t* __restrict__ out) {
  constexpr int PER = GV_SMALL_N / 1024;
  using BRS = hipcub::BlockRadixSort<uint32_t, 1024, PER, uint32_t>;
  __shared__ typename BRS::TempStorage tmp;
  uint32_t k[PER], v[PER];
#pragma unroll
  for (int j = 0; j < PER; j++) {
    const uint32_t i = threadIdx.x * PER + j;
    k[j] = i < n ? key[i] : 0u;
    v[j] = i < n ? val[i] : 0xffffffffu;
  }
  BRS(tmp).SortDescending(k, v, 0, end_bit);
#pragma unroll
  for (int j = 0; j < PER; j++) {
    const uint32_t i = threadIdx.x * PER + j;
    if (i < n) out[i] = v[j];
  }
}

inline unsigned nblk(uint64_t n, unsigned b = 256) { return (unsigned)std::max<uint64_t>(1, (n + b - 1) / b); }
inline unsigned gs_grid(Run& X, uint64_t n) {
  return (unsigned)std::min<uint64_t>(nblk(n), (uint64_t)X.ctx->n_cu * 16);
}

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

// the first n (<= 4) totals the last kernels wrote to X.dtot
void read_tot(Run& X, uint64_t* v, int n = 2) {
  if (X.hpin && X.dtot == X.hpin_dev) {
    host_wait(X);
    const volatile uint64_t* h = X.hpin;
    for (int i = 0; i < n; i++) v[i] = h[i];
  } else {
    HIPCHK(hipMemcpyAsync(v, X.dtot, n * sizeof(uint64_t), hipMemcpyDeviceToHost, X.st));
    host_wait(X);
  }
}

template <typename T>
uint64_t d2h1(Run& X, const T* p) {
  T v{};
  HIPCHK(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, X.st));
  host_wait(X);
  return (uint64_t)v;
}

// Autotune cache file: one line per choice,
//   <arch> <compute units> <family 1..kLastFam> <choice> <value>
// choice 0: count grid, 1: compaction grid (value: blocks per CU);
// choice 2: count tile (value: log2 entries per work item)
void tune_load(gv_ctx* c) {
  if (c->tune_path.empty()) return;
  FILE* f = std::fopen(c->tune_path.c_str(), "r");
  if (!f) return;
  char arch[128];
  int ncu, fam, kind, gpc;
  while (std::fscanf(f, "%127s %d %d %d %d", arch, &ncu, &fam, &kind, &gpc) == 5) {
    if (c->arch != arch || ncu != c->n_cu || fam < 1 || fam > kLastFam || kind < 0 || kind >= kTuneKinds) continue;
    for (int k = 0; k < tune_ncand(kind); k++)
      if (tune_value(kind, k) == gpc) c->tune[fam][kind].chosen = gpc;
  }
  std::fclose(f);
}

// Rewrites the cache file with this context's choices, keeping the lines of
// other devices (called with c->tmu held).
void tune_save(gv_ctx* c) {
  if (c->tune_path.empty()) return;
  std::vector<std::string> keep;
  if (FILE* f = std::fopen(c->tune_path.c_str(), "r")) {
    char arch[128];
    int ncu, fam, kind, gpc;
    while (std::fscanf(f, "%127s %d %d %d %d", arch, &ncu, &fam, &kind, &gpc) == 5) {
      const bool mine = c->arch == arch && ncu == c->n_cu && fam >= 1 && fam <= kLastFam && kind >= 0 &&
                        kind < kTuneKinds && c->tune[fam][kind].chosen;
      if (!mine) keep.push_back(std::string(arch) + " " + std::to_string(ncu) + " " + std::to_string(fam) + " " +
                                std::to_string(kind) + " " + std::to_string(gpc));
    }
    std::fclose(f);
  }
  const std::string tmp = c->tune_path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const std::string& l : keep) std::fprintf(f, "%s\n", l.c_str());
  for (int fam = 1; fam <= kLastFam; fam++)
    for (int kind = 0; kind < kTuneKinds; kind++)
      if (c->tune[fam][kind].chosen)
        std::fprintf(f, "%s %d %d %d %d\n", c->arch.c_str(), c->n_cu, fam, kind, c->tune[fam][kind].chosen);
  std::fclose(f);
  std::rename(tmp.c_str(), c->tune_path.c_str());
}

// One timed tuning launch; once every candidate has its samples the slot
// keeps the lowest time per byte.
void tune_sample(Run& X, int kind, int cand, double ms, uint64_t units) {
  gv_ctx* c = X.ctx;
  std::lock_guard<std::mutex> g(c->tmu);
  gvi_tune_slot& t = c->tune[X.P0.fam][kind];
  if (t.chosen) return;
  if (t.n[cand] >= kTuneSamples) return;
  t.r[cand][t.n[cand]++] = ms / std::max(1.0, (double)units);
  const int nc = tune_ncand(kind);
  for (int k = 0; k < nc; k++)
    if (t.n[k] < kTuneSamples) return;
  double med[kNCand];
  for (int k = 0; k < nc; k++) {
    double v[kTuneSamples];
    std::copy(t.r[k], t.r[k] + kTuneSamples, v);
    std::sort(v, v + kTuneSamples);
    med[k] = 0.5 * (v[kTuneSamples / 2 - 1] + v[kTuneSamples / 2]);
  }
  int best = 0;
  for (int k = 1; k < nc; k++)
    if (med[k] < med[best]) best = k;
  t.chosen = tune_value(kind, best);
  if (X.trace) {
    static const char* what[kTuneKinds] = {"count grid", "compaction grid", "count tile"};
    std::fprintf(stderr, "gv: autotune family %d %s:", X.P0.fam, what[kind]);
    for (int k = 0; k < nc; k++)
      std::fprintf(stderr, " %d:%.3g", kind == 2 ? 1 << tune_value(kind, k) : tune_value(kind, k), med[k] * 1e9);
    if (kind == 2)
      std::fprintf(stderr, " ps/byte -> %d entries per item\n", 1 << t.chosen);
    else
      std::fprintf(stderr, " ps/byte -> %d blocks per CU\n", t.chosen);
  }
  tune_save(c);
}

// Blocks per CU of the next count (kind 0) or compaction (kind 1) launch
// moving `units` entry bytes; *cand = the candidate index when the launch is a tuning
// sample, else -1.
int grid_pick(Run& X, int kind, uint64_t units, int* cand) {
  *cand = -1;
  if (X.grid_env[kind]) return X.grid_env[kind];
  if (X.fixed) {
    std::lock_guard<std::mutex> g(X.ctx->tmu);
    const int ch = X.ctx->tune[X.P0.fam][kind].chosen;
    return ch ? ch : kGridDefault;
  }
  gv_ctx* c = X.ctx;
  if (!c->autotune) return kGridDefault;
  std::lock_guard<std::mutex> g(c->tmu);
  gvi_tune_slot& t = c->tune[X.P0.fam][kind];
  if (t.chosen) return t.chosen;
  if (units < c->tune_min) return kGridDefault;
  *cand = t.next;
  t.next = (t.next + 1) % kNCand;
  return kTuneCand[*cand];
}

// log2 of the entries per work item of a batch whose count pass reads
// `units` entry bytes; *cand as in grid_pick.  Samples are taken only once the
// family's count grid is chosen; the allocation-free solve keeps GV_ITEM.
uint32_t tile_pick(Run& X, uint64_t units, int* cand) {
  *cand = -1;
  if (X.tile_env) return X.tile_env;
  gv_ctx* c = X.ctx;
  if (X.fixed || !c->autotune) return GV_ITEM_LOG;
  std::lock_guard<std::mutex> g(c->tmu);
  gvi_tune_slot& t = c->tune[X.P0.fam][2];
  if (t.chosen) return (uint32_t)t.chosen;
  if (units < c->tune_min || !c->tune[X.P0.fam][0].chosen) return GV_ITEM_LOG;
  *cand = t.next;
  t.next = (t.next + 1) % kNTile;
  return (uint32_t)kTileCand[*cand];
}

std::pair<hipEvent_t, hipEvent_t> ev_begin(Run& X, int kind, int cand = -1, uint64_t units = 0, int tcand = -1) {
  gv_ctx* c = X.ctx;
  std::pair<hipEvent_t, hipEvent_t> p{nullptr, nullptr};
  if ((!c->kernel_timing && cand < 0 && tcand < 0) || X.fixed) return p;
  std::vector<hipEvent_t>& pool = *X.ev_pool;
  while (pool.size() < 2 * (X.ev_used + 1)) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    pool.push_back(e);
  }
  p.first = pool[2 * X.ev_used];
  p.second = pool[2 * X.ev_used + 1];
  X.ev_used++;
  HIPCHK(hipEventRecord(p.first, X.st));
  X.ev.push_back({p, kind, cand, units, tcand});
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
  host_wait(X);
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
  if (fam_pose(X.fam) || X.P0.exact) return false;
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
  const ProbC& P = X.P0;
  const int m = b.level;
  const LevelC lv = P.lev[m];
  const uint32_t nch = 1u << lv.abits;
  const bool leaf = (m + 1 == P.Lstar);
  const uint64_t nk = (uint64_t)b.ncell * nch;
  const uint64_t nlive = std::min(b.nent, b.nlive);
  X.stats.tests += nlive * nch;
  X.stats.cells_expanded += b.ncell;

  Parent* pa = new Parent();
  pa->level = m;
  pa->ncell = b.ncell;
  pa->nent = b.nent;
  pa->cells = b.cells;
  pa->ents = b.ents;
  pa->own_ents = own_ents;
  pa->unit = b.unit;

  // work items: at most 2^ilog <= GV_ITEM entries of one cell each (the
  // count pass's surface tile, autotuned on large batches)
  const uint64_t tbytes = fam_masked(FAM) ? nlive * (sizeof(E) + sizeof(M)) : nlive * sizeof(E);
  int tcand;
  uint32_t ilog = tile_pick(X, tbytes, &tcand);
  if constexpr (FAM == FAM_POSE5DOF)
    if (tcand < 0 && !X.tile_env)
      while (ilog > kItemLogMin5 && (b.nent >> ilog) < (uint64_t)X.ctx->n_cu * kItemsPerCu5) ilog--;
  uint32_t* nitem = b.ncell <= GV_SMALL_N ? nullptr : dalloc<uint32_t>(X, b.ncell);
  pa->ioff = dalloc<uint32_t>(X, b.ncell);
  pa->max_items = b.ncell + (b.nent >> ilog) + 1;
  pa->items = dalloc<Item>(X, pa->max_items);
  pa->nitems = dalloc<uint32_t>(X, 1);
  if (b.ncell <= GV_SMALL_N) {
    k_items_small<<<1, 1024, 0, X.st>>>(b.cells, b.ncell, ilog, pa->ioff, pa->items, pa->nitems);
  } else {
    HIPCHK(hipMemsetAsync(pa->nitems, 0, sizeof(uint32_t), X.st));
    k_item_counts<<<nblk(b.ncell), 256, 0, X.st>>>(b.cells, b.ncell, ilog, nitem);
    excl_scan(X, nitem, pa->ioff, b.ncell);
    k_item_fill<<<nblk(b.ncell), 256, 0, X.st>>>(b.cells, b.ncell, ilog, nitem, pa->ioff, pa->items, pa->nitems);
  }
  dfree(X, nitem);
  pa->istride = (uint32_t)pa->max_items;
  // POSE4DOF keeps per-entry pass masks and counts with atomics, per-item
  // survivors child-major; linear families write one row of per-child
  // counts per item (item-major) and repeat the test in the compaction
  const bool linear = !fam_masked(FAM);
  uint32_t* itemcnt = nullptr;
  uint32_t* itemw = nullptr;
  if (linear) {
    itemcnt = dalloc<uint32_t>(X, (uint64_t)nch * pa->max_items);
    if (!b.unit) itemw = dalloc<uint32_t>(X, (uint64_t)nch * pa->max_items);
  } else if (!leaf) {
    itemcnt = dalloc<uint32_t>(X, (uint64_t)nch * pa->istride);
  }
  if (!linear) pa->masks = dalloc<M>(X, b.nent);
  uint32_t* ccnt = dalloc<uint32_t>(X, nk);
  pa->cnent = dalloc<uint32_t>(X, nk);
  if (!linear) {
    const uint64_t ni = itemcnt ? (uint64_t)nch * pa->istride : 0;
    k_zero3<<<gs_grid(X, std::max(nk, ni)), 256, 0, X.st>>>(ccnt, nk, pa->cnent, nk, itemcnt, ni);
  }
  int cand;
  const int gpc = grid_pick(X, 0, tbytes, &cand);
  const unsigned grid = (unsigned)std::min<uint64_t>((pa->max_items + 3) / 4, (uint64_t)X.ctx->n_cu * gpc);
  auto evp = ev_begin(X, 0, cand, tbytes, tcand);
  X.stats.test_launches++;
  X.stats.test_bytes += tbytes;
  if constexpr (FAM == FAM_POSE5DOF) {
#define GV_COUNT_POSE5(U, A)                                                                                     \
  k_count_pose5<E, U, A><<<grid, 256, 0, X.st>>>(X.dP, m, lv, b.cells, pa->items, pa->nitems, (const E*)b.ents,   \
                                                X.m64, X.Ntot, (uint32_t*)pa->masks, ccnt, pa->cnent, X.drecheck, \
                                                itemcnt ? itemcnt : X.dummy, itemcnt ? pa->istride : 0u)
    static_assert(std::is_same<M, uint32_t>::value, "5-DoF masks are 32-bit");
    const bool all = lv.abits == 5;
    if (b.unit) {
      if (all) GV_COUNT_POSE5(true, true);
      else GV_COUNT_POSE5(true, false);
    } else {
      if (all) GV_COUNT_POSE5(false, true);
      else GV_COUNT_POSE5(false, false);
    }
#undef GV_COUNT_POSE5
  } else if constexpr (FAM == FAM_POSE4DOF) {
#define GV_COUNT_POSE(U, A)                                                                                 \
  k_count_pose<E, U, A><<<grid, 256, 0, X.st>>>(X.dP, m, lv, b.cells, pa->items, pa->nitems, (const E*)b.ents, \
                                                X.m64, X.Ntot, (uint16_t*)pa->masks, ccnt, pa->cnent, X.drecheck, \
                                                itemcnt ? itemcnt : X.dummy, itemcnt ? pa->istride : 0u)
    // every axis splits at most levels: that variant has no per-axis checks
    const bool all = lv.abits == 4;
    if (b.unit) {
      if (all) GV_COUNT_POSE(true, true);
      else GV_COUNT_POSE(true, false);
    } else {
      if (all) GV_COUNT_POSE(false, true);
      else GV_COUNT_POSE(false, false);
    }
#undef GV_COUNT_POSE
  } else if constexpr (fam_exact(FAM)) {
    if (b.unit)
      k_count_x<fam_base(FAM), true, M><<<grid, 256, 0, X.st>>>(X.dP, m, lv, b.cells, pa->items, pa->nitems,
                                                            (const EntX*)b.ents, (M*)pa->masks, ccnt, pa->cnent,
                                                            itemcnt ? itemcnt : X.dummy, itemcnt ? pa->istride : 0u);
    else
      k_count_x<fam_base(FAM), false, M><<<grid, 256, 0, X.st>>>(X.dP, m, lv, b.cells, pa->items, pa->nitems,
                                                             (const EntX*)b.ents, (M*)pa->masks, ccnt,
                                                             pa->cnent, itemcnt ? itemcnt : X.dummy,
                                                             itemcnt ? pa->istride : 0u);
  } else {
#define GV_COUNT_LIN(U, N) \
  k_count_lin<FAM, U, E, N><<<grid, 256, 0, X.st>>>(lv, pa->items, pa->nitems, (const E*)b.ents, itemcnt, itemw)
    switch ((b.unit ? 32 : 0) | nch) {
      case 32 | 2: GV_COUNT_LIN(true, 2); break;
      case 32 | 4: GV_COUNT_LIN(true, 4); break;
      case 32 | 8: GV_COUNT_LIN(true, 8); break;
      case 2: GV_COUNT_LIN(false, 2); break;
      case 4: GV_COUNT_LIN(false, 4); break;
      case 8: GV_COUNT_LIN(false, 8); break;
      case 32 | 16:
        if constexpr (FAM == FAM_SIM2D) GV_COUNT_LIN(true, 16);
        else throw DevErr{GV_EINVAL};
        break;
      case 16:
        if constexpr (FAM == FAM_SIM2D) GV_COUNT_LIN(false, 16);
        else throw DevErr{GV_EINVAL};
        break;
      default: throw DevErr{GV_EINVAL};
    }
#undef GV_COUNT_LIN
  }
  ev_end(X, evp);
  HIPCHK(hipGetLastError());
  if constexpr (!fam_masked(FAM)) {
    // per-cell counts and per-item offsets from the items' rows
    if (!leaf) pa->itemoff = dalloc<uint64_t>(X, (uint64_t)nch * pa->max_items);
#define GV_CELL_SCAN(U, N)                                                                                      \
  k_cell_scan<N, U><<<nblk((uint64_t)b.ncell * N), 256, 0, X.st>>>(b.cells, b.ncell, ilog, pa->ioff, itemcnt, itemw, \
                                                                   pa->itemoff, ccnt, pa->cnent)
    switch ((b.unit ? 32 : 0) | nch) {
      case 32 | 2: GV_CELL_SCAN(true, 2); break;
      case 32 | 4: GV_CELL_SCAN(true, 4); break;
      case 32 | 8: GV_CELL_SCAN(true, 8); break;
      case 32 | 16: GV_CELL_SCAN(true, 16); break;
      case 2: GV_CELL_SCAN(false, 2); break;
      case 4: GV_CELL_SCAN(false, 4); break;
      case 8: GV_CELL_SCAN(false, 8); break;
      case 16: GV_CELL_SCAN(false, 16); break;
      default: throw DevErr{GV_EINVAL};
    }
#undef GV_CELL_SCAN
    HIPCHK(hipGetLastError());
    dfree(X, itemcnt);
    dfree(X, itemw);
    itemcnt = itemw = nullptr;
  }

  if (dive && !leaf) {
    // greedy dive: one child per cell in parent order; the kept list is
    // written directly (no selection scan, no sort), its entries summed by
    // the offsets' scan
    const uint32_t nkept = b.ncell;
    pa->nkept = nkept;
    pa->sorted = false;
    pa->order = dalloc<uint32_t>(X, nkept);
    pa->scount = dalloc<uint32_t>(X, nkept);
    pa->rank_of = dalloc<uint32_t>(X, nk);
    uint32_t* sn = dalloc<uint32_t>(X, nkept);
    k_pick_kept<<<nblk(nkept), 256, 0, X.st>>>(lv, nkept, ccnt, pa->cnent, pa->order, pa->scount, sn, pa->rank_of);
    dfree(X, ccnt);
    pa->soff = dalloc<uint64_t>(X, nkept + 1);
    if (nkept <= GV_SMALL_N) {
      k_scan_small<uint32_t, uint64_t><<<1, 1024, 0, X.st>>>(sn, pa->soff, nkept, pa->soff + nkept);
    } else {
      excl_scan(X, sn, pa->soff, nkept);
      k_soff_last<<<1, 64, 0, X.st>>>(pa->soff, sn, nkept);
    }
    k_tot_from<<<1, 64, 0, X.st>>>(nkept, pa->soff + nkept, X.dtot);
    dfree(X, sn);
    if (itemcnt) {  // POSE4DOF: child-major offsets for k_compact
      pa->itemoff = dalloc<uint64_t>(X, (uint64_t)nch * pa->istride);
      excl_scan(X, itemcnt, pa->itemoff, (uint64_t)nch * pa->istride);
      dfree(X, itemcnt);
    }
    HIPCHK(hipGetLastError());
    uint64_t kt[2];
    read_tot(X, kt);
    pa->kept_entries = kt[1];
    X.stats.cells_pruned += nk - nkept;
    if (X.trace) {
      const uint64_t bst = d2h1(X, X.dbest);
      std::fprintf(stderr, "gv: level %d cells %u entries %llu kept %llu best %llu (dive)%s\n", m, b.ncell,
                   (unsigned long long)b.nent, (unsigned long long)nkept, (unsigned long long)(bst >> P.B),
                   (b.unit && m >= X.unit_from) ? " one-word" : (m >= X.pack_from ? " packed" : ""));
    }
    return pa;
  }
  uint32_t* keepf = dalloc<uint32_t>(X, nk);
  uint64_t* keptn = dalloc<uint64_t>(X, nk);
  if (dive) {
    k_pick_best<<<nblk(b.ncell), 256, 0, X.st>>>(lv, P.B, P.idxmask, leaf ? 1 : 0, b.cells, b.ncell, ccnt,
                                                 pa->cnent, X.dbest, keepf, keptn);
  } else if (leaf && X.report) {
    // (the leaves are reported below; the bound stays fixed)
  } else {
    k_prune<<<nblk(nk), 256, 0, X.st>>>(lv, P.B, P.idxmask, leaf ? 1 : 0, b.cells, b.ncell, ccnt, pa->cnent,
                                        X.dbest, keepf, keptn);
  }
  HIPCHK(hipGetLastError());
  if (leaf && X.report) {
    k_report_leaves<<<nblk(nk), 256, 0, X.st>>>(lv, P.B, P.idxmask, b.cells, b.ncell, ccnt, X.dbest, X.rep_idx,
                                                 X.rep_cnt, X.rep_n, X.rep_cap);
    HIPCHK(hipGetLastError());
  }
  if (leaf) {
    dfree(X, keptn);
    if (!dive) X.beam = false;
    dfree(X, keepf);
    dfree(X, ccnt);
    pa->pending = 0;
    free_parent(X, pa);
    return nullptr;
  }
  uint32_t* keepscan = dalloc<uint32_t>(X, nk);
  if (nk <= GV_SMALL_N) {
    k_keep_small<<<1, 1024, 0, X.st>>>(keepf, keptn, (uint32_t)nk, keepscan, X.dtot);
  } else {
    excl_scan(X, keepf, keepscan, nk);
    uint64_t* esum = dalloc<uint64_t>(X, 1);
    size_t tb = 0;
    HIPCHK(hipcub::DeviceReduce::Sum(nullptr, tb, keptn, esum, (int)nk, X.st));
    void* tmp = dalloc<char>(X, tb);
    HIPCHK(hipcub::DeviceReduce::Sum(tmp, tb, keptn, esum, (int)nk, X.st));
    dfree(X, tmp);
    k_kept_total<<<1, 64, 0, X.st>>>(keepf, keepscan, nk, esum, X.dtot);
    dfree(X, esum);
  }
  dfree(X, keptn);
  uint64_t kt[2];
  read_tot(X, kt);
  const uint64_t nkept = kt[0];
  pa->kept_entries = kt[1];
  X.stats.cells_pruned += nk - nkept;
  if (X.trace) {
    const uint64_t bst = d2h1(X, X.dbest);
    std::fprintf(stderr, "gv: level %d cells %u entries %llu kept %llu best %llu%s%s\n", m, b.ncell,
                 (unsigned long long)b.nent, (unsigned long long)nkept, (unsigned long long)(bst >> P.B),
                 dive ? " (dive)" : "",
                 (b.unit && m >= X.unit_from) ? " one-word" : (m >= X.pack_from ? " packed" : ""));
  }
  if (nkept == 0) {
    dfree(X, keepf);
    dfree(X, keepscan);
    dfree(X, ccnt);
    dfree(X, itemcnt);
    free_parent(X, pa);
    return nullptr;
  }
  if (itemcnt) {  // POSE4DOF: child-major offsets for k_compact
    pa->itemoff = dalloc<uint64_t>(X, (uint64_t)nch * pa->istride);
    excl_scan(X, itemcnt, pa->itemoff, (uint64_t)nch * pa->istride);
    dfree(X, itemcnt);
  }
  pa->nkept = (uint32_t)nkept;
  uint32_t* kcnt = dalloc<uint32_t>(X, nkept);
  uint32_t* kid = dalloc<uint32_t>(X, nkept);
  pa->rank_of = dalloc<uint32_t>(X, nk);
  k_select_kept<<<nblk(nk), 256, 0, X.st>>>(keepf, keepscan, ccnt, nk, kcnt, kid, pa->rank_of);
  dfree(X, keepf);
  dfree(X, keepscan);
  // Count order only during the first descent.  After it a chunk is capped
  // by memory alone, so the kept children of a parent mostly go in one
  // chunk and their order changes little: the 4-DoF and 5-DoF workloads
  // count the same tests in parent order, and the sort is saved.  Parent
  // order also makes a chunk a contiguous range of parents, each read once.
  // The greedy dive keeps one child per cell and takes them all at once:
  // parent order, no sort.
  pa->sorted = !dive && X.beam;
  pa->scount = dalloc<uint32_t>(X, nkept);
  if (!pa->sorted) {
    // after the first descent the bounds are strong: keep parent order so
    // that a chunk is a contiguous range of parents, each read once
    pa->order = kid;
    kid = nullptr;
  } else {
    pa->order = dalloc<uint32_t>(X, nkept);
    uint32_t* key = kcnt;
    uint32_t* pmax = nullptr;
    if (X.probs.size() > 1) {
      pmax = dalloc<uint32_t>(X, X.probs.size());
      key = dalloc<uint32_t>(X, nkept);
      HIPCHK(hipMemsetAsync(pmax, 0, X.probs.size() * sizeof(uint32_t), X.st));
      k_prob_max<<<nblk(nkept), 256, 0, X.st>>>(kcnt, kid, (uint32_t)nkept, b.cells, nch, pmax);
      k_prob_norm<<<nblk(nkept), 256, 0, X.st>>>(kcnt, kid, (uint32_t)nkept, b.cells, nch, pmax, key);
    }
    // one problem: the key is a count, at most n, so only its low bits are
    // sorted (fewer radix passes on small problems)
    int end_bit = 32;
    if (!pmax) {
      end_bit = 1;
      while (end_bit < 32 && (uint64_t)X.probs[0]->n >> end_bit) end_bit++;
    }
    if (nkept <= GV_SMALL_N) {
      k_sort_desc_small<<<1, 1024, 0, X.st>>>(key, kid, (uint32_t)nkept, end_bit, pa->order);
    } else {
      uint32_t* skey = dalloc<uint32_t>(X, nkept);
      size_t tb = 0;
      HIPCHK(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tb, key, skey, kid, pa->order, (int)nkept, 0,
                                                           end_bit, X.st));
      void* tmp = dalloc<char>(X, tb);
      HIPCHK(hipcub::DeviceRadixSort::SortPairsDescending(tmp, tb, key, skey, kid, pa->order, (int)nkept, 0, end_bit,
                                                           X.st));
      dfree(X, tmp);
      dfree(X, skey);
    }
    if (pmax) {
      dfree(X, pmax);
      dfree(X, key);
    }
  }
  dfree(X, kcnt);
  dfree(X, kid);
  uint32_t* sn = dalloc<uint32_t>(X, nkept);
  k_rank<<<nblk(nkept), 256, 0, X.st>>>(pa->order, (uint32_t)nkept, pa->cnent, ccnt, pa->rank_of, sn, pa->scount);
  dfree(X, ccnt);
  pa->soff = dalloc<uint64_t>(X, nkept + 1);
  if (nkept <= GV_SMALL_N) {
    k_scan_small<uint32_t, uint64_t><<<1, 1024, 0, X.st>>>(sn, pa->soff, (uint32_t)nkept, pa->soff + nkept);
  } else {
    excl_scan(X, sn, pa->soff, nkept);
    k_soff_last<<<1, 64, 0, X.st>>>(pa->soff, sn, (uint32_t)nkept);
  }
  dfree(X, sn);
  return pa;
}

// Chunk schedule over the sorted children: chunk j holds at most
// first_cells * 4^j cells (so the first descent follows a narrow beam of
// the highest-count cells) and at most chunk_bytes of estimated device
// memory once expanded: its lists plus the per-cell and per-child arrays.
void plan_chunks(Run& X, Parent* pa, std::vector<std::pair<uint32_t, uint32_t>>& chunks) {
  const uint32_t nk = pa->nkept;
  const uint64_t stride = std::max<uint64_t>(1, ((uint64_t)nk + kStageN - 1) / kStageN);
  const uint64_t ns = (nk + stride - 1) / stride;  // samples soff[i*stride], plus soff[nk]
  std::vector<uint64_t> s(ns + 1);
  if (X.hpin) {
    // gathered straight into host-coherent memory: no copy
    k_gather_u64<<<nblk(ns + 1), 256, 0, X.st>>>(pa->soff, nk, stride, X.hpin_dev + 8);
    host_wait(X);
    std::memcpy(s.data(), X.hpin + 8, (ns + 1) * sizeof(uint64_t));
  } else {
    uint64_t* d = dalloc<uint64_t>(X, ns + 1);
    k_gather_u64<<<nblk(ns + 1), 256, 0, X.st>>>(pa->soff, nk, stride, d);
    HIPCHK(hipMemcpyAsync(s.data(), d, (ns + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, X.st));
    host_wait(X);
    dfree(X, d);
  }
  auto at = [&](uint64_t i) { return i >= ns ? s[ns] : s[i]; };  // sample i -> soff[min(i*stride, nk)]
  auto rk = [&](uint64_t i) { return (uint32_t)std::min<uint64_t>(i * stride, nk); };
  const int lc = std::min(pa->level + 1, X.P0.Lstar - 1);
  const double per_cell = 64.0 + 40.0 * (double)(1u << X.P0.lev[lc].abits);
  const double per_ent = (double)X.ent_bytes + 8.0;
  auto fits = [&](uint64_t a, uint64_t b) {
    return (double)(at(b) - at(a)) * per_ent + (double)(rk(b) - rk(a)) * per_cell <= (double)X.chunk_bytes;
  };
  uint64_t i0 = 0, cap = X.beam ? X.first_cells : (1ull << 30);
  while (rk(i0) < nk) {
    uint64_t i1 = i0 + 1;
    while (i1 < ns && (rk(i1 + 1) - rk(i0)) <= cap && fits(i0, i1 + 1)) i1++;
    chunks.push_back({rk(i0), rk(i1)});
    i0 = i1;
    cap = X.beam ? std::min<uint64_t>(cap * 4, 1ull << 30) : (1ull << 30);
  }
}

// Materialize one chunk [r0, r1) of a parent as a new batch (after cutting it
// against the current best).  Returns false when nothing remains.
template <int FAM, typename E, typename EO, typename M>
bool materialize(Run& X, Parent* pa, uint32_t r0, uint32_t r1, Batch& nb) {
  const ProbC& P = X.P0;
  const LevelC lv = P.lev[pa->level];
  const uint32_t nch = 1u << lv.abits;
  const uint32_t nr = r1 - r0;
  // drop the children that can no longer reach their problem's best leaf
  uint32_t* keepc = dalloc<uint32_t>(X, nr);
  uint32_t* cidx = dalloc<uint32_t>(X, nr);
  uint64_t* csize = dalloc<uint64_t>(X, nr);
  uint64_t* coff = dalloc<uint64_t>(X, nr);
  // A chunk of every kept child materialized right after its parent's
  // pruning: no bound has moved since, so nothing is re-cut and its sizes
  // are the parent's totals (no wait for the device).
  const bool fresh = pa->fresh && r0 == 0 && r1 == pa->nkept;
  pa->fresh = false;
  k_chunk_keep<<<nblk(nr), 256, 0, X.st>>>(pa->order, pa->scount, pa->cells, nch, X.dbest, P.B, r0, r1, pa->cnent,
                                            keepc, csize, fresh ? 1 : 0);
  if (nr <= GV_SMALL_N) {
    k_chunk_small<<<1, 1024, 0, X.st>>>(keepc, csize, nr, cidx, coff, X.dtot);
  } else {
    excl_scan(X, keepc, cidx, nr);
    excl_scan(X, csize, coff, nr);
    k_chunk_totals<<<1, 64, 0, X.st>>>(keepc, cidx, csize, coff, nr, X.dtot);
  }
  // linear families: the item range the chunk draws from (read with the totals)
  const bool linear = !fam_masked(FAM);
  uint32_t* nwork = nullptr;
  if (linear) {
    nwork = dalloc<uint32_t>(X, 1);
    k_chunk_range<<<1, 64, 0, X.st>>>(pa->order, r0, r1, nch, pa->ioff, pa->ncell, pa->nitems, pa->sorted ? 1 : 0,
                                      nwork, X.dtot + 2);
  }
  uint64_t tot[4];
  if (fresh) {
    tot[0] = pa->nkept;
    tot[1] = pa->kept_entries;
    tot[2] = 0;
    tot[3] = pa->max_items;  // every item (clamped to the count on the device)
  } else {
    read_tot(X, tot, linear ? 4 : 2);
  }
  bool made = false;
  X.stats.cells_pruned += nr - tot[0];
  if (tot[0] > 0) {
    nb.level = pa->level + 1;
    nb.ncell = (uint32_t)tot[0];
    nb.nent = tot[1];
    nb.cells = dalloc<Cell>(X, nb.ncell);
    nb.ents = dalloc<EO>(X, nb.nent);
    k_emit_ranked<<<nblk(nr), 256, 0, X.st>>>(lv, pa->cells, pa->order, r0, r1, keepc, cidx, coff, pa->cnent,
                                              nb.cells);
    int cand;
    const int gpc = grid_pick(X, 1, nb.nent * sizeof(EO), &cand);
    const unsigned grid = (unsigned)std::min<uint64_t>((pa->max_items + 3) / 4, (uint64_t)X.ctx->n_cu * gpc);
    // linear families: the items with a child in this chunk become a work
    // list (offsets resolved), then one wave per work item
    void* work = nullptr;
    if (linear) {
      const uint32_t i0 = (uint32_t)tot[2], i1 = (uint32_t)std::max(tot[2], tot[3]);
#define GV_WORK(N)                                                                                                \
  work = dalloc<CWork<N>>(X, std::max<uint64_t>(1, i1 - i0));                                                     \
  k_chunk_work<N><<<nblk(i1 - i0), 256, 0, X.st>>>(pa->items, pa->nitems, i0, i1, pa->itemoff, pa->rank_of, r0, r1, \
                                                  keepc, coff,                                                    \
                                                  (CWork<N>*)work, nwork, (uint32_t)(8 * sizeof(E)),             \
                                                  X.ctx->kernel_timing ? X.dreads : nullptr)
      switch (nch) {
        case 2: GV_WORK(2); break;
        case 4: GV_WORK(4); break;
        case 8: GV_WORK(8); break;
        case 16: GV_WORK(16); break;
        default: throw DevErr{GV_EINVAL};
      }
#undef GV_WORK
    }
    if (X.ctx->kernel_timing && !linear)
      k_chunk_reads<<<nblk(pa->ncell), 256, 0, X.st>>>(
          pa->cells, pa->ncell, nch, pa->rank_of, r0, r1, keepc,
          (uint32_t)(linear ? 8 * sizeof(E) : 8 * (sizeof(E) + sizeof(M))), X.dreads);
    auto evp = ev_begin(X, 1, cand, nb.nent * sizeof(EO));
    X.stats.compact_launches++;
    X.stats.compact_bytes += nb.nent * sizeof(EO);
    X.stats.compact_write_bytes += nb.nent * sizeof(EO);
    if constexpr (fam_masked(FAM)) {
      k_compact<FAM, E, EO, M, true><<<grid, 256, 0, X.st>>>(
          lv, pa->cells, pa->items, pa->nitems, pa->ioff, pa->itemoff, pa->istride, (const E*)pa->ents,
          (const M*)pa->masks, pa->rank_of, r0, r1, keepc, coff, (EO*)nb.ents, X.dovf);
    } else {
#define GV_COMPACT_LIN(N)                                                                                         \
  k_compact_lin<FAM, E, EO, N><<<grid, 256, 0, X.st>>>(lv, (const CWork<N>*)work, nwork, (const E*)pa->ents,      \
                                                       (EO*)nb.ents, X.dovf)
      switch (nch) {
        case 2: GV_COMPACT_LIN(2); break;
        case 4: GV_COMPACT_LIN(4); break;
        case 8: GV_COMPACT_LIN(8); break;
        case 16:
          if constexpr (FAM == FAM_SIM2D) GV_COMPACT_LIN(16);
          else throw DevErr{GV_EINVAL};
          break;
        default: throw DevErr{GV_EINVAL};
      }
#undef GV_COMPACT_LIN
    }
    ev_end(X, evp);
    HIPCHK(hipGetLastError());
    dfree(X, work);
    nb.unit = pa->unit;
    made = true;
  }
  dfree(X, nwork);
  dfree(X, keepc);
  dfree(X, cidx);
  dfree(X, csize);
  dfree(X, coff);
  if (--pa->pending == 0) free_parent(X, pa);
  if constexpr (std::is_same<EO, EntQ24>::value) {
    // used only where no list is grouped
    if (made && want_group(X, nb)) throw DevErr{GV_EINVAL};
  } else if constexpr (std::is_same<EO, EntP3u>::value) {
    // merged entries carry weights: widen to the 8-byte entry, then group
    if (made && want_group(X, nb)) {
      if (X.trace) std::fprintf(stderr, "gv: level %d one-word lists widened for grouping\n", nb.level);
      EntP3p* w = dalloc<EntP3p>(X, nb.nent);
      k_unit_to_p3<<<gs_grid(X, nb.nent), 256, 0, X.st>>>((const EntP3u*)nb.ents, nb.nent, w);
      dfree(X, nb.ents);
      nb.ents = w;
      nb.unit = false;
      group_batch<EntP3p>(X, nb, true);
    }
  } else {
    if (made && want_group(X, nb)) group_batch<EO>(X, nb, true);
  }
  return made;
}

// Entry type of a level's lists: the packed entry from pack_from on.
template <int FAM, typename E>
using PackedT = std::conditional_t<fam_pose(FAM) || std::is_void_v<typename PackOf<FAM>::T>, E,
                                   typename PackOf<FAM>::T>;

template <int FAM, typename E, typename M>
Parent* expand_at(Run& X, Batch& b, bool own_ents, bool dive) {
  if constexpr (FAM == FAM_PLANE3D)
    if (b.unit && b.level >= X.unit_from) return expand<FAM, EntP3u, M>(X, b, own_ents, dive);
  if constexpr ((FAM == FAM_POSE4DOF || FAM == FAM_POSE5DOF) && std::is_same<E, EntQ32>::value)
    if (b.unit && b.level >= 1 && X.q24) return expand<FAM, EntQ24, M>(X, b, own_ents, dive);
  if (b.level >= X.pack_from) return expand<FAM, PackedT<FAM, E>, M>(X, b, own_ents, dive);
  return expand<FAM, E, M>(X, b, own_ents, dive);
}

template <int FAM, typename E, typename M>
bool materialize_at(Run& X, Parent* pa, uint32_t r0, uint32_t r1, Batch& nb) {
  using EP = PackedT<FAM, E>;
  if constexpr ((FAM == FAM_POSE4DOF || FAM == FAM_POSE5DOF) && std::is_same<E, EntQ32>::value) {
    if (pa->unit && X.q24) {
      if (pa->level >= 1) return materialize<FAM, EntQ24, EntQ24, M>(X, pa, r0, r1, nb);
      return materialize<FAM, EntQ32, EntQ24, M>(X, pa, r0, r1, nb);
    }
  }
  if constexpr (FAM == FAM_PLANE3D) {
    if (pa->unit && pa->level + 1 >= X.unit_from) {
      if (pa->level >= X.unit_from) return materialize<FAM, EntP3u, EntP3u, M>(X, pa, r0, r1, nb);
      if (pa->level >= X.pack_from) return materialize<FAM, EP, EntP3u, M>(X, pa, r0, r1, nb);
      return materialize<FAM, E, EntP3u, M>(X, pa, r0, r1, nb);
    }
  }
  if (pa->level >= X.pack_from) return materialize<FAM, EP, EP, M>(X, pa, r0, r1, nb);
  if (pa->level + 1 >= X.pack_from) return materialize<FAM, E, EP, M>(X, pa, r0, r1, nb);
  return materialize<FAM, E, E, M>(X, pa, r0, r1, nb);
}

// Whether every kept child fits the first chunk the schedule would cut (the
// same rule as plan_chunks, decided from the totals already on the host).
bool one_chunk(const Run& X, const Parent* pa) {
  const int lc = std::min(pa->level + 1, X.P0.Lstar - 1);
  const double per_cell = 64.0 + 40.0 * (double)(1u << X.P0.lev[lc].abits);
  const double per_ent = (double)X.ent_bytes + 8.0;
  const uint64_t cap = X.beam ? X.first_cells : (1ull << 30);
  return (uint64_t)pa->nkept <= cap &&
         (double)pa->kept_entries * per_ent + (double)pa->nkept * per_cell <= (double)X.chunk_bytes;
}

template <int FAM, typename E, typename M>
void push_children(Run& X, Parent* pa, std::vector<Task>& stack) {
  std::vector<std::pair<uint32_t, uint32_t>> chunks;
  // all kept children in one chunk when they fit (no need to sample the
  // list offsets), else the chunk schedule
  if (one_chunk(X, pa)) {
    chunks.push_back({0u, pa->nkept});
    pa->fresh = true;  // (the next step materializes it)
  } else {
    plan_chunks(X, pa, chunks);
  }
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


// ===========================================================================
// Epochs
// ===========================================================================
void decode_leaf(const ProbC& P, uint64_t idx, PathC& path, int32_t* coords) {
  path.sector = fam_pose(P.fam) ? (int32_t)(idx >> P.Bcell) : 0;
  int32_t cc[GV_MAXD] = {0, 0, 0, 0, 0};
  for (int m = 0; m < P.Lstar; m++) {
    const LevelC& lv = P.lev[m];
    const uint32_t dg = (uint32_t)((idx >> lv.rem_next) & ((1ull << lv.abits) - 1ull));
    path.digit[m] = (uint8_t)dg;
    const uint32_t cb = lv.cbits[dg];
    for (int a = 0; a < GV_MAXD; a++)
      if (lv.split[a]) cc[a] = 2 * cc[a] + (int32_t)((cb >> a) & 1u);
  }
  for (int a = 0; a < GV_MAXD; a++) coords[a] = cc[a];
}

int ncols_of(int fam, int d) { return fam == GV_RAY3D ? 6 : (fam_pose(fam) ? 5 : d); }

// host-side validation and constants of one problem
gv_status prepare_problem(ProbRec* pr) {
  std::string why;
  gv_status st = setup_axes(&pr->p, pr->S, why);
  if (st != GV_OK) {
    pr->err = why;
    return st;
  }
  pr->n = pr->p.n;
  pr->epsk = pr->p.eps[3];
  const int nc = ncols_of(pr->S.fam, pr->S.d);
  for (int k = 0; k < nc; k++)
    if (!pr->p.col[k] && pr->n > 0) {
      pr->err = "missing column";
      return GV_EINVAL;
    }
  const uint64_t eb = pr->S.fam == GV_POSE5DOF ? 4 * (96 + 2 * 52)
                      : pr->S.fam == GV_POSE4DOF ? 4 * (80 + 2 * 34)
                      : (pr->S.fam == GV_SIM2D ? 4 * 34 : (pr->S.fam == GV_RAY3D ? 4 * 26 : 4 * 18));
  pr->est_bytes = (uint64_t)std::max<int64_t>(pr->n, 1) * eb + (64ull << 20);
  return GV_OK;
}

// problems can share an epoch when their level structure is identical
bool same_structure(const ProbRec* a, const ProbRec* b) {
  const ProbC &A = a->S.P, &B = b->S.P;
  if (a->S.fam != b->S.fam || A.Lstar != B.Lstar || A.B != B.B || A.exact != B.exact) return false;
  if (a->p.precision != b->p.precision || a->p.group != b->p.group) return false;
  for (int j = 0; j < GV_MAXD; j++)
    if (A.L[j] != B.L[j]) return false;
  return std::memcmp(A.lev, B.lev, sizeof(LevelC) * A.Lstar) == 0;
}

void fail_all(Run& X, gv_status st) {
  for (ProbRec* pr : X.probs)
    if (pr->st == GV_OK) {
      pr->st = st;
      pr->err = *X.err;
    }
}

// tables, columns, counters of a new epoch
void epoch_begin(Run& X) {
  X.t0 = std::chrono::steady_clock::now();
  X.trace = std::getenv("GV_TRACE") != nullptr;
  ProbRec* p0 = X.probs[0];
  X.P0 = p0->S.P;
  X.fam = p0->S.fam;
  X.group_mode = p0->p.group;
  // the parent batches of the levels above stay alive under the one being
  // built, but only the deepest few are large (the lists grow with depth
  // until pruning bites): measured peaks are about twice one chunk, and a
  // fifth of the budget per chunk leaves room for four large levels
  X.chunk_bytes = std::max<uint64_t>(X.fixed ? (4ull << 20) : (64ull << 20), X.budget / 5);
  if (const char* cb = std::getenv("GV_CHUNK_BYTES")) X.chunk_bytes = std::max<uint64_t>(4096, std::strtoull(cb, nullptr, 10));
  if (const char* e = std::getenv("GV_GRID_COUNT")) X.grid_env[0] = std::max(1, std::min(64, atoi(e)));
  if (const char* e = std::getenv("GV_GRID_COMPACT")) X.grid_env[1] = std::max(1, std::min(64, atoi(e)));
  if (const char* e = std::getenv("GV_ITEM_ENTRIES")) {
    const int v = atoi(e);
    for (int k = 0; k < kNTile; k++)
      if (v == 1 << kTileCand[k]) X.tile_env = (uint32_t)kTileCand[k];
  }
  const uint32_t np = (uint32_t)X.probs.size();
  X.ooff.assign(np + 1, 0);
  for (uint32_t p = 0; p < np; p++) X.ooff[p + 1] = X.ooff[p] + (uint64_t)X.probs[p]->n;
  X.Ntot = X.ooff[np];
  // first-descent beam: 65536 cells per problem keeps the planted cells of a
  // large problem in it at the coarse levels and pays for itself in bound
  // quality on small ones; problems sharing an epoch each keep that width
  // (262144: the hardest problems of the 256-problem pose set find their
  // bound in the first chunk; 65536 left one solving 8x longer)
  // diversified dive: greedy from the first level holding 4096 cells per
  // problem (16384 expanded the 32-child 5-DoF levels once more, to 131072
  // cells, before going greedy: 2.2x the solve time on pose5dof_20k, the
  // same bound; the 4-DoF and serving searches are unchanged, the plane
  // search 3% faster; 1024 made the 256-problem pose set 2x slower)
  // (GV_FIRST_CELLS, GV_DIVE_CELLS: per-problem values)
  uint64_t fc1 = 262144, dc1 = 4096;
  if (const char* fc = std::getenv("GV_FIRST_CELLS")) fc1 = std::max<uint64_t>(1, std::strtoull(fc, nullptr, 10));
  if (const char* dc = std::getenv("GV_DIVE_CELLS")) dc1 = std::strtoull(dc, nullptr, 10);
  X.first_cells = fc1 * (uint64_t)np;
  X.dive_cells = dc1 * (uint64_t)np;
  if (const char* e = std::getenv("GV_REUSE")) X.reuse = atoi(e) != 0;
  if (const char* rd = std::getenv("GV_ROOT_DIVE")) X.root_dive = atoi(rd) != 0;
  HIPCHK(hipSetDevice(X.ctx->device));
  X.dP = dalloc<ProbC>(X, np);
  X.dbest = dalloc<unsigned long long>(X, np);
  X.drecheck = dalloc<unsigned long long>(X, 1);
  X.dtests = dalloc<unsigned long long>(X, 1);
  HIPCHK(hipMemsetAsync(X.dtests, 0, 8, X.st));
  if (const char* e = std::getenv("GV_SUBTREE")) X.subtree = atoi(e) != 0;
  if (const char* e = std::getenv("GV_SUBTREE_FROM")) X.subtree_from = atoi(e);
  if (X.subtree_from < 0) X.subtree_from = std::max(1, X.P0.Lstar + X.subtree_from);
  X.dtot = X.hpin_dev ? X.hpin_dev : dalloc<uint64_t>(X, 4);
  X.dummy = dalloc<uint32_t>(X, 64);
  X.dreads = dalloc<unsigned long long>(X, 1);
  X.dovf = dalloc<int>(X, 1);
  X.pack_from = 1 << 30;
  X.dooff = dalloc<uint64_t>(X, np + 1);
  if (X.report) {
    std::vector<unsigned long long> b0(np);
    for (uint32_t p = 0; p < np; p++) b0[p] = (unsigned long long)((X.tau << X.probs[p]->S.P.B) - 1ull);
    HIPCHK(hipMemcpyAsync(X.dbest, b0.data(), np * 8, hipMemcpyHostToDevice, X.st));
    host_wait(X);
  } else {
    HIPCHK(hipMemsetAsync(X.dbest, 0, np * 8, X.st));
  }
  HIPCHK(hipMemsetAsync(X.drecheck, 0, 8, X.st));
  HIPCHK(hipMemsetAsync(X.dreads, 0, 8, X.st));
  HIPCHK(hipMemsetAsync(X.dovf, 0, sizeof(int), X.st));
  HIPCHK(hipMemcpyAsync(X.dooff, X.ooff.data(), (np + 1) * 8, hipMemcpyHostToDevice, X.st));
  std::vector<ProbC> tab(np);
  for (uint32_t p = 0; p < np; p++) tab[p] = X.probs[p]->S.P;
  HIPCHK(hipMemcpyAsync(X.dP, tab.data(), np * sizeof(ProbC), hipMemcpyHostToDevice, X.st));
  for (ProbRec* pr : X.probs) {
    const int nc = ncols_of(pr->S.fam, pr->S.d);
    for (int k = 0; k < nc; k++) {
      if (pr->p.cols_on_device || pr->n == 0) {
        pr->cols.c[k] = pr->p.col[k];
      } else {
        double* d = dalloc<double>(X, pr->n);
        HIPCHK(hipMemcpyAsync(d, pr->p.col[k], pr->n * sizeof(double), hipMemcpyHostToDevice, X.st));
        pr->dev_owned.push_back(d);
        pr->cols.c[k] = d;
      }
    }
  }
  host_wait(X);  // tables and copied columns are read below
}

// Root cells of every valid problem, grouping of equal root surfaces, one
// private list per (problem, sector), greedy dive, first task of the search.
template <int FAM, typename E, typename M>
void start_search(Run& X) {
  const ProbC& P = X.P0;
  X.ent_bytes = sizeof(E) + sizeof(M);
  const uint32_t np = (uint32_t)X.probs.size();
  const int nsec = P.nsec;
  std::vector<Cell> rc;
  for (uint32_t p = 0; p < np; p++) {
    if (X.probs[p]->st != GV_OK) continue;
    Cell c{};
    c.off = X.ooff[p];
    c.len = (uint32_t)X.probs[p]->n;
    c.prob = p;
    rc.push_back(c);
  }
  if (rc.empty()) return;
  bool unit = true;
  {
    Batch rb;
    rb.level = 0;
    rb.ncell = (uint32_t)rc.size();
    rb.nent = X.Ntot;
    rb.cells = dalloc<Cell>(X, rc.size());
    // (rc stays alive and is next written by a copy later on the same stream)
    HIPCHK(hipMemcpyAsync(rb.cells, rc.data(), rc.size() * sizeof(Cell), hipMemcpyHostToDevice, X.st));
    rb.ents = X.root;
    if (X.group_mode >= 0) group_batch<E>(X, rb, true);
    X.root = rb.ents;
    unit = rb.unit;
    HIPCHK(hipMemcpyAsync(rc.data(), rb.cells, rc.size() * sizeof(Cell), hipMemcpyDeviceToHost, X.st));
    host_wait(X);
    dfree(X, rb.cells);
  }
  // one list per (problem, sector): the pass masks are written per entry
  std::vector<Cell> cells;
  uint64_t tot = 0;
  for (const Cell& c : rc)
    for (int s = 0; s < nsec; s++) {
      Cell o = c;
      o.prefix = (uint64_t)s;
      o.sector = (uint32_t)s;
      o.off = tot;
      tot += c.len;
      cells.push_back(o);
    }
  E* ents = (E*)X.root;
  if (nsec > 1) {
    ents = dalloc<E>(X, tot);
    for (size_t i = 0; i < cells.size(); i++) {
      const Cell& src = rc[i / nsec];
      if (src.len)
        HIPCHK(hipMemcpyAsync(ents + cells[i].off, (E*)X.root + src.off, (size_t)src.len * sizeof(E),
                              hipMemcpyDeviceToDevice, X.st));
    }
    dfree(X, X.root);
  }
  X.root = nullptr;
  Cell* dcells = dalloc<Cell>(X, cells.size());
  HIPCHK(hipMemcpyAsync(dcells, cells.data(), cells.size() * sizeof(Cell), hipMemcpyHostToDevice, X.st));
  host_wait(X);
  // greedy dive in every cell: achieved leaf keys are valid starting bounds
  if (X.root_dive && !X.report) {
    Batch b;
    b.level = 0;
    b.ncell = (uint32_t)cells.size();
    b.nent = tot;
    b.unit = unit;
    b.cells = dalloc<Cell>(X, cells.size());
    HIPCHK(hipMemcpyAsync(b.cells, dcells, cells.size() * sizeof(Cell), hipMemcpyDeviceToDevice, X.st));
    b.ents = ents;
    bool own = false;
    while (true) {
      Parent* pa = expand_at<FAM, E, M>(X, b, own, true);
      if (!pa) break;
      pa->pending = 1;
      if (!materialize_at<FAM, E, M>(X, pa, 0, pa->nkept, b)) break;
      own = true;
    }
  }
  // diversified dive: every kept child (up to one chunk of the count order)
  // while the batch holds fewer than dive_cells cells, then the best child of
  // each cell down to a leaf.  Thousands of greedy paths from different
  // coarse cells find a strong bound early where the top-count coarse cells
  // are clutter; like the dive above it only changes bounds, never a result.
  // When the dive carried every kept child of its full levels, the batch at
  // which it goes greedy holds every cell of that level that any leaf can be
  // reached through (cut only against bounds): the main search starts there
  // instead of expanding the levels above it again.  The result cannot
  // change (the maximum leaf lies below one of these cells); measured:
  // pose4dof_1m 53 against 62 ms, eight pose problems of 1e5-1e6 matches
  // 8-14% faster, the 256-problem set 0.77 against 0.83 s.
  Batch reuse{};
  bool have_reuse = false;
  if (X.dive_cells > 0 && !X.report) {
    const bool beam = X.beam;
    Batch b;
    b.level = 0;
    b.ncell = (uint32_t)cells.size();
    b.nent = tot;
    b.unit = unit;
    b.cells = dalloc<Cell>(X, cells.size());
    HIPCHK(hipMemcpyAsync(b.cells, dcells, cells.size() * sizeof(Cell), hipMemcpyDeviceToDevice, X.st));
    b.ents = ents;
    bool own = false;
    bool carried = X.reuse && !X.root_dive && !X.fixed;
    while (true) {
      const bool dv = b.ncell >= X.dive_cells;
      bool keep = false;
      if (dv && carried && !have_reuse && b.level > 0) {
        // the greedy expansion below keeps this batch's entries (not owned)
        // and frees its own copy of the cell array
        reuse = b;
        reuse.cells = dalloc<Cell>(X, b.ncell);
        HIPCHK(hipMemcpyAsync(reuse.cells, b.cells, (size_t)b.ncell * sizeof(Cell), hipMemcpyDeviceToDevice, X.st));
        have_reuse = true;
        keep = true;
      }
      Parent* pa = expand_at<FAM, E, M>(X, b, keep ? false : own, dv);
      if (!pa) break;
      uint32_t r1 = pa->nkept;
      if (!dv) {
        if (one_chunk(X, pa)) {
          pa->fresh = true;
        } else {
          std::vector<std::pair<uint32_t, uint32_t>> ch;
          plan_chunks(X, pa, ch);
          r1 = ch.front().second;
        }
        if (r1 != pa->nkept) carried = false;
      }
      pa->pending = 1;
      if (!materialize_at<FAM, E, M>(X, pa, 0, r1, b)) break;
      own = true;
    }
    X.beam = beam;
  }
  Task t{};
  t.chunk = false;
  if (have_reuse) {
    t.b = reuse;
    dfree(X, dcells);
    dfree(X, ents);
  } else {
    t.b.level = 0;
    t.b.ncell = (uint32_t)cells.size();
    t.b.nent = tot;
    t.b.unit = unit;
    t.b.cells = dcells;
    t.b.ents = ents;
  }
  X.stack.push_back(t);
  X.own_first = true;
}

// Device search of a batch's small cells (k_subtree_pose); cells with longer
// lists come back as a batch of the same list buffer for the host-driven
// path.
template <int FAM, typename E>
void run_subtree(Run& X, Batch& b) {
  using M = typename SubFam<FAM>::M;
  const int nframes = X.P0.Lstar - b.level;
  // workgroups: up to four per CU, their frame buffers within an eighth of
  // the epoch's memory budget
  const uint64_t per_wg =
      (uint64_t)(nframes - 1) * GV_SUB_T * sizeof(E) + (uint64_t)nframes * GV_SUB_T * sizeof(M);
  const uint64_t fit = std::max<uint64_t>(1, X.budget / 8 / per_wg);
  const uint32_t G = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(b.ncell, (uint64_t)X.ctx->n_cu * 4u), fit);
  E* fbuf = dalloc<E>(X, (uint64_t)G * (uint64_t)(nframes - 1) * GV_SUB_T);
  M* mbuf = dalloc<M>(X, (uint64_t)G * (uint64_t)nframes * GV_SUB_T);
  Cell* over = dalloc<Cell>(X, b.ncell);
  uint32_t* ctr = dalloc<uint32_t>(X, 3);
  HIPCHK(hipMemsetAsync(ctr, 0, 3 * sizeof(uint32_t), X.st));
  k_subtree_pose<FAM, E><<<G, GV_SUB_WG, 0, X.st>>>(X.dP, b.level, b.cells, b.ncell, (const E*)b.ents, X.m64,
                                                     X.Ntot, X.dbest, X.drecheck, X.dtests, ctr, over, ctr + 1, fbuf,
                                                     mbuf, nframes);
  HIPCHK(hipGetLastError());
  uint32_t back[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(back, ctr + 1, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, X.st));
  host_wait(X);
  dfree(X, fbuf);
  dfree(X, mbuf);
  dfree(X, ctr);
  dfree(X, b.cells);
  X.stats.cells_expanded += b.ncell - back[0];
  if (X.trace)
    std::fprintf(stderr, "gv: level %d cells %u entries %llu searched on the device, %u cells back\n", b.level,
                 b.ncell, (unsigned long long)b.nent, back[0]);
  if (back[0] == 0) {
    dfree(X, over);
    dfree(X, b.ents);
    return;
  }
  Task t{};
  t.chunk = false;
  t.b = b;
  t.b.cells = over;
  t.b.ncell = back[0];
  t.b.nlive = back[1];
  X.stack.push_back(t);
}

template <int FAM, typename E>
bool subtree_at(Run& X, Batch& b) {
  if constexpr (!fam_pose(FAM)) {
    return false;
  } else {
    if (!X.subtree || X.report || b.level < X.subtree_from || b.level + 1 >= X.P0.Lstar) return false;
    if constexpr (std::is_same<E, EntQ32>::value) {
      if (b.unit && b.level >= 1 && X.q24) {
        run_subtree<FAM, EntQ24>(X, b);
        return true;
      }
    }
    run_subtree<FAM, E>(X, b);
    return true;
  }
}

// one expansion of the epoch's depth-first search; false when finished
template <int FAM, typename E, typename M>
bool epoch_step(Run& X) {
  if (X.stack.empty()) return false;
  Task t = X.stack.back();
  X.stack.pop_back();
  Batch b;
  if (t.chunk) {
    if (!materialize_at<FAM, E, M>(X, t.par, t.r0, t.r1, b)) return !X.stack.empty();
  } else {
    b = t.b;
  }
  // a batch that came back from the device search goes to the host path
  if (b.nlive == ~0ull && subtree_at<FAM, E>(X, b)) return !X.stack.empty();
  Parent* pa = expand_at<FAM, E, M>(X, b, true, false);
  if (pa) push_children<FAM, E, M>(X, pa, X.stack);
  return !X.stack.empty();
}

template <int FAM>
void build_linear(Run& X) {
  using E = typename EntOf<FAM>::T;
  const uint32_t np = (uint32_t)X.probs.size();
  E* root = dalloc<E>(X, X.Ntot);
  unsigned* dmax = dalloc<unsigned>(X, 2 * np);
  int* dbad = dalloc<int>(X, np);
  HIPCHK(hipMemsetAsync(dmax, 0, 2 * np * sizeof(unsigned), X.st));
  HIPCHK(hipMemsetAsync(dbad, 0, np * sizeof(int), X.st));
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    if (pr->n > 0)
      k_root_lin<FAM><<<gs_grid(X, pr->n), 256, 0, X.st>>>(X.dP + p, pr->cols, pr->n, root + X.ooff[p], dmax + 2 * p,
                                                           dbad + p);
  }
  std::vector<unsigned> mx(2 * np);
  std::vector<int> bad(np);
  HIPCHK(hipMemcpyAsync(mx.data(), dmax, 2 * np * sizeof(unsigned), hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipMemcpyAsync(bad.data(), dbad, np * sizeof(int), hipMemcpyDeviceToHost, X.st));
  host_wait(X);
  dfree(X, dmax);
  dfree(X, dbad);
  const ProbC& P = X.P0;
  double Hmax = 0, padmax = 0;
  for (int j = 0; j < X.probs[0]->S.d; j++) {
    Hmax = std::max(Hmax, (double)P.lev[0].H[j]);
    padmax = std::max(padmax, (double)P.lev[0].padu[j]);
  }
  const double npar = (FAM == FAM_PLANE3D || FAM == FAM_SIM2D) ? 2.0 : 1.0;
  unsigned mk_all = 0;
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    pr->maxK = mx[2 * p];
    pr->maxF = mx[2 * p + 1];
    if (bad[p] & 1) {
      pr->st = GV_EINVAL;
      pr->err = "non-finite observation or zero ray direction";
      continue;
    }
    // every intermediate of the integer test stays below 2^30
    const double Fb = std::max((double)pr->maxF, Hmax + padmax + npar * pr->maxK);
    if ((bad[p] & 2) || 2.0 * Fb + 2.0 * npar * pr->maxK + 2.0 * Hmax + padmax >= 1073741824.0) {
      pr->st = GV_ERANGE;
      pr->err = "lattice too fine for 32-bit cells";
      continue;
    }
    mk_all = std::max(mk_all, pr->maxK);
  }
  // canonical surfaces a cell of level m can hold: slopes shrink by 2 per
  // split of their parameter axis, heights span the cell plus its pads
  X.lat_bound[0] = 1e300;
  for (int m = 1; m <= P.Lstar; m++) {
    double D = (FAM == FAM_RAY3D) ? 3.0 : 1.0;
    const int nq = (FAM == FAM_RAY3D || FAM == FAM_SIM2D) ? 2 : 1;
    const int npp = (FAM == FAM_PLANE3D || FAM == FAM_SIM2D) ? 2 : 1;
    for (int qi = 0; qi < nq; qi++) {
      const int q = (FAM == FAM_LINE2D) ? 1 : (FAM == FAM_SIM2D ? 2 + qi : 2);
      double ks = 0.0, kprod = 1.0;
      for (int pi = 0; pi < npp; pi++) {
        const int pax = (FAM == FAM_PLANE3D || FAM == FAM_SIM2D) ? pi : 0;
        const double km = std::ceil((double)mk_all / std::ldexp(1.0, std::min(m, P.L[pax]))) + 1.0;
        ks += km;
        kprod *= 2.0 * km + 1.0;
      }
      const double Hm = std::ldexp(1.0, -std::min(m, P.L[q])) * P.inv_sf[q];
      D *= (Hm + (double)P.lev[m - 1].padu[q] + 4.0 * ks + 2.0) * kprod;
    }
    X.lat_bound[m] = D;
  }
  // first level from which every list value fits the packed entry: slopes
  // as above, heights within the cell plus its pads plus the slope spans
  uint64_t nmax = 0;
  for (ProbRec* pr : X.probs) nmax = std::max<uint64_t>(nmax, (uint64_t)pr->n);
  X.pack_from = 1 << 30;
  if (X.ctx->pack && (FAM == FAM_LINE2D || (FAM == FAM_PLANE3D && nmax <= GV_P3_WMAX))) {
    const int q = (FAM == FAM_LINE2D) ? 1 : 2;
    const double kmax = (FAM == FAM_LINE2D) ? GV_L2_MAX : GV_P3_KMAX;
    const double fmax = (FAM == FAM_LINE2D) ? GV_L2_MAX : GV_P3_FMAX;
    for (int m = P.Lstar - 1; m >= 1; m--) {
      double kb = 0.0, ks = 0.0;
      for (int pi = 0; pi < ((FAM == FAM_PLANE3D) ? 2 : 1); pi++) {
        const double km = std::ceil((double)mk_all / std::ldexp(1.0, std::min(m, P.L[pi]))) + 1.0;
        kb = std::max(kb, km);
        ks += km;
      }
      const double fb = (double)P.lev[m].H[q] + (double)P.lev[m - 1].padu[q] + 2.0 * ks + 4.0;
      if (kb > kmax || fb > fmax) break;
      X.pack_from = m;
    }
  }
  // PLANE3D: first level from which unit-weight lists fit one word (slopes
  // 8 bits, heights 16).  A one-word list that is to be grouped is widened to
  // the 8-byte entry first, so these levels lie within the packed ones.
  X.unit_from = 1 << 30;
  if (FAM == FAM_PLANE3D && X.ctx->pack) {
    for (int m = P.Lstar - 1; m >= std::max(1, X.pack_from); m--) {
      double kb = 0.0, ks = 0.0;
      for (int pi = 0; pi < 2; pi++) {
        const double km = std::ceil((double)mk_all / std::ldexp(1.0, std::min(m, P.L[pi]))) + 1.0;
        kb = std::max(kb, km);
        ks += km;
      }
      const double fb = (double)P.lev[m].H[2] + (double)P.lev[m - 1].padu[2] + 2.0 * ks + 4.0;
      if (kb > GV_P3U_KMAX || fb > GV_P3_FMAX) break;
      X.unit_from = m;
    }
  }
  X.root = root;
  if (!X.root_only) start_search<FAM, E, uint8_t>(X);
}

// exact mode of a linear family: root quantization, then the search over
// unchanged surfaces (pass masks, copying compaction)
template <int BF>
void build_exact(Run& X) {
  const uint32_t np = (uint32_t)X.probs.size();
  EntX* root = dalloc<EntX>(X, X.Ntot);
  int* dbad = dalloc<int>(X, np);
  HIPCHK(hipMemsetAsync(dbad, 0, np * sizeof(int), X.st));
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    if (pr->n > 0)
      k_root_x<BF><<<gs_grid(X, pr->n), 256, 0, X.st>>>(X.dP + p, pr->cols, pr->n, root + X.ooff[p], dbad + p);
  }
  std::vector<int> bad(np);
  HIPCHK(hipMemcpyAsync(bad.data(), dbad, np * sizeof(int), hipMemcpyDeviceToHost, X.st));
  host_wait(X);
  dfree(X, dbad);
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    if (bad[p] & 1) {
      pr->st = GV_EINVAL;
      pr->err = "non-finite observation or zero ray direction";
    } else if (bad[p] & 2) {
      pr->st = GV_ERANGE;
      pr->err = "surface parameters beyond the exact-mode range";
    }
  }
  X.root = root;
  // sixteen children when all four axes of the similarity family split
  using M = std::conditional_t<BF == FAM_SIM2D, uint16_t, uint8_t>;
  if (!X.root_only) start_search<BF + 8, EntX, M>(X);
}

template <typename E>
bool step_pose(Run& X) { return epoch_step<FAM_POSE4DOF, E, uint16_t>(X); }
template <typename E>
bool step_pose5(Run& X) { return epoch_step<FAM_POSE5DOF, E, uint32_t>(X); }

// returns true when the binary32 filter is used
bool build_pose(Run& X) {
  const uint32_t np = (uint32_t)X.probs.size();
  unsigned long long* dmx = dalloc<unsigned long long>(X, 8 * np);
  int* dbad = dalloc<int>(X, np);
  HIPCHK(hipMemsetAsync(dmx, 0, 8 * np * sizeof(unsigned long long), X.st));
  HIPCHK(hipMemsetAsync(dbad, 0, np * sizeof(int), X.st));
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    if (pr->n > 0)
      k_pose_bounds<<<gs_grid(X, pr->n), 256, 0, X.st>>>(X.dP + p, X.fam, pr->cols, pr->n, dmx + 8 * p, dbad + p);
  }
  std::vector<unsigned long long> mxb(8 * np);
  std::vector<int> bad(np);
  HIPCHK(hipMemcpyAsync(mxb.data(), dmx, mxb.size() * 8, hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipMemcpyAsync(bad.data(), dbad, np * sizeof(int), hipMemcpyDeviceToHost, X.st));
  host_wait(X);
  std::vector<ProbC> tab(np);
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    double H, R2, Xm;
    std::memcpy(&H, &mxb[8 * p], 8);
    std::memcpy(&R2, &mxb[8 * p + 1], 8);
    std::memcpy(&Xm, &mxb[8 * p + 7], 8);
    const bool arc_ok = pose_lattice(pr->S, H, R2, pr->epsk, Xm, &pr->p);
    if (bad[p] & 1) {
      pr->st = GV_EINVAL;
      pr->err = "non-finite observation";
    } else if (!arc_ok) {
      pr->st = GV_EINVAL;
      pr->err = "POSE5DOF: image coordinates times the f range too wide (2 atan(1 + 2 eps[3]) + atan(max|xi| hi[4]) "
                "must stay below 3.1)";
    }
    tab[p] = pr->S.P;
  }
  X.P0 = X.probs[0]->S.P;
  HIPCHK(hipMemcpyAsync(X.dP, tab.data(), np * sizeof(ProbC), hipMemcpyHostToDevice, X.st));
  X.m64 = dalloc<double>(X, X.Ntot * 5);
  EntQ32* e32 = dalloc<EntQ32>(X, X.Ntot);
  EntQ64* e64 = dalloc<EntQ64>(X, X.Ntot);
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    if (pr->n > 0 && pr->st == GV_OK)
      k_root_pose<<<gs_grid(X, pr->n), 256, 0, X.st>>>(X.dP + p, X.fam, pr->cols, pr->n, X.ooff[p], X.Ntot, X.m64,
                                                       e32, e64, dmx + 8 * p);
  }
  HIPCHK(hipMemcpyAsync(mxb.data(), dmx, mxb.size() * 8, hipMemcpyDeviceToHost, X.st));
  host_wait(X);
  dfree(X, dmx);
  dfree(X, dbad);
  bool all32 = true;
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    double mx[8];
    std::memcpy(mx, &mxb[8 * p], 64);
    pr->filter_ok = pr->p.precision == GV_FP32_FILTER &&
                    (pr->S.fam == GV_POSE4DOF ? pose_filter_exact(pr->S, mx) : pose5_filter_exact(pr->S, mx));
    if (pr->st == GV_OK && !pr->filter_ok) all32 = false;
  }
  // (grouping below the root is off for this family unless forced)
  X.q24 = X.ctx->pack && X.group_mode <= 0;
  if (X.fam == GV_POSE5DOF) {
    if (all32) {
      dfree(X, e64);
      X.root = e32;
      if (!X.root_only) start_search<FAM_POSE5DOF, EntQ32, uint32_t>(X);
    } else {
      dfree(X, e32);
      X.root = e64;
      if (!X.root_only) start_search<FAM_POSE5DOF, EntQ64, uint32_t>(X);
    }
    return all32;
  }
  if (all32) {
    dfree(X, e64);
    X.root = e32;
    if (!X.root_only) start_search<FAM_POSE4DOF, EntQ32, uint16_t>(X);
  } else {
    dfree(X, e32);
    X.root = e64;
    if (!X.root_only) start_search<FAM_POSE4DOF, EntQ64, uint16_t>(X);
  }
  return all32;
}

// per-problem winner, replay, inliers, point; releases the epoch's memory
void epoch_finish(Run& X) {
  const uint32_t np = (uint32_t)X.probs.size();
  const ProbC& P = X.P0;
  std::vector<unsigned long long> best(np);
  unsigned long long rech = 0;
  int ovf = 0;
  HIPCHK(hipMemcpyAsync(best.data(), X.dbest, np * 8, hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipMemcpyAsync(&rech, X.drecheck, 8, hipMemcpyDeviceToHost, X.st));
  HIPCHK(hipMemcpyAsync(&ovf, X.dovf, sizeof(int), hipMemcpyDeviceToHost, X.st));
  host_wait(X);
  if (ovf)
    for (ProbRec* pr : X.probs)
      if (pr->st == GV_OK) {
        pr->st = GV_ERANGE;
        pr->err = "internal: a lattice value outgrew its packed list entry";
      }
  std::vector<PathC> paths(np);
  std::vector<Cols> ctab(np);
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    ctab[p] = pr->cols;
    pr->count = best[p] >> P.B;
    pr->leaf = P.idxmask - (best[p] & P.idxmask);
    decode_leaf(P, pr->leaf, pr->path, pr->coords);
    paths[p] = pr->path;
  }
  PathC* dpaths = dalloc<PathC>(X, np);
  Cols* dctab = dalloc<Cols>(X, np);
  HIPCHK(hipMemcpyAsync(dpaths, paths.data(), np * sizeof(PathC), hipMemcpyHostToDevice, X.st));
  HIPCHK(hipMemcpyAsync(dctab, ctab.data(), np * sizeof(Cols), hipMemcpyHostToDevice, X.st));
  std::vector<uint64_t> bnd(np + 1, 0);
  std::vector<int64_t> all;
  if (X.Ntot > 0) {
    uint32_t* flag = dalloc<uint32_t>(X, X.Ntot);
    uint32_t* pos = dalloc<uint32_t>(X, X.Ntot + 1);
    int* dbad = dalloc<int>(X, 1);
    HIPCHK(hipMemsetAsync(dbad, 0, sizeof(int), X.st));
    const unsigned gg = gs_grid(X, X.Ntot);
    if (X.P0.exact && !fam_pose(X.fam)) {
      switch (X.fam) {
        case GV_LINE2D: k_replay_x<FAM_LINE2D><<<gg, 256, 0, X.st>>>(X.dP, dctab, X.dooff, np, X.Ntot, dpaths, flag, dbad); break;
        case GV_PLANE3D: k_replay_x<FAM_PLANE3D><<<gg, 256, 0, X.st>>>(X.dP, dctab, X.dooff, np, X.Ntot, dpaths, flag, dbad); break;
        case GV_SIM2D: k_replay_x<FAM_SIM2D><<<gg, 256, 0, X.st>>>(X.dP, dctab, X.dooff, np, X.Ntot, dpaths, flag, dbad); break;
        default: k_replay_x<FAM_RAY3D><<<gg, 256, 0, X.st>>>(X.dP, dctab, X.dooff, np, X.Ntot, dpaths, flag, dbad); break;
      }
    } else switch (X.fam) {
      case GV_LINE2D: k_replay_lin<FAM_LINE2D><<<gg, 256, 0, X.st>>>(X.dP, dctab, X.dooff, np, X.Ntot, dpaths, flag, dbad); break;
      case GV_PLANE3D: k_replay_lin<FAM_PLANE3D><<<gg, 256, 0, X.st>>>(X.dP, dctab, X.dooff, np, X.Ntot, dpaths, flag, dbad); break;
      case GV_RAY3D: k_replay_lin<FAM_RAY3D><<<gg, 256, 0, X.st>>>(X.dP, dctab, X.dooff, np, X.Ntot, dpaths, flag, dbad); break;
      case GV_SIM2D: k_replay_lin<FAM_SIM2D><<<gg, 256, 0, X.st>>>(X.dP, dctab, X.dooff, np, X.Ntot, dpaths, flag, dbad); break;
      case GV_POSE5DOF: k_replay_pose5<<<gg, 256, 0, X.st>>>(X.dP, X.m64, X.Ntot, X.dooff, np, dpaths, flag); break;
      default: k_replay_pose<<<gg, 256, 0, X.st>>>(X.dP, X.m64, X.Ntot, X.dooff, np, dpaths, flag); break;
    }
    HIPCHK(hipGetLastError());
    excl_scan(X, flag, pos, X.Ntot);
    uint32_t lastf = 0;
    HIPCHK(hipMemcpyAsync(&lastf, flag + X.Ntot - 1, 4, hipMemcpyDeviceToHost, X.st));
    std::vector<uint32_t> pb(np + 1);
    for (uint32_t p = 0; p < np; p++)
      HIPCHK(hipMemcpyAsync(&pb[p], pos + std::min<uint64_t>(X.ooff[p], X.Ntot - 1), 4, hipMemcpyDeviceToHost, X.st));
    HIPCHK(hipMemcpyAsync(&pb[np], pos + X.Ntot - 1, 4, hipMemcpyDeviceToHost, X.st));
    host_wait(X);
    pb[np] += lastf;
    for (uint32_t p = 0; p < np; p++)
      if (X.ooff[p] >= X.Ntot) pb[p] = pb[np];
    for (uint32_t p = 0; p <= np; p++) bnd[p] = pb[p];
    const uint64_t tot = bnd[np];
    if (tot > 0) {
      int64_t* dout = dalloc<int64_t>(X, tot);
      k_write_inliers<<<gg, 256, 0, X.st>>>(flag, pos, X.dooff, np, X.Ntot, dout);
      all.resize(tot);
      HIPCHK(hipMemcpyAsync(all.data(), dout, tot * sizeof(int64_t), hipMemcpyDeviceToHost, X.st));
      host_wait(X);
      dfree(X, dout);
    }
    dfree(X, flag);
    dfree(X, pos);
    dfree(X, dbad);
  }
  // kernel timing
  for (auto& e : X.ev) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e.e.first, e.e.second));
    if (X.ctx->kernel_timing) (e.kind == 0 ? X.stats.test_ms : X.stats.compact_ms) += (double)ms;
    if (e.cand >= 0) tune_sample(X, e.kind, e.cand, (double)ms, e.units);
    if (e.tcand >= 0) tune_sample(X, 2, e.tcand, (double)ms, e.units);
  }
  if (X.ctx->kernel_timing) X.stats.compact_bytes += d2h1(X, X.dreads) / 8;
  X.stats.fp64_rechecks = rech;
  X.stats.tests += d2h1(X, X.dtests);
  X.stats.levels = (uint32_t)P.Lstar;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - X.t0).count();
  X.stats.ms_total = ms;
  X.stats.ms_kernels = ms;
  if (X.trace)
    std::fprintf(stderr,
                 "gv: epoch of %u problems: %.3g tests, %llu cells expanded, %.1f ms, peak %.2f GB, %llu host waits "
                 "(%.1f ms)\n",
                 np, (double)X.stats.tests, (unsigned long long)X.stats.cells_expanded, ms,
                 (double)X.cache->peak * 1e-9, (unsigned long long)X.waits, X.wait_ms);
  for (uint32_t p = 0; p < np; p++) {
    ProbRec* pr = X.probs[p];
    pr->stats = X.stats;
    if (pr->st != GV_OK) continue;
    pr->inliers.assign(all.begin() + (int64_t)bnd[p], all.begin() + (int64_t)bnd[p + 1]);
    if ((uint64_t)pr->inliers.size() != pr->count) {
      pr->st = GV_EDEVICE;
      pr->err = "internal: replayed inlier count differs from the leaf count";
    }
  }
  dfree(X, dpaths);
  dfree(X, dctab);
}

// free everything an epoch may still hold (also after an error)
void epoch_release(Run& X) {
  (void)hipStreamSynchronize(X.st);
  while (!X.stack.empty()) {
    Task t = X.stack.back();
    X.stack.pop_back();
    if (t.chunk) {
      if (--t.par->pending == 0) free_parent(X, t.par);
    } else {
      dfree(X, t.b.cells);
      dfree(X, t.b.ents);
    }
  }
  dfree(X, X.root);
  X.root = nullptr;
  dfree(X, X.m64);
  X.m64 = nullptr;
  for (ProbRec* pr : X.probs) {
    for (void* q : pr->dev_owned) dfree(X, q);
    pr->dev_owned.clear();
  }
  dfree(X, X.dP);
  dfree(X, X.dbest);
  dfree(X, X.drecheck);
  dfree(X, X.dtests);
  X.dtests = nullptr;
  if (X.dtot != X.hpin_dev) dfree(X, X.dtot);
  dfree(X, X.dummy);
  dfree(X, X.dreads);
  dfree(X, X.dovf);
  dfree(X, X.dooff);
  X.dP = nullptr;
  X.dbest = nullptr;
  X.drecheck = nullptr;
  X.dtot = nullptr;
  X.dummy = nullptr;
  X.dreads = nullptr;
  X.dovf = nullptr;
  X.dooff = nullptr;
}

// build an epoch and return its step function
std::function<bool(Run&)> epoch_build(Run& X) {
  epoch_begin(X);
  if (X.P0.exact && !fam_pose(X.fam)) {
    switch (X.fam) {
      case GV_LINE2D: build_exact<FAM_LINE2D>(X); return epoch_step<FAM_XLINE2D, EntX, uint8_t>;
      case GV_PLANE3D: build_exact<FAM_PLANE3D>(X); return epoch_step<FAM_XPLANE3D, EntX, uint8_t>;
      case GV_SIM2D: build_exact<FAM_SIM2D>(X); return epoch_step<FAM_XSIM2D, EntX, uint16_t>;
      default: build_exact<FAM_RAY3D>(X); return epoch_step<FAM_XRAY3D, EntX, uint8_t>;
    }
  }
  switch (X.fam) {
    case GV_LINE2D: build_linear<FAM_LINE2D>(X); return epoch_step<FAM_LINE2D, EntL2, uint8_t>;
    case GV_PLANE3D: build_linear<FAM_PLANE3D>(X); return epoch_step<FAM_PLANE3D, EntP3, uint8_t>;
    case GV_RAY3D: build_linear<FAM_RAY3D>(X); return epoch_step<FAM_RAY3D, EntR3, uint8_t>;
    case GV_SIM2D: build_linear<FAM_SIM2D>(X); return epoch_step<FAM_SIM2D, EntS2, uint8_t>;
    case GV_POSE5DOF:
      if (build_pose(X)) return step_pose5<EntQ32>;
      return step_pose5<EntQ64>;
    default:
      if (build_pose(X)) return step_pose<EntQ32>;
      return step_pose<EntQ64>;
  }
}

void fill_result(const ProbRec* pr, gv_result* r) {
  const ProbC& P = pr->S.P;
  r->count = pr->count;
  r->leaf_index = pr->leaf;
  r->sector = pr->path.sector;
  for (int a = 0; a < GV_MAXD; a++) r->leaf_coords[a] = a < pr->S.d ? pr->coords[a] : 0;
  for (int j = 0; j < GV_MAXD; j++) r->point[j] = 0.0;
  for (int j = 0; j < pr->S.d; j++) {
    double u = (double)(2 * pr->coords[j] + 1) * std::ldexp(1.0, -(P.L[j] + 1));
    r->point[j] = P.lo[j] + P.E[j] * u;
  }
  if (fam_pose(pr->S.fam)) {
    double yaw = (double)pr->path.sector * (M_PI / 2.0) + std::atan(r->point[3]);
    if (yaw < 0.0) yaw += 2.0 * M_PI;
    if (yaw >= 2.0 * M_PI) yaw -= 2.0 * M_PI;
    r->point[3] = yaw;
  }
  // Certified bound per axis (the approximation guarantee of Sec. 3.2):
  // on an axis a surface depends on, every reported inlier's range over the
  // leaf's parameter box comes within bound[q] of the leaf's q-interval (the
  // canonical surface of the last level passes within its pad, and differs
  // from the original by at most the canonization allowance); on a pure
  // parameter axis, half the leaf side (the distance from the returned point
  // to any point of the leaf).
  const double h37 = 0x1p-37;
  for (int j = 0; j < GV_MAXD; j++) r->bound[j] = 0.0;
  for (int j = 0; j < pr->S.d; j++) r->bound[j] = 0.5 * std::ldexp(P.E[j], -P.L[j]);
  if (fam_pose(pr->S.fam)) {
    if (pr->S.exact) {
      // 2^-37 per parameter: z moves by at most (1 + R + 2 H) 2^-37, kappa
      // by (1 + k^2)(1 + 2/R_g) 2^-37 with |k| <= 1 + pad
      const double R = std::sqrt(pr->S.R2), kk = 1.0 + P.padk;
      r->bound[2] = (P.padz + (1.0 + R + 2.0 * pr->S.Hmax) * h37) * P.E[2];
      r->bound[3] = P.padk + (1.0 + kk * kk) * (1.0 + 2.0 / std::sqrt(P.Rg2)) * h37;
    } else {
      r->bound[2] = (P.padz + pr->S.ez * 0.5) * P.E[2];
      // kappa units; also a yaw bound in radians, as |d yaw / d kappa| <= 1.
      // Holds where the leaf is farther than the apex guard from the match.
      r->bound[3] = P.padk + pr->S.ek * 0.5;
    }
  } else {
    const int npar = pr->S.fam == GV_PLANE3D ? 2 : 1;
    for (int q = 0; q < pr->S.d; q++) {
      const bool dep = pr->S.fam == GV_RAY3D || (pr->S.fam == GV_SIM2D ? q >= 2 : q == pr->S.d - 1);
      if (!dep) continue;
      double b;
      if (pr->S.exact) {
        b = P.xpad[q] + (double)(npar + 1) * h37;
      } else {
        const int m = P.Lstar - 1;
        const double Em = (double)((m + 1) * (pr->S.ell + 1)) * P.sf[q] * 0.5;
        b = 0.5 * (double)P.lev[m].padu[q] * P.sf[q] + Em;
      }
      r->bound[q] = b * P.E[q];
    }
  }
  r->stats = pr->stats;
  r->stats.ms_queued = pr->ms_queued;
  r->n_inliers = pr->inliers.size();
}

// copy the inliers out; GV_EBUFSZ (with n_inliers set) if they do not fit
gv_status deliver(const ProbRec* pr, gv_result* r) {
  fill_result(pr, r);
  if (pr->inliers.size() > r->inliers_cap || (!r->inliers && !pr->inliers.empty())) return GV_EBUFSZ;
  if (!pr->inliers.empty()) std::memcpy(r->inliers, pr->inliers.data(), pr->inliers.size() * sizeof(int64_t));
  return GV_OK;
}

// run an epoch to completion on the calling thread (ctx->mu held)
void run_epoch(gv_ctx* ctx, std::vector<ProbRec*>& probs) {
  Run X;
  bind_ctx(X, ctx);
  X.probs = probs;
  try {
    auto step = epoch_build(X);
    while (step(X)) {
    }
    epoch_finish(X);
  } catch (DevErr& e) {
    fail_all(X, e.st);
  }
  epoch_release(X);
}

// ===========================================================================
// Continuous batching: lanes (host thread + HIP stream + allocator each) take
// queued problems as memory allows and run them as epochs, so requests that
// arrive while others are on the device start as soon as a lane frees up and
// their work overlaps the others' on the GPU.
// ===========================================================================
struct Lane {
  gv_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  DevCache cache;
  uint64_t* hpin = nullptr;
  uint64_t* hpin_dev = nullptr;
  std::vector<hipEvent_t> ev_pool;
  std::string err;
  std::thread th;
};

void publish(gv_ctx* ctx, std::vector<ProbRec*>& probs) {
  std::lock_guard<std::mutex> g(ctx->qmu);
  for (ProbRec* pr : probs) {
    pr->done = true;
    ctx->inflight -= std::min(ctx->inflight, pr->est_bytes);
  }
  ctx->running--;
  ctx->cv_done.notify_all();
  ctx->cv_work.notify_all();  // memory was released: a waiting lane may admit now
}

void lane_main(Lane* L) {
  gv_ctx* ctx = L->ctx;
  (void)hipSetDevice(ctx->device);
  while (true) {
    std::vector<ProbRec*> admit;
    {
      std::unique_lock<std::mutex> lk(ctx->qmu);
      while (true) {
        if (ctx->stop && ctx->queue.empty()) return;
        if (!ctx->queue.empty()) {
          ProbRec* first = nullptr;
          uint64_t nsum = 0;
          for (auto it = ctx->queue.begin(); it != ctx->queue.end() && admit.size() < ctx->max_batch;) {
            ProbRec* pr = *it;
            if (pr->canceled) {
              it = ctx->queue.erase(it);
              pr->done = true;
              continue;
            }
            if (!first) first = pr;
            // a problem is admitted when its estimate fits in half the budget
            // next to the running ones (or nothing else runs); small ones may
            // share an epoch up to batch_n observations
            const bool fits =
                ctx->inflight + pr->est_bytes <= ctx->budget / 2 || (ctx->running == 0 && admit.empty());
            const bool small = admit.empty() || nsum + (uint64_t)pr->n <= ctx->batch_n;
            if (!small || !fits) break;
            if (same_structure(first, pr)) {
              pr->ms_queued =
                  std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - pr->t_submit).count();
              admit.push_back(pr);
              nsum += (uint64_t)pr->n;
              ctx->inflight += pr->est_bytes;
              it = ctx->queue.erase(it);
            } else {
              ++it;
            }
          }
          ctx->cv_done.notify_all();
        }
        if (!admit.empty()) {
          ctx->running++;
          break;
        }
        if (ctx->stop && ctx->queue.empty()) return;
        ctx->cv_work.wait(lk);
      }
    }
    Run X;
    X.ctx = ctx;
    X.st = L->st;
    X.cache = &L->cache;
    X.ev_pool = &L->ev_pool;
    X.hpin = L->hpin;
    X.hpin_dev = L->hpin_dev;
    X.err = &L->err;
    // lanes share the device: smaller chunks keep their allocations small
    // and their latency steady (measured: 8 GB chunks per lane raised the
    // p50 latency under Poisson arrivals from 31 ms to 1.5 s)
    X.budget = ctx->budget / (uint64_t)(3 * std::max(1, ctx->nlanes));
    X.probs = admit;
    L->err.clear();
    try {
      auto step = epoch_build(X);
      bool dropped = false;
      while (step(X)) {
        // a running epoch stops at its next expansion once every problem in
        // it has been cancelled
        std::lock_guard<std::mutex> g(ctx->qmu);
        dropped = std::all_of(admit.begin(), admit.end(), [](const ProbRec* pr) { return pr->canceled; });
        if (dropped) break;
      }
      if (dropped) fail_all(X, GV_ECANCELED);
      else epoch_finish(X);
    } catch (DevErr& e) {
      fail_all(X, e.st);
    }
    epoch_release(X);
    // keep this lane's share of cached blocks bounded
    if (L->cache.cached > ctx->budget / (uint64_t)(2 * std::max(1, ctx->nlanes)))
      L->cache.release_to(ctx->budget / (uint64_t)(4 * std::max(1, ctx->nlanes)), L->st);
    publish(ctx, admit);
  }
}

void start_lanes(gv_ctx* ctx) {
  for (int i = 0; i < ctx->nlanes; i++) {
    Lane* L = new Lane();
    L->ctx = ctx;
    (void)hipSetDevice(ctx->device);
    if (hipStreamCreateWithFlags(&L->st, hipStreamNonBlocking) != hipSuccess) {
      delete L;
      break;
    }
    alloc_hpin(L->hpin, L->hpin_dev);
    L->th = std::thread(lane_main, L);
    ctx->lanes.push_back(L);
  }
}

void stop_lanes(gv_ctx* ctx) {
  for (Lane* L : ctx->lanes)
    if (L->th.joinable()) L->th.join();
  for (Lane* L : ctx->lanes) {
    (void)hipStreamSynchronize(L->st);
    L->cache.trim(L->st);
    for (auto& kv : L->cache.live) (void)hipFree(kv.first);
    for (hipEvent_t e : L->ev_pool) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(L->st);
    free_hpin(L->hpin, L->hpin_dev);
    delete L;
  }
  ctx->lanes.clear();
}

}  // namespace gvi

using namespace gvi;

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
  std::lock_guard<std::mutex> g(ctx->emu);
  tl_err = ctx->last_err;
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
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    for (char& ch : c->arch)
      if (ch == ' ') ch = '_';
  }
  if (c->arch.empty()) c->arch = "unknown";
  if (c->device >= 0 && c->device < kMaxDevices) {
    // the scratch region's address on this device (device current)
    ScratchSlot& S = g_scratch[c->device];
    std::lock_guard<std::mutex> g(S.mu);
    if (!S.init) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e == hipSuccess && ptr) {
        S.ptr = ptr;
      } else {
        (void)hipGetLastError();
        S.err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      }
      S.init = true;
    }
  }
  if (cfg && cfg->autotune_cache) c->tune_path = cfg->autotune_cache;
  if (const char* e = std::getenv("GV_AUTOTUNE")) c->autotune = atoi(e) != 0;
  if (const char* e = std::getenv("GV_TUNE_MIN_BYTES")) c->tune_min = std::strtoull(e, nullptr, 10);
  tune_load(c);
  if (cfg && cfg->hip_stream) {
    c->stream = (hipStream_t)cfg->hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return GV_EDEVICE;
    }
    c->own_stream = true;
  }
  alloc_hpin(c->hpin, c->hpin_dev);
  size_t fr = 0, tot = 0;
  (void)hipMemGetInfo(&fr, &tot);
  c->budget = (cfg && cfg->mem_budget_bytes) ? cfg->mem_budget_bytes : (uint64_t)(0.6 * (double)fr);
  if (const char* e = std::getenv("GV_LANES")) c->nlanes = std::max(1, std::min(16, atoi(e)));
  if (const char* e = std::getenv("GV_MAX_BATCH")) c->max_batch = (size_t)std::max(1, atoi(e));
  if (const char* e = std::getenv("GV_BATCH_N")) c->batch_n = std::strtoull(e, nullptr, 10);
  if (const char* e = std::getenv("GV_PACK")) c->pack = atoi(e) != 0;
  *out = c;
  return GV_OK;
}

gv_status gv_destroy(gv_ctx* ctx) {
  if (!ctx) return GV_EINVAL;
  {
    std::lock_guard<std::mutex> g(ctx->qmu);
    ctx->stop = true;
    for (ProbRec* pr : ctx->queue) pr->canceled = true;
  }
  ctx->cv_work.notify_all();
  stop_lanes(ctx);
  for (auto& kv : ctx->tickets) delete kv.second;
  ctx->tickets.clear();
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->cache.trim(ctx->stream);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto& kv : ctx->cache.live) (void)hipFree(kv.first);
  ctx->cache.live.clear();
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  free_hpin(ctx->hpin, ctx->hpin_dev);
  delete ctx;
  return GV_OK;
}

static void set_err(gv_ctx* ctx, const std::string& e) {
  std::lock_guard<std::mutex> g(ctx->emu);
  ctx->last_err = e;
}

gv_status gv_solve(gv_ctx* ctx, const gv_problem* p, gv_result* r) {
  if (!ctx || !p || !r) return GV_EINVAL;
  std::memset(&r->stats, 0, sizeof(r->stats));
  ProbRec pr;
  pr.p = *p;
  gv_status st = prepare_problem(&pr);
  if (st != GV_OK) {
    set_err(ctx, pr.err);
    return st;
  }
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->err.clear();
    std::vector<ProbRec*> v{&pr};
    run_epoch(ctx, v);
    // bounded cache: many problems of different sizes would otherwise fill
    // the device with idle blocks, and then free them all at once
    if (ctx->cache.cached > ctx->budget / 2) ctx->cache.release_to(ctx->budget / 4, ctx->stream);
  }
  if (pr.st != GV_OK) {
    set_err(ctx, pr.err.empty() ? ctx->err : pr.err);
    return pr.st;
  }
  set_err(ctx, "");
  return deliver(&pr, r);
}

gv_status gv_report(gv_ctx* ctx, const gv_problem* p, uint64_t tau, uint64_t* leaves, uint32_t* counts,
                    uint64_t cap, uint64_t* n_out, gv_stats* stats_out) {
  if (!ctx || !p || !n_out || (cap > 0 && (!leaves || !counts))) return GV_EINVAL;
  *n_out = 0;
  ProbRec pr;
  pr.p = *p;
  gv_status st = prepare_problem(&pr);
  if (st != GV_OK) {
    set_err(ctx, pr.err);
    return st;
  }
  if (tau < 1 || pr.S.P.B >= 63 || tau >= (1ull << (63 - pr.S.P.B))) {
    set_err(ctx, "tau must be at least 1 and fit the key");
    return GV_EINVAL;
  }
  uint64_t total = 0;
  std::vector<std::pair<uint64_t, uint32_t>> found;
  gv_stats stats{};
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->err.clear();
    Run X;
    bind_ctx(X, ctx);
    X.probs = {&pr};
    X.report = true;
    X.tau = tau;
    X.rep_cap = cap;
    try {
      X.rep_idx = dalloc<uint64_t>(X, std::max<uint64_t>(1, cap));
      X.rep_cnt = dalloc<uint32_t>(X, std::max<uint64_t>(1, cap));
      X.rep_n = dalloc<unsigned long long>(X, 1);
      HIPCHK(hipMemsetAsync(X.rep_n, 0, 8, X.st));
      auto step = epoch_build(X);
      while (step(X)) {
      }
      unsigned long long nn = 0;
      HIPCHK(hipMemcpyAsync(&nn, X.rep_n, 8, hipMemcpyDeviceToHost, X.st));
      host_wait(X);
      total = nn;
      const uint64_t k = std::min<uint64_t>(nn, cap);
      if (k > 0) {
        std::vector<uint64_t> hi(k);
        std::vector<uint32_t> hc(k);
        HIPCHK(hipMemcpyAsync(hi.data(), X.rep_idx, k * 8, hipMemcpyDeviceToHost, X.st));
        HIPCHK(hipMemcpyAsync(hc.data(), X.rep_cnt, k * 4, hipMemcpyDeviceToHost, X.st));
        host_wait(X);
        found.resize(k);
        for (uint64_t i = 0; i < k; i++) found[i] = {hi[i], hc[i]};
        std::sort(found.begin(), found.end());
      }
      X.stats.levels = (uint32_t)X.P0.Lstar;
      X.stats.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - X.t0).count();
      stats = X.stats;
    } catch (DevErr& e) {
      fail_all(X, e.st);
    }
    dfree(X, X.rep_idx);
    dfree(X, X.rep_cnt);
    dfree(X, X.rep_n);
    epoch_release(X);
  }
  if (stats_out) *stats_out = stats;
  if (pr.st != GV_OK) {
    set_err(ctx, pr.err.empty() ? ctx->err : pr.err);
    return pr.st;
  }
  *n_out = total;
  if (total > cap) {
    set_err(ctx, "more leaves reach tau than the output holds");
    return GV_EBUFSZ;
  }
  for (size_t i = 0; i < found.size(); i++) {
    leaves[i] = found[i].first;
    counts[i] = found[i].second;
  }
  set_err(ctx, "");
  return GV_OK;
}

gv_status gv_solve_noalloc(gv_ctx* ctx, const gv_problem* p, gv_result* r) {
  if (!ctx || !p || !r) return GV_EINVAL;
  std::memset(&r->stats, 0, sizeof(r->stats));
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return GV_EINVAL;
  ProbRec pr;
  pr.p = *p;
  gv_status st = prepare_problem(&pr);
  if (st != GV_OK) {
    set_err(ctx, pr.err);
    return st;
  }
  if (pr.n > kNoAllocMaxN) {
    set_err(ctx, "more observations than the allocation-free solve takes (2^19)");
    return GV_ETOOBIG;
  }
  ScratchSlot& S = g_scratch[ctx->device];
  std::lock_guard<std::mutex> gs(S.mu);
  if (!S.ptr) {
    set_err(ctx, S.err.empty() ? "scratch region unavailable" : S.err);
    return GV_EDEVICE;
  }
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->err.clear();
    // a fresh free list over the whole region: blocks hold the previous
    // call's contents, and every buffer the search reads is written (or
    // cleared) before it is read, as with reused blocks of the caching
    // allocator
    S.arena.arena_reset((char*)S.ptr, kScratchBytes);
    Run X;
    bind_ctx(X, ctx);
    X.cache = &S.arena;
    X.fixed = true;
    X.budget = kScratchBytes / 2;
    X.probs = {&pr};
    try {
      auto step = epoch_build(X);
      while (step(X)) {
      }
      epoch_finish(X);
    } catch (DevErr& e) {
      fail_all(X, e.st == GV_ENOMEM ? GV_ETOOBIG : e.st);
    }
    epoch_release(X);
  }
  if (pr.st != GV_OK) {
    set_err(ctx, pr.err.empty() ? ctx->err : pr.err);
    return pr.st;
  }
  set_err(ctx, "");
  return deliver(&pr, r);
}

gv_status gv_submit(gv_ctx* ctx, const gv_problem* p, uint64_t* ticket) {
  if (!ctx || !p || !ticket) return GV_EINVAL;
  ProbRec* pr = new (std::nothrow) ProbRec();
  if (!pr) return GV_ENOMEM;
  pr->p = *p;
  gv_status st = prepare_problem(pr);
  if (st != GV_OK) {
    set_err(ctx, pr->err);
    delete pr;
    return st;
  }
  if (pr->est_bytes > ctx->budget) {
    set_err(ctx, "problem exceeds the memory budget");
    delete pr;
    return GV_ETOOBIG;
  }
  if (!p->cols_on_device && p->n > 0) {
    // host columns are borrowed only for this call
    const int nc = ncols_of(pr->S.fam, pr->S.d);
    for (int k = 0; k < nc; k++) {
      pr->host_cols[k].assign(p->col[k], p->col[k] + p->n);
      pr->p.col[k] = pr->host_cols[k].data();
    }
  }
  std::lock_guard<std::mutex> g(ctx->qmu);
  pr->t_submit = std::chrono::steady_clock::now();
  pr->ticket = ctx->next_ticket++;
  ctx->tickets[pr->ticket] = pr;
  ctx->queue.push_back(pr);
  if (ctx->lanes.empty()) start_lanes(ctx);
  if (ctx->lanes.empty()) {
    ctx->tickets.erase(pr->ticket);
    ctx->queue.pop_back();
    delete pr;
    set_err(ctx, "could not create a serving stream");
    return GV_EDEVICE;
  }
  ctx->cv_work.notify_one();
  *ticket = pr->ticket;
  return GV_OK;
}

gv_status gv_poll(gv_ctx* ctx, uint64_t ticket, gv_result* r, int timeout_ms) {
  if (!ctx || !r) return GV_EINVAL;
  std::unique_lock<std::mutex> lk(ctx->qmu);
  auto it = ctx->tickets.find(ticket);
  if (it == ctx->tickets.end()) return GV_EINVAL;
  ProbRec* pr = it->second;
  if (!pr->done) {
    if (timeout_ms == 0) return GV_EAGAIN;
    auto pred = [&] { return pr->done; };
    if (timeout_ms < 0) ctx->cv_done.wait(lk, pred);
    else if (!ctx->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) return GV_ETIMEDOUT;
  }
  if (pr->canceled) {
    ctx->tickets.erase(it);
    delete pr;
    return GV_ECANCELED;
  }
  if (pr->st != GV_OK) {
    gv_status st = pr->st;
    std::string e = pr->err;
    ctx->tickets.erase(it);
    delete pr;
    lk.unlock();
    set_err(ctx, e);
    return st;
  }
  gv_status st = deliver(pr, r);
  if (st == GV_OK) {
    ctx->tickets.erase(it);
    delete pr;
  }
  return st;
}

gv_status gv_cancel(gv_ctx* ctx, uint64_t ticket) {
  if (!ctx) return GV_EINVAL;
  std::lock_guard<std::mutex> g(ctx->qmu);
  auto it = ctx->tickets.find(ticket);
  if (it == ctx->tickets.end()) return GV_EINVAL;
  ProbRec* pr = it->second;
  pr->canceled = true;
  auto q = std::find(ctx->queue.begin(), ctx->queue.end(), pr);
  if (q != ctx->queue.end()) {
    ctx->queue.erase(q);
    pr->done = true;
    ctx->cv_done.notify_all();
  }
  return GV_OK;
}

gv_status gv_incidence(gv_ctx* ctx, const gv_problem* p, int32_t level, int32_t sector, const int32_t* coords,
                       uint32_t* masks_out, gv_stats* stats_out) {
  if (!ctx || !p || !coords || (!masks_out && p->n > 0)) return GV_EINVAL;
  ProbRec pr;
  pr.p = *p;
  gv_status st = prepare_problem(&pr);
  if (st != GV_OK) {
    set_err(ctx, pr.err);
    return st;
  }
  const ProbC& P = pr.S.P;
  if (level < 0 || level >= P.Lstar || sector < 0 || sector >= P.nsec) {
    set_err(ctx, "level or sector out of range");
    return GV_EINVAL;
  }
  for (int j = 0; j < GV_MAXD; j++) {
    const int bits = j < P.d ? std::min(level, P.L[j]) : 0;
    if (coords[j] < 0 || (int64_t)coords[j] >= (1ll << bits)) {
      set_err(ctx, "cell coordinates out of range");
      return GV_EINVAL;
    }
  }
  // the path's child digits: split axes' bits in axis order, MSB first
  PathC path{};
  path.sector = sector;
  for (int k = 0; k < level; k++) {
    uint32_t dg = 0;
    for (int j = 0; j < P.d; j++)
      if (k < P.L[j]) dg = (dg << 1) | (uint32_t)((coords[j] >> (std::min(level, P.L[j]) - 1 - k)) & 1);
    path.digit[k] = (uint8_t)dg;
  }
  Cell C{};
  for (int j = 0; j < GV_MAXD; j++) C.c[j] = coords[j];
  C.sector = (uint32_t)sector;
  const uint32_t nch = 1u << P.lev[level].abits;
  gv_stats stats{};
  stats.levels = (uint32_t)P.Lstar;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->err.clear();
    Run X;
    bind_ctx(X, ctx);
    X.probs = {&pr};
    X.root_only = true;
    try {
      epoch_begin(X);
      bool f32 = false;
      if (fam_pose(pr.S.fam)) {
        f32 = build_pose(X);
      } else if (pr.S.exact) {
        switch (pr.S.fam) {
          case GV_LINE2D: build_exact<FAM_LINE2D>(X); break;
          case GV_PLANE3D: build_exact<FAM_PLANE3D>(X); break;
          case GV_SIM2D: build_exact<FAM_SIM2D>(X); break;
          default: build_exact<FAM_RAY3D>(X); break;
        }
      } else {
        switch (pr.S.fam) {
          case GV_LINE2D: build_linear<FAM_LINE2D>(X); break;
          case GV_PLANE3D: build_linear<FAM_PLANE3D>(X); break;
          case GV_SIM2D: build_linear<FAM_SIM2D>(X); break;
          default: build_linear<FAM_RAY3D>(X); break;
        }
      }
      if (pr.st == GV_OK && pr.n > 0) {
        uint32_t* dm = dalloc<uint32_t>(X, (uint64_t)pr.n);
        const unsigned gg = gs_grid(X, (uint64_t)pr.n);
        if (pr.S.fam == GV_POSE5DOF) {
          if (f32)
            k_incidence_pose5<EntQ32><<<gg, 256, 0, X.st>>>(X.dP, (const EntQ32*)X.root, pr.n, X.m64, X.Ntot, C,
                                                           level, dm, X.drecheck);
          else
            k_incidence_pose5<EntQ64><<<gg, 256, 0, X.st>>>(X.dP, (const EntQ64*)X.root, pr.n, X.m64, X.Ntot, C,
                                                           level, dm, X.drecheck);
        } else if (pr.S.fam == GV_POSE4DOF) {
          if (f32)
            k_incidence_pose<EntQ32><<<gg, 256, 0, X.st>>>(X.dP, (const EntQ32*)X.root, pr.n, X.m64, X.Ntot, C, level,
                                                          dm, X.drecheck);
          else
            k_incidence_pose<EntQ64><<<gg, 256, 0, X.st>>>(X.dP, (const EntQ64*)X.root, pr.n, X.m64, X.Ntot, C, level,
                                                          dm, X.drecheck);
        } else if (pr.S.exact) {
          switch (pr.S.fam) {
            case GV_LINE2D: k_incidence_x<FAM_LINE2D><<<gg, 256, 0, X.st>>>(X.dP, (const EntX*)X.root, pr.n, C, level, dm); break;
            case GV_PLANE3D: k_incidence_x<FAM_PLANE3D><<<gg, 256, 0, X.st>>>(X.dP, (const EntX*)X.root, pr.n, C, level, dm); break;
            case GV_SIM2D: k_incidence_x<FAM_SIM2D><<<gg, 256, 0, X.st>>>(X.dP, (const EntX*)X.root, pr.n, C, level, dm); break;
            default: k_incidence_x<FAM_RAY3D><<<gg, 256, 0, X.st>>>(X.dP, (const EntX*)X.root, pr.n, C, level, dm); break;
          }
        } else {
#define GV_INC(F, N) \
  k_incidence_lin<F, typename EntOf<F>::T, N><<<gg, 256, 0, X.st>>>(X.dP, (const typename EntOf<F>::T*)X.root, pr.n, path, level, dm)
          switch (pr.S.fam == GV_SIM2D ? pr.S.fam * 32 + (int)nch : pr.S.fam * 16 + (int)nch) {
            case GV_LINE2D * 16 + 2: GV_INC(FAM_LINE2D, 2); break;
            case GV_LINE2D * 16 + 4: GV_INC(FAM_LINE2D, 4); break;
            case GV_PLANE3D * 16 + 2: GV_INC(FAM_PLANE3D, 2); break;
            case GV_PLANE3D * 16 + 4: GV_INC(FAM_PLANE3D, 4); break;
            case GV_PLANE3D * 16 + 8: GV_INC(FAM_PLANE3D, 8); break;
            case GV_RAY3D * 16 + 2: GV_INC(FAM_RAY3D, 2); break;
            case GV_RAY3D * 16 + 4: GV_INC(FAM_RAY3D, 4); break;
            case GV_RAY3D * 16 + 8: GV_INC(FAM_RAY3D, 8); break;
            case GV_SIM2D * 32 + 2: GV_INC(FAM_SIM2D, 2); break;
            case GV_SIM2D * 32 + 4: GV_INC(FAM_SIM2D, 4); break;
            case GV_SIM2D * 32 + 8: GV_INC(FAM_SIM2D, 8); break;
            case GV_SIM2D * 32 + 16: GV_INC(FAM_SIM2D, 16); break;
            default: throw DevErr{GV_EINVAL};
          }
#undef GV_INC
        }
        HIPCHK(hipGetLastError());
        unsigned long long rech = 0;
        HIPCHK(hipMemcpyAsync(masks_out, dm, (size_t)pr.n * sizeof(uint32_t), hipMemcpyDeviceToHost, X.st));
        HIPCHK(hipMemcpyAsync(&rech, X.drecheck, 8, hipMemcpyDeviceToHost, X.st));
        host_wait(X);
        dfree(X, dm);
        stats.tests = (uint64_t)pr.n * nch;
        stats.fp64_rechecks = rech;
      }
    } catch (DevErr& e) {
      fail_all(X, e.st);
    }
    epoch_release(X);
  }
  if (stats_out) *stats_out = stats;
  if (pr.st != GV_OK) {
    set_err(ctx, pr.err.empty() ? ctx->err : pr.err);
    return pr.st;
  }
  set_err(ctx, "");
  return GV_OK;
}

gv_status gv_parametrize(gv_ctx* ctx, const gv_problem* p, double* t_out, double* f_out, int32_t* tag_out) {
  if (!ctx || !p || (!t_out && p->n > 0) || (!f_out && p->n > 0)) return GV_EINVAL;
  ProbRec pr;
  pr.p = *p;
  std::string why;
  gv_status st = setup_axes(p, pr.S, why);
  if (st != GV_OK && st != GV_ERANGE) {
    set_err(ctx, why);
    return st;
  }
  std::lock_guard<std::mutex> g(ctx->mu);
  Run X;
  bind_ctx(X, ctx);
  st = GV_OK;
  std::vector<void*> owned;
  try {
    HIPCHK(hipSetDevice(ctx->device));
    X.dP = dalloc<ProbC>(X, 1);
    HIPCHK(hipMemcpyAsync(X.dP, &pr.S.P, sizeof(ProbC), hipMemcpyHostToDevice, X.st));
    const int ncol = ncols_of(pr.S.fam, pr.S.d);
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
      host_wait(X);
      dfree(X, t);
      dfree(X, f);
      dfree(X, tg);
      dfree(X, bad);
      if (hb) {
        set_err(ctx, "non-finite observation or zero ray direction");
        st = GV_EINVAL;
      }
    }
  } catch (DevErr& e) {
    st = e.st;
  }
  for (void* q : owned) dfree(X, q);
  dfree(X, X.dP);
  (void)hipStreamSynchronize(X.st);
  return st;
}

gv_status gv_refine(gv_ctx* ctx, const gv_problem* p, uint64_t leaf_index, const int64_t* idx, uint64_t n_idx,
                    double tau0, double tau, int32_t rounds, int32_t iters, gv_refined* out) {
  if (!ctx || !p || !out || (!idx && n_idx > 0)) return GV_EINVAL;
  ProbRec pr;
  pr.p = *p;
  gv_status st = prepare_problem(&pr);
  if (st != GV_OK) {
    set_err(ctx, pr.err);
    return st;
  }
  const ProbC& P = pr.S.P;
  if (!fam_pose(pr.S.fam)) {
    set_err(ctx, "gv_refine: pose families only");
    return GV_EINVAL;
  }
  if (!(tau > 0.0 && tau < 1.5) || !(tau0 > 0.0 && tau0 < 1.5) || rounds < 0 || iters < 0 || rounds > 64 ||
      iters > 256) {
    set_err(ctx, "gv_refine: tau, tau0 in (0, 1.5), 0 <= rounds <= 64, 0 <= iters <= 256");
    return GV_EINVAL;
  }
  if (leaf_index > P.idxmask) {
    set_err(ctx, "gv_refine: leaf index out of range");
    return GV_EINVAL;
  }
  for (uint64_t k = 0; k < n_idx; k++)
    if (idx[k] < 0 || idx[k] >= pr.n) {
      set_err(ctx, "gv_refine: match index out of range");
      return GV_EINVAL;
    }
  // start: the centre of the vote's leaf, kappa at its interval's centre
  RefState S0{};
  PathC path{};
  int32_t coords[GV_MAXD] = {0, 0, 0, 0, 0};
  decode_leaf(P, leaf_index, path, coords);
  for (int j = 0; j < pr.S.d; j++) {
    const double u = (double)(2 * coords[j] + 1) * std::ldexp(1.0, -(P.L[j] + 1));
    S0.q[j] = P.lo[j] + P.E[j] * u;
  }
  if (pr.S.fam != GV_POSE5DOF) S0.q[4] = 1.0;
  S0.sector = path.sector;
  S0.five = pr.S.fam == GV_POSE5DOF ? 1 : 0;
  const double T20 = std::tan(tau0) * std::tan(tau0), T2 = std::tan(tau) * std::tan(tau);
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->err.clear();
  Run X;
  bind_ctx(X, ctx);
  std::vector<void*> owned;
  std::vector<int64_t> ver;
  RefState S{}, S0out{};
  st = GV_OK;
  try {
    HIPCHK(hipSetDevice(ctx->device));
    const int ncol = ncols_of(pr.S.fam, pr.S.d);
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
    const uint64_t n = n_idx;
    int64_t* didx = dalloc<int64_t>(X, std::max<uint64_t>(1, n));
    uint32_t* ok = dalloc<uint32_t>(X, std::max<uint64_t>(1, n));
    uint32_t* pos = dalloc<uint32_t>(X, std::max<uint64_t>(1, n));
    RefState* dS = dalloc<RefState>(X, 2);  // [0]: the pose; [1]: the first sums, at the leaf centre
    const uint32_t nb = (uint32_t)std::min<uint64_t>(nblk(std::max<uint64_t>(1, n), GV_RF_WG), 1024);
    double* part = dalloc<double>(X, (uint64_t)nb * GV_RF_NV);
    owned.insert(owned.end(), {didx, ok, pos, dS, part});
    if (n) HIPCHK(hipMemcpyAsync(didx, idx, n * sizeof(int64_t), hipMemcpyHostToDevice, X.st));
    HIPCHK(hipMemcpyAsync(dS, &S0, sizeof(RefState), hipMemcpyHostToDevice, X.st));
    const unsigned gv = gs_grid(X, std::max<uint64_t>(1, n));
    // one round: verification at the current pose, then Gauss-Newton steps
    // on the verified matches; after the last round, verification and sums
    for (int round = 0; round <= rounds; round++) {
      k_rf_verify<<<gv, 256, 0, X.st>>>(dS, cols, didx, n, round == 0 ? T20 : T2, ok);
      if (round == 0) {
        k_rf_accum<<<nb, GV_RF_WG, 0, X.st>>>(dS, cols, didx, n, ok, part);
        k_rf_solve<<<1, 64, 0, X.st>>>(dS, part, nb, 0);
        HIPCHK(hipMemcpyAsync(dS + 1, dS, sizeof(RefState), hipMemcpyDeviceToDevice, X.st));
      }
      if (round == rounds) break;
      for (int it = 0; it < iters; it++) {
        k_rf_accum<<<nb, GV_RF_WG, 0, X.st>>>(dS, cols, didx, n, ok, part);
        k_rf_solve<<<1, 64, 0, X.st>>>(dS, part, nb, 1);
      }
    }
    k_rf_accum<<<nb, GV_RF_WG, 0, X.st>>>(dS, cols, didx, n, ok, part);
    k_rf_solve<<<1, 64, 0, X.st>>>(dS, part, nb, 0);
    HIPCHK(hipGetLastError());
    uint64_t nv = 0;
    if (n) {
      excl_scan(X, ok, pos, n);
      uint32_t last[2] = {0, 0};
      HIPCHK(hipMemcpyAsync(&last[0], pos + n - 1, 4, hipMemcpyDeviceToHost, X.st));
      HIPCHK(hipMemcpyAsync(&last[1], ok + n - 1, 4, hipMemcpyDeviceToHost, X.st));
      host_wait(X);
      nv = (uint64_t)last[0] + last[1];
      if (nv) {
        int64_t* dv = dalloc<int64_t>(X, nv);
        owned.push_back(dv);
        k_rf_scatter<<<gv, 256, 0, X.st>>>(didx, n, ok, pos, dv);
        ver.resize(nv);
        HIPCHK(hipMemcpyAsync(ver.data(), dv, nv * sizeof(int64_t), hipMemcpyDeviceToHost, X.st));
      }
    }
    HIPCHK(hipMemcpyAsync(&S, dS, sizeof(RefState), hipMemcpyDeviceToHost, X.st));
    HIPCHK(hipMemcpyAsync(&S0out, dS + 1, sizeof(RefState), hipMemcpyDeviceToHost, X.st));
    host_wait(X);
  } catch (DevErr& e) {
    st = e.st;
  }
  for (void* q : owned) dfree(X, q);
  (void)hipStreamSynchronize(X.st);
  if (st != GV_OK) return st;
  // pose in user units; yaw from kappa and the sector, in [0, 2 pi)
  for (int j = 0; j < GV_MAXD; j++) out->pose[j] = j < pr.S.d ? S.q[j] : 0.0;
  double yaw = (double)S.sector * (M_PI / 2.0) + std::atan(S.q[3]);
  if (yaw < 0.0) yaw += 2.0 * M_PI;
  if (yaw >= 2.0 * M_PI) yaw -= 2.0 * M_PI;
  out->pose[3] = yaw;
  out->rms = S.cnt > 0.0 ? std::sqrt(S.cost / S.cnt) : 0.0;
  out->rms0 = S0out.cnt > 0.0 ? std::sqrt(S0out.cost / S0out.cnt) : 0.0;
  out->n_verified = ver.size();
  if (ver.size() > out->verified_cap || (!out->verified && !ver.empty())) return GV_EBUFSZ;
  if (!ver.empty()) std::memcpy(out->verified, ver.data(), ver.size() * sizeof(int64_t));
  set_err(ctx, "");
  return GV_OK;
}

}  // extern "C"
