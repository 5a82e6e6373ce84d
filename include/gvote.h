/*
 * gvote.h -- C ABI of the MI355X general-voting library.
 *
 * The library finds, among k-surfaces in parametric form, the point of a
 * domain box in R^d that the most surfaces pass within eps of, together with
 * those surfaces (the maximum-depth / maximum-incidence problem of Aiger,
 * Lynen, Hosang, Zeisl, ICCV 2021, Sec. 3; Alg. 2 "Efficient Generalized
 * Voting", with the canonization of Sec. 3.2.1 and pruning of every cell
 * whose count cannot beat the best leaf found so far).
 *
 * All calls return gv_status: GV_OK (0) or a negative error code.  No call
 * takes or returns a framework type: pointers are plain host or device
 * addresses, sizes are 64-bit.
 *
 * Families and their observation columns (structure of arrays, binary64):
 *   GV_LINE2D   cols (x, y)             axes (a, b):   point -> dual line
 *                                        b = y - x a (Sec. 3, Eq. 2).
 *   GV_PLANE3D  cols (x, y, z)          axes (a1, a2, a0): point -> dual plane
 *                                        a0 = z - x a1 - y a2 (Sec. 4.1, Eq. 3).
 *   GV_RAY3D    cols (wx, wy, wz, ux, uy, uz)  axes (x, y, z): ray w + s u as
 *                                        two lines over its dominant axis
 *                                        (Sec. 4.3, the y = ax+b, z = cx+d form).
 *   GV_POSE4DOF cols (wx, wy, wz, xi, eta)  axes (x, y, z, yaw): a 2D-3D match
 *                                        for a camera with known gravity and
 *                                        unit focal length (the surface of
 *                                        Sec. 4.2.1 with f = 1); xi = lateral
 *                                        over forward, eta = elevation tangent.
 *                                        Requires hi[0]-lo[0] == hi[1]-lo[1];
 *                                        yaw always spans [0, 2 pi) in four
 *                                        sectors, lo[3]/hi[3] are ignored.
 *   GV_POSE5DOF cols (wx, wy, wz, xi, eta)  axes (x, y, z, yaw, f): a 2D-3D
 *                                        match for a camera with known gravity
 *                                        and unknown focal length (Sec. 4.2.1,
 *                                        the (x, y, z, kappa, f) surface):
 *                                        (xi, eta) are image coordinates whose
 *                                        product with f gives the lateral and
 *                                        elevation tangents, so f is the
 *                                        reference focal length over the true
 *                                        one.  Box as POSE4DOF plus lo[4] <
 *                                        hi[4] with lo[4] > 0; eps[4] is the f
 *                                        tolerance.  GV_FP32_FILTER applies
 *                                        where f stays within [2^-10, 2^10]
 *                                        and the lattice fits binary32, else
 *                                        binary64 throughout.  GV_EINVAL unless
 *                                        2 atan(1 + 2 eps[3]) + atan(max|xi|
 *                                        hi[4]) < 3.1 (the directions one cell
 *                                        admits then span less than pi).
 *   GV_SIM2D    cols (px, py, qx, qy)   axes (a, b, c, d): a candidate
 *                                        correspondence p -> q of two planar
 *                                        point sets under the similarity
 *                                        q = [[a, b], [-b, a]] p + (c, d)
 *                                        (Sec. 4.4): c = qx - a px - b py,
 *                                        d = qy + b px - a py.
 *
 * Per-axis eps (Sec. 3.2, "different eps for each coordinate"): leaves are
 * the cells of the dyadic subdivision of the box whose side on axis j is at
 * most eps[j]; a surface counts at a leaf when, at every level of the
 * descent, its canonized version passes within eps plus the accumulated
 * rounding allowance of the child cell, separately on each dependent axis.
 * The chosen leaf has the largest count; ties go to the lowest leaf index
 * (child digits in axis order, most significant first, the pose families'
 * sector on top).  Results are deterministic and do not depend on batching.
 */
#ifndef GVOTE_H
#define GVOTE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gv_status;
enum {
  GV_OK = 0,
  GV_EINVAL = -1,    /* bad family, n, box, eps, NaN input, E_x != E_y, ... */
  GV_ENOMEM = -2,    /* device or host allocation failed */
  GV_ETOOBIG = -3,   /* the problem alone exceeds the context memory budget */
  GV_EBUFSZ = -4,    /* inlier buffer too small: n_inliers holds the need */
  GV_EAGAIN = -5,    /* gv_poll: not finished yet */
  GV_ETIMEDOUT = -6, /* gv_poll: timeout expired */
  GV_ECANCELED = -7, /* ticket was cancelled */
  GV_EDEVICE = -8,   /* HIP runtime error; text in gv_last_error */
  GV_ERANGE = -9     /* lattice too fine for the exact device arithmetic */
};

typedef enum { GV_LINE2D = 1, GV_PLANE3D = 2, GV_RAY3D = 3, GV_POSE4DOF = 4, GV_SIM2D = 5, GV_POSE5DOF = 6 } gv_family;

/* axes of the largest family (POSE5DOF); per-axis arrays below hold this
 * many values, the unused ones ignored (inputs) or 0 (outputs) */
#define GV_AXES 5

/* GV_FP64_PLAIN: every predicate decision in binary64.
 * GV_FP32_FILTER: binary32 evaluation with a certified forward-error bound;
 * only decisions inside the bound are re-evaluated in binary64, so every
 * decision (hence every count) equals the binary64 one (pose families, where
 * the problem's lattice values fit binary32; else binary64 throughout).  For
 * the linear families both modes evaluate the same exact small-integer
 * predicate. */
typedef enum { GV_FP64_PLAIN = 0, GV_FP32_FILTER = 1 } gv_precision;

typedef struct gv_ctx gv_ctx;

typedef struct {
  int device;                 /* HIP device ordinal */
  uint64_t mem_budget_bytes;  /* 0: 60% of the device's free memory */
  void *hip_stream;           /* optional hipStream_t to run on; NULL: own stream */
  const char *autotune_cache; /* path of a text file for the launch-shape
                                 autotuner, or NULL to keep its choices in
                                 this context only.  The count and compaction
                                 kernels loop over list items (one wave per
                                 item of <= 1024 entries), so their grid
                                 changes nothing but speed.  Per family and
                                 kernel the library times each candidate grid
                                 (2, 4, 8, 16 or 32 blocks of 4 waves per CU)
                                 on its large launches with HIP events and
                                 keeps the one with the least time per byte
                                 of list entries moved;
                                 launches before that use 8.  Once the count
                                 grid is chosen, the count pass's surface
                                 tile (entries per work item: 256, 512 or
                                 1024) is chosen the same way; 1024 until
                                 then.  The choices are
                                 read from the file at creation (lines
                                 "arch CUs family choice value" of this
                                 device; choice 0 count grid, 1 compaction
                                 grid (value: blocks per CU), 2 count tile
                                 (value: log2 entries per item)) and written
                                 to it when made; an
                                 unreadable or unwritable file only means
                                 tuning again.  Results never depend on it. */
  int kernel_timing;          /* 1: time the incidence and compaction kernels
                                 with HIP events on the solve stream (adds
                                 one event pair per launch) */
} gv_ctx_config;

typedef struct {
  gv_family family;
  int64_t n;                  /* number of observations, 0 <= n < 2^31 */
  const double *col[6];       /* SoA columns in the family order above */
  int cols_on_device;         /* 1: col[] are device pointers (borrowed until
                                 the call returns / the ticket is polled);
                                 0: host pointers (copied during the call) */
  double lo[GV_AXES], hi[GV_AXES]; /* domain box, user units, family axis order */
  double eps[GV_AXES];        /* per-axis eps, user units.  Pose eps[3] is
                                 the yaw tolerance in radians, applied to
                                 kappa = tan(yaw offset inside the sector), so
                                 the tolerance on the yaw angle itself is
                                 eps / (1 + kappa^2), between eps/2 and eps */
  double canon_c;             /* eps' = eps / (c (L*+1)); 0 -> 1.0.  +INFINITY:
                                 exact mode, the plain definition (Sec. 3.1,
                                 Alg. 1 on the leaf grid): every surface is
                                 quantized once to a fixed 2^-36 lattice and
                                 never re-canonized, pads are eps rounded up
                                 to that lattice, tests run in binary64 */
  gv_precision precision;
  int group;                  /* merging of equal canonical surfaces (never
                                 changes a result): 0 at the root and in cells
                                 whose list outgrows their lattice, 1 in every
                                 cell, -1 never */
} gv_problem;

typedef struct {
  uint64_t tests;             /* (canonical surface, child cell) predicate evaluations */
  uint64_t fp64_rechecks;     /* predicate halves re-evaluated in binary64 */
  uint64_t cells_expanded, cells_pruned, groups_merged;
  uint32_t levels;            /* L*: depth of the leaves */
  double ms_total, ms_kernels;
  /* with kernel_timing: summed event time, launches and algorithmic bytes
   * of the incidence-test kernel (entries read; the pose families also write a pass
   * mask per entry) and of the compaction kernel (entries of the parents
   * with a child in the chunk read, pose masks read, children written) */
  double test_ms, compact_ms;
  uint64_t test_launches, compact_launches;
  uint64_t test_bytes, compact_bytes;
  double ms_queued;           /* gv_submit: time from submission until a
                                 serving lane admitted the problem (memory
                                 admission); 0 for gv_solve */
  uint64_t compact_write_bytes; /* with kernel_timing: the part of
                                 compact_bytes that is child entries written */
} gv_stats;

typedef struct {
  double point[GV_AXES];      /* leaf centre, user units; pose (x,y,z,yaw[,f]), yaw in [0,2pi) */
  uint64_t count;             /* maximum depth: number of original surfaces */
  uint64_t leaf_index;
  int32_t sector;             /* pose families: yaw sector (0..3), else 0 */
  int32_t leaf_coords[GV_AXES];
  int64_t *inliers;           /* caller buffer (host), sorted ascending */
  uint64_t inliers_cap;
  uint64_t n_inliers;         /* on GV_EBUFSZ: required capacity */
  double bound[GV_AXES];      /* certified approximation bound per axis, user
                                 units (Sec. 3.2): on an axis that surfaces
                                 depend on (LINE2D b, PLANE3D a0, every RAY3D
                                 axis, pose z and yaw), every reported
                                 inlier's range over the leaf's parameter box
                                 comes within bound[j] of the leaf's interval
                                 on that axis: the last pad plus the
                                 accumulated canonization allowance.  Pose
                                 bound[3] is in kappa units, which also bounds
                                 the yaw angle in radians (|d yaw/d kappa| <=
                                 1), and holds where the leaf is farther from
                                 the match than the apex guard (one leaf xy
                                 side).  On a pure parameter axis (LINE2D a,
                                 PLANE3D a1 a2, pose x y and f): half the leaf
                                 side, the distance from point[] to any point
                                 of the leaf. */
  gv_stats stats;
} gv_result;

/* Create a context on cfg->device.  Owns all library device memory; *out is
 * NULL on failure. */
gv_status gv_create(gv_ctx **out, const gv_ctx_config *cfg);

/* Release the context and every device allocation it owns. */
gv_status gv_destroy(gv_ctx *ctx);

/* Solve one problem, blocking (Alg. 2 end to end: front end, root
 * canonization and grouping, a dive that seeds the best key, depth-first
 * frontier expansion with pruning, best-key reduction, path-replay inlier
 * extraction) on the context's stream.  gv_solve calls on one context are
 * serialized; they may run while submitted problems are served. */
gv_status gv_solve(gv_ctx *ctx, const gv_problem *p, gv_result *r);

/* Threshold reporting (the ray-intersection setting of Sec. 4.3: every cell
 * of the leaf grid that more than a threshold of surfaces meet): the same
 * search with the cut "count < tau" in place of the best key.  Writes every
 * leaf whose count is at least tau (>= 1) with its count, in ascending leaf
 * index order, to leaves[] / counts[] (host buffers of cap entries).
 * *n_out = the number of such leaves; GV_EBUFSZ when it exceeds cap.  Exact
 * mode, precision and grouping as in gv_problem.  stats_out may be NULL. */
gv_status gv_report(gv_ctx *ctx, const gv_problem *p, uint64_t tau, uint64_t *leaves, uint32_t *counts,
                    uint64_t cap, uint64_t *n_out, gv_stats *stats_out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): gv_solve with every
 * device buffer of the search taken from one region of 256 MiB that the
 * library holds, as static device memory, on each GPU it runs on until the
 * process ends; no device or pinned allocation, no event, no tuning sample.
 * Results equal gv_solve's.  At most 2^19 observations (GV_ETOOBIG beyond,
 * and when a search outgrows the region).  Calls on one device share the
 * region, which keeps the last call's contents, so they run one after the
 * other (a per-device lock); overlapping calls on one GPU queue behind each
 * other.  Host columns are copied into the region. */
gv_status gv_solve_noalloc(gv_ctx *ctx, const gv_problem *p, gv_result *r);

/* Front end only (Eq. 1-3 and the posing surface): writes the normalized
 * parameters, row-major, t_out n x 4 and f_out n x 2 (host buffers), and
 * tag_out n (RAY3D parameter axis, else 0; may be NULL).  Layout per family:
 * LINE2D t=(t,0,0,0) f=(f,0); PLANE3D t=(t1,t2,0,0) f=(f,0); RAY3D
 * t=(t_q1,0,t_q2,0) f=(f_q1,f_q2); POSE4DOF and POSE5DOF t=(W1,W2,xi,eta') f=(W3,0); SIM2D
 * t=(t_ca,t_cb,t_da,t_db) f=(f_c,f_d) (slopes of the dependent axes c, d over
 * the parameter axes a, b). */
gv_status gv_parametrize(gv_ctx *ctx, const gv_problem *p, double *t_out, double *f_out,
                         int32_t *tag_out);

/* Continuous batching: enqueue a problem (columns copied or borrowed as in
 * gv_problem) and return a ticket.  The first call starts the context's
 * serving lanes (three by default: a host thread, HIP stream and allocator
 * each); a free lane takes queued problems as the memory budget allows, so
 * problems run concurrently on the device.  Results equal gv_solve's.
 * The lanes overlap best when each stream has a hardware queue of its own:
 * HIP gives a process four unless GPU_MAX_HW_QUEUES (read when the process
 * first initializes HIP) asks for more; eight serve three lanes and the
 * context's stream. */
gv_status gv_submit(gv_ctx *ctx, const gv_problem *p, uint64_t *ticket);

/* Wait up to timeout_ms (0: do not wait, <0: forever) for a ticket; on
 * success fills *r (inliers into r->inliers) and retires the ticket. */
gv_status gv_poll(gv_ctx *ctx, uint64_t ticket, gv_result *r, int timeout_ms);

/* Cancel a ticket: a queued problem is dropped, a running one stops at its
 * next frontier expansion; a later poll returns GV_ECANCELED. */
gv_status gv_cancel(gv_ctx *ctx, uint64_t ticket);

/* Incidence test only (the sub-box step of Alg. 2: which surfaces pass
 * within eps of each child, Sec. 3.2.1 and the Surface-Box paragraph of Sec.
 * 3.3), for parity checks of that step.  Every observation of p becomes its
 * canonical surface at the cell of `level` with integer coordinates
 * coords[0..4] (each in [0, 2^min(level, L_j)), 0 beyond the family's axes)
 * and, for the pose families, yaw
 * sector `sector` (0..3, else 0): the root canonization followed by the
 * child canonization of every level on the path to that cell (pose and
 * exact mode: the root quantization only).  It is then tested against each
 * child of the cell exactly as the search tests it, in p->precision.
 * masks_out[i] (host buffer of n words) gets bit d set when surface i passes
 * child digit d (the split axes' bits in axis order, most significant
 * first).  stats_out (may be NULL): tests = n * children, fp64_rechecks =
 * decisions the binary32 filter left to binary64.  0 <= level < L*. */
gv_status gv_incidence(gv_ctx *ctx, const gv_problem *p, int32_t level, int32_t sector, const int32_t coords[GV_AXES],
                       uint32_t *masks_out, gv_stats *stats_out);

/* Verification and refinement after the vote (pose families).  The vote's
 * pose is handed to a more accurate method that works on its nearly
 * outlier-free inlier set (Sec. 4.2, opening remark), and the angular error
 * of the final inlier set is verified (Sec. 5).  Start: the centre of leaf
 * `leaf_index` (as gv_solve returns it) with the kappa of its interval's
 * centre.  Verification keeps the matches of idx[0..n_idx) (host buffer,
 * indices into p's observations, e.g. the vote's inliers) whose angle
 * between the observed bearing and the direction from the camera to their
 * point is at most tau0 at the leaf centre (a tau0 that covers the leaf) and
 * at most tau at later poses; the decision uses only +, -, *, / and sqrt
 * in binary64, so it is exact IEEE arithmetic.  Then `rounds` times: `iters`
 * damped Gauss-Newton steps on the kept matches minimizing the sum of
 * |d/|d| - o/|o||^2 (the unit bearing differences; (2 sin(angle/2))^2 each)
 * over (x, y, z, kappa[, f]) inside the leaf's yaw sector, then
 * verification again.  Every step runs on the device without a host wait.
 * Results: out->pose (x, y, z, yaw in [0, 2 pi)[, f]); out->verified (caller
 * buffer of verified_cap entries) the kept matches in idx order, n_verified
 * their number (GV_EBUFSZ when it exceeds the cap); out->rms the root mean
 * square of |d/|d| - o/|o|| over them at the final pose, out->rms0 over the
 * first verification's matches at the leaf centre.  GV_EINVAL for a family
 * other than the pose ones, tau or tau0 outside (0, 1.5), rounds outside
 * [0, 64], iters outside [0, 256], a leaf index or match index out of range. */
typedef struct {
  double pose[GV_AXES];
  double rms0, rms;
  int64_t *verified;
  uint64_t verified_cap;
  uint64_t n_verified;
} gv_refined;
gv_status gv_refine(gv_ctx *ctx, const gv_problem *p, uint64_t leaf_index, const int64_t *idx, uint64_t n_idx,
                    double tau0, double tau, int32_t rounds, int32_t iters, gv_refined *out);

/* Static text for a status code. */
const char *gv_status_str(gv_status s);

/* Text of the last error on this context (thread-local copy), "" if none. */
const char *gv_last_error(gv_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
