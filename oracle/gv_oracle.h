/*
 * gv_oracle.h -- plain CPU reference for the general-voting maximum-depth
 * search of Aiger, Lynen, Hosang, Zeisl, "Efficient Large Scale Inlier Voting
 * for Geometric Vision Problems" (ICCV 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * Everything is IEEE binary64, round-to-nearest-even, compiled with
 * -ffp-contract=off and without fast-math.  Operation order in every formula
 * is exactly as written in gv_oracle.c.
 */
#ifndef GV_ORACLE_H
#define GV_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_LINE2D = 1, OR_PLANE3D = 2, OR_RAY3D = 3, OR_POSE4DOF = 4, OR_SIM2D = 5, OR_POSE5DOF = 6 };

/* Up to five axes: (x, y, z, kappa, f) for OR_POSE5DOF, the camera position,
 * the tangent of the yaw offset inside a sector and the factor f that turns
 * image coordinates into direction tangents (tangent = xi f); four or fewer
 * for the other families. */
#define OR_MAXD 5

enum {
  OR_OK = 0,
  OR_EINVAL = -1,   /* bad family, n, box, eps, NaN, E_x != E_y, ... */
  OR_ENOMEM = -2,
  OR_EBUFSZ = -3,   /* inlier buffer too small; n_inliers holds the need */
  OR_ERANGE = -4,   /* lattice too fine for exact binary64 evaluation */
  OR_EBUDGET = -5   /* test budget exhausted (sampled timing runs only) */
};

typedef struct {
  int family;
  int64_t n;
  const double *col[6];  /* SoA observation columns, family order */
  double lo[OR_MAXD], hi[OR_MAXD]; /* domain box, user units, family axis order */
  double eps[OR_MAXD];   /* per-axis eps, user units */
  double canon_c;        /* 0 -> 1.0; +INFINITY -> exact mode */
  int no_prune;          /* 1: never prune (pins only) */
  int no_group;          /* 1: never merge equal canonical surfaces */
  int no_dive;           /* 1: no greedy dive for the starting lower bound */
  uint64_t test_budget;  /* 0: unlimited; else stop with OR_EBUDGET */
  int threads;           /* > 1: search disjoint subtrees on that many
                            threads sharing the best key (same result) */
  int has_seed;          /* 1: seed_leaf's achieved key (its count by
                            replay) starts the best key; any achieved leaf
                            key is a valid bound, so the result is the same */
  uint64_t seed_leaf;
} or_problem;

typedef struct {
  uint64_t count;        /* max depth: number of original surfaces */
  uint64_t leaf_index;   /* [sector bits] || per-level child digits */
  uint64_t key;          /* count * 2^B + (2^B - 1 - leaf_index) */
  int32_t sector;        /* pose families: yaw sector 0..3, else 0 */
  int32_t leaf_coords[OR_MAXD];
  int32_t levels[OR_MAXD]; /* L_j per axis */
  int32_t lstar, index_bits;
  double point[OR_MAXD];   /* leaf centre, user units; pose: x,y,z,yaw(,f) */
  int64_t n_inliers;
  uint64_t tests, cells_expanded, cells_pruned, groups_merged;
  double seconds;        /* wall time of the search (not the front end) */
} or_result;

/* Full solve.  inliers: caller buffer of cap entries (may be NULL if cap 0);
 * receives the sorted original indices counted at the chosen leaf. */
int or_solve(const or_problem *p, or_result *r, int64_t *inliers, int64_t cap);

/* Threshold reporting: every leaf whose count reaches tau (>= 1), in index
 * order, with its count; cap entries at most (OR_EBUFSZ beyond, n_out then
 * holds the number found). */
int or_report(const or_problem *p, uint64_t tau, uint64_t *leaves, uint32_t *counts, int64_t cap,
              int64_t *n_out, uint64_t *tests);

/* Front end only: normalized surface parameters.  t: n x 4 (row-major, unused
 * slots 0), f: n x 2, tag: n (RAY3D parameter axis, else 0). */
int or_parametrize(const or_problem *p, double *t, double *f, int32_t *tag);

/* Root canonical parameters (the quantized surfaces before any descent), same
 * layout as or_parametrize. */
int or_root_canon(const or_problem *p, double *t, double *f, int32_t *tag);

/* Count at one leaf by per-surface chain replay; optional inlier output. */
int or_leaf_count(const or_problem *p, uint64_t leaf_index, uint64_t *count,
                  int64_t *inliers, int64_t cap);

/* Chain counts of every leaf (tiny problems only): out has 2^B entries. */
int or_all_leaf_counts(const or_problem *p, uint32_t *out, uint64_t out_len);

/* Chain counts of every cell of one level (tiny problems only): out has
 * 2^(bits) entries, a cell's index being [sector] || its child digits of
 * levels 0..level-1; level L* gives the leaf counts. */
int or_level_counts(const or_problem *p, int level, uint32_t *out, uint64_t out_len);

/* Whether surface i's chain reaches each leaf (tiny problems only): out has
 * 2^B bytes, 1 where the surface is counted. */
int or_leaf_indicator(const or_problem *p, int64_t i, uint8_t *out, uint64_t out_len);

/* Every surface's canonical form at one cell (root canonization, then the
 * canonization at each cell of the path to it) tested against each child of
 * that cell: masks[i] bit d = passes child digit d. */
int or_cell_masks(const or_problem *p, int level, int32_t sector, const int32_t *coords, uint32_t *masks);

/* One canonized-surface/cell test, for unit pins.  level: cell level of the
 * surface's canonization (the tested cell is at level+1); coords: tested cell
 * integer coordinates; sector for POSE4DOF.  Params as from or_root_canon or
 * or_canon_at.  Returns 1/0, or <0 on error. */
int or_meets(const or_problem *p, const double *t, const double *f,
             int32_t tag, int level, int32_t sector, const int32_t *coords);

/* Canonize one surface (t,f,tag as from or_parametrize) to the cell at
 * `level` with integer coordinates `coords`; writes t_out/f_out. */
int or_canon_at(const or_problem *p, const double *t, const double *f,
                int32_t tag, int level, const int32_t *coords,
                double *t_out, double *f_out);

/* Lattice and pad constants, for pins: out[0..]=
 * {Lstar, B, L0..L3, sf0..sf3 (linear) or sW,sW3,sXi,sEta (pose),
 *  pad0..pad3 at level 0, pad0..pad3 at level Lstar-1, Rg, epsn0..epsn3,
 *  exact, L4, epsn4, Fb} (out_len >= 27) */
int or_constants(const or_problem *p, double *out, int out_len);

/* After the vote (pose families): verification of the angular error of the
 * vote's inliers idx[0..n_idx) at the centre of leaf `leaf_index` (angle at
 * most tau0), then `rounds` rounds of `iters` Gauss-Newton steps on the
 * verified ones, each followed by verification again at the new pose (angle
 * at most tau) (Sec. 4.2 opening remark, Sec. 5 angular verification).  pose_out (OR_MAXD values): x, y, z, yaw in
 * [0, 2 pi) (, f); verified (cap n_idx, may be NULL): the matches whose
 * angle at the final pose is at most tau, in idx order; rms_out: root mean
 * square of |d/|d| - o/|o|| over them at the final pose; rms0_out (may be
 * NULL): the same over the first verification at the leaf centre. */
int or_refine(const or_problem *p, uint64_t leaf_index, const int64_t *idx, int64_t n_idx, double tau0, double tau,
              int rounds, int iters, double *pose_out, int64_t *verified, int64_t *n_verified, double *rms_out,
              double *rms0_out);

const char *or_status_str(int st);

#ifdef __cplusplus
}
#endif
#endif
