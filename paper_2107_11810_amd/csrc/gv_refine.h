// gv_refine.h -- verification and refinement after the vote (pose families).
//
// The vote's pose (the centre of its leaf) is handed to a more accurate
// method that works on the vote's nearly outlier-free inlier set (Sec. 4.2,
// opening remark), and the angular error of the final inlier set is
// verified (Sec. 5).  Pose q = (x, y, z, kappa[, f]) in user units inside
// the vote's yaw sector s: the camera's forward direction, turned into the
// sector's frame, is (1, kappa)/sqrt(1 + kappa^2).  In camera axes
// (forward, lateral, up) match i is observed along
//   o = (1, a, b sqrt(1 + a^2)),  a = xi f, b = eta f  (f = 1 for 4-DoF),
// and its point w lies along
//   d = ((u1 + kappa u2)/n, (u2 - kappa u1)/n, w3 - z),
// u = Rot_s(w1 - x, w2 - y), n = sqrt(1 + kappa^2).
//   verification: angle(o, d) <= tau, tested as o.d > 0 and
//     |o x d|^2 <= tan^2(tau) (o.d)^2 (+, -, *, /, sqrt only: exact IEEE
//     binary64, so the decision does not depend on the machine);
//   refinement: Gauss-Newton steps with a small fixed damping on
//     sum |d/|d| - o/|o||^2 over the verified matches.
// One thread per match computes its residual and Jacobian and adds them
// into per-block sums (a fixed reduction tree); one thread then sums the
// blocks in order, solves the 4x4 or 5x5 system by Cholesky and updates the
// pose in device memory, so a whole refinement is one stream of launches
// without a host wait.
#pragma once
#include "gv_kernels.h"
#include "gv_root.h"

#define GV_RF_DAMP 1e-6
#define GV_RF_NV 22  // per-block sums: A (15, lower triangle), g (5), cost, count
#define GV_RF_WG 256

struct RefState {
  double q[5];      // pose: x, y, z, kappa, f (user units; f = 1 for 4-DoF)
  double cost, cnt;  // sum of squared residuals and matches in the last sums
  int32_t sector, five;
};

__device__ inline void rf_rot_d(int s, double a, double b, double& u1, double& u2) {
  if (s == 0) { u1 = a; u2 = b; }
  else if (s == 1) { u1 = b; u2 = -a; }
  else if (s == 2) { u1 = -a; u2 = -b; }
  else { u1 = -b; u2 = a; }
}

// observed (o) and predicted (d) camera-frame directions of one match
__device__ inline void rf_dirs_d(const RefState& S, const double* const* col, int64_t i, double o[3], double d[3]) {
  const double f = S.five ? S.q[4] : 1.0;
  const double a = col[3][i] * f, b = col[4][i] * f;
  o[0] = 1.0;
  o[1] = a;
  o[2] = b * sqrt(1.0 + a * a);
  double u1, u2;
  rf_rot_d(S.sector, col[0][i] - S.q[0], col[1][i] - S.q[1], u1, u2);
  const double n = sqrt(1.0 + S.q[3] * S.q[3]);
  d[0] = (u1 + S.q[3] * u2) / n;
  d[1] = (u2 - S.q[3] * u1) / n;
  d[2] = col[2][i] - S.q[2];
}

__device__ inline uint32_t rf_ok(const double o[3], const double d[3], double T2) {
  const double dot = (o[0] * d[0] + o[1] * d[1]) + o[2] * d[2];
  const double c0 = o[1] * d[2] - o[2] * d[1], c1 = o[2] * d[0] - o[0] * d[2], c2 = o[0] * d[1] - o[1] * d[0];
  const double cr = (c0 * c0 + c1 * c1) + c2 * c2;
  return (dot > 0.0 && cr <= T2 * (dot * dot)) ? 1u : 0u;
}

// flags of the vote's inliers idx[0..n) at the current pose
__global__ void k_rf_verify(const RefState* __restrict__ Sp, Cols cols, const int64_t* __restrict__ idx, uint64_t n,
                            double T2, uint32_t* __restrict__ ok) {
  const RefState S = *Sp;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
    double o[3], d[3];
    rf_dirs_d(S, cols.c, idx[k], o, d);
    ok[k] = rf_ok(o, d, T2);
  }
}

// residual r = d/|d| - o/|o| and Jacobian J (3 x 5) of one match
__device__ inline void rf_resid_d(const RefState& S, const double* const* col, int64_t i, double r[3],
                                  double J[3][5]) {
  double o[3], d[3];
  rf_dirs_d(S, col, i, o, d);
  const double nd = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  const double no = sqrt((o[0] * o[0] + o[1] * o[1]) + o[2] * o[2]);
  const double dh[3] = {d[0] / nd, d[1] / nd, d[2] / nd}, oh[3] = {o[0] / no, o[1] / no, o[2] / no};
#pragma unroll
  for (int c = 0; c < 3; c++) r[c] = dh[c] - oh[c];
  const double k = S.q[3], n2 = 1.0 + k * k, n = sqrt(n2);
  double ux1, ux2, uy1, uy2;
  rf_rot_d(S.sector, -1.0, 0.0, ux1, ux2);
  rf_rot_d(S.sector, 0.0, -1.0, uy1, uy2);
  // derivatives of d by x, y, z, kappa
  const double dd[4][3] = {{(ux1 + k * ux2) / n, (ux2 - k * ux1) / n, 0.0},
                           {(uy1 + k * uy2) / n, (uy2 - k * uy1) / n, 0.0},
                           {0.0, 0.0, -1.0},
                           {d[1] / n2, -d[0] / n2, 0.0}};
#pragma unroll
  for (int p = 0; p < 4; p++) {
    const double pr = (dh[0] * dd[p][0] + dh[1] * dd[p][1]) + dh[2] * dd[p][2];
#pragma unroll
    for (int c = 0; c < 3; c++) J[c][p] = (dd[p][c] - dh[c] * pr) / nd;
  }
  if (S.five) {
    // o depends on f: do/df = (0, xi, eta s + b a xi / s)
    const double xi = col[3][i], eta = col[4][i];
    const double a = xi * S.q[4], b = eta * S.q[4];
    const double sa = sqrt(1.0 + a * a);
    const double dof[3] = {0.0, xi, eta * sa + (b * a) * xi / sa};
    const double pr = (oh[0] * dof[0] + oh[1] * dof[1]) + oh[2] * dof[2];
#pragma unroll
    for (int c = 0; c < 3; c++) J[c][4] = -((dof[c] - oh[c] * pr) / no);
  } else {
#pragma unroll
    for (int c = 0; c < 3; c++) J[c][4] = 0.0;
  }
}

__device__ inline double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// per-block sums of J^T J (lower triangle), J^T r, cost and count over the
// verified matches; part[block * GV_RF_NV + k]
__global__ void __launch_bounds__(GV_RF_WG) k_rf_accum(const RefState* __restrict__ Sp, Cols cols,
                                                       const int64_t* __restrict__ idx, uint64_t n,
                                                       const uint32_t* __restrict__ ok, double* __restrict__ part) {
  const RefState S = *Sp;
  const int P = S.five ? 5 : 4;
  double acc[GV_RF_NV];
#pragma unroll
  for (int v = 0; v < GV_RF_NV; v++) acc[v] = 0.0;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
    if (!ok[k]) continue;
    double r[3], J[3][5];
    rf_resid_d(S, cols.c, idx[k], r, J);
    int t = 0;
#pragma unroll
    for (int a = 0; a < 5; a++) {
#pragma unroll
      for (int b = 0; b <= a; b++) {
        if (a < P) acc[t] += (J[0][a] * J[0][b] + J[1][a] * J[1][b]) + J[2][a] * J[2][b];
        t++;
      }
    }
#pragma unroll
    for (int a = 0; a < 5; a++)
      if (a < P) acc[15 + a] += (J[0][a] * r[0] + J[1][a] * r[1]) + J[2][a] * r[2];
    acc[20] += (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    acc[21] += 1.0;
  }
  __shared__ double ws[GV_RF_WG / 64][GV_RF_NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < GV_RF_NV; v++) {
    const double s = wave_sum_f64(acc[v]);
    if (lane == 0) ws[wv][v] = s;
  }
  __syncthreads();
  if (threadIdx.x < GV_RF_NV) {
    double s = 0.0;
    for (int w = 0; w < GV_RF_WG / 64; w++) s += ws[w][threadIdx.x];
    part[(uint64_t)blockIdx.x * GV_RF_NV + threadIdx.x] = s;
  }
}

// Sum the blocks' partial sums in block order; update = 1: one damped
// Gauss-Newton step (Cholesky; no step when the system is not positive
// definite); always record the cost and count.
__global__ void k_rf_solve(RefState* __restrict__ Sp, const double* __restrict__ part, uint32_t nblk, int update) {
  __shared__ double sum[GV_RF_NV];
  if (threadIdx.x < GV_RF_NV) {
    double s = 0.0;
    for (uint32_t b = 0; b < nblk; b++) s += part[(uint64_t)b * GV_RF_NV + threadIdx.x];
    sum[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  RefState S = *Sp;
  S.cost = sum[20];
  S.cnt = sum[21];
  if (update) {
    const int P = S.five ? 5 : 4;
    double M[5][5], L[5][5], y[5], x[5];
    int t = 0;
    for (int a = 0; a < 5; a++)
      for (int b = 0; b <= a; b++) {
        M[a][b] = sum[t];
        M[b][a] = sum[t];
        t++;
      }
    for (int a = 0; a < P; a++) M[a][a] = M[a][a] + GV_RF_DAMP * M[a][a];
    bool pd = true;
    for (int j = 0; j < P && pd; j++) {
      double sd = M[j][j];
      for (int k = 0; k < j; k++) sd -= L[j][k] * L[j][k];
      if (!(sd > 0.0) || !isfinite(sd)) {
        pd = false;
        break;
      }
      L[j][j] = sqrt(sd);
      for (int r = j + 1; r < P; r++) {
        double v = M[r][j];
        for (int k = 0; k < j; k++) v -= L[r][k] * L[j][k];
        L[r][j] = v / L[j][j];
      }
    }
    if (pd) {
      for (int r = 0; r < P; r++) {
        double v = -sum[15 + r];
        for (int k = 0; k < r; k++) v -= L[r][k] * y[k];
        y[r] = v / L[r][r];
      }
      for (int r = P - 1; r >= 0; r--) {
        double v = y[r];
        for (int k = r + 1; k < P; k++) v -= L[k][r] * x[k];
        x[r] = v / L[r][r];
      }
      for (int a = 0; a < P; a++) S.q[a] += x[a];
    }
  }
  *Sp = S;
}

// indices of the flagged matches, in idx order (pos: exclusive scan of ok)
__global__ void k_rf_scatter(const int64_t* __restrict__ idx, uint64_t n, const uint32_t* __restrict__ ok,
                             const uint32_t* __restrict__ pos, int64_t* __restrict__ out) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x)
    if (ok[k]) out[pos[k]] = idx[k];
}
