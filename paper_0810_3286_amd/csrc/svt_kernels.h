// Launch wrappers for the gfx950 kernels of the SVT hot path.
//
// Every wrapper enqueues on the given stream and returns the launch status.
// Device buffers are plain pointers; sizes are element counts.  Layouts:
//   - compressed sparse rows of one orientation of Omega: ptr[nrows+1],
//     idx[nnz] (int32), values[nnz];
//   - Lanczos bases: column-major, leading dimension ld (>= vector length);
//   - Ritz factors: row-major with row stride rs (>= r, zero padded).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace svt {

constexpr int kBlock = 256;
// Arrival counters (ReduceScratch::counters) by user; the tiled dot-product
// kernels use one counter per column tile.
constexpr int kMaxTiles = 512;
constexpr int kCounterUpdate = 0;
constexpr int kCounterFinish = 1;
constexpr int kCounterSample = 2;
constexpr int kCounterDots = 16;
constexpr int kCounterDots2 = kCounterDots + kMaxTiles;
constexpr int kNumCounters = kCounterDots2 + kMaxTiles;

// Scratch the reductions share (device memory owned by the solver).
struct ReduceScratch {
  double *partial;     // >= (kmax + 2) * max_blocks doubles
  double *h1;          // first Gram-Schmidt coefficients, kmax + 2
  double *h2;          // second Gram-Schmidt coefficients, kmax + 2
  double *scal;        // small scalars: [2] residual^2, [3] second-pass flag, [4], [5] scratch norms
  unsigned *counters;  // arrival counters, zeroed at allocation, reset by the last block
  int max_blocks;
};

// Chunking of rows into workgroups for the kernels that also reduce.
struct RowChunks {
  int nblk;            // workgroups
  int rows_per_blk;    // rows per workgroup
};
RowChunks row_chunks(int nrows, int target_rows);

// Lanes per row for the compressed-row kernels, from the mean row length.
int lanes_for(double mean_per_row);

// p = A x - coef * prev (prev may be null; coef is read on the device).
template <typename T>
hipError_t launch_spmv(hipStream_t s, int lanes, const int32_t *ptr, const int32_t *idx, const T *val,
                       const T *x, const T *prev, const double *coef, T *p, int nrows);

// First-pass Gram-Schmidt coefficients h1[c] = Q[:,c] . p (c < nq) and
// h1[nq] = |p|^2; norm_out = |p|.
template <typename T>
hipError_t launch_dots(hipStream_t s, const T *p, int nrows, const T *Q, int64_t ldq, int nq,
                       ReduceScratch &rs, double *norm_out);

// Workgroup chunking of the Gram-Schmidt kernels (<= 256 workgroups).
RowChunks vec_chunks(int nrows);

// p' = p - Q h1 (in place), h2[c] = Q[:,c] . p', h2[nq] = |p'|^2.  If the
// first pass cancelled (|p'|^2 < eta^2 |p|^2) or force_second, flags a second
// pass in scal[3]; otherwise norm_out = |p'|.
template <typename T>
hipError_t launch_cgs_update(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                             ReduceScratch &rs, double *norm_out, int force_second);

// If the second pass is flagged: p'' = p' - Q h2 (in place), norm_out = |p''|.
template <typename T>
hipError_t launch_cgs_finish(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                             ReduceScratch &rs, double *norm_out);

// out = p / *nrm (out = 0 when *nrm underflows).
template <typename T>
hipError_t launch_scale(hipStream_t s, const T *p, const double *nrm, T *out, int n);

// out[i] = standard normal draw i of stream (seed, ctr); counter-based.
template <typename T>
hipError_t launch_randn(hipStream_t s, T *out, int n, uint64_t seed, uint64_t ctr);

// out[i, l] = w[l] * sum_c Q[i, c] P[c, l] for l < r; zero for r <= l < rs.
// P is k x r row-major (double), w may be null (no scaling).
template <typename T>
hipError_t launch_ritz(hipStream_t s, const T *Q, int64_t ldq, int nrows, int k,
                       const double *P, const double *w, int r, T *out, int rs);

// For each stored entry t of row i (col j = idx[t]):
//   x = sum_l F_row[i, l] G[j, l]  (fma chain in l order, F_row first operand
//       always the row-side factor of X = U V^T in the given orientation),
//   e = M[t] - x, Y[t] = Y[t] + delta e.
// If res2_out is non-null, also reduces sum e^2 (compensated in FP32) into it.
template <typename T>
hipError_t launch_sample_update(hipStream_t s, int lanes, const int32_t *ptr, const int32_t *idx,
                                const T *M, T *Y, int nrows, const T *Urow, const T *Vcol,
                                int r, int rs, bool row_side_is_u, double delta,
                                ReduceScratch &rs_, double *res2_out);

// y[t] = a * x[t] for both value copies (the kick: Y = k0 delta M).
template <typename T>
hipError_t launch_axpby(hipStream_t s, const T *x, T *y, int64_t n, double a);

// Convert a value array between precisions / copy.
hipError_t launch_d2f(hipStream_t s, const double *x, float *y, int64_t n);
hipError_t launch_f2d(hipStream_t s, const float *x, double *y, int64_t n);

// Gather: y[i] = x[map[i]] (used to reorder host-order values on device).
template <typename T>
hipError_t launch_gather(hipStream_t s, const T *x, const int32_t *map, T *y, int64_t n);

}  // namespace svt
