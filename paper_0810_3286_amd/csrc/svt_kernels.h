// Launch wrappers for the gfx950 kernels of the SVT hot path.
//
// Every wrapper enqueues on the given stream and returns the launch status.
// Device buffers are plain pointers; sizes are element counts.  Layouts:
//   - compressed sparse rows of one orientation of Omega: ptr[nrows+1],
//     idx[nnz] (int32), values[nnz];
//   - Lanczos bases: column-major, leading dimension ld (>= vector length);
//   - Ritz factors: row-major with row stride rs (>= r, even, zero padded).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace svt {

// Kernel timing: the next kernel this thread launches through the wrappers
// below records its own start and end in these events (hipExtLaunchKernel),
// so their elapsed time is the kernel's duration without the gaps around
// it; the launch clears them.  Null: no timing.
void set_launch_events(hipEvent_t start, hipEvent_t stop);

constexpr int kBlock = 256;
constexpr int kSpmvBlock = 1024;  // workgroup of the LDS-staged sparse product
constexpr int kGsChunks1 = 32;    // row chunks of the first Gram-Schmidt dot products
constexpr int kGsChunks2 = 256;   // row chunks of the Gram-Schmidt updates
constexpr int kSampleMaxBlocks = 1024;

// Partial-sum buffers of the Gram-Schmidt kernels (device memory owned by
// the solver): part1 >= max_cols * kGsChunks1, part2 >= max_cols *
// kGsChunks2, part3 >= kGsChunks2 doubles.
struct GsScratch {
  double *part1, *part2, *part3;
  int max_cols;
};

struct RowChunks {
  int nblk;            // workgroups
  int rows_per_blk;    // rows per workgroup
};
RowChunks row_chunks(int nrows, int target_rows);

struct GsPlan {
  int nrc1, rpb1;      // dot-product row chunks and their size
  int nrc2, rpb2;      // update row chunks and their size
};
GsPlan gs_plan(int nrows);
size_t gs_update_lds(int nq, int rows_per_blk);

// Lanes per row for the compressed-row kernels, from the mean row length.
int lanes_for(double mean_per_row);

// LDS-staged sparse product: one workgroup per compute unit owns a row range;
// x is copied into LDS in nseg column segments of segcols entries.
struct SpmvLdsPlan {
  int nblk, rows_per_blk, segcols, nseg;
  int lanes;  // lanes per row (all of a workgroup's rows at once when possible)
  size_t lds;
  bool ok;  // false: x needs many small segments; use the gather kernel
};
SpmvLdsPlan spmv_lds_plan(int nrows, int ncols, int elem_bytes, int num_cus, int lds_bytes);

// p = A (x / s) - s prev, with s^2 the sum of the xnp partials in xpart
// (xpart null: s = 1, x already normalised; prev may be null).  With x_out
// non-null the normalised x is written to x_out (ncols entries) and s to
// *s_out: the previous half-step's vector joins its basis.  pl non-null:
// x staged in LDS (segptr: nrows x (nseg + 1) segment starts, null when
// nseg == 1); null: x gathered from memory.
template <typename T>
hipError_t launch_spmv(hipStream_t s, int lanes, const SpmvLdsPlan *pl, const int32_t *ptr, const int32_t *idx,
                       const T *val, const int32_t *segptr, const T *x, const double *xpart, int xnp, T *x_out,
                       double *s_out, int ncols, const T *prev, T *p, int nrows);

// Orthogonalise p (length nrows, overwritten) against the nq orthonormal
// columns of Q by classical Gram-Schmidt applied twice, leaving the |p|^2
// partials in gs.part3 (gs_plan(nrows).nrc2 of them) for the consumer's
// lazy normalisation.  Three kernels (one when nq == 0); the coefficients
// never leave the device.
template <typename T>
hipError_t launch_orthonormalize(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                                 const GsScratch &gs);

// The three kernels of launch_orthonormalize (nq >= 1), for callers that
// time them one by one: the first pass's dot products into gs.part1; then
// the first update with the second pass's dot products into gs.part2
// (second = false), or the second update with the |p|^2 partials into
// gs.part3 (second = true).
template <typename T>
hipError_t launch_gs_dots(hipStream_t s, const T *p, int nrows, const T *Q, int64_t ldq, int nq,
                          const GsScratch &gs);
template <typename T>
hipError_t launch_gs_update(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                            const GsScratch &gs, bool second);

// |p|^2 partials into gs.part3.
template <typename T>
hipError_t launch_sumsq(hipStream_t s, T *p, int nrows, const GsScratch &gs);

// out = p / |p| with |p|^2 from gs.part3; *coef_out = |p|.
template <typename T>
hipError_t launch_finalize(hipStream_t s, const T *p, int nrows, const GsScratch &gs, T *out, double *coef_out);

// out[i] = standard normal draw i of stream (seed, ctr); counter-based.
template <typename T>
hipError_t launch_randn(hipStream_t s, T *out, int n, uint64_t seed, uint64_t ctr);

// out[i, l] = w[l] * sum_c Q[i, c] P[c, l] for l < r; zero for r <= l < rs.
// P is k x r row-major (double), w may be null (no scaling).
template <typename T>
hipError_t launch_ritz(hipStream_t s, const T *Q, int64_t ldq, int nrows, int k,
                       const double *P, const double *w, int r, T *out, int rs);

// For each stored entry t of row i (col j = idx[t]):
//   x = sum_l U[u_row, l] V[v_row, l]  (fma chain in l order, u entry first),
//   e = M[t] - x, Y[t] = Y[t] + delta e.
// With part_out non-null, workgroup b writes its sum of e^2 to part_out[b]
// (sample_blocks() workgroups).
template <typename T>
hipError_t launch_sample_update(hipStream_t s, int lanes, const int32_t *ptr, const int32_t *idx,
                                const T *M, T *Y, int nrows, const T *Fu, const T *Fv,
                                int r, int rs, bool row_side_is_u, double delta, double *part_out);
int sample_blocks(int nrows, int lanes);

// y[t] = a * x[t] (the kick: Y = k0 delta M).
template <typename T>
hipError_t launch_axpby(hipStream_t s, const T *x, T *y, int64_t n, double a);

// Convert a value array between precisions.
hipError_t launch_d2f(hipStream_t s, const double *x, float *y, int64_t n);
hipError_t launch_f2d(hipStream_t s, const float *x, double *y, int64_t n);

// Gather: y[i] = x[map[i]].
template <typename T>
hipError_t launch_gather(hipStream_t s, const T *x, const int32_t *map, T *y, int64_t n);

}  // namespace svt
