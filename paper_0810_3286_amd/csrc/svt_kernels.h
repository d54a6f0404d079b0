// Launch wrappers for the gfx950 kernels of the SVT hot path.
//
// Every wrapper enqueues on the given stream and returns the launch status.
// Device buffers are plain pointers; sizes are element counts.  Layouts:
//   - compressed sparse rows of one orientation of Omega: ptr[nrows+1],
//     idx[nnz] (int32), values[nnz];
//   - Lanczos bases: column-major, leading dimension ld (>= vector length);
//   - Ritz factors: row-major with row stride rs (>= r, even, zero padded);
//   - reduction partials: column c of a partial array holds one value per
//     workgroup of the row partition (row_plan), at part[c * nblk + b].
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

constexpr int kBlock = 256;            // elementwise and sampled-update kernels
constexpr int kRowBlock = 1024;        // row-range kernels (sparse product, Gram-Schmidt)
constexpr int kMaxRowBlocks = 256;     // row ranges per vector: one per compute unit ...
constexpr int kMaxRowsPerBlock = 2048; // ... unless that would give longer ranges
constexpr int kSampleMaxBlocks = 1024;

// Partition of a vector of nrows entries into nblk contiguous row ranges of
// rows_per_blk (the last one shorter), shared by the sparse product, the
// Gram-Schmidt kernels and the norm kernels: the partial sums they exchange
// have one entry per range.  At most kMaxRowBlocks ranges of at least
// min_rows rows (kDefaultMinRows unless a solve asks for more: fewer, fuller
// workgroups leave compute units to other solves running at the same time).
constexpr int kDefaultMinRows = 8;
struct RowPlan {
  int nblk, rows_per_blk;
};
RowPlan row_plan(int nrows, int min_rows = kDefaultMinRows);

// Partial-sum buffers of the bidiagonalisation (device memory owned by the
// solver): part1 and part2 hold max_cols columns of max_blocks partials,
// part3 max_blocks partials, red max_cols column sums.
struct GsScratch {
  double *part1, *part2, *part3;
  double *red;
  int max_cols, max_blocks;
};

struct RowChunks {
  int nblk;            // workgroups
  int rows_per_blk;    // rows per workgroup
};
RowChunks row_chunks(int nrows, int target_rows);

// Lanes per row for the sampled-update kernel, from the mean row length.
int lanes_for(double mean_per_row);

// Sparse product plan: the row partition of row_plan(nrows), lanes per row,
// and nseg column segments of segcols entries of x staged in LDS (nseg = 0:
// x gathered from memory).  mode 0 and 2 stage x in one segment, or in up
// to 8 segments of >= 1024 entries; 1 always gathers.
struct SpmvPlan {
  int nblk, rows_per_blk, lanes, nseg, segcols;
  size_t lds;  // dynamic LDS bytes of a launch
  int min_rows;  // of row_plan
};
SpmvPlan spmv_plan(int nrows, int ncols, int elem_bytes, int lds_bytes, int mode,
                   int min_rows = kDefaultMinRows);

// The input of a sparse product: the other side's new vector x (ncols
// entries) as the previous half-step left it, with its one-pass
// reorthogonalisation still pending.  pend holds nqx + 1 columns of np
// partials (row_plan of x's length): x's dot products with the nqx columns
// of its basis Q_x, then |x|^2.  The product uses x' = (x - Q_x h) / s, h
// the column sums, s = sqrt(|x|^2 - |h|^2); nqx = 0: x' = x / |x|; pend
// null: x' = x.  alpha and beta (device, alpha[c] = alpha_{c+1}, beta[c] =
// beta_{c+1}) give the image of Q_x h through the bidiagonal relations; side
// 0: the product is A v (x on the v side), 1: A^T u.
constexpr int kSpmvAuxCols = 1024;  // largest nqx + side fused into the product
// LDS scratch of the column reductions (64 columns x 17 padded strands, then
// 64 sums of squares)
constexpr int kReduceScratch = 1152;
constexpr long kSpmvAuxBytes = (long)sizeof(double) * (2 * kSpmvAuxCols + 2 + kReduceScratch);
template <typename T>
struct SpmvInput {
  const T *x = nullptr;
  const double *pend = nullptr;
  int np = 0;
  const T *Qx = nullptr;          // x's basis, column-major, leading dimension ldqx
  int64_t ldqx = 0;
  int nqx = 0;
  T *x_out = nullptr;             // receives x' (may be null)
  double *s_out = nullptr;        // receives s (may be null)
  double *removed_out = nullptr;  // receives |h|^2 / |x|^2 (may be null)
  const double *alpha = nullptr, *beta = nullptr;
  int side = 0;
};

// p = A x' - s prev over nrows rows (prev may be null), x' as above; with
// nqx > 0 it is taken as (A x - Q g) / s - s prev, where Q must hold the nq
// = nqx + side basis columns of p's side.  Column indices: idx16 (16-bit,
// ncols <= 65536: a quarter less streamed per entry) when not null, else
// idx.  segptr: nrows x (nseg + 1) segment starts (null unless nseg > 1).  With dots_out non-null the kernel
// also writes the partial dot products of p with the first ndots columns of
// Q (ndots = nq, or 0 when p is left unorthogonalised) and |p|^2 (column
// ndots): ndots + 1 columns, p's own pending update.  Returns
// hipErrorInvalidValue for inconsistent arguments (nqx > 0 with a missing
// pointer, nq != nqx + side, nq > kSpmvAuxCols, or ndots not 0 or nq).
template <typename T>
hipError_t launch_spmv(hipStream_t s, const SpmvPlan &pl, const int32_t *ptr, const int32_t *idx,
                       const uint16_t *idx16, const T *val, const int32_t *segptr, const SpmvInput<T> &in,
                       int ncols, const T *prev, T *p, int nrows, const T *Q, int64_t ldq, int nq, int ndots,
                       double *dots_out);

// s (and |h|^2 / |x|^2) of a pending vector, exactly as the sparse product
// that consumes it computes them: *s_out, *removed_out (may be null).
// nqx <= kSpmvAuxCols.
hipError_t launch_pending_norm(hipStream_t s, const double *pend, int np, int nqx, double *s_out,
                               double *removed_out);

// The nqx + 1 column sums of a pending vector's partials (np each) into
// out, bit for bit as a sparse product or launch_pending_norm would form
// them; either then takes out as one partial (np = 1).  nqx <= kSpmvAuxCols.
hipError_t launch_pending_reduce(hipStream_t s, const double *pend, int np, int nqx, double *out);

// One classical Gram-Schmidt update of p (length nrows, overwritten)
// against the nq >= 1 orthonormal columns of Q, with coefficients h summed
// from the nq + 1 columns of part_in (column nq: |p|^2).  second = false:
// part_out receives the next pass's partial dot products (nq + 1 columns);
// second = true: the |p|^2 partials of the result (one column).  One call
// with second = true after launch_spmv's dots is one pass; a call with
// second = false and one with second = true make CGS2.  removed (may be
// null): receives |h|^2 / |p|^2.
template <typename T>
hipError_t launch_gs_update(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                            const double *part_in, double *part_out, bool second, double *removed,
                            int min_rows = kDefaultMinRows);

// |p|^2 partials (one column).
template <typename T>
hipError_t launch_sumsq(hipStream_t s, const T *p, int nrows, double *part_out,
                       int min_rows = kDefaultMinRows);

// out = p / |p| with |p|^2 the sum of the partials in part; *coef_out = |p|.
template <typename T>
hipError_t launch_finalize(hipStream_t s, const T *p, int nrows, const double *part, T *out,
                           double *coef_out, int min_rows = kDefaultMinRows);

// out[i] = standard normal draw i of stream (seed, ctr); counter-based.
template <typename T>
hipError_t launch_randn(hipStream_t s, T *out, int n, uint64_t seed, uint64_t ctr);

// out[i, l] = w[l] * sum_c Q[i, c] P[c, l] for l < r; zero for r <= l < rs.
// P is k x r row-major (double), w may be null (no scaling).  FP64 sums on
// the matrix cores in both precisions.  hipErrorInvalidValue for k < 1,
// r > rs or ldq < nrows.
template <typename T>
hipError_t launch_ritz(hipStream_t s, const T *Q, int64_t ldq, int nrows, int k,
                       const double *P, const double *w, int r, T *out, int rs);

// For each stored entry t of row i (col j = idx[t]):
//   x = sum_l U[u_row, l] V[v_row, l]  (fma chain in l order, u entry first),
//   e = M[t] - x, Y[t] = Y[t] + delta e.
// rs: row stride of both factors, a multiple of 16 / sizeof(T) (>= r), rows
// zero padded.  With part_out non-null, workgroup b writes its sum of e^2 to
// part_out[b] (sample_blocks() workgroups).
// With Yp and Ym (the Dantzig selector's multipliers, same order as Y): Yp[t]
// = max(Yp[t] + delta (e - E), 0), Ym[t] = max(Ym[t] + delta (-e - E), 0),
// Y[t] = Yp[t] - Ym[t], and the partials sum max(|e| - E, 0)^2 instead;
// part2_out (may be null) then receives the partial sums of e^2.
// hipErrorInvalidValue for a bad stride, one multiplier array without the
// other, or E < 0.
template <typename T>
hipError_t launch_sample_update(hipStream_t s, int lanes, const int32_t *ptr, const int32_t *idx,
                                const T *M, T *Y, int nrows, const T *Fu, const T *Fv, int r, int rs,
                                bool row_side_is_u, double delta, double *part_out, T *Yp = nullptr,
                                T *Ym = nullptr, double E = 0.0, double *part2_out = nullptr);

// General linear operator A(X) = G x_S (measurements; G in CSR over the p
// measurements, gidx into the support's row-compressed order):
// launch_measure: r_i = b_i - (G x)_i, y_i += delta r_i, and the partial
// sums of r_i^2 into part_out (measure_blocks(p) <= kSampleMaxBlocks
// entries).  launch_adjoint: Y = G^T y on the support (GT in CSR over the
// support entries, tidx the measurement of each term).
int measure_blocks(int64_t p);
template <typename T>
hipError_t launch_measure(hipStream_t s, const int64_t *gptr, const int32_t *gidx, const T *gval, const T *x,
                          const T *b, T *y, int64_t p, double delta, double *part_out);
template <typename T>
hipError_t launch_adjoint(hipStream_t s, const int64_t *tptr, const int32_t *tidx, const T *tval, const T *y, T *Y,
                          int64_t ns);

// The Dantzig selector's start: Yp = a max(B - E, 0), Ym = a max(-B - E, 0),
// Y = Yp - Ym; with Yp = Ym = null, Y = S_E(B) = sign(B) max(|B| - E, 0).
template <typename T>
hipError_t launch_ds_init(hipStream_t s, const T *B, int64_t n, double E, double a, T *Yp, T *Ym, T *Y);
int sample_blocks(int nrows, int lanes);

// Allocation-free sampled pass: a fixed device array of
// kNoAllocScratchDoubles doubles per device (at least sample_blocks() for
// any size) receives the workgroup partials.  noalloc_scratch(device, &p)
// gives its address on `device`, which must be the current device on the
// first call for that device (the address is looked up with
// hipGetSymbolAddress and cached).  hipErrorInvalidValue for a device index
// outside [0, kMaxDevices), hipErrorInvalidDevice when another device is
// current on that first call.
constexpr int kNoAllocScratchDoubles = kSampleMaxBlocks + 8;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, double **out);

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
