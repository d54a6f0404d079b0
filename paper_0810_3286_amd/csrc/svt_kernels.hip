// gfx950 kernels of the SVT hot path (Algorithm 1 of Cai, Candes and Shen).
//
// Design notes (CDNA4):
//   * 64-lane wavefronts; a compressed row is handled by a sub-wave of
//     `lanes` (4..64) lanes chosen from the mean row length, so that lanes
//     stride contiguous index/value runs (coalesced) and a sub-wave shuffle
//     tree reduces the row;
//   * no kernel uses a device-scope fence or atomic: on a multi-XCD part a
//     release fence writes back the L2 and the fences of different
//     workgroups serialise (tens of microseconds per kernel).  Instead every
//     reduction is split at a kernel boundary: a kernel writes one partial
//     per workgroup, and every workgroup of the next kernel sums those
//     partials itself, in the same fixed order, so all of them hold the same
//     coefficients and the results do not depend on scheduling;
//   * full reorthogonalisation is one classical Gram-Schmidt pass, and its
//     update is deferred into the next sparse product (the product of the
//     basis with the coefficients follows from the bidiagonal relations), so
//     a half-step of the bidiagonalisation is one kernel; after a failed
//     orthogonality check the solver switches to two explicit passes (CGS2);
//     the bidiagonalisation coefficients stay on the device within a step.
#include "svt_kernels.h"

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>

namespace svt {

namespace {

// Events for the next launch of this thread (set_launch_events): the
// runtime stamps them with the kernel's own start and end.
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

}  // namespace

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  t_ev_start = start;
  t_ev_stop = stop;
}

// A launch with pending timing events goes through hipExtLaunchKernelGGL,
// which stamps them (and clears them); otherwise through the plain launch,
// whose host cost is several times lower (the host issues hundreds of
// launches per SVT iteration and must stay ahead of the device).
#define SVT_LAUNCH(kern, grid, block, lds, stream, ...)                                       \
  do {                                                                                        \
    if (t_ev_start != nullptr) {                                                              \
      hipEvent_t ev_a_ = t_ev_start, ev_b_ = t_ev_stop;                                       \
      t_ev_start = t_ev_stop = nullptr;                                                       \
      hipExtLaunchKernelGGL(kern, grid, block, (std::uint32_t)(lds), stream, ev_a_, ev_b_, 0u, \
                            __VA_ARGS__);                                                     \
    } else {                                                                                  \
      hipLaunchKernelGGL(kern, grid, block, lds, stream, __VA_ARGS__);                        \
    }                                                                                         \
  } while (0)

namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;

template <int W, typename A>
__device__ __forceinline__ A seg_sum(A v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_down(v, off, W);
  return v;  // first lane of each W-lane segment holds the sum
}

// Block-wide sum of one double (all threads call; result valid in thread 0).
__device__ __forceinline__ double block_sum(double v, double *sbuf) {
  v = seg_sum<kWave>(v);
  const int w = threadIdx.x / kWave, wl = threadIdx.x % kWave;
  if (wl == 0) sbuf[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += sbuf[i];
  }
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// Norms at or below this are treated as zero: the reciprocal of a larger one
// is finite in the value type.
template <typename T> __device__ __forceinline__ double norm_floor();
template <> __device__ __forceinline__ double norm_floor<double>() { return 1e-280; }
template <> __device__ __forceinline__ double norm_floor<float>() { return 1e-30; }

// ---------------------------------------------------------------------------
// Row-range kernels: kRowBlock threads own the rows [r0, r0 + rows_per_blk)
// of a vector (row_plan); the sparse product and both Gram-Schmidt updates
// use the same partition, so a workgroup's rows were written by the
// workgroup of the same index in the kernel before.
constexpr int kRowWaves = kRowBlock / kWave;   // 16
constexpr int kRowLanes = 128;                 // row slots of the column-group layout
constexpr int kColGroups = kRowBlock / kRowLanes;  // 8 column groups
constexpr int kColsPerPass = 8 * kColGroups;   // 64 columns per pass, 8 per thread

// Block-wide sum of one double over kRowBlock threads (result in thread 0).
__device__ __forceinline__ double row_block_sum(double v, double *sh /* kRowWaves */) {
  v = seg_sum<kWave>(v);
  const int w = threadIdx.x / kWave, wl = threadIdx.x % kWave;
  if (wl == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kRowWaves; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// hs[c] = sum_i part[c * np + i] for c < C (C, np >= 1), into LDS; red:
// kReduceScratch doubles of LDS.  A pass takes 64 columns with 16 strands
// each: strand k of column c adds the partials k, k + 16, ... in order (only
// the threads of existing columns load; within a thread the loads are
// unconditional, from clamped addresses, and issued together: a
// conditional load becomes a branch after which the compiler waits for the
// value), and thread c of the pass adds the 16 strand sums in order.  No
// shuffle trees: every level of a double shuffle is a round trip through
// the LDS crossbar.  Every workgroup gets the same values.  kRowBlock
// threads; ends synchronised.
constexpr int kRedStrands = 16;
constexpr int kRedCols = kRowBlock / kRedStrands;  // 64 columns per pass
constexpr int kRedLoads = 16;                      // loads in flight per strand
static_assert(kReduceScratch >= kRedCols * (kRedStrands + 1), "reduction scratch");
__device__ void reduce_columns(const double *__restrict__ part, int np, int C, double *hs, double *red) {
  const int cl = threadIdx.x / kRedStrands, k = threadIdx.x % kRedStrands;
  for (int cb = 0; cb < C; cb += kRedCols) {
    double t = 0.0;
    if (cb + cl < C) {
      const size_t col = (size_t)(cb + cl) * np;
      for (int i0 = 0; i0 < np; i0 += kRedStrands * kRedLoads) {
        double v[kRedLoads];
#pragma unroll
        for (int j = 0; j < kRedLoads; ++j) v[j] = part[col + min(i0 + k + kRedStrands * j, np - 1)];
#pragma unroll
        for (int j = 0; j < kRedLoads; ++j)
          if (i0 + k + kRedStrands * j < np) t += v[j];
      }
    }
    red[cl * (kRedStrands + 1) + k] = t;  // padded rows: few bank conflicts either way
    __syncthreads();
    if (threadIdx.x < kRedCols && cb + threadIdx.x < C) {
      double u = 0.0;
#pragma unroll
      for (int kk = 0; kk < kRedStrands; ++kk) u += red[threadIdx.x * (kRedStrands + 1) + kk];
      hs[cb + threadIdx.x] = u;
    }
    __syncthreads();
  }
}

// A pending one-pass reorthogonalisation (the bidiagonalisation of Section
// 5.1.1 with full reorthogonalisation): the new vector x of one side is kept
// unorthogonalised, with the partials of its dot products with the nqx basis
// columns Q_x of its side (columns 0 .. nqx - 1 of pend) and of |x|^2
// (column nqx).  reduce_pending sums them into hs (h = hs[0 .. nqx), |x|^2 =
// hs[nqx]) like reduce_columns, and thread 0 then forms |h|^2 and s = |x -
// Q_x h| = sqrt(|x|^2 - |h|^2) (Q_x orthonormal) into scal[0] and scal[1].
// |h|^2: thread t < 64 of each pass adds the squares of its columns in pass
// order, and thread 0 adds the 64 sums in order.  Every workgroup computes
// the same values.  kRowBlock threads; hs is visible to all threads on
// return, scal only to thread 0 until the caller's next barrier.  red:
// kReduceScratch doubles of LDS.
static_assert(kReduceScratch >= kRedCols * (kRedStrands + 2), "reduction scratch");
__device__ void reduce_pending(const double *__restrict__ pend, int np, int nqx, double *hs, double *red,
                               double *scal) {
  const int C = nqx + 1;
  const int cl = threadIdx.x / kRedStrands, k = threadIdx.x % kRedStrands;
  double *sqs = red + kRedCols * (kRedStrands + 1);
  double sq = 0.0;
  if (np == 1) {
    // one partial per column (the sums k_pending_reduce formed, or the
    // output of a one-workgroup product): one load each gives the values
    // the passes below would, and |h|^2 is added in their order (thread
    // t < 64 adds the squares of columns t, t + 64, ... in pass order)
    for (int c = threadIdx.x; c < C; c += blockDim.x) hs[c] = pend[c];
    __syncthreads();
    if (threadIdx.x < kRedCols) {
      for (int c = threadIdx.x; c < nqx; c += kRedCols) sq = fma(hs[c], hs[c], sq);
      sqs[threadIdx.x] = sq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double hh = 0.0;
      if (nqx > 0) {
#pragma unroll
        for (int l = 0; l < kRedCols; ++l) hh += sqs[l];
      }
      scal[0] = hh;
      scal[1] = sqrt(fmax(hs[nqx] - hh, 0.0));
    }
    return;
  }
  for (int cb = 0; cb < C; cb += kRedCols) {
    double t = 0.0;
    if (cb + cl < C) {
      const size_t col = (size_t)(cb + cl) * np;
      for (int i0 = 0; i0 < np; i0 += kRedStrands * kRedLoads) {
        double v[kRedLoads];
#pragma unroll
        for (int j = 0; j < kRedLoads; ++j) v[j] = pend[col + min(i0 + k + kRedStrands * j, np - 1)];
#pragma unroll
        for (int j = 0; j < kRedLoads; ++j)
          if (i0 + k + kRedStrands * j < np) t += v[j];
      }
    }
    red[cl * (kRedStrands + 1) + k] = t;
    __syncthreads();
    if (threadIdx.x < kRedCols) {
      const int c = cb + threadIdx.x;
      if (c < C) {
        double u = 0.0;
#pragma unroll
        for (int kk = 0; kk < kRedStrands; ++kk) u += red[threadIdx.x * (kRedStrands + 1) + kk];
        hs[c] = u;
        if (c < nqx) sq = fma(u, u, sq);
      }
      if (cb + kRedCols >= C) sqs[threadIdx.x] = sq;  // last pass
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double hh = 0.0;
    if (nqx > 0) {
#pragma unroll
      for (int l = 0; l < kRedCols; ++l) hh += sqs[l];
    }
    scal[0] = hh;
    scal[1] = sqrt(fmax(hs[nqx] - hh, 0.0));
  }
}

// Workgroup b writes x_out[i] = (x[i] - sum_c Qx[i, c] h[c]) * inv for its
// slice of [0, ncols) (ceil(ncols / gridDim.x) entries): the pending vector,
// orthogonalised and normalised, joins its basis.  Thread (row slot i, column
// group g) adds the columns g + 8 j of each 64-column pass in order; the
// eight group sums of an entry are added in group order (upd: kRowBlock
// doubles of LDS).  The result does not depend on the slicing.
template <typename T>
__device__ void write_corrected(const T *__restrict__ x, int ncols, const T *__restrict__ Qx, int64_t ldqx,
                                int nqx, const double *h, double inv, T *__restrict__ x_out, double *upd) {
  const int chunk = (ncols + gridDim.x - 1) / gridDim.x;
  const int i0 = blockIdx.x * chunk, i1 = min(ncols, i0 + chunk);
  if (nqx == 0) {
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) x_out[i] = (T)((double)x[i] * inv);
    return;
  }
  const int il = threadIdx.x % kRowLanes, g = threadIdx.x / kRowLanes;
  const int last = nqx - 1;
  for (int rb = i0; rb < i1; rb += kRowLanes) {
    const int row = rb + il;
    const bool valid = row < i1;
    double a = 0.0;
    if (valid) {
      for (int cb = 0; cb < nqx; cb += kColsPerPass) {
        T q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = Qx[(size_t)min(cb + g + 8 * j, last) * ldqx + row];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int c = cb + g + 8 * j;
          if (c < nqx) a = fma((double)q[j], h[c], a);
        }
      }
    }
    upd[g * kRowLanes + il] = a;
    __syncthreads();
    if (g == 0 && valid) {
      double tot = 0.0;
#pragma unroll
      for (int gg = 0; gg < kColGroups; ++gg) tot += upd[gg * kRowLanes + il];
      x_out[row] = (T)(((double)x[row] - tot) * inv);
    }
    __syncthreads();
  }
}

// write_corrected when the slice has at most kRowLanes entries and nqx <
// kColsPerPass: the thread's eight Q_x values of its entry (qx, loaded by
// load_q8 at the slice's entry i0 + row slot) and the entry's x (xv, in the
// column group 0 threads) were loaded earlier.  Same arithmetic and order.
template <typename T>
__device__ void write_corrected_pre(const T (&qx)[8], double xv, int ncols, int nqx, const double *h, double inv,
                                    T *__restrict__ x_out, double *upd) {
  const int chunk = (ncols + gridDim.x - 1) / gridDim.x;
  const int i0 = blockIdx.x * chunk, i1 = min(ncols, i0 + chunk);
  const int il = threadIdx.x % kRowLanes, g = threadIdx.x / kRowLanes;
  const int row = i0 + il;
  const bool valid = row < i1;
  double a = 0.0;
  if (valid) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = g + 8 * j;
      if (c < nqx) a = fma((double)qx[j], h[c], a);
    }
  }
  upd[g * kRowLanes + il] = a;
  __syncthreads();
  if (g == 0 && valid) {
    double tot = 0.0;
#pragma unroll
    for (int gg = 0; gg < kColGroups; ++gg) tot += upd[gg * kRowLanes + il];
    x_out[row] = (T)((xv - tot) * inv);
  }
  __syncthreads();
}

// Partial dot products of the workgroup's rows: part[c * gridDim.x + b] =
// sum_rows Q[row, c] v[row - r0] for c < nq and sum_rows v^2 for c = nq.
// Layout: thread (row slot i, column group g) takes rows r0 + i + 128 t and
// columns cb + g + 8 j (j < 8) of each 64-column pass; its Q loads are
// coalesced across the row slots and issued together.  The row sums reduce
// over the two waves of a column group (shuffles, then LDS), in a fixed order.
template <typename T, typename VF>
__device__ __forceinline__ void row_dots(VF v, int r0, int r1, const T *__restrict__ Q, int64_t ldq, int nq,
                                         double *__restrict__ part, double (*sred)[8]) {
  const int C = nq + 1;
  const int i = threadIdx.x % kRowLanes, g = threadIdx.x / kRowLanes;
  const int w = threadIdx.x / kWave, wl = threadIdx.x % kWave;
  const int last = nq > 0 ? nq - 1 : 0;
  for (int cb = 0; cb < C; cb += kColsPerPass) {
    double acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.0;
    for (int row = r0 + i; row < r1; row += kRowLanes) {
      const double pv = v(row);
      T q[8];
      if (nq > 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = Q[(size_t)min(cb + g + 8 * j, last) * ldq + row];
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = (T)0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = cb + g + 8 * j;
        const double f = (c < nq) ? (double)q[j] : ((c == nq) ? pv : 0.0);
        acc[j] = fma(f, pv, acc[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double sv = seg_sum<kWave>(acc[j]);
      if (wl == 0) sred[w][j] = sv;
    }
    __syncthreads();
    if (threadIdx.x < kColsPerPass) {
      const int gg = threadIdx.x / 8, j = threadIdx.x % 8;
      const int c = cb + gg + 8 * j;
      if (c < C) part[(size_t)c * gridDim.x + blockIdx.x] = sred[2 * gg][j] + sred[2 * gg + 1][j];
    }
    __syncthreads();
  }
}

// Fast path of row_dots when nq < kColsPerPass and the workgroup has at most
// kRowLanes rows: the thread's eight Q values of its row (q, loaded before)
// and its row's value v are already in registers.  The 64 column sums over
// the 128 row slots go through LDS instead of shuffle trees (the double
// shuffles cost more than the rest of the kernel): the products go to buf,
// 16 threads per column add eight of them each, and one thread per column
// adds those 16 in order.  buf: kDotsLds bytes.
constexpr int kDotsLds = sizeof(double) * (8 * kRowBlock + kColsPerPass * 16);

template <typename T>
__device__ __forceinline__ void row_dots_lds(const T (&q)[8], double v, bool valid, int nq,
                                             double *__restrict__ part, double *buf, int cb = 0) {
  // cb: the pass's first column (q holds columns cb + g + 8 j)
  const int C = nq + 1;
  const int g = threadIdx.x / kRowLanes;
  double *prod = buf;                  // 8 x kRowBlock products
  double *mid = buf + 8 * kRowBlock;   // 64 columns x 16 partial sums
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = cb + g + 8 * j;
    const double f = (c < nq) ? (double)q[j] : ((c == nq) ? v : 0.0);
    prod[j * kRowBlock + threadIdx.x] = valid ? f * v : 0.0;
  }
  __syncthreads();
  {
    // column (gg, j) = threadIdx.x / 16: its 128 row-slot products are
    // prod[j][gg * 128 + 0 .. 127]; strand s adds rows s, s + 16, ...
    const int col = threadIdx.x / 16, sidx = threadIdx.x % 16;
    const int gg = col % 8, j = col / 8;
    const double *src = prod + j * kRowBlock + gg * kRowLanes + sidx;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += src[16 * k];
    mid[col * 16 + sidx] = t;
  }
  __syncthreads();
  if (threadIdx.x < kColsPerPass) {
    const int col = threadIdx.x, gg = col % 8, j = col / 8;
    const int c = cb + gg + 8 * j;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += mid[col * 16 + k];
    if (c < C) part[(size_t)c * gridDim.x + blockIdx.x] = t;
  }
}

// The thread's eight Q values of row `row` in the column-group layout
// (columns g + 8 j, clamped to a valid column).  Invalid threads load row 0
// instead, and with nq = 0 or Q null every load reads fallback[0] (a valid
// element): the loads have no branch, so the compiler has no merged value to
// convert, and waits for them only where they are used; every use masks
// them (c < nq, valid rows).
template <typename T>
__device__ __forceinline__ void load_q8(T (&q)[8], const T *__restrict__ Q, int64_t ldq, int nq, int row,
                                        bool valid, const T *__restrict__ fallback, int cb = 0) {
  // cb: first column of the pass (columns cb + g + 8 j)
  const int g = threadIdx.x / kRowLanes;
  const bool have = nq > 0 && Q != nullptr;
  const T *base = have ? Q : fallback;
  const int64_t ld = have ? ldq : 0;
  const int last = have ? nq - 1 : 0;
  const int r = (have && valid) ? row : 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) q[j] = base[(size_t)min(cb + g + 8 * j, last) * ld + r];
}

// The sparse product of one bidiagonalisation half-step, p = A x - s prev
// over one compressed orientation, with x = (x_raw - Q_x h) / s the pending
// vector of the other side (pending_norm; in.pend null: x_raw is normalised,
// s = 1; nqx = 0: x = x_raw / s).  Workgroups also write x to in.x_out
// (write_corrected) and workgroup 0 writes s and |h|^2 / |x_raw|^2.
//
// The product is taken of x_raw: A Q_x h = Q g with g from the bidiagonal
// relations (A v_c = beta_c u_{c-1} + alpha_c u_c and A^T u_c = alpha_c v_c +
// beta_{c+1} v_{c+1}, valid to rounding for the stored, reorthogonalised
// vectors), so p = (A x_raw - Q g) / s - s prev needs only the rows of Q the
// workgroup owns, not all of Q_x.  side 0 (p on the u side, x on the v side,
// nq = nqx): g[c] = alpha[c] h[c] + beta[c + 1] h[c + 1]; side 1 (nq = nqx +
// 1): g[c] = alpha[c] h[c] + beta[c] h[c - 1] (terms with indices outside h
// vanish).  alpha[c], beta[c]: alpha_{c+1}, beta_{c+1}.
//
// PLAIN (a half-step with nothing to orthogonalise: nq = nqx = 0, so no
// update of x and no dot products beyond |p|^2): the same arithmetic without
// the basis loads, whose registers the general kernel holds through the
// product; measured, on average over all half-steps, 16.5 -> 16.1 us at
// 30000^2 (FP64) and 18.1 -> 17.0 us at 10000^2, rank 50.
//
// STAGE: x_raw is copied into LDS in nseg column segments of segcols entries
// (coalesced, every thread's loads issued before its stores) and the
// per-entry gathers hit LDS; otherwise they gather x_raw from memory.
// segptr[row * (nseg + 1) + s] is the first entry of segment s of the row
// (null when nseg == 1: ptr is used).  L lanes take a row and each lane keeps
// kSpmvUnroll entries in flight, accumulating them in index order (the
// result does not depend on the unrolling).  With part_out, the partial dot
// products of p with the nq columns of Q and |p|^2 follow in the same kernel
// (row_dots) with its first ndots columns (nq, or 0 for |p|^2 alone: a vector
// that partial reorthogonalisation leaves alone): p's own pending update.
//
// Order of work: the loads that depend on nothing are issued first (this
// thread's rows of Q and prev, this workgroup's slice of x and Q_x, x's first
// segment), then the pending partials are summed; measured, this beats
// staging x after the update of x is written.
//
// Dynamic LDS: the row sums (16-byte aligned); a region of max(x's segment,
// kDotsLds) bytes rounded up to 16, holding x's segment during the product
// and the dot products' scratch after it; then kSpmvAuxBytes for h, g and
// kReduceScratch partial sums.
constexpr int kSpmvUnroll = 16;
constexpr int kStageVec = 4;  // 16-byte loads in flight per thread while staging x

template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; };
template <> struct Vec16<double> { using type = double2; };

// xs[0 .. cn) = src[0 .. cn); each thread's loads are issued before its
// stores.  FP32: 16-byte loads and stores (four in flight per thread) when
// src is 16-byte aligned (xs is); FP64: sixteen 8-byte loads in flight per
// thread (measured faster than 16-byte loads for a two-segment x).
template <typename T>
__device__ __forceinline__ void stage_segment(const T *__restrict__ src, int cn, T *xs) {
  if constexpr (sizeof(T) == 8) {
    for (int base = threadIdx.x; base < cn; base += kRowBlock * 16) {
      T v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = src[min(base + j * kRowBlock, cn - 1)];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int ii = base + j * kRowBlock;
        if (ii < cn) xs[ii] = v[j];
      }
    }
  } else {
    using V = typename Vec16<T>::type;
    constexpr int kv = 16 / sizeof(T);
    int done = 0;
    if ((reinterpret_cast<uintptr_t>(src) & 15) == 0 && cn >= kv) {
      const int nv = cn / kv;
      const V *s4 = reinterpret_cast<const V *>(src);
      V *d4 = reinterpret_cast<V *>(xs);
      for (int base = threadIdx.x; base < nv; base += kRowBlock * kStageVec) {
        V v[kStageVec];
#pragma unroll
        for (int j = 0; j < kStageVec; ++j) v[j] = s4[min(base + j * kRowBlock, nv - 1)];
#pragma unroll
        for (int j = 0; j < kStageVec; ++j) {
          const int ii = base + j * kRowBlock;
          if (ii < nv) d4[ii] = v[j];
        }
      }
      done = nv * kv;
    }
    for (int ii = done + threadIdx.x; ii < cn; ii += kRowBlock) xs[ii] = src[ii];
  }
}

// stage_segment through the LDS DMA path (global_load_lds_dwordx4): wave w
// copies the 1 KB chunks w, w + 16, ... of src straight into LDS, without
// registers and with every chunk in flight at once; lanes past the end of
// the segment are masked off (a wave's LDS writes are 16 bytes per active
// lane from its uniform chunk base).  src 16-byte aligned; the tail of cn
// that is not a whole 16-byte unit is copied first, by plain loads.  Returns
// with the copies in flight: the caller waits (stage_wait) before the
// barrier after which the segment is read, so that loads issued in between
// travel together with them.
template <typename T>
__device__ __forceinline__ void stage_segment_dma(const T *__restrict__ src, int cn, T *xs) {
  constexpr int kv = 16 / sizeof(T);
  const int nv = cn / kv;
  if (nv * kv < cn)
    for (int ii = nv * kv + threadIdx.x; ii < cn; ii += kRowBlock) xs[ii] = src[ii];
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int nchunks = (nv + kWave - 1) / kWave;
  for (int ch = w; ch < nchunks; ch += kRowWaves) {
    const int e = ch * kWave + l;
    if (e < nv)
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src + (size_t)e * kv),
                                       (__attribute__((address_space(3))) void *)(xs + (size_t)ch * kWave * kv),
                                       16, 0, 0);
  }
}

// This thread's LDS DMA copies have landed (they count as vector memory
// operations); a barrier after it covers the workgroup's.
__device__ __forceinline__ void stage_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The dot products for nq >= kColsPerPass with at most one row per row
// slot: 64 columns per pass through LDS (row_dots_lds with a column base;
// the general row_dots reduces through shuffle trees).  Not inlined, so
// that its registers do not add to the sparse product's.
template <typename T>
__device__ __attribute__((noinline)) void row_dots_passes(const T *racc, int r0, int r1, const T *__restrict__ Q,
                                                          int64_t ldq, int nq, const T *__restrict__ fallback,
                                                          double *__restrict__ part, double *buf) {
  const int il = threadIdx.x % kRowLanes;
  const int row = r0 + il;
  const bool valid = row < r1;
  const double v = valid ? (double)racc[il] : 0.0;
  for (int cb = 0; cb < nq + 1; cb += kColsPerPass) {
    T qa[8];
    load_q8<T>(qa, Q, ldq, nq, row, valid, fallback, cb);
    if (cb > 0) __syncthreads();  // the previous pass's scratch is read
    row_dots_lds<T>(qa, v, valid, nq, part, buf, cb);
  }
}

// The wide-basis passes for row blocks of at most kNarrowLanes rows: the
// same work as the 128-row-slot layout (load_q8, row_dots_lds,
// write_corrected and the correction loop) with 64 row slots and 16 column
// groups, so a pass covers kNarrowCols = 128 columns and a block of 40 rows
// (10000 rows over 250 workgroups) leaves 24 of 64 slots idle instead of 88
// of 128; half as many passes, each one memory round trip and a few
// barriers.  Thread t: row slot t % 64, columns cb + t / 64 + 16 j.
constexpr int kNarrowLanes = 64;
constexpr int kNarrowGroups = kRowBlock / kNarrowLanes;   // 16
constexpr int kNarrowCols = 8 * kNarrowGroups;            // 128 columns per pass
constexpr int kNarrowStrands = kRowBlock / kNarrowCols;   // 8 strands per column

template <typename T>
__device__ __forceinline__ void load_q8_narrow(T (&q)[8], const T *__restrict__ Q, int64_t ldq, int nq, int row,
                                               bool valid, const T *__restrict__ fallback, int cb) {
  const int g = threadIdx.x / kNarrowLanes;
  const bool have = nq > 0 && Q != nullptr;
  const T *base = have ? Q : fallback;
  const int64_t ld = have ? ldq : 0;
  const int last = have ? nq - 1 : 0;
  const int r = (have && valid) ? row : 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) q[j] = base[(size_t)min(cb + g + kNarrowGroups * j, last) * ld + r];
}

// One pass of the dot products in the narrow layout: columns cb + gg + 16 j
// of Q (and column nq: |p|^2), each summed over the 64 row slots by 8
// strands of 8 slots, then the 8 strand sums in order.  buf: kDotsLds bytes.
template <typename T>
__device__ __forceinline__ void row_dots_lds_narrow(const T (&q)[8], double v, bool valid, int nq,
                                                    double *__restrict__ part, double *buf, int cb) {
  static_assert(8 * kRowBlock + kNarrowCols * kNarrowStrands <= kDotsLds / (int)sizeof(double), "dots scratch");
  const int C = nq + 1;
  const int g = threadIdx.x / kNarrowLanes;
  double *prod = buf;                  // 8 x kRowBlock products
  double *mid = buf + 8 * kRowBlock;   // 128 columns x 8 partial sums
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = cb + g + kNarrowGroups * j;
    const double f = (c < nq) ? (double)q[j] : ((c == nq) ? v : 0.0);
    prod[j * kRowBlock + threadIdx.x] = valid ? f * v : 0.0;
  }
  __syncthreads();
  {
    const int col = threadIdx.x / kNarrowStrands, sidx = threadIdx.x % kNarrowStrands;
    const int gg = col % kNarrowGroups, j = col / kNarrowGroups;
    const double *src = prod + j * kRowBlock + gg * kNarrowLanes + sidx;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kNarrowLanes / kNarrowStrands; ++k) t += src[kNarrowStrands * k];
    mid[col * kNarrowStrands + sidx] = t;
  }
  __syncthreads();
  if (threadIdx.x < kNarrowCols) {
    const int col = threadIdx.x, gg = col % kNarrowGroups, j = col / kNarrowGroups;
    const int c = cb + gg + kNarrowGroups * j;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kNarrowStrands; ++k) t += mid[col * kNarrowStrands + k];
    if (c < C) part[(size_t)c * gridDim.x + blockIdx.x] = t;
  }
}

template <typename T>
__device__ __attribute__((noinline)) void row_dots_passes_narrow(const T *racc, int r0, int r1,
                                                                 const T *__restrict__ Q, int64_t ldq, int nq,
                                                                 const T *__restrict__ fallback,
                                                                 double *__restrict__ part, double *buf) {
  const int il = threadIdx.x % kNarrowLanes;
  const int row = r0 + il;
  const bool valid = row < r1;
  const double v = valid ? (double)racc[il] : 0.0;
  for (int cb = 0; cb < nq + 1; cb += kNarrowCols) {
    T qa[8];
    load_q8_narrow<T>(qa, Q, ldq, nq, row, valid, fallback, cb);
    if (cb > 0) __syncthreads();  // the previous pass's scratch is read
    row_dots_lds_narrow<T>(qa, v, valid, nq, part, buf, cb);
  }
}

// Sum over the narrow layout's column passes of Q[row, c] * w[c] (c < nq)
// for this thread's row slot and column group, in pass order.
template <typename T>
__device__ __forceinline__ double narrow_combine(const T *__restrict__ Q, int64_t ldq, int nq, int row,
                                                 const double *w) {
  const int g = threadIdx.x / kNarrowLanes;
  const int last = nq - 1;
  double a = 0.0;
  for (int cb = 0; cb < nq; cb += kNarrowCols) {
    T q[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) q[j] = Q[(size_t)min(cb + g + kNarrowGroups * j, last) * ldq + row];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = cb + g + kNarrowGroups * j;
      if (c < nq) a = fma((double)q[j], w[c], a);
    }
  }
  return a;
}

// write_corrected for a slice of at most kNarrowLanes entries (nqx >= 1):
// x_out[i] = (x[i] - sum_c Qx[i, c] h[c]) * inv, the 16 group sums of an
// entry added in group order (upd: kRowBlock doubles of LDS).
template <typename T>
__device__ void write_corrected_narrow(const T *__restrict__ x, int ncols, const T *__restrict__ Qx, int64_t ldqx,
                                       int nqx, const double *h, double inv, T *__restrict__ x_out, double *upd) {
  const int chunk = (ncols + gridDim.x - 1) / gridDim.x;
  const int i0 = blockIdx.x * chunk, i1 = min(ncols, i0 + chunk);
  const int il = threadIdx.x % kNarrowLanes, g = threadIdx.x / kNarrowLanes;
  const int row = i0 + il;
  const bool valid = row < i1;
  const double a = valid ? narrow_combine<T>(Qx, ldqx, nqx, row, h) : 0.0;
  upd[g * kNarrowLanes + il] = a;
  __syncthreads();
  if (g == 0 && valid) {
    double tot = 0.0;
#pragma unroll
    for (int gg = 0; gg < kNarrowGroups; ++gg) tot += upd[gg * kNarrowLanes + il];
    x_out[row] = (T)(((double)x[row] - tot) * inv);
  }
  __syncthreads();
}

template <typename T, typename I, int L, bool STAGE, bool PLAIN>
__global__ __launch_bounds__(kRowBlock) void k_spmv_rows(
    const int32_t *__restrict__ ptr, const I *__restrict__ idx, const T *__restrict__ val,
    const int32_t *__restrict__ segptr, int nseg, int segcols, const SpmvInput<T> in, int ncols,
    const T *__restrict__ prev, T *__restrict__ p, int nrows, int rows_per_blk, const T *__restrict__ Q,
    int64_t ldq, int nq, int ndots, double *__restrict__ part_out) {
  extern __shared__ double smem_d[];
  __shared__ double sred[kRowWaves][8];
  T *racc = reinterpret_cast<T *>(smem_d);  // rows_per_blk row sums, then the rows of p
  const size_t racc_bytes = ((sizeof(T) * rows_per_blk + 15) / 16) * 16;
  char *region = reinterpret_cast<char *>(smem_d) + racc_bytes;
  const size_t xseg_bytes = sizeof(T) * (size_t)segcols;
  const size_t region_bytes = ((xseg_bytes > (size_t)kDotsLds ? xseg_bytes : (size_t)kDotsLds) + 15) / 16 * 16;
  T *xs = reinterpret_cast<T *>(region);                          // x's segment (STAGE)
  double *hs = reinterpret_cast<double *>(region + region_bytes);  // h, |x_raw|^2: kSpmvAuxCols + 1
  double *gl = hs + kSpmvAuxCols + 1;                               // g: kSpmvAuxCols
  double *upd = gl + kSpmvAuxCols + 1;                              // kReduceScratch partial sums
  __shared__ double scal[2];  // |h|^2, s (reduce_pending)
  const bool corr = !PLAIN && in.nqx > 0;
  const int il = threadIdx.x % kRowLanes, g = threadIdx.x / kRowLanes;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  constexpr int kGroups = kRowBlock / L;
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  // x staged in LDS and at most one row per lane group: the row's bounds in
  // the first segment are loaded first, its first half batch of entries
  // right after the other independent loads, so both round trips overlap
  // the staging of x and the pending update (a full batch held that long
  // would spill; loading a later segment's bounds during its staging, too,
  // made the FP64 kernel spill and measured slower)
  const bool early = STAGE && L >= 8 && rows_per_blk <= kGroups;
  const int erow = r0 + grp;
  int ebeg = 0, eend = 0;
  if (early && erow < r1) {
    if (nseg == 1) {
      ebeg = ptr[erow];
      eend = ptr[erow + 1];
    } else {
      ebeg = segptr[(size_t)erow * (nseg + 1)];
      eend = segptr[(size_t)erow * (nseg + 1) + 1];
    }
  }
  // this thread's Q values and prev for the epilogue (rows of at most
  // kRowLanes per workgroup and nq < kColsPerPass)
  const bool fast = (part_out != nullptr || corr) && nq < kColsPerPass && rows_per_blk <= kRowLanes;
  const int frow = blockIdx.x * rows_per_blk + il;
  const bool fvalid = fast && il < rows_per_blk && frow < nrows;
  T q8[8];
  if constexpr (PLAIN) {
#pragma unroll
    for (int j = 0; j < 8; ++j) q8[j] = (T)0;
  } else {
    load_q8<T>(q8, Q, ldq, nq, frow, fvalid, in.x);
  }
  const T prev8 = (prev != nullptr ? prev : in.x)[(fvalid && prev != nullptr) ? frow : 0];
  // this workgroup's slice of x and its rows of Q_x (x' = (x - Q_x h) / s),
  // one entry per row slot: loaded now in FP32, after the product in FP64
  // (whose product loop has no registers to spare)
  const int xchunk = (ncols + gridDim.x - 1) / gridDim.x;
  const int xrow = blockIdx.x * xchunk + il;
  const bool xfast = in.x_out != nullptr && xchunk <= kRowLanes && in.nqx < kColsPerPass;
  const bool xvalid = xfast && il < xchunk && xrow < ncols;
  constexpr bool kEarlyX = sizeof(T) == 4;
  T qx8[8];
  T xv0 = (T)0;
  if constexpr (PLAIN) {
#pragma unroll
    for (int j = 0; j < 8; ++j) qx8[j] = (T)0;
  }
  if (kEarlyX) {
    if constexpr (!PLAIN) load_q8<T>(qx8, in.Qx, in.ldqx, in.nqx, xrow, xvalid, in.x);
    xv0 = in.x[xvalid ? xrow : 0];
  }
  // the bidiagonal coefficients of g (thread c = threadIdx.x < nq <=
  // kSpmvAuxCols = kRowBlock needs alpha[c] and beta[c + 1] (side 0) or
  // beta[c] (side 1)), from clamped indices: loaded here in FP32, just
  // before g in FP64 (no registers to spare there)
  const int gc = threadIdx.x;
  double ga = 0.0, gb = 0.0;
  auto load_g = [&]() {
    if (corr) {
      ga = in.alpha[min(gc, in.nqx - 1)];
      gb = in.side == 0 ? in.beta[min(gc + 1, in.nqx - 1)] : in.beta[min(gc, in.nqx)];
    }
  };
  if constexpr (sizeof(T) == 4) load_g();
  constexpr int kEarly = kSpmvUnroll / 2;
  int eii[kEarly];
  T evv[kEarly];
  if (early) {
#pragma unroll
    for (int j = 0; j < kEarly; ++j) {
      const int t = ebeg + lane + j * L;
      const bool inr = t < eend;
      eii[j] = inr ? (int)idx[t] : 0;
      evv[j] = inr ? val[t] : (T)0;
    }
  }
  const T *x = in.x;
  if constexpr (STAGE) stage_segment_dma<T>(x, min(segcols, ncols), xs);
  // h, |x|^2 (all threads), then s (thread 0; the others read it after the
  // next barrier) and g
  if (in.pend != nullptr) {
    reduce_pending(in.pend, in.np, in.nqx, hs, upd, scal);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (in.removed_out != nullptr) {
        const double nn = hs[in.nqx];
        *in.removed_out = nn > 0.0 ? scal[0] / nn : 0.0;
      }
      if (in.s_out != nullptr) *in.s_out = scal[1];
    }
  } else {
    if (threadIdx.x == 0) scal[1] = 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && in.s_out != nullptr) *in.s_out = 1.0;
  }
  if constexpr (sizeof(T) == 8) load_g();
  if (corr && gc < nq) {
    double t = 0.0;
    if (gc < in.nqx) t = ga * hs[gc];
    if (in.side == 0) {
      if (gc + 1 < in.nqx) t = fma(gb, hs[gc + 1], t);
    } else {
      if (gc >= 1 && gc - 1 < in.nqx) t = fma(gb, hs[gc - 1], t);
    }
    gl[gc] = t;
  }
  const int nsg = STAGE ? nseg : 1;
  for (int sgm = 0; sgm < nsg; ++sgm) {
    const int c0 = STAGE ? sgm * segcols : 0;
    const T *xv = x;
    if constexpr (STAGE) {
      if (sgm > 0) {
        __syncthreads();  // the previous segment's gathers are done
        stage_segment_dma<T>(x + c0, min(segcols, ncols - c0), xs);
      }
      stage_wait();
      __syncthreads();
      xv = xs;
    }
    for (int row = r0 + grp; row < r1; row += kGroups) {
      int beg, end;
      const bool pre = early && sgm == 0;  // the first segment's batch was loaded early
      if (pre) {
        beg = ebeg;  // row == erow: one row per lane group
        end = eend;
      } else if (!STAGE || nseg == 1) {
        beg = ptr[row];
        end = ptr[row + 1];
      } else {
        beg = segptr[(size_t)row * (nseg + 1) + sgm];
        end = segptr[(size_t)row * (nseg + 1) + sgm + 1];
      }
      T acc = (T)0;
      int t = beg + lane;
      if (pre) {
        // the first batch arrived with the early loads (same order)
#pragma unroll
        for (int j = 0; j < kEarly; ++j)
          if (t + j * L < end) acc = fma(evv[j], xv[eii[j]], acc);
        t += kEarly * L;
      }
      for (; t + (kSpmvUnroll - 1) * L < end; t += kSpmvUnroll * L) {
        int ii[kSpmvUnroll];
        T vv[kSpmvUnroll];
#pragma unroll
        for (int j = 0; j < kSpmvUnroll; ++j) {
          ii[j] = (int)idx[t + j * L];
          vv[j] = val[t + j * L];
        }
#pragma unroll
        for (int j = 0; j < kSpmvUnroll; ++j) acc = fma(vv[j], xv[ii[j] - c0], acc);
      }
      if (t < end) {
        // fewer than kSpmvUnroll entries left: one masked batch, same order
        int ii[kSpmvUnroll];
        T vv[kSpmvUnroll];
#pragma unroll
        for (int j = 0; j < kSpmvUnroll; ++j) {
          const bool inr = t + j * L < end;
          ii[j] = inr ? (int)idx[t + j * L] : c0;
          vv[j] = inr ? val[t + j * L] : (T)0;
        }
#pragma unroll
        for (int j = 0; j < kSpmvUnroll; ++j)
          if (t + j * L < end) acc = fma(vv[j], xv[ii[j] - c0], acc);
      }
      acc = seg_sum<L>(acc);
      if (lane == 0) racc[row - r0] = (sgm == 0) ? acc : racc[row - r0] + acc;
    }
  }
  if (!kEarlyX) {
    if constexpr (!PLAIN) load_q8<T>(qx8, in.Qx, in.ldqx, in.nqx, xrow, xvalid, in.x);
    xv0 = in.x[xvalid ? xrow : 0];
  }
  __syncthreads();  // racc complete, s published; the region is free again
  const double sn = scal[1];
  const double inv = (sn > norm_floor<T>()) ? 1.0 / sn : 0.0;
  double *updp = reinterpret_cast<double *>(region);  // the epilogue's partial sums
  if (xfast && fast) {
    // x' and p in one round: thread (row slot, column group) adds its
    // columns of Q_x h and Q g, and the group sums are added in group order
    double ax = 0.0, ap = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = g + 8 * j;
      if (xvalid && c < in.nqx) ax = fma((double)qx8[j], hs[c], ax);
      if (corr && fvalid && c < nq) ap = fma((double)q8[j], gl[c], ap);
    }
    upd[g * kRowLanes + il] = ax;
    updp[g * kRowLanes + il] = ap;
    __syncthreads();
    if (g == 0) {
      if (xvalid) {
        double tx = 0.0;
#pragma unroll
        for (int gg = 0; gg < kColGroups; ++gg) tx += upd[gg * kRowLanes + il];
        in.x_out[xrow] = (T)(((double)xv0 - tx) * inv);
      }
      if (fvalid) {
        double tp = 0.0;
#pragma unroll
        for (int gg = 0; gg < kColGroups; ++gg) tp += updp[gg * kRowLanes + il];
        double y = ((double)racc[il] - tp) * inv;
        if (prev != nullptr) y = fma(-sn, (double)prev8, y);
        const T pv = (T)y;
        p[frow] = pv;
        racc[il] = pv;
      }
    }
    __syncthreads();
  } else {
    if (xfast) {
      write_corrected_pre<T>(qx8, (double)xv0, ncols, in.nqx, hs, inv, in.x_out, upd);
    } else if (in.x_out != nullptr) {
      if (in.nqx > 0 && xchunk <= kNarrowLanes)
        write_corrected_narrow<T>(x, ncols, in.Qx, in.ldqx, in.nqx, hs, inv, in.x_out, upd);
      else
        write_corrected<T>(x, ncols, in.Qx, in.ldqx, in.nqx, hs, inv, in.x_out, upd);
    }
    if (corr && !fast && nq > 0 && rows_per_blk <= kNarrowLanes) {
      // p = (A x_raw - Q g) / s - s prev in the narrow layout
      const int nl = threadIdx.x % kNarrowLanes, ng = threadIdx.x / kNarrowLanes;
      const int row = r0 + nl;
      const bool valid = row < r1;
      const double a = valid ? narrow_combine<T>(Q, ldq, nq, row, gl) : 0.0;
      updp[ng * kNarrowLanes + nl] = a;
      __syncthreads();
      if (ng == 0 && valid) {
        double tot = 0.0;
#pragma unroll
        for (int gg = 0; gg < kNarrowGroups; ++gg) tot += updp[gg * kNarrowLanes + nl];
        double y = ((double)racc[row - r0] - tot) * inv;
        if (prev != nullptr) y = fma(-sn, (double)prev[row], y);
        const T pv = (T)y;
        p[row] = pv;
        racc[row - r0] = pv;
      }
      __syncthreads();
    } else if (corr) {
      // p = (A x_raw - Q g) / s - s prev, Q g summed like write_corrected
      const int last = nq > 0 ? nq - 1 : 0;
      for (int rb = r0; rb < r1; rb += kRowLanes) {
        const int row = rb + il;
        const bool valid = row < r1;
        double a = 0.0;
        if (fast) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int c = g + 8 * j;
            if (fvalid && c < nq) a = fma((double)q8[j], gl[c], a);
          }
        } else if (valid) {
          for (int cb = 0; cb < nq; cb += kColsPerPass) {
            T q[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) q[j] = Q[(size_t)min(cb + g + 8 * j, last) * ldq + row];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int c = cb + g + 8 * j;
              if (c < nq) a = fma((double)q[j], gl[c], a);
            }
          }
        }
        updp[g * kRowLanes + il] = a;
        __syncthreads();
        if (g == 0 && valid) {
          double tot = 0.0;
#pragma unroll
          for (int gg = 0; gg < kColGroups; ++gg) tot += updp[gg * kRowLanes + il];
          double y = ((double)racc[row - r0] - tot) * inv;
          if (prev != nullptr) y = fma(-sn, (double)(fast ? prev8 : prev[row]), y);
          const T pv = (T)y;
          p[row] = pv;
          racc[row - r0] = pv;
        }
        __syncthreads();
      }
    } else {
      for (int row = r0 + threadIdx.x; row < r1; row += kRowBlock) {
        // with `fast`, a workgroup has at most kRowLanes rows and thread i
        // (< kRowLanes) loaded prev of row r0 + i at the start
        double y = (double)racc[row - r0] * inv;
        if (prev != nullptr) y = fma(-sn, (double)(fast ? prev8 : prev[row]), y);
        const T pv = (T)y;
        p[row] = pv;
        racc[row - r0] = pv;
      }
      __syncthreads();
    }
  }
  if (part_out == nullptr) return;  // uniform
  if (fast) {
    row_dots_lds<T>(q8, fvalid ? (double)racc[frow - r0] : 0.0, fvalid, ndots, part_out,
                    reinterpret_cast<double *>(region));
  } else if (rows_per_blk <= kNarrowLanes) {
    row_dots_passes_narrow<T>(racc, r0, r1, Q, ldq, ndots, in.x, part_out, reinterpret_cast<double *>(region));
  } else if (rows_per_blk <= kRowLanes) {
    row_dots_passes<T>(racc, r0, r1, Q, ldq, ndots, in.x, part_out, reinterpret_cast<double *>(region));
  } else {
    row_dots<T>([&](int row) { return (double)racc[row - r0]; }, r0, r1, Q, ldq, ndots, part_out, sred);
  }
}

// The column sums of a pending vector's partials (nqx + 1 columns of np),
// formed exactly as reduce_pending forms them (the same strands, added in
// the same order), into out[0 .. nqx].  A consumer given out as a single
// partial (np = 1) takes the same values with one load each, where every
// workgroup of a sparse product would otherwise read all (nqx + 1) np
// partials in 64-column passes.  kPreCols columns per workgroup.
constexpr int kPreCols = 16;
__global__ __launch_bounds__(kPreCols * kRedStrands) void k_pending_reduce(const double *__restrict__ pend, int np,
                                                                           int C, double *__restrict__ out) {
  __shared__ double red[kPreCols * (kRedStrands + 1)];
  const int cl = threadIdx.x / kRedStrands, k = threadIdx.x % kRedStrands;
  const int c = blockIdx.x * kPreCols + cl;
  double t = 0.0;
  if (c < C) {
    const size_t col = (size_t)c * np;
    for (int i0 = 0; i0 < np; i0 += kRedStrands * kRedLoads) {
      double v[kRedLoads];
#pragma unroll
      for (int j = 0; j < kRedLoads; ++j) v[j] = pend[col + min(i0 + k + kRedStrands * j, np - 1)];
#pragma unroll
      for (int j = 0; j < kRedLoads; ++j)
        if (i0 + k + kRedStrands * j < np) t += v[j];
    }
  }
  red[cl * (kRedStrands + 1) + k] = t;
  __syncthreads();
  if (threadIdx.x < kPreCols) {
    const int cc = blockIdx.x * kPreCols + threadIdx.x;
    if (cc < C) {
      double u = 0.0;
#pragma unroll
      for (int kk = 0; kk < kRedStrands; ++kk) u += red[threadIdx.x * (kRedStrands + 1) + kk];
      out[cc] = u;
    }
  }
}

// s and |h|^2 / |x_raw|^2 of a pending vector (pending_norm, the same
// arithmetic as the sparse product that consumes it) into *s_out and
// *removed_out (may be null).  One workgroup; dynamic LDS: nqx + 1 doubles.
__global__ __launch_bounds__(kRowBlock) void k_pending_norm(const double *__restrict__ pend, int np, int nqx,
                                                            double *__restrict__ s_out,
                                                            double *__restrict__ removed_out) {
  extern __shared__ double hs_d[];
  __shared__ double scal[2];
  __shared__ double red[kReduceScratch];
  reduce_pending(pend, np, nqx, hs_d, red, scal);
  if (threadIdx.x == 0) {
    *s_out = scal[1];
    if (removed_out != nullptr) *removed_out = hs_d[nqx] > 0.0 ? scal[0] / hs_d[nqx] : 0.0;
  }
}

// p <- p - Q h over the workgroup's rows, with h = the column sums of
// part_in (np_in partials each, reduced by every workgroup).  Each thread
// takes the 8-column slices of its column group (loads batched), the eight
// group sums of a row are added in group order.  SECOND = false: the partial
// dot products of the new p with Q and itself follow (the second pass's
// coefficients); SECOND = true: only the |p|^2 partials.
// Fraction of |p|^2 that the pass removes, |h|^2 / |p|^2 (h = Q^T p in hs,
// |p|^2 in hs[nq]), written by workgroup 0 to *removed (when not null):
// the orthogonality check of a one-pass reorthogonalisation.
__device__ __forceinline__ void record_removed(const double *hs, int nq, double *removed) {
  if (removed == nullptr || blockIdx.x != 0 || threadIdx.x != 0) return;
  double hh = 0.0;
  for (int c = 0; c < nq; ++c) hh = fma(hs[c], hs[c], hh);
  *removed = hs[nq] > 0.0 ? hh / hs[nq] : 0.0;
}

template <typename T, bool SECOND>
__global__ __launch_bounds__(kRowBlock) void k_gs_update(T *__restrict__ p, int nrows, int rows_per_blk,
                                                         const T *__restrict__ Q, int64_t ldq, int nq,
                                                         const double *__restrict__ part_in, int np_in,
                                                         double *__restrict__ part_out,
                                                         double *__restrict__ removed) {
  extern __shared__ double smem[];
  double *hs = smem;                       // nq + 1 coefficients
  double *pc = hs + nq + 1;                // rows_per_blk values of the new p
  double *upd = pc + rows_per_blk;         // kReduceScratch: partial updates, reduction scratch
  double *dbuf = upd + kReduceScratch;     // kDotsLds bytes for the fused dot products
  __shared__ double sh[kRowWaves];
  __shared__ double sred[kRowWaves][8];
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  const int i = threadIdx.x % kRowLanes, g = threadIdx.x / kRowLanes;
  if (nq < kColsPerPass && rows_per_blk <= kRowLanes) {
    // fast path: one row per row slot and at most eight columns per thread;
    // the Q values and p are loaded before the coefficients are summed, and
    // the Q values are reused by the fused dot products
    const int row = r0 + i;
    const bool valid = row < r1;
    T q[8];
    load_q8<T>(q, Q, ldq, nq, row, valid, p);
    const T p0 = p[valid ? row : r0];
    reduce_columns(part_in, np_in, nq + 1, hs, upd);
    record_removed(hs, nq, removed);
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = g + 8 * j;
      if (c < nq) a = fma((double)q[j], hs[c], a);
    }
    upd[g * kRowLanes + i] = a;
    __syncthreads();
    if (g == 0 && valid) {
      double tot = 0.0;
#pragma unroll
      for (int gg = 0; gg < kColGroups; ++gg) tot += upd[gg * kRowLanes + i];
      const T pv = (T)((double)p0 - tot);
      p[row] = pv;
      pc[i] = (double)pv;
    }
    __syncthreads();
    const double pn = valid ? pc[i] : 0.0;
    if constexpr (!SECOND) {
      row_dots_lds<T>(q, pn, valid, nq, part_out, dbuf);
    } else {
      const double tot = row_block_sum(g == 0 ? pn * pn : 0.0, sh);
      if (threadIdx.x == 0) part_out[blockIdx.x] = tot;
    }
    return;
  }
  reduce_columns(part_in, np_in, nq + 1, hs, upd);
  record_removed(hs, nq, removed);
  const int last = nq - 1;
  for (int rb = r0; rb < r1; rb += kRowLanes) {
    const int row = rb + i;
    const bool valid = row < r1;
    double a = 0.0;
    if (valid) {
      for (int cb = 0; cb < nq; cb += kColsPerPass) {
        T q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = Q[(size_t)min(cb + g + 8 * j, last) * ldq + row];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int c = cb + g + 8 * j;
          if (c < nq) a = fma((double)q[j], hs[c], a);
        }
      }
    }
    upd[g * kRowLanes + i] = a;
    __syncthreads();
    if (g == 0 && valid) {
      double tot = 0.0;
#pragma unroll
      for (int gg = 0; gg < kColGroups; ++gg) tot += upd[gg * kRowLanes + i];
      const T pv = (T)((double)p[row] - tot);
      p[row] = pv;
      pc[row - r0] = (double)pv;
    }
    __syncthreads();
  }
  if constexpr (!SECOND) {
    row_dots<T>([&](int row) { return pc[row - r0]; }, r0, r1, Q, ldq, nq, part_out, sred);
  } else {
    double ss = 0.0;
    for (int row = r0 + threadIdx.x; row < r1; row += kRowBlock) ss = fma(pc[row - r0], pc[row - r0], ss);
    const double tot = row_block_sum(ss, sh);
    if (threadIdx.x == 0) part_out[blockIdx.x] = tot;
  }
}

// |p|^2 partials of the workgroup's rows (row_plan partition).
template <typename T>
__global__ __launch_bounds__(kRowBlock) void k_sumsq(const T *__restrict__ p, int nrows, int rows_per_blk,
                                                     double *__restrict__ part_out) {
  __shared__ double sh[kRowWaves];
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  double ss = 0.0;
  for (int row = r0 + threadIdx.x; row < r1; row += kRowBlock) {
    const double v = (double)p[row];
    ss = fma(v, v, ss);
  }
  const double tot = row_block_sum(ss, sh);
  if (threadIdx.x == 0) part_out[blockIdx.x] = tot;
}

// out = p / |p| with |p|^2 = the sum of part[0..np) (pending_norm with no
// basis columns: the same arithmetic as the sparse product that would
// normalise it); workgroup 0 stores |p| in *coef_out.  out = 0 when |p|
// underflows.
template <typename T>
__global__ __launch_bounds__(kRowBlock) void k_gs_scale(const T *__restrict__ p, int n,
                                                        const double *__restrict__ part, int np,
                                                        T *__restrict__ out, double *__restrict__ coef_out) {
  __shared__ double hs[1];
  __shared__ double scal[2];
  __shared__ double red[kReduceScratch];
  reduce_pending(part, np, 0, hs, red, scal);
  __syncthreads();
  const double nrm = scal[1];
  const double inv = (nrm > norm_floor<T>()) ? 1.0 / nrm : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *coef_out = nrm;
  for (int i = blockIdx.x * kRowBlock + threadIdx.x; i < n; i += gridDim.x * kRowBlock)
    out[i] = (T)((double)p[i] * inv);
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014) as a counter-based hash.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_randn(T *__restrict__ out, int n, uint64_t seed, uint64_t ctr) {
  const uint64_t key = mix64(seed ^ mix64(ctr));
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const uint64_t a = mix64(key + 2ull * (uint64_t)i);
    const uint64_t b = mix64(key + 2ull * (uint64_t)i + 1ull);
    // Box-Muller on two uniforms in (0, 1]
    const double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    out[i] = (T)(sqrt(-2.0 * log(u1)) * cospi(2.0 * u2));
  }
}

// Ritz vectors: out[i, l] = w[l] sum_c Q[i, c] P[c, l] for l < r, zero for
// r <= l < rs: a tall-skinny product (rows x k) times (k x r), on the FP64
// matrix cores (v_mfma_f64_16x16x4f64; FP32 bases are widened on load, so the
// sums are FP64 in both precisions).  A workgroup owns kRitzRT 16-row tiles
// and up to 64 output columns (four 16-column tiles; wider factors take more
// workgroups along y), so every basis entry is read once per 64 output
// columns.  The k basis columns are cut into 16-column chunks dealt round
// robin to the four wavefronts (wave w takes chunks w, w + 4, ...); each wave
// accumulates its chunks for all the workgroup's rows and columns, reading
// the P entries it multiplies straight from memory (P is small and stays in
// L2), and issues the next chunk's loads before the current chunk's matrix
// operations, so no barrier sits in the loop.  The four partial products are
// added through LDS in wave order at the end.  Loads use clamped addresses;
// a P entry outside (c < k, l < r) is taken as zero, which also cancels the
// clamped basis columns; rows past the end are computed but not stored.
// Operand layouts of the 16x16x4 FP64 instruction, lane l: A[l % 16][l / 16]
// (row, c), B[l / 16][l % 16] (c, column), and element v of the result holds
// D[l / 16 + 4 v][l % 16] (rows interleaved by four; checked on the device).
constexpr int kRitzRT = 1;         // 16-row tiles per workgroup
constexpr int kRitzCols = 64;      // output columns per workgroup
constexpr int kRitzKc = 16;        // basis columns per chunk (4 matrix steps)
constexpr int kRitzWaves = 4;
constexpr int kRitzThreads = kRitzWaves * kWave;
using d4_t = __attribute__((ext_vector_type(4))) double;

template <typename T, int NT>
struct RitzChunk {
  T a[kRitzRT][kRitzKc / 4];  // basis values, as loaded
  double b[kRitzKc / 4][NT];  // P values, as loaded (masked where used)
};

template <typename T, int NT>
__device__ __forceinline__ void ritz_load(RitzChunk<T, NT> &ch, const T *const (&qrow)[kRitzRT], int64_t ldq,
                                          const double *__restrict__ P, int r, int k, int c0, int kq, int pcol0,
                                          int lane16) {
#pragma unroll
  for (int st = 0; st < kRitzKc / 4; ++st) {
    const int c = c0 + 4 * st + kq;
    const int cc = min(c, k - 1);
#pragma unroll
    for (int rt = 0; rt < kRitzRT; ++rt) ch.a[rt][st] = qrow[rt][(size_t)cc * ldq];
#pragma unroll
    for (int t = 0; t < NT; ++t) ch.b[st][t] = P[(size_t)cc * r + min(pcol0 + t * 16 + lane16, r - 1)];
  }
}

template <typename T, int NT>
__global__ __launch_bounds__(kRitzThreads) void k_ritz(const T *__restrict__ Q, int64_t ldq, int nrows, int k,
                                                       const double *__restrict__ P, const double *__restrict__ w,
                                                       int r, T *__restrict__ out, int rs) {
  // the partial products of waves 1..3: [wave - 1][rt][t][v][lane]
  __shared__ double red[(kRitzWaves - 1) * kRitzRT * NT * 4 * kWave];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int kq = lane / 16, lane16 = lane % 16;
  const int row0 = blockIdx.x * (16 * kRitzRT);
  const int l0 = blockIdx.y * kRitzCols;
  const T *qrow[kRitzRT];
#pragma unroll
  for (int rt = 0; rt < kRitzRT; ++rt) qrow[rt] = Q + min(row0 + rt * 16 + lane16, nrows - 1);
  d4_t acc[kRitzRT][NT];
#pragma unroll
  for (int rt = 0; rt < kRitzRT; ++rt)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[rt][t] = d4_t{0.0, 0.0, 0.0, 0.0};
  const int nchunks = (k + kRitzKc - 1) / kRitzKc;
  // the P entries outside l < r (the same for every chunk)
  bool colok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) colok[t] = l0 + t * 16 + lane16 < r;
  auto mma = [&](const RitzChunk<T, NT> &ch, int jc, bool use) {
#pragma unroll
    for (int st = 0; st < kRitzKc / 4; ++st) {
      const bool cok = use && jc * kRitzKc + 4 * st + kq < k;
#pragma unroll
      for (int rt = 0; rt < kRitzRT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const double b = (cok && colok[t]) ? ch.b[st][t] : 0.0;
          acc[rt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ch.a[rt][st], b, acc[rt][t], 0, 0, 0);
        }
    }
  };
  // two chunks per round: both chunks' loads are issued before the first
  // chunk's matrix operations, which then wait only for their own operands
  // while the second chunk's are in flight.  Past the wave's last chunk the
  // second load repeats the first (already in cache) and its P operands are
  // taken as zero (an unconditional use keeps the loads where they are).
  RitzChunk<T, NT> c0, c1;
  for (int j = wave; j < nchunks; j += 2 * kRitzWaves) {
    const int j1 = j + kRitzWaves < nchunks ? j + kRitzWaves : j;
    ritz_load(c0, qrow, ldq, P, r, k, j * kRitzKc, kq, l0, lane16);
    ritz_load(c1, qrow, ldq, P, r, k, j1 * kRitzKc, kq, l0, lane16);
    mma(c0, j, true);
    mma(c1, j1, j1 != j);
  }
  if (wave > 0) {
#pragma unroll
    for (int rt = 0; rt < kRitzRT; ++rt)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[((((wave - 1) * kRitzRT + rt) * NT + t) * 4 + v) * kWave + lane] = acc[rt][t][v];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int rt = 0; rt < kRitzRT; ++rt)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = l0 + t * 16 + lane16;
      const double scale = col < r ? (w ? w[col] : 1.0) : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double x = acc[rt][t][v];
#pragma unroll
        for (int ww = 1; ww < kRitzWaves; ++ww) x += red[((((ww - 1) * kRitzRT + rt) * NT + t) * 4 + v) * kWave + lane];
        const int row = row0 + rt * 16 + kq + 4 * v;
        if (row < nrows && col < rs) out[(size_t)row * rs + col] = (T)(x * scale);
      }
    }
}

// Sampled product, residual and iterate update in one pass over a compressed
// orientation of Omega.  The dot product is the same fma chain in either
// orientation (u-factor entry first).  The other orientation's copy of Y is
// refreshed from this one by a permutation gather (k_gather4), which costs
// less than a second sampled product or a scatter of 4-byte stores.  Each
// workgroup writes its (compensated) sum of e^2; the host adds the partials
// in order.

template <typename T>
__device__ __forceinline__ T sampled_dot(const T *__restrict__ urow, const T *__restrict__ vrow, int r) {
  T x = (T)0;
  for (int l = 0; l < r; ++l) x = fma(urow[l], vrow[l], x);
  return x;
}

// RB > 0: the fixed (row-side) factor row is held in RB registers (r <= RB);
// RB == 0: any r, both factors read from memory.  rs: a multiple of
// 16 / sizeof(T), rows zero padded (the gathered rows are read 16 bytes at a
// time).
// DS (the Dantzig-selector iteration for |X - B| <= E on Omega, Section
// 3.3): with d = B - x, the two nonnegative multipliers take
// Y+ = max(Y+ + delta (d - E), 0) and Y- = max(Y- + delta (-d - E), 0), the
// iterate is Y = Y+ - Y-, and the partial sums are of the squared
// violation max(|d| - E, 0)^2; with part2_out the sums of d^2 go there too.
template <typename T, int L, int RB, bool DS>
__global__ __launch_bounds__(kBlock) void k_sample_update(
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx, const T *__restrict__ M,
    T *__restrict__ Y, int nrows, int rows_per_blk,
    const T *__restrict__ Fu, const T *__restrict__ Fv, int r, int rs, int row_side_is_u, T delta,
    double *__restrict__ part_out, T *__restrict__ Yp, T *__restrict__ Ym, T E, double *__restrict__ part2_out) {
  __shared__ double sbuf[kWaves];
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  constexpr int kGroups = kBlock / L;
  const T *other = row_side_is_u ? Fv : Fu;
  T sum = (T)0, comp = (T)0;    // compensated sum of e^2 (DS: of the violation^2)
  T sum2 = (T)0, comp2 = (T)0;  // DS: compensated sum of e^2
  for (int row = r0 + grp; row < r1; row += kGroups) {
    const int beg = ptr[row], end = ptr[row + 1];
    const T *fixed = (row_side_is_u ? Fu : Fv) + (size_t)row * rs;
    T f[RB > 0 ? RB : 1];
    if constexpr (RB > 0) {
#pragma unroll
      for (int l = 0; l < RB; ++l) f[l] = (l < r) ? fixed[l] : (T)0;
    }
    // kBatch entries per lane at a time: their indices, M and Y values, then
    // their factor rows, are loaded before any is used; the entries are then
    // finished in index order (the same sums as one at a time)
    constexpr int kBatch = (RB > 0 && RB <= 16) ? 4 : ((RB > 0 && RB <= 32) ? 2 : 1);
    for (int t0 = beg + lane; t0 < end; t0 += kBatch * L) {
      int jj[kBatch];
      T mv[kBatch], yv[kBatch], ymv[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int t = t0 + q * L;
        const bool in = t < end;
        jj[q] = in ? idx[t] : 0;
        mv[q] = in ? M[t] : (T)0;
        if constexpr (DS) {
          yv[q] = in ? Yp[t] : (T)0;
          ymv[q] = in ? Ym[t] : (T)0;
        } else {
          yv[q] = in ? Y[t] : (T)0;
        }
      }
      T x[kBatch];
      if constexpr (RB > 0) {
        // 16 bytes of the gathered factor row per load (rows are 16-byte
        // aligned and zero padded); the fma chain still runs in l order with
        // the u-factor entry first, in either orientation
        using V = typename Vec16<T>::type;
        constexpr int kv = 16 / sizeof(T);
        V gv[kBatch][RB / kv];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          const T *g = other + (size_t)jj[q] * rs;
#pragma unroll
          for (int l = 0; l < RB; l += kv)
            if (l < r) gv[q][l / kv] = *reinterpret_cast<const V *>(g + l);
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          T xx = (T)0;
#pragma unroll
          for (int l = 0; l < RB; l += kv) {
            const T *gc = reinterpret_cast<const T *>(&gv[q][l / kv]);
#pragma unroll
            for (int c = 0; c < kv; ++c) {
              if (l + c < r) xx = row_side_is_u ? fma(f[l + c], gc[c], xx) : fma(gc[c], f[l + c], xx);
            }
          }
          x[q] = xx;
        }
      } else {
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          const T *g = other + (size_t)jj[q] * rs;
          x[q] = row_side_is_u ? sampled_dot<T>(fixed, g, r) : sampled_dot<T>(g, fixed, r);
        }
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int t = t0 + q * L;
        if (t < end) {
          const T e = mv[q] - x[q];
          T g = e;  // the term whose square is summed
          if constexpr (DS) {
            const T yp2 = fmax(fma(delta, e - E, yv[q]), (T)0);
            const T ym2 = fmax(fma(delta, -e - E, ymv[q]), (T)0);
            Yp[t] = yp2;
            Ym[t] = ym2;
            Y[t] = yp2 - ym2;
            g = fmax(fabs(e) - E, (T)0);
          } else {
            Y[t] = fma(delta, e, yv[q]);
          }
          const T yk = fma(g, g, -comp);
          const T tk = sum + yk;
          comp = (tk - sum) - yk;
          sum = tk;
          if constexpr (DS) {
            const T y2 = fma(e, e, -comp2);
            const T t2 = sum2 + y2;
            comp2 = (t2 - sum2) - y2;
            sum2 = t2;
          }
        }
      }
    }
  }
  if (part_out == nullptr) return;  // uniform: no residual wanted
  const double tot = block_sum((double)sum - (double)comp, sbuf);
  if (threadIdx.x == 0) part_out[blockIdx.x] = tot;
  if constexpr (DS) {
    if (part2_out != nullptr) {
      __syncthreads();  // sbuf is reused
      const double tot2 = block_sum((double)sum2 - (double)comp2, sbuf);
      if (threadIdx.x == 0) part2_out[blockIdx.x] = tot2;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpby(const T *__restrict__ x, T *__restrict__ y, int64_t n, double a) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    y[i] = (T)(a * (double)x[i]);
}

__global__ __launch_bounds__(kBlock) void k_d2f(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    y[i] = (float)x[i];
}

__global__ __launch_bounds__(kBlock) void k_f2d(const float *__restrict__ x, double *__restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    y[i] = (double)x[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(const T *__restrict__ x, const int32_t *__restrict__ map,
                                                   T *__restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    y[i] = x[map[i]];
}

// y[i] = x[map[i]], four consecutive i per thread: one 16-byte load of the
// map, the four gathers in flight together, 16-byte stores (map and y
// 16-byte aligned).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather4(const T *__restrict__ x, const int32_t *__restrict__ map,
                                                    T *__restrict__ y, int64_t n) {
  const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 4;
  if (i0 + 3 < n) {
    const int4 m = *reinterpret_cast<const int4 *>(map + i0);
    const T a = x[m.x], b = x[m.y], c = x[m.z], d = x[m.w];
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<float4 *>(y + i0) = make_float4(a, b, c, d);
    } else {
      *reinterpret_cast<double2 *>(y + i0) = make_double2(a, b);
      *reinterpret_cast<double2 *>(y + i0 + 2) = make_double2(c, d);
    }
  } else {
    for (int64_t i = i0; i < n; ++i) y[i] = x[map[i]];
  }
}


int grid_for(int64_t n, int cap = 4096) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

RowChunks row_chunks(int nrows, int target_rows) {
  RowChunks c;
  if (target_rows < 1) target_rows = 1;
  c.nblk = (nrows + target_rows - 1) / target_rows;
  if (c.nblk < 1) c.nblk = 1;
  c.rows_per_blk = (nrows + c.nblk - 1) / c.nblk;
  if (c.rows_per_blk < 1) c.rows_per_blk = 1;
  c.nblk = (nrows + c.rows_per_blk - 1) / c.rows_per_blk;
  if (c.nblk < 1) c.nblk = 1;
  return c;
}

int lanes_for(double mean) {
  if (mean < 6.0) return 4;
  if (mean < 12.0) return 8;
  if (mean < 40.0) return 16;
  if (mean < 160.0) return 32;
  return 64;
}

RowPlan row_plan(int nrows, int min_rows) {
  RowPlan rp;
  min_rows = std::max(1, min_rows);
  rp.nblk = std::max(1, std::min(kMaxRowBlocks, (nrows + min_rows - 1) / min_rows));
  // very long vectors: more workgroups rather than more rows each
  rp.nblk = std::max(rp.nblk, (nrows + kMaxRowsPerBlock - 1) / kMaxRowsPerBlock);
  rp.rows_per_blk = std::max(1, (nrows + rp.nblk - 1) / rp.nblk);
  rp.nblk = std::max(1, (nrows + rp.rows_per_blk - 1) / rp.rows_per_blk);
  return rp;
}

// The dynamic-LDS limit is a per-kernel attribute shared by every stream and
// thread: raise it once to the largest size the kernel can take (the
// device's per-workgroup maximum less the kernel's static LDS) and never
// lower it, so concurrent solves with different plans cannot shrink it under
// each other's launches.
hipError_t allow_dynamic_lds(const void *kern, size_t bytes) {
  static std::mutex mu;
  static std::map<const void *, size_t> raised;
  std::lock_guard<std::mutex> lk(mu);
  auto it = raised.find(kern);
  if (it != raised.end() && it->second >= bytes) return hipSuccess;
  int dev = 0, maxlds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  hipFuncAttributes fa{};
  e = hipFuncGetAttributes(&fa, kern);
  if (e != hipSuccess) return e;
  const size_t room = (size_t)maxlds > fa.sharedSizeBytes ? (size_t)maxlds - fa.sharedSizeBytes : 0;
  if (bytes > room) return hipErrorInvalidValue;
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)room);
  if (e != hipSuccess) return e;
  raised[kern] = room;
  return hipSuccess;
}

SpmvPlan spmv_plan(int nrows, int ncols, int elem_bytes, int lds_bytes, int mode, int min_rows) {
  SpmvPlan pl{};
  const RowPlan rp = row_plan(nrows, min_rows);
  pl.min_rows = min_rows;
  pl.nblk = rp.nblk;
  pl.rows_per_blk = rp.rows_per_blk;
  // lanes per row: the widest power of two that still runs all of a
  // workgroup's rows at once (4 .. 64)
  pl.lanes = 64;
  while (pl.lanes > 4 && (kRowBlock / pl.lanes) < pl.rows_per_blk) pl.lanes /= 2;
  const long racc = (((long)elem_bytes * pl.rows_per_blk + 15) / 16) * 16;
  pl.nseg = 0;
  pl.segcols = 0;
  if (mode != 1) {
    // 2 KiB of headroom for the kernel's static LDS
    const long budget = ((long)lds_bytes - 2048 - racc - kSpmvAuxBytes) / elem_bytes;
    long seg = std::min<long>(ncols, budget);
    if (seg < ncols) seg = (seg / 64) * 64;
    if (seg >= 1) {
      const int nseg = (int)((ncols + seg - 1) / seg);
      // one segment holding all of x, or a few segments that are not tiny
      // (two 120 KB segments of FP64 x beat gathering it: 20 vs 26 us at 30000^2)
      const bool ok = nseg == 1 || (seg >= 1024 && nseg <= 8);
      if (ok) {
        pl.nseg = nseg;
        pl.segcols = (int)seg;
      }
    }
  }
  // the region after racc holds x's segment, then the fused dot products;
  // h and g follow it
  const size_t region = (std::max((size_t)elem_bytes * (size_t)pl.segcols, (size_t)kDotsLds) + 15) / 16 * 16;
  pl.lds = (size_t)racc + region + kSpmvAuxBytes;
  return pl;
}

template <typename T, typename I>
hipError_t launch_spmv_i(hipStream_t s, const SpmvPlan &pl, const int32_t *ptr, const I *idx, const T *val,
                         const int32_t *segptr, const SpmvInput<T> &in, int ncols, const T *prev, T *p,
                         int nrows, const T *Q, int64_t ldq, int nq, int ndots, double *dots_out) {
#define SVT_SPMVR(LN, ST, PL)                                                                      \
  do {                                                                                            \
    auto kern = k_spmv_rows<T, I, LN, ST, PL>;                                                    \
    hipError_t ea = allow_dynamic_lds(reinterpret_cast<const void *>(kern), pl.lds);              \
    if (ea != hipSuccess) return ea;                                                              \
    SVT_LAUNCH(kern, dim3(pl.nblk), dim3(kRowBlock), pl.lds, s, ptr, idx, val, segptr, pl.nseg,    \
               pl.segcols, in, ncols, prev, p, nrows, pl.rows_per_blk, Q, ldq, nq, ndots, dots_out); \
  } while (0)
#define SVT_SPMVS(ST, PL)                      \
  switch (pl.lanes) {                          \
    case 4: SVT_SPMVR(4, ST, PL); break;       \
    case 8: SVT_SPMVR(8, ST, PL); break;       \
    case 16: SVT_SPMVR(16, ST, PL); break;     \
    case 32: SVT_SPMVR(32, ST, PL); break;     \
    default: SVT_SPMVR(64, ST, PL); break;     \
  }
  // a half-step with nothing to orthogonalise (no update of x, no dot
  // products of p) takes the PLAIN kernel when x is staged
  const bool plain = nq == 0 && in.nqx == 0;
  if (pl.nseg > 0 && plain) {
    SVT_SPMVS(true, true);
  } else if (pl.nseg > 0) {
    SVT_SPMVS(true, false);
  } else {
    SVT_SPMVS(false, false);
  }
#undef SVT_SPMVS
#undef SVT_SPMVR
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spmv(hipStream_t s, const SpmvPlan &pl, const int32_t *ptr, const int32_t *idx,
                       const uint16_t *idx16, const T *val, const int32_t *segptr, const SpmvInput<T> &in,
                       int ncols, const T *prev, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                       int ndots, double *dots_out) {
  if (pl.nseg > 1 && segptr == nullptr) return hipErrorInvalidValue;
  if (ndots != 0 && ndots != nq) return hipErrorInvalidValue;
  if (in.x == nullptr || p == nullptr) return hipErrorInvalidValue;
  if (idx16 != nullptr && ncols > 65536) return hipErrorInvalidValue;
  if ((dots_out != nullptr || in.nqx > 0) && nq > 0 && Q == nullptr) return hipErrorInvalidValue;
  if (in.nqx < 0 || nq < 0) return hipErrorInvalidValue;
  if (in.nqx > 0) {
    // the deferred update: its coefficients and their image must fit the
    // LDS reserved for them, and Q must be the basis the relations name
    if (in.pend == nullptr || in.Qx == nullptr || in.alpha == nullptr || in.beta == nullptr) return hipErrorInvalidValue;
    if (in.side != 0 && in.side != 1) return hipErrorInvalidValue;
    if (nq != in.nqx + in.side || nq > kSpmvAuxCols) return hipErrorInvalidValue;
    if (in.x_out != nullptr && in.ldqx < ncols) return hipErrorInvalidValue;
  }
  if (in.pend != nullptr && in.np < 1) return hipErrorInvalidValue;
  const RowPlan rp = row_plan(nrows, pl.min_rows);
  if (rp.nblk != pl.nblk || rp.rows_per_blk != pl.rows_per_blk) return hipErrorInvalidValue;
  if (idx16 != nullptr)
    return launch_spmv_i<T, uint16_t>(s, pl, ptr, idx16, val, segptr, in, ncols, prev, p, nrows, Q, ldq, nq,
                                      ndots, dots_out);
  if (idx == nullptr) return hipErrorInvalidValue;
  return launch_spmv_i<T, int32_t>(s, pl, ptr, idx, val, segptr, in, ncols, prev, p, nrows, Q, ldq, nq,
                                   ndots, dots_out);
}

size_t gs_update_lds(int nq, int rows_per_blk) {
  return sizeof(double) * ((size_t)nq + 1 + (size_t)rows_per_blk + kReduceScratch) + kDotsLds;
}

template <typename T>
hipError_t launch_gs_update(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                            const double *part_in, double *part_out, bool second, double *removed,
                            int min_rows) {
  const RowPlan rp = row_plan(nrows, min_rows);
  if (nq < 1 || Q == nullptr) return hipErrorInvalidValue;
  const size_t lds = gs_update_lds(nq, rp.rows_per_blk);
  if (!second) {
    auto kern = k_gs_update<T, false>;
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void *>(kern), lds);
    if (e != hipSuccess) return e;
    SVT_LAUNCH(kern, dim3(rp.nblk), dim3(kRowBlock), lds, s, p, nrows, rp.rows_per_blk, Q, ldq, nq, part_in,
               rp.nblk, part_out, removed);
  } else {
    auto kern = k_gs_update<T, true>;
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void *>(kern), lds);
    if (e != hipSuccess) return e;
    SVT_LAUNCH(kern, dim3(rp.nblk), dim3(kRowBlock), lds, s, p, nrows, rp.rows_per_blk, Q, ldq, nq, part_in,
               rp.nblk, part_out, removed);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sumsq(hipStream_t s, const T *p, int nrows, double *part_out, int min_rows) {
  const RowPlan rp = row_plan(nrows, min_rows);
  SVT_LAUNCH((k_sumsq<T>), dim3(rp.nblk), dim3(kRowBlock), 0, s, p, nrows, rp.rows_per_blk, part_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(hipStream_t s, const T *p, int nrows, const double *part, T *out,
                           double *coef_out, int min_rows) {
  const RowPlan rp = row_plan(nrows, min_rows);
  SVT_LAUNCH((k_gs_scale<T>), dim3(rp.nblk), dim3(kRowBlock), 0, s, p, nrows, part, rp.nblk, out, coef_out);
  return hipGetLastError();
}

hipError_t launch_pending_norm(hipStream_t s, const double *pend, int np, int nqx, double *s_out,
                               double *removed_out) {
  if (pend == nullptr || s_out == nullptr || np < 1 || nqx < 0 || nqx > kSpmvAuxCols) return hipErrorInvalidValue;
  SVT_LAUNCH(k_pending_norm, dim3(1), dim3(kRowBlock), sizeof(double) * ((size_t)nqx + 1), s, pend, np, nqx,
             s_out, removed_out);
  return hipGetLastError();
}

hipError_t launch_pending_reduce(hipStream_t s, const double *pend, int np, int nqx, double *out) {
  if (pend == nullptr || out == nullptr || np < 1 || nqx < 0 || nqx > kSpmvAuxCols) return hipErrorInvalidValue;
  const int C = nqx + 1;
  SVT_LAUNCH(k_pending_reduce, dim3((C + kPreCols - 1) / kPreCols), dim3(kPreCols * kRedStrands), 0, s, pend, np, C,
             out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_randn(hipStream_t s, T *out, int n, uint64_t seed, uint64_t ctr) {
  SVT_LAUNCH((k_randn<T>), dim3(grid_for(n, 2048)), dim3(kBlock), 0, s, out, n, seed, ctr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ritz(hipStream_t s, const T *Q, int64_t ldq, int nrows, int k, const double *P,
                       const double *w, int r, T *out, int rs) {
  if (rs < 1 || nrows < 1) return hipSuccess;
  if (k < 1 || r > rs || ldq < nrows) return hipErrorInvalidValue;
  const dim3 grid((nrows + 16 * kRitzRT - 1) / (16 * kRitzRT), (rs + kRitzCols - 1) / kRitzCols);
  // 16-column tiles per workgroup: enough for the first kRitzCols columns
  const int nt = std::min(kRitzCols, rs + 15) / 16;
  switch (nt) {
    case 1: SVT_LAUNCH((k_ritz<T, 1>), grid, dim3(kRitzThreads), 0, s, Q, ldq, nrows, k, P, w, r, out, rs); break;
    case 2: SVT_LAUNCH((k_ritz<T, 2>), grid, dim3(kRitzThreads), 0, s, Q, ldq, nrows, k, P, w, r, out, rs); break;
    case 3: SVT_LAUNCH((k_ritz<T, 3>), grid, dim3(kRitzThreads), 0, s, Q, ldq, nrows, k, P, w, r, out, rs); break;
    default: SVT_LAUNCH((k_ritz<T, 4>), grid, dim3(kRitzThreads), 0, s, Q, ldq, nrows, k, P, w, r, out, rs); break;
  }
  return hipGetLastError();
}

// The residual partials of the allocation-free sampled pass
// (svt_sample_update_noalloc): one fixed array per device, shared by every
// such call on that device (calls that overlap on one device race).  Host
// code never passes `scratch` itself to a kernel: its device address comes
// from hipGetSymbolAddress, looked up once per device with that device
// current, and cached.
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

hipError_t noalloc_scratch(int device, double **out) {
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices || out == nullptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lk(mu);
  if (addr[device] == nullptr) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<double *>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

int sample_blocks(int nrows, int lanes) {
  return row_chunks(nrows, std::max((kBlock / lanes) * 4, (nrows + kSampleMaxBlocks - 1) / kSampleMaxBlocks))
      .nblk;
}

template <typename T, bool DS>
static void sample_update_variant(hipStream_t s, int lanes, const int32_t *ptr, const int32_t *idx, const T *M,
                                  T *Y, int nrows, const T *Fu, const T *Fv, int r, int rs, bool row_side_is_u,
                                  double delta, double *part_out, T *Yp, T *Ym, double E, double *part2_out) {
  const RowChunks ch =
      row_chunks(nrows, std::max((kBlock / lanes) * 4, (nrows + kSampleMaxBlocks - 1) / kSampleMaxBlocks));
#define SVT_SU2(LN, RB)                                                                              \
  SVT_LAUNCH((k_sample_update<T, LN, RB, DS>), dim3(ch.nblk), dim3(kBlock), 0, s, ptr, idx, M, Y, nrows, \
             ch.rows_per_blk, Fu, Fv, r, rs, row_side_is_u ? 1 : 0, (T)delta, part_out, Yp, Ym, (T)E, part2_out)
#define SVT_SU(LN)                         \
  do {                                     \
    if (r <= 8) SVT_SU2(LN, 8);            \
    else if (r <= 16) SVT_SU2(LN, 16);     \
    else if (r <= 32) SVT_SU2(LN, 32);     \
    else if (r <= 64) SVT_SU2(LN, 64);     \
    else SVT_SU2(LN, 0);                   \
  } while (0)
  switch (lanes) {
    case 4: SVT_SU(4); break;
    case 8: SVT_SU(8); break;
    case 16: SVT_SU(16); break;
    case 32: SVT_SU(32); break;
    default: SVT_SU(64); break;
  }
#undef SVT_SU
#undef SVT_SU2
}

template <typename T>
hipError_t launch_sample_update(hipStream_t s, int lanes, const int32_t *ptr, const int32_t *idx,
                                const T *M, T *Y, int nrows, const T *Fu, const T *Fv, int r, int rs,
                                bool row_side_is_u, double delta, double *part_out, T *Yp, T *Ym, double E,
                                double *part2_out) {
  if (rs % (16 / (int)sizeof(T)) != 0 || rs < r) return hipErrorInvalidValue;
  if ((Yp == nullptr) != (Ym == nullptr) || !(E >= 0.0)) return hipErrorInvalidValue;
  if (Yp) sample_update_variant<T, true>(s, lanes, ptr, idx, M, Y, nrows, Fu, Fv, r, rs, row_side_is_u, delta,
                                         part_out, Yp, Ym, E, part2_out);
  else sample_update_variant<T, false>(s, lanes, ptr, idx, M, Y, nrows, Fu, Fv, r, rs, row_side_is_u, delta,
                                       part_out, nullptr, nullptr, 0.0, nullptr);
  return hipGetLastError();
}

// The Dantzig-selector kick: Y+ = a max(B - E, 0), Y- = a max(-B - E, 0),
// Y = Y+ - Y- (= a S_E(B)); with Yp null only Y = S_E(B) (a ignored).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ds_init(const T *__restrict__ B, int64_t n, double E, double a,
                                                    T *__restrict__ Yp, T *__restrict__ Ym, T *__restrict__ Y) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double b = (double)B[i];
    const double p = fmax(b - E, 0.0), q = fmax(-b - E, 0.0);
    if (Yp) {
      const T yp = (T)(a * p), ym = (T)(a * q);
      Yp[i] = yp;
      Ym[i] = ym;
      Y[i] = yp - ym;
    } else {
      Y[i] = (T)(p - q);
    }
  }
}

// General linear operator (measurements b = G x_S): each thread takes
// measurements i, r_i = b_i - sum_t G[i, t] x[gidx[t]] (fma chain in t
// order), y_i += delta r_i, and its sum of r_i^2 (FP64) joins the
// workgroup's partial in part_out.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_measure(const int64_t *__restrict__ gptr, const int32_t *__restrict__ gidx,
                                                    const T *__restrict__ gval, const T *__restrict__ x,
                                                    const T *__restrict__ b, T *__restrict__ y, int64_t p, T delta,
                                                    double *__restrict__ part_out) {
  __shared__ double sbuf[kWaves];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < p; i += (int64_t)gridDim.x * kBlock) {
    T v = (T)0;
    for (int64_t t = gptr[i]; t < gptr[i + 1]; ++t) v = fma(gval[t], x[gidx[t]], v);
    const T r = b[i] - v;
    y[i] = fma(delta, r, y[i]);
    acc = fma((double)r, (double)r, acc);
  }
  const double tot = block_sum(acc, sbuf);
  if (threadIdx.x == 0) part_out[blockIdx.x] = tot;
}

// The adjoint onto the support: Y[s] = sum_t GT[s, t] y[tidx[t]] for each
// support entry s (fma chain in t order).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adjoint(const int64_t *__restrict__ tptr, const int32_t *__restrict__ tidx,
                                                    const T *__restrict__ tval, const T *__restrict__ y,
                                                    T *__restrict__ Y, int64_t ns) {
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < ns; s += (int64_t)gridDim.x * kBlock) {
    T v = (T)0;
    for (int64_t t = tptr[s]; t < tptr[s + 1]; ++t) v = fma(tval[t], y[tidx[t]], v);
    Y[s] = v;
  }
}

int measure_blocks(int64_t p) { return (int)std::min<int64_t>(kSampleMaxBlocks, std::max<int64_t>(1, (p + kBlock - 1) / kBlock)); }

template <typename T>
hipError_t launch_measure(hipStream_t s, const int64_t *gptr, const int32_t *gidx, const T *gval, const T *x,
                          const T *b, T *y, int64_t p, double delta, double *part_out) {
  if (p <= 0 || part_out == nullptr) return hipErrorInvalidValue;
  SVT_LAUNCH((k_measure<T>), dim3(measure_blocks(p)), dim3(kBlock), 0, s, gptr, gidx, gval, x, b, y, p, (T)delta,
             part_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint(hipStream_t s, const int64_t *tptr, const int32_t *tidx, const T *tval, const T *y, T *Y,
                          int64_t ns) {
  if (ns <= 0) return hipSuccess;
  SVT_LAUNCH((k_adjoint<T>), dim3(grid_for(ns)), dim3(kBlock), 0, s, tptr, tidx, tval, y, Y, ns);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ds_init(hipStream_t s, const T *B, int64_t n, double E, double a, T *Yp, T *Ym, T *Y) {
  if (n <= 0) return hipSuccess;
  if ((Yp == nullptr) != (Ym == nullptr) || !(E >= 0.0)) return hipErrorInvalidValue;
  SVT_LAUNCH((k_ds_init<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, B, n, E, a, Yp, Ym, Y);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpby(hipStream_t s, const T *x, T *y, int64_t n, double a) {
  SVT_LAUNCH((k_axpby<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n, a);
  return hipGetLastError();
}

hipError_t launch_d2f(hipStream_t s, const double *x, float *y, int64_t n) {
  SVT_LAUNCH(k_d2f, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t launch_f2d(hipStream_t s, const float *x, double *y, int64_t n) {
  SVT_LAUNCH(k_f2d, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(hipStream_t s, const T *x, const int32_t *map, T *y, int64_t n) {
  if (n <= 0) return hipSuccess;
  if ((reinterpret_cast<uintptr_t>(map) & 15) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0) {
    const int64_t threads = (n + 3) / 4;
    SVT_LAUNCH((k_gather4<T>), dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, x, map, y, n);
  } else {
    SVT_LAUNCH((k_gather<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, x, map, y, n);
  }
  return hipGetLastError();
}

#define SVT_INSTANTIATE(T)                                                                          \
  template hipError_t launch_spmv<T>(hipStream_t, const SpmvPlan &, const int32_t *, const int32_t *,      \
                                     const uint16_t *, const T *, const int32_t *, const SpmvInput<T> &, \
                                     int, const T *, T *, int, const T *, int64_t, int, int, double *);     \
  template hipError_t launch_gs_update<T>(hipStream_t, T *, int, const T *, int64_t, int, const double *, \
                                          double *, bool, double *, int);                              \
  template hipError_t launch_sumsq<T>(hipStream_t, const T *, int, double *, int);                     \
  template hipError_t launch_finalize<T>(hipStream_t, const T *, int, const double *, T *, double *,   \
                                         int);                                                         \
  template hipError_t launch_randn<T>(hipStream_t, T *, int, uint64_t, uint64_t);                  \
  template hipError_t launch_ritz<T>(hipStream_t, const T *, int64_t, int, int, const double *,    \
                                     const double *, int, T *, int);                                \
  template hipError_t launch_sample_update<T>(hipStream_t, int, const int32_t *, const int32_t *,  \
                                              const T *, T *, int, const T *, const T *, int, int,  \
                                              bool, double, double *, T *, T *, double, double *);  \
  template hipError_t launch_ds_init<T>(hipStream_t, const T *, int64_t, double, double, T *, T *, T *); \
  template hipError_t launch_measure<T>(hipStream_t, const int64_t *, const int32_t *, const T *, const T *, \
                                        const T *, T *, int64_t, double, double *);                  \
  template hipError_t launch_adjoint<T>(hipStream_t, const int64_t *, const int32_t *, const T *, const T *, \
                                        T *, int64_t);                                                \
  template hipError_t launch_axpby<T>(hipStream_t, const T *, T *, int64_t, double);               \
  template hipError_t launch_gather<T>(hipStream_t, const T *, const int32_t *, T *, int64_t);

SVT_INSTANTIATE(double)
SVT_INSTANTIATE(float)

}  // namespace svt
