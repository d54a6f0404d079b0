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
//   * reorthogonalisation is classical Gram-Schmidt applied twice (CGS2);
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

// Every launch goes through hipExtLaunchKernelGGL and takes (and clears) the
// pending timing events, if any.
#define SVT_LAUNCH(kern, grid, block, lds, stream, ...)                                     \
  do {                                                                                      \
    hipEvent_t ev_a_ = t_ev_start, ev_b_ = t_ev_stop;                                       \
    t_ev_start = t_ev_stop = nullptr;                                                       \
    hipExtLaunchKernelGGL(kern, grid, block, (std::uint32_t)(lds), stream, ev_a_, ev_b_, 0u, \
                          __VA_ARGS__);                                                     \
  } while (0)

namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr int kTile = 16;  // Gram-Schmidt columns per pass of a workgroup

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

// hs[c] = sum_i part[c * np + i] for c < C, into LDS, in a fixed order that
// does not depend on the workgroup: column c is split into G interleaved
// strands (G = kBlock / min(C, kBlock)), each summed with four accumulators,
// then the strands are added in strand order.
__device__ void reduce_columns(const double *__restrict__ part, int np, int C, double *hs,
                               double *scratch /* kBlock doubles of LDS */) {
  for (int cb = 0; cb < C; cb += kBlock) {
    const int Cb = min(kBlock, C - cb);
    const int G = kBlock / Cb;
    const int t = threadIdx.x, g = t / Cb, c = t % Cb;
    double acc = 0.0;
    if (g < G) {
      const double *src = part + (size_t)(cb + c) * np;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int i = g;
      for (; i + 3 * G < np; i += 4 * G) {
        a0 += src[i];
        a1 += src[i + G];
        a2 += src[i + 2 * G];
        a3 += src[i + 3 * G];
      }
      for (; i < np; i += G) a0 += src[i];
      acc = (a0 + a1) + (a2 + a3);
    }
    scratch[t] = acc;
    __syncthreads();
    if (t < Cb) {
      double sum = 0.0;
      for (int gg = 0; gg < G; ++gg) sum += scratch[gg * Cb + t];
      hs[cb + t] = sum;
    }
    __syncthreads();
  }
}

// Partial Gram-Schmidt dot products of one workgroup's rows [r0, r1) with
// the columns c0 .. c0+kTile-1 of Q (column nq stands for the vector itself):
// part[c * np + rc] = sum_rows Q[c][row] v(row).  Every thread issues its
// tile's loads together; the kTile sums reduce as independent shuffle chains.
template <typename T, typename VF>
__device__ __forceinline__ void tile_partials(VF v, int r0, int r1, const T *__restrict__ Q, int64_t ldq,
                                              int nq, int c0, double *__restrict__ part, int np, int rc,
                                              double (*sred)[kTile]) {
  double acc[kTile];
#pragma unroll
  for (int j = 0; j < kTile; ++j) acc[j] = 0.0;
  // Branch-free tile: columns past nq - 1 load column nq - 1 (any valid
  // column) and are masked, so the kTile loads of a row issue back to back.
  const int last = nq > 0 ? nq - 1 : 0;
  // two rows per round: 2 kTile loads in flight per thread
  for (int row = r0 + threadIdx.x; row < r1; row += 2 * kBlock) {
    const int row2 = row + kBlock;
    const bool has2 = row2 < r1;
    const double pv = v(row);
    const double pv2 = has2 ? v(row2) : 0.0;
    double q[kTile], q2[kTile];
    if (nq > 0) {
#pragma unroll
      for (int j = 0; j < kTile; ++j) {
        const size_t off = (size_t)min(c0 + j, last) * ldq;
        q[j] = (double)Q[off + row];
        q2[j] = has2 ? (double)Q[off + row2] : 0.0;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kTile; ++j) q[j] = q2[j] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < kTile; ++j) {
      const int c = c0 + j;
      const double f = (c < nq) ? q[j] : ((c == nq) ? pv : 0.0);
      const double f2 = (c < nq) ? q2[j] : ((c == nq) ? pv2 : 0.0);
      acc[j] = fma(f, pv, acc[j]);
      acc[j] = fma(f2, pv2, acc[j]);
    }
  }
  const int w = threadIdx.x / kWave, wl = threadIdx.x % kWave;
#pragma unroll
  for (int j = 0; j < kTile; ++j) {
    const double sv = seg_sum<kWave>(acc[j]);
    if (wl == 0) sred[w][j] = sv;
  }
  __syncthreads();
  if (threadIdx.x < kTile) {
    const int c = c0 + threadIdx.x;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += sred[i][threadIdx.x];
    if (c <= nq) part[(size_t)c * np + rc] = t;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Norms at or below this are treated as zero: the reciprocal of a larger one
// is finite in the value type.
template <typename T> __device__ __forceinline__ double norm_floor();
template <> __device__ __forceinline__ double norm_floor<double>() { return 1e-280; }
template <> __device__ __forceinline__ double norm_floor<float>() { return 1e-30; }

// Lazy normalisation of the input vector of a sparse product: x = x_raw / s
// with s^2 the sum of the np partials in xpart (every workgroup sums them in
// the same order).  Returns s (1 when xpart is null: x_raw is normalised).
__device__ __forceinline__ double input_norm(const double *__restrict__ xpart, int np, double *sh) {
  if (xpart == nullptr) return 1.0;
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v += xpart[i];
  v = seg_sum<kWave>(v);
  const int w = threadIdx.x / kWave, wl = threadIdx.x % kWave, nw = blockDim.x / kWave;
  if (wl == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += sh[i];
  __syncthreads();
  return sqrt(t);
}

// Workgroup b writes x_raw[i] / s for its slice of [0, ncols) into x_out and
// workgroup 0 stores s: the normalised vector joins its basis.
template <typename T>
__device__ __forceinline__ void write_normalised(const T *__restrict__ x_raw, int ncols, double s,
                                                 T *__restrict__ x_out, double *__restrict__ s_out) {
  if (x_out == nullptr) return;
  const double inv = (s > norm_floor<T>()) ? 1.0 / s : 0.0;
  const int chunk = (ncols + gridDim.x - 1) / gridDim.x;
  const int i0 = blockIdx.x * chunk, i1 = min(ncols, i0 + chunk);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) x_out[i] = (T)((double)x_raw[i] * inv);
  if (blockIdx.x == 0 && threadIdx.x == 0 && s_out) *s_out = s;
}

// p = A (x_raw / s) - s prev over a compressed orientation (one sub-wave per
// row), s from xpart (see input_norm); with x_out, the normalised x is also
// written out (the previous half-step's vector joins its basis).
template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_spmv(
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx, const T *__restrict__ val,
    const T *__restrict__ x, const double *__restrict__ xpart, int xnp, T *__restrict__ x_out,
    double *__restrict__ s_out, int ncols, const T *__restrict__ prev, T *__restrict__ p, int nrows) {
  __shared__ double sh[kWaves];
  const double sn = input_norm(xpart, xnp, sh);
  write_normalised<T>(x, ncols, sn, x_out, s_out);
  const T inv = (T)((sn > norm_floor<T>()) ? 1.0 / sn : 0.0);
  const int lane = threadIdx.x % L;
  constexpr int kGroups = kBlock / L;
  const int row = blockIdx.x * kGroups + threadIdx.x / L;
  if (row >= nrows) return;  // whole sub-wave leaves together
  const int beg = ptr[row], end = ptr[row + 1];
  T acc = (T)0;
  int t = beg + lane;
  // four entries per lane per round: the index loads, then the gathers, issue
  // together
  for (; t + 3 * L < end; t += 4 * L) {
    const int i0 = idx[t], i1 = idx[t + L], i2 = idx[t + 2 * L], i3 = idx[t + 3 * L];
    const T v0 = val[t], v1 = val[t + L], v2 = val[t + 2 * L], v3 = val[t + 3 * L];
    const T x0 = x[i0], x1 = x[i1], x2 = x[i2], x3 = x[i3];
    acc = fma(v0, x0, acc);
    acc = fma(v1, x1, acc);
    acc = fma(v2, x2, acc);
    acc = fma(v3, x3, acc);
  }
  if (t < end) {
    // fewer than four entries left: one masked batch, same order
    const bool in1 = t + L < end, in2 = t + 2 * L < end;
    const int i0 = idx[t], i1 = in1 ? idx[t + L] : 0, i2 = in2 ? idx[t + 2 * L] : 0;
    const T v0 = val[t], v1 = in1 ? val[t + L] : (T)0, v2 = in2 ? val[t + 2 * L] : (T)0;
    const T x0 = x[i0], x1 = in1 ? x[i1] : (T)0, x2 = in2 ? x[i2] : (T)0;
    acc = fma(v0, x0, acc);
    if (in1) acc = fma(v1, x1, acc);
    if (in2) acc = fma(v2, x2, acc);
  }
  acc = seg_sum<L>(acc);
  if (lane == 0) {
    acc = acc * inv;
    p[row] = prev ? fma(-(T)sn, prev[row], acc) : acc;
  }
}

// p = A (x_raw / s) - s prev with x staged in LDS.  A workgroup owns a
// contiguous range of rows; the columns are split into segments of at most
// `segcols` entries, each copied once into LDS (coalesced, every thread's
// loads issued before its stores), so the per-entry gathers of x hit LDS
// instead of L2.  segptr[row * (nseg + 1) + s] is the first entry of segment
// s of the row (null when nseg == 1: ptr is used).  L lanes take a row (L is
// chosen so that all of a workgroup's rows run at once) and each lane keeps
// kSpmvUnroll entries in flight; a lane accumulates its entries in index
// order, so the result does not depend on the unrolling.
constexpr int kSpmvUnroll = 16;
constexpr int kStageUnroll = 16;

template <typename T, int L>
__global__ __launch_bounds__(kSpmvBlock) void k_spmv_lds(
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx, const T *__restrict__ val,
    const int32_t *__restrict__ segptr, int nseg, int segcols, const T *__restrict__ x,
    const double *__restrict__ xpart, int xnp, T *__restrict__ x_out, double *__restrict__ s_out, int ncols,
    const T *__restrict__ prev, T *__restrict__ p, int nrows, int rows_per_blk) {
  extern __shared__ double smem_d[];
  __shared__ double sh[kSpmvBlock / kWave];
  T *xs = reinterpret_cast<T *>(smem_d);  // segcols entries
  T *racc = xs + segcols;                  // rows_per_blk partial row sums
  const double sn = input_norm(xpart, xnp, sh);
  write_normalised<T>(x, ncols, sn, x_out, s_out);
  const T inv = (T)((sn > norm_floor<T>()) ? 1.0 / sn : 0.0);
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  constexpr int kGroups = kSpmvBlock / L;
  for (int sgm = 0; sgm < nseg; ++sgm) {
    const int c0 = sgm * segcols;
    const int cn = min(segcols, ncols - c0);
    __syncthreads();  // the previous segment's gathers are done
    for (int base = threadIdx.x; base < cn; base += kSpmvBlock * kStageUnroll) {
      T v[kStageUnroll];
#pragma unroll
      for (int j = 0; j < kStageUnroll; ++j) {
        const int i = base + j * kSpmvBlock;
        v[j] = (i < cn) ? x[c0 + i] : (T)0;
      }
#pragma unroll
      for (int j = 0; j < kStageUnroll; ++j) {
        const int i = base + j * kSpmvBlock;
        if (i < cn) xs[i] = v[j];
      }
    }
    __syncthreads();
    for (int row = r0 + grp; row < r1; row += kGroups) {
      int beg, end;
      if (nseg == 1) {
        beg = ptr[row];
        end = ptr[row + 1];
      } else {
        beg = segptr[(size_t)row * (nseg + 1) + sgm];
        end = segptr[(size_t)row * (nseg + 1) + sgm + 1];
      }
      T acc = (T)0;
      int t = beg + lane;
      for (; t + (kSpmvUnroll - 1) * L < end; t += kSpmvUnroll * L) {
        int ii[kSpmvUnroll];
        T vv[kSpmvUnroll];
#pragma unroll
        for (int j = 0; j < kSpmvUnroll; ++j) {
          ii[j] = idx[t + j * L];
          vv[j] = val[t + j * L];
        }
#pragma unroll
        for (int j = 0; j < kSpmvUnroll; ++j) acc = fma(vv[j], xs[ii[j] - c0], acc);
      }
      if (t < end) {
        // fewer than kSpmvUnroll entries left: one masked batch, same order
        int ii[kSpmvUnroll];
        T vv[kSpmvUnroll];
#pragma unroll
        for (int j = 0; j < kSpmvUnroll; ++j) {
          const bool in = t + j * L < end;
          ii[j] = in ? idx[t + j * L] : c0;
          vv[j] = in ? val[t + j * L] : (T)0;
        }
#pragma unroll
        for (int j = 0; j < kSpmvUnroll; ++j)
          if (t + j * L < end) acc = fma(vv[j], xs[ii[j] - c0], acc);
      }
      acc = seg_sum<L>(acc);
      if (lane == 0) {
        const T tot = (sgm == 0) ? acc : racc[row - r0] + acc;
        if (sgm + 1 < nseg) {
          racc[row - r0] = tot;
        } else {
          const T y = tot * inv;
          p[row] = prev ? fma(-(T)sn, prev[row], y) : y;
        }
      }
    }
  }
}

// First Gram-Schmidt pass, dot products: part[c * nrc + rc] over a
// (row chunk, column tile) grid; column nq holds |p|^2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gs_dots(const T *__restrict__ p, int nrows, int rows_per_blk,
                                                    const T *__restrict__ Q, int64_t ldq, int nq,
                                                    double *__restrict__ part) {
  __shared__ double sred[kWaves][kTile];
  const int rc = blockIdx.x;
  const int r0 = rc * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  tile_partials<T>([&](int row) { return (double)p[row]; }, r0, r1, Q, ldq, nq, blockIdx.y * kTile, part,
                   gridDim.x, rc, sred);
}

// p <- p - Q h, with h = the column sums of part_in (np_in partials each,
// reduced by every workgroup).  SECOND = false: then the partial dot products
// of the new p with Q and itself go to part_out (the second pass's
// coefficients).  SECOND = true: only |p|^2 partials go to part_out.
template <typename T, bool SECOND>
__global__ __launch_bounds__(kBlock) void k_gs_update(T *__restrict__ p, int nrows, int rows_per_blk,
                                                      const T *__restrict__ Q, int64_t ldq, int nq,
                                                      const double *__restrict__ part_in, int np_in,
                                                      double *__restrict__ part_out) {
  extern __shared__ double smem[];
  double *hs = smem;                   // nq + 1 coefficients
  double *scratch = hs + nq + 1;       // kBlock
  double *pc = scratch + kBlock;       // rows_per_blk values of the updated p
  __shared__ double sred[kWaves][kTile];
  __shared__ double sbuf[kWaves];
  reduce_columns(part_in, np_in, nq + 1, hs, scratch);
  const int rc = blockIdx.x;
  const int r0 = rc * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  double ss = 0.0;
  for (int row = r0 + threadIdx.x; row < r1; row += kBlock) {
    // eight independent loads per round, four accumulators
    double a[4] = {(double)p[row], 0.0, 0.0, 0.0};
    int c = 0;
    for (; c + 8 <= nq; c += 8) {
      double q[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) q[j] = (double)Q[(size_t)(c + j) * ldq + row];
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j & 3] = fma(-q[j], hs[c + j], a[j & 3]);
    }
    for (; c < nq; ++c) a[0] = fma(-(double)Q[(size_t)c * ldq + row], hs[c], a[0]);
    const T pv = (T)((a[0] + a[1]) + (a[2] + a[3]));
    p[row] = pv;
    pc[row - r0] = (double)pv;
    ss = fma((double)pv, (double)pv, ss);
  }
  __syncthreads();
  if constexpr (!SECOND) {
    for (int c0 = 0; c0 <= nq; c0 += kTile)
      tile_partials<T>([&](int row) { return pc[row - r0]; }, r0, r1, Q, ldq, nq, c0, part_out,
                       gridDim.x, rc, sred);
  } else {
    const double tot = block_sum(ss, sbuf);
    if (threadIdx.x == 0) part_out[rc] = tot;
  }
}

// out = p / |p| with |p|^2 = sum of part[0..np) (summed by every workgroup in
// the same order); workgroup 0 stores |p| in *coef_out.  out = 0 when |p|
// underflows.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gs_scale(const T *__restrict__ p, int n,
                                                     const double *__restrict__ part, int np,
                                                     T *__restrict__ out, double *__restrict__ coef_out) {
  __shared__ double hs[1];
  __shared__ double scratch[kBlock];
  reduce_columns(part, np, 1, hs, scratch);
  const double nrm = sqrt(hs[0]);
  const double inv = (nrm > norm_floor<T>()) ? 1.0 / nrm : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *coef_out = nrm;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
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

// Ritz vectors: a thread owns one row and a tile of up to 4 outputs.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ritz(const T *__restrict__ Q, int64_t ldq, int nrows, int k,
                                                 const double *__restrict__ P, const double *__restrict__ w,
                                                 int r, T *__restrict__ out, int rs) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int l0 = blockIdx.y * 4;
  if (i >= nrows) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < k; ++c) {
    const double q = (double)Q[(size_t)c * ldq + i];
    const double *pr = P + (size_t)c * r;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (l0 + t < r) acc[t] = fma(q, pr[l0 + t], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int l = l0 + t;
    if (l < r) out[(size_t)i * rs + l] = (T)(w ? acc[t] * w[l] : acc[t]);
    else if (l < rs) out[(size_t)i * rs + l] = (T)0;
  }
}

// Sampled product, residual and iterate update in one pass over a compressed
// orientation of Omega.  The dot product is the same fma chain in either
// orientation (u-factor entry first), so the row- and column-compressed
// copies of Y receive bit-identical updates.  Each workgroup writes its
// (compensated) sum of e^2; the host adds the partials in order.
template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename T>
__device__ __forceinline__ T sampled_dot(const T *__restrict__ urow, const T *__restrict__ vrow, int r) {
  T x = (T)0;
  for (int l = 0; l < r; ++l) x = fma(urow[l], vrow[l], x);
  return x;
}

// RB > 0: the fixed (row-side) factor row is held in RB registers (r <= RB);
// RB == 0: any r, both factors read from memory.
template <typename T, int L, int RB>
__global__ __launch_bounds__(kBlock) void k_sample_update(
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx, const T *__restrict__ M,
    T *__restrict__ Y, int nrows, int rows_per_blk, const T *__restrict__ Fu, const T *__restrict__ Fv,
    int r, int rs, int row_side_is_u, T delta, double *__restrict__ part_out) {
  __shared__ double sbuf[kWaves];
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  constexpr int kGroups = kBlock / L;
  const T *other = row_side_is_u ? Fv : Fu;
  T sum = (T)0, comp = (T)0;  // compensated sum of e^2
  for (int row = r0 + grp; row < r1; row += kGroups) {
    const int beg = ptr[row], end = ptr[row + 1];
    const T *fixed = (row_side_is_u ? Fu : Fv) + (size_t)row * rs;
    T f[RB > 0 ? RB : 1];
    if constexpr (RB > 0) {
#pragma unroll
      for (int l = 0; l < RB; ++l) f[l] = (l < r) ? fixed[l] : (T)0;
    }
    for (int t = beg + lane; t < end; t += L) {
      const T *g = other + (size_t)idx[t] * rs;
      T x = (T)0;
      if constexpr (RB > 0) {
        // pairs of factor entries per load (rows are 2-element aligned: the
        // row stride is even and the padding is zero); the fma chain still
        // runs in l order with the u-factor entry first, in either orientation
#pragma unroll
        for (int l = 0; l < RB; l += 2) {
          if (l < r) {
            const auto gv = *reinterpret_cast<const typename Vec2<T>::type *>(g + l);
            if (row_side_is_u) {
              x = fma(f[l], gv.x, x);
              if (l + 1 < r) x = fma(f[l + 1], gv.y, x);
            } else {
              x = fma(gv.x, f[l], x);
              if (l + 1 < r) x = fma(gv.y, f[l + 1], x);
            }
          }
        }
      } else {
        x = row_side_is_u ? sampled_dot<T>(fixed, g, r) : sampled_dot<T>(g, fixed, r);
      }
      const T e = M[t] - x;
      Y[t] = fma(delta, e, Y[t]);
      const T yk = fma(e, e, -comp);
      const T tk = sum + yk;
      comp = (tk - sum) - yk;
      sum = tk;
    }
  }
  if (part_out == nullptr) return;  // uniform: no residual wanted
  const double tot = block_sum((double)sum - (double)comp, sbuf);
  if (threadIdx.x == 0) part_out[blockIdx.x] = tot;
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

GsPlan gs_plan(int nrows) {
  GsPlan g;
  const RowChunks a = row_chunks(nrows, std::max(kBlock, (nrows + kGsChunks1 - 1) / kGsChunks1));
  const RowChunks b = row_chunks(nrows, std::max(kBlock, (nrows + kGsChunks2 - 1) / kGsChunks2));
  g.nrc1 = a.nblk;
  g.rpb1 = a.rows_per_blk;
  g.nrc2 = b.nblk;
  g.rpb2 = b.rows_per_blk;
  return g;
}

size_t gs_update_lds(int nq, int rows_per_blk) {
  return sizeof(double) * ((size_t)nq + 1 + kBlock + (size_t)rows_per_blk);
}

// The dynamic-LDS limit is a per-kernel attribute shared by every stream and
// thread: raise it once to the largest size any plan uses (the device's
// per-workgroup maximum) and never lower it, so concurrent solves with
// different plans cannot shrink it under each other's launches.
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
  // the dynamic limit plus the kernel's static LDS must fit the device's
  // per-workgroup maximum
  const size_t room = (size_t)maxlds > fa.sharedSizeBytes ? (size_t)maxlds - fa.sharedSizeBytes : 0;
  if (bytes > room) return hipErrorInvalidValue;
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)room);
  if (e != hipSuccess) return e;
  raised[kern] = room;
  return hipSuccess;
}

template <typename T>
hipError_t launch_spmv(hipStream_t s, int lanes, const SpmvLdsPlan *pl, const int32_t *ptr, const int32_t *idx,
                       const T *val, const int32_t *segptr, const T *x, const double *xpart, int xnp, T *x_out,
                       double *s_out, int ncols, const T *prev, T *p, int nrows) {
  if (pl) {
    if (!pl->ok || (pl->nseg > 1 && segptr == nullptr)) return hipErrorInvalidValue;
    lanes = pl->lanes;
#define SVT_SPMVL(LN)                                                                              \
  do {                                                                                            \
    auto kern = k_spmv_lds<T, LN>;                                                                \
    hipError_t ea = allow_dynamic_lds(reinterpret_cast<const void *>(kern), pl->lds);             \
    if (ea != hipSuccess) return ea;                                                              \
    SVT_LAUNCH(kern, dim3(pl->nblk), dim3(kSpmvBlock), pl->lds, s, ptr, idx, val, segptr, \
                       pl->nseg, pl->segcols, x, xpart, xnp, x_out, s_out, ncols, prev, p, nrows,  \
                       pl->rows_per_blk);                                                         \
  } while (0)
    switch (lanes) {
      case 4: SVT_SPMVL(4); break;
      case 8: SVT_SPMVL(8); break;
      case 16: SVT_SPMVL(16); break;
      case 32: SVT_SPMVL(32); break;
      default: SVT_SPMVL(64); break;
    }
#undef SVT_SPMVL
    return hipGetLastError();
  }
#define SVT_SPMV(LN)                                                                              \
  SVT_LAUNCH((k_spmv<T, LN>), dim3((nrows + kBlock / LN - 1) / (kBlock / LN)), dim3(kBlock), 0, s, \
                     ptr, idx, val, x, xpart, xnp, x_out, s_out, ncols, prev, p, nrows)
  switch (lanes) {
    case 4: SVT_SPMV(4); break;
    case 8: SVT_SPMV(8); break;
    case 16: SVT_SPMV(16); break;
    case 32: SVT_SPMV(32); break;
    default: SVT_SPMV(64); break;
  }
#undef SVT_SPMV
  return hipGetLastError();
}

SpmvLdsPlan spmv_lds_plan(int nrows, int ncols, int elem_bytes, int num_cus, int lds_bytes) {
  SpmvLdsPlan pl{};
  pl.nblk = std::max(1, std::min(num_cus, (nrows + 7) / 8));
  pl.rows_per_blk = (nrows + pl.nblk - 1) / pl.nblk;
  pl.nblk = (nrows + pl.rows_per_blk - 1) / pl.rows_per_blk;
  // 1 KiB of headroom for the kernel's static LDS
  const long budget = ((long)lds_bytes - 1024) / elem_bytes - pl.rows_per_blk;
  long seg = std::min<long>(ncols, budget);
  if (seg < ncols) seg = (seg / 64) * 64;
  pl.segcols = (int)std::max<long>(seg, 0);
  pl.nseg = pl.segcols > 0 ? (ncols + pl.segcols - 1) / pl.segcols : 0;
  pl.lds = (size_t)elem_bytes * ((size_t)pl.segcols + (size_t)pl.rows_per_blk);
  // lanes per row: the widest power of two that still runs all of a
  // workgroup's rows at once (4 .. 64)
  pl.lanes = 64;
  while (pl.lanes > 4 && (kSpmvBlock / pl.lanes) < pl.rows_per_blk) pl.lanes /= 2;
  // one segment holding all of x, or a few segments that are not tiny
  pl.ok = pl.segcols >= 1 && (pl.nseg == 1 || (pl.segcols >= 1024 && pl.nseg <= 8));
  return pl;
}

template <typename T>
hipError_t launch_sumsq(hipStream_t s, T *p, int nrows, const GsScratch &gs) {
  const GsPlan g = gs_plan(nrows);
  SVT_LAUNCH((k_gs_update<T, true>), dim3(g.nrc2), dim3(kBlock), gs_update_lds(0, g.rpb2), s, p, nrows,
                     g.rpb2, (const T *)nullptr, (int64_t)0, 0, gs.part1, 1, gs.part3);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(hipStream_t s, const T *p, int nrows, const GsScratch &gs, T *out,
                           double *coef_out) {
  const GsPlan g = gs_plan(nrows);
  SVT_LAUNCH((k_gs_scale<T>), dim3(grid_for(nrows, 1024)), dim3(kBlock), 0, s, p, nrows, gs.part3, g.nrc2,
                     out, coef_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gs_dots(hipStream_t s, const T *p, int nrows, const T *Q, int64_t ldq, int nq,
                          const GsScratch &gs) {
  const GsPlan g = gs_plan(nrows);
  if (nq < 1 || g.nrc1 > kGsChunks1 || nq + 1 > gs.max_cols) return hipErrorInvalidValue;
  const int ntiles = (nq + 1 + kTile - 1) / kTile;
  SVT_LAUNCH((k_gs_dots<T>), dim3(g.nrc1, ntiles), dim3(kBlock), 0, s, p, nrows, g.rpb1, Q, ldq,
                     nq, gs.part1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gs_update(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                            const GsScratch &gs, bool second) {
  const GsPlan g = gs_plan(nrows);
  if (nq < 1 || g.nrc1 > kGsChunks1 || g.nrc2 > kGsChunks2 || nq + 1 > gs.max_cols) return hipErrorInvalidValue;
  const size_t lds = gs_update_lds(nq, g.rpb2);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  if (!second)
    SVT_LAUNCH((k_gs_update<T, false>), dim3(g.nrc2), dim3(kBlock), lds, s, p, nrows, g.rpb2, Q,
                       ldq, nq, gs.part1, g.nrc1, gs.part2);
  else
    SVT_LAUNCH((k_gs_update<T, true>), dim3(g.nrc2), dim3(kBlock), lds, s, p, nrows, g.rpb2, Q,
                       ldq, nq, gs.part2, g.nrc2, gs.part3);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_orthonormalize(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                                 const GsScratch &gs) {
  if (nq == 0) return launch_sumsq<T>(s, p, nrows, gs);
  hipError_t e = launch_gs_dots<T>(s, p, nrows, Q, ldq, nq, gs);
  if (e != hipSuccess) return e;
  e = launch_gs_update<T>(s, p, nrows, Q, ldq, nq, gs, false);
  if (e != hipSuccess) return e;
  return launch_gs_update<T>(s, p, nrows, Q, ldq, nq, gs, true);
}

template <typename T>
hipError_t launch_randn(hipStream_t s, T *out, int n, uint64_t seed, uint64_t ctr) {
  SVT_LAUNCH((k_randn<T>), dim3(grid_for(n, 2048)), dim3(kBlock), 0, s, out, n, seed, ctr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ritz(hipStream_t s, const T *Q, int64_t ldq, int nrows, int k, const double *P,
                       const double *w, int r, T *out, int rs) {
  if (rs < 1) return hipSuccess;
  dim3 grid((nrows + kBlock - 1) / kBlock, (rs + 3) / 4);
  SVT_LAUNCH((k_ritz<T>), grid, dim3(kBlock), 0, s, Q, ldq, nrows, k, P, w, r, out, rs);
  return hipGetLastError();
}

int sample_blocks(int nrows, int lanes) {
  return row_chunks(nrows, std::max((kBlock / lanes) * 4, (nrows + kSampleMaxBlocks - 1) / kSampleMaxBlocks))
      .nblk;
}

template <typename T>
hipError_t launch_sample_update(hipStream_t s, int lanes, const int32_t *ptr, const int32_t *idx,
                                const T *M, T *Y, int nrows, const T *Fu, const T *Fv, int r, int rs,
                                bool row_side_is_u, double delta, double *part_out) {
  const RowChunks ch =
      row_chunks(nrows, std::max((kBlock / lanes) * 4, (nrows + kSampleMaxBlocks - 1) / kSampleMaxBlocks));
#define SVT_SU2(LN, RB)                                                                          \
  SVT_LAUNCH((k_sample_update<T, LN, RB>), dim3(ch.nblk), dim3(kBlock), 0, s, ptr, idx, M, Y, \
                     nrows, ch.rows_per_blk, Fu, Fv, r, rs, row_side_is_u ? 1 : 0, (T)delta, part_out)
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
  SVT_LAUNCH((k_gather<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, x, map, y, n);
  return hipGetLastError();
}

#define SVT_INSTANTIATE(T)                                                                          \
  template hipError_t launch_spmv<T>(hipStream_t, int, const SpmvLdsPlan *, const int32_t *,          \
                                     const int32_t *, const T *, const int32_t *, const T *,          \
                                     const double *, int, T *, double *, int, const T *, T *, int);   \
  template hipError_t launch_orthonormalize<T>(hipStream_t, T *, int, const T *, int64_t, int,     \
                                               const GsScratch &);                                  \
  template hipError_t launch_gs_dots<T>(hipStream_t, const T *, int, const T *, int64_t, int,      \
                                        const GsScratch &);                                         \
  template hipError_t launch_gs_update<T>(hipStream_t, T *, int, const T *, int64_t, int,          \
                                          const GsScratch &, bool);                                 \
  template hipError_t launch_sumsq<T>(hipStream_t, T *, int, const GsScratch &);                    \
  template hipError_t launch_finalize<T>(hipStream_t, const T *, int, const GsScratch &, T *, double *); \
  template hipError_t launch_randn<T>(hipStream_t, T *, int, uint64_t, uint64_t);                  \
  template hipError_t launch_ritz<T>(hipStream_t, const T *, int64_t, int, int, const double *,    \
                                     const double *, int, T *, int);                                \
  template hipError_t launch_sample_update<T>(hipStream_t, int, const int32_t *, const int32_t *,  \
                                              const T *, T *, int, const T *, const T *, int, int,  \
                                              bool, double, double *);                              \
  template hipError_t launch_axpby<T>(hipStream_t, const T *, T *, int64_t, double);               \
  template hipError_t launch_gather<T>(hipStream_t, const T *, const int32_t *, T *, int64_t);

SVT_INSTANTIATE(double)
SVT_INSTANTIATE(float)

}  // namespace svt
