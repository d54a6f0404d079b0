// gfx950 kernels of the SVT hot path (Algorithm 1 of Cai, Candes and Shen).
//
// Design notes (CDNA4):
//   * 64-lane wavefronts; a compressed row is handled by a sub-wave of
//     `lanes` (4..64) lanes chosen from the mean row length, so that lanes
//     stride contiguous index/value runs (coalesced) and a sub-wave shuffle
//     tree reduces the row;
//   * the vector-side reductions (Gram-Schmidt coefficients, norms, residual)
//     are deterministic: each workgroup owns a fixed chunk of rows, writes one
//     partial per output, and the last workgroup to arrive sums the partials
//     in a fixed order (no floating-point atomics, so results do not depend on
//     scheduling);
//   * the bidiagonalisation coefficients never leave the device inside a
//     step: kernels read them through pointers.
#include "svt_kernels.h"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdint>

namespace svt {

namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
// Second Gram-Schmidt pass when |p'| < eta |p| (Daniel-Gragg-Kaufman-Stewart).
constexpr double kEta2 = 0.5;

template <int W, typename A>
__device__ __forceinline__ A seg_sum(A v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_down(v, off, W);
  return v;  // first lane of each W-lane segment holds the sum
}

__device__ __forceinline__ double ld_acquire(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in every thread of the last workgroup to finish its partials.
// Writers publish with a device-scope fence before arriving; the last block
// fences again before it reads.
__device__ __forceinline__ bool last_block(unsigned *counter) {
  __shared__ unsigned s_prev;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_prev = atomicAdd(counter, 1u);
  __syncthreads();
  const bool last = (s_prev == gridDim.x - 1);
  if (last) __threadfence();
  return last;
}

// As last_block, for `total` arrivals on this counter (e.g. one grid column).
__device__ __forceinline__ bool last_block_of(unsigned *counter, unsigned total) {
  __shared__ unsigned s_prev2;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_prev2 = atomicAdd(counter, 1u);
  __syncthreads();
  const bool last = (s_prev2 == total - 1);
  if (last) __threadfence();
  return last;
}

// Sum of partial[col * nblk + 0..nblk-1] in a fixed order, by one wave.
__device__ __forceinline__ double reduce_partials(const double *partial, int col, int nblk, int wl) {
  const double *src = partial + (size_t)col * nblk;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = wl;
  for (; i + 3 * kWave < nblk; i += 4 * kWave) {
    a0 += src[i];
    a1 += src[i + kWave];
    a2 += src[i + 2 * kWave];
    a3 += src[i + 3 * kWave];
  }
  for (; i < nblk; i += kWave) a0 += src[i];
  return seg_sum<kWave>((a0 + a1) + (a2 + a3));
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

// Dot products of the chunk's p (in LDS, as double) with Q[:, 0..nq-1] and
// with itself (column nq); one wave per column.
template <typename T>
__device__ __forceinline__ void chunk_dots(const double *ps, int r0, int r1, const T *__restrict__ Q,
                                           int64_t ldq, int nq, double *partial, int nblk) {
  const int w = threadIdx.x / kWave, wl = threadIdx.x % kWave;
  for (int col = w; col <= nq; col += kWaves) {
    double acc = 0.0;
    if (col < nq) {
      const T *qc = Q + (size_t)col * ldq;
      for (int row = r0 + wl; row < r1; row += kWave) acc = fma((double)qc[row], ps[row - r0], acc);
    } else {
      for (int row = r0 + wl; row < r1; row += kWave) acc = fma(ps[row - r0], ps[row - r0], acc);
    }
    acc = seg_sum<kWave>(acc);
    if (wl == 0) partial[(size_t)col * nblk + blockIdx.x] = acc;
  }
}

// ---------------------------------------------------------------------------
// p = A x - coef prev over a compressed orientation (one sub-wave per row).
template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_spmv(
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx, const T *__restrict__ val,
    const T *__restrict__ x, const T *__restrict__ prev, const double *__restrict__ coef,
    T *__restrict__ p, int nrows) {
  const int lane = threadIdx.x % L;
  constexpr int kGroups = kBlock / L;
  const int row = blockIdx.x * kGroups + threadIdx.x / L;
  if (row >= nrows) return;  // whole sub-wave leaves together
  const int beg = ptr[row], end = ptr[row + 1];
  T acc = (T)0;
  for (int t = beg + lane; t < end; t += L) acc = fma(val[t], x[idx[t]], acc);
  acc = seg_sum<L>(acc);
  if (lane == 0) p[row] = prev ? fma(-(T)(*coef), prev[row], acc) : acc;
}

constexpr int kTile = 16;  // Gram-Schmidt coefficients per workgroup

// h = Q^T p (nq columns) and h[nq] = |p|^2, on a (row chunk, column tile)
// grid: every thread issues its tile's loads together and the 16 partial sums
// reduce as independent shuffle chains; the last row chunk to finish a tile
// sums that tile's partials.  With `flag` non-null the kernel does nothing
// unless *flag is set (the optional second Gram-Schmidt pass).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dots(
    const T *__restrict__ p, int nrows, int rows_per_blk, const T *__restrict__ Q, int64_t ldq,
    int nq, const double *__restrict__ flag, double *__restrict__ partial, double *__restrict__ h_out,
    double *__restrict__ norm_out, unsigned *__restrict__ counters) {
  if (flag && *flag == 0.0) return;  // uniform across the grid
  __shared__ double sred[kWaves][kTile];
  const int rc = blockIdx.x, nrc = gridDim.x;
  const int c0 = blockIdx.y * kTile;
  const int r0 = rc * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  double acc[kTile];
#pragma unroll
  for (int j = 0; j < kTile; ++j) acc[j] = 0.0;
  for (int row = r0 + threadIdx.x; row < r1; row += kBlock) {
    const double pv = (double)p[row];
#pragma unroll
    for (int j = 0; j < kTile; ++j) {
      const int c = c0 + j;
      if (c < nq) acc[j] = fma((double)Q[(size_t)c * ldq + row], pv, acc[j]);
      else if (c == nq) acc[j] = fma(pv, pv, acc[j]);
    }
  }
  const int w = threadIdx.x / kWave, wl = threadIdx.x % kWave;
#pragma unroll
  for (int j = 0; j < kTile; ++j) {
    const double v = seg_sum<kWave>(acc[j]);
    if (wl == 0) sred[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < kTile) {
    const int c = c0 + threadIdx.x;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += sred[i][threadIdx.x];
    if (c <= nq) partial[(size_t)c * nrc + rc] = t;
  }
  if (last_block_of(counters + blockIdx.y, nrc)) {
    for (int j = w; j < kTile; j += kWaves) {
      const int c = c0 + j;
      if (c > nq) break;
      const double s = reduce_partials(partial, c, nrc, wl);
      if (wl == 0) {
        h_out[c] = s;
        if (c == nq) *norm_out = sqrt(s);
      }
    }
    if (threadIdx.x == 0) counters[blockIdx.y] = 0u;
  }
}

// p' = p - Q h1 (in place) and |p'|^2.  The last workgroup takes the
// Daniel-Gragg-Kaufman-Stewart decision: a second pass is flagged in scal[3]
// when |p'|^2 < eta^2 |p|^2 (or when forced); otherwise norm_out = |p'|.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgs_update(
    T *__restrict__ p, int nrows, int rows_per_blk, const T *__restrict__ Q, int64_t ldq, int nq,
    const double *__restrict__ h1, double *__restrict__ partial, double *__restrict__ scal,
    double *__restrict__ norm_out, int force_second, unsigned *__restrict__ counter) {
  extern __shared__ double hs[];  // nq coefficients
  __shared__ double sbuf[kWaves];
  for (int c = threadIdx.x; c < nq; c += kBlock) hs[c] = h1[c];
  __syncthreads();
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  double ss = 0.0;
  for (int row = r0 + threadIdx.x; row < r1; row += kBlock) {
    double a0 = (double)p[row], a1 = 0.0;
    int c = 0;
    for (; c + 1 < nq; c += 2) {
      a0 = fma(-(double)Q[(size_t)c * ldq + row], hs[c], a0);
      a1 = fma(-(double)Q[(size_t)(c + 1) * ldq + row], hs[c + 1], a1);
    }
    if (c < nq) a0 = fma(-(double)Q[(size_t)c * ldq + row], hs[c], a0);
    const T pv = (T)(a0 + a1);
    p[row] = pv;
    ss = fma((double)pv, (double)pv, ss);
  }
  const double tot = block_sum(ss, sbuf);
  const int nblk = gridDim.x;
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
  if (last_block(counter)) {
    if (threadIdx.x < kWave) {
      const double pp2 = reduce_partials(partial, 0, nblk, threadIdx.x);
      if (threadIdx.x == 0) {
        const double pp1 = h1[nq];
        const bool second = (nq > 0) && (force_second || (pp2 < kEta2 * pp1));
        scal[3] = second ? 1.0 : 0.0;
        if (!second) *norm_out = sqrt(pp2);
      }
    }
    if (threadIdx.x == 0) *counter = 0u;
  }
}

// Optional second Gram-Schmidt pass and the final norm.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgs_finish(
    T *__restrict__ p, int nrows, int rows_per_blk, const T *__restrict__ Q, int64_t ldq, int nq,
    const double *__restrict__ h2, double *__restrict__ partial, const double *__restrict__ scal,
    double *__restrict__ norm_out, unsigned *__restrict__ counter) {
  if (scal[3] == 0.0) return;  // uniform across the grid
  extern __shared__ double hs[];
  __shared__ double sbuf[kWaves];
  for (int c = threadIdx.x; c < nq; c += kBlock) hs[c] = h2[c];
  __syncthreads();
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(nrows, r0 + rows_per_blk);
  double ss = 0.0;
  for (int row = r0 + threadIdx.x; row < r1; row += kBlock) {
    double acc = (double)p[row];
    for (int c = 0; c < nq; ++c) acc = fma(-(double)Q[(size_t)c * ldq + row], hs[c], acc);
    const T pv = (T)acc;
    p[row] = pv;
    ss = fma((double)pv, (double)pv, ss);
  }
  const double tot = block_sum(ss, sbuf);
  const int nblk = gridDim.x;
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
  if (last_block(counter)) {
    if (threadIdx.x < kWave) {
      const double s = reduce_partials(partial, 0, nblk, threadIdx.x);
      if (threadIdx.x == 0) *norm_out = sqrt(s);
    }
    if (threadIdx.x == 0) *counter = 0u;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale(const T *__restrict__ p, const double *__restrict__ nrm,
                                                  T *__restrict__ out, int n) {
  const double v = *nrm;
  const double inv = (v > 1e-280) ? 1.0 / v : 0.0;
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
// copies of Y receive bit-identical updates.
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
    int r, int rs, int row_side_is_u, T delta, double *__restrict__ partial,
    double *__restrict__ res2_out, unsigned *__restrict__ counter) {
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
  if (res2_out == nullptr) return;  // uniform: no residual wanted
  const double tot = block_sum((double)sum - (double)comp, sbuf);
  const int nblk = gridDim.x;
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
  if (last_block(counter)) {
    if (threadIdx.x < kWave) {
      const double s = reduce_partials(partial, 0, nblk, threadIdx.x);
      if (threadIdx.x == 0) *res2_out = s;
    }
    if (threadIdx.x == 0) *counter = 0u;
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

// Chunking of the Gram-Schmidt kernels: at most 256 workgroups (so the last
// one reduces at most 256 partials per coefficient) of at least 256 rows.
RowChunks vec_chunks(int nrows) {
  int nblk = (nrows + kBlock - 1) / kBlock;
  if (nblk > 256) nblk = 256;
  if (nblk < 1) nblk = 1;
  return row_chunks(nrows, (nrows + nblk - 1) / nblk);
}

template <typename T>
hipError_t launch_spmv(hipStream_t s, int lanes, const int32_t *ptr, const int32_t *idx, const T *val,
                       const T *x, const T *prev, const double *coef, T *p, int nrows) {
#define SVT_SPMV(LN)                                                                            \
  hipLaunchKernelGGL((k_spmv<T, LN>), dim3((nrows + kBlock / LN - 1) / (kBlock / LN)), dim3(kBlock), \
                     0, s, ptr, idx, val, x, prev, coef, p, nrows)
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

template <typename T>
hipError_t launch_dots_into(hipStream_t s, const T *p, int nrows, const T *Q, int64_t ldq, int nq,
                            const double *flag, double *h_out, unsigned *counters, ReduceScratch &rs,
                            double *norm_out) {
  const RowChunks ch = vec_chunks(nrows);
  if (ch.nblk > rs.max_blocks) return hipErrorInvalidValue;
  const int ntiles = (nq + 1 + kTile - 1) / kTile;
  if (ntiles > kMaxTiles) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_dots<T>), dim3(ch.nblk, ntiles), dim3(kBlock), 0, s, p, nrows, ch.rows_per_blk,
                     Q, ldq, nq, flag, rs.partial, h_out, norm_out, counters);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dots(hipStream_t s, const T *p, int nrows, const T *Q, int64_t ldq, int nq,
                       ReduceScratch &rs, double *norm_out) {
  return launch_dots_into<T>(s, p, nrows, Q, ldq, nq, nullptr, rs.h1, rs.counters + kCounterDots, rs,
                             norm_out);
}

template <typename T>
hipError_t launch_cgs_update(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                             ReduceScratch &rs, double *norm_out, int force_second) {
  const RowChunks ch = vec_chunks(nrows);
  if (ch.nblk > rs.max_blocks) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * (size_t)nq;
  if (lds > 60 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_cgs_update<T>), dim3(ch.nblk), dim3(kBlock), lds, s, p, nrows, ch.rows_per_blk,
                     Q, ldq, nq, rs.h1, rs.partial, rs.scal, norm_out, force_second,
                     rs.counters + kCounterUpdate);
  return hipGetLastError();
}

// Second pass when flagged: h2 = Q^T p', then p'' = p' - Q h2 and its norm.
template <typename T>
hipError_t launch_cgs_finish(hipStream_t s, T *p, int nrows, const T *Q, int64_t ldq, int nq,
                             ReduceScratch &rs, double *norm_out) {
  hipError_t e = launch_dots_into<T>(s, p, nrows, Q, ldq, nq, rs.scal + 3, rs.h2,
                                     rs.counters + kCounterDots2, rs, rs.scal + 5);
  if (e != hipSuccess) return e;
  const RowChunks ch = vec_chunks(nrows);
  const size_t lds = sizeof(double) * (size_t)nq;
  if (lds > 60 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_cgs_finish<T>), dim3(ch.nblk), dim3(kBlock), lds, s, p, nrows, ch.rows_per_blk,
                     Q, ldq, nq, rs.h2, rs.partial, rs.scal, norm_out, rs.counters + kCounterFinish);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale(hipStream_t s, const T *p, const double *nrm, T *out, int n) {
  hipLaunchKernelGGL((k_scale<T>), dim3(grid_for(n, 2048)), dim3(kBlock), 0, s, p, nrm, out, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_randn(hipStream_t s, T *out, int n, uint64_t seed, uint64_t ctr) {
  hipLaunchKernelGGL((k_randn<T>), dim3(grid_for(n, 2048)), dim3(kBlock), 0, s, out, n, seed, ctr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ritz(hipStream_t s, const T *Q, int64_t ldq, int nrows, int k, const double *P,
                       const double *w, int r, T *out, int rs) {
  if (rs < 1) return hipSuccess;
  dim3 grid((nrows + kBlock - 1) / kBlock, (rs + 3) / 4);
  hipLaunchKernelGGL((k_ritz<T>), grid, dim3(kBlock), 0, s, Q, ldq, nrows, k, P, w, r, out, rs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sample_update(hipStream_t s, int lanes, const int32_t *ptr, const int32_t *idx,
                                const T *M, T *Y, int nrows, const T *Fu, const T *Fv, int r, int rs,
                                bool row_side_is_u, double delta, ReduceScratch &rsc,
                                double *res2_out) {
  const RowChunks ch = row_chunks(nrows, std::max((kBlock / lanes) * 4, (nrows + 1023) / 1024));
  if (res2_out && ch.nblk > rsc.max_blocks) return hipErrorInvalidValue;
#define SVT_SU2(LN, RB)                                                                          \
  hipLaunchKernelGGL((k_sample_update<T, LN, RB>), dim3(ch.nblk), dim3(kBlock), 0, s, ptr, idx, M, Y, \
                     nrows, ch.rows_per_blk, Fu, Fv, r, rs, row_side_is_u ? 1 : 0, (T)delta,          \
                     rsc.partial, res2_out, rsc.counters + kCounterSample)
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
  hipLaunchKernelGGL((k_axpby<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n, a);
  return hipGetLastError();
}

hipError_t launch_d2f(hipStream_t s, const double *x, float *y, int64_t n) {
  hipLaunchKernelGGL(k_d2f, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t launch_f2d(hipStream_t s, const float *x, double *y, int64_t n) {
  hipLaunchKernelGGL(k_f2d, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(hipStream_t s, const T *x, const int32_t *map, T *y, int64_t n) {
  hipLaunchKernelGGL((k_gather<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, x, map, y, n);
  return hipGetLastError();
}

#define SVT_INSTANTIATE(T)                                                                          \
  template hipError_t launch_spmv<T>(hipStream_t, int, const int32_t *, const int32_t *, const T *,   \
                                     const T *, const T *, const double *, T *, int);              \
  template hipError_t launch_dots<T>(hipStream_t, const T *, int, const T *, int64_t, int,         \
                                     ReduceScratch &, double *);                                    \
  template hipError_t launch_cgs_update<T>(hipStream_t, T *, int, const T *, int64_t, int,         \
                                           ReduceScratch &, double *, int);                         \
  template hipError_t launch_cgs_finish<T>(hipStream_t, T *, int, const T *, int64_t, int,         \
                                           ReduceScratch &, double *);                              \
  template hipError_t launch_scale<T>(hipStream_t, const T *, const double *, T *, int);           \
  template hipError_t launch_randn<T>(hipStream_t, T *, int, uint64_t, uint64_t);                  \
  template hipError_t launch_ritz<T>(hipStream_t, const T *, int64_t, int, int, const double *,    \
                                     const double *, int, T *, int);                                \
  template hipError_t launch_sample_update<T>(hipStream_t, int, const int32_t *, const int32_t *,  \
                                              const T *, T *, int, const T *, const T *, int, int,  \
                                              bool, double, ReduceScratch &, double *);             \
  template hipError_t launch_axpby<T>(hipStream_t, const T *, T *, int64_t, double);               \
  template hipError_t launch_gather<T>(hipStream_t, const T *, const int32_t *, T *, int64_t);

SVT_INSTANTIATE(double)
SVT_INSTANTIATE(float)

}  // namespace svt
