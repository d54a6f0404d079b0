// Host driver of the SVT iteration and the C ABI (include/svt.h).
//
// Algorithm 1 of Cai, Candes and Shen (Section 5.1.5) on one GPU:
//   a1  setup: Omega in row- and column-compressed form (int32), values and
//       P_Omega(M) uploaded once (Section 2.2, sparsity property);
//   a2  kick: ||P_Omega M||_2 by bidiagonalisation, k0 from eq. (5.3),
//       Y = k0 delta P_Omega(M);
//   a3  Golub-Kahan-Lanczos bidiagonalisation of the sparse iterate with full
//       reorthogonalisation (Section 5.1.1 computes the partial SVD this way);
//   a4  s_k = r_{k-1} + 1, grown by ell while the s_k-th value is above tau;
//       the bidiagonalisation is extended, never restarted (Section 5.1.1);
//   a5  shrink: r_k = #{sigma_j > tau}, w_j = sigma_j - tau (eq. (2.2));
//   a6  Ritz vectors U diag(w), V from the bases (dense, small);
//   a7/a8 sampled product, residual and the update of Y in one pass per
//       compressed copy, stop test of eq. (5.5) (or eq. (5.10)).
//
// Orientation: the bidiagonalisation runs on A = Y when m >= n and on A = Y^T
// otherwise, so its right-hand basis spans the smaller dimension and can be
// completed exactly when every singular value is needed.
#include "../../include/svt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "bidiag.h"
#include "dense_host.h"
#include "orth_estimate.h"
#include "svt_kernels.h"

namespace svt {

// ---------------------------------------------------------------------------
// errors

struct Error : std::runtime_error {
  svt_status code;
  Error(svt_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIP_CHECK(expr)                                                                          \
  do {                                                                                           \
    hipError_t _e = (expr);                                                                      \
    if (_e != hipSuccess)                                                                        \
      throw Error(_e == hipErrorOutOfMemory ? SVT_ENOMEM : SVT_EDEVICE,                          \
                  std::string(#expr) + ": " + hipGetErrorString(_e));                            \
  } while (0)

static thread_local std::string g_create_error = "";

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// device memory

// Stream-ordered device memory: allocated and freed in the order of the
// handle's stream (hipMallocAsync / hipFreeAsync from the device's pool), so
// freeing a buffer never waits for the whole device -- a served solve that
// ends or grows its bases does not stall the solves on other streams.  The
// owner releases every buffer before its stream is destroyed.
struct DevMem {
  void *p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  DevMem() = default;
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
  ~DevMem() { release(); }
  void release() {
    if (p) (void)hipFreeAsync(p, s);
    p = nullptr;
    bytes = 0;
  }
  void alloc(hipStream_t st, size_t b) {
    release();
    if (b == 0) b = 8;
    s = st;
    HIP_CHECK(hipMallocAsync(&p, b, st));
    bytes = b;
  }
  template <typename T>
  T *as() const { return static_cast<T *>(p); }
};

// Pinned host memory for the small transfers of every SVT iteration (the
// bidiagonal coefficients, the Ritz combination, the residual partials):
// copies from pageable memory cost tens of microseconds each.
struct PinnedMem {
  void *p = nullptr;
  size_t bytes = 0;
  PinnedMem() = default;
  PinnedMem(const PinnedMem &) = delete;
  PinnedMem &operator=(const PinnedMem &) = delete;
  ~PinnedMem() {
    if (p) (void)hipHostFree(p);
  }
  // Room for b bytes (contents not kept).  Callers synchronise the stream
  // before the buffer is written again.
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    HIP_CHECK(hipHostMalloc(&p, b, hipHostMallocDefault));
    bytes = b;
  }
  template <typename U>
  U *as() const { return static_cast<U *>(p); }
};

// ---------------------------------------------------------------------------
// kernel-class timing with HIP events (params.profile = 1)

// One kind per kernel (each bracket times exactly one launch):
//   0 k_spmv_rows (with the deferred one-pass update of its input and the
//   dot products of its output), 1 k_gather4 (column copy of Y), 2
//   k_gs_update (first of two
//   passes, with the second pass's dot products), 3 k_ritz, 4
//   k_sample_update, 5 k_gs_update (one pass with the |p|^2 partials: the
//   second of two, or a deferred update too wide to fuse).
enum KernelKind {
  kSpmv = 0, kGather = 1, kGsUpdate1 = 2, kRitz = 3, kSample = 4, kGsUpdate2 = 5, kPendReduce = 6, kKinds = 7
};

struct Profiler {
  bool on = false;
  hipStream_t stream = nullptr;
  struct Pending { hipEvent_t a, b; int kind; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[kKinds] = {};
  double ms[kKinds] = {};
  double bytes[kKinds] = {};
  hipEvent_t cur_a = nullptr;

  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    return e;
  }
  hipEvent_t cur_b = nullptr;
  // The bracketed launch stamps the pair itself (set_launch_events), so the
  // time is the kernel's own duration.
  void begin() {
    if (!on) return;
    cur_a = get();
    cur_b = get();
    set_launch_events(cur_a, cur_b);
  }
  void end(int kind, double nbytes) {
    if (!on) return;
    set_launch_events(nullptr, nullptr);  // in case the bracket launched nothing
    pending.push_back({cur_a, cur_b, kind});
    launches[kind] += 1;
    bytes[kind] += nbytes;
  }
  // Resolve recorded pairs (the stream must be synchronised).
  void flush() {
    for (auto &p : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) ms[p.kind] += t;
      else (void)hipGetLastError();
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  void reset() {
    for (int i = 0; i < kKinds; ++i) { launches[i] = 0; ms[i] = 0; bytes[i] = 0; }
  }
  ~Profiler() {
    for (auto &p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// ---------------------------------------------------------------------------
// host-side index build (a1)

struct Index {
  int64_t m = 0, n = 0, nnz = 0;
  std::vector<int32_t> rowptr, colidx;   // CSR
  std::vector<int32_t> colptr, rowidx;   // CSC
  std::vector<int32_t> csr_of_input;     // input position -> CSR position
  std::vector<int32_t> csc_of_csr;       // CSR position -> CSC position
  std::vector<double> vals_csr;
};

static void build_index(int64_t m, int64_t n, int64_t nnz, const int32_t *rows, const int32_t *cols,
                        const double *vals, Index &ix) {
  ix.m = m; ix.n = n; ix.nnz = nnz;
  // counting sort by row (stable), then sort each row by column
  ix.rowptr.assign((size_t)m + 1, 0);
  for (int64_t t = 0; t < nnz; ++t) ix.rowptr[(size_t)rows[t] + 1]++;
  for (int64_t i = 0; i < m; ++i) ix.rowptr[i + 1] += ix.rowptr[i];
  std::vector<int32_t> order((size_t)nnz);
  {
    std::vector<int32_t> fill(ix.rowptr.begin(), ix.rowptr.end() - 1);
    for (int64_t t = 0; t < nnz; ++t) order[(size_t)fill[rows[t]]++] = (int32_t)t;
  }
  for (int64_t i = 0; i < m; ++i) {
    auto b = order.begin() + ix.rowptr[i], e = order.begin() + ix.rowptr[i + 1];
    std::sort(b, e, [&](int32_t a, int32_t c) { return cols[a] < cols[c]; });
  }
  ix.colidx.resize((size_t)nnz);
  ix.vals_csr.resize((size_t)nnz);
  ix.csr_of_input.resize((size_t)nnz);
  for (int64_t t = 0; t < nnz; ++t) {
    const int32_t src = order[(size_t)t];
    ix.colidx[(size_t)t] = cols[src];
    ix.vals_csr[(size_t)t] = vals[src];
    ix.csr_of_input[(size_t)src] = (int32_t)t;
  }
  for (int64_t i = 0; i < m; ++i)
    for (int32_t t = ix.rowptr[i] + 1; t < ix.rowptr[i + 1]; ++t)
      if (ix.colidx[(size_t)t] == ix.colidx[(size_t)t - 1])
        throw Error(SVT_EINVAL, "duplicate position (" + std::to_string(i) + ", " +
                                    std::to_string(ix.colidx[(size_t)t]) + ") in Omega");
  // CSC by a stable counting sort of the CSR entries on the column
  ix.colptr.assign((size_t)n + 1, 0);
  for (int64_t t = 0; t < nnz; ++t) ix.colptr[(size_t)ix.colidx[(size_t)t] + 1]++;
  for (int64_t j = 0; j < n; ++j) ix.colptr[j + 1] += ix.colptr[j];
  ix.rowidx.resize((size_t)nnz);
  ix.csc_of_csr.resize((size_t)nnz);
  std::vector<int32_t> fill(ix.colptr.begin(), ix.colptr.end() - 1);
  for (int64_t i = 0; i < m; ++i)
    for (int32_t t = ix.rowptr[i]; t < ix.rowptr[i + 1]; ++t) {
      const int32_t pos = fill[ix.colidx[(size_t)t]]++;
      ix.rowidx[(size_t)pos] = (int32_t)i;
      ix.csc_of_csr[(size_t)t] = pos;
    }
}

// ---------------------------------------------------------------------------
// the solver state for one problem, templated on the bulk value type

struct Record {
  int32_t rank, s, steps;
  double res;
};

struct ProblemBase {
  virtual ~ProblemBase() = default;
  svt_params prm{};
  Index ix;
  double norm_pm = 0.0;
  std::string last_error;
  double t_setup = 0.0;
  virtual svt_status solve(svt_info *info) = 0;
  virtual void factors(int32_t *rank, double *U, double *w, double *V) const = 0;
  virtual void set_iterate(const double *y) = 0;
  virtual void get_iterate(int which, double *y) const = 0;
  virtual void set_multipliers(const double *yp, const double *ym) = 0;
  virtual void setup_sensing(int64_t p, const int64_t *gptr, const int32_t *gidx, const double *gval,
                             const double *b) = 0;
  virtual void get_multipliers(double *yp, double *ym) const = 0;
  bool ds_soft_nonzero = false;  // some |B_ij| > E (the Dantzig selector's kick exists)
  virtual void apply(int trans, const double *x, double *out) = 0;
  virtual int partial_svd(int count, double *sigma, double *U, double *V) = 0;
  virtual double sample_update(int r, const double *U, const double *V, double delta) = 0;
  virtual double sample_update_noalloc(int r, const void *U, const void *V, int64_t rs, double delta) = 0;
  virtual void kick(double *sigma1, int32_t *k0) = 0;
  // x segments staged in LDS by the row- (0) or column-compressed (1)
  // product; 0 when that product gathers x from memory
  virtual int spmv_segments(int which) const = 0;
  virtual void mem_stats(size_t *cur, size_t *peak) const = 0;
  virtual void reorth_stats(int64_t *vectors, int64_t *orthogonalised, int64_t *two_pass_restarts,
                            int64_t *partial_fallbacks) const = 0;
  size_t peak_bytes = 0;
  std::vector<Record> history;
  Profiler prof;
};

template <typename T>
struct Problem final : ProblemBase {
  // dimensions of the bidiagonalised orientation A
  int64_t arows = 0, acols = 0;
  bool a_is_y = true;
  int lanes_r = 32, lanes_c = 32;  // lanes per row of the CSR / CSC sampled updates
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;

  DevMem rowptr, colidx, colptr, rowidx, csr_of_csc;
  SpmvPlan plan_r{}, plan_c{};        // sparse products (CSR, CSC)
  int lds_limit = 64 * 1024;          // LDS bytes a workgroup may use
  DevMem seg_r, seg_c;                // their segment starts (when nseg > 1)
  DevMem colidx16, rowidx16;          // 16-bit copies of colidx / rowidx (n, m <= 65536)
  DevMem Mr, Mc, Yr, Yc;          // values, T
  DevMem Yp, Ym;                  // Dantzig selector: the two multipliers (row order), T
  // general linear operator A(X) = G x_S (svt_create_sensing): G and G^T in
  // compressed form over the measurements and the support, b, the dual
  // iterate y, and X on the support
  bool sensing = false;
  int64_t pmeas = 0;
  DevMem g_ptr, g_idx, g_val, gt_ptr, gt_idx, gt_val, b_d, y_d, xs_d;
  DevMem Ub, Vb;                  // bases, T, column-major
  int kcap = 0;                   // columns available in Ub (Vb has kcap + 1)
  DevMem pbuf_u, pbuf_v;          // unnormalised new vectors of each side, T
  DevMem coef;                    // alpha[0..], beta[0..], removed[0..]: double, 4 (kcap + 4)
  DevMem gs1, gs2, gs3;           // Gram-Schmidt partial sums
  DevMem gsr;                     // a pending vector's column sums (k_pending_reduce)
  GsScratch gs{};
  DevMem sample_part;             // residual partials, kSampleMaxBlocks + 8 doubles
  double *noalloc_part = nullptr; // the device's fixed scratch (svt_sample_update_noalloc)
  PinnedMem sample_host;          // their host copy
  DevMem ritzd;                   // Ritz combination (double): P (k x r), Q (k x r), w (r)
  PinnedMem ritz_host;            // its host staging
  PinnedMem coef_host;            // alpha and beta as fetched
  hipEvent_t fetch_ev = nullptr;  // behind the copy into coef_host
  int fetch_k = 0, fetch_kcap = 0;
  static constexpr int kAheadSteps = 2;  // steps queued while the host checks
  static constexpr int kProbeMaxK = 128;  // bases from which the first check does not probe below
  DevMem Fu, Fv;                  // factors of X, T, row-major with stride fstride
  int fstride = 0, fcap = 0;
  int rank = 0;
  std::vector<double> w;          // sigma - tau
  uint64_t rng_ctr = 0;
  uint64_t rs_ctr = 0;            // test matrices drawn by the randomised partial SVD in a solve
  DevMem rs_a, rs_b;              // its device blocks (rows x l, column-major, T)
  int k_hint = 0;
  int log_level = 0;
  int64_t steps_total = 0;
  double reorth_trigger = 0.5;
  // basis width from which a pending vector's partials are summed by their
  // own kernel before the sparse product: the width where the product
  // leaves its single-pass epilogue (below it each workgroup of the product
  // sums them in one pass, cheaper than the extra launch)
  int prereduce_min = 64;
  int passes_now = 2;          // Gram-Schmidt passes per vector right now
  int64_t reorth_restarts = 0; // bidiagonalisations restarted with two passes
  // partial reorthogonalisation (reorth_eta > 0): the schedule of the
  // current bidiagonalisation, whether it is still in use in this solve,
  // the growth factor carried to the next bidiagonalisation, and counts
  ReorthSchedule rsched;
  bool partial_now = false;
  bool partial_run = false;    // the current bidiagonalisation follows rsched
  bool full_this_run = false;  // ... unless its check failed: then all vectors
  double growth_carry = 0.0;
  int hold_hint = 0;           // no predicted trigger before this half-step
  // the vectors the exact policy orthogonalises, replayed on the previous SVT
  // step's coefficients (empty: none)
  std::vector<uint8_t> replay_hint;
  // the degrees-of-freedom bound (dof_bound): the largest rank it allows in
  // this solve (-1: off), and whether the current step passed it
  int dof_rmax = -1;
  bool dof_hit = false;
  int64_t vec_made = 0, vec_orth = 0, partial_fallbacks = 0;

  // the Dantzig-selector iteration (Section 3.3) instead of Algorithm 1's
  // equality-constrained one
  bool ds() const { return prm.constraint == SVT_CONSTRAINT_INEQUALITY; }

  // ----------------------------------------------------------------- setup
  void setup(const svt_params &p) {
    prm = p;
    if (const char *lv = std::getenv("SVT_LOG")) log_level = std::atoi(lv);
    // the one-pass check's threshold (test hook; default 1/2, the DGKS
    // criterion with eta = 1/sqrt(2))
    if (const char *tv = std::getenv("SVT_REORTH_TRIGGER")) reorth_trigger = std::atof(tv);
    // the basis width that switches on the separate partial sums (tuning
    // and test hook; both sides of it give the same bits)
    if (const char *pv = std::getenv("SVT_PREREDUCE_MIN")) prereduce_min = std::max(1, std::atoi(pv));
    HIP_CHECK(hipGetDevice(&device));
    if (p.stream) {
      stream = static_cast<hipStream_t>(p.stream);
    } else {
      HIP_CHECK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
      own_stream = true;
    }
    prof.on = p.profile != 0;
    prof.stream = stream;
    const int64_t m = ix.m, n = ix.n, nnz = ix.nnz;
    a_is_y = (m >= n);
    arows = std::max(m, n);
    acols = std::min(m, n);
    lanes_r = lanes_for((double)nnz / (double)m);
    lanes_c = lanes_for((double)nnz / (double)n);

    rowptr.alloc(stream, sizeof(int32_t) * (m + 1));
    colidx.alloc(stream, sizeof(int32_t) * nnz);
    colptr.alloc(stream, sizeof(int32_t) * (n + 1));
    rowidx.alloc(stream, sizeof(int32_t) * nnz);
    Mr.alloc(stream, sizeof(T) * nnz);
    Mc.alloc(stream, sizeof(T) * nnz);
    Yr.alloc(stream, sizeof(T) * nnz);
    Yc.alloc(stream, sizeof(T) * nnz);
    pbuf_u.alloc(stream, sizeof(T) * arows);
    pbuf_v.alloc(stream, sizeof(T) * acols);
    HIP_CHECK(hipMemcpyAsync(rowptr.p, ix.rowptr.data(), sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(colidx.p, ix.colidx.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(colptr.p, ix.colptr.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(rowidx.p, ix.rowidx.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, stream));
    // the inverse permutation: the column copy of Y gathers its values from
    // the row copy after each sampled pass
    std::vector<int32_t> inv((size_t)nnz);
    for (int64_t t = 0; t < nnz; ++t) inv[(size_t)ix.csc_of_csr[(size_t)t]] = (int32_t)t;
    csr_of_csc.alloc(stream, sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    HIP_CHECK(hipMemcpyAsync(csr_of_csc.p, inv.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, stream));
    // 16-bit column indices where they fit: the sparse product streams 6
    // instead of 8 bytes per FP32 entry
    std::vector<uint16_t> c16, r16;
    if (n <= 65536) {
      c16.assign(ix.colidx.begin(), ix.colidx.end());
      colidx16.alloc(stream, sizeof(uint16_t) * std::max<int64_t>(nnz, 1));
      HIP_CHECK(hipMemcpyAsync(colidx16.p, c16.data(), sizeof(uint16_t) * nnz, hipMemcpyHostToDevice, stream));
    }
    if (m <= 65536) {
      r16.assign(ix.rowidx.begin(), ix.rowidx.end());
      rowidx16.alloc(stream, sizeof(uint16_t) * std::max<int64_t>(nnz, 1));
      HIP_CHECK(hipMemcpyAsync(rowidx16.p, r16.data(), sizeof(uint16_t) * nnz, hipMemcpyHostToDevice, stream));
    }
    {
      int lds = 0;
      HIP_CHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
      lds_limit = std::min(lds, 160 * 1024);
      plan_r = spmv_plan((int)m, (int)n, (int)sizeof(T), lds_limit, prm.spmv_mode, mrows());
      plan_c = spmv_plan((int)n, (int)m, (int)sizeof(T), lds_limit, prm.spmv_mode, mrows());
      if (plan_r.nseg > 1) {
        const auto sr = segment_starts(ix.rowptr, ix.colidx, (int)m, plan_r);
        seg_r.alloc(stream, sizeof(int32_t) * sr.size());
        HIP_CHECK(hipMemcpyAsync(seg_r.p, sr.data(), sizeof(int32_t) * sr.size(), hipMemcpyHostToDevice, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
      }
      if (plan_c.nseg > 1) {
        const auto sc = segment_starts(ix.colptr, ix.rowidx, (int)n, plan_c);
        seg_c.alloc(stream, sizeof(int32_t) * sc.size());
        HIP_CHECK(hipMemcpyAsync(seg_c.p, sc.data(), sizeof(int32_t) * sc.size(), hipMemcpyHostToDevice, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
      }
    }
    upload_values(ix.vals_csr.data(), Mr.as<T>(), Mc.as<T>());
    HIP_CHECK(hipMemsetAsync(Yr.p, 0, sizeof(T) * nnz, stream));
    HIP_CHECK(hipMemsetAsync(Yc.p, 0, sizeof(T) * nnz, stream));
    if (ds()) {
      Yp.alloc(stream, sizeof(T) * nnz);
      Ym.alloc(stream, sizeof(T) * nnz);
      HIP_CHECK(hipMemsetAsync(Yp.p, 0, sizeof(T) * nnz, stream));
      HIP_CHECK(hipMemsetAsync(Ym.p, 0, sizeof(T) * nnz, stream));
    }

    // residual partials; the Dantzig selector's second sum (of the plain
    // residual) in the upper half
    sample_part.alloc(stream, sizeof(double) * 2 * (kSampleMaxBlocks + 8));
    sample_host.ensure(sizeof(double) * 2 * (kSampleMaxBlocks + 8));
    // the allocation-free pass's scratch address on this device (looked up
    // once per device, with the device current)
    HIP_CHECK(noalloc_scratch(device, &noalloc_part));
    ensure_basis(std::min<int64_t>(acols, 64));
    note_peak(0);
    HIP_CHECK(hipStreamSynchronize(stream));
  }

  // values given in CSR order (double, host) -> row and column copies (T, device)
  void upload_values(const double *csr_vals, T *dr, T *dc) {
    const int64_t nnz = ix.nnz;
    std::vector<T> tr((size_t)nnz), tc((size_t)nnz);
    for (int64_t t = 0; t < nnz; ++t) {
      tr[(size_t)t] = (T)csr_vals[t];
      tc[(size_t)ix.csc_of_csr[(size_t)t]] = (T)csr_vals[t];
    }
    HIP_CHECK(hipMemcpyAsync(dr, tr.data(), sizeof(T) * nnz, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(dc, tc.data(), sizeof(T) * nnz, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
  }

  // Bases with room for `cap` bidiagonalisation steps (grown geometrically).
  // Growth never passes the step cap (lanczos_maxsteps, else min(m, n)):
  // the footprint a server admits a request on assumes that bound.
  void ensure_basis(int cap) {
    cap = std::min(cap, step_cap());
    if (cap <= kcap) return;
    int newcap = std::max(cap, std::min<int>((int)acols, std::max(kcap * 2, 16)));
    newcap = std::min(newcap, step_cap());
    DevMem nU, nV, ncoef, n1, n2, n3, nr;
    nU.alloc(stream, sizeof(T) * (size_t)arows * (size_t)(newcap + 1));
    nV.alloc(stream, sizeof(T) * (size_t)acols * (size_t)(newcap + 2));
    ncoef.alloc(stream, sizeof(double) * 4 * (size_t)(newcap + 4));
    const int cols = newcap + 4;
    const int blocks = std::max(row_plan((int)arows, mrows()).nblk, row_plan((int)acols, mrows()).nblk);
    n1.alloc(stream, sizeof(double) * (size_t)cols * blocks);
    n2.alloc(stream, sizeof(double) * (size_t)cols * blocks);
    n3.alloc(stream, sizeof(double) * (size_t)blocks);
    nr.alloc(stream, sizeof(double) * (size_t)cols);
    // old and new bases are both live until the copies below complete
    note_peak(nU.bytes + nV.bytes + ncoef.bytes + n1.bytes + n2.bytes + n3.bytes + nr.bytes);
    HIP_CHECK(hipMemsetAsync(ncoef.p, 0, ncoef.bytes, stream));
    if (kcap > 0) {
      // the pending vector's partials (its dot products and |.|^2, in any
      // of the three buffers) cross the growth: the next half-step
      // orthogonalises and normalises that vector with them
      HIP_CHECK(hipMemcpyAsync(n1.p, gs1.p, gs1.bytes, hipMemcpyDeviceToDevice, stream));
      HIP_CHECK(hipMemcpyAsync(n2.p, gs2.p, gs2.bytes, hipMemcpyDeviceToDevice, stream));
      HIP_CHECK(hipMemcpyAsync(n3.p, gs3.p, sizeof(double) * (size_t)blocks, hipMemcpyDeviceToDevice, stream));
      HIP_CHECK(hipMemcpyAsync(nU.p, Ub.p, sizeof(T) * (size_t)arows * (size_t)(kcap + 1), hipMemcpyDeviceToDevice, stream));
      HIP_CHECK(hipMemcpyAsync(nV.p, Vb.p, sizeof(T) * (size_t)acols * (size_t)(kcap + 2), hipMemcpyDeviceToDevice, stream));
      HIP_CHECK(hipMemcpyAsync(ncoef.as<double>(), coef.as<double>(), sizeof(double) * (kcap + 4), hipMemcpyDeviceToDevice, stream));
      HIP_CHECK(hipMemcpyAsync(ncoef.as<double>() + (newcap + 4), coef.as<double>() + (kcap + 4),
                               sizeof(double) * (kcap + 4), hipMemcpyDeviceToDevice, stream));
      HIP_CHECK(hipMemcpyAsync(ncoef.as<double>() + 2 * (newcap + 4), coef.as<double>() + 2 * (kcap + 4),
                               sizeof(double) * 2 * (kcap + 4), hipMemcpyDeviceToDevice, stream));
    }
    HIP_CHECK(hipStreamSynchronize(stream));
    std::swap(Ub.p, nU.p); std::swap(Ub.bytes, nU.bytes);
    std::swap(Vb.p, nV.p); std::swap(Vb.bytes, nV.bytes);
    std::swap(coef.p, ncoef.p); std::swap(coef.bytes, ncoef.bytes);
    std::swap(gs1.p, n1.p); std::swap(gs1.bytes, n1.bytes);
    std::swap(gs2.p, n2.p); std::swap(gs2.bytes, n2.bytes);
    std::swap(gs3.p, n3.p); std::swap(gs3.bytes, n3.bytes);
    std::swap(gsr.p, nr.p); std::swap(gsr.bytes, nr.bytes);
    kcap = newcap;
    note_peak(0);
    gs.part1 = gs1.as<double>();
    gs.part2 = gs2.as<double>();
    gs.part3 = gs3.as<double>();
    gs.red = gsr.as<double>();
    gs.max_cols = cols;
    gs.max_blocks = blocks;
  }

  double *alpha_d() { return coef.as<double>(); }                 // alpha_{i+1} at [i]
  double *beta_d() { return coef.as<double>() + (kcap + 4); }     // beta_{i+1} at [i]
  // fraction of |p|^2 removed by the one-pass reorthogonalisation of
  // half-step j (j = 0, 1 in gkl_start, 2k and 2k + 1 in step k)
  double *removed_d() { return coef.as<double>() + 2 * (kcap + 4); }
  T *ucol(int i) { return Ub.as<T>() + (size_t)i * (size_t)arows; }
  T *vcol(int i) { return Vb.as<T>() + (size_t)i * (size_t)acols; }

  // Room for rank-r factors (row stride even, zero padded) and the k x r
  // combination matrices.
  void ensure_factors(int r, int k) {
    if (r > fcap) {
      // doubling, but never past the largest rank the step cap allows
      const int cap = std::max(r, std::min(fcap * 2, step_cap()));
      // rows of 16 bytes' multiples (the sampled update reads them 16 bytes at a time)
      constexpr int al = 16 / (int)sizeof(T);
      fstride = std::max(al, (cap + al - 1) / al * al);
      fcap = cap;
      Fu.alloc(stream, sizeof(T) * (size_t)ix.m * fstride);
      Fv.alloc(stream, sizeof(T) * (size_t)ix.n * fstride);
    }
    const size_t need = sizeof(double) * (2 * (size_t)std::max(k, 1) * (size_t)std::max(r, 1) + (size_t)r);
    if (ritzd.bytes < need) ritzd.alloc(stream, need * 2);
    ritz_host.ensure(need * 2);
    note_peak(0);
  }

  // Device bytes held now (every buffer of the handle) and the most held at
  // once, including the moments when a growing buffer's old and new copies
  // are both live.
  std::vector<DevMem *> all_mem() {
    return {&rowptr, &colidx, &colptr, &rowidx, &csr_of_csc, &seg_r, &seg_c, &colidx16, &rowidx16,
            &Mr, &Mc, &Yr, &Yc, &Yp, &Ym, &g_ptr, &g_idx, &g_val, &gt_ptr,
            &gt_idx, &gt_val, &b_d, &y_d, &xs_d, &Ub, &Vb, &pbuf_u, &pbuf_v, &coef, &gs1, &gs2, &gs3, &gsr,
            &sample_part, &ritzd, &Fu, &Fv, &rs_a, &rs_b};
  }
  size_t device_bytes() const {
    size_t b = 0;
    for (const DevMem *d : const_cast<Problem *>(this)->all_mem()) b += d->bytes;
    return b;
  }
  void note_peak(size_t extra) { peak_bytes = std::max(peak_bytes, device_bytes() + extra); }
  void mem_stats(size_t *cur, size_t *peak) const override {
    if (cur) *cur = device_bytes();
    if (peak) *peak = peak_bytes;
  }

  // --------------------------------------------------------- sparse products
  // orientation helpers: A's row-compressed and column-compressed structures
  struct Csx {
    const int32_t *ptr, *idx;
    const uint16_t *idx16;     // 16-bit copy of idx (null when ncols > 65536)
    int nrows, ncols;
    SpmvPlan *plan;            // row partition, lanes, LDS segments of x (0: gather)
    const int32_t *segptr;
  };
  Csx csr_struct() {
    return {rowptr.as<int32_t>(), colidx.as<int32_t>(), colidx16.as<uint16_t>(), (int)ix.m, (int)ix.n, &plan_r,
            seg_r.as<int32_t>()};
  }
  Csx csc_struct() {
    return {colptr.as<int32_t>(), rowidx.as<int32_t>(), rowidx16.as<uint16_t>(), (int)ix.n, (int)ix.m, &plan_c,
            seg_c.as<int32_t>()};
  }
  int spmv_segments(int which) const override { return (which == 0 ? plan_r : plan_c).nseg; }
  // rows per row block of the vector partition: at least this many
  int mrows() const { return prm.min_block_rows > 0 ? (int)prm.min_block_rows : kDefaultMinRows; }
  Csx a_rows_struct() { return a_is_y ? csr_struct() : csc_struct(); }
  Csx a_cols_struct() { return a_is_y ? csc_struct() : csr_struct(); }

  // out = A x' - s prev, x' the input `in` (launch_spmv); with dots, the
  // partial dot products of out with the nq columns of Q and |out|^2 follow
  // in the same kernel.
  void spmv(const Csx &c, const T *vals, const SpmvInput<T> &in, const T *prev, T *out, const T *Q = nullptr,
            int64_t ldq = 0, int nq = 0, double *dots = nullptr, int ndots = -1) {
    if (ndots < 0) ndots = nq;
    hipError_t e = launch_spmv<T>(stream, *c.plan, c.ptr, c.idx, c.idx16, vals, c.segptr, in, c.ncols, prev,
                                  out, c.nrows, Q, ldq, nq, ndots, dots);
    if (e == hipErrorInvalidValue && c.plan->nseg > 0) {
      // the device refused the LDS size: gather x from memory from now on
      (void)hipGetLastError();
      *c.plan = spmv_plan(c.nrows, c.ncols, (int)sizeof(T), lds_limit, 1, mrows());
      e = launch_spmv<T>(stream, *c.plan, c.ptr, c.idx, c.idx16, vals, nullptr, in, c.ncols, prev, out, c.nrows,
                         Q, ldq, nq, ndots, dots);
    }
    HIP_CHECK(e);
  }

  // Segment starts of every row of a compressed structure for the LDS plan.
  static std::vector<int32_t> segment_starts(const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                                             int nrows, const SpmvPlan &pl) {
    std::vector<int32_t> out((size_t)nrows * (pl.nseg + 1));
    for (int i = 0; i < nrows; ++i) {
      const int32_t *b = idx.data() + ptr[i], *e = idx.data() + ptr[i + 1];
      for (int sg = 0; sg <= pl.nseg; ++sg) {
        const int32_t bound = (int32_t)std::min<int64_t>((int64_t)sg * pl.segcols, INT32_MAX);
        out[(size_t)i * (pl.nseg + 1) + sg] =
            sg == pl.nseg ? ptr[i + 1] : (int32_t)(std::lower_bound(b, e, bound) - idx.data());
      }
    }
    return out;
  }

  // Algorithmic bytes: index (2 or 4 bytes, as stored) and value of every
  // stored entry, the gathered vector once, the previous vector and the
  // result.
  double spmv_bytes(const Csx &c, int ncols_x, bool has_prev) const {
    const double vb = sizeof(T);
    const double ib = c.idx16 ? 2.0 : 4.0;
    return (double)ix.nnz * (vb + ib) + 4.0 * (c.nrows + 1) + vb * ncols_x + vb * c.nrows +
           (has_prev ? vb * c.nrows : 0.0);
  }

  // A new vector of the bidiagonalisation whose orthogonalisation is still
  // pending: its partials are in part buffer `buf` (1, 2, 3: gs.part1 ..
  // part3), nq dot products with its side's basis, then |.|^2.  nq = 0: only
  // the norm is pending (the vector is already orthogonal).
  struct PendingVec {
    int buf = 3;
    int nq = 0;
  };
  double *part_buf(int b) { return b == 1 ? gs.part1 : (b == 2 ? gs.part2 : gs.part3); }

  // Whether the one-pass update of a pending vector with nqx basis columns is
  // fused into the next sparse product (p's side then has nqx + side
  // columns); wider updates run as their own kernel first.
  static bool fused_update(int nqx, int side) { return nqx > 0 && nqx + side <= kSpmvAuxCols; }

  // One half-step of the bidiagonalisation: p = A x' - s prev (side 0) or
  // A^T x' - s prev (side 1), where x' = (x_raw - Q_x h) / s is the other
  // side's pending vector xp orthogonalised against its nqx basis columns
  // Q_x and normalised; x' goes to x_col, s to *x_coef and |h|^2 / |x_raw|^2
  // to *x_removed.  p is left in place with its own update pending against
  // the nq columns of Q (returned).  Two passes (passes_now == 2): every
  // vector is orthogonalised in its own half-step (the pending part is only
  // its norm, in gs.part3).
  PendingVec half_step(const Csx &c, const T *vals, T *x_raw, PendingVec xp, const T *Qx, int64_t ldqx, T *x_col,
                       double *x_coef, double *x_removed, const T *prev, T *Q, int64_t ldq, int nq, bool orth,
                       T *p, int side) {
    const double vb = sizeof(T);
    const double len = (double)c.nrows;
    const int xnp = xnp_of(c.ncols);
    SpmvInput<T> in;
    in.x = x_raw;
    in.np = xnp;
    in.x_out = x_col;
    in.s_out = x_coef;
    if (passes_now == 1) {
      if (xp.nq > 0 && !fused_update(xp.nq, side)) {
        // too wide to fuse: x's update runs first, in place
        prof.begin();
        HIP_CHECK(launch_gs_update<T>(stream, x_raw, c.ncols, Qx, ldqx, xp.nq, part_buf(xp.buf), gs.part3, true,
                                      x_removed, mrows()));
        prof.end(kGsUpdate2, vb * c.ncols * (xp.nq + 2.0));
        xp = PendingVec{3, 0};
      }
      in.pend = part_buf(xp.buf);
      if (xp.nq >= prereduce_min) {
        // a wide basis: the partials are summed once, here, instead of by
        // every workgroup of the product (the same sums, bit for bit)
        prof.begin();
        HIP_CHECK(launch_pending_reduce(stream, in.pend, xnp, xp.nq, gs.red));
        prof.end(kPendReduce, 8.0 * (xp.nq + 1.0) * (xnp + 1.0));
        in.pend = gs.red;
        in.np = 1;
      }
      in.Qx = Qx;
      in.ldqx = ldqx;
      in.nqx = xp.nq;
      in.removed_out = xp.nq > 0 ? x_removed : nullptr;
      in.alpha = alpha_d();
      in.beta = beta_d();
      in.side = side;
      const int out_buf = side == 0 ? 1 : 2;
      // p's dot products with its basis when it is to be orthogonalised; the
      // update of x (nqx > 0) needs the basis of p's side either way
      const int ndots = orth ? nq : 0;
      const int nq_k = xp.nq > 0 ? nq : ndots;
      // algorithmic bytes: the product's (spmv_bytes), x' written to its
      // basis column, Q_x read once for it, and Q read once for the image
      // of the update and the dot products
      prof.begin();
      spmv(c, vals, in, prev, p, Q, ldq, nq_k, part_buf(out_buf), ndots);
      prof.end(kSpmv, spmv_bytes(c, c.ncols, prev != nullptr) + vb * c.ncols * (1.0 + xp.nq) + vb * len * nq_k);
      return PendingVec{out_buf, ndots};
    }
    in.pend = part_buf(xp.buf);  // x already orthogonal: only its norm
    prof.begin();
    spmv(c, vals, in, prev, p, Q, ldq, nq, nq > 0 ? gs.part1 : nullptr);
    prof.end(kSpmv, spmv_bytes(c, c.ncols, prev != nullptr) + vb * c.ncols + vb * len * nq);
    if (nq == 0) {
      HIP_CHECK(launch_sumsq<T>(stream, p, c.nrows, gs.part3, mrows()));
      return PendingVec{3, 0};
    }
    // each update: Q read once, p read and written (the fused dot products
    // and norms reuse the same rows)
    prof.begin();
    HIP_CHECK(launch_gs_update<T>(stream, p, c.nrows, Q, ldq, nq, gs.part1, gs.part2, false, nullptr, mrows()));
    prof.end(kGsUpdate1, vb * len * (nq + 2.0));
    prof.begin();
    HIP_CHECK(launch_gs_update<T>(stream, p, c.nrows, Q, ldq, nq, gs.part2, gs.part3, true, nullptr, mrows()));
    prof.end(kGsUpdate2, vb * len * (nq + 2.0));
    return PendingVec{3, 0};
  }

  // ------------------------------------------------- bidiagonalisation (a3)
  struct Gkl {
    int k = 0;                // completed steps: u_1..u_k, v_1..v_k, raw v_{k+1}
    bool finalized = false;   // beta_{k+1} stored
    std::vector<double> alpha, beta;  // host copies, alpha[i] = alpha_{i+1}, beta[i] = beta_{i+1}
    std::vector<double> removed;      // removed fraction of each one-pass half-step's vector
    PendingVec pu, pv;        // the raw vectors in pbuf_u and pbuf_v
  };

  int xnp_of(int nrows) const { return row_plan(nrows, mrows()).nblk; }

  // Start: v_1 random unit, u_1 = A v_1 / alpha_1, then v_2, beta_2.  The
  // removed fraction of the vector made by half-step j goes to slot j (it is
  // computed where that vector is orthogonalised: in half-step j + 1).
  void gkl_start(const T *vr, const T *vc, Gkl &g) {
    ensure_basis(std::min<int64_t>(acols, 8));
    const Csx R = a_rows_struct(), C = a_cols_struct();
    partial_run = partial_now && passes_now == 1 && !full_this_run;
    if (partial_run)
      rsched.start(orth_eta(), kUnit, orth_root(), growth_carry, hold_hint,
                   replay_hint.empty() ? nullptr : &replay_hint, std::sqrt(kUnit));
    HIP_CHECK(launch_randn<T>(stream, pbuf_v.as<T>(), (int)acols, prm.seed, rng_ctr++));
    HIP_CHECK(launch_sumsq<T>(stream, pbuf_v.as<T>(), (int)acols, gs.part3, mrows()));
    g.pv = PendingVec{3, 0};
    // u_1 = A v_1 / alpha_1 (v_1 = the normalised start vector)
    g.pu = half_step(R, vr, pbuf_v.as<T>(), g.pv, Vb.as<T>(), acols, vcol(0), beta_d(), nullptr, nullptr,
                     Ub.as<T>(), arows, 0, orth_vec(0, 0), pbuf_u.as<T>(), 0);
    // v_2 = A^T u_1 - alpha_1 v_1, orthogonal to v_1
    g.pv = half_step(C, vc, pbuf_u.as<T>(), g.pu, Ub.as<T>(), arows, ucol(0), alpha_d(), removed_d(), vcol(0),
                     Vb.as<T>(), acols, 1, orth_vec(1, 1), pbuf_v.as<T>(), 1);
    g.k = 1;
    g.finalized = false;
    steps_total += 1;
  }

  // One more step: u_{k+1}, alpha_{k+1}, v_{k+2} (pending).
  void gkl_step(const T *vr, const T *vc, Gkl &g) {
    const int k = g.k;
    ensure_basis(k + 1);
    const Csx R = a_rows_struct(), C = a_cols_struct();
    // u_{k+1} = A v_{k+1} - beta_{k+1} u_k, orthogonal to u_1..u_k
    g.pu = half_step(R, vr, pbuf_v.as<T>(), g.pv, Vb.as<T>(), acols, vcol(k), beta_d() + k, removed_d() + 2 * k - 1,
                     ucol(k - 1), Ub.as<T>(), arows, k, orth_vec(2 * k, k), pbuf_u.as<T>(), 0);
    // v_{k+2} = A^T u_{k+1} - alpha_{k+1} v_{k+1}, orthogonal to v_1..v_{k+1}
    g.pv = half_step(C, vc, pbuf_u.as<T>(), g.pu, Ub.as<T>(), arows, ucol(k), alpha_d() + k, removed_d() + 2 * k,
                     vcol(k), Vb.as<T>(), acols, k + 1, orth_vec(2 * k + 1, k + 1), pbuf_v.as<T>(), 1);
    g.k = k + 1;
    g.finalized = false;
    steps_total += 1;
  }

  // Start the fetch of B_k: store beta_{k+1} = |v_{k+1}| (and the removed
  // fraction of v_{k+1}'s update; the next step redoes both, bit for bit),
  // then copy alpha, beta and the removed fractions (one allocation, one
  // copy) to pinned memory and record fetch_ev behind it.
  void gkl_fetch_begin(Gkl &g) {
    const int k = g.k;
    if (!g.finalized) {
      const int xnp = xnp_of((int)acols);
      if (passes_now == 1 && fused_update(g.pv.nq, 0)) {
        HIP_CHECK(launch_pending_norm(stream, part_buf(g.pv.buf), xnp, g.pv.nq, beta_d() + k,
                                      removed_d() + 2 * k - 1));
      } else {
        if (g.pv.nq > 0) {
          // an update too wide to fuse runs here, as the next step would
          HIP_CHECK(launch_gs_update<T>(stream, pbuf_v.as<T>(), (int)acols, Vb.as<T>(), acols, g.pv.nq,
                                        part_buf(g.pv.buf), gs.part3, true, removed_d() + 2 * k - 1, mrows()));
          g.pv = PendingVec{3, 0};
        }
        HIP_CHECK(launch_finalize<T>(stream, pbuf_v.as<T>(), (int)acols, part_buf(g.pv.buf), vcol(k),
                                     beta_d() + k, mrows()));
      }
      g.finalized = true;
    }
    // alpha, beta and the removed fractions of half-steps 0 .. 2k - 1
    const size_t span = 2 * (size_t)(kcap + 4) + 2 * (size_t)k;
    coef_host.ensure(sizeof(double) * span);
    HIP_CHECK(hipMemcpyAsync(coef_host.p, alpha_d(), sizeof(double) * span, hipMemcpyDeviceToHost, stream));
    if (!fetch_ev) HIP_CHECK(hipEventCreateWithFlags(&fetch_ev, hipEventDisableTiming));
    HIP_CHECK(hipEventRecord(fetch_ev, stream));
    fetch_k = k;
    fetch_kcap = kcap;
  }

  // Wait for the copy and fill snap with B_k of the fetch (later steps may
  // already be queued or running).
  void gkl_fetch_end(Gkl &snap) {
    HIP_CHECK(hipEventSynchronize(fetch_ev));
    const int k = fetch_k;
    const double *h = coef_host.as<double>();
    snap.k = k;
    snap.finalized = true;
    snap.alpha.assign(h, h + k);
    snap.beta.assign(h + (fetch_kcap + 4), h + (fetch_kcap + 4) + (k + 1));
    snap.removed.assign(h + 2 * (fetch_kcap + 4), h + 2 * (fetch_kcap + 4) + 2 * k);
  }

  // B_k as diagonal d and superdiagonal e.
  static void bidiag_of(const Gkl &g, std::vector<double> &d, std::vector<double> &e) {
    const int k = g.k;
    d.assign(g.alpha.begin(), g.alpha.begin() + k);
    e.assign(k > 1 ? k - 1 : 0, 0.0);
    for (int i = 0; i + 1 < k; ++i) e[i] = g.beta[i + 1];
  }

  // Singular values of B_k (with the rotation log for gkl_vectors) and the
  // residual bounds res_i = beta_{k+1} |P_{k,i}|.
  void gkl_ritz(const Gkl &g, BidiagSVD &out, std::vector<double> &res) {
    const int k = g.k;
    std::vector<double> d, e;
    bidiag_of(g, d, e);
    if (log_level > 1) {
      std::fprintf(stderr, "[svt] coefficients k %d:", k);
      for (int i = 0; i < k; ++i) std::fprintf(stderr, " a%d %.3e b%d %.3e", i + 1, g.alpha[i], i + 2, g.beta[i + 1]);
      std::fprintf(stderr, "\n");
    }
    for (int i = 0; i <= k; ++i)
      if ((i < k && !std::isfinite(g.alpha[i])) || !std::isfinite(g.beta[i]))
        throw Error(SVT_EDIVERGED, "non-finite bidiagonalisation coefficient at step " + std::to_string(i + 1) +
                                       " of " + std::to_string(k));
    if (!bidiag_svd(d, e, out))
      throw Error(SVT_ELANCZOS, "bidiagonal SVD did not converge (k = " + std::to_string(k) + ")");
    const double bk1 = (k >= acols) ? 0.0 : std::fabs(g.beta[k]);
    res.resize(k);
    for (int i = 0; i < k; ++i) res[i] = bk1 * std::fabs(out.p_last[i]);
  }

  int step_cap() const {
    int cap = (int)acols;
    if (prm.lanczos_maxsteps > 0) cap = std::min(cap, (int)prm.lanczos_maxsteps);
    return cap;
  }

  // Run the bidiagonalisation until the decision of Algorithm 1's inner loop
  // is certain.  mode 0 (SVT step): every Ritz value above tau converged and
  // the first one at or below tau is either converged or certainly below tau
  // (value + residual <= tau).  mode 1 (fixed count): the `count` largest
  // triplets converged.  Returns k and fills the final SVD with vectors.
  int gkl_run(const T *vr, const T *vc, int mode, int count, double tau, Gkl &g, BidiagSVD &sv,
              int &r_out) {
    const double tol = prm.lanczos_tol;
    const int cap = step_cap();
    full_this_run = false;
    gkl_start(vr, vc, g);
    // the first check: where the previous iteration stopped, less 2 on
    // small bases (a check there costs about two steps, so probing below is
    // cheap); on wide bases a check costs tens of steps (its host SVD grows
    // as k^2), so it is placed at the previous count itself
    const int probe = k_hint >= kProbeMaxK ? 0 : 2;
    int first_check = std::max(std::min(cap, mode == 1 ? count + 2 : 3), std::min(cap, k_hint - probe));
    first_check = std::max(first_check, 1);
    int next_check = first_check;
    std::vector<double> res;
    Gkl snap;
    for (;;) {
      while (g.k < next_check && g.k < cap) gkl_step(vr, vc, g);
      // the check of B_k runs on the host while the device already takes
      // the next steps: if the check decides they are discarded (they write
      // only basis columns and coefficients beyond k), otherwise they are
      // the continuation; the decisions are those of checking without them
      gkl_fetch_begin(g);
      for (int a = 0; a < kAheadSteps && g.k < cap; ++a) gkl_step(vr, vc, g);
      gkl_fetch_end(snap);
      if (partial_run && !rsched.advance(snap.alpha.data(), snap.beta.data(), snap.k)) {
        // a vector left alone lost more orthogonality than semi-orthogonality
        // allows (the prediction fell short of the estimate): this
        // bidiagonalisation starts again with every vector orthogonalised,
        // and the next one takes no hold and no replayed pattern
        full_this_run = true;
        hold_hint = 0;
        replay_hint.clear();
        ++partial_fallbacks;
        if (log_level > 0)
          std::fprintf(stderr, "[svt] partial reorthogonalisation: an estimate passed %.2e by step %d "
                               "(growth %.2f): restarting with full reorthogonalisation\n",
                       rsched.verify(), snap.k, rsched.growth());
        gkl_start(vr, vc, g);
        next_check = first_check;
        continue;
      }
      if (prm.reorth_passes == 0 && passes_now == 1) {
        // one pass per vector is enough while no pass removes a large part
        // of its vector (the vector then already was nearly orthogonal, as
        // the recurrence makes it in exact arithmetic); a pass that removed
        // more than reorth_trigger of |p|^2 (DGKS: 1/2) left the basis less
        // orthogonal than two passes would: start this bidiagonalisation
        // again with two passes, and keep them for the rest of the solve
        double worst = 0.0;
        bool bad = false;
        for (int j = 1; j < 2 * snap.k; ++j) {
          if (partial_run && !rsched.reorthogonalised(j)) continue;  // no pass made: no fraction
          const double f = snap.removed[(size_t)j];
          if (!(f <= reorth_trigger)) bad = true;  // also a non-finite value
          if (f > worst) worst = f;
        }
        if (bad) {
          passes_now = 2;
          ++reorth_restarts;
          if (log_level > 0)
            std::fprintf(stderr, "[svt] one-pass reorthogonalisation removed %.3e of a vector by step %d: "
                                 "restarting with two passes\n", worst, snap.k);
          gkl_start(vr, vc, g);
          next_check = first_check;
          continue;
        }
      }
      BidiagSVD chk;
      gkl_ritz(snap, chk, res);
      const int k = snap.k;
      if (mode == 0 && dof_rmax >= 0) {
        // Ritz values bound the singular values from below: more of them
        // above tau than the degrees-of-freedom bound allows settles it
        int above = 0;
        while (above < k && chk.sigma[above] > tau) ++above;
        if (above > dof_rmax) {
          dof_hit = true;
          r_out = above;
          return k;
        }
      }
      const double top = chk.sigma.empty() ? 0.0 : chk.sigma[0];
      const double atol = tol * std::max(top, 1e-300);
      bool done = false;
      int r = 0;
      if (k >= acols) {
        done = true;  // the bases span the whole smaller dimension: exact
        if (mode == 0)
          while (r < k && chk.sigma[r] > tau) ++r;
      } else if (mode == 0) {
        while (r < k && chk.sigma[r] > tau) ++r;
        bool ok = true;
        for (int i = 0; i < r && ok; ++i) ok = res[i] <= atol;
        // The first value at or below tau decides r.  It must be converged,
        // or else its whole residual interval must lie well below tau, and
        // only once at least one Ritz value above tau has converged.  A
        // residual interval certifies a singular value near the Ritz value,
        // not which one: before the Krylov space has found the leading
        // singular values (few steps), or while a Ritz value still sits
        // between two close singular values, the bound alone would miss a
        // singular value above tau (Ritz values approach from below).
        if (ok && r < k)
          ok = (res[r] <= atol) ||
               (r >= 1 && chk.sigma[r] + res[r] <= tau * (1.0 - prm.decide_margin));
        if (ok && r == k) ok = false;  // no value below tau seen yet: extend (s_k += ell)
        done = ok;
      } else {
        const int c = std::min(count, k);
        bool ok = (k >= count);
        for (int i = 0; i < c && ok; ++i) ok = res[i] <= atol;
        done = ok;
      }
      if (done) {
        r_out = r;
        if (log_level > 0) {
          std::fprintf(stderr, "[svt] gkl mode %d k %d r %d top %.6e", mode, k, r, top);
          for (int i = std::max(0, r - 1); i < std::min(k, r + 2); ++i)
            std::fprintf(stderr, " | s%d %.10e res %.2e", i + 1, chk.sigma[i], res[i]);
          std::fprintf(stderr, " | tau %.10e\n", tau);
        }
        // the singular vectors that are used, from this check's rotations
        std::vector<double> d, e;
        bidiag_of(snap, d, e);
        bidiag_vectors(d, e, mode == 1 ? std::min(count, k) : r, chk);
        sv = std::move(chk);
        // the next bidiagonalisation starts from this one's growth (half of
        // the carried value decays away when a run measures less)
        if (partial_run) {
          growth_carry = std::max(rsched.growth_seen(), 0.5 * growth_carry);
          // an SVT step's bidiagonalisation: where the next one may start
          // orthogonalising (the exact policy replayed on these coefficients).
          // FP64 vectors only: for FP32 vectors it gained nothing measurable
          // and moved a small general-operator run past the mixed form's bar
          if (mode == 0 && sizeof(T) == 8)
            hold_hint = std::max(0, first_trigger(snap.alpha.data(), snap.beta.data(), k, orth_eta(), kUnit,
                                                  orth_root()) - kHoldMargin);
          if (mode == 0) {
            // and, after a long one, the whole pattern, which the next one
            // follows slightly ahead, its predictions then guarding only
            // semi-orthogonality (on short bidiagonalisations consecutive
            // SVT steps differ too much: such a schedule fell back to full)
            if (k >= kReplayMinSteps)
              replay_hint = exact_pattern(snap.alpha.data(), snap.beta.data(), k, orth_eta(), kUnit, orth_root());
            else
              replay_hint.clear();
          }
        }
        // the factors are formed from the first k columns of the bases
        g.k = k;
        g.alpha = snap.alpha;
        g.beta = snap.beta;
        return k;
      }
      if (k >= cap) {
        throw Error(SVT_ELANCZOS, "bidiagonalisation reached its step cap (" + std::to_string(cap) +
                                      ") before the Ritz triplets converged");
      }
      next_check = std::min(cap, std::max(g.k, k + std::max(2, std::min(8, k / 16))));
    }
  }

  // ------------------------------------------- randomised partial SVD
  // p = Y x (trans 0, rows m) or Y^T x (trans 1, rows n), x and p on the
  // device: the sparse product with nothing pending and no previous vector.
  void plain_product(int trans, const T *x, T *out) {
    SpmvInput<T> in;
    in.x = x;
    const Csx c = trans == 0 ? csr_struct() : csc_struct();
    spmv(c, trans == 0 ? Yr.as<T>() : Yc.as<T>(), in, nullptr, out);
  }

  // out (rows x l, device) = Y or Y^T times the l columns of x (device).
  void block_product(int trans, const T *x, int l, T *out) {
    const int64_t xr = trans == 0 ? ix.n : ix.m, orows = trans == 0 ? ix.m : ix.n;
    for (int j = 0; j < l; ++j) plain_product(trans, x + (size_t)j * xr, out + (size_t)j * orows);
  }

  void to_host(const DevMem &d, int64_t count, std::vector<double> &h) {
    std::vector<T> t((size_t)count);
    HIP_CHECK(hipMemcpyAsync(t.data(), d.p, sizeof(T) * count, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    h.assign(t.begin(), t.end());
  }
  void to_device(const std::vector<double> &h, DevMem &d) {
    std::vector<T> t(h.begin(), h.end());
    HIP_CHECK(hipMemcpyAsync(d.p, t.data(), sizeof(T) * t.size(), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
  }

  // The s largest singular triplets of Y, approximated by the randomised
  // range finder with power iterations (Section 6 proposes randomised
  // low-rank SVDs for D_tau; the method is that of Halko, Martinsson and
  // Tropp, 2011): l = min(m, n, s + oversample) Gaussian columns Omega
  // (the counter-based generator of the start vectors, one counter per
  // matrix drawn in a solve), Q = orth(Y Omega), then `power` times
  // P = orth(Y^T Q), Q = orth(Y P); W = Y^T Q = Vw S Uw^T; U = Q Uw, V = Vw.
  // The sparse products run on the device, one vector at a time; the
  // orthonormalisations and the small SVD on the host.  Returns the number
  // of sparse products.
  int randomized_triplets(int s, std::vector<double> &sigma, std::vector<double> &U, std::vector<double> &V) {
    const int64_t m = ix.m, n = ix.n;
    const int64_t cap = std::min(m, n);
    const int l = (int)std::min<int64_t>(cap, (int64_t)s + prm.rsvd_oversample);
    const int64_t big = std::max(m, n);
    if (big * (int64_t)l > INT32_MAX)
      throw Error(SVT_EINVAL, "randomised partial SVD: max(m, n) x (s_k + oversample) exceeds 2^31 entries");
    if (rs_a.bytes < sizeof(T) * (size_t)big * l) {
      rs_a.alloc(stream, sizeof(T) * (size_t)big * l);
      rs_b.alloc(stream, sizeof(T) * (size_t)big * l);
      note_peak(0);
    }
    T *a = rs_a.as<T>(), *b = rs_b.as<T>();
    int products = 0;
    HIP_CHECK(launch_randn<T>(stream, a, (int)(n * l), prm.seed, rs_ctr++));   // Omega, n x l
    block_product(0, a, l, b);                                                 // Y Omega, m x l
    products += l;
    std::vector<double> Q, P, W;
    to_host(rs_b, m * l, Q);
    orth_columns(Q.data(), m, l);
    for (int it = 0; it < prm.rsvd_power; ++it) {
      to_device(Q, rs_a);
      block_product(1, a, l, b);      // Y^T Q, n x l
      to_host(rs_b, n * l, P);
      orth_columns(P.data(), n, l);
      to_device(P, rs_a);
      block_product(0, a, l, b);      // Y P, m x l
      to_host(rs_b, m * l, Q);
      orth_columns(Q.data(), m, l);
      products += 2 * l;
    }
    to_device(Q, rs_a);
    block_product(1, a, l, b);        // W = Y^T Q, n x l
    products += l;
    to_host(rs_b, n * l, W);
    std::vector<double> Vw, Uw;
    if (!jacobi_svd_tall(W.data(), n, l, sigma, Vw, Uw))
      throw Error(SVT_ELANCZOS, "randomised partial SVD: the small SVD did not settle");
    U.assign((size_t)m * l, 0.0);     // Q Uw
    for (int c = 0; c < l; ++c)
      for (int j = 0; j < l; ++j) {
        const double f = Uw[(size_t)c * l + j];
        const double *qj = Q.data() + (size_t)j * m;
        double *uc = U.data() + (size_t)c * m;
        for (int64_t i = 0; i < m; ++i) uc[i] += qj[i] * f;
      }
    V.swap(Vw);
    return products;
  }

  // One SVT iteration's D_tau by the randomised triplets, with Algorithm 1's
  // repeat loop over s_k (Section 5.1.1) and the factors of X^k into Fu, Fv.
  void randomized_iteration(int r_prev, int &r, int &s, int &steps, std::vector<double> &ws) {
    const int64_t m = ix.m, n = ix.n;
    const int cap = (int)std::min(m, n);
    const int scap = step_cap();   // lanczos_maxsteps, when given, bounds s_k here too
    s = std::min(r_prev + 1, cap);
    std::vector<double> sigma, U, V;
    int products = 0;
    for (;;) {
      products += randomized_triplets(s, sigma, U, V);
      if (sigma[(size_t)s - 1] <= prm.tau || s >= cap) break;
      if (s >= scap)
        throw Error(SVT_ELANCZOS, "randomised partial SVD: s_k reached the step cap (" + std::to_string(scap) +
                                      ") with its last value above tau");
      s = std::min(s + (int)prm.incr, cap);
    }
    r = 0;
    while (r < s && sigma[(size_t)r] > prm.tau) ++r;
    steps = (products + 1) / 2;
    steps_total += steps;
    ws.assign(std::max(r, 1), 0.0);
    for (int i = 0; i < r; ++i) ws[(size_t)i] = sigma[(size_t)i] - prm.tau;
    ensure_factors(std::max(r, 1), 1);
    rank = r;
    if (r == 0) return;
    std::vector<T> fu((size_t)m * fstride, (T)0), fv((size_t)n * fstride, (T)0);
    for (int c = 0; c < r; ++c) {
      for (int64_t i = 0; i < m; ++i) fu[(size_t)i * fstride + c] = (T)(U[(size_t)c * m + i] * ws[(size_t)c]);
      for (int64_t j = 0; j < n; ++j) fv[(size_t)j * fstride + c] = (T)V[(size_t)c * n + j];
    }
    HIP_CHECK(hipMemcpyAsync(Fu.p, fu.data(), sizeof(T) * fu.size(), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(Fv.p, fv.data(), sizeof(T) * fv.size(), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
  }

  // Ritz vectors for the first r triplets; ws scales the left factor of Y.
  void form_factors(const Gkl &g, const BidiagSVD &sv, int r, const double *ws) {
    const int k = g.k;
    ensure_factors(std::max(r, 1), k);
    if (r == 0) { rank = 0; return; }
    // P (u side) and Q (v side) restricted to the first r columns, k x r
    // row-major, then w: packed into one pinned block and one copy (the
    // previous iteration's copy has completed: its residual was synchronised)
    const size_t kr = (size_t)k * r;
    double *Ph = ritz_host.as<double>(), *Qh = Ph + kr, *wh = Qh + kr;
    for (int c = 0; c < k; ++c)
      for (int l = 0; l < r; ++l) {
        Ph[(size_t)c * r + l] = sv.P[(size_t)l * k + c];
        Qh[(size_t)c * r + l] = sv.Q[(size_t)l * k + c];
      }
    for (int l = 0; l < r; ++l) wh[l] = ws[l];
    HIP_CHECK(hipMemcpyAsync(ritzd.p, Ph, sizeof(double) * (2 * kr + r), hipMemcpyHostToDevice, stream));
    const double *Pd = ritzd.as<double>(), *Qd = Pd + kr, *wd = Qd + kr;
    // Y's left factor (rows m) takes the weights
    T *u_out = a_is_y ? Fu.as<T>() : Fv.as<T>();   // A-rows side
    T *v_out = a_is_y ? Fv.as<T>() : Fu.as<T>();   // A-cols side
    const double *wu = a_is_y ? wd : nullptr;
    const double *wv = a_is_y ? nullptr : wd;
    // algorithmic bytes: the basis read once, the factor written
    prof.begin();
    HIP_CHECK(launch_ritz<T>(stream, Ub.as<T>(), arows, (int)arows, k, Pd, wu, r, u_out, fstride));
    prof.end(kRitz, (double)sizeof(T) * (double)arows * (k + fstride));
    prof.begin();
    HIP_CHECK(launch_ritz<T>(stream, Vb.as<T>(), acols, (int)acols, k, Qd, wv, r, v_out, fstride));
    prof.end(kRitz, (double)sizeof(T) * (double)acols * (k + fstride));
    rank = r;
  }

  // Sampled product + residual + update of Y in one pass over the
  // row-compressed order, then the column copy gathered from it through
  // csr_of_csc; returns residual^2 (workgroup partials added on the host in
  // order, compensated).
  // Dantzig selector: the violation^2 is returned and ||P_Omega(X - B)||^2
  // goes to *plain2 (when not null).
  double sample_pass(int r, double delta, bool want_res, double *plain2 = nullptr) {
    double *part2 = (want_res && ds()) ? sample_part.as<double>() + kSampleMaxBlocks + 8 : nullptr;
    return sample_pass_on(Fu.as<T>(), Fv.as<T>(), fstride, r, delta, want_res ? sample_part.as<double>() : nullptr,
                          part2, plain2);
  }

  // The same pass with the factors (row stride rs) and the partials' buffers
  // given; part null: no residual; part2 (Dantzig selector, may be null):
  // the partials of ||P_Omega(X - B)||^2, summed into *plain2.
  double sample_pass_on(const T *fu, const T *fv, int rs, int r, double delta, double *part,
                        double *part2 = nullptr, double *plain2 = nullptr) {
    const bool want_res = part != nullptr;
    const double vb = sizeof(T);
    // algorithmic bytes of the sampled pass: index, M and Y read, Y written,
    // the row pointers, both factors once
    const double pass_bytes = (double)ix.nnz * (4.0 + 3.0 * vb) + vb * (double)(ix.m + ix.n) * r;
    prof.begin();
    HIP_CHECK(launch_sample_update<T>(stream, lanes_r, rowptr.as<int32_t>(), colidx.as<int32_t>(), Mr.as<T>(),
                                      Yr.as<T>(), (int)ix.m, fu, fv, r, rs, true, delta, part,
                                      ds() ? Yp.as<T>() : nullptr, ds() ? Ym.as<T>() : nullptr,
                                      ds() ? prm.ineq_tol : 0.0, part2));
    prof.end(kSample, pass_bytes + 4.0 * (ix.m + 1));
    // the column copy: the map read, one value gathered and one written per entry
    prof.begin();
    HIP_CHECK(launch_gather<T>(stream, Yr.as<T>(), csr_of_csc.as<int32_t>(), Yc.as<T>(), ix.nnz));
    prof.end(kGather, (double)ix.nnz * (4.0 + 2.0 * vb));
    if (!want_res) return 0.0;
    const int nb = sample_blocks((int)ix.m, lanes_r);
    HIP_CHECK(hipMemcpyAsync(sample_host.p, part, sizeof(double) * nb, hipMemcpyDeviceToHost, stream));
    if (part2)
      HIP_CHECK(hipMemcpyAsync(sample_host.as<double>() + kSampleMaxBlocks + 8, part2, sizeof(double) * nb,
                               hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    auto total = [&](const double *v) {
      double sum = 0.0, comp = 0.0;
      for (int b = 0; b < nb; ++b) {
        const double y = v[b] - comp;
        const double t = sum + y;
        comp = (t - sum) - y;
        sum = t;
      }
      return sum;
    };
    if (part2 && plain2) *plain2 = total(sample_host.as<double>() + kSampleMaxBlocks + 8);
    return total(sample_host.as<double>());
  }

  // ------------------------------------------- general linear operator
  // Section 3.1: measurements b = A(M) = G M_S on a support S (this
  // handle's Omega).  gidx refers to S in the order given to
  // svt_create_sensing; here it is mapped to the row-compressed order, and
  // G^T is built over that order with its terms in measurement order.
  void setup_sensing(int64_t p, const int64_t *gptr, const int32_t *gidx, const double *gval,
                     const double *b) override {
    sensing = true;
    pmeas = p;
    const int64_t ns = ix.nnz, ng = gptr[p];
    std::vector<int32_t> gi((size_t)ng);
    std::vector<T> gv((size_t)ng), bv((size_t)p);
    for (int64_t t = 0; t < ng; ++t) {
      gi[(size_t)t] = ix.csr_of_input[(size_t)gidx[t]];
      gv[(size_t)t] = (T)gval[t];
    }
    for (int64_t i = 0; i < p; ++i) bv[(size_t)i] = (T)b[i];
    std::vector<int64_t> tp((size_t)ns + 1, 0);
    for (int64_t t = 0; t < ng; ++t) tp[(size_t)gi[(size_t)t] + 1]++;
    for (int64_t s2 = 0; s2 < ns; ++s2) tp[(size_t)s2 + 1] += tp[(size_t)s2];
    std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
    std::vector<int32_t> ti((size_t)std::max<int64_t>(ng, 1));
    std::vector<T> tv((size_t)std::max<int64_t>(ng, 1));
    for (int64_t i = 0; i < p; ++i)
      for (int64_t t = gptr[i]; t < gptr[i + 1]; ++t) {
        const int64_t pos = fill[(size_t)gi[(size_t)t]]++;
        ti[(size_t)pos] = (int32_t)i;
        tv[(size_t)pos] = gv[(size_t)t];
      }
    g_ptr.alloc(stream, sizeof(int64_t) * (p + 1));
    g_idx.alloc(stream, sizeof(int32_t) * std::max<int64_t>(ng, 1));
    g_val.alloc(stream, sizeof(T) * std::max<int64_t>(ng, 1));
    gt_ptr.alloc(stream, sizeof(int64_t) * (ns + 1));
    gt_idx.alloc(stream, sizeof(int32_t) * std::max<int64_t>(ng, 1));
    gt_val.alloc(stream, sizeof(T) * std::max<int64_t>(ng, 1));
    b_d.alloc(stream, sizeof(T) * p);
    y_d.alloc(stream, sizeof(T) * p);
    xs_d.alloc(stream, sizeof(T) * ns);
    HIP_CHECK(hipMemcpyAsync(g_ptr.p, gptr, sizeof(int64_t) * (p + 1), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(g_idx.p, gi.data(), sizeof(int32_t) * ng, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(g_val.p, gv.data(), sizeof(T) * ng, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(gt_ptr.p, tp.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(gt_idx.p, ti.data(), sizeof(int32_t) * ng, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(gt_val.p, tv.data(), sizeof(T) * ng, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(b_d.p, bv.data(), sizeof(T) * p, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemsetAsync(y_d.p, 0, sizeof(T) * p, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    note_peak(0);
  }

  // Y = A*(y): G^T y on the support, both compressed copies
  void sensing_adjoint(const T *y) {
    HIP_CHECK(launch_adjoint<T>(stream, gt_ptr.as<int64_t>(), gt_idx.as<int32_t>(), gt_val.as<T>(), y, Yr.as<T>(),
                                ix.nnz));
    HIP_CHECK(launch_gather<T>(stream, Yr.as<T>(), csr_of_csc.as<int32_t>(), Yc.as<T>(), ix.nnz));
  }

  // One pass of eq. (3.3)'s second line: x_S = X on the support (the sampled
  // product with M = 0 into a cleared buffer and delta = -1, so the "update"
  // writes x itself), r = b - G x_S, y += delta r, Y = A*(y); returns |r|^2.
  double sensing_pass(int r, double delta) {
    HIP_CHECK(hipMemsetAsync(xs_d.p, 0, sizeof(T) * ix.nnz, stream));
    HIP_CHECK(launch_sample_update<T>(stream, lanes_r, rowptr.as<int32_t>(), colidx.as<int32_t>(), Mr.as<T>(),
                                      xs_d.as<T>(), (int)ix.m, Fu.as<T>(), Fv.as<T>(), r, fstride, true, -1.0,
                                      nullptr));
    HIP_CHECK(launch_measure<T>(stream, g_ptr.as<int64_t>(), g_idx.as<int32_t>(), g_val.as<T>(), xs_d.as<T>(),
                                b_d.as<T>(), y_d.as<T>(), pmeas, delta, sample_part.as<double>()));
    sensing_adjoint(y_d.as<T>());
    const int nb = measure_blocks(pmeas);
    HIP_CHECK(hipMemcpyAsync(sample_host.p, sample_part.p, sizeof(double) * nb, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    double sum = 0.0, comp = 0.0;
    for (int b = 0; b < nb; ++b) {
      const double y = sample_host.as<double>()[b] - comp;
      const double t = sum + y;
      comp = (t - sum) - y;
      sum = t;
    }
    return sum;
  }

  // The kick for a general operator: while X = 0, y^k = k delta b, so X
  // stays 0 up to k0 = ceil(tau / (delta ||A*(b)||_2)) (eq. (5.3) with A*(b)
  // in place of P_Omega M).
  void do_kick_sensing(double *sigma1, int32_t *k0_out) {
    sensing_adjoint(b_d.as<T>());
    Gkl g;
    BidiagSVD sv;
    int r = 0;
    const int saved_hint = k_hint;
    k_hint = 0;
    const T *yr = a_is_y ? Yr.as<T>() : Yc.as<T>();
    const T *yc = a_is_y ? Yc.as<T>() : Yr.as<T>();
    gkl_run(yr, yc, 1, 1, 0.0, g, sv, r);
    k_hint = saved_hint;
    const double s1 = sv.sigma.empty() ? 0.0 : sv.sigma[0];
    if (!(s1 > 0.0)) throw Error(SVT_EINVAL, "||A*(b)||_2 is zero");
    const int32_t k0 = prm.k0_override > 0 ? prm.k0_override
                                           : (int32_t)std::max(1.0, std::ceil(prm.tau / (prm.delta * s1)));
    HIP_CHECK(launch_axpby<T>(stream, b_d.as<T>(), y_d.as<T>(), pmeas, (double)k0 * prm.delta));
    sensing_adjoint(y_d.as<T>());
    HIP_CHECK(hipStreamSynchronize(stream));
    *sigma1 = s1;
    *k0_out = k0;
  }

  // --------------------------------------------------------------- kick (a2)
  void do_kick(double *sigma1, int32_t *k0_out) {
    if (sensing) return do_kick_sensing(sigma1, k0_out);
    if (ds()) return do_kick_ds(sigma1, k0_out);
    Gkl g;
    BidiagSVD sv;
    int r = 0;
    const int saved_hint = k_hint;
    k_hint = 0;
    const T *mr = a_is_y ? Mr.as<T>() : Mc.as<T>();
    const T *mc = a_is_y ? Mc.as<T>() : Mr.as<T>();
    gkl_run(mr, mc, 1, 1, 0.0, g, sv, r);
    k_hint = saved_hint;
    const double s1 = sv.sigma.empty() ? 0.0 : sv.sigma[0];
    if (!(s1 > 0.0)) throw Error(SVT_EINVAL, "||P_Omega M||_2 is zero");
    int32_t k0 = prm.k0_override > 0 ? prm.k0_override
                                     : (int32_t)std::max(1.0, std::ceil(prm.tau / (prm.delta * s1)));
    const double a = (double)k0 * prm.delta;
    HIP_CHECK(launch_axpby<T>(stream, Mr.as<T>(), Yr.as<T>(), ix.nnz, a));
    HIP_CHECK(launch_axpby<T>(stream, Mc.as<T>(), Yc.as<T>(), ix.nnz, a));
    HIP_CHECK(hipStreamSynchronize(stream));
    *sigma1 = s1;
    *k0_out = k0;
  }

  // The Dantzig selector's kick.  While X = 0 the multipliers grow
  // linearly, Y+ = k delta max(B - E, 0) and Y- = k delta max(-B - E, 0), so
  // Y = k delta S_E(B); X stays 0 up to k0 = ceil(tau / (delta ||S_E(P_Omega
  // B)||_2)) (eq. (5.3) with S_E(B) in place of M).  With S_E(B) = 0 X = 0 is
  // feasible: k0 = 0 and the iteration starts from zero multipliers.
  void do_kick_ds(double *sigma1, int32_t *k0_out) {
    const double E = prm.ineq_tol;
    *sigma1 = 0.0;
    *k0_out = 0;
    if (!ds_soft_nonzero) return;
    // S_E(B) in both copies of Y, then its largest singular value
    HIP_CHECK(launch_ds_init<T>(stream, Mr.as<T>(), ix.nnz, E, 0.0, nullptr, nullptr, Yr.as<T>()));
    HIP_CHECK(launch_gather<T>(stream, Yr.as<T>(), csr_of_csc.as<int32_t>(), Yc.as<T>(), ix.nnz));
    Gkl g;
    BidiagSVD sv;
    int r = 0;
    const int saved_hint = k_hint;
    k_hint = 0;
    const T *yr = a_is_y ? Yr.as<T>() : Yc.as<T>();
    const T *yc = a_is_y ? Yc.as<T>() : Yr.as<T>();
    gkl_run(yr, yc, 1, 1, 0.0, g, sv, r);
    k_hint = saved_hint;
    const double s1 = sv.sigma.empty() ? 0.0 : sv.sigma[0];
    if (!(s1 > 0.0)) return;
    const int32_t k0 = prm.k0_override > 0 ? prm.k0_override
                                           : (int32_t)std::max(1.0, std::ceil(prm.tau / (prm.delta * s1)));
    const double a = (double)k0 * prm.delta;
    HIP_CHECK(launch_ds_init<T>(stream, Mr.as<T>(), ix.nnz, E, a, Yp.as<T>(), Ym.as<T>(), Yr.as<T>()));
    HIP_CHECK(launch_gather<T>(stream, Yr.as<T>(), csr_of_csc.as<int32_t>(), Yc.as<T>(), ix.nnz));
    HIP_CHECK(hipStreamSynchronize(stream));
    *sigma1 = s1;
    *k0_out = k0;
  }

  // -------------------------------------------------------------- solve
  void reset_passes() {
    passes_now = prm.reorth_passes == 2 ? 2 : 1;
    reorth_restarts = 0;
    partial_now = reorth_level() > 0.0 && passes_now == 1;
    partial_run = false;
    full_this_run = false;
    growth_carry = kFirstGrowth;
    hold_hint = 0;
    replay_hint.clear();
    vec_made = vec_orth = partial_fallbacks = 0;
  }

  // The level as an absolute estimate (a multiple of sqrt(u), semi-
  // orthogonality in the vectors' precision) and the rounding term's factor
  // (as OrthEstimate states).
  double orth_eta() const { return reorth_level() * std::sqrt(kUnit); }
  double orth_root() const { return sizeof(T) == 8 ? std::sqrt((double)(arows + acols)) : 1.0; }

  // The partial-reorthogonalisation level as a multiple of sqrt(u): the
  // caller's, or (negative) 0.01 for FP64 vectors and 0.1 for FP32 vectors,
  // whose rounding term sits closer to semi-orthogonality (a shorter horizon
  // for the prediction; 0.1 in FP64 fails the check, measured on the CPU).
  double reorth_level() const {
    if (prm.reorth_eta >= 0.0) return prm.reorth_eta;
    return sizeof(T) == 8 ? 0.01 : 0.1;
  }

  // the growth per half-step assumed by the first partially reorthogonalised
  // bidiagonalisation of a solve, before any has been measured (the largest
  // measured on the completion workloads is about 6.5)
  static constexpr double kFirstGrowth = 8.0;
  // half-steps before the previous bidiagonalisation's replayed first
  // trigger from which predicted triggers are allowed (the first trigger of
  // consecutive SVT iterates moves by about 3)
  static constexpr int kHoldMargin = 8;
  static constexpr int kReplayMinSteps = 64;  // steps of a bidiagonalisation whose pattern is replayed
  static constexpr double kUnit = sizeof(T) == 8 ? 0x1p-53 : 0x1p-24;

  // The largest rank r with r (m + n - r) <= dof_bound * (observations), or
  // -1 when the bound is off (Section 1.1's degrees of freedom of a rank-r
  // matrix; observations: |Omega|, or the measurements of a general operator).
  int dof_rank() const {
    if (!(prm.dof_bound > 0.0)) return -1;
    const double F = prm.dof_bound * (double)(sensing ? pmeas : ix.nnz);
    const double sm = (double)(arows + acols);
    const int rmax = (int)std::min<int64_t>(arows, acols);
    const double disc = sm * sm - 4.0 * F;
    int r = disc <= 0.0 ? rmax : (int)std::floor(0.5 * (sm - std::sqrt(disc)));
    r = std::max(0, std::min(r, rmax));
    auto dof = [&](int q) { return (double)q * (sm - (double)q); };
    while (r > 0 && dof(r) > F) --r;
    while (r < rmax && dof(r + 1) <= F) ++r;
    return r;
  }

  // Whether the vector made by half-step h is orthogonalised against the nq
  // columns of its basis (always, unless partial reorthogonalisation leaves
  // it alone).
  bool orth_vec(int h, int nq) {
    bool r = nq > 0;
    if (partial_run) r = rsched.decide(h) && r;  // every vector is decided, in order
    ++vec_made;
    if (r) ++vec_orth;
    return r;
  }

  void reorth_stats(int64_t *vectors, int64_t *orthogonalised, int64_t *two_pass_restarts,
                    int64_t *fallbacks) const override {
    if (vectors) *vectors = vec_made;
    if (orthogonalised) *orthogonalised = vec_orth;
    if (two_pass_restarts) *two_pass_restarts = reorth_restarts;
    if (fallbacks) *fallbacks = partial_fallbacks;
  }

  svt_status solve(svt_info *info) override {
    reset_passes();
    history.clear();
    prof.reset();
    steps_total = 0;
    rng_ctr = 0;
    rs_ctr = 0;
    k_hint = 0;
    rank = 0;
    w.clear();
    svt_info inf{};
    inf.norm_pm = norm_pm;
    inf.t_setup_s = t_setup;
    const double t0 = now_s();
    double t1 = t0;
    const T *yr = a_is_y ? Yr.as<T>() : Yc.as<T>();
    const T *yc = a_is_y ? Yc.as<T>() : Yr.as<T>();
    int r_prev = 0;
    svt_status st = SVT_NOT_CONVERGED;
    int k = 0;
    double res = 1.0;
    // the stall bound: the smallest residual so far and its iteration
    double best_res = std::numeric_limits<double>::infinity();
    int best_k = 0;
    dof_rmax = dof_rank();
    dof_hit = false;
    // an error in the kick or the loop still reports the iterations completed
    auto report = [&](int iters, svt_status status) {
      inf.t_solve_s = now_s() - t1;
      inf.iters = iters;
      inf.rank = rank;
      inf.rel_residual = res;
      inf.status = status;
      inf.gkl_steps = steps_total;
      if (info) *info = inf;
    };
    try {
      double s1 = 0.0;
      int32_t k0 = 0;
      if (!prm.warm_start) {
        // a cold start: Y = 0, then the kick; a warm start keeps the
        // handle's iterate (Section 6's continuation)
        HIP_CHECK(hipMemsetAsync(Yr.p, 0, sizeof(T) * ix.nnz, stream));
        HIP_CHECK(hipMemsetAsync(Yc.p, 0, sizeof(T) * ix.nnz, stream));
        if (ds()) {
          HIP_CHECK(hipMemsetAsync(Yp.p, 0, sizeof(T) * ix.nnz, stream));
          HIP_CHECK(hipMemsetAsync(Ym.p, 0, sizeof(T) * ix.nnz, stream));
        }
        if (sensing) HIP_CHECK(hipMemsetAsync(y_d.p, 0, sizeof(T) * pmeas, stream));
        if (prm.kick) do_kick(&s1, &k0);
      }
      HIP_CHECK(hipStreamSynchronize(stream));
      t1 = now_s();
      inf.t_kick_s = t1 - t0;
      inf.sigma1 = s1;
      inf.k0 = k0;

      for (k = 1; k <= prm.maxiter; ++k) {
        int r = 0, s = 0, steps = 0;
        std::vector<double> ws;
        if (prm.svd_method == SVT_SVD_RANDOMIZED) {
          randomized_iteration(r_prev, r, s, steps, ws);
        } else {
          Gkl g;
          BidiagSVD sv;
          steps = gkl_run(yr, yc, 0, 0, prm.tau, g, sv, r);
          k_hint = steps;
          if (dof_hit) {
            // the step's rank passes the degrees-of-freedom bound: it ends
            // without its update; the factors keep the last completed iterate
            st = SVT_UNDERDETERMINED;
            break;
          }
          // s_k bookkeeping of Algorithm 1's repeat loop (Section 5.1.1)
          s = std::min<int64_t>(r_prev + 1, acols);
          while (s <= r && s < acols) s = (int)std::min<int64_t>(s + prm.incr, acols);
          ws.assign(std::max(r, 1), 0.0);
          for (int i = 0; i < r; ++i) ws[i] = sv.sigma[i] - prm.tau;
          form_factors(g, sv, r, ws.data());
        }
        w.assign(ws.begin(), ws.begin() + r);
        double plain2 = 0.0;  // Dantzig selector: ||P_Omega(X - B)||^2 beside the violation
        const double res2 = sensing ? sensing_pass(r, prm.delta) : sample_pass(r, prm.delta, true, &plain2);
        res = std::sqrt(res2) / norm_pm;
        history.push_back({r, s, steps, res});
        if (log_level > 0)
          std::fprintf(stderr, "[svt] iter %d rank %d steps %d res %.3e t %.3f s\n", k, r, steps, res, now_s() - t1);
        if (!std::isfinite(res)) { st = SVT_EDIVERGED; break; }
        bool stop;
        if (prm.stop_rule == SVT_STOP_NOISY)
          stop = (ds() ? plain2 : res2) <= (1.0 + prm.eps) * (double)ix.nnz * prm.noise_sigma * prm.noise_sigma;
        else
          stop = res <= prm.eps;
        if (stop) { st = SVT_OK; break; }
        if (prm.stall_window > 0) {
          if (res < best_res) {
            best_res = res;
            best_k = k;
          } else if (k - best_k >= prm.stall_window) {
            st = SVT_STALLED;
            break;
          }
        }
        r_prev = r;
      }
    } catch (const Error &e) {
      report((int)history.size(), e.code);
      throw;
    }
    if (k > prm.maxiter) k = prm.maxiter;
    if (st == SVT_UNDERDETERMINED) k -= 1;  // step k did not complete
    HIP_CHECK(hipStreamSynchronize(stream));
    prof.flush();
    report(k, st);
    return st;
  }

  // ---------------------------------------------------------- outputs
  void factors(int32_t *rank_out, double *U, double *wout, double *V) const override {
    if (rank_out) *rank_out = rank;
    if (rank == 0) return;
    const int64_t m = ix.m, n = ix.n;
    std::vector<T> hu((size_t)m * fstride), hv((size_t)n * fstride);
    HIP_CHECK(hipMemcpyAsync(hu.data(), Fu.p, sizeof(T) * hu.size(), hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipMemcpyAsync(hv.data(), Fv.p, sizeof(T) * hv.size(), hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    if (U)
      for (int64_t i = 0; i < m; ++i)
        for (int l = 0; l < rank; ++l) U[(size_t)i * rank + l] = (double)hu[(size_t)i * fstride + l];
    if (V)
      for (int64_t j = 0; j < n; ++j)
        for (int l = 0; l < rank; ++l) V[(size_t)j * rank + l] = (double)hv[(size_t)j * fstride + l];
    if (wout)
      for (int l = 0; l < rank; ++l) wout[l] = w[l];
  }

  void set_iterate(const double *y) override {
    std::vector<double> csr((size_t)ix.nnz);
    for (int64_t t = 0; t < ix.nnz; ++t) csr[(size_t)ix.csr_of_input[(size_t)t]] = y[t];
    upload_values(csr.data(), Yr.as<T>(), Yc.as<T>());
  }

  // Dantzig selector: Y+ and Y- given in the order of the input triplets;
  // the iterate becomes Y = Y+ - Y- (both compressed copies).
  void set_multipliers(const double *yp, const double *ym) override {
    if (!ds()) throw Error(SVT_ESTATE, "the handle does not run the Dantzig-selector iteration");
    const int64_t nnz = ix.nnz;
    std::vector<T> hp((size_t)nnz), hm((size_t)nnz), hy((size_t)nnz);
    for (int64_t t = 0; t < nnz; ++t) {
      const size_t c = (size_t)ix.csr_of_input[(size_t)t];
      hp[c] = (T)yp[t];
      hm[c] = (T)ym[t];
      hy[c] = hp[c] - hm[c];
    }
    HIP_CHECK(hipMemcpyAsync(Yp.p, hp.data(), sizeof(T) * nnz, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(Ym.p, hm.data(), sizeof(T) * nnz, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(Yr.p, hy.data(), sizeof(T) * nnz, hipMemcpyHostToDevice, stream));
    HIP_CHECK(launch_gather<T>(stream, Yr.as<T>(), csr_of_csc.as<int32_t>(), Yc.as<T>(), nnz));
    HIP_CHECK(hipStreamSynchronize(stream));
  }

  void get_multipliers(double *yp, double *ym) const override {
    if (!ds()) throw Error(SVT_ESTATE, "the handle does not run the Dantzig-selector iteration");
    const int64_t nnz = ix.nnz;
    std::vector<T> hp((size_t)nnz), hm((size_t)nnz);
    HIP_CHECK(hipMemcpyAsync(hp.data(), Yp.p, sizeof(T) * nnz, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipMemcpyAsync(hm.data(), Ym.p, sizeof(T) * nnz, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    for (int64_t t = 0; t < nnz; ++t) {
      const size_t c = (size_t)ix.csr_of_input[(size_t)t];
      if (yp) yp[t] = (double)hp[c];
      if (ym) ym[t] = (double)hm[c];
    }
  }

  void get_iterate(int which, double *y) const override {
    std::vector<T> h((size_t)ix.nnz);
    HIP_CHECK(hipMemcpyAsync(h.data(), which ? Yc.p : Yr.p, sizeof(T) * ix.nnz, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    for (int64_t t = 0; t < ix.nnz; ++t) {
      const int32_t c = ix.csr_of_input[(size_t)t];
      y[t] = (double)(which ? h[(size_t)ix.csc_of_csr[(size_t)c]] : h[(size_t)c]);
    }
  }

  void apply(int trans, const double *x, double *out) override {
    // trans = 0: Y x through the row-compressed copy; 1: Y^T x through the column copy
    const int64_t nin = trans ? ix.m : ix.n, nout = trans ? ix.n : ix.m;
    std::vector<T> hx((size_t)nin);
    for (int64_t i = 0; i < nin; ++i) hx[(size_t)i] = (T)x[i];
    DevMem dx, dout;
    dx.alloc(stream, sizeof(T) * nin);
    dout.alloc(stream, sizeof(T) * nout);
    note_peak(dx.bytes + dout.bytes);
    HIP_CHECK(hipMemcpyAsync(dx.p, hx.data(), sizeof(T) * nin, hipMemcpyHostToDevice, stream));
    const Csx c = trans ? csc_struct() : csr_struct();
    SpmvInput<T> in;
    in.x = dx.as<T>();
    spmv(c, trans ? Yc.as<T>() : Yr.as<T>(), in, nullptr, dout.as<T>());
    std::vector<T> ho((size_t)nout);
    HIP_CHECK(hipMemcpyAsync(ho.data(), dout.p, sizeof(T) * nout, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    for (int64_t i = 0; i < nout; ++i) out[i] = (double)ho[(size_t)i];
  }

  int partial_svd(int count, double *sigma, double *U, double *V) override {
    if (count > acols) throw Error(SVT_EINVAL, "count exceeds min(m, n)");
    reset_passes();
    Gkl g;
    BidiagSVD sv;
    int r = 0;
    const T *yr = a_is_y ? Yr.as<T>() : Yc.as<T>();
    const T *yc = a_is_y ? Yc.as<T>() : Yr.as<T>();
    k_hint = 0;
    const int steps = gkl_run(yr, yc, 1, count, 0.0, g, sv, r);
    std::vector<double> ones(count, 1.0);
    form_factors(g, sv, count, ones.data());
    for (int i = 0; i < count; ++i) sigma[i] = sv.sigma[i];
    factors(nullptr, U, nullptr, V);
    rank = 0;  // the handle's X is not this partial SVD
    return steps;
  }

  double sample_update(int r, const double *U, const double *V, double delta) override {
    ensure_factors(std::max(r, 1), 1);
    const int64_t m = ix.m, n = ix.n;
    std::vector<T> hu((size_t)m * fstride, (T)0), hv((size_t)n * fstride, (T)0);
    for (int64_t i = 0; i < m; ++i)
      for (int l = 0; l < r; ++l) hu[(size_t)i * fstride + l] = (T)U[(size_t)i * r + l];
    for (int64_t j = 0; j < n; ++j)
      for (int l = 0; l < r; ++l) hv[(size_t)j * fstride + l] = (T)V[(size_t)j * r + l];
    HIP_CHECK(hipMemcpyAsync(Fu.p, hu.data(), sizeof(T) * hu.size(), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(Fv.p, hv.data(), sizeof(T) * hv.size(), hipMemcpyHostToDevice, stream));
    rank = 0;
    return sample_pass(r, delta, true);
  }

  // svt_sample_update_noalloc: device factors in the value type T, row
  // stride rs; the partials go to the device's fixed scratch array.  No
  // device or host allocation: the partials' host copy is the pinned buffer
  // made at setup.
  double sample_update_noalloc(int r, const void *U, const void *V, int64_t rs, double delta) override {
    constexpr int al = 16 / (int)sizeof(T);
    if (rs < std::max(r, 1) || rs % al != 0 || rs > INT32_MAX)
      throw Error(SVT_EINVAL, "stride must be >= max(r, 1) and a multiple of " + std::to_string(al) +
                                  " elements of the handle's value type");
    if (r > 0 && ((reinterpret_cast<uintptr_t>(U) & 15) || (reinterpret_cast<uintptr_t>(V) & 15)))
      throw Error(SVT_EINVAL, "U and V must be 16-byte aligned device pointers");
    const int nb = sample_blocks((int)ix.m, lanes_r);
    if (nb > kNoAllocScratchDoubles || (size_t)nb * sizeof(double) > sample_host.bytes)
      throw Error(SVT_EINVAL, "the residual partials (" + std::to_string(nb) +
                                  ") exceed the fixed scratch of the allocation-free pass");
    if (!noalloc_part) throw Error(SVT_ESTATE, "no scratch address for this device");
    int cur = -1;
    HIP_CHECK(hipGetDevice(&cur));
    if (cur != device) throw Error(SVT_EINVAL, "the handle's device is not the current device");
    rank = 0;  // the handle's X is not this caller's X
    return sample_pass_on(static_cast<const T *>(U), static_cast<const T *>(V), (int)rs, r, delta, noalloc_part);
  }

  void kick(double *sigma1, int32_t *k0) override {
    reset_passes();
    do_kick(sigma1, k0);
  }

  ~Problem() override {
    if (stream) (void)hipStreamSynchronize(stream);
    // every buffer goes back to the pool on its stream before the stream ends
    for (DevMem *d : all_mem()) d->release();
    if (stream) (void)hipStreamSynchronize(stream);
    if (fetch_ev) (void)hipEventDestroy(fetch_ev);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

// ---------------------------------------------------------------------------
// validation (before any device call)

static void validate_params(const svt_params &p) {
  auto finite = [](double v) { return std::isfinite(v); };
  if (!finite(p.tau) || p.tau <= 0) throw Error(SVT_EINVAL, "tau must be finite and > 0");
  if (!finite(p.delta) || p.delta <= 0) throw Error(SVT_EINVAL, "delta must be finite and > 0");
  if (!finite(p.eps) || p.eps < 0) throw Error(SVT_EINVAL, "eps must be finite and >= 0");
  if (p.maxiter < 1) throw Error(SVT_EINVAL, "maxiter must be >= 1");
  if (p.incr < 1) throw Error(SVT_EINVAL, "incr (ell) must be >= 1");
  if (p.kick != 0 && p.kick != 1) throw Error(SVT_EINVAL, "kick must be 0 or 1");
  if (p.k0_override < 0) throw Error(SVT_EINVAL, "k0_override must be >= 0");
  if (p.precision != SVT_FP64 && p.precision != SVT_MIXED) throw Error(SVT_EINVAL, "unknown precision");
  if (p.stop_rule != SVT_STOP_RELRES && p.stop_rule != SVT_STOP_NOISY) throw Error(SVT_EINVAL, "unknown stop rule");
  if (!finite(p.noise_sigma) || p.noise_sigma < 0) throw Error(SVT_EINVAL, "noise_sigma must be finite and >= 0");
  if (p.stop_rule == SVT_STOP_NOISY && p.noise_sigma <= 0) throw Error(SVT_EINVAL, "the noisy stop rule needs noise_sigma > 0");
  if (p.constraint != SVT_CONSTRAINT_EQUALITY && p.constraint != SVT_CONSTRAINT_INEQUALITY)
    throw Error(SVT_EINVAL, "unknown constraint kind");
  if (!finite(p.ineq_tol) || p.ineq_tol < 0) throw Error(SVT_EINVAL, "ineq_tol must be finite and >= 0");
  if (p.warm_start != 0 && p.warm_start != 1) throw Error(SVT_EINVAL, "warm_start must be 0 or 1");
  if (p.min_block_rows < 0 || p.min_block_rows > kMaxRowsPerBlock)
    throw Error(SVT_EINVAL, "min_block_rows must be in [0, 2048]");
  if (p.svd_method != SVT_SVD_LANCZOS && p.svd_method != SVT_SVD_RANDOMIZED)
    throw Error(SVT_EINVAL, "unknown svd_method");
  if (p.rsvd_oversample < 0 || p.rsvd_power < 0 || p.rsvd_power > 64)
    throw Error(SVT_EINVAL, "rsvd_oversample must be >= 0 and rsvd_power in [0, 64]");
  if (p.svd_method == SVT_SVD_RANDOMIZED && p.constraint != SVT_CONSTRAINT_EQUALITY)
    throw Error(SVT_EINVAL, "the randomised partial SVD serves the equality form only");

  if (!finite(p.lanczos_tol) || p.lanczos_tol < 0 || p.lanczos_tol >= 1) throw Error(SVT_EINVAL, "lanczos_tol must be in [0, 1)");
  if (p.lanczos_maxsteps < 0) throw Error(SVT_EINVAL, "lanczos_maxsteps must be >= 0");
  if (p.reorth_passes < 0 || p.reorth_passes > 2) throw Error(SVT_EINVAL, "reorth_passes must be 0, 1 or 2");
  if (!finite(p.reorth_eta) || p.reorth_eta > 100)
    throw Error(SVT_EINVAL, "reorth_eta must be finite and at most 100");
  if (!finite(p.dof_bound)) throw Error(SVT_EINVAL, "dof_bound must be finite");
  if (!finite(p.decide_margin) || p.decide_margin < 0) throw Error(SVT_EINVAL, "decide_margin must be finite and >= 0");
  if (p.spmv_mode < 0 || p.spmv_mode > 2) throw Error(SVT_EINVAL, "spmv_mode must be 0, 1 or 2");
}

}  // namespace svt

// ===========================================================================
// C ABI

struct svt_problem {
  std::unique_ptr<svt::ProblemBase> impl;
};

using svt::Error;

template <typename F>
static svt_status guarded(const svt_problem *h, F &&f) {
  try {
    return f();
  } catch (const Error &e) {
    if (h && h->impl) h->impl->last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    if (h && h->impl) h->impl->last_error = "host allocation failed";
    return SVT_ENOMEM;
  } catch (const std::exception &e) {
    if (h && h->impl) h->impl->last_error = e.what();
    return SVT_EDEVICE;
  } catch (...) {
    if (h && h->impl) h->impl->last_error = "unknown error";
    return SVT_EDEVICE;
  }
}

extern "C" {

svt_status svt_params_default(int64_t m, int64_t n, int64_t nnz, svt_params *out) {
  if (!out || m < 1 || n < 1 || nnz < 1) return SVT_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->tau = 5.0 * std::sqrt((double)m * (double)n);
  out->delta = 1.2 * (double)m * (double)n / (double)nnz;
  out->eps = 1e-4;
  out->maxiter = 500;
  out->incr = 5;
  out->kick = 1;
  out->k0_override = 0;
  out->precision = SVT_FP64;
  out->stop_rule = SVT_STOP_RELRES;
  out->constraint = SVT_CONSTRAINT_EQUALITY;
  out->ineq_tol = 0.0;
  out->noise_sigma = 0.0;
  out->lanczos_tol = 0.0;  // auto: 1e-12 (FP64) or 1e-6 (MIXED)
  out->lanczos_maxsteps = 0;
  out->reorth_passes = 0;
  out->reorth_eta = -1.0;  // automatic: 0.01 (FP64 vectors), 0.1 (FP32 vectors)
  out->dof_bound = 0.0;
  out->decide_margin = 0.05;
  out->svd_method = SVT_SVD_LANCZOS;
  out->rsvd_oversample = 10;
  out->rsvd_power = 2;
  out->seed = 0x5EEDull;
  out->profile = 0;
  out->stream = nullptr;
  return SVT_OK;
}

svt_status svt_create(int64_t m, int64_t n, int64_t nnz, int32_t fmt, const void *idx0,
                      const int32_t *idx1, const double *vals, const svt_params *params,
                      svt_problem **out) {
  if (out) *out = nullptr;
  svt::g_create_error.clear();
  try {
    if (!out) throw Error(SVT_EINVAL, "out is NULL");
    if (m < 1 || n < 1) throw Error(SVT_EINVAL, "m and n must be >= 1");
    if (m > INT32_MAX - 1 || n > INT32_MAX - 1) throw Error(SVT_EINVAL, "m and n must be < 2^31 - 1");
    if (nnz < 1) throw Error(SVT_EINVAL, "nnz must be >= 1");
    if ((double)nnz > (double)m * (double)n || nnz > m * n) throw Error(SVT_EINVAL, "nnz exceeds m*n");
    if (nnz > INT32_MAX) throw Error(SVT_EINVAL, "nnz must be < 2^31");
    if (!idx0 || !idx1 || !vals) throw Error(SVT_EINVAL, "index or value pointer is NULL");
    if (fmt != SVT_COO && fmt != SVT_CSR) throw Error(SVT_EINVAL, "unknown index format");
    svt_params prm;
    if (params) prm = *params;
    else svt_params_default(m, n, nnz, &prm);
    svt::validate_params(prm);
    if (prm.lanczos_tol == 0.0) prm.lanczos_tol = (prm.precision == SVT_MIXED) ? 1e-6 : 1e-12;
    // rows of every entry
    std::vector<int32_t> rows_buf;
    const int32_t *rows = nullptr;
    if (fmt == SVT_COO) {
      rows = static_cast<const int32_t *>(idx0);
    } else {
      const int64_t *rp = static_cast<const int64_t *>(idx0);
      if (rp[0] != 0 || rp[m] != nnz) throw Error(SVT_EINVAL, "rowptr must start at 0 and end at nnz");
      rows_buf.resize((size_t)nnz);
      for (int64_t i = 0; i < m; ++i) {
        if (rp[i + 1] < rp[i]) throw Error(SVT_EINVAL, "rowptr must be non-decreasing");
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t) rows_buf[(size_t)t] = (int32_t)i;
      }
      rows = rows_buf.data();
    }
    bool any_nonzero = false;
    for (int64_t t = 0; t < nnz; ++t) {
      if (rows[t] < 0 || rows[t] >= m) throw Error(SVT_EINVAL, "row index out of range at entry " + std::to_string(t));
      if (idx1[t] < 0 || idx1[t] >= n) throw Error(SVT_EINVAL, "column index out of range at entry " + std::to_string(t));
      if (!std::isfinite(vals[t])) throw Error(SVT_EINVAL, "non-finite value at entry " + std::to_string(t));
      any_nonzero |= (vals[t] != 0.0);
    }
    if (!any_nonzero) throw Error(SVT_EINVAL, "all observed values are zero: the stop test is undefined");

    const double t0 = svt::now_s();
    std::unique_ptr<svt::ProblemBase> impl;
    if (prm.precision == SVT_MIXED) impl.reset(new svt::Problem<float>());
    else impl.reset(new svt::Problem<double>());
    svt::build_index(m, n, nnz, rows, idx1, vals, impl->ix);
    {
      // ||P_Omega M||_F with a compensated sum
      double s = 0.0, c = 0.0;
      for (int64_t t = 0; t < nnz; ++t) {
        const double y = vals[t] * vals[t] - c;
        const double tt = s + y;
        c = (tt - s) - y;
        s = tt;
      }
      impl->norm_pm = std::sqrt(s);
    }
    for (int64_t t = 0; t < nnz && !impl->ds_soft_nonzero; ++t)
      impl->ds_soft_nonzero = std::fabs(vals[t]) > prm.ineq_tol;
    if (prm.precision == SVT_MIXED) static_cast<svt::Problem<float> *>(impl.get())->setup(prm);
    else static_cast<svt::Problem<double> *>(impl.get())->setup(prm);
    impl->t_setup = svt::now_s() - t0;
    svt_problem *h = new svt_problem();
    h->impl = std::move(impl);
    *out = h;
    return SVT_OK;
  } catch (const Error &e) {
    svt::g_create_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    svt::g_create_error = "host allocation failed";
    return SVT_ENOMEM;
  } catch (const std::exception &e) {
    svt::g_create_error = e.what();
    return SVT_EDEVICE;
  }
}

svt_status svt_create_sensing(int64_t m, int64_t n, int64_t ns, const int32_t *srows, const int32_t *scols,
                              int64_t p, const int64_t *gptr, const int32_t *gidx, const double *gval,
                              const double *b, const svt_params *params, svt_problem **out) {
  if (out) *out = nullptr;
  svt::g_create_error.clear();
  try {
    if (!out) throw Error(SVT_EINVAL, "out is NULL");
    if (m < 1 || n < 1 || m > INT32_MAX - 1 || n > INT32_MAX - 1) throw Error(SVT_EINVAL, "bad dimensions");
    if (ns < 1 || (double)ns > (double)m * (double)n || ns > INT32_MAX) throw Error(SVT_EINVAL, "bad support size");
    if (p < 1 || p > INT32_MAX) throw Error(SVT_EINVAL, "bad measurement count");
    if (!srows || !scols || !gptr || !gidx || !gval || !b) throw Error(SVT_EINVAL, "NULL array");
    if (params && params->svd_method != SVT_SVD_LANCZOS)
      throw Error(SVT_EINVAL, "the randomised partial SVD serves matrix completion only");
    if (gptr[0] != 0) throw Error(SVT_EINVAL, "gptr must start at 0");
    for (int64_t i = 0; i < p; ++i)
      if (gptr[i + 1] < gptr[i]) throw Error(SVT_EINVAL, "gptr must be non-decreasing");
    const int64_t ng = gptr[p];
    if (ng > INT32_MAX) throw Error(SVT_EINVAL, "too many measurement terms");
    for (int64_t t = 0; t < ng; ++t) {
      if (gidx[t] < 0 || gidx[t] >= ns) throw Error(SVT_EINVAL, "gidx out of range at term " + std::to_string(t));
      if (!std::isfinite(gval[t])) throw Error(SVT_EINVAL, "non-finite weight at term " + std::to_string(t));
    }
    bool any = false;
    for (int64_t i = 0; i < p; ++i) {
      if (!std::isfinite(b[i])) throw Error(SVT_EINVAL, "non-finite measurement");
      any |= b[i] != 0.0;
    }
    if (!any) throw Error(SVT_EINVAL, "all measurements are zero: the stop test is undefined");
    for (int64_t t = 0; t < ns; ++t)
      if (srows[t] < 0 || srows[t] >= m || scols[t] < 0 || scols[t] >= n)
        throw Error(SVT_EINVAL, "support index out of range at entry " + std::to_string(t));
    svt_params prm;
    if (params) prm = *params;
    else svt_params_default(m, n, p, &prm);
    svt::validate_params(prm);
    if (prm.constraint != SVT_CONSTRAINT_EQUALITY || prm.stop_rule != SVT_STOP_RELRES)
      throw Error(SVT_EINVAL, "a general operator takes equality constraints and the relative-residual stop");
    if (prm.lanczos_tol == 0.0) prm.lanczos_tol = (prm.precision == SVT_MIXED) ? 1e-6 : 1e-12;
    const double t0 = svt::now_s();
    std::unique_ptr<svt::ProblemBase> impl;
    if (prm.precision == SVT_MIXED) impl.reset(new svt::Problem<float>());
    else impl.reset(new svt::Problem<double>());
    std::vector<double> zeros((size_t)ns, 0.0);
    svt::build_index(m, n, ns, srows, scols, zeros.data(), impl->ix);
    {
      double s2 = 0.0, c = 0.0;
      for (int64_t i = 0; i < p; ++i) {
        const double y = b[i] * b[i] - c;
        const double tt = s2 + y;
        c = (tt - s2) - y;
        s2 = tt;
      }
      impl->norm_pm = std::sqrt(s2);
    }
    if (prm.precision == SVT_MIXED) static_cast<svt::Problem<float> *>(impl.get())->setup(prm);
    else static_cast<svt::Problem<double> *>(impl.get())->setup(prm);
    impl->setup_sensing(p, gptr, gidx, gval, b);
    impl->t_setup = svt::now_s() - t0;
    svt_problem *h = new svt_problem();
    h->impl = std::move(impl);
    *out = h;
    return SVT_OK;
  } catch (const Error &e) {
    svt::g_create_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    svt::g_create_error = "host allocation failed";
    return SVT_ENOMEM;
  } catch (const std::exception &e) {
    svt::g_create_error = e.what();
    return SVT_EDEVICE;
  }
}

svt_status svt_solve(svt_problem *h, svt_info *info) {
  if (!h || !h->impl) return SVT_EINVAL;
  return guarded(h, [&] { return h->impl->solve(info); });
}

svt_status svt_solve_path(svt_problem *h, const double *taus, int32_t count, svt_info *infos) {
  if (!h || !h->impl || !taus || count < 1) return SVT_EINVAL;
  for (int32_t i = 0; i < count; ++i)
    if (!std::isfinite(taus[i]) || taus[i] <= 0) return SVT_EINVAL;
  auto &prm = h->impl->prm;
  const double tau0 = prm.tau;
  const int32_t warm0 = prm.warm_start;
  svt_status st = SVT_OK;
  for (int32_t i = 0; i < count; ++i) {
    prm.tau = taus[i];
    prm.warm_start = i == 0 ? warm0 : 1;
    st = guarded(h, [&] { return h->impl->solve(infos ? infos + i : nullptr); });
    if (st != SVT_OK && st != SVT_NOT_CONVERGED && st != SVT_STALLED && st != SVT_UNDERDETERMINED) break;
  }
  prm.tau = tau0;
  prm.warm_start = warm0;
  return st;
}

svt_status svt_history(const svt_problem *h, int32_t cap, int32_t *ranks, int32_t *s_hist,
                       double *residuals, int32_t *gkl_steps, int32_t *len_out) {
  if (!h || !h->impl || cap < 0) return SVT_EINVAL;
  const auto &hist = h->impl->history;
  const int32_t len = (int32_t)hist.size();
  if (len_out) *len_out = len;
  for (int32_t i = 0; i < std::min(cap, len); ++i) {
    if (ranks) ranks[i] = hist[i].rank;
    if (s_hist) s_hist[i] = hist[i].s;
    if (residuals) residuals[i] = hist[i].res;
    if (gkl_steps) gkl_steps[i] = hist[i].steps;
  }
  return SVT_OK;
}

svt_status svt_factors(const svt_problem *h, int32_t *rank_out, double *U, double *w, double *V) {
  if (!h || !h->impl) return SVT_EINVAL;
  return guarded(h, [&] {
    h->impl->factors(rank_out, U, w, V);
    return SVT_OK;
  });
}

svt_status svt_predict(const svt_problem *h, int64_t q, const int32_t *rows, const int32_t *cols,
                       double *out) {
  if (!h || !h->impl || q < 0 || (q > 0 && (!rows || !cols || !out))) return SVT_EINVAL;
  return guarded(h, [&] {
    const auto &ix = h->impl->ix;
    for (int64_t t = 0; t < q; ++t)
      if (rows[t] < 0 || rows[t] >= ix.m || cols[t] < 0 || cols[t] >= ix.n)
        throw Error(SVT_EINVAL, "predict index out of range at " + std::to_string(t));
    int32_t r = 0;
    h->impl->factors(&r, nullptr, nullptr, nullptr);
    std::vector<double> U((size_t)ix.m * std::max(r, 1)), V((size_t)ix.n * std::max(r, 1));
    if (r > 0) h->impl->factors(&r, U.data(), nullptr, V.data());
    for (int64_t t = 0; t < q; ++t) {
      double s = 0.0;
      for (int l = 0; l < r; ++l) s += U[(size_t)rows[t] * r + l] * V[(size_t)cols[t] * r + l];
      out[t] = s;
    }
    return SVT_OK;
  });
}

void svt_destroy(svt_problem *h) { delete h; }

const char *svt_status_string(int32_t s) {
  switch (s) {
    case SVT_OK: return "ok";
    case SVT_NOT_CONVERGED: return "not converged (maxiter reached)";
    case SVT_STALLED: return "stalled (no new residual minimum within stall_window iterations)";
    case SVT_UNDERDETERMINED: return "underdetermined (the rank has more degrees of freedom than dof_bound observations)";
    case SVT_EINVAL: return "invalid argument";
    case SVT_ENOMEM: return "out of memory";
    case SVT_EDEVICE: return "device error";
    case SVT_ESTATE: return "invalid state";
    case SVT_EDIVERGED: return "diverged (non-finite residual)";
    case SVT_EBUSY: return "busy";
    case SVT_ELANCZOS: return "partial SVD did not converge";
    default: return "unknown status";
  }
}

const char *svt_last_error(const svt_problem *h) {
  if (!h || !h->impl) return svt::g_create_error.c_str();
  return h->impl->last_error.c_str();
}

svt_status svt_set_iterate(svt_problem *h, const double *y) {
  if (!h || !h->impl || !y) return SVT_EINVAL;
  return guarded(h, [&] {
    for (int64_t t = 0; t < h->impl->ix.nnz; ++t)
      if (!std::isfinite(y[t])) throw Error(SVT_EINVAL, "non-finite iterate value");
    h->impl->set_iterate(y);
    return SVT_OK;
  });
}

svt_status svt_set_multipliers(svt_problem *h, const double *yp, const double *ym) {
  if (!h || !h->impl || !yp || !ym) return SVT_EINVAL;
  return guarded(h, [&] {
    for (int64_t t = 0; t < h->impl->ix.nnz; ++t)
      if (!std::isfinite(yp[t]) || !std::isfinite(ym[t]) || yp[t] < 0 || ym[t] < 0)
        throw Error(SVT_EINVAL, "multipliers must be finite and >= 0");
    h->impl->set_multipliers(yp, ym);
    return SVT_OK;
  });
}

svt_status svt_get_multipliers(const svt_problem *h, double *yp, double *ym) {
  if (!h || !h->impl) return SVT_EINVAL;
  return guarded(h, [&] {
    h->impl->get_multipliers(yp, ym);
    return SVT_OK;
  });
}

svt_status svt_get_iterate(const svt_problem *h, int32_t which, double *y) {
  if (!h || !h->impl || !y || (which != 0 && which != 1)) return SVT_EINVAL;
  return guarded(h, [&] {
    h->impl->get_iterate(which, y);
    return SVT_OK;
  });
}

svt_status svt_apply(svt_problem *h, int32_t trans, const double *x, double *out) {
  if (!h || !h->impl || !x || !out || (trans != 0 && trans != 1)) return SVT_EINVAL;
  return guarded(h, [&] {
    h->impl->apply(trans, x, out);
    return SVT_OK;
  });
}

svt_status svt_partial_svd(svt_problem *h, int32_t count, double *sigma, double *U, double *V,
                           int32_t *steps_out) {
  if (!h || !h->impl || !sigma || count < 1) return SVT_EINVAL;
  return guarded(h, [&] {
    const int steps = h->impl->partial_svd(count, sigma, U, V);
    if (steps_out) *steps_out = steps;
    return SVT_OK;
  });
}

svt_status svt_sample_update(svt_problem *h, int32_t r, const double *U, const double *V,
                             double delta, double *res2) {
  if (!h || !h->impl || r < 0 || (r > 0 && (!U || !V)) || !std::isfinite(delta)) return SVT_EINVAL;
  return guarded(h, [&] {
    const double v = h->impl->sample_update(r, U, V, delta);
    if (res2) *res2 = v;
    return SVT_OK;
  });
}

svt_status svt_sample_update_noalloc(svt_problem *h, int32_t r, const void *U, const void *V, int64_t stride,
                                     double delta, double *res2) {
  if (!h || !h->impl || r < 0 || (r > 0 && (!U || !V)) || !std::isfinite(delta)) return SVT_EINVAL;
  return guarded(h, [&] {
    const double v = h->impl->sample_update_noalloc(r, U, V, stride, delta);
    if (res2) *res2 = v;
    return SVT_OK;
  });
}

svt_status svt_kick(svt_problem *h, double *sigma1, int32_t *k0) {
  if (!h || !h->impl) return SVT_EINVAL;
  return guarded(h, [&] {
    double s = 0.0;
    int32_t k = 0;
    h->impl->kick(&s, &k);
    if (sigma1) *sigma1 = s;
    if (k0) *k0 = k;
    return SVT_OK;
  });
}

svt_status svt_spmv_plan(const svt_problem *h, int32_t which, int32_t *segments) {
  if (!h || !h->impl || (which != 0 && which != 1) || !segments) return SVT_EINVAL;
  *segments = h->impl->spmv_segments(which);
  return SVT_OK;
}

svt_status svt_device_bytes(const svt_problem *h, size_t *current, size_t *peak) {
  if (!h || !h->impl) return SVT_EINVAL;
  h->impl->mem_stats(current, peak);
  return SVT_OK;
}

svt_status svt_reorth_stats(const svt_problem *h, int64_t *vectors, int64_t *orthogonalised,
                            int64_t *two_pass_restarts, int64_t *partial_fallbacks) {
  if (!h || !h->impl) return SVT_EINVAL;
  h->impl->reorth_stats(vectors, orthogonalised, two_pass_restarts, partial_fallbacks);
  return SVT_OK;
}

svt_status svt_kernel_stats(const svt_problem *h, int32_t kind, int64_t *launches, double *total_ms,
                            double *total_bytes) {
  if (!h || !h->impl || kind < 0 || kind >= svt::kKinds) return SVT_EINVAL;
  const auto &p = h->impl->prof;
  if (launches) *launches = p.launches[kind];
  if (total_ms) *total_ms = p.ms[kind];
  if (total_bytes) *total_bytes = p.bytes[kind];
  return SVT_OK;
}

}  // extern "C"
