// Serving form: a request loop that admits completion problems of different
// sizes as device memory and slots free up, and runs the admitted solves
// concurrently on one GPU.
//
// Design:
//   * svt_submit copies the request (Omega, values, parameters) and validates
//     it on the host; nothing touches the device until admission;
//   * admission is first-come first-served: the oldest queued request is
//     admitted when a slot is free and its predicted device footprint fits in
//     the remaining budget (svt_footprint); a request larger than the whole
//     budget is refused at submission;
//   * each slot is a worker thread with its own HIP stream: it creates the
//     problem (index build, upload), solves it, copies the factors back and
//     releases the device memory, so solves admitted at different times
//     overlap on the device and every kernel of one solve stays in its own
//     stream order;
//   * a solve's arithmetic does not depend on what else runs: every
//     reduction has a fixed order and no buffer is shared between solves, so
//     each result is bit-identical alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/svt.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  int64_t m = 0, n = 0, nnz = 0;
  std::vector<int32_t> rows, cols;
  std::vector<double> vals;
  svt_params prm{};
  size_t footprint = 0;
  // outcome
  int state = 0;  // 0 queued, 1 running, 2 done
  svt_status status = SVT_OK;
  svt_info info{};
  std::string error;
  int32_t rank = 0;
  std::vector<double> U, w, V;
  double t_submit = 0, t_start = 0, t_done = 0;
};

// Device bytes of one solve whose bidiagonalisation runs at most kmax steps
// (the handle's step cap: its bases never grow past it, and the rank of X,
// hence the factor width, cannot exceed it).  Counts every buffer a handle
// allocates, with a growing buffer's old and new copies both live.
size_t footprint_bytes(int64_t m, int64_t n, int64_t nnz, int32_t precision, double kmax, bool ds = false,
                       int rsvd_oversample = -1) {
  const double vb = precision == SVT_MIXED ? 4.0 : 8.0;
  const double big = (double)std::max(m, n), small = (double)std::min(m, n);
  const double kcap = std::min(small, kmax);
  const double nblk = std::max(256.0, std::ceil(big / 2048.0));   // reduction partials per column
  const double rank = kcap;                                        // rank bound of X
  double b = 0.0;
  b += 4.0 * (3.0 * (double)nnz + (double)(m + n + 2));    // colidx, rowidx, csr_of_csc, rowptr, colptr
  b += 2.0 * 2.0 * (double)nnz;                            // 16-bit index copies
  b += 4.0 * 9.0 * (double)(m + n);                        // LDS plan segment starts (up to 8 segments)
  b += 4.0 * vb * (double)nnz;                             // M and Y, both orders
  if (ds) b += 2.0 * vb * (double)nnz;                     // the Dantzig selector's two multipliers
  if (rsvd_oversample >= 0)                                // the randomised SVD's two blocks
    b += 2.0 * vb * big * std::min(small, kmax + (double)rsvd_oversample);
  double grow = 0.0;                                       // buffers that grow with the basis
  grow += vb * (big * (kcap + 1) + small * (kcap + 2));    // Lanczos bases
  grow += 8.0 * (kcap + 4) * (4.0 + 2.0 * nblk + 1.0) + 8.0 * nblk;  // coefficients and partials
  b += 2.0 * grow;                                         // old and new copies during growth
  b += vb * (big + small);                                 // working vectors
  b += vb * (double)(m + n) * (rank + 16.0 / vb) * 1.0;    // factors (row stride padded to 16 bytes)
  b += 2.0 * 8.0 * (2.0 * kcap * rank + rank);             // Ritz combination matrices
  b += 8.0 * (1024 + 8);                                   // residual partials
  return (size_t)(b * 1.05) + (1u << 20);                  // margin for allocation granularity
}

// Without a step cap in the parameters, a request runs (and is admitted) with
// 512 steps: about 3.5 steps per singular value above tau are typical, so
// ranks up to ~140.
constexpr double kDefaultStepCap = 512.0;

double request_cap(const svt_params &p) {
  return p.lanczos_maxsteps > 0 ? (double)p.lanczos_maxsteps : kDefaultStepCap;
}

// A served request that leaves stall_window 0 stops once 20 consecutive
// iterations set no new minimum of its residual (SVT_STALLED): requests
// outside the method's regime oscillate for hundreds of iterations and
// would otherwise hold a slot up to maxiter; converging runs set a new
// minimum at every iteration.  A negative window turns the bound off.
constexpr int32_t kDefaultStallWindow = 20;

int32_t request_stall(const svt_params &p) {
  return p.stall_window == 0 ? kDefaultStallWindow : p.stall_window;
}

// A served request that leaves dof_bound 0 stops once its iterate's rank has
// more degrees of freedom than it has observations (SVT_UNDERDETERMINED):
// requests that far outside the method's regime would otherwise grow their
// bidiagonalisations to the step cap.  A negative value turns it off.
constexpr double kDefaultDofBound = 1.0;

double request_dof(const svt_params &p) {
  return p.dof_bound == 0.0 ? kDefaultDofBound : (p.dof_bound < 0.0 ? 0.0 : p.dof_bound);
}

// A served request that leaves min_block_rows 0 cuts its vectors into row
// blocks of at least 64 rows: a request of a few thousand rows then runs its
// half-steps on a few dozen compute units instead of all of them, so that
// the solves of other slots find free units (a block of 64 rows still
// takes one workgroup pass).
constexpr int32_t kServedMinBlockRows = 64;

int32_t request_min_rows(const svt_params &p) {
  return p.min_block_rows == 0 ? kServedMinBlockRows : p.min_block_rows;
}


}  // namespace

struct svt_server {
  size_t budget = 0, in_use = 0, peak = 0;
  int slots = 0;
  int device = 0;
  bool stopping = false;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<std::thread> workers;
  int running = 0, max_running = 0;

  void worker() {
    (void)hipSetDevice(device);
    hipStream_t stream = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
      Request *r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          return stopping || (!queue.empty() && in_use + reqs[queue.front()]->footprint <= budget);
        });
        if (queue.empty() || in_use + reqs[queue.front()]->footprint > budget) {
          if (stopping) break;
          continue;
        }
        r = reqs[queue.front()].get();
        queue.pop_front();
        in_use += r->footprint;
        peak = std::max(peak, in_use);
        r->state = 1;
        r->t_start = now_s();
        running += 1;
        max_running = std::max(max_running, running);
      }
      run(r, have_stream ? stream : nullptr);
      {
        std::lock_guard<std::mutex> lk(mu);
        in_use -= r->footprint;
        running -= 1;
        r->state = 2;
        r->t_done = now_s();
        r->rows.clear(); r->rows.shrink_to_fit();
        r->cols.clear(); r->cols.shrink_to_fit();
        r->vals.clear(); r->vals.shrink_to_fit();
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (have_stream) (void)hipStreamDestroy(stream);
  }

  void run(Request *r, hipStream_t stream) {
    svt_params p = r->prm;
    p.stream = stream;  // the slot's own stream (library-owned when null)
    // the step cap the admission footprint assumed
    p.lanczos_maxsteps = (int32_t)request_cap(p);
    p.stall_window = request_stall(p);
    p.dof_bound = request_dof(p);
    p.min_block_rows = request_min_rows(p);
    svt_problem *h = nullptr;
    svt_status st = svt_create(r->m, r->n, r->nnz, SVT_COO, r->rows.data(), r->cols.data(), r->vals.data(), &p, &h);
    if (st != SVT_OK) {
      r->status = st;
      r->error = svt_last_error(nullptr);
      return;
    }
    st = svt_solve(h, &r->info);
    r->status = st;
    if (st == SVT_OK || st == SVT_NOT_CONVERGED || st == SVT_STALLED || st == SVT_UNDERDETERMINED) {
      int32_t rank = 0;
      svt_factors(h, &rank, nullptr, nullptr, nullptr);
      r->rank = rank;
      r->U.resize((size_t)r->m * rank);
      r->V.resize((size_t)r->n * rank);
      r->w.resize(rank);
      if (rank > 0) {
        const svt_status sf = svt_factors(h, &rank, r->U.data(), r->w.data(), r->V.data());
        if (sf != SVT_OK) r->status = sf;
      }
    } else {
      r->error = svt_last_error(h);
    }
    svt_destroy(h);
  }
};


extern "C" {

svt_status svt_footprint(int64_t m, int64_t n, int64_t nnz, int32_t precision, size_t *bytes) {
  if (!bytes || m < 1 || n < 1 || nnz < 1) return SVT_EINVAL;
  *bytes = footprint_bytes(m, n, nnz, precision, kDefaultStepCap);
  return SVT_OK;
}

svt_status svt_server_create(size_t hbm_budget_bytes, int32_t max_slots, svt_server **out) {
  if (!out || hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 64) return SVT_EINVAL;
  *out = nullptr;
  try {
    auto s = std::make_unique<svt_server>();
    s->budget = hbm_budget_bytes;
    s->slots = max_slots;
    if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
    for (int i = 0; i < max_slots; ++i) s->workers.emplace_back([p = s.get()] { p->worker(); });
    *out = s.release();
    return SVT_OK;
  } catch (...) {
    return SVT_ENOMEM;
  }
}

svt_status svt_submit(svt_server *s, int64_t m, int64_t n, int64_t nnz, const int32_t *rows, const int32_t *cols,
                      const double *vals, const svt_params *params, uint64_t *ticket) {
  if (!s || !ticket || !rows || !cols || !vals || m < 1 || n < 1 || nnz < 1) return SVT_EINVAL;
  if ((double)nnz > (double)m * (double)n || nnz > INT32_MAX) return SVT_EINVAL;
  for (int64_t t = 0; t < nnz; ++t)
    if (rows[t] < 0 || rows[t] >= m || cols[t] < 0 || cols[t] >= n || !std::isfinite(vals[t])) return SVT_EINVAL;
  auto r = std::make_unique<Request>();
  r->m = m; r->n = n; r->nnz = nnz;
  if (params) r->prm = *params;
  else svt_params_default(m, n, nnz, &r->prm);
  r->footprint = footprint_bytes(m, n, nnz, r->prm.precision, request_cap(r->prm),
                                 r->prm.constraint == SVT_CONSTRAINT_INEQUALITY,
                                 r->prm.svd_method == SVT_SVD_RANDOMIZED ? r->prm.rsvd_oversample : -1);
  r->rows.assign(rows, rows + nnz);
  r->cols.assign(cols, cols + nnz);
  r->vals.assign(vals, vals + nnz);
  std::lock_guard<std::mutex> lk(s->mu);
  if (r->footprint > s->budget) return SVT_ENOMEM;  // could never be admitted
  r->ticket = s->next_ticket++;
  r->t_submit = now_s();
  *ticket = r->ticket;
  s->queue.push_back(r->ticket);
  s->reqs[r->ticket] = std::move(r);
  s->cv_work.notify_all();
  return SVT_OK;
}

svt_status svt_poll(svt_server *s, uint64_t ticket, int32_t *state) {
  if (!s || !state) return SVT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return SVT_EINVAL;
  *state = it->second->state;
  return SVT_OK;
}

svt_status svt_wait(svt_server *s, uint64_t ticket, svt_info *info) {
  if (!s) return SVT_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return SVT_EINVAL;
  Request *r = it->second.get();
  s->cv_done.wait(lk, [&] { return r->state == 2; });
  if (info) *info = r->info;
  return r->status;
}

svt_status svt_result(svt_server *s, uint64_t ticket, int32_t *rank_out, double *U, double *w, double *V,
                      double *times) {
  if (!s) return SVT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return SVT_EINVAL;
  Request *r = it->second.get();
  if (r->state != 2) return SVT_EBUSY;
  if (rank_out) *rank_out = r->rank;
  if (U) std::copy(r->U.begin(), r->U.end(), U);
  if (w) std::copy(r->w.begin(), r->w.end(), w);
  if (V) std::copy(r->V.begin(), r->V.end(), V);
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_start;
    times[2] = r->t_done;
  }
  return r->status;
}

svt_status svt_release(svt_server *s, uint64_t ticket) {
  if (!s) return SVT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return SVT_EINVAL;
  if (it->second->state != 2) return SVT_EBUSY;
  s->reqs.erase(it);
  return SVT_OK;
}

svt_status svt_server_stats(svt_server *s, size_t *peak_bytes, int32_t *max_running, int32_t *queued) {
  if (!s) return SVT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (peak_bytes) *peak_bytes = s->peak;
  if (max_running) *max_running = s->max_running;
  if (queued) *queued = (int32_t)s->queue.size();
  return SVT_OK;
}

svt_status svt_server_destroy(svt_server *s) {
  if (!s) return SVT_OK;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // let queued work finish: wait until nothing is queued or running
    s->cv_done.wait(lk, [&] { return s->queue.empty() && s->running == 0; });
    s->stopping = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->workers) t.join();
  delete s;
  return SVT_OK;
}

}  // extern "C"
