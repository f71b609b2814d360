// Continuous-batching server of independent space-time solves, built on the
// public C ABI: FIFO admission by HBM budget, one worker thread and one
// non-blocking HIP stream per slot, so solves of different sizes overlap on
// the device and a finished solve's memory admits the next request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "stwr.h"

namespace {

struct Request {
  int64_t id = 0;
  stwr_problem_desc desc{};
  std::vector<int32_t> psi_ab, p_ab;
  std::vector<double> psi_coef, p_coef;
  stwr_solver_opts opts{};
  double* host_out = nullptr;
  double submit_time = 0.0;
  uint64_t bytes = 0;
  int64_t n_st = 0;
};

double clock_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct stwr_server {
  int device = 0;
  uint64_t budget = 0;
  double t0 = 0.0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> queue;
  std::vector<stwr_result> done;
  uint64_t reserved = 0;
  int active = 0;
  int64_t next_id = 0;
  int64_t submitted = 0, finished = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  double now() const { return clock_s() - t0; }
  void worker(int slot);
};

namespace {

void finish(stwr_server* S, const Request& r, int32_t status, int slot, double t_start, const stwr_stats* st) {
  stwr_result res{};
  res.id = r.id;
  res.status = status;
  res.slot = slot;
  res.submit_time = r.submit_time;
  res.start_time = t_start;
  res.end_time = S->now();
  res.bytes = r.bytes;
  if (st) {
    res.newton_its = st->newton_its;
    res.linear_its = st->linear_its_total;
    res.fnorm_ratio = st->fnorm[0] > 0 ? st->fnorm[st->newton_its] / st->fnorm[0] : 0.0;
  }
  std::lock_guard<std::mutex> g(S->mu);
  S->done.push_back(res);
  S->finished++;
}

}  // namespace

void stwr_server::worker(int slot) {
  (void)hipSetDevice(device);
  hipStream_t stream = nullptr;
  stwr_ctx* ctx = nullptr;
  bool ok = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess &&
            stwr_ctx_create(device, stream, 0, &ctx) == STWR_OK;
  if (ok) stwr_ctx_set_alloc_mode(ctx, 1);
  for (;;) {
    Request r;
    {
      std::unique_lock<std::mutex> lk(mu);
      // FIFO: only the head of the queue may be admitted
      cv.wait(lk, [&] {
        return stop || (!queue.empty() && (budget == 0 || reserved + queue.front().bytes <= budget));
      });
      if (stop) break;
      r = std::move(queue.front());
      queue.pop_front();
      reserved += r.bytes;
      active++;
    }
    const double t_start = now();
    int32_t status = ok ? STWR_OK : STWR_ERR_DEVICE;
    stwr_stats st{};
    stwr_problem* p = nullptr;
    double* U = nullptr;
    if (status == STWR_OK) {
      r.desc.psi_ab = r.psi_ab.data();
      r.desc.psi_coef = r.psi_coef.data();
      r.desc.p_ab = r.p_ab.data();
      r.desc.p_coef = r.p_coef.data();
      status = stwr_problem_create(ctx, &r.desc, &r.opts, &p);
    }
    if (status == STWR_OK) {
      // the solution length the request was sized and budgeted for must be
      // the created problem's (host_out holds that many doubles)
      int64_t n_st = -1;
      if (stwr_problem_sizes(p, 0, &n_st, nullptr, nullptr) != STWR_OK || n_st != r.n_st) status = STWR_ERR_STATE;
    }
    if (status == STWR_OK) {
      if (hipMallocAsync((void**)&U, r.n_st * sizeof(double), stream) != hipSuccess ||
          hipMemsetAsync(U, 0, r.n_st * sizeof(double), stream) != hipSuccess)
        status = STWR_ERR_OOM;
    }
    if (status == STWR_OK) status = stwr_newton_solve(p, U, &st);
    if (U && r.host_out && (status == STWR_OK || status == STWR_ERR_NOT_CONVERGED)) {
      if (hipMemcpyAsync(r.host_out, U, r.n_st * sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess)
        status = STWR_ERR_DEVICE;
    }
    if (U) (void)hipFreeAsync(U, stream);
    if (stream) (void)hipStreamSynchronize(stream);
    if (p) stwr_problem_destroy(p);
    {
      std::lock_guard<std::mutex> g(mu);
      reserved -= r.bytes;
      active--;
    }
    finish(this, r, status, slot, t_start, &st);
    cv.notify_all();
  }
  if (ctx) stwr_ctx_destroy(ctx);
  if (stream) (void)hipStreamDestroy(stream);
}

extern "C" {

int32_t stwr_server_create(int32_t device, int32_t n_slots, uint64_t hbm_budget, stwr_server** out) {
  if (!out || n_slots < 1 || n_slots > 64) return STWR_ERR_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return STWR_ERR_DEVICE;
  auto* S = new stwr_server();
  S->device = device;
  S->budget = hbm_budget;
  S->t0 = clock_s();
  for (int i = 0; i < n_slots; ++i) S->workers.emplace_back([S, i] { S->worker(i); });
  *out = S;
  return STWR_OK;
}

int32_t stwr_server_submit(stwr_server* S, const stwr_problem_desc* desc, const stwr_solver_opts* opts,
                           double* host_out, int64_t* id_out) {
  if (!S || !desc || !opts) return STWR_ERR_ARG;
  Request r;
  r.desc = *desc;
  r.opts = *opts;
  if (desc->n_psi_modes > 0) {
    if (!desc->psi_ab || !desc->psi_coef) return STWR_ERR_ARG;
    r.psi_ab.assign(desc->psi_ab, desc->psi_ab + 2 * desc->n_psi_modes);
    r.psi_coef.assign(desc->psi_coef, desc->psi_coef + 3 * desc->n_psi_modes);
  }
  if (desc->n_p_modes > 0) {
    if (!desc->p_ab || !desc->p_coef) return STWR_ERR_ARG;
    r.p_ab.assign(desc->p_ab, desc->p_ab + 2 * desc->n_p_modes);
    r.p_coef.assign(desc->p_coef, desc->p_coef + 3 * desc->n_p_modes);
  }
  r.desc.psi_ab = r.psi_ab.data();
  r.desc.psi_coef = r.psi_coef.data();
  r.desc.p_ab = r.p_ab.data();
  r.desc.p_coef = r.p_coef.data();
  uint64_t bytes = 0;
  const int32_t rc = stwr_problem_bytes(&r.desc, &r.opts, &bytes);
  if (rc != STWR_OK) return rc;
  const int32_t rn = stwr_problem_n_st(&r.desc, &r.n_st);
  if (rn != STWR_OK) return rn;
  r.bytes = bytes + (uint64_t)r.n_st * 8;
  r.host_out = host_out;
  std::unique_lock<std::mutex> lk(S->mu);
  r.id = S->next_id++;
  r.submit_time = S->now();
  if (id_out) *id_out = r.id;
  S->submitted++;
  if (S->budget && r.bytes > S->budget) {
    stwr_result res{};
    res.id = r.id;
    res.status = STWR_ERR_BUDGET;
    res.slot = -1;
    res.submit_time = res.start_time = res.end_time = r.submit_time;
    res.bytes = r.bytes;
    S->done.push_back(res);
    S->finished++;
    return STWR_OK;
  }
  S->queue.push_back(std::move(r));
  lk.unlock();
  S->cv.notify_all();
  return STWR_OK;
}

int32_t stwr_server_poll(stwr_server* S, stwr_result* results, int32_t max_results, int32_t* n_out) {
  if (!S || !n_out || max_results < 0 || (max_results > 0 && !results)) return STWR_ERR_ARG;
  std::lock_guard<std::mutex> g(S->mu);
  const int n = std::min<int>(max_results, (int)S->done.size());
  for (int i = 0; i < n; ++i) results[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + n);
  *n_out = n;
  return STWR_OK;
}

int32_t stwr_server_wait(stwr_server* S, double timeout_s) {
  if (!S) return STWR_ERR_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  const bool ok = S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                 [&] { return S->finished == S->submitted; });
  return ok ? STWR_OK : STWR_ERR_STATE;
}

int32_t stwr_server_now(const stwr_server* S, double* t) {
  if (!S || !t) return STWR_ERR_ARG;
  *t = S->now();
  return STWR_OK;
}

int32_t stwr_server_destroy(stwr_server* S) {
  if (!S) return STWR_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->queue.clear();
  }
  S->cv.notify_all();
  for (auto& t : S->workers) t.join();
  delete S;
  return STWR_OK;
}

}  // extern "C"
