// Internal types of the library shared by its host sources (not part of the
// C ABI): the context and problem objects, a level's host and device data,
// and the host helpers of the solver's control (defined in api.hip).
#pragma once
#include <chrono>
#include <complex>
#include <cstdint>
#include <mutex>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "device.h"
#include "stwr.h"

namespace stwr {
namespace impl {


struct StwrError : std::runtime_error {
  int32_t code;
  StwrError(int32_t c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::stwr::impl::StwrError(e_ == hipErrorOutOfMemory ? STWR_ERR_OOM : STWR_ERR_DEVICE,          \
                      std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}


}  // namespace impl
}  // namespace stwr

struct stwr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t budget = 0;
  uint64_t in_use = 0;
  std::string last_error;
  std::mutex mu;
  // stream-ordered allocation (server workers: no device-wide sync on free)
  bool stream_alloc = false;
  // kernel timing: event pairs recorded around launches of each class
  bool timing = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> marks[3];

  hipEvent_t take_event() {
    if (pool.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  ~stwr_ctx() {
    for (auto& v : marks)
      for (auto& pr : v) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

namespace stwr {
namespace impl {
// RAII bracket of one kernel launch with a pair of events (timing mode only).
struct KernelMark {
  stwr_ctx* c;
  int cls;
  hipEvent_t a = nullptr;
  KernelMark(stwr_ctx* ctx, int k) : c(ctx), cls(k) {
    if (c->timing && (a = c->take_event())) (void)hipEventRecord(a, c->stream);
  }
  ~KernelMark() {
    if (!a) return;
    hipEvent_t b = c->take_event();
    if (!b) { c->pool.push_back(a); return; }
    (void)hipEventRecord(b, c->stream);
    c->marks[cls].push_back({a, b});
  }
};
}  // namespace impl
}  // namespace stwr

namespace stwr {
namespace impl {

// Device allocation owned by a problem.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Level {
  HostLevel H;
  HostTransfer Tr;        // to the next coarser level (valid if not coarsest)
  int N = 0, NQ = 0;
  double dt = 0.0;
  int64_t n_st = 0;
  LevelView view{};
  PatchView pview{};
  int fac_prec = -1;      // precision of the current factors, -1 = none
  int fac_layout = -1;    // precision whose panel layout the (zeroed) storage holds
  size_t fac_budgeted = 0;  // factor bytes already charged to the context
  double lambda = 0.0;
  bool has_lambda = false;
  // time chunks of the sweeps (cyclic reduction in time): buffers for up to
  // chunk_cap chunks, and the autotuner's choice once made
  double* chunk_buf = nullptr;
  int chunk_cap = 0;
  size_t chunk_bytes = 0;
  int chunk_choice = 0;   // 0: not chosen yet
  std::vector<int64_t> fac_off, y_off, mp_off;
  std::vector<int> order;   // host copy of the patch order (pview.order)
  // device arrays
  int *cell_vn = nullptr, *cell_pn = nullptr;   // Taylor-Hood P3-P2 lattice nodes of the cells
  int* color_cells = nullptr;                    // the cells colour by colour (deterministic assembly)
  int *row_ptr = nullptr, *col = nullptr, *cells = nullptr, *cell_p2 = nullptr,
      *cell_dofs = nullptr, *cell_nz = nullptr, *node_free = nullptr, *node_cell_ptr = nullptr,
      *node_cell = nullptr;
  int *patch_ptr = nullptr, *patch_dofs = nullptr, *patch_nbu = nullptr, *patch_nz = nullptr,
      *dof_ptr = nullptr, *dof_slot = nullptr, *slot_patch = nullptr;
  int64_t *patch_nz_off = nullptr, *d_fac_off = nullptr, *d_y_off = nullptr, *d_mp_off = nullptr;
  double *Jv = nullptr, *Mv = nullptr, *Mp = nullptr, *Y = nullptr;
  double* Kv = nullptr;   // heat equation: spatial stiffness values
  void* fac = nullptr;
  size_t fac_bytes = 0;
  int *P_ptr = nullptr, *P_col = nullptr, *R_ptr = nullptr, *R_col = nullptr, *inject = nullptr;
  double *P_val = nullptr, *R_val = nullptr;
  double *r = nullptr, *d = nullptr, *x = nullptr, *b = nullptr;
  float* rf = nullptr;   // FP32 residual of the FP32 interior sweep (inside the factor storage)
  double* Binv = nullptr;   // coarsest only
  double* gbuf = nullptr;   // coarsest only: right-hand side of one slab
  int* perm = nullptr;      // coarsest only: pivot rows of the slab inverses
  double* colbuf = nullptr; // coarsest only: pivot columns of the slab inverses
  double* rbuf = nullptr;   // coarsest only: panel rows for the blocked inverse
  int coarse_mm = 0;
};

}  // namespace impl
}  // namespace stwr

struct stwr_problem {
  stwr_ctx* ctx = nullptr;
  stwr_problem_desc desc{};
  stwr_solver_opts opts{};
  std::vector<int> psi_ab, p_ab;
  std::vector<double> psi_coef, p_coef;
  std::vector<stwr::impl::Level> lv;
  stwr::RefTables tab{};
  stwr::RefTables* d_tab = nullptr;
  stwr::MmsDev mms{};
  double* b0 = nullptr;     // heat equation: right-hand side e0 (x) M U_0 of level 0
  bool heat() const { return desc.equation == STWR_EQ_HEAT; }
  std::vector<stwr::impl::DBuf> bufs;
  uint64_t bytes = 0;
  bool assembled = false;
  // Krylov workspace
  int restart = 0;
  double *V = nullptr, *Z = nullptr;
  double *dscal = nullptr, *partial = nullptr;
  int* dstatus = nullptr;
  int* hstatus_pinned = nullptr;
  // captured V-cycle: its executable graph, the state it was captured for,
  // and its fixed input/output vectors
  hipGraphExec_t vc_exec = nullptr;
  std::vector<double> vc_sig;
  double *vc_in = nullptr, *vc_out = nullptr;
  hipStream_t vc_stream = nullptr;   // capture stream (the context's may be the null stream)

  hipStream_t s() const { return ctx->stream; }

  template <typename T>
  T* alloc(size_t count) {
    if (count == 0) count = 1;
    void* ptr = nullptr;
    hipError_t e = ctx->stream_alloc ? hipMallocAsync(&ptr, count * sizeof(T), ctx->stream)
                                     : hipMalloc(&ptr, count * sizeof(T));
    if (e != hipSuccess) throw stwr::impl::StwrError(STWR_ERR_OOM, "device allocation failed for " + std::to_string(count * sizeof(T)) + " bytes");
    bufs.push_back({ptr, count * sizeof(T)});
    return (T*)ptr;
  }
  // copies on the context's stream and waits, so the host vector may go away
  template <typename T>
  T* upload(const std::vector<T>& v) {
    T* d = alloc<T>(v.size());
    if (!v.empty()) {
      HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return d;
  }
  void free_one(void* ptr) {
    if (ctx->stream_alloc) (void)hipFreeAsync(ptr, ctx->stream);
    else (void)hipFree(ptr);
  }
  void release(void* ptr) {
    for (auto it = bufs.begin(); it != bufs.end(); ++it)
      if (it->p == ptr) {
        free_one(it->p);
        bufs.erase(it);
        return;
      }
  }
};

namespace stwr {
namespace impl {

// ---- helpers defined in api.hip --------------------------------------------
int32_t fail(stwr_ctx* ctx, int32_t code, const std::string& msg);

// Runs f, turning exceptions into a status and the context's last error.
template <typename F>
int32_t guarded(stwr_ctx* ctx, F&& f) {
  try {
    return f();
  } catch (const StwrError& e) {
    return fail(ctx, e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(ctx, STWR_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ctx, STWR_ERR_ARG, e.what());
  }
}

Level& level_at(stwr_problem* P, int l);
void check_status_flag(stwr_problem* P, const char* what);
double dot_host(stwr_problem* P, int64_t n, const double* x, const double* y);
double norm_host(stwr_problem* P, int64_t n, const double* x);
void spmv(stwr_problem* P, int l, const double* x, const double* b, double* y);
void project(stwr_problem* P, int l, double* x);
void ensure_factor_storage(stwr_problem* P, Level& L, int prec);
void set_time_chunks(stwr_problem* P, Level& L, int nc);
void coarse_solve(stwr_problem* P, const double* b, double* x);
void assemble(stwr_problem* P, const double* U);
void residual(stwr_problem* P, const double* U, double* F);
std::vector<std::complex<double>> hessenberg_eigs(std::vector<double> Hr, int m);
double ew_forcing(int k, double f, double f_prev, double eta_prev);
// Newton stops as diverged once ||F|| exceeds this multiple of ||F_0||.
constexpr double kNewtonDiverged = 1e2;

}  // namespace impl
}  // namespace stwr
