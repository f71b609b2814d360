// Batched solves (the C ABI's stwr_batch_*): many independent space-time
// Navier-Stokes problems advanced together, one Newton-FGMRES-WRMG solve
// each (Secs. 3 and 4.2, Alg. 1), with their patch work in shared launches.
//
// The patch systems are independent across patches (eq.
// waveform_patch_solve), and so across problems: every relaxation sweep of
// the batch covers the patches of every problem at that multigrid depth in
// one persistent launch per temporal-node count, and every patch
// factorization covers all levels of all problems in one persistent launch
// per block class.  Launch tiles (patches per grab for the sweep, blocks per
// grab for the factorization) are chosen per block-size class by timing the
// candidates on the batch itself.  The rest of each solve (operator
// applications, transfers, coarsest solves, Krylov vectors) runs per problem
// on the batch's stream, in lock step: one stwr_batch_step is one FGMRES
// iteration of every problem in its Krylov phase, with one V-cycle launch
// sequence (captured into a HIP graph and replayed while the set of problems
// in that phase is unchanged) and one host synchronisation for all of them,
// plus the Newton bookkeeping, assembly, factorization and eigen-estimates of
// the problems at the start of a Newton step.  Every problem runs exactly
// the operations of stwr_newton_solve with FP32 smoothers and the plain
// sweep in time, in the same order, so its result is the one it has alone.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <numeric>
#include <vector>

#include "problem.h"

using namespace stwr;
using namespace stwr::impl;

namespace {

// A device array owned by the batch, grown on demand, with the host copy it
// was uploaded from (kept until the next upload).
template <typename T>
struct DevArray {
  T* d = nullptr;
  size_t cap = 0;
  std::vector<T> h;
  DevArray() = default;
  DevArray(const DevArray&) = delete;
  DevArray& operator=(const DevArray&) = delete;
  ~DevArray() { release(); }
  void upload(hipStream_t s) {
    if (h.size() > cap) {
      HIPCHK(hipStreamSynchronize(s));
      if (d) HIPCHK(hipFree(d));
      d = nullptr;
      cap = std::max<size_t>(h.size(), 2 * cap);
      HIPCHK(hipMalloc(&d, cap * sizeof(T)));
    }
    if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void release() {
    if (d) (void)hipFree(d);
    d = nullptr;
    cap = 0;
  }
};

enum Phase { kSetup = 0, kKrylov = 1, kDone = 2 };

// One problem of the batch and the state of its Newton and FGMRES iterations.
struct Item {
  int64_t id = 0;
  stwr_problem* P = nullptr;
  double* U = nullptr;          // current iterate (device, n_st(0))
  double* host_out = nullptr;   // caller's buffer for the solution, or null
  uint64_t bytes = 0;           // device bytes charged to the context
  Phase phase = kSetup;
  int status = STWR_OK;
  stwr_stats st{};
  int k = 0;                    // Newton steps taken
  double f0 = 0.0, eta = 0.0;
  // linear solve of the current Newton step: A dU = b with b = -F in L0.b,
  // dU in L0.x
  double bnorm = 0.0, target = 0.0;
  int its = 0, j = 0;
  std::vector<double> H, cs, sn, g, y;
  double submit_time = 0.0, start_time = 0.0;
  int slot = 0;                 // row of the pinned readback buffer this step
  int levels() const { return (int)P->lv.size(); }
};

}  // namespace

namespace stwr {
namespace impl {

// A batched FP32 sweep: one job per (problem, level), the tiles of each
// temporal-node class (interior-patch tiles first, each part by decreasing
// work) and the persistent grid of each class.
struct SweepPlan {
  DevArray<SweepJob> jobs;
  DevArray<SweepTile> tiles;
  int off[2] = {0, 0}, n[2] = {0, 0}, nfull[2] = {0, 0}, grid[2] = {0, 0};
  std::vector<std::pair<stwr_problem*, int>> who;   // (problem, level) of each job
};

}  // namespace impl
}  // namespace stwr

struct stwr_batch {
  stwr_ctx* ctx = nullptr;
  int use_graph = 1;
  int64_t next_id = 1;
  std::vector<std::unique_ptr<Item>> items;
  std::deque<stwr_result> done;
  int nu_pre = -1, nu_post = -1;
  int n_cu = 0;
  // launch tiles per class (0: not tuned yet) and occupancies
  int sweep_tile[2] = {0, 0};
  int factor_tile[kFacClasses] = {0, 0, 0};
  int sweep_occ[2] = {1, 1};
  int factor_occ[kFacClasses] = {1, 1, 1};
  int* ctr = nullptr;            // counter pairs: [0..3] sweeps (per class), [4..9] factor classes
  double* pinned = nullptr;      // readback rows of 512 doubles
  int pinned_rows = 0;
  // V-cycle: per-depth plans and the captured graph, for the problems in
  // their Krylov phase identified by (id, Newton step)
  std::vector<std::unique_ptr<SweepPlan>> vc_plans;
  std::vector<int64_t> vc_key;
  hipGraphExec_t vc_exec = nullptr;
  hipStream_t cap = nullptr;
  SweepPlan eig_plan;
  DevArray<FactorJob> fjobs;
  DevArray<FactorTile> ftiles;
  // counters reported by stwr_batch_info
  int64_t n_steps = 0, n_captures = 0, n_vcycles = 0, n_sweep_launches = 0, n_factor_launches = 0;
  double t_origin = 0.0;
  double now() const { return now_s() - t_origin; }
};

namespace {

constexpr int kReadRow = 512;     // doubles per problem in the pinned readback buffer
const int kSweepTiles[] = {1, 2, 4};
const int kFactorTiles[] = {4, 16, 64};

hipStream_t bs(stwr_batch* B) { return B->ctx->stream; }

void ensure_pinned(stwr_batch* B, int rows) {
  if (rows <= B->pinned_rows) return;
  HIPCHK(hipStreamSynchronize(bs(B)));
  if (B->pinned) HIPCHK(hipHostFree(B->pinned));
  B->pinned = nullptr;
  const int n = std::max(rows, 2 * B->pinned_rows);
  HIPCHK(hipHostMalloc((void**)&B->pinned, (size_t)n * kReadRow * sizeof(double), hipHostMallocDefault));
  B->pinned_rows = n;
}

double* row_of(stwr_batch* B, const Item& it) { return B->pinned + (size_t)it.slot * kReadRow; }

// ---- batched sweeps -----------------------------------------------------------

// Work of one patch sweep: N slabs of an m x m block, m = (q+1) nb.
double patch_work(const Level& L, int pos) {
  const int v = L.order[pos];
  const double m = (double)(L.H.patch_ptr[v + 1] - L.H.patch_ptr[v]) * L.NQ;
  return (double)L.N * m * m;
}

// Tiles of every job of class c into t (interior tiles first, then the
// others, each part by decreasing work); returns the interior-tile count.
int build_sweep_tiles(const SweepPlan& plan, const std::vector<SweepJob>& jobs, int c, int tile,
                      std::vector<SweepTile>& t) {
  struct W {
    SweepTile tl;
    double w;
  };
  std::vector<W> full, rest;
  for (int j = 0; j < (int)jobs.size(); ++j) {
    if (jobs[j].L.NQ != c + 1) continue;
    const Level& L = plan.who[j].first->lv[plan.who[j].second];
    const int nf = jobs[j].P.n_full, np = jobs[j].P.n_patch;
    for (int a = 0; a < nf; a += tile) {
      const int cnt = std::min(tile, nf - a);
      full.push_back({{j, a, cnt}, patch_work(L, a) * cnt});
    }
    for (int a = nf; a < np; a += tile) {
      const int cnt = std::min(tile, np - a);
      double w = 0.0;
      for (int q = a; q < a + cnt; ++q) w += patch_work(L, q);
      rest.push_back({{j, a, cnt}, w});
    }
  }
  auto by_work = [](const W& x, const W& y) { return x.w > y.w; };
  std::stable_sort(full.begin(), full.end(), by_work);
  std::stable_sort(rest.begin(), rest.end(), by_work);
  t.clear();
  for (auto& x : full) t.push_back(x.tl);
  for (auto& x : rest) t.push_back(x.tl);
  return (int)full.size();
}

void upload_sweep_tiles(stwr_batch* B, SweepPlan& plan) {
  plan.tiles.h.clear();
  for (int c = 0; c < 2; ++c) {
    std::vector<SweepTile> t;
    plan.nfull[c] = build_sweep_tiles(plan, plan.jobs.h, c, B->sweep_tile[c] > 0 ? B->sweep_tile[c] : 1, t);
    plan.off[c] = (int)plan.tiles.h.size();
    plan.n[c] = (int)t.size();
    plan.grid[c] = std::max(1, std::min(plan.n[c], B->sweep_occ[c] * B->n_cu));
    plan.tiles.h.insert(plan.tiles.h.end(), t.begin(), t.end());
  }
  plan.tiles.upload(bs(B));
}

void launch_sweep_plan(stwr_batch* B, SweepPlan& plan) {
  for (int c = 0; c < 2; ++c) {
    if (!plan.n[c]) continue;
    HIPCHK(launch_patch_sweep_batch(c + 1, plan.jobs.d, plan.tiles.d + plan.off[c], plan.nfull[c], plan.n[c],
                                    plan.grid[c], B->ctr + 2 * c, bs(B)));
    ++B->n_sweep_launches;
  }
}

// Times the candidate tiles of every class present in the plan (three sweeps
// each, HIP events) and keeps the fastest; once per batch.
void tune_sweep_tiles(stwr_batch* B, SweepPlan& plan) {
  for (int c = 0; c < 2; ++c) {
    if (B->sweep_tile[c] > 0) continue;
    bool present = false;
    for (auto& j : plan.jobs.h) present |= j.L.NQ == c + 1;
    if (!present) continue;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best_ms = 0.0f;
    int best = kSweepTiles[0];
    for (int tile : kSweepTiles) {
      B->sweep_tile[c] = tile;
      upload_sweep_tiles(B, plan);
      HIPCHK(launch_patch_sweep_batch(c + 1, plan.jobs.d, plan.tiles.d + plan.off[c], plan.nfull[c], plan.n[c],
                                      plan.grid[c], B->ctr + 2 * c, bs(B)));
      HIPCHK(hipEventRecord(e0, bs(B)));
      for (int r = 0; r < 3; ++r)
        HIPCHK(launch_patch_sweep_batch(c + 1, plan.jobs.d, plan.tiles.d + plan.off[c], plan.nfull[c],
                                        plan.n[c], plan.grid[c], B->ctr + 2 * c, bs(B)));
      HIPCHK(hipEventRecord(e1, bs(B)));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (tile == kSweepTiles[0] || ms < 0.97f * best_ms) {
        best = tile;
        best_ms = ms;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    B->sweep_tile[c] = best;
  }
  upload_sweep_tiles(B, plan);
}

// Plan of one batched sweep over (problem, level) pairs: residual L.r in,
// FP32 patch outputs L.Y out.
void build_sweep_plan(stwr_batch* B, SweepPlan& plan, const std::vector<std::pair<stwr_problem*, int>>& who) {
  plan.who = who;
  plan.jobs.h.clear();
  for (auto& w : who) {
    stwr_problem* P = w.first;
    Level& L = P->lv[w.second];
    SweepJob j{};
    j.L = L.view;
    j.P = L.pview;
    j.fac = (const float*)L.fac;
    j.Mp = L.Mp;
    j.r = L.r;
    j.Y = (float*)L.Y;
    j.e00 = P->tab.e0[0];
    j.e01 = L.NQ > 1 ? P->tab.e0[1] : 0.0;
    j.e10 = P->tab.e1[0];
    j.e11 = L.NQ > 1 ? P->tab.e1[1] : 0.0;
    plan.jobs.h.push_back(j);
  }
  plan.jobs.upload(bs(B));
  tune_sweep_tiles(B, plan);
  HIPCHK(hipStreamSynchronize(bs(B)));
}

// ---- batched factorization -------------------------------------------------------

void factor_tiles(stwr_batch* B, int cls, int tile, std::vector<FactorTile>& t, std::vector<double>& w) {
  t.clear();
  w.clear();
  for (int j = 0; j < (int)B->fjobs.h.size(); ++j) {
    const FactorJob& J = B->fjobs.h[j];
    const int nq = J.L.NQ, ns = J.P.fac_slabs;
    int a = 0, b = 0;   // class positions [a, b)
    if (cls == kFacSmall1) {
      if (nq != 1) continue;
      a = 0, b = J.P.n_patch;
    } else if (cls == kFacSmall2) {
      if (nq != 2) continue;
      a = J.P.n_big, b = J.P.n_patch;
    } else {
      if (nq != 2) continue;
      a = 0, b = J.P.n_big;
    }
    const int64_t first = (int64_t)a * ns, last = (int64_t)b * ns;
    for (int64_t x = first; x < last; x += tile) {
      const int cnt = (int)std::min<int64_t>(tile, last - x);
      t.push_back({j, (int)x, cnt});
      w.push_back(cnt);
    }
  }
}

void launch_factor_class(stwr_batch* B, int cls, const std::vector<FactorTile>& t, int off) {
  if (t.empty()) return;
  const int grid = std::max(1, std::min((int)t.size(), B->factor_occ[cls] * B->n_cu));
  HIPCHK(launch_patch_factor_batch(cls, B->fjobs.d, B->ftiles.d + off, (int)t.size(), grid, B->ctr + 4 + 2 * cls,
                                   bs(B)));
  ++B->n_factor_launches;
}

// Factor every smoothed level of the given problems in FP32: one persistent
// launch per block class; the tiles of a class not tuned yet are timed first
// (each candidate factors the same blocks, so the last pass leaves the
// factors in place).
void factor_batch(stwr_batch* B, const std::vector<Item*>& S) {
  B->fjobs.h.clear();
  for (Item* it : S) {
    stwr_problem* P = it->P;
    for (int l = 0; l + 1 < it->levels(); ++l) {
      Level& L = P->lv[l];
      ensure_factor_storage(P, L, STWR_FP32);
      L.pview.factor_mfma = 1;
      L.pview.time_chunks = 1;
      L.pview.chunk_len = L.N;
      B->fjobs.h.push_back({L.view, L.pview, L.Jv, (float*)L.fac, P->dstatus});
    }
  }
  B->fjobs.upload(bs(B));
  for (int cls = 0; cls < kFacClasses; ++cls) {
    std::vector<FactorTile> t;
    std::vector<double> w;
    if (B->factor_tile[cls] == 0) {
      factor_tiles(B, cls, kFactorTiles[0], t, w);
      if (t.empty()) continue;
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      float best_ms = 0.0f;
      int best = kFactorTiles[0];
      for (int tile : kFactorTiles) {
        factor_tiles(B, cls, tile, t, w);
        B->ftiles.h = t;
        B->ftiles.upload(bs(B));
        HIPCHK(hipEventRecord(e0, bs(B)));
        launch_factor_class(B, cls, t, 0);
        HIPCHK(hipEventRecord(e1, bs(B)));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (tile == kFactorTiles[0] || ms < 0.97f * best_ms) {
          best = tile;
          best_ms = ms;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      B->factor_tile[cls] = best;
      if (best == kFactorTiles[sizeof(kFactorTiles) / sizeof(int) - 1]) continue;   // last pass used it
    }
    factor_tiles(B, cls, B->factor_tile[cls], t, w);
    if (t.empty()) continue;
    HIPCHK(hipStreamSynchronize(bs(B)));   // the tile array is rewritten
    B->ftiles.h = t;
    B->ftiles.upload(bs(B));
    launch_factor_class(B, cls, t, 0);
  }
  for (Item* it : S) {
    stwr_problem* P = it->P;
    for (int l = 0; l + 1 < it->levels(); ++l) {
      Level& L = P->lv[l];
      HIPCHK(launch_patch_mass(L.view, L.pview, L.Mv, L.Mp, bs(B)));
      L.fac_prec = STWR_FP32;
      L.has_lambda = false;
    }
  }
  HIPCHK(hipStreamSynchronize(bs(B)));
}

// ---- batched eigen-estimates -------------------------------------------------------

// lambda of every smoothed level of the given problems: the Arnoldi process
// of eig_estimate on M^{-1} A_l, all (problem, level) pairs in lock step, the
// patch applications of a step in one batched sweep and one synchronisation
// per step.  Level l of a problem keeps its basis in the problem's Krylov
// space at an offset of its own and its scalars at dscal + l (steps + 2).
void eig_batch(stwr_batch* B, const std::vector<Item*>& S) {
  struct Pair {
    Item* it;
    int l;
    int64_t n, off;
    int steps, m;
    bool live;
    std::vector<double> H;
  };
  std::vector<Pair> pairs;
  for (Item* it : S) {
    int64_t off = 0;
    for (int l = 0; l + 1 < it->levels(); ++l) {
      const Level& L = it->P->lv[l];
      const int steps = it->P->opts.eig_steps;
      pairs.push_back({it, l, L.n_st, off, steps, steps, true, std::vector<double>((steps + 1) * steps, 0.0)});
      off += (int64_t)(steps + 1) * L.n_st;
    }
  }
  auto vec = [](Pair& p, int j) { return p.it->P->V + p.off + (int64_t)j * p.n; };
  auto scal = [](Pair& p) { return p.it->P->dscal + p.l * (p.steps + 2); };
  // start vectors and their norms
  for (auto& p : pairs) {
    HIPCHK(launch_start_vector(p.n, vec(p, 0), bs(B)));
    HIPCHK(launch_mdot(p.n, 1, vec(p, 0), 0, vec(p, 0), p.it->P->partial, scal(p), bs(B)));
  }
  int slot = 0;
  ensure_pinned(B, (int)pairs.size());
  std::vector<int> row(pairs.size());
  for (size_t i = 0; i < pairs.size(); ++i) {
    row[i] = slot++;
    HIPCHK(hipMemcpyAsync(B->pinned + (size_t)row[i] * kReadRow, scal(pairs[i]), 8, hipMemcpyDeviceToHost, bs(B)));
  }
  HIPCHK(hipStreamSynchronize(bs(B)));
  for (size_t i = 0; i < pairs.size(); ++i) {
    const double nv0 = std::sqrt(B->pinned[(size_t)row[i] * kReadRow]);
    if (!std::isfinite(nv0)) throw StwrError(STWR_ERR_NONFINITE, "non-finite norm");
    HIPCHK(launch_axpby(pairs[i].n, 1.0 / nv0, vec(pairs[i], 0), 0.0, vec(pairs[i], 0), bs(B)));
  }
  const int max_steps = pairs.empty() ? 0 : std::max_element(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) {
                                              return a.steps < b.steps;
                                            })->steps;
  std::vector<std::pair<stwr_problem*, int>> who_prev;
  for (int j = 0; j < max_steps; ++j) {
    std::vector<std::pair<stwr_problem*, int>> who;
    for (auto& p : pairs)
      if (p.live && j < p.steps) who.push_back({p.it->P, p.l});
    if (who.empty()) break;
    if (who != who_prev) {
      build_sweep_plan(B, B->eig_plan, who);
      who_prev = who;
    }
    for (auto& p : pairs)
      if (p.live && j < p.steps) spmv(p.it->P, p.l, vec(p, j), nullptr, p.it->P->lv[p.l].r);
    launch_sweep_plan(B, B->eig_plan);
    for (auto& p : pairs) {
      if (!(p.live && j < p.steps)) continue;
      stwr_problem* P = p.it->P;
      Level& L = P->lv[p.l];
      double* w = vec(p, j + 1);
      HIPCHK(launch_patch_gather(L.view, L.pview, STWR_FP32, L.Y, 0, 0.0, 0.0, w, nullptr, nullptr, bs(B)));
      for (int i = 0; i <= j; ++i) {
        HIPCHK(launch_mdot(p.n, 1, vec(p, i), 0, w, P->partial, scal(p) + i, bs(B)));
        HIPCHK(launch_axpy_dev(p.n, scal(p) + i, -1.0, vec(p, i), w, bs(B)));
      }
      HIPCHK(launch_mdot(p.n, 1, w, 0, w, P->partial, scal(p) + j + 1, bs(B)));
    }
    for (size_t i = 0; i < pairs.size(); ++i) {
      Pair& p = pairs[i];
      if (!(p.live && j < p.steps)) continue;
      HIPCHK(hipMemcpyAsync(B->pinned + (size_t)row[i] * kReadRow, scal(p), (j + 2) * 8, hipMemcpyDeviceToHost,
                            bs(B)));
    }
    HIPCHK(hipStreamSynchronize(bs(B)));
    for (size_t i = 0; i < pairs.size(); ++i) {
      Pair& p = pairs[i];
      if (!(p.live && j < p.steps)) continue;
      const double* hcol = B->pinned + (size_t)row[i] * kReadRow;
      for (int r = 0; r <= j; ++r) p.H[r * p.steps + j] = hcol[r];
      const double h = std::sqrt(hcol[j + 1]);
      if (!std::isfinite(h)) throw StwrError(STWR_ERR_NONFINITE, "eigen-estimate produced a non-finite value");
      p.H[(j + 1) * p.steps + j] = h;
      if (h <= 1e-14 * std::fabs(p.H[0])) {
        p.m = j + 1;
        p.live = false;
        continue;
      }
      HIPCHK(launch_axpby(p.n, 1.0 / h, vec(p, j + 1), 0.0, vec(p, j + 1), bs(B)));
    }
  }
  for (auto& p : pairs) {
    std::vector<double> Hm(p.m * p.m);
    for (int i = 0; i < p.m; ++i)
      for (int c = 0; c < p.m; ++c) Hm[i * p.m + c] = p.H[i * p.steps + c];
    auto ev = hessenberg_eigs(Hm, p.m);
    double lam = -1e300;
    for (auto& e : ev) lam = std::max(lam, e.real());
    Level& L = p.it->P->lv[p.l];
    L.lambda = lam;
    L.has_lambda = true;
  }
}

// ---- batched V-cycle ----------------------------------------------------------------

const double* vb(Item* it, int d) { return d == 0 ? it->P->vc_in : it->P->lv[d].b; }
double* vx(Item* it, int d) { return d == 0 ? it->P->vc_out : it->P->lv[d].x; }

// Chebyshev-accelerated relaxation (the recurrence of relax()) of depth d for
// every problem of S, the sweeps of a step in one batched launch.
void relax_batch(stwr_batch* B, const std::vector<Item*>& S, int d, SweepPlan& plan, int n_steps, bool x_is_zero) {
  std::vector<double> rho_old(S.size(), 0.0);
  for (int k = 0; k < n_steps; ++k) {
    for (Item* it : S) {
      Level& L = it->P->lv[d];
      if (k == 0 && x_is_zero) HIPCHK(hipMemcpyAsync(L.r, vb(it, d), L.n_st * 8, hipMemcpyDeviceToDevice, bs(B)));
      else spmv(it->P, d, vx(it, d), vb(it, d), L.r);
    }
    launch_sweep_plan(B, plan);
    for (size_t i = 0; i < S.size(); ++i) {
      Item* it = S[i];
      stwr_problem* P = it->P;
      Level& L = P->lv[d];
      const double a = P->opts.cheb_lo * L.lambda, bnd = P->opts.cheb_hi * L.lambda;
      const double theta = 0.5 * (a + bnd), delta = 0.5 * (bnd - a);
      double c1, c2, rho;
      if (k == 0) {
        rho = delta / theta;
        c1 = 0.0;
        c2 = 1.0 / theta;
      } else {
        rho = 1.0 / (2.0 * theta / delta - rho_old[i]);
        c1 = rho * rho_old[i];
        c2 = 2.0 * rho / delta;
      }
      HIPCHK(launch_patch_gather(L.view, L.pview, STWR_FP32, L.Y, 1, c1, c2, nullptr, L.d, vx(it, d), bs(B)));
      rho_old[i] = rho;
    }
  }
}

// One V-cycle of Alg. 1 for every problem of K (vc_in -> vc_out), depth by
// depth, with the sweeps of all problems at a depth in shared launches.
void vcycle_batch(stwr_batch* B, const std::vector<Item*>& K) {
  int maxL = 0;
  for (Item* it : K) maxL = std::max(maxL, it->levels());
  for (int d = 0; d < maxL; ++d) {
    std::vector<Item*> S, C;
    for (Item* it : K) {
      if (d < it->levels() - 1) S.push_back(it);
      else if (d == it->levels() - 1) C.push_back(it);
    }
    if (!S.empty()) {
      for (Item* it : S) HIPCHK(launch_fill(it->P->lv[d].n_st, 0.0, vx(it, d), bs(B)));
      relax_batch(B, S, d, *B->vc_plans[d], B->nu_pre, true);
      for (Item* it : S) {
        Level& Lv = it->P->lv[d];
        Level& Cv = it->P->lv[d + 1];
        spmv(it->P, d, vx(it, d), vb(it, d), Lv.r);
        HIPCHK(launch_transfer(Cv.H.nf, Cv.N * Cv.NQ, Lv.R_ptr, Lv.R_col, Lv.R_val, Lv.r, Cv.b, 0, bs(B)));
      }
    }
    for (Item* it : C) coarse_solve(it->P, vb(it, d), vx(it, d));
  }
  for (int d = maxL - 2; d >= 0; --d) {
    std::vector<Item*> S;
    for (Item* it : K)
      if (d < it->levels() - 1) S.push_back(it);
    if (S.empty()) continue;
    for (Item* it : S) {
      Level& Lv = it->P->lv[d];
      HIPCHK(launch_transfer(Lv.H.nf, Lv.N * Lv.NQ, Lv.P_ptr, Lv.P_col, Lv.P_val, vx(it, d + 1), vx(it, d), 1,
                             bs(B)));
    }
    relax_batch(B, S, d, *B->vc_plans[d], B->nu_post, false);
  }
  ++B->n_vcycles;
}

void drop_graph(stwr_batch* B) {
  if (B->vc_exec) (void)hipGraphExecDestroy(B->vc_exec);
  B->vc_exec = nullptr;
}

// The V-cycles of K.  The plans are rebuilt whenever K or a member's Newton
// step changes; with graphs, the launch sequence is captured once the same
// K has come back on the next step (a set that changes every step runs its
// launches directly rather than paying a capture it would use once).
void vcycles(stwr_batch* B, const std::vector<Item*>& K) {
  std::vector<int64_t> key;
  for (Item* it : K) {
    key.push_back(it->id);
    key.push_back(it->k);
  }
  if (key != B->vc_key || B->vc_plans.empty()) {
    drop_graph(B);
    int maxL = 0;
    for (Item* it : K) maxL = std::max(maxL, it->levels());
    HIPCHK(hipStreamSynchronize(bs(B)));   // no launch still reads the old plans
    B->vc_plans.clear();
    for (int d = 0; d + 1 < maxL; ++d) {
      std::vector<std::pair<stwr_problem*, int>> who;
      for (Item* it : K)
        if (d < it->levels() - 1) who.push_back({it->P, d});
      B->vc_plans.emplace_back(new SweepPlan());
      build_sweep_plan(B, *B->vc_plans.back(), who);
    }
    B->vc_key = key;
  } else if (!B->vc_exec && B->use_graph && !B->ctx->timing) {
    if (!B->cap) HIPCHK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamSynchronize(bs(B)));
    hipStream_t saved = B->ctx->stream;
    HIPCHK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    B->ctx->stream = B->cap;
    hipGraph_t g = nullptr;
    try {
      vcycle_batch(B, K);
    } catch (...) {
      B->ctx->stream = saved;
      if (hipStreamEndCapture(B->cap, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      B->vc_key.clear();
      throw;
    }
    B->ctx->stream = saved;
    --B->n_vcycles;   // captured, not run
    HIPCHK(hipStreamEndCapture(B->cap, &g));
    const hipError_t e = hipGraphInstantiate(&B->vc_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      B->vc_exec = nullptr;
      B->vc_key.clear();
      HIPCHK(e);
    }
    ++B->n_captures;
  }
  if (B->vc_exec) {
    HIPCHK(hipGraphLaunch(B->vc_exec, bs(B)));
    ++B->n_vcycles;
  } else {
    vcycle_batch(B, K);
  }
}

// ---- Newton and FGMRES state machines ----------------------------------------------

void finish(stwr_batch* B, Item* it, int status) {
  it->phase = kDone;
  it->status = status;
}

// Start of a Newton step for every problem of S: ||F(U)|| and the stopping
// tests, then (for those that go on) assembly, factorization, eigen-estimates
// and the first FGMRES vector.
void newton_setup(stwr_batch* B, std::vector<Item*> S) {
  ensure_pinned(B, (int)S.size());
  for (size_t i = 0; i < S.size(); ++i) {
    Item* it = S[i];
    it->slot = (int)i;
    stwr_problem* P = it->P;
    Level& L0 = P->lv[0];
    residual(P, it->U, L0.b);
    HIPCHK(launch_mdot(L0.n_st, 1, L0.b, 0, L0.b, P->partial, P->dscal, bs(B)));
    HIPCHK(hipMemcpyAsync(row_of(B, *it), P->dscal, 8, hipMemcpyDeviceToHost, bs(B)));
  }
  HIPCHK(hipStreamSynchronize(bs(B)));
  std::vector<Item*> go;
  for (Item* it : S) {
    const stwr_solver_opts& o = it->P->opts;
    const double f = std::sqrt(row_of(B, *it)[0]);
    if (!std::isfinite(f)) {
      finish(B, it, STWR_ERR_NONFINITE);
      continue;
    }
    it->st.fnorm[it->k] = f;
    if (it->k == 0) it->f0 = f;
    it->st.newton_its = it->k;
    if (f <= o.newton_rtol * it->f0 || it->f0 == 0.0) {
      finish(B, it, STWR_OK);
      continue;
    }
    if (it->k > 0 && f > kNewtonDiverged * it->f0) {
      finish(B, it, STWR_ERR_NOT_CONVERGED);
      continue;
    }
    if (it->k >= o.newton_maxit) {
      finish(B, it, STWR_ERR_NOT_CONVERGED);
      continue;
    }
    go.push_back(it);
  }
  if (go.empty()) return;
  const double ts = now_s();
  for (Item* it : go) {
    assemble(it->P, it->U);
    HIPCHK(launch_axpby(it->P->lv[0].n_st, -1.0, it->P->lv[0].b, 0.0, it->P->lv[0].b, bs(B)));   // b = -F
  }
  factor_batch(B, go);
  for (Item* it : go) check_status_flag(it->P, "patch factorization");
  eig_batch(B, go);
  const double dts = now_s() - ts;
  // FGMRES start: x = 0, r = b, beta = ||b||
  for (size_t i = 0; i < go.size(); ++i) {
    Item* it = go[i];
    it->slot = (int)i;
    it->st.setup_seconds += dts / go.size();
    stwr_problem* P = it->P;
    Level& L0 = P->lv[0];
    HIPCHK(launch_fill(L0.n_st, 0.0, L0.x, bs(B)));
    HIPCHK(launch_mdot(L0.n_st, 1, L0.b, 0, L0.b, P->partial, P->dscal, bs(B)));
    HIPCHK(hipMemcpyAsync(row_of(B, *it), P->dscal, 8, hipMemcpyDeviceToHost, bs(B)));
  }
  HIPCHK(hipStreamSynchronize(bs(B)));
  for (Item* it : go) {
    stwr_problem* P = it->P;
    const stwr_solver_opts& o = P->opts;
    Level& L0 = P->lv[0];
    const int m = P->restart;
    it->bnorm = std::sqrt(row_of(B, *it)[0]);
    const double f = it->st.fnorm[it->k];
    double rtol = o.gmres_rtol;
    if (o.newton_ew) rtol = it->eta = ew_forcing(it->k, f, it->k > 0 ? it->st.fnorm[it->k - 1] : it->f0, it->eta);
    it->target = std::max(rtol * it->bnorm, std::max(1e-3 * o.newton_rtol * it->f0, o.gmres_atol));
    it->its = 0;
    it->j = 0;
    it->H.assign((m + 1) * m, 0.0);
    it->cs.assign(m, 0.0);
    it->sn.assign(m, 0.0);
    it->g.assign(m + 1, 0.0);
    it->y.assign(m, 0.0);
    it->g[0] = it->bnorm;
    if (it->bnorm <= it->target) {   // the zero correction already meets the bar
      it->st.linear_its[it->k] = 0;
      it->st.linear_rel[it->k] = it->bnorm > 0.0 ? 1.0 : 0.0;
      ++it->k;
      continue;
    }
    HIPCHK(hipMemcpyAsync(P->V, L0.b, L0.n_st * 8, hipMemcpyDeviceToDevice, bs(B)));
    HIPCHK(launch_axpby(L0.n_st, 1.0 / it->bnorm, P->V, 0.0, P->V, bs(B)));
    it->phase = kKrylov;
  }
}

// x += Z y for the first kk basis vectors (the host solve of the Hessenberg
// system as in fgmres()).
void apply_update(stwr_batch* B, Item* it, int kk) {
  stwr_problem* P = it->P;
  const int m = P->restart;
  for (int i = kk - 1; i >= 0; --i) {
    double s = it->g[i];
    for (int c = i + 1; c < kk; ++c) s -= it->H[i * m + c] * it->y[c];
    it->y[i] = s / it->H[i * m + i];
  }
  const int64_t n = P->lv[0].n_st;
  // the scalars go through the problem's own pinned-free path: a synchronous
  // copy would stall the batch, so they are staged in the readback row
  double* row = row_of(B, *it) + 256;
  std::copy(it->y.begin(), it->y.begin() + kk, row);
  HIPCHK(hipMemcpyAsync(P->dscal, row, kk * 8, hipMemcpyHostToDevice, bs(B)));
  HIPCHK(launch_gemv_cols(n, kk, P->Z, n, P->dscal, P->lv[0].x, bs(B)));
}

// One FGMRES iteration for every problem of K.
void krylov_step(stwr_batch* B, std::vector<Item*> K) {
  ensure_pinned(B, (int)K.size());
  for (size_t i = 0; i < K.size(); ++i) K[i]->slot = (int)i;
  for (Item* it : K) {
    stwr_problem* P = it->P;
    const int64_t n = P->lv[0].n_st;
    HIPCHK(hipMemcpyAsync(P->vc_in, P->V + (int64_t)it->j * n, n * 8, hipMemcpyDeviceToDevice, bs(B)));
  }
  vcycles(B, K);
  for (Item* it : K) {
    stwr_problem* P = it->P;
    const int64_t n = P->lv[0].n_st;
    const int j = it->j;
    double* Zj = P->Z + (int64_t)j * n;
    double* Vn = P->V + (int64_t)(j + 1) * n;
    HIPCHK(hipMemcpyAsync(Zj, P->vc_out, n * 8, hipMemcpyDeviceToDevice, bs(B)));
    project(P, 0, Zj);
    spmv(P, 0, Zj, nullptr, Vn);
    for (int i = 0; i <= j; ++i) {
      HIPCHK(launch_mdot(n, 1, P->V + (int64_t)i * n, 0, Vn, P->partial, P->dscal + i, bs(B)));
      HIPCHK(launch_axpy_dev(n, P->dscal + i, -1.0, P->V + (int64_t)i * n, Vn, bs(B)));
    }
    HIPCHK(launch_mdot(n, 1, Vn, 0, Vn, P->partial, P->dscal + j + 1, bs(B)));
    HIPCHK(hipMemcpyAsync(row_of(B, *it), P->dscal, (j + 2) * 8, hipMemcpyDeviceToHost, bs(B)));
  }
  HIPCHK(hipStreamSynchronize(bs(B)));
  std::vector<Item*> restart;
  for (Item* it : K) {
    stwr_problem* P = it->P;
    const stwr_solver_opts& o = P->opts;
    const int m = P->restart;
    const int64_t n = P->lv[0].n_st;
    const int j = it->j;
    const double* hcol = row_of(B, *it);
    std::vector<double>& H = it->H;
    for (int i = 0; i <= j; ++i) H[i * m + j] = hcol[i];
    const double hn = std::sqrt(hcol[j + 1]);
    if (!std::isfinite(hn)) {
      finish(B, it, STWR_ERR_NONFINITE);
      continue;
    }
    H[(j + 1) * m + j] = hn;
    if (hn != 0.0) HIPCHK(launch_axpby(n, 1.0 / hn, P->V + (int64_t)(j + 1) * n, 0.0, P->V + (int64_t)(j + 1) * n, bs(B)));
    for (int i = 0; i < j; ++i) {
      const double t = it->cs[i] * H[i * m + j] + it->sn[i] * H[(i + 1) * m + j];
      H[(i + 1) * m + j] = -it->sn[i] * H[i * m + j] + it->cs[i] * H[(i + 1) * m + j];
      H[i * m + j] = t;
    }
    const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
    it->cs[j] = H[j * m + j] / den;
    it->sn[j] = H[(j + 1) * m + j] / den;
    H[j * m + j] = den;
    H[(j + 1) * m + j] = 0.0;
    it->g[j + 1] = -it->sn[j] * it->g[j];
    it->g[j] = it->cs[j] * it->g[j];
    ++it->its;
    it->j = j + 1;
    const bool conv = std::fabs(it->g[j + 1]) <= it->target;
    const bool limit = it->its >= o.gmres_maxit;
    if (conv || limit) {
      apply_update(B, it, it->j);
      Level& L0 = P->lv[0];
      HIPCHK(launch_axpby(L0.n_st, 1.0, L0.x, 1.0, it->U, bs(B)));   // U += dU
      it->st.linear_its[it->k] = it->its;
      it->st.linear_rel[it->k] = std::fabs(it->g[j + 1]) / it->bnorm;
      it->st.linear_its_total += it->its;
      ++it->k;
      it->phase = kSetup;
    } else if (it->j == m) {
      apply_update(B, it, m);
      restart.push_back(it);
    }
  }
  if (restart.empty()) return;
  // restarts: r = b - A x into V(0), beta = ||r||
  for (size_t i = 0; i < restart.size(); ++i) {
    Item* it = restart[i];
    it->slot = (int)i;
    stwr_problem* P = it->P;
    Level& L0 = P->lv[0];
    spmv(P, 0, L0.x, L0.b, P->V);
    HIPCHK(launch_mdot(L0.n_st, 1, P->V, 0, P->V, P->partial, P->dscal, bs(B)));
    HIPCHK(hipMemcpyAsync(row_of(B, *it), P->dscal, 8, hipMemcpyDeviceToHost, bs(B)));
  }
  HIPCHK(hipStreamSynchronize(bs(B)));
  for (Item* it : restart) {
    stwr_problem* P = it->P;
    const double beta = std::sqrt(row_of(B, *it)[0]);
    if (!std::isfinite(beta)) {
      finish(B, it, STWR_ERR_NONFINITE);
      continue;
    }
    std::fill(it->g.begin(), it->g.end(), 0.0);
    it->g[0] = beta;
    it->j = 0;
    if (beta <= it->target) {   // the restart's own residual already meets the bar
      Level& L0 = P->lv[0];
      HIPCHK(launch_axpby(L0.n_st, 1.0, L0.x, 1.0, it->U, bs(B)));
      it->st.linear_its[it->k] = it->its;
      it->st.linear_rel[it->k] = beta / it->bnorm;
      it->st.linear_its_total += it->its;
      ++it->k;
      it->phase = kSetup;
      continue;
    }
    HIPCHK(launch_axpby(P->lv[0].n_st, 1.0 / beta, P->V, 0.0, P->V, bs(B)));
  }
}

// Results of finished problems: copy the solution out, release the problem.
void collect(stwr_batch* B) {
  for (auto itp = B->items.begin(); itp != B->items.end();) {
    Item* it = itp->get();
    if (it->phase != kDone) {
      ++itp;
      continue;
    }
    stwr_problem* P = it->P;
    stwr_result r{};
    r.id = it->id;
    r.status = it->status;
    r.newton_its = it->k;
    r.linear_its = it->st.linear_its_total;
    r.slot = -1;
    r.submit_time = it->submit_time;
    r.start_time = it->start_time;
    r.fnorm_ratio = it->f0 > 0.0 ? it->st.fnorm[it->k] / it->f0 : 0.0;
    r.bytes = it->bytes;
    if (it->host_out)
      HIPCHK(hipMemcpyAsync(it->host_out, it->U, P->lv[0].n_st * 8, hipMemcpyDeviceToHost, bs(B)));
    HIPCHK(hipStreamSynchronize(bs(B)));
    r.end_time = B->now();
    {
      std::lock_guard<std::mutex> g(B->ctx->mu);
      B->ctx->in_use -= std::min<uint64_t>(B->ctx->in_use, (uint64_t)P->lv[0].n_st * 8);
    }
    stwr_problem_destroy(P);
    B->done.push_back(r);
    itp = B->items.erase(itp);
    drop_graph(B);
    B->vc_key.clear();
  }
}

}  // namespace

extern "C" {

int32_t stwr_batch_create(stwr_ctx* ctx, int32_t use_graph, stwr_batch** out) {
  return guarded(ctx, [&]() -> int32_t {
    if (!ctx || !out) throw StwrError(STWR_ERR_ARG, "null argument");
    if (use_graph != 0 && use_graph != 1) throw StwrError(STWR_ERR_ARG, "use_graph must be 0 or 1");
    HIPCHK(hipSetDevice(ctx->device));
    std::unique_ptr<stwr_batch> B(new stwr_batch());
    B->ctx = ctx;
    B->use_graph = use_graph;
    B->t_origin = now_s();
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, ctx->device));
    B->n_cu = prop.multiProcessorCount;
    for (int c = 0; c < 2; ++c) B->sweep_occ[c] = patch_sweep_batch_occupancy(c + 1);
    for (int c = 0; c < kFacClasses; ++c) B->factor_occ[c] = patch_factor_batch_occupancy(c);
    HIPCHK(hipMalloc(&B->ctr, 16 * sizeof(int)));
    HIPCHK(hipMemsetAsync(B->ctr, 0, 16 * sizeof(int), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = B.release();
    return STWR_OK;
  });
}

int32_t stwr_batch_add(stwr_batch* b, const stwr_problem_desc* desc, const stwr_solver_opts* opts,
                       double* host_out, int64_t* id_out) {
  if (!b) return STWR_ERR_ARG;
  return guarded(b->ctx, [&]() -> int32_t {
    if (!desc || !opts || !id_out) throw StwrError(STWR_ERR_ARG, "null argument");
    if (desc->equation != STWR_EQ_NAVIER_STOKES) throw StwrError(STWR_ERR_ARG, "the batch solves Navier-Stokes problems");
    if (desc->degree > 1) throw StwrError(STWR_ERR_ARG, "the batch solves P2-P1 problems (patches of at most 39 DoFs)");
    if (opts->smoother_prec != STWR_FP32) throw StwrError(STWR_ERR_ARG, "the batch runs FP32 patch factors and sweeps");
    if (b->nu_pre >= 0 && (opts->nu_pre != b->nu_pre || opts->nu_post != b->nu_post))
      throw StwrError(STWR_ERR_ARG, "every problem of a batch has the same nu_pre and nu_post");
    if (desc->n_levels < 2) throw StwrError(STWR_ERR_ARG, "the batch needs at least two levels");
    if ((opts->eig_steps + 2) * (desc->n_levels - 1) > 256)
      throw StwrError(STWR_ERR_ARG, "eig_steps too large for the batched eigen-estimates");
    stwr_solver_opts o = *opts;
    o.vcycle_graph = 1;     // the V-cycle input and output vectors are allocated with the problem
    o.time_chunks = 1;
    o.factor_mfma = 1;
    stwr_problem* P = nullptr;
    const int32_t rc = stwr_problem_create(b->ctx, desc, &o, &P);
    if (rc != STWR_OK) return rc;
    std::unique_ptr<Item> it(new Item());
    it->P = P;
    try {
      // the Arnoldi bases of all smoothed levels side by side in the Krylov space
      int64_t need = 0;
      for (int l = 0; l + 1 < (int)P->lv.size(); ++l) need += (int64_t)(o.eig_steps + 1) * P->lv[l].n_st;
      if (need > (int64_t)(P->restart + 1) * P->lv[0].n_st)
        throw StwrError(STWR_ERR_ARG, "gmres_restart too small for the batched eigen-estimates");
      const int64_t n0 = P->lv[0].n_st;
      {
        std::lock_guard<std::mutex> g(b->ctx->mu);
        if (b->ctx->budget && b->ctx->in_use + n0 * 8 > b->ctx->budget)
          throw StwrError(STWR_ERR_BUDGET, "solution vector exceeds the HBM budget");
        b->ctx->in_use += n0 * 8;
      }
      it->U = P->alloc<double>(n0);
      if (!P->vc_in) {
        P->vc_in = P->alloc<double>(n0);
        P->vc_out = P->alloc<double>(n0);
      }
      HIPCHK(launch_fill(n0, 0.0, it->U, b->ctx->stream));
    } catch (...) {
      stwr_problem_destroy(P);
      throw;
    }
    it->bytes = P->bytes + (uint64_t)P->lv[0].n_st * 8;
    it->host_out = host_out;
    it->id = b->next_id++;
    it->submit_time = it->start_time = b->now();
    if (b->nu_pre < 0) {
      b->nu_pre = o.nu_pre;
      b->nu_post = o.nu_post;
    }
    *id_out = it->id;
    b->items.push_back(std::move(it));
    return STWR_OK;
  });
}

int32_t stwr_batch_step(stwr_batch* b, int32_t* n_live) {
  if (!b) return STWR_ERR_ARG;
  return guarded(b->ctx, [&]() -> int32_t {
    std::vector<Item*> S, K;
    for (auto& it : b->items)
      if (it->phase == kSetup) S.push_back(it.get());
    if (!S.empty()) newton_setup(b, S);
    for (auto& it : b->items)
      if (it->phase == kKrylov) K.push_back(it.get());
    if (!K.empty()) krylov_step(b, K);
    collect(b);
    ++b->n_steps;
    if (n_live) *n_live = (int32_t)b->items.size();
    return STWR_OK;
  });
}

int32_t stwr_batch_poll(stwr_batch* b, stwr_result* results, int32_t max_results, int32_t* n_out) {
  if (!b || !n_out || (max_results > 0 && !results)) return STWR_ERR_ARG;
  int32_t n = 0;
  while (n < max_results && !b->done.empty()) {
    results[n++] = b->done.front();
    b->done.pop_front();
  }
  *n_out = n;
  return STWR_OK;
}

int32_t stwr_batch_info(const stwr_batch* b, int64_t* out) {
  if (!b || !out) return STWR_ERR_ARG;
  out[0] = b->n_steps;
  out[1] = b->n_captures;
  out[2] = b->n_vcycles;
  out[3] = b->n_sweep_launches;
  out[4] = b->n_factor_launches;
  out[5] = b->sweep_tile[0];
  out[6] = b->sweep_tile[1];
  for (int c = 0; c < kFacClasses; ++c) out[7 + c] = b->factor_tile[c];
  out[10] = (int64_t)b->items.size();
  return STWR_OK;
}

int32_t stwr_batch_destroy(stwr_batch* b) {
  if (!b) return STWR_OK;
  (void)hipStreamSynchronize(b->ctx->stream);
  drop_graph(b);
  b->vc_key.clear();
  for (auto& it : b->items) {
    {
      std::lock_guard<std::mutex> g(b->ctx->mu);
      b->ctx->in_use -= std::min<uint64_t>(b->ctx->in_use, (uint64_t)it->P->lv[0].n_st * 8);
    }
    stwr_problem_destroy(it->P);
  }
  b->items.clear();
  for (auto& p : b->vc_plans) {
    p->jobs.release();
    p->tiles.release();
  }
  b->eig_plan.jobs.release();
  b->eig_plan.tiles.release();
  b->fjobs.release();
  b->ftiles.release();
  if (b->ctr) (void)hipFree(b->ctr);
  if (b->pinned) (void)hipHostFree(b->pinned);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return STWR_OK;
}

}  // extern "C"
