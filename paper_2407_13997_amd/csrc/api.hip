// C ABI of the space-time WR multigrid library: problem object, allocation
// plan and HBM budget, and the host control of Alg. 1 (V-cycle), Chebyshev
// relaxation, the eigen-estimate, FGMRES and Newton (Secs. 3 and 4.2).  Every
// arithmetic step on space-time data runs in the gfx950 kernels; the host only
// keeps scalars (Krylov Hessenberg columns, Givens rotations, the 10x10 Ritz
// problem) and launches.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "problem.h"

using namespace stwr;
using namespace stwr::impl;

// Patch-output area of stwr_patch_apply_noalloc: one per device, held until
// the process ends.  Host code never passes the array's name to a kernel or a
// copy: it uses the device address from hipGetSymbolAddress, taken once per
// device when the first context on that device is created.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // per device; null until resolved

// Resolves (once per device, the device current) the device address of the
// scratch array; throws on failure.
void resolve_scratch(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (g_scratch_ptr[device]) return;
  double* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    throw StwrError(STWR_ERR_DEVICE, std::string("scratch symbol address: ") + hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
}

double* scratch_of(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return device < (int)g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}
}  // namespace

namespace stwr {
namespace impl {

thread_local std::string g_tls_error;

int32_t fail(stwr_ctx* ctx, int32_t code, const std::string& msg) {
  if (ctx) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->last_error = msg;
  }
  g_tls_error = msg;
  return code;
}


bool is_heat(const stwr_problem_desc* d) { return d->equation == STWR_EQ_HEAT; }

// Free spatial DoFs of a level with M squares a side: Taylor-Hood P2-P1 with
// the boundary velocity eliminated, 2 (2M-1)^2 + (M+1)^2; the heat equation's
// P_k lattice, (kM+1)^2 (every node free).  The level builders give the same
// counts.
// Taylor-Hood pressure degree k of a Navier-Stokes problem (degree 0 or 1:
// P2-P1; 2: P3-P2).
int th_degree(const stwr_problem_desc* d) { return (!is_heat(d) && d->degree == kThK) ? kThK : 1; }

int64_t free_dofs(const stwr_problem_desc* d, int M) {
  if (is_heat(d)) return (int64_t)(d->degree * M + 1) * (d->degree * M + 1);
  if (th_degree(d) == kThK) {
    const int64_t nv = (kThK + 1) * M - 1, np = kThK * M + 1;
    return 2 * nv * nv + np * np;
  }
  return 2LL * (2 * M - 1) * (2 * M - 1) + (int64_t)(M + 1) * (M + 1);
}

void check_desc(const stwr_problem_desc* d) {
  if (!d) throw StwrError(STWR_ERR_ARG, "null problem descriptor");
  if (d->equation != STWR_EQ_NAVIER_STOKES && d->equation != STWR_EQ_HEAT)
    throw StwrError(STWR_ERR_ARG, "bad equation");
  if (is_heat(d) && (d->degree < 1 || d->degree > kMaxPk))
    throw StwrError(STWR_ERR_ARG, "heat equation degree must be 1, 2 or 3");
  if (!is_heat(d) && (d->degree < 0 || d->degree > kThK))
    throw StwrError(STWR_ERR_ARG, "Navier-Stokes pressure degree must be 1 (P2-P1) or 2 (P3-P2)");
  if (d->q < 0 || d->q > (is_heat(d) ? kMaxNQ - 1 : 1))
    throw StwrError(STWR_ERR_ARG, is_heat(d) ? "q must be 0..3 for the heat equation" : "q must be 0 or 1");
  if (d->n_levels < 1 || d->n_levels > STWR_MAX_LEVELS) throw StwrError(STWR_ERR_ARG, "bad n_levels");
  if (d->mesh_n < 2 || d->n_slabs < 1) throw StwrError(STWR_ERR_ARG, "bad mesh_n or n_slabs");
  if (d->mesh_n % (1 << (d->n_levels - 1)) != 0 || (d->mesh_n >> (d->n_levels - 1)) < 2)
    throw StwrError(STWR_ERR_ARG, "mesh_n must be divisible by 2^(n_levels-1) with a coarsest mesh of >= 2");
  if (!(d->t_final > 0.0)) throw StwrError(STWR_ERR_ARG, "t_final must be positive");
  if (d->n_psi_modes < 0 || d->n_p_modes < 0) throw StwrError(STWR_ERR_ARG, "bad mode counts");
  if (d->flow != STWR_FLOW_MODES && d->flow != STWR_FLOW_CHORIN && d->flow != STWR_FLOW_CAVITY)
    throw StwrError(STWR_ERR_ARG, "bad flow");
  if (d->temporal_nodes != STWR_NODES_RADAU && d->temporal_nodes != STWR_NODES_GAUSS)
    throw StwrError(STWR_ERR_ARG, "bad temporal nodes");
  if ((d->n_psi_modes > 0 && (!d->psi_ab || !d->psi_coef)) || (d->n_p_modes > 0 && (!d->p_ab || !d->p_coef)))
    throw StwrError(STWR_ERR_ARG, "null mode arrays");
  const int64_t nfc = free_dofs(d, d->mesh_n >> (d->n_levels - 1));
  if (nfc * (d->q + 1) + (is_heat(d) ? 0 : d->q + 1) > 4096)
    throw StwrError(STWR_ERR_ARG, "coarsest level too large for the dense coarse solve (use more levels)");
}

// time chunks per sweep: at most this many, and the autotuner only tries
// them on levels with at most kTuneMaxPatches patches (larger levels fill
// the chip with patches alone, and chunking doubles their block traffic)
constexpr int kMaxTimeChunks = 64;
constexpr int kTuneMaxPatches = 2048;

void check_opts(const stwr_solver_opts* o) {
  if (!o) throw StwrError(STWR_ERR_ARG, "null options");
  if (o->nu_pre < 0 || o->nu_post < 0 || o->eig_steps < 1 || o->eig_steps > 64 || o->gmres_restart < 1 ||
      o->gmres_restart > 200 || o->gmres_maxit < 1 || o->newton_maxit < 0 || o->newton_maxit > STWR_MAX_NEWTON ||
      (o->smoother_prec != STWR_FP64 && o->smoother_prec != STWR_FP32) || !(o->cheb_hi > o->cheb_lo) ||
      !(o->cheb_lo > 0.0) || (o->vcycle_graph != 0 && o->vcycle_graph != 1) ||
      (o->newton_ew != 0 && o->newton_ew != 1) || !(o->gmres_atol >= 0.0) || o->time_chunks < 0 ||
      o->time_chunks > kMaxTimeChunks || (o->factor_mfma != 0 && o->factor_mfma != 1) ||
      (o->deterministic != 0 && o->deterministic != 1))
    throw StwrError(STWR_ERR_ARG, "invalid solver options");
}

int vw_of(int prec) { return prec == STWR_FP32 ? 4 : 2; }
int round_up(int m, int w) { return (m + w - 1) / w * w; }

// Elements reserved for one stored inverse slab block of size m (layout shared
// with the patch kernels), rounded up to 256 bytes so that every block, and so
// every 1 KiB wavefront load inside it, starts on a cache-line boundary.
int64_t block_elems(int m, int VW) { return round_up(BlockLayout(m, VW).size(), 16 * VW); }
// The same for a level's own block layout (the large-block layout on
// Taylor-Hood P3-P2 levels).
int64_t level_block_elems(const HostLevel& H, int m, int VW) {
  return H.thk > 0 ? round_up(big_block_size(m, VW), 16 * VW) : block_elems(m, VW);
}

// Slabs with their own patch blocks: the heat operator is the same on every
// slab (uniform slabs, time-independent coefficients), so its blocks are
// factored once and read for every slab.
int fac_slabs_of(const HostLevel& H, int N) { return H.kdeg > 0 ? 1 : N; }

// Levels whose FP32 sweep reads an FP32 residual (P2-P1 Navier-Stokes); it
// sits after the blocks in the factor storage.
bool has_f32_residual(const HostLevel& H, int prec) { return prec == STWR_FP32 && H.kdeg == 0 && H.thk == 0; }

// Element count of the factor storage of one level at a precision.
int64_t fac_elems(const HostLevel& H, int N, int NQ, int prec) {
  const int NS = fac_slabs_of(H, N);
  int64_t tot = 0;
  for (int v = 0; v < H.nv; ++v) {
    const int m = (H.patch_ptr[v + 1] - H.patch_ptr[v]) * NQ;
    tot += (int64_t)NS * level_block_elems(H, m, vw_of(prec));
  }
  if (has_f32_residual(H, prec)) tot += (int64_t)H.nf * N * NQ;
  return tot;
}

// Doubles reserved for one patch's outputs (nb DoFs x N slabs x (q+1)
// nodes), rounded up to whole 128-byte lines so every patch's outputs start
// on a line boundary.
int64_t y_elems(int nb, int N, int NQ) { return ((int64_t)nb * N * NQ + 15) / 16 * 16; }

struct Plan {
  uint64_t bytes = 0;
};

uint64_t level_bytes(const HostLevel& H, const HostTransfer* T, int N, int NQ, int prec, bool coarsest) {
  const int64_t nnz = H.row_ptr[H.nf];
  const int64_t n_st = (int64_t)H.nf * N * NQ;
  uint64_t b = 0;
  b += (uint64_t)nnz * N * NQ * NQ * 8 + nnz * 8;                       // Jv, Mv
  if (H.kdeg > 0) b += (uint64_t)nnz * 8;                               // Kv
  b += (uint64_t)(H.nf + 1 + nnz) * 4;                                  // CSR
  b += (uint64_t)(H.cells.size() + H.cell_p2.size() + H.cell_vn.size() + H.cell_pn.size() +
                 H.cell_dofs.size() + H.cell_nz.size() +
                 H.node_free.size() + H.node_cell_ptr.size() + H.node_cell.size() +
                 (H.kdeg == 0 ? H.color_cells.size() : 0)) * 4;   // cell maps
  b += (uint64_t)(H.nv + 1) * 4 * 2 + (uint64_t)H.patch_dofs.size() * 4 * 2 + H.patch_nz.size() * 4;
  b += (uint64_t)(H.nv + 1) * 8 * 4 + (uint64_t)(H.nf + 1 + H.patch_dofs.size()) * 4;
  b += (uint64_t)4 * n_st * 8;                                          // r, d, x, b
  if (!coarsest) {
    b += (uint64_t)fac_elems(H, N, NQ, prec) * (prec == STWR_FP32 ? 4 : 8);
    int64_t mp = 0;
    for (int v = 0; v < H.nv; ++v) mp += (int64_t)H.patch_nbu[v] * H.patch_nbu[v];
    b += (uint64_t)mp * 8;
    for (int v = 0; v < H.nv; ++v)                                      // Y
      b += (uint64_t)y_elems(H.patch_ptr[v + 1] - H.patch_ptr[v], N, NQ) * 8;
  } else {
    const int64_t mm = (int64_t)H.nf * NQ + (H.po < H.nf ? NQ : 0);
    const int64_t cs = fac_slabs_of(H, N);
    b += (uint64_t)cs * mm * mm * 8 + (uint64_t)cs * mm * 12 + mm * 8 + (mm > kCoarseSmall ? (uint64_t)cs * kRbufRows * mm * 8 : 0);
  }
  if (T) b += (T->p_col.size() + T->r_col.size()) * 12 + (T->p_ptr.size() + T->r_ptr.size()) * 4;
  return b;
}

// Host construction of every level, then of every transfer, each on a
// thread of its own (the builders split their larger loops further).
void build_levels(const stwr_problem_desc* d, std::vector<Level>& lv) {
  lv.resize(d->n_levels);
  std::vector<std::exception_ptr> err(d->n_levels);
  auto run_all = [&](int count, auto&& job) {
    std::vector<std::thread> th;
    for (int l = 0; l < count; ++l)
      th.emplace_back([&, l]() {
        try {
          job(l);
        } catch (...) {
          err[l] = std::current_exception();
        }
      });
    for (auto& t : th) t.join();
    for (auto& e : err)
      if (e) std::rethrow_exception(e);
  };
  run_all(d->n_levels, [&](int l) {
    if (is_heat(d)) build_level_heat(d->mesh_n >> l, d->degree, lv[l].H);
    else if (th_degree(d) == kThK) build_level_th(d->mesh_n >> l, kThK, lv[l].H);
    else build_level(d->mesh_n >> l, lv[l].H);
    lv[l].N = d->n_slabs;
    lv[l].NQ = d->q + 1;
    lv[l].dt = d->t_final / d->n_slabs;
    lv[l].n_st = (int64_t)lv[l].H.nf * d->n_slabs * (d->q + 1);
  });
  run_all(d->n_levels - 1, [&](int l) {
    if (is_heat(d)) build_transfer_heat(lv[l].H, lv[l + 1].H, lv[l].Tr);
    else if (th_degree(d) == kThK) build_transfer_th(lv[l].H, lv[l + 1].H, lv[l].Tr);
    else build_transfer(lv[l].H, lv[l + 1].H, lv[l].Tr);
  });
}

uint64_t plan_bytes(const stwr_problem_desc* d, const stwr_solver_opts* o, const std::vector<Level>& lv) {
  uint64_t b = 0;
  const int L = (int)lv.size();
  for (int l = 0; l < L; ++l)
    b += level_bytes(lv[l].H, l + 1 < L ? &lv[l].Tr : nullptr, d->n_slabs, d->q + 1, o->smoother_prec, l == L - 1);
  const int64_t n0 = lv[0].n_st;
  b += (uint64_t)(2 * o->gmres_restart + 1) * n0 * 8;
  if (o->vcycle_graph) b += (uint64_t)2 * n0 * 8;                       // graph input, output
  if (is_heat(d)) b += (uint64_t)n0 * 8;                                // heat right-hand side
  b += (uint64_t)(256 + 4) * 256 * 8 + sizeof(RefTables) + 4096;
  return b;
}

// ---------------------------------------------------------------------------
// Level upload
void upload_level(stwr_problem* P, Level& L, bool coarsest) {
  HostLevel& H = L.H;
  L.row_ptr = P->upload(H.row_ptr);
  L.col = P->upload(H.col);
  L.cells = P->upload(H.cells);
  L.cell_p2 = P->upload(H.cell_p2);
  if (H.thk > 0) {
    L.cell_vn = P->upload(H.cell_vn);
    L.cell_pn = P->upload(H.cell_pn);
  }
  L.cell_dofs = P->upload(H.cell_dofs);
  L.cell_nz = P->upload(H.cell_nz);
  if (H.kdeg == 0) L.color_cells = P->upload(H.color_cells);
  L.node_free = P->upload(H.node_free);
  if (H.kdeg > 0) {
    L.node_cell_ptr = P->upload(H.node_cell_ptr);
    L.node_cell = P->upload(H.node_cell);
  }
  const int64_t nnz = H.row_ptr[H.nf];
  L.Jv = P->alloc<double>((size_t)nnz * L.N * L.NQ * L.NQ);
  L.Mv = P->alloc<double>((size_t)nnz);
  if (H.kdeg > 0) L.Kv = P->alloc<double>((size_t)nnz);
  L.r = P->alloc<double>(L.n_st);
  L.d = P->alloc<double>(L.n_st);
  L.x = P->alloc<double>(L.n_st);
  L.b = P->alloc<double>(L.n_st);
  LevelView& v = L.view;
  v.M = H.M; v.nf = H.nf; v.po = H.po; v.nv = H.nv; v.nc = H.nc; v.N = L.N; v.NQ = L.NQ;
  v.dt = L.dt; v.h = 1.0 / H.M; v.nnz = nnz;
  v.row_ptr = L.row_ptr; v.col = L.col; v.cells = L.cells; v.cell_p2 = L.cell_p2;
  v.cell_dofs = L.cell_dofs; v.cell_nz = L.cell_nz; v.node_free = L.node_free;
  v.n2 = H.n2; v.n1 = H.n1;
  v.kdeg = H.kdeg; v.nloc = H.nloc;
  v.thk = H.thk; v.n3 = H.n3; v.nlv = H.nlv; v.nlp = H.nlp;
  v.cell_vn = L.cell_vn; v.cell_pn = L.cell_pn;
  v.color_cells = L.color_cells; v.color_first = 0;
  v.node_cell_ptr = L.node_cell_ptr; v.node_cell = L.node_cell;
  v.nbord = H.po < H.nf ? L.NQ : 0;
  v.coarse_slabs = fac_slabs_of(H, L.N);
  // patches (the coarsest level is solved directly and needs none)
  PatchView& pv = L.pview;
  pv.n_patch = H.nv;
  pv.fac_slabs = fac_slabs_of(H, L.N);
  if (!coarsest) {
    L.patch_ptr = P->upload(H.patch_ptr);
    L.patch_dofs = P->upload(H.patch_dofs);
    L.patch_nbu = P->upload(H.patch_nbu);
    L.patch_nz_off = P->upload(H.patch_nz_off);
    L.patch_nz = P->upload(H.patch_nz);
    L.dof_ptr = P->upload(H.dof_ptr);
    L.dof_slot = P->upload(H.dof_slot);
    L.slot_patch = P->upload(H.slot_patch);
    L.y_off.assign(H.nv + 1, 0);
    L.mp_off.assign(H.nv + 1, 0);
    for (int p = 0; p < H.nv; ++p) {
      const int nb = H.patch_ptr[p + 1] - H.patch_ptr[p];
      L.y_off[p + 1] = L.y_off[p] + y_elems(nb, L.N, L.NQ);
      L.mp_off[p + 1] = L.mp_off[p] + (int64_t)H.patch_nbu[p] * H.patch_nbu[p];
    }
    L.d_y_off = P->upload(L.y_off);
    L.d_mp_off = P->upload(L.mp_off);
    L.Mp = P->alloc<double>(L.mp_off[H.nv]);
    L.Y = P->alloc<double>(L.y_off[H.nv]);
    L.d_fac_off = P->alloc<int64_t>(H.nv + 1);
    pv.patch_ptr = L.patch_ptr; pv.patch_dofs = L.patch_dofs; pv.patch_nbu = L.patch_nbu;
    pv.patch_nz_off = L.patch_nz_off; pv.patch_nz = L.patch_nz; pv.fac_off = L.d_fac_off;
    pv.y_off = L.d_y_off; pv.mp_off = L.d_mp_off; pv.dof_ptr = L.dof_ptr; pv.dof_slot = L.dof_slot;
    pv.slot_patch = L.slot_patch;
    // patches by decreasing size (stable): the interior ones (nb = 39)
    // first, then the blocks larger than a wavefront's 64 rows
    std::vector<int> order(H.nv);
    for (int v = 0; v < H.nv; ++v) order[v] = v;
    auto nb_of = [&](int v) { return H.patch_ptr[v + 1] - H.patch_ptr[v]; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nb_of(x) > nb_of(y); });
    pv.n_full = 0;
    pv.n_big = 0;
    for (int v : order) {
      pv.n_full += nb_of(v) == kMaxNb;
      pv.n_big += nb_of(v) * L.NQ > 64;
    }
    pv.order = P->upload(order);
    L.order = order;
    L.P_ptr = P->upload(L.Tr.p_ptr);
    L.P_col = P->upload(L.Tr.p_col);
    L.P_val = P->upload(L.Tr.p_val);
    L.R_ptr = P->upload(L.Tr.r_ptr);
    L.R_col = P->upload(L.Tr.r_col);
    L.R_val = P->upload(L.Tr.r_val);
  } else {
    L.coarse_mm = H.nf * L.NQ + L.view.nbord;
    const size_t cs = L.view.coarse_slabs;
    L.Binv = P->alloc<double>(cs * L.coarse_mm * L.coarse_mm);
    L.gbuf = P->alloc<double>((size_t)L.coarse_mm);
    L.perm = P->alloc<int>(cs * L.coarse_mm);
    L.colbuf = P->alloc<double>(cs * L.coarse_mm);
    if (L.coarse_mm > kCoarseSmall) L.rbuf = P->alloc<double>(cs * kRbufRows * L.coarse_mm);
  }
}

void ensure_factor_storage(stwr_problem* P, Level& L, int prec) {
  const int64_t elems = fac_elems(L.H, L.N, L.NQ, prec);
  const size_t need = (size_t)elems * (prec == STWR_FP32 ? 4 : 8);
  if (L.fac && L.fac_bytes >= need) {
    // offsets depend on the precision's panel width
  } else {
    if (L.fac) {
      P->release(L.fac);
      L.fac = nullptr;
    }
    const size_t extra = need > L.fac_budgeted ? need - L.fac_budgeted : 0;
    {
      std::lock_guard<std::mutex> g(P->ctx->mu);
      const uint64_t budget = P->ctx->budget;
      if (budget && P->ctx->in_use + extra > budget)
        throw StwrError(STWR_ERR_BUDGET, "patch factors exceed the HBM budget");
      P->ctx->in_use += extra;
    }
    P->bytes += extra;
    L.fac_budgeted += extra;
    L.fac = P->alloc<char>(need);
    L.fac_bytes = need;
    L.fac_layout = -1;
  }
  // the panel layout's padding must read as zero; the factor kernel writes
  // every entry but never the padding, so clear the storage whenever its
  // layout (the precision) changes
  if (L.fac_layout != prec) {
    HIPCHK(hipMemsetAsync(L.fac, 0, L.fac_bytes, P->s()));
    L.fac_layout = prec;
  }
  // [slab][patch] order: the patches resident at one time (which start
  // together and advance at similar rates) read from a few compact regions
  L.fac_off.assign(L.H.nv + 1, 0);
  for (int v = 0; v < L.H.nv; ++v) {
    const int m = (L.H.patch_ptr[v + 1] - L.H.patch_ptr[v]) * L.NQ;
    L.fac_off[v + 1] = L.fac_off[v] + level_block_elems(L.H, m, vw_of(prec));
  }
  L.pview.slab_stride = L.pview.fac_slabs == 1 ? 0 : L.fac_off[L.H.nv];
  L.rf = has_f32_residual(L.H, prec) ? (float*)L.fac + (int64_t)L.pview.fac_slabs * L.fac_off[L.H.nv] : nullptr;
  HIPCHK(hipMemcpyAsync(L.d_fac_off, L.fac_off.data(), L.fac_off.size() * 8, hipMemcpyHostToDevice, P->s()));
}

// ---------------------------------------------------------------------------
// Small host helpers
Level& level_at(stwr_problem* P, int l) {
  if (l < 0 || l >= (int)P->lv.size()) throw StwrError(STWR_ERR_ARG, "level out of range");
  return P->lv[l];
}

void check_status_flag(stwr_problem* P, const char* what) {
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, P->dstatus, sizeof(int), hipMemcpyDeviceToHost, P->s()));
  HIPCHK(hipStreamSynchronize(P->s()));
  if (h) {
    int z = 0;
    HIPCHK(hipMemcpyAsync(P->dstatus, &z, sizeof(int), hipMemcpyHostToDevice, P->s()));
    HIPCHK(hipStreamSynchronize(P->s()));
    throw StwrError(STWR_ERR_SINGULAR, std::string(what) + ": zero or non-finite pivot");
  }
}

double dot_host(stwr_problem* P, int64_t n, const double* x, const double* y) {
  HIPCHK(launch_mdot(n, 1, x, 0, y, P->partial, P->dscal, P->s()));
  double h = 0.0;
  HIPCHK(hipMemcpyAsync(&h, P->dscal, 8, hipMemcpyDeviceToHost, P->s()));
  HIPCHK(hipStreamSynchronize(P->s()));
  return h;
}

double norm_host(stwr_problem* P, int64_t n, const double* x) {
  const double v = dot_host(P, n, x, x);
  if (!std::isfinite(v)) throw StwrError(STWR_ERR_NONFINITE, "non-finite norm");
  return std::sqrt(v);
}

void spmv(stwr_problem* P, int l, const double* x, const double* b, double* y) {
  Level& L = P->lv[l];
  KernelMark mark(P->ctx, 1);
  if (P->heat()) {
    HIPCHK(launch_heat_spmv(L.view, P->d_tab, L.Mv, L.Kv, x, b, y, P->s()));
    return;
  }
  HIPCHK(launch_spmv(L.view, L.Jv, L.Mv, P->tab.e0, P->tab.e1, x, b, y, P->s()));
}

void project(stwr_problem* P, int l, double* x) {
  Level& L = P->lv[l];
  if (L.H.po >= L.H.nf) return;   // no pressure (heat equation)
  HIPCHK(launch_pressure_project(L.H.nf, L.H.po, L.N * L.NQ, x, P->dscal + 256, P->s()));
}

void require_factor(stwr_problem* P, int l) {
  if (!P->assembled) throw StwrError(STWR_ERR_STATE, "operator not assembled");
  if (l >= (int)P->lv.size() - 1) throw StwrError(STWR_ERR_ARG, "the coarsest level has no smoother");
  if (P->lv[l].fac_prec < 0) throw StwrError(STWR_ERR_STATE, "patch factors missing (call stwr_patch_factor)");
}

// Large blocks (Taylor-Hood P3-P2, up to 162 rows): the blocks are copied
// out dense in chunks, inverted in FP64 by the blocked Gauss-Jordan of the
// coarsest level (partial pivoting), and written into the factor storage at
// the requested precision.  The chunk workspace is temporary.
void patch_factor_big(stwr_problem* P, Level& L, int prec) {
  int mmax = 0;
  for (int v = 0; v < L.H.nv; ++v) mmax = std::max(mmax, (L.H.patch_ptr[v + 1] - L.H.patch_ptr[v]) * L.NQ);
  const int64_t nblocks = (int64_t)L.H.nv * L.pview.fac_slabs;
  const size_t per = (size_t)mmax * mmax * 8 + (size_t)mmax * 12 + (size_t)kRbufRows * mmax * 8;
  const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>({nblocks, (int64_t)((size_t(1) << 30) / per), 32768}));
  double *B = nullptr, *colbuf = nullptr, *rbuf = nullptr;
  int* perm = nullptr;
  auto release = [&]() {
    (void)hipStreamSynchronize(P->s());
    for (void* q : {(void*)B, (void*)colbuf, (void*)rbuf, (void*)perm})
      if (q) (void)hipFree(q);
  };
  try {
    HIPCHK(hipMalloc(&B, (size_t)chunk * mmax * mmax * 8));
    HIPCHK(hipMalloc(&colbuf, (size_t)chunk * mmax * 8));
    HIPCHK(hipMalloc(&rbuf, (size_t)chunk * kRbufRows * mmax * 8));
    HIPCHK(hipMalloc(&perm, (size_t)chunk * mmax * 4));
    for (int64_t b0 = 0; b0 < nblocks; b0 += chunk) {
      const int cnt = (int)std::min<int64_t>(chunk, nblocks - b0);
      HIPCHK(launch_patch_extract_dense(L.view, L.pview, L.Jv, (int)b0, cnt, mmax, B, P->s()));
      HIPCHK(launch_dense_inverse(cnt, mmax, B, P->dstatus, perm, colbuf, rbuf, P->s()));
      HIPCHK(launch_patch_store_big(L.view, L.pview, prec, B, (int)b0, cnt, mmax, L.fac, P->s()));
    }
  } catch (...) {
    release();
    throw;
  }
  release();
}

void patch_factor(stwr_problem* P, int l, int prec) {
  if (!P->assembled) throw StwrError(STWR_ERR_STATE, "operator not assembled");
  if (l >= (int)P->lv.size() - 1) throw StwrError(STWR_ERR_ARG, "the coarsest level has no smoother");
  if (prec != STWR_FP32 && prec != STWR_FP64) throw StwrError(STWR_ERR_ARG, "bad precision");
  Level& L = P->lv[l];
  ensure_factor_storage(P, L, prec);
  if (L.H.thk > 0) {
    // in registers where a row fits (FP32, and FP64 at one temporal node),
    // else through dense FP64 copies
    if (!P->opts.factor_mfma ||
        launch_patch_factor_big_reg(L.view, L.pview, L.Jv, prec, L.fac, P->dstatus, P->s()) != hipSuccess) {
      (void)hipGetLastError();
      patch_factor_big(P, L, prec);
    }
    HIPCHK(launch_patch_mass(L.view, L.pview, L.Mv, L.Mp, P->s()));
    L.fac_prec = prec;
    check_status_flag(P, "patch factorization");
    return;
  }
  L.pview.factor_mfma = P->opts.factor_mfma;
  HIPCHK(launch_patch_factor(L.view, L.pview, L.Jv, prec, L.fac, P->dstatus, P->s()));
  HIPCHK(launch_patch_mass(L.view, L.pview, L.Mv, L.Mp, P->s()));
  L.fac_prec = prec;
  HIPCHK(launch_patch_chunk_transfer(L.view, L.pview, prec, L.fac, L.Mp, P->tab.e0, P->tab.e1, P->s()));
  check_status_flag(P, "patch factorization");
}

// Split every sweep of level L into nc time chunks (1: the plain sweep; nc is
// capped at N and rounded so that no chunk is empty).  The chunk buffers
// (transfer matrices, end values) grow on demand against the budget; the
// transfer matrices of the current factors are rebuilt.
void set_time_chunks(stwr_problem* P, Level& L, int nc) {
  nc = std::max(1, std::min(nc, L.N));
  if (L.H.thk > 0) nc = 1;   // the large-block sweep runs the plain forward substitution
  const int len = (L.N + nc - 1) / nc;
  nc = (L.N + len - 1) / len;
  if (nc > 1 && nc > L.chunk_cap) {
    const size_t bound = L.H.kdeg > 0 ? kHeatMaxNb : kMaxNbu;
    const size_t nT = (size_t)L.H.nv * nc * bound * bound, nW = (size_t)L.H.nv * nc * bound;
    const size_t need = (nT + 2 * nW) * sizeof(double);
    {
      std::lock_guard<std::mutex> g(P->ctx->mu);
      const uint64_t budget = P->ctx->budget;
      const size_t extra = need - L.chunk_bytes;
      if (budget && P->ctx->in_use + extra > budget)
        throw StwrError(STWR_ERR_BUDGET, "time-chunk buffers exceed the HBM budget");
      P->ctx->in_use += extra;
      P->bytes += extra;
    }
    if (L.chunk_buf) P->release(L.chunk_buf);
    L.chunk_buf = P->alloc<double>(nT + 2 * nW);
    L.chunk_bytes = need;
    L.chunk_cap = nc;
    L.pview.chunk_T = L.chunk_buf;
    L.pview.chunk_w_end = L.chunk_buf + nT;
    L.pview.chunk_w_in = L.chunk_buf + nT + nW;
  }
  L.pview.time_chunks = nc;
  L.pview.chunk_len = len;
  if (nc > 1 && L.fac_prec >= 0)
    HIPCHK(launch_patch_chunk_transfer(L.view, L.pview, L.fac_prec, L.fac, L.Mp, P->tab.e0, P->tab.e1, P->s()));
}

// Time chunks of level l: the options' fixed count, or (time_chunks = 0) the
// fastest of 1, 2, 4, ... chunks (at least two slabs each) by timing three
// sweeps of each with HIP events, chosen once per level; levels with more
// than kTuneMaxPatches patches keep the plain sweep.
void tune_time_chunks(stwr_problem* P, int l) {
  Level& L = P->lv[l];
  // a deterministic problem takes no timing-based choice: plain sweeps
  const int want = P->opts.time_chunks == 0 && P->opts.deterministic ? 1 : P->opts.time_chunks;
  if (want >= 1) { set_time_chunks(P, L, want); return; }
  if (L.chunk_choice > 0) { set_time_chunks(P, L, L.chunk_choice); return; }
  if (L.H.nv > kTuneMaxPatches || L.N < 4 || L.H.thk > 0) {
    L.chunk_choice = 1;
    set_time_chunks(P, L, 1);
    return;
  }
  HIPCHK(launch_fill(L.n_st, 0.0, L.r, P->s()));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int best = 1;
  float best_ms = 0.0f;
  for (int c = 1; c <= L.N / 2 && c <= kMaxTimeChunks; c *= 2) {
    set_time_chunks(P, L, c);
    auto sweep = [&]() {
      HIPCHK(launch_patch_sweep(L.view, L.pview, L.fac_prec, L.fac, L.Mp, P->tab.e0, P->tab.e1, L.r, L.Y, P->s()));
    };
    sweep();
    HIPCHK(hipEventRecord(e0, P->s()));
    for (int k = 0; k < 3; ++k) sweep();
    HIPCHK(hipEventRecord(e1, P->s()));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (c == 1 || ms < 0.97f * best_ms) { best = c; best_ms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  L.chunk_choice = best;
  set_time_chunks(P, L, best);
}

void patch_apply(stwr_problem* P, int l, const double* r, double* z) {
  require_factor(P, l);
  Level& L = P->lv[l];
  HIPCHK(launch_patch_sweep(L.view, L.pview, L.fac_prec, L.fac, L.Mp, P->tab.e0, P->tab.e1, r, L.Y, P->s()));
  HIPCHK(launch_patch_gather(L.view, L.pview, L.fac_prec, L.Y, 0, 0.0, 0.0, z, nullptr, nullptr, P->s()));
}

// Chebyshev-accelerated relaxation (three-term recurrence over [a, bnd]).
void relax(stwr_problem* P, int l, const double* b, double* x, int n_steps, double a, double bnd,
           bool x_is_zero) {
  require_factor(P, l);
  Level& L = P->lv[l];
  const double theta = 0.5 * (a + bnd), delta = 0.5 * (bnd - a);
  double rho_old = 0.0;
  // the FP32 interior sweep rounds its residual to FP32 on reading, so the
  // operator kernel may as well store it rounded: half the residual's bytes
  const bool f32r = L.rf && sweep_takes_f32_residual(L.view, L.pview, L.fac_prec);
  for (int k = 0; k < n_steps; ++k) {
    if (k == 0 && x_is_zero) {   // b - A 0 = b exactly
      KernelMark mark(P->ctx, 0);
      HIPCHK(launch_patch_sweep(L.view, L.pview, L.fac_prec, L.fac, L.Mp, P->tab.e0, P->tab.e1, b, L.Y, P->s()));
    } else if (f32r) {
      {
        KernelMark mark(P->ctx, 1);
        HIPCHK(launch_spmv_f32out(L.view, L.Jv, L.Mv, P->tab.e0, P->tab.e1, x, b, L.rf, P->s()));
      }
      KernelMark mark(P->ctx, 0);
      HIPCHK(launch_patch_sweep_f32r(L.view, L.pview, L.fac_prec, L.fac, L.Mp, P->tab.e0, P->tab.e1, L.rf, L.Y,
                                     P->s()));
    } else {
      spmv(P, l, x, b, L.r);
      KernelMark mark(P->ctx, 0);
      HIPCHK(launch_patch_sweep(L.view, L.pview, L.fac_prec, L.fac, L.Mp, P->tab.e0, P->tab.e1, L.r, L.Y, P->s()));
    }
    double c1, c2, rho;
    if (k == 0) {
      rho = delta / theta;
      c1 = 0.0;
      c2 = 1.0 / theta;
    } else {
      rho = 1.0 / (2.0 * theta / delta - rho_old);
      c1 = rho * rho_old;
      c2 = 2.0 * rho / delta;
    }
    {
      KernelMark mark(P->ctx, 2);
      // the last step's direction is not needed again: it is not stored
      HIPCHK(launch_patch_gather(L.view, L.pview, L.fac_prec, L.Y, k + 1 < n_steps ? 1 : 2, c1, c2, nullptr, L.d, x,
                                 P->s()));
    }
    rho_old = rho;
  }
}

void coarse_solve(stwr_problem* P, const double* b, double* x) {
  if (!P->assembled) throw StwrError(STWR_ERR_STATE, "operator not assembled");
  Level& C = P->lv.back();
  HIPCHK(launch_coarse_solve(C.view, C.Binv, C.Mv, P->tab.e0, P->tab.e1, b, x, C.gbuf, P->s()));
}

void require_smoothers(stwr_problem* P) {
  for (int l = 0; l + 1 < (int)P->lv.size(); ++l)
    if (!P->lv[l].has_lambda || P->lv[l].fac_prec < 0)
      throw StwrError(STWR_ERR_STATE, "smoothers not set up (call stwr_setup_smoothers)");
}

void vcycle(stwr_problem* P, const double* b0, double* x0) {
  const int L = (int)P->lv.size();
  const stwr_solver_opts& o = P->opts;
  require_smoothers(P);
  std::vector<const double*> bs(L);
  std::vector<double*> xs(L);
  for (int l = 0; l < L; ++l) {
    bs[l] = l == 0 ? b0 : P->lv[l].b;
    xs[l] = l == 0 ? x0 : P->lv[l].x;
  }
  if (L == 1) {
    coarse_solve(P, bs[0], xs[0]);
    return;
  }
  for (int l = 0; l + 1 < L; ++l) {
    Level& Lv = P->lv[l];
    HIPCHK(launch_fill(Lv.n_st, 0.0, xs[l], P->s()));
    const double lam = Lv.lambda;
    relax(P, l, bs[l], xs[l], o.nu_pre, o.cheb_lo * lam, o.cheb_hi * lam, true);
    spmv(P, l, xs[l], bs[l], Lv.r);
    Level& Cv = P->lv[l + 1];
    HIPCHK(launch_transfer(Cv.H.nf, Cv.N * Cv.NQ, Lv.R_ptr, Lv.R_col, Lv.R_val, Lv.r, P->lv[l + 1].b, 0, P->s()));
  }
  coarse_solve(P, bs[L - 1], xs[L - 1]);
  for (int l = L - 2; l >= 0; --l) {
    Level& Lv = P->lv[l];
    HIPCHK(launch_transfer(Lv.H.nf, Lv.N * Lv.NQ, Lv.P_ptr, Lv.P_col, Lv.P_val, xs[l + 1], xs[l], 1, P->s()));
    const double lam = Lv.lambda;
    relax(P, l, bs[l], xs[l], o.nu_post, o.cheb_lo * lam, o.cheb_hi * lam, false);
  }
}

// What a captured V-cycle depends on beyond device memory contents: the
// Chebyshev intervals, the smoother precisions and factor storage, the
// smoothing counts.
std::vector<double> vcycle_signature(stwr_problem* P) {
  const stwr_solver_opts& o = P->opts;
  std::vector<double> s = {(double)o.nu_pre, (double)o.nu_post, o.cheb_lo, o.cheb_hi};
  for (const Level& L : P->lv) {
    s.push_back(L.lambda);
    s.push_back((double)L.fac_prec);
    s.push_back((double)(uintptr_t)L.fac);
    s.push_back((double)L.pview.time_chunks);
    s.push_back((double)L.pview.chunk_len);
    s.push_back((double)(uintptr_t)L.chunk_buf);
  }
  return s;
}

void drop_vcycle_graph(stwr_problem* P) {
  if (P->vc_exec) (void)hipGraphExecDestroy(P->vc_exec);
  P->vc_exec = nullptr;
  P->vc_sig.clear();
}

// x = V-cycle(b).  With vcycle_graph the cycle is captured once and replayed
// on the context's stream between a copy into its input and out of its
// output.  Capture runs on a stream of the problem's own (thread-local mode,
// so other threads' streams are not affected), with the context's stream
// pointed at it while the launches are recorded.
void vcycle_apply(stwr_problem* P, const double* b, double* x) {
  require_smoothers(P);   // before any capture begins
  if (!P->opts.vcycle_graph || P->ctx->timing) {
    vcycle(P, b, x);
    return;
  }
  const int64_t n0 = P->lv[0].n_st;
  std::vector<double> sig = vcycle_signature(P);
  if (!P->vc_exec || sig != P->vc_sig) {
    drop_vcycle_graph(P);
    if (!P->vc_in) {
      P->vc_in = P->alloc<double>(n0);
      P->vc_out = P->alloc<double>(n0);
    }
    if (!P->vc_stream) HIPCHK(hipStreamCreateWithFlags(&P->vc_stream, hipStreamNonBlocking));
    // the capture stream starts after everything already queued on the context's
    HIPCHK(hipStreamSynchronize(P->s()));
    hipStream_t saved = P->ctx->stream;
    HIPCHK(hipStreamBeginCapture(P->vc_stream, hipStreamCaptureModeThreadLocal));
    P->ctx->stream = P->vc_stream;
    hipGraph_t g = nullptr;
    try {
      vcycle(P, P->vc_in, P->vc_out);
    } catch (...) {
      P->ctx->stream = saved;
      if (hipStreamEndCapture(P->vc_stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      throw;
    }
    P->ctx->stream = saved;
    HIPCHK(hipStreamEndCapture(P->vc_stream, &g));
    const hipError_t e = hipGraphInstantiate(&P->vc_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      P->vc_exec = nullptr;
      HIPCHK(e);
    }
    P->vc_sig = sig;
  }
  HIPCHK(hipMemcpyAsync(P->vc_in, b, n0 * sizeof(double), hipMemcpyDeviceToDevice, P->s()));
  HIPCHK(hipGraphLaunch(P->vc_exec, P->s()));
  HIPCHK(hipMemcpyAsync(x, P->vc_out, n0 * sizeof(double), hipMemcpyDeviceToDevice, P->s()));
}

// Eigenvalues of a small real upper-Hessenberg matrix by shifted complex QR
// iterations (Wilkinson shifts, deflation at the bottom).
std::vector<std::complex<double>> hessenberg_eigs(std::vector<double> Hr, int m) {
  using C = std::complex<double>;
  std::vector<C> A(m * m);
  for (int i = 0; i < m * m; ++i) A[i] = Hr[i];
  auto at = [&](int i, int j) -> C& { return A[i * m + j]; };
  std::vector<C> eig;
  int n = m;
  int iter = 0;
  while (n > 0) {
    if (n == 1) { eig.push_back(at(0, 0)); break; }
    const double sub = std::abs(at(n - 1, n - 2));
    const double scale = std::abs(at(n - 1, n - 1)) + std::abs(at(n - 2, n - 2));
    if (sub <= 1e-15 * (scale > 0 ? scale : 1.0) || iter > 500) {
      eig.push_back(at(n - 1, n - 1));
      --n;
      iter = 0;
      continue;
    }
    // Wilkinson shift from the trailing 2x2 block
    const C a = at(n - 2, n - 2), b = at(n - 2, n - 1), c = at(n - 1, n - 2), d = at(n - 1, n - 1);
    const C tr = a + d, det = a * d - b * c;
    const C disc = std::sqrt(tr * tr - 4.0 * det);
    const C l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
    C mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
    if (iter % 11 == 10) mu += C(sub, 0.0);   // exceptional shift
    for (int i = 0; i < n; ++i) at(i, i) -= mu;
    std::vector<C> cs(n - 1), sn(n - 1);
    for (int k = 0; k < n - 1; ++k) {
      const C x = at(k, k), y = at(k + 1, k);
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      C cc = 1.0, ss = 0.0;
      if (r > 0.0) { cc = x / r; ss = y / r; }
      cs[k] = cc; sn[k] = ss;
      for (int j = k; j < n; ++j) {
        const C u = at(k, j), v = at(k + 1, j);
        at(k, j) = std::conj(cc) * u + std::conj(ss) * v;
        at(k + 1, j) = -ss * u + cc * v;
      }
    }
    for (int k = 0; k < n - 1; ++k) {
      const C cc = cs[k], ss = sn[k];
      for (int i = 0; i <= std::min(k + 1, n - 1); ++i) {
        const C u = at(i, k), v = at(i, k + 1);
        at(i, k) = u * cc + v * ss;
        at(i, k + 1) = -u * std::conj(ss) + v * std::conj(cc);
      }
    }
    for (int i = 0; i < n; ++i) at(i, i) += mu;
    ++iter;
  }
  return eig;
}

double eig_estimate(stwr_problem* P, int l) {
  require_factor(P, l);
  Level& L = P->lv[l];
  const int steps = P->opts.eig_steps;
  const int64_t n = L.n_st;
  const int64_t ld = P->lv[0].n_st;
  if (steps + 1 > P->restart + 1 + P->restart) throw StwrError(STWR_ERR_ARG, "eig_steps exceeds workspace");
  // basis vectors live in the FGMRES workspace (V then Z)
  auto vec = [&](int j) -> double* { return j <= P->restart ? P->V + j * ld : P->Z + (j - P->restart - 1) * ld; };
  HIPCHK(launch_start_vector(n, vec(0), P->s()));
  const double nv0 = norm_host(P, n, vec(0));
  HIPCHK(launch_axpby(n, 1.0 / nv0, vec(0), 0.0, vec(0), P->s()));
  std::vector<double> H((steps + 1) * steps, 0.0);
  int m = steps;
  std::vector<double> hcol(steps + 2);
  for (int j = 0; j < steps; ++j) {
    double* w = vec(j + 1);
    spmv(P, l, vec(j), nullptr, L.r);
    patch_apply(P, l, L.r, w);
    for (int i = 0; i <= j; ++i) {
      HIPCHK(launch_mdot(n, 1, vec(i), 0, w, P->partial, P->dscal + i, P->s()));
      HIPCHK(launch_axpy_dev(n, P->dscal + i, -1.0, vec(i), w, P->s()));
    }
    HIPCHK(launch_mdot(n, 1, w, 0, w, P->partial, P->dscal + j + 1, P->s()));
    HIPCHK(hipMemcpyAsync(hcol.data(), P->dscal, (j + 2) * 8, hipMemcpyDeviceToHost, P->s()));
    HIPCHK(hipStreamSynchronize(P->s()));
    for (int i = 0; i <= j; ++i) H[i * steps + j] = hcol[i];
    const double h = std::sqrt(hcol[j + 1]);
    if (!std::isfinite(h)) throw StwrError(STWR_ERR_NONFINITE, "eigen-estimate produced a non-finite value");
    H[(j + 1) * steps + j] = h;
    if (h <= 1e-14 * std::fabs(H[0])) { m = j + 1; break; }
    HIPCHK(launch_axpby(n, 1.0 / h, w, 0.0, w, P->s()));
  }
  std::vector<double> Hm(m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Hm[i * m + j] = H[i * steps + j];
  auto ev = hessenberg_eigs(Hm, m);
  double lam = -1e300;
  for (auto& e : ev) lam = std::max(lam, e.real());
  L.lambda = lam;
  L.has_lambda = true;
  return lam;
}

void assemble(stwr_problem* P, const double* U) {
  const int L = (int)P->lv.size();
  for (int l = 0; l < L; ++l) {
    Level& Lv = P->lv[l];
    if (P->heat()) {
      // linear and state-independent: every entry is written
      HIPCHK(launch_heat_operator(Lv.view, P->d_tab, Lv.Jv, Lv.Mv, Lv.Kv, P->s()));
      Lv.fac_prec = -1;
      Lv.has_lambda = false;
      continue;
    }
    const double* Ul = U;
    if (l > 0) {
      Level& F = P->lv[l - 1];
      const double* src = l == 1 ? U : F.d;
      HIPCHK(launch_gather(Lv.H.nf, Lv.N * Lv.NQ, F.Tr.inject.empty() ? nullptr : F.inject, src, Lv.d, P->s()));
      Ul = Lv.d;
    }
    HIPCHK(launch_fill((int64_t)Lv.view.nnz * Lv.N * Lv.NQ * Lv.NQ, 0.0, Lv.Jv, P->s()));
    HIPCHK(launch_fill(Lv.view.nnz, 0.0, Lv.Mv, P->s()));
    HIPCHK(launch_assemble_jacobian(Lv.view, P->d_tab, P->mms, Ul, Lv.Jv, Lv.Mv, Lv.H.color_ptr, P->s()));
    Lv.fac_prec = -1;
    Lv.has_lambda = false;
  }
  Level& C = P->lv.back();
  HIPCHK(launch_fill((int64_t)C.view.coarse_slabs * C.coarse_mm * C.coarse_mm, 0.0, C.Binv, P->s()));
  HIPCHK(launch_coarse_build(C.view, C.Jv, C.Binv, P->s()));
  HIPCHK(launch_dense_inverse(C.view.coarse_slabs, C.coarse_mm, C.Binv, P->dstatus, C.perm, C.colbuf, C.rbuf,
                              P->s()));
  check_status_flag(P, "coarse factorization");
  P->assembled = true;
}

// F(U) on level 0: the nonlinear residual of eq. nsfem, or A U - b of the
// heat equation
void residual(stwr_problem* P, const double* U, double* F) {
  Level& L = P->lv[0];
  if (P->heat()) {
    spmv(P, 0, U, P->b0, F);                                  // b - A U
    HIPCHK(launch_axpby(L.n_st, -1.0, F, 0.0, F, P->s()));
    return;
  }
  HIPCHK(launch_fill(L.n_st, 0.0, F, P->s()));
  HIPCHK(launch_assemble_residual(L.view, P->d_tab, P->mms, U, F, L.H.color_ptr, P->s()));
}

void setup_smoothers(stwr_problem* P) {
  for (int l = 0; l + 1 < (int)P->lv.size(); ++l) {
    patch_factor(P, l, P->opts.smoother_prec);
    tune_time_chunks(P, l);
    eig_estimate(P, l);
  }
}

// Right-preconditioned restarted FGMRES with modified Gram-Schmidt.
// Stops when ||r|| <= max(rtol ||b||, atol).
void fgmres(stwr_problem* P, const double* b, double* x, stwr_stats* st, int* its_out, double* rel_out,
            double atol = 0.0, double rtol = -1.0, bool* conv_out = nullptr) {
  const stwr_solver_opts& o = P->opts;
  Level& L0 = P->lv[0];
  const int64_t n = L0.n_st;
  const int m = P->restart;
  HIPCHK(launch_fill(n, 0.0, x, P->s()));
  const double bnorm = norm_host(P, n, b);
  int its = 0;
  double rel = 0.0;
  if (bnorm == 0.0) {
    if (its_out) *its_out = 0;
    if (rel_out) *rel_out = 0.0;
    if (conv_out) *conv_out = true;
    return;
  }
  const double target = std::max((rtol >= 0.0 ? rtol : o.gmres_rtol) * bnorm, std::max(atol, o.gmres_atol));
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), hcol(m + 2), y(m);
  auto V = [&](int j) { return P->V + j * n; };
  auto Z = [&](int j) { return P->Z + j * n; };
  bool done = false;
  while (!done) {
    spmv(P, 0, x, b, V(0));
    const double beta = norm_host(P, n, V(0));
    rel = beta / bnorm;
    if (beta <= target || its >= o.gmres_maxit) break;
    HIPCHK(launch_axpby(n, 1.0 / beta, V(0), 0.0, V(0), P->s()));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      vcycle_apply(P, V(j), Z(j));
      project(P, 0, Z(j));
      spmv(P, 0, Z(j), nullptr, V(j + 1));
      for (int i = 0; i <= j; ++i) {
        HIPCHK(launch_mdot(n, 1, V(i), 0, V(j + 1), P->partial, P->dscal + i, P->s()));
        HIPCHK(launch_axpy_dev(n, P->dscal + i, -1.0, V(i), V(j + 1), P->s()));
      }
      HIPCHK(launch_mdot(n, 1, V(j + 1), 0, V(j + 1), P->partial, P->dscal + j + 1, P->s()));
      HIPCHK(hipMemcpyAsync(hcol.data(), P->dscal, (j + 2) * 8, hipMemcpyDeviceToHost, P->s()));
      HIPCHK(hipStreamSynchronize(P->s()));
      for (int i = 0; i <= j; ++i) H[i * m + j] = hcol[i];
      const double hn = std::sqrt(hcol[j + 1]);
      if (!std::isfinite(hn)) throw StwrError(STWR_ERR_NONFINITE, "FGMRES produced a non-finite value");
      H[(j + 1) * m + j] = hn;
      if (hn != 0.0) HIPCHK(launch_axpby(n, 1.0 / hn, V(j + 1), 0.0, V(j + 1), P->s()));
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
        H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t;
      }
      const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
      cs[j] = H[j * m + j] / den;
      sn[j] = H[(j + 1) * m + j] / den;
      H[j * m + j] = den;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      k = j + 1;
      rel = std::fabs(g[j + 1]) / bnorm;
      if (std::fabs(g[j + 1]) <= target || its >= o.gmres_maxit) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int c = i + 1; c < k; ++c) s -= H[i * m + c] * y[c];
      y[i] = s / H[i * m + i];
    }
    HIPCHK(hipMemcpyAsync(P->dscal, y.data(), k * 8, hipMemcpyHostToDevice, P->s()));
    HIPCHK(launch_gemv_cols(n, k, P->Z, n, P->dscal, x, P->s()));
    HIPCHK(hipStreamSynchronize(P->s()));
    if (std::fabs(g[k]) <= target || its >= o.gmres_maxit) done = true;
  }
  HIPCHK(hipStreamSynchronize(P->s()));
  if (its_out) *its_out = its;
  if (rel_out) *rel_out = rel;
  if (conv_out) *conv_out = rel * bnorm <= target;
  (void)st;
}

// Eisenstat and Walker's second forcing term (SIAM J. Sci. Comput. 17, 1996):
// eta_k = gamma (||F_k|| / ||F_{k-1}||)^alpha, kept at least
// gamma eta_{k-1}^alpha when that exceeds a threshold, at most eta_max; the
// parameters are the PETSc defaults (the paper cites the method only).
double ew_forcing(int k, double f, double f_prev, double eta_prev) {
  const double eta0 = 0.3, eta_max = 0.9, gamma = 1.0, threshold = 0.1;
  const double alpha = 0.5 * (1.0 + std::sqrt(5.0));
  if (k == 0) return eta0;
  double eta = gamma * std::pow(f / f_prev, alpha);
  const double safe = gamma * std::pow(eta_prev, alpha);
  if (safe > threshold) eta = std::max(eta, safe);
  return std::min(eta, eta_max);
}

}  // namespace impl
}  // namespace stwr


// ===========================================================================
extern "C" {

int32_t stwr_default_opts(stwr_solver_opts* o) {
  if (!o) return STWR_ERR_ARG;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->cheb_lo = 0.25;
  o->cheb_hi = 1.05;
  o->eig_steps = 10;
  o->smoother_prec = STWR_FP64;
  o->gmres_restart = 30;
  o->gmres_maxit = 200;
  o->gmres_rtol = 1e-10;
  o->newton_maxit = 20;
  o->newton_rtol = 1e-10;
  o->vcycle_graph = 1;
  o->newton_ew = 0;
  o->gmres_atol = 0.0;
  o->time_chunks = 0;
  o->factor_mfma = 1;
  o->deterministic = 0;
  return STWR_OK;
}

int32_t stwr_ctx_create(int32_t device, void* hip_stream, uint64_t hbm_budget, stwr_ctx** out) {
  return guarded(nullptr, [&]() -> int32_t {
    if (!out) throw StwrError(STWR_ERR_ARG, "null output");
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) throw StwrError(STWR_ERR_ARG, "bad device index");
    HIPCHK(hipSetDevice(device));
    resolve_scratch(device);
    auto* c = new stwr_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->budget = hbm_budget;
    *out = c;
    return STWR_OK;
  });
}

int32_t stwr_ctx_destroy(stwr_ctx* ctx) {
  delete ctx;
  return STWR_OK;
}

int32_t stwr_ctx_set_stream(stwr_ctx* ctx, void* hip_stream) {
  if (!ctx) return STWR_ERR_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return STWR_OK;
}

const char* stwr_last_error(const stwr_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : g_tls_error.c_str();
}

int32_t stwr_ctx_bytes_in_use(const stwr_ctx* ctx, uint64_t* bytes) {
  if (!ctx || !bytes) return STWR_ERR_ARG;
  *bytes = ctx->in_use;
  return STWR_OK;
}

int32_t stwr_ctx_set_alloc_mode(stwr_ctx* ctx, int32_t stream_ordered) {
  if (!ctx) return STWR_ERR_ARG;
  ctx->stream_alloc = stream_ordered != 0;
  return STWR_OK;
}

int32_t stwr_ctx_read_rate(stwr_ctx* ctx, const void* buf, uint64_t bytes, int32_t reps, double* gbs) {
  if (!ctx || !buf || !gbs || bytes < ((uint64_t)64 << 20) || bytes % 16 != 0 || reps < 1) return STWR_ERR_ARG;
  return guarded(ctx, [&]() -> int32_t {
    HIPCHK(hipSetDevice(ctx->device));
    int cus = 0;
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int grid = 8 * (cus > 0 ? cus : 1);   // eight 256-thread workgroups per CU
    float* out = nullptr;
    HIPCHK(hipMalloc(&out, (size_t)grid * 256 * sizeof(float)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best = 0.0f;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    if (err == hipSuccess) err = launch_stream_read(buf, (int64_t)bytes, grid, out, ctx->stream);   // warm-up
    for (int k = 0; k < reps && err == hipSuccess; ++k) {
      err = hipEventRecord(e0, ctx->stream);
      if (err == hipSuccess) err = launch_stream_read(buf, (int64_t)bytes, grid, out, ctx->stream);
      if (err == hipSuccess) err = hipEventRecord(e1, ctx->stream);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err == hipSuccess && (k == 0 || ms < best)) best = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    HIPCHK(err);
    *gbs = best > 0.0f ? (double)bytes / ((double)best * 1e6) : 0.0;
    return STWR_OK;
  });
}

int32_t stwr_ctx_set_timing(stwr_ctx* ctx, int32_t enable) {
  if (!ctx) return STWR_ERR_ARG;
  ctx->timing = enable != 0;
  return STWR_OK;
}

int32_t stwr_ctx_kernel_times(stwr_ctx* ctx, double* ms, int64_t* launches) {
  if (!ctx || !ms || !launches) return STWR_ERR_ARG;
  return guarded(ctx, [&]() -> int32_t {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 3; ++k) {
      double tot = 0.0;
      for (auto& pr : ctx->marks[k]) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, pr.first, pr.second));
        tot += t;
        ctx->pool.push_back(pr.first);
        ctx->pool.push_back(pr.second);
      }
      ms[k] = tot;
      launches[k] = (int64_t)ctx->marks[k].size();
      ctx->marks[k].clear();
    }
    return STWR_OK;
  });
}

int32_t stwr_problem_bytes(const stwr_problem_desc* desc, const stwr_solver_opts* opts, uint64_t* bytes) {
  return guarded(nullptr, [&]() -> int32_t {
    check_desc(desc);
    check_opts(opts);
    if (!bytes) throw StwrError(STWR_ERR_ARG, "null output");
    std::vector<Level> lv;
    build_levels(desc, lv);
    *bytes = plan_bytes(desc, opts, lv);
    return STWR_OK;
  });
}

int32_t stwr_problem_n_st(const stwr_problem_desc* desc, int64_t* n_st) {
  return guarded(nullptr, [&]() -> int32_t {
    check_desc(desc);
    if (!n_st) throw StwrError(STWR_ERR_ARG, "null output");
    *n_st = free_dofs(desc, desc->mesh_n) * desc->n_slabs * (desc->q + 1);
    return STWR_OK;
  });
}

int32_t stwr_level_patches(int32_t mesh_n, int32_t degree, int64_t* counts, int32_t* patch_ptr,
                           int32_t* patch_dofs) {
  return guarded(nullptr, [&]() -> int32_t {
    if (!counts || mesh_n < 1 || degree < 1 || degree > kThK) throw StwrError(STWR_ERR_ARG, "bad arguments");
    HostLevel H;
    if (degree == kThK) build_level_th(mesh_n, kThK, H);
    else build_level(mesh_n, H);
    int mx = 0;
    for (int v = 0; v < H.nv; ++v) mx = std::max(mx, H.patch_ptr[v + 1] - H.patch_ptr[v]);
    // structural nonzeros of the patch of the vertex nearest the centre (the
    // pressure-pressure pairs, which the operator never fills, left out)
    const int c = H.n1 / 2, v = c + H.n1 * c;
    const int nb = H.patch_ptr[v + 1] - H.patch_ptr[v], nbu = H.patch_nbu[v];
    int64_t pnz = 0;
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j)
        pnz += (i < nbu || j < nbu) && H.patch_nz[H.patch_nz_off[v] + (int64_t)i * nb + j] >= 0;
    counts[0] = H.nf;
    counts[1] = H.nv;
    counts[2] = (int64_t)H.patch_dofs.size();
    counts[3] = H.row_ptr[H.nf];
    counts[4] = mx;
    counts[5] = pnz;
    counts[6] = H.nc;
    if (patch_ptr) std::copy(H.patch_ptr.begin(), H.patch_ptr.end(), patch_ptr);
    if (patch_dofs) std::copy(H.patch_dofs.begin(), H.patch_dofs.end(), patch_dofs);
    return STWR_OK;
  });
}

int32_t stwr_level_transfer(int32_t mesh_n, int32_t degree, int64_t* counts, int32_t* p_ptr, int32_t* p_col,
                            double* p_val, int32_t* inject) {
  return guarded(nullptr, [&]() -> int32_t {
    if (!counts || mesh_n < 2 || mesh_n % 2 || degree < 1 || degree > kThK)
      throw StwrError(STWR_ERR_ARG, "bad arguments");
    HostLevel F, C;
    HostTransfer T;
    if (degree == kThK) {
      build_level_th(mesh_n, kThK, F);
      build_level_th(mesh_n / 2, kThK, C);
      build_transfer_th(F, C, T);
    } else {
      build_level(mesh_n, F);
      build_level(mesh_n / 2, C);
      build_transfer(F, C, T);
    }
    counts[0] = F.nf;
    counts[1] = C.nf;
    counts[2] = (int64_t)T.p_col.size();
    if (p_ptr) std::copy(T.p_ptr.begin(), T.p_ptr.end(), p_ptr);
    if (p_col) std::copy(T.p_col.begin(), T.p_col.end(), p_col);
    if (p_val) std::copy(T.p_val.begin(), T.p_val.end(), p_val);
    if (inject) std::copy(T.inject.begin(), T.inject.end(), inject);
    return STWR_OK;
  });
}

int32_t stwr_mesh_info(int32_t mesh_n, int64_t* out) {
  return guarded(nullptr, [&]() -> int32_t {
    if (!out || mesh_n < 1) throw StwrError(STWR_ERR_ARG, "bad arguments");
    HostLevel H;
    build_level(mesh_n, H);
    std::memset(out, 0, 52 * sizeof(int64_t));
    out[0] = H.nf;
    out[1] = H.nn;
    out[2] = H.nv;
    out[3] = H.nc;
    out[4] = H.row_ptr[H.nf];
    out[5] = H.nv;
    out[6] = (int64_t)H.patch_dofs.size();
    int mx = 0;
    for (int v = 0; v < H.nv; ++v) {
      const int nb = H.patch_ptr[v + 1] - H.patch_ptr[v];
      mx = std::max(mx, nb);
      if (nb < 40) out[12 + nb]++;
    }
    out[7] = mx;
    // nonzeros of the patch of the vertex nearest the centre
    const int c = H.n1 / 2;
    const int v = c + H.n1 * c;
    const int s0 = H.patch_ptr[v], nb = H.patch_ptr[v + 1] - s0, nbu = H.patch_nbu[v];
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) {
        if (H.patch_nz[H.patch_nz_off[v] + (int64_t)i * nb + j] < 0) continue;
        if (i < nbu && j < nbu) out[8]++;
        else if (i < nbu) out[9]++;
        else if (j < nbu) out[10]++;
      }
    int distinct = 0;
    for (int k = 0; k < 40; ++k) distinct += out[12 + k] > 0;
    out[11] = distinct;
    return STWR_OK;
  });
}

int32_t stwr_problem_create(stwr_ctx* ctx, const stwr_problem_desc* desc, const stwr_solver_opts* opts,
                            stwr_problem** out) {
  return guarded(ctx, [&]() -> int32_t {
    if (!ctx || !out) throw StwrError(STWR_ERR_ARG, "null argument");
    check_desc(desc);
    check_opts(opts);
    HIPCHK(hipSetDevice(ctx->device));
    std::unique_ptr<stwr_problem> P(new stwr_problem());
    P->ctx = ctx;
    P->desc = *desc;
    P->opts = *opts;
    P->psi_ab.assign(desc->psi_ab, desc->psi_ab + 2 * desc->n_psi_modes);
    P->psi_coef.assign(desc->psi_coef, desc->psi_coef + 3 * desc->n_psi_modes);
    P->p_ab.assign(desc->p_ab, desc->p_ab + 2 * desc->n_p_modes);
    P->p_coef.assign(desc->p_coef, desc->p_coef + 3 * desc->n_p_modes);
    P->desc.psi_ab = nullptr; P->desc.psi_coef = nullptr; P->desc.p_ab = nullptr; P->desc.p_coef = nullptr;
    build_levels(desc, P->lv);
    const uint64_t need = plan_bytes(desc, opts, P->lv);
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      if (ctx->budget && ctx->in_use + need > ctx->budget)
        throw StwrError(STWR_ERR_BUDGET, "problem needs " + std::to_string(need) + " bytes; budget left " +
                                             std::to_string(ctx->budget - ctx->in_use));
      ctx->in_use += need;
    }
    P->bytes = need;
    try {
      build_ref_tables(desc->q, desc->temporal_nodes, P->tab);
      if (is_heat(desc)) build_pk_tables(desc->degree, P->tab);
      if (th_degree(desc) == kThK) build_th_tables(kThK, P->tab);
      P->d_tab = P->alloc<RefTables>(1);
      HIPCHK(hipMemcpyAsync(P->d_tab, &P->tab, sizeof(RefTables), hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      P->mms.n_psi = desc->n_psi_modes;
      P->mms.n_p = desc->n_p_modes;
      P->mms.psi_ab = P->upload(P->psi_ab);
      P->mms.psi_coef = P->upload(P->psi_coef);
      P->mms.p_ab = P->upload(P->p_ab);
      P->mms.p_coef = P->upload(P->p_coef);
      P->mms.reynolds = desc->reynolds;
      P->mms.flow = desc->flow;
      const int L = (int)P->lv.size();
      for (int l = 0; l < L; ++l) upload_level(P.get(), P->lv[l], l == L - 1);
      for (int l = 0; l + 1 < L; ++l)
        P->lv[l].fac_budgeted = (size_t)fac_elems(P->lv[l].H, P->lv[l].N, P->lv[l].NQ, opts->smoother_prec) *
                                (opts->smoother_prec == STWR_FP32 ? 4 : 8);
      for (int l = 0; l + 1 < L; ++l) P->lv[l].inject = P->upload(P->lv[l].Tr.inject);
      P->restart = opts->gmres_restart;
      const int64_t n0 = P->lv[0].n_st;
      P->V = P->alloc<double>((size_t)(P->restart + 1) * n0);
      P->Z = P->alloc<double>((size_t)P->restart * n0);
      P->dscal = P->alloc<double>(256 + (size_t)desc->n_slabs * (desc->q + 1));
      P->partial = P->alloc<double>(256 * 256);
      P->dstatus = P->alloc<int>(4);
      HIPCHK(hipMemsetAsync(P->dstatus, 0, 4 * sizeof(int), ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      if (is_heat(desc)) {
        // the heat operator does not depend on the state: assemble it and
        // the right-hand side once
        P->b0 = P->alloc<double>((size_t)n0);
        assemble(P.get(), nullptr);
        HIPCHK(launch_heat_rhs(P->lv[0].view, P->d_tab, P->lv[0].Mv, P->b0, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
      }
      // host copies no longer needed on the device side can be dropped
      for (auto& Lv : P->lv) {
        std::vector<int>().swap(Lv.H.cell_nz);
        std::vector<int>().swap(Lv.H.patch_nz);
        std::vector<int>().swap(Lv.H.dof_slot);
      }
    } catch (...) {
      for (auto& b : P->bufs) P->free_one(b.p);
      P->bufs.clear();
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->in_use -= need;
      throw;
    }
    *out = P.release();
    return STWR_OK;
  });
}

int32_t stwr_problem_destroy(stwr_problem* p) {
  if (!p) return STWR_OK;
  (void)hipStreamSynchronize(p->s());
  drop_vcycle_graph(p);
  if (p->vc_stream) (void)hipStreamDestroy(p->vc_stream);
  for (auto& b : p->bufs) p->free_one(b.p);
  if (p->ctx->stream_alloc) (void)hipStreamSynchronize(p->s());
  {
    std::lock_guard<std::mutex> g(p->ctx->mu);
    p->ctx->in_use -= std::min(p->ctx->in_use, p->bytes);
  }
  delete p;
  return STWR_OK;
}

int32_t stwr_problem_sizes(const stwr_problem* p, int32_t level, int64_t* n_st, int64_t* n_spatial_free,
                           int32_t* n_patches) {
  if (!p || level < 0 || level >= (int)p->lv.size()) return STWR_ERR_ARG;
  const Level& L = p->lv[level];
  if (n_st) *n_st = L.n_st;
  if (n_spatial_free) *n_spatial_free = L.H.nf;
  if (n_patches) *n_patches = L.H.nv;
  return STWR_OK;
}

int32_t stwr_patch_sizes(const stwr_problem* p, int32_t level, int32_t* nb) {
  if (!p || !nb || level < 0 || level >= (int)p->lv.size()) return STWR_ERR_ARG;
  const HostLevel& H = p->lv[level].H;
  for (int v = 0; v < H.nv; ++v) nb[v] = H.patch_ptr[v + 1] - H.patch_ptr[v];
  return STWR_OK;
}

int32_t stwr_level_time_chunks(const stwr_problem* p, int32_t level, int32_t* chunks) {
  if (!p || !chunks || level < 0 || level >= (int)p->lv.size()) return STWR_ERR_ARG;
  const int c = p->lv[level].pview.time_chunks;
  *chunks = c > 1 ? c : 1;
  return STWR_OK;
}

int32_t stwr_set_opts(stwr_problem* p, const stwr_solver_opts* opts) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    check_opts(opts);
    if (opts->gmres_restart != p->restart) throw StwrError(STWR_ERR_ARG, "gmres_restart is fixed at creation");
    if (opts->smoother_prec != p->opts.smoother_prec)
      for (auto& L : p->lv) { L.fac_prec = -1; L.has_lambda = false; }
    if (opts->time_chunks != p->opts.time_chunks || opts->smoother_prec != p->opts.smoother_prec ||
        opts->deterministic != p->opts.deterministic)
      for (auto& L : p->lv) L.chunk_choice = 0;
    p->opts = *opts;
    return STWR_OK;
  });
}

int32_t stwr_nonlinear_residual(stwr_problem* p, const double* U, double* F) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (!U || !F) throw StwrError(STWR_ERR_ARG, "null vector");
    residual(p, U, F);
    return STWR_OK;
  });
}

int32_t stwr_linear_rhs(stwr_problem* p, double* b) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (!b) throw StwrError(STWR_ERR_ARG, "null vector");
    Level& L = p->lv[0];
    if (p->heat()) {
      HIPCHK(hipMemcpyAsync(b, p->b0, L.n_st * 8, hipMemcpyDeviceToDevice, p->s()));
      return STWR_OK;
    }
    // -F(0): the residual at zero, negated (L.x is scratch outside solves)
    HIPCHK(launch_fill(L.n_st, 0.0, L.x, p->s()));
    residual(p, L.x, b);
    HIPCHK(launch_axpby(L.n_st, -1.0, b, 0.0, b, p->s()));
    return STWR_OK;
  });
}

int32_t stwr_velocity_l2_error(stwr_problem* p, const double* U, double* err) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (!U || !err) throw StwrError(STWR_ERR_ARG, "null pointer");
    if (p->heat()) throw StwrError(STWR_ERR_STATE, "no velocity in the heat equation");
    Level& L = p->lv[0];
    // per-(cell, slab) partial sums in the finest level's residual buffer
    // (nc N <= n_st), the total in the scalar buffer
    HIPCHK(launch_velocity_error(L.view, p->d_tab, p->mms, U, L.r, p->dscal, p->s()));
    double h = 0.0;
    HIPCHK(hipMemcpyAsync(&h, p->dscal, 8, hipMemcpyDeviceToHost, p->s()));
    HIPCHK(hipStreamSynchronize(p->s()));
    *err = std::sqrt(h);
    return STWR_OK;
  });
}

int32_t stwr_expand(stwr_problem* p, const double* U, double* full) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (!U || !full) throw StwrError(STWR_ERR_ARG, "null vector");
    if (p->heat()) throw StwrError(STWR_ERR_STATE, "the heat equation has no eliminated DoFs");
    if (p->lv[0].H.thk > 0) throw StwrError(STWR_ERR_STATE, "no full nodal vector for P3-P2 problems");
    HIPCHK(launch_expand(p->lv[0].view, p->d_tab, p->mms, U, full, p->s()));
    return STWR_OK;
  });
}

int32_t stwr_assemble(stwr_problem* p, const double* U) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (!U && !p->heat()) throw StwrError(STWR_ERR_ARG, "null vector");
    assemble(p, U);
    return STWR_OK;
  });
}

int32_t stwr_get_operator(stwr_problem* p, int32_t level, int64_t* nnz, int32_t* row_ptr, int32_t* col,
                          double* values, double* mass) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    Level& L = level_at(p, level);
    const int64_t nz = L.view.nnz;
    if (nnz) *nnz = nz;
    if (row_ptr) std::memcpy(row_ptr, L.H.row_ptr.data(), (L.H.nf + 1) * sizeof(int));
    if (col) std::memcpy(col, L.H.col.data(), nz * sizeof(int));
    if (values || mass) {
      if (!p->assembled) throw StwrError(STWR_ERR_STATE, "operator not assembled");
      if (values) HIPCHK(hipMemcpyAsync(values, L.Jv, (size_t)nz * L.N * L.NQ * L.NQ * 8, hipMemcpyDeviceToHost, p->s()));
      if (mass) HIPCHK(hipMemcpyAsync(mass, L.Mv, (size_t)nz * 8, hipMemcpyDeviceToHost, p->s()));
      HIPCHK(hipStreamSynchronize(p->s()));
    }
    return STWR_OK;
  });
}

int32_t stwr_apply(stwr_problem* p, int32_t level, const double* x, double* y) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    level_at(p, level);
    if (!x || !y) throw StwrError(STWR_ERR_ARG, "null vector");
    if (!p->assembled) throw StwrError(STWR_ERR_STATE, "operator not assembled");
    spmv(p, level, x, nullptr, y);
    return STWR_OK;
  });
}

int32_t stwr_residual(stwr_problem* p, int32_t level, const double* b, const double* x, double* r) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    level_at(p, level);
    if (!x || !b || !r) throw StwrError(STWR_ERR_ARG, "null vector");
    if (!p->assembled) throw StwrError(STWR_ERR_STATE, "operator not assembled");
    spmv(p, level, x, b, r);
    return STWR_OK;
  });
}

int32_t stwr_patch_factor(stwr_problem* p, int32_t level, int32_t prec) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    level_at(p, level);
    patch_factor(p, level, prec);
    return STWR_OK;
  });
}

int32_t stwr_patch_apply(stwr_problem* p, int32_t level, const double* r, double* z) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    level_at(p, level);
    if (!r || !z) throw StwrError(STWR_ERR_ARG, "null vector");
    patch_apply(p, level, r, z);
    return STWR_OK;
  });
}

int32_t stwr_patch_apply_noalloc(stwr_problem* p, int32_t level, const double* r, double* z) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    Level& L = level_at(p, level);
    if (!r || !z) throw StwrError(STWR_ERR_ARG, "null vector");
    if (level >= (int)p->lv.size() - 1 || L.y_off.empty())
      throw StwrError(STWR_ERR_ARG, "the coarsest level has no smoother");
    const uint64_t need = (uint64_t)L.y_off.back() * sizeof(double);
    if (need > kScratchBytes)
      throw StwrError(STWR_ERR_ARG, "patch outputs of level " + std::to_string(level) + " need " +
                                        std::to_string(need) + " bytes, more than the " +
                                        std::to_string(kScratchBytes) + "-byte scratch area");
    double* ybuf = scratch_of(p->ctx->device);
    if (!ybuf) throw StwrError(STWR_ERR_STATE, "scratch area not resolved on this device");
    require_factor(p, level);
    HIPCHK(launch_patch_sweep(L.view, L.pview, L.fac_prec, L.fac, L.Mp, p->tab.e0, p->tab.e1, r, ybuf, p->s()));
    HIPCHK(launch_patch_gather(L.view, L.pview, L.fac_prec, ybuf, 0, 0.0, 0.0, z, nullptr, nullptr, p->s()));
    return STWR_OK;
  });
}

int32_t stwr_eig_estimate(stwr_problem* p, int32_t level, double* lambda) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    level_at(p, level);
    const double lam = eig_estimate(p, level);
    if (lambda) *lambda = lam;
    return STWR_OK;
  });
}

int32_t stwr_relax(stwr_problem* p, int32_t level, const double* b, double* x, int32_t n_steps, double a,
                   double bnd) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    level_at(p, level);
    if (!b || !x || n_steps < 0 || !(bnd > a) || !(a > 0.0)) throw StwrError(STWR_ERR_ARG, "bad relax arguments");
    relax(p, level, b, x, n_steps, a, bnd, false);
    return STWR_OK;
  });
}

int32_t stwr_restrict(stwr_problem* p, int32_t fine_level, const double* rf, double* rc) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (fine_level < 0 || fine_level + 1 >= (int)p->lv.size()) throw StwrError(STWR_ERR_ARG, "level out of range");
    if (!rf || !rc) throw StwrError(STWR_ERR_ARG, "null vector");
    Level& F = p->lv[fine_level];
    Level& C = p->lv[fine_level + 1];
    HIPCHK(launch_transfer(C.H.nf, C.N * C.NQ, F.R_ptr, F.R_col, F.R_val, rf, rc, 0, p->s()));
    return STWR_OK;
  });
}

int32_t stwr_prolong_add(stwr_problem* p, int32_t fine_level, const double* ec, double* xf) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (fine_level < 0 || fine_level + 1 >= (int)p->lv.size()) throw StwrError(STWR_ERR_ARG, "level out of range");
    if (!ec || !xf) throw StwrError(STWR_ERR_ARG, "null vector");
    Level& F = p->lv[fine_level];
    HIPCHK(launch_transfer(F.H.nf, F.N * F.NQ, F.P_ptr, F.P_col, F.P_val, ec, xf, 1, p->s()));
    return STWR_OK;
  });
}

int32_t stwr_coarse_solve(stwr_problem* p, const double* b, double* x) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (!b || !x) throw StwrError(STWR_ERR_ARG, "null vector");
    coarse_solve(p, b, x);
    return STWR_OK;
  });
}

int32_t stwr_setup_smoothers(stwr_problem* p) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    setup_smoothers(p);
    return STWR_OK;
  });
}

int32_t stwr_vcycle(stwr_problem* p, const double* b, double* x) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (!b || !x) throw StwrError(STWR_ERR_ARG, "null vector");
    if (!p->assembled) throw StwrError(STWR_ERR_STATE, "operator not assembled");
    vcycle_apply(p, b, x);
    return STWR_OK;
  });
}

int32_t stwr_project_pressure(stwr_problem* p, int32_t level, double* x) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    level_at(p, level);
    if (!x) throw StwrError(STWR_ERR_ARG, "null vector");
    project(p, level, x);
    return STWR_OK;
  });
}

int32_t stwr_fgmres(stwr_problem* p, const double* b, double* x, stwr_stats* stats) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (!b || !x) throw StwrError(STWR_ERR_ARG, "null vector");
    if (!p->assembled) throw StwrError(STWR_ERR_STATE, "operator not assembled");
    int its = 0;
    double rel = 0.0;
    bool conv = false;
    const double t0 = now_s();
    fgmres(p, b, x, stats, &its, &rel, 0.0, -1.0, &conv);
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->linear_its_total = its;
      stats->linear_its[0] = its;
      stats->final_rel_residual = rel;
      stats->solve_seconds = now_s() - t0;
      for (int l = 0; l < (int)p->lv.size() && l < STWR_MAX_LEVELS; ++l) stats->lambda[l] = p->lv[l].lambda;
    }
    if (!conv) return fail(p->ctx, STWR_ERR_NOT_CONVERGED, "FGMRES reached its iteration limit");
    return STWR_OK;
  });
}


int32_t stwr_newton_solve(stwr_problem* p, double* U, stwr_stats* stats) {
  if (!p) return STWR_ERR_ARG;
  return guarded(p->ctx, [&]() -> int32_t {
    if (!U) throw StwrError(STWR_ERR_ARG, "null vector");
    const stwr_solver_opts& o = p->opts;
    Level& L0 = p->lv[0];
    const int64_t n = L0.n_st;
    // F lives in L0.b, the correction in L0.x (both level-0 work vectors are
    // free outside V-cycles, which take their level-0 vectors from FGMRES).
    double* F = L0.b;
    double* dU = L0.x;
    stwr_stats local{};
    stwr_stats& st = stats ? *stats : local;
    std::memset(&st, 0, sizeof(st));
    auto resid = [&]() {
      residual(p, U, F);
      return norm_host(p, n, F);
    };
    double f = resid();
    const double f0 = f;
    st.fnorm[0] = f;
    int k = 0;
    bool converged = f0 == 0.0;
    double eta = 0.0;
    for (; k < o.newton_maxit && !converged; ++k) {
      const double ts = now_s();
      assemble(p, U);
      setup_smoothers(p);
      st.setup_seconds += now_s() - ts;
      // F is recomputed after the update, so it can hold the right-hand side -F
      HIPCHK(launch_axpby(n, -1.0, F, 0.0, F, p->s()));
      int its = 0;
      double rel = 0.0;
      const double tk = now_s();
      // absolute floor of the linear solve: three orders below the Newton
      // target (a relative tolerance alone would chase rounding once F is tiny)
      double rtol = -1.0;   // options' gmres_rtol
      if (o.newton_ew) rtol = eta = ew_forcing(k, f, k > 0 ? st.fnorm[k - 1] : f0, eta);
      fgmres(p, F, dU, &st, &its, &rel, 1e-3 * o.newton_rtol * f0, rtol);
      st.solve_seconds += now_s() - tk;
      HIPCHK(launch_axpby(n, 1.0, dU, 1.0, U, p->s()));
      st.linear_its[k] = its;
      st.linear_rel[k] = rel;
      st.linear_its_total += its;
      f = resid();
      st.fnorm[k + 1] = f;
      converged = f <= o.newton_rtol * f0;
      if (f > kNewtonDiverged * f0) {   // full steps that leave the basin: give up early
        ++k;
        break;
      }
    }
    st.newton_its = k;
    for (int l = 0; l < (int)p->lv.size() && l < STWR_MAX_LEVELS; ++l) st.lambda[l] = p->lv[l].lambda;
    if (!converged)
      return fail(p->ctx, STWR_ERR_NOT_CONVERGED,
                  f > kNewtonDiverged * f0 ? "Newton diverged" : "Newton reached its iteration limit");
    return STWR_OK;
  });
}

}  // extern "C"
