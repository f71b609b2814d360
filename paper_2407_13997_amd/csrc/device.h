// Device-side views of a level and launch wrappers for the gfx950 kernels.
// Every launcher enqueues on the stream it is given and returns the HIP error
// of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "host_setup.h"

namespace stwr {

// Manufactured-solution modes in device memory (see stwr.h for the family).
struct MmsDev {
  int n_psi, n_p;
  const int* psi_ab;      // n_psi x 2
  const double* psi_coef; // n_psi x 3  (c, w, th)
  const int* p_ab;        // n_p x 2
  const double* p_coef;   // n_p x 3
  double reynolds;
  int flow;               // 0: the modes; 1: Chorin problem; 2: lid-driven cavity (modes unused)
};

// Slab-end values of the temporal Lagrange basis, e0[a] = phi_a(0) and
// e1[a] = phi_a(1), passed to kernels by value (first NQ entries used).
struct TimeEnds {
  double e0[kMaxNQ], e1[kMaxNQ];
};
inline TimeEnds time_ends(int NQ, const double* e0, const double* e1) {
  TimeEnds t{};
  for (int a = 0; a < NQ && a < kMaxNQ; ++a) {
    t.e0[a] = e0[a];
    t.e1[a] = e1[a];
  }
  return t;
}

// Read-only structure of one level on the device.
struct LevelView {
  int M, nf, po, nv, nc, N, NQ;
  double dt, h;
  int64_t nnz;
  const int* row_ptr;
  const int* col;
  const int* cells;      // nc x 3
  const int* cell_p2;    // nc x 6
  const int* cell_dofs;  // nc x 15
  const int* cell_nz;    // nc x 225
  const int* node_free;  // nn
  int n2, n1;
  // heat equation (kdeg = k >= 1; 0 for Navier-Stokes): cells hold nloc
  // lattice nodes, n2 is the lattice width, node_cell the (cell * nloc +
  // local) slots of each node
  int kdeg, nloc;
  const int* node_cell_ptr;
  const int* node_cell;
  int nbord;             // constraint rows bordering a coarsest slab block: q+1 with pressure, else 0
  int coarse_slabs;      // coarsest slab blocks stored: N, or 1 when every slab's block is the same
  // Taylor-Hood P_{k+1}-P_k of the general path (thk = k = 2; 0 for P2-P1):
  // velocity lattice width n2, pressure lattice width n3, the nlv velocity and
  // nlp pressure lattice nodes of each cell (lattice order)
  int thk, n3, nlv, nlp;
  const int* cell_vn;
  const int* cell_pn;
  // assembly by colour: the cells dealt into 8 colours, no two cells of a
  // colour sharing a vertex (so no DoF), listed colour by colour
  // (color_cells, nc entries); an assembly launch covers one colour from
  // color_first, so no other workgroup of the launch writes an entry a
  // workgroup adds to, and the colours run in a fixed order
  const int* color_cells;
  int color_first;
};

// cell of the calling workgroup of an assembly launch (one workgroup per
// (cell, slab) of one colour, slab fastest)
__device__ __forceinline__ int cell_of(const LevelView& L) {
  return L.color_cells[L.color_first + (int)(blockIdx.x / L.N)];
}
// a cell's contribution to an assembled entry: a plain addition (the
// launch's other workgroups touch other entries), so the sums come out the
// same bit for bit every run; measured faster than one launch over every
// cell with FP64 atomic additions (all levels of the 128 x 128 workload:
// 0.087 s against 0.106 s)
__device__ __forceinline__ void scatter_add(const LevelView&, double* p, double v) { *p += v; }

// Time chunks of one sweep (see k_patch_sweep): chunk c covers slabs
// [c len, min(N, (c+1) len)); outputs are written for chunks <= y_max;
// w_in / w_end: incoming and final slab-end values, [patch][chunk][bound]
// (bound: kMaxNbu, or kHeatMaxNb for the heat equation), or null.
struct ChunkArgs {
  int len, first, y_max, n_chunks;
  const double* w_in;
  double* w_end;
};

struct PatchView {
  int n_patch;
  const int* patch_ptr;
  const int* patch_dofs;
  const int* patch_nbu;
  const int64_t* patch_nz_off;
  const int* patch_nz;
  const int64_t* fac_off;   // n_patch + 1, element offset of each patch's block inside a slab
  int64_t slab_stride;      // elements of one slab's blocks (all patches): blocks are [slab][patch]
  int fac_slabs;            // slabs with their own blocks: N, or 1 when every slab's blocks are
                            // the same (the heat equation; slab_stride is then 0)
  int factor_mfma;          // 1: FP32 blocks over 64 rows by the MFMA blocked Gauss-Jordan
  const int64_t* y_off;     // n_patch + 1, offsets into the patch output buffer
  const int64_t* mp_off;    // n_patch + 1, offsets of the patch mass blocks
  const int* dof_ptr;
  const int* dof_slot;
  const int* slot_patch;
  const int* order;         // n_patch, by decreasing size: interior (full-size) patches first
  int n_full;               // number of full-size patches at the front of order
  int n_big;                // number of patches with (q+1) nb > 64 at the front of order
  // cyclic reduction in time: time_chunks > 1 splits every sweep into that
  // many chunks of chunk_len slabs (buffers as in ChunkArgs; chunk_T holds
  // the chunk transfer matrices, [patch][chunk][bound^2])
  int time_chunks, chunk_len;
  const double* chunk_T;
  double* chunk_w_end;
  double* chunk_w_in;
};

// Storage of one inverted m x m slab block for the patch sweep, in T-typed
// elements.  Columns are grouped in panels of VW = 16 / sizeof(T) (one 16-byte
// vector); the panels are dealt to wavefronts, at most panels_per_wave each.
// Inside wavefront w's share (PH_w panels): rows r < r1 = min(m, 64) hold
// (panel ql, row r) at (ql * r1 + r) * VW, so lane r of a 16-byte load reads
// one contiguous segment; rows 64 + rr (rr < r2 = m - r1) are split over four
// lanes 4 rr + s, lane s taking local panels s, s + 4, ..., stored as (k, lane)
// at PH_w r1 VW + (k * 4 r2 + lane) * VW, k < ceil(PH_w / 4).  Padding is zero.
// FP32 blocks (at most 20 panels) go to one wavefront; FP64 blocks are dealt
// ten panels per wavefront.  The FP32 block of an interior q = 1 patch (m =
// 2 nb = 78) stores the rows r < r1 of its last panel two columns wide
// (8-byte loads at (P - 1) r1 4 + 2 r), so that only the rows past 64 carry
// padding: 6,112 floats instead of 6,240.
__host__ __device__ constexpr int panels_per_wave(int vw) { return vw == 4 ? 20 : 10; }

struct BlockLayout {
  int m, VW, P, r1, r2, waves, ppw, wl;   // wl: width of the rows r < r1 of the last panel
  __host__ __device__ BlockLayout(int m_, int vw_) : m(m_), VW(vw_) {
    ppw = panels_per_wave(VW);
    P = (m + VW - 1) / VW;
    r1 = m < 64 ? m : 64;
    r2 = m - r1;
    waves = (P + ppw - 1) / ppw;
    wl = (VW == 4 && m == 2 * kMaxNb) ? 2 : VW;
  }
  __host__ __device__ bool half() const { return wl != VW; }
  __host__ __device__ int panels(int w) const {
    const int p = P - w * ppw;
    return p < 0 ? 0 : (p > ppw ? ppw : p);
  }
  __host__ __device__ int k2(int w) const { return r2 > 0 ? (panels(w) + 3) / 4 : 0; }
  // elements of the rows r < r1 of wavefront w's panels (the last wavefront
  // holds the last panel)
  __host__ __device__ int part1(int w) const { return panels(w) * r1 * VW - (w == waves - 1 ? r1 * (VW - wl) : 0); }
  __host__ __device__ int share(int w) const { return part1(w) + k2(w) * 4 * r2 * VW; }
  __host__ __device__ int offset(int w) const {
    int o = 0;
    for (int v = 0; v < w; ++v) o += share(v);
    return o;
  }
  __host__ __device__ int size() const { return offset(waves); }
  // element offset of (r, c), r, c < m
  __host__ __device__ int at(int r, int c) const {
    const int q = c / VW, w = q / ppw, ql = q % ppw;
    if (r < r1) return offset(w) + ql * r1 * VW + r * (q == P - 1 ? wl : VW) + c % VW;
    const int lane = (r - 64) * 4 + ql % 4, k = ql / 4;
    return offset(w) + part1(w) + (k * 4 * r2 + lane) * VW + c % VW;
  }
};

// Storage of one inverted m x m block of the large-block sweep (Taylor-Hood
// P3-P2 patches, m up to 162): column panels of VW = 16 / sizeof(T) columns,
// every row of a panel in turn, element (r, c) at ((c / VW) m + r) VW + c % VW;
// the columns of the last panel past m are zero.  A wavefront's 16-byte loads
// of one panel (consecutive rows, one per lane) read one contiguous segment.
__host__ __device__ constexpr int big_block_size(int m, int VW) { return (m + VW - 1) / VW * m * VW; }

// ---- cross-lane helpers (64-lane wavefronts) ------------------------------------
// A lane's value read by every lane (the lane index is uniform).
__device__ inline float read_lane(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline double read_lane(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}
// A DPP exchange of a value between lanes (CTRL: the dpp_ctrl pattern).
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false));
}
// Maximum over the 64 lanes of a wavefront (all active; NaN entries are
// ignored unless every entry is NaN): DPP exchanges inside each row of 16
// lanes (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror), then the four row maxima through scalar registers.
template <typename T>
__device__ inline T wave_max(T v) {
  v = fmax(v, dpp_move<0xB1>(v));
  v = fmax(v, dpp_move<0x4E>(v));
  v = fmax(v, dpp_move<0x141>(v));
  v = fmax(v, dpp_move<0x140>(v));
  return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

// ---- assembly ---------------------------------------------------------------
// color_ptr: the host copy of the 9 colour offsets into L.color_cells; one
// launch per colour, in colour order.
hipError_t launch_assemble_jacobian(const LevelView& L, const RefTables* tab, MmsDev mms,
                                    const double* U, double* Jv, double* Mv, const int* color_ptr,
                                    hipStream_t s);
hipError_t launch_assemble_residual(const LevelView& L, const RefTables* tab, MmsDev mms,
                                    const double* U, double* F, const int* color_ptr, hipStream_t s);
// out[0] = squared space-time velocity L2 error; part: nc * N doubles of workspace
hipError_t launch_velocity_error(const LevelView& L, const RefTables* tab, MmsDev mms,
                                 const double* U, double* part, double* out, hipStream_t s);
// full: (2 nn + nv) N NQ doubles (ux, uy at every P2 node, p at every vertex)
hipError_t launch_expand(const LevelView& L, const RefTables* tab, MmsDev mms, const double* U,
                         double* full, hipStream_t s);

// Heat equation: slab blocks Jv = T (x) M + dt W (x) K, the jump mass Mv = M
// and the stiffness Kv = K of the P_k discretisation, every CSR entry summed
// over its cells in a fixed order (no atomics)
hipError_t launch_heat_operator(const LevelView& L, const RefTables* tab, double* Jv, double* Mv,
                                double* Kv, hipStream_t s);
// y = A x or y = b - A x for the heat equation from the spatial M and K
// alone: per slab (T (x) M + dt W (x) K) x_n - e0 (x) M (e1 . x_{n-1})
hipError_t launch_heat_spmv(const LevelView& L, const RefTables* tab, const double* Mv,
                            const double* Kv, const double* x, const double* b, double* y,
                            hipStream_t s);
// b0 = e0 (x) M U_0 on slab 0 (U_0 the nodal interpolant of sin(pi x) +
// cos(2 pi y)), zero on the other slabs
hipError_t launch_heat_rhs(const LevelView& L, const RefTables* tab, const double* Mv, double* b0,
                           hipStream_t s);

// ---- linear algebra ----------------------------------------------------------
hipError_t launch_spmv(const LevelView& L, const double* Jv, const double* Mv, const double* e0,
                       const double* e1, const double* x, const double* b, double* y,
                       hipStream_t s);
// the same with y = b - A x rounded to FP32 (b required)
hipError_t launch_spmv_f32out(const LevelView& L, const double* Jv, const double* Mv, const double* e0,
                              const double* e1, const double* x, const double* b, float* y, hipStream_t s);
hipError_t launch_transfer(int n_rows, int nt, const int* ptr, const int* col, const double* val,
                           const double* x, double* y, int accumulate, hipStream_t s);
hipError_t launch_gather(int n, int nt, const int* map, const double* x, double* y, hipStream_t s);

// ---- vectors ------------------------------------------------------------------
// out[k] = <x_k, y> for k < nvec, with x_k = X + k * ldx; deterministic two-pass.
hipError_t launch_mdot(int64_t n, int nvec, const double* X, int64_t ldx, const double* y,
                       double* partial, double* out, hipStream_t s);
hipError_t launch_axpy_dev(int64_t n, const double* coef, double scale, const double* x,
                           double* y, hipStream_t s);   // y += scale * (*coef) * x
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y,
                        hipStream_t s);                  // y = a x + b y
hipError_t launch_scale_dev(int64_t n, const double* num, int invert, const double* x, double* y,
                            hipStream_t s);  // y = x * (*num) or x / (*num)
hipError_t launch_fill(int64_t n, double v, double* y, hipStream_t s);
// read `bytes` (a multiple of 16) of device memory with `grid` workgroups of
// 256 threads; out receives grid * 256 partial sums
hipError_t launch_stream_read(const void* buf, int64_t bytes, int grid, float* out, hipStream_t s);
hipError_t launch_start_vector(int64_t n, double* y, hipStream_t s);
hipError_t launch_pressure_project(int nf, int po, int nt, double* x, double* work,
                                   hipStream_t s);
hipError_t launch_gemv_cols(int64_t n, int k, const double* Z, int64_t ldz, const double* y,
                            double* x, hipStream_t s);   // x += Z[:, :k] y (y on device)

// ---- patches -------------------------------------------------------------------
hipError_t launch_patch_factor(const LevelView& L, const PatchView& P, const double* Jv,
                               int prec, void* fac, int* status, hipStream_t s);
// FP32 blocks of more than 64 (at most 80) rows, patches order[first ..
// first + count): blocked Gauss-Jordan with MFMA trailing updates
hipError_t launch_patch_factor_mfma(const LevelView& L, const PatchView& P, const double* Jv, float* fac,
                                    int* status, int first, int count, hipStream_t s);
hipError_t launch_patch_mass(const LevelView& L, const PatchView& P, const double* Mv,
                             double* Mp, hipStream_t s);
// Y: patch outputs, FP64 at element offset y_off[p] ([slab][patch DoF][node];
// prec 0, FP32 factors of the heat equation's scalar patches, of P3-P2
// patches and of time-chunked sweeps), or FP32 at element offset 2 y_off[p]
// ([patch DoF][slab][node]; the plain FP32 sweep of P2-P1 patches,
// sweep_outputs_f32); the buffer holds y_off[n_patch] doubles.
hipError_t launch_patch_sweep(const LevelView& L, const PatchView& P, int prec, const void* fac,
                              const double* Mp, const double* e0, const double* e1,
                              const double* r, void* Y, hipStream_t s);
// The FP32 interior sweep (P2-P1, FP32 blocks, one time chunk) on an FP32
// residual; sweep_takes_f32_residual tells whether a level takes it.
bool sweep_takes_f32_residual(const LevelView& L, const PatchView& P, int prec);
hipError_t launch_patch_sweep_f32r(const LevelView& L, const PatchView& P, int prec, const void* fac,
                                   const double* Mp, const double* e0, const double* e1, const float* r,
                                   void* Y, hipStream_t s);
// Large blocks (L.thk > 0): dense FP64 copies of blocks b0 .. b0 + count - 1
// of the level (block b: patch at position b / fac_slabs of the patch order,
// slab b % fac_slabs) into B (count x mmax x mmax, row-major), each padded with
// the identity past its own order; and, once B holds their inverses, the
// inverses written into the factor storage in the large-block layout at
// precision prec.
hipError_t launch_patch_factor_big_reg(const LevelView& L, const PatchView& P, const double* Jv, int prec,
                                       void* fac, int* status, hipStream_t s);
hipError_t launch_patch_extract_dense(const LevelView& L, const PatchView& P, const double* Jv, int b0,
                                      int count, int mmax, double* B, hipStream_t s);
hipError_t launch_patch_store_big(const LevelView& L, const PatchView& P, int prec, const double* B, int b0,
                                  int count, int mmax, void* fac, hipStream_t s);
// Chunk transfer matrices of the current factors (time_chunks > 1 only).
hipError_t launch_patch_chunk_transfer(const LevelView& L, const PatchView& P, int prec, const void* fac,
                                       const double* Mp, const double* e0, const double* e1,
                                       hipStream_t s);
// Whether the sweep leaves FP32 outputs (the gather reads them as such).
inline bool sweep_outputs_f32(const LevelView& L, const PatchView& P, int prec) {
  return prec == 1 && L.kdeg == 0 && L.thk == 0 && P.time_chunks <= 1;
}
// mode 0: z = sum; mode 1: d = c1 d + c2 sum, x += d; mode 2: the same x update
// without storing d (the last step of a Chebyshev sequence).
hipError_t launch_patch_gather(const LevelView& L, const PatchView& P, int prec, const void* Y,
                               int mode, double c1, double c2, double* z, double* d, double* x,
                               hipStream_t s);

// ---- batched patch kernels over many problems ----------------------------------
// One (problem, level) of a batched FP32 sweep: the level's structure, its
// FP32 factors and patch mass, the residual it reads and the FP32 outputs it
// writes (Navier-Stokes, plain sweep in time).
struct SweepJob {
  LevelView L;
  PatchView P;
  const float* fac;
  const double* Mp;
  const double* r;
  float* Y;
  double e00, e01, e10, e11;
};
// A tile of a batched sweep: patches at positions first .. first + count - 1
// of job's patch order, swept one after another by one workgroup.
struct SweepTile {
  int job, first, count;
};
// Persistent FP32 sweep over a list of tiles whose jobs all have nq temporal
// nodes, the tiles of interior (full-size) patches first (n_full_tiles of
// them), then the tiles of the other patches: grid workgroups take tiles in
// list order from a counter (ctr[0]; ctr[1] counts finished workgroups, and
// the last one resets both, so the pair starts at zero for the next launch).
hipError_t launch_patch_sweep_batch(int nq, const SweepJob* jobs, const SweepTile* tiles, int n_full_tiles,
                                    int n_tiles, int grid, int* ctr, hipStream_t s);

// One (problem, level) of a batched FP32 factorization.
struct FactorJob {
  LevelView L;
  PatchView P;
  const double* Jv;
  float* fac;
  int* status;
};
// Block classes of the batched factorization: FP32 blocks of one temporal
// node (at most 39 rows), of two nodes with at most 64 rows, and of two
// nodes with more than 64 rows (MFMA blocked Gauss-Jordan).
enum { kFacSmall1 = 0, kFacSmall2 = 1, kFacBig2 = 2, kFacClasses = 3 };
// A tile of a batched factorization: blocks first .. first + count - 1 of a
// job, block b being the block of the patch at position b / fac_slabs of the
// job's patch order, at slab b % fac_slabs (a tile stays inside one class).
struct FactorTile {
  int job, first, count;
};
// Persistent factorization of one block class over a list of tiles (counter
// pair as for the sweep).
hipError_t launch_patch_factor_batch(int cls, const FactorJob* jobs, const FactorTile* tiles, int n_tiles,
                                     int grid, int* ctr, hipStream_t s);
hipError_t launch_patch_factor_mfma_batch(const FactorJob* jobs, const FactorTile* tiles, int n_tiles,
                                          int grid, int* ctr, hipStream_t s);
// Workgroups of each kind that fit on one compute unit at once (from the
// kernels' register and LDS use), for sizing persistent grids.
int patch_sweep_batch_occupancy(int nq);
int patch_factor_batch_occupancy(int cls);
int patch_factor_mfma_batch_occupancy();

// ---- coarsest level ---------------------------------------------------------------
// Bordered slab blocks of at most this order are inverted and applied by one
// workgroup; larger ones by the blocked, chip-wide kernels.
constexpr int kCoarseSmall = 64;
hipError_t launch_coarse_build(const LevelView& L, const double* Jv, double* B, hipStream_t s);
// perm: nmat * m ints, colbuf: nmat * m doubles, rbuf: nmat * kRbufRows * m
// doubles of workspace (the panel rows of two panels; used when m >
// kCoarseSmall; rbuf = NULL selects the unblocked form)
constexpr int kRbufRows = 64;
hipError_t launch_dense_inverse(int nmat, int m, double* B, int* status, int* perm,
                                double* colbuf, double* rbuf, hipStream_t s);
// gbuf: nf (q+1) + nbord doubles of workspace (used for large coarsest levels)
hipError_t launch_coarse_solve(const LevelView& L, const double* Binv, const double* Mv,
                               const double* e0, const double* e1, const double* b, double* x,
                               double* gbuf, hipStream_t s);

}  // namespace stwr
