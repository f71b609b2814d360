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
};

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
};

struct PatchView {
  int n_patch;
  const int* patch_ptr;
  const int* patch_dofs;
  const int* patch_nbu;
  const int64_t* patch_nz_off;
  const int* patch_nz;
  const int64_t* fac_off;   // n_patch + 1, element offsets of each patch's N blocks
  const int64_t* y_off;     // n_patch + 1, offsets into the patch output buffer
  const int64_t* mp_off;    // n_patch + 1, offsets of the patch mass blocks
  const int* dof_ptr;
  const int* dof_slot;
  const int* slot_patch;
};

// ---- assembly ---------------------------------------------------------------
hipError_t launch_assemble_jacobian(const LevelView& L, const RefTables* tab, MmsDev mms,
                                    const double* U, double* Jv, double* Mv, hipStream_t s);
hipError_t launch_assemble_residual(const LevelView& L, const RefTables* tab, MmsDev mms,
                                    const double* U, double* F, hipStream_t s);

// ---- linear algebra ----------------------------------------------------------
hipError_t launch_spmv(const LevelView& L, const double* Jv, const double* Mv, const double* e0,
                       const double* e1, const double* x, const double* b, double* y,
                       hipStream_t s);
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
hipError_t launch_start_vector(int64_t n, double* y, hipStream_t s);
hipError_t launch_pressure_project(int nf, int po, int nt, double* x, double* work,
                                   hipStream_t s);
hipError_t launch_gemv_cols(int64_t n, int k, const double* Z, int64_t ldz, const double* y,
                            double* x, hipStream_t s);   // x += Z[:, :k] y (y on device)

// ---- patches -------------------------------------------------------------------
hipError_t launch_patch_factor(const LevelView& L, const PatchView& P, const double* Jv,
                               int prec, void* fac, int* status, hipStream_t s);
hipError_t launch_patch_mass(const LevelView& L, const PatchView& P, const double* Mv,
                             double* Mp, hipStream_t s);
hipError_t launch_patch_sweep(const LevelView& L, const PatchView& P, int prec, const void* fac,
                              const double* Mp, const double* e0, const double* e1,
                              const double* r, double* Y, hipStream_t s);
// mode 0: z = sum; mode 1: d = c1 d + c2 sum, x += d.
hipError_t launch_patch_gather(const LevelView& L, const PatchView& P, const double* Y, int mode,
                               double c1, double c2, double* z, double* d, double* x,
                               hipStream_t s);

// ---- coarsest level ---------------------------------------------------------------
hipError_t launch_coarse_build(const LevelView& L, const double* Jv, double* B, hipStream_t s);
hipError_t launch_dense_inverse(int nmat, int m, double* B, int* status, hipStream_t s);
hipError_t launch_coarse_solve(const LevelView& L, const double* Binv, const double* Mv,
                               const double* e0, const double* e1, const double* b, double* x,
                               hipStream_t s);

}  // namespace stwr
