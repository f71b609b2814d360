// Waveform-relaxation Vanka+star patch smoother on gfx950 (Sec. 3, Vanka+star
// patches extended over all temporal nodes; eq. waveform_patch_solve).
//
// * k_patch_factor: one workgroup per (patch, slab) gathers the slab block
//   A_{v,n} = R_v J_n R_v^T (nb' = nb (q+1) rows, nb <= 39) from the assembled
//   operator into LDS and inverts it in place by Gauss-Jordan elimination with
//   partial pivoting, in FP64 or FP32.  The inverse is stored in column panels
//   of VW = 16 / sizeof(T) columns: element (r, c) of a block sits at
//   (c / VW) * (m * VW) + r * VW + c % VW, so a wavefront whose lane r reads a
//   16-byte vector of row r touches one contiguous 1 KB segment.
// * k_patch_sweep: one wavefront per patch walks the slabs in order (forward
//   block substitution): gather the residual of the patch DoFs, add the jump
//   coupling e0 (x) (M_v * (e1 . y_{n-1})), multiply by the stored inverse and
//   write the slab result to a per-patch output buffer.
// * k_patch_gather: each DoF sums its contributions from the <= 7 patches that
//   hold it in a fixed order (deterministic additive scatter), optionally
//   fused with the Chebyshev update d = c1 d + c2 z, x += d.
#include "device.h"

namespace stwr {

namespace {

constexpr int kFacThreads = 256;

template <typename T>
struct Vec;
template <>
struct Vec<float> {
  using type = float4;
  static constexpr int W = 4;
};
template <>
struct Vec<double> {
  using type = double2;
  static constexpr int W = 2;
};

__host__ __device__ inline int round_up(int m, int w) { return (m + w - 1) / w * w; }

template <int NQ, typename T>
__global__ __launch_bounds__(kFacThreads) void k_patch_factor(LevelView L, PatchView P,
                                                              const double* __restrict__ Jv,
                                                              T* __restrict__ fac,
                                                              int* __restrict__ status) {
  constexpr int MAXM = kMaxNb * NQ;
  constexpr int VW = Vec<T>::W;
  __shared__ T A[MAXM][MAXM + 1];
  __shared__ T colk[MAXM];
  __shared__ int perm[MAXM];
  __shared__ T rv[kFacThreads / 64];
  __shared__ int ri[kFacThreads / 64];
  __shared__ int piv_s;
  const int p = blockIdx.x / L.N, n = blockIdx.x % L.N;
  const int tid = threadIdx.x;
  const int s0 = P.patch_ptr[p];
  const int nb = P.patch_ptr[p + 1] - s0;
  const int m = nb * NQ;
  const int* nzp = P.patch_nz + P.patch_nz_off[p];
  for (int e = tid; e < m * m; e += kFacThreads) {
    const int r = e / m, c = e % m;
    const int i = r / NQ, a = r % NQ, j = c / NQ, b = c % NQ;
    const int k = nzp[i * nb + j];
    A[r][c] = k >= 0 ? (T)Jv[(((int64_t)k * L.N + n) * NQ + a) * NQ + b] : (T)0;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    T best = (T)-1;
    int bi = m;
    for (int i = k + tid; i < m; i += kFacThreads) {
      const T v = fabs(A[i][k]);
      if (v > best) { best = v; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const T ov = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (tid % 64 == 0) { rv[tid / 64] = best; ri[tid / 64] = bi; }
    __syncthreads();
    if (tid == 0) {
      T b = rv[0];
      int pi = ri[0];
      for (int w = 1; w < kFacThreads / 64; ++w)
        if (rv[w] > b || (rv[w] == b && ri[w] < pi)) { b = rv[w]; pi = ri[w]; }
      if (!(b > (T)0) || !isfinite(b) || pi >= m) { status[0] = 1; pi = k; }
      piv_s = pi;
      perm[k] = pi;
    }
    __syncthreads();
    const int pr = piv_s;
    if (pr != k)
      for (int j = tid; j < m; j += kFacThreads) {
        const T t = A[k][j];
        A[k][j] = A[pr][j];
        A[pr][j] = t;
      }
    __syncthreads();
    const T pv = A[k][k];
    __syncthreads();
    for (int j = tid; j < m; j += kFacThreads) A[k][j] = (j == k ? (T)1 : A[k][j]) / pv;
    for (int i = tid; i < m; i += kFacThreads) colk[i] = A[i][k];
    __syncthreads();
    for (int e = tid; e < m * m; e += kFacThreads) {
      const int i = e / m, j = e % m;
      if (i == k) continue;
      const T f = colk[i];
      if (j == k) A[i][j] = -f * A[k][k];
      else A[i][j] -= f * A[k][j];
    }
    __syncthreads();
  }
  for (int k = m - 1; k >= 0; --k) {
    const int pr = perm[k];
    if (pr != k)
      for (int i = tid; i < m; i += kFacThreads) {
        const T t = A[i][k];
        A[i][k] = A[i][pr];
        A[i][pr] = t;
      }
    __syncthreads();
  }
  const int CP = round_up(m, VW);
  T* out = fac + P.fac_off[p] + (int64_t)n * m * CP;
  for (int e = tid; e < m * CP; e += kFacThreads) {
    const int panel = e / (m * VW), rem = e % (m * VW);
    const int r = rem / VW, c = panel * VW + rem % VW;
    out[e] = c < m ? A[r][c] : (T)0;
  }
}

__global__ __launch_bounds__(256) void k_patch_mass(PatchView P, const double* __restrict__ Mv,
                                                    double* __restrict__ Mp) {
  const int p = blockIdx.x;
  const int s0 = P.patch_ptr[p];
  const int nb = P.patch_ptr[p + 1] - s0, nbu = P.patch_nbu[p];
  const int* nzp = P.patch_nz + P.patch_nz_off[p];
  double* out = Mp + P.mp_off[p];
  for (int e = threadIdx.x; e < nbu * nbu; e += 256) {
    const int i = e / nbu, j = e % nbu;
    const int k = nzp[i * nb + j];
    out[e] = k >= 0 ? Mv[k] : 0.0;
  }
}

template <int NQ, typename T>
__global__ __launch_bounds__(64) void k_patch_sweep(LevelView L, PatchView P, const T* __restrict__ fac,
                                                    const double* __restrict__ Mp, double e00,
                                                    double e01, double e10, double e11,
                                                    const double* __restrict__ r,
                                                    double* __restrict__ Y) {
  constexpr int MAXM = kMaxNb * NQ;
  constexpr int VW = Vec<T>::W;
  using V = typename Vec<T>::type;
  __shared__ int dofs[kMaxNb];
  __shared__ double Ms[kMaxNbu * kMaxNbu];
  __shared__ T g[MAXM + 4];
  __shared__ double ys[MAXM];
  __shared__ double ylast[kMaxNbu];
  const double e0[2] = {e00, e01}, e1[2] = {e10, e11};
  const int p = blockIdx.x, tid = threadIdx.x;
  const int s0 = P.patch_ptr[p];
  const int nb = P.patch_ptr[p + 1] - s0, nbu = P.patch_nbu[p];
  const int m = nb * NQ, CP = round_up(m, VW), N = L.N;
  for (int i = tid; i < nb; i += 64) dofs[i] = P.patch_dofs[s0 + i];
  const double* mp = Mp + P.mp_off[p];
  for (int e = tid; e < nbu * nbu; e += 64) Ms[e] = mp[e];
  for (int i = tid; i < nbu; i += 64) ylast[i] = 0.0;
  __syncthreads();
  const T* Ab = fac + P.fac_off[p];
  double* yout = Y + P.y_off[p];
  for (int n = 0; n < N; ++n) {
    for (int row = tid; row < CP; row += 64) {
      T v = (T)0;
      if (row < m) {
        const int i = row / NQ, a = row % NQ;
        double rv = r[((int64_t)dofs[i] * N + n) * NQ + a];
        if (n > 0 && i < nbu) {
          double acc = 0.0;
          for (int j = 0; j < nbu; ++j) acc += Ms[i * nbu + j] * ylast[j];
          rv += e0[a] * acc;
        }
        v = (T)rv;
      }
      g[row] = v;
    }
    __syncthreads();
    const T* An = Ab + (int64_t)n * m * CP;
    for (int row = tid; row < m; row += 64) {
      T acc = (T)0;
      for (int pc = 0; pc < CP / VW; ++pc) {
        const V w = *reinterpret_cast<const V*>(An + (int64_t)pc * m * VW + row * VW);
        if constexpr (VW == 4) {
          acc += w.x * g[pc * 4] + w.y * g[pc * 4 + 1] + w.z * g[pc * 4 + 2] + w.w * g[pc * 4 + 3];
        } else {
          acc += w.x * g[pc * 2] + w.y * g[pc * 2 + 1];
        }
      }
      ys[row] = (double)acc;
      yout[(int64_t)n * m + row] = (double)acc;
    }
    __syncthreads();
    for (int i = tid; i < nbu; i += 64) {
      double v = 0.0;
      for (int b = 0; b < NQ; ++b) v += e1[b] * ys[i * NQ + b];
      ylast[i] = v;
    }
    __syncthreads();
  }
}

template <int NQ>
__global__ __launch_bounds__(256) void k_patch_gather(int nf, int N, PatchView P,
                                                      const double* __restrict__ Y, int mode,
                                                      double c1, double c2, double* __restrict__ z,
                                                      double* __restrict__ d, double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)nf * N) return;
  const int dof = (int)(t / N), n = (int)(t % N);
  double acc[NQ];
  for (int a = 0; a < NQ; ++a) acc[a] = 0.0;
  for (int k = P.dof_ptr[dof]; k < P.dof_ptr[dof + 1]; ++k) {
    const int s = P.dof_slot[k];
    const int p = P.slot_patch[s];
    const int s0 = P.patch_ptr[p];
    const int m = (P.patch_ptr[p + 1] - s0) * NQ;
    const double* yp = Y + P.y_off[p] + (int64_t)n * m + (s - s0) * NQ;
    for (int a = 0; a < NQ; ++a) acc[a] += yp[a];
  }
  const int64_t o = t * NQ;
  if (mode == 0) {
    for (int a = 0; a < NQ; ++a) z[o + a] = acc[a];
  } else {
    for (int a = 0; a < NQ; ++a) {
      const double dd = (c1 == 0.0 ? 0.0 : c1 * d[o + a]) + c2 * acc[a];
      d[o + a] = dd;
      x[o + a] += dd;
    }
  }
}

}  // namespace

hipError_t launch_patch_factor(const LevelView& L, const PatchView& P, const double* Jv, int prec,
                               void* fac, int* status, hipStream_t s) {
  dim3 grid((unsigned)P.n_patch * L.N), block(kFacThreads);
  if (prec == 1) {
    if (L.NQ == 1) hipLaunchKernelGGL((k_patch_factor<1, float>), grid, block, 0, s, L, P, Jv, (float*)fac, status);
    else hipLaunchKernelGGL((k_patch_factor<2, float>), grid, block, 0, s, L, P, Jv, (float*)fac, status);
  } else {
    if (L.NQ == 1) hipLaunchKernelGGL((k_patch_factor<1, double>), grid, block, 0, s, L, P, Jv, (double*)fac, status);
    else hipLaunchKernelGGL((k_patch_factor<2, double>), grid, block, 0, s, L, P, Jv, (double*)fac, status);
  }
  return hipGetLastError();
}

hipError_t launch_patch_mass(const LevelView& L, const PatchView& P, const double* Mv, double* Mp,
                             hipStream_t s) {
  (void)L;
  hipLaunchKernelGGL(k_patch_mass, dim3(P.n_patch), dim3(256), 0, s, P, Mv, Mp);
  return hipGetLastError();
}

hipError_t launch_patch_sweep(const LevelView& L, const PatchView& P, int prec, const void* fac,
                              const double* Mp, const double* e0, const double* e1,
                              const double* r, double* Y, hipStream_t s) {
  const double e01 = L.NQ > 1 ? e0[1] : 0.0, e11 = L.NQ > 1 ? e1[1] : 0.0;
  dim3 grid(P.n_patch), block(64);
  if (prec == 1) {
    if (L.NQ == 1) hipLaunchKernelGGL((k_patch_sweep<1, float>), grid, block, 0, s, L, P, (const float*)fac, Mp, e0[0], e01, e1[0], e11, r, Y);
    else hipLaunchKernelGGL((k_patch_sweep<2, float>), grid, block, 0, s, L, P, (const float*)fac, Mp, e0[0], e01, e1[0], e11, r, Y);
  } else {
    if (L.NQ == 1) hipLaunchKernelGGL((k_patch_sweep<1, double>), grid, block, 0, s, L, P, (const double*)fac, Mp, e0[0], e01, e1[0], e11, r, Y);
    else hipLaunchKernelGGL((k_patch_sweep<2, double>), grid, block, 0, s, L, P, (const double*)fac, Mp, e0[0], e01, e1[0], e11, r, Y);
  }
  return hipGetLastError();
}

hipError_t launch_patch_gather(const LevelView& L, const PatchView& P, const double* Y, int mode,
                               double c1, double c2, double* z, double* d, double* x,
                               hipStream_t s) {
  const int64_t n = (int64_t)L.nf * L.N;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (L.NQ == 1) hipLaunchKernelGGL(k_patch_gather<1>, grid, block, 0, s, L.nf, L.N, P, Y, mode, c1, c2, z, d, x);
  else hipLaunchKernelGGL(k_patch_gather<2>, grid, block, 0, s, L.nf, L.N, P, Y, mode, c1, c2, z, d, x);
  return hipGetLastError();
}

}  // namespace stwr
