// Waveform-relaxation Vanka+star patch smoother on gfx950 (Sec. 3, Vanka+star
// patches extended over all temporal nodes; eq. waveform_patch_solve).
//
// * k_patch_factor: one workgroup per (patch, slab) gathers the slab block
//   A_{v,n} = R_v J_n R_v^T (nb' = nb (q+1) rows, nb <= 39) from the assembled
//   operator into LDS and inverts it in place by Gauss-Jordan elimination with
//   partial pivoting, in FP64 or FP32.  The inverse is stored for a 64-lane
//   wavefront (see block_offset): columns are grouped in panels of
//   VW = 16 / sizeof(T); rows 0..63 are one row per lane, panel-major, and the
//   rows past 64 (at most 14) are split over four lanes each, so every 16-byte
//   vector load of a wavefront reads one contiguous segment and no lane idles.
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

// Layout of one inverted m x m slab block for the sweep wavefront.
//   P  = ceil(m / VW) column panels, r1 = min(m, 64) lane rows, r2 = m - r1.
//   Region 1: (panel q, row r < r1) at (q * r1 + r) * VW.
//   Region 2: row 64 + rr is handled by lanes 4 rr + s (s = 0..3), which take
//   panels s, s + 4, s + 8, ...: (k, lane) at P r1 VW + (k * 4 r2 + lane) * VW
//   for k < K2 = ceil(P / 4).  Padding columns and panels hold zeros.
struct BlockShape {
  int m, P, r1, r2, K2, S;
  __host__ __device__ BlockShape(int m_, int VW) : m(m_) {
    P = (m + VW - 1) / VW;
    r1 = m < 64 ? m : 64;
    r2 = m - r1;
    K2 = (P + 3) / 4;
    S = P * r1 * VW + (r2 > 0 ? K2 * 4 * r2 * VW : 0);
  }
};

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
  const BlockShape sh(m, VW);
  T* out = fac + P.fac_off[p] + (int64_t)n * sh.S;
  const int R1 = sh.P * sh.r1 * VW;
  for (int e = tid; e < sh.S; e += kFacThreads) {
    int r, c;
    if (e < R1) {
      const int q = e / (sh.r1 * VW), rem = e % (sh.r1 * VW);
      r = rem / VW;
      c = q * VW + rem % VW;
    } else {
      const int e2 = e - R1;
      const int k = e2 / (4 * sh.r2 * VW), rem = e2 % (4 * sh.r2 * VW);
      const int lane = rem / VW;
      const int q = (lane & 3) + 4 * k;
      r = 64 + lane / 4;
      c = q < sh.P ? q * VW + rem % VW : m;
    }
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

template <typename V, typename T>
__device__ inline T dotv(const V& w, const T* g) {
  if constexpr (sizeof(V) / sizeof(T) == 4) return w.x * g[0] + w.y * g[1] + w.z * g[2] + w.w * g[3];
  else return w.x * g[0] + w.y * g[1];
}

// One wavefront per patch.  Per slab: issue every load of the slab's inverse
// block at once (the block does not depend on the previous slab), then form
// the right-hand side g = r_n + e0 (x) (M_v ylast) in LDS while the loads are
// in flight, then the matrix-vector product.  The residual values of slab
// n + 1 are loaded one slab ahead.
template <int NQ, typename T>
__global__ __launch_bounds__(64) void k_patch_sweep(LevelView L, PatchView P, const T* __restrict__ fac,
                                                    const double* __restrict__ Mp, double e00,
                                                    double e01, double e10, double e11,
                                                    const double* __restrict__ r,
                                                    double* __restrict__ Y) {
  constexpr int MAXM = kMaxNb * NQ;
  constexpr int VW = Vec<T>::W;
  constexpr int MAXP = (MAXM + VW - 1) / VW;
  constexpr int MAXK2 = (MAXP + 3) / 4;
  constexpr bool kTwo = MAXM > 64;
  using V = typename Vec<T>::type;
  __shared__ int dofs[kMaxNb];
  __shared__ double Ms[kMaxNbu * kMaxNbu];
  __shared__ T g[MAXP * VW + 64];
  __shared__ double ys[MAXM + 64];
  __shared__ double ylast[kMaxNbu];
  const double e0[2] = {e00, e01}, e1[2] = {e10, e11};
  const int p = blockIdx.x, lane = threadIdx.x;
  const int s0 = P.patch_ptr[p];
  const int nb = P.patch_ptr[p + 1] - s0, nbu = P.patch_nbu[p];
  const int m = nb * NQ, N = L.N;
  const BlockShape sh(m, VW);
  for (int i = lane; i < nb; i += 64) dofs[i] = P.patch_dofs[s0 + i];
  const double* mp = Mp + P.mp_off[p];
  for (int e = lane; e < nbu * nbu; e += 64) Ms[e] = mp[e];
  for (int i = lane; i < nbu; i += 64) ylast[i] = 0.0;
  __syncthreads();
  const T* Ab = fac + P.fac_off[p];
  double* yout = Y + P.y_off[p];
  // the (at most two) rows whose right-hand side this lane forms
  const int rowA = lane, rowB = lane + 64;
  const bool hasA = rowA < m, hasB = kTwo && rowB < m;
  const int64_t baseA = hasA ? (int64_t)dofs[rowA / NQ] * N * NQ + rowA % NQ : 0;
  const int64_t baseB = hasB ? (int64_t)dofs[rowB / NQ] * N * NQ + rowB % NQ : 0;
  double rA = hasA ? r[baseA] : 0.0, rB = hasB ? r[baseB] : 0.0;
  const int R1 = sh.P * sh.r1 * VW;
  const int quarter = lane & 3;
  for (int n = 0; n < N; ++n) {
    const T* blk = Ab + (int64_t)n * sh.S;
    V a1[MAXP];
    V a2[kTwo ? MAXK2 : 1];
#pragma unroll
    for (int q = 0; q < MAXP; ++q)
      if (q < sh.P && lane < sh.r1) a1[q] = *reinterpret_cast<const V*>(blk + (q * sh.r1 + lane) * VW);
    if constexpr (kTwo) {
#pragma unroll
      for (int k = 0; k < MAXK2; ++k)
        if (k < sh.K2 && lane < 4 * sh.r2)
          a2[k] = *reinterpret_cast<const V*>(blk + R1 + (k * 4 * sh.r2 + lane) * VW);
    }
    double rA_next = 0.0, rB_next = 0.0;
    if (n + 1 < N) {
      if (hasA) rA_next = r[baseA + (int64_t)(n + 1) * NQ];
      if (hasB) rB_next = r[baseB + (int64_t)(n + 1) * NQ];
    }
    double gA = rA, gB = rB;
    if (n > 0) {
      if (hasA && rowA / NQ < nbu) {
        const double* mrow = Ms + (rowA / NQ) * nbu;
        double acc = 0.0;
        for (int j = 0; j < nbu; ++j) acc += mrow[j] * ylast[j];
        gA += e0[rowA % NQ] * acc;
      }
      if (hasB && rowB / NQ < nbu) {
        const double* mrow = Ms + (rowB / NQ) * nbu;
        double acc = 0.0;
        for (int j = 0; j < nbu; ++j) acc += mrow[j] * ylast[j];
        gB += e0[rowB % NQ] * acc;
      }
    }
    if (rowA < sh.P * VW) g[rowA] = hasA ? (T)gA : (T)0;
    if (rowB < sh.P * VW) g[rowB] = hasB ? (T)gB : (T)0;
    __syncthreads();
    T acc1 = (T)0;
#pragma unroll
    for (int q = 0; q < MAXP; ++q)
      if (q < sh.P) acc1 += dotv<V, T>(a1[q], g + q * VW);
    if (lane < sh.r1) {
      ys[lane] = (double)acc1;
      yout[(int64_t)n * m + lane] = (double)acc1;
    }
    if constexpr (kTwo) {
      T acc2 = (T)0;
#pragma unroll
      for (int k = 0; k < MAXK2; ++k) {
        const int q = quarter + 4 * k;
        if (k < sh.K2 && q < sh.P) acc2 += dotv<V, T>(a2[k], g + q * VW);
      }
      acc2 += __shfl_xor(acc2, 1);
      acc2 += __shfl_xor(acc2, 2);
      if (lane < 4 * sh.r2 && quarter == 0) {
        const int row = 64 + lane / 4;
        ys[row] = (double)acc2;
        yout[(int64_t)n * m + row] = (double)acc2;
      }
    }
    __syncthreads();
    for (int i = lane; i < nbu; i += 64) {
      double v = 0.0;
      for (int b = 0; b < NQ; ++b) v += e1[b] * ys[i * NQ + b];
      ylast[i] = v;
    }
    __syncthreads();
    rA = rA_next;
    rB = rB_next;
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
