// Inversion of the large FP32 patch blocks (more than 64 rows: the interior
// Vanka+star patches at q = 1, 78 x 78) by blocked Gauss-Jordan elimination
// with matrix-core (MFMA) trailing updates on gfx950.
//
// One wavefront per (patch, slab) block, two temporal nodes (q = 1).  The
// block is staged in LDS from the patch's nonzero list (one 32-byte 2 x 2
// load per spatial pair), zero padded to 80 x 80, and inverted in place with partial pivoting, sixteen
// columns (a panel) at a time:
//   panel steps, with the panel's 80 x 16 values in registers (rows lane and
//     lane + 64): pivot search in column k (largest magnitude, ties to the
//     smaller row: a DPP wave maximum and a ballot), a full-row swap
//     (registers and LDS), then the pivot row read from its lane, scaled by
//     the pivot's reciprocal, and the elimination applied to the panel's
//     columns only;
//   trailing update: every other column receives the panel's combined
//     transform at once, A += W R, with W = the panel columns minus the
//     selector of the panel rows (80 x 16) and R = the panel rows of those
//     columns (16 x 80); as 16 x 16 tiles, four v_mfma_f32_16x16x4f32 each.
// Per element the transform is the one the column-at-a-time Gauss-Jordan
// inverse applies (its blocked form, as in the coarsest-level solver).  The
// pivot order is recorded and undone on the columns while the inverse is
// written in the sweep's FP32 panel layout.
#include "device.h"

namespace stwr {

namespace {

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

constexpr int kFM = 80;        // padded block order: five 16-wide tiles
constexpr int kFS = kFM + 1;   // LDS row stride (column reads fall in distinct banks)
constexpr int kFP = 16;        // panel width
constexpr int kFT = kFM / 16;  // tiles per side

struct MfmaFactorLds {
  float A[kFM * kFS];
  int perm[kFM];
  int ofs[kFM];   // at the end: the A column of each output column
  float swp[2][kFP];
};

// The block of patch p (its id) at slab n.
__device__ __forceinline__ void factor_block_mfma(const LevelView& L, const PatchView& P, const int p, const int n,
                                                  const double* __restrict__ Jv, float* __restrict__ fac,
                                                  int* __restrict__ status, MfmaFactorLds& S) {
  float* A = S.A;
  int* perm = S.perm;
  int* ofs = S.ofs;
  const int lane = threadIdx.x;
  // two temporal nodes (q = 1): each spatial pair (I, J) of the patch is a
  // 2 x 2 block, 32 contiguous bytes of Jv
  const int s0 = P.patch_ptr[p], nb = P.patch_ptr[p + 1] - s0, m = 2 * nb;
  const int* nzp = P.patch_nz + P.patch_nz_off[p];
  for (int e = lane; e < kFM * kFM; e += 64) A[(e / kFM) * kFS + e % kFM] = 0.0f;
  __syncthreads();
#pragma unroll 4
  for (int e = lane; e < nb * nb; e += 64) {
    const int k = nzp[e];
    if (k < 0) continue;
    const int I = e / nb, J = e % nb;
    const double2* src = reinterpret_cast<const double2*>(Jv + ((int64_t)k * L.N + n) * 4);
    const double2 u = src[0], v = src[1];
    A[(2 * I) * kFS + 2 * J] = (float)u.x;
    A[(2 * I) * kFS + 2 * J + 1] = (float)u.y;
    A[(2 * I + 1) * kFS + 2 * J] = (float)v.x;
    A[(2 * I + 1) * kFS + 2 * J + 1] = (float)v.y;
  }
  __syncthreads();
  bool bad = false;
  const int lr = lane % 16, lk = lane / 16;
  float (*swp)[kFP] = S.swp;
  // lane l holds rows l and l + 64 (the latter for l < 16) of the panel
  const int row0 = lane, row1 = lane + 64;
  const bool has1 = row1 < kFM;
  for (int k0 = 0; k0 < m; k0 += kFP) {
    const int b = m - k0 < kFP ? m - k0 : kFP;
    float pr[2][kFP];
#pragma unroll
    for (int jj = 0; jj < kFP; ++jj) {
      pr[0][jj] = A[row0 * kFS + k0 + jj];
      pr[1][jj] = has1 ? A[row1 * kFS + k0 + jj] : 0.0f;
    }
#pragma clang loop unroll(full)
    for (int kk = 0; kk < kFP; ++kk) {
      if (kk < b) {   // uniform
        const int k = k0 + kk;
        // pivot: largest |entry| of column k among rows k .. m-1, ties to the
        // smaller row: the wave's maximum, then the first lane (rows < 64
        // before rows >= 64) that holds it
        const float v0 = (row0 >= k && row0 < m) ? fabsf(pr[0][kk]) : -1.0f;
        const float v1 = (has1 && row1 >= k && row1 < m) ? fabsf(pr[1][kk]) : -1.0f;
        const float best = wave_max(fmaxf(v0, v1));
        const uint64_t hit0 = __ballot(v0 == best), hit1 = __ballot(v1 == best);
        int pi = hit0 ? __ffsll((unsigned long long)hit0) - 1
                      : (hit1 ? 64 + __ffsll((unsigned long long)hit1) - 1 : m);
        if (!(best > 0.0f) || !isfinite(best) || pi >= m) {
          bad = true;
          pi = k;
        }
        if (lane == 0) perm[k] = pi;
        if (pi != k) {   // uniform: swap rows k and pi (panel in registers, the rest in LDS)
          for (int j = lane; j < kFM; j += 64) {
            if (j >= k0 && j < k0 + kFP) continue;
            const float t = A[k * kFS + j];
            A[k * kFS + j] = A[pi * kFS + j];
            A[pi * kFS + j] = t;
          }
#pragma unroll
          for (int jj = 0; jj < kFP; ++jj) {
            if (row0 == pi) swp[0][jj] = pr[0][jj];
            if (row0 == k) swp[1][jj] = pr[0][jj];
            if (has1 && row1 == pi) swp[0][jj] = pr[1][jj];
            if (has1 && row1 == k) swp[1][jj] = pr[1][jj];
          }
          __syncthreads();
#pragma unroll
          for (int jj = 0; jj < kFP; ++jj) {
            if (row0 == k) pr[0][jj] = swp[0][jj];
            if (row0 == pi) pr[0][jj] = swp[1][jj];
            if (has1 && row1 == k) pr[1][jj] = swp[0][jj];
            if (has1 && row1 == pi) pr[1][jj] = swp[1][jj];
          }
        }
        // the pivot row, read from its lane (k < 64: lane k, first register
        // set; else lane k - 64, second set) and scaled so that its pivot
        // entry becomes 1 / pivot
        float pw[kFP];
        if (k < 64) {   // uniform
#pragma unroll
          for (int jj = 0; jj < kFP; ++jj) pw[jj] = read_lane(pr[0][jj], k);
        } else {
#pragma unroll
          for (int jj = 0; jj < kFP; ++jj) pw[jj] = read_lane(pr[1][jj], k - 64);
        }
        const float rpv = 1.0f / pw[kk];
#pragma unroll
        for (int jj = 0; jj < kFP; ++jj) pw[jj] = (jj == kk ? 1.0f : pw[jj]) * rpv;
        // the pivot row takes the scaled values, the others eliminate column k
        // (panel columns)
        {
          const float f = pr[0][kk];
#pragma unroll
          for (int jj = 0; jj < kFP; ++jj)
            pr[0][jj] = row0 == k ? pw[jj] : (jj == kk ? 0.0f : pr[0][jj]) - f * pw[jj];
        }
        if (has1) {
          const float f = pr[1][kk];
#pragma unroll
          for (int jj = 0; jj < kFP; ++jj)
            pr[1][jj] = row1 == k ? pw[jj] : (jj == kk ? 0.0f : pr[1][jj]) - f * pw[jj];
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < kFP; ++jj) {
      A[row0 * kFS + k0 + jj] = pr[0][jj];
      if (has1) A[row1 * kFS + k0 + jj] = pr[1][jj];
    }
    __syncthreads();
    // trailing update of the columns outside the panel: operands to
    // registers first (R's rows are among those the tiles rewrite)
    const int pt = k0 / kFP;
    float wa[kFT][4], rb[kFT][4];
#pragma unroll
    for (int t = 0; t < kFT; ++t)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int jj = kk * 4 + lk;
        const int i = t * 16 + lr;
        wa[t][kk] = jj < b ? A[i * kFS + k0 + jj] - (i == k0 + jj ? 1.0f : 0.0f) : 0.0f;
        const int c = t * 16 + lr;
        rb[t][kk] = jj < b ? A[(k0 + jj) * kFS + c] : 0.0f;
      }
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < kFT; ++rt) {
#pragma unroll
      for (int ct = 0; ct < kFT; ++ct) {
        if (ct == pt) continue;   // the panel's own columns are final
        mfma_f4 acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = A[(rt * 16 + 4 * lk + q) * kFS + ct * 16 + lr];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[rt][kk], rb[ct][kk], acc, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) A[(rt * 16 + 4 * lk + q) * kFS + ct * 16 + lr] = acc[q];
      }
    }
    __syncthreads();
  }
  if (bad && lane == 0) status[0] = 1;
  // undo the column permutation of the pivoting (the swaps (k, perm[k]) for
  // k = m-1 .. 0): output column pos(c) receives A's column c, and ofs[pos]
  // records c.  Then every (row, four-column panel) of the layout is one
  // 16-byte store (8-byte in a narrow last panel), consecutive lanes on
  // consecutive rows.
  for (int c = lane; c < m; c += 64) {
    int pos = c;
    for (int k = m - 1; k >= 0; --k) {
      const int pk = perm[k];
      if (pos == k) pos = pk;
      else if (pos == pk) pos = k;
    }
    ofs[pos] = c;
  }
  __syncthreads();
  const BlockLayout lay(m, 4);
  float* out = fac + P.fac_off[p] + (int64_t)n * P.slab_stride;
  const int np = (m + 3) / 4;
  for (int e = lane; e < m * np; e += 64) {
    const int r = e % m, q = e / m;
    float4 v;
    v.x = A[r * kFS + ofs[4 * q]];
    v.y = 4 * q + 1 < m ? A[r * kFS + ofs[4 * q + 1]] : 0.0f;
    v.z = 4 * q + 2 < m ? A[r * kFS + ofs[4 * q + 2]] : 0.0f;
    v.w = 4 * q + 3 < m ? A[r * kFS + ofs[4 * q + 3]] : 0.0f;
    if (r < 64 && q == lay.P - 1 && lay.half()) {
      // the narrow last panel of the rows below 64: its two columns only
      *reinterpret_cast<float2*>(out + lay.at(r, 4 * q)) = make_float2(v.x, v.y);
    } else {
      *reinterpret_cast<float4*>(out + lay.at(r, 4 * q)) = v;
    }
  }
}

__global__ __launch_bounds__(64) void k_patch_factor_mfma(LevelView L, PatchView P, int first,
                                                          const double* __restrict__ Jv,
                                                          float* __restrict__ fac,
                                                          int* __restrict__ status) {
  __shared__ MfmaFactorLds S;
  const int p = P.order[first + blockIdx.x / P.fac_slabs], n = blockIdx.x % P.fac_slabs;
  factor_block_mfma(L, P, p, n, Jv, fac, status, S);
}

// Persistent form over the big blocks of many problems (see
// launch_patch_factor_batch): tiles taken from a counter, the last
// workgroup to finish resets the counter pair.
__global__ __launch_bounds__(64) void k_patch_factor_mfma_batch(const FactorJob* __restrict__ jobs,
                                                                const FactorTile* __restrict__ tiles,
                                                                int n_tiles, int* __restrict__ ctr) {
  __shared__ MfmaFactorLds S;
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(&ctr[0], 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (t >= n_tiles) break;
    const FactorTile tl = tiles[t];
    const FactorJob& J = jobs[tl.job];
    const int ns = J.P.fac_slabs;
    for (int b = tl.first; b < tl.first + tl.count; ++b) {
      const int p = J.P.order[b / ns], n = b % ns;
      factor_block_mfma(J.L, J.P, p, n, J.Jv, J.fac, J.status, S);
      __syncthreads();
    }
  }
  if (threadIdx.x == 0 && atomicAdd(&ctr[1], 1) == (int)gridDim.x - 1) {
    atomicExch(&ctr[0], 0);
    atomicExch(&ctr[1], 0);
  }
}

}  // namespace

hipError_t launch_patch_factor_mfma_batch(const FactorJob* jobs, const FactorTile* tiles, int n_tiles, int grid,
                                          int* ctr, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_patch_factor_mfma_batch, dim3((unsigned)grid), dim3(64), 0, s, jobs, tiles, n_tiles, ctr);
  return hipGetLastError();
}

int patch_factor_mfma_batch_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_patch_factor_mfma_batch, 64, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

hipError_t launch_patch_factor_mfma(const LevelView& L, const PatchView& P, const double* Jv, float* fac,
                                    int* status, int first, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_patch_factor_mfma, dim3((unsigned)count * P.fac_slabs), dim3(64), 0, s, L, P, first, Jv,
                     fac, status);
  return hipGetLastError();
}

}  // namespace stwr
