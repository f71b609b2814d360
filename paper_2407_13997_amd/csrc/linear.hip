// Space-time operator application, grid transfers, Krylov vector kernels and
// the coarsest-level direct solve on gfx950.
//
// Vector layout: [free DoF][slab][temporal node], so one DoF's N * NQ values
// are contiguous and a lane per (row, slab) reads its row's coefficients
// Jv[k][n][.][.] coalesced across consecutive slabs.
#include "device.h"

namespace stwr {

namespace {

constexpr int kBlock = 256;

// y = A x or y = b - A x for the space-time operator of one level:
// block diagonal part from Jv, plus the jump coupling of slab n to slab n-1,
// -e0 (x) (M * (e1 . x_{n-1})), on velocity rows.  One lane per (row, slab).
// TO: the output's type (FP32 for the residual of the FP32 sweep: the value
// is formed in FP64 and rounded once on the store).  U > 1: a row's entries
// U at a time, every load of a group issued before any is used (the long
// rows of the Taylor-Hood P3-P2 levels; on P2-P1 rows the extra registers
// cost more than the shorter wait).  The arithmetic is the same either way.
template <int NQ, typename TO = double, int U = 1>
__global__ __launch_bounds__(kBlock) void k_spmv(int nf, int po, int N, const int* __restrict__ rp,
                                                 const int* __restrict__ col,
                                                 const double* __restrict__ Jv,
                                                 const double* __restrict__ Mv, TimeEnds te,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ b,
                                                 TO* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (int64_t)nf * N) return;
  const int i = (int)(t / N), n = (int)(t % N);
  const double* e0 = te.e0;
  const double* e1 = te.e1;
  double acc[NQ];
  for (int a = 0; a < NQ; ++a) acc[a] = 0.0;
  double jump = 0.0;
  const bool prow = i >= po;
  if constexpr (U == 1) {
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int j = col[k];
      const double m = Mv[k];
      const double* xv = x + ((int64_t)j * N + n) * NQ;
      // an entry of a pressure row or column is the pressure coupling
      // -dt W (x) B, the same in every slab (linear in the state, uniform
      // slabs): read slab 0's copy, one line for the whole row, so the
      // operator streams only the slab-dependent velocity-velocity blocks
      const bool pc = prow || j >= po;
      const double* v = Jv + ((int64_t)k * N + (pc ? 0 : n)) * NQ * NQ;
      // the previous slab's values (unused at n = 0), loaded with the entry's
      // other values and its mass coefficient so that an entry costs two
      // memory round trips (its column, then everything else) instead of three
      const double* xq = xv - (n > 0 ? NQ : 0);
      double xb[NQ], xp[NQ];
      for (int bb = 0; bb < NQ; ++bb) { xb[bb] = xv[bb]; xp[bb] = xq[bb]; }
      for (int a = 0; a < NQ; ++a)
        for (int bb = 0; bb < NQ; ++bb) acc[a] += v[a * NQ + bb] * xb[bb];
      if (n > 0 && m != 0.0) {
        double xl = 0.0;
        for (int bb = 0; bb < NQ; ++bb) xl += e1[bb] * xp[bb];
        jump += m * xl;
      }
    }
  } else {
    const int kb = rp[i], ke = rp[i + 1];
    for (int k0 = kb; k0 < ke; k0 += U) {
      int jg[U];
      double mg[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u < ke ? k0 + u : ke - 1;   // clamped: past the row's end the entry is unused
        jg[u] = col[k];
        mg[u] = Mv[k];
      }
      double xb[U][NQ], xp[U][NQ], v[U][NQ * NQ];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u < ke ? k0 + u : ke - 1;
        const double* xv = x + ((int64_t)jg[u] * N + n) * NQ;
        const bool pc = prow || jg[u] >= po;
        const double* vk = Jv + ((int64_t)k * N + (pc ? 0 : n)) * NQ * NQ;
        const double* xq = xv - (n > 0 ? NQ : 0);
#pragma unroll
        for (int bb = 0; bb < NQ; ++bb) {
          xb[u][bb] = xv[bb];
          xp[u][bb] = xq[bb];
        }
#pragma unroll
        for (int e = 0; e < NQ * NQ; ++e) v[u][e] = vk[e];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k0 + u < ke) {
          for (int a = 0; a < NQ; ++a)
            for (int bb = 0; bb < NQ; ++bb) acc[a] += v[u][a * NQ + bb] * xb[u][bb];
          if (n > 0 && mg[u] != 0.0) {
            double xl = 0.0;
            for (int bb = 0; bb < NQ; ++bb) xl += e1[bb] * xp[u][bb];
            jump += mg[u] * xl;
          }
        }
      }
    }
  }
  TO* yo = y + t * NQ;
  for (int a = 0; a < NQ; ++a) {
    const double out = acc[a] - e0[a] * jump;
    yo[a] = (TO)(b ? b[t * NQ + a] - out : out);
  }
}

// y[r][t] (+)= sum_k val[k] x[col[k]][t]  (nt values per row)
__global__ __launch_bounds__(kBlock) void k_transfer(int n_rows, int nt, const int* __restrict__ ptr,
                                                     const int* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ y, int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)n_rows * nt) return;
  const int r = (int)(e / nt), t = (int)(e % nt);
  double acc = 0.0;
  for (int k = ptr[r]; k < ptr[r + 1]; ++k) acc += val[k] * x[(int64_t)col[k] * nt + t];
  y[e] = accumulate ? y[e] + acc : acc;
}

__global__ __launch_bounds__(kBlock) void k_gather(int n, int nt, const int* __restrict__ map,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)n * nt) return;
  const int r = (int)(e / nt), t = (int)(e % nt);
  y[e] = x[(int64_t)map[r] * nt + t];
}

__device__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kBlock / 64; ++k) s += red[k];
  __syncthreads();
  return s;
}

constexpr int kDotBlocks = 256;

__global__ __launch_bounds__(kBlock) void k_mdot_partial(int64_t n, const double* __restrict__ X,
                                                         int64_t ldx, const double* __restrict__ y,
                                                         double* __restrict__ partial) {
  const int k = blockIdx.y;
  const double* xk = X + k * ldx;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (int64_t)kDotBlocks * kBlock)
    s += xk[e] * y[e];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[k * kDotBlocks + blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_mdot_final(const double* __restrict__ partial,
                                                       double* __restrict__ out) {
  const int k = blockIdx.x;
  double s = block_sum(partial[k * kDotBlocks + threadIdx.x]);
  if (threadIdx.x == 0) out[k] = s;
}

__global__ __launch_bounds__(kBlock) void k_axpy_dev(int64_t n, const double* __restrict__ coef,
                                                     double scale, const double* __restrict__ x,
                                                     double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) y[e] += scale * coef[0] * x[e];
}

__global__ __launch_bounds__(kBlock) void k_axpby(int64_t n, double a, const double* x, double b,
                                                  double* y) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) y[e] = (b == 0.0 ? 0.0 : b * y[e]) + a * x[e];
}

__global__ __launch_bounds__(kBlock) void k_scale_dev(int64_t n, const double* __restrict__ num,
                                                      int invert, const double* x, double* y) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) y[e] = invert ? x[e] / num[0] : x[e] * num[0];
}

// Attainable HBM read rate: a grid-stride read of n4 16-byte vectors with
// nontemporal loads (each lane one vector in flight at a time), one partial
// sum per thread written out so the loads are not dropped.
typedef float stream_f4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kBlock) void k_stream_read(const stream_f4* __restrict__ x, int64_t n4,
                                                        float* __restrict__ out) {
  float acc = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) {
    const stream_f4 v = __builtin_nontemporal_load(x + i);
    acc += (v.x + v.y) + (v.z + v.w);
  }
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, double v, double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) y[e] = v;
}

// v[i] = frac(0.6180339887498949 i) - 0.5, the fixed Arnoldi start vector
__global__ __launch_bounds__(kBlock) void k_start_vector(int64_t n, double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) {
    const double v = (double)e * 0.6180339887498949;
    y[e] = (v - floor(v)) - 0.5;
  }
}

// mean of the pressure DoFs per (slab, temporal node) column t
__global__ __launch_bounds__(kBlock) void k_pmean(int nf, int po, int nt, const double* __restrict__ x,
                                                  double* __restrict__ mean) {
  const int t = blockIdx.x;
  double s = 0.0;
  for (int i = po + threadIdx.x; i < nf; i += kBlock) s += x[(int64_t)i * nt + t];
  s = block_sum(s);
  if (threadIdx.x == 0) mean[t] = s / (nf - po);
}

__global__ __launch_bounds__(kBlock) void k_psub(int nf, int po, int nt, double* __restrict__ x,
                                                 const double* __restrict__ mean) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)(nf - po) * nt) return;
  const int t = (int)(e % nt);
  x[(int64_t)po * nt + e] -= mean[t];
}

__global__ __launch_bounds__(kBlock) void k_gemv_cols(int64_t n, int k, const double* __restrict__ Z,
                                                      int64_t ldz, const double* __restrict__ yv,
                                                      double* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc += Z[j * ldz + e] * yv[j];
  x[e] += acc;
}

// Dense bordered slab blocks of the coarsest level: B_n = [J_nn C; C^T 0],
// C = one indicator column of the pressure DoFs per temporal node (nbord =
// q + 1 columns); without a pressure (nbord = 0) B_n = J_nn.
template <int NQ>
__global__ __launch_bounds__(kBlock) void k_coarse_build(int nf, int po, int N, int nbord, int nbuild,
                                                         const int* __restrict__ rp,
                                                         const int* __restrict__ col,
                                                         const double* __restrict__ Jv,
                                                         double* __restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (int64_t)nf * N) return;
  const int i = (int)(t / N), n = (int)(t % N);
  if (n >= nbuild) return;   // slabs sharing the first slab's block
  const int m = nf * NQ, mm = m + nbord;
  double* Bn = B + (int64_t)n * mm * mm;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = col[k];
    const double* v = Jv + ((int64_t)k * N + n) * NQ * NQ;
    for (int a = 0; a < NQ; ++a)
      for (int b = 0; b < NQ; ++b) Bn[(int64_t)(i * NQ + a) * mm + j * NQ + b] = v[a * NQ + b];
  }
  if (i >= po) {
    for (int a = 0; a < NQ; ++a) {
      Bn[(int64_t)(i * NQ + a) * mm + m + a] = 1.0;
      Bn[(int64_t)(m + a) * mm + i * NQ + a] = 1.0;
    }
  }
}

constexpr int kMaxCoarse = 4096;

// In-place Gauss-Jordan inversion with partial pivoting of B[blockIdx.x]
// (m x m, row-major, global memory), one workgroup per matrix.
__global__ __launch_bounds__(kBlock) void k_dense_inverse(int m, double* __restrict__ Ball,
                                                          int* __restrict__ status) {
  double* B = Ball + (int64_t)blockIdx.x * m * m;
  __shared__ int perm[kCoarseSmall];
  __shared__ double colk[kCoarseSmall];
  __shared__ double rv[kBlock / 64];
  __shared__ int ri[kBlock / 64];
  __shared__ int piv_s;
  const int tid = threadIdx.x;
  for (int k = 0; k < m; ++k) {
    double best = -1.0;
    int bi = m;
    for (int i = k + tid; i < m; i += kBlock) {
      const double v = fabs(B[(int64_t)i * m + k]);
      if (v > best || (v == best && i < bi)) { best = v; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (tid % 64 == 0) { rv[tid / 64] = best; ri[tid / 64] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = rv[0];
      int p = ri[0];
      for (int w = 1; w < kBlock / 64; ++w)
        if (rv[w] > b || (rv[w] == b && ri[w] < p)) { b = rv[w]; p = ri[w]; }
      if (!(b > 0.0) || !isfinite(b) || p >= m) {
        status[0] = 1;
        p = k;
      }
      piv_s = p;
      perm[k] = p;
    }
    __syncthreads();
    const int p = piv_s;
    if (p != k)
      for (int j = tid; j < m; j += kBlock) {
        const double a = B[(int64_t)k * m + j];
        B[(int64_t)k * m + j] = B[(int64_t)p * m + j];
        B[(int64_t)p * m + j] = a;
      }
    __syncthreads();
    const double pv = B[(int64_t)k * m + k];
    __syncthreads();
    for (int j = tid; j < m; j += kBlock)
      B[(int64_t)k * m + j] = (j == k ? 1.0 : B[(int64_t)k * m + j]) / pv;
    for (int i = tid; i < m; i += kBlock) colk[i] = B[(int64_t)i * m + k];
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)m * m; e += kBlock) {
      const int i = (int)(e / m), j = (int)(e % m);
      if (i == k) continue;
      const double f = colk[i];
      if (j == k) B[e] = -f * B[(int64_t)k * m + k];
      else B[e] -= f * B[(int64_t)k * m + j];
    }
    __syncthreads();
  }
  for (int k = m - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = tid; i < m; i += kBlock) {
        const double a = B[(int64_t)i * m + k];
        B[(int64_t)i * m + k] = B[(int64_t)i * m + p];
        B[(int64_t)i * m + p] = a;
      }
    __syncthreads();
  }
}

// Dense inverses over kCoarseSmall rows when no panel workspace is given
// (rbuf = NULL): Gauss-Jordan with partial pivoting spread
// over the chip, one elimination step per pair of launches.  k_gj_pivot (one
// workgroup per matrix) picks the pivot of column k, swaps it into row k,
// scales row k and saves column k; k_gj_update applies the rank-1 update to
// every other row of every matrix; k_gj_unpermute undoes the column order.
__global__ __launch_bounds__(kBlock) void k_gj_pivot(int m, int k, double* __restrict__ Ball,
                                                     int* __restrict__ perm,
                                                     double* __restrict__ colbuf,
                                                     int* __restrict__ status) {
  double* B = Ball + (int64_t)blockIdx.x * m * m;
  __shared__ double rv[kBlock / 64];
  __shared__ int ri[kBlock / 64];
  __shared__ int piv_s;
  const int tid = threadIdx.x;
  double best = -1.0;
  int bi = m;
  for (int i = k + tid; i < m; i += kBlock) {
    const double v = fabs(B[(int64_t)i * m + k]);
    if (v > best || (v == best && i < bi)) { best = v; bi = i; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
  }
  if (tid % 64 == 0) { rv[tid / 64] = best; ri[tid / 64] = bi; }
  __syncthreads();
  if (tid == 0) {
    double b = rv[0];
    int p = ri[0];
    for (int w = 1; w < kBlock / 64; ++w)
      if (rv[w] > b || (rv[w] == b && ri[w] < p)) { b = rv[w]; p = ri[w]; }
    if (!(b > 0.0) || !isfinite(b) || p >= m) {
      status[0] = 1;
      p = k;
    }
    piv_s = p;
    perm[(int64_t)blockIdx.x * m + k] = p;
  }
  __syncthreads();
  const int p = piv_s;
  if (p != k)
    for (int j = tid; j < m; j += kBlock) {
      const double a = B[(int64_t)k * m + j];
      B[(int64_t)k * m + j] = B[(int64_t)p * m + j];
      B[(int64_t)p * m + j] = a;
    }
  __syncthreads();
  const double pv = B[(int64_t)k * m + k];
  __syncthreads();
  for (int j = tid; j < m; j += kBlock)
    B[(int64_t)k * m + j] = (j == k ? 1.0 : B[(int64_t)k * m + j]) / pv;
  double* col = colbuf + (int64_t)blockIdx.x * m;
  for (int i = tid; i < m; i += kBlock) col[i] = B[(int64_t)i * m + k];
}

__global__ __launch_bounds__(kBlock) void k_gj_update(int m, int k, double* __restrict__ Ball,
                                                      const double* __restrict__ colbuf) {
  double* B = Ball + (int64_t)blockIdx.y * m * m;
  const double* col = colbuf + (int64_t)blockIdx.y * m;
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int i = (int)(e / m), j = (int)(e % m);
  if (i == k) return;
  const double f = col[i];
  if (j == k) B[e] = -f * B[(int64_t)k * m + k];
  else B[e] -= f * B[(int64_t)k * m + j];
}

__global__ __launch_bounds__(kBlock) void k_gj_unpermute(int m, double* __restrict__ Ball,
                                                         const int* __restrict__ perm) {
  double* B = Ball + (int64_t)blockIdx.y * m * m;
  const int* pm = perm + (int64_t)blockIdx.y * m;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= m) return;
  double* row = B + (int64_t)i * m;
  for (int k = m - 1; k >= 0; --k) {
    const int p = pm[k];
    if (p != k) {
      const double a = row[k];
      row[k] = row[p];
      row[p] = a;
    }
  }
}

// Blocked form for the largest coarse blocks: column panels of kGjPanel.
// The elimination steps of a panel compose to a transform that differs from
// the identity only in the panel columns (which the in-place steps leave
// holding it), so the other columns only need the panel's row swaps and one
// rank-kGjPanel update A += W R with W = (panel columns - selector) and R the
// panel rows of those columns: one pass over each matrix per panel instead of
// one per column.
constexpr int kGjPanel = 32;
// narrower panels where a thread keeps 4, 6 or 8 rows' segments in registers
constexpr int kGjPanel4 = 24;   // 1536 < m <= 2048
constexpr int kGjPanel6 = 16;   // 2048 < m <= 3072
constexpr int kGjPanel8 = 10;   // 3072 < m <= kMaxCoarse
static_assert(kGjPanel8 <= kGjPanel6 && kGjPanel4 <= kGjPanel, "the update's staging bounds the narrow panels");

// Row swaps of the panel applied to every non-panel column, then the panel
// rows of those columns copied to R (rows roff.. of the rstride elements of
// each matrix's R).
__global__ __launch_bounds__(kBlock) void k_bgj_swap(int m, int k0, int k1, double* __restrict__ Ball,
                                                     const int* __restrict__ perm,
                                                     double* __restrict__ Rall, int64_t rstride, int roff) {
  double* B = Ball + (int64_t)blockIdx.y * m * m;
  const int* pm = perm + (int64_t)blockIdx.y * m;
  double* R = Rall + (int64_t)blockIdx.y * rstride + (int64_t)roff * m;
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= m || (j >= k0 && j < k1)) return;
  for (int k = k0; k < k1; ++k) {
    const int p = pm[k];
    if (p != k) {
      const double a = B[(int64_t)k * m + j];
      B[(int64_t)k * m + j] = B[(int64_t)p * m + j];
      B[(int64_t)p * m + j] = a;
    }
  }
  for (int k = k0; k < k1; ++k) R[(int64_t)(k - k0) * m + j] = B[(int64_t)k * m + j];
}

// A[i][j] += sum_t W[i][t] R[t][j] over non-panel columns j, in 64 x 64 tiles
// (panels of at most PBM columns: the staging takes no more LDS than that),
// on the FP64 matrix cores: each of the four wavefronts takes a 16-row strip
// of the tile, four 16 x 16 output tiles held in accumulators initialised
// with the matrix's own values, and every four panel columns issue one
// v_mfma_f64_16x16x4f64 per output tile (lane l holds W[l % 16][l / 16] and
// R[l / 16][l % 16] of the 16 x 4 and 4 x 16 operands, and rows l / 16 + 4 r,
// r < 4, of column l % 16 of the output).
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
template <int PBM>
__global__ __launch_bounds__(kBlock) void k_bgj_update(int m, int k0, int k1, double* __restrict__ Ball,
                                                       const double* __restrict__ Rall, int64_t rstride) {
  double* B = Ball + (int64_t)blockIdx.z * m * m;
  const double* R = Rall + (int64_t)blockIdx.z * rstride;
  __shared__ double Ws[64][PBM + 1];
  __shared__ double Rs[PBM][64 + 1];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64, tid = threadIdx.x, b = k1 - k0;
  if (j0 + 64 > k0 && j0 < k1 && j0 >= k0 && j0 + 64 <= k1) return;   // tile inside the panel
  const int w = tid / 64, lane = tid % 64, lr = lane % 16, lk = lane / 16;
  // this lane's outputs, loaded first (clamped addresses, so every load is
  // issued at once and their latency overlaps the staging below)
  mfma_d4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int j = min(j0 + 16 * ct + lr, m - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[ct][q] = B[(int64_t)min(i0 + 16 * w + lk + 4 * q, m - 1) * m + j];
  }
  // W and R staged in LDS: every thread's loads issued at once (clamped
  // addresses, zeros selected afterwards), then stored, so the staging costs
  // one memory latency instead of one per element a thread stages
  static_assert((64 * PBM) % kBlock == 0, "whole staging rounds");
  constexpr int NS = 64 * PBM / kBlock;
  double wv[NS], rv[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const int e = tid + u * kBlock;
    const int r = e / PBM, t = e % PBM, i = i0 + r;
    wv[u] = B[(int64_t)min(i, m - 1) * m + k0 + min(t, b - 1)];
    const int t2 = e / 64, c = e % 64;
    rv[u] = R[(int64_t)min(t2, b - 1) * m + min(j0 + c, m - 1)];
  }
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const int e = tid + u * kBlock;
    const int r = e / PBM, t = e % PBM, i = i0 + r;
    Ws[r][t] = (i < m && t < b) ? wv[u] - (i == k0 + t ? 1.0 : 0.0) : 0.0;
    const int t2 = e / 64, c = e % 64;
    Rs[t2][c] = (t2 < b && j0 + c < m) ? rv[u] : 0.0;
  }
  __syncthreads();
  // the staging is zero past b, so whole groups of four are exact
  for (int t0 = 0; t0 < b; t0 += 4) {
    const double a = Ws[16 * w + lr][t0 + lk];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Rs[t0 + lk][16 * ct + lr], acc[ct], 0, 0, 0);
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int j = j0 + 16 * ct + lr;
    if (j >= m || (j >= k0 && j < k1)) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + 16 * w + lk + 4 * q;
      if (i < m) B[(int64_t)i * m + j] = acc[ct][q];
    }
  }
}

// Two panels per pass over the matrix (look-ahead): after panel p (columns
// [k0, k1)) is factored and swapped, the next panel's columns receive p's
// update alone (k_bgj_cols), panel p+1 is factored and swapped, its rows R2
// of the columns not yet updated are brought up to date with p's transform
// (k_bgj_rfix: R2 += W_p[rows of p+1] R_p), and one rank-(b_p + b_p+1) pass
// updates every other column with both transforms, W = A[:, k0:k2] - the
// selector of rows k0..k2, R = [R_p; R2].  Finally panel p's own columns
// receive p+1's update (k_bgj_cols).  The composition is the product of the
// two panels' Gauss-Jordan transforms, as two passes would apply it, at half
// the memory traffic of the dominant update.
//
// A[i][c] += sum_s (A[i][w0 + s] - [i == w0 + s]) R[roff + s][c] for the
// columns c in [c0, c1), every row i.
__global__ __launch_bounds__(kBlock) void k_bgj_cols(int m, int w0, int bw, int c0, int c1,
                                                     double* __restrict__ Ball,
                                                     const double* __restrict__ Rall, int64_t rstride,
                                                     int roff) {
  double* B = Ball + (int64_t)blockIdx.y * m * m;
  const double* R = Rall + (int64_t)blockIdx.y * rstride + (int64_t)roff * m;
  const int nc = c1 - c0;
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)m * nc) return;
  const int i = (int)(e / nc), c = c0 + (int)(e % nc);
  const double* wrow = B + (int64_t)i * m + w0;
  double acc = 0.0;
#pragma unroll 8
  for (int s2 = 0; s2 < bw; ++s2) acc += (wrow[s2] - (i == w0 + s2 ? 1.0 : 0.0)) * R[(int64_t)s2 * m + c];
  B[(int64_t)i * m + c] += acc;
}

// R[roff2 + t][j] += sum_s A[k1 + t][k0 + s] R[s][j], t < k2 - k1, s < k1 - k0,
// for the columns j outside [k0, k2): the second panel's rows brought up to
// date with the first panel's transform (their rows k1.. are not the first
// panel's rows, so its selector contributes nothing).
__global__ __launch_bounds__(kBlock) void k_bgj_rfix(int m, int k0, int k1, int k2,
                                                     const double* __restrict__ Ball,
                                                     double* __restrict__ Rall, int64_t rstride, int roff2) {
  const double* B = Ball + (int64_t)blockIdx.z * m * m;
  double* R = Rall + (int64_t)blockIdx.z * rstride;
  const int t = blockIdx.y, j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= m || (j >= k0 && j < k2)) return;
  const double* wrow = B + (int64_t)(k1 + t) * m + k0;
  double acc = 0.0;
#pragma unroll 8
  for (int s2 = 0; s2 < k1 - k0; ++s2) acc += wrow[s2] * R[(int64_t)s2 * m + j];
  R[(int64_t)(roff2 + t) * m + j] += acc;
}

// Register-resident panel of the blocked Gauss-Jordan inverse, for m <= 512 RP:
// thread t keeps the panel segments (PB columns) of rows t + 512 r, r < RP,
// in registers for the whole panel, so a column step costs a few LDS
// exchanges instead of a pass over the panel in memory.  After each step the
// segments rotate left by one column, so the active column is always
// register 0 and every register index is static; after b steps position j
// holds panel column (j + b) mod PB.  Per element the arithmetic is that of
// the column-at-a-time Gauss-Jordan inverse restricted to the panel columns
// (the pivot row scaled by the pivot's reciprocal), and the pivot is the
// largest magnitude, ties to the smaller row.
constexpr int kPanelThreads = 512;
template <int RP, int PB>
__global__ __launch_bounds__(kPanelThreads) void k_bgj_panel_reg(int m, int k0, int k1,
                                                                 double* __restrict__ Ball,
                                                                 int* __restrict__ perm,
                                                                 int* __restrict__ status) {
  constexpr int T = kPanelThreads, NW = T / 64;
  double* B = Ball + (int64_t)blockIdx.x * m * m;
  int* pm = perm + (int64_t)blockIdx.x * m;
  __shared__ double rv[NW];
  __shared__ int ri[NW];
  __shared__ double swp[2][PB];
  __shared__ double prow[PB];
  const int tid = threadIdx.x, b = k1 - k0;
  double a[RP][PB];
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int i = tid + T * r;
#pragma unroll
    for (int j = 0; j < PB; ++j) a[r][j] = (i < m && j < b) ? B[(int64_t)i * m + k0 + j] : 0.0;
  }
  for (int kk = 0; kk < b; ++kk) {
    const int k = k0 + kk;
    // pivot: largest |a| in column k among rows >= k, ties to the smaller
    // row: each wavefront's maximum (DPP) and the first of its rows holding
    // it (ballots; register r = 0 holds its smaller rows), then the best over
    // the wavefronts through LDS
    double vr[RP];
    double vmax = -1.0;
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int i = tid + T * r;
      vr[r] = (i >= k && i < m) ? fabs(a[r][0]) : -1.0;
      vmax = fmax(vmax, vr[r]);
    }
    const double best = wave_max(vmax);
    int bi = m;
#pragma unroll
    for (int r = RP - 1; r >= 0; --r) {
      const uint64_t hit = __ballot(vr[r] == best);
      if (hit) bi = T * r + (tid / 64) * 64 + __ffsll((unsigned long long)hit) - 1;
    }
    if (tid % 64 == 0) { rv[tid / 64] = best; ri[tid / 64] = bi; }
    __syncthreads();
    double bb = rv[0];
    int p = ri[0];
    for (int w = 1; w < NW; ++w)
      if (rv[w] > bb || (rv[w] == bb && ri[w] < p)) { bb = rv[w]; p = ri[w]; }
    if (!(bb > 0.0) || !isfinite(bb) || p >= m) {
      if (tid == 0) status[0] = 1;
      p = k;
    }
    if (tid == 0) pm[k] = p;
    // swap rows k and p of the panel (uniform branch)
    if (p != k) {
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const int i = tid + T * r;
        if (i == p)
#pragma unroll
          for (int j = 0; j < PB; ++j) swp[0][j] = a[r][j];
        if (i == k)
#pragma unroll
          for (int j = 0; j < PB; ++j) swp[1][j] = a[r][j];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const int i = tid + T * r;
        if (i == k)
#pragma unroll
          for (int j = 0; j < PB; ++j) a[r][j] = swp[0][j];
        if (i == p)
#pragma unroll
          for (int j = 0; j < PB; ++j) a[r][j] = swp[1][j];
      }
    }
    // scale the pivot row by the pivot's reciprocal: the pivot entry becomes
    // 1 / pivot
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      if (tid + T * r == k) {
        const double rp = 1.0 / a[r][0];
#pragma unroll
        for (int j = 0; j < PB; ++j) {
          a[r][j] = (j == 0 ? 1.0 : a[r][j]) * rp;
          prow[j] = a[r][j];
        }
      }
    }
    __syncthreads();
    // eliminate column k from every other row (column by column, so each
    // pivot-row value is read from LDS just before its use), then rotate
    double f[RP];
    bool live[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int i = tid + T * r;
      live[r] = i < m && i != k;
      f[r] = a[r][0];
    }
    {
      const double p0 = prow[0];
#pragma unroll
      for (int r = 0; r < RP; ++r)
        if (live[r]) a[r][0] = -f[r] * p0;
    }
#pragma unroll
    for (int j = 1; j < PB; ++j) {
      const double pj = prow[j];
#pragma unroll
      for (int r = 0; r < RP; ++r)
        if (live[r]) a[r][j] = a[r][j] - f[r] * pj;
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const double t0 = a[r][0];
#pragma unroll
      for (int j = 0; j + 1 < PB; ++j) a[r][j] = a[r][j + 1];
      a[r][PB - 1] = t0;
    }
  }
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int i = tid + T * r;
    if (i < m)
#pragma unroll
      for (int j = 0; j < PB; ++j) {
        const int c = (j + b) % PB;
        if (c < b) B[(int64_t)i * m + k0 + c] = a[r][j];
      }
  }
}

// Forward block substitution over the slabs of the coarsest level with the
// inverted bordered slab blocks; one workgroup walks the slabs in order.
template <int NQ>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(int nf, int po, int N, int nbord, int cs,
                                                         const int* __restrict__ rp,
                                                         const int* __restrict__ col,
                                                         const double* __restrict__ Mv, TimeEnds te,
                                                         const double* __restrict__ Binv,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ x) {
  __shared__ double g[kCoarseSmall];
  const int m = nf * NQ, mm = m + nbord;
  const double* e0 = te.e0;
  const double* e1 = te.e1;
  const int tid = threadIdx.x;
  for (int n = 0; n < N; ++n) {
    for (int r = tid; r < m; r += kBlock) {
      const int i = r / NQ, a = r % NQ;
      double v = b[((int64_t)i * N + n) * NQ + a];
      if (n > 0 && i < po) {
        double jump = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
          const double mk = Mv[k];
          if (mk == 0.0) continue;
          const double* xv = x + ((int64_t)col[k] * N + n - 1) * NQ;
          double xl = 0.0;
          for (int bb = 0; bb < NQ; ++bb) xl += e1[bb] * xv[bb];
          jump += mk * xl;
        }
        v += e0[a] * jump;
      }
      g[r] = v;
    }
    if (tid < nbord) g[m + tid] = 0.0;
    __syncthreads();
    const double* Bn = Binv + (int64_t)(n % cs) * mm * mm;
    for (int r = tid; r < m; r += kBlock) {
      double acc = 0.0;
      for (int c = 0; c < mm; ++c) acc += Bn[(int64_t)r * mm + c] * g[c];
      const int i = r / NQ, a = r % NQ;
      x[((int64_t)i * N + n) * NQ + a] = acc;
    }
    __syncthreads();
  }
}

// Large coarsest levels: one slab at a time, with the right-hand side
// g = b_n + e0 (x) (M (e1 . x_{n-1})) formed by one kernel and the product with
// the inverted bordered block by another, many workgroups each.  The
// right-hand side takes 16 lanes per row, each summing every 16th nonzero of
// the row's mass entries.
template <int NQ>
__global__ __launch_bounds__(kBlock) void k_coarse_rhs(int nf, int po, int N, int n, int nbord,
                                                       const int* __restrict__ rp,
                                                       const int* __restrict__ col,
                                                       const double* __restrict__ Mv, TimeEnds te,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ g) {
  const int r = blockIdx.x * (kBlock / 16) + threadIdx.x / 16, l = threadIdx.x % 16;
  const int m = nf * NQ;
  if (r >= m + nbord) return;
  if (r >= m) {
    if (l == 0) g[r] = 0.0;
    return;
  }
  const double* e0 = te.e0;
  const double* e1 = te.e1;
  const int i = r / NQ, a = r % NQ;
  const bool jumps = n > 0 && i < po;
  double jump = 0.0;
  if (jumps) {
    for (int k = rp[i] + l; k < rp[i + 1]; k += 16) {
      const double* xv = x + ((int64_t)col[k] * N + n - 1) * NQ;
      double xl = 0.0;
      for (int bb = 0; bb < NQ; ++bb) xl += e1[bb] * xv[bb];
      jump += Mv[k] * xl;
    }
  }
  for (int off = 8; off > 0; off >>= 1) jump += __shfl_xor(jump, off, 16);
  if (l == 0) {
    const double v = b[((int64_t)i * N + n) * NQ + a];
    g[r] = jumps ? v + e0[a] * jump : v;
  }
}

// x_n = (inverse slab block) g, one wavefront per row, four rows per
// workgroup; every lane issues all its loads of the row before reducing.
template <int NQ>
__global__ __launch_bounds__(kBlock) void k_coarse_gemv(int nf, int N, int n, int mm,
                                                        const double* __restrict__ Bn,
                                                        const double* __restrict__ g,
                                                        double* __restrict__ x) {
  const int row = blockIdx.x * (kBlock / 64) + threadIdx.x / 64, l = threadIdx.x % 64;
  const int m = nf * NQ;
  if (row >= m) return;
  const double* br = Bn + (int64_t)row * mm;
  double acc = 0.0;
  int c = l;
  for (; c + 192 < mm; c += 256)
    acc += br[c] * g[c] + br[c + 64] * g[c + 64] + br[c + 128] * g[c + 128] + br[c + 192] * g[c + 192];
  for (; c < mm; c += 64) acc += br[c] * g[c];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (l == 0) {
    const int i = row / NQ, a = row % NQ;
    x[((int64_t)i * N + n) * NQ + a] = acc;
  }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// one launch per temporal-node count: every NQ-templated launcher below
// switches over 1..kMaxNQ
#define STWR_NQ_SWITCH(NQ, CALL)                 \
  switch (NQ) {                                  \
    case 1: { constexpr int Q = 1; CALL; } break; \
    case 2: { constexpr int Q = 2; CALL; } break; \
    case 3: { constexpr int Q = 3; CALL; } break; \
    case 4: { constexpr int Q = 4; CALL; } break; \
    default: return hipErrorInvalidValue;        \
  }

hipError_t launch_spmv(const LevelView& L, const double* Jv, const double* Mv, const double* e0,
                       const double* e1, const double* x, const double* b, double* y,
                       hipStream_t s) {
  const int64_t n = (int64_t)L.nf * L.N;
  const TimeEnds te = time_ends(L.NQ, e0, e1);
  if (L.thk > 0) {
    STWR_NQ_SWITCH(L.NQ, hipLaunchKernelGGL((k_spmv<Q, double, 4>), dim3(nblk(n)), dim3(kBlock), 0, s, L.nf, L.po, L.N,
                                            L.row_ptr, L.col, Jv, Mv, te, x, b, y));
  } else {
    STWR_NQ_SWITCH(L.NQ, hipLaunchKernelGGL((k_spmv<Q, double>), dim3(nblk(n)), dim3(kBlock), 0, s, L.nf, L.po, L.N,
                                            L.row_ptr, L.col, Jv, Mv, te, x, b, y));
  }
  return hipGetLastError();
}

hipError_t launch_spmv_f32out(const LevelView& L, const double* Jv, const double* Mv, const double* e0,
                              const double* e1, const double* x, const double* b, float* y, hipStream_t s) {
  if (!b) return hipErrorInvalidValue;
  const int64_t n = (int64_t)L.nf * L.N;
  const TimeEnds te = time_ends(L.NQ, e0, e1);
  STWR_NQ_SWITCH(L.NQ, hipLaunchKernelGGL((k_spmv<Q, float>), dim3(nblk(n)), dim3(kBlock), 0, s, L.nf, L.po, L.N,
                                          L.row_ptr, L.col, Jv, Mv, te, x, b, y));
  return hipGetLastError();
}

hipError_t launch_transfer(int n_rows, int nt, const int* ptr, const int* col, const double* val,
                           const double* x, double* y, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_transfer, dim3(nblk((int64_t)n_rows * nt)), dim3(kBlock), 0, s, n_rows, nt,
                     ptr, col, val, x, y, accumulate);
  return hipGetLastError();
}

hipError_t launch_gather(int n, int nt, const int* map, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(nblk((int64_t)n * nt)), dim3(kBlock), 0, s, n, nt, map, x, y);
  return hipGetLastError();
}

hipError_t launch_mdot(int64_t n, int nvec, const double* X, int64_t ldx, const double* y,
                       double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mdot_partial, dim3(kDotBlocks, nvec), dim3(kBlock), 0, s, n, X, ldx, y,
                     partial);
  hipLaunchKernelGGL(k_mdot_final, dim3(nvec), dim3(kBlock), 0, s, partial, out);
  return hipGetLastError();
}

hipError_t launch_axpy_dev(int64_t n, const double* coef, double scale, const double* x, double* y,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_dev, dim3(nblk(n)), dim3(kBlock), 0, s, n, coef, scale, x, y);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(kBlock), 0, s, n, a, x, b, y);
  return hipGetLastError();
}

hipError_t launch_scale_dev(int64_t n, const double* num, int invert, const double* x, double* y,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_scale_dev, dim3(nblk(n)), dim3(kBlock), 0, s, n, num, invert, x, y);
  return hipGetLastError();
}

hipError_t launch_stream_read(const void* buf, int64_t bytes, int grid, float* out, hipStream_t s) {
  if (bytes < 16 || bytes % 16 != 0 || grid <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(kBlock), 0, s, (const stream_f4*)buf, bytes / 16, out);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(kBlock), 0, s, n, v, y);
  return hipGetLastError();
}

hipError_t launch_start_vector(int64_t n, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_start_vector, dim3(nblk(n)), dim3(kBlock), 0, s, n, y);
  return hipGetLastError();
}

hipError_t launch_pressure_project(int nf, int po, int nt, double* x, double* work, hipStream_t s) {
  hipLaunchKernelGGL(k_pmean, dim3(nt), dim3(kBlock), 0, s, nf, po, nt, x, work);
  hipLaunchKernelGGL(k_psub, dim3(nblk((int64_t)(nf - po) * nt)), dim3(kBlock), 0, s, nf, po, nt, x,
                     work);
  return hipGetLastError();
}

hipError_t launch_gemv_cols(int64_t n, int k, const double* Z, int64_t ldz, const double* y,
                            double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_cols, dim3(nblk(n)), dim3(kBlock), 0, s, n, k, Z, ldz, y, x);
  return hipGetLastError();
}

hipError_t launch_coarse_build(const LevelView& L, const double* Jv, double* B, hipStream_t s) {
  const int64_t n = (int64_t)L.nf * L.N;
  STWR_NQ_SWITCH(L.NQ, hipLaunchKernelGGL(k_coarse_build<Q>, dim3(nblk(n)), dim3(kBlock), 0, s, L.nf,
                                          L.po, L.N, L.nbord, L.coarse_slabs, L.row_ptr, L.col, Jv, B));
  return hipGetLastError();
}

hipError_t launch_dense_inverse(int nmat, int m, double* B, int* status, int* perm,
                                double* colbuf, double* rbuf, hipStream_t s) {
  if (m > kMaxCoarse) return hipErrorInvalidValue;
  if (m <= kCoarseSmall) {
    hipLaunchKernelGGL(k_dense_inverse, dim3(nmat), dim3(kBlock), 0, s, m, B, status);
    return hipGetLastError();
  }
  if (!rbuf) {
    const dim3 gu(nblk((int64_t)m * m), nmat), gp(nblk(m), nmat);
    for (int k = 0; k < m; ++k) {
      hipLaunchKernelGGL(k_gj_pivot, dim3(nmat), dim3(kBlock), 0, s, m, k, B, perm, colbuf, status);
      hipLaunchKernelGGL(k_gj_update, gu, dim3(kBlock), 0, s, m, k, B, colbuf);
    }
    hipLaunchKernelGGL(k_gj_unpermute, gp, dim3(kBlock), 0, s, m, B, perm);
    return hipGetLastError();
  }
  const dim3 gs(nblk(m), nmat), gt((m + 63) / 64, (m + 63) / 64, nmat), gp(nblk(m), nmat);
  // panels of kGjPanel columns up to 3 rows per thread, narrower ones (4, 6
  // or 8 rows per thread, up to kMaxCoarse) so that the panel stays in registers
  const int pw = m <= kPanelThreads * 3 ? kGjPanel
               : m <= kPanelThreads * 4 ? kGjPanel4
               : m <= kPanelThreads * 6 ? kGjPanel6 : kGjPanel8;
  auto panel = [&](int k0, int k1) {
    if (m <= kPanelThreads)
      hipLaunchKernelGGL((k_bgj_panel_reg<1, kGjPanel>), dim3(nmat), dim3(kPanelThreads), 0, s, m, k0, k1, B, perm, status);
    else if (m <= kPanelThreads * 2)
      hipLaunchKernelGGL((k_bgj_panel_reg<2, kGjPanel>), dim3(nmat), dim3(kPanelThreads), 0, s, m, k0, k1, B, perm, status);
    else if (m <= kPanelThreads * 3)
      hipLaunchKernelGGL((k_bgj_panel_reg<3, kGjPanel>), dim3(nmat), dim3(kPanelThreads), 0, s, m, k0, k1, B, perm, status);
    else if (m <= kPanelThreads * 4)
      hipLaunchKernelGGL((k_bgj_panel_reg<4, kGjPanel4>), dim3(nmat), dim3(kPanelThreads), 0, s, m, k0, k1, B, perm, status);
    else if (m <= kPanelThreads * 6)
      hipLaunchKernelGGL((k_bgj_panel_reg<6, kGjPanel6>), dim3(nmat), dim3(kPanelThreads), 0, s, m, k0, k1, B, perm, status);
    else
      hipLaunchKernelGGL((k_bgj_panel_reg<8, kGjPanel8>), dim3(nmat), dim3(kPanelThreads), 0, s, m, k0, k1, B, perm, status);
  };
  // the update pass with W = A[:, k0:k1] and R's first k1 - k0 rows
  auto update = [&](int k0, int k1) {
    const int b = k1 - k0;
    if (b <= 32) hipLaunchKernelGGL(k_bgj_update<32>, gt, dim3(kBlock), 0, s, m, k0, k1, B, rbuf, kRbufRows * (int64_t)m);
    else if (b <= 48) hipLaunchKernelGGL(k_bgj_update<48>, gt, dim3(kBlock), 0, s, m, k0, k1, B, rbuf, kRbufRows * (int64_t)m);
    else hipLaunchKernelGGL(k_bgj_update<64>, gt, dim3(kBlock), 0, s, m, k0, k1, B, rbuf, kRbufRows * (int64_t)m);
  };
  const int64_t rs = kRbufRows * (int64_t)m;
  for (int k0 = 0; k0 < m;) {
    const int k1 = k0 + pw < m ? k0 + pw : m;
    panel(k0, k1);
    hipLaunchKernelGGL(k_bgj_swap, gs, dim3(kBlock), 0, s, m, k0, k1, B, perm, rbuf, rs, 0);
    if (k1 == m) {
      update(k0, k1);
      break;
    }
    // a second panel, then one pass for both
    const int k2 = k1 + pw < m ? k1 + pw : m, b1 = k1 - k0, b2 = k2 - k1;
    hipLaunchKernelGGL(k_bgj_cols, dim3(nblk((int64_t)m * b2), nmat), dim3(kBlock), 0, s, m, k0, b1, k1, k2, B, rbuf,
                       rs, 0);
    panel(k1, k2);
    hipLaunchKernelGGL(k_bgj_swap, gs, dim3(kBlock), 0, s, m, k1, k2, B, perm, rbuf, rs, b1);
    hipLaunchKernelGGL(k_bgj_rfix, dim3(nblk(m), b2, nmat), dim3(kBlock), 0, s, m, k0, k1, k2, B, rbuf, rs, b1);
    update(k0, k2);
    hipLaunchKernelGGL(k_bgj_cols, dim3(nblk((int64_t)m * b1), nmat), dim3(kBlock), 0, s, m, k1, b2, k0, k1, B, rbuf,
                       rs, b1);
    k0 = k2;
  }
  hipLaunchKernelGGL(k_gj_unpermute, gp, dim3(kBlock), 0, s, m, B, perm);
  return hipGetLastError();
}

hipError_t launch_coarse_solve(const LevelView& L, const double* Binv, const double* Mv,
                               const double* e0, const double* e1, const double* b, double* x,
                               double* gbuf, hipStream_t s) {
  const int mm = L.nf * L.NQ + L.nbord;
  if (mm > kMaxCoarse) return hipErrorInvalidValue;
  const TimeEnds te = time_ends(L.NQ, e0, e1);
  if (mm > kCoarseSmall) {
    const unsigned gr = (unsigned)((mm + kBlock / 16 - 1) / (kBlock / 16));
    const unsigned gg = (unsigned)((L.nf * L.NQ + kBlock / 64 - 1) / (kBlock / 64));
    for (int n = 0; n < L.N; ++n) {
      const double* Bn = Binv + (int64_t)(n % L.coarse_slabs) * mm * mm;
      STWR_NQ_SWITCH(L.NQ, {
        hipLaunchKernelGGL(k_coarse_rhs<Q>, dim3(gr), dim3(kBlock), 0, s, L.nf, L.po, L.N, n, L.nbord,
                           L.row_ptr, L.col, Mv, te, b, x, gbuf);
        hipLaunchKernelGGL(k_coarse_gemv<Q>, dim3(gg), dim3(kBlock), 0, s, L.nf, L.N, n, mm, Bn, gbuf, x);
      });
    }
    return hipGetLastError();
  }
  STWR_NQ_SWITCH(L.NQ, hipLaunchKernelGGL(k_coarse_solve<Q>, dim3(1), dim3(kBlock), 0, s, L.nf, L.po,
                                          L.N, L.nbord, L.coarse_slabs, L.row_ptr, L.col, Mv, te, Binv, b, x));
  return hipGetLastError();
}

}  // namespace stwr
