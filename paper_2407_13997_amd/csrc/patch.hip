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
#include <climits>

#include "device.h"

namespace stwr {

namespace {


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

// 16-byte nontemporal load of streamed data (read once per sweep): it does
// not displace the reused residual and output lines from L2
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ inline float4 load_stream(const float* p) {
  const f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(t.x, t.y, t.z, t.w);
}

// Pointers into device (global) memory.  A pointer read from a descriptor in
// memory is generic to the compiler, which then emits flat accesses with a
// 64-bit address per lane; typing it global gives global accesses, as for
// kernel arguments.
#define GLOBAL_AS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL_AS T* gptr(T* p) {
  return (GLOBAL_AS T*)p;
}
__device__ inline float4 load_stream(const GLOBAL_AS float* p) {
  const f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const GLOBAL_AS f32x4*>(p));
  return make_float4(t.x, t.y, t.z, t.w);
}
// 8 bytes (two floats) of a narrow last panel, as a 16-byte panel value
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ inline float4 load_stream2(const GLOBAL_AS float* p) {
  const f32x2 t = __builtin_nontemporal_load(reinterpret_cast<const GLOBAL_AS f32x2*>(p));
  return make_float4(t.x, t.y, 0.0f, 0.0f);
}

// the same for 16 bytes of T (four floats or two doubles), as a vector
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T>
struct NtVec;
template <>
struct NtVec<float> {
  using type = f32x4;
};
template <>
struct NtVec<double> {
  using type = f64x2;
};
template <typename T>
__device__ inline typename NtVec<T>::type load_stream16(const T* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const typename NtVec<T>::type*>(p));
}

// Inverse of one (patch, slab) block by Gauss-Jordan elimination with
// partial pivoting, held in registers: thread t owns rows t + TPB r (r < RPL),
// each a full row of MAXM entries.  After each step the rows rotate left by
// one column, so the active column is always register 0 and every register
// index is static; after m steps position j holds column (j + m) mod MAXM
// (columns past m are zero padding and stay zero).  A step is a pivot search
// among the rows not yet used as pivots (DPP wavefront maximum and ballots,
// plus LDS across wavefronts when TPB > 64), the pivot row scaled by the
// pivot's reciprocal and broadcast through LDS, and the elimination in
// registers.  The rows are never swapped: step k's pivot row p_k stays in
// its thread, so the registers hold (Pi A)^-1 with its row k in physical
// row p_k, where Pi puts row p_k of A at position k; the inverse is A^-1 =
// (Pi A)^-1 Pi, written out row k from physical row p_k and stored column k
// to column p_k of the sweep's layout.  Per element the arithmetic is that
// of the textbook in-place Gauss-Jordan inverse with partial pivoting
// (largest magnitude, ties to the smaller physical row); not moving rows
// saves the swap's register selects and LDS round trip every step.
template <int NQ, typename T, int TPB, int NBMAX = kMaxNb>
struct FactorLds {
  static constexpr int MAXM = NBMAX * NQ;
  static constexpr int NW = TPB / 64;
  // row buffers padded to whole 16-byte vectors
  static constexpr int RV = 16 / sizeof(T), MP = (MAXM + RV - 1) / RV * RV;
  __align__(16) T prow[MP];
  T rv[NW];
  int ri[NW];
  int perm[MAXM];   // perm[k]: pivot row of step k
  int invp[MAXM];   // invp[row]: the step it was the pivot of
  int ofs1[MAXM], ofs2[MAXM];
};

// The block of patch p (its id, not its position) at slab n.  BIG writes
// the inverse in the large-block layout (big_block_size) instead of the
// wavefront panel layout.
template <int NQ, typename T, int TPB, int RPL, int NBMAX = kMaxNb, bool BIG = false>
__device__ __forceinline__ void factor_block(const LevelView& L, const PatchView& P, const int p, const int n,
                                             const double* __restrict__ Jv, T* __restrict__ fac,
                                             int* __restrict__ status, FactorLds<NQ, T, TPB, NBMAX>& S) {
  constexpr int MAXM = NBMAX * NQ;
  constexpr int NW = TPB / 64;
  constexpr int VW = Vec<T>::W;
  constexpr int RV = 16 / sizeof(T), MP = (MAXM + RV - 1) / RV * RV;
  using V16 = typename Vec<T>::type;
  T* prow = S.prow;
  T* rv = S.rv;
  int* ri = S.ri;
  int* perm = S.perm;
  int* ofs1 = S.ofs1;
  int* ofs2 = S.ofs2;
  const int tid = threadIdx.x;
  const int s0 = P.patch_ptr[p];
  const int nb = P.patch_ptr[p + 1] - s0;
  const int m = nb * NQ;
  const int* nzp = P.patch_nz + P.patch_nz_off[p];
  T a[RPL][MAXM];
  // row r of the registers to an LDS row buffer, 16 bytes at a time
  auto put = [&](T* dst, int r) {
#pragma unroll
    for (int j = 0; j < MP; j += RV) {
      V16 v;
      T* e = reinterpret_cast<T*>(&v);
#pragma unroll
      for (int t = 0; t < RV; ++t) e[t] = j + t < MAXM ? a[r][j + t] : (T)0;
      *reinterpret_cast<V16*>(dst + j) = v;
    }
  };
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = tid + TPB * r;
    const int ii = i < m ? i : 0;
    const int* nzr = nzp + (ii / NQ) * nb;
    // the row's CSR positions CK patch DoFs at a time, then their entries:
    // every load unconditional (clamped), the zeros selected afterwards, so
    // a chunk's loads are in flight together instead of one index-then-entry
    // round trip per entry
    constexpr int CK = MAXM > 100 ? 4 : 8;   // fewer loads in flight where the row fills the registers
    const double* jrow = Jv + (int64_t)n * NQ * NQ + (ii % NQ) * NQ;
#pragma unroll
    for (int b0 = 0; b0 < NBMAX; b0 += CK) {
      int kk[CK];
#pragma unroll
      for (int b = 0; b < CK; ++b) kk[b] = b0 + b < NBMAX ? nzr[b0 + b < nb ? b0 + b : 0] : -1;
#pragma unroll
      for (int b = 0; b < CK; ++b) {
#pragma unroll
        for (int e = 0; e < NQ; ++e) {
          const int c = (b0 + b) * NQ + e;
          if (c < MAXM) {
            const bool ok = i < m && c < m && kk[b] >= 0;
            const double v = jrow[(int64_t)(ok ? kk[b] : 0) * L.N * NQ * NQ + e];
            a[r][c] = ok ? (T)v : (T)0;
          }
        }
      }
      // one chunk's loads at a time: hoisting every chunk's loads ahead
      // would need as many registers again as the row itself
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  bool used[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) used[r] = false;
  for (int k = 0; k < m; ++k) {
    // pivot: largest |entry| of column k among the rows not yet used, ties
    // to the smaller row: each wavefront's maximum (DPP), the first of its
    // rows holding it (ballots; register r = 0 holds the wavefront's smaller
    // rows), then the best over the wavefronts through LDS
    T vr[RPL];
    T vmax = (T)-1;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = tid + TPB * r;
      vr[r] = (!used[r] && i < m) ? fabs(a[r][0]) : (T)-1;
      vmax = fmax(vmax, vr[r]);
    }
    T best = wave_max(vmax);
    int bi = m;
#pragma unroll
    for (int r = RPL - 1; r >= 0; --r) {
      const uint64_t hit = __ballot(vr[r] == best);
      if (hit) bi = TPB * r + (tid / 64) * 64 + __ffsll((unsigned long long)hit) - 1;
    }
    if constexpr (NW > 1) {
      if (tid % 64 == 0) { rv[tid / 64] = best; ri[tid / 64] = bi; }
      __syncthreads();
      best = rv[0];
      bi = ri[0];
      for (int w = 1; w < NW; ++w)
        if (rv[w] > best || (rv[w] == best && ri[w] < bi)) { best = rv[w]; bi = ri[w]; }
    }
    int pi = bi;
    if (!(best > (T)0) || !isfinite(best) || pi >= m) {
      if (tid == 0) status[0] = 1;
      pi = pi < m ? pi : 0;   // a failed block: keep going on some row, the status reports it
    }
    if (tid == 0) perm[k] = pi;
    // the owner of row pi scales it by the pivot's reciprocal (the pivot
    // entry becomes 1 / pivot) and publishes it; every row multiplies by its
    // factor (1 off the pivot row), which is cheaper than selecting the
    // owner's values element by element
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const bool own = tid + TPB * r == pi;
      used[r] = used[r] || own;
      const T rp = (T)1 / a[r][0];
      const T sc = own ? rp : (T)1;
      a[r][0] = own ? rp : a[r][0];
#pragma unroll
      for (int j = 1; j < MAXM; ++j) a[r][j] *= sc;
      if (own) put(prow, r);
    }
    __syncthreads();
    // every other row eliminates column k (a zero factor leaves the pivot
    // row and the padding rows as they are)
    T f[RPL];
    bool live[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = tid + TPB * r;
      live[r] = i < m && i != pi;
      f[r] = live[r] ? a[r][0] : (T)0;
    }
    {
      const T p0 = prow[0];
#pragma unroll
      for (int r = 0; r < RPL; ++r)
        if (live[r]) a[r][0] = -f[r] * p0;
    }
    // the pivot row in batches of EB 16-byte reads: a batch's reads are in
    // flight together, so a step waits for the LDS once per batch instead of
    // once per 16 bytes (with one or two wavefronts per SIMD nothing else
    // hides that latency), while the batch's registers stay within the two
    // wavefronts per SIMD the row registers allow (162-row blocks: 10 reads,
    // 222 VGPRs; 2 reads took 5% longer)
    constexpr int EB = MAXM > 100 ? 10 : 8;
#pragma unroll
    for (int j0 = 0; j0 < MP; j0 += RV * EB) {
      V16 v[EB];
#pragma unroll
      for (int b = 0; b < EB; ++b)
        if (j0 + b * RV < MP) v[b] = *reinterpret_cast<const V16*>(prow + j0 + b * RV);
#pragma unroll
      for (int b = 0; b < EB; ++b) {
        const T* pj = reinterpret_cast<const T*>(&v[b]);
#pragma unroll
        for (int t = 0; t < RV; ++t) {
          const int j = j0 + b * RV + t;
          if (j >= 1 && j < MAXM) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) a[r][j] -= f[r] * pj[t];
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const T t0 = a[r][0];
#pragma unroll
      for (int j = 0; j + 1 < MAXM; ++j) a[r][j] = a[r][j + 1];
      a[r][MAXM - 1] = t0;
    }
  }
  // A^-1 = (Pi A)^-1 Pi: stored column k goes to column perm[k], and row k
  // (physical row perm[k]) to row k; record the layout offsets of each
  // stored column's destination (rows < 64 and rows >= 64) and each
  // physical row's output row (rows of a failed block fall back to their own)
  const BlockLayout lay(m, VW);
  __syncthreads();
  int* invp = S.invp;
  for (int i = tid; i < m; i += TPB) invp[i] = i;
  __syncthreads();
  for (int k = tid; k < m; k += TPB) invp[perm[k]] = k;
  for (int c = tid; c < m; c += TPB) {
    const int pos = perm[c];
    if constexpr (BIG) {
      ofs1[c] = (pos / VW) * m * VW + pos % VW;
      ofs2[c] = 0;
    } else {
      ofs1[c] = lay.at(0, pos);
      ofs2[c] = m > 64 ? lay.at(64, pos) : 0;
    }
  }
  // the padding of the layout is zeroed once when the storage is allocated;
  // every entry is written here
  T* out = fac + P.fac_off[p] + (int64_t)n * P.slab_stride;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int ip = tid + TPB * r;
    if (ip < m) {
      const int i = invp[ip];   // the output row this physical row holds
      if constexpr (BIG) {
#pragma unroll
        for (int q = 0; q < MAXM; ++q) {
          const int c = (q + m) % MAXM;
          if (c < m) out[ofs1[c] + i * VW] = a[r][q];
        }
      } else {
        // rows < 64 step VW per row, or the last panel's width wl when it is
        // narrow (its columns start at (P - 1) r1 VW); rows >= 64 step 4 VW
        const int last0 = (lay.P - 1) * lay.r1 * VW;
#pragma unroll
        for (int q = 0; q < MAXM; ++q) {
          const int c = (q + m) % MAXM;
          if (c < m) {
            const int o = i < 64 ? ofs1[c] + i * (ofs1[c] >= last0 ? lay.wl : VW) : ofs2[c] + (i - 64) * 4 * VW;
            out[o] = a[r][q];
          }
        }
      }
    }
  }
}

template <int NQ, typename T, int TPB, int RPL, int NBMAX = kMaxNb, bool BIG = false>
__global__ __launch_bounds__(TPB) void k_patch_factor(LevelView L, PatchView P, int first,
                                                      const double* __restrict__ Jv,
                                                      T* __restrict__ fac, int* __restrict__ status) {
  __shared__ FactorLds<NQ, T, TPB, NBMAX> S;
  const int p = P.order[first + blockIdx.x / P.fac_slabs], n = blockIdx.x % P.fac_slabs;
  factor_block<NQ, T, TPB, RPL, NBMAX, BIG>(L, P, p, n, Jv, fac, status, S);
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

// An empty asm that reads and rewrites the lanes of a loaded vector: the
// load is complete here, and later uses of the registers wait for nothing.
__device__ inline void pin_loaded(float4& v) { asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w)); }
__device__ inline void pin_loaded(double2& v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }

template <typename V, typename T>
__device__ inline T dotv(const V& w, const T* g) {
  if constexpr (sizeof(V) / sizeof(T) == 4) return w.x * g[0] + w.y * g[1] + w.z * g[2] + w.w * g[3];
  else return w.x * g[0] + w.y * g[1];
}

// FP32 sweep, one wavefront per patch (every FP32 block fits one wavefront's
// registers).  The right-hand side stays distributed, one value per lane
// (rows lane and 64 + lane); the lane-per-row part of the product broadcasts
// it with v_readlane into scalar operands, so it needs neither LDS nor
// replicated registers, and only the rows past 64 read it from LDS.
// Software pipeline: the loads of slab n + 1's block are issued as soon as
// slab n's product has consumed its registers, so they are in flight while
// slab n's output is stored and the jump coupling is formed; every load is
// unconditional (clamped addresses), so the wait counts leave them
// outstanding.  The residual is staged 16 / (q+1) slabs of every patch DoF
// at a time (a 128-byte line of FP64 values, or half a line of FP32 values
// when the operator kernel stores it rounded), with one batch of coalesced
// loads issued ahead of a block.  The outputs are FP32 (they are computed in FP32, so nothing
// is lost; the gather widens them), collected in LDS for 64 / (q+1) slabs
// and written DoF by DoF ([patch DoF][slab][node], two whole 128-byte lines
// per DoF and chunk) with nontemporal stores: writes interleaved with the
// block stream cost HBM time far beyond their share of the bytes (1.2% of
// the bytes, 15% of the time when measured against the same kernel storing
// to a few lines that stay in L2), so they are kept few, whole and
// streaming.  The blocks are read once per sweep and are loaded
// nontemporal, so they do not push the residual and output lines out of L2.  The jump coupling works in FP32 from the scalar patch mass
// block: the velocity mass couples equal components only, with the same
// scalar block for both, and the patch velocity DoFs come in (x, y) pairs of
// a node.  FULL = true is the interior patch (nb = 39), whose sizes are all
// compile-time constants; FULL = false handles the smaller boundary patches.
// Panels past a block's last one re-read its last panel: their columns meet
// zeros of the right-hand side, so they add nothing.  Both forms run in one
// launch (interior patches first), so on small meshes the boundary patches
// overlap the interior ones instead of following them.
template <int NQ>
struct SweepF32Lds {
  static constexpr int MAXM = kMaxNb * NQ;
  static constexpr int MAXP = (MAXM + 3) / 4;
  static constexpr int CH = 16 / NQ;           // slabs per 128-byte residual line
  static constexpr int RW = MAXM > 64 ? 128 : 64;
  static constexpr int kMaxNn = kMaxNbu / 2;   // velocity nodes of a patch
  int dofs[kMaxNb];
  float MsT[kMaxNn * kMaxNn];                  // scalar patch mass block, transposed
  float g[MAXP * 4 + 4];
  float ylast[kMaxNbu];
  float mj[kMaxNbu];
  float rch[CH][RW];                           // residual of the current CH slabs
  alignas(16) float ych[4 * CH * MAXM];        // outputs of the current 4 CH slabs, [patch DoF][slab][node]
};

template <int NQ, bool FULL, typename TR = double>
__device__ __forceinline__ void sweep_f32_patch(const LevelView& L, const PatchView& P, const int p,
                                                const float* __restrict__ fac,
                                                const double* __restrict__ Mp, const double e00,
                                                const double e01, const double e10,
                                                const double e11, const TR* __restrict__ r,
                                                float* __restrict__ Y, SweepF32Lds<NQ>& S) {
  constexpr int MAXM = kMaxNb * NQ;
  constexpr int VW = 4;
  constexpr int MAXP = (MAXM + VW - 1) / VW;   // 10 or 20 panels
  constexpr int K2 = (MAXP + 3) / 4;
  constexpr bool kTwo = MAXM > 64;
  constexpr int R1F = MAXM < 64 ? MAXM : 64, R2F = MAXM - R1F;
  constexpr int kLine = 16;                    // residual values of a DoF staged at a time (a 128-byte line of doubles)
  constexpr int CH = kLine / NQ;               // slabs per residual line
  constexpr int RL = (kMaxNb * kLine + 63) / 64;   // residual loads per lane and line
  constexpr int RW = kTwo ? 128 : 64;
  int* dofs = S.dofs;
  float* MsT = S.MsT;
  float* g = S.g;
  float* ylast = S.ylast;
  float* mj = S.mj;
  float (*rch)[RW] = S.rch;
  constexpr int YCH = 4 * CH;                  // slabs per output chunk (two 128-byte lines of FP32 outputs)
  float* ych = S.ych;
  static_assert(YCH * NQ == 64, "an output chunk is two 128-byte lines per DoF");
  constexpr int YL = (kMaxNb * 16 + 63) / 64;  // 16-byte output stores per lane and chunk
  const float e0[2] = {(float)e00, (float)e01}, e1[2] = {(float)e10, (float)e11};
  const int lane = threadIdx.x;
  const GLOBAL_AS int* patch_ptr = gptr(P.patch_ptr);
  const GLOBAL_AS TR* gr = gptr(r);
  const int s0 = patch_ptr[p];
  const int nb = FULL ? kMaxNb : patch_ptr[p + 1] - s0;
  const int nbu = FULL ? kMaxNbu : gptr(P.patch_nbu)[p];
  const int nn = nbu / 2;
  const int m = nb * NQ, N = L.N;
  const BlockLayout lay(m, VW);
  const int PH = FULL ? MAXP : lay.P;
  const int r1 = FULL ? R1F : lay.r1, r2 = FULL ? R2F : lay.r2;
  const int nk2 = FULL ? (R2F > 0 ? K2 : 0) : lay.k2(0);
  for (int i = lane; i < nb; i += 64) dofs[i] = gptr(P.patch_dofs)[s0 + i];
  const GLOBAL_AS double* mp = gptr(Mp) + gptr(P.mp_off)[p];
  for (int e = lane; e < nn * nn; e += 64) {
    const int i = e / nn, j = e % nn;
    MsT[j * nn + i] = (float)mp[2 * i * nbu + 2 * j];
  }
  for (int i = lane; i < kMaxNbu; i += 64) mj[i] = 0.0f;
  for (int i = lane; i < MAXP * VW + 4; i += 64) g[i] = 0.0f;
  __syncthreads();
  const GLOBAL_AS float* Ab = gptr(fac) + gptr(P.fac_off)[p];
  const int64_t SS = P.slab_stride;
  GLOBAL_AS float* yout = gptr(Y) + 2 * gptr(P.y_off)[p];   // FP32 outputs at the byte offset of the FP64 layout,
                                                            // [patch DoF][slab][node]
  // a narrow last panel (m = 2 mod 4): its rows below 64 are two columns
  // wide, 8-byte loads at baseh, and the rows past 64 start right after them
  constexpr bool kHalfF = MAXM % 4 == 2;
  const bool half = FULL && kHalfF;
  const unsigned row1 = lane < r1 ? lane : 0;
  const unsigned base1 = row1 * VW, step1 = r1 * VW;
  const int lastq = PH - 1, lastk = nk2 > 0 ? nk2 - 1 : 0;
  const unsigned baseh = lastq * step1 + row1 * 2;
  const unsigned lane2 = lane < 4 * r2 ? lane : 0;
  const unsigned base2 = (half ? lastq * r1 * VW + r1 * 2 : PH * r1 * VW) + lane2 * VW, step2 = 4 * r2 * VW;
  const int rowA = lane, rowB = lane + 64;
  const bool hasA = rowA < m, hasB = kTwo && rowB < m;
  const int iA = rowA / NQ, iB = rowB / NQ;
  const int quarter = lane & 3;
  const int nq = N * NQ;
  const int nel = nb * kLine;
  float4 a1[MAXP];
  float4 a2[kTwo ? K2 : 1];
  TR rv[RL];
  auto issue = [&](int n) {
    const GLOBAL_AS float* blk = Ab + (int64_t)n * SS;
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
      if constexpr (FULL) {
        if (kHalfF && q == MAXP - 1) a1[q] = load_stream2(blk + baseh);
        else a1[q] = load_stream(blk + base1 + q * step1);
      } else {
        // the smaller blocks have full-width panels
        a1[q] = load_stream(blk + base1 + (q < lastq ? q : lastq) * step1);
      }
    }
    if constexpr (kTwo) {
#pragma unroll
      for (int k = 0; k < K2; ++k) {
        const unsigned kk = FULL ? k : (k < lastk ? k : lastk);
        a2[k] = load_stream(blk + base2 + kk * step2);
      }
    }
  };
  // line of CH slabs from slab n0 (a multiple of CH) of every patch DoF:
  // element id = 16 d + j of the chunk is value j of DoF d's line
  auto stage_issue = [&](int n0) {
#pragma unroll
    for (int i = 0; i < RL; ++i) {
      int id = i * 64 + lane;
      id = id < nel ? id : nel - 1;
      int e = n0 * NQ + (id & (kLine - 1));
      e = e < nq ? e : nq - 1;
      rv[i] = gr[(int64_t)dofs[id >> 4] * nq + e];
    }
  };
  auto stage_store = [&]() {
#pragma unroll
    for (int i = 0; i < RL; ++i) {
      const int id = i * 64 + lane, j = id & (kLine - 1);
      if (id < nel) rch[j / NQ][(id >> 4) * NQ + j % NQ] = (float)rv[i];
    }
  };
  // outputs of slabs n0 .. n0 + ns - 1 (n0 a multiple of YCH), stored DoF
  // by DoF: patch row i holds its N slabs' NQ values contiguously (nq
  // floats from i nq), so a DoF's values of a whole chunk are two 128-byte
  // lines, and the gather reads each DoF's slabs as one coalesced run.  Four
  // values a lane and store (sixteen stores per DoF and chunk); 16-byte
  // stores where the rows are 16-byte aligned (nq a multiple of 4), single
  // values at a ragged chunk end
  auto flush = [&](int n0, int ns) {
    const int run = ns * NQ;
    const bool vec = (nq & 3) == 0;
    // one store at a time: the next slab's block loads are in flight, so
    // every register the flush holds adds to the kernel's peak
#pragma unroll 1
    for (int i = 0; i < YL; ++i) {
      const int id = i * 64 + lane, dd = id >> 4, t0 = 4 * (id & 15);
      if (dd < nb && t0 < run) {
        GLOBAL_AS float* yo = yout + (int64_t)dd * nq + n0 * NQ + t0;
        const float* ys = ych + dd * 64 + t0;
        if (vec && t0 + 3 < run) {
          __builtin_nontemporal_store(*reinterpret_cast<const f32x4*>(ys), reinterpret_cast<GLOBAL_AS f32x4*>(yo));
        } else {
          for (int t = 0; t < 4 && t0 + t < run; ++t) yo[t] = ys[t];
        }
      }
    }
  };
  if (N > 0) {
    stage_issue(0);
    issue(0);
    stage_store();
  }
  for (int n = 0; n < N; ++n) {
    const int s = n % CH;
    float gA = 0.0f, gB = 0.0f;
    if (hasA) gA = rch[s][lane] + ((n > 0 && iA < nbu) ? e0[rowA % NQ] * mj[iA] : 0.0f);
    if (kTwo && hasB) gB = rch[s][RW - 64 + lane] + ((n > 0 && iB < nbu) ? e0[rowB % NQ] * mj[iB] : 0.0f);
    if constexpr (kTwo) {
      g[rowA] = gA;
      if (rowB < MAXP * VW) g[rowB] = gB;
    }
    // rows r < r1: g broadcast lane by lane
    float acc1 = 0.0f;
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int col = 4 * q + c;
        const float gc = col < 64 ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gA), col))
                                  : __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gB), col - 64));
        acc1 += (c == 0 ? a1[q].x : c == 1 ? a1[q].y : c == 2 ? a1[q].z : a1[q].w) * gc;
      }
      // keep each panel's broadcasts next to their use (bounded scalar registers)
      __builtin_amdgcn_sched_barrier(0);
    }
    float acc2 = 0.0f;
    if constexpr (kTwo) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < K2; ++k) {
        const float* gq = g + (quarter + 4 * k) * VW;
        acc2 += a2[k].x * gq[0] + a2[k].y * gq[1] + a2[k].z * gq[2] + a2[k].w * gq[3];
      }
      acc2 += __shfl_xor(acc2, 1);
      acc2 += __shfl_xor(acc2, 2);
    }
    // the block registers are free: start the next slab's loads (the last
    // slab re-reads its own block, an L2 hit, so the loads stay unconditional).
    // The empty asm pins the products here: without it the compiler sinks
    // them to their stores, past the loads, and needs a second register set.
    asm volatile("" : "+v"(acc1), "+v"(acc2) : : "memory");
    __builtin_amdgcn_sched_barrier(0);
    const bool line = n + 1 < N && (n + 1) % CH == 0;
    if (line) stage_issue(n + 1);
    issue(n + 1 < N ? n + 1 : n);
    __builtin_amdgcn_sched_barrier(0);
    const int sy = n % YCH;
    // slab end value of each DoF, sum_b e1[b] y(row of node b): the nodes of
    // a DoF sit in adjacent lanes (rows < 64) or adjacent quads (rows >= 64)
    float v1 = e1[lane % NQ] * acc1;
    if constexpr (NQ == 2) v1 += __shfl_xor(v1, 1);
    if (lane < r1) {
      ych[(lane / NQ) * 64 + sy * NQ + lane % NQ] = acc1;
      if (lane % NQ == NQ - 1) ylast[lane / NQ] = v1;
    }
    if constexpr (kTwo) {
      const int row = 64 + lane / 4;
      float v2 = e1[row % NQ] * acc2;
      if constexpr (NQ == 2) v2 += __shfl_xor(v2, 4);
      if (lane < 4 * r2 && quarter == 0) {
        ych[(row / NQ) * 64 + sy * NQ + row % NQ] = acc2;
        if (row % NQ == NQ - 1) ylast[row / NQ] = v2;
      }
    }
    __syncthreads();
    // jump coupling of the next slab: mj = M_v y_n(end of slab)
    if (lane < nbu) {
      const int a = lane >> 1, c = lane & 1;
      float acc = 0.0f;
#pragma unroll 4
      for (int k = 0; k < nn; ++k) acc += MsT[k * nn + a] * ylast[2 * k + c];
      mj[lane] = acc;
    }
    if (sy == YCH - 1 || n == N - 1) flush(n - sy, sy + 1);
    if (line) stage_store();
    __syncthreads();
  }
}

// TR: the residual's type.  FP32 residuals (rounded by the operator kernel
// that writes them) give the same outputs as FP64 ones rounded here, and
// halve the residual's bytes on both sides.
template <int NQ, typename TR>
__global__ __launch_bounds__(64) void k_patch_sweep_f32(LevelView L, PatchView P,
                                                       const float* __restrict__ fac,
                                                       const double* __restrict__ Mp, double e00,
                                                       double e01, double e10, double e11,
                                                       const TR* __restrict__ r,
                                                       float* __restrict__ Y) {
  __shared__ SweepF32Lds<NQ> S;
  const int p = P.order[blockIdx.x];
  if ((int)blockIdx.x < P.n_full) sweep_f32_patch<NQ, true, TR>(L, P, p, fac, Mp, e00, e01, e10, e11, r, Y, S);
  else sweep_f32_patch<NQ, false, TR>(L, P, p, fac, Mp, e00, e01, e10, e11, r, Y, S);
}

// Persistent FP32 sweep over the patches of many (problem, level) jobs with
// NQ temporal nodes: workgroups take tiles of patches from a counter in list
// order and sweep each patch as k_patch_sweep_f32 does; the last workgroup to
// finish resets the counter pair.  The list holds the tiles of interior
// (full-size) patches first, then the others, each part sorted by decreasing
// work; the two parts run in two loops one after the other, so the
// compile-time interior form and the general form never share live
// registers.  One launch per node count, for the same reason.
template <int NQ>
__global__ __launch_bounds__(64) void k_patch_sweep_f32_batch(const SweepJob* __restrict__ jobs,
                                                             const SweepTile* __restrict__ tiles,
                                                             int n_full_tiles, int n_tiles,
                                                             int* __restrict__ ctr) {
  __shared__ SweepF32Lds<NQ> S;
  __shared__ int next;
  auto grab = [&]() {
    if (threadIdx.x == 0) next = atomicAdd(&ctr[0], 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    return t;
  };
  int t = grab();
  for (; t < n_full_tiles; t = grab()) {
    const SweepTile tl = tiles[t];
    const SweepJob& J = jobs[tl.job];
    for (int pos = tl.first; pos < tl.first + tl.count; ++pos) {
      sweep_f32_patch<NQ, true>(J.L, J.P, gptr(J.P.order)[pos], J.fac, J.Mp, J.e00, J.e01, J.e10, J.e11, J.r,
                                J.Y, S);
      __syncthreads();
    }
  }
  for (; t < n_tiles; t = grab()) {
    const SweepTile tl = tiles[t];
    const SweepJob& J = jobs[tl.job];
    for (int pos = tl.first; pos < tl.first + tl.count; ++pos) {
      sweep_f32_patch<NQ, false>(J.L, J.P, gptr(J.P.order)[pos], J.fac, J.Mp, J.e00, J.e01, J.e10, J.e11, J.r,
                                 J.Y, S);
      __syncthreads();
    }
  }
  if (threadIdx.x == 0 && atomicAdd(&ctr[1], 1) == (int)gridDim.x - 1) {
    atomicExch(&ctr[0], 0);
    atomicExch(&ctr[1], 0);
  }
}

// Persistent FP32 factorization of the blocks of at most 64 rows of many
// jobs (one class per launch: NQ = 1 or 2), as k_patch_factor.
template <int NQ>
__global__ __launch_bounds__(64) void k_patch_factor_f32_batch(const FactorJob* __restrict__ jobs,
                                                              const FactorTile* __restrict__ tiles,
                                                              int n_tiles, int* __restrict__ ctr) {
  __shared__ FactorLds<NQ, float, 64> S;
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
      factor_block<NQ, float, 64, 1>(J.L, J.P, p, n, J.Jv, J.fac, J.status, S);
      __syncthreads();
    }
  }
  if (threadIdx.x == 0 && atomicAdd(&ctr[1], 1) == (int)gridDim.x - 1) {
    atomicExch(&ctr[0], 0);
    atomicExch(&ctr[1], 0);
  }
}

// One workgroup per patch, WAVES wavefronts, each owning at most
// kPanelsPerWave column panels of every slab block (see BlockLayout).  The
// slabs are walked in order (forward block substitution).  Software pipeline:
// while slab n is formed and multiplied, the block of slab n + 1 is already in
// flight into a second register set (every load is unconditional, with
// clamped addresses, so the wait counts leave the prefetch outstanding).  INV
// (one block shared by every slab, slab_stride 0) keeps the block in
// registers for the whole sweep and drops the second set.  The residual of
// kRGroup slabs at a time is loaded a whole group ahead into registers and
// parked in LDS (each thread reads back only its own row), so the slab loop
// waits on memory once per group, not once per slab.  The jump coupling
// mj = M_v (e1 . y_{n-1}) is formed at the end of the previous slab: first the
// slab-end value of each DoF, then one row of M_v per thread.
//
// Time chunks (cyclic reduction in time): blockIdx.y + ca.first is the chunk
// c, covering slabs [c len, min(N, (c + 1) len)).  The chunk's sweep starts
// from the incoming slab-end values w_in of the previous chunk (none: zero)
// and may leave its own final slab-end values in w_end; outputs are written
// for chunks c <= y_max.  One chunk of length N is the plain sweep.
constexpr int kRGroup = 4;

template <int NQ, typename T, int WAVES, bool INV, int NBMAX = kMaxNb, int NBUMAX = kMaxNbu>
__global__ __launch_bounds__(64 * WAVES) void k_patch_sweep(LevelView L, PatchView P,
                                                            const T* __restrict__ fac,
                                                            const double* __restrict__ Mp,
                                                            TimeEnds te, const double* __restrict__ r,
                                                            double* __restrict__ Y, ChunkArgs ca) {
  constexpr int MAXM = NBMAX * NQ;
  constexpr int VW = Vec<T>::W;
  constexpr int MAXP = (MAXM + VW - 1) / VW;
  constexpr int PW = panels_per_wave(VW);
  // panels a wavefront can hold for blocks up to MAXM (the loops and block
  // registers need no more than the block has)
  constexpr int PWU = MAXP < PW ? MAXP : PW;
  constexpr int K2 = (PWU + 3) / 4;
  constexpr bool kTwo = MAXM > 64;
  // one wavefront and at most 64 rows: row i's product ends on lane i
  constexpr bool kLane = WAVES == 1 && !kTwo;
  // one wavefront and at most two temporal nodes: the slab-end values and the
  // jump coupling stay in registers (DPP pair sums and v_readlane broadcasts)
  constexpr bool kFast = kLane && NQ <= 2;
  constexpr int G = kRGroup;
  static_assert(MAXM <= 64 * WAVES && NBUMAX <= 64, "a thread per row and per velocity DoF");
  static_assert(!kLane || MAXP <= PW, "one wavefront holds every panel");
  using V = typename Vec<T>::type;
  __shared__ int dofs[NBMAX];
  __shared__ double MsT[NBUMAX * NBUMAX];   // MsT[j nbu + i] = M_v(i, j)
  __shared__ T g[WAVES * PW * VW];
  __shared__ double part[kLane ? 1 : WAVES][kLane ? 1 : MAXM];
  __shared__ double ys[MAXM];
  __shared__ double yend[NBUMAX];
  __shared__ double mj[NBUMAX];
  __shared__ double rs[G][64 * WAVES];
  const double* e1 = te.e1;
  const int p = blockIdx.x, tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  const int s0 = P.patch_ptr[p];
  const int nb = P.patch_ptr[p + 1] - s0, nbu = P.patch_nbu[p];
  const int m = nb * NQ, N = L.N;
  const int chunk = ca.first + (int)blockIdx.y;
  const int n0 = chunk * ca.len, n1 = n0 + ca.len < N ? n0 + ca.len : N;
  if (n0 >= N) return;   // uniform over the workgroup
  const bool write_y = chunk <= ca.y_max;
  const BlockLayout lay(m, VW);
  const int PH = lay.panels(w), r1 = lay.r1, r2 = lay.r2;
  for (int i = tid; i < nb; i += 64 * WAVES) dofs[i] = P.patch_dofs[s0 + i];
  const double* mp = Mp + P.mp_off[p];
  for (int e = tid; e < nbu * nbu; e += 64 * WAVES) MsT[(e % nbu) * nbu + e / nbu] = mp[e];
  for (int i = tid; i < WAVES * PW * VW; i += 64 * WAVES) g[i] = (T)0;
  __syncthreads();
  // coupling into the chunk's first slab: M_v times the incoming end values
  for (int i = tid; i < NBUMAX; i += 64 * WAVES) {
    double acc = 0.0;
    if (ca.w_in && n0 > 0 && i < nbu) {
      const double* wi = ca.w_in + ((int64_t)p * ca.n_chunks + chunk) * NBUMAX;
      for (int j = 0; j < nbu; ++j) acc += MsT[j * nbu + i] * wi[j];
    }
    mj[i] = acc;
  }
  const int64_t S = P.slab_stride;
  const T* Ab = fac + P.fac_off[p];
  double* yout = Y + P.y_off[p];
  // this lane's load offsets inside a block (clamped to valid elements)
  const int wbase = lay.offset(w);
  const int row1 = lane < r1 ? lane : 0;
  const int off2 = wbase + lay.part1(w);
  // FP32 blocks with a narrow last panel: 8-byte loads of its rows below 64
  const bool halfw = lay.half() && w == lay.waves - 1;
  const int baseh = wbase + (PH - 1) * r1 * VW + row1 * 2;
  const int lane2 = lane < 4 * r2 ? lane : 0;
  // element offsets: region 1 = base1 + q * step1 (q < PH), region 2 = base2 + k * step2
  const int base1 = wbase + row1 * VW, step1 = r1 * VW;
  const int base2 = off2 + lane2 * VW, step2 = 4 * r2 * VW, nk2 = lay.k2(w);
#define O1(q) ((q) < PH ? base1 + (q) * step1 : 0)
#define O2(k) ((kTwo && (k) < nk2) ? base2 + (k) * step2 : 0)
  auto ld1 = [&](const T* blk, int q) -> V {
    if constexpr (sizeof(T) == 4) {
      if (halfw && q == PH - 1) {
        const float2 t = *reinterpret_cast<const float2*>(blk + baseh);
        return make_float4(t.x, t.y, 0.0f, 0.0f);
      }
    }
    return *reinterpret_cast<const V*>(blk + O1(q));
  };
  // the row whose right-hand side this thread forms (threads past the block
  // read row 0's residual and discard it)
  const bool hasRow = tid < m;
  const int64_t rbase = hasRow ? (int64_t)dofs[tid / NQ] * N * NQ + tid % NQ : 0;
  const int ia = tid / NQ, aa = tid % NQ;
  double e0a = te.e0[aa], e1a = te.e1[aa];
  V cur1[PWU], cur2[K2];
  V nxt1[INV ? 1 : PWU], nxt2[INV ? 1 : K2];
  {
    const T* blk0 = Ab + (int64_t)n0 * S;
#pragma unroll
    for (int q = 0; q < PWU; ++q) cur1[q] = ld1(blk0, q);
    if constexpr (kTwo) {
#pragma unroll
      for (int k = 0; k < K2; ++k) cur2[k] = *reinterpret_cast<const V*>(blk0 + O2(k));
    }
  }
  // residual of slabs [na, na + G), clamped to the chunk's last slab
  double rn[G];
  auto issue_r = [&](int na) {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int n = na + j < n1 ? na + j : n1 - 1;
      rn[j] = r[rbase + (int64_t)n * NQ];
    }
  };
  // every thread parks its registers (rows past the block too): the waits
  // for these loads then also cover the block loads issued before them
  auto park_r = [&]() {
#pragma unroll
    for (int j = 0; j < G; ++j) rs[j][tid] = rn[j];
  };
  issue_r(n0);
  park_r();
  // the block registers and e0a count as written here (an empty asm takes
  // them in and out), so the slab loop waits on memory only for the residual
  // groups and, without INV, for the next block
  asm volatile("" : "+v"(e0a), "+v"(e1a));
#pragma unroll
  for (int q = 0; q < PWU; ++q) pin_loaded(cur1[q]);
  if constexpr (kTwo) {
#pragma unroll
    for (int k = 0; k < K2; ++k) pin_loaded(cur2[k]);
  }
  const int quarter = lane & 3;
  __syncthreads();
  // kFast: this lane's DoF's coupling (mjr) and slab-end value (yendr)
  double mjr = (kFast && ia < nbu) ? mj[ia] : 0.0, yendr = 0.0;
  const int iac = ia < nbu ? ia : 0;
  for (int n = n0; n < n1; ++n) {
    const int jr = (n - n0) % G;
    // a group's first slab starts the loads of the next group (uniform)
    if (jr == 0 && n + G < n1) issue_r(n + G);
    if constexpr (!INV) {
      const T* nblk = Ab + (int64_t)(n + 1 < n1 ? n + 1 : n) * S;
#pragma unroll
      for (int q = 0; q < PWU; ++q) nxt1[q] = ld1(nblk, q);
      if constexpr (kTwo) {
#pragma unroll
        for (int k = 0; k < K2; ++k) nxt2[k] = *reinterpret_cast<const V*>(nblk + O2(k));
      }
    }
    if (hasRow) {
      double gv = rs[jr][tid];
      if (n > 0 && ia < nbu) gv += e0a * (kFast ? mjr : mj[ia]);
      g[tid] = (T)gv;
    }
    __syncthreads();
    // this wavefront's share of y = A_n^{-1} g
    const T* gw = g + w * PW * VW;
    T acc1 = (T)0;
#pragma unroll
    for (int q = 0; q < PWU; ++q) {
      const T d = dotv<V, T>(cur1[q], gw + q * VW);
      acc1 += q < PH ? d : (T)0;
    }
    double y = 0.0;
    if constexpr (kLane) {
      y = (double)acc1;
    } else {
      if (lane < r1) part[w][lane] = (double)acc1;
      if constexpr (kTwo) {
        T acc2 = (T)0;
#pragma unroll
        for (int k = 0; k < K2; ++k) {
          const int ql = quarter + 4 * k;
          const T d = dotv<V, T>(cur2[k], gw + (ql < PWU ? ql : 0) * VW);
          acc2 += ql < PH ? d : (T)0;
        }
        acc2 += __shfl_xor(acc2, 1);
        acc2 += __shfl_xor(acc2, 2);
        if (lane < 4 * r2 && quarter == 0) part[w][64 + lane / 4] = (double)acc2;
      }
      __syncthreads();
      if (hasRow) {
#pragma unroll
        for (int v = 0; v < WAVES; ++v) y += v < lay.waves ? part[v][tid] : 0.0;
      }
    }
    if constexpr (kFast) {
      // a plain store: the one-wavefront patches (the heat equation) write little,
      // and the gather finds it in cache (a nontemporal store was slower)
      if (hasRow && write_y) yout[(int64_t)n * m + tid] = y;
      // slab-end value of the lane's DoF: its NQ rows sit in adjacent lanes
      double ve = e1a * y;
      if constexpr (NQ == 2) ve += dpp_move<0xB1>(ve);   // quad_perm [1,0,3,2]
      yendr = ve;
      // the next group's residual, loaded since this group's first slab (uniform)
      if (jr == G - 1 && n + 1 < n1) park_r();
      // coupling of the next slab, mj(ia) = sum_k M_v(ia, k) (slab-end value
      // of DoF k, from lane k NQ), formed by every lane of the DoF
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
      for (int k = 0; k < NBUMAX; ++k) {
        if (k < nbu) {   // uniform
          const double t = MsT[k * nbu + iac] * read_lane(ve, k * NQ);
          if (k % 4 == 0) a0 += t;
          else if (k % 4 == 1) a1 += t;
          else if (k % 4 == 2) a2 += t;
          else a3 += t;
        }
      }
      mjr = (a0 + a1) + (a2 + a3);
      if constexpr (!INV) {
#pragma unroll
        for (int q = 0; q < PWU; ++q) cur1[q] = nxt1[q];
      }
      continue;
    }
    if (hasRow) {
      ys[tid] = y;
      if (write_y) __builtin_nontemporal_store(y, yout + (int64_t)n * m + tid);
    }
    __syncthreads();
    if (tid < nbu) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < NQ; ++b) v += e1[b] * ys[tid * NQ + b];
      yend[tid] = v;
    }
    // the next group's residual, loaded since this group's first slab (uniform)
    if (jr == G - 1 && n + 1 < n1) park_r();
    __syncthreads();
    if (tid < nbu) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int k = 0;
      for (; k + 4 <= nbu; k += 4) {
        a0 += MsT[k * nbu + tid] * yend[k];
        a1 += MsT[(k + 1) * nbu + tid] * yend[k + 1];
        a2 += MsT[(k + 2) * nbu + tid] * yend[k + 2];
        a3 += MsT[(k + 3) * nbu + tid] * yend[k + 3];
      }
      for (; k < nbu; ++k) a0 += MsT[k * nbu + tid] * yend[k];
      mj[tid] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    if constexpr (!INV) {
#pragma unroll
      for (int q = 0; q < PWU; ++q) cur1[q] = nxt1[q];
      if constexpr (kTwo) {
#pragma unroll
        for (int k = 0; k < K2; ++k) cur2[k] = nxt2[k];
      }
    }
  }
  // the chunk's final slab-end values (yend, or with kFast yendr in lane
  // d NQ, holds its last slab's)
  if constexpr (kFast) {
    if (ca.w_end && aa == 0 && ia < nbu) ca.w_end[((int64_t)p * ca.n_chunks + chunk) * NBUMAX + ia] = yendr;
  } else {
    if (ca.w_end && tid < nbu) ca.w_end[((int64_t)p * ca.n_chunks + chunk) * NBUMAX + tid] = yend[tid];
  }
#undef O1
#undef O2
}

// Transfer of slab-end values across a time chunk: with
// K_n = E1 A_n^{-1} E0 (K[i][k] = sum_ab e1[b] A_n^{-1}(i q1 + b, k q1 + a) e0[a])
// the end values obey w_n = K_n (M_v w_{n-1}) + (E1 A_n^{-1} r_n), so a chunk
// maps its incoming values by T_c = K_{n1-1} M_v ... K_{n0} M_v.  One
// workgroup per (patch, chunk); T_c in FP64, nbu x nbu in a slot of NBUMAX^2.
template <int NQ, typename T, int NBUMAX>
__global__ __launch_bounds__(256) void k_patch_chunk_transfer(LevelView L, PatchView P,
                                                              const T* __restrict__ fac,
                                                              const double* __restrict__ Mp,
                                                              TimeEnds te, ChunkArgs ca,
                                                              double* __restrict__ Tc) {
  __shared__ double Ms[NBUMAX * NBUMAX], Tm[NBUMAX * NBUMAX], Q[NBUMAX * NBUMAX], K[NBUMAX * NBUMAX];
  constexpr int VW = Vec<T>::W;
  const int p = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const int nb = P.patch_ptr[p + 1] - P.patch_ptr[p], nbu = P.patch_nbu[p];
  const int m = nb * NQ, N = L.N;
  const int n0 = c * ca.len, n1 = n0 + ca.len < N ? n0 + ca.len : N;
  const BlockLayout lay(m, VW);
  const double* mp = Mp + P.mp_off[p];
  const int nn = nbu * nbu;
  for (int e = tid; e < nn; e += 256) {
    Ms[e] = mp[e];
    Tm[e] = (e / nbu == e % nbu) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int n = n0; n < n1; ++n) {
    const T* blk = fac + P.fac_off[p] + (int64_t)n * P.slab_stride;
    for (int e = tid; e < nn; e += 256) {
      const int i = e / nbu, j = e % nbu;
      double q = 0.0, k = 0.0;
      for (int t = 0; t < nbu; ++t) q += Ms[i * nbu + t] * Tm[t * nbu + j];
      for (int b = 0; b < NQ; ++b)
        for (int a = 0; a < NQ; ++a) k += te.e1[b] * (double)blk[lay.at(i * NQ + b, j * NQ + a)] * te.e0[a];
      Q[e] = q;
      K[e] = k;
    }
    __syncthreads();
    for (int e = tid; e < nn; e += 256) {
      const int i = e / nbu, j = e % nbu;
      double v = 0.0;
      for (int t = 0; t < nbu; ++t) v += K[i * nbu + t] * Q[t * nbu + j];
      Tm[e] = v;
    }
    __syncthreads();
  }
  double* out = Tc + ((int64_t)p * ca.n_chunks + c) * NBUMAX * NBUMAX;
  for (int e = tid; e < nn; e += 256) out[e] = Tm[e];
}

// Incoming end values of every chunk: w_in(0) = 0 and
// w_in(c) = w_end0(c-1) + T_{c-1} w_in(c-1), with w_end0 the chunk ends of
// the sweep from zero incoming values.  One wavefront per patch.
template <int NBUMAX>
__global__ __launch_bounds__(64) void k_patch_chunk_interface(PatchView P, ChunkArgs ca,
                                                              const double* __restrict__ Tc,
                                                              const double* __restrict__ w_end0,
                                                              double* __restrict__ w_in) {
  __shared__ double wv[NBUMAX];
  const int p = blockIdx.x, tid = threadIdx.x, nbu = P.patch_nbu[p];
  if (tid < NBUMAX) wv[tid] = 0.0;
  __syncthreads();
  for (int c = 1; c < ca.n_chunks; ++c) {
    double v = 0.0;
    if (tid < nbu) {
      const double* t = Tc + ((int64_t)p * ca.n_chunks + c - 1) * NBUMAX * NBUMAX + tid * nbu;
      v = w_end0[((int64_t)p * ca.n_chunks + c - 1) * NBUMAX + tid];
      for (int j = 0; j < nbu; ++j) v += t[j] * wv[j];
    }
    __syncthreads();
    if (tid < nbu) {
      wv[tid] = v;
      w_in[((int64_t)p * ca.n_chunks + c) * NBUMAX + tid] = v;
    }
    __syncthreads();
  }
}

// ---- large patch blocks (Taylor-Hood P3-P2) ------------------------------------------
// Dense identity-padded FP64 copies of the slab blocks A_{v,n} = R_v J_n R_v^T
// (eq. waveform_patch_solve), one workgroup per block.
template <int NQ>
__global__ __launch_bounds__(256) void k_patch_extract_dense(LevelView L, PatchView P,
                                                             const double* __restrict__ Jv, int b0, int mmax,
                                                             double* __restrict__ B) {
  const int b = b0 + blockIdx.x;
  const int p = P.order[b / P.fac_slabs], n = b % P.fac_slabs;
  const int s0 = P.patch_ptr[p], nb = P.patch_ptr[p + 1] - s0, m = nb * NQ;
  const int* nzp = P.patch_nz + P.patch_nz_off[p];
  double* out = B + (int64_t)blockIdx.x * mmax * mmax;
  for (int e = threadIdx.x; e < mmax * mmax; e += 256) {
    const int i = e / mmax, j = e % mmax;
    double v = i == j ? 1.0 : 0.0;
    if (i < m && j < m) {
      const int k = nzp[(i / NQ) * nb + j / NQ];
      v = k >= 0 ? Jv[(((int64_t)k * L.N + n) * NQ + i % NQ) * NQ + j % NQ] : 0.0;
    }
    out[e] = v;
  }
}

// The inverses of k_patch_extract_dense's blocks (their leading m x m parts)
// into the large-block layout at precision T.
template <int NQ, typename T>
__global__ __launch_bounds__(256) void k_patch_store_big(PatchView P, const double* __restrict__ B, int b0,
                                                         int mmax, T* __restrict__ fac) {
  constexpr int VW = Vec<T>::W;
  const int b = b0 + blockIdx.x;
  const int p = P.order[b / P.fac_slabs], n = b % P.fac_slabs;
  const int m = (P.patch_ptr[p + 1] - P.patch_ptr[p]) * NQ;
  const double* in = B + (int64_t)blockIdx.x * mmax * mmax;
  T* out = fac + P.fac_off[p] + (int64_t)n * P.slab_stride;
  const int size = big_block_size(m, VW);
  for (int e = threadIdx.x; e < size; e += 256) {
    const int q = e / (m * VW), rem = e % (m * VW), r = rem / VW, c = q * VW + rem % VW;
    out[e] = c < m ? (T)in[(int64_t)r * mmax + c] : (T)0;
  }
}

// Sweep of the large blocks (m = (q+1) nb up to 162): one workgroup of WAVES
// wavefronts per patch, thread r owning row r; per slab the right-hand side
// (residual of the patch DoFs plus the jump coupling e0 (x) M_v y_{n-1}(end))
// goes to LDS, each row's product streams its 16-byte panel vectors (a
// wavefront's loads of a panel are one contiguous segment), the result is
// written to the patch's FP64 outputs, and the slab-end values and the next
// coupling are formed in LDS.  Arithmetic in T (the factor precision).
template <int NQ, typename T, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_patch_sweep_big(LevelView L, PatchView P,
                                                                const T* __restrict__ fac,
                                                                const double* __restrict__ Mp, TimeEnds te,
                                                                const double* __restrict__ r,
                                                                double* __restrict__ Y) {
  constexpr int MAXM = kThMaxNb * NQ;
  constexpr int VW = Vec<T>::W;
  constexpr int MAXP = (MAXM + VW - 1) / VW;
  constexpr int NN = kThMaxNbu / 2;
  static_assert(64 * WAVES >= MAXP * VW, "one thread per padded row");
  __shared__ int dofs[kThMaxNb];
  __shared__ T MsT[NN * NN];
  __shared__ T g[MAXP * VW];
  __shared__ T yv[MAXM];
  __shared__ T ylast[kThMaxNbu], mj[kThMaxNbu];
  const int p = P.order[blockIdx.x];
  const int row = threadIdx.x;
  const int s0 = P.patch_ptr[p], nb = P.patch_ptr[p + 1] - s0, nbu = P.patch_nbu[p], nn = nbu / 2;
  const int m = nb * NQ, PH = (m + VW - 1) / VW, N = L.N;
  for (int i = row; i < nb; i += 64 * WAVES) dofs[i] = P.patch_dofs[s0 + i];
  const double* mp = Mp + P.mp_off[p];
  for (int e = row; e < nn * nn; e += 64 * WAVES) {
    const int i = e / nn, j = e % nn;
    MsT[j * nn + i] = (T)mp[2 * i * nbu + 2 * j];
  }
  for (int i = row; i < kThMaxNbu; i += 64 * WAVES) mj[i] = (T)0;
  __syncthreads();
  const T* A = fac + P.fac_off[p];
  double* yo = Y + P.y_off[p];
  const bool has = row < m;
  const int idof = row / NQ, a = row % NQ;
  const int64_t nq = (int64_t)N * NQ;
  for (int n = 0; n < N; ++n) {
    if (row < PH * VW) {
      T gv = (T)0;
      if (has) {
        gv = (T)r[(int64_t)dofs[idof] * nq + (int64_t)n * NQ + a];
        if (n > 0 && idof < nbu) gv += (T)te.e0[a] * mj[idof];
      }
      g[row] = gv;
    }
    __syncthreads();
    T acc = (T)0;
    if (has) {
      const T* blk = A + (int64_t)n * P.slab_stride + row * VW;
#pragma unroll 8
      for (int q = 0; q < PH; ++q) {
        // nontemporal: the blocks stream once per sweep, and keeping them out
        // of L2 keeps the residual lines every slab of the patch reads there
        const auto v = load_stream16(blk + (int64_t)q * m * VW);
#pragma unroll
        for (int c = 0; c < VW; ++c) acc += v[c] * g[q * VW + c];
      }
      __builtin_nontemporal_store((double)acc, yo + (int64_t)n * m + row);   // streaming output
      yv[row] = acc;
    }
    __syncthreads();
    if (row < nbu) {
      T v = (T)0;
#pragma unroll
      for (int b = 0; b < NQ; ++b) v += (T)te.e1[b] * yv[row * NQ + b];
      ylast[row] = v;
    }
    __syncthreads();
    if (row < nbu) {
      const int a2 = row >> 1, c = row & 1;
      T v = (T)0;
      for (int k = 0; k < nn; ++k) v += MsT[k * nn + a2] * ylast[2 * k + c];
      mj[row] = v;
    }
    __syncthreads();
  }
}

// Y: FP64 patch outputs at y_off, [slab][patch DoF][node], or FP32 ones at
// twice y_off (same bytes), [patch DoF][slab][node] (the FP32 sweep's layout)
template <int NQ, typename TY>
__global__ __launch_bounds__(256) void k_patch_gather(int nf, int N, PatchView P,
                                                      const TY* __restrict__ Y, int mode,
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
    const TY* yp = sizeof(TY) == 4 ? Y + 2 * P.y_off[p] + ((int64_t)(s - s0) * N + n) * NQ
                                   : Y + P.y_off[p] + (int64_t)n * m + (s - s0) * NQ;
    for (int a = 0; a < NQ; ++a) acc[a] += (double)yp[a];
  }
  const int64_t o = t * NQ;
  if (mode == 0) {
    for (int a = 0; a < NQ; ++a) z[o + a] = acc[a];
  } else {
    for (int a = 0; a < NQ; ++a) {
      const double dd = (c1 == 0.0 ? 0.0 : c1 * d[o + a]) + c2 * acc[a];
      if (mode == 1) d[o + a] = dd;   // mode 2: a sequence's last step, d is not read again
      x[o + a] += dd;
    }
  }
}

// The same gather over whole DoFs: a workgroup takes R = 256 / N DoFs and
// every slab of each (thread r N + n).  The slot -> patch -> output offset
// chain of the workgroup's patch slots is resolved once per slot into LDS
// (when the slots fit), so each (DoF, slab) thread only reads the outputs.
constexpr int kGatherStage = 1024;

template <int NQ, typename TY>
__global__ __launch_bounds__(256) void k_patch_gather_rows(int nf, int N, PatchView P,
                                                           const TY* __restrict__ Y, int mode,
                                                           double c1, double c2, double* __restrict__ z,
                                                           double* __restrict__ d, double* __restrict__ x) {
  __shared__ int64_t s_base[kGatherStage];
  __shared__ int s_m[kGatherStage];
  // FP32 outputs are [patch DoF][slab][node] (a DoF's slabs adjacent), FP64
  // ones [slab][patch DoF][node]: the slab stride is NQ or the patch's rows
  constexpr bool kDofMajor = sizeof(TY) == 4;
  constexpr int YS = kDofMajor ? 2 : 1;
  const int R = 256 / N, tid = threadIdx.x;
  const int i0 = blockIdx.x * R, i1 = i0 + R < nf ? i0 + R : nf;
  const int k0 = P.dof_ptr[i0], nk = P.dof_ptr[i1] - k0;
  const bool staged = nk <= kGatherStage;   // uniform over the workgroup
  // output offset of slot k (its value of slab 0) and its slab stride
  auto slot = [&](int k, int64_t& base, int& m) {
    const int sl = P.dof_slot[k];
    const int p = P.slot_patch[sl];
    const int s0 = P.patch_ptr[p];
    m = kDofMajor ? NQ : (P.patch_ptr[p + 1] - s0) * NQ;
    base = YS * P.y_off[p] + (int64_t)(sl - s0) * (kDofMajor ? N * NQ : NQ);
  };
  if (staged) {
    for (int e = tid; e < nk; e += 256) slot(k0 + e, s_base[e], s_m[e]);
  }
  __syncthreads();
  const int r = tid / N, n = tid % N, dof = i0 + r;
  if (r >= R || dof >= nf) return;
  double acc[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) acc[a] = 0.0;
  const int ka = P.dof_ptr[dof], kb = P.dof_ptr[dof + 1];
  if (staged) {
    for (int k = ka - k0; k < kb - k0; ++k) {
      const TY* yp = Y + s_base[k] + (int64_t)n * s_m[k];
#pragma unroll
      for (int a = 0; a < NQ; ++a) acc[a] += (double)yp[a];
    }
  } else {
    for (int k = ka; k < kb; ++k) {
      int64_t base;
      int m;
      slot(k, base, m);
      const TY* yp = Y + base + (int64_t)n * m;
#pragma unroll
      for (int a = 0; a < NQ; ++a) acc[a] += (double)yp[a];
    }
  }
  const int64_t o = ((int64_t)dof * N + n) * NQ;
  if (mode == 0) {
#pragma unroll
    for (int a = 0; a < NQ; ++a) z[o + a] = acc[a];
  } else {
    // a thread's NQ values of x (and d) are loaded together, then stored
    // together, so that they move as one 16-byte vector where x and d are
    // 16-byte aligned (o is even); a caller's vector of another alignment
    // takes the value-by-value path
    double xv[NQ], dv[NQ], dd[NQ];
    bool v16 = false;
    if constexpr (NQ == 2) {
      v16 = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(d)) & 15) == 0;
      if (v16) {
        const double2 t = *reinterpret_cast<const double2*>(x + o);
        xv[0] = t.x;
        xv[1] = t.y;
        if (c1 != 0.0) {
          const double2 u = *reinterpret_cast<const double2*>(d + o);
          dv[0] = u.x;
          dv[1] = u.y;
        } else {
          dv[0] = dv[1] = 0.0;
        }
      }
    }
    if (!v16) {
#pragma unroll
      for (int a = 0; a < NQ; ++a) {
        xv[a] = x[o + a];
        dv[a] = c1 == 0.0 ? 0.0 : d[o + a];
      }
    }
#pragma unroll
    for (int a = 0; a < NQ; ++a) dd[a] = (c1 == 0.0 ? 0.0 : c1 * dv[a]) + c2 * acc[a];
    if constexpr (NQ == 2) {
      if (v16) {
        if (mode == 1) *reinterpret_cast<double2*>(d + o) = make_double2(dd[0], dd[1]);
        *reinterpret_cast<double2*>(x + o) = make_double2(xv[0] + dd[0], xv[1] + dd[1]);
      }
    }
    if (!v16) {
      if (mode == 1) {   // mode 2: a sequence's last step, d is not read again
#pragma unroll
        for (int a = 0; a < NQ; ++a) d[o + a] = dd[a];
      }
#pragma unroll
      for (int a = 0; a < NQ; ++a) x[o + a] = xv[a] + dd[a];
    }
  }
}

}  // namespace

hipError_t launch_patch_factor(const LevelView& L, const PatchView& P, const double* Jv, int prec,
                               void* fac, int* status, hipStream_t s) {
  // blocks larger than 64 rows (the front of the patch order) take two rows
  // per lane (FP32) or two wavefronts (FP64); the others one row per lane
  const int big = L.NQ == 2 ? P.n_big : 0, small = P.n_patch - big;
  const dim3 gb((unsigned)big * P.fac_slabs), gs((unsigned)small * P.fac_slabs);
  if (L.kdeg > 0) {
    // scalar heat patches: at most kHeatMaxNb DoFs, so (q+1) kHeatMaxNb rows:
    // one row per lane up to 64 rows, two (FP32) or two wavefronts (FP64) at q = 3
    constexpr int H = kHeatMaxNb;
    const dim3 ga((unsigned)P.n_patch * P.fac_slabs);
    if (prec == 1) {
      float* f = (float*)fac;
      switch (L.NQ) {
        case 1: hipLaunchKernelGGL((k_patch_factor<1, float, 64, 1, H>), ga, dim3(64), 0, s, L, P, 0, Jv, f, status); break;
        case 2: hipLaunchKernelGGL((k_patch_factor<2, float, 64, 1, H>), ga, dim3(64), 0, s, L, P, 0, Jv, f, status); break;
        case 3: hipLaunchKernelGGL((k_patch_factor<3, float, 64, 1, H>), ga, dim3(64), 0, s, L, P, 0, Jv, f, status); break;
        case 4: hipLaunchKernelGGL((k_patch_factor<4, float, 64, 2, H>), ga, dim3(64), 0, s, L, P, 0, Jv, f, status); break;
        default: return hipErrorInvalidValue;
      }
    } else {
      double* f = (double*)fac;
      switch (L.NQ) {
        case 1: hipLaunchKernelGGL((k_patch_factor<1, double, 64, 1, H>), ga, dim3(64), 0, s, L, P, 0, Jv, f, status); break;
        case 2: hipLaunchKernelGGL((k_patch_factor<2, double, 64, 1, H>), ga, dim3(64), 0, s, L, P, 0, Jv, f, status); break;
        case 3: hipLaunchKernelGGL((k_patch_factor<3, double, 64, 1, H>), ga, dim3(64), 0, s, L, P, 0, Jv, f, status); break;
        case 4: hipLaunchKernelGGL((k_patch_factor<4, double, 128, 1, H>), ga, dim3(128), 0, s, L, P, 0, Jv, f, status); break;
        default: return hipErrorInvalidValue;
      }
    }
    return hipGetLastError();
  }
  if (prec == 1) {
    float* f = (float*)fac;
    if (L.NQ == 2 && big && P.factor_mfma) {
      hipError_t e = launch_patch_factor_mfma(L, P, Jv, f, status, 0, big, s);
      if (e != hipSuccess) return e;
      if (small) hipLaunchKernelGGL((k_patch_factor<2, float, 64, 1>), gs, dim3(64), 0, s, L, P, big, Jv, f, status);
      return hipGetLastError();
    }
    if (L.NQ == 1) {
      hipLaunchKernelGGL((k_patch_factor<1, float, 64, 1>), gs, dim3(64), 0, s, L, P, 0, Jv, f, status);
    } else {
      if (big) hipLaunchKernelGGL((k_patch_factor<2, float, 64, 2>), gb, dim3(64), 0, s, L, P, 0, Jv, f, status);
      if (small) hipLaunchKernelGGL((k_patch_factor<2, float, 64, 1>), gs, dim3(64), 0, s, L, P, big, Jv, f, status);
    }
  } else {
    double* f = (double*)fac;
    if (L.NQ == 1) {
      hipLaunchKernelGGL((k_patch_factor<1, double, 64, 1>), gs, dim3(64), 0, s, L, P, 0, Jv, f, status);
    } else {
      if (big) hipLaunchKernelGGL((k_patch_factor<2, double, 128, 1>), gb, dim3(128), 0, s, L, P, 0, Jv, f, status);
      if (small) hipLaunchKernelGGL((k_patch_factor<2, double, 64, 1>), gs, dim3(64), 0, s, L, P, big, Jv, f, status);
    }
  }
  return hipGetLastError();
}

hipError_t launch_patch_sweep_batch(int nq, const SweepJob* jobs, const SweepTile* tiles, int n_full_tiles,
                                    int n_tiles, int grid, int* ctr, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (nq == 1)
    hipLaunchKernelGGL(k_patch_sweep_f32_batch<1>, dim3((unsigned)grid), dim3(64), 0, s, jobs, tiles, n_full_tiles,
                       n_tiles, ctr);
  else if (nq == 2)
    hipLaunchKernelGGL(k_patch_sweep_f32_batch<2>, dim3((unsigned)grid), dim3(64), 0, s, jobs, tiles, n_full_tiles,
                       n_tiles, ctr);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_patch_factor_batch(int cls, const FactorJob* jobs, const FactorTile* tiles, int n_tiles,
                                     int grid, int* ctr, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (cls) {
    case kFacSmall1:
      hipLaunchKernelGGL(k_patch_factor_f32_batch<1>, dim3((unsigned)grid), dim3(64), 0, s, jobs, tiles, n_tiles, ctr);
      break;
    case kFacSmall2:
      hipLaunchKernelGGL(k_patch_factor_f32_batch<2>, dim3((unsigned)grid), dim3(64), 0, s, jobs, tiles, n_tiles, ctr);
      break;
    case kFacBig2:
      return launch_patch_factor_mfma_batch(jobs, tiles, n_tiles, grid, ctr, s);
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int patch_sweep_batch_occupancy(int nq) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if (nq == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_patch_sweep_f32_batch<1>, 64, 0);
  if (nq == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_patch_sweep_f32_batch<2>, 64, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

int patch_factor_batch_occupancy(int cls) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if (cls == kFacSmall1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_patch_factor_f32_batch<1>, 64, 0);
  if (cls == kFacSmall2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_patch_factor_f32_batch<2>, 64, 0);
  if (cls == kFacBig2) return patch_factor_mfma_batch_occupancy();
  return (e == hipSuccess && n > 0) ? n : 1;
}

// Large blocks inverted in registers (one row per thread, as k_patch_factor)
// where a row fits: FP32 blocks, and FP64 blocks of one temporal node.
// Returns hipErrorNotSupported for the others (FP64 at two nodes), which take
// the dense path.
hipError_t launch_patch_factor_big_reg(const LevelView& L, const PatchView& P, const double* Jv, int prec,
                                       void* fac, int* status, hipStream_t s) {
  const dim3 grid((unsigned)P.n_patch * P.fac_slabs);
  constexpr int NB = kThMaxNb;
  if (prec == 1) {
    float* f = (float*)fac;
    if (L.NQ == 1) hipLaunchKernelGGL((k_patch_factor<1, float, 128, 1, NB, true>), grid, dim3(128), 0, s, L, P, 0, Jv, f, status);
    else if (L.NQ == 2) hipLaunchKernelGGL((k_patch_factor<2, float, 192, 1, NB, true>), grid, dim3(192), 0, s, L, P, 0, Jv, f, status);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (L.NQ == 1) {
    hipLaunchKernelGGL((k_patch_factor<1, double, 128, 1, NB, true>), grid, dim3(128), 0, s, L, P, 0, Jv, (double*)fac, status);
    return hipGetLastError();
  }
  return hipErrorNotSupported;
}

hipError_t launch_patch_extract_dense(const LevelView& L, const PatchView& P, const double* Jv, int b0,
                                      int count, int mmax, double* B, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (L.NQ == 1) hipLaunchKernelGGL(k_patch_extract_dense<1>, dim3(count), dim3(256), 0, s, L, P, Jv, b0, mmax, B);
  else if (L.NQ == 2) hipLaunchKernelGGL(k_patch_extract_dense<2>, dim3(count), dim3(256), 0, s, L, P, Jv, b0, mmax, B);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_patch_store_big(const LevelView& L, const PatchView& P, int prec, const double* B, int b0,
                                  int count, int mmax, void* fac, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const dim3 grid(count), block(256);
  if (prec == 1) {
    float* f = (float*)fac;
    if (L.NQ == 1) hipLaunchKernelGGL((k_patch_store_big<1, float>), grid, block, 0, s, P, B, b0, mmax, f);
    else hipLaunchKernelGGL((k_patch_store_big<2, float>), grid, block, 0, s, P, B, b0, mmax, f);
  } else {
    double* f = (double*)fac;
    if (L.NQ == 1) hipLaunchKernelGGL((k_patch_store_big<1, double>), grid, block, 0, s, P, B, b0, mmax, f);
    else hipLaunchKernelGGL((k_patch_store_big<2, double>), grid, block, 0, s, P, B, b0, mmax, f);
  }
  return hipGetLastError();
}

hipError_t launch_patch_mass(const LevelView& L, const PatchView& P, const double* Mv, double* Mp,
                             hipStream_t s) {
  (void)L;
  hipLaunchKernelGGL(k_patch_mass, dim3(P.n_patch), dim3(256), 0, s, P, Mv, Mp);
  return hipGetLastError();
}

// The generic sweep over all patches, as one launch or, with time chunks,
// as the chunked passes: every chunk from zero incoming values (outputs of
// chunk 0, end values of every chunk), the interface recurrence, then the
// chunks after the first from their true incoming values.
template <int NQ, typename T, int WAVES, bool INV, int NBMAX, int NBUMAX>
hipError_t sweep_generic(const LevelView& L, const PatchView& P, const void* fac, const double* Mp,
                         TimeEnds te, const double* r, double* Y, hipStream_t s) {
  if (INV && P.slab_stride != 0) return hipErrorInvalidValue;   // INV: one block for every slab
  const T* f = (const T*)fac;
  const dim3 block(64 * WAVES);
  const int nc = P.time_chunks > 1 ? P.time_chunks : 1;
  if (nc == 1) {
    const ChunkArgs ca{L.N, 0, INT_MAX, 1, nullptr, nullptr};
    hipLaunchKernelGGL((k_patch_sweep<NQ, T, WAVES, INV, NBMAX, NBUMAX>), dim3(P.n_patch), block, 0, s, L, P, f, Mp, te, r, Y, ca);
    return hipGetLastError();
  }
  const ChunkArgs a{P.chunk_len, 0, 0, nc, nullptr, P.chunk_w_end};
  hipLaunchKernelGGL((k_patch_sweep<NQ, T, WAVES, INV, NBMAX, NBUMAX>), dim3(P.n_patch, nc), block, 0, s, L, P, f, Mp, te, r, Y, a);
  const ChunkArgs ci{P.chunk_len, 0, 0, nc, nullptr, nullptr};
  hipLaunchKernelGGL((k_patch_chunk_interface<NBUMAX>), dim3(P.n_patch), dim3(64), 0, s, P, ci, P.chunk_T, P.chunk_w_end, P.chunk_w_in);
  const ChunkArgs c{P.chunk_len, 1, INT_MAX, nc, P.chunk_w_in, nullptr};
  hipLaunchKernelGGL((k_patch_sweep<NQ, T, WAVES, INV, NBMAX, NBUMAX>), dim3(P.n_patch, nc - 1), block, 0, s, L, P, f, Mp, te, r, Y, c);
  return hipGetLastError();
}

hipError_t launch_patch_sweep(const LevelView& L, const PatchView& P, int prec, const void* fac,
                              const double* Mp, const double* e0, const double* e1,
                              const double* r, void* Y, hipStream_t s) {
  const TimeEnds te = time_ends(L.NQ, e0, e1);
  double* Yd = (double*)Y;
  if (L.thk > 0) {
    // Taylor-Hood P3-P2 patches: the large-block sweep, FP64 outputs
    const dim3 grid(P.n_patch);
    if (prec == 1) {
      const float* f = (const float*)fac;
      if (L.NQ == 1) hipLaunchKernelGGL((k_patch_sweep_big<1, float, 2>), grid, dim3(128), 0, s, L, P, f, Mp, te, r, Yd);
      else hipLaunchKernelGGL((k_patch_sweep_big<2, float, 3>), grid, dim3(192), 0, s, L, P, f, Mp, te, r, Yd);
    } else {
      const double* f = (const double*)fac;
      if (L.NQ == 1) hipLaunchKernelGGL((k_patch_sweep_big<1, double, 2>), grid, dim3(128), 0, s, L, P, f, Mp, te, r, Yd);
      else hipLaunchKernelGGL((k_patch_sweep_big<2, double, 3>), grid, dim3(192), 0, s, L, P, f, Mp, te, r, Yd);
    }
    return hipGetLastError();
  }
  if (L.kdeg > 0) {
    // scalar heat patches (at most kHeatMaxNb DoFs, (q+1) kHeatMaxNb rows):
    // a wavefront's threads form up to 64 rows and hold up to 20 FP32 or 10
    // FP64 column panels; outputs stay FP64
    constexpr int H = kHeatMaxNb;
    if (prec == 1) {
      switch (L.NQ) {
        case 1: return sweep_generic<1, float, 1, true, H, H>(L, P, fac, Mp, te, r, Yd, s);
        case 2: return sweep_generic<2, float, 1, true, H, H>(L, P, fac, Mp, te, r, Yd, s);
        case 3: return sweep_generic<3, float, 1, true, H, H>(L, P, fac, Mp, te, r, Yd, s);
        case 4: return sweep_generic<4, float, 2, true, H, H>(L, P, fac, Mp, te, r, Yd, s);
        default: return hipErrorInvalidValue;
      }
    }
    switch (L.NQ) {
      case 1: return sweep_generic<1, double, 1, true, H, H>(L, P, fac, Mp, te, r, Yd, s);
      case 2: return sweep_generic<2, double, 2, true, H, H>(L, P, fac, Mp, te, r, Yd, s);
      case 3: return sweep_generic<3, double, 3, true, H, H>(L, P, fac, Mp, te, r, Yd, s);
      case 4: return sweep_generic<4, double, 4, true, H, H>(L, P, fac, Mp, te, r, Yd, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (prec == 1 && P.time_chunks > 1) {
    // chunked FP32 Navier-Stokes sweeps take the generic kernel (FP64 outputs)
    if (L.NQ == 1) return sweep_generic<1, float, 1, false, kMaxNb, kMaxNbu>(L, P, fac, Mp, te, r, Yd, s);
    return sweep_generic<2, float, 2, false, kMaxNb, kMaxNbu>(L, P, fac, Mp, te, r, Yd, s);
  }
  if (prec == 1) {
    const double e01 = L.NQ > 1 ? e0[1] : 0.0, e11 = L.NQ > 1 ? e1[1] : 0.0;
    dim3 grid(P.n_patch);
    if (L.NQ == 1) {
      hipLaunchKernelGGL((k_patch_sweep_f32<1, double>), grid, dim3(64), 0, s, L, P, (const float*)fac, Mp, e0[0], e01, e1[0], e11, r, (float*)Y);
    } else {
      hipLaunchKernelGGL((k_patch_sweep_f32<2, double>), grid, dim3(64), 0, s, L, P, (const float*)fac, Mp, e0[0], e01, e1[0], e11, r, (float*)Y);
    }
    return hipGetLastError();
  }
  if (L.NQ == 1) return sweep_generic<1, double, 2, false, kMaxNb, kMaxNbu>(L, P, fac, Mp, te, r, Yd, s);
  return sweep_generic<2, double, 4, false, kMaxNb, kMaxNbu>(L, P, fac, Mp, te, r, Yd, s);
}

bool sweep_takes_f32_residual(const LevelView& L, const PatchView& P, int prec) {
  return L.thk == 0 && L.kdeg == 0 && prec == 1 && P.time_chunks <= 1 && (L.NQ == 1 || L.NQ == 2);
}

hipError_t launch_patch_sweep_f32r(const LevelView& L, const PatchView& P, int prec, const void* fac,
                                   const double* Mp, const double* e0, const double* e1, const float* r,
                                   void* Y, hipStream_t s) {
  if (!sweep_takes_f32_residual(L, P, prec)) return hipErrorInvalidValue;
  const double e01 = L.NQ > 1 ? e0[1] : 0.0, e11 = L.NQ > 1 ? e1[1] : 0.0;
  dim3 grid(P.n_patch);
  if (L.NQ == 1) {
    hipLaunchKernelGGL((k_patch_sweep_f32<1, float>), grid, dim3(64), 0, s, L, P, (const float*)fac, Mp, e0[0], e01, e1[0], e11, r, (float*)Y);
  } else {
    hipLaunchKernelGGL((k_patch_sweep_f32<2, float>), grid, dim3(64), 0, s, L, P, (const float*)fac, Mp, e0[0], e01, e1[0], e11, r, (float*)Y);
  }
  return hipGetLastError();
}

template <int NQ, typename T, int NBUMAX>
hipError_t chunk_transfer(const LevelView& L, const PatchView& P, const void* fac, const double* Mp,
                          TimeEnds te, hipStream_t s) {
  const ChunkArgs ca{P.chunk_len, 0, 0, P.time_chunks, nullptr, nullptr};
  hipLaunchKernelGGL((k_patch_chunk_transfer<NQ, T, NBUMAX>), dim3(P.n_patch, P.time_chunks), dim3(256), 0, s, L, P,
                     (const T*)fac, Mp, te, ca, (double*)P.chunk_T);
  return hipGetLastError();
}

hipError_t launch_patch_chunk_transfer(const LevelView& L, const PatchView& P, int prec, const void* fac,
                                       const double* Mp, const double* e0, const double* e1,
                                       hipStream_t s) {
  if (P.time_chunks <= 1) return hipSuccess;
  const TimeEnds te = time_ends(L.NQ, e0, e1);
  constexpr int H = kHeatMaxNb;
  if (L.kdeg > 0) {
    if (prec == 1) {
      switch (L.NQ) {
        case 1: return chunk_transfer<1, float, H>(L, P, fac, Mp, te, s);
        case 2: return chunk_transfer<2, float, H>(L, P, fac, Mp, te, s);
        case 3: return chunk_transfer<3, float, H>(L, P, fac, Mp, te, s);
        case 4: return chunk_transfer<4, float, H>(L, P, fac, Mp, te, s);
        default: return hipErrorInvalidValue;
      }
    }
    switch (L.NQ) {
      case 1: return chunk_transfer<1, double, H>(L, P, fac, Mp, te, s);
      case 2: return chunk_transfer<2, double, H>(L, P, fac, Mp, te, s);
      case 3: return chunk_transfer<3, double, H>(L, P, fac, Mp, te, s);
      case 4: return chunk_transfer<4, double, H>(L, P, fac, Mp, te, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (prec == 1) return L.NQ == 1 ? chunk_transfer<1, float, kMaxNbu>(L, P, fac, Mp, te, s)
                                  : chunk_transfer<2, float, kMaxNbu>(L, P, fac, Mp, te, s);
  return L.NQ == 1 ? chunk_transfer<1, double, kMaxNbu>(L, P, fac, Mp, te, s)
                   : chunk_transfer<2, double, kMaxNbu>(L, P, fac, Mp, te, s);
}

hipError_t launch_patch_gather(const LevelView& L, const PatchView& P, int prec, const void* Y,
                               int mode, double c1, double c2, double* z, double* d, double* x,
                               hipStream_t s) {
  if (L.N <= 256) {
    const int R = 256 / L.N;
    const dim3 grid((unsigned)((L.nf + R - 1) / R)), block(256);
    if (sweep_outputs_f32(L, P, prec)) {
      const float* Yf = (const float*)Y;
      if (L.NQ == 1) hipLaunchKernelGGL((k_patch_gather_rows<1, float>), grid, block, 0, s, L.nf, L.N, P, Yf, mode, c1, c2, z, d, x);
      else hipLaunchKernelGGL((k_patch_gather_rows<2, float>), grid, block, 0, s, L.nf, L.N, P, Yf, mode, c1, c2, z, d, x);
      return hipGetLastError();
    }
    const double* Yd = (const double*)Y;
    switch (L.NQ) {
      case 1: hipLaunchKernelGGL((k_patch_gather_rows<1, double>), grid, block, 0, s, L.nf, L.N, P, Yd, mode, c1, c2, z, d, x); break;
      case 2: hipLaunchKernelGGL((k_patch_gather_rows<2, double>), grid, block, 0, s, L.nf, L.N, P, Yd, mode, c1, c2, z, d, x); break;
      case 3: hipLaunchKernelGGL((k_patch_gather_rows<3, double>), grid, block, 0, s, L.nf, L.N, P, Yd, mode, c1, c2, z, d, x); break;
      case 4: hipLaunchKernelGGL((k_patch_gather_rows<4, double>), grid, block, 0, s, L.nf, L.N, P, Yd, mode, c1, c2, z, d, x); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  // more than 256 slabs: one thread per (DoF, slab) with its own index chain
  const int64_t n = (int64_t)L.nf * L.N;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (sweep_outputs_f32(L, P, prec)) {
    const float* Yf = (const float*)Y;
    if (L.NQ == 1) hipLaunchKernelGGL((k_patch_gather<1, float>), grid, block, 0, s, L.nf, L.N, P, Yf, mode, c1, c2, z, d, x);
    else hipLaunchKernelGGL((k_patch_gather<2, float>), grid, block, 0, s, L.nf, L.N, P, Yf, mode, c1, c2, z, d, x);
  } else {
    const double* Yd = (const double*)Y;
    switch (L.NQ) {
      case 1: hipLaunchKernelGGL((k_patch_gather<1, double>), grid, block, 0, s, L.nf, L.N, P, Yd, mode, c1, c2, z, d, x); break;
      case 2: hipLaunchKernelGGL((k_patch_gather<2, double>), grid, block, 0, s, L.nf, L.N, P, Yd, mode, c1, c2, z, d, x); break;
      case 3: hipLaunchKernelGGL((k_patch_gather<3, double>), grid, block, 0, s, L.nf, L.N, P, Yd, mode, c1, c2, z, d, x); break;
      case 4: hipLaunchKernelGGL((k_patch_gather<4, double>), grid, block, 0, s, L.nf, L.N, P, Yd, mode, c1, c2, z, d, x); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace stwr
