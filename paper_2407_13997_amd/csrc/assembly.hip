// Space-time assembly of Taylor-Hood P2-P1 x DG(q) Navier-Stokes on gfx950
// (Sec. 2, eq. nsfem with forcing; upwind jump of eq. dgintime), and of the
// P_k x DG(q) heat equation (eq. heatfem) at the end of the file.
//
// One 64-lane workgroup per (cell, slab).  The workgroup stages the cell's
// nodal values, its physical basis gradients and the fields at the
// 25 x (q+3) space-time quadrature points in LDS; lanes then own local matrix
// (or vector) entries and add them into the global space-time operator with
// FP64 atomics.  Values of the operator are stored per spatial nonzero k as
// Jv[((k * N + n) * NQ + a) * NQ + b] (test temporal node a, trial node b);
// Mv[k] holds the velocity mass matrix, which is all the jump coupling of
// slab n to slab n-1 needs (-e0 e1^T (x) M).
//
// Pressure convention: the momentum equation is tested as -(P, div psi) and
// the continuity equation as -(div U, chi).  Boundary velocities are the
// exact velocity at the temporal nodes; the value entering slab 0 from the
// left is the P2 interpolant of the velocity at t = 0.
#include "device.h"

namespace stwr {

namespace {

struct ModeSums {
  double px, py, pxx, pxy, pyy, pxt, pyt, lapx, lapy;
};

// Stream-function derivative sums of the manufactured solution at (t, x, y).
__device__ ModeSums psi_sums(const MmsDev& m, double t, double x, double y) {
  ModeSums s{};
  for (int k = 0; k < m.n_psi; ++k) {
    const double A = M_PI * m.psi_ab[2 * k], B = M_PI * m.psi_ab[2 * k + 1];
    const double c = m.psi_coef[3 * k], w = m.psi_coef[3 * k + 1], th = m.psi_coef[3 * k + 2];
    double sx, cx, sy, cy, st, ct;
    sincos(A * x, &sx, &cx);
    sincos(B * y, &sy, &cy);
    sincos(w * t + th, &st, &ct);
    const double psx = c * A * cx * sy, psy = c * B * sx * cy;
    s.px += psx * ct;
    s.py += psy * ct;
    s.pxx -= c * A * A * sx * sy * ct;
    s.pyy -= c * B * B * sx * sy * ct;
    s.pxy += c * A * B * cx * cy * ct;
    s.pxt -= psx * w * st;
    s.pyt -= psy * w * st;
    // each mode is an eigenfunction of the Laplacian: lap(psi_m) = -(A^2 + B^2) psi_m
    const double k2 = A * A + B * B;
    s.lapx -= k2 * psy * ct;   // lap(u_x) = lap(psi_y)
    s.lapy += k2 * psx * ct;   // lap(u_y) = -lap(psi_x)
  }
  return s;
}

__device__ void exact_velocity(const MmsDev& m, double t, double x, double y, double& ux, double& uy) {
  ux = 0.0;
  uy = 0.0;
  if (m.flow == 1) {   // Chorin test problem (Sec. 2)
    const double e = exp(-2.0 * M_PI * M_PI * t);
    ux = -cos(M_PI * x) * sin(M_PI * y) * e;
    uy = sin(M_PI * x) * cos(M_PI * y) * e;
    return;
  }
  if (m.flow == 2) {   // lid-driven cavity: the lid is the open top side
    if (y > 1.0 - 1e-12 && x > 1e-12 && x < 1.0 - 1e-12) ux = 1.0;
    return;
  }
  for (int k = 0; k < m.n_psi; ++k) {
    const double A = M_PI * m.psi_ab[2 * k], B = M_PI * m.psi_ab[2 * k + 1];
    const double c = m.psi_coef[3 * k], w = m.psi_coef[3 * k + 1], th = m.psi_coef[3 * k + 2];
    const double tau = cos(w * t + th);
    ux += c * B * sin(A * x) * cos(B * y) * tau;
    uy -= c * A * cos(A * x) * sin(B * y) * tau;
  }
}

// Initial velocity: the velocity at t = 0, except for the cavity, which
// starts at rest (the lid included).
__device__ void initial_velocity(const MmsDev& m, double x, double y, double& ux, double& uy) {
  if (m.flow == 2) {
    ux = 0.0;
    uy = 0.0;
    return;
  }
  exact_velocity(m, 0.0, x, y, ux, uy);
}

__device__ void forcing(const MmsDev& m, double t, double x, double y, double& fx, double& fy) {
  if (m.flow != 0) {   // the Chorin pair solves the equations unforced; the cavity has none
    fx = 0.0;
    fy = 0.0;
    return;
  }
  const ModeSums s = psi_sums(m, t, x, y);
  const double ux = s.py, uy = -s.px;
  const double convx = ux * s.pxy + uy * s.pyy;
  const double convy = -ux * s.pxx - uy * s.pxy;
  double gpx = 0.0, gpy = 0.0;
  for (int k = 0; k < m.n_p; ++k) {
    const double A = M_PI * m.p_ab[2 * k], B = M_PI * m.p_ab[2 * k + 1];
    const double d = m.p_coef[3 * k], w = m.p_coef[3 * k + 1], th = m.p_coef[3 * k + 2];
    const double tau = cos(w * t + th);
    gpx -= d * A * sin(A * x) * cos(B * y) * tau;
    gpy -= d * B * cos(A * x) * sin(B * y) * tau;
  }
  fx = s.pyt + m.reynolds * convx - s.lapx + gpx;
  fy = -s.pxt + m.reynolds * convy - s.lapy + gpy;
}

// Cell geometry: inverse Jacobian (row-major 2x2), |det| and vertex 0.
__device__ void cell_geometry(const LevelView& L, int c, double inv[4], double& adet, double v0[2],
                              double Jc[4]) {
  const int a = L.cells[3 * c], b = L.cells[3 * c + 1], d = L.cells[3 * c + 2];
  const double ax = (a % L.n1) * L.h, ay = (a / L.n1) * L.h;
  const double bx = (b % L.n1) * L.h, by = (b / L.n1) * L.h;
  const double dx = (d % L.n1) * L.h, dy = (d / L.n1) * L.h;
  Jc[0] = bx - ax; Jc[1] = dx - ax;   // column 0 = v1 - v0, column 1 = v2 - v0
  Jc[2] = by - ay; Jc[3] = dy - ay;
  const double det = Jc[0] * Jc[3] - Jc[1] * Jc[2];
  inv[0] = Jc[3] / det; inv[1] = -Jc[1] / det;
  inv[2] = -Jc[2] / det; inv[3] = Jc[0] / det;
  adet = fabs(det);
  v0[0] = ax; v0[1] = ay;
}

// Shared staging common to both kernels.
template <int NQ>
struct CellStage {
  double ul[2][6][NQ];            // velocity nodal values (free or Dirichlet)
  double gN[kQx][6][2];           // physical P2 gradients
  double wdet[kQx];
  double xp[kQx][2];              // physical quadrature points
  double uq[kMaxG][kQx][2];
  double gq[kMaxG][kQx][2][2];    // [comp][d/dx_k]
};

template <int NQ>
__device__ void stage_cell(const LevelView& L, const RefTables* __restrict__ T, const MmsDev& mms,
                           const double* __restrict__ U, int c, int n, CellStage<NQ>& S) {
  const int tid = threadIdx.x;
  __shared__ double inv_s[4], adet_s, v0_s[2], J_s[4];
  if (tid == 0) {
    double inv[4], adet, v0[2], Jc[4];
    cell_geometry(L, c, inv, adet, v0, Jc);
    for (int k = 0; k < 4; ++k) { inv_s[k] = inv[k]; J_s[k] = Jc[k]; }
    adet_s = adet;
    v0_s[0] = v0[0]; v0_s[1] = v0[1];
  }
  if (tid < 12 * NQ) {
    const int comp = tid / (6 * NQ), i = (tid / NQ) % 6, a = tid % NQ;
    const int node = L.cell_p2[6 * c + i];
    const int k = L.node_free[node];
    double v;
    if (k >= 0) {
      v = U[((int64_t)(2 * k + comp) * L.N + n) * NQ + a];
    } else {
      const double t = (n + T->tnode[a]) * L.dt;
      const double x = (node % L.n2) * 0.5 * L.h, y = (node / L.n2) * 0.5 * L.h;
      double ux, uy;
      exact_velocity(mms, t, x, y, ux, uy);
      v = comp == 0 ? ux : uy;
    }
    S.ul[comp][i][a] = v;
  }
  __syncthreads();
  for (int e = tid; e < kQx * 6; e += 64) {
    const int x = e / 6, i = e % 6;
    for (int k = 0; k < 2; ++k)
      S.gN[x][i][k] = T->dN2[x][i][0] * inv_s[0 * 2 + k] + T->dN2[x][i][1] * inv_s[1 * 2 + k];
  }
  if (tid < kQx) {
    S.wdet[tid] = T->wq[tid] * adet_s;
    S.xp[tid][0] = v0_s[0] + J_s[0] * T->xq[tid][0] + J_s[1] * T->xq[tid][1];
    S.xp[tid][1] = v0_s[1] + J_s[2] * T->xq[tid][0] + J_s[3] * T->xq[tid][1];
  }
  __syncthreads();
  const int G = T->G;
  for (int e = tid; e < G * kQx; e += 64) {
    const int g = e / kQx, x = e % kQx;
    for (int comp = 0; comp < 2; ++comp) {
      double u = 0.0, gx = 0.0, gy = 0.0;
      for (int i = 0; i < 6; ++i) {
        double ui = 0.0;
        for (int b = 0; b < NQ; ++b) ui += T->Phi[g][b] * S.ul[comp][i][b];
        u += ui * T->N2[x][i];
        gx += ui * S.gN[x][i][0];
        gy += ui * S.gN[x][i][1];
      }
      S.uq[g][x][comp] = u;
      S.gq[g][x][comp][0] = gx;
      S.gq[g][x][comp][1] = gy;
    }
  }
  __syncthreads();
}

// Symmetric temporal pair s of NQ nodes (a <= b), s = 0 .. NQ (NQ + 1) / 2 - 1.
template <int NQ>
__device__ __forceinline__ void temporal_pair(int s, int& a, int& b) {
  a = 0;
  while (s >= NQ - a) { s -= NQ - a; ++a; }
  b = a + s;
}

template <int NQ>
__global__ __launch_bounds__(64) void k_jacobian(LevelView L, const RefTables* __restrict__ T,
                                                 MmsDev mms, const double* __restrict__ U,
                                                 double* __restrict__ Jv, double* __restrict__ Mv) {
  // one workgroup per (cell, slab), slab fastest: consecutive workgroups
  // update the same operator lines (each holds several slabs of a nonzero)
  const int c = cell_of(L), n = blockIdx.x % L.N, tid = threadIdx.x;
  constexpr int NS = NQ * (NQ + 1) / 2;   // temporal pairs a <= b
  __shared__ CellStage<NQ> S;
  // the convection terms with the temporal quadrature folded in first: for a
  // temporal pair (a, b) and a spatial point x, w_x sum_g wg Phi_a Phi_b of
  // the state's gradient (the Newton term) and of its value (the transport
  // term).  Both are symmetric in (a, b), so NS pairs cover all NQ^2.
  __shared__ double WD[NS][kQx][4], WU[NS][kQx][2];
  stage_cell<NQ>(L, T, mms, U, c, n, S);
  constexpr int G = NQ + 2;   // temporal Gauss points (q + 3), as the tables are built
  const double dt = L.dt, R = mms.reynolds;
  const int* nzc = L.cell_nz + (int64_t)225 * c;
  for (int e = tid; e < NS * kQx; e += 64) {
    const int sp = e / kQx, x = e % kQx;
    int a, b;
    temporal_pair<NQ>(sp, a, b);
    double d[4] = {0.0, 0.0, 0.0, 0.0}, u[2] = {0.0, 0.0};
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const double cw = T->wg[g] * T->Phi[g][a] * T->Phi[g][b];
#pragma unroll
      for (int k = 0; k < 4; ++k) d[k] += cw * S.gq[g][x][k / 2][k % 2];
      u[0] += cw * S.uq[g][x][0];
      u[1] += cw * S.uq[g][x][1];
    }
    const double w = S.wdet[x];
#pragma unroll
    for (int k = 0; k < 4; ++k) WD[sp][x][k] = w * d[k];
    WU[sp][x][0] = w * u[0];
    WU[sp][x][1] = w * u[1];
  }
  __syncthreads();
  // tasks spread over all lanes: (temporal pair, velocity pair i, j), each
  // the spatial sums of its entries, then the 18 pressure-velocity pairs
  constexpr int NV = 36 * NS, NT = NV + 18;
#pragma unroll 1
  for (int task = tid; task < NT; task += 64) {
    if (task < NV) {
      const int sp = task / 36, i = (task % 36) / 6, j = task % 6;
      int a, b;
      temporal_pair<NQ>(sp, a, b);
      // the entries this task adds to, (ci, cj) blocks of the pairs (a, b)
      // and (b, a): their current values are loaded now, so the read of the
      // read-modify-write overlaps the sums below (no other workgroup of
      // this colour and no other task touches them)
      double* dst[2][4];
      double old[2][4];
#pragma unroll
      for (int pass = 0; pass < 2; ++pass)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ci = e / 2, cj = e % 2;
          const int nz = nzc[15 * (6 * ci + i) + 6 * cj + j];
          const int aa = pass ? b : a, bb = pass ? a : b;
          dst[pass][e] = (nz >= 0 && (pass == 0 || a != b)) ? &Jv[(((int64_t)nz * L.N + n) * NQ + aa) * NQ + bb] : nullptr;
          old[pass][e] = dst[pass][e] ? *dst[pass][e] : 0.0;
        }
      double Mij = 0.0, Kij = 0.0, C1 = 0.0, C2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
      for (int x = 0; x < kQx; ++x) {
        const double w = S.wdet[x], Ni = T->N2[x][i], Nj = T->N2[x][j];
        Mij += w * Ni * Nj;
        Kij += w * (S.gN[x][i][0] * S.gN[x][j][0] + S.gN[x][i][1] * S.gN[x][j][1]);
        C1 += Ni * (WU[sp][x][0] * S.gN[x][j][0] + WU[sp][x][1] * S.gN[x][j][1]);
        const double nn = Ni * Nj;
#pragma unroll
        for (int k = 0; k < 4; ++k) C2[k] += nn * WD[sp][x][k];
      }
      // the entries (a, b) and, off the diagonal, (b, a)
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        const int aa = pass ? b : a, bb = pass ? a : b;
        const double diag = T->T[aa][bb] * Mij + dt * T->W[aa][bb] * Kij + dt * R * C1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ci = e / 2, cj = e % 2;
          const double v = dt * R * C2[e] + (ci == cj ? diag : 0.0);
          if (dst[pass][e]) *dst[pass][e] = old[pass][e] + v;
        }
      }
      if (n == 0 && sp == 0) {
        for (int ci = 0; ci < 2; ++ci) {
          const int nz = nzc[15 * (6 * ci + i) + 6 * ci + j];
          if (nz >= 0) scatter_add(L, &Mv[nz], Mij);
        }
      }
    } else {
      const int t = task - NV, j = t / 6, i = t % 6;   // pressure j, velocity node i
      double B[2] = {0.0, 0.0};
      for (int x = 0; x < kQx; ++x) {
        const double w = S.wdet[x] * T->N1[x][j];
        B[0] += w * S.gN[x][i][0];
        B[1] += w * S.gN[x][i][1];
      }
      for (int a = 0; a < NQ; ++a)
        for (int b = 0; b < NQ; ++b)
          for (int ci = 0; ci < 2; ++ci) {
            const double v = -dt * T->W[a][b] * B[ci];
            const int nz1 = nzc[15 * (6 * ci + i) + 12 + j];
            if (nz1 >= 0) scatter_add(L, &Jv[(((int64_t)nz1 * L.N + n) * NQ + a) * NQ + b], v);
            const int nz2 = nzc[15 * (12 + j) + 6 * ci + i];
            if (nz2 >= 0) scatter_add(L, &Jv[(((int64_t)nz2 * L.N + n) * NQ + a) * NQ + b], v);
          }
    }
  }
}

template <int NQ>
__global__ __launch_bounds__(64) void k_residual(LevelView L, const RefTables* __restrict__ T,
                                                 MmsDev mms, const double* __restrict__ U,
                                                 double* __restrict__ F) {
  // slab fastest, as in k_jacobian
  const int c = cell_of(L), n = blockIdx.x % L.N, tid = threadIdx.x;
  __shared__ CellStage<NQ> S;
  __shared__ double pl[3][NQ];
  __shared__ double prev[2][6];
  // per (temporal, spatial) quadrature point, weighted: the value term
  // (u_t + R (u . grad) u - f), the gradient term dt (grad u - p I) and the
  // divergence; then their sums over the spatial points against each basis
  // function (all lanes take part in both), then the sums over the temporal
  // points
  __shared__ double Av[kMaxG][kQx][2], Bv[kMaxG][kQx][2][2], Dv[kMaxG][kQx];
  __shared__ double jq[kQx][2];   // U(s=0) - U_{n-1}(1) at the quadrature points
  __shared__ double Pv[kMaxG][2][6], Jm[2][6], Qv[kMaxG][3];
  stage_cell<NQ>(L, T, mms, U, c, n, S);
  const int G = T->G;
  if (tid < 3 * NQ) {
    const int j = tid / NQ, a = tid % NQ;
    pl[j][a] = U[((int64_t)(L.po + L.cells[3 * c + j]) * L.N + n) * NQ + a];
  } else if (tid >= 32 && tid < 44) {
    const int comp = (tid - 32) / 6, i = (tid - 32) % 6;
    const int node = L.cell_p2[6 * c + i];
    const int k = L.node_free[node];
    const double x = (node % L.n2) * 0.5 * L.h, y = (node / L.n2) * 0.5 * L.h;
    double v = 0.0;
    if (n == 0) {
      double ux, uy;
      initial_velocity(mms, x, y, ux, uy);
      v = comp == 0 ? ux : uy;
    } else {
      for (int b = 0; b < NQ; ++b) {
        double vb;
        if (k >= 0) {
          vb = U[((int64_t)(2 * k + comp) * L.N + n - 1) * NQ + b];
        } else {
          double ux, uy;
          exact_velocity(mms, (n - 1 + T->tnode[b]) * L.dt, x, y, ux, uy);
          vb = comp == 0 ? ux : uy;
        }
        v += T->e1[b] * vb;
      }
    }
    prev[comp][i] = v;
  }
  __syncthreads();
  const double dt = L.dt, R = mms.reynolds;
  for (int e = tid; e < G * kQx; e += 64) {
    const int g = e / kQx, x = e % kQx;
    double p = 0.0;
    for (int j = 0; j < 3; ++j) {
      double pj = 0.0;
      for (int b = 0; b < NQ; ++b) pj += T->Phi[g][b] * pl[j][b];
      p += pj * T->N1[x][j];
    }
    double f[2];
    forcing(mms, (n + T->sg[g]) * L.dt, S.xp[x][0], S.xp[x][1], f[0], f[1]);
    const double w = S.wdet[x];
    for (int comp = 0; comp < 2; ++comp) {
      double d = 0.0;
      for (int i = 0; i < 6; ++i) {
        double ui = 0.0;
        for (int b = 0; b < NQ; ++b) ui += T->dPhi[g][b] * S.ul[comp][i][b];
        d += ui * T->N2[x][i];
      }
      const double conv = S.uq[g][x][0] * S.gq[g][x][comp][0] + S.uq[g][x][1] * S.gq[g][x][comp][1];
      Av[g][x][comp] = w * (d + dt * (R * conv - f[comp]));
      Bv[g][x][comp][0] = w * dt * (S.gq[g][x][comp][0] - (comp == 0 ? p : 0.0));
      Bv[g][x][comp][1] = w * dt * (S.gq[g][x][comp][1] - (comp == 1 ? p : 0.0));
    }
    Dv[g][x] = w * (S.gq[g][x][0][0] + S.gq[g][x][1][1]);
  }
  if (tid < kQx) {
    for (int comp = 0; comp < 2; ++comp) {
      double u0 = 0.0, up = 0.0;
      for (int i = 0; i < 6; ++i) {
        double ui = 0.0;
        for (int b = 0; b < NQ; ++b) ui += T->e0[b] * S.ul[comp][i][b];
        u0 += ui * T->N2[tid][i];
        up += prev[comp][i] * T->N2[tid][i];
      }
      jq[tid][comp] = u0 - up;
    }
  }
  __syncthreads();
  // sums over the spatial points: Pv[g][comp][i] (value and gradient terms
  // against velocity basis i), Jm[comp][i] (the jump), Qv[g][j] (divergence
  // against pressure basis j)
  for (int e = tid; e < G * 12 + 12 + G * 3; e += 64) {
    double acc = 0.0;
    if (e < G * 12) {
      const int g = e / 12, comp = (e / 6) % 2, i = e % 6;
      for (int x = 0; x < kQx; ++x)
        acc += Av[g][x][comp] * T->N2[x][i] + Bv[g][x][comp][0] * S.gN[x][i][0] + Bv[g][x][comp][1] * S.gN[x][i][1];
      Pv[g][comp][i] = acc;
    } else if (e < G * 12 + 12) {
      const int comp = (e - G * 12) / 6, i = (e - G * 12) % 6;
      for (int x = 0; x < kQx; ++x) acc += S.wdet[x] * jq[x][comp] * T->N2[x][i];
      Jm[comp][i] = acc;
    } else {
      const int g = (e - G * 12 - 12) / 3, j = (e - G * 12 - 12) % 3;
      for (int x = 0; x < kQx; ++x) acc += Dv[g][x] * T->N1[x][j];
      Qv[g][j] = acc;
    }
  }
  __syncthreads();
  if (tid < 12 * NQ) {
    const int comp = tid / (6 * NQ), i = (tid / NQ) % 6, a = tid % NQ;
    double acc = 0.0;
    for (int g = 0; g < G; ++g) acc += T->wg[g] * T->Phi[g][a] * Pv[g][comp][i];
    acc += T->e0[a] * Jm[comp][i];
    const int dof = L.cell_dofs[15 * c + 6 * comp + i];
    if (dof >= 0) scatter_add(L, &F[((int64_t)dof * L.N + n) * NQ + a], acc);
  } else if (tid >= 32 && tid < 32 + 3 * NQ) {
    const int j = (tid - 32) / NQ, a = (tid - 32) % NQ;
    double acc = 0.0;
    for (int g = 0; g < G; ++g) acc += T->wg[g] * T->Phi[g][a] * Qv[g][j];
    const int dof = L.po + L.cells[3 * c + j];
    scatter_add(L, &F[((int64_t)dof * L.N + n) * NQ + a], -dt * acc);
  }
}

// Space-time velocity L2 error (Sec. 5, the error norm of the convergence
// tables): part[n * nc + c] = int_{I_n} int_c |u - U|^2, by the residual's
// quadrature (q + 3 Gauss points in time, the 25-point rule in space).
// The per-workgroup sum runs in a fixed tree, so the result is deterministic.
template <int NQ>
__global__ __launch_bounds__(64) void k_velocity_error(LevelView L, const RefTables* __restrict__ T,
                                                       MmsDev mms, const double* __restrict__ U,
                                                       double* __restrict__ part) {
  const int c = blockIdx.x, n = blockIdx.y, tid = threadIdx.x;
  __shared__ CellStage<NQ> S;
  __shared__ double red[64];
  stage_cell<NQ>(L, T, mms, U, c, n, S);
  double acc = 0.0;
  for (int e = tid; e < T->G * kQx; e += 64) {
    const int g = e / kQx, x = e % kQx;
    double ux, uy;
    exact_velocity(mms, (n + T->sg[g]) * L.dt, S.xp[x][0], S.xp[x][1], ux, uy);
    const double dx = ux - S.uq[g][x][0], dy = uy - S.uq[g][x][1];
    acc += T->wg[g] * S.wdet[x] * (dx * dx + dy * dy);
  }
  red[tid] = acc;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) part[(int64_t)n * L.nc + c] = L.dt * red[0];
}

// out[0] = sum of part[0 .. n), one workgroup, fixed summation order.
__global__ __launch_bounds__(256) void k_sum(int64_t n, const double* __restrict__ part,
                                             double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// Full nodal vector from a free one: [ux: nn][N][NQ], [uy: nn][N][NQ],
// [p: nv][N][NQ]; Dirichlet velocity values are the exact velocity at the
// node and temporal node (the boundary data of the problem).
__global__ __launch_bounds__(256) void k_expand(LevelView L, const RefTables* __restrict__ T,
                                                MmsDev mms, const double* __restrict__ U,
                                                double* __restrict__ full) {
  const int64_t nn = (int64_t)L.n2 * L.n2, nv = (int64_t)L.n1 * L.n1;
  const int64_t nt = (int64_t)L.N * L.NQ;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (2 * nn + nv) * nt) return;
  const int64_t row = e / nt, tt = e % nt;
  double v;
  if (row < 2 * nn) {
    const int comp = (int)(row / nn), node = (int)(row % nn);
    const int k = L.node_free[node];
    if (k >= 0) {
      v = U[(int64_t)(2 * k + comp) * nt + tt];
    } else {
      const int n = (int)(tt / L.NQ), a = (int)(tt % L.NQ);
      double ux, uy;
      exact_velocity(mms, (n + T->tnode[a]) * L.dt, (node % L.n2) * 0.5 * L.h,
                     (node / L.n2) * 0.5 * L.h, ux, uy);
      v = comp == 0 ? ux : uy;
    }
  } else {
    v = U[(L.po + (row - 2 * nn)) * nt + tt];
  }
  full[e] = v;
}


// ---- heat equation ------------------------------------------------------------
// Slab blocks of the heat equation (Sec. 2, eq. heatfem): per spatial nonzero
// (r, c), M_rc and K_rc are summed over the cells that hold both nodes, in
// the fixed order of the node's cell slots (deterministic, no atomics), from
// the P_k basis at the 25 quadrature points; then every slab's block
// T (x) M + dt W (x) K is written, and Mv = M.  One thread per row.
__global__ __launch_bounds__(256) void k_heat_operator(LevelView L, const RefTables* __restrict__ T,
                                                       double* __restrict__ Jv, double* __restrict__ Mv,
                                                       double* __restrict__ Kv) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= L.nf) return;
  const int nloc = L.nloc, NQ = T->NQ, N = L.N;
  for (int k = L.row_ptr[r]; k < L.row_ptr[r + 1]; ++k) {
    const int c = L.col[k];
    double m = 0.0, st = 0.0;
    for (int e = L.node_cell_ptr[r]; e < L.node_cell_ptr[r + 1]; ++e) {
      const int slot = L.node_cell[e], cell = slot / nloc, i = slot % nloc;
      const int* cd = L.cell_dofs + (int64_t)cell * nloc;
      int j = -1;
      for (int t = 0; t < nloc; ++t)
        if (cd[t] == c) j = t;
      if (j < 0) continue;
      const int* cv = L.cells + 3 * cell;
      double px[3], py[3];
      for (int t = 0; t < 3; ++t) {
        px[t] = (cv[t] % L.n1) * L.h;
        py[t] = (cv[t] / L.n1) * L.h;
      }
      const double j00 = px[1] - px[0], j01 = px[2] - px[0], j10 = py[1] - py[0], j11 = py[2] - py[0];
      const double det = j00 * j11 - j01 * j10, ad = fabs(det), id = 1.0 / det;
      double me = 0.0, ke = 0.0;
      for (int q = 0; q < kQx; ++q) {
        const double w = T->wq[q] * ad;
        const double* gi = T->dNk[q][i];
        const double* gj = T->dNk[q][j];
        const double ix = (j11 * gi[0] - j10 * gi[1]) * id, iy = (-j01 * gi[0] + j00 * gi[1]) * id;
        const double jx = (j11 * gj[0] - j10 * gj[1]) * id, jy = (-j01 * gj[0] + j00 * gj[1]) * id;
        me += w * T->Nk[q][i] * T->Nk[q][j];
        ke += w * (ix * jx + iy * jy);
      }
      m += me;
      st += ke;
    }
    Mv[k] = m;
    Kv[k] = st;
    double* out = Jv + (int64_t)k * N * NQ * NQ;
    for (int n = 0; n < N; ++n)
      for (int a = 0; a < NQ; ++a)
        for (int b = 0; b < NQ; ++b) out[(n * NQ + a) * NQ + b] = T->T[a][b] * m + L.dt * T->W[a][b] * st;
  }
}

// y = A x (or b - A x) of the heat equation, one thread per (row, slab):
// the spatial products M x_n and K x_n per temporal node, then the slab's
// temporal matrices, minus the jump coupling to slab n-1 (the path for more
// than 256 slabs; k_heat_spmv_rows below takes the others)
template <int NQ>
__global__ __launch_bounds__(256) void k_heat_spmv(LevelView L, const RefTables* __restrict__ T,
                                                   const double* __restrict__ Mv,
                                                   const double* __restrict__ Kv,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int N = L.N;
  if (t >= (int64_t)L.nf * N) return;
  const int i = (int)(t / N), n = (int)(t % N);
  double mx[NQ], kx[NQ];
  for (int a = 0; a < NQ; ++a) mx[a] = kx[a] = 0.0;
  double jump = 0.0;
  for (int k = L.row_ptr[i]; k < L.row_ptr[i + 1]; ++k) {
    const double* xv = x + ((int64_t)L.col[k] * N + n) * NQ;
    const double m = Mv[k], st = Kv[k];
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      mx[a] += m * xv[a];
      kx[a] += st * xv[a];
    }
    if (n > 0) {
      double xl = 0.0;
#pragma unroll
      for (int a = 0; a < NQ; ++a) xl += T->e1[a] * xv[a - NQ];
      jump += m * xl;
    }
  }
  for (int a = 0; a < NQ; ++a) {
    double out = -T->e0[a] * jump;
#pragma unroll
    for (int c = 0; c < NQ; ++c) out += T->T[a][c] * mx[c] + L.dt * T->W[a][c] * kx[c];
    y[t * NQ + a] = b ? b[t * NQ + a] - out : out;
  }
}

// The same operator over whole rows: a workgroup takes R = 256 / N rows and
// every slab of each (thread r N + n), stages the rows' CSR entries in LDS
// (when they fit), and forms per (row, slab) the mass and stiffness products
// of the slab's nodal values.  The jump coupling of slab n needs
// sum_k M_ik (e1 . x_{n-1}(col k)) = e1 . (M x)_{n-1}, the previous slab's
// mass product, which the neighbouring thread of the same row holds: x is
// read once per CSR entry, and the entries once per workgroup.
constexpr int kHeatStage = 768;   // staged CSR entries per workgroup (15 KB)

template <int NQ>
__global__ __launch_bounds__(256) void k_heat_spmv_rows(LevelView L, const RefTables* __restrict__ T,
                                                        const double* __restrict__ Mv,
                                                        const double* __restrict__ Kv,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ y) {
  __shared__ int s_col[kHeatStage];
  __shared__ double s_m[kHeatStage], s_k[kHeatStage];
  __shared__ double s_end[256];
  const int N = L.N, R = 256 / N, tid = threadIdx.x;
  const int i0 = blockIdx.x * R, i1 = i0 + R < L.nf ? i0 + R : L.nf;
  const int k0 = L.row_ptr[i0], nk = L.row_ptr[i1] - k0;
  const bool staged = nk <= kHeatStage;   // uniform over the workgroup
  if (staged) {
    for (int e = tid; e < nk; e += 256) {
      s_col[e] = L.col[k0 + e];
      s_m[e] = Mv[k0 + e];
      s_k[e] = Kv[k0 + e];
    }
  }
  __syncthreads();
  const int r = tid / N, n = tid % N, i = i0 + r;
  const bool active = r < R && i < L.nf;
  double mx[NQ], kx[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) mx[a] = kx[a] = 0.0;
  auto entry = [&](int c, double m, double st) {
    const double* xv = x + ((int64_t)c * N + n) * NQ;
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      mx[a] += m * xv[a];
      kx[a] += st * xv[a];
    }
  };
  if (active) {
    const int ka = L.row_ptr[i], kb = L.row_ptr[i + 1];
    if (staged) {
#pragma unroll 4
      for (int k = ka - k0; k < kb - k0; ++k) entry(s_col[k], s_m[k], s_k[k]);
    } else {
      for (int k = ka; k < kb; ++k) entry(L.col[k], Mv[k], Kv[k]);
    }
  }
  double e = 0.0;
#pragma unroll
  for (int a = 0; a < NQ; ++a) e += T->e1[a] * mx[a];
  s_end[tid] = e;
  __syncthreads();
  if (!active) return;
  const double jump = n > 0 ? s_end[tid - 1] : 0.0;
  const int64_t t = (int64_t)i * N + n;
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    double out = -T->e0[a] * jump;
#pragma unroll
    for (int c = 0; c < NQ; ++c) out += T->T[a][c] * mx[c] + L.dt * T->W[a][c] * kx[c];
    y[t * NQ + a] = b ? b[t * NQ + a] - out : out;
  }
}

__device__ inline double heat_u0(double x, double y) { return sin(M_PI * x) + cos(2.0 * M_PI * y); }

// b0 = e0 (x) (M U_0) on slab 0, zero elsewhere; one thread per (row, slab)
__global__ __launch_bounds__(256) void k_heat_rhs(LevelView L, const RefTables* __restrict__ T,
                                                  const double* __restrict__ Mv, double* __restrict__ b0) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)L.nf * L.N) return;
  const int i = (int)(t / L.N), n = (int)(t % L.N);
  const int NQ = T->NQ;
  double s = 0.0;
  if (n == 0) {
    const double hs = L.h / L.kdeg;
    for (int k = L.row_ptr[i]; k < L.row_ptr[i + 1]; ++k) {
      const int c = L.col[k];
      s += Mv[k] * heat_u0((c % L.n2) * hs, (c / L.n2) * hs);
    }
  }
  for (int a = 0; a < NQ; ++a) b0[t * NQ + a] = n == 0 ? T->e0[a] * s : 0.0;
}

// ---- Taylor-Hood P3-P2 ------------------------------------------------------------
// The same space-time forms for the general Taylor-Hood level (thk = k = 2):
// velocity of degree k+1 with NLV lattice nodes per cell (basis T->Nk /
// T->dNk), pressure of degree k with NLP nodes (basis T->Nq), both in
// lattice order; cell_dofs holds [x DoFs of the velocity nodes, y DoFs,
// pressure DoFs].  One 64-lane workgroup per (cell, slab), slab fastest, FP64
// atomics into the operator as for P2-P1.
template <int NQ, int NLV>
struct ThStage {
  double ul[2][NLV][NQ];
  double gN[kQx][NLV][2];
  double wdet[kQx];
  double xp[kQx][2];
  double uq[kMaxG][kQx][2];
  double gq[kMaxG][kQx][2][2];
};

// coordinates of velocity lattice node g (spacing h / (k + 1))
__device__ inline void th_vnode_xy(const LevelView& L, int g, double& x, double& y) {
  const double hv = L.h / (L.thk + 1);
  x = (g % L.n2) * hv;
  y = (g / L.n2) * hv;
}

template <int NQ, int NLV>
__device__ void th_stage(const LevelView& L, const RefTables* __restrict__ T, const MmsDev& mms,
                         const double* __restrict__ U, int c, int n, ThStage<NQ, NLV>& S) {
  const int tid = threadIdx.x;
  __shared__ double inv_s[4], adet_s, v0_s[2], J_s[4];
  if (tid == 0) {
    double inv[4], adet, v0[2], Jc[4];
    cell_geometry(L, c, inv, adet, v0, Jc);
    for (int k = 0; k < 4; ++k) { inv_s[k] = inv[k]; J_s[k] = Jc[k]; }
    adet_s = adet;
    v0_s[0] = v0[0]; v0_s[1] = v0[1];
  }
  for (int e = tid; e < 2 * NLV * NQ; e += 64) {
    const int comp = e / (NLV * NQ), i = (e / NQ) % NLV, a = e % NQ;
    const int node = L.cell_vn[NLV * c + i];
    const int k = L.node_free[node];
    double v;
    if (k >= 0) {
      v = U[((int64_t)(2 * k + comp) * L.N + n) * NQ + a];
    } else {
      double x, y, ux, uy;
      th_vnode_xy(L, node, x, y);
      exact_velocity(mms, (n + T->tnode[a]) * L.dt, x, y, ux, uy);
      v = comp == 0 ? ux : uy;
    }
    S.ul[comp][i][a] = v;
  }
  __syncthreads();
  for (int e = tid; e < kQx * NLV; e += 64) {
    const int x = e / NLV, i = e % NLV;
    for (int k = 0; k < 2; ++k)
      S.gN[x][i][k] = T->dNk[x][i][0] * inv_s[0 * 2 + k] + T->dNk[x][i][1] * inv_s[1 * 2 + k];
  }
  if (tid < kQx) {
    S.wdet[tid] = T->wq[tid] * adet_s;
    S.xp[tid][0] = v0_s[0] + J_s[0] * T->xq[tid][0] + J_s[1] * T->xq[tid][1];
    S.xp[tid][1] = v0_s[1] + J_s[2] * T->xq[tid][0] + J_s[3] * T->xq[tid][1];
  }
  __syncthreads();
  const int G = T->G;
  for (int e = tid; e < G * kQx; e += 64) {
    const int g = e / kQx, x = e % kQx;
    for (int comp = 0; comp < 2; ++comp) {
      double u = 0.0, gx = 0.0, gy = 0.0;
      for (int i = 0; i < NLV; ++i) {
        double ui = 0.0;
        for (int b = 0; b < NQ; ++b) ui += T->Phi[g][b] * S.ul[comp][i][b];
        u += ui * T->Nk[x][i];
        gx += ui * S.gN[x][i][0];
        gy += ui * S.gN[x][i][1];
      }
      S.uq[g][x][comp] = u;
      S.gq[g][x][comp][0] = gx;
      S.gq[g][x][comp][1] = gy;
    }
  }
  __syncthreads();
}

template <int NQ, int NLV, int NLP>
__global__ __launch_bounds__(64) void k_th_jacobian(LevelView L, const RefTables* __restrict__ T,
                                                    MmsDev mms, const double* __restrict__ U,
                                                    double* __restrict__ Jv, double* __restrict__ Mv) {
  constexpr int NL = 2 * NLV + NLP;
  const int c = cell_of(L), n = blockIdx.x % L.N, tid = threadIdx.x;
  __shared__ ThStage<NQ, NLV> S;
  th_stage<NQ, NLV>(L, T, mms, U, c, n, S);
  constexpr int G = NQ + 2;
  const double dt = L.dt, R = mms.reynolds;
  const int* nzc = L.cell_nz + (int64_t)NL * NL * c;
  for (int e = tid; e < NLV * NLV + NLP * NLV; e += 64) {
    if (e < NLV * NLV) {
      const int i = e / NLV, j = e % NLV;
      double Mij = 0.0, Kij = 0.0;
      double c1[G], c2[G][2][2];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        c1[g] = 0.0;
        c2[g][0][0] = c2[g][0][1] = c2[g][1][0] = c2[g][1][1] = 0.0;
      }
#pragma unroll 1
      for (int x = 0; x < kQx; ++x) {
        const double w = S.wdet[x], Ni = T->Nk[x][i], Nj = T->Nk[x][j];
        Mij += w * Ni * Nj;
        Kij += w * (S.gN[x][i][0] * S.gN[x][j][0] + S.gN[x][i][1] * S.gN[x][j][1]);
#pragma unroll
        for (int g = 0; g < G; ++g) {
          c1[g] += w * Ni * (S.uq[g][x][0] * S.gN[x][j][0] + S.uq[g][x][1] * S.gN[x][j][1]);
          const double wnn = w * Ni * Nj;
          for (int ci = 0; ci < 2; ++ci)
            for (int cj = 0; cj < 2; ++cj) c2[g][ci][cj] += wnn * S.gq[g][x][ci][cj];
        }
      }
      for (int a = 0; a < NQ; ++a)
        for (int b = 0; b < NQ; ++b) {
          double C1 = 0.0, C2[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const double cw = T->wg[g] * T->Phi[g][a] * T->Phi[g][b];
            C1 += cw * c1[g];
            for (int ci = 0; ci < 2; ++ci)
              for (int cj = 0; cj < 2; ++cj) C2[ci][cj] += cw * c2[g][ci][cj];
          }
          const double diag = T->T[a][b] * Mij + dt * T->W[a][b] * Kij + dt * R * C1;
          for (int ci = 0; ci < 2; ++ci)
            for (int cj = 0; cj < 2; ++cj) {
              const int nz = nzc[NL * (NLV * ci + i) + NLV * cj + j];
              if (nz < 0) continue;
              const double v = dt * R * C2[ci][cj] + (ci == cj ? diag : 0.0);
              scatter_add(L, &Jv[(((int64_t)nz * L.N + n) * NQ + a) * NQ + b], v);
            }
        }
      if (n == 0) {
        for (int ci = 0; ci < 2; ++ci) {
          const int nz = nzc[NL * (NLV * ci + i) + NLV * ci + j];
          if (nz >= 0) scatter_add(L, &Mv[nz], Mij);
        }
      }
    } else {
      const int t = e - NLV * NLV, j = t / NLV, i = t % NLV;   // pressure node j, velocity node i
      double B[2] = {0.0, 0.0};
      for (int x = 0; x < kQx; ++x) {
        const double w = S.wdet[x] * T->Nq[x][j];
        B[0] += w * S.gN[x][i][0];
        B[1] += w * S.gN[x][i][1];
      }
      for (int a = 0; a < NQ; ++a)
        for (int b = 0; b < NQ; ++b)
          for (int ci = 0; ci < 2; ++ci) {
            const double v = -dt * T->W[a][b] * B[ci];
            const int nz1 = nzc[NL * (NLV * ci + i) + 2 * NLV + j];
            if (nz1 >= 0) scatter_add(L, &Jv[(((int64_t)nz1 * L.N + n) * NQ + a) * NQ + b], v);
            const int nz2 = nzc[NL * (2 * NLV + j) + NLV * ci + i];
            if (nz2 >= 0) scatter_add(L, &Jv[(((int64_t)nz2 * L.N + n) * NQ + a) * NQ + b], v);
          }
    }
  }
}

template <int NQ, int NLV, int NLP>
__global__ __launch_bounds__(64) void k_th_residual(LevelView L, const RefTables* __restrict__ T,
                                                    MmsDev mms, const double* __restrict__ U,
                                                    double* __restrict__ F) {
  const int c = cell_of(L), n = blockIdx.x % L.N, tid = threadIdx.x;
  __shared__ ThStage<NQ, NLV> S;
  __shared__ double pl[NLP][NQ];
  __shared__ double prev[2][NLV];
  // the weighted point values, their spatial sums against each basis
  // function and then the temporal sums, as in k_residual
  __shared__ double Av[kMaxG][kQx][2], Bv[kMaxG][kQx][2][2], Dv[kMaxG][kQx];
  __shared__ double jq[kQx][2];   // U(s=0) - U_{n-1}(1) at the quadrature points
  __shared__ double Pv[kMaxG][2][NLV], Jm[2][NLV], Qv[kMaxG][NLP];
  th_stage<NQ, NLV>(L, T, mms, U, c, n, S);
  const int G = T->G;
  for (int e = tid; e < NLP * NQ; e += 64) {
    const int j = e / NQ, a = e % NQ;
    pl[j][a] = U[((int64_t)(L.po + L.cell_pn[NLP * c + j]) * L.N + n) * NQ + a];
  }
  for (int e = tid; e < 2 * NLV; e += 64) {
    const int comp = e / NLV, i = e % NLV;
    const int node = L.cell_vn[NLV * c + i];
    const int k = L.node_free[node];
    double x, y;
    th_vnode_xy(L, node, x, y);
    double v = 0.0;
    if (n == 0) {
      double ux, uy;
      initial_velocity(mms, x, y, ux, uy);
      v = comp == 0 ? ux : uy;
    } else {
      for (int b = 0; b < NQ; ++b) {
        double vb;
        if (k >= 0) {
          vb = U[((int64_t)(2 * k + comp) * L.N + n - 1) * NQ + b];
        } else {
          double ux, uy;
          exact_velocity(mms, (n - 1 + T->tnode[b]) * L.dt, x, y, ux, uy);
          vb = comp == 0 ? ux : uy;
        }
        v += T->e1[b] * vb;
      }
    }
    prev[comp][i] = v;
  }
  __syncthreads();
  const double dt = L.dt, R = mms.reynolds;
  for (int e = tid; e < G * kQx; e += 64) {
    const int g = e / kQx, x = e % kQx;
    double p = 0.0;
    for (int j = 0; j < NLP; ++j) {
      double pj = 0.0;
      for (int b = 0; b < NQ; ++b) pj += T->Phi[g][b] * pl[j][b];
      p += pj * T->Nq[x][j];
    }
    double f[2];
    forcing(mms, (n + T->sg[g]) * L.dt, S.xp[x][0], S.xp[x][1], f[0], f[1]);
    const double w = S.wdet[x];
    for (int comp = 0; comp < 2; ++comp) {
      double d = 0.0;
      for (int i = 0; i < NLV; ++i) {
        double ui = 0.0;
        for (int b = 0; b < NQ; ++b) ui += T->dPhi[g][b] * S.ul[comp][i][b];
        d += ui * T->Nk[x][i];
      }
      const double conv = S.uq[g][x][0] * S.gq[g][x][comp][0] + S.uq[g][x][1] * S.gq[g][x][comp][1];
      Av[g][x][comp] = w * (d + dt * (R * conv - f[comp]));
      Bv[g][x][comp][0] = w * dt * (S.gq[g][x][comp][0] - (comp == 0 ? p : 0.0));
      Bv[g][x][comp][1] = w * dt * (S.gq[g][x][comp][1] - (comp == 1 ? p : 0.0));
    }
    Dv[g][x] = w * (S.gq[g][x][0][0] + S.gq[g][x][1][1]);
  }
  if (tid < kQx) {
    for (int comp = 0; comp < 2; ++comp) {
      double u0 = 0.0, up = 0.0;
      for (int i = 0; i < NLV; ++i) {
        double ui = 0.0;
        for (int b = 0; b < NQ; ++b) ui += T->e0[b] * S.ul[comp][i][b];
        u0 += ui * T->Nk[tid][i];
        up += prev[comp][i] * T->Nk[tid][i];
      }
      jq[tid][comp] = u0 - up;
    }
  }
  __syncthreads();
  const int NP = G * 2 * NLV, NJ = 2 * NLV, NQS = G * NLP;
  for (int e = tid; e < NP + NJ + NQS; e += 64) {
    double acc = 0.0;
    if (e < NP) {
      const int g = e / (2 * NLV), comp = (e / NLV) % 2, i = e % NLV;
      for (int x = 0; x < kQx; ++x)
        acc += Av[g][x][comp] * T->Nk[x][i] + Bv[g][x][comp][0] * S.gN[x][i][0] + Bv[g][x][comp][1] * S.gN[x][i][1];
      Pv[g][comp][i] = acc;
    } else if (e < NP + NJ) {
      const int comp = (e - NP) / NLV, i = (e - NP) % NLV;
      for (int x = 0; x < kQx; ++x) acc += S.wdet[x] * jq[x][comp] * T->Nk[x][i];
      Jm[comp][i] = acc;
    } else {
      const int g = (e - NP - NJ) / NLP, j = (e - NP - NJ) % NLP;
      for (int x = 0; x < kQx; ++x) acc += Dv[g][x] * T->Nq[x][j];
      Qv[g][j] = acc;
    }
  }
  __syncthreads();
  constexpr int NL = 2 * NLV + NLP;
  for (int e = tid; e < NL * NQ; e += 64) {
    double acc = 0.0;
    if (e < 2 * NLV * NQ) {
      const int comp = e / (NLV * NQ), i = (e / NQ) % NLV, a = e % NQ;
      for (int g = 0; g < G; ++g) acc += T->wg[g] * T->Phi[g][a] * Pv[g][comp][i];
      acc += T->e0[a] * Jm[comp][i];
      const int dof = L.cell_dofs[NL * c + NLV * comp + i];
      if (dof >= 0) scatter_add(L, &F[((int64_t)dof * L.N + n) * NQ + a], acc);
    } else {
      const int t = e - 2 * NLV * NQ, j = t / NQ, a = t % NQ;
      for (int g = 0; g < G; ++g) acc += T->wg[g] * T->Phi[g][a] * Qv[g][j];
      const int dof = L.po + L.cell_pn[NLP * c + j];
      scatter_add(L, &F[((int64_t)dof * L.N + n) * NQ + a], -dt * acc);
    }
  }
}

// Space-time velocity L2 error of the P3 velocity (as k_velocity_error).
template <int NQ, int NLV>
__global__ __launch_bounds__(64) void k_th_velocity_error(LevelView L, const RefTables* __restrict__ T,
                                                          MmsDev mms, const double* __restrict__ U,
                                                          double* __restrict__ part) {
  const int c = blockIdx.x, n = blockIdx.y, tid = threadIdx.x;
  __shared__ ThStage<NQ, NLV> S;
  __shared__ double red[64];
  th_stage<NQ, NLV>(L, T, mms, U, c, n, S);
  double acc = 0.0;
  for (int e = tid; e < T->G * kQx; e += 64) {
    const int g = e / kQx, x = e % kQx;
    double ux, uy;
    exact_velocity(mms, (n + T->sg[g]) * L.dt, S.xp[x][0], S.xp[x][1], ux, uy);
    const double dx = ux - S.uq[g][x][0], dy = uy - S.uq[g][x][1];
    acc += T->wg[g] * S.wdet[x] * (dx * dx + dy * dy);
  }
  red[tid] = acc;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) part[(int64_t)n * L.nc + c] = L.dt * red[0];
}

}  // namespace

hipError_t launch_heat_operator(const LevelView& L, const RefTables* tab, double* Jv, double* Mv,
                                double* Kv, hipStream_t s) {
  hipLaunchKernelGGL(k_heat_operator, dim3((unsigned)((L.nf + 255) / 256)), dim3(256), 0, s, L, tab, Jv, Mv, Kv);
  return hipGetLastError();
}

hipError_t launch_heat_spmv(const LevelView& L, const RefTables* tab, const double* Mv,
                            const double* Kv, const double* x, const double* b, double* y,
                            hipStream_t s) {
  if (L.N <= 256) {
    const int R = 256 / L.N;
    const dim3 grid((unsigned)((L.nf + R - 1) / R));
    switch (L.NQ) {
      case 1: hipLaunchKernelGGL(k_heat_spmv_rows<1>, grid, dim3(256), 0, s, L, tab, Mv, Kv, x, b, y); break;
      case 2: hipLaunchKernelGGL(k_heat_spmv_rows<2>, grid, dim3(256), 0, s, L, tab, Mv, Kv, x, b, y); break;
      case 3: hipLaunchKernelGGL(k_heat_spmv_rows<3>, grid, dim3(256), 0, s, L, tab, Mv, Kv, x, b, y); break;
      case 4: hipLaunchKernelGGL(k_heat_spmv_rows<4>, grid, dim3(256), 0, s, L, tab, Mv, Kv, x, b, y); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const dim3 grid((unsigned)(((int64_t)L.nf * L.N + 255) / 256));
  switch (L.NQ) {
    case 1: hipLaunchKernelGGL(k_heat_spmv<1>, grid, dim3(256), 0, s, L, tab, Mv, Kv, x, b, y); break;
    case 2: hipLaunchKernelGGL(k_heat_spmv<2>, grid, dim3(256), 0, s, L, tab, Mv, Kv, x, b, y); break;
    case 3: hipLaunchKernelGGL(k_heat_spmv<3>, grid, dim3(256), 0, s, L, tab, Mv, Kv, x, b, y); break;
    case 4: hipLaunchKernelGGL(k_heat_spmv<4>, grid, dim3(256), 0, s, L, tab, Mv, Kv, x, b, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_heat_rhs(const LevelView& L, const RefTables* tab, const double* Mv, double* b0,
                           hipStream_t s) {
  const int64_t n = (int64_t)L.nf * L.N;
  hipLaunchKernelGGL(k_heat_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L, tab, Mv, b0);
  return hipGetLastError();
}

hipError_t launch_velocity_error(const LevelView& L, const RefTables* tab, MmsDev mms,
                                 const double* U, double* part, double* out, hipStream_t s) {
  dim3 grid(L.nc, L.N);
  if (L.thk == kThK) {
    if (L.NQ == 1) hipLaunchKernelGGL((k_th_velocity_error<1, kThNlv>), grid, dim3(64), 0, s, L, tab, mms, U, part);
    else hipLaunchKernelGGL((k_th_velocity_error<2, kThNlv>), grid, dim3(64), 0, s, L, tab, mms, U, part);
  } else if (L.NQ == 1) {
    hipLaunchKernelGGL(k_velocity_error<1>, grid, dim3(64), 0, s, L, tab, mms, U, part);
  } else {
    hipLaunchKernelGGL(k_velocity_error<2>, grid, dim3(64), 0, s, L, tab, mms, U, part);
  }
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, (int64_t)L.nc * L.N, part, out);
  return hipGetLastError();
}

hipError_t launch_expand(const LevelView& L, const RefTables* tab, MmsDev mms, const double* U,
                         double* full, hipStream_t s) {
  const int64_t n = ((int64_t)2 * L.n2 * L.n2 + (int64_t)L.n1 * L.n1) * L.N * L.NQ;
  hipLaunchKernelGGL(k_expand, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L, tab, mms, U, full);
  return hipGetLastError();
}

// One launch per colour (color_ptr: 9 offsets into L.color_cells), in
// colour order.
template <typename F>
static hipError_t by_colour(const LevelView& L, const int* color_ptr, F launch) {
  for (int k = 0; k < 8; ++k) {
    const int cnt = color_ptr[k + 1] - color_ptr[k];
    if (cnt == 0) continue;
    LevelView Lc = L;
    Lc.color_first = color_ptr[k];
    launch(Lc, dim3((unsigned)((int64_t)cnt * L.N)));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_assemble_jacobian(const LevelView& L, const RefTables* tab, MmsDev mms,
                                    const double* U, double* Jv, double* Mv, const int* color_ptr,
                                    hipStream_t s) {
  return by_colour(L, color_ptr, [&](const LevelView& Lc, dim3 grid) {
    if (L.thk == kThK) {
      if (L.NQ == 1) hipLaunchKernelGGL((k_th_jacobian<1, kThNlv, kThNlp>), grid, dim3(64), 0, s, Lc, tab, mms, U, Jv, Mv);
      else hipLaunchKernelGGL((k_th_jacobian<2, kThNlv, kThNlp>), grid, dim3(64), 0, s, Lc, tab, mms, U, Jv, Mv);
    } else if (L.NQ == 1) {
      hipLaunchKernelGGL(k_jacobian<1>, grid, dim3(64), 0, s, Lc, tab, mms, U, Jv, Mv);
    } else {
      hipLaunchKernelGGL(k_jacobian<2>, grid, dim3(64), 0, s, Lc, tab, mms, U, Jv, Mv);
    }
  });
}

hipError_t launch_assemble_residual(const LevelView& L, const RefTables* tab, MmsDev mms,
                                    const double* U, double* F, const int* color_ptr, hipStream_t s) {
  return by_colour(L, color_ptr, [&](const LevelView& Lc, dim3 grid) {
    if (L.thk == kThK) {
      if (L.NQ == 1) hipLaunchKernelGGL((k_th_residual<1, kThNlv, kThNlp>), grid, dim3(64), 0, s, Lc, tab, mms, U, F);
      else hipLaunchKernelGGL((k_th_residual<2, kThNlv, kThNlp>), grid, dim3(64), 0, s, Lc, tab, mms, U, F);
    } else if (L.NQ == 1) {
      hipLaunchKernelGGL(k_residual<1>, grid, dim3(64), 0, s, Lc, tab, mms, U, F);
    } else {
      hipLaunchKernelGGL(k_residual<2>, grid, dim3(64), 0, s, Lc, tab, mms, U, F);
    }
  });
}

}  // namespace stwr
