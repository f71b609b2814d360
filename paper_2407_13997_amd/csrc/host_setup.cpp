// Host construction of levels, patches, transfers and reference tables.
#include "host_setup.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace stwr {

// ---------------------------------------------------------------------------
// Quadrature: Gauss-Legendre nodes by Newton iteration on the three-term
// recurrence of the Legendre polynomials, mapped to [0, 1].
void gauss_legendre01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    // ascending order on [0, 1]
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2) P'^2) scaled by 1/2
  }
}

static void p2_eval(double xi, double eta, double* v, double (*g)[2]) {
  const double l[3] = {1.0 - xi - eta, xi, eta};
  const double dl[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
  for (int i = 0; i < 3; ++i) {
    v[i] = l[i] * (2.0 * l[i] - 1.0);
    if (g) for (int k = 0; k < 2; ++k) g[i][k] = (4.0 * l[i] - 1.0) * dl[i][k];
  }
  const int e[3][2] = {{1, 2}, {0, 2}, {0, 1}};
  for (int m = 0; m < 3; ++m) {
    int a = e[m][0], b = e[m][1];
    v[3 + m] = 4.0 * l[a] * l[b];
    if (g) for (int k = 0; k < 2; ++k) g[3 + m][k] = 4.0 * (l[b] * dl[a][k] + l[a] * dl[b][k]);
  }
}

static void p1_eval(double xi, double eta, double* v) {
  v[0] = 1.0 - xi - eta;
  v[1] = xi;
  v[2] = eta;
}

// Legendre P_n(z) by the three-term recurrence
static double legendre(int n, double z) {
  double p0 = 1.0, p1 = z;
  if (n == 0) return p0;
  for (int k = 2; k <= n; ++k) {
    const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  return p1;
}

// Right Gauss-Radau points of [0, 1]: z = 1 and the q roots of
// P_{q+1} - P_q in (-1, 1), mapped by (z + 1) / 2; roots bracketed on a fine
// grid and bisected.
static void radau_right01(int q, double* x) {
  int found = 0;
  const int G = 4000;
  auto f = [&](double z) { return legendre(q + 1, z) - legendre(q, z); };
  double za = -1.0, fa = f(za);
  for (int i = 1; i <= G && found < q; ++i) {
    const double zb = -1.0 + 2.0 * i / (G + 1.0), fb = f(zb);
    if (fa == 0.0 || fa * fb < 0.0) {
      double lo = za, hi = zb, flo = fa;
      for (int it = 0; it < 200 && hi - lo > 1e-16; ++it) {
        const double mid = 0.5 * (lo + hi), fm = f(mid);
        if (flo * fm <= 0.0) hi = mid;
        else { lo = mid; flo = fm; }
      }
      x[found++] = 0.5 * (0.5 * (lo + hi) + 1.0);
    }
    za = zb;
    fa = fb;
  }
  if (found != q) throw std::logic_error("Radau node search failed");
  x[q] = 1.0;
}

void build_ref_tables(int q, int nodes, RefTables& t) {
  if (q < 0 || q > kMaxNQ - 1) throw std::invalid_argument("q must be 0..3");
  if (nodes != 0 && nodes != 1) throw std::invalid_argument("temporal nodes must be 0 or 1");
  double u[5], wu[5];
  gauss_legendre01(5, u, wu);
  int k = 0;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j, ++k) {
      t.xq[k][0] = u[i];
      t.xq[k][1] = u[j] * (1.0 - u[i]);
      t.wq[k] = wu[i] * wu[j] * (1.0 - u[i]);
    }
  const double dl1[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
  for (int x = 0; x < kQx; ++x) {
    p2_eval(t.xq[x][0], t.xq[x][1], t.N2[x], t.dN2[x]);
    p1_eval(t.xq[x][0], t.xq[x][1], t.N1[x]);
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 2; ++d) t.dN1[x][i][d] = dl1[i][d];
  }
  t.NQ = q + 1;
  t.G = q + 3;
  gauss_legendre01(t.G, t.sg, t.wg);
  if (nodes == 0) {
    // right Gauss-Radau nodes of the slab: {1}, {1/3, 1}, ...
    radau_right01(q, t.tnode);
  } else {
    // Gauss-Legendre nodes of the slab
    double w[kMaxNQ];
    gauss_legendre01(q + 1, t.tnode, w);
  }
  auto lag = [&](int a, double s, double* d) {
    double v = 1.0, dv = 0.0;
    for (int b = 0; b < t.NQ; ++b) {
      if (b == a) continue;
      double den = t.tnode[a] - t.tnode[b];
      dv = dv * (s - t.tnode[b]) / den + v / den;
      v *= (s - t.tnode[b]) / den;
    }
    if (d) *d = dv;
    return v;
  };
  for (int g = 0; g < t.G; ++g)
    for (int a = 0; a < t.NQ; ++a) t.Phi[g][a] = lag(a, t.sg[g], &t.dPhi[g][a]);
  for (int a = 0; a < t.NQ; ++a) {
    t.e0[a] = lag(a, 0.0, nullptr);
    t.e1[a] = lag(a, 1.0, nullptr);
  }
  for (int a = 0; a < t.NQ; ++a)
    for (int b = 0; b < t.NQ; ++b) {
      double T = t.e0[a] * t.e0[b], W = 0.0;
      for (int g = 0; g < t.G; ++g) {
        T += t.wg[g] * t.Phi[g][a] * t.dPhi[g][b];
        W += t.wg[g] * t.Phi[g][a] * t.Phi[g][b];
      }
      t.T[a][b] = T;
      t.W[a][b] = W;
    }
}

// f(i) for i in [0, n): independent items split over up to 16 host threads
// (serially below a few thousand items)
template <class F>
static void parallel_for(int n, F&& f) {
  const int hw = (int)std::thread::hardware_concurrency();
  const int T = std::min(std::max(hw, 1), 16);
  if (n < 4096 || T == 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  const int chunk = (n + T - 1) / T;
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t)
    th.emplace_back([&, t]() {
      const int a = t * chunk, b = std::min(n, a + chunk);
      for (int i = a; i < b; ++i) f(i);
    });
  for (auto& x : th) x.join();
}

// CSR pattern of the DoF pairs that share a cell, and each cell's positions
// in it (cell_dofs holds nloc DoFs per cell, -1 for eliminated ones).
static int find_nz(const HostLevel& L, int r, int c) {
  auto b = L.col.begin() + L.row_ptr[r], e = L.col.begin() + L.row_ptr[r + 1];
  auto it = std::lower_bound(b, e, c);
  return (it != e && *it == c) ? int(it - L.col.begin()) : -1;
}

static void csr_from_cells(HostLevel& L) {
  const int nl = L.nloc;
  std::vector<std::vector<int>> rows(L.nf);
  for (int c = 0; c < L.nc; ++c) {
    const int* d = &L.cell_dofs[(size_t)nl * c];
    for (int I = 0; I < nl; ++I) {
      if (d[I] < 0) continue;
      for (int J = 0; J < nl; ++J)
        if (d[J] >= 0) rows[d[I]].push_back(d[J]);
    }
  }
  parallel_for(L.nf, [&](int r) {
    auto& v = rows[r];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  });
  L.row_ptr.assign(L.nf + 1, 0);
  for (int r = 0; r < L.nf; ++r) L.row_ptr[r + 1] = L.row_ptr[r] + (int)rows[r].size();
  L.col.resize(L.row_ptr[L.nf]);
  parallel_for(L.nf, [&](int r) { std::copy(rows[r].begin(), rows[r].end(), L.col.begin() + L.row_ptr[r]); });
  rows.clear();
  rows.shrink_to_fit();
  L.cell_nz.resize((size_t)nl * nl * L.nc);
  parallel_for(L.nc, [&](int c) {
    const int* d = &L.cell_dofs[(size_t)nl * c];
    for (int I = 0; I < nl; ++I)
      for (int J = 0; J < nl; ++J)
        L.cell_nz[(size_t)nl * nl * c + nl * I + J] = (d[I] >= 0 && d[J] >= 0) ? find_nz(L, d[I], d[J]) : -1;
  });
}

// Patch-block CSR positions and the DoF -> patch-slot transpose, from
// patch_ptr / patch_dofs.
static void patch_maps(HostLevel& L) {
  L.patch_nz_off.assign(L.nv + 1, 0);
  for (int v = 0; v < L.nv; ++v) {
    int64_t nb = L.patch_ptr[v + 1] - L.patch_ptr[v];
    L.patch_nz_off[v + 1] = L.patch_nz_off[v] + nb * nb;
  }
  L.patch_nz.resize(L.patch_nz_off[L.nv]);
  parallel_for(L.nv, [&](int v) {
    int s = L.patch_ptr[v], nb = L.patch_ptr[v + 1] - s;
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j)
        L.patch_nz[L.patch_nz_off[v] + (int64_t)i * nb + j] = find_nz(L, L.patch_dofs[s + i], L.patch_dofs[s + j]);
  });
  const int ns = (int)L.patch_dofs.size();
  L.slot_patch.resize(ns);
  for (int v = 0; v < L.nv; ++v)
    for (int s = L.patch_ptr[v]; s < L.patch_ptr[v + 1]; ++s) L.slot_patch[s] = v;
  L.dof_ptr.assign(L.nf + 1, 0);
  for (int s = 0; s < ns; ++s) L.dof_ptr[L.patch_dofs[s] + 1]++;
  for (int r = 0; r < L.nf; ++r) L.dof_ptr[r + 1] += L.dof_ptr[r];
  L.dof_slot.resize(ns);
  std::vector<int> fill(L.dof_ptr.begin(), L.dof_ptr.end() - 1);
  for (int s = 0; s < ns; ++s) L.dof_slot[fill[L.patch_dofs[s]]++] = s;
}

// structured mesh cells: square (i, j) gives (v_ij, v_i+1,j, v_i,j+1) and
// (v_i+1,j+1, v_i,j+1, v_i+1,j)
static void mesh_cells(HostLevel& L) {
  const int M = L.M, n1 = L.n1;
  L.cells.resize(3 * L.nc);
  for (int j = 0; j < M; ++j)
    for (int i = 0; i < M; ++i) {
      int a = i + n1 * j, b = i + 1 + n1 * j, c = i + n1 * (j + 1), d = i + 1 + n1 * (j + 1);
      int c0 = 2 * (i + M * j);
      int tri[2][3] = {{a, b, c}, {d, c, b}};
      for (int s = 0; s < 2; ++s)
        for (int k = 0; k < 3; ++k) L.cells[3 * (c0 + s) + k] = tri[s][k];
    }
  auto colour = [&](int c) { const int sq = c / 2, i = sq % M, j = sq / M; return (i & 1) + 2 * (j & 1) + 4 * (c & 1); };
  for (int k = 0; k < 9; ++k) L.color_ptr[k] = 0;
  for (int c = 0; c < L.nc; ++c) ++L.color_ptr[colour(c) + 1];
  for (int k = 0; k < 8; ++k) L.color_ptr[k + 1] += L.color_ptr[k];
  L.color_cells.assign(L.nc, 0);
  int fill[8];
  for (int k = 0; k < 8; ++k) fill[k] = L.color_ptr[k];
  for (int c = 0; c < L.nc; ++c) L.color_cells[fill[colour(c)]++] = c;
}

// ---------------------------------------------------------------------------
void build_level(int M, HostLevel& L) {
  if (M < 1) throw std::invalid_argument("mesh size must be positive");
  L.kdeg = 0;
  L.nloc = 15;
  L.M = M;
  L.n1 = M + 1;
  L.n2 = 2 * M + 1;
  L.nv = L.n1 * L.n1;
  L.nc = 2 * M * M;
  L.nn = L.n2 * L.n2;
  L.nfn = (L.n2 - 2) * (L.n2 - 2);
  L.po = 2 * L.nfn;
  L.nf = L.po + L.nv;
  const int n1 = L.n1, n2 = L.n2;
  mesh_cells(L);
  L.cell_p2.resize(6 * L.nc);
  auto vnode = [&](int v) { return 2 * (v % n1) + n2 * 2 * (v / n1); };
  for (int c = 0; c < L.nc; ++c) {
    int g[3];
    for (int k = 0; k < 3; ++k) g[k] = vnode(L.cells[3 * c + k]);
    auto mid = [&](int x, int y) {
      return (g[x] % n2 + g[y] % n2) / 2 + n2 * ((g[x] / n2 + g[y] / n2) / 2);
    };
    int* cp = &L.cell_p2[6 * c];
    cp[0] = g[0]; cp[1] = g[1]; cp[2] = g[2];
    cp[3] = mid(1, 2); cp[4] = mid(0, 2); cp[5] = mid(0, 1);
  }
  L.node_free.assign(L.nn, -1);
  for (int gj = 1; gj < n2 - 1; ++gj)
    for (int gi = 1; gi < n2 - 1; ++gi) L.node_free[gi + n2 * gj] = (gi - 1) + (n2 - 2) * (gj - 1);
  L.cell_dofs.resize(15 * L.nc);
  for (int c = 0; c < L.nc; ++c) {
    int* d = &L.cell_dofs[15 * c];
    for (int i = 0; i < 6; ++i) {
      int k = L.node_free[L.cell_p2[6 * c + i]];
      d[i] = k >= 0 ? 2 * k : -1;
      d[6 + i] = k >= 0 ? 2 * k + 1 : -1;
    }
    for (int i = 0; i < 3; ++i) d[12 + i] = L.po + L.cells[3 * c + i];
  }
  csr_from_cells(L);
  // Vanka+star patches: every free velocity DoF on the closure of the vertex
  // star, plus the pressure DoF of the vertex.
  std::vector<std::vector<int>> inc(L.nv);
  for (int c = 0; c < L.nc; ++c)
    for (int k = 0; k < 3; ++k) inc[L.cells[3 * c + k]].push_back(c);
  L.patch_ptr.assign(L.nv + 1, 0);
  L.patch_nbu.assign(L.nv, 0);
  L.patch_dofs.clear();
  for (int v = 0; v < L.nv; ++v) {
    std::vector<int> d;
    for (int c : inc[v])
      for (int i = 0; i < 6; ++i) {
        int k = L.node_free[L.cell_p2[6 * c + i]];
        if (k >= 0) { d.push_back(2 * k); d.push_back(2 * k + 1); }
      }
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    L.patch_nbu[v] = (int)d.size();
    d.push_back(L.po + v);
    L.patch_dofs.insert(L.patch_dofs.end(), d.begin(), d.end());
    L.patch_ptr[v + 1] = (int)L.patch_dofs.size();
  }
  patch_maps(L);
}

// ---------------------------------------------------------------------------
// Nested interpolation: the coarse P2 (P1) function is evaluated at each fine
// free node (vertex); the coarse cell is found from the structured layout.
static void locate(const HostLevel& C, double x, double y, int& cell, double& xi, double& eta) {
  const int M = C.M;
  const double h = 1.0 / M;
  int i = std::min((int)std::floor(x / h), M - 1);
  int j = std::min((int)std::floor(y / h), M - 1);
  double fx = x / h - i, fy = y / h - j;
  if (fx + fy <= 1.0 + 1e-12) {
    cell = 2 * (i + M * j);
    xi = fx; eta = fy;
  } else {
    cell = 2 * (i + M * j) + 1;
    xi = 1.0 - fx; eta = 1.0 - fy;
  }
}

// P by fine rows from per-row (coarse column, value) lists, and R = P^T.
static void transfer_csr(const HostLevel& F, const HostLevel& C,
                         std::vector<std::vector<std::pair<int, double>>>& rows, HostTransfer& T) {
  parallel_for(F.nf, [&](int r) { std::sort(rows[r].begin(), rows[r].end()); });
  T.p_ptr.assign(F.nf + 1, 0);
  for (int r = 0; r < F.nf; ++r) T.p_ptr[r + 1] = T.p_ptr[r] + (int)rows[r].size();
  T.p_col.resize(T.p_ptr[F.nf]);
  T.p_val.resize(T.p_ptr[F.nf]);
  parallel_for(F.nf, [&](int r) {
    int o = T.p_ptr[r];
    for (auto& pr : rows[r]) { T.p_col[o] = pr.first; T.p_val[o] = pr.second; ++o; }
  });
  T.r_ptr.assign(C.nf + 1, 0);
  for (int c : T.p_col) T.r_ptr[c + 1]++;
  for (int r = 0; r < C.nf; ++r) T.r_ptr[r + 1] += T.r_ptr[r];
  T.r_col.resize(T.p_col.size());
  T.r_val.resize(T.p_col.size());
  std::vector<int> fill(T.r_ptr.begin(), T.r_ptr.end() - 1);
  for (int r = 0; r < F.nf; ++r)
    for (int k = T.p_ptr[r]; k < T.p_ptr[r + 1]; ++k) {
      int c = T.p_col[k];
      T.r_col[fill[c]] = r;
      T.r_val[fill[c]] = T.p_val[k];
      fill[c]++;
    }
}

void build_transfer(const HostLevel& F, const HostLevel& C, HostTransfer& T) {
  if (F.M != 2 * C.M) throw std::invalid_argument("transfer needs a factor-2 refinement");
  std::vector<std::vector<std::pair<int, double>>> rows(F.nf);
  const double hf2 = 0.5 / F.M;
  for (int g = 0; g < F.nn; ++g) {
    int k = F.node_free[g];
    if (k < 0) continue;
    double x = (g % F.n2) * hf2, y = (g / F.n2) * hf2;
    int cell; double xi, eta;
    locate(C, x, y, cell, xi, eta);
    double v[6];
    p2_eval(xi, eta, v, nullptr);
    for (int i = 0; i < 6; ++i) {
      if (std::fabs(v[i]) < 1e-14) continue;
      int kc = C.node_free[C.cell_p2[6 * cell + i]];
      if (kc < 0) continue;
      rows[2 * k].push_back({2 * kc, v[i]});
      rows[2 * k + 1].push_back({2 * kc + 1, v[i]});
    }
  }
  const double hf = 1.0 / F.M;
  for (int vf = 0; vf < F.nv; ++vf) {
    double x = (vf % F.n1) * hf, y = (vf / F.n1) * hf;
    int cell; double xi, eta;
    locate(C, x, y, cell, xi, eta);
    double v[3];
    p1_eval(xi, eta, v);
    for (int i = 0; i < 3; ++i) {
      if (std::fabs(v[i]) < 1e-14) continue;
      rows[F.po + vf].push_back({C.po + C.cells[3 * cell + i], v[i]});
    }
  }
  transfer_csr(F, C, rows, T);
  // injection: coarse node (a, b) on the coarse node grid is fine node (2a, 2b)
  T.inject.assign(C.nf, -1);
  for (int g = 0; g < C.nn; ++g) {
    int kc = C.node_free[g];
    if (kc < 0) continue;
    int gf = 2 * (g % C.n2) + F.n2 * 2 * (g / C.n2);
    int kf = F.node_free[gf];
    T.inject[2 * kc] = 2 * kf;
    T.inject[2 * kc + 1] = 2 * kf + 1;
  }
  for (int v = 0; v < C.nv; ++v) {
    int vf = 2 * (v % C.n1) + F.n1 * 2 * (v / C.n1);
    T.inject[C.po + v] = F.po + vf;
  }
}


// ---------------------------------------------------------------------------
// Heat equation: scalar P_k (Sec. 2, Definition of the heat equation).
//
// Basis: for the node (a, b) / k with c = k - a - b, in barycentric
// coordinates (l0, l1, l2) = (1 - xi - eta, xi, eta),
//   phi = F_a(l1) F_b(l2) F_c(l0),  F_n(l) = prod_{i < n} (k l - i) / (i + 1),
// which is one at its node and vanishes at every other lattice node of the
// triangle (some factor k l_j - i is zero there).
static void pk_factor(int k, int n, double l, double& f, double& df) {
  f = 1.0;
  df = 0.0;
  for (int i = 0; i < n; ++i) {
    const double t = (k * l - i) / (i + 1.0), dt = k / (i + 1.0);
    df = df * t + f * dt;
    f *= t;
  }
}

void pk_eval(int k, double xi, double eta, double* v, double (*g)[2]) {
  const double l0 = 1.0 - xi - eta, l1 = xi, l2 = eta;
  int i = 0;
  for (int b = 0; b <= k; ++b)
    for (int a = 0; a + b <= k; ++a, ++i) {
      const int c = k - a - b;
      double f1, d1, f2, d2, f0, d0;
      pk_factor(k, a, l1, f1, d1);
      pk_factor(k, b, l2, f2, d2);
      pk_factor(k, c, l0, f0, d0);
      v[i] = f1 * f2 * f0;
      if (g) {
        // d/dxi: l1' = 1, l0' = -1; d/deta: l2' = 1, l0' = -1
        g[i][0] = d1 * f2 * f0 - f1 * f2 * d0;
        g[i][1] = f1 * d2 * f0 - f1 * f2 * d0;
      }
    }
}

void build_pk_tables(int k, RefTables& t) {
  if (k < 1 || k > kMaxPk) throw std::invalid_argument("spatial degree must be 1, 2 or 3");
  t.kdeg = k;
  t.nloc = (k + 1) * (k + 2) / 2;
  for (int x = 0; x < kQx; ++x) pk_eval(k, t.xq[x][0], t.xq[x][1], t.Nk[x], t.dNk[x]);
}

void build_level_heat(int M, int k, HostLevel& L) {
  if (M < 1) throw std::invalid_argument("mesh size must be positive");
  if (k < 1 || k > kMaxPk) throw std::invalid_argument("spatial degree must be 1, 2 or 3");
  L.kdeg = k;
  L.nloc = (k + 1) * (k + 2) / 2;
  L.M = M;
  L.n1 = M + 1;
  L.n2 = k * M + 1;            // node lattice width
  L.nv = L.n1 * L.n1;
  L.nc = 2 * M * M;
  L.nn = L.n2 * L.n2;
  L.nfn = L.nn;
  L.nf = L.nn;
  L.po = L.nf;                 // no pressure
  const int n1 = L.n1, nl = L.n2, nloc = L.nloc;
  mesh_cells(L);
  L.cell_p2.clear();
  L.node_free.resize(L.nn);
  for (int g = 0; g < L.nn; ++g) L.node_free[g] = g;
  // local node (a, b) of a lower cell with corner vertex (i, j) is lattice
  // node (k i + a, k j + b); of an upper cell with corner (i+1, j+1) it is
  // (k (i+1) - a, k (j+1) - b) (its reference axes point left and down)
  L.cell_dofs.resize((size_t)nloc * L.nc);
  for (int c = 0; c < L.nc; ++c) {
    const int v0 = L.cells[3 * c], vi = v0 % n1, vj = v0 / n1;
    const bool lower = c % 2 == 0;
    int i = 0;
    for (int b = 0; b <= k; ++b)
      for (int a = 0; a + b <= k; ++a, ++i) {
        const int gi = lower ? k * vi + a : k * vi - a;
        const int gj = lower ? k * vj + b : k * vj - b;
        L.cell_dofs[(size_t)nloc * c + i] = gi + nl * gj;
      }
  }
  csr_from_cells(L);
  // node -> (cell, local index) slots, cells in increasing order
  L.node_cell_ptr.assign(L.nn + 1, 0);
  for (int e = 0; e < nloc * L.nc; ++e) L.node_cell_ptr[L.cell_dofs[e] + 1]++;
  for (int g = 0; g < L.nn; ++g) L.node_cell_ptr[g + 1] += L.node_cell_ptr[g];
  L.node_cell.resize((size_t)nloc * L.nc);
  {
    std::vector<int> fill(L.node_cell_ptr.begin(), L.node_cell_ptr.end() - 1);
    for (int e = 0; e < nloc * L.nc; ++e) L.node_cell[fill[L.cell_dofs[e]]++] = e;
  }
  // vertex-star patches: the nodes of each incident cell whose barycentric
  // coordinate for the vertex is positive (the vertex and the interiors of
  // its incident edges and cells); the incident cells are those holding the
  // vertex's lattice node, with the vertex at one of their corners
  std::vector<int> lam_a(nloc), lam_b(nloc);
  {
    int i = 0;
    for (int b = 0; b <= k; ++b)
      for (int a = 0; a + b <= k; ++a, ++i) { lam_a[i] = a; lam_b[i] = b; }
  }
  std::vector<std::vector<int>> pd(L.nv);
  parallel_for(L.nv, [&](int v) {
    const int g = k * (v % n1) + nl * k * (v / n1);
    auto& d = pd[v];
    for (int e = L.node_cell_ptr[g]; e < L.node_cell_ptr[g + 1]; ++e) {
      const int c = L.node_cell[e] / nloc;
      int corner = 0;
      for (int t = 0; t < 3; ++t)
        if (L.cells[3 * c + t] == v) corner = t;
      for (int i = 0; i < nloc; ++i) {
        const int lam[3] = {k - lam_a[i] - lam_b[i], lam_a[i], lam_b[i]};
        if (lam[corner] > 0) d.push_back(L.cell_dofs[(size_t)nloc * c + i]);
      }
    }
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
  });
  L.patch_ptr.assign(L.nv + 1, 0);
  L.patch_nbu.assign(L.nv, 0);
  L.patch_dofs.clear();
  for (int v = 0; v < L.nv; ++v) {
    const auto& d = pd[v];
    if ((int)d.size() > kHeatMaxNb) throw std::logic_error("vertex-star patch larger than its bound");
    L.patch_nbu[v] = (int)d.size();   // every DoF carries the jump coupling
    L.patch_dofs.insert(L.patch_dofs.end(), d.begin(), d.end());
    L.patch_ptr[v + 1] = (int)L.patch_dofs.size();
  }
  patch_maps(L);
}

void build_transfer_heat(const HostLevel& F, const HostLevel& C, HostTransfer& T) {
  if (F.M != 2 * C.M || F.kdeg != C.kdeg || F.kdeg < 1)
    throw std::invalid_argument("heat transfer needs a factor-2 refinement of the same degree");
  const int k = F.kdeg, nloc = C.nloc;
  std::vector<std::vector<std::pair<int, double>>> rows(F.nf);
  const double hs = 1.0 / (F.M * k);
  parallel_for(F.nf, [&](int g) {
    const double x = (g % F.n2) * hs, y = (g / F.n2) * hs;
    int cell; double xi, eta;
    locate(C, x, y, cell, xi, eta);
    double v[kMaxLoc];
    pk_eval(k, xi, eta, v, nullptr);
    for (int i = 0; i < nloc; ++i)
      if (std::fabs(v[i]) >= 1e-14) rows[g].push_back({C.cell_dofs[(size_t)nloc * cell + i], v[i]});
  });
  transfer_csr(F, C, rows, T);
  T.inject.clear();
}

// ---------------------------------------------------------------------------
// Taylor-Hood P_{k+1}-P_k on the same mesh (k = 2, the paper's P3-P2).

void build_th_tables(int k, RefTables& t) {
  if (k < 1 || k + 1 > kMaxPk) throw std::invalid_argument("Taylor-Hood pressure degree must be 1 or 2");
  build_pk_tables(k + 1, t);
  for (int x = 0; x < kQx; ++x) pk_eval(k, t.xq[x][0], t.xq[x][1], t.Nq[x], nullptr);
}

// Lattice nodes of degree K of cell c on a lattice of width nl: node (a, b)
// of the reference triangle (b outer, a inner) is (K i + a, K j + b) for a
// lower cell with corner vertex (i, j) and (K i - a, K j - b) for an upper
// cell with corner vertex (i, j) = (i0 + 1, j0 + 1).
static void cell_lattice(const HostLevel& L, int c, int K, int nl, int* out) {
  const int v0 = L.cells[3 * c], vi = v0 % L.n1, vj = v0 / L.n1;
  const bool lower = c % 2 == 0;
  int i = 0;
  for (int b = 0; b <= K; ++b)
    for (int a = 0; a + b <= K; ++a, ++i) {
      const int gi = lower ? K * vi + a : K * vi - a;
      const int gj = lower ? K * vj + b : K * vj - b;
      out[i] = gi + nl * gj;
    }
}

void build_level_th(int M, int k, HostLevel& L) {
  if (M < 1) throw std::invalid_argument("mesh size must be positive");
  if (k < 2 || k + 1 > kMaxPk) throw std::invalid_argument("the general Taylor-Hood level takes k = 2");
  const int K = k + 1;
  L.kdeg = 0;
  L.thk = k;
  L.nlv = (K + 1) * (K + 2) / 2;
  L.nlp = (k + 1) * (k + 2) / 2;
  L.nloc = 2 * L.nlv + L.nlp;
  L.M = M;
  L.n1 = M + 1;
  L.n2 = K * M + 1;
  L.n3 = k * M + 1;
  L.nv = L.n1 * L.n1;
  L.nc = 2 * M * M;
  L.nn = L.n2 * L.n2;
  L.nfn = (L.n2 - 2) * (L.n2 - 2);
  L.po = 2 * L.nfn;
  L.nf = L.po + L.n3 * L.n3;
  const int n2 = L.n2, nlv = L.nlv, nlp = L.nlp, nloc = L.nloc;
  mesh_cells(L);
  L.cell_p2.clear();
  L.cell_vn.resize((size_t)nlv * L.nc);
  L.cell_pn.resize((size_t)nlp * L.nc);
  for (int c = 0; c < L.nc; ++c) {
    cell_lattice(L, c, K, n2, &L.cell_vn[(size_t)nlv * c]);
    cell_lattice(L, c, k, L.n3, &L.cell_pn[(size_t)nlp * c]);
  }
  L.node_free.assign(L.nn, -1);
  for (int gj = 1; gj < n2 - 1; ++gj)
    for (int gi = 1; gi < n2 - 1; ++gi) L.node_free[gi + n2 * gj] = (gi - 1) + (n2 - 2) * (gj - 1);
  L.cell_dofs.resize((size_t)nloc * L.nc);
  for (int c = 0; c < L.nc; ++c) {
    int* d = &L.cell_dofs[(size_t)nloc * c];
    for (int i = 0; i < nlv; ++i) {
      const int f = L.node_free[L.cell_vn[(size_t)nlv * c + i]];
      d[i] = f >= 0 ? 2 * f : -1;
      d[nlv + i] = f >= 0 ? 2 * f + 1 : -1;
    }
    for (int i = 0; i < nlp; ++i) d[2 * nlv + i] = L.po + L.cell_pn[(size_t)nlp * c + i];
  }
  csr_from_cells(L);
  // barycentric lattice coordinates (c, a, b) of the pressure nodes of a cell
  std::vector<int> lam_a(nlp), lam_b(nlp);
  {
    int i = 0;
    for (int b = 0; b <= k; ++b)
      for (int a = 0; a + b <= k; ++a, ++i) { lam_a[i] = a; lam_b[i] = b; }
  }
  std::vector<std::vector<int>> inc(L.nv);
  for (int c = 0; c < L.nc; ++c)
    for (int t = 0; t < 3; ++t) inc[L.cells[3 * c + t]].push_back(c);
  std::vector<std::vector<int>> pd(L.nv);
  parallel_for(L.nv, [&](int v) {
    auto& d = pd[v];
    for (int c : inc[v]) {
      for (int i = 0; i < nlv; ++i) {
        const int f = L.node_free[L.cell_vn[(size_t)nlv * c + i]];
        if (f >= 0) { d.push_back(2 * f); d.push_back(2 * f + 1); }
      }
      int corner = 0;
      for (int t = 0; t < 3; ++t)
        if (L.cells[3 * c + t] == v) corner = t;
      for (int i = 0; i < nlp; ++i) {
        const int lam[3] = {k - lam_a[i] - lam_b[i], lam_a[i], lam_b[i]};
        if (lam[corner] > 0) d.push_back(L.po + L.cell_pn[(size_t)nlp * c + i]);
      }
    }
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
  });
  L.patch_ptr.assign(L.nv + 1, 0);
  L.patch_nbu.assign(L.nv, 0);
  L.patch_dofs.clear();
  for (int v = 0; v < L.nv; ++v) {
    const auto& d = pd[v];
    if ((int)d.size() > kThMaxNb) throw std::logic_error("Vanka+star patch larger than its bound");
    L.patch_nbu[v] = (int)(std::lower_bound(d.begin(), d.end(), L.po) - d.begin());
    L.patch_dofs.insert(L.patch_dofs.end(), d.begin(), d.end());
    L.patch_ptr[v + 1] = (int)L.patch_dofs.size();
  }
  patch_maps(L);
}

void build_transfer_th(const HostLevel& F, const HostLevel& C, HostTransfer& T) {
  if (F.M != 2 * C.M || F.thk != C.thk || F.thk < 2)
    throw std::invalid_argument("Taylor-Hood transfer needs a factor-2 refinement of the same degree");
  const int k = F.thk, K = k + 1;
  std::vector<std::vector<std::pair<int, double>>> rows(F.nf);
  const double hv = 1.0 / (F.M * K), hp = 1.0 / (F.M * k);
  parallel_for(F.nn, [&](int g) {
    const int kf = F.node_free[g];
    if (kf < 0) return;
    const double x = (g % F.n2) * hv, y = (g / F.n2) * hv;
    int cell; double xi, eta;
    locate(C, x, y, cell, xi, eta);
    double v[kMaxLoc];
    pk_eval(K, xi, eta, v, nullptr);
    for (int i = 0; i < C.nlv; ++i) {
      if (std::fabs(v[i]) < 1e-14) continue;
      const int kc = C.node_free[C.cell_vn[(size_t)C.nlv * cell + i]];
      if (kc < 0) continue;
      rows[2 * kf].push_back({2 * kc, v[i]});
      rows[2 * kf + 1].push_back({2 * kc + 1, v[i]});
    }
  });
  const int np = F.n3 * F.n3;
  parallel_for(np, [&](int g) {
    const double x = (g % F.n3) * hp, y = (g / F.n3) * hp;
    int cell; double xi, eta;
    locate(C, x, y, cell, xi, eta);
    double v[kMaxLoc];
    pk_eval(k, xi, eta, v, nullptr);
    for (int i = 0; i < C.nlp; ++i)
      if (std::fabs(v[i]) >= 1e-14) rows[F.po + g].push_back({C.po + C.cell_pn[(size_t)C.nlp * cell + i], v[i]});
  });
  transfer_csr(F, C, rows, T);
  // injection: coarse lattice node (a, b) is fine lattice node (2a, 2b)
  T.inject.assign(C.nf, -1);
  for (int g = 0; g < C.nn; ++g) {
    const int kc = C.node_free[g];
    if (kc < 0) continue;
    const int kf = F.node_free[2 * (g % C.n2) + F.n2 * 2 * (g / C.n2)];
    T.inject[2 * kc] = 2 * kf;
    T.inject[2 * kc + 1] = 2 * kf + 1;
  }
  for (int g = 0; g < C.n3 * C.n3; ++g)
    T.inject[C.po + g] = F.po + 2 * (g % C.n3) + F.n3 * 2 * (g / C.n3);
}

}  // namespace stwr
