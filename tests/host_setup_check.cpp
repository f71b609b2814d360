// Host-side consistency checks of the level builders (CSR patterns, patch
// maps and their transpose, transfer stencils), for Taylor-Hood P2-P1 and
// the heat equation's P_k; built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "host_setup.h"

using namespace stwr;

static int fails = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                       \
    }                                                                \
  } while (0)

static void check_level(const HostLevel& L) {
  // CSR rows sorted and unique, diagonal present
  for (int r = 0; r < L.nf; ++r) {
    bool diag = false;
    for (int k = L.row_ptr[r]; k < L.row_ptr[r + 1]; ++k) {
      CHECK(L.col[k] >= 0 && L.col[k] < L.nf);
      if (k > L.row_ptr[r]) CHECK(L.col[k] > L.col[k - 1]);
      diag |= L.col[k] == r;
    }
    CHECK(diag);
  }
  // patch maps: every slot's transpose entry points back; a patch pair is
  // either its CSR entry or a structural zero (nodes of the patch that share
  // no cell), and the diagonal is always present
  const int ns = (int)L.patch_dofs.size();
  std::vector<int> seen(ns, 0);
  for (int d = 0; d < L.nf; ++d)
    for (int k = L.dof_ptr[d]; k < L.dof_ptr[d + 1]; ++k) {
      const int s = L.dof_slot[k];
      CHECK(s >= 0 && s < ns && L.patch_dofs[s] == d);
      seen[s]++;
    }
  for (int s = 0; s < ns; ++s) CHECK(seen[s] == 1);
  for (int v = 0; v < L.nv; ++v) {
    const int s0 = L.patch_ptr[v], nb = L.patch_ptr[v + 1] - s0;
    CHECK(nb > 0 && L.patch_nbu[v] <= nb);
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) {
        const int k = L.patch_nz[L.patch_nz_off[v] + (int64_t)i * nb + j];
        CHECK(k == -1 || (k >= L.row_ptr[L.patch_dofs[s0 + i]] && k < L.row_ptr[L.patch_dofs[s0 + i] + 1] &&
                          L.col[k] == L.patch_dofs[s0 + j]));
        if (i == j) CHECK(k >= 0);
      }
  }
}

// deterministic assembly colours: every cell in exactly one colour, and no
// DoF written by two cells of one colour (cell_dofs, nd per cell)
static void check_colours(const HostLevel& L, int nd) {
  CHECK(L.color_ptr[0] == 0 && L.color_ptr[8] == L.nc);
  std::vector<int> seen(L.nc, 0);
  for (int k = 0; k < 8; ++k) {
    CHECK(L.color_ptr[k] <= L.color_ptr[k + 1]);
    std::vector<int> owner(L.nf, -1);
    for (int e = L.color_ptr[k]; e < L.color_ptr[k + 1]; ++e) {
      const int c = L.color_cells[e];
      CHECK(c >= 0 && c < L.nc);
      seen[c]++;
      for (int i = 0; i < nd; ++i) {
        const int d = L.cell_dofs[(size_t)nd * c + i];
        if (d < 0) continue;
        CHECK(owner[d] == -1 || owner[d] == c);
        owner[d] = c;
      }
    }
  }
  for (int c = 0; c < L.nc; ++c) CHECK(seen[c] == 1);
}

static void check_transfer(const HostLevel& F, const HostLevel& C, const HostTransfer& T, bool unit_rows) {
  for (int r = 0; r < F.nf; ++r) {
    double s = 0.0;
    for (int k = T.p_ptr[r]; k < T.p_ptr[r + 1]; ++k) {
      CHECK(T.p_col[k] >= 0 && T.p_col[k] < C.nf);
      s += T.p_val[k];
    }
    if (unit_rows) CHECK(std::fabs(s - 1.0) < 1e-12);
  }
  CHECK(T.r_ptr[C.nf] == T.p_ptr[F.nf]);
}

int main() {
  for (int M : {4, 8}) {
    HostLevel F, C;
    HostTransfer T;
    build_level(M, F);
    build_level(M / 2, C);
    build_transfer(F, C, T);
    check_level(F);
    check_level(C);
    check_colours(F, 15);
    check_colours(C, 15);
    {
      HostLevel Ft;
      build_level_th(M, 2, Ft);
      check_colours(Ft, (int)(Ft.cell_dofs.size() / Ft.nc));
    }
    // velocity rows away from the boundary and pressure rows interpolate constants
    check_transfer(F, C, T, false);
    for (int k = 1; k <= 3; ++k) {
      HostLevel Fh, Ch;
      HostTransfer Th;
      build_level_heat(M, k, Fh);
      build_level_heat(M / 2, k, Ch);
      build_transfer_heat(Fh, Ch, Th);
      check_level(Fh);
      check_transfer(Fh, Ch, Th, true);
      CHECK(Fh.nf == (k * M + 1) * (k * M + 1));
    }
  }
  for (int q = 0; q <= 3; ++q)
    for (int nodes = 0; nodes <= (q <= 3 ? 1 : 0); ++nodes) {
      RefTables t{};
      build_ref_tables(q, nodes, t);
      // T + T^T = e1 e1^T + e0 e0^T (integration by parts on the slab)
      for (int a = 0; a <= q; ++a)
        for (int b = 0; b <= q; ++b)
          CHECK(std::fabs(t.T[a][b] + t.T[b][a] - t.e1[a] * t.e1[b] - t.e0[a] * t.e0[b]) < 1e-12);
    }
  std::printf("host setup checks: %d failures\n", fails);
  return fails ? 1 : 0;
}
