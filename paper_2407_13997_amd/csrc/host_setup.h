// Host-side construction of one space-time level: structured triangle-split
// mesh, Taylor-Hood P2-P1 free-DoF numbering (or the heat equation's P_k
// node lattice), CSR sparsity pattern, cell and patch index maps (Vanka+star
// or vertex-star patches, Sec. 3), nested-grid transfer stencils
// (P = I (x) blockdiag(P_u, P_phi), or I (x) P_k, Sec. 3) and the quadrature
// and temporal reference tables.  Pure C++: no device calls.
#pragma once
#include <cstdint>
#include <vector>

namespace stwr {

constexpr int kQx = 25;       // spatial quadrature points (5x5 collapsed Gauss rule)
constexpr int kMaxG = 6;      // temporal Gauss points (q + 3)
constexpr int kMaxNQ = 4;     // temporal nodes per slab (q <= 3; Navier-Stokes q <= 1)
constexpr int kMaxNb = 39;    // spatial DoFs in a Vanka+star patch (interior)
constexpr int kMaxNbu = 38;   // velocity DoFs in a patch

constexpr int kMaxPk = 3;     // highest spatial degree of the heat equation's P_k
constexpr int kMaxLoc = 10;   // nodes of a P_k cell, (k + 1)(k + 2) / 2
constexpr int kHeatMaxNb = 19;  // DoFs of a P_k vertex-star patch, 3k^2 - 3k + 1 at k = 3
// Taylor-Hood P_{k+1}-P_k with k = 2 (P3-P2): an interior Vanka+star patch
// holds 74 velocity DoFs (37 nodes) and 7 pressure DoFs (Sec. 3.1)
constexpr int kThK = 2;
constexpr int kThMaxNb = 81;
constexpr int kThMaxNbu = 74;
constexpr int kThNlv = 10;    // P3 nodes of a cell
constexpr int kThNlp = 6;     // P2 nodes of a cell

// Reference tables consumed by the assembly kernels (plain doubles so the
// struct can be copied to device memory as is).
struct RefTables {
  double xq[kQx][2];
  double wq[kQx];
  double N2[kQx][6];
  double dN2[kQx][6][2];
  double N1[kQx][3];
  double dN1[kQx][3][2];
  int G;                    // temporal Gauss points
  int NQ;                   // q + 1
  double sg[kMaxG], wg[kMaxG];
  double Phi[kMaxG][kMaxNQ], dPhi[kMaxG][kMaxNQ];
  double e0[kMaxNQ], e1[kMaxNQ], tnode[kMaxNQ];
  double T[kMaxNQ][kMaxNQ];  // int phi_b' phi_a + phi_b(0) phi_a(0)
  double W[kMaxNQ][kMaxNQ];  // int phi_a phi_b
  // heat equation: P_k basis (k = kdeg) at the spatial quadrature points;
  // Taylor-Hood P3-P2: the P3 velocity basis (kdeg = 3)
  int kdeg, nloc;
  double Nk[kQx][kMaxLoc];
  double dNk[kQx][kMaxLoc][2];
  // Taylor-Hood P3-P2: the P2 pressure basis in lattice order
  double Nq[kQx][kMaxLoc];
};

// nodes: 0 right Gauss-Radau, 1 Gauss-Legendre (the slab's Lagrange nodes)
void build_ref_tables(int q, int nodes, RefTables& t);
void gauss_legendre01(int n, double* x, double* w);
// P_k Lagrange basis of the heat equation (1 <= k <= 3) into t.Nk, t.dNk
void build_pk_tables(int k, RefTables& t);
// P_k basis on the reference triangle, equispaced nodes (a, b) / k with
// a + b <= k ordered b outer, a inner: values v[nloc], gradients g[nloc][2]
void pk_eval(int k, double xi, double eta, double* v, double (*g)[2]);
// Taylor-Hood P_{k+1}-P_k bases in lattice order: P_{k+1} into Nk/dNk, P_k into Nq
void build_th_tables(int k, RefTables& t);

// One level of either discretisation.  Navier-Stokes (kdeg = 0): Taylor-Hood
// P2-P1, cell_dofs 15 per cell, Vanka+star patches.  Heat (kdeg = k): scalar
// P_k on the (kM+1)^2 node lattice (n2 = kM+1, every node free, po = nf),
// cell_dofs nloc per cell, cell_nz nloc^2 per cell, vertex-star patches, and
// node_cell_ptr / node_cell = the (cell * nloc + local index) slots of each
// node for the gather-form assembly.
struct HostLevel {
  int kdeg = 0, nloc = 15;
  int M = 0, n1 = 0, n2 = 0;
  int nv = 0, nc = 0, nn = 0;
  int nfn = 0, nf = 0, po = 0;   // free P2 nodes, free DoFs, pressure offset
  std::vector<int> cells;        // nc x 3 vertex ids
  std::vector<int> cell_p2;      // nc x 6 P2 node ids (3 vertices, edges opposite v0, v1, v2)
  std::vector<int> cell_dofs;    // nc x 15: 6 ux, 6 uy, 3 p (-1 = Dirichlet)
  std::vector<int> node_free;    // nn: free node index or -1
  std::vector<int> row_ptr, col; // CSR over free DoFs
  std::vector<int> cell_nz;      // nc x 15 x 15: CSR position or -1
  std::vector<int> patch_ptr;    // nv + 1
  std::vector<int> patch_dofs;   // sum nb, sorted (velocity DoFs, then the vertex pressure)
  std::vector<int> patch_nbu;    // nv: velocity DoFs per patch
  std::vector<int64_t> patch_nz_off;  // nv + 1: offsets into patch_nz (sum nb^2)
  std::vector<int> patch_nz;     // nb x nb CSR positions per patch (-1 = structural zero)
  std::vector<int> dof_ptr;      // nf + 1: transpose map, DoF -> patch slots
  std::vector<int> dof_slot;     // positions in patch_dofs that hold the DoF
  std::vector<int> slot_patch;   // sum nb: patch owning each slot
  std::vector<int> node_cell_ptr, node_cell;   // heat only
  // Taylor-Hood P_{k+1}-P_k built by build_level_th (thk = k >= 2; 0 for the
  // P2-P1 level of build_level): velocity lattice of width n2 = (k+1)M + 1,
  // pressure lattice of width n3 = kM + 1, nlv / nlp lattice nodes per cell in
  // cell_vn / cell_pn, cell_dofs = [x DoFs of the nlv nodes, y DoFs, pressure]
  int thk = 0, n3 = 0, nlv = 0, nlp = 0;
  std::vector<int> cell_vn, cell_pn;
  // the cells in 8 colours, colour (i mod 2) + 2 (j mod 2) + 4 t for triangle
  // t of square (i, j): two cells of one colour are triangles of the same
  // orientation in squares at least two apart in i or in j, so they share no
  // vertex and no DoF.  color_cells lists the cells colour by colour
  // (ascending within a colour); colour k starts at color_ptr[k].
  std::vector<int> color_cells;
  int color_ptr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
};

void build_level(int M, HostLevel& L);
// Taylor-Hood P_{k+1}-P_k level (k = 2): free numbering as for P2-P1 on the
// velocity lattice (interior node (gi, gj) -> (gi-1) + (n2-2)(gj-1), DoFs 2k,
// 2k+1), pressure lattice node g -> 2 (n2-2)^2 + g; Vanka+star patches of
// every vertex: the free velocity DoFs of every node of the star's cells and
// the pressure nodes of the star's cells not on the edges opposite the vertex.
void build_level_th(int M, int k, HostLevel& L);
void build_level_heat(int M, int k, HostLevel& L);

// Prolongation from coarse (M/2) to fine (M) in free-DoF numbering, stored by
// fine rows (P) and by coarse rows (R = P^T).  Injection map: coarse free DoF
// -> fine free DoF at the same node.
struct HostTransfer {
  std::vector<int> p_ptr, p_col;
  std::vector<double> p_val;
  std::vector<int> r_ptr, r_col;
  std::vector<double> r_val;
  std::vector<int> inject;   // coarse nf
};

void build_transfer(const HostLevel& fine, const HostLevel& coarse, HostTransfer& T);
// P_k interpolation of the coarse heat space at the fine lattice nodes (no injection map)
void build_transfer_heat(const HostLevel& fine, const HostLevel& coarse, HostTransfer& T);
// Taylor-Hood P_{k+1}-P_k nested interpolation: each velocity component by
// P_{k+1} interpolation at the fine free nodes, the pressure by P_k, with the
// injection map (every coarse lattice node is a fine one)
void build_transfer_th(const HostLevel& fine, const HostLevel& coarse, HostTransfer& T);

}  // namespace stwr
