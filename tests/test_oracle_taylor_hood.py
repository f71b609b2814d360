"""Pins of the Taylor-Hood P_{k+1}-P_k structure (oracle/taylor_hood.py)
against the closed forms of Sec. 3.1, for the P2-P1 discretization the GPU
path implements (k = 1) and the P3-P2 one (k = 2, the paper's second
discretization) and beyond: global DoFs, DoFs and nonzeros of an interior
Vanka+star patch, the vertex-star pressure count, and at k = 1 the patches
of the independent P2-P1 oracle (oracle/mesh.py)."""
import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle.taylor_hood import TaylorHood


def global_dofs(M, k):
    # Sec. 3.1: velocity of degree k + 1 (two components), pressure of degree
    # k, every DoF of the M x M mesh (M_x = M + 1 vertices per side)
    return 3 * M ** 2 * k ** 2 + (4 * M ** 2 + 6 * M) * k + 2 * M ** 2 + 4 * M + 3


def patch_dofs(k):
    return 9 * k ** 2 + 15 * k + 15            # Sec. 3.1, Vanka-star patch


def patch_nnz(k):
    return 12 * k ** 4 + 96 * k ** 3 + 240 * k ** 2 + 252 * k + 128   # Sec. 3.1 / App. A.1


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("M", [2, 3, 5, 8])
def test_global_dof_count(M, k):
    assert TaylorHood(M, k).n_dofs_total() == global_dofs(M, k)


@pytest.mark.parametrize("k,dofs,nnz", [(1, 39, 728), (2, 81, 2552), (3, 141, 6608)])
def test_interior_patch_dofs_and_nonzeros(k, dofs, nnz):
    assert patch_dofs(k) == dofs and patch_nnz(k) == nnz
    th = TaylorHood(6, k)
    for v in [(2, 2), (3, 3), (2, 4), (4, 3)]:   # vertices whose star is away from the boundary
        assert th.patch_dofs(v) == dofs
        assert th.patch_nnz(v) == nnz


@pytest.mark.parametrize("k", [1, 2, 3])
def test_patch_pressure_is_the_vertex_star(k):
    # the pressure part of a Vanka+star patch is the degree-k vertex star:
    # 3k^2 - 3k + 1 nodes (Sec. 3.1, the heat-equation patch count)
    th = TaylorHood(6, k)
    _, pres = th.patch((3, 3))
    assert len(pres) == 3 * k ** 2 - 3 * k + 1


@pytest.mark.parametrize("M", [3, 4, 5])
def test_p2p1_patches_match_the_p2p1_oracle(M):
    # k = 1: the same free DoFs as oracle/mesh.py's patches, at every vertex
    # (boundary vertices included, Dirichlet velocity DoFs left out)
    mesh = Mesh(M)
    th = TaylorHood(M, 1)
    ref = mesh.patches()
    n1 = M + 1
    for vid in range(mesh.nv):
        vel, pres = th.patch((vid % n1, vid // n1))
        free = mesh.node_free[vel]
        assert np.all(free >= 0)
        dofs = np.sort(np.concatenate([2 * free, 2 * free + 1, mesh.p_offset + pres]))
        assert np.array_equal(dofs, ref[vid]), vid


def test_boundary_patches_are_smaller():
    th = TaylorHood(6, 2)
    interior = th.patch_dofs((3, 3))
    assert th.patch_dofs((0, 0)) < th.patch_dofs((0, 3)) < interior
    assert th.n_dofs_free() == 2 * (3 * 6 - 1) ** 2 + (2 * 6 + 1) ** 2
