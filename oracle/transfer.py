"""Space-time grid transfers (oracle), Sec. 3: P = I (x) P_h with P_h =
blockdiag(P_u, P_phi) the finite-element interpolation from the mesh of size
2h to the mesh of size h, and R = P^T.

P_h is built by evaluating each coarse basis function at the fine nodes (the
coarse P2 and P1 spaces are nested in the fine ones), then keeping the rows of
free fine DoFs and the columns of free coarse DoFs (corrections vanish on the
Dirichlet boundary).  With time innermost in the vector layout, P = kron(P_h, I).
"""
import numpy as np
import scipy.sparse as sp

from . import fe


def _locate(coarse, pts):
    """Coarse cell index and reference coordinates of each point."""
    M, h = coarse.M, coarse.h
    i = np.minimum((pts[:, 0] / h).astype(int), M - 1)
    j = np.minimum((pts[:, 1] / h).astype(int), M - 1)
    fx = pts[:, 0] / h - i
    fy = pts[:, 1] / h - j
    upper = fx + fy > 1.0 + 1e-12
    cell = 2 * (i + M * j) + upper.astype(int)
    v = coarse.vxy[coarse.cells[cell]]
    Jc = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)
    ref = np.linalg.solve(Jc, (pts - v[:, 0])[..., None])[..., 0]
    return cell, ref


def spatial_prolongation(fine, coarse):
    """P_h as CSR (fine.n_free x coarse.n_free) in the free-DoF numbering."""
    rows, cols, vals = [], [], []
    # velocity: fine free nodes
    fnodes = np.nonzero(fine.node_free >= 0)[0]
    cell, ref = _locate(coarse, fine.nxy[fnodes])
    val, _ = fe.p2(ref)
    cn = coarse.cell_p2[cell]                         # (n, 6)
    for comp in range(2):
        r = np.repeat(fine.vel_dof(fnodes, comp)[:, None], 6, axis=1)
        c = coarse.vel_dof(cn, comp)
        ok = (c >= 0) & (np.abs(val) > 1e-14)
        rows.append(r[ok]); cols.append(c[ok]); vals.append(val[ok])
    # pressure: all fine vertices
    fv = np.arange(fine.nv)
    cell, ref = _locate(coarse, fine.vxy)
    val, _ = fe.p1(ref)
    r = np.repeat(fine.p_dof(fv)[:, None], 3, axis=1)
    c = coarse.p_dof(coarse.cells[cell])
    ok = np.abs(val) > 1e-14
    rows.append(r[ok]); cols.append(c[ok]); vals.append(val[ok])
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.n_free, coarse.n_free))
    P.sum_duplicates()
    return P


def spacetime_prolongation(fine, coarse, n_time):
    """P = P_h (x) I_{n_time} for the [DoF][slab][node] layout."""
    return sp.kron(spatial_prolongation(fine, coarse), sp.identity(n_time), format="csr")


def inject_full(fine_level, coarse_level, ux, uy, p):
    """Inject full nodal arrays to the coarse level (coarse nodes are fine nodes)."""
    fm, cm = fine_level.mesh, coarse_level.mesh
    g = np.arange(cm.nn)
    gf = 2 * (g % cm.n2) + fm.n2 * 2 * (g // cm.n2)
    v = np.arange(cm.nv)
    vf = 2 * (v % cm.n1) + fm.n1 * 2 * (v // cm.n1)
    return ux[gf], uy[gf], p[vf]
