"""Exact discrete solutions by direct routes (oracle).

* R2, slab by slab: the space-time system is block lower triangular in time
  (eq. waveform_patch_solve), so it can be solved one slab after another, each
  by Newton with a sparse direct solve of the slab block bordered by the
  zero-mean pressure constraints (the timestepping view of Sec. 3, where the
  same discretisation is coupled over one time element at a time).
* Space-time Newton with exact linear solves: each Newton correction solves
  the whole space-time Jacobian system exactly, by forward substitution over
  the slabs (the Jacobian is block lower bidiagonal in time) with a sparse
  direct solve of each bordered slab block.  This is the direct-solver
  comparison of Sec. 4.3, which counts Newton steps with direct linear solves.
* R3, all at once: Newton on the whole space-time system with a dense LU of
  the bordered space-time Jacobian (the monolithic direct comparison of
  Sec. 4.1), for tiny meshes only.
Both return free vectors whose pressure has zero mean per temporal node.
"""
import numpy as np
import scipy.linalg as la
import scipy.sparse as sp
import scipy.sparse.linalg as spla




def solve_slab_by_slab(level, tol=0.0, maxit=40, info=None):
    """Newton per slab until ||F_n|| <= tol * max(1, ||U_n||) or, by default,
    until it reaches its rounding floor (no decrease by a factor 2 once below
    1e-10 relative).  ``info`` (a list) receives each slab's final ||F_n||."""
    nf, N, nq = level.n_free, level.N, level.nq
    st = N * nq
    po = level.mesh.p_offset
    x = np.zeros((nf, N, nq))
    rows = (np.arange(po, nf)[:, None] * nq + np.arange(nq)[None, :]).ravel()
    cols = np.tile(np.arange(nq), nf - po)
    C = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(nf * nq, nq))
    for n in range(N):
        idx = (np.arange(nf)[:, None] * st + n * nq + np.arange(nq)[None, :]).ravel()
        f0 = None
        fprev = None
        for it in range(maxit):
            F = level.residual(x, slabs=[n]).ravel()[idx]
            fn = np.linalg.norm(F)
            f0 = fn if f0 is None else f0
            if fn <= tol * max(1.0, np.linalg.norm(x[:, n, :])):
                break
            if fprev is not None and fn <= 1e-10 * f0 and fn > 0.5 * fprev:
                break
            if fn == 0.0:
                break
            fprev = fn
            J = level.jacobian(x, slabs=[n])
            Jn = J[idx][:, idx]
            B = sp.bmat([[Jn, C], [C.T, None]], format="csc")
            d = spla.spsolve(B, np.concatenate([-F, np.zeros(nq)]))[: nf * nq]
            x[:, n, :] += d.reshape(nf, nq)
        if info is not None:
            info.append(float(fn))
    return x


def solve_all_at_once(level, tol=1e-13, maxit=30):
    nf, N, nq = level.n_free, level.N, level.nq
    po = level.mesh.p_offset
    n = level.n_st
    C = np.zeros((n, N * nq))
    st = N * nq
    for k in range(N * nq):
        C[np.arange(po, nf) * st + k, k] = 1.0
    x = np.zeros(n)
    for it in range(maxit):
        F = level.residual(x.reshape(nf, N, nq)).ravel()
        if np.linalg.norm(F) <= tol * max(1.0, np.linalg.norm(x)):
            break
        J = level.jacobian(x.reshape(nf, N, nq)).toarray()
        B = np.block([[J, C], [C.T, np.zeros((N * nq, N * nq))]])
        d = la.solve(B, np.concatenate([-F, np.zeros(N * nq)]))[:n]
        x += d
    return x.reshape(nf, N, nq)


def newton_exact_linear(level, rtol=1e-8, maxit=20):
    """Newton on the whole space-time system, started from zero, with full
    steps and exact linear solves, stopped once ||F|| <= rtol ||F_0||.
    Returns (solution, [||F_k||])."""
    nf, N, nq = level.n_free, level.N, level.nq
    st = N * nq
    po = level.mesh.p_offset
    ns = nf * nq
    rows = (np.arange(po, nf)[:, None] * nq + np.arange(nq)[None, :]).ravel()
    cols = np.tile(np.arange(nq), nf - po)
    C = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(ns, nq))
    # slab-major order: slab n occupies rows n*ns .. (n+1)*ns of the permuted system
    perm = np.concatenate([(np.arange(nf)[:, None] * st + n * nq + np.arange(nq)[None, :]).ravel()
                           for n in range(N)])
    x = np.zeros(nf * st)
    fnorm = []
    for _ in range(maxit + 1):
        F = level.residual(x.reshape(nf, N, nq)).ravel()
        fnorm.append(np.linalg.norm(F))
        if fnorm[-1] <= rtol * fnorm[0]:
            break
        J = level.jacobian(x.reshape(nf, N, nq)).tocsr()[perm][:, perm].tocsr()
        b = -F[perm]
        d = np.zeros(nf * st)
        for n in range(N):
            r = slice(n * ns, (n + 1) * ns)
            rhs = b[r]
            if n > 0:
                rhs = rhs - J[r, (n - 1) * ns:n * ns] @ d[(n - 1) * ns:n * ns]
            B = sp.bmat([[J[r, r], C], [C.T, None]], format="csc")
            d[r] = spla.spsolve(B, np.concatenate([rhs, np.zeros(nq)]))[:ns]
        x[perm] += d
    return x.reshape(nf, N, nq), fnorm

