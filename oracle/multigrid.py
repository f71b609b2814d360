"""Newton-Krylov-multigrid driver (oracle): Alg. 1 V-cycle preconditioning
FGMRES (Sec. 3), inside Newton's method (Sec. 4.2).

Readings where the paper is silent:
* coarse operators are rediscretised Jacobians at the Newton iterate injected
  to the coarse nodes (coarse P2/P1 nodes are fine nodes);
* the coarsest solve is exact: forward block substitution over slabs, with a
  dense LU per slab of the slab block bordered by one zero-mean pressure
  constraint per temporal node (the constant pressure is the null space when
  every velocity boundary value is prescribed);
* in FGMRES the constant pressure per (slab, temporal node) is projected out of
  every preconditioned vector, so every correction has zero-mean pressure;
* Newton starts from zero at the free DoFs (boundary data fixed), takes full
  steps and stops on ||F|| <= rtol ||F_0|| (l2 over free DoFs).
"""
import dataclasses

import numpy as np
import scipy.linalg as la

from .assembly import Level
from .mms import make_flow
from .smoother import PatchSmoother, chebyshev, eig_estimate
from .transfer import spacetime_prolongation, inject_full


@dataclasses.dataclass
class Options:
    nu_pre: int = 2
    nu_post: int = 2
    cheb_lo: float = 0.25
    cheb_hi: float = 1.05
    eig_steps: int = 10
    gmres_restart: int = 30
    gmres_maxit: int = 200
    gmres_rtol: float = 1e-10
    newton_maxit: int = 20
    newton_rtol: float = 1e-10
    newton_ew: bool = False      # Eisenstat-Walker linear tolerances (see ew_forcing)


# Eisenstat and Walker's second choice of forcing term (SIAM J. Sci. Comput.
# 17, 1996): eta_k = gamma (||F_k|| / ||F_{k-1}||)^alpha, kept at least
# gamma eta_{k-1}^alpha when that exceeds a threshold, and at most eta_max;
# eta_0 given.  The paper cites the method without its parameters; these are
# the defaults of the PETSc implementation it ran on.
EW_ETA0, EW_ETA_MAX, EW_GAMMA, EW_ALPHA, EW_THRESHOLD = 0.3, 0.9, 1.0, (1 + 5 ** 0.5) / 2, 0.1


def ew_forcing(k, fnorm, fnorm_prev, eta_prev):
    """Relative tolerance of the k-th Newton linear solve."""
    if k == 0:
        return EW_ETA0
    eta = EW_GAMMA * (fnorm / fnorm_prev) ** EW_ALPHA
    safe = EW_GAMMA * eta_prev ** EW_ALPHA
    if safe > EW_THRESHOLD:
        eta = max(eta, safe)
    return min(eta, EW_ETA_MAX)


def project_pressure(level, v):
    """Remove the mean pressure per (slab, temporal node) from a free vector."""
    w = np.array(v, dtype=float, copy=True).reshape(level.n_free, level.N, level.nq)
    po = level.mesh.p_offset
    w[po:] -= w[po:].mean(axis=0, keepdims=True)
    return w.ravel()


class CoarseSolver:
    """Exact coarsest-grid solve by slab-wise bordered dense LU."""

    def __init__(self, level, A):
        self.level = level
        nf, N, nq = level.n_free, level.N, level.nq
        st = N * nq
        self.idx = [(np.arange(nf)[:, None] * st + n * nq + np.arange(nq)[None, :]).ravel()
                    for n in range(N)]
        po = level.mesh.p_offset
        C = np.zeros((nf * nq, nq))
        for a in range(nq):
            C[(np.arange(po, nf) * nq + a), a] = 1.0
        self.lus, self.subs = [], []
        A = A.tocsr()
        for n in range(N):
            An = A[self.idx[n]][:, self.idx[n]].toarray()
            Bn = np.block([[An, C], [C.T, np.zeros((nq, nq))]])
            self.lus.append(la.lu_factor(Bn))
            self.subs.append(A[self.idx[n]][:, self.idx[n - 1]] if n > 0 else None)
        self.k = nf * nq
        self.nq = nq

    def solve(self, b):
        x = np.zeros_like(b)
        for n in range(self.level.N):
            g = b[self.idx[n]].copy()
            if n > 0:
                g -= self.subs[n] @ x[self.idx[n - 1]]
            sol = la.lu_solve(self.lus[n], np.concatenate([g, np.zeros(self.nq)]))
            x[self.idx[n]] = sol[:self.k]
        return x


class Hierarchy:
    def __init__(self, prob, opts=None):
        self.opts = opts or Options()
        self.mms = make_flow(prob)
        nodes = "gauss" if getattr(prob, "nodes", 0) == 1 else "radau"
        self.levels = [Level(prob.mesh_n >> l, prob.q, prob.n_slabs, prob.t_final, self.mms, nodes)
                       for l in range(prob.n_levels)]
        L0 = self.levels[0]
        self.P = [spacetime_prolongation(self.levels[l].mesh, self.levels[l + 1].mesh,
                                         L0.N * L0.nq) for l in range(prob.n_levels - 1)]
        self.A = None

    # --- state injection -------------------------------------------------------
    def level_states(self, x_fine):
        """Free vectors of the Newton iterate injected to every level."""
        out = [x_fine]
        ux, uy, p = self.levels[0].full_state(x_fine.reshape(self.levels[0].n_free, -1,
                                                             self.levels[0].nq))
        for l in range(1, len(self.levels)):
            ux, uy, p = inject_full(self.levels[l - 1], self.levels[l], ux, uy, p)
            m = self.levels[l].mesh
            fr = m.node_free >= 0
            k = m.node_free[fr]
            x = np.zeros((m.n_free, self.levels[l].N, self.levels[l].nq))
            x[2 * k] = ux[fr]
            x[2 * k + 1] = uy[fr]
            x[m.p_offset:] = p
            out.append(x)
        return out

    def assemble(self, x_fine, with_smoothers=True):
        """Jacobians on every level at x_fine; patch factors, lambdas, coarse LU."""
        xs = self.level_states(np.asarray(x_fine).reshape(self.levels[0].n_free,
                                                          self.levels[0].N, self.levels[0].nq))
        self.A = [lev.jacobian(x) for lev, x in zip(self.levels, xs)]
        self.smoothers, self.lams = [], []
        if with_smoothers:
            for l in range(len(self.levels) - 1):
                sm = PatchSmoother(self.levels[l], self.A[l])
                self.smoothers.append(sm)
                self.lams.append(eig_estimate(self.A[l], sm.apply, self.levels[l].n_st,
                                              self.opts.eig_steps))
            self.coarse = CoarseSolver(self.levels[-1], self.A[-1])

    def relax(self, l, b, x, n_steps):
        lam = self.lams[l]
        return chebyshev(self.A[l], self.smoothers[l].apply, b, x, n_steps,
                         self.opts.cheb_lo * lam, self.opts.cheb_hi * lam)

    def vcycle(self, b, l=0):
        """Alg. 1: pre-relax, residual, restrict (zero coarse guess), ..., coarsest
        direct solve, then interpolate-add and post-relax on the way up."""
        if l == len(self.levels) - 1:
            return self.coarse.solve(b)
        x = self.relax(l, b, np.zeros_like(b), self.opts.nu_pre)
        r = b - self.A[l] @ x
        xc = self.vcycle(self.P[l].T @ r, l + 1)
        x = x + self.P[l] @ xc
        return self.relax(l, b, x, self.opts.nu_post)


def fgmres(A, prec, b, rtol, restart, maxit, project=lambda v: v, atol=0.0):
    """Right-preconditioned restarted FGMRES with MGS, stopping when the
    residual is at most max(rtol ||b||, atol); returns (x, iterations, history)."""
    n = b.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = []
    its = 0
    if bnorm == 0.0:
        return x, 0, [0.0]
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta <= max(rtol * bnorm, atol) or its >= maxit:
            break
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_last = 0
        for j in range(restart):
            Z[j] = project(prec(V[j]))
            w = A @ Z[j]
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_last = j
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= max(rtol * bnorm, atol) or its >= maxit:
                break
        k = j_last + 1
        y = la.solve_triangular(H[:k, :k], g[:k])
        x = x + Z[:k].T @ y
        if abs(g[k]) <= rtol * bnorm or its >= maxit:
            break
    return x, its, hist


def newton_solve(prob, opts=None, max_newton=None, x0=None):
    """Newton-FGMRES-WRMG solve; returns (x_free, stats dict)."""
    H = Hierarchy(prob, opts)
    o = H.opts
    L0 = H.levels[0]
    x = L0.initial_guess().ravel() if x0 is None else np.array(x0, dtype=float).ravel()
    F = L0.residual(x.reshape(L0.n_free, L0.N, L0.nq)).ravel()
    f0 = np.linalg.norm(F)
    stats = {"newton": 0, "linear": [], "fnorm": [f0], "eta": []}
    maxit = o.newton_maxit if max_newton is None else max_newton
    eta = None
    for k in range(maxit):
        if np.linalg.norm(F) <= o.newton_rtol * f0:
            break
        H.assemble(x)
        rtol = o.gmres_rtol
        if o.newton_ew:
            eta = ew_forcing(k, stats["fnorm"][-1], stats["fnorm"][-2] if k else f0, eta)
            rtol = eta
            stats["eta"].append(eta)
        # absolute floor three orders below the Newton target: a relative
        # tolerance alone would chase rounding once F is tiny
        dx, its, _ = fgmres(H.A[0], H.vcycle, -F, rtol, o.gmres_restart,
                            o.gmres_maxit, lambda v: project_pressure(L0, v),
                            atol=1e-3 * o.newton_rtol * f0)
        x = x + dx
        F = L0.residual(x.reshape(L0.n_free, L0.N, L0.nq)).ravel()
        stats["newton"] += 1
        stats["linear"].append(its)
        stats["fnorm"].append(np.linalg.norm(F))
        if stats["fnorm"][-1] > 1e2 * f0:     # divergence: stop (full steps, no line search)
            stats["diverged"] = True
            break
    return x, stats, H
