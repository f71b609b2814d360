"""Space-time residual and Jacobian of Taylor-Hood P2-P1 x DG(q) Navier-Stokes
(oracle), written as literal quadrature of the weak form eq. nsfem (Sec. 2).

Per slab I_n = (t_n, t_n + dt), with s in [0, 1], U(s) = sum_b phi_b(s) U_b,
test functions phi_a(s) psi_i and phi_a(s) chi_i:

  F^u = int_0^1 phi_a (d_s U, psi_i) ds + phi_a(0) (U(0) - U_{n-1}(1), psi_i)
        + dt int_0^1 phi_a [ (grad U, grad psi_i) + R ((U.grad) U, psi_i)
                             - (P, div psi_i) - (f, psi_i) ] ds
  F^p = - dt int_0^1 phi_a (div U, chi_i) ds

Readings: the jump term uses the upwind convention (the previous slab's end
value, eq. dgintime with U_0^- the P2 interpolant of the initial velocity);
the pressure enters as -(P, div psi) and -(div U, chi) (the form as printed
carries +(P, div psi), which only flips the sign of P); the forcing f is added
as the paper allows.  Dirichlet velocity values are the exact velocity at the
temporal nodes, interpolated at the boundary P2 nodes; those DoFs are not
unknowns.  The Jacobian is the exact derivative of F (full Newton), and its
sub-diagonal blocks (slab n against slab n-1) come only from the jump term.
"""
import numpy as np
import scipy.sparse as sp

from . import fe
from .quadrature import duffy_triangle
from .temporal import SlabBasis
from .mesh import Mesh


class Level:
    """One space-time level: a spatial mesh times the fixed temporal mesh."""

    def __init__(self, M, q, n_slabs, t_final, mms, nodes="radau"):
        self.mesh = Mesh(M)
        self.q, self.N, self.nq = q, n_slabs, q + 1
        self.T = t_final
        self.dt = t_final / n_slabs
        self.tb = SlabBasis(q, nodes)
        self.mms = mms
        self.R = mms.R
        m = self.mesh
        self.n_free = m.n_free
        self.n_st = m.n_free * n_slabs * self.nq
        self.xq, self.wq = duffy_triangle(5)
        self.N2, dN2 = fe.p2(self.xq)
        self.N1, dN1 = fe.p1(self.xq)
        v = m.vxy[m.cells]                          # (C, 3, 2)
        Jc = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)  # columns
        det = Jc[:, 0, 0] * Jc[:, 1, 1] - Jc[:, 0, 1] * Jc[:, 1, 0]
        inv = np.linalg.inv(Jc)
        self.wdet = self.wq[None, :] * np.abs(det)[:, None]          # (C, Q)
        self.gN2 = np.einsum("qim,cmk->cqik", dN2, inv)               # (C, Q, 6, 2)
        self.gN1 = np.einsum("qim,cmk->cqik", dN1, inv)               # (C, Q, 3, 2)
        self.xphys = v[:, 0, None, :] + np.einsum("ckm,qm->cqk", Jc, self.xq)  # (C,Q,2)
        self.cdofs = m.cell_dofs()                                    # (C, 15)
        self._mass = None

    # ---- boundary / initial data ------------------------------------------
    def node_times(self):
        """(N, nq) times of the temporal nodes."""
        n = np.arange(self.N)[:, None]
        return (n + self.tb.nodes[None, :]) * self.dt

    def dirichlet_full(self):
        """Exact velocity at every P2 node and temporal node: (nn, N, nq) x 2."""
        if getattr(self, "_dir", None) is None:
            t = self.node_times()[None, :, :]
            x = self.mesh.nxy[:, 0][:, None, None]
            y = self.mesh.nxy[:, 1][:, None, None]
            self._dir = self.mms.velocity(t, x, y)
        return self._dir

    def initial_full(self):
        """P2 interpolant of the initial velocity on every node: (nn,) x 2 (the
        velocity at t = 0, unless the flow states its own initial value)."""
        x, y = self.mesh.nxy[:, 0], self.mesh.nxy[:, 1]
        if hasattr(self.mms, "initial_velocity"):
            return self.mms.initial_velocity(x, y)
        return self.mms.velocity(0.0, x, y)

    def full_state(self, x_free):
        """Full nodal arrays (ux, uy, p) from a free space-time vector (n_free, N, nq)."""
        bx, by = self.dirichlet_full()
        m = self.mesh
        fr = m.node_free >= 0
        k = m.node_free[fr]
        ux, uy = bx.copy(), by.copy()
        ux[fr] = x_free[2 * k]
        uy[fr] = x_free[2 * k + 1]
        p = x_free[m.p_offset:].copy()
        return ux, uy, p

    def initial_guess(self):
        """Zero at every free DoF (boundary data sits outside the free vector)."""
        return np.zeros((self.n_free, self.N, self.nq))

    # ---- local evaluation ---------------------------------------------------
    def _slab_fields(self, ux, uy, p, n):
        tb = self.tb
        m = self.mesh
        uxc = ux[m.cell_p2, n, :]     # (C, 6, nq)
        uyc = uy[m.cell_p2, n, :]
        pc = p[m.cells, n, :]         # (C, 3, nq)
        f = {}
        for name, uc in (("x", uxc), ("y", uyc)):
            f["u" + name] = np.einsum("gb,cib,qi->cgq", tb.Phi, uc, self.N2)
            f["g" + name] = np.einsum("gb,cib,cqik->cgqk", tb.Phi, uc, self.gN2)
            f["d" + name] = np.einsum("gb,cib,qi->cgq", tb.dPhi, uc, self.N2)
            f["s0" + name] = np.einsum("b,cib,qi->cq", tb.e0, uc, self.N2)
        f["p"] = np.einsum("gb,cjb,qj->cgq", tb.Phi, pc, self.N1)
        return f

    # ---- residual -------------------------------------------------------------
    def residual(self, x_free, slabs=None):
        """F(U) at the free DoFs, shape (n_free, N, nq); only ``slabs`` if given."""
        ux, uy, p = self.full_state(x_free)
        m, tb, dt, R = self.mesh, self.tb, self.dt, self.R
        i0x, i0y = self.initial_full()
        Fx = np.zeros((m.nn, self.N, self.nq))
        Fy = np.zeros((m.nn, self.N, self.nq))
        Fp = np.zeros((m.nv, self.N, self.nq))
        wg = tb.wg
        for n in (range(self.N) if slabs is None else slabs):
            f = self._slab_fields(ux, uy, p, n)
            tg = (n + tb.sg) * dt
            fx, fy = self.mms.forcing(tg[None, :, None], self.xphys[:, None, :, 0],
                                      self.xphys[:, None, :, 1])       # (C, G, Q)
            if n == 0:
                px_, py_ = i0x, i0y
            else:
                px_ = ux[:, n - 1, :] @ tb.e1
                py_ = uy[:, n - 1, :] @ tb.e1
            prevx = np.einsum("ci,qi->cq", px_[m.cell_p2], self.N2)
            prevy = np.einsum("ci,qi->cq", py_[m.cell_p2], self.N2)
            div = f["gx"][..., 0] + f["gy"][..., 1]
            for comp, (u_, g_, d_, s0, prev, ff) in enumerate(
                    [(f["ux"], f["gx"], f["dx"], f["s0x"], prevx, fx),
                     (f["uy"], f["gy"], f["dy"], f["s0y"], prevy, fy)]):
                conv = f["ux"] * g_[..., 0] + f["uy"] * g_[..., 1]
                # volume terms at (c, g, q), against N2_i and grad N2_i
                val = d_ + dt * (R * conv - ff)              # * N2_i
                grd = dt * g_.copy()                         # . grad N2_i
                grd[..., comp] -= dt * f["p"]
                loc = (np.einsum("g,ga,cgq,cq,qi->cai", wg, tb.Phi, val, self.wdet, self.N2)
                       + np.einsum("g,ga,cgqk,cq,cqik->cai", wg, tb.Phi, grd, self.wdet, self.gN2)
                       + np.einsum("a,cq,cq,qi->cai", tb.e0, s0 - prev, self.wdet, self.N2))
                target = Fx if comp == 0 else Fy
                for a in range(self.nq):
                    np.add.at(target[:, n, a], m.cell_p2, loc[:, a, :])
            locp = -dt * np.einsum("g,ga,cgq,cq,qj->caj", wg, tb.Phi, div, self.wdet, self.N1)
            for a in range(self.nq):
                np.add.at(Fp[:, n, a], m.cells, locp[:, a, :])
        out = np.zeros((self.n_free, self.N, self.nq))
        fr = m.node_free >= 0
        k = m.node_free[fr]
        out[2 * k] = Fx[fr]
        out[2 * k + 1] = Fy[fr]
        out[m.p_offset:] = Fp
        return out

    # ---- Jacobian ---------------------------------------------------------------
    def mass_matrix(self):
        """Velocity mass matrix over free DoFs (pressure rows/cols zero), CSR."""
        if self._mass is None:
            m = self.mesh
            Mloc = np.einsum("cq,qi,qj->cij", self.wdet, self.N2, self.N2)
            rows, cols, vals = [], [], []
            for comp in range(2):
                d = self.cdofs[:, 6 * comp:6 * comp + 6]
                r = np.repeat(d[:, :, None], 6, axis=2)
                c = np.repeat(d[:, None, :], 6, axis=1)
                ok = (r >= 0) & (c >= 0)
                rows.append(r[ok]); cols.append(c[ok]); vals.append(Mloc[ok])
            self._mass = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows),
                                        np.concatenate(cols))), shape=(m.n_free, m.n_free))
        return self._mass

    def jacobian(self, x_free, slabs=None):
        """Space-time Jacobian dF/dU at U (free DoFs), CSR of size n_st; only the
        diagonal blocks of ``slabs`` (no jump blocks) if given."""
        ux, uy, p = self.full_state(x_free)
        m, tb, dt, R = self.mesh, self.tb, self.dt, self.R
        nq, N = self.nq, self.N
        wg = tb.wg
        Mloc = np.einsum("cq,qi,qj->cij", self.wdet, self.N2, self.N2)
        Kloc = np.einsum("cq,cqik,cqjk->cij", self.wdet, self.gN2, self.gN2)
        Bq = np.einsum("cq,qj,cqik->cjik", self.wdet, self.N1, self.gN2)  # (C,3,6,2): int chi_j d_k N_i
        Tq = np.einsum("g,ga,gb->ab", wg, tb.Phi, tb.dPhi) + np.outer(tb.e0, tb.e0)
        Wq = np.einsum("g,ga,gb->gab", wg, tb.Phi, tb.Phi)                # (G, nq, nq)
        rows, cols, vals = [], [], []
        st = N * nq
        C = m.nc
        for n in (range(N) if slabs is None else slabs):
            f = self._slab_fields(ux, uy, p, n)
            # conv1[c,g,i,j] = int N_i (u . grad N_j); conv2[c,g,ci,cj,i,j] = int N_i N_j d_cj u_ci
            conv1 = (np.einsum("cq,qi,cgq,cqj->cgij", self.wdet, self.N2, f["ux"], self.gN2[..., 0])
                     + np.einsum("cq,qi,cgq,cqj->cgij", self.wdet, self.N2, f["uy"], self.gN2[..., 1]))
            gu = np.stack([f["gx"], f["gy"]], axis=2)                 # (C,G,ci,Q,cj)
            conv2 = np.einsum("cq,qi,qj,cgaqb->cgabij", self.wdet, self.N2, self.N2, gu)
            J = np.zeros((C, nq, nq, 15, 15))
            for ci in range(2):
                sl = slice(6 * ci, 6 * ci + 6)
                J[:, :, :, sl, sl] += (Tq[None, :, :, None, None] * Mloc[:, None, None]
                                       + dt * np.einsum("gab,cij->cabij", Wq, Kloc)
                                       + dt * R * np.einsum("gab,cgij->cabij", Wq, conv1))
                for cj in range(2):
                    slj = slice(6 * cj, 6 * cj + 6)
                    J[:, :, :, sl, slj] += dt * R * np.einsum("gab,cgij->cabij", Wq,
                                                              conv2[:, :, ci, cj])
                # velocity test (ci, i), pressure trial j: -dt (chi_j, d_ci N_i)
                J[:, :, :, sl, 12:15] += -dt * np.einsum("gab,cji->cabij", Wq, Bq[..., ci])
                # pressure test j, velocity trial (ci, i): -dt (d_ci N_i, chi_j)
                J[:, :, :, 12:15, sl] += -dt * np.einsum("gab,cji->cabji", Wq, Bq[..., ci])
            d = self.cdofs
            base = d * st
            for a in range(nq):
                for b in range(nq):
                    r = np.repeat((base + n * nq + a)[:, :, None], 15, axis=2)
                    c = np.repeat((base + n * nq + b)[:, None, :], 15, axis=1)
                    ok = (np.repeat(d[:, :, None], 15, 2) >= 0) & (np.repeat(d[:, None, :], 15, 1) >= 0)
                    rows.append(r[ok]); cols.append(c[ok]); vals.append(J[:, a, b][ok])
        # sub-diagonal jump blocks: -phi_a(0) phi_b(1) M_ij
        Mm = self.mass_matrix().tocoo()
        for n in (range(1, N) if slabs is None else []):
            for a in range(nq):
                for b in range(nq):
                    coef = -tb.e0[a] * tb.e1[b]
                    if coef == 0.0:
                        continue
                    rows.append(Mm.row * st + n * nq + a)
                    cols.append(Mm.col * st + (n - 1) * nq + b)
                    vals.append(coef * Mm.data)
        Jst = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                            shape=(self.n_st, self.n_st))
        Jst.sum_duplicates()
        return Jst

    # ---- diagnostics -----------------------------------------------------------
    def velocity_l2_error(self, x_free):
        """Space-time velocity L2 error sqrt(sum_n int_In ||u - U||^2 dt)."""
        ux, uy, p = self.full_state(x_free)
        tot = 0.0
        tb = self.tb
        for n in range(self.N):
            f = self._slab_fields(ux, uy, p, n)
            tg = (n + tb.sg) * self.dt
            ex, ey = self.mms.velocity(tg[None, :, None], self.xphys[:, None, :, 0],
                                       self.xphys[:, None, :, 1])
            e2 = (ex - f["ux"]) ** 2 + (ey - f["uy"]) ** 2
            tot += self.dt * np.einsum("g,cgq,cq->", tb.wg, e2, self.wdet)
        return np.sqrt(tot)
