"""Taylor-Hood P_{k+1}-P_k structure on the structured mesh, for any k >= 1
(oracle; test infrastructure only): Lagrange node lattices, the nodes of each
cell, Vanka+star patches and the structural nonzeros of their matrices
(Sec. 2 eq. nsfem with velocity of degree k+1 and pressure of degree k;
Sec. 3 and Sec. 3.1 for the patches and their counts).

The mesh is the one of oracle/mesh.py: M x M squares, square (i, j) split into
the cells (v_ij, v_i+1,j, v_i,j+1) and (v_i+1,j+1, v_i,j+1, v_i+1,j).  A
degree-K Lagrange space has the (KM+1)^2 lattice nodes of spacing h/K; node
(gi, gj) is gi + (KM+1) gj.  A cell with vertex grid coordinates A, B, C
holds the lattice nodes K A + s (B - A) + t (C - A), s, t >= 0, s + t <= K.

Vanka+star patch of vertex v: every velocity node in the closure of the star
of v (all nodes of the cells around v), both components, and the pressure
nodes in the interior of the star (v and the nodes inside the edges and cells
incident to v).  Two DoFs are structurally coupled when their nodes share a
cell; the patch matrix holds the 2 x 2 component block of every coupled
velocity node pair, both off-diagonal velocity-pressure blocks of every
coupled (velocity node, pressure node) pair, and no pressure-pressure block.

Every count here is a plain enumeration: no formula of the paper is used to
produce it, so that the paper's closed forms can pin it.  The spatial
operators of eq. nsfem's linear terms (velocity mass and stiffness of one
component, the two divergence blocks) are assembled cell by cell with the
degree-8 triangle rule, which integrates every one of them exactly for
k <= 2.  TaylorHoodLevel assembles the full space-time Jacobian (DG(q) in
time, full Newton, as oracle/assembly.py does at k = 1) for any k <= 2.
"""
import numpy as np
import scipy.sparse as sp

from .heat import HeatSpace, lagrange_pk
from .quadrature import duffy_triangle


def _cells(M):
    """(2 M^2, 3) vertex grid coordinates (i, j) of each cell's vertices."""
    out = []
    for j in range(M):
        for i in range(M):
            out.append([(i, j), (i + 1, j), (i, j + 1)])
            out.append([(i + 1, j + 1), (i, j + 1), (i + 1, j)])
    return np.array(out, dtype=np.int64)


def cell_lattice_nodes(M, K):
    """(2 M^2, (K+1)(K+2)/2) lattice node ids of the degree-K nodes of each cell."""
    C = _cells(M)
    n = K * M + 1
    nodes = []
    for A, B, Cv in C:
        A, B, Cv = np.array(A), np.array(B), np.array(Cv)
        row = []
        for t in range(K + 1):
            for s in range(K + 1 - t):
                g = K * A + s * (B - A) + t * (Cv - A)
                row.append(g[0] + n * g[1])
        nodes.append(row)
    return np.array(nodes, dtype=np.int64)


class TaylorHood:
    """P_{k+1} velocity / P_k pressure on the M x M mesh."""

    def __init__(self, M, k):
        if k < 1:
            raise ValueError("pressure degree k must be at least 1")
        self.M, self.k = M, k
        self.Kv, self.Kp = k + 1, k
        self.nv_side = (k + 1) * M + 1
        self.np_side = k * M + 1
        self.vel_cells = cell_lattice_nodes(M, self.Kv)
        self.p_cells = cell_lattice_nodes(M, self.Kp)
        self.cells = _cells(M)
        self.nc = len(self.cells)

    # --- counts over the whole mesh -----------------------------------------
    def n_dofs_total(self):
        """Every DoF, Dirichlet ones included: two velocity components on the
        velocity lattice and one pressure per pressure-lattice node."""
        return 2 * self.nv_side ** 2 + self.np_side ** 2

    def n_dofs_free(self):
        """Velocity DoFs at interior lattice nodes (Dirichlet boundary) plus all pressures."""
        return 2 * (self.nv_side - 2) ** 2 + self.np_side ** 2

    def _vel_interior(self, g):
        gi, gj = g % self.nv_side, g // self.nv_side
        return (gi > 0) & (gi < self.nv_side - 1) & (gj > 0) & (gj < self.nv_side - 1)

    # --- patches --------------------------------------------------------------
    def star_cells(self, v):
        """Cells having grid vertex v = (i, j) as a vertex."""
        i, j = v
        hit = np.all(self.cells == np.array([i, j]), axis=2).any(axis=1)
        return np.nonzero(hit)[0]

    def patch(self, v, free_only=True):
        """(velocity lattice nodes, pressure lattice nodes) of the Vanka+star
        patch of grid vertex v.  With free_only, velocity nodes on the
        Dirichlet boundary are left out."""
        cs = self.star_cells(v)
        vel = np.unique(self.vel_cells[cs].ravel())
        if free_only:
            vel = vel[self._vel_interior(vel)]
        # pressure nodes inside the star: those of the star's cells that lie
        # on no edge opposite v (the star's outer boundary)
        Kp, n = self.Kp, self.np_side
        pres = set()
        for c in cs:
            verts = [tuple(x) for x in self.cells[c]]
            a = verts.index(tuple(v))
            A = np.array(verts[a])
            B, Cv = np.array(verts[(a + 1) % 3]), np.array(verts[(a + 2) % 3])
            for t in range(Kp + 1):
                for s in range(Kp + 1 - t):
                    if s + t == Kp and Kp > 0:   # on the edge opposite v
                        continue
                    g = Kp * A + s * (B - A) + t * (Cv - A)
                    pres.add(int(g[0] + n * g[1]))
        return vel, np.array(sorted(pres), dtype=np.int64)

    def patch_dofs(self, v, free_only=True):
        vel, pres = self.patch(v, free_only)
        return 2 * len(vel) + len(pres)

    def patch_nnz(self, v, free_only=True):
        """Structural nonzeros of the patch matrix: 4 per coupled (ordered)
        velocity node pair, 2 x 2 per coupled (velocity node, pressure node)
        pair (the (1,2) and (2,1) blocks), none between pressures."""
        vel, pres = self.patch(v, free_only)
        vset, pset = set(vel.tolist()), set(pres.tolist())
        vv, vp = set(), set()
        for c in range(self.nc):
            cv = [g for g in self.vel_cells[c] if g in vset]
            cp = [g for g in self.p_cells[c] if g in pset]
            for a in cv:
                for b in cv:
                    vv.add((a, b))
                for r in cp:
                    vp.add((a, r))
        return 4 * len(vv) + 4 * len(vp)


def spatial_operators(M, k):
    """Velocity mass Mu and stiffness Ku of one component (degree k+1) and the
    divergence blocks Bx[r, u] = int psi_r d(phi_u)/dx, By likewise (pressure
    degree k rows, velocity degree k+1 columns), over every lattice node
    (Dirichlet nodes included), as CSR matrices.  Velocity and pressure nodes
    are numbered on their own lattices, as in TaylorHood."""
    V, P = HeatSpace(M, k + 1), HeatSpace(M, k)
    Mu, Ku = V.matrices()
    pts, w = duffy_triangle(5)
    _, vgrad = lagrange_pk(k + 1, pts)
    pval, _ = lagrange_pk(k, pts)
    mesh = V.mesh
    rows, cols, bx, by = [], [], [], []
    for c in range(mesh.nc):
        v = mesh.vxy[mesh.cells[c]]
        J = np.stack([v[1] - v[0], v[2] - v[0]], axis=1)
        det = abs(np.linalg.det(J))
        G = vgrad @ np.linalg.inv(J)           # physical velocity gradients (nq, nloc_v, 2)
        Bxe = np.einsum("q,qr,qu->ru", w * det, pval, G[:, :, 0])
        Bye = np.einsum("q,qr,qu->ru", w * det, pval, G[:, :, 1])
        pn, vn = P.cell_nodes[c], V.cell_nodes[c]
        rows.append(np.repeat(pn, len(vn)))
        cols.append(np.tile(vn, len(pn)))
        bx.append(Bxe.ravel())
        by.append(Bye.ravel())
    r, cc = np.concatenate(rows), np.concatenate(cols)
    Bx = sp.csr_matrix((np.concatenate(bx), (r, cc)), shape=(P.n, V.n))
    By = sp.csr_matrix((np.concatenate(by), (r, cc)), shape=(P.n, V.n))
    Bx.sum_duplicates()
    By.sum_duplicates()
    return Mu, Ku, Bx, By, V, P


def prolongation(M_fine, k):
    """Prolongation of the Taylor-Hood space from the M_fine / 2 mesh to the
    M_fine mesh (Sec. 3: the spaces are nested, P = blockdiag(P_u, P_u,
    P_phi)): nodal interpolation of each coarse field at the fine lattice
    nodes, velocity (degree k+1) and pressure (degree k) on their own
    lattices.  Returns (P_u, P_p), CSR, every lattice node included."""
    if M_fine % 2:
        raise ValueError("the fine mesh must have an even number of squares per side")
    Vf, Vc = HeatSpace(M_fine, k + 1), HeatSpace(M_fine // 2, k + 1)
    Pf, Pc = HeatSpace(M_fine, k), HeatSpace(M_fine // 2, k)
    return Vf.prolongation(Vc), Pf.prolongation(Pc)


def convection_operators(M, k, ux, uy):
    """The two parts of the Newton linearization of the convection term of
    eq. nsfem about a velocity field (ux, uy) of degree k+1, given by its
    values at the velocity lattice nodes, on one component's lattice:
    C[i, j] = int phi_i (u . grad phi_j)   (the same block for both components),
    D[a][b][i, j] = int phi_i phi_j d u_a / d x_b   (a, b in {x, y}),
    CSR.  The integrands have degree 3(k+1) - 1, at most 8 for k <= 2."""
    V = HeatSpace(M, k + 1)
    pts, w = duffy_triangle(5)
    val, grad = lagrange_pk(k + 1, pts)
    mesh = V.mesh
    nloc = V.cell_nodes.shape[1]
    rows, cols = [], []
    cv = []
    dv = [[[], []], [[], []]]
    for c in range(mesh.nc):
        v = mesh.vxy[mesh.cells[c]]
        J = np.stack([v[1] - v[0], v[2] - v[0]], axis=1)
        wd = w * abs(np.linalg.det(J))
        G = grad @ np.linalg.inv(J)
        nodes = V.cell_nodes[c]
        u = [val @ ux[nodes], val @ uy[nodes]]                       # (nq,)
        gu = [G.transpose(0, 2, 1) @ ux[nodes], G.transpose(0, 2, 1) @ uy[nodes]]   # (nq, 2)
        adv = u[0][:, None] * G[:, :, 0] + u[1][:, None] * G[:, :, 1]               # (nq, nloc)
        cv.append(np.einsum("q,qi,qj->ij", wd, val, adv).ravel())
        for a in range(2):
            for b in range(2):
                dv[a][b].append(np.einsum("q,qi,qj->ij", wd * gu[a][:, b], val, val).ravel())
        rows.append(np.repeat(nodes, nloc))
        cols.append(np.tile(nodes, nloc))
    r, cc = np.concatenate(rows), np.concatenate(cols)

    def mat(parts):
        A = sp.csr_matrix((np.concatenate(parts), (r, cc)), shape=(V.n, V.n))
        A.sum_duplicates()
        return A

    return mat(cv), [[mat(dv[a][b]) for b in range(2)] for a in range(2)], V


class _LevelMesh:
    """The part of a level's mesh that oracle/multigrid.py and
    oracle/smoother.py read: the pressure offset and the patches."""

    def __init__(self, level):
        self._level = level
        self.p_offset = level.p_offset

    def patches(self):
        return self._level.patches()


class TaylorHoodLevel:
    """One space-time level of Taylor-Hood P_{k+1}-P_k x DG(q) Navier-Stokes
    (oracle): the space-time Jacobian of eq. nsfem (full Newton, as the P2-P1
    level of oracle/assembly.py defines it, with the element degrees as
    parameters).  Free numbering: interior velocity lattice node
    (gi, gj) -> k = (gi-1) + (n-2)(gj-1) with DoFs 2k (x), 2k+1 (y); pressure
    lattice node r -> 2 (n-2)^2 + r (n the velocity lattice side); Dirichlet
    velocity values are the flow's velocity at the boundary lattice nodes."""

    def __init__(self, M, k, q, n_slabs, t_final, mms, nodes="radau"):
        from .temporal import SlabBasis
        self.V, self.P = HeatSpace(M, k + 1), HeatSpace(M, k)
        self.M, self.k, self.q, self.N, self.nq = M, k, q, n_slabs, q + 1
        self.dt = t_final / n_slabs
        self.tb = SlabBasis(q, nodes)
        self.mms, self.R = mms, mms.R
        nl = self.V.nl
        g = np.arange(self.V.n)
        gi, gj = g % nl, g // nl
        interior = (gi > 0) & (gi < nl - 1) & (gj > 0) & (gj < nl - 1)
        self.node_free = np.full(self.V.n, -1, dtype=np.int64)
        self.node_free[interior] = (gi[interior] - 1) + (nl - 2) * (gj[interior] - 1)
        self.p_offset = 2 * (nl - 2) ** 2
        self.n_free = self.p_offset + self.P.n
        self.n_st = self.n_free * n_slabs * self.nq
        xq, wq = duffy_triangle(5)
        self.Nv, dNv = lagrange_pk(k + 1, xq)
        self.Np, _ = lagrange_pk(k, xq)
        mesh = self.V.mesh
        v = mesh.vxy[mesh.cells]
        Jc = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)
        det = Jc[:, 0, 0] * Jc[:, 1, 1] - Jc[:, 0, 1] * Jc[:, 1, 0]
        inv = np.linalg.inv(Jc)
        self.wdet = wq[None, :] * np.abs(det)[:, None]
        self.gNv = np.einsum("qim,cmk->cqik", dNv, inv)
        cv, cp = self.V.cell_nodes, self.P.cell_nodes
        fv = self.node_free[cv]
        self.cdofs = np.concatenate([np.where(fv >= 0, 2 * fv, -1), np.where(fv >= 0, 2 * fv + 1, -1),
                                     self.p_offset + cp], axis=1)
        self.nlv, self.nlp = cv.shape[1], cp.shape[1]
        # what the shared multigrid code reads from a level's mesh
        self.mesh = _LevelMesh(self)

    def patches(self):
        """Vanka+star patches (one per vertex, boundary vertices included) as
        sorted free DoF lists, for oracle/smoother.py's PatchSmoother."""
        th = TaylorHood(self.M, self.k)
        n1 = self.M + 1
        out = []
        for vid in range(n1 * n1):
            vel, pres = th.patch((vid % n1, vid // n1))
            f = self.node_free[vel]
            out.append(np.sort(np.concatenate([2 * f, 2 * f + 1, self.p_offset + pres])))
        return out

    def full_state(self, x_free):
        """Nodal (ux, uy) of shape (velocity nodes, N, nq) from a free space-time vector."""
        t = ((np.arange(self.N)[:, None] + self.tb.nodes[None, :]) * self.dt)[None, :, :]
        bx, by = self.mms.velocity(t, self.V.xy[:, 0][:, None, None], self.V.xy[:, 1][:, None, None])
        ux, uy = np.array(bx, dtype=float), np.array(by, dtype=float)
        fr = self.node_free >= 0
        kf = self.node_free[fr]
        ux[fr] = x_free[2 * kf]
        uy[fr] = x_free[2 * kf + 1]
        return ux, uy

    def initial_full(self):
        """Interpolant of the initial velocity at every velocity lattice node
        (the flow's own initial value where it states one, else u(0))."""
        x, y = self.V.xy[:, 0], self.V.xy[:, 1]
        if hasattr(self.mms, "initial_velocity"):
            return self.mms.initial_velocity(x, y)
        return self.mms.velocity(0.0, x, y)

    def residual(self, x_free):
        """F(U) at the free DoFs, shape (n_free, N, nq): the weak form of eq.
        nsfem per slab, as oracle/assembly.py writes it at k = 1 (upwind jump
        against the previous slab's end value, pressure as -(P, div psi) and
        -(div U, chi), the flow's forcing)."""
        xf = np.asarray(x_free).reshape(self.n_free, self.N, self.nq)
        ux, uy = self.full_state(xf)
        p = xf[self.p_offset:]
        tb, dt, R, nq = self.tb, self.dt, self.R, self.nq
        mesh = self.V.mesh
        cv, cp = self.V.cell_nodes, self.P.cell_nodes
        v = mesh.vxy[mesh.cells]
        Jc = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)
        xq, _ = duffy_triangle(5)
        xphys = v[:, 0, None, :] + np.einsum("ckm,qm->cqk", Jc, xq)
        i0x, i0y = self.initial_full()
        Fx = np.zeros((self.V.n, self.N, nq))
        Fy = np.zeros((self.V.n, self.N, nq))
        Fp = np.zeros((self.P.n, self.N, nq))
        for n in range(self.N):
            f = {}
            for name, u in (("x", ux), ("y", uy)):
                uc = u[cv, n, :]
                f["u" + name] = np.einsum("gb,cib,qi->cgq", tb.Phi, uc, self.Nv)
                f["g" + name] = np.einsum("gb,cib,cqik->cgqk", tb.Phi, uc, self.gNv)
                f["d" + name] = np.einsum("gb,cib,qi->cgq", tb.dPhi, uc, self.Nv)
                f["s0" + name] = np.einsum("b,cib,qi->cq", tb.e0, uc, self.Nv)
            f["p"] = np.einsum("gb,cjb,qj->cgq", tb.Phi, p[cp, n, :], self.Np)
            tg = (n + tb.sg) * dt
            fx, fy = self.mms.forcing(tg[None, :, None], xphys[:, None, :, 0], xphys[:, None, :, 1])
            if n == 0:
                px_, py_ = i0x, i0y
            else:
                px_, py_ = ux[:, n - 1, :] @ tb.e1, uy[:, n - 1, :] @ tb.e1
            prevx = np.einsum("ci,qi->cq", px_[cv], self.Nv)
            prevy = np.einsum("ci,qi->cq", py_[cv], self.Nv)
            div = f["gx"][..., 0] + f["gy"][..., 1]
            for comp, (g_, d_, s0, prev, ff) in enumerate(
                    [(f["gx"], f["dx"], f["s0x"], prevx, fx), (f["gy"], f["dy"], f["s0y"], prevy, fy)]):
                conv = f["ux"] * g_[..., 0] + f["uy"] * g_[..., 1]
                val = d_ + dt * (R * conv - ff)
                grd = dt * g_.copy()
                grd[..., comp] -= dt * f["p"]
                loc = (np.einsum("g,ga,cgq,cq,qi->cai", tb.wg, tb.Phi, val, self.wdet, self.Nv)
                       + np.einsum("g,ga,cgqk,cq,cqik->cai", tb.wg, tb.Phi, grd, self.wdet, self.gNv)
                       + np.einsum("a,cq,cq,qi->cai", tb.e0, s0 - prev, self.wdet, self.Nv))
                target = Fx if comp == 0 else Fy
                for a in range(nq):
                    np.add.at(target[:, n, a], cv, loc[:, a, :])
            locp = -dt * np.einsum("g,ga,cgq,cq,qj->caj", tb.wg, tb.Phi, div, self.wdet, self.Np)
            for a in range(nq):
                np.add.at(Fp[:, n, a], cp, locp[:, a, :])
        out = np.zeros((self.n_free, self.N, nq))
        fr = self.node_free >= 0
        kf = self.node_free[fr]
        out[2 * kf] = Fx[fr]
        out[2 * kf + 1] = Fy[fr]
        out[self.p_offset:] = Fp
        return out

    def jacobian(self, x_free):
        """Space-time Jacobian dF/dU at U (free DoFs), CSR of size n_st."""
        ux, uy = self.full_state(np.asarray(x_free).reshape(self.n_free, self.N, self.nq))
        tb, dt, R, nq, N = self.tb, self.dt, self.R, self.nq, self.N
        nlv, nlp = self.nlv, self.nlp
        ndl = 2 * nlv + nlp
        cv = self.V.cell_nodes
        Mloc = np.einsum("cq,qi,qj->cij", self.wdet, self.Nv, self.Nv)
        Kloc = np.einsum("cq,cqik,cqjk->cij", self.wdet, self.gNv, self.gNv)
        Bq = np.einsum("cq,qj,cqik->cjik", self.wdet, self.Np, self.gNv)   # int chi_j d_k phi_i
        Tq = np.einsum("g,ga,gb->ab", tb.wg, tb.Phi, tb.dPhi) + np.outer(tb.e0, tb.e0)
        Wq = np.einsum("g,ga,gb->gab", tb.wg, tb.Phi, tb.Phi)
        st = N * nq
        rows, cols, vals = [], [], []
        for n in range(N):
            f = {}
            for name, u in (("x", ux), ("y", uy)):
                uc = u[cv, n, :]
                f["u" + name] = np.einsum("gb,cib,qi->cgq", tb.Phi, uc, self.Nv)
                f["g" + name] = np.einsum("gb,cib,cqik->cgqk", tb.Phi, uc, self.gNv)
            conv1 = (np.einsum("cq,qi,cgq,cqj->cgij", self.wdet, self.Nv, f["ux"], self.gNv[..., 0])
                     + np.einsum("cq,qi,cgq,cqj->cgij", self.wdet, self.Nv, f["uy"], self.gNv[..., 1]))
            gu = np.stack([f["gx"], f["gy"]], axis=2)
            conv2 = np.einsum("cq,qi,qj,cgaqb->cgabij", self.wdet, self.Nv, self.Nv, gu)
            J = np.zeros((len(cv), nq, nq, ndl, ndl))
            pv = slice(2 * nlv, ndl)
            for ci in range(2):
                sl = slice(nlv * ci, nlv * ci + nlv)
                J[:, :, :, sl, sl] += (Tq[None, :, :, None, None] * Mloc[:, None, None]
                                       + dt * np.einsum("gab,cij->cabij", Wq, Kloc)
                                       + dt * R * np.einsum("gab,cgij->cabij", Wq, conv1))
                for cj in range(2):
                    slj = slice(nlv * cj, nlv * cj + nlv)
                    J[:, :, :, sl, slj] += dt * R * np.einsum("gab,cgij->cabij", Wq, conv2[:, :, ci, cj])
                J[:, :, :, sl, pv] += -dt * np.einsum("gab,cji->cabij", Wq, Bq[..., ci])
                J[:, :, :, pv, sl] += -dt * np.einsum("gab,cji->cabji", Wq, Bq[..., ci])
            d = self.cdofs
            ok = (d[:, :, None] >= 0) & (d[:, None, :] >= 0)
            for a in range(nq):
                for b in range(nq):
                    r = np.broadcast_to((d * st + n * nq + a)[:, :, None], ok.shape)
                    c = np.broadcast_to((d * st + n * nq + b)[:, None, :], ok.shape)
                    rows.append(r[ok]); cols.append(c[ok]); vals.append(J[:, a, b][ok])
        # jump blocks -phi_a(0) phi_b(1) M between slab n and slab n - 1 (velocity rows)
        dv = self.cdofs[:, :2 * nlv]
        Mblk = np.zeros((len(cv), 2 * nlv, 2 * nlv))
        Mblk[:, :nlv, :nlv] = Mloc
        Mblk[:, nlv:, nlv:] = Mloc
        okm = (dv[:, :, None] >= 0) & (dv[:, None, :] >= 0)
        for n in range(1, N):
            for a in range(nq):
                for b in range(nq):
                    coef = -tb.e0[a] * tb.e1[b]
                    if coef == 0.0:
                        continue
                    r = np.broadcast_to((dv * st + n * nq + a)[:, :, None], okm.shape)
                    c = np.broadcast_to((dv * st + (n - 1) * nq + b)[:, None, :], okm.shape)
                    rows.append(r[okm]); cols.append(c[okm]); vals.append(coef * Mblk[okm])
        Jst = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                            shape=(self.n_st, self.n_st))
        Jst.sum_duplicates()
        return Jst


def free_prolongation(fine, coarse):
    """Prolongation between two TaylorHoodLevels in the free numbering: the
    nested-space interpolation of each velocity component restricted to free
    nodes (Dirichlet coarse nodes carry no correction) and the pressure one,
    then the identity over the [slab][temporal node] positions."""
    Pu, Pp = prolongation(fine.M, fine.k)
    ff = np.nonzero(fine.node_free >= 0)[0]
    cf = np.nonzero(coarse.node_free >= 0)[0]
    Puf = Pu[ff][:, cf].tocoo()
    rf, rc = fine.node_free[ff][Puf.row], coarse.node_free[cf][Puf.col]
    Ppc = Pp.tocoo()
    rows = np.concatenate([2 * rf, 2 * rf + 1, fine.p_offset + Ppc.row])
    cols = np.concatenate([2 * rc, 2 * rc + 1, coarse.p_offset + Ppc.col])
    vals = np.concatenate([Puf.data, Puf.data, Ppc.data])
    P = sp.csr_matrix((vals, (rows, cols)), shape=(fine.n_free, coarse.n_free))
    return sp.kron(P, sp.identity(fine.N * fine.nq), format="csr")


def _hierarchy_base():
    from .multigrid import Hierarchy
    return Hierarchy


class TaylorHoodHierarchy(_hierarchy_base()):
    """The multigrid hierarchy of oracle/multigrid.py (V-cycle of Alg. 1,
    WR Vanka+star smoothing, bordered coarsest solve) over TaylorHoodLevels:
    meshes M, M/2, ..., nested-space transfers, the Newton iterate injected at
    the coarse lattice nodes (every coarse node is a fine node)."""

    def __init__(self, M, n_levels, k, q, n_slabs, t_final, mms, opts=None, nodes="radau"):
        from .multigrid import Options
        self.opts = opts or Options()
        self.mms = mms
        self.levels = [TaylorHoodLevel(M >> l, k, q, n_slabs, t_final, mms, nodes)
                       for l in range(n_levels)]
        self.P = [free_prolongation(self.levels[l], self.levels[l + 1]) for l in range(n_levels - 1)]
        self.A = None

    def level_states(self, x_fine):
        out = [x_fine]
        L0 = self.levels[0]
        ux, uy = L0.full_state(x_fine.reshape(L0.n_free, L0.N, L0.nq))
        p = x_fine.reshape(L0.n_free, L0.N, L0.nq)[L0.p_offset:]
        for l in range(1, len(self.levels)):
            F, C = self.levels[l - 1], self.levels[l]

            def inject(n_f, n_c):
                g = np.arange(n_c * n_c)
                return 2 * (g % n_c) + n_f * 2 * (g // n_c)

            iv, ip = inject(F.V.nl, C.V.nl), inject(F.P.nl, C.P.nl)
            ux, uy, p = ux[iv], uy[iv], p[ip]
            fr = C.node_free >= 0
            kf = C.node_free[fr]
            x = np.zeros((C.n_free, C.N, C.nq))
            x[2 * kf] = ux[fr]
            x[2 * kf + 1] = uy[fr]
            x[C.p_offset:] = p
            out.append(x)
        return out
