"""Heat equation with P_k x DG(q) and its waveform-relaxation multigrid
solver (oracle; test infrastructure only, never part of the product path).

* Discretisation (Sec. 2, Definition of the heat equation, eq. heatfem):
  u_t - Laplace u = 0 on the unit square, natural (homogeneous Neumann)
  boundary conditions, continuous Lagrange P_k in space (k = 1, 2, 3) and
  upwind DG(q) in time.  Per slab the operator is T (x) M + dt W (x) K with
  the spatial mass M and stiffness K and the temporal matrices of
  ``SlabBasis``; slab n couples to slab n-1 through -e0 e1^T (x) M.  With the
  [DoF][slab][node] layout the space-time matrix is
  kron(M, S_M) + kron(K, S_K), S_M = blockdiag(T) - subdiag(e0 e1^T),
  S_K = dt blockdiag(W).  The right-hand side is e0 (x) M U_0 on slab 0,
  U_0 the nodal interpolant of u_0.
* Mesh (Sec. 4): the triangle-split unit square of ``oracle.mesh``.  The P_k
  nodes of all cells are the points of the (kM+1)^2 lattice of spacing h/k;
  node g = gi + (kM+1) gj.  Every node is an unknown (no Dirichlet data).
* Patches (Sec. 3, the vertex-star relaxation of Fig. patches, left): one
  per vertex, the vertex itself and the nodes interior to its incident
  edges and cells, i.e. every node of an incident cell whose barycentric
  coordinate for the vertex is positive; 3k^2 - 3k + 1 nodes at an interior
  vertex.
* Solver (Sec. 4.1): FGMRES right-preconditioned by one V-cycle of Alg. 1
  with Chebyshev-accelerated additive patch relaxation, stopped when the
  residual falls by 1e-6 or below 1e-6 in norm.
* Initial data of the paper's runs: u_0 = sin(pi x) + cos(2 pi y).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import Mesh
from .multigrid import Options, fgmres
from .quadrature import duffy_triangle
from .smoother import PatchSmoother, chebyshev, eig_estimate
from .temporal import SlabBasis


def local_nodes(k):
    """Reference-triangle lattice nodes (a, b) / k, a + b <= k, b outer."""
    return [(a, b) for b in range(k + 1) for a in range(k + 1 - b)]


def lagrange_pk(k, pts):
    """Values (n, nloc) and reference gradients (n, nloc, 2) of the P_k
    Lagrange basis on the equispaced nodes, from the inverse of the monomial
    Vandermonde matrix (column i of the inverse holds basis function i's
    monomial coefficients)."""
    pts = np.atleast_2d(np.asarray(pts, dtype=float))
    mono = [(p, r) for p in range(k + 1) for r in range(k + 1 - p)]
    nod = np.array(local_nodes(k), dtype=float) / k
    V = np.array([[x ** p * y ** r for (p, r) in mono] for x, y in nod])
    C = np.linalg.inv(V)                       # (nmono, nloc)
    x, y = pts[:, 0], pts[:, 1]
    mv = np.stack([x ** p * y ** r for (p, r) in mono], axis=1)
    mx = np.stack([p * x ** max(p - 1, 0) * y ** r if p > 0 else 0.0 * x for (p, r) in mono], axis=1)
    my = np.stack([r * x ** p * y ** max(r - 1, 0) if r > 0 else 0.0 * x for (p, r) in mono], axis=1)
    return mv @ C, np.stack([mx @ C, my @ C], axis=2)


class HeatSpace:
    """P_k on the triangle-split M x M mesh, lattice node numbering."""

    def __init__(self, M, k):
        self.mesh = Mesh(M)
        self.M, self.k, self.h = M, k, 1.0 / M
        nl = k * M + 1
        self.nl = nl
        self.n = nl * nl
        g = np.arange(self.n)
        self.xy = np.stack([(g % nl) * self.h / k, (g // nl) * self.h / k], axis=1)
        loc = np.array(local_nodes(k))
        cells = self.mesh.cells
        n1 = self.mesh.n1
        vi, vj = cells[:, 0] % n1, cells[:, 0] // n1
        lower = np.arange(self.mesh.nc) % 2 == 0
        gi = np.where(lower[:, None], k * vi[:, None] + loc[None, :, 0], k * vi[:, None] - loc[None, :, 0])
        gj = np.where(lower[:, None], k * vj[:, None] + loc[None, :, 1], k * vj[:, None] - loc[None, :, 1])
        self.cell_nodes = gi + nl * gj             # (nc, nloc)
        self.loc = loc

    def patches(self):
        """Vertex-star patches: sorted node lists, one per vertex."""
        k = self.k
        lam = np.stack([k - self.loc[:, 0] - self.loc[:, 1], self.loc[:, 0], self.loc[:, 1]], axis=1)
        sets = [set() for _ in range(self.mesh.nv)]
        for c in range(self.mesh.nc):
            for corner in range(3):
                v = self.mesh.cells[c, corner]
                sets[v].update(self.cell_nodes[c, lam[:, corner] > 0].tolist())
        return [np.array(sorted(s), dtype=np.int64) for s in sets]

    def matrices(self):
        """Spatial mass M and stiffness K (CSR), by the degree-8 rule."""
        pts, w = duffy_triangle(5)
        val, grad = lagrange_pk(self.k, pts)
        m = self.mesh
        nloc = self.cell_nodes.shape[1]
        rows, cols, mv, kv = [], [], [], []
        for c in range(m.nc):
            v = m.vxy[m.cells[c]]
            J = np.stack([v[1] - v[0], v[2] - v[0]], axis=1)
            det = abs(np.linalg.det(J))
            G = grad @ np.linalg.inv(J)                 # physical gradients (nq, nloc, 2)
            Me = np.einsum("q,qi,qj->ij", w * det, val, val)
            Ke = np.einsum("q,qid,qjd->ij", w * det, G, G)
            nodes = self.cell_nodes[c]
            rows.append(np.repeat(nodes, nloc))
            cols.append(np.tile(nodes, nloc))
            mv.append(Me.ravel())
            kv.append(Ke.ravel())
        r, cc = np.concatenate(rows), np.concatenate(cols)
        Mm = sp.csr_matrix((np.concatenate(mv), (r, cc)), shape=(self.n, self.n))
        Km = sp.csr_matrix((np.concatenate(kv), (r, cc)), shape=(self.n, self.n))
        Mm.sum_duplicates()
        Km.sum_duplicates()
        return Mm, Km

    def prolongation(self, coarse):
        """Nodal interpolation of the coarse P_k space (mesh 2h) at the fine
        nodes: P[f, c] = phi_c(x_f)."""
        cm = coarse.mesh
        h = cm.h
        pts = self.xy
        i = np.minimum((pts[:, 0] / h).astype(int), cm.M - 1)
        j = np.minimum((pts[:, 1] / h).astype(int), cm.M - 1)
        fx, fy = pts[:, 0] / h - i, pts[:, 1] / h - j
        upper = fx + fy > 1.0 + 1e-12
        cell = 2 * (i + cm.M * j) + upper.astype(int)
        v = cm.vxy[cm.cells[cell]]
        Jc = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)
        ref = np.linalg.solve(Jc, (pts - v[:, 0])[..., None])[..., 0]
        rows, cols, vals = [], [], []
        for f in range(self.n):
            phi, _ = lagrange_pk(self.k, ref[f])
            nz = np.abs(phi[0]) > 1e-14
            rows.append(np.full(int(nz.sum()), f))
            cols.append(coarse.cell_nodes[cell[f], nz])
            vals.append(phi[0, nz])
        P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.n, coarse.n))
        P.sum_duplicates()
        return P


def initial_value(x, y):
    """u_0 of the paper's heat runs (Sec. 4.1)."""
    return np.sin(np.pi * x) + np.cos(2.0 * np.pi * y)


class HeatLevel:
    """One level of the heat problem: space, slab basis, space-time matrix."""

    def __init__(self, M, k, q, N, t_final, nodes="radau"):
        self.space = HeatSpace(M, k)
        self.mesh = self.space.mesh
        self.k, self.q, self.N = k, q, N
        self.nq = q + 1
        self.dt = t_final / N
        self.basis = SlabBasis(q, nodes)
        self.n_free = self.space.n
        self.n_st = self.n_free * N * self.nq
        self.Ms, self.Ks = self.space.matrices()
        b = self.basis
        nt = N * self.nq
        SM = np.zeros((nt, nt))
        SK = np.zeros((nt, nt))
        for n in range(N):
            s = slice(n * self.nq, (n + 1) * self.nq)
            SM[s, s] = b.T
            SK[s, s] = self.dt * b.W
            if n > 0:
                SM[s, (n - 1) * self.nq:n * self.nq] = -np.outer(b.e0, b.e1)
        self.A = (sp.kron(self.Ms, sp.csr_matrix(SM)) + sp.kron(self.Ks, sp.csr_matrix(SK))).tocsr()

    def rhs(self, u0=initial_value):
        """e0 (x) M U_0 on slab 0, zero elsewhere."""
        U0 = u0(self.space.xy[:, 0], self.space.xy[:, 1])
        b = np.zeros((self.n_free, self.N, self.nq))
        b[:, 0, :] = np.outer(self.Ms @ U0, self.basis.e0)
        return b.ravel()

    def end_values(self, x):
        """Slab-end values (N, n_free) of a space-time vector."""
        X = np.asarray(x).reshape(self.n_free, self.N, self.nq)
        return (X @ self.basis.e1).T


class HeatHierarchy:
    """Rediscretised levels M, M/2, ..., transfers P = P_h (x) I, vertex-star
    smoothers with their eigen-estimates, and an exact coarsest solve."""

    def __init__(self, M, n_levels, k, q, N, t_final, opts=None, nodes="radau"):
        self.opts = opts or Options()
        self.levels = [HeatLevel(M >> l, k, q, N, t_final, nodes) for l in range(n_levels)]
        nt = N * (q + 1)
        self.P = [sp.kron(self.levels[l].space.prolongation(self.levels[l + 1].space),
                          sp.identity(nt), format="csr") for l in range(n_levels - 1)]
        self.A = [lev.A for lev in self.levels]
        self.smoothers, self.lams = [], []
        for l in range(n_levels - 1):
            lev = self.levels[l]
            sm = PatchSmoother(lev, lev.A, patches=lev.space.patches())
            self.smoothers.append(sm)
            self.lams.append(eig_estimate(lev.A, sm.apply, lev.n_st, self.opts.eig_steps))
        self.coarse = spla.splu(self.A[-1].tocsc())

    def relax(self, l, b, x, n_steps):
        lam = self.lams[l]
        return chebyshev(self.A[l], self.smoothers[l].apply, b, x, n_steps,
                         self.opts.cheb_lo * lam, self.opts.cheb_hi * lam)

    def vcycle(self, b, l=0):
        """Alg. 1, as for the Navier-Stokes hierarchy."""
        if l == len(self.levels) - 1:
            return self.coarse.solve(b)
        x = self.relax(l, b, np.zeros_like(b), self.opts.nu_pre)
        r = b - self.A[l] @ x
        xc = self.vcycle(self.P[l].T @ r, l + 1)
        x = x + self.P[l] @ xc
        return self.relax(l, b, x, self.opts.nu_post)


def heat_solve(M, n_levels, k, q, N=20, t_final=0.02, rtol=1e-6, atol=1e-6, opts=None,
               nodes="gauss"):
    """FGMRES-WRMG solve of the paper's heat problem; returns
    (x, iterations, residual history, hierarchy)."""
    H = HeatHierarchy(M, n_levels, k, q, N, t_final, opts, nodes)
    o = H.opts
    b = H.levels[0].rhs()
    x, its, hist = fgmres(H.A[0], H.vcycle, b, rtol, o.gmres_restart, o.gmres_maxit, atol=atol)
    return x, its, hist, H
