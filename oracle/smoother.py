"""Waveform-relaxation Vanka+star smoother, Chebyshev acceleration and the
eigenvalue estimate (oracle), Sec. 3.

* Patch operator (eq. waveform_patch_solve): for every vertex patch S_v the
  space-time patch matrix A_v = R_v A R_v^T is extracted algebraically from the
  assembled space-time matrix; it is block lower bidiagonal in the slabs, so
  A_v^{-1} r is computed by forward block substitution with one LU per slab
  block.  The smoother is additive and unweighted: z = sum_v R_v^T A_v^{-1} R_v r
  (the fixed linear operator that Chebyshev weighting requires).
* Chebyshev acceleration over [a, b] = [0.25 lam, 1.05 lam] of the
  relaxation-preconditioned operator (the classical three-term recurrence of
  Saad, Iterative Methods, Ch. 12), one sweep = one residual + one patch solve.
* lam = largest real part of the Ritz values after 10 Arnoldi (GMRES) steps on
  M^{-1} A from a fixed start vector v0[i] = frac(i * 0.6180339887498949) - 0.5
  (the paper does not state the start vector; this one is a reading).
"""
import numpy as np
import scipy.linalg as la


class PatchSmoother:
    def __init__(self, level, A, patches=None):
        self.level = level
        N, nq = level.N, level.nq
        self.N, self.nq = N, nq
        self.patches = level.mesh.patches() if patches is None else patches
        st = N * nq
        self.blocks = []
        A = A.tocsr()
        for S in self.patches:
            idx = (S[:, None] * st + np.arange(st)[None, :]).ravel()   # [dof][n][a]
            Ap = A[idx][:, idx].toarray()
            nb = len(S)
            # reorder to slab-major: [n][dof][a]
            perm = (np.arange(nb)[None, :, None] * st + np.arange(N)[:, None, None] * nq
                    + np.arange(nq)[None, None, :]).ravel()
            Ap = Ap[np.ix_(perm, perm)]
            k = nb * nq
            lus, subs = [], []
            for n in range(N):
                lus.append(la.lu_factor(Ap[n * k:(n + 1) * k, n * k:(n + 1) * k]))
                # a copy: a view would keep the whole dense patch matrix alive
                subs.append(Ap[n * k:(n + 1) * k, (n - 1) * k:n * k].copy() if n > 0 else None)
            self.blocks.append((idx, perm, lus, subs, k))

    def patch_solve(self, i, rp_slab_major):
        """Forward block substitution for patch i (input/output slab-major)."""
        idx, perm, lus, subs, k = self.blocks[i]
        y = np.zeros_like(rp_slab_major)
        for n in range(self.N):
            g = rp_slab_major[n * k:(n + 1) * k].copy()
            if n > 0:
                g -= subs[n] @ y[(n - 1) * k:n * k]
            y[n * k:(n + 1) * k] = la.lu_solve(lus[n], g)
        return y

    def apply(self, r):
        """z = sum over patches of R_v^T A_v^{-1} R_v r, r of length n_st."""
        r = np.asarray(r).ravel()
        z = np.zeros_like(r)
        for i, (idx, perm, lus, subs, k) in enumerate(self.blocks):
            rp = r[idx][perm]
            y = self.patch_solve(i, rp)
            out = np.empty_like(y)
            out[perm] = y
            np.add.at(z, idx, out)
        return z


def chebyshev(A, Minv, b, x, n_steps, a, bnd):
    """n_steps Chebyshev-accelerated relaxation sweeps on A x = b over [a, bnd]."""
    theta = 0.5 * (a + bnd)
    delta = 0.5 * (bnd - a)
    x = x.copy()
    d = None
    rho_old = None
    for k in range(n_steps):
        z = Minv(b - A @ x)
        if k == 0:
            rho = delta / theta
            d = z / theta
        else:
            rho = 1.0 / (2.0 * theta / delta - rho_old)
            d = rho * rho_old * d + (2.0 * rho / delta) * z
        x = x + d
        rho_old = rho
    return x


def start_vector(n):
    i = np.arange(n, dtype=np.float64)
    v = np.mod(i * 0.6180339887498949, 1.0) - 0.5
    return v / np.linalg.norm(v)


def eig_estimate(A, Minv, n, steps=10):
    """Largest real Ritz value of M^{-1} A after ``steps`` Arnoldi steps (MGS)."""
    V = np.zeros((steps + 1, n))
    H = np.zeros((steps + 1, steps))
    V[0] = start_vector(n)
    m = steps
    for j in range(steps):
        w = Minv(A @ V[j])
        for i in range(j + 1):
            H[i, j] = np.dot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] <= 1e-14 * abs(H[0, 0]):
            m = j + 1
            break
        V[j + 1] = w / H[j + 1, j]
    ev = np.linalg.eigvals(H[:m, :m])
    return float(np.max(ev.real))
