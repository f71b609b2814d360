"""Seeded synthetic workloads for the space-time Navier-Stokes solver.

This module only draws random numbers and names problem sizes.  It holds none
of the method's arithmetic: the manufactured-solution modes it draws are passed
explicitly, as plain arrays, to both the CPU oracle and the HIP library, so the
two consume identical numbers without sharing any code that computes with them.

Manufactured solution family (stated here so the arrays can be read):

* stream function  psi(t,x,y) = sum_m c_m sin(a_m pi x) sin(b_m pi y) cos(w_m t + th_m)
  with velocity u = (d psi/dy, -d psi/dx); every mode gives u.n = 0 on the
  boundary of the unit square, so the Dirichlet data has zero net flux;
* pressure  p(t,x,y) = sum_m d_m cos(al_m pi x) cos(be_m pi y) cos(w'_m t + th'_m)
  with (al_m, be_m) != (0, 0), so every mode has zero mean over the square.

Arrays: ``psi_ab`` int32 (n_psi, 2) = (a, b); ``psi_coef`` float64 (n_psi, 3)
= (c, w, th); ``p_ab`` int32 (n_p, 2) = (al, be); ``p_coef`` float64 (n_p, 3)
= (d, w', th').
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["Problem", "draw_modes", "named_problem", "batch_problems", "arrival_times",
           "seeded_vector", "chorin_problem", "cavity_problem", "WORKLOADS", "SMOKE", "MEDIUM",
           "LARGE"]


@dataclasses.dataclass
class Problem:
    """One space-time problem on the unit square: Navier-Stokes (equation 0)
    or the heat equation with P_degree elements (equation 1)."""
    mesh_n: int            # finest mesh: mesh_n x mesh_n squares, each cut into 2 triangles
    n_levels: int          # spatial multigrid levels (finest .. mesh_n / 2**(n_levels-1))
    q: int                 # DG degree in time
    n_slabs: int           # N time slabs on [0, t_final]
    t_final: float
    reynolds: float
    psi_ab: np.ndarray
    psi_coef: np.ndarray
    p_ab: np.ndarray
    p_coef: np.ndarray
    seed: int = 0
    flow: int = 0          # 0: manufactured modes; 1: Chorin problem; 2: lid-driven cavity
    nodes: int = 0         # temporal nodes: 0 right Gauss-Radau, 1 Gauss-Legendre
    equation: int = 0      # 0: Navier-Stokes; 1: heat equation
    degree: int = 0        # heat equation: spatial degree k of P_k

    @property
    def n_free_spatial(self) -> int:
        m = self.mesh_n
        if self.equation == 1:
            return (self.degree * m + 1) ** 2
        k = 2 if self.degree == 2 else 1      # Taylor-Hood P_{k+1}-P_k
        return 2 * ((k + 1) * m - 1) ** 2 + (k * m + 1) ** 2

    @property
    def n_st(self) -> int:
        return self.n_free_spatial * self.n_slabs * (self.q + 1)


def draw_modes(seed: int, n_psi: int = 4, n_p: int = 3, max_wave: int = 4,
               omega: float = math.pi):
    """Draw manufactured-solution modes with numpy's default_rng(seed).

    a, b ~ U{1..max_wave}; c = N(0,1) / (pi sqrt(a^2 + b^2)) (so each mode's
    velocity has an N(0,1) amplitude); th ~ U[0, 2 pi); (al, be) ~ U{0..4}^2
    without (0,0); d ~ N(0,1); every temporal frequency is ``omega``.
    """
    rng = np.random.default_rng(seed)
    psi_ab = rng.integers(1, max_wave + 1, size=(n_psi, 2)).astype(np.int32)
    # N(0,1) amplitude of each mode's velocity: the stream-function coefficient
    # is divided by pi * sqrt(a^2 + b^2), so |u_m| ~ |N(0,1)| as in the
    # O(1)-velocity flows the Reynolds numbers refer to
    c = rng.standard_normal(n_psi) / (np.pi * np.sqrt((psi_ab.astype(float) ** 2).sum(axis=1)))
    th = rng.uniform(0.0, 2.0 * math.pi, n_psi)
    psi_coef = np.stack([c, np.full(n_psi, omega), th], axis=1)
    p_ab = np.zeros((n_p, 2), dtype=np.int32)
    for m in range(n_p):
        while True:
            ab = rng.integers(0, 5, size=2)
            if ab[0] != 0 or ab[1] != 0:
                break
        p_ab[m] = ab
    d = rng.standard_normal(n_p)
    thp = rng.uniform(0.0, 2.0 * math.pi, n_p)
    p_coef = np.stack([d, np.full(n_p, omega), thp], axis=1)
    return (np.ascontiguousarray(psi_ab), np.ascontiguousarray(psi_coef),
            np.ascontiguousarray(p_ab), np.ascontiguousarray(p_coef))


# The fixed single-solve workloads, by name: (mesh, levels, q, slabs, Re,
# stream-function modes, highest wave number, base seed); seed = base + index.
WORKLOADS = {
    "ns_p2p1_dg0_m4_n4_re1": (4, 2, 0, 4, 1.0, 4, 4, 0),
    "ns_p2p1_dg1_m32_n32_re100": (32, 4, 1, 32, 100.0, 4, 4, 1000),
    "ns_p2p1_dg1_m128_n64_re1000": (128, 6, 1, 64, 1000.0, 16, 8, 4000),
}
SMOKE = "ns_p2p1_dg0_m4_n4_re1"
MEDIUM = "ns_p2p1_dg1_m32_n32_re100"
LARGE = "ns_p2p1_dg1_m128_n64_re1000"


def named_problem(name: str, index: int = 0) -> Problem:
    """One of the fixed workloads (4x4 smoke solve, 32x32 solve, 128x128 sweep)."""
    if name not in WORKLOADS:
        raise ValueError(f"no fixed workload named {name}")
    mesh, levels, q, slabs, re, n_psi, wave, base = WORKLOADS[name]
    seed = base + index
    modes = draw_modes(seed, n_psi, 3, wave)
    return Problem(mesh, levels, q, slabs, 1.0, re, *modes, seed=seed)


def chorin_problem(mesh_n: int, n_levels: int, q: int, n_slabs: int, reynolds: float = 10.0,
                   t_final: float = 0.1, nodes: int = 1, degree: int = 1) -> Problem:
    """The Chorin test problem on [0, t_final] (the paper's runs: 80 x 80 mesh
    from a 10 x 10 base, 4 levels, R = 10, t in [0, 0.1], N = 10, 20, 40),
    with Gauss-Legendre temporal nodes by default (nodes=0: right Radau);
    degree is the Taylor-Hood pressure degree (1: P2-P1, 2: P3-P2)."""
    none_i = np.zeros((0, 2), dtype=np.int64)
    none_f = np.zeros((0, 3))
    return Problem(mesh_n, n_levels, q, n_slabs, t_final, reynolds, none_i, none_f, none_i, none_f,
                   seed=0, flow=1, nodes=nodes, degree=2 if degree == 2 else 0)


def cavity_problem(mesh_n: int, n_levels: int, q: int, n_slabs: int, reynolds: float,
                   t_final: float = 0.02, nodes: int = 1) -> Problem:
    """The lid-driven cavity on [0, t_final] (the paper's runs: 40 x 40 and
    80 x 80 meshes from a 10 x 10 base, R = 1, 10, 100, t in [0, 0.02],
    N = 20), Gauss-Legendre temporal nodes by default."""
    none_i = np.zeros((0, 2), dtype=np.int64)
    none_f = np.zeros((0, 3))
    return Problem(mesh_n, n_levels, q, n_slabs, t_final, reynolds, none_i, none_f, none_i, none_f,
                   seed=0, flow=2, nodes=nodes)


def heat_problem(mesh_n: int, n_levels: int, degree: int, q: int, n_slabs: int = 20,
                 t_final: float = 0.02, nodes: int = 1) -> Problem:
    """The heat equation with P_degree x DG(q) and the paper's initial data
    sin(pi x) + cos(2 pi y) (its runs: 80 x 80 and 160 x 160 meshes from a
    10 x 10 base, k = 1..3, t in [0, 0.02], N = 20), Gauss-Legendre temporal
    nodes by default.  Nothing is drawn: the problem has no random data."""
    none_i = np.zeros((0, 2), dtype=np.int64)
    none_f = np.zeros((0, 3))
    return Problem(mesh_n, n_levels, q, n_slabs, t_final, 0.0, none_i, none_f, none_i, none_f,
                   seed=0, nodes=nodes, equation=1, degree=degree)


def small_problem(mesh_n: int, n_levels: int, q: int, n_slabs: int,
                  reynolds: float, seed: int, t_final: float = 1.0,
                  n_psi: int = 4, n_p: int = 3, degree: int = 1) -> Problem:
    """A seeded problem of arbitrary (small) size for tests; degree is the
    Taylor-Hood pressure degree k (1: P2-P1, 2: P3-P2)."""
    modes = draw_modes(seed, n_psi, n_p, 4)
    return Problem(mesh_n, n_levels, q, n_slabs, t_final, reynolds, *modes, seed=seed,
                   degree=2 if degree == 2 else 0)


def batch_problems(n: int = 64, seed0: int = 2000, meshes=(8, 16, 32, 64),
                   slab_range=(8, 128), log10_re=(0.0, 3.0)) -> list:
    """The uneven batch: mesh ~ U{meshes}, N ~ U[slab_range], q ~ U{0,1},
    R = 10**U[log10_re]; problem j uses seed seed0 + j.  Levels go down to an
    8x8 coarsest mesh (4x4 for the 8x8 mesh)."""
    out = []
    for j in range(n):
        rng = np.random.default_rng(seed0 + j)
        m = int(rng.choice(meshes))
        nsl = int(rng.integers(slab_range[0], slab_range[1] + 1))
        q = int(rng.integers(0, 2))
        re = float(10.0 ** rng.uniform(log10_re[0], log10_re[1]))
        coarsest = 8 if m >= 16 else 4
        levels = int(round(math.log2(m / coarsest))) + 1
        modes = draw_modes(seed0 + j, 4, 3, 4)
        out.append(Problem(m, levels, q, nsl, 1.0, re, *modes, seed=seed0 + j))
    return out


def arrival_times(rate: float, n: int, seed: int = 3000) -> np.ndarray:
    """Poisson arrivals: cumulative sums of exponential gaps with mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def seeded_vector(n: int, seed: int) -> np.ndarray:
    """n standard normal values from numpy's default generator with this seed
    (a right-hand side or residual for tests and references)."""
    return np.random.default_rng(seed).standard_normal(n)
