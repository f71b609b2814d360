"""Shared set-up for the GPU parity tests: seeded inputs, the library handle
and the oracle counterpart of the same problem."""
import functools
import sys

import numpy as np
import pytest

import stwr_workloads as w


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def ctx():
    torch_cuda()
    from paper_2407_13997_amd import binding
    return binding.Context(0)


def gpu_problem(prob, **opt):
    from paper_2407_13997_amd import binding
    o = binding.default_opts()
    for k, v in opt.items():
        setattr(o, k, v)
    return binding.Problem(ctx(), prob, o)


def to_dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def seeded(n, seed, scale=1.0):
    return np.random.default_rng(seed).standard_normal(n) * scale


def oracle_hierarchy(prob, **opt):
    from oracle.multigrid import Hierarchy, Options
    return Hierarchy(prob, Options(**opt))


def spacetime_from_bsr(rp, col, val, mass, nf, N, NQ, e0, e1):
    """Assemble the GPU operator (slab blocks + jump coupling) as a scipy matrix."""
    import scipy.sparse as sp
    nnz = len(col)
    rows = np.repeat(np.arange(nf), np.diff(rp))
    V = val.reshape(nnz, N, NQ, NQ)
    st = N * NQ
    R, C, D = [], [], []
    for n in range(N):
        for a in range(NQ):
            for b in range(NQ):
                R.append(rows * st + n * NQ + a)
                C.append(col * st + n * NQ + b)
                D.append(V[:, n, a, b])
    for n in range(1, N):
        for a in range(NQ):
            for b in range(NQ):
                cf = -e0[a] * e1[b]
                if cf == 0.0:
                    continue
                R.append(rows * st + n * NQ + a)
                C.append(col * st + (n - 1) * NQ + b)
                D.append(cf * mass)
    A = sp.csr_matrix((np.concatenate(D), (np.concatenate(R), np.concatenate(C))),
                      shape=(nf * st, nf * st))
    A.sum_duplicates()
    return A


def entrywise(got, want, n_free, N, nq, floor=1e-2):
    """Element-wise errors of a space-time vector [DoF][slab][node]:
    (worst over slabs of max|got - want| / max|want| on that slab,
     worst |got - want| / |want| over the entries with |want| >= floor times
     their slab's largest |want|)."""
    g = np.asarray(got, dtype=float).reshape(n_free, N, nq)
    r = np.asarray(want, dtype=float).reshape(n_free, N, nq)
    d = np.abs(g - r)
    ref = np.abs(r)
    smax = ref.max(axis=(0, 2))
    slab = (d.max(axis=(0, 2)) / np.maximum(smax, 1e-300)).max()
    big = ref >= floor * smax[None, :, None]
    entry = (d[big] / ref[big]).max() if big.any() else 0.0
    return float(slab), float(entry)
