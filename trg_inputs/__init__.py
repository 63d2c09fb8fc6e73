"""Seeded synthetic inputs shared by the oracle tests and the HIP-path tests.

This module holds random numbers and workload descriptions only: no step of
the tensor-network method is computed here.  Both sides of a parity test draw
their inputs from it; neither side's arithmetic lives here.
"""
from __future__ import annotations

import numpy as np


def random_site_tensor(dims, seed: int, positive_bias: bool = False) -> np.ndarray:
    """A dense FP64 site tensor with legs (x, x', y, y', ...), one dim per axis
    (both legs of an axis share it), entries N(0, 1) from a fixed seed.

    With ``positive_bias`` the entries are |N(0,1)|/10 plus 1 on the first
    element, so that Gram spectra resemble a high-temperature Ising tensor (a
    dominant leading eigenvalue and a decaying tail)."""
    shape = tuple(int(x) for x in dims for _ in range(2))
    rng = np.random.default_rng(seed)
    T = rng.standard_normal(shape)
    if positive_bias:
        T = np.abs(T) * 0.1
        T.flat[0] += 1.0
    return T


def random_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    """An FP64 matrix with N(0, 1) entries from a fixed seed."""
    return np.random.default_rng(seed).standard_normal((rows, cols))


def random_symmetric(n: int, seed: int, spread: float = 1.0) -> np.ndarray:
    """A symmetric n x n FP64 matrix (entries N(0,1), symmetrised) plus
    ``spread`` times a diagonal ramp, so that its spectrum is non-degenerate."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = 0.5 * (A + A.T)
    A += spread * np.diag(np.linspace(0.0, float(n), n))
    return A


def gram_like(n: int, rank: int, seed: int) -> np.ndarray:
    """A symmetric positive semidefinite n x n matrix X X^T with X of shape
    n x rank, entries N(0,1) scaled by a geometric decay per column, so the
    spectrum decays like that of a HOSVD environment."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, rank)) * (0.5 ** np.arange(rank))[None, :]
    return X @ X.T


def decaying_site_tensor(dims, seed: int, rank: int = 20, ratio: float = 0.8, noise: float = 1e-3) -> np.ndarray:
    """A site tensor whose HOSVD spectra decay geometrically, as those of the
    Ising tensor do: sum_r ratio^r prod_legs v_{r,leg} with N(0,1) vectors,
    plus `noise` times N(0,1) entries.  One dim per axis, legs (x, x', y, y', ...)."""
    shape = tuple(int(x) for x in dims for _ in range(2))
    rng = np.random.default_rng(seed)
    T = noise * rng.standard_normal(shape)
    for r in range(rank):
        term = np.array(ratio ** r)
        for n in shape:
            term = np.multiply.outer(term, rng.standard_normal(n))
        T += term
    return T


def serving_requests(n: int, rate: float, seed: int, dcuts=(6, 8, 10), kmin: int = 4, kmax: int = 10,
                     fields=(0.0, 1e-6, 1e-5), beta_range=(0.1490, 0.1505), methods=("hotrg",)):
    """A Poisson stream of n solve requests (arrival rate `rate` per
    second): beta ~ U[beta_range], h uniform on `fields`, Dcut uniform on
    `dcuts`, L = 2^k with k ~ U{kmin..kmax}, method uniform on `methods`
    (one method: the stream of a single method).  Returns dicts sorted by
    arrival time (seconds from the start)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for i in range(n):
        out.append({
            "id": i,
            "arrival": float(t[i]),
            "beta": float(rng.uniform(*beta_range)),
            "h": float(fields[rng.integers(len(fields))]),
            "dcut": int(dcuts[rng.integers(len(dcuts))]),
            "L": int(2 ** rng.integers(kmin, kmax + 1)),
            "method": methods[0] if len(methods) == 1 else str(methods[rng.integers(len(methods))]),
        })
    return out
