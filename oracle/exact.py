"""Exact references that pin the oracle (test infrastructure).

None of these uses tensor networks; each is an independent statement of the
Ising model's statistical mechanics:

* brute_force    sum over all 2^V spin configurations of a small periodic
                 lattice (bonds counted once per site and axis, so an axis of
                 extent 2 couples a pair twice, as the periodic network does)
* onsager_*      Onsager's exact free energy and internal energy per site of
                 the infinite square lattice, Yang's spontaneous magnetization
* high_temp_lnz  high-temperature (tanh) expansion of ln Z / V
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def brute_force(beta: float, h: float, d: int, L: int):
    """(ln Z / V, <H>/V, <s>) by explicit enumeration; V = L^d <= 20."""
    V = L ** d
    if V > 20:
        raise ValueError("lattice too large for enumeration")
    coords = list(itertools.product(range(L), repeat=d))
    index = {c: i for i, c in enumerate(coords)}
    bonds = []
    for c in coords:
        for mu in range(d):
            nb = list(c)
            nb[mu] = (nb[mu] + 1) % L
            bonds.append((index[c], index[tuple(nb)]))
    bonds = np.array(bonds)
    configs = 1 - 2 * ((np.arange(2 ** V)[:, None] >> np.arange(V)[None, :]) & 1)
    configs = configs.astype(np.float64)
    interaction = np.sum(configs[:, bonds[:, 0]] * configs[:, bonds[:, 1]], axis=1)
    magnet = np.sum(configs, axis=1)
    energy = -interaction - h * magnet
    logw = -beta * energy
    mx = logw.max()
    w = np.exp(logw - mx)
    Z = w.sum()
    lnz = mx + math.log(Z)
    E = float(np.sum(w * energy) / Z)
    M = float(np.sum(w * magnet) / Z)
    return lnz / V, E / V, M / V


def onsager_lnz(K: float) -> float:
    """ln Z / N of the infinite square lattice at coupling K = beta (h = 0).

    Onsager: ln 2 + (1/(8 pi^2)) int int_{[0, 2pi]^2}
    ln[cosh^2 2K - sinh 2K (cos t1 + cos t2)] dt1 dt2.  The t2 integral is
    done in closed form, int_0^{2pi} ln(a - b cos t) dt = 2 pi ln((a +
    sqrt(a^2 - b^2)) / 2) for a >= |b|, leaving one quadrature over t1."""
    from scipy import integrate
    c2, s2 = math.cosh(2 * K) ** 2, math.sinh(2 * K)

    def f(t1):
        a = c2 - s2 * math.cos(t1)
        return math.log(0.5 * (a + math.sqrt(max(a * a - s2 * s2, 0.0))))

    val = integrate.quad(f, 0.0, math.pi, epsabs=1e-15, epsrel=1e-15, limit=400)[0]
    return math.log(2.0) + val / (2.0 * math.pi)


def onsager_energy(K: float) -> float:
    """<H>/N of the infinite square lattice (J = 1, h = 0):
    -coth 2K [1 + (2/pi)(2 tanh^2 2K - 1) K(k)], k = 2 sinh 2K / cosh^2 2K,
    K(k) the complete elliptic integral of the first kind."""
    from scipy.special import ellipk
    k = 2.0 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    return -(1.0 / math.tanh(2 * K)) * (1.0 + (2.0 / math.pi) * (2.0 * math.tanh(2 * K) ** 2 - 1.0) * ellipk(k * k))


def yang_magnetization(K: float) -> float:
    """Spontaneous magnetization (1 - sinh^{-4} 2K)^{1/8} for K > K_c, else 0."""
    s = math.sinh(2 * K)
    return (1.0 - s ** -4) ** 0.125 if s > 1.0 else 0.0


def high_temp_lnz(beta: float, d: int) -> float:
    """Leading terms of ln Z / V at small beta, h = 0, infinite volume:
    ln 2 + d ln cosh beta + (d(d-1)/2) t^4, t = tanh beta (elementary
    plaquettes; the next correction is O(t^6))."""
    t = math.tanh(beta)
    return math.log(2.0) + d * math.log(math.cosh(beta)) + 0.5 * d * (d - 1) * t ** 4
