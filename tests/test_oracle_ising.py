"""Pins of the oracle's initial tensors (closed form vs the sum over the spin,
bond-split identity, trace on a one-site lattice, dT0/dbeta)."""
import math

import numpy as np
import pytest

from oracle import ising


@pytest.mark.parametrize("beta", [0.05, 0.1497, 0.44, 1.3])
def test_bond_split_reproduces_bond_weight(beta):
    W = ising.bond_split(beta)
    spins = np.array([1.0, -1.0])
    expect = np.exp(beta * np.outer(spins, spins))
    assert np.allclose(W @ W.T, expect, rtol=1e-15, atol=0)


@pytest.mark.parametrize("d", [2, 3, 4])
@pytest.mark.parametrize("beta,h", [(0.1497, 0.0), (0.1497, 1e-2), (0.4, -0.3), (0.9, 0.05)])
def test_closed_form_equals_spin_sum(d, beta, h):
    a = ising.site_tensors(beta, h, d)
    b = ising.site_tensors_by_spin_sum(beta, h, d)
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) <= 1e-14 * np.max(np.abs(y))


@pytest.mark.parametrize("d", [2, 3, 4])
@pytest.mark.parametrize("beta,h", [(0.1497, 0.0), (0.3, 1e-5), (0.7, -0.2)])
def test_one_site_trace(d, beta, h):
    """On a periodic 1^d lattice every axis couples the spin to itself:
    Z = sum_s e^{beta h s} e^{d beta}."""
    T0, SM, SE = ising.site_tensors(beta, h, d)
    L = "abcd"[:d]
    tr = lambda X: np.einsum("".join(c + c for c in L) + "->", X)
    assert math.isclose(tr(T0), 2 * math.cosh(beta * h) * math.exp(d * beta), rel_tol=1e-14)
    assert math.isclose(tr(SM), 2 * math.sinh(beta * h) * math.exp(d * beta), rel_tol=1e-13, abs_tol=1e-15)
    # dZ/dbeta of that one-site system
    dz = 2 * (h * math.sinh(beta * h) + d * math.cosh(beta * h)) * math.exp(d * beta)
    assert math.isclose(tr(SE), dz, rel_tol=1e-13)


@pytest.mark.parametrize("d", [2, 4])
def test_energy_impurity_is_beta_derivative(d):
    beta, h, eps = 0.1497, 1e-3, 1e-5
    SE = ising.site_tensors(beta, h, d)[2]
    Tp = ising.site_tensors(beta + eps, h, d)[0]
    Tm = ising.site_tensors(beta - eps, h, d)[0]
    fd = (Tp - Tm) / (2 * eps)
    assert np.max(np.abs(fd - SE)) <= 1e-8 * np.max(np.abs(SE))


def test_small_field_keeps_relative_accuracy():
    """The closed form has no e^{bh} - e^{-bh} cancellation: odd entries of
    T0 are exactly proportional to sinh(beta h)."""
    beta, h = 0.1497, 1e-9
    T0 = ising.site_tensors(beta, h, 4)[0]
    ratio = T0[1, 0, 0, 0, 0, 0, 0, 0] / T0[0, 0, 0, 0, 0, 0, 0, 0]
    expect = math.sqrt(math.tanh(beta)) * math.tanh(beta * h)
    assert math.isclose(ratio, expect, rel_tol=1e-14)
