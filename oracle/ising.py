"""Initial site tensors of the d-dimensional Ising model (oracle, test infrastructure).

The paper (Sec. 1 and 3.1) studies the ferromagnetic Ising model on a
hypercubic lattice but does not write its Hamiltonian, the coupling, the field
convention or the initial tensor.  Readings used here:

* Weight e^{-beta H}, H = -sum_{i,mu} s_i s_{i+mu} - h sum_i s_i, J = 1, T = 1/beta.
* Each bond weight e^{beta s s'} is split symmetrically,
  e^{beta s s'} = sum_k W[s,k] W[s',k], with
  W = [[sqrt(cosh b), sqrt(sinh b)], [sqrt(cosh b), -sqrt(sinh b)]],
  rows s = +1, -1.
* Site tensor legs in the order (x, x', y, y', z, z', t, t'): for every axis
  the backward leg comes before the forward leg.
* T0  = sum_s e^{beta h s}     prod_l W[s, i_l]
  S_M = sum_s s e^{beta h s}   prod_l W[s, i_l]         (magnetization impurity)
  S_E = d T0 / d beta                                    (energy impurity)

Two evaluations are given.  ``site_tensors_by_spin_sum`` is the sum over s as
written above; ``site_tensors`` uses its closed form.  With n the number of
legs carrying index 1, prod_l W[s,i_l] = cosh^{(2d-n)/2} b sinh^{n/2} b s^n,
and the sum over s gives 2 cosh(beta h) (n even) or 2 sinh(beta h) (n odd).
The closed form avoids the cancellation e^{bh} - e^{-bh} of the literal sum at
small h, which costs about 1e-16/(beta h) relative accuracy.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def bond_split(beta: float) -> np.ndarray:
    """W with sum_k W[s,k] W[s',k] = exp(beta s s'); rows s=+1, s=-1."""
    c, s = math.sqrt(math.cosh(beta)), math.sqrt(math.sinh(beta))
    return np.array([[c, s], [c, -s]], dtype=np.float64)


def bond_split_dbeta(beta: float) -> np.ndarray:
    """Elementwise d W / d beta (requires beta > 0)."""
    ch, sh = math.cosh(beta), math.sinh(beta)
    dc = sh / (2.0 * math.sqrt(ch))
    ds = ch / (2.0 * math.sqrt(sh))
    return np.array([[dc, ds], [dc, -ds]], dtype=np.float64)


def site_tensors_by_spin_sum(beta: float, h: float, d: int):
    """T0, S_M, S_E by the literal sum over the site spin s = +1, -1.

    S_E differentiates every beta dependence: the field factor and each of the
    2d bond-split legs (product rule).  Needs beta > 0 for S_E.
    """
    W = bond_split(beta)
    nl = 2 * d
    T0 = np.zeros((2,) * nl)
    SM = np.zeros((2,) * nl)
    SE = np.zeros((2,) * nl)
    dW = bond_split_dbeta(beta) if beta > 0 else None
    for row, spin in enumerate((1.0, -1.0)):
        w = math.exp(beta * h * spin)
        for idx in itertools.product((0, 1), repeat=nl):
            prod = 1.0
            for i in idx:
                prod *= W[row, i]
            T0[idx] += w * prod
            SM[idx] += spin * w * prod
            if dW is not None:
                der = h * spin * prod
                for l in range(nl):
                    p = dW[row, idx[l]]
                    for m in range(nl):
                        if m != l:
                            p *= W[row, idx[m]]
                    der += p
                SE[idx] += w * der
    return T0, SM, SE


def site_tensors(beta: float, h: float, d: int):
    """T0, S_M, S_E from the closed form in the module docstring.

    S_E = 2 c^a s^b [(a tanh b + b coth b) g(beta h) + h g'(beta h)] with
    c = cosh b, s = sinh b, a = (2d-n)/2, b = n/2, g = cosh (n even) or
    sinh (n odd).  S_E needs beta > 0 (sqrt(sinh b) is not differentiable at 0);
    for beta = 0 it is returned as NaN where undefined.
    """
    nl = 2 * d
    ch, sh = math.cosh(beta), math.sinh(beta)
    chh, shh = math.cosh(beta * h), math.sinh(beta * h)
    T0 = np.zeros((2,) * nl)
    SM = np.zeros((2,) * nl)
    SE = np.zeros((2,) * nl)
    for idx in itertools.product((0, 1), repeat=nl):
        n = sum(idx)
        a, b = (nl - n) / 2.0, n / 2.0
        base = 2.0 * ch ** a * sh ** b
        even = n % 2 == 0
        g, gp = (chh, shh) if even else (shh, chh)
        T0[idx] = base * g
        SM[idx] = base * gp
        if beta > 0:
            SE[idx] = base * ((a * math.tanh(beta) + b / math.tanh(beta)) * g + h * gp)
        else:
            SE[idx] = float("nan") if n > 0 else base * h * gp
    return T0, SM, SE
