"""The degeneracy indicator X on the GPU against the oracle, and the
transition it brackets."""
import math

import numpy as np
import pytest

from oracle import hotrg
from oracle.ising import site_tensors
from tests.gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,dcut,beta,steps", [(4, 4, 0.1497, 12), (3, 6, 0.2216, 9), (2, 8, 0.44, 20)])
def test_indicator_matches_oracle(d, dcut, beta, steps):
    need_gpu()
    from paper_1911_12954_amd import trg_init_ising
    announce("indicator X", d, dcut, beta, steps)
    ctx = trg_init_ising(beta, 0.0, d, dcut=dcut, precision="fp64")
    T = site_tensors(beta, 0.0, d)[0]
    T = T / np.linalg.norm(T)
    for n in range(steps):
        ctx.hotrg_step(n % d, dcut)
        T, _, _, _ = hotrg.hotrg_step(T, n % d, dcut, [], None, "fro", None)
        if n % d == d - 1:
            for axis in range(d):
                assert ctx.indicator_x(axis) == pytest.approx(hotrg.indicator_x(T, axis), rel=1e-9)
    ctx.close()


def test_gpu_bisection_brackets_the_onsager_transition():
    """2D Dcut 8: the GPU bisection takes the oracle's decisions and lands
    within 3e-4 of ln(1 + sqrt 2)/2."""
    need_gpu()
    from paper_1911_12954_amd.scan import bisect_transition
    announce("X bisection 2D Dcut 8")

    def oracle_x(beta):
        T = site_tensors(beta, 0.0, 2)[0]
        T = T / np.linalg.norm(T)
        for n in range(30):
            T, _, _, _ = hotrg.hotrg_step(T, n % 2, 8, [], None, "fro", None)
        return hotrg.indicator_x(T)

    gpu = bisect_transition(2, 8, 0.40, 0.48, 30, 1e-4)
    ref = bisect_transition(2, 8, 0.40, 0.48, 30, 1e-4, evaluate=oracle_x)
    assert (gpu.beta_lo, gpu.beta_hi) == (ref.beta_lo, ref.beta_hi)
    for (b1, x1), (b2, x2) in zip(gpu.evaluations, ref.evaluations):
        assert b1 == b2 and x1 == pytest.approx(x2, rel=1e-9)
    exact = 0.5 * math.log(1.0 + math.sqrt(2.0))
    assert abs(0.5 * (gpu.beta_lo + gpu.beta_hi) - exact) < 3e-4 * exact


@pytest.mark.parametrize("d,dcut,beta,L", [(4, 4, 0.1497, 4), (2, 8, 0.44, 2 ** 6)])
def test_atrg_indicator_matches_oracle(d, dcut, beta, L):
    """X of the factored ATRG tensor against the oracle's X of its own run
    (same trial matrices), on every axis."""
    need_gpu()
    from oracle import atrg
    from paper_1911_12954_amd import trg_init_ising
    announce("atrg indicator", d, dcut, beta, L)
    r = atrg.run(beta, 0.0, d, dcut, L, seed=3)
    ctx = trg_init_ising(beta, 0.0, d, dcut=dcut, method="atrg", seed=3)
    m = L.bit_length() - 1
    for n in range(1, d * m + 1):
        ctx.atrg_step((n - 1) % d, dcut)
    for axis in range(d):
        assert ctx.indicator_x(axis) == pytest.approx(atrg.indicator_x(r.G, r.H, axis), rel=1e-9)
    ctx.close()
