"""ATRG on the GPU (through the C-ABI) against the ATRG oracle and exact
results.  Parity is on gauge-invariant outputs: ln Z/V, ln c_n per step and
the swap's singular values."""
import math

import numpy as np
import pytest

from oracle import atrg, exact
from tests.gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


def _gpu_run(beta, h, d, dcut, L, **cfg):
    from paper_1911_12954_amd import trg_init_ising
    ctx = trg_init_ising(beta, h, d, dcut=dcut, method="atrg", **cfg)
    m = L.bit_length() - 1
    sig = []
    for n in range(1, d * m + 1):
        ctx.atrg_step((n - 1) % d, dcut)
        sig.append(ctx.atrg_spectrum())
    out = {"f": ctx.free_energy(), "log": ctx.step_log(), "sigma": sig}
    ctx.close()
    return out


@pytest.mark.parametrize("beta,h", [(0.4407, 0.0), (0.3, 0.1)])
def test_2d_L4_untruncated_equals_brute_force(beta, h):
    need_gpu()
    announce("atrg 2d brute", beta, h)
    g = _gpu_run(beta, h, 2, 128, 4, rsvd_p=8, rsvd_q=2)
    assert abs(g["f"] - exact.brute_force(beta, h, 2, 4)[0]) < 1e-12


@pytest.mark.parametrize("dcut", [4, 6])
def test_4d_L4_matches_oracle(dcut):
    """Same trial matrices (Philox keyed by seed and step) on both sides."""
    need_gpu()
    announce("atrg 4d L4", dcut)
    g = _gpu_run(0.1497, 1e-3, 4, dcut, 4, seed=5)
    r = atrg.run(0.1497, 1e-3, 4, dcut, 4, seed=5)
    assert abs(g["f"] - r.ln_z_per_site) <= 1e-10 * abs(r.ln_z_per_site)
    for gs, rs in zip(g["log"], r.steps):
        assert abs(gs.ln_c - rs.ln_c) <= 1e-10 * max(1.0, abs(rs.ln_c))
    for gsig, rs in zip(g["sigma"], r.steps):
        assert np.allclose(gsig, rs.swap_sigma, rtol=1e-9, atol=1e-12 * rs.swap_sigma[0])


def test_beta_zero_gives_ln2():
    need_gpu()
    announce("atrg beta 0")
    g = _gpu_run(0.0, 0.2, 4, 4, 4)
    assert abs(g["f"] - math.log(2.0)) < 1e-13


def test_fp32_contraction_error():
    need_gpu()
    announce("atrg fp32 contraction")
    a = _gpu_run(0.1497, 0.0, 4, 6, 16)
    b = _gpu_run(0.1497, 0.0, 4, 6, 16, precision="fp32")
    err = abs(a["f"] - b["f"]) / abs(a["f"])
    print(f"[atrg fp32] rel err f {err:.3e}", flush=True)
    assert err < 1e-6


def test_dcut24_swap_spectrum_on_random_pieces():
    """One step at the production bond dimension from seeded random pieces
    (every leg 24, rank 24, geometrically decaying core): the swap's singular
    values against the oracle's factored randomized SVD with the same trial
    matrix (both sides fix the sign gauge of the canonical form, so the swap
    matrices agree even though two power iterations do not converge this
    flat spectrum), plus the accumulator of the first step."""
    need_gpu()
    from paper_1911_12954_amd import trg_init_factors
    announce("atrg dcut24 random pieces")
    D, d = 24, 4
    rng = np.random.default_rng(17)
    decay = 0.5 ** np.arange(D)
    G = rng.standard_normal((D,) * d + (D,)) * decay
    H = rng.standard_normal((D,) + (D,) * d) * decay.reshape((D,) + (1,) * d)
    ctx = trg_init_factors(G, H, dcut=D, rsvd_p=16, rsvd_q=2, seed=3)
    ctx.atrg_step(0, D)
    sig = ctx.atrg_spectrum()
    F = atrg.canonical(G, H, D)
    X, ref, Y = atrg.rsvd_swap(F, 0, D, 16, 2, 1, 3)
    err = np.max(np.abs(sig - ref)) / ref[0]
    print(f"[atrg dcut24] max |sigma_gpu - sigma_oracle| / sigma_max = {err:.3e}", flush=True)
    assert err < 1e-8
    # the pieces start unnormalised: after one step acc = ln c_1 / 2
    assert abs(ctx.accumulator() - 0.5 * ctx.step_log()[-1].ln_c) < 1e-12
    ctx.close()


# ------------------------------------------------------------ impure tensors ---
def _gpu_impure(beta, h, d, dcut, L, **cfg):
    from paper_1911_12954_amd import trg_init_ising
    ctx = trg_init_ising(beta, h, d, dcut=dcut, method="atrg", impure=("E", "M"), **cfg)
    m = L.bit_length() - 1
    for n in range(1, d * m + 1):
        ctx.atrg_step((n - 1) % d, dcut)
    out = {"f": ctx.free_energy(), "E": ctx.impure_energy(), "M": ctx.impure_magnetization()}
    ctx.close()
    return out


@pytest.mark.parametrize("beta,h", [(0.4407, 0.0), (0.3, 0.05)])
def test_impure_2d_L4_untruncated_equals_brute_force(beta, h):
    """Every partial SVD keeps the whole space: E and M are the spin sums."""
    need_gpu()
    announce("atrg impure 2d brute", beta, h)
    g = _gpu_impure(beta, h, 2, 128, 4, rsvd_p=8, rsvd_q=2)
    lnz, E, M = exact.brute_force(beta, h, 2, 4)
    print(f"[atrg impure 2d] dE {g['E'] - E:.3e} dM {g['M'] - M:.3e}", flush=True)
    assert abs(g["f"] - lnz) < 1e-12
    assert abs(g["E"] - E) < 1e-11 * abs(E)
    assert abs(g["M"] - M) < 1e-11 * max(abs(M), 1.0)


@pytest.mark.parametrize("dcut", [4, 6])
def test_impure_4d_L4_matches_oracle(dcut):
    """Truncated 4D run: the impurity SVDs draw the same trial matrices
    (counter word 1 + 2 kind + term) on both sides."""
    need_gpu()
    announce("atrg impure 4d L4", dcut)
    g = _gpu_impure(0.1497, 1e-3, 4, dcut, 4, seed=5)
    r = atrg.run(0.1497, 1e-3, 4, dcut, 4, seed=5, impure=True)
    print(f"[atrg impure 4d dcut {dcut}] E {g['E']:.12f} / {r.energy:.12f}  M {g['M']:.12f} / "
          f"{r.magnetization:.12f}", flush=True)
    assert abs(g["f"] - r.ln_z_per_site) <= 1e-10 * abs(r.ln_z_per_site)
    assert abs(g["E"] - r.energy) <= 1e-9 * abs(r.energy)
    assert abs(g["M"] - r.magnetization) <= 1e-9 * abs(r.magnetization)


def test_impurities_leave_the_pure_atrg_run_unchanged():
    need_gpu()
    announce("atrg impure pure unchanged")
    a = _gpu_run(0.1497, 1e-3, 4, 4, 4, seed=5)
    b = _gpu_impure(0.1497, 1e-3, 4, 4, 4, seed=5)
    assert a["f"] == b["f"]


@pytest.mark.parametrize("name", ["atrg_4d_dcut4_L4_h1e-3", "atrg_2d_dcut8_L64_h1e-2", "atrg_4d_dcut10_L16_h1e-3"])
def test_impure_matches_stored_oracle_values(name):
    """The GPU path against the stored oracle values of tests/golden
    (written by the oracle alone).  The 4D Dcut 10 case runs at h = 1e-3:
    at h = 1e-5, 0.45 % from the transition, the same run's M (0.011)
    differed between GPU and oracle by 2.0e-11 (1.8e-9 relative) while f
    and E agreed to 1e-10 and 1e-9.  There M is ill-conditioned: in the
    oracle alone a seeded one-ulp perturbation of the initial pieces moves
    it by up to 4e-10 relative (f by 1e-15)."""
    import json
    import os
    need_gpu()
    announce("atrg golden", name)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")) as f:
        c = json.load(f)["cases"][name]
    g = _gpu_impure(c["beta"], c["h"], c["d"], c["dcut"], c["L"], seed=c["seed"])
    assert abs(g["f"] - float(c["ln_z_per_site"])) <= 1e-10 * abs(float(c["ln_z_per_site"]))
    assert abs(g["E"] - float(c["energy"])) <= 1e-9 * abs(float(c["energy"]))
    assert abs(g["M"] - float(c["magnetization"])) <= 1e-9 * abs(float(c["magnetization"]))


def test_impure_fp32_contraction_error():
    """ATRG impurities with the contraction GEMMs in FP32 against FP64 (4D,
    Dcut 6, 16 steps, h = 1e-3)."""
    need_gpu()
    announce("atrg impure fp32 contraction")
    a = _gpu_impure(0.1497, 1e-3, 4, 6, 16)
    b = _gpu_impure(0.1497, 1e-3, 4, 6, 16, precision="fp32")
    err = {k: abs(a[k] - b[k]) / abs(a[k]) for k in ("f", "E", "M")}
    print(f"[atrg impure fp32] rel err {err}", flush=True)
    assert err["f"] < 1e-6 and err["E"] < 1e-4 and err["M"] < 1e-3
