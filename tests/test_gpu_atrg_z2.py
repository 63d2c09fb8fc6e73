"""ATRG in the Z2 mode on the GPU (through the C-ABI) against the oracle's
Z2 mode, brute-force spin sums and the stored oracle values.  The leg and
bond parities are integers and compared exactly; the zeros that the
symmetry puts into the pieces must be exact zeros on the GPU too."""
import json
import os

import numpy as np
import pytest

from oracle import atrg, exact
from tests.gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _gpu_z2(beta, d, dcut, L, impure=(), **cfg):
    from paper_1911_12954_amd import trg_init_ising
    ctx = trg_init_ising(beta, 0.0, d, dcut=dcut, method="atrg", z2=True, impure=impure, **cfg)
    m = L.bit_length() - 1
    sig, par = [], []
    for n in range(1, d * m + 1):
        ctx.atrg_step((n - 1) % d, dcut)
        sig.append(ctx.atrg_spectrum())
        par.append(ctx.atrg_parities())
    G, H = ctx.factors()
    out = {"f": ctx.free_energy(), "log": ctx.step_log(), "sigma": sig, "par": par, "G": G, "H": H,
           "x": ctx.indicator_x(0)}
    if impure:
        out["E"], out["M"] = ctx.impure_energy(), ctx.impure_magnetization()
    ctx.close()
    return out


def _assert_exact_zeros(G, H, legs, bond):
    """G[b, l] and H[l, f] are exactly zero unless the parities of the legs
    add up to the bond's."""
    rp = atrg.composite_parity(legs)
    r = len(bond)
    Gm, Hm = G.reshape(-1, r), H.reshape(r, -1)
    wrong = rp[:, None] != np.asarray(bond)[None, :]
    assert np.all(Gm[wrong] == 0.0)
    assert np.all(Hm.T[wrong] == 0.0)
    # and the allowed entries are not all zero (the check is not vacuous)
    assert np.count_nonzero(Gm[~wrong]) > 0


def _assert_bond_parities_match(gbond, gsig, obond, osig):
    """The parity of each new bond index, where it is unique: a singular
    value at the rounding level (a rank-deficient swap) has a singular vector
    of either parity, and two singular values closer than the rounding of
    the two computations may come in either order.  Returns the number of
    indices compared."""
    assert len(gbond) == len(obond) == len(gsig) == len(osig)
    n = 0
    for i, s in enumerate(osig):
        if s <= 1e-10 * osig[0]:
            continue
        if any(abs(s - osig[j]) <= 1e-8 * s for j in range(len(osig)) if j != i):
            continue
        assert gbond[i] == obond[i], (i, list(gbond), list(obond))
        n += 1
    return n


@pytest.mark.parametrize("d,L,beta", [(2, 4, 0.3), (2, 4, 0.6), (3, 2, 0.25)])
def test_z2_untruncated_equals_brute_force(d, L, beta):
    need_gpu()
    announce("atrg z2 brute", d, L, beta)
    g = _gpu_z2(beta, d, 128, L, rsvd_p=8, rsvd_q=2)
    assert abs(g["f"] - exact.brute_force(beta, 0.0, d, L)[0]) < 1e-12
    legs, bond = g["par"][-1]
    _assert_exact_zeros(g["G"], g["H"], legs, bond)


@pytest.mark.parametrize("dcut", [4, 6])
def test_z2_4d_L4_matches_oracle(dcut):
    """Same trial matrices (Philox keyed by seed and step, masked by the same
    sectors) on both sides: ln Z/V, ln c_n and the swap spectrum per step,
    the parities of every leg and bond index after every step (exactly), and
    exact zeros in the GPU pieces."""
    need_gpu()
    announce("atrg z2 4d L4", dcut)
    g = _gpu_z2(0.1497, 4, dcut, 4, seed=5)
    r = atrg.run(0.1497, 0.0, 4, dcut, 4, seed=5, z2=True)
    assert abs(g["f"] - r.ln_z_per_site) <= 1e-10 * abs(r.ln_z_per_site)
    for gs, rs in zip(g["log"], r.steps):
        assert abs(gs.ln_c - rs.ln_c) <= 1e-10 * max(1.0, abs(rs.ln_c))
    for gsig, rs in zip(g["sigma"], r.steps):
        assert np.allclose(gsig, rs.swap_sigma, rtol=1e-9, atol=1e-12 * rs.swap_sigma[0])
    checked = 0
    for (glegs, gbond), gsig, rs in zip(g["par"], g["sigma"], r.steps):
        assert [list(x) for x in glegs] == [list(x) for x in rs.legs]
        checked += _assert_bond_parities_match(gbond, gsig, rs.bond, rs.swap_sigma)
    assert checked >= 2 * len(r.steps)
    legs, bond = g["par"][-1]
    _assert_exact_zeros(g["G"], g["H"], legs, bond)


def test_z2_symmetric_fixed_point_4d_L1024():
    """4D, beta = 0.2 (ordered phase), h = 0, Dcut 6, L = 1024 (40 steps),
    impure E and M: the GPU's Z2 run keeps the tensor symmetric, so M = 0
    and X = 2 (Sec. 3.1-3.2), and ln Z/V and E agree with the stored oracle
    values of the same run."""
    need_gpu()
    announce("atrg z2 fixed point beta 0.2 dcut 6 L1024")
    with open(os.path.join(HERE, "golden", "oracle_values.json")) as f:
        c = json.load(f)["cases"]["atrg_z2_4d_dcut6_L1024_b0.2"]
    g = _gpu_z2(c["beta"], c["d"], c["dcut"], c["L"], impure=("E", "M"), seed=c["seed"])
    print(f"[atrg z2 L1024] f {g['f']!r} E {g['E']!r} M {g['M']!r} X {g['x']!r}", flush=True)
    assert abs(g["M"]) < 1e-12
    assert abs(g["x"] - 2.0) < 1e-10
    assert abs(g["f"] - float(c["ln_z_per_site"])) <= 1e-10 * abs(float(c["ln_z_per_site"]))
    assert abs(g["E"] - float(c["energy"])) <= 1e-8 * abs(float(c["energy"]))
    legs, bond = g["par"][-1]
    _assert_exact_zeros(g["G"], g["H"], legs, bond)


def test_z2_disordered_phase_gives_x_one():
    """4D, beta = 0.12 (disordered), h = 0, Dcut 4, L = 1024: X -> 1."""
    need_gpu()
    announce("atrg z2 disordered beta 0.12")
    g = _gpu_z2(0.12, 4, 4, 1024)
    assert abs(g["x"] - 1.0) < 1e-6


def test_z2_checkpoint_resume_is_bitwise():
    """Export after 3 steps, import, continue: the parities travel with the
    state and the resumed run ends on the bits of the uninterrupted one."""
    need_gpu()
    from paper_1911_12954_amd import trg_import_state, trg_init_ising
    announce("atrg z2 checkpoint")
    cfg = dict(dcut=6, method="atrg", z2=True, impure=("E", "M"), seed=3)

    def steps(ctx, first, last):
        for n in range(first, last):
            ctx.atrg_step(n % 4, 6)

    a = trg_init_ising(0.1497, 0.0, 4, **cfg)
    steps(a, 0, 8)
    straight = (a.free_energy(), a.impure_energy(), a.impure_magnetization(), a.atrg_parities())
    a.close()
    b = trg_init_ising(0.1497, 0.0, 4, **cfg)
    steps(b, 0, 3)
    blob = b.export_state()
    b.close()
    c2 = trg_import_state(blob)
    steps(c2, 3, 8)
    resumed = (c2.free_energy(), c2.impure_energy(), c2.impure_magnetization(), c2.atrg_parities())
    c2.close()
    assert resumed[:3] == straight[:3]
    assert [list(x) for x in resumed[3][0]] == [list(x) for x in straight[3][0]]
    assert list(resumed[3][1]) == list(straight[3][1])
