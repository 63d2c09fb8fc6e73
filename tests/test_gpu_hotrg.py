"""HOTRG on the GPU (through the C-ABI) against the FP64 oracle and exact
results: single steps on seeded random tensors element by element, whole
Ising runs on gauge-invariant outputs (ln c_n, f, E, M)."""
import math

import numpy as np
import pytest

from oracle import exact, hotrg, ising
from tests.gpu_util import announce, need_gpu
from trg_inputs import random_site_tensor

pytestmark = pytest.mark.gpu


def _oracle_step(T, mu, dcut):
    Tn = T / np.sqrt(np.sum(T * T))
    T2, _, c, choices = hotrg.hotrg_step(Tn, mu, dcut)
    return T2, c, choices


@pytest.mark.parametrize("d,dims,mu,dcut,seed", [
    (2, (3, 4), 0, 6, 1),
    (2, (5, 3), 1, 30, 2),
    (3, (2, 3, 2), 1, 5, 3),
    (3, (3, 2, 3), 0, 4, 4),
    (4, (2, 3, 2, 3), 2, 4, 5),
    (4, (3, 3, 3, 3), 0, 9, 6),
    (4, (4, 4, 4, 4), 3, 6, 7),
    (4, (5, 4, 3, 2), 1, 7, 8),
    # transverse orders 169 and 256 > 160: the selection eigensolver
    # (bisection + inverse iteration), a cut at 14 inside the spectrum
    (2, (13, 16), 0, 14, 9),
    (3, (13, 3, 2), 2, 14, 10),
])
def test_single_step_matches_oracle(d, dims, mu, dcut, seed):
    need_gpu()
    from paper_1911_12954_amd import trg_init_tensor
    announce("single step", d, dims, mu, dcut, seed)
    T = random_site_tensor(dims, seed, positive_bias=True)
    ref, c, choices = _oracle_step(T, mu, dcut)
    ctx = trg_init_tensor(T, precision="fp64")
    ctx.hotrg_step(mu, dcut)
    got = ctx.tensor()
    rec = ctx.step_log()[-1]
    assert got.shape == ref.shape
    assert abs(rec.ln_c - math.log(c)) < 1e-12 * max(1.0, abs(math.log(c)))
    assert np.max(np.abs(got - ref)) < 1e-10
    for ch in choices:
        U, spec = ctx.isometry(ch.nu)
        n = ch.U.shape[0] * ch.U.shape[1]
        assert rec.side[ch.nu] == ch.side and rec.kept[ch.nu] == ch.k
        assert np.max(np.abs(spec - ch.spectrum)) < 1e-13 * max(abs(ch.spectrum[0]), 1e-300)
        assert np.max(np.abs(U - ch.U.reshape(n, ch.k))) < 1e-10
    ctx.close()


@pytest.mark.parametrize("budget", [14_000_000, 30_000_000])
def test_sliced_join_is_bitwise_equal(budget):
    """A small workspace forces the join into x0/x2 slices (14 MB: one value
    of x0 and x2 per slice; 30 MB: ragged slices of x2): the result must not
    change at all."""
    need_gpu()
    from paper_1911_12954_amd import trg_init_tensor
    announce("sliced join", (5, 4, 3, 4), budget)
    T = random_site_tensor((5, 4, 3, 4), 11, positive_bias=True)
    a = trg_init_tensor(T)
    a.hotrg_step(0, 6)
    b = trg_init_tensor(T, workspace_bytes=budget)
    b.hotrg_step(0, 6)
    assert np.array_equal(a.tensor(), b.tensor())
    assert a.step_log()[-1].ln_c == b.step_log()[-1].ln_c


_FP64_REF = {}


def _fp64_ref(*args):
    """FP64 GPU run shared by the parametrised mixed-precision cases."""
    if args not in _FP64_REF:
        _FP64_REF[args] = _gpu_run(*args)
    return _FP64_REF[args]


def _gpu_run(beta, h, d, dcut, L, impure=("E", "M"), precision="fp64"):
    from paper_1911_12954_amd import trg_init_ising
    ctx = trg_init_ising(beta, h, d, dcut=dcut, impure=impure, precision=precision)
    ctx.run(L)
    out = {"f": ctx.free_energy(), "log": ctx.step_log()}
    if "E" in impure:
        out["E"] = ctx.impure_energy()
    if "M" in impure:
        out["M"] = ctx.impure_magnetization()
    ctx.close()
    return out


@pytest.mark.parametrize("h", [0.0, 1e-5])
def test_4d_dcut4_L16_matches_oracle(h):
    """4D Ising, beta = 0.1497, Dcut = 4, 16^4 periodic (16 steps)."""
    need_gpu()
    announce("4d run", 0.1497, h, 4, 16)
    g = _gpu_run(0.1497, h, 4, 4, 16)
    r = hotrg.run(0.1497, h, 4, 4, 16)
    assert abs(g["f"] - r.ln_z_per_site) <= 1e-10 * abs(r.ln_z_per_site)
    assert abs(g["E"] - r.energy) <= 1e-10 * abs(r.energy)
    assert abs(g["M"] - r.magnetization) <= 1e-10 * abs(r.magnetization) + 1e-12
    for gs, rs in zip(g["log"], r.steps[1:]):
        assert abs(gs.ln_c - rs.ln_c) <= 1e-12 * max(1.0, abs(rs.ln_c))


@pytest.mark.parametrize("beta,h", [(0.4407, 0.0), (0.3, 0.1)])
def test_2d_L4_untruncated_equals_brute_force(beta, h):
    need_gpu()
    announce("2d brute", beta, h)
    g = _gpu_run(beta, h, 2, 16, 4)
    lnz, E, M = exact.brute_force(beta, h, 2, 4)
    assert abs(g["f"] - lnz) < 1e-12
    assert abs(g["E"] - E) < 1e-12
    assert abs(g["M"] - M) < 1e-12


def test_3d_L2_untruncated_equals_brute_force():
    need_gpu()
    announce("3d brute")
    g = _gpu_run(0.25, 0.05, 3, 16, 2)
    lnz, E, M = exact.brute_force(0.25, 0.05, 3, 2)
    assert abs(g["f"] - lnz) < 1e-12
    assert abs(g["E"] - E) < 1e-12
    assert abs(g["M"] - M) < 1e-12


def test_4d_two_steps_then_exact_equals_brute_force():
    """Two untruncated GPU steps (x, y) on the 2^4 lattice, then the x/y legs
    closed and the periodic 2x2 (z, t) network contracted exactly on the host."""
    need_gpu()
    from paper_1911_12954_amd import trg_init_ising
    announce("4d brute two steps")
    beta, h = 0.2, 0.1
    ctx = trg_init_ising(beta, h, 4, dcut=256, impure=("E", "M"))
    ctx.hotrg_step(0, 256)
    ctx.hotrg_step(1, 256)
    acc = ctx.accumulator()
    T, SE, SM = ctx.tensor(0), ctx.tensor(1), ctx.tensor(2)
    close = lambda X: np.einsum("aabbcdef->cdef", X)
    Q, QE, QM = close(T), close(SE), close(SM)
    net = lambda A, B, Cc, D: np.einsum("abcd,baef,ghdc,hgfe->", A, B, Cc, D, optimize=True)
    z = net(Q, Q, Q, Q)
    lnz = acc + math.log(z) / 16
    bl, bE, bM = exact.brute_force(beta, h, 4, 2)
    assert abs(lnz - bl) < 1e-12
    assert abs(-net(QE, Q, Q, Q) / z - bE) < 1e-12
    assert abs(net(QM, Q, Q, Q) / z - bM) < 1e-12


@pytest.mark.parametrize("d", [2, 3, 4])
def test_beta_zero_gives_ln2(d):
    need_gpu()
    announce("beta zero", d)
    g = _gpu_run(0.0, 0.3, d, 4, 4, impure=("M",))
    assert abs(g["f"] - math.log(2.0)) < 1e-14
    assert abs(g["M"]) < 1e-14


def test_field_reversal_symmetry():
    need_gpu()
    announce("field reversal")
    a = _gpu_run(0.1497, 1e-3, 4, 4, 4)
    b = _gpu_run(0.1497, -1e-3, 4, 4, 4)
    assert abs(a["f"] - b["f"]) < 1e-13
    assert abs(a["E"] - b["E"]) < 1e-12
    assert abs(a["M"] + b["M"]) < 1e-12


@pytest.mark.parametrize("precision,n64,tol_f,tol_E,tol_M", [("fp32", 0, 1e-6, 1e-6, 1e-3),
                                                           ("bf16x6", 0, 1e-6, 1e-6, 1e-5),
                                                           ("bf16x3", 0, 2e-5, 1e-3, 1e-1),
                                                           ("bf16x3", 8, 1e-6, 1e-3, 1e-1)])
def test_mixed_precision_error_dcut8(precision, n64, tol_f, tol_E, tol_M):
    """4D, Dcut = 8, L = 16, beta = 0.1497, h = 1e-5: f, E, M of the mixed
    joins (optionally with the first n64 steps in FP64) against the GPU FP64
    path.  The FP32 join (FP64 sums of 128-product groups) meets 1e-6 on f
    and E; BF16x3 meets it on f with 8 leading FP64 steps; M near T_c is
    amplified by the field response (errors printed)."""
    need_gpu()
    from paper_1911_12954_amd import trg_init_ising
    announce("mixed dcut8", precision, n64)
    ref = _fp64_ref(0.1497, 1e-5, 4, 8, 16)
    ctx = trg_init_ising(0.1497, 1e-5, 4, dcut=8, impure=("E", "M"), precision=precision, fp64_steps=n64)
    ctx.run(16)
    got = {"f": ctx.free_energy(), "E": ctx.impure_energy(), "M": ctx.impure_magnetization()}
    ctx.close()
    ef = abs(got["f"] - ref["f"]) / abs(ref["f"])
    eE = abs(got["E"] - ref["E"]) / abs(ref["E"])
    eM = abs(got["M"] - ref["M"]) / abs(ref["M"])
    print(f"[mixed {precision} fp64x{n64} dcut8] rel err f {ef:.3e} E {eE:.3e} M {eM:.3e}", flush=True)
    assert ef < tol_f
    assert eE < tol_E and eM < tol_M


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("bf16x6", 1e-4), ("bf16x3", 1e-4)])
def test_mixed_precision_dcut4_degenerate_case(precision, tol):
    """Config of the smoke case (Dcut = 4, L = 16): its truncation at step 3
    goes through an exactly degenerate pair, which the FP64 path (window
    1e-10) and the mixed paths (window 1e-6 after a mixed join) both keep in
    its canonical basis.  At Dcut 4 this run is very sensitive to rounding
    (2^-24 noise on every contracted tensor moves f by 3e-5 in the oracle),
    so every mixed path is held to 1e-4 (measured: FP32 4.2e-5, BF16x3
    3.7e-5, BF16x6 5.6e-8, the last one a fortunate rounding pattern)."""
    need_gpu()
    announce("mixed dcut4", precision)
    ref = _gpu_run(0.1497, 1e-5, 4, 4, 16)
    got = _gpu_run(0.1497, 1e-5, 4, 4, 16, precision=precision)
    ef = abs(got["f"] - ref["f"]) / abs(ref["f"])
    print(f"[mixed {precision} dcut4] rel err f {ef:.3e}", flush=True)
    assert ef < tol


def test_fp64_steps_schedule():
    """fp64_steps = n joins the first n steps in FP64: with n covering the
    whole run the mixed-precision context gives the FP64 bits; with n = 5
    the log shows the switch after step 5."""
    need_gpu()
    from paper_1911_12954_amd import trg_init_ising
    announce("fp64_steps schedule")
    ref = trg_init_ising(0.1497, 1e-5, 4, dcut=5, precision="fp64", impure=("E", "M"))
    ref.run(8)
    for prec in ("fp32", "bf16x3", "bf16x6"):
        a = trg_init_ising(0.1497, 1e-5, 4, dcut=5, precision=prec, impure=("E", "M"), fp64_steps=12)
        a.run(8)
        assert [r.join_precision for r in a.step_log()] == ["fp64"] * 12
        assert (a.free_energy(), a.impure_energy(), a.impure_magnetization()) == \
               (ref.free_energy(), ref.impure_energy(), ref.impure_magnetization())
        a.close()
        b = trg_init_ising(0.1497, 1e-5, 4, dcut=5, precision=prec, impure=("E", "M"), fp64_steps=5)
        b.run(8)
        assert [r.join_precision for r in b.step_log()] == ["fp64"] * 5 + [prec] * 7
        assert abs(b.free_energy() - ref.free_energy()) < 1e-5 * abs(ref.free_energy())
        b.close()
    ref.close()


@pytest.mark.parametrize("name", ["4d_dcut4_L16_h0", "4d_dcut4_L16_h1e-5", "3d_dcut6_L16_h1e-4",
                                  "2d_dcut8_L1024_h0", "4d_dcut6_L16_h1e-5"])
def test_fp64_path_matches_stored_oracle_values(name):
    """The FP64 path against the oracle's stored results (tests/golden)."""
    need_gpu()
    import json
    import os
    from paper_1911_12954_amd import trg_init_ising
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")) as f:
        c = json.load(f)["cases"][name]
    announce("stored oracle values", name)
    ctx = trg_init_ising(c["beta"], c["h"], c["d"], dcut=c["dcut"], precision="fp64", impure=("E", "M"))
    ctx.run(c["L"])
    f_, E, M = ctx.free_energy(), ctx.impure_energy(), ctx.impure_magnetization()
    ctx.close()
    assert abs(f_ - float(c["ln_z_per_site"])) <= 1e-10 * abs(float(c["ln_z_per_site"]))
    assert abs(E - float(c["energy"])) <= 1e-10 * abs(float(c["energy"]))
    m_ref = float(c["magnetization"])
    assert abs(M - m_ref) <= 1e-10 * abs(m_ref) + 1e-12
