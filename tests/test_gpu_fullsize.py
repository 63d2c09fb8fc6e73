"""One steady-state HOTRG step at the benchmark's size (4D, every leg at
Dcut = 10, the same chunking of the join) against the oracle, on sampled
output blocks T'[x0, x2, Y, Y', Z, Z', :, :] that the oracle computes one by
one, plus properties that hold at any size.  The input has geometrically
decaying HOSVD spectra (as the Ising tensor has), so that the kept
eigenvectors are well conditioned and an element-by-element comparison is
meaningful (a flat spectrum with relative gaps ~1e-7 would determine them
only to ~2e-9)."""
import math

import numpy as np
import pytest

from oracle import hotrg
from tests.gpu_util import announce, need_gpu
from trg_inputs import decaying_site_tensor

pytestmark = pytest.mark.gpu

D = 10
# (x0, x2, Y, Y', Z, Z'): corners, the ragged last x0 slice and interior values
BLOCKS = [(0, 0, 0, 0, 0, 0), (9, 9, 9, 9, 9, 9), (9, 2, 3, 7, 1, 8), (4, 6, 5, 0, 9, 2)]


@pytest.fixture(scope="module")
def problem():
    T = decaying_site_tensor((D,) * 4, seed=101)
    Tn = T / np.sqrt(np.sum(T * T))
    choices = [hotrg.isometry(Tn, 0, nu, D) for nu in (1, 2, 3)]
    U = {ch.nu: ch.U for ch in choices}
    blocks = {}
    for (x0, x2, y, yp, z, zp) in BLOCKS:
        Ub, Uf = dict(U), dict(U)
        Ub[1], Uf[1] = U[1][:, :, [y]], U[1][:, :, [yp]]
        Ub[2], Uf[2] = U[2][:, :, [z]], U[2][:, :, [zp]]
        blk = hotrg.coarse_grain(Tn, Tn, Ub, 0, x0s=[x0], x2s=[x2], U_forward=Uf)
        blocks[(x0, x2, y, yp, z, zp)] = blk[0, 0, 0, 0, 0, 0]
    return T, choices, blocks


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16x3", 2e-4), ("bf16x6", 1e-5)])
def test_dcut10_step_on_sampled_blocks(problem, precision, tol):
    need_gpu()
    from paper_1911_12954_amd import trg_init_tensor
    T, choices, blocks = problem
    announce("full-size step", precision, "D", D)
    ctx = trg_init_tensor(T, precision=precision)
    ctx.hotrg_step(0, D)
    got = ctx.tensor()
    rec = ctx.step_log()[-1]
    c = math.exp(rec.ln_c)
    # isometries come from FP64 Grams of the same input in every precision
    for ch in choices:
        U, spec = ctx.isometry(ch.nu)
        assert np.max(np.abs(U - ch.U.reshape(D * D, D))) < 1e-10
    worst = 0.0
    for key, ref in blocks.items():
        x0, x2, y, yp, z, zp = key
        blk = c * got[x0, x2, y, yp, z, zp]
        err = np.max(np.abs(blk - ref)) / np.max(np.abs(ref))
        worst = max(worst, err)
    print(f"[full-size {precision}] worst block error {worst:.3e}", flush=True)
    assert worst < tol
    # properties at any size: unit norm, finite, the chosen sides
    assert abs(np.sqrt(np.sum(got * got)) - 1.0) < 1e-12
    assert np.all(np.isfinite(got))
    assert rec.kept[1:] == (D, D, D)
    ctx.close()
