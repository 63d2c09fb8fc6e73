"""The solve server on the GPU: results in a mix of concurrent, batched runs
are bit-for-bit those of the same runs alone, and one of them matches the
oracle."""
import pytest

from oracle import atrg, hotrg
from tests.gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu

MIX = [
    {"id": 0, "arrival": 0.00, "beta": 0.1490, "h": 0.0, "dcut": 4, "L": 16, "method": "hotrg"},
    {"id": 1, "arrival": 0.00, "beta": 0.1497, "h": 1e-5, "dcut": 4, "L": 16, "method": "hotrg"},
    {"id": 2, "arrival": 0.00, "beta": 0.1505, "h": 1e-6, "dcut": 4, "L": 16, "method": "hotrg"},
    {"id": 3, "arrival": 0.02, "beta": 0.1500, "h": 0.0, "dcut": 5, "L": 4, "method": "hotrg"},
    {"id": 4, "arrival": 0.05, "beta": 0.1495, "h": 1e-5, "dcut": 4, "L": 8, "method": "hotrg"},
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_results_in_the_mix_equal_results_alone(precision):
    need_gpu()
    from paper_1911_12954_amd.serve import Server, TrgBackend
    announce("serve mix", precision)
    srv = Server(TrgBackend(precision), 64 * 2 ** 30)
    out = srv.serve(MIX)
    assert out["completed"] == len(MIX)
    assert out["mean_runs_per_call"] > 1.0       # same-shape steps were batched
    mix = {r["id"]: r["lnz"] for r in srv.results}
    for req in MIX:
        alone = Server(TrgBackend(precision), 64 * 2 ** 30)
        alone.serve([dict(req, arrival=0.0)])
        assert alone.results[0]["lnz"] == mix[req["id"]], req
    if precision == "fp64":
        r = hotrg.run(0.1497, 1e-5, 4, 4, 16, impure=False)
        assert abs(mix[1] - r.ln_z_per_site) <= 1e-10 * abs(r.ln_z_per_site)


def test_shared_workspace_gives_the_same_bits():
    """Two runs stepped in turn on one stream with one shared workspace give
    the bits of the same runs with their own workspaces, also after the
    workspace's creator is freed."""
    need_gpu()
    import torch
    from paper_1911_12954_amd import trg
    announce("shared workspace")
    st = torch.cuda.Stream()
    betas, steps = (0.1490, 0.1500), 13

    def alone(beta):
        c = trg.trg_init_ising(beta, 0.0, 4, dcut=5, precision="fp64", stream=st)
        for n in range(steps):
            c.hotrg_step(n % 4, 5)
        out = c.free_energy()
        c.close()
        return out

    own = [alone(b) for b in betas]
    a, b = (trg.trg_init_ising(x, 0.0, 4, dcut=5, precision="fp64", stream=st) for x in betas)
    trg.trg_share_workspace(b, a)
    for n in range(steps - 1):
        a.hotrg_step(n % 4, 5)
        b.hotrg_step(n % 4, 5)
    a.hotrg_step((steps - 1) % 4, 5)
    fa = a.free_energy()
    a.close()                     # b keeps the shared workspace alive
    b.hotrg_step((steps - 1) % 4, 5)
    fb = b.free_energy()
    b.close()
    assert [fa, fb] == own
    # contexts on different streams cannot share
    e = trg.trg_init_ising(0.15, 0.0, 4, dcut=5, precision="fp64", stream=st)
    other = trg.trg_init_ising(0.15, 0.0, 4, dcut=5, precision="fp64", stream=torch.cuda.Stream())
    with pytest.raises(trg.TrgError):
        trg.trg_share_workspace(e, other)
    other.close()
    e.close()


MIX_METHODS = [
    {"id": 0, "arrival": 0.00, "beta": 0.1490, "h": 0.0, "dcut": 4, "L": 8, "method": "atrg"},
    {"id": 1, "arrival": 0.00, "beta": 0.1497, "h": 1e-3, "dcut": 4, "L": 4, "method": "atrg"},
    {"id": 2, "arrival": 0.00, "beta": 0.1497, "h": 1e-3, "dcut": 4, "L": 4, "method": "hotrg"},
    {"id": 3, "arrival": 0.01, "beta": 0.1505, "h": 0.0, "dcut": 6, "L": 4, "method": "atrg"},
    {"id": 4, "arrival": 0.01, "beta": 0.1500, "h": 0.0, "dcut": 4, "L": 8, "method": "hotrg"},
]


def test_atrg_and_hotrg_requests_in_one_stream():
    """ATRG requests get their own lanes next to the HOTRG ones; every result
    equals the run alone, and an ATRG one equals the oracle (same trial
    matrices, seed 0)."""
    need_gpu()
    from paper_1911_12954_amd.serve import Server, TrgBackend
    announce("serve methods")
    srv = Server(TrgBackend("fp64"), 64 * 2 ** 30)
    out = srv.serve(MIX_METHODS)
    assert out["completed"] == len(MIX_METHODS)
    assert {k[0] for k in srv.lanes} == {"hotrg", "atrg"}
    mix = {r["id"]: r["lnz"] for r in srv.results}
    for req in MIX_METHODS:
        alone = Server(TrgBackend("fp64"), 64 * 2 ** 30)
        alone.serve([dict(req, arrival=0.0)])
        assert alone.results[0]["lnz"] == mix[req["id"]], req
    r = atrg.run(0.1497, 1e-3, 4, 4, 4)
    assert abs(mix[1] - r.ln_z_per_site) <= 1e-10 * abs(r.ln_z_per_site)
