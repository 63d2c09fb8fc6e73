"""Checkpoint and resume through the C-ABI: a run exported after step k,
freed, imported and continued gives the bits of the uninterrupted run."""
import pytest

from tests.gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


def _steps(ctx, method, d, dcut, first, last):
    for n in range(first, last):
        if method == "atrg":
            ctx.atrg_step(n % d, dcut)
        else:
            ctx.hotrg_step(n % d, dcut)


def _observables(ctx):
    return (ctx.free_energy(), ctx.impure_energy(), ctx.impure_magnetization(),
            [r.ln_c for r in ctx.step_log()])


@pytest.mark.parametrize("method,precision,dcut,nsteps,k", [
    ("hotrg", "fp64", 4, 12, 5), ("hotrg", "bf16x3", 5, 9, 4), ("atrg", "fp64", 4, 8, 3)])
def test_resume_reproduces_the_run_bitwise(method, precision, dcut, nsteps, k):
    need_gpu()
    from paper_1911_12954_amd import trg_import_state, trg_init_ising
    announce("checkpoint", method, precision, dcut, nsteps, k)
    cfg = dict(dcut=dcut, precision=precision, method=method, impure=("E", "M"), seed=7)
    a = trg_init_ising(0.1497, 1e-4, 4, **cfg)
    _steps(a, method, 4, dcut, 0, nsteps)
    straight = _observables(a)
    a.close()
    b = trg_init_ising(0.1497, 1e-4, 4, **cfg)
    _steps(b, method, 4, dcut, 0, k)
    blob = b.export_state()
    b.close()
    c = trg_import_state(blob)
    assert c.dims()[1] == k
    _steps(c, method, 4, dcut, k, nsteps)
    resumed = _observables(c)
    c.close()
    assert resumed == straight


def test_export_size_query_and_short_buffer():
    need_gpu()
    import ctypes as C
    from paper_1911_12954_amd import _lib as L
    from paper_1911_12954_amd import trg_init_ising
    announce("checkpoint buffer")
    a = trg_init_ising(0.15, 0.0, 4, dcut=4)
    a.hotrg_step(0, 4)
    n = C.c_size_t()
    lib = L.load()
    assert lib.trg_export_state(a.handle, None, 0, C.byref(n)) == L.TRG_OK
    buf = C.create_string_buffer(n.value)
    assert lib.trg_export_state(a.handle, buf, n.value - 1, C.byref(n)) == L.TRG_EINVAL
    assert len(a.export_state()) == n.value
    a.close()


def test_run_continues_an_imported_checkpoint():
    """trg_run on an imported context takes the remaining steps of the
    lattice and ends on the bits of the uninterrupted run."""
    need_gpu()
    from paper_1911_12954_amd import trg_import_state, trg_init_ising
    announce("checkpoint run")
    a = trg_init_ising(0.1497, 1e-4, 4, dcut=4, impure=("E", "M"))
    a.run(8)
    straight = _observables(a)
    a.close()
    b = trg_init_ising(0.1497, 1e-4, 4, dcut=4, impure=("E", "M"))
    _steps(b, "hotrg", 4, 4, 0, 7)
    c = trg_import_state(b.export_state())
    b.close()
    c.run(8)
    assert _observables(c) == straight
    c.close()
