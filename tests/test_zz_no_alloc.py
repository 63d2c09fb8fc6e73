"""trg_indicator_x_noalloc (static device scratch, no allocation) against
trg_indicator_x (workspace from the context's allocator) through the C-ABI:
two calls in a row on the same GPU, the second on a smaller tensor, the
same bits as the allocating entry point, no allocation request, and the
size limit."""
import pytest

from tests.gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


def _allocs(torch):
    return torch.cuda.memory_stats().get("allocation.all.allocated", 0)


def test_noalloc_indicator_equals_allocating_entry_point():
    torch = need_gpu()
    from oracle import hotrg
    from paper_1911_12954_amd import trg_init_ising
    announce("noalloc indicator: 4D Dcut 8 then 3D Dcut 3")
    big = trg_init_ising(0.16, 1e-5, 4, dcut=8)
    for n in range(1, 9):
        big.hotrg_step((n - 1) % 4, 8)
    big.sync()
    assert big.dims()[0] == (8, 8, 8, 8)
    small = trg_init_ising(0.25, 0.0, 3, dcut=3)
    for n in range(1, 4):
        small.hotrg_step((n - 1) % 3, 3)
    small.sync()
    # the allocation-free calls come first, on contexts that have never
    # asked for the indicator workspace: no allocation request may appear
    before = _allocs(torch)
    x_big = [big.indicator_x_noalloc(ax) for ax in range(4)]
    x_small = [small.indicator_x_noalloc(ax) for ax in range(3)]
    assert _allocs(torch) == before
    # the allocating entry point gives the same bits (same kernels, same order)
    assert [big.indicator_x(ax) for ax in range(4)] == x_big
    assert [small.indicator_x(ax) for ax in range(3)] == x_small
    assert _allocs(torch) > before      # it did allocate its workspace
    # and the small case against the oracle's X of the same run
    T, imps = None, []
    from oracle import ising
    import numpy as np
    T0 = ising.site_tensors(0.25, 0.0, 3)[0]
    T = T0 / np.sqrt(np.sum(T0 * T0))
    for n in range(1, 4):
        T, _, _, _ = hotrg.hotrg_step(T, (n - 1) % 3, 3)
    for ax in range(3):
        ref = hotrg.indicator_x(T, ax)
        assert abs(x_small[ax] - ref) <= 1e-10 * abs(ref)
    # a third call on the larger context after the smaller one
    assert big.indicator_x_noalloc(2) == x_big[2]
    big.close()
    small.close()


def test_noalloc_indicator_limits():
    need_gpu()
    import numpy as np
    from paper_1911_12954_amd import TrgError, trg_init_ising, trg_init_tensor
    announce("noalloc indicator: limits")
    wide = trg_init_tensor(np.random.default_rng(0).standard_normal((300, 300, 2, 2)))
    with pytest.raises(TrgError) as e:
        wide.indicator_x_noalloc(0)
    assert e.value.code == -1
    assert wide.indicator_x_noalloc(1) == wide.indicator_x(1)
    wide.close()
    at = trg_init_ising(0.2, 0.0, 2, dcut=4, method="atrg")
    with pytest.raises(TrgError) as e:
        at.indicator_x_noalloc(0)
    assert e.value.code == -1
    at.close()
