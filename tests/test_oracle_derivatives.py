"""The impure-tensor observables against central differences of the free
energy of the same method (E = -d(ln Z/V)/d beta, M = d(ln Z/V)/d(beta h)):
equal up to the difference step when nothing is truncated, and at the
truncation level otherwise (the isometries and SVDs move with beta and h,
the impurities do not see that; reported, with loose bounds)."""
import pytest

from oracle import atrg, hotrg


def _diffs(run, beta, h, step=1e-5):
    base = run(beta, h)
    fb = (run(beta + step, h).ln_z_per_site - run(beta - step, h).ln_z_per_site) / (2 * step)
    fh = (run(beta, h + step).ln_z_per_site - run(beta, h - step).ln_z_per_site) / (2 * step)
    return base, -fb, fh / beta


def test_untruncated_impurities_are_derivatives():
    """2D 4x4, nothing truncated: HOTRG and ATRG (dense SVDs) impurities equal
    the central differences to the O(step^2) error."""
    for run in (lambda b, h: hotrg.run(b, h, 2, 64, 4),
                lambda b, h: atrg.run(b, h, 2, 4096, 4, dense_swap=True, impure=True)):
        r, E_fd, M_fd = _diffs(run, 0.35, 0.05)
        assert abs(r.energy - E_fd) < 1e-8 * abs(E_fd)
        assert abs(r.magnetization - M_fd) < 1e-8 * abs(M_fd)


@pytest.mark.parametrize("method", ["hotrg", "atrg"])
def test_truncated_impurities_against_derivatives(method):
    """2D, K = 0.4, h = 0.01, Dcut 8: the impurity E and M agree with the
    derivatives of the truncated free energy to the truncation level."""
    if method == "hotrg":
        run = lambda b, h: hotrg.run(b, h, 2, 8, 2 ** 8)
    else:
        run = lambda b, h: atrg.run(b, h, 2, 8, 2 ** 6, p=16, q=4, impure=True)
    r, E_fd, M_fd = _diffs(run, 0.4, 0.01)
    dE = abs(r.energy - E_fd) / abs(E_fd)
    dM = abs(r.magnetization - M_fd) / abs(M_fd)
    print(f"[{method} Dcut 8] E {r.energy:.10f} vs {E_fd:.10f} ({dE:.2e}); M {r.magnetization:.10f} vs "
          f"{M_fd:.10f} ({dM:.2e})")
    assert dE < 3e-2 and dM < 3e-2
