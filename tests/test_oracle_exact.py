"""Pins of the exact references themselves (closed forms they must reduce to)."""
import math
import warnings

import pytest

warnings.filterwarnings("ignore", message=".*roundoff error.*")

from oracle import exact

CATALAN = 0.915965594177219015054603514932  # Catalan's constant G


def test_onsager_at_critical_coupling():
    """At K_c = ln(1 + sqrt 2)/2: ln Z/N = ln(2)/2 + 2G/pi."""
    Kc = 0.5 * math.log(1 + math.sqrt(2))
    assert abs(exact.onsager_lnz(Kc) - (0.5 * math.log(2) + 2 * CATALAN / math.pi)) < 1e-12


def test_onsager_energy_is_beta_derivative():
    for K in (0.2, 0.35, 0.55):
        eps = 1e-5
        fd = -(exact.onsager_lnz(K + eps) - exact.onsager_lnz(K - eps)) / (2 * eps)
        assert abs(fd - exact.onsager_energy(K)) < 1e-8


@pytest.mark.parametrize("K", [0.02, 0.1])
def test_onsager_small_coupling_series(K):
    """Square-lattice high-temperature series: polygons of perimeter 4..10
    give ln Z/N = ln 2 + 2 ln cosh K + t^4 + 2t^6 + (9/2)t^8 + 12t^10 + O(t^12)."""
    t = math.tanh(K)
    series = math.log(2) + 2 * math.log(math.cosh(K)) + t ** 4 + 2 * t ** 6 + 4.5 * t ** 8 + 12 * t ** 10
    assert abs(exact.onsager_lnz(K) - series) < 50 * t ** 12 + 1e-15


@pytest.mark.parametrize("L,beta,h", [(8, 0.3, 0.0), (12, 0.7, 0.0)])
def test_brute_force_one_dimensional_chain(L, beta, h):
    """Periodic chain at h = 0: Z = (2 cosh b)^L + (2 sinh b)^L."""
    lnz, E, M = exact.brute_force(beta, h, 1, L)
    z = (2 * math.cosh(beta)) ** L + (2 * math.sinh(beta)) ** L
    assert abs(lnz - math.log(z) / L) < 1e-14
    dz = L * (2 * math.cosh(beta)) ** (L - 1) * 2 * math.sinh(beta) + L * (2 * math.sinh(beta)) ** (L - 1) * 2 * math.cosh(beta)
    assert abs(E - (-dz / z / L)) < 1e-13
    assert abs(M) < 1e-15


def test_yang_limits():
    assert exact.yang_magnetization(0.3) == 0.0
    assert abs(exact.yang_magnetization(5.0) - 1.0) < 1e-12
