"""Stored expected values: the oracle's own results for small runs (written
by tests/golden/make_golden.py, which calls only the oracle) must still be
reproduced by the oracle, and the paper's printed numbers are kept as
context."""
import json
import os

import pytest

from oracle import atrg, hotrg

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _oracle_values():
    with open(os.path.join(HERE, "oracle_values.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("name", ["4d_dcut4_L16_h0", "4d_dcut4_L16_h1e-5", "3d_dcut6_L16_h1e-4"])
def test_stored_oracle_values_are_reproduced(name):
    c = _oracle_values()[name]
    r = hotrg.run(c["beta"], c["h"], c["d"], c["dcut"], c["L"], impure=True)
    assert r.ln_z_per_site == pytest.approx(float(c["ln_z_per_site"]), rel=1e-13, abs=0)
    assert r.energy == pytest.approx(float(c["energy"]), rel=1e-12, abs=0)
    assert r.magnetization == pytest.approx(float(c["magnetization"]), rel=1e-10, abs=1e-13)


@pytest.mark.parametrize("name", ["atrg_4d_dcut4_L4_h1e-3", "atrg_2d_dcut8_L64_h1e-2"])
def test_stored_atrg_oracle_values_are_reproduced(name):
    c = _oracle_values()[name]
    r = atrg.run(c["beta"], c["h"], c["d"], c["dcut"], c["L"], seed=c["seed"], impure=True)
    assert r.ln_z_per_site == pytest.approx(float(c["ln_z_per_site"]), rel=1e-12, abs=0)
    assert r.energy == pytest.approx(float(c["energy"]), rel=1e-10, abs=0)
    assert r.magnetization == pytest.approx(float(c["magnetization"]), rel=1e-10, abs=1e-13)


def test_paper_transition_lies_in_the_scanned_window():
    """The beta window of the synthetic scans (0.1490 - 0.1505) brackets the
    paper's transition 1/T_c; the paper's ATRG/HOTRG gap is 0.12 %."""
    with open(os.path.join(HERE, "paper_values.json")) as f:
        v = json.load(f)["values"]
    beta_c = 1.0 / v["Tc_hotrg_dcut13_Linf"]["value"]
    assert 0.1490 < beta_c < 0.1505
    assert v["Tc_atrg39_vs_hotrg13_relative_difference"]["value"] == pytest.approx(0.0012)
    assert 1.0 / v["free_energy_comparison_temperature"]["value"] == pytest.approx(beta_c, rel=1e-5)
