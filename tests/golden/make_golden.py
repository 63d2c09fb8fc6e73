"""Write oracle_values.json: HOTRG and ATRG results of the FP64 oracle for
small, fully specified runs, used as stored expected values by the GPU tests.

Run from the repository root:  python tests/golden/make_golden.py
Calls nothing but `oracle/`."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import atrg, hotrg  # noqa: E402

CASES = [
    # (name, beta, h, d, dcut, L)
    ("4d_dcut4_L16_h0", 0.1497, 0.0, 4, 4, 16),
    ("4d_dcut4_L16_h1e-5", 0.1497, 1e-5, 4, 4, 16),
    ("3d_dcut6_L16_h1e-4", 0.2200, 1e-4, 3, 6, 16),
    ("2d_dcut8_L1024_h0", 0.4000, 0.0, 2, 8, 1024),
]


ATRG_CASES = [
    # (name, beta, h, d, dcut, L, seed); p = 4 dcut, q = 2 dcut
    ("atrg_4d_dcut4_L4_h1e-3", 0.1497, 1e-3, 4, 4, 4, 5),
    ("atrg_2d_dcut8_L64_h1e-2", 0.4000, 1e-2, 2, 8, 64, 1),
]


def main():
    out = {"source": "oracle/hotrg.py run(beta, h, d, dcut, L, impure=True) and oracle/atrg.py "
                     "run(beta, h, d, dcut, L, seed=seed, impure=True), FP64", "cases": {}}
    for name, beta, h, d, dcut, L in CASES:
        r = hotrg.run(beta, h, d, dcut, L, impure=True)
        out["cases"][name] = {"beta": beta, "h": h, "d": d, "dcut": dcut, "L": L,
                              "ln_z_per_site": repr(r.ln_z_per_site), "energy": repr(r.energy),
                              "magnetization": repr(r.magnetization)}
        print(name, out["cases"][name], flush=True)
    for name, beta, h, d, dcut, L, seed in ATRG_CASES:
        r = atrg.run(beta, h, d, dcut, L, seed=seed, impure=True)
        out["cases"][name] = {"method": "atrg", "beta": beta, "h": h, "d": d, "dcut": dcut, "L": L, "seed": seed,
                              "ln_z_per_site": repr(r.ln_z_per_site), "energy": repr(r.energy),
                              "magnetization": repr(r.magnetization)}
        print(name, out["cases"][name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
