"""Write oracle_values.json: HOTRG and ATRG results of the FP64 oracle for
small, fully specified runs, used as stored expected values by the GPU tests.

Run from the repository root:  python tests/golden/make_golden.py [case ...]
(no case: all of them).  Calls nothing but `oracle/`."""
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
    ("4d_dcut6_L16_h1e-5", 0.1497, 1e-5, 4, 6, 16),
]


ATRG_CASES = [
    # (name, beta, h, d, dcut, L, seed, z2); p = 4 dcut, q = 2 dcut
    ("atrg_4d_dcut4_L4_h1e-3", 0.1497, 1e-3, 4, 4, 4, 5, False),
    ("atrg_2d_dcut8_L64_h1e-2", 0.4000, 1e-2, 2, 8, 64, 1, False),
    ("atrg_z2_4d_dcut6_L1024_b0.2", 0.2000, 0.0, 4, 6, 1024, 0, True),
    ("atrg_4d_dcut10_L16_h1e-3", 0.1497, 1e-3, 4, 10, 16, 3, False),
]


def main(names):
    """Recompute the named cases (all when none is named) and merge them
    into the stored file."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
    out = {"cases": {}}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    out["source"] = ("oracle/hotrg.py run(beta, h, d, dcut, L, impure=True) and oracle/atrg.py "
                     "run(beta, h, d, dcut, L, seed=seed, impure=True, z2=z2), FP64")
    for name, beta, h, d, dcut, L in CASES:
        if names and name not in names:
            continue
        r = hotrg.run(beta, h, d, dcut, L, impure=True)
        out["cases"][name] = {"beta": beta, "h": h, "d": d, "dcut": dcut, "L": L,
                              "ln_z_per_site": repr(r.ln_z_per_site), "energy": repr(r.energy),
                              "magnetization": repr(r.magnetization)}
        print(name, out["cases"][name], flush=True)
    for name, beta, h, d, dcut, L, seed, z2 in ATRG_CASES:
        if names and name not in names:
            continue
        r = atrg.run(beta, h, d, dcut, L, seed=seed, impure=True, z2=z2)
        case = {"method": "atrg", "beta": beta, "h": h, "d": d, "dcut": dcut, "L": L, "seed": seed,
                "ln_z_per_site": repr(r.ln_z_per_site), "energy": repr(r.energy),
                "magnetization": repr(r.magnetization)}
        if z2:
            case["z2"] = True
            case["x"] = repr(atrg.indicator_x(r.G, r.H, 0))
        out["cases"][name] = case
        print(name, out["cases"][name], flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
