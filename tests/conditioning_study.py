"""CPU study (not collected by pytest): how far FP32-level rounding of the
contractions alone moves f, E and M of a HOTRG run, using only the FP64
oracle.  Every tensor that the block-spin contraction produces (pure and
impure, before normalisation) is multiplied elementwise by (1 + 2^-24 g),
g ~ N(0, 1) from a seeded generator, at every step; the spread of f, E, M
over seeds against the unperturbed run is the conditioning of the result
under rounding at FP32 precision, the floor that any FP32-accurate join can
reach.  The degeneracy window is the one the library uses after FP32 or
split-BF16 joins (1e-6 lambda_max) in both the perturbed and the reference
runs.

    python tests/conditioning_study.py 5 1024 0.1497 1e-5 8   # Dcut, L, beta, h, seeds

prints one JSON line per run and the spread (rms and max, relative and
absolute) of f, E and M.
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def one_run(args):
    dcut, L, beta, h, seed = args
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)    # one BLAS thread per run; the runs go in parallel
    from oracle import hotrg
    hotrg.CLUSTER_REL = 1e-6
    exact = hotrg.coarse_grain
    if seed >= 0:
        rng = np.random.default_rng(seed)

        def rounded(*a, **k):
            out = exact(*a, **k)
            return out * (1.0 + 2.0 ** -24 * rng.standard_normal(out.shape))

        hotrg.coarse_grain = rounded
    r = hotrg.run(beta, h, 4, dcut, L)
    return {"seed": seed, "f": r.ln_z_per_site, "E": r.energy, "M": r.magnetization}


def main():
    dcut, L, beta, h, nseed = int(sys.argv[1]), int(sys.argv[2]), float(sys.argv[3]), float(sys.argv[4]), \
        int(sys.argv[5])
    jobs = [(dcut, L, beta, h, s) for s in range(-1, nseed)]
    with ProcessPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        rows = list(ex.map(one_run, jobs))
    for r in rows:
        print(json.dumps(r))
    ref = rows[0]
    out = {"dcut": dcut, "L": L, "beta": beta, "h": h, "seeds": nseed}
    for k in ("f", "E", "M"):
        d = np.array([r[k] - ref[k] for r in rows[1:]])
        out[k] = {"rms_rel": float(np.sqrt(np.mean(d ** 2)) / abs(ref[k])) if ref[k] else None,
                  "max_rel": float(np.max(np.abs(d)) / abs(ref[k])) if ref[k] else None,
                  "rms_abs": float(np.sqrt(np.mean(d ** 2)))}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
