"""Benchmark: 4D Ising HOTRG RG-steps/s at Dcut = 10 on one MI355X.

A step is one steady-state HOTRG coarse-graining step (Gram matrices, FP64
eigendecomposition and isometries, block-spin contraction, post-join
compression, FP64 normalisation) of the 4D Ising tensor at beta = 0.1497,
h = 0, with every leg at Dcut = 10; inputs are resident in HBM.  The first
four steps (leg dims 2 -> 4 -> 10) and `--warmup` steady steps are untimed;
then `--steps` steps are timed between two stream synchronisations.  The
headline join precision is BF16x6 (FP32-accurate operands, FP64 sums of
128-element groups), the mixed path that meets 1e-6 on f and E against the
FP64 path; FP64 and BF16x3 are timed beside it (warm, several steps) and
every precision's ln Z/V after the same step is compared with the FP64 one.

The join GEMM (the D^15 contraction) is timed with HIP events on the
library's stream; its algorithmic flops per step are 2 D^15 (6 x or 3 x
2 D^15 BF16 MFMA flops for the BF16x6 / BF16x3 splits).  The oracle (FP64
NumPy) is timed on a bounded sample of the same step on the host cores, in a
child process while the GPU runs the FP64 comparison.  A time-boxed window
of the serving stream (Poisson arrivals of HOTRG solves, Dcut 6/8/10,
L = 2^4 .. 2^10) reports served solves/s and latency.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}
# BF16 MFMA products per multiply-add of the split joins
SPLIT_PRODUCTS = {"bf16x3": 3.0, "bf16x6": 6.0}
HBM_PEAK_GBS = 8000.0
# HBM bytes per join launch of the steady Dcut 10 step (three full x0
# slices and one of a single x0 value per step, averaged), from rocprofv3
# FETCH_SIZE and WRITE_SIZE of the join kernel, each scaled by what the
# counter reads for a device-to-device copy of 4 GiB (FETCH x 2.0, WRITE x
# 1.0).  Each entry names the SHA-256 of the kernel source it was taken on;
# the figure is reported only while csrc/gemm.hip still has that hash.
JOIN_TRAFFIC = {
    ("bf16x6", 10): {"bytes_per_launch": 4.912e12, "algorithmic_bytes_per_launch": 8.51e10,
                     "gemm_sha16": "372fd768a9adad15",
                     "source": "profiles/join_gemm_hotrg_dcut10_bf16x6.md (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)"},
    ("fp64", 10): {"bytes_per_launch": 1.510e13, "algorithmic_bytes_per_launch": 1.202e11,
                   "gemm_sha16": "372fd768a9adad15",
                   "source": "profiles/join_gemm_hotrg_dcut10_fp64.md (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)"},
    ("fp32", 10): {"bytes_per_launch": 3.121e12, "algorithmic_bytes_per_launch": 6.01e10,
                   "gemm_sha16": "372fd768a9adad15",
                   "source": "profiles/join_gemm_hotrg_dcut10_fp32.md (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)"},
}
GEMM_SRC = os.path.join(ROOT, "paper_1911_12954_amd", "csrc", "gemm.hip")


def gemm_source_hash():
    import hashlib
    with open(GEMM_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def join_traffic(precision, dcut):
    t = JOIN_TRAFFIC.get((precision, dcut))
    if not t or t.get("gemm_sha16") != gemm_source_hash():
        return None
    return t


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--dcut", type=int, default=10)
    p.add_argument("--precision", default="bf16x6", choices=["fp64", "fp32", "bf16x3", "bf16x6"])
    p.add_argument("--beta", type=float, default=0.1497)
    p.add_argument("--compare", default="fp64,bf16x3",
                   help="other join precisions timed beside the headline (comma list, '' = none)")
    p.add_argument("--compare-warmup", type=int, default=1)
    p.add_argument("--compare-steps", type=int, default=2)
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    p.add_argument("--cpu-only", action="store_true",
                   help="only the oracle baseline (run as a child process by the benchmark)")
    p.add_argument("--no-serve", action="store_true", help="skip the serving window")
    p.add_argument("--impure", action="store_true",
                   help="time the step with the impure E and M tensors (five joins per step)")
    p.add_argument("--cpu-sample-blocks", type=int, default=1)
    p.add_argument("--method", default="hotrg", choices=["hotrg", "atrg"],
                   help="atrg: time steady-state ATRG steps (default Dcut 24 there) instead of HOTRG")
    p.add_argument("--serve", action="store_true",
                   help="serving benchmark: Poisson stream of HOTRG solves, time-boxed window")
    p.add_argument("--serve-n", type=int, default=200)
    p.add_argument("--serve-rate", type=float, default=0.0,
                   help="arrivals per second; 0 = 0.8 of the capacity measured by a calibration pass; "
                        "<0 = every request arrives at the start (saturation)")
    p.add_argument("--serve-window", type=float, default=60.0)
    p.add_argument("--window-rate", type=float, default=0.5,
                   help="arrival rate of the serving window of the default run (requests/s)")
    p.add_argument("--window-seconds", type=float, default=35.0,
                   help="length of the serving window of the default run")
    p.add_argument("--serve-dcuts", default="6,8,10")
    p.add_argument("--serve-k", default="4,10", help="L = 2^k, k uniform in [kmin, kmax]")
    p.add_argument("--serve-precision", default="bf16x6", choices=["fp64", "fp32", "bf16x3", "bf16x6"])
    p.add_argument("--serve-methods", default="hotrg", help="methods of the request stream, e.g. hotrg,atrg")
    p.add_argument("--serve-budget-gb", type=float, default=200.0)
    p.add_argument("--tc-bisect", default=None,
                   help="instead of timing: 'd,dcut,steps,beta_lo,beta_hi,tol[,method]' bisection of the "
                        "transition on the degeneracy indicator X (FP64; method hotrg, atrg or atrg-z2)")
    p.add_argument("--atrg-study", default=None,
                   help="instead of timing: 'dcuts;pq_dcut;hotrg_dcut' (e.g. '8,12,16,20,24;16;8'): ATRG f at "
                        "T = 6.65035, L = 1024 for each Dcut, the RSVD (p, q) study at pq_dcut and the ratio to "
                        "HOTRG at hotrg_dcut (FP64)")
    p.add_argument("--copy-cal", type=float, default=0.0,
                   help="only copy this many GiB device to device three times (calibration of the "
                        "FETCH_SIZE / WRITE_SIZE counters)")
    p.add_argument("--step-error", default=None,
                   help="instead of timing: 'D,prec[,prec...]' one HOTRG step of a seeded 4D tensor with every leg "
                        "D (decaying HOSVD spectra) in FP64 and in each precision; errors of ln c and of the "
                        "new tensor against FP64")
    p.add_argument("--atrg-scan", default=None,
                   help="instead of timing: 'dcut;L;beta0,dbeta,n;precisions' (e.g. '24;1024;0.1490,0.0001,4;"
                        "fp64,fp32'): ATRG ln Z/V over a beta scan in each contraction precision, with the "
                        "FP32 - FP64 differences")
    p.add_argument("--atrg-impure", default=None,
                   help="instead of timing: 'd;T;h;L;dcuts;hotrg_dcut' (e.g. '4;6.64;0;1024;8,12,16;8'): E and M "
                        "by ATRG impure tensors for each Dcut next to HOTRG's at hotrg_dcut (0: none) (FP64)")
    p.add_argument("--vendor-gemm", default=None,
                   help="instead of timing the step: 'M,N,K[,precision]' (e.g. '30208,100096,100000', the "
                        "full-slice join of the Dcut = 10 step): the BF16x3 (or bf16x6) join kernel against one "
                        "plain BF16 torch.matmul (hipBLASLt) of the same shape, in MFMA TFLOP/s issued")
    p.add_argument("--accuracy", default=None,
                   help="instead of timing: run 'dcut,L,beta,h[,pure|E|M]' in FP64 and the variants with impure E "
                        "and M (neither with 'pure', one with 'E' or 'M') and print the relative errors of f, "
                        "E, M against the FP64 path")
    p.add_argument("--accuracy-variants", default="fp32:0,bf16x3:0",
                   help="precision:fp64_steps pairs compared with the FP64 path")
    return p.parse_args()


def vendor_gemm(spec):
    """Issue rate of a split-BF16 join kernel (three or six BF16 products per
    multiply-add) next to a plain BF16 GEMM of the vendor library at one
    shape: both run the same MFMA instruction class, so the two TFLOP/s
    figures say how close the hand-written kernel comes to the library.
    spec: 'M,N,K[,precision]' (precision bf16x3, the default, or bf16x6)."""
    import torch
    from paper_1911_12954_amd import trg_gemm, trg_gemm_tile
    fields = spec.split(",")
    M, N, K = (int(x) for x in fields[:3])
    prec = fields[3] if len(fields) > 3 else "bf16x3"
    planes, mult = {"bf16x3": (2, 3.0), "bf16x6": (3, 6.0)}[prec]
    tm, tn, tk = trg_gemm_tile(prec)
    assert M % tm == 0 and N % tn == 0 and K % tk == 0, "M, N, K must be multiples of the join tile"
    out = {"metric": "BF16 MFMA issue rate at the join shape", "M": M, "N": N, "K": K, "unit": "TFLOP/s",
           "join_precision": prec}
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    # bf16 planes per operand, values in [1, 2)
    A = torch.randint(0x3F80, 0x4000, (planes, M, K), dtype=torch.int16, device="cuda", generator=g)
    Bt = torch.randint(0x3F80, 0x4000, (planes, N, K), dtype=torch.int16, device="cuda", generator=g)
    Cm = torch.empty(M, N, dtype=torch.float32, device="cuda")
    ms = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        trg_gemm(prec, A.data_ptr(), Bt.data_ptr(), Cm.data_ptr(), M, N, K, K, K, N)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = min(ms)
    out["join_ms"] = t
    out["join_issued_tflops"] = mult * 2.0 * M * N * K / (t * 1e-3) / 1e12
    out["join_algorithmic_tflops"] = 2.0 * M * N * K / (t * 1e-3) / 1e12
    progress(f"vendor-gemm: {prec} join kernel {t:.1f} ms")
    del A, Bt, Cm
    torch.cuda.empty_cache()
    x = torch.randn(M, K, dtype=torch.bfloat16, device="cuda", generator=g)
    y = torch.randn(K, N, dtype=torch.bfloat16, device="cuda", generator=g)
    ms = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        z = torch.matmul(x, y)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
        del z
    t = min(ms)
    out["torch_matmul_bf16_ms"] = t
    out["torch_matmul_bf16_tflops"] = 2.0 * M * N * K / (t * 1e-3) / 1e12
    out["join_vs_library"] = out["join_issued_tflops"] / out["torch_matmul_bf16_tflops"]
    out["peak"] = 2500.0
    return out


def accuracy(spec, variants):
    """Errors of mixed-precision joins against the FP64 path on one whole
    run (4D, impure-tensor E and M).  `variants`: "prec:n,..." with n the
    number of leading steps joined in FP64 (fp64_steps)."""
    import torch
    from paper_1911_12954_amd import trg_init_ising
    fields = spec.split(",")
    # fifth field: "pure" (ln Z/V only), "E" or "M" (that impurity alone, a
    # third of the joins of both), absent: both
    which = fields[4] if len(fields) > 4 else "EM"
    if which not in ("pure", "E", "M", "EM"):
        raise SystemExit(f"--accuracy: unknown fifth field {which!r}")
    pure = which == "pure"
    impure = () if pure else tuple(which)
    dcut, L, beta, h = int(fields[0]), int(fields[1]), float(fields[2]), float(fields[3])
    runs = [("fp64", 0)] + [(v.split(":")[0], int(v.split(":")[1])) for v in variants.split(",") if v]
    res = {}
    for prec, n64 in runs:
        key = prec if n64 == 0 else f"{prec}+fp64x{n64}"
        t0 = time.perf_counter()
        ctx = trg_init_ising(beta, h, 4, dcut=dcut, precision=prec, impure=impure, fp64_steps=n64)
        m = L.bit_length() - 1
        for n in range(1, 4 * m + 1):
            ctx.hotrg_step((n - 1) % 4, dcut)
            if n % 2 == 0 or impure:
                ctx.sync()
                progress(f"accuracy {key}: step {n}/{4 * m} at {time.perf_counter() - t0:.1f} s")
        log = ctx.step_log()
        res[key] = {"f": ctx.free_energy(), "E": ctx.impure_energy() if "E" in impure else float("nan"),
                    "M": ctx.impure_magnetization() if "M" in impure else float("nan"),
                    "seconds": time.perf_counter() - t0,
                    "fp64_join_steps": sum(r.join_precision == "fp64" for r in log),
                    "degenerate_cuts": sum(sum(r.degenerate_cut) for r in log)}
        ctx.close()
        torch.cuda.empty_cache()
        progress(f"accuracy {key}: {res[key]}")
    ref = res["fp64"]
    out = {"workload": f"4D Ising HOTRG Dcut={dcut} L={L} beta={beta} h={h}, "
                       + ("ln Z/V only" if pure else "impure " + " and ".join(impure)), "runs": res}
    for key in res:
        if key == "fp64":
            continue
        out[f"rel_err_{key}"] = {k: abs(res[key][k] - ref[k]) / max(abs(ref[k]), 1e-300) for k in ("f", "E", "M")}
        out[f"abs_err_{key}"] = {k: abs(res[key][k] - ref[k]) for k in ("f", "E", "M")}
    return out


def step_error(spec):
    """One steady-state HOTRG step (all legs D, axis 0) from the same seeded
    tensor with decaying HOSVD spectra, in FP64 and in each listed join
    precision: |ln c - ln c_64| and |T' - T'_64| / |T'_64| (Frobenius and
    max-abs), T' the normalised new tensor."""
    import numpy as np
    import torch
    from paper_1911_12954_amd import trg_init_tensor
    from trg_inputs import decaying_site_tensor
    fields = spec.split(",")
    D, precs = int(fields[0]), [p for p in fields[1:] if p != "fp64"]
    if "TRG_PROGRESS" not in os.environ:
        progress("step-error: set TRG_PROGRESS=1 to see each join of the step finish")
    t0 = time.perf_counter()
    T = decaying_site_tensor((D,) * 4, seed=1201)
    progress(f"step-error: D = {D} input built in {time.perf_counter() - t0:.1f} s")
    out = {"workload": f"one HOTRG step, 4D, every leg D = {D}, seeded tensor with decaying HOSVD spectra", "runs": {}}
    ref = None
    for prec in ["fp64"] + precs:
        t1 = time.perf_counter()
        ctx = trg_init_tensor(T, precision=prec)
        ctx.hotrg_step(0, D)
        ln_c = ctx.step_log()[-1].ln_c
        Tn = ctx.tensor()
        ctx.close()
        torch.cuda.empty_cache()
        row = {"ln_c": ln_c, "seconds": time.perf_counter() - t1}
        if ref is None:
            ref = (ln_c, Tn)
        else:
            d = Tn - ref[1]
            row["abs_err_ln_c"] = abs(ln_c - ref[0])
            row["rel_err_tensor_fro"] = float(np.linalg.norm(d.ravel()) / np.linalg.norm(ref[1].ravel()))
            row["rel_err_tensor_max"] = float(np.max(np.abs(d)) / np.max(np.abs(ref[1])))
            del d
        out["runs"][prec] = row
        progress(f"step-error: {prec} {row}")
        del Tn
    return out


def atrg_scan(spec):
    """ATRG free energy over a beta scan (h = 0, p = 4 Dcut, q = 2 Dcut) for
    each contraction precision, run after run on one GPU."""
    import torch
    from paper_1911_12954_amd import trg_init_ising
    dcut, L, betas, precs = spec.split(";")
    dcut, L = int(dcut), int(L)
    b0, db, nb = betas.split(",")
    betas = [float(b0) + i * float(db) for i in range(int(nb))]
    precs = precs.split(",")
    out = {"workload": f"4D Ising ATRG Dcut={dcut} L={L} h=0, beta scan", "runs": []}
    for beta in betas:
        row = {"beta": beta}
        for prec in precs:
            t0 = time.perf_counter()
            ctx = trg_init_ising(beta, 0.0, 4, dcut=dcut, precision=prec, method="atrg")
            m = L.bit_length() - 1
            for n in range(1, 4 * m + 1):
                ctx.atrg_step((n - 1) % 4, dcut)
                if n % 8 == 0:
                    progress(f"atrg-scan: beta {beta:.5f} {prec} step {n}/{4 * m} lnZ/V {ctx.free_energy():.12f} "
                             f"at {time.perf_counter() - t0:.1f} s")
            row[prec] = ctx.free_energy()
            row[prec + "_seconds"] = time.perf_counter() - t0
            ctx.close()
            torch.cuda.empty_cache()
        if "fp64" in row and "fp32" in row:
            row["rel_diff_fp32"] = abs(row["fp32"] - row["fp64"]) / abs(row["fp64"])
        out["runs"].append(row)
        # each finished point in full precision, so that a scan cut short
        # still leaves its completed rows
        progress("atrg-scan row " + json.dumps(row))
    return out


def atrg_impure(spec):
    """E = <H>/V and M = <s> from the ATRG impure tensors at several Dcut,
    with HOTRG's impure-tensor values beside them."""
    import torch
    from paper_1911_12954_amd import trg_init_ising
    d, T, h, L, dcuts, hdcut = spec.split(";")
    d, T, h, L, hdcut = int(d), float(T), float(h), int(L), int(hdcut)
    beta = 1.0 / T
    out = {"workload": f"{d}D Ising, T = {T} (beta = {beta:.8f}), h = {h}, L = {L}, FP64", "atrg": []}

    def run(method, D):
        t0 = time.perf_counter()
        ctx = trg_init_ising(beta, h, d, dcut=D, precision="fp64", method=method, impure=("E", "M"))
        nsteps = d * (L.bit_length() - 1)
        for n in range(1, nsteps + 1):
            if method == "atrg":
                ctx.atrg_step((n - 1) % d, D)
            else:
                ctx.hotrg_step((n - 1) % d, D)
            if n % 8 == 0:
                progress(f"atrg-impure: {method} Dcut {D}: step {n}/{nsteps} lnZ/V {ctx.free_energy():.12f} "
                         f"at {time.perf_counter() - t0:.1f} s")
        r = {"dcut": D, "lnZ_per_site": ctx.free_energy(), "E": ctx.impure_energy(),
             "M": ctx.impure_magnetization()}
        ctx.close()
        torch.cuda.empty_cache()
        r["seconds"] = time.perf_counter() - t0
        progress(f"atrg-impure: {method} Dcut {D}: lnZ/V {r['lnZ_per_site']:.12f} E {r['E']:.10f} "
                 f"M {r['M']:.10f} in {r['seconds']:.1f} s")
        return r

    if hdcut > 0:
        out["hotrg"] = run("hotrg", hdcut)
    for D in (int(x) for x in dcuts.split(",")):
        out["atrg"].append(run("atrg", D))
    return out


def atrg_study(spec):
    """ATRG free energy at the paper's comparison temperature T = 6.65035 on
    the 1024^4 lattice for several Dcut (p = 4 Dcut, q = 2 Dcut), the RSVD
    (p, q) dependence at one Dcut, and the ratio to HOTRG at another."""
    import torch
    from paper_1911_12954_amd import trg_init_ising
    dcuts, pq_dcut, hdcut = spec.split(";")
    dcuts = [int(x) for x in dcuts.split(",")]
    pq_dcut, hdcut = int(pq_dcut), int(hdcut)
    beta, L = 1.0 / 6.65035, 1024

    def run(method, D, p=0, q=0):
        t0 = time.perf_counter()
        ctx = trg_init_ising(beta, 0.0, 4, dcut=D, precision="fp64", method=method, rsvd_p=p, rsvd_q=q)
        ctx.run(L)
        f = ctx.free_energy()
        ctx.close()
        torch.cuda.empty_cache()
        dt = time.perf_counter() - t0
        progress(f"atrg-study: {method} Dcut {D} p {p} q {q}: lnZ/V {f:.12f} in {dt:.1f} s")
        return f, dt

    f_h, t_h = run("hotrg", hdcut)
    out = {"workload": "4D Ising, T = 6.65035 (beta = %.8f), h = 0, L = 1024 (40 steps), FP64" % beta,
           "hotrg": {"dcut": hdcut, "lnZ_per_site": f_h, "seconds": t_h}, "atrg": [], "pq": []}
    for D in dcuts:
        f, dt = run("atrg", D)
        out["atrg"].append({"dcut": D, "p": 4 * D, "q": 2 * D, "lnZ_per_site": f, "seconds": dt,
                            "ratio_to_hotrg": f / f_h})
    for p, q in ((2 * pq_dcut, pq_dcut), (4 * pq_dcut, 2 * pq_dcut), (6 * pq_dcut, 3 * pq_dcut)):
        f, dt = run("atrg", pq_dcut, p, q)
        out["pq"].append({"dcut": pq_dcut, "p": p, "q": q, "lnZ_per_site": f, "seconds": dt})
    return out


def progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_steps(precision, dcut, beta, warmup, steps, impure=False, probe_step=0):
    """Ramp to every leg at dcut, `warmup` untimed steps, then `steps` timed
    steps.  ln Z/V of the periodic block after step `probe_step` is read if
    that step is untimed (ramp or warm-up; the read synchronises)."""
    import torch
    from paper_1911_12954_amd import trg_init_ising
    d = 4
    ctx = trg_init_ising(beta, 0.0, d, dcut=dcut, precision=precision, impure=("E", "M") if impure else ())
    n = 0
    probe = None

    def after_step():
        nonlocal probe
        if n == probe_step:
            probe = ctx.free_energy()
    # ramp: legs grow 2 -> 4 -> ... -> dcut
    while min(ctx.dims()[0]) < dcut or n < d:
        ctx.hotrg_step(n % d, dcut)
        n += 1
        after_step()
        if n > 3 * d:
            break
    ctx.sync()
    progress(f"{precision}: ramp done after {n} steps, dims {ctx.dims()[0]}")
    for _ in range(warmup):
        tw = time.perf_counter()
        ctx.hotrg_step(n % d, dcut)
        n += 1
        ctx.sync()
        progress(f"{precision}: warmup step {n} took {time.perf_counter() - tw:.3f} s")
        after_step()
    ctx.sync()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    ctx.join_profile()  # reset counters
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.hotrg_step(n % d, dcut)
        n += 1
        if steps > 1 and dcut >= 10:
            ctx.sync()  # keeps a progress line per step on long runs
            progress(f"{precision}: timed step {n} done at {time.perf_counter() - t0:.3f} s")
    ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, launches, _ = ctx.join_profile()
    lnz = ctx.free_energy()
    ctx.close()
    torch.cuda.empty_cache()
    return {"elapsed": elapsed, "join_ms": ms, "launches": launches, "lnz": lnz, "steps_total": n,
            "probe": probe}


def time_atrg(precision, dcut, beta, warmup, steps):
    """Steady-state ATRG steps of the 4D Ising model (every leg at dcut,
    p = 4 dcut, q = 2 dcut).  Returns elapsed, contraction-GEMM ms, launches,
    algorithmic flops of those GEMMs."""
    import torch
    from paper_1911_12954_amd import trg_init_ising
    d = 4
    ctx = trg_init_ising(beta, 0.0, d, dcut=dcut, precision=precision, method="atrg")
    n = 0
    while min(ctx.dims()[0]) < dcut or n < d:
        t0 = time.perf_counter()
        ctx.atrg_step(n % d, dcut)
        n += 1
        ctx.sync()
        progress(f"atrg {precision}: ramp step {n} dims {ctx.dims()[0]} {time.perf_counter() - t0:.2f} s")
        if n > 4 * d:
            break
    for _ in range(warmup):
        ctx.atrg_step(n % d, dcut)
        n += 1
        ctx.sync()
    ctx.set_profiling(True)
    ctx.join_profile()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.atrg_step(n % d, dcut)
        n += 1
        ctx.sync()
        progress(f"atrg {precision}: timed step {n} at {time.perf_counter() - t0:.2f} s")
    elapsed = time.perf_counter() - t0
    ms, launches, flops = ctx.join_profile()
    lnz = ctx.free_energy()
    ctx.close()
    torch.cuda.empty_cache()
    return elapsed, ms, launches, flops, lnz


def cpu_baseline(dcut, blocks):
    """Time the oracle on a bounded sample of one steady-state step: the six
    isometries (all Gram matrices and eigendecompositions) plus `blocks`
    blocks T'[x0, x2, Y, Y', :, :, :, :] of the block-spin contraction, each
    1/D^4 of the join, then scale the join part to the whole step; once with
    every host thread the BLAS pool has and once with one thread."""
    import numpy as np
    from oracle import hotrg
    from trg_inputs import random_site_tensor
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    D = dcut
    T = random_site_tensor((D,) * 4, seed=0, positive_bias=True)
    T /= np.sqrt(np.sum(T * T))
    mu = 0

    def sample():
        t0 = time.perf_counter()
        choices = [hotrg.isometry(T, mu, nu, D) for nu in (1, 2, 3)]
        t_iso = time.perf_counter() - t0
        U = {ch.nu: ch.U for ch in choices}
        t0 = time.perf_counter()
        for b in range(blocks):
            # one (x0, x2) pair and one kept column Y of the first pre-join axis
            Ub = dict(U)
            Ub[1] = U[1][:, :, b % D: b % D + 1]
            hotrg.coarse_grain(T, T, Ub, mu, x0s=[b % D], x2s=[(b + 1) % D])
        t_blk = (time.perf_counter() - t0) / blocks
        # whole step: D^2 (x0, x2) pairs x D^2 (Y, Y') pairs of such blocks
        return t_iso, t_blk, t_iso + t_blk * D ** 4

    t_iso, t_blk, t_step = sample()
    with threadpool_limits(limits=1):
        t_iso1, t_blk1, t_step1 = sample()
    return {
        "value": 1.0 / t_step,
        "unit": "RG-steps/s",
        "cores": int(threads),
        "kind": "oracle",
        "extrapolated": True,
        "sample": (f"oracle FP64 NumPy, seeded random D={D} 4D tensor (the shape of the Dcut={D} step): the 6 "
                   f"HOSVD isometries of one step ({t_iso:.2f} s) plus {blocks} block(s) "
                   f"T'[x0,x2,Y,Y',:,:,:,:] of the block-spin contraction ({t_blk:.2f} s each, 1/D^4 of the "
                   f"join), join scaled by D^4 = {D ** 4}"),
        "one_core": {"value": 1.0 / t_step1, "unit": "RG-steps/s", "cores": 1, "extrapolated": True,
                     "isometries_s": t_iso1, "block_s": t_blk1},
    }


def start_cpu_baseline(dcut, blocks):
    """The oracle baseline in a child process, so that it runs on the host
    cores while the GPU runs the comparison precisions."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-only", "--dcut", str(dcut),
           "--cpu-sample-blocks", str(blocks)]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def finish_cpu_baseline(proc):
    out, err = proc.communicate(timeout=600)
    if proc.returncode != 0:
        progress(f"cpu baseline failed: {err[-2000:]}")
        return None
    return json.loads(out.strip().splitlines()[-1])


def serving_window(precision, rate, window, budget_gb=200.0):
    """A time-boxed window of the serving stream: the first arrivals of a
    Poisson stream of HOTRG solves (beta ~ U[0.1490, 0.1505], h uniform on
    {0, 1e-6, 1e-5}, Dcut uniform on {6, 8, 10}, L = 2^k with k ~ U{4..10})
    at `rate` per second, served by continuous batching for `window`
    seconds; unfinished solves are censored and counted."""
    from paper_1911_12954_amd.serve import Server, TrgBackend
    from trg_inputs import serving_requests
    n = max(1, int(rate * window * 2) + 8)
    reqs = [r for r in serving_requests(n, rate, seed=0, dcuts=(6, 8, 10), kmin=4, kmax=10)
            if r["arrival"] < window]
    srv = Server(TrgBackend(precision), int(budget_gb * 2 ** 30))
    progress(f"serving window: {len(reqs)} arrivals in {window:.0f} s")
    summ = srv.serve(reqs, window=window)
    waiting = len(reqs) - summ["completed"] - summ["censored_active"]
    done_by = {}
    for r in srv.results:
        done_by.setdefault(str(r["dcut"]), []).append(r["latency"])
    srv.close()
    arrived_by = {}
    for r in reqs:
        arrived_by[str(r["dcut"])] = arrived_by.get(str(r["dcut"]), 0) + 1
    return {
        "solves_per_s": summ["solves_per_s"], "p50_latency_s": summ["p50_latency_s"],
        "p99_latency_s": summ["p99_latency_s"], "join_precision": precision,
        "window_s": window, "arrival_rate_per_s": rate, "arrived": len(reqs), "completed": summ["completed"],
        "censored_running": summ["censored_active"], "censored_waiting": waiting,
        "arrived_by_dcut": arrived_by, "completed_by_dcut": {k: len(v) for k, v in sorted(done_by.items())},
        "mean_runs_per_step_call": summ["mean_runs_per_call"],
        "stream": "Poisson, seed 0: beta~U[0.1490,0.1505], h in {0,1e-6,1e-5}, Dcut in {6,8,10}, L=2^k, "
                  "k~U{4..10}; first arrivals within the window",
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the multi-GPU sharding of the "
                                   "step is a design, not built); use --gpus 1"}))
        sys.exit(2)
    if a.cpu_only:
        print(json.dumps(cpu_baseline(a.dcut, a.cpu_sample_blocks)), flush=True)
        return
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.copy_cal > 0:
        n = int(a.copy_cal * 2 ** 30) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}), flush=True)
        return
    if a.step_error:
        print(json.dumps(step_error(a.step_error)), flush=True)
        return
    if a.atrg_scan:
        print(json.dumps(atrg_scan(a.atrg_scan)), flush=True)
        return
    if a.atrg_impure:
        print(json.dumps(atrg_impure(a.atrg_impure)), flush=True)
        return
    if a.vendor_gemm:
        print(json.dumps(vendor_gemm(a.vendor_gemm)), flush=True)
        return
    if a.accuracy:
        print(json.dumps(accuracy(a.accuracy, a.accuracy_variants)), flush=True)
        return
    if a.atrg_study:
        print(json.dumps(atrg_study(a.atrg_study)), flush=True)
        return
    if a.tc_bisect:
        from paper_1911_12954_amd.scan import bisect_transition, indicator_after
        fields = a.tc_bisect.split(",")
        d, dcut, steps, blo, bhi, tol = fields[:6]
        method = fields[6] if len(fields) > 6 else "hotrg"
        z2 = method == "atrg-z2"
        run_method = "atrg" if z2 else method
        d, dcut, steps, blo, bhi, tol = int(d), int(dcut), int(steps), float(blo), float(bhi), float(tol)
        t0 = time.perf_counter()

        def ev(beta):
            x = indicator_after(beta, d, dcut, steps, method=run_method, z2=z2)
            progress(f"tc-bisect: beta {beta:.8f} X {x:.6f} at {time.perf_counter() - t0:.1f} s")
            return x

        b = bisect_transition(d, dcut, blo, bhi, steps, tol, evaluate=ev)
        print(json.dumps({"metric": "transition bracket from the indicator X (bisection on beta)",
                          "method": method, "d": d, "dcut": dcut, "steps": steps, "beta_lo": b.beta_lo, "beta_hi": b.beta_hi,
                          "T_lo": 1.0 / b.beta_hi, "T_hi": 1.0 / b.beta_lo, "evaluations": b.evaluations,
                          "seconds": time.perf_counter() - t0}), flush=True)
        return
    if a.serve:
        from paper_1911_12954_amd.serve import Server, TrgBackend
        from trg_inputs import serving_requests
        dcuts = tuple(int(x) for x in a.serve_dcuts.split(","))
        methods = tuple(a.serve_methods.split(","))
        kmin, kmax = (int(x) for x in a.serve_k.split(","))
        budget = int(a.serve_budget_gb * 2 ** 30)
        rate, calib = a.serve_rate, None
        if rate == 0:
            # calibration: one solve per Dcut alone at L = 2^kmin; a solve of
            # L = 2^k costs about k/kmin times as much; the stream runs at 0.8
            # of the capacity these service times give
            calib = {}
            for m in methods:
                for D in dcuts:
                    one = Server(TrgBackend(a.serve_precision), budget)
                    t = time.perf_counter()
                    one.serve([{"id": 0, "arrival": 0.0, "beta": 0.1497, "h": 0.0, "dcut": D, "L": 2 ** kmin,
                                "method": m}], idle_sleep=1e-4)
                    calib[f"{m}:{D}"] = time.perf_counter() - t
                    one.close()
                    progress(f"calibration: {m} Dcut {D}, L 2^{kmin} alone: {calib[f'{m}:{D}']:.3f} s")
            ks = range(kmin, kmax + 1)
            mean_service = sum(v * k / kmin for v in calib.values() for k in ks) / (len(calib) * len(ks))
            rate = 0.8 / mean_service
            progress(f"calibration: mean service {mean_service:.3f} s, arrival rate {rate:.3f}/s")
        if rate < 0:
            # saturation: every request is there at the start
            reqs = serving_requests(a.serve_n, 1.0, seed=0, dcuts=dcuts, kmin=kmin, kmax=kmax, methods=methods)
            for r in reqs:
                r["arrival"] = 0.0
        else:
            reqs = serving_requests(a.serve_n, rate, seed=0, dcuts=dcuts, kmin=kmin, kmax=kmax, methods=methods)
        srv = Server(TrgBackend(a.serve_precision), budget)
        progress(f"serving {len(reqs)} requests, window {a.serve_window} s")
        summ = srv.serve(reqs, window=a.serve_window)
        srv.close()
        by_dcut = {}
        for r in srv.results:
            key = r["dcut"] if len(methods) == 1 else f"{r['method']}:{r['dcut']}"
            by_dcut.setdefault(key, []).append(r["latency"])
        print(json.dumps({
            "metric": "served %s solves/s and latency (continuous batching, 1 GPU)" % "+".join(
                m.upper() for m in methods),
            "value": summ["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
            "p50_latency_s": summ["p50_latency_s"], "p99_latency_s": summ["p99_latency_s"],
            "dtype": a.serve_precision, "data": "synthetic Poisson stream",
            "config": {"workload": "Poisson stream: beta~U[0.1490,0.1505], h in {0,1e-6,1e-5}, Dcut in %s, "
                                   "L=2^k, k~U{%d..%d}, methods %s, rate %.3f/s (<0: all at t=0), window %.0f s" %
                                   (list(dcuts), kmin, kmax, list(methods), rate, a.serve_window),
                       "calibration_s": calib},
            "summary": summ,
            "completed_by_dcut": {str(k): len(v) for k, v in sorted(by_dcut.items(), key=lambda kv: str(kv[0]))}}),
              flush=True)
        return
    if a.method == "atrg":
        D = a.dcut if a.dcut != 10 else 24
        prec = a.precision if a.precision in ("fp64", "fp32") else "fp64"
        el, ms, nl, fl, lnz = time_atrg(prec, D, a.beta, a.warmup, a.steps)
        ach = fl / (ms * 1e-3) / 1e12 if ms > 0 else None
        print(json.dumps({
            "metric": "4D ATRG RG-steps/s at Dcut=%d (steady-state step, 1 GPU)" % D,
            "value": a.steps / el, "unit": "RG-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": 1e3 * el / a.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": prec, "data": "synthetic (closed-form 4D Ising tensor, beta=%.4f, h=0)" % a.beta,
            "config": {"workload": "4D Ising ATRG, Dcut=%d, p=4Dcut, q=2Dcut, contraction %s" % (D, prec),
                       "lnZ_per_site_after_run": lnz},
            "roofline": {"bound": "mfma", "kernel": "gemm_nt_kernel (ATRG contraction, M=D^4 K=D^2 N=D^3)",
                         "achieved": ach, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                         "frac": (ach / PEAK_TFLOPS[prec]) if ach else None, "traffic": None,
                         "launches": nl, "gemm_ms_per_step": ms / a.steps,
                         "gemm_share_of_step": ms * 1e-3 / el}}), flush=True)
        return
    D = a.dcut
    compare = [x for x in a.compare.split(",") if x in PEAK_TFLOPS and x != a.precision]
    # ln Z/V of every precision is compared after the last step of the
    # comparison runs (ramp of 4 steps, warm-up, timed steps)
    probe_step = 4 + a.compare_warmup + a.compare_steps
    head = time_steps(a.precision, D, a.beta, a.warmup, a.steps, a.impure, probe_step=probe_step)
    elapsed, join_ms, launches = head["elapsed"], head["join_ms"], head["launches"]
    steps_per_s = a.steps / elapsed
    # each impure tensor adds the joins C(S, T) and C(T, S)
    joins_per_step = 5 if a.impure else 1
    alg_flops_step = 2.0 * D ** 15 * joins_per_step
    mult = SPLIT_PRODUCTS.get(a.precision, 1.0)   # BF16 MFMA products per multiply-add
    achieved = alg_flops_step * a.steps / (join_ms * 1e-3) / 1e12 if join_ms > 0 else None
    peak = PEAK_TFLOPS[a.precision]
    traffic = None if a.impure else join_traffic(a.precision, D)
    out = {
        "metric": "4D HOTRG RG-steps/s at Dcut=%d (steady-state step%s, 1 GPU)" % (
            D, ", impure E and M" if a.impure else ""),
        "value": steps_per_s,
        "unit": "RG-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16x3 (bf16 MFMA, fp32 accumulate; fp64 Gram/eigh/norm)",
                  "bf16x6": "bf16x6 (bf16 MFMA, fp32 groups of 128 summed in fp64; fp64 Gram/eigh/norm)",
                  "fp32": "fp32 (fp32 MFMA; fp64 Gram/eigh/norm)", "fp64": "fp64"}[a.precision],
        "data": "synthetic (closed-form 4D Ising tensor, beta=%.4f, h=0)" % a.beta,
        "config": {"workload": "4D Ising HOTRG, Dcut=%d, steady-state coarse-graining step%s, beta=%.4f, h=0, "
                               "join precision %s" % (D, " with impure E and M (5 joins)" if a.impure else "",
                                                      a.beta, a.precision),
                   "dcut": D, "join_precision": a.precision, "lnZ_per_site_after_run": head["lnz"],
                   "steps_in_run": head["steps_total"]},
        "roofline": {
            "bound": "mfma",
            "kernel": "gemm_nt_kernel (join, D^15 block-spin contraction)",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": (achieved / peak) if achieved else None,
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "traffic_algorithmic": traffic["algorithmic_bytes_per_launch"] if traffic else None,
            "traffic_counters": traffic["source"] if traffic else None,
            "join_launches": launches,
            "join_ms_per_step": join_ms / a.steps,
            "join_share_of_step": (join_ms * 1e-3) / elapsed,
            "mfma_issued_tflops": mult * achieved if achieved else None,
            "mfma_issued_frac": (mult * achieved / peak) if achieved else None,
            "achieved_over_fp32_mfma_peak": (achieved / PEAK_TFLOPS["fp32"]) if achieved else None,
        },
    }
    cpu_proc = None
    if not a.no_cpu:
        cpu_proc = start_cpu_baseline(D, a.cpu_sample_blocks)
    others = {}
    for prec in compare:
        r = time_steps(prec, D, a.beta, a.compare_warmup, a.compare_steps, a.impure, probe_step=probe_step)
        ach = alg_flops_step * a.compare_steps / (r["join_ms"] * 1e-3) / 1e12
        others[prec] = {"rg_steps_per_s": a.compare_steps / r["elapsed"], "warmup": a.compare_warmup,
                        "steps": a.compare_steps, "join_tflops": ach, "frac_of_peak": ach / PEAK_TFLOPS[prec],
                        "lnZ_per_site_after_step_%d" % probe_step: r["lnz"] if r["steps_total"] == probe_step
                        else None}
    if others:
        out["other_precisions"] = others
        if "fp64" in others:
            ref = others["fp64"]["lnZ_per_site_after_step_%d" % probe_step]
            out["speedup_vs_fp64_path"] = steps_per_s / others["fp64"]["rg_steps_per_s"]
            rel = lambda x: abs(x - ref) / abs(ref) if x is not None and ref is not None else None
            errs = {a.precision: rel(head["probe"])}
            for prec in others:
                if prec != "fp64":
                    errs[prec] = rel(others[prec]["lnZ_per_site_after_step_%d" % probe_step])
            out["f_rel_err_vs_fp64_path"] = {"after_step": probe_step, **errs}
            out["accuracy_records"] = ("f, E, M of whole runs against the FP64 path (4D Dcut 8, L = 1024, "
                                       "h = 1e-5, and the other configurations): bench.py --accuracy")
    if cpu_proc is not None:
        cb = finish_cpu_baseline(cpu_proc)
        if cb is not None:
            out["cpu_baseline"] = cb
    if not a.no_serve and a.method == "hotrg":
        out["serving"] = serving_window(a.precision, a.window_rate, a.window_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
