"""Location of the transition from the degeneracy indicator X (the paper's
diagnostic, Sec. 3.1 and Figs. 3-4): after enough coarse-graining steps X
tends to 1 in the disordered phase and to 2 in the ordered one, so a
bisection on beta between a disordered and an ordered bracket end brackets
the transition at the given bond dimension.  Every step and every X runs in
the HIP library; this module only orchestrates runs."""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass
class Bisection:
    beta_lo: float          # disordered (X < threshold)
    beta_hi: float          # ordered (X >= threshold)
    evaluations: list = field(default_factory=list)   # (beta, X) in the order run


def indicator_after(beta: float, d: int, dcut: int, steps: int, precision: str = "fp64", axis: int = 0,
                    h: float = 0.0, method: str = "hotrg", z2: bool = False) -> float:
    """X of the tensor after `steps` HOTRG (or ATRG) steps (axes cycled
    from 0); `z2` runs ATRG in its Z2 mode (h = 0), which keeps the ordered
    phase's symmetric fixed point (X -> 2) that a plain randomized swap
    loses over many steps."""
    from .trg import trg_init_ising
    ctx = trg_init_ising(beta, h, d, dcut=dcut, precision=precision, method=method, z2=z2)
    try:
        for n in range(steps):
            if method == "atrg":
                ctx.atrg_step(n % d, dcut)
            else:
                ctx.hotrg_step(n % d, dcut)
        return ctx.indicator_x(axis)
    finally:
        ctx.close()


def bisect_transition(d: int, dcut: int, beta_lo: float, beta_hi: float, steps: int, tol: float,
                      precision: str = "fp64", threshold: float = 1.5, evaluate=None,
                      method: str = "hotrg", z2: bool = False) -> Bisection:
    """Halve [beta_lo, beta_hi] until it is narrower than `tol`, keeping X
    below `threshold` at beta_lo and above it at beta_hi.  `evaluate(beta)`
    replaces the GPU run (tests)."""
    ev = evaluate or (lambda b: indicator_after(b, d, dcut, steps, precision, method=method, z2=z2))
    out = Bisection(beta_lo, beta_hi)
    x_lo, x_hi = ev(beta_lo), ev(beta_hi)
    out.evaluations += [(beta_lo, x_lo), (beta_hi, x_hi)]
    if not (x_lo < threshold <= x_hi):
        raise ValueError(f"the interval does not bracket the transition: X({beta_lo}) = {x_lo}, X({beta_hi}) = {x_hi}")
    while out.beta_hi - out.beta_lo > tol:
        mid = 0.5 * (out.beta_lo + out.beta_hi)
        x = ev(mid)
        out.evaluations.append((mid, x))
        if x < threshold:
            out.beta_lo = mid
        else:
            out.beta_hi = mid
    return out
