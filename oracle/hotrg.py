"""HOTRG coarse-graining of a d-dimensional tensor network (oracle, test infrastructure).

Method: Sec. 2 and Fig. 1 of the paper.  A HOTRG step along axis mu joins two
neighbouring site tensors (site 1 below, site 2 above along mu) by contracting
the forward mu leg of site 1 with the backward mu leg of site 2.  The pairs of
transverse legs that the join creates are compressed by isometries U_nu taken
from a higher-order SVD (HOSVD, Fig. 1B) of the two-site tensor.  The memory
cost is D^{2d}; the D^{4d-1} part of the time is the contraction that completes
the block-spin transformation (the red dotted circle of Fig. 1B, Sec. 2).  The
lattice halves along mu (Fig. 1C); volume 2^n after n steps (Fig. 5 caption).

Readings of details the paper leaves to its references (listed in the design doc):

* Legs in the order (x, x', y, y', ...): backward leg 2*nu, forward leg 2*nu+1.
* HOSVD environment of axis nu on side s (backward or forward pair):
  Gram^s_nu = M_(nu s) M_(nu s)^T, M the two-site tensor.  It is evaluated as
  Gram[(a,b),(a',b')] = sum_{i,i'} P[i,a,i',a'] Q[i,b,i',b'], with P the
  environment of site 1 keeping its forward mu leg and its nu leg on side s,
  and Q that of site 2 keeping its backward mu leg and its nu leg on side s.
  This regroups the sum of M_(nu s) M_(nu s)^T exactly.
* Truncation keeps k = min(d_nu^2, Dcut) leading eigenvectors;
  eps^s = sum of the discarded max(lambda, 0).  The forward side is used
  unless eps^- < (1 - 1e-10) eps^+.
* The sign of each eigenvector and the basis of each degenerate eigenspace
  (neighbouring eigenvalues within 1e-10 lambda_max) are fixed canonically:
  the basis is built from the eigenspace's projector P by taking P e_r /
  sqrt(P_rr) for the first coordinate r of largest remaining weight (ties
  within a relative 1e-9 go to the lowest index), then deflating.  Inside the
  kept space this is gauge freedom (f, E, M and ln c_n do not depend on it);
  when the cut splits a degenerate eigenspace it decides which vectors are
  kept, and fixing it makes that choice reproducible.  The window only has
  to hold the degeneracies that a symmetry makes exact, which FP64 rounding
  leaves as gaps of about 1e-17 lambda_max; every gap above it is resolved
  by plain truncated HOSVD (the leading k eigenvectors).
* The same U_nu[a, b, k] (a from site 1, b from site 2) compresses both the
  backward pair and the forward pair of legs along nu.
* Normalisation c_n = Frobenius norm; ln Z/V = sum_{n=0}^{N} 2^{-n} ln c_n
  + 2^{-N} ln Tr T_N for N steps on a periodic lattice of 2^N sites.
* Impure tensors (Sec. 3.1, the impure-tensor method):
  S_n = [C(S, T) + C(T, S)] / (2 c_n), C built with the pure step's U's;
  M = Tr S_M / Tr T and E = -Tr S_E / Tr T at the end (S_E = dT0/dbeta).
"""
from __future__ import annotations

import math
import string
from dataclasses import dataclass, field

import numpy as np

SIDE_BACKWARD = 0
SIDE_FORWARD = 1
TIE_REL = 1e-10          # side-rule tie window
SIGN_REL = 1e-9          # sign-fix tie window
DEGEN_REL = 1e-8         # degenerate-cut flag
CLUSTER_REL = 1e-10      # eigenvalues closer than this * lambda_max are degenerate


def transverse_axes(d: int, mu: int):
    """Transverse axes of a step along mu, split into the ones compressed on the
    operands before the join (first ceil((d-1)/2)) and the rest (after).  The
    split is an evaluation order only: every split gives the same tensor."""
    others = [nu for nu in range(d) if nu != mu]
    ns = (len(others) + 1) // 2
    return others, others[:ns], others[ns:]


# --------------------------------------------------------------------------
# HOSVD environment (Fig. 1B): Gram matrices and isometries
# --------------------------------------------------------------------------

def _letters(n):
    pool = string.ascii_letters
    assert n <= len(pool)
    return pool[:n]


def gram(A: np.ndarray, B: np.ndarray, mu: int, nu: int, side: int) -> np.ndarray:
    """Gram^s_nu of the two-site tensor made of A (site 1) and B (site 2).

    Returns the (dA*dB) x (dA*dB) matrix over the pair (a, b) of the nu legs on
    side s, where a is site 1's leg and b site 2's leg."""
    nl = A.ndim
    L = _letters(nl)
    # P[i, a, i', a'] = sum over the other legs of A[..] A[..]
    s1 = list(L[:nl]); s2 = list(s1)
    s2[2 * mu + 1] = "I"; s2[2 * nu + side] = "J"
    P = np.einsum("".join(s1) + "," + "".join(s2) + "->" + s1[2 * mu + 1] + s1[2 * nu + side] + "IJ",
                  A, A, optimize=True)
    t1 = list(L[:nl]); t2 = list(t1)
    t2[2 * mu] = "I"; t2[2 * nu + side] = "J"
    Q = np.einsum("".join(t1) + "," + "".join(t2) + "->" + t1[2 * mu] + t1[2 * nu + side] + "IJ",
                  B, B, optimize=True)
    # Gram[a, b, a', b'] = sum_{i, i'} P[i, a, i', a'] Q[i, b, i', b']
    G = np.einsum("iakc,ibkd->abcd", P, Q, optimize=True)
    n = G.shape[0] * G.shape[1]
    return G.reshape(n, n)


@dataclass
class AxisChoice:
    nu: int
    side: int
    k: int
    eps: tuple            # (eps_backward, eps_forward)
    spectrum: np.ndarray  # eigenvalues of the chosen side, descending
    degenerate_cut: bool
    U: np.ndarray         # (d_nu, d_nu, k)


def _eig_desc(G):
    G = 0.5 * (G + G.T)
    w, v = np.linalg.eigh(G)
    order = np.argsort(-w, kind="stable")
    return w[order], v[:, order]


def _clusters(w, tol):
    """Split a descending spectrum into runs of consecutive eigenvalues whose
    neighbouring gaps are at most ``tol``; returns [(start, stop), ...]."""
    runs, start = [], 0
    for i in range(1, len(w) + 1):
        if i == len(w) or w[i - 1] - w[i] > tol:
            runs.append((start, i))
            start = i
    return runs


def _canonical_basis(V):
    """A basis of span(V) that does not depend on the basis V itself.

    Repeatedly take the first coordinate r whose weight in the remaining
    projector P is within a relative SIGN_REL of the largest, and emit
    P e_r / sqrt(P_rr); then remove that vector from P.  For one vector this
    is the vector signed so that its largest component is positive."""
    n, m = V.shape
    out = np.zeros((n, m))
    for j in range(m):
        diag = np.sum(V * V, axis=1) - np.sum(out[:, :j] ** 2, axis=1)
        r = int(np.nonzero(diag >= (1.0 - SIGN_REL) * diag.max())[0][0])
        col = V @ V[r, :] - out[:, :j] @ out[r, :j]
        out[:, j] = col / math.sqrt(col[r])
    return out


def _kept_vectors(w, v, k):
    """The first k eigenvectors with every degenerate eigenspace that overlaps
    them expressed in its canonical basis (clusters: gaps <= CLUSTER_REL *
    lambda_max)."""
    tol = CLUSTER_REL * max(float(w[0]), 0.0)
    U = np.zeros((v.shape[0], k))
    for a, b in _clusters(w, tol):
        if a >= k:
            break
        basis = _canonical_basis(v[:, a:b])
        stop = min(b, k)
        U[:, a:stop] = basis[:, : stop - a]
    return U


def isometry(T: np.ndarray, mu: int, nu: int, dcut: int, force_side=None) -> AxisChoice:
    """Truncated isometry U_nu for a step along mu (HOSVD, Fig. 1B)."""
    dn = T.shape[2 * nu]
    n = dn * dn
    k = min(n, dcut)
    res = []
    for side in (SIDE_BACKWARD, SIDE_FORWARD):
        w, v = _eig_desc(gram(T, T, mu, nu, side))
        eps = float(np.sum(np.maximum(w[k:], 0.0)))
        res.append((w, v, eps))
    eps_b, eps_f = res[0][2], res[1][2]
    if force_side is not None:
        side = force_side
    else:
        side = SIDE_BACKWARD if eps_b < (1.0 - TIE_REL) * eps_f else SIDE_FORWARD
    w, v, _ = res[side]
    degenerate = bool(k < n and w[k - 1] > 0 and (w[k - 1] - w[k]) <= DEGEN_REL * w[k - 1])
    U = _kept_vectors(w, v, k).reshape(dn, dn, k)
    return AxisChoice(nu, side, k, (eps_b, eps_f), w, degenerate, U)


# --------------------------------------------------------------------------
# Block-spin contraction C(A, B) (Fig. 1B red circle, Fig. 1C)
# --------------------------------------------------------------------------

def _coarse_grain_block(a, b, U, mu, d, Uf=None):
    """C(A, B) restricted to the x0 values present in ``a`` and the x2 values
    present in ``b``: ``a`` is A with its backward mu leg cut to those x0,
    ``b`` is B with its forward mu leg cut to those x2.

    Sums over the joined mu leg i (A's forward mu leg = B's backward mu leg)
    and over each transverse pair through U_nu[a_nu, b_nu, K_nu] (backward
    legs) and U_nu[a'_nu, b'_nu, L_nu] (forward legs; ``Uf`` when given
    supplies these, e.g. column subsets for sampling).  Legs of the result in
    the canonical order: (x0, x2) on axis mu and (K_nu, L_nu) elsewhere."""
    Uf = U if Uf is None else Uf
    others, pre, post = transverse_axes(d, mu)
    L = iter(_letters(3 + 6 * len(others)))
    i, x0, x2 = next(L), next(L), next(L)
    la, lp, lb, lq, lK, lL = {}, {}, {}, {}, {}, {}
    for nu in others:
        la[nu], lp[nu], lb[nu], lq[nu], lK[nu], lL[nu] = (next(L) for _ in range(6))
    sa, sb = [], []
    for ax in range(d):
        sa += [x0, i] if ax == mu else [la[ax], lp[ax]]
        sb += [i, x2] if ax == mu else [lb[ax], lq[ax]]

    def ein(s_in, s_u, s_out, x, u):
        return np.einsum("".join(s_in) + "," + s_u + "->" + "".join(s_out), x, u, optimize=True)

    # compress site 1's backward legs and site 2's forward legs along pre axes
    for nu in pre:
        new = [x for x in sa if x != la[nu]] + [lb[nu], lK[nu]]
        a, sa = ein(sa, la[nu] + lb[nu] + lK[nu], new, a, U[nu]), new
        new = [x for x in sb if x != lq[nu]] + [lp[nu], lL[nu]]
        b, sb = ein(sb, lp[nu] + lq[nu] + lL[nu], new, b, Uf[nu]), new
    # join: sum over i and the pre-axis legs shared by a and b
    shared = set(sa) & set(sb)
    se = [x for x in sa if x not in shared] + [x for x in sb if x not in shared]
    e = np.einsum("".join(sa) + "," + "".join(sb) + "->" + "".join(se), a, b, optimize=True)
    # compress the remaining transverse pairs
    for nu in post:
        new = [x for x in se if x not in (la[nu], lb[nu])] + [lK[nu]]
        e, se = ein(se, la[nu] + lb[nu] + lK[nu], new, e, U[nu]), new
        new = [x for x in se if x not in (lp[nu], lq[nu])] + [lL[nu]]
        e, se = ein(se, lp[nu] + lq[nu] + lL[nu], new, e, Uf[nu]), new
    target = []
    for ax in range(d):
        target += [x0, x2] if ax == mu else [lK[ax], lL[ax]]
    return np.einsum("".join(se) + "->" + "".join(target), e)


SLICE_ELEMENTS = 1 << 24   # slice over (x0, x2) when an operand would exceed this


def coarse_grain(A: np.ndarray, B: np.ndarray, U: dict, mu: int, x0s=None, x2s=None,
                 U_forward=None) -> np.ndarray:
    """C(A, B): the coarse-grained tensor of site 1 = A and site 2 = B along mu.

    ``U`` maps each transverse axis nu to U_nu[a, b, k].  Legs of the result are
    in the canonical order with dims d_mu on the mu legs and k_nu elsewhere.
    ``x0s``/``x2s`` restrict the output to some values of the new backward and
    forward mu legs (used to sample large outputs); default all.
    ``U_forward`` (default ``U``) compresses the forward pairs; passing column
    subsets of U and U_forward samples blocks of the output.  Large problems
    are evaluated one (x0, x2) pair at a time to bound memory."""
    d = A.ndim // 2
    x0s = list(range(A.shape[2 * mu])) if x0s is None else list(x0s)
    x2s = list(range(B.shape[2 * mu + 1])) if x2s is None else list(x2s)
    a_all = np.take(A, x0s, axis=2 * mu)
    b_all = np.take(B, x2s, axis=2 * mu + 1)
    # size of the compressed operand: A's elements times the growth d_nu -> (d_nu, k_nu)
    _, pre, _ = transverse_axes(d, mu)
    grow = 1
    for nu in pre:
        grow *= U[nu].shape[1] * U[nu].shape[2] // U[nu].shape[0]
    if a_all.size * grow <= SLICE_ELEMENTS:
        return _coarse_grain_block(a_all, b_all, U, mu, d, U_forward)
    shape = list(A.shape)
    shape[2 * mu], shape[2 * mu + 1] = len(x0s), len(x2s)
    Uf = U if U_forward is None else U_forward
    for nu in range(d):
        if nu != mu:
            shape[2 * nu], shape[2 * nu + 1] = U[nu].shape[2], Uf[nu].shape[2]
    out = np.zeros(shape)
    for p in range(len(x0s)):
        a = np.take(a_all, [p], axis=2 * mu)
        for q in range(len(x2s)):
            b = np.take(b_all, [q], axis=2 * mu + 1)
            idx = [slice(None)] * (2 * d)
            idx[2 * mu], idx[2 * mu + 1] = slice(p, p + 1), slice(q, q + 1)
            out[tuple(idx)] = _coarse_grain_block(a, b, U, mu, d, U_forward)
    return out


# --------------------------------------------------------------------------
# Steps and whole runs
# --------------------------------------------------------------------------

@dataclass
class StepRecord:
    n: int
    mu: int
    ln_c: float
    dims: tuple
    axes: list = field(default_factory=list)   # AxisChoice per transverse axis


def hotrg_step(T: np.ndarray, mu: int, dcut: int, impurities=(), force_side=None,
               norm: str = "fro", transform_u=None):
    """One HOTRG step along mu on the normalised tensor T.

    Returns (T_new normalised, [S_new normalised ...], c, [AxisChoice ...]).
    ``norm`` picks the normalisation ("fro" or "max", both are gauge choices
    that leave ln Z/V, E and M unchanged); ``transform_u`` (tests only) maps
    the isometry dict before use, e.g. to apply a gauge rotation."""
    d = T.ndim // 2
    choices = [isometry(T, mu, nu, dcut, force_side) for nu in range(d) if nu != mu]
    U = {ch.nu: ch.U for ch in choices}
    if transform_u is not None:
        U = transform_u(U)
    Tn = coarse_grain(T, T, U, mu)
    if norm == "fro":
        c = float(np.sqrt(np.sum(Tn * Tn)))
    elif norm == "max":
        c = float(np.max(np.abs(Tn)))
    else:
        raise ValueError(norm)
    imps = [(coarse_grain(S, T, U, mu) + coarse_grain(T, S, U, mu)) / (2.0 * c) for S in impurities]
    return Tn / c, imps, c, choices


def periodic_trace(T: np.ndarray) -> float:
    """Tr T on a one-site periodic lattice: each backward leg joined to the
    forward leg of the same axis."""
    d = T.ndim // 2
    L = _letters(d)
    return float(np.einsum("".join(ch + ch for ch in L) + "->", T))


def indicator_matrix(T: np.ndarray, axis: int = 0) -> np.ndarray:
    """M[a][a'] = T with its two legs on `axis` open (a backward, a' forward)
    and every other axis' leg pair joined (traced), as on a lattice that is
    one site wide in all other directions."""
    d = T.ndim // 2
    L = _letters(d)            # lower-case letters: the open pair uses upper case
    spec = "".join(("YZ" if k == axis else ch + ch) for k, ch in enumerate(L))
    return np.einsum(spec + "->YZ", T)


def indicator_x(T: np.ndarray, axis: int = 0) -> float:
    """Degeneracy indicator of the largest tensor components (the quantity
    the paper plots against the HOTRG iteration, Sec. 3.1, Fig. 3, taken from
    Gu and Wen): X = (Tr M)^2 / Tr(M M), with M the matrix above, i.e. the
    squared one-site trace over the trace of two sites joined along `axis`.
    It is 1 for a single dominant component (disordered phase) and 2 for
    two degenerate ones (Z2 broken)."""
    M = indicator_matrix(T, axis)
    return float(np.trace(M) ** 2 / np.trace(M @ M))


@dataclass
class RunResult:
    ln_z_per_site: float
    energy: float
    magnetization: float
    acc: float
    trace: float
    steps: list


def run(beta: float, h: float, d: int, dcut: int, L: int, impure: bool = True,
        initial=None, force_side=None, norm: str = "fro", transform_u=None,
        axes=None) -> RunResult:
    """HOTRG on the periodic L^d lattice (L = 2^m): d*m steps along
    mu = (n-1) mod d (or the axis sequence ``axes``), then the final trace.
    Returns ln Z / V, E = <H>/V and M = <s> (E, M from the impure tensors;
    NaN when impure is False)."""
    m = int(round(math.log2(L)))
    if 2 ** m != L or m < 1:
        raise ValueError("L must be a power of two >= 2")
    from .ising import site_tensors
    T0, SM, SE = site_tensors(beta, h, d) if initial is None else initial
    c0 = float(np.sqrt(np.sum(T0 * T0)))
    T = T0 / c0
    imps = [SE / c0, SM / c0] if impure else []
    acc = math.log(c0)
    steps = [StepRecord(0, -1, math.log(c0), T.shape)]
    N = d * m
    seq = [(n - 1) % d for n in range(1, N + 1)] if axes is None else list(axes)
    if sorted(seq) != sorted((n - 1) % d for n in range(1, N + 1)):
        raise ValueError("axis sequence must halve every axis m times")
    for n, mu in enumerate(seq, start=1):
        T, imps, c, choices = hotrg_step(T, mu, dcut, imps, force_side, norm, transform_u)
        acc += 2.0 ** (-n) * math.log(c)
        steps.append(StepRecord(n, mu, math.log(c), T.shape, choices))
    tr = periodic_trace(T)
    lnz = acc + 2.0 ** (-N) * math.log(tr)
    if impure:
        E = -periodic_trace(imps[0]) / tr
        M = periodic_trace(imps[1]) / tr
    else:
        E = M = float("nan")
    return RunResult(lnz, E, M, acc, tr, steps)
