"""ATRG coarse-graining of a d-dimensional tensor network (oracle, test infrastructure).

Method: Sec. 2 and Fig. 2 of the paper.  ATRG keeps every site tensor as a
product of two pieces and makes two approximations: a singular value
decomposition of each local tensor, and a HOSVD of the two adjacent
decomposed tensors.  The partial SVD that swaps tensor indices (the dark-blue
tensors of Fig. 2B) and the contraction completing the block-spin
transformation (the red dotted circle of Fig. 2B) are the two D^{2d+1} parts;
the memory is D^{d+1}.  The partial SVD is a randomized SVD (RSVD) with a
trial matrix drawn from N(0,1), oversampling p and q iterations of the
orthogonal-matrix update (Sec. 3.2: p = 4 Dcut, q = 2 Dcut).

Readings (the algorithm is given in Adachi et al., which the paper cites;
each choice below is listed in the design doc):

* A tensor T[b, f] (b = backward legs, f = forward legs, each in axis order)
  is held as T = U diag(s) V with U[b, k], V[k, f].  The first local SVD of
  the Ising tensor is exact (it has rank 2 in that bipartition); after a step
  the new tensor is already a product over one index of dim <= Dcut, so the
  "local SVD" is a canonicalisation (QR of both pieces, SVD of the small core)
  and the approximations are the swap and the HOSVD.  The sign of each
  singular-vector pair is fixed (largest entry of the left vector positive),
  so that the randomized SVD, which is not converged for every input, sees
  the same swap matrix in every implementation.
* Step along mu with site A below and site B above: with
  Ut = U sqrt(s) and Vt = sqrt(s) V,
  M[(k_A, b^B_perp), (f^A_perp, k_B)] = sum_j Vt[k_A, f^A_perp, f_mu = j] Ut[b_mu = j, b^B_perp, k_B]
  is truncated to rank Dcut by RSVD: M ~ X diag(sigma) Y.  This swaps the
  transverse legs between the pieces.
* G[b^A, b^B_perp, l] = sum_kA Ut[b^A, k_A] X[k_A, b^B_perp, l] sqrt(sigma_l) holds all
  backward legs, H[l, f^A_perp, f^B] = sqrt(sigma_l) sum_kB Y[l, f^A_perp, k_B] Vt[k_B, f^B]
  all forward legs; the two-site tensor is sum_l G H.
* HOSVD: for each transverse nu, the Gram matrix of the two-site tensor over
  the backward pair (b^A_nu, b^B_nu) and over the forward pair (f^A_nu,
  f^B_nu); the same selection rule as HOTRG (smaller discarded weight,
  forward on a tie, canonical basis of degenerate eigenspaces) gives P_nu,
  applied to both pairs.
* New pieces G'[b_mu, B_perp, l] and H'[l, F_perp, f_mu]; normalisation
  c = ||G' H'||_F = sqrt(Tr[(G'^T G')(H' H'^T)]), both pieces scaled by
  c^{-1/2}, acc += 2^{-n} ln c.  Tr T = sum_l sum_b G'[b, l] H'[l, b].
* Impure tensors (Sec. 3.2 applies the impure-tensor method within ATRG
  without spelling it out).  An impurity is kept as its own pair of pieces,
  S = sum_m G_S[b, m] H_S[m, f].  Initially G_S is the pure backward piece
  and H_S carries the impurity: S_M exactly, and the energy impurity with the
  derivative of each bond weight put on the bond's forward end
  (sum_k 2 W'[s, k] W[s', k] = d e^{beta s s'} / d beta), so that
  -Tr S_E / Tr T is again <H>/V.  A step forms C(S, T) + C(T, S) over 2c:
  - impurity on the lower site: the two-site middle matrix
    M_1[(m, b_perp), (f_perp, kB)] = sum_j H_S[m, f_perp, j] Ut[j, b_perp, kB]
    gets its own partial SVD of rank Dcut (the same randomized SVD as the
    pure swap), M_1 ~ X_1 sigma_1 Y_1, and the pieces G_S X_1 sqrt(sigma_1),
    sqrt(sigma_1) Y_1 Vt;
  - impurity on the upper site: M_2[(kA, b_perp), (f_perp, m)] =
    sum_j Vt[kA, f_perp, j] G_S[j, b_perp, m] likewise, pieces
    Ut X_2 sqrt(sigma_2) and sqrt(sigma_2) Y_2 H_S;
  - the two terms side by side (bond 2 Dcut), the pure step's HOSVD
    isometries on the backward and the forward legs, c^{-1/2} on each piece
    and the 1/2 on the forward one.
  Only the isometries are shared with the pure tensor: projecting the
  impure middle matrices on the pure swap's singular vectors instead loses
  about 2 % of E in 2D at Dcut = 16 (their dominant directions differ).
  The trial matrix of the impurity SVDs is drawn like the pure one with the
  third counter word 1 + 2 kind + term (kind 0 energy, 1 magnetization;
  term 0 lower site, 1 upper site).  With nothing truncated every SVD is
  exact and E, M are exact.
* RSVD (Halko et al. as in Erichson et al.): Q = orth(M Omega); q times
  Z = orth(M^T Q), Q = orth(M Z); then the SVD of Q^T M.  Omega has
  Dcut + p columns; entry (i, c) of step n comes from Philox4x32-10 with key
  (seed low, seed high) and counter (i * ncols + c, n, 0, 0): the first two
  output words give uniforms u = (w + 0.5) / 2^32 and one Box-Muller normal
  sqrt(-2 ln u1) cos(2 pi u2).
"""
from __future__ import annotations

import math
import string
from dataclasses import dataclass, field

import numpy as np

from . import hotrg
from .ising import bond_split, bond_split_dbeta

# ------------------------------------------------------------------ Philox ---
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11) on four
    32-bit counter words and two 32-bit key words; returns four words."""
    c = [int(x) & MASK32 for x in counter]
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c[0]
        p1 = PHILOX_M1 * c[2]
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def philox4x32_10_vec(ctr0, ctr1, key, ctr2=0):
    """Vectorised Philox4x32-10 over arrays of the first two counter words
    (the third is ctr2, the last zero); returns the first two output words."""
    c0 = np.asarray(ctr0, dtype=np.uint64) & MASK32
    c1 = np.asarray(ctr1, dtype=np.uint64) & MASK32
    c2 = np.full_like(c0, int(ctr2) & MASK32)
    c3 = np.zeros_like(c0)
    k0, k1 = np.uint64(key[0] & MASK32), np.uint64(key[1] & MASK32)
    m0, m1 = np.uint64(PHILOX_M0), np.uint64(PHILOX_M1)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + PHILOX_W0) & MASK32)
            k1 = np.uint64((int(k1) + PHILOX_W1) & MASK32)
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1


def trial_matrix(rows: int, cols: int, step: int, seed: int, stream: int = 0) -> np.ndarray:
    """Gaussian trial matrix Omega[rows, cols] of ATRG step `step` (stream 0:
    the pure swap; stream s > 0: counter word 2 = s, the impurity SVDs)."""
    e = np.arange(rows * cols, dtype=np.uint64)
    w0, w1 = philox4x32_10_vec(e, np.full_like(e, step), (seed & MASK32, (seed >> 32) & MASK32), stream)
    u1 = (w0.astype(np.float64) + 0.5) / 4294967296.0
    u2 = (w1.astype(np.float64) + 0.5) / 4294967296.0
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return z.reshape(rows, cols)


# ------------------------------------------------------------ factored state ---
@dataclass
class Factors:
    """T[b, f] = sum_k U[b..., k] s[k] V[k, f...] (b, f: d legs each)."""
    U: np.ndarray
    s: np.ndarray
    V: np.ndarray

    @property
    def d(self):
        return self.U.ndim - 1

    def dims(self):
        return self.U.shape[:-1]

    def dense(self):
        d = self.d
        Um = self.U.reshape(-1, self.U.shape[-1])
        Vm = self.V.reshape(self.V.shape[0], -1)
        return ((Um * self.s) @ Vm).reshape(self.U.shape[:-1] + self.V.shape[1:])


def ising_factors(beta: float, h: float, d: int) -> Factors:
    """Exact rank-2 factorisation of the Ising site tensor in the
    (backward | forward) bipartition: T0[b, f] = sum_sigma u_sigma[b] v_sigma[f]
    with u_sigma[b] = e^{beta h sigma/2} prod W[sigma, b_nu] (v the same)."""
    W = bond_split(beta)
    U = np.zeros((2,) * d + (2,))
    for row, spin in enumerate((1.0, -1.0)):
        u = np.array(math.exp(0.5 * beta * h * spin))
        for _ in range(d):
            u = np.multiply.outer(u, W[row])
        U[..., row] = u
    V = np.moveaxis(U, -1, 0).copy()
    return Factors(U, np.ones(2), V)


def ising_impurity_pieces(beta: float, h: float, d: int):
    """Forward pieces H_E, H_M [sigma, f...] of the energy and magnetization
    impurities on the backward piece of ising_factors: S = sum_sigma
    u_sigma[b] H_S[sigma, f], with H_M = sigma v_sigma and
    H_E = e^{beta h sigma/2} (h sigma prod_nu W[sigma, f_nu]
          + sum_nu 2 W'[sigma, f_nu] prod_{nu' != nu} W[sigma, f_nu'])."""
    W = bond_split(beta)
    dW = bond_split_dbeta(beta) if beta > 0 else np.zeros((2, 2))
    HE = np.zeros((2,) + (2,) * d)
    HM = np.zeros((2,) + (2,) * d)
    for row, spin in enumerate((1.0, -1.0)):
        pref = math.exp(0.5 * beta * h * spin)
        v = np.array(pref)
        for _ in range(d):
            v = np.multiply.outer(v, W[row])
        HM[row] = spin * v
        e = h * spin * v
        for nu in range(d):
            t = np.array(pref)
            for a in range(d):
                t = np.multiply.outer(t, 2.0 * dW[row] if a == nu else W[row])
            e = e + t
        HE[row] = e
    return HE, HM


def canonical(G: np.ndarray, H: np.ndarray, dcut: int) -> Factors:
    """Local SVD of T = G H (G[b..., l], H[l, f...]): QR of both pieces and an
    SVD of the small core; keeps at most dcut singular values."""
    r = G.shape[-1]
    Gm = G.reshape(-1, r)
    Hm = H.reshape(r, -1)
    Qg, Rg = np.linalg.qr(Gm)
    Qh, Rh = np.linalg.qr(Hm.T)
    W, s, Zt = np.linalg.svd(Rg @ Rh.T)
    k = min(dcut, int(np.count_nonzero(s > 0)) or 1, len(s))
    Um = Qg @ W[:, :k]
    Vm = Zt[:k] @ Qh.T
    # sign gauge: the first largest-modulus entry of each left singular
    # vector (within a relative 1e-9) is positive; the right vector follows
    for j in range(k):
        col = np.abs(Um[:, j])
        i = int(np.nonzero(col >= (1.0 - 1e-9) * col.max())[0][0])
        if Um[i, j] < 0:
            Um[:, j] = -Um[:, j]
            Vm[j] = -Vm[j]
    U = Um.reshape(G.shape[:-1] + (k,))
    V = Vm.reshape((k,) + H.shape[1:])
    return Factors(U, s[:k], V)


# ------------------------------------------------------------------- swap ---
def _swap_operands(F: Factors, mu: int):
    """Ut = U sqrt(s), Vt = sqrt(s) V with the mu legs moved next to the core:
    Vt -> [k_A, f_perp..., j], Ut -> [j, b_perp..., k_B]."""
    d = F.d
    rs = np.sqrt(F.s)
    Ut = F.U * rs
    Vt = F.V * rs.reshape((-1,) + (1,) * d)
    Ut = np.moveaxis(Ut, mu, 0)            # [j, b_perp..., k]
    Vt = np.moveaxis(Vt, 1 + mu, -1)       # [k, f_perp..., j]
    return Ut, Vt


def swap_matrix(F: Factors, mu: int) -> np.ndarray:
    """The regrouped matrix M[(k_A, b^B_perp), (f^A_perp, k_B)] (dense; small
    problems only)."""
    Ut, Vt = _swap_operands(F, mu)
    k = F.s.shape[0]
    nperp = int(np.prod(Ut.shape[1:-1]))
    # [k_A, f_perp, j] x [j, b_perp, k_B] -> [k_A, f_perp, b_perp, k_B]
    M = np.tensordot(Vt, Ut, axes=([Vt.ndim - 1], [0]))
    M = M.reshape(k, nperp, nperp, k)
    M = M.transpose(0, 2, 1, 3).reshape(k * nperp, nperp * k)
    return M


def _apply(Ut, Vt, Z, transpose: bool):
    """M @ Z (or M^T @ Z) without forming M: Z has rows (f_perp, k_B) (or
    (k_A, b_perp)) and c columns."""
    k = Vt.shape[0]
    nperp = int(np.prod(Vt.shape[1:-1]))
    Um = Ut.reshape(Ut.shape[0], nperp, k)       # [j, b, kB]
    Vm = Vt.reshape(k, nperp, Vt.shape[-1])      # [kA, f, j]
    c = Z.shape[1]
    if not transpose:
        Zr = Z.reshape(nperp, k, c)              # [f, kB, c]
        t = np.einsum("afj,fbc->ajbc", Vm, Zr, optimize=True)      # [kA, j, kB, c]
        out = np.einsum("ajbc,jpb->apc", t, Um, optimize=True)     # [kA, b_perp, c]
        return out.reshape(k * nperp, c)
    Zr = Z.reshape(k, nperp, c)                  # [kA, b, c]
    t = np.einsum("jpb,apc->jbac", Um, Zr, optimize=True)          # [j, kB, kA, c]
    out = np.einsum("afj,jbac->fbc", Vm, t, optimize=True)         # [f_perp, kB, c]
    return out.reshape(nperp * k, c)


def rsvd_swap(F: Factors, mu: int, dcut: int, p: int, q: int, step: int, seed: int, dense: bool = False):
    """Truncated partial SVD of the swap matrix: X[(k_A, b_perp), l], sigma[l],
    Y[l, (f_perp, k_B)] with l < dcut.  ``dense`` uses a full SVD instead of
    the randomized one (a pin for small problems)."""
    Ut, Vt = _swap_operands(F, mu)
    k = F.s.shape[0]
    nperp = int(np.prod(Ut.shape[1:-1]))
    n = k * nperp
    if dense:
        M = swap_matrix(F, mu)
        X, sig, Y = np.linalg.svd(M, full_matrices=False)
        r = min(dcut, len(sig))
        return X[:, :r], sig[:r], Y[:r]
    r = min(dcut + p, n)
    Om = trial_matrix(n, r, step, seed)
    Q, _ = np.linalg.qr(_apply(Ut, Vt, Om, False))
    for _ in range(q):
        Z, _ = np.linalg.qr(_apply(Ut, Vt, Q, True))
        Q, _ = np.linalg.qr(_apply(Ut, Vt, Z, False))
    Bt = _apply(Ut, Vt, Q, True)                 # M^T Q = (Q^T M)^T, n x r
    Wb, sig, Zt = np.linalg.svd(Bt.T, full_matrices=False)
    keep = min(dcut, len(sig))
    return Q @ Wb[:, :keep], sig[:keep], Zt[:keep]


# ------------------------------------------------------------------ HOSVD ---
def _pieces(F: Factors, X, sig, Y, mu: int):
    """G[b^A (d legs), b^B_perp (d-1 legs), l] and H[l, f^A_perp, f^B (d legs)]."""
    d = F.d
    k = F.s.shape[0]
    rs = np.sqrt(F.s)
    dims = F.dims()
    perp = [dims[a] for a in range(d) if a != mu]
    r = sig.shape[0]
    Xs = (X * np.sqrt(sig)).reshape((k,) + tuple(perp) + (r,))
    Ys = (np.sqrt(sig)[:, None] * Y).reshape((r,) + tuple(perp) + (k,))
    Ut = F.U * rs
    Vt = F.V * rs.reshape((-1,) + (1,) * d)
    G = np.tensordot(Ut, Xs, axes=([d], [0]))          # [b^A..., b^B_perp..., l]
    H = np.tensordot(Ys, Vt, axes=([Ys.ndim - 1], [0]))  # [l, f^A_perp..., f^B...]
    return G, H


def grams(G: np.ndarray, H: np.ndarray, mu: int, d: int):
    """Gram matrices of the two-site tensor sum_l G[.., l] H[l, ..] (HOSVD of
    two adjacent decomposed tensors, Sec. 2, Fig. 2B), for every transverse
    axis nu in axis order: (backward, forward), each (d_nu^2) x (d_nu^2).

    Backward pair (b^A_nu, b^B_nu), legs of G: the other legs of G are summed
    directly, and H enters through its own Gram Wf[l, l'] = sum_f H[l, f]
    H[l', f].  Forward pair (f^A_nu, f^B_nu), legs of H: likewise with
    Wb[l, l'] = sum_b G[b, l] G[b, l'].  Both are exact regroupings of
    M M^T for the two-site tensor M with that pair as its row index."""
    perp = [a for a in range(d) if a != mu]
    # leg positions: G = [bA_0..bA_{d-1}, bB_perp..., l]; H = [l, fA_perp..., fB_0..fB_{d-1}]
    Wf = np.tensordot(H, H, axes=(list(range(1, H.ndim)), list(range(1, H.ndim))))   # [l, l']
    Wb = np.tensordot(G, G, axes=(list(range(G.ndim - 1)), list(range(G.ndim - 1))))  # [l, l']
    out = []
    L = string.ascii_letters
    for j, nu in enumerate(perp):
        dn = G.shape[nu]
        # backward pair: G legs nu (site A) and d + j (site B)
        sub1 = list(L[: G.ndim])
        sub2 = list(sub1)
        sub2[nu], sub2[d + j], sub2[-1] = "W", "X", "Y"
        gb = np.einsum("".join(sub1) + "," + "".join(sub2) + "," + sub1[-1] + "Y" + "->" +
                       sub1[nu] + sub1[d + j] + "WX", G, G, Wf, optimize=True)
        # forward pair: H legs 1 + j (site A) and 1 + (d - 1) + nu (site B)
        a_pos, b_pos = 1 + j, d + nu
        sub1 = list(L[: H.ndim])
        sub2 = list(sub1)
        sub2[a_pos], sub2[b_pos], sub2[0] = "W", "X", "Y"
        gf = np.einsum(sub1[0] + "Y" + "," + "".join(sub1) + "," + "".join(sub2) + "->" +
                       sub1[a_pos] + sub1[b_pos] + "WX", Wb, H, H, optimize=True)
        out.append((gb.reshape(dn * dn, dn * dn), gf.reshape(dn * dn, dn * dn)))
    return out


def isometries(G: np.ndarray, H: np.ndarray, mu: int, d: int, dcut: int):
    """HOSVD isometries P_nu from the Gram matrices of sum_l G H over the
    backward pair (b^A_nu, b^B_nu) (legs of G) and the forward pair (f^A_nu,
    f^B_nu) (legs of H); same selection rule as HOTRG."""
    perp = [a for a in range(d) if a != mu]
    out = []
    for nu, pair in zip(perp, grams(G, H, mu, d)):
        dn = G.shape[nu]
        n = dn * dn
        k = min(n, dcut)
        res = []
        for g in pair:
            w, v = hotrg._eig_desc(g)
            res.append((w, v, float(np.sum(np.maximum(w[k:], 0.0)))))
        eps_b, eps_f = res[0][2], res[1][2]
        side = hotrg.SIDE_BACKWARD if eps_b < (1.0 - hotrg.TIE_REL) * eps_f else hotrg.SIDE_FORWARD
        w, v, _ = res[side]
        P = hotrg._kept_vectors(w, v, k).reshape(dn, dn, k)
        out.append(hotrg.AxisChoice(nu, side, k, (eps_b, eps_f), w, False, P))
    return out


def contract(G: np.ndarray, H: np.ndarray, P: dict, mu: int, d: int):
    """G'[b_mu, B_perp..., l] and H'[l, F_perp..., f_mu] in the canonical leg
    order (axis order within the backward and the forward group)."""
    perp = [a for a in range(d) if a != mu]
    # G legs: bA_0..bA_{d-1}, bB_perp..., l; compress (bA_nu, bB_nu) -> B_nu
    L = string.ascii_letters
    gA = list(L[:d])
    gB = {nu: L[d + j] for j, nu in enumerate(perp)}
    gl = L[2 * d]
    outB = {nu: L[2 * d + 1 + j] for j, nu in enumerate(perp)}
    sub_G = "".join(gA) + "".join(gB[nu] for nu in perp) + gl
    ops = [G]
    subs = [sub_G]
    for nu in perp:
        ops.append(P[nu])
        subs.append(gA[nu] + gB[nu] + outB[nu])
    target = "".join(gA[a] if a == mu else outB[a] for a in range(d)) + gl
    Gn = np.einsum(",".join(subs) + "->" + target, *ops, optimize=True)
    # H legs: l, fA_perp..., fB_0..fB_{d-1}
    hl = L[0]
    hA = {nu: L[1 + j] for j, nu in enumerate(perp)}
    hB = list(L[d: 2 * d])
    outF = {nu: L[2 * d + j] for j, nu in enumerate(perp)}
    sub_H = hl + "".join(hA[nu] for nu in perp) + "".join(hB)
    ops = [H]
    subs = [sub_H]
    for nu in perp:
        ops.append(P[nu])
        subs.append(hA[nu] + hB[nu] + outF[nu])
    target = hl + "".join(hB[a] if a == mu else outF[a] for a in range(d))
    Hn = np.einsum(",".join(subs) + "->" + target, *ops, optimize=True)
    return Gn, Hn


# -------------------------------------------------------------------- Z2 ---
# The Ising tensor at h = 0 is invariant under the Z2 transformation that
# acts on every leg index with (-1)^index in the W basis (index 0 even, 1
# odd): its entries vanish unless the parities of all its legs add up to even.
# In the "z2" mode every decomposition of the ATRG step is done sector by
# sector, so the tensors stay exactly symmetric and the symmetric fixed point
# of the ordered phase (X -> 2) survives (Sec. 3.2 follows X with ATRG;
# reading: a trial matrix drawn across both sectors lets the randomized SVD
# mix them, and over tens of steps in the ordered phase the mixture grows
# until X -> 1).  Each leg index and each bond index carries a parity.


def composite_parity(pars) -> np.ndarray:
    """Parity of the row-major composite index of legs with the given
    per-leg parity arrays (outermost first)."""
    out = np.zeros(1, dtype=np.int64)
    for p in pars:
        out = ((out[:, None] + np.asarray(p, dtype=np.int64)[None, :]) % 2).reshape(-1)
    return out


def ising_factors_z2(beta: float, d: int):
    """ising_factors at h = 0 with the bond rotated to definite parity:
    u_e = (u_+ + u_-) / sqrt 2 (even |b|), u_o = (u_+ - u_-) / sqrt 2 (odd
    |b|); likewise v.  Returns the factors, the leg parities [0, 1] of every
    axis and the bond parities [0, 1]."""
    F = ising_factors(beta, 0.0, d)
    rot = np.array([[1.0, 1.0], [1.0, -1.0]]) / math.sqrt(2.0)
    U = np.tensordot(F.U, rot, axes=([d], [0]))             # [b..., k]: k = e, o
    V = np.tensordot(rot.T, F.V, axes=([1], [0]))           # [k, f...]
    legs = [np.array([0, 1]) for _ in range(d)]
    return Factors(U, np.ones(2), V), legs, np.array([0, 1])


def _sectors(par):
    return [np.nonzero(par == s)[0] for s in (0, 1)]


def _qr_sectors(Y, rpar, csec):
    """Orthonormal basis of the columns of Y, sector by sector (rows of
    parity s, columns of sector s); columns beyond a sector's rank are 0."""
    Q = np.zeros_like(Y)
    for rows, cols in zip(_sectors(rpar), _sectors(csec)):
        if len(rows) == 0 or len(cols) == 0:
            continue
        q, _ = np.linalg.qr(Y[np.ix_(rows, cols)])
        Q[np.ix_(rows, cols[:q.shape[1]])] = q
    return Q


def trial_sectors(r: int, room) -> np.ndarray:
    """Sector of each of the r trial columns: alternating (c mod 2) for the
    first 2 min(room) columns, then the sector with more room."""
    h = min(room)
    big = 0 if room[0] >= room[1] else 1
    return np.array([c % 2 if c < 2 * h else big for c in range(r)], dtype=np.int64)


def _merge(parts, keep):
    """parts: per sector (values descending, payload); returns the `keep`
    largest values across sectors (even sector first on equal values) as
    (value, sector, index in sector)."""
    allv = [(-float(v), s, i) for s, vals in enumerate(parts) for i, v in enumerate(vals)]
    allv.sort()
    return [(-v, s, i) for v, s, i in allv[:keep]]


def canonical_z2(G: np.ndarray, H: np.ndarray, dcut: int, legs, bond):
    """canonical() sector by sector: the parity-s rows of G and columns of
    H with the bonds of parity s; singular values of both sectors merged and
    the largest dcut kept.  Returns the factors and the kept bonds' parities."""
    d = G.ndim - 1
    r = G.shape[-1]
    Gm = G.reshape(-1, r)
    Hm = H.reshape(r, -1)
    rp = composite_parity(legs)
    res = []
    for rows, bonds in zip(_sectors(rp), _sectors(bond)):
        if len(rows) == 0 or len(bonds) == 0:
            res.append((np.zeros(0), None, None, rows))
            continue
        Qg, Rg = np.linalg.qr(Gm[np.ix_(rows, bonds)])
        Qh, Rh = np.linalg.qr(Hm[np.ix_(bonds, rows)].T)
        W, sv, Zt = np.linalg.svd(Rg @ Rh.T)
        res.append((sv, Qg @ W, Zt @ Qh.T, rows))
    nz = sum(int(np.count_nonzero(x[0] > 0)) for x in res)
    k = min(dcut, nz or 1, sum(len(x[0]) for x in res))
    kept = _merge([x[0] for x in res], k)
    Um = np.zeros((Gm.shape[0], k))
    Vm = np.zeros((k, Hm.shape[1]))
    sv = np.zeros(k)
    par = np.zeros(k, dtype=np.int64)
    for j, (v, sec, i) in enumerate(kept):
        _, Us, Vs, rows = res[sec]
        Um[rows, j] = Us[:, i]
        Vm[j, rows] = Vs[i]
        sv[j] = v
        par[j] = sec
    for j in range(k):
        col = np.abs(Um[:, j])
        i = int(np.nonzero(col >= (1.0 - 1e-9) * col.max())[0][0])
        if Um[i, j] < 0:
            Um[:, j] = -Um[:, j]
            Vm[j] = -Vm[j]
    return Factors(Um.reshape(G.shape[:-1] + (k,)), sv, Vm.reshape((k,) + H.shape[1:])), par


def rsvd_swap_z2(F: Factors, legs, bond, mu: int, dcut: int, p: int, q: int, step: int, seed: int):
    """rsvd_swap with the swap matrix's two parity sectors kept apart: the
    trial matrix keeps only the entries whose row parity (f_perp, k_B) equals
    the sector of its column, the QR factorisations and the final SVD are
    done per sector, and the largest dcut singular values of both sectors are
    kept.  Column c is in sector c mod 2 while both sectors have room for
    another column (a sector holds at most as many columns as the swap
    matrix has rows and columns of its parity); the remaining columns go to
    the larger sector.  Returns X, sigma, Y and the parities of the new
    bond."""
    d = F.d
    Ut, Vt = _swap_operands(F, mu)
    k = F.s.shape[0]
    perp = [a for a in range(d) if a != mu]
    nperp = int(np.prod(Ut.shape[1:-1]))
    n = k * nperp
    rpar = composite_parity([bond] + [legs[a] for a in perp])
    cpar = composite_parity([legs[a] for a in perp] + [bond])
    room = [min(int(np.sum(rpar == s)), int(np.sum(cpar == s))) for s in (0, 1)]
    r = min(dcut + p, room[0] + room[1])
    csec = trial_sectors(r, room)
    Om = trial_matrix(n, r, step, seed) * (cpar[:, None] == csec[None, :])
    Q = _qr_sectors(_apply(Ut, Vt, Om, False), rpar, csec)
    for _ in range(q):
        Z = _qr_sectors(_apply(Ut, Vt, Q, True), cpar, csec)
        Q = _qr_sectors(_apply(Ut, Vt, Z, False), rpar, csec)
    Bt = _apply(Ut, Vt, Q, True)                 # M^T Q, rows (f_perp, k_B)
    res = []
    for crows, cols in zip(_sectors(cpar), _sectors(csec)):
        if len(crows) == 0 or len(cols) == 0:
            res.append((np.zeros(0), None, None, crows, cols))
            continue
        Wb, sig, Zt = np.linalg.svd(Bt[np.ix_(crows, cols)].T, full_matrices=False)
        res.append((sig, Wb, Zt, crows, cols))
    keep = min(dcut, sum(len(x[0]) for x in res))
    kept = _merge([x[0] for x in res], keep)
    X = np.zeros((n, keep))
    Y = np.zeros((keep, n))
    sig = np.zeros(keep)
    par = np.zeros(keep, dtype=np.int64)
    for j, (v, sec, i) in enumerate(kept):
        _, Wb, Zt, crows, cols = res[sec]
        X[:, j] = Q[:, cols] @ Wb[:, i]
        Y[j, crows] = Zt[i]
        sig[j] = v
        par[j] = sec
    return X, sig, Y, par


def isometries_z2(G: np.ndarray, H: np.ndarray, mu: int, d: int, dcut: int, legs):
    """isometries() with each Gram's two pair-parity sectors diagonalised
    apart and their spectra merged; returns the choices and the parities of
    the new legs (those of the kept isometry columns)."""
    perp = [a for a in range(d) if a != mu]
    out, new_legs = [], {}
    for nu, pair in zip(perp, grams(G, H, mu, d)):
        dn = G.shape[nu]
        n = dn * dn
        k = min(n, dcut)
        pp = composite_parity([legs[nu], legs[nu]])
        res = []
        for g in pair:
            g = 0.5 * (g + g.T)
            vals, vecs = [], []
            for rows in _sectors(pp):
                if len(rows) == 0:
                    vals.append(np.zeros(0))
                    vecs.append(None)
                    continue
                w, v = np.linalg.eigh(g[np.ix_(rows, rows)])
                order = np.argsort(-w, kind="stable")
                vals.append(w[order])
                vecs.append((rows, v[:, order]))
            merged = _merge(vals, n)
            w = np.array([x[0] for x in merged])
            V = np.zeros((n, n))
            for j, (_, sec, i) in enumerate(merged):
                rows, v = vecs[sec]
                V[rows, j] = v[:, i]
            res.append((w, V, float(np.sum(np.maximum(w[k:], 0.0)))))
        eps_b, eps_f = res[0][2], res[1][2]
        side = hotrg.SIDE_BACKWARD if eps_b < (1.0 - hotrg.TIE_REL) * eps_f else hotrg.SIDE_FORWARD
        w, V, _ = res[side]
        Pm = hotrg._kept_vectors(w, V, k)
        new_legs[nu] = np.array([int(np.sum(Pm[pp == 1, j] ** 2) > np.sum(Pm[pp == 0, j] ** 2))
                                 for j in range(k)])
        out.append(hotrg.AxisChoice(nu, side, k, (eps_b, eps_f), w, False, Pm.reshape(dn, dn, k)))
    return out, new_legs


# ------------------------------------------------------------- step / run ---
@dataclass
class AtrgStep:
    n: int
    mu: int
    ln_c: float
    swap_sigma: np.ndarray
    local_s: np.ndarray
    axes: list = field(default_factory=list)
    legs: list = None       # Z2 mode: leg parities after the step (per axis)
    bond: np.ndarray = None  # Z2 mode: bond parities after the step


def middle_svd(A: np.ndarray, B: np.ndarray, dcut: int, p: int, q: int, step: int, seed: int, stream: int,
               dense: bool = False):
    """Rank-dcut partial SVD of M[(a, b), (f, c)] = sum_j A[a, f, j] B[j, b, c]
    (A: [ra, nperp, dmu], B: [dmu, nperp, cb]) by the randomized SVD of the
    pure swap (trial matrix of the given stream), or densely."""
    ra, nperp, dmu = A.shape
    cb = B.shape[2]
    nr, nc = ra * nperp, nperp * cb

    def mz(Z):          # M Z, Z rows (f, c)
        t = np.einsum("afj,fcx->ajcx", A, Z.reshape(nperp, cb, -1), optimize=True)
        return np.einsum("ajcx,jbc->abx", t, B, optimize=True).reshape(nr, -1)

    def mtq(Q):         # M^T Q, Q rows (a, b)
        t = np.einsum("jbc,abx->jcax", B, Q.reshape(ra, nperp, -1), optimize=True)
        return np.einsum("afj,jcax->fcx", A, t, optimize=True).reshape(nc, -1)

    if dense:
        M = np.einsum("afj,jbc->abfc", A, B).reshape(nr, nc)
        X, sig, Y = np.linalg.svd(M, full_matrices=False)
        r = min(dcut, len(sig))
        return X[:, :r], sig[:r], Y[:r]
    r = min(dcut + p, nr, nc)
    Q, _ = np.linalg.qr(mz(trial_matrix(nc, r, step, seed, stream)))
    for _ in range(q):
        Z, _ = np.linalg.qr(mtq(Q))
        Q, _ = np.linalg.qr(mz(Z))
    Wb, sig, Zt = np.linalg.svd(mtq(Q).T, full_matrices=False)
    keep = min(dcut, len(sig))
    return Q @ Wb[:, :keep], sig[:keep], Zt[:keep]


def impurity_pieces_step(F: Factors, mu: int, GS: np.ndarray, HS: np.ndarray, kind: int, dcut: int, p: int,
                         q: int, step: int, seed: int, dense: bool = False):
    """The impurity's two-site pieces before the isometries: backward
    [b^A..., b^B_perp..., m'] and forward [m', f^A_perp..., f^B...], m' =
    (lower-site term, upper-site term)."""
    d = F.d
    k = F.s.shape[0]
    rs = np.sqrt(F.s)
    dims = F.dims()
    perp = tuple(dims[a] for a in range(d) if a != mu)
    nperp = int(np.prod(perp))
    dmu = dims[mu]
    m = GS.shape[-1]
    Ut = F.U * rs                                           # [b..., k]
    Vt = F.V * rs.reshape((-1,) + (1,) * d)                 # [k, f...]
    Utp = np.moveaxis(Ut, mu, 0).reshape(dmu, nperp, k)     # [j, b_perp, kB]
    Vtp = np.moveaxis(Vt, 1 + mu, -1).reshape(k, nperp, dmu)  # [kA, f_perp, j]
    # lower site: M_1 = H_S (x)_j Ut
    HSp = np.moveaxis(HS, 1 + mu, -1).reshape(m, nperp, dmu)
    X1, s1, Y1 = middle_svd(HSp, Utp, dcut, p, q, step, seed, 1 + 2 * kind, dense)
    r1 = len(s1)
    X1s = (X1 * np.sqrt(s1)).reshape((m,) + perp + (r1,))
    Y1s = (np.sqrt(s1)[:, None] * Y1).reshape((r1,) + perp + (k,))
    G1 = np.tensordot(GS, X1s, axes=([d], [0]))
    H1 = np.tensordot(Y1s, Vt, axes=([d], [0]))
    # upper site: M_2 = Vt (x)_j G_S
    GSp = np.moveaxis(GS, mu, 0).reshape(dmu, nperp, m)
    X2, s2, Y2 = middle_svd(Vtp, GSp, dcut, p, q, step, seed, 2 + 2 * kind, dense)
    r2 = len(s2)
    X2s = (X2 * np.sqrt(s2)).reshape((k,) + perp + (r2,))
    Y2s = (np.sqrt(s2)[:, None] * Y2).reshape((r2,) + perp + (m,))
    G2 = np.tensordot(Ut, X2s, axes=([d], [0]))
    H2 = np.tensordot(Y2s, HS, axes=([d], [0]))
    return np.concatenate([G1, G2], axis=-1), 0.5 * np.concatenate([H1, H2], axis=0)


def atrg_step(F: Factors, mu: int, dcut: int, p: int, q: int, step: int, seed: int, dense_swap=False,
              imps=None):
    """One ATRG step along mu on canonical factors F.  Returns the new pieces
    (G', H') normalised, c, and the step record; given a list of impurity
    piece pairs ``imps`` (G_S, H_S) the return has a fifth entry, their new
    pairs."""
    with_imps = imps is not None
    imps = imps or []
    d = F.d
    X, sig, Y = rsvd_swap(F, mu, dcut, p, q, step, seed, dense=dense_swap)
    G, H = _pieces(F, X, sig, Y, mu)
    choices = isometries(G, H, mu, d, dcut)
    P = {ch.nu: ch.U for ch in choices}
    Gn, Hn = contract(G, H, P, mu, d)
    r = Gn.shape[-1]
    GtG = Gn.reshape(-1, r).T @ Gn.reshape(-1, r)
    HHt = Hn.reshape(r, -1) @ Hn.reshape(r, -1).T
    c = math.sqrt(float(np.sum(GtG * HHt)))
    rec = AtrgStep(step, mu, math.log(c), sig, F.s, choices)
    new_imps = []
    for kind, (GS, HS) in enumerate(imps):
        Gc, Hc = impurity_pieces_step(F, mu, GS, HS, kind, dcut, p, q, step, seed, dense_swap)
        GSn, HSn = contract(Gc, Hc, P, mu, d)
        new_imps.append((GSn / math.sqrt(c), HSn / math.sqrt(c)))
    Gn = Gn / math.sqrt(c)
    Hn = Hn / math.sqrt(c)
    if not with_imps:
        return Gn, Hn, c, rec
    return Gn, Hn, c, rec, new_imps


def atrg_step_z2(F: Factors, bond, legs, mu: int, dcut: int, p: int, q: int, step: int, seed: int, imps=None):
    """atrg_step for the symmetric (h = 0) tensor with the swap and the HOSVD
    done sector by sector.  `bond` and `legs` are the parities of F's bond
    and of its legs; returns G', H' normalised, c, the record, the impurity
    pairs (plain randomized SVDs: they do not feed back into the pure
    tensor), the new legs' parities and the new bond's."""
    d = F.d
    X, sig, Y, lpar = rsvd_swap_z2(F, legs, bond, mu, dcut, p, q, step, seed)
    G, H = _pieces(F, X, sig, Y, mu)
    choices, new = isometries_z2(G, H, mu, d, dcut, legs)
    P = {ch.nu: ch.U for ch in choices}
    Gn, Hn = contract(G, H, P, mu, d)
    r = Gn.shape[-1]
    GtG = Gn.reshape(-1, r).T @ Gn.reshape(-1, r)
    HHt = Hn.reshape(r, -1) @ Hn.reshape(r, -1).T
    c = math.sqrt(float(np.sum(GtG * HHt)))
    rec = AtrgStep(step, mu, math.log(c), sig, F.s, choices)
    new_imps = []
    for kind, (GS, HS) in enumerate(imps or []):
        Gc, Hc = impurity_pieces_step(F, mu, GS, HS, kind, dcut, p, q, step, seed)
        GSn, HSn = contract(Gc, Hc, P, mu, d)
        new_imps.append((GSn / math.sqrt(c), HSn / math.sqrt(c)))
    legs = [new.get(a, legs[a]) for a in range(d)]
    return Gn / math.sqrt(c), Hn / math.sqrt(c), c, rec, new_imps, legs, lpar


def periodic_trace(G: np.ndarray, H: np.ndarray) -> float:
    """Tr T for T = sum_l G[b..., l] H[l, f...] with each f_nu joined to b_nu."""
    r = G.shape[-1]
    return float(np.sum(G.reshape(-1, r) * H.reshape(r, -1).T))


@dataclass
class AtrgResult:
    ln_z_per_site: float
    acc: float
    trace: float
    steps: list
    energy: float = float("nan")
    magnetization: float = float("nan")
    G: np.ndarray = None
    H: np.ndarray = None


def dense_tensor(G: np.ndarray, H: np.ndarray) -> np.ndarray:
    """sum_l G[b..., l] H[l, f...] with the legs interleaved per axis
    (b_0, f_0, b_1, f_1, ...), the layout of the HOTRG tensors."""
    d = G.ndim - 1
    T = np.tensordot(G, H, axes=([d], [0]))
    return np.transpose(T, [x for a in range(d) for x in (a, d + a)])


def indicator_x(G: np.ndarray, H: np.ndarray, axis: int = 0) -> float:
    """The degeneracy indicator X (Sec. 3.1, defined as for HOTRG) of the
    factored tensor, evaluated on its dense form."""
    return hotrg.indicator_x(dense_tensor(G, H), axis)


def run(beta: float, h: float, d: int, dcut: int, L: int, p=None, q=None, seed: int = 0,
        dense_swap: bool = False, impure: bool = False, z2: bool = False) -> AtrgResult:
    """ATRG on the periodic L^d lattice: d*m steps along (n-1) mod d.  With
    ``impure`` (beta > 0) also E = -Tr S_E / Tr T and M = Tr S_M / Tr T.
    ``z2`` (h = 0 only) keeps the pure tensor exactly Z2 symmetric."""
    m = int(round(math.log2(L)))
    if 2 ** m != L or m < 1:
        raise ValueError("L must be a power of two >= 2")
    if z2 and (h != 0.0 or dense_swap):
        raise ValueError("the Z2 mode needs h = 0 and the randomized swap")
    p = 4 * dcut if p is None else p
    q = 2 * dcut if q is None else q
    if z2:
        F0, legs, bond = ising_factors_z2(beta, d)
    else:
        F0 = ising_factors(beta, h, d)
    G, H = F0.U * 1.0, F0.V * 1.0
    r = G.shape[-1]
    c0 = math.sqrt(float(np.sum((G.reshape(-1, r).T @ G.reshape(-1, r)) * (H.reshape(r, -1) @ H.reshape(r, -1).T))))
    G, H = G / math.sqrt(c0), H / math.sqrt(c0)
    imps = None
    if impure:
        pieces = ising_impurity_pieces(beta, h, d)
        if z2:   # the impurity's bond rotated like the pure one
            rot = np.array([[1.0, 1.0], [1.0, -1.0]]) / math.sqrt(2.0)
            pieces = [np.tensordot(rot.T, x, axes=([1], [0])) for x in pieces]
        imps = [(G.copy(), x / math.sqrt(c0)) for x in pieces]
    acc = math.log(c0)
    steps = []
    for n in range(1, d * m + 1):
        mu = (n - 1) % d
        if z2:
            F, kpar = canonical_z2(G, H, dcut, legs, bond)
            G, H, c, rec, imps2, legs, bond = atrg_step_z2(F, kpar, legs, mu, dcut, p, q, n, seed, imps)
            imps = imps2 if impure else None
            rec.legs, rec.bond = [x.copy() for x in legs], bond.copy()
        else:
            F = canonical(G, H, dcut)
            if impure:
                G, H, c, rec, imps = atrg_step(F, mu, dcut, p, q, n, seed, dense_swap, imps=imps)
            else:
                G, H, c, rec = atrg_step(F, mu, dcut, p, q, n, seed, dense_swap)
        acc += 2.0 ** (-n) * math.log(c)
        steps.append(rec)
    tr = periodic_trace(G, H)
    res = AtrgResult(acc + 2.0 ** (-(d * m)) * math.log(tr), acc, tr, steps, G=G, H=H)
    if impure:
        res.energy = -periodic_trace(*imps[0]) / tr
        res.magnetization = periodic_trace(*imps[1]) / tr
    return res
