"""Pins of the ATRG oracle: the counter-based generator against its published
known answers, exactness against brute-force spin sums when nothing is
truncated, RSVD against a dense SVD, the p,q-independence the paper reports,
and Onsager's solution on a large 2D lattice."""
import json
import math
import os
import warnings

import numpy as np
import pytest

from oracle import atrg, exact

warnings.filterwarnings("ignore", message=".*roundoff error.*")


@pytest.mark.parametrize("ctr,key,expect", [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
])
def test_philox_known_answers(ctr, key, expect):
    """Known-answer vectors of Philox4x32-10 published with the generator."""
    assert tuple(atrg.philox4x32_10(ctr, key)) == expect


def test_philox_vectorised_equals_scalar():
    c0 = np.array([0, 5, 123456789, 0xFFFFFFFF])
    c1 = np.array([0, 7, 3, 1])
    w0, w1 = atrg.philox4x32_10_vec(c0, c1, (0xDEADBEEF, 42))
    for i in range(4):
        s = atrg.philox4x32_10((int(c0[i]), int(c1[i]), 0, 0), (0xDEADBEEF, 42))
        assert (int(w0[i]), int(w1[i])) == (s[0], s[1])


def test_trial_matrix_is_standard_normal():
    Om = atrg.trial_matrix(400, 250, 3, 99)
    assert abs(Om.mean()) < 0.01 and abs(Om.std() - 1.0) < 0.01
    assert np.array_equal(Om, atrg.trial_matrix(400, 250, 3, 99))
    assert not np.array_equal(Om, atrg.trial_matrix(400, 250, 4, 99))


def test_ising_factors_are_exact():
    from oracle import ising
    for d in (2, 4):
        F = atrg.ising_factors(0.3, 0.1, d)
        T0 = ising.site_tensors(0.3, 0.1, d)[0]
        # factor legs (b..., f...) -> canonical interleaved (b0, f0, b1, f1, ...)
        dense = F.dense()
        order = [x for a in range(d) for x in (a, d + a)]
        assert np.allclose(np.transpose(dense, order), T0, atol=1e-14)


@pytest.mark.parametrize("beta,h", [(0.4407, 0.0), (0.3, 0.1)])
@pytest.mark.parametrize("dense", [True, False])
def test_2d_L4_untruncated_equals_brute_force(beta, h, dense):
    r = atrg.run(beta, h, 2, 128, 4, p=8, q=2, dense_swap=dense)
    assert abs(r.ln_z_per_site - exact.brute_force(beta, h, 2, 4)[0]) < 1e-12


def test_3d_L2_untruncated_equals_brute_force():
    r = atrg.run(0.25, 0.05, 3, 1024, 2, dense_swap=True)
    assert abs(r.ln_z_per_site - exact.brute_force(0.25, 0.05, 3, 2)[0]) < 1e-12


def test_4d_two_steps_then_exact_equals_brute_force():
    """Two untruncated ATRG steps on the 2^4 lattice, then the coarse-grained
    legs closed and the periodic 2x2 network of the other two axes contracted
    exactly (as for HOTRG)."""
    beta, h = 0.2, 0.1
    F0 = atrg.ising_factors(beta, h, 4)
    G, H = F0.U, F0.V
    r = G.shape[-1]
    c0 = math.sqrt(float(np.sum((G.reshape(-1, r).T @ G.reshape(-1, r)) * (H.reshape(r, -1) @ H.reshape(r, -1).T))))
    G, H = G / math.sqrt(c0), H / math.sqrt(c0)
    lnz = math.log(c0)
    for n, mu in ((1, 0), (2, 1)):
        F = atrg.canonical(G, H, 4096)
        G, H, c, _ = atrg.atrg_step(F, mu, 4096, 0, 0, n, 0, dense_swap=True)
        lnz += 2.0 ** -n * math.log(c)
    T = np.tensordot(G, H, axes=([4], [0]))  # [b0..b3, f0..f3]
    Q = np.einsum("abcdabef->cdef", T)       # close x, y: Q[z, t, z', t']
    Q = Q.transpose(0, 2, 1, 3)              # -> [z, z', t, t']
    net = lambda A, B, C, D: np.einsum("abcd,baef,ghdc,hgfe->", A, B, C, D, optimize=True)
    lnz += math.log(net(Q, Q, Q, Q)) / 16
    assert abs(lnz - exact.brute_force(beta, h, 4, 2)[0]) < 1e-12


@pytest.mark.parametrize("dcut", [4, 6])
def test_rsvd_equals_dense_svd_and_pq_independence(dcut):
    a = atrg.run(0.1497, 0.0, 4, dcut, 4)                         # p = 4 Dcut, q = 2 Dcut
    b = atrg.run(0.1497, 0.0, 4, dcut, 4, dense_swap=True)
    c = atrg.run(0.1497, 0.0, 4, dcut, 4, p=2 * dcut, q=dcut)      # p = 2 Dcut, q = Dcut
    assert abs(a.ln_z_per_site - b.ln_z_per_site) < 1e-12
    assert abs(c.ln_z_per_site - a.ln_z_per_site) < 1e-6


def test_beta_zero_and_field_symmetry():
    assert abs(atrg.run(0.0, 0.2, 4, 4, 4).ln_z_per_site - math.log(2.0)) < 1e-14
    a = atrg.run(0.1497, 1e-3, 4, 4, 4)
    b = atrg.run(0.1497, -1e-3, 4, 4, 4)
    assert abs(a.ln_z_per_site - b.ln_z_per_site) < 1e-12


def test_2d_large_lattice_approaches_onsager():
    r = atrg.run(0.2, 0.0, 2, 16, 2 ** 20)
    assert abs(r.ln_z_per_site - exact.onsager_lnz(0.2)) < 1e-7


# ------------------------------------------------------------ impure tensors ---
def test_impurity_pieces_reproduce_the_site_sums():
    """S_M = sum_s s (...) exactly; the forward-carried energy impurity has
    every bond derivative on the forward end: with each forward leg closed
    on its own bond partner it sums the bond energies of the site."""
    from oracle import ising
    beta, h, d = 0.3, 0.1, 2
    F = atrg.ising_factors(beta, h, d)
    HE, HM = atrg.ising_impurity_pieces(beta, h, d)
    order = [x for a in range(d) for x in (a, d + a)]
    SM = np.transpose(np.tensordot(F.U, HM, axes=([d], [0])), order)
    assert np.allclose(SM, ising.site_tensors(beta, h, d)[1], atol=1e-14)
    # one site with a closed loop on every axis: T[b, f] with b_nu = f_nu is
    # the single-site periodic lattice, sum_s e^{beta h s} prod_nu e^{beta}
    SE = np.tensordot(F.U, HE, axes=([d], [0]))
    T = F.dense()
    idx = np.arange(2)
    tr = lambda X: float(sum(X[i, j, i, j] for i in idx for j in idx))
    z = 2.0 * math.cosh(beta * h) * math.exp(d * beta)
    assert abs(tr(T) - z) < 1e-12 * z
    # d/dbeta of the same sum: the bonds give d e^{d beta} / dbeta, the field h
    dz = 2.0 * math.exp(d * beta) * (d * math.cosh(beta * h) + h * math.sinh(beta * h))
    assert abs(tr(SE) - dz) < 1e-12 * dz


@pytest.mark.parametrize("beta,h,d,L", [(0.3, 0.05, 2, 4), (0.4407, 0.0, 2, 4), (0.2, -0.1, 2, 4),
                                        (0.25, 0.05, 3, 2)])
def test_impure_untruncated_equals_brute_force(beta, h, d, L):
    """Nothing truncated (dense SVDs): E and M of the impurity pieces equal
    the spin sums."""
    r = atrg.run(beta, h, d, 4096, L, dense_swap=True, impure=True)
    lnz, E, M = exact.brute_force(beta, h, d, L)
    assert abs(r.ln_z_per_site - lnz) < 1e-12
    assert abs(r.energy - E) < 1e-12 * abs(E)
    assert abs(r.magnetization - M) < 1e-12 * max(abs(M), 1.0)


def test_impure_randomized_untruncated_equals_brute_force():
    """The randomized partial SVDs (small p, q) with rank covering the whole
    space are exact too."""
    r = atrg.run(0.3, 0.05, 2, 64, 4, p=8, q=1, impure=True)
    lnz, E, M = exact.brute_force(0.3, 0.05, 2, 4)
    assert abs(r.energy - E) < 1e-11 * abs(E) and abs(r.magnetization - M) < 1e-11 * abs(M)


def test_impurities_leave_the_pure_run_unchanged():
    a = atrg.run(0.3, 0.05, 2, 8, 16, p=8, q=2)
    b = atrg.run(0.3, 0.05, 2, 8, 16, p=8, q=2, impure=True)
    assert a.ln_z_per_site == b.ln_z_per_site


def test_impure_truncated_2d_energy_near_onsager():
    """2D, K = 0.3 (disordered side), Dcut = 8, L = 2^10: E within 1e-2 of
    Onsager's energy, M = 0 by symmetry at h = 0."""
    K = 0.3
    r = atrg.run(K, 0.0, 2, 8, 2 ** 10, p=16, q=4, impure=True)
    assert abs(r.energy - exact.onsager_energy(K)) < 1e-2 * abs(exact.onsager_energy(K))
    assert abs(r.magnetization) < 1e-10


# ------------------------------------------------------------- indicator X ---
def test_indicator_on_pieces_equals_dense_definition():
    """The factored form's X is the HOTRG definition on the dense tensor; at
    the start it is the single-site value computed by hand."""
    from oracle import hotrg
    F = atrg.ising_factors(0.3, 0.0, 2)
    T = atrg.dense_tensor(F.U, F.V)
    assert atrg.indicator_x(F.U, F.V, 0) == hotrg.indicator_x(T, 0)
    # M[a][a'] = sum_y T[a, a', y, y]; X = (Tr M)^2 / Tr(M M)
    M = np.einsum("abyy->ab", T)
    assert abs(atrg.indicator_x(F.U, F.V, 0) - np.trace(M) ** 2 / np.trace(M @ M)) < 1e-14


@pytest.mark.parametrize("K,expect", [(1.0, 2.0), (0.1, 1.0)])
def test_indicator_phases_2d(K, expect):
    """Deep in the ordered phase X -> 2 (two degenerate fixed-point
    components), deep in the disordered phase X -> 1."""
    r = atrg.run(K, 0.0, 2, 8, 2 ** 8, p=16, q=4)
    assert abs(atrg.indicator_x(r.G, r.H, 0) - expect) < 1e-6


def _explicit_two_site_gram(G, H, mu, d, j, nu, side):
    """Gram of one leg pair of the dense two-site tensor M = sum_l G H, built
    by one plain einsum and a reshape (no regrouping): M has the legs
    (bA_0..bA_{d-1}, bB_perp..., fA_perp..., fB_0..fB_{d-1})."""
    M = np.tensordot(G, H, axes=([G.ndim - 1], [0]))
    if side == 0:
        pos = (nu, d + j)                          # bA_nu, bB_nu
    else:
        pos = (2 * d - 1 + j, 3 * d - 2 + nu)      # fA_nu, fB_nu
    Mm = np.moveaxis(M, pos, (0, 1))
    n = Mm.shape[0] * Mm.shape[1]
    Mm = Mm.reshape(n, -1)
    return Mm @ Mm.T


@pytest.mark.parametrize("d,dims,mu,r", [(2, (3, 2), 0, 3), (2, (2, 3), 1, 4), (3, (2, 3, 2), 1, 3),
                                         (3, (3, 2, 2), 0, 2), (4, (2, 3, 2, 2), 2, 3), (4, (2, 2, 3, 2), 0, 2)])
def test_hosvd_grams_equal_explicit_two_site_gram(d, dims, mu, r):
    """HOSVD of two adjacent decomposed tensors (Sec. 2, Fig. 2B): the
    factored Grams of both leg pairs equal M M^T of the explicit two-site
    tensor, and the selected isometry spans the leading eigenvectors of the
    explicit Gram (with the truncation error computed from it)."""
    rng = np.random.default_rng(17 + d)
    perp = [a for a in range(d) if a != mu]
    G = rng.standard_normal(tuple(dims) + tuple(dims[a] for a in perp) + (r,))
    H = rng.standard_normal((r,) + tuple(dims[a] for a in perp) + tuple(dims))
    got = atrg.grams(G, H, mu, d)
    dcut = 3
    choices = atrg.isometries(G, H, mu, d, dcut)
    for j, nu in enumerate(perp):
        ref = [_explicit_two_site_gram(G, H, mu, d, j, nu, s) for s in (0, 1)]
        for s in (0, 1):
            assert np.allclose(got[j][s], ref[s], rtol=0, atol=1e-12 * np.abs(ref[s]).max())
        ch = choices[j]
        n = dims[nu] ** 2
        k = min(n, dcut)
        spectra = [np.sort(np.linalg.eigvalsh(g))[::-1] for g in ref]
        for s in (0, 1):
            assert abs(ch.eps[s] - np.sum(np.maximum(spectra[s][k:], 0.0))) <= 1e-10 * spectra[s][0]
        w, v = np.linalg.eigh(ref[ch.side])
        lead = v[:, np.argsort(-w)[:k]]
        w_sorted = np.sort(w)[::-1]
        assert k == n or w_sorted[k - 1] - w_sorted[k] > 1e-6 * w_sorted[0]
        U = ch.U.reshape(n, k)
        assert np.allclose(U @ U.T, lead @ lead.T, atol=1e-10)


@pytest.mark.parametrize("d,L,beta", [(2, 4, 0.3), (2, 4, 0.6), (3, 2, 0.25)])
def test_z2_mode_untruncated_equals_brute_force(d, L, beta):
    """The sector-by-sector ATRG of the symmetric (h = 0) tensor is exact
    when nothing is truncated."""
    r = atrg.run(beta, 0.0, d, 128, L, p=8, q=2, z2=True)
    assert abs(r.ln_z_per_site - exact.brute_force(beta, 0.0, d, L)[0]) < 1e-12


def test_z2_mode_keeps_the_symmetric_fixed_point_in_4d():
    """4D, beta = 0.2 (deep in the ordered phase), h = 0, L = 1024, Dcut 6:
    with the sectors kept apart the pure tensor stays exactly symmetric, so
    M = 0 and the degeneracy indicator X = 2 (Sec. 3.1-3.2); the plain
    randomized swap has already broken the symmetry at this bond dimension
    (M ~ 3e-4, X below 2), while f agrees."""
    z = atrg.run(0.2, 0.0, 4, 6, 1024, z2=True, impure=True)
    plain = atrg.run(0.2, 0.0, 4, 6, 1024, impure=True)
    assert abs(z.magnetization) < 1e-12
    assert abs(atrg.indicator_x(z.G, z.H, 0) - 2.0) < 1e-10
    assert abs(plain.magnetization) > 1e-6
    assert abs(z.ln_z_per_site - plain.ln_z_per_site) < 1e-10 * abs(plain.ln_z_per_site)
    # the stored values of this run (tests/golden) are still the oracle's
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")) as f:
        c = json.load(f)["cases"]["atrg_z2_4d_dcut6_L1024_b0.2"]
    assert (c["beta"], c["h"], c["d"], c["dcut"], c["L"], c["seed"], c["z2"]) == (0.2, 0.0, 4, 6, 1024, 0, True)
    assert z.ln_z_per_site == pytest.approx(float(c["ln_z_per_site"]), rel=1e-12, abs=0)
    assert z.energy == pytest.approx(float(c["energy"]), rel=1e-10, abs=0)
    assert abs(float(c["magnetization"])) < 1e-12


def test_z2_mode_disordered_phase_gives_x_one():
    """4D, beta = 0.12 (disordered), h = 0: X -> 1 in the Z2 mode too."""
    z = atrg.run(0.12, 0.0, 4, 4, 1024, z2=True)
    assert abs(atrg.indicator_x(z.G, z.H, 0) - 1.0) < 1e-6


def test_trial_sectors_alternate_then_fill_the_larger_sector():
    assert list(atrg.trial_sectors(6, (8, 8))) == [0, 1, 0, 1, 0, 1]
    s = atrg.trial_sectors(13, (3, 10))
    assert list(s[:6]) == [0, 1, 0, 1, 0, 1] and set(s[6:]) == {1}
    assert int(np.sum(s == 0)) == 3 and int(np.sum(s == 1)) == 10


def _symmetric_factors(dims, legs, bond, seed):
    """Random pieces G[b..., l], H[l, f...] that vanish unless the parity of
    the legs equals that of the bond index."""
    rng = np.random.default_rng(seed)
    rp = atrg.composite_parity(legs)
    bond = np.asarray(bond)
    n = int(np.prod(dims))
    G = rng.standard_normal((n, len(bond))) * (rp[:, None] == bond[None, :])
    H = rng.standard_normal((len(bond), n)) * (bond[:, None] == rp[None, :])
    return G.reshape(tuple(dims) + (len(bond),)), H.reshape((len(bond),) + tuple(dims))


@pytest.mark.parametrize("mu", [0, 1, 2])
def test_z2_swap_with_unbalanced_sectors_equals_dense_svd(mu):
    """Unbalanced leg parities: one parity sector of the swap matrix has
    fewer rows than half the trial columns.  With every column kept (rank
    = matrix order) the sector-by-sector randomized swap reproduces the
    dense SVD of the swap matrix: its singular values, and X sigma Y = M."""
    legs = [np.array([0, 0, 1]), np.array([0, 0]), np.array([0, 0, 0, 1])]
    bond = np.array([0, 0, 0, 1])
    G, H = _symmetric_factors([3, 2, 4], legs, bond, seed=5 + mu)
    F, kpar = atrg.canonical_z2(G, H, 8, legs, bond)
    perp = [a for a in range(3) if a != mu]
    rpar = atrg.composite_parity([kpar] + [legs[a] for a in perp])
    n = len(rpar)
    assert min(np.sum(rpar == 0), np.sum(rpar == 1)) < n // 2    # alternation alone would overfill
    M = atrg.swap_matrix(F, mu)
    X, sig, Y, par = atrg.rsvd_swap_z2(F, legs, kpar, mu, n, 0, 2, 1, 7)
    ref = np.linalg.svd(M, compute_uv=False)
    assert np.max(np.abs(np.sort(sig)[::-1] - ref[:len(sig)])) < 1e-12 * ref[0]
    assert np.max(np.abs((X * sig) @ Y - M)) < 1e-12 * ref[0]
    # each kept vector lies in the sector its parity names
    assert np.all(np.abs(X[rpar[:, None] != par[None, :]]) == 0.0)
