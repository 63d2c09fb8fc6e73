"""GPU kernels against plain references: the join GEMM in its four
precisions and the Jacobi eigensolver."""
import numpy as np
import pytest

from tests.gpu_util import announce, need_gpu
from trg_inputs import random_matrix, random_symmetric, gram_like

pytestmark = pytest.mark.gpu


def _pad(x, r, c):
    out = np.zeros((r, c), dtype=x.dtype)
    out[: x.shape[0], : x.shape[1]] = x
    return out


@pytest.mark.parametrize("M,N,K", [(128, 128, 16), (256, 384, 160), (1024, 512, 1040), (128, 1280, 4096)])
@pytest.mark.parametrize("accumulate", [False, True])
def test_gemm_fp64(M, N, K, accumulate):
    torch = need_gpu()
    from paper_1911_12954_amd import trg_gemm
    announce("gemm fp64", M, N, K, accumulate)
    A = random_matrix(M, K, 1)
    B = random_matrix(N, K, 2)
    C0 = random_matrix(M, N, 3)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    dC = torch.from_numpy(C0).cuda()
    trg_gemm("fp64", dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), M, N, K, K, K, N, accumulate,
             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ref = A @ B.T + (C0 if accumulate else 0)
    got = dC.cpu().numpy()
    scale = np.abs(A) @ np.abs(B).T
    assert np.max(np.abs(got - ref) / scale) < 1e-14 * K ** 0.5 + 1e-15


@pytest.mark.parametrize("M,N,K", [(128, 128, 32), (384, 256, 1056), (256, 1024, 4096)])
def test_gemm_fp32(M, N, K):
    torch = need_gpu()
    from paper_1911_12954_amd import trg_gemm
    announce("gemm fp32", M, N, K)
    A = random_matrix(M, K, 4).astype(np.float32)
    B = random_matrix(N, K, 5).astype(np.float32)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.empty((M, N), dtype=torch.float32, device="cuda")
    trg_gemm("fp32", dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), M, N, K, K, K, N, False,
             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ref = A.astype(np.float64) @ B.astype(np.float64).T
    scale = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64)).T
    assert np.max(np.abs(dC.cpu().numpy() - ref) / scale) < 4 * 2.0 ** -24 * np.sqrt(K) + 1e-7


@pytest.mark.parametrize("M,N,K,accumulate", [(256, 256, 32, False), (512, 768, 1088, False),
                                              (768, 256, 4096, False), (512, 512, 1056, True)])
def test_gemm_bf16x3(M, N, K, accumulate):
    torch = need_gpu()
    from paper_1911_12954_amd import trg_gemm, trg_gemm_tile
    announce("gemm bf16x3", M, N, K, accumulate)
    tm, tn, tk = trg_gemm_tile("bf16x3")
    assert M % tm == 0 and N % tn == 0 and K % tk == 0
    A = random_matrix(M, K, 6)
    B = random_matrix(N, K, 7)

    def split(X):
        x32 = torch.from_numpy(X).float()
        hi = x32.to(torch.bfloat16)
        lo = (x32 - hi.float()).to(torch.bfloat16)
        return hi, lo

    ah, al = split(A)
    bh, bl = split(B)
    dA = torch.stack([ah, al]).cuda().contiguous()
    dB = torch.stack([bh, bl]).cuda().contiguous()
    C0 = random_matrix(M, N, 8).astype(np.float32)
    dC = torch.from_numpy(C0).cuda()
    trg_gemm("bf16x3", dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), M, N, K, K, K, N, accumulate,
             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    f = lambda t: t.double().numpy()
    ref = f(ah) @ f(bh).T + f(ah) @ f(bl).T + f(al) @ f(bh).T
    scale = np.abs(A) @ np.abs(B).T
    exact = A @ B.T
    if accumulate:
        c0 = C0.astype(np.float64)
        ref, exact, scale = ref + c0, exact + c0, scale + np.abs(c0)
    err = np.max(np.abs(dC.cpu().numpy() - ref) / scale)
    assert err < 4 * 2.0 ** -24 * np.sqrt(K) + 1e-7
    # and the split product is within ~2^-16 of the exact one
    assert np.max(np.abs(dC.cpu().numpy() - exact) / scale) < 2.0 ** -14


def _split3(X):
    """fl32(X) = hi + mid + lo exactly (three bfloat16 planes, round to
    nearest even at each stage), as torch tensors."""
    import torch
    x32 = torch.from_numpy(X).float()
    hi = x32.to(torch.bfloat16)
    r1 = x32 - hi.float()
    mid = r1.to(torch.bfloat16)
    lo = (r1 - mid.float()).to(torch.bfloat16)
    return hi, mid, lo


@pytest.mark.parametrize("M,N,K,accumulate", [(128, 128, 32, False), (384, 256, 1056, False),
                                              (256, 640, 4128, False), (256, 384, 1056, True)])
def test_gemm_bf16x6(M, N, K, accumulate):
    """Three-plane split join: the six products reproduce the product of the
    FP32-rounded operands to FP32 accuracy (the dropped mid*lo, lo*mid and
    lo*lo terms are below 2^-24 of each product), with FP64 sums of the
    FP32 groups (K = 4128: 32 groups and a ragged last one)."""
    torch = need_gpu()
    from paper_1911_12954_amd import trg_gemm, trg_gemm_tile
    announce("gemm bf16x6", M, N, K, accumulate)
    tm, tn, tk = trg_gemm_tile("bf16x6")
    assert M % tm == 0 and N % tn == 0 and K % tk == 0
    A = random_matrix(M, K, 16)
    B = random_matrix(N, K, 17)
    pa, pb = _split3(A), _split3(B)
    # the split is exact on the host side too
    f = lambda t: t.double().numpy()
    A32, B32 = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    assert np.array_equal(f(pa[0]) + f(pa[1]) + f(pa[2]), A32)
    dA = torch.stack(list(pa)).cuda().contiguous()
    dB = torch.stack(list(pb)).cuda().contiguous()
    C0 = random_matrix(M, N, 18).astype(np.float32)
    dC = torch.from_numpy(C0).cuda()
    trg_gemm("bf16x6", dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), M, N, K, K, K, N, accumulate,
             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ref = A32 @ B32.T
    scale = np.abs(A) @ np.abs(B).T
    if accumulate:
        c0 = C0.astype(np.float64)
        ref, scale = ref + c0, scale + np.abs(c0)
    err = np.max(np.abs(dC.cpu().numpy() - ref) / scale)
    print(f"[gemm bf16x6] max err / scale {err:.3e}", flush=True)
    # FP32 output rounding (2^-24 of |C|) plus the dropped terms and the
    # FP32 group sums; no sqrt(K) growth beyond the group length
    assert err < 12 * 2.0 ** -24


@pytest.mark.parametrize("n", [1, 2, 4, 7, 16, 33, 100, 144, 161, 200, 333, 576])
def test_jacobi_eigh(n):
    """Orders up to 160 use cyclic Jacobi, larger ones Householder
    tridiagonalisation + implicit QL."""
    torch = need_gpu()
    from paper_1911_12954_amd import trg_eigh
    announce("eigh", n)
    mats = [random_symmetric(n, 10 + n), gram_like(n, min(n, 12), 20 + n)]
    A = np.stack(mats)
    dA = torch.from_numpy(A.copy()).cuda()
    dw = torch.empty((2, n), dtype=torch.float64, device="cuda")
    dV = torch.empty((2, n, n), dtype=torch.float64, device="cuda")
    ds = torch.empty(2, dtype=torch.int32, device="cuda")
    trg_eigh(dA.data_ptr(), dw.data_ptr(), dV.data_ptr(), ds.data_ptr(), n, 2,
             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    w, V, sw = dw.cpu().numpy(), dV.cpu().numpy(), ds.cpu().numpy()
    for b in range(2):
        assert sw[b] >= 0
        ref = np.sort(np.linalg.eigvalsh(A[b]))[::-1]
        nrm = np.linalg.norm(A[b])
        assert np.max(np.abs(w[b] - ref)) < 1e-13 * nrm
        assert np.all(np.diff(w[b]) <= 0)
        assert np.allclose(V[b].T @ V[b], np.eye(n), atol=1e-13)
        assert np.allclose(V[b] @ np.diag(w[b]) @ V[b].T, A[b], atol=1e-13 * nrm)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_gemm_empty_products(precision):
    """K = 0: C is zeroed (or left as it was when accumulating); M = 0 or
    N = 0: nothing is written."""
    torch = need_gpu()
    from paper_1911_12954_amd import trg_gemm, trg_gemm_tile
    announce("gemm empty", precision)
    tm, tn, _ = trg_gemm_tile(precision)
    ct = torch.float64 if precision == "fp64" else torch.float32
    st = torch.cuda.current_stream().cuda_stream
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda")
    C = torch.full((tm, tn), 3.0, dtype=ct, device="cuda")
    trg_gemm(precision, dummy.data_ptr(), dummy.data_ptr(), C.data_ptr(), tm, tn, 0, 16, 16, tn, True, st)
    torch.cuda.synchronize()
    assert bool((C == 3.0).all())
    trg_gemm(precision, dummy.data_ptr(), dummy.data_ptr(), C.data_ptr(), tm, tn, 0, 16, 16, tn, False, st)
    torch.cuda.synchronize()
    assert bool((C == 0.0).all())
    C.fill_(5.0)
    trg_gemm(precision, dummy.data_ptr(), dummy.data_ptr(), C.data_ptr(), 0, tn, 32, 32, 32, tn, False, st)
    trg_gemm(precision, dummy.data_ptr(), dummy.data_ptr(), C.data_ptr(), tm, 0, 32, 32, 32, tn, False, st)
    torch.cuda.synchronize()
    assert bool((C == 5.0).all())


@pytest.mark.parametrize("n", [16, 200])
def test_eigh_degenerate_and_zero_matrices(n):
    """Exactly repeated eigenvalues (any orthonormal basis of the eigenspace
    is correct: check the eigenvalues, orthonormality and reconstruction)
    and the zero matrix, on both solver paths."""
    torch = need_gpu()
    from paper_1911_12954_amd import trg_eigh
    announce("eigh degenerate", n)
    rng = np.random.default_rng(n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat(np.array([3.0, 1.0, -2.0, 0.5]), n // 4)
    A = np.stack([Q @ np.diag(lam) @ Q.T, np.eye(n), np.zeros((n, n))])
    A = 0.5 * (A + A.transpose(0, 2, 1))
    dA = torch.from_numpy(A.copy()).cuda()
    dw = torch.empty((3, n), dtype=torch.float64, device="cuda")
    dV = torch.empty((3, n, n), dtype=torch.float64, device="cuda")
    ds = torch.empty(3, dtype=torch.int32, device="cuda")
    trg_eigh(dA.data_ptr(), dw.data_ptr(), dV.data_ptr(), ds.data_ptr(), n, 3,
             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    w, V = dw.cpu().numpy(), dV.cpu().numpy()
    for b in range(3):
        ref = np.sort(np.linalg.eigvalsh(A[b]))[::-1]
        scale = max(np.linalg.norm(A[b]), 1.0)
        assert np.max(np.abs(w[b] - ref)) < 1e-13 * scale
        assert np.allclose(V[b].T @ V[b], np.eye(n), atol=1e-13)
        assert np.allclose(V[b] @ np.diag(w[b]) @ V[b].T, A[b], atol=1e-13 * scale)


@pytest.mark.parametrize("n", [100, 200, 400])
@pytest.mark.parametrize("tiny", [1e-160, 1e-250])
def test_eigh_block_far_below_the_matrix_scale(n, tiny):
    """Two diagonal blocks (contiguous, as in a parity-sorted Gram), the
    second scaled by `tiny`, so that sums of squares of its columns fall
    below the FP64 normal range (1e-160: into the subnormals, where an
    unscaled Householder reflector's 2 / v^T v overflows): eigenvalues to
    1e-13 of the matrix norm, orthonormal and finite eigenvectors, each lying
    in one block with exact zeros in the other, and the reconstruction.
    Both solver paths (Jacobi to 160, Householder + QL above)."""
    torch = need_gpu()
    from paper_1911_12954_amd import trg_eigh
    announce("eigh tiny block", n, tiny)
    n0 = n // 2 + 3
    a = gram_like(n0, min(n0, 12), 5 + n)
    b = random_symmetric(n - n0, 6 + n)
    b = b @ b.T / (n - n0)                  # positive semi-definite, O(1)
    A = np.zeros((n, n))
    A[:n0, :n0] = a
    A[n0:, n0:] = tiny * b
    dA = torch.from_numpy(A.copy()).cuda()
    dw = torch.empty((1, n), dtype=torch.float64, device="cuda")
    dV = torch.empty((1, n, n), dtype=torch.float64, device="cuda")
    ds = torch.empty(1, dtype=torch.int32, device="cuda")
    trg_eigh(dA.data_ptr(), dw.data_ptr(), dV.data_ptr(), ds.data_ptr(), n, 1,
             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    w, V = dw.cpu().numpy()[0], dV.cpu().numpy()[0]
    assert np.all(np.isfinite(w)) and np.all(np.isfinite(V))
    nrm = np.linalg.norm(A)
    assert np.max(np.abs(w - np.sort(np.linalg.eigvalsh(A))[::-1])) < 1e-13 * nrm
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-13)
    assert np.allclose(V @ np.diag(w) @ V.T, A, atol=1e-13 * nrm)
    in_a = np.abs(V[:n0]).sum(0) > 0
    in_b = np.abs(V[n0:]).sum(0) > 0
    assert not np.any(in_a & in_b)
    assert int(in_a.sum()) == n0 and int(in_b.sum()) == n - n0


def _eigh_top(A, k, rel):
    torch = need_gpu()
    from paper_1911_12954_amd import trg_eigh_top, trg_eigh_top_work_bytes
    batch, n = A.shape[0], A.shape[1]
    dA = torch.from_numpy(A.copy()).cuda()
    dw = torch.empty((batch, n), dtype=torch.float64, device="cuda")
    dV = torch.empty((batch, n, n), dtype=torch.float64, device="cuda")
    ds = torch.empty(batch, dtype=torch.int32, device="cuda")
    nb = trg_eigh_top_work_bytes(n, batch)
    work = torch.empty(max(nb // 8, 1), dtype=torch.float64, device="cuda")
    trg_eigh_top(dA.data_ptr(), dw.data_ptr(), dV.data_ptr(), ds.data_ptr(), n, batch, k, rel, work.data_ptr(),
                 torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return dw.cpu().numpy(), dV.cpu().numpy(), ds.cpu().numpy()


@pytest.mark.parametrize("n", [150, 169, 256, 576])
def test_eigh_top_leading_pairs(n):
    """Every eigenvalue and the leading eigenvectors of Gram-like matrices
    (fast-decaying spectra, as the HOSVD Grams) and of random symmetric ones,
    against LAPACK: eigenvalues to 1e-13 of the norm, each computed vector an
    eigenvector (residual 1e-12 of the norm) orthonormal to the others, the
    columns beyond those needed zero."""
    announce("eigh_top", n)
    k = 24
    A = np.stack([gram_like(n, min(n, 60), 30 + n), random_symmetric(n, 40 + n)])
    w, V, kk = _eigh_top(A, k, 1e-10)
    for b in range(2):
        ref = np.sort(np.linalg.eigvalsh(A[b]))[::-1]
        nrm = np.linalg.norm(A[b])
        assert np.max(np.abs(w[b] - ref)) < 1e-13 * nrm
        q = int(kk[b]) if n > 160 else n     # the Jacobi path returns every vector (and its sweeps)
        assert k <= q <= n
        Vk = V[b][:, :q]
        assert np.all(V[b][:, q:] == 0.0)
        assert np.allclose(Vk.T @ Vk, np.eye(q), atol=1e-12)
        assert np.max(np.abs(A[b] @ Vk - Vk * w[b][:q])) < 1e-12 * nrm


def test_eigh_top_extends_over_a_split_cluster():
    """Eigenvalues 5, 4, 3 (x3), 2, ...: with k = 3 the cut splits the triple,
    so kk = 5 vectors come back, spanning the triple's eigenspace."""
    announce("eigh_top cluster")
    n = 200
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([[5.0, 4.0, 3.0, 3.0, 3.0, 2.0], np.linspace(1.0, 0.0, n - 6)])
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    w, V, kk = _eigh_top(A[None], 3, 1e-10)
    assert int(kk[0]) == 5
    P = V[0][:, 2:5] @ V[0][:, 2:5].T
    Pref = Q[:, 2:5] @ Q[:, 2:5].T
    assert np.max(np.abs(P - Pref)) < 1e-12


def test_eigh_top_parity_blocks_stay_exact():
    """A sector-ordered block-diagonal matrix (second block 1e-160 of the
    first, and exactly degenerate eigenvalues across the blocks): every
    computed vector lies in one block with exact zeros in the other, and the
    degenerate pair across the blocks gives one vector in each."""
    announce("eigh_top parity blocks")
    n, n0 = 300, 170
    a = gram_like(n0, 40, 11)
    b = gram_like(n - n0, 40, 12)
    A = np.zeros((2, n, n))
    A[0, :n0, :n0] = a
    A[0, n0:, n0:] = 1e-160 * b
    A[1, :n0, :n0] = a
    A[1, n0:, n0:] = a[: n - n0, : n - n0] * 0.0 + np.diag(np.linalg.eigvalsh(a)[::-1][: n - n0])
    w, V, kk = _eigh_top(A, 10, 1e-10)
    for bb in range(2):
        q = int(kk[bb])
        Vk = V[bb][:, :q]
        in_a = np.abs(Vk[:n0]).sum(0) > 0
        in_b = np.abs(Vk[n0:]).sum(0) > 0
        assert not np.any(in_a & in_b)
        assert np.all(np.isfinite(Vk))
        nrm = np.linalg.norm(A[bb])
        assert np.max(np.abs(A[bb] @ Vk - Vk * w[bb][:q])) < 1e-12 * nrm
    # the second matrix: block b holds the leading eigenvalues of block a, so
    # every leading eigenvalue is doubly degenerate across the blocks
    q = int(kk[1])
    in_b = np.abs(V[1][n0:, :q]).sum(0) > 0
    assert 0 < int(in_b.sum()) < q
