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
