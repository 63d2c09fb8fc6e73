"""The C-ABI library loads and exports every symbol include/trg.h declares;
host-side argument checks return error codes without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1911_12954_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "trg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(trg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libtrg.so is not built (python -m paper_1911_12954_amd.build)")
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_declares_every_header_symbol():
    assert sorted(L.SIGNATURES) == declared_symbols()


def test_invalid_arguments_are_rejected_on_the_host(lib):
    h = C.c_void_p()
    assert lib.trg_init_ising(None, 0.1, 0.0, 4, None) == L.TRG_EINVAL
    assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 5, None) == L.TRG_EINVAL
    assert b"d must be" in lib.trg_last_error(None)
    assert lib.trg_init_ising(C.byref(h), -1.0, 0.0, 4, None) == L.TRG_EINVAL
    assert lib.trg_init_ising(C.byref(h), float("nan"), 0.0, 4, None) == L.TRG_EINVAL
    cfg = L.TrgConfig()
    cfg.impure = L.TRG_IMPURE_E
    assert lib.trg_init_ising(C.byref(h), 0.0, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    cfg = L.TrgConfig()
    cfg.precision = 7
    assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    assert lib.trg_hotrg_step(None, 0, 4) == L.TRG_EINVAL
    assert lib.trg_run(None, 16) == L.TRG_EINVAL
    lib.trg_free(None)


def test_gemm_tile_and_footprint(lib):
    m, n, k = C.c_int(), C.c_int(), C.c_int()
    for prec, tile in ((L.TRG_FP64, (128, 128, 16)), (L.TRG_FP32, (128, 128, 32)), (L.TRG_BF16X3, (256, 256, 32)),
                       (L.TRG_BF16X6, (128, 128, 32))):
        assert lib.trg_gemm_tile(prec, C.byref(m), C.byref(n), C.byref(k)) == 0
        assert (m.value, n.value, k.value) == tile
    f8 = lib.trg_footprint_bytes(4, 8, L.TRG_FP64, L.TRG_HOTRG, 0)
    f10 = lib.trg_footprint_bytes(4, 10, L.TRG_FP64, L.TRG_HOTRG, 0)
    f10m = lib.trg_footprint_bytes(4, 10, L.TRG_FP32, L.TRG_HOTRG, 0)
    assert 0 < f8 < f10 and f10m < f10
    # resident part alone: 2 buffers x D^8 doubles
    assert f10 > 2 * 10 ** 8 * 8
    assert lib.trg_footprint_bytes(5, 8, 0, 0, 0) == 0
    for args in ((4, 10, L.TRG_FP64, L.TRG_HOTRG, 0), (4, 6, L.TRG_FP32, L.TRG_HOTRG, 3),
                 (3, 12, L.TRG_BF16X3, L.TRG_HOTRG, 1), (4, 10, L.TRG_BF16X6, L.TRG_HOTRG, 3),
                 (4, 24, L.TRG_FP64, L.TRG_ATRG, 0)):
        res, ws = lib.trg_resident_bytes(*args), lib.trg_workspace_bytes(*args)
        assert res > 0 and ws > 0 and lib.trg_footprint_bytes(*args) == res + ws
    # resident: T, S_E, S_M and their next-step buffers, D^8 doubles each
    assert lib.trg_resident_bytes(4, 6, L.TRG_FP32, L.TRG_HOTRG, 3) == 6 * 6 ** 8 * 8
    # the workspace at Dcut 10 holds at least the whole Bt operand and the
    # D^9 operand-build temporary
    assert lib.trg_workspace_bytes(4, 10, L.TRG_FP64, L.TRG_HOTRG, 0) > 10 ** 9 * 8 + 10 ** 5 * 10 ** 5 * 8


def test_more_argument_checks_on_the_host(lib):
    """Every rejected call returns TRG_EINVAL and sets a message before any
    device work (these run without a GPU)."""
    h = C.c_void_p()
    cfg = L.TrgConfig()
    cfg.fp64_steps = -1
    assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    assert b"fp64_steps" in lib.trg_last_error(None)
    for prec in (L.TRG_BF16X3, L.TRG_BF16X6):
        cfg = L.TrgConfig()
        cfg.method, cfg.precision = L.TRG_ATRG, prec
        assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    cfg = L.TrgConfig()
    cfg.precision = 4
    assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    cfg = L.TrgConfig()
    cfg.method, cfg.impure = L.TRG_ATRG, L.TRG_IMPURE_E
    assert lib.trg_init_ising(C.byref(h), 0.0, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    assert b"beta > 0" in lib.trg_last_error(None)
    # checkpoint blobs are validated before any device work
    assert lib.trg_import_state(C.byref(h), None, 0, None) == L.TRG_EINVAL
    junk = C.create_string_buffer(b"NOTSTATE" + bytes(200))
    assert lib.trg_import_state(C.byref(h), junk, 208, None) == L.TRG_EINVAL
    assert b"magic" in lib.trg_last_error(None)
    assert lib.trg_import_state(C.byref(h), junk, 4, None) == L.TRG_EINVAL
    cfg = L.TrgConfig()
    cfg.dcut = 2000
    assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    cfg = L.TrgConfig()
    cfg.impure = 4
    assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    cfg = L.TrgConfig()
    cfg.alloc = L.ALLOC_FN(lambda n, u: None)     # alloc without free
    assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    assert b"together" in lib.trg_last_error(None)
    assert lib.trg_init_ising(C.byref(h), 0.1, float("inf"), 4, None) == L.TRG_EINVAL
    # batches, sharing, kernel-level entries
    assert lib.trg_hotrg_step_batch(None, 1, 0, 4) == L.TRG_EINVAL
    arr = (C.c_void_p * 2)(None, None)
    assert lib.trg_hotrg_step_batch(arr, 0, 0, 4) == L.TRG_EINVAL
    assert lib.trg_hotrg_step_batch(arr, 2, 0, 4) == L.TRG_EINVAL
    # the same context twice is rejected before any context is read (the
    # pointer names a host buffer, never dereferenced)
    fake = C.create_string_buffer(64)
    dup = (C.c_void_p * 3)(C.addressof(fake), C.addressof(fake) + 16, C.addressof(fake))
    assert lib.trg_hotrg_step_batch(dup, 3, 0, 4) == L.TRG_EINVAL
    assert b"twice" in lib.trg_last_error(None)
    assert lib.trg_share_workspace(None, None) == L.TRG_EINVAL
    assert lib.trg_atrg_step(None, 0, 4) == L.TRG_EINVAL
    assert lib.trg_free_energy(None, None) == L.TRG_EINVAL
    one = C.c_double()
    # GEMM sizes that are not tile multiples, eigh orders out of range
    assert lib.trg_gemm(L.TRG_FP64, C.byref(one), C.byref(one), C.byref(one), 100, 128, 16, 16, 16, 128, 0, None) \
        == L.TRG_EINVAL
    assert b"tile multiples" in lib.trg_last_error(None)
    assert lib.trg_gemm(5, C.byref(one), C.byref(one), C.byref(one), 128, 128, 16, 16, 16, 128, 0, None) == L.TRG_EINVAL
    iv = C.c_int()
    assert lib.trg_eigh(C.byref(one), C.byref(one), C.byref(one), C.byref(iv), 0, 1, None) == L.TRG_EINVAL
    assert lib.trg_eigh(C.byref(one), C.byref(one), C.byref(one), C.byref(iv), 2000, 1, None) == L.TRG_EINVAL
    dims = (C.c_int * 4)(2, 2, 2, 2)
    assert lib.trg_init_factors(C.byref(h), 4, dims, 2, None, None, None) == L.TRG_EINVAL


def test_z2_mode_argument_checks_on_the_host(lib):
    """The Z2 mode is an ATRG mode for the h = 0 tensor built by
    trg_init_ising; everything else is refused before device work."""
    h = C.c_void_p()
    cfg = L.TrgConfig()
    cfg.z2 = 1                                   # HOTRG
    assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    assert b"ATRG" in lib.trg_last_error(None)
    cfg.method = L.TRG_ATRG
    assert lib.trg_init_ising(C.byref(h), 0.1, 1e-5, 4, C.byref(cfg)) == L.TRG_EINVAL
    assert b"h = 0" in lib.trg_last_error(None)
    cfg.z2 = 2
    assert lib.trg_init_ising(C.byref(h), 0.1, 0.0, 4, C.byref(cfg)) == L.TRG_EINVAL
    cfg.z2 = 1
    dims = (C.c_int * 2)(2, 2)
    g = (C.c_double * 8)()
    assert lib.trg_init_factors(C.byref(h), 2, dims, 2, g, g, C.byref(cfg)) == L.TRG_EINVAL
    assert b"trg_init_ising" in lib.trg_last_error(None)
    assert lib.trg_atrg_parities(None, None, 0, None, 0, None) == L.TRG_EINVAL
    assert lib.trg_get_factors(None, None, 0, None, 0, None) == L.TRG_EINVAL
