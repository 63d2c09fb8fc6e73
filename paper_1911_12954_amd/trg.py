"""Python binding of libtrg: the C-ABI entry points under the same names,
plus a small Context wrapper.  Argument marshalling only; every step of the
computation runs in the HIP library.  PyTorch supplies the device allocator
(its caching allocator) and the stream."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L

PRECISIONS = {"fp64": L.TRG_FP64, "fp32": L.TRG_FP32, "bf16x3": L.TRG_BF16X3, "bf16x6": L.TRG_BF16X6}
METHODS = {"hotrg": L.TRG_HOTRG, "atrg": L.TRG_ATRG}


class TrgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libtrg error {code}: {msg}")
        self.code = code


def _lib():
    return L.load()


def _err(rc: int, handle=None):
    if rc != L.TRG_OK:
        msg = _lib().trg_last_error(handle)
        raise TrgError(rc, msg.decode() if msg else "")


def _torch_allocator(stream_ptr):
    """ctypes callbacks that allocate through torch's caching allocator on
    the given stream."""
    import torch

    dev = torch.cuda.current_device()

    @L.ALLOC_FN
    def alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream_ptr or 0))
        except Exception:
            return None

    @L.FREE_FN
    def free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


def make_config(precision="fp64", method="hotrg", dcut=8, impure=(), stream=None,
                use_torch_allocator=True, workspace_bytes=0, rsvd_p=0, rsvd_q=0, seed=0, fp64_steps=0, z2=False):
    """Build a trg_config.  ``stream``: a torch.cuda.Stream, an int handle or
    None (torch's current stream when torch has a GPU, else the default)."""
    cfg = L.TrgConfig()
    cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    cfg.method = METHODS[method] if isinstance(method, str) else int(method)
    cfg.dcut = int(dcut)
    bits = 0
    for x in impure:
        bits |= {"E": L.TRG_IMPURE_E, "M": L.TRG_IMPURE_M}[x]
    cfg.impure = bits
    cfg.rsvd_p, cfg.rsvd_q, cfg.seed = int(rsvd_p), int(rsvd_q), int(seed)
    cfg.workspace_bytes = int(workspace_bytes)
    cfg.fp64_steps = int(fp64_steps)
    cfg.z2 = 1 if z2 else 0
    keep = []
    sp = None
    try:
        import torch
        if torch.cuda.is_available():
            if stream is None:
                stream = torch.cuda.current_stream()
            sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
            if use_torch_allocator:
                a, f = _torch_allocator(sp)
                cfg.alloc, cfg.free = a, f
                keep += [a, f]
    except ImportError:
        sp = stream
    cfg.stream = C.c_void_p(sp) if sp else None
    return cfg, keep


@dataclass
class StepRecord:
    n: int
    axis: int
    dims: tuple
    side: tuple
    kept: tuple
    degenerate_cut: tuple
    sweeps: tuple
    ln_c: float
    eps: tuple
    join_precision: str = "fp64"


class Context:
    """Owns one trg_ctx handle."""

    def __init__(self, handle, keep, d):
        self.handle = handle
        self._keep = keep
        self.d = d

    # -- steps
    def hotrg_step(self, axis: int, dcut: int):
        _err(_lib().trg_hotrg_step(self.handle, axis, dcut), self.handle)

    def run(self, L_: int):
        _err(_lib().trg_run(self.handle, L_), self.handle)

    # -- results
    def _dbl(self, fn):
        out = C.c_double()
        _err(fn(self.handle, C.byref(out)), self.handle)
        return out.value

    def free_energy(self) -> float:
        return self._dbl(_lib().trg_free_energy)

    def export_state(self) -> bytes:
        """Checkpoint blob of the current state (trg_export_state)."""
        n = C.c_size_t()
        _err(_lib().trg_export_state(self.handle, None, 0, C.byref(n)), self.handle)
        buf = C.create_string_buffer(n.value)
        _err(_lib().trg_export_state(self.handle, buf, n.value, C.byref(n)), self.handle)
        return buf.raw[:n.value]

    def impure_energy(self) -> float:
        return self._dbl(_lib().trg_impure_energy)

    def impure_magnetization(self) -> float:
        return self._dbl(_lib().trg_impure_magnetization)

    def indicator_x(self, axis: int = 0) -> float:
        out = C.c_double()
        _err(_lib().trg_indicator_x(self.handle, int(axis), C.byref(out)), self.handle)
        return out.value

    def indicator_x_noalloc(self, axis: int = 0) -> float:
        """trg_indicator_x_noalloc: the same X without any device allocation."""
        out = C.c_double()
        _err(_lib().trg_indicator_x_noalloc(self.handle, int(axis), C.byref(out)), self.handle)
        return out.value

    def accumulator(self) -> float:
        return self._dbl(_lib().trg_accumulator)

    def dims(self):
        arr = (C.c_int * 4)()
        steps = C.c_int()
        _err(_lib().trg_get_dims(self.handle, arr, C.byref(steps)), self.handle)
        return tuple(arr[: self.d]), steps.value

    def tensor(self, which: int = 0) -> np.ndarray:
        dims, _ = self.dims()
        shape = tuple(x for x in dims for _ in range(2))
        out = np.empty(shape, dtype=np.float64)
        _err(_lib().trg_get_tensor(self.handle, which, out.ctypes.data_as(C.POINTER(C.c_double)), out.size),
             self.handle)
        return out

    def isometry(self, nu: int):
        log = self.step_log()
        rec = log[-1]
        k = rec.kept[nu]
        dims_prev = self._prev_dim(nu)
        n = dims_prev * dims_prev
        U = np.empty((n, k))
        spec = np.empty(n)
        _err(_lib().trg_get_isometry(self.handle, nu, U.ctypes.data_as(C.POINTER(C.c_double)), U.size,
                                     spec.ctypes.data_as(C.POINTER(C.c_double)), spec.size), self.handle)
        return U, spec

    def _prev_dim(self, nu):
        log = self.step_log()
        if len(log) >= 2:
            return log[-2].dims[nu]
        return self._initial_dims[nu]

    def step_log(self):
        n = C.c_int()
        _err(_lib().trg_step_log(self.handle, None, 0, C.byref(n)), self.handle)
        recs = (L.TrgStepRec * max(n.value, 1))()
        _err(_lib().trg_step_log(self.handle, recs, n.value, C.byref(n)), self.handle)
        out = []
        for r in recs[: n.value]:
            out.append(StepRecord(r.n, r.axis, tuple(r.dims[: self.d]), tuple(r.side[: self.d]),
                                  tuple(r.kept[: self.d]), tuple(r.degenerate_cut[: self.d]),
                                  tuple(r.sweeps[: self.d]), r.ln_c,
                                  tuple(tuple(r.eps[a]) for a in range(self.d)),
                                  {v: k for k, v in PRECISIONS.items()}.get(r.join_precision, "?")))
        return out

    def atrg_step(self, axis: int, dcut: int):
        _err(_lib().trg_atrg_step(self.handle, axis, dcut), self.handle)

    def atrg_spectrum(self):
        n = C.c_int()
        _err(_lib().trg_atrg_spectrum(self.handle, None, 0, C.byref(n)), self.handle)
        out = np.empty(max(n.value, 1))
        _err(_lib().trg_atrg_spectrum(self.handle, out.ctypes.data_as(C.POINTER(C.c_double)), out.size,
                                      C.byref(n)), self.handle)
        return out[: n.value]

    def atrg_parities(self):
        """trg_atrg_parities: (per-axis leg parity arrays, bond parity array)
        of a Z2-mode ATRG context."""
        dims, _ = self.dims()
        ip = C.POINTER(C.c_int)
        r = C.c_int()
        _err(_lib().trg_atrg_parities(self.handle, None, 0, None, 0, C.byref(r)), self.handle)
        legs = np.zeros(max(sum(dims), 1), dtype=np.int32)
        bond = np.zeros(max(r.value, 1), dtype=np.int32)
        _err(_lib().trg_atrg_parities(self.handle, legs.ctypes.data_as(ip), legs.size, bond.ctypes.data_as(ip),
                                      bond.size, None), self.handle)
        out, o = [], 0
        for n in dims:
            out.append(legs[o:o + n].copy())
            o += n
        return out, bond[: r.value].copy()

    def factors(self):
        """trg_get_factors: the ATRG pieces G [b0..b_{d-1}, l] and H [l, f0..f_{d-1}]."""
        dims, _ = self.dims()
        r = C.c_int()
        _err(_lib().trg_get_factors(self.handle, None, 0, None, 0, C.byref(r)), self.handle)
        G = np.empty(tuple(dims) + (r.value,))
        H = np.empty((r.value,) + tuple(dims))
        dp = C.POINTER(C.c_double)
        _err(_lib().trg_get_factors(self.handle, G.ctypes.data_as(dp), G.size, H.ctypes.data_as(dp), H.size, None),
             self.handle)
        return G, H

    def set_profiling(self, on=True):
        _err(_lib().trg_set_profiling(self.handle, 1 if on else 0), self.handle)

    def join_profile(self):
        ms, n, fl = C.c_double(), C.c_longlong(), C.c_double()
        _err(_lib().trg_join_profile(self.handle, C.byref(ms), C.byref(n), C.byref(fl)), self.handle)
        return ms.value, n.value, fl.value

    def set_force_side(self, side: int):
        _err(_lib().trg_set_force_side(self.handle, side), self.handle)

    def sync(self):
        _err(_lib().trg_sync(self.handle), self.handle)

    def close(self):
        if self.handle:
            _lib().trg_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------- C-ABI names ---

def trg_init_ising(beta: float, h: float, d: int, **cfg) -> Context:
    conf, keep = make_config(**cfg)
    h_ = C.c_void_p()
    _err(_lib().trg_init_ising(C.byref(h_), float(beta), float(h), int(d), C.byref(conf)))
    ctx = Context(h_, keep + [conf], d)
    ctx._initial_dims = (2,) * d
    return ctx


def trg_init_tensor(T: np.ndarray, **cfg) -> Context:
    T = np.ascontiguousarray(T, dtype=np.float64)
    d = T.ndim // 2
    dims = (C.c_int * d)(*[T.shape[2 * a] for a in range(d)])
    conf, keep = make_config(**cfg)
    h_ = C.c_void_p()
    _err(_lib().trg_init_tensor(C.byref(h_), d, dims, T.ctypes.data_as(C.POINTER(C.c_double)), C.byref(conf)))
    ctx = Context(h_, keep + [conf], d)
    ctx._initial_dims = tuple(T.shape[2 * a] for a in range(d))
    return ctx


def trg_export_state(ctx: Context) -> bytes:
    return ctx.export_state()


def trg_import_state(blob: bytes, **cfg) -> Context:
    """Context from a checkpoint blob; cfg contributes the stream, allocator
    and workspace budget (the blob fixes the numerics)."""
    import struct
    if len(blob) < 20:
        raise TrgError(L.TRG_EINVAL, "state blob too short")
    d = struct.unpack_from("<i", blob, 16)[0]
    conf, keep = make_config(**cfg)
    h_ = C.c_void_p()
    buf = C.create_string_buffer(blob, len(blob))
    _err(_lib().trg_import_state(C.byref(h_), buf, len(blob), C.byref(conf)))
    return Context(h_, keep + [conf], d)


def trg_init_factors(G: np.ndarray, H: np.ndarray, **cfg) -> Context:
    """ATRG context from pieces G[b0..b_{d-1}, l] and H[l, f0..f_{d-1}]."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    d = G.ndim - 1
    r = G.shape[-1]
    dims = (C.c_int * d)(*G.shape[:-1])
    cfg.setdefault("method", "atrg")
    conf, keep = make_config(**cfg)
    h_ = C.c_void_p()
    _err(_lib().trg_init_factors(C.byref(h_), d, dims, r, G.ctypes.data_as(C.POINTER(C.c_double)),
                                 H.ctypes.data_as(C.POINTER(C.c_double)), C.byref(conf)))
    ctx = Context(h_, keep + [conf], d)
    ctx._initial_dims = tuple(G.shape[:-1])
    return ctx


def trg_hotrg_step(ctx: Context, axis: int, dcut: int):
    ctx.hotrg_step(axis, dcut)


def trg_hotrg_step_batch(ctxs, axis: int, dcut: int):
    arr = (C.c_void_p * len(ctxs))(*[c.handle.value if isinstance(c.handle, C.c_void_p) else c.handle
                                      for c in ctxs])
    _err(_lib().trg_hotrg_step_batch(arr, len(ctxs), axis, dcut))


def trg_atrg_step(ctx: Context, axis: int, dcut: int):
    ctx.atrg_step(axis, dcut)


def trg_run(ctx: Context, L_: int):
    ctx.run(L_)


def trg_free_energy(ctx: Context) -> float:
    return ctx.free_energy()


def trg_impure_energy(ctx: Context) -> float:
    return ctx.impure_energy()


def trg_impure_magnetization(ctx: Context) -> float:
    return ctx.impure_magnetization()


def trg_footprint_bytes(d, dcut, precision="fp64", method="hotrg", impure=()) -> int:
    bits = 0
    for x in impure:
        bits |= {"E": L.TRG_IMPURE_E, "M": L.TRG_IMPURE_M}[x]
    return int(_lib().trg_footprint_bytes(d, dcut, PRECISIONS[precision], METHODS[method], bits))


def trg_indicator_x(ctx: Context, axis: int = 0) -> float:
    return ctx.indicator_x(axis)


def trg_resident_bytes(d, dcut, precision="fp64", method="hotrg", impure=()) -> int:
    bits = sum({"E": L.TRG_IMPURE_E, "M": L.TRG_IMPURE_M}[x] for x in impure)
    return int(_lib().trg_resident_bytes(d, dcut, PRECISIONS[precision], METHODS[method], bits))


def trg_workspace_bytes(d, dcut, precision="fp64", method="hotrg", impure=()) -> int:
    bits = sum({"E": L.TRG_IMPURE_E, "M": L.TRG_IMPURE_M}[x] for x in impure)
    return int(_lib().trg_workspace_bytes(d, dcut, PRECISIONS[precision], METHODS[method], bits))


def trg_share_workspace(ctx: Context, donor: Context):
    """ctx uses donor's workspace from now on (same stream required)."""
    _err(_lib().trg_share_workspace(ctx.handle, donor.handle), ctx.handle)
    # the shared workspace is released through donor's free callback
    ctx._keep = list(ctx._keep) + list(donor._keep)


def trg_gemm(precision, A_ptr, Bt_ptr, C_ptr, M, N, K, lda, ldb, ldc, accumulate=False, stream=None):
    _err(_lib().trg_gemm(PRECISIONS[precision] if isinstance(precision, str) else precision,
                         A_ptr, Bt_ptr, C_ptr, M, N, K, lda, ldb, ldc, 1 if accumulate else 0, stream))


def trg_gemm_tile(precision):
    m, n, k = C.c_int(), C.c_int(), C.c_int()
    _err(_lib().trg_gemm_tile(PRECISIONS[precision], C.byref(m), C.byref(n), C.byref(k)))
    return m.value, n.value, k.value


def trg_eigh(A_ptr, w_ptr, V_ptr, sweeps_ptr, n, batch, stream=None):
    _err(_lib().trg_eigh(A_ptr, w_ptr, V_ptr, sweeps_ptr, n, batch, stream))


def trg_eigh_top(A_ptr, w_ptr, V_ptr, sweeps_ptr, n, batch, k, cluster_rel, work_ptr, stream=None):
    _err(_lib().trg_eigh_top(A_ptr, w_ptr, V_ptr, sweeps_ptr, n, batch, k, float(cluster_rel), work_ptr, stream))


def trg_eigh_top_work_bytes(n, batch):
    return int(_lib().trg_eigh_top_work_bytes(n, batch))
