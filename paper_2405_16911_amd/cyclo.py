"""ctypes binding of libcyclo.so (C ABI in include/cyclo.h).

Argument marshalling only: every step of the estimator runs in the HIP
library.  Device buffers are torch tensors (used for memory and streams).  If
the library is not built this module raises on first use; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcyclo.so")

CYC_OK = 0
CYC_EINVAL = -1
CYC_ENOMEM = -2
CYC_EDEVICE = -3
CYC_ESTATE = -4
CYC_EUNSUPPORTED = -5

CYC_OP_FP32 = 0x0
CYC_OP_BF16 = 0x1
CYC_OP_FP16 = 0x2
CYC_TW_SPLIT = 0x4
CYC_OUT_C128 = 0x8
CYC_TBL_R = 0x10
CYC_TBL_RCONJ = 0x20
CYC_NN_NO_LOCAL = 0x100

#: exported symbols and their ctypes signatures (restype, argtypes)
SIGNATURES = {
    "cyc_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double),
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p]),
    "cyc_push": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "cyc_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "cyc_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "cyc_destroy": (None, [ctypes.c_void_p]),
    "cyc_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "cyc_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int32)]),
    "cyc_kernel_cfg_count": (ctypes.c_int, []),
    "cyc_kernel_cfg_info": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_uint32),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_char_p)]),
    "cyc_set_kernel_cfg": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "cyc_autotune": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                    ctypes.c_void_p]),
    "cyc_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                        ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p]),
    "cyc_batch_push": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "cyc_batch_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_void_p]),
    "cyc_batch_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "cyc_batch_destroy": (None, [ctypes.c_void_p]),
    "cyc_batch_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "cyc_batch_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "cyc_batch_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "cyc_model_num_params": (ctypes.c_int64, []),
    "cyc_model_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_uint32,
                                        ctypes.c_void_p]),
    "cyc_model_destroy": (None, [ctypes.c_void_p]),
    "cyc_model_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cyc_model_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cyc_model_spectra": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "cyc_model_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "cyc_model_gradients": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "cyc_create2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p]),
    "cyc_create_window": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p]),
    "cyc_push2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p]),
    "cyc_grid_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_uint32, ctypes.c_void_p]),
    "cyc_grid_create2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                                        ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p]),
    "cyc_grid_push2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p]),
    "cyc_grid_push": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "cyc_grid_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "cyc_grid_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "cyc_grid_destroy": (None, [ctypes.c_void_p]),
    "cyc_scf": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "cyc_scf_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "cyc_cfe_detect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cyc_cfe_refine": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "cyc_estimate_cycle_freqs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                                ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                                ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cyc_propose": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cyc_model_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_float, ctypes.c_float, ctypes.POINTER(ctypes.c_double),
                                            ctypes.c_void_p]),
    "cyc_select": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cyc_peak_labels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "cyc_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "cyc_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


class CycloError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {status_str(code)} ({code})")
        self.code = code


def lib() -> ctypes.CDLL:
    """Loads libcyclo.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2405_16911_amd.build "
                               "(the estimator has no non-HIP implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(code: int) -> str:
    return lib().cyc_status_str(int(code)).decode()


def _check(code: int, where: str):
    if code != CYC_OK:
        raise CycloError(code, where)


def _stream_handle(stream) -> int | None:
    """hipStream_t of a torch stream (None -> torch's current stream)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


# ----------------------------------------------------------------------------- same-name calls

def cyc_create(alphas, n_lag: int, flags: int = 0, stream=None) -> ctypes.c_void_p:
    a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).reshape(-1))
    out = ctypes.c_void_p()
    code = lib().cyc_create(ctypes.byref(out), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            int(a.size), int(n_lag), int(flags), _stream_handle(stream))
    _check(code, "cyc_create")
    return out


def cyc_push(state, x, stream=None):
    """x: 1-D contiguous torch.complex64 tensor on the GPU."""
    import torch
    if x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous() or x.dim() != 1:
        raise ValueError("x must be a contiguous 1-D complex64 CUDA tensor")
    _check(lib().cyc_push(state, ctypes.c_void_p(x.data_ptr()) if x.numel() else None,
                          int(x.numel()), _stream_handle(stream)), "cyc_push")


def cyc_read(state, R=None, Rc=None, stream=None) -> int:
    """Writes the tables into the given [T, A] tensors (either may be None); returns N_used."""
    n_used = ctypes.c_int64(0)
    pr = ctypes.c_void_p(R.data_ptr()) if R is not None else None
    prc = ctypes.c_void_p(Rc.data_ptr()) if Rc is not None else None
    _check(lib().cyc_read(state, pr, prc, ctypes.byref(n_used), _stream_handle(stream)), "cyc_read")
    return int(n_used.value)


def cyc_reset(state):
    _check(lib().cyc_reset(state), "cyc_reset")


def cyc_destroy(state):
    lib().cyc_destroy(state)


def cyc_status_str(code: int) -> str:
    return status_str(code)


def cyc_query(state) -> dict:
    n, c = ctypes.c_int64(), ctypes.c_int64()
    k, cfg = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().cyc_query(state, ctypes.byref(n), ctypes.byref(c), ctypes.byref(k), ctypes.byref(cfg)),
           "cyc_query")
    return dict(n_pushed=n.value, n_committed=c.value, chunk=k.value, kernel_cfg=cfg.value)


def cyc_profile(state, enable: bool):
    _check(lib().cyc_profile(state, 1 if enable else 0), "cyc_profile")


def cyc_profile_read(state) -> dict:
    ms, n, w = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().cyc_profile_read(state, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(w)),
           "cyc_profile_read")
    return dict(total_ms=ms.value, launches=n.value, work=w.value)


def cyc_kernel_cfg_count() -> int:
    return int(lib().cyc_kernel_cfg_count())


def cyc_kernel_cfg_info(idx: int) -> dict:
    fl, tw, aw, nt = ctypes.c_uint32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    name = ctypes.c_char_p()
    _check(lib().cyc_kernel_cfg_info(int(idx), ctypes.byref(fl), ctypes.byref(tw), ctypes.byref(aw),
                                     ctypes.byref(nt), ctypes.byref(name)), "cyc_kernel_cfg_info")
    return dict(index=int(idx), flags=fl.value, lag_tile=tw.value, alpha_tile=aw.value,
                threads=nt.value, name=name.value.decode())


def cyc_set_kernel_cfg(state, idx: int):
    _check(lib().cyc_set_kernel_cfg(state, int(idx)), "cyc_set_kernel_cfg")


def cyc_autotune(n_alpha: int, n_lag: int, flags: int = 0, stream=None) -> dict:
    best, ms = ctypes.c_int32(-1), ctypes.c_double(0.0)
    _check(lib().cyc_autotune(int(n_alpha), int(n_lag), int(flags), ctypes.byref(best), ctypes.byref(ms),
                              _stream_handle(stream)), "cyc_autotune")
    return dict(cfg=best.value, ms_per_push=ms.value, name=cyc_kernel_cfg_info(best.value)["name"])


# ----------------------------------------------------------------------------- convenience wrapper

class CyclicStream:
    """One streaming estimator state on the current GPU."""

    def __init__(self, alphas, n_lag: int, flags: int = 0, stream=None):
        self.alphas = np.asarray(alphas, dtype=np.float64).reshape(-1)
        self.T = int(n_lag)
        self.flags = int(flags)
        self._s = cyc_create(self.alphas, self.T, self.flags, stream)

    def push(self, x, stream=None):
        cyc_push(self._s, x, stream)

    def tables(self):
        """(keeps R, keeps Rc) from the table flags (neither or both flags: both)."""
        r, rc = bool(self.flags & CYC_TBL_R), bool(self.flags & CYC_TBL_RCONJ)
        return (True, True) if r == rc else (r, rc)

    def read(self, stream=None, which=None):
        """Returns (R, Rc, n_used) as new [T, A] complex tensors on the GPU (None for a
        table not asked for; by default every table the state keeps)."""
        import torch
        if which is None:
            which = self.tables()
        dt = torch.complex128 if self.flags & CYC_OUT_C128 else torch.complex64
        shape = (self.T, self.alphas.size)
        R = torch.empty(shape, dtype=dt, device="cuda") if which[0] else None
        Rc = torch.empty(shape, dtype=dt, device="cuda") if which[1] else None
        n = cyc_read(self._s, R, Rc, stream)
        return R, Rc, n

    def reset(self):
        cyc_reset(self._s)

    def query(self) -> dict:
        return cyc_query(self._s)

    def set_kernel_cfg(self, idx: int):
        cyc_set_kernel_cfg(self._s, idx)

    def profile(self, enable: bool):
        cyc_profile(self._s, enable)

    def profile_read(self) -> dict:
        return cyc_profile_read(self._s)

    def close(self):
        if self._s is not None:
            cyc_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CrossStream(CyclicStream):
    """Two inputs x, y and lags lag_min .. lag_min + n_lag - 1 (lag m pairs x[k + m] with y[k])."""

    def __init__(self, alphas, lag_min: int, n_lag: int, flags: int = 0, stream=None):
        self.alphas = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).reshape(-1))
        self.T = int(n_lag)
        self.lag_min = int(lag_min)
        self.flags = int(flags)
        out = ctypes.c_void_p()
        _check(lib().cyc_create2(ctypes.byref(out), self.alphas.ctypes.data_as(ctypes.c_void_p), self.alphas.size,
                                 self.lag_min, self.T, self.flags, _stream_handle(stream)), "cyc_create2")
        self._s = out

    def push2(self, x, y, stream=None):
        import torch
        for t in (x, y):
            if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 1:
                raise ValueError("x and y must be contiguous 1-D complex64 CUDA tensors")
        if x.numel() != y.numel():
            raise ValueError("x and y must have the same length")
        _check(lib().cyc_push2(self._s, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                               int(x.numel()), _stream_handle(stream)), "cyc_push2")


class WindowStream(CyclicStream):
    """Estimate over the last n_hops complete hops of `hop` products (phase from the window start)."""

    def __init__(self, alphas, n_lag: int, hop: int, n_hops: int, flags: int = 0, stream=None):
        self.alphas = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).reshape(-1))
        self.T, self.hop, self.n_hops, self.flags = int(n_lag), int(hop), int(n_hops), int(flags)
        out = ctypes.c_void_p()
        _check(lib().cyc_create_window(ctypes.byref(out), self.alphas.ctypes.data_as(ctypes.c_void_p),
                                       self.alphas.size, self.T, self.hop, self.n_hops, self.flags,
                                       _stream_handle(stream)), "cyc_create_window")
        self._s = out


# ----------------------------------------------------------------------------- batches

def cyc_batch_create(alpha_lists, n_lag: int, flags: int = 0, stream=None) -> ctypes.c_void_p:
    lists = [np.asarray(a, dtype=np.float64).reshape(-1) for a in alpha_lists]
    offs = np.zeros(len(lists) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([a.size for a in lists])
    flat = np.ascontiguousarray(np.concatenate(lists)) if lists else np.zeros(0)
    out = ctypes.c_void_p()
    code = lib().cyc_batch_create(ctypes.byref(out), len(lists),
                                  offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  int(n_lag), int(flags), _stream_handle(stream))
    _check(code, "cyc_batch_create")
    return out


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr() if (t is not None and t.numel() > 0) else None
    return arr


def cyc_batch_push(batch, xs, stream=None):
    """xs: one 1-D contiguous complex64 CUDA tensor (or None) per stream."""
    import torch
    for x in xs:
        if x is not None and (x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous()
                              or x.dim() != 1):
            raise ValueError("each x must be a contiguous 1-D complex64 CUDA tensor")
    ns = (ctypes.c_int64 * len(xs))(*[0 if x is None else int(x.numel()) for x in xs])
    _check(lib().cyc_batch_push(batch, _ptr_array(xs), ns, _stream_handle(stream)), "cyc_batch_push")


def cyc_batch_read(batch, Rs=None, Rcs=None, n_streams=None, stream=None):
    n = n_streams if n_streams is not None else len(Rs if Rs is not None else Rcs)
    nu = (ctypes.c_int64 * n)()
    pr = _ptr_array(Rs) if Rs is not None else None
    prc = _ptr_array(Rcs) if Rcs is not None else None
    _check(lib().cyc_batch_read(batch, pr, prc, nu, _stream_handle(stream)), "cyc_batch_read")
    return [int(v) for v in nu]


def cyc_batch_reset(batch):
    _check(lib().cyc_batch_reset(batch), "cyc_batch_reset")


def cyc_batch_destroy(batch):
    lib().cyc_batch_destroy(batch)


def cyc_batch_query(batch) -> dict:
    cfg, rounds, graph = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().cyc_batch_query(batch, ctypes.byref(cfg), ctypes.byref(rounds), ctypes.byref(graph)),
           "cyc_batch_query")
    return dict(kernel_cfg=cfg.value, rounds=rounds.value, graph=bool(graph.value))


class CyclicBatch:
    """Many stream states with a common lag count, advanced together."""

    def __init__(self, alpha_lists, n_lag: int, flags: int = 0, stream=None):
        self.alphas = [np.asarray(a, dtype=np.float64).reshape(-1) for a in alpha_lists]
        self.T = int(n_lag)
        self.flags = int(flags)
        self._b = cyc_batch_create(self.alphas, self.T, self.flags, stream)

    def push(self, xs, stream=None):
        cyc_batch_push(self._b, xs, stream)

    def read(self, stream=None):
        """Returns ([R_s], [Rc_s], [n_used_s]) as new [T, A_s] tensors on the GPU."""
        import torch
        dt = torch.complex128 if self.flags & CYC_OUT_C128 else torch.complex64
        Rs = [torch.empty((self.T, a.size), dtype=dt, device="cuda") for a in self.alphas]
        Rcs = [torch.empty_like(r) for r in Rs]
        nu = cyc_batch_read(self._b, Rs, Rcs, stream=stream)
        return Rs, Rcs, nu

    def reset(self):
        cyc_batch_reset(self._b)

    def query(self) -> dict:
        return cyc_batch_query(self._b)

    def profile(self, enable: bool):
        _check(lib().cyc_batch_profile(self._b, 1 if enable else 0), "cyc_batch_profile")

    def profile_read(self) -> dict:
        ms, n, w = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().cyc_batch_profile_read(self._b, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(w)),
               "cyc_batch_profile_read")
        return dict(total_ms=ms.value, launches=n.value, work=w.value)

    def close(self):
        if self._b is not None:
            cyc_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- uniform grids

class GridStream:
    """Tables on the whole grid alpha_k = alpha0 + k / n_alpha by fold and FFT (n_alpha a power of two)."""

    def __init__(self, alpha0: float, n_alpha: int, n_lag: int, flags: int = 0, stream=None, lag_min=None):
        """lag_min given: two inputs (push2) and lags lag_min .. lag_min + n_lag - 1."""
        self.alpha0, self.A, self.T, self.flags = float(alpha0), int(n_alpha), int(n_lag), int(flags)
        self.lag_min = lag_min
        out = ctypes.c_void_p()
        if lag_min is None:
            _check(lib().cyc_grid_create(ctypes.byref(out), self.alpha0, self.A, self.T, self.flags,
                                         _stream_handle(stream)), "cyc_grid_create")
        else:
            _check(lib().cyc_grid_create2(ctypes.byref(out), self.alpha0, self.A, int(lag_min), self.T, self.flags,
                                          _stream_handle(stream)), "cyc_grid_create2")
        self._g = out

    def push2(self, x, y, stream=None):
        import torch
        for t in (x, y):
            if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("x and y must be contiguous complex64 CUDA tensors")
        if x.numel() != y.numel():
            raise ValueError("x and y must have the same length")
        _check(lib().cyc_grid_push2(self._g, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                    int(x.numel()), _stream_handle(stream)), "cyc_grid_push2")

    @property
    def alphas(self) -> np.ndarray:
        return self.alpha0 + np.arange(self.A) / self.A

    def push(self, x, stream=None):
        import torch
        if x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous complex64 CUDA tensor")
        _check(lib().cyc_grid_push(self._g, ctypes.c_void_p(x.data_ptr()), int(x.numel()), _stream_handle(stream)),
               "cyc_grid_push")

    def read_into(self, R=None, Rc=None, stream=None) -> int:
        nu = ctypes.c_int64()
        _check(lib().cyc_grid_read(self._g, _p(R), _p(Rc), ctypes.byref(nu), _stream_handle(stream)),
               "cyc_grid_read")
        return nu.value

    def read(self, stream=None):
        """Returns (R, Rc, n_used) as new [T, A] tensors on the GPU."""
        import torch
        dt = torch.complex128 if self.flags & CYC_OUT_C128 else torch.complex64
        R = torch.empty((self.T, self.A), dtype=dt, device="cuda")
        Rc = torch.empty_like(R)
        n = self.read_into(R, Rc, stream)
        return R, Rc, n

    def reset(self):
        _check(lib().cyc_grid_reset(self._g), "cyc_grid_reset")

    def close(self):
        if self._g is not None:
            lib().cyc_grid_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cyc_scf(R, alphas, lag_min: int, n_freq: int, window: str = "rect", stream=None, noalloc: bool = False,
            out=None):
    """Cyclic spectrum [n_freq, A] (complex64, GPU) of a complex64 [T, A] lag table R on the GPU.

    noalloc: call cyc_scf_noalloc (the library allocates nothing; T*A <= 2^21).
    out: a contiguous complex64 [n_freq, A] CUDA tensor to write (else a new one)."""
    import torch
    if R.dtype != torch.complex64 or not R.is_cuda or not R.is_contiguous() or R.dim() != 2:
        raise ValueError("R must be a contiguous complex64 [T, A] CUDA tensor")
    T, A = R.shape
    al = torch.as_tensor(np.asarray(alphas, dtype=np.float64).reshape(-1), device=R.device)
    if al.numel() != A:
        raise ValueError("one cycle frequency per column")
    if out is None:
        S = torch.empty((int(n_freq), A), dtype=torch.complex64, device=R.device)
    else:
        S = out
        if S.dtype != torch.complex64 or not S.is_cuda or not S.is_contiguous() or tuple(S.shape) != (int(n_freq), A):
            raise ValueError("out must be a contiguous complex64 [n_freq, A] CUDA tensor")
    name = "cyc_scf_noalloc" if noalloc else "cyc_scf"
    _check(getattr(lib(), name)(_p(R), _p(al), A, int(lag_min), T, int(n_freq), {"rect": 0, "hann": 1}[window],
                                _p(S), _stream_handle(stream)), name)
    return S


# ----------------------------------------------------------------------------- cycle-frequency estimation

def cyc_cfe_detect(R, n_used: int, kappa: float = 7.0, exclude_bin: int = -1, max_out: int = 1024, stream=None):
    """Detections on a complex64 [T, A] CUDA table: (bins int32 array ascending, sigma [T, A/64] FP64 tensor)."""
    import torch
    if R.dtype != torch.complex64 or not R.is_cuda or not R.is_contiguous() or R.dim() != 2:
        raise ValueError("R must be a contiguous complex64 [T, A] CUDA tensor")
    T, A = R.shape
    bins = torch.empty(max(int(max_out), 1), dtype=torch.int32, device=R.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=R.device)
    sigma = torch.empty((T, A // 64), dtype=torch.float64, device=R.device)
    _check(lib().cyc_cfe_detect(_p(R), T, A, int(n_used), float(kappa), int(exclude_bin), int(max_out), _p(bins),
                                _p(cnt), _p(sigma), _stream_handle(stream)), "cyc_cfe_detect")
    n = int(cnt.item())
    return bins[:min(n, int(max_out))].cpu().numpy(), sigma, n


def cyc_estimate_cycle_freqs(x, alpha0: float, n_alpha: int, n_lag: int, table: str = "R", kappa: float = 7.0,
                             zoom: int = 16, exclude_zero: bool = True, max_out: int = 1024, stream=None):
    """Cycle-frequency estimates from a 1-D complex64 CUDA tensor of samples: a list of
    (coarse bin, alpha_hat, statistic), ascending in bin, and the total detection count."""
    import torch
    if x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous() or x.dim() != 1:
        raise ValueError("x must be a contiguous 1-D complex64 CUDA tensor")
    ah = np.zeros(max(int(max_out), 1), dtype=np.float64)
    st = np.zeros_like(ah)
    bn = np.zeros(max(int(max_out), 1), dtype=np.int32)
    cnt = ctypes.c_int32(0)
    _check(lib().cyc_estimate_cycle_freqs(_p(x), int(x.numel()), float(alpha0), int(n_alpha), int(n_lag),
                                          {"R": 0, "Rc": 1}[table], float(kappa), int(zoom), 1 if exclude_zero else 0,
                                          int(max_out), ah.ctypes.data_as(ctypes.c_void_p),
                                          st.ctypes.data_as(ctypes.c_void_p), bn.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.byref(cnt), _stream_handle(stream)), "cyc_estimate_cycle_freqs")
    n = min(cnt.value, int(max_out))
    return [(int(bn[i]), float(ah[i]), float(st[i])) for i in range(n)], cnt.value


# ----------------------------------------------------------------------------- learned proposal

WINDOW = 65536
N_COARSE = 1024
FEAT_LEN = 1024


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class ProposalModel:
    """The proposal network (features, forward, gradients, AdamW) on the GPU."""

    def __init__(self, max_batch: int, flags: int = CYC_OP_BF16, stream=None):
        self.max_batch = int(max_batch)
        self.flags = int(flags)
        out = ctypes.c_void_p()
        _check(lib().cyc_model_create(ctypes.byref(out), self.max_batch, self.flags, _stream_handle(stream)),
               "cyc_model_create")
        self._m = out

    @staticmethod
    def num_params() -> int:
        return int(lib().cyc_model_num_params())

    def set_params(self, flat: np.ndarray, stream=None):
        a = np.ascontiguousarray(np.asarray(flat, dtype=np.float32).reshape(-1))
        if a.size != self.num_params():
            raise ValueError("wrong parameter count")
        _check(lib().cyc_model_set_params(self._m, a.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream)),
               "cyc_model_set_params")

    def get_params(self, stream=None) -> np.ndarray:
        a = np.empty(self.num_params(), dtype=np.float32)
        _check(lib().cyc_model_get_params(self._m, a.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream)),
               "cyc_model_get_params")
        return a

    def spectra(self, x, stream=None):
        """x: complex64 CUDA tensor of n*65536 samples -> float tensor [3, n, 1024]."""
        import torch
        n = x.numel() // WINDOW
        feat = torch.empty((3, n, FEAT_LEN), dtype=torch.float32, device=x.device)
        _check(lib().cyc_model_spectra(self._m, _p(x), n, _p(feat), _stream_handle(stream)), "cyc_model_spectra")
        return feat

    def forward(self, feat, stream=None):
        import torch
        n = feat.shape[1]
        prob = torch.empty((n, N_COARSE), dtype=torch.float32, device=feat.device)
        _check(lib().cyc_model_forward(self._m, _p(feat), n, _p(prob), _stream_handle(stream)), "cyc_model_forward")
        return prob

    def gradients(self, feat, labels, stream=None):
        import torch
        g = torch.empty(self.num_params(), dtype=torch.float32, device=feat.device)
        loss = ctypes.c_double()
        _check(lib().cyc_model_gradients(self._m, _p(feat), _p(labels), feat.shape[1], _p(g), ctypes.byref(loss),
                                         _stream_handle(stream)), "cyc_model_gradients")
        return g, loss.value

    def loss(self, feat, labels, stream=None) -> float:
        """Mean BCE of the current parameters (gradients are computed, not returned)."""
        loss = ctypes.c_double()
        _check(lib().cyc_model_gradients(self._m, _p(feat), _p(labels), feat.shape[1], None, ctypes.byref(loss),
                                         _stream_handle(stream)), "cyc_model_gradients")
        return loss.value

    def train_step(self, feat, labels, lr: float, weight_decay: float, stream=None) -> float:
        loss = ctypes.c_double()
        _check(lib().cyc_model_train_step(self._m, _p(feat), _p(labels), feat.shape[1], float(lr),
                                          float(weight_decay), ctypes.byref(loss), _stream_handle(stream)),
               "cyc_model_train_step")
        return loss.value

    def propose(self, x, topk: int = 16, width: int = 2, zero_bin: int = N_COARSE // 2, theta: float = 0.0,
                stream=None):
        """x: complex64 CUDA tensor of n*65536 samples -> (bins int32 [n, 1024] (-1 padded), n_bins int32 [n],
        conf float [n], fallback uint8 [n]) on the GPU."""
        import torch
        n = x.numel() // WINDOW
        bins = torch.empty((n, N_COARSE), dtype=torch.int32, device=x.device)
        nb_ = torch.empty(n, dtype=torch.int32, device=x.device)
        conf = torch.empty(n, dtype=torch.float32, device=x.device)
        fb = torch.empty(n, dtype=torch.uint8, device=x.device)
        _check(lib().cyc_propose(self._m, _p(x), n, int(topk), int(width), int(zero_bin), float(theta), _p(bins),
                                 _p(nb_), _p(conf), _p(fb), _stream_handle(stream)), "cyc_propose")
        return bins, nb_, conf, fb

    @staticmethod
    def save(path: str, params: np.ndarray):
        """Writes an FP32 parameter vector (as from get_params) to a .npy file."""
        np.save(path, np.asarray(params, dtype=np.float32), allow_pickle=False)

    @staticmethod
    def load(path: str) -> np.ndarray:
        """Reads a parameter vector written by save (for set_params)."""
        v = np.load(path, allow_pickle=False)
        if v.dtype != np.float32 or v.ndim != 1 or v.size != ProposalModel.num_params():
            raise ValueError("not a parameter vector of this network")
        return v

    def close(self):
        if self._m is not None:
            lib().cyc_model_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cyc_select(prob, topk: int = 16, width: int = 2, zero_bin: int = N_COARSE // 2, stream=None):
    """Returns (sel uint8 [n, 1024], conf float [n]) on the GPU."""
    import torch
    n = prob.shape[0]
    sel = torch.empty((n, N_COARSE), dtype=torch.uint8, device=prob.device)
    conf = torch.empty(n, dtype=torch.float32, device=prob.device)
    _check(lib().cyc_select(_p(prob), n, int(topk), int(width), int(zero_bin), _p(sel), _p(conf),
                            _stream_handle(stream)), "cyc_select")
    return sel, conf


def cyc_peak_labels(R, Rc, n_coarse: int = N_COARSE, zero_bin: int = N_COARSE // 2, thresh: float = 7.0,
                    stream=None):
    """R, Rc: complex64 CUDA tensors [T, A] (either may be None) -> float labels [n_coarse] on the GPU."""
    import torch
    ref = R if R is not None else Rc
    lab = torch.empty(n_coarse, dtype=torch.float32, device=ref.device)
    _check(lib().cyc_peak_labels(_p(R), _p(Rc), ref.shape[0], ref.shape[1], int(n_coarse), int(zero_bin),
                                 float(thresh), _p(lab), _stream_handle(stream)), "cyc_peak_labels")
    return lab
