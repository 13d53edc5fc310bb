"""Python binding of libsvdphat (SVD-PHAT on MI355X / gfx950).

Argument marshalling only: every step of the localisation runs in the HIP
library.  PyTorch provides device memory and streams; tensors are passed by
``data_ptr()`` and the current HIP stream.  The functions mirror the C ABI
declared in ``include/svdphat.h``; :class:`Plan` wraps them.

The library is built in place by ``paper_1811_11785_amd.build.build()``;
importing this module does not build it, and every call fails loudly if the
shared library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SVDPHAT_LIB") or os.path.join(HERE, "libsvdphat.so")  # (a variant build: testing)

OK, E_INVAL, E_NOMEM, E_DEVICE, E_NUMERIC, E_NODEV, E_UNSUPPORTED, E_IO = 0, -1, -2, -3, -4, -5, -6, -7
KEEP_W, NO_DEDUP = 0x1, 0x2
FP32, BF16, FP16 = 0, 1, 2
RESCORE, HILO, HILO_ALL, NORMALIZED = 0x1, 0x2, 0x4, 0x8
RAGGED_TUNE = 0x1
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16}


class SvdphatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"svdphat error {code}: {msg}")
        self.code = code


class Info(C.Structure):
    _fields_ = [("M", C.c_int32), ("P", C.c_int32), ("B", C.c_int32), ("L", C.c_int32),
                ("Q", C.c_int32), ("n_classes", C.c_int32), ("K", C.c_int32),
                ("K_paper", C.c_int32), ("N", C.c_int32), ("has_w", C.c_int32),
                ("residual", C.c_double), ("sigma1", C.c_double), ("sigmaK", C.c_double),
                ("fro2", C.c_double), ("u_rownorm_max", C.c_double),
                ("device_bytes", C.c_int64), ("input_hash", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

# exported symbols and their C signatures (restype, argtypes)
SIGNATURES = {
    "svdphat_version": (C.c_int, []),
    "svdphat_last_error": (C.c_char_p, []),
    "svdphat_plan_create": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_double,
                                      C.c_double, C.c_int32, C.c_double, C.c_uint32,
                                      C.POINTER(C.c_void_p)]),
    "svdphat_plan_info": (C.c_int, [C.c_void_p, C.POINTER(Info)]),
    "svdphat_plan_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "svdphat_plan_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_void_p)]),
    "svdphat_plan_input_hash": (C.c_uint64, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_double,
                                             C.c_double, C.c_int32, C.c_double, C.c_uint32]),
    "svdphat_proposal_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "svdphat_proposal_load": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_void_p)]),
    "svdphat_plan_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "svdphat_locate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_uint32,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "svdphat_srp_locate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "svdphat_locate_masked": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_uint32,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "svdphat_locate_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_uint32,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "svdphat_noalloc_scratch_bytes": (C.c_int64, []),
    "svdphat_plan_destroy": (None, [C.c_void_p]),
    "svdphat_sync": (C.c_int, [C.c_void_p]),
    "svdphat_stft_frames": (C.c_int64, [C.c_int64, C.c_int32, C.c_int32]),
    "svdphat_peaks": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_void_p, C.c_int32, C.c_float,
                                C.c_void_p, C.c_void_p, C.c_void_p]),
    "svdphat_stft": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_void_p,
                               C.c_void_p]),
    "svdphat_ragged_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_int64),
                                        C.c_uint32, C.c_char_p, C.POINTER(C.c_void_p)]),
    "svdphat_ragged_locate": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32, C.c_void_p]),
    "svdphat_ragged_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "svdphat_ragged_destroy": (None, [C.c_void_p]),
    "svdphat_proposal_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_uint64,
                                          C.POINTER(C.c_void_p)]),
    "svdphat_proposal_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_float,
                                              C.POINTER(C.c_float), C.c_void_p]),
    "svdphat_proposal_locate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_float,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "svdphat_proposal_nparams": (C.c_int64, [C.c_void_p]),
    "svdphat_proposal_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "svdphat_proposal_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                        C.POINTER(C.c_float)]),
    "svdphat_proposal_cells": (C.c_int, [C.c_void_p, C.c_void_p]),
    "svdphat_proposal_features": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "svdphat_proposal_apply_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_float]),
    "svdphat_proposal_destroy": (None, [C.c_void_p]),
    "svdphat_timing_enable": (C.c_int, [C.c_int]),
    "svdphat_timing_reset": (C.c_int, []),
    "svdphat_timing_read": (C.c_int, [C.c_int32, C.c_char_p, C.c_int32, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64)]),
}


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1811_11785_amd.build.build() first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise SvdphatError(code, lib().svdphat_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------ C ABI mirror
def svdphat_version() -> int:
    return lib().svdphat_version()


def svdphat_plan_create(mics, grid, fs, c, N, delta, flags=0):
    mics = np.ascontiguousarray(mics, dtype=np.float64)
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    out = C.c_void_p()
    _check(lib().svdphat_plan_create(mics.ctypes.data, mics.shape[0], grid.ctypes.data,
                                     grid.shape[0], float(fs), float(c), int(N), float(delta),
                                     int(flags), C.byref(out)))
    return out


def svdphat_plan_info(plan) -> dict:
    info = Info()
    _check(lib().svdphat_plan_info(plan, C.byref(info)))
    return info.as_dict()


def svdphat_plan_export(plan):
    info = svdphat_plan_info(plan)
    Q, L, K = info["Q"], info["L"], info["K"]
    sig = np.zeros(min(Q, L))
    U = np.zeros((Q, K, 2))
    V = np.zeros((L, K, 2))
    rep = np.zeros(Q, dtype=np.int32)
    _check(lib().svdphat_plan_export(plan, sig.ctypes.data, U.ctypes.data, V.ctypes.data,
                                     rep.ctypes.data))
    return sig, U[..., 0] + 1j * U[..., 1], V[..., 0] + 1j * V[..., 1], rep


def svdphat_locate(plan, X, precision, mode, doa, power, yhat=None, margin=None, y_opt=None,
                   stream=None):
    _check(lib().svdphat_locate(plan, _ptr(X), X.shape[0], precision, mode, _ptr(doa), _ptr(power),
                                _ptr(yhat), _ptr(margin), _ptr(y_opt), _stream(stream)))


def svdphat_locate_noalloc(plan, X, precision, mode, doa, power, yhat=None, margin=None, stream=None):
    _check(lib().svdphat_locate_noalloc(plan, _ptr(X), X.shape[0], precision, mode, _ptr(doa), _ptr(power),
                                        _ptr(yhat), _ptr(margin), _stream(stream)))


def svdphat_noalloc_scratch_bytes() -> int:
    return lib().svdphat_noalloc_scratch_bytes()


def svdphat_srp_locate(plan, X, doa, power, y_opt=None, stream=None):
    _check(lib().svdphat_srp_locate(plan, _ptr(X), X.shape[0], _ptr(doa), _ptr(power), _ptr(y_opt),
                                    _stream(stream)))


def svdphat_plan_destroy(plan):
    lib().svdphat_plan_destroy(plan)


def svdphat_sync(stream=None):
    _check(lib().svdphat_sync(_stream(stream)))


def svdphat_stft(pcm, N, hop, X, stream=None):
    """pcm: float32 CUDA tensor [M, T] (row stride ld = pcm.stride(0));
    X: complex64 CUDA tensor [F, M, N/2+1] with F = stft_frames(T, N, hop)."""
    M, T = pcm.shape
    assert pcm.stride(1) == 1
    _check(lib().svdphat_stft(_ptr(pcm), M, T, pcm.stride(0), N, hop, _ptr(X), _stream(stream)))


def peaks(y, dirs, n, cos_sep, stream=None):
    """The n strongest separated directions per frame: y float32 CUDA [F, Q]
    (row stride y.stride(0)), dirs float32 CUDA [Q, 3] unit vectors.  Returns
    (idx int32 [F, n], val float32 [F, n]) on y's device."""
    import torch
    F, Q = y.shape
    assert y.stride(1) == 1 and dirs.is_contiguous() and dirs.shape == (Q, 3)
    idx = torch.empty((F, n), dtype=torch.int32, device=y.device)
    val = torch.empty((F, n), dtype=torch.float32, device=y.device)
    _check(lib().svdphat_peaks(_ptr(y), F, Q, y.stride(0), _ptr(dirs), n, float(cos_sep), _ptr(idx), _ptr(val),
                               _stream(stream)))
    return idx, val


def stft_frames(T, N, hop):
    return lib().svdphat_stft_frames(T, N, hop)


def stft(pcm, N=512, hop=256, stream=None):
    """STFT frames [F, M, N/2+1] (complex64, on pcm's device) of the
    microphone signals pcm [M, T] (float32 CUDA tensor), sine window."""
    import torch
    assert pcm.is_cuda and pcm.dtype == torch.float32
    F = stft_frames(pcm.shape[1], N, hop)
    if F < 0:
        raise SvdphatError(E_INVAL, "invalid STFT sizes")
    X = torch.empty((F, pcm.shape[0], N // 2 + 1), dtype=torch.complex64, device=pcm.device)
    svdphat_stft(pcm, N, hop, X, stream)
    return X


def svdphat_timing_enable(enable, counts: bool = False):
    """enable: kernel timing on/off; counts: event counters (not with timing)."""
    _check(lib().svdphat_timing_enable((1 if enable else 0) | (2 if counts else 0)))


def svdphat_timing_reset():
    _check(lib().svdphat_timing_reset())


def svdphat_timing_read() -> dict:
    """{kernel name: (total ms, launches)} of the instrumented launches."""
    out = {}
    i = 0
    buf = C.create_string_buffer(64)
    while True:
        ms, n = C.c_double(), C.c_int64()
        if lib().svdphat_timing_read(i, buf, 64, C.byref(ms), C.byref(n)) != OK:
            break
        out[buf.value.decode()] = (ms.value, n.value)
        i += 1
    return out


def svdphat_ragged_create(plans, max_frames, flags=0, tune_cache=None):
    n = len(plans)
    arr = (C.c_void_p * n)(*[p.value if isinstance(p, C.c_void_p) else p for p in plans])
    mf = (C.c_int64 * n)(*[int(v) for v in max_frames])
    out = C.c_void_p()
    _check(lib().svdphat_ragged_create(arr, n, mf, int(flags),
                                       None if tune_cache is None else str(tune_cache).encode(),
                                       C.byref(out)))
    return out


def svdphat_ragged_locate(ragged, Xs, doas, powers, stream=None, precision=FP16):
    n = len(Xs)
    X = (C.c_void_p * n)(*[x.data_ptr() if x.shape[0] else None for x in Xs])
    F = (C.c_int64 * n)(*[x.shape[0] for x in Xs])
    D = (C.c_void_p * n)(*[d.data_ptr() if d.numel() else None for d in doas])
    P = (C.c_void_p * n)(*[p.data_ptr() if p.numel() else None for p in powers])
    _check(lib().svdphat_ragged_locate(ragged, X, F, D, P, precision, _stream(stream)))


def svdphat_ragged_info(ragged):
    t, c = C.c_int64(), C.c_int64()
    _check(lib().svdphat_ragged_info(ragged, C.byref(t), C.byref(c)))
    return t.value, c.value


def svdphat_ragged_destroy(ragged):
    lib().svdphat_ragged_destroy(ragged)


# ------------------------------------------------------------ convenience
def svdphat_plan_input_hash(mics, grid, fs, c, N, delta, flags=0) -> int:
    mics = np.ascontiguousarray(mics, dtype=np.float64)
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    return lib().svdphat_plan_input_hash(mics.ctypes.data, mics.shape[0], grid.ctypes.data, grid.shape[0],
                                         float(fs), float(c), int(N), float(delta), int(flags))


class Plan:
    """Offline plan (Algorithm 1, offline) and online search on device tensors."""

    def __init__(self, mics, grid, fs=16000.0, c=343.0, N=512, delta=1e-5, keep_w=False,
                 dedup=True, _handle=None):
        if _handle is None:
            flags = (KEEP_W if keep_w else 0) | (0 if dedup else NO_DEDUP)
            _handle = svdphat_plan_create(mics, grid, fs, c, N, delta, flags)
        self._h = _handle
        self.info = svdphat_plan_info(self._h)

    def save(self, path):
        _check(lib().svdphat_plan_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path):
        out = C.c_void_p()
        _check(lib().svdphat_plan_load(os.fsencode(path), C.byref(out)))
        return cls(None, None, _handle=out)

    @property
    def handle(self):
        return self._h

    def locate(self, X, precision="fp32", rescore=True, hilo=False, want_y=False, stream=None, hilo_all=False,
               normalized=False, mask=None):
        """X: complex64 CUDA tensor [F, M, N/2+1].  Returns a dict of device
        tensors doa (int32), power, yhat, margin (f32) and y ([F, Q]) if asked.
        hilo_all: the hi/lo pass for every frame (16-bit precisions);
        normalized: the search of eq. (15) instead of eq. (14); mask: uint8
        CUDA tensor [F, N/2+1], the binary time-frequency mask (0 drops a bin)."""
        import torch
        assert X.is_cuda and X.dtype == torch.complex64 and X.is_contiguous()
        F = X.shape[0]
        dev = X.device
        doa = torch.empty(F, dtype=torch.int32, device=dev)
        power = torch.empty(F, dtype=torch.float32, device=dev)
        yhat = torch.empty(F, dtype=torch.float32, device=dev)
        margin = torch.empty(F, dtype=torch.float32, device=dev)
        y = torch.empty((F, self.info["Q"]), dtype=torch.float32, device=dev) if want_y else None
        mode = ((RESCORE if rescore else 0) | (HILO if hilo else 0) | (HILO_ALL if hilo_all else 0)
                | (NORMALIZED if normalized else 0))
        if mask is None:
            svdphat_locate(self._h, X, PRECISIONS[precision], mode, doa, power, yhat, margin, y, stream)
        else:
            assert mask.is_cuda and mask.dtype == torch.uint8 and mask.is_contiguous()
            assert tuple(mask.shape) == (F, self.info["B"])
            _check(lib().svdphat_locate_masked(self._h, _ptr(X), F, _ptr(mask), PRECISIONS[precision], mode,
                                               _ptr(doa), _ptr(power), _ptr(yhat), _ptr(margin), _ptr(y),
                                               _stream(stream)))
        out = dict(doa=doa, power=power, yhat=yhat, margin=margin)
        if want_y:
            out["y"] = y
        return out

    def srp_locate(self, X, want_y=False, stream=None):
        import torch
        F = X.shape[0]
        dev = X.device
        doa = torch.empty(F, dtype=torch.int32, device=dev)
        power = torch.empty(F, dtype=torch.float32, device=dev)
        y = torch.empty((F, self.info["Q"]), dtype=torch.float32, device=dev) if want_y else None
        svdphat_srp_locate(self._h, X, doa, power, y, stream)
        out = dict(doa=doa, power=power)
        if want_y:
            out["y"] = y
        return out

    def export(self):
        return svdphat_plan_export(self._h)

    def close(self):
        if self._h is not None:
            svdphat_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ragged:
    """Many plans located together in one graph launch (FP16 + rescoring)."""

    def __init__(self, plans, max_frames, tune=False, tune_cache=None):
        self.plans = list(plans)   # keep the plans alive
        self._h = svdphat_ragged_create([p.handle for p in self.plans], max_frames,
                                        RAGGED_TUNE if tune else 0, tune_cache)

    def locate(self, Xs, stream=None):
        import torch
        doas = [torch.empty(x.shape[0], dtype=torch.int32, device=x.device) for x in Xs]
        powers = [torch.empty(x.shape[0], dtype=torch.float32, device=x.device) for x in Xs]
        svdphat_ragged_locate(self._h, Xs, doas, powers, stream)
        return doas, powers

    def info(self):
        return svdphat_ragged_info(self._h)

    def close(self):
        if self._h is not None:
            svdphat_ragged_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Proposal:
    """Learned coarse-cell proposal over a fine plan (see svdphat.h)."""

    def __init__(self, plan, coarse, hidden=256, seed=0, _handle=None):
        self.plan = plan
        if _handle is None:
            coarse = np.ascontiguousarray(coarse, dtype=np.float64)
            self.C = coarse.shape[0]
            out = C.c_void_p()
            _check(lib().svdphat_proposal_create(plan.handle, coarse.ctypes.data, self.C, hidden, seed,
                                                 C.byref(out)))
            self._h = out
        else:
            self._h = _handle
            self.C = coarse

    def save(self, path):
        _check(lib().svdphat_proposal_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, plan, path):
        """A proposal saved over a plan with the same inputs as `plan`."""
        out = C.c_void_p()
        _check(lib().svdphat_proposal_load(plan.handle, os.fsencode(path), C.byref(out)))
        obj = cls(plan, None, _handle=out)
        obj.C = None
        return obj

    def train_step(self, X, lr=1e-3, stream=None):
        loss = C.c_float()
        _check(lib().svdphat_proposal_train_step(self._h, _ptr(X), X.shape[0], lr, C.byref(loss),
                                                 _stream(stream)))
        return loss.value

    def locate(self, X, topk=8, conf_min=0.5, stream=None):
        import torch
        F = X.shape[0]
        doa = torch.empty(F, dtype=torch.int32, device=X.device)
        power = torch.empty(F, dtype=torch.float32, device=X.device)
        fell = torch.empty(F, dtype=torch.uint8, device=X.device)
        _check(lib().svdphat_proposal_locate(self._h, _ptr(X), F, topk, conf_min, _ptr(doa), _ptr(power),
                                             _ptr(fell), _stream(stream)))
        return dict(doa=doa, power=power, fell_back=fell)

    def nparams(self):
        return lib().svdphat_proposal_nparams(self._h)

    def get_params(self):
        buf = np.zeros(self.nparams(), dtype=np.float32)
        _check(lib().svdphat_proposal_params(self._h, buf.ctypes.data, buf.size, 0))
        return buf

    def set_params(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.float32)
        _check(lib().svdphat_proposal_params(self._h, buf.ctypes.data, buf.size, 1))

    def grad(self, features, labels):
        features = np.ascontiguousarray(features, dtype=np.float32)
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        g = np.zeros(self.nparams(), dtype=np.float32)
        loss = C.c_float()
        _check(lib().svdphat_proposal_grad(self._h, features.ctypes.data, labels.ctypes.data,
                                           features.shape[0], g.ctypes.data, C.byref(loss)))
        return loss.value, g

    def features(self, X, stream=None):
        """Network input [F, 2K] (float32 device tensor) of device frames X."""
        import torch
        F = X.shape[0]
        out = torch.empty((F, 2 * self.plan.info["K"]), dtype=torch.float32, device=X.device)
        _check(lib().svdphat_proposal_features(self._h, _ptr(X), F, _ptr(out), _stream(stream)))
        return out

    def apply_grad(self, grad, lr):
        """One Adam step with the given mean gradient (host, parameter layout)."""
        grad = np.ascontiguousarray(grad, dtype=np.float32)
        _check(lib().svdphat_proposal_apply_grad(self._h, grad.ctypes.data, grad.size, lr))

    def cells(self):
        out = np.zeros(self.plan.info["Q"], dtype=np.int32)
        _check(lib().svdphat_proposal_cells(self._h, out.ctypes.data))
        return out

    def close(self):
        if self._h is not None:
            lib().svdphat_proposal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
