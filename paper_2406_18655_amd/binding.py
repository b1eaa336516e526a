"""Thin ctypes binding over libqlsd's C ABI (include/qlsd.h).

Argument marshalling only: torch supplies device memory and the current stream;
every decoding step runs in the HIP kernels.  Loading fails loudly when the
library has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqlsd.so")

QLSD_OK = 0
ST_BP_CONVERGED, ST_LSD_RUN, ST_UNSAT, ST_BAD_LLR, ST_OVERFLOW = 1, 2, 4, 8, 16
FLAG_NO_EARLY_EXIT = 1
FLAG_STAGE_TIMING = 2
FLAG_SEPARATE_LSD = 4
FLAG_OSD0_POST = 8

# every symbol include/qlsd.h declares
EXPORTS = ["qlsd_code_create", "qlsd_decoder_create", "qlsd_decode", "qlsd_decode_static", "qlsd_bp", "qlsd_lsd",
           "qlsd_osd0", "qlsd_osd_cs", "qlsd_lsd_stats", "qlsd_error_clusters",
           "qlsd_decoder_stage_ms", "qlsd_decoder_set_stage_timing", "qlsd_decoder_tune",
           "qlsd_decoder_set_lsd_capacity", "qlsd_decoder_set_lsd_schedule", "qlsd_sync", "qlsd_last_error",
           "qlsd_decoder_destroy",
           "qlsd_code_destroy"]

INFO_DTYPE = np.dtype([("status", np.uint8), ("reserved", np.uint8), ("bp_iters", np.int16),
                       ("n_clusters", np.int16), ("rounds", np.int16), ("max_cluster_cols", np.int32)])
assert INFO_DTYPE.itemsize == 12


class QlsdParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("ms_scaling", ctypes.c_float),
                ("lsd_order", ctypes.c_int32), ("osd_method", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("osd_order", ctypes.c_int32)]


OSD_E, OSD_CS = 0, 1
LSD_PER_COLUMN, LSD_CLUSTER_BATCHED = 0, 1


class QlsdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qlsd status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Loads libqlsd.so (built by paper_2406_18655_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built: run paper_2406_18655_amd/build.py (no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.qlsd_code_create.argtypes = [I32, I32, I64, P, P, ctypes.POINTER(P)]
        L.qlsd_decoder_create.argtypes = [P, ctypes.POINTER(QlsdParams), P, I32, ctypes.POINTER(P)]
        L.qlsd_decode.argtypes = [P, P, I32, P, P, P]
        L.qlsd_decode_static.argtypes = [P, P, I32, P, P, P]
        L.qlsd_bp.argtypes = [P, P, I32, P, P, P, P]
        L.qlsd_lsd.argtypes = [P, P, P, I32, P, P, P]
        L.qlsd_osd0.argtypes = [P, P, P, I32, P, P, P]
        L.qlsd_osd_cs.argtypes = [P, P, P, I32, I32, P, P, P]
        L.qlsd_lsd_stats.argtypes = [P, P, P, I32, P, P, P, P]
        L.qlsd_error_clusters.argtypes = [P, P, I32, P, P]
        L.qlsd_decoder_stage_ms.argtypes = [P, P, P]
        L.qlsd_decoder_set_stage_timing.argtypes = [P, I32]
        L.qlsd_decoder_tune.argtypes = [P, P, I32, I32, P, P, I32]
        L.qlsd_decoder_set_lsd_capacity.argtypes = [P, I32]
        L.qlsd_decoder_set_lsd_schedule.argtypes = [P, I32]
        L.qlsd_sync.argtypes = [P]
        L.qlsd_last_error.restype = ctypes.c_char_p
        L.qlsd_decoder_destroy.argtypes = [P]
        L.qlsd_code_destroy.argtypes = [P]
        for fn in ("qlsd_code_create", "qlsd_decoder_create", "qlsd_decode", "qlsd_decode_static", "qlsd_bp", "qlsd_lsd",
                   "qlsd_osd0", "qlsd_osd_cs", "qlsd_lsd_stats", "qlsd_error_clusters",
                   "qlsd_decoder_stage_ms", "qlsd_decoder_set_stage_timing", "qlsd_decoder_tune",
                   "qlsd_decoder_set_lsd_capacity", "qlsd_decoder_set_lsd_schedule", "qlsd_sync"):
            getattr(L, fn).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != QLSD_OK:
        raise QlsdError(st, lib().qlsd_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device pointer of a tensor whose memory is the dense row-major layout the ABI expects."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to libqlsd must be contiguous (row-major)")
    return t.data_ptr()


def _need(t, shape, dtype_name: str, what: str, optional: bool = False):
    """The ABI takes raw device pointers and trusts their sizes: check every tensor here."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{what} is required")
    if str(t.dtype) != f"torch.{dtype_name}" or not t.is_cuda or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must be a {dtype_name} CUDA tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


def _stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream


def csr_of(H: np.ndarray):
    H = np.asarray(H, dtype=np.uint8)
    rows, cols = np.nonzero(H)
    row_ptr = np.zeros(H.shape[0] + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32)


class Code:
    """qlsd_code: H uploaded once to the current HIP device."""

    def __init__(self, m: int, n: int, row_ptr: np.ndarray, col_idx: np.ndarray):
        self.m, self.n = int(m), int(n)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().qlsd_code_create(self.m, self.n, int(rp[-1]), rp.ctypes.data, ci.ctypes.data,
                                      ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_dense(cls, H: np.ndarray) -> "Code":
        rp, ci = csr_of(H)
        return cls(H.shape[0], H.shape[1], rp, ci)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.qlsd_code_destroy(self._h)
            self._h = None


class Decoder:
    """qlsd_decoder: params + priors + device workspace for up to max_batch shots."""

    def __init__(self, code: Code, priors: np.ndarray, max_batch: int, max_iter: int = 30,
                 ms_scaling: float = 0.625, lsd_order: int = 0, flags: int = 0, osd_method: int = OSD_E,
                 osd_order: int = 0):
        self.code = code
        self.max_batch = int(max_batch)
        pri = np.ascontiguousarray(priors, dtype=np.float64)
        if pri.shape != (code.n,):
            raise ValueError("priors must have shape (n,)")
        self.params = QlsdParams(int(max_iter), float(ms_scaling), int(lsd_order), int(osd_method), int(flags),
                                 int(osd_order))
        h = ctypes.c_void_p()
        _check(lib().qlsd_decoder_create(code._h, ctypes.byref(self.params), pri.ctypes.data,
                                         self.max_batch, ctypes.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.qlsd_decoder_destroy(self._h)
            self._h = None

    # -- raw entry points (device pointers, caller-owned outputs) --------------------
    def _check_io(self, syndromes, B, **outs):
        _need(syndromes, (B, self.code.m), "uint8", "syndromes")
        spec = {"corrections": ((B, self.code.n), "uint8"), "hard_out": ((B, self.code.n), "uint8"),
                "llr": ((B, self.code.n), "float32"), "llr_out": ((B, self.code.n), "float32"),
                "info": ((B, 12), "uint8")}
        for name, t in outs.items():
            _need(t, spec[name][0], spec[name][1], name, optional=name in ("info", "hard_out"))

    def decode_into(self, syndromes, corrections, info=None, stream: Optional[int] = None):
        B = syndromes.shape[0]
        self._check_io(syndromes, B, corrections=corrections, info=info)
        _check(lib().qlsd_decode(self._h, _ptr(syndromes), B, _ptr(corrections), _ptr(info),
                                 _stream() if stream is None else stream))

    def decode_static_into(self, syndromes, corrections, info=None, stream: Optional[int] = None):
        """qlsd_decode_static: the same decode with its scratch in the library's static array."""
        B = syndromes.shape[0]
        self._check_io(syndromes, B, corrections=corrections, info=info)
        _check(lib().qlsd_decode_static(self._h, _ptr(syndromes), B, _ptr(corrections), _ptr(info),
                                        _stream() if stream is None else stream))

    def bp_into(self, syndromes, llr_out, hard_out=None, info=None, stream: Optional[int] = None):
        B = syndromes.shape[0]
        self._check_io(syndromes, B, llr_out=llr_out, hard_out=hard_out, info=info)
        _check(lib().qlsd_bp(self._h, _ptr(syndromes), B, _ptr(llr_out), _ptr(hard_out), _ptr(info),
                             _stream() if stream is None else stream))

    def lsd_into(self, syndromes, llr, corrections, info=None, stream: Optional[int] = None):
        B = syndromes.shape[0]
        self._check_io(syndromes, B, llr=llr, corrections=corrections, info=info)
        _check(lib().qlsd_lsd(self._h, _ptr(syndromes), _ptr(llr), B, _ptr(corrections), _ptr(info),
                              _stream() if stream is None else stream))

    def osd0_into(self, syndromes, llr, corrections, info=None, stream: Optional[int] = None):
        B = syndromes.shape[0]
        self._check_io(syndromes, B, llr=llr, corrections=corrections, info=info)
        _check(lib().qlsd_osd0(self._h, _ptr(syndromes), _ptr(llr), B, _ptr(corrections), _ptr(info),
                               _stream() if stream is None else stream))

    def osd_cs_into(self, syndromes, llr, order: int, corrections, info=None, stream: Optional[int] = None):
        B = syndromes.shape[0]
        self._check_io(syndromes, B, llr=llr, corrections=corrections, info=info)
        _check(lib().qlsd_osd_cs(self._h, _ptr(syndromes), _ptr(llr), B, int(order), _ptr(corrections), _ptr(info),
                                 _stream() if stream is None else stream))

    def sync(self):
        _check(lib().qlsd_sync(self._h))

    def tune(self, syndromes, reps: int = 5, stream: Optional[int] = None) -> str:
        """Autotune launch shapes on a sample batch (include/qlsd.h); returns the timing report."""
        self._check_io(syndromes, syndromes.shape[0])
        buf = ctypes.create_string_buffer(8192)
        _check(lib().qlsd_decoder_tune(self._h, _ptr(syndromes), syndromes.shape[0], int(reps),
                                       _stream() if stream is None else stream, buf, len(buf)))
        return buf.value.decode()

    def set_lsd_capacity(self, local_rows: int):
        """LSD capacity tier: 64, 128 or 256 local rows per wavefront, shots beyond it finished by
        the overflow kernels (include/qlsd.h); outputs do not depend on it."""
        _check(lib().qlsd_decoder_set_lsd_capacity(self._h, int(local_rows)))

    def set_lsd_schedule(self, schedule: int):
        """LSD_PER_COLUMN or LSD_CLUSTER_BATCHED (256-row kernel only; include/qlsd.h); outputs
        do not depend on it."""
        _check(lib().qlsd_decoder_set_lsd_schedule(self._h, int(schedule)))

    def stage_ms(self):
        """(bp_ms, lsd_ms) of the last decode call made with stage events on (needs FLAG_STAGE_TIMING)."""
        a, b = ctypes.c_float(), ctypes.c_float()
        _check(lib().qlsd_decoder_stage_ms(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_stage_timing(self, enable: bool):
        """Stage events on or off for later decode calls (a FLAG_STAGE_TIMING decoder starts with them on)."""
        _check(lib().qlsd_decoder_set_stage_timing(self._h, 1 if enable else 0))

    # -- torch conveniences ----------------------------------------------------------
    def _prep(self, syndromes):
        import torch
        s = syndromes
        if not s.is_cuda or s.dtype != torch.uint8 or s.dim() != 2 or s.shape[1] != self.code.m:
            raise ValueError("syndromes must be a uint8 CUDA tensor [B, m]")
        return s.contiguous()

    def decode(self, syndromes, want_info: bool = False):
        import torch
        s = self._prep(syndromes)
        B = s.shape[0]
        corr = torch.empty((B, self.code.n), dtype=torch.uint8, device=s.device)
        info = torch.empty((B, 12), dtype=torch.uint8, device=s.device) if want_info else None
        self.decode_into(s, corr, info)
        return (corr, info) if want_info else corr

    def decode_static(self, syndromes, want_info: bool = False):
        import torch
        s = self._prep(syndromes)
        B = s.shape[0]
        corr = torch.empty((B, self.code.n), dtype=torch.uint8, device=s.device)
        info = torch.empty((B, 12), dtype=torch.uint8, device=s.device) if want_info else None
        self.decode_static_into(s, corr, info)
        return (corr, info) if want_info else corr

    def bp(self, syndromes, want_info: bool = True):
        import torch
        s = self._prep(syndromes)
        B = s.shape[0]
        llr = torch.empty((B, self.code.n), dtype=torch.float32, device=s.device)
        hard = torch.empty((B, self.code.n), dtype=torch.uint8, device=s.device)
        info = torch.empty((B, 12), dtype=torch.uint8, device=s.device) if want_info else None
        self.bp_into(s, llr, hard, info)
        return llr, hard, info

    def lsd(self, syndromes, llr, want_info: bool = True):
        import torch
        s = self._prep(syndromes)
        B = s.shape[0]
        if llr.dtype != torch.float32 or tuple(llr.shape) != (B, self.code.n) or not llr.is_cuda:
            raise ValueError("llr must be a float32 CUDA tensor [B, n]")
        corr = torch.empty((B, self.code.n), dtype=torch.uint8, device=s.device)
        info = torch.empty((B, 12), dtype=torch.uint8, device=s.device) if want_info else None
        self.lsd_into(s, llr.contiguous(), corr, info)
        return corr, info

    def lsd_stats(self, syndromes, llr):
        """LSD on llr -> (corrections, info, cluster stats int32 [B, 4]: nu, kappa, total, sum of squares)."""
        import torch
        s = self._prep(syndromes)
        B = s.shape[0]
        if llr.dtype != torch.float32 or tuple(llr.shape) != (B, self.code.n) or not llr.is_cuda:
            raise ValueError("llr must be a float32 CUDA tensor [B, n]")
        corr = torch.empty((B, self.code.n), dtype=torch.uint8, device=s.device)
        info = torch.empty((B, 12), dtype=torch.uint8, device=s.device)
        stats = torch.empty((B, 4), dtype=torch.int32, device=s.device)
        _check(lib().qlsd_lsd_stats(self._h, _ptr(s), _ptr(llr.contiguous()), B, _ptr(corr), _ptr(info), _ptr(stats),
                                    _stream()))
        return corr, info, stats

    def osd0(self, syndromes, llr, want_info: bool = True):
        import torch
        s = self._prep(syndromes)
        B = s.shape[0]
        if llr.dtype != torch.float32 or tuple(llr.shape) != (B, self.code.n) or not llr.is_cuda:
            raise ValueError("llr must be a float32 CUDA tensor [B, n]")
        corr = torch.empty((B, self.code.n), dtype=torch.uint8, device=s.device)
        info = torch.empty((B, 12), dtype=torch.uint8, device=s.device) if want_info else None
        self.osd0_into(s, llr.contiguous(), corr, info)
        return corr, info

    def osd_cs(self, syndromes, llr, order: int, want_info: bool = True):
        """Global OSD-CS of the given order (qlsd_osd_cs) on float32 [B, n] soft information."""
        import torch
        s = self._prep(syndromes)
        B = s.shape[0]
        if llr.dtype != torch.float32 or tuple(llr.shape) != (B, self.code.n) or not llr.is_cuda:
            raise ValueError("llr must be a float32 CUDA tensor [B, n]")
        corr = torch.empty((B, self.code.n), dtype=torch.uint8, device=s.device)
        info = torch.empty((B, 12), dtype=torch.uint8, device=s.device) if want_info else None
        self.osd_cs_into(s, llr.contiguous(), int(order), corr, info)
        return corr, info


def error_clusters(code: Code, errors):
    """Optimal factorization of each error (qlsd_error_clusters) -> int32 [B, 4] device tensor:
    nu, kappa, total faults, sum of squared cluster sizes."""
    import torch
    B = errors.shape[0]
    _need(errors, (B, code.n), "uint8", "errors")
    out = torch.empty((B, 4), dtype=torch.int32, device=errors.device)
    _check(lib().qlsd_error_clusters(code._h, _ptr(errors), B, _ptr(out), _stream()))
    return out


def mu_from_fraction(n: int, fraction: float) -> int:
    """LSD-mu growth steps as a fraction of the faults (Appendix D's parametrisation): round(f n)."""
    return int(max(0, round(fraction * n)))


def parse_info(info) -> np.ndarray:
    """uint8 tensor/array [B, 12] -> structured numpy array with INFO_DTYPE fields."""
    a = info.cpu().numpy() if hasattr(info, "cpu") else np.asarray(info)
    return np.ascontiguousarray(a).view(INFO_DTYPE).reshape(-1)


# --------------------------------------------------------------------------- sampler
SAMPLE_EXPORTS = ["qlsd_sampler_create", "qlsd_sample", "qlsd_syndromes", "qlsd_failures", "qlsd_sampler_destroy"]


def _sample_lib():
    L = lib()
    if not getattr(L, "_sample_ready", False):
        P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.qlsd_sampler_create.argtypes = [P, P, I32, P, P, ctypes.POINTER(P)]
        L.qlsd_sample.argtypes = [P, U64, I64, I32, P, P, P]
        L.qlsd_syndromes.argtypes = [P, P, I32, P, P]
        L.qlsd_failures.argtypes = [P, P, P, I32, P, P]
        L.qlsd_sampler_destroy.argtypes = [P]
        for fn in SAMPLE_EXPORTS[:-1]:
            getattr(L, fn).restype = ctypes.c_int
        L._sample_ready = True
    return L


class Sampler:
    """qlsd_sampler: the library's Philox4x64-10 code-capacity sampler (include/qlsd_sample.h).
    Shots (seed, start .. start+B-1) equal the host generator's (workloads.sample) bit for bit."""

    def __init__(self, code: Code, priors: np.ndarray, logicals: Optional[np.ndarray] = None):
        self.code = code
        pri = np.ascontiguousarray(priors, dtype=np.float64)
        if pri.shape != (code.n,):
            raise ValueError("priors must have shape (n,)")
        k = 0
        self._lrp = np.zeros(1, dtype=np.int32)
        self._lci = np.zeros(1, dtype=np.int32)
        if logicals is not None and len(logicals):
            L = np.asarray(logicals, dtype=np.uint8)
            k = L.shape[0]
            self._lrp, self._lci = csr_of(L)
        h = ctypes.c_void_p()
        _check(_sample_lib().qlsd_sampler_create(code._h, pri.ctypes.data, k, self._lrp.ctypes.data,
                                                 self._lci.ctypes.data, ctypes.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.qlsd_sampler_destroy(self._h)
            self._h = None

    def sample_into(self, seed: int, start: int, errors, syndromes=None, stream: Optional[int] = None):
        B = errors.shape[0]
        _need(errors, (B, self.code.n), "uint8", "errors")
        _need(syndromes, (B, self.code.m), "uint8", "syndromes", optional=True)
        _check(_sample_lib().qlsd_sample(self._h, int(seed) & (2 ** 64 - 1), int(start), B, _ptr(errors),
                                         _ptr(syndromes), _stream() if stream is None else stream))

    def syndromes_into(self, x, out, stream: Optional[int] = None):
        B = x.shape[0]
        _need(x, (B, self.code.n), "uint8", "x")
        _need(out, (B, self.code.m), "uint8", "syndromes")
        _check(_sample_lib().qlsd_syndromes(self._h, _ptr(x), B, _ptr(out), _stream() if stream is None else stream))

    def failures_into(self, errors, corrections, out, stream: Optional[int] = None):
        B = errors.shape[0]
        _need(errors, (B, self.code.n), "uint8", "errors")
        _need(corrections, (B, self.code.n), "uint8", "corrections")
        _need(out, (B,), "uint8", "fail")
        _check(_sample_lib().qlsd_failures(self._h, _ptr(errors), _ptr(corrections), B, _ptr(out),
                                           _stream() if stream is None else stream))


class DeviceSampler:
    """Bulk shots on the GPU for training, serving pools and scoring: the library's sampler with
    device tensors in and out.  sample(shots, seed) returns shots 0..shots-1 of stream `seed`,
    identical to workloads.sample(code, shots, seed); failures and syndromes run in the library."""

    def __init__(self, code_matrix, device="cuda"):
        self.code = code_matrix
        self.bc = Code.from_dense(code_matrix.H)
        self.smp = Sampler(self.bc, code_matrix.priors, code_matrix.logicals)

    def sample(self, shots: int, seed: int, start: int = 0):
        """(errors uint8 [shots,n], syndromes uint8 [shots,m]) as device tensors."""
        import torch
        e = torch.empty((shots, self.code.n), dtype=torch.uint8, device="cuda")
        s = torch.empty((shots, self.code.m), dtype=torch.uint8, device="cuda")
        self.smp.sample_into(seed, start, e, s)
        return e, s

    def failures(self, errors, corrections):
        """bool [shots] on the device: logical failure (or word error without logicals)."""
        import torch
        f = torch.empty((errors.shape[0],), dtype=torch.uint8, device="cuda")
        self.smp.failures_into(errors.contiguous(), corrections.contiguous(), f)
        return f.bool()

    def syndromes(self, corrections):
        import torch
        out = torch.empty((corrections.shape[0], self.code.m), dtype=torch.uint8, device="cuda")
        self.smp.syndromes_into(corrections.contiguous(), out)
        return out


# --------------------------------------------------------------------------- windows
WINDOW_EXPORTS = ["qlsd_window_create", "qlsd_window_decode", "qlsd_window_count", "qlsd_window_destroy"]


def _window_lib():
    L = lib()
    if not getattr(L, "_window_ready", False):
        P, I32 = ctypes.c_void_p, ctypes.c_int32
        L.qlsd_window_create.argtypes = [P, P, P, I32, I32, ctypes.POINTER(QlsdParams), I32, ctypes.POINTER(P)]
        L.qlsd_window_create.restype = ctypes.c_int
        L.qlsd_window_decode.argtypes = [P, P, I32, P, P]
        L.qlsd_window_decode.restype = ctypes.c_int
        L.qlsd_window_count.argtypes = [P]
        L.qlsd_window_count.restype = ctypes.c_int32
        L.qlsd_window_destroy.argtypes = [P]
        L._window_ready = True
    return L


class WindowDecoder:
    """qlsd_window: (w, c) overlapping-window BP + LSD over a multi-round DEM (include/qlsd_window.h)."""

    def __init__(self, code: Code, priors: np.ndarray, det_round: np.ndarray, w: int, c: int, max_batch: int,
                 max_iter: int = 30, ms_scaling: float = 0.625, lsd_order: int = 0, flags: int = 0):
        self.code = code
        self.max_batch = int(max_batch)
        pri = np.ascontiguousarray(priors, dtype=np.float64)
        dr = np.ascontiguousarray(det_round, dtype=np.int32)
        if pri.shape != (code.n,) or dr.shape != (code.m,):
            raise ValueError("priors must have shape (n,) and det_round shape (m,)")
        self.params = QlsdParams(int(max_iter), float(ms_scaling), int(lsd_order), 0, int(flags), 0)
        h = ctypes.c_void_p()
        _check(_window_lib().qlsd_window_create(code._h, pri.ctypes.data, dr.ctypes.data, int(w), int(c),
                                                ctypes.byref(self.params), self.max_batch, ctypes.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.qlsd_window_destroy(self._h)
            self._h = None

    @property
    def windows(self) -> int:
        return int(_window_lib().qlsd_window_count(self._h))

    def decode_into(self, syndromes, corrections, stream: Optional[int] = None):
        B = syndromes.shape[0]
        _need(syndromes, (B, self.code.m), "uint8", "syndromes")
        _need(corrections, (B, self.code.n), "uint8", "corrections")
        _check(_window_lib().qlsd_window_decode(self._h, _ptr(syndromes), B, _ptr(corrections),
                                                _stream() if stream is None else stream))

    def decode(self, syndromes):
        import torch
        corr = torch.empty((syndromes.shape[0], self.code.n), dtype=torch.uint8, device=syndromes.device)
        self.decode_into(syndromes.contiguous(), corr)
        return corr


# --------------------------------------------------------------------------- serving
SERVE_EXPORTS = ["qlsd_server_create", "qlsd_server_add_code", "qlsd_server_set_net", "qlsd_server_submit_many",
                 "qlsd_server_submit_many_device", "qlsd_server_lanes", "qlsd_server_set_retire_us",
                 "qlsd_server_start", "qlsd_server_wait", "qlsd_server_completions",
                 "qlsd_server_now_us", "qlsd_server_destroy"]

COMPLETION_DTYPE = np.dtype([("tag", np.uint64), ("code_id", np.int32), ("status", np.uint8),
                             ("r0", np.uint8, 3), ("arrival_us", np.float64), ("done_us", np.float64),
                             ("batch_size", np.int32), ("r1", np.int32)])
assert COMPLETION_DTYPE.itemsize == 40


def _serve_lib():
    L = lib()
    if not getattr(L, "_serve_ready", False):
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.qlsd_server_create.argtypes = [ctypes.c_size_t, ctypes.POINTER(P)]
        L.qlsd_server_add_code.argtypes = [P, P, ctypes.POINTER(QlsdParams), P, I32, I32,
                                           ctypes.POINTER(I32), ctypes.POINTER(I32)]
        L.qlsd_server_submit_many.argtypes = [P, I32, I32, P, P, P, P]
        L.qlsd_server_submit_many_device.argtypes = [P, I32, I32, P, P, P, P]
        L.qlsd_server_lanes.argtypes = [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]
        L.qlsd_server_set_retire_us.argtypes = [P, D]
        L.qlsd_server_set_net.argtypes = [P, I32, P]
        L.qlsd_server_start.argtypes = [P]
        L.qlsd_server_wait.argtypes = [P, I64, D]
        L.qlsd_server_completions.argtypes = [P, P, I32, ctypes.POINTER(I32)]
        L.qlsd_server_now_us.argtypes = [P]
        L.qlsd_server_now_us.restype = D
        L.qlsd_server_destroy.argtypes = [P]
        for fn in ("qlsd_server_create", "qlsd_server_add_code", "qlsd_server_set_net", "qlsd_server_submit_many",
                   "qlsd_server_submit_many_device", "qlsd_server_lanes", "qlsd_server_set_retire_us",
                   "qlsd_server_start", "qlsd_server_wait", "qlsd_server_completions"):
            getattr(L, fn).restype = ctypes.c_int
        L._serve_ready = True
    return L


class Server:
    """Continuous-batching decode service over several codes (include/qlsd_serve.h).

    Requests are numpy host arrays; the server keeps references until it is closed."""

    def __init__(self, device_budget_bytes: int):
        L = _serve_lib()
        h = ctypes.c_void_p()
        _check(L.qlsd_server_create(int(device_budget_bytes), ctypes.byref(h)))
        self._h = h
        self._keep = []
        self.codes = {}

    def add_code(self, code: "Code", priors: np.ndarray, batch_shots: int, max_lanes: int = 2,
                 max_iter: int = 30, ms_scaling: float = 0.625, lsd_order: int = 0, flags: int = 0):
        pri = np.ascontiguousarray(priors, dtype=np.float64)
        params = QlsdParams(int(max_iter), float(ms_scaling), int(lsd_order), 0, int(flags), 0)
        cid, lanes = ctypes.c_int32(), ctypes.c_int32()
        _check(_serve_lib().qlsd_server_add_code(self._h, code._h, ctypes.byref(params), pri.ctypes.data,
                                                 int(batch_shots), int(max_lanes), ctypes.byref(cid),
                                                 ctypes.byref(lanes)))
        self.codes[cid.value] = (code.m, code.n)
        self._keep.append(code)
        return cid.value, lanes.value

    def set_net(self, code_id: int, net: Optional["Net"]):
        """Attach a learned refinement to every lane of code_id (before start); the server keeps
        a reference so the net outlives it."""
        _net_lib()
        _check(_serve_lib().qlsd_server_set_net(self._h, int(code_id), None if net is None else net._h))
        self._keep.append(net)

    def submit_many(self, code_id: int, syndromes: np.ndarray, outputs: np.ndarray, tags: np.ndarray,
                    arrival_us: Optional[np.ndarray] = None):
        m, n = self.codes[code_id]
        S = np.ascontiguousarray(syndromes, dtype=np.uint8)
        if S.ndim != 2 or S.shape[1] != m or outputs.shape != (S.shape[0], n) or outputs.dtype != np.uint8 \
                or not outputs.flags["C_CONTIGUOUS"]:
            raise ValueError("syndromes [N, m] and contiguous uint8 outputs [N, n] expected")
        tg = np.ascontiguousarray(tags, dtype=np.uint64)
        ar = None if arrival_us is None else np.ascontiguousarray(arrival_us, dtype=np.float64)
        self._keep += [S, outputs, tg, ar]
        _check(_serve_lib().qlsd_server_submit_many(self._h, int(code_id), S.shape[0], S.ctypes.data,
                                                    outputs.ctypes.data, tg.ctypes.data,
                                                    None if ar is None else ar.ctypes.data))

    def submit_many_device(self, code_id: int, syndromes, outputs, tags: np.ndarray,
                           arrival_us: Optional[np.ndarray] = None):
        """Device-resident requests: syndromes uint8 CUDA [N, m], outputs uint8 CUDA [N, n]."""
        m, n = self.codes[code_id]
        N = syndromes.shape[0]
        _need(syndromes, (N, m), "uint8", "syndromes")
        _need(outputs, (N, n), "uint8", "outputs")
        tg = np.ascontiguousarray(tags, dtype=np.uint64)
        ar = None if arrival_us is None else np.ascontiguousarray(arrival_us, dtype=np.float64)
        self._keep += [syndromes, outputs, tg, ar]
        _check(_serve_lib().qlsd_server_submit_many_device(self._h, int(code_id), N, _ptr(syndromes), _ptr(outputs),
                                                           tg.ctypes.data, None if ar is None else ar.ctypes.data))

    def lanes(self, code_id: int):
        """(lanes held now, created so far, retired so far) of a code."""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_serve_lib().qlsd_server_lanes(self._h, int(code_id), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def set_retire_us(self, us: float):
        _check(_serve_lib().qlsd_server_set_retire_us(self._h, float(us)))

    def start(self):
        _check(_serve_lib().qlsd_server_start(self._h))

    def wait(self, count: int, timeout_s: float = 120.0):
        _check(_serve_lib().qlsd_server_wait(self._h, int(count), float(timeout_s)))

    def completions(self, max_records: int = 1 << 22) -> np.ndarray:
        out = np.empty(max_records, dtype=COMPLETION_DTYPE)
        k = ctypes.c_int32()
        _check(_serve_lib().qlsd_server_completions(self._h, out.ctypes.data, int(max_records), ctypes.byref(k)))
        return out[:k.value].copy()

    def now_us(self) -> float:
        return float(_serve_lib().qlsd_server_now_us(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _serve_lib().qlsd_server_destroy(self._h)
            self._h = None
        self._keep = []

    def __del__(self):
        if _lib is not None:
            self.close()


# ------------------------------------------------------------------ learned refinement
NET_PARAMS = 9537
NET_EXPORTS = ["qlsd_net_create", "qlsd_net_set_params", "qlsd_net_set_priors", "qlsd_net_get_params", "qlsd_net_forward",
               "qlsd_net_gradient", "qlsd_net_train_step", "qlsd_decoder_set_net", "qlsd_net_destroy"]


def _net_lib():
    L = lib()
    if not getattr(L, "_net_ready", False):
        P, I32, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
        L.qlsd_net_create.argtypes = [P, P, P, ctypes.POINTER(P)]
        L.qlsd_net_set_params.argtypes = [P, P]
        L.qlsd_net_set_priors.argtypes = [P, P]
        L.qlsd_net_get_params.argtypes = [P, P]
        L.qlsd_net_forward.argtypes = [P, P, P, I32, P, P]
        L.qlsd_net_gradient.argtypes = [P, P, P, P, I32, P, P, P]
        L.qlsd_net_train_step.argtypes = [P, P, P, P, I32, F, P]
        L.qlsd_decoder_set_net.argtypes = [P, P]
        L.qlsd_net_destroy.argtypes = [P]
        for fn in NET_EXPORTS[:-1]:
            getattr(L, fn).restype = ctypes.c_int
        L._net_ready = True
    return L


class Net:
    """Learned LLR refinement (include/qlsd_net.h) for one code; parameters live on the device."""

    def __init__(self, code: "Code", priors: np.ndarray, params: np.ndarray):
        pri = np.ascontiguousarray(priors, dtype=np.float64)
        th = np.ascontiguousarray(params, dtype=np.float32)
        if th.shape != (NET_PARAMS,):
            raise ValueError(f"params must have shape ({NET_PARAMS},)")
        h = ctypes.c_void_p()
        _check(_net_lib().qlsd_net_create(code._h, pri.ctypes.data, th.ctypes.data, ctypes.byref(h)))
        self._h = h
        self.code = code

    def set_params(self, params: np.ndarray):
        th = np.ascontiguousarray(params, dtype=np.float32)
        _check(_net_lib().qlsd_net_set_params(self._h, th.ctypes.data))

    def set_priors(self, priors: np.ndarray):
        pri = np.ascontiguousarray(priors, dtype=np.float64)
        if pri.shape != (self.code.n,):
            raise ValueError(f"priors must have shape ({self.code.n},)")
        _check(_net_lib().qlsd_net_set_priors(self._h, pri.ctypes.data))

    def get_params(self) -> np.ndarray:
        out = np.empty(NET_PARAMS, dtype=np.float32)
        _check(_net_lib().qlsd_net_get_params(self._h, out.ctypes.data))
        return out

    def _check_in(self, syndromes, llr, errors=None):
        B = llr.shape[0]
        _need(syndromes, (B, self.code.m), "uint8", "syndromes")
        _need(llr, (B, self.code.n), "float32", "llr")
        if errors is not None:
            _need(errors, (B, self.code.n), "uint8", "errors")

    def forward(self, syndromes, llr):
        import torch
        self._check_in(syndromes, llr)
        out = torch.empty_like(llr)
        _check(_net_lib().qlsd_net_forward(self._h, _ptr(syndromes), _ptr(llr), llr.shape[0], _ptr(out), _stream()))
        return out

    def gradient(self, syndromes, llr, errors):
        import torch
        self._check_in(syndromes, llr, errors)
        g = torch.empty(NET_PARAMS, dtype=torch.float32, device=llr.device)
        loss = torch.empty(1, dtype=torch.float32, device=llr.device)
        _check(_net_lib().qlsd_net_gradient(self._h, _ptr(syndromes), _ptr(llr), _ptr(errors), llr.shape[0],
                                            _ptr(g), _ptr(loss), _stream()))
        return g, loss

    def train_step(self, syndromes, llr, errors, lr: float):
        self._check_in(syndromes, llr, errors)
        _check(_net_lib().qlsd_net_train_step(self._h, _ptr(syndromes), _ptr(llr), _ptr(errors), llr.shape[0],
                                              float(lr), _stream()))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _net_lib().qlsd_net_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def attach_net(decoder: "Decoder", net: Optional[Net]):
    """decoder.decode then runs BP, the refinement on the shots BP did not solve, and LSD."""
    _check(_net_lib().qlsd_decoder_set_net(decoder._h, None if net is None else net._h))
    decoder._net = net
