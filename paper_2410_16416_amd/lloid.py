"""Python binding of the C ABI in include/lloid.h (argument marshalling only).

Every function here has the name of the C entry point it wraps; all
filtering work runs in the HIP library liblloid.so built for gfx950.  The
library must be built first (``python -m paper_2410_16416_amd.build``);
importing this module without it raises, there is no fallback path.
Device buffers may be given as torch tensors (their data_ptr is passed).
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblloid.so")

LLOID_OK, LLOID_EINVAL, LLOID_ENOMEM, LLOID_EAGAIN = 0, -1, -2, -3
LLOID_ETRUNC, LLOID_EDEVICE, LLOID_EORDER, LLOID_EDATA = -4, -5, -6, -7
LLOID_F64, LLOID_F32, LLOID_F16, LLOID_BF16 = 0, 1, 2, 3
NOALLOC_SCRATCH_BYTES = 256 << 20   # LLOID_NOALLOC_SCRATCH_BYTES
FIR_VARIANTS = 6                    # LLOID_FIR_VARIANTS
MIX_VARIANTS = 5                    # LLOID_MIX_VARIANTS
DTYPES = {"f64": LLOID_F64, "f32": LLOID_F32, "f16": LLOID_F16, "bf16": LLOID_BF16}
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EAGAIN", -4: "ETRUNC",
                -5: "EDEVICE", -6: "EORDER", -7: "EDATA"}


class LloidError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class lloid_slice(ctypes.Structure):
    _fields_ = [("rate_hz", ctypes.c_int32), ("n_taps", ctypes.c_int32),
                ("start_tap", ctypes.c_int64), ("n_basis", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("basis", ctypes.POINTER(ctypes.c_double)),
                ("mixing", ctypes.POINTER(ctypes.c_double))]


class lloid_bank_desc(ctypes.Structure):
    _fields_ = [("full_rate_hz", ctypes.c_int32), ("n_templates", ctypes.c_int32),
                ("n_slices", ctypes.c_int32), ("compute", ctypes.c_int32),
                ("slices", ctypes.POINTER(lloid_slice)),
                ("autocorr_half", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("autocorr", ctypes.POINTER(ctypes.c_double))]


class lloid_bank_info(ctypes.Structure):
    _fields_ = [("full_rate_hz", ctypes.c_int32), ("n_templates", ctypes.c_int32),
                ("n_slices", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("compute", ctypes.c_int32), ("concat_k", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64)]


class lloid_trigger_opts(ctypes.Structure):
    _fields_ = [("window_num", ctypes.c_int64), ("window_den", ctypes.c_int64),
                ("threshold", ctypes.c_float), ("strain_scale", ctypes.c_float)]


class lloid_peaks(ctypes.Structure):
    _fields_ = [("snr", ctypes.c_void_p), ("sample", ctypes.c_void_p),
                ("phase", ctypes.c_void_p), ("n_windows", ctypes.c_int64)]


class lloid_condition_opts(ctypes.Structure):
    _fields_ = [("seg_len", ctypes.c_int32), ("gate_half_width", ctypes.c_int32),
                ("gate_threshold", ctypes.c_float), ("reserved", ctypes.c_int32),
                ("psd", ctypes.POINTER(ctypes.c_double))]


class lloid_stream_opts(ctypes.Structure):
    _fields_ = [("n_detectors", ctypes.c_int32), ("min_rate_hz", ctypes.c_int32),
                ("max_windows_per_tick", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("max_filter_s", ctypes.c_double), ("hbm_budget", ctypes.c_int64),
                ("trig", lloid_trigger_opts), ("queue_strides", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lloid_stream_stats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("windows", ctypes.c_int64), ("triggers", ctypes.c_int64),
                ("next_window", ctypes.c_int64), ("latency_p50_ms", ctypes.c_double),
                ("latency_p99_ms", ctypes.c_double), ("latency_max_ms", ctypes.c_double),
                ("active_slots", ctypes.c_int32), ("queued_banks", ctypes.c_int32),
                ("bytes_in_use", ctypes.c_int64), ("graph_captures", ctypes.c_int64),
                ("graph_replays", ctypes.c_int64), ("queued_strides", ctypes.c_int64),
                ("ticks_in_flight", ctypes.c_int64)]


TRIGGER_DTYPE = np.dtype([("bank", np.int32), ("detector", np.int32), ("template_id", np.int32),
                          ("xi2", np.float32), ("window", np.int64), ("sample", np.int64),
                          ("snr", np.float32), ("phase", np.float32),
                          ("snr_interp", np.float32), ("dt", np.float32)])
assert TRIGGER_DTYPE.itemsize == 48

TUNE_DTYPE = np.dtype([("fir_variant", np.int32), ("mix_variant", np.int32), ("ms", np.float64)])

COINC_DTYPE = np.dtype([("a", np.int64), ("b", np.int64), ("bank", np.int32), ("template_id", np.int32),
                        ("snr_net", np.float32), ("dt", np.float32)])
assert COINC_DTYPE.itemsize == 32


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_16416_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "lloid_last_error": ([], ctypes.c_char_p),
        "lloid_version": ([], ctypes.c_char_p),
        "lloid_ctx_create": ([ctypes.c_int, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "lloid_ctx_destroy": ([vp], ctypes.c_int),
        "lloid_ctx_profile": ([vp, ctypes.c_int], ctypes.c_int),
        "lloid_ctx_stage_times": ([vp, vp, vp, ctypes.c_int], ctypes.c_int),
        "lloid_bank_create": ([vp, ctypes.POINTER(lloid_bank_desc), ctypes.POINTER(vp)], ctypes.c_int),
        "lloid_bank_sigma2": ([vp, vp], ctypes.c_int),
        "lloid_bank_query": ([vp, ctypes.POINTER(lloid_bank_info)], ctypes.c_int),
        "lloid_bank_destroy": ([vp], ctypes.c_int),
        "lloid_filter": ([vp, i32, vp, ctypes.c_int, i64, ctypes.POINTER(lloid_trigger_opts), vp, i64,
                          ctypes.POINTER(i64), vp, ctypes.POINTER(lloid_peaks)], ctypes.c_int),
        "lloid_filter_noalloc": ([vp, i32, vp, ctypes.c_int, i64, ctypes.POINTER(lloid_trigger_opts), vp, i64,
                                  ctypes.POINTER(i64), ctypes.POINTER(lloid_peaks)], ctypes.c_int),
        "lloid_ctx_set_tiles": ([vp, i32, i32], ctypes.c_int),
        "lloid_ctx_get_tiles": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], ctypes.c_int),
        "lloid_autotune": ([vp, ctypes.POINTER(vp), i32, ctypes.c_double, ctypes.c_char_p, vp, i32,
                            ctypes.POINTER(i32)], ctypes.c_int),
        "lloid_condition": ([vp, i32, vp, ctypes.c_int, i64, ctypes.POINTER(lloid_condition_opts), vp, vp,
                             ctypes.POINTER(i64)], ctypes.c_int),
        "lloid_coincide": ([vp, vp, i64, vp, i64, i64, vp, i64, ctypes.POINTER(i64), vp], ctypes.c_int),
        "lloid_filter_batch": ([ctypes.POINTER(vp), i32, i32, vp, ctypes.c_int, i64,
                                ctypes.POINTER(lloid_trigger_opts), vp, i64, ctypes.POINTER(i64),
                                ctypes.POINTER(lloid_peaks)], ctypes.c_int),
        "lloid_ctx_set_chunk_bytes": ([vp, i64], ctypes.c_int),
        "lloid_stream_create": ([vp, i32, ctypes.c_int, ctypes.POINTER(lloid_stream_opts), ctypes.POINTER(vp)],
                                ctypes.c_int),
        "lloid_stream_admit": ([vp, vp, ctypes.POINTER(i32)], ctypes.c_int),
        "lloid_stream_remove": ([vp, i32], ctypes.c_int),
        "lloid_stream_push": ([vp, i32, i64, vp, ctypes.c_int, i64], ctypes.c_int),
        "lloid_stream_poll": ([vp, vp, i64, ctypes.POINTER(i64), i32], ctypes.c_int),
        "lloid_stream_stats_reset": ([vp], ctypes.c_int),
        "lloid_stream_flush": ([vp], ctypes.c_int),
        "lloid_stream_stats_get": ([vp, ctypes.POINTER(lloid_stream_stats)], ctypes.c_int),
        "lloid_stream_destroy": ([vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def _check(status: int):
    if status != LLOID_OK:
        raise LloidError(status, _lib.lloid_last_error().decode())


def _ptr(a):
    """Address of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())


def exported_symbols():
    return ["lloid_last_error", "lloid_version", "lloid_ctx_create", "lloid_ctx_destroy",
            "lloid_ctx_profile", "lloid_ctx_stage_times",
            "lloid_bank_create", "lloid_bank_sigma2", "lloid_bank_query", "lloid_bank_destroy",
            "lloid_filter", "lloid_filter_noalloc", "lloid_filter_batch", "lloid_ctx_set_chunk_bytes",
            "lloid_stream_create", "lloid_stream_admit", "lloid_stream_remove", "lloid_stream_push",
            "lloid_stream_poll", "lloid_stream_flush", "lloid_stream_stats_get", "lloid_stream_stats_reset",
            "lloid_stream_destroy",
            "lloid_coincide", "lloid_condition", "lloid_ctx_set_tiles", "lloid_ctx_get_tiles", "lloid_autotune"]


def lloid_version() -> str:
    return _lib.lloid_version().decode()


def lloid_ctx_create(device: int = 0, stream=None):
    """stream: a hipStream_t as int (e.g. torch.cuda.current_stream().cuda_stream) or None."""
    out = ctypes.c_void_p()
    _check(_lib.lloid_ctx_create(device, ctypes.c_void_p(stream) if stream else None, ctypes.byref(out)))
    return out


def lloid_ctx_destroy(ctx):
    _check(_lib.lloid_ctx_destroy(ctx))


STAGES = ["ingest", "decimate", "fir", "interp", "mix", "phase", "trigger", "d2h"]


def lloid_ctx_profile(ctx, enable: bool):
    _check(_lib.lloid_ctx_profile(ctx, 1 if enable else 0))


def lloid_ctx_stage_times(ctx, reset: bool = False):
    """{stage: (total device ms, calls)} since the last reset."""
    ms = np.zeros(len(STAGES), dtype=np.float64)
    calls = np.zeros(len(STAGES), dtype=np.int64)
    _check(_lib.lloid_ctx_stage_times(ctx, ms.ctypes.data, calls.ctypes.data, 1 if reset else 0))
    return {k: (float(ms[i]), int(calls[i])) for i, k in enumerate(STAGES)}


def lloid_ctx_set_chunk_bytes(ctx, nbytes: int):
    _check(_lib.lloid_ctx_set_chunk_bytes(ctx, int(nbytes)))


def lloid_bank_create(ctx, full_rate_hz: int, n_templates: int, slices, compute: str = "f16",
                      autocorr=None):
    """slices: objects with rate, start_tap, n_taps, basis [L, N], mixing [2F, L] (float64).
    autocorr: None, or complex [F, 2K + 1] normalised template autocorrelations
    (column K + k for lag k), the input of each trigger's xi2."""
    keep = []
    arr = (lloid_slice * len(slices))()
    for k, s in enumerate(slices):
        b = np.ascontiguousarray(s.basis, dtype=np.float64)
        m = np.ascontiguousarray(s.mixing, dtype=np.float64)
        keep += [b, m]
        arr[k].rate_hz = int(s.rate)
        arr[k].n_taps = int(s.n_taps)
        arr[k].start_tap = int(s.start_tap)
        arr[k].n_basis = int(b.shape[0])
        arr[k].basis = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        arr[k].mixing = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    desc = lloid_bank_desc(int(full_rate_hz), int(n_templates), len(slices), DTYPES[compute], arr)
    if autocorr is not None:
        ac = np.asarray(autocorr)
        if ac.ndim != 2 or ac.shape[0] != int(n_templates) or ac.shape[1] % 2 != 1:
            raise ValueError("autocorr must be [n_templates, 2K + 1]")
        pairs = np.ascontiguousarray(np.stack([ac.real, ac.imag], axis=-1), dtype=np.float64)
        keep.append(pairs)
        desc.autocorr_half = (ac.shape[1] - 1) // 2
        desc.autocorr = pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    out = ctypes.c_void_p()
    _check(_lib.lloid_bank_create(ctx, ctypes.byref(desc), ctypes.byref(out)))
    return out


def lloid_bank_query(bank) -> lloid_bank_info:
    info = lloid_bank_info()
    _check(_lib.lloid_bank_query(bank, ctypes.byref(info)))
    return info


def lloid_bank_sigma2(bank) -> np.ndarray:
    out = np.empty(lloid_bank_query(bank).n_templates, dtype=np.float64)
    _check(_lib.lloid_bank_sigma2(bank, out.ctypes.data))
    return out


def lloid_bank_destroy(bank):
    _check(_lib.lloid_bank_destroy(bank))


@dataclass
class FilterResult:
    triggers: np.ndarray          # TRIGGER_DTYPE records
    n_triggers: int
    peak_snr: np.ndarray | None = None
    peak_sample: np.ndarray | None = None
    peak_phase: np.ndarray | None = None
    snr: object = None


def lloid_ctx_set_tiles(ctx, fir_variant: int, mix_variant: int):
    _check(_lib.lloid_ctx_set_tiles(ctx, int(fir_variant), int(mix_variant)))


def lloid_ctx_get_tiles(ctx):
    f, m = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(_lib.lloid_ctx_get_tiles(ctx, ctypes.byref(f), ctypes.byref(m)))
    return f.value, m.value


def lloid_autotune(ctx, banks, seconds: float, cache_path: str | None = None):
    """Pick the tile variants for these banks (see include/lloid.h); returns
    the chosen (fir, mix) pair and the TUNE_DTYPE timings (empty when the
    cache held the choice)."""
    arr = (ctypes.c_void_p * len(banks))(*[b.value for b in banks])
    res = np.zeros(64, dtype=TUNE_DTYPE)
    n = ctypes.c_int32(0)
    _check(_lib.lloid_autotune(ctx, arr, len(banks), float(seconds),
                               cache_path.encode() if cache_path else None, res.ctypes.data, res.shape[0],
                               ctypes.byref(n)))
    return lloid_ctx_get_tiles(ctx), res[:n.value].copy()


def lloid_condition(ctx, full_rate_hz: int, strain, seg_len: int, gate_threshold: float = 0.0,
                    gate_half_width: int = 0, psd=None, out=None):
    """Whiten and gate one block of strain (numpy float64/float32, or a torch
    tensor).  psd: None (estimate it from the block) or [seg_len/2 + 1] float64.
    Returns (conditioned float32 strain, PSD used, samples gated); out may be a
    preallocated float32 numpy array or device tensor of n values."""
    strain, dt, n = _strain_arg(strain)
    keep = None
    opts = lloid_condition_opts(int(seg_len), int(gate_half_width), float(gate_threshold), 0, None)
    if psd is not None:
        keep = np.ascontiguousarray(psd, dtype=np.float64)
        if keep.shape != (seg_len // 2 + 1,):
            raise ValueError("psd must have seg_len / 2 + 1 values")
        opts.psd = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if out is None:
        out = np.empty(n, dtype=np.float32)
    psd_out = np.empty(seg_len // 2 + 1, dtype=np.float64)
    gated = ctypes.c_int64(0)
    _check(_lib.lloid_condition(ctx, int(full_rate_hz), _ptr(strain), dt, n, ctypes.byref(opts), _ptr(out),
                                psd_out.ctypes.data, ctypes.byref(gated)))
    return out, psd_out, int(gated.value)


def lloid_coincide(ctx, a, b, max_dt: int, cap: int | None = None, background: bool = False):
    """Coincidences of two trigger lists (numpy TRIGGER_DTYPE arrays, or torch
    uint8 tensors of 48-byte records on the device), each sorted by (bank,
    template_id, sample).  Returns the COINC_DTYPE pairs and, with background,
    a uint8 array of n_a + n_b flags (1: the trigger is in no pair)."""
    def count(x):
        return x.shape[0] if isinstance(x, np.ndarray) else x.numel() // TRIGGER_DTYPE.itemsize
    n_a, n_b = count(a), count(b)
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a, dtype=TRIGGER_DTYPE)
    if isinstance(b, np.ndarray):
        b = np.ascontiguousarray(b, dtype=TRIGGER_DTYPE)
    if cap is None:
        cap = max(16, 4 * max(n_a, n_b))
    for _ in range(2):
        out = np.zeros(max(cap, 1), dtype=COINC_DTYPE)
        bg = np.zeros(n_a + n_b, dtype=np.uint8) if background else None
        n = ctypes.c_int64(0)
        st = _lib.lloid_coincide(ctx, _ptr(a) if n_a else None, n_a, _ptr(b) if n_b else None, n_b, int(max_dt),
                                 out.ctypes.data, cap, ctypes.byref(n), _ptr(bg) if bg is not None and bg.size else None)
        if st == LLOID_ETRUNC:
            cap = n.value
            continue
        _check(st)
        break
    pairs = out[:n.value].copy()
    return (pairs, bg) if background else pairs


def lloid_filter(bank, detector: int, strain, window=(1, 1), threshold: float = 4.0,
                 strain_scale: float = 0.0, trig_cap: int | None = None, triggers_out=None,
                 snr_out=None, peaks: bool = False, n_windows: int | None = None) -> FilterResult:
    """strain: float64/float32 numpy array (host) or torch tensor (host or device).

    triggers_out: optional preallocated host buffer (numpy TRIGGER_DTYPE array or a
    pinned torch uint8 tensor of 48*cap bytes).  snr_out: optional [F, n, 2] float32
    numpy array or torch tensor receiving the complex SNR.
    """
    strain, dt, n = _strain_arg(strain)
    info = lloid_bank_query(bank)
    n_templates = info.n_templates
    num, den = window
    opts = lloid_trigger_opts(int(num), int(den), float(threshold), float(strain_scale))
    if n_windows is None:
        n_windows = -(-n * int(den) // (info.full_rate_hz * int(num)))
    pk = None
    res = FilterResult(triggers=None, n_triggers=0)
    if peaks:
        res.peak_snr = np.empty((n_templates, n_windows), dtype=np.float32)
        res.peak_sample = np.empty((n_templates, n_windows), dtype=np.int64)
        res.peak_phase = np.empty((n_templates, n_windows), dtype=np.float32)
        pk = lloid_peaks(res.peak_snr.ctypes.data, res.peak_sample.ctypes.data, res.peak_phase.ctypes.data,
                         n_windows)
    if triggers_out is None:
        cap = trig_cap if trig_cap is not None else n_templates * max(1, n_windows or 1)
        triggers_out = np.empty(cap, dtype=TRIGGER_DTYPE)
    cap = (triggers_out.shape[0] if isinstance(triggers_out, np.ndarray)
           else triggers_out.numel() // TRIGGER_DTYPE.itemsize)
    n_trig = ctypes.c_int64()
    st = _lib.lloid_filter(bank, int(detector), ctypes.c_void_p(_ptr(strain)), dt, int(n), ctypes.byref(opts),
                           ctypes.c_void_p(_ptr(triggers_out)), int(cap), ctypes.byref(n_trig),
                           ctypes.c_void_p(_ptr(snr_out)) if snr_out is not None else None,
                           ctypes.byref(pk) if pk is not None else None)
    if st == LLOID_ETRUNC and pk is not None and pk.n_windows > n_windows:
        return lloid_filter(bank, detector, strain, window, threshold, strain_scale, trig_cap,
                            None, snr_out, peaks, int(pk.n_windows))
    if st == LLOID_ETRUNC and triggers_out is not None and trig_cap is None and n_trig.value > cap:
        return lloid_filter(bank, detector, strain, window, threshold, strain_scale,
                            int(n_trig.value), None, snr_out, peaks, n_windows)
    _check(st)
    res.n_triggers = int(n_trig.value)
    if isinstance(triggers_out, np.ndarray):
        res.triggers = triggers_out[: res.n_triggers]
    else:
        res.triggers = triggers_out
    res.snr = snr_out
    return res


def lloid_filter_noalloc(bank, detector: int, strain, window=(1, 1), threshold: float = 4.0,
                         strain_scale: float = 0.0, trig_cap: int | None = None,
                         peaks: bool = False) -> FilterResult:
    """lloid_filter through the allocation-free entry point (static device
    scratch of NOALLOC_SCRATCH_BYTES per GPU).  The caller's outputs are host
    numpy arrays allocated here."""
    strain, dt, n = _strain_arg(strain)
    info = lloid_bank_query(bank)
    num, den = window
    opts = lloid_trigger_opts(int(num), int(den), float(threshold), float(strain_scale))
    n_windows = -(-n * int(den) // (info.full_rate_hz * int(num)))
    res = FilterResult(triggers=None, n_triggers=0)
    pk = None
    if peaks:
        res.peak_snr = np.empty((info.n_templates, n_windows), dtype=np.float32)
        res.peak_sample = np.empty((info.n_templates, n_windows), dtype=np.int64)
        res.peak_phase = np.empty((info.n_templates, n_windows), dtype=np.float32)
        pk = lloid_peaks(res.peak_snr.ctypes.data, res.peak_sample.ctypes.data, res.peak_phase.ctypes.data,
                         n_windows)
    cap = trig_cap if trig_cap is not None else info.n_templates * max(1, n_windows)
    out = np.empty(max(cap, 1), dtype=TRIGGER_DTYPE)
    n_trig = ctypes.c_int64()
    st = _lib.lloid_filter_noalloc(bank, int(detector), ctypes.c_void_p(_ptr(strain)), dt, int(n),
                                   ctypes.byref(opts), ctypes.c_void_p(out.ctypes.data), int(cap),
                                   ctypes.byref(n_trig), ctypes.byref(pk) if pk is not None else None)
    _check(st)
    res.n_triggers = int(n_trig.value)
    res.triggers = out[: res.n_triggers]
    return res


def _strain_arg(strain):
    if isinstance(strain, np.ndarray):
        strain = np.ascontiguousarray(strain)
        dt = LLOID_F64 if strain.dtype == np.float64 else LLOID_F32 if strain.dtype == np.float32 else None
    else:
        import torch
        dt = {torch.float64: LLOID_F64, torch.float32: LLOID_F32}.get(strain.dtype)
    if dt is None:
        raise LloidError(LLOID_EINVAL, "strain must be float64 or float32")
    return strain, dt, int(strain.shape[0])


@dataclass
class BatchResult:
    triggers: np.ndarray
    n_triggers: int
    peak_snr: list | None = None       # per bank [F_b, W]
    peak_sample: list | None = None
    peak_phase: list | None = None


def lloid_filter_batch(banks, detector: int, strain, window=(1, 1), threshold: float = 4.0,
                       strain_scale: float = 0.0, trig_cap: int | None = None, triggers_out=None,
                       peaks: bool = False) -> BatchResult:
    """Filter one detector's strain with every bank in `banks` (one launch per stage)."""
    strain, dt, n = _strain_arg(strain)
    infos = [lloid_bank_query(b) for b in banks]
    num, den = window
    opts = lloid_trigger_opts(int(num), int(den), float(threshold), float(strain_scale))
    n_windows = -(-n * int(den) // (infos[0].full_rate_hz * int(num)))
    res = BatchResult(triggers=None, n_triggers=0)
    pk = None
    if peaks:
        res.peak_snr = [np.empty((i.n_templates, n_windows), np.float32) for i in infos]
        res.peak_sample = [np.empty((i.n_templates, n_windows), np.int64) for i in infos]
        res.peak_phase = [np.empty((i.n_templates, n_windows), np.float32) for i in infos]
        pk = (lloid_peaks * len(banks))()
        for k in range(len(banks)):
            pk[k] = lloid_peaks(res.peak_snr[k].ctypes.data, res.peak_sample[k].ctypes.data,
                                res.peak_phase[k].ctypes.data, n_windows)
    if triggers_out is None:
        cap = trig_cap if trig_cap is not None else sum(i.n_templates for i in infos) * n_windows
        triggers_out = np.empty(max(cap, 1), dtype=TRIGGER_DTYPE)
        cap = cap if trig_cap is not None else triggers_out.shape[0]
    else:
        cap = (triggers_out.shape[0] if isinstance(triggers_out, np.ndarray)
               else triggers_out.numel() // TRIGGER_DTYPE.itemsize)
    handles = (ctypes.c_void_p * len(banks))(*[b.value for b in banks])
    n_trig = ctypes.c_int64()
    st = _lib.lloid_filter_batch(handles, len(banks), int(detector), ctypes.c_void_p(_ptr(strain)), dt, n,
                                 ctypes.byref(opts), ctypes.c_void_p(_ptr(triggers_out)), int(cap),
                                 ctypes.byref(n_trig), pk)
    _check(st)
    res.n_triggers = int(n_trig.value)
    res.triggers = triggers_out[: res.n_triggers] if isinstance(triggers_out, np.ndarray) else triggers_out
    return res


def bank_from_svd(ctx, svd_bank, compute: str = "f16"):
    """Upload an SVD bank object (attributes f0, n_templates, slices and,
    optionally, autocorr)."""
    return lloid_bank_create(ctx, svd_bank.f0, svd_bank.n_templates, svd_bank.slices, compute,
                             autocorr=getattr(svd_bank, "autocorr", None))


# ------------------------------------------------------------------ streaming

def lloid_stream_create(ctx, full_rate_hz: int, compute: str = "f16", n_detectors: int = 1,
                        min_rate_hz: int | None = None, window=(1, 1), threshold: float = 4.0,
                        strain_scale: float = 0.0, hbm_budget: int = 0, max_filter_s: float = 0.0,
                        max_windows_per_tick: int = 0, use_graph: bool = False, queue_strides: int = 0):
    opts = lloid_stream_opts(int(n_detectors), int(min_rate_hz or max(1, full_rate_hz // 16)),
                             int(max_windows_per_tick), 1 if use_graph else 0, float(max_filter_s),
                             int(hbm_budget),
                             lloid_trigger_opts(int(window[0]), int(window[1]), float(threshold),
                                                float(strain_scale)), int(queue_strides), 0)
    out = ctypes.c_void_p()
    _check(_lib.lloid_stream_create(ctx, int(full_rate_hz), DTYPES[compute], ctypes.byref(opts),
                                    ctypes.byref(out)))
    return out


def lloid_stream_admit(stream, bank):
    """Returns (slot, active); a queued bank (EAGAIN) returns active=False."""
    slot = ctypes.c_int32(-1)
    st = _lib.lloid_stream_admit(stream, bank, ctypes.byref(slot))
    if st == LLOID_EAGAIN:
        return int(slot.value), False
    _check(st)
    return int(slot.value), True


def lloid_stream_remove(stream, slot: int):
    _check(_lib.lloid_stream_remove(stream, int(slot)))


def lloid_stream_push(stream, detector: int, t0: int, data):
    data, dt, n = _strain_arg(data)
    _check(_lib.lloid_stream_push(stream, int(detector), int(t0), ctypes.c_void_p(_ptr(data)), dt, n))


def lloid_stream_poll(stream, cap: int = 1 << 20, wait_ms: int = 0) -> np.ndarray:
    """Queued triggers; wait_ms > 0 (or < 0: no limit) first waits for the
    strides pushed so far to be filtered."""
    out = np.empty(max(cap, 1), dtype=TRIGGER_DTYPE)
    n = ctypes.c_int64()
    _check(_lib.lloid_stream_poll(stream, ctypes.c_void_p(out.ctypes.data), int(cap), ctypes.byref(n),
                                  int(wait_ms)))
    return out[: n.value]


def lloid_stream_flush(stream):
    _check(_lib.lloid_stream_flush(stream))


def lloid_stream_stats_get(stream) -> lloid_stream_stats:
    st = lloid_stream_stats()
    _check(_lib.lloid_stream_stats_get(stream, ctypes.byref(st)))
    return st


def lloid_stream_stats_reset(stream):
    _check(_lib.lloid_stream_stats_reset(stream))


def lloid_stream_destroy(stream):
    _check(_lib.lloid_stream_destroy(stream))
