"""ctypes binding of liblp.so (see include/lp.h for the ABI).

Argument marshalling only: every stage runs in the library's HIP kernels on
the caller's stream.  torch supplies device memory and streams.  There is
no CPU fallback: importing this module on a machine without the built
library or without a GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblp.so")

LP_OK, LP_EINVAL, LP_ENOMEM, LP_EAGAIN, LP_EHIP, LP_ECLOSED, LP_ETIMEOUT = (
    0, -1, -2, -3, -4, -5, -6)
LP_CI8, LP_CI16 = 1, 2
LP_FP32, LP_FP16_MFMA = 0, 1
LP_M, LP_TAPS, LP_NFFT, LP_HOP, LP_DELAY = 1024, 16, 4096, 2048, 1024
LP_DD_KEEP_TAIL = 1
WARM_FRAMES = LP_DELAY + LP_TAPS


class LpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblp error {code}: {msg}")
        self.code = code


class lp_array(C.Structure):
    _fields_ = [("n_st", C.c_int32), ("n_pol", C.c_int32),
                ("enu_m", C.POINTER(C.c_double)),
                ("gain", C.POINTER(C.c_float))]


class lp_band(C.Structure):
    _fields_ = [("n_sb", C.c_int32), ("k", C.POINTER(C.c_int32)),
                ("f0_hz", C.c_double), ("fs_hz", C.c_double),
                ("M", C.c_int32), ("taps", C.c_int32),
                ("kaiser_beta", C.c_double)]


class lp_dir(C.Structure):
    _fields_ = [("az_rad", C.c_double), ("el_rad", C.c_double)]


class lp_groups(C.Structure):
    _fields_ = [("n_groups", C.c_int32), ("group", C.POINTER(C.c_int32))]


class lp_sim_cfg(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_in", C.c_int32),
                ("noise_words", C.c_int32), ("adc_bits", C.c_int32)]


class lp_trig(C.Structure):
    _fields_ = [("sample", C.c_int64), ("beam", C.c_int32),
                ("tec", C.c_int32), ("snr", C.c_float), ("peak", C.c_float)]


class lp_stream_cfg(C.Structure):
    _fields_ = [("array", lp_array), ("band", lp_band),
                ("beams", C.POINTER(lp_dir)), ("n_beams", C.c_int32),
                ("tec_tecu", C.POINTER(C.c_double)), ("n_tec", C.c_int32),
                ("dtype", C.c_int32), ("prec", C.c_int32),
                ("k_sigma", C.c_float), ("max_n_t", C.c_int64),
                ("trig_cap", C.c_int32), ("deadline_s", C.c_double)]


class lp_result(C.Structure):
    _fields_ = [("stream", C.c_int32), ("status", C.c_int32),
                ("tag", C.c_uint64), ("n_t", C.c_int64),
                ("frame0", C.c_int64), ("n_trig", C.c_int32),
                ("n_beams", C.c_int32), ("n_tec", C.c_int32),
                ("trig", C.POINTER(lp_trig)), ("snr", C.POINTER(C.c_float)),
                ("best_tec", C.POINTER(C.c_int32)),
                ("submit_ns", C.c_int64), ("done_ns", C.c_int64),
                ("latency_ns", C.c_int64), ("deadline_ns", C.c_int64)]


LP_SUBMIT_RESET = 1

TRIG_DTYPE = np.dtype([("sample", np.int64), ("beam", np.int32),
                       ("tec", np.int32), ("snr", np.float32),
                       ("peak", np.float32)])

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run python -m paper_1612_06592_amd.build")
    # torch ships its own HIP and HSA runtimes under the same sonames as
    # the system ones liblp.so links.  Loading torch first makes the dynamic
    # linker bind liblp.so to those, so the process has one HIP runtime;
    # loading liblp.so first would map a second pair, after which torch
    # finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    L.lp_last_error.restype = C.c_char_p
    L.lp_version.restype = C.c_char_p
    L.lp_ctx_create.argtypes = [i32, C.POINTER(vp)]
    L.lp_ctx_create.restype = i32
    L.lp_ctx_destroy.argtypes = [vp]
    L.lp_ctx_destroy.restype = None
    L.lp_ctx_bind_const.argtypes = [vp, vp, C.c_size_t]
    L.lp_ctx_plan_cache.argtypes = [vp, i32]
    L.lp_ctx_plan_stats.argtypes = [vp, C.POINTER(i32), C.POINTER(i32),
                                    C.POINTER(C.c_size_t)]
    for name in ("lp_ctx_bind_const", "lp_ctx_plan_cache",
                 "lp_ctx_plan_stats"):
        getattr(L, name).restype = i32
    for name, args in [("lp_beam_bytes", [i32, i32, i64]),
                       ("lp_dd_state_bytes", [i32, i32]),
                       ("lp_dd_bytes", [i32, i32, i32, i64]),
                       ("lp_syn_state_bytes", [i32, i32]),
                       ("lp_cand_bytes", [i32, i64]),
                       ("lp_trigger_work_bytes", [i32, i32, i64])]:
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_size_t
    L.lp_beamform.argtypes = [vp, C.POINTER(lp_array), C.POINTER(lp_band),
                              C.POINTER(lp_dir), i32, vp, i32, i64, i32, vp,
                              vp]
    L.lp_dedisperse.argtypes = [vp, C.POINTER(lp_band),
                                C.POINTER(C.c_double), i32, vp, i32, i64, vp,
                                i32, vp, vp]
    L.lp_synthesize.argtypes = [vp, C.POINTER(lp_band), vp, i32, i64, i64,
                                vp, vp, vp, vp]
    L.lp_trigger.argtypes = [vp, vp, i32, i32, i64, i64, f32, vp, i32, vp,
                             vp, vp, vp, vp, vp]
    L.lp_trigger_noalloc.argtypes = [vp, vp, i32, i32, i64, i64, f32, vp,
                                     i32, vp, vp, vp, vp, vp]
    L.lp_ddsyn_work_bytes.argtypes = [i32, i64, i32]
    L.lp_ddsyn_work_bytes.restype = C.c_size_t
    L.lp_dedisperse_synthesize.argtypes = [vp, C.POINTER(lp_band),
                                           C.POINTER(C.c_double), i32, vp,
                                           i32, i64, i64, vp, vp, vp, i32, vp,
                                           C.c_size_t, vp]
    L.lp_dedisperse_synthesize.restype = i32
    for name in ("lp_beamform", "lp_dedisperse", "lp_synthesize",
                 "lp_trigger", "lp_trigger_noalloc"):
        getattr(L, name).restype = i32
    L.lp_plain_work_bytes.argtypes = [i32, i32, i32, i64]
    L.lp_plain_work_bytes.restype = C.c_size_t
    L.lp_dedisperse_plain.argtypes = [vp, C.POINTER(lp_band),
                                      C.POINTER(C.c_double), i32, vp, i32,
                                      i64, vp, i32, vp, vp, C.c_size_t, vp]
    L.lp_synthesize_plain.argtypes = [vp, C.POINTER(lp_band), vp, i32, i64,
                                      i64, vp, vp, vp, vp, C.c_size_t, vp]
    L.lp_dedisperse_plain.restype = i32
    L.lp_synthesize_plain.restype = i32
    L.lp_beamform_groups.argtypes = [vp, C.POINTER(lp_array),
                                     C.POINTER(lp_groups), C.POINTER(lp_band),
                                     C.POINTER(lp_dir), i32, vp, i32, i64,
                                     i32, vp, vp]
    L.lp_beamform_stage2.argtypes = [vp, C.POINTER(lp_array),
                                     C.POINTER(lp_groups), C.POINTER(lp_band),
                                     C.POINTER(lp_dir), i32, C.POINTER(lp_dir),
                                     i32, vp, i64, vp, vp]
    for name in ("lp_beamform_groups", "lp_beamform_stage2"):
        getattr(L, name).restype = i32
    L.lp_sim_adc.argtypes = [vp, C.POINTER(lp_sim_cfg), i64, i64, vp, i64,
                             i64, vp, vp]
    L.lp_sim_adc.restype = i32
    L.lp_station_work_bytes.argtypes = [i32, i32, i64]
    L.lp_station_work_bytes.restype = C.c_size_t
    L.lp_station_ppf.argtypes = [vp, C.POINTER(lp_band), vp, i32, i64, f32,
                                 i32, vp, vp, C.c_size_t, vp]
    L.lp_station_ppf.restype = i32
    L.lp_ppf_analyze.argtypes = [vp, C.POINTER(lp_band), vp, i32, i64, vp, vp]
    L.lp_ppf_adjoint.argtypes = [vp, C.POINTER(lp_band), vp, i32, i64, vp, vp]
    L.lp_ppf_work_bytes.argtypes = [i32, i32, i64]
    L.lp_ppf_work_bytes.restype = C.c_size_t
    L.lp_ppf_invert.argtypes = [vp, C.POINTER(lp_band), vp, i32, i64, i32,
                                vp, vp, vp, vp, C.c_size_t, vp]
    for name in ("lp_ppf_analyze", "lp_ppf_adjoint", "lp_ppf_invert"):
        getattr(L, name).restype = i32
    sp = C.POINTER(lp_stream_cfg)
    L.lp_stream_resident_bytes.argtypes = [sp, i64]
    L.lp_stream_resident_bytes.restype = C.c_size_t
    L.lp_block_bytes.argtypes = [sp, i64]
    L.lp_block_bytes.restype = C.c_size_t
    L.lp_server_create.argtypes = [vp, vp, C.c_size_t, i32, i64,
                                   C.POINTER(vp)]
    L.lp_server_create_sim.argtypes = [C.c_double, C.c_size_t, i32, i64,
                                       C.POINTER(vp)]
    L.lp_stream_open.argtypes = [vp, sp, C.POINTER(i32)]
    L.lp_stream_submit.argtypes = [vp, i32, vp, i64, C.c_uint64, i32]
    L.lp_stream_poll.argtypes = [vp, C.POINTER(lp_result), i32,
                                 C.POINTER(i32), i32]
    L.lp_stream_close.argtypes = [vp, i32]
    L.lp_server_destroy.argtypes = [vp]
    L.lp_server_destroy.restype = None
    L.lp_server_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64),
                                  C.POINTER(i64)]
    for name in ("lp_server_create", "lp_server_create_sim",
                 "lp_stream_open", "lp_stream_submit", "lp_stream_poll",
                 "lp_stream_close", "lp_server_stats"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def exported_symbols():
    """Names every build must export (those declared in include/lp.h)."""
    return ["lp_last_error", "lp_version", "lp_ctx_create", "lp_ctx_destroy",
            "lp_ctx_bind_const", "lp_ctx_plan_cache", "lp_ctx_plan_stats",
            "lp_beam_bytes", "lp_dd_state_bytes", "lp_dd_bytes",
            "lp_syn_state_bytes", "lp_cand_bytes", "lp_trigger_work_bytes",
            "lp_beamform", "lp_dedisperse", "lp_synthesize", "lp_trigger",
            "lp_trigger_noalloc", "lp_ddsyn_work_bytes",
            "lp_dedisperse_synthesize",
            "lp_plain_work_bytes", "lp_dedisperse_plain",
            "lp_synthesize_plain", "lp_beamform_groups", "lp_beamform_stage2",
            "lp_ppf_analyze", "lp_ppf_adjoint",
            "lp_ppf_work_bytes", "lp_ppf_invert", "lp_sim_adc",
            "lp_station_work_bytes", "lp_station_ppf",
            "lp_stream_resident_bytes",
            "lp_block_bytes", "lp_server_create", "lp_server_create_sim",
            "lp_stream_open", "lp_stream_submit", "lp_stream_poll",
            "lp_stream_close", "lp_server_destroy", "lp_server_stats"]


def check(rc: int):
    if rc != LP_OK:
        raise LpError(rc, lib().lp_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


_raw_stream = None


def _stream(stream):
    """HIP stream handle: `stream`'s, else the current stream of the current
    device (read through torch's raw-stream query, which skips building a
    Stream object: ~0.5 instead of ~3 us per call)."""
    global _raw_stream
    if stream is not None:
        return C.c_void_p(stream.cuda_stream)
    if _raw_stream is None:
        import torch
        torch.cuda.init()
        q = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        _raw_stream = ((lambda: q(torch._C._cuda_getDevice())) if q else
                       (lambda: torch.cuda.current_stream().cuda_stream))
    return C.c_void_p(_raw_stream())


def _tec(tec):
    """(pointer, count) of the TEC trials: a ctypes double array as it is,
    anything else through a contiguous float64 copy (kept alive by the
    returned pointer object)."""
    if isinstance(tec, C.Array):
        return tec, len(tec)
    t = np.ascontiguousarray(np.atleast_1d(tec), dtype=np.float64)
    return t.ctypes.data_as(C.POINTER(C.c_double)), len(t)


# ----------------------------------------------------------- descriptors

class Array:
    """Station array descriptor (keeps its host buffers alive)."""

    def __init__(self, enu, n_pol: int = 2, gain=None):
        self.enu = np.ascontiguousarray(enu, dtype=np.float64)
        self.gain = None if gain is None else np.ascontiguousarray(gain, np.float32)
        self.n_pol = n_pol
        self.c = lp_array(self.enu.shape[0], n_pol,
                          self.enu.ctypes.data_as(C.POINTER(C.c_double)),
                          None if self.gain is None else
                          self.gain.ctypes.data_as(C.POINTER(C.c_float)))

    @property
    def n_in(self) -> int:
        return self.enu.shape[0] * self.n_pol


class Band:
    def __init__(self, k, f0: float = 100e6, fs: float = 200e6,
                 beta: float = 9.0):
        self.k = np.ascontiguousarray(k, dtype=np.int32)
        self.c = lp_band(len(self.k),
                         self.k.ctypes.data_as(C.POINTER(C.c_int32)), f0, fs,
                         LP_M, LP_TAPS, beta)

    @property
    def n_sb(self) -> int:
        return len(self.k)


class Dirs:
    def __init__(self, az_el):
        a = np.ascontiguousarray(az_el, dtype=np.float64).reshape(-1, 2)
        self.arr = (lp_dir * len(a))(*[lp_dir(float(x), float(y)) for x, y in a])
        self.n = len(a)


class Ctx:
    def __init__(self, device: int = 0):
        self.h = C.c_void_p()
        check(lib().lp_ctx_create(device, C.byref(self.h)))

    def close(self):
        if self.h:
            lib().lp_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def bind_const(self, buf=None):
        """Plan tables from a caller device buffer (None: library memory)."""
        self._const = buf
        check(lib().lp_ctx_bind_const(self.h, _ptr(buf),
                                      0 if buf is None else buf.numel()
                                      * buf.element_size()))

    def plan_cache(self, max_plans: int):
        check(lib().lp_ctx_plan_cache(self.h, max_plans))

    def plan_stats(self):
        """(cached plans, plans in use, device bytes of their tables)."""
        n, held, nb = C.c_int32(), C.c_int32(), C.c_size_t()
        check(lib().lp_ctx_plan_stats(self.h, C.byref(n), C.byref(held),
                                      C.byref(nb)))
        return n.value, held.value, nb.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- stages

def beamform(ctx: Ctx, array: Array, band: Band, dirs: Dirs, x, n_t: int,
             dtype: int, prec: int, y, stream=None):
    check(lib().lp_beamform(ctx.h, C.byref(array.c), C.byref(band.c),
                            dirs.arr, dirs.n, _ptr(x), dtype, n_t, prec,
                            _ptr(y), _stream(stream)))


def dedisperse(ctx: Ctx, band: Band, tec, y, n_beams: int, n_t: int, tail, d,
               flags: int = 0, stream=None):
    tp, nt = _tec(tec)
    check(lib().lp_dedisperse(ctx.h, C.byref(band.c), tp, nt, _ptr(y),
                              n_beams, n_t, _ptr(tail), flags, _ptr(d),
                              _stream(stream)))


def synthesize(ctx: Ctx, band: Band, d, n_series: int, n_t: int, frame0: int,
               hist, cand, x_out=None, stream=None):
    check(lib().lp_synthesize(ctx.h, C.byref(band.c), _ptr(d), n_series, n_t,
                              frame0, _ptr(hist), _ptr(x_out), _ptr(cand),
                              _stream(stream)))


def trigger(ctx: Ctx, cand, n_beams: int, n_tec: int, n_t: int, frame0: int,
            k_sigma: float, out, cap: int, n_out, work, snr_out=None,
            best_tec=None, sigma_out=None, stream=None):
    check(lib().lp_trigger(ctx.h, _ptr(cand), n_beams, n_tec, n_t, frame0,
                           k_sigma, _ptr(out), cap, _ptr(n_out),
                           _ptr(snr_out), _ptr(best_tec), _ptr(sigma_out),
                           _ptr(work), _stream(stream)))


def dedisperse_synthesize(ctx: Ctx, band: Band, tec, y, n_beams: int,
                          n_t: int, frame0: int, tail, hist, cand,
                          trial_group: int, work, stream=None):
    tp, nt = _tec(tec)
    check(lib().lp_dedisperse_synthesize(
        ctx.h, C.byref(band.c), tp, nt, _ptr(y), n_beams, n_t, frame0,
        _ptr(tail), _ptr(hist),
        _ptr(cand), trial_group, _ptr(work), work.numel(), _stream(stream)))


def trigger_noalloc(ctx: Ctx, cand, n_beams: int, n_tec: int, n_t: int,
                    frame0: int, k_sigma: float, out, cap: int, n_out,
                    snr_out=None, best_tec=None, sigma_out=None, stream=None):
    check(lib().lp_trigger_noalloc(ctx.h, _ptr(cand), n_beams, n_tec, n_t,
                                   frame0, k_sigma, _ptr(out), cap,
                                   _ptr(n_out), _ptr(snr_out),
                                   _ptr(best_tec), _ptr(sigma_out),
                                   _stream(stream)))


TRIGGER_SCRATCH_BYTES = 128 << 20   # LP_TRIGGER_SCRATCH_BYTES


def dedisperse_plain(ctx: Ctx, band: Band, tec, y, n_beams: int, n_t: int,
                     tail, d, work, flags: int = 0, stream=None):
    tp, nt = _tec(tec)
    check(lib().lp_dedisperse_plain(ctx.h, C.byref(band.c), tp, nt, _ptr(y),
                                    n_beams, n_t, _ptr(tail), flags, _ptr(d),
                                    _ptr(work), work.numel(),
                                    _stream(stream)))


def synthesize_plain(ctx: Ctx, band: Band, d, n_series: int, n_t: int,
                     frame0: int, hist, cand, work, x_out=None, stream=None):
    check(lib().lp_synthesize_plain(ctx.h, C.byref(band.c), _ptr(d), n_series,
                                    n_t, frame0, _ptr(hist), _ptr(x_out),
                                    _ptr(cand), _ptr(work), work.numel(),
                                    _stream(stream)))


class Groups:
    """Station grouping for two-stage beamforming (keeps the host array)."""

    def __init__(self, group, n_groups: int | None = None):
        self.arr = np.ascontiguousarray(group, dtype=np.int32)
        self.n = int(self.arr.max()) + 1 if n_groups is None else n_groups
        self.c = lp_groups(self.n, self.arr.ctypes.data_as(
            C.POINTER(C.c_int32)))


def beamform_groups(ctx: Ctx, array: Array, groups: Groups, band: Band,
                    prelim: Dirs, x, n_t: int, y1, dtype: int = LP_CI8,
                    prec: int = LP_FP16_MFMA, stream=None):
    """Stage 1: y1 [G * P][n_sb][n_t] complex (include/lp.h)."""
    check(lib().lp_beamform_groups(ctx.h, C.byref(array.c), C.byref(groups.c),
                                   C.byref(band.c), prelim.arr, prelim.n,
                                   _ptr(x), dtype, n_t, prec, _ptr(y1),
                                   _stream(stream)))


def beamform_stage2(ctx: Ctx, array: Array, groups: Groups, band: Band,
                    prelim: Dirs, beams: Dirs, y1, n_t: int, y, stream=None):
    """Stage 2: y [B][n_sb][n_t] complex from y1 (include/lp.h)."""
    check(lib().lp_beamform_stage2(ctx.h, C.byref(array.c), C.byref(groups.c),
                                   C.byref(band.c), prelim.arr, prelim.n,
                                   beams.arr, beams.n, _ptr(y1), n_t, _ptr(y),
                                   _stream(stream)))


def sim_adc(ctx: Ctx, seed: int, n_in: int, noise_words: int, adc_bits: int,
            n0: int, n_samp: int, adc, pulse=None, pulse_n0: int = 0,
            stream=None):
    """ADC codes int16 [n_in][n_samp] (include/lp.h, lp_sim_adc); pulse:
    device float32 [n_in][len] or None."""
    cfg = lp_sim_cfg(seed, n_in, noise_words, adc_bits)
    plen = 0 if pulse is None else int(pulse.shape[-1])
    check(lib().lp_sim_adc(ctx.h, C.byref(cfg), n0, n_samp, _ptr(pulse),
                           pulse_n0, plen, _ptr(adc), _stream(stream)))


def station_ppf(ctx: Ctx, band: Band, adc, n_in: int, n_frames: int,
                scale: float, x, work, dtype: int = LP_CI8, stream=None):
    """Station subbands x [n_sb][n_frames][n_in][2] (int8 or int16) from
    ADC codes [n_in][(n_frames + 15) * 1024] (include/lp.h)."""
    check(lib().lp_station_ppf(ctx.h, C.byref(band.c), _ptr(adc), n_in,
                               n_frames, scale, dtype, _ptr(x), _ptr(work),
                               work.numel() * work.element_size(),
                               _stream(stream)))


def ppf_analyze(ctx: Ctx, band: Band, x, n_series: int, n_frames: int, y,
                stream=None):
    """y = H x: x float [n_series][(n_frames - 15) * 1024] -> y complex
    float [n_series][n_sb][n_frames] (trailing dim 2 for re, im)."""
    check(lib().lp_ppf_analyze(ctx.h, C.byref(band.c), _ptr(x), n_series,
                               n_frames, _ptr(y), _stream(stream)))


def ppf_adjoint(ctx: Ctx, band: Band, y, n_series: int, n_frames: int, x,
                stream=None):
    """x = H^T y (shapes as in ppf_analyze)."""
    check(lib().lp_ppf_adjoint(ctx.h, C.byref(band.c), _ptr(y), n_series,
                               n_frames, _ptr(x), _stream(stream)))


def ppf_invert(ctx: Ctx, band: Band, y, n_series: int, n_frames: int,
               n_iter: int, x, work, anorm=None, rnorm=None, stream=None):
    """n_iter LSMR iterations on H x = y per series (x, y as in
    ppf_analyze); anorm double [n_series][n_iter + 1], rnorm double
    [n_series] (optional); work uint8 of lp_ppf_work_bytes()."""
    check(lib().lp_ppf_invert(ctx.h, C.byref(band.c), _ptr(y), n_series,
                              n_frames, n_iter, _ptr(x), _ptr(anorm),
                              _ptr(rnorm), _ptr(work), work.numel(),
                              _stream(stream)))


def nbytes(name: str, *args) -> int:
    return int(getattr(lib(), name)(*args))


# ------------------------------------------------------ stream pipeline

@dataclass
class Pipeline:
    """Device buffers and carried state for one observation stream, and the
    four-stage chain per block.  Buffers are torch tensors on `device`."""

    ctx: Ctx
    array: Array
    band: Band
    dirs: Dirs
    tec: np.ndarray
    n_t: int
    dtype: int = LP_CI8
    prec: int = LP_FP16_MFMA
    k_sigma: float = 6.0
    trig_cap: int = 4096
    want_series: bool = False
    plain: bool = False          # plain FP32 comparator stages
    trial_group: int = 0         # > 0: lp_dedisperse_synthesize, one beam's
                                 # group of this many trials at a time
    device: str = "cuda:0"
    frame0: int = 0
    cand_slots: int = 1          # 2: the candidates of consecutive blocks
                                 # alternate between two buffers, so block
                                 # i's trigger can still read its own while
                                 # block i + 1 is synthesised
    bufs: dict = field(default_factory=dict)

    def __post_init__(self):
        import torch
        self.tec = np.atleast_1d(np.asarray(self.tec, dtype=np.float64))
        B, S, J, n_t = self.dirs.n, self.band.n_sb, len(self.tec), self.n_t
        u8 = dict(dtype=torch.uint8, device=self.device)

        def buf(n):
            return torch.empty(n, **u8)

        grouped = 0 < self.trial_group and not self.plain
        if self.cand_slots not in (1, 2):
            raise ValueError("cand_slots must be 1 or 2")
        self.bufs = dict(
            y=buf(nbytes("lp_beam_bytes", B, S, n_t)),
            d=(buf(nbytes("lp_ddsyn_work_bytes", S, n_t,
                          min(self.trial_group, J)))
               if grouped else buf(nbytes("lp_dd_bytes", B, J, S, n_t))),
            tail=torch.zeros(nbytes("lp_dd_state_bytes", B, S), **u8),
            hist=torch.zeros(nbytes("lp_syn_state_bytes", B * J, S), **u8),
            cand=buf(nbytes("lp_cand_bytes", B * J, n_t)),
            **({"cand1": buf(nbytes("lp_cand_bytes", B * J, n_t))}
               if self.cand_slots == 2 else {}),
            work=buf(nbytes("lp_trigger_work_bytes", B, J, n_t)),
            trig=torch.zeros(self.trig_cap * TRIG_DTYPE.itemsize, **u8),
            n_trig=torch.zeros(1, dtype=torch.int32, device=self.device),
            snr=torch.zeros((B, J), dtype=torch.float32, device=self.device),
            best=torch.zeros(B, dtype=torch.int32, device=self.device),
            sigma=torch.zeros((B, J), dtype=torch.float32, device=self.device),
        )
        if self.plain:
            self.prec = LP_FP32
            self.bufs["pwork"] = buf(nbytes("lp_plain_work_bytes", B, J, S,
                                            n_t))
        if self.want_series:
            self.bufs["x_out"] = torch.empty((B * J, n_t * LP_M),
                                             dtype=torch.float32,
                                             device=self.device)

    @property
    def n_beams(self):
        return self.dirs.n

    @property
    def n_tec(self):
        return len(self.tec)

    def _cand(self, frame0=None):
        """Candidate buffer of the block starting at frame0 (default: the
        block the next stage call works on)."""
        f = self.frame0 if frame0 is None else frame0
        if self.cand_slots == 2 and (f // self.n_t) % 2:
            return self.bufs["cand1"]
        return self.bufs["cand"]

    def _tec_arg(self):
        """The trials as a ctypes double array, rebuilt whenever their values
        change (a byte compare, cheaper than converting on every call)."""
        key = np.ascontiguousarray(self.tec, dtype=np.float64).tobytes()
        c = self.__dict__.get("_tec_c")
        if c is None or c[0] != key:
            c = (key, (C.c_double * len(self.tec))(*np.frombuffer(key)))
            self.__dict__["_tec_c"] = c
        return c[1]

    def beamform(self, x, stream=None):
        beamform(self.ctx, self.array, self.band, self.dirs, x, self.n_t,
                 self.dtype, self.prec, self.bufs["y"], stream)

    def dedisperse(self, stream=None):
        if self.plain:
            return dedisperse_plain(self.ctx, self.band, self._tec_arg(),
                                    self.bufs["y"], self.n_beams, self.n_t,
                                    self.bufs["tail"], self.bufs["d"],
                                    self.bufs["pwork"], 0, stream)
        dedisperse(self.ctx, self.band, self._tec_arg(), self.bufs["y"],
                   self.n_beams, self.n_t, self.bufs["tail"], self.bufs["d"],
                   0, stream)

    def synthesize(self, stream=None):
        if self.plain:
            return synthesize_plain(self.ctx, self.band, self.bufs["d"],
                                    self.n_beams * self.n_tec, self.n_t,
                                    self.frame0, self.bufs["hist"],
                                    self._cand(), self.bufs["pwork"],
                                    self.bufs.get("x_out"), stream)
        synthesize(self.ctx, self.band, self.bufs["d"],
                   self.n_beams * self.n_tec, self.n_t, self.frame0,
                   self.bufs["hist"], self._cand(),
                   self.bufs.get("x_out"), stream)

    def trigger(self, stream=None):
        b = self.bufs
        trigger(self.ctx, self._cand(), self.n_beams, self.n_tec, self.n_t,
                self.frame0, self.k_sigma, b["trig"], self.trig_cap,
                b["n_trig"], b["work"], b["snr"], b["best"], b["sigma"],
                stream)

    def dedisperse_synthesize(self, stream=None):
        """Both stages, one beam's group of trial_group trials at a time
        (bufs["d"] holds one group)."""
        b = self.bufs
        dedisperse_synthesize(self.ctx, self.band, self._tec_arg(), b["y"],
                              self.n_beams, self.n_t, self.frame0, b["tail"],
                              b["hist"], self._cand(), self.trial_group,
                              b["d"],
                              stream)

    def step_graph(self, x):
        """step() with beamform, de-dispersion and synthesis replayed from
        a HIP graph captured on the first call with this input buffer.  The
        three stages depend on frame0 only through the start-up rule, so the
        graph is used once frame0 >= WARM_FRAMES (before that the block runs
        as step()); the trigger, which reports samples from frame0, is issued
        with the current frame0 after each replay.  No stage issues a memset
        or host synchronisation, so the captured work is the eager work.
        The graph holds the plan tables by address: it stays valid while the
        context keeps this pipeline's plans (at most lp_ctx_plan_cache other
        unused plans are created meanwhile)."""
        import torch
        if self.frame0 < WARM_FRAMES:
            return self.step(x)
        # With two candidate slots, one graph per slot (a graph holds the
        # buffer it writes by address).
        name = "_graph1" if self._cand() is self.bufs.get("cand1") else "_graph"
        g = self.bufs.get(name)
        if g is None or g[1] != x.data_ptr():
            graph = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream(device=self.device)
            cs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.graph(graph, stream=cs):
                self._stages(x, None)
            torch.cuda.current_stream().wait_stream(cs)
            g = (graph, x.data_ptr())
            self.bufs[name] = g
            # (capture records the work without running it)
        g[0].replay()
        self.trigger()
        self.frame0 += self.n_t

    def _stages(self, x, stream):
        self.beamform(x, stream)
        if 0 < self.trial_group and not self.plain:
            self.dedisperse_synthesize(stream)
        else:
            self.dedisperse(stream)
            self.synthesize(stream)

    def step(self, x, stream=None):
        """Whole chain on one block (asynchronous); advances the stream."""
        self.beamform(x, stream)
        if 0 < self.trial_group and not self.plain:
            self.dedisperse_synthesize(stream)
        else:
            self.dedisperse(stream)
            self.synthesize(stream)
        self.trigger(stream)
        self.frame0 += self.n_t

    def triggers(self) -> np.ndarray:
        n = int(self.bufs["n_trig"].item())
        raw = self.bufs["trig"][: min(n, self.trig_cap) * TRIG_DTYPE.itemsize]
        return raw.cpu().numpy().view(TRIG_DTYPE).copy()

    # views of the intermediate device buffers
    def y_view(self):
        import torch
        B, S = self.n_beams, self.band.n_sb
        return self.bufs["y"].view(torch.float32).view(B, S, self.n_t, 2)

    def d_view(self):
        import torch
        if 0 < self.trial_group and not self.plain:
            raise ValueError("a trial-group pipeline holds one group of d")
        B, J, S = self.n_beams, self.n_tec, self.band.n_sb
        return self.bufs["d"].view(torch.float32).view(B, J, S, self.n_t, 2)

    def cand_view(self, frame0=None):
        """(emax [ns][n_t] f32, arg [ns][n_t] i32, psum [ns][n_t/16] f32) of
        the block starting at frame0; by default the last block step() or
        step_graph() completed (with one candidate slot: the only buffer)."""
        import torch
        ns, n_t = self.n_beams * self.n_tec, self.n_t
        c = self._cand(self.frame0 - n_t if frame0 is None else frame0)
        head = c[: ns * n_t * 8].view(torch.int32).view(ns, n_t, 2)
        emax = head[..., 0].view(torch.float32)
        arg = head[..., 1]
        psum = c[ns * n_t * 8: ns * n_t * 8 + ns * (n_t // 16) * 4].view(
            torch.float32).view(ns, n_t // 16)
        return emax, arg, psum


# ---------------------------------------------------------------- serving

class StreamCfg:
    """Keeps the host buffers of one lp_stream_cfg alive."""

    def __init__(self, enu, k, az_el, tec, max_n_t: int, dtype: int = LP_CI8,
                 prec: int = LP_FP16_MFMA, n_pol: int = 2, k_sigma: float = 6.0,
                 trig_cap: int = 0, deadline_s: float = 0.0, gain=None):
        self.array = Array(enu, n_pol, gain)
        self.band = Band(k)
        self.dirs = Dirs(az_el)
        self.tec = np.ascontiguousarray(np.atleast_1d(tec), dtype=np.float64)
        self.c = lp_stream_cfg(self.array.c, self.band.c, self.dirs.arr,
                               self.dirs.n,
                               self.tec.ctypes.data_as(C.POINTER(C.c_double)),
                               len(self.tec), dtype, prec, k_sigma, max_n_t,
                               trig_cap, deadline_s)

    def resident_bytes(self, chunk_t: int = 0) -> int:
        return int(lib().lp_stream_resident_bytes(C.byref(self.c), chunk_t))

    def block_bytes(self, n_t: int) -> int:
        return int(lib().lp_block_bytes(C.byref(self.c), n_t))


class Server:
    """lp_server_*: the persistent request loop (see include/lp.h)."""

    def __init__(self, ctx: Ctx | None = None, arena=None, arena_bytes=None,
                 max_slots: int = 0, chunk_t: int = 0,
                 sim_ns_per_sample: float | None = None):
        self.h = C.c_void_p()
        self._cfgs = {}
        self.arena = arena
        if sim_ns_per_sample is not None:
            check(lib().lp_server_create_sim(sim_ns_per_sample, arena_bytes,
                                             max_slots, chunk_t,
                                             C.byref(self.h)))
        else:
            check(lib().lp_server_create(ctx.h, _ptr(arena),
                                         arena_bytes or arena.numel(),
                                         max_slots, chunk_t, C.byref(self.h)))

    def open(self, cfg: StreamCfg) -> int:
        sid = C.c_int32()
        check(lib().lp_stream_open(self.h, C.byref(cfg.c), C.byref(sid)))
        self._cfgs[sid.value] = cfg
        return sid.value

    def submit(self, sid: int, block, n_t: int, tag: int = 0, flags: int = 0):
        ptr = block if isinstance(block, (int, type(None))) else block.data_ptr()
        check(lib().lp_stream_submit(self.h, sid, C.c_void_p(ptr), n_t, tag,
                                     flags))

    def poll(self, cap: int = 64, timeout_us: int = 100000):
        """Returns a list of result dicts (copies)."""
        arr = (lp_result * cap)()
        n = C.c_int32()
        rc = lib().lp_stream_poll(self.h, arr, cap, C.byref(n), timeout_us)
        if rc == LP_ETIMEOUT:
            return []
        check(rc)
        out = []
        for r in arr[:n.value]:
            nt = min(r.n_trig, self._cap(r.stream)) if r.status == LP_OK else 0
            trig = np.zeros(nt, dtype=TRIG_DTYPE)
            if nt:
                C.memmove(trig.ctypes.data, r.trig, nt * TRIG_DTYPE.itemsize)
            nbj = r.n_beams * r.n_tec
            snr = np.ctypeslib.as_array(r.snr, (nbj,)).copy() if nbj else None
            best = (np.ctypeslib.as_array(r.best_tec, (r.n_beams,)).copy()
                    if r.n_beams else None)
            out.append(dict(stream=r.stream, status=r.status, tag=r.tag,
                            n_t=r.n_t, frame0=r.frame0, n_trig=r.n_trig,
                            trig=trig, snr=snr, best_tec=best,
                            submit_ns=r.submit_ns, done_ns=r.done_ns,
                            latency_ns=r.latency_ns,
                            deadline_ns=r.deadline_ns))
        return out

    def _cap(self, sid):
        c = self._cfgs.get(sid)
        return (c.c.trig_cap or 1024) if c is not None else 1024

    def close_stream(self, sid: int):
        check(lib().lp_stream_close(self.h, sid))

    def stats(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        rc = lib().lp_server_stats(self.h, C.byref(a), C.byref(b), C.byref(c))
        return dict(blocks_done=a.value, chunks_issued=b.value,
                    admit_waits=c.value, status=rc)

    def destroy(self):
        if self.h:
            lib().lp_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
