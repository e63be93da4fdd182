"""FP64 CPU oracle for the lunar ns-pulse hot path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liblpo.so`` (plain C,
``lpo.c``), which shares no code with the GPU library.  Every function
follows the definition cited in ``lpo.h``; the paper is Winchen et al.,
arXiv:1612.06592 (Sec. 2 for the processing chain, Sec. 3 for beamforming,
PPF inversion and ionospheric de-dispersion).

Pins for each function live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblpo.so")
_lib = None

# Stream geometry shared by the oracle's own driver below (the paper leaves
# these open; see the conventions in lpo.h).
M_DEFAULT = 1024
P_DEFAULT = 16
N_FFT = 4096
HOP = 2048
DELAY = 1024


def build(force: bool = True) -> str:
    """Compile liblpo.so with gcc (no GPU toolchain involved)."""
    src = os.path.join(_HERE, "lpo.c")
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(src)):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-Wno-unused-parameter",
               src, "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_long
        L.lpo_kappa.restype = C.c_double
        L.lpo_speed_of_light.restype = C.c_double
        L.lpo_threads.restype = C.c_int
        L.lpo_set_threads.argtypes = [C.c_int]
        L.lpo_fft.argtypes = [lp, dp, C.c_int]
        L.lpo_bessel_i0.restype = C.c_double
        L.lpo_bessel_i0.argtypes = [C.c_double]
        L.lpo_prototype.argtypes = [C.c_int, C.c_int, C.c_double, dp]
        L.lpo_analysis.argtypes = [C.c_int, C.c_int, dp, lp, dp, lp, lp,
                                   C.c_int, ip, dp]
        L.lpo_beamform.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int, ip,
                                   C.c_double, C.c_double, C.c_int, C.c_int,
                                   dp, lp, dp, dp]
        L.lpo_chirp.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int,
                                C.c_double, dp]
        L.lpo_dedisperse.restype = C.c_int
        L.lpo_dedisperse.argtypes = [C.c_int, ip, C.c_double, C.c_double,
                                     C.c_int, C.c_int, dp, C.c_int, C.c_int,
                                     C.c_int, C.c_int, lp, dp, dp, dp]
        L.lpo_synthesize.argtypes = [C.c_int, C.c_int, dp, C.c_int, ip,
                                     C.c_int, lp, dp, dp, dp]
        L.lpo_detect.argtypes = [C.c_int, lp, lp, lp, C.c_int, dp, dp, dp,
                                 C.POINTER(C.c_int64)]
        L.lpo_trigger.restype = C.c_long
        L.lpo_trigger.argtypes = [C.c_int, C.c_int, C.c_int, lp, lp, lp,
                                  C.c_int, C.c_int, dp, dp,
                                  C.POINTER(C.c_int64), C.c_double, lp,
                                  C.c_void_p, dp, ip]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def kappa() -> float:
    """Ionospheric constant in s^-1 per TECU (phase 2*pi*kappa*T/f)."""
    return lib().lpo_kappa()


def speed_of_light() -> float:
    return lib().lpo_speed_of_light()


def threads() -> int:
    return lib().lpo_threads()


def set_threads(n: int) -> None:
    """Thread count of the oracle's later parallel loops."""
    lib().lpo_set_threads(int(n))


def fft(x, inverse: bool = False) -> np.ndarray:
    x = _c128(x).copy()
    n = x.shape[-1]
    assert n & (n - 1) == 0
    flat = x.reshape(-1, n)
    for row in flat:
        lib().lpo_fft(n, _dp(row.view(np.float64)), int(inverse))
    return flat.reshape(x.shape)


def bessel_i0(x: float) -> float:
    return lib().lpo_bessel_i0(float(x))


def prototype(M: int = M_DEFAULT, P: int = P_DEFAULT,
              beta: float = 9.0) -> np.ndarray:
    h = np.zeros(M * P, dtype=np.float64)
    lib().lpo_prototype(M, P, beta, _dp(h))
    return h


def analysis(h, M: int, P: int, x, m0: int, n_frames: int,
             channels) -> np.ndarray:
    """Analysis PFB of a complex series x; returns [n_ch][n_frames]."""
    x = _c128(x)
    h = np.ascontiguousarray(h, dtype=np.float64)
    ch = np.ascontiguousarray(channels, dtype=np.int32)
    y = np.zeros((len(ch), n_frames), dtype=np.complex128)
    lib().lpo_analysis(M, P, _dp(h), len(x), _dp(x.view(np.float64)), m0,
                       n_frames, len(ch), _ip(ch), _dp(y.view(np.float64)))
    return y


def beamform(enu, n_pol: int, k, az_el, x, f0: float = 100e6,
             fs: float = 200e6, M: int = M_DEFAULT, gain=None) -> np.ndarray:
    """x: [n_sb][n_t][n_st*n_pol][2] (ints or floats, taken as FP64);
    returns [B][n_sb][n_t]."""
    enu = np.ascontiguousarray(enu, dtype=np.float64)
    n_st = enu.shape[0]
    k = np.ascontiguousarray(k, dtype=np.int32)
    az_el = np.ascontiguousarray(az_el, dtype=np.float64).reshape(-1, 2)
    n_sb, n_t = x.shape[0], x.shape[1]
    assert x.shape[2] == n_st * n_pol and x.shape[3] == 2
    g = None if gain is None else np.ascontiguousarray(gain, np.float64)
    y = np.zeros((az_el.shape[0], n_sb, n_t), dtype=np.complex128)
    # Subbands are independent: convert and sum a few at a time so a large
    # integer block is never held whole in FP64.
    step = max(1, (1 << 27) // max(1, n_t * n_st * n_pol * 2))
    for s0 in range(0, n_sb, step):
        s1 = min(n_sb, s0 + step)
        xs = np.ascontiguousarray(x[s0:s1], dtype=np.float64)
        ys = np.zeros((az_el.shape[0], s1 - s0, n_t), dtype=np.complex128)
        lib().lpo_beamform(n_st, n_pol, _dp(enu),
                           None if g is None else _dp(g), s1 - s0,
                           _ip(k[s0:s1]), f0, fs, M, az_el.shape[0],
                           _dp(az_el), n_t, _dp(xs), _dp(ys.view(np.float64)))
        y[:, s0:s1] = ys
    return y


def chirp(f_k: float, tec: float, n_fft: int = N_FFT, delay: int = DELAY,
          df: float = 200e6 / M_DEFAULT) -> np.ndarray:
    c = np.zeros(n_fft, dtype=np.complex128)
    lib().lpo_chirp(f_k, tec, n_fft, delay, df, _dp(c.view(np.float64)))
    return c


def dedisperse(k, tec, y, tail, f0: float = 100e6, fs: float = 200e6,
               M: int = M_DEFAULT, n_fft: int = N_FFT, hop: int = HOP,
               delay: int = DELAY) -> np.ndarray:
    """y: [B][S][n_t]; tail: [B][S][n_fft-hop] updated in place.

    Returns d: [B][J][S][n_t]."""
    k = np.ascontiguousarray(k, dtype=np.int32)
    tec = np.ascontiguousarray(np.atleast_1d(tec), dtype=np.float64)
    y = _c128(y)
    B, S, n_t = y.shape
    assert tail.dtype == np.complex128 and tail.flags.c_contiguous
    assert tail.shape == (B, S, n_fft - hop)
    d = np.zeros((B, len(tec), S, n_t), dtype=np.complex128)
    rc = lib().lpo_dedisperse(S, _ip(k), f0, fs, M, len(tec), _dp(tec),
                              n_fft, hop, delay, B, n_t,
                              _dp(y.view(np.float64)),
                              _dp(tail.view(np.float64)),
                              _dp(d.view(np.float64)))
    if rc != 0:
        raise ValueError("lpo_dedisperse: bad arguments")
    return d


def synthesize(h, k, d, hist, M: int = M_DEFAULT,
               P: int = P_DEFAULT) -> np.ndarray:
    """d: [n_series][S][n_t]; hist: [n_series][P-1][S] updated in place.

    Returns z: [n_series][n_t*M] (analytic; real series is 2*Re z)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.int32)
    d = _c128(d)
    ns, S, n_t = d.shape
    assert hist.dtype == np.complex128 and hist.flags.c_contiguous
    assert hist.shape == (ns, P - 1, S)
    z = np.zeros((ns, n_t * M), dtype=np.complex128)
    lib().lpo_synthesize(M, P, _dp(h), S, _ip(k), ns, n_t,
                         _dp(d.view(np.float64)), _dp(hist.view(np.float64)),
                         _dp(z.view(np.float64)))
    return z


def detect(z, n_t: int, frame0: int, warm: int, M: int = M_DEFAULT):
    """Returns sigma [ns], wmax [ns][n_t], warg [ns][n_t]."""
    z = _c128(z)
    ns = z.shape[0]
    assert z.shape[1] == n_t * M
    sigma = np.zeros(ns)
    wmax = np.zeros((ns, n_t))
    warg = np.zeros((ns, n_t), dtype=np.int64)
    lib().lpo_detect(M, n_t, frame0, warm, ns, _dp(z.view(np.float64)),
                     _dp(sigma), _dp(wmax),
                     warg.ctypes.data_as(C.POINTER(C.c_int64)))
    return sigma, wmax, warg


TRIG_DTYPE = np.dtype([("sample", np.int64), ("beam", np.int32),
                       ("tec", np.int32), ("snr", np.float64),
                       ("peak", np.float64)])


def trigger(sigma, wmax, warg, n_beams: int, n_tec: int, n_t: int,
            frame0: int, warm: int, k_sigma: float = 6.0,
            M: int = M_DEFAULT, P: int = P_DEFAULT, D: int = DELAY):
    """Returns (triggers structured array, snr_peak [B][J], best_tec [B])."""
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    wmax = np.ascontiguousarray(wmax, dtype=np.float64)
    warg = np.ascontiguousarray(warg, dtype=np.int64)
    snr_peak = np.zeros((n_beams, n_tec))
    best = np.zeros(n_beams, dtype=np.int32)
    cap = 1024
    while True:
        out = np.zeros(cap, dtype=TRIG_DTYPE)
        n = lib().lpo_trigger(M, P, D, n_t, frame0, warm, n_beams, n_tec,
                              _dp(sigma), _dp(wmax),
                              warg.ctypes.data_as(C.POINTER(C.c_int64)),
                              k_sigma, cap, out.ctypes.data, _dp(snr_peak),
                              _ip(best))
        if n <= cap:
            return out[:n].copy(), snr_peak, best
        cap = n


@dataclass
class BlockResult:
    y: np.ndarray
    d: np.ndarray
    z: np.ndarray
    sigma: np.ndarray
    wmax: np.ndarray
    warg: np.ndarray
    triggers: np.ndarray
    snr_peak: np.ndarray
    best_tec: np.ndarray


@dataclass
class Stream:
    """The whole chain over consecutive blocks of one observation stream,
    with the overlap-save tail and synthesis history carried between
    blocks (both zero at the stream origin)."""

    enu: np.ndarray
    n_pol: int
    k: np.ndarray
    az_el: np.ndarray
    tec: np.ndarray
    f0: float = 100e6
    fs: float = 200e6
    beta: float = 9.0
    k_sigma: float = 6.0
    gain: np.ndarray | None = None
    series_group: int = 0          # synthesise this many series at a time
    keep_z: bool = True            # return the analytic series
    frame0: int = 0
    h: np.ndarray = field(init=False)
    tail: np.ndarray = field(init=False)
    hist: np.ndarray = field(init=False)

    def __post_init__(self):
        self.k = np.asarray(self.k, dtype=np.int32)
        self.az_el = np.asarray(self.az_el, dtype=np.float64).reshape(-1, 2)
        self.tec = np.atleast_1d(np.asarray(self.tec, dtype=np.float64))
        self.h = prototype(M_DEFAULT, P_DEFAULT, self.beta)
        B, S, J = self.az_el.shape[0], len(self.k), len(self.tec)
        self.tail = np.zeros((B, S, N_FFT - HOP), dtype=np.complex128)
        self.hist = np.zeros((B * J, P_DEFAULT - 1, S), dtype=np.complex128)

    @property
    def warm(self) -> int:
        return DELAY + P_DEFAULT

    def process(self, x) -> BlockResult:
        n_t = x.shape[1]
        B, S, J = self.az_el.shape[0], len(self.k), len(self.tec)
        y = beamform(self.enu, self.n_pol, self.k, self.az_el, x, self.f0,
                     self.fs, gain=self.gain)
        d = dedisperse(self.k, self.tec, y, self.tail, self.f0, self.fs)
        # Series are independent from here to the trigger: synthesise and
        # detect a group at a time (only memory changes with the group).
        ns = B * J
        dq = d.reshape(ns, S, n_t)
        g = self.series_group or ns
        zs = []
        sigma = np.zeros(ns)
        wmax = np.zeros((ns, n_t))
        warg = np.zeros((ns, n_t), dtype=np.int64)
        for q0 in range(0, ns, g):
            q1 = min(ns, q0 + g)
            hq = np.ascontiguousarray(self.hist[q0:q1])
            zq = synthesize(self.h, self.k, dq[q0:q1], hq)
            self.hist[q0:q1] = hq
            sigma[q0:q1], wmax[q0:q1], warg[q0:q1] = detect(
                zq, n_t, self.frame0, self.warm)
            if self.keep_z:
                zs.append(zq)
        z = np.concatenate(zs) if self.keep_z else None
        trig, snr_peak, best = trigger(sigma, wmax, warg, B, J, n_t,
                                       self.frame0, self.warm, self.k_sigma)
        self.frame0 += n_t
        return BlockResult(y, d, z, sigma, wmax, warg, trig, snr_peak, best)
