"""Oracle (test infrastructure only; never on the product path): the station
simulator, in plain numpy.

Winchen et al., Sec. 2: every LOFAR station samples its antennas at 5 ns
(200 MHz real sampling) and its polyphase filterbank forms the ~5 us
subbands that are sent on; Sec. 5: the simulation chain has a module that
turns a time-domain trace into the polyphase-filtered one.  The simulator
produces those station subbands from ADC samples:

ADC samples.  Input i (station x polarisation) at absolute sample n:
    noise_i[n] = sum_{r < R} (popcount(w_r) - 16)
where w_0, w_1, ... are the 32-bit words of Philox4x32-10 (Salmon, Moraes,
Dror & Shaw 2011, "Parallel random numbers: as easy as 1, 2, 3") with key
(seed mod 2^32, seed div 2^32) and counter (n mod 2^32, n div 2^32, i, g)
for g = 0, 1, ... (four words per counter).  This is Binomial(32 R, 1/2)
centred, variance 8 R, in exact integer arithmetic.  A pulse (a float
waveform per input, prepared by the caller) is rounded half to even and
added; the sum saturates to a signed adc_bits-bit code.

Station PPF.  The analysis filterbank (prototype h, M = 1024, 16 taps) over
the ADC stream with 15 frames of history: output frame m of a block sees
ADC frames m .. m + 15 of the given stream,
    y_s[m] = sum_{l < 16384} h[l] exp(+2 pi i k_s l / M) adc[(m + 16) M - 1 - l],
scaled, rounded half to even (real and imaginary parts) and saturated to
the output integer type; layout [n_sb][n_frames][n_in] (the beamformer's).
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Philox4x32 with 10 rounds on arrays of 32-bit counters (uint32)."""
    c = [np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3)]
    k0, k1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return [v.astype(np.uint32) for v in c]


def _popcount32(w):
    w = np.asarray(w, dtype=np.uint32)
    return np.unpackbits(w.view(np.uint8).reshape(w.shape + (4,)),
                         axis=-1).sum(axis=-1).astype(np.int64)


def adc(seed: int, n_in: int, noise_words: int, adc_bits: int, n0: int,
        n_samp: int, pulse=None, pulse_n0: int = 0) -> np.ndarray:
    """ADC codes [n_in][n_samp] (int16) for absolute samples n0 .. n0 +
    n_samp - 1.  pulse: float32 [n_in][len] added from sample pulse_n0."""
    n = np.arange(n0, n0 + n_samp, dtype=np.uint64)
    lo = (n & _MASK).astype(np.uint32)
    hi = (n >> np.uint64(32)).astype(np.uint32)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    out = np.zeros((n_in, n_samp), dtype=np.int64)
    for i in range(n_in):
        acc = np.zeros(n_samp, dtype=np.int64)
        for g in range((noise_words + 3) // 4):
            w = philox4x32_10(lo, hi, np.full(n_samp, i, np.uint32),
                              np.full(n_samp, g, np.uint32), k0, k1)
            for j in range(4):
                if 4 * g + j < noise_words:
                    acc += _popcount32(w[j]) - 16
        out[i] = acc
    if pulse is not None:
        pulse = np.asarray(pulse, dtype=np.float32)
        a = max(n0, pulse_n0)
        b = min(n0 + n_samp, pulse_n0 + pulse.shape[1])
        if a < b:
            out[:, a - n0:b - n0] += np.rint(
                pulse[:, a - pulse_n0:b - pulse_n0]).astype(np.int64)
    lim = 1 << (adc_bits - 1)
    return np.clip(out, -lim, lim - 1).astype(np.int16)


def station_ppf(h: np.ndarray, M: int, k, codes: np.ndarray, scale: float,
                out_bits: int) -> np.ndarray:
    """Station subbands [n_sb][n_frames][n_in][2] (int8 for out_bits 8,
    int16 for 16) from ADC codes [n_in][(n_frames + 15) M]; FP64."""
    from oracle import ppf_lsmr
    n_in, n = codes.shape
    P = h.size // M
    nf = n // M - (P - 1)
    assert nf >= 1 and n == (nf + P - 1) * M
    k = np.asarray(k)
    out = np.zeros((len(k), nf, n_in, 2), dtype=np.int64)
    lim = 1 << (out_bits - 1)
    for i in range(n_in):
        y = ppf_lsmr.analysis(h, M, k, codes[i].astype(np.float64))
        v = y[:, P - 1:P - 1 + nf] * scale           # the valid frames
        out[:, :, i, 0] = np.clip(np.rint(v.real), -lim, lim - 1)
        out[:, :, i, 1] = np.clip(np.rint(v.imag), -lim, lim - 1)
    return out.astype(np.int8 if out_bits == 8 else np.int16)


def boundary_mask(h: np.ndarray, M: int, k, codes: np.ndarray, scale: float,
                  eps: float) -> np.ndarray:
    """True where a scaled subband value lies within eps of a rounding
    boundary (k + 1/2): an FP32 computation may round such a value the
    other way.  Shape as station_ppf's output."""
    from oracle import ppf_lsmr
    n_in, n = codes.shape
    P = h.size // M
    nf = n // M - (P - 1)
    m = np.zeros((len(k), nf, n_in, 2), dtype=bool)
    for i in range(n_in):
        y = ppf_lsmr.analysis(h, M, k, codes[i].astype(np.float64))
        v = y[:, P - 1:P - 1 + nf] * scale
        for c, part in ((0, v.real), (1, v.imag)):
            fr = np.abs(part - np.floor(part) - 0.5)
            m[:, :, i, c] = fr < eps
    return m
