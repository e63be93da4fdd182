"""Pins for the oracle's analysis and synthesis filterbanks.

* Analysis: a cosine at a channel centre gives |y_k0| = A/2, constant in
  time, with the other channels at the stopband level; the direct sum
  agrees with an independent polyphase + FFT implementation (the
  generator's station PPF, and a small complex one written here).
* Synthesis is the adjoint of analysis up to a fixed shift and a per-channel
  phase: <A x, y~> = <x, (1/M) S(y)[. + L - 1]>, y~_k = y_k e^{-2 pi i k/M}
  (dot-product test on complex random data with all M channels).
* Analysis then synthesis: an impulse peaks at n0 + L; band-limited signals
  come back to a stated SNR (the inversion is not loss-less).
* Re(2z) equals the Hermitian (irfft-style) synthesis; the envelope of a
  tone is constant; |2z| agrees with an FFT-Hilbert envelope of 2 Re z.
"""
import numpy as np
import pytest

import lofarsim


def polyphase_complex(x, h, M, P, n_frames):
    """Independent analysis: per frame, polyphase sums then an FFT."""
    L = M * P
    ext = np.concatenate([np.zeros(L, complex), x,
                          np.zeros(L + n_frames * M, complex)])
    out = np.zeros((M, n_frames), complex)
    for m in range(n_frames):
        top = L + m * M
        seg = ext[top - L + 1:top + 1][::-1]
        u = (h.reshape(P, M) * seg.reshape(P, M)).sum(0)
        out[:, m] = np.fft.ifft(u) * M
    return out


def test_analysis_vs_polyphase_fft_small(oracle_lib):
    M, P = 16, 4
    h = oracle_lib.prototype(M, P, 5.0)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    y = oracle_lib.analysis(h, M, P, x, 0, 20, np.arange(M))
    ref = polyphase_complex(x, h, M, P, 20)
    assert np.max(np.abs(y - ref)) < 1e-12 * np.max(np.abs(ref))


def test_analysis_vs_generator_station_ppf(oracle_lib):
    M, P = 1024, 16
    h = oracle_lib.prototype(M, P, 9.0)
    rng = np.random.default_rng(5)
    n = 24 * M
    x = rng.standard_normal(n)
    chans = np.array([0, 1, 52, 205, 295, 511, 700])
    y = oracle_lib.analysis(h, M, P, x, 3, 20, chans)
    g = lofarsim.station_ppf(x, 0, lofarsim.kaiser_sinc(M, P, 9.0), M, 3, 20)
    assert np.max(np.abs(y - g[chans])) < 1e-11 * np.max(np.abs(y))


def test_analysis_tone_gain_and_leakage(oracle_lib):
    M, P = 1024, 16
    h = oracle_lib.prototype(M, P, 9.0)
    k0, A = 205, 3.0
    n = 40 * M
    x = A * np.cos(2 * np.pi * k0 * np.arange(n) / M)
    chans = np.array([k0, k0 - 1, k0 + 1, k0 + 5, 100])
    y = oracle_lib.analysis(h, M, P, x, 20, 10, chans)
    # 16384-term sums: rounding and the image at 2*k0 stay below 1e-10.
    assert np.max(np.abs(np.abs(y[0]) - A / 2)) < 1e-10
    # Neighbour channels see the tone at their band edge+: stated level.
    leak_db = 20 * np.log10(np.max(np.abs(y[1:])) / (A / 2))
    assert leak_db < -60, leak_db


def test_synthesis_is_adjoint_dot_product(oracle_lib):
    M, P, F = 16, 4, 12
    L = M * P
    h = oracle_lib.prototype(M, P, 5.0)
    rng = np.random.default_rng(1)
    nx = F * M
    x = rng.standard_normal(nx) + 1j * rng.standard_normal(nx)
    nfr = F + P
    y = np.zeros((M, nfr), complex)
    y[:, :F] = rng.standard_normal((M, F)) + 1j * rng.standard_normal((M, F))
    Ax = oracle_lib.analysis(h, M, P, x, 0, nfr, np.arange(M))
    ytil = y * np.exp(-2j * np.pi * np.arange(M) / M)[:, None]
    lhs = np.vdot(ytil, Ax)                       # sum Ax * conj(ytil)
    hist = np.zeros((1, P - 1, M), complex)
    z = oracle_lib.synthesize(h, np.arange(M), y[None], hist, M=M, P=P)[0]
    Sy = z[L - 1:L - 1 + nx] / M
    rhs = np.vdot(Sy, x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _analysis_synthesis(oracle_lib, x, chans, n_frames, M=1024, P=16):
    h = oracle_lib.prototype(M, P, 9.0)
    y = oracle_lib.analysis(h, M, P, x, 0, n_frames, chans)
    hist = np.zeros((1, P - 1, len(chans)), complex)
    z = oracle_lib.synthesize(h, chans, y[None], hist, M=M, P=P)[0]
    return z


def test_impulse_peaks_at_n0_plus_L(oracle_lib):
    M, P = 1024, 16
    L = M * P
    chans = np.arange(1, 512)
    for n0 in [5 * M, 5 * M + 1, 6 * M + 517, 7 * M - 1]:
        x = np.zeros(40 * M)
        x[n0] = 1.0
        z = _analysis_synthesis(oracle_lib, x, chans, 40)
        e = np.abs(2 * z)
        assert int(np.argmax(e)) == n0 + L


def test_reconstruction_snr_band_limited(oracle_lib):
    """Tones at subband centres and noise confined to the inner +-50% of
    each selected subband: analysis -> synthesis SNR above 50 dB."""
    M, P = 1024, 16
    L = M * P
    chans = np.arange(52, 296)
    n = 96 * M
    t = np.arange(n)
    rng = np.random.default_rng(2)
    x = np.zeros(n)
    for k0 in [60, 150, 290]:
        x += np.cos(2 * np.pi * k0 * t / M + rng.uniform(0, 6.3))
    spec = np.fft.rfft(rng.standard_normal(n))
    fb = np.arange(spec.size) / n * M            # in units of subbands
    keep = np.zeros(spec.size, bool)
    for k in chans:
        keep |= np.abs(fb - k) <= 0.25
    x += 0.3 * np.fft.irfft(np.where(keep, spec, 0), n) * np.sqrt(n)
    z = _analysis_synthesis(oracle_lib, x, chans, 96 + P)
    xr = 2 * z.real
    a, b = 2 * L, n - 2 * L          # interior, away from start-up
    err = xr[a + L:b + L] - x[a:b]
    snr_db = 10 * np.log10(np.sum(x[a:b] ** 2) / np.sum(err ** 2))
    assert snr_db > 50, snr_db
    # The tone envelope is constant (single tone through one subband).
    xt = np.cos(2 * np.pi * 150 * t / M)
    zt = _analysis_synthesis(oracle_lib, xt, chans, 96 + P)
    env = np.abs(2 * zt[a + L:b + L])
    assert np.max(np.abs(env - 1.0)) < 1e-3


def test_real_part_is_hermitian_synthesis_and_hilbert(oracle_lib):
    M, P = 64, 4
    h = oracle_lib.prototype(M, P, 7.0)
    chans = np.arange(3, 29)
    rng = np.random.default_rng(4)
    nt = 40
    d = rng.standard_normal((1, chans.size, nt)) + 1j * rng.standard_normal((1, chans.size, nt))
    hist = np.zeros((1, P - 1, chans.size), complex)
    z = oracle_lib.synthesize(h, chans, d, hist, M=M, P=P)[0]
    # Hermitian synthesis: full spectrum with X_k = d_k and X_{M-k} = conj,
    # real inverse transform (numpy irfft) times M, then the same FIR.
    g = M * h
    Zr = np.zeros((nt, M))
    for m in range(nt):
        spec = np.zeros(M // 2 + 1, complex)
        spec[chans] = d[0, :, m]
        Zr[m] = np.fft.irfft(spec, M) * M
    xr = np.zeros(nt * M)
    for m in range(nt):
        for n in range(M):
            acc = 0.0
            for t in range(P):
                if m - t >= 0:
                    acc += g[t * M + n] * Zr[m - t, n]
            xr[m * M + n] = acc
    assert np.max(np.abs(2 * z.real - xr)) < 1e-12 * np.max(np.abs(xr))


def test_envelope_vs_fft_hilbert_interior(oracle_lib):
    M, P = 1024, 16
    L = M * P
    chans = np.arange(52, 296)
    rng = np.random.default_rng(9)
    n = 128 * M
    spec = np.fft.rfft(rng.standard_normal(n))
    fb = np.arange(spec.size) / n * M
    keep = (fb > 52) & (fb < 295)
    x = np.fft.irfft(np.where(keep, spec, 0), n)
    z = _analysis_synthesis(oracle_lib, x, chans, 128)
    xr = 2 * z.real
    # FFT-Hilbert analytic signal of xr.
    X = np.fft.fft(xr)
    Hh = np.zeros(n)
    Hh[0] = 1
    Hh[1:n // 2] = 2
    Hh[n // 2] = 1
    an = np.fft.ifft(X * Hh)
    a, b = 2 * L, n - 2 * L
    rel = np.sqrt(np.mean(np.abs(an[a:b] - 2 * z[a:b]) ** 2) / np.mean(np.abs(an[a:b]) ** 2))
    assert rel < 1e-3, rel
