"""Pins for the oracle's radix-2 FFT, Bessel I0 and PPF prototype.

The FFT is checked against the DFT written as a brute-force sum and against
numpy's FFT; I0 against scipy and its large-x asymptotic series; the
prototype against numpy's own Kaiser window (an independent I0) and against
its defining properties (symmetry, unit sum, polyphase partition of unity).
"""
import numpy as np
import pytest
import scipy.special


def brute_dft(x, sign):
    n = len(x)
    out = np.zeros(n, dtype=np.complex128)
    for q in range(n):
        acc = 0j
        for m in range(n):
            acc += x[m] * np.exp(sign * 2j * np.pi * q * m / n)
        out[q] = acc
    return out


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64])
def test_fft_vs_brute_dft(oracle_lib, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = oracle_lib.fft(x)
    ref = brute_dft(x, -1)
    assert np.max(np.abs(X - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    xi = oracle_lib.fft(x, inverse=True)
    refi = brute_dft(x, +1) / n
    assert np.max(np.abs(xi - refi)) <= 1e-12 * max(1.0, np.max(np.abs(refi)))


def test_fft_1024_vs_matrix_dft_and_numpy(oracle_lib):
    n = 1024
    rng = np.random.default_rng(7)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    q = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(q, q) / n)
    X = oracle_lib.fft(x)
    ref = F @ x
    assert np.max(np.abs(X - ref)) / np.max(np.abs(ref)) < 1e-12
    assert np.max(np.abs(X - np.fft.fft(x))) / np.max(np.abs(ref)) < 1e-13


def test_fft_parseval_impulse_tone_roundtrip(oracle_lib):
    n = 4096
    rng = np.random.default_rng(3)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = oracle_lib.fft(x)
    assert abs(np.sum(np.abs(X) ** 2) / n - np.sum(np.abs(x) ** 2)) < 1e-10 * np.sum(np.abs(x) ** 2)
    back = oracle_lib.fft(X, inverse=True)
    assert np.max(np.abs(back - x)) < 1e-12
    imp = np.zeros(n, complex)
    imp[0] = 1.0
    assert np.max(np.abs(oracle_lib.fft(imp) - 1.0)) < 1e-15
    tone = np.exp(2j * np.pi * 37 * np.arange(n) / n)
    T = oracle_lib.fft(tone)
    assert abs(T[37] - n) < 1e-9
    T[37] = 0
    assert np.max(np.abs(T)) < 1e-9


def test_bessel_i0(oracle_lib):
    assert oracle_lib.bessel_i0(0.0) == 1.0
    for x in [0.1, 1.0, 2.5, 9.0, 20.0]:
        assert abs(oracle_lib.bessel_i0(x) / scipy.special.i0(x) - 1) < 1e-14
    # Large-x asymptotic series e^x / sqrt(2 pi x) * sum (2m-1)!!^2/(m! (8x)^m)
    for x in [40.0, 60.0]:
        s, term = 1.0, 1.0
        for m in range(1, 12):
            term *= (2 * m - 1) ** 2 / (m * 8.0 * x)
            s += term
        asym = np.exp(x) / np.sqrt(2 * np.pi * x) * s
        assert abs(oracle_lib.bessel_i0(x) / asym - 1) < 1e-12


def test_prototype_properties(oracle_lib):
    M, P, beta = 1024, 16, 9.0
    h = oracle_lib.prototype(M, P, beta)
    L = M * P
    assert h.shape == (L,)
    assert abs(h.sum() - 1.0) < 1e-13
    assert np.max(np.abs(h - h[::-1])) < 1e-17
    # numpy's Kaiser window uses its own I0 approximation.
    ref = np.kaiser(L, beta) * np.sinc((np.arange(L) - (L - 1) / 2) / M)
    ref /= ref.sum()
    assert np.max(np.abs(h - ref)) < 1e-12 * np.max(h)
    # Polyphase partition of unity: sum_t h[tM + n] ~ 1/M for every n.
    part = h.reshape(P, M).sum(0) * M
    ripple = np.max(np.abs(part - 1.0))
    assert ripple < 2e-3, ripple   # stated ripple: measured ~1e-3


def test_kappa_textbook(oracle_lib):
    # Ionospheric range delay 40.3 TEC / f^2 metres: 1 TECU at GPS L1
    # (1575.42 MHz) delays by ~0.1624 m (textbook value).
    kap = oracle_lib.kappa()
    c = oracle_lib.speed_of_light()
    delay_m = kap * 1.0 / 1575.42e6 ** 2 * c
    assert abs(delay_m - 0.1624) < 2e-4
    # Phase at 10 TECU, 110 MHz is ~767.998 rad; group delay ~1.111 us.
    assert abs(2 * np.pi * kap * 10 / 110e6 - 767.998) < 5e-3
    assert abs(kap * 10 / 110e6 ** 2 - 1.111e-6) < 1e-9
