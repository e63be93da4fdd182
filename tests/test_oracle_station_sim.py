"""Pins of the station-simulator oracle (oracle/station_sim.py).

  * noise: exact Binomial(32 R, 1/2) moments (mean 0, variance 8 R) and its
    histogram against the binomial pmf (chi-square); independence across
    inputs and samples (correlations); counter-based: any split of a
    sample range gives the same codes;
  * pulse and ADC rules: round half to even, saturation at the ADC range;
  * station PPF: equal to the oracle's direct-sum analysis filterbank with
    the stated frame alignment (output frame m sees ADC frames m .. m+15);
    a tone at a subband centre gives |y| = A/2 per unit scale; rounding and
    saturation of the output codes.
"""
import numpy as np
from scipy import stats

import oracle
from oracle import station_sim as ss


def test_noise_is_binomial():
    R = 4
    c = ss.adc(seed=0x1234_5678_9abc, n_in=3, noise_words=R, adc_bits=16,
               n0=10_000, n_samp=1 << 16)
    v = c.astype(np.float64).ravel()
    n = v.size
    assert abs(v.mean()) < 5 * np.sqrt(8 * R / n)
    assert abs(v.var() / (8 * R) - 1) < 5 * np.sqrt(2 / n)
    # Histogram against Binomial(128, 1/2) - 64 over the central values.
    vals, cnt = np.unique(c.astype(np.int64).ravel(), return_counts=True)
    pmf = stats.binom.pmf(vals + 16 * R, 32 * R, 0.5) * n
    keep = pmf > 20
    chi2 = np.sum((cnt[keep] - pmf[keep]) ** 2 / pmf[keep])
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4
    # Inputs and neighbouring samples are uncorrelated.
    x = c.astype(np.float64)
    assert abs(np.corrcoef(x[0], x[1])[0, 1]) < 5 / np.sqrt(x.shape[1])
    assert abs(np.corrcoef(x[0, :-1], x[0, 1:])[0, 1]) < 5 / np.sqrt(x.shape[1])


def test_counter_based_splits_agree_and_seeds_differ():
    a = ss.adc(7, 2, 3, 12, 1000, 4096)
    b = np.concatenate([ss.adc(7, 2, 3, 12, 1000, 1000),
                        ss.adc(7, 2, 3, 12, 2000, 3096)], axis=1)
    assert np.array_equal(a, b)
    c = ss.adc(8, 2, 3, 12, 1000, 4096)
    assert np.mean(a == c) < 0.2
    # Samples beyond 2^32 use the high counter word.
    d = ss.adc(7, 1, 1, 12, (1 << 32) - 2, 4)
    e = ss.adc(7, 1, 1, 12, 0, 4)
    assert not np.array_equal(d[0, 2:], e[0, :2])


def test_pulse_rounding_and_saturation():
    pulse = np.array([[0.5, 1.5, 2.5, -0.5, -1.5, 5000.0, -5000.0, 3.49]],
                     dtype=np.float32)
    base = ss.adc(1, 1, 1, 12, 0, 16)
    got = ss.adc(1, 1, 1, 12, 0, 16, pulse=pulse, pulse_n0=4)
    add = np.array([0, 2, 2, 0, -2, 0, 0, 3])          # half to even
    exp = base.astype(np.int64)
    exp[0, 4:12] += add
    exp[0, 9] = 2047
    exp[0, 10] = -2048
    assert np.array_equal(got, exp.astype(np.int16))


def test_station_ppf_is_the_direct_sum():
    M, P = 64, 16
    h = oracle.prototype(M, P, 9.0)
    k = np.array([3, 7, 8, 20])
    nf = 5
    rng = np.random.default_rng(0)
    codes = rng.integers(-300, 300, size=(2, (nf + P - 1) * M)).astype(np.int16)
    got = ss.station_ppf(h, M, k, codes, 1.0 / 64, 16)
    for i in range(2):
        x = codes[i].astype(np.complex128)
        # y_s[m] = sum_l h[l] e^{+2 pi i k l / M} adc[(m + 16) M - 1 - l]
        # = lpo_analysis frame (m + 16) of the stream shifted by one sample.
        xo = np.concatenate([[0.0], x])
        ref = oracle.analysis(h, M, P, xo, P, nf, k) / 64
        assert np.array_equal(got[:, :, i, 0], np.clip(np.rint(ref.real), -32768, 32767))
        assert np.array_equal(got[:, :, i, 1], np.clip(np.rint(ref.imag), -32768, 32767))


def test_station_ppf_tone_gain_and_saturation():
    M, P = 1024, 16
    h = oracle.prototype(M, P, 9.0)
    k = np.array([100, 101])
    nf = 8
    n = np.arange((nf + P - 1) * M)
    A = 1000.0
    codes = np.rint(A * np.cos(2 * np.pi * 100 * n / M)).astype(np.int16)[None]
    y = ss.station_ppf(h, M, k, codes, 1.0 / 8, 16)
    mag = np.hypot(y[0, :, 0, 0].astype(float), y[0, :, 0, 1].astype(float))
    assert np.all(np.abs(mag - A / 2 / 8) <= 1.0)
    assert np.all(np.abs(y[1, :, 0, :]) <= 2)             # next channel: ~0
    y8 = ss.station_ppf(h, M, k, codes, 1.0, 8)
    assert y8.dtype == np.int8
    assert np.abs(y8[0].astype(int)).max() in (127, 128)
