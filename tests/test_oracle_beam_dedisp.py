"""Pins for the oracle's beamformer and de-dispersion.

Beamformer: a plane-wave tone at a subband centre frequency, built from the
station geometry, adds up to the coherent gain N_st per polarisation toward
its source and to less off-source; a random case matches numpy einsum with
weights built from the plane-wave delays.

De-dispersion: at T = 0 it is an exact delay of D subband samples; two
chirps compose (T1 then T2 equals T1 + T2, up to a second delay D); a
pulse dispersed at T (through the generator's independent forward model)
and de-dispersed at T comes back at its injected ADC index, with most of
its undispersed peak, and de-dispersing at T +- 5 TECU loses peak; the
overlap-save state makes two half blocks equal one whole block.
"""
import numpy as np

import lofarsim
from lofarsim.generate import _pulse_subbands, kaiser_sinc

C = 299792458.0


def _dir(az, el):
    return np.array([np.cos(el) * np.sin(az), np.cos(el) * np.cos(az), np.sin(el)])


def test_plane_wave_coherent_gain(oracle_lib):
    rng = np.random.default_rng(3)
    n_st, M, fs, f0 = 24, 1024, 200e6, 100e6
    enu = np.c_[rng.uniform(-1000, 1000, (n_st, 2)), np.zeros(n_st)]
    k = np.array([60, 205, 290])
    src = (1.1, 0.7)
    A, n_t = 5.0, 8
    x = np.zeros((k.size, n_t, n_st * 2, 2))
    for s, kk in enumerate(k):
        f = f0 + kk * fs / M
        for st in range(n_st):
            tau = -(enu[st] @ _dir(*src)) / C
            v = A * np.exp(-2j * np.pi * f * tau) * np.exp(2j * np.pi * 0.1 * np.arange(n_t))
            x[s, :, 2 * st, 0] = v.real       # polarisation 0 only
            x[s, :, 2 * st, 1] = v.imag
    az_el = np.array([src, (1.1 + 0.01, 0.7), (1.0, 0.75)])
    y = oracle_lib.beamform(enu, 2, k, az_el, x)
    assert np.max(np.abs(np.abs(y[0]) - n_st * A)) < 1e-9 * n_st * A
    assert np.all(np.abs(y[1:]) < 0.9 * n_st * A)
    # Both polarisations carrying the wave: gain 2 N_st.
    x2 = x.copy()
    x2[:, :, 1::2, :] = x[:, :, 0::2, :]
    y2 = oracle_lib.beamform(enu, 2, k, az_el[:1], x2)
    assert np.max(np.abs(np.abs(y2[0]) - 2 * n_st * A)) < 1e-9 * n_st * A


def test_beamform_vs_einsum(oracle_lib):
    rng = np.random.default_rng(8)
    n_st, n_pol, M, fs, f0 = 5, 2, 1024, 200e6, 100e6
    enu = rng.uniform(-150, 150, (n_st, 3))
    enu[:, 2] = 0
    k = np.array([190, 191, 220])
    az_el = np.array([[0.3, 0.8], [2.0, 0.5]])
    gain = rng.uniform(0.5, 2.0, n_st * n_pol)
    x = rng.integers(-100, 100, (k.size, 7, n_st * n_pol, 2))
    y = oracle_lib.beamform(enu, n_pol, k, az_el, x, gain=gain)
    f = f0 + k * fs / M
    delays = np.stack([enu @ _dir(*d) / C for d in az_el])       # [B][st]
    w = np.exp(-2j * np.pi * f[None, :, None] * delays[:, None, :])  # B,S,st
    w = np.repeat(w, n_pol, axis=2) * gain[None, None, :]
    xc = x[..., 0] + 1j * x[..., 1]
    ref = np.einsum("bsi,sti->bst", w, xc)
    assert np.max(np.abs(y - ref)) < 1e-10 * np.max(np.abs(ref))


def test_chirp_phase_identity_and_composition(oracle_lib):
    df = 200e6 / 1024
    kap = oracle_lib.kappa()
    f_k = 110e6
    c = oracle_lib.chirp(f_k, 10.0, 4096, 0, df)
    # Bin 0 (nu = 0): phase -2 pi kappa T / f mod 2 pi.
    expect = np.exp(-2j * np.pi * kap * 10.0 / f_k)
    assert abs(c[0] - expect) < 1e-12
    c0 = oracle_lib.chirp(f_k, 0.0, 4096, 1024, df)
    q = np.arange(4096)
    qs = np.where(q < 2048, q, q - 4096)
    assert np.max(np.abs(c0 - np.exp(-2j * np.pi * qs * 1024 / 4096))) < 1e-12
    c1 = oracle_lib.chirp(f_k, 7.0, 4096, 1024, df)
    c2 = oracle_lib.chirp(f_k, 13.0, 4096, 1024, df)
    c12 = oracle_lib.chirp(f_k, 20.0, 4096, 2048, df)
    assert np.max(np.abs(c1 * c2 - c12)) < 1e-11


def test_dedisperse_tec0_is_pure_delay(oracle_lib):
    rng = np.random.default_rng(2)
    B, S, n_t = 2, 3, 8192
    y = rng.standard_normal((B, S, n_t)) + 1j * rng.standard_normal((B, S, n_t))
    tail = np.zeros((B, S, 2048), complex)
    d = oracle_lib.dedisperse(np.array([60, 61, 62]), [0.0], y, tail)
    D = 1024
    assert np.max(np.abs(d[:, 0, :, D:] - y[:, :, :-D])) < 1e-12
    assert np.max(np.abs(d[:, 0, :, :D])) < 1e-12
    assert np.array_equal(tail, y[:, :, -2048:])


def test_dedisperse_stream_split_equals_whole(oracle_lib):
    rng = np.random.default_rng(6)
    B, S, n_t = 1, 2, 8192
    y = rng.standard_normal((B, S, n_t)) + 1j * rng.standard_normal((B, S, n_t))
    k = np.array([100, 250])
    tecs = [3.0, 25.0]
    t1 = np.zeros((B, S, 2048), complex)
    whole = oracle_lib.dedisperse(k, tecs, y, t1)
    t2 = np.zeros((B, S, 2048), complex)
    a = oracle_lib.dedisperse(k, tecs, y[:, :, :4096].copy(), t2)
    b = oracle_lib.dedisperse(k, tecs, y[:, :, 4096:].copy(), t2)
    assert np.array_equal(np.concatenate([a, b], axis=-1), whole)


def _dispersed_pulse_peak(oracle_lib, tec_true, tec_trial, n0):
    cfg = lofarsim.get_config("c2", n_t=4096, tec=(tec_trial,),
                              true_tec=tec_trial)
    enu = np.zeros((1, 3))
    h = kaiser_sinc(1024, 16)
    m_first, y, _ = _pulse_subbands(cfg, enu, (0.5, 0.9), n0, 1000.0,
                                    tec_true, h)
    n_t = cfg.n_t
    x = np.zeros((cfg.n_sb, n_t, 2, 2))
    a, b = max(m_first, 0), min(m_first + y.shape[2], n_t)
    for s in range(cfg.n_sb):
        seg = y[0, s, a - m_first:b - m_first]
        x[s, a:b, 0, 0] = seg.real
        x[s, a:b, 0, 1] = seg.imag
    st = oracle_lib.Stream(enu, 2, cfg.k, [(0.5, 0.9)], [tec_trial])
    r = st.process(x)
    e = np.abs(2 * r.z[0])
    i = int(np.argmax(e))
    return i - 1024 * 16 - 1024 * 1024, e[i]


def test_dispersed_pulse_recovered(oracle_lib):
    n0 = 2100 * 1024 + 333
    idx0, ref = _dispersed_pulse_peak(oracle_lib, 0.0, 0.0, n0)
    assert idx0 == n0
    idx, pk = _dispersed_pulse_peak(oracle_lib, 10.0, 10.0, n0)
    assert idx == n0
    assert pk >= 0.95 * ref, pk / ref
    # Wrong trial TEC: the pulse stays smeared.
    for off in (-5.0, 5.0):
        _, pk_off = _dispersed_pulse_peak(oracle_lib, 10.0, 10.0 + off, n0)
        assert pk_off < 0.5 * pk
