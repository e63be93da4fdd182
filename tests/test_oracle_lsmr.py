"""Pins of the oracle's PPF inversion (LSMR on H x = y, Sec. 3 of the
paper; LSMR of Fong & Saunders 2011).

Independent references:
  * H against the oracle's direct-sum analysis filterbank (a different
    code path: no polyphase split, no FFT), with the frame alignment that
    the operator's definition states;
  * H^T against the conjugate transpose of H's dense matrix, built column
    by column from that same direct sum, and by the dot-product test;
  * the LSMR iterates against scipy's implementation of LSMR on the same
    operator (a third-party implementation of the published method);
  * convergence to the minimum-norm least-squares solution of the dense
    system (numpy's pseudo-inverse);
  * LSMR's defining property: ||A^T r_k|| decreases monotonically, and the
    recurrence's |zetabar| equals ||A^T r_k|| computed from x_k;
  * exact recovery of a signal in the row space of H, and zero input.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from oracle import ppf_lsmr as pl


def _setup(M, P, F, k, seed=0):
    h = oracle.prototype(M, P, 9.0)
    rng = np.random.default_rng(seed)
    return h, rng, np.asarray(k)


def _dense(h, M, P, k, F):
    """H as a dense complex matrix [len(k) * n_frames][F M], columns from
    the direct-sum analysis of unit impulses."""
    nf = F + P - 1
    A = np.zeros((len(k) * nf, F * M), dtype=np.complex128)
    for n in range(F * M):
        e = np.zeros(F * M + 1, dtype=np.complex128)
        e[n + 1] = 1.0           # x_o[n + 1] = x[n]: frame m of H is frame m + 1
        A[:, n] = oracle.analysis(h, M, P, e, 1, nf, k).reshape(-1)
    return A


def _real_op(h, M, k, F, P):
    nf = F + P - 1
    S = len(k)

    def mv(x):
        y = pl.analysis(h, M, k, x).reshape(-1)
        return np.concatenate([y.real, y.imag])

    def rmv(w):
        y = (w[:S * nf] + 1j * w[S * nf:]).reshape(S, nf)
        return pl.adjoint(h, M, k, y)

    return spla.LinearOperator((2 * S * nf, F * M), matvec=mv, rmatvec=rmv,
                               dtype=np.float64)


def test_analysis_is_the_direct_sum():
    M, P, F = 64, 16, 7
    h, rng, k = _setup(M, P, F, [1, 3, 5, 6, 9, 20, 31])
    x = rng.standard_normal(F * M)
    y = pl.analysis(h, M, k, x)
    xo = np.concatenate([[0.0], x]).astype(np.complex128)
    yd = oracle.analysis(h, M, P, xo, 1, F + P - 1, k)
    assert y.shape == (len(k), F + P - 1)
    assert np.abs(y - yd).max() <= 1e-13 * np.abs(yd).max()


def test_adjoint_is_the_conjugate_transpose():
    M, P, F = 16, 4, 3
    h, rng, k = _setup(M, P, F, [1, 2, 5, 7])
    A = _dense(h, M, P, k, F)
    y = rng.standard_normal((len(k), F + P - 1)) + \
        1j * rng.standard_normal((len(k), F + P - 1))
    ref = (A.conj().T @ y.reshape(-1)).real
    got = pl.adjoint(h, M, k, y)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    x = rng.standard_normal(F * M)
    assert np.abs(pl.analysis(h, M, k, x).reshape(-1) - A @ x).max() <= \
        1e-13 * np.abs(A @ x).max()


@pytest.mark.parametrize("M,P,F", [(64, 16, 5), (1024, 16, 3)])
def test_dot_product(M, P, F):
    h, rng, k = _setup(M, P, F, range(M // 8, M // 8 + M // 5))
    x = rng.standard_normal(F * M)
    y = rng.standard_normal((len(k), F + P - 1)) + \
        1j * rng.standard_normal((len(k), F + P - 1))
    a = np.real(np.vdot(pl.analysis(h, M, k, x), y))
    b = np.dot(x, pl.adjoint(h, M, k, y))
    assert abs(a - b) <= 1e-12 * (abs(a) + 1e-300) * 10


@pytest.mark.parametrize("iters", [1, 2, 5, 25])
def test_iterates_match_scipy_lsmr(iters):
    M, P, F = 64, 16, 12
    h, rng, k = _setup(M, P, F, [2, 3, 4, 5, 6, 7, 8, 11, 12, 13, 20, 25], 3)
    y = rng.standard_normal((len(k), F + P - 1)) + \
        1j * rng.standard_normal((len(k), F + P - 1))
    x, an = pl.invert(h, M, k, y, iters)
    op = _real_op(h, M, k, F, P)
    b = np.concatenate([y.real.reshape(-1), y.imag.reshape(-1)])
    out = spla.lsmr(op, b, damp=0.0, atol=0.0, btol=0.0, conlim=0.0,
                    maxiter=iters)
    xs, itn, normr = out[0], out[2], out[3]
    assert itn == iters
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    # scipy's own estimate of ||r_k|| (its recurrence, not ours) agrees
    # with the residual of our iterate.
    r = np.linalg.norm(b - op.matvec(x))
    assert abs(r - normr) <= 1e-9 * r


def test_converges_to_minimum_norm_solution():
    """Underdetermined with full row rank (3 of 16 channels, as the
    recorded band is a fraction of all channels); condition number ~3e4
    from the segment's edge frames, so it takes a few hundred iterations."""
    M, P, F = 16, 4, 4
    h, rng, k = _setup(M, P, F, [2, 3, 4])
    A = _dense(h, M, P, k, F)
    Ar = np.concatenate([A.real, A.imag])
    y = rng.standard_normal((len(k), F + P - 1)) + \
        1j * rng.standard_normal((len(k), F + P - 1))
    b = np.concatenate([y.real.reshape(-1), y.imag.reshape(-1)])
    assert np.linalg.matrix_rank(Ar) == Ar.shape[0] < Ar.shape[1]
    ref = np.linalg.pinv(Ar) @ b
    x, an = pl.invert(h, M, k, y, 300)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


def test_anorm_recurrence_is_true_and_monotone():
    M, P, F = 64, 16, 10
    h, rng, k = _setup(M, P, F, range(5, 25), 7)
    y = rng.standard_normal((len(k), F + P - 1)) + \
        1j * rng.standard_normal((len(k), F + P - 1))
    _, an = pl.invert(h, M, k, y, 12)
    assert all(an[i + 1] <= an[i] * (1 + 1e-12) for i in range(len(an) - 1))
    for it in (0, 1, 4, 12):
        x, _ = pl.invert(h, M, k, y, it)
        r = y - pl.analysis(h, M, k, x)
        true = np.linalg.norm(pl.adjoint(h, M, k, r))
        assert abs(true - an[it]) <= 1e-9 * an[0]


def test_recovers_signal_in_row_space():
    """x = H^T z is its own minimum-norm solution: LSMR on y = H x must
    return x; after the paper's 25 iterations the residual is small."""
    M, P, F = 1024, 16, 24
    h, rng, k = _setup(M, P, F, range(52, 296), 11)
    z = rng.standard_normal((len(k), F + P - 1)) + \
        1j * rng.standard_normal((len(k), F + P - 1))
    x = pl.adjoint(h, M, k, z)
    y = pl.analysis(h, M, k, x)
    x25, _ = pl.invert(h, M, k, y, 25)
    r = np.linalg.norm(y - pl.analysis(h, M, k, x25)) / np.linalg.norm(y)
    assert r < 2e-4
    assert np.linalg.norm(x25 - x) / np.linalg.norm(x) < 3e-3
    x80, _ = pl.invert(h, M, k, y, 80)
    assert np.linalg.norm(x80 - x) < np.linalg.norm(x25 - x)


def test_zero_input():
    M, P, F = 64, 16, 4
    h, rng, k = _setup(M, P, F, [3, 4, 5])
    x, an = pl.invert(h, M, k, np.zeros((3, F + P - 1), complex), 25)
    assert x.shape == (F * M,) and not np.any(x) and an == [0.0]


def _band_noise(rng, N, M, k):
    X = np.fft.rfft(rng.standard_normal(N))
    f = np.arange(X.size) / N
    X[(f < (k[0] - 0.5) / M) | (f > (k[-1] + 0.5) / M)] = 0
    return np.fft.irfft(X, N)


def test_fidelity_gain_over_one_shot_synthesis():
    """The gain LSMR buys over the one-shot synthesis filterbank (the trigger
    path's inversion): noise filling the recorded band, including the
    subband crossovers, is reconstructed at ~35 dB after 25 iterations
    against ~14 dB; a tone at a subband edge keeps its amplitude (synthesis:
    -6 dB, the scalloping of two crossing channels)."""
    M, P, F = 1024, 16, 48
    h, rng, k = _setup(M, P, F, range(100, 132), 0)
    N = F * M
    lag = 15 * M + 1           # synthesis delay in this frame alignment
    a, b = 16 * M, N - 16 * M

    def synth(y):
        z = oracle.synthesize(h, k, y[None], np.zeros((1, 15, len(k)), complex))
        seg = 2 * z[0].real[lag:lag + N]
        return np.concatenate([seg, np.zeros(N - seg.size)])

    def snr(v, x):
        return 10 * np.log10(np.sum(x[a:b] ** 2) / np.sum((v - x)[a:b] ** 2))

    x = _band_noise(rng, N, M, k)
    y = pl.analysis(h, M, k, x)
    s_syn = snr(synth(y), x)
    s_lsmr = snr(pl.invert(h, M, k, y, 25)[0], x)
    assert 10 < s_syn < 20 and s_lsmr > 30, (s_syn, s_lsmr)
    n = np.arange(N)
    for d, syn_db in ((0.0, 0.0), (0.25, 0.0), (0.5, -6.02)):
        nu = (115 + d) / M
        xt = np.cos(2 * np.pi * nu * n + 0.3)
        yt = pl.analysis(h, M, k, xt)
        ref = np.exp(2j * np.pi * nu * n[a:b])

        def amp_db(v):
            return 20 * np.log10(abs(np.dot(v[a:b], np.conj(ref))) / ((b - a) / 2))

        assert abs(amp_db(synth(yt)) - syn_db) < 0.05
        assert abs(amp_db(pl.invert(h, M, k, yt, 25)[0])) < 0.01
