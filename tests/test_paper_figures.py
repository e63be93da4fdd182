"""The figures the paper states (tests/golden/paper_figures.txt, each with
its section) against the constants of the library and the oracle and the
work model bench.py reports rooflines with.

Sec. 2 fixes the sampling (5 ns, ~5 us subbands, > 6.4 Gbit/s per station);
Sec. 3 gives the cost rules (8 FLOP per station sample and beam, 2e8
complex samples per station, 6 FLOP per complex multiply, 5 N log2 N per
FFT) and the totals they imply.
"""
import math
import os

import pytest

import bench
import lofarsim
import oracle
from paper_1612_06592_amd import lp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_figures.txt")

FS = 200e6        # the library's and the oracle's sampling rate (band default)
M = oracle.M_DEFAULT
N_KEPT = 512      # subbands a station can send (bins 0..511)


@pytest.fixture(scope="module")
def fig():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            name, value = line.split()[:2]
            out[name] = float(value)
    return out


def test_sampling_and_subbands(fig):
    assert lp.LP_M == M == 1024
    assert 1.0 / FS == pytest.approx(fig["adc_sample_interval"], rel=1e-12)
    # One subband sample spans M ADC samples: 5.12 us, "about 5 us".
    assert M / FS == pytest.approx(fig["subband_time_resolution"], rel=0.05)


def test_station_data_rate(fig):
    # 512 subbands of fs / M, two polarisations, 16-bit real and imaginary
    # parts: exactly the stated rate, and 2e8 complex samples per station.
    complex_rate = N_KEPT * FS / M * 2
    assert complex_rate == pytest.approx(fig["station_complex_rate"], rel=1e-12)
    assert complex_rate * 2 * 16 == pytest.approx(fig["station_data_rate"],
                                                  rel=1e-12)


def test_beamforming_cost(fig):
    assert fig["beamform_flop_per_sample"] * fig["station_complex_rate"] == \
        pytest.approx(fig["beamform_rate_per_station"], rel=1e-12)
    # The reported work: 8 FLOP per input sample, subband and beam.
    cfg = lofarsim.get_config("c3")
    per = bench.algorithmic_flop("beamform", cfg, cfg.n_t) / (
        cfg.n_in * cfg.n_sb * cfg.n_t * cfg.n_beams)
    assert per == fig["beamform_flop_per_sample"]


def test_dedispersion_cost(fig):
    c6, c5 = fig["complex_multiply_flop"], fig["fft_flop_coefficient"]
    # The stated ~27 GFLOP/s per beam is the rule (forward and inverse
    # N-point FFT plus one chirp multiply per sample) at 2e8 samples/s with
    # N = 2^13.
    rate = fig["station_complex_rate"] * (2 * c5 * 13 + c6)
    assert rate == pytest.approx(fig["dedispersion_rate_per_beam"], rel=0.02)
    # The reported work, per beam-subband-sample, for the overlap-save form
    # (4096-point transforms, 2048 new samples each): the forward transform
    # once, the chirp (4096 products) and the inverse per trial.
    n, hop = 4096, 2048
    fwd = c5 * n * math.log2(n) / hop
    trial = (c6 * n + c5 * n * math.log2(n)) / hop
    for J in (1, 32):
        cfg = lofarsim.get_config("c4", tec=tuple(float(t) for t in range(J)),
                                  true_tec_index=0)
        per = bench.algorithmic_flop("dedisperse", cfg, cfg.n_t) / (
            cfg.n_sb * cfg.n_t * cfg.n_beams)
        assert per == pytest.approx(fwd + J * trial, rel=1e-12)


def test_synthesis_cost(fig):
    # Per 5 ns output sample: the 1024-point transform (5 log2 1024), the
    # 16-tap complex-by-real FIR (16 x 4) and 6 for envelope and statistics.
    c5 = fig["fft_flop_coefficient"]
    cfg = lofarsim.get_config("c2")
    per = bench.algorithmic_flop("synthesize", cfg, cfg.n_t) / (
        cfg.n_beams * cfg.n_tec * cfg.n_t * M)
    assert per == pytest.approx(c5 * math.log2(M) + 16 * 4 + 6, rel=1e-12)


def test_deadline_and_iterations(fig):
    # The transient buffer sets the block deadline bench.py reports (C2:
    # 5 s less the 335.5 ms block); the PPF-inversion leg runs the stated
    # number of LSMR iterations by default.
    cfg = lofarsim.get_config("c2")
    block_s = cfg.n_t * M / FS
    assert fig["transient_buffer_length"] - block_s == pytest.approx(4.6645,
                                                                    abs=1e-3)
    assert bench.LSMR_ITERS == fig["lsmr_iterations"]
