"""The station simulator on the GPU (lp_sim_adc, lp_station_ppf) against the
oracle (oracle/station_sim.py), and a simulated pulse through the whole
chain.

ADC codes are integer arithmetic on both sides (Philox4x32-10 and
popcounts): bit-exact.  Station subbands are FP32 on the GPU and FP64 in the
oracle before the same rounding: codes must be equal except where the
oracle's scaled value lies within 1e-3 of a rounding boundary (there the
two precisions may round differently; such codes may differ by one).
"""
import numpy as np
import pytest

import lofarsim
import oracle
from oracle import station_sim as ss
from paper_1612_06592_amd import lp

pytestmark = pytest.mark.gpu

M, P = 1024, 16


def test_adc_codes_bit_exact():
    import torch
    n_in, R, bits = 6, 4, 12
    n0 = (1 << 32) - 40_000                 # crosses the counter's high word
    n = 70_000
    rng = np.random.default_rng(3)
    pulse = (rng.standard_normal((n_in, 5000)) * 300).astype(np.float32)
    pulse[0, :6] = [0.5, 1.5, 2.5, -0.5, 4000.0, -4000.0]
    p0 = n0 + 20_000
    ctx = lp.Ctx(0)
    adc = torch.empty((n_in, n), dtype=torch.int16, device="cuda:0")
    print("case sim adc n_in=6 R=4 12 bits, pulse", flush=True)
    lp.sim_adc(ctx, 0xfeed_beef_1234, n_in, R, bits, n0, n, adc,
               pulse=torch.from_numpy(pulse).to("cuda:0"), pulse_n0=p0)
    torch.cuda.synchronize()
    got = adc.cpu().numpy()
    ref = ss.adc(0xfeed_beef_1234, n_in, R, bits, n0, n, pulse, p0)
    print("mismatching codes:", int(np.sum(got != ref)), flush=True)
    assert np.array_equal(got, ref)
    ctx.close()


@pytest.mark.parametrize("n_in", [4, 8])
@pytest.mark.parametrize("dtype,bits", [(lp.LP_CI8, 8), (lp.LP_CI16, 16)])
def test_station_ppf_matches_oracle(dtype, bits, n_in):
    import torch
    nf = 300
    k = np.arange(52, 84)
    h = oracle.prototype(M, P, 9.0)
    codes = ss.adc(77, n_in, 16, 12, 1, (nf + P - 1) * M)
    sigma_adc = np.sqrt(8 * 16)
    scale = (8.0 if bits == 8 else 200.0) / (sigma_adc * np.sqrt(np.sum(h * h) / 2))
    ref = ss.station_ppf(h, M, k, codes, scale, bits)
    near = ss.boundary_mask(h, M, k, codes, scale, 1e-3)
    ctx = lp.Ctx(0)
    band = lp.Band(k)
    adc = torch.from_numpy(codes).to("cuda:0")
    x = torch.empty((len(k), nf, n_in, 2),
                    dtype=torch.int8 if bits == 8 else torch.int16,
                    device="cuda:0")
    work = torch.empty(lp.nbytes("lp_station_work_bytes", n_in, len(k), nf),
                       dtype=torch.uint8, device="cuda:0")
    print(f"case station ppf n_in={n_in} nf=300 32 subbands, {bits}-bit",
          flush=True)
    lp.station_ppf(ctx, band, adc, n_in, nf, float(scale), x, work, dtype)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    diff = got.astype(np.int64) - ref.astype(np.int64)
    bad = diff != 0
    print(f"codes {got.size}, differing {int(bad.sum())}, "
          f"near a boundary {int(near.sum())}, sigma {got.std():.2f}",
          flush=True)
    assert np.all(np.abs(diff) <= 1)
    assert not np.any(bad & ~near)
    ctx.close()


def test_simulated_pulse_through_the_chain():
    """A dispersed pulse from the beam direction, simulated at 5 ns with
    noise and station filterbank on the GPU, is triggered at its ADC
    sample in the right beam and at the injected TEC trial."""
    import torch
    cfg = lofarsim.get_config("c2", n_t=8192, k=tuple(range(52, 116)),
                              tec=(0.0, 10.0, 20.0), true_tec=10.0,
                              n_pulses=0)
    rng = np.random.default_rng(11)
    enu = lofarsim.stations_in_disk(rng, cfg.n_st, cfg.disk_m)
    az_el = np.array([[1.2, 0.8]])
    n_in, nf = 2 * cfg.n_st, cfg.n_t
    B0 = 16 * M                  # first ADC sample of the block (absolute)
    n0 = B0 + 4000 * M + 321     # the pulse at the array origin
    R = 16
    sigma_adc = np.sqrt(8 * R)
    h = oracle.prototype(M, P, 9.0)
    # Amplitude for a subband-domain SNR of about 25 (the generator's rule
    # with this ADC noise).
    from lofarsim.generate import PULSE_WINDOW as Nw
    fb = np.arange(Nw // 2 + 1) * cfg.fs / Nw
    df = cfg.fs / M
    n_band = int(((fb >= (min(cfg.k) - 0.5) * df) &
                  (fb <= (max(cfg.k) + 0.5) * df)).sum())
    amp = 25 * sigma_adc * np.sqrt(n_band / (Nw / 2)) * Nw / (2 * n_band)
    w0, xs = lofarsim.pulse_waveforms(cfg, enu, tuple(az_el[0]), n0, amp, 10.0)
    pulse = np.repeat(xs, 2, axis=0).astype(np.float32)
    scale = 8.0 / (sigma_adc * np.sqrt(np.sum(h * h) / 2))
    ctx = lp.Ctx(0)
    adc = torch.empty((n_in, (nf + P - 1) * M), dtype=torch.int16,
                      device="cuda:0")
    # The stream starts one sample after B0 - 16 M: then block frame m is
    # the window ending at ADC sample B0 + m M, the generator's frames.
    print("case simulated block 48 inputs x 8192 frames, pulse at", n0 - B0,
          flush=True)
    lp.sim_adc(ctx, 2024, n_in, R, 12, B0 - 16 * M + 1, adc.shape[1], adc,
               pulse=torch.from_numpy(pulse).to("cuda:0"), pulse_n0=w0)
    band = lp.Band(cfg.k)
    x = torch.empty((len(cfg.k), nf, n_in, 2), dtype=torch.int8,
                    device="cuda:0")
    work = torch.empty(lp.nbytes("lp_station_work_bytes", n_in, len(cfg.k), nf),
                       dtype=torch.uint8, device="cuda:0")
    lp.station_ppf(ctx, band, adc, n_in, nf, float(scale), x, work, lp.LP_CI8)
    del adc
    p = lp.Pipeline(ctx, lp.Array(enu, 2), band, lp.Dirs(az_el),
                    np.asarray(cfg.tec), nf)
    p.step(x)
    torch.cuda.synchronize()
    trig = p.triggers()
    print("subband sigma", float(x.float().std()), "triggers",
          [(int(t["sample"]), int(t["tec"]), round(float(t["snr"]), 1))
           for t in trig], flush=True)
    hit = [t for t in trig if abs(int(t["sample"]) - (n0 - B0)) <= 1]
    assert hit, trig
    assert int(hit[0]["beam"]) == 0 and int(hit[0]["tec"]) == 1
    assert float(hit[0]["snr"]) > 12
    ctx.close()
