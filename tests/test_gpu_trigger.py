"""lp_trigger alone against the oracle's trigger rules, on candidates built
on the host (seeded), so the list logic is checked exactly and at sizes
where a series has thousands of runs.

The candidates are chosen so that every decision is exact in any
precision: sigma is a power of two (the per-16-frame sums are equal powers
of two), every window maximum is sigma times a multiple of 1/256, and
k_sigma lies between two such multiples.  Then the FP32 threshold
comparisons and SNR products on the GPU and the FP64 ones in the oracle
take the same decisions, equal SNRs tie exactly on both sides, and the
lists must be identical: same length, same (beam, sample, trial), same
SNR and peak.
"""
import numpy as np
import pytest

import oracle
from paper_1612_06592_amd import lp

pytestmark = pytest.mark.gpu

M = 1024
WARM = lp.WARM_FRAMES


def make_cand(rng, n_beams, n_tec, n_t, frame0, sig_exp, fire_frac,
              k_sigma):
    """Window maxima, offsets and per-16-frame sums; returns the packed
    candidate bytes and the oracle's (sigma, wmax, warg)."""
    ns = n_beams * n_tec
    sigma = np.ldexp(1.0, sig_exp).astype(np.float64).reshape(ns)
    first_valid = max(0, WARM - frame0)
    assert first_valid % 16 == 0
    # Envelope maxima on a grid of sigma / 256; the threshold k_sigma * 256
    # lies strictly between grid points.  About fire_frac of the windows
    # exceed it.
    kt = k_sigma * 256.0
    assert kt != np.floor(kt)
    lo = int(np.floor(kt)) - 400
    hi = int(np.floor(kt)) + 1
    u = np.where(rng.random((ns, n_t)) < fire_frac,
                 rng.integers(hi, hi + 600, (ns, n_t)),
                 rng.integers(max(1, lo), hi, (ns, n_t)))
    wmax = sigma[:, None] * u / 256.0
    warg_in = rng.integers(0, M, (ns, n_t))
    psum = np.zeros((ns, n_t // 16), np.float32)
    n_valid = n_t - min(first_valid, n_t)
    for q in range(ns):
        if sigma[q] == 0:
            continue
        # sum over valid chunks = sigma^2 * n_valid * M, equal chunks
        psum[q, first_valid // 16:] = sigma[q] ** 2 * 16 * M
    for q in range(ns):
        if n_valid:
            s = np.sqrt(psum[q].astype(np.float64).sum() / (n_valid * M))
            assert s == sigma[q] or (sigma[q] == 0 and s == 0), (s, sigma[q])
    head = np.zeros((ns, n_t, 2), np.int32)
    head[..., 0] = wmax.astype(np.float32).view(np.int32)
    head[..., 1] = warg_in
    raw = np.concatenate([head.reshape(-1).view(np.uint8),
                          psum.reshape(-1).view(np.uint8)])
    warg = np.arange(n_t)[None, :] * M + warg_in
    return raw, sigma, wmax, warg


def run_gpu_trigger(raw, n_beams, n_tec, n_t, frame0, k_sigma, cap):
    import torch
    dev = "cuda:0"
    ctx = lp.Ctx(0)
    cand = torch.from_numpy(raw).to(dev)
    assert cand.numel() == lp.nbytes("lp_cand_bytes", n_beams * n_tec, n_t)
    work = torch.empty(lp.nbytes("lp_trigger_work_bytes", n_beams, n_tec, n_t),
                       dtype=torch.uint8, device=dev)
    out = torch.zeros(max(cap, 1) * lp.TRIG_DTYPE.itemsize, dtype=torch.uint8,
                      device=dev)
    n_out = torch.zeros(1, dtype=torch.int32, device=dev)
    snr = torch.zeros((n_beams, n_tec), dtype=torch.float32, device=dev)
    best = torch.zeros(n_beams, dtype=torch.int32, device=dev)
    sig = torch.zeros((n_beams, n_tec), dtype=torch.float32, device=dev)
    lp.trigger(ctx, cand, n_beams, n_tec, n_t, frame0, k_sigma, out, cap,
               n_out, work, snr, best, sig)
    torch.cuda.synchronize()
    n = int(n_out.item())
    trig = out[: min(n, cap) * lp.TRIG_DTYPE.itemsize].cpu().numpy().view(
        lp.TRIG_DTYPE).copy()
    res = dict(n=n, trig=trig, snr=snr.cpu().numpy(), best=best.cpu().numpy(),
               sigma=sig.cpu().numpy())
    ctx.close()
    return res


def check_equal(g, o_trig, cap):
    n = len(o_trig)
    assert g["n"] == n, (g["n"], n)
    k = min(n, cap)
    gt, ot = g["trig"], o_trig[:k]
    assert len(gt) == k
    np.testing.assert_array_equal(gt["beam"], ot["beam"])
    np.testing.assert_array_equal(gt["sample"], ot["sample"])
    np.testing.assert_array_equal(gt["tec"], ot["tec"])
    np.testing.assert_array_equal(gt["snr"].astype(np.float64), ot["snr"])
    np.testing.assert_array_equal(gt["peak"].astype(np.float64), ot["peak"])


@pytest.mark.parametrize("frame0", [0, 5000])
def test_many_runs_per_series_equal_oracle(frame0):
    """Thousands of runs per series (far above any fixed per-series limit),
    several trials with different sigma, cross-trial chains, a series with
    sigma 0, the start-up rule at frame0 = 0."""
    rng = np.random.default_rng([1612, 6592, frame0])
    n_beams, n_tec, n_t = 3, 5, 16384
    k_sigma = 2.0 + 1.0 / 512
    sig_exp = rng.integers(-2, 4, n_beams * n_tec)
    raw, sigma, wmax, warg = make_cand(rng, n_beams, n_tec, n_t, frame0,
                                       sig_exp, 0.45, k_sigma)
    print(f"case trigger many runs frame0={frame0}", flush=True)
    ot, osnr, obest = oracle.trigger(sigma, wmax, warg, n_beams, n_tec, n_t,
                                     frame0, WARM, k_sigma)
    # runs per series in the oracle's terms (before the cross-trial merge)
    fired = wmax > k_sigma * sigma[:, None]
    fired[:, :max(0, WARM - frame0)] = False
    runs = (fired[:, 1:] & ~fired[:, :-1]).sum(1) + fired[:, 0]
    print("runs per series", int(runs.min()), "..", int(runs.max()),
          "merged triggers", len(ot), flush=True)
    assert runs.max() > 2000
    cap = len(ot) + 10
    g = run_gpu_trigger(raw, n_beams, n_tec, n_t, frame0, k_sigma, cap)
    check_equal(g, ot, cap)
    np.testing.assert_allclose(g["snr"], osnr, rtol=0, atol=0)
    np.testing.assert_array_equal(g["best"], obest)
    np.testing.assert_array_equal(g["sigma"].ravel(), sigma.astype(np.float32))


def test_sigma_zero_and_truncation():
    """A series with sigma 0 never fires; with cap below the count, the
    first cap triggers are written and n_out is the true count."""
    rng = np.random.default_rng([1612, 6592, 7])
    n_beams, n_tec, n_t = 2, 3, 8192
    k_sigma = 3.0 + 1.0 / 512
    sig_exp = np.array([1, 2, 0, 3, 1, 2])
    raw, sigma, wmax, warg = make_cand(rng, n_beams, n_tec, n_t, 2000,
                                       sig_exp, 0.3, k_sigma)
    # series 4 (beam 1, trial 1): all sums zero -> sigma 0
    ns = n_beams * n_tec
    head = raw[: ns * n_t * 8].view(np.int32).reshape(ns, n_t, 2)
    psum = raw[ns * n_t * 8:].view(np.float32).reshape(ns, n_t // 16)
    psum[4] = 0.0
    sigma = sigma.copy()
    sigma[4] = 0.0
    ot, osnr, obest = oracle.trigger(sigma, wmax, warg, n_beams, n_tec, n_t,
                                     2000, WARM, k_sigma)
    assert not np.any(ot["tec"][ot["beam"] == 1] == 1)
    cap = len(ot) // 3
    print(f"case trigger truncation n={len(ot)} cap={cap}", flush=True)
    g = run_gpu_trigger(raw, n_beams, n_tec, n_t, 2000, k_sigma, cap)
    check_equal(g, ot, cap)
    np.testing.assert_array_equal(g["best"], obest)
    assert g["snr"][1, 1] == 0.0 and g["sigma"][1, 1] == 0.0
    del head


def test_long_chains_across_trials():
    """Every trial of one beam fires at shifted, overlapping windows, so
    chains span many triggers of all trials (the segmented scan crosses
    thread ranges)."""
    rng = np.random.default_rng([1612, 6592, 11])
    n_beams, n_tec, n_t = 2, 32, 8192
    k_sigma = 4.0 + 1.0 / 512
    sig_exp = np.zeros(n_beams * n_tec, np.int64) + 1
    raw, sigma, wmax, warg = make_cand(rng, n_beams, n_tec, n_t, 3000,
                                       sig_exp, 0.5, k_sigma)
    ot, osnr, obest = oracle.trigger(sigma, wmax, warg, n_beams, n_tec, n_t,
                                     3000, WARM, k_sigma)
    print(f"case trigger long chains n={len(ot)}", flush=True)
    g = run_gpu_trigger(raw, n_beams, n_tec, n_t, 3000, k_sigma, len(ot) + 1)
    check_equal(g, ot, len(ot) + 1)
    np.testing.assert_array_equal(g["best"], obest)
