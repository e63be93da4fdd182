"""lp_trigger_noalloc (workspace in the library's fixed device array)
against lp_trigger (workspace passed by the caller) on the same
candidates: two calls in a row, the second smaller than the first, so the
second runs on the array as the first left it.  The lists, counts, SNR,
sigma and best trial must be bitwise equal, and both must equal the
oracle's trigger rules.  A size whose workspace exceeds the array is
rejected before anything runs."""
import numpy as np
import pytest

import oracle
from paper_1612_06592_amd import lp
from test_gpu_trigger import make_cand

pytestmark = pytest.mark.gpu

M = 1024
WARM = lp.WARM_FRAMES


def _outputs(dev, n_beams, n_tec, cap):
    import torch
    out = torch.full((max(cap, 1) * lp.TRIG_DTYPE.itemsize,), 0xA5,
                     dtype=torch.uint8, device=dev)
    return dict(out=out,
                n_out=torch.full((1,), -7, dtype=torch.int32, device=dev),
                snr=torch.full((n_beams, n_tec), -1.0, dtype=torch.float32,
                               device=dev),
                best=torch.full((n_beams,), -1, dtype=torch.int32, device=dev),
                sigma=torch.full((n_beams, n_tec), -1.0, dtype=torch.float32,
                                 device=dev))


def _read(o, cap):
    n = int(o["n_out"].item())
    k = min(n, cap)
    trig = o["out"][: k * lp.TRIG_DTYPE.itemsize].cpu().numpy().view(
        lp.TRIG_DTYPE).copy()
    return dict(n=n, trig=trig, snr=o["snr"].cpu().numpy(),
                best=o["best"].cpu().numpy(), sigma=o["sigma"].cpu().numpy())


def _same(a, b):
    assert a["n"] == b["n"], (a["n"], b["n"])
    assert a["trig"].tobytes() == b["trig"].tobytes()
    for key in ("snr", "best", "sigma"):
        assert a[key].tobytes() == b[key].tobytes(), key


def test_noalloc_trigger_equals_trigger_with_workspace():
    import torch
    dev = "cuda:0"
    rng = np.random.default_rng([1612, 6592, 77])
    ctx = lp.Ctx(0)
    # (beams, trials, samples, frame0, k_sigma, fire fraction, cap): a large
    # first call with long lists, then a smaller one that reuses the array.
    cases = [(7, 8, 16384, 0, 5.9999, 0.3, 1 << 16),
             (3, 2, 4096, 6144, 6.0001, 0.05, 64)]
    for (nb, nj, n_t, frame0, ks, frac, cap) in cases:
        need = lp.nbytes("lp_trigger_work_bytes", nb, nj, n_t)
        assert 0 < need <= lp.TRIGGER_SCRATCH_BYTES
        print(f"case noalloc trigger beams={nb} trials={nj} n_t={n_t} "
              f"frame0={frame0} workspace={need}", flush=True)
        sig_exp = rng.integers(-3, 6, nb * nj)
        raw, sigma, wmax, warg = make_cand(rng, nb, nj, n_t, frame0, sig_exp,
                                           frac, ks)
        cand = torch.from_numpy(raw).to(dev)
        ref = _outputs(dev, nb, nj, cap)
        work = torch.empty(need, dtype=torch.uint8, device=dev)
        lp.trigger(ctx, cand, nb, nj, n_t, frame0, ks, ref["out"], cap,
                   ref["n_out"], work, ref["snr"], ref["best"], ref["sigma"])
        new = _outputs(dev, nb, nj, cap)
        lp.trigger_noalloc(ctx, cand, nb, nj, n_t, frame0, ks, new["out"],
                           cap, new["n_out"], new["snr"], new["best"],
                           new["sigma"])
        torch.cuda.synchronize()
        a, b = _read(ref, cap), _read(new, cap)
        _same(a, b)
        o_trig, o_snr, o_best = oracle.trigger(sigma, wmax, warg, nb, nj,
                                               n_t, frame0, WARM,
                                               k_sigma=ks)
        assert b["n"] == len(o_trig)
        k = min(b["n"], cap)
        np.testing.assert_array_equal(b["trig"]["beam"], o_trig["beam"][:k])
        np.testing.assert_array_equal(b["trig"]["sample"],
                                      o_trig["sample"][:k])
        np.testing.assert_array_equal(b["trig"]["tec"], o_trig["tec"][:k])
        np.testing.assert_array_equal(b["best"], o_best)
        print(f"noalloc trigger: {b['n']} triggers, equal to lp_trigger and "
              f"the oracle", flush=True)
        del work
    ctx.close()


def test_noalloc_trigger_rejects_oversized_workspace():
    import torch
    dev = "cuda:0"
    ctx = lp.Ctx(0)
    nb, nj, n_t = 64, 32, 65536
    assert lp.nbytes("lp_trigger_work_bytes", nb, nj, n_t) > \
        lp.TRIGGER_SCRATCH_BYTES
    o = _outputs(dev, nb, nj, 16)
    cand = torch.zeros(16, dtype=torch.uint8, device=dev)
    with pytest.raises(lp.LpError) as ei:
        lp.trigger_noalloc(ctx, cand, nb, nj, n_t, 0, 6.0, o["out"], 16,
                           o["n_out"], o["snr"], o["best"], o["sigma"])
    assert ei.value.code == lp.LP_EINVAL
    assert "workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert int(o["n_out"].item()) == -7   # nothing ran
    ctx.close()
