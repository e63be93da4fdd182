"""Full-size workloads on the GPU, in the launch configuration bench.py
times, checked against the oracle.

C2 (24 stations, 244 subbands, 65536 samples, 1 beam): the oracle runs the
whole block (in memory-bounded pieces) and every stage output is compared.

C3 (61 beams x 96 inputs, 32768 samples) and C4 (7 beams x 32 TEC trials,
65536 samples) are too large for the oracle as a whole, so:
  * beam sums are compared on sampled subbands (all beams, all samples);
  * the chain is compared on a time slice around each pulse: the oracle
    starts one hop (2048 samples) before the slice with zero state, so its
    de-dispersed output is exact from the slice's first hop and its
    synthesised frames from 16 frames later; window maxima there must match;
  * properties that hold at any size: each pulse's best trigger is in its
    source beam (C3); the best trial is the injected TEC index (C4).
"""
import numpy as np
import pytest

import lofarsim
import oracle
from chain import OracleChain, compare_triggers, rel_rms, run_gpu
from paper_1612_06592_amd import lp

pytestmark = pytest.mark.gpu

HOP = 2048


def test_c2_full_block_against_oracle():
    blk = lofarsim.generate(lofarsim.get_config("c2"))
    print("case c2 full", flush=True)
    g = run_gpu(blk, lp.LP_FP16_MFMA)
    o = OracleChain(blk, sb_group=16, series_group=1).process(
        blk.x, keep_series=(0,))
    for name, a, b in (("y", g["y"], o["y"]), ("d", g["d"], o["d"]),
                       ("x", g["x"][0], 2 * o["z"][0].real),
                       ("window max", g["emax"], o["wmax"])):
        e = rel_rms(a, b)
        print(f"c2 full {name} rel-rms {e:.2e}", flush=True)
        assert e <= 1e-3
    assert abs(g["sigma"].ravel()[0] / o["sigma"][0] - 1) <= 1e-3
    miss, extra = compare_triggers(g["trig"], o["trig"], o["sigma"])
    print(f"c2 full triggers gpu={len(g['trig'])} oracle={len(o['trig'])}",
          flush=True)
    assert not miss and not extra, (miss, extra)
    for p in blk.pulses:
        assert any(abs(int(t["sample"]) - p["n0"]) <= 1 for t in g["trig"]), p


def _slice_chain(blk, beams, tec, t0, n):
    """Oracle chain for a subset of beams/trials on samples [t0, t0 + n)."""
    sub = lofarsim.Block(blk.cfg, np.ascontiguousarray(blk.x[:, t0:t0 + n]),
                         blk.enu, blk.az_el[list(beams)], blk.k,
                         np.atleast_1d(tec), blk.pulses, blk.seeds)
    oc = OracleChain(sub, sb_group=16, series_group=4)
    oc.frame0 = t0           # stream position (start-up rule)
    return oc.process(sub.x)


def _gpu_full(blk, prec=lp.LP_FP16_MFMA):
    import torch
    from chain import as_complex, gpu_pipeline, to_device
    ctx, p = gpu_pipeline(blk, prec, want_series=False)
    p.step(to_device(blk.x))
    torch.cuda.synchronize()
    emax, arg, _ = p.cand_view()
    return ctx, p, dict(emax=emax.cpu().numpy(), arg=arg.cpu().numpy(),
                        trig=p.triggers(), best=p.bufs["best"].cpu().numpy(),
                        snr=p.bufs["snr"].cpu().numpy())


def _check_slice(gq_emax, o_wmax, t0, n, label):
    a = t0 + HOP + 16                 # first exact frame of the slice
    e = rel_rms(gq_emax[a:t0 + n], o_wmax[a - t0:])
    print(f"{label} window-max rel-rms {e:.2e}", flush=True)
    assert e <= 1e-3


def test_c3_full_61_beams():
    import torch
    from chain import as_complex
    cfg = lofarsim.get_config("c3")
    blk = lofarsim.generate(cfg)
    print("case c3 full", blk.x.shape, flush=True)
    ctx, p, g = _gpu_full(blk)
    # Beam sums on sampled subbands.
    ys = p.y_view()
    for s in (0, 97, 243):
        ref = oracle.beamform(blk.enu, 2, blk.k[s:s + 1], blk.az_el,
                              blk.x[s:s + 1])
        e = rel_rms(as_complex(ys[:, s:s + 1]), ref)
        print(f"c3 full y[subband {s}] rel-rms {e:.2e}", flush=True)
        assert e <= 1e-3
    ctx.close()
    del ys
    torch.cuda.empty_cache()
    B = blk.az_el.shape[0]
    for pl in blk.pulses:
        frame = pl["n0"] // 1024 + 16 + 1024          # output frame
        t0 = max(0, (frame // HOP - 2) * HOP)
        n = min(4 * HOP, blk.n_t - t0)
        o = _slice_chain(blk, [pl["beam"]], cfg.tec, t0, n)
        _check_slice(g["emax"][pl["beam"]], o["wmax"][0], t0, n,
                     f"c3 full beam {pl['beam']}")
        near = [t for t in g["trig"] if abs(int(t["sample"]) - pl["n0"]) <= 4]
        assert near, pl
        assert int(max(near, key=lambda t: t["snr"])["beam"]) == pl["beam"]
    assert g["best"].shape == (B,)


def test_c4_full_tec_grid():
    import torch
    cfg = lofarsim.get_config("c4")
    blk = lofarsim.generate(cfg)
    J = cfg.n_tec
    print("case c4 full true tec index", cfg.true_tec_index, flush=True)
    ctx, p, g = _gpu_full(blk)
    ctx.close()
    torch.cuda.empty_cache()
    # The centre beam's best trial is the injected grid index (the pulses
    # come from beam 0's direction).
    assert g["best"][0] == cfg.true_tec_index
    snr0 = g["snr"][0]
    print("c4 peak snr vs trial (beam 0):",
          np.round(snr0, 1).tolist(), flush=True)
    assert np.argmax(snr0) == cfg.true_tec_index
    pl = blk.pulses[0]
    frame = pl["n0"] // 1024 + 16 + 1024
    t0 = max(0, (frame // HOP - 2) * HOP)
    n = min(4 * HOP, blk.n_t - t0)
    trials = [0, cfg.true_tec_index, J - 1]
    o = _slice_chain(blk, [0], np.asarray(cfg.tec)[trials], t0, n)
    for i, j in enumerate(trials):
        _check_slice(g["emax"][j], o["wmax"][i], t0, n, f"c4 full trial {j}")
    hit = [t for t in g["trig"] if abs(int(t["sample"]) - pl["n0"]) <= 2
           and int(t["beam"]) == 0]
    assert hit and int(hit[0]["tec"]) == cfg.true_tec_index
