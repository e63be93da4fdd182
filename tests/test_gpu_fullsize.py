"""Full-size workloads on the GPU, in the launch configuration bench.py
times, checked against the oracle.

C2 (24 stations, 244 subbands, 65536 samples, 1 beam): the oracle runs the
whole block (in memory-bounded pieces) and every stage output is compared.

C3 (61 beams x 96 inputs, 32768 samples) and C4 (7 beams x 32 TEC trials,
65536 samples): the oracle runs the whole block a few beams at a time (its
FP64 intermediates of all beams would not fit in host memory at once;
beams are independent and the trigger merge is per beam), and the beam
sums, de-dispersed subbands, window maxima, sigma, peak SNR per trial,
best trial and the full trigger list are compared; plus the properties
that name the workloads: each pulse's best trigger is in its source beam
(C3), the best trial is the injected TEC index (C4).
"""
import numpy as np
import pytest

import lofarsim
from chain import PER_ELEM, OracleChain, compare_triggers, max_err, rel_rms, run_gpu
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
        e, m = rel_rms(a, b), max_err(a, b)
        print(f"c2 full {name} rel-rms {e:.2e} max {m:.2e}", flush=True)
        assert e <= 1e-3 and m <= PER_ELEM[lp.LP_FP16_MFMA]
    assert abs(g["sigma"].ravel()[0] / o["sigma"][0] - 1) <= 1e-3
    miss, extra = compare_triggers(g["trig"], o["trig"], o["sigma"])
    print(f"c2 full triggers gpu={len(g['trig'])} oracle={len(o['trig'])}",
          flush=True)
    assert not miss and not extra, (miss, extra)
    for p in blk.pulses:
        assert any(abs(int(t["sample"]) - p["n0"]) <= 1 for t in g["trig"]), p


def _gpu_full(blk, prec=lp.LP_FP16_MFMA):
    import torch
    from chain import gpu_pipeline, to_device
    ctx, p = gpu_pipeline(blk, prec, want_series=False)
    p.step(to_device(blk.x))
    torch.cuda.synchronize()
    emax, arg, _ = p.cand_view()
    return ctx, p, dict(emax=emax.cpu().numpy(), arg=arg.cpu().numpy(),
                        trig=p.triggers(), best=p.bufs["best"].cpu().numpy(),
                        snr=p.bufs["snr"].cpu().numpy(),
                        sigma=p.bufs["sigma"].cpu().numpy(),
                        n_trig=int(p.bufs["n_trig"].item()))


def _oracle_by_beams(blk, p, group, label):
    """The oracle's chain over the whole block, a few beams at a time
    (beams are independent; the trigger rules merge trials per beam), each
    group's beam sums and de-dispersed subbands compared with the GPU's as
    they are produced.  Returns the oracle's window maxima, sigma, peak
    SNR, best trial and trigger list of every beam."""
    from chain import as_complex
    B = blk.az_el.shape[0]
    J = len(blk.tec)
    wmax, sigma, snr, best, trig = [], [], [], [], []
    ey = ed = 0.0
    ny = nd = 0.0
    my = md = 0.0  # largest element errors
    for b0 in range(0, B, group):
        b1 = min(B, b0 + group)
        sub = lofarsim.Block(blk.cfg, blk.x, blk.enu, blk.az_el[b0:b1], blk.k,
                             blk.tec, blk.pulses, blk.seeds)
        o = OracleChain(sub, sb_group=16, series_group=4).process(blk.x)
        gy = as_complex(p.y_view()[b0:b1])
        ey += np.sum(np.abs(gy - o["y"]) ** 2)
        ny += np.sum(np.abs(o["y"]) ** 2)
        my = max(my, float(np.max(np.abs(gy - o["y"]))))
        del gy
        gd = as_complex(p.d_view()[b0:b1])
        ed += np.sum(np.abs(gd - o["d"]) ** 2)
        nd += np.sum(np.abs(o["d"]) ** 2)
        md = max(md, float(np.max(np.abs(gd - o["d"]))))
        del gd
        t = o["trig"].copy()
        t["beam"] += b0
        trig.append(t)
        wmax.append(o["wmax"])
        sigma.append(o["sigma"])
        snr.append(o["snr"])
        best.append(o["best"])
        print(f"{label} oracle beams {b0}..{b1 - 1}: {len(t)} triggers",
              flush=True)
        del o
    out = dict(wmax=np.concatenate(wmax), sigma=np.concatenate(sigma),
               snr=np.concatenate(snr).reshape(B, J),
               best=np.concatenate(best), trig=np.concatenate(trig))
    out["y_rel_rms"] = float(np.sqrt(ey / ny))
    out["d_rel_rms"] = float(np.sqrt(ed / nd))
    n_el = blk.x.shape[0] * blk.x.shape[1]  # subbands x samples per beam
    out["y_max"] = my / np.sqrt(ny / (B * n_el))
    out["d_max"] = md / np.sqrt(nd / (B * len(blk.tec) * n_el))
    return out


def _check_full(g, o, label):
    for name, e, m in (("y", o["y_rel_rms"], o["y_max"]),
                       ("d", o["d_rel_rms"], o["d_max"]),
                       ("window max", rel_rms(g["emax"], o["wmax"]),
                        max_err(g["emax"], o["wmax"]))):
        print(f"{label} {name} rel-rms {e:.2e} max {m:.2e}", flush=True)
        assert e <= 1e-3 and m <= PER_ELEM[lp.LP_FP16_MFMA], name
    e = np.max(np.abs(g["sigma"].ravel() - o["sigma"]) / o["sigma"])
    print(f"{label} sigma max rel err {e:.2e}", flush=True)
    assert e <= 1e-3
    e = np.max(np.abs(g["snr"] - o["snr"]) / np.maximum(o["snr"], 1e-30))
    assert e <= 2e-3
    assert np.array_equal(g["best"], o["best"])
    assert g["n_trig"] == len(g["trig"])
    miss, extra = compare_triggers(g["trig"], o["trig"], o["sigma"])
    print(f"{label} triggers gpu={len(g['trig'])} oracle={len(o['trig'])}, "
          f"unmatched beyond the borderline rule: {len(miss)} / {len(extra)}",
          flush=True)
    assert not miss and not extra, (miss, extra)


@pytest.mark.timeout(1200)
def test_c3_full_61_beams():
    """The whole 61-beam block: every beam's trigger list, window maxima,
    sigma and the beam sums and de-dispersed subbands against the oracle."""
    cfg = lofarsim.get_config("c3")
    blk = lofarsim.generate(cfg)
    print("case c3 full", blk.x.shape, flush=True)
    ctx, p, g = _gpu_full(blk)
    o = _oracle_by_beams(blk, p, 8, "c3 full")
    ctx.close()
    _check_full(g, o, "c3 full")
    # each pulse's highest-SNR trigger is in its source beam
    for pl in blk.pulses:
        near = [t for t in g["trig"] if abs(int(t["sample"]) - pl["n0"]) <= 4]
        assert near, pl
        assert int(max(near, key=lambda t: t["snr"])["beam"]) == pl["beam"]


@pytest.mark.timeout(1200)
def test_c4_full_tec_grid():
    """The whole 7-beam x 32-trial block: every beam's merged trigger list,
    the 224 series' window maxima, sigma and peak SNR, the best trial."""
    cfg = lofarsim.get_config("c4")
    blk = lofarsim.generate(cfg)
    print("case c4 full true tec index", cfg.true_tec_index, flush=True)
    ctx, p, g = _gpu_full(blk)
    o = _oracle_by_beams(blk, p, 1, "c4 full")
    ctx.close()
    _check_full(g, o, "c4 full")
    # The centre beam's best trial is the injected grid index (the pulses
    # come from beam 0's direction).
    assert g["best"][0] == cfg.true_tec_index
    print("c4 peak snr vs trial (beam 0):",
          np.round(g["snr"][0], 1).tolist(), flush=True)
    pl = blk.pulses[0]
    hit = [t for t in g["trig"] if abs(int(t["sample"]) - pl["n0"]) <= 2
           and int(t["beam"]) == 0]
    assert hit and int(hit[0]["tec"]) == cfg.true_tec_index
