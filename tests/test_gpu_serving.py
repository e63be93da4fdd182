"""Serving loop on the GPU: results through lp_server/lp_stream equal the
direct stage calls on the same blocks (bitwise: chunking changes no
arithmetic), and each stream's results are the same alone and in a mix of
concurrent streams of other shapes."""
import numpy as np
import pytest

import lofarsim
from chain import OracleChain, compare_triggers
from paper_1612_06592_amd import lp

pytestmark = pytest.mark.gpu


def make_stream(seed, n_st, rings, k0, n_sb, tec, lens, n_pulses=2,
                snr=(12.0, 12.0), trials=None, dtype="ci8", sigma=8.0):
    """One generated observation cut into consecutive blocks (device).
    trials: TEC trial list (default: the true TEC alone)."""
    import torch
    if trials is None:
        trials, idx = (tec,), 0
    else:
        idx = int(np.argmin(np.abs(np.asarray(trials) - tec)))
    cfg = lofarsim.get_config("c2", n_st=n_st, hex_rings=rings,
                              k=tuple(range(k0, k0 + n_sb)), n_t=sum(lens),
                              tec=tuple(trials), true_tec_index=idx,
                              true_tec=tec, n_pulses=n_pulses,
                              snr=snr, seed=(seed,), dtype=dtype,
                              sigma=sigma)
    blk = lofarsim.generate(cfg)
    blocks, a = [], 0
    for n_t in lens:
        part = lofarsim.Block(cfg, np.ascontiguousarray(blk.x[:, a:a + n_t]),
                              blk.enu, blk.az_el, blk.k, blk.tec, blk.pulses,
                              blk.seeds)
        blocks.append((part, torch.from_numpy(part.x).to("cuda:0")))
        a += n_t
    return blocks


def stream_cfg(blk, max_n_t, prec=lp.LP_FP16_MFMA):
    dtype = lp.LP_CI8 if blk.x.dtype == np.int8 else lp.LP_CI16
    return lp.StreamCfg(blk.enu, blk.k, blk.az_el, blk.tec, max_n_t,
                        dtype=dtype, prec=prec, trig_cap=256)


def direct(blocks):
    """The same blocks through lp_beamform .. lp_trigger, one stream."""
    import torch
    out = []
    blk0 = blocks[0][0]
    ctx = lp.Ctx(0)
    frame0 = 0
    state = None
    for blk, x in blocks:
        p = lp.Pipeline(ctx, lp.Array(blk0.enu, 2), lp.Band(blk0.k),
                        lp.Dirs(blk0.az_el), blk0.tec, blk.n_t, trig_cap=256)
        if state is not None:
            p.bufs["tail"].copy_(state[0])
            p.bufs["hist"].copy_(state[1])
        p.frame0 = frame0
        p.step(x)
        torch.cuda.synchronize()
        out.append(dict(trig=p.triggers(), snr=p.bufs["snr"].cpu().numpy().ravel(),
                        best=p.bufs["best"].cpu().numpy()))
        state = (p.bufs["tail"].clone(), p.bufs["hist"].clone())
        frame0 += blk.n_t
    ctx.close()
    return out


def serve(streams, chunk_t=2048, interleave=True, precs=None):
    """Submit every stream's blocks to one server; returns results per
    stream in submission order."""
    import torch
    ctx = lp.Ctx(0)
    arena = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
    srv = lp.Server(ctx, arena, arena.numel(), max_slots=8, chunk_t=chunk_t)
    ids = []
    for si, blocks in enumerate(streams):
        max_n_t = max(b.n_t for b, _ in blocks)
        prec = lp.LP_FP16_MFMA if precs is None else precs[si]
        ids.append(srv.open(stream_cfg(blocks[0][0], max_n_t, prec)))
    order = []
    n_max = max(len(s) for s in streams)
    for i in range(n_max):
        for si, blocks in enumerate(streams):
            if i < len(blocks):
                order.append((si, i))
    total = len(order)
    for si, i in order:
        blk, x = streams[si][i]
        srv.submit(ids[si], x, blk.n_t, tag=si * 100 + i)
    res = []
    import time
    t0 = time.time()
    while len(res) < total and time.time() - t0 < 60:
        res += srv.poll(timeout_us=100000)
    stats = srv.stats()
    srv.destroy()
    ctx.close()
    assert len(res) == total, (len(res), total)
    per = {}
    for r in res:
        assert r["status"] == lp.LP_OK
        per.setdefault(r["stream"], []).append(r)
    return [sorted(per[sid], key=lambda r: r["tag"]) for sid in ids], stats


def same(a, b):
    return (np.array_equal(a["trig"], b["trig"]) and
            np.array_equal(a["snr"], b["snr"]) and
            np.array_equal(a["best_tec"] if "best_tec" in a else a["best"],
                           b["best_tec"] if "best_tec" in b else b["best"]))


def test_served_equals_direct_calls():
    A = make_stream(1, 8, 1, 52, 32, 7.0, [4096, 8192, 2048])
    ref = direct(A)
    (got,), stats = serve([A], chunk_t=2048)
    assert stats["chunks_issued"] == 2 + 4 + 1
    for g, r in zip(got, ref):
        assert np.array_equal(g["trig"], r["trig"])
        assert np.array_equal(g["snr"], r["snr"])
        assert np.array_equal(g["best_tec"], r["best"])
    assert sum(len(g["trig"]) for g in got) >= 1


def test_alone_equals_in_the_mix():
    A = make_stream(2, 8, 1, 52, 32, 5.0, [4096, 4096, 8192])
    B = make_stream(3, 12, 0, 100, 48, 20.0, [8192, 2048])
    Cs = make_stream(4, 6, 2, 300, 16, 0.0, [2048, 2048, 2048, 4096])
    alone, _ = serve([A])
    mix, stats = serve([A, B, Cs], chunk_t=2048)
    for a, m in zip(alone[0], mix[0]):
        assert same(a, m)
    refB = direct(B)
    for g, r in zip(mix[1], refB):
        assert np.array_equal(g["trig"], r["trig"])
        assert np.array_equal(g["snr"], r["snr"])
    lat = np.array([r["latency_ns"] for s in mix for r in s]) / 1e6
    dl = np.array([r["deadline_ns"] for s in mix for r in s]) / 1e6
    print(f"mix latency ms p50 {np.percentile(lat, 50):.2f} "
          f"p99 {np.percentile(lat, 99):.2f} max {lat.max():.2f}; "
          f"chunks {stats['chunks_issued']}", flush=True)
    assert np.all(lat < dl)


def test_served_mix_against_oracle():
    """Every stream of a concurrent mix against the FP64 oracle's chain run
    over the same consecutive, uneven blocks (state carried from block to
    block): per-series peak SNR within the FP16 bound, trigger lists equal
    (beam exact, sample within 1, decisions within 1 % of the threshold
    excepted), best trial equal.  The mix has an FP16-MFMA stream, an FP32
    stream, a 4-trial stream and an int16 stream."""
    A = make_stream(11, 8, 1, 52, 32, 7.0, [4096, 8192, 2048])
    B = make_stream(12, 12, 0, 100, 48, 20.0, [8192, 2048, 4096])
    Cm = make_stream(13, 6, 1, 300, 24, 10.0, [2048, 4096, 2048, 6144],
                     trials=(0.0, 5.0, 10.0, 15.0), snr=(14.0, 14.0))
    D = make_stream(14, 4, 0, 200, 20, 3.0, [6144, 2048], dtype="ci16",
                    sigma=16.0)
    streams = [A, B, Cm, D]
    precs = [lp.LP_FP16_MFMA, lp.LP_FP32, lp.LP_FP16_MFMA, lp.LP_FP16_MFMA]
    tol = {lp.LP_FP16_MFMA: 1e-3, lp.LP_FP32: 1e-5}
    got, stats = serve(streams, chunk_t=2048, precs=precs)
    n_trig = 0
    for si, blocks in enumerate(streams):
        blk0 = blocks[0][0]
        oc = OracleChain(blk0)
        for bi, (blk, _) in enumerate(blocks):
            o = oc.process(blk.x)
            g = got[si][bi]
            label = f"stream {si} block {bi} (n_t {blk.n_t})"
            snr_g = np.asarray(g["snr"], np.float64).ravel()
            snr_o = o["snr"].ravel()
            e = np.max(np.abs(snr_g - snr_o) / np.maximum(snr_o, 1e-30))
            print(f"{label}: peak-SNR max rel err {e:.2e}, triggers "
                  f"gpu {len(g['trig'])} oracle {len(o['trig'])}", flush=True)
            assert e <= 2 * tol[precs[si]], label
            assert g["n_trig"] == len(g["trig"])
            miss, extra = compare_triggers(g["trig"], o["trig"], o["sigma"])
            assert not miss and not extra, (label, miss, extra)
            assert np.array_equal(np.asarray(g["best_tec"]), o["best"]), label
            n_trig += len(o["trig"])
    assert n_trig >= 4
