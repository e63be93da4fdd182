"""Benchmark of the lunar ns-pulse hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
                    [--prec fp16|fp32] [--no-cpu-baseline]

One step = the whole chain (beamform -> de-disperse -> synthesise ->
trigger) over one block of synthetic station data already resident in
HBM; consecutive steps continue the same stream (state carried).  Prints
one JSON line: station-beam Msamples/s (station-polarisation inputs x
subbands x samples x beams per second), the real-time factor, block
latency percentiles against the 5 s transient-buffer deadline, the
roofline position of the dominant kernel (timed with HIP events on the
stream the kernels run on), and the FP64 oracle timed on the host on a
bounded sample of the same block.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector: 256 CU x 4 SIMD x 32
                               # lanes x 2 FLOP x 2.4 GHz
METRIC = ("station-beam Msamples/s real-time factor at ≤1e-3 rel RMS; "
          "p99 block latency")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
LSMR_ITERS = 25                # iterations of the PPF-inversion leg (Sec. 3)


def kernel_source_hash(name: str) -> str:
    p = os.path.join(ROOT, "paper_1612_06592_amd", "csrc", name)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def algorithmic_bytes(stage: str, cfg, n_t: int) -> float:
    """HBM bytes a launch must move at minimum (read once, write once)."""
    es = 1 if cfg.dtype == "ci8" else 2
    K, S, B, J = cfg.n_in, cfg.n_sb, cfg.n_beams, cfg.n_tec
    if stage == "beamform":
        return K * S * n_t * 2 * es + B * S * n_t * 8
    if stage == "dedisperse":
        return B * S * n_t * 8 + B * J * S * n_t * 8
    if stage == "synthesize":
        return B * J * S * n_t * 8 + B * J * n_t * 8 + B * J * n_t // 16 * 4
    return 0.0


def device_copy_gbs(dev, mib: int = 1024, reps: int = 5) -> float:
    """Read + write GB/s of the runtime's device copy of `mib` MiB (HIP
    events around `reps` copies after one warm-up)."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * reps / (ms * 1e-3) / 1e9


def algorithmic_flop(stage: str, cfg, n_t: int) -> float:
    """FLOP a launch must do, by the paper's cost rules (Sec. 3: 8 FLOP per
    station sample and beam for beamforming, 6 per complex multiply,
    5 N log2 N per N-point FFT).  Beamforming: 8 per input (station-
    polarisation) sample, subband and beam.  De-dispersion, per
    beam-subband-sample (each 4096-point transform yields 2048 new
    samples): 120 for the forward transforms, plus per trial 12 for the
    chirp (4096 products) and 120 for the inverse.  Synthesis, per 5 ns
    output sample: 50 for the 1024-point transform, 64 for the 16-tap
    complex-by-real FIR, 6 for envelope and statistics."""
    K, S, B, J = cfg.n_in, cfg.n_sb, cfg.n_beams, cfg.n_tec
    if stage == "beamform":
        return 8.0 * K * S * n_t * B
    if stage == "dedisperse":
        return B * S * n_t * (120.0 + 132.0 * J)
    if stage == "synthesize":
        return B * J * n_t * 1024 * 120.0
    return 0.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3",
                    help="c1 tiny, c2 single beam, c3 61 beams (default: the "
                         "largest single-GPU workload by station-beam "
                         "samples), c4 32 TEC trials, c5 serving")
    ap.add_argument("--prec", default="fp16", choices=["fp16", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-beams", type=int, default=0,
                    help="beams in the oracle's sample of the first block "
                         "(0: the pulses' beams, then others, up to "
                         "max(1, 8 // trials))")
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="steps of the plain FP32 comparator pipeline (0: skip)")
    ap.add_argument("--graph-steps", type=int, default=20,
                    help="steps with beamform, de-dispersion and synthesis "
                         "replayed from a HIP graph (0: skip)")
    ap.add_argument("--duration", type=float, default=20.0,
                    help="c5: seconds of Poisson arrivals")
    ap.add_argument("--load", type=float, default=0.8,
                    help="c5: offered load as a fraction of the GPU")
    ap.add_argument("--max-log2-nt", type=int, default=18,
                    help="c5: longest block is 2^this samples per subband")
    ap.add_argument("--arena-frac", type=float, default=1.0,
                    help="c5: arena = resident state + this fraction of every "
                         "stream's longest in-flight block (1: all fit at "
                         "once; below 1 admission has to wait)")
    ap.add_argument("--plain-max-log2-nt", type=int, default=15,
                    help="c5: time the plain FP32 pipeline alone on every "
                         "stream for blocks up to 2^this (0: skip)")
    ap.add_argument("--ppf-iters", type=int, default=LSMR_ITERS,
                    help="LSMR iterations of the PPF-inversion leg (0: skip)")
    ap.add_argument("--ppf-steps", type=int, default=3,
                    help="timed PPF-inversion solves")
    ap.add_argument("--no-sim", action="store_true",
                    help="skip the station-simulator leg")
    ap.add_argument("--trial-group", type=int, default=8,
                    help="with several TEC trials: also time the chain with "
                         "the de-dispersed subbands held for one beam's "
                         "group of this many trials (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for "
                         "calibrating HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU only (the hot path "
              "would shard by beam or TEC trial with a broadcast of the "
              "station block; that multi-GPU path is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import lofarsim
    from paper_1612_06592_amd import lp

    if a.workload == "c5":
        return serving_bench(a)
    cfg = lofarsim.get_config(a.workload)
    t0 = time.time()
    blk = lofarsim.generate(cfg)
    gen_s = time.time() - t0
    print(f"[bench] generated {cfg.name}: x {blk.x.shape} {blk.x.dtype} "
          f"in {gen_s:.1f} s", file=sys.stderr, flush=True)
    prec = lp.LP_FP16_MFMA if a.prec == "fp16" else lp.LP_FP32
    dev = "cuda:0"
    x = torch.from_numpy(blk.x).to(dev)
    ctx = lp.Ctx(0)
    p = lp.Pipeline(ctx, lp.Array(blk.enu, 2), lp.Band(blk.k),
                    lp.Dirs(blk.az_el), blk.tec, cfg.n_t,
                    dtype=lp.LP_CI8 if cfg.dtype == "ci8" else lp.LP_CI16,
                    prec=prec, want_series=False, device=dev, cand_slots=2)
    stream = torch.cuda.current_stream()
    if a.calib_copy_mib:
        n = a.calib_copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # The first block of the fresh stream, kept for the error leg: the
    # sampled beams' beam sums, de-dispersed subbands, window maxima,
    # sigma, peak SNR and triggers.
    sel = sample_beams(cfg, blk, a.cpu_beams)
    p.step(x)
    torch.cuda.synchronize()
    first = first_block_outputs(p, sel)
    print(f"[bench] first block kept for beams {sel}", file=sys.stderr,
          flush=True)
    # The trigger of block i (one workgroup per series) runs on a second
    # stream beside block i + 1; the candidates alternate between two
    # buffers, so only the synthesis of block i + 2, which overwrites block
    # i's, waits for it.
    side = torch.cuda.Stream(device=dev)      # default priority
    stages = ["beamform", "dedisperse", "synthesize", "trigger"]

    def run_steps(n, ev):
        trig_done = []
        for i in range(n):
            e = ev[i]
            e[0].record(stream)
            p.beamform(x)
            e[1].record(stream)
            p.dedisperse()
            e[2].record(stream)
            if len(trig_done) >= p.cand_slots:
                stream.wait_event(trig_done[-p.cand_slots])
            p.synthesize()
            e[3].record(stream)
            side.wait_event(e[3])
            p.trigger(stream=side)
            e[4].record(side)
            trig_done = (trig_done + [e[4]])[-2:]
            p.frame0 += cfg.n_t

    def events(n):
        return [[torch.cuda.Event(enable_timing=True) for _ in range(5)]
                for _ in range(n)]

    run_steps(a.warmup, events(a.warmup))
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({a.warmup} steps)", file=sys.stderr, flush=True)
    ev = events(a.steps)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    run_steps(a.steps, ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    stage_ms = {s: [] for s in stages}
    block_ms = []
    for e in ev:
        for k, s in enumerate(stages):
            stage_ms[s].append(e[k].elapsed_time(e[k + 1]))
        block_ms.append(e[0].elapsed_time(e[4]))
    stage_avg = {s: float(np.mean(v)) for s, v in stage_ms.items()}
    ms_per_step = wall * 1e3 / a.steps
    samples = cfg.station_beam_samples
    value = samples / (ms_per_step * 1e-3) / 1e6
    block_s = cfg.block_seconds
    deadline_ms = (5.0 - block_s) * 1e3
    lat = np.array(block_ms)

    dom = max(["beamform", "dedisperse", "synthesize"], key=stage_avg.get)
    alg = algorithmic_bytes(dom, cfg, cfg.n_t)
    src = {"beamform": "beamform.hip", "dedisperse": "dedisperse.hip",
           "synthesize": "synthesize.hip"}[dom]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tj = json.load(open(TRAFFIC_FILE))
        rec = tj.get(f"{dom}:{cfg.name}:{a.prec}")
        if rec and rec.get("source_sha") == kernel_source_hash(src):
            traffic = rec["bytes_per_launch"]
    if dom == "beamform":
        # Streams the station block once: bound by HBM.  Beside the 8 TB/s
        # peak, the read + write rate of the runtime's own 1 GiB device copy
        # measured now, after the timed region.
        achieved = alg / (stage_avg[dom] * 1e-3) / 1e9
        copy_gbs = device_copy_gbs(dev)
        roofline = {"bound": "hbm", "kernel": dom,
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "algorithmic_bytes_per_launch": alg,
                    "avg_launch_ms": round(stage_avg[dom], 4),
                    "device_copy_GBps": round(copy_gbs, 1),
                    "frac_of_device_copy": round(achieved / copy_gbs, 4)}
    else:
        # The transforms and the FIR: bound by FP32 vector arithmetic.
        flop = algorithmic_flop(dom, cfg, cfg.n_t)
        achieved = flop / (stage_avg[dom] * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": dom,
                    "achieved": round(achieved, 2), "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s",
                    "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                    "traffic": traffic, "algorithmic_flop_per_launch": flop,
                    "algorithmic_bytes_per_launch": alg,
                    "avg_launch_ms": round(stage_avg[dom], 4)}

    # Trigger sanity on the last block: the injected pulses are found.
    # The stream has run 1 + warmup + steps blocks (the error leg's first
    # block included); the last one starts at this ADC offset.
    t_last = (a.warmup + a.steps) * cfg.n_t * 1024
    trig = p.triggers()
    found = sum(any(abs(int(t["sample"]) - (pl["n0"] + t_last)) <= 1
                    for t in trig) for pl in blk.pulses)
    injected = sorted({int(pl["beam"]) for pl in blk.pulses})
    # Per pulse: the beam of its highest-SNR trigger (a strong pulse's
    # sidelobes also trigger neighbouring beams).
    best_beam = []
    for pl in blk.pulses:
        near = [t for t in trig
                if abs(int(t["sample"]) - (pl["n0"] + t_last)) <= 4]
        best_beam.append(int(max(near, key=lambda t: t["snr"])["beam"])
                         if near else None)
    triggers = {"n": int(len(trig)),
                "beams": sorted({int(t["beam"]) for t in trig}),
                "injected_beams": [int(pl["beam"]) for pl in blk.pulses],
                "best_trigger_beam_per_pulse": best_beam}
    # TEC search: best trial and peak envelope SNR per trial of the beams
    # that hold a pulse (last block).
    tec_search = None
    if cfg.n_tec > 1:
        best = p.bufs["best"].cpu().numpy()
        snr = p.bufs["snr"].cpu().numpy()
        tec_search = {
            "true_tec_index": cfg.true_tec_index,
            "true_tec_tecu": float(cfg.true_tec),
            "best_tec_index": {str(b): int(best[b]) for b in injected},
            "peak_snr_vs_trial": {str(b): [round(float(v), 2) for v in snr[b]]
                                  for b in injected}}
    # The beamformer on the matrix cores: per subband the complex GEMM is
    # the real GEMM [n_t x 2K] by [2K x 2B], 8 K B n_t FLOP.
    mfma = None
    if a.prec == "fp16":
        fl = algorithmic_flop("beamform", cfg, cfg.n_t)
        tf = fl / (stage_avg["beamform"] * 1e-3) / 1e12
        mfma = {"kernel": "beamform", "achieved": round(tf, 2),
                "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tf / 2500.0, 4),
                "algorithmic_flop_per_launch": fl}

    graph = None
    if a.graph_steps > 0:
        graph = graph_leg(a, p, x, samples)

    ppf = None
    if a.ppf_iters > 0:
        ppf = ppf_leg(a, ctx, p, cfg, stream)
    two = None
    if cfg.n_beams > 1:
        two = two_stage_leg(a, ctx, p, blk, x, stream)
    sim = None
    if not a.no_sim:
        sim = station_sim_leg(a, ctx, cfg, blk, stream)

    grouped = None
    if cfg.n_tec > 1 and a.trial_group > 0:
        grouped = trial_group_leg(a, ctx, p, cfg, blk, x, ms_per_step)

    plain = None
    if a.plain_steps > 0:
        del p
        torch.cuda.empty_cache()
        pp = lp.Pipeline(ctx, lp.Array(blk.enu, 2), lp.Band(blk.k),
                         lp.Dirs(blk.az_el), blk.tec, cfg.n_t,
                         dtype=lp.LP_CI8 if cfg.dtype == "ci8" else lp.LP_CI16,
                         prec=lp.LP_FP32, plain=True, device=dev)
        pp.step(x)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(a.plain_steps):
            pp.step(x)
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - tp) * 1e3 / a.plain_steps
        plain = {"ms_per_step": round(ms_plain, 3),
                 "value": round(samples / (ms_plain * 1e-3) / 1e6, 1),
                 "speedup": round(ms_plain / ms_per_step, 2),
                 "speedup_graph": (round(ms_plain / graph["ms_per_step"], 2)
                                   if graph else None),
                 "kind": "same stages, FP32 beamformer, every intermediate "
                         "in HBM, radix-2 global-memory FFT passes"}
        del pp
        torch.cuda.empty_cache()

    cpu = error = None
    if not a.no_cpu_baseline:
        cpu, error = run_cpu_baseline(blk, sel, first)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Msamples/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f16-mfma/f32" if prec == lp.LP_FP16_MFMA else "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "stations": cfg.n_st,
                   "pol": cfg.n_pol, "subbands": cfg.n_sb,
                   "samples_per_block": cfg.n_t, "beams": cfg.n_beams,
                   "tec_trials": cfg.n_tec, "sample_type": cfg.dtype,
                   "precision": a.prec},
        "rtf": round(block_s * 1e3 / ms_per_step, 1),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4),
                       "max": round(float(lat.max()), 4),
                       "deadline": round(deadline_ms, 1)},
        "stage_ms": {s: round(v, 4) for s, v in stage_avg.items()},
        "pulses_found": f"{found}/{len(blk.pulses)}",
        "triggers": triggers,
        "tec_search": tec_search,
        "beamformer_mfma": mfma,
        "roofline": roofline,
        "whole_step": whole_step(cfg, ms_per_step),
        "error_vs_oracle": error,
        "graph_replay": graph,
        "trial_groups": grouped,
        "plain_fp32_pipeline": plain,
        "ppf_inversion": ppf,
        "two_stage_beamforming": two,
        "station_simulator": sim,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out))


def graph_leg(a, p, x, samples):
    """Steps with beamform, de-dispersion and synthesis replayed from a HIP
    graph and the trigger issued per block on the same stream (no second
    stream): the host issues two calls per block instead of four stages."""
    import torch
    for _ in range(p.cand_slots):
        p.step_graph(x)        # capture, one graph per candidate slot (the
    torch.cuda.synchronize()   # stream is past its start-up)
    t0 = time.perf_counter()
    for _ in range(a.graph_steps):
        p.step_graph(x)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / a.graph_steps
    return {"steps": a.graph_steps, "ms_per_step": round(ms, 4),
            "value": round(samples / (ms * 1e-3) / 1e6, 1),
            "kind": "beamform, de-dispersion and synthesis from a captured "
                    "HIP graph (one per candidate slot); trigger per block "
                    "with its frame0 on the same stream"}


def trial_group_leg(a, ctx, p, cfg, blk, x, ms_all):
    """The chain with lp_dedisperse_synthesize: the de-dispersed subbands
    held for one beam's group of a.trial_group trials instead of every
    beam and trial; timed over 3 blocks after one."""
    import torch
    from paper_1612_06592_amd import lp
    G = min(a.trial_group, cfg.n_tec)
    pg = lp.Pipeline(ctx, p.array, p.band, p.dirs, p.tec, cfg.n_t,
                     dtype=p.dtype, prec=p.prec, trial_group=G,
                     device=x.device)
    pg.step(x)
    torch.cuda.synchronize()
    n = 3
    t0 = time.perf_counter()
    for _ in range(n):
        pg.step(x)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / n
    d_all = cfg.n_beams * cfg.n_tec * cfg.n_sb * cfg.n_t * 8
    d_grp = G * cfg.n_sb * cfg.n_t * 8
    del pg
    torch.cuda.empty_cache()
    return {"trial_group": G, "d_bytes": d_grp, "d_bytes_all_trials": d_all,
            "ms_per_step": round(ms, 3),
            "vs_all_at_once": round(ms / ms_all, 3)}


def ppf_bytes_per_iteration(n_sb: int, n_frames: int) -> float:
    """HBM bytes one LSMR iteration must move per series: H reads v and
    reads/writes h, hbar, x (FP32, F frames of 1024) and reads/writes u
    (complex FP32, n_sb x n_frames); H^T reads u and reads/writes v."""
    F = n_frames - 15
    return F * 1024 * 4 * (1 + 6 + 2) + n_sb * n_frames * 8 * (2 + 1)


def ppf_leg(a, ctx, p, cfg, stream):
    """PPF inversion (LSMR on H x = y) of the last block's de-dispersed
    subbands (up to 8 (beam, trial) series), timed with HIP events."""
    import torch
    from paper_1612_06592_amd import lp
    # At most 8 series (the first beams/trials of the block) keep the
    # workspace bounded on the many-series workloads.
    ns, nf, S = min(8, cfg.n_beams * cfg.n_tec), cfg.n_t, cfg.n_sb
    F = nf - 15
    d = p.d_view().reshape(-1, S, nf, 2)[:ns]
    x = torch.empty((ns, F * 1024), dtype=torch.float32, device=d.device)
    wb = lp.nbytes("lp_ppf_work_bytes", S, ns, nf)
    work = torch.empty(wb, dtype=torch.uint8, device=d.device)
    an = torch.empty((ns, a.ppf_iters + 1), dtype=torch.float64,
                     device=d.device)
    rn = torch.empty(ns, dtype=torch.float64, device=d.device)
    lp.ppf_invert(ctx, p.band, d, ns, nf, a.ppf_iters, x, work, an, rn,
                  stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(a.ppf_steps)]
    for e0, e1 in ev:
        e0.record(stream)
        lp.ppf_invert(ctx, p.band, d, ns, nf, a.ppf_iters, x, work, an, rn,
                      stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
    ynorm = torch.linalg.vector_norm(d.reshape(ns, -1).double(), dim=1)
    rel = (rn / ynorm).cpu().numpy()
    an_h = an.cpu().numpy()
    it_bytes = ns * ppf_bytes_per_iteration(S, nf)
    achieved = it_bytes * a.ppf_iters / (ms * 1e-3) / 1e9
    out = {"iterations": a.ppf_iters, "series": ns, "frames": nf,
           "value": round(ns * nf / (ms * 1e-3), 1),
           "unit": "frames/s per series (25 iterations)" if a.ppf_iters == 25
           else f"frames/s per series ({a.ppf_iters} iterations)",
           "ms_per_solve": round(ms, 3),
           "ms_per_iteration": round(ms / a.ppf_iters, 4),
           "rtf": round(cfg.block_seconds * 1e3 / ms, 1),
           "residual_rel": float(np.max(rel)),
           "atr_reduction": float(np.max(an_h[:, -1] / an_h[:, 0])),
           "roofline": {"bound": "hbm",
                        "kernel": "LSMR iteration (ppf_fwd + ppf_adj)",
                        "achieved": round(achieved, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "algorithmic_bytes_per_iteration": it_bytes}}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = ppf_cpu_baseline(cfg, d, a.ppf_iters)
    del x, work
    torch.cuda.empty_cache()
    return out


def two_stage_leg(a, ctx, p, blk, x, stream, n_groups: int = 8,
                  steps: int = 5):
    """Two-stage beamforming of the block (8 compact station groups, 7
    preliminary beams: the centre beam and a ring at 0.2 deg), timed with
    HIP events beside the single-stage beamformer on the same block."""
    import torch

    import lofarsim
    from paper_1612_06592_amd import lp
    cfg = blk.cfg
    group = lofarsim.station_groups(blk.enu, n_groups)
    prelim = lofarsim.hex_beams(blk.az_el[0][0], blk.az_el[0][1], 1,
                                spacing_deg=0.2)
    G, P, S, n_t = n_groups, len(prelim), cfg.n_sb, cfg.n_t
    grp, pre = lp.Groups(group, G), lp.Dirs(prelim)
    y1 = torch.empty((G * P, S, n_t, 2), dtype=torch.float32, device=x.device)
    dt = lp.LP_CI8 if cfg.dtype == "ci8" else lp.LP_CI16

    def s1():
        lp.beamform_groups(ctx, p.array, grp, p.band, pre, x, n_t, y1,
                           dtype=dt, prec=p.prec, stream=stream)

    def s2():
        lp.beamform_stage2(ctx, p.array, grp, p.band, pre, p.dirs, y1, n_t,
                           p.y_view(), stream=stream)

    def single():
        p.beamform(x, stream)

    out = {}
    for name, fn in (("stage1_ms", s1), ("stage2_ms", s2),
                     ("single_stage_ms", single)):
        fn()
        ev = [(torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for e0, e1 in ev:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        out[name] = round(float(np.mean([e0.elapsed_time(e1)
                                         for e0, e1 in ev])), 4)
    bytes2 = (G * P + cfg.n_beams) * S * n_t * 8
    gbs = bytes2 / (out["stage2_ms"] * 1e-3) / 1e9
    out.update({"groups": G, "preliminary_beams": P,
                "final_beams": cfg.n_beams,
                "stage2_roofline": {"bound": "hbm", "achieved": round(gbs, 1),
                                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(gbs / HBM_PEAK_GBS, 4),
                                    "algorithmic_bytes_per_launch": bytes2}})
    del y1
    torch.cuda.empty_cache()
    return out


def station_sim_leg(a, ctx, cfg, blk, stream, steps: int = 3):
    """The station simulator for one block of the workload's shape: every
    input's 5 ns ADC stream (Philox noise, 16 words) with 15 frames of
    history, then the station filterbank into the beamformer's input
    layout; HIP events around each stage."""
    import torch
    from paper_1612_06592_amd import lp
    n_in, S, nf = cfg.n_in, cfg.n_sb, cfg.n_t
    n_samp = (nf + 15) * 1024
    band = lp.Band(blk.k)
    adc = torch.empty((n_in, n_samp), dtype=torch.int16, device="cuda:0")
    x = torch.empty((S, nf, n_in, 2),
                    dtype=torch.int8 if cfg.dtype == "ci8" else torch.int16,
                    device="cuda:0")
    work = torch.empty(lp.nbytes("lp_station_work_bytes", n_in, S, nf),
                       dtype=torch.uint8, device="cuda:0")
    dt = lp.LP_CI8 if cfg.dtype == "ci8" else lp.LP_CI16
    # Subband sigma 8 from ADC sigma sqrt(128) (16 noise words).
    import lofarsim
    hp = lofarsim.kaiser_sinc(1024, 16)
    scale = 8.0 / (np.sqrt(128.0) * np.sqrt(np.sum(hp * hp) / 2))

    def run(e):
        e[0].record(stream)
        lp.sim_adc(ctx, 1612, n_in, 16, 12, 1, n_samp, adc, stream=stream)
        e[1].record(stream)
        lp.station_ppf(ctx, band, adc, n_in, nf, scale, x, work, dt,
                       stream=stream)
        e[2].record(stream)

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)]
          for _ in range(steps + 1)]
    for e in ev:
        run(e)
    torch.cuda.synchronize()
    t_adc = float(np.mean([e[0].elapsed_time(e[1]) for e in ev[1:]]))
    t_ppf = float(np.mean([e[1].elapsed_time(e[2]) for e in ev[1:]]))
    total = t_adc + t_ppf
    samples = n_in * n_samp
    out = {"inputs": n_in, "adc_samples": samples, "subbands": S,
           "frames": nf, "adc_ms": round(t_adc, 3),
           "station_ppf_ms": round(t_ppf, 3),
           "value": round(samples / (total * 1e-3) / 1e9, 2),
           "unit": "G ADC samples/s (noise + station filterbank)",
           "rtf": round(cfg.block_seconds * 1e3 / total, 1)}
    del adc, x, work
    torch.cuda.empty_cache()
    if not a.no_cpu_baseline:
        import oracle
        from oracle import station_sim
        h = oracle.prototype(1024, 16, 9.0)
        t0 = time.perf_counter()
        codes = station_sim.adc(1612, 1, 16, 12, 1, (1024 + 15) * 1024)
        station_sim.station_ppf(h, 1024, np.asarray(blk.k), codes, scale, 8)
        dt_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round((1024 + 15) * 1024 / dt_cpu / 1e9, 6),
            "unit": "G ADC samples/s", "cores": 1, "kind": "oracle",
            "sample": "1 input x 1024 frames (numpy)",
            "seconds": round(dt_cpu, 2)}
    return out


def ppf_cpu_baseline(cfg, d, iters: int, frames: int = 1024):
    """The oracle's LSMR (numpy FP64) on the first `frames` frames of
    series 0, scaled to the leg's unit (series-frames per second)."""
    import oracle
    from oracle import ppf_lsmr
    y = d[0, :, :frames].cpu().numpy().astype(np.float64)
    y = y[..., 0] + 1j * y[..., 1]
    h = oracle.prototype(1024, 16, 9.0)
    t0 = time.perf_counter()
    ppf_lsmr.invert(h, 1024, np.asarray(cfg.k), y, iters)
    dt = time.perf_counter() - t0
    # numpy's FFT and elementwise operations run on one thread.
    return {"value": round(frames / dt, 1), "unit": "frames/s per series",
            "cores": 1, "kind": "oracle",
            "sample": f"{iters} LSMR iterations on frames 0..{frames - 1} "
                      f"of series 0", "seconds": round(dt, 2)}


def sample_beams(cfg, blk, n_beams: int = 0):
    """Beams of the oracle's sample: the injected pulses' beams first, then
    the lowest others, up to n_beams (0: max(1, 8 // trials))."""
    B = cfg.n_beams
    n = n_beams or max(1, 8 // cfg.n_tec)
    n = min(n, B)
    sel = []
    for pl in blk.pulses:
        b = int(pl["beam"])
        if b not in sel and len(sel) < n:
            sel.append(b)
    for b in range(B):
        if len(sel) >= n:
            break
        if b not in sel:
            sel.append(b)
    return sorted(sel)


def first_block_outputs(p, sel):
    """Host copies of the sampled beams' outputs of the block just run."""
    import torch
    idx = torch.tensor(sel, device=p.bufs["y"].device)
    J, n_t = p.n_tec, p.n_t
    emax, _, _ = p.cand_view()
    qs = [b * J + j for b in sel for j in range(J)]
    q = torch.tensor(qs, device=idx.device)
    trig = p.triggers()
    return dict(
        y=p.y_view().index_select(0, idx).cpu().numpy(),
        d=p.d_view().index_select(0, idx).cpu().numpy(),
        emax=emax.index_select(0, q).cpu().numpy(),
        sigma=p.bufs["sigma"].index_select(0, idx).cpu().numpy().ravel(),
        snr=p.bufs["snr"].index_select(0, idx).cpu().numpy().ravel(),
        best=p.bufs["best"].index_select(0, idx).cpu().numpy(),
        trig=trig[np.isin(trig["beam"], sel)],
        n_trig=int(p.bufs["n_trig"].item()), n_kept=len(trig), n_t=n_t)


def _c(a):
    return a[..., 0].astype(np.float64) + 1j * a[..., 1].astype(np.float64)


def _rel_rms(a, b) -> float:
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))


def compare_trigger_lists(g, o, k_sigma: float, tol: int = 1,
                          border: float = 0.01):
    """Beam exact, sample within tol; a trigger without partner whose SNR is
    within `border` (relative) of the threshold is a borderline decision
    (FP16 and FP64 envelopes differ by ~1e-4) and is listed, not failed."""
    used, missing, border_n = set(), 0, 0
    for t in o:
        hit = None
        for i, u in enumerate(g):
            if i not in used and int(u["beam"]) == int(t["beam"]) and \
                    abs(int(u["sample"]) - int(t["sample"])) <= tol:
                hit = i
                break
        if hit is None:
            if abs(t["snr"] / k_sigma - 1.0) > border:
                missing += 1
            else:
                border_n += 1
        else:
            used.add(hit)
    extra = 0
    for i, u in enumerate(g):
        if i not in used:
            if abs(u["snr"] / k_sigma - 1.0) > border:
                extra += 1
            else:
                border_n += 1
    return {"equal": missing == 0 and extra == 0, "gpu": int(len(g)),
            "oracle": int(len(o)), "missing": missing, "extra": extra,
            "borderline": border_n}


def run_cpu_baseline(blk, sel, first):
    """Time the oracle chain (as it stands) on the sampled beams of the
    first block (fresh stream: all subbands, inputs, trials and samples),
    and compare the GPU's outputs of that block with it."""
    import oracle
    cfg = blk.cfg
    n_t = blk.n_t
    st = oracle.Stream(blk.enu, 2, blk.k, blk.az_el[sel], blk.tec,
                       series_group=4, keep_z=False)
    t0 = time.perf_counter()
    r = st.process(blk.x)
    dt = time.perf_counter() - t0
    samples = cfg.n_in * cfg.n_sb * n_t * len(sel)
    out = {"value": round(samples / dt / 1e6, 3), "unit": "Msamples/s",
           "cores": oracle.threads(), "kind": "oracle",
           "sample": f"first block (fresh stream), beams {sel} of "
                     f"{cfg.n_beams}: all {cfg.n_sb} subbands, {cfg.n_in} "
                     f"inputs, {cfg.n_tec} trials, {n_t} samples",
           "seconds": round(dt, 2), "cpu_model": cpu_model(),
           "nproc": os.cpu_count()}
    o_trig = r.triggers.copy()
    o_trig["beam"] = np.asarray(sel)[o_trig["beam"]]
    err = {"block": "first (fresh stream)", "beams": sel,
           "y_rel_rms": _rel_rms(_c(first["y"]), r.y),
           "d_rel_rms": _rel_rms(_c(first["d"]), r.d),
           "window_max_rel_rms": _rel_rms(first["emax"].astype(np.float64),
                                          r.wmax),
           "sigma_max_rel": float(np.max(np.abs(first["sigma"] - r.sigma)
                                         / r.sigma)),
           "peak_snr_max_rel": float(np.max(
               np.abs(first["snr"] - r.snr_peak.ravel())
               / np.maximum(r.snr_peak.ravel(), 1e-30))),
           "best_tec_equal": bool(np.array_equal(first["best"], r.best_tec)),
           "triggers": compare_trigger_lists(first["trig"], o_trig, 6.0),
           "bound": 1e-3}
    err["within_bound"] = bool(
        max(err["y_rel_rms"], err["d_rel_rms"],
            err["window_max_rel_rms"]) <= 1e-3 and
        err["triggers"]["equal"] and err["best_tec_equal"] and
        first["n_trig"] == first["n_kept"])
    # The same chain on one thread, over its first hop only (a fresh
    # stream, so the same arithmetic as the first hop above); for the
    # single-beam, single-trial workloads (C1, C2), where it takes seconds.
    if cfg.n_beams * cfg.n_tec > 1:
        return out, err
    n1 = min(2048, n_t)
    cores = oracle.threads()
    oracle.set_threads(1)
    try:
        st1 = oracle.Stream(blk.enu, 2, blk.k, blk.az_el, blk.tec)
        t0 = time.perf_counter()
        st1.process(blk.x[:, :n1])
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    out["single_thread"] = {
        "value": round(cfg.n_in * cfg.n_sb * n1 * cfg.n_beams / dt1 / 1e6, 3),
        "unit": "Msamples/s", "sample": f"first {n1} samples per subband",
        "seconds": round(dt1, 2)}
    return out, err


def whole_step(cfg, ms_per_step: float):
    """The whole chain per step against both rooflines: algorithmic HBM
    bytes and FP32 FLOP of beamform + de-dispersion + synthesis."""
    n_t = cfg.n_t
    by = sum(algorithmic_bytes(s, cfg, n_t)
             for s in ("beamform", "dedisperse", "synthesize"))
    fl = sum(algorithmic_flop(s, cfg, n_t)
             for s in ("dedisperse", "synthesize"))
    sec = ms_per_step * 1e-3
    return {"hbm_bytes": by, "GBps": round(by / sec / 1e9, 1),
            "frac_hbm": round(by / sec / 1e9 / HBM_PEAK_GBS, 4),
            "fp32_flop": fl, "TFLOPs": round(fl / sec / 1e12, 2),
            "frac_fp32": round(fl / sec / 1e12 / FP32_PEAK_TFLOPS, 4)}


def cpu_model() -> str:
    """The host CPU's model name, as the kernel reports it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def serving_bench(a):
    """C5: concurrent observation streams through the serving loop."""
    import threading

    import torch

    import lofarsim
    from paper_1612_06592_amd import lp

    dev = "cuda:0"
    specs = lofarsim.serving_streams(12, max_log2_nt=a.max_log2_nt)
    gen = torch.Generator(device=dev)
    pools, cfgs, args = [], [], []
    for sp in specs:
        gen.manual_seed(sp["seed"])
        rng = np.random.default_rng(sp["seed"])
        n_in, n_sb = sp["n_st"] * 2, len(sp["k"])
        nbytes = n_sb * (1 << a.max_log2_nt) * n_in * 2
        pool = torch.empty(nbytes, dtype=torch.int8, device=dev)
        step = 1 << 28
        for o in range(0, nbytes, step):
            m = min(step, nbytes - o)
            v = torch.randn(m, generator=gen, device=dev) * 8.0
            pool[o:o + m] = v.round_().clamp_(-127, 127).to(torch.int8)
            del v
        pools.append(pool)
        enu = lofarsim.stations_in_disk(rng, sp["n_st"], 2000.0)
        az0, el0 = lofarsim.moon_direction(rng)
        rings = {7: 1, 19: 2, 37: 3, 61: 4}[sp["n_beams"]]
        args.append((enu, sp["k"], lofarsim.hex_beams(az0, el0, rings),
                     [sp["tec"]], 1 << a.max_log2_nt))
        cfgs.append(lp.StreamCfg(*args[-1], dtype=lp.LP_CI8,
                                 prec=lp.LP_FP16_MFMA, trig_cap=256))
    torch.cuda.synchronize()
    print(f"[bench] c5: {len(specs)} stream pools generated", file=sys.stderr,
          flush=True)
    ctx = lp.Ctx(0)
    chunk_t = 16384
    resident = sum(c.resident_bytes(chunk_t) for c in cfgs)
    blk_max = [c.block_bytes(1 << a.max_log2_nt) for c in cfgs]
    if a.arena_frac >= 1.0:
        arena_bytes = resident + sum(blk_max) + (1 << 30)
    else:
        # Smaller than what all streams' blocks need at once, never smaller
        # than the largest single block (it must be admissible alone).
        arena_bytes = resident + max(max(blk_max),
                                     int(a.arena_frac * sum(blk_max))) + (256 << 20)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    lens = [1 << e for e in range(12, a.max_log2_nt + 1)]

    def calibrate(srv, ids):
        """Service time alone: one block of each length per stream (the
        first run also creates the stream's tables)."""
        def run_alone(i, n_t):
            srv.submit(ids[i], pools[i], n_t, tag=1 << 40)
            while True:
                r = srv.poll(timeout_us=1000000)
                if r:
                    return r[0]
        svc = []
        for i in range(len(ids)):
            run_alone(i, lens[0])
            t = [run_alone(i, n)["latency_ns"] * 1e-9 for n in lens]
            svc.append(dict(zip(lens, t)))
        return svc

    # The same streams at FP32 (the fused path without the matrix cores),
    # alone, for the precision comparison.
    srv = lp.Server(ctx, arena, arena_bytes, max_slots=16, chunk_t=chunk_t)
    cfgs32 = [lp.StreamCfg(*g, dtype=lp.LP_CI8, prec=lp.LP_FP32, trig_cap=256)
              for g in args]
    ids = [srv.open(c) for c in cfgs32]
    svc32 = calibrate(srv, ids)
    srv.destroy()

    srv = lp.Server(ctx, arena, arena_bytes, max_slots=16, chunk_t=chunk_t)
    ids = [srv.open(c) for c in cfgs]
    sbs = [c.array.n_in * c.band.n_sb * c.dirs.n for c in cfgs]
    svc = calibrate(srv, ids)
    mean_svc = [float(np.mean(list(d.values()))) for d in svc]
    rate = [a.load / (len(ids) * m) for m in mean_svc]   # blocks per second
    print(f"[bench] c5: calibrated; mean service ms "
          f"{[round(m * 1e3, 2) for m in mean_svc]}", file=sys.stderr, flush=True)

    # Poisson arrivals, block length log-uniform (uniform exponent).
    rng = np.random.default_rng(7)
    events = []
    for i in range(len(ids)):
        t = 0.0
        while True:
            t += rng.exponential(1.0 / rate[i])
            if t > a.duration:
                break
            events.append((t, i, int(rng.choice(lens))))
    events.sort()
    results = []
    done = threading.Event()

    def poller():
        while not (done.is_set() and len(results) >= len(events)):
            results.extend(srv.poll(timeout_us=20000))

    th = threading.Thread(target=poller)
    th.start()
    t_start = time.perf_counter()
    for k, (t, i, n) in enumerate(events):
        now = time.perf_counter() - t_start
        if t > now:
            time.sleep(t - now)
        srv.submit(ids[i], pools[i], n, tag=k)
    done.set()
    th.join()
    wall = time.perf_counter() - t_start
    stats = srv.stats()
    srv.destroy()
    del arena
    torch.cuda.empty_cache()
    plain = None
    if a.plain_max_log2_nt > 0:
        plain = plain_alone(a, ctx, args, pools, svc, lens)
    ctx.close()
    ok = [r for r in results if r["status"] == lp.LP_OK]
    lat = np.array([r["latency_ns"] for r in ok]) * 1e-6
    dl = np.array([r["deadline_ns"] for r in ok]) * 1e-6
    samples = sum(sbs[r["stream"] - ids[0]] * r["n_t"] for r in ok)
    busy = sum(svc[r["stream"] - ids[0]][r["n_t"]] for r in ok)
    out = {
        "metric": METRIC, "value": round(samples / wall / 1e6, 1),
        "unit": "Msamples/s", "n_gpus": 1, "steps": len(ok), "warmup": 0,
        "ms_per_step": round(wall * 1e3 / max(1, len(ok)), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16-mfma/f32", "data": "synthetic",
        "config": {"workload": "c5-serving", "streams": len(ids),
                   "block_samples": [lens[0], lens[-1]], "chunk": chunk_t,
                   "offered_load": a.load, "duration_s": a.duration},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "max": round(float(lat.max()), 3),
                       "deadline_min": round(float(dl.min()), 1),
                       "missed": int(np.sum(lat > dl))},
        "blocks": {"done": len(ok), "failed": len(results) - len(ok),
                   "chunks": stats["chunks_issued"],
                   "admit_waits": stats["admit_waits"]},
        "arena": {"bytes": arena_bytes, "frac": a.arena_frac,
                  "resident_bytes": resident,
                  "longest_blocks_bytes": sum(blk_max)},
        "measured_load": round(busy / wall, 3),
        # Sum over streams and block lengths of the time alone per block.
        "service_alone_s": {
            "fp16_mfma": round(sum(sum(d.values()) for d in svc), 4),
            "fp32": round(sum(sum(d.values()) for d in svc32), 4),
            "fp32_over_fp16": round(sum(sum(d.values()) for d in svc32)
                                    / sum(sum(d.values()) for d in svc), 3)},
        "plain_fp32_alone": plain,
    }
    print(json.dumps(out))


def plain_alone(a, ctx, args, pools, svc, lens):
    """The plain FP32 pipeline (every intermediate in HBM) on each stream
    alone, one block of each length up to 2^plain_max_log2_nt, against the
    served FP16-MFMA blocks' service times at the same lengths."""
    import torch
    from paper_1612_06592_amd import lp
    use = [n for n in lens if n <= (1 << a.plain_max_log2_nt)]
    t_plain = t_fp16 = 0.0
    for i, (enu, k, dirs, tec, _) in enumerate(args):
        for n in use:
            pp = lp.Pipeline(ctx, lp.Array(enu, 2), lp.Band(k), lp.Dirs(dirs),
                             tec, n, dtype=lp.LP_CI8, plain=True,
                             device=pools[i].device)
            nb = len(k) * n * enu.shape[0] * 2 * 2
            xb = pools[i][:nb]
            pp.step(xb)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pp.step(xb)
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t0
            t_fp16 += svc[i][n]
            del pp
            torch.cuda.empty_cache()
    return {"lengths": [use[0], use[-1]], "blocks": len(use) * len(args),
            "plain_s": round(t_plain, 4), "fp16_mfma_served_s": round(t_fp16, 4),
            "plain_over_fp16": round(t_plain / t_fp16, 2),
            "kind": "sum over streams and lengths of one block alone: the plain "
                    "pipeline called directly, the FP16-MFMA block through the "
                    "server"}


if __name__ == "__main__":
    main()
