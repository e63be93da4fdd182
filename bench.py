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
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
METRIC = ("station-beam Msamples/s real-time factor at ≤1e-3 rel RMS; "
          "p99 block latency")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--prec", default="fp16", choices=["fp16", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-hops", type=int, default=32,
                    help="hops (2048 samples each) in the oracle sample")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for "
                         "calibrating HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (the hot path "
              "shards by beam or TEC trial with a broadcast of the station "
              "block; that multi-GPU path is not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import lofarsim
    from paper_1612_06592_amd import lp

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
                    prec=prec, want_series=False, device=dev)
    stream = torch.cuda.current_stream()
    if a.calib_copy_mib:
        n = a.calib_copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(a.warmup):
        p.step(x)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({a.warmup} steps)", file=sys.stderr, flush=True)

    stages = ["beamform", "dedisperse", "synthesize", "trigger"]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)]
          for _ in range(a.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(a.steps):
        e = ev[i]
        e[0].record(stream)
        p.beamform(x)
        e[1].record(stream)
        p.dedisperse()
        e[2].record(stream)
        p.synthesize()
        e[3].record(stream)
        p.trigger()
        e[4].record(stream)
        p.frame0 += cfg.n_t
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
    achieved = alg / (stage_avg[dom] * 1e-3) / 1e9
    src = {"beamform": "beamform.hip", "dedisperse": "dedisperse.hip",
           "synthesize": "synthesize.hip"}[dom]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tj = json.load(open(TRAFFIC_FILE))
        rec = tj.get(f"{dom}:{cfg.name}:{a.prec}")
        if rec and rec.get("source_sha") == kernel_source_hash(src):
            traffic = rec["bytes_per_launch"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "algorithmic_bytes_per_launch": alg,
                "avg_launch_ms": round(stage_avg[dom], 4)}

    # Trigger sanity on the last block: the injected pulses are found.
    trig = p.triggers()
    found = sum(any(abs(int(t["sample"]) - (pl["n0"] + (a.warmup + a.steps - 1)
                                             * cfg.n_t * 1024)) <= 1
                    for t in trig) for pl in blk.pulses)

    cpu = None
    if not a.no_cpu_baseline:
        cpu = run_cpu_baseline(blk, a.cpu_hops)

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
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out))


def run_cpu_baseline(blk, hops: int):
    """Time the oracle chain (as it stands) on the first `hops` hops of the
    block: all subbands, inputs, beams and trials of that time range."""
    import oracle
    cfg = blk.cfg
    n = min(hops * 2048, blk.n_t)
    xs = blk.x[:, :n]
    st = oracle.Stream(blk.enu, 2, blk.k, blk.az_el, blk.tec)
    t0 = time.perf_counter()
    st.process(xs)
    dt = time.perf_counter() - t0
    samples = cfg.n_in * cfg.n_sb * n * cfg.n_beams
    return {"value": round(samples / dt / 1e6, 3), "unit": "Msamples/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"first {n} of {blk.n_t} samples per subband "
                      f"(all {cfg.n_sb} subbands, {cfg.n_in} inputs, "
                      f"{cfg.n_beams} beams, {cfg.n_tec} trials)",
            "seconds": round(dt, 2)}


if __name__ == "__main__":
    main()
