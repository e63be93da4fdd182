"""GPU parity: the HIP chain (through the C ABI) against the FP64 oracle on
the same seeded blocks.

Tolerances (relative RMS over each stage's whole output):
  FP16-MFMA beamformer path: 1e-3 (the target bound); FP32 path: 1e-5.
Triggers: beam exact and sample within +-1, except decisions within 1% of
the 6-sigma threshold (see chain.compare_triggers).  Window maxima are
compared in value; their positions must agree except where the oracle's
own envelope at the GPU's position is within 1e-3 of its maximum.
"""
import numpy as np
import pytest

import lofarsim
from chain import (PER_ELEM, WARM, OracleChain, compare_triggers, max_err,
                   rel_rms, run_gpu)
from paper_1612_06592_amd import lp

pytestmark = pytest.mark.gpu

TOL = {lp.LP_FP16_MFMA: 1e-3, lp.LP_FP32: 1e-5}


def _check_block(g, o, prec, keep=(0,), label="", frame0=0):
    tol, pe = TOL[prec], PER_ELEM[prec]
    e, m = rel_rms(g["y"], o["y"]), max_err(g["y"], o["y"])
    print(f"{label} y rel-rms {e:.2e} max {m:.2e}", flush=True)
    assert e <= tol and m <= pe
    e, m = rel_rms(g["d"], o["d"]), max_err(g["d"], o["d"])
    print(f"{label} d rel-rms {e:.2e} max {m:.2e}", flush=True)
    assert e <= tol and m <= pe
    for q in keep:
        if g["x"] is not None and q in o["z"]:
            xo = 2 * o["z"][q].real
            e, m = rel_rms(g["x"][q], xo), max_err(g["x"][q], xo)
            print(f"{label} x[{q}] rel-rms {e:.2e} max {m:.2e}", flush=True)
            assert e <= tol and m <= pe
    ns, n_t = o["wmax"].shape
    e, m = rel_rms(g["emax"], o["wmax"]), max_err(g["emax"], o["wmax"])
    print(f"{label} window-max rel-rms {e:.2e} max {m:.2e}", flush=True)
    assert e <= tol and m <= pe, (e, m)
    gs = g["sigma"].reshape(-1)
    assert np.max(np.abs(gs - o["sigma"]) / np.maximum(o["sigma"], 1e-30)) <= tol
    # Window arg-max over valid frames (start-up frames of a fresh stream
    # are numerically zero on both sides): equal, or an equally good
    # sample of the oracle.
    first = max(0, WARM - frame0)
    for q in keep:
        if q not in o["z"]:
            continue
        env = np.abs(2 * o["z"][q]).reshape(n_t, 1024)
        ga = g["arg"][q]
        oa = o["warg"][q] % 1024
        bad = [m for m in np.nonzero(ga != oa)[0] if m >= first]
        for m in bad:
            assert env[m, ga[m]] >= (1 - 1e-3) * env[m, oa[m]], (q, m)
        assert len(bad) <= max(2, n_t // 100)
    miss, extra = compare_triggers(g["trig"], o["trig"], o["sigma"])
    print(f"{label} triggers gpu={len(g['trig'])} oracle={len(o['trig'])}",
          flush=True)
    assert not miss and not extra, (miss, extra)
    assert g["n_trig"] == len(g["trig"])
    assert np.array_equal(g["best"], o["best"])
    assert np.max(np.abs(g["snr"].reshape(-1) - o["snr"].reshape(-1))
                  / np.maximum(o["snr"].reshape(-1), 1e-30)) <= 2 * tol


@pytest.mark.parametrize("prec", [lp.LP_FP32, lp.LP_FP16_MFMA])
def test_c1_tiny_full(prec):
    blk = lofarsim.generate(lofarsim.get_config("c1"))
    print("case c1", prec, flush=True)
    g = run_gpu(blk, prec)
    o = OracleChain(blk).process(blk.x, keep_series=(0,))
    _check_block(g, o, prec, label=f"c1 prec={prec}")
    # The injected pulse is found.
    assert any(abs(int(t["sample"]) - blk.pulses[0]["n0"]) <= 1 for t in g["trig"])


@pytest.mark.parametrize("prec", [lp.LP_FP32, lp.LP_FP16_MFMA])
def test_c2_slice_core_single_beam(prec):
    cfg = lofarsim.get_config("c2", n_t=4096, n_pulses=1)
    blk = lofarsim.generate(cfg)
    print("case c2-slice", prec, flush=True)
    g = run_gpu(blk, prec)
    o = OracleChain(blk).process(blk.x, keep_series=(0,))
    _check_block(g, o, prec, label=f"c2s prec={prec}")


def test_c3_slice_multibeam_19():
    cfg = lofarsim.get_config("c3", n_t=4096, hex_rings=2,
                              k=tuple(range(52, 76)))
    blk = lofarsim.generate(cfg)
    print("case c3-slice 19 beams", flush=True)
    g = run_gpu(blk, lp.LP_FP16_MFMA)
    o = OracleChain(blk).process(blk.x, keep_series=(0, 5, 18))
    _check_block(g, o, lp.LP_FP16_MFMA, keep=(0, 5, 18), label="c3s")


def test_beamform_61_beams_96_inputs():
    """C3's GEMM shape (96 inputs x 61 beams): two n-tiles per wave."""
    cfg = lofarsim.get_config("c3", n_t=2048, k=tuple(range(52, 84)))
    blk = lofarsim.generate(cfg)
    import oracle
    import torch
    from chain import as_complex, gpu_pipeline, to_device
    for prec in (lp.LP_FP16_MFMA, lp.LP_FP32):
        ctx, p = gpu_pipeline(blk, prec, want_series=False)
        p.beamform(to_device(blk.x))
        torch.cuda.synchronize()
        y = as_complex(p.y_view())
        ctx.close()
        ref = oracle.beamform(blk.enu, 2, blk.k, blk.az_el, blk.x)
        e = rel_rms(y, ref)
        print("bf61 prec", prec, "rel-rms", e, flush=True)
        assert e <= TOL[prec]


@pytest.mark.parametrize("n_st,precs", [
    (64, (lp.LP_FP32,)),                     # 128 inputs: 512-byte rows
    (32, (lp.LP_FP16_MFMA, lp.LP_FP32)),     # 64 inputs: the MFMA maximum
])
def test_beamform_largest_shapes_ci16(n_st, precs):
    """The largest documented beamformer calls with int16 samples and 64
    beams: 128 inputs on the FP32 path (its tile is halved to fit LDS; the
    MFMA path rejects 512-byte rows with LP_EINVAL), 64 inputs on both."""
    cfg = lofarsim.get_config("c1", n_st=n_st, hex_rings=4, n_t=256,
                              k=tuple(range(200, 206)), n_pulses=0)
    blk = lofarsim.generate(cfg)
    blk.az_el = np.concatenate([blk.az_el, blk.az_el[:3] + 0.001])
    assert blk.az_el.shape[0] == 64 and blk.x.dtype == np.int16
    import oracle
    import torch
    from chain import as_complex, gpu_pipeline, to_device
    ref = oracle.beamform(blk.enu, 2, blk.k, blk.az_el, blk.x)
    for prec in precs:
        print("case bf-max n_st", n_st, "prec", prec, flush=True)
        ctx, p = gpu_pipeline(blk, prec, want_series=False)
        p.beamform(to_device(blk.x))
        torch.cuda.synchronize()
        e = rel_rms(as_complex(p.y_view()), ref)
        ctx.close()
        print("bf-max prec", prec, "rel-rms", e, flush=True)
        assert e <= TOL[prec]
    if n_st == 64:
        ctx, p = gpu_pipeline(blk, lp.LP_FP16_MFMA, want_series=False)
        with pytest.raises(lp.LpError, match="256 bytes"):
            p.beamform(to_device(blk.x))
        ctx.close()


def test_c4_slice_tec_grid():
    tec = tuple(np.linspace(0, 30, 32).tolist())
    cfg = lofarsim.get_config("c4", n_t=2048, k=tuple(range(52, 68)),
                              n_pulses=1, snr=(30.0, 30.0))
    blk = lofarsim.generate(cfg)
    print("case c4-slice", cfg.true_tec_index, flush=True)
    g = run_gpu(blk, lp.LP_FP16_MFMA)
    keep = (0, cfg.true_tec_index, 6 * 32 + 31)
    o = OracleChain(blk).process(blk.x, keep_series=keep)
    _check_block(g, o, lp.LP_FP16_MFMA, keep=keep, label="c4s")


def test_odd_shapes_and_ci16_mfma():
    """Inputs not a multiple of 16 real rows (6 stations), 3 beams, int16
    samples on the MFMA path, a single hop."""
    cfg = lofarsim.get_config("c1", n_st=6, hex_rings=0, n_t=2048,
                              k=tuple(range(300, 311)))
    blk = lofarsim.generate(cfg)
    blk.az_el = np.concatenate([blk.az_el, blk.az_el + 0.002,
                                blk.az_el - 0.003])
    for prec in (lp.LP_FP16_MFMA, lp.LP_FP32):
        g = run_gpu(blk, prec)
        o = OracleChain(blk).process(blk.x, keep_series=(0, 2))
        _check_block(g, o, prec, keep=(0, 2), label=f"odd prec={prec}")


@pytest.mark.parametrize("n_st", [3, 6])
def test_beamform_narrow_int8_rows(n_st):
    """int8 rows that are not a multiple of 16 bytes (3 stations: 12-byte
    rows, loaded as 4-byte vectors; 6 stations: 24-byte rows, 8-byte
    vectors), zero-padded to a 16-sample k-step, on both precisions."""
    cfg = lofarsim.get_config("c2", n_st=n_st, hex_rings=1, n_t=1024,
                              k=tuple(range(52, 61)), n_pulses=0)
    blk = lofarsim.generate(cfg)
    assert blk.x.dtype == np.int8 and (2 * 2 * n_st) % 16 != 0
    import oracle
    import torch
    from chain import as_complex, gpu_pipeline, to_device
    ref = oracle.beamform(blk.enu, 2, blk.k, blk.az_el, blk.x)
    for prec in (lp.LP_FP16_MFMA, lp.LP_FP32):
        print("case bf-narrow n_st", n_st, "prec", prec, flush=True)
        ctx, p = gpu_pipeline(blk, prec, want_series=False)
        p.beamform(to_device(blk.x))
        torch.cuda.synchronize()
        e = rel_rms(as_complex(p.y_view()), ref)
        ctx.close()
        print("bf-narrow prec", prec, "rel-rms", e, flush=True)
        assert e <= TOL[prec]


def test_stream_state_carry_bitwise():
    """Two consecutive blocks through carried state equal one long block
    (bitwise for every sample-local output)."""
    cfg = lofarsim.get_config("c2", n_t=8192, k=tuple(range(52, 84)),
                              n_pulses=1)
    blk = lofarsim.generate(cfg)
    one = run_gpu(blk, lp.LP_FP16_MFMA)
    two = run_gpu(blk, lp.LP_FP16_MFMA, blocks=4096)
    assert np.array_equal(np.concatenate([two[0]["d"], two[1]["d"]], -1),
                          one["d"])
    assert np.array_equal(np.concatenate([two[0]["x"], two[1]["x"]], -1),
                          one["x"])
    assert np.array_equal(np.concatenate([two[0]["emax"], two[1]["emax"]], -1),
                          one["emax"])
    # And both match the oracle run the same way.
    oc = OracleChain(blk)
    o1 = oc.process(blk.x[:, :4096], keep_series=(0,))
    o2 = oc.process(blk.x[:, 4096:], keep_series=(0,))
    assert rel_rms(two[1]["x"][0], 2 * o2["z"][0].real) <= 1e-3
    miss, extra = compare_triggers(two[1]["trig"], o2["trig"], o2["sigma"])
    assert not miss and not extra


def test_determinism_bitwise():
    cfg = lofarsim.get_config("c2", n_t=4096, k=tuple(range(52, 100)))
    blk = lofarsim.generate(cfg)
    a = run_gpu(blk, lp.LP_FP16_MFMA)
    b = run_gpu(blk, lp.LP_FP16_MFMA)
    for k in ("y", "d", "x", "emax", "arg", "sigma", "snr"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["trig"], b["trig"])


@pytest.mark.parametrize("frame0", [0, 8, 16, 1000, 1037, 1040, 4096])
def test_synthesis_warmup_statistics(frame0):
    """Variance sums exclude exactly the warm-up frames (stream time below
    WARM) also where that boundary falls inside a 16-frame chunk (stream
    positions that are not multiples of 16); window maxima do not depend
    on the position.  Against the oracle's synthesis and detection on the
    same FP32 subband samples."""
    import torch

    import oracle
    rng = np.random.default_rng(1612 + frame0)
    k = np.arange(52, 84)
    S, n_t, ns = len(k), 2048, 2
    d = (rng.standard_normal((ns, S, n_t))
         + 1j * rng.standard_normal((ns, S, n_t))).astype(np.complex64)
    ctx = lp.Ctx(0)
    band = lp.Band(k)
    dd = torch.from_numpy(d.view(np.float32).reshape(ns, S, n_t, 2)).to("cuda:0")
    hist = torch.zeros(ns * S * 16 * 2, dtype=torch.float32, device="cuda:0")
    cand = torch.empty(lp.nbytes("lp_cand_bytes", ns, n_t), dtype=torch.uint8,
                       device="cuda:0")
    print(f"synthesis warm-up statistics, frame0 {frame0}", flush=True)
    lp.synthesize(ctx, band, dd, ns, n_t, frame0, hist, cand)
    torch.cuda.synchronize()
    cb = cand.cpu().numpy()
    c = cb[:ns * n_t * 8].view(np.float32).reshape(ns, n_t, 2)
    emax, arg = c[..., 0], c[..., 1].view(np.int32)
    psum = cb[ns * n_t * 8:ns * n_t * 8 + ns * (n_t // 16) * 4].view(
        np.float32).reshape(ns, n_t // 16)
    ctx.close()
    h = oracle.prototype()
    z = oracle.synthesize(h, k, d.astype(np.complex128),
                          np.zeros((ns, 15, S), np.complex128))
    sigma, wmax, warg = oracle.detect(z, n_t, frame0, WARM)
    n_valid = int(np.sum(frame0 + np.arange(n_t) >= WARM))
    if n_valid:
        gs = np.sqrt(psum.astype(np.float64).sum(1) / (n_valid * 1024))
        assert np.max(np.abs(gs - sigma) / sigma) <= 1e-5, (gs, sigma)
    else:
        assert not np.any(psum)
    # Chunks wholly inside the warm-up contribute nothing.
    whole = (WARM - frame0) // 16
    if whole > 0:
        assert not np.any(psum[:, :min(whole, n_t // 16)])
    assert rel_rms(emax, wmax) <= 1e-5
    # Arg-max: the oracle's, or a sample whose envelope is within 1e-5 of
    # the window maximum (a near tie).
    env = np.abs(2 * z).reshape(ns, n_t, 1024)
    for q in range(ns):
        for m in np.nonzero(arg[q] != warg[q] % 1024)[0]:
            assert env[q, m, arg[q, m]] >= (1 - 1e-5) * wmax[q, m], (q, m)


@pytest.mark.parametrize("lo,hi", [(189, 221), (280, 312), (330, 362),
                                   (480, 512), (1, 512)])
def test_synthesis_band_rows(lo, hi):
    """Synthesis of bands whose highest bin selects each transform variant
    (pass-0 rows 4, 5, 6 and 8 of 64 bins): real series, window maxima,
    arg-max and sigma against the oracle on the same FP32 subband samples."""
    import torch

    import oracle
    rng = np.random.default_rng(lo * 1000 + hi)
    k = np.arange(lo, hi)
    S, n_t, ns = len(k), 2048, 2
    d = (rng.standard_normal((ns, S, n_t))
         + 1j * rng.standard_normal((ns, S, n_t))).astype(np.complex64)
    ctx = lp.Ctx(0)
    band = lp.Band(k)
    dd = torch.from_numpy(d.view(np.float32).reshape(ns, S, n_t, 2)).to("cuda:0")
    hist = torch.zeros(ns * S * 16 * 2, dtype=torch.float32, device="cuda:0")
    cand = torch.empty(lp.nbytes("lp_cand_bytes", ns, n_t), dtype=torch.uint8,
                       device="cuda:0")
    xs = torch.empty((ns, n_t * 1024), dtype=torch.float32, device="cuda:0")
    print(f"synthesis band {lo}..{hi - 1}", flush=True)
    lp.synthesize(ctx, band, dd, ns, n_t, 0, hist, cand, x_out=xs)
    torch.cuda.synchronize()
    cb = cand.cpu().numpy()
    x = xs.cpu().numpy()
    c = cb[:ns * n_t * 8].view(np.float32).reshape(ns, n_t, 2)
    emax, arg = c[..., 0], c[..., 1].view(np.int32)
    psum = cb[ns * n_t * 8:ns * n_t * 8 + ns * (n_t // 16) * 4].view(
        np.float32).reshape(ns, n_t // 16)
    ctx.close()
    z = oracle.synthesize(oracle.prototype(), k, d.astype(np.complex128),
                          np.zeros((ns, 15, S), np.complex128))
    sigma, wmax, warg = oracle.detect(z, n_t, 0, WARM)
    assert rel_rms(x, 2 * z.real) <= 1e-5
    assert rel_rms(emax, wmax) <= 1e-5
    gs = np.sqrt(psum.astype(np.float64).sum(1) / ((n_t - WARM) * 1024))
    assert np.max(np.abs(gs - sigma) / sigma) <= 1e-5
    env = np.abs(2 * z).reshape(ns, n_t, 1024)
    for q in range(ns):
        for m in np.nonzero(arg[q] != warg[q] % 1024)[0]:
            assert env[q, m, arg[q, m]] >= (1 - 1e-5) * wmax[q, m], (q, m)


@pytest.mark.parametrize("case", ["c1", "c2s"])
def test_plain_fp32_comparator(case):
    """The plain comparator pipeline matches the oracle at FP32 accuracy
    and agrees with the fused pipeline."""
    if case == "c1":
        blk = lofarsim.generate(lofarsim.get_config("c1"))
    else:
        blk = lofarsim.generate(lofarsim.get_config("c2", n_t=4096,
                                                    k=tuple(range(52, 116))))
    g = run_gpu(blk, lp.LP_FP32, plain=True, blocks=blk.n_t // 2)
    f = run_gpu(blk, lp.LP_FP32, blocks=blk.n_t // 2)
    oc = OracleChain(blk)
    for i, half in enumerate((blk.x[:, :blk.n_t // 2], blk.x[:, blk.n_t // 2:])):
        o = oc.process(np.ascontiguousarray(half), keep_series=(0,))
        _check_block(g[i], o, lp.LP_FP32, label=f"plain {case} block {i}",
                     frame0=i * blk.n_t // 2)
        assert rel_rms(g[i]["x"][0], f[i]["x"][0]) <= 1e-5


def test_invalid_arguments_rejected():
    import torch
    from chain import gpu_pipeline
    blk = lofarsim.generate(lofarsim.get_config("c1"))
    ctx, p = gpu_pipeline(blk, lp.LP_FP16_MFMA)
    x = torch.zeros(8, device="cuda:0", dtype=torch.int8)
    with pytest.raises(lp.LpError) as e:
        lp.beamform(ctx, p.array, p.band, p.dirs, x, 100, lp.LP_CI16,
                    lp.LP_FP16_MFMA, p.bufs["y"])
    assert e.value.code == lp.LP_EINVAL
    with pytest.raises(lp.LpError):
        lp.dedisperse(ctx, p.band, [5.0], p.bufs["y"], 1, 3000,
                      p.bufs["tail"], p.bufs["d"])
    with pytest.raises(lp.LpError):
        lp.dedisperse(ctx, p.band, [-1.0], p.bufs["y"], 1, 4096,
                      p.bufs["tail"], p.bufs["d"])
    many = lp.Dirs(np.tile(blk.az_el, (65, 1)))
    with pytest.raises(lp.LpError):
        lp.beamform(ctx, p.array, p.band, many, x, 4096, lp.LP_CI16,
                    lp.LP_FP16_MFMA, p.bufs["y"])
    bad = lp.Band([5, 5, 6])
    with pytest.raises(lp.LpError):
        lp.synthesize(ctx, bad, p.bufs["d"], 1, 4096, 0, p.bufs["hist"],
                      p.bufs["cand"])
    # One series of 256 subbands x 2^21 frames is 2^32 bytes: beyond the
    # synthesis kernel's 32-bit offsets, rejected before any launch.
    wide = lp.Band(np.arange(1, 257))
    with pytest.raises(lp.LpError) as e:
        lp.synthesize(ctx, wide, p.bufs["d"], 1, 1 << 21, 0, p.bufs["hist"],
                      p.bufs["cand"])
    assert "too large" in str(e.value)
    ctx.close()


@pytest.mark.parametrize("grid", ["uniform32", "nonuniform32", "descending8",
                                  "pair"])
def test_dedisperse_trial_grids(grid):
    """lp_dedisperse alone against the oracle's overlap-save chirp on every
    trial of a grid, over two consecutive blocks (the tail carried): a
    uniform grid takes the trial-to-trial chirp step, any other grid the
    per-trial phases.  Up to 30 TECU (2300 cycles of phase at 110 MHz).
    Element-wise: relative RMS per trial and the largest error of any
    sample against the trial's RMS."""
    import oracle
    import torch
    from chain import as_complex
    tec = {"uniform32": np.linspace(0, 30, 32),
           "nonuniform32": np.sort(np.random.default_rng(7).uniform(0, 30, 32)),
           "descending8": np.linspace(30, 2, 8),
           "pair": np.array([12.5, 25.0])}[grid]
    k = np.arange(52, 68)
    B, S, n_t = 2, len(k), 4096
    rng = np.random.default_rng([1612, len(tec)])
    dev = "cuda:0"
    ctx = lp.Ctx(0)
    band = lp.Band(k)
    tail_g = torch.zeros((B, S, 2048, 2), dtype=torch.float32, device=dev)
    tail_o = np.zeros((B, S, 2048), complex)
    d = torch.empty((B, len(tec), S, n_t, 2), dtype=torch.float32, device=dev)
    print("case dd grid", grid, flush=True)
    for blk in range(2):
        y = (rng.normal(0, 50, (B, S, n_t, 2))).astype(np.float32)
        lp.dedisperse(ctx, band, tec, torch.from_numpy(y).to(dev), B, n_t,
                      tail_g, d)
        torch.cuda.synchronize()
        o = oracle.dedisperse(k, tec, y[..., 0].astype(np.float64) +
                              1j * y[..., 1].astype(np.float64), tail_o)
        g = as_complex(d)
        for j in range(len(tec)):
            err = np.abs(g[:, j] - o[:, j])
            rms = np.sqrt(np.mean(np.abs(o[:, j]) ** 2))
            e = np.sqrt(np.mean(err ** 2)) / rms
            m = err.max() / rms
            if j in (0, len(tec) - 1):
                print(f"dd {grid} block {blk} trial {j} ({tec[j]:.2f} TECU): "
                      f"rel-rms {e:.2e}, max {m:.2e}", flush=True)
            assert e <= 1e-5, (j, e)
            assert m <= 1e-4, (j, m)
    ctx.close()


@pytest.mark.parametrize("group", [1, 5])
def test_trial_groups_equal_all_at_once(group):
    """lp_dedisperse_synthesize (the de-dispersed subbands held for one
    beam's group of trials) against lp_dedisperse + lp_synthesize over two
    consecutive blocks of a 2-beam, 32-trial stream: window maxima, sigma,
    peak SNR within the chirp-step rounding, identical trigger lists and best
    trials; and both against the oracle."""
    import torch
    from chain import gpu_pipeline, to_device
    tec = tuple(np.linspace(0, 30, 32).tolist())
    cfg = lofarsim.get_config("c4", n_t=4096, k=tuple(range(52, 68)),
                              n_pulses=1, snr=(30.0, 30.0), hex_rings=0)
    blk = lofarsim.generate(cfg)
    blk.az_el = np.concatenate([blk.az_el, blk.az_el + 0.002])
    print("case trial groups", group, flush=True)
    ctx, pa = gpu_pipeline(blk, lp.LP_FP16_MFMA, n_t=2048, want_series=False)
    pg = lp.Pipeline(ctx, pa.array, pa.band, pa.dirs, pa.tec, 2048,
                     dtype=pa.dtype, prec=pa.prec, trial_group=group)
    oc = OracleChain(blk)
    for i in range(2):
        x = to_device(blk.x[:, 2048 * i:2048 * (i + 1)])
        pa.step(x)
        pg.step(x)
        torch.cuda.synchronize()
        ea, eg = pa.cand_view()[0].cpu().numpy(), pg.cand_view()[0].cpu().numpy()
        e, m = rel_rms(eg, ea), max_err(eg, ea)
        print(f"block {i}: grouped vs all-at-once window max rel-rms {e:.2e} "
              f"max {m:.2e}", flush=True)
        assert e <= 1e-5 and m <= 1e-4
        sa, sg = pa.bufs["sigma"].cpu().numpy(), pg.bufs["sigma"].cpu().numpy()
        assert np.max(np.abs(sg - sa) / sa) <= 1e-5
        ta, tg = pa.triggers(), pg.triggers()
        assert len(ta) == len(tg)
        np.testing.assert_array_equal(ta["beam"], tg["beam"])
        np.testing.assert_array_equal(ta["tec"], tg["tec"])
        assert np.all(np.abs(ta["sample"] - tg["sample"]) <= 1)
        assert np.array_equal(pa.bufs["best"].cpu().numpy(),
                              pg.bufs["best"].cpu().numpy())
        o = oc.process(blk.x[:, 2048 * i:2048 * (i + 1)])
        e = rel_rms(eg, o["wmax"])
        assert e <= 1e-3, e
        miss, extra = compare_triggers(tg, o["trig"], o["sigma"])
        print(f"block {i}: {len(tg)} triggers, oracle {len(o['trig'])}",
              flush=True)
        assert not miss and not extra, (miss, extra)
    with pytest.raises(ValueError):
        pg.d_view()
    ctx.close()


def test_graph_replay_equals_eager():
    """Pipeline.step_graph (beamform, de-dispersion and synthesis replayed
    from a captured HIP graph, the trigger issued per block) against
    Pipeline.step on the same stream of five blocks, with eager work and
    synchronisations between the replays: every block's candidates, sigma,
    peak SNR and trigger list bitwise equal."""
    import torch
    from chain import gpu_pipeline, to_device
    cfg = lofarsim.get_config("c1", n_t=8192, n_pulses=2)
    blk = lofarsim.generate(cfg)
    n_t = 2048
    ctx, pa = gpu_pipeline(blk, lp.LP_FP16_MFMA, n_t=n_t, want_series=False)
    pg = lp.Pipeline(ctx, pa.array, pa.band, pa.dirs, pa.tec, n_t,
                     dtype=pa.dtype, prec=pa.prec)
    xd = torch.empty((blk.x.shape[0], n_t) + blk.x.shape[2:],
                     dtype=torch.int16, device="cuda:0")
    n_trig = 0
    for i in range(4):
        xi = to_device(blk.x[:, n_t * i:n_t * (i + 1)])
        xd.copy_(xi)            # the graph reads the same input buffer
        pa.step(xi)
        pg.step_graph(xd)
        torch.cuda.synchronize()
        for key in ("cand", "sigma", "snr", "best", "n_trig"):
            assert torch.equal(pa.bufs[key], pg.bufs[key]), (i, key)
        ta, tg = pa.triggers(), pg.triggers()
        assert ta.tobytes() == tg.tobytes(), i
        n_trig += len(ta)
        print(f"block {i} (frame0 {pa.frame0 - n_t}): graph "
              f"{'replayed' if '_graph' in pg.bufs else 'not used'}, "
              f"{len(ta)} triggers equal", flush=True)
    assert "_graph" in pg.bufs
    ctx.close()


def _trigger_snapshot(p):
    """Copies of the trigger's outputs and of the block's candidates, queued
    on the current stream (no host synchronisation)."""
    snap = {k: p.bufs[k].clone() for k in ("trig", "n_trig", "sigma", "snr",
                                           "best")}
    snap["cand"] = p._cand().clone()
    return snap


def _triggers_of(snap, cap):
    n = int(snap["n_trig"].item())
    raw = snap["trig"][: min(n, cap) * lp.TRIG_DTYPE.itemsize]
    return raw.cpu().numpy().view(lp.TRIG_DTYPE).copy()


def test_two_candidate_slots_overlapped_trigger():
    """Two candidate slots: each block's trigger on a second stream beside
    the next block, the synthesis waiting only for the trigger two blocks
    back (the bench's schedule), and the same pipeline replayed from HIP
    graphs (one per slot), against one slot run step by step: every block's
    candidates, sigma, peak SNR, best trial and trigger list bitwise
    equal."""
    import torch
    from chain import gpu_pipeline, to_device
    cfg = lofarsim.get_config("c1", n_t=8192, n_pulses=2)
    blk = lofarsim.generate(cfg)
    n_t, n_blk = 2048, 4
    ctx, pa = gpu_pipeline(blk, lp.LP_FP16_MFMA, n_t=n_t, want_series=False)
    kw = dict(dtype=pa.dtype, prec=pa.prec, cand_slots=2)
    p2 = lp.Pipeline(ctx, pa.array, pa.band, pa.dirs, pa.tec, n_t, **kw)
    pg = lp.Pipeline(ctx, pa.array, pa.band, pa.dirs, pa.tec, n_t, **kw)
    with pytest.raises(ValueError):
        lp.Pipeline(ctx, pa.array, pa.band, pa.dirs, pa.tec, n_t,
                    cand_slots=3)
    xs = [to_device(blk.x[:, n_t * i:n_t * (i + 1)]) for i in range(n_blk)]
    ref = []
    for i in range(n_blk):
        pa.step(xs[i])
        ref.append(_trigger_snapshot_after(pa))
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    done, got = [], []
    for i in range(n_blk):
        p2.beamform(xs[i])
        p2.dedisperse()
        if len(done) >= 2:
            main.wait_event(done[-2])
        p2.synthesize()
        ev = torch.cuda.Event()
        ev.record(main)
        side.wait_event(ev)
        p2.trigger(stream=side)
        with torch.cuda.stream(side):
            got.append(_trigger_snapshot(p2))
            ev2 = torch.cuda.Event()
            ev2.record(side)
        done.append(ev2)
        p2.frame0 += n_t
    torch.cuda.synchronize()
    xd = torch.empty_like(xs[0])
    graphed = []
    for i in range(n_blk):
        xd.copy_(xs[i])         # the graphs read the same input buffer
        pg.step_graph(xd)
        torch.cuda.synchronize()
        graphed.append(_trigger_snapshot_after(pg))
    for i in range(n_blk):
        for name, res in (("overlapped", got[i]), ("graph", graphed[i])):
            for key in ("cand", "n_trig", "sigma", "snr", "best"):
                assert torch.equal(ref[i][key], res[key]), (name, i, key)
            assert (_triggers_of(ref[i], pa.trig_cap).tobytes()
                    == _triggers_of(res, pa.trig_cap).tobytes()), (name, i)
        print(f"block {i}: {len(_triggers_of(ref[i], pa.trig_cap))} triggers "
              f"equal (overlapped, graph)", flush=True)
    assert "_graph" in pg.bufs and "_graph1" in pg.bufs
    emax, _, _ = pg.cand_view()
    assert torch.equal(emax, pa.cand_view()[0])
    ctx.close()


def _trigger_snapshot_after(p):
    """_trigger_snapshot of the block p just completed (frame0 advanced)."""
    p.frame0 -= p.n_t
    try:
        return _trigger_snapshot(p)
    finally:
        p.frame0 += p.n_t
