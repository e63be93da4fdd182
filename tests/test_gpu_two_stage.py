"""Two-stage beamforming on the GPU (lp_beamform_groups, lp_beamform_stage2)
against the FP64 oracle (oracle/two_stage.py), and its effect on the
pulses' SNR through the rest of the chain.

Geometry: C3's 48 stations split into 8 compact groups
(lofarsim.station_groups), 7 preliminary beams (the Moon centre and a ring
at 0.2 deg), final beams C3's hexagonal grid at 0.1 deg spacing.
Tolerances as for the single-stage beamformer: 1e-3 relative RMS on the
FP16-MFMA path, 1e-5 on FP32; stage 2 alone (FP32) 1e-5.
"""
import numpy as np
import pytest

import lofarsim
from oracle import two_stage as ts
from paper_1612_06592_amd import lp

pytestmark = pytest.mark.gpu

TOL = {lp.LP_FP16_MFMA: 1e-3, lp.LP_FP32: 1e-5}


def _rel(a, b):
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))


def _geometry(blk, G=8):
    group = lofarsim.station_groups(blk.enu, G)
    az0, el0 = blk.az_el[0]
    prelim = lofarsim.hex_beams(az0, el0, 1, spacing_deg=0.2)
    return group, prelim


def _c(t):
    a = t.detach().cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def _dev_c(y):
    import torch
    a = np.stack([y.real, y.imag], -1).astype(np.float32)
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _run(blk, group, prelim, prec):
    import torch
    G, P, B = int(group.max()) + 1, len(prelim), len(blk.az_el)
    S, n_t = len(blk.k), blk.n_t
    ctx = lp.Ctx(0)
    arr, band = lp.Array(blk.enu, 2), lp.Band(blk.k)
    grp, pre, fin = lp.Groups(group, G), lp.Dirs(prelim), lp.Dirs(blk.az_el)
    x = torch.from_numpy(blk.x).to("cuda:0")
    y1 = torch.empty((G * P, S, n_t, 2), dtype=torch.float32, device="cuda:0")
    y = torch.empty((B, S, n_t, 2), dtype=torch.float32, device="cuda:0")
    dt = lp.LP_CI8 if blk.x.dtype == np.int8 else lp.LP_CI16
    lp.beamform_groups(ctx, arr, grp, band, pre, x, n_t, y1, dtype=dt,
                       prec=prec)
    lp.beamform_stage2(ctx, arr, grp, band, pre, fin, y1, n_t, y)
    torch.cuda.synchronize()
    out = _c(y1), _c(y)
    ctx.close()
    return out


def test_stages_match_oracle():
    cfg = lofarsim.get_config("c3", n_t=2048, hex_rings=2,
                              k=tuple(range(52, 68)), n_pulses=0)
    blk = lofarsim.generate(cfg)
    group, prelim = _geometry(blk)
    G = int(group.max()) + 1
    o1 = ts.stage1(blk.enu, 2, group, G, blk.k, prelim, blk.x)
    o2 = ts.stage2(blk.enu, group, G, blk.k, prelim, blk.az_el, o1)
    for prec in (lp.LP_FP16_MFMA, lp.LP_FP32):
        print("case two-stage 8 groups x 7 prelim, 19 beams, prec", prec,
              flush=True)
        g1, g2 = _run(blk, group, prelim, prec)
        e1, e2 = _rel(g1, o1), _rel(g2, o2)
        print(f"stage 1 rel-rms {e1:.2e}, stages 1+2 rel-rms {e2:.2e}",
              flush=True)
        assert e1 <= TOL[prec] and e2 <= TOL[prec]


@pytest.mark.parametrize("n_t,G", [(1000, 5), (999, 5), (1000, 9)])
def test_stage2_alone_and_identities(n_t, G):
    """Stage 2 on the oracle's own stage-1 beams (FP32 input), and the exact
    identity: a final beam at a preliminary direction is the sum of the
    groups' beams, i.e. the single-stage beam.  Even n_t takes the kernel
    with two samples per thread, odd n_t one; more than 8 groups take the
    kernel sized for 32."""
    import torch
    cfg = lofarsim.get_config("c3", n_t=n_t, hex_rings=1,
                              k=tuple(range(200, 212)), n_pulses=0)
    blk = lofarsim.generate(cfg, with_noise=True)
    group, prelim = _geometry(blk, G=G)
    P = len(prelim)
    finals = np.concatenate([blk.az_el, prelim[3:5]])
    o1 = ts.stage1(blk.enu, 2, group, G, blk.k, prelim, blk.x)
    o2 = ts.stage2(blk.enu, group, G, blk.k, prelim, finals, o1)
    ctx = lp.Ctx(0)
    y = torch.empty((len(finals), len(blk.k), blk.n_t, 2),
                    dtype=torch.float32, device="cuda:0")
    print(f"case stage2 alone, n_t={n_t} (ragged), {G} groups", flush=True)
    lp.beamform_stage2(ctx, lp.Array(blk.enu, 2), lp.Groups(group, G),
                       lp.Band(blk.k), lp.Dirs(prelim), lp.Dirs(finals),
                       _dev_c(o1), blk.n_t, y)
    torch.cuda.synchronize()
    g2 = _c(y)
    e = _rel(g2, o2)
    print(f"stage 2 rel-rms {e:.2e}", flush=True)
    assert e <= 1e-5
    single = o1.reshape(G, P, len(blk.k), blk.n_t).sum(axis=0)
    for i, p in ((len(blk.az_el), 3), (len(blk.az_el) + 1, 4)):
        assert _rel(g2[i], single[p]) <= 1e-5
    with pytest.raises(lp.LpError):
        lp.beamform_stage2(ctx, lp.Array(blk.enu, 2),
                           lp.Groups(np.zeros_like(group), 2),   # empty group
                           lp.Band(blk.k), lp.Dirs(prelim), lp.Dirs(finals),
                           _dev_c(o1), blk.n_t, y)
    ctx.close()


def test_snr_impact_through_the_chain():
    """The pulses of a C3-like block (61 final beams) through de-dispersion,
    synthesis and trigger with single-stage and with two-stage beams; the
    two-stage beam recovers each pulse with the SNR lost to the stations'
    spread about their group centre (printed), and a pulse in a beam at a
    preliminary direction keeps its single-stage SNR."""
    import torch
    cfg = lofarsim.get_config("c3", n_t=8192, k=tuple(range(52, 116)),
                              snr=(25.0, 25.0))
    blk = lofarsim.generate(cfg)
    group, prelim = _geometry(blk)
    G, P, B = 8, len(prelim), len(blk.az_el)
    pb = ts.nearest_prelim(prelim, blk.az_el)
    off = np.degrees(np.arccos(np.clip(np.sum(
        ts.direction(blk.az_el) * ts.direction(prelim)[pb], 1), -1, 1)))
    res = {}
    for mode in ("single", "two-stage"):
        ctx = lp.Ctx(0)
        p = lp.Pipeline(ctx, lp.Array(blk.enu, 2), lp.Band(blk.k),
                        lp.Dirs(blk.az_el), blk.tec, blk.n_t)
        x = torch.from_numpy(blk.x).to("cuda:0")
        if mode == "single":
            p.beamform(x)
        else:
            y1 = torch.empty((G * P, len(blk.k), blk.n_t, 2),
                             dtype=torch.float32, device="cuda:0")
            lp.beamform_groups(ctx, p.array, lp.Groups(group, G), p.band,
                               lp.Dirs(prelim), x, blk.n_t, y1)
            lp.beamform_stage2(ctx, p.array, lp.Groups(group, G), p.band,
                               lp.Dirs(prelim), p.dirs, y1, blk.n_t,
                               p.y_view())
        p.dedisperse()
        p.synthesize()
        p.trigger()
        torch.cuda.synchronize()
        res[mode] = (p.triggers(), p.bufs["snr"].cpu().numpy().ravel())
        ctx.close()
    for pl in blk.pulses:
        b = int(pl["beam"])
        s1 = res["single"][1][b]
        s2 = res["two-stage"][1][b]
        near = [t for t in res["two-stage"][0]
                if abs(int(t["sample"]) - pl["n0"]) <= 4]
        print(f"pulse in beam {b} ({off[b]:.3f} deg from its preliminary "
              f"beam): peak SNR single {s1:.1f}, two-stage {s2:.1f} "
              f"(ratio {s2 / s1:.3f}); two-stage triggers near it: "
              f"{[(int(t['beam']), round(float(t['snr']), 1)) for t in near]}",
              flush=True)
        assert s2 <= s1 * 1.05
        if off[b] < 1e-6:
            assert abs(s2 / s1 - 1) < 1e-3
