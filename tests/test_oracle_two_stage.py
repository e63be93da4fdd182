"""Pins of the oracle's two-stage beamformer (oracle/two_stage.py; the
paper's two-step beam formation of Sec. 4).

  * one station per group: the two-stage beam equals the single-stage beam
    towards every final direction (the group centre is the station);
  * final directions equal to preliminary ones: the two-stage beam equals
    the single-stage beam for any grouping (all coefficients are 1);
  * a plane wave: the two-stage response of every final beam equals the
    coherent sum over stations of exp(2 pi i f (r_st - r_g) . (n_b - n_p)
    / c), written from the geometry rather than from the weights;
  * stage 1 of all groups sums to the single-stage beam (the groups
    partition the stations);
  * the nearest preliminary direction of a preliminary direction is itself.
"""
import numpy as np

import lofarsim
import oracle
from oracle import two_stage as ts

C = 299792458.0


def _setup(n_st=12, n_sb=3, n_t=64, rings=2, seed=1):
    rng = np.random.default_rng(seed)
    enu = lofarsim.stations_in_disk(rng, n_st, 800.0)
    k = np.arange(120, 120 + n_sb)
    az0, el0 = 1.1, 0.7
    prelim = lofarsim.hex_beams(az0, el0, 1, spacing_deg=0.2)     # 7
    beams = lofarsim.hex_beams(az0, el0, rings, spacing_deg=0.1)  # 19
    x = rng.standard_normal((n_sb, n_t, 2 * n_st, 2))
    return rng, enu, k, prelim, beams, x


def _rel(a, b):
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))


def test_singleton_groups_equal_single_stage():
    rng, enu, k, prelim, beams, x = _setup()
    n_st = enu.shape[0]
    group = np.arange(n_st)
    y1 = ts.stage1(enu, 2, group, n_st, k, prelim[:1], x)
    y = ts.stage2(enu, group, n_st, k, prelim[:1], beams, y1)
    ref = oracle.beamform(enu, 2, k, beams, x)
    assert _rel(y, ref) < 1e-12


def test_final_equal_prelim_any_grouping():
    rng, enu, k, prelim, beams, x = _setup(seed=2)
    group = lofarsim.station_groups(enu, 4)
    y1 = ts.stage1(enu, 2, group, 4, k, prelim, x)
    y = ts.stage2(enu, group, 4, k, prelim, prelim, y1)
    ref = oracle.beamform(enu, 2, k, prelim, x)
    assert _rel(y, ref) < 1e-12
    assert np.array_equal(ts.nearest_prelim(prelim, prelim), np.arange(7))


def test_stage1_groups_sum_to_single_stage():
    rng, enu, k, prelim, beams, x = _setup(seed=3)
    group = lofarsim.station_groups(enu, 3)
    y1 = ts.stage1(enu, 2, group, 3, k, prelim, x).reshape(3, 7, 3, -1)
    ref = oracle.beamform(enu, 2, k, prelim, x)
    assert _rel(y1.sum(axis=0), ref) < 1e-12


def test_plane_wave_response_matches_geometry():
    rng, enu, k, prelim, beams, _ = _setup(seed=4, n_t=4)
    n_st, G = enu.shape[0], 4
    group = lofarsim.station_groups(enu, G)
    rg = np.stack([enu[group == g].mean(0) for g in range(G)])
    f = 100e6 + k * 200e6 / 1024
    nb = ts.direction(beams)
    npre = ts.direction(prelim)
    pb = ts.nearest_prelim(prelim, beams)
    for b in (0, 5, 12):
        # Unit plane wave from final direction b on every input.
        ph = np.exp(2j * np.pi * f[:, None] * (enu @ nb[b])[None, :] / C)
        x = np.zeros((len(k), 4, 2 * n_st, 2))
        xc = np.repeat(ph, 2, axis=1)                 # both pols
        x[..., 0] = xc.real[:, None, :]
        x[..., 1] = xc.imag[:, None, :]
        y1 = ts.stage1(enu, 2, group, G, k, prelim, x)
        y = ts.stage2(enu, group, G, k, prelim, beams, y1)
        d = nb[b] - npre[pb[b]]
        off = enu - rg[group]                          # r_st - r_g
        ref = 2 * np.exp(2j * np.pi * f[:, None] * (off @ d)[None, :] / C
                         ).sum(axis=1)
        assert np.abs(y[b, :, 0] - ref).max() < 1e-9 * 2 * n_st
        assert np.abs(y[b, :, 3] - ref).max() < 1e-9 * 2 * n_st
        # The coherent single-stage response is 2 n_st; two-stage is not
        # larger.
        assert np.all(np.abs(ref) <= 2 * n_st * (1 + 1e-12))
