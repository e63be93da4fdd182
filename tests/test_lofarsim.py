"""Generator checks: seeds reproduce bytes, noise level, hexagonal beam
counts and spacing, quantisation limits, and the closed-form pulse SNR."""
import numpy as np

import lofarsim
from lofarsim.generate import _unit


def test_seeds_reproduce_bytes():
    cfg = lofarsim.get_config("c1")
    a = lofarsim.generate(cfg)
    b = lofarsim.generate(cfg)
    assert np.array_equal(a.x, b.x)
    assert np.array_equal(a.enu, b.enu) and a.pulses == b.pulses
    c = lofarsim.generate(lofarsim.get_config("c2", n_t=2048,
                                              k=tuple(range(52, 60))))
    assert not np.array_equal(a.enu[:4], c.enu[:4])


def test_noise_sigma_and_quantisation():
    cfg = lofarsim.get_config("c2", n_t=4096, k=tuple(range(52, 68)))
    blk = lofarsim.generate(cfg, with_pulses=False)
    assert blk.x.dtype == np.int8
    s = blk.x.astype(np.float64).std()
    assert abs(s - np.sqrt(64 + 1 / 12)) < 0.05
    assert blk.x.max() <= 127 and blk.x.min() >= -127


def test_hex_beam_counts_and_spacing():
    for R, n in [(0, 1), (1, 7), (2, 19), (3, 37), (4, 61)]:
        b = lofarsim.hex_beams(1.0, 0.8, R)
        assert b.shape == (n, 2)
    b = lofarsim.hex_beams(1.0, 0.8, 1)
    c = _unit(*b[0])
    ang = [np.degrees(np.arccos(np.clip(_unit(*x) @ c, -1, 1))) for x in b[1:]]
    assert np.allclose(ang, 0.1, rtol=1e-3)
    assert np.allclose(b[0], (1.0, 0.8))


def test_stations_inside_disk():
    rng = np.random.default_rng(0)
    enu = lofarsim.stations_in_disk(rng, 1000, 2000.0)
    r = np.hypot(enu[:, 0], enu[:, 1])
    assert r.max() <= 1000.0 and r.mean() > 600


def test_c4_true_tec_on_grid():
    cfg = lofarsim.get_config("c4")
    assert 1 <= cfg.true_tec_index <= 30
    assert cfg.true_tec == cfg.tec[cfg.true_tec_index]
    assert len(cfg.tec) == 32 and cfg.tec[-1] == 30.0


def test_serving_stream_shapes():
    ss = lofarsim.serving_streams()
    assert len(ss) == 12
    for s in ss:
        assert 24 <= s["n_st"] <= 48 and s["n_beams"] in (7, 19, 37, 61)
        assert min(s["k"]) >= 1 and max(s["k"]) <= 511


def test_station_groups_partition():
    """Every station in exactly one of n non-empty groups, deterministic,
    and groups are compact: each station is nearer its own group centre
    than any other centre (the k-means fixed point)."""
    import numpy as np
    rng = np.random.default_rng(5)
    enu = lofarsim.stations_in_disk(rng, 48, 2000.0)
    a = lofarsim.station_groups(enu, 8)
    b = lofarsim.station_groups(enu.copy(), 8)
    assert np.array_equal(a, b)
    assert a.shape == (48,) and set(a.tolist()) == set(range(8))
    cent = np.stack([enu[a == g, :2].mean(0) for g in range(8)])
    d = np.sum((enu[:, None, :2] - cent[None]) ** 2, axis=2)
    assert np.array_equal(np.argmin(d, axis=1), a)
    one = lofarsim.station_groups(enu, 48)
    assert sorted(one.tolist()) == list(range(48))
