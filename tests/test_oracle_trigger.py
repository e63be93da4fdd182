"""Pins for the oracle's envelope statistics and trigger rules on
hand-built inputs, and end-to-end on generated blocks (the generator's
forward model is independent of the oracle):

* ties keep the lowest index; the threshold is strict; runs of fired
  windows give one trigger at the run's maximum; triggers of different
  trials within one window merge, keeping the best SNR;
* warm-up frames of a stream's first block neither fire nor enter sigma;
* C1: the injected impulse is found at n0 +- 1 in beam 0 with SNR >> 6;
* a TEC grid recovers the injected grid index as best trial;
* several beams: the highest-SNR trigger of each pulse is in its beam.
"""
import numpy as np

import lofarsim

M, P, D = 1024, 16, 1024
OFF = M * P + D * M


def test_detect_sigma_ties_and_warmup(oracle_lib):
    n_t = 4
    z = np.zeros((1, n_t * M), complex)
    z[0, :] = 0.5                      # x = 2 Re z = 1, e = 1 everywhere
    z[0, 2 * M + 7] = 3.0              # tie at two places in frame 2
    z[0, 2 * M + 9] = 3.0j
    z[0, 0 * M + 3] = 10.0             # in a warm-up frame
    sigma, wmax, warg = oracle_lib.detect(z, n_t, frame0=D + P - 1, warm=D + P)
    # Frame 0 is warm-up; sigma over frames 1..3.
    xr = 2 * z.real[0, M:]
    assert abs(sigma[0] - np.sqrt(np.mean(xr ** 2))) < 1e-14
    assert wmax[0, 2] == 6.0 and warg[0, 2] == 2 * M + 7
    assert wmax[0, 1] == 1.0 and warg[0, 1] == M      # all equal -> first


def _trig(sigma, wmax, warg, B, J, n_t, frame0=10_000, k=6.0):
    return oracle_lib_trigger(sigma, wmax, warg, B, J, n_t, frame0, k)


def oracle_lib_trigger(sigma, wmax, warg, B, J, n_t, frame0, k):
    import oracle
    return oracle.trigger(np.asarray(sigma, float), np.asarray(wmax, float),
                          np.asarray(warg, np.int64), B, J, n_t, frame0,
                          D + P, k)


def test_trigger_runs_threshold_and_merge(oracle_lib):
    n_t = 12
    sig = [1.0, 1.0]
    wm = np.ones((2, n_t))
    wa = np.arange(n_t)[None, :] * M + np.array([[5], [6]])
    wm[0, 2] = 6.0                     # exactly 6 sigma: does not fire
    wm[0, 4], wm[0, 5], wm[0, 6] = 7.0, 9.0, 9.0   # one run, max at 5 (first)
    wm[0, 9] = 8.0                     # second run
    wm[1, 5] = 9.5                     # trial 1 near trial 0's pulse
    wm[1, 11] = 6.5
    trig, snr, best = _trig(sig, wm, wa, 1, 2, n_t)
    f0 = 10_000
    samples = [t["sample"] for t in trig]
    assert samples == [f0 * M + 5 * M + 6 - OFF, f0 * M + 9 * M + 5 - OFF,
                       f0 * M + 11 * M + 6 - OFF]
    assert [int(t["tec"]) for t in trig] == [1, 0, 1]
    assert trig[0]["snr"] == 9.5
    assert best[0] == 1 and snr[0, 0] == 9.0 and snr[0, 1] == 9.5


def test_trigger_merge_ties_prefer_lowest_trial(oracle_lib):
    n_t = 4
    wm = np.ones((3, n_t))
    wa = np.arange(n_t)[None, :] * M + np.array([[100], [200], [50]])
    wm[:, 2] = 8.0                     # all trials equal at frame 2
    trig, snr, best = _trig([1, 1, 1], wm, wa, 1, 3, n_t)
    assert len(trig) == 1 and int(trig[0]["tec"]) == 0
    assert best[0] == 0


def test_trigger_sigma_zero_and_warmup_never_fire(oracle_lib):
    n_t = 4
    wm = np.full((1, n_t), 100.0)
    wa = np.zeros((1, n_t), np.int64)
    trig, snr, _ = _trig([0.0], wm, wa, 1, 1, n_t)
    assert len(trig) == 0 and snr[0, 0] == 0.0
    import oracle
    trig, _, _ = oracle.trigger(np.array([1.0]), wm, wa, 1, 1, n_t,
                                frame0=0, warm=D + P)
    assert len(trig) == 0


def test_end_to_end_c1_pulse_found(oracle_lib):
    blk = lofarsim.generate(lofarsim.get_config("c1"))
    st = oracle_lib.Stream(blk.enu, 2, blk.k, blk.az_el, blk.tec)
    r = st.process(blk.x)
    assert len(r.triggers) == 1
    t = r.triggers[0]
    assert abs(int(t["sample"]) - blk.pulses[0]["n0"]) <= 1
    assert int(t["beam"]) == 0 and t["snr"] > 15


def test_end_to_end_tec_grid_best_trial(oracle_lib):
    tec = tuple(np.linspace(0, 30, 7).tolist())
    cfg = lofarsim.get_config("c4", n_t=4096, k=tuple(range(52, 116)),
                              hex_rings=0, tec=tec, true_tec_index=4,
                              true_tec=tec[4], n_pulses=1, snr=(12.0, 12.0))
    blk = lofarsim.generate(cfg)
    st = oracle_lib.Stream(blk.enu, 2, blk.k, blk.az_el, blk.tec)
    r = st.process(blk.x)
    assert r.best_tec[0] == 4
    assert np.argmax(r.snr_peak[0]) == 4
    hit = [t for t in r.triggers if abs(int(t["sample"]) - blk.pulses[0]["n0"]) <= 2]
    assert len(hit) == 1 and int(hit[0]["tec"]) == 4


def test_end_to_end_multibeam_highest_snr_in_source_beam(oracle_lib):
    cfg = lofarsim.get_config("c3", n_st=12, n_t=4096, hex_rings=1,
                              k=tuple(range(52, 100)), n_pulses=2,
                              pulse_beams=2)
    blk = lofarsim.generate(cfg)
    st = oracle_lib.Stream(blk.enu, 2, blk.k, blk.az_el, blk.tec)
    r = st.process(blk.x)
    for p in blk.pulses:
        near = [t for t in r.triggers if abs(int(t["sample"]) - p["n0"]) <= 4]
        assert near, p
        best = max(near, key=lambda t: t["snr"])
        assert int(best["beam"]) == p["beam"]
