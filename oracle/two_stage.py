"""Oracle (test infrastructure only; never on the product path): two-stage
beamforming, in plain numpy FP64 on top of the oracle's direct-sum
beamformer.

Winchen et al., Sec. 4 (network paragraph): when the link between the
station-side cluster and the processing cluster cannot carry every
station, preliminary beams are formed on the station side, each from a
subset of the stations, and the final beams are formed from those on the
processing side.  The paper leaves the details open; the reading here:

Stage 1 (station side).  Stations are partitioned into G groups.  For every
group g and preliminary direction p, the regular beam over the group's
stations only (both polarisations):
    y1[g P + p][s][t] = sum_{st in g, pol} w(st, pol, s, n_p) x[s][t][st][pol]
with the single-stage weight w = exp(-2 pi i frac(f_s (r_st . n) / c)).

Stage 2 (processing side).  Final beam b uses, from every group, the
preliminary beam nearest to its direction (p(b): largest n_p . n_b, lowest
p on ties) and re-phases it by the group's phase centre r_g (the mean
station position of the group):
    y[b][s][t] = sum_g exp(-2 pi i frac(f_s (r_g . (n_b - n_p(b))) / c))
                 y1[g P + p(b)][s][t].
With one station per group this is exactly the single-stage beam towards
n_b; with n_b = n_p it is exactly the single-stage beam towards n_p.  In
between, the stations' offsets from their group centre decorrelate the
sum (the beam-shape and SNR effect the paper leaves open).
"""
from __future__ import annotations

import numpy as np

import oracle

C_LIGHT = 299792458.0


def direction(az_el) -> np.ndarray:
    """Unit vectors (east, north, up) of [n][2] (az, el) in radians."""
    a = np.asarray(az_el, dtype=np.float64).reshape(-1, 2)
    az, el = a[:, 0], a[:, 1]
    return np.stack([np.cos(el) * np.sin(az), np.cos(el) * np.cos(az),
                     np.sin(el)], axis=1)


def nearest_prelim(prelim, beams) -> np.ndarray:
    """p(b): index of the preliminary direction with the largest cosine to
    each final direction (lowest index on ties)."""
    cos = direction(beams) @ direction(prelim).T
    return np.argmax(cos, axis=1)


def group_centres(enu, group, n_groups) -> np.ndarray:
    enu = np.asarray(enu, dtype=np.float64)
    group = np.asarray(group)
    return np.stack([enu[group == g].mean(axis=0) for g in range(n_groups)])


def stage1(enu, n_pol, group, n_groups, k, prelim, x, f0=100e6, fs=200e6,
           M=1024) -> np.ndarray:
    """y1 [G * P][n_sb][n_t]: the regular beam of each group's stations."""
    group = np.asarray(group)
    P = np.asarray(prelim).reshape(-1, 2).shape[0]
    out = []
    for g in range(n_groups):
        gain = np.repeat((group == g).astype(np.float64), n_pol)
        out.append(oracle.beamform(enu, n_pol, k, prelim, x, f0, fs, M,
                                   gain=gain))
    y1 = np.stack(out)                      # [G][P][n_sb][n_t]
    return y1.reshape(n_groups * P, *y1.shape[2:])


def stage2_coefficients(enu, group, n_groups, k, prelim, beams, f0=100e6,
                        fs=200e6, M=1024):
    """(p(b) [B], c [n_sb][B][G] complex) of the definition above."""
    rg = group_centres(enu, group, n_groups)
    nb = direction(beams)
    npre = direction(prelim)
    pb = nearest_prelim(prelim, beams)
    f = f0 + np.asarray(k, dtype=np.float64) * fs / M          # [S]
    proj = (rg @ (nb - npre[pb]).T).T                           # [B][G]
    cyc = f[:, None, None] * proj[None, :, :] / C_LIGHT         # [S][B][G]
    fr = cyc - np.floor(cyc)
    return pb, np.exp(-2j * np.pi * fr)


def stage2(enu, group, n_groups, k, prelim, beams, y1, f0=100e6, fs=200e6,
           M=1024) -> np.ndarray:
    """y [B][n_sb][n_t] from y1 [G * P][n_sb][n_t]."""
    P = np.asarray(prelim).reshape(-1, 2).shape[0]
    pb, c = stage2_coefficients(enu, group, n_groups, k, prelim, beams, f0,
                                fs, M)
    B = len(pb)
    y1 = np.asarray(y1).reshape(n_groups, P, y1.shape[1], y1.shape[2])
    y = np.zeros((B, y1.shape[2], y1.shape[3]), dtype=np.complex128)
    for b in range(B):
        for g in range(n_groups):
            y[b] += c[:, b, g][:, None] * y1[g, pb[b]]
    return y
