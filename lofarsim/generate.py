"""Seeded generation of one block of station-subband data.

Forward model (the instrument, not the hot path):

* Stations: uniform by area in a disk of the configured diameter, z = 0,
  ENU metres.  Sky direction n(az, el) = (cos el sin az, cos el cos az,
  sin el); a plane wave from n reaches station r at tau = -(r . n) / c
  relative to the array origin.
* Pointing: the Moon at az ~ U[0, 2 pi), el ~ U[25, 65] deg; beams on a
  hexagonal lattice of 0.1 deg spacing in the tangent plane, ring by ring
  (beam 0 is the centre).
* Noise: iid N(0, sigma^2) per real and imaginary part of every
  (subband, sample, station, polarisation).
* Pulse: a one-sample impulse of amplitude A at integer ADC index n0 (at
  the array origin).  Per station, on a 2^17-sample full-rate window
  aligned to the PPF frame, its real spectrum is multiplied by the
  geometric delay exp(-2 pi i f_RF tau) and the ionospheric response
  exp(+2 pi i kappa T / f_RF) (f_RF = f0 + f_baseband, second Nyquist zone
  with the flip undone), limited to the band of the selected subbands,
  transformed back and passed through the station PPF
  y_k[m] = sum_l h[l] e^{+2 pi i k l / M} x[mM - l] (Kaiser(beta)-windowed
  sinc, 16 taps, sum h = 1).  Both polarisations receive the same pulse.
* SNR: per input, the band-limited impulse's analytic-envelope peak
  2 A N_B / N_w over the rms of the same band of the equivalent ADC noise
  (variance 2 sigma^2 / sum h^2 over the full band).
* Quantisation: round half to even, saturate to +-127 (ci8) or +-32767
  (ci16).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
from dataclasses import dataclass

import numpy as np

from .configs import SEED_ROOT, Workload

C_LIGHT = 299792458.0
# First-order ionospheric constant e^2/(8 pi^2 eps0 m_e) (CODATA 2018).
_E, _EPS0, _ME = 1.602176634e-19, 8.8541878128e-12, 9.1093837015e-31
K_ION = _E * _E / (8.0 * np.pi ** 2 * _EPS0 * _ME)       # m^3 s^-2
TECU = 1e16                                                # m^-2

PULSE_WINDOW = 1 << 17


@dataclass
class Block:
    cfg: Workload
    x: np.ndarray          # [n_sb][n_t][n_in][2] int8 / int16
    enu: np.ndarray        # [n_st][3] metres
    az_el: np.ndarray      # [n_beams][2] radians
    k: np.ndarray          # [n_sb] int32
    tec: np.ndarray        # [n_tec] TECU
    pulses: list           # ground truth dicts
    seeds: dict

    @property
    def n_t(self) -> int:
        return self.x.shape[1]


def _children(cfg: Workload, extra=()):
    ss = np.random.SeedSequence([SEED_ROOT, cfg.index, *cfg.seed, *extra])
    names = ["geometry", "pointing", "pulses", "noise"]
    return dict(zip(names, ss.spawn(len(names)))), ss.entropy


def stations_in_disk(rng, n_st: int, diameter: float) -> np.ndarray:
    r = 0.5 * diameter * np.sqrt(rng.uniform(0.0, 1.0, n_st))
    phi = rng.uniform(0.0, 2.0 * np.pi, n_st)
    return np.stack([r * np.sin(phi), r * np.cos(phi), np.zeros(n_st)], 1)


def moon_direction(rng):
    az = rng.uniform(0.0, 2.0 * np.pi)
    el = np.deg2rad(rng.uniform(25.0, 65.0))
    return az, el


def _unit(az, el):
    return np.array([np.cos(el) * np.sin(az), np.cos(el) * np.cos(az),
                     np.sin(el)])


def hex_beams(az0: float, el0: float, rings: int,
              spacing_deg: float = 0.1) -> np.ndarray:
    """Hexagonal lattice of beam centres, ring by ring; [n][2] (az, el)."""
    a = np.deg2rad(spacing_deg)
    pts = [(0, 0)]
    for R in range(1, rings + 1):
        # Walk the ring of hex distance R in axial coordinates.
        dirs = [(1, -1), (0, -1), (-1, 0), (-1, 1), (0, 1), (1, 0)]
        q, r = 0, R
        for dq, dr in dirs:
            for _ in range(R):
                pts.append((q, r))
                q, r = q + dq, r + dr
    n0 = _unit(az0, el0)
    e_az = np.array([np.cos(az0), -np.sin(az0), 0.0])
    e_el = np.array([-np.sin(el0) * np.sin(az0), -np.sin(el0) * np.cos(az0),
                     np.cos(el0)])
    out = []
    for q, r in pts:
        u = a * (q + 0.5 * r)
        v = a * (np.sqrt(3.0) / 2.0 * r)
        n = n0 + u * e_az + v * e_el
        n /= np.linalg.norm(n)
        out.append((np.arctan2(n[0], n[1]) % (2 * np.pi), np.arcsin(n[2])))
    return np.array(out, dtype=np.float64)


def station_groups(enu, n_groups: int, iters: int = 50) -> np.ndarray:
    """Partition stations into n_groups spatially compact groups (Lloyd's
    k-means on the horizontal positions, seeded by farthest-point picks from
    the station nearest the array centre; deterministic).  Returns the group
    index of every station; every group is non-empty."""
    xy = np.asarray(enu, dtype=np.float64)[:, :2]
    n = xy.shape[0]
    if not 1 <= n_groups <= n:
        raise ValueError("need 1 <= n_groups <= n_stations")
    c0 = int(np.argmin(np.sum((xy - xy.mean(0)) ** 2, axis=1)))
    seeds = [c0]
    d = np.sum((xy - xy[c0]) ** 2, axis=1)
    while len(seeds) < n_groups:
        i = int(np.argmax(d))
        seeds.append(i)
        d = np.minimum(d, np.sum((xy - xy[i]) ** 2, axis=1))
    cent = xy[seeds].copy()
    lab = np.zeros(n, dtype=np.int32)
    for _ in range(iters):
        dist = np.sum((xy[:, None, :] - cent[None]) ** 2, axis=2)
        new = np.argmin(dist, axis=1).astype(np.int32)
        for g in range(n_groups):          # keep every group non-empty
            if not np.any(new == g):
                far = int(np.argmax(np.min(dist, axis=1)))
                new[far] = g
        if np.array_equal(new, lab) and _ > 0:
            break
        lab = new
        cent = np.stack([xy[lab == g].mean(0) for g in range(n_groups)])
    return lab


def kaiser_sinc(M: int, P: int, beta: float = 9.0) -> np.ndarray:
    """Station PPF prototype: numpy's Kaiser window times a sinc with its
    cutoff at half a subband, normalised to unit sum."""
    L = M * P
    h = np.kaiser(L, beta) * np.sinc((np.arange(L) - (L - 1) / 2.0) / M)
    return h / h.sum()


def station_ppf(x: np.ndarray, w0: int, h: np.ndarray, M: int,
                m_first: int, n_frames: int) -> np.ndarray:
    """Polyphase analysis of a real window x covering ADC samples
    [w0, w0 + len(x)); returns y[k][i] for k = 0..M-1 and frames
    m = m_first + i, computed as M * ifft of the polyphase sums."""
    L = h.size
    P = L // M
    hp = h.reshape(P, M)
    ext = np.zeros(L + x.size + L)
    ext[L:L + x.size] = x
    out = np.empty((M, n_frames), dtype=np.complex128)
    for i in range(n_frames):
        m = m_first + i
        top = L + m * M - w0            # position of sample m*M in ext
        seg = ext[top - L + 1:top + 1][::-1]   # x[mM - l], l = 0..L-1
        u = (hp * seg.reshape(P, M)).sum(0)
        out[:, i] = M * np.fft.ifft(u)
    return out


def pulse_waveforms(cfg: Workload, enu, src_dir, n0: int, amp: float,
                    tec: float):
    """5 ns waveform of one pulse at every station: (w0, xs) with xs[st][j]
    the real ADC-domain signal at absolute sample w0 + j (PULSE_WINDOW
    samples).  An impulse at ADC sample n0 at the array origin, arriving
    (r . n) / c earlier at station r, dispersed by the ionosphere
    (exp(+2 pi i kappa T / f_RF)), band-limited to the selected subbands;
    baseband frequency f_b maps to f_RF = f0 + f_b."""
    M, fs, f0 = cfg.M, cfg.fs, cfg.f0
    Nw = PULSE_WINDOW
    frame = n0 // M
    w0 = (frame - Nw // (2 * M)) * M
    nb = np.arange(Nw // 2 + 1)
    fb = nb * fs / Nw
    kmin, kmax = min(cfg.k), max(cfg.k)
    df = fs / M
    band = (fb >= (kmin - 0.5) * df) & (fb <= (kmax + 0.5) * df)
    f_rf = f0 + fb
    base = amp * np.exp(-2j * np.pi * nb * (n0 - w0) / Nw)
    iono = np.exp(2j * np.pi * (K_ION * tec * TECU / C_LIGHT) / f_rf)
    nvec = _unit(*src_dir)
    xs = np.empty((enu.shape[0], Nw))
    for st in range(enu.shape[0]):
        tau = -(enu[st] @ nvec) / C_LIGHT
        spec = np.where(band, base * iono * np.exp(-2j * np.pi * f_rf * tau),
                        0.0)
        xs[st] = np.fft.irfft(spec, n=Nw)
    return w0, xs


def _pulse_subbands(cfg: Workload, enu, src_dir, n0: int, amp: float,
                    tec: float, h: np.ndarray):
    """Per-station subband contribution of one pulse: (m_first, y) with
    y[st][s][i] complex for frames m_first + i."""
    M = cfg.M
    Nw = PULSE_WINDOW
    w0, xs = pulse_waveforms(cfg, enu, src_dir, n0, amp, tec)
    m_first = w0 // M
    n_frames = Nw // M + h.size // M
    ks = np.asarray(cfg.k)
    y = np.empty((enu.shape[0], ks.size, n_frames), dtype=np.complex128)
    for st in range(enu.shape[0]):
        y[st] = station_ppf(xs[st], w0, h, M, m_first, n_frames)[ks]
    fb = np.arange(Nw // 2 + 1) * cfg.fs / Nw
    df = cfg.fs / M
    n_band = int(((fb >= (min(cfg.k) - 0.5) * df) &
                  (fb <= (max(cfg.k) + 0.5) * df)).sum())
    return m_first, y, n_band


def pulse_amplitude(cfg: Workload, snr: float, h: np.ndarray) -> float:
    Nw = PULSE_WINDOW
    df = cfg.fs / cfg.M
    fb = np.arange(Nw // 2 + 1) * cfg.fs / Nw
    kmin, kmax = min(cfg.k), max(cfg.k)
    n_band = int(((fb >= (kmin - 0.5) * df) & (fb <= (kmax + 0.5) * df)).sum())
    var_adc = 2.0 * cfg.sigma ** 2 / float(np.sum(h * h))
    sigma_bl = np.sqrt(var_adc * n_band / (Nw / 2.0))
    return snr * sigma_bl * Nw / (2.0 * n_band)


def generate(cfg: Workload, with_noise: bool = True,
             with_pulses: bool = True, beta: float = 9.0) -> Block:
    ch, entropy = _children(cfg)
    g_rng = np.random.default_rng(ch["geometry"])
    p_rng = np.random.default_rng(ch["pointing"])
    u_rng = np.random.default_rng(ch["pulses"])
    M, n_t = cfg.M, cfg.n_t
    enu = stations_in_disk(g_rng, cfg.n_st, cfg.disk_m)
    az0, el0 = moon_direction(p_rng)
    az_el = hex_beams(az0, el0, cfg.hex_rings)
    k = np.asarray(cfg.k, dtype=np.int32)
    tec = np.asarray(cfg.tec, dtype=np.float64)
    h = kaiser_sinc(M, 16, beta)

    # Pulse times: frames in [P + 16, n_t - D - 16], at least 64 frames
    # apart; sources at the centres of `pulse_beams` distinct beams.
    pulses = []
    if with_pulses and cfg.n_pulses > 0:
        lo, hi = 32, n_t - 1024 - 16
        src_beams = u_rng.choice(cfg.n_beams, size=cfg.pulse_beams,
                                 replace=False)
        frames = []
        while len(frames) < cfg.n_pulses:
            f = int(u_rng.integers(lo, hi + 1))
            if all(abs(f - g) >= 64 for g in frames):
                frames.append(f)
        frames.sort()
        for i, f in enumerate(frames):
            n0 = f * M + int(u_rng.integers(0, M))
            snr = float(u_rng.uniform(*cfg.snr))
            b = int(src_beams[i % cfg.pulse_beams])
            amp = pulse_amplitude(cfg, snr, h)
            pulses.append(dict(n0=n0, beam=b, snr=snr, amp=amp,
                               tec=float(cfg.true_tec),
                               tec_index=cfg.true_tec_index))

    contrib = []
    for p in pulses:
        m_first, y, _ = _pulse_subbands(cfg, enu, tuple(az_el[p["beam"]]),
                                        p["n0"], p["amp"], p["tec"], h)
        contrib.append((m_first, y))

    itype = np.int8 if cfg.dtype == "ci8" else np.int16
    lim = 127 if cfg.dtype == "ci8" else 32767
    x = np.empty((cfg.n_sb, n_t, cfg.n_in, 2), dtype=itype)
    # One noise generator per subband (spawned from the noise seed), so the
    # bytes do not depend on how many threads fill the block.
    sb_seeds = ch["noise"].spawn(cfg.n_sb)

    def fill(s):
        if with_noise:
            rng = np.random.default_rng(sb_seeds[s])
            v = rng.standard_normal((n_t, cfg.n_in, 2), dtype=np.float32)
            v *= np.float32(cfg.sigma)
        else:
            v = np.zeros((n_t, cfg.n_in, 2), dtype=np.float32)
        for m_first, y in contrib:
            a, b = max(m_first, 0), min(m_first + y.shape[2], n_t)
            if a >= b:
                continue
            seg = y[:, s, a - m_first:b - m_first]           # [st][frames]
            seg = np.repeat(seg.T, cfg.n_pol, axis=1)        # [frames][in]
            v[a:b, :, 0] += seg.real.astype(np.float32)
            v[a:b, :, 1] += seg.imag.astype(np.float32)
        np.rint(v, out=v)
        np.clip(v, -lim, lim, out=v)
        x[s] = v.astype(itype)

    workers = max(1, min(16, os.cpu_count() or 1))
    if cfg.n_sb * n_t * cfg.n_in < (1 << 22) or workers == 1:
        for s in range(cfg.n_sb):
            fill(s)
    else:
        with cf.ThreadPoolExecutor(workers) as ex:
            list(ex.map(fill, range(cfg.n_sb)))
    return Block(cfg=cfg, x=x, enu=enu, az_el=az_el, k=k, tec=tec,
                 pulses=pulses, seeds=dict(entropy=int(entropy) if
                                          isinstance(entropy, int) else
                                          str(entropy), root=SEED_ROOT,
                                          index=cfg.index))
