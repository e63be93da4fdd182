"""The five synthetic workloads (tiny correctness block, single-beam core,
61-beam lunar tiling, 32-trial TEC grid, multi-stream serving).

Shapes follow the paper's instrument (Winchen et al., arXiv:1612.06592,
Sec. 2): 200 MHz real sampling, 1024-point critically sampled station PPF
(195.3125 kHz subbands, 5.12 us), HBA band 110-190 MHz, up to 24 core
stations x 2 polarisations in a ~2 km core; ~50-61 beams to tile the Moon
(Sec. 4); STEC trials (Sec. 3).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

SEED_ROOT = 161206592


@dataclass(frozen=True)
class Workload:
    name: str
    index: int
    n_st: int
    disk_m: float                     # diameter of the station disk
    k: tuple                          # subband ids (ascending, 1..511)
    n_t: int                          # subband samples per block
    hex_rings: int                    # 0 -> 1 beam, R -> 1 + 3R(R+1) beams
    tec: tuple                        # trial STEC values (TECU)
    true_tec_index: int | None        # index into tec of the pulses' STEC
    true_tec: float                   # STEC of the pulses (TECU)
    dtype: str                        # "ci8" or "ci16"
    sigma: float                      # noise rms per real component
    n_pulses: int
    snr: tuple                        # (lo, hi) per-input SNR, uniform
    pulse_beams: int = 1              # number of distinct source beams
    n_pol: int = 2
    f0: float = 100e6
    fs: float = 200e6
    M: int = 1024
    seed: tuple = field(default=())

    @property
    def n_in(self) -> int:
        return self.n_st * self.n_pol

    @property
    def n_beams(self) -> int:
        R = self.hex_rings
        return 1 + 3 * R * (R + 1)

    @property
    def n_sb(self) -> int:
        return len(self.k)

    @property
    def n_tec(self) -> int:
        return len(self.tec)

    @property
    def block_seconds(self) -> float:
        return self.n_t * self.M / self.fs

    @property
    def station_beam_samples(self) -> int:
        """Complex subband samples of one input contributing to one beam
        (the unit of the paper's 8*N_S FLOP per sample, Sec. 3)."""
        return self.n_in * self.n_sb * self.n_t * self.n_beams

    def sliced(self, **kw) -> "Workload":
        """A smaller block with the same per-sample structure."""
        return replace(self, **kw)


def _band(k0: int, n: int) -> tuple:
    return tuple(range(k0, k0 + n))


CONFIGS = {
    # Plain FP32 pipeline, tiny: 4 stations x 2 pol, 32 subbands centred on
    # ~140 MHz, 4096 ci16 samples, one impulse of SNR 8 at 5 TECU.
    "c1": Workload("c1-tiny", 0, n_st=4, disk_m=300.0, k=_band(189, 32),
                   n_t=4096, hex_rings=0, tec=(5.0,), true_tec_index=0,
                   true_tec=5.0, dtype="ci16", sigma=16.0, n_pulses=1,
                   snr=(8.0, 8.0)),
    # Single beam, LOFAR-core scale: 24 stations, 244 subbands spanning
    # 110.06-157.71 MHz, 65536 ci8 samples, 3 pulses SNR 6-15, 10 TECU.
    "c2": Workload("c2-core-1beam", 1, n_st=24, disk_m=2000.0,
                   k=_band(52, 244), n_t=65536, hex_rings=0, tec=(10.0,),
                   true_tec_index=0, true_tec=10.0, dtype="ci8", sigma=8.0,
                   n_pulses=3, snr=(6.0, 15.0)),
    # Multi-beam tiling of the lunar disk: 48 stations, 61 hexagonal beams at
    # 0.1 deg spacing, 32768 samples; pulses from the centres of 2 beams.
    "c3": Workload("c3-61beam", 2, n_st=48, disk_m=2000.0, k=_band(52, 244),
                   n_t=32768, hex_rings=4, tec=(10.0,), true_tec_index=0,
                   true_tec=10.0, dtype="ci8", sigma=8.0, n_pulses=2,
                   snr=(6.0, 15.0), pulse_beams=2),
    # TEC trial grid: 24 stations, 7 beams, 32 trials uniform in 0-30 TECU,
    # pulses at a true TEC on the grid (index seeded in 1..30).
    "c4": Workload("c4-tec32", 3, n_st=24, disk_m=2000.0, k=_band(52, 244),
                   n_t=65536, hex_rings=1,
                   tec=tuple(np.linspace(0.0, 30.0, 32).tolist()),
                   true_tec_index=None, true_tec=float("nan"), dtype="ci8",
                   sigma=8.0, n_pulses=2, snr=(10.0, 10.0)),
}


def get_config(name: str, **overrides) -> Workload:
    cfg = CONFIGS[name]
    if cfg.true_tec_index is None and "true_tec_index" not in overrides:
        rng = np.random.default_rng(
            np.random.SeedSequence([SEED_ROOT, cfg.index, 7]))
        idx = int(rng.integers(1, 31))
        cfg = replace(cfg, true_tec_index=idx, true_tec=cfg.tec[idx])
    if overrides:
        cfg = replace(cfg, **overrides)
        if "tec" in overrides and "true_tec" not in overrides:
            cfg = replace(cfg, true_tec=cfg.tec[cfg.true_tec_index or 0])
    return cfg


def serving_streams(n_streams: int = 12, seed: int = 5, max_log2_nt: int = 18,
                    max_sb: int = 488, max_beams: int = 61):
    """Stream shapes of the serving workload: 24-48 stations x 2 pol, 7-61
    beams, 122-488 contiguous subbands, block lengths 2^12..2^max_log2_nt.

    Subbands start at k = 52 when they fit below 512, else end at 511."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 4, seed]))
    out = []
    beams_choices = [b for b in (7, 19, 37, 61) if b <= max_beams]
    for i in range(n_streams):
        n_st = int(rng.integers(6, 13)) * 4           # 24..48, multiple of 4
        n_beams = int(rng.choice(beams_choices))
        n_sb = int(rng.integers(1, max_sb // 122 + 1)) * 122
        k0 = min(52, 512 - n_sb)
        tec = float(rng.uniform(0.0, 30.0))
        out.append(dict(stream=i, n_st=n_st, n_beams=n_beams,
                        k=tuple(range(k0, k0 + n_sb)), tec=tec,
                        seed=int(rng.integers(0, 2**31)),
                        log2_nt=(12, max_log2_nt)))
    return out
