"""Seeded synthetic LOFAR HBA station-subband data.

This package is the forward model of the instrument upstream of the hot
path: station positions, beam pointings on the lunar disk, receiver noise,
and broadband ns pulses that travel through the ionosphere and the station
polyphase filterbank (Winchen et al., arXiv:1612.06592, Sec. 2: 5 ns ADC
sampling, station PPF into ~5 us subbands; Sec. 5: the simulated-PPF and
simulated-beamformer modules of the paper's framework).

It holds none of the hot path's arithmetic (no beamformer, de-dispersion
filter, synthesis filterbank or trigger) and shares no code with either the
GPU library or the oracle: both consume its output.  Everything is seeded
from ``numpy.random.SeedSequence``.
"""
from .configs import CONFIGS, Workload, get_config, serving_streams  # noqa
from .generate import (Block, generate, hex_beams, kaiser_sinc,  # noqa
                       pulse_waveforms, station_groups, station_ppf,
                       stations_in_disk, moon_direction)
