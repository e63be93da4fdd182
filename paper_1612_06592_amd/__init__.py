"""MI355X (gfx950) hot path of the LOFAR lunar ns-pulse pipeline.

Winchen et al., "Realtime processing of LOFAR data for the detection of
nano-second pulses from the Moon", arXiv:1612.06592: beamforming toward the
Moon, ionospheric de-dispersion over trial STEC values, synthesis of the
5 ns time series from the polyphase-filtered subbands, and an envelope
trigger -- as hand-written HIP kernels behind the C ABI in include/lp.h.
"""
__all__ = ["lp", "build"]
