"""Per-input gains through the beamformer against the oracle's direct beam
sums with the same gains (paper Sec. 3: a complex weight per station and
beam; the gain is the real amplitude factor of that weight).

On the FP16-MFMA path each input's weights are divided by 2^e (e = ceil
log2 |gain|) and its samples multiplied by 2^e at conversion; int16
samples keep factors above 1 in the weights.  The gains span 2^-14 .. 2^8,
so each input is checked on its own (one-hot inputs: the output is that
input's weighted samples alone) as well as all together.
"""
import numpy as np
import pytest

import lofarsim
import oracle
from chain import PER_ELEM, as_complex, max_err, rel_rms
from paper_1612_06592_amd import lp

pytestmark = pytest.mark.gpu

TOL = {lp.LP_FP16_MFMA: 1e-3, lp.LP_FP32: 1e-5}


def gains_spanning(n_in, rng):
    """Magnitudes 2^k * u, u in (0.5, 1] (so ceil(log2) = k) for k from -14
    to 8, mixed signs, one input at gain 0."""
    ks = np.linspace(-14, 8, n_in - 1).round().astype(int)
    u = rng.uniform(0.51, 1.0, n_in - 1)
    g = np.ldexp(u, ks) * rng.choice([-1.0, 1.0], n_in - 1)
    g = np.concatenate([g, [0.0]]).astype(np.float32)
    e = np.ceil(np.log2(np.abs(g[:-1]).astype(np.float64)))
    assert e.min() == -14 and e.max() == 8
    return g


def block(dtype, rng, n_st=8, n_sb=6, n_t=256):
    cfg = lofarsim.get_config("c1", n_st=n_st, hex_rings=1, n_t=n_t,
                              k=tuple(range(200, 200 + n_sb)), n_pulses=0)
    blk = lofarsim.generate(cfg)
    n_in = 2 * n_st
    if dtype == lp.LP_CI8:
        x = rng.integers(-127, 128, (n_sb, n_t, n_in, 2)).astype(np.int8)
    else:
        # mostly noise, some samples at the int16 extremes (their FP16
        # conversion rounds, and scaling them up would overflow FP16)
        x = np.clip(rng.normal(0, 300, (n_sb, n_t, n_in, 2)), -32767,
                    32767).astype(np.int16)
        hot = rng.random(x.shape) < 0.01
        x[hot] = rng.choice([-32767, 32767], hot.sum()).astype(np.int16)
    return blk, x


def gpu_beams(blk, x, gain, dtype, prec):
    import torch
    ctx = lp.Ctx(0)
    try:
        S, n_t = x.shape[0], x.shape[1]
        B = blk.az_el.shape[0]
        y = torch.empty(lp.nbytes("lp_beam_bytes", B, S, n_t),
                        dtype=torch.uint8, device="cuda:0")
        lp.beamform(ctx, lp.Array(blk.enu, 2, gain=gain), lp.Band(blk.k),
                    lp.Dirs(blk.az_el),
                    torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0"),
                    n_t, dtype, prec, y)
        torch.cuda.synchronize()
        return as_complex(y.view(torch.float32).view(B, S, n_t, 2))
    finally:
        ctx.close()


@pytest.mark.parametrize("dtype", [lp.LP_CI8, lp.LP_CI16])
@pytest.mark.parametrize("prec", [lp.LP_FP16_MFMA, lp.LP_FP32])
def test_gains_against_oracle(dtype, prec):
    rng = np.random.default_rng([1612, 6592, dtype, prec])
    blk, x = block(dtype, rng)
    n_in = x.shape[2]
    g = gains_spanning(n_in, rng)
    print(f"case gains dtype={dtype} prec={prec}", flush=True)
    ref = oracle.beamform(blk.enu, 2, blk.k, blk.az_el, x, gain=g)
    y = gpu_beams(blk, x, g, dtype, prec)
    assert np.all(np.isfinite(y))
    e, m = rel_rms(y, ref), max_err(y, ref)
    print(f"all inputs rel-rms {e:.2e} max {m:.2e}", flush=True)
    assert e <= TOL[prec] and m <= PER_ELEM[prec]
    worst = 0.0
    for i in range(n_in - 1):
        xi = np.zeros_like(x)
        xi[:, :, i] = x[:, :, i]
        ref = oracle.beamform(blk.enu, 2, blk.k, blk.az_el, xi, gain=g)
        yi = gpu_beams(blk, xi, g, dtype, prec)
        assert np.all(np.isfinite(yi)), i
        e, m = rel_rms(yi, ref), max_err(yi, ref)
        worst = max(worst, e)
        assert e <= TOL[prec] and m <= PER_ELEM[prec], (i, float(g[i]), e, m)
    print(f"worst single-input rel-rms {worst:.2e}", flush=True)
    # the zero-gain input contributes nothing
    xz = np.zeros_like(x)
    xz[:, :, n_in - 1] = x[:, :, n_in - 1]
    assert np.all(gpu_beams(blk, xz, g, dtype, prec) == 0)


@pytest.mark.parametrize("bad", [2.0 ** -15, 2.0 ** 8 * 1.01, -(2.0 ** 9)])
@pytest.mark.parametrize("dtype", [lp.LP_CI8, lp.LP_CI16])
def test_gain_outside_fp16_range_rejected(bad, dtype):
    rng = np.random.default_rng(5)
    blk, x = block(dtype, rng)
    g = np.ones(x.shape[2], np.float32)
    g[3] = bad
    with pytest.raises(lp.LpError, match="scaling range"):
        gpu_beams(blk, x, g, dtype, lp.LP_FP16_MFMA)
    # just inside the range is accepted
    g[3] = np.float32(2.0 ** 8) if bad > 1 else np.float32(2.0 ** -14 * 0.51)
    y = gpu_beams(blk, x, g, dtype, lp.LP_FP16_MFMA)
    assert np.all(np.isfinite(y))
    # the FP32 path has no such range
    g[3] = bad
    y = gpu_beams(blk, x, g, dtype, lp.LP_FP32)
    assert np.all(np.isfinite(y))
