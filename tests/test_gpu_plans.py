"""The context's plan cache on the GPU: bounded memory as pointings change,
plans released when serving streams close, tables in a caller-bound
buffer giving bitwise the same results, and LP_ENOMEM when that buffer is
too small.
"""
import numpy as np
import pytest

import lofarsim
from chain import as_complex, run_gpu
from paper_1612_06592_amd import lp

pytestmark = pytest.mark.gpu


def small_block():
    cfg = lofarsim.get_config("c1", n_t=4096, n_pulses=1)
    return lofarsim.generate(cfg)


def test_direct_calls_with_new_pointings_stay_bounded():
    import torch
    blk = small_block()
    ctx = lp.Ctx(0)
    ctx.plan_cache(8)
    S, n_t = len(blk.k), 2048
    x = torch.from_numpy(np.ascontiguousarray(blk.x[:, :n_t])).to("cuda:0")
    y = torch.empty(lp.nbytes("lp_beam_bytes", 1, S, n_t), dtype=torch.uint8,
                    device="cuda:0")
    arr, band = lp.Array(blk.enu, 2), lp.Band(blk.k)
    sizes = []
    for i in range(300):
        az_el = blk.az_el + np.array([[1e-4 * i, 0.0]])
        lp.beamform(ctx, arr, band, lp.Dirs(az_el), x, n_t, lp.LP_CI16,
                    lp.LP_FP16_MFMA, y)
        n, held, nbytes = ctx.plan_stats()
        assert n <= 8 and held == 0, (i, n, held)
        sizes.append(nbytes)
    torch.cuda.synchronize()
    print("plans bytes after 10 / 300 pointings:", sizes[9], sizes[-1],
          flush=True)
    assert max(sizes[8:]) <= max(sizes[:8])
    ctx.close()


def test_serving_streams_release_plans_at_close():
    """Open and close 1000 streams, each with a new pointing and TEC: the
    cache holds no plan of a closed stream and its size stays flat."""
    import torch
    blk = small_block()
    ctx = lp.Ctx(0)
    ctx.plan_cache(16)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda:0")
    srv = lp.Server(ctx, arena=arena)
    counts, sizes = [], []
    for i in range(1000):
        az_el = blk.az_el + np.array([[2e-4 * i, 1e-4]])
        cfg = lp.StreamCfg(blk.enu, blk.k, az_el, [0.01 * i], max_n_t=4096,
                           dtype=lp.LP_CI16)
        sid = srv.open(cfg)
        n, held, nbytes = ctx.plan_stats()
        assert held >= 2  # this stream's weight and chirp plans
        srv.close_stream(sid)
        if i % 100 == 99:
            # the loop releases closed streams asynchronously
            for _ in range(200):
                n, held, nbytes = ctx.plan_stats()
                if held == 0:
                    break
                import time
                time.sleep(0.005)
            counts.append(n)
            sizes.append(nbytes)
            assert held == 0, (i, n, held)
            assert n <= 16 + 3, (i, n)
    print("cached plans every 100 streams:", counts, flush=True)
    print("plan bytes every 100 streams:", sizes, flush=True)
    assert max(sizes) <= 1.05 * sizes[0] + (1 << 20)
    srv.destroy()
    ctx.close()


def test_bound_constant_buffer_bitwise_and_enomem():
    import torch
    cfg = lofarsim.get_config("c2", n_t=4096, n_pulses=1)
    blk = lofarsim.generate(cfg)
    ref = run_gpu(blk, lp.LP_FP16_MFMA, want_series=False)
    # the same chain with every plan table in a caller buffer
    from chain import gpu_pipeline, to_device
    ctx, p = gpu_pipeline(blk, lp.LP_FP16_MFMA, want_series=False)
    const = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda:0")
    ctx.bind_const(const)
    p.step(to_device(blk.x))
    torch.cuda.synchronize()
    n, held, nbytes = ctx.plan_stats()
    print("bound buffer: plans", n, "bytes", nbytes, flush=True)
    assert n >= 3 and nbytes <= const.numel()
    emax, arg, _ = p.cand_view()
    assert np.array_equal(as_complex(p.y_view()), ref["y"])
    assert np.array_equal(as_complex(p.d_view()), ref["d"])
    assert np.array_equal(emax.cpu().numpy(), ref["emax"])
    tr = p.triggers()
    assert len(tr) == len(ref["trig"])
    assert np.array_equal(tr["sample"], ref["trig"]["sample"])
    # a buffer too small for the chirp table of 244 subbands
    tiny = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda:0")
    ctx.bind_const(tiny)
    with pytest.raises(lp.LpError) as ei:
        p.step(to_device(blk.x))
    assert ei.value.code == lp.LP_ENOMEM
    torch.cuda.synchronize()
    ctx.bind_const(None)
    ctx.close()
