"""The serving loop on the simulated executor (no GPU): the real request
loop, admission and chunk scheduling, with every device action replaced by
a modelled completion time on one in-order queue."""
import threading
import time

import numpy as np
import pytest

from paper_1612_06592_amd import lp

NS_PER_SAMPLE = 1e-4        # modelled device cost per station-beam sample


def cfg(n_st=4, n_sb=8, beams=1, tec=(5.0,), max_n_t=65536, deadline_s=0.0,
        trig_cap=0):
    az = [(0.1 + 0.001 * b, 0.6) for b in range(beams)]
    return lp.StreamCfg(np.zeros((n_st, 3)), range(60, 60 + n_sb), az, tec,
                        max_n_t, deadline_s=deadline_s, trig_cap=trig_cap)


def drain(srv, n, timeout=10.0):
    out, t0 = [], time.time()
    while len(out) < n and time.time() - t0 < timeout:
        out += srv.poll(timeout_us=20000)
    return out


def test_admission_by_arena_budget():
    c = cfg()
    per = c.resident_bytes(8192)
    srv = lp.Server(arena_bytes=3 * per + 1000, sim_ns_per_sample=NS_PER_SAMPLE,
                    chunk_t=8192)
    ids = [srv.open(c) for _ in range(3)]
    with pytest.raises(lp.LpError) as e:
        srv.open(c)
    assert e.value.code == lp.LP_EAGAIN
    srv.close_stream(ids[0])
    for _ in range(100):                      # released once idle
        try:
            ids.append(srv.open(c))
            break
        except lp.LpError:
            time.sleep(0.01)
    assert len(ids) == 4
    srv.destroy()


def test_submit_validation():
    srv = lp.Server(arena_bytes=1 << 30, sim_ns_per_sample=NS_PER_SAMPLE)
    sid = srv.open(cfg(max_n_t=8192))
    for bad in (0, 1000, 2048 * 5):
        with pytest.raises(lp.LpError) as e:
            srv.submit(sid, None, bad)
        assert e.value.code == lp.LP_EINVAL
    with pytest.raises(lp.LpError):
        srv.submit(sid + 99, None, 2048)
    with pytest.raises(lp.LpError):
        srv.submit(sid, None, 2048, flags=8)
    srv.close_stream(sid)
    with pytest.raises(lp.LpError) as e:
        srv.submit(sid, None, 2048)
    assert e.value.code in (lp.LP_ECLOSED, lp.LP_EINVAL)
    bad = cfg()
    bad.c.n_beams = 65
    with pytest.raises(lp.LpError):
        srv.open(bad)
    # int16 samples from 64 stations x 2 pol: 512-byte rows, beyond the
    # FP16-MFMA tile; accepted at FP32.
    wide = lp.StreamCfg(np.zeros((64, 3)), range(60, 68), [(0.1, 0.6)], (5.0,),
                        8192, dtype=lp.LP_CI16, prec=lp.LP_FP16_MFMA)
    with pytest.raises(lp.LpError, match="256 bytes") as e:
        srv.open(wide)
    assert e.value.code == lp.LP_EINVAL
    wide32 = lp.StreamCfg(np.zeros((64, 3)), range(60, 68), [(0.1, 0.6)],
                          (5.0,), 8192, dtype=lp.LP_CI16, prec=lp.LP_FP32)
    srv.close_stream(srv.open(wide32))
    srv.destroy()


def test_blocks_complete_in_order_with_stream_positions():
    srv = lp.Server(arena_bytes=1 << 30, sim_ns_per_sample=NS_PER_SAMPLE,
                    chunk_t=4096)
    c = cfg()
    sid = srv.open(c)
    lens = [4096, 16384, 2048, 8192]
    for i, n in enumerate(lens):
        srv.submit(sid, None, n, tag=100 + i)
    res = drain(srv, len(lens))
    assert [r["tag"] for r in res] == [100, 101, 102, 103]
    assert [r["frame0"] for r in res] == [0, 4096, 20480, 22528]
    per_sample = 4 * 2 * 8 * 1 * NS_PER_SAMPLE
    for r, n in zip(res, lens):
        assert r["status"] == lp.LP_OK
        assert r["latency_ns"] >= per_sample * n * 0.99
        assert r["deadline_ns"] == pytest.approx((5.0 - n * 1024 / 200e6) * 1e9,
                                                 rel=1e-6)
    st = srv.stats()
    assert st["blocks_done"] == 4 and st["chunks_issued"] == 1 + 4 + 1 + 2
    srv.destroy()


def test_reset_flag_restarts_stream_position():
    srv = lp.Server(arena_bytes=1 << 30, sim_ns_per_sample=NS_PER_SAMPLE)
    sid = srv.open(cfg())
    srv.submit(sid, None, 4096, tag=1)
    srv.submit(sid, None, 4096, tag=2, flags=lp.LP_SUBMIT_RESET)
    res = drain(srv, 2)
    assert [r["frame0"] for r in res] == [0, 0]
    srv.destroy()


def test_earliest_deadline_chunk_goes_first():
    """A long block on a relaxed stream is preempted at chunk granularity by
    a block with an earlier deadline that arrives later."""
    # 2 ns per station-beam sample: the long block takes ~134 ms, the
    # urgent one ~4 ms.
    srv = lp.Server(arena_bytes=1 << 32, sim_ns_per_sample=2.0, chunk_t=2048)
    slow = srv.open(cfg(n_sb=64, deadline_s=100.0, max_n_t=1 << 17))
    urgent = srv.open(cfg(n_sb=64, deadline_s=0.001, max_n_t=1 << 17))
    srv.submit(slow, None, 1 << 17, tag=1)      # 64 chunks
    time.sleep(0.005)
    srv.submit(urgent, None, 4096, tag=2)       # 2 chunks
    res = drain(srv, 2)
    assert [r["tag"] for r in res] == [2, 1]
    srv.destroy()


def test_close_drops_queued_blocks():
    srv = lp.Server(arena_bytes=1 << 32, sim_ns_per_sample=1.0, chunk_t=2048)
    sid = srv.open(cfg(n_sb=64, max_n_t=1 << 16))
    for i in range(5):
        srv.submit(sid, None, 1 << 16, tag=i)
    time.sleep(0.002)
    srv.close_stream(sid)
    res = drain(srv, 5)
    ok = sorted(r["tag"] for r in res if r["status"] == lp.LP_OK)
    dropped = sorted(r["tag"] for r in res if r["status"] == lp.LP_ECLOSED)
    assert ok and dropped and max(ok) < min(dropped)   # in-flight ones finish
    assert sorted(ok + dropped) == list(range(5))
    srv.destroy()


def test_blocks_wait_for_arena_space():
    c = cfg(n_sb=64, beams=4, max_n_t=1 << 16)
    resident = c.resident_bytes(8192)
    blk = c.block_bytes(1 << 16)
    srv = lp.Server(arena_bytes=2 * resident + blk + blk // 2,
                    sim_ns_per_sample=NS_PER_SAMPLE, chunk_t=8192)
    a, b = srv.open(c), srv.open(c)
    for i in range(3):
        srv.submit(a, None, 1 << 16, tag=i)
        srv.submit(b, None, 1 << 16, tag=10 + i)
    res = drain(srv, 6)
    assert len(res) == 6 and all(r["status"] == lp.LP_OK for r in res)
    assert srv.stats()["admit_waits"] > 0
    srv.destroy()


def test_concurrent_submit_and_poll_threads():
    srv = lp.Server(arena_bytes=1 << 32, sim_ns_per_sample=NS_PER_SAMPLE,
                    chunk_t=4096)
    ids = [srv.open(cfg(n_sb=16, max_n_t=16384)) for _ in range(6)]
    rng = np.random.default_rng(0)
    plan = {sid: [int(2048 * rng.integers(1, 9)) for _ in range(10)]
            for sid in ids}

    def producer(sid):
        for i, n in enumerate(plan[sid]):
            srv.submit(sid, None, n, tag=sid * 1000 + i)
            time.sleep(rng.uniform(0, 0.001))

    th = [threading.Thread(target=producer, args=(s,)) for s in ids]
    for t in th:
        t.start()
    res = drain(srv, 60, timeout=20)
    for t in th:
        t.join()
    assert len(res) == 60
    for sid in ids:
        mine = [r for r in res if r["stream"] == sid]
        assert [r["tag"] for r in mine] == [sid * 1000 + i for i in range(10)]
        assert [r["frame0"] for r in mine] == list(np.cumsum([0] + plan[sid][:-1]))
    srv.destroy()


def test_destroy_with_work_in_flight():
    srv = lp.Server(arena_bytes=1 << 32, sim_ns_per_sample=NS_PER_SAMPLE,
                    chunk_t=2048)
    sid = srv.open(cfg(n_sb=64, max_n_t=1 << 16))
    for i in range(4):
        srv.submit(sid, None, 1 << 16, tag=i)
    srv.destroy()                    # must return (admitted block finishes)
