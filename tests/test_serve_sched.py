"""Host logic of the render server on the CPU: the stub launcher completes a
batch after a fixed time and touches no GPU, so queueing, admission, batch
formation, deferred unload, cancellation and timeouts are tested without one."""
import threading
import time

import pytest

import gen
from paper_2311_18561_amd import _lib as L
from paper_2311_18561_amd.serve import Server

CAM = gen.make_camera(640, 480)


def test_continuous_batching_admits_requests_as_lanes_free():
    with Server(max_batch=4, max_inflight=2, stub_launch_us=400_000, max_batch_gaussians=100_000_000) as s:
        sid = s.load_scene(n=1000)
        tks = [s.submit(sid, CAM, 0.0)]
        time.sleep(0.08)            # launched alone on the first lane
        tks.append(s.submit(sid, CAM, 0.1))
        time.sleep(0.08)            # launched alone on the second lane, overlapping the first
        tks += [s.submit(sid, CAM, 0.1 * i) for i in range(2, 10)]  # both lanes busy: these queue
        res = [s.wait(t) for t in tks]
        assert all(r.status == 0 for r in res)
        assert [r.batch_size for r in res] == [1, 1, 4, 4, 4, 4, 4, 4, 4, 4]
        # the second request ran while the first was still on the "device"
        assert res[1].t_launch_ns < res[0].t_done_ns
        launches = [r.t_launch_ns for r in res]
        assert launches == sorted(launches)  # FIFO
        st = s.stats()
        assert st["completed"] == 10 and st["batches"] == 4 and st["mean_batch"] == 2.5


def test_late_arrivals_join_the_next_batch_while_one_runs():
    with Server(max_batch=8, max_inflight=1, stub_launch_us=300_000) as s:
        sid = s.load_scene(n=1000)
        first = s.submit(sid, CAM, 0.0)
        time.sleep(0.08)
        late = [s.submit(sid, CAM, 0.0) for _ in range(3)]
        r0 = s.wait(first)
        rl = [s.wait(t) for t in late]
        assert r0.batch_size == 1
        assert all(r.batch_size == 3 for r in rl)
        assert all(r.t_launch_ns >= r0.t_done_ns - 1_000_000 for r in rl)


def test_admission_by_batch_budget():
    with Server(max_batch=8, max_inflight=1, stub_launch_us=300_000, max_batch_gaussians=5_000_000,
                max_batch_pixels=3 * 640 * 480) as s:
        big = s.load_scene(n=3_000_000)
        small = s.load_scene(n=1_000_000)
        huge = s.load_scene(n=6_000_000)
        blocker = s.submit(small, CAM, 0.0)
        time.sleep(0.08)  # the blocker holds the only lane while the rest queue
        tks = [s.submit(big, CAM, 0.0), s.submit(small, CAM, 0.0), s.submit(big, CAM, 0.0),
               s.submit(small, CAM, 0.0), s.submit(small, CAM, 0.0), s.submit(small, CAM, 0.0)]
        bad = s.submit(huge, CAM, 0.0)
        s.wait(blocker)
        res = [s.wait(t) for t in tks]
        # FIFO batches within 5M Gaussians and 3 frames: (3M + 1M), (3M + 1M + 1M), (1M)
        assert [r.batch_size for r in res] == [2, 2, 3, 3, 3, 1]
        r = s.wait(bad)
        assert r.status == L.PVG_ERR_NOMEM


def test_memory_budget_on_scene_load():
    with Server(max_batch=2, max_inflight=1, stub_launch_us=1000, max_batch_gaussians=1000,
                max_batch_pixels=640 * 480, instance_capacity=1000, mem_budget_bytes=64 << 20) as s:
        s.load_scene(n=100_000)  # 100k x 56 floats ~ 22 MB
        with pytest.raises(L.PVGError) as e:
            s.load_scene(n=1_000_000)
        assert e.value.status == L.PVG_ERR_NOMEM


def test_unload_is_deferred_until_pending_requests_finish():
    with Server(max_batch=1, max_inflight=1, stub_launch_us=30_000) as s:
        sid = s.load_scene(n=1000)
        tks = [s.submit(sid, CAM, 0.0) for _ in range(3)]
        s.unload_scene(sid)
        with pytest.raises(L.PVGError) as e:
            s.submit(sid, CAM, 0.0)
        assert e.value.status == L.PVG_ERR_NOT_FOUND
        assert all(s.wait(t).status == 0 for t in tks)
        with pytest.raises(L.PVGError):
            s.unload_scene(sid)


def test_wait_timeout_poll_and_cancel():
    with Server(max_batch=1, max_inflight=1, stub_launch_us=400_000) as s:
        sid = s.load_scene(n=1000)
        a = s.submit(sid, CAM, 0.0)
        b = s.submit(sid, CAM, 0.0)
        c = s.submit(sid, CAM, 0.0)
        with pytest.raises(L.PVGError) as e:
            s.wait(b, timeout_s=0.001)
        assert e.value.status == L.PVG_ERR_TIMEOUT
        assert not s.poll(c)
        s.release(c)  # still queued: cancelled
        with pytest.raises(L.PVGError) as e:
            s.poll(c)
        assert e.value.status == L.PVG_ERR_NOT_FOUND
        time.sleep(0.08)
        with pytest.raises(L.PVGError) as e:
            s.release(a)  # launched, not finished
        assert e.value.status == L.PVG_ERR_BUSY
        assert s.wait(a).status == 0 and s.wait(b).status == 0
        assert s.stats()["completed"] == 2


def test_concurrent_clients():
    with Server(max_batch=8, max_inflight=2, stub_launch_us=5_000) as s:
        sids = [s.load_scene(n=1000 * (k + 1)) for k in range(3)]
        out = []

        def client(k):
            for i in range(20):
                out.append(s.wait(s.submit(sids[(k + i) % 3], CAM, 0.0)).status)

        th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert out == [0] * 80
        assert s.stats()["completed"] == 80


def test_destroy_drains_queued_work():
    s = Server(max_batch=2, max_inflight=1, stub_launch_us=10_000)
    sid = s.load_scene(n=1000)
    tks = [s.submit(sid, CAM, 0.0) for _ in range(6)]
    s.close()  # returns only after all six ran
    del tks


def test_invalid_configuration_rejected():
    with pytest.raises(L.PVGError) as e:
        Server(max_batch=0, stub_launch_us=1000)
    assert e.value.status == L.PVG_ERR_INVALID
    with pytest.raises(L.PVGError):
        Server(max_inflight=9, stub_launch_us=1000)
    with Server(max_batch=1, max_inflight=1, stub_launch_us=1000) as s:
        bad = dict(CAM)
        bad["width"] = 0
        sid = s.load_scene(n=10)
        with pytest.raises(L.PVGError) as e:
            s.submit(sid, bad, 0.0)
        assert e.value.status == L.PVG_ERR_INVALID
        with pytest.raises(L.PVGError) as e:
            s.submit(sid + 100, CAM, 0.0)
        assert e.value.status == L.PVG_ERR_NOT_FOUND


def test_injected_launch_fault_fails_its_tickets_and_the_server_carries_on(monkeypatch):
    """PVG_FAULT_INJECT=2: every second batch launch fails before any device
    work.  Requests go one batch at a time, so exactly the even-numbered
    batches fail with PVG_ERR_HIP and the others complete."""
    monkeypatch.setenv("PVG_FAULT_INJECT", "2")
    with Server(max_batch=4, max_inflight=1, stub_launch_us=2_000) as s:
        sid = s.load_scene(n=1000)
        status = [s.wait(s.submit(sid, CAM, 0.0)).status for _ in range(6)]
        assert status == [0, L.PVG_ERR_HIP] * 3
        # a batch of several requests fails as a whole
        tks = [s.submit(sid, CAM, 0.0) for _ in range(3)]
        res = [s.wait(t) for t in tks]
        assert {r.status for r in res} <= {0, L.PVG_ERR_HIP}
        st = s.stats()
        assert st["completed"] + st["failed"] == 9 and st["failed"] >= 3
    monkeypatch.delenv("PVG_FAULT_INJECT")
    with Server(max_batch=4, max_inflight=1, stub_launch_us=2_000) as s:  # off again
        sid = s.load_scene(n=1000)
        assert [s.wait(s.submit(sid, CAM, 0.0)).status for _ in range(4)] == [0] * 4


def test_scene_files_round_trip_into_a_server(tmp_path):
    """save_scene / load_scene: one float32 .npy per field, bit-exact round
    trip, shape checks on load, and the loaded scene accepted by a server."""
    import numpy as np
    import paper_2311_18561_amd as pvg
    scene = gen.make_scene(500, 3, sh_degree=2)
    params = [scene[f] for f in pvg.FIELDS]
    pvg.save_scene(str(tmp_path / "s"), params)
    back = pvg.load_scene(str(tmp_path / "s"))
    assert all(np.array_equal(a, b) and b.dtype == np.float32 for a, b in zip(params, back))
    assert sorted(p.name for p in (tmp_path / "s").iterdir()) == sorted(f + ".npy" for f in pvg.FIELDS)
    np.save(tmp_path / "s" / "tau.npy", np.zeros(499, np.float32))
    with pytest.raises(ValueError):
        pvg.load_scene(str(tmp_path / "s"))
    with pytest.raises(ValueError):
        pvg.save_scene(str(tmp_path / "t"), params[:3] + [params[3][:, :, :10]] + params[4:])
    with Server(max_batch=2, max_inflight=1, stub_launch_us=1_000) as s:
        sid = s.load_scene(n=back[0].shape[1], sh_degree=2)
        assert s.wait(s.submit(sid, CAM, 0.0)).status == 0
