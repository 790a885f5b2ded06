"""The serving loop's policy on the CPU: a fake clock and a fake executor
stand in for time and the device (admission order, the HBM budget,
rejection, per-request failure, cancellation, deadlines, latency stats)."""

import numpy as np
import pytest

from paper_2411_16680_amd import serve, synth


def _reqs(arrivals, w=640, h=360, scene=0):
    cam = synth.Camera(np.eye(3), np.eye(4), w, h)
    return [synth.ServeRequest(i, scene, w, h, cam, t) for i, t in enumerate(arrivals)]


def _server(budget, cost=0.010, concurrency=1, bytes_fn=lambda r: 100, fail_on=lambda r: False):
    clk = serve.FakeClock()
    ex = serve.FakeExecutor(clk, lambda r: cost, bytes_fn=bytes_fn, fail_on=fail_on,
                            concurrency=concurrency)
    return serve.Server(ex, budget, clock=clk), clk, ex


def test_fifo_latency_single_lane():
    srv, clk, ex = _server(budget=10_000, cost=0.010)
    jobs = srv.run(_reqs([0.0, 0.001, 0.050]), sleep=clk.sleep, poll=1e-4)
    assert [j.status for j in jobs] == ["done"] * 3
    assert ex.launched == [0, 1, 2]
    # the second queues behind the first on the single lane; the third finds it idle
    assert jobs[0].latency == pytest.approx(0.010, abs=2e-4)
    assert jobs[1].latency == pytest.approx(0.019, abs=2e-4)
    assert jobs[2].latency == pytest.approx(0.010, abs=2e-4)


def test_budget_forces_queueing_in_order():
    # budget holds one request at a time: each starts when the previous ends
    srv, clk, ex = _server(budget=150, cost=0.010, concurrency=4)
    jobs = srv.run(_reqs([0.0, 0.0, 0.0]), sleep=clk.sleep, poll=1e-4)
    assert [j.status for j in jobs] == ["done"] * 3
    assert jobs[1].t_start == pytest.approx(jobs[0].t_done, abs=1e-9)
    assert jobs[2].t_start == pytest.approx(jobs[1].t_done, abs=1e-9)
    assert srv.used == 0


def test_head_of_line_order_kept():
    sizes = {0: 100, 1: 900, 2: 50}
    srv, clk, ex = _server(budget=1000, cost=0.010, concurrency=4,
                           bytes_fn=lambda r: sizes[r.rid])
    jobs = srv.run(_reqs([0.0, 0.0, 0.0]), sleep=clk.sleep, poll=1e-4)
    # request 1 cannot start beside request 0 (100 + 900 fits exactly -> it can);
    # request 2 must not overtake request 1
    assert ex.launched == [0, 1, 2]
    assert jobs[2].t_start >= jobs[1].t_start


def test_request_larger_than_budget_is_rejected_and_loop_continues():
    srv, clk, ex = _server(budget=500, bytes_fn=lambda r: 1000 if r.rid == 1 else 100)
    jobs = srv.run(_reqs([0.0, 0.0, 0.0]), sleep=clk.sleep, poll=1e-4)
    assert [j.status for j in jobs] == ["done", "rejected", "done"]
    assert "budget" in jobs[1].error
    assert ex.launched == [0, 2]


def test_library_rejection_fails_only_that_request():
    srv, clk, ex = _server(budget=10_000, fail_on=lambda r: r.rid == 0)
    jobs = srv.run(_reqs([0.0, 0.002]), sleep=clk.sleep, poll=1e-4)
    assert [j.status for j in jobs] == ["failed", "done"]
    assert "QK_ESHAPE" in jobs[0].error
    assert srv.used == 0


def test_cancel_before_start():
    srv, clk, ex = _server(budget=10_000)
    reqs = _reqs([0.0, 1.0])
    for r in reqs:
        srv.submit(r)
    srv.start()
    srv.step()
    assert srv.cancel(1) is True
    assert srv.cancel(0) is False            # already running
    while not srv.idle():
        clk.sleep(1e-3)
        srv.step()
    assert srv.jobs[1].status == "cancelled" and ex.launched == [0]


def test_deadline_miss_flagged():
    srv, clk, ex = _server(budget=10_000, cost=0.040)
    jobs = srv.run(_reqs([0.0]), deadline=1.0 / 30.0, sleep=clk.sleep, poll=1e-4)
    assert jobs[0].status == "done" and jobs[0].missed
    st = serve.summarize(jobs)
    assert st["deadline_missed"] == 1 and st["frac_under_slo"] == 0.0


def test_poisson_stream_statistics():
    scenes, model, reqs = synth.make_serving(n_scenes=4, n_requests=400, rate=60.0, seed=9)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 60.0) < 0.2 / 60.0
    srv, clk, ex = _server(budget=10 ** 12, cost=0.004, concurrency=2,
                           bytes_fn=serve.request_bytes)
    jobs = srv.run(reqs, sleep=clk.sleep, poll=1e-4)
    st = serve.summarize(jobs)
    assert st["done"] == 400
    assert 4.0 <= st["p50_ms"] <= st["p99_ms"] < 40.0
    assert st["throughput_rps"] == pytest.approx(60.0, rel=0.2)


@pytest.mark.parametrize("V,wh", [(8, (1920, 1080)), (4, (640, 360)), (6, (1280, 720))])
def test_request_bytes_match_the_frame_buffers(V, wh):
    """The admission estimate equals what a frame allocates: its buffers
    (runner.frame_buffers, allocated here on the CPU) and the ray-encoded
    copy of the pyramid."""
    import torch
    from paper_2411_16680_amd import runner
    r = _reqs([0.0], *wh)[0]
    chain, frame = runner.frame_buffers(synth.QUARK_STEPS, 32, V, (wh[1], wh[0]), "bf16",
                                        device="cpu")
    seen, total = set(), 0
    for t in list(chain.values()) + list(frame.values()):
        for x in (t if isinstance(t, list) else [t]):
            if x is not None and id(x) not in seen:
                seen.add(id(x))
                total += x.numel() * x.element_size()
    total += sum(h * w * 32 * 2 for h, w in synth.QUARK_FEAT_HW) * V
    assert serve.request_bytes(r, V=V) == total


def test_novel_cameras_in_ball_and_facing_centre():
    scenes, model, reqs = synth.make_serving(n_scenes=3, n_requests=50, seed=2)
    for r in reqs:
        sc = scenes[r.scene_id]
        c = -r.novel.E[:3, :3].T @ r.novel.E[:3, 3]
        assert np.linalg.norm(c - sc.centroid) <= 0.3 + 1e-12
        z = r.novel.E[2, :3]                              # optical axis in world
        to_c = (sc.centre - c) / np.linalg.norm(sc.centre - c)
        assert np.dot(z, to_c) > 0.999
