"""Scheduler tests of the continuous-batching server, without a GPU.

A simulated backend models each slot as a device queue that runs slices at a
fixed rate, on a manual clock, so admission, fairness, cancellation and
failure handling can be checked deterministically.
"""
import pytest

from paper_1902_04446_amd.serving import ApspServer, Request, SimBackend, percentile


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def drive(server, clock, reqs, dt=1e-4, limit=1e5):
    reqs = sorted(reqs, key=lambda r: r.arrival)
    i = 0
    peak_used = 0
    peak_active = 0
    steps = 0
    while i < len(reqs) or not server.idle():
        while i < len(reqs) and reqs[i].arrival <= clock.t:
            server.submit(reqs[i])
            i += 1
        server.step(clock.t)
        peak_used = max(peak_used, server.used)
        peak_active = max(peak_active, len(server.active))
        clock.t += dt
        steps += 1
        assert steps < limit, "scheduler did not drain"
    return peak_used, peak_active


def mk(sizes, arrivals=None):
    arrivals = arrivals or [0.0] * len(sizes)
    return [Request(rid=i, n=n, arrival=a) for i, (n, a) in enumerate(zip(sizes, arrivals))]


def test_all_requests_complete_and_latency_covers_service_time():
    clock = Clock()
    be = SimBackend(rate=1e12, clock=clock)
    srv = ApspServer(be, hbm_budget=1 << 34, slots=4, slice_rounds=4, clock=clock)
    reqs = mk([256, 1024, 4096, 256, 1024])
    drive(srv, clock, reqs)
    assert all(r.status == "done" for r in reqs)
    for r in reqs:
        assert r.latency >= r.n ** 3 / 1e12 - 1e-3
    assert be.allocated == be.freed == len(reqs)


def test_admission_respects_memory_budget():
    clock = Clock()
    be = SimBackend(rate=1e12, clock=clock)
    need = be.bytes_needed(2048)
    srv = ApspServer(be, hbm_budget=2 * need + 10, slots=8, slice_rounds=2, clock=clock)
    reqs = mk([2048] * 6)
    peak_used, peak_active = drive(srv, clock, reqs)
    assert peak_used <= srv.budget
    assert peak_active == 2
    assert all(r.status == "done" for r in reqs)


def test_slots_bound_concurrency():
    clock = Clock()
    be = SimBackend(rate=1e12, clock=clock)
    srv = ApspServer(be, hbm_budget=1 << 40, slots=3, slice_rounds=2, clock=clock)
    _, peak_active = drive(srv, clock, mk([512] * 10))
    assert peak_active == 3


def test_oversized_request_is_rejected_not_queued():
    clock = Clock()
    be = SimBackend(clock=clock)
    srv = ApspServer(be, hbm_budget=be.bytes_needed(1000), slots=2, clock=clock)
    reqs = mk([1001, 500])
    drive(srv, clock, reqs)
    assert reqs[0].status == "rejected" and reqs[1].status == "done"


def test_small_request_overtakes_a_running_large_one():
    # continuous batching: a small request that arrives while a large one is
    # on the device is admitted into a free slot and finishes first
    clock = Clock()
    be = SimBackend(rate=1e12, clock=clock)
    srv = ApspServer(be, hbm_budget=1 << 36, slots=2, slice_rounds=1, clock=clock)
    reqs = mk([8192, 256], arrivals=[0.0, 0.05])
    drive(srv, clock, reqs)
    big, small = reqs
    assert small.done < big.done
    assert small.latency < 0.01


def test_bypass_is_bounded():
    clock = Clock()
    be = SimBackend(rate=1e12, clock=clock)
    need_big = be.bytes_needed(4096)
    # room for one big request; a second big one must wait while smalls flow
    srv = ApspServer(be, hbm_budget=need_big + be.bytes_needed(256) * 2, slots=8,
                     slice_rounds=1, max_bypass=3, clock=clock)
    sizes = [4096, 4096] + [256] * 30
    arrivals = [0.0, 0.0] + [0.001 * i for i in range(30)]
    reqs = mk(sizes, arrivals)
    drive(srv, clock, reqs)
    assert all(r.status == "done" for r in reqs)
    second_big = reqs[1]
    overtakers = [r for r in reqs[2:] if r.admitted < second_big.admitted]
    # each pending pass that skips the big request counts one bypass
    assert second_big.bypassed > 3
    assert len(overtakers) <= 30


def test_cancel_pending_and_running():
    clock = Clock()
    be = SimBackend(rate=1e12, clock=clock)
    srv = ApspServer(be, hbm_budget=1 << 36, slots=1, slice_rounds=1, clock=clock)
    reqs = mk([4096, 4096])
    for r in reqs:
        srv.submit(r)
    srv.step(0.0)
    assert srv.cancel(1)                 # still pending
    assert reqs[1].status == "cancelled"
    assert srv.cancel(0)                 # running: drains its enqueued slices
    drive(srv, clock, [])
    assert reqs[0].status == "cancelled" and srv.used == 0 and srv.free_slots == [0]
    assert not srv.cancel(7)


def test_failed_slice_is_retried_then_gives_up():
    clock = Clock()
    be = SimBackend(rate=1e12, clock=clock, fail=(0,))
    srv = ApspServer(be, hbm_budget=1 << 36, slots=2, slice_rounds=2, max_retries=1,
                     clock=clock)
    reqs = mk([1024, 512])
    drive(srv, clock, reqs)
    assert reqs[0].status == "done" and reqs[0].retries == 1
    clock2 = Clock()
    be2 = SimBackend(rate=1e12, clock=clock2, fail=(0,))
    srv2 = ApspServer(be2, hbm_budget=1 << 36, slots=2, slice_rounds=2, max_retries=0,
                      clock=clock2)
    reqs2 = mk([1024])
    drive(srv2, clock2, reqs2)
    assert reqs2[0].status == "failed" and srv2.used == 0


@pytest.mark.parametrize("inflight", [1, 3])
def test_retry_resumes_from_the_last_good_checkpoint(inflight):
    """A slice of rounds 4..5 fails (forced): the request resumes from the
    checkpoint at round 4, not from round 0, and ends with every round applied
    once in order; with inflight 3 the slices enqueued behind the failed one
    ran on bad data and are discarded with it."""
    clock = Clock()
    be = SimBackend(rate=1e12, b=64, clock=clock, fail_at={0: 5})
    srv = ApspServer(be, hbm_budget=1 << 36, slots=1, slice_rounds=2, inflight=inflight,
                     checkpoint_rounds=4, clock=clock)
    reqs = mk([1024])          # 16 rounds of 64
    drive(srv, clock, reqs)
    r = reqs[0]
    assert r.status == "done" and r.retries == 1
    assert r.result == list(range(16))
    assert be.loads == 1 and be.restores == 1
    assert srv.used == 0


def test_retry_without_checkpoints_reingests_the_input():
    clock = Clock()
    be = SimBackend(rate=1e12, b=64, clock=clock, fail_at={0: 9})
    srv = ApspServer(be, hbm_budget=1 << 36, slots=1, slice_rounds=2, clock=clock)
    reqs = mk([1024])
    drive(srv, clock, reqs)
    assert reqs[0].status == "done" and reqs[0].result == list(range(16))
    assert be.loads == 2 and be.restores == 0


def test_checkpoints_count_against_the_budget():
    clock = Clock()
    be = SimBackend(clock=clock)
    srv = ApspServer(be, hbm_budget=2 * be.bytes_needed(1000), slots=2, checkpoint_rounds=4,
                     clock=clock)
    reqs = mk([1000])
    drive(srv, clock, reqs)
    assert reqs[0].status == "rejected"      # matrix + 2 checkpoint buffers > 2 matrices


def test_srpt_serves_the_least_remaining_work_first():
    # one request runs at a time: a small request arriving behind a large one
    # gets the device at the large one's next slice boundary under srpt, and
    # waits for it to finish under fifo
    out = {}
    for policy in ("srpt", "fifo"):
        clock = Clock()
        be = SimBackend(rate=1e12, clock=clock)
        srv = ApspServer(be, hbm_budget=1 << 36, slots=2, slice_rounds=1, inflight=1,
                         policy=policy, max_running=1, clock=clock)
        reqs = mk([4096, 256], arrivals=[0.0, 0.001])
        drive(srv, clock, reqs, dt=1e-5, limit=1e7)
        big, small = reqs
        assert big.status == small.status == "done"
        out[policy] = (small.done < big.done)
    assert out == {"srpt": True, "fifo": False}


def test_large_requests_run_one_at_a_time():
    clock = Clock()
    be = SimBackend(rate=1e12, clock=clock)
    srv = ApspServer(be, hbm_budget=1 << 40, slots=4, slice_rounds=2, policy="fifo",
                     large_n=4096, max_large=1, clock=clock)
    reqs = mk([4096, 8192, 256, 4096, 512], arrivals=[0.0, 0.0, 0.001, 0.002, 0.003])
    peak = 0
    i = 0
    while i < len(reqs) or not srv.idle():
        while i < len(reqs) and reqs[i].arrival <= clock.t:
            srv.submit(reqs[i])
            i += 1
        srv.step(clock.t)
        peak = max(peak, sum(1 for r in srv.active if r.n >= 4096 and r.inflight))
        clock.t += 1e-4
    assert peak == 1
    assert all(r.status == "done" for r in reqs)
    # the small ones ran beside the large ones and finished first
    assert reqs[2].done < reqs[0].done and reqs[4].done < reqs[1].done
    # fifo among the large ones
    assert reqs[0].done < reqs[1].done < reqs[3].done


def test_unknown_policy_is_rejected():
    with pytest.raises(ValueError):
        ApspServer(SimBackend(), hbm_budget=1, policy="lifo")


def test_warmup_requests_are_left_out_of_latency():
    from paper_1902_04446_amd.serving import summarize

    reqs = mk([256, 256, 512], arrivals=[0.0, 1.0, 2.0])
    for r, lat in zip(reqs, (5.0, 0.001, 0.002)):
        r.status, r.done = "done", r.arrival + lat
    st = summarize(reqs, 3.0, warmup=1)
    assert st["warmup_excluded"] == 1 and st["done"] == 3
    assert st["p99_ms"] == pytest.approx(2.0)
    assert st["per_size"]["256"]["count"] == 1
    assert st["per_size"]["512"]["p50_ms"] == pytest.approx(2.0)


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50
    assert percentile(v, 99) == 99
    assert percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0


def test_slot_state_is_counted_once_per_slot():
    """A backend whose slots keep solver state (growing with the largest
    request they solved): admission counts the growth, the state stays
    counted after the request leaves, and a request that cannot fit with its
    state is rejected."""
    class StateSim(SimBackend):
        def state_bytes(self, n):
            return 1000 * n

    clock = Clock()
    be = StateSim(rate=1e12, clock=clock)
    budget = be.bytes_needed(512) + 1000 * 512 + 10
    srv = ApspServer(be, hbm_budget=budget, slots=1, slice_rounds=2, clock=clock)
    reqs = mk([512, 256, 512])
    peak, _ = drive(srv, clock, reqs)
    assert all(r.status == "done" for r in reqs)
    assert peak <= budget
    assert srv.slot_state == [1000 * 512] and srv.used == 1000 * 512
    srv2 = ApspServer(be, hbm_budget=be.bytes_needed(512) + 10, slots=1, clock=clock)
    r = srv2.submit(Request(rid=9, n=512, arrival=0.0))
    assert r.status == "rejected"
