"""The serving scheduler, exercised on the CPU through its dry-run executor.

No device work happens here: a launch completes after a simulated time per
probe key.  The checks are the admission rules: first-in first-out, the HBM
budget is never exceeded, a request larger than the budget is refused at
once, every admitted request completes, packing respects its limits.
"""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def A():
    from paper_2411_18183_amd import asjoin as A
    A.lib()
    return A


def request(n, key_len=10):
    off = np.arange(n + 1, dtype=np.int64) * key_len
    return np.zeros(max(n * key_len, 1), np.uint8), off, np.zeros((max(n, 1), 2), np.int32)


def footprint(n, key_len=10, cap=None):
    al = lambda x: (x + 255) // 256 * 256
    cap = n if cap is None else cap
    return al(n * key_len) + al(8 * (n + 1)) + 2 * al(4 * n) + al(16 * (n // 64 + 1)) + al(8 * cap) + 2048


def run(A, sizes, **opts):
    s = A.Server(None, dry_run=True, **opts)
    tickets = []
    for n in sizes:
        d, o, out = request(n)
        tickets.append(s.submit(d, o, out))
    infos = [s.wait(t) for t in tickets]
    st = s.stats()
    s.close()
    return infos, st


def test_fifo_and_budget(A):
    rng = np.random.default_rng(0)
    sizes = [int(x) for x in rng.integers(100, 5000, size=60)]
    budget = 3 * footprint(5000)
    infos, st = run(A, sizes, slots=3, hbm_budget=budget, dry_ns_per_key=200.0)
    assert all(i["status"] == 0 for i in infos)
    assert st["peak_budget_used"] <= budget and st["budget_used"] == 0
    launches = [i["t_launch_ms"] for i in infos]
    batches = [i["batch_id"] for i in infos]
    assert launches == sorted(launches) and batches == sorted(batches)  # first in, first out
    assert all(i["t_arrive_ms"] <= i["t_launch_ms"] <= i["t_done_ms"] for i in infos)


def test_request_larger_than_budget_is_refused(A):
    s = A.Server(None, dry_run=True, hbm_budget=footprint(1000), dry_ns_per_key=10.0)
    d, o, out = request(1000)
    t = s.submit(d, o, out)  # exactly fits
    d2, o2, out2 = request(1100)
    with pytest.raises(A.AsjError) as e:
        s.submit(d2, o2, out2)
    assert e.value.code == A.ASJ_ENOMEM
    assert s.wait(t)["status"] == 0
    s.close()


def test_small_budget_blocks_but_never_drops(A):
    sizes = [1000] * 12
    infos, st = run(A, sizes, slots=4, hbm_budget=footprint(1000), dry_ns_per_key=2000.0)
    assert all(i["status"] == 0 for i in infos)
    assert all(i["batch_requests"] == 1 for i in infos)  # one request fits at a time
    # strictly one after another: each launch waits for the previous completion
    for a, b in zip(infos, infos[1:]):
        assert b["t_launch_ms"] >= a["t_done_ms"] - 1e-6


def test_packing_limits(A):
    sizes = [500] * 40
    infos, st = run(A, sizes, slots=1, max_batch_requests=4, dry_ns_per_key=5000.0)
    assert max(i["batch_requests"] for i in infos) <= 4
    assert st["launches"] < len(sizes)  # queued requests were packed
    infos, st = run(A, sizes, slots=1, max_batch_keys=1200, dry_ns_per_key=5000.0)
    assert max(i["batch_requests"] for i in infos) <= 2
    infos, st = run(A, sizes, slots=2, max_batch_requests=1, dry_ns_per_key=1000.0)
    assert st["launches"] == len(sizes)


def test_bad_arguments(A):
    s = A.Server(None, dry_run=True)
    with pytest.raises(A.AsjError):
        s.submit(np.zeros(4, np.uint8), np.array([3, 1], dtype=np.int64), np.zeros((1, 2), np.int32))
    s.close()
    with pytest.raises(A.AsjError):
        A.Server(None)  # a real server needs a table


def test_decreasing_offsets_are_refused_at_submission(A):
    s = A.Server(None, dry_run=True, dry_ns_per_key=1.0)
    d, o, out = request(100)
    o[40], o[41] = o[41], o[40]
    with pytest.raises(A.AsjError) as e:
        s.submit(d, o, out)
    assert e.value.code == A.ASJ_EINVAL
    s.close()


def test_second_waiter_on_a_ticket_is_refused(A):
    """One waiter per ticket: while one thread waits, a second wait on the same
    ticket returns ASJ_EINVAL at once (it must not share the request the first
    waiter frees); after the first wait the ticket is released."""
    import threading
    s = A.Server(None, dry_run=True, dry_ns_per_key=20000.0)  # ~40 ms for 2000 keys
    d, o, out = request(2000)
    t = s.submit(d, o, out)
    first = {}
    th = threading.Thread(target=lambda: first.update(s.wait(t)))
    th.start()
    import time
    time.sleep(0.01)
    assert s.wait(t)["status"] == A.ASJ_EINVAL
    th.join()
    assert first["status"] == 0
    assert s.wait(t)["status"] == A.ASJ_EINVAL  # released
    s.close()


def test_submit_checks_buffers(A):
    s = A.Server(None, dry_run=True, dry_ns_per_key=10.0)
    d, o, out = request(100)
    with pytest.raises(ValueError):
        s.submit(d, o, out, out_cap=out.shape[0] + 1)  # more rows than out holds
    with pytest.raises(ValueError):
        s.submit(d, o.astype(np.int32), out)
    with pytest.raises(ValueError):
        s.submit(d.astype(np.int16), o, out)
    with pytest.raises(ValueError):
        s.submit(d, o, out.astype(np.int64))
    s.wait(s.submit(d, o, out, out_cap=10))
    s.close()
