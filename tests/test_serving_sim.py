"""Serving-loop scheduler on the host (simulated executor, no GPU).

The native scheduler runs unchanged; only the executor is replaced by one
that completes a batch after n / rate microseconds without touching the
device (seed spectra take pool memory but are not built).  Checks: every
request completes, the HBM budget (workspace and resident spectra) and
the in-flight limit are never exceeded, unused spectra are evicted when
the pool needs room, oversize and overflow submissions are refused,
admission continues while earlier work is running (continuous batching),
queued requests can be cancelled, seeds can be registered while requests
run, and the budget can come from PA_HBM_BUDGET.
"""
import pytest

import paper_1809_07592_amd as pa
from paper_1809_07592_amd import build as pa_build
import os

FAKE_SEED, FAKE_KEY, FAKE_OUT = 0x100000, 0x200000, 0x300000


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not os.path.exists(pa.LIB_PATH):
        pa_build.build()
    pa.lib()


def ws(n, m):
    return 4 * pa.transform_len(n, m)


def test_all_complete_within_budget_and_inflight_limit():
    budget = 160 << 20
    with pa.Server(budget, max_inflight=6, executor=pa.EXEC_SIMULATED, sim_bits_per_us=2e5) as s:
        sid = s.register_seed(FAKE_SEED, 20_000_000)
        shapes = [(int(1e5 * 1.37 ** (i % 15)), 0) for i in range(200)]
        tickets = []
        for i, (n, _) in enumerate(shapes):
            m = max(1, n // (2 + i % 7))
            tickets.append(s.submit(sid, FAKE_KEY, n, m, FAKE_OUT))
        s.drain()
        st = s.stats()
        assert st["submitted"] == st["completed"] == 200 and st["rejected"] == 0
        assert st["peak_bytes_in_flight"] <= st["budget_bytes"] <= budget
        assert 1 <= st["peak_inflight"] <= 6
        # after the drain only resident seed spectra hold pool memory
        assert st["inflight"] == 0 and st["pending"] == 0
        assert st["bytes_in_flight"] == st["spectrum_bytes"] > 0
        assert st["batches"] >= 200 / 6
        for t in tickets:
            assert s.poll(t) and s.latency_us(t) >= 0


def test_memory_bound_admission_overlaps_work():
    # budget fits the seed spectrum and three of these blocks: later
    # arrivals are admitted as earlier ones finish, while others are still
    # running
    n, m = 1_000_000, 250_000
    budget = 4 * ws(n, m) + 4096
    with pa.Server(budget, max_inflight=64, executor=pa.EXEC_SIMULATED, sim_bits_per_us=1e4) as s:
        sid = s.register_seed(FAKE_SEED, n + m)
        ts = [s.submit(sid, FAKE_KEY, n, m, FAKE_OUT) for _ in range(12)]
        s.drain()
        st = s.stats()
        assert st["completed"] == 12
        assert st["peak_inflight"] == 3
        assert st["peak_bytes_in_flight"] <= budget
        assert st["spectra_resident"] == 1 and st["spectrum_bytes"] == ws(n, m) and st["spectra_built"] == 1
        assert st["batches"] >= 4
        lat = sorted(s.latency_us(t) for t in ts)
        assert lat[-1] > lat[0]


def test_refusals():
    with pa.Server(8 << 20, max_inflight=1, max_queue=2, executor=pa.EXEC_SIMULATED, sim_bits_per_us=1.0) as s:
        sid = s.register_seed(FAKE_SEED, 5_000_000)
        with pytest.raises(pa.PAError) as e:
            s.submit(sid, FAKE_KEY, 4_000_000, 1_000_000, FAKE_OUT)   # workspace > budget
        assert e.value.status == pa.PA_ERR_BUSY
        with pytest.raises(pa.PAError) as e:
            s.submit(sid + 1, FAKE_KEY, 100, 10, FAKE_OUT)              # unknown seed
        assert e.value.status == pa.PA_ERR_INVALID_ARG
        with pytest.raises(pa.PAError):
            s.submit(sid, FAKE_KEY, 100, 101, FAKE_OUT)                 # m > n
        with pytest.raises(pa.PAError):
            s.submit(sid, FAKE_KEY, 4_000_000, 1_000_002, FAKE_OUT)     # seed too short
        # a slow executor: the first request runs, two wait, the fourth overflows
        s.submit(sid, FAKE_KEY, 100_000, 10, FAKE_OUT)
        import time
        time.sleep(0.05)
        s.submit(sid, FAKE_KEY, 100_000, 10, FAKE_OUT)
        s.submit(sid, FAKE_KEY, 100_000, 10, FAKE_OUT)
        with pytest.raises(pa.PAError) as e:
            s.submit(sid, FAKE_KEY, 100_000, 10, FAKE_OUT)
        assert e.value.status == pa.PA_ERR_BUSY
        assert s.stats()["rejected"] == 2


def test_bad_configs():
    for kw in [dict(hbm_budget_bytes=1024), dict(max_inflight=0), dict(streams=0), dict(streams=17),
               dict(executor=7)]:
        args = dict(hbm_budget_bytes=64 << 20, executor=pa.EXEC_SIMULATED)
        args.update(kw)
        with pytest.raises(pa.PAError):
            pa.Server(**args)


def test_unused_spectra_are_evicted_when_the_pool_needs_room():
    # room for one spectrum and one workspace: each request on another seed
    # evicts the previous seed's spectrum, which no request uses any more
    n, m = 500_000, 100_000
    budget = 2 * ws(n, m) + 4096
    with pa.Server(budget, max_inflight=8, executor=pa.EXEC_SIMULATED, sim_bits_per_us=1e5) as s:
        sids = [s.register_seed(FAKE_SEED + 0x1000 * i, n + m) for i in range(4)]
        for i in range(12):
            s.submit(sids[i % 4], FAKE_KEY, n, m, FAKE_OUT)
        s.drain()
        st = s.stats()
        assert st["completed"] == 12 and st["failed"] == 0
        assert st["spectra_built"] == 12 and st["spectra_evicted"] == 11 and st["spectra_resident"] == 1
        assert st["peak_bytes_in_flight"] <= budget and st["peak_inflight"] == 1
        assert st["bytes_in_flight"] == st["spectrum_bytes"] == ws(n, m)


def test_the_spectrum_a_request_needs_is_never_evicted_for_it():
    # room for two spectra and one workspace.  Seeds A and B both resident,
    # A least recently used; while a request on B runs, a request on A must
    # wait for the running one's workspace instead of evicting A's spectrum
    # (which it is about to use) to make room
    n, m = 200_000, 50_000
    u = ws(n, m)
    budget = 3 * u + 4096
    with pa.Server(budget, max_inflight=8, executor=pa.EXEC_SIMULATED, sim_bits_per_us=1e4) as s:
        a = s.register_seed(FAKE_SEED, n + m)
        b = s.register_seed(FAKE_SEED + 0x1000, n + m)
        s.wait(s.submit(a, FAKE_KEY, n, m, FAKE_OUT))
        s.wait(s.submit(b, FAKE_KEY, n, m, FAKE_OUT))
        assert s.stats()["spectra_resident"] == 2
        running = s.submit(b, FAKE_KEY, n, m, FAKE_OUT)       # about 20 ms
        waiting = s.submit(a, FAKE_KEY, n, m, FAKE_OUT)
        s.wait(running)
        s.wait(waiting)
        st = s.stats()
        assert st["completed"] == 4 and st["failed"] == 0
        assert st["spectra_built"] == 2 and st["spectra_evicted"] == 0 and st["spectra_resident"] == 2
        assert st["peak_bytes_in_flight"] <= budget
        assert st["bytes_in_flight"] == st["spectrum_bytes"] == 2 * u


def test_cancel_a_queued_request():
    with pa.Server(8 << 20, max_inflight=1, executor=pa.EXEC_SIMULATED, sim_bits_per_us=1.0) as s:
        sid = s.register_seed(FAKE_SEED, 5_000_000)
        first = s.submit(sid, FAKE_KEY, 100_000, 10, FAKE_OUT)     # runs for about 0.1 s
        queued = [s.submit(sid, FAKE_KEY, 100_000, 10, FAKE_OUT) for _ in range(3)]
        import time
        time.sleep(0.02)
        with pytest.raises(pa.PAError) as e:
            s.cancel(first)                                         # already on the device
        assert e.value.status == pa.PA_ERR_BUSY
        s.cancel(queued[1])
        assert s.poll(queued[1])
        with pytest.raises(pa.PAError) as e:
            s.wait(queued[1])
        assert e.value.status == pa.PA_ERR_CANCELLED
        with pytest.raises(pa.PAError) as e:
            s.cancel(queued[1])                                     # already complete
        assert e.value.status == pa.PA_ERR_INVALID_ARG
        s.drain()
        st = s.stats()
        assert st["cancelled"] == 1 and st["completed"] == 3 and st["submitted"] == 4
        for t in (first, queued[0], queued[2]):
            s.wait(t)


def test_seeds_registered_while_requests_run():
    import threading
    with pa.Server(256 << 20, max_inflight=16, executor=pa.EXEC_SIMULATED, sim_bits_per_us=5e4) as s:
        sids = [s.register_seed(FAKE_SEED, 3_000_000)]
        errors = []

        def register_more():
            try:
                for i in range(200):
                    sids.append(s.register_seed(FAKE_SEED + 0x100 * (i + 1), 3_000_000))
            except Exception as exc:  # surfaced below
                errors.append(exc)

        th = threading.Thread(target=register_more)
        th.start()
        tickets = []
        for i in range(400):
            sid = sids[i % len(sids)]
            n = 100_000 + 7_919 * (i % 50)
            tickets.append(s.submit(sid, FAKE_KEY, n, n // 4, FAKE_OUT))
        th.join()
        s.drain()
        assert not errors
        st = s.stats()
        assert st["completed"] == 400 and st["failed"] == 0 and len(sids) == 201
        assert st["peak_bytes_in_flight"] <= st["budget_bytes"]


def test_budget_from_environment(monkeypatch):
    monkeypatch.setenv("PA_HBM_BUDGET", "48M")
    with pa.Server(0, executor=pa.EXEC_SIMULATED) as s:
        assert s.stats()["budget_bytes"] == 48 << 20
    monkeypatch.setenv("PA_HBM_BUDGET", "lots")
    with pytest.raises(pa.PAError):
        pa.Server(0, executor=pa.EXEC_SIMULATED)
    monkeypatch.delenv("PA_HBM_BUDGET")
    with pa.Server(0, executor=pa.EXEC_SIMULATED) as s:
        assert s.stats()["budget_bytes"] == 16 << 30


def test_executor_failures_fail_only_their_requests():
    # the simulated executor fails every 5th ticket: those requests complete
    # with PA_ERR_DEVICE, the others as usual; a drain reports the failure
    # once, and the server keeps serving (no sticky error)
    with pa.Server(64 << 20, max_inflight=4, executor=pa.EXEC_SIMULATED, sim_bits_per_us=1e6,
                   sim_fail_every=5) as s:
        sid = s.register_seed(FAKE_SEED, 2_000_000)
        tickets = [s.submit(sid, FAKE_KEY, 300_000, 60_000, FAKE_OUT) for _ in range(23)]
        with pytest.raises(pa.PAError) as e:
            s.drain()
        assert e.value.status == pa.PA_ERR_DEVICE
        for t in tickets:
            assert s.poll(t)
            if t % 5 == 0:
                with pytest.raises(pa.PAError) as e:
                    s.wait(t)
                assert e.value.status == pa.PA_ERR_DEVICE
            else:
                s.wait(t)
        st = s.stats()
        assert st["failed"] == sum(1 for t in tickets if t % 5 == 0) and st["completed"] == 23
        assert st["inflight"] == 0 and st["bytes_in_flight"] == st["spectrum_bytes"]
        # later work is served, and a drain with no new failure succeeds
        t = s.submit(sid, FAKE_KEY, 300_000, 60_000, FAKE_OUT)
        if t % 5:
            s.wait(t)
            s.drain()
