"""Host tests of the serving engine's scheduler (mock executor: admission,
HBM-arena accounting, FIFO order, cancellation, rejection); no device."""
import numpy as np
import pytest

from paper_2606_11402_amd import VecchiaError, _lib
from paper_2606_11402_amd.serve import Server


def pts(n, seed):
    return np.random.default_rng(seed).random((n, 3))


def wait_built(srv, ids, steps=2000):
    import time
    for _ in range(steps):
        st = srv.stats()
        if st["building"] == 0:
            return
        time.sleep(0.005)
    raise TimeoutError


def test_request_bytes_grow_with_n_and_k():
    a = Server.request_bytes(1000, 8)
    b = Server.request_bytes(2000, 8)
    c = Server.request_bytes(2000, 32)
    assert a < b < c
    # rough model: N (8 kp + 28) bytes plus the dense block
    assert abs(c - 2000 * (8 * 32 + 28)) < 2000 * 40 + 128 * 128 * 8 + 8192


def test_rejects_request_larger_than_budget():
    srv = Server(Server.request_bytes(1000, 8) + 1024, mock=True)
    with pytest.raises(VecchiaError) as e:
        srv.submit(pts(5000, 0), 8, 1, 1.0, 0.1, "logdet")
    assert e.value.code == -6
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_budget_forces_queueing_and_fifo_completion():
    one = Server.request_bytes(3000, 16)
    srv = Server(2 * one + 512, n_streams=4, graph_workers=1, mock=True)   # one worker: graphs finish in order
    ids = [srv.submit(pts(3000, i), 16, 1, 1.0, 0.1, "forward", np.full(3000, i, np.float32)) for i in range(6)]
    wait_built(srv, ids)
    srv.progress()
    st = srv.stats()
    assert st["running"] == 2 and st["queued"] == 4
    assert st["bytes_in_use"] <= st["arena_bytes"]
    order = []
    while len(order) < 6:
        srv.progress()
        while True:
            rid = srv.take()
            if not rid:
                break
            out, times = srv.result(rid)
            assert (out == ids.index(rid)).all()      # mock returns the input
            order.append(rid)
    assert order == ids          # admission is FIFO over graph-ready requests; equal mock latency
    st = srv.stats()
    assert st["bytes_in_use"] == 0 and st["completed"] == 6 and st["peak_bytes"] <= 2 * one + 512
    assert st["peak_running"] == 2          # the budget holds two requests at a time
    srv.close()


def test_cancel_queued_request():
    one = Server.request_bytes(2000, 8)
    srv = Server(one + 512, graph_workers=1, mock=True)   # one worker: a is ready (and admitted) first
    a = srv.submit(pts(2000, 1), 8, 0, 1.0, 0.2, "logdet")
    b = srv.submit(pts(2000, 2), 8, 0, 1.0, 0.2, "logdet")
    wait_built(srv, [a, b])
    srv.progress()                      # a admitted, b waits for memory
    srv.cancel(b)
    with pytest.raises(VecchiaError):
        srv.cancel(a)                   # already running
    done = srv.drain()
    assert set(done) == {a}
    assert srv.stats()["cancelled"] == 1
    srv.close()


def test_cancel_then_release_at_once_keeps_the_queues_valid():
    """A cancelled request is released right away (queued and still
    building); the scheduler must not touch it again afterwards."""
    one = Server.request_bytes(2000, 8)
    srv = Server(one + 512, graph_workers=1, mock=True)
    a = srv.submit(pts(2000, 1), 8, 0, 1.0, 0.2, "logdet")
    b = srv.submit(pts(2000, 2), 8, 0, 1.0, 0.2, "logdet")
    wait_built(srv, [a, b])
    srv.progress()                      # a admitted, b waits for memory
    srv.cancel(b)                       # Server.cancel releases it at once, while it sat in the ready queue
    c = srv.submit(pts(1900, 3), 8, 0, 1.0, 0.2, "logdet")
    srv.cancel(c)                       # still in the build queue or being built
    d = srv.submit(pts(1500, 4), 8, 0, 1.0, 0.2, "logdet")
    done = srv.drain()
    assert set(done) == {a, d}
    assert srv.stats()["cancelled"] == 2
    srv.close()


def test_mixed_sizes_never_exceed_budget():
    rng = np.random.default_rng(3)
    sizes = rng.integers(200, 4000, 40)
    budget = 3 * Server.request_bytes(4000, 32)
    srv = Server(budget, n_streams=3, mock=True)
    ids = []
    for i, n in enumerate(sizes):
        k = int(rng.choice([8, 16, 32]))
        ids.append(srv.submit(pts(int(n), 100 + i), k, 1, 1.0, 0.05, "inverse", np.zeros(int(n), np.float32)))
    done = srv.drain()
    assert len(done) == 40
    st = srv.stats()
    assert st["peak_bytes"] <= budget and st["bytes_in_use"] == 0 and st["failed"] == 0


def test_invalid_submissions():
    srv = Server(1 << 24, mock=True)
    with pytest.raises(VecchiaError):
        srv.submit(pts(100, 0), _lib.KMAX + 1, 1, 1.0, 0.1, "logdet")   # k above the compiled maximum
    with pytest.raises(VecchiaError):
        srv.submit(pts(100, 0), 8, 1, -1.0, 0.1, "logdet")          # sigma <= 0
    with pytest.raises(VecchiaError):
        srv.submit(pts(100, 0), 8, 5, 1.0, 0.1, "logdet")           # kind
    srv.close()
