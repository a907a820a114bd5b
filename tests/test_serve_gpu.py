"""GPU tests of the server (slim_serve_*): jobs submitted concurrently, from
host or device memory, batched in whatever way the workers find them, must
each produce exactly what the single-graph call produces alone; admission
respects the HBM budget; cancel, release and the statistics behave."""
import threading
import time

import numpy as np
import pytest

from paper_1912_08950_amd import graphgen as gg
from test_parity_gpu import SMALL, assert_same, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slim(gpu):
    from paper_1912_08950_amd import slim as s
    return s


def single(slim, g, op, p, seed):
    dg = slim.Graph.from_csr(g)
    return slim.result_numpy(slim.compress(dg, op, p, seed))


def test_serve_mix_equals_alone(slim):
    """Four client threads submit a mix of graphs (host and device inputs, TR
    and ES, p and seeds varying) with random gaps; every result equals the
    single-graph call on the same job."""
    graphs = [f() for f in SMALL.values()] + gg.batch_mix(40, 11, 1000, 20000)
    ps = (0.2, 0.5, 0.8, 0.0, 1.0)
    jobs = []
    ops = (slim.OP_TR, slim.OP_TR2, slim.OP_MCTR, slim.OP_ES, slim.OP_EOTR)
    for i, g in enumerate(graphs):
        op = ops[i % 5] if i % 3 else slim.OP_TR
        jobs.append((g, op, ps[i % 5], gg.mix_seed(21, i), i % 2 == 0))
    want = [single(slim, g, op, p, seed) for g, op, p, seed, _ in jobs]
    dev_graphs = {i: slim.Graph.from_csr(j[0]) for i, j in enumerate(jobs) if j[4]}
    srv = slim.Server(64 << 30, n_streams=2)
    tickets = [None] * len(jobs)

    def client(k):
        rng = np.random.default_rng(k)
        for i in range(k, len(jobs), 4):
            g, op, p, seed, on_dev = jobs[i]
            tickets[i] = srv.submit(dev_graphs[i] if on_dev else g, op, p, seed)
            time.sleep(float(rng.uniform(0, 0.003)))

    ths = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    for i, t in enumerate(tickets):
        assert_same(srv.result_numpy(t), want[i], f"job {i} {jobs[i][0].name}")
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["queued"] == 0 and st["running"] == 0 and st["hbm_in_use"] == 0
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["batches"] >= 1 and st["hbm_peak"] <= st["hbm_budget"]
    srv.close()


def test_serve_against_oracle(slim):
    srv = slim.Server(8 << 30, n_streams=3)
    g = gg.er(2000, 16.0, 1)
    ts = [srv.submit(g, slim.OP_TR, 0.5, s) for s in range(1, 9)]
    ts += [srv.submit(g, slim.OP_ES, 0.5, s) for s in range(1, 5)]
    for k, t in enumerate(ts):
        op, seed = ("tr", k + 1) if k < 8 else ("es", k - 7)
        assert_same(srv.result_numpy(t), oracle_run(g, op, 0.5, seed))
        srv.release(t)
    srv.close()


def test_serve_budget_admission(slim):
    """A budget that holds one job at a time: jobs queue, run one by one, and
    the server never holds more than the budget; a job larger than the
    budget is refused at submit."""
    g = gg.rmat(13, 16, 3)
    probe = slim.Server(1 << 40, n_streams=1)
    t = probe.submit(g, slim.OP_TR, 0.5, 1)
    probe.wait(t)
    probe.release(t)
    one = probe.stats()["hbm_peak"]
    probe.close()
    srv = slim.Server(int(one * 1.5), n_streams=2)
    ts = [srv.submit(g, slim.OP_TR, 0.5, s) for s in range(5)]
    st = srv.stats()
    assert st["queued"] + st["running"] + st["completed"] == 5
    want = single(slim, g, slim.OP_TR, 0.5, 3)
    for s, t in enumerate(ts):
        got = srv.result_numpy(t)
        if s == 3:
            assert_same(got, want)
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == 5 and st["hbm_peak"] <= st["hbm_budget"]
    assert st["mean_batch_jobs"] == 1.0
    big = gg.rmat(15, 16, 1)
    with pytest.raises(slim.SlimError) as e:
        srv.submit(big, slim.OP_TR, 0.5, 1)
    assert e.value.code == slim.EBUDGET
    srv.close()


def test_serve_cancel_and_errors(slim):
    g = gg.rmat(12, 16, 5)
    probe = slim.Server(1 << 40, n_streams=1)
    t = probe.submit(g, slim.OP_TR, 0.5, 1)
    probe.wait(t)
    one = probe.stats()["hbm_peak"]
    probe.release(t)
    probe.close()
    srv = slim.Server(int(one * 1.2), n_streams=1)
    a = srv.submit(g, slim.OP_TR, 0.5, 1)
    b = srv.submit(g, slim.OP_TR, 0.5, 2)  # waits for a's memory
    srv.wait(a)
    cancelled = srv.cancel(b)  # queued or admitted: removable until it runs
    if not cancelled:
        srv.wait(b)
        srv.release(b)
    srv.release(a)
    with pytest.raises(slim.SlimError):
        srv.release(a)  # unknown ticket now
    with pytest.raises(slim.SlimError):
        srv.submit(g, 9, 0.5, 1)
    with pytest.raises(slim.SlimError):
        srv.submit(g, slim.OP_TR, 1.5, 1)
    c = srv.submit(g, slim.OP_ES, 0.5, 3)
    r = srv.wait(c)
    assert r.status == slim.OK and r.latency_ms >= r.queue_ms >= 0
    srv.release(c)
    srv.reset_stats()
    assert srv.stats()["completed"] == 0
    srv.close()


def test_serve_completion_queue(slim):
    """slim_serve_next returns every finished job exactly once, in completion
    order, and skips jobs released before it reached them."""
    srv = slim.Server(16 << 30, n_streams=2)
    gs = gg.batch_mix(12, 17, 1000, 5000)
    ts = [srv.submit(g, slim.OP_TR, 0.5, i) for i, g in enumerate(gs)]
    first = srv.wait(ts[0])
    assert first.status == slim.OK
    srv.release(ts[0])  # released before next() sees it
    seen = []
    while len(seen) < len(ts) - 1:
        tr = srv.next(10000)
        assert tr is not None
        t, r = tr
        assert r.status == slim.OK and t not in seen and t != ts[0]
        seen.append(t)
        srv.release(t)
    assert sorted(seen) == sorted(ts[1:])
    assert srv.next(0) is None
    srv.close()


def test_serve_scale22_job_among_small_ones(slim):
    """The serving stream's large jobs: an R-MAT scale-22 job (6.4e7 edges,
    the 1% class of the stream) submitted between small jobs of the batch
    population, host and device inputs; each result equals the single-graph
    call on the same job."""
    big = gg.rmat(22, 16, 1)
    small = gg.batch_mix(12, 51, 1000, 20000)
    jobs = [(g, (slim.OP_TR, slim.OP_ES, slim.OP_TR2)[i % 3], (0.2, 0.5, 0.8)[i % 3],
             gg.mix_seed(61, i)) for i, g in enumerate(small)]
    jobs.insert(5, (big, slim.OP_TR, 0.5, 1))
    jobs.insert(9, (big, slim.OP_TR, 0.8, 2))
    print(f"serve mix: {len(jobs)} jobs, big m={big.m}", flush=True)
    dbig = slim.Graph.from_csr(big)
    srv = slim.Server(64 << 30, n_streams=2)
    tickets = []
    for i, (g, op, p, seed) in enumerate(jobs):
        src = dbig if (g is big and i == 5) else g  # one big job from device, one from host
        tickets.append(srv.submit(src, op, p, seed))
    for i, t in enumerate(tickets):
        g, op, p, seed = jobs[i]
        got = srv.result_numpy(t)
        srv.release(t)
        want = slim.result_numpy(slim.compress(dbig if g is big else slim.Graph.from_csr(g),
                                               op, p, seed))
        assert_same(got, want, f"job {i} {g.name}")
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    srv.close()
