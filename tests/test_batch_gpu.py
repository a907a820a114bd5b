"""GPU parity of batches (slim_batch_*): every job of a batch must produce
exactly what the single-graph call produces for the same (graph, op, p,
seed) -- and so what the CPU oracle produces -- whatever the batch's mix of
sizes, operations, parameters and knobs, on first capture and on replays."""
import os

import numpy as np
import pytest

from paper_1912_08950_amd import graphgen as gg
from test_parity_gpu import SMALL, assert_same, oracle_run, oracle_run_x

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slim(gpu):
    from paper_1912_08950_amd import slim as s
    return s


def single(slim, dg, op, p, seed):
    return slim.result_numpy(slim.compress(dg, op, p, seed))


def check_batch(slim, graphs, jobs, dgs=None, oracle_idx=None, knobs=None, use_graph=True,
                runs=2):
    dgs = dgs or [slim.Graph.from_csr(g) for g in graphs]
    b = slim.Batch(dgs, jobs)
    b.set("use_graph", 1 if use_graph else 0)
    for k, v in (knobs or {}).items():
        b.set(k, v)
    want = [single(slim, dg, *job) for dg, job in zip(dgs, jobs)]
    for r in range(runs):
        b.run()
        for i, w in enumerate(want):
            assert_same(b.result_numpy(i), w, f"run {r} graph {i} {graphs[i].name} {jobs[i]}")
    for i in (oracle_idx if oracle_idx is not None else range(len(graphs))):
        op, p, seed = jobs[i]
        if op in (slim.OP_TR, slim.OP_ES):
            want_o = oracle_run(graphs[i], "tr" if op == slim.OP_TR else "es", p, seed)
        else:
            name = {slim.OP_TR2: "tr2", slim.OP_MCTR: "mctr", slim.OP_EOTR: "eotr"}[op]
            want_o = oracle_run_x(graphs[i], name, p, seed)
        assert_same(b.result_numpy(i), want_o, f"oracle graph {i}")
    return b


def test_batch_of_small_graphs_mixed_ops(slim):
    """Every small fixture graph (empty, edgeless, single edge, hubs over
    several tiles, ...) in one batch, TR and ES mixed, different p and seeds."""
    graphs = [f() for f in SMALL.values()]
    ps = (0.5, 0.0, 1.0, 0.2, 0.8)
    jobs = [(slim.OP_TR if i % 3 else slim.OP_ES, ps[i % 5], 1000 + i) for i in range(len(graphs))]
    check_batch(slim, graphs, jobs)


def test_batch_all_operations_mixed(slim):
    """TR, ES, TR2, Min-Count and Edge-Once jobs in one batch (the counting
    pass visits only the Min-Count graphs, the Edge-Once rounds only the
    Edge-Once graphs, the general kernel serves TR2 and Min-Count)."""
    graphs = [f() for f in SMALL.values()] + gg.batch_mix(12, 8, 1000, 6000)
    ops = (slim.OP_TR, slim.OP_ES, slim.OP_TR2, slim.OP_MCTR, slim.OP_EOTR)
    jobs = [(ops[i % 5], (0.5, 1.0, 0.2, 0.8)[(i // 5) % 4], gg.mix_seed(5, i))
            for i in range(len(graphs))]
    check_batch(slim, graphs, jobs)
    mc_only = [(slim.OP_MCTR, 0.5, i) for i in range(len(graphs))]
    check_batch(slim, graphs, mc_only, oracle_idx=[0, 3, len(graphs) - 1])


@pytest.mark.parametrize("use_graph,eo_rounds", [(True, 16), (True, 1), (False, 2)])
def test_batch_edge_once(slim, use_graph, eo_rounds):
    """Edge-Once jobs only, captured or direct, with the rounds that the
    capture holds (eo_rounds) too few for some graphs: the rounds past them
    run after the replay and the outputs are compacted again."""
    graphs = gg.batch_mix(10, 13, 1000, 20000) + [gg.rmat(12, 16, 9)]
    jobs = [(slim.OP_EOTR, (0.3, 0.6, 1.0)[i % 3], gg.mix_seed(9, i))
            for i in range(len(graphs))]
    check_batch(slim, graphs, jobs, knobs={"eo_rounds": eo_rounds}, use_graph=use_graph, runs=3)


def test_batch_spectral_weights(slim):
    """Spectral sparsification jobs (p carries upsilon) beside TR jobs: CSR
    and float32 weights equal the single-graph call bit for bit."""
    import torch
    from oracle import oracle as O
    graphs = gg.batch_mix(10, 21, 1000, 8000)
    jobs = [(slim.OP_SPECTRAL if i % 2 else slim.OP_TR, 2.5 if i % 2 else 0.5, i)
            for i in range(len(graphs))]
    dgs = [slim.Graph.from_csr(g) for g in graphs]
    b = slim.Batch(dgs, jobs)
    b.run()
    torch.cuda.synchronize()
    for i, (g, (op, p, seed)) in enumerate(zip(graphs, jobs)):
        ro, col, st = b.result_numpy(i)
        if op == slim.OP_SPECTRAL:
            oro, ocol, ow, ost = O.spectral_sparsify(g, p, seed)
            assert np.array_equal(ro, oro) and np.array_equal(col, ocol)
            c0 = int(b.col_base[i])
            w = b.w_all[c0:c0 + len(col)].cpu().numpy()
            assert np.array_equal(w.view(np.uint32), ow.view(np.uint32))
            assert st["deleted"] == ost["deleted"]
        else:
            assert_same((ro, col, st), oracle_run(g, "tr", p, seed))


def test_batch_same_graph_many_seeds(slim):
    g = gg.er(2000, 16.0, 1)
    dg = slim.Graph.from_csr(g)
    jobs = [(slim.OP_TR, 0.5, s) for s in range(1, 33)] + [(slim.OP_ES, 0.5, s) for s in range(1, 9)]
    check_batch(slim, [g] * len(jobs), jobs, dgs=[dg] * len(jobs), oracle_idx=[0, 7, 31, 32, 39])


def test_batch_single_graph(slim):
    g = gg.rmat(12, 16, 4)
    check_batch(slim, [g], [(slim.OP_TR, 0.5, 3)])


def test_batch_only_edgeless(slim):
    graphs = [gg.empty(1), gg.empty(7), gg.empty(4100)]
    check_batch(slim, graphs, [(slim.OP_TR, 0.5, 1), (slim.OP_ES, 0.5, 1), (slim.OP_TR, 1.0, 2)])


def test_batch_only_es(slim):
    graphs = [gg.er(3000, 10.0, 5), gg.rmat(11, 8, 2), gg.path(9)]
    check_batch(slim, graphs, [(slim.OP_ES, 0.3, 1), (slim.OP_ES, 0.7, 2), (slim.OP_ES, 1.0, 3)])


@pytest.mark.parametrize("knobs", [{"tri_tile": 256}, {"tri_tile": 512, "tri_chunk": 64},
                                   {"tri_tile": 1024, "tri_blocks_per_cu": 1},
                                   {"tri_tile": 256, "tri_blocks_per_cu": 4, "tri_chunk": 32}])
def test_batch_knobs_and_direct_launch(slim, knobs):
    graphs = gg.batch_mix(24, 3, 1000, 8000)
    jobs = [(slim.OP_TR, (0.2, 0.5, 0.8)[i % 3], gg.mix_seed(99, i)) for i in range(len(graphs))]
    check_batch(slim, graphs, jobs, knobs=knobs, oracle_idx=[0, 1, 5])
    check_batch(slim, graphs, jobs, knobs=knobs, use_graph=False, runs=1, oracle_idx=[])


def test_batch_mix_population_against_oracle(slim):
    """64 graphs of the mixed population (half G(n,q), half R-MAT, n
    log-uniform in [1e3, 2e4], average degree 4..64), p = 0.5, per-graph
    seeds: every graph against the single-graph call and the oracle."""
    graphs = gg.batch_mix(64, 1, 1000, 20000)
    jobs = [(slim.OP_TR, 0.5, gg.mix_seed(7, i)) for i in range(len(graphs))]
    check_batch(slim, graphs, jobs)


def test_batch_output_buffers_change(slim):
    """A replay into other output arrays refreshes the device table."""
    graphs = [gg.rmat(10, 8, i) for i in range(1, 5)]
    jobs = [(slim.OP_TR, 0.5, i) for i in range(4)]
    dgs = [slim.Graph.from_csr(g) for g in graphs]
    b1 = check_batch(slim, graphs, jobs, dgs=dgs, oracle_idx=[])
    want = [b1.result_numpy(i) for i in range(4)]
    import torch
    b1.row_off_all = torch.full_like(b1.row_off_all, -1)
    b1.col_all = torch.full_like(b1.col_all, -1)
    b1.stats_all = torch.zeros_like(b1.stats_all)
    rp, cp, sp = b1.row_off_all.data_ptr(), b1.col_all.data_ptr(), b1.stats_all.data_ptr()
    for i in range(4):
        b1._outs[i].row_off = rp + 8 * int(b1.ro_base[i])
        b1._outs[i].col = cp + 4 * int(b1.col_base[i])
        b1._outs[i].stats = sp + 8 * len(slim.STAT_KEYS) * i
    b1.run()
    for i in range(4):
        assert_same(b1.result_numpy(i), want[i])


def test_batch_tune_and_cache(slim, tmp_path):
    graphs = gg.batch_mix(16, 5, 1000, 10000)
    jobs = [(slim.OP_TR, 0.5, i) for i in range(len(graphs))]
    dgs = [slim.Graph.from_csr(g) for g in graphs]
    want = [single(slim, dg, *j) for dg, j in zip(dgs, jobs)]
    cache = str(tmp_path / "tune.txt")
    b = slim.Batch(dgs, jobs)
    b.tune(cache)
    for i, w in enumerate(want):
        assert_same(b.result_numpy(i), w)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and "tri_tile=" in lines[0]
    chosen = {k: b.get(k) for k in ("tri_tile", "tri_blocks_per_cu", "tri_chunk")}
    b2 = slim.Batch(dgs, jobs)
    b2.tune(cache)  # a cache hit: same knobs, no new line
    assert {k: b2.get(k) for k in chosen} == chosen
    assert len(open(cache).read().splitlines()) == 1
    for i, w in enumerate(want):
        assert_same(b2.result_numpy(i), w)


def test_batch_errors(slim):
    import ctypes
    g = slim.Graph.from_csr(gg.complete(5))
    with pytest.raises(slim.SlimError) as e:
        slim.Batch([g], [(7, 0.5, 1)])
    assert e.value.code == slim.EINVAL
    with pytest.raises(slim.SlimError) as e:
        slim.Batch([g], [(slim.OP_TR, float("nan"), 1)])
    assert e.value.code == slim.EINVAL
    b = slim.Batch([g], [(slim.OP_TR, 0.5, 1)])
    rc = slim._lib.slim_batch_run(b._h, b.ws.data_ptr(), b.ws_bytes - 1, b._outs, None)
    assert rc == slim.ENOMEM
    outs = (slim.Out * 1)(slim.Out(b._outs[0].row_off, None, None))
    rc = slim._lib.slim_batch_run(b._h, b.ws.data_ptr(), b.ws_bytes, outs, None)
    assert rc == slim.EINVAL
    with pytest.raises(slim.SlimError):
        b.set("tri_tile", 384)
    with pytest.raises(slim.SlimError):
        b.set("use_graph", 2)
    assert ctypes is not None and os is not None and np is not None


def test_batch_union_beyond_2_31_edges(slim):
    """One R-MAT s20 graph batched 134 times: the union has m = 2.15e9 > 2^31
    edges, so DAG positions of the last jobs exceed 2^31 (a midpoint of two
    such positions overflows 32 bits unless computed as lo + (hi-lo)/2).
    Every job equals its single-graph call; the seed-1 job equals the
    oracle's stored digest."""
    import json
    import os

    import torch
    from make_oracle_digests import csr_digest

    g = gg.rmat(20, 16, 1)
    copies = (2**31) // g.m + 6
    assert copies * g.m > 2**31
    dg = slim.Graph.from_csr(g)
    jobs = [(slim.OP_TR, 0.5, s) for s in range(1, copies + 1)]
    b = slim.Batch([dg] * copies, jobs)
    b.run()
    torch.cuda.synchronize()
    bufs = slim.Buffers(dg, slim.OP_TR)
    for i in (0, 1, copies // 2, copies - 3, copies - 2, copies - 1):
        slim.triangle_reduce(dg, 0.5, jobs[i][2], bufs)
        torch.cuda.synchronize()
        a, z = int(b.ro_base[i]), int(b.ro_base[i + 1])
        assert torch.equal(b.row_off_all[a:z], bufs.out_row_off), i
        k = int(bufs.out_row_off[-1])
        c0 = int(b.col_base[i])
        assert torch.equal(b.col_all[c0:c0 + k], bufs.out_col[:k]), i
        assert torch.equal(b.stats_all[i], bufs.stats), i
    d = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                    "oracle_digests.json")))["rmat20_tr_p0.5"]
    ro, col, st = b.result_numpy(0)
    assert csr_digest(ro, col) == d["out_sha256"] and st["triangles"] == d["stats"]["T"]
    ro, col, st = b.result_numpy(copies - 1)
    assert st["triangles"] == d["stats"]["T"]


def _oracle_many(graphs, jobs, slim, workers=8):
    """Oracle results of many jobs, in threads (the C oracle runs outside the
    GIL), in job order."""
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        op, p, seed = jobs[i]
        return oracle_run(graphs[i], "tr" if op == slim.OP_TR else "es", p, seed)

    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(one, range(len(graphs))))


def test_batch_full_size_range_against_oracle(slim):
    """The batch population over its whole size range: n log-uniform in
    [1e3, 2e5], average degree uniform in [4, 64], half G(n,q) half R-MAT,
    plus the largest corner (n near 2e5, degree near 64) of both kinds.
    Every job against the single-graph call (first run and replay) and the
    oracle."""
    graphs = (gg.batch_mix(24, 17, 1000, 200000) +
              gg.batch_mix(2, 23, 199000, 200000, 60.0, 64.0))
    print(f"batch full range: {len(graphs)} graphs, max n {max(g.n for g in graphs)}, "
          f"sum m {sum(g.m for g in graphs)}", flush=True)
    assert max(g.n for g in graphs) >= 199000
    jobs = [(slim.OP_TR if i % 5 else slim.OP_ES, 0.5, gg.mix_seed(31, i))
            for i in range(len(graphs))]
    b = check_batch(slim, graphs, jobs, oracle_idx=[])
    want = _oracle_many(graphs, jobs, slim)
    for i, w in enumerate(want):
        assert_same(b.result_numpy(i), w, f"oracle graph {i} {graphs[i].name}")


def test_batch_stats_without_output_stats(slim):
    """slim_batch_stats returns every graph's counters of the last run, also
    when no output stats pointer was given; before a run it is refused."""
    graphs = gg.batch_mix(6, 41, 1000, 5000) + [gg.empty(3)]
    jobs = [((slim.OP_TR, slim.OP_ES, slim.OP_MCTR)[i % 3], 0.5, i + 1)
            for i in range(len(graphs))]
    dgs = [slim.Graph.from_csr(g) for g in graphs]
    want = [single(slim, dg, *j)[2] for dg, j in zip(dgs, jobs)]
    b = slim.Batch(dgs, jobs)
    with pytest.raises(slim.SlimError):
        b.stats()
    for i in range(len(graphs)):
        b._outs[i].stats = None
    for _ in range(2):
        b.run()
        assert b.stats() == want


def test_batch_workspace_shared_with_other_calls(slim):
    """A batch run, then a single-graph call and another batch on the same
    workspace (each writes its own header there), then the first batch
    again: its replay must read its own per-graph table, not theirs."""
    import torch
    graphs = gg.batch_mix(8, 43, 1000, 6000)
    jobs = [(slim.OP_TR, 0.5, gg.mix_seed(3, i)) for i in range(len(graphs))]
    dgs = [slim.Graph.from_csr(g) for g in graphs]
    want = [single(slim, dg, *j) for dg, j in zip(dgs, jobs)]
    b = slim.Batch(dgs, jobs)
    other = slim.Batch(dgs[:3], [(slim.OP_ES, 0.3, 9)] * 3)
    ws_bytes = max(b.ws_bytes, other.ws_bytes, dgs[0].workspace_size(slim.OP_TR))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    b.ws, b.ws_bytes = ws, ws_bytes
    other.ws, other.ws_bytes = ws, ws_bytes
    b.run()
    for i, w in enumerate(want):
        assert_same(b.result_numpy(i), w, f"first run {i}")
    bufs = slim.Buffers(dgs[0], slim.OP_TR)
    bufs.ws, bufs.ws_bytes = ws, ws_bytes
    slim.triangle_reduce(dgs[0], 0.9, 77, bufs)
    other.run()
    torch.cuda.synchronize()
    for i in range(len(graphs)):  # poison the outputs, then replay
        a, z = int(b.ro_base[i]), int(b.ro_base[i + 1])
        b.row_off_all[a:z] = -1
    b.col_all.fill_(-1)
    b.run()
    for i, w in enumerate(want):
        assert_same(b.result_numpy(i), w, f"replay after shared use {i}")
