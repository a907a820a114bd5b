"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer work, so the bar is bit-exact: the same output CSR (offsets and
columns) and the same counters (T, selected, deleted, m_out) as the oracle
for the same (graph, p, seed).  Small and medium graphs run the oracle live;
graphs the single-threaded oracle needs minutes for are compared with the
oracle's stored output digests (tests/golden/oracle_digests.json, written by
tests/golden/make_oracle_digests.py) and on rows sampled from the per-row
oracle.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1912_08950_amd import graphgen as gg

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
from make_oracle_digests import CASES, csr_digest  # noqa: E402


@pytest.fixture(scope="module")
def slim(gpu):
    from paper_1912_08950_amd import slim as s
    return s


def gpu_run(slim, g, op, p, seed, validate=True):
    dg = slim.Graph.from_csr(g, validate=validate)
    code = {"tr": slim.OP_TR, "es": slim.OP_ES, "tr2": slim.OP_TR2, "mctr": slim.OP_MCTR,
            "eotr": slim.OP_EOTR}[op]
    return slim.result_numpy(slim.compress(dg, code, p, seed))


def oracle_run(g, op, p, seed):
    fn = O.triangle_reduce if op == "tr" else O.edge_sample
    ro, col, st = fn(g, p, seed)
    return ro, col, {"n": st["n"], "m_in": st["m_in"], "triangles": st["T"],
                     "selected": st["selected"], "deleted": st["deleted"], "m_out": st["m_out"]}


def assert_same(got, want, label=""):
    ro, col, st = got
    oro, ocol, ost = want
    assert st == ost, label
    assert np.array_equal(ro, oro), label
    assert np.array_equal(col, ocol), label


def wheel(n_rim):
    """Hub 0 joined to a path 1..n_rim: n_rim-1 triangles, one huge row."""
    pairs = [(0, i) for i in range(1, n_rim + 1)] + [(i, i + 1) for i in range(1, n_rim)]
    return gg.from_pairs(n_rim + 1, pairs, f"wheel{n_rim}")


def bipartite_plus_matching(a, b):
    """K_{a,b} plus a perfect matching on the b side: vertex out-degrees above
    2048 in the degree-ordered DAG (several LDS passes) and a*b/2 triangles."""
    pairs = [(i, a + j) for i in range(a) for j in range(b)]
    pairs += [(a + 2 * k, a + 2 * k + 1) for k in range(b // 2)]
    return gg.from_pairs(a + b, pairs, f"K{a},{b}+M")


def sort_classes(lengths=(2, 31, 32, 33, 64, 65, 128, 129, 256, 257, 512, 513, 1024, 1025,
                           2048, 2049)):
    """DAG rows of given lengths: hubs 0..H-1 on a path, each with H+1
    private leaves (so every hub outranks every other vertex), and one vertex
    per length L joined to hubs 0..L-1, whose DAG row is exactly those L
    hubs. Vertex L's triangles are its L-1 consecutive hub pairs; a mis-sorted
    row would misplace its in-edge searches and its suffix scans."""
    H = max(lengths)
    pairs = [(h, h + 1) for h in range(H - 1)]
    nxt = H
    for L in lengths:
        pairs += [(nxt, h) for h in range(L)]
        nxt += 1
    for h in range(H):
        pairs += [(h, nxt + i) for i in range(H + 1)]
        nxt += H + 1
    g = gg.from_pairs(nxt, pairs, "sort_classes")
    return g


SMALL = {
    "K3": lambda: gg.complete(3),
    "K4": lambda: gg.complete(4),
    "K40": lambda: gg.complete(40),
    "single_edge": lambda: gg.from_pairs(2, [(0, 1)]),
    "one_vertex": lambda: gg.empty(1),
    "empty5": lambda: gg.empty(5),
    "path50": lambda: gg.path(50),
    "star9000": lambda: gg.star(9000),          # triangle-free hub row over 5 tiles
    "wheel9000": lambda: wheel(9000),           # triangles through a multi-tile row
    "C2048": lambda: gg.cycle(2048),            # nnz = 4096: exactly one full tile
    "friendship700": lambda: gg.friendship(700),
    "grid30x40": lambda: gg.grid(30, 40),
    "er_sparse_isolated": lambda: gg.er(30000, 0.7, 3),  # many empty rows
    "er_cfg1": lambda: gg.er(2000, 16.0, 1),
    "er_dense": lambda: gg.er(600, 150.0, 2),
    "rmat12": lambda: gg.rmat(12, 16, 7),
    "rmat14_noperm": lambda: gg.rmat(14, 8, 3, permute=False),
    "rmat10_n700": lambda: gg.rmat(10, 8, 5, n=700),
    "K60,60+M": lambda: bipartite_plus_matching(60, 60),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("op", ["tr", "es"])
def test_small_graphs(slim, name, op):
    g = SMALL[name]()
    for p, seed in ((0.5, 1), (0.0, 2), (1.0, 3), (0.2, 4), (0.8, 5)):
        assert_same(gpu_run(slim, g, op, p, seed), oracle_run(g, op, p, seed),
                    f"{name} {op} p={p} seed={seed}")


def test_cfg1_many_seeds(slim):
    """G(2000, avg degree 16), seed 1: TR and ES at p = 0.5 over many op seeds."""
    g = gg.er(2000, 16.0, 1)
    for seed in range(1, 21):
        for op in ("tr", "es"):
            assert_same(gpu_run(slim, g, op, 0.5, seed), oracle_run(g, op, 0.5, seed),
                        f"{op} seed={seed}")


def test_seed_high_word(slim):
    g = gg.er(2000, 16.0, 1)
    for seed in (2**32, 2**63 + 12345, 2**64 - 1):
        for op in ("tr", "es"):
            assert_same(gpu_run(slim, g, op, 0.5, seed), oracle_run(g, op, 0.5, seed))


@pytest.mark.parametrize("scale", [14, 16])
def test_rmat_medium(slim, scale):
    g = gg.rmat(scale, 16, 1)
    for p in (0.2, 0.5, 0.8):
        assert_same(gpu_run(slim, g, "tr", p, 1, validate=False), oracle_run(g, "tr", p, 1),
                    f"s{scale} p={p}")


@pytest.mark.parametrize("knobs", [{"tri_chunk": 32}, {"tri_chunk": 64, "tri_blocks_per_cu": 1},
                                   {"tri_chunk": 512, "tri_blocks_per_cu": 3},
                                   {"tri_blocks_per_cu": 64}, {"tri_tile": 256},
                                   {"tri_tile": 512, "tri_chunk": 64}])
def test_schedule_independence(slim, knobs):
    """Launch shape and LDS pass size change the schedule, never the result."""
    graphs = [gg.rmat(13, 16, 2), bipartite_plus_matching(3, 300), wheel(5000), gg.complete(70)]
    want = [oracle_run(g, "tr", 0.5, 9) for g in graphs]
    old = {k: slim.tune_get(k) for k in knobs}
    try:
        for k, v in knobs.items():
            slim.tune_set(k, v)
        for g, w in zip(graphs, want):
            assert_same(gpu_run(slim, g, "tr", 0.5, 9), w, f"{g.name} {knobs}")
    finally:
        for k, v in old.items():
            slim.tune_set(k, v)


def test_buffer_reuse_and_determinism(slim):
    g = gg.rmat(12, 16, 4)
    dg = slim.Graph.from_csr(g)
    bufs = slim.Buffers(dg, slim.OP_TR)
    first = slim.result_numpy(slim.triangle_reduce(dg, 0.5, 77, bufs))
    for seed in (78, 77):
        got = slim.result_numpy(slim.triangle_reduce(dg, 0.5, seed, bufs))
        if seed == 77:
            assert_same(got, first)
    assert_same(first, oracle_run(g, "tr", 0.5, 77))


def test_invalid_inputs_rejected(slim):
    import torch
    dev = "cuda:0"

    def load(ro, col, n=None):
        ro_t = torch.tensor(ro, dtype=torch.int64, device=dev)
        col_t = torch.tensor(np.asarray(col, dtype=np.uint32).view(np.int32), device=dev)
        return slim.Graph(ro_t, col_t, validate=True)

    load([0, 1, 2], [1, 0])  # valid single edge
    bad = {
        "unsorted": ([0, 2, 3, 4], [2, 1, 0, 0]),
        "self_loop": ([0, 2, 4], [0, 1, 0, 1]),
        "asymmetric": ([0, 1, 2, 2], [1, 2]),
        "id_out_of_range": ([0, 1, 2], [1, 7]),
        "bad_offsets": ([0, 2, 1], [1, 0]),
    }
    for name, (ro, col) in bad.items():
        with pytest.raises(slim.SlimError) as e:
            load(ro, col)
        assert e.value.code == slim.EINVAL, name


def test_workspace_too_small(slim):
    import ctypes
    g = gg.er(500, 8.0, 1)
    dg = slim.Graph.from_csr(g)
    bufs = slim.Buffers(dg, slim.OP_TR)
    rc = slim._lib.slim_triangle_reduce(dg._h, 0.5, 1, bufs.ws.data_ptr(), bufs.ws_bytes - 1,
                                        bufs.out_row_off.data_ptr(), bufs.out_col.data_ptr(),
                                        None, None)
    assert rc == slim.ENOMEM
    rc = slim._lib.slim_triangle_reduce(dg._h, float("nan"), 1, bufs.ws.data_ptr(),
                                        bufs.ws_bytes, bufs.out_row_off.data_ptr(),
                                        bufs.out_col.data_ptr(), None, None)
    assert rc == slim.EINVAL
    assert ctypes is not None


# ----------------------------------------------- full-size workloads

def _digests():
    path = os.path.join(GOLDEN, "oracle_digests.json")
    return json.load(open(path)) if os.path.exists(path) else {}


def _check_digest(slim, g, name):
    d = _digests().get(name)
    if d is None:
        pytest.skip(f"no stored oracle digest for {name}")
    assert csr_digest(g.row_off, g.col) == d["graph_sha256"], "generator output changed"
    _, op, p = CASES[name]
    ro, col, st = gpu_run(slim, g, op, p, d["seed"], validate=False)
    ost = d["stats"]
    assert st["triangles"] == ost["T"] and st["selected"] == ost["selected"], name
    assert st["deleted"] == ost["deleted"] and st["m_out"] == ost["m_out"], name
    assert csr_digest(ro, col) == d["out_sha256"], name
    return ro, col, st


def _check_sampled_rows(g, ro, col, p, seed, rows):
    want = O.tr_rows(g, p, seed, rows)
    for r, w in zip(rows, want):
        assert np.array_equal(col[ro[r]:ro[r + 1]], w), r


@pytest.fixture(scope="module")
def rmat20():
    return gg.rmat(20, 16, 1)


@pytest.mark.parametrize("p", [0.2, 0.5, 0.8])
def test_rmat20_tr_full(slim, rmat20, p):
    """R-MAT scale 20 (edge factor 16), one graph per launch, p in {.2,.5,.8}."""
    ro, col, st = _check_digest(slim, rmat20, f"rmat20_tr_p{p}")
    rng = np.random.default_rng(5)
    deg = rmat20.degrees()
    rows = rng.choice(np.flatnonzero((deg > 0) & (deg < 400)), 300, replace=False)
    _check_sampled_rows(rmat20, ro, col, p, 1, rows)


@pytest.mark.parametrize("variant", ["tr2", "mctr", "eotr"])
def test_rmat20_variants_full(slim, rmat20, variant):
    """R-MAT scale 20: Triangle p-2, Min-Count p-1 and Edge-Once p-1
    Reduction against the oracle's stored digests."""
    _check_digest(slim, rmat20, f"rmat20_{variant}_p0.5")


def test_rmat20_es_full(slim, rmat20):
    assert_same(gpu_run(slim, rmat20, "es", 0.5, 1, validate=False),
                oracle_run(rmat20, "es", 0.5, 1))


@pytest.fixture(scope="module")
def rmat24():
    return gg.rmat(24, 16, 1)


def test_rmat24_tr_full(slim, rmat24):
    """R-MAT scale 24 (edge factor 16, ~0.5B CSR entries), p = 0.5, the
    benchmark workload in the benchmark's launch configuration: the whole
    output against the oracle's stored digest, and sampled rows recomputed
    by the per-row oracle."""
    ro, col, st = _check_digest(slim, rmat24, "rmat24_tr_p0.5")
    rng = np.random.default_rng(11)
    deg = rmat24.degrees()
    rows = np.concatenate([rng.choice(np.flatnonzero((deg > 0) & (deg < 200)), 200, replace=False),
                           rng.choice(np.flatnonzero((deg >= 200) & (deg < 2000)), 10,
                                      replace=False)])
    _check_sampled_rows(rmat24, ro, col, 0.5, 1, rows)


def test_rmat24_es_full(slim, rmat24):
    _check_digest(slim, rmat24, "rmat24_es_p0.5")


def test_rmat24_spectral_full(slim, rmat24):
    """R-MAT scale 24: spectral sparsification with upsilon = p m / n, the
    output CSR and every float32 weight against the oracle's stored digests."""
    import hashlib
    name = "rmat24_spectral_p0.5"
    d = _digests().get(name)
    if d is None:
        pytest.skip(f"no stored oracle digest for {name}")
    assert csr_digest(rmat24.row_off, rmat24.col) == d["graph_sha256"], "generator output changed"
    ups = 0.5 * rmat24.m / rmat24.n
    assert ups == d["upsilon"]
    dg = slim.Graph.from_csr(rmat24)
    bufs = slim.spectral_sparsify(dg, ups, d["seed"])
    ro, col, st = slim.result_numpy(bufs)
    w = slim.weights_numpy(bufs)
    assert st["deleted"] == d["stats"]["deleted"] and st["m_out"] == d["stats"]["m_out"]
    assert csr_digest(ro, col) == d["out_sha256"]
    assert hashlib.sha256(np.ascontiguousarray(w, dtype="<f4").tobytes()).hexdigest() == \
        d["weights_sha256"]


def test_rmat24_eotr_properties(slim, rmat24):
    """R-MAT scale 24, Edge-Once p-1 (the oracle's sort of 5e9 selected
    triangles does not fit in host memory, so properties that hold at any
    size): the same triangles and selections as p-1 (stored digest), at most
    m/3 deletions, output rows are subsets of the input rows, and every
    deleted edge of 300 sampled rows keeps a two-edge path (2-spanner)."""
    ref = _digests().get("rmat24_tr_p0.5")
    if ref is None:
        pytest.skip("no stored oracle digest for rmat24_tr_p0.5")
    ro, col, st = gpu_run(slim, rmat24, "eotr", 0.5, 1, validate=False)
    assert st["triangles"] == ref["stats"]["T"] and st["selected"] == ref["stats"]["selected"]
    assert st["deleted"] == st["m_in"] - st["m_out"] and 0 < st["deleted"] <= st["m_in"] // 3
    assert ro[-1] == 2 * st["m_out"]
    rng = np.random.default_rng(13)
    deg = rmat24.degrees()
    rows = rng.choice(np.flatnonzero((deg > 1) & (deg < 300)), 300, replace=False)
    n_del = 0
    for u in rows:
        a = rmat24.col[rmat24.row_off[u]:rmat24.row_off[u + 1]]
        b = col[ro[u]:ro[u + 1]]
        assert np.all(np.diff(b.astype(np.int64)) > 0) and np.all(np.isin(b, a)), u
        for v in np.setdiff1d(a, b):
            n_del += 1
            bv = col[ro[v]:ro[v + 1]]
            assert np.intersect1d(b, bv).size > 0, (u, v)
    assert n_del > 0


def test_rmat24_tr2_full(slim, rmat24):
    """R-MAT scale 24: Triangle p-2-Reduction (general kernel) against the
    oracle's stored digest."""
    _check_digest(slim, rmat24, "rmat24_tr2_p0.5")


def test_rmat24_mctr_full(slim, rmat24):
    """R-MAT scale 24: Min-Count p-1-Reduction (counting pass + selection)
    against the oracle's stored digest."""
    _check_digest(slim, rmat24, "rmat24_mctr_p0.5")


def test_rmat24_eotr_full(slim, rmat24):
    """R-MAT scale 24: Edge-Once p-1-Reduction (its parallel rounds) against
    the oracle's stored digest of the priority-order walk (taken in pieces
    of the priority range to fit host memory)."""
    _check_digest(slim, rmat24, "rmat24_eotr_p0.5")



# ------------------------------- Triangle p-2 and Min-Count p-1 variants

VARIANTS = {"tr2": 2, "mctr": 3, "eotr": 4}


def gpu_run_op(slim, g, name, p, seed, validate=False):
    op = {"tr2": slim.OP_TR2, "mctr": slim.OP_MCTR, "eotr": slim.OP_EOTR}[name]
    dg = slim.Graph.from_csr(g, validate=validate)
    return slim.result_numpy(slim.compress(dg, op, p, seed))


def oracle_run_x(g, name, p, seed):
    ro, col, st = O.triangle_reduce_x(g, p, seed, VARIANTS[name])
    return ro, col, {"n": st["n"], "m_in": st["m_in"], "triangles": st["T"],
                     "selected": st["selected"], "deleted": st["deleted"], "m_out": st["m_out"]}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("variant", list(VARIANTS))
def test_small_graphs_variants(slim, name, variant):
    g = SMALL[name]()
    for p, seed in ((0.5, 1), (0.0, 2), (1.0, 3), (0.2, 4), (0.8, 5)):
        assert_same(gpu_run_op(slim, g, variant, p, seed), oracle_run_x(g, variant, p, seed),
                    f"{name} {variant} p={p} seed={seed}")


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_variants_cfg1_and_rmat(slim, variant):
    g = gg.er(2000, 16.0, 1)
    for seed in range(1, 9):
        assert_same(gpu_run_op(slim, g, variant, 0.5, seed), oracle_run_x(g, variant, 0.5, seed))
    for scale in (14, 16):
        g = gg.rmat(scale, 16, 1)
        for p in (0.2, 0.8):
            assert_same(gpu_run_op(slim, g, variant, p, 1), oracle_run_x(g, variant, p, 1),
                        f"s{scale} {variant} p={p}")


@pytest.mark.parametrize("knobs", [{"tri_chunk": 32}, {"tri_tile": 256, "tri_blocks_per_cu": 1},
                                   {"tri_chunk": 512, "tri_blocks_per_cu": 3},
                                   {"eo_rounds": 1}, {"eo_rounds": 2, "tri_chunk": 64}])
def test_variants_schedule_independence(slim, knobs):
    graphs = [gg.rmat(13, 16, 2), bipartite_plus_matching(3, 300), wheel(5000)]
    want = {(g.name, v): oracle_run_x(g, v, 0.6, 4) for g in graphs for v in VARIANTS}
    old = {k: slim.tune_get(k) for k in knobs}
    try:
        for k, v in knobs.items():
            slim.tune_set(k, v)
        for g in graphs:
            for v in VARIANTS:
                assert_same(gpu_run_op(slim, g, v, 0.6, 4), want[(g.name, v)], f"{g.name} {v}")
    finally:
        for k, v in old.items():
            slim.tune_set(k, v)


@pytest.mark.parametrize("try_pct", [0, 100000])
def test_edge_once_list_start_and_overflow(slim, try_pct):
    """Edge-Once with the triangle list never started (0) and started as
    early as possible (100000: the second round already tries; on these
    graphs its bidders overflow the list, which is then dropped, and the
    third round lists again).  K_120 keeps 51,650 of its 168,128 selected
    triangles undecided after the first round against a list of 21,420, the
    R-MAT s16 graph 2.86e6 against 2.73e6."""
    old = slim.tune_get("eo_list_try")
    try:
        slim.tune_set("eo_list_try", try_pct)
        for g in (gg.complete(120), gg.rmat(16, 16, 1), gg.rmat(13, 16, 2)):
            assert_same(gpu_run_op(slim, g, "eotr", 0.6, 4), oracle_run_x(g, "eotr", 0.6, 4),
                        f"{g.name} eo_list_try={try_pct}")
    finally:
        slim.tune_set("eo_list_try", old)


@pytest.mark.parametrize("p", [1.0, 0.5])
def test_dag_rows_of_every_sort_class(slim, p):
    """Rows of 2 to 2049 entries cover the thread, wave-register (64 x 1 to
    64 x 32 values) and block sorts and their boundaries."""
    g = sort_classes()
    for op in ("tr",):
        assert_same(gpu_run(slim, g, op, p, 3), oracle_run(g, op, p, 3), f"sort classes {op} p={p}")
    assert_same(gpu_run_op(slim, g, "eotr", p, 3), oracle_run_x(g, "eotr", p, 3), "sort classes eotr")


def double_star(n_leaves):
    """Vertices 0 and 1 joined to each other and to every leaf 2..n+1: the n
    triangles {0,1,leaf} are all found from vertex 0's row, whose n in-edges
    (leaf, 0) each scan one item, the edge to vertex 1."""
    leaves = range(2, n_leaves + 2)
    pairs = [(0, 1)] + [(0, i) for i in leaves] + [(1, i) for i in leaves]
    return gg.from_pairs(n_leaves + 2, pairs, f"double_star{n_leaves}")


# In-edges per batch are 512 (p-1), 384 (p-2, Min-Count) and 352 (Edge-Once).
# A double star puts its n scanning in-edges in one batch run of a tile; the
# wheels' second tile holds 352, 353, 384, 385, 512 and 513 in-edges.
BATCH_EDGE_GRAPHS = ([double_star(n) for n in (351, 352, 353, 383, 384, 385, 511, 512, 513,
                                               1023, 1024, 1025)]
                     + [wheel(n) for n in (1041, 1042, 1089, 1090, 1281, 1282)])


@pytest.mark.parametrize("op", ["tr", "tr2", "mctr", "eotr"])
def test_batch_boundaries(slim, op):
    """Tiles whose in-edges fill each instantiation's batch exactly, or by one."""
    for g in BATCH_EDGE_GRAPHS:
        for p, seed in ((0.5, 1), (1.0, 2)):
            if op == "tr":
                got, want = gpu_run(slim, g, op, p, seed), oracle_run(g, op, p, seed)
            else:
                got, want = gpu_run_op(slim, g, op, p, seed), oracle_run_x(g, op, p, seed)
            assert_same(got, want, f"{g.name} {op} p={p} seed={seed}")


# ------------------------------------------------- spectral sparsification

def oracle_spectral(g, ups, seed):
    ro, col, w, st = O.spectral_sparsify(g, ups, seed)
    return (ro, col, {"n": st["n"], "m_in": st["m_in"], "triangles": 0, "selected": 0,
                      "deleted": st["deleted"], "m_out": st["m_out"]}), w


@pytest.mark.parametrize("name", list(SMALL))
def test_spectral_small_graphs(slim, name):
    """Output CSR, counters and every float32 weight bit for bit."""
    g = SMALL[name]()
    dg = slim.Graph.from_csr(g)
    for ups, seed in ((1.0, 1), (0.0, 2), (3.5, 3), (1e9, 4), (0.37, 2**40 + 5)):
        bufs = slim.spectral_sparsify(dg, ups, seed)
        want, w = oracle_spectral(g, ups, seed)
        assert_same(slim.result_numpy(bufs), want, f"{name} ups={ups}")
        assert np.array_equal(slim.weights_numpy(bufs).view(np.uint32), w.view(np.uint32))


def test_spectral_rmat20(slim, rmat20):
    """R-MAT scale 20 (~31M CSR entries, hubs of degree > 10^4): upsilon =
    p m / n with p = 0.5 (the paper's average-degree choice)."""
    ups = 0.5 * rmat20.m / rmat20.n
    dg = slim.Graph.from_csr(rmat20)
    bufs = slim.spectral_sparsify(dg, ups, 1)
    want, w = oracle_spectral(rmat20, ups, 1)
    assert_same(slim.result_numpy(bufs), want)
    assert np.array_equal(slim.weights_numpy(bufs).view(np.uint32), w.view(np.uint32))


def test_spectral_bad_upsilon(slim):
    dg = slim.Graph.from_csr(gg.complete(5))
    for bad in (float("nan"), -0.5):
        with pytest.raises(slim.SlimError) as e:
            slim.spectral_sparsify(dg, bad, 1)
        assert e.value.code == slim.EINVAL
