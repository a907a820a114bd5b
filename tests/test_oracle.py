"""Pins of the CPU oracle against facts the paper and mathematics fix.

Nothing here compares the oracle with itself: every check is brute force on
tiny inputs, a closed form, an exact expectation, a special case with a
textbook answer, a published known-answer vector, or a number the paper
prints (Table `tab:tcv`).
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1912_08950_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ----------------------------------------------------------------- helpers

def dense(g):
    a = np.zeros((g.n, g.n), dtype=np.int64)
    for r in range(g.n):
        a[r, g.col[g.row_off[r]:g.row_off[r + 1]]] = 1
    return a


def brute_triangles(g):
    """O(n^3) enumeration of {a<b<c} with all three edges present."""
    a = dense(g)
    return {(x, y, z) for x, y, z in itertools.combinations(range(g.n), 3)
            if a[x, y] and a[x, z] and a[y, z]}


def edge_set(row_off, col):
    s = set()
    for r in range(len(row_off) - 1):
        for c in col[row_off[r]:row_off[r + 1]]:
            s.add((r, int(c)))
    return s


def undirected(row_off, col):
    return {(r, c) for (r, c) in edge_set(row_off, col) if r < c}


def is_valid_csr(n, row_off, col):
    g = gg.CSR(np.asarray(row_off, dtype=np.int64), np.asarray(col, dtype=np.uint32))
    return len(row_off) == n + 1 and O.validate(g) == 0


def trace_triangles(row_off, col, n):
    """Triangle count of a CSR from trace(A^3)/6 (dense numpy)."""
    g = gg.CSR(np.asarray(row_off), np.asarray(col))
    a = dense(g).astype(np.float64)
    return int(round(np.trace(a @ a @ a) / 6.0))


CFG1 = dict(n=2000, d=16.0, seed=1)


@pytest.fixture(scope="module")
def cfg1():
    return gg.er(CFG1["n"], CFG1["d"], CFG1["seed"])


# ------------------------------------------------------------ Philox KAT

def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert O.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_threshold_endpoints():
    assert O.threshold(0.0) == 0
    assert O.threshold(1.0) == 2**32
    assert O.threshold(0.5) == 2**31
    assert O.threshold(0.25) == 2**30
    for bad in (-0.1, 1.5, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            O.threshold(bad)


# ------------------------------------------------------- triangle listing

@pytest.mark.parametrize("n,q,seed", [(12, 0.5, 1), (25, 0.3, 2), (40, 0.2, 3), (40, 0.6, 4),
                                      (30, 0.9, 5)])
def test_listing_matches_brute_force(n, q, seed):
    g = gg.er(n, q * (n - 1), seed)
    got = {tuple(int(x) for x in t) for t in O.list_triangles(g)}
    assert len(got) == len(O.list_triangles(g))  # each triangle exactly once
    assert got == brute_triangles(g)


@pytest.mark.parametrize("n", range(3, 13))
def test_complete_graph_triangles(n):
    g = gg.complete(n)
    assert len(O.list_triangles(g)) == math.comb(n, 3)


def test_k4_small_case():
    g = gg.complete(4)
    _, _, st = O.triangle_reduce(g, 0.0, 1)
    assert st["T"] == 4 and st["m_in"] == 6


@pytest.mark.parametrize("g", [gg.path(50), gg.star(40), gg.grid(7, 9), gg.complete_bipartite(6, 9),
                               gg.cycle(20), gg.cycle(4), gg.empty(5)], ids=lambda g: g.name)
@pytest.mark.parametrize("p", [0.0, 0.5, 1.0])
def test_triangle_free_families_unchanged(g, p):
    ro, col, st = O.triangle_reduce(g, p, 7)
    assert st["T"] == 0 and st["selected"] == 0 and st["deleted"] == 0
    assert np.array_equal(ro, g.row_off) and np.array_equal(col, g.col)


def test_cycle_c3_is_a_triangle():
    assert len(O.list_triangles(gg.cycle(3))) == 1


def test_per_vertex_counts_sum_to_3T(cfg1):
    """Triangles per vertex (the Table `tab:tcv` quantity, summed) = 3T."""
    tris = O.list_triangles(cfg1)
    per_vertex = np.bincount(tris.ravel(), minlength=cfg1.n)
    assert per_vertex.sum() == 3 * len(tris)
    a = dense(cfg1).astype(np.float64)
    a2 = a @ a
    assert np.array_equal(per_vertex, (np.sum(a2 * a, axis=1) / 2).round().astype(np.int64))


# ------------------------------------------------ G(n,q) triangle counts

def _er_T_mean_var(n, q):
    c3 = math.comb(n, 3)
    mean = c3 * q**3
    var = c3 * (q**3 - q**6) + 3 * c3 * (n - 3) * (q**5 - q**6)
    return mean, var


def test_gnq_expected_triangles(cfg1):
    """E[T] = C(n,3) q^3 for G(n,q); 682.67 for n=2000, q=16/1999."""
    n, q = CFG1["n"], CFG1["d"] / (CFG1["n"] - 1)
    mean, var = _er_T_mean_var(n, q)
    assert abs(mean - 682.67) < 0.01
    t1 = len(O.list_triangles(cfg1))
    assert abs(t1 - mean) < 4 * math.sqrt(var)
    ts = [len(O.list_triangles(gg.er(n, CFG1["d"], s))) for s in range(100, 200)]
    assert abs(np.mean(ts) - mean) < 4 * math.sqrt(var / len(ts))
    assert 0.5 * var < np.var(ts) < 2.0 * var


# ------------------------------------------------ Triangle p-1-Reduction

def test_tr_p0_is_identity(cfg1):
    ro, col, st = O.triangle_reduce(cfg1, 0.0, 3)
    assert st["selected"] == 0 and st["deleted"] == 0
    assert np.array_equal(ro, cfg1.row_off) and np.array_equal(col, cfg1.col)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tr_p1_output_triangle_free(cfg1, seed):
    """p = 1 reduces every input triangle, so none survives; the output has
    no triangle at all because it is a subgraph of the input."""
    ro, col, st = O.triangle_reduce(cfg1, 1.0, seed)
    assert st["selected"] == st["T"]
    assert trace_triangles(ro, col, cfg1.n) == 0


def test_k3_p1_deletes_exactly_one_edge():
    g = gg.complete(3)
    hits = np.zeros(3, dtype=np.int64)
    edges = [(0, 1), (0, 2), (1, 2)]
    for seed in range(3000):
        ro, col, st = O.triangle_reduce(g, 1.0, seed)
        assert st["T"] == 1 and st["selected"] == 1 and st["deleted"] == 1 and st["m_out"] == 2
        missing = set(edges) - undirected(ro, col)
        assert len(missing) == 1
        hits[edges.index(missing.pop())] += 1
    # rand(triangle) is uniform over the three edges: chi-square, 2 dof
    chi2 = float(np.sum((hits - 1000.0) ** 2 / 1000.0))
    assert chi2 < 13.8  # p = 0.001


@pytest.mark.parametrize("p", [0.2, 0.5, 0.8])
def test_tr_invariants(cfg1, p):
    ro, col, st = O.triangle_reduce(cfg1, p, 11)
    assert is_valid_csr(cfg1.n, ro, col)  # symmetric, sorted, same n
    e_in = undirected(cfg1.row_off, cfg1.col)
    e_out = undirected(ro, col)
    d = e_in - e_out
    assert e_out <= e_in
    assert len(d) == st["deleted"] <= st["selected"] <= st["T"]
    assert st["m_out"] == st["m_in"] - st["deleted"] == len(e_out)
    in_tri = set()
    for a, b, c in O.list_triangles(cfg1):
        in_tri |= {(int(a), int(b)), (int(a), int(c)), (int(b), int(c))}
    assert d <= in_tri  # every deleted edge lies in some input triangle


def test_tr_selected_is_binomial(cfg1):
    """Each triangle is selected independently with probability p."""
    for p in (0.1, 0.5, 0.9):
        zs = []
        for seed in range(20):
            _, _, st = O.triangle_reduce(cfg1, p, 1000 + seed)
            t = st["T"]
            zs.append((st["selected"] - p * t) / math.sqrt(t * p * (1 - p)))
        z = np.sum(zs) / math.sqrt(len(zs))
        assert abs(z) < 4.0, (p, z)


def test_tr_expected_deletions_exact():
    """E[|D|] = sum_e 1 - (1 - p/3)^{t_e}; t_e from dense A^2 (numpy)."""
    g = gg.er(300, 60.0, 5)  # ~ 9k triangles, overlapping heavily
    a = dense(g).astype(np.float64)
    te = (a @ a)[np.triu_indices(g.n, 1)][a[np.triu_indices(g.n, 1)] > 0]
    for p in (0.3, 0.7):
        expect = float(np.sum(1.0 - (1.0 - p / 3.0) ** te))
        var_ub = float(np.sum((1.0 - p / 3.0) ** te * (1.0 - (1.0 - p / 3.0) ** te)))
        ds = [O.triangle_reduce(g, p, s)[2]["deleted"] for s in range(40)]
        # deletions of different edges are not independent; allow a wide band
        assert abs(np.mean(ds) - expect) < 6 * math.sqrt(3 * var_ub / len(ds)) + 1, (p, expect)
        # "m - pT" (Table `tab:theory-schemes`) only bounds it: |D| <= pT on average
        t = O.triangle_reduce(g, p, 0)[2]["T"]
        assert expect <= p * t


def test_tr_edge_disjoint_triangles_m_minus_pT():
    """With edge-disjoint triangles E[|D|] = pT exactly (the m - pT entry)."""
    g = gg.friendship(400)
    p = 0.5
    ds = [O.triangle_reduce(g, p, s)[2]["deleted"] for s in range(50)]
    mean = np.mean(ds)
    assert abs(mean - p * 400) < 4 * math.sqrt(400 * p * (1 - p) / 50)


def test_tr_direction_matches_table_tcv(cfg1):
    """Table `tab:tcv`: 0.9-1-TR keeps fewer triangles than 0.2-1-TR on every
    graph; the oracle must show the same direction (p = reduction prob.)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "tcv_triangles_per_vertex.txt"))
            if l.strip() and not l.startswith("#")]
    assert all(float(r[3]) < float(r[2]) < float(r[1]) for r in rows)
    g = gg.er(400, 40.0, 3)
    t_after = {}
    for p in (0.2, 0.9):
        ro, col, _ = O.triangle_reduce(g, p, 9)
        t_after[p] = trace_triangles(ro, col, g.n)
    assert t_after[0.9] < t_after[0.2] < len(O.list_triangles(g))


# ----------------------------------------------------- uniform sampling

def test_es_direction_matches_table_tcv():
    """Table `tab:tcv`: uniform sampling at p keeps a (1-p)^3 share of the
    triangles (e.g. s-you 11.38 * 0.2^3 = 0.091).  The table is reproduced
    to within its own noise, and the oracle's ratio on a triangle-rich graph
    matches the table's ratio for each p."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "tcv_triangles_per_vertex.txt"))
            if l.strip() and not l.startswith("#")]
    cols = {0.8: 4, 0.5: 5, 0.2: 6}
    g = gg.er(300, 90.0, 4)
    t0 = trace_triangles(g.row_off, g.col, g.n)
    for p, ci in cols.items():
        table_ratio = float(np.median([float(r[ci]) / float(r[1]) for r in rows]))
        assert abs(table_ratio - (1 - p) ** 3) < 0.05 * (1 - p) ** 3
        ratios = []
        for s in range(4):
            ro, col, _ = O.edge_sample(g, p, 50 + s)
            ratios.append(trace_triangles(ro, col, g.n) / t0)
        assert abs(np.mean(ratios) - table_ratio) < 0.1 * table_ratio, (p, ratios, table_ratio)


def test_es_deleted_is_binomial(cfg1):
    m = cfg1.m
    for p in (0.1, 0.5, 0.9):
        zs = []
        for seed in range(10):
            ro, col, st = O.edge_sample(cfg1, p, seed)
            assert st["m_out"] == m - st["deleted"] == len(col) // 2
            zs.append((st["deleted"] - p * m) / math.sqrt(m * p * (1 - p)))
        assert abs(np.sum(zs) / math.sqrt(len(zs))) < 4.0


def test_es_symmetric_and_endpoints(cfg1):
    ro, col, st = O.edge_sample(cfg1, 0.5, 3)
    assert is_valid_csr(cfg1.n, ro, col)
    ro0, col0, _ = O.edge_sample(cfg1, 0.0, 3)
    assert np.array_equal(ro0, cfg1.row_off) and np.array_equal(col0, cfg1.col)
    ro1, col1, st1 = O.edge_sample(cfg1, 1.0, 3)
    assert len(col1) == 0 and st1["deleted"] == cfg1.m and np.all(ro1 == 0)


def test_es_decisions_match_definition():
    """Edge by edge on a small graph: {a<b} is deleted iff Philox(a,b,0,1)
    word 0 < floor(p 2^32), and both CSR copies follow that one decision
    (section 4.2.2 kernel random_uniform with p the deletion probability)."""
    g = gg.er(300, 12.0, 5)
    for p, seed in ((0.5, 91), (0.2, 2**33 + 5), (0.9, 4)):
        ro, col, st = O.edge_sample(g, p, seed)
        kept = edge_set(ro, col)
        key = (seed & 0xFFFFFFFF, seed >> 32)
        thr = O.threshold(p)
        gone = 0
        for a, b in undirected(g.row_off, g.col):
            deleted = O.philox4x32_10((a, b, 0, 1), key)[0] < thr
            gone += deleted
            assert ((a, b) in kept) == (not deleted) and ((b, a) in kept) == (not deleted)
        assert st["deleted"] == gone and st["m_out"] == g.m - gone


# ------------------------------------------------- input-contract checker

def _csr(ro, col):
    return gg.CSR(np.asarray(ro, dtype=np.int64), np.asarray(col, dtype=np.uint32))


# a triangle 0-1-2 plus the edge 2-3, in a valid symmetric sorted CSR
_VALID_RO = [0, 2, 4, 7, 8]
_VALID_COL = [1, 2, 0, 2, 0, 1, 3, 2]


@pytest.mark.parametrize("name,ro,col,code", [
    ("offsets not starting at 0", [1, 2, 4, 7, 8], _VALID_COL, -2),
    ("non-monotone offsets", [0, 2, 1, 7, 8], _VALID_COL, -3),
    ("id >= n", [0, 2, 4, 7, 8], [1, 2, 0, 2, 0, 1, 4, 2], -4),
    ("self-loop", [0, 2, 4, 7, 8], [0, 2, 0, 2, 0, 1, 3, 2], -5),
    ("unsorted row", [0, 2, 4, 7, 8], [2, 1, 0, 2, 0, 1, 3, 2], -6),
    ("duplicate in a row", [0, 2, 4, 7, 8], [1, 1, 0, 2, 0, 1, 3, 2], -6),
    ("missing reverse copy", [0, 2, 4, 7, 7], [1, 2, 0, 2, 0, 1, 3], -7),
    ("odd entry count", [0, 2, 4, 6, 7], [1, 2, 0, 2, 0, 1, 2], -7),
])
def test_validate_rejects_each_broken_contract(name, ro, col, code):
    """The input contract (a simple undirected graph as a symmetric CSR with
    strictly increasing rows): each broken clause gets its own nonzero code,
    while the valid graph next to them passes."""
    assert O.validate(_csr(_VALID_RO, _VALID_COL)) == 0
    assert O.validate(_csr(ro, col)) == code, name


def test_validate_accepts_valid_families(cfg1):
    for g in (cfg1, gg.complete(7), gg.empty(5), gg.star(9), gg.rmat(10, 8, 3)):
        assert O.validate(g) == 0


# ------------------------------------------------- local per-row oracle

@pytest.mark.parametrize("p,seed", [(0.5, 1), (0.2, 2), (1.0, 3)])
def test_tr_rows_match_definition_on_every_row(p, seed):
    """The per-row oracle (per-edge merge of full rows) gives the same rows
    as the whole-graph oracle (forward listing)."""
    g = gg.rmat(10, 8, 3)
    ro, col, _ = O.triangle_reduce(g, p, seed)
    rows = np.arange(g.n, dtype=np.uint32)
    got = O.tr_rows(g, p, seed, rows)
    for r in range(g.n):
        assert np.array_equal(got[r], col[ro[r]:ro[r + 1]]), r


def test_edge_triangle_counts_sum(cfg1):
    t = O.edge_triangle_counts(cfg1)
    assert int(t.sum()) == 6 * len(O.list_triangles(cfg1))
    a = dense(cfg1)
    a2 = a @ a
    rows = np.repeat(np.arange(cfg1.n), np.diff(cfg1.row_off))
    assert np.array_equal(t, a2[rows, cfg1.col.astype(np.int64)])


def test_oracle_rejects_bad_p(cfg1):
    for bad in (-0.01, 1.01, float("nan")):
        with pytest.raises(ValueError):
            O.triangle_reduce(cfg1, bad, 1)
        with pytest.raises(ValueError):
            O.edge_sample(cfg1, bad, 1)


def test_determinism(cfg1):
    a = O.triangle_reduce(cfg1, 0.5, 42)
    b = O.triangle_reduce(cfg1, 0.5, 42)
    c = O.triangle_reduce(cfg1, 0.5, 43)
    assert np.array_equal(a[1], b[1]) and a[2] == b[2]
    assert not np.array_equal(a[1], c[1])


# ------------------------------- Triangle p-2 and Min-Count p-1 variants

def brute_reduce_x(g, p, seed, variant):
    """The variants written out on tiny graphs with sets: O(n^3) triangles,
    per-edge counts from the triangle list, selection and edge choice from
    the Philox words (Philox itself is pinned by the known-answer vectors)."""
    thr = O.threshold(p)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    tris = sorted(brute_triangles(g))
    count = {}
    for x, y, z in tris:
        for e in ((x, y), (x, z), (y, z)):
            count[e] = count.get(e, 0) + 1
    dele, sel = set(), 0
    for x, y, z in tris:
        w = O.philox4x32_10((x, y, z, 0), key)
        if w[0] >= thr:
            continue
        sel += 1
        edges = [(x, y), (x, z), (y, z)]
        if variant == 3:
            tmin = min(count[e] for e in edges)
            tied = [e for e in edges if count[e] == tmin]
            dele.add(tied[(w[1] * len(tied)) >> 32])
        else:
            k = (w[1] * 3) >> 32
            dele |= {e for i, e in enumerate(edges) if (i != k) == (variant == 2)}
    keep = undirected(g.row_off, g.col) - dele
    return keep, len(tris), sel, len(dele)


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("n,q,seed", [(9, 0.6, 1), (12, 0.5, 2), (14, 0.45, 3), (10, 0.8, 4)])
def test_reduce_x_matches_brute_force(variant, n, q, seed):
    g = gg.er(n, q * (n - 1), seed)
    for p, s in ((1.0, 7), (0.5, 8), (0.7, 2**40 + 3)):
        ro, col, st = O.triangle_reduce_x(g, p, s, variant)
        keep, t, sel, nd = brute_reduce_x(g, p, s, variant)
        assert undirected(ro, col) == keep and is_valid_csr(g.n, ro, col)
        assert (st["T"], st["selected"], st["deleted"]) == (t, sel, nd)


def test_reduce_x_variant1_is_p1(cfg1):
    for p, s in ((0.5, 1), (0.2, 9), (1.0, 3)):
        a, b = O.triangle_reduce(cfg1, p, s), O.triangle_reduce_x(cfg1, p, s, 1)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_p2_and_p1_split_a_triangle():
    """On K3 with p = 1 the same draw deletes edge k under p-1 and the other
    two under p-2: together every edge, never one twice."""
    g = gg.complete(3)
    full = undirected(g.row_off, g.col)
    for s in range(50):
        r1, c1, _ = O.triangle_reduce_x(g, 1.0, s, 1)
        r2, c2, st2 = O.triangle_reduce_x(g, 1.0, s, 2)
        d1, d2 = full - undirected(r1, c1), full - undirected(r2, c2)
        assert len(d1) == 1 and len(d2) == 2 and not (d1 & d2) and (d1 | d2) == full
        assert st2["m_out"] == 1


def test_p2_kept_edge_is_uniform():
    g = gg.complete(3)
    counts = {}
    for s in range(600):
        ro, col, _ = O.triangle_reduce_x(g, 1.0, s, 2)
        e = next(iter(undirected(ro, col)))
        counts[e] = counts.get(e, 0) + 1
    chi2 = sum((c - 200) ** 2 / 200 for c in counts.values())
    assert len(counts) == 3 and chi2 < 16.3  # chi-square, 2 dof, p ~ 3e-4


def test_p2_edge_disjoint_triangles():
    """Friendship graph F_k (k edge-disjoint triangles): p-2 deletes exactly
    two edges per selected triangle; p = 1 keeps one edge of each."""
    g = gg.friendship(200)
    for s in range(5):
        _, _, st = O.triangle_reduce_x(g, 0.6, s, 2)
        assert st["deleted"] == 2 * st["selected"]
    assert O.triangle_reduce_x(g, 1.0, 1, 2)[2]["m_out"] == 200


def test_p2_expected_deletions_exact():
    """E[|D|] = sum_e 1 - (1 - 2p/3)^{t_e} for p-2 (t_e from dense A^2)."""
    g = gg.er(300, 60.0, 5)
    a = dense(g).astype(np.float64)
    te = (a @ a)[np.triu_indices(g.n, 1)][a[np.triu_indices(g.n, 1)] > 0]
    for p in (0.2, 0.5):
        expect = float(np.sum(1.0 - (1.0 - 2 * p / 3.0) ** te))
        var_ub = float(np.sum((1.0 - 2 * p / 3.0) ** te * (1.0 - (1.0 - 2 * p / 3.0) ** te)))
        ds = [O.triangle_reduce_x(g, p, s, 2)[2]["deleted"] for s in range(40)]
        assert abs(np.mean(ds) - expect) < 6 * math.sqrt(3 * var_ub / len(ds)) + 1, (p, expect)


@pytest.mark.parametrize("g", [gg.friendship(150), gg.complete(4), gg.complete(9)],
                         ids=["friendship150", "K4", "K9"])
def test_min_count_equals_p1_when_counts_are_equal(g):
    """Every edge in the same number of triangles: all three tie, the uniform
    tie-break picks index floor(x1*3/2^32) -- exactly the p-1 choice."""
    for p, s in ((0.5, 1), (1.0, 2), (0.3, 3)):
        a, b = O.triangle_reduce(g, p, s), O.triangle_reduce_x(g, p, s, 3)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_min_count_diamond_keeps_the_shared_edge():
    """Two triangles {0,1,2}, {1,2,3} share {1,2} (in 2 triangles; the others
    in 1): with p = 1 the shared edge always survives and each triangle loses
    one of its own edges."""
    g = gg.from_pairs(4, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)])
    for s in range(40):
        ro, col, st = O.triangle_reduce_x(g, 1.0, s, 3)
        kept = undirected(ro, col)
        assert (1, 2) in kept and st["deleted"] == 2 and len(kept) == 3


def test_min_count_deletes_only_minimal_edges(cfg1):
    """Each deleted edge has the smallest triangle count among the edges of
    some triangle containing it (counts from the per-edge merge oracle)."""
    ro_in, col_in = cfg1.row_off, cfg1.col
    t = O.edge_triangle_counts(cfg1)
    cnt = {}
    for r in range(cfg1.n):
        for j in range(ro_in[r], ro_in[r + 1]):
            cnt[(r, int(col_in[j]))] = int(t[j])
    tris = O.list_triangles(cfg1)
    ro, col, st = O.triangle_reduce_x(cfg1, 1.0, 5, 3)
    deleted = undirected(ro_in, col_in) - undirected(ro, col)
    ok = set()
    for x, y, z in tris:
        es = [(int(x), int(y)), (int(x), int(z)), (int(y), int(z))]
        tmin = min(cnt[e] for e in es)
        ok |= {e for e in es if cnt[e] == tmin}
    assert deleted and deleted <= ok
    assert st["deleted"] <= st["selected"] == st["T"]


# ------------------------------------------ Edge-Once p-1-Reduction

def brute_eo(g, p, seed):
    """Edge-Once p-1 on tiny graphs by rounds of local minima instead of the
    oracle's sorted walk: every undecided selected triangle whose priority
    (x2, a, b, c) is below that of every other undecided selected triangle
    sharing an edge with it is considered; triangles sharing an edge with a
    considered one are dropped; repeat.  With fixed priorities these rounds
    reach the same set as the greedy walk in priority order (the
    lexicographically first maximal independent set of the conflict graph),
    so agreement checks the walk by a different algorithm."""
    thr = O.threshold(p)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    tris = sorted(brute_triangles(g))
    pri, kk = {}, {}
    for t in tris:
        w = O.philox4x32_10((*t, 0), key)
        if w[0] < thr:
            pri[t] = (w[2], t)
            kk[t] = (w[1] * 3) >> 32

    def edges(t):
        x, y, z = t
        return [(x, y), (x, z), (y, z)]

    und, taken, dele, rounds = set(pri), set(), set(), 0
    while und:
        rounds += 1
        best = {}
        for t in und:
            for e in edges(t):
                best[e] = min(best.get(e, pri[t]), pri[t])
        win = [t for t in und if all(best[e] == pri[t] for e in edges(t))]
        assert win  # the undecided triangle of lowest priority always wins
        for t in win:
            dele.add(edges(t)[kk[t]])
            taken |= set(edges(t))
        und = {t for t in und if t not in win and not (set(edges(t)) & taken)}
    keep = undirected(g.row_off, g.col) - dele
    return keep, len(tris), len(pri), len(dele), rounds


@pytest.mark.parametrize("n,q,seed", [(9, 0.6, 1), (12, 0.5, 2), (14, 0.45, 3), (10, 0.8, 4),
                                      (16, 0.7, 5)])
def test_eo_matches_rounds_of_local_minima(n, q, seed):
    g = gg.er(n, q * (n - 1), seed)
    for p, s in ((1.0, 7), (0.5, 8), (0.7, 2**40 + 3), (0.9, 11)):
        ro, col, st = O.triangle_reduce_x(g, p, s, 4)
        keep, t, sel, nd, _ = brute_eo(g, p, s)
        assert undirected(ro, col) == keep and is_valid_csr(g.n, ro, col)
        assert (st["T"], st["selected"], st["deleted"]) == (t, sel, nd)


@pytest.mark.parametrize("n,q,seed", [(12, 0.5, 2), (16, 0.7, 5), (20, 0.5, 9)])
def test_eo_bucketed_walk_matches_rounds_of_local_minima(n, q, seed):
    """The walk done in several consecutive ranges of the priority word
    (what bounds its memory on large graphs) against the same independent
    algorithm as above, for several range counts."""
    g = gg.er(n, q * (n - 1), seed)
    for p, s in ((1.0, 7), (0.6, 2**40 + 3)):
        keep, t, sel, nd, _ = brute_eo(g, p, s)
        for buckets in (1, 2, 3, 7, 64):
            ro, col, st = O.triangle_reduce_eo(g, p, s, buckets)
            assert undirected(ro, col) == keep and is_valid_csr(g.n, ro, col)
            assert (st["T"], st["selected"], st["deleted"]) == (t, sel, nd)


def test_eo_equals_p1_on_edge_disjoint_triangles():
    """Friendship graph F_k: no two triangles share an edge, so every
    selected triangle is considered and Edge-Once p-1 is plain p-1."""
    g = gg.friendship(200)
    for p, s in ((0.5, 1), (1.0, 2), (0.3, 3)):
        a, b = O.triangle_reduce(g, p, s), O.triangle_reduce_x(g, p, s, 4)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_eo_k4_deletes_one_edge_of_the_first_triangle():
    """K4 with p = 1: its four triangles pairwise share an edge, so only the
    triangle of lowest priority (Philox word 2, then ids) is considered and
    exactly its edge k goes."""
    g = gg.complete(4)
    for s in range(30):
        key = (s & 0xFFFFFFFF, s >> 32)
        ws = {t: O.philox4x32_10((*t, 0), key) for t in itertools.combinations(range(4), 3)}
        first = min(ws, key=lambda t: (ws[t][2], t))
        x, y, z = first
        gone = [(x, y), (x, z), (y, z)][(ws[first][1] * 3) >> 32]
        ro, col, st = O.triangle_reduce_x(g, 1.0, s, 4)
        assert undirected(g.row_off, g.col) - undirected(ro, col) == {gone}
        assert (st["T"], st["selected"], st["deleted"]) == (4, 4, 1)


def test_eo_p0_is_identity(cfg1):
    ro, col, st = O.triangle_reduce_x(cfg1, 0.0, 3, 4)
    assert np.array_equal(ro, cfg1.row_off) and np.array_equal(col, cfg1.col)
    assert st["selected"] == 0 and st["deleted"] == 0


@pytest.mark.parametrize("p,seed", [(1.0, 1), (0.5, 2)])
def test_eo_output_is_a_2_spanner(cfg1, p, seed):
    """Section 6.2: at most one edge goes per considered triangle and no
    edge is considered twice, so every deleted {u,v} keeps a path u-w-v of
    two surviving edges (the rest of its triangle), and at most m/3 edges go."""
    ro, col, st = O.triangle_reduce_x(cfg1, p, seed, 4)
    kept = undirected(ro, col)
    gone = undirected(cfg1.row_off, cfg1.col) - kept
    nb = {}
    for a, b in kept:
        nb.setdefault(a, set()).add(b)
        nb.setdefault(b, set()).add(a)
    assert gone and len(gone) == st["deleted"] <= st["m_in"] // 3
    for u, v in gone:
        assert nb.get(u, set()) & nb.get(v, set()), (u, v)


def test_eo_removes_no_more_than_one_edge_per_triangle_it_considers():
    """Two triangles sharing an edge (a diamond) with p = 1: only the one of
    lower priority is considered, so exactly one edge goes, never two."""
    g = gg.from_pairs(4, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)])
    for s in range(40):
        ro, col, st = O.triangle_reduce_x(g, 1.0, s, 4)
        assert st["deleted"] == 1 and len(undirected(ro, col)) == 4


def test_eo_edge_count_bound_of_table_theory():
    """The Edge-Once row of the schemes table bounds the edge count by
    m - pT/(3d) in expectation (d the maximum degree): the mean number of
    deleted edges over seeds is at least pT/(3d)."""
    g = gg.rmat(11, 8, 2)
    d = int(np.max(np.diff(g.row_off)))
    for p in (0.3, 0.8):
        sts = [O.triangle_reduce_x(g, p, s, 4)[2] for s in range(8)]
        assert np.mean([x["deleted"] for x in sts]) >= p * sts[0]["T"] / (3 * d)


# --------------------------------------------- degree-distribution KL

def test_degree_kl_closed_form():
    """P = degrees {1, 2} half each, Q = {1: 3/4, 2: 1/4}:
    D = 1/2 log2(2/3) + 1/2 log2(2) = 1 - log2(3)/2."""
    p = gg.from_pairs(4, [(0, 1), (1, 2), (2, 3), (3, 0)])  # C4: all degree 2
    p_ro = np.array([0, 1, 2, 4, 6])  # degrees 1, 1, 2, 2
    q_ro = np.array([0, 1, 2, 3, 5])  # degrees 1, 1, 1, 2
    assert O.degree_kl(p_ro, q_ro) == pytest.approx(1 - math.log2(3) / 2, rel=1e-15)
    assert O.degree_kl(p.row_off, p.row_off) == 0.0


@pytest.mark.parametrize("n", [5, 12, 1000])
def test_degree_kl_cycle_vs_path(n):
    """Cycle C_n (all degree 2) against the path P_n (two ends of degree 1):
    Q(2) = (n-2)/n, so D = log2(n/(n-2)); the reverse direction is
    infinite (degree 1 is missing from the cycle)."""
    c, pth = gg.cycle(n), gg.path(n)
    assert O.degree_kl(c.row_off, pth.row_off) == pytest.approx(math.log2(n / (n - 2)), rel=1e-13)
    assert O.degree_kl(pth.row_off, c.row_off) == float("inf")


def test_degree_kl_matches_scipy_entropy():
    """scipy.stats.entropy(P, Q, base=2) is the same divergence."""
    from scipy.stats import entropy
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = int(rng.integers(5, 300))
        dp = rng.integers(0, 7, n)
        dq = np.maximum(dp - rng.integers(0, 2, n), 0)
        dq[: 7] = np.arange(7)  # every degree of P also in Q
        ro_p = np.concatenate([[0], np.cumsum(dp)])
        ro_q = np.concatenate([[0], np.cumsum(dq)])
        K = max(dp.max(), dq.max()) + 1
        P = np.bincount(dp, minlength=K) / n
        Q = np.bincount(dq, minlength=K) / n
        assert O.degree_kl(ro_p, ro_q) == pytest.approx(float(entropy(P, Q, base=2)), rel=1e-12,
                                                        abs=1e-15)
        assert O.degree_kl(ro_p, ro_q) >= 0.0  # Gibbs' inequality


def test_degree_kl_of_sampled_cycle():
    """Uniform sampling of the cycle C_n: P is all degree 2 and Q(2) is the
    fraction of vertices that keep both edges, about (1-p)^2, so D is about
    -2 log2(1-p) and grows with p (as Table `tab:pr-KL` shows for its
    metric: p = 0.2 below p = 0.5)."""
    g = gg.cycle(20000)
    kl = []
    for p in (0.2, 0.5):
        ro, _, _ = O.edge_sample(g, p, 3)
        kl.append(O.degree_kl(g.row_off, ro))
        assert kl[-1] == pytest.approx(-2 * math.log2(1 - p), abs=0.05)
    assert 0 < kl[0] < kl[1]


# ------------------------------------------------- spectral sparsification

def _pe(g, a, b, ups):
    da = g.row_off[a + 1] - g.row_off[a]
    db = g.row_off[b + 1] - g.row_off[b]
    return min(1.0, ups / float(min(da, db)))


def test_spectral_keeps_everything_when_upsilon_reaches_degrees(cfg1):
    """upsilon >= every degree: p_uv = 1 for all edges, weights exactly 1."""
    dmax = int(np.diff(cfg1.row_off).max())
    ro, col, w, st = O.spectral_sparsify(cfg1, float(dmax), 3)
    assert np.array_equal(ro, cfg1.row_off) and np.array_equal(col, cfg1.col)
    assert np.all(w == 1.0) and st["deleted"] == 0


def test_spectral_zero_upsilon_deletes_everything(cfg1):
    ro, col, w, st = O.spectral_sparsify(cfg1, 0.0, 3)
    assert ro[-1] == 0 and st["m_out"] == 0 and st["deleted"] == cfg1.m


def test_spectral_regular_graph_is_uniform_sampling():
    """On a cycle (all degrees 2) with upsilon = 1, p_uv = 1/2 for every edge:
    deletions ~ Bin(m, 1/2), every kept weight is exactly 2."""
    g = gg.cycle(4000)
    zs = []
    for s in range(20):
        ro, col, w, st = O.spectral_sparsify(g, 1.0, s)
        assert np.all(w == 2.0)
        zs.append((st["deleted"] - 2000) / math.sqrt(4000 * 0.25))
    assert abs(np.sum(zs) / math.sqrt(len(zs))) < 4.0


def test_spectral_star_keeps_leaf_edges():
    """Star: every edge has a degree-1 end, so p_uv = min(1, upsilon) = 1 for
    upsilon >= 1 -- the scheme never disconnects a leaf."""
    g = gg.star(500)
    ro, col, w, st = O.spectral_sparsify(g, 1.0, 9)
    assert st["deleted"] == 0 and np.all(w == 1.0)


def test_spectral_decisions_match_definition(cfg1):
    """Edge by edge on a small graph: kept iff Philox(u,v,0,2) word 0 <
    floor(p_uv 2^32), weight (float)(1/p_uv), both copies alike."""
    g = gg.er(300, 12.0, 4)
    ups = 4.5
    ro, col, w, st = O.spectral_sparsify(g, ups, 77)
    kept = {}
    for r in range(g.n):
        for k in range(ro[r], ro[r + 1]):
            kept[(r, int(col[k]))] = float(w[k])
    key = (77, 0)
    for a, b in undirected(g.row_off, g.col):
        pe = _pe(g, a, b, ups)
        thr = O.threshold(pe)
        x = O.philox4x32_10((a, b, 0, 2), key)
        stays = x[0] < thr
        assert ((a, b) in kept) == stays and ((b, a) in kept) == stays
        if stays:
            assert kept[(a, b)] == float(np.float32(1.0 / pe)) == kept[(b, a)]


def test_spectral_weighted_edge_count_is_unbiased():
    """E[sum of kept weights] = m (each edge contributes p_uv * 1/p_uv), and
    E[edges kept] = sum p_uv."""
    g = gg.rmat(11, 8, 2)
    ups = 3.0
    pes = np.array([_pe(g, a, b, ups) for a, b in undirected(g.row_off, g.col)])
    wsum, kept = [], []
    for s in range(40):
        ro, col, w, st = O.spectral_sparsify(g, ups, s)
        wsum.append(w.sum(dtype=np.float64) / 2)
        kept.append(st["m_out"])
    var_w = float(np.sum((1 - pes) / pes))
    var_k = float(np.sum(pes * (1 - pes)))
    assert abs(np.mean(wsum) - g.m) < 5 * math.sqrt(var_w / 40) + 1
    assert abs(np.mean(kept) - pes.sum()) < 5 * math.sqrt(var_k / 40) + 1


def test_spectral_rejects_bad_upsilon(cfg1):
    with pytest.raises(ValueError):
        O.spectral_sparsify(cfg1, float("nan"), 1)
    with pytest.raises(ValueError):
        O.spectral_sparsify(cfg1, -1.0, 1)
