"""GPU parity of the accuracy metric (slim_degree_kl): the Kullback-Leibler
divergence of the degree distribution of a compressed graph from that of its
input, computed by the HIP kernels, against the oracle's float64 sum.

Bar: the two sides add the same terms in different orders, each term with a
few roundings (a quotient, log2, two products), so they may differ by about
(K + 8) * eps * sum|terms| for K nonzero bins; +infinity and 0 must match
exactly."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1912_08950_amd import graphgen as gg

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def slim(gpu):
    from paper_1912_08950_amd import slim as s
    return s


def gpu_kl(slim, ro_p, ro_q):
    import torch
    a = torch.from_numpy(np.asarray(ro_p, dtype=np.int64)).cuda()
    b = torch.from_numpy(np.asarray(ro_q, dtype=np.int64)).cuda()
    return float(slim.degree_kl(a, b).cpu().item())


def assert_kl(got, ro_p, ro_q, label=""):
    want = O.degree_kl(ro_p, ro_q)
    if math.isinf(want) or want == 0.0:
        assert got == want, label
        return
    P, Q = O.degree_distribution(ro_p), O.degree_distribution(ro_q)
    abs_sum = sum(abs(P[k] * math.log2(P[k] / Q[k])) for k in P)
    assert abs(got - want) <= (len(P) + 8) * EPS * abs_sum, (label, got, want)


def compressed(slim, g, op, p, seed):
    dg = slim.Graph.from_csr(g)
    ro, _, _ = slim.result_numpy(slim.compress(dg, op, p, seed))
    return ro


@pytest.mark.parametrize("make", [lambda: gg.er(2000, 16.0, 1), lambda: gg.rmat(14, 16, 2),
                                  lambda: gg.cycle(5000), lambda: gg.grid(40, 70)],
                         ids=["er2000", "rmat14", "cycle5000", "grid40x70"])
def test_degree_kl_of_compressions(slim, make):
    g = make()
    for op, p in ((slim.OP_TR, 0.5), (slim.OP_ES, 0.2), (slim.OP_EOTR, 0.8), (slim.OP_TR2, 0.3)):
        ro = compressed(slim, g, op, p, 7)
        assert_kl(gpu_kl(slim, g.row_off, ro), g.row_off, ro, f"{g.name} op={op}")


def test_degree_kl_special_cases(slim):
    c, pth = gg.cycle(1000), gg.path(1000)
    assert gpu_kl(slim, c.row_off, c.row_off) == 0.0
    assert_kl(gpu_kl(slim, c.row_off, pth.row_off), c.row_off, pth.row_off, "cycle||path")
    assert gpu_kl(slim, pth.row_off, c.row_off) == math.inf
    assert gpu_kl(slim, [0], [0]) == 0.0  # n = 0
    assert gpu_kl(slim, [0, 0], [0, 0]) == 0.0  # one isolated vertex
    # degrees above the LDS-counted range (a hub of degree 5000 losing edges)
    star = gg.star(6000)
    ro = compressed(slim, star, slim.OP_ES, 0.5, 3)
    assert_kl(gpu_kl(slim, star.row_off, ro), star.row_off, ro, "star")


def test_degree_kl_rmat20_reproducible(slim):
    g = gg.rmat(20, 16, 1)
    ro = compressed(slim, g, slim.OP_EOTR, 0.5, 1)
    a, b = gpu_kl(slim, g.row_off, ro), gpu_kl(slim, g.row_off, ro)
    assert a == b
    assert_kl(a, g.row_off, ro, "rmat20 eotr")


def test_degree_kl_workspace_too_small(slim):
    import torch
    a = torch.zeros(5, dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        slim.degree_kl(a, torch.zeros(6, dtype=torch.int64, device="cuda"))
    ws = torch.zeros(256, dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    rc = slim._lib.slim_degree_kl(a.data_ptr(), a.data_ptr(), 4, ws.data_ptr(), 256,
                                  out.data_ptr(), None)
    assert rc == slim.ENOMEM


# --------------------------------------------- PageRank and its divergence

def to_dev(g):
    import torch
    ro = torch.from_numpy(np.asarray(g.row_off, dtype=np.int64)).cuda()
    col = torch.from_numpy(np.asarray(g.col, dtype=np.uint32).view(np.int32)).cuda()
    return ro, col


def gpu_pr(slim, g, d=0.85, iters=20):
    ro, col = to_dev(g)
    return slim.pagerank(ro, col, d, iters).cpu().numpy()


def pr_rtol(g, iters):
    """Each step adds at most deg terms in another order than the oracle:
    relative error <= (deg + 2) eps per step, carried on with factor d < 1."""
    deg = np.diff(g.row_off)
    return max(iters, 1) * (int(deg.max(initial=0)) + 2) * EPS


PR_GRAPHS = {
    "er2000": lambda: gg.er(2000, 16.0, 1),
    "rmat14": lambda: gg.rmat(14, 16, 2),  # hubs above the per-lane row limit, isolated vertices
    "star3000": lambda: gg.star(3000),
    "complete50": lambda: gg.complete(50),
    "path7": lambda: gg.path(7),
}


@pytest.mark.parametrize("name", list(PR_GRAPHS))
@pytest.mark.parametrize("iters", [0, 1, 20, 33])
def test_pagerank_matches_oracle(slim, name, iters):
    g = PR_GRAPHS[name]()
    got, want = gpu_pr(slim, g, 0.85, iters), O.pagerank(g, 0.85, iters)
    assert np.allclose(got, want, rtol=pr_rtol(g, iters), atol=0), name


def test_pagerank_reproducible_and_damping_edges(slim):
    g = gg.rmat(13, 16, 5)
    a, b = gpu_pr(slim, g), gpu_pr(slim, g)
    assert np.array_equal(a, b)
    assert np.allclose(gpu_pr(slim, g, 0.0, 5), 1.0 / g.n, rtol=1e-15, atol=0)
    assert np.allclose(gpu_pr(slim, g, 1.0, 7), O.pagerank(g, 1.0, 7), rtol=pr_rtol(g, 7), atol=0)
    import torch
    ro, col = to_dev(g)
    with pytest.raises(slim.SlimError):
        slim.pagerank(ro, col, 1.5, 3)


def test_pagerank_kl_of_compressions(slim):
    """Table `tab:pr-KL`'s metric on synthetic graphs: the divergence of the
    PageRank distribution of each output from the input's, GPU (scores and
    sum) against the oracle (its own scores and sum)."""
    import torch
    g = gg.rmat(14, 16, 1)
    pin_d = slim.pagerank(*to_dev(g))
    pin_o = O.pagerank(g)
    dg = slim.Graph.from_csr(g)
    kls = {}
    for name, op, p in (("eo0.8", slim.OP_EOTR, 0.8), ("eo1.0", slim.OP_EOTR, 1.0),
                        ("es0.2", slim.OP_ES, 0.2), ("es0.5", slim.OP_ES, 0.5),
                        ("tr0.5", slim.OP_TR, 0.5)):
        ro, col, _ = slim.result_numpy(slim.compress(dg, op, p, 1))
        h = gg.CSR(ro, col)
        pout_d = slim.pagerank(*to_dev(h))
        got = float(slim.kl_divergence(pin_d, pout_d).cpu().item())
        want = O.kl_divergence(pin_o, O.pagerank(h))
        tol = 4 * pr_rtol(g, 20) + 4 * pr_rtol(h, 20) + 64 * EPS * abs(want)
        assert abs(got - want) <= tol, (name, got, want)
        kls[name] = got
    # more compression, larger divergence (the paper's observation)
    assert 0 < kls["es0.2"] < kls["es0.5"]


def test_kl_divergence_vectors(slim):
    import torch
    from scipy.stats import entropy
    rng = np.random.default_rng(2)
    for n in (1, 7, 256, 100003):
        p, q = rng.random(n) + 1e-6, rng.random(n) + 1e-6
        got = float(slim.kl_divergence(torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
                    .cpu().item())
        want = float(entropy(p, q, base=2))
        assert abs(got - want) <= (n + 8) * EPS * 8 * max(want, 1e-300) + 1e-15 * n, n
    z = torch.zeros(4, dtype=torch.float64, device="cuda")
    o = torch.ones(4, dtype=torch.float64, device="cuda")
    assert float(slim.kl_divergence(o, z.clone().fill_(1.0)).cpu().item()) == 0.0
    zq = o.clone()
    zq[2] = 0.0
    assert float(slim.kl_divergence(o, zq).cpu().item()) == math.inf
