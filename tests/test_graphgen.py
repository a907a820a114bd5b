"""The seeded input generators produce valid, deterministic inputs."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1912_08950_amd import graphgen as gg


@pytest.mark.parametrize("make", [lambda: gg.er(2000, 16, 1), lambda: gg.er(500, 499, 2),
                                  lambda: gg.rmat(12, 16, 1), lambda: gg.rmat(10, 8, 5, n=700),
                                  lambda: gg.rmat(11, 4, 9, permute=False)])
def test_valid_csr(make):
    g = make()
    assert O.validate(g) == 0
    assert g.row_off[0] == 0 and g.row_off[-1] == g.nnz and g.nnz % 2 == 0


def test_deterministic():
    a, b = gg.rmat(14, 16, 3), gg.rmat(14, 16, 3)
    assert np.array_equal(a.row_off, b.row_off) and np.array_equal(a.col, b.col)
    c = gg.rmat(14, 16, 4)
    assert not (a.nnz == c.nnz and np.array_equal(a.col, c.col))


def test_er_mean_degree():
    g = gg.er(20000, 16, 7)
    assert abs(g.nnz / g.n - 16) < 0.2
    k = gg.er(60, 59, 1)
    assert k.m == 60 * 59 // 2  # q = 1 gives the complete graph


def test_rmat_shape():
    g = gg.rmat(16, 16, 1)
    assert g.n == 2**16
    assert 0.8 * 16 * 2**16 < g.m <= 16 * 2**16  # duplicates and loops removed
    d = g.degrees()
    assert d.max() > 50 * d.mean()  # heavy tail


def test_rmat_reject_above_n():
    g = gg.rmat(10, 8, 5, n=700)
    assert g.n == 700 and (g.col < 700).all()


def test_batch_mix_equals_single_generators():
    """The many-graph generator returns exactly the single-graph generators'
    output for each drawn parameter set, and draws the stated population."""
    import numpy as np
    gs = gg.batch_mix(48, 4, 1000, 30000)
    for g, (kind, n, d, s, scale, samples) in zip(gs, gg.batch_mix_params(48, 4, 1000, 30000)):
        h = gg.er(n, d, s) if kind == "er" else gg.rmat(scale, d / 2, s, n=n, samples=samples)
        assert g.n == n and np.array_equal(g.row_off, h.row_off) and np.array_equal(g.col, h.col)
        assert 1000 <= n <= 30000 and 4 <= d <= 64
        assert 0.5 * d <= 2 * g.m / g.n <= 1.1 * d, (kind, n, d, 2 * g.m / g.n)
    assert gg.mix_seed(1, 0) != gg.mix_seed(1, 1) and gg.mix_seed(1, 0) == gg.mix_seed(1, 0)
