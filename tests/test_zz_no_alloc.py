"""The entry point that allocates nothing (slim_triangle_reduce_noalloc),
called through the C ABI, against slim_triangle_reduce with a caller
workspace: the same output CSR and counters, bit for bit, on two calls in a
row where the second graph is smaller than the first (the fixed device array
keeps the first call's contents), then the first graph again; and its
refusal of a graph whose workspace exceeds the array."""
import ctypes

import numpy as np
import pytest

from paper_1912_08950_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slim(gpu):
    from paper_1912_08950_amd import slim as s
    return s


def noalloc(slim, dg, p, seed):
    import torch
    ro = torch.full((dg.n + 1,), -7, dtype=torch.int64, device=dg.device)
    col = torch.full((max(dg.nnz, 1),), -7, dtype=torch.int32, device=dg.device)
    st = torch.zeros(6, dtype=torch.int64, device=dg.device)
    with torch.cuda.device(dg.device):
        rc = slim._lib.slim_triangle_reduce_noalloc(
            dg._h, float(p), int(seed), ro.data_ptr(), col.data_ptr(), st.data_ptr(),
            torch.cuda.current_stream(dg.device).cuda_stream)
    slim._check(rc)
    torch.cuda.synchronize(dg.device)
    r = ro.cpu().numpy()
    k = int(r[-1])
    return r, col[:k].cpu().numpy().view(np.uint32), [int(x) for x in st.cpu().numpy()]


def with_workspace(slim, dg, p, seed):
    ro, col, st = slim.result_numpy(slim.triangle_reduce(dg, p, seed))
    return ro, col, [st[k] for k in slim.STAT_KEYS]


def test_noalloc_matches_workspace_call_twice_in_a_row(slim):
    big = gg.rmat(20, 16, 1)     # R-MAT scale 20: the largest class the array holds
    small = gg.er(2000, 16.0, 1)  # then a smaller graph over the same array
    cases = [(big, 0.5, 1), (small, 0.5, 1), (big, 0.8, 7), (gg.empty(10), 0.5, 3)]
    for g, p, seed in cases:
        print(f"noalloc case n={g.n} nnz={g.nnz} p={p} seed={seed}", flush=True)
        dg = slim.Graph.from_csr(g)
        assert dg.workspace_size(slim.OP_TR) <= slim.NOALLOC_WS_BYTES
        got = noalloc(slim, dg, p, seed)
        want = with_workspace(slim, dg, p, seed)
        assert got[2] == want[2], (g.n, p, seed)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (g.n, p, seed)
        dg.close()


def test_noalloc_refuses_a_graph_beyond_the_array(slim):
    g = gg.rmat(21, 16, 1)
    dg = slim.Graph.from_csr(g)
    assert dg.workspace_size(slim.OP_TR) > slim.NOALLOC_WS_BYTES
    import torch
    ro = torch.empty(g.n + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(g.nnz, dtype=torch.int32, device="cuda")
    rc = slim._lib.slim_triangle_reduce_noalloc(dg._h, 0.5, 1, ro.data_ptr(), col.data_ptr(),
                                                None, None)
    assert rc == slim.ENOMEM
    assert b"static workspace" in slim._lib.slim_last_error()
    assert slim._lib.slim_triangle_reduce_noalloc(None, 0.5, 1, ro.data_ptr(), col.data_ptr(),
                                                  None, None) == slim.EINVAL
    assert slim._lib.slim_triangle_reduce_noalloc(dg._h, 1.5, 1, ro.data_ptr(), col.data_ptr(),
                                                  None, None) == slim.EINVAL
