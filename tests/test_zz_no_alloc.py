"""pcamg_orient_noalloc (no allocation, fixed device workspace) against
pcamg_orient through the C ABI: identical outputs bit for bit on two calls in a
row, the second on a smaller cover, and sizes beyond the workspace refused."""
import ctypes as C

import numpy as np
import pytest

from paper_1806_07028_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cover(oracle, g, seed):
    n, rp, ci, w = g
    rp2, ci2 = oracle.a2_pattern(n, rp, ci)
    e = I.uniform(seed, n)
    su, sv = oracle.sorted_edges(n, rp2, ci2, e)
    return oracle.path_cover(n, su, sv).reshape(-1)


def _orient(L, name, nb):
    n = nb.size // 2
    nbd = torch.as_tensor(nb, dtype=torch.int32, device="cuda")
    out = [torch.full((n,), -7, dtype=torch.int32, device="cuda") for _ in range(3)]
    st = torch.cuda.current_stream().cuda_stream
    rc = getattr(L, name)(n, nbd.data_ptr(), out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), st)
    assert rc == 0, L.pcamg_last_error()
    return [o.cpu().numpy() for o in out]


def test_orient_noalloc_equals_orient(gpu, oracle):
    from paper_1806_07028_amd import _lib
    L = _lib.lib()
    big = _cover(oracle, I.grid2d(400, 300, weight_seed=2), 11)      # 120,000 vertices
    small = _cover(oracle, I.rgg(3000, 5), 12)                         # a smaller cover next
    head = big[: 2 * 1000]
    head = np.where(head < 1000, head, -1).astype(np.int32)  # the cover restricted to vertices 0..999
    for nb in (big, small, head):
        ref = _orient(L, "pcamg_orient", nb)
        got = _orient(L, "pcamg_orient_noalloc", nb)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        # and against the oracle's orientation
        pid, pos, plen, _ = oracle.orient(nb)
        assert np.array_equal(got[0], pid) and np.array_equal(got[1], pos) and np.array_equal(got[2], plen)


def test_orient_noalloc_limit(gpu):
    from paper_1806_07028_amd import _lib
    L = _lib.lib()
    n = (1 << 19) + 1
    d = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = L.pcamg_orient_noalloc(n, d.data_ptr(), d.data_ptr(), d.data_ptr(), d.data_ptr(), None)
    assert rc == -1
    assert b"exceeds its fixed workspace" in L.pcamg_last_error()
