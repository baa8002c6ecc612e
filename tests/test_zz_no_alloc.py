"""tatrg_rsvd_noalloc (the randomized SVD for callers that cannot allocate) against the
existing entry point tatrg_rsvd on the same inputs, two calls in a row with the second on a
smaller matrix (the scratch keeps the first call's contents), through the C ABI."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2412_14104_amd as p
    return p


def vp(t):
    return ctypes.c_void_p(t.data_ptr())


def outputs(m, n, k):
    return (torch.empty((m, k), dtype=torch.float64, device="cuda"),
            torch.empty(k, dtype=torch.float64, device="cuda"),
            torch.empty((k, n), dtype=torch.float64, device="cuda"))


def low_rank(seed, m, n, rank):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((m, rank)) * np.logspace(0, -4, rank)) @ rng.standard_normal(
        (rank, n))


@pytest.mark.parametrize("first,second", [((3000, 800, 60, 96, 2), (500, 300, 10, 24, 1))])
def test_noalloc_rsvd_matches_the_handle_rsvd(pkg, first, second):
    eng = pkg.Engine(16, 2, 2, 1)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for idx, (m, n, k, w, q) in enumerate((first, second)):
        print("no-alloc rsvd call", idx, "m n k w q =", m, n, k, w, q, flush=True)
        a = low_rank(100 + idx, m, n, k)
        da = torch.from_numpy(a).cuda()
        u1, s1, v1 = outputs(m, n, k)
        u2, s2, v2 = outputs(m, n, k)
        assert pkg.lib.tatrg_rsvd(eng.handle, vp(da), m, n, n, k, w, q, 7, 3, vp(u1), vp(s1),
                                  vp(v1)) == 0
        assert pkg.lib.tatrg_rsvd_noalloc(vp(da), m, n, n, k, w, q, 7, 3, vp(u2), vp(s2),
                                          vp(v2), stream) == 0
        torch.cuda.synchronize()
        s_ref, s_got = s1.cpu().numpy(), s2.cpu().numpy()
        assert np.abs(s_got - s_ref).max() <= 1e-12 * s_ref[0]
        rec_ref = u1.cpu().numpy() @ np.diag(s_ref) @ v1.cpu().numpy()
        rec_got = u2.cpu().numpy() @ np.diag(s_got) @ v2.cpu().numpy()
        assert np.abs(rec_got - rec_ref).max() <= 1e-12 * np.abs(a).max()
        # and both are the truncated SVD (the matrix has rank k)
        assert np.abs(s_got - np.linalg.svd(a, compute_uv=False)[:k]).max() <= 1e-12 * s_ref[0]


def test_noalloc_rsvd_rejects_sizes_beyond_its_scratch(pkg):
    fake = ctypes.c_void_p(1 << 20)
    for m, n in ((8193, 100), (100, 8193)):
        assert pkg.lib.tatrg_rsvd_noalloc(fake, m, n, n, 4, 8, 1, 0, 0, fake, fake, fake,
                                          None) == -1
    assert pkg.lib.tatrg_rsvd_noalloc(fake, 500, 400, 400, 4, 97, 1, 0, 0, fake, fake, fake,
                                      None) == -1
