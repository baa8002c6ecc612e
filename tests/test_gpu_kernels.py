"""Kernel-level parity of libtatrg on the GPU against float64 numpy / oracle references.

Every call goes through the C ABI (include/tatrg_testing.h) via the ctypes binding.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2412_14104_amd as pkg
    return pkg.lib


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def vp(t):
    return ctypes.c_void_p(t.data_ptr())


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def gemm_bound(a, b, k):
    return 4 * np.finfo(float).eps * (k + 2) * (np.abs(a) @ np.abs(b)) + 1e-300


GEMM_CASES = [
    (1, 1, 1, False, False), (17, 33, 5, False, False), (128, 128, 16, False, False),
    (200, 130, 70, True, False), (130, 200, 70, False, True), (257, 300, 1000, True, True),
    (64, 3, 4096, False, False), (5, 700, 33, True, False),
    # narrow tiles (N <= 32, 64, 96) with every transpose combination
    (1000, 96, 96, False, False), (300, 96, 70, False, True), (129, 65, 40, True, True),
    (77, 50, 19, True, False), (260, 32, 96, True, True), (33, 90, 8, False, True),
]


@pytest.mark.parametrize("m,n,k,ta,tb", GEMM_CASES)
def test_gemm_f64_matches_numpy(lib, m, n, k, ta, tb):
    rng = np.random.default_rng(m * 1000 + n + k)
    batch = 3
    a = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    b = rng.standard_normal((batch, n, k) if tb else (batch, k, n))
    c0 = rng.standard_normal((batch, m, n))
    da, db, dc = dev(a), dev(b), dev(c0)
    rc = lib.tatrg_test_gemm(vp(da), vp(db), vp(dc), m, n, k, a.shape[2], b.shape[2], n,
                             int(ta), int(tb), 0.75, -0.5, batch, a[0].size, b[0].size,
                             c0[0].size, 1, None, stream())
    assert rc == 0
    got = host(dc)
    for i in range(batch):
        aa = a[i].T if ta else a[i]
        bb = b[i].T if tb else b[i]
        ref = 0.75 * aa @ bb - 0.5 * c0[i]
        bound = 0.75 * gemm_bound(aa, bb, k) + 0.5 * np.abs(c0[i]) * 1e-16
        assert np.all(np.abs(got[i] - ref) <= bound), (i, np.abs(got[i] - ref).max())


@pytest.mark.parametrize("m,n,k,ta,tb", GEMM_CASES[:6] + [(384, 256, 9216, True, False)])
def test_gemm_bf16x3_is_fp32_class(lib, m, n, k, ta, tb):
    """Three bf16 planes, six products: |C - AB| is about 2^-24 * |A||B| (the dropped products
    and the last plane's rounding) plus the float32 rounding of one 32-term dot product per
    flush of the leading product; bound 3e-7 * |A||B| (measured worst 7e-8)."""
    rng = np.random.default_rng(m + 7 * n + k)
    batch = 2
    a = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    b = rng.standard_normal((batch, n, k) if tb else (batch, k, n))
    da, db = dev(a), dev(b)
    dc = torch.zeros((batch, m, n), dtype=torch.float64, device="cuda")
    nws = lib.tatrg_test_gemm_bf16x3_ws(m, n, k, a.shape[2], b.shape[2], int(ta), int(tb),
                                        batch, a[0].size, b[0].size)
    ws = torch.empty(nws, dtype=torch.float64, device="cuda")
    rc = lib.tatrg_test_gemm_bf16x3(vp(da), vp(db), vp(dc), m, n, k, a.shape[2], b.shape[2], n,
                                    int(ta), int(tb), 1.0, 0.0, batch, a[0].size, b[0].size,
                                    m * n, vp(ws), stream())
    assert rc == 0
    got = host(dc)
    worst = 0.0
    for i in range(batch):
        aa = a[i].T if ta else a[i]
        bb = b[i].T if tb else b[i]
        ref = aa @ bb
        scale = np.abs(aa) @ np.abs(bb)
        worst = max(worst, (np.abs(got[i] - ref) / scale).max())
    print("split-bf16 GEMM worst |C - AB| / (|A||B|) =", worst, flush=True)
    assert worst < 3e-7, worst


@pytest.mark.parametrize("R1,R2,C1,C2,K1,M2", [
    (3, 12, 36, 12, 36, 40),     # K2 = 144: P's planes padded to 160 (zeroed tail)
    (2, 96, 1024, 96, 64, 256),  # the contraction's shape at chi = 32 with fewer rows
    (5, 7, 130, 9, 33, 129),     # ragged: no dimension a multiple of a tile
])
def test_gemm_bf16x3_chain_through_planes(lib, R1, R2, C1, C2, K1, M2):
    """P = A1 B1 written as bf16 planes by the GEMM's epilogue and read by the next GEMM
    (C[r1] = A2^T P[r1]) gives bit for bit what the float64 route gives: P stored in float64
    (same kernel, columns ordered (c2, c1) so that P[r1] is a strided K x N matrix), then
    split and multiplied; and both are within the split engine's bound of the exact product."""
    rng = np.random.default_rng(R1 + R2 + C1 + K1)
    a1 = rng.standard_normal((R1 * R2, K1))
    b1 = rng.standard_normal((K1, C1 * C2))
    a2 = rng.standard_normal((R2 * C2, M2))
    print("case chain", R1, R2, C1, C2, K1, M2, flush=True)
    da1, db1, da2 = dev(a1), dev(b1), dev(a2)
    dc = torch.zeros((R1, M2, C1), dtype=torch.float64, device="cuda")
    nws = lib.tatrg_test_gemm_bf16x3_chain_ws(R1, R2, C1, C2, K1, M2)
    assert nws > 0
    ws = torch.empty(nws, dtype=torch.float64, device="cuda")
    assert lib.tatrg_test_gemm_bf16x3_chain(vp(da1), vp(db1), vp(da2), vp(dc), R1, R2, C1, C2,
                                            K1, M2, vp(ws), nws - 1, stream()) == -1
    assert lib.tatrg_test_gemm_bf16x3_chain(vp(da1), vp(db1), vp(da2), vp(dc), R1, R2, C1, C2,
                                            K1, M2, vp(ws), nws, stream()) == 0
    got = host(dc)
    # float64 route: P64[(r1 r2)][(c2 c1)], then C[r1] = A2^T P64[r1] as [(r2 c2)][c1]
    b1p = np.ascontiguousarray(b1.reshape(K1, C1, C2).transpose(0, 2, 1).reshape(K1, C2 * C1))
    db1p = dev(b1p)
    p64 = torch.zeros((R1 * R2, C2 * C1), dtype=torch.float64, device="cuda")
    n1 = lib.tatrg_test_gemm_bf16x3_ws(R1 * R2, C2 * C1, K1, K1, C2 * C1, 0, 0, 1, 0, 0)
    ws1 = torch.empty(n1, dtype=torch.float64, device="cuda")
    assert lib.tatrg_test_gemm_bf16x3(vp(da1), vp(db1p), vp(p64), R1 * R2, C2 * C1, K1, K1,
                                      C2 * C1, C2 * C1, 0, 0, 1.0, 0.0, 1, 0, 0, 0, vp(ws1),
                                      stream()) == 0
    ref = torch.zeros((R1, M2, C1), dtype=torch.float64, device="cuda")
    K2 = R2 * C2
    n2 = lib.tatrg_test_gemm_bf16x3_ws(M2, C1, K2, M2, C1, 1, 0, R1, 0, K2 * C1)
    ws2 = torch.empty(n2, dtype=torch.float64, device="cuda")
    assert lib.tatrg_test_gemm_bf16x3(vp(da2), vp(p64), vp(ref), M2, C1, K2, M2, C1, C1, 1, 0,
                                      1.0, 0.0, R1, 0, K2 * C1, M2 * C1, vp(ws2), stream()) == 0
    assert np.array_equal(got, host(ref))
    # against the exact product: each GEMM within 3e-7 |A||B|, the second also carries the
    # first's error through |A2|
    p_ex = (a1 @ b1).reshape(R1, R2, C1, C2).transpose(0, 2, 1, 3).reshape(R1, C1, K2)
    p_abs = (np.abs(a1) @ np.abs(b1)).reshape(R1, R2, C1, C2).transpose(0, 2, 1, 3).reshape(
        R1, C1, K2)
    for r in range(R1):
        ex = a2.T @ p_ex[r].T
        scale = np.abs(a2.T) @ np.abs(p_ex[r].T) + np.abs(a2.T) @ p_abs[r].T
        assert np.all(np.abs(got[r] - ex) <= 3e-7 * scale), r


def test_gemm_bf16x3_three_product_ablation(lib):
    """With three products (i + j <= 1) the dropped terms are about 2^-16 of |A||B|: the
    error grows by orders of magnitude over the six-product engine but stays below
    3 x 2^-16; the engine's default comes back afterwards."""
    rng = np.random.default_rng(17)
    m, n, k = 256, 192, 4096
    a = rng.standard_normal((m, k))
    b = rng.standard_normal((k, n))
    da, db = dev(a), dev(b)
    ref = a @ b
    scale = np.abs(a) @ np.abs(b)
    nws = lib.tatrg_test_gemm_bf16x3_ws(m, n, k, k, n, 0, 0, 1, 0, 0)
    ws = torch.empty(nws, dtype=torch.float64, device="cuda")
    worst = {}
    for nprod in (3, 6):
        assert lib.tatrg_test_split_products(nprod) in (3, 6)
        dc = torch.zeros((m, n), dtype=torch.float64, device="cuda")
        assert lib.tatrg_test_gemm_bf16x3(vp(da), vp(db), vp(dc), m, n, k, k, n, n, 0, 0, 1.0,
                                          0.0, 1, 0, 0, 0, vp(ws), stream()) == 0
        worst[nprod] = (np.abs(host(dc) - ref) / scale).max()
    assert lib.tatrg_test_split_products(5) == -1
    assert lib.tatrg_test_split_products(6) == 6
    print("worst |C - AB| / (|A||B|): 3 products", worst[3], "6 products", worst[6], flush=True)
    assert worst[6] < 3e-7 and 100 * worst[6] < worst[3] < 3 * 2.0 ** -16, worst


def test_gemm_degenerate_shapes(lib):
    """K = 0 leaves beta C; M = 0 or N = 0 touches nothing (both FP64 and split-bf16)."""
    rng = np.random.default_rng(11)
    c0 = rng.standard_normal((5, 7))
    a = dev(np.ones((5, 1)))
    b = dev(np.ones((1, 7)))
    dc = dev(c0)
    assert lib.tatrg_test_gemm(vp(a), vp(b), vp(dc), 5, 7, 0, 1, 7, 7, 0, 0, 1.0, 0.5, 1, 0, 0,
                               0, 1, None, stream()) == 0
    assert np.array_equal(host(dc), 0.5 * c0)
    dc = dev(c0)
    for m, n in ((0, 7), (5, 0)):
        assert lib.tatrg_test_gemm(vp(a), vp(b), vp(dc), m, n, 1, 1, 7, 7, 0, 0, 1.0, 0.5, 1,
                                   0, 0, 0, 1, None, stream()) == 0
        nws = lib.tatrg_test_gemm_bf16x3_ws(m, n, 1, 1, 7, 0, 0, 1, 0, 0)
        ws = torch.empty(max(nws, 1), dtype=torch.float64, device="cuda")
        assert lib.tatrg_test_gemm_bf16x3(vp(a), vp(b), vp(dc), m, n, 1, 1, 7, 7, 0, 0, 1.0,
                                          0.5, 1, 0, 0, 0, vp(ws), stream()) == 0
    assert np.array_equal(host(dc), c0)


def test_gemm_split_k_is_deterministic_and_correct(lib):
    rng = np.random.default_rng(5)
    m, n, k, parts = 40, 24, 50000, 16
    a = rng.standard_normal((m, k))
    b = rng.standard_normal((k, n))
    da, db = dev(a), dev(b)
    part = torch.empty(parts * m * n, dtype=torch.float64, device="cuda")
    outs = []
    for _ in range(2):
        dc = torch.zeros((m, n), dtype=torch.float64, device="cuda")
        assert lib.tatrg_test_gemm(vp(da), vp(db), vp(dc), m, n, k, k, n, n, 0, 0, 1.0, 0.0, 1,
                                   0, 0, 0, parts, vp(part), stream()) == 0
        outs.append(host(dc))
    assert np.array_equal(outs[0], outs[1])
    assert np.all(np.abs(outs[0] - a @ b) <= gemm_bound(a, b, k))


@pytest.mark.parametrize("m,k,ta", [(300, 20000, False), (1024, 32768, False), (257, 9000, True)])
def test_symmetric_split_k_gram(lib, m, k, ta):
    """X X^T (or X^T X) through split-K with one operand: upper tiles computed, lower mirrored."""
    rng = np.random.default_rng(m + k)
    x = rng.standard_normal((k, m) if ta else (m, k))
    dx = dev(x)
    dc = torch.zeros((m, m), dtype=torch.float64, device="cuda")
    parts = 8
    part = torch.empty(parts * m * m, dtype=torch.float64, device="cuda")
    ld = x.shape[1]
    assert lib.tatrg_test_gemm(vp(dx), vp(dx), vp(dc), m, m, k, ld, ld, m, int(ta), int(not ta),
                               1.0, 0.0, 1, 0, 0, 0, parts, vp(part), stream()) == 0
    got = host(dc)
    ref = x.T @ x if ta else x @ x.T
    xx = x.T if ta else x
    assert np.array_equal(got, got.T)
    assert np.all(np.abs(got - ref) <= gemm_bound(xx, xx.T, k))


@pytest.mark.parametrize("m,n,k,same", [(32, 32, 1048576, False), (96, 96, 5000, False),
                                        (40, 17, 100003, False), (1, 1, 4096, False),
                                        (96, 96, 300001, True), (32, 32, 1048576, True),
                                        (70, 70, 9000, True)])
def test_skinny_gram_kernel(lib, m, n, k, same):
    """C = alpha X^T Y + beta C with X (k x m), Y (k x n): the kernel behind the long Grams;
    same=True passes one buffer as X and Y (the symmetric variant, upper blocks mirrored)."""
    rng = np.random.default_rng(m + n + k)
    x = rng.standard_normal((k, m))
    if same:
        y = x
    else:
        y = x[:, :n].copy() if n <= m else rng.standard_normal((k, n))
        y[::7] *= -1.0
    c0 = rng.standard_normal((m, n))
    dx, dc = dev(x), dev(c0)
    dy = dx if same else dev(y)
    part = torch.empty(64 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
    rc = lib.tatrg_test_gemm(vp(dx), vp(dy), vp(dc), m, n, k, m, n, n, 1, 0, 0.5, 2.0, 1, 0, 0,
                             0, -(part.numel() // 1024), vp(part), stream())
    assert rc == 0
    ref = 0.5 * x.T @ y + 2.0 * c0
    bound = 0.5 * gemm_bound(x.T, y, k) + 2.0 * np.abs(c0) * 1e-16
    got = host(dc)
    assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref).max()


@pytest.mark.parametrize("m,n,k,same", [(32, 32, 1048576, True), (96, 96, 300001, True),
                                        (40, 17, 100003, False), (70, 70, 9000, True),
                                        (33, 65, 4099, False), (1, 1, 4096, False)])
def test_skinny_row_gram_kernel(lib, m, n, k, same):
    """C = alpha X Y^T + beta C with X (m x k), Y (n x k) row-major and long rows: the kernel
    behind the Grams over rows (same=True: one buffer as X and Y, upper blocks mirrored)."""
    rng = np.random.default_rng(m + 3 * n + k)
    x = rng.standard_normal((m, k))
    y = x if same else rng.standard_normal((n, k))
    c0 = rng.standard_normal((m, n))
    dx, dc = dev(x), dev(c0)
    dy = dx if same else dev(y)
    part = torch.empty(64 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
    rc = lib.tatrg_test_gemm(vp(dx), vp(dy), vp(dc), m, n, k, k, k, n, 0, 1, 0.5, 2.0, 1, 0, 0,
                             0, -(part.numel() // 1024), vp(part), stream())
    assert rc == 0
    ref = 0.5 * x @ y.T + 2.0 * c0
    bound = 0.5 * gemm_bound(x, y.T, k) + 2.0 * np.abs(c0) * 1e-16
    got = host(dc)
    assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref).max()


def test_skinny_row_gram_declines_the_general_96_case(lib):
    """The general (non-symmetric) 96 x 96 row product is left to the tiled GEMM."""
    x = dev(np.ones((96, 5000)))
    y = dev(np.ones((96, 5000)))
    c = torch.zeros((96, 96), dtype=torch.float64, device="cuda")
    part = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
    assert lib.tatrg_test_gemm(vp(x), vp(y), vp(c), 96, 96, 5000, 5000, 5000, 96, 0, 1, 1.0,
                               0.0, 1, 0, 0, 0, -1024, vp(part), stream()) == -1


TSQR_CASES = [(10, 1), (100, 7), (1000, 32), (5000, 96), (300000, 32), (120000, 96), (96, 96)]


@pytest.mark.parametrize("m,n", TSQR_CASES)
def test_tsqr_orthonormal_factor(lib, m, n):
    rng = np.random.default_rng(m + n)
    y = rng.standard_normal((m, n)) * np.logspace(0, -8, n)[None, :]
    dy = dev(y)
    ws = torch.empty(lib.tatrg_test_tsqr_ws(m, n), dtype=torch.float64, device="cuda")
    dr = torch.empty((n, n), dtype=torch.float64, device="cuda")
    assert lib.tatrg_test_tsqr(vp(dy), m, n, n, vp(dr), vp(ws), stream()) == 0
    q, r = host(dy), host(dr)
    assert np.abs(q.T @ q - np.eye(n)).max() < 1e-13 * max(1, np.sqrt(m) / 100)
    assert np.abs(np.tril(r, -1)).max() == 0.0
    assert np.abs(q @ r - y).max() < 1e-14 * np.abs(y).max() * np.sqrt(n)
    # same span as LAPACK's factor
    qref, _ = np.linalg.qr(y)
    assert np.abs(np.abs(np.linalg.svd(q.T @ qref, compute_uv=False)) - 1).max() < 1e-9


def test_tsqr_rank_deficient_panel(lib):
    rng = np.random.default_rng(11)
    m, n = 50000, 40
    y = rng.standard_normal((m, n))
    y[:, 3] = 0.0
    y[:, 10] = y[:, 2] * 2.0
    y[:, 20:30] = 0.0
    y[:1000, :] = 0.0
    dy = dev(y)
    ws = torch.empty(lib.tatrg_test_tsqr_ws(m, n), dtype=torch.float64, device="cuda")
    dr = torch.empty((n, n), dtype=torch.float64, device="cuda")
    assert lib.tatrg_test_tsqr(vp(dy), m, n, n, vp(dr), vp(ws), stream()) == 0
    q, r = host(dy), host(dr)
    assert np.abs(q.T @ q - np.eye(n)).max() < 1e-13
    assert np.abs(q @ r - y).max() < 1e-13 * np.abs(y).max()


@pytest.mark.parametrize("n", [2, 7, 32, 48, 96])
def test_jacobi_svd_matches_lapack(lib, n):
    rng = np.random.default_rng(n)
    u0, _ = np.linalg.qr(rng.standard_normal((n, n)))
    v0, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sv = np.logspace(0, -12, n)
    a = np.stack([u0 @ np.diag(sv) @ v0.T, rng.standard_normal((n, n))])
    if n > 4:
        a[1][:, -2:] = 0.0           # two zero singular values
    da = dev(a)
    du = torch.empty_like(da)
    dv = torch.empty_like(da)
    ds = torch.empty((2, n), dtype=torch.float64, device="cuda")
    assert lib.tatrg_test_svd(vp(da), vp(du), vp(ds), vp(dv), n, 2, stream()) == 0
    u, s, v = host(du), host(ds), host(dv)
    for i in range(2):
        ref = np.linalg.svd(a[i], compute_uv=False)
        assert np.abs(s[i] - ref).max() < 1e-14 * ref[0] * n
        assert np.all(np.diff(s[i]) <= 0)
        assert np.abs(u[i] @ np.diag(s[i]) @ v[i].T - a[i]).max() < 1e-14 * ref[0] * n
        assert np.abs(v[i].T @ v[i] - np.eye(n)).max() < 1e-13
        nz = s[i] > 1e-300
        assert np.abs(u[i][:, nz].T @ u[i][:, nz] - np.eye(nz.sum())).max() < 1e-12


@pytest.mark.parametrize("n,batch", [(5, 1), (64, 2), (100, 3), (1024, 2)])
def test_cholesky_shifted(lib, n, batch):
    rng = np.random.default_rng(n)
    g = rng.standard_normal((batch, n, n + 3))
    a = g @ g.transpose(0, 2, 1)
    da = dev(a)
    flag = torch.zeros(4, dtype=torch.int32, device="cuda")
    shift = 1e-13
    assert lib.tatrg_test_cholesky(vp(da), n, batch, shift, vp(flag), stream()) == 0
    low = host(da)
    assert host(flag)[0] == 0
    for i in range(batch):
        ref = a[i] + shift * np.trace(a[i]) * np.eye(n)
        assert np.abs(np.triu(low[i], 1)).max() == 0.0
        assert np.abs(low[i] @ low[i].T - ref).max() < 1e-13 * np.abs(ref).max()


def test_cholesky_flags_indefinite_matrix(lib):
    a = -np.eye(8)
    da = dev(a)
    flag = torch.zeros(4, dtype=torch.int32, device="cuda")
    assert lib.tatrg_test_cholesky(vp(da), 8, 1, 0.0, vp(flag), stream()) == 0
    assert host(flag)[0] == 1


@pytest.mark.parametrize("n,batch", [(36, 1), (64, 2), (256, 2), (320, 1), (448, 1), (576, 2),
                                     (1024, 2)])
def test_cholesky_blocked_with_inverse(lib, n, batch):
    """Right-looking blocked Cholesky (64-wide blocks, diagonal blocks inverted in one wave,
    panels and trailing updates as GEMMs) and the triangular inverse by doubling the inverted
    blocks, including sizes that leave a partial last block or an unpaired block at some
    doubling level."""
    rng = np.random.default_rng(7 * n + batch)
    g = rng.standard_normal((batch, n, n + 5)) * np.logspace(0, -3, n + 5)[None, None, :]
    a = g @ g.transpose(0, 2, 1)
    da = dev(a)
    nb = (n + 63) // 64
    dinv = torch.empty(batch * nb * 64 * 64, dtype=torch.float64, device="cuda")
    linv = torch.empty((batch, n, n), dtype=torch.float64, device="cuda")
    tmp = torch.empty(n * n, dtype=torch.float64, device="cuda")
    flag = torch.zeros(4, dtype=torch.int32, device="cuda")
    assert lib.tatrg_test_cholesky_blocked_inv(vp(da), vp(dinv), vp(linv), vp(tmp), n, batch,
                                               vp(flag), stream()) == 0
    low, inv = host(da), host(linv)
    assert host(flag)[0] == 0
    for i in range(batch):
        assert np.abs(np.triu(low[i], 1)).max() == 0.0
        assert np.abs(np.triu(inv[i], 1)).max() == 0.0
        assert np.abs(low[i] @ low[i].T - a[i]).max() < 1e-13 * np.abs(a[i]).max()
        # backward error of the inverse: |Linv L - I| <= c n u cond(L)
        cond = np.linalg.cond(low[i])
        assert np.abs(inv[i] @ low[i] - np.eye(n)).max() < 4 * n * 1.1e-16 * cond


def test_cholesky_blocked_flags_indefinite_matrix(lib):
    n = 100
    a = np.eye(n)
    a[70, 70] = -1.0
    da = dev(a)
    dinv = torch.empty(2 * 64 * 64, dtype=torch.float64, device="cuda")
    linv = torch.empty((n, n), dtype=torch.float64, device="cuda")
    tmp = torch.empty(n * n, dtype=torch.float64, device="cuda")
    flag = torch.zeros(4, dtype=torch.int32, device="cuda")
    assert lib.tatrg_test_cholesky_blocked_inv(vp(da), vp(dinv), vp(linv), vp(tmp), n, 1,
                                               vp(flag), stream()) == 0
    assert host(flag)[0] == 1


@pytest.mark.parametrize("n,pass_", [(1, 1), (7, 0), (32, 1), (96, 0), (96, 1), (96, 2)])
def test_chol_inv_factor_and_inverse(lib, n, pass_):
    rng = np.random.default_rng(100 * n + pass_)
    if pass_ == 2:   # near the identity, as in the last CholeskyQR pass
        e = rng.standard_normal((n, n)) * 1e-3
        gram = np.eye(n) + e @ e.T
    else:
        y = rng.standard_normal((3 * n + 5, n)) * np.logspace(0, -4, n)[None, :]
        gram = y.T @ y
    shift = 1e-10 if pass_ == 0 else 0.0
    dr = torch.empty((n, n), dtype=torch.float64, device="cuda")
    dri = torch.empty((n, n), dtype=torch.float64, device="cuda")
    fail = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert lib.tatrg_test_chol_inv(vp(dev(gram)), vp(dr), vp(dri), n, pass_, shift, vp(fail),
                                   stream()) == 0
    assert host(fail)[0] == 0
    r, ri = host(dr), host(dri)
    ref = gram + shift * np.trace(gram) * np.eye(n)
    assert np.abs(np.tril(r, -1)).max() == 0.0 and np.abs(np.tril(ri, -1)).max() == 0.0
    assert np.abs(r.T @ r - ref).max() < 1e-14 * np.abs(ref).max() * n
    assert np.abs(r - np.linalg.cholesky(ref).T).max() < 1e-10 * np.abs(r).max()
    assert np.abs(ri @ r - np.eye(n)).max() < 1e-12 * np.linalg.cond(r)


def test_chol_inv_flags_a_singular_gram(lib):
    n = 12
    y = np.random.default_rng(1).standard_normal((40, n))
    y[:, 5] = 0.0          # pivot 5 is exactly zero
    gram = y.T @ y
    fail = torch.zeros(1, dtype=torch.int32, device="cuda")
    dr = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    dri = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    assert lib.tatrg_test_chol_inv(vp(dev(gram)), vp(dr), vp(dri), n, 1, 0.0, vp(fail),
                                   stream()) == 0
    assert host(fail)[0] == 2          # pass 1 failed
    assert not host(dr).any()


def test_chol_inv_batched_flags_each_entry(lib):
    """Three Grams in one launch, the middle one singular: its flag reads pass + 1 and its
    factors stay unwritten, the other two match the single-matrix kernel bit for bit."""
    n = 40
    rng = np.random.default_rng(8)
    grams = []
    for b in range(3):
        y = rng.standard_normal((3 * n, n)) * np.logspace(0, -3, n)[None, :]
        if b == 1:
            y[:, 7] = 0.0
        grams.append(y.T @ y)
    g = dev(np.stack(grams))
    dr = torch.zeros((3, n, n), dtype=torch.float64, device="cuda")
    dri = torch.zeros((3, n, n), dtype=torch.float64, device="cuda")
    fail = torch.zeros(3, dtype=torch.int32, device="cuda")
    assert lib.tatrg_test_chol_inv_batched(vp(g), vp(dr), vp(dri), n, 1, 0.0, vp(fail), 3,
                                           stream()) == 0
    assert list(host(fail)) == [0, 2, 0]
    assert not host(dr)[1].any() and not host(dri)[1].any()
    for b in (0, 2):
        r1 = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        ri1 = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        f1 = torch.zeros(1, dtype=torch.int32, device="cuda")
        assert lib.tatrg_test_chol_inv(vp(dev(grams[b])), vp(r1), vp(ri1), n, 1, 0.0, vp(f1),
                                       stream()) == 0
        assert np.array_equal(host(dr)[b], host(r1)) and np.array_equal(host(dri)[b], host(ri1))


def test_philox_sketch_matches_oracle(lib):
    from oracle import philox
    for (rows, cols, seed, step, site) in [(7, 5, 0, 0, 0), (1000, 96, 0, 39, 0),
                                           (33, 17, 2 ** 40 + 7, 3, 9)]:
        out = torch.empty((rows, cols), dtype=torch.float64, device="cuda")
        assert lib.tatrg_test_philox(vp(out), rows, cols, seed, step, site, stream()) == 0
        ref = philox.gaussian_matrix(seed, step, site, rows, cols)
        got = host(out)
        assert np.abs(got - ref).max() <= 8 * np.finfo(float).eps * max(1.0, np.abs(ref).max())


def test_permute_is_exact(lib):
    rng = np.random.default_rng(3)
    # cases four to seven take the tiled path (output- and input-innermost legs differ, both
    # >= 8), with ragged tiles
    for dims, perm in [((3, 4, 5), (2, 0, 1)), ((2, 3, 4, 5, 6), (1, 2, 4, 0, 3)),
                       ((5, 1, 7, 2, 3, 2), (5, 4, 3, 2, 1, 0)), ((40, 33, 50), (2, 0, 1)),
                       ((9, 37, 3, 35), (3, 0, 2, 1)), ((6, 8, 7, 9, 10), (1, 4, 0, 2, 3)),
                       ((2, 64, 3, 32, 5, 40), (0, 5, 2, 4, 3, 1)),
                       # innermost leg kept, its length a multiple of 4 (vectorised path)
                       ((6, 5, 7, 8), (2, 0, 1, 3)), ((3, 4, 2, 5, 12), (3, 2, 0, 1, 4))]:
        x = rng.standard_normal(dims)
        dx = dev(x)
        out = torch.empty(x.size, dtype=torch.float64, device="cuda")
        d = (ctypes.c_int64 * len(dims))(*dims)
        p = (ctypes.c_int * len(perm))(*perm)
        assert lib.tatrg_test_permute(vp(dx), vp(out), len(dims), d, p, stream()) == 0
        assert np.array_equal(host(out).reshape(x.transpose(perm).shape), x.transpose(perm))


def test_gauge_rotation_matches_oracle(lib):
    from oracle import tatrg as t
    rng = np.random.default_rng(4)
    s = np.array([5.0, 3.0, 3.0, 3.0, 1.0, 0.5, 0.5, 1e-14, 0.0])
    p = rng.standard_normal((8, s.size))
    o = torch.empty((s.size, s.size), dtype=torch.float64, device="cuda")
    assert lib.tatrg_test_gauge(vp(dev(s)), vp(dev(p)), vp(o), s.size, 8, t.TAU_NULL, t.TAU_DEG,
                                stream()) == 0
    assert np.abs(host(o) - t.gauge_fix(s, p)).max() < 1e-14
