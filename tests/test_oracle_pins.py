"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every check uses an independent reference
(brute-force enumeration of Z, closed-form limits, published Philox test vectors, a dense
SVD of an explicitly formed matrix, or a direct evaluation of a defining formula without
the factorised contraction order).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from bond_moments import bond_moments
from oracle import bruteforce as bf
from oracle import philox
from oracle import tatrg as t

BETA_C = 0.1496947


# ----------------------------------------------------------------------------- RNG
@pytest.mark.parametrize("ctr,key,expect", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, expect):
    """Philox4x32-10 known-answer vectors published with Salmon et al. (SC'11)."""
    out = philox.philox4x32_10(np.array(ctr, dtype=np.uint64).reshape(4, 1),
                               np.array(key, dtype=np.uint64))
    assert tuple(int(v[0]) for v in out) == expect


def test_gaussian_moments_and_layouts():
    g = philox.gaussian(0, 0, 0, 1_000_000)
    assert abs(g.mean()) < 5e-3
    assert abs(g.var() - 1.0) < 5e-3
    assert abs((g ** 4).mean() - 3.0) < 3e-2
    # the pairing of elements with counters does not depend on the chunking / offset
    assert np.array_equal(philox.gaussian(0, 0, 0, 17, offset=5), g[5:22])
    a = philox.gaussian_matrix(7, 3, 2, 300, 11)
    assert np.array_equal(philox.gaussian_matrix_t(7, 3, 2, 300, 11), a.T)
    assert np.array_equal(a.reshape(-1), philox.gaussian(7, 3, 2, 3300))
    # different (step, site, seed) give independent streams
    b = philox.gaussian_matrix(7, 3, 3, 300, 11)
    assert abs(np.corrcoef(a.reshape(-1), b.reshape(-1))[0, 1]) < 0.1


# ----------------------------------------------------------------------------- initial tensor
def test_w_gives_boltzmann_weight_and_printed_w_does_not():
    for beta in (0.0, 0.1, BETA_C, 0.7):
        w = t.ising_w(beta)
        boltz = np.array([[math.exp(beta), math.exp(-beta)], [math.exp(-beta), math.exp(beta)]])
        assert np.allclose(w @ w.T, boltz, rtol=1e-14, atol=1e-15)
    wp = t.ising_w(0.3, paper_form=True)
    assert not np.allclose(wp @ wp.T, [[math.exp(0.3), math.exp(-0.3)],
                                       [math.exp(-0.3), math.exp(0.3)]], rtol=1e-3)


def test_initial_tensor_symmetry_rank_parity():
    phi, psi = t.initial_state(0.2, 2)
    tt = np.einsum("abcdz,efghz->abcdefgh", phi, psi)
    # symmetric under any permutation of the 8 legs
    assert np.allclose(tt, tt.transpose(4, 5, 6, 7, 0, 1, 2, 3), atol=1e-15)
    assert np.allclose(tt, tt.transpose(1, 0, 2, 3, 4, 5, 6, 7), atol=1e-15)
    assert np.allclose(tt, tt.transpose(0, 1, 2, 7, 4, 5, 6, 3), atol=1e-15)
    # Z2: vanishes when the total number of "1" indices is odd
    idx = np.indices((2,) * 8).sum(axis=0)
    assert np.all(tt[idx % 2 == 1] == 0.0)
    # rank 2 as a 16 x 16 matrix
    sv = np.linalg.svd(tt.reshape(16, 16), compute_uv=False)
    assert sv[1] > 1e-3 * sv[0] and sv[2] < 1e-13 * sv[0]
    # one site with all legs traced onto itself: Z = 2 exp(4 beta)
    z = np.einsum("abcdabcd->", tt)
    assert abs(z - 2 * math.exp(0.8)) < 1e-12 * z


# ----------------------------------------------------------------------------- RSVD
def test_rsvd_exact_when_width_covers_rank():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((200, 10)) @ np.diag(np.logspace(0, -6, 10)) @ rng.standard_normal((10, 150))
    u, s, v = t.rsvd_dense(a, 10, 12, 0, 0, 0, 0)
    ref = np.linalg.svd(a, compute_uv=False)[:10]
    assert np.allclose(s, ref, rtol=1e-10, atol=0)
    assert np.abs(u @ np.diag(s) @ v.T - a).max() < 1e-12 * np.abs(a).max()
    assert np.abs(u.T @ u - np.eye(10)).max() < 1e-13
    assert np.abs(v.T @ v - np.eye(10)).max() < 1e-13


def test_rsvd_power_iterations_reach_the_truncated_svd():
    rng = np.random.default_rng(2)
    q1, _ = np.linalg.qr(rng.standard_normal((120, 120)))
    q2, _ = np.linalg.qr(rng.standard_normal((90, 90)))
    sv = np.concatenate([np.linspace(10, 5, 8), 0.1 * np.exp(-np.arange(82) / 10)])
    a = q1[:, :90] @ np.diag(sv) @ q2.T
    k = 8
    # error bound of the randomized range finder (Halko, Martinsson, Tropp 2011, Thm 10.6 style)
    u, s, v = t.rsvd_dense(a, k, 12, 0, 0, 0, 0)
    err0 = np.linalg.norm(a - u @ np.diag(s) @ v.T, 2)
    assert err0 < 30 * sv[k]
    u, s, v = t.rsvd_dense(a, k, 12, 6, 0, 0, 0)
    assert np.allclose(s, sv[:k], rtol=1e-12)
    assert abs(np.linalg.norm(a - u @ np.diag(s) @ v.T, 2) - sv[k]) < 1e-10


# ----------------------------------------------------------------------------- gauge
def test_canonical_form_is_gauge_fixed_including_degenerate_clusters():
    """Two factorisations Phi Psi^T of one T (related by a random orthogonal O on gamma)
    give the same A, s, B, also with an exactly degenerate pair of singular values."""
    rng = np.random.default_rng(3)
    chi = 3
    n = chi ** 4
    qa, _ = np.linalg.qr(rng.standard_normal((n, chi)))
    qb, _ = np.linalg.qr(rng.standard_normal((n, chi)))
    s = np.array([3.0, 2.0, 2.0])
    phi = (qa * s).reshape((chi,) * 5)
    psi = qb.reshape((chi,) * 5)
    o, _ = np.linalg.qr(rng.standard_normal((chi, chi)))
    phi2 = (phi.reshape(n, chi) @ o).reshape((chi,) * 5)
    psi2 = (psi.reshape(n, chi) @ o).reshape((chi,) * 5)
    a1, s1, b1, c1, m1 = t.canonicalize(phi, psi, 0, 4)
    a2, s2, b2, c2, m2 = t.canonicalize(phi2, psi2, 0, 4)
    assert abs(c1 - math.sqrt(17.0)) < 1e-13
    assert np.allclose(s1, s / math.sqrt(17.0), atol=1e-15)
    assert np.abs(a1 - a2).max() < 1e-12 and np.abs(b1 - b2).max() < 1e-12
    # T is reproduced and A, B are isometric
    assert np.abs(m1 - m2).max() < 1e-13
    tt = (a1.reshape(n, chi) @ m1) @ b1.reshape(n, chi).T * c1
    assert np.abs(tt - phi.reshape(n, chi) @ psi.reshape(n, chi).T).max() < 1e-13
    assert np.abs(a1.reshape(n, chi).T @ a1.reshape(n, chi) - np.eye(chi)).max() < 1e-14


def test_gauge_rotation_keeps_the_tensor_for_a_split_cluster():
    """A cluster of unequal but close singular values is rotated into the probe basis; the
    weight matrix S' = O^T diag(s) O keeps c A' S' B'^T equal to T exactly."""
    rng = np.random.default_rng(8)
    chi = 3
    n = chi ** 4
    qa, _ = np.linalg.qr(rng.standard_normal((n, chi)))
    qb, _ = np.linalg.qr(rng.standard_normal((n, chi)))
    s = np.array([3.0, 2.0, 2.0 - 1e-7])
    phi = (qa * s).reshape((chi,) * 5)
    psi = qb.reshape((chi,) * 5)
    a, sn, b, c, smat = t.canonicalize(phi, psi, 0, 1)
    assert np.abs(smat - np.diag(sn)).max() > 1e-12          # the cluster was rotated
    tt = c * (a.reshape(n, chi) @ smat) @ b.reshape(n, chi).T
    assert np.abs(tt - phi.reshape(n, chi) @ psi.reshape(n, chi).T).max() < 1e-13
    assert np.allclose(np.linalg.eigvalsh(smat)[::-1], sn, atol=1e-15)


# ----------------------------------------------------------------------------- swap
def _random_canonical(chi, rng):
    n = chi ** 4
    a, _ = np.linalg.qr(rng.standard_normal((n, chi)))
    b, _ = np.linalg.qr(rng.standard_normal((n, chi)))
    s = np.sort(rng.random(chi))[::-1]
    s /= np.linalg.norm(s)
    return a.reshape((chi,) * 5), s, b.reshape((chi,) * 5)


def test_bond_swap_matches_dense_svd_of_the_cell_middle():
    """With sketch width >= rank the swap is the exact SVD of
    M[(alpha,f'),(beta,b')] = sum_x s_alpha B[x,b',alpha] A[x,f',beta] s_beta (Eq. (1))."""
    rng = np.random.default_rng(4)
    chi = 3
    a, s, b = _random_canonical(chi, rng)
    m = np.einsum("xpqra,xfghb,a,b->afghbpqr", b, a, s, s).reshape(chi ** 4, chi ** 4)
    x, sig, y = t.bond_swap(a, np.diag(s), b, chi ** 4, 1, 0, 0)
    ref = np.linalg.svd(m, compute_uv=False)
    assert np.allclose(sig, ref[:chi], rtol=1e-12)
    # X sigma Y^T is the best rank-chi approximation of M
    xs = x.reshape(chi ** 4, chi) * sig
    approx = xs @ y.reshape(chi ** 4, chi).T
    assert abs(np.linalg.norm(m - approx) ** 2 - np.sum(ref[chi:] ** 2)) < 1e-12
    assert np.abs(y.reshape(-1, chi).T @ y.reshape(-1, chi) - np.eye(chi)).max() < 1e-13


# ----------------------------------------------------------------------------- isometries
def test_isometry_grams_are_grams_of_the_cell():
    """rho_A and rho_X equal the Gram of Gamma over the (i2 i3) pair of site n+1 (resp. n),
    computed from the explicit cell A X sigma (Eqs. (2)-(3)); the isometry spans them."""
    rng = np.random.default_rng(5)
    chi = 3
    a, s, b = _random_canonical(chi, rng)
    x, sig, y = t.bond_swap(a, np.diag(s), b, chi ** 4, 1, 0, 0)
    dbg = {}
    iso = t.isometries(a, x, sig, y, b, 9, 1, 0, 0, debug=dbg)
    axs = np.einsum("ijklA,Apqrg,g->ijklpqrg", a, x, sig)       # f(n+1), f'(n), gamma
    rho_a = np.einsum("iJKlpqrg,iMNlpqrg->JKMN", axs, axs)
    rho_x = np.einsum("ijklPQrg,ijklMNrg->PQMN", axs, axs)
    # sigma Y^T D^T for the backward half: D = B(n)
    ysd = np.einsum("Bpqrg,g,ijklB->ijklpqrg", y, sig, b)
    rho_d = np.einsum("iJKlpqrg,iMNlpqrg->JKMN", ysd, ysd)
    rho_y = np.einsum("ijklPQrg,ijklMNrg->PQMN", ysd, ysd)
    for name, ref in (("A", rho_a), ("X", rho_x), ("D", rho_d), ("Y", rho_y)):
        assert np.abs(dbg[name] - ref).max() < 1e-13, name
        u = iso[name]
        r = ref.reshape(9, 9)
        assert np.abs(u @ (u.T @ r) - r).max() < 1e-12      # L = chi^2: full range


# ----------------------------------------------------------------------------- squeezers
def test_squeezer_pair_is_the_eckart_young_truncation():
    rng = np.random.default_rng(6)
    n, chi = 9, 3
    gl = rng.standard_normal((n, 30))
    gr = rng.standard_normal((n, 30))
    rho_l, rho_r = gl @ gl.T, gr @ gr.T
    m, nn, s = t.squeezer_pair(rho_l, rho_r, chi, n, 1, 0, 0, 5, 9)
    r_l = sla.cholesky(rho_l + t.CHOL_SHIFT * np.trace(rho_l) * np.eye(n), lower=False)
    r_r = sla.cholesky(rho_r + t.CHOL_SHIFT * np.trace(rho_r) * np.eye(n), lower=False)
    c = r_l @ r_r.T
    full = np.linalg.svd(c, compute_uv=False)
    assert np.allclose(s, full[:chi], rtol=1e-12)
    resid = np.linalg.norm(r_l @ (np.eye(n) - m @ nn) @ r_r.T) ** 2
    assert abs(resid - np.sum(full[chi:] ** 2)) < 1e-10 * np.sum(full ** 2)
    # (M N) is an oblique projector: (M N)^2 = M N, N M = I_chi
    assert np.abs(nn @ m - np.eye(chi)).max() < 1e-11


def test_squeezer_grams_and_contraction_follow_their_definitions():
    """rho_L / rho_R equal the Grams of the explicit triad cell over the forward / backward
    mu pair (Section 2), and Phi, Psi equal Eqs. (makeMG), (makeMH) evaluated directly."""
    rng = np.random.default_rng(7)
    chi, lw = 3, 4
    a, s, b = _random_canonical(chi, rng)
    x, sig, y = t.bond_swap(a, np.diag(s), b, chi ** 4, 1, 0, 0)
    iso = t.isometries(a, x, sig, y, b, lw, 1, 0, 0)
    e, f, g, h, ua, ux, uy, ud = t.triad(a, x, sig, y, b, iso)
    dbg = {}
    sq = t.squeezers(e, f, g, h, ua, ux, uy, ud, lw, 1, 0, 0, debug=dbg)
    pa = ua.reshape(9, lw) @ ua.reshape(9, lw).T
    px = ux.reshape(9, lw) @ ux.reshape(9, lw).T
    py = uy.reshape(9, lw) @ uy.reshape(9, lw).T
    pd = ud.reshape(9, lw) @ ud.reshape(9, lw).T
    ah = np.einsum("iJKlA,JKjk->ijklA", a, pa.reshape(3, 3, 3, 3))
    xh = np.einsum("aJKlg,JKjk->ajklg", x, px.reshape(3, 3, 3, 3)) * sig
    yh = np.einsum("bJKlg,JKjk->bjklg", y, py.reshape(3, 3, 3, 3))
    dh = np.einsum("iJKlB,JKjk->ijklB", b, pd.reshape(3, 3, 3, 3))
    # explicit triad cell: forward legs f(n+1)=ABCD, f'(n)=EFG; backward b(n)=HIJK, b'(n+1)=LMN
    cell = np.einsum("ABCDa,aEFGg,bLMNg,HIJKb->ABCDEFGHIJKLMN", ah, xh, yh, dh)
    letters = "ABCDEFGHIJKLMN"
    fwd = {2: (1, 4), 3: (2, 5), 4: (3, 6)}       # (f_mu(n+1), f_mu(n)) positions
    bwd = {2: (11, 8), 3: (12, 9), 4: (13, 10)}   # (b_mu(n+1), b_mu(n)) positions
    for mu in (2, 3, 4):
        for side, pos in (("rho_l", fwd[mu]), ("rho_r", bwd[mu])):
            l2 = list(letters)
            l2[pos[0]] = "u"
            l2[pos[1]] = "v"
            spec = letters + "," + "".join(l2) + "->" + letters[pos[0]] + letters[pos[1]] + "uv"
            ref = np.einsum(spec, cell, cell, optimize="greedy").reshape(9, 9)
            assert np.abs(dbg[mu][side] - ref).max() < 1e-12 * np.abs(ref).max(), (mu, side)
    phi, psi = t.contract(e, f, g, h, ua, ux, uy, ud, sq)
    m2, m3, m4 = (sq[mu][0] for mu in (2, 3, 4))
    n2, n3, n4 = (sq[mu][1] for mu in (2, 3, 4))
    phi_ref = np.einsum("iabcA,Adefg,adk,bel,cfm->iklmg", ah, xh, m2, m3, m4, optimize="greedy")
    psi_ref = np.einsum("jdefB,Babcg,kad,lbe,mcf->jklmg", dh, yh, n2, n3, n4, optimize="greedy")
    assert np.abs(phi - phi_ref).max() < 1e-12 * np.abs(phi_ref).max()
    assert np.abs(psi - psi_ref).max() < 1e-12 * np.abs(psi_ref).max()


# ----------------------------------------------------------------------------- whole pipeline
@pytest.mark.parametrize("beta", [0.15, BETA_C, 0.4])
def test_one_step_is_exact_on_two_sites(beta):
    ex = bf.ising_lnz_bruteforce(beta, (2, 1, 1, 1)) / 2
    for chi in (4, 8):
        r = t.run(beta, chi, chi, 2, 0, 1)
        assert abs(r["lnZV"] - ex) < 1e-13


@pytest.mark.parametrize("beta,value", [(0.15, 1.039281932133400), (BETA_C, 1.038479948613929)])
def test_two_steps_exact_against_brute_force_2x2x1x1(beta, value):
    ex = bf.ising_lnz_bruteforce(beta, (2, 2, 1, 1)) / 4
    assert abs(ex - value) < 1e-13
    r = t.run(beta, 16, 2, 2, 0, 2)
    assert abs(r["lnZV"] - ex) < 1e-12


@pytest.mark.parametrize("beta", [0.15, BETA_C])
def test_2x2x2x2_lattice_two_steps_then_exact_residual(beta):
    """2^4 lattice (2^16 configurations): two untruncated RG steps, then the exact
    contraction of the remaining 1x1x2x2 network."""
    ex = bf.ising_lnz_bruteforce(beta, (2, 2, 2, 2)) / 16
    phi, psi, acc = t.run_partial(beta, 16, 2, 2, 0, 2)
    lnz_res = bf.exact_lnz_slots(phi, psi, (2, 2, 1, 1))
    assert abs(acc + lnz_res / 16 - ex) < 1e-12


def test_beta_zero_gives_ln2():
    for chi, r, n in ((6, 2, 16), (4, 1, 9)):
        res = t.run(0.0, chi, r, 2, 0, n)
        assert abs(res["lnZV"] - math.log(2.0)) < 1e-14
        assert math.isnan(res["f"])


def test_large_beta_limit():
    """ln Z / V -> 4 beta + ln 2 / V: two ground states, excitations cost exp(-16 beta)."""
    beta = 3.0
    # The two ground-state modes of T are split by only ~2 exp(-8 beta) = 7.5e-11 relative,
    # so rounding is amplified: relative 1e-11 here (exact arithmetic would give 0).
    ex = bf.ising_lnz_bruteforce(beta, (2, 2, 1, 1)) / 4
    r = t.run(beta, 16, 2, 2, 0, 2)
    assert abs(r["lnZV"] - ex) < 1e-11 * ex
    r = t.run(beta, 6, 2, 2, 0, 16)
    ref = 4 * beta + math.log(2.0) / 2 ** 16
    assert abs(r["lnZV"] - ref) < 1e-11 * ref


def test_gauge_of_w_does_not_change_z_when_exact():
    """Any W with W W^T equal to the bond weight gives the same Z when nothing is truncated."""
    beta = 0.3
    boltz = np.array([[math.exp(beta), math.exp(-beta)], [math.exp(-beta), math.exp(beta)]])
    w_sym = np.real(sla.sqrtm(boltz))
    r1 = t.run(beta, 16, 2, 2, 0, 2)
    r2 = t.run(beta, 16, 2, 2, 0, 2, w=w_sym)
    assert abs(r1["lnZV"] - r2["lnZV"]) < 1e-12


def test_high_temperature_series():
    """Sanity bound only: at small beta the truncated RG (chi = 6) is within the size of the
    first loop correction 6 t^4 of ln 2 + 4 ln cosh b + 6 t^4 (its residual shrinks with chi:
    -2.9e-7, -2.2e-7, -1.4e-7, -9.5e-8 at chi = 6, 8, 12, 16 for b = 0.02).  Losing the
    ln 2 or ln cosh term, or a factor in the plaquette weight, fails it."""
    for beta in (0.02, 0.05):
        r = t.run(beta, 6, 2, 2, 0, 16)
        tt = math.tanh(beta)
        assert abs(r["lnZV"] - bf.high_t_series(beta)) < 6 * tt ** 4


# ----------------------------------------------------------------------------- order parameter
@pytest.mark.parametrize("beta", [0.0, 0.1, BETA_C, 0.4, 2.0])
def test_order_parameter_of_the_initial_tensor_in_closed_form(beta):
    """The initial tensor traced over three directions is A = 2 e^{3b} diag(cosh b, sinh b)
    (each closed leg contributes sum_i W[a, i]^2 = e^b), so X^(0) = e^{2b} / cosh 2b."""
    phi, psi = t.initial_state(beta, 4)
    x = t.order_parameter(phi, psi, 0)
    assert abs(x - math.exp(2 * beta) / math.cosh(2 * beta)) < 1e-14


@pytest.mark.parametrize("beta", [0.15, BETA_C, 0.4])
def test_order_parameter_after_exact_steps_is_a_ratio_of_partition_functions(beta):
    """Untruncated steps keep T exact up to leg gauges, which X does not see.  Tr A^(m) is Z of
    the m-step block with direction 4 closed on itself and Tr (A^(m))^2 is Z of two blocks
    stacked along direction 4, so X^(m) = Z(e)^2 / Z(e1, e2, e3, 2 e4) by enumeration."""
    r = t.run(beta, 16, 2, 2, 0, 2)
    xs = [st["X"] for st in r["steps"]] + [r["X_final"]]
    blocks = {0: (1, 1, 1, 1), 1: (2, 1, 1, 1), 2: (2, 2, 1, 1)}
    for m, e in blocks.items():
        lz1 = bf.ising_lnz_bruteforce(beta, e)
        lz2 = bf.ising_lnz_bruteforce(beta, e[:3] + (2 * e[3],))
        assert abs(xs[m] - math.exp(2 * lz1 - lz2)) < 1e-12, m


def test_order_parameter_is_one_at_infinite_temperature():
    """At beta = 0 every coarse tensor has rank one, and so has A: (Tr A)^2 = Tr A^2."""
    r = t.run(0.0, 6, 2, 2, 0, 8)
    for x in [st["X"] for st in r["steps"]] + [r["X_final"]]:
        assert abs(x - 1.0) < 1e-13


def test_order_parameter_counts_two_ground_states_at_low_temperature():
    """Deep in the ordered phase a block has two degenerate ground states: X -> 2.  A single
    flipped boundary spin costs exp(-4 beta) on the one- and two-site blocks; from the
    four-site block on the gap is large enough that X = 2 to rounding."""
    beta = 3.0
    r = t.run(beta, 6, 2, 2, 0, 16)
    xs = [st["X"] for st in r["steps"]] + [r["X_final"]]
    for m, x in enumerate(xs):
        assert abs(x - 2.0) < (8 * math.exp(-4 * beta) if m < 2 else 1e-12), m


def test_order_parameter_separates_the_phases():
    """Sanity only: on the isotropic 2^8-site block (m = 8), far from the transition
    (beta_c ~ 0.1497), X is near the disordered (1) or ordered (2) fixed point."""
    lo = t.run(0.10, 6, 2, 2, 0, 8)["X_final"]
    hi = t.run(0.20, 6, 2, 2, 0, 8)["X_final"]
    assert abs(lo - 1.0) < 0.15 and abs(hi - 2.0) < 0.05


# ----------------------------------------------------------------------------- plain ATRG
def test_plain_atrg_contraction_follows_its_definition():
    """atrg.contract (one squeezer at a time) against the defining sum evaluated in one
    unfactorised einsum, on random tensors at chi = 3."""
    from oracle import atrg
    rng = np.random.default_rng(17)
    chi = 3
    a, x, y, b = (rng.standard_normal((chi,) * 5) for _ in range(4))
    sig = rng.random(chi)
    sq = {mu: (rng.standard_normal((chi,) * 3), rng.standard_normal((chi,) * 3), None)
          for mu in (2, 3, 4)}
    phi, psi = atrg.contract(a, x, sig, y, b, sq)
    m2, m3, m4 = (sq[mu][0] for mu in (2, 3, 4))
    n2, n3, n4 = (sq[mu][1] for mu in (2, 3, 4))
    ref_phi = np.einsum("iabcA,Adefg,g,adk,bel,cfm->iklmg", a, x, sig, m2, m3, m4,
                        optimize=False)
    ref_psi = np.einsum("jabcB,Bdefg,kda,leb,mfc->jklmg", b, y, n2, n3, n4, optimize=False)
    assert np.allclose(phi, ref_phi, rtol=1e-13, atol=1e-13 * np.abs(ref_phi).max())
    assert np.allclose(psi, ref_psi, rtol=1e-13, atol=1e-13 * np.abs(ref_psi).max())


@pytest.mark.parametrize("chi,n", [(4, 8), (5, 6), (6, 4)])
def test_triad_with_r_equal_chi_is_plain_atrg(chi, n):
    """With r chi = chi^2 internal lines the oversampled isometries are complete unitaries
    and the triad step is plain ATRG (Section 2, the remark on r = chi; Table 1): f, ln c_k
    and every spectrum agree to rounding."""
    from oracle import atrg
    tr = t.run(BETA_C, chi, chi, 2, 0, n)
    at = atrg.run(BETA_C, chi, 2, 0, n)
    assert abs(tr["f"] - at["f"]) <= 1e-12 * abs(at["f"])
    for st_t, st_a in zip(tr["steps"], at["steps"]):
        assert abs(st_t["lnc"] - st_a["lnc"]) <= 1e-12
        for key in ("s", "sigma"):
            assert np.abs(st_t[key] - st_a[key]).max() <= 1e-12
        for mu in (2, 3, 4):
            assert np.abs(st_t["sqz"][mu] - st_a["sqz"][mu]).max() <= 1e-12 * st_a["sqz"][mu][0]


def test_triad_with_fewer_internal_lines_truncates():
    """The identity above is not vacuous: at r = 2 < chi the isometries truncate and f moves
    at the truncation level."""
    from oracle import atrg
    tr = t.run(BETA_C, 6, 2, 2, 0, 4, record=False)
    at = atrg.run(BETA_C, 6, 2, 0, 4)
    assert abs(tr["f"] - at["f"]) > 1e-8 * abs(at["f"])


@pytest.mark.parametrize("beta,extents,chi,r,n", [(0.15, (2, 1, 1, 1), 4, 4, 1),
                                                  (0.4, (2, 1, 1, 1), 4, 4, 1),
                                                  (BETA_C, (2, 2, 1, 1), 16, 2, 2)])
def test_lnz_derivatives_exact(beta, extents, chi, r, n):
    """Central differences (h = 1e-4) of untruncated runs reproduce the exact cumulants of
    the bond sum: d(ln Z/V)/d beta = <E>/V within the difference's h^2 k3 / 6 error, and the
    second derivative Var(E)/V to 1e-6."""
    h = 1e-4
    m, var, k3 = bond_moments(beta, extents)
    l0, d1, d2 = t.lnz_derivatives(beta, h, chi, r, 2, 0, n)
    v = int(np.prod(extents))
    assert abs(l0 - bf.ising_lnz_bruteforce(beta, extents) / v) < 1e-12
    assert abs(d1 - m) < h * h * abs(k3) / 6 * 1.1 + 1e-10, (d1, m)
    assert abs(d2 - var) < 1e-6, (d2, var)
