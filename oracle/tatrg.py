"""FP64 CPU oracle of the Triad-ATRG coarse-graining step for the 4D Ising model.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of
bench.py may import this package.  It shares no code with the HIP path.

Plain numpy + LAPACK, float64, static zero-padded shapes.  Every function cites the passage of
Sugimoto & Sasaki, "Applying the Triad network representation to four-dimensional ATRG method"
(LATTICE2024, arXiv:2412.14104) that it follows; readings of points the paper leaves open are
marked READING and listed in the design notes of the repository.

Leg conventions (all legs padded to chi):
  Phi[f1,f2,f3,f4,g], Psi[b1,b2,b3,b4,g]     T = sum_g Phi[f,g] Psi[b,g]
  f = forward legs i_mu(n), b = backward legs j_mu(n) (Section 3, definition of T).
  The coarse-graining direction always sits in slot 1; after a step the slots rotate
  (k2,k3,k4,i1) so that the next direction is in slot 1 (READING: cyclic 1,2,3,4 order).

Parity status: every function is pinned by tests/test_oracle_*.py (brute-force enumeration,
beta -> 0 and beta -> infinity limits, exact-SVD limit of the randomized SVD, Eckart-Young
identities of the squeezers, symmetry of the initial tensor).
"""
import math
import numpy as np
import scipy.linalg as sla

from . import philox

# Sketch / probe call-site identifiers used in the Philox counter (READING).
SITE_SWAP = 0
SITE_ISO = {"A": 1, "X": 2, "Y": 3, "D": 4}
SITE_SQZ = {2: 5, 3: 6, 4: 7}
SITE_PROBE_CANON = 8
SITE_PROBE_SQZ = {2: 9, 3: 10, 4: 11}

N_PROBES = 8          # largest degenerate cluster whose basis is fixed by probes
TAU_NULL = 1e-11      # singular values below TAU_NULL * s_max carry no gauge
TAU_DEG = 1e-6        # neighbours closer than TAU_DEG * s_max form one cluster
SQZ_CUTOFF = 1e-10    # squeezer modes with S < SQZ_CUTOFF * S_max are masked
CHOL_SHIFT = 1e-13    # rho + CHOL_SHIFT * tr(rho) * I before Cholesky


def ein(spec, *ops):
    return np.einsum(spec, *ops, optimize="greedy")


# --------------------------------------------------------------------------- a0: initial tensor
def ising_w(beta, paper_form=False):
    """W of the Ising tensor (Section 3, definition of W).

    READING: the printed W = [[cosh b, sinh b], [cosh b, -sinh b]] does not give the Boltzmann
    weight exp(b s s') on a bond; its element-wise square root does:
      sum_i W[a,i] W[a',i] = cosh b + s_a s_a' sinh b = exp(b s_a s_a').
    paper_form=True returns the printed matrix (used only by a test showing it is wrong).
    """
    c, s = math.cosh(beta), math.sinh(beta)
    if paper_form:
        return np.array([[c, s], [c, -s]])
    return np.array([[math.sqrt(c), math.sqrt(s)], [math.sqrt(c), -math.sqrt(s)]])


def initial_state(beta, chi, w=None):
    """Phi0 = Psi0 = [u_+, u_-], u_a[f1..f4] = prod_mu W[a, f_mu], zero padded to chi.

    T[i1..i4, j1..j4] = sum_a prod W[a,i] prod W[a,j] (Section 3, definition of T).
    """
    if w is None:
        w = ising_w(beta)
    d = w.shape[1]
    phi = np.zeros((chi,) * 5)
    for a in range(w.shape[0]):
        u = ein("i,j,k,l->ijkl", w[a], w[a], w[a], w[a])
        phi[:d, :d, :d, :d, a] = u
    return phi, phi.copy()


# --------------------------------------------------------------------------- linear algebra
def qr_thin(y):
    """Thin Householder QR (LAPACK geqrf/orgqr) of a tall matrix: y = q r, q orthonormal.
    Every use depends only on span(q) and on q r = y."""
    q, r = sla.qr(np.asfortranarray(y), mode="economic", check_finite=False)
    return q, r


def orth_t(pt):
    """Given P^T (w x m, row-major), return Q^T for an orthonormal basis Q of span(P).
    P^T row-major is P column-major, which LAPACK factorises without a copy."""
    q, _ = sla.qr(pt.T, mode="economic", check_finite=False)
    return q.T


def rsvd(apply_t, apply_tt, n_cols, k, w, q, seed, step, site, range_only=False):
    """Randomized SVD with a Gaussian sketch and q QR (power) iterations (Introduction;
    Table 1 counts q as the number of QR iterations of the RSVD).

    READING: Y = A Omega, Q = qr(Y); repeat q times: Q' = qr(A^T Q), Q = qr(A Q');
    then B^T = A^T Q = Qb Rb and the small SVD Rb^T = Uh S Vh^T gives
    A ~= (Q Uh) S (Qb Vh)^T.  Omega is n_cols x w, element (i, j) drawn as number i*w+j.
    range_only returns Q itself (its span is the oversampled range).
    Tall panels are passed transposed: apply_t(P^T) = (A P)^T, apply_tt(Q^T) = (A^T Q)^T.
    """
    omt = philox.gaussian_matrix_t(seed, step, site, n_cols, w)
    qt = orth_t(apply_t(omt))
    for _ in range(q):
        qzt = orth_t(apply_tt(qt))
        qt = orth_t(apply_t(qzt))
    if range_only:
        return np.ascontiguousarray(qt.T)
    btt = apply_tt(qt)                              # (A^T Q)^T
    qb, rb = sla.qr(btt.T, mode="economic", check_finite=False)
    uh, s, vht = np.linalg.svd(rb.T)
    return qt.T @ uh[:, :k], s[:k], qb @ vht.T[:, :k]


def rsvd_dense(a, k, w, q, seed, step, site, range_only=False):
    """rsvd of an explicit matrix a."""
    w = min(w, a.shape[0], a.shape[1])
    return rsvd(lambda pt: pt @ a.T, lambda qt: qt @ a, a.shape[1], k, w, q, seed, step, site,
                range_only)


def gauge_fix(s, probe_proj):
    """Orthogonal block-diagonal O that fixes the basis freedom of an SVD.

    READING (the paper is silent; needed so that seeded sketches of later steps do not depend
    on the rounding of an SVD, nor on perturbations that split a degenerate multiplet):
    singular vectors with s <= TAU_NULL*s_max carry no weight and are left alone.  Runs of
    neighbours with s_j - s_{j+1} <= TAU_DEG*s_max form a cluster [j0, j0+m).  The callers
    apply the rotation so that the represented tensor is unchanged for any O.  With P = probe_proj[:m, j0:j0+m] (probe p against singular vector j), the
    cluster is rotated by O_c where P^T = O_c R (QR, diag R >= 0), so that P O_c is lower
    triangular with a non-negative diagonal.  Clusters of more than N_PROBES vectors are left
    alone.  Returns O (n x n).
    """
    n = s.shape[0]
    o = np.eye(n)
    smax = s[0] if n else 0.0
    if smax <= 0.0:
        return o
    j = 0
    while j < n:
        if s[j] <= TAU_NULL * smax:
            break
        j1 = j + 1
        while j1 < n and s[j1] > TAU_NULL * smax and s[j1 - 1] - s[j1] <= TAU_DEG * smax:
            j1 += 1
        m = j1 - j
        if m <= N_PROBES:
            p = probe_proj[:m, j:j1]
            qo, ro = np.linalg.qr(p.T)
            d = np.where(np.diag(ro) < 0.0, -1.0, 1.0)
            o[j:j1, j:j1] = qo * d[None, :]
        j = j1
    return o


def probes(seed, step, site, n_rows):
    """N_PROBES Gaussian probe vectors as a (N_PROBES, n_rows) array (probe p = row p)."""
    return philox.gaussian(seed, step, site, N_PROBES * n_rows).reshape(N_PROBES, n_rows)


# --------------------------------------------------------------------------- S0
def canonicalize(phi, psi, seed, step):
    """T = Phi Psi^T = A s B^T with isometric A, B (canonical form, Section 2).

    Thin QR of Phi and Psi, SVD of R_Phi R_Psi^T, gauge fixed with probes against A: with the
    rotation O, A' = A O, B' = B O and the weight matrix S' = O^T diag(s) O, so that
    T = c A' S' B'^T exactly.  Returns A'[f,a], s (normalised to |s|=1), B'[b,a], c = |T|_F
    and S' (normalised).
    """
    chi = phi.shape[-1]
    n = chi ** 4
    qp, rp = qr_thin(phi.reshape(n, chi))
    qs, rs = qr_thin(psi.reshape(n, chi))
    u, s, vt = np.linalg.svd(rp @ rs.T)
    v = vt.T
    a = qp @ u
    pw = probes(seed, step, SITE_PROBE_CANON, n)
    o = gauge_fix(s, pw @ a)
    a = a @ o
    b = (qs @ v) @ o
    c = float(np.sqrt(np.sum(s * s)))
    sn = s / c
    smat = o.T @ (sn[:, None] * o)
    return a.reshape((chi,) * 5), sn, b.reshape((chi,) * 5), c, smat


# --------------------------------------------------------------------------- S1
def bond_swap(a, smat, b, ls, q, seed, step):
    """Bond swapping of the unit cell (Section 2, Eq. (1); cost row "Bond swapping" of Table 1).

    Cell of site n+1 (upper) and site n along direction 1, inner bond x = i1(n) = j1(n+1).
    READING: s is placed on both sides of the middle so that A(n+1) and D = B(n) stay
    isometric:  M[(alpha,f'),(beta,b')] = sum_x (B S)[x,b',alpha] (A S)[x,f',beta], with the
    weight matrix S of the canonical form (diag(s) up to the gauge rotation),
    with f' = (f2 f3 f4) of site n and b' = (b2 b3 b4) of site n+1.  Its rank-chi
    randomized SVD M ~= X sigma Y^T gives Gamma = A X sigma Y D.  Omega is indexed by the
    columns (beta, b') of M.
    Returns X[alpha,f2,f3,f4,g], sigma[g], Y[beta,b2,b3,b4,g] and the full sketch spectrum.
    """
    chi = a.shape[0]
    n3 = chi ** 3
    n2 = chi * chi
    at = (a.reshape(-1, chi) @ smat).reshape(chi, n3, chi)      # A~[x, f', beta]
    bt = (b.reshape(-1, chi) @ smat).reshape(chi, n3, chi)      # B~[x, b', alpha]
    at_f = at.transpose(1, 0, 2).reshape(n3, n2)    # [f', (x beta)]
    bt_x = bt.transpose(0, 2, 1).reshape(n2, n3)    # [(x alpha), b']
    # Rows of the left space are stored in (f', alpha) order; a row permutation does not
    # change the span of any sketch.  Panels arrive and leave transposed (j first).

    def apply_m_t(omt):                     # Omega^T[j, (beta,b')] -> (M Omega)^T[j, (f',alpha)]
        w = omt.shape[0]
        t1 = omt.reshape(w * chi, n3) @ bt_x.T                 # [(j beta), (x alpha)]
        t1 = t1.reshape(w, chi, chi, chi).transpose(0, 2, 1, 3).reshape(w, n2, chi)
        return np.matmul(at_f, t1).reshape(w, n3 * chi)       # sum over (x, beta)

    def apply_mt_t(qt):                     # Q^T[j, (f',alpha)] -> (M^T Q)^T[j, (beta,b')]
        w = qt.shape[0]
        t2 = np.matmul(qt.reshape(w, n3, chi).transpose(0, 2, 1), at_f)   # [j, alpha, (x beta)]
        t2 = t2.reshape(w, chi, chi, chi).transpose(0, 3, 2, 1).reshape(w * chi, n2)
        return (t2 @ bt_x).reshape(w, chi * n3)                # sum over (x, alpha)

    w = min(ls, chi ** 4)
    x, sig, y = rsvd(apply_m_t, apply_mt_t, chi ** 4, chi, w, q, seed, step, SITE_SWAP)
    x = x.reshape(n3, chi, chi).transpose(1, 0, 2)             # [alpha, f', gamma]
    return (np.ascontiguousarray(x).reshape((chi,) * 5), sig,
            np.ascontiguousarray(y).reshape((chi,) * 5))


# --------------------------------------------------------------------------- S2
def isometries(a, x, sig, y, b, lw, q, seed, step, debug=None):
    """Oversampled isometries U^A, U^X, U^Y, U^D (Section 2, Eqs. (2)-(3)).

    Because Gamma is canonical only the Gram of A X sigma (resp. sigma Y D) over the (i2 i3)
    leg pair is needed (Eq. (3)).  READING: the isometry is the full width-L range of a
    randomized SVD of that Gram (L = r chi, capped at chi^2), no truncation.
    Returns dict name -> (chi^2, L) orthonormal columns, rows = (l2 l3).
    """
    chi = a.shape[0]
    n2 = chi * chi
    xs = x * sig
    ys = y * sig
    px = ein("afghz,Afghz->aA", xs, xs)
    py = ein("bfghz,Bfghz->bB", ys, ys)
    rho = {
        "A": ein("ijklA,AB,imnlB->jkmn", a, px, a),
        "X": ein("ajklz,amnlz->jkmn", xs, xs),
        "Y": ein("bjklz,bmnlz->jkmn", ys, ys),
        "D": ein("ijklA,AB,imnlB->jkmn", b, py, b),
    }
    w = min(lw, n2)
    out = {}
    if debug is not None:
        debug.update(rho)
    for name in ("A", "X", "Y", "D"):
        r = rho[name].reshape(n2, n2)
        out[name] = rsvd_dense(r, w, w, q, seed, step, SITE_ISO[name], range_only=True)
    return out


# --------------------------------------------------------------------------- S3
def triad(a, x, sig, y, b, iso):
    """Triad representation E, F, G, H (4-leg) and I, J, K, L (3-leg) (Section 2, Eqs.
    (4)-(11)); real tensors, so U^* = U.  sigma is attached to F as in Eq. (5)."""
    chi = a.shape[0]
    lw = iso["A"].shape[1]
    ua, ux, uy, ud = (iso[k].reshape(chi, chi, lw) for k in ("A", "X", "Y", "D"))
    e = ein("ijklA,jkp->iplA", a, ua)          # E[i1, kA, i4, alpha]
    f = ein("ajklg,jkp->aplg", x, ux) * sig    # F[alpha, kX, i4, gamma]
    g = ein("bjklg,jkp->bplg", y, uy)          # G[beta, kY, j4, gamma]
    h = ein("ijklB,jkp->iplB", b, ud)          # H[j1, kD, j4, beta]
    return e, f, g, h, ua, ux, uy, ud


# --------------------------------------------------------------------------- S4
def _chol_upper(rho):
    n = rho.shape[0]
    shift = CHOL_SHIFT * float(np.trace(rho))
    return sla.cholesky(rho + shift * np.eye(n), lower=False)


# Gram of a [f1 f2 f3 f4, a]-type tensor over all f except f_mu: result [u, a, u', a'].
_A_SPEC = {2: "iuklA,iUklB->uAUB", 3: "ijulA,ijUlB->uAUB", 4: "ijkuA,ijkUB->uAUB"}
# Gram of a [a, f2 f3 f4, g]-type tensor with its G-weighted copy over all f except f_mu and
# over g: result [a, u, a', u'].
_X_SPEC = {2: "Aukdz,BUkdz->AuBU", 3: "Akudz,BkUdz->AuBU", 4: "Akduz,BkdUz->AuBU"}


def squeezer_pair(rho_l, rho_r, chi, lw, q, seed, step, site, probe_site):
    """Optimal oblique projector pair for one bond from the Grams of its two sides.

    READING (the paper gives only the cost function): rho = R^T R with R = chol(rho + shift),
    rank-chi randomized SVD R_L R_R^T ~= U S V^T (sketch width L), basis fixed with probes,
    M = R_R^T V D and N = D U^T R_L with D = S^-1/2 (0 for S <= SQZ_CUTOFF S_max).  Then
    R_L M N R_R^T is the rank-chi truncation of R_L R_R^T (Eckart-Young).
    Returns M (n x chi), N (chi x n), S (chi).
    """
    n2 = rho_l.shape[0]
    rho_l = 0.5 * (rho_l + rho_l.T)
    rho_r = 0.5 * (rho_r + rho_r.T)
    r_l = _chol_upper(rho_l)
    r_r = _chol_upper(rho_r)
    c = r_l @ r_r.T
    w = min(lw, n2)
    u, s_, v = rsvd_dense(c, chi, w, q, seed, step, site)
    pw = probes(seed, step, probe_site, n2)
    o = gauge_fix(s_, pw @ v)
    smax = s_[0] if s_.size else 0.0
    keep = s_ > SQZ_CUTOFF * smax
    d = np.where(keep, 1.0 / np.sqrt(np.where(keep, s_, 1.0)), 0.0)
    # rotate after the S^-1/2 weights: M N = R_R^T V S^-1 U^T R_L for any O
    m_sq = ((r_r.T @ v) * d[None, :]) @ o
    n_sq = o.T @ ((d[:, None] * u.T) @ r_l)
    return m_sq, n_sq, s_


def squeezers(e, f, g, h, ua, ux, uy, ud, lw, q, seed, step, debug=None):
    """Squeezers M^(mu), N^(mu), mu = 2, 3, 4 (Section 2, the squeezer cost function).

    The squeezers minimise |Gamma^triad(n) Gamma^triad(n+mu) - Gamma^triad(n) M N
    Gamma^triad(n+mu)|; the triad form is no longer canonical, so every fundamental tensor
    enters (Section 2).  READING: with rho_L (rho_R) the Gram of the triad unit cell over its
    forward (backward) mu pair and R = chol(rho + shift) (rho = R^T R), the rank-chi
    randomized SVD R_L R_R^T ~= U S V^T gives the optimal oblique pair
        M = R_R^T V S^-1/2,   N = S^-1/2 U^T R_L      (modes with tiny S masked).
    Pair order: forward (f_mu(n+1), f_mu(n)); backward (b_mu(n+1), b_mu(n)).
    Returns dict mu -> (M[u1,u2,k], N[k,v1,v2], S).
    """
    # Projected fundamental tensors of the triad cell: A P_A, X sigma P_X, Y P_Y, D P_D.
    ah = ein("iplA,jkp->ijklA", e, ua)
    xh = ein("aplg,jkp->ajklg", f, ux)
    yh = ein("bplg,jkp->bjklg", g, uy)
    dh = ein("iplB,jkp->ijklB", h, ud)
    return squeezers_of_cell(ah, xh, yh, dh, lw, q, seed, step, debug)


def squeezers_of_cell(ah, xh, yh, dh, lw, q, seed, step, debug=None):
    """Squeezers of a unit cell given by its four fundamental tensors A[f1..f4, a],
    X sigma[a, f2 f3 f4, g], Y[b, b2 b3 b4, g], D[b1..b4, b] (each possibly projected):
    the Grams rho_L, rho_R of every mu pair and the optimal pair of squeezer_pair.  The
    triad cell passes the projected tensors A P_A, X sigma P_X, Y P_Y, D P_D; the plain ATRG
    cell passes A, X sigma, Y, D themselves."""
    chi = ah.shape[0]
    n2 = chi * chi
    # Grams of the two halves of the cell over the swap bond gamma.
    aag = ein("ijklA,ijklB->AB", ah, ah)
    ddg = ein("ijklA,ijklB->AB", dh, dh)
    g_f = ein("afghz,aA,AfghZ->zZ", xh, aag, xh)    # forward half  (A X sigma)
    g_b = ein("bfghz,bB,BfghZ->zZ", yh, ddg, yh)    # backward half (Y D)
    xg = ein("afghz,zZ->afghZ", xh, g_b)
    yg = ein("bfghz,zZ->bfghZ", yh, g_f)
    out = {}
    for mu in (2, 3, 4):
        aa = ein(_A_SPEC[mu], ah, ah)                 # [u1, alpha, u1', alpha']
        xx = ein(_X_SPEC[mu], xh, xg)                 # [alpha, u2, alpha', u2']
        rho_l = ein("pAPB,AqBQ->pqPQ", aa, xx).reshape(n2, n2)
        yy = ein(_X_SPEC[mu], yh, yg)                 # [beta, v1, beta', v1']
        dd = ein(_A_SPEC[mu], dh, dh)                 # [v2, beta, v2', beta']
        rho_r = ein("ApBP,qAQB->pqPQ", yy, dd).reshape(n2, n2)
        m_sq, n_sq, s_ = squeezer_pair(rho_l, rho_r, chi, lw, q, seed, step, SITE_SQZ[mu],
                                       SITE_PROBE_SQZ[mu])
        if debug is not None:
            debug[mu] = {"rho_l": rho_l, "rho_r": rho_r}
        out[mu] = (m_sq.reshape(chi, chi, chi), n_sq.reshape(chi, chi, chi), s_)
    return out


# --------------------------------------------------------------------------- S5, S6
def contract(e, f, g, h, ua, ux, uy, ud, sq):
    """Renormalised tensors Phi, Psi (Section 2, Eqs. (makeMG), (makeMH)).

    Phi[i1,k2,k3,k4,g] = sum (E F M4)(I J M2 M3): the O(r^2 chi^7) bottleneck (Section 2,
    Table 1).  Psi likewise with G, H, N4, K, L, N2, N3.  The chain follows the grouping of
    the two brackets of the equation.
    """
    m2, n2_ = sq[2][0], sq[2][1]
    m3, n3_ = sq[3][0], sq[3][1]
    m4, n4_ = sq[4][0], sq[4][1]
    chi = e.shape[0]
    lw = e.shape[1]

    def bracket1(e_, f_, m4_):
        # (E F M4)[i1, kA, kX, gamma, k4] = sum_{alpha, i4a, i4b} E F M4
        fm4 = np.tensordot(m4_, f_, axes=([1], [2]))            # [i4a, k4, alpha, kX, gamma]
        fm4 = np.ascontiguousarray(fm4.transpose(0, 2, 3, 4, 1)).reshape(chi * chi, -1)
        return e_.reshape(chi * lw, chi * chi) @ fm4             # [(i1 kA), (kX gamma k4)]

    def bracket2(u1, u2, s2, s3):
        # (I J M2 M3)[kA, kX, k2, k3] = sum_{i2a i2b i3a i3b} I[i2a,i3a,kA] J[i2b,i3b,kX]
        #                                   M2[i2a,i2b,k2] M3[i3a,i3b,k3]
        t = np.tensordot(u1, s2, axes=([0], [0]))               # [i3a, kA, i2b, k2]
        t = np.tensordot(t, s3, axes=([0], [0]))                # [kA, i2b, k2, i3b, k3]
        t = np.tensordot(t, u2, axes=([1, 3], [0, 1]))          # [kA, k2, k3, kX]
        return np.ascontiguousarray(t.transpose(0, 3, 1, 2))

    def finish_half(p, qt):
        # sum_{kA, kX} P[i1, (kA kX), (gamma k4)] Qt[(kA kX), (k2 k3)]
        out = np.matmul(qt.reshape(lw * lw, chi * chi).T, p.reshape(chi, lw * lw, chi * chi))
        return out.reshape(chi, chi, chi, chi, chi).transpose(0, 1, 2, 4, 3)  # [i1,k2,k3,k4,g]

    # Phi: first bracket E F M4, second bracket I J M2 M3.
    p = bracket1(e, f, m4)
    qt = bracket2(ua, ux, m2, m3)
    phi = finish_half(p, qt)
    del p
    # Psi: G H N4, K L N2 N3 (H plays the role of E, G of F with N4 stored [k4', j4a, j4b]).
    p2 = bracket1(h, g, n4_.transpose(2, 1, 0).copy())     # [(j1 kD), (kY gamma k4')]
    # N stored [k', j_a, j_b]; L (site n) pairs with E's role, K (site n+1) with F's.
    qt2 = bracket2(ud, uy, n2_.transpose(2, 1, 0), n3_.transpose(2, 1, 0))   # [kD, kY, k2', k3']
    psi = finish_half(p2, qt2)
    return phi, psi


def rotate(t):
    """(l1, l2, l3, l4, g) -> (l2, l3, l4, l1, g): the next direction moves to slot 1."""
    return np.ascontiguousarray(t.transpose(1, 2, 3, 0, 4))


# --------------------------------------------------------------------------- order parameter
def open_slot(m):
    """Slot that holds physical direction 4 after m steps: the slots rotate cyclically, so
    after m steps slot j holds direction (j + m) mod 4 (0-based).  READING: the open leg of
    X^(m) is the fourth direction of the lattice, wherever the rotation has put it."""
    return (3 - m) % 4


def order_parameter(phi, psi, m):
    """X^(m) = (Tr A)^2 / Tr(A^2) with A_kl = sum_{i1,i2,i3} T_{i1 i2 i3 k, i1 i2 i3 l}
    (Section 3, the order parameter used for the transition point): forward and backward legs
    of three directions are identified and summed, the fourth stays open.  T = sum_g
    Phi[f, g] Psi[b, g] is the m-th coarse tensor; X does not depend on its normalisation."""
    j = open_slot(m)
    ph = np.moveaxis(phi, j, 3)      # open leg to slot 4, the other three keep their order
    ps = np.moveaxis(psi, j, 3)
    a = np.einsum("xyzkg,xyzlg->kl", ph, ps)
    return float(np.trace(a) ** 2 / np.trace(a @ a))


# --------------------------------------------------------------------------- driver
def widths(chi, r):
    """Internal-line (isometry / squeezer sketch) width L and swap sketch width Ls."""
    return min(r * chi, chi * chi), min(r * chi, chi ** 4)


def step(phi, psi, k, chi, r, q, seed):
    """One coarse-graining step along slot 1 (Section 2 and Fig. 3 flow): canonical form,
    bond swap, isometries, triad tensors, squeezers, contraction, slot rotation."""
    lw, ls = widths(chi, r)
    x_m = order_parameter(phi, psi, k)
    a, s, b, c, smat = canonicalize(phi, psi, seed, k)
    x, sig, y = bond_swap(a, smat, b, ls, q, seed, k)
    iso = isometries(a, x, sig, y, b, lw, q, seed, k)
    e, f, g, h, ua, ux, uy, ud = triad(a, x, sig, y, b, iso)
    sq = squeezers(e, f, g, h, ua, ux, uy, ud, lw, q, seed, k)
    phi, psi = contract(e, f, g, h, ua, ux, uy, ud, sq)
    info = {"lnc": math.log(c), "X": x_m, "s": s, "sigma": sig,
            "sqz": {mu: sq[mu][2] for mu in (2, 3, 4)}}
    return rotate(phi), rotate(psi), info


def finish(phi, psi, seed, n_steps):
    """Trace of the last tensor on the 1x1x1x1 periodic lattice, after one more canonical
    normalisation: returns (ln c_N, tTr of the normalised tensor)."""
    a, s, b, c, smat = canonicalize(phi, psi, seed, n_steps)
    chi = a.shape[-1]
    ttr = float(np.sum((a.reshape(-1, chi) @ smat) * b.reshape(-1, chi)))
    return math.log(c), ttr


def run(beta, chi, r, q, seed, n_steps, w=None, record=True):
    """Free energy of the 4D Ising model on the 2^n_steps-site periodic lattice.

    Z = tTr prod T (Section 3).  Each step normalises T by c_k = |T|_F, so
      ln Z / V = sum_{k=0}^{N} 2^-k ln c_k + 2^-N ln tTr(T_N / c_N),
    and f = -(ln Z / V) / beta (READING: the sign and scale of Table 2 require this form).
    The lattice has extents 2^ceil((N - mu + 1) / 4) in direction mu (READING).
    """
    phi, psi = initial_state(beta, chi, w)
    acc = 0.0
    steps = []
    for k in range(n_steps):
        phi, psi, info = step(phi, psi, k, chi, r, q, seed)
        acc += 2.0 ** (-k) * info["lnc"]
        if record:
            steps.append(info)
        else:
            steps.append({"lnc": info["lnc"], "X": info["X"]})
    x_n = order_parameter(phi, psi, n_steps)
    lnc_n, ttr = finish(phi, psi, seed, n_steps)
    if not ttr > 0.0:
        raise FloatingPointError("non-positive trace of the final tensor")
    lnzv = acc + 2.0 ** (-n_steps) * (lnc_n + math.log(ttr))
    f = -lnzv / beta if beta > 0 else float("nan")
    return {"lnZV": lnzv, "f": f, "steps": steps, "lnc_final": lnc_n, "ttr": ttr,
            "X_final": x_n}


def lnz_derivatives(beta, delta, chi, r, q, seed, n_steps):
    """d(ln Z/V)/d beta and d^2(ln Z/V)/d beta^2 of the truncated RG by central differences
    at beta - delta, beta, beta + delta (Z of Section 3; u = -d(ln Z/V)/d beta is the internal
    energy per site, c = beta^2 d^2(ln Z/V)/d beta^2 the specific heat).  The sketches do not
    depend on beta (READING: beta is not in the generator's key), so the three runs share them
    and ln Z/V is a smooth function of beta between truncation changes.
    Returns (ln Z/V at beta, first derivative, second derivative)."""
    lm = run(beta - delta, chi, r, q, seed, n_steps, record=False)["lnZV"]
    l0 = run(beta, chi, r, q, seed, n_steps, record=False)["lnZV"]
    lp = run(beta + delta, chi, r, q, seed, n_steps, record=False)["lnZV"]
    return l0, (lp - lm) / (2.0 * delta), (lp - 2.0 * l0 + lm) / (delta * delta)


def run_partial(beta, chi, r, q, seed, n_steps, w=None):
    """First n_steps steps only: returns (Phi, Psi, sum_{k<n} 2^-k ln c_k)."""
    phi, psi = initial_state(beta, chi, w)
    acc = 0.0
    for k in range(n_steps):
        phi, psi, info = step(phi, psi, k, chi, r, q, seed)
        acc += 2.0 ** (-k) * info["lnc"]
    return phi, psi, acc
