"""FP64 CPU oracle of one plain ATRG coarse-graining step of the 4D Ising model.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of
bench.py may import this package.  It shares no code with the HIP path.

Plain ATRG is the method the triad representation is applied to (Introduction; Section 2):
the same canonical form, bond swap and squeezers, but the renormalised tensors are
contracted directly from A, X sigma, Y, D and the squeezers, without the triad tensors and
their internal lines -- the O(chi^9) contraction of the ATRG column of Table 1 (the cost
also holds memory of chi^7 numbers, so this oracle is for chi <= 8).  With the internal
line dimension r chi = chi^2 the oversampled isometries of the triad step are complete
unitaries, the projectors U U^T are the identity and the triad step reduces to this one
(Section 2, the remark on r = chi): that identity pins both.

Legs and readings as in oracle/tatrg.py; every random number comes from the same Philox
streams (the swap at site 0, the squeezers at sites 5-7, the probes at 8-11).
"""
import math

import numpy as np

from . import tatrg


def contract(a, x, sig, y, b, sq):
    """Phi[i1,k2,k3,k4,g] = sum A[i1,a2,a3,a4,alpha] X[alpha,x2,x3,x4,g] sigma_g
    M2[a2,x2,k2] M3[a3,x3,k3] M4[a4,x4,k4], and Psi[j1,k2,k3,k4,g] = sum B[j1,b2,b3,b4,beta]
    Y[beta,y2,y3,y4,g] N2[k2,y2,b2] N3[k3,y3,b3] N4[k4,y4,b4] (squeezer pairs ordered as in
    tatrg.squeezers: M[leg of site n+1, leg of site n, k], N[k, leg of site n+1, leg of site
    n]).  Contracted one squeezer at a time; the intermediate after X has chi^7 entries."""
    m2, m3, m4 = (sq[mu][0] for mu in (2, 3, 4))
    n2_, n3_, n4_ = (sq[mu][1] for mu in (2, 3, 4))
    xs = x * sig
    t = np.einsum("iabcA,apk->ibcApk", a, m2)               # [i1,a3,a4,alpha,x2,k2]
    t = np.einsum("ibcApk,Apefg->ibckefg", t, xs)           # [i1,a3,a4,k2,x3,x4,g]
    t = np.einsum("ibckefg,bel->icklfg", t, m3)             # [i1,a4,k2,k3,x4,g]
    phi = np.einsum("icklfg,cfm->iklmg", t, m4)             # [i1,k2,k3,k4,g]
    t = np.einsum("jabcB,kpa->jbcBpk", b, n2_)              # [j1,b3,b4,beta,y2,k2]
    t = np.einsum("jbcBpk,Bpefg->jbckefg", t, y)            # [j1,b3,b4,k2,y3,y4,g]
    t = np.einsum("jbckefg,leb->jcklfg", t, n3_)            # [j1,b4,k2,k3,y4,g]
    psi = np.einsum("jcklfg,mfc->jklmg", t, n4_)            # [j1,k2,k3,k4,g]
    return phi, psi


def step(phi, psi, k, chi, q, seed, ls=None, lw=None):
    """One plain ATRG step along slot 1: canonical form, bond swap (randomized SVD of the
    cell middle, sketch width ls), squeezers from the unprojected cell (sketch width lw),
    the direct contraction and the slot rotation.  Widths default to the full chi^2."""
    n2 = chi * chi
    ls = n2 if ls is None else ls
    lw = n2 if lw is None else lw
    x_m = tatrg.order_parameter(phi, psi, k)
    a, s, b, c, smat = tatrg.canonicalize(phi, psi, seed, k)
    x, sig, y = tatrg.bond_swap(a, smat, b, ls, q, seed, k)
    sq = tatrg.squeezers_of_cell(a, x * sig, y, b, lw, q, seed, k)
    phi, psi = contract(a, x, sig, y, b, sq)
    info = {"lnc": math.log(c), "X": x_m, "s": s, "sigma": sig,
            "sqz": {mu: sq[mu][2] for mu in (2, 3, 4)}}
    return tatrg.rotate(phi), tatrg.rotate(psi), info


def run(beta, chi, q, seed, n_steps, ls=None, lw=None):
    """ln Z / V and f = -(ln Z / V) / beta of the 2^n_steps-site periodic lattice by plain
    ATRG, normalised and finished exactly as tatrg.run."""
    phi, psi = tatrg.initial_state(beta, chi)
    acc = 0.0
    steps = []
    for k in range(n_steps):
        phi, psi, info = step(phi, psi, k, chi, q, seed, ls, lw)
        acc += 2.0 ** (-k) * info["lnc"]
        steps.append(info)
    lnc_n, ttr = tatrg.finish(phi, psi, seed, n_steps)
    lnzv = acc + 2.0 ** (-n_steps) * (lnc_n + math.log(ttr))
    f = -lnzv / beta if beta > 0 else float("nan")
    return {"lnZV": lnzv, "f": f, "steps": steps}
