"""Exact references that pin the oracle.  TEST INFRASTRUCTURE ONLY.

* brute-force enumeration of the 4D Ising partition function on a small periodic lattice,
  straight from Z = sum_s exp(beta sum_<nm> s_n s_m) (Section 3: the tensor network of T and
  W represents this Z);
* exact contraction of a small periodic network of coarse tensors (no truncation);
* the leading terms of the high-temperature series (a sanity bound only).
"""
import itertools
import math
import numpy as np


def ising_lnz_bruteforce(beta, extents):
    """ln Z of the Ising model on a periodic lattice with the given extents (L1..L4).

    Every site n has one bond to n + mu_hat (mod L_mu) for each mu, so an extent of 1 gives a
    self-bond (weight exp(beta)) and an extent of 2 gives two bonds between the same pair;
    this is exactly the periodic tensor network tTr prod_n T.
    """
    dims = tuple(extents)
    v = int(np.prod(dims))
    if v > 24:
        raise ValueError("lattice too large for enumeration")
    sites = list(itertools.product(*[range(n) for n in dims]))
    index = {s: i for i, s in enumerate(sites)}
    bonds = []
    for s in sites:
        for mu in range(4):
            t = list(s)
            t[mu] = (t[mu] + 1) % dims[mu]
            bonds.append((index[s], index[tuple(t)]))
    bonds = np.array(bonds)
    # all 2^v configurations, spins +-1
    cfg = ((np.arange(2 ** v)[:, None] >> np.arange(v)[None, :]) & 1) * -2 + 1
    energy = np.zeros(2 ** v)
    for i, j in bonds:
        energy += cfg[:, i] * cfg[:, j]
    e0 = energy.max()
    return beta * e0 + math.log(np.sum(np.exp(beta * (energy - e0))))


def exact_lnz_slots(phi, psi, slot_extents):
    """ln Z of a periodic network of identical tensors T = sum_g Phi[f,g] Psi[b,g].

    slot_extents = (e1, e2, 1, 1) with e1, e2 in {1, 2}: slots 3 and 4 are traced on each
    tensor, slots 1 and 2 form an e1 x e2 periodic lattice (extent 2: two bonds per pair).
    """
    e1, e2, e3, e4 = slot_extents
    if e3 != 1 or e4 != 1 or e1 not in (1, 2) or e2 not in (1, 2):
        raise ValueError("unsupported extents")
    # t[f1, f2, b1, b2]: slots 3, 4 closed on the tensor itself.
    t = np.einsum("abklg,cdklg->abcd", phi, psi, optimize="greedy")
    if (e1, e2) == (1, 1):
        z = np.einsum("abab->", t)
    elif (e1, e2) == (2, 1):
        # sites 0, 1 along slot 1: h0 = 0->1, h1 = 1->0; slot 2 self-bond per site
        z = np.einsum("pvqv,qwpw->", t, t)
    elif (e1, e2) == (1, 2):
        z = np.einsum("apaq,bqbp->", t, t)
    else:
        # sites (x, y); bond h[x][y]: (x,y)->(x+1,y); v[x][y]: (x,y)->(x,y+1)
        # t[(x,y)] = t[h[x][y], v[x][y], h[x-1][y], v[x][y-1]]
        z = np.einsum("aebf,bgah,cfde,dhcg->", t, t, t, t, optimize="greedy")
    return math.log(z)


def high_t_series(beta):
    """ln Z / V ~= ln 2 + 4 ln cosh b + 6 t^4 + O(t^6), t = tanh b (4D hypercubic lattice:
    6 elementary plaquettes per site).  Used only as a loose sanity bound."""
    t = math.tanh(beta)
    return math.log(2.0) + 4.0 * math.log(math.cosh(beta)) + 6.0 * t ** 4
