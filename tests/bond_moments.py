"""Exact beta-derivatives of ln Z / V of the periodic Ising lattice by enumeration (test
helper, no oracle or library code): d^k(ln Z)/d beta^k are the cumulants of the bond sum
E = sum_<ij> s_i s_j over the Boltzmann weight e^{beta E}."""
import itertools

import numpy as np


def bond_moments(beta, extents):
    """First three cumulants of E per site on the periodic lattice with the given extents
    (one bond from every site to its neighbour in each of the four directions, so an extent
    of 1 is a self-bond and an extent of 2 a double bond, as in the tensor network)."""
    sites = list(itertools.product(*[range(n) for n in extents]))
    v = len(sites)
    idx = {s: i for i, s in enumerate(sites)}
    bonds = [(idx[s], idx[tuple((s[m] + 1) % extents[m] if m == mu else s[m]
                                for m in range(4))]) for s in sites for mu in range(4)]
    e = []
    for bits in range(2 ** v):
        spin = [1 - 2 * ((bits >> i) & 1) for i in range(v)]
        e.append(sum(spin[i] * spin[j] for i, j in bonds))
    e = np.array(e, dtype=np.float64)
    w = np.exp(beta * (e - e.max()))
    w /= np.sum(w)
    mean = float(np.sum(w * e))
    return (mean / v, float(np.sum(w * (e - mean) ** 2)) / v,
            float(np.sum(w * (e - mean) ** 3)) / v)
