"""Gauge alignment of the swap bond gamma for element-wise comparisons of Phi and Psi (test
infrastructure, pure numpy; no arithmetic of the method).

gamma is internal to T = sum_g Phi[., g] Psi[., g]: a common orthogonal rotation of a block
of (near-)degenerate singular values of the swap (a sign for a single value) in Phi and Psi
leaves T unchanged, and two correct implementations may fix it differently (LAPACK's SVD
and the GPU's Jacobi SVD choose different signs).  The rotation is taken from Phi alone
(orthogonal Procrustes against the reference Phi) and applied to both, so Psi is compared
with no freedom of its own.
"""
import numpy as np

TAU_NULL = 1e-11      # singular values at or below this fraction of the largest carry no weight
TAU_DEG = 1e-6        # neighbours closer than this fraction of the largest form one block


def gamma_blocks(sig):
    """Blocks of consecutive gamma indices with weight, and the number of weighted ones."""
    sig = np.asarray(sig)
    smax = sig[0]
    blocks, j = [], 0
    while j < len(sig) and sig[j] > TAU_NULL * smax:
        j1 = j + 1
        while (j1 < len(sig) and sig[j1] > TAU_NULL * smax
               and sig[j1 - 1] - sig[j1] <= TAU_DEG * smax):
            j1 += 1
        blocks.append(list(range(j, j1)))
        j = j1
    return blocks, j


def align_gamma(phi, psi, phi_ref, sig):
    """Copies of (phi, psi) (rows x chi) with every gamma block rotated onto phi_ref by the
    Procrustes rotation of phi's block; also returns the number of weighted gamma columns
    (Psi columns beyond it span the swap's null space and are arbitrary on either side)."""
    chi = len(sig)
    pg = np.array(phi, dtype=float).reshape(-1, chi)
    sg = np.array(psi, dtype=float).reshape(-1, chi)
    po = np.asarray(phi_ref).reshape(-1, chi)
    blocks, n_live = gamma_blocks(sig)
    for blk in blocks:
        u, _, vt = np.linalg.svd(pg[:, blk].T @ po[:, blk])
        o = u @ vt
        pg[:, blk] = pg[:, blk] @ o
        sg[:, blk] = sg[:, blk] @ o
    return pg, sg, n_live
