"""Column transfer matrix of the CTMRG environment and its leading spectrum.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The correlation
length of the converged environment (Sec. IV, where the paper quotes xi in
lattice constants of the rhombic lattice) comes from the leading eigenvalues
of the transfer matrix that moves one lattice column (or row) along.

Reading: the transfer matrix of one column is the top edge tensor, the site
tensor and the bottom edge tensor,
    v'[x', r, y'] = sum T1[x, m, x'] a[m, l, n, r] T3[y', n, y] v[x, l, y]
(horizontal; with site=False the site tensor is left out and the inner legs
of T1 and T3 are joined), and for the vertical direction the same with T2,
a rotated by 90 degrees, and T4.  xi = -1 / ln |lambda_2 / lambda_1|, and
the eigenvalues are sorted by decreasing magnitude.  The dense matrix is
built here by einsum and diagonalised by LAPACK.
"""
import numpy as np

from . import ctmrg as O


def transfer_matrix(env, a, direction=0, site=True):
    """Dense column (direction 0) or row (direction 1) transfer matrix."""
    if direction == 0:
        Tt, Tb, at = env.T[0], env.T[2], a
    else:
        Tt, Tb, at = env.T[1], env.T[3], O.rotate(a, 1)
    chi = Tt.shape[0]
    if site:
        d = at.shape[1]
        M = np.einsum('amx,mlnr,yne->xryale', Tt, at, Tb)
        return M.reshape(chi * d * chi, chi * d * chi)
    M = np.einsum('amx,yme->xyae', Tt, Tb)
    return M.reshape(chi * chi, chi * chi)


def leading_eigenvalues(env, a, direction=0, site=True, nev=4):
    ev = np.linalg.eigvals(transfer_matrix(env, a, direction, site))
    return ev[np.argsort(-np.abs(ev), kind='stable')][:nev]


def correlation_length(ev):
    """-1 / ln |lambda_2 / lambda_1| (0 if lambda_2 vanishes)."""
    r = abs(ev[1]) / abs(ev[0])
    return 0.0 if r == 0.0 else -1.0 / np.log(r)
