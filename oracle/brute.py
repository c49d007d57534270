"""Exact contraction of a finite open square lattice by a row transfer matrix.

TEST INFRASTRUCTURE ONLY.  Independent of the CTMRG code: no truncation, no
environment.  Used to pin the move semantics: an untruncated CTMRG run of k
sweeps from the boundary-vector start represents exactly the
(2k+1) x (2k+1) lattice computed here.
"""
import numpy as np


def finite_lattice_log_z(a, b, Lx, Ly):
    """log |Z| and sign of Z for Ly rows x Lx columns of a[u, l, d, r].

    Every outer leg (top u, bottom d, left l, right r) is contracted with b.
    Rows are absorbed top to bottom; within a row sites are absorbed left to
    right with the horizontal bond carried as the last axis of the state.
    The state is renormalised after every row and the log of the factors kept.
    """
    d = a.shape[0]
    psi = b
    for _ in range(Lx - 1):
        psi = np.multiply.outer(psi, b)
    psi = np.asarray(psi).reshape((d,) * Lx)
    log_scale = 0.0
    for _ in range(Ly):
        st = np.multiply.outer(psi, b)              # carry = left boundary
        for j in range(Lx):
            # contract axis j (up leg) and the carry (left leg) with a[u, l, dd, r]
            st = np.tensordot(st, a, axes=([j, Lx], [0, 1]))   # rest + (dd, r)
            st = np.moveaxis(st, Lx - 1, j)         # dd back to slot j, r last
        psi = np.tensordot(st, b, axes=([Lx], [0]))  # right boundary
        m = np.abs(psi).max()
        psi = psi / m
        log_scale += np.log(m)
    z = psi
    for _ in range(Lx):
        z = np.tensordot(z, b, axes=([0], [0]))
    z = float(z)
    return log_scale + np.log(abs(z)), np.sign(z)
