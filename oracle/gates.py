"""Two-site imaginary-time gate and its rank-4 split (Fig. 3(b)).

TEST INFRASTRUCTURE ONLY: builds exact A', B' inputs with a 4D gamma bond
for the single-gate pin.  Not part of the CTMRG path.
"""
import numpy as np


def gate(H, tau):
    """exp(-tau H / 2) for a real symmetric 4x4 two-site H, index (sA sB)(sA' sB')."""
    w, V = np.linalg.eigh(H)
    return (V * np.exp(-0.5 * tau * w)[None, :]) @ V.T


def split_gate(G):
    """G[(s t), (s' t')] = sum_r gL[s, s', r] gR[r, t, t'] by SVD (rank <= 4)."""
    g = G.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)  # (s s') x (t t')
    U, S, Vh = np.linalg.svd(g)
    gL = (U * np.sqrt(S)[None, :]).reshape(2, 2, 4)
    gR = (np.sqrt(S)[:, None] * Vh).reshape(4, 2, 2)
    return gL, gR


def apply_gate(A, B, G, gamma=2):
    """A'[s, a, ..., (g r), ...] = sum_s' gL[s, s', r] A[s', a, ..., g, ...] and
    B' likewise with gR, so the gamma bond grows from D to 4D."""
    gL, gR = split_gate(G)
    Ap = np.einsum('sur,uaxyz->saxyzr', gL, A)
    Bp = np.einsum('rtv,vaxyz->taxyzr', gR, B)
    ax = 2 + gamma
    # merge (gamma, r) into one leg at position ax
    Ap = np.moveaxis(Ap, 5, ax + 1)
    Bp = np.moveaxis(Bp, 5, ax + 1)
    sh = list(A.shape)
    sh[ax] = sh[ax] * 4
    return Ap.reshape(sh), Bp.reshape(sh)
