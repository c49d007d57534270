"""Pins of the oracle's full-update bond truncation (oracle/fu.py).

With the identity as metric the optimum is the best rank-D approximation
of the gamma-bond matrix (Eckart-Young), which alternating least squares
must reach; with the identity gate the old tensors are exact; and every ALS
round can only lower the error.
"""
import numpy as np

from oracle import ctmrg as O, fu, gates
from paper_1906_02220_amd import synth


def _inputs(D, seed, gamma=2):
    A, B = synth.random_purification(D, seed, gamma=gamma)
    H = synth.bond_operator_real(synth.random_coefficients(seed + 1))
    return A, B, H


def test_identity_metric_reaches_eckart_young():
    D, gamma = 2, 2
    A, B, H = _inputs(D, 3, gamma)
    Ag, Bg = gates.apply_gate(A, B, gates.gate(H, 0.7), gamma)
    Agp, Bgp = fu.to_fused(Ag, gamma), fu.to_fused(Bg, gamma)
    # gamma-bond matrix [(s a l u), (t c r d)] and its discarded weight beyond rank D
    M = np.einsum('salug,tcrdg->salutcrd', Agp, Bgp).reshape(4 * D * D, 4 * D * D)
    sv = np.linalg.svd(M, compute_uv=False)
    best = np.sum(sv[D:] ** 2) / np.sum(sv ** 2)
    E = np.eye(D ** 4)
    _, _, errs = fu.truncate(Agp, Bgp, E, fu.to_fused(A, gamma), fu.to_fused(B, gamma), 400)
    assert abs(errs[-1] - best) < 1e-10 * max(best, 1e-3)
    assert errs[-1] < errs[0]


def test_identity_gate_keeps_the_tensors():
    D, gamma = 2, 1
    A, B, H = _inputs(D, 5, gamma)
    A2, B2, errs, _ = fu.bond_update(A, B, gamma, H, 0.0, 8, 4, 2)
    assert errs[0] < 1e-28 and errs[-1] < 1e-20
    K0 = O.composite(A, B, gamma)
    K2 = O.composite(A2, B2, gamma)
    assert np.abs(K2 - K0).max() < 1e-10 * np.abs(K0).max()


def test_als_rounds_never_raise_the_error():
    D, gamma = 2, 0
    A, B, H = _inputs(D, 7, gamma)
    _, _, errs, E = fu.bond_update(A, B, gamma, H, 0.4, 8, 6, 12)
    assert np.all(np.diff(errs) <= 1e-12 * errs[0])
    assert errs[-1] < errs[0]
    # the metric of a physical environment is (nearly) symmetric positive
    Es = 0.5 * (E + E.T)
    assert np.abs(E - E.T).max() < 1e-6 * np.abs(E).max()
    assert np.linalg.eigvalsh(Es).min() > -1e-8 * np.abs(Es).max()


def test_trotter_step_with_only_z_bonds_is_one_z_update():
    """H_x = H_y = 0: the four x and y gates are the identity, so the step is
    the z-bond update with tau = dbeta (Sec. III gate sequence)."""
    D = 2
    A, B = synth.random_purification(D, 9)
    Hz = synth.bond_operator_real(synth.random_coefficients(10))
    Z = np.zeros((4, 4))
    A1, B1, _ = fu.trotter_step(A, B, [Z, Z, Hz], 0.3, 8, 5, 3)
    A2, B2, _, _ = fu.bond_update(A, B, 2, Hz, 0.3, 8, 5, 3)
    K1, K2 = O.composite(A1, B1, 2), O.composite(A2, B2, 2)
    assert np.abs(K1 - K2).max() < 1e-9 * np.abs(K2).max()


def _only(gamma, H):
    Z = np.zeros((4, 4))
    return [H if g == gamma else Z for g in range(3)]


def test_trotter_step_x_and_y_fractions_and_order():
    """Sec. III: the second-order step is G_x(db/2) G_y(db/2) G_z(db) G_y(db/2)
    G_x(db/2).  With only x terms the y and z gates are the identity (which a
    bond update keeps exactly), so the step is two x updates of db/2 each, at
    the first and last positions; with only y terms it is two y updates of
    db/2 at the second and fourth positions.  A wrong fraction (db instead
    of db/2, or db/2 once) or a wrong position fails here, because a bond
    update with truncation is not additive in tau."""
    D, db = 2, 0.6
    A, B = synth.random_purification(D, 13)
    H = synth.bond_operator_real(synth.random_coefficients(14))
    for gamma, where in ((0, (0, 4)), (1, (1, 3))):
        A1, B1, hist = fu.trotter_step(A, B, _only(gamma, H), db, 8, 5, 3)
        Ah, Bh, _, _ = fu.bond_update(A, B, gamma, H, 0.5 * db, 8, 5, 3)
        A2, B2, _, _ = fu.bond_update(Ah, Bh, gamma, H, 0.5 * db, 8, 5, 3)
        K1, K2 = O.composite(A1, B1, gamma), O.composite(A2, B2, gamma)
        assert np.abs(K1 - K2).max() < 1e-9 * np.abs(K2).max()
        # the gates of the other bond types are the identity: no error there
        for i in range(5):
            if i in where:
                assert hist[i][0] > 1e-8
            else:
                assert hist[i][0] < 1e-20
        # one full-db update is a different tensor: the fraction is pinned
        Af, Bf, _, _ = fu.bond_update(A, B, gamma, H, db, 8, 5, 3)
        Kf = O.composite(Af, Bf, gamma)
        assert np.abs(K1 - Kf).max() > 1e-6 * np.abs(Kf).max()
