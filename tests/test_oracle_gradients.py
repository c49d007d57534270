"""Pins of the oracle's derivatives (finite differences of its objectives).

The gradient parity tests compare the hand-written adjoint of the HIP path
with directional derivatives of the oracle's objectives.  These tests pin
those derivatives to values fixed by mathematics: the exactness of the
difference formula on quartics, Euler homogeneity of ln kappa in A and B,
and the closed-form nearest-neighbour correlations of the square (Onsager)
and honeycomb (Houtappel) Ising models, which are derivatives of the free
energies the norm per site reproduces.
"""
import numpy as np
import pytest

from oracle import closed_forms as CF, gradients as G
from paper_1906_02220_amd import synth


def test_central_difference_is_exact_on_quartics():
    g = lambda t: 1.0 + 2.0 * t - 3.0 * t ** 2 + 5.0 * t ** 3 - 7.0 * t ** 4
    for h in (1e-1, 1e-2):
        assert abs(G.central_difference(g, h) - 2.0) < 1e-12
    # leading error -h^4 g^(5)(0) / 30: for g = exp and h = 1e-2, -1e-8 / 30
    assert abs(G.central_difference(np.exp, 1e-2) - (1.0 - 1e-8 / 30.0)) < 1e-12


def test_log_kappa_is_homogeneous_in_A_and_B():
    """kappa scales as lambda^2 under A -> lambda A (the double layer is
    quadratic in A), so d ln kappa along A is 2; <O> does not change."""
    A, B = synth.random_purification(2, 3)
    H = synth.bond_operator_real(synth.random_coefficients(6))
    kw = dict(gamma=2, chi=8, sweeps=3, op=H)
    assert abs(G.purification_directional(A, B, A, 0 * B, 1e-3, **kw) - 2.0) < 1e-9
    assert abs(G.purification_directional(A, B, 0 * A, B, 1e-3, **kw) - 2.0) < 1e-9
    e = G.purification_directional(A, B, A, 0 * B, 1e-3, w_log_kappa=0.0, w_expect=1.0, **kw)
    assert abs(e) < 1e-9


def test_onsager_derivative_of_log_kappa():
    """d ln kappa / d beta = d(-beta f)/d beta = 2 <s s> (two bonds per site),
    taken along da/dbeta; chi = 16 at beta = 0.4."""
    beta = 0.4
    a = synth.ising_square_tensor(beta)
    da = sum(synth.ising_square_tensor_leg_derivative(beta, leg) for leg in range(4))
    fd = G.tensor_directional(a, da, 1e-3, chi=16, sweeps=120)
    assert abs(fd - 2.0 * CF.onsager_nn_correlation(beta)) < 1e-7


@pytest.mark.parametrize("which", [0, 2])
def test_honeycomb_derivative_of_log_kappa(which):
    """ln kappa = 2 (-beta f) per rhombic site, so d ln kappa / dK_w is the
    bond correlation <s_A s_B> on the bonds of type w (Houtappel)."""
    K = (0.3, 0.5, 0.7)
    A, B = synth.honeycomb_ising_tensors(*K)
    dA, dB = synth.honeycomb_ising_tensors_derivative(*K, which)
    fd = G.purification_directional(A, B, dA, dB, 1e-3, gamma=2, chi=16, sweeps=80)
    assert abs(fd - CF.honeycomb_bond_correlation(*K, which=which)) < 1e-7
