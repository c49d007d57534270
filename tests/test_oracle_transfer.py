"""Pins of the oracle's column transfer matrix (oracle/transfer.py).

The ratio of the leading eigenvalues with and without the site row is the
partition function per site, which must equal the CTMRG norm per site and
Onsager's free energy; a product state has no second eigenvalue; the
symmetric Ising tensor gives the same spectrum along both axes; and the
finite-chi correlation length approaches the exact one from below.
"""
import numpy as np

from oracle import closed_forms as CF, ctmrg as O, transfer as TR
from paper_1906_02220_amd import synth


def _ising_env(beta, chi, sweeps=300):
    a = synth.ising_square_tensor(beta)
    env, _ = O.ctmrg(a, chi, O.boundary_vector_classical(2), sweeps, 1e-13)
    return env, a


def test_leading_eigenvalue_ratio_is_the_free_energy():
    beta = 0.4
    env, a = _ising_env(beta, 16)
    with_site = TR.leading_eigenvalues(env, a, 0, True, 1)[0]
    without = TR.leading_eigenvalues(env, a, 0, False, 1)[0]
    lr = np.log(abs(with_site) / abs(without))
    assert abs(lr - np.log(O.kappa(env, a))) < 1e-9
    assert abs(lr - CF.onsager_minus_beta_f(beta)) < 1e-8


def test_product_state_has_no_second_eigenvalue():
    env, a = _ising_env(0.0, 4, 4)
    ev = TR.leading_eigenvalues(env, a, 0, True, 2)
    assert abs(ev[1]) < 1e-14 * abs(ev[0])
    assert TR.correlation_length(ev) < 1e-2


def test_symmetric_tensor_has_equal_axes_and_xi_below_exact():
    beta = 0.3
    env, a = _ising_env(beta, 16)
    h = TR.leading_eigenvalues(env, a, 0, True, 4)
    v = TR.leading_eigenvalues(env, a, 1, True, 4)
    assert np.allclose(np.abs(h), np.abs(v), rtol=1e-7, atol=0)
    # exact: 1/xi = 2 (K* - K), tanh K* = exp(-2K)
    xi_exact = 1.0 / (2.0 * (np.arctanh(np.exp(-2.0 * beta)) - beta))
    xi = TR.correlation_length(h)
    assert 0.9 * xi_exact < xi < xi_exact
