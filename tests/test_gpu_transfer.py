"""Transfer-matrix spectrum and correlation length (ctm_transfer_spectrum)
against the oracle's dense diagonalisation of the same transfer matrix.

Also pinned on the GPU side: the leading eigenvalue ratio with and without
the site row is the norm per site; a product state has no second
eigenvalue; more Arnoldi steps do not move the leading Ritz values.
"""
import sys

import numpy as np
import pytest

from oracle import ctmrg as O, transfer as TR
from paper_1906_02220_amd import ctm, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = ctm.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("site", [True, False])
def test_purification_spectrum_matches_oracle(ctx, direction, site):
    """D = 2, chi = 12, 20 sweeps of a random purification (seed 3)."""
    say("case: transfer spectrum D=2 chi=12 direction=%d site=%d" % (direction, site))
    A, B = synth.random_purification(2, 3)
    env = ctm.Environment.from_purification(ctx, A, B, 2, 12)
    env.sweep(20)
    ev, xi = env.transfer_spectrum(direction, site, 4, 48)
    oenv, a, _, _, _ = O.environment_from_purification(A, B, 2, 12, 20)
    ref = TR.leading_eigenvalues(oenv, a, direction, site, 4)
    say("  gpu |ev| %s xi %.12f" % (np.array2string(np.abs(ev), precision=12), xi))
    say("  orc |ev| %s xi %.12f" % (np.array2string(np.abs(ref), precision=12),
                                   TR.correlation_length(ref)))
    # the environments themselves agree to about 1e-10; the subleading
    # eigenvalues follow them to a few 1e-9
    assert np.allclose(np.abs(ev), np.abs(ref), rtol=1e-8, atol=0)
    assert abs(xi / TR.correlation_length(ref) - 1.0) < 1e-8


def test_ising_free_energy_and_axes(ctx):
    """Square Ising at beta = 0.4, chi = 16, converged: ln(lambda_1 with the
    site row / lambda_1 without) = ln kappa; both axes agree; the Arnoldi
    Ritz values do not move between 40 and 60 steps."""
    say("case: transfer spectrum Ising beta=0.4 chi=16")
    a = synth.ising_square_tensor(0.4)
    env = ctm.Environment.from_tensor(ctx, a, 16)
    env.sweep(400, 1e-12)
    e1, xi1 = env.transfer_spectrum(0, True, 3, 40)
    e0, _ = env.transfer_spectrum(0, False, 1, 40)
    say("  ln ratio %.15f  ln kappa %.15f  xi %.10f" % (np.log(abs(e1[0]) / abs(e0[0])),
                                                      np.log(env.norm()), xi1))
    assert abs(np.log(abs(e1[0]) / abs(e0[0])) - np.log(env.norm())) < 1e-9
    e2, xi2 = env.transfer_spectrum(1, True, 3, 40)
    assert abs(xi2 / xi1 - 1.0) < 1e-6
    e3, xi3 = env.transfer_spectrum(0, True, 3, 60)
    assert np.allclose(np.abs(e3), np.abs(e1), rtol=1e-10, atol=0)
    oenv, _ = O.ctmrg(a, 16, O.boundary_vector_classical(2), 400, 1e-12)
    ref = TR.leading_eigenvalues(oenv, a, 0, True, 3)
    assert abs(xi1 / TR.correlation_length(ref) - 1.0) < 1e-7


def test_product_state_has_zero_correlation_length(ctx):
    say("case: transfer spectrum of a product state")
    env = ctm.Environment.from_tensor(ctx, synth.ising_square_tensor(0.0), 4)
    env.sweep(4)
    ev, xi = env.transfer_spectrum(0, True, 2, 16)
    # lambda_2 is zero up to rounding (xi = -1/ln(1e-16) = 0.03 at most)
    assert abs(ev[1]) < 1e-12 * abs(ev[0])
    assert xi < 0.05
