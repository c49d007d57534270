"""Full-update bond truncation and Trotter step (ctm_fu_*) against the oracle.

The GPU path computes the gate by scaling and squaring, splits it with its
own Jacobi SVD, builds the environment with the engine's CTMRG and solves
the least-squares problems with its Cholesky kernel; the oracle uses an
eigendecomposition, LAPACK's SVD, its own CTMRG and numpy.linalg.solve.
The ALS iterates are deterministic given the inputs, so A'' and B'' are
compared directly, besides the error histories.
"""
import sys

import numpy as np
import pytest

from oracle import ctmrg as O, fu as OF
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


def _rel(x, y):
    return np.abs(x - y).max() / np.abs(y).max()


@pytest.mark.parametrize("D,chi,gamma,iters", [(2, 8, 0, 0), (2, 8, 1, 0), (2, 8, 2, 0),
                                               (3, 12, 2, 12), (4, 16, 2, 0), (5, 20, 0, 0)])
def test_bond_update_matches_oracle(ctx, D, chi, gamma, iters):
    """D = 2 ... 5: normal matrices of n = D^3 = 8, 27, 64 and 125 unknowns,
    so the one-workgroup Cholesky solve runs its trailing update over n^2
    entries in one pass (n <= 27) and in strided passes of 1024 (n = 64,
    125); the gated composites' cut matrices (chi d = 256, 500) go through
    the subspace SVD."""
    say("case: FU bond update D=%d chi=%d gamma=%d" % (D, chi, gamma))
    A, B = synth.random_purification(D, 21, gamma=gamma)
    H = synth.bond_operator_real(synth.random_coefficients(22))
    kw = dict(svd_iters=iters, svd_iters_cold=iters) if iters else {}
    A2, B2, errs = ctm.fu_bond_update(ctx, A, B, gamma, H, 0.4, chi, 6, 6, **kw)
    Ao, Bo, erro, _ = OF.bond_update(A, B, gamma, H, 0.4, chi, 6, 6)
    say("  errors gpu %s" % np.array2string(errs, precision=10))
    say("  errors orc %s" % np.array2string(np.array(erro), precision=10))
    say("  A'' rel %.2e  B'' rel %.2e" % (_rel(A2, Ao), _rel(B2, Bo)))
    assert np.all(np.abs(errs - np.array(erro)) <= 1e-9 * np.array(erro) + 1e-15)
    assert _rel(A2, Ao) < 1e-8 and _rel(B2, Bo) < 1e-8
    K2, Ko = O.composite(A2, B2, gamma), O.composite(Ao, Bo, gamma)
    assert _rel(K2, Ko) < 1e-9


def test_identity_gate_keeps_the_tensors(ctx):
    say("case: FU bond update with tau = 0")
    A, B = synth.random_purification(2, 5, gamma=1)
    H = synth.bond_operator_real(synth.random_coefficients(6))
    A2, B2, errs = ctm.fu_bond_update(ctx, A, B, 1, H, 0.0, 8, 4, 2)
    assert errs[0] < 1e-26 and errs[-1] < 1e-20
    K0, K2 = O.composite(A, B, 1), O.composite(A2, B2, 1)
    assert _rel(K2, K0) < 1e-10


def test_trotter_step_matches_oracle(ctx):
    """Kitaev-Heisenberg bond terms at phi = -63 degrees, dbeta = 0.05, from
    random D = 2 tensors."""
    say("case: FU Trotter step D=2 chi=8 KH phi=-63")
    phi = np.deg2rad(-63.0)
    H3 = [synth.kitaev_heisenberg_bond(phi, g) for g in range(3)]
    A, B = synth.random_purification(2, 31)
    A2, B2, errs = ctm.fu_trotter_step(ctx, A, B, H3, 0.05, 8, 6, 4)
    Ao, Bo, hist = OF.trotter_step(A, B, H3, 0.05, 8, 6, 4)
    say("  final errors gpu %s" % np.array2string(errs[:, -1], precision=6))
    say("  A rel %.2e B rel %.2e" % (_rel(A2, Ao), _rel(B2, Bo)))
    assert np.allclose(errs, np.array(hist), rtol=1e-7, atol=1e-15)
    assert _rel(A2, Ao) < 1e-7 and _rel(B2, Bo) < 1e-7


def test_fu_argument_errors(ctx):
    A, B = synth.random_purification(2, 1)
    H = np.eye(4)
    o = ctm.default_opts()
    out = np.zeros_like(A)
    rc = ctm.ctm_fu_bond_update(ctx.h, A.ctypes.data_as(ctm._D), B.ctypes.data_as(ctm._D), 2, 3,
                                H.ctypes.data_as(ctm._D), 0.1, 8, o, 2, 2,
                                out.ctypes.data_as(ctm._D), out.ctypes.data_as(ctm._D), None)
    assert rc == ctm.CTM_EINVAL
