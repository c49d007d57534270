"""Derivatives of the oracle's CTMRG objectives by finite differences.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The reference value of
a gradient is the derivative by its definition: the limit of difference
quotients of the oracle's own FP64 objective along a direction, evaluated
with the fourth-order central formula

    g'(0) ~ [8 (g(h) - g(-h)) - (g(2h) - g(-2h))] / (12 h),

whose truncation error is -h^4 g^(5)(0) / 30 to leading order.  The
objectives are those of the paper's problem statement (Sec. III): the log
norm per rhombic site and the expectation value of an operator on the fused
bond, after a fixed number of sweeps from the boundary environment, with the
oracle's full-SVD projectors.  Pinned in tests/test_oracle_gradients.py by
Euler homogeneity and by the closed-form Ising correlations (Onsager,
Houtappel), which are derivatives of the free energies.
"""
import numpy as np

from . import ctmrg as O


def central_difference(g, h):
    """Fourth-order central difference of the scalar function g at 0."""
    return (8.0 * (g(h) - g(-h)) - (g(2.0 * h) - g(-2.0 * h))) / (12.0 * h)


def purification_objective(A, B, gamma, chi, sweeps, op=None, op_dim=4, w_log_kappa=1.0,
                           w_expect=0.0, eps_cut=O.EPS_CUT_DEFAULT):
    """w_log_kappa ln(kappa) + w_expect <op> after `sweeps` sweeps from the
    boundary environment of the composite of A and B."""
    env, a, K, D, _ = O.environment_from_purification(A, B, gamma, chi, sweeps, 0.0, eps_cut)
    val = w_log_kappa * np.log(O.kappa(env, a))
    if w_expect != 0.0:
        a_O = O.double_layer(K, O.full_operator(op, op_dim))
        val += w_expect * O.expect(env, a, a_O)
    return val


def tensor_objective(a, chi, sweeps, a_imp=None, w_log_kappa=1.0, w_expect=0.0, b=None,
                     eps_cut=O.EPS_CUT_DEFAULT):
    """w_log_kappa ln(kappa) + w_expect <E, a_imp> / <E, a> for a site tensor a
    after `sweeps` sweeps from the boundary vector b (default e_0)."""
    d = a.shape[0]
    if b is None:
        b = O.boundary_vector_classical(d)
    env, _ = O.ctmrg(a, chi, b, sweeps, 0.0, eps_cut)
    val = w_log_kappa * np.log(O.kappa(env, a))
    if w_expect != 0.0:
        val += w_expect * O.expect(env, a, a_imp)
    return val


def purification_directional(A, B, dA, dB, h, **kw):
    """d/dt of purification_objective(A + t dA, B + t dB) at t = 0."""
    return central_difference(
        lambda t: purification_objective(A + t * dA, B + t * dB, **kw), h)


def tensor_directional(a, da, h, **kw):
    """d/dt of tensor_objective(a + t da) at t = 0."""
    return central_difference(lambda t: tensor_objective(a + t * da, **kw), h)
