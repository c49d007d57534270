"""Hand-written adjoint of the CTMRG environment (ctm_grad_*) on the GPU.

The reference is the derivative by definition: fourth-order central
differences of the oracle's objective (small cases) or of the library's own
forward (the D = 5, chi = 50, 30-sweep workload), plus properties that hold
at any size (Euler homogeneity, invariance under a gauge of the fused bond)
and closed-form Ising correlations, which are derivatives of the free energy.
"""
import sys

import numpy as np
import pytest

from oracle import closed_forms as CF, gradients as OG
from paper_1906_02220_amd import ctm, synth

pytestmark = pytest.mark.gpu

H = synth.bond_operator_real(synth.random_coefficients(6))


@pytest.fixture(scope="module")
def ctx():
    c = ctm.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dirs(shape, seed, count):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal(shape), rng.standard_normal(shape)) for _ in range(count)]


def _dot(gA, gB, dA, dB):
    return float(np.sum(gA * dA) + np.sum(gB * dB))


@pytest.mark.parametrize("D,chi,sweeps,gamma,iters", [(2, 4, 10, 2, 0), (2, 4, 10, 0, 0),
                                                      (4, 16, 8, 2, 6)])
def test_gradient_matches_oracle_differences(ctx, D, chi, sweeps, gamma, iters):
    """D = 2, chi = 4 (n = 16: direct Jacobi SVD) and D = 4, chi = 16
    (n = 256: subspace SVD with 6 iterations per move), both objectives,
    random directions; the oracle uses LAPACK's full SVD.  In these cases the
    kept singular values of every cut matrix stay above 1e-8 of the largest
    (seed 7); where the kept spectrum reaches the rounding level of the cut
    matrix, the derivative is as ill-conditioned as those directions are
    noisy, for the differences as for the adjoint."""
    say("case: gradient vs oracle FD D=%d chi=%d sweeps=%d gamma=%d" % (D, chi, sweeps, gamma))
    A, B = synth.random_purification(D, 7, gamma=gamma)
    kw = dict(svd_iters=iters, svd_iters_cold=iters) if iters else {}
    for wk, wo in ((1.0, 0.0), (0.0, 1.0)):
        lk, ex, gA, gB, info = ctm.grad_purification(ctx, A, B, gamma, chi, sweeps, op=H,
                                                     w_log_kappa=wk, w_expect=wo, **kw)
        for dA, dB in _dirs(A.shape, 11, 2):
            an = _dot(gA, gB, dA, dB)
            fd = OG.purification_directional(A, B, dA, dB, 1e-3, gamma=gamma, chi=chi,
                                             sweeps=sweeps, op=H, w_log_kappa=wk, w_expect=wo)
            say("  w=(%g,%g) adjoint %.12e  oracle FD %.12e  rel %.2e  cg max %d"
                % (wk, wo, an, fd, abs(an - fd) / abs(fd), info["cg_iters_max"]))
            assert abs(an - fd) <= 1e-6 * abs(fd)


def test_checkpointing_gives_identical_gradients(ctx):
    """D = 3, chi = 12, 6 sweeps on the subspace SVD path: recomputing the
    segments from checkpoints every 1 or 4 sweeps reproduces the forward
    bit for bit, so the gradient does not depend on the checkpoint spacing."""
    say("case: checkpoint spacing 0 / 1 / 4, D=3 chi=12")
    A, B = synth.random_purification(3, 4)
    ref = ctm.grad_purification(ctx, A, B, 2, 12, 6, op=H, w_log_kappa=1.0, w_expect=0.5)
    for every in (1, 4):
        got = ctm.grad_purification(ctx, A, B, 2, 12, 6, op=H, w_log_kappa=1.0, w_expect=0.5,
                                    checkpoint_every=every)
        assert got[0] == ref[0] and got[1] == ref[1]
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3])
    # the value is the forward's: the same as a plain environment after 6 sweeps
    env = ctm.Environment.from_purification(ctx, A, B, 2, 12)
    env.sweep(6)
    assert abs(ref[0] - np.log(env.norm())) < 1e-13
    assert abs(ref[1] - env.expect(H)) < 1e-13


def test_homogeneity_and_fused_bond_gauge(ctx):
    """D = 4, chi = 32 (n = 512), 10 sweeps.  kappa scales as lambda^2 under
    A -> lambda A (and B -> lambda B), <O> not at all; a gauge G, G^-T on the
    fused gamma bond leaves the composite, hence both objectives, unchanged."""
    say("case: homogeneity and gamma-bond gauge D=4 chi=32")
    A, B = synth.random_purification(4, 1234)
    X = np.random.default_rng(3).standard_normal((4, 4))
    dA = np.einsum('sauvg,gh->sauvh', A, X)
    dB = -np.einsum('sauvg,hg->sauvh', B, X)
    lk, ex, gA, gB, _ = ctm.grad_purification(ctx, A, B, 2, 32, 10, op=H)
    scale = np.sqrt(np.sum(gA * gA) + np.sum(gB * gB)) * np.sqrt(np.sum(A * A))
    say("  <gA,A> %.15f <gB,B> %.15f gauge %.3e" % (np.sum(gA * A), np.sum(gB * B),
                                                    _dot(gA, gB, dA, dB)))
    assert abs(np.sum(gA * A) - 2.0) < 1e-10
    assert abs(np.sum(gB * B) - 2.0) < 1e-10
    assert abs(_dot(gA, gB, dA, dB)) < 1e-12 * scale
    lk, ex, gA, gB, _ = ctm.grad_purification(ctx, A, B, 2, 32, 10, op=H, w_log_kappa=0.0,
                                              w_expect=1.0)
    scale = np.sqrt(np.sum(gA * gA) + np.sum(gB * gB)) * np.sqrt(np.sum(A * A))
    say("  <O>: <gA,A> %.3e <gB,B> %.3e gauge %.3e scale %.3e"
        % (np.sum(gA * A), np.sum(gB * B), _dot(gA, gB, dA, dB), scale))
    assert abs(np.sum(gA * A)) < 1e-10 * scale
    assert abs(np.sum(gB * B)) < 1e-10 * scale
    assert abs(_dot(gA, gB, dA, dB)) < 1e-10 * scale


def test_onsager_correlation_from_the_gradient(ctx):
    """Square Ising at beta = 0.4, chi = 16, 120 sweeps: d ln kappa / d beta
    along da/dbeta is d(-beta f)/d beta = 2 <s s> (Onsager)."""
    say("case: Ising d ln kappa / d beta, chi=16")
    beta = 0.4
    a = synth.ising_square_tensor(beta)
    da = sum(synth.ising_square_tensor_leg_derivative(beta, leg) for leg in range(4))
    lk, ex, ga, info = ctm.grad_tensor(ctx, a, 16, 120, checkpoint_every=10)
    got = float(np.sum(ga * da))
    say("  %.15f vs %.15f" % (got, 2.0 * CF.onsager_nn_correlation(beta)))
    assert abs(got - 2.0 * CF.onsager_nn_correlation(beta)) < 1e-7
    assert abs(lk - CF.onsager_minus_beta_f(beta)) < 1e-8
    # the impurity objective <E, a_imp> / <E, a> with a_imp = a held fixed: it
    # is 1 at a and scales as 1 / lambda under a -> lambda a
    lk, ex, ga, info = ctm.grad_tensor(ctx, a, 16, 20, a_imp=a, w_log_kappa=0.0, w_expect=1.0)
    assert abs(ex - 1.0) < 1e-13
    assert abs(np.sum(ga * a) + 1.0) < 1e-12


@pytest.mark.parametrize("which", [0, 1, 2])
def test_honeycomb_bond_correlations_from_the_gradient(ctx, which):
    """Honeycomb Ising K = (0.3, 0.5, 0.7) through the double-layer composite,
    chi = 16, 80 sweeps: d ln kappa / dK_w along d(A, B)/dK_w is the
    correlation on the bonds of type w (Houtappel)."""
    say("case: honeycomb d ln kappa / dK_%d" % which)
    K = (0.3, 0.5, 0.7)
    A, B = synth.honeycomb_ising_tensors(*K)
    dA, dB = synth.honeycomb_ising_tensors_derivative(*K, which)
    lk, ex, gA, gB, _ = ctm.grad_purification(ctx, A, B, 2, 16, 80, checkpoint_every=20)
    got = _dot(gA, gB, dA, dB)
    ref = CF.honeycomb_bond_correlation(*K, which=which)
    say("  %.15f vs %.15f" % (got, ref))
    assert abs(got - ref) < 1e-7


def test_c5_workload_against_finite_differences(ctx):
    """D = 5, chi = 50 (n = 1250), 30 sweeps, checkpoints every 5 sweeps,
    seeds 5 (tensors) and 6 (bond operator): d ln kappa and d<H_bond> along
    two random directions and two single coordinates of A, against central
    differences (h = 1e-3 fourth order, h = 1e-6 second order) of the
    library's forward.

    The cut matrices of this random state have about 23 singular values
    above 1e-7 of the largest and then a plateau of values between 1e-8 and
    1e-11, 0.05% apart at chi.  The forward value hardly depends on the
    plateau (its differences agree with the oracle's full-SVD differences to
    1e-10), but the adjoint would use the plateau's singular vectors, which
    no SVD resolves to better than about 1e-4 there.  The projector cutoff is
    therefore raised to eps_cut = 5e-8 (every move's singular values stay at
    least 17% away from it), which drops the plateau from the projectors."""
    say("case: C5 D=5 chi=50 30 sweeps, checkpoints every 5, eps_cut 5e-8")
    A, B = synth.random_purification(5, 5)
    opts = dict(eps_cut=5e-8)

    def forward(Ap, Bp):
        env = ctm.Environment.from_purification(ctx, Ap, Bp, 2, 50, **opts)
        env.sweep(30)
        v = (np.log(env.norm()), env.expect(H))
        env.close()
        return v

    rng = np.random.default_rng(8)
    dirs = [(rng.standard_normal(A.shape), rng.standard_normal(B.shape)) for _ in range(2)]
    for idx in ((0, 0, 1, 2, 3), (1, 1, 4, 0, 2)):
        e = np.zeros(A.shape)
        e[idx] = 1.0
        dirs.append((e, np.zeros(B.shape)))
    for wk, wo in ((1.0, 0.0), (0.0, 1.0)):
        lk, ex, gA, gB, info = ctm.grad_purification(ctx, A, B, 2, 50, 30, op=H, w_log_kappa=wk,
                                                     w_expect=wo, checkpoint_every=5, **opts)
        say("  w=(%g,%g) info %s" % (wk, wo, info))
        gn = np.sqrt(np.sum(gA * gA) + np.sum(gB * gB))
        for dA, dB in dirs:
            an = _dot(gA, gB, dA, dB)
            scale = gn * np.sqrt(np.sum(dA * dA) + np.sum(dB * dB))
            g = lambda t: np.dot((wk, wo), forward(A + t * dA, B + t * dB))
            fd4 = OG.central_difference(g, 1e-3)
            fd2 = (g(1e-6) - g(-1e-6)) / 2e-6
            say("    adjoint %.12e  FD4 %.12e rel %.2e normwise %.2e  FD2(h=1e-6) rel %.2e"
                % (an, fd4, abs(an - fd4) / abs(fd4), abs(an - fd4) / scale,
                   abs(an - fd2) / abs(fd4)))
            assert abs(an - fd4) <= 1e-6 * abs(fd4)
            assert abs(an - fd2) <= 1e-5 * abs(fd4)


def test_gradient_argument_errors(ctx):
    A, B = synth.random_purification(2, 1)
    with pytest.raises(ctm.CtmError) as ei:
        ctm.grad_purification(ctx, A, B, 2, 8, 2, precision=ctm.CTM_PREC_F32)
    assert ei.value.code == ctm.CTM_EINVAL
    with pytest.raises(ctm.CtmError) as ei:
        ctm.grad_purification(ctx, A, B, 2, 8, 2, op=None, w_expect=1.0)
    assert ei.value.code == ctm.CTM_EINVAL
    # zero sweeps: the boundary environment itself
    lk, ex, gA, gB, info = ctm.grad_purification(ctx, A, B, 2, 8, 0, op=H)
    assert info["moves"] == 0 and np.isfinite(lk)
    assert abs(np.sum(gA * A) - 2.0) < 1e-12


def test_torch_autograd_function(ctx):
    """The torch.autograd binding returns the library's value and propagates
    its gradient through further torch arithmetic."""
    import torch
    from paper_1906_02220_amd import autograd as AG
    say("case: torch.autograd binding D=2 chi=4")
    A, B = synth.random_purification(2, 7)
    At = torch.tensor(A, device="cuda", requires_grad=True)
    Bt = torch.tensor(B, device="cuda", requires_grad=True)
    L = AG.purification_objective(ctx, At, Bt, 2, 4, 10, op=H, w_log_kappa=1.0, w_expect=0.5)
    (3.0 * L + L * L).backward()
    lk, ex, gA, gB, _ = ctm.grad_purification(ctx, A, B, 2, 4, 10, op=H, w_log_kappa=1.0,
                                              w_expect=0.5)
    assert abs(L.item() - (lk + 0.5 * ex)) < 1e-14
    f = 3.0 + 2.0 * L.item()
    assert np.allclose(At.grad.cpu().numpy(), f * gA, rtol=1e-13, atol=0)
    assert np.allclose(Bt.grad.cpu().numpy(), f * gB, rtol=1e-13, atol=0)
    a = torch.tensor(synth.ising_square_tensor(0.4), requires_grad=True)
    La = AG.tensor_objective(ctx, a, 8, 10)
    La.backward()
    lk, ex, ga, _ = ctm.grad_tensor(ctx, synth.ising_square_tensor(0.4), 8, 10)
    assert np.array_equal(a.grad.numpy(), ga)
