"""No kernel reads device memory the library never wrote, or writes past
the ends of a buffer.

ctm_debug_poison_allocations fills every buffer the library allocates with
all-ones bytes (NaN doubles, -1 ints) between two guard bands.  Each case
below runs twice in fresh contexts, once with the fill and once without, and
the two runs must agree bit for bit: a read of an unwritten element would
turn the poisoned run's results into NaN or move them, while on a fresh
allocation (usually zeros) or after an earlier run of the same shape (stale
but plausible values) it can go unnoticed.  Every buffer of the poisoned run
is freed before the case ends, and none may have a damaged guard band.  The
shapes cover the direct Jacobi SVD (n <= 128), the subspace SVD with b > chi
and b = n, odd and ragged tile edges, every precision mode, graph replay,
autotuned tilings, the residual-controlled SVD, batches on one and on several
contexts, the grouped lock-step batch, gradients, the bond update and the
transfer spectrum.
"""
import sys

import numpy as np
import pytest

from paper_1906_02220_amd import ctm, synth

pytestmark = pytest.mark.gpu

H = synth.bond_operator_real(synth.random_coefficients(5))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _twice(fn):
    prev = ctm.poison_allocations(False)
    try:
        clean = fn()
        ctm.poison_allocations(True)
        g0 = ctm.guard_violations()
        dirty = fn()
        damaged = ctm.guard_violations() - g0
    finally:
        ctm.poison_allocations(prev)
    assert damaged == 0, "%d guard band(s) damaged: a kernel wrote past a buffer" % damaged
    assert len(clean) == len(dirty)
    for k, (a, b) in enumerate(zip(clean, dirty)):
        a, b = np.asarray(a), np.asarray(b)
        assert np.all(np.isfinite(b)), "output %d not finite with poisoned allocations" % k
        assert np.array_equal(a, b), ("output %d differs with poisoned allocations: max |diff| %.3e"
                                      % (k, float(np.max(np.abs(a - b)))))


def _env_outputs(env):
    return [env.norm(), env.corner_spectra(), env.expect(H), env.bond_metric()]


@pytest.mark.parametrize("D,chi,prec,sweeps", [
    (2, 6, ctm.CTM_PREC_F64, 3),       # n = 24: direct Jacobi SVD of the cut matrix
    (3, 12, ctm.CTM_PREC_F64, 3),      # n = 108, odd tile edges
    (4, 72, ctm.CTM_PREC_F32, 3),      # n = 1152, b = 96 > chi
    (4, 72, ctm.CTM_PREC_F64, 3),
    (7, 32, ctm.CTM_PREC_F32, 2),      # n = 1568, b = 96
    (5, 50, ctm.CTM_PREC_BF16X3, 2),   # ragged slice-GEMM tiles
    (6, 72, ctm.CTM_PREC_BF16X4, 2),
])
def test_sweeps_do_not_read_unwritten_memory(D, chi, prec, sweeps):
    say("case: poisoned allocations, sweeps D=%d chi=%d precision=%d" % (D, chi, prec))
    A, B = synth.random_purification(D, 31 + D)

    def run():
        c = ctm.Context(0)
        e = ctm.Environment.from_purification(c, A, B, 2, chi, precision=prec)
        e.sweep(sweeps)
        out = _env_outputs(e)
        e.close()
        c.close()
        return out
    _twice(run)


def test_graphs_autotune_and_residual_control():
    say("case: poisoned allocations, graph replay + autotune (D=4 chi=40) and svd_tol (D=4 chi=48)")
    A, B = synth.random_purification(4, 41)

    def run():
        c = ctm.Context(0)
        c.graphs(True)
        c.autotune(True)
        e = ctm.Environment.from_purification(c, A, B, 2, 40, precision=ctm.CTM_PREC_BF16X3,
                                              svd_iters=1)
        e.sweep(4)
        out = _env_outputs(e)
        e.close()
        c.close()
        c = ctm.Context(0)
        e = ctm.Environment.from_purification(c, A, B, 2, 48, svd_tol=1e-11)
        e.sweep(2)
        out += _env_outputs(e) + [e.svd_stats()[2]]
        e.close()
        c.close()
        return out
    _twice(run)


@pytest.mark.parametrize("grouped", [False, True])
def test_batches_do_not_read_unwritten_memory(grouped):
    say("case: poisoned allocations, batch of 4 mixed shapes, grouped=%s" % grouped)
    cfg = [(4, 72), (7, 32), (5, 48), (6, 40)]
    ins = [synth.random_purification(D, 778 + i, dtype=np.float32) for i, (D, _) in enumerate(cfg)]

    def run():
        out = []
        for one_ctx in ((True, False) if not grouped else (False,)):
            ctxs = [ctm.Context(0)] if one_ctx else [ctm.Context(0) for _ in cfg]
            envs = [ctm.Environment.from_purification(ctxs[0 if one_ctx else i], A, B, 2, chi,
                                                      precision=ctm.CTM_PREC_F32)
                    for i, ((D, chi), (A, B)) in enumerate(zip(cfg, ins))]
            ctm.sweep_batch(envs, 3, grouped=grouped)
            out += [e.norm() for e in envs]
            for e in envs:
                e.close()
            for c in ctxs:
                c.close()
        return out
    _twice(run)


def test_gradient_bond_update_and_transfer():
    say("case: poisoned allocations, gradient (D=3 chi=12), FU (D=3 chi=12), transfer (D=2 chi=12)")
    A, B = synth.random_purification(3, 51)
    A2, B2 = synth.random_purification(2, 3)

    def run():
        c = ctm.Context(0)
        lk, ex, gA, gB, _ = ctm.grad_purification(c, A, B, 2, 12, 4, op=H, w_log_kappa=1.0,
                                                   w_expect=0.5)
        An, Bn, errs = ctm.fu_bond_update(c, A, B, 2, H, 0.2, 12, 4, 3)
        e = ctm.Environment.from_purification(c, A2, B2, 2, 12)
        e.sweep(10)
        ev, xi = e.transfer_spectrum(0, True, 3, 30)
        e.close()
        c.close()
        return [lk, ex, gA, gB, An, Bn, errs, np.abs(ev), xi]
    _twice(run)
