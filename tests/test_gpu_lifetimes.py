"""Lifetimes across the C ABI: environments that outlive their context handle.

A context handle may be destroyed while environments created on it are still
alive (as happens at interpreter teardown, when a module-scoped context is
collected before the environments).  Each environment keeps the context's
streams and workspaces alive until it is destroyed itself, so it stays
usable and its destruction is safe.  Before the environments shared the
ownership of the context, this order ended the process with a bus error.
"""
import sys

import numpy as np
import pytest

from paper_1906_02220_amd import ctm, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_environments_outlive_their_context_handle():
    say("case: context handle destroyed before its environments (D=3, chi=12 and D=4, chi=20)")
    A, B = synth.random_purification(3, 2)
    A4, B4 = synth.random_purification(4, 3)
    ref = ctm.Context(0)
    r1 = ctm.Environment.from_purification(ref, A, B, 2, 12)
    r1.sweep(3)
    k_ref = r1.norm()
    r1.close()
    ctx = ctm.Context(0)
    e1 = ctm.Environment.from_purification(ctx, A, B, 2, 12)
    e2 = ctm.Environment.from_purification(ctx, A4, B4, 2, 20)
    e1.sweep(2)
    ctm.sweep_batch([e1, e2], 1)
    lib, h = ctx.lib, ctx.h
    ctx.close()                      # the handle goes first
    assert ctx.h is None
    # the environments still run on the context they were created on
    rc, done, delta = e2.sweep(1)
    assert rc == ctm.CTM_OK and done == 1 and np.isfinite(delta)
    k1 = e1.norm()
    assert abs(k1 / k_ref - 1.0) < 1e-13   # three sweeps, as the reference
    assert np.isfinite(e2.norm())
    e2.close()
    e1.close()                       # the last owner releases the context
    ref.close()
    del lib, h
