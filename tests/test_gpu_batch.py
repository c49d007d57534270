"""Batched sweeps and graph replay.

ctm_sweep_batch runs one sweep of every environment per round, with
environments on different contexts overlapping on their streams; graph
replay captures one warm sweep into a HIP graph.  Neither changes the
arithmetic: every kernel of an environment runs in the same order with the
same arguments, so the results must equal those of plain ctm_sweep calls
exactly (the oracle parity of the plain path is covered elsewhere).
"""
import sys

import numpy as np
import pytest

from oracle import ctmrg as O
from paper_1906_02220_amd import ctm, synth

pytestmark = pytest.mark.gpu

H = synth.bond_operator_real(synth.random_coefficients(6))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _env(ctx, D, chi, seed, gamma=2, **kw):
    A, B = synth.random_purification(D, seed, gamma=gamma)
    return ctm.Environment.from_purification(ctx, A, B, gamma, chi, **kw)


def _state(env):
    return env.norm(), env.expect(H), env.corner_spectra(), env.bond_metric()


def _same(s1, s2):
    k1, e1, sp1, E1 = s1
    k2, e2, sp2, E2 = s2
    assert k1 == k2
    assert e1 == e2
    assert np.array_equal(sp1, sp2)
    assert np.array_equal(E1, E2)


def test_graph_replay_matches_eager_sweep_by_sweep():
    """D = 4, chi = 32 (subspace SVD with warm starts): every sweep replayed
    from the graph, with observables computed eagerly between replays,
    equals the eager sweep.  A fixed iteration count lets the graph be
    captured from the third sweep on."""
    say("case: graph replay D=4 chi=32 seed=1234, 8 sweeps")
    ce, cg = ctm.Context(0), ctm.Context(0)
    cg.graphs(True)
    ee, eg = _env(ce, 4, 32, 1234, svd_iters=1), _env(cg, 4, 32, 1234, svd_iters=1)
    for s in range(8):
        r1, r2 = ee.sweep(1), eg.sweep(1)
        assert r1 == r2
        _same(_state(ee), _state(eg))
    # a state change drops the graph; replay resumes after two warm sweeps
    C, T, logs = ee.get()
    ee.set(C, T, logs)
    eg.set(C, T, logs)
    for s in range(4):
        assert ee.sweep(1) == eg.sweep(1)
        _same(_state(ee), _state(eg))
    ce.close()
    cg.close()


def test_graph_replay_with_automatic_iteration_count():
    """The automatic subspace iteration count runs two iterations for the
    first eight warm moves of each direction and one afterwards; the graph is
    captured only once the count has settled (from the tenth sweep on).
    Sweep by sweep, 14 sweeps with graphs on equal the eager sweeps."""
    say("case: graph replay D=4 chi=32 seed=99, automatic iteration count, 14 sweeps")
    ce, cg = ctm.Context(0), ctm.Context(0)
    cg.graphs(True)
    ee, eg = _env(ce, 4, 32, 99), _env(cg, 4, 32, 99)
    for s in range(14):
        r1, r2 = ee.sweep(1), eg.sweep(1)
        assert r1 == r2
        _same(_state(ee), _state(eg))
    calls, iters, _ = ee.svd_stats()
    # 4 cold calls of 5 iterations, 32 warm calls of 2, the rest 1
    assert calls == 56 and iters == 4 * 5 + 32 * 2 + 20 * 1
    ce.close()
    cg.close()


CASES = [(2, 12, 3, 2), (3, 20, 4, 1), (4, 32, 1234, 2), (2, 30, 5, 0)]


def test_sweep_batch_matches_sequential():
    """Four environments of different D and chi (direct-Jacobi and subspace
    SVD paths, three bond types), each on its own context, two of them with
    graph replay."""
    say("case: batch of %d environments, 10 sweeps" % len(CASES))
    ctxs = [ctm.Context(0) for _ in CASES]
    for c in ctxs[::2]:
        c.graphs(True)
    batch = [_env(c, D, chi, seed, gamma) for c, (D, chi, seed, gamma) in zip(ctxs, CASES)]
    rc, done, delta = ctm.sweep_batch(batch, 10, 0.0)
    assert rc == ctm.CTM_OK and list(done) == [10] * len(CASES)
    cs = ctm.Context(0)
    for (D, chi, seed, gamma), eb, db in zip(CASES, batch, delta):
        es = _env(cs, D, chi, seed, gamma)
        rcs, ds, dels = es.sweep(10)
        assert dels == db
        _same(_state(eb), _state(es))
    # one member against the oracle as well
    A, B = synth.random_purification(3, 4, gamma=1)
    oenv, a, _, _, _ = O.environment_from_purification(A, B, 1, 20, 10)
    assert abs(batch[1].norm() / O.kappa(oenv, a) - 1.0) < 1e-10


@pytest.mark.parametrize("prec", [ctm.CTM_PREC_F32, ctm.CTM_PREC_F64])
def test_many_concurrent_members_match_plain_sweeps(prec):
    """24 purifications with (D, chi) uniform on {4,5,6} x {32,48,72}
    (seed 777), each on its own context so that their kernels share the CUs,
    against the same members swept alone: bit for bit.  This is the setting
    in which an unsynchronised read of the sign pivot in the singular-vector
    sign fix (a wave could read the pivot after another wave had already
    flipped it, and leave its own rows unflipped) once gave one member a
    kappa off by 5e-6."""
    say("case: 24 concurrent members, 3 sweeps, precision %d" % prec)
    rng = np.random.default_rng(777)
    cfg = list(zip(rng.choice([4, 5, 6], size=24).tolist(), rng.choice([32, 48, 72], size=24).tolist()))
    ins = [synth.random_purification(D, 778 + i, dtype=np.float32) for i, (D, _) in enumerate(cfg)]
    ctxs = [ctm.Context(0) for _ in cfg]
    batch = [ctm.Environment.from_purification(c, A, B, 2, chi, precision=prec)
             for c, (D, chi), (A, B) in zip(ctxs, cfg, ins)]
    rc, done, delta = ctm.sweep_batch(batch, 3, 0.0)
    assert rc == ctm.CTM_OK
    kb = [e.norm() for e in batch]
    for e in batch:
        e.close()
    for c in ctxs:
        c.close()
    cs = ctm.Context(0)
    bad = []
    for i, ((D, chi), (A, B)) in enumerate(zip(cfg, ins)):
        es = ctm.Environment.from_purification(cs, A, B, 2, chi, precision=prec)
        _, _, dels = es.sweep(3)
        if not (dels == delta[i] and es.norm() == kb[i]):
            bad.append((i, D, chi, dels, delta[i], es.norm(), kb[i]))
        es.close()
    cs.close()
    for b in bad:
        say("  member %d D=%d chi=%d: delta %.17g vs %.17g, kappa %.17g vs %.17g" % b)
    assert not bad


def test_sweep_batch_tolerance_and_sharing_a_context():
    """With tol > 0 each environment stops on its own; environments may share
    a context (they then run in turn on its stream)."""
    say("case: batch with tol=1e-9 on one shared context")
    ctx = ctm.Context(0)
    tensors = [synth.ising_square_tensor(0.3), synth.ising_square_tensor(0.38)]
    envs = [ctm.Environment.from_tensor(ctx, a, 8) for a in tensors]
    rc, done, delta = ctm.sweep_batch(envs, 400, 1e-9)
    say("  done %s delta %s" % (list(done), list(delta)))
    assert rc == ctm.CTM_OK
    assert np.all(delta < 1e-9)
    for a, d, dl in zip(tensors, done, delta):
        _, dr, delr = ctm.Environment.from_tensor(ctx, a, 8).sweep(400, 1e-9)
        assert dr == d and delr == dl
    one = ctm.Environment.from_tensor(ctx, tensors[0], 8)
    rc, done, delta = ctm.sweep_batch([one], 2, 1e-300)
    assert rc == ctm.CTM_ENOTCONV and list(done) == [2]


def test_sweep_batch_reports_the_failing_environment():
    say("case: batch with a non-finite environment")
    c1, c2 = ctm.Context(0), ctm.Context(0)
    good = _env(c1, 2, 12, 3)
    A, B = synth.random_purification(2, 1)
    A = A.copy()
    A[0, 0, 0, 0, 0] = np.nan
    bad = ctm.Environment.from_purification(c2, A, B, 2, 12)
    with pytest.raises(ctm.CtmError) as ei:
        ctm.sweep_batch([good, bad], 3, 0.0)
    assert ei.value.code == ctm.CTM_ENUMERIC
    assert "environment 1" in str(ei.value)
    # the good environment is still usable
    assert np.isfinite(good.norm())


@pytest.mark.parametrize("mode", [ctm.CTM_PREC_F64, ctm.CTM_PREC_F32])
def test_autotuned_tilings_give_identical_results(mode):
    """D = 4, chi = 32 (n = 512, 512 x 512 x 512 and 1024 x 256 x 256
    products): the autotuner may pick any tiling, all accumulate in the same
    order."""
    say("case: autotune on vs off, precision mode %d" % mode)
    c0, c1 = ctm.Context(0), ctm.Context(0)
    c1.autotune(True)
    e0 = _env(c0, 4, 32, 1234, precision=mode)
    e1 = _env(c1, 4, 32, 1234, precision=mode)
    assert e0.sweep(6) == e1.sweep(6)
    _same(_state(e0), _state(e1))


# (D, chi, seed, gamma, precision): F64 at n = 512 (grouped, FP64 tile
# kernel), F32 at n = 512 and n = 500 (grouped, FP32 tile kernel), F64 at
# n = 1152 (split-K in a plain sweep, so not grouped), BF16x3 (not grouped),
# F64 at n = 180 (generic kernel, not grouped) and D = 2 (direct SVD)
GROUPED = [(4, 32, 1234, 2, ctm.CTM_PREC_F64), (4, 32, 7, 1, ctm.CTM_PREC_F32),
           (5, 20, 11, 0, ctm.CTM_PREC_F32), (4, 72, 5, 2, ctm.CTM_PREC_F64),
           (4, 32, 8, 2, ctm.CTM_PREC_BF16X3), (3, 20, 4, 1, ctm.CTM_PREC_F64),
           (2, 12, 3, 2, ctm.CTM_PREC_F64)]


def test_grouped_batch_matches_sequential():
    """Lock-step batch with grouped n x n x n products equals plain sweeps
    bit for bit, for grouped and ungrouped members alike; two members share
    a context, one context has graphs on (its graph is dropped)."""
    say("case: grouped batch of %d environments, 6 sweeps" % len(GROUPED))
    ctxs = [ctm.Context(0) for _ in GROUPED[:-1]]
    ctxs.append(ctxs[0])
    ctxs[1].graphs(True)
    batch = [_env(c, D, chi, seed, gamma, precision=p, svd_iters=1)
             for c, (D, chi, seed, gamma, p) in zip(ctxs, GROUPED)]
    batch[1].sweep(3)  # captures a graph on the graph-enabled context
    rc, done, delta = ctm.sweep_batch(batch, 6, 0.0, grouped=True)
    assert rc == ctm.CTM_OK and list(done) == [6] * len(GROUPED)
    cs = ctm.Context(0)
    for i, ((D, chi, seed, gamma, p), eb, db) in enumerate(zip(GROUPED, batch, delta)):
        say("  member %d: D=%d chi=%d precision %d" % (i, D, chi, p))
        es = _env(cs, D, chi, seed, gamma, precision=p, svd_iters=1)
        _, _, dels = es.sweep(9 if i == 1 else 6)
        assert dels == db
        _same(_state(eb), _state(es))
    # graph replay resumes on the member whose graph was dropped
    es = _env(cs, 4, 32, 7, 1, precision=ctm.CTM_PREC_F32, svd_iters=1)
    es.sweep(9)
    assert batch[1].sweep(3) == es.sweep(3)
    _same(_state(batch[1]), _state(es))


def test_grouped_batch_tolerance_and_errors():
    say("case: grouped batch with tol, ENOTCONV and a non-finite member")
    c1, c2 = ctm.Context(0), ctm.Context(0)
    envs = [_env(c1, 4, 32, 1234), _env(c2, 4, 32, 7, 1)]
    rc, done, delta = ctm.sweep_batch(envs, 40, 1e-6, grouped=True)
    say("  rc %d done %s delta %s" % (rc, list(done), list(delta)))
    # each member stops on its own, exactly where a plain sweep loop stops
    for (D, chi, seed, gamma), d, dl in zip([(4, 32, 1234, 2), (4, 32, 7, 1)], done, delta):
        rcs, dr, delr = _env(c1, D, chi, seed, gamma).sweep(40, 1e-6)
        assert dr == d and delr == dl
        assert (rcs == ctm.CTM_OK) == (dl < 1e-6)
    assert (rc == ctm.CTM_OK) == bool(np.all(delta < 1e-6))
    rc, done, delta = ctm.sweep_batch([_env(c1, 2, 12, 3)], 2, 1e-300, grouped=True)
    assert rc == ctm.CTM_ENOTCONV and list(done) == [2]
    A, B = synth.random_purification(4, 1)
    A = A.copy()
    A[0, 0, 0, 0, 0] = np.nan
    bad = ctm.Environment.from_purification(c2, A, B, 2, 32)
    good = _env(c1, 4, 32, 3)
    with pytest.raises(ctm.CtmError) as ei:
        ctm.sweep_batch([good, bad], 3, 0.0, grouped=True)
    assert ei.value.code == ctm.CTM_ENUMERIC
    assert "environment 1" in str(ei.value)
    assert np.isfinite(good.norm())


def test_grouped_batch_splits_large_groups():
    """20 FP32 environments at n = 512: 40 half-system products per phase,
    more than one grouped launch holds (32), still equal to plain sweeps."""
    say("case: grouped batch of 20 environments (two grouped launches per phase)")
    ctxs = [ctm.Context(0) for _ in range(20)]
    batch = [_env(c, 4, 32, 500 + i, gamma=i % 3, precision=ctm.CTM_PREC_F32)
             for i, c in enumerate(ctxs)]
    rc, done, delta = ctm.sweep_batch(batch, 3, 0.0, grouped=True)
    assert rc == ctm.CTM_OK and list(done) == [3] * 20
    cs = ctm.Context(0)
    for i in (0, 7, 19):
        es = _env(cs, 4, 32, 500 + i, gamma=i % 3, precision=ctm.CTM_PREC_F32)
        _, _, dels = es.sweep(3)
        assert dels == delta[i]
        _same(_state(batch[i]), _state(es))


def test_batch_argument_errors():
    """Empty batches are a no-op; null members, repeated members and negative
    counts are refused without touching any environment."""
    say("case: batch argument errors")
    c = ctm.Context(0)
    e = _env(c, 2, 12, 3)
    lib = ctm.load_library()
    for name in ("ctm_sweep_batch", "ctm_sweep_batch_grouped"):
        fn = getattr(lib, name)
        assert fn((ctm._P * 1)(), 0, 3, 0.0, None, None) == ctm.CTM_OK
        assert fn((ctm._P * 1)(None), 1, 3, 0.0, None, None) == ctm.CTM_EINVAL
        arr = (ctm._P * 2)(e.h, e.h)
        assert fn(arr, 2, 3, 0.0, None, None) == ctm.CTM_EINVAL
        assert "twice" in lib.ctm_last_error(c.h).decode()
        assert fn((ctm._P * 1)(e.h), -1, 3, 0.0, None, None) == ctm.CTM_EINVAL
        assert fn((ctm._P * 1)(e.h), 1, -2, 0.0, None, None) == ctm.CTM_EINVAL
    # the environment is untouched and still sweeps
    assert e.sweep(2)[0] == ctm.CTM_OK
