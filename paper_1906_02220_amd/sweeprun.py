"""Run CTMRG sweeps of a seeded purification, for profiling.

    python -m paper_1906_02220_amd.sweeprun --D 6 --chi 72 --precision bf16x3 --sweeps 30

Builds the environment of the random purification of `seed` (A then B i.i.d.
N(0,1), each scaled to unit max-abs, fused across the z bond; Sec. III,
Figs. 3(a) and 4) from the boundary start and runs `sweeps` sweeps L, R, U, D
(Fig. 4(c)) in one call, then prints kappa.  Under a kernel trace, the
difference of two runs with different sweep counts is the steady-state cost
of the extra sweeps, free of the start-up work.
"""
import argparse
import sys

# torch first, so that the library binds to torch's HIP runtime
import torch  # noqa: F401

from paper_1906_02220_amd import ctm, synth

PRECISIONS = {"f64": ctm.CTM_PREC_F64, "f32": ctm.CTM_PREC_F32,
              "bf16x3": ctm.CTM_PREC_BF16X3, "bf16x4": ctm.CTM_PREC_BF16X4}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--D", type=int, default=6)
    ap.add_argument("--chi", type=int, default=72)
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--precision", choices=sorted(PRECISIONS), default="bf16x3")
    ap.add_argument("--sweeps", type=int, default=10)
    a = ap.parse_args(argv)
    ctx = ctm.Context(0)
    A, B = synth.random_purification(a.D, a.seed)
    env = ctm.Environment.from_purification(ctx, A, B, 2, a.chi, precision=PRECISIONS[a.precision])
    env.sweep(a.sweeps)
    print("D=%d chi=%d %s: %d sweeps, kappa %.15g" % (a.D, a.chi, a.precision, a.sweeps, env.norm()))
    env.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
