"""Write the full-size parity values of the D = 6, chi = 72 workload, or of
the largest member of the ragged batch (D = 7, chi = 96).

    python tests/golden/make_c3_golden.py 2    # two sweeps, about 2 minutes on 8 cores
    python tests/golden/make_c3_golden.py 20   # twenty sweeps, about 20 minutes
    python tests/golden/make_c3_golden.py 2 ragged   # D = 7, chi = 96, about 10 minutes

The ragged member is member 25 of the 32 purifications of the batch
benchmark ((D, chi) drawn uniformly from {4,5,6,7} x {32,48,72,96} with
seed 777): seed 778 + 25 = 803, entries drawn in FP32 (then used as FP64);
it is written to c4_D7_chi96_<sweeps>_sweeps.json with the same fields.


Runs the FP64 oracle only (oracle/ctmrg.py): the purification of seed 1234
(A then B i.i.d. N(0,1), each scaled to unit max-abs), fused across the z
bond (Sec. III, Fig. 4(b)), environment from the boundary start, two full
sweeps L, R, U, D (Fig. 4(c)), then the observables of the fused bond
(Sec. III, last paragraph): kappa, <H_bond> for the seeded real bond
operator, the bond metric E (its Frobenius norm, three projections on
seeded random tensors, its largest |entry| and the entries at 65536 sampled
flat indices), the corner spectra, and for every move the gap
s_chi / s_(chi+1) of the cut spectrum.

Sampled entries: flat index i_k = (7919 k + 13) mod D^8 of the bond metric
in its layout [u_k][l_k][d_k][r_k][u_b][l_b][d_b][r_b], k = 0 .. 65535
(7919 is prime and D^8 = 2^8 3^8, so the indices are distinct and spread
over every leg).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import ctmrg as O  # noqa: E402
from paper_1906_02220_amd import synth  # noqa: E402

D, CHI, SEED, GAMMA = 6, 72, 1234, 2
PROJ_SEEDS = (101, 102, 103)
N_SAMPLES, SAMPLE_STRIDE, SAMPLE_OFFSET = 65536, 7919, 13


def sample_indices(size):
    """Flat indices of the stored bond-metric entries."""
    k = np.arange(N_SAMPLES, dtype=np.int64)
    return (SAMPLE_STRIDE * k + SAMPLE_OFFSET) % size


RAGGED = {"D": 7, "chi": 96, "seed": 803, "dtype": "float32", "prefix": "c4"}


def out_path(sweeps, prefix="c3", d=D, chi=CHI):
    return os.path.join(HERE, "%s_D%d_chi%d_%d_sweeps.json" % (prefix, d, chi, sweeps))


def projections(E8):
    out = []
    for s in PROJ_SEEDS:
        R = np.random.default_rng(s).standard_normal(E8.shape)
        out.append(float(np.vdot(E8, R) / np.linalg.norm(R)))
    return out


def main(SWEEPS, ragged=False):
    global D, CHI, SEED
    prefix, dtype = "c3", np.float64
    if ragged:
        D, CHI, SEED, prefix, dtype = (RAGGED["D"], RAGGED["chi"], RAGGED["seed"], RAGGED["prefix"],
                                       np.float32)
    t0 = time.time()
    A, B = synth.random_purification(D, SEED, dtype=dtype)
    A, B = A.astype(np.float64), B.astype(np.float64)
    K = O.composite(A, B, GAMMA)
    a = O.double_layer(K)
    arot = [O.rotate(a, k) for k in range(4)]
    env = O.init_env(D * D, CHI, O.boundary_vector_double_layer(D))
    gaps, cut_margin = [], []
    for _ in range(SWEEPS):
        for k in O.MOVE_ORDER:
            s = O.left_move(env, arot, k, CHI)
            gaps.append(float(s[CHI - 1] / s[CHI]) if s[CHI] > 0 else float("inf"))
            r = s[:CHI] / s[0]
            near = np.abs(np.log10(r[r > 0]) + 12.0)
            cut_margin.append(float(near.min()) if near.size else float("inf"))
    H = synth.bond_operator_real(synth.random_coefficients(6))
    kap = float(O.kappa(env, a))
    e_h = float(O.expect(env, a, O.double_layer(K, O.full_operator(H, 4))))
    E8 = O.bond_metric(env, a, D)
    spectra = np.array(O.corner_spectra(env))
    res = {
        "source": "oracle/ctmrg.py via tests/golden/make_c3_golden.py",
        "passage": "arXiv:1906.02220 Sec. III, Figs. 3(a) and 4",
        "D": D, "chi": CHI, "seed": SEED, "gamma": GAMMA, "sweeps": SWEEPS,
        "entries": "float32" if ragged else "float64",
        "kappa": kap, "energy_bond": e_h,
        "bond_metric_norm": float(np.linalg.norm(E8)),
        "bond_metric_projections": projections(E8),
        "projection_seeds": list(PROJ_SEEDS),
        "bond_metric_max_abs": float(np.abs(E8).max()),
        "bond_metric_sample": {"count": N_SAMPLES, "stride": SAMPLE_STRIDE,
                               "offset": SAMPLE_OFFSET,
                               "values": [float(v) for v in E8.reshape(-1)[sample_indices(E8.size)]]},
        "corner_spectra": spectra.tolist(),
        "cut_gap_per_move": gaps,
        "cut_margin_decades_per_move": cut_margin,
        "oracle_seconds": round(time.time() - t0, 1),
    }
    out = out_path(SWEEPS, prefix, D, CHI)
    with open(out, "w") as f:
        json.dump(res, f)
    print("wrote %s (kappa %.15g, <H> %.15g, min gap %.6f, %.0f s)" % (
        out, kap, e_h, min(gaps), res["oracle_seconds"]))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2, len(sys.argv) > 2 and sys.argv[2] == "ragged")
