"""Full-update truncation of a gated bond in the CTMRG environment.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy FP64 of
one bond update of the exact-environment full update (Sec. III, Fig. 3(b),
Fig. 4):

1. the gate exp(-tau H/2) on the pseudospins of a gamma bond, split by SVD
   into two gate tensors joined by an index of dimension 4 (oracle.gates);
   contracted with A and B it gives the exact A', B' with a 4D gamma bond;
2. the environment of the composite A'-B' (the gamma bond hidden inside it)
   from CTMRG on the rhombic lattice of those composites, as the bond metric
   E[ket legs][bra legs] of the composite's four outer legs;
3. new tensors A'', B'' with a D gamma bond that minimise the error of the
   purification in that environment,
     d(A'', B'') = sum_p <K'(p) - K''(p), E (K'(p) - K''(p))>,
   K = composite over the gamma bond, p its pseudospin and ancilla index.

Every multi-operand contraction is one ``numpy.einsum`` of its defining
expression, evaluated pairwise (``optimize=True``).

Readings (the paper gives the objective, not the optimiser):
  * the minimisation alternates exact least-squares solves for A'' with B''
    fixed and for B'' with A'' fixed (alternating least squares), starting
    from A'' = A, B'' = B, for a fixed number of rounds (A then B);
  * E is symmetrised, (E + E^T)/2, and every normal matrix N gets the ridge
    1e-12 tr(N)/dim(N) on its diagonal (zero-padded bonds make N singular);
  * the error reported is d / <K', E K'>.
"""
import numpy as np

from . import ctmrg as O
from . import gates

RIDGE = 1e-12


def _perm5(gamma):
    al, be = O._CYCLIC_REST[gamma]
    return [0, 1, 2 + al, 2 + be, 2 + gamma]


def to_fused(T, gamma):
    """[s, a, x, y, z] -> [s, a, alpha, beta, gamma] (l, u, g for A; r, d, g for B)."""
    return np.ascontiguousarray(T.transpose(_perm5(gamma)))


def from_fused(Tp, gamma):
    return np.ascontiguousarray(Tp.transpose(np.argsort(_perm5(gamma))))


def composite_matrix(Ap, Bp):
    """K[(s a t c), (u l d r)] of fused tensors Ap[s,a,l,u,g], Bp[t,c,r,d,g]."""
    K = np.einsum('salug,tcrdg->satculdr', Ap, Bp)
    Du, Dl = Ap.shape[3], Ap.shape[2]
    Dd, Dr = Bp.shape[3], Bp.shape[2]
    return K.reshape(16, Du * Dl * Dd * Dr)


def metric_error(Kt, K, E):
    """sum_p <Kt_p - K_p, E (Kt_p - K_p)>."""
    dK = Kt - K
    return float(np.einsum('pi,ij,pj->', dK, E, dK, optimize=True))


def als_update_A(Kp, E, Bp, D):
    """Least-squares A'' for fixed B'' in the metric E (4 right-hand sides)."""
    Dg = Bp.shape[4]
    E4 = E.reshape(D, D, D, D, D, D, D, D)  # u l d r | u' l' d' r'
    N = np.einsum('tcrdg,uldrvmef,tcfeh->lugmvh', Bp, E4, Bp, optimize=True).reshape(D * D * Dg, D * D * Dg)
    K4 = Kp.reshape(2, 2, 2, 2, D, D, D, D)  # s a t c u l d r
    b = np.einsum('tcrdg,uldrvmef,satcvmef->salug', Bp, E4, K4, optimize=True).reshape(4, D * D * Dg)
    N = N + RIDGE * np.trace(N) / N.shape[0] * np.eye(N.shape[0])
    X = np.linalg.solve(N, b.T)
    return X.T.reshape(2, 2, D, D, Dg)


def als_update_B(Kp, E, Ap, D):
    """Least-squares B'' for fixed A'' in the metric E."""
    Dg = Ap.shape[4]
    E4 = E.reshape(D, D, D, D, D, D, D, D)
    N = np.einsum('salug,uldrvmef,samvh->rdgfeh', Ap, E4, Ap, optimize=True).reshape(D * D * Dg, D * D * Dg)
    K4 = Kp.reshape(2, 2, 2, 2, D, D, D, D)
    b = np.einsum('salug,uldrvmef,satcvmef->tcrdg', Ap, E4, K4, optimize=True).reshape(4, D * D * Dg)
    N = N + RIDGE * np.trace(N) / N.shape[0] * np.eye(N.shape[0])
    X = np.linalg.solve(N, b.T)
    return X.T.reshape(2, 2, D, D, Dg)


def truncate(Ap_gated, Bp_gated, E, A0p, B0p, als_iters):
    """ALS minimisation of the metric error from the start (A0p, B0p).

    Returns (A''p, B''p, errors) with errors[0] at the start and errors[k]
    after k rounds, each divided by <K', E K'>.
    """
    D = A0p.shape[2]
    Kp = composite_matrix(Ap_gated, Bp_gated)
    Es = 0.5 * (E + E.T)
    norm = float(np.einsum('pi,ij,pj->', Kp, Es, Kp, optimize=True))
    Ap, Bp = A0p.copy(), B0p.copy()
    errs = [metric_error(Kp, composite_matrix(Ap, Bp), Es) / norm]
    for _ in range(als_iters):
        Ap = als_update_A(Kp, Es, Bp, D)
        Bp = als_update_B(Kp, Es, Ap, D)
        errs.append(metric_error(Kp, composite_matrix(Ap, Bp), Es) / norm)
    return Ap, Bp, errs


def bond_update(A, B, gamma, H, tau, chi, sweeps, als_iters, eps_cut=O.EPS_CUT_DEFAULT):
    """One eeFU bond update: gate, environment of the gated composite after
    `sweeps` sweeps, ALS truncation back to bond dimension D.

    Returns (A'', B'', errors, E) in the layout of the inputs."""
    D = A.shape[2]
    G = gates.gate(H, tau)
    Ag, Bg = gates.apply_gate(A, B, G, gamma)
    env, a, K, Dc, _ = O.environment_from_purification(Ag, Bg, gamma, chi, sweeps, 0.0, eps_cut)
    E8 = O.bond_metric(env, a, Dc).reshape(D ** 4, D ** 4)
    Ap, Bp, errs = truncate(to_fused(Ag, gamma), to_fused(Bg, gamma), E8,
                           to_fused(A, gamma), to_fused(B, gamma), als_iters)
    return from_fused(Ap, gamma), from_fused(Bp, gamma), errs, E8


TROTTER = ((0, 0.5), (1, 0.5), (2, 1.0), (1, 0.5), (0, 0.5))  # (gamma, fraction of dbeta)


def trotter_step(A, B, H3, dbeta, chi, sweeps, als_iters, eps_cut=O.EPS_CUT_DEFAULT):
    """Second-order Trotter step (Sec. III): G_x(db/2) G_y(db/2) G_z(db)
    G_y(db/2) G_x(db/2) applied right to left, G_gamma(t) the bond update
    with the gate exp(-t H_gamma / 2).  Returns (A, B, error histories)."""
    hist = []
    for gamma, frac in TROTTER:
        A, B, errs, _ = bond_update(A, B, gamma, H3[gamma], frac * dbeta, chi, sweeps, als_iters,
                                    eps_cut)
        hist.append(errs)
    return A, B, hist
