"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module only draws or assembles input tensors (site tensors, bond operators,
gauge matrices).  It holds none of the CTMRG arithmetic: no composite or double
layer, no environment, no projector, no contraction of the network.

Workload recipe (Sec. III, Fig. 3a of the paper: the purification has two
sublattice tensors A and B with a pseudospin leg s, an ancilla leg a and three
bond legs x, y, z of dimension D; Table I gives D = 6..8 and chi up to 42):
A and B are drawn i.i.d. standard normal from numpy's default_rng(seed), A
first, each divided by its own max |entry|; the gamma bond (z by default) may
carry the enlarged dimension 4D that a gate produces (Fig. 3b).
"""
import numpy as np

#: pseudospin-1/2 operators S = sigma/2 (Sec. II).  S^y is purely imaginary;
#: only its real-valued products enter real-state expectation values.
SX = 0.5 * np.array([[0.0, 1.0], [1.0, 0.0]])
SZ = 0.5 * np.array([[1.0, 0.0], [0.0, -1.0]])
SY_IM = 0.5 * np.array([[0.0, -1.0], [1.0, 0.0]])  # S^y = i * SY_IM
ID2 = np.eye(2)


def bond_dims(D, D_gamma=None, gamma=2):
    """Bond dimensions (x, y, z) with the gamma bond enlarged to D_gamma."""
    dims = [D, D, D]
    dims[gamma] = D if D_gamma is None else D_gamma
    return tuple(dims)


def random_purification(D, seed, D_gamma=None, gamma=2, dtype=np.float64):
    """Seeded random sublattice tensors A, B of shape (2, 2, Dx, Dy, Dz).

    Entries are i.i.d. N(0, 1) (A drawn first, then B), each tensor scaled to
    unit max-abs.  Returned C-contiguous, row-major [s][a][x][y][z].
    """
    rng = np.random.default_rng(seed)
    shape = (2, 2) + bond_dims(D, D_gamma, gamma)
    A = rng.standard_normal(shape)
    B = rng.standard_normal(shape)
    A /= np.abs(A).max()
    B /= np.abs(B).max()
    return np.ascontiguousarray(A, dtype=dtype), np.ascontiguousarray(B, dtype=dtype)


def random_site_tensor(d, seed):
    """Seeded random rank-4 classical site tensor a[u,l,d,r], unit max-abs."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((d, d, d, d))
    return a / np.abs(a).max()


def random_coefficients(seed):
    """Seeded 3x3 coefficients c[alpha, beta] of a two-spin bond operator."""
    return np.random.default_rng(seed).standard_normal((3, 3))


def bond_operator_real(c):
    """Real part of H = sum_{alpha,beta} c[alpha,beta] S^alpha_A S^beta_B.

    Index order of the 4x4 result is (s_A, s_B) x (s_A', s_B').  Terms with a
    single S^y are imaginary and drop out; S^y S^y = -(SY_IM x SY_IM) is real.
    """
    ops = [SX, None, SZ]
    H = np.zeros((4, 4))
    for al in range(3):
        for be in range(3):
            if al == 1 and be == 1:
                H += c[1, 1] * (-np.kron(SY_IM, SY_IM))
            elif al != 1 and be != 1:
                H += c[al, be] * np.kron(ops[al], ops[be])
    return H


def kitaev_heisenberg_bond(phi, gamma, A=1.0):
    """Real 4x4 Kitaev-Heisenberg bond term J S.S + K S^g S^g (Eq. 2-3).

    J = A cos(phi), K = 2 A sin(phi); gamma in {0, 1, 2} for x, y, z.
    """
    J = A * np.cos(phi)
    K = 2.0 * A * np.sin(phi)
    c = J * np.eye(3)
    c[gamma, gamma] += K
    return bond_operator_real(c)


def ising_square_tensor(beta):
    """Classical square-lattice Ising site tensor with one spin per tensor.

    The bond weight Q = [[e^b, e^-b], [e^-b, e^b]] is split as Q = W W^T with
    W = U diag(sqrt(lambda)), lambda = (2 cosh b, 2 sinh b), U the 2x2
    Hadamard; a[u,l,d,r] = sum_s W[s,u] W[s,l] W[s,d] W[s,r].
    """
    lam = np.array([2.0 * np.cosh(beta), 2.0 * np.sinh(beta)])
    U = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    W = U * np.sqrt(lam)[None, :]
    return np.einsum('su,sl,sd,sr->uldr', W, W, W, W)


def _bond_split(K):
    """Return V with V V^T = [[e^K, e^-K], [e^-K, e^K]] (K >= 0)."""
    lam = np.array([2.0 * np.cosh(K), 2.0 * np.sinh(K)])
    U = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    return U * np.sqrt(lam)[None, :]


def honeycomb_ising_tensors(Kx, Ky, Kz):
    """Honeycomb Ising model written as a two-sublattice state (D = 2).

    Each layer carries half of every bond weight: the weight e^{(K_g/2) s s'}
    of bond type g is split as V_g V_g^T, and A[s, a, x, y, z] =
    V_x[s,x] V_y[s,y] V_z[s,z] delta_{a0}, B the same.  The ket amplitude is
    then exp(sum_<ij> (K_g/2) s_i s_j), so the double-layer norm network equals
    the classical partition function at couplings (Kx, Ky, Kz), and
    <sigma^z_A sigma^z_B> on a bond is the classical nearest-neighbour
    correlation.
    """
    Vx, Vy, Vz = _bond_split(0.5 * Kx), _bond_split(0.5 * Ky), _bond_split(0.5 * Kz)
    A = np.zeros((2, 2, 2, 2, 2))
    A[:, 0] = np.einsum('sx,sy,sz->sxyz', Vx, Vy, Vz)
    return A.copy(), A.copy()


def honeycomb_ising_tensors_derivative(Kx, Ky, Kz, which):
    """d(A, B)/dK_which of honeycomb_ising_tensors: V_g is replaced by its
    derivative on the leg of bond type ``which``."""
    Ks = [Kx, Ky, Kz]
    Vs = [_bond_split(0.5 * k) for k in Ks]
    k = 0.5 * Ks[which]
    lam = np.array([2.0 * np.cosh(k), 2.0 * np.sinh(k)])
    dlam = np.array([2.0 * np.sinh(k), 2.0 * np.cosh(k)])
    U = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    Vs[which] = U * (0.25 * dlam / np.sqrt(lam))[None, :]
    dA = np.zeros((2, 2, 2, 2, 2))
    dA[:, 0] = np.einsum('sx,sy,sz->sxyz', *Vs)
    return dA.copy(), dA.copy()


def singlet_tensors():
    """Infinite-temperature purification, D = 1: every pseudospin maximally
    entangled with its ancilla, A[s,a] = (delta_s0 delta_a1 - delta_s1 delta_a0)/sqrt 2."""
    A = np.zeros((2, 2, 1, 1, 1))
    A[0, 1, 0, 0, 0] = 1.0 / np.sqrt(2.0)
    A[1, 0, 0, 0, 0] = -1.0 / np.sqrt(2.0)
    return A.copy(), A.copy()


def random_invertible(n, seed, cond_max=10.0):
    """Seeded well-conditioned random n x n matrix and its inverse."""
    rng = np.random.default_rng(seed)
    while True:
        G = np.eye(n) + 0.5 * rng.standard_normal((n, n)) / np.sqrt(n)
        if np.linalg.cond(G) < cond_max:
            return G, np.linalg.inv(G)


def pad_and_gauge(A, B, D_new, seed):
    """Zero-pad every bond of A and B to D_new and insert a random G, G^-1 pair
    on each bond type (A side gets G, B side gets G^-1 transposed), leaving the
    contracted network unchanged."""
    shp = A.shape
    Ap = np.zeros((2, 2, D_new, D_new, D_new))
    Bp = np.zeros((2, 2, D_new, D_new, D_new))
    Ap[:, :, :shp[2], :shp[3], :shp[4]] = A
    Bp[:, :, :shp[2], :shp[3], :shp[4]] = B
    for g in range(3):
        G, Gi = random_invertible(D_new, seed + 17 * g)
        Ap = np.moveaxis(np.tensordot(Ap, G, axes=([2 + g], [0])), -1, 2 + g)
        Bp = np.moveaxis(np.tensordot(Bp, Gi.T, axes=([2 + g], [0])), -1, 2 + g)
    return np.ascontiguousarray(Ap), np.ascontiguousarray(Bp)


def ising_square_tensor_leg_derivative(beta, leg):
    """The square Ising site tensor with W replaced by dW/dbeta on one leg
    (leg 0..3 = u, l, d, r).  Summing the two such tensors at the two ends of a
    bond gives the derivative of that bond's weight, i.e. an s_i s_j insertion."""
    lam = np.array([2.0 * np.cosh(beta), 2.0 * np.sinh(beta)])
    dlam = np.array([2.0 * np.sinh(beta), 2.0 * np.cosh(beta)])
    U = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    W = U * np.sqrt(lam)[None, :]
    dW = U * (0.5 * dlam / np.sqrt(lam))[None, :]
    Ws = [W, W, W, W]
    Ws[leg] = dW
    return np.einsum('su,sl,sd,sr->uldr', *Ws)


def random_symmetric(n, seed):
    """Seeded random real symmetric n x n matrix."""
    M = np.random.default_rng(seed).standard_normal((n, n))
    return 0.5 * (M + M.T)


def gauge_bonds(A, B, seed, dims=None):
    """Insert a random G, G^-1 pair on each bond type without padding."""
    Ap, Bp = A, B
    for g in range(3):
        n = A.shape[2 + g]
        if n == 1:
            continue
        G, Gi = random_invertible(n, seed + 17 * g)
        Ap = np.moveaxis(np.tensordot(Ap, G, axes=([2 + g], [0])), -1, 2 + g)
        Bp = np.moveaxis(np.tensordot(Bp, Gi.T, axes=([2 + g], [0])), -1, 2 + g)
    return np.ascontiguousarray(Ap), np.ascontiguousarray(Bp)
