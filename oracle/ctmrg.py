"""Plain FP64 CTMRG on the rhombic (square) lattice of composite tensors.

TEST INFRASTRUCTURE ONLY (see the package docstring): a slow, obviously
correct reference for the HIP path.  Every contraction is one ``numpy.einsum``
of the defining expression; the projector SVD is LAPACK's full SVD.

Paper references (arXiv:1906.02220):
  * Sec. III and Fig. 3(a): purification tensors A, B with a pseudospin, an
    ancilla and three bond legs x, y, z.
  * Fig. 3(b): after a gate the gamma bond has dimension 4D.
  * Sec. III, Fig. 4(a): ket and bra layers contracted into double tensors.
  * Sec. III, Fig. 4(b): the two double tensors joined by a gamma bond are
    fused into one composite ("quadruple") tensor with all bonds D^2; the
    composites form a rhombic lattice, i.e. a square lattice.
  * Sec. III, Fig. 4(c): CTMRG replaces the semi-infinite sectors by corner
    tensors C and edge tensors (called E in the paper, T here) of bond chi.
  * Sec. III, last paragraph: the environment of the gamma bond obtained from
    CTMRG is what the full update needs.

Where the paper defers to the cited CTMRG literature, the readings used here
are listed in the repository's design notes and in the docstrings below.

Conventions
-----------
Site tensor ``a[u, l, d, r]`` (row-major), each leg of dimension ``d``.
Environment, clockwise from the top-left: C1, T1, C2, T2, C3, T3, C4, T4,
stored as ``C[0..3]`` and ``T[0..3]``.  A corner ``C[a, b]`` has ``a`` on the
counter-clockwise neighbour and ``b`` on the clockwise one; an edge
``T[a, m, b]`` likewise, with ``m`` pointing into the lattice.  Rotating the
lattice by 90 degrees counter-clockwise maps (C, T)[i] -> (C, T)[i+1] and
``a -> a.transpose(3, 0, 1, 2)``, so every directional move is the left move
of a rotated frame.
"""
import numpy as np

EPS_CUT_DEFAULT = 1e-12

def _c(spec, x, y):
    """One pairwise contraction written as its einsum expression (BLAS-backed)."""
    return np.einsum(spec, x, y, optimize=True)


# --------------------------------------------------------------------------
# a1, a2: composite tensor and double layer (Sec. III, Fig. 4(a,b))
# --------------------------------------------------------------------------

# For the fused bond gamma, the two remaining bond types in cyclic order after
# gamma are (alpha, beta); A.alpha -> l, A.beta -> u, B.alpha -> r, B.beta -> d.
_CYCLIC_REST = {0: (1, 2), 1: (2, 0), 2: (0, 1)}


def composite(A, B, gamma=2):
    """Composite tensor of one A-B pair fused across its gamma bond.

    K[p, u, l, d, r] with p = (s_A, a_A, s_B, a_B) (16 values) and
    u = A.beta, l = A.alpha, d = B.beta, r = B.alpha.
    """
    al, be = _CYCLIC_REST[gamma]
    # move bond axes of A to (alpha, beta, gamma) order, same for B
    Ap = np.moveaxis(A, (2 + al, 2 + be, 2 + gamma), (2, 3, 4))
    Bp = np.moveaxis(B, (2 + al, 2 + be, 2 + gamma), (2, 3, 4))
    # A[s,a,l,u,g] B[t,c,r,d,g] -> K[s,a,t,c,u,l,d,r]
    K = np.einsum('salug,tcrdg->satculdr', Ap, Bp)
    D_l, D_u = Ap.shape[2], Ap.shape[3]
    D_r, D_d = Bp.shape[2], Bp.shape[3]
    return K.reshape(16, D_u, D_l, D_d, D_r)


def double_layer(K, O=None):
    """Double-layer site tensor a[u, l, d, r], each leg fused as (ket, bra).

    a[(u_k u_b), ...] = sum_p K[p, ket legs] K[p, bra legs]; fused index
    k * D + b.  With an operator O (16 x 16 on the composite's physical index,
    O[p_bra, p_ket]) the result is a_O = sum O[p, q] K[q, ket] K[p, bra], so
    that <E, a_O> / <E, a> is <psi|O|psi> / <psi|psi> for real tensors.
    """
    _, Du, Dl, Dd, Dr = K.shape
    if O is None:
        a8 = np.einsum('pulvr,pxyzw->uxlyvzrw', K, K)
    else:
        a8 = np.einsum('qp,pulvr,qxyzw->uxlyvzrw', O, K, K)
    return a8.reshape(Du * Du, Dl * Dl, Dd * Dd, Dr * Dr)


def full_operator(op, op_dim):
    """Lift a real operator to the 16-dim composite physical space.

    op_dim = 4: op acts on (s_A, s_B) (row-major 4x4), identity on ancillas.
    op_dim = 16: op is already on p = (s_A, a_A, s_B, a_B).
    """
    op = np.asarray(op, dtype=np.float64)
    if op_dim == 16:
        return op.reshape(16, 16)
    if op_dim != 4:
        raise ValueError("op_dim must be 4 or 16")
    o = op.reshape(2, 2, 2, 2)  # [sA, sB, sA', sB']
    I2 = np.eye(2)
    full = np.einsum('stuv,ab,cd->satcubvd', o, I2, I2)
    return full.reshape(16, 16)


def rotate(a, times=1):
    """Site tensor in the frame rotated ``times`` x 90 degrees counter-clockwise."""
    for _ in range(times % 4):
        a = np.transpose(a, (3, 0, 1, 2))
    return np.ascontiguousarray(a)


# --------------------------------------------------------------------------
# a3: environment initialisation
# --------------------------------------------------------------------------

class Env:
    """Corner and edge tensors plus the log of the scale divided out of each."""

    def __init__(self, C, T, logC, logT):
        self.C = [np.array(c) for c in C]
        self.T = [np.array(t) for t in T]
        self.logC = list(logC)
        self.logT = list(logT)
        self.spectra = None

    def copy(self):
        e = Env(self.C, self.T, self.logC, self.logT)
        e.spectra = None if self.spectra is None else [s.copy() for s in self.spectra]
        return e


def boundary_vector_double_layer(D):
    """Ket-bra identity on a fused leg (index k * D + b): vec(I_D)."""
    return np.eye(D).reshape(D * D)


def boundary_vector_classical(d):
    """First basis vector e_0."""
    b = np.zeros(d)
    b[0] = 1.0
    return b


def init_env(d, chi, b):
    """C_i = [[1]] and T_i[0, :, 0] = b, zero-padded to chi.

    After k sweeps from this start in which nothing is truncated (every cut
    singular value above the cutoff and kept) the environment is exactly the
    (2k+1) x (2k+1) open lattice whose outer legs all end in b.
    """
    C = []
    T = []
    for _ in range(4):
        c = np.zeros((chi, chi))
        c[0, 0] = 1.0
        t = np.zeros((chi, d, chi))
        t[0, :, 0] = b
        C.append(c)
        T.append(t)
    return Env(C, T, [0.0] * 4, [0.0] * 4)


# --------------------------------------------------------------------------
# a4 .. a7: one directional move (Fig. 4(c)); projectors from the four
# enlarged corners, the directional scheme of the cited CTMRG literature
# --------------------------------------------------------------------------

def enlarged_corner(C1, T1, T4, a):
    """Top-left enlarged corner as an n x n matrix, n = chi * d.

    Q[(delta, dd), (gamma, r)] = sum C1[al, be] T1[be, u, gamma]
                                     T4[delta, l, al] a[u, l, dd, r]
    Rows: the cut below the block; columns: the cut to its right.
    """
    chi = C1.shape[0]
    d = a.shape[0]
    X1 = _c('ab,bug->aug', C1, T1)            # C1 T1
    X2 = _c('dla,aug->dlug', T4, X1)          # T4 C1 T1
    Q = _c('dlug,ulxr->dxgr', X2, a)          # ... a
    return Q.reshape(chi * d, chi * d)


def frame(env, k):
    """(C1..C4, T1..T4) as seen in the frame rotated k times."""
    C = [env.C[(k + i) % 4] for i in range(4)]
    T = [env.T[(k + i) % 4] for i in range(4)]
    return C, T


def projectors(env, arot, k, chi, eps_cut):
    """Projector pair for the cut between the two left enlarged corners.

    Q_r is the enlarged corner of frame k + r.  U = Q_0 Q_1 (upper half,
    rows: the left cut i, columns: the right cut j); Lt = Q_2 Q_3 (lower half
    transposed, rows j', columns i); M = U^T L with L = Lt^T, i.e.
    M[j, j'] = sum_i U[i, j] L[i, j'].  With M = X S Y^T (top chi kept):
        Pu = L Y S^{-1/2}   (n x chi, attaches to the upper side of the cut)
        Pl = U X S^{-1/2}   (n x chi, attaches to the lower side)
    so that Pu Pl^T is the oblique projector L M^+ U^T.  Singular values
    below eps_cut * s_1 get S^{-1/2} := 0 (shapes are kept).
    """
    Q = []
    for r in range(4):
        f = (k + r) % 4
        Q.append(enlarged_corner(env.C[f], env.T[f], env.T[(f + 3) % 4], arot[f]))
    U = Q[0] @ Q[1]
    Lt = Q[2] @ Q[3]
    L = Lt.T
    M = U.T @ L
    X, s, Yh = np.linalg.svd(M)
    Y = Yh.T
    n = M.shape[0]
    kk = min(chi, n)
    s_k = s[:kk]
    inv_sqrt = np.zeros(chi)
    keep = s_k > eps_cut * s[0] if s[0] > 0 else np.zeros(kk, bool)
    inv_sqrt[:kk][keep] = 1.0 / np.sqrt(s_k[keep])
    Xc = np.zeros((n, chi))
    Yc = np.zeros((n, chi))
    Xc[:, :kk] = X[:, :kk]
    Yc[:, :kk] = Y[:, :kk]
    Pu = (L @ Yc) * inv_sqrt[None, :]
    Pl = (U @ Xc) * inv_sqrt[None, :]
    return Pu, Pl, s


def _normalise(t):
    m = np.abs(t).max()
    if not np.isfinite(m) or m == 0.0:
        raise FloatingPointError("environment tensor vanished or is not finite")
    return t / m, np.log(m)


def left_move(env, arot, k, chi, eps_cut=EPS_CUT_DEFAULT):
    """Absorb one column into the left side of frame k (updates C1, T4, C4).

    C1' = C1 T1 with cut (al, u); T4' = T4 a with cuts (delta, dd) below and
    (al, u) above; C4' = T3 C4 with cut (delta, dd) above.  Then
        C1_new[k1, g]     = sum_i Pu[i, k1] C1'[i, g]
        T4_new[k1, r, k2] = sum Pu[(delta,dd), k1] T4'[(delta,dd), r, (al,u)] Pl[(al,u), k2]
        C4_new[i3, k2]    = sum_i C4'[i3, i] Pl[i, k2]
    and each is divided by its max |entry| (the log of the factor is kept).
    """
    Pu, Pl, s = projectors(env, arot, k, chi, eps_cut)
    C, T = frame(env, k)
    a = arot[k % 4]
    d = a.shape[0]
    chi_old = C[0].shape[0]
    Pu4 = Pu.reshape(chi_old, d, chi)
    Pl4 = Pl.reshape(chi_old, d, chi)
    C1p = _c('ab,bug->aug', C[0], T[0])       # C1' = C1 T1
    C1n = _c('aug,auk->kg', C1p, Pu4)
    X = _c('dla,aum->dlum', T[3], Pl4)        # T4 Pl
    Y = _c('dlum,ulxr->dmxr', X, a)           # (T4 Pl) a
    T4n = _c('dmxr,dxk->krm', Y, Pu4)         # Pu^T (T4 a) Pl
    C4p = _c('ixc,cd->ixd', T[2], C[3])       # C4' = T3 C4
    C4n = _c('ixd,dxm->im', C4p, Pl4)
    i1, i4 = k % 4, (k + 3) % 4
    lC1 = env.logC[i1] + env.logT[k % 4]
    lT4 = env.logT[i4]
    lC4 = env.logC[i4] + env.logT[(k + 2) % 4]
    C1n, f1 = _normalise(C1n)
    T4n, f2 = _normalise(T4n)
    C4n, f3 = _normalise(C4n)
    env.C[i1], env.logC[i1] = C1n, lC1 + f1
    env.T[i4], env.logT[i4] = T4n, lT4 + f2
    env.C[i4], env.logC[i4] = C4n, lC4 + f3
    return s


# --------------------------------------------------------------------------
# a8: sweeps and convergence
# --------------------------------------------------------------------------

MOVE_ORDER = (0, 2, 1, 3)  # left, right, up, down (frames rotated 0, 2, 1, 3 times)


def corner_spectra(env):
    """Normalised singular values s / ||s||_2 of the four corners."""
    out = []
    for c in env.C:
        s = np.linalg.svd(c, compute_uv=False)
        nrm = np.linalg.norm(s)
        out.append(s / nrm if nrm > 0 else s)
    return out


def sweep(env, arot, chi, eps_cut=EPS_CUT_DEFAULT):
    """One sweep = the left move in frames 0, 2, 1, 3 (L, R, U, D).

    Returns delta = max over corners of ||s_hat - s_hat_old||_2.
    """
    old = env.spectra if env.spectra is not None else corner_spectra(env)
    for k in MOVE_ORDER:
        left_move(env, arot, k, chi, eps_cut)
    new = corner_spectra(env)
    env.spectra = new
    return max(np.linalg.norm(n - o) for n, o in zip(new, old))


def ctmrg(a, chi, b, max_sweeps, tol=0.0, eps_cut=EPS_CUT_DEFAULT, env=None):
    """Run sweeps until delta < tol (tol <= 0: exactly max_sweeps sweeps)."""
    d = a.shape[0]
    arot = [rotate(a, k) for k in range(4)]
    if env is None:
        env = init_env(d, chi, b)
    deltas = []
    for _ in range(max_sweeps):
        delta = sweep(env, arot, chi, eps_cut)
        deltas.append(delta)
        if tol > 0 and delta < tol:
            break
    return env, deltas


# --------------------------------------------------------------------------
# a9: bond environment, norm per site, expectation values
# --------------------------------------------------------------------------

def ring(env):
    """E[u, l, d, r]: the eight environment tensors with the site removed,
    sum C1[a,b] T1[b,u,g] C2[g,e] T2[e,r,h] C3[h,q] T3[q,x,c] C4[c,d] T4[d,l,a]."""
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    up = _c('ab,bug->aug', C1, T1)
    up = _c('aug,ge->aue', up, C2)            # C1 T1 C2
    up = _c('aue,dla->dlue', up, T4)
    up = _c('dlue,erh->dlurh', up, T2)        # upper half with T4, T2
    lo = _c('hq,qxc->hxc', C3, T3)
    lo = _c('hxc,cd->hxd', lo, C4)            # C3 T3 C4
    return _c('dlurh,hxd->ulxr', up, lo)


def kappa(env, a):
    """Norm per site: Z_site Z_corners / (Z_row Z_col) (scale-invariant)."""
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    z_site = np.einsum('ulxr,ulxr->', ring(env), a)
    z_0 = np.einsum('ab,bc,cd,da->', C1, C2, C3, C4)
    z_row = np.einsum('ab,bmg,ge,eq,qmc,ca->', C1, T1, C2, C3, T3, C4, optimize=True)
    z_col = np.einsum('ab,be,erh,hq,qd,dra->', C1, C2, T2, C3, C4, T4, optimize=True)
    return z_site * z_0 / (z_row * z_col)


def log_z(env, a):
    """log |<E, a>| + all logged scales: the log of the finite-lattice value
    represented by the (untruncated) environment and the centre site."""
    z = np.einsum('ulxr,ulxr->', ring(env), a)
    return np.log(abs(z)) + sum(env.logC) + sum(env.logT), np.sign(z)


def bond_metric(env, a, D):
    """The full-update bond metric: E normalised to <E, a> = 1, reshaped to
    [u_k, l_k, d_k, r_k, u_b, l_b, d_b, r_b] (each fused leg is k * D + b)."""
    E = ring(env)
    E = E / np.einsum('ulxr,ulxr->', E, a)
    E8 = E.reshape(D, D, D, D, D, D, D, D)  # u_k u_b l_k l_b d_k d_b r_k r_b
    return np.ascontiguousarray(E8.transpose(0, 2, 4, 6, 1, 3, 5, 7))


def expect(env, a, a_O):
    """<O> = <E, a_O> / <E, a>."""
    E = ring(env)
    return np.einsum('ulxr,ulxr->', E, a_O) / np.einsum('ulxr,ulxr->', E, a)


def environment_from_purification(A, B, gamma, chi, max_sweeps, tol=0.0,
                                  eps_cut=EPS_CUT_DEFAULT):
    """a1 + a2 + a3 + sweeps for a purification pair; returns (env, a, K, D)."""
    K = composite(A, B, gamma)
    a = double_layer(K)
    D = K.shape[1]
    if not (K.shape[1] == K.shape[2] == K.shape[3] == K.shape[4]):
        raise ValueError("non-fused bonds must share one dimension D")
    b = boundary_vector_double_layer(D)
    env, deltas = ctmrg(a, chi, b, max_sweeps, tol, eps_cut)
    return env, a, K, D, deltas
