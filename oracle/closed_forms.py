"""Closed forms that pin the oracle; independent of the CTMRG code.

TEST INFRASTRUCTURE ONLY.

* Onsager's free energy of the square-lattice Ising model (J = 1), in the
  double-integral form and, as a cross-check, the single-integral form.
* Houtappel's free energy of the anisotropic honeycomb Ising model.
* Two-site algebra for the infinite-temperature purification (Sec. III: the
  purification at beta = 0 is a product of pseudospin-ancilla singlets) and
  for one layer of gates applied to it.

The double integrals have analytic periodic integrands, so the trapezoidal
rule on a uniform grid converges geometrically; n = 400 points per axis
gives ~1e-15 away from the critical couplings used nowhere here.
"""
import numpy as np
from scipy import integrate


def _torus_mean(f, n=400):
    th = 2.0 * np.pi * np.arange(n) / n
    t1, t2 = np.meshgrid(th, th, indexing='ij')
    return f(t1, t2).mean()


def onsager_minus_beta_f(beta, n=400):
    """-beta f = ln 2 + (1/(8 pi^2)) int int ln[cosh^2 2b - sinh 2b (cos t1 + cos t2)]."""
    c2, s2 = np.cosh(2 * beta) ** 2, np.sinh(2 * beta)
    m = _torus_mean(lambda t1, t2: np.log(c2 - s2 * (np.cos(t1) + np.cos(t2))), n)
    return np.log(2.0) + 0.5 * m


def onsager_minus_beta_f_single(beta):
    """Single-integral form: ln(2 cosh 2b) + (1/pi) int_0^{pi/2}
    ln[(1 + sqrt(1 - k^2 sin^2 t)) / 2] dt with k = 2 sinh 2b / cosh^2 2b."""
    k = 2.0 * np.sinh(2 * beta) / np.cosh(2 * beta) ** 2
    val, _ = integrate.quad(lambda t: np.log(0.5 * (1.0 + np.sqrt(1.0 - (k * np.sin(t)) ** 2))),
                            0.0, 0.5 * np.pi, epsabs=1e-15, epsrel=1e-15, limit=200)
    return np.log(2.0 * np.cosh(2 * beta)) + val / np.pi


def onsager_nn_correlation(beta, n=400):
    """<s_i s_j> for nearest neighbours = (1/2) d(-beta f)/d beta (two bonds
    per site), with the derivative taken under the integral."""
    c, s = np.cosh(2 * beta), np.sinh(2 * beta)

    def g(t1, t2):
        den = c * c - s * (np.cos(t1) + np.cos(t2))
        num = 4.0 * c * s - 2.0 * c * (np.cos(t1) + np.cos(t2))
        return num / den
    return 0.5 * (0.5 * _torus_mean(g, n))


def honeycomb_minus_beta_f(Kx, Ky, Kz, n=400):
    """Houtappel: -beta f per site = (3/4) ln 2 + (1/(16 pi^2)) int int
    ln[cx cy cz + 1 - sx sy cos t1 - sy sz cos t2 - sz sx cos(t1 + t2)],
    with c_g = cosh 2K_g, s_g = sinh 2K_g."""
    cx, cy, cz = np.cosh(2 * Kx), np.cosh(2 * Ky), np.cosh(2 * Kz)
    sx, sy, sz = np.sinh(2 * Kx), np.sinh(2 * Ky), np.sinh(2 * Kz)
    m = _torus_mean(lambda t1, t2: np.log(cx * cy * cz + 1.0 - sx * sy * np.cos(t1)
                                          - sy * sz * np.cos(t2) - sz * sx * np.cos(t1 + t2)), n)
    return 0.75 * np.log(2.0) + 0.25 * m


def honeycomb_bond_correlation(Kx, Ky, Kz, which=2, n=400):
    """<s_A s_B> on a bond of type ``which``: d(2 (-beta f))/dK_which (one bond
    of each type per pair of sites), derivative under the integral."""
    K = [Kx, Ky, Kz]
    c = [np.cosh(2 * k) for k in K]
    s = [np.sinh(2 * k) for k in K]

    def arg(t1, t2, c, s):
        return (c[0] * c[1] * c[2] + 1.0 - s[0] * s[1] * np.cos(t1)
                - s[1] * s[2] * np.cos(t2) - s[2] * s[0] * np.cos(t1 + t2))

    def darg(t1, t2):
        # d/dK_w of arg: dc_w = 2 s_w, ds_w = 2 c_w
        dc = [0.0, 0.0, 0.0]
        ds = [0.0, 0.0, 0.0]
        dc[which] = 2.0 * s[which]
        ds[which] = 2.0 * c[which]
        prod = (dc[0] * c[1] * c[2] + c[0] * dc[1] * c[2] + c[0] * c[1] * dc[2])
        cross = ((ds[0] * s[1] + s[0] * ds[1]) * np.cos(t1)
                 + (ds[1] * s[2] + s[1] * ds[2]) * np.cos(t2)
                 + (ds[2] * s[0] + s[2] * ds[0]) * np.cos(t1 + t2))
        return (prod - cross) / arg(t1, t2, c, s)
    return 2.0 * 0.25 * _torus_mean(darg, n)


def honeycomb_high_temperature(Kx, Ky, Kz):
    """High-temperature (loop) expansion per site through order t^10:
    ln 2 + (1/2) sum_g ln cosh K_g + (1/2) h + (1/2) h^2 sum_g 1/t_g^2, with
    t_g = tanh K_g and h = (tx ty tz)^2 the weight of one hexagon (six bonds,
    one hexagon per two sites); the last term counts the ten-bond loops around
    two hexagons sharing a g bond (one per g bond, half a g bond per site).
    The error is O(h^2) (order t^12)."""
    t = np.tanh([Kx, Ky, Kz])
    h = (t[0] * t[1] * t[2]) ** 2
    return (np.log(2.0) + 0.5 * np.sum(np.log(np.cosh([Kx, Ky, Kz])))
            + 0.5 * h + 0.5 * h * h * np.sum(1.0 / t ** 2))


def dimer_norm_and_expectation(H, tau, O):
    """One gate layer exp(-tau H/2) applied to the beta = 0 singlet pair.

    The pair state is (G x 1_anc)|singlet_A>|singlet_B>; its norm is
    Tr(G^T G)/4 = Tr(e^{-tau H})/4 for symmetric H, and <O> (O on the two
    pseudospins) is Tr(O e^{-tau H}) / Tr(e^{-tau H}).  Eigen-decomposition
    gives both without any tensor network.
    """
    w, V = np.linalg.eigh(H)
    rho = (V * np.exp(-tau * w)[None, :]) @ V.T
    return np.trace(rho) / 4.0, np.trace(O @ rho) / np.trace(rho)
