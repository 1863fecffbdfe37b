"""Closed forms of the coupled-mode theory, used to pin the oracle.

TEST INFRASTRUCTURE ONLY.  Part of the CPU oracle: only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.
"""
import numpy as np


def h0(g, gamma=1.76e11):
    """Feedback conversion factor h0 = 2 g / gamma [T], Sec. II A Eq. (5)."""
    return 2.0 * g / gamma


def polariton(wc, wm, g):
    """Hermitian polariton branches, Sec. II B Eq. (6)."""
    mid = 0.5 * (wc + wm)
    half = np.sqrt(g * g + (0.5 * (wc - wm)) ** 2)
    return mid - half, mid + half


def polariton_complex(wc, kappa, wm, gamma_m, gt):
    """Complex branches of (w - wc + i kappa)(w - wm + i gamma_m) = gt^2
    (Sec. II B Eq. (7); Sec. IV H Eq. (20) with gt = g - i g_d)."""
    wct = wc - 1j * kappa
    wmt = wm - 1j * gamma_m
    mid = 0.5 * (wct + wmt)
    root = np.sqrt(gt * gt + (0.5 * (wct - wmt)) ** 2 + 0j)
    return mid - root, mid + root


def cooperativity(g, kappa, alpha, wm):
    """C = g^2 / (kappa gamma_m), gamma_m = alpha w_m, Sec. II C Eq. (8)."""
    return g * g / (kappa * alpha * wm)


def kittel(B0, gamma=1.76e11):
    """Uniform-precession frequency of a sphere, Sec. II D Eq. (9)."""
    return gamma * B0


def rabi_period(g):
    """Vacuum Rabi period pi/g at resonance, Sec. IV B."""
    return np.pi / g


def three_mode(w1, wm, w2, g1, g2):
    """Eigenvalues and eigenvectors of the 3x3 matrix of Sec. II F Eq. (14),
    basis (|1>, |m>, |2>)."""
    H = np.array([[w1, g1, 0.0], [g1, wm, g2], [0.0, g2, w2]])
    return np.linalg.eigh(H)


def afmr(BE, BA, gamma=1.76e11):
    """Zero-field AFM resonance gamma sqrt(2 B_E B_A + B_A^2), Sec. II G
    Eq. (15), fields in tesla (B = mu0 H)."""
    return gamma * np.sqrt(2.0 * BE * BA + BA * BA)


def afm_split(BE, BA, B, gamma=1.76e11):
    """Field-split AFM branches w_AFMR -+ gamma B, Sec. II G Eq. (16)."""
    w0 = afmr(BE, BA, gamma)
    return w0 - gamma * B, w0 + gamma * B


def overlap(u, G=None):
    """<u> over the magnetic cells, Sec. II E Eq. (10)."""
    if G is None:
        return float(np.mean(u))
    return float(np.sum(u * G) / np.sum(G))


def rk4_stability(z):
    """One-step amplification of classical RK4 on y' = z y / dt."""
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


def dp5_stability(z):
    """5th-order Dormand-Prince stability polynomial."""
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24 + z ** 5 / 120 + z ** 6 / 600


def dp4_stability(z):
    """Embedded 4th-order Dormand-Prince stability polynomial."""
    return (1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24 + 1097 / 120000 * z ** 5
            + 161 / 120000 * z ** 6 + z ** 7 / 24000)


def dp_error_polynomial(z):
    """dp5_stability - dp4_stability written out, free of cancellation."""
    return -97 / 120000 * z ** 5 + 39 / 120000 * z ** 6 - z ** 7 / 24000


def _prism_dz(a, b, c):
    """Magnetometric demagnetizing factor along z of a rectangular prism
    of half-sides a, b, c (along x, y, z): A. Aharoni, J. Appl. Phys. 83,
    3432 (1998), Eq. (1)."""
    r = np.sqrt(a * a + b * b + c * c)
    ab, bc, ac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    t = ((b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
         + b / (2 * c) * np.log((ab + a) / (ab - a))
         + a / (2 * c) * np.log((ab + b) / (ab - b))
         + c / (2 * a) * np.log((bc - b) / (bc + b))
         + c / (2 * b) * np.log((ac - a) / (ac + a))
         + 2 * np.arctan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return t / np.pi


def prism_demag_factors(lx, ly, lz):
    """(N_xx, N_yy, N_zz) of a uniformly magnetised rectangular block of
    edges lx, ly, lz: the volume average of its demagnetizing tensor, which
    is also the average of the cell-pair (Newell) tensor over all cell pairs
    of the block when it is cut into cells.  Aharoni's Eq. (1) with the
    axes permuted."""
    a, b, c = 0.5 * lx, 0.5 * ly, 0.5 * lz
    return _prism_dz(b, c, a), _prism_dz(c, a, b), _prism_dz(a, b, c)


def exchange_mode_field(k, n, A, Ms, d):
    """Exchange field per unit amplitude [T] of the Neumann standing wave
    cos(k pi (i + 1/2) / n) along an axis of n cells of size d: the
    eigenvalue (2A/Ms)(2/d^2)(1 - cos(k pi / n)) of the six-neighbour
    stencil with free ends, so that the wave precesses at
    gamma (B0 + this field) in a bias B0 along z without demag."""
    return 2.0 * A / Ms * 2.0 / (d * d) * (1.0 - np.cos(k * np.pi / n))


def profile_coupling(g, u, phi):
    """Coupling of a cavity mode of profile u to the spin-wave mode of
    profile phi (Sec. II E, Eq. (10)-(11) and Eq. (18)): the cavity sees
    g <u m^-> and the wave is driven by g u(r) a projected on phi, so the
    pair exchanges at g_eff = g <u phi> / sqrt(<phi^2>) (means over the
    magnetic cells); <u> for a uniform phi."""
    u = np.asarray(u, float)
    phi = np.asarray(phi, float)
    return g * np.mean(u * phi) / np.sqrt(np.mean(phi * phi))
