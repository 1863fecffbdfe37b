"""Right-hand side of the coupled LLG + N-cavity-mode system, plain FP64.

TEST INFRASTRUCTURE ONLY.  Part of the CPU oracle: only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.

State: m with shape (S, 3, nz, ny, nx) (S = 1 ferromagnet, 2 antiferromagnet
sublattices), zero on non-magnetic cells; a, complex, shape (N,).

Equations (SI units, fields in tesla, rates in rad/s):
  * cavity modes, Sec. II A Eq. (1) and Sec. II F Eq. (12), with the
    dissipative phase of Sec. IV H Eq. (19) written as g e^{-i Phi}:
        da_n/dt = (-i w_n - k_n) a_n + i g_n e^{-i Phi_n} m^-_n + eta_n(t)
    with the external microwave drive eta_n(t) of Eq. (1) / Eq. (12) taken as
    the Gaussian pulse of Sec. IV A, eta_n(t) = A_n exp(-(t - t0_n)^2 / (2 sigma_n^2))
    with a complex amplitude A_n [1/s] (zero when no drive is set)
  * cavity-model variants of Sec. II A and Sec. V (optional, per mode):
    nonreciprocal coupling, g_n (= g_f) in the cavity equation and
    h0_n = 2 g_b,n / gamma in the feedback; a self-Kerr term
    -i K_n |a_n|^2 a_n added to da_n/dt
  * direct photon-photon coupling (the H_13 entry of the Sec. II F
    coupling matrix, Eq. (14)): da_n/dt gains -i sum_m J_nm a_m with J real
    symmetric and zero on the diagonal
  * a degenerate parametric pump (Sec. V names parametric drives without an
    equation): da_n/dt gains -i lam_n e^{-2 i wp_n t} conj(a_n), a pump at
    twice wp_n with complex strength lam_n [rad/s]; in the frame rotating
    at wp_n at resonance one quadrature decays at kappa + |lam| and the
    other at kappa - |lam| (gain above the threshold |lam| = kappa)
  * co-rotating average, Eq. (2) weighted by the mode profile as in Eq. (18):
        m^-_n = 1/N_geo sum_i G_i u_n(r_i) (1/S) sum_s c_s (m_sx - i m_sy)
  * RF feedback along x, Eq. (3) and Eq. (13), h0_n = 2 g_n / gamma (Eq. (5)):
        B_rf = x * c_s sum_n h0_n u_n(r) Re[e^{-i Phi_n} a_n]
  * effective field: Zeeman B0 + exchange (6-neighbour, Neumann) + uniaxial
    anisotropy + demag (none | local diagonal | cell-averaged tensor) + B_rf,
    and for two sublattices the intersublattice term -B_E m_{s'}
  * Landau-Lifshitz torque, gamma' = gamma / (1 + alpha^2):
        dm/dt = -gamma' [m x B + alpha m x (m x B)]
"""
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import newell

MU0 = newell.MU0
DEMAG_NONE, DEMAG_LOCAL, DEMAG_FFT = 0, 1, 2


@dataclass
class Problem:
    grid: Sequence[int]                      # (nx, ny, nz)
    cell: Sequence[float]                    # (dx, dy, dz) [m]
    Ms: float                                # [A/m], per sublattice
    Aex: float                               # [J/m]
    alpha: float
    gamma: float = 1.76e11                   # [rad/(s T)]
    Ku: float = 0.0                          # [J/m^3]
    ku_axis: Sequence[float] = (0.0, 0.0, 1.0)
    B0: Sequence[float] = (0.0, 0.0, 0.0)    # [T]
    demag: int = DEMAG_NONE
    n_local: Sequence[float] = (0.0, 0.0, 0.0)
    geometry: Optional[np.ndarray] = None    # bool (nz, ny, nx); None = all magnetic
    sublattices: int = 1
    B_E: float = 0.0                         # [T]
    # cavity modes
    omega: Sequence[float] = ()
    kappa: Sequence[float] = ()
    g: Sequence[float] = ()
    u: Optional[np.ndarray] = None           # (N, nz, ny, nx); None = uniform
    phi: Optional[Sequence[float]] = None    # (N,); None = 0
    csign: Optional[Sequence[float]] = None  # (S,); None = +1
    g_back: Optional[Sequence[float]] = None   # (N,) backward coupling g_b [rad/s]; None = g
    kerr: Optional[Sequence[float]] = None     # (N,) self-Kerr K [rad/s]; None = 0
    photon_coupling: Optional[np.ndarray] = None  # (N, N) J [rad/s], symmetric, zero diagonal; None = 0
    # Gaussian cavity drive eta_n(t); None = undriven
    drive_amp: Optional[Sequence[complex]] = None   # (N,) complex amplitude [1/s]
    drive_t0: Optional[Sequence[float]] = None      # (N,) pulse centre [s]
    drive_sigma: Optional[Sequence[float]] = None   # (N,) pulse width [s], > 0
    # degenerate parametric pump -i lam_n e^{-2 i wp_n t} conj(a_n); None = off
    param_lambda: Optional[Sequence[complex]] = None  # (N,) complex strength [rad/s]
    param_wp: Optional[Sequence[float]] = None        # (N,) half the pump frequency [rad/s]

    @property
    def n_modes(self):
        return len(self.omega)


class Model:
    """Precomputed constants and the right-hand side for one Problem.

    `leaves` may hold torch tensors for 'alpha', 'B0', 'g' and 'u' (e.g.
    with requires_grad) that replace the Problem's numbers, so that the
    whole run can be differentiated by autograd."""

    def __init__(self, p: Problem, leaves=None):
        leaves = leaves or {}
        self.p = p
        nx, ny, nz = (int(v) for v in p.grid)
        self.shape = (nz, ny, nx)
        if p.geometry is None:
            G = np.ones(self.shape, bool)
        else:
            G = np.asarray(p.geometry, bool).reshape(self.shape)
        self.Gmask = torch.tensor(G)
        self.G = torch.tensor(G, dtype=torch.float64)
        self.n_geo = float(G.sum())
        self.S = int(p.sublattices)
        N = p.n_modes
        self.N = N
        self.alpha = leaves.get("alpha", p.alpha)
        self.gamma_ll = p.gamma / (1.0 + self.alpha * self.alpha)
        self.cex = 2.0 * p.Aex / p.Ms
        self.inv_d2 = [1.0 / (c * c) for c in p.cell]              # x, y, z
        e = np.asarray(p.ku_axis, float)
        self.ku_axis = torch.tensor(e / np.linalg.norm(e)) if np.linalg.norm(e) > 0 else torch.zeros(3, dtype=torch.float64)
        self.cK = 2.0 * p.Ku / p.Ms
        self.B0 = leaves["B0"] if "B0" in leaves else torch.tensor(np.asarray(p.B0, float))
        self.omega = torch.tensor(np.asarray(p.omega, float))
        self.kappa = torch.tensor(np.asarray(p.kappa, float))
        self.g = leaves["g"] if "g" in leaves else torch.tensor(np.asarray(p.g, float))
        self.phi = torch.tensor(np.zeros(N) if p.phi is None else np.asarray(p.phi, float))
        if p.g_back is None:
            self.h0 = 2.0 * self.g / p.gamma                         # Eq. (5)
        else:
            self.h0 = 2.0 * torch.tensor(np.asarray(p.g_back, float)) / p.gamma
        self.kerr = None if p.kerr is None else torch.tensor(np.asarray(p.kerr, float))
        self.J = None if p.photon_coupling is None else torch.tensor(np.asarray(p.photon_coupling, float))
        if "u" in leaves:
            self.u = leaves["u"]
        elif p.u is None:
            self.u = torch.ones((N,) + self.shape, dtype=torch.float64)
        else:
            self.u = torch.tensor(np.asarray(p.u, float).reshape((N,) + self.shape))
        self.param_on = p.param_lambda is not None
        if self.param_on:
            self.param_lambda = torch.tensor(np.asarray(p.param_lambda, complex))
            self.param_wp = torch.tensor(np.asarray(p.param_wp, float))
        self.drive_on = p.drive_amp is not None
        if self.drive_on:
            self.drive_amp = torch.tensor(np.asarray(p.drive_amp, complex))
            self.drive_t0 = torch.tensor(np.asarray(p.drive_t0, float))
            self.drive_sigma = torch.tensor(np.asarray(p.drive_sigma, float))
        cs = np.ones(self.S) if p.csign is None else np.asarray(p.csign, float)
        self.csign = torch.tensor(cs)
        self.spectrum = None
        if p.demag == DEMAG_FFT:
            spec = newell.kernel_spectrum(p.grid, p.cell)
            self.spectrum = torch.tensor(spec)
            self.pad = tuple(newell.padded_size(n) for n in (nz, ny, nx))

    # ---------------------------------------------------------------- fields
    def exchange(self, ms):
        """(2A/Ms) sum_d sum_+- G_nbr (m_nbr - m) / d^2 on one sublattice,
        ms: (3, nz, ny, nx).  Only pairs of magnetic cells contribute."""
        B = torch.zeros_like(ms)
        G = self.G
        # spatial axes of ms: 1 = z, 2 = y, 3 = x
        for axis, w in ((3, self.inv_d2[0]), (2, self.inv_d2[1]), (1, self.inv_d2[2])):
            n = ms.shape[axis]
            if n < 2:
                continue
            lo = ms.narrow(axis, 0, n - 1)
            hi = ms.narrow(axis, 1, n - 1)
            pair = G.narrow(axis - 1, 0, n - 1) * G.narrow(axis - 1, 1, n - 1)
            d = (hi - lo) * pair * w
            B = B + torch.nn.functional.pad(d, _pad_spec(axis, after=1)) \
                  - torch.nn.functional.pad(d, _pad_spec(axis, before=1))
        return self.cex * B

    def anisotropy(self, ms):
        e = self.ku_axis.view(3, 1, 1, 1)
        return self.cK * (ms * e).sum(0, keepdim=True) * e

    def demag(self, m):
        """Demag field [T] for all sublattices, m: (S, 3, nz, ny, nx)."""
        p = self.p
        if p.demag == DEMAG_NONE:
            return torch.zeros_like(m[0])
        if p.demag == DEMAG_LOCAL:
            n = torch.tensor(np.asarray(p.n_local, float)).view(3, 1, 1, 1)
            return -MU0 * p.Ms * n * m.sum(0)
        M = p.Ms * m.sum(0) * self.G
        Mh = torch.fft.rfftn(M, s=self.pad, dim=(1, 2, 3))
        xx, yy, zz, xy, xz, yz = self.spectrum
        Hx = xx * Mh[0] + xy * Mh[1] + xz * Mh[2]
        Hy = xy * Mh[0] + yy * Mh[1] + yz * Mh[2]
        Hz = xz * Mh[0] + yz * Mh[1] + zz * Mh[2]
        H = torch.fft.irfftn(torch.stack([Hx, Hy, Hz]), s=self.pad, dim=(1, 2, 3))
        nz, ny, nx = self.shape
        return -MU0 * H[:, :nz, :ny, :nx]

    def feedback_x(self, a):
        """Sum_n h0_n u_n(r) Re[e^{-i Phi_n} a_n] (before the sublattice sign)."""
        coef = self.h0 * torch.real(torch.exp(-1j * self.phi) * a)
        return (coef.view(-1, 1, 1, 1) * self.u).sum(0)

    def field(self, m, a):
        """Effective field [T], shape (S, 3, nz, ny, nx)."""
        Bd = self.demag(m)
        brf = self.feedback_x(a)
        out = []
        for s in range(self.S):
            B = self.exchange(m[s]) + self.anisotropy(m[s]) + Bd
            B = B + self.B0.view(3, 1, 1, 1)
            rf = torch.zeros_like(B)
            rf[0] = self.csign[s] * brf
            B = B + rf
            if self.S == 2:
                B = B - self.p.B_E * m[1 - s]
            out.append(B)
        return torch.stack(out)

    # ---------------------------------------------------------------- torque
    def torque(self, m, B):
        mxB = torch.cross(m, B, dim=1)
        mxmxB = torch.cross(m, mxB, dim=1)
        return -self.gamma_ll * (mxB + self.alpha * mxmxB) * self.G

    # ---------------------------------------------------------------- cavity
    def m_minus(self, m):
        """m^-_n, complex (N,)."""
        mm = (self.csign.view(-1, 1, 1, 1) * (m[:, 0] - 1j * m[:, 1])).sum(0) / self.S
        return (self.u * (self.G * mm)).sum(dim=(1, 2, 3)) / self.n_geo

    def drive(self, t):
        """eta_n(t), complex (N,): the Gaussian pulse of Sec. IV A."""
        x = (t - self.drive_t0) / self.drive_sigma
        return self.drive_amp * torch.exp(-0.5 * x * x)

    def cavity_rhs(self, a, mminus, t=0.0):
        """Eq. (12) with the dissipative phase of Eq. (19); the Kerr term, the
        mode coupling, the parametric pump and the drive enter only when set,
        the pump and the drive at the time t of the stage."""
        f = (-1j * self.omega - self.kappa) * a + 1j * self.g * torch.exp(-1j * self.phi) * mminus
        if self.kerr is not None:
            f = f - 1j * self.kerr * (a.real * a.real + a.imag * a.imag) * a
        if self.J is not None:
            f = f - 1j * (self.J.to(a.dtype) @ a)
        if self.param_on:
            f = f - 1j * self.param_lambda * torch.exp(-2j * self.param_wp * t) * torch.conj(a)
        if self.drive_on:
            f = f + self.drive(t)
        return f

    def rhs(self, m, a, t=0.0):
        """(dm/dt, da/dt, m^-) at state (m, a) and time t."""
        B = self.field(m, a)
        km = self.torque(m, B)
        mm = self.m_minus(m)
        return km, self.cavity_rhs(a, mm, t), mm

    def normalize(self, m):
        """m / |m| on magnetic cells, unchanged (zero) elsewhere.  The norm is
        taken of a value that is never zero, so reverse-mode derivatives stay
        finite on non-magnetic cells."""
        norm2 = (m * m).sum(1, keepdim=True)
        mask = self.Gmask.view(1, 1, *self.shape)
        safe = torch.where(mask, norm2, torch.ones_like(norm2))
        return torch.where(mask, m / torch.sqrt(safe), m)


def _pad_spec(axis, before=0, after=0):
    """torch pad spec for a (3, nz, ny, nx) tensor along one spatial axis."""
    spec = [0, 0, 0, 0, 0, 0]
    k = 3 - axis                           # axis 3 (x) -> first pair
    spec[2 * k] = before
    spec[2 * k + 1] = after
    return spec
