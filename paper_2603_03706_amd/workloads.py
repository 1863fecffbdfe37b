"""Seeded synthetic inputs for the five workloads (no arithmetic of the method).

Every array here is an input handed to the stepper: grid and cell sizes,
material constants, geometry masks, standing-wave mode profiles (the
cos(n pi x / L) profiles of Sec. II E, Eq. (11)), initial states and bias
fields.  Both the oracle-side tests and the HIP-side tests and benchmark draw
their inputs from here, so the two sides see bit-identical inputs.

Frequencies in the workload descriptions are f = w / 2 pi; everything
returned here is in SI units with angular rates in rad/s.
"""
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

GAMMA = 1.76e11
MU0 = 4e-7 * math.pi
TWO_PI = 2.0 * math.pi

# YIG-like material of the film and sphere workloads
YIG = dict(Ms=140e3, Aex=3.65e-12, alpha=1e-4)

DEMAG_NONE, DEMAG_LOCAL, DEMAG_FFT = 0, 1, 2


@dataclass
class Instance:
    """One stepper instance: parameters, modes and initial state."""
    grid: tuple
    cell: tuple
    Ms: float
    Aex: float
    alpha: float
    gamma: float = GAMMA
    Ku: float = 0.0
    ku_axis: tuple = (0.0, 0.0, 1.0)
    B0: tuple = (0.0, 0.0, 0.0)
    demag: int = DEMAG_NONE
    n_local: tuple = (0.0, 0.0, 0.0)
    geometry: Optional[np.ndarray] = None      # uint8 (nz, ny, nx)
    sublattices: int = 1
    B_E: float = 0.0
    omega: np.ndarray = field(default_factory=lambda: np.zeros(0))
    kappa: np.ndarray = field(default_factory=lambda: np.zeros(0))
    g: np.ndarray = field(default_factory=lambda: np.zeros(0))
    u: Optional[np.ndarray] = None             # float32 (N, nz, ny, nx)
    phi: Optional[np.ndarray] = None
    csign: Optional[np.ndarray] = None         # int8 (S,)
    g_back: Optional[np.ndarray] = None        # (N,) backward coupling g_b [rad/s] (None: g)
    kerr: Optional[np.ndarray] = None          # (N,) self-Kerr coefficient [rad/s] (None: 0)
    photon_coupling: Optional[np.ndarray] = None  # (N, N) direct mode coupling J [rad/s] (None: 0)
    drive_amp: Optional[np.ndarray] = None     # complex128 (N,) Gaussian drive amplitude [1/s]
    drive_t0: Optional[np.ndarray] = None      # (N,) pulse centre [s]
    drive_sigma: Optional[np.ndarray] = None   # (N,) pulse width [s]
    param_lambda: Optional[np.ndarray] = None  # complex128 (N,) parametric pump strength [rad/s]
    param_wp: Optional[np.ndarray] = None      # (N,) half the pump frequency [rad/s]
    m0: Optional[np.ndarray] = None            # float32 (S, 3, nz, ny, nx)
    a0: Optional[np.ndarray] = None            # complex128 (N,)
    method: str = "rk4"
    dt0: float = 1e-12
    tol: float = 0.0
    T: float = 0.0
    dt_sample: float = 0.0

    @property
    def cells(self):
        nx, ny, nz = self.grid
        return nx * ny * nz

    def oracle_kwargs(self):
        """Keyword arguments for oracle.model.Problem."""
        return dict(grid=self.grid, cell=self.cell, Ms=self.Ms, Aex=self.Aex, alpha=self.alpha,
                    gamma=self.gamma, Ku=self.Ku, ku_axis=self.ku_axis, B0=self.B0,
                    demag=self.demag, n_local=self.n_local,
                    geometry=None if self.geometry is None else self.geometry.astype(bool),
                    sublattices=self.sublattices, B_E=self.B_E,
                    omega=list(self.omega), kappa=list(self.kappa), g=list(self.g),
                    u=None if self.u is None else self.u.astype(np.float64),
                    phi=None if self.phi is None else list(self.phi),
                    csign=None if self.csign is None else list(self.csign.astype(float)),
                    g_back=None if self.g_back is None else list(self.g_back),
                    kerr=None if self.kerr is None else list(self.kerr),
                    photon_coupling=None if self.photon_coupling is None else np.asarray(self.photon_coupling, float),
                    drive_amp=None if self.drive_amp is None else list(self.drive_amp),
                    drive_t0=None if self.drive_t0 is None else list(self.drive_t0),
                    drive_sigma=None if self.drive_sigma is None else list(self.drive_sigma),
                    param_lambda=None if self.param_lambda is None else list(self.param_lambda),
                    param_wp=None if self.param_wp is None else list(self.param_wp))


def tilted(grid, theta_deg, azimuth, sublattices=1):
    """Uniform state tilted theta from +z at the given azimuth; for two
    sublattices the second is the negative of the first."""
    nx, ny, nz = grid
    th = math.radians(theta_deg)
    v = np.array([math.sin(th) * math.cos(azimuth), math.sin(th) * math.sin(azimuth), math.cos(th)])
    m = np.empty((sublattices, 3, nz, ny, nx), np.float32)
    for s in range(sublattices):
        sign = 1.0 if s == 0 else -1.0
        for c in range(3):
            m[s, c] = sign * v[c]
    return m


def sphere_mask(n, radius_cells):
    """Cells whose centre lies within radius_cells of the grid centre."""
    idx = np.arange(n) + 0.5 - n / 2.0
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    return (xx * xx + yy * yy + zz * zz <= radius_cells * radius_cells).astype(np.uint8)


def standing_wave(grid, nx_mode, ny_mode=0, nz_mode=0, normalise=True):
    """cos(n_x pi x/L_x) cos(n_y pi y/L_y) cos(n_z pi z/L_z) at cell centres,
    x measured from the sample edge; scaled to max |u| = 1."""
    nx, ny, nz = grid
    fx = np.cos(nx_mode * math.pi * (np.arange(nx) + 0.5) / nx)
    fy = np.cos(ny_mode * math.pi * (np.arange(ny) + 0.5) / ny)
    fz = np.cos(nz_mode * math.pi * (np.arange(nz) + 0.5) / nz)
    u = fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    if normalise:
        u = u / np.abs(u).max()
    return u


# ----------------------------------------------------------------- workloads
def plain_tiny():
    """8x8x8 cube at 5 nm, local sphere demag N = 1/3, one uniform mode at
    5 GHz, RK4 at 1 ps for 20 ns; m tilted 1 degree at one seeded azimuth."""
    grid = (8, 8, 8)
    w = TWO_PI * 5.0e9
    az = TWO_PI * np.random.default_rng(1).uniform()
    return Instance(grid=grid, cell=(5e-9,) * 3, **YIG, B0=(0.0, 0.0, w / GAMMA),
                    demag=DEMAG_LOCAL, n_local=(1 / 3, 1 / 3, 1 / 3),
                    omega=np.array([w]), kappa=np.array([TWO_PI * 1e6]), g=np.array([TWO_PI * 50e6]),
                    m0=tilted(grid, 1.0, az), a0=np.zeros(1, complex),
                    method="rk4", dt0=1e-12, tol=0.0, T=20e-9, dt_sample=10e-12)


def paper_sim1(B0=None, g=None, kappa=None, T=16e-9, drive_amp=2e8):
    """Benchmark geometry of Sec. IV and Sim 1 of Table I: an 8x8x1 grid of
    10 nm cells, Ms = 140 kA/m, A = 3.5 pJ/m, alpha = 3e-4, no demag, m(0) =
    +z, one uniform mode at 5 GHz with Q = 5000 (kappa = w_c / 2Q) and
    g/2pi = 50 MHz, B0 at the resonance w_c / gamma unless given [T].  The
    cavity starts empty and is excited by the Gaussian pulse of Sec. IV A
    (sigma = 20 ps, t0 = 0.1 ns); the paper gives no amplitude, the default
    keeps |a| near 1e-2 (linear regime).  RK4 at 1 ps for 16 ns."""
    grid = (8, 8, 1)
    wc = TWO_PI * 5.0e9
    kp = wc / (2 * 5000) if kappa is None else kappa
    gg = TWO_PI * 50e6 if g is None else g
    b = wc / GAMMA if B0 is None else B0
    return Instance(grid=grid, cell=(10e-9,) * 3, Ms=140e3, Aex=3.5e-12, alpha=3e-4,
                    B0=(0.0, 0.0, b), demag=DEMAG_NONE,
                    omega=np.array([wc]), kappa=np.array([kp]), g=np.array([gg]),
                    drive_amp=np.array([complex(drive_amp)]), drive_t0=np.array([0.1e-9]),
                    drive_sigma=np.array([20e-12]),
                    m0=tilted(grid, 0.0, 0.0), a0=np.zeros(1, complex),
                    method="rk4", dt0=1e-12, tol=0.0, T=T, dt_sample=1e-12)


# AFM material of Sim 7 (Table I notes, Sec. IV G): per sublattice
# Ms = 200 kA/m, K = 100 J/m^3 (mu0 H_A = 2K/Ms = 1 mT), alpha = 1e-3,
# A = 3.5 pJ/m; intersublattice field mu0 H_E = 15.9 T (from J_cell)
AFM_PAPER = dict(Ms=200e3, Ku=100.0, alpha=1e-3, Aex=3.5e-12, B_E=15.9)


def paper_sim7(B0=0.0, alpha=None, g=None, csign=(1, 1), m0=None, T=16e-9):
    """Sim 7 of Table I: the two-sublattice antiferromagnet of Sec. IV G on
    the 8x8x1 geometry at 10 nm, easy axis z, bias B0 along z [T], sublattice
    1 along +z and 2 along -z, one uniform mode at 5 GHz with Q = 5000 and
    g/2pi = 50 MHz coupled to the net magnetization (signs +1, +1) and
    excited by the pulse of Sec. IV A; RK4 at 4 ps for 16 ns (4,000 steps)."""
    grid = (8, 8, 1)
    wc = TWO_PI * 5.0e9
    if m0 is None:
        m0 = tilted(grid, 0.0, 0.0, sublattices=2)
    return Instance(grid=grid, cell=(10e-9,) * 3, Ms=AFM_PAPER["Ms"], Aex=AFM_PAPER["Aex"],
                    alpha=AFM_PAPER["alpha"] if alpha is None else alpha, Ku=AFM_PAPER["Ku"],
                    ku_axis=(0.0, 0.0, 1.0), B0=(0.0, 0.0, B0), demag=DEMAG_NONE, sublattices=2,
                    B_E=AFM_PAPER["B_E"], omega=np.array([wc]), kappa=np.array([wc / (2 * 5000)]),
                    g=np.array([TWO_PI * 50e6 if g is None else g]), csign=np.array(csign, np.int8),
                    drive_amp=np.array([2e8 + 0j]), drive_t0=np.array([0.1e-9]), drive_sigma=np.array([20e-12]),
                    m0=m0, a0=np.zeros(1, complex), method="rk4", dt0=4e-12, tol=0.0, T=T, dt_sample=4e-12)


def sweep_sphere(k, count=64, n=32):
    """Instance k of the field sweep: YIG sphere of diameter n cells on an n^3
    grid at 5 nm, FFT demag, gamma B0/2pi from 4.5 to 5.5 GHz, one uniform
    mode at 5 GHz; cavity excited with a(0) = 0.01, m(0) = +z."""
    grid = (n, n, n)
    f = 4.5e9 + 1.0e9 * k / max(1, count - 1)
    mask = sphere_mask(n, n / 2.0)
    m0 = tilted(grid, 0.0, 0.0) * mask[None, None]
    return Instance(grid=grid, cell=(5e-9,) * 3, **YIG, B0=(0.0, 0.0, TWO_PI * f / GAMMA),
                    demag=DEMAG_FFT, geometry=mask,
                    omega=np.array([TWO_PI * 5e9]), kappa=np.array([TWO_PI * 1e6]),
                    g=np.array([TWO_PI * 50e6]),
                    m0=m0.astype(np.float32), a0=np.array([0.01 + 0j]),
                    method="dp45", dt0=1e-13, tol=1e-6, T=100e-9, dt_sample=10e-12)


# Shape term N_zz - N_xx of the volume-averaged demagnetizing tensor of the
# film blocks (cubic cells), written by tests/golden/film_shape_terms.py
# from the oracle and checked against it by a test.
FILM_SHAPE_TERMS = {
    (128, 128, 32): 0.47594880860161287,
    (16, 12, 4): 0.45608201895187317,
    (16, 16, 4): 0.47594880860161287,
    (8, 6, 3): 0.3260951818600196,
    (6, 5, 3): 0.23458240488129364,
    (6, 5, 2): 0.37251086212134954,
    (5, 4, 2): 0.308786125759433,
}


def multimode_film(nx=128, ny=128, nz=32):
    """YIG film at 5 nm with FFT demag and four standing-wave modes at 4.8,
    4.9, 5.0 and 5.1 GHz; g_n/2pi drawn from U(10, 60) MHz; a_1(0) = 1.
    Bias along z: 2 pi 5 GHz / gamma + mu0 Ms (N_zz - N_xx) with the block's
    own volume-averaged tensor, so that its uniform mode sits at 5 GHz."""
    grid = (nx, ny, nz)
    if grid not in FILM_SHAPE_TERMS:
        raise ValueError(f"no stored shape term for a {grid} film")
    g = TWO_PI * 1e6 * np.random.default_rng(3).uniform(10.0, 60.0, 4)
    u = np.stack([standing_wave(grid, n, 1) for n in (1, 2, 3, 4)]).astype(np.float32)
    B0 = TWO_PI * 5.0e9 / GAMMA + MU0 * YIG["Ms"] * FILM_SHAPE_TERMS[grid]
    a0 = np.array([1.0, 0.0, 0.0, 0.0], complex)
    return Instance(grid=grid, cell=(5e-9,) * 3, **YIG, B0=(0.0, 0.0, B0), demag=DEMAG_FFT,
                    omega=TWO_PI * np.array([4.8e9, 4.9e9, 5.0e9, 5.1e9]),
                    kappa=np.full(4, TWO_PI * 1e6), g=g, u=u,
                    m0=tilted(grid, 0.0, 0.0), a0=a0,
                    method="dp45", dt0=1e-13, tol=1e-6, T=200e-9, dt_sample=10e-12)


AFM = dict(Ms=400e3, Aex=3.65e-12, alpha=1e-3, Ku=1e5, B_E=50.0)


def afm_size(k):
    return 64 + 16 * int(round(12 * k / 31))


def afm_instance(k, size=None, nz=16):
    """Instance k of the AFM batch: two sublattices on size^2 x nz at 2 nm,
    B_E = 50 T, K = 1e5 J/m^3 along z, no demag, cavity at the AFM resonance
    coupled to the Neel vector (signs +1, -1) with phase (0, pi/4, pi/2)[k%3]."""
    s = afm_size(k) if size is None else size
    grid = (s, s, nz)
    BA = 2.0 * AFM["Ku"] / AFM["Ms"]
    wc = GAMMA * math.sqrt(2.0 * AFM["B_E"] * BA + BA * BA)      # resonance of Sec. II G, Eq. (15)
    az = TWO_PI * np.random.default_rng(4).uniform()
    return Instance(grid=grid, cell=(2e-9,) * 3, Ms=AFM["Ms"], Aex=AFM["Aex"], alpha=AFM["alpha"],
                    Ku=AFM["Ku"], ku_axis=(0.0, 0.0, 1.0), B0=(0.0, 0.0, 0.0), demag=DEMAG_NONE,
                    sublattices=2, B_E=AFM["B_E"],
                    omega=np.array([wc]), kappa=np.array([TWO_PI * 20e6]), g=np.array([TWO_PI * 40e6]),
                    phi=np.array([(0.0, math.pi / 4, math.pi / 2)[k % 3]]),
                    csign=np.array([1, -1], np.int8),
                    m0=tilted(grid, 1.0, az, sublattices=2), a0=np.zeros(1, complex),
                    method="dp45", dt0=1e-14, tol=1e-6, T=20e-9, dt_sample=1e-12)


def adjoint_film(nx=128, ny=128, nz=32):
    """Film of the multimode workload stepped with RK4 at 0.5 ps for 50 ns."""
    inst = multimode_film(nx, ny, nz)
    inst.method = "rk4"
    inst.dt0 = 0.5e-12
    inst.tol = 0.0
    inst.T = 50e-9
    return inst
