"""Python binding of libmmcav.so (ctypes; argument marshalling only).

Every step of the stepper runs in the HIP library.  PyTorch supplies device
memory (a uint8 tensor bound as the workspace) and the stream; it is
imported first so that the library shares the HIP runtime torch loaded.
There is no fallback: if the library is missing, loading fails loudly.
"""
import ctypes
import os

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmmcav.so")

MM_OK, MM_ERR_ARG, MM_ERR_HIP, MM_ERR_OOM, MM_ERR_STATE, MM_ERR_DT_UNDERFLOW, MM_ERR_NONFINITE = 0, -1, -2, -3, -4, -5, -6
DEMAG_NONE, DEMAG_LOCAL, DEMAG_FFT = 0, 1, 2
RK4, DP45, RK4_SPLIT = 0, 1, 2
MAX_MODES = 16

_STATUS_NAMES = {0: "MM_OK", -1: "MM_ERR_ARG", -2: "MM_ERR_HIP", -3: "MM_ERR_OOM", -4: "MM_ERR_STATE",
                 -5: "MM_ERR_DT_UNDERFLOW", -6: "MM_ERR_NONFINITE"}


class MMError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("Ms", ctypes.c_double), ("Aex", ctypes.c_double), ("alpha", ctypes.c_double),
                ("Ku", ctypes.c_double), ("ku_axis", ctypes.c_double * 3), ("gamma", ctypes.c_double),
                ("B0", ctypes.c_double * 3), ("demag", ctypes.c_int32), ("n_local", ctypes.c_double * 3),
                ("geometry", ctypes.c_void_p), ("sublattices", ctypes.c_int32), ("B_E", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64), ("t", ctypes.c_double),
                ("dt", ctypes.c_double), ("dt_min_seen", ctypes.c_double), ("dt_max_seen", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("status", ctypes.c_int32)]


_lib = None

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "mm_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(_P)]),
    "mm_destroy": (ctypes.c_int, [_P]),
    "mm_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "mm_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "mm_set_stream": (ctypes.c_int, [_P, _P]),
    "mm_set_modes": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P]),
    "mm_set_m": (ctypes.c_int, [_P, _P]),
    "mm_set_a": (ctypes.c_int, [_P, _P]),
    "mm_set_drive": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "mm_set_parametric": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "mm_set_cavity_model": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "mm_adjoint_trace": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "mm_set_stepper": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "mm_set_sampling": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int64]),
    "mm_run": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double]),
    "mm_run_noalloc": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double]),
    "mm_get_m": (ctypes.c_int, [_P, _P]),
    "mm_get_a": (ctypes.c_int, [_P, _P]),
    "mm_get_trace": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)]),
    "mm_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(Stats)]),
    "mm_get_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_size_t)]),
    "mm_set_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "mm_batch_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(_P)]),
    "mm_batch_run": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double]),
    "mm_batch_step": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_double]),
    "mm_batch_begin": (ctypes.c_int, [_P, ctypes.c_double]),
    "mm_batch_advance": (ctypes.c_int, [_P, ctypes.c_int64]),
    "mm_batch_end": (ctypes.c_int, [_P]),
    "mm_batch_destroy": (ctypes.c_int, [_P]),
    "mm_batch_profile": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _P, _P, _P, _P,
                                        ctypes.POINTER(ctypes.c_int32)]),
    "mm_batch_tune": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_size_t]),
    "mm_batch_counts": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "mm_batch_set_fft_path": (ctypes.c_int, [_P, ctypes.c_int32]),
    "mm_batch_set_fft_x": (ctypes.c_int, [_P, ctypes.c_int32]),
    "mm_batch_set_streams": (ctypes.c_int, [_P, ctypes.c_int32]),
    "mm_batch_tune_fft": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_size_t]),
    "mm_batch_get_streams": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "mm_run_record": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int32]),
    "mm_run_record_adaptive": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int32]),
    "mm_get_step_log": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int64)]),
    "mm_adjoint": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "mm_demag_tensor": (ctypes.c_int, [ctypes.c_double] * 6 + [_P]),
    "mm_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libmmcav.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_03706_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != MM_OK:
        raise MMError(status, lib().mm_last_error().decode())
    return status


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def demag_tensor(X, Y, Z, dx, dy, dz):
    out = np.zeros(6)
    _check(lib().mm_demag_tensor(X, Y, Z, dx, dy, dz, _ptr(out)))
    return out


def make_params(grid, cell, Ms, Aex, alpha, gamma=1.76e11, Ku=0.0, ku_axis=(0, 0, 1), B0=(0, 0, 0),
                demag=DEMAG_NONE, n_local=(0, 0, 0), geometry=None, sublattices=1, B_E=0.0):
    p = Params()
    p.nx, p.ny, p.nz = (int(v) for v in grid)
    p.dx, p.dy, p.dz = (float(v) for v in cell)
    p.Ms, p.Aex, p.alpha, p.Ku, p.gamma = float(Ms), float(Aex), float(alpha), float(Ku), float(gamma)
    p.ku_axis[:] = [float(v) for v in ku_axis]
    p.B0[:] = [float(v) for v in B0]
    p.demag = int(demag)
    p.n_local[:] = [float(v) for v in n_local]
    p.sublattices = int(sublattices)
    p.B_E = float(B_E)
    geo = None
    if geometry is not None:
        geo = np.ascontiguousarray(geometry, dtype=np.uint8)
        p.geometry = geo.ctypes.data
    return p, geo


class Context:
    """One stepper instance.  workspace='torch' binds a torch uint8 tensor as
    device memory; 'library' lets the library allocate."""

    def __init__(self, grid, cell, Ms, Aex, alpha, n_modes=1, workspace="torch", stream="torch", **kw):
        self._lib = lib()
        p, geo = make_params(grid, cell, Ms, Aex, alpha, **kw)
        self.params = p
        self.grid = tuple(int(v) for v in grid)
        self.S = int(kw.get("sublattices", 1))
        self.N = 0
        handle = ctypes.c_void_p()
        _check(self._lib.mm_create(ctypes.byref(p), ctypes.byref(handle)))
        self.h = handle
        self._ws = None
        if workspace == "torch":
            nbytes = ctypes.c_size_t()
            _check(self._lib.mm_workspace_bytes(ctypes.byref(p), int(n_modes), ctypes.byref(nbytes)))
            self._ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            off = (-base) % 256
            _check(self._lib.mm_bind_workspace(self.h, ctypes.c_void_p(base + off), int(nbytes.value)))
        if stream == "torch":
            _check(self._lib.mm_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    @classmethod
    def from_instance(cls, inst, workspace="torch"):
        """Create, set modes, state and stepper from a workloads.Instance."""
        c = cls(inst.grid, inst.cell, inst.Ms, inst.Aex, inst.alpha, n_modes=len(inst.omega),
                workspace=workspace, gamma=inst.gamma, Ku=inst.Ku, ku_axis=inst.ku_axis, B0=inst.B0,
                demag=inst.demag, n_local=inst.n_local, geometry=inst.geometry,
                sublattices=inst.sublattices, B_E=inst.B_E)
        c.set_modes(inst.omega, inst.kappa, inst.g, u=inst.u, phi=inst.phi, csign=inst.csign)
        if any(getattr(inst, k, None) is not None for k in ("g_back", "kerr", "photon_coupling")):
            c.set_cavity_model(inst.g_back, inst.kerr, inst.photon_coupling)
        if getattr(inst, "drive_amp", None) is not None:
            c.set_drive(inst.drive_amp, inst.drive_t0, inst.drive_sigma)
        if getattr(inst, "param_lambda", None) is not None:
            c.set_parametric(inst.param_lambda, inst.param_wp)
        c.set_m(inst.m0)
        c.set_a(inst.a0)
        c.set_stepper({"rk4": RK4, "dp45": DP45, "split": RK4_SPLIT}[inst.method], inst.dt0)
        return c

    def set_modes(self, omega, kappa, g, u=None, phi=None, csign=None):
        n = len(omega)
        om = np.ascontiguousarray(omega, np.float64)
        ka = np.ascontiguousarray(kappa, np.float64)
        gg = np.ascontiguousarray(g, np.float64)
        uu = None if u is None else np.ascontiguousarray(u, np.float32)
        ph = None if phi is None else np.ascontiguousarray(phi, np.float64)
        cs = None if csign is None else np.ascontiguousarray(csign, np.int8)
        _check(self._lib.mm_set_modes(self.h, n, _ptr(om), _ptr(ka), _ptr(gg), _ptr(uu), _ptr(ph), _ptr(cs)))
        self.N = n

    def set_cavity_model(self, g_back=None, kerr=None, coupling=None):
        """Nonreciprocal backward coupling g_b and self-Kerr K per mode, and
        the direct mode coupling J [N][N] (all rad/s); None leaves that
        variant off (all None: reciprocal, linear, uncoupled modes)."""
        gb = None if g_back is None else np.ascontiguousarray(g_back, np.float64)
        kr = None if kerr is None else np.ascontiguousarray(kerr, np.float64)
        jc = None if coupling is None else np.ascontiguousarray(coupling, np.float64)
        n = 0 if gb is None and kr is None and jc is None else self.N
        _check(self._lib.mm_set_cavity_model(self.h, n, _ptr(gb), _ptr(kr), _ptr(jc)))

    def set_parametric(self, lam=None, omega_p=None):
        """Degenerate parametric pump -i lam_n e^{-2 i wp_n t} conj(a_n) per
        mode (complex strengths [rad/s], wp [rad/s]); lam=None switches it off."""
        if lam is None:
            _check(self._lib.mm_set_parametric(self.h, 0, None, None))
            return
        la = np.asarray(lam, np.complex128)
        buf = np.ascontiguousarray(np.stack([la.real, la.imag], axis=-1).reshape(-1))
        wp = np.ascontiguousarray(omega_p, np.float64)
        _check(self._lib.mm_set_parametric(self.h, len(la), _ptr(buf), _ptr(wp)))

    def set_drive(self, amp=None, t0=None, sigma=None):
        """Gaussian cavity drive A_n exp(-((t - t0_n)/sigma_n)^2 / 2) per mode
        (complex amplitudes [1/s]); amp=None switches it off."""
        if amp is None:
            _check(self._lib.mm_set_drive(self.h, 0, None, None, None))
            return
        a = np.asarray(amp, np.complex128)
        buf = np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1).reshape(-1))
        t = np.ascontiguousarray(t0, np.float64)
        sg = np.ascontiguousarray(sigma, np.float64)
        _check(self._lib.mm_set_drive(self.h, len(a), _ptr(buf), _ptr(t), _ptr(sg)))

    def set_m(self, m):
        mm = np.ascontiguousarray(m, np.float32)
        _check(self._lib.mm_set_m(self.h, _ptr(mm)))

    def set_a(self, a):
        a = np.asarray(a, np.complex128)
        buf = np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1).reshape(-1))
        _check(self._lib.mm_set_a(self.h, _ptr(buf)))

    def set_stepper(self, method, dt0, dt_min=1e-18, dt_max=0.0):
        _check(self._lib.mm_set_stepper(self.h, int(method), float(dt0), float(dt_min), float(dt_max)))

    def set_sampling(self, dt_sample, max_samples):
        _check(self._lib.mm_set_sampling(self.h, float(dt_sample), int(max_samples)))

    def run(self, T, tol=0.0):
        _check(self._lib.mm_run(self.h, float(T), float(tol)))

    def run_noalloc(self, T, tol=0.0):
        """mm_run whose per-run scratch is the library's fixed device array (no device allocation)."""
        _check(self._lib.mm_run_noalloc(self.h, float(T), float(tol)))

    def run_record(self, T, checkpoint_every=256):
        _check(self._lib.mm_run_record(self.h, float(T), int(checkpoint_every)))

    def run_record_adaptive(self, T, tol, checkpoint_every=256):
        """DP45 run of T at tol keeping its accepted step sizes, with
        checkpoints along their replay, for a later adjoint."""
        _check(self._lib.mm_run_record_adaptive(self.h, float(T), float(tol), int(checkpoint_every)))

    def step_log(self):
        """Accepted step sizes of the last adaptive recorded run (negative:
        clipped onto the end time)."""
        n = ctypes.c_int64(0)
        _check(self._lib.mm_get_step_log(self.h, None, ctypes.byref(n)))
        out = np.zeros(n.value)
        _check(self._lib.mm_get_step_log(self.h, _ptr(out), ctypes.byref(n)))
        return out

    def adjoint(self, dL_da, dL_dm=None, dL_dtrace=None):
        """Gradients of the loss of the recorded run; dL_da complex (N,) at T
        (may be None with dL_dtrace), dL_dtrace complex (steps + 1, N): the
        derivative with respect to a at every step end and the start."""
        nx, ny, nz = self.grid
        dl = np.zeros(self.N, np.complex128) if dL_da is None else np.asarray(dL_da, np.complex128)
        buf = np.ascontiguousarray(np.stack([dl.real, dl.imag], axis=-1).reshape(-1))
        dm = None if dL_dm is None else np.ascontiguousarray(dL_dm, np.float32)
        gu = np.zeros((max(self.N, 1), nz, ny, nx), np.float32)
        gg = np.zeros(max(self.N, 1))
        ga = np.zeros(1)
        gb = np.zeros(3)
        ga0 = np.zeros(2 * max(self.N, 1))
        gm0 = np.zeros((self.S, 3, nz, ny, nx), np.float32)
        if dL_dtrace is None:
            _check(self._lib.mm_adjoint(self.h, _ptr(buf), _ptr(dm), _ptr(gu), _ptr(gg), _ptr(ga), _ptr(gb),
                                        _ptr(ga0), _ptr(gm0)))
        else:
            dt = np.asarray(dL_dtrace, np.complex128).reshape(-1, self.N)
            tb = np.ascontiguousarray(np.stack([dt.real, dt.imag], axis=-1).reshape(-1))
            _check(self._lib.mm_adjoint_trace(self.h, _ptr(tb), dt.shape[0], _ptr(buf), _ptr(dm), _ptr(gu),
                                              _ptr(gg), _ptr(ga), _ptr(gb), _ptr(ga0), _ptr(gm0)))
        return {"u": gu[:self.N], "g": gg[:self.N], "alpha": float(ga[0]), "B0": gb,
                "a0": ga0[0:2 * self.N:2] + 1j * ga0[1:2 * self.N:2], "m0": gm0}

    def get_m(self):
        nx, ny, nz = self.grid
        out = np.empty((self.S, 3, nz, ny, nx), np.float32)
        _check(self._lib.mm_get_m(self.h, _ptr(out)))
        return out

    def get_a(self):
        out = np.empty(2 * max(self.N, 1))
        _check(self._lib.mm_get_a(self.h, _ptr(out)))
        return out[0:2 * self.N:2] + 1j * out[1:2 * self.N:2]

    def get_trace(self, capacity):
        t = np.empty(capacity)
        a = np.empty((capacity, max(self.N, 1), 2))
        m = np.empty((capacity, max(self.N, 1), 2))
        n = ctypes.c_int64(capacity)
        _check(self._lib.mm_get_trace(self.h, _ptr(t), _ptr(a), _ptr(m), ctypes.byref(n)))
        k = n.value
        return t[:k], a[:k, :self.N, 0] + 1j * a[:k, :self.N, 1], m[:k, :self.N, 0] + 1j * m[:k, :self.N, 1]

    def stats(self):
        s = Stats()
        _check(self._lib.mm_get_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def get_state(self):
        n = ctypes.c_size_t()
        _check(self._lib.mm_get_state(self.h, None, ctypes.byref(n)))
        buf = np.empty(n.value, np.uint8)
        _check(self._lib.mm_get_state(self.h, _ptr(buf), ctypes.byref(n)))
        return buf

    def set_state(self, blob):
        blob = np.ascontiguousarray(blob, np.uint8)
        _check(self._lib.mm_set_state(self.h, _ptr(blob), blob.size))

    def close(self):
        if getattr(self, "h", None):
            self._lib.mm_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Instances advanced together by one launch sequence per stage."""

    def __init__(self, contexts):
        self._lib = lib()
        self.contexts = list(contexts)
        arr = (ctypes.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        handle = ctypes.c_void_p()
        _check(self._lib.mm_batch_create(arr, len(self.contexts), ctypes.byref(handle)))
        self.h = handle

    def run(self, T, tol=0.0):
        _check(self._lib.mm_batch_run(self.h, float(T), float(tol)))

    def step(self, steps, tol=0.0):
        _check(self._lib.mm_batch_step(self.h, int(steps), float(tol)))

    def begin(self, tol=0.0):
        """Open an unbounded run (run-start derivative, graph capture); returns without waiting."""
        _check(self._lib.mm_batch_begin(self.h, float(tol)))

    def advance(self, steps):
        """Enqueue exactly `steps` more attempted steps of the open run; returns without waiting."""
        _check(self._lib.mm_batch_advance(self.h, int(steps)))

    def end(self):
        """Wait for the open run and read every instance's statistics back."""
        _check(self._lib.mm_batch_end(self.h))

    def counts(self):
        """(accepted, rejected) steps summed over the instances once the
        enqueued work has finished; allowed during an open run."""
        acc, rej = ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib.mm_batch_counts(self.h, ctypes.byref(acc), ctypes.byref(rej)))
        return acc.value, rej.value

    def tune(self, streams=True):
        """Autotune the sub-batch count (unless streams=False) and the FFT
        tiles / path per grid shape; returns the report."""
        import json
        buf = ctypes.create_string_buffer(65536)
        fn = self._lib.mm_batch_tune if streams else self._lib.mm_batch_tune_fft
        _check(fn(self.h, buf, len(buf)))
        return json.loads(buf.value.decode())

    YZ_PATHS = {"fused": 0, "reg": 1, "split": 2, "reg8": 3, "xch": 4, "splitx": 5}

    def set_fft_path(self, path):
        """Force the demag y-z strategy ("fused", "reg", "reg8", "xch", "split" or "splitx") for every grid shape."""
        _check(self._lib.mm_batch_set_fft_path(self.h, self.YZ_PATHS[path]))

    def set_fft_x(self, path):
        """Force the x-pass strategy ("lds", "reg" or "stage") for every grid shape."""
        _check(self._lib.mm_batch_set_fft_x(self.h, {"lds": 0, "reg": 1, "stage": 2}[path]))

    def set_streams(self, parts):
        """Run the batch as `parts` concurrent sub-batches (1 = one launch sequence)."""
        _check(self._lib.mm_batch_set_streams(self.h, int(parts)))

    def streams(self):
        n = ctypes.c_int32()
        _check(self._lib.mm_batch_get_streams(self.h, ctypes.byref(n)))
        return n.value

    def profile(self, steps, tol=0.0, cap=32):
        names = ctypes.create_string_buffer(48 * cap)
        launches = np.zeros(cap, np.int64)
        ms = np.zeros(cap)
        nbytes = np.zeros(cap)
        n = ctypes.c_int32()
        _check(self._lib.mm_batch_profile(self.h, int(steps), float(tol), cap, names, _ptr(launches), _ptr(ms),
                                          _ptr(nbytes), ctypes.byref(n)))
        out = []
        for i in range(min(n.value, cap)):
            nm = names.raw[48 * i:48 * (i + 1)].split(b"\0", 1)[0].decode()
            out.append({"name": nm, "launches": int(launches[i]), "total_ms": float(ms[i]),
                        "bytes_per_launch": float(nbytes[i])})
        return out

    def close(self):
        if getattr(self, "h", None):
            self._lib.mm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RecordedRunFunction(torch.autograd.Function):
    """Differentiable run of one instance: the forward pass records the run
    on the GPU (fixed-step RK4: mm_run_record; adaptive DP45 at inst.tol:
    mm_run_record_adaptive, whose adjoint holds the accepted step sizes;
    checkpoints every `checkpoint_every` steps), the backward pass is the
    library's discrete adjoint (mm_adjoint, or mm_adjoint_trace when the
    trace output of an RK4 run carries a gradient).  Inputs that carry
    gradients: the mode profiles u (float32
    [N][nz][ny][nx]), the couplings g (float64 [N], rad/s), the damping alpha
    (float64 scalar) and the bias field B0 (float64 [3], T).  Outputs: a(T)
    as float64 [N][2] (real, imaginary part), m(T) as float32
    [S][3][nz][ny][nx] and, with `with_trace`, a at the start and every step
    end as float64 [steps + 1][N][2] (else an empty tensor), so that losses
    on the trace (spectra) differentiate too.  The other parameters come from
    `inst` (workloads.Instance, method rk4 or dp45).  Arguments and results are only
    marshalled here; both passes run in the library's kernels."""

    @staticmethod
    def forward(fctx, u, g, alpha, B0, inst, T, checkpoint_every, with_trace=False):
        import dataclasses
        run = dataclasses.replace(inst, u=u.detach().cpu().numpy().astype(np.float32),
                                  g=g.detach().cpu().numpy().astype(np.float64),
                                  alpha=float(alpha.detach().cpu()),
                                  B0=tuple(float(v) for v in B0.detach().cpu()))
        if run.method not in ("rk4", "dp45"):
            raise ValueError("the discrete adjoint is built for RK4 runs and adaptive DP45 runs")
        if run.method == "dp45" and with_trace:
            raise ValueError("losses on the trace are built for fixed-step RK4 runs")
        c = Context.from_instance(run)
        steps = int(round(T / run.dt0))
        if with_trace:
            c.set_sampling(run.dt0, steps + 1)
        if run.method == "dp45":
            c.run_record_adaptive(T, run.tol, checkpoint_every)
        else:
            c.run_record(T, checkpoint_every)
        a = c.get_a()
        tr = torch.zeros(0, dtype=torch.float64)
        if with_trace:
            _, at, _ = c.get_trace(steps + 1)
            if at.shape[0] != steps + 1:
                raise RuntimeError("trace of the recorded run has %d samples, expected %d" % (at.shape[0], steps + 1))
            tr = torch.from_numpy(np.stack([at.real, at.imag], axis=-1))
        fctx.context = c
        # outputs on the device of u; gradients go back on each input's own
        # device and dtype
        fctx.like = [(x.device, x.dtype) for x in (u, g, alpha, B0)]
        dev = u.device
        return (torch.from_numpy(np.stack([a.real, a.imag], axis=-1)).to(dev), torch.from_numpy(c.get_m()).to(dev),
                tr.to(dev))

    @staticmethod
    def backward(fctx, grad_a, grad_m, grad_trace):
        c = fctx.context
        ga = np.zeros((c.N, 2)) if grad_a is None else grad_a.detach().cpu().numpy().astype(np.float64)
        gm = None if grad_m is None else grad_m.detach().cpu().numpy().astype(np.float32)
        gt = None
        if grad_trace is not None and grad_trace.numel() > 0:
            q = grad_trace.detach().cpu().numpy().astype(np.float64)
            gt = q[..., 0] + 1j * q[..., 1]
        g = c.adjoint(ga[:, 0] + 1j * ga[:, 1], gm, gt)
        c.close()
        fctx.context = None
        grads = (torch.from_numpy(g["u"]), torch.from_numpy(g["g"]), torch.tensor(g["alpha"], dtype=torch.float64),
                 torch.from_numpy(np.asarray(g["B0"], np.float64)))
        grads = tuple(x.to(device=d, dtype=t) for x, (d, t) in zip(grads, fctx.like))
        return grads + (None, None, None, None)


def recorded_run(inst, T, u, g, alpha, B0, checkpoint_every=256, with_trace=False):
    """a(T) [N][2] and m(T) of `inst` run for T with the given u, g, alpha and
    B0 (tensors; gradients flow through the GPU discrete adjoint), and with
    `with_trace` also a at the start and every step end, [steps + 1][N][2]."""
    a, m, tr = RecordedRunFunction.apply(u, g, alpha, B0, inst, T, checkpoint_every, with_trace)
    return (a, m, tr) if with_trace else (a, m)


def exported_symbols():
    """Names declared in include/mmcav.h."""
    return list(_SIGS)
