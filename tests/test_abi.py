"""C-ABI checks that need no GPU: the library loads, exports every symbol
the header declares, validates arguments before touching the device, and its
host-side demag tensor agrees with the oracle's independent one."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2603_03706_amd import mmcav

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmcav.h")


def header_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = mmcav.lib()
    names = header_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(mmcav.exported_symbols())


def _params(**kw):
    base = dict(grid=(4, 4, 4), cell=(5e-9,) * 3, Ms=140e3, Aex=3.65e-12, alpha=1e-4)
    base.update(kw)
    return mmcav.make_params(**base)


@pytest.mark.parametrize("bad", [
    dict(grid=(0, 4, 4)), dict(cell=(0.0, 5e-9, 5e-9)), dict(Ms=0.0), dict(alpha=-1.0), dict(gamma=0.0),
    dict(demag=7), dict(sublattices=3), dict(demag=2, sublattices=2), dict(grid=(600, 4, 4), demag=2),
    dict(B0=(float("nan"), 0, 0)), dict(geometry=np.zeros((4, 4, 4), np.uint8)),
])
def test_create_rejects_invalid_parameters(bad):
    L = mmcav.lib()
    p, geo = _params(**bad)
    h = ctypes.c_void_p()
    assert L.mm_create(ctypes.byref(p), ctypes.byref(h)) == mmcav.MM_ERR_ARG
    assert h.value is None
    assert len(L.mm_last_error()) > 0


def test_create_bounds_cells_times_sublattices():
    """The kernels address an instance's fields with unsigned 32-bit byte
    offsets, so cells x sublattices is bounded by 2^26 (accepted exactly at
    the bound, refused one cell beyond it, for one and two sublattices)."""
    L = mmcav.lib()
    for grid, sub, ok in (((512, 512, 256), 1, True), ((512, 512, 257), 1, False),
                          ((512, 512, 128), 2, True), ((512, 512, 129), 2, False)):
        p, _ = _params(grid=grid, sublattices=sub)
        h = ctypes.c_void_p()
        st = L.mm_create(ctypes.byref(p), ctypes.byref(h))
        assert st == (mmcav.MM_OK if ok else mmcav.MM_ERR_ARG), (grid, sub)
        if ok:
            assert L.mm_destroy(h) == mmcav.MM_OK
        else:
            assert h.value is None and b"too large" in L.mm_last_error()


def test_create_destroy_and_host_only_calls():
    L = mmcav.lib()
    p, geo = _params()
    for _ in range(50):
        h = ctypes.c_void_p()
        assert L.mm_create(ctypes.byref(p), ctypes.byref(h)) == mmcav.MM_OK
        # stepper validation happens on the host
        assert L.mm_set_stepper(h, 5, 1e-13, 1e-18, 0.0) == mmcav.MM_ERR_ARG
        assert L.mm_set_stepper(h, mmcav.RK4, -1.0, 1e-18, 0.0) == mmcav.MM_ERR_ARG
        assert L.mm_set_stepper(h, mmcav.DP45, 1e-13, 1e-12, 0.0) == mmcav.MM_ERR_ARG
        assert L.mm_set_stepper(h, mmcav.RK4, 1e-12, 1e-18, 0.0) == mmcav.MM_OK
        assert L.mm_set_sampling(h, 1.5e-12, 10) == mmcav.MM_ERR_ARG      # not a multiple of dt0
        assert L.mm_set_sampling(h, 1e-12, -1) == mmcav.MM_ERR_ARG
        assert L.mm_run(h, -1.0, 0.0) == mmcav.MM_ERR_ARG
        assert L.mm_run(h, 1e-9, 0.0) == mmcav.MM_ERR_STATE             # no modes / state yet
        assert L.mm_set_a(h, None) == mmcav.MM_ERR_ARG
        assert L.mm_set_modes(h, 17, None, None, None, None, None, None) == mmcav.MM_ERR_ARG
        om = np.array([1e10]); ka = np.array([-1.0]); g = np.array([1e8])
        assert L.mm_set_modes(h, 1, om.ctypes.data, ka.ctypes.data, g.ctypes.data, None, None, None) == mmcav.MM_ERR_ARG
        assert L.mm_destroy(h) == mmcav.MM_OK
    assert L.mm_destroy(None) == mmcav.MM_OK
    assert L.mm_batch_create(None, 0, None) == mmcav.MM_ERR_ARG


def test_workspace_bytes_scales_with_modes():
    L = mmcav.lib()
    p, _ = _params(grid=(32, 32, 32), demag=2)
    b0, b4 = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.mm_workspace_bytes(ctypes.byref(p), 0, ctypes.byref(b0)) == 0
    assert L.mm_workspace_bytes(ctypes.byref(p), 4, ctypes.byref(b4)) == 0
    assert b4.value - b0.value >= 4 * 4 * 32 ** 3
    assert L.mm_workspace_bytes(ctypes.byref(p), 17, ctypes.byref(b4)) == mmcav.MM_ERR_ARG


def test_host_demag_tensor_matches_oracle():
    """Two independent implementations of the cell-averaged tensor (the
    library's C++ setup code and the oracle's numpy code) agree."""
    from oracle import newell
    d = (5e-9, 4e-9, 3e-9)
    rng = np.random.default_rng(11)
    pts = [(0, 0, 0), (1, 0, 0), (0, 1, 1), (3, -2, 1), (5, 5, 5), (7, 1, -2), (13, 0, 4), (-30, 12, 5), (90, -40, 7)]
    pts += [tuple(int(v) for v in rng.integers(-60, 61, 3)) for _ in range(20)]
    for r in pts:
        X, Y, Z = r[0] * d[0], r[1] * d[1], r[2] * d[2]
        got = mmcav.demag_tensor(X, Y, Z, *d)
        ref = newell.tensor(np.array([X]), np.array([Y]), np.array([Z]), *d)[:, 0]
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(got - ref).max() <= 1e-10 * scale, (r, got, ref)
    with pytest.raises(mmcav.MMError):
        mmcav.demag_tensor(0, 0, 0, 0.0, 1e-9, 1e-9)


def test_host_demag_tensor_against_high_precision_closed_form():
    """The library's tensor (80-bit closed form below ten cells of distance,
    a tenth-order moment expansion of the averaged kernel beyond) against
    Newell's closed form evaluated here in 40-digit arithmetic, on both
    sides of the switch and far out, all six components."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40

    def q(a, b):
        return a / b if b != 0 else mp.mpf(0)

    def f(x, y, z):
        x, y, z = abs(x), abs(y), abs(z)
        R = mp.sqrt(x * x + y * y + z * z)
        out = (2 * x * x - y * y - z * z) * R / 6
        out += y / 2 * (z * z - x * x) * mp.asinh(q(y, mp.sqrt(x * x + z * z)))
        out += z / 2 * (y * y - x * x) * mp.asinh(q(z, mp.sqrt(x * x + y * y)))
        out -= x * y * z * mp.atan(q(y * z, x * R))
        return out

    def g(x, y, z):
        sg = mp.sign(x) * mp.sign(y)
        x, y, z = abs(x), abs(y), abs(z)
        R = mp.sqrt(x * x + y * y + z * z)
        out = -x * y * R / 3 + x * y * z * mp.asinh(q(z, mp.sqrt(x * x + y * y)))
        out += y / 6 * (3 * z * z - y * y) * mp.asinh(q(x, mp.sqrt(y * y + z * z)))
        out += x / 6 * (3 * z * z - x * x) * mp.asinh(q(y, mp.sqrt(x * x + z * z)))
        out -= z ** 3 / 6 * mp.atan(q(x * y, z * R)) + z * y * y / 2 * mp.atan(q(x * z, y * R))
        out -= z * x * x / 2 * mp.atan(q(y * z, x * R))
        return sg * out

    def diff(fn, X, Y, Z, a, b, c):
        w = (-1, 2, -1)
        acc = mp.mpf(0)
        for i in range(3):
            for j in range(3):
                for k in range(3):
                    acc += w[i] * w[j] * w[k] * fn(X + (i - 1) * a, Y + (j - 1) * b, Z + (k - 1) * c)
        return acc / (4 * mp.pi * a * b * c)

    d = (5e-9, 4e-9, 3e-9)
    D = [mp.mpf(5), mp.mpf(4), mp.mpf(3)]
    for r in [(0, 0, 0), (1, 2, 0), (6, -5, 3), (9, 3, -2), (11, 0, 1), (20, -7, 12), (40, 25, -30)]:
        X, Y, Z = (r[i] * D[i] for i in range(3))
        ref = np.array([float(v) * 1.0 for v in (
            diff(f, X, Y, Z, D[0], D[1], D[2]), diff(f, Y, X, Z, D[1], D[0], D[2]), diff(f, Z, Y, X, D[2], D[1], D[0]),
            diff(g, X, Y, Z, D[0], D[1], D[2]), diff(g, X, Z, Y, D[0], D[2], D[1]), diff(g, Y, Z, X, D[1], D[2], D[0]))])
        got = mmcav.demag_tensor(r[0] * d[0], r[1] * d[1], r[2] * d[2], *d)
        # the tensor is dimensionless: cells in nm or in m give the same values
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (r, got, ref)
