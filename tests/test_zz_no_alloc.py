"""The no-allocation run (mm_run_noalloc) against mm_run, through the C ABI.

mm_run_noalloc takes its per-run scratch from the library's fixed device
array instead of allocating; its arithmetic is mm_run's, so its outputs must
equal mm_run's bit for bit.  Two calls in a row on one GPU, the second on a
smaller instance, check that the array's leftover contents from the first
call do not leak into the second."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2603_03706_amd import mmcav, workloads as W
from tests.helpers import gpu_for

pytestmark = pytest.mark.gpu


def _outputs(c, cap):
    st = c.stats()
    return c.get_m(), c.get_a(), c.get_trace(cap), (st["accepted"], st["rejected"], st["t"], st["dt"])


def _assert_same(x, y):
    (m, a, tr, st), (m1, a1, tr1, st1) = x, y
    assert np.array_equal(m, m1)
    assert np.array_equal(a, a1)
    for u, v in zip(tr, tr1):
        assert np.array_equal(u, v)
    assert st == st1


def _case(inst, T, tol, cap=2000):
    ref = gpu_for(inst)
    ref.set_sampling(5e-12, cap)
    ref.run(T, tol)
    want = _outputs(ref, cap)
    ref.close()
    got = gpu_for(inst)
    got.set_sampling(5e-12, cap)
    print(f"mm_run_noalloc grid={inst.grid} demag={inst.demag} method={inst.method} T={T:g}", flush=True)
    status = mmcav.lib().mm_run_noalloc(got.h, ctypes.c_double(T), ctypes.c_double(tol))
    assert status == mmcav.MM_OK, mmcav.lib().mm_last_error()
    have = _outputs(got, cap)
    got.close()
    return want, have


def test_noalloc_equals_run_two_calls_second_smaller():
    big = W.sweep_sphere(40, count=64, n=16)          # 16^3 sphere, FFT demag on 32^3, DP45
    small = W.sweep_sphere(7, count=64, n=8)          # 8^3 sphere, FFT demag on 16^3, DP45
    want, have = _case(big, 0.2e-9, 1e-6)
    _assert_same(have, want)
    assert have[3][0] > 10
    want, have = _case(small, 0.15e-9, 1e-6)
    _assert_same(have, want)


def test_noalloc_wide_y_split_path():
    """A grid whose padded y (256) takes the split y-z passes, whose y-pass
    spectra are carved from the scratch array too: equal to mm_run."""
    inst = W.Instance(grid=(4, 100, 20), cell=(5e-9, 4e-9, 3e-9), Ms=140e3, Aex=3.65e-12, alpha=0.01,
                      B0=(0.01, 0.0, 0.15), demag=W.DEMAG_FFT,
                      omega=np.array([2 * np.pi * 5e9]), kappa=np.array([2 * np.pi * 2e6]),
                      g=np.array([2 * np.pi * 80e6]), m0=W.tilted((4, 100, 20), 10.0, 0.3),
                      a0=np.array([0.05 + 0.02j]), method="dp45", dt0=0.2e-12)
    want, have = _case(inst, 20e-12, 1e-6)
    _assert_same(have, want)
    assert have[3][0] > 5


def test_noalloc_rk4_local_demag_and_resume():
    inst = W.plain_tiny()
    inst.T = 0.0
    ref = gpu_for(inst)
    ref.run(50e-12)
    ref.run(30e-12)
    got = gpu_for(inst)
    got.run_noalloc(50e-12)
    got.run(30e-12)                                    # a plain run continues from it
    assert np.array_equal(got.get_m(), ref.get_m())
    assert np.array_equal(got.get_a(), ref.get_a())


def test_noalloc_takes_no_device_memory():
    inst = W.sweep_sphere(3, count=64, n=16)
    warm = gpu_for(inst)
    warm.run_noalloc(20e-12, 1e-6)                     # first use of every kernel and copy path
    warm.close()
    c = gpu_for(inst)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    c.run_noalloc(0.1e-9, 1e-6)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    c.close()


def test_noalloc_rejects_instance_beyond_scratch():
    film = W.multimode_film()                          # 524,288 cells, FFT demag on 256x256x64
    c = gpu_for(film)
    with pytest.raises(mmcav.MMError) as e:
        c.run_noalloc(1e-12, 1e-6)
    assert e.value.status == mmcav.MM_ERR_ARG
    assert "scratch" in str(e.value)
    c.close()
