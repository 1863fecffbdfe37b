"""HIP path against the FP64 oracle, element by element, through the C ABI.

Fixed-step runs compare states and traces directly (max|dm| and
max_t|da|/max_t|a| within 1e-4 over the run; tighter where the run is
short).  Adaptive runs compare the sampled traces and spectral peaks."""
import math

import numpy as np
import pytest
import torch

from oracle.spectrum import spectrum, peaks
from paper_2603_03706_amd import workloads as W
from tests.helpers import oracle_for, gpu_for, run_oracle, m_err, rel_a_err, variant

pytestmark = pytest.mark.gpu

TWO_PI = 2 * math.pi


def _random_state(grid, seed, S=1, geometry=None):
    rng = np.random.default_rng(seed)
    nx, ny, nz = grid
    m = rng.normal(size=(S, 3, nz, ny, nx))
    m[:, 2] += 2.0
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    if geometry is not None:
        m = m * geometry[None, None]
        m[:, 2] += (1 - geometry)[None]          # non-magnetic cells: any finite value
    return m.astype(np.float32)


def _run_pair(inst, T, tol=0.0, dt_sample=None, cap=100000):
    st = oracle_for(inst)
    ctx = gpu_for(inst)
    if dt_sample:
        st.set_sampling(dt_sample, cap)
        ctx.set_sampling(dt_sample, cap)
    run_oracle(st, T, tol)
    ctx.run(T, tol)
    return st, ctx


# ------------------------------------------------------------- plain tiny
def test_plain_tiny_rk4_2ns():
    inst = W.plain_tiny()
    st, ctx = _run_pair(inst, 2e-9, dt_sample=10e-12)
    t_o, a_o, mm_o = st.trace_arrays()
    t_g, a_g, mm_g = ctx.get_trace(100000)
    assert len(t_g) == len(t_o) == 201
    assert np.array_equal(t_g, t_o.numpy())
    assert rel_a_err(a_g, a_o.numpy()) <= 1e-5
    assert rel_a_err(mm_g, mm_o.numpy()) <= 1e-5
    assert m_err(ctx.get_m(), st) <= 1e-5
    s = ctx.stats()
    assert s["accepted"] == st.accepted == 2000 and s["t"] == st.t


def test_reduction_against_fsum():
    """m^- at t = 0 (first trace sample) is an FP64 sum over cells."""
    inst = W.plain_tiny()
    inst = variant(inst, m0=_random_state(inst.grid, 3))
    ctx = gpu_for(inst)
    ctx.set_sampling(1e-12, 4)
    ctx.run(1e-12)
    _, _, mm = ctx.get_trace(4)
    m = inst.m0.astype(np.float64)
    m = m / np.linalg.norm(m, axis=1, keepdims=True)
    m32 = m.astype(np.float32).astype(np.float64)
    ref_r = math.fsum(m32[0, 0].ravel()) / m32[0, 0].size
    ref_i = -math.fsum(m32[0, 1].ravel()) / m32[0, 1].size
    assert abs(mm[0, 0].real - ref_r) <= 1e-15 * max(1.0, abs(ref_r))
    assert abs(mm[0, 0].imag - ref_i) <= 1e-15 * max(1.0, abs(ref_i))


# ------------------------------------------------------------ FFT demag
@pytest.mark.parametrize("grid,mask", [((5, 4, 3), None), ((8, 8, 8), "sphere"), ((6, 1, 4), None),
                                       ((16, 8, 1), None), ((1, 6, 5), None), ((12, 10, 7), "sphere")])
def test_fft_demag_rk4(grid, mask):
    nx, ny, nz = grid
    geo = None
    if mask == "sphere":
        geo = W.sphere_mask(nx, nx / 2.0)[:nz, :ny, :nx].copy() if nx == ny == nz else None
        if geo is None:
            idx = lambda n: np.arange(n) + 0.5 - n / 2.0
            zz, yy, xx = np.meshgrid(idx(nz), idx(ny), idx(nx), indexing="ij")
            geo = ((xx / (nx / 2)) ** 2 + (yy / (ny / 2)) ** 2 + (zz / (nz / 2)) ** 2 <= 1).astype(np.uint8)
    inst = W.Instance(grid=grid, cell=(5e-9, 4e-9, 3e-9), Ms=140e3, Aex=3.65e-12, alpha=0.01,
                      B0=(0.01, 0.0, 0.15), demag=W.DEMAG_FFT, geometry=geo,
                      omega=np.array([TWO_PI * 5e9]), kappa=np.array([TWO_PI * 2e6]), g=np.array([TWO_PI * 80e6]),
                      m0=_random_state(grid, 5, geometry=geo), a0=np.array([0.05 + 0.02j]),
                      method="rk4", dt0=0.1e-12)
    st, ctx = _run_pair(inst, 30e-12, dt_sample=1e-12)
    assert m_err(ctx.get_m(), st) <= 2e-5
    _, a_o, _ = st.trace_arrays()
    _, a_g, _ = ctx.get_trace(1000)
    assert rel_a_err(a_g, a_o.numpy()) <= 2e-5


def test_fft_demag_split_path():
    """A padded (y, z) plane too large for LDS takes the split y / z passes."""
    grid = (3, 100, 40)
    inst = W.Instance(grid=grid, cell=(5e-9,) * 3, Ms=140e3, Aex=3.65e-12, alpha=0.01,
                      B0=(0.0, 0.0, 0.2), demag=W.DEMAG_FFT,
                      omega=np.array([TWO_PI * 5e9]), kappa=np.array([TWO_PI * 1e6]), g=np.array([TWO_PI * 50e6]),
                      m0=_random_state(grid, 9), a0=np.array([0.01 + 0j]), method="rk4", dt0=0.1e-12)
    st, ctx = _run_pair(inst, 2e-12)
    assert m_err(ctx.get_m(), st) <= 2e-5
    assert rel_a_err(ctx.get_a(), st.a.numpy()) <= 2e-5


# ------------------------------------------------------ multimode, AFM, Phi
def test_multimode_profiled_film():
    inst = W.multimode_film(16, 12, 4)
    inst = variant(inst, method="rk4", dt0=0.2e-12, m0=_random_state((16, 12, 4), 21),
                   a0=np.array([0.3, 0.1j, -0.2, 0.05 + 0.05j]), phi=np.array([0.0, 0.3, math.pi / 2, 1.0]))
    st, ctx = _run_pair(inst, 40e-12, dt_sample=1e-12)
    assert m_err(ctx.get_m(), st) <= 2e-5
    _, a_o, mm_o = st.trace_arrays()
    _, a_g, mm_g = ctx.get_trace(1000)
    assert rel_a_err(a_g, a_o.numpy()) <= 2e-5
    assert rel_a_err(mm_g, mm_o.numpy()) <= 1e-4


def test_afm_neel_coupling_rk4_short():
    """Random two-sublattice state: strongly nonlinear, it amplifies a 1e-7
    perturbation about 5x in 0.2 ps (and 1e5x in 4 ps), so the horizon is
    kept short."""
    inst = W.afm_instance(1, size=8, nz=4)
    inst = variant(inst, method="rk4", dt0=2e-14, m0=_random_state((8, 8, 4), 31, S=2) * np.array([1, -1]).reshape(2, 1, 1, 1, 1),
                   a0=np.array([0.2 + 0.1j]))
    st, ctx = _run_pair(inst, 0.2e-12, dt_sample=2e-14)
    assert m_err(ctx.get_m(), st) <= 5e-6
    _, a_o, _ = st.trace_arrays()
    _, a_g, _ = ctx.get_trace(1000)
    assert rel_a_err(a_g, a_o.numpy()) <= 2e-6


def test_afm_neel_coupling_rk4_smooth():
    """The tilted antiparallel state of the AFM workload with a long-wave
    perturbation, coupled to the Neel vector at phase pi/4, over 20 ps."""
    inst = W.afm_instance(1, size=16, nz=4)
    m0 = inst.m0.astype(np.float64).copy()
    x = (np.arange(16) + 0.5) / 16
    m0[:, 0] += 0.05 * np.cos(np.pi * x)[None, None, None, :] * np.array([1, -1]).reshape(2, 1, 1, 1)
    inst = variant(inst, method="rk4", dt0=2e-14, m0=m0.astype(np.float32), a0=np.array([0.2 + 0.1j]))
    st, ctx = _run_pair(inst, 20e-12, dt_sample=1e-12)
    assert m_err(ctx.get_m(), st) <= 2e-5
    _, a_o, _ = st.trace_arrays()
    _, a_g, _ = ctx.get_trace(1000)
    assert rel_a_err(a_g, a_o.numpy()) <= 2e-5


def test_local_demag_anisotropy_geometry_rk4():
    grid = (9, 7, 5)
    geo = (np.random.default_rng(2).uniform(size=(5, 7, 9)) > 0.3).astype(np.uint8)
    inst = W.Instance(grid=grid, cell=(4e-9, 5e-9, 6e-9), Ms=300e3, Aex=5e-12, alpha=0.02, Ku=2e4,
                      ku_axis=(0.2, 0.3, 1.0), B0=(0.02, -0.01, 0.1), demag=W.DEMAG_LOCAL, n_local=(0.2, 0.3, 0.5),
                      geometry=geo, omega=np.array([TWO_PI * 6e9, TWO_PI * 7e9]), kappa=np.array([1e7, 3e7]),
                      g=np.array([TWO_PI * 40e6, TWO_PI * 20e6]), m0=_random_state(grid, 8, geometry=geo),
                      a0=np.array([0.1, -0.2j]), method="rk4", dt0=0.1e-12)
    st, ctx = _run_pair(inst, 20e-12, dt_sample=1e-12)
    assert m_err(ctx.get_m(), st) <= 2e-5
    _, a_o, _ = st.trace_arrays()
    _, a_g, _ = ctx.get_trace(1000)
    assert rel_a_err(a_g, a_o.numpy()) <= 2e-5


# --------------------------------------------------------------- adaptive
def test_dp45_adaptive_trace_and_peaks():
    inst = W.sweep_sphere(32, n=8)
    inst = variant(inst, dt0=1e-13)
    st, ctx = _run_pair(inst, 2e-9, tol=1e-6, dt_sample=10e-12)
    t_o, a_o, mm_o = st.trace_arrays()
    t_g, a_g, mm_g = ctx.get_trace(100000)
    assert len(t_g) == len(t_o) == 201
    assert np.abs(t_g - t_o.numpy()).max() < 1e-21
    # two different accepted-step sequences, each with local errors <= tol:
    # the traces agree to the accumulated global error, the peaks to 0.5 MHz
    assert rel_a_err(a_g, a_o.numpy()) <= 2e-3
    f, S_o = spectrum(a_o.numpy()[:, 0] , 10e-12)
    _, S_g = spectrum(a_g[:, 0], 10e-12)
    po = peaks(f, S_o, count=2, fmin=3e9, fmax=7e9)
    pg = peaks(f, S_g, count=2, fmin=3e9, fmax=7e9)
    assert np.allclose(sorted(po), sorted(pg), atol=0.5e6)
    s = ctx.stats()
    assert s["status"] == 0 and s["t"] == st.t
    assert abs(s["accepted"] - st.accepted) <= max(2, st.accepted // 20)


def test_dt_underflow_reported():
    inst = W.plain_tiny()
    inst = variant(inst, method="dp45", dt0=1e-13)
    ctx = gpu_for(inst)
    ctx.set_stepper(1, 1e-13, 1e-15)
    from paper_2603_03706_amd import mmcav
    with pytest.raises(mmcav.MMError) as e:
        ctx.run(1e-12, 1e-30)
    assert e.value.status == mmcav.MM_ERR_DT_UNDERFLOW
    s = ctx.stats()
    assert s["accepted"] == 0 and s["t"] == 0.0
    m = ctx.get_m()
    assert np.isfinite(m).all()


# ---------------------------------------------- batching, determinism, state
def test_batched_equals_plain_bitwise():
    from paper_2603_03706_amd import mmcav
    insts = [W.sweep_sphere(k, count=4, n=8) for k in range(4)]
    plain = []
    for inst in insts:
        c = gpu_for(inst)
        c.set_sampling(10e-12, 1000)
        c.run(0.3e-9, 1e-6)
        plain.append((c.get_m(), c.get_a(), c.get_trace(1000)))
    ctxs = [gpu_for(inst) for inst in insts]
    for c in ctxs:
        c.set_sampling(10e-12, 1000)
    b = mmcav.Batch(ctxs)
    b.run(0.3e-9, 1e-6)
    for c, (m, a, tr) in zip(ctxs, plain):
        assert np.array_equal(c.get_m(), m)
        assert np.array_equal(c.get_a(), a)
        t2 = c.get_trace(1000)
        assert np.array_equal(t2[0], tr[0]) and np.array_equal(t2[1], tr[1]) and np.array_equal(t2[2], tr[2])
    b.close()


def test_batch_streams_bitwise():
    """Splitting a batch into concurrent sub-batches (streams) changes no
    instance's arithmetic: states, amplitudes and traces are bit-identical
    for 1, 2 and 3 parts, on a batch mixing two grid shapes."""
    from paper_2603_03706_amd import mmcav
    insts = [W.sweep_sphere(k, count=5, n=8 if k % 2 else 12) for k in range(5)]
    out = {}
    for parts in (1, 2, 3):
        ctxs = [gpu_for(inst) for inst in insts]
        for c in ctxs:
            c.set_sampling(10e-12, 1000)
        b = mmcav.Batch(ctxs)
        assert b.streams() == 1
        b.set_streams(parts)
        assert b.streams() == parts
        b.run(0.2e-9, 1e-6)
        b.step(3, 1e-6)
        out[parts] = [(c.get_m(), c.get_a(), c.get_trace(1000), c.stats()["accepted"]) for c in ctxs]
        b.close()
        for c in ctxs:
            c.close()
    for parts in (2, 3):
        for (m, a, tr, acc), (m1, a1, tr1, acc1) in zip(out[parts], out[1]):
            assert acc == acc1
            assert np.array_equal(m, m1) and np.array_equal(a, a1)
            assert all(np.array_equal(x, y) for x, y in zip(tr, tr1))
    c = gpu_for(insts[0])
    b = mmcav.Batch([c])
    assert b.streams() == 1
    for bad in (0, 9):
        with pytest.raises(mmcav.MMError):
            b.set_streams(bad)
    b.close()


def test_deterministic_and_resume_bitwise():
    inst = W.sweep_sphere(10, count=16, n=8)
    runs = []
    for _ in range(2):
        c = gpu_for(inst)
        c.run(0.2e-9, 1e-6)
        runs.append((c.get_m(), c.get_a()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    c = gpu_for(inst)
    c.run(0.1e-9, 1e-6)
    blob = c.get_state()
    c.run(0.1e-9, 1e-6)
    m_ref, a_ref = c.get_m(), c.get_a()
    c2 = gpu_for(inst)
    c2.set_state(blob)
    c2.run(0.1e-9, 1e-6)
    assert np.array_equal(c2.get_m(), m_ref) and np.array_equal(c2.get_a(), a_ref)


def test_library_owned_workspace_matches_torch_workspace():
    inst = W.plain_tiny()
    c1 = gpu_for(inst, workspace="torch")
    c2 = gpu_for(inst, workspace="library")
    c1.run(50e-12)
    c2.run(50e-12)
    assert np.array_equal(c1.get_m(), c2.get_m()) and np.array_equal(c1.get_a(), c2.get_a())


# -------------------------------------------------------- full-size checks
def test_sweep_batch_full_size_first_step():
    """The 64-instance sweep (32^3 spheres, FFT on 64^3) batched as the
    benchmark runs it (tuned: sub-batch count and FFT strategies): one DP45
    step, sampled instances against the oracle."""
    from paper_2603_03706_amd import mmcav
    insts = [W.sweep_sphere(k) for k in range(64)]
    ctxs = [gpu_for(inst) for inst in insts]
    b = mmcav.Batch(ctxs)
    b.tune()
    b.step(1, 1e-6)
    for k in (0, 31, 63):
        st = oracle_for(insts[k])
        with torch.no_grad():
            st._dp_first()
            y, a, err, st7 = st._dp_step(insts[k].dt0)
        assert err / 1e-6 <= 1.0
        assert float(np.abs(ctxs[k].get_m().astype(np.float64) - y.numpy()).max()) <= 1e-6
        assert rel_a_err(ctxs[k].get_a(), a.numpy()) <= 1e-6
    b.close()


def test_multimode_film_full_size_one_step():
    inst = W.multimode_film()
    inst = variant(inst, method="rk4", dt0=0.5e-12, m0=_random_state(inst.grid, 4))
    st, ctx = _run_pair(inst, 0.5e-12)
    assert m_err(ctx.get_m(), st) <= 1e-6
    assert rel_a_err(ctx.get_a(), st.a.numpy()) <= 1e-6


@pytest.mark.parametrize("k", [0, 31])
def test_afm_batch_sizes_one_step(k):
    inst = W.afm_instance(k)
    inst = variant(inst, method="rk4", dt0=2e-14)
    st, ctx = _run_pair(inst, 1e-13)
    assert m_err(ctx.get_m(), st) <= 1e-6


def test_tuned_batch_keeps_parity():
    """The autotuner changes only tile shapes / the y-z path: results stay
    within FP32 rounding of the untuned batch and the state is not advanced."""
    from paper_2603_03706_amd import mmcav
    insts = [W.sweep_sphere(k, count=3, n=12) for k in range(3)]
    for inst in insts:
        inst.method, inst.dt0 = "rk4", 0.2e-12
    ref = [gpu_for(i) for i in insts]
    b0 = mmcav.Batch(ref)
    ctxs = [gpu_for(i) for i in insts]
    for c in ctxs + ref:
        c.set_sampling(5e-12, 100)
    b0.run(20e-12)
    b1 = mmcav.Batch(ctxs)
    m0 = [c.get_m() for c in ctxs]
    rep = b1.tune()
    assert len(rep) == b1.streams() and all(r["path"] in ("fused", "reg", "reg8", "xch", "split", "splitx") for r in rep)
    assert all(r["streams"] == b1.streams() and len(r["streams_ms_per_step"]) == 3 for r in rep)
    # the timed steps of the tuner leave no trace: state, counters, samples
    assert all(c.stats()["accepted"] == 0 and c.stats()["t"] == 0.0 for c in ctxs)
    assert all(np.array_equal(c.get_m(), m) for c, m in zip(ctxs, m0))
    assert all(len(c.get_trace(100)[0]) == 0 for c in ctxs)
    b1.run(20e-12)
    for c, r in zip(ctxs, ref):
        assert np.abs(c.get_m() - r.get_m()).max() <= 2e-6
        t1, a1, _ = c.get_trace(100)
        t0, a0, _ = r.get_trace(100)
        assert np.array_equal(t1, t0) and np.abs(a1 - a0).max() <= 1e-5 * np.abs(a0).max()
    st = oracle_for(insts[1])
    run_oracle(st, 20e-12)
    assert m_err(ctxs[1].get_m(), st) <= 2e-5
    b0.close()
    b1.close()


@pytest.mark.gpu
@pytest.mark.parametrize("shape", [(12, 12, 12), (10, 6, 5), (16, 6, 5), (16, 12, 9), (16, 5, 7), (32, 7, 9),
                                   (8, 20, 17), (8, 40, 20), (8, 40, 12)])
def test_fft_yz_paths_agree(shape):
    """The y-z strategies of the demag convolution (LDS-fused, register lines,
    two-pass lines with an LDS exchange, split passes) and the x-pass
    strategies (LDS tiles, register lines, inside the stage kernels) give the
    same trajectory to FP32 rounding, and the oracle's within the parity
    bound, on a sphere and on ragged boxes (odd row counts per workgroup among
    them: 16 x 5 x 7 and 32 x 7 x 9 leave 3 and 15 x-rows in the last
    workgroup of 512 cells; 8 x 20 x 17 and 8 x 40 x 20 pad y to 64 and 128
    and z to 64, with z rows past nz in every column).  For padded (y, z) of
    (64, 64) and (128, 32) (8 x 20 x 17, 8 x 40 x 12) the two-pass kernel
    carries the real planes kx = 0 and Px/2 in one work item."""
    from paper_2603_03706_amd import mmcav
    if shape == (12, 12, 12):
        inst = variant(W.sweep_sphere(5, count=8, n=12), method="rk4", dt0=0.2e-12)
    else:
        inst = W.Instance(grid=shape, cell=(5e-9, 4e-9, 3e-9), Ms=140e3, Aex=3.65e-12, alpha=0.01,
                          B0=(0.01, 0.0, 0.15), demag=W.DEMAG_FFT,
                          omega=np.array([TWO_PI * 5e9]), kappa=np.array([TWO_PI * 2e6]),
                          g=np.array([TWO_PI * 80e6]), m0=_random_state(shape, 17),
                          a0=np.array([0.05 + 0.02j]), method="rk4", dt0=0.2e-12)
    st = oracle_for(inst)
    run_oracle(st, 20e-12)
    out = {}
    combos = [("fused", "lds"), ("reg", "reg"), ("split", "lds"), ("fused", "reg")]
    if shape[0] & (shape[0] - 1) == 0:       # x passes inside the stage kernels need nx = 2^k
        combos += [("reg", "stage"), ("split", "stage")]
    if shape[2] > 8:                         # eight lanes per z column need a padded z of 32 or 64
        combos += [("reg8", "lds"), ("xch", "lds"), ("splitx", "lds")]
        if shape[0] & (shape[0] - 1) == 0:
            combos += [("reg8", "stage"), ("xch", "stage"), ("splitx", "stage")]
    for path, xpath in combos:
        c = gpu_for(inst)
        b = mmcav.Batch([c])
        b.set_fft_path(path)
        b.set_fft_x(xpath)
        b.run(20e-12)
        out[path, xpath] = c.get_m()
        assert m_err(out[path, xpath], st) <= 2e-5, (path, xpath)
        b.close()
        c.close()
    # paths differ by FP32 rounding only (summation orders of the line
    # transforms), accumulated over 100 steps: up to 2.7e-6 with 128-point y lines
    ref = out["fused", "lds"]
    diff = {key: float(np.abs(m - ref).max()) for key, m in out.items()}
    print(shape, diff)
    assert max(diff.values()) <= 4e-6, diff


@pytest.mark.gpu
@pytest.mark.parametrize("shape", [(4, 100, 20), (8, 70, 9)])
def test_split_exchange_wide_y(shape):
    """Padded y of 256 (wider than the one-workgroup y-z kernels take): the
    split passes whose y passes use the two-pass line transforms agree with
    the LDS split passes to FP32 rounding and with the oracle within the
    parity bound, for padded z of 64 and of 32 (with z rows past nz)."""
    from paper_2603_03706_amd import mmcav
    inst = W.Instance(grid=shape, cell=(5e-9, 4e-9, 3e-9), Ms=140e3, Aex=3.65e-12, alpha=0.01,
                      B0=(0.01, 0.0, 0.15), demag=W.DEMAG_FFT,
                      omega=np.array([TWO_PI * 5e9]), kappa=np.array([TWO_PI * 2e6]),
                      g=np.array([TWO_PI * 80e6]), m0=_random_state(shape, 23),
                      a0=np.array([0.05 + 0.02j]), method="rk4", dt0=0.2e-12)
    st = oracle_for(inst)
    run_oracle(st, 20e-12)
    out = {}
    for path in ("split", "splitx"):
        c = gpu_for(inst)
        b = mmcav.Batch([c])
        b.set_fft_path(path)
        b.set_fft_x("lds")
        b.run(20e-12)
        out[path] = c.get_m()
        assert m_err(out[path], st) <= 2e-5, path
        b.close()
        c.close()
    assert np.abs(out["splitx"] - out["split"]).max() <= 2e-6


@pytest.mark.gpu
def test_fft_path_rejects_unfit_shape():
    """A shape outside the register strategies' sizes is refused without change."""
    from paper_2603_03706_amd import mmcav
    grid = (100, 3, 2)       # padded (256, 8, 4): outside both register strategies
    inst = W.Instance(grid=grid, cell=(5e-9,) * 3, Ms=140e3, Aex=3.65e-12, alpha=0.01,
                      B0=(0.0, 0.0, 0.2), demag=W.DEMAG_FFT,
                      omega=np.array([TWO_PI * 5e9]), kappa=np.array([TWO_PI * 1e6]), g=np.array([TWO_PI * 50e6]),
                      m0=_random_state(grid, 3), a0=np.array([0.01 + 0j]), method="rk4", dt0=0.1e-12)
    c = gpu_for(inst)
    b = mmcav.Batch([c])
    with pytest.raises(mmcav.MMError):
        b.set_fft_path("reg")
    with pytest.raises(mmcav.MMError):
        b.set_fft_path("reg8")
    with pytest.raises(mmcav.MMError):
        b.set_fft_path("xch")
    with pytest.raises(mmcav.MMError):
        b.set_fft_x("reg")
    with pytest.raises(mmcav.MMError):
        b.set_fft_x("stage")
    b.set_fft_path("split")
    b.set_fft_x("lds")
    b.close()
    c.close()
