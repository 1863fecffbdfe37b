"""The configurations of the workloads at their specified horizons and
methods, HIP path against the FP64 oracle through the C ABI, plus the
controller and failure paths.

  * the tiny parity run over its whole protocol (20 ns of RK4 at 1 ps) and
    the closed forms of Sec. II B on the device trace;
  * DP45 steps whose error is set by the FP64 cavity alone take the
    oracle's step sequence (counts, step size, trace to 1e-12);
  * non-finite states: status MM_ERR_NONFINITE with the state left at the
    last accepted step; DP45 rejects a non-finite candidate and recovers;
  * DP45 on two sublattices (the AFM batch's method) on a reduced smooth
    instance for each coupling phase, and one tuned batched DP45 step of
    the largest AFM instance;
  * the sweep at full size (32^3 spheres, FFT on 64^3) over 100 DP45 steps
    in the benchmark's batched configuration, and the polariton branches of
    a 20 ns run against Eq. (7) with the measured magnon rate;
  * 50 accepted DP45 steps of the 524,288-cell film."""
import math

import numpy as np
import pytest
import torch

from oracle.spectrum import prony
from paper_2603_03706_amd import mmcav, workloads as W
from tests.helpers import oracle_for, gpu_for, run_oracle, m_err, rel_a_err, variant

pytestmark = pytest.mark.gpu

TWO_PI = 2 * math.pi


def _pair(inst, T, tol=0.0, dt_sample=10e-12, cap=100000):
    st, ctx = oracle_for(inst), gpu_for(inst)
    st.set_sampling(dt_sample, cap)
    ctx.set_sampling(dt_sample, cap)
    print(f"pair grid={inst.grid} S={inst.sublattices} method={inst.method} T={T:g}", flush=True)
    run_oracle(st, T, tol)
    ctx.run(T, tol)
    return st, ctx


def _traces_close(st, ctx, cap, bound, bound_mm=None):
    t_o, a_o, mm_o = st.trace_arrays()
    t, a, mm = ctx.get_trace(cap)
    assert len(t) == len(t_o) and np.array_equal(t, t_o.numpy())
    assert rel_a_err(a, a_o.numpy()) <= bound
    assert rel_a_err(mm, mm_o.numpy()) <= (bound if bound_mm is None else bound_mm)
    return t, a, mm


def _branch_fit(a, mm, dt):
    """Complex rates shared by the cavity and m^- traces, each channel scaled
    to unit peak: m^- also carries the counter-rotating response at -w and
    the two co-rotating branches differ in weight between the channels, so
    six rates are fitted and the caller keeps the ones nearest the band (on
    a macrospin this recovers Eq. (7) to ~0.2 MHz over 20 ns)."""
    return prony(np.stack([a / np.abs(a).max(), mm / np.abs(mm).max()]), dt, 6)


# ----------------------------------------------------- tiny: whole protocol
def test_plain_tiny_full_protocol_20ns():
    """8x8x8 at 5 nm, local N = 1/3, one mode at resonance, RK4 at 1 ps for
    20 ns (20,000 steps): m and the traces against the oracle (1e-4 of the
    north star; measured ~1e-6), the device trace against the rotating-wave
    solution a = i sin(g t) e^{-i w t} e^{-(kappa + gamma_m) t / 2} m^-(0)
    (Sec. II B, 2e-3 of max|a|) and its Rabi period against pi/g (0.2 %)."""
    inst = W.plain_tiny()
    st, ctx = _pair(inst, 20e-9)
    t, a, mm = _traces_close(st, ctx, 100000, 1e-4)
    assert len(t) == 2001
    assert m_err(ctx.get_m(), st) <= 1e-4
    s = ctx.stats()
    assert s["accepted"] == st.accepted == 20000 and s["t"] == st.t
    g, kap, w = inst.g[0], inst.kappa[0], inst.omega[0]
    gm = inst.alpha * w
    pred = 1j * np.sin(g * t) * np.exp(-1j * w * t) * np.exp(-(kap + gm) * t / 2) * mm[0, 0]
    assert np.abs(a[:, 0] - pred).max() <= 2e-3 * np.abs(pred).max()
    rates = _branch_fit(a[:, 0], mm[:, 0], t[1] - t[0])
    lo, hi = (rates[np.argmin(np.abs(-rates.imag - (w + sg * g)))] for sg in (-1, 1))
    split = abs(lo.imag - hi.imag)
    assert abs(math.pi / (split / 2) - math.pi / g) / (math.pi / g) < 2e-3


# ------------------------------------------------------------ controller
def _static_magnet_cavity(a0=1.0 + 0j, **kw):
    """Paper geometry with g = 0 and m along the bias: the magnetisation is
    an exact equilibrium (every torque term is exactly zero in both
    precisions), so the DP45 error norm is the FP64 cavity's alone."""
    return variant(W.paper_sim1(g=0.0), drive_amp=None, a0=np.array([a0]), method="dp45", **kw)


def test_controller_takes_oracle_step_sequence():
    """From dt0 = 50 ps (w dt = 1.6) the first attempts are rejected, the
    step after a rejection may not grow, and the controller then settles:
    the device accepts and rejects exactly the oracle's steps (counts equal,
    next step size and the Hermite trace to 1e-12)."""
    inst = _static_magnet_cavity(dt0=50e-12)
    st, ctx = _pair(inst, 2e-9, tol=1e-6, dt_sample=5e-12)
    s = ctx.stats()
    assert st.rejected >= 1
    assert (s["accepted"], s["rejected"]) == (st.accepted, st.rejected)
    # the error estimate cancels to ~1e-6 of the stage increments, so FP64
    # summation order moves each new step size by ~1e-11 relative
    assert abs(s["dt"] - st.dt) <= 1e-9 * st.dt
    assert s["t"] == st.t
    _traces_close(st, ctx, 100000, 1e-12)
    assert np.array_equal(ctx.get_m(), inst.m0)


def test_dp45_rejects_nonfinite_candidate():
    """A Kerr cavity far beyond the first attempt's stability: the oracle's
    first candidate is non-finite (the error counts as +inf), the step is
    rejected with the smallest factor and the run recovers; the device
    takes the same steps."""
    inst = _static_magnet_cavity(a0=2.0 + 0j, kerr=np.array([1e10]), dt0=1e-9)
    probe = oracle_for(inst)
    with torch.no_grad():
        probe._dp_first()
        _, _, err, _ = probe._dp_step(0.5e-9)
    assert math.isinf(err)
    st, ctx = _pair(inst, 0.5e-9, tol=1e-6, dt_sample=5e-12)
    s = ctx.stats()
    assert st.rejected >= 3 and s["status"] == 0
    assert (s["accepted"], s["rejected"]) == (st.accepted, st.rejected)
    assert abs(s["dt"] - st.dt) <= 1e-9 * st.dt
    _traces_close(st, ctx, 100000, 1e-10)


def _kerr_blowup(g):
    """RK4 at 1 ps on a Kerr cavity with K |a0|^2 dt = 3.2, beyond RK4's
    stability bound 2 sqrt(2): |a| grows faster than exponentially and
    overflows within a few steps."""
    inst = variant(W.paper_sim1(g=g), drive_amp=None, a0=np.array([math.sqrt(3.2) + 0j]),
                   kerr=np.array([1e12]))
    return inst


def _steps_from_start(inst, n):
    """A fresh context advanced by exactly n unclipped steps."""
    ref = gpu_for(inst)
    b = mmcav.Batch([ref])
    b.step(n, 0.0)
    b.close()
    return ref


def test_nonfinite_status_keeps_last_accepted_state():
    """The overflowing cavity (g = 0: both sides decide in FP64): the device
    stops with MM_ERR_NONFINITE after the same number of accepted steps as
    the oracle, and its state is bit for bit that of a run stopped after
    those steps."""
    inst = _kerr_blowup(0.0)
    st = oracle_for(inst)
    status = run_oracle(st, 0.1e-9)
    assert status == -6 and 0 < st.accepted < 100
    ctx = gpu_for(inst)
    with pytest.raises(mmcav.MMError) as e:
        ctx.run(0.1e-9)
    assert e.value.status == mmcav.MM_ERR_NONFINITE
    s = ctx.stats()
    assert s["status"] == -6 and s["accepted"] == st.accepted
    assert s["t"] == pytest.approx(st.t, rel=1e-12)
    assert rel_a_err(ctx.get_a(), st.a.numpy()) <= 1e-12
    ref = _steps_from_start(inst, st.accepted)
    assert np.array_equal(ctx.get_m(), ref.get_m()) and np.array_equal(ctx.get_a(), ref.get_a())
    assert np.isfinite(ctx.get_a().view(np.float64)).all()


def test_nonfinite_through_the_magnet():
    """Coupled (g/2pi = 50 MHz): the overflowing amplitude's feedback makes
    the FP32 torque non-finite before the FP64 amplitude overflows, so the
    device stops no later than the oracle, again with the state of its last
    accepted step."""
    inst = _kerr_blowup(TWO_PI * 50e6)
    st = oracle_for(inst)
    assert run_oracle(st, 0.1e-9) == -6
    ctx = gpu_for(inst)
    with pytest.raises(mmcav.MMError) as e:
        ctx.run(0.1e-9)
    assert e.value.status == mmcav.MM_ERR_NONFINITE
    n = ctx.stats()["accepted"]
    assert 0 < n <= st.accepted
    ref = _steps_from_start(inst, n)
    assert np.array_equal(ctx.get_m(), ref.get_m()) and np.array_equal(ctx.get_a(), ref.get_a())
    assert np.isfinite(ctx.get_m()).all()


# ------------------------------------------------------ AFM batch: DP45
@pytest.mark.parametrize("k", [0, 1, 2])
def test_afm_dp45_two_sublattices(k):
    """The AFM workload's method (DP45, tol 1e-6) on two sublattices at
    16^2 x 4 from its tilted antiparallel state, coupling phase
    (0, pi/4, pi/2)[k], over 0.3 ns (~650 attempted steps, a fifth of them
    rejected).  The device and the oracle take different valid step
    sequences, and at this tolerance the method's own error in the small
    transverse components grows to a few percent of the cavity trace over
    the window, so: over the first 20 ps the traces agree within 2e-3; over
    the whole window the device's distance to the oracle is at most twice
    the oracle's own change when the tolerance is tightened to 1e-7, and so
    is the distance of the exchange-damped Neel resonances (+-w_AFMR) of
    m^- (plus 0.5 MHz)."""
    inst = W.afm_instance(k, size=16, nz=4)
    st, ctx = _pair(inst, 0.3e-9, tol=1e-6, dt_sample=1e-12)
    fine = oracle_for(inst)
    fine.set_sampling(1e-12, 100000)
    run_oracle(fine, 0.3e-9, 1e-7)
    assert ctx.stats()["rejected"] > 0
    t, a, mm = ctx.get_trace(100000)
    _, a_o, mm_o = st.trace_arrays()
    _, a_f, mm_f = fine.trace_arrays()
    a_o, mm_o, a_f, mm_f = a_o.numpy(), mm_o.numpy(), a_f.numpy(), mm_f.numpy()
    assert len(t) == len(a_o) == 301
    head = slice(0, 21)
    assert rel_a_err(a[head], a_o[head]) <= 2e-3 and rel_a_err(mm[head], mm_o[head]) <= 2e-3
    for x, xo, xf in ((a, a_o, a_f), (mm, mm_o, mm_f)):
        assert np.abs(x - xo).max() <= 2 * np.abs(xf - xo).max() + 1e-6 * np.abs(xo).max()
    w_afm = inst.omega[0]
    rates = [prony(np.stack([u[:, 0], v[:, 0]]), 1e-12, 3) for u, v in ((a, mm), (a_o, mm_o), (a_f, mm_f))]
    for sign in (1, -1):
        g_, o_, f_ = (r[np.argmin(np.abs(r.imag + sign * w_afm))] for r in rates)
        assert abs(abs(o_.imag) - w_afm) < TWO_PI * 50e6
        assert abs(g_ - o_) <= 2 * abs(f_ - o_) + TWO_PI * 0.5e6


def test_afm_largest_instance_batched_dp45_step():
    """The 256^2 x 16 instance (2 x 1,048,576 sublattice-cells) inside a
    tuned batch with the smallest one: the first DP45 step against the
    oracle's."""
    insts = [W.afm_instance(0), W.afm_instance(31)]
    ctxs = [gpu_for(i) for i in insts]
    b = mmcav.Batch(ctxs)
    b.tune()
    b.step(1, 1e-6)
    for inst, c in zip(insts, ctxs):
        st = oracle_for(inst)
        with torch.no_grad():
            st._dp_first()
            y, a, err, _ = st._dp_step(inst.dt0)
        assert err / 1e-6 <= 1.0 and c.stats()["accepted"] == 1
        assert float(np.abs(c.get_m().astype(np.float64) - y.numpy()).max()) <= 1e-6
        assert rel_a_err(c.get_a(), a.numpy()) <= 1e-6
    b.close()


# ------------------------------------------------------ sweep at full size
def test_sweep_full_size_batched_100_steps():
    """Instances 0, 32 and 63 of the 64-instance sweep, batched and tuned as
    the benchmark runs them, over 100 DP45 steps (~38 ps): m within 1e-4 and
    traces within 2e-3 of the oracle; the same instances run plain give the
    batched result bit for bit."""
    picks = (0, 32, 63)
    insts = [W.sweep_sphere(k) for k in range(64)]
    ctxs = [gpu_for(i) for i in insts]
    for c in ctxs:
        c.set_sampling(1e-12, 1000)
    b = mmcav.Batch(ctxs)
    b.tune()
    b.step(100, 1e-6)
    for k in picks:
        c = ctxs[k]
        T = c.stats()["t"]
        assert c.stats()["accepted"] + c.stats()["rejected"] == 100
        st = oracle_for(insts[k])
        st.set_sampling(1e-12, 1000)
        print(f"sweep instance {k}: oracle to t = {T:.4g}", flush=True)
        run_oracle(st, T, 1e-6)
        assert m_err(c.get_m(), st) <= 1e-4
        _traces_close(st, c, 1000, 2e-3)
        p = gpu_for(insts[k])
        p.set_sampling(1e-12, 1000)
        pb = mmcav.Batch([p])
        pb.step(100, 1e-6)
        assert np.array_equal(p.get_m(), c.get_m()) and np.array_equal(p.get_a(), c.get_a())
        pb.close()
    b.close()


def test_sweep_polaritons_against_eq7():
    """20 ns on the device for instances 0, 32 and 63 (g/2pi = 50 MHz) and
    the same spheres uncoupled and tilted 1 degree, one batch: the two
    complex rates of each coupled trace lie within 1 MHz of the lossy
    branches of Sec. II B, Eq. (7), evaluated with the magnon rate measured
    on its uncoupled twin (Bloch-Siegert shift ~0.1 MHz)."""
    picks = (0, 32, 63)
    coupled = [W.sweep_sphere(k) for k in picks]
    bare = []
    for k in picks:
        inst = W.sweep_sphere(k)
        mask = inst.geometry
        inst = variant(inst, g=np.array([0.0]), a0=np.array([0j]),
                       m0=(W.tilted(inst.grid, 1.0, 0.3) * mask[None, None]).astype(np.float32))
        bare.append(inst)
    ctxs = [gpu_for(i) for i in coupled + bare]
    for c in ctxs:
        c.set_sampling(10e-12, 2001)
    b = mmcav.Batch(ctxs)
    b.run(20e-9, 1e-6)
    b.close()
    for j, k in enumerate(picks):
        inst = coupled[j]
        wc, kap, g = inst.omega[0], inst.kappa[0], inst.g[0]
        _, _, mm_b = ctxs[3 + j].get_trace(2001)
        rb = prony(mm_b[:, 0], 10e-12, 6)
        sm = rb[np.argmin(np.abs(-rb.imag - inst.gamma * inst.B0[2]))]
        wm, gm = -sm.imag, -sm.real
        _, a, mm = ctxs[j].get_trace(2001)
        got = _branch_fit(a[:, 0], mm[:, 0], 10e-12)
        ev = np.linalg.eigvals(np.array([[wc - 1j * kap, g], [g, wm - 1j * gm]]))
        want = np.sort(ev.real)
        have = np.array([-got[np.argmin(np.abs(-got.imag - w_))].imag for w_ in want])
        print(f"sweep {k}: w_m/2pi = {wm / TWO_PI / 1e9:.6f} GHz, branches {have / TWO_PI / 1e9} "
              f"vs {want / TWO_PI / 1e9}", flush=True)
        assert np.abs(have - want).max() < TWO_PI * 1e6


# ------------------------------------------------------------------ film
def test_multimode_film_50_dp45_steps():
    """The 524,288-cell film (FFT on 256 x 256 x 64, four profiled modes,
    a_1(0) = 1) with DP45 at tol 1e-6 over 32 ps (at least 50 accepted steps
    on both sides): m within 1e-4, traces within 2e-3 of the oracle."""
    inst = W.multimode_film()
    st, ctx = _pair(inst, 32e-12, tol=1e-6, dt_sample=1e-12, cap=100)
    assert ctx.stats()["accepted"] >= 50 and st.accepted >= 50
    assert m_err(ctx.get_m(), st) <= 1e-4
    _traces_close(st, ctx, 100, 2e-3)
