"""Cavity-model variants on the HIP path (nonreciprocal coupling g_f != g_b,
Sec. II A; self-Kerr term, Sec. V) against the oracle and closed forms."""
import math

import numpy as np
import pytest

from oracle.spectrum import prony
from paper_2603_03706_amd import workloads as W
from tests.helpers import oracle_for, gpu_for, run_oracle, m_err, rel_a_err, variant

pytestmark = pytest.mark.gpu

TWO_PI = 2 * math.pi


def _pair(inst, T, tol=0.0, dt_sample=10e-12, cap=2000):
    st, ctx = oracle_for(inst), gpu_for(inst)
    st.set_sampling(dt_sample, cap)
    ctx.set_sampling(dt_sample, cap)
    run_oracle(st, T, tol)
    ctx.run(T, tol)
    return st, ctx


@pytest.mark.parametrize("method", ["rk4", "dp45"])
def test_kerr_uncoupled_closed_form(method):
    """g = 0: the FP64 Kerr cavity on the device follows the oracle to
    rounding and the exact solution (|a| = |a0| e^{-kappa t}, phase
    w t + K |a0|^2 (1 - e^{-2 kappa t}) / 2 kappa) to the method error."""
    w, kp, K, a0 = TWO_PI * 5e9, TWO_PI * 20e6, TWO_PI * 2e9, 0.3 + 0.1j
    inst = variant(W.paper_sim1(g=0.0), drive_amp=None, kappa=np.array([kp]), kerr=np.array([K]),
                   a0=np.array([a0]), method=method, dt0=0.5e-12)
    st, ctx = _pair(inst, 2e-9, tol=1e-12)
    t_o, a_o, _ = st.trace_arrays()
    t, a, _ = ctx.get_trace(2000)
    assert len(t) == len(t_o) == 201
    assert rel_a_err(a, a_o.numpy()) <= 1e-12
    want = a0 * np.exp((-1j * w - kp) * t) * np.exp(-1j * K * abs(a0) ** 2 * (1 - np.exp(-2 * kp * t)) / (2 * kp))
    assert np.abs(a[:, 0] - want).max() / abs(a0) < (2e-7 if method == "rk4" else 2e-8)


def test_kerr_coupled_parity():
    """Kerr cavity coupled to the 8x8x1 film of Sec. IV, RK4 at 1 ps for 1 ns."""
    inst = variant(W.paper_sim1(), drive_amp=None, kerr=np.array([TWO_PI * 1e9]),
                   a0=np.array([0.1 + 0j]))
    st, ctx = _pair(inst, 1e-9)
    _, a_o, mm_o = st.trace_arrays()
    _, a, mm = ctx.get_trace(2000)
    assert rel_a_err(a, a_o.numpy()) <= 1e-5
    assert rel_a_err(mm, mm_o.numpy()) <= 1e-5
    assert m_err(ctx.get_m(), st) <= 1e-5


def test_nonreciprocal_parity_and_splitting():
    """g_f = 2pi 50 MHz in the cavity equation, g_b = 2pi 12.5 MHz in the
    feedback: parity with the oracle over 1 ns, then the rates of a 10 ns run
    at w_c +- sqrt(g_f g_b) (1 MHz)."""
    gb = TWO_PI * 12.5e6
    inst = variant(W.paper_sim1(), drive_amp=None, g_back=np.array([gb]), a0=np.array([0.01 + 0j]))
    st, ctx = _pair(inst, 1e-9)
    _, a_o, mm_o = st.trace_arrays()
    _, a, mm = ctx.get_trace(2000)
    assert rel_a_err(a, a_o.numpy()) <= 1e-5
    assert rel_a_err(mm, mm_o.numpy()) <= 1e-5
    ctx = gpu_for(inst)
    ctx.set_sampling(10e-12, 2000)
    ctx.run(10e-9)
    _, a, mm = ctx.get_trace(2000)
    s = prony(np.stack([a[:, 0], mm[:, 0]]), 10e-12, 4)
    got = np.sort(-s[s.imag < 0].imag)
    wc = inst.omega[0]
    half = math.sqrt(inst.g[0] * gb)
    assert got.size == 2
    assert np.abs(got - np.array([wc - half, wc + half])).max() / TWO_PI < 1e6


def test_cavity_model_arguments_and_adjoint_gate():
    from paper_2603_03706_amd import mmcav
    ctx = gpu_for(W.paper_sim1(T=0.1e-9))
    with pytest.raises(mmcav.MMError) as e:
        mmcav._check(ctx._lib.mm_set_cavity_model(ctx.h, 2, None, None, None))
    assert e.value.status == mmcav.MM_ERR_ARG
    with pytest.raises(mmcav.MMError) as e:
        ctx.set_cavity_model(kerr=[float("inf")])
    assert e.value.status == mmcav.MM_ERR_ARG
    ctx.set_cavity_model(g_back=[TWO_PI * 10e6])
    with pytest.raises(mmcav.MMError) as e:
        ctx.run_record(10e-12, 4)
    assert e.value.status == mmcav.MM_ERR_STATE
    ctx.set_cavity_model()
    ctx.run_record(10e-12, 4)


def _two_mode(w1, w2, g, J, **kw):
    inst = W.paper_sim1(g=0.0)
    return variant(inst, drive_amp=None, omega=np.array([w1, w2]), kappa=np.array([TWO_PI * 1e6] * 2),
                   g=np.array([g, g]), photon_coupling=np.array([[0.0, J], [J, 0.0]]), **kw)


@pytest.mark.parametrize("method", ["rk4", "dp45"])
def test_photon_coupling_two_cavities(method):
    """g = 0, two equal cavities joined by J: device against the oracle
    (FP64 cavity step on both sides) and the exact beat solution."""
    w, J = TWO_PI * 5e9, TWO_PI * 80e6
    a0 = np.array([0.02 + 0.01j, -0.005j])
    inst = _two_mode(w, w, 0.0, J, a0=a0, method=method, dt0=0.5e-12)
    st, ctx = _pair(inst, 3e-9, tol=1e-14, cap=1000)
    _, a_o, _ = st.trace_arrays()
    t, a, _ = ctx.get_trace(1000)
    assert len(t) == 301 and rel_a_err(a, a_o.numpy()) <= 1e-12
    e = np.exp((-1j * w - inst.kappa[0]) * t)
    want = np.stack([e * (a0[0] * np.cos(J * t) - 1j * a0[1] * np.sin(J * t)),
                     e * (a0[1] * np.cos(J * t) - 1j * a0[0] * np.sin(J * t))], axis=1)
    assert np.abs(a - want).max() / np.abs(a0).max() < (2e-7 if method == "rk4" else 1e-9)


def test_three_mode_direct_coupling():
    """Two cavities at w_m -+ g, both coupled to the 8x8x1 film and to each
    other by J (Eq. (14) with H_13 = J): parity with the oracle over 1 ns, then
    the rates of a 10 ns run at the eigenvalues of the 3x3 matrix (1 MHz)."""
    g, J = TWO_PI * 50e6, TWO_PI * 30e6
    wm = TWO_PI * 5e9
    inst = _two_mode(wm - g, wm + g, g, J, a0=np.array([0.01 + 0j, 0j]))
    inst = variant(inst, B0=(0.0, 0.0, wm / W.GAMMA))
    st, ctx = _pair(inst, 1e-9)
    _, a_o, mm_o = st.trace_arrays()
    _, a, mm = ctx.get_trace(2000)
    assert rel_a_err(a, a_o.numpy()) <= 1e-5 and rel_a_err(mm, mm_o.numpy()) <= 1e-5
    ctx = gpu_for(inst)
    ctx.set_sampling(10e-12, 2000)
    ctx.run(10e-9)
    _, a, mm = ctx.get_trace(2000)
    # the fit uses the cavity channels: m^- carries the FP32 rounding of the
    # state, which a sixth-order fit over three channels absorbs as a
    # spurious rate and a bias of a few MHz
    s = prony(np.stack([a[:, 0], a[:, 1]]), 10e-12, 6)
    got = np.sort(-s[s.imag < 0].imag)
    got = got[(got > TWO_PI * 4e9) & (got < TWO_PI * 6e9)]
    want = np.linalg.eigvalsh(np.array([[wm - g, g, J], [g, wm, g], [J, g, wm + g]]))
    assert got.size == 3 and np.abs(got - want).max() / TWO_PI < 1e6


def test_photon_coupling_arguments():
    from paper_2603_03706_amd import mmcav
    w = TWO_PI * 5e9
    ctx = gpu_for(_two_mode(w, w, 0.0, TWO_PI * 10e6, a0=np.zeros(2, complex)))
    for J in ([[0.0, 1e6], [2e6, 0.0]], [[1e6, 1e6], [1e6, 0.0]], [[0.0, np.nan], [np.nan, 0.0]]):
        with pytest.raises(mmcav.MMError) as e:
            ctx.set_cavity_model(coupling=J)
        assert e.value.status == mmcav.MM_ERR_ARG
    # the adjoint covers the mode coupling (its gradient is checked with the
    # adjoint tests); only a backward coupling is refused
    ctx.run_record(10e-12, 4)


def test_batch_mixing_variants_equals_plain_bitwise():
    """One batch whose instances carry different cavity options (the pulse,
    a Kerr term, a backward coupling, two modes joined by J, the split
    scheme) gives each instance exactly its plain run: every option lives
    in the instance's own descriptor."""
    from paper_2603_03706_amd import mmcav
    w = TWO_PI * 5e9
    base = W.paper_sim1(T=0.5e-9)
    insts = [base,
             variant(base, drive_amp=None, kerr=np.array([TWO_PI * 1e9]), a0=np.array([0.1 + 0j])),
             variant(base, g_back=np.array([TWO_PI * 20e6])),
             _two_mode(w - TWO_PI * 30e6, w + TWO_PI * 30e6, TWO_PI * 50e6, TWO_PI * 40e6,
                       a0=np.array([0.01 + 0j, 0j]), T=0.5e-9),
             variant(base, method="split")]
    plain = []
    for inst in insts:
        c = gpu_for(inst)
        c.set_sampling(10e-12, 100)
        c.run(base.T)
        plain.append((c.get_m(), c.get_a(), c.get_trace(100)))
    ctxs = [gpu_for(inst) for inst in insts]
    for c in ctxs:
        c.set_sampling(10e-12, 100)
    b = mmcav.Batch(ctxs)
    b.run(base.T)
    for c, (m, a, tr) in zip(ctxs, plain):
        assert np.array_equal(c.get_m(), m) and np.array_equal(c.get_a(), a)
        t2 = c.get_trace(100)
        assert all(np.array_equal(x, y) for x, y in zip(t2, tr))
    b.close()


# ------------------------------------------- degenerate parametric pump
@pytest.mark.parametrize("method", ["rk4", "dp45"])
def test_parametric_uncoupled_closed_form(method):
    """g = 0, pump -i lam e^{-2 i wp t} conj(a) with |lam| = 1.5 kappa at
    20 MHz detuning: the FP64 cavity on the device follows the oracle to
    rounding and the rotating-frame matrix exponential to the method error."""
    from tests.test_oracle_pins import _parametric_rotating
    wp, kp = TWO_PI * 5e9, TWO_PI * 20e6
    lam = 1.5 * kp * np.exp(0.4j)
    w = wp + TWO_PI * 20e6
    a0 = 0.3 + 0.1j
    inst = variant(W.paper_sim1(g=0.0), drive_amp=None, omega=np.array([w]), kappa=np.array([kp]),
                   param_lambda=np.array([lam]), param_wp=np.array([wp]), a0=np.array([a0]),
                   method=method, dt0=0.5e-12)
    st, ctx = _pair(inst, 2e-9, tol=1e-12)
    t_o, a_o, _ = st.trace_arrays()
    t, a, _ = ctx.get_trace(2000)
    assert len(t) == len(t_o) == 201
    assert rel_a_err(a, a_o.numpy()) <= 1e-12
    want = np.exp(-1j * wp * t) * _parametric_rotating(lam, kp, w - wp, t, a0)
    assert np.abs(a[:, 0] - want).max() / np.abs(want).max() < (2e-7 if method == "rk4" else 2e-8)


def test_parametric_coupled_parity():
    """The pumped cavity (|lam| = 0.8 kappa, pump at twice the cavity
    frequency) coupled to the 8x8x1 film of Sec. IV, RK4 at 1 ps for 1 ns,
    and the same with the operator-split scheme: against the oracle."""
    wc, kp = W.paper_sim1().omega[0], W.paper_sim1().kappa[0]
    for method in ("rk4", "split"):
        inst = variant(W.paper_sim1(), drive_amp=None, param_lambda=np.array([0.8 * kp * np.exp(-0.6j)]),
                       param_wp=np.array([wc]), a0=np.array([0.05 + 0.02j]), method=method)
        st, ctx = _pair(inst, 1e-9)
        _, a_o, mm_o = st.trace_arrays()
        _, a, mm = ctx.get_trace(2000)
        assert rel_a_err(a, a_o.numpy()) <= 1e-5
        assert rel_a_err(mm, mm_o.numpy()) <= 1e-5
        assert m_err(ctx.get_m(), st) <= 1e-5


def test_parametric_argument_checks():
    from paper_2603_03706_amd import mmcav
    ctx = gpu_for(W.paper_sim1(T=0.1e-9))
    with pytest.raises(mmcav.MMError):
        ctx.set_parametric([1e6, 2e6], [1e10, 1e10])          # count != modes
    with pytest.raises(mmcav.MMError):
        ctx.set_parametric([complex(np.nan)], [1e10])
    ctx.set_parametric([1e6], [1e10])
    ctx.set_parametric(None)                                  # off again: the plain run
    ref = gpu_for(W.paper_sim1(T=0.1e-9))
    ctx.run(0.1e-9)
    ref.run(0.1e-9)
    assert np.array_equal(ctx.get_a(), ref.get_a()) and np.array_equal(ctx.get_m(), ref.get_m())
