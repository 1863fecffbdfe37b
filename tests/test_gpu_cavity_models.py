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
        mmcav._check(ctx._lib.mm_set_cavity_model(ctx.h, 2, None, None))
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
