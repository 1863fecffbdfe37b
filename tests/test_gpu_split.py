"""The operator-split co-simulation scheme (Sec. III B) on the HIP path,
against the oracle's split scheme and against the joint stepper."""
import math

import numpy as np
import pytest

from paper_2603_03706_amd import workloads as W
from tests.helpers import oracle_for, gpu_for, run_oracle, m_err, rel_a_err, variant

pytestmark = pytest.mark.gpu

TWO_PI = 2 * math.pi


def test_split_parity_sim1():
    """Sim 1 of Table I with its Gaussian pulse, split scheme at 1 ps for
    1 ns, element by element against the oracle's split scheme."""
    inst = variant(W.paper_sim1(T=1e-9), method="split")
    st, ctx = oracle_for(inst), gpu_for(inst)
    st.set_sampling(10e-12, 1000)
    ctx.set_sampling(10e-12, 1000)
    run_oracle(st, inst.T)
    ctx.run(inst.T)
    t_o, a_o, mm_o = st.trace_arrays()
    t, a, mm = ctx.get_trace(1000)
    assert len(t) == len(t_o) == 101
    assert rel_a_err(a, a_o.numpy()) <= 1e-5 and rel_a_err(mm, mm_o.numpy()) <= 1e-5
    assert m_err(ctx.get_m(), st) <= 1e-5


def test_split_equals_joint_when_uncoupled():
    """g = 0 (pulse on, m tilted): the split and joint runs agree bit for bit
    on the device, as they do in the oracle."""
    base = variant(W.paper_sim1(g=0.0, T=0.2e-9), m0=W.tilted((8, 8, 1), 3.0, 0.2))
    outs = []
    for method in ("rk4", "split"):
        ctx = gpu_for(variant(base, method=method))
        ctx.set_a(np.array([0.01 + 0j]))
        ctx.run(base.T)
        outs.append((ctx.get_m(), ctx.get_a()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_split_error_first_order():
    """Resonant Rabi exchange on the 8x8x1 film (a(0) = 0.01, no pulse, 1 ns):
    against a quarter-step joint run, the split scheme's error halves with
    dt and, at 1 ps, is far above the joint stepper's."""
    base = variant(W.paper_sim1(T=1e-9), drive_amp=None, a0=np.array([0.01 + 0j]))

    def trace(method, dt):
        ctx = gpu_for(variant(base, method=method, dt0=dt))
        ctx.set_sampling(20e-12, 1000)
        ctx.run(base.T)
        return ctx.get_trace(1000)[1][:, 0]

    ref = trace("rk4", 0.25e-12)
    es = [np.abs(trace("split", dt) - ref).max() for dt in (1e-12, 0.5e-12)]
    ej = np.abs(trace("rk4", 1e-12) - ref).max()
    assert 1.7 < es[0] / es[1] < 2.4
    assert es[0] > 30 * ej


def test_split_has_no_adjoint():
    from paper_2603_03706_amd import mmcav
    ctx = gpu_for(variant(W.paper_sim1(T=0.1e-9), method="split"))
    with pytest.raises(mmcav.MMError) as e:
        ctx.run_record(10e-12, 4)
    assert e.value.status == mmcav.MM_ERR_STATE
