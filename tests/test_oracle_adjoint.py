"""The oracle's gradient (autograd of the FP64 discrete map) against central
finite differences in FP64 and a Taylor test: the pin for the adjoint."""
import math

import numpy as np
import pytest
import torch

from oracle.adjoint import run_with_grad, run_loss
from oracle.model import Problem
from paper_2603_03706_amd import workloads as W


def small_film():
    inst = W.multimode_film(6, 5, 2)
    inst.method, inst.dt0 = "rk4", 0.5e-12
    rng = np.random.default_rng(12)
    m0 = inst.m0.astype(np.float64).copy()
    m0[0, 0] += 0.05 * rng.normal(size=m0.shape[2:])
    m0[0, 1] += 0.05 * rng.normal(size=m0.shape[2:])
    kw = inst.oracle_kwargs()
    kw["alpha"] = 0.01
    return Problem(**kw), m0, np.array([1.0, 0.2j, 0.0, 0.1])


def loss_mode2(m, a):
    return (a[1].real ** 2 + a[1].imag ** 2) * 1e4


def test_oracle_gradient_matches_central_differences():
    prob, m0, a0 = small_film()
    dt, T = 0.5e-12, 15e-12
    L, g, status = run_with_grad(prob, m0, a0, dt, T, loss_mode2)
    assert status == 0 and L > 0
    base = {"u": torch.tensor(np.asarray(prob.u, float)), "g": torch.tensor(np.asarray(prob.g, float)),
            "alpha": torch.tensor(prob.alpha, dtype=torch.float64), "B0": torch.tensor(np.asarray(prob.B0, float))}
    rng = np.random.default_rng(5)
    for _ in range(4):
        d = {"u": rng.normal(size=base["u"].shape), "g": rng.normal(size=4) * base["g"].numpy(),
             "alpha": rng.normal() * prob.alpha, "B0": rng.normal(size=3) * 0.01}
        ad = (np.sum(g["u"] * d["u"]) + np.dot(g["g"], d["g"]) + g["alpha"] * d["alpha"] + np.dot(g["B0"], d["B0"]))
        vals = {}
        for sgn in (+1, -1):
            h = 1e-4 * sgn
            lv = {k: base[k] + h * torch.as_tensor(d[k], dtype=torch.float64) for k in base}
            vals[sgn] = run_loss(prob, m0, a0, dt, T, loss_mode2, leaves=lv)
        fd = (vals[1] - vals[-1]) / 2e-4
        assert abs(fd - ad) <= 1e-5 * max(abs(fd), 1e-12 * L), (fd, ad)


def test_oracle_gradient_taylor_remainder():
    """|L(p + h d) - L(p) - h <grad, d>| falls as h^2."""
    prob, m0, a0 = small_film()
    dt, T = 0.5e-12, 10e-12
    L, g, _ = run_with_grad(prob, m0, a0, dt, T, loss_mode2)
    rng = np.random.default_rng(9)
    du = rng.normal(size=np.asarray(prob.u).shape)
    ad = np.sum(g["u"] * du)
    res = []
    for h in (1e-1, 5e-2, 2.5e-2):
        lv = {"u": torch.tensor(np.asarray(prob.u, float) + h * du)}
        res.append(abs(run_loss(prob, m0, a0, dt, T, loss_mode2, leaves=lv) - L - h * ad))
    assert res[1] / res[0] == pytest.approx(0.25, rel=0.15)
    assert res[2] / res[1] == pytest.approx(0.25, rel=0.15)


def test_oracle_gradient_with_geometry_mask():
    """Non-magnetic cells (m = 0) keep the reverse pass finite, and the
    gradient still matches central differences."""
    geo = np.ones((2, 4, 5), bool)
    geo[0, 1, 2] = False
    geo[1, 3, :2] = False
    inst = W.multimode_film(5, 4, 2)
    kw = inst.oracle_kwargs()
    kw.update(geometry=geo, alpha=0.01)
    prob = Problem(**kw)
    rng = np.random.default_rng(4)
    m0 = inst.m0.astype(np.float64).copy()
    m0[0, 0] += 0.1 * rng.normal(size=m0.shape[2:])
    m0 = m0 * geo
    m0[0, 2] += (~geo)
    dt, T = 0.5e-12, 5e-12
    L, g, _ = run_with_grad(prob, m0, np.array([1.0, 0.3j, 0.0, 0.0]), dt, T, loss_mode2)
    assert all(np.isfinite(np.asarray(v)).all() for v in g.values())
    du = rng.normal(size=np.asarray(prob.u).shape)
    vals = []
    for h in (1e-4, -1e-4):
        lv = {"u": torch.tensor(np.asarray(prob.u, float) + h * du)}
        vals.append(run_loss(prob, m0, np.array([1.0, 0.3j, 0.0, 0.0]), dt, T, loss_mode2, leaves=lv))
    fd = (vals[0] - vals[1]) / 2e-4
    assert abs(fd - np.sum(g["u"] * du)) <= 1e-6 * abs(fd)


def test_oracle_gradient_with_parametric_pump():
    """With the pump -i lam e^{-2 i wp t} conj(a) on two modes (whose
    Jacobian mixes a and conj(a)), the autograd gradient with respect to the
    initial amplitudes and the couplings matches central differences."""
    prob, m0, a0 = small_film()
    kw = dict(prob.__dict__)
    kw["param_lambda"] = [0, 2e8 * np.exp(0.5j), 0, 1e8 * np.exp(-1.2j)]
    kw["param_wp"] = [0.0, prob.omega[1], 0.0, prob.omega[3] + 1e8]
    prob = Problem(**kw)
    dt, T = 0.5e-12, 10e-12
    L, g, status = run_with_grad(prob, m0, a0, dt, T, loss_mode2)
    assert status == 0 and L > 0
    rng = np.random.default_rng(6)
    da = rng.normal(size=4) + 1j * rng.normal(size=4)
    dg = rng.normal(size=4) * np.asarray(prob.g)
    ad = float(np.real(np.vdot(g["a0"], da))) + float(np.dot(g["g"], dg))
    vals = {}
    for sgn in (+1, -1):
        h = 1e-4 * sgn
        lv = {"g": torch.tensor(np.asarray(prob.g, float) + h * dg)}
        vals[sgn] = run_loss(prob, m0, a0 + h * da, dt, T, loss_mode2, leaves=lv)
    fd = (vals[1] - vals[-1]) / 2e-4
    assert abs(fd - ad) <= 1e-6 * abs(fd), (fd, ad)


def test_dp45_replay_reaches_the_adaptive_states():
    """The replay of an adaptive run's accepted steps (rejected attempts
    leave the state untouched, FSAL is f at the new state) reaches the same
    state bit for bit; its autograd gradient, with the steps held, matches
    central differences of the replayed map."""
    from oracle.model import Model
    from oracle.stepper import Stepper
    prob, m0, a0 = small_film()
    st = Stepper(Model(prob), m0, a0, method="dp45", dt0=2e-12)
    with torch.no_grad():
        assert st.run(12e-12, 1e-7) == 0
    hs = list(st.accepted_h)
    assert st.rejected >= 1 and len(hs) == st.accepted and hs[-1] < 0
    rp = Stepper(Model(prob), m0, a0, method="dp45", dt0=2e-12)
    with torch.no_grad():
        rp.replay(hs, t_end=12e-12)
    assert torch.equal(rp.m, st.m) and torch.equal(rp.a, st.a) and rp.t == st.t
    L, g, _ = run_with_grad(prob, m0, a0, 2e-12, 12e-12, loss_mode2, steps=hs)
    rng = np.random.default_rng(8)
    du = rng.normal(size=np.asarray(prob.u).shape)
    dg = rng.normal(size=4) * np.asarray(prob.g)
    ad = np.sum(g["u"] * du) + np.dot(g["g"], dg)
    vals = []
    for h in (1e-4, -1e-4):
        lv = {"u": torch.tensor(np.asarray(prob.u, float) + h * du), "g": torch.tensor(np.asarray(prob.g, float) + h * dg)}
        vals.append(run_loss(prob, m0, a0, 2e-12, 12e-12, loss_mode2, leaves=lv, steps=hs))
    fd = (vals[0] - vals[1]) / 2e-4
    assert abs(fd - ad) <= 1e-6 * abs(fd), (fd, ad)
