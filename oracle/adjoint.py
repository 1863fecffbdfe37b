"""Gradients of a scalar loss of the final state, by reverse-mode automatic
differentiation of the FP64 oracle (the exact adjoint of the oracle's
discrete map, RK4 steps and renormalisation included).

TEST INFRASTRUCTURE ONLY.  Part of the CPU oracle: only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.
"""
import numpy as np
import torch

from .model import Model, Problem
from .stepper import Stepper


def run_with_grad(problem: Problem, m0, a0, dt, T, loss_fn, method="rk4", trace_loss=None, steps=None):
    """Return (loss, grads) where grads has d loss / d u (N, nz, ny, nx),
    d g (N,), d alpha, d B0 (3,), d a0 (N complex, as d/dRe + i d/dIm) and
    d m0 (S, 3, nz, ny, nx, taken with respect to the normalised state).
    With trace_loss, the loss also has trace_loss(A) for A the complex
    amplitudes at the start and every step end, shape (steps + 1, N).
    With steps (a sequence of accepted Dormand-Prince step sizes, negative
    for one clipped onto T), the run is that replayed sequence instead of a
    fixed-step run: the adjoint of an adaptive run with its steps held."""
    N = len(problem.omega)
    nx, ny, nz = problem.grid
    u0 = np.ones((N, nz, ny, nx)) if problem.u is None else np.asarray(problem.u, float).reshape(N, nz, ny, nx)
    leaves = {
        "u": torch.tensor(u0, dtype=torch.float64, requires_grad=True),
        "g": torch.tensor(np.asarray(problem.g, float), requires_grad=True),
        "alpha": torch.tensor(float(problem.alpha), dtype=torch.float64, requires_grad=True),
        "B0": torch.tensor(np.asarray(problem.B0, float), requires_grad=True),
    }
    M = Model(problem, leaves)
    ar = torch.tensor(np.real(np.asarray(a0, complex)), requires_grad=True)
    ai = torch.tensor(np.imag(np.asarray(a0, complex)), requires_grad=True)
    st = Stepper(M, np.asarray(m0, float), np.zeros(N, complex), method=method, dt0=dt)
    m_start = st.m.detach().clone().requires_grad_(True)
    st.m = m_start
    st.a = torch.complex(ar, ai)
    if trace_loss is not None:
        st.set_sampling(dt, 1 << 30)
    if steps is not None:
        st.replay(steps, t_end=T)
        status = 0
    else:
        status = st.run(T)
    loss = loss_fn(st.m, st.a)
    if trace_loss is not None:
        loss = loss + trace_loss(torch.stack(st.trace["a"]))
    loss.backward()
    grads = {
        "u": leaves["u"].grad.numpy(),
        "g": leaves["g"].grad.numpy(),
        "alpha": float(leaves["alpha"].grad),
        "B0": leaves["B0"].grad.numpy(),
        "a0": ar.grad.numpy() + 1j * ai.grad.numpy(),
        "m0": m_start.grad.numpy(),
    }
    return float(loss.detach()), grads, status


def run_loss(problem: Problem, m0, a0, dt, T, loss_fn, method="rk4", leaves=None, steps=None):
    """Loss only (no gradient), optionally with perturbed parameter leaves
    (and, with steps, of the replayed Dormand-Prince sequence)."""
    M = Model(problem, leaves)
    st = Stepper(M, np.asarray(m0, float), np.asarray(a0, complex), method=method, dt0=dt)
    with torch.no_grad():
        if steps is not None:
            st.replay(steps, t_end=T)
        else:
            st.run(T)
        return float(loss_fn(st.m, st.a))
