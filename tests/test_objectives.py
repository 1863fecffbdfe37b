"""The differentiable spectral objectives (host-side torch arithmetic of a
loss on the recorded trace) on synthetic sums of exponentials: exact rates,
a gradient that matches central differences, and agreement with the
oracle's own linear-prediction fits (numpy and torch)."""
import math

import numpy as np
import torch

from oracle.spectrum import prony, prony_torch
from paper_2603_03706_amd import objectives as O

TWO_PI = 2 * math.pi


def _signal(n=400, dt=10e-12, c=(0.3, 0.2 - 0.1j, 0.01)):
    t = np.arange(n) * dt
    return (c[0] * np.exp((-1j * TWO_PI * 4.95e9 - 3e6) * t) + c[1] * np.exp((-1j * TWO_PI * 5.05e9 - 5e6) * t)
            + c[2] * np.exp((1j * TWO_PI * 5.0e9 - 2e6) * t))


def test_rates_of_a_sum_of_exponentials():
    x = _signal()
    s = O.linear_prediction_rates(torch.tensor(x), 10e-12, 3).numpy()
    want = np.array([-1j * TWO_PI * 4.95e9 - 3e6, -1j * TWO_PI * 5.05e9 - 5e6, 1j * TWO_PI * 5.0e9 - 2e6])
    for w in want:
        assert np.abs(s - w).min() < 1.0
    assert np.abs(np.sort_complex(s) - np.sort_complex(prony(x, 10e-12, 3))).max() < 10.0
    assert np.abs(np.sort_complex(s) - np.sort_complex(prony_torch(torch.tensor(x), 10e-12, 3).numpy())).max() < 10.0
    # two channels sharing the rates
    x2 = np.stack([x, _signal(c=(0.1j, 0.7, 0.05))])
    s2 = O.linear_prediction_rates(torch.tensor(x2), 10e-12, 3).numpy()
    assert np.abs(np.sort_complex(s2) - np.sort_complex(s)).max() < 10.0


def test_branch_frequency_and_linewidth_gradients():
    x = _signal()
    xt = torch.tensor(x, requires_grad=True)
    for fn in (O.peak_frequency, O.linewidth):
        xt.grad = None
        L = fn(O.branch(O.linear_prediction_rates(xt, 10e-12, 3), TWO_PI * 5.05e9))
        L.backward()
        d = np.random.default_rng(3).normal(size=x.size) + 1j * np.random.default_rng(4).normal(size=x.size)
        f = lambda v: float(fn(O.branch(O.linear_prediction_rates(torch.tensor(v), 10e-12, 3), TWO_PI * 5.05e9)))
        h = 1e-8
        fd = (f(x + h * d) - f(x - h * d)) / (2 * h)
        ad = float(np.real(np.vdot(xt.grad.numpy(), d)))
        assert abs(fd - ad) <= 1e-4 * abs(fd), (fn.__name__, fd, ad)
    assert abs(float(O.peak_frequency(torch.tensor(-1j * 3.0 - 2.0))) - 3.0) == 0.0
    assert abs(float(O.linewidth(torch.tensor(-1j * 3.0 - 2.0))) - 2.0) == 0.0
