"""Differentiable spectral objectives of a recorded cavity trace.

The trace output of `mmcav.recorded_run(..., with_trace=True)` carries a
gradient through the library's discrete adjoint (mm_adjoint_trace); the
functions here turn it into the quantities a mode-profile design optimises
(Sec. IV F): the frequency and the linewidth of one polariton branch.  A
branch is a complex rate s = -i w - Gamma of the trace, x(t_k) ~ sum_j c_j
e^{s_j t_k}, found by least-squares linear prediction (Prony's method): the
prediction coefficients solve x[k] = sum_{q=1..p} b_q x[k - q] in the least
squares sense (by a QR factorisation), and the rates are log(z)/dt for the roots
z of z^p - sum_q b_q z^{p-q} (the eigenvalues of the companion matrix).
Every step is a torch operation, so autograd differentiates the branch with
respect to the trace; choosing which root is the branch is a discrete step
and is not differentiated.  This is host-side arithmetic of the loss, not of
the stepper.
"""
import torch


def linear_prediction_rates(x, dt, order):
    """Complex rates (order,) shared by the channels of x, a complex tensor
    of shape (n,) or (channels, n) sampled at spacing dt."""
    if x.dim() == 1:
        x = x.unsqueeze(0)
    rows, rhs = [], []
    for ch in x:
        n = ch.shape[0]
        # row k: x[k-1], x[k-2], ..., x[k-order]
        idx = torch.arange(order, n).unsqueeze(1) - torch.arange(1, order + 1).unsqueeze(0)
        rows.append(ch[idx])
        rhs.append(ch[order:])
    A = torch.cat(rows)
    b = torch.cat(rhs)
    Q, R = torch.linalg.qr(A)
    coef = torch.linalg.solve_triangular(R, (Q.conj().transpose(0, 1) @ b).unsqueeze(1), upper=True).squeeze(1)
    comp = torch.zeros((order, order), dtype=coef.dtype)
    comp[0] = coef
    if order > 1:
        comp[1:, :-1] = torch.eye(order - 1, dtype=coef.dtype)
    z = torch.linalg.eigvals(comp)
    return torch.log(z) / dt


def branch(rates, omega):
    """The rate whose frequency -Im(s) lies nearest omega [rad/s]."""
    k = int(torch.argmin(torch.abs(-rates.imag.detach() - omega)))
    return rates[k]


def peak_frequency(rate):
    """Angular frequency w of a rate s = -i w - Gamma."""
    return -rate.imag


def linewidth(rate):
    """Decay rate Gamma (half width of the line, rad/s) of s = -i w - Gamma."""
    return -rate.real


def trace_complex(trace):
    """The trace output of recorded_run ([samples][modes][2], re/im) as a
    complex tensor [modes][samples]."""
    return torch.complex(trace[..., 0], trace[..., 1]).transpose(0, 1)
