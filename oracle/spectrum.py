"""Spectral analysis of sampled complex traces.

TEST INFRASTRUCTURE ONLY.  Part of the CPU oracle: only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.

S(f) = |sum_k x(t_k) e^{+2 pi i f t_k}|^2 on a uniform grid, zero-padded by a
factor of 4 (Sec. IV C), no window; the + sign puts signals that go as
e^{-i w t} (the convention of Sec. II A) at positive f.  Peaks are local
maxima refined by a 3-point parabola through log S.
"""
import numpy as np


def spectrum(x, dt, pad=4):
    x = np.asarray(x, complex)
    n = x.size * pad
    X = np.fft.ifft(x, n=n) * n            # sum_k x_k e^{+2 pi i j k / n}
    f = np.fft.fftfreq(n, d=dt)
    order = np.argsort(f)
    return f[order], np.abs(X[order]) ** 2


def peaks(f, S, count=None, fmin=-np.inf, fmax=np.inf, rel_floor=1e-6):
    """Refined local maxima of S in (fmin, fmax), strongest first."""
    logS = np.log(np.maximum(S, 1e-300))
    out = []
    top = S[(f > fmin) & (f < fmax)].max()
    for i in range(1, len(S) - 1):
        if not (fmin < f[i] < fmax):
            continue
        if S[i] > S[i - 1] and S[i] >= S[i + 1] and S[i] > rel_floor * top:
            y0, y1, y2 = logS[i - 1], logS[i], logS[i + 1]
            den = y0 - 2 * y1 + y2
            d = 0.5 * (y0 - y2) / den if den != 0 else 0.0
            out.append((f[i] + d * (f[1] - f[0]), S[i]))
    out.sort(key=lambda p: -p[1])
    if count is not None:
        out = out[:count]
    return [p[0] for p in out]


def prony(x, dt, count):
    """Complex rates s_j of x(t_k) ~ sum_j c_j e^{s_j t_k}, by least-squares
    linear prediction of order `count` (uniform samples, spacing dt).
    Returns s_j = -i w_j - decay_j sorted by frequency w_j = -Im s_j.
    x may be (n,) or (channels, n): channels share the same rates."""
    x = np.atleast_2d(np.asarray(x, complex))
    rows, rhs = [], []
    for ch in x:
        n = ch.size
        for k in range(count, n):
            rows.append(ch[k - count:k][::-1])
            rhs.append(ch[k])
    A = np.array(rows)
    b = np.array(rhs)
    coef = np.linalg.lstsq(A, b, rcond=None)[0]
    z = np.roots(np.concatenate([[1.0], -coef]))
    s = np.log(z) / dt
    return s[np.argsort(-s.imag)]


def prony_torch(x, dt, count):
    """prony() written with torch operations, so that autograd
    differentiates the rates with respect to the samples: the prediction
    coefficients by the pseudo-inverse of the linear-prediction matrix, the
    rates from the eigenvalues of the companion matrix.  x: complex tensor
    (n,) or (channels, n)."""
    import torch
    if x.dim() == 1:
        x = x.unsqueeze(0)
    rows, rhs = [], []
    for ch in x:
        for k in range(count, ch.shape[0]):
            rows.append(torch.flip(ch[k - count:k], dims=(0,)))
            rhs.append(ch[k])
    A = torch.stack(rows)
    b = torch.stack(rhs)
    coef = torch.linalg.pinv(A) @ b
    comp = torch.diag(torch.ones(count - 1, dtype=coef.dtype), -1)
    comp = torch.cat([coef.unsqueeze(0), comp[1:]], dim=0)
    return torch.log(torch.linalg.eigvals(comp)) / dt
