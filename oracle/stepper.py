"""Time integration of the joint state (m, a), plain FP64.

TEST INFRASTRUCTURE ONLY.  Part of the CPU oracle: only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.

The magnetisation and the cavity amplitudes advance together inside one
Runge-Kutta step (Sec. III A: the cavity ODEs are integrated in the same
adaptive RK45 step as the LLG equation), with no operator splitting.

  * fixed step: classical RK4;
  * operator-split (the co-simulation scheme of Sec. III B, kept as an
    accuracy baseline): per step, one RK4 step of the cavity ODE with m^-
    held at its step-start value, then one RK4 step of the LLG with the
    feedback field of the new amplitudes held over the whole step;
  * adaptive: Dormand-Prince 5(4) (Dormand & Prince, J. Comput. Appl. Math. 6,
    19 (1980)), first-same-as-last, advancing with the 5th-order weights.
    Error  eps = max(|E_m| over magnetic cells, components and sublattices,
    |Re E_a|, |Im E_a| over modes) / tol, E = dt sum_j (b_j - bhat_j) k_j,
    NaN counts as +inf.  Accept iff eps <= 1.  New step
    dt * min(fmax, max(0.2, 0.9 eps^{-1/5})), fmax = 5, or 1 on the step that
    follows a rejection.  The stage-7 point is the normalised candidate.
  * after every accepted step m <- m/|m| on magnetic cells.
  * the last step is clipped so that the run ends exactly on t0 + T.
  * stage s of a step from t with size h is evaluated at t + c_s h (RK4:
    c = 0, 1/2, 1/2, 1; DP45: the c column of the tableau), which matters
    only for the time-dependent cavity terms (drive, parametric pump).
  * an adaptive run keeps the sizes of its accepted steps (`accepted_h`,
    negative for a step clipped onto the end time); `replay` applies the
    5th-order steps of such a sequence, every one accepted.  Rejected
    attempts leave no trace in the state, so the replay reaches the adaptive
    run's states; it is the map the adjoint of an adaptive run
    differentiates (the step sizes held fixed).

Status values: 0 ok, -5 step size below dt_min, -6 non-finite state.
"""
import math

import torch

OK, DT_UNDERFLOW, NONFINITE = 0, -5, -6

# Dormand-Prince 5(4) tableau
DP_C = [0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0]
DP_A = [
    [],
    [1 / 5],
    [3 / 40, 9 / 40],
    [44 / 45, -56 / 15, 32 / 9],
    [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
    [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
    [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84],
]
DP_B = [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0]
DP_BHAT = [5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40]
DP_E = [b - bh for b, bh in zip(DP_B, DP_BHAT)]


def hermite(theta, h, y0, f0, y1, f1):
    """Cubic Hermite interpolant on [t, t+h] at t + theta h."""
    t2 = theta * theta
    t3 = t2 * theta
    h00 = 2 * t3 - 3 * t2 + 1
    h10 = t3 - 2 * t2 + theta
    h01 = -2 * t3 + 3 * t2
    h11 = t3 - t2
    return h00 * y0 + h10 * h * f0 + h01 * y1 + h11 * h * f1


class Stepper:
    def __init__(self, model, m0, a0, method="rk4", dt0=1e-12, dt_min=1e-18, dt_max=math.inf):
        self.model = model
        self.m = model.normalize(torch.as_tensor(m0, dtype=torch.float64) * model.G)
        self.a = torch.as_tensor(a0, dtype=torch.complex128).clone()
        self.method = method
        self.dt = float(dt0)
        self.dt0 = float(dt0)
        self.dt_min = float(dt_min)
        self.dt_max = float(dt_max)
        self.t = 0.0
        self.accepted = 0
        self.rejected = 0
        self.last_rejected = False
        self.fsal = None            # (k1, ka1, m^-_1, dm^-/dt_1) at the current state
        self.trace = None
        self.accepted_h = []        # sizes of the accepted adaptive steps (negative: clipped)

    # ----------------------------------------------------------- observables
    def m_minus_rate(self, k):
        """d m^-_n / dt from the torque k (same weighting as m^-_n)."""
        return self.model.m_minus(k)

    def set_sampling(self, dt_sample, max_samples):
        self.trace = {"dt": float(dt_sample), "max": int(max_samples), "t0": None,
                      "t": [], "a": [], "mm": [], "steps": 0}

    def _record(self, t, a, mm):
        tr = self.trace
        if len(tr["t"]) < tr["max"]:
            tr["t"].append(t)
            tr["a"].append(a.clone())
            tr["mm"].append(mm.clone())

    def trace_arrays(self):
        tr = self.trace
        if not tr["t"]:
            return torch.zeros(0, dtype=torch.float64), None, None
        return (torch.tensor(tr["t"], dtype=torch.float64), torch.stack(tr["a"]), torch.stack(tr["mm"]))

    # ----------------------------------------------------------------- steps
    def _rk4_step(self, h):
        M = self.model
        y, a = self.m, self.a
        t = self.t
        k1, ka1, _ = M.rhs(y, a, t)
        k2, ka2, _ = M.rhs(y + 0.5 * h * k1, a + 0.5 * h * ka1, t + 0.5 * h)
        k3, ka3, _ = M.rhs(y + 0.5 * h * k2, a + 0.5 * h * ka2, t + 0.5 * h)
        k4, ka4, _ = M.rhs(y + h * k3, a + h * ka3, t + h)
        y_new = M.normalize(y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4))
        a_new = a + h / 6.0 * (ka1 + 2 * ka2 + 2 * ka3 + ka4)
        return y_new, a_new

    def _split_step(self, h):
        M = self.model
        y, a, t = self.m, self.a, self.t
        mm = M.m_minus(y)
        k1 = M.cavity_rhs(a, mm, t)
        k2 = M.cavity_rhs(a + 0.5 * h * k1, mm, t + 0.5 * h)
        k3 = M.cavity_rhs(a + 0.5 * h * k2, mm, t + 0.5 * h)
        k4 = M.cavity_rhs(a + h * k3, mm, t + h)
        a_new = a + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

        def f(m):
            return M.torque(m, M.field(m, a_new))
        q1 = f(y)
        q2 = f(y + 0.5 * h * q1)
        q3 = f(y + 0.5 * h * q2)
        q4 = f(y + h * q3)
        return M.normalize(y + h / 6.0 * (q1 + 2 * q2 + 2 * q3 + q4)), a_new

    def _dp_first(self):
        M = self.model
        k1, ka1, mm1 = M.rhs(self.m, self.a, self.t)
        self.fsal = (k1, ka1, mm1, self.m_minus_rate(k1))

    def _dp_step(self, h):
        """One attempted DP45 step; returns (y_cand, a_cand, eps_num, stage-7 data)."""
        M = self.model
        y, a = self.m, self.a
        ks = [self.fsal[0]]
        kas = [self.fsal[1]]
        for s in range(1, 7):
            ys = y.clone()
            as_ = a.clone()
            for j, c in enumerate(DP_A[s]):
                if c != 0.0:
                    ys = ys + h * c * ks[j]
                    as_ = as_ + h * c * kas[j]
            if s == 6:
                ys = M.normalize(ys)
                y_cand, a_cand = ys, as_
            k, ka, mm = M.rhs(ys, as_, self.t + DP_C[s] * h)
            ks.append(k)
            kas.append(ka)
        Em = torch.zeros_like(y)
        Ea = torch.zeros_like(a)
        for j, e in enumerate(DP_E):
            if e != 0.0:
                Em = Em + e * ks[j]
                Ea = Ea + e * kas[j]
        Em = (h * Em) * M.G
        Ea = h * Ea
        err = max(float(Em.abs().max()) if Em.numel() else 0.0,
                  float(torch.cat([Ea.real.abs(), Ea.imag.abs()]).max()) if Ea.numel() else 0.0)
        if not math.isfinite(err) or not bool(torch.isfinite(Em).all()) or not bool(torch.isfinite(Ea).all()):
            err = math.inf
        stage7 = (ks[6], kas[6], mm, self.m_minus_rate(ks[6]))
        return y_cand, a_cand, err, stage7

    # ------------------------------------------------------------------- run
    def run(self, T, tol=0.0):
        """Advance by T seconds; tol > 0 selects the adaptive method."""
        t_end = self.t + float(T)
        status = OK
        if self.trace is not None and self.trace["t0"] is None:
            self.trace["t0"] = self.t
            self._record(self.t, self.a, self.model.m_minus(self.m))
        adaptive = self.method == "dp45"
        if adaptive and self.fsal is None:
            self._dp_first()
        while self.t < t_end:
            remaining = t_end - self.t
            h = self.dt if adaptive else self.dt0
            clipped = h * (1.0 + 1e-9) >= remaining
            if clipped:
                h = remaining
            if not adaptive:
                y_new, a_new = self._split_step(h) if self.method == "split" else self._rk4_step(h)
                if not (bool(torch.isfinite(y_new).all()) and bool(torch.isfinite(a_new.real).all())
                        and bool(torch.isfinite(a_new.imag).all())):
                    status = NONFINITE
                    break
                self.m, self.a = y_new, a_new
                self.t = t_end if clipped else self.t + h
                self.accepted += 1
                if self.trace is not None:
                    self.trace["steps"] += 1
                    stride = max(1, int(round(self.trace["dt"] / self.dt0)))
                    if self.trace["steps"] % stride == 0:
                        self._record(self.t, self.a, self.model.m_minus(self.m))
                continue
            y_c, a_c, err, st7 = self._dp_step(h)
            eps = err / tol
            if eps <= 1.0:
                if self.trace is not None:
                    self._sample_interval(h, self.fsal, a_c, st7)
                self.m, self.a = y_c, a_c
                self.t = t_end if clipped else self.t + h
                self.fsal = st7
                self.accepted += 1
                self.accepted_h.append(-h if clipped else h)
                fmax = 1.0 if self.last_rejected else 5.0
                fac = 5.0 if eps == 0.0 else 0.9 * eps ** (-0.2)
                fac = min(fmax, max(0.2, fac))
                self.last_rejected = False
            else:
                self.rejected += 1
                fac = 0.2 if not math.isfinite(eps) else max(0.2, 0.9 * eps ** (-0.2))
                fac = min(1.0, fac)
                self.last_rejected = True
            self.dt = min(self.dt_max, h * fac)
            if self.t < t_end and self.dt < self.dt_min:
                status = NONFINITE if not math.isfinite(eps) else DT_UNDERFLOW
                break
        return status

    def replay(self, steps, t_end=None):
        """Apply accepted Dormand-Prince steps of the given sizes (negative:
        a step that lands on t_end, the end time of the recorded run): the
        stages of the tableau from the current state, the 5th-order
        combination, the renormalised candidate.  Returns the number of
        steps taken."""
        M = self.model
        for hs in steps:
            h = abs(hs)
            y, a, t = self.m, self.a, self.t
            ks, kas = [], []
            for s in range(6):
                ys, as_ = y, a
                for j, c in enumerate(DP_A[s]):
                    if c != 0.0:
                        ys = ys + h * c * ks[j]
                        as_ = as_ + h * c * kas[j]
                k, ka, _ = M.rhs(ys, as_, t + DP_C[s] * h)
                ks.append(k)
                kas.append(ka)
            yn, an = y, a
            for j, b in enumerate(DP_B[:6]):
                if b != 0.0:
                    yn = yn + h * b * ks[j]
                    an = an + h * b * kas[j]
            self.m, self.a = M.normalize(yn), an
            self.t = t_end if (hs < 0 and t_end is not None) else t + h
            self.accepted += 1
        self.fsal = None
        return len(steps)

    def _sample_interval(self, h, start, a1, end):
        tr = self.trace
        t0 = self.t
        k_next = len(tr["t"])
        while k_next < tr["max"]:
            tk = tr["t0"] + k_next * tr["dt"]
            if tk > t0 + h * (1.0 + 1e-12):
                break
            if tk > t0:
                th = (tk - t0) / h
                a_s = hermite(th, h, self.a, start[1], a1, end[1])
                m_s = hermite(th, h, start[2], start[3], end[2], end[3])
                tr["t"].append(tk)
                tr["a"].append(a_s)
                tr["mm"].append(m_s)
            k_next = len(tr["t"])
            if tk <= t0:
                break
