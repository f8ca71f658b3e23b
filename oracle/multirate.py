"""Two-rate Adams-Bashforth time stepping (FP64 oracle).

Test infrastructure only.  Sec. 1 names local time stepping as an advantage
of DG methods and Sec. 5 calls a multi-rate scheme essential for large
meshes, without giving one; the scheme here is our reading, a two-class
multi-rate Adams-Bashforth method built from eq. (4):

* elements are split into a fast class, stepped with h = dt/2, and a slow
  class, stepped with dt; each class keeps its own history of right-hand
  sides (fast: at every fine time, slow: at every coarse time) and its own
  start-up (Euler, then the two-step formula, then AB3);
* one macro step from t_n:
  1. r = L q(t_n) for every element (both classes are at t_n);
  2. fast elements: one AB step of size h with r and their fine history;
  3. slow elements: the AB step of size dt to t_n + dt, and their state at
     t_n + h from the same history polynomial (dense output: the integral
     over [t_n, t_n + h] of the polynomial through the slow right-hand
     sides, which at the full step is exactly the AB weights);
  4. r = L q at t_n + h, with the fast elements' new state and the slow
     elements' dense-output state, for the fast elements only;
  5. fast elements: the second AB step of size h.
  Both classes are back at a common time t_n + dt.

With every element in one class the macro step is one AB3 step of size dt
(all slow) or two of size dt/2 (all fast), with the same arithmetic as
``AB3Stepper``.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np

from .dg import ab3_coefficients


def history_weights(nhist: int, theta) -> list:
    """Weights w_i with  int_0^theta P(s) ds = sum_i w_i r_i,  P the
    polynomial through (s = -i, r_i), i = 0 .. nhist - 1 (r_0 the newest),
    in units of the step.  Exact rational arithmetic."""
    theta = Fraction(theta)
    nodes = [-i for i in range(nhist)]
    out = []
    for i in range(nhist):
        # Lagrange basis l_i(s) = prod_{j != i} (s - s_j) / (s_i - s_j) as
        # polynomial coefficients (lowest power first), then integrated
        coef = [Fraction(1)]
        denom = Fraction(1)
        for j in range(nhist):
            if j == i:
                continue
            coef = [Fraction(0)] + coef  # times s
            for k in range(len(coef) - 1):
                coef[k] -= nodes[j] * coef[k + 1]
            denom *= nodes[i] - nodes[j]
        integral = sum(c * theta ** (k + 1) / (k + 1) for k, c in enumerate(coef))
        out.append(integral / denom)
    return out


class TwoRateAB3:
    """Two-rate AB stepping over an oracle's right-hand side.

    ``fast`` is a (K,) bool mask of the elements stepped with dt/2.
    """

    def __init__(self, oracle, q0: np.ndarray, fast: np.ndarray, history=None):
        """``history``: optional exact start, ((r(-h), r(-2h)), (r(-dt), r(-2dt)))
        as full (K, ...) arrays; both classes then start with AB3."""
        self.oracle = oracle
        self.q = np.array(q0, dtype=float, copy=True)
        self.fast = np.asarray(fast, dtype=bool)
        if self.fast.shape != (self.q.shape[0],):
            raise ValueError("the class mask needs one entry per element")
        self.slow = ~self.fast
        self.rf = []  # fast history, newest first: r at t - h, t - 2h
        self.rs = []  # slow history, newest first: r at t - dt, t - 2dt
        self.mf = 0   # fine steps taken by the fast class
        self.ms = 0   # coarse steps taken by the slow class
        if history is not None:
            (f1, f2), (s1, s2) = history
            self.rf = [np.asarray(f1)[self.fast], np.asarray(f2)[self.fast]]
            self.rs = [np.asarray(s1)[self.slow], np.asarray(s2)[self.slow]]
            self.mf = self.ms = 2
        self.t = 0.0

    @staticmethod
    def _ab_update(q, step, m, r0, hist):
        """q + step * (a1 r0 + a2 r1 + a3 r2), the arithmetic of AB3Stepper."""
        a1, a2, a3 = ab3_coefficients(m)
        upd = a1 * r0
        if a2 != 0.0:
            upd = upd + a2 * hist[0]
        if a3 != 0.0:
            upd = upd + a3 * hist[1]
        return q + step * upd

    def macro_step(self, nsteps: int, dt: float):
        h = 0.5 * dt
        f, s = self.fast, self.slow
        for _ in range(nsteps):
            # 1. every element at t_n
            r = self.oracle.rhs(self.q)
            q_new = self.q.copy(order="K")
            # 2. fast: first fine step
            q_new[f] = self._ab_update(self.q[f], h, self.mf, r[f], self.rf)
            self.rf = [r[f]] + self.rf[:1]
            self.mf += 1
            # 3. slow: state at t_n + h (dense output) and at t_n + dt
            hist = [r[s]] + self.rs[:2]
            w_half = history_weights(min(self.ms + 1, 3), Fraction(1, 2))
            q_half = self.q[s] + dt * sum(float(w) * ri for w, ri in zip(w_half, hist))
            q_slow = self._ab_update(self.q[s], dt, self.ms, r[s], self.rs)
            self.rs = hist[:2]
            self.ms += 1
            # 4. fast right-hand side at t_n + h
            q_mid = q_new.copy(order="K")
            q_mid[s] = q_half
            r2 = self.oracle.rhs(q_mid)
            # 5. fast: second fine step
            q_new[f] = self._ab_update(q_new[f], h, self.mf, r2[f], self.rf)
            self.rf = [r2[f]] + self.rf[:1]
            self.mf += 1
            q_new[s] = q_slow
            self.q = q_new
            self.t += dt
        return self.q
