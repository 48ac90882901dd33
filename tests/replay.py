"""Replay of a registration trajectory through the oracle, one evaluation at a
time (test infrastructure).

A trajectory is the sequence of evaluations a registration made: per pass the
transform T it evaluated, the Welsch parameter nu and the energy E it found.
The replay applies the oracle's un-accelerated map (oracle.eval_map) at every
recorded T and re-runs the control flow of the paper's algorithms on the
oracle's results:

* Algorithm 1 (Sec. 4.3; Fast ICP of Sec. 4.2 is its L2 case): stage start
  at T^(k-1), un-accelerated update T', Anderson mixing of the 4x4 logarithms
  (F^(k) = log T' - log T^(k), Frobenius metric), the energy safeguard that
  reverts to T' when E(T^(k)) >= E(T^(k-1)), the stage test
  ||T^(k) - T'||_F < eps, the iteration cap I_nu and nu <- max(nu/2, nu_min).
* Algorithm 2 (Sec. 5): the Gauss-Newton candidate xi* (eq. GNMapping),
  Anderson mixing in R^6 (Euclidean metric), the line search from xi^(k-1)
  towards xi*^(k) with tau halving (up to l_max trials, lowest energy kept),
  the stage test ||xi*^(k+1) - xi^(k)|| < eps, caps 6 + stage <= 10.

Each step predicts the next evaluation (its transform, nu and the reason for
it) and compares it with the recorded one; the replay then continues from the
recorded transform, so that rounding differences between the recorder and the
oracle do not compound over the trajectory. A decision (safeguard, line
search, stage test) that differs from the recorder's is accepted only at a
near-tie of the compared quantities, and counted.

Rows may also carry the recorder's un-accelerated update (columns 20..35:
T' for point-to-point, xi* in 20..25 for point-to-plane). It is then checked
against the oracle's update at the same transform, and the replay mixes the
recorded updates. Point-to-plane rows also carry the evaluated parameters xi
(26..31): Algorithm 2 iterates in R^6, where an iterate may rotate by more than
pi and log T is then a different point; the oracle's map is applied at xi.

Anderson extrapolation is ill-conditioned when its columns are nearly
parallel: the least-squares coefficients then move far for last-bit changes
of the history, so two correct implementations (different logarithm code,
summation order) can predict iterates further apart than t_tol. An iterate
predicted by mixing is therefore compared within max(t_tol, 20 x spread),
where the spread is the largest change of the predicted transform over four
seeded perturbations of the mixing history by 2^-50 relative (a few units in
the last place, the size of the rounding differences being allowed for).
"""
from __future__ import annotations

import math

import numpy as np

import oracle

# solver positions recorded in the GPU trace (the reason for an evaluation)
SM_INIT, SM_STAGE, SM_ITER, SM_REVERT, SM_LS = 0, 1, 2, 3, 4


class ReplayError(AssertionError):
    pass


class Replay:
    def __init__(self, P, Q, Qn, mode, rows, *, m, eps, nu_min, iter_first, iter_inc, iter_cap,
                 max_total=0, lmax=10, T0=None, e_rtol=1e-10, t_tol=1e-9, tie_rtol=1e-9,
                 has_sm=True):
        self.P, self.Q, self.Qn, self.mode = P, Q, Qn, mode
        self.rows = np.asarray(rows)
        self.m, self.eps, self.nu_min = m, eps, nu_min
        self.iter_first, self.iter_inc, self.iter_cap = iter_first, iter_inc, iter_cap
        self.max_total, self.lmax = max_total, lmax
        self.T0 = np.eye(4) if T0 is None else np.asarray(T0, np.float64).reshape(4, 4)
        self.e_rtol, self.t_tol, self.tie_rtol = e_rtol, t_tol, tie_rtol
        self.has_sm = has_sm
        self.i = 0
        self.checked = 0
        self.ties = 0
        self.max_e = 0.0
        self.max_t = 0.0
        self.max_u = 0.0
        self.max_spread = 0.0
        self.decisions = 0

    # ---------------------------------------------------------------- rows

    def _next(self, T_pred, nu_pred, sm_pred, what, tol=None):
        if self.i >= len(self.rows):
            raise ReplayError(f"trajectory ends before {what} (row {self.i})")
        r = self.rows[self.i]
        T = r[4:20].reshape(4, 4)
        ok_sm = int(r[2]) == sm_pred or (self.i == 0 and sm_pred == SM_STAGE and int(r[2]) == SM_INIT)
        if self.has_sm and not ok_sm:
            raise ReplayError(f"row {self.i}: recorded position {int(r[2])}, replay expects {sm_pred} ({what})")
        if not self.mode_l2() and r[1] != nu_pred:
            raise ReplayError(f"row {self.i}: nu {r[1]!r} vs replay {nu_pred!r}")
        if T_pred is not None:
            dt = float(np.abs(T - T_pred).max())
            self.max_t = max(self.max_t, dt)
            if dt > (self.t_tol if tol is None else max(self.t_tol, tol)):
                raise ReplayError(f"row {self.i}: transform differs from the replay's by {dt:.3e} ({what})")
        self.i += 1
        return r, T.copy()

    def mode_l2(self):
        return self.mode in (oracle.P2P_L2, oracle.P2PL_L2)

    def _eval(self, row, T, nu, xi=None):
        """Oracle map at T: (E, update, flags); the update is T' (4 x 4) for
        point-to-point, xi* (6) for point-to-plane (linearised at the
        parameters xi when given, else at log T), the recorder's own when the
        row carries it (after checking it against the oracle's)."""
        plane = self.mode in (oracle.P2PL_WELSCH, oracle.P2PL_L2)
        if plane and xi is not None:
            E, upd, fl = oracle.eval_map_xi(self.P, self.Q, self.Qn, self.mode, xi, nu)
        else:
            E, Tn, fl = oracle.eval_map(self.P, self.Q, self.Qn, self.mode, T, nu)
            upd = oracle.se3_log(Tn) if plane else Tn
        d = abs(E - row[0]) / max(1.0, abs(E))
        self.max_e = max(self.max_e, d)
        if d > self.e_rtol:
            raise ReplayError(f"row {self.i - 1}: energy {row[0]!r} vs oracle {E!r}")
        if len(row) >= 36:
            rec = row[20:26].copy() if plane else row[20:36].reshape(4, 4).copy()
            du = float(np.abs(rec - upd).max())
            self.max_u = max(self.max_u, du)
            if du > self.t_tol:
                raise ReplayError(f"row {self.i - 1}: update differs from the oracle's by {du:.3e}")
            upd = rec
        self.checked += 1
        return E, upd, fl

    def _decide(self, a, b, recorded, what):
        """a < b as the oracle finds it, reconciled with the recorder's choice."""
        self.decisions += 1
        mine = a < b
        if recorded is None or mine == recorded:
            return mine
        if abs(a - b) <= self.tie_rtol * max(abs(a), abs(b), 1e-300):
            self.ties += 1
            return recorded
        raise ReplayError(f"row {self.i}: {what}: oracle {a!r} < {b!r} is {mine}, recorder chose {recorded}")

    def _peek_sm(self):
        if not self.has_sm or self.i >= len(self.rows):
            return None
        return int(self.rows[self.i][2])

    def _cap(self, stage):
        v = self.iter_first + stage * self.iter_inc
        return min(v, self.iter_cap) if self.iter_cap > 0 else v

    def _done(self):
        if self.i != len(self.rows):
            raise ReplayError(f"replay ended at row {self.i} of {len(self.rows)}")

    # ---------------------------------------------------------------- Algorithm 1

    def _anderson(self, G, F, k, mk, metric, to_T=None):
        """Mixed parameters G^k - sum theta_j dG_j (Sec. 4.1), and the spread of
        to_T(result) under rounding-level perturbations of the history."""
        def mix(Gp, Fp):
            dF = np.array([Fp[k - j + 1] - Fp[k - j] for j in range(1, mk + 1)])
            dG = np.array([Gp[k - j + 1] - Gp[k - j] for j in range(1, mk + 1)])
            th, sing = oracle.anderson_solve(dF, Fp[k], metric)
            return Gp[k] - th @ dG, sing
        x, sing = mix(G, F)
        to_T = to_T or (lambda v: v)
        base = to_T(x)
        spread = 0.0
        rng = np.random.default_rng(k)
        idx = range(k - mk, k + 1)
        for _ in range(4):
            pert = lambda v: v * (1.0 + 2.0 ** -50 * rng.uniform(-1, 1, v.shape)) + \
                2.0 ** -50 * 1e-2 * np.abs(v).max() * rng.uniform(-1, 1, v.shape)
            Gp = dict(G)
            Fp = dict(F)
            for j in idx:
                Gp[j], Fp[j] = pert(G[j]), pert(F[j])
            spread = max(spread, float(np.abs(to_T(mix(Gp, Fp)[0]) - base).max()))
        self.max_spread = max(self.max_spread, spread)
        return x, sing, 20.0 * spread

    def run_alg1(self, nu0):
        L2 = self.mode == oracle.P2P_L2
        m = self.m
        nu = 0.0 if L2 else nu0
        Tkm1 = self.T0.copy()
        k, stage, total = 1, 0, 0
        G, F = {}, {}
        while True:
            Inu = self._cap(stage)
            kstart = k - 1
            Eprev = math.inf
            row, Tkm1 = self._next(Tkm1, nu, SM_STAGE, "stage start")
            E, Tp, fl = self._eval(row, Tkm1, nu)
            if fl & oracle.FLAG_ZERO_WEIGHT:
                return self._done()
            lp, lq = oracle.se3_log(Tp), oracle.se3_log(Tkm1)
            G[k - 1], F[k - 1] = lp, lp - lq
            row, Tk = self._next(Tp, nu, SM_ITER, "first iterate")
            E, Tprop, fl = self._eval(row, Tk, nu)
            stop = False
            while k - kstart <= Inu:
                if self.max_total > 0 and total >= self.max_total:
                    stop = True
                    break
                total += 1
                if m > 0:
                    nxt = self._peek_sm()
                    rec = None if nxt is None else (nxt != SM_REVERT)
                    accept = self._decide(E, Eprev, rec, "safeguard E < E_prev")
                    if not accept:
                        row, Tk = self._next(Tp, nu, SM_REVERT, "safeguard revert")
                        E, Tprop, fl = self._eval(row, Tk, nu)
                Eprev = E
                if fl & oracle.FLAG_ZERO_WEIGHT:
                    return self._done()
                Tp = Tprop
                nxt = self._peek_sm()
                rec = None if nxt is None else (nxt != SM_ITER)
                if nxt is None and self.i >= len(self.rows):
                    rec = True
                if self._decide(float(np.sqrt(((Tk - Tp) ** 2).sum())), self.eps, rec, "stage test"):
                    break
                tol = None
                if m == 0:
                    Tn = Tp
                else:
                    lp, lk = oracle.se3_log(Tp), oracle.se3_log(Tk)
                    G[k], F[k] = lp, lp - lk
                    mk = min(k - kstart, m)
                    xa, _, tol = self._anderson(G, F, k, mk, 0, oracle.se3_exp)
                    Tn = oracle.se3_exp(xa)
                row, Tk = self._next(Tn, nu, SM_ITER, "next iterate", tol)
                E, Tprop, fl = self._eval(row, Tk, nu)
                k += 1
            if stop or L2 or nu == self.nu_min:
                return self._done()
            nu = max(nu / 2.0, self.nu_min)
            k += 1
            stage += 1
            Tkm1 = Tk

    # ---------------------------------------------------------------- Algorithm 2

    def run_alg2(self, nu0):
        L2 = self.mode_l2()
        m = self.m
        nu = 0.0 if L2 else nu0
        xkm1 = oracle.se3_log(self.T0)
        k, stage, total = 1, 0, 0
        G, F = {}, {}

        def ev(xi_pred, sm, what, tol=None):
            row, T = self._next(None if xi_pred is None else oracle.se3_exp(xi_pred), nu, sm, what, tol)
            xi = self._row_xi(row, T, xi_pred, tol)
            E, xs, fl = self._eval(row, T, nu, xi)
            return xi, E, xs, fl

        while True:
            Inu = self._cap(stage)
            kstart = k - 1
            Eprev = math.inf
            xkm1, E, prop, fl = ev(xkm1, SM_STAGE, "stage start")
            if fl & (oracle.FLAG_ZERO_WEIGHT | oracle.FLAG_DEGENERATE):
                return self._done()
            xstar = prop
            G[k - 1], F[k - 1] = xstar, xstar - xkm1
            xk, E, prop, fl = ev(xstar, SM_ITER, "first iterate")
            stop = False
            while k - kstart <= Inu:
                if self.max_total > 0 and total >= self.max_total:
                    stop = True
                    break
                total += 1
                best = (prop, fl)
                nxt = self._peek_sm()
                rec = None if nxt is None else (nxt != SM_LS)
                if self.lmax >= 1 and not self._decide(E, Eprev, rec, "E < E_prev"):
                    tau = 1.0
                    for trial in range(1, self.lmax + 1):
                        xt_pred = xkm1 + tau * (xstar - xkm1)
                        xt, Et, pt, ft = ev(xt_pred, SM_LS, "line-search trial")
                        if Et < E:
                            E, xk, best = Et, xt, (pt, ft)
                        nxt = self._peek_sm()
                        rec = None if (nxt is None or trial == self.lmax) else (nxt != SM_LS)
                        if self._decide(Et, Eprev, rec, "trial E < E_prev"):
                            break
                        tau *= 0.5
                Eprev = E
                if best[1] & (oracle.FLAG_ZERO_WEIGHT | oracle.FLAG_DEGENERATE):
                    return self._done()
                xs_next = best[0]
                if L2:
                    dn = float(np.sqrt(((oracle.se3_exp(xs_next) - oracle.se3_exp(xk)) ** 2).sum()))
                else:
                    dn = float(np.linalg.norm(xs_next - xk))
                nxt = self._peek_sm()
                rec = None if nxt is None else (nxt != SM_ITER)
                if nxt is None and self.i >= len(self.rows):
                    rec = True
                if self._decide(dn, self.eps, rec, "stage test"):
                    break
                G[k], F[k] = xs_next, xs_next - xk
                tol = None
                if m == 0:
                    xn = xs_next
                else:
                    xn, _, tol = self._anderson(G, F, k, min(k - kstart, m), 1, oracle.se3_exp)
                xkm1, xstar = xk, xs_next
                xk, E, prop, fl = ev(xn, SM_ITER, "next iterate", tol)
                k += 1
            if stop or L2 or nu == self.nu_min:
                return self._done()
            nu = max(nu / 2.0, self.nu_min)
            k += 1
            stage += 1
            xkm1 = xk

    def _row_xi(self, row, T, xi_pred, tol):
        """The parameters of a point-to-plane evaluation: the recorded ones
        (columns 26..31) when the row carries them, checked to give the
        recorded transform and to lie on the replay's branch (an iterate that
        has rotated by more than pi is not log T), else log T."""
        if len(row) < 36:
            return oracle.se3_log(T)
        xi = row[26:32].copy()
        de = float(np.abs(oracle.se3_exp(xi) - T).max())
        if de > 1e-12:
            raise ReplayError(f"row {self.i - 1}: exp of the recorded parameters is {de:.3e} off its transform")
        if xi_pred is not None:
            dx = float(np.abs(xi - xi_pred).max())
            if dx > max(1e-6, 10.0 * (tol or 0.0)):
                raise ReplayError(f"row {self.i - 1}: parameters differ from the replay's by {dx:.3e}")
        return xi

    def summary(self):
        return (f"{self.checked} evaluations replayed, {self.decisions} decisions ({self.ties} near-ties), "
                f"max energy diff {self.max_e:.2e} rel, max update diff {self.max_u:.2e}, "
                f"max transform diff {self.max_t:.2e} (largest mixing spread {self.max_spread:.2e})")


def initial_nu(P, Q, Qn, mode, T0=None):
    """nu_max = 3 x median of the initial residuals (Sec. 4.3: distances;
    Sec. 5: absolute point-to-plane distances), medians of rank n/2, from an
    independent numpy evaluation of the residuals at T0 with the oracle's
    closest points."""
    T0 = np.eye(4) if T0 is None else np.asarray(T0, np.float64).reshape(4, 4)
    idx, _ = oracle.nn_query(P, Q, T0)
    x = np.asarray(P, np.float64) @ T0[:3, :3].T + T0[:3, 3]
    dq = x - np.asarray(Q, np.float64)[idx]
    if mode in (oracle.P2PL_WELSCH,):
        r = np.abs((dq * np.asarray(Qn, np.float64)[idx]).sum(1))
        return 3.0 * np.sort(r)[len(r) // 2]
    r = (dq ** 2).sum(1)
    return 3.0 * math.sqrt(np.sort(r)[len(r) // 2])
