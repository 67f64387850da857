"""CPU oracle of the adaptive propagation (TEST INFRASTRUCTURE ONLY: only tests/, the smoke check
and the benchmark's CPU baseline use it; the GPU library shares no code with it).

arXiv:2405.08737, Sec. "Adaptive Time Stepping" and Sec. "Adaptive History Integration": the
stacked Kadanoff-Baym state of oracle/propagate.py advanced by variable-step, variable-order
Adams methods with fixed-point iteration and error control, on a grid that grows by one point per
accepted step, with the history integrals' order chosen anew at every fixed-point iteration.
Plain PyTorch / numpy on the CPU in FP64.

Step n (from t_{n-1} by h, method order q <= n), for every element:
  predictor   y_pred = y_{n-1} + sum_i beta_i f(t_{n-q+i}): the integral over [t_{n-1}, t_n] of
              the interpolant of f through t_{n-q..n-1} (the paper's predictor polynomial: value
              y_{n-1} at t_{n-1}, derivatives f at the q points before);
  corrector   y_n = y_{n-1} + sum_i alpha_i f(t_{n-q+1+i}): the Adams-Moulton rule of order q,
              the local weights of Eq. weights;
  The blocks born at t_n (kp[n][.] and kp[.][n]) get their right sides at the q_max points
  before t_n reconstructed (Sec. "Implementation": the lesser and greater equations hold on both
  sides of the diagonal): with C^<(j,n), C^>(j,n) the history sums of Eq. KBE2 at row j < n and
  column n (upper limits t_j in I^R, t_n in I^<; Sigma(t_j, t_s) for s > j from row s by
  symmetry), f of kp[.][n] at t_j is i (G^<(t_n,t_j) eps(t_j) - C^<(j,n)^dagger) and f of
  kp[n][.] continued below the diagonal, G^>(t_j,t_n) - G^<(t_j,t_n) = -kp[n][j]^dagger, is
  -i (eps(t_j) (-kp[n][j]^dagger) + C^>(j,n) - C^<(j,n)): the same formulas as above the
  diagonal.  So every block has a history of q points;
  solved by fixed-point iteration from y_pred: y^(m) = base + alpha_last f(y^(m-1)), at most
  `maxcor` corrections, converged when min(1, R_m) d_m C < 0.1 with d_m the WRMS norm of
  y^(m) - y^(m-1), R_m = max(0.3 R_{m-1}, d_m / d_{m-1}) (R_1 = 1) and C the error-estimate
  coefficient below; diverging when d_m > 2 d_{m-1}.  Non-convergence: h <- h / 4, retry.
  Before every evaluation of f the history order is chosen: the test integral of
  u(s) = G^R(t_n,s) Sigma^<(s,t_n) + G^<(t_n,s) Sigma^A(s,t_n) over [t_{n-1}, t_n] with k nodes,
  I^(k), for k = 1..min(K, n+1), and k_opt = the smallest k in 2..min(K, n+1) minimising
  ||I^(k) - I^(k-1)||_F; row n of the history weights is row n-1 plus the local weights of
  interval n on k_opt nodes.
Local error: with the principal error coefficients c_AM = int prod_{i<q}(s - t_{n-i}) ds / q! and
  c_AB = int prod_{1<=i<=q}(s - t_{n-i}) ds / q! over [t_{n-1}, t_n], the error of the corrector is
  estimated as C (y_n - y_pred), C = |c_AM / (c_AB - c_AM)| (Milne's device for a predictor and a
  corrector of the same order).  E = its WRMS norm with weights 1 / (rtol |y_{n-1}| + atol) over the complex entries of the state
  (Eq. wrms_norm, Eq. ewt).  E > 1: the step is rejected, h <- h max(0.2, min(0.9,
  0.9 E^(-1/(q+1)))); after 3 rejections of one step, q <- 1 and h <- h / 4.
After an accepted step the right sides are evaluated once more at y_n (they are the history of
  later steps).  Next step and order: eta_q = 1 / ((6 E)^(1/(q+1)) + 1e-6); once q + 1 steps have
  been taken at order q, also eta_{q-1} = 1 / ((6 E_{q-1})^(1/q) + 1e-6) and eta_{q+1} =
  1 / ((10 E_{q+1})^(1/(q+2)) + 1e-6), where E_{q-1}, E_{q+1} are the WRMS norms of
  int prod_{i<q-1}(s - t_{n-i}) ds f[t_n..t_{n-q+1}] and int prod_{i<=q}(s - t_{n-i}) ds
  f[t_n..t_{n-q-1}] (divided differences of each element's right sides: the derivatives the
  error of orders q -/+ 1 would multiply; q + 1 <= n + 1 points are needed).  The
  largest eta wins (q on ties, then q - 1); below 1.5 nothing changes; otherwise h <- h min(eta, 10).
The last step is shortened to end at t_end.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from oracle import propagate as _pr
import oracle as _orc

CT = torch.complex128


@dataclass
class Controls:
    t_end: float
    rtol: float = 1e-6
    atol: float = 1e-10
    h0: float = 1e-3
    qmax: int = 12
    kmax: int = 10
    maxcor: int = 3
    nt_max: int = 4096


def lagrange_integrals(x, a, b):
    """int_a^b l_j(s) ds for the Lagrange basis of the nodes x (Gauss-Legendre, exact)."""
    x = np.asarray(x, np.float64)
    k = len(x)
    g, gw = np.polynomial.legendre.leggauss(max(1, (k + 2) // 2 + 1))
    s = 0.5 * (b - a) * g + 0.5 * (a + b)
    out = np.zeros(k)
    for j in range(k):
        lj = np.ones_like(s)
        for i in range(k):
            if i != j:
                lj *= (s - x[i]) / (x[j] - x[i])
        out[j] = 0.5 * (b - a) * np.dot(gw, lj)
    return out


def node_poly_integral(x, a, b):
    """int_a^b prod_i (s - x_i) ds (Gauss-Legendre, exact)."""
    x = np.asarray(x, np.float64)
    g, gw = np.polynomial.legendre.leggauss(len(x) // 2 + 2)
    s = 0.5 * (b - a) * g + 0.5 * (a + b)
    p = np.ones_like(s)
    for xi in x:
        p *= s - xi
    return 0.5 * (b - a) * np.dot(gw, p)


def divided_difference(ts, fs):
    """f[ts_0, ..., ts_k] of tensor values fs (Newton's recursion)."""
    d = list(fs)
    for lev in range(1, len(ts)):
        d = [(d[i + 1] - d[i]) / (ts[i + lev] - ts[i]) for i in range(len(d) - 1)]
    return d[0]


class Adaptive:
    """The adaptive propagation of an oracle.propagate.Problem (its h0, pulse, thermal branch,
    initial state; its grid and orders are not used: the grid is built here)."""

    def __init__(self, P: _pr.Problem, ctl: Controls):
        self.P, self.c = P, ctl
        N, ntau = P.N, P.ntau
        self.N, self.ntau = N, ntau
        self.W = {"w": torch.zeros((ctl.nt_max, ctl.nt_max), dtype=torch.float64)}
        if ntau:
            wf, wb, wfull = _orc.tau_weights(P.beta, ntau, P.tau_order)
            self.W["tau"] = tuple(torch.tensor(x) for x in (wf, wb, wfull))
        self.t = [0.0]
        self.S = _pr.State(N, ntau)
        # right-side histories {step j: f}: U_m and R_m from t_{m - qmax} (reconstructed below
        # their birth), D and T_j from t_0
        self.fU, self.fR, self.fD, self.fT = [], [], {}, {}
        self.sig = []     # Sigma rows (ret, les, stv) of the accepted steps
        self.eps = []     # Fock matrices of the accepted steps
        self.trace = []
        self.rejected = 0

    # -- history order ---------------------------------------------------------------------
    def _choose(self, n, force=None):
        """A `choose` hook for propagate.rhs: k_opt from the test integral, then row n of w."""
        tn = np.array(self.t[: n + 1])

        def hook(GL, GR, sig):
            ret, les, _ = sig
            hook.sig = sig
            if n == 0:
                hook.k = 1
                return
            K = min(self.c.kmax, n + 1)
            if force is not None:
                k = force
            else:
                s = np.arange(n - K + 1, n + 1)
                u = torch.stack([GR[n, j] @ (-_pr.H(les[j])) + GL[n, j] @ _pr.H(ret[j])
                                 for j in s])
                I = [None]
                for kk in range(1, K + 1):
                    lam = torch.tensor(lagrange_integrals(tn[n - kk + 1: n + 1], tn[n - 1], tn[n]),
                                       dtype=CT)
                    I.append(torch.einsum("i,iab->ab", lam, u[K - kk:]))
                d = [torch.linalg.norm(I[kk] - I[kk - 1]).item() for kk in range(2, K + 1)]
                k = 2 + int(np.argmin(d))
            lam = torch.tensor(_orc.local_weights(tn, n, k))
            w = self.W["w"]
            w[n] = w[n - 1]
            w[n, n - k + 1: n + 1] += lam
            hook.k = k
        hook.k = None
        hook.sig = None
        return hook

    def _eps(self, j, D, u, A):
        P, N = self.P, self.N
        g = math.exp(-(self.t[j] - P.pulse_t0) ** 2 / (2 * P.pulse_sigma ** 2))
        e = torch.tensor(P.h0, dtype=CT).clone()
        e[0, 0] += float(A) * g
        return e + torch.diag(-1j * u.to(CT) * torch.diagonal(D))

    # -- the blocks born at t_n: right sides below their birth ---------------------------------
    def _upper_sums(self, j, n, KP, mat):
        """(C^<(j,n), C^>(j,n)) for j < n: the history sums of Eq. KBE2 at row j, column n, in the
        lesser and the greater form."""
        N = self.N
        GL, GR, GG = _pr.views(KP, N)
        w = self.W["w"]
        ret = lambda s: self.sig[j][0][s] if s <= j else -_pr.H(self.sig[s][0][j])
        les = lambda s: self.sig[j][1][s] if s <= j else -_pr.H(self.sig[s][1][j])
        # Sigma^R(t_j, t_s) is needed for s <= j only; Sigma^<(t_j,t_s) for s > j from row s:
        # Sigma^<(t_j,t_s) = -Sigma^<(t_s,t_j)^dagger; Sigma^>(t_j,t_s) = -Sigma^>(t_s,t_j)^dagger
        # with Sigma^> = Sigma^R + Sigma^< in the stored rows
        IRl = sum(w[j, s].item() * self.sig[j][0][s] @ GL[s, n] for s in range(j + 1))
        IRg = sum(w[j, s].item() * self.sig[j][0][s] @ GG[s, n] for s in range(j + 1))
        ILl = torch.zeros((N, N), dtype=CT)
        ILg = torch.zeros((N, N), dtype=CT)
        for s in range(n + 1):
            GA = _pr.H(GR[n, s])                          # G^A(t_s, t_n) = G^R(t_n, t_s)^dagger
            if s <= j:
                sl, sg = self.sig[j][1][s], self.sig[j][0][s] + self.sig[j][1][s]
            else:
                sl = -_pr.H(self.sig[s][1][j])
                sg = -_pr.H(self.sig[s][0][j] + self.sig[s][1][j])
            ILl = ILl + w[n, s].item() * sl @ GA
            ILg = ILg + w[n, s].item() * sg @ GA
        Itv = torch.zeros((N, N), dtype=CT)
        if self.ntau:
            wfull = self.W["tau"][2]
            stv = self.sig[j][2]
            J = self.ntau - 1
            tvn = self.S.tv[n]
            Itv = -1j * sum(wfull[l].item() * stv[l] @ _pr.H(tvn[J - l]) for l in range(self.ntau))
        return IRl + ILl + Itv, IRg + ILg + Itv

    def _reconstruct(self, n, mat):
        """Right sides of U_n (kp[.][n]) and R_n (kp[n][.]) at t_j, max(0, n - qmax) <= j < n."""
        KP, _ = self.S.dense(n, self.S.col[n], self.S.row[n], self.S.tv[n])
        for j in range(max(0, n - self.c.qmax), n):
            Cl, Cg = self._upper_sums(j, n, KP, mat)
            e = self.eps[j]
            self.fU[n][j] = 1j * ((-_pr.H(KP[j, n])) @ e - _pr.H(Cl))
            self.fR[n][j] = -1j * (e @ (-_pr.H(KP[n, j])) + Cg - Cl)

    # -- one step ----------------------------------------------------------------------------
    def _elements(self, n):
        """(prev values, f histories) of the elements of step n, in the order U_0..U_{n-1}, D,
        R_0..R_{n-1}, T_0..T_{ntau-1}."""
        S, N = self.S, self.N
        prevU = [S.col[n - 1][m] for m in range(n)]
        prevR = [S.row[n - 1][m] for m in range(n - 1)] + [-1j * torch.eye(N, dtype=CT)]
        prev = prevU + [S.col[n - 1][n - 1]] + prevR + [S.tv[n - 1][j] for j in range(self.ntau)]
        hist = [self.fU[m] for m in range(n)] + [self.fD] + [self.fR[m] for m in range(n)] + \
            [{k: v[j] for k, v in self.fT.items()} for j in range(self.ntau)]
        return prev, hist

    def _wrms(self, vals, wts):
        num = sum(float(((torch.abs(v) * w) ** 2).sum()) for v, w in zip(vals, wts))
        cnt = sum(v.numel() for v in vals)
        return math.sqrt(num / max(cnt, 1))

    def _evaluate(self, n, y, u, A, mat, force_k=None):
        N = self.N
        col_n = torch.stack(y[:n + 1])
        row_n = torch.stack(y[n + 1: 2 * n + 1]) if n else torch.zeros((0, N, N), dtype=CT)
        tv_n = torch.stack(y[2 * n + 1:]) if self.ntau else torch.zeros((0, N, N), dtype=CT)
        hook = self._choose(n, force_k)
        f = _pr.rhs(self.P, self.S, n, col_n, row_n, tv_n, u, A, mat, W=self.W, tn=self.t[n],
                    choose=hook)
        fe = [f[0][m] for m in range(n)] + [f[2]] + [f[1][m] for m in range(n)] + \
            [f[3][j] for j in range(self.ntau)]
        return fe, f, hook, (col_n, row_n, tv_n)

    def _store(self, n, f, hook, col_n, row_n, tv_n, u, A, mat):
        """Accept the values of step n with their right sides f (from _evaluate)."""
        S = self.S
        S.col.append(col_n)
        S.row.append(row_n)
        S.tv.append(tv_n)
        for mm in range(n):
            self.fU[mm][n] = f[0][mm]
            self.fR[mm][n] = f[1][mm]
        self.fU.append({n: f[4]})
        self.fR.append({n: f[5]})
        self.fD[n] = f[2]
        self.fT[n] = f[3]
        self.sig.append(hook.sig)
        self.eps.append(self._eps(n, col_n[n], u, A))
        if n > 0:
            self._reconstruct(n, mat)

    def run(self, U, A, replay=None):
        """Propagate to t_end.  replay: a trace (list of dicts with t, q, m, ks) whose accepted
        steps are repeated exactly (same times, orders, iteration counts and history orders)."""
        P, c, N = self.P, self.c, self.N
        u = torch.full((N,), float(U), dtype=torch.float64)
        A = torch.tensor(float(A), dtype=torch.float64)
        mat = torch.tensor(P.mat, dtype=CT) if self.ntau else torch.zeros((0, N, N), dtype=CT)
        d0, tv0 = _pr.initial_state(P)
        y0 = [d0] + ([tv0[j] for j in range(self.ntau)])
        fe, f, hook, vals = self._evaluate(0, y0, u, A, mat)
        self._store(0, f, hook, *vals, u, A, mat)
        dens = [torch.real(-1j * torch.diagonal(d0))]
        h, q, at_q = c.h0, 1, 0
        n = 1
        while True:
            if replay is not None:
                if n >= len(replay):
                    break
            elif self.t[-1] >= c.t_end * (1 - 1e-14) or n >= c.nt_max:
                break
            prev, hist = self._elements(n)
            ewt = [1.0 / (c.rtol * torch.abs(p) + c.atol) for p in prev]
            nfail = 0
            while True:
                if replay is not None:
                    h, q = replay[n]["t"] - self.t[-1], replay[n]["q"]
                else:
                    h = min(h, c.t_end - self.t[-1])
                    if not h > 1e-13 * max(1.0, self.t[-1]):
                        raise FloatingPointError(f"step size underflow at t = {self.t[-1]}")
                q = min(q, n)
                tn = self.t[-1] + h
                tg = np.array(self.t + [tn])
                self.t.append(tn)
                al = lagrange_integrals(tg[n - q + 1: n + 1], tg[n - 1], tg[n])
                be = lagrange_integrals(tg[n - q: n], tg[n - 1], tg[n])
                base = [p + sum(al[i] * hi[n - q + 1 + i] for i in range(q - 1))
                        for p, hi in zip(prev, hist)]
                pred = [p + sum(be[i] * hi[n - q + i] for i in range(q)) for p, hi in zip(prev, hist)]
                cam = node_poly_integral(tg[n - q + 1: n + 1], tg[n - 1], tg[n]) / math.factorial(q)
                cab = node_poly_integral(tg[n - q: n], tg[n - 1], tg[n]) / math.factorial(q)
                C = abs(cam / (cab - cam))
                y, ks = pred, []
                conv, R, dprev, m = False, 1.0, None, 0
                mmax = replay[n]["m"] if replay is not None else c.maxcor
                while m < mmax:
                    m += 1
                    fk = replay[n]["ks"][m - 1] if replay is not None else None
                    fe, _, hook, _ = self._evaluate(n, y, u, A, mat, fk)
                    ks.append(hook.k)
                    ynew = [b_ + al[q - 1] * f_ for b_, f_ in zip(base, fe)]
                    d = self._wrms([a_ - b_ for a_, b_ in zip(ynew, y)], ewt)
                    y = ynew
                    if replay is not None:
                        continue
                    if not math.isfinite(d):
                        break
                    if m > 1:
                        R = max(0.3 * R, d / dprev) if dprev > 0 else 0.0
                    if min(1.0, R) * d * C < 0.1:
                        conv = True
                        break
                    if m > 1 and d > 2.0 * dprev:
                        break
                    dprev = d
                E = self._wrms([C * (a_ - b_) for a_, b_ in zip(y, pred)], ewt)
                if replay is None and (not conv or not math.isfinite(E)):
                    self.t.pop()
                    self.rejected += 1
                    h *= 0.25
                    continue
                if replay is None and E > 1.0:
                    self.t.pop()
                    self.rejected += 1
                    nfail += 1
                    if nfail >= 3:
                        q, at_q, h = 1, 0, h * 0.25
                    else:
                        h *= max(0.2, min(0.9, 0.9 * E ** (-1.0 / (q + 1))))
                    continue
                break
            # accept: the right sides once more at y_n, then the state
            fk = replay[n]["ks"][m] if replay is not None else None
            fe, f, hook, vals = self._evaluate(n, y, u, A, mat, fk)
            ks.append(hook.k)
            self._store(n, f, hook, *vals, u, A, mat)
            dens.append(torch.real(-1j * torch.diagonal(vals[0][n])))
            self.trace.append({"t": tn, "q": q, "m": m, "ks": ks, "E": E, "h": h})
            if replay is None:
                h, q, at_q = self._next(n, h, q, at_q, E, ewt)
            n += 1
        return torch.stack(dens)

    def _next(self, n, h, q, at_q, E, ewt):
        """Step size and order for step n + 1 after accepting step n."""
        c = self.c
        at_q += 1
        tg = np.array(self.t)
        cand = [(1.0 / ((6.0 * E) ** (1.0 / (q + 1)) + 1e-6), q)]
        if at_q >= q + 1:
            _, hist = self._elements(n)                      # histories now include t_n
            for dq, bias in ((-1, 6.0), (1, 10.0)):
                qq = q + dq
                npts = qq + 1   # f over qq + 1 points ~ y^(qq+1) / qq!
                if qq < 1 or qq > c.qmax or npts > n + 1:
                    continue
                coef = node_poly_integral(tg[n - qq + 1: n + 1], tg[n - 1], tg[n])
                ts = tg[n - npts + 1: n + 1]
                vals = [coef * divided_difference(ts, [hi[j] for j in range(n - npts + 1, n + 1)])
                        for hi in hist]
                Eq = self._wrms(vals, ewt)
                if not math.isfinite(Eq):
                    continue
                cand.append((1.0 / ((bias * Eq) ** (1.0 / (qq + 1)) + 1e-6), qq))
        eta, qn = cand[0]
        for e, qq in cand[1:]:
            if e > eta:
                eta, qn = e, qq
        if eta < 1.5:
            return h, q, at_q
        if qn != q:
            at_q = 0
        return h * min(eta, 10.0), qn, at_q

    def storage(self):
        return _pr.storage(self.S)
