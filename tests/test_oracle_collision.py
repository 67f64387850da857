"""Pins for the oracle's history integrals (Eq. KBE2 lesser form and the history terms of
Eq. KBE3)."""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

import oracle
import synth
from tests.helpers import (FreeSystem, expm_h, pack_kp, random_hermitian, random_symmetric_full,
                           relerr, tight_binding)


def free_setup(N=3, nt=24, ntau=17, beta=2.0, seed=1):
    rng = np.random.default_rng(seed)
    h = tight_binding(N) + random_hermitian(rng, N, 0.3)
    fs = FreeSystem(h, beta)
    t, order = synth.grid(seed, nt, 0.02, 0.08, 3, 6)
    taus = beta * np.arange(ntau) / (ntau - 1)
    W = oracle.Weights.build(t, order, beta, ntau, 5)
    return fs, t, taus, W


@pytest.mark.parametrize("N,nt,seed", [(3, 24, 1), (1, 9, 2), (4, 40, 3), (6, 17, 4)])
def test_free_closed_forms_real_time(N, nt, seed):
    """Sigma^R := G^R_h, G^< := G^<_h  =>  I^R(n,m) = t_n e^{-iht_n} rho e^{iht_m};
    Sigma^< := G^<_h, G^R := G^R_h  =>  I^<(n,m) = -t_m e^{-iht_n} rho e^{iht_m}
    (the integrand is constant in s; only the weight sums enter).  Several orbital counts,
    grids and per-interval orders."""
    fs, t, taus, W = free_setup(N=N, nt=nt, seed=seed)
    nt = len(t)
    n = nt - 1
    G = oracle.Green(fs.kp(t), fs.rdiag(nt))
    ret = np.array([fs.ret(t[n], t[s]) for s in range(n + 1)])
    les = np.array([fs.les(t[n], t[s]) for s in range(n + 1)])
    sig = (ret, les, np.zeros((0, fs.N, fs.N)))
    IR, IL, _, _ = oracle.collision(G, sig, W, n, flags=oracle.F_IR | oracle.F_IL)
    for m in range(n + 1):
        core = expm_h(fs.h, -1j * t[n]) @ fs.rho @ expm_h(fs.h, 1j * t[m])
        assert relerr(IR[m], t[n] * core) < 1e-12
        assert relerr(IL[m], -t[m] * core) < 1e-12


@pytest.mark.parametrize("N,nt,ntau,seed", [(3, 24, 17, 1), (2, 12, 9, 5), (5, 30, 25, 6)])
def test_free_closed_forms_thermal(N, nt, ntau, seed):
    """With the free mixed and Matsubara components:
    I^](n,m) = -i beta e^{-iht_n} f e^{beta h} f e^{iht_m};
    J^] real-time part (Sigma^R := G^R_h) = t_n e^{-iht_n} f e^{h tau_j};
    J^] Matsubara part (Sigma^] := G^]_h) = i e^{-iht_n} f e^{h tau_j} [tau_j f - (beta-tau_j)(1-f)]
    (constant integrand on each side of the jump of G^M)."""
    fs, t, taus, W = free_setup(N=N, nt=nt, ntau=ntau, seed=seed)
    nt, ntau, N = len(t), len(taus), fs.N
    n, beta = nt - 1, fs.beta
    tv = fs.tv(t, taus)
    mat = fs.mat(taus)
    G = oracle.Green(fs.kp(t), fs.rdiag(nt), tv, mat)
    stv = np.array([fs.mixed(t[n], tau) for tau in taus])
    zero = np.zeros((n + 1, N, N), np.complex128)
    ret = np.array([fs.ret(t[n], t[s]) for s in range(n + 1)])
    f = fs.rho
    eb = expm_h(fs.h, beta)
    _, _, Itv, _ = oracle.collision(G, (zero, zero, stv), W, n, flags=oracle.F_ITV)
    for m in range(n + 1):
        ref = -1j * beta * expm_h(fs.h, -1j * t[n]) @ f @ eb @ f @ expm_h(fs.h, 1j * t[m])
        assert relerr(Itv[m], ref) < 1e-12
    # real-time part of J^] alone (Sigma^] = 0)
    _, _, _, J1 = oracle.collision(G, (ret, zero, np.zeros_like(stv)), W, n, flags=oracle.F_JTV)
    # Matsubara part alone (Sigma^R = 0)
    _, _, _, J2 = oracle.collision(G, (zero, zero, stv), W, n, flags=oracle.F_JTV)
    one = np.eye(N)
    for j, tau in enumerate(taus):
        core = expm_h(fs.h, -1j * t[n]) @ f @ expm_h(fs.h, tau)
        assert relerr(J1[j], t[n] * core) < 1e-12
        ref2 = 1j * core @ (tau * f - (beta - tau) * (one - f))
        assert relerr(J2[j], ref2) < 1e-12


def _poly_vals(c, x):
    return P.polyval(x, c)


def test_polynomial_integrands_exact():
    """Integrands that are polynomials of degree < k are integrated exactly:
    Sigma(n,s) = B p1(t_s), G(s,m) = A p2(t_s)  =>  integral = B A int p1 p2."""
    rng = np.random.default_rng(8)
    N, nt, ntau, beta = 2, 30, 21, 3.0
    t, order = synth.grid(8, nt, 0.02, 0.08, 4, 6)
    W = oracle.Weights.build(t, order, beta, ntau, 5)
    taus = beta * np.arange(ntau) / (ntau - 1)
    n, m, J = nt - 1, 17, ntau - 1
    rnd = lambda *s: rng.normal(size=s) + 1j * rng.normal(size=s)
    A, B, C = rnd(N, N), rnd(N, N), rnd(N, N)
    # tau integrals: degree 1 * degree 2 = 3 < 5 nodes.  Real time: the first intervals of the
    # causal rule have only 2 and 3 nodes, so the whole-range rule is exact to degree 1 only.
    p1, p2 = np.array([0.3, -1.1]), np.array([0.7, 0.2, 0.5])
    q1, q2 = np.array([0.3, -1.1]), np.array([0.7])
    kp = rnd(nt, nt, N, N)
    rdiag = rnd(nt, N, N)
    tv = rnd(nt, ntau, N, N)
    mat = rnd(ntau, N, N)
    ret = np.array([B * _poly_vals(q1, t[s]) for s in range(n + 1)])
    les = np.array([B * _poly_vals(q1, t[s]) for s in range(n + 1)])
    stv = np.array([B * _poly_vals(p1, tau) for tau in taus])
    for s in range(nt):  # G^<(s,m) = p2(t_s) A for all s: stored column m (s <= m), row m (s > m)
        if s <= m:
            kp[s, m] = _poly_vals(q2, t[s]) * A
        else:
            kp[m, s] = -(_poly_vals(q2, t[s]) * A).conj().T
    for s in range(m):  # G^R(m,s) = q2(t_s) C
        kp[m, s] = _poly_vals(q2, t[s]) * C
    rdiag[m] = _poly_vals(q2, t[m]) * C
    for j in range(ntau):  # G^[(tau_j, t_m) = G^](t_m, beta - tau_j)^dagger = p2(tau_j) C
        tv[m, J - j] = (_poly_vals(p2, taus[j]) * C).conj().T
    tv_j = tv.copy()  # separate array for the real-time part of J^] (probed column 5)
    for s in range(n + 1):  # G^](s, tau_5) = q2(t_s) C
        tv_j[s, 5] = _poly_vals(q2, t[s]) * C
    prod, qprod = P.polymul(p1, p2), P.polymul(q1, q2)
    integ = lambda a, b: P.polyval(b, P.polyint(prod)) - P.polyval(a, P.polyint(prod))
    qinteg = lambda a, b: P.polyval(b, P.polyint(qprod)) - P.polyval(a, P.polyint(qprod))
    G = oracle.Green(kp, rdiag, tv, mat)
    IR, IL, Itv, Jtv = oracle.collision(G, (ret, les, stv), W, n, m, m + 1)
    assert relerr(IR[0], B @ A * qinteg(0, t[n])) < 1e-12
    assert relerr(IL[0], B @ C.conj().T * qinteg(0, t[m])) < 1e-12
    assert relerr(Itv[0], -1j * B @ C * integ(0, beta)) < 1e-12
    # Matsubara pieces: mat[q] = p2(tau_q) C; for column j the pieces integrate
    # -p1(x) p2(beta + x - tau_j) over [0, tau_j] and p1(x) p2(x - tau_j) over [tau_j, beta]
    mat2 = np.array([_poly_vals(p2, tau) * C for tau in taus])
    G2 = oracle.Green(kp, rdiag, tv, mat2)
    _, _, _, Jm = oracle.collision(G2, (0 * ret, les, stv), W, n, flags=oracle.F_JTV)
    def shifted(c):  # coefficients of p2(x + c)
        out = np.zeros(len(p2))
        for d, coef in enumerate(p2):
            out[: d + 1] += coef * P.polypow([c, 1.0], d)[: d + 1]
        return out

    for j in range(4, ntau - 4):  # pieces with at least k nodes on both sides
        tj = taus[j]
        left = P.polymul(p1, shifted(beta - tj))
        right = P.polymul(p1, shifted(-tj))
        I_left = P.polyval(tj, P.polyint(left)) - P.polyval(0, P.polyint(left))
        I_right = P.polyval(beta, P.polyint(right)) - P.polyval(tj, P.polyint(right))
        ref = B @ C * (-I_left + I_right)
        assert relerr(Jm[j], ref) < 1e-11, j
    # real-time part of J^] at the probed column
    G3 = oracle.Green(kp, rdiag, tv_j, mat)
    _, _, _, Jr = oracle.collision(G3, (ret, les, 0 * stv), W, n, flags=oracle.F_JTV)
    assert relerr(Jr[5], B @ C * qinteg(0, t[n])) < 1e-12


def test_particle_number_conservation():
    """With Sigma from the second-Born formula of the same G, Re Tr[I^R(n,n) + I^<(n,n)] = 0 and
    Re Tr[I^](n,n)] = 0 for any real weights (symmetric in tau): the discrete form of the
    conservation law of a Phi-derivable self-energy."""
    rng = np.random.default_rng(21)
    N, nt, ntau = 3, 14, 11
    les, gtr = random_symmetric_full(rng, N, nt)
    ret_full = gtr - les
    kp = pack_kp(les, ret_full)
    rdiag = np.array([ret_full[a, a] for a in range(nt)])
    tv = rng.normal(size=(nt, ntau, N, N)) + 1j * rng.normal(size=(nt, ntau, N, N))
    G = oracle.Green(kp, rdiag, tv, rng.normal(size=(ntau, N, N)) + 0j)
    t, order = synth.grid(21, nt, 0.02, 0.08, 3, 6)
    W = oracle.Weights.build(t, order, 4.0, ntau, 5)
    u = rng.uniform(0.5, 1.5, size=N)
    for n in (nt - 1, 7):
        sig = oracle.sigma_row(G, u, n)
        IR, IL, Itv, _ = oracle.collision(G, sig, W, n, n, n + 1)
        scale = sum(abs(W.w[n, s]) * np.abs(sig[0][s]).sum() * np.abs(kp).max() for s in range(n + 1))
        assert abs(np.trace(IR[0] + IL[0]).real) < 1e-13 * scale
        assert abs(np.trace(IR[0]).real) > 1e-6 * scale  # each part alone is not conserving
        assert abs(np.trace(Itv[0]).real) < 1e-13 * np.abs(Itv[0]).sum() * ntau


def test_retarded_integral_is_one_gemm():
    """At fixed n, I^R(n, :) = [w_ns Sigma^R(n,s)]_s @ [G^<(s,m)]_{s,m}: one matrix product."""
    rng = np.random.default_rng(2)
    N, nt = 3, 20
    les, gtr = random_symmetric_full(rng, N, nt)
    kp = pack_kp(les, gtr - les)
    rdiag = np.array([(gtr - les)[a, a] for a in range(nt)])
    G = oracle.Green(kp, rdiag)
    t, order = synth.grid(2, nt, 0.02, 0.08, 3, 6)
    W = oracle.Weights.build(t, order)
    n = nt - 1
    ret = rng.normal(size=(n + 1, N, N)) + 1j * rng.normal(size=(n + 1, N, N))
    sig = (ret, ret, np.zeros((0, N, N)))
    IR, _, _, _ = oracle.collision(G, sig, W, n, flags=oracle.F_IR)
    left = np.concatenate([W.w[n, s] * ret[s] for s in range(n + 1)], axis=1)
    big = np.block([[les[s, m] for m in range(n + 1)] for s in range(n + 1)])
    ref = left @ big
    for m in range(n + 1):
        assert relerr(IR[m], ref[:, m * N:(m + 1) * N]) < 1e-13


def _interp_integral(ts, gs, a, b):
    """Integral over [a, b] of the polynomial through (ts, gs) (matrix-valued), exactly."""
    x0 = ts[-1]
    scale = ts[-1] - ts[0] if len(ts) > 1 else 1.0
    xs = (ts - x0) / scale
    out = np.zeros(gs.shape[1:], np.complex128)
    V = np.vander(xs, len(ts), increasing=True)
    for idx in np.ndindex(*gs.shape[1:]):
        c = np.linalg.solve(V, gs[(slice(None),) + idx])
        ci = P.polyint(c)
        out[idx] = scale * (P.polyval((b - x0) / scale, ci) - P.polyval((a - x0) / scale, ci))
    return out


@pytest.mark.parametrize("N,nt", [(1, 7), (2, 9)])
def test_brute_force_interval_interpolants(N, nt):
    """Tiny grids: interpolate the integrand on each interval's nodes explicitly and integrate
    the interpolant exactly; summing the intervals must reproduce the quadrature."""
    rng = np.random.default_rng(nt)
    les, gtr = random_symmetric_full(rng, N, nt)
    ret_full = gtr - les
    kp = pack_kp(les, ret_full)
    rdiag = np.array([ret_full[a, a] for a in range(nt)])
    G = oracle.Green(kp, rdiag)
    t, order = synth.grid(nt, nt, 0.05, 0.3, 2, 5)
    W = oracle.Weights.build(t, order)
    n = nt - 1
    sret = rng.normal(size=(n + 1, N, N)) + 1j * rng.normal(size=(n + 1, N, N))
    sles = rng.normal(size=(n + 1, N, N)) + 1j * rng.normal(size=(n + 1, N, N))
    IR, IL, _, _ = oracle.collision(G, (sret, sles, np.zeros((0, N, N))), W, n,
                                    flags=oracle.F_IR | oracle.F_IL)
    for m in range(n + 1):
        gR = np.array([sret[s] @ les[s, m] for s in range(n + 1)])
        gL = np.array([sles[s] @ ret_full[m, s].conj().T for s in range(n + 1)])
        refR = sum(_interp_integral(t[p - min(order[p], p + 1) + 1:p + 1],
                                    gR[p - min(order[p], p + 1) + 1:p + 1], t[p - 1], t[p])
                   for p in range(1, n + 1))
        refL = sum(_interp_integral(t[p - min(order[p], p + 1) + 1:p + 1],
                                    gL[p - min(order[p], p + 1) + 1:p + 1], t[p - 1], t[p])
                   for p in range(1, m + 1)) if m > 0 else np.zeros((N, N))
        assert np.abs(IR[m] - refR).max() < 1e-12 * max(1, np.abs(refR).max())
        assert np.abs(IL[m] - refL).max() < 1e-12 * max(1, np.abs(refL).max())


def test_m_range_is_a_slice():
    w = synth.PARITY_SMALL
    g = synth.green(w)
    G = oracle.Green(g["kp"], g["rdiag"], g["tv"], g["mat"])
    W = oracle.Weights.build(g["t"], g["order"], w.beta, w.ntau, w.tau_order)
    n = w.nt - 1
    sig = synth.sigma_row(w.seed, w.N, n, w.ntau, g["t"])
    full = oracle.collision(G, sig, W, n)
    part = oracle.collision(G, sig, W, n, 10, 37)
    for a, b in zip(full[:3], part[:3]):
        np.testing.assert_array_equal(a[10:37], b)
    np.testing.assert_array_equal(full[3], part[3])


@pytest.mark.parametrize("N,nt,ntau", [(1, 20, 0), (2, 30, 6), (3, 25, 9), (5, 18, 4)])
def test_row_from_cross_equals_full_system(N, nt, ntau):
    """oracle.collision_row (one (t_n, t_m) from the blocks that row reads) against
    oracle.collision on the full system, for rows with m = 0, m = n, n = 0 and interior m: the
    same sums in the same order, so the blocks agree to the last bit or nearly."""
    t, order = synth.grid(40 + N, nt, 0.02, 0.08, 3, 6)
    kp = synth.kp(40 + N, N, t)
    rd = synth.rdiag(N, nt)
    tv = synth.tv(40 + N, N, ntau, t)
    mat = synth.mat(40 + N, N, ntau)
    G = oracle.Green(kp, rd, tv, mat)
    W = oracle.Weights.build(t, order, 3.0 if ntau else None, ntau, 5)
    flags = oracle.F_IR | oracle.F_IL | (oracle.F_ITV if ntau else 0)
    for n, m in [(0, 0), (nt - 1, 0), (nt - 1, nt - 1), (nt - 1, nt // 2), (nt // 2, 3)]:
        sig = synth.sigma_row(7 + n, N, n, ntau, t)
        if not ntau:
            sig = (sig[0], sig[1], np.zeros((0, N, N), np.complex128))
        IR, IL, Itv, _ = oracle.collision(G, sig, W, n, m, m + 1, flags)
        r = oracle.collision_row(N, ntau, n, m, sig, kp[:m + 1, m], kp[m, :n + 1], rd[m],
                                 tv[m] if ntau else None, W.w[n, :n + 1], W.w[m, :m + 1],
                                 W.wfull if ntau else None, flags)
        for got, want in zip(r, (IR[0], IL[0], Itv[0])):
            assert np.abs(got - want).max() <= 1e-14 * (np.abs(want).max() + 1e-300)


def test_greater_form_from_full_matrices():
    """F_GREATER against direct sums over the full G^< and G^> matrices (no KP storage logic):
    I^R(n, :) = [w_ns Sigma^R(n,s)]_s @ [G^>(s,m)]_{s,m} and
    I^<(n,m) = sum_{s<=m} w_ms (Sigma^R + Sigma^<)(n,s) G^R(m,s)^dagger, G^R = G^> - G^< below and
    on the diagonal; the tau outputs are the same in both forms."""
    rng = np.random.default_rng(12)
    N, nt, ntau = 2, 14, 6
    les, gtr = random_symmetric_full(rng, N, nt)
    kp = pack_kp(les, gtr - les)
    rdiag = np.array([(gtr - les)[a, a] for a in range(nt)])
    tv = rng.normal(size=(nt, ntau, N, N)) + 1j * rng.normal(size=(nt, ntau, N, N))
    mat = rng.normal(size=(ntau, N, N)) + 1j * rng.normal(size=(ntau, N, N))
    G = oracle.Green(kp, rdiag, tv, mat)
    t, order = synth.grid(12, nt, 0.02, 0.08, 3, 6)
    W = oracle.Weights.build(t, order, 3.0, ntau, 5)
    n = nt - 2
    cm = lambda *s: rng.normal(size=s) + 1j * rng.normal(size=s)
    sig = (cm(n + 1, N, N), cm(n + 1, N, N), cm(ntau, N, N))
    ret, sles, _ = sig
    IRg, ILg, Itvg, Jg = oracle.collision(G, sig, W, n, flags=oracle.F_ALL | oracle.F_GREATER)
    IRl, ILl, Itvl, Jl = oracle.collision(G, sig, W, n, flags=oracle.F_ALL)
    left = np.concatenate([W.w[n, s] * ret[s] for s in range(n + 1)], axis=1)
    big = np.block([[gtr[s, m] for m in range(n + 1)] for s in range(n + 1)])
    ref = left @ big
    for m in range(n + 1):
        assert relerr(IRg[m], ref[:, m * N:(m + 1) * N]) < 1e-13
        want = sum(W.w[m, s] * (ret[s] + sles[s]) @ (gtr[m, s] - les[m, s]).conj().T
                   for s in range(m + 1))
        assert relerr(ILg[m], want) < 1e-13
    assert np.array_equal(Itvg, Itvl) and np.array_equal(Jg, Jl)
    assert relerr(IRg[3], IRl[3]) > 1e-3  # the forms differ where G^R is nonzero
