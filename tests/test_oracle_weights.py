"""Pins for the oracle's quadrature weights (Sec. "Adaptive History Integration", Eq. weights
and the weight-row recursion)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

# Textbook Adams-Moulton coefficients on a uniform grid (h = 1), oldest node first: the local
# weights of the k-node rule over the last interval.
ADAMS_MOULTON = {
    2: [Fraction(1, 2), Fraction(1, 2)],
    3: [Fraction(-1, 12), Fraction(8, 12), Fraction(5, 12)],
    4: [Fraction(1, 24), Fraction(-5, 24), Fraction(19, 24), Fraction(9, 24)],
    5: [Fraction(-19, 720), Fraction(106, 720), Fraction(-264, 720), Fraction(646, 720),
        Fraction(251, 720)],
    6: [Fraction(27, 1440), Fraction(-173, 1440), Fraction(482, 1440), Fraction(-798, 1440),
        Fraction(1427, 1440), Fraction(475, 1440)],
}


def exact_lagrange_integrals(nodes, a, b):
    """Integral over [a, b] of each Lagrange basis polynomial, in exact rational arithmetic."""
    k = len(nodes)
    out = []
    for j in range(k):
        # coefficients of prod_{i != j} (x - x_i) / (x_j - x_i), lowest degree first
        poly = [Fraction(1)]
        den = Fraction(1)
        for i in range(k):
            if i == j:
                continue
            poly = [Fraction(0)] + poly  # multiply by x
            for d in range(len(poly) - 1):
                poly[d] -= nodes[i] * poly[d + 1]
            den *= nodes[j] - nodes[i]
        val = sum(c * (b ** (d + 1) - a ** (d + 1)) / (d + 1) for d, c in enumerate(poly))
        out.append(val / den)
    return out


def test_gauss_legendre_exact_on_monomials():
    for m in range(1, 12):
        x, w = oracle.gauss_legendre(m)
        xl, wl = np.polynomial.legendre.leggauss(m)
        np.testing.assert_allclose(np.sort(x), np.sort(xl), atol=1e-14)
        for d in range(2 * m):
            exact = 0.0 if d % 2 else 2.0 / (d + 1)
            assert abs(np.dot(w, x ** d) - exact) < 1e-13


@pytest.mark.parametrize("k", sorted(ADAMS_MOULTON))
def test_uniform_grid_gives_adams_moulton(k):
    t = np.arange(12, dtype=np.float64)
    lam = oracle.local_weights(t, 11, k)
    np.testing.assert_allclose(lam, [float(c) for c in ADAMS_MOULTON[k]], rtol=0, atol=2e-15)


@pytest.mark.parametrize("k", [2, 3, 5, 8, 12, 16, 20])
def test_local_weights_equal_exact_rational_integrals(k):
    rng = np.random.default_rng(k)
    steps = [Fraction(int(v), 1000) for v in rng.integers(20, 80, size=k + 1)]
    tq = [Fraction(0)]
    for s in steps:
        tq.append(tq[-1] + s)
    p = len(tq) - 1
    nodes = tq[p - k + 1:p + 1]
    ref = exact_lagrange_integrals(nodes, tq[p - 1], tq[p])
    lam = oracle.local_weights(np.array([float(x) for x in tq]), p, k)
    scale = max(abs(float(r)) for r in ref)
    assert max(abs(lam[j] - float(ref[j])) for j in range(k)) < 1e-13 * max(1.0, scale) * k


@pytest.mark.parametrize("hmin,hmax", [(0.02, 0.08), (0.005, 0.05)])
def test_composite_weights_exact_on_polynomials(hmin, hmax):
    t, order = synth.grid(7, 60, hmin, hmax, 3, 6)
    w = oracle.weights(t, order)
    for n in range(1, 60):
        kmin = min(min(order[p], p + 1) for p in range(1, n + 1))
        for d in range(kmin):
            # shifted Legendre polynomial on [0, t_n]; its integral over [0, t_n] is 0 for d > 0
            c = np.zeros(d + 1)
            c[d] = 1.0
            vals = np.polynomial.legendre.legval(2 * t[: n + 1] / t[n] - 1, c)
            exact = t[n] if d == 0 else 0.0
            assert abs(np.dot(w[n, : n + 1], vals) - exact) < 1e-12 * max(1, t[n]), (n, d)
        assert np.all(w[n, n + 1:] == 0)


def test_sum_rules():
    t, order = synth.grid(3, 80, 0.005, 0.05, 3, 6)
    w = oracle.weights(t, order)
    np.testing.assert_allclose(w.sum(axis=1), t, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(w @ t, t ** 2 / 2, rtol=1e-12, atol=1e-15)
    assert np.all(w[0] == 0)


def test_vandermonde_route_matches():
    """The paper computes local weights by solving the (transposed) Vandermonde system
    V^T omega = T with V_{jl} = (x_j - x_0)^l, T_l = int (t - x_0)^l dt (Eq. weights).  Solve that
    system with a library solver and compare to the oracle's Lagrange-integral route."""
    t, _ = synth.grid(11, 40, 0.005, 0.05, 3, 6)
    for k in range(1, 9):
        p = 30
        x = t[p - k + 1:p + 1]
        h = t[p] - t[p - 1]
        xs = (x - x[0]) / h
        a, b = (t[p - 1] - x[0]) / h, (t[p] - x[0]) / h
        V = np.vander(xs, k, increasing=True)
        T = np.array([(b ** (l + 1) - a ** (l + 1)) / (l + 1) for l in range(k)])
        om = h * np.linalg.solve(V.T, T)
        np.testing.assert_allclose(oracle.local_weights(t, p, k), om, rtol=1e-11, atol=1e-15)


def test_order_two_is_trapezoid():
    t, _ = synth.grid(5, 30, 0.005, 0.05, 2, 2)
    order = np.full(30, 2, np.int32)
    w = oracle.weights(t, order)
    n = 29
    trap = np.zeros(30)
    h = np.diff(t)
    trap[:-1] += h / 2
    trap[1:] += h / 2
    np.testing.assert_allclose(w[n], trap, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_convergence_order(k):
    """Scalar integrand e^{i D s}: the error of the composite rule falls as h^k once every
    interval has its full k nodes.  (The first k-2 intervals have fewer points available, so the
    rule over [0, t_n] is limited by them; rows n and k-1 are differenced to remove them.)"""
    D = 3.0
    errs = []
    for nt in (41, 81, 161):
        t = np.linspace(0, 2.0, nt)
        w = oracle.weights(t, np.full(nt, k, np.int32))
        a = t[k - 1]
        exact = (np.exp(1j * D * t[-1]) - np.exp(1j * D * a)) / (1j * D)
        errs.append(abs(np.dot(w[-1] - w[k - 1], np.exp(1j * D * t)) - exact))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > k - 0.6), (errs, rates)


def test_tau_weights():
    """Every tau piece is exact for polynomials of degree < min(k, nodes in the piece); the full
    range rule is exact for degree < k and symmetric."""
    beta, ntau, order = 10.0, 33, 5
    wf, wb, wfull = oracle.tau_weights(beta, ntau, order)
    tau = beta * np.arange(ntau) / (ntau - 1)
    np.testing.assert_allclose(wfull, wfull[::-1], rtol=1e-14)
    for d in range(order):
        f = (tau / beta) ** d
        assert abs(wfull @ f - beta / (d + 1)) < 1e-12
        for j in range(ntau):
            # forward piece over [0, tau_j], backward piece over [tau_j, beta]
            if d < min(order, j + 1):
                assert abs(wf[j] @ f - tau[j] * (tau[j] / beta) ** d / (d + 1)) < 1e-12
            if d < min(order, ntau - j):
                assert abs(wb[j] @ f - (beta - tau[j] * (tau[j] / beta) ** d) / (d + 1)) < 1e-12
            assert np.all(wf[j, j + 1:] == 0) and np.all(wb[j, :j] == 0)
    # on a uniform grid the backward rule is the forward rule reflected
    np.testing.assert_allclose(wb, wf[::-1, ::-1], rtol=1e-13, atol=1e-16)
