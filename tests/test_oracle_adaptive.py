"""Pins for the oracle's adaptive propagation (oracle/adaptive.py).

  * the predictor and corrector weights against Adams-Bashforth and Adams-Moulton rules computed
    in exact rational arithmetic on uniform grids, and against numpy's polynomial fit and
    integration on random non-uniform nodes; the error coefficients against numpy's polynomial
    integration; divided differences against the leading coefficient of a polynomial;
  * the history sums above the diagonal used to reconstruct new blocks' right sides, C^<(j,n) for
    j < n, against -K1(n,j)^dagger, the history sums of Eq. KBE1 at (t_n, t_j) computed by plain
    loops from full G and Sigma matrices (the two are adjoint term by term);
  * tolerance proportionality on a single orbital with a pulse (closed form: an erf phase): the
    error at t_end falls with rtol and stays within a small multiple of it;
  * particle-number conservation to rounding in an interacting adaptive run, with the order and
    the history order actually varying;
  * the replay of a run's decisions reproduces the run bit for bit (the GPU parity tests replay
    the GPU's decisions on the oracle).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch
from scipy.special import erf

import synth
from oracle import adaptive as ad
from oracle import propagate as op
from tests.helpers import pack_kp, random_symmetric_full
from tests.test_oracle_weights import exact_lagrange_integrals


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6])
def test_predictor_weights_are_adams_bashforth(q):
    nodes = [Fraction(-i) for i in range(q - 1, -1, -1)]        # t_{n-q..n-1} = -(q-1)..0
    exact = exact_lagrange_integrals(nodes, Fraction(0), Fraction(1))
    got = ad.lagrange_integrals(np.array([float(x) for x in nodes]), 0.0, 1.0)
    np.testing.assert_allclose(got, [float(x) for x in exact], rtol=0, atol=1e-14)
    if q == 2:
        assert exact == [Fraction(-1, 2), Fraction(3, 2)]


@pytest.mark.parametrize("q", [1, 2, 4, 7, 12])
def test_weights_match_polynomial_fit_on_random_nodes(q):
    rng = np.random.default_rng(q)
    x = np.cumsum(rng.uniform(0.5, 1.5, q))
    a, b = x[-1] - 0.7, x[-1] + 0.9          # an interval extending past the last node
    lam = ad.lagrange_integrals(x, a, b)
    for deg in range(q):
        f = lambda s: (s - x.mean()) ** deg
        P = np.polynomial.Polynomial.fit(x, f(x), q - 1)
        I = P.integ()
        exact = I(b) - I(a)
        assert abs(lam @ f(x) - exact) < 1e-10 * max(1.0, abs(exact))


@pytest.mark.parametrize("q", [1, 2, 3, 5, 8])
def test_error_coefficients_and_divided_differences(q):
    rng = np.random.default_rng(20 + q)
    x = np.cumsum(rng.uniform(0.1, 0.3, q))
    a, b = x[-1] - 0.2, x[-1]
    P = np.polynomial.Polynomial.fromroots(x).integ()
    assert abs(ad.node_poly_integral(x, a, b) - (P(b) - P(a))) < 1e-12 * (abs(P(b)) + abs(P(a)))
    c = rng.normal(size=q + 1)
    poly = np.polynomial.Polynomial(c)
    ts = np.cumsum(rng.uniform(0.2, 0.5, q + 1))
    dd = ad.divided_difference(ts, [torch.tensor(poly(z)) for z in ts])
    assert abs(float(dd) - c[-1]) < 1e-9 * max(1.0, abs(c[-1]))


def _k1(j, n, GL, GR, SL, SR, w):
    """Plain loops: sum_s w[n][s] G^R(n,s) Sigma^<(s,j) + sum_s w[j][s] G^<(n,s) Sigma^A(s,j)."""
    acc = 0
    for s in range(n + 1):
        acc = acc + w[n, s] * GR[n, s] @ SL[s, j]
    for s in range(j + 1):
        acc = acc + w[j, s] * GL[n, s] @ SR[j, s].conj().T
    return acc


def test_upper_history_sums_are_adjoint_to_kbe1():
    rng = np.random.default_rng(3)
    N, nt = 2, 9
    les, gtr = random_symmetric_full(rng, N, nt)
    sles, sgtr = random_symmetric_full(rng, N, nt)
    kp = pack_kp(les, gtr - les)
    t, order = synth.grid(4, nt, 0.02, 0.08, 3, 5)
    h0 = np.zeros((N, N))
    P = op.Problem(t=t, order=order, h0=h0, ntau=0, rho0=np.eye(N))
    A = ad.Adaptive(P, ad.Controls(t_end=1.0, nt_max=nt))
    A.W["w"][:nt, :nt] = P.weights()["w"]
    w = P.weights()["w"].numpy()
    SR = np.where(np.arange(nt)[:, None, None, None] >= np.arange(nt)[None, :, None, None],
                  sgtr - sles, 0)
    for n in range(nt):
        A.sig.append((torch.tensor(np.array([SR[n, s] for s in range(n + 1)])),
                      torch.tensor(np.array([sles[n, s] for s in range(n + 1)])),
                      torch.zeros((0, N, N), dtype=torch.complex128)))
    GR = np.where(np.arange(nt)[:, None, None, None] > np.arange(nt)[None, :, None, None],
                  gtr - les, 0)
    for a_ in range(nt):
        GR[a_, a_] = -1j * np.eye(N)
    A.S.tv = [torch.zeros((0, N, N), dtype=torch.complex128)] * nt
    KP = torch.tensor(kp)
    for n in (3, 8):
        for j in range(n):
            Cl, Cg = A._upper_sums(j, n, KP[: n + 1, : n + 1], None)
            ref = -_k1(j, n, les, GR, sles, SR, w).conj().T
            np.testing.assert_allclose(Cl.numpy(), ref, atol=1e-13 * np.abs(ref).max())


def _single_orbital(rtol, A_=0.8, h0=0.3, rho=0.6, T_end=4.0):
    P = op.Problem(t=np.zeros(1), order=np.zeros(1, np.int32), h0=np.array([[h0]]), ntau=0,
                   rho0=np.array([[rho]]))
    run = ad.Adaptive(P, ad.Controls(t_end=T_end, rtol=rtol, atol=rtol * 1e-3, nt_max=3000))
    run.run(0.0, A_)
    kp, _ = run.storage()
    t = np.array(run.t)
    s2 = np.sqrt(2.0)
    phi = h0 * t + A_ * np.sqrt(np.pi / 2) * (erf((t - 2.0) / s2) - erf(-2.0 / s2))
    exact = 1j * rho * np.exp(1j * (phi[-1] - phi))
    return np.abs(kp[:, -1, 0, 0] - exact).max(), len(run.trace), run


def test_tolerance_proportionality_single_orbital():
    errs, steps = [], []
    for rtol in (1e-4, 1e-6, 1e-8):
        e, n, _ = _single_orbital(rtol)
        errs.append(e)
        steps.append(n)
    assert steps[0] < steps[1] < steps[2]
    assert errs[0] > errs[1] > errs[2]
    for e, rtol in zip(errs, (1e-4, 1e-6, 1e-8)):
        assert e < 100 * rtol


def test_interacting_run_conserves_and_adapts():
    N, ntau, beta = 2, 6, 2.0
    h0 = synth.tight_binding(N)
    mat, _ = synth.free_thermal(h0, beta, ntau)
    P = op.Problem(t=np.zeros(1), order=np.zeros(1, np.int32), h0=h0, ntau=ntau, beta=beta,
                   mat=mat)
    run = ad.Adaptive(P, ad.Controls(t_end=1.5, rtol=1e-5, atol=1e-8, nt_max=1000))
    d = run.run(1.0, 0.7).numpy()
    tr = d.sum(axis=1)
    assert np.abs(tr - tr[0]).max() < 1e-13
    qs = {x["q"] for x in run.trace}
    ks = {k for x in run.trace for k in x["ks"]}
    hs = np.diff(run.t)
    assert len(qs) >= 3 and len(ks) >= 3 and hs.max() > 10 * hs.min()
    # replay of the decisions reproduces the run bit for bit
    rep = ad.Adaptive(P, ad.Controls(t_end=1.5, rtol=1e-5, atol=1e-8, nt_max=1000))
    d2 = rep.run(1.0, 0.7, replay=[None] + run.trace).numpy()
    assert np.array_equal(d, d2)
    assert np.array_equal(np.array(run.t), np.array(rep.t))
