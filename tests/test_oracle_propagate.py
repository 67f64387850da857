"""Pins for the oracle's fixed-grid propagation (oracle/propagate.py) and its gradients.

Each is fixed independently of the code under test:
  * its self-energy row and history sums against the C oracle's (orc_sigma_row, orc_collision,
    lesser and greater form), which carry their own pins;
  * closed forms of single-orbital problems: with the pulse alone, G^<(t_m,t_n) =
    i rho exp(i (phi(t_n) - phi(t_m))), phi the integral of h(t) = h0 + A exp(-(t-2)^2/2) (an erf);
    with a fully occupied orbital and U != 0, Sigma = 0 and the Fock term gives the phase
    (h0 + U) (t_n - t_m); both converge at the order the scheme has (2 with one fixed-point
    iteration, 3 with more: each element's first step is trapezoidal), which pins the pulse's
    centre, width, sign and amplitude, and the sign and size of the Fock term;
  * a stationary state: without interaction or pulse the thermal initial state commutes with
    h0, so the densities stay constant to rounding on any grid;
  * particle-number conservation with interaction and pulse (the Phi-derivable invariant: the
    trace of every density increment is zero), and anti-Hermiticity of G^<(t,t);
  * reverse-mode gradients against central finite differences (h = 1e-6), and the vanishing
    gradient of the conserved total density.
"""
import numpy as np
import pytest
import torch
from scipy.special import erf

import oracle
import synth
from oracle import propagate as op
from tests.helpers import pack_kp, random_symmetric_full, tight_binding


def free_matsubara(h, beta, ntau):
    e, v = np.linalg.eigh(h)
    f = 1.0 / (np.exp(beta * e) + 1.0)
    taus = np.linspace(0.0, beta, ntau)
    return np.array([(v * (-np.exp(-e * x) * (1.0 - f))) @ v.T for x in taus])


def problem(N=2, nt=16, ntau=6, beta=2.0, seed=5, iters=2, omin=3, omax=5):
    t, order = synth.grid(seed, nt, 0.02, 0.08, omin, omax)
    h0 = tight_binding(N)
    return op.Problem(t=t, order=order, h0=h0, ntau=ntau, beta=beta,
                      mat=free_matsubara(h0, beta, ntau) if ntau else None,
                      rho0=None if ntau else np.diag(np.linspace(0.2, 0.8, N)), iters=iters)


def T(x):
    return torch.tensor(x, dtype=torch.float64)


@pytest.mark.parametrize("greater", [False, True])
@pytest.mark.parametrize("N,nt,ntau,n", [(2, 9, 5, 8), (3, 7, 4, 4), (1, 6, 0, 5), (2, 5, 3, 0)])
def test_sums_match_the_c_oracle(greater, N, nt, ntau, n):
    rng = np.random.default_rng(10 * N + nt)
    les, gtr = random_symmetric_full(rng, N, nt)
    kp = pack_kp(les, gtr - les)
    rd = np.array([gtr[a, a] - les[a, a] for a in range(nt)])
    tv = rng.normal(size=(nt, ntau, N, N)) + 1j * rng.normal(size=(nt, ntau, N, N))
    mat = rng.normal(size=(ntau, N, N)) + 1j * rng.normal(size=(ntau, N, N))
    t, order = synth.grid(3, nt, 0.02, 0.08, 3, 6)
    u = np.linspace(0.8, 1.3, N)
    P = op.Problem(t=t, order=order, h0=np.zeros((N, N)), ntau=ntau, beta=2.0, mat=mat)
    W = P.weights()
    KP = torch.tensor(kp[: n + 1, : n + 1])
    GL, GR, GG = op.views(KP, N)
    sig = op.sigma_row(GL, GG, torch.tensor(tv[n]), torch.tensor(u), n)
    G = oracle.Green(kp, rd, tv if ntau else None, mat if ntau else None)
    sref = oracle.sigma_row(G, u, n)
    for a, b in zip(sig, sref):
        if b.size:
            np.testing.assert_allclose(a.numpy(), b, rtol=1e-13, atol=1e-13 * np.abs(b).max())
    out = op.collision(GL, GR, GG, torch.tensor(tv[: n + 1]), torch.tensor(mat), sig, W, n,
                       greater=greater)
    Wo = oracle.Weights.build(t, order, 2.0, ntau, 5)
    ref = oracle.collision(G, sref, Wo, n, 0, n + 1,
                           oracle.F_ALL | (oracle.F_GREATER if greater else 0))
    for name, a, b in zip(("IR", "IL", "Itv", "Jtv"), out, ref):
        if b.size == 0:
            continue
        np.testing.assert_allclose(a.numpy(), b, rtol=0, atol=1e-12 * (np.abs(b).max() + 1e-300),
                                   err_msg=name)


def _single_orbital(nt, order, iters, h0, A=0.0, U=0.0, rho=0.6, T_end=4.0):
    t = np.linspace(0.0, T_end, nt)
    P = op.Problem(t=t, order=np.full(nt, order, np.int32), h0=np.array([[h0]]), ntau=0,
                   rho0=np.array([[rho]]), iters=iters)
    dens, S = op.propagate(P, T(U), T(A))
    kp, _ = op.storage(S)
    return t, kp


def _rate(errs):
    return np.log2(errs[-2] / errs[-1])


@pytest.mark.parametrize("iters,order,want", [(1, 4, 1.9), (2, 4, 2.9), (3, 5, 2.9), (2, 3, 2.9)])
def test_pulse_closed_form_converges(iters, order, want):
    A, h0, rho = 0.8, 0.3, 0.6
    errs = []
    for nt in (41, 81, 161):
        t, kp = _single_orbital(nt, order, iters, h0, A=A, rho=rho)
        s2 = np.sqrt(2.0)
        phi = h0 * t + A * np.sqrt(np.pi / 2) * (erf((t - 2.0) / s2) - erf(-2.0 / s2))
        exact = 1j * rho * np.exp(1j * (phi[-1] - phi))      # G^<(t_m, t_end)
        errs.append(np.abs(kp[:, -1, 0, 0] - exact).max())
    assert errs[-1] < 1e-3
    assert _rate(errs) > want, errs


def test_fock_term_closed_form_converges():
    """A fully occupied single orbital: G^> = 0, so Sigma = 0, and eps = h0 + U n with n = 1."""
    U, h0 = 0.7, 0.3
    errs = []
    for nt in (41, 81, 161):
        t, kp = _single_orbital(nt, 4, 2, h0, U=U, rho=1.0)
        exact = 1j * np.exp(1j * (h0 + U) * (t[-1] - t))
        errs.append(np.abs(kp[:, -1, 0, 0] - exact).max())
    assert errs[-1] < 1e-4
    assert _rate(errs) > 2.9, errs


def test_free_thermal_state_is_stationary():
    P = problem(N=3, nt=14, ntau=8, beta=3.0)
    dens, S = op.propagate(P, T(0.0), T(0.0))
    d = dens.detach().numpy()
    assert np.abs(d - d[0]).max() < 1e-13


@pytest.mark.parametrize("ntau", [6, 0])
def test_particle_number_conserved(ntau):
    P = problem(N=3, nt=16, ntau=ntau)
    dens, S = op.propagate(P, T(1.5), T(0.7))
    tr = dens.detach().numpy().sum(axis=1)
    assert np.abs(tr - tr[0]).max() < 1e-13 * max(1.0, abs(tr[0]))
    assert np.abs(dens.detach().numpy()[-1] - dens.detach().numpy()[0]).max() > 1e-3  # it moves
    kp, _ = op.storage(S)
    for n in range(len(kp)):
        np.testing.assert_allclose(kp[n, n], -kp[n, n].conj().T, atol=1e-13)


@pytest.mark.parametrize("ntau,iters", [(6, 2), (0, 1), (5, 3)])
def test_gradients_match_central_differences(ntau, iters):
    P = problem(N=2, nt=14, ntau=ntau, iters=iters)
    c = np.array([1.0, 0.0])
    U, A, last, h = 1.3, 0.6, 5, 1e-6
    L, gU, gA = op.loss_and_grad(P, U, A, c, last)
    fU = (op.loss(P, U + h, A, c, last) - op.loss(P, U - h, A, c, last)) / (2 * h)
    fA = (op.loss(P, U, A + h, c, last) - op.loss(P, U, A - h, c, last)) / (2 * h)
    assert abs(fU - gU) < 1e-6 * abs(gU) + 1e-9
    assert abs(fA - gA) < 1e-6 * abs(gA) + 1e-9
    assert abs(gU) > 1e-4 and abs(gA) > 1e-4


def test_conserved_total_density_has_no_gradient():
    P = problem(N=3, nt=12, ntau=5)
    L, gU, gA = op.loss_and_grad(P, 1.1, 0.9, np.ones(3), 4)
    assert abs(gU) < 1e-12 * abs(L) and abs(gA) < 1e-12 * abs(L)
