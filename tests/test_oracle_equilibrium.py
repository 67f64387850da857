"""Pins for the oracle's interacting equilibrium initial state (oracle/equilibrium.py).

Each is fixed independently of the code under test:
  * the free Matsubara function against a matrix exponential (scipy.linalg.expm):
    G0(tau) = -exp(-eps tau) (1 + exp(-beta eps))^-1, and its jump G0(0+) + G0(beta-) = -1;
  * the split convolution against closed forms: for scalar free functions a, b of energies e1, e2
    times constant matrices M, K that do not commute, (aM * bK)(tau) = (a - b)(tau) / (e1 - e2) MK
    (the product of the Matsubara transforms 1/(iw - e1) and 1/(iw - e2)); and the resolvent
    identity G0[eps1] - G0[eps2] = G0[eps1] * ((eps1 - eps2) G0[eps2]) for matrices;
  * the Matsubara self-energy against the propagation's mixed self-energy at t = 0, which the
    boundary condition ties to it (Sigma^](0, tau) = -i Sigma^M(beta - tau)), for a complex
    Hermitian G^M;
  * the atomic limit: for one orbital at half filling (h0 = 0, mu = U/2) the second-order
    self-energy of the free G0 = -1/2 is -U^2/8, i.e. U^2 / (4 i w), the exact one of the Hubbard
    atom, whose Dyson solution is the exact atomic G = (G0[U/2] + G0[-U/2]) / 2;
  * the solver: without interaction it returns the free function of h0 - mu; at half filling of a
    particle-hole symmetric chain (mu = U/2) every density is 1/2; the converged G^M satisfies the
    differential form -dG/dtau = eps G + Sigma * G (central differences);
  * the physical pin: a propagation (the oracle's own, pinned elsewhere) started from the
    converged G^M is stationary to its time-stepping error, while one started from the free
    state of the same mean field (eps of the converged densities, no correlation) is not.
"""
import numpy as np
import pytest
import scipy.linalg
import torch

import oracle
import synth
from oracle import equilibrium as eq
from oracle import propagate as op


def sym(rng, N, scale=1.0):
    a = rng.standard_normal((N, N)) * scale
    return 0.5 * (a + a.T)


def test_free_matsubara_matches_matrix_exponential():
    rng = np.random.default_rng(3)
    N, beta, ntau = 4, 3.0, 9
    eps = sym(rng, N, 1.5)
    G = eq.free_matsubara(eps, beta, ntau)
    inv = np.linalg.inv(np.eye(N) + scipy.linalg.expm(-beta * eps))
    for j in range(ntau):
        tau = j * beta / (ntau - 1)
        ref = -scipy.linalg.expm(-tau * eps) @ inv
        np.testing.assert_allclose(G[j], ref, atol=1e-13, rtol=0)
    np.testing.assert_allclose(G[0] + G[-1], -np.eye(N), atol=1e-14)


def test_free_matsubara_stable_at_low_temperature():
    rng = np.random.default_rng(4)
    N, beta, ntau = 3, 400.0, 33
    G = eq.free_matsubara(sym(rng, N, 3.0), beta, ntau)
    assert np.all(np.isfinite(G))
    np.testing.assert_allclose(G[0] + G[-1], -np.eye(N), atol=1e-13)


def scalar_free(e, beta, ntau):
    return eq.free_matsubara(np.array([[e]]), beta, ntau)[:, 0, 0]


# the tau rules use fewer nodes on the intervals next to the ends (a window kept inside the
# range), so the error there falls as h^3; at interior points as h^5
@pytest.mark.parametrize("ntau,tol,tol_in", [(65, 4e-6, 3e-8), (257, 6e-8, 4e-11)])
def test_convolution_of_free_functions(ntau, tol, tol_in):
    beta, e1, e2 = 2.5, 0.7, -1.3
    rng = np.random.default_rng(11)
    M = rng.standard_normal((3, 3))
    K = rng.standard_normal((3, 3))
    assert np.abs(M @ K - K @ M).max() > 0.5
    a, b = scalar_free(e1, beta, ntau), scalar_free(e2, beta, ntau)
    wf, wb, _ = oracle.tau_weights(beta, ntau, 5)
    out = eq.convolution(a[:, None, None] * M, b[:, None, None] * K, wf, wb)
    ref = ((a - b) / (e1 - e2))[:, None, None] * (M @ K)
    err = np.abs(out - ref).max(axis=(1, 2)) / np.abs(M @ K).max()
    assert err.max() < tol and err[8:-8].max() < tol_in, (err.max(), err[8:-8].max())


def test_convolution_resolvent_identity():
    rng = np.random.default_rng(12)
    N, beta, ntau = 3, 2.0, 129
    e1, e2 = sym(rng, N), sym(rng, N)
    G1, G2 = eq.free_matsubara(e1, beta, ntau), eq.free_matsubara(e2, beta, ntau)
    wf, wb, _ = oracle.tau_weights(beta, ntau, 5)
    DG2 = np.einsum('ab,jbc->jac', e1 - e2, G2)
    err = np.abs(eq.convolution(G1, DG2, wf, wb) - (G1 - G2)).max(axis=(1, 2))
    assert err.max() < 2e-6 and err[8:-8].max() < 5e-9, (err.max(), err[8:-8].max())


def test_sigma_matches_the_mixed_self_energy_at_t0():
    rng = np.random.default_rng(13)
    N, beta, ntau = 3, 2.0, 7
    a = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    e, V = np.linalg.eigh(0.5 * (a + a.conj().T))
    J = ntau - 1
    mat = np.stack([(V * (-np.exp(-e * j * beta / J) / (1 + np.exp(-beta * e)))) @ V.conj().T
                    for j in range(ntau)])
    u = np.array([0.7, 1.1, 0.4])
    SM = eq.sigma_matsubara(mat, u)
    tv0 = np.stack([-1j * mat[J - j] for j in range(ntau)])
    kp = (-tv0[0].conj().T)[None, None]
    G = oracle.Green(kp, np.full((1, N, N), 0) + (-1j * np.eye(N))[None], tv0[None], mat)
    stv = oracle.sigma_row(G, u, 0)[2]
    np.testing.assert_allclose(stv, np.stack([-1j * SM[J - j] for j in range(ntau)]),
                               atol=1e-14, rtol=0)


def test_atomic_limit_of_second_order():
    U, beta, ntau = 1.0, 2.0, 129
    u = np.array([U])
    G0 = eq.free_matsubara(np.zeros((1, 1)), beta, ntau)
    S = eq.sigma_matsubara(G0, u)
    np.testing.assert_allclose(S, -U * U / 8, atol=1e-15)
    wf, wb, _ = oracle.tau_weights(beta, ntau, 5)
    G = G0.copy()
    for _ in range(200):
        Gn = G0 + eq.convolution(G0, eq.convolution(S, G, wf, wb), wf, wb)
        if np.abs(Gn - G).max() < 1e-15:
            break
        G = Gn
    ref = 0.5 * (scalar_free(U / 2, beta, ntau) + scalar_free(-U / 2, beta, ntau))
    np.testing.assert_allclose(G[:, 0, 0], ref, atol=1e-8, rtol=0)   # end intervals: h^3


def test_no_interaction_is_free():
    h0 = synth.tight_binding(4)
    G, info = eq.solve(h0, 0.0, 0.3, 4.0, 17)
    assert info["iterations"] == 1
    np.testing.assert_array_equal(G.real, eq.free_matsubara(h0 - 0.3 * np.eye(4), 4.0, 17))
    assert np.abs(G.imag).max() == 0


def test_half_filling():
    N, U, beta, ntau = 6, 1.5, 6.0, 129
    G, info = eq.solve(synth.tight_binding(N), U, U / 2, beta, ntau)
    assert info["change"] < 1e-13
    np.testing.assert_allclose(-np.diag(G[-1]).real, 0.5, atol=1e-6)
    # away from half filling the densities move the other way
    G2, _ = eq.solve(synth.tight_binding(N), U, U / 2 - 0.5, beta, ntau)
    assert np.all(-np.diag(G2[-1]).real < 0.47)


def test_solution_satisfies_equation_of_motion():
    N, U, beta, ntau = 3, 1.0, 4.0, 513
    h0 = synth.tight_binding(N) + np.diag([0.3, -0.1, 0.2])
    u = np.full(N, U)
    G, _ = eq.solve(h0, u, 0.4, beta, ntau)
    G = G.real
    wf, wb, _ = oracle.tau_weights(beta, ntau, 5)
    rhs = np.einsum('ab,jbc->jac', eq.fock(G, h0, u, 0.4), G) + \
        eq.convolution(eq.sigma_matsubara(G, u), G, wf, wb)
    h = beta / (ntau - 1)
    j = np.arange(2, ntau - 2)
    dG = (G[j - 2] - 8 * G[j - 1] + 8 * G[j + 1] - G[j + 2]) / (12 * h)
    np.testing.assert_allclose(-dG, rhs[j], atol=2e-6, rtol=0)
    # the interaction term is far above that tolerance
    assert np.abs(eq.convolution(eq.sigma_matsubara(G, u), G, wf, wb)).max() > 1e-2


def test_equilibrium_is_stationary_under_propagation():
    N, U, beta, ntau, nt = 3, 1.0, 2.0, 33, 21
    h0 = synth.tight_binding(N) + np.diag([0.3, -0.1, 0.2])
    u = np.full(N, U)
    G, _ = eq.solve(h0, u, 0.4, beta, ntau)
    t = np.linspace(0.0, 1.0, nt)
    order = np.full(nt, 5)

    def drift(mat):
        P = op.Problem(t=t, order=order, h0=h0, ntau=ntau, beta=beta, mat=mat, iters=3)
        with torch.no_grad():
            _, S = op.propagate(P, torch.tensor(U, dtype=torch.float64),
                                torch.tensor(0.0, dtype=torch.float64))
        return max(float((S.col[n][n] - S.col[0][0]).abs().max()) for n in range(nt))

    free = eq.free_matsubara(eq.fock(G.real, h0, u, 0.4), beta, ntau).astype(np.complex128)
    assert drift(G) < 3e-5
    assert drift(free) > 3e-3
