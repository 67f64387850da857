"""CPU oracle of the interacting equilibrium initial state (TEST INFRASTRUCTURE ONLY: only tests/,
the smoke check and the benchmark's CPU baseline use it; the GPU library shares no code with it).

The propagations start from the Matsubara Green's function G^M(tau) on the uniform tau grid
tau_j = j beta / J (j = 0..J, ntau = J + 1 points; tau_0 = 0+, tau_J = beta-).  The paper takes
G^M as given (Sec. "Kadanoff Baym Equations"); for an interacting system it is the solution of the
Matsubara Dyson equation, which follows from Eq. KBE3 and the boundary conditions of Eq. BC in
equilibrium: G^](t, tau) then depends on t + i tau only, so i d/dt G^] = d/dtau G^], and at t = 0
(with G^](0, tau) = i G^M(-tau), Sigma^](0, tau) = i Sigma^M(-tau)) Eq. KBE3 becomes

    -dG^M/dtau (tau) = eps G^M(tau) + int_0^beta Sigma^M(u) G^M(tau - u) du,

G^M and Sigma^M antiperiodic, with the jump G^M(0+) + G^M(beta-) = -1 (the free solution
-exp(-eps tau)(1 - f(eps)) has it).  Its integral form is the Dyson equation

    G^M = G0 + G0 * Sigma^M * G^M,   (A * B)(tau) = int_0^beta A(tau - u) B(u) du,

with G0 the free Matsubara function of eps.  Here, for the local interaction of the propagation:
  * eps = h0 + diag(u_i n_i) - mu, n_i = -G^M_ii(beta-) (the Hartree shift of Eq. eps at t = 0,
    with G^<(0,0) = i rho; mu = u / 2 keeps a particle-hole symmetric chain at half filling);
  * Sigma^M_ij(tau) = u_i u_j G^M_ij(tau)^2 G^M_ji(beta - tau): the second-Born Sigma^] of the
    propagation at t = 0 through Sigma^](0, tau) = i Sigma^M(-tau) and antiperiodicity;
  * every * is split at u = tau (where G^M(tau - u) jumps): the forward rule over [0, tau_j] with
    A(tau_{j-l}), minus the backward rule over [tau_j, beta] with A(tau_{J+j-l}) (antiperiodic
    continuation), the tau rules of the propagation (oracle.tau_weights).
The self-consistency is a fixed point on G^M with linear mixing, from the free solution of h0,
until the largest change is below tol.  Plain numpy; eigendecompositions by numpy.linalg.eigh.
"""
from __future__ import annotations

import numpy as np

import oracle as _orc


def free_matsubara(eps: np.ndarray, beta: float, ntau: int) -> np.ndarray:
    """G0(tau_j) = -exp(-eps tau_j)(1 - f(eps)) for real symmetric eps, in its eigenbasis:
    -exp(-e tau) / (1 + exp(-beta e)) for e >= 0, -exp(e (beta - tau)) / (1 + exp(beta e)) else."""
    e, V = np.linalg.eigh(eps)
    J = ntau - 1
    out = np.empty((ntau,) + eps.shape)
    for j in range(ntau):
        tau = j * beta / J
        ep, en = np.maximum(e, 0.0), np.minimum(e, 0.0)   # each branch sees its own sign only
        x = np.where(e >= 0, -np.exp(-ep * tau) / (1.0 + np.exp(-beta * ep)),
                     -np.exp(en * (beta - tau)) / (1.0 + np.exp(beta * en)))
        out[j] = (V * x) @ V.T
    return out


def convolution(A: np.ndarray, B: np.ndarray, wf: np.ndarray, wb: np.ndarray) -> np.ndarray:
    """(A * B)(tau_j) = int_0^beta A(tau_j - u) B(u) du with A antiperiodic: for u < tau_j the
    argument is tau_{j-l}; for u > tau_j, A(tau_j - u) = -A(tau_{J+j-l})."""
    ntau = A.shape[0]
    J = ntau - 1
    out = np.zeros(A.shape, np.result_type(A, B))
    for j in range(ntau):
        lo = np.arange(0, j + 1)
        out[j] += np.einsum('l,lab,lbc->ac', wf[j, lo], A[j - lo], B[lo])
        hi = np.arange(j, ntau)
        out[j] -= np.einsum('l,lab,lbc->ac', wb[j, hi], A[J + j - hi], B[hi])
    return out


def sigma_matsubara(G: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Sigma^M_ij(tau_j) = u_i u_j G_ij(tau_j)^2 G_ji(beta - tau_j) (beta - tau_j = tau_{J-j})."""
    return (u[:, None] * u[None, :]) * G ** 2 * np.transpose(G[::-1], (0, 2, 1))


def fock(G: np.ndarray, h0: np.ndarray, u: np.ndarray, mu: float) -> np.ndarray:
    n = -np.real(np.diag(G[-1]))
    return h0 + np.diag(u * n) - mu * np.eye(len(u))


def solve(h0, u, mu: float, beta: float, ntau: int, tau_order: int = 5, mix: float = 0.5,
          tol: float = 1e-13, maxit: int = 1000):
    """G^M [ntau][N][N] (complex128) and {"iterations", "change"}."""
    h0 = np.asarray(h0, np.float64)
    u = np.broadcast_to(np.asarray(u, np.float64), (h0.shape[0],)).copy()
    wf, wb, _ = _orc.tau_weights(beta, ntau, tau_order)
    G = free_matsubara(h0 - mu * np.eye(len(u)), beta, ntau)
    change = np.inf
    for it in range(1, maxit + 1):
        G0 = free_matsubara(fock(G, h0, u, mu), beta, ntau)
        Gn = G0 + convolution(G0, convolution(sigma_matsubara(G, u), G, wf, wb), wf, wb)
        change = float(np.abs(Gn - G).max())
        G = (1.0 - mix) * G + mix * Gn
        if change < tol:
            break
    return G.astype(np.complex128), {"iterations": it, "change": change}
