"""Test-side helpers: building Green's functions with known structure.

These construct inputs (closed-form free-fermion Green's functions, random
symmetric full two-time arrays) and pack them into the KP storage.  They hold
no part of the method's arithmetic under test.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def expm_h(h: np.ndarray, z: complex) -> np.ndarray:
    """exp(z h) for Hermitian h via its eigendecomposition."""
    e, v = np.linalg.eigh(h)
    return (v * np.exp(z * e)) @ v.conj().T


def fermi(h: np.ndarray, beta: float) -> np.ndarray:
    e, v = np.linalg.eigh(h)
    return (v * (1.0 / (np.exp(beta * e) + 1.0))) @ v.conj().T


def tight_binding(N: int, hop: float = -1.0) -> np.ndarray:
    h = np.zeros((N, N))
    for i in range(N - 1):
        h[i, i + 1] = h[i + 1, i] = hop
    return h


def random_hermitian(rng, N, scale=1.0):
    a = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    return scale * 0.5 * (a + a.conj().T)


class FreeSystem:
    """Non-interacting Green's functions of a Hermitian h (closed forms):
    G^R(t,t') = -i e^{-ih(t-t')}, G^<(t,t') = i e^{-iht} rho e^{iht'},
    G^](t,tau) = i e^{-iht} f e^{h tau}, G^M(tau) = -e^{-h tau}(1 - f) (0 < tau < beta),
    with rho = f = Fermi function at inverse temperature beta."""

    def __init__(self, h, beta=None, rho=None):
        self.h = np.asarray(h, np.complex128)
        self.N = self.h.shape[0]
        self.beta = beta
        if rho is None:
            rho = fermi(self.h, beta)
        self.rho = rho

    def ret(self, t, tp):
        return -1j * expm_h(self.h, -1j * (t - tp))

    def les(self, t, tp):
        return 1j * expm_h(self.h, -1j * t) @ self.rho @ expm_h(self.h, 1j * tp)

    def mixed(self, t, tau):
        return 1j * expm_h(self.h, -1j * t) @ self.rho @ expm_h(self.h, tau)

    def matsubara(self, tau):
        return -expm_h(self.h, -tau) @ (np.eye(self.N) - self.rho)

    def kp(self, t):
        nt = len(t)
        N = self.N
        kp = np.zeros((nt, nt, N, N), np.complex128)
        U = [expm_h(self.h, -1j * x) for x in t]
        for a in range(nt):
            for b in range(nt):
                if a <= b:
                    kp[a, b] = 1j * U[a] @ self.rho @ U[b].conj().T
                else:
                    kp[a, b] = -1j * U[a] @ U[b].conj().T
        return kp

    def rdiag(self, nt):
        return np.broadcast_to(-1j * np.eye(self.N), (nt, self.N, self.N)).copy()

    def tv(self, t, taus):
        return np.array([[self.mixed(x, tau) for tau in taus] for x in t])

    def mat(self, taus):
        """mat[j] = G^M(tau_j); endpoints are the one-sided limits 0+ and beta-."""
        return np.array([self.matsubara(tau) for tau in taus])


def pack_kp(les_full, ret_full):
    """KP storage from full two-time arrays: upper (incl. diagonal) = G^<, strictly lower = G^R."""
    nt = les_full.shape[0]
    kp = np.empty_like(les_full)
    for a in range(nt):
        for b in range(nt):
            kp[a, b] = les_full[a, b] if a <= b else ret_full[a, b]
    return kp


def random_symmetric_full(rng, N, nt):
    """Random full G^<(a,b), G^>(a,b) for all pairs obeying G^<>(a,b) = -G^<>(b,a)^dagger and
    G^>(a,a) - G^<(a,a) = -i (so the equal-time retarded value is -i)."""
    def draw():
        return rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    les = np.empty((nt, nt, N, N), np.complex128)
    gtr = np.empty((nt, nt, N, N), np.complex128)
    for a in range(nt):
        for b in range(a, nt):
            x, y = draw(), draw()
            if a == b:
                x = 0.5 * (x - x.conj().T)
                y = x - 1j * np.eye(N)
            les[a, b], gtr[a, b] = x, y
            les[b, a], gtr[b, a] = -x.conj().T, -y.conj().T
    return les, gtr


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)
