"""GPU parity on structured inputs and at 64-bit element offsets.

* The free tight-binding family at 16 orbitals (the headline chain: open, hopping -1, on-site 0):
  G is the non-interacting Green's function of h, in closed form.  With the self-energy row taken
  from the same free functions the history integrals have closed forms that hold for any weights
  (only the weight sums t_n, t_m and beta enter), so the matrix-core path is checked against exact
  values as well as against the oracle.  With Sigma = second Born of that G, against the oracle.
* Element offsets beyond 2^31: a 16-orbital history stored with a row stride of 30000 blocks, so
  kp offsets reach 2.3e9 elements (3.7e10 bytes), forward, adjoint and the Sigma row.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.cases import (Case, assert_blocks_close, bnorm, device_green, device_weights, scales,
                         to_dev, to_host, vjp_scales)
from tests.helpers import tight_binding

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


class FreeEig:
    """Free-fermion Green's functions of a real symmetric h evaluated in its eigenbasis, so that
    the large and small exponentials of the thermal branch never meet in a matrix product:
    G^R(t,t') = -i e^{-ih(t-t')}, G^<(t,t') = i e^{-iht} f e^{iht'}, G^](t,tau) = i e^{-iht} f
    e^{h tau}, G^M(tau) = -e^{-h tau}(1 - f), f the Fermi function at beta."""

    def __init__(self, h, beta):
        self.e, self.v = np.linalg.eigh(h)
        self.f = 1.0 / (np.exp(beta * self.e) + 1.0)
        self.beta = beta

    def _m(self, d):
        return ((self.v * d) @ self.v.T).astype(np.complex128)

    def ret(self, t, tp):
        return self._m(-1j * np.exp(-1j * self.e * (t - tp)))

    def les(self, t, tp):
        return self._m(1j * np.exp(-1j * self.e * (t - tp)) * self.f)

    def mixed(self, t, tau):
        return self._m(1j * np.exp(-1j * self.e * t + self.e * tau) * self.f)

    def matsubara(self, tau):
        return self._m(-np.exp(-self.e * tau) * (1.0 - self.f))

    def storage(self, t, ntau):
        nt, N = len(t), len(self.e)
        kp = np.empty((nt, nt, N, N), np.complex128)
        for a in range(nt):
            for b in range(nt):
                kp[a, b] = self.les(t[a], t[b]) if a <= b else self.ret(t[a], t[b])
        rd = np.broadcast_to(-1j * np.eye(N), (nt, N, N)).copy()
        taus = np.linspace(0.0, self.beta, ntau)
        tv = np.array([[self.mixed(x, tau) for tau in taus] for x in t])
        mat = np.array([self.matsubara(tau) for tau in taus])
        return kp, rd, tv, mat


def _free_case(nt=160, ntau=40, beta=20.0, seed=1001):
    t, order = synth.grid(seed, nt, 0.005, 0.05, 3, 6)
    F = FreeEig(tight_binding(16), beta)
    kp, rd, tv, mat = F.storage(t, ntau)
    W = oracle.Weights.build(t, order, beta, ntau, 5)
    return t, order, F, kp, rd, tv, mat, W


def test_free_tight_binding_closed_forms_n16(gpu):
    """Sigma row = the free functions themselves (Sigma^R(t_n,t_s) = G^R, Sigma^< = G^<, Sigma^] =
    G^]): I^R(n,m) = t_n e^{-iht_n} f e^{iht_m}, I^<(n,m) = -t_m e^{-iht_n} f e^{iht_m} and
    I^](n,m) = -i beta e^{-iht_n} f (1 - f) e^{iht_m}, exact for any weights with the right sums;
    every output also against the oracle."""
    kbe = gpu
    t, order, F, kp, rd, tv, mat, W = _free_case()
    nt, ntau, n = len(t), tv.shape[1], len(t) - 1
    ret = np.array([kp[n, s] if s < n else rd[n] for s in range(n + 1)])
    les = np.array([-kp[s, n].conj().T for s in range(n + 1)])
    sig = (ret, les, tv[n].copy())
    _print("free N16: collision")
    out = kbe.collision(device_green(kp, rd, tv, mat), tuple(to_dev(x) for x in sig),
                        device_weights(W), n)
    ref = oracle.collision(oracle.Green(kp, rd, tv, mat), sig, W, n)
    sc = scales(kp, rd, tv, mat, sig, W, n, range(n + 1), range(ntau))
    for name, g, r in zip(("IR", "IL", "Itv", "Jtv"), out, ref):
        assert_blocks_close(to_host(g), r, sc[name], name)
    e, f = F.e, F.f
    for m in range(n + 1):
        ph = np.exp(-1j * e * (t[n] - t[m]))  # e^{-iht_n} ... e^{iht_m} in the eigenbasis
        want = {"IR": F._m(t[n] * ph * f), "IL": F._m(-t[m] * ph * f),
                "Itv": F._m(-1j * F.beta * ph * f * (1.0 - f))}
        for k, name in enumerate(("IR", "IL", "Itv")):
            d = np.linalg.norm(to_host(out[k])[m] - want[name])
            assert d <= 1e-12 * sc[name][m] + 1e-300, (name, m, d / sc[name][m])


def test_free_tight_binding_second_born_n16(gpu):
    """Sigma = second Born (U = 1) of the free tight-binding G at 16 orbitals: the Sigma row and the
    collision (matrix-core path) against the oracle, lesser and greater form."""
    kbe = gpu
    t, order, F, kp, rd, tv, mat, W = _free_case(nt=200, ntau=32)
    nt, ntau, n = len(t), tv.shape[1], len(t) - 1
    u = np.ones(16)
    Go = oracle.Green(kp, rd, tv, mat)
    Gd = device_green(kp, rd, tv, mat)
    _print("free N16 second Born: sigma row")
    sig_d = kbe.sigma_2b(Gd, to_dev(u), n)
    sig = oracle.sigma_row(Go, u, n)
    for g, r in zip(sig_d, sig):
        g = to_host(g)
        assert np.all(bnorm(g - r) <= 1e-13 * (bnorm(r) + 1e-300))
    for greater in (False, True):
        _print("free N16 second Born: collision, greater =", greater)
        fl = kbe.OUT_ALL | (kbe.GREATER if greater else 0)
        out = kbe.collision(Gd, tuple(to_dev(x) for x in sig), device_weights(W), n, 0, n + 1, fl)
        ref = oracle.collision(Go, sig, W, n, 0, n + 1,
                               oracle.F_ALL | (oracle.F_GREATER if greater else 0))
        sc = scales(kp, rd, tv, mat, sig, W, n, range(n + 1), range(ntau), greater=greater)
        for name, g, r in zip(("IR", "IL", "Itv", "Jtv"), out, ref):
            assert_blocks_close(to_host(g), r, sc[name], name)


def test_offsets_beyond_2_pow_31(gpu):
    """kp with a row stride of 30000 blocks at 16 orbitals: the last stored block starts at element
    (299 * 30000 + 299) * 256 = 2.3e9 > 2^31.  Only the used blocks are written; the Sigma row, the
    collision (all outputs) and its adjoint against the oracle on the compact storage."""
    import torch
    kbe = gpu
    N, nt, ntau, ldt = 16, 300, 24, 30000
    assert (nt - 1) * ldt * N * N > 2 ** 31
    case = Case(N=N, nt=nt, ntau=ntau, beta=4.0, seed=91, hmin=0.005, hmax=0.05)
    t, order, kp, rd, tv, mat = case.host()
    n = nt - 1
    W = oracle.Weights.build(t, order, case.beta, ntau, case.tau_order)
    Go = oracle.Green(kp, rd, tv, mat)
    dev = torch.device("cuda:0")
    _print("offsets: allocating two 37 GB strided arrays")
    kp_d = torch.empty((nt, ldt, N, N), dtype=torch.complex128, device=dev)
    kp_d[:, :nt] = to_dev(kp)
    Gd = kbe.Green(kp_d, to_dev(rd), to_dev(tv), to_dev(mat))
    u = np.linspace(0.8, 1.2, N)
    _print("offsets: sigma row")
    sig_d = kbe.sigma_2b(Gd, to_dev(u), n)
    sig = oracle.sigma_row(Go, u, n)
    for g, r in zip(sig_d, sig):
        assert np.all(bnorm(to_host(g) - r) <= 1e-13 * (bnorm(r) + 1e-300))
    _print("offsets: collision")
    Wd = device_weights(W)
    out = kbe.collision(Gd, sig_d, Wd, n)
    ref = oracle.collision(Go, sig, W, n)
    sc = scales(kp, rd, tv, mat, sig, W, n, range(n + 1), range(ntau))
    for name, g, r in zip(("IR", "IL", "Itv", "Jtv"), out, ref):
        assert_blocks_close(to_host(g), r, sc[name], name)
    _print("offsets: adjoint")
    cot = (synth.normal(12, 0, (nt, N, N)), synth.normal(12, 1, (nt, N, N)),
           synth.normal(12, 2, (nt, N, N)), synth.normal(12, 3, (ntau, N, N)))
    gG = kbe.Green(torch.zeros((nt, ldt, N, N), dtype=torch.complex128, device=dev),
                   torch.zeros((nt, N, N), dtype=torch.complex128, device=dev),
                   torch.zeros((nt, ntau, N, N), dtype=torch.complex128, device=dev),
                   torch.zeros((ntau, N, N), dtype=torch.complex128, device=dev))
    gG, gs = kbe.collision_vjp(Gd, sig_d, Wd, n, 0, nt, tuple(to_dev(c) for c in cot), kbe.OUT_ALL,
                               gG)
    rg = oracle.collision_vjp(Go, sig, W, n, 0, nt, cot)
    S = vjp_scales(kp, rd, tv, mat, sig, W, n, 0, nt, cot, oracle.F_ALL)
    got = [to_host(gG.kp[:, :nt]), to_host(gG.rdiag), to_host(gG.tv), to_host(gG.mat)] + \
        [to_host(x) for x in gs]
    for name, g, r in zip(["kp", "rdiag", "tv", "mat", "ret", "les", "stv"], got, rg):
        assert_blocks_close(g.reshape(-1, N, N), r.reshape(-1, N, N), S[name].ravel(), "g" + name)
    del kp_d, gG
    torch.cuda.empty_cache()
