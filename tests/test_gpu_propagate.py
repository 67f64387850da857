"""The fixed-grid propagation on the GPU (kbe_propagate, kbe_propagate_vjp) against the oracle
(oracle/propagate.py): the whole solution and the densities element by element, the gradients
dL/dU and dL/dA of a density loss against the oracle's reverse-mode derivatives and against
central finite differences of the GPU forward, conservation of the particle number, and the
differentiation workload at full size (8 orbitals, 1024 points, 256 tau points, U = 2)."""
import numpy as np
import pytest
import torch

import synth
from oracle import propagate as op
from tests.helpers import tight_binding

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def free_matsubara(h, beta, ntau):
    e, v = np.linalg.eigh(h)
    f = 1.0 / (np.exp(beta * e) + 1.0)
    taus = np.linspace(0.0, beta, ntau)
    return np.array([(v * (-np.exp(-e * x) * (1.0 - f))) @ v.T for x in taus]).astype(np.complex128)


def setup(N, nt, ntau, iters, seed=5, beta=2.0, hmin=0.02, hmax=0.08, omin=3, omax=5):
    t, order = synth.grid(seed, nt, hmin, hmax, omin, omax)
    h0 = tight_binding(N)
    mat = free_matsubara(h0, beta, ntau) if ntau else None
    rho0 = None if ntau else np.diag(np.linspace(0.2, 0.8, N))
    P = op.Problem(t=t, order=order, h0=h0, ntau=ntau, beta=beta, mat=mat, rho0=rho0, iters=iters)
    return t, order, h0, mat, rho0, P


def gpu_prop(kbe, t, order, h0, ntau, beta, mat, rho0, iters):
    return kbe.Propagation(t, order, h0, ntau=ntau, beta=beta, tau_order=5, mat=mat, rho0=rho0,
                           iters=iters)


# Bar: the two sides compute the same discrete map with the same inputs; their sums differ in
# order (matrix cores, chunked reductions), i.e. at rounding, ~1e-16 of each step's terms, and the
# propagation carries those differences forward through <= 16 steps with a Lipschitz factor of
# order one per step (h ||d f / d y|| < 1 here).  1e-12 of the solution's norm leaves two orders of
# magnitude for that growth.
RTOL = 1e-12


@pytest.mark.parametrize("N,nt,ntau,iters", [(2, 16, 6, 2), (3, 14, 0, 1), (4, 12, 5, 3),
                                             (8, 10, 4, 2), (16, 8, 3, 2), (1, 16, 4, 2)])
def test_propagation_matches_oracle(gpu, N, nt, ntau, iters):
    kbe = gpu
    _print("propagate", N, nt, ntau, iters)
    U, A = 1.3, 0.7
    t, order, h0, mat, rho0, P = setup(N, nt, ntau, iters)
    pr = gpu_prop(kbe, t, order, h0, ntau, 2.0, mat, rho0, iters)
    dens = pr.run(torch.full((N,), U, dtype=torch.float64, device="cuda"), A).cpu().numpy()
    dref, S = op.propagate(P, torch.tensor(U, dtype=torch.float64),
                           torch.tensor(A, dtype=torch.float64))
    kp_ref, tv_ref = op.storage(S)
    kp = pr.G.kp.cpu().numpy()
    err = np.linalg.norm(kp - kp_ref) / np.linalg.norm(kp_ref)
    _print("  kp relative error %.3e" % err)
    assert err < RTOL
    if ntau:
        etv = np.linalg.norm(pr.G.tv.cpu().numpy() - tv_ref) / np.linalg.norm(tv_ref)
        _print("  tv relative error %.3e" % etv)
        assert etv < RTOL
    assert np.abs(dens - dref.detach().numpy()).max() < RTOL * np.abs(dref.detach().numpy()).max()
    np.testing.assert_array_equal(pr.G.rdiag.cpu().numpy(),
                                  np.broadcast_to(-1j * np.eye(N), (nt, N, N)))
    tr = dens.sum(axis=1)
    assert np.abs(tr - tr[0]).max() < 1e-13 * max(1.0, abs(tr[0]))


@pytest.mark.parametrize("N,nt,ntau,iters", [(2, 14, 6, 2), (3, 12, 0, 1), (4, 10, 5, 3)])
def test_propagation_gradients(gpu, N, nt, ntau, iters):
    """dL/dU (u_i = U) and dL/dA of L = sum over the last 5 steps of n_0: the GPU adjoint against
    the oracle's reverse mode and against central finite differences (h = 1e-6) of the GPU
    forward."""
    kbe = gpu
    _print("propagate vjp", N, nt, ntau, iters)
    U, A, last, h = 1.3, 0.6, 5, 1e-6
    c = np.zeros(N)
    c[0] = 1.0
    t, order, h0, mat, rho0, P = setup(N, nt, ntau, iters)
    pr = gpu_prop(kbe, t, order, h0, ntau, 2.0, mat, rho0, iters)
    gd = torch.zeros((nt, N), dtype=torch.float64, device="cuda")
    gd[-last:, 0] = 1.0

    def L(Uv, Av):
        d = pr.run(torch.full((N,), Uv, dtype=torch.float64, device="cuda"), Av)
        return float((d * gd).sum())

    L0 = L(U, A)
    gu, ga = pr.vjp(gd)
    gU, gA = float(gu.sum()), float(ga)
    Lr, gUr, gAr = op.loss_and_grad(P, U, A, c, last)
    _print("  dL/dU gpu %.15e oracle %.15e; dL/dA gpu %.15e oracle %.15e" % (gU, gUr, gA, gAr))
    assert abs(L0 - Lr) < 1e-12 * abs(Lr)
    assert abs(gU - gUr) < 1e-10 * abs(gUr)
    assert abs(gA - gAr) < 1e-10 * abs(gAr)
    fU = (L(U + h, A) - L(U - h, A)) / (2 * h)
    fA = (L(U, A + h) - L(U, A - h)) / (2 * h)
    _print("  finite differences dL/dU %.15e dL/dA %.15e" % (fU, fA))
    assert abs(fU - gU) < 1e-6 * abs(gU)
    assert abs(fA - gA) < 1e-6 * abs(gA)
    # per-orbital u: the GPU gradient vector against the oracle's
    ut = torch.full((N,), U, dtype=torch.float64, requires_grad=True)
    At = torch.tensor(A, dtype=torch.float64, requires_grad=True)
    d, _ = op.propagate(P, ut, At)
    (gvec,) = torch.autograd.grad((d[-last:, 0]).sum(), [ut])
    np.testing.assert_allclose(gu.cpu().numpy(), gvec.numpy(), rtol=1e-10,
                               atol=1e-10 * np.abs(gvec.numpy()).max())


def test_trace_loss_gradient_vanishes_on_gpu(gpu):
    """The total particle number is conserved, so its gradient is zero (to rounding)."""
    kbe = gpu
    N, nt, ntau = 3, 12, 5
    t, order, h0, mat, rho0, P = setup(N, nt, ntau, 2)
    pr = gpu_prop(kbe, t, order, h0, ntau, 2.0, mat, rho0, 2)
    d = pr.run(torch.full((N,), 1.1, dtype=torch.float64, device="cuda"), 0.9)
    gd = torch.zeros((nt, N), dtype=torch.float64, device="cuda")
    gd[-4:] = 1.0
    L0 = float((d * gd).sum())
    gu, ga = pr.vjp(gd)
    assert abs(float(gu.sum())) < 1e-12 * L0 and abs(float(ga)) < 1e-12 * L0


@pytest.mark.parametrize("U,ntau", [(1.0, 256), (2.0, 0)])
def test_differentiation_workload_full_size(gpu, U, ntau):
    """The differentiation workload: 8-site tight-binding chain, 1024 points with steps
    U[0.005, 0.05] and orders 3..6, beta = 10, pulse A = 1 at t = 2 with width 1, loss = n_0 over the
    last 32 steps; with the thermal branch (256 tau points, free thermal G^M) at U = 1, and at
    U = 2 without it (initial density matrix of the free thermal state): the free G^M is not an
    equilibrium of the U = 2 second-Born mixed branch, and that propagation grows without bound
    from t = 5.6 at any step size.  Checked: the first 8 steps against the oracle on the same grid
    prefix (the propagation is causal), particle-number conservation over the whole run, and
    dL/dU, dL/dA against central finite differences of the GPU forward."""
    from tests.helpers import fermi
    kbe = gpu
    N, nt, beta, A, last = 8, 1024, 10.0, 1.0, 32
    t, order = synth.grid(1003, nt, 0.005, 0.05, 3, 6)
    h0 = tight_binding(N)
    mat = free_matsubara(h0, beta, ntau) if ntau else None
    rho0 = None if ntau else fermi(h0, beta).real
    _print("full size U =", U, "ntau =", ntau, ": setup")
    pr = kbe.Propagation(t, order, h0, ntau=ntau, beta=beta, mat=mat, rho0=rho0, iters=2)
    gd = torch.zeros((nt, N), dtype=torch.float64, device="cuda")
    gd[-last:, 0] = 1.0
    u = lambda x: torch.full((N,), x, dtype=torch.float64, device="cuda")
    _print("full size: forward")
    d = pr.run(u(U), A).cpu().numpy()
    L0 = float((d[-last:, 0]).sum())
    tr = d.sum(axis=1)
    assert np.all(np.isfinite(d))
    assert np.abs(tr - tr[0]).max() < 1e-11 * abs(tr[0])
    assert np.abs(d[:, 0] - d[0, 0]).max() > 1e-2
    _print("full size: adjoint")
    gu, ga = pr.vjp(gd)
    gU, gA = float(gu.sum()), float(ga)
    kp8 = pr.G.kp[:8, :8].cpu().numpy()
    tv8 = pr.G.tv[:8].cpu().numpy() if ntau else None
    _print("full size: finite differences")
    Lf = lambda Uv, Av: float((pr.run(u(Uv), Av)[-last:, 0]).sum())
    # central differences with h = 1e-6; over 1024 steps the rounding noise of L (about 1e-13
    # of it) divided by 2h limits them to a few parts in 1e6 of these gradients, so they are also
    # checked with the fourth-order five-point stencil at h = 1e-3 (truncation ~ h^4 L^(5) / 30)
    h = 1e-6
    fU = (Lf(U + h, A) - Lf(U - h, A)) / (2 * h)
    fA = (Lf(U, A + h) - Lf(U, A - h)) / (2 * h)
    H = 1e-3
    five = lambda g: (8 * (g(H) - g(-H)) - (g(2 * H) - g(-2 * H))) / (12 * H)
    f5U = five(lambda d: Lf(U + d, A))
    f5A = five(lambda d: Lf(U, A + d))
    _print("  L %.15e dL/dU %.12e (fd %.12e, 5-point %.12e) dL/dA %.12e (fd %.12e, 5-point %.12e)"
           % (L0, gU, fU, f5U, gA, fA, f5A))
    assert abs(fU - gU) < 1e-5 * abs(gU)
    assert abs(fA - gA) < 1e-5 * abs(gA)
    assert abs(f5U - gU) < 1e-7 * abs(gU)
    assert abs(f5A - gA) < 1e-7 * abs(gA)
    _print("full size: oracle on the first 8 steps")
    P = op.Problem(t=t[:8], order=order[:8], h0=h0, ntau=ntau, beta=beta, mat=mat, rho0=rho0,
                   iters=2)
    dref, S = op.propagate(P, torch.tensor(U, dtype=torch.float64),
                           torch.tensor(A, dtype=torch.float64))
    kp_ref, tv_ref = op.storage(S)
    assert np.linalg.norm(kp8 - kp_ref) < RTOL * np.linalg.norm(kp_ref)
    if ntau:
        assert np.linalg.norm(tv8 - tv_ref) < RTOL * np.linalg.norm(tv_ref)
