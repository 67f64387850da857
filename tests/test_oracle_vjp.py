"""Pins for the oracle's adjoints: the dot-product identity (the collision is real-linear in
each argument), exact five-point derivatives of the self-energy (a cubic polynomial in the
perturbation), and central finite differences with h = 1e-6."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import pack_kp, random_symmetric_full


def rdot(a, b):
    """Real inner product Re sum conj(a) b (PyTorch's complex-gradient pairing)."""
    return float(np.real(np.vdot(np.asarray(a).ravel(), np.asarray(b).ravel())))


def setup(N=2, nt=12, ntau=9, seed=0):
    rng = np.random.default_rng(seed)
    rnd = lambda *s: rng.normal(size=s) + 1j * rng.normal(size=s)
    G = oracle.Green(rnd(nt, nt, N, N), rnd(nt, N, N), rnd(nt, ntau, N, N), rnd(ntau, N, N))
    t, order = synth.grid(seed, nt, 0.02, 0.08, 3, 6)
    W = oracle.Weights.build(t, order, 3.0, ntau, 5)
    return rng, rnd, G, W


@pytest.mark.parametrize("m0,m1,flags", [(0, 12, oracle.F_ALL), (3, 9, oracle.F_ALL),
                                         (5, 6, oracle.F_IR), (0, 7, oracle.F_IL | oracle.F_JTV),
                                         (0, 12, oracle.F_ALL | oracle.F_GREATER),
                                         (3, 9, oracle.F_IR | oracle.F_IL | oracle.F_GREATER),
                                         (5, 6, oracle.F_IR | oracle.F_GREATER),
                                         (0, 7, oracle.F_IL | oracle.F_GREATER)])
def test_collision_adjoint_dot_product(m0, m1, flags):
    """Exact adjoint: Re<cot, I(dG)> = Re<gG, dG> and Re<cot, I(dSigma)> = Re<gSigma, dSigma>
    (the integrals are real-linear in G for fixed Sigma and in Sigma for fixed G), for the lesser
    and the greater form of Eq. KBE2, with the forward oracle pinned on its own."""
    rng, rnd, G, W = setup()
    N, nt, ntau = G.N, G.nt, G.ntau
    n = nt - 1
    sig = (rnd(n + 1, N, N), rnd(n + 1, N, N), rnd(ntau, N, N))
    cot = (rnd(m1 - m0, N, N), rnd(m1 - m0, N, N), rnd(m1 - m0, N, N), rnd(ntau, N, N))
    gkp, grd, gtv, gmat, gret, gles, gstv = oracle.collision_vjp(G, sig, W, n, m0, m1, cot, flags)
    # linear in G: perturb all Green's-function arrays
    dG = oracle.Green(rnd(nt, nt, N, N), rnd(nt, N, N), rnd(nt, ntau, N, N), rnd(ntau, N, N))
    out = oracle.collision(dG, sig, W, n, m0, m1, flags)
    lhs = sum(rdot(c, o) for c, o in zip(cot, out))
    rhs = rdot(gkp, dG.kp) + rdot(grd, dG.rdiag) + rdot(gtv, dG.tv) + rdot(gmat, dG.mat)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1e-300) * 10, (lhs, rhs)
    # linear in Sigma
    dsig = (rnd(n + 1, N, N), rnd(n + 1, N, N), rnd(ntau, N, N))
    out = oracle.collision(G, dsig, W, n, m0, m1, flags)
    lhs = sum(rdot(c, o) for c, o in zip(cot, out))
    rhs = rdot(gret, dsig[0]) + rdot(gles, dsig[1]) + rdot(gstv, dsig[2])
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1e-300) * 10, (lhs, rhs)


def test_collision_vjp_accumulates_green():
    rng, rnd, G, W = setup()
    N, nt, ntau = G.N, G.nt, G.ntau
    n = nt - 1
    sig = (rnd(n + 1, N, N), rnd(n + 1, N, N), rnd(ntau, N, N))
    cot = (rnd(nt, N, N), rnd(nt, N, N), rnd(nt, N, N), rnd(ntau, N, N))
    base = (rnd(nt, nt, N, N), rnd(nt, N, N), rnd(nt, ntau, N, N), rnd(ntau, N, N))
    fresh = oracle.collision_vjp(G, sig, W, n, 0, nt, cot)
    acc = oracle.collision_vjp(G, sig, W, n, 0, nt, cot, grads=tuple(b.copy() for b in base))
    for f, a, b in zip(fresh[:4], acc[:4], base):
        np.testing.assert_allclose(a, b + f, rtol=1e-14, atol=1e-14)


def _sigma_setup(seed=1, N=3, nt=7, ntau=6):
    rng = np.random.default_rng(seed)
    les, gtr = random_symmetric_full(rng, N, nt)
    kp = pack_kp(les, gtr - les)
    rdiag = np.array([(gtr - les)[a, a] for a in range(nt)])
    tv = rng.normal(size=(nt, ntau, N, N)) + 1j * rng.normal(size=(nt, ntau, N, N))
    G = oracle.Green(kp, rdiag, tv)
    u = rng.uniform(0.5, 1.5, size=N)
    return rng, G, u


def _sigma_obj(G, u, n, gsig):
    return sum(rdot(g, s) for g, s in zip(gsig, oracle.sigma_row(G, u, n)))


@pytest.mark.parametrize("n", [6, 3, 0])
def test_sigma_vjp_exact_derivative(n):
    """f(eps) = Re<gSigma, Sigma(G + eps dG)> is a cubic polynomial in eps, so the five-point
    stencil f'(0) = [8(f(h)-f(-h)) - (f(2h)-f(-2h))]/(12h) is exact for any h."""
    rng, G, u = _sigma_setup()
    N, nt, ntau = G.N, G.nt, G.ntau
    rnd = lambda *s: rng.normal(size=s) + 1j * rng.normal(size=s)
    gsig = (rnd(n + 1, N, N), rnd(n + 1, N, N), rnd(ntau, N, N))
    gkp, grd, gtv, gu = oracle.sigma_row_vjp(G, u, n, gsig)
    dkp, drd, dtv = rnd(nt, nt, N, N), rnd(nt, N, N), rnd(nt, ntau, N, N)

    def f(eps):
        Ge = oracle.Green(G.kp + eps * dkp, G.rdiag + eps * drd, G.tv + eps * dtv)
        return _sigma_obj(Ge, u, n, gsig)

    h = 0.5
    d5 = (8 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12 * h)
    pred = rdot(gkp, dkp) + rdot(grd, drd) + rdot(gtv, dtv)
    assert abs(d5 - pred) < 1e-11 * max(1.0, abs(pred)), (d5, pred)
    # interaction: quadratic in u
    du = rng.normal(size=N)
    g = lambda eps: _sigma_obj(G, u + eps * du, n, gsig)
    d5u = (8 * (g(h) - g(-h)) - (g(2 * h) - g(-2 * h))) / (12 * h)
    assert abs(d5u - gu @ du) < 1e-11 * max(1.0, abs(d5u)), (d5u, gu @ du)


def test_sigma_vjp_central_difference():
    """Central finite differences with h = 1e-6 (the check a user would run)."""
    rng, G, u = _sigma_setup(seed=7, N=2, nt=6, ntau=5)
    N, nt, ntau = G.N, G.nt, G.ntau
    n = nt - 1
    rnd = lambda *s: rng.normal(size=s) + 1j * rng.normal(size=s)
    gsig = (rnd(n + 1, N, N), rnd(n + 1, N, N), rnd(ntau, N, N))
    gkp, grd, gtv, gu = oracle.sigma_row_vjp(G, u, n, gsig)
    dkp, drd, dtv = rnd(nt, nt, N, N), rnd(nt, N, N), rnd(nt, ntau, N, N)
    h = 1e-6

    def f(eps):
        Ge = oracle.Green(G.kp + eps * dkp, G.rdiag + eps * drd, G.tv + eps * dtv)
        return _sigma_obj(Ge, u, n, gsig)

    fd = (f(h) - f(-h)) / (2 * h)
    pred = rdot(gkp, dkp) + rdot(grd, drd) + rdot(gtv, dtv)
    assert abs(fd - pred) < 1e-7 * abs(pred)


def test_end_to_end_density_gradient_wrt_u():
    """d/dU of the (real) density-like functional Re sum_m Tr[I^R + I^< + I^]](n,m) c_m through
    Sigma = second Born of G: chain the two adjoints and compare with the exact stencil."""
    rng, G, u0 = _sigma_setup(seed=3, N=2, nt=8, ntau=5)
    N, nt, ntau = G.N, G.nt, G.ntau
    n = nt - 1
    t, order = synth.grid(3, nt, 0.02, 0.08, 3, 6)
    W = oracle.Weights.build(t, order, 2.0, ntau, 5)
    cot = tuple(rng.normal(size=(k, N, N)) + 1j * rng.normal(size=(k, N, N))
                for k in (nt, nt, nt, ntau))

    def L(U):
        sig = oracle.sigma_row(G, U * u0, n)
        return sum(rdot(c, o) for c, o in zip(cot, oracle.collision(G, sig, W, n)))

    sig = oracle.sigma_row(G, u0, n)
    *_, gret, gles, gstv = oracle.collision_vjp(G, sig, W, n, 0, nt, cot)
    _, _, _, gu = oracle.sigma_row_vjp(G, u0, n, (gret, gles, gstv))
    dLdU = gu @ u0  # u = U * u0
    h = 0.25
    d5 = (8 * (L(1 + h) - L(1 - h)) - (L(1 + 2 * h) - L(1 - 2 * h))) / (12 * h)
    assert abs(d5 - dLdU) < 1e-11 * max(1.0, abs(d5))


@pytest.mark.parametrize("N,nt,ntau,m0,m1,flags", [
    (2, 12, 5, 0, 12, oracle.F_ALL),
    (3, 10, 4, 2, 8, oracle.F_ALL),
    (2, 9, 0, 1, 9, oracle.F_IR | oracle.F_IL),
    (3, 10, 4, 0, 10, oracle.F_ALL | oracle.F_GREATER),
    (2, 11, 6, 3, 9, oracle.F_IR | oracle.F_IL | oracle.F_GREATER),
    (1, 8, 5, 0, 8, oracle.F_ITV | oracle.F_JTV),
])
def test_gradient_rounding_scales_bound_the_gradients(N, nt, ntau, m0, m1, flags):
    """The per-block rounding scales the GPU adjoint tests use (sum over the terms that read a
    block of |c| and the norms of the other two factors) bound the norm of every gradient block
    of the oracle: a term the scales leave out would show as a block above its scale."""
    from tests.cases import Case, bnorm, vjp_scales
    case = Case(N=N, nt=nt, ntau=ntau, beta=2.0 if ntau else 0.0, seed=30 + N)
    t, order, kp, rd, tv, mat = case.host()
    n = nt - 1
    W = oracle.Weights.build(t, order, case.beta, ntau, case.tau_order)
    sig = synth.sigma_row(case.seed, N, n, ntau, t)
    M = m1 - m0
    cot = [synth.normal(3, k, (M, N, N)) for k in range(3)] + [synth.normal(3, 3, (ntau, N, N))]
    cot = [c if flags & (1 << k) else None for k, c in enumerate(cot)]
    full = [c if c is not None else np.zeros_like(z) for c, z in
            zip(cot, [np.zeros((M, N, N))] * 3 + [np.zeros((ntau, N, N))])]
    ref = oracle.collision_vjp(oracle.Green(kp, rd, tv, mat), sig, W, n, m0, m1, full, flags)
    S = vjp_scales(kp, rd, tv, mat, sig, W, n, m0, m1, cot, flags)
    for name, g in zip(["kp", "rdiag", "tv", "mat", "ret", "les", "stv"], ref):
        if g.size == 0:
            continue
        assert np.all(bnorm(g) <= S[name] * (1 + 1e-9) + 1e-300), name


@pytest.mark.parametrize("N,n", [(2, 7), (3, 0), (1, 5)])
def test_sigma_gradient_rounding_scales_bound_the_gradients(N, n):
    from tests.cases import Case, bnorm, sigma_vjp_scales
    case = Case(N=N, nt=9, ntau=6, beta=2.0, seed=50 + N)
    t, order, kp, rd, tv, mat = case.host()
    u = np.linspace(0.7, 1.3, N)
    gsig = (synth.normal(4, 0, (n + 1, N, N)), synth.normal(4, 1, (n + 1, N, N)),
            synth.normal(4, 2, (6, N, N)))
    gk, gr, gt, _ = oracle.sigma_row_vjp(oracle.Green(kp, rd, tv, mat), u, n, gsig)
    S_kp, S_rd, S_tv = sigma_vjp_scales(kp, rd, tv, u, n, gsig)
    assert np.all(bnorm(gk) <= S_kp * (1 + 1e-9) + 1e-300)
    assert np.all(bnorm(gr) <= S_rd * (1 + 1e-9) + 1e-300)
    assert np.all(bnorm(gt) <= S_tv * (1 + 1e-9) + 1e-300)
