"""GPU adjoints against the oracle's adjoints, autograd wrappers, and finite differences."""
import numpy as np
import pytest

import oracle
import synth
from tests.cases import Case, bnorm, device_green, device_weights, to_dev, to_host

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def vjp_case(kbe, case: Case, m0, m1, flags, extra=0, seed_cot=5):
    t, order, kp, rd, tv, mat = case.host()
    n = case.nt - 1
    W = oracle.Weights.build(t, order, case.beta, case.ntau, case.tau_order)
    sig = synth.sigma_row(case.seed, case.N, n, case.ntau, t)
    M, N = m1 - m0, case.N
    cot = (synth.normal(seed_cot, 0, (M, N, N)), synth.normal(seed_cot, 1, (M, N, N)),
           synth.normal(seed_cot, 2, (M, N, N)), synth.normal(seed_cot, 3, (case.ntau, N, N)))
    base = (synth.normal(seed_cot, 4, kp.shape), synth.normal(seed_cot, 5, rd.shape),
            synth.normal(seed_cot, 6, tv.shape), synth.normal(seed_cot, 7, mat.shape))
    ref = oracle.collision_vjp(oracle.Green(kp, rd, tv, mat), sig, W, n, m0, m1, cot, flags,
                               grads=tuple(b.copy() for b in base))
    Gd = device_green(kp, rd, tv, mat)
    gG = device_green(*base)
    sel = lambda k, x: to_dev(x) if flags & (1 << k) else None
    gG, gs = kbe.collision_vjp(Gd, tuple(to_dev(x) for x in sig), device_weights(W), n, m0, m1,
                               tuple(sel(k, c) for k, c in enumerate(cot)), flags | extra, gG)
    return ref, (gG, gs), base


@pytest.mark.parametrize("N,nt,ntau,m0,m1,flags,generic", [
    (2, 64, 64, 0, 64, oracle.F_ALL, False),
    (2, 64, 64, 10, 40, oracle.F_ALL, False),
    (8, 90, 20, 0, 90, oracle.F_ALL, False),
    (16, 170, 17, 0, 170, oracle.F_ALL, False),
    (16, 170, 17, 0, 170, oracle.F_ALL, True),
    (16, 150, 12, 33, 101, oracle.F_ALL, False),
    (16, 60, 8, 0, 60, oracle.F_IR | oracle.F_JTV, False),
    (16, 300, 40, 0, 300, oracle.F_ALL, False),
    (16, 9, 3, 0, 9, oracle.F_ALL, False),
    (16, 60, 8, 0, 60, oracle.F_ITV | oracle.F_JTV, False),
    (16, 60, 8, 0, 60, oracle.F_IR, False),
    (16, 260, 2, 0, 260, oracle.F_ALL, False),
    (5, 40, 0, 0, 40, oracle.F_IR | oracle.F_IL, False),
    (8, 300, 140, 0, 300, oracle.F_ALL, False),
    (8, 300, 140, 0, 300, oracle.F_ALL, True),
    (4, 600, 40, 100, 480, oracle.F_ALL, False),
    (3, 530, 260, 0, 530, oracle.F_ALL, False),
    (1, 1500, 300, 0, 1500, oracle.F_ALL, False),
    (6, 140, 30, 20, 120, oracle.F_ALL, False),
    (7, 100, 50, 0, 100, oracle.F_IR | oracle.F_JTV, False),
    (7, 100, 50, 10, 90, oracle.F_IL | oracle.F_ITV, False),
])
def test_collision_vjp_matches_oracle(gpu, N, nt, ntau, m0, m1, flags, generic):
    kbe = gpu
    print("vjp", N, nt, ntau, m0, m1, flags, generic, flush=True)
    case = Case(N=N, nt=nt, ntau=ntau, beta=3.0 if ntau else 0.0, seed=40 + N)
    ref, (gG, gs), _ = vjp_case(kbe, case, m0, m1, flags, kbe.FORCE_GENERIC if generic else 0)
    names = ["gkp", "grdiag", "gtv", "gmat", "gret", "gles", "gstv"]
    got = [gG.kp, gG.rdiag, gG.tv, gG.mat, gs[0], gs[1], gs[2]]
    for name, g, r in zip(names, got, ref):
        if r.size == 0:
            continue
        assert rel(to_host(g), r) < RTOL, name


@pytest.mark.parametrize("N,nt,ntau,m0,m1,flags", [
    (3, 40, 8, 0, 40, oracle.F_ALL),
    (16, 60, 8, 10, 50, oracle.F_ALL),
    (8, 50, 6, 0, 50, oracle.F_IR | oracle.F_IL),
    (5, 30, 0, 4, 25, oracle.F_IR),
    (2, 30, 6, 0, 30, oracle.F_IL | oracle.F_ITV),
    (1, 70, 4, 7, 64, oracle.F_ALL),
    (16, 300, 17, 0, 300, oracle.F_ALL),
    (16, 280, 9, 30, 270, oracle.F_ALL),
    (8, 300, 20, 7, 290, oracle.F_ALL),
])
def test_greater_form_vjp_matches_oracle(gpu, N, nt, ntau, m0, m1, flags):
    """kbe_collision_vjp with KBE_GREATER (vector-ALU kernels) against the oracle's adjoint of
    the greater form, every gradient array, accumulate mode."""
    kbe = gpu
    print("greater vjp", N, nt, ntau, m0, m1, flags, flush=True)
    case = Case(N=N, nt=nt, ntau=ntau, beta=3.0 if ntau else 0.0, seed=60 + N)
    ref, (gG, gs), _ = vjp_case(kbe, case, m0, m1, flags | oracle.F_GREATER)
    names = ["gkp", "grdiag", "gtv", "gmat", "gret", "gles", "gstv"]
    got = [gG.kp, gG.rdiag, gG.tv, gG.mat, gs[0], gs[1], gs[2]]
    for name, g, r in zip(names, got, ref):
        if r.size == 0:
            continue
        assert rel(to_host(g), r) < RTOL, name


@pytest.mark.parametrize("N", [4, 16])
def test_greater_form_vjp_overwrite_mode(gpu, N):
    """Overwrite mode with KBE_GREATER and I^R alone: the forward reads row m and column m of kp
    and rdiag[m] for m in the range (G^> assembled from both triangles); exactly those blocks are
    overwritten, including the lower-triangle ones that only the greater form's terms reach."""
    kbe = gpu
    nt, m0, m1 = 30, 10, 20
    case = Case(N=N, nt=nt, ntau=6, beta=2.0, seed=9)
    flags = oracle.F_IR | oracle.F_GREATER
    ref, (gG, _), base = vjp_case(kbe, case, m0, m1, flags, kbe.GRAD_OVERWRITE)
    read = np.zeros((nt, nt), bool)
    read[:, m0:m1] = True
    read[m0:m1, :] = True
    rd_read = np.zeros(nt, bool)
    rd_read[m0:m1] = True
    want_kp = np.where(read[:, :, None, None], ref[0] - base[0], base[0])
    want_rd = np.where(rd_read[:, None, None], ref[1] - base[1], base[1])
    assert rel(to_host(gG.kp), want_kp) < RTOL
    assert rel(to_host(gG.rdiag), want_rd) < RTOL


def test_collision_vjp_overwrite_mode(gpu):
    """KBE_GRAD_OVERWRITE writes exactly the blocks the forward reads (here: all of [0,n]^2 and
    tv rows 0..n) and leaves the rest of the arrays as they were."""
    kbe = gpu
    case = Case(N=16, nt=80, ntau=10, beta=2.0, seed=3)
    ref, (gG, gs), base = vjp_case(kbe, case, 0, 80, oracle.F_ALL, kbe.GRAD_OVERWRITE)
    # accumulate-mode reference minus the initial content = the overwrite result
    for g, r, b in zip([gG.kp, gG.rdiag, gG.tv, gG.mat], ref[:4], base):
        assert rel(to_host(g), r - b) < RTOL
    # a partial range: blocks nobody reads keep their initial values (generic gradient kernel
    # at N = 4, the padded MFMA one at N = 8)
    for N in (4, 8):
        case2 = Case(N=N, nt=30, ntau=6, beta=2.0, seed=4)
        ref2, (gG2, _), base2 = vjp_case(kbe, case2, 10, 20, oracle.F_IR | oracle.F_IL,
                                         kbe.GRAD_OVERWRITE)
        kp = to_host(gG2.kp)
        read = np.zeros((30, 30), bool)
        for m in range(10, 20):
            read[: m + 1, m] = True   # IR column part
            read[m, m + 1:] = True    # IR row part
            read[m, :m] = True        # IL
        assert np.array_equal(kp[~read], base2[0][~read])
        assert rel(kp[read], (ref2[0] - base2[0])[read]) < RTOL


@pytest.mark.parametrize("N,n", [(2, 63), (3, 0), (16, 45), (16, 0)])
def test_sigma_vjp_matches_oracle(gpu, N, n):
    kbe = gpu
    case = Case(N=N, nt=64 if N < 16 else 46, ntau=10, beta=2.0, seed=60 + N)
    t, order, kp, rd, tv, mat = case.host()
    u = np.linspace(0.7, 1.3, N)
    gsig = (synth.normal(9, 0, (n + 1, N, N)), synth.normal(9, 1, (n + 1, N, N)),
            synth.normal(9, 2, (case.ntau, N, N)))
    base = (synth.normal(9, 3, kp.shape), synth.normal(9, 4, rd.shape), synth.normal(9, 5, tv.shape))
    gu0 = np.arange(N, dtype=np.float64)
    rk, rr, rt, ru = oracle.sigma_row_vjp(oracle.Green(kp, rd, tv, mat), u, n, gsig,
                                         grads=tuple(b.copy() for b in base), gu=gu0.copy())
    gG = device_green(base[0], base[1], base[2], mat)
    gG, gu = kbe.sigma_2b_vjp(device_green(kp, rd, tv, mat), to_dev(u), n,
                              tuple(to_dev(x) for x in gsig), gG, to_dev(gu0.copy()))
    assert rel(to_host(gG.kp), rk) < RTOL
    assert rel(to_host(gG.rdiag), rr) < RTOL
    assert rel(to_host(gG.tv), rt) < RTOL
    assert rel(to_host(gu), ru) < 1e-12


@pytest.mark.parametrize("greater", [False, True])
def test_autograd_wrappers_and_finite_differences(gpu, greater):
    """Loss = Re sum c * (IR + IL + Itv) at the last rows, through Sigma = second Born(G, U):
    torch autograd over the two Functions equals the oracle's chained adjoint, and dL/dU agrees
    with a central finite difference (h = 1e-6) of the GPU forward; lesser and greater form."""
    import torch
    kbe = gpu
    case = Case(N=8, nt=60, ntau=12, beta=3.0, seed=70)
    t, order, kp, rd, tv, mat = case.host()
    n, m0, m1 = 59, 40, 60
    W = oracle.Weights.build(t, order, case.beta, case.ntau)
    Wd = device_weights(W)
    cot = [synth.normal(2, k, (m1 - m0, 8, 8)) for k in range(3)] + [synth.normal(2, 3, (12, 8, 8))]
    ct = [to_dev(c) for c in cot]

    def loss_gpu(U, kp_t):
        u = U * torch.ones(8, dtype=torch.float64, device="cuda")
        ret, les, stv = kbe.KBESigma2B.apply(kp_t, to_dev(rd), to_dev(tv), to_dev(mat), u, n)
        outs = kbe.KBECollision.apply(kp_t, to_dev(rd), to_dev(tv), to_dev(mat), ret, les, stv,
                                      Wd, n, m0, m1, greater)
        return sum(torch.real(torch.sum(torch.conj(c) * o)) for c, o in zip(ct, outs))

    U = torch.tensor(1.7, dtype=torch.float64, device="cuda", requires_grad=True)
    kp_t = to_dev(kp).requires_grad_(True)
    L = loss_gpu(U, kp_t)
    L.backward()
    # oracle chain
    Go = oracle.Green(kp, rd, tv, mat)
    u = np.full(8, 1.7)
    sig = oracle.sigma_row(Go, u, n)
    flags = oracle.F_ALL | (oracle.F_GREATER if greater else 0)
    gk, grd, _, _, gret, gles, gstv = oracle.collision_vjp(Go, sig, W, n, m0, m1, cot, flags)
    gk2, _, _, gu = oracle.sigma_row_vjp(Go, u, n, (gret, gles, gstv), grads=(gk, grd.copy(),
                                                                             np.zeros_like(tv)))
    assert rel(to_host(kp_t.grad), gk2) < 1e-12
    assert abs(U.grad.item() - gu.sum()) < 1e-12 * abs(gu.sum())
    h = 1e-6
    with torch.no_grad():
        kp0 = to_dev(kp)
        fd = (loss_gpu(torch.tensor(1.7 + h, dtype=torch.float64, device="cuda"), kp0)
              - loss_gpu(torch.tensor(1.7 - h, dtype=torch.float64, device="cuda"), kp0)) / (2 * h)
    assert abs(fd.item() - U.grad.item()) < 1e-7 * abs(U.grad.item())
