"""GPU adjoints against the oracle's adjoints, autograd wrappers, and finite differences."""
import numpy as np
import pytest

import oracle
import synth
from tests.cases import (Case, assert_blocks_close, bnorm, device_green, device_weights, to_dev,
                         sigma_vjp_scales, to_host, vjp_scales)

pytestmark = pytest.mark.gpu

RTOL = 1e-12
NAMES = ["kp", "rdiag", "tv", "mat", "ret", "les", "stv"]


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def vjp_case(kbe, case: Case, m0, m1, flags, extra=0, seed_cot=5, base="zero"):
    """The GPU adjoint and the oracle's pure gradient (accumulated into zeros).  The GPU's
    Green's-function gradient arrays start from `base`: zeros (the accumulated result is then the
    pure gradient) or random N(0,1) values (to check that accumulation keeps them)."""
    t, order, kp, rd, tv, mat = case.host()
    n = case.nt - 1
    W = oracle.Weights.build(t, order, case.beta, case.ntau, case.tau_order)
    sig = synth.sigma_row(case.seed, case.N, n, case.ntau, t)
    M, N = m1 - m0, case.N
    cot = (synth.normal(seed_cot, 0, (M, N, N)), synth.normal(seed_cot, 1, (M, N, N)),
           synth.normal(seed_cot, 2, (M, N, N)), synth.normal(seed_cot, 3, (case.ntau, N, N)))
    shapes = (kp.shape, rd.shape, tv.shape, mat.shape)
    if base == "zero":
        b0 = tuple(np.zeros(s, np.complex128) for s in shapes)
    else:
        b0 = tuple(synth.normal(seed_cot, 4 + k, s) for k, s in enumerate(shapes))
    ref = oracle.collision_vjp(oracle.Green(kp, rd, tv, mat), sig, W, n, m0, m1, cot, flags)
    Gd = device_green(kp, rd, tv, mat)
    gG = device_green(*b0)
    sel = lambda k, x: to_dev(x) if flags & (1 << k) else None
    gG, gs = kbe.collision_vjp(Gd, tuple(to_dev(x) for x in sig), device_weights(W), n, m0, m1,
                               tuple(sel(k, c) for k, c in enumerate(cot)), flags | extra, gG)
    scale = vjp_scales(kp, rd, tv, mat, sig, W, n, m0, m1,
                       tuple(c if flags & (1 << k) else None for k, c in enumerate(cot)), flags)
    return ref, (gG, gs), b0, scale


def check_gradients(ref, got, base, scale):
    """Accumulate mode: every gradient array against base + the oracle's pure gradient (the
    self-energy gradients are overwritten), each block within RTOL of its rounding scale (R14
    applied to the adjoint; the final addition to the base adds the base's norm to the scale)
    and globally within RTOL.  With a zero base this is the bar on the pure gradient itself."""
    gG, gs = got
    arrays = [gG.kp, gG.rdiag, gG.tv, gG.mat, gs[0], gs[1], gs[2]]
    for k, (name, g, r) in enumerate(zip(NAMES, arrays, ref)):
        if r.size == 0:
            continue
        g = to_host(g)
        sc = scale[name]
        if k < 4:
            r = r + base[k]
            if name == "kp":
                nt = sc.shape[0]
                g, r, b = g[:, :nt], r[:, :nt], base[0][:, :nt]
            else:
                b = base[k]
            sc = sc + bnorm(b)
        assert_blocks_close(g.reshape(-1, *g.shape[-2:]), r.reshape(-1, *r.shape[-2:]),
                            sc.ravel(), "g" + name)


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
    ref, got, base, scale = vjp_case(kbe, case, m0, m1, flags,
                                     kbe.FORCE_GENERIC if generic else 0)
    check_gradients(ref, got, base, scale)


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
    ref, got, base, scale = vjp_case(kbe, case, m0, m1, flags | oracle.F_GREATER)
    check_gradients(ref, got, base, scale)


@pytest.mark.parametrize("N,nt,ntau,m0,m1,greater", [(16, 120, 10, 0, 120, False),
                                                   (8, 90, 12, 5, 80, True),
                                                   (3, 70, 6, 0, 70, False)])
def test_collision_vjp_accumulates_onto_existing_values(gpu, N, nt, ntau, m0, m1, greater):
    """Accumulate mode on random N(0,1) initial gradient arrays: the result is the initial
    values plus the pure gradient, to the bar of the final addition."""
    kbe = gpu
    case = Case(N=N, nt=nt, ntau=ntau, beta=3.0, seed=90 + N)
    flags = oracle.F_ALL | (oracle.F_GREATER if greater else 0)
    ref, got, base, scale = vjp_case(kbe, case, m0, m1, flags, base="random")
    check_gradients(ref, got, base, scale)


def check_overwrite(ref, gG, base, scale, read_kp, read_rd):
    """Overwrite mode: blocks the forward reads hold the pure gradient (the oracle's, accumulated
    into zeros) to the R14 bar; every other block keeps its initial value bit for bit."""
    nt = read_kp.shape[0]
    kp, rd = to_host(gG.kp)[:, :nt], to_host(gG.rdiag)
    want_kp, want_rd = ref[0][:, :nt], ref[1]
    assert np.array_equal(kp[~read_kp], base[0][:, :nt][~read_kp])
    assert np.array_equal(rd[~read_rd], base[1][~read_rd])
    assert_blocks_close(kp[read_kp], want_kp[read_kp], scale["kp"][read_kp], "gkp")
    assert_blocks_close(rd[read_rd], want_rd[read_rd], scale["rdiag"][read_rd], "grdiag")


@pytest.mark.parametrize("N,flags", [(4, oracle.F_IR), (6, oracle.F_IR), (8, oracle.F_IR),
                                     (16, oracle.F_IR), (6, oracle.F_IR | oracle.F_IL),
                                     (8, oracle.F_IR | oracle.F_IL),
                                     (16, oracle.F_IR | oracle.F_IL)])
def test_greater_form_vjp_overwrite_mode(gpu, N, flags):
    """Overwrite mode with KBE_GREATER: the forward reads row m and column m of kp and rdiag[m]
    for m in the range (G^> assembled from both triangles; I^< reads the left part of row m);
    exactly those blocks are overwritten, including the lower-triangle ones that only the greater
    form's terms reach, on the generic (N = 4), padded 8x8 (N = 6, 8) and 16x16 gradient
    kernels."""
    kbe = gpu
    nt, m0, m1 = 30, 10, 20
    print("greater overwrite", N, flags, flush=True)
    case = Case(N=N, nt=nt, ntau=6, beta=2.0, seed=9)
    ref, (gG, _), base, scale = vjp_case(kbe, case, m0, m1, flags | oracle.F_GREATER,
                                         kbe.GRAD_OVERWRITE, base="random")
    read = np.zeros((nt, nt), bool)
    read[:, m0:m1] = True
    read[m0:m1, :] = True
    rd_read = np.zeros(nt, bool)
    rd_read[m0:m1] = True
    check_overwrite(ref, gG, base, scale, read, rd_read)


def test_collision_vjp_overwrite_mode(gpu):
    """KBE_GRAD_OVERWRITE writes exactly the blocks the forward reads (here: all of [0,n]^2 and
    tv rows 0..n) and leaves the rest of the arrays as they were."""
    kbe = gpu
    case = Case(N=16, nt=80, ntau=10, beta=2.0, seed=3)
    ref, (gG, gs), base, scale = vjp_case(kbe, case, 0, 80, oracle.F_ALL, kbe.GRAD_OVERWRITE,
                                          base="random")
    # every block is read: the arrays hold the pure gradient
    check_gradients(ref, (gG, gs), tuple(np.zeros_like(b) for b in base), scale)
    # a partial range: blocks nobody reads keep their initial values (generic gradient kernel
    # at N = 4, the padded MFMA one at N = 6 and 8)
    for N in (4, 6, 8):
        case2 = Case(N=N, nt=30, ntau=6, beta=2.0, seed=4)
        ref2, (gG2, _), base2, scale2 = vjp_case(kbe, case2, 10, 20, oracle.F_IR | oracle.F_IL,
                                                 kbe.GRAD_OVERWRITE, base="random")
        read = np.zeros((30, 30), bool)
        for m in range(10, 20):
            read[: m + 1, m] = True   # IR column part
            read[m, m + 1:] = True    # IR row part
            read[m, :m] = True        # IL
        rd_read = np.zeros(30, bool)
        rd_read[10:20] = True
        check_overwrite(ref2, gG2, base2, scale2, read, rd_read)


@pytest.mark.parametrize("N,n", [(2, 63), (3, 0), (16, 45), (16, 0)])
def test_sigma_vjp_matches_oracle(gpu, N, n):
    kbe = gpu
    case = Case(N=N, nt=64 if N < 16 else 46, ntau=10, beta=2.0, seed=60 + N)
    t, order, kp, rd, tv, mat = case.host()
    u = np.linspace(0.7, 1.3, N)
    gsig = (synth.normal(9, 0, (n + 1, N, N)), synth.normal(9, 1, (n + 1, N, N)),
            synth.normal(9, 2, (case.ntau, N, N)))
    base = (np.zeros(kp.shape, np.complex128), np.zeros(rd.shape, np.complex128),
            np.zeros(tv.shape, np.complex128))
    gu0 = np.zeros(N)
    rk, rr, rt, ru = oracle.sigma_row_vjp(oracle.Green(kp, rd, tv, mat), u, n, gsig,
                                         grads=tuple(b.copy() for b in base), gu=gu0.copy())
    gG = device_green(base[0], base[1], base[2], mat)
    gG, gu = kbe.sigma_2b_vjp(device_green(kp, rd, tv, mat), to_dev(u), n,
                              tuple(to_dev(x) for x in gsig), gG, to_dev(gu0.copy()))
    # pure gradients (zero initial arrays): the blocks of row and column n, rdiag[n] and tv row n
    # that the row reads, each to its rounding scale; nothing else is written
    S_kp, S_rd, S_tv = sigma_vjp_scales(kp, rd, tv, u, n, gsig)
    touched = S_kp > 0
    kpg, rdg, tvg = to_host(gG.kp), to_host(gG.rdiag), to_host(gG.tv)
    assert_blocks_close(kpg[touched], rk[touched], S_kp[touched], "gkp")
    assert np.array_equal(kpg[~touched], base[0][~touched])
    assert_blocks_close(rdg[n:n + 1], rr[n:n + 1], S_rd[n:n + 1], "grdiag")
    assert_blocks_close(tvg[n], rt[n], S_tv[n], "gtv")
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


@pytest.mark.parametrize("N,nt,ntau,m0,m1,same", [
    (16, 120, 10, 0, 120, False), (16, 80, 6, 10, 70, False), (8, 90, 12, 5, 80, False),
    (6, 60, 0, 0, 60, False), (3, 70, 6, 10, 50, False), (12, 40, 5, 0, 40, False),
    # one array for the greater form's two cotangents (as the propagations pass them): the
    # small-block and generic paths merge two of its classes
    (16, 80, 6, 10, 70, True), (8, 90, 12, 5, 80, True), (6, 60, 0, 0, 60, True),
    (3, 70, 6, 10, 50, True), (12, 40, 5, 3, 37, True)])
def test_both_forms_vjp_matches_oracle(gpu, N, nt, ntau, m0, m1, same):
    """kbe_collision_both_vjp (the lesser adjoint on the summed cotangents plus the greater form's
    own terms) against the sum of the oracle's lesser adjoint (cotangents of IR, IL, Itv, Jtv) and
    greater adjoint (cotangents of the greater IR, IL), every gradient array, pure gradients, on
    every kernel path and on partial ranges."""
    kbe = gpu
    print("both vjp", N, nt, ntau, m0, m1, same, flush=True)
    case = Case(N=N, nt=nt, ntau=ntau, beta=3.0 if ntau else 0.0, seed=70 + N)
    t, order, kp, rd, tv, mat = case.host()
    n = nt - 1
    W = oracle.Weights.build(t, order, case.beta, ntau, case.tau_order)
    sig = synth.sigma_row(case.seed, N, n, ntau, t)
    M = m1 - m0
    c = [synth.normal(11, k, (M, N, N)) for k in range(3)] + \
        [synth.normal(11, 3, (ntau, N, N))] + [synth.normal(11, 4 + k, (M, N, N)) for k in range(2)]
    if same:
        c[5] = c[4]
    z = lambda *sh: np.zeros(sh, np.complex128)
    Go = oracle.Green(kp, rd, tv, mat)
    les = oracle.collision_vjp(Go, sig, W, n, m0, m1, tuple(c[:4]), oracle.F_ALL)
    gre = oracle.collision_vjp(Go, sig, W, n, m0, m1, (c[4], c[5], z(M, N, N), z(ntau, N, N)),
                               oracle.F_IR | oracle.F_IL | oracle.F_GREATER, grads=les[:4])
    ref = (gre[0], gre[1], gre[2], gre[3], les[4] + gre[4], les[5] + gre[5], les[6])
    s1 = vjp_scales(kp, rd, tv, mat, sig, W, n, m0, m1, tuple(c[:4]), oracle.F_ALL)
    s2 = vjp_scales(kp, rd, tv, mat, sig, W, n, m0, m1, (c[4], c[5], None, None),
                    oracle.F_IR | oracle.F_IL | oracle.F_GREATER)
    scale = {k: s1[k] + s2[k] for k in s1}
    base = tuple(np.zeros(x.shape, np.complex128) for x in (kp, rd, tv, mat))
    Gd = device_green(kp, rd, tv, mat)
    cot = tuple(to_dev(x) if x.size else None for x in c)
    if same:  # the same device array, not an equal copy
        cot = cot[:5] + (cot[4],)
    if not ntau:
        cot = (cot[0], cot[1], None, None, cot[4], cot[5])
    sigd = tuple(to_dev(x) if x.size else None for x in sig)
    got = kbe.collision_both_vjp(Gd, sigd, device_weights(W), n, m0, m1, cot)
    check_gradients(ref, got, base, scale)
