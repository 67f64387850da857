"""GPU parity: the HIP library (called through its C ABI) against the CPU oracle on the same
seeded inputs, to the FP64 bar (per block 1e-12 of the rounding scale, and 1e-12 globally)."""
import numpy as np
import pytest

import oracle
import synth
from tests.cases import (RTOL, Case, assert_blocks_close, bnorm, device_green, device_weights,
                         scales, to_dev, to_host)

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def run_collision(kbe, case: Case, n=None, m0=0, m1=None, flags=None, gpu_weights=False,
                  extra_flags=0, sig_mode="random"):
    t, order, kp, rd, tv, mat = case.host()
    n = case.nt - 1 if n is None else n
    m1 = n + 1 if m1 is None else m1
    flags = oracle.F_ALL if flags is None else flags
    W = oracle.Weights.build(t, order, case.beta, case.ntau, case.tau_order)
    Go = oracle.Green(kp, rd, tv, mat)
    Gd = device_green(kp, rd, tv, mat)
    if sig_mode == "random":
        sig = synth.sigma_row(case.seed, case.N, n, case.ntau, t)
        if not case.ntau:
            sig = (sig[0], sig[1], np.zeros((0, case.N, case.N), np.complex128))
    else:  # second Born from the same G
        sig = oracle.sigma_row(Go, np.full(case.N, case.U), n)
    sigd = tuple(to_dev(x) if x.size else None for x in sig)
    if gpu_weights:
        Wd = kbe.weights(t, order, case.ntau, case.beta, case.tau_order)
    else:
        Wd = device_weights(W)
    gpu = kbe.collision(Gd, sigd, Wd, n, m0, m1, flags | extra_flags)
    ref = oracle.collision(Go, sig, W, n, m0, m1, flags)
    sc = scales(kp, rd, tv, mat, sig, W, n, range(m0, m1), range(case.ntau))
    return gpu, ref, sc


def check_all(gpu, ref, sc, flags=oracle.F_ALL, rtol=RTOL):
    names = ["IR", "IL", "Itv", "Jtv"]
    for k, name in enumerate(names):
        if not flags & (1 << k):
            continue
        g = to_host(gpu[k])
        if g is None:
            assert ref[k].size == 0, name
            continue
        assert_blocks_close(g, ref[k], sc[name], name, rtol)


def test_weights_match_oracle(gpu):
    kbe = gpu
    for seed, nt, hmin, hmax, omin, omax, ntau, beta, to in [
        (1000, 64, 0.02, 0.08, 5, 5, 64, 10.0, 5),
        (1001, 2048, 0.005, 0.05, 3, 6, 512, 20.0, 5),
        (7, 300, 0.005, 0.05, 1, 12, 33, 3.0, 8),
        (8, 50, 0.01, 0.1, 2, 2, 9, 1.0, 1),
    ]:
        _print("weights case", seed, nt, omin, omax, ntau, to)
        t, order = synth.grid(seed, nt, hmin, hmax, omin, omax)
        Wd = kbe.weights(t, order, ntau, beta, to)
        W = oracle.Weights.build(t, order, beta, ntau, to)
        w = to_host(Wd.w)
        scale = np.abs(W.w).max(axis=1, keepdims=True) + 1e-300
        assert (np.abs(w - W.w) / scale).max() < 1e-12
        assert np.all(w[np.triu_indices(nt, 1)] == 0)
        np.testing.assert_allclose(to_host(Wd.wtau), W.wfull, rtol=0, atol=1e-12 * np.abs(W.wfull).max())
        np.testing.assert_allclose(to_host(Wd.wtau_fwd), W.wf, rtol=0, atol=1e-12 * np.abs(W.wf).max())


def test_weights_high_order(gpu):
    """Orders up to KBE_KMAX = 20 (the paper's maximum history order K).  The moment system is
    ill-conditioned there (on this grid the local rules reach sum |lambda| / h of about 4e5), so the
    bar is what both routes guarantee, interval by interval: the local weights of every interval,
    lambda = w[p] - w[p-1] on its nodes, integrate every polynomial of degree < k exactly, to
    rounding of the sum of |lambda| (Legendre polynomials in the variable scaled to the node
    window, so |P| <= 1 there).  The weights themselves agree with the oracle's (a different
    route: Gauss-Legendre integration of the Lagrange basis) only to the conditioning of the
    moment system, about 1e6 at order 20 in that basis, hence 1e-9 of the sum of |lambda|."""
    from numpy.polynomial import legendre as L
    kbe = gpu
    t, order = synth.grid(3, 120, 0.01, 0.05, 13, 20)
    w = to_host(kbe.weights(t, order).w)
    W = oracle.weights(t, order)
    assert np.abs(w - W).max() < 1e-9 * np.abs(W).max()
    n = 119
    for d in range(2):  # start-up intervals limit the whole-range exactness to degree 1
        # high-order weights alternate in sign; rounding scales with sum |w|
        assert abs(w[n] @ (t / t[n]) ** d - t[n] / (d + 1)) < 1e-14 * np.abs(w[n]).sum()
    checked = 0
    for p in range(1, 120):
        k = min(int(order[p]), p + 1)
        nodes = np.arange(p - k + 1, p + 1)
        lam = w[p, nodes] - w[p - 1, nodes]
        sc = np.abs(w[p, nodes]).sum() + np.abs(w[p - 1, nodes]).sum()
        lam_o = oracle.local_weights(t, p, k)
        assert np.abs(lam - lam_o).max() <= 1e-9 * sc, p
        a, b = t[p - k + 1], t[p]
        x = lambda y: (2.0 * y - a - b) / (b - a) if k > 1 else 0.0 * y
        for deg in range(k):
            c = np.zeros(deg + 1)
            c[deg] = 1.0
            P = L.legval(x(t[nodes]), c)
            ci = L.legint(c)
            exact = 0.5 * (b - a) * (L.legval(x(t[p]), ci) - L.legval(x(t[p - 1]), ci)) \
                if k > 1 else (t[p] - t[p - 1]) * (deg == 0)
            assert abs(lam @ P - exact) <= 1e-13 * sc, (p, k, deg)
            checked += 1
    assert checked > 1500


@pytest.mark.parametrize("N,n", [(1, 5), (2, 0), (2, 63), (3, 17), (16, 0), (16, 39)])
def test_sigma_row_matches_oracle(gpu, N, n):
    kbe = gpu
    case = Case(N=N, nt=40 if N == 16 else 64, ntau=12, beta=4.0, seed=11 + N)
    t, order, kp, rd, tv, mat = case.host()
    u = np.linspace(0.6, 1.4, N)
    ref = oracle.sigma_row(oracle.Green(kp, rd, tv, mat), u, n)
    got = kbe.sigma_2b(device_green(kp, rd, tv, mat), to_dev(u), n)
    for g, r in zip(got, ref):
        g = to_host(g)
        d = bnorm(g - r)
        assert np.all(d <= 1e-13 * (bnorm(r) + 1e-300) + 1e-300)


def test_sigma_batch_matches_oracle_and_rows(gpu):
    """kbe_sigma_2b_batch over rows of systems with different N (1, 3, 8, 16), storage (a padded
    row stride) and thermal branches (none, 12 and 7 tau points): every row against the oracle
    (as test_sigma_row_matches_oracle) and bit for bit against kbe_sigma_2b on its own."""
    import torch
    kbe = gpu
    specs = [(1, 30, 0, 21, 0), (3, 50, 12, 22, 7), (8, 40, 7, 23, 0), (16, 25, 12, 24, 0)]
    systems, rows = [], []
    for N, nt, ntau, seed, pad in specs:
        case = Case(N=N, nt=nt, ntau=ntau, beta=3.0, seed=seed)
        t, order, kp, rd, tv, mat = case.host()
        if pad:
            kpp = np.zeros((nt, nt + pad, N, N), np.complex128)
            kpp[:, :nt] = kp
            kp = kpp
        u = np.linspace(0.5, 1.3, N)
        Gd = kbe.Green(to_dev(kp), to_dev(rd), to_dev(tv) if ntau else None,
                       to_dev(mat) if ntau else None)
        systems.append(dict(G=oracle.Green(kp[:, :nt] if pad else kp, rd, tv if ntau else None,
                                           mat if ntau else None), Gd=Gd, u=u, ud=to_dev(u)))
        for n in sorted({0, nt // 3, nt - 1}):
            rows.append((len(systems) - 1, n))
    sb = kbe.SigmaBatch([(systems[si]["Gd"], systems[si]["ud"], n) for si, n in rows])
    _print("sigma batch", len(rows), "rows")
    got = sb.run()
    torch.cuda.synchronize()
    for (si, n), g in zip(rows, got):
        S = systems[si]
        ref = oracle.sigma_row(S["G"], S["u"], n)
        one = kbe.sigma_2b(S["Gd"], S["ud"], n)
        for x, r, o in zip(g, ref, one):
            if x is None:
                assert r.shape[0] == 0 and o is None
                continue
            x = to_host(x)
            d = bnorm(x - r)
            assert np.all(d <= 1e-13 * (bnorm(r) + 1e-300) + 1e-300), (si, n)
            assert np.array_equal(x, to_host(o)), (si, n)


@pytest.mark.parametrize("N,nt,ntau,mr", [(2, 70, 9, None), (5, 140, 6, (10, 90)),
                                          (8, 300, 20, (7, 290)), (8, 40, 0, None),
                                          (16, 300, 17, None), (16, 280, 9, (30, 270)),
                                          (16, 30, 6, (12, 12)), (12, 50, 7, (3, 41))])
def test_both_forms_match_oracle(gpu, N, nt, ntau, mr):
    """kbe_collision_both (the propagations' call: the lesser form's four outputs and the greater
    form's I^R and I^< from one pass) against the oracle's lesser and greater forms, whole,
    partial and empty m-ranges, with and without a thermal branch, on every kernel path (MFMA
    task at N = 16, small-block tasks at N <= 8, generic otherwise)."""
    kbe = gpu
    case = Case(N=N, nt=nt, ntau=ntau, beta=4.0, seed=900 + N)
    t, order, kp, rd, tv, mat = case.host()
    G = oracle.Green(kp, rd, tv if ntau else None, mat if ntau else None)
    W = oracle.Weights.build(t, order, case.beta if ntau else None, ntau, case.tau_order)
    n = nt - 1
    sig = synth.sigma_row(case.seed + 3, N, n, ntau, t)
    m0, m1 = mr if mr else (0, n + 1)
    Gd = device_green(kp, rd, tv, mat)
    sigd = tuple(to_dev(x) if x.size else None for x in sig)
    out = kbe.collision_both(Gd, sigd, device_weights(W), n, m0, m1)
    les = oracle.collision(G, sig, W, n, m0, m1, oracle.F_ALL)
    gre = oracle.collision(G, sig, W, n, m0, m1, oracle.F_IR | oracle.F_IL | oracle.F_GREATER)
    rng = range(m0, m1)
    sl = scales(kp, rd, tv if ntau else None, mat, sig, W, n, rng, range(ntau))
    sg = scales(kp, rd, tv if ntau else None, mat, sig, W, n, rng, range(ntau), greater=True)
    for name, g, r, sc in zip(("IR", "IL", "Itv", "Jtv", "IR", "IL"), out,
                              (les[0], les[1], les[2], les[3], gre[0], gre[1]),
                              (sl["IR"], sl["IL"], sl["Itv"], sl["Jtv"], sg["IR"], sg["IL"])):
        if g is None:
            assert not ntau and name in ("Itv", "Jtv")
            continue
        if m1 == m0 and name != "Jtv":
            assert g.shape[0] == 0
            continue
        assert_blocks_close(to_host(g), r, sc, name)


def test_collision_parity_small(gpu):
    """N = 2, nt = 64, ntau = 64, beta = 10, order 5: every output for every m."""
    kbe = gpu
    case = Case(N=2, nt=64, ntau=64, beta=10.0, seed=1000, omin=5, omax=5)
    check_all(*run_collision(kbe, case))


def test_collision_whole_path_gpu_weights(gpu):
    kbe = gpu
    case = Case(N=2, nt=64, ntau=64, beta=10.0, seed=1000, omin=5, omax=5)
    gpu_out, ref, sc = run_collision(kbe, case, gpu_weights=True)
    check_all(gpu_out, ref, sc, rtol=1e-11)  # the two weight routes differ at rounding level


@pytest.mark.parametrize("generic", [False, True])
def test_collision_parity_n16_several_chunks(gpu, generic):
    """N = 16 over 300 points (two full 128-term chunks and a ragged tail), MFMA and generic."""
    kbe = gpu
    case = Case(N=16, nt=300, ntau=40, beta=6.0, seed=77, hmin=0.005, hmax=0.05)
    _print("N16 nt300 generic" if generic else "N16 nt300 mfma")
    out = run_collision(kbe, case, extra_flags=kbe.FORCE_GENERIC if generic else 0)
    check_all(*out)


@pytest.mark.parametrize("nt,ntau,n,flags", [
    (9, 3, None, oracle.F_ALL),
    (2, 2, None, oracle.F_ALL),
    (257, 9, None, oracle.F_ALL),
    (300, 17, 170, oracle.F_ALL),
    (300, 17, None, oracle.F_ITV | oracle.F_JTV),
    (300, 17, None, oracle.F_IR),
    (300, 17, None, oracle.F_ITV),
    (300, 17, None, oracle.F_JTV),
    (130, 2, None, oracle.F_ALL),
])
def test_collision_n16_sizes_and_subsets(gpu, nt, ntau, n, flags):
    """N = 16 (MFMA path) over the whole output range at small, ragged and two-chunk sizes (chunks
    of 256 terms, groups of 8 outputs), every output alone or with the others, at the last row
    and with row n inside the stored history."""
    kbe = gpu
    _print("n16 sizes", nt, ntau, n, flags)
    case = Case(N=16, nt=nt, ntau=ntau, beta=2.5, seed=300 + nt)
    check_all(*run_collision(kbe, case, n=n, flags=flags), flags)


@pytest.mark.parametrize("N", [1, 3, 4, 5, 7, 8, 9, 13, 16])
def test_collision_orbital_counts(gpu, N):
    kbe = gpu
    case = Case(N=N, nt=37, ntau=9, beta=2.0, seed=100 + N)
    check_all(*run_collision(kbe, case))


@pytest.mark.parametrize("N,nt,ntau", [(8, 300, 140), (6, 290, 20), (4, 600, 300), (3, 530, 300),
                                        (2, 2100, 30), (1, 2200, 10)])
def test_collision_small_blocks_several_chunks(gpu, N, nt, ntau):
    """Small-block path (N <= 8) over several term chunks with ragged tails (chunks of 128 terms
    for N >= 5, 256 for N = 3, 4 and 1024 below), real-time and Matsubara classes."""
    kbe = gpu
    _print("small blocks", N, nt, ntau)
    case = Case(N=N, nt=nt, ntau=ntau, beta=3.0, seed=200 + N)
    check_all(*run_collision(kbe, case))


@pytest.mark.parametrize("flags", [oracle.F_IR, oracle.F_ITV | oracle.F_JTV,
                                   oracle.F_IR | oracle.F_IL, oracle.F_ALL])
def test_collision_small_blocks_output_subsets(gpu, flags):
    """N = 8 over the full m range with output subsets (I^R alone, the two tau integrals alone,
    I^R with I^<, all four), at the last row and with row n in the middle of the stored history
    (the tasks stop short of the arrays' ends) and at n = 0."""
    kbe = gpu
    case = Case(N=8, nt=90, ntau=21, beta=2.0, seed=31)
    for n in (89, 40, 0):
        _print("output subsets", flags, n)
        out = run_collision(kbe, case, n=n, flags=flags)
        check_all(*out, flags=flags)


@pytest.mark.parametrize("N", [2, 5, 8])
def test_small_block_path_agrees_with_generic(gpu, N):
    """The small-block task and the generic one-output-per-wave task sum the same terms in
    different orders: they agree to rounding."""
    kbe = gpu
    case = Case(N=N, nt=260, ntau=150, beta=3.0, seed=300 + N)
    t, order, kp, rd, tv, mat = case.host()
    W = device_weights(oracle.Weights.build(t, order, case.beta, case.ntau))
    Gd = device_green(kp, rd, tv, mat)
    sig = tuple(to_dev(x) for x in synth.sigma_row(case.seed, N, 259, case.ntau, t))
    a = kbe.collision(Gd, sig, W, 259)
    b = kbe.collision(Gd, sig, W, 259, flags=kbe.OUT_ALL | kbe.FORCE_GENERIC)
    for x, y in zip(a, b):
        x, y = to_host(x), to_host(y)
        assert np.linalg.norm((x - y).ravel()) <= 1e-13 * np.linalg.norm(y.ravel())


def test_collision_ragged_ranges_and_edges(gpu):
    kbe = gpu
    case = Case(N=4, nt=50, ntau=10, beta=2.0, seed=5)
    for (n, m0, m1) in [(0, 0, 1), (49, 0, 0), (49, 50, 50), (49, 13, 29), (20, 20, 21), (30, 0, 31)]:
        _print("range", n, m0, m1)
        check_all(*run_collision(kbe, case, n=n, m0=m0, m1=m1))
    # no thermal branch
    case0 = Case(N=3, nt=40, ntau=0, beta=0.0, seed=6)
    check_all(*run_collision(kbe, case0, flags=oracle.F_IR | oracle.F_IL), oracle.F_IR | oracle.F_IL)
    # padded leading dimension, N = 16 (MFMA path)
    case1 = Case(N=16, nt=30, ntau=6, beta=2.0, seed=9, ldt=37)
    check_all(*run_collision(kbe, case1))
    # single outputs selected
    for f in (oracle.F_IR, oracle.F_IL, oracle.F_ITV, oracle.F_JTV):
        g, r, s = run_collision(kbe, Case(N=16, nt=25, ntau=7, beta=2.0, seed=10), flags=f)
        check_all(g, r, s, f)


def test_collision_partial_range_is_slice_and_deterministic(gpu):
    kbe = gpu
    case = Case(N=16, nt=200, ntau=20, beta=3.0, seed=12)
    t, order, kp, rd, tv, mat = case.host()
    W = device_weights(oracle.Weights.build(t, order, case.beta, case.ntau))
    Gd = device_green(kp, rd, tv, mat)
    sig = tuple(to_dev(x) for x in synth.sigma_row(case.seed, case.N, 199, case.ntau, t))
    full = [to_host(x) for x in kbe.collision(Gd, sig, W, 199)]
    again = [to_host(x) for x in kbe.collision(Gd, sig, W, 199)]
    for a, b in zip(full, again):
        assert np.array_equal(a, b)  # bitwise run-to-run determinism
    part = [to_host(x) for x in kbe.collision(Gd, sig, W, 199, 50, 130)]
    for a, b in zip(full[:3], part[:3]):
        np.testing.assert_array_equal(a[50:130], b)
    np.testing.assert_array_equal(full[3], part[3])


def test_mfma_agrees_with_generic(gpu):
    kbe = gpu
    case = Case(N=16, nt=160, ntau=24, beta=3.0, seed=13)
    t, order, kp, rd, tv, mat = case.host()
    W = device_weights(oracle.Weights.build(t, order, case.beta, case.ntau))
    Gd = device_green(kp, rd, tv, mat)
    sig = tuple(to_dev(x) for x in synth.sigma_row(case.seed, case.N, 159, case.ntau, t))
    a = kbe.collision(Gd, sig, W, 159)
    b = kbe.collision(Gd, sig, W, 159, flags=kbe.OUT_ALL | kbe.FORCE_GENERIC)
    for x, y in zip(a, b):
        x, y = to_host(x), to_host(y)
        assert np.linalg.norm((x - y).ravel()) <= 1e-13 * np.linalg.norm(y.ravel())


def test_conservation_invariant_on_gpu(gpu):
    """With Sigma = kbe_sigma_2b(G) and anti-Hermitian diagonal blocks, Re Tr of the m = n
    integrals vanishes to rounding (the conservation law of the second-Born self-energy)."""
    kbe = gpu
    case = Case(N=16, nt=150, ntau=20, beta=3.0, seed=21)
    t, order, kp, rd, tv, mat = case.host()
    Gd = device_green(kp, rd, tv, mat)
    Wd = kbe.weights(t, order, case.ntau, case.beta, 5)
    n = 149
    sig = kbe.sigma_2b(Gd, to_dev(np.full(16, 1.3)), n)
    IR, IL, Itv, _ = (to_host(x) for x in kbe.collision(Gd, sig, Wd, n, n, n + 1))
    scale = np.abs(IR[0]).sum() + np.abs(IL[0]).sum()
    assert abs(np.trace(IR[0] + IL[0]).real) < 1e-13 * scale
    assert abs(np.trace(Itv[0]).real) < 1e-13 * np.abs(Itv[0]).sum()


@pytest.mark.parametrize("N", [16, 8])
def test_sigma_and_collision_graph_capture(gpu, N):
    """[kbe_sigma_2b -> kbe_collision (stream kernels and chunk reduce)] captured once in a graph
    (no host copies, no allocation inside the library, no memset nodes): every replay, with
    eager work and synchronisation between replays, reproduces the eager result bitwise."""
    import torch
    kbe = gpu
    case = Case(N=N, nt=120, ntau=16, beta=3.0, seed=60 + N)
    t, order, kp, rd, tv, mat = case.host()
    Gd = device_green(kp, rd, tv, mat)
    Wd = device_weights(oracle.Weights.build(t, order, case.beta, case.ntau))
    u = to_dev(np.full(N, 1.3))
    n = case.nt - 1
    eager = [to_host(x) for x in kbe.collision(Gd, kbe.sigma_2b(Gd, u, n), Wd, n)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        kbe.collision(Gd, kbe.sigma_2b(Gd, u, n), Wd, n)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sig = kbe.sigma_2b(Gd, u, n)
        out = kbe.collision(Gd, sig, Wd, n)
    for rep in range(3):
        for x in out:
            x.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, eager):
            assert np.array_equal(to_host(a), b), rep


@pytest.mark.parametrize("N", [4, 16])
def test_weights_sigma_collision_graph_capture(gpu, N):
    """The whole forward step [kbe_weights_dev -> kbe_sigma_2b -> kbe_collision] captured in one
    graph (the grid in device memory): every replay, with eager work between replays, reproduces
    the eager result bitwise, weights included; kbe_weights (host grid) refuses the capturing
    stream with KBE_ENOTSUP."""
    import torch
    kbe = gpu
    case = Case(N=N, nt=150, ntau=20, beta=3.0, seed=80 + N)
    t, order, kp, rd, tv, mat = case.host()
    Gd = device_green(kp, rd, tv, mat)
    u = to_dev(np.full(N, 1.1))
    n = case.nt - 1
    td, od = to_dev(t), to_dev(np.asarray(order, np.int32))

    def step():
        W = kbe.weights_dev(td, od, case.ntau, case.beta, case.tau_order, check=False)
        return (W.w, W.wtau, W.wtau_fwd) + kbe.collision(Gd, kbe.sigma_2b(Gd, u, n), W, n)

    eager = [to_host(x) for x in step()]
    Wo = oracle.Weights.build(t, order, case.beta, case.ntau, case.tau_order)
    assert np.abs(eager[0] - Wo.w).max() < 1e-12 * np.abs(Wo.w).max()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = step()
        with pytest.raises(kbe.KBEError, match="KBE_ENOTSUP"):
            kbe.weights(t, order, case.ntau, case.beta, case.tau_order)
    for rep in range(3):
        for x in out:
            x.fill_(float("nan"))
        kbe.collision(Gd, kbe.sigma_2b(Gd, u, n), device_weights(Wo), n)  # eager work between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, eager):
            assert np.array_equal(to_host(a), b), rep


@pytest.mark.parametrize("N,nt,ntau,sldt", [(1, 9, 5, 9), (3, 12, 0, 12), (8, 10, 6, 13),
                                            (16, 7, 4, 7)])
def test_sigma_full_mode_matches_oracle(gpu, N, nt, ntau, sldt):
    """kbe_sigma_2b_full: every stored block of Sigma (KP triangle pair, rdiag, tv) against the
    oracle, including a Sigma whose row stride exceeds G's."""
    import torch
    kbe = gpu
    case = Case(N=N, nt=nt, ntau=ntau, beta=4.0, seed=700 + N)
    t, order, kp, rd, tv, mat = case.host()
    Gd = device_green(kp, rd, tv, mat)
    u = np.linspace(0.6, 1.4, N)
    dev = torch.device("cuda:0")
    S = kbe.Green(torch.full((nt, sldt, N, N), float("nan"), dtype=torch.complex128, device=dev),
                  torch.full((nt, N, N), float("nan"), dtype=torch.complex128, device=dev),
                  torch.full((nt, ntau, N, N), float("nan"), dtype=torch.complex128, device=dev),
                  torch.zeros((ntau, N, N), dtype=torch.complex128, device=dev))
    kbe.sigma_2b_full(Gd, to_dev(u), S)
    G = oracle.Green(kp, rd, tv if ntau else None, mat if ntau else None)
    rkp, rrd, rtv = oracle.sigma_full(G, u)
    got = to_host(S.kp)[:, :nt]
    for name, g, r in (("kp", got, rkp), ("rdiag", to_host(S.rdiag), rrd), ("tv", to_host(S.tv), rtv)):
        assert np.all(np.isfinite(g)), name
        assert np.all(bnorm(g - r) <= 1e-13 * (bnorm(r) + 1e-300)), name


@pytest.mark.parametrize("N,nt,ntau,mr", [(1, 20, 6, None), (3, 25, 0, (4, 17)), (8, 18, 5, None),
                                          (16, 14, 4, (0, 9)), (16, 300, 17, None),
                                          (16, 280, 9, (30, 270)), (8, 300, 20, (7, 290)),
                                          (5, 140, 6, None)])
def test_greater_form_matches_oracle(gpu, N, nt, ntau, mr):
    """kbe_collision with KBE_GREATER against the oracle's greater form, all outputs, whole and
    partial m-ranges, on the lesser form's kernels (MFMA task at N = 16, small-block tasks at
    N <= 8, generic otherwise) over one and several 256-term chunks."""
    kbe = gpu
    case = Case(N=N, nt=nt, ntau=ntau, beta=4.0, seed=800 + N)
    t, order, kp, rd, tv, mat = case.host()
    G = oracle.Green(kp, rd, tv if ntau else None, mat if ntau else None)
    W = oracle.Weights.build(t, order, case.beta if ntau else None, ntau, case.tau_order)
    n = nt - 1
    sig = synth.sigma_row(case.seed + 5, N, n, ntau, t)
    m0, m1 = mr if mr else (0, n + 1)
    Gd = device_green(kp, rd, tv, mat)
    Wd = device_weights(W)
    out = kbe.collision(Gd, tuple(to_dev(x) for x in sig), Wd, n, m0, m1,
                        kbe.OUT_ALL | kbe.GREATER)
    ref = oracle.collision(G, sig, W, n, m0, m1, oracle.F_ALL | oracle.F_GREATER)
    sc = scales(kp, rd, tv if ntau else None, mat, sig, W, n, range(m0, m1), range(ntau),
                greater=True)
    for name, g, r in zip(("IR", "IL", "Itv", "Jtv"), out, ref):
        if g is None or (not ntau and name in ("Itv", "Jtv")):
            assert g is None or not np.any(to_host(g)), name  # no thermal branch: zero
            continue
        assert_blocks_close(to_host(g), r, sc[name], name)
