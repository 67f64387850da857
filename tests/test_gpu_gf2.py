"""kbe_sigma_gf2 (Eq. SE with a general four-index U) against the oracle, to the FP64 bar.

Small systems over every padded block size (N = 1..16, with and without a thermal branch, first,
middle and last rows, general and symmetric U), the local-U case against kbe_sigma_2b, and the
16-orbital headline row (n = 2047, ntau = 512) run as one launch and sampled block by block."""
import numpy as np
import pytest

import oracle
import synth
from tests.cases import RTOL, Case, bnorm, device_green, to_dev, to_host

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _check_row(got, ref, s_list=None, l_list=None, rtol=RTOL):
    """Blocks of (ret, les, stv) against the oracle, each relative to max(|Sigma^>|, |Sigma^<|)
    (ret = Sigma^> - Sigma^< may cancel) or |Sigma^]|."""
    ret, les, stv = (to_host(x) for x in got)
    rr, rl, rs = ref
    s_idx = slice(None) if s_list is None else list(s_list)
    sc = np.maximum(bnorm(rr[s_idx] + rl[s_idx]), bnorm(rl[s_idx])) + 1e-300
    assert np.all(bnorm(ret[s_idx] - rr[s_idx]) <= rtol * sc), "ret"
    assert np.all(bnorm(les[s_idx] - rl[s_idx]) <= rtol * sc), "les"
    if rs.shape[0]:
        l_idx = slice(None) if l_list is None else list(l_list)
        assert np.all(bnorm(stv[l_idx] - rs[l_idx]) <= rtol * (bnorm(rs[l_idx]) + 1e-300)), "stv"


@pytest.mark.parametrize("N,ntau", [(1, 6), (2, 0), (3, 7), (4, 4), (5, 6), (8, 0), (8, 9),
                                    (11, 5), (16, 4)])
def test_sigma_gf2_matches_oracle(gpu, N, ntau):
    kbe = gpu
    case = Case(N=N, nt=10, ntau=ntau, beta=4.0, seed=500 + N + ntau)
    t, order, kp, rd, tv, mat = case.host()
    G = oracle.Green(kp, rd, tv if ntau else None, mat if ntau else None)
    Gd = device_green(kp, rd, tv, mat)
    rng = np.random.default_rng(N)
    for U in (synth.coulomb(N, N), rng.normal(size=(N,) * 4)):  # symmetric and general
        Ud = to_dev(U)
        for n in (0, 4, case.nt - 1):
            _print("gf2", N, ntau, n)
            _check_row(kbe.sigma_gf2(Gd, Ud, n), oracle.sigma_gf2_row(G, U, n))


@pytest.mark.parametrize("N", [1, 3, 8, 16])
def test_sigma_gf2_local_u_equals_sigma_2b(gpu, N):
    """A local U (U_iiii = u_i, all else 0) through the general kernel gives kbe_sigma_2b's row."""
    kbe = gpu
    case = Case(N=N, nt=12, ntau=6, beta=4.0, seed=600 + N)
    t, order, kp, rd, tv, mat = case.host()
    Gd = device_green(kp, rd, tv, mat)
    u = np.linspace(0.7, 1.6, N)
    U = np.zeros((N,) * 4)
    for i in range(N):
        U[i, i, i, i] = u[i]
    n = case.nt - 1
    got = kbe.sigma_gf2(Gd, to_dev(U), n)
    ref = [to_host(x) for x in kbe.sigma_2b(Gd, to_dev(u), n)]
    G = oracle.Green(kp, rd, tv, mat)
    want = oracle.sigma_row(G, u, n)
    for g, r, o in zip(got, ref, want):
        g = to_host(g)
        sc = bnorm(o) + 1e-300
        assert np.all(bnorm(g - o) <= RTOL * sc)
        assert np.all(bnorm(g - r) <= RTOL * sc)


def test_sigma_gf2_rejects_bad_u(gpu):
    import torch
    kbe = gpu
    case = Case(N=4, nt=6, ntau=0, beta=4.0, seed=7)
    t, order, kp, rd, tv, mat = case.host()
    Gd = device_green(kp, rd, tv, mat)
    with pytest.raises(kbe.KBEError):
        kbe.sigma_gf2(Gd, torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda"), 3)
    with pytest.raises(kbe.KBEError):
        kbe.sigma_gf2(Gd, torch.zeros((4,) * 4, dtype=torch.float32, device="cuda"), 3)


def test_sigma_gf2_headline_row_sampled(gpu):
    """The 16-orbital headline row (nt = 2048, n = 2047, ntau = 512) in one launch, as bench.py
    runs it; sampled blocks (first, chunk edges, diagonal; tau ends and middle) against the
    oracle, and the inherited symmetry of the diagonal block."""
    import torch
    kbe = gpu
    W = synth.HEADLINE
    N, nt, ntau, n = W.N, W.nt, W.ntau, W.nt - 1
    t, order = synth.grid(W.seed, nt, W.hmin, W.hmax, W.omin, W.omax)
    _print("gf2 headline: inputs (row and column n of kp, rdiag, tv row n: all the row reads)")
    kp = np.zeros((nt, nt, N, N), np.complex128)  # calloc: untouched pages stay unmapped
    kp[n] = synth.kp(W.seed, N, t, rows=(n, n + 1))[0]
    kp[:, n] = synth.kp_col(W.seed, N, t, n)
    rd = synth.rdiag(N, nt)
    tv = np.zeros((nt, ntau, N, N), np.complex128)
    tv[n] = synth.tv(W.seed, N, ntau, t, rows=(n, n + 1))[0]
    mat = synth.mat(W.seed, N, ntau)
    U = synth.coulomb(W.seed, N)
    dev = torch.device("cuda:0")
    kpd = torch.zeros(kp.shape, dtype=torch.complex128, device=dev)
    kpd[n].copy_(torch.from_numpy(kp[n]))
    kpd[:, n].copy_(torch.from_numpy(np.ascontiguousarray(kp[:, n])))
    tvd = torch.zeros(tv.shape, dtype=torch.complex128, device=dev)
    tvd[n].copy_(torch.from_numpy(tv[n]))
    Gd = kbe.Green(kpd, to_dev(rd), tvd, to_dev(mat))
    _print("gf2 headline: run")
    got = kbe.sigma_gf2(Gd, to_dev(U), n)
    torch.cuda.synchronize()
    del Gd, kpd, tvd
    s_list = [0, 1, 511, 512, 1500, n - 1, n]
    l_list = [0, 1, 255, 256, ntau - 1]
    G = oracle.Green(kp, rd, tv, mat)
    _print("gf2 headline: oracle")
    ref = oracle.sigma_gf2_row(G, U, n, s_list=s_list, l_list=l_list)
    _check_row(got, ref, s_list, l_list)
    ret, les, stv = (to_host(x) for x in got)
    for x in (ret, les, stv):
        assert np.all(np.isfinite(x))
    # Sigma^<(t_n, t_n) is anti-Hermitian like G^<(t_n, t_n) when U has the eight-fold symmetry
    d = les[n]
    assert np.linalg.norm(d + d.conj().T) <= 1e-12 * np.linalg.norm(d)
