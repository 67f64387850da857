"""Parity at the benchmark's full sizes: the 16-orbital headline (nt = 2048, ntau = 512, row
n = 2047) and the 8-orbital differentiation shape (nt = 1024, ntau = 256, row n = 1023), every m.

The GPU runs the calls exactly as bench.py launches them (all outputs, the whole m range, the
adjoint in overwrite mode).  The oracle computes a sample of the outputs one by one.  The
adjoint is checked at full size by properties that hold at any size: the integrals are linear in
G for a fixed Sigma and linear in Sigma for a fixed G, so the exact adjoint satisfies
Re<cot, I(dG)> = Re<gG, dG> and Re<cot, I(dSigma)> = Re<gSigma, dSigma> (to rounding).  The
self-energy adjoint touches only row and column n, which the oracle computes in full."""
import numpy as np
import pytest

import oracle
import synth
from tests.cases import RTOL, assert_blocks_close, bnorm, scales, to_dev, to_host

pytestmark = pytest.mark.gpu

# workload, sampled m (term-chunk edges, middle, diagonal) and sampled tau points
WORKLOADS = {
    "headline": (synth.HEADLINE, [0, 1, 2, 5, 511, 1024, 1500, 2040, 2046, 2047],
                 [0, 1, 255, 256, 510, 511]),
    "differentiation": (synth.DIFFERENTIATION, [0, 1, 2, 127, 128, 511, 1000, 1022, 1023],
                        [0, 1, 127, 128, 254, 255]),
}


def _print(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", params=list(WORKLOADS))
def big(gpu, request):
    import torch
    kbe = gpu
    W_, m_sample, j_sample = WORKLOADS[request.param]
    N, NT, NTAU, NROW = W_.N, W_.nt, W_.ntau, W_.nt - 1
    _print(request.param, ": generating host inputs")
    t, order = synth.grid(W_.seed, NT, W_.hmin, W_.hmax, W_.omin, W_.omax)
    kp = synth.kp(W_.seed, N, t)
    rd = synth.rdiag(N, NT)
    tv = synth.tv(W_.seed, N, NTAU, t)
    mat = synth.mat(W_.seed, N, NTAU)
    _print(request.param, ": copying to the device")
    dev = torch.device("cuda:0")
    kpd = torch.empty(kp.shape, dtype=torch.complex128, device=dev)
    for a0 in range(0, NT, 128):
        kpd[a0:a0 + 128].copy_(torch.from_numpy(kp[a0:a0 + 128]))
    G = kbe.Green(kpd, to_dev(rd), to_dev(tv), to_dev(mat))
    Go = oracle.Green(kp, rd, tv, mat)
    u = np.full(N, W_.U)
    _print(request.param, ": oracle weights and self-energy")
    Wo = oracle.Weights.build(t, order, W_.beta, NTAU, W_.tau_order)
    sig_o = oracle.sigma_row(Go, u, NROW)
    d = dict(kbe=kbe, t=t, order=order, kp=kp, rd=rd, tv=tv, mat=mat, G=G, Go=Go, u=u, Wo=Wo,
             sig_o=sig_o, W=W_, N=N, NT=NT, NTAU=NTAU, NROW=NROW, M=m_sample, J=j_sample)
    yield d
    d.clear()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _sampled_reference(big, sig):
    """Oracle outputs for the sampled m and j, one output at a time."""
    Go, Wo, NROW = big["Go"], big["Wo"], big["NROW"]
    ref = {"IR": [], "IL": [], "Itv": [], "Jtv": []}
    for m in big["M"]:
        IR, IL, Itv, _ = oracle.collision(Go, sig, Wo, NROW, m, m + 1,
                                          oracle.F_IR | oracle.F_IL | oracle.F_ITV, jrange=(0, 0))
        ref["IR"].append(IR[0])
        ref["IL"].append(IL[0])
        ref["Itv"].append(Itv[0])
    for j in big["J"]:
        _, _, _, Jtv = oracle.collision(Go, sig, Wo, NROW, 0, 0, oracle.F_JTV, jrange=(j, j + 1))
        ref["Jtv"].append(Jtv[0])
    return {k: np.array(v) for k, v in ref.items()}


def _check_sampled(big, out, sig, rtol):
    M_SAMPLE, J_SAMPLE, N = big["M"], big["J"], big["N"]
    ref = _sampled_reference(big, sig)
    sc = scales(big["kp"], big["rd"], big["tv"], big["mat"], sig, big["Wo"], big["NROW"],
                M_SAMPLE, J_SAMPLE)
    IR, IL, Itv, Jtv = (to_host(x) for x in out)
    assert IR.shape == (big["NT"], N, N) and Jtv.shape == (big["NTAU"], N, N)
    assert_blocks_close(IR[M_SAMPLE], ref["IR"], sc["IR"], "IR", rtol)
    assert_blocks_close(IL[M_SAMPLE], ref["IL"], sc["IL"], "IL", rtol)
    assert_blocks_close(Itv[M_SAMPLE], ref["Itv"], sc["Itv"], "Itv", rtol)
    assert_blocks_close(Jtv[J_SAMPLE], ref["Jtv"], sc["Jtv"], "Jtv", rtol)
    for name, x in (("IR", IR), ("IL", IL), ("Itv", Itv), ("Jtv", Jtv)):
        assert np.all(np.isfinite(x)), name


def test_full_size_sigma_row(big):
    """kbe_sigma_2b at the last row against the oracle, every block."""
    kbe = big["kbe"]
    got = kbe.sigma_2b(big["G"], to_dev(big["u"]), big["NROW"])
    for g, r in zip(got, big["sig_o"]):
        d = bnorm(to_host(g) - r)
        assert np.all(d <= 1e-13 * (bnorm(r) + 1e-300))


def test_full_size_collision_sampled_oracle_inputs(big):
    """The collision alone: oracle weights and oracle Sigma as inputs, 1e-12 bar."""
    kbe = big["kbe"]
    Wo = big["Wo"]
    Wd = kbe.Weights(to_dev(Wo.w), to_dev(Wo.wfull), to_dev(Wo.wf))
    sig = big["sig_o"]
    _print("collision, oracle inputs")
    out = kbe.collision(big["G"], tuple(to_dev(x) for x in sig), Wd, big["NROW"])
    _check_sampled(big, out, sig, RTOL)


def test_full_size_whole_path_sampled(big):
    """The benchmark's path: GPU weights and GPU Sigma feed the GPU collision; the oracle runs
    its own weights and Sigma.  The two weight routes differ at rounding level, hence 1e-11."""
    kbe = big["kbe"]
    import torch
    W_, NROW = big["W"], big["NROW"]
    Wd = kbe.weights(big["t"], big["order"], big["NTAU"], W_.beta, W_.tau_order,
                     device=torch.device("cuda:0"))
    sig_d = kbe.sigma_2b(big["G"], to_dev(big["u"]), NROW)
    _print("collision, whole path")
    out = kbe.collision(big["G"], sig_d, Wd, NROW)
    _check_sampled(big, out, big["sig_o"], 1e-11)


def _rdot(a, b):
    """Real inner product Re sum conj(a) b over device tensors, in FP64."""
    import torch
    return float(torch.sum((a.conj() * b).real).item()) if a is not None else 0.0


def _nrm(a):
    import torch
    return float(torch.linalg.vector_norm(a).item()) if a is not None else 0.0


def test_full_size_collision_vjp_adjoint_identity(big):
    """Full-size exact-adjoint identities of kbe_collision_vjp (overwrite mode, as benchmarked):
    linear in G for fixed Sigma, linear in Sigma for fixed G."""
    import torch
    kbe = big["kbe"]
    G, Wo, NROW, NT = big["G"], big["Wo"], big["NROW"], big["NT"]
    Wd = kbe.Weights(to_dev(Wo.w), to_dev(Wo.wfull), to_dev(Wo.wf))
    sig = tuple(to_dev(x) for x in big["sig_o"])
    gen = torch.Generator(device="cuda").manual_seed(2025)

    def rnd(x):
        return torch.randn(x.shape, dtype=x.dtype, device=x.device, generator=gen)

    cot = (rnd(G.rdiag), rnd(G.rdiag), rnd(G.rdiag), rnd(G.mat))
    gG = kbe.Green(torch.empty_like(G.kp), torch.empty_like(G.rdiag), torch.empty_like(G.tv),
                   torch.empty_like(G.mat))
    _print("collision vjp")
    gG, gsig = kbe.collision_vjp(G, sig, Wd, NROW, 0, NT, cot,
                                 kbe.OUT_ALL | kbe.GRAD_OVERWRITE, gG)
    # Green's function direction
    dG = kbe.Green(rnd(G.kp), rnd(G.rdiag), rnd(G.tv), rnd(G.mat))
    out = kbe.collision(dG, sig, Wd, NROW)
    lhs = sum(_rdot(c, o) for c, o in zip(cot, out))
    rhs = sum(_rdot(g, d) for g, d in zip((gG.kp, gG.rdiag, gG.tv, gG.mat),
                                          (dG.kp, dG.rdiag, dG.tv, dG.mat)))
    scale = sum(_nrm(c) * _nrm(o) for c, o in zip(cot, out))
    _print("G direction", lhs, rhs, scale)
    assert abs(lhs - rhs) <= 1e-12 * scale
    del dG, out
    # self-energy direction
    dS = tuple(rnd(x) for x in sig)
    out = kbe.collision(G, dS, Wd, NROW)
    lhs = sum(_rdot(c, o) for c, o in zip(cot, out))
    rhs = sum(_rdot(g, d) for g, d in zip(gsig, dS))
    scale = sum(_nrm(c) * _nrm(o) for c, o in zip(cot, out))
    _print("Sigma direction", lhs, rhs, scale)
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_full_size_sigma_vjp(big):
    """kbe_sigma_2b_vjp at full size against the oracle's adjoint, on every block it touches
    (row and column n of kp, rdiag[n], tv row n) and on dL/du; every other block stays 0."""
    import torch
    kbe = big["kbe"]
    G, N, NROW = big["G"], big["N"], big["NROW"]
    gs = tuple(synth.normal(77, k, x.shape) for k, x in enumerate(big["sig_o"]))
    gG = kbe.Green(torch.zeros_like(G.kp), torch.zeros_like(G.rdiag), torch.zeros_like(G.tv),
                   torch.zeros_like(G.mat))
    gu = torch.zeros(N, dtype=torch.float64, device="cuda")
    kbe.sigma_2b_vjp(G, to_dev(big["u"]), NROW, tuple(to_dev(x) for x in gs), gG, gu)
    zk = np.zeros(big["kp"].shape, np.complex128)  # calloc-backed: untouched pages stay unmapped
    ref = oracle.sigma_row_vjp(big["Go"], big["u"], NROW, gs,
                               grads=(zk, np.zeros(big["rd"].shape, np.complex128),
                                      np.zeros(big["tv"].shape, np.complex128)))
    rk, rr, rt, ru = ref
    n = NROW
    col = to_host(gG.kp[:, n])
    row = to_host(gG.kp[n, :])
    for got, want, name in ((col, rk[:, n], "kp column n"), (row, rk[n, :], "kp row n"),
                            (to_host(gG.rdiag), rr, "rdiag"), (to_host(gG.tv[n]), rt[n], "tv row n")):
        d = np.linalg.norm((got - want).ravel())
        assert d <= RTOL * np.linalg.norm(want.ravel()), name
    np.testing.assert_allclose(to_host(gu), ru, rtol=1e-12, atol=0)
    # nothing outside row/column n of kp and row n of tv
    gG.kp[:, n] = 0
    gG.kp[n, :] = 0
    assert float(torch.abs(gG.kp).max().item()) == 0.0
    assert float(torch.abs(gG.tv[:n]).max().item()) == 0.0
    assert float(torch.abs(gG.mat).max().item()) == 0.0
