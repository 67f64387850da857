"""The adjoint of batches of rows (kbe_collision_batch_vjp) against the oracle's row adjoint,
on systems of every orbital-count path, with output subsets (exact zeros where no selected output
reads a block), under graph capture and replay, and on the full batching workload (sampled)."""
import numpy as np
import pytest

import oracle
import synth
from tests.cases import bnorm, to_dev, to_host
from tests.test_gpu_batch import _cross_from_system, _system

pytestmark = pytest.mark.gpu
F3 = 0x1 | 0x2 | 0x4
NAMES = ("sig_ret", "sig_les", "sig_tv", "col", "row", "rdiag", "tv")


def _print(*a):
    print(*a, flush=True)


def _item(kbe, cr, n, m, wn, wm, wf, flags):
    c = lambda a: to_dev(np.ascontiguousarray(a))
    ntau = cr["stv"].shape[0]
    return kbe.BatchItem(n=n, m=m, sig_ret=c(cr["ret"]), sig_les=c(cr["les"]), col=c(cr["col"]),
                         row=c(cr["row"]), rdiag=c(cr["rdiag"]), wn=c(wn), wm=c(wm),
                         sig_tv=c(cr["stv"]) if ntau else None, tv=c(cr["tv"]) if ntau else None,
                         wtau=c(wf) if ntau else None, flags=flags)


def _check(bv, refs):
    for i, ref in enumerate(refs):
        got = bv.g[i]
        for name, want in zip(NAMES, ref):
            g = got[name]
            if g is None:
                assert want.size == 0 or not np.any(want), (i, name)
                continue
            g = to_host(g)
            zero = bnorm(want) == 0 if want.ndim == 3 else np.array(not np.any(want))
            if want.ndim == 3:
                assert np.all(g[zero] == 0), (i, name, "zero blocks")
                err, sc = bnorm(g - want), bnorm(want)
                assert np.all(err <= 1e-12 * sc + 1e-300), (i, name, float((err / (sc + 1e-300)).max()))
            else:
                assert np.linalg.norm(g - want) <= 1e-12 * np.linalg.norm(want) + 1e-300, (i, name)


def _mixed(kbe, seed=1):
    systems = [_system(*a) for a in [(1, 30, 0, 11), (2, 64, 64, 12), (3, 40, 7, 13),
                                     (4, 150, 70, 18), (5, 50, 0, 14), (8, 90, 20, 15),
                                     (9, 21, 3, 20), (13, 27, 0, 21), (16, 70, 12, 17)]]
    rng = np.random.default_rng(seed)
    items, cots, refs = [], [], []
    for si, S in enumerate(systems):
        nt, N, ntau = S["nt"], S["N"], S["ntau"]
        for k, (n, m, f) in enumerate([(nt - 1, 0, F3), (nt - 1, nt - 1, F3), (nt - 1, nt // 2, F3),
                                       (nt // 2, nt // 5, 0x1), (nt // 3, nt // 3, 0x2 | 0x4),
                                       (0, 0, F3)]):
            cr = _cross_from_system(S, n, m, 300 * si + k)
            W = S["W"]
            wf = W.wfull if ntau else None
            cm = lambda: rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
            cot = (cm(), cm(), cm())
            items.append(_item(kbe, cr, n, m, W.w[n, :n + 1], W.w[m, :m + 1], wf, f))
            cots.append(tuple(to_dev(c) for c in cot))
            refs.append(oracle.collision_row_vjp(N, ntau, n, m, (cr["ret"], cr["les"], cr["stv"]),
                                                 cr["col"], cr["row"], cr["rdiag"], cr["tv"],
                                                 W.w[n, :n + 1], W.w[m, :m + 1], wf, cot, f))
    order = sorted(range(len(items)), key=lambda r: (r * 7919) % 97)  # interleave systems
    return ([items[r] for r in order], [cots[r] for r in order], [refs[r] for r in order])


def test_batch_vjp_matches_oracle(gpu):
    import torch
    kbe = gpu
    items, cots, refs = _mixed(kbe)
    bv = kbe.BatchVJP(items, cots)
    for g in bv.g:  # poison: every block must be written
        for x in g.values():
            if x is not None:
                x.fill_(float("nan"))
    _print("batch vjp", bv.count, "items")
    bv.run()
    torch.cuda.synchronize()
    _check(bv, refs)


def test_batch_vjp_graph_capture_replay(gpu):
    import torch
    kbe = gpu
    items, cots, refs = _mixed(kbe, seed=2)
    bv = kbe.BatchVJP(items, cots)
    bv.run()
    torch.cuda.synchronize()
    eager = [to_host(x) for g in bv.g for x in g.values() if x is not None]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bv.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bv.run()
    for rep in range(3):
        for g in bv.g:
            for x in g.values():
                if x is not None:
                    x.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [to_host(x) for g in bv.g for x in g.values() if x is not None]
        for a, b in zip(got, eager):
            assert np.array_equal(a, b), rep
    _check(bv, refs)


def test_batch_vjp_full_size_sampled(gpu):
    """The batching workload (256 rows, N in {2,4,8,16}, n up to 4096, ntau = 256) in one adjoint
    launch; sampled rows against the oracle's row adjoint."""
    import torch
    kbe = gpu
    B = synth.BATCH
    specs = synth.batch_specs(B["seed"], B["count"], B["Ns"], B["nmin"], B["nmax"])
    _, _, wfull = oracle.tau_weights(B["beta"], B["ntau"], B["tau_order"])
    sample = sorted({0, len(specs) - 1} | {next(i for i, s in enumerate(specs) if s.N == N)
                                          for N in B["Ns"]})
    items, cots, keep = [], [], {}
    rng = np.random.default_rng(5)
    _print("full batch vjp: building")
    for i, sp in enumerate(specs):
        cr = synth.batch_cross(sp, B["ntau"], B["hmin"], B["hmax"], B["omin"], B["omax"])
        w = oracle.weights(cr["t"], cr["order"])
        wn, wm = w[sp.n].copy(), w[sp.m, :sp.m + 1].copy()
        del w
        cm = lambda: rng.normal(size=(sp.N, sp.N)) + 1j * rng.normal(size=(sp.N, sp.N))
        cot = (cm(), cm(), cm())
        items.append(_item(kbe, cr, sp.n, sp.m, wn, wm, wfull, F3))
        cots.append(tuple(to_dev(c) for c in cot))
        if i in sample:
            keep[i] = oracle.collision_row_vjp(sp.N, B["ntau"], sp.n, sp.m,
                                               (cr["ret"], cr["les"], cr["stv"]), cr["col"],
                                               cr["row"], cr["rdiag"], cr["tv"], wn, wm, wfull,
                                               cot, F3)
    bv = kbe.BatchVJP(items, cots)
    _print("full batch vjp: run")
    bv.run()
    torch.cuda.synchronize()
    for i in sample:
        _print("row", i, specs[i])
    sub = type("S", (), {})()
    sub.g = [bv.g[i] for i in sample]
    _check(sub, [keep[i] for i in sample])
