"""Batches of history rows (kbe_collision_batch): many rows of independent systems with mixed
orbital counts and lengths in one launch, against the oracle to the FP64 bar, at every chunk
size, run to run, under graph capture and replay, and at the full batching size (sampled)."""
import numpy as np
import pytest

import oracle
import synth
from tests.cases import RTOL, batch_item, device_weights, row_scales, to_dev, to_host

pytestmark = pytest.mark.gpu

F3 = 0x1 | 0x2 | 0x4  # I^R, I^<, I^]


def _print(*a):
    print(*a, flush=True)


def _cross_from_system(S, n, m, seed):
    """A row's cross arrays cut from a full synthetic system (plus its own self-energy row)."""
    N, ntau, t = S["N"], S["ntau"], S["t"]
    ret, les, stv = synth.sigma_row(seed, N, n, ntau, t)
    kp, tv = S["kp"], S["tv"]
    return dict(ret=ret, les=les, stv=stv, col=kp[:m + 1, m], row=kp[m, :n + 1],
                rdiag=S["rd"][m], tv=tv[m] if ntau else np.zeros((0, N, N), np.complex128))


def _system(N, nt, ntau, seed):
    t, order = synth.grid(seed, nt, 0.02, 0.08, 3, 6)
    S = dict(N=N, nt=nt, ntau=ntau, t=t, kp=synth.kp(seed, N, t), rd=synth.rdiag(N, nt),
             tv=synth.tv(seed, N, ntau, t), mat=synth.mat(seed, N, ntau))
    S["W"] = oracle.Weights.build(t, order, 3.0 if ntau else None, ntau, 5)
    S["G"] = oracle.Green(S["kp"], S["rd"], S["tv"], S["mat"])
    return S


@pytest.fixture(scope="module")
def mixed(gpu):
    """Rows of eleven systems (N = 1, 2, 3, 4, 5, 6, 8, 9, 11, 13, 16: every code path and
    padding; with and without a thermal branch), including m = 0, m = n, n = 0, rows longer than
    one 64-term pass, and output subsets, interleaved in one batch."""
    kbe = gpu
    systems = [_system(*a) for a in [(1, 30, 0, 11), (2, 64, 64, 12), (3, 40, 7, 13),
                                     (4, 150, 70, 18), (5, 50, 0, 14), (6, 33, 5, 19),
                                     (8, 90, 20, 15), (9, 21, 3, 20), (11, 45, 9, 16),
                                     (13, 27, 0, 21), (16, 70, 12, 17)]]
    rows = []
    for si, S in enumerate(systems):
        nt = S["nt"]
        for k, (n, m, f) in enumerate([(nt - 1, 0, F3), (nt - 1, nt - 1, F3),
                                       (nt - 1, nt // 2, F3), (nt // 2, nt // 5, 0x1),
                                       (nt // 3, nt // 3, 0x2 | 0x4), (0, 0, F3)]):
            rows.append((si, n, m, f, 100 * si + k))
    order = sorted(range(len(rows)), key=lambda r: (rows[r][4] * 7919) % 101)  # interleave
    items, refs = [], []
    for r in order:
        si, n, m, f, seed = rows[r]
        S = systems[si]
        cr = _cross_from_system(S, n, m, seed)
        W = S["W"]
        wf = W.wfull if S["ntau"] else None
        items.append(batch_item(kbe, cr, n, m, W.w[n, :n + 1], W.w[m, :m + 1], wf, f))
        sig = (cr["ret"], cr["les"], cr["stv"])
        of = (f & 0x3) | (f & 0x4 if S["ntau"] else 0)
        IR, IL, Itv, _ = oracle.collision(S["G"], sig, W, n, m, m + 1, of)
        sc = row_scales(S["N"], S["ntau"], n, m, cr, W.w[n], W.w[m], wf)
        refs.append(dict(f=f, ref=(IR[0], IL[0], Itv[0]), sc=sc, N=S["N"], nm=(n, m)))
    return kbe.Batch(items), refs


def _check(batch, refs, rtol=RTOL):
    for i, r in enumerate(refs):
        for k, (got, name) in enumerate(((batch.IR[i], "IR"), (batch.IL[i], "IL"),
                                         (batch.Itv[i], "Itv"))):
            if not r["f"] & (1 << k):
                assert got is None
                continue
            g, want = to_host(got), r["ref"][k]
            err = np.linalg.norm(g - want)
            assert err <= rtol * r["sc"][k] + 1e-300, (i, name, r["N"], r["nm"], err, r["sc"][k])


@pytest.mark.parametrize("chunk", [0, 32, 128, 256])
def test_batch_matches_oracle(mixed, chunk):
    import torch
    batch, refs = mixed
    _print("batch chunk", chunk, "items", batch.count)
    batch.run(chunk)
    torch.cuda.synchronize()
    _check(batch, refs)


def test_batch_deterministic_and_chunks_agree(mixed):
    import torch
    batch, _ = mixed
    outs = {}
    for chunk in (32, 64, 32):
        batch.run(chunk)
        torch.cuda.synchronize()
        outs.setdefault(chunk, []).append([to_host(x) for x in batch.IR + batch.IL + batch.Itv
                                           if x is not None])
    for a, b in zip(*outs[32]):
        assert np.array_equal(a, b)  # bitwise run to run
    for a, b in zip(outs[32][0], outs[64][0]):
        assert np.linalg.norm(a - b) <= 1e-13 * (np.linalg.norm(b) + 1e-300)


def test_batch_graph_capture_replay(mixed):
    """The call allocates nothing and copies nothing from the host: captured once, every replay
    (with eager work and synchronisation between replays) reproduces the eager result."""
    import torch
    batch, refs = mixed
    batch.run(64)
    torch.cuda.synchronize()
    eager = [to_host(x) for x in batch.IR + batch.IL + batch.Itv if x is not None]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run(64)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run(64)
    for rep in range(3):
        for x in batch.IR + batch.IL + batch.Itv:
            if x is not None:
                x.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [to_host(x) for x in batch.IR + batch.IL + batch.Itv if x is not None]
        for a, b in zip(got, eager):
            assert np.array_equal(a, b), rep
    _check(batch, refs)


@pytest.mark.parametrize("sigma", ["per_row", "batched"])
def test_batch_graph_with_sigma_rows(gpu, sigma):
    """[self-energy rows -> kbe_collision_batch (plan, stream, reduce)] as one captured graph, for
    rows of two systems held in KP storage on the device (N = 4 and 16): the rows' self-energies
    (kbe_sigma_2b per row, with the rows' kp columns gathered into arrays; or every row in one
    kbe_sigma_2b_batch launch, with the columns read in place) and the batch reading both.  Every replay (outputs and intermediates set to NaN
    before it, with eager work and synchronisation between replays) equals the eager pipeline bit
    for bit, and that matches the oracle (its own self-energy rows) to the FP64 bar."""
    import ctypes
    import torch
    kbe = gpu
    L = kbe.lib()
    systems = []
    for N, nt, ntau, seed, uval in [(4, 40, 6, 31, 0.8), (16, 30, 5, 32, 1.1)]:
        S = _system(N, nt, ntau, seed)
        S["u"] = np.full(N, uval)
        S["Gd"] = kbe.Green(to_dev(S["kp"]), to_dev(S["rd"]), to_dev(S["tv"]), to_dev(S["mat"]))
        S["Wd"] = device_weights(S["W"])
        S["ud"] = to_dev(S["u"])
        systems.append(S)
    rows = [(0, 39, 0), (0, 39, 39), (0, 25, 11), (0, 10, 10), (1, 29, 3), (1, 29, 29),
            (1, 17, 9), (1, 0, 0)]
    z = lambda *sh: torch.empty(sh, dtype=torch.complex128, device="cuda")
    sigb = kbe.SigmaBatch([(systems[si]["Gd"], systems[si]["ud"], n) for si, n, _ in rows])
    sig_bufs, col_bufs, items, refs = [], [], [], []
    for r, (si, n, m) in enumerate(rows):
        S = systems[si]
        N, ntau, Gd, Wd = S["N"], S["ntau"], S["Gd"], S["Wd"]
        sb = sigb.rows[r]
        sig_bufs.append((si, n, sb))
        if sigma == "batched":  # kp column m in place: block s at kp + (s ldt + m) blocks
            cb, cld = Gd.kp[0, m], Gd.kp.shape[1]
        else:
            cb, cld = z(m + 1, N, N), 0
            col_bufs.append((si, m, cb))
        items.append(kbe.BatchItem(n=n, m=m, sig_ret=sb[0], sig_les=sb[1], col=cb,
                                   row=Gd.kp[m, :n + 1], rdiag=Gd.rdiag[m], wn=Wd.w[n, :n + 1],
                                   wm=Wd.w[m, :m + 1], sig_tv=sb[2], tv=Gd.tv[m], wtau=Wd.wtau,
                                   flags=F3, col_ld=cld))
        sig = oracle.sigma_row(S["G"], S["u"], n)
        IR, IL, Itv, _ = oracle.collision(S["G"], sig, S["W"], n, m, m + 1, F3)
        cr = dict(ret=sig[0], les=sig[1], stv=sig[2], col=S["kp"][:m + 1, m],
                  row=S["kp"][m, :n + 1], rdiag=S["rd"][m], tv=S["tv"][m])
        sc = row_scales(N, ntau, n, m, cr, S["W"].w[n], S["W"].w[m], S["W"].wfull)
        refs.append(dict(f=F3, ref=(IR[0], IL[0], Itv[0]), sc=sc, N=N, nm=(n, m)))
    batch = kbe.Batch(items)

    def pipeline():
        st = torch.cuda.current_stream().cuda_stream
        if sigma == "batched":
            sigb.run()
        else:
            for si, n, sb in sig_bufs:
                S = systems[si]
                row = kbe._row(*sb)
                assert L.kbe_sigma_2b(ctypes.byref(S["Gd"].c()), S["ud"].data_ptr(), n,
                                      ctypes.byref(row), st) == 0
        for si, m, cb in col_bufs:
            cb.copy_(systems[si]["Gd"].kp[:m + 1, m])
        batch.run(64)

    outs = lambda: [to_host(x) for x in batch.IR + batch.IL + batch.Itv]
    pipeline()
    torch.cuda.synchronize()
    eager = outs()
    _check(batch, refs)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pipeline()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pipeline()
    nan = float("nan")
    for rep in range(3):
        for _, _, sb in sig_bufs:
            for x in sb:
                x.fill_(nan)
        for _, _, cb in col_bufs:
            cb.fill_(nan)
        for x in batch.IR + batch.IL + batch.Itv:
            x.fill_(nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs(), eager):
            assert np.array_equal(a, b), rep


def test_batch_columns_in_place(gpu):
    """Items that read kp column m of a KP storage in place (col_ld = ldt) give bit for bit the
    results of the same items over gathered column arrays, forward (kbe_collision_batch) and
    adjoint (kbe_collision_batch_vjp), for rows of two systems (N = 3 and 16, one with a padded
    row stride)."""
    import torch
    kbe = gpu
    F = 0x1 | 0x2 | 0x4
    built = []
    for N, nt, ntau, seed, pad in [(3, 45, 6, 41, 0), (16, 28, 5, 42, 5)]:
        S = _system(N, nt, ntau, seed)
        kp = S["kp"]
        if pad:
            kpp = np.zeros((nt, nt + pad, N, N), np.complex128)
            kpp[:, :nt] = kp
            kp = kpp
        Gd = kbe.Green(to_dev(kp), to_dev(S["rd"]), to_dev(S["tv"]), to_dev(S["mat"]))
        built.append((S, Gd, device_weights(S["W"])))
    rows = [(0, 44, 0), (0, 44, 44), (0, 30, 12), (0, 0, 0), (1, 27, 27), (1, 27, 4),
            (1, 15, 15), (1, 9, 2)]
    both = {}
    for mode in ("gathered", "in_place"):
        items, cots = [], []
        for r, (si, n, m) in enumerate(rows):
            S, Gd, Wd = built[si]
            N = S["N"]
            ret, les, stv = synth.sigma_row(500 + r, N, n, S["ntau"], S["t"])
            if mode == "in_place":
                col, cld = Gd.kp[0, m], Gd.kp.shape[1]
            else:
                col, cld = Gd.kp[:m + 1, m].contiguous(), 0
            items.append(kbe.BatchItem(n=n, m=m, sig_ret=to_dev(ret), sig_les=to_dev(les),
                                       col=col, row=Gd.kp[m, :n + 1], rdiag=Gd.rdiag[m],
                                       wn=Wd.w[n, :n + 1], wm=Wd.w[m, :m + 1], sig_tv=to_dev(stv),
                                       tv=Gd.tv[m], wtau=Wd.wtau, flags=F, col_ld=cld))
            cots.append(tuple(to_dev(synth.normal(600 + r, k, (N, N))) for k in range(3)))
        b = kbe.Batch(items)
        b.run(32)
        v = kbe.BatchVJP(items, cots)
        v.run()
        torch.cuda.synchronize()
        both[mode] = ([to_host(x) for x in b.IR + b.IL + b.Itv],
                      [{k: to_host(x) for k, x in g.items()} for g in v.g])
    fa, ga = both["gathered"]
    fb, gb = both["in_place"]
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)
    for x, y in zip(ga, gb):
        for k in x:
            assert (x[k] is None and y[k] is None) or np.array_equal(x[k], y[k]), k


def test_batch_autotuner(mixed):
    import torch
    batch, refs = mixed
    best, times = batch.tune()
    _print("tuner", best, times)
    assert best in (32, 64, 128, 256)
    assert all(v > 0 for v in times.values())
    batch.run(best)
    torch.cuda.synchronize()
    _check(batch, refs)


def test_batch_full_size_sampled(gpu):
    """The batching workload at full size (256 rows, N in {2,4,8,16}, n up to 4096, ntau = 256),
    oracle weights; sampled rows against the oracle's row function, one launch."""
    import torch
    kbe = gpu
    B = synth.BATCH
    specs = synth.batch_specs(B["seed"], B["count"], B["Ns"], B["nmin"], B["nmax"])
    _print("full batch: building", len(specs), "rows")
    items, keep = [], {}
    sample = sorted({0, 1, 2, len(specs) - 1} |
                    {max(range(len(specs)), key=lambda i: specs[i].n * specs[i].N ** 2)} |
                    {next(i for i, s in enumerate(specs) if s.N == N) for N in B["Ns"]})
    _, _, wfull = oracle.tau_weights(B["beta"], B["ntau"], B["tau_order"])
    for i, sp in enumerate(specs):
        cr = synth.batch_cross(sp, B["ntau"], B["hmin"], B["hmax"], B["omin"], B["omax"])
        w = oracle.weights(cr["t"], cr["order"])
        wn, wm = w[sp.n].copy(), w[sp.m, :sp.m + 1].copy()
        items.append(batch_item(kbe, cr, sp.n, sp.m, wn, wm, wfull, F3))
        if i in sample:
            keep[i] = (cr, wn, wm)
        del w
    batch = kbe.Batch(items)
    _print("full batch: run")
    batch.run()
    torch.cuda.synchronize()
    for i in sample:
        sp = specs[i]
        cr, wn, wm = keep[i]
        ref = oracle.collision_row(sp.N, B["ntau"], sp.n, sp.m, (cr["ret"], cr["les"], cr["stv"]),
                                   cr["col"], cr["row"], cr["rdiag"], cr["tv"], wn, wm, wfull, F3)
        sc = row_scales(sp.N, B["ntau"], sp.n, sp.m, cr, wn, wm, wfull)
        _print("row", i, sp)
        for k, got in enumerate((batch.IR[i], batch.IL[i], batch.Itv[i])):
            err = np.linalg.norm(to_host(got) - ref[k])
            assert err <= RTOL * sc[k], (i, k, err, sc[k])


def test_batch_tile_table(mixed, tmp_path):
    """The per-group autotuner: every item gets its group's chunk (one of the allowed sizes); the
    table runs through chunk 0 to the oracle bar; a saved and reloaded table gives the same
    chunks and bitwise the same results."""
    import torch
    batch, refs = mixed
    ms, table = batch.tune_groups()
    _print("tile table", ms, table)
    assert ms > 0 and set(table.values()) <= {32, 64, 128, 256}
    for i, it in enumerate(batch.items):
        assert batch._host[i].chunk == table[batch.group(it.N, it.n)]
    batch.run(0)
    torch.cuda.synchronize()
    _check(batch, refs)
    first = [to_host(x) for x in batch.IR + batch.IL + batch.Itv if x is not None]
    path = tmp_path / "tiles.json"
    batch.save_table(path)
    batch.apply_table({})            # every item back to the default chunk
    assert all(batch._host[i].chunk == 0 for i in range(batch.count))
    batch.run(0)
    torch.cuda.synchronize()
    _check(batch, refs)
    batch.load_table(path)
    assert batch.table() == table
    batch.run(0)
    torch.cuda.synchronize()
    again = [to_host(x) for x in batch.IR + batch.IL + batch.Itv if x is not None]
    for a, b in zip(first, again):
        assert np.array_equal(a, b)
    batch.apply_table({})
