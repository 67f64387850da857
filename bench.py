"""Benchmark of the history-integral hot path on one MI355X.

One step = the whole path over the 16-orbital, 2048-point workload (n_tau = 512):
  kbe_weights -> kbe_sigma_2b (row n = 2047) -> kbe_collision (all m <= n, all four integrals)
  -> kbe_collision_vjp (all cotangents) -> kbe_sigma_2b_vjp,
all through the C ABI of libkbe.so.  Inputs are seeded synthetic arrays, resident in HBM before
timing starts.  After the timed steps, the forward and adjoint collision calls are also timed on
the 8-orbital differentiation shape (nt = 1024, n_tau = 256: the small-block path, bound by HBM
bandwidth), and the batching workload (256 independent rows, N in {2,4,8,16}, n up to 4096) is
timed as one batched launch, as a graph replay and as 256 separate launches, and 256 rows of the
headline system as one batched launch against 256 plain kbe_collision calls; the end-to-end
gradient of a propagation (kbe_propagate and its adjoint on the 8-orbital grid), the adaptive
propagation of the 8-site chain (kbe_propagate_adaptive) and the interacting equilibrium solve
that starts it (kbe_equilibrium, at 8 and 16 orbitals) are timed too; all are reported beside
the step, with the FP64 matrix-core and HBM ceilings measured live by the library's
microbenchmarks.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-propagation]
  python bench.py --adaptive-only      # only the adaptive propagation and equilibrium cases
  python bench.py --copy-calibration   # 3 plain 1 GiB device copies (PMC byte-counter scale)
  python bench.py --ceilings           # the ceiling microbenchmarks -> profiles/ceilings.json
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "collision-integral FP64 GFLOP/s + HBM GB/s, N_orb=16 n=2048; adjoint/fwd time"
HBM_PEAK_GBS = 8000.0
MFMA_F64_PEAK_TFLOPS = 78.6
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CUs x 128 FP64 flop per clock x 2.4 GHz
RIDGE = MFMA_F64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
CEILING_SOURCES = ("kbe_ceilings.hip",)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ceilings(kbe, torch, reps=5):
    """The library's ceiling microbenchmarks (kbe_ceilings.hip), timed with HIP events on the
    stream they run on: independent chains of v_mfma_f64_4x4x4 and v_mfma_f64_16x16x4 products
    over the whole chip, and a 4 GiB HBM read and copy.  Median of `reps` launches after two
    warm-up launches."""
    import ctypes
    L = kbe.lib()
    L.kbe_internal_ceiling_run.restype = ctypes.c_int32
    L.kbe_internal_ceiling_run.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.c_void_p]
    L.kbe_internal_ceiling_counts.restype = ctypes.c_double
    L.kbe_internal_ceiling_counts.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    L.kbe_internal_ceiling_out_count.restype = ctypes.c_int64
    dev = torch.device("cuda:0")
    out = torch.empty(L.kbe_internal_ceiling_out_count(), dtype=torch.float64, device=dev)
    nbytes = 4 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream(dev).cuda_stream
    res = {}
    for kind, name, iters, unit in ((0, "mfma_f64_4x4x4", 2000, 1e12),
                                    (1, "mfma_f64_16x16x4", 500, 1e12),
                                    (2, "hbm_read", 0, 1e9), (3, "hbm_copy", 0, 1e9)):
        run = lambda: L.kbe_internal_ceiling_run(kind, src.data_ptr(), dst.data_ptr(), nbytes,
                                                 out.data_ptr(), iters, st)
        for _ in range(2):
            assert run() == 0
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            assert run() == 0
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        rate = L.kbe_internal_ceiling_counts(kind, nbytes, iters) / float(np.median(ts)) / unit
        res[name + ("_tflops" if kind < 2 else "_gbs")] = rate
    del src, dst
    torch.cuda.empty_cache()
    res["source_hash"] = kernel_source_hash(CEILING_SOURCES)
    return res


def counts(N, nt, ntau, n):
    """Algorithmic FLOP and HBM bytes of one forward and one adjoint call at row n, all m.
    FLOP = 8 per complex multiply-add of the block products the method needs; bytes = each
    required array block read once and each output block written once."""
    n1 = n + 1
    blk_flop = 8.0 * N ** 3
    blk = 16.0 * N * N
    fwd_terms = n1 * n1 + n1 * (n1 + 1) / 2 + n1 * ntau + ntau * n1 + ntau * (ntau + 1)
    fwd_read = (n1 * n1 + n1 + n1 * ntau + ntau + 2 * n1 + ntau) * blk + 8.0 * (n1 * (n1 + 1) / 2 + ntau * ntau)
    fwd_write = (3 * n1 + ntau) * blk
    # adjoint: self-energy gradients (same terms as the forward), Green's-function gradients
    # (the upper triangle gets two terms off the diagonal), Matsubara gradient
    adj_terms = fwd_terms + (n1 * n1 + n1 * (n1 + 1) / 2 + 2 * n1 * ntau + ntau * (ntau + 1))
    adj_read = fwd_read + (3 * n1 + ntau) * blk
    adj_write = (n1 * n1 + n1 + n1 * ntau + ntau + 2 * n1 + ntau) * blk
    return dict(fwd_flop=fwd_terms * blk_flop, fwd_bytes=fwd_read + fwd_write,
                adj_flop=adj_terms * blk_flop, adj_bytes=adj_read + adj_write)


def kernel_source_hash(files=("kbe_collision.hip", "kbe_dev.h")):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2405_08737_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


BATCH_SOURCES = ("kbe_batch.hip", "kbe_dev.h")


def measured_traffic(name="traffic_collision_N16_nt2048.json", files=None):
    """HBM bytes per stream launch from a committed rocprofv3 counter summary, or None when the
    kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_hash") != (kernel_source_hash(files) if files else kernel_source_hash()):
        return None
    return d.get("hbm_bytes_per_call")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_other_rows(w, host, threads):
    """The oracle, as it stands, on bounded samples of the other benchmarked calls, for the
    GPU figures beside it: the whole forward row of the 8-orbital differentiation workload
    (n = 1023, all m, all four integrals), the 32 shortest rows of the batching workload (their
    own weights, I^R, I^<, I^]), and the general four-index self-energy of the headline row at 64
    real-time pairs and 32 tau points.  Rates count the same algorithmic FLOP as the GPU objects."""
    import oracle
    import synth
    oracle.set_threads(threads)
    out = {}
    d = synth.DIFFERENTIATION
    t, order = synth.grid(d.seed, d.nt, d.hmin, d.hmax, d.omin, d.omax)
    G = oracle.Green(synth.kp(d.seed, d.N, t), synth.rdiag(d.N, d.nt),
                     synth.tv(d.seed, d.N, d.ntau, t), synth.mat(d.seed, d.N, d.ntau))
    W = oracle.Weights.build(t, order, d.beta, d.ntau, d.tau_order)
    n = d.nt - 1
    sig = oracle.sigma_row(G, np.full(d.N, d.U), n)
    t0 = time.perf_counter()
    oracle.collision(G, sig, W, n)
    dt = time.perf_counter() - t0
    fl = counts(d.N, d.nt, d.ntau, n)["fwd_flop"]
    out["small_orbital"] = {"sample": f"{d.name}: the whole forward row n={n}", "seconds": dt,
                            "gflops": fl / dt / 1e9}
    del G, W, sig
    B = synth.BATCH
    specs = sorted(synth.batch_specs(B["seed"], B["count"], B["Ns"], B["nmin"], B["nmax"]),
                   key=lambda sp: sp.n)[:32]
    fl, dt = 0.0, 0.0
    for sp in specs:
        cr = synth.batch_cross(sp, B["ntau"], B["hmin"], B["hmax"], B["omin"], B["omax"])
        Wb = oracle.Weights.build(cr["t"], cr["order"], B["beta"], B["ntau"], B["tau_order"])
        t0 = time.perf_counter()
        oracle.collision_row(sp.N, B["ntau"], sp.n, sp.m, (cr["ret"], cr["les"], cr["stv"]),
                             cr["col"], cr["row"], cr["rdiag"], cr["tv"], Wb.w[sp.n],
                             Wb.w[sp.m, :sp.m + 1], Wb.wfull)
        dt += time.perf_counter() - t0
        fl += 8.0 * sp.N ** 3 * ((sp.n + 1) + (sp.m + 1) + B["ntau"])
    out["batching"] = {"sample": "the 32 shortest rows of the batching workload "
                                 f"(n {specs[0].n}..{specs[-1].n})",
                       "seconds": dt, "gflops": fl / dt / 1e9}
    t, order, kp, rd, tv, mat = host
    Gh = oracle.Green(kp, rd, tv, mat)
    U = synth.coulomb(w.seed, w.N)
    n = w.nt - 1
    s_list, l_list = list(range(n - 63, n + 1)), list(range(32))
    t0 = time.perf_counter()
    oracle.sigma_gf2_row(Gh, U, n, s_list=s_list, l_list=l_list)
    dt = time.perf_counter() - t0
    fl = 24.0 * w.N ** 5 * (2 * len(s_list) + len(l_list))
    out["gf2"] = {"sample": f"{w.name} row n={n}: 64 real-time pairs (both components) and 32 "
                            "tau points", "seconds": dt, "gflops": fl / dt / 1e9}
    oracle.set_threads(threads)
    return out


def cpu_baseline(w, host, target_s=6.0):
    """The oracle, as it stands, timed on the host cores (median of 3 runs each): the small parity
    workload (N = 2, nt = 64, ntau = 64: the whole row) and the headline workload, at one thread
    and at all the threads the process may use.  On the headline the whole forward row (all m, all
    four integrals) is run when a calibration says it takes at most target_s seconds at that
    thread count, else a band of rows m around the middle sized to about target_s (I^R, I^<, I^]).
    `value` is the headline figure at all threads."""
    import oracle
    import synth
    threads_all = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def forward_row(wk, hostk):
        t, order, kp, rd, tv, mat = hostk
        n = wk.nt - 1
        G = oracle.Green(kp, rd, tv, mat)
        W = oracle.Weights.build(t, order, wk.beta, wk.ntau, wk.tau_order)
        sig = oracle.sigma_row(G, np.full(wk.N, wk.U), n)
        return G, W, sig, n

    def measure(wk, hostk, threads):
        oracle.set_threads(threads)
        G, W, sig, n = forward_row(wk, hostk)
        N = wk.N
        blk_flop = 8.0 * N ** 3
        rows_flop = lambda m0, m1: sum((n + 1) + (m + 1) + wk.ntau for m in range(m0, m1)) * blk_flop
        full = rows_flop(0, n + 1) + wk.ntau * ((n + 1) + (wk.ntau + 1)) * blk_flop
        mid = n // 2
        t0 = time.perf_counter()
        oracle.collision(G, sig, W, n, mid, min(n + 1, mid + threads),
                         oracle.F_IR | oracle.F_IL | oracle.F_ITV)
        rate = rows_flop(mid, min(n + 1, mid + threads)) / max(time.perf_counter() - t0, 1e-9)
        if full / rate <= target_s:
            run = lambda: oracle.collision(G, sig, W, n)
            fl, what = full, f"the whole forward row n={n} (all m, all four integrals)"
        else:
            rows = max(threads, int(target_s * rate / rows_flop(mid, mid + 1)) // threads * threads)
            m0 = max(0, mid - rows // 2)
            m1 = min(n + 1, m0 + rows)
            run = lambda: oracle.collision(G, sig, W, n, m0, m1,
                                           oracle.F_IR | oracle.F_IL | oracle.F_ITV)
            fl, what = rows_flop(m0, m1), f"rows m in [{m0},{m1}) of row n={n}: I^R, I^<, I^]"
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            run()
            ts.append(time.perf_counter() - t0)
        dt = float(np.median(ts))
        return {"gflops": fl / dt / 1e9, "threads": threads, "median_s": dt, "runs_s": ts,
                "gflop": fl / 1e9, "sample": what}

    small = synth.PARITY_SMALL
    t0_, o0_ = synth.grid(small.seed, small.nt, small.hmin, small.hmax, small.omin, small.omax)
    host0 = (t0_, o0_, synth.kp(small.seed, small.N, t0_), synth.rdiag(small.N, small.nt),
             synth.tv(small.seed, small.N, small.ntau, t0_), synth.mat(small.seed, small.N, small.ntau))
    res = {"parity_small": {f"threads_{k}": measure(small, host0, k) for k in (1, threads_all)},
           "headline": {f"threads_{k}": measure(w, host, k) for k in (1, threads_all)}}
    oracle.set_threads(threads_all)
    top = res["headline"][f"threads_{threads_all}"]
    return {"value": top["gflops"], "unit": "GFLOP/s", "cores": threads_all, "kind": "oracle",
            "sample": top["sample"] + f" ({top['gflop']:.1f} GFLOP, median of 3 runs)",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "runs": res}


def small_orbital_shape(kbe, torch, dev, reps=5):
    """Forward and adjoint collision calls on the 8-orbital differentiation workload (row
    n = nt - 1, all m), timed with HIP events on the library's stream, after two warm-up calls.
    The sustained figures time `reps` calls issued back to back, as a propagation issues them;
    the isolated figures time single calls after a synchronisation, host launch latency
    included."""
    import synth
    w = synth.DIFFERENTIATION
    N, nt, ntau, n = w.N, w.nt, w.ntau, w.nt - 1
    t, order = synth.grid(w.seed, nt, w.hmin, w.hmax, w.omin, w.omax)
    G = kbe.Green(torch.from_numpy(synth.kp(w.seed, N, t)).to(dev),
                  torch.from_numpy(synth.rdiag(N, nt)).to(dev),
                  torch.from_numpy(synth.tv(w.seed, N, ntau, t)).to(dev),
                  torch.from_numpy(synth.mat(w.seed, N, ntau)).to(dev))
    gG = G.zeros_like()
    u = torch.full((N,), w.U, dtype=torch.float64, device=dev)
    cot = tuple(torch.from_numpy(synth.normal(7, k, (nt if k < 3 else ntau, N, N))).to(dev)
                for k in range(4))
    W = kbe.weights(t, order, ntau, w.beta, w.tau_order, device=dev)
    sig = kbe.sigma_2b(G, u, n)
    flags = kbe.OUT_ALL | kbe.GRAD_OVERWRITE
    for _ in range(2):
        kbe.collision(G, sig, W, n)
        kbe.collision_vjp(G, sig, W, n, 0, n + 1, cot, flags, gG)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def sustained(fn):
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    f_ms = sustained(lambda: kbe.collision(G, sig, W, n))
    b_ms = sustained(lambda: kbe.collision_vjp(G, sig, W, n, 0, n + 1, cot, flags, gG))
    tf, tb = [], []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        kbe.collision(G, sig, W, n)
        e[1].record()
        kbe.collision_vjp(G, sig, W, n, 0, n + 1, cot, flags, gG)
        e[2].record()
        torch.cuda.synchronize()
        tf.append(e[0].elapsed_time(e[1]))
        tb.append(e[1].elapsed_time(e[2]))
    c = counts(N, nt, ntau, n)
    return {"workload": w.name, "N_orb": N, "nt": nt, "n": n, "ntau": ntau, "U": w.U,
            "seed": w.seed, "calls": reps,
            "collision_ms": f_ms, "collision_vjp_ms": b_ms, "adjoint_over_forward": b_ms / f_ms,
            "collision_ms_isolated": float(np.mean(tf)),
            "collision_vjp_ms_isolated": float(np.mean(tb)),
            "collision_gflops": c["fwd_flop"] / f_ms / 1e6,
            "collision_gbps": c["fwd_bytes"] / f_ms / 1e6,
            "collision_hbm_frac": c["fwd_bytes"] / f_ms / 1e6 / HBM_PEAK_GBS,
            "collision_vjp_gbps": c["adj_bytes"] / b_ms / 1e6,
            "algorithmic_bytes": c["fwd_bytes"], "algorithmic_flop": c["fwd_flop"],
            "traffic": measured_traffic("traffic_collision_N8_nt1024.json")}


def graph_pair(kbe, torch, G, u, n, t, order, w, reps=10):
    """[kbe_sigma_2b -> kbe_collision] captured once as a HIP graph and replayed (no host work
    between the kernels), against the same pair issued eagerly; weights computed beforehand."""
    W = kbe.weights(t, order, G.ntau, w.beta, w.tau_order, device=G.device)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    eager = timed(lambda: kbe.collision(G, kbe.sigma_2b(G, u, n), W, n))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        kbe.collision(G, kbe.sigma_2b(G, u, n), W, n)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        kbe.collision(G, kbe.sigma_2b(G, u, n), W, n)
    replay = timed(g.replay)
    del g
    return {"eager_ms": eager, "graph_replay_ms": replay}


def greater_form(kbe, torch, G, u, n, t, order, w, cot, gG, reps=3):
    """The greater form of Eq. KBE2 (KBE_GREATER) on the headline row: kbe_collision and
    kbe_collision_vjp (overwrite mode) back to back, against the lesser form in the same run;
    and kbe_collision_both and its adjoint kbe_collision_both_vjp (both forms from one pass each;
    the adjoint accumulates, so it is compared with the lesser adjoint in accumulate mode) against
    the lesser form alone."""
    W = kbe.weights(t, order, G.ntau, w.beta, w.tau_order, device=G.device)
    sig = kbe.sigma_2b(G, u, n)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fl in (("lesser", kbe.OUT_ALL), ("greater", kbe.OUT_ALL | kbe.GREATER)):
        f = lambda: kbe.collision(G, sig, W, n, flags=fl)
        b = lambda: kbe.collision_vjp(G, sig, W, n, 0, n + 1, cot, fl | kbe.GRAD_OVERWRITE, gG)
        f()
        b()
        torch.cuda.synchronize()
        e = [ev() for _ in range(3)]
        e[0].record()
        for _ in range(reps):
            f()
        e[1].record()
        for _ in range(reps):
            b()
        e[2].record()
        torch.cuda.synchronize()
        out[name] = {"collision_ms": e[0].elapsed_time(e[1]) / reps,
                     "collision_vjp_ms": e[1].elapsed_time(e[2]) / reps}
    out["greater_over_lesser"] = {k: out["greater"][k] / out["lesser"][k]
                                  for k in ("collision_ms", "collision_vjp_ms")}
    # both forms from one pass (kbe_collision_both: the propagations' call), against the lesser
    # form alone and against the two separate calls
    kbe.collision_both(G, sig, W, n)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(reps):
        kbe.collision_both(G, sig, W, n)
    e1.record()
    torch.cuda.synchronize()
    both = e0.elapsed_time(e1) / reps
    cot6 = (cot[0], cot[1], cot[2], cot[3], cot[0], cot[1])
    bv = lambda: kbe.collision_both_vjp(G, sig, W, n, 0, n + 1, cot6, gG)
    bv()
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(reps):
        bv()
    e1.record()
    torch.cuda.synchronize()
    both_vjp = e0.elapsed_time(e1) / reps
    # the lesser adjoint in the same (accumulate) mode, for the comparison of the adjoints
    lv = lambda: kbe.collision_vjp(G, sig, W, n, 0, n + 1, cot, kbe.OUT_ALL, gG)
    lv()
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(reps):
        lv()
    e1.record()
    torch.cuda.synchronize()
    les_acc = e0.elapsed_time(e1) / reps
    out["both_forms"] = {"collision_ms": both, "collision_vjp_ms": both_vjp,
                         "lesser_collision_vjp_accumulate_ms": les_acc,
                         "over_lesser": {"collision_ms": both / out["lesser"]["collision_ms"],
                                         "collision_vjp_ms": both_vjp / les_acc},
                         "forward_over_separate_calls":
                             both / (out["lesser"]["collision_ms"] +
                                     out["greater"]["collision_ms"])}
    return out


def general_u_sigma(kbe, torch, G, n, w, reps=5):
    """kbe_sigma_gf2 on the headline row (same G, n, ntau) with a synthetic symmetric U, calls
    back to back.  Algorithmic FLOP per block: 24 N^5 (two real-by-complex and two complex
    contractions of N^5 multiply-adds); blocks: 2 (n + 1) real-time + ntau mixed."""
    import synth
    N = G.N
    U = torch.from_numpy(synth.coulomb(w.seed, N)).to(G.device)
    for _ in range(2):
        kbe.sigma_gf2(G, U, n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        kbe.sigma_gf2(G, U, n)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flop = 24.0 * N ** 5 * (2 * (n + 1) + G.ntau)
    return {"workload": f"N{N}_nt{G.nt}_ntau{G.ntau} row n={n}, U: symmetric (ij|kl), on-site 1",
            "ms": ms, "algorithmic_flop": flop, "tflops": flop / ms / 1e9,
            "frac_f64_peak": flop / ms / 1e9 / MFMA_F64_PEAK_TFLOPS}


def batch_vs_plain(kbe, torch, dev, G, W, u, nrows=256, seed=1004, reps=5):
    """The same rows run both ways: 256 rows (n, m) of the 16-orbital headline system (n
    log-uniform in [128, nt - 1], m uniform in 0..n), as one kbe_collision_batch launch (items
    reading the system's KP storage in place: kp column m with col_ld = ldt, kp row m, tv row m,
    the weight rows) and as 256 plain kbe_collision calls (m-range [m, m + 1), I^R, I^<, I^]),
    with the outputs, workspace and arguments of the plain calls prepared beforehand.  Both read
    the same algorithmic bytes; the plain calls' outputs are compared with the batch's.  Then the
    whole pipeline [self-energy rows -> batch] eager and captured as one graph, with the rows'
    self-energies by one kbe_sigma_2b call each (and the columns gathered into arrays) or by one
    kbe_sigma_2b_batch launch (and the columns read in place)."""
    import ctypes
    rng = np.random.default_rng(seed)
    nt = G.nt
    ns = np.minimum(np.exp(rng.uniform(np.log(128), np.log(nt - 1), nrows)).astype(int), nt - 1)
    ms = np.array([int(rng.integers(0, n + 1)) for n in ns])
    flags = kbe.OUT_IR | kbe.OUT_IL | kbe.OUT_ITV
    distinct = sorted(set(ns.tolist()))
    sigb = kbe.SigmaBatch([(G, u, n) for n in distinct])  # one launch for every row's Sigma
    sigb.run()
    sigs = dict(zip(distinct, sigb.rows))
    ldt = G.kp.shape[1]

    def make_items(in_place):
        out = []
        for n, m in zip(ns.tolist(), ms.tolist()):
            sr = sigs[n]
            col, cld = (G.kp[0, m], ldt) if in_place else (G.kp[:m + 1, m].contiguous(), 0)
            out.append(kbe.BatchItem(n=n, m=m, sig_ret=sr[0], sig_les=sr[1], col=col,
                                     row=G.kp[m, :n + 1], rdiag=G.rdiag[m], wn=W.w[n, :n + 1],
                                     wm=W.w[m, :m + 1], sig_tv=sr[2], tv=G.tv[m], wtau=W.wtau,
                                     flags=flags, col_ld=cld))
        return out

    items_ip, items_ga = make_items(True), make_items(False)
    batch, batch_ga = kbe.Batch(items_ip), kbe.Batch(items_ga)
    best, _ = batch.tune()
    L = kbe.lib()
    N = G.N
    nb = max(L.kbe_collision_workspace(N, nt, G.ntau, int(n), int(m), int(m) + 1, flags)
             for n, m in zip(ns, ms))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    outs = torch.empty((nrows, 3, N, N), dtype=torch.complex128, device=dev)
    gc, wc = G.c(), W.c()
    rows = [kbe._row(*sigs[int(n)]) for n in ns]
    stream = torch.cuda.current_stream(dev).cuda_stream

    def plain():
        for i in range(nrows):
            o = outs[i]
            st = L.kbe_collision(ctypes.byref(gc), ctypes.byref(rows[i]), ctypes.byref(wc),
                                 int(ns[i]), int(ms[i]), int(ms[i]) + 1, flags,
                                 o[0].data_ptr(), o[1].data_ptr(), o[2].data_ptr(), None,
                                 ws.data_ptr(), nb, stream)
            if st != 0:
                raise RuntimeError(f"kbe_collision: status {st}")

    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn, k):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    stack = lambda b: torch.stack([torch.stack([b.IR[i], b.IL[i], b.Itv[i]])
                                   for i in range(nrows)])
    batched_ms = timed(lambda: batch.run(best), reps)
    gathered_ms = timed(lambda: batch_ga.run(best), reps)
    plain_ms = timed(plain, reps)
    torch.cuda.synchronize()
    got, got_ga = stack(batch), stack(batch_ga)
    rel = float(((got - outs).abs().amax(dim=(2, 3)) /
                 outs.abs().amax(dim=(2, 3)).clamp_min(1e-300)).max())
    ud = u.contiguous()

    def pipeline(batched_sigma):
        st = torch.cuda.current_stream(dev).cuda_stream
        if batched_sigma:
            sigb.run()
            batch.run(best)
            return
        for n in distinct:
            r = kbe._row(*sigs[n])
            if L.kbe_sigma_2b(ctypes.byref(gc), ud.data_ptr(), int(n), ctypes.byref(r), st):
                raise RuntimeError("kbe_sigma_2b failed")
        for it in items_ga:
            it.col.copy_(G.kp[:it.m + 1, it.m])
        batch_ga.run(best)

    pipe = {}
    for mode, bs, b, ref in (("sigma_per_row_columns_gathered", False, batch_ga, got_ga),
                             ("sigma_batched_columns_in_place", True, batch, got)):
        eager_ms = timed(lambda: pipeline(bs), reps)
        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            pipeline(bs)
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            pipeline(bs)
        graph_ms = timed(graph.replay, reps)
        torch.cuda.synchronize()
        pipe[mode] = {"eager_ms": eager_ms, "graph_replay_ms": graph_ms,
                      "graph_equals_eager": bool(torch.equal(stack(b), ref))}
        del graph
    sig_one_ms = timed(sigb.run, reps)
    nbytes = 0.0
    for n, m in zip(ns.tolist(), ms.tolist()):
        blocks = (n + 1) + (m + 1) + (n - m) + (m + 1) + m + 1 + 2 * G.ntau + 3  # as batching()
        nbytes += 16.0 * N * N * blocks + 8.0 * ((n + 1) + (m + 1) + G.ntau)
    same_ga = bool(torch.equal(got, got_ga))
    del batch, batch_ga, ws, outs, sigb
    return {"workload": f"{nrows} rows (n, m) of the N{N}_nt{nt}_ntau{G.ntau} headline system, "
                        f"n log-uniform in [128, {nt - 1}], m uniform in 0..n; I^R, I^<, I^]",
            "chunk": best, "batched_ms": batched_ms, "batched_gathered_columns_ms": gathered_ms,
            "in_place_equals_gathered": same_ga, "plain_calls_ms": plain_ms,
            "speedup_vs_plain": plain_ms / batched_ms, "algorithmic_bytes": nbytes,
            "batched_gbps": nbytes / batched_ms / 1e6, "plain_gbps": nbytes / plain_ms / 1e6,
            "max_rel_diff_batched_vs_plain": rel,
            "pipeline": {"stages": f"{len(distinct)} self-energy rows -> kbe_collision_batch "
                                   f"over {nrows} rows",
                         "sigma_batch_launch_ms": sig_one_ms, **pipe}}


def batching(kbe, torch, dev, reps=10):
    """The batching workload: one kbe_collision_batch launch over 256 rows of independent systems
    (the best common chunk, then the per-group tile table from the library's autotuners), its
    graph replay, the adjoint of the same rows in one kbe_collision_batch_vjp launch, and the
    rows as 256 separate launches.  Algorithmic bytes: every block a row reads once, its three
    outputs written once, its weights (adjoint: the blocks its nonzero gradients read, every
    gradient block written once, the cotangents); FLOP: 8 N^3 per block product."""
    import synth
    B = synth.BATCH
    specs = synth.batch_specs(B["seed"], B["count"], B["Ns"], B["nmin"], B["nmax"])
    c = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    items, nbytes, flop = [], 0.0, 0.0
    wtau = None
    for sp in specs:
        cr = synth.batch_cross(sp, B["ntau"], B["hmin"], B["hmax"], B["omin"], B["omax"])
        W = kbe.weights(cr["t"], cr["order"], B["ntau"], B["beta"], B["tau_order"], device=dev)
        wtau = W.wtau if wtau is None else wtau
        items.append(kbe.BatchItem(n=sp.n, m=sp.m, sig_ret=c(cr["ret"]), sig_les=c(cr["les"]),
                                   col=c(cr["col"]), row=c(cr["row"]), rdiag=c(cr["rdiag"]),
                                   wn=W.w[sp.n].contiguous(), wm=W.w[sp.m, :sp.m + 1].contiguous(),
                                   sig_tv=c(cr["stv"]), tv=c(cr["tv"]), wtau=W.wtau))
        del W
        N, n, m, nt = sp.N, sp.n, sp.m, B["ntau"]
        blocks = (n + 1) + (m + 1) + (n - m) + (m + 1) + m + 1 + 2 * nt + 3
        nbytes += 16.0 * N * N * blocks + 8.0 * ((n + 1) + (m + 1) + nt)
        flop += 8.0 * N ** 3 * ((n + 1) + (m + 1) + nt)
    batch = kbe.Batch(items)
    best, tuned = batch.tune()
    table_ms, table = batch.tune_groups()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn, k):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    common_ms = timed(lambda: batch.run(best), reps)
    batched_ms = timed(lambda: batch.run(0), reps)  # the tile table
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run(0)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run(0)
    graph_ms = timed(g.replay, reps)
    # the adjoint of the same rows (one launch), random cotangents
    cots, vbytes, vflop = [], 0.0, 0.0
    for r, sp in enumerate(specs):
        cots.append(tuple(c(synth.normal(900 + r, k, (sp.N, sp.N))) for k in range(3)))
        N, n, m, nt = sp.N, sp.n, sp.m, B["ntau"]
        prods = (n + 1) + (m + 1) + (m + 1) + n + 1 + 2 * nt  # nonzero gradient blocks
        vbytes += 16.0 * N * N * (prods + 3 * (n + 1) + (m + 1) + 1 + 2 * nt + 3)
        vbytes += 8.0 * ((n + 1) + (m + 1) + nt)
        vflop += 8.0 * N ** 3 * prods
    bv = kbe.BatchVJP(items, cots)
    vjp_ms = timed(bv.run, reps)
    del bv
    singles = [kbe.Batch([it]) for it in items]
    for b in singles:
        b.apply_table(table)
    separate_ms = timed(lambda: [b.run(0) for b in singles], 3)
    Ns = [sp.N for sp in specs]
    return {"workload": "256 rows, N in {2,4,8,16}, n log-uniform [128,4096], m uniform, ntau 256",
            "items": len(specs), "rows_per_N": {str(N): Ns.count(N) for N in B["Ns"]},
            "chunk": best, "tuner_ms": {str(k): v for k, v in tuned.items()},
            "common_chunk_ms": common_ms, "tile_table": dict(sorted(table.items())),
            "tile_table_tuner_ms": table_ms, "batched_ms": batched_ms, "graph_replay_ms": graph_ms,
            "separate_launches_ms": separate_ms, "speedup_vs_separate": separate_ms / batched_ms,
            "gbps": nbytes / batched_ms / 1e6, "hbm_frac": nbytes / batched_ms / 1e6 / HBM_PEAK_GBS,
            "gflops": flop / batched_ms / 1e6, "algorithmic_bytes": nbytes,
            "algorithmic_flop": flop,
            "traffic": measured_traffic("traffic_batch_256rows.json", BATCH_SOURCES),
            "vjp": {"ms": vjp_ms, "algorithmic_bytes": vbytes, "gbps": vbytes / vjp_ms / 1e6,
                    "hbm_frac": vbytes / vjp_ms / 1e6 / HBM_PEAK_GBS,
                    "gflops": vflop / vjp_ms / 1e6, "over_forward": vjp_ms / batched_ms}}


def propagation(kbe, torch, dev):
    """End-to-end gradients through a propagation (kbe_propagate, kbe_propagate_vjp) on the
    8-orbital differentiation grid (1024 points): the forward sweep and the adjoint sweep timed
    with HIP events after one warm-up run, with the loss, its gradients and the drift of the
    particle number (conserved by the method)."""
    import synth
    P = synth.PROPAGATION
    N, nt, last = P["N"], P["nt"], P["last"]
    t, order = synth.grid(P["seed"], nt, P["hmin"], P["hmax"], P["omin"], P["omax"])
    h0 = synth.tight_binding(N)
    out = []
    for U, ntau in P["cases"]:
        mat, rho = synth.free_thermal(h0, P["beta"], ntau)
        pr = kbe.Propagation(t, order, h0, ntau=ntau, beta=P["beta"], mat=mat,
                             rho0=None if ntau else rho, iters=P["iters"],
                             pulse_t0=P["pulse_t0"], pulse_sigma=P["pulse_sigma"], device=dev)
        u = torch.full((N,), U, dtype=torch.float64, device=dev)
        gd = torch.zeros((nt, N), dtype=torch.float64, device=dev)
        gd[-last:, 0] = 1.0
        pr.run(u, P["pulse_amp"])
        pr.vjp(gd)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        d = pr.run(u, P["pulse_amp"])
        e[1].record()
        gu, ga = pr.vjp(gd)
        e[2].record()
        torch.cuda.synchronize()
        fwd, adj = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
        dh = d.cpu().numpy()
        tr = dh.sum(axis=1)
        out.append({"U": U, "ntau": ntau, "forward_ms": fwd, "adjoint_ms": adj,
                    "adjoint_over_forward": adj / fwd, "ms_per_step_forward": fwd / nt,
                    "loss": float(dh[-last:, 0].sum()), "dL_dU": float(gu.sum()),
                    "dL_dA": float(ga), "particle_number_drift": float(np.abs(tr - tr[0]).max()),
                    "workspace_gb": pr.nb / 1e9})
        del pr
        torch.cuda.empty_cache()
    return {"workload": f"N{N}_nt{nt} propagation, steps U[{P['hmin']},{P['hmax']}], orders "
                        f"{P['omin']}..{P['omax']}, beta {P['beta']}, pulse A={P['pulse_amp']} "
                        f"at t={P['pulse_t0']} width {P['pulse_sigma']}, loss n_0 over the last "
                        f"{last} steps, {P['iters']} fixed-point iterations",
            "cases": out}


def adaptive(kbe, torch, dev):
    """The adaptive propagation (kbe_propagate_adaptive): the 8-site chain at U = 1, beta = 10,
    pulse on site 0, variable step and order at rtol 1e-8, atol 1e-10, to t = 40 with the thermal
    branch (256 tau points, from the interacting equilibrium of kbe_equilibrium, whose solve is
    timed too) and without it.  Each case: one warm-up run to t = 0.5,
    then the whole run timed by the host clock (inputs resident, the controller synchronising at
    every fixed-point iteration), the step and order statistics, the particle-number drift, and
    the first `prefix` steps run again on their own (to t = t_prefix) for the oracle comparison.
    Returns the report and, per case, what the oracle needs to replay the prefix."""
    import synth
    A = synth.ADAPTIVE
    N = A["N"]
    h0 = synth.tight_binding(N)
    out, replays = [], []
    for ntau, t_end, prefix in A["cases"]:
        mat, rho = synth.free_thermal(h0, A["beta"], ntau)
        eqr = None
        if ntau:
            # the interacting equilibrium (kbe_equilibrium), timed after a first solve
            kbe.equilibrium(h0, A["U"], A["mu"], A["beta"], ntau, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mat, info = kbe.equilibrium(h0, A["U"], A["mu"], A["beta"], ntau, device=dev)
            torch.cuda.synchronize()
            we = time.perf_counter() - t0
            eqr = {"iterations": info["iterations"], "change": info["change"], "wall_s": we,
                   "ms_per_iteration": 1e3 * we / info["iterations"],
                   "density_0": float(-mat[-1, 0, 0].real)}

        def run(te, cap):
            return kbe.propagate_adaptive(
                h0, A["U"], A["pulse_amp"], te, ntau=ntau, beta=A["beta"], mat=mat,
                rho0=None if ntau else rho, capacity=cap, rtol=A["rtol"], atol=A["atol"],
                h_first=A["h_first"], qmax=A["qmax"], kmax=A["kmax"], maxcor=A["maxcor"],
                pulse_t0=A["pulse_t0"], pulse_sigma=A["pulse_sigma"], device=dev)

        run(0.5, 256)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = run(t_end, A["capacity"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t, d = g["t"], g["dens"].cpu().numpy()
        tr = d.sum(axis=1)
        steps = len(t) - 1
        ks = np.concatenate([np.asarray(k) for k in g["ks"]])
        tp = float(t[prefix])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gp = run(tp, prefix + 8)
        torch.cuda.synchronize()
        wall_p = time.perf_counter() - t0
        same = len(gp["t"]) == prefix + 1 and bool(np.all(gp["q"] == g["q"][: prefix + 1]))
        out.append({
            "ntau": ntau, "t_end": t_end, "steps": steps, "rejected": int(g["rejected"]),
            "wall_s": wall, "ms_per_step": 1e3 * wall / steps,
            "fixed_point_iterations_mean": float(g["m"][1:].mean()),
            "h_min": float(np.diff(t).min()), "h_max": float(np.diff(t).max()),
            "adams_order_histogram": np.bincount(g["q"][1:], minlength=A["qmax"] + 1).tolist(),
            "history_order_histogram": np.bincount(ks, minlength=A["kmax"] + 1).tolist(),
            "particle_number": float(tr[0]),
            "particle_number_drift": float(np.abs(tr - tr[0]).max()),
            "n0_final": float(d[-1, 0]), "workspace_gb": g["workspace_bytes"] / 1e9,
            "initial_state": "interacting equilibrium" if ntau else "free thermal density matrix",
            **({"equilibrium": eqr} if eqr else {}),
            "prefix": {"steps": prefix, "t": tp, "wall_s": wall_p,
                       "ms_per_step": 1e3 * wall_p / prefix, "same_decisions": same}})
        replays.append({"ntau": ntau, "mat": mat.cpu().numpy() if ntau else None, "rho": rho,
                        "replay": g["replay"][: prefix + 1],
                        "dens": d[: prefix + 1],
                        "kp": g["G"].kp[: prefix + 1, : prefix + 1].cpu().numpy(),
                        "gpu_ms_per_step": 1e3 * wall_p / prefix})
        del g, gp
        torch.cuda.empty_cache()
    return ({"workload": f"N{N} chain, U={A['U']}, beta={A['beta']}, half filling, pulse "
                         f"A={A['pulse_amp']} on site 0 at t={A['pulse_t0']} width "
                         f"{A['pulse_sigma']}; rtol {A['rtol']}, atol {A['atol']}, Adams orders "
                         f"1..{A['qmax']}, history orders 1..{A['kmax']}, at most {A['maxcor']} "
                         f"fixed-point corrections; to t=40 with the thermal branch (256 tau "
                         f"points, interacting equilibrium at mu={A['mu']}) and without it",
             "cases": out}, replays)


def equilibrium(kbe, torch, dev):
    """The interacting equilibrium solve (kbe_equilibrium) on the adaptive workload's chain (U = 1,
    beta = 10, half filling) at 8 and 16 orbitals and 256 and 1024 tau points: one solve to warm
    up, then one timed by the host clock (the call synchronises once per iteration).  The
    convolutions do 4 ntau^2 N^3 flops per iteration; their rate is given against the FP64
    vector peak (they run on the vector ALU)."""
    import synth
    A = synth.ADAPTIVE
    out = []
    for N, ntau in ((8, 256), (16, 256), (8, 1024), (16, 1024)):
        h0 = synth.tight_binding(N)
        kbe.equilibrium(h0, A["U"], A["mu"], A["beta"], ntau, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = kbe.equilibrium(h0, A["U"], A["mu"], A["beta"], ntau, device=dev)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        it = info["iterations"]
        flop = 4.0 * ntau * ntau * N ** 3
        out.append({"N": N, "ntau": ntau, "iterations": it, "change": info["change"],
                    "wall_ms": 1e3 * wall, "ms_per_iteration": 1e3 * wall / it,
                    "convolution_gflop_per_iteration": flop / 1e9,
                    "tflops": flop * it / wall / 1e12,
                    "frac_of_fp64_vector_peak": flop * it / wall / 1e12 / FP64_VECTOR_PEAK_TFLOPS})
    return {"workload": f"open chain, U={A['U']}, beta={A['beta']}, mu={A['mu']} (half filling), "
                        f"tol 1e-13, mixing 1/2", "cases": out}


def adaptive_oracle(replays):
    """The oracle replaying the GPU's first steps of each adaptive case on the same grid (same
    orders and history orders): its time per step beside the GPU's, and the largest deviations of
    the densities and of the stored Green's function."""
    import synth
    from oracle import adaptive as oad
    from oracle import propagate as oprop
    A = synth.ADAPTIVE
    h0 = synth.tight_binding(A["N"])
    from oracle import equilibrium as oeq
    res = []
    for r in replays:
        ntau = r["ntau"]
        eqr, mat = {}, None
        if ntau:
            # the oracle's own equilibrium (no input of the oracle comes from the GPU)
            t0 = time.perf_counter()
            mat, info = oeq.solve(h0, A["U"], A["mu"], A["beta"], ntau)
            eqr = {"equilibrium_oracle_s": time.perf_counter() - t0,
                   "equilibrium_oracle_iterations": info["iterations"],
                   "equilibrium_max_abs_diff": float(np.abs(mat - r["mat"]).max())}
        P = oprop.Problem(t=np.zeros(1), order=np.zeros(1, np.int32), h0=h0, ntau=ntau,
                          beta=A["beta"], mat=mat, rho0=None if ntau else r["rho"],
                          pulse_t0=A["pulse_t0"], pulse_sigma=A["pulse_sigma"])
        ctl = oad.Controls(t_end=r["replay"][-1]["t"], rtol=A["rtol"], atol=A["atol"],
                           h0=A["h_first"], qmax=A["qmax"], kmax=A["kmax"], maxcor=A["maxcor"],
                           nt_max=len(r["replay"]))
        o = oad.Adaptive(P, ctl)
        t0 = time.perf_counter()
        dens = o.run(A["U"], A["pulse_amp"], replay=r["replay"]).numpy()
        dt = time.perf_counter() - t0
        kp, _ = o.storage()
        steps = len(r["replay"]) - 1
        res.append({"ntau": ntau, "steps": steps, "oracle_s": dt,
                    "oracle_ms_per_step": 1e3 * dt / steps,
                    "gpu_ms_per_step": r["gpu_ms_per_step"],
                    "dens_max_abs_diff": float(np.abs(dens - r["dens"]).max()),
                    "kp_rel_diff": float(np.linalg.norm(kp - r["kp"]) / np.linalg.norm(kp)),
                    **eqr})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ceilings", action="store_true",
                    help="only run the ceiling microbenchmarks and write profiles/ceilings.json")
    ap.add_argument("--adaptive-only", action="store_true",
                    help="only run the adaptive propagation cases (no oracle leg)")
    ap.add_argument("--no-propagation", action="store_true",
                    help="skip the two propagations (for counter runs over the collision kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three plain 1 GiB device-to-device copies: the reference "
                         "reading that scales FETCH_SIZE / WRITE_SIZE to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        nbytes = 1 << 30
        x = torch.ones(nbytes // 16, dtype=torch.complex128, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": 3}), flush=True)
        return

    import paper_2405_08737_amd as kbe
    import synth

    kbe.lib()
    if args.ceilings:
        c = ceilings(kbe, torch)
        c["command"] = "python bench.py --ceilings"
        c["gpu"] = torch.cuda.get_device_name(0)
        path = os.path.join(ROOT, "profiles", "ceilings.json")
        with open(path, "w") as f:
            json.dump(c, f, indent=1)
            f.write("\n")
        print(json.dumps(c), flush=True)
        return
    dev = torch.device("cuda:0")
    if args.adaptive_only:
        t0 = time.perf_counter()
        rep, _ = adaptive(kbe, torch, dev)
        rep["process_wall_s"] = time.perf_counter() - t0
        rep["equilibrium"] = equilibrium(kbe, torch, dev)
        print(json.dumps(rep), flush=True)
        return
    log("ceiling microbenchmarks")
    ceil = ceilings(kbe, torch)
    w = synth.HEADLINE
    N, nt, ntau, n = w.N, w.nt, w.ntau, w.nt - 1
    log(f"generating {w.name} inputs on the host")
    t, order = synth.grid(w.seed, nt, w.hmin, w.hmax, w.omin, w.omax)
    kp_h = synth.kp(w.seed, N, t)
    rd_h = synth.rdiag(N, nt)
    tv_h = synth.tv(w.seed, N, ntau, t)
    mat_h = synth.mat(w.seed, N, ntau)
    log("copying to HBM")
    kp = torch.empty(kp_h.shape, dtype=torch.complex128, device=dev)
    for a0 in range(0, nt, 128):
        kp[a0:a0 + 128].copy_(torch.from_numpy(kp_h[a0:a0 + 128]))
    tvd = torch.empty(tv_h.shape, dtype=torch.complex128, device=dev)
    for a0 in range(0, nt, 256):
        tvd[a0:a0 + 256].copy_(torch.from_numpy(tv_h[a0:a0 + 256]))
    G = kbe.Green(kp, torch.from_numpy(rd_h).to(dev), tvd, torch.from_numpy(mat_h).to(dev))
    gG = kbe.Green(torch.empty_like(kp), torch.empty_like(G.rdiag), torch.empty_like(tvd),
                   torch.empty_like(G.mat))
    u = torch.full((N,), w.U, dtype=torch.float64, device=dev)
    gu = torch.zeros(N, dtype=torch.float64, device=dev)
    cot = tuple(torch.from_numpy(synth.normal(7, k, (nt if k < 3 else ntau, N, N))).to(dev)
                for k in range(4))
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)
    phases = []

    def step(record):
        e = [ev() for _ in range(6)] if record else None
        if record:
            e[0].record()
        W = kbe.weights(t, order, ntau, w.beta, w.tau_order, device=dev)
        if record:
            e[1].record()
        sig = kbe.sigma_2b(G, u, n)
        if record:
            e[2].record()
        kbe.collision(G, sig, W, n)
        if record:
            e[3].record()
        _, gsig = kbe.collision_vjp(G, sig, W, n, 0, n + 1, cot,
                                    kbe.OUT_ALL | kbe.GRAD_OVERWRITE, gG)
        if record:
            e[4].record()
        gu.zero_()
        kbe.sigma_2b_vjp(G, u, n, gsig, gG, gu)
        if record:
            e[5].record()
            phases.append(e)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / args.steps * 1e3
    ph = np.array([[p[i].elapsed_time(p[i + 1]) for i in range(5)] for p in phases])
    ph_ms = ph.mean(axis=0)  # weights, sigma, collision, collision_vjp, sigma_vjp
    c = counts(N, nt, ntau, n)
    fwd_ms = ph_ms[0] + ph_ms[1] + ph_ms[2]
    adj_ms = ph_ms[3] + ph_ms[4]
    coll_s = ph_ms[2] / 1e3
    achieved = c["fwd_flop"] / coll_s / 1e12
    traffic = measured_traffic()
    result = {
        "metric": METRIC,
        "value": (c["fwd_flop"] + c["adj_flop"]) / (ms_step / 1e3) / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "collision_history_row", "N_orb": N, "nt": nt, "n": n,
                   "m_range": [0, n + 1], "ntau": ntau, "beta": w.beta,
                   "steps_dt": [w.hmin, w.hmax], "orders": [w.omin, w.omax],
                   "tau_order": w.tau_order, "U": w.U, "seed": w.seed,
                   "inputs": "random KP/tv/mat (N(0,1) x exp(-0.3|t-t'|)), Sigma = second Born"},
        "forward": {"ms": fwd_ms, "collision_ms": ph_ms[2], "weights_ms": ph_ms[0],
                    "sigma_ms": ph_ms[1],
                    "collision_gflops": c["fwd_flop"] / coll_s / 1e9,
                    "collision_gbps": c["fwd_bytes"] / coll_s / 1e9},
        "adjoint": {"ms": adj_ms, "collision_vjp_ms": ph_ms[3], "sigma_vjp_ms": ph_ms[4],
                    "collision_vjp_gflops": c["adj_flop"] / (ph_ms[3] / 1e3) / 1e9,
                    "collision_vjp_gbps": c["adj_bytes"] / (ph_ms[3] / 1e3) / 1e9},
        "adjoint_over_forward": adj_ms / fwd_ms,
        "hbm_gbps": (c["fwd_bytes"] + c["adj_bytes"]) / (ms_step / 1e3) / 1e9,
        "roofline": {
            "kernel": "kbe_collision forward call: stream_fused<16, false> (the MFMA task, about "
                      "99% of it) + zero_heads + chunk reduces, timed with HIP events around the "
                      "call",
            "bound": "mfma" if c["fwd_flop"] / c["fwd_bytes"] > RIDGE else "hbm",
            "achieved": achieved, "peak": MFMA_F64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / MFMA_F64_PEAK_TFLOPS,
            "traffic": traffic,
            "algorithmic_flop": c["fwd_flop"], "algorithmic_bytes": c["fwd_bytes"],
            "intensity_flop_per_byte": c["fwd_flop"] / c["fwd_bytes"],
            "hbm_frac": c["fwd_bytes"] / coll_s / 1e9 / HBM_PEAK_GBS,
            "frac_of_measured_mfma_ceiling": achieved / ceil["mfma_f64_4x4x4_tflops"],
            "measured_read_gbps": (traffic / coll_s / 1e9) if traffic else None,
            "measured_read_frac_of_ceiling":
                (traffic / coll_s / 1e9 / ceil["hbm_read_gbs"]) if traffic else None},
        "ceilings": ceil,
        "per_call_ms": {name: {"median": float(np.median(ph[:, i])), "min": float(ph[:, i].min())}
                        for i, name in enumerate(("weights", "sigma_2b", "collision",
                                                  "collision_vjp", "sigma_2b_vjp"))},
    }
    log("sigma row -> collision as a graph")
    result["sigma_collision_graph"] = graph_pair(kbe, torch, G, u, n, t, order, w)
    log("greater form")
    result["greater_form"] = greater_form(kbe, torch, G, u, n, t, order, w, cot, gG)
    log("general four-index self-energy")
    result["gf2"] = general_u_sigma(kbe, torch, G, n, w)
    log("batched against plain per-row calls")
    Wh = kbe.weights(t, order, ntau, w.beta, w.tau_order, device=dev)
    plain_rows = batch_vs_plain(kbe, torch, dev, G, Wh, u)
    del gG, kp, tvd, G, Wh
    torch.cuda.empty_cache()
    log("8-orbital differentiation shape")
    result["small_orbital"] = small_orbital_shape(kbe, torch, dev)
    log("batching workload")
    result["batching"] = batching(kbe, torch, dev)
    result["batching"]["plain_per_row"] = plain_rows
    torch.cuda.empty_cache()
    torch.cuda.empty_cache()
    replays = []
    if not args.no_propagation:
        log("end-to-end gradients through a propagation")
        result["propagation"] = propagation(kbe, torch, dev)
        torch.cuda.empty_cache()
        log("adaptive propagation")
        result["adaptive"], replays = adaptive(kbe, torch, dev)
        log("equilibrium solve")
        result["equilibrium"] = equilibrium(kbe, torch, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        result["cpu_baseline"] = cpu_baseline(w, (t, order, kp_h, rd_h, tv_h, mat_h))
        if replays:
            log("oracle replaying the adaptive prefixes")
            result["cpu_baseline"]["adaptive"] = adaptive_oracle(replays)
        log("oracle on samples of the other calls")
        other = cpu_other_rows(w, (t, order, kp_h, rd_h, tv_h, mat_h),
                               result["cpu_baseline"]["cores"])
        gpu_rates = {"small_orbital": result["small_orbital"]["collision_gflops"],
                     "batching": result["batching"]["gflops"],
                     "gf2": result["gf2"]["tflops"] * 1e3}
        for k, v in other.items():
            v["gpu_gflops"] = gpu_rates[k]
        result["cpu_baseline"]["other_calls"] = other
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
