"""kbe_collision_noalloc, the entry point that allocates nothing: its output against
kbe_collision's (bit for bit: the same kernels and plan) and against the oracle to the FP64 bar,
on two calls in a row, the second with a smaller input, and its refusal of a call whose workspace
exceeds the fixed scratch array."""
import numpy as np
import pytest

import oracle
import synth
from tests.cases import (Case, assert_blocks_close, device_green, device_weights, scales, to_dev,
                         to_host)

pytestmark = pytest.mark.gpu


def _one(kbe, case, m0, m1, flags):
    t, order, kp, rd, tv, mat = case.host()
    n = case.nt - 1
    W = oracle.Weights.build(t, order, case.beta, case.ntau, case.tau_order)
    sig = synth.sigma_row(case.seed, case.N, n, case.ntau, t)
    Gd, Wd = device_green(kp, rd, tv, mat), device_weights(W)
    sigd = tuple(to_dev(x) for x in sig)
    print("noalloc", case.N, case.nt, case.ntau, m0, m1, hex(flags), flush=True)
    got = kbe.collision_noalloc(Gd, sigd, Wd, n, m0, m1, flags)
    want = kbe.collision(Gd, sigd, Wd, n, m0, m1, flags)
    ref = oracle.collision(oracle.Green(kp, rd, tv, mat), sig, W, n, m0, m1,
                           (flags & 0xF) | (oracle.F_GREATER if flags & kbe.GREATER else 0))
    sc = scales(kp, rd, tv, mat, sig, W, n, range(m0, m1), range(case.ntau),
                greater=bool(flags & kbe.GREATER))
    for name, g, w, r in zip(("IR", "IL", "Itv", "Jtv"), got, want, ref):
        assert (g is None) == (w is None), name
        if g is None:
            continue
        g, w = to_host(g), to_host(w)
        assert np.array_equal(g, w), name
        assert_blocks_close(g, r, sc[name], name)


def test_noalloc_matches_collision_twice(gpu):
    """Two calls in a row on one device (the second smaller, so the scratch array holds the first
    call's contents when it starts), each equal to kbe_collision bit for bit."""
    kbe = gpu
    _one(kbe, Case(N=8, nt=300, ntau=40, beta=4.0, seed=501), 0, 300,
         kbe.OUT_ALL | kbe.GREATER)
    _one(kbe, Case(N=4, nt=60, ntau=8, beta=2.0, seed=502), 10, 50, kbe.OUT_ALL)
    _one(kbe, Case(N=16, nt=40, ntau=6, beta=2.0, seed=503), 0, 40, kbe.OUT_ALL)


def test_noalloc_rejects_oversized_call(gpu):
    """A 16-orbital greater-form history of 1024 points needs more workspace than the fixed
    array: the call is refused with KBE_ENOMEM before anything is enqueued."""
    import torch
    kbe = gpu
    N, nt, ntau = 16, 1024, 64
    need = kbe.lib().kbe_collision_workspace(N, nt, ntau, nt - 1, 0, nt, kbe.OUT_ALL | kbe.GREATER)
    assert need > 64 << 20
    dev = torch.device("cuda:0")
    z = lambda *s: torch.zeros(s, dtype=torch.complex128, device=dev)
    G = kbe.Green(z(nt, nt, N, N), z(nt, N, N), z(nt, ntau, N, N), z(ntau, N, N))
    t, order = synth.grid(1, nt, 0.005, 0.05, 3, 6)
    W = device_weights(oracle.Weights.build(t, order, 4.0, ntau, 5))
    sig = (z(nt, N, N), z(nt, N, N), z(ntau, N, N))
    with pytest.raises(kbe.KBEError, match="KBE_ENOMEM|scratch"):
        kbe.collision_noalloc(G, sig, W, nt - 1, 0, nt, kbe.OUT_ALL | kbe.GREATER)
    torch.cuda.synchronize()
