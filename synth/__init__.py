"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the CPU oracle.

The arrays are drawn by ``synth.c`` (a counter-based generator: SplitMix64
finaliser + Box-Muller), so any slice can be regenerated independently and
both sides of a parity check see bit-identical inputs.  Nothing here computes
any part of the method (weights, self-energy, integrals).

Layout conventions (complex128, N x N row-major blocks):
  kp    [nt][ldt][N][N]  kp[a][b] = G^<(t_a,t_b) for a <= b, G^R(t_a,t_b) for a > b
  rdiag [nt][N][N]       G^R(t_a,t_a) = -i * 1
  tv    [nt][ntau][N][N] mixed component G^(t_m, tau_j)
  mat   [ntau][N][N]     Matsubara component G^M(tau_j)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build() -> str:
    """Compile synth.c into libsynth.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        c = ctypes
        P = c.c_void_p
        lib.synth_grid.argtypes = [c.c_uint64, c.c_int32, c.c_double, c.c_double, c.c_int32,
                                   c.c_int32, P, P]
        lib.synth_kp_rows.argtypes = [c.c_uint64, c.c_int32, c.c_int32, c.c_int64, P, c.c_double,
                                      c.c_int32, c.c_int32, P]
        lib.synth_kp_col.argtypes = [c.c_uint64, c.c_int32, c.c_int32, P, c.c_double, c.c_int32,
                                     c.c_int32, c.c_int32, P]
        lib.synth_rdiag.argtypes = [c.c_int32, c.c_int32, P]
        lib.synth_tv_rows.argtypes = [c.c_uint64, c.c_int32, c.c_int32, P, c.c_double, c.c_int32,
                                      c.c_int32, P]
        lib.synth_mat.argtypes = [c.c_uint64, c.c_int32, c.c_int32, P]
        lib.synth_sigma_row.argtypes = [c.c_uint64, c.c_int32, c.c_int32, c.c_int32, P, c.c_double,
                                        P, P, P]
        lib.synth_normal.argtypes = [c.c_uint64, c.c_uint64, c.c_int64, P]
        for f in (lib.synth_grid, lib.synth_kp_rows, lib.synth_kp_col, lib.synth_rdiag, lib.synth_tv_rows,
                  lib.synth_mat, lib.synth_sigma_row, lib.synth_normal):
            f.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags.c_contiguous
    return a.ctypes.data


def grid(seed: int, nt: int, hmin: float, hmax: float, omin: int, omax: int):
    """Non-uniform grid t[0]=0, steps ~ U[hmin,hmax]; per-interval orders ~ U{omin..omax}."""
    t = np.empty(nt, np.float64)
    order = np.empty(nt, np.int32)
    _load().synth_grid(seed, nt, hmin, hmax, omin, omax, _ptr(t), _ptr(order))
    return t, order


def kp(seed: int, N: int, t: np.ndarray, decay: float = 0.3, rows=None, ldt: int | None = None,
       out: np.ndarray | None = None) -> np.ndarray:
    """KP two-time array rows [a0,a1) x columns [0,nt) (columns padded to ldt)."""
    nt = len(t)
    ldt = nt if ldt is None else ldt
    a0, a1 = (0, nt) if rows is None else rows
    if out is None:
        out = np.zeros((a1 - a0, ldt, N, N), np.complex128)
    assert out.shape == (a1 - a0, ldt, N, N) and out.dtype == np.complex128
    _load().synth_kp_rows(seed, N, nt, ldt, _ptr(np.ascontiguousarray(t)), decay, a0, a1, _ptr(out))
    return out


def kp_col(seed: int, N: int, t: np.ndarray, col: int, rows=None, decay: float = 0.3) -> np.ndarray:
    """Column `col` of the KP array of `kp(seed, N, t)`, rows [a0, a1): shape (a1-a0, N, N)."""
    nt = len(t)
    a0, a1 = (0, nt) if rows is None else rows
    out = np.zeros((a1 - a0, N, N), np.complex128)
    _load().synth_kp_col(seed, N, nt, _ptr(np.ascontiguousarray(t)), decay, col, a0, a1, _ptr(out))
    return out


def rdiag(N: int, nt: int) -> np.ndarray:
    out = np.empty((nt, N, N), np.complex128)
    _load().synth_rdiag(N, nt, _ptr(out))
    return out


def tv(seed: int, N: int, ntau: int, t: np.ndarray, decay: float = 0.3, rows=None,
       out: np.ndarray | None = None) -> np.ndarray:
    nt = len(t)
    m0, m1 = (0, nt) if rows is None else rows
    if out is None:
        out = np.empty((m1 - m0, ntau, N, N), np.complex128)
    assert out.shape == (m1 - m0, ntau, N, N)
    if ntau > 0:
        _load().synth_tv_rows(seed, N, ntau, _ptr(np.ascontiguousarray(t)), decay, m0, m1, _ptr(out))
    return out


def mat(seed: int, N: int, ntau: int) -> np.ndarray:
    out = np.empty((ntau, N, N), np.complex128)
    if ntau > 0:
        _load().synth_mat(seed, N, ntau, _ptr(out))
    return out


def sigma_row(seed: int, N: int, n: int, ntau: int, t: np.ndarray, decay: float = 0.3):
    """Self-energy row at t_n given as independent random input: (ret[n+1], les[n+1], tv[ntau])."""
    ret = np.empty((n + 1, N, N), np.complex128)
    les = np.empty((n + 1, N, N), np.complex128)
    stv = np.empty((ntau, N, N), np.complex128)
    _load().synth_sigma_row(seed, N, n, ntau, _ptr(np.ascontiguousarray(t)), decay, _ptr(ret),
                            _ptr(les), _ptr(stv))
    return ret, les, stv


def normal(seed: int, stream: int, shape) -> np.ndarray:
    out = np.empty(shape, np.complex128)
    _load().synth_normal(seed, stream, out.size, _ptr(out))
    return out


@dataclass(frozen=True)
class Workload:
    """Sizes of one synthetic workload (paper-shaped, see the input recipe)."""
    name: str
    N: int
    nt: int
    ntau: int
    beta: float
    hmin: float
    hmax: float
    omin: int
    omax: int
    tau_order: int
    U: float
    seed: int

    @property
    def n(self) -> int:
        return self.nt - 1


# The parity-size case, the headline size, and the differentiation size.
PARITY_SMALL = Workload("N2_nt64_ntau64", 2, 64, 64, 10.0, 0.02, 0.08, 5, 5, 5, 1.0, 1000)
HEADLINE = Workload("N16_nt2048_ntau512", 16, 2048, 512, 20.0, 0.005, 0.05, 3, 6, 5, 1.0, 1001)
DIFFERENTIATION = Workload("N8_nt1024_ntau256", 8, 1024, 256, 10.0, 0.005, 0.05, 3, 6, 5, 2.0, 1003)

# The propagation (end-to-end gradients) on the differentiation grid: 8-site open tight-binding
# chain (hopping -1), initial state the free thermal state at beta (G^M with a thermal branch, its
# density matrix without one), Gaussian pulse of amplitude 1 at t = 2 with width 1 on h_00, loss
# n_0 summed over the last 32 steps, two fixed-point iterations per step.  Thermal branch at
# U = 1; U = 2 without it (the free G^M is not an equilibrium of the U = 2 mixed branch).
PROPAGATION = dict(N=8, nt=1024, beta=10.0, hmin=0.005, hmax=0.05, omin=3, omax=6, seed=1003,
                   pulse_amp=1.0, pulse_t0=2.0, pulse_sigma=1.0, last=32, iters=2,
                   cases=((1.0, 256), (2.0, 0)))

# The adaptive propagation: the same 8-site chain at half filling, U = 1, beta = 10, quenched by
# the same pulse on site 0, variable step and order with the paper's tightest tolerances
# (rtol 1e-8, atol 1e-10) and its largest history order K = 20, up to t = 40.  Two cases: the
# thermal branch (256 tau points) from the interacting equilibrium G^M at mu = U/2 (the
# self-consistent second-Born Matsubara Dyson solution; with the free G^M instead, this problem
# runs into a finite-time singularity at t ~ 32.88), and no thermal branch (initial density
# matrix the free thermal one).  The oracle replays the first `prefix` steps of each case on the
# same grid.
ADAPTIVE = dict(N=8, U=1.0, mu=0.5, beta=10.0, pulse_amp=1.0, pulse_t0=2.0, pulse_sigma=1.0,
                rtol=1e-8, atol=1e-10, h_first=1e-3, qmax=12, kmax=20, maxcor=3, capacity=4096,
                cases=((256, 40.0, 8), (0, 40.0, 48)))


def tight_binding(N: int, hop: float = -1.0) -> np.ndarray:
    """Open chain: h[i][i+1] = h[i+1][i] = hop, on-site 0."""
    h = np.zeros((N, N))
    for i in range(N - 1):
        h[i, i + 1] = h[i + 1, i] = hop
    return h


def free_thermal(h: np.ndarray, beta: float, ntau: int):
    """Initial state of a propagation: the free thermal state of the real symmetric h at beta, as
    (G^M(tau_j) for tau_j = j beta / (ntau - 1), complex128 [ntau][N][N], or None when ntau == 0;
    the density matrix f(h) [N][N]).  G^M(tau) = -exp(-h tau)(1 - f(h)) with its endpoints the
    one-sided limits 0+ and beta-, evaluated in the eigenbasis of h so the large and small
    exponentials never meet in a matrix product."""
    e, v = np.linalg.eigh(h)
    f = 1.0 / (np.exp(beta * e) + 1.0)
    rho = (v * f) @ v.T
    if ntau == 0:
        return None, rho
    taus = np.linspace(0.0, beta, ntau)
    mat = np.array([(v * (-np.exp(-e * x) * (1.0 - f))) @ v.T for x in taus])
    return mat.astype(np.complex128), rho


def green(w: Workload, decay: float = 0.3, ldt: int | None = None):
    """Full random Green's function of a workload: dict with t, order, kp, rdiag, tv, mat."""
    t, order = grid(w.seed, w.nt, w.hmin, w.hmax, w.omin, w.omax)
    return dict(t=t, order=order, kp=kp(w.seed, w.N, t, decay, ldt=ldt), rdiag=rdiag(w.N, w.nt),
                tv=tv(w.seed, w.N, w.ntau, t, decay), mat=mat(w.seed, w.N, w.ntau))


@dataclass
class BatchSpec:
    """Shape of one history row of a batch: orbitals N, row n, column m, and the seed of the
    row's own system (grid of n+1 points, KP, tv and self-energy row all drawn from it)."""
    N: int
    n: int
    m: int
    seed: int


# Batching workload: 256 rows, N ~ U{2,4,8,16}, n log-uniform in [128, 4096], m ~ U{0..n},
# ntau = 256, per-interval orders U{3..6}, steps U[0.005, 0.05], beta = 10.
BATCH = dict(count=256, Ns=(2, 4, 8, 16), nmin=128, nmax=4096, ntau=256, beta=10.0,
             hmin=0.005, hmax=0.05, omin=3, omax=6, tau_order=5, seed=1002)


def batch_specs(seed: int, count: int, Ns=(2, 4, 8, 16), nmin: int = 128, nmax: int = 4096):
    """The rows of a batch: N uniform over Ns, n log-uniform in [nmin, nmax], m uniform in
    0..n.  The uniform draws are the steps of `grid` with steps U[0, 1) on the batch's seed."""
    u, _ = grid(seed, 3 * count + 1, 0.0, 1.0, 1, 1)  # cumulative sums of U[0,1) draws
    d = np.diff(u)                                     # the draws themselves
    out = []
    for i in range(count):
        N = Ns[min(int(d[3 * i] * len(Ns)), len(Ns) - 1)]
        n = int(round(np.exp(np.log(nmin) + (np.log(nmax) - np.log(nmin)) * d[3 * i + 1])))
        m = min(int(d[3 * i + 2] * (n + 1)), n)
        out.append(BatchSpec(N, n, m, seed * 100003 + i))
    return out


def batch_cross(spec: BatchSpec, ntau: int, hmin: float, hmax: float, omin: int, omax: int,
                decay: float = 0.3):
    """Host arrays of one batch row: its grid (t, order), self-energy row at t_n, KP column m
    (rows 0..m), KP row m (columns 0..n), G^R(t_m, t_m), tv row m."""
    N, n, m, s = spec.N, spec.n, spec.m, spec.seed
    t, order = grid(s, n + 1, hmin, hmax, omin, omax)
    ret, les, stv = sigma_row(s, N, n, ntau, t, decay)
    col = kp_col(s, N, t, m, rows=(0, m + 1), decay=decay)
    row = kp(s, N, t, decay, rows=(m, m + 1))[0]
    rd = rdiag(N, 1)[0]
    tvm = tv(s, N, ntau, t, decay, rows=(m, m + 1))[0] if ntau > 0 else np.zeros((0, N, N), np.complex128)
    return dict(t=t, order=order, ret=ret, les=les, stv=stv, col=col, row=row, rdiag=rd, tv=tvm)


def coulomb(seed: int, N: int, onsite: float = 1.0, spread: float = 0.1) -> np.ndarray:
    """A real four-index interaction U[i, f, d, e] in chemists' notation (ij|kl): on-site value
    `onsite` on U[i, i, i, i] plus N(0, spread^2) entries averaged over the eight index
    permutations (ij|kl) = (ji|kl) = (ij|lk) = (kl|ij) ..., so it has the symmetry of real
    two-electron integrals.  Stands in for molecular integrals (none are available offline)."""
    U0 = spread * normal(seed, 99, (N, N, N, N)).real
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
             (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    U = sum(np.transpose(U0, p) for p in perms) / 8.0
    for i in range(N):
        U[i, i, i, i] += onsite
    return np.ascontiguousarray(U)
