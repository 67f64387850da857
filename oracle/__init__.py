"""CPU oracle for the Kadanoff-Baym history-integral path (TEST INFRASTRUCTURE ONLY).

A ctypes shim over ``oracle.c``: plain FP64 loops written from the paper
(arXiv:2405.08737).  Only ``tests/``, the package's ``smoke()`` check and the
benchmark's CPU-baseline leg may import this module; the GPU library never
does, and the two share no code.

Arrays are numpy complex128 / float64, C-contiguous, in the layout stated at
the top of ``oracle.c``.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
mathematics fixed independently of this code (closed forms, exactness on
polynomials, textbook Adams-Moulton coefficients, symmetry and conservation
invariants, brute force on tiny inputs, finite differences).  No function is
"parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

F_IR, F_IL, F_ITV, F_JTV = 1, 2, 4, 8
F_ALL = F_IR | F_IL | F_ITV | F_JTV
F_GREATER = 1024  # the greater form of Eq. KBE2 (see orc_collision)


def build() -> str:
    """Compile oracle.c into liboracle.so (always recompiles). Plain FP64: no contraction."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-o", _SO + ".tmp",
           _SRC, "-lm"]
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
        P, I32, I64, D = c.c_void_p, c.c_int, c.c_int64, c.c_double
        lib.orc_gauss_legendre.argtypes = [I32, P, P]
        lib.orc_local_weights.argtypes = [P, I32, I32, P]
        lib.orc_weights.argtypes = [P, P, I32, P]
        lib.orc_tau_weights.argtypes = [D, I32, I32, P, P, P]
        lib.orc_sigma_pair.argtypes = [I32, I32, I32, I64, P, P, P, I32, I32, P, P]
        lib.orc_sigma_row.argtypes = [I32, I32, I32, I64, P, P, P, P, I32, P, P, P]
        lib.orc_collision.argtypes = [I32, I32, I32, I64, P, P, P, P, P, P, P, P, P, P, P, I32, I32,
                                      I32, I32, I32, I32, P, P, P, P]
        lib.orc_collision_row.argtypes = [I32, I32, I32, I32, P, P, P, P, P, P, P, P, P, P, I32,
                                          P, P, P]
        lib.orc_collision_vjp.argtypes = [I32, I32, I32, I64, P, P, P, P, P, P, P, P, P, P, P, I32,
                                          I32, I32, I32, P, P, P, P, P, P, P, P, P, P, P]
        lib.orc_sigma_row_vjp.argtypes = [I32, I32, I32, I64, P, P, P, P, I32, P, P, P, P, P, P, P]
        lib.orc_gf2_block.argtypes = [I32, P, P, P, P]
        lib.orc_set_threads.argtypes = [I32]
        for name in ("orc_gauss_legendre", "orc_local_weights", "orc_weights", "orc_tau_weights",
                     "orc_sigma_pair", "orc_sigma_row", "orc_collision", "orc_collision_vjp",
                     "orc_sigma_row_vjp", "orc_gf2_block", "orc_set_threads"):
            getattr(lib, name).restype = None
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    assert isinstance(a, np.ndarray) and a.flags.c_contiguous, "oracle arrays must be C-contiguous"
    return a.ctypes.data


def _c(a, dtype=np.complex128):
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(k: int) -> None:
    """Thread count of the oracle's OpenMP loops (results do not depend on it)."""
    _load().orc_set_threads(int(k))


def gauss_legendre(m: int):
    x = np.empty(m)
    w = np.empty(m)
    _load().orc_gauss_legendre(m, _p(x), _p(w))
    return x, w


def local_weights(t, p: int, k: int) -> np.ndarray:
    t = _c(t, np.float64)
    lam = np.empty(k)
    _load().orc_local_weights(_p(t), p, k, _p(lam))
    return lam


def weights(t, order) -> np.ndarray:
    """Composite weight matrix w[n][s] (nt x nt)."""
    t = _c(t, np.float64)
    order = _c(order, np.int32)
    nt = len(t)
    w = np.empty((nt, nt))
    _load().orc_weights(_p(t), _p(order), nt, _p(w))
    return w


def tau_weights(beta: float, ntau: int, tau_order: int):
    """(wf, wb, wfull): forward [0,tau_j] rule, backward [tau_j,beta] rule, full-range rule."""
    wf = np.empty((ntau, ntau))
    wb = np.empty((ntau, ntau))
    wfull = np.empty(ntau)
    _load().orc_tau_weights(beta, ntau, tau_order, _p(wf), _p(wb), _p(wfull))
    return wf, wb, wfull


class Green:
    """Host Green's function in KP storage (see oracle.c)."""

    def __init__(self, kp, rdiag, tv=None, mat=None):
        self.kp = _c(kp)
        self.rdiag = _c(rdiag)
        self.nt_rows, self.ldt, self.N, _ = self.kp.shape
        self.nt = self.rdiag.shape[0]
        ntau = 0 if tv is None else tv.shape[1]
        self.ntau = ntau
        self.tv = _c(tv) if tv is not None else np.zeros((self.nt, 0, self.N, self.N), np.complex128)
        self.mat = (_c(mat) if mat is not None
                    else np.zeros((ntau, self.N, self.N), np.complex128))
        assert self.tv.shape == (self.nt, ntau, self.N, self.N), self.tv.shape
        assert self.mat.shape == (ntau, self.N, self.N), self.mat.shape
        assert self.rdiag.shape == (self.nt, self.N, self.N) and self.nt_rows == self.nt

    def args(self):
        return (self.N, self.nt, self.ntau, self.ldt)


def sigma_pair(G: Green, u, a: int, b: int):
    u = _c(u, np.float64)
    N = G.N
    les = np.empty((N, N), np.complex128)
    gtr = np.empty((N, N), np.complex128)
    _load().orc_sigma_pair(*G.args(), _p(G.kp), _p(G.rdiag), _p(u), a, b, _p(les), _p(gtr))
    return les, gtr


def sigma_row(G: Green, u, n: int):
    """(ret[n+1], les[n+1], stv[ntau]) at t_n."""
    u = _c(u, np.float64)
    N = G.N
    ret = np.empty((n + 1, N, N), np.complex128)
    les = np.empty((n + 1, N, N), np.complex128)
    stv = np.empty((G.ntau, N, N), np.complex128)
    _load().orc_sigma_row(*G.args(), _p(G.kp), _p(G.rdiag), _p(G.tv), _p(u), n, _p(ret), _p(les),
                          _p(stv))
    return ret, les, stv


class Weights:
    def __init__(self, w, wfull=None, wf=None, wb=None):
        self.w = _c(w, np.float64)
        self.wfull = _c(wfull if wfull is not None else np.zeros(0), np.float64)
        self.wf = _c(wf if wf is not None else np.zeros((0, 0)), np.float64)
        self.wb = _c(wb if wb is not None else np.zeros((0, 0)), np.float64)

    @classmethod
    def build(cls, t, order, beta=None, ntau=0, tau_order=5):
        w = weights(t, order)
        if ntau > 0:
            wf, wb, wfull = tau_weights(beta, ntau, tau_order)
            return cls(w, wfull, wf, wb)
        return cls(w)


def collision(G: Green, sig, W: Weights, n: int, m0: int = 0, m1: int | None = None,
              flags: int = F_ALL, jrange=None):
    """(IR, IL, Itv, Jtv) for m in [m0, m1) at row n; Jtv for j in jrange (default all)."""
    m1 = n + 1 if m1 is None else m1
    j0, j1 = (0, G.ntau) if jrange is None else jrange
    ret, les, stv = (_c(x) for x in sig)
    N, nm = G.N, m1 - m0
    IR = np.zeros((nm, N, N), np.complex128)
    IL = np.zeros((nm, N, N), np.complex128)
    Itv = np.zeros((nm, N, N), np.complex128)
    Jtv = np.zeros((j1 - j0, N, N), np.complex128)
    _load().orc_collision(*G.args(), _p(G.kp), _p(G.rdiag), _p(G.tv), _p(G.mat), _p(ret), _p(les),
                          _p(stv), _p(W.w), _p(W.wfull), _p(W.wf), _p(W.wb), n, m0, m1, j0, j1,
                          flags, _p(IR), _p(IL), _p(Itv), _p(Jtv))
    return IR, IL, Itv, Jtv


def collision_row(N: int, ntau: int, n: int, m: int, sig, col, row, rdg, tvm, wn, wm, wfull,
                  flags: int = F_IR | F_IL | F_ITV):
    """(IR, IL, Itv) blocks at one (t_n, t_m) from the row's own blocks (see orc_collision_row):
    sig = (ret [n+1], les [n+1], stv [ntau]); col [m+1] = kp[:m+1, m]; row [n+1] = kp[m, :n+1];
    rdg = rdiag[m]; tvm [ntau] = tv[m]; wn [n+1], wm [m+1] weight rows; wfull [ntau]."""
    ret, les, stv = (_c(x) for x in sig)
    args = [_c(col), _c(row), _c(rdg), _c(tvm) if ntau > 0 else np.zeros((1, N, N), np.complex128),
            _c(wn, np.float64), _c(wm, np.float64),
            _c(wfull, np.float64) if ntau > 0 else np.zeros(1)]
    if ntau == 0:
        stv = np.zeros((1, N, N), np.complex128)
    out = [np.zeros((N, N), np.complex128) for _ in range(3)]
    _load().orc_collision_row(N, ntau, n, m, _p(ret), _p(les), _p(stv), *(_p(a) for a in args),
                              flags, *(_p(o) for o in out))
    return tuple(out)


def collision_vjp(G: Green, sig, W: Weights, n: int, m0: int, m1: int, cot, flags: int = F_ALL,
                  grads=None):
    """Adjoint of collision.  cot = (gIR, gIL, gItv, gJtv).
    Returns (gkp, grdiag, gtv, gmat, gret, gles, gstv); Green's-function gradients are
    accumulated into ``grads`` when given (else into zeros)."""
    ret, les, stv = (_c(x) for x in sig)
    gIR, gIL, gItv, gJtv = (_c(x) for x in cot)
    N = G.N
    if grads is None:
        grads = (np.zeros_like(G.kp), np.zeros_like(G.rdiag), np.zeros_like(G.tv),
                 np.zeros_like(G.mat))
    gkp, grd, gtv, gmat = grads
    gret = np.empty((n + 1, N, N), np.complex128)
    gles = np.empty((n + 1, N, N), np.complex128)
    gstv = np.empty((G.ntau, N, N), np.complex128)
    _load().orc_collision_vjp(*G.args(), _p(G.kp), _p(G.rdiag), _p(G.tv), _p(G.mat), _p(ret),
                              _p(les), _p(stv), _p(W.w), _p(W.wfull), _p(W.wf), _p(W.wb), n, m0,
                              m1, flags, _p(gIR), _p(gIL), _p(gItv), _p(gJtv), _p(gkp), _p(grd),
                              _p(gtv), _p(gmat), _p(gret), _p(gles), _p(gstv))
    return gkp, grd, gtv, gmat, gret, gles, gstv


def sigma_row_vjp(G: Green, u, n: int, gsig, grads=None, gu=None):
    """Adjoint of sigma_row.  gsig = (gret, gles, gstv).  Returns (gkp, grdiag, gtv, gu)."""
    u = _c(u, np.float64)
    gret, gles, gstv = (_c(x) for x in gsig)
    if grads is None:
        grads = (np.zeros_like(G.kp), np.zeros_like(G.rdiag), np.zeros_like(G.tv))
    gkp, grd, gtv = grads
    gu = np.zeros(G.N) if gu is None else gu
    _load().orc_sigma_row_vjp(*G.args(), _p(G.kp), _p(G.rdiag), _p(G.tv), _p(u), n, _p(gret),
                              _p(gles), _p(gstv), _p(gkp), _p(grd), _p(gtv), _p(gu))
    return gkp, grd, gtv, gu


# ------------------------------------------------------------------------------------------
# Second-Born self-energy with a general four-index interaction (Eq. SE).
#
# Sigma_ij = sum_{f,d,e,a,b,c} U_ifde Uex_jabc A_fb A_ea C_cd, with Uex_jabc = 2 U_jbac - U_jabc,
# A = G^<>(t,t') and C = G^><(t',t) on the real axis, A = G^](t,tau) and C = G^[(tau,t) on the
# mixed branch.  The sum is handed to numpy as the printed expression itself, one einsum over all
# six summed indices; numpy picks the order in which it contracts them (a library step).  The
# plain six-fold loop in C (orc_gf2_block) pins it at the full orbital count.  U is real,
# U[i, f, d, e] = U_ifde.
# ------------------------------------------------------------------------------------------
def uex(U):
    """Exchange tensor of Eq. SE: Uex[j, a, b, c] = 2 U[j, b, a, c] - U[j, a, b, c]."""
    U = np.asarray(U, np.float64)
    return 2.0 * np.transpose(U, (0, 2, 1, 3)) - U


def gf2_block(U, A, C):
    """Eq. SE at one time argument pair: sum U_ifde Uex_jabc A_fb A_ea C_cd."""
    U = np.asarray(U, np.float64)
    return np.einsum("ifde,jabc,fb,ea,cd->ij", U, uex(U), A, A, C, optimize="optimal")


def gf2_block_loops(U, A, C):
    """Eq. SE at one time argument pair as the plain six-fold loop of orc_gf2_block (C, OpenMP
    over the output entries): the exchange tensor is formed inside the loop from U."""
    U = _c(U, np.float64)
    A, C = _c(A), _c(C)
    N = A.shape[0]
    out = np.empty((N, N), np.complex128)
    _load().orc_gf2_block(N, _p(U), _p(A), _p(C), _p(out))
    return out


def les_block(G: Green, a: int, b: int):
    """G^<(t_a, t_b) from the storage: kp[a][b] for a <= b, else -kp[b][a]^dagger."""
    return G.kp[a, b].copy() if a <= b else -G.kp[b, a].conj().T


def gtr_block(G: Green, a: int, b: int):
    """G^>(t_a, t_b): G^R + G^< for a >= b (G^R in rdiag at a = b), else -G^>(t_b, t_a)^dagger."""
    if a >= b:
        ret = G.rdiag[a] if a == b else G.kp[a, b]
        return ret + les_block(G, a, b)
    return -gtr_block(G, b, a).conj().T


def sigma_gf2_row(G: Green, U, n: int, s_list=None, l_list=None):
    """(ret[n+1], les[n+1], stv[ntau]) at t_n with a general U: ret = Sigma^> - Sigma^<,
    les = Sigma^<, stv[l] = Sigma^](t_n, tau_l) with G^[(tau_l, t_n) = G^](t_n, beta - tau_l)^dagger
    (symmetric tau grid: beta - tau_l = tau_{J-l}).  s_list / l_list restrict the computed
    entries (the others stay NaN)."""
    N = G.N
    ntau = G.ntau
    ret = np.full((n + 1, N, N), np.nan, np.complex128)
    les = np.full((n + 1, N, N), np.nan, np.complex128)
    stv = np.full((ntau, N, N), np.nan, np.complex128)
    for s in (range(n + 1) if s_list is None else s_list):
        l_ns, g_ns = les_block(G, n, s), gtr_block(G, n, s)
        l_sn, g_sn = les_block(G, s, n), gtr_block(G, s, n)
        sl = gf2_block(U, l_ns, g_sn)
        sg = gf2_block(U, g_ns, l_sn)
        les[s] = sl
        ret[s] = sg - sl
    J = ntau - 1
    for l in (range(ntau) if l_list is None else l_list):
        stv[l] = gf2_block(U, G.tv[n, l], G.tv[n, J - l].conj().T)
    return ret, les, stv


# ------------------------------------------------------------------------------------------
# Adjoint of one row's integrals (the row function above), from its sums term by term.
#
# With PyTorch's convention for complex gradients (g = dL/dRe + i dL/dIm), a term c A B adds
# conj(c) g B^dagger to the gradient of A and conj(c) A^dagger g to that of B, and a term
# c A B^dagger adds conj(c) g B to A's and c g^dagger A to B's.  Each input block of a row enters
# exactly one term, so every gradient block is one such product (zero for blocks the selected
# outputs do not read).
# ------------------------------------------------------------------------------------------
def collision_row_vjp(N: int, ntau: int, n: int, m: int, sig, col, row, rdg, tvm, wn, wm, wfull,
                      cot, flags: int = F_IR | F_IL | F_ITV):
    """Gradients (g_ret [n+1], g_les [n+1], g_stv [ntau], g_col [m+1], g_row [n+1], g_rdiag,
    g_tv [ntau]) of a real loss with cotangents cot = (gIR, gIL, gItv) of collision_row."""
    ret, les, stv = (np.asarray(x, np.complex128) for x in sig)
    gIR, gIL, gItv = (np.asarray(x, np.complex128) if x is not None else np.zeros((N, N), complex)
                      for x in cot)
    H = lambda x: x.conj().T
    z = lambda k: np.zeros((k, N, N), np.complex128)
    g_ret, g_les, g_stv, g_col, g_row, g_tv = z(n + 1), z(n + 1), z(ntau), z(m + 1), z(n + 1), z(ntau)
    g_rdg = np.zeros((N, N), np.complex128)
    if flags & F_IR:
        for s in range(m + 1):        # wn[s] ret[s] col[s]
            g_ret[s] = wn[s] * gIR @ H(col[s])
            g_col[s] = wn[s] * H(ret[s]) @ gIR
        for s in range(m + 1, n + 1):  # -wn[s] ret[s] row[s]^dagger
            g_ret[s] = -wn[s] * gIR @ row[s]
            g_row[s] = -wn[s] * H(gIR) @ ret[s]
    if flags & F_IL:
        for s in range(m):            # wm[s] les[s] row[s]^dagger
            g_les[s] = wm[s] * gIL @ row[s]
            g_row[s] = wm[s] * H(gIL) @ les[s]
        g_les[m] = wm[m] * gIL @ rdg  # wm[m] les[m] rdiag^dagger
        g_rdg = wm[m] * H(gIL) @ les[m]
    if (flags & F_ITV) and ntau > 0:
        J = ntau - 1
        for j in range(ntau):         # -i wfull[j] stv[j] tv[J-j]^dagger
            c = -1j * wfull[j]
            g_stv[j] = np.conj(c) * gItv @ tvm[J - j]
            g_tv[J - j] = c * H(gItv) @ stv[j]
    return g_ret, g_les, g_stv, g_col, g_row, g_rdg, g_tv


def sigma_full(G: Green, u):
    """Second-Born self-energy (local U) for every time pair, in KP storage like G:
    kp[a][b] = Sigma^<(t_a,t_b) for a <= b and Sigma^R(t_a,t_b) = Sigma^> - Sigma^< for a > b,
    rdiag[a] = Sigma^>(t_a,t_a) - Sigma^<(t_a,t_a), tv[a][l] = Sigma^](t_a,tau_l) (each entry from
    sigma_pair / sigma_row at its own arguments).  The Matsubara component is not produced (Eq. SE
    gives none)."""
    nt, N, ntau = G.nt, G.N, G.ntau
    kp = np.zeros((nt, nt, N, N), np.complex128)
    rd = np.zeros((nt, N, N), np.complex128)
    tv = np.zeros((nt, ntau, N, N), np.complex128)
    for a in range(nt):
        for b in range(nt):
            les, gtr = sigma_pair(G, u, a, b)
            if a <= b:
                kp[a, b] = les
            else:
                kp[a, b] = gtr - les
            if a == b:
                rd[a] = gtr - les
        if ntau:
            tv[a] = sigma_row(G, u, a)[2]
    return kp, rd, tv
