"""MI355X-native history integrals for adaptive Kadanoff-Baym propagation (arXiv:2405.08737).

Python binding of ``libkbe.so``: argument marshalling only.  Every step of the path runs in the
library's HIP kernels, called through its C ABI (``include/kbe.h``); PyTorch provides device
memory and the current stream.  Importing works without the library; the first call raises
``RuntimeError`` if ``libkbe.so`` has not been built (``python -m paper_2405_08737_amd.build``).

Arrays are torch tensors on a ROCm device: complex128 for Green's functions and self-energies
(layout in ``include/kbe.h``), float64 for weights and the interaction.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libkbe.so")

OUT_IR, OUT_IL, OUT_ITV, OUT_JTV = 0x1, 0x2, 0x4, 0x8
OUT_ALL = 0xF
FORCE_GENERIC = 0x100
GRAD_OVERWRITE = 0x200
GREATER = 0x400  # kbe_collision: the greater form of Eq. KBE2
NMAX, KMAX = 16, 20

_lib = None


class KBEError(RuntimeError):
    """A non-zero kbe_status.  `status` is the code; `partial` holds what a call that stopped
    part-way produced (kbe_propagate_adaptive's accepted steps on KBE_ESTEP), else None."""

    def __init__(self, msg, status=None, partial=None):
        super().__init__(msg)
        self.status = status
        self.partial = partial


KBE_ESTEP = 6
KBE_ECONV = 7


class _Prop(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("h0", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("pulse_amp", ctypes.c_double), ("pulse_t0", ctypes.c_double),
                ("pulse_sigma", ctypes.c_double), ("t", ctypes.c_void_p),
                ("order", ctypes.c_void_p), ("lam", ctypes.c_void_p)]


class _AdaptCtl(ctypes.Structure):
    _fields_ = [("t_end", ctypes.c_double), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("h0", ctypes.c_double), ("qmax", ctypes.c_int32), ("kmax", ctypes.c_int32),
                ("maxcor", ctypes.c_int32)]


class _AdaptTrace(ctypes.Structure):
    _fields_ = [("t", ctypes.c_void_p), ("q", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("ks", ctypes.c_void_p), ("err", ctypes.c_void_p), ("nt", ctypes.c_int32),
                ("rejected", ctypes.c_int32)]


class _EqCtl(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("mix", ctypes.c_double), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("change", ctypes.c_double)]


class _Green(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nt", ctypes.c_int32), ("ntau", ctypes.c_int32),
                ("ldt", ctypes.c_int64), ("kp", ctypes.c_void_p), ("rdiag", ctypes.c_void_p),
                ("tv", ctypes.c_void_p), ("mat", ctypes.c_void_p)]


class _Row(ctypes.Structure):
    _fields_ = [("ret", ctypes.c_void_p), ("les", ctypes.c_void_p), ("tv", ctypes.c_void_p)]


class _Grid(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int32), ("t", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("ntau", ctypes.c_int32), ("beta", ctypes.c_double), ("tau_order", ctypes.c_int32)]


class _Wts(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("wtau", ctypes.c_void_p), ("wtau_fwd", ctypes.c_void_p)]


class _SigBatchItem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nt", ctypes.c_int32), ("ntau", ctypes.c_int32),
                ("n", ctypes.c_int32), ("ldt", ctypes.c_int64)] + [
        (name, ctypes.c_void_p) for name in ("kp", "rdiag", "tv", "u", "ret", "les", "stv")]


class _BatchItem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("ntau", ctypes.c_int32), ("flags", ctypes.c_uint32), ("chunk", ctypes.c_int32)] + [
        (name, ctypes.c_void_p) for name in ("sig_ret", "sig_les", "sig_tv", "col", "row", "rdiag",
                                             "tv", "wn", "wm", "wtau", "IR", "IL", "Itv")] + [
        ("col_ld", ctypes.c_int64)]


class _BatchVjpItem(ctypes.Structure):
    _fields_ = [("row", _BatchItem)] + [
        (name, ctypes.c_void_p) for name in ("gIR", "gIL", "gItv", "g_sig_ret", "g_sig_les",
                                             "g_sig_tv", "g_col", "g_row", "g_rdiag", "g_tv")]


EXPORTS = ("kbe_weights_workspace", "kbe_weights", "kbe_sigma_2b", "kbe_collision_workspace",
           "kbe_collision", "kbe_collision_noalloc", "kbe_collision_both_workspace",
           "kbe_collision_both", "kbe_collision_both_vjp_workspace", "kbe_collision_both_vjp",
           "kbe_collision_vjp_workspace",
           "kbe_collision_vjp",
           "kbe_sigma_2b_vjp_workspace", "kbe_sigma_2b_vjp", "kbe_sigma_2b_full",
           "kbe_sigma_2b_batch",
           "kbe_sigma_gf2_workspace",
           "kbe_sigma_gf2", "kbe_collision_batch_workspace",
           "kbe_collision_batch", "kbe_collision_batch_tune", "kbe_collision_batch_tune_groups",
           "kbe_collision_batch_vjp_workspace", "kbe_collision_batch_vjp",
           "kbe_weights_dev_workspace", "kbe_weights_dev", "kbe_step_weights",
           "kbe_propagate_workspace", "kbe_propagate", "kbe_propagate_vjp",
           "kbe_propagate_adaptive_workspace", "kbe_propagate_adaptive",
           "kbe_equilibrium_workspace", "kbe_equilibrium",
           "kbe_status_string",
           "kbe_last_error", "kbe_version")


def lib():
    """Load libkbe.so (raises RuntimeError if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is not built: run `python -m paper_2405_08737_amd.build`")
        L = ctypes.CDLL(_SO)
        P, I32, I64, SZ, U32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                                ctypes.c_uint32)
        G, R, GR, W = (ctypes.POINTER(_Green), ctypes.POINTER(_Row), ctypes.POINTER(_Grid),
                       ctypes.POINTER(_Wts))
        sig = {
            "kbe_weights_workspace": (SZ, [GR]),
            "kbe_weights": (I32, [GR, P, P, P, P, SZ, P]),
            "kbe_sigma_2b": (I32, [G, P, I32, R, P]),
            "kbe_sigma_2b_full": (I32, [G, P, G, P]),
            "kbe_sigma_2b_batch": (I32, [P, P, I32, P]),
            "kbe_sigma_gf2_workspace": (SZ, [I32]),
            "kbe_sigma_gf2": (I32, [G, P, I32, R, P, SZ, P]),
            "kbe_collision_workspace": (SZ, [I32, I32, I32, I32, I32, I32, U32]),
            "kbe_collision": (I32, [G, R, W, I32, I32, I32, U32, P, P, P, P, P, SZ, P]),
            "kbe_collision_noalloc": (I32, [G, R, W, I32, I32, I32, U32, P, P, P, P, P]),
            "kbe_collision_both_workspace": (SZ, [I32, I32, I32, I32, I32, I32]),
            "kbe_collision_both": (I32, [G, R, W, I32, I32, I32, P, P, P, P, P, P, P, SZ, P]),
            "kbe_collision_both_vjp_workspace": (SZ, [I32, I32, I32, I32, I32, I32]),
            "kbe_collision_both_vjp": (I32, [G, R, W, I32, I32, I32, P, P, P, P, P, P, G, R, P,
                                             SZ, P]),
            "kbe_collision_vjp_workspace": (SZ, [I32, I32, I32, I32, I32, I32, U32]),
            "kbe_collision_vjp": (I32, [G, R, W, I32, I32, I32, U32, P, P, P, P, G, R, P, SZ, P]),
            "kbe_sigma_2b_vjp_workspace": (SZ, [I32, I32, I32]),
            "kbe_sigma_2b_vjp": (I32, [G, P, I32, R, G, P, P, SZ, P]),
            "kbe_collision_batch_workspace": (SZ, [P, I32, I32]),
            "kbe_collision_batch": (I32, [P, P, I32, I32, P, SZ, P]),
            "kbe_collision_batch_tune": (I32, [P, P, I32, P, SZ, P, P, P]),
            "kbe_collision_batch_tune_groups": (I32, [P, P, I32, P, SZ, P, P]),
            "kbe_collision_batch_vjp_workspace": (SZ, [I32]),
            "kbe_collision_batch_vjp": (I32, [P, P, I32, P, SZ, P]),
            "kbe_weights_dev_workspace": (SZ, [I32, I32]),
            "kbe_weights_dev": (I32, [P, P, I32, I32, ctypes.c_double, I32, P, P, P, P, P, SZ, P]),
            "kbe_step_weights": (I32, [P, P, I32, P, P, P]),
            "kbe_propagate_workspace": (SZ, [I32, I32, I32, I64, I32]),
            "kbe_propagate": (I32, [ctypes.POINTER(_Prop), W, G, P, P, SZ, P]),
            "kbe_propagate_vjp": (I32, [ctypes.POINTER(_Prop), W, G, P, P, P, P, SZ, P]),
            "kbe_propagate_adaptive_workspace": (SZ, [I32, I32, I32]),
            "kbe_propagate_adaptive": (I32, [ctypes.POINTER(_Prop), ctypes.POINTER(_AdaptCtl), W,
                                             G, P, ctypes.POINTER(_AdaptTrace), P, SZ, P]),
            "kbe_equilibrium_workspace": (SZ, [I32, I32]),
            "kbe_equilibrium": (I32, [I32, I32, ctypes.c_double, P, P, P,
                                      ctypes.POINTER(_EqCtl), P, P, SZ, P]),
            "kbe_status_string": (ctypes.c_char_p, [I32]),
            "kbe_last_error": (ctypes.c_char_p, []),
            "kbe_version": (I32, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(st: int, what: str):
    if st != 0:
        L = lib()
        raise KBEError(f"{what}: {L.kbe_status_string(st).decode()}: {L.kbe_last_error().decode()}",
                       st)


def _ptr(x: Optional[torch.Tensor]):
    if x is None:
        return None
    assert x.is_contiguous(), "tensors passed to libkbe must be contiguous"
    return x.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _as_dev(x, dtype, device) -> torch.Tensor:
    """A contiguous device copy of x (a tensor on any device, or array-like)."""
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    import numpy as np
    return torch.tensor(np.asarray(x, {torch.complex128: np.complex128,
                                       torch.float64: np.float64}[dtype]), device=device)


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class Green:
    """A Keldysh function in KP storage (device tensors, complex128)."""
    kp: torch.Tensor                 # [nt, ldt, N, N]
    rdiag: torch.Tensor              # [nt, N, N]
    tv: Optional[torch.Tensor] = None   # [nt, ntau, N, N]
    mat: Optional[torch.Tensor] = None  # [ntau, N, N]

    @property
    def N(self):
        return self.kp.shape[-1]

    @property
    def nt(self):
        return self.rdiag.shape[0]

    @property
    def ntau(self):
        return 0 if self.tv is None else self.tv.shape[1]

    @property
    def device(self):
        return self.kp.device

    def c(self) -> _Green:
        for name in ("kp", "rdiag", "tv", "mat"):
            x = getattr(self, name)
            if x is not None and (x.dtype != torch.complex128 or not x.is_contiguous()):
                raise TypeError(f"Green.{name} must be a contiguous complex128 tensor "
                                f"(got {x.dtype})")
        return _Green(self.N, self.nt, self.ntau, self.kp.shape[1], _ptr(self.kp),
                      _ptr(self.rdiag), _ptr(self.tv), _ptr(self.mat))

    def zeros_like(self) -> "Green":
        z = lambda x: None if x is None else torch.zeros_like(x)
        return Green(z(self.kp), z(self.rdiag), z(self.tv), z(self.mat))


@dataclass
class Weights:
    w: torch.Tensor                      # [nt, nt] float64
    wtau: Optional[torch.Tensor] = None  # [ntau]
    wtau_fwd: Optional[torch.Tensor] = None  # [ntau, ntau]

    def c(self) -> _Wts:
        return _Wts(_ptr(self.w), _ptr(self.wtau), _ptr(self.wtau_fwd))


def _row(ret, les, tv) -> _Row:
    return _Row(_ptr(ret), _ptr(les), _ptr(tv))


def weights(t, order, ntau: int = 0, beta: float = 0.0, tau_order: int = 5,
            device="cuda") -> Weights:
    """kbe_weights: composite real-time weights w[n][s] and the tau weights."""
    import numpy as np
    t = np.ascontiguousarray(t, dtype=np.float64)
    order = np.ascontiguousarray(order, dtype=np.int32)
    nt = len(t)
    g = _Grid(nt, t.ctypes.data, order.ctypes.data, ntau, float(beta), int(tau_order))
    w = torch.empty((nt, nt), dtype=torch.float64, device=device)
    wtau = torch.empty(ntau, dtype=torch.float64, device=device) if ntau > 0 else None
    wf = torch.empty((ntau, ntau), dtype=torch.float64, device=device) if ntau > 0 else None
    L = lib()
    nb = L.kbe_weights_workspace(ctypes.byref(g))
    ws = _ws(nb, device)
    _check(L.kbe_weights(ctypes.byref(g), _ptr(w), _ptr(wtau), _ptr(wf), _ptr(ws), nb,
                         _stream(w.device)), "kbe_weights")
    return Weights(w, wtau, wf)


def sigma_2b(G: Green, u: torch.Tensor, n: int):
    """kbe_sigma_2b: (ret[n+1], les[n+1], tv[ntau]) second-Born row at t_n."""
    N, dev = G.N, G.device
    ret = torch.empty((n + 1, N, N), dtype=torch.complex128, device=dev)
    les = torch.empty_like(ret)
    stv = torch.empty((G.ntau, N, N), dtype=torch.complex128, device=dev) if G.ntau else None
    row = _row(ret, les, stv)
    _check(lib().kbe_sigma_2b(ctypes.byref(G.c()), _ptr(u), n, ctypes.byref(row), _stream(dev)),
           "kbe_sigma_2b")
    return ret, les, stv


def sigma_2b_full(G: Green, u: torch.Tensor, S: Optional[Green] = None):
    """kbe_sigma_2b_full: Sigma for every time pair in KP storage (a Green with G's shapes;
    its mat is left as allocated)."""
    if S is None:
        S = G.zeros_like()
    _check(lib().kbe_sigma_2b_full(ctypes.byref(G.c()), _ptr(u), ctypes.byref(S.c()),
                                   _stream(G.device)), "kbe_sigma_2b_full")
    return S


def sigma_gf2(G: Green, U: torch.Tensor, n: int):
    """kbe_sigma_gf2: (ret[n+1], les[n+1], tv[ntau]) second-Born row at t_n with a general
    four-index interaction U [N, N, N, N] (float64, U[i, f, d, e] = U_ifde of Eq. SE)."""
    N, dev = G.N, G.device
    if tuple(U.shape) != (N, N, N, N) or U.dtype != torch.float64 or not U.is_contiguous():
        raise KBEError(f"U must be a contiguous float64 [{N}]*4 tensor, got {tuple(U.shape)} "
                       f"{U.dtype}")
    ret = torch.empty((n + 1, N, N), dtype=torch.complex128, device=dev)
    les = torch.empty_like(ret)
    stv = torch.empty((G.ntau, N, N), dtype=torch.complex128, device=dev) if G.ntau else None
    row = _row(ret, les, stv)
    L = lib()
    nb = L.kbe_sigma_gf2_workspace(N)
    ws = _ws(nb, dev)
    _check(L.kbe_sigma_gf2(ctypes.byref(G.c()), _ptr(U), n, ctypes.byref(row), _ptr(ws), nb,
                           _stream(dev)), "kbe_sigma_gf2")
    return ret, les, stv


def collision(G: Green, sig, W: Weights, n: int, m0: int = 0, m1: Optional[int] = None,
              flags: int = OUT_ALL):
    """kbe_collision: (IR, IL, Itv, Jtv); unselected outputs are None."""
    m1 = n + 1 if m1 is None else m1
    N, dev, M = G.N, G.device, m1 - m0
    mk = lambda k: torch.empty((k, N, N), dtype=torch.complex128, device=dev)
    IR = mk(M) if flags & OUT_IR else None
    IL = mk(M) if flags & OUT_IL else None
    Itv = mk(M) if flags & OUT_ITV else None
    Jtv = mk(G.ntau) if (flags & OUT_JTV) and G.ntau else None
    L = lib()
    nb = L.kbe_collision_workspace(N, G.nt, G.ntau, n, m0, m1, flags)
    ws = _ws(nb, dev)
    row = _row(*sig)
    _check(L.kbe_collision(ctypes.byref(G.c()), ctypes.byref(row), ctypes.byref(W.c()), n, m0, m1,
                           flags, _ptr(IR), _ptr(IL), _ptr(Itv), _ptr(Jtv), _ptr(ws), nb,
                           _stream(dev)), "kbe_collision")
    return IR, IL, Itv, Jtv


def collision_both(G: Green, sig, W: Weights, n: int, m0: int = 0, m1: Optional[int] = None):
    """kbe_collision_both: (IR, IL, Itv, Jtv) of the lesser form and (IRg, ILg) of the greater
    form from one pass; Itv and Jtv are None without a thermal branch."""
    m1 = n + 1 if m1 is None else m1
    N, dev, M = G.N, G.device, m1 - m0
    mk = lambda k: torch.empty((k, N, N), dtype=torch.complex128, device=dev)
    IR, IL, IRg, ILg = mk(M), mk(M), mk(M), mk(M)
    Itv = mk(M) if G.ntau else None
    Jtv = mk(G.ntau) if G.ntau else None
    L = lib()
    nb = L.kbe_collision_both_workspace(N, G.nt, G.ntau, n, m0, m1)
    ws = _ws(nb, dev)
    _check(L.kbe_collision_both(ctypes.byref(G.c()), ctypes.byref(_row(*sig)),
                                ctypes.byref(W.c()), n, m0, m1, _ptr(IR), _ptr(IL), _ptr(Itv),
                                _ptr(Jtv), _ptr(IRg), _ptr(ILg), _ptr(ws), nb, _stream(dev)),
           "kbe_collision_both")
    return IR, IL, Itv, Jtv, IRg, ILg


def collision_noalloc(G: Green, sig, W: Weights, n: int, m0: int = 0, m1: Optional[int] = None,
                      flags: int = OUT_ALL, out=None):
    """kbe_collision_noalloc: kbe_collision with the library's fixed scratch array as workspace.
    out: optional preallocated (IR, IL, Itv, Jtv) (created here when None)."""
    m1 = n + 1 if m1 is None else m1
    N, dev, M = G.N, G.device, m1 - m0
    if out is None:
        mk = lambda k: torch.empty((k, N, N), dtype=torch.complex128, device=dev)
        out = (mk(M) if flags & OUT_IR else None, mk(M) if flags & OUT_IL else None,
               mk(M) if flags & OUT_ITV else None,
               mk(G.ntau) if (flags & OUT_JTV) and G.ntau else None)
    IR, IL, Itv, Jtv = out
    _check(lib().kbe_collision_noalloc(ctypes.byref(G.c()), ctypes.byref(_row(*sig)),
                                       ctypes.byref(W.c()), n, m0, m1, flags, _ptr(IR), _ptr(IL),
                                       _ptr(Itv), _ptr(Jtv), _stream(dev)),
           "kbe_collision_noalloc")
    return IR, IL, Itv, Jtv


def collision_vjp(G: Green, sig, W: Weights, n: int, m0: int, m1: int, cot, flags: int = OUT_ALL,
                  gG: Optional[Green] = None):
    """kbe_collision_vjp: returns (gG, (gret, gles, gstv)); gG is accumulated into (or created
    zero) unless flags has GRAD_OVERWRITE."""
    N, dev = G.N, G.device
    if gG is None:
        gG = G.zeros_like()
    gret = torch.empty((n + 1, N, N), dtype=torch.complex128, device=dev)
    gles = torch.empty_like(gret)
    gstv = torch.empty((G.ntau, N, N), dtype=torch.complex128, device=dev) if G.ntau else None
    gIR, gIL, gItv, gJ = cot
    L = lib()
    nb = L.kbe_collision_vjp_workspace(N, G.nt, G.ntau, n, m0, m1, flags)
    ws = _ws(nb, dev)
    _check(L.kbe_collision_vjp(ctypes.byref(G.c()), ctypes.byref(_row(*sig)), ctypes.byref(W.c()),
                               n, m0, m1, flags, _ptr(gIR), _ptr(gIL), _ptr(gItv), _ptr(gJ),
                               ctypes.byref(gG.c()), ctypes.byref(_row(gret, gles, gstv)),
                               _ptr(ws), nb, _stream(dev)), "kbe_collision_vjp")
    return gG, (gret, gles, gstv)


def collision_both_vjp(G: Green, sig, W: Weights, n: int, m0: int, m1: int, cot,
                       gG: Optional[Green] = None):
    """kbe_collision_both_vjp: cot = (gIR, gIL, gItv, gJtv, gIRg, gILg) (gItv, gJtv None without a
    thermal branch); returns (gG, (gret, gles, gstv)); gG is accumulated into (or created zero)."""
    N, dev = G.N, G.device
    if gG is None:
        gG = G.zeros_like()
    gret = torch.empty((n + 1, N, N), dtype=torch.complex128, device=dev)
    gles = torch.empty_like(gret)
    gstv = torch.empty((G.ntau, N, N), dtype=torch.complex128, device=dev) if G.ntau else None
    gIR, gIL, gItv, gJ, gIRg, gILg = cot
    L = lib()
    nb = L.kbe_collision_both_vjp_workspace(N, G.nt, G.ntau, n, m0, m1)
    ws = _ws(nb, dev)
    _check(L.kbe_collision_both_vjp(ctypes.byref(G.c()), ctypes.byref(_row(*sig)),
                                    ctypes.byref(W.c()), n, m0, m1, _ptr(gIR), _ptr(gIL),
                                    _ptr(gItv), _ptr(gJ), _ptr(gIRg), _ptr(gILg),
                                    ctypes.byref(gG.c()), ctypes.byref(_row(gret, gles, gstv)),
                                    _ptr(ws), nb, _stream(dev)), "kbe_collision_both_vjp")
    return gG, (gret, gles, gstv)


def sigma_2b_vjp(G: Green, u: torch.Tensor, n: int, gsig, gG: Optional[Green] = None,
                 gu: Optional[torch.Tensor] = None):
    """kbe_sigma_2b_vjp: accumulates into gG and gu (created zero when None)."""
    dev = G.device
    if gG is None:
        gG = G.zeros_like()
    if gu is None:
        gu = torch.zeros(G.N, dtype=torch.float64, device=dev)
    L = lib()
    nb = L.kbe_sigma_2b_vjp_workspace(G.N, n, G.ntau)
    ws = _ws(nb, dev)
    _check(L.kbe_sigma_2b_vjp(ctypes.byref(G.c()), _ptr(u), n, ctypes.byref(_row(*gsig)),
                              ctypes.byref(gG.c()), _ptr(gu), _ptr(ws), nb, _stream(dev)),
           "kbe_sigma_2b_vjp")
    return gG, gu


# ------------------------------------------------------------------------------------------
# torch.autograd wrappers: forward and backward both run in libkbe's kernels.
# ------------------------------------------------------------------------------------------
class KBESigma2B(torch.autograd.Function):
    """(kp, rdiag, tv, u) -> (ret, les, stv) at row n; backward via kbe_sigma_2b_vjp (the row is
    recomputed from G, never stored)."""

    @staticmethod
    def forward(ctx, kp, rdiag, tv, mat, u, n: int):
        G = Green(kp, rdiag, tv, mat)
        ret, les, stv = sigma_2b(G, u, n)
        ctx.save_for_backward(kp, rdiag, tv, mat, u)
        ctx.n = n
        return ret, les, stv

    @staticmethod
    def backward(ctx, gret, gles, gstv):
        kp, rdiag, tv, mat, u = ctx.saved_tensors
        G = Green(kp, rdiag, tv, mat)
        z = lambda g, like: torch.zeros_like(like) if g is None else g.contiguous()
        gsig = (z(gret, kp[0, :ctx.n + 1]), z(gles, kp[0, :ctx.n + 1]),
                None if tv is None else z(gstv, tv[0]))
        gG, gu = sigma_2b_vjp(G, u, ctx.n, gsig)
        return gG.kp, gG.rdiag, gG.tv, gG.mat, gu, None


class KBECollision(torch.autograd.Function):
    """(kp, rdiag, tv, mat, ret, les, stv) -> (IR, IL, Itv, Jtv); backward via kbe_collision_vjp.
    greater=True takes the greater form of Eq. KBE2 (KBE_GREATER) in both directions."""

    @staticmethod
    def forward(ctx, kp, rdiag, tv, mat, ret, les, stv, W: Weights, n: int, m0: int, m1: int,
                greater: bool = False):
        G = Green(kp, rdiag, tv, mat)
        flags = OUT_ALL if tv is not None else (OUT_IR | OUT_IL)
        if greater:
            flags |= GREATER
        IR, IL, Itv, Jtv = collision(G, (ret, les, stv), W, n, m0, m1, flags)
        ctx.save_for_backward(kp, rdiag, tv, mat, ret, les, stv)
        ctx.W, ctx.n, ctx.m0, ctx.m1, ctx.flags = W, n, m0, m1, flags
        outs = [IR, IL] + ([Itv, Jtv] if tv is not None else [])
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        kp, rdiag, tv, mat, ret, les, stv = ctx.saved_tensors
        G = Green(kp, rdiag, tv, mat)
        M = ctx.m1 - ctx.m0
        N = kp.shape[-1]
        zeros = lambda k: torch.zeros((k, N, N), dtype=torch.complex128, device=kp.device)
        g = [gr.contiguous() if gr is not None else None for gr in grads]
        gIR = g[0] if g[0] is not None else zeros(M)
        gIL = g[1] if g[1] is not None else zeros(M)
        gItv = gJ = None
        if tv is not None:
            gItv = g[2] if g[2] is not None else zeros(M)
            gJ = g[3] if g[3] is not None else zeros(G.ntau)
        gG, (gret, gles, gstv) = collision_vjp(G, (ret, les, stv), ctx.W, ctx.n, ctx.m0, ctx.m1,
                                               (gIR, gIL, gItv, gJ), ctx.flags)
        return gG.kp, gG.rdiag, gG.tv, gG.mat, gret, gles, gstv, None, None, None, None, None


# ------------------------------------------------------------------------------------------
# Batches of history rows (kbe_collision_batch).
# ------------------------------------------------------------------------------------------
@dataclass
class BatchItem:
    """One history row (t_n, t_m) of one system in cross storage (device tensors of that system's
    N; layout in include/kbe.h): the self-energy row at t_n, kp column m (rows 0..m), kp row m
    (columns 0..n), G^R(t_m, t_m), tv row m, the weight rows w[n][:n+1] and w[m][:m+1], the tau
    rule.  flags selects I^R, I^<, I^] (OUT_IR | OUT_IL | OUT_ITV)."""
    n: int
    m: int
    sig_ret: torch.Tensor              # [n+1, N, N]
    sig_les: torch.Tensor              # [n+1, N, N]
    col: torch.Tensor                  # [m+1, N, N]; or, with col_ld > 1, the first block
    row: torch.Tensor                  # [n+1, N, N]
    rdiag: torch.Tensor                # [N, N]
    wn: torch.Tensor                   # [n+1] float64
    wm: torch.Tensor                   # [m+1] float64
    sig_tv: Optional[torch.Tensor] = None  # [ntau, N, N]
    tv: Optional[torch.Tensor] = None      # [ntau, N, N]
    wtau: Optional[torch.Tensor] = None    # [ntau] float64
    flags: int = OUT_IR | OUT_IL | OUT_ITV
    col_ld: int = 0  # blocks between col[s] and col[s+1] (0: contiguous; a KP column: its ldt)

    @property
    def N(self):
        return self.rdiag.shape[-1]

    @property
    def ntau(self):
        return 0 if self.tv is None else self.tv.shape[0]


class Batch:
    """A fixed batch of rows: the item table (host array and device copy), the outputs and the
    workspace are allocated once; run() then only enqueues the library call, so it can be
    captured in a CUDA/HIP graph and replayed.  Outputs: self.IR[i], self.IL[i], self.Itv[i]
    (N x N blocks; None where the item's flag is off)."""

    def __init__(self, items, device=None):
        self.items = list(items)
        self.count = len(self.items)
        dev = device if device is not None else self.items[0].rdiag.device
        self.device = dev
        mk = lambda it, f: (torch.empty((it.N, it.N), dtype=torch.complex128, device=dev)
                            if it.flags & f else None)
        self.IR = [mk(it, OUT_IR) for it in self.items]
        self.IL = [mk(it, OUT_IL) for it in self.items]
        self.Itv = [mk(it, OUT_ITV) for it in self.items]
        host = (_BatchItem * max(self.count, 1))()
        for i, it in enumerate(self.items):
            host[i] = _BatchItem(it.N, it.n, it.m, it.ntau, it.flags, 0, _ptr(it.sig_ret),
                                 _ptr(it.sig_les), _ptr(it.sig_tv), _ptr(it.col), _ptr(it.row),
                                 _ptr(it.rdiag), _ptr(it.tv), _ptr(it.wn), _ptr(it.wm),
                                 _ptr(it.wtau), _ptr(self.IR[i]), _ptr(self.IL[i]),
                                 _ptr(self.Itv[i]), int(it.col_ld))
        self._host = host
        raw = bytes(host)[:ctypes.sizeof(_BatchItem) * self.count]
        self._dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
        L = lib()
        self.ws_bytes = L.kbe_collision_batch_workspace(host, self.count, 32)  # the largest chunk need
        if self.count and self.ws_bytes == 0:
            raise KBEError("kbe_collision_batch_workspace: invalid items")
        self.ws = _ws(self.ws_bytes, dev)

    def run(self, chunk: int = 0):
        """Enqueue kbe_collision_batch on the current stream (chunk 0: each item's own chunk from
        the tile table, or the library default where it has none)."""
        _check(lib().kbe_collision_batch(self._host, _ptr(self._dev), self.count, chunk,
                                         _ptr(self.ws), self.ws_bytes, _stream(self.device)),
               "kbe_collision_batch")
        return self.IR, self.IL, self.Itv

    def tune(self):
        """The library's autotuner: (best chunk, {chunk: ms})."""
        best = ctypes.c_int32(0)
        times = (ctypes.c_float * 4)()
        _check(lib().kbe_collision_batch_tune(self._host, _ptr(self._dev), self.count,
                                              _ptr(self.ws), self.ws_bytes, _stream(self.device),
                                              ctypes.byref(best), times),
               "kbe_collision_batch_tune")
        return best.value, dict(zip((32, 64, 128, 256), list(times)))

    @staticmethod
    def group(N: int, n: int) -> str:
        """Tile-table key of a row: its N and length bucket floor(log2(n + 1))."""
        return f"{N}:{(n + 1).bit_length() - 1}"

    def tune_groups(self):
        """The library's per-group autotuner (kbe_collision_batch_tune_groups): sets every item's
        chunk to its group's and returns (ms of the tuned call, tile table {group: chunk})."""
        ms = ctypes.c_float(0.0)
        _check(lib().kbe_collision_batch_tune_groups(self._host, _ptr(self._dev), self.count,
                                                     _ptr(self.ws), self.ws_bytes,
                                                     _stream(self.device), ctypes.byref(ms)),
               "kbe_collision_batch_tune_groups")
        return ms.value, self.table()

    def table(self):
        """The items' chunks as a tile table {group: chunk} (items of a group share one)."""
        return {self.group(it.N, it.n): int(self._host[i].chunk)
                for i, it in enumerate(self.items)}

    def apply_table(self, table):
        """Set each item's chunk from a tile table (0, the default, for groups it lacks) and copy
        the item array to the device again."""
        for i, it in enumerate(self.items):
            c = int(table.get(self.group(it.N, it.n), 0))
            if c not in (0, 32, 64, 128, 256):
                raise KBEError(f"tile table: chunk {c} for group {self.group(it.N, it.n)}")
            self._host[i].chunk = c
        raw = bytes(self._host)[:ctypes.sizeof(_BatchItem) * self.count]
        self._dev.copy_(torch.frombuffer(bytearray(raw), dtype=torch.uint8))

    def save_table(self, path):
        """Write the tile table as JSON."""
        with open(path, "w") as f:
            json.dump({"key": "N:floor(log2(n+1))", "chunk": self.table()}, f, indent=1,
                      sort_keys=True)

    def load_table(self, path):
        """Read a tile table written by save_table and apply it."""
        with open(path) as f:
            self.apply_table(json.load(f)["chunk"])


class SigmaBatch:
    """Self-energy rows of many systems in one launch (kbe_sigma_2b_batch).  rows: a list of
    (G, u, n) with G a Green (its own N, storage and grid), u [N] float64 on the device and n the
    row.  The outputs self.rows[i] = (ret[n+1], les[n+1], stv[ntau] or None), the item table
    (host and device copy) are allocated once; run() only enqueues the call, so it can be captured
    in a graph."""

    def __init__(self, rows, device=None):
        self.specs = list(rows)
        self.count = len(self.specs)
        dev = device if device is not None else (self.specs[0][0].device if self.specs else None)
        self.device = dev
        host = (_SigBatchItem * max(self.count, 1))()
        self.rows = []
        for i, (G, u, n) in enumerate(self.specs):
            mk = lambda k: torch.empty((k, G.N, G.N), dtype=torch.complex128, device=dev)
            out = (mk(n + 1), mk(n + 1), mk(G.ntau) if G.ntau else None)
            self.rows.append(out)
            host[i] = _SigBatchItem(G.N, G.nt, G.ntau, int(n), G.kp.shape[1], _ptr(G.kp),
                                    _ptr(G.rdiag), _ptr(G.tv) if G.ntau else None, _ptr(u),
                                    _ptr(out[0]), _ptr(out[1]), _ptr(out[2]))
        self._host = host
        raw = bytes(host)[:ctypes.sizeof(_SigBatchItem) * self.count]
        self._dev = (torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
                     if self.count else None)

    def run(self):
        _check(lib().kbe_sigma_2b_batch(self._host, _ptr(self._dev), self.count,
                                        _stream(self.device) if self.count else None),
               "kbe_sigma_2b_batch")
        return self.rows


class BatchVJP:
    """The adjoint of a fixed batch of rows (kbe_collision_batch_vjp): items as for Batch, cot a
    list of (gIR, gIL, gItv) N x N cotangent tensors per item (None where a flag is off).  The
    gradient arrays, the item table (host and device copy) and the workspace are allocated once;
    run() only enqueues the call.  Gradients: self.g[i] = dict(sig_ret, sig_les, sig_tv, col,
    row, rdiag, tv) of device tensors (sig_tv and tv None without a thermal branch)."""

    def __init__(self, items, cot, device=None):
        self.items = list(items)
        self.count = len(self.items)
        dev = device if device is not None else self.items[0].rdiag.device
        self.device = dev
        self.cot = [tuple(c) for c in cot]
        mk = lambda k, N: torch.empty((k, N, N), dtype=torch.complex128, device=dev)
        self.g = []
        host = (_BatchVjpItem * max(self.count, 1))()
        for i, (it, c) in enumerate(zip(self.items, self.cot)):
            N, n, m, nt = it.N, it.n, it.m, it.ntau
            g = dict(sig_ret=mk(n + 1, N), sig_les=mk(n + 1, N), sig_tv=mk(nt, N) if nt else None,
                     col=mk(m + 1, N), row=mk(n + 1, N),
                     rdiag=torch.empty((N, N), dtype=torch.complex128, device=dev),
                     tv=mk(nt, N) if nt else None)
            self.g.append(g)
            row = _BatchItem(N, n, m, nt, it.flags, 0, _ptr(it.sig_ret), _ptr(it.sig_les),
                             _ptr(it.sig_tv), _ptr(it.col), _ptr(it.row), _ptr(it.rdiag),
                             _ptr(it.tv), _ptr(it.wn), _ptr(it.wm), _ptr(it.wtau), None, None, None,
                             int(it.col_ld))
            host[i] = _BatchVjpItem(row, _ptr(c[0]), _ptr(c[1]), _ptr(c[2]), _ptr(g["sig_ret"]),
                                    _ptr(g["sig_les"]), _ptr(g["sig_tv"]), _ptr(g["col"]),
                                    _ptr(g["row"]), _ptr(g["rdiag"]), _ptr(g["tv"]))
        self._host = host
        raw = bytes(host)[:ctypes.sizeof(_BatchVjpItem) * self.count]
        self._dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
        L = lib()
        self.ws_bytes = L.kbe_collision_batch_vjp_workspace(self.count)
        self.ws = _ws(self.ws_bytes, dev)

    def run(self):
        """Enqueue kbe_collision_batch_vjp on the current stream."""
        _check(lib().kbe_collision_batch_vjp(self._host, _ptr(self._dev), self.count,
                                             _ptr(self.ws), self.ws_bytes,
                                             _stream(self.device)), "kbe_collision_batch_vjp")
        return self.g


# ------------------------------------------------------------------------------------------------
# Grid on the device; fixed-grid propagation and its adjoint.
# ------------------------------------------------------------------------------------------------
KMAX = 20


def weights_dev(t: torch.Tensor, order: torch.Tensor, ntau: int = 0, beta: float = 0.0,
                tau_order: int = 5, check: bool = True) -> Weights:
    """kbe_weights_dev: the weights of a grid held in device memory (t float64, order int32).
    With check, the device-side grid status is read back and a bad grid raises."""
    nt, dev = t.shape[0], t.device
    w = torch.empty((nt, nt), dtype=torch.float64, device=dev)
    wtau = torch.empty(ntau, dtype=torch.float64, device=dev) if ntau > 0 else None
    wf = torch.empty((ntau, ntau), dtype=torch.float64, device=dev) if ntau > 0 else None
    status = torch.zeros(1, dtype=torch.int32, device=dev) if check else None
    L = lib()
    nb = L.kbe_weights_dev_workspace(nt, ntau)
    ws = _ws(nb, dev)
    _check(L.kbe_weights_dev(_ptr(t), _ptr(order), nt, ntau, float(beta), int(tau_order), _ptr(w),
                             _ptr(wtau), _ptr(wf), _ptr(status), _ptr(ws), nb, _stream(dev)),
           "kbe_weights_dev")
    if check and int(status.item()) != 0:
        raise KBEError(f"kbe_weights_dev: grid status {int(status.item())}")
    return Weights(w, wtau, wf)


def step_weights(t: torch.Tensor, order: torch.Tensor) -> torch.Tensor:
    """kbe_step_weights: lam [nt, KMAX, KMAX] local weights for every interval and node count."""
    nt, dev = t.shape[0], t.device
    lam = torch.empty((nt, KMAX, KMAX), dtype=torch.float64, device=dev)
    _check(lib().kbe_step_weights(_ptr(t), _ptr(order), nt, _ptr(lam), None, _stream(dev)),
           "kbe_step_weights")
    return lam


class Propagation:
    """A fixed-grid propagation problem on the device (kbe_propagate / kbe_propagate_vjp).

    t, order: the grid (host arrays); h0 [N, N] real; ntau, beta, tau_order: the thermal branch;
    mat [ntau, N, N] complex (G^M, the initial state) or, without a thermal branch, rho0 [N, N]
    (G^<(0,0) = i rho0); iters: fixed-point iterations per step; the pulse is
    amp * exp(-(t - pulse_t0)^2 / (2 pulse_sigma^2)) on h0[0][0]."""

    def __init__(self, t, order, h0, ntau=0, beta=1.0, tau_order=5, mat=None, rho0=None,
                 iters=2, pulse_t0=2.0, pulse_sigma=1.0, device="cuda:0"):
        import numpy as np
        dev = torch.device(device)
        self.device = dev
        h0 = np.ascontiguousarray(h0, np.float64)
        N, nt = h0.shape[0], len(t)
        self.N, self.nt, self.ntau, self.iters = N, nt, ntau, int(iters)
        self.t = torch.tensor(np.asarray(t, np.float64), device=dev)
        self.order = torch.tensor(np.asarray(order, np.int32), device=dev)
        self.h0 = torch.tensor(h0, device=dev)
        self.pulse_t0, self.pulse_sigma = float(pulse_t0), float(pulse_sigma)
        self.W = weights_dev(self.t, self.order, ntau, beta, tau_order)
        self.lam = step_weights(self.t, self.order)
        z = lambda *sh: torch.zeros(sh, dtype=torch.complex128, device=dev)
        self.G = Green(z(nt, nt, N, N), z(nt, N, N), z(nt, ntau, N, N) if ntau else None,
                       _as_dev(mat, torch.complex128, dev) if ntau else None)
        if not ntau:
            self.G.kp[0, 0] = 1j * torch.tensor(np.asarray(rho0, np.complex128), device=dev)
        self.dens = torch.empty((nt, N), dtype=torch.float64, device=dev)
        L = lib()
        self.nb = L.kbe_propagate_workspace(N, nt, ntau, nt, self.iters)
        self.ws = _ws(self.nb, dev)
        self._u = None
        self._amp = None

    def _p(self, u: torch.Tensor, amp: float) -> _Prop:
        self._u = u
        return _Prop(self.iters, _ptr(self.h0), _ptr(u), float(amp), self.pulse_t0,
                     self.pulse_sigma, _ptr(self.t), _ptr(self.order), _ptr(self.lam))

    def run(self, u: torch.Tensor, amp: float) -> torch.Tensor:
        """kbe_propagate: densities n_i(t_n) [nt, N]; the solution is left in self.G."""
        u = u.detach().to(device=self.device, dtype=torch.float64).contiguous()
        self._amp = float(amp)
        P = self._p(u, amp)
        _check(lib().kbe_propagate(ctypes.byref(P), ctypes.byref(self.W.c()),
                                   ctypes.byref(self.G.c()), _ptr(self.dens), _ptr(self.ws),
                                   self.nb, _stream(self.device)), "kbe_propagate")
        return self.dens

    def vjp(self, gdens: torch.Tensor):
        """kbe_propagate_vjp after run(): (dL/du [N], dL/dA) for the cotangent gdens [nt, N]."""
        gdens = gdens.detach().to(device=self.device, dtype=torch.float64).contiguous()
        gu = torch.empty(self.N, dtype=torch.float64, device=self.device)
        ga = torch.empty(1, dtype=torch.float64, device=self.device)
        P = self._p(self._u, self._amp)
        _check(lib().kbe_propagate_vjp(ctypes.byref(P), ctypes.byref(self.W.c()),
                                       ctypes.byref(self.G.c()), _ptr(gdens), _ptr(gu), _ptr(ga),
                                       _ptr(self.ws), self.nb, _stream(self.device)),
               "kbe_propagate_vjp")
        return gu, ga[0]


class KBEPropagate(torch.autograd.Function):
    """dens = KBEPropagate.apply(prop, u, amp): differentiable in u [N] and amp (0-dim tensor)."""

    @staticmethod
    def forward(ctx, prop: Propagation, u, amp):
        ctx.prop = prop
        return prop.run(u, float(amp)).clone()

    @staticmethod
    def backward(ctx, gdens):
        gu, ga = ctx.prop.vjp(gdens)
        return None, gu, ga


def equilibrium(h0, u, mu, beta, ntau, *, tau_order=5, wtau_fwd=None, mix=0.5, tol=1e-13,
                maxit=1000, device="cuda:0"):
    """kbe_equilibrium: the interacting equilibrium G^M [ntau, N, N] (complex128, real valued) of
    the local-U second-Born approximation at inverse temperature beta and chemical potential mu,
    and {"iterations", "change"}.  wtau_fwd: the tau rule (computed here when None).  A run that
    does not converge raises KBEError with (G^M, info) of the last iterate in `partial`."""
    import numpy as np
    dev = torch.device(device)
    h0 = torch.as_tensor(np.ascontiguousarray(h0, np.float64), device=dev)
    N = h0.shape[0]
    ud = torch.as_tensor(np.broadcast_to(np.asarray(u, np.float64), (N,)).copy(), device=dev)
    if wtau_fwd is None:
        wtau_fwd = weights_dev(torch.zeros(1, dtype=torch.float64, device=dev),
                               torch.ones(1, dtype=torch.int32, device=dev), ntau, beta,
                               tau_order).wtau_fwd
    mat = torch.empty((ntau, N, N), dtype=torch.complex128, device=dev)
    C = _EqCtl(float(mu), float(mix), float(tol), int(maxit), 0, 0.0)
    L = lib()
    nb = L.kbe_equilibrium_workspace(N, ntau)
    ws = _ws(nb, dev)
    st = L.kbe_equilibrium(N, ntau, float(beta), _ptr(wtau_fwd), _ptr(h0), _ptr(ud),
                           ctypes.byref(C), _ptr(mat), _ptr(ws), nb, _stream(dev))
    info = {"iterations": C.iterations, "change": C.change}
    if st == KBE_ECONV:
        raise KBEError(f"kbe_equilibrium: {L.kbe_status_string(st).decode()}: "
                       f"{L.kbe_last_error().decode()}", st, (mat, info))
    _check(st, "kbe_equilibrium")
    return mat, info


KS_STRIDE = 14  # history orders recorded per step in the adaptive trace


def propagate_adaptive(h0, u, pulse_amp, t_end, *, ntau=0, beta=1.0, tau_order=5, mat=None,
                       rho0=None, capacity=4096, rtol=1e-6, atol=1e-10, h_first=1e-3, qmax=12,
                       kmax=10, maxcor=3, pulse_t0=2.0, pulse_sigma=1.0, device="cuda:0"):
    """kbe_propagate_adaptive: returns a dict with the grid t, the per-step orders q, iteration
    counts m, history orders ks (one list per step, the iterations and the final evaluation),
    error norms err, the number of rejected attempts, the densities dens [nt, N] and the solution
    G (capacity points allocated, the first len(t) used).  The trace has the oracle's replay
    format in `replay` ([None] + one dict per step).  A run that stops before t_end (step-size
    underflow, capacity exhausted) raises KBEError with that dict, up to the stop, in `partial`."""
    import numpy as np
    dev = torch.device(device)
    h0 = np.ascontiguousarray(h0, np.float64)
    N = h0.shape[0]
    u = torch.as_tensor(np.broadcast_to(np.asarray(u, np.float64), (N,)).copy(), device=dev)
    zero_t = torch.zeros(1, dtype=torch.float64, device=dev)
    one_o = torch.ones(1, dtype=torch.int32, device=dev)
    W = weights_dev(zero_t, one_o, ntau, beta, tau_order)
    z = lambda *sh: torch.zeros(sh, dtype=torch.complex128, device=dev)
    G = Green(z(capacity, capacity, N, N), z(capacity, N, N),
              z(capacity, ntau, N, N) if ntau else None,
              _as_dev(mat, torch.complex128, dev) if ntau else None)
    if not ntau:
        G.kp[0, 0] = 1j * torch.tensor(np.asarray(rho0, np.complex128), device=dev)
    dens = torch.zeros((capacity, N), dtype=torch.float64, device=dev)
    h0d = torch.tensor(h0, device=dev)
    P = _Prop(1, _ptr(h0d), _ptr(u), float(pulse_amp), float(pulse_t0), float(pulse_sigma), None,
              None, None)
    C = _AdaptCtl(float(t_end), float(rtol), float(atol), float(h_first), int(qmax), int(kmax),
                  int(maxcor))
    tt = np.zeros(capacity)
    qq = np.zeros(capacity, np.int32)
    mm = np.zeros(capacity, np.int32)
    kk = np.zeros((capacity, KS_STRIDE), np.int32)
    ee = np.zeros(capacity)
    T = _AdaptTrace(tt.ctypes.data, qq.ctypes.data, mm.ctypes.data, kk.ctypes.data,
                    ee.ctypes.data, 0, 0)
    L = lib()
    nb = L.kbe_propagate_adaptive_workspace(N, capacity, ntau)
    ws = _ws(nb, dev)
    st = L.kbe_propagate_adaptive(ctypes.byref(P), ctypes.byref(C), ctypes.byref(W.c()),
                                  ctypes.byref(G.c()), _ptr(dens), ctypes.byref(T), _ptr(ws), nb,
                                  _stream(dev))
    del ws
    if st not in (0, KBE_ESTEP):
        _check(st, "kbe_propagate_adaptive")
    n = T.nt
    replay = [None] + [{"t": float(tt[i]), "q": int(qq[i]), "m": int(mm[i]),
                        "ks": [int(x) for x in kk[i, : mm[i] + 1]]} for i in range(1, n)]
    res = {"t": tt[:n].copy(), "q": qq[:n].copy(), "m": mm[:n].copy(),
           "ks": [r["ks"] for r in replay[1:]], "err": ee[:n].copy(), "rejected": T.rejected,
           "dens": dens[:n], "G": G, "replay": replay, "workspace_bytes": nb}
    if st == KBE_ESTEP:
        raise KBEError(f"kbe_propagate_adaptive: {L.kbe_status_string(st).decode()}: "
                       f"{L.kbe_last_error().decode()}", st, res)
    return res

