"""Seeded parity cases shared by the GPU tests: host inputs (numpy, from ``synth``), their device
copies, and the scale-aware comparison used for the FP64 parity bar."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle
import synth

RTOL = 1e-12  # FP64 parity bar: per block relative to the sum of |term| norms, and globally


@dataclass
class Case:
    N: int
    nt: int
    ntau: int
    beta: float
    seed: int
    omin: int = 3
    omax: int = 6
    hmin: float = 0.02
    hmax: float = 0.08
    tau_order: int = 5
    ldt: int | None = None
    U: float = 1.0

    def host(self):
        t, order = synth.grid(self.seed, self.nt, self.hmin, self.hmax, self.omin, self.omax)
        kp = synth.kp(self.seed, self.N, t, ldt=self.ldt)
        rd = synth.rdiag(self.N, self.nt)
        tv = synth.tv(self.seed, self.N, self.ntau, t)  # [nt, 0, N, N] without a thermal branch
        mat = synth.mat(self.seed, self.N, self.ntau)
        return t, order, kp, rd, tv, mat


def to_dev(x):
    import torch
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def to_host(x):
    return None if x is None else x.detach().cpu().numpy()


def device_green(kp, rd, tv, mat):
    import paper_2405_08737_amd as kbe
    return kbe.Green(to_dev(kp), to_dev(rd), to_dev(tv), to_dev(mat))


def device_weights(W: oracle.Weights):
    """Oracle weights handed to the GPU as inputs (so a collision test isolates the collision)."""
    import paper_2405_08737_amd as kbe
    has_tau = W.wfull.size > 0
    return kbe.Weights(to_dev(W.w), to_dev(W.wfull) if has_tau else None,
                       to_dev(W.wf) if has_tau else None)


def bnorm(x):
    """Frobenius norm of every N x N block of an array [..., N, N]."""
    return np.sqrt((np.abs(x) ** 2).sum(axis=(-1, -2)))


def scales(kp, rd, tv, mat, sig, W: oracle.Weights, n, ms, js):
    """Sum over terms of |c| ||Q||_F ||P||_F for outputs IR(m), IL(m), Itv(m) (m in ms) and Jtv(j)
    (j in js): the rounding-error scale of each output block."""
    ret, les, stv = sig
    rn, ln = bnorm(ret), bnorm(les)
    w = W.w
    out = {"IR": [], "IL": [], "Itv": [], "Jtv": []}
    ntau = 0 if tv is None else tv.shape[1]
    J = ntau - 1
    for m in ms:
        col = bnorm(kp[: m + 1, m])                # G^<(s,m) for s <= m
        rowb = bnorm(kp[m, : n + 1])               # kp[m][s]
        sR = np.sum(np.abs(w[n, : m + 1]) * rn[: m + 1] * col)
        sR += np.sum(np.abs(w[n, m + 1: n + 1]) * rn[m + 1: n + 1] * rowb[m + 1: n + 1])
        sL = np.sum(np.abs(w[m, :m]) * ln[:m] * rowb[:m]) + abs(w[m, m]) * ln[m] * bnorm(rd[m])
        out["IR"].append(sR)
        out["IL"].append(sL)
        if ntau:
            sn = bnorm(stv)
            out["Itv"].append(np.sum(np.abs(W.wfull) * sn * bnorm(tv[m])[::-1]))
    if ntau:
        sn, mn = bnorm(stv), bnorm(mat)
        for j in js:
            s = np.sum(np.abs(w[n, : n + 1]) * rn * bnorm(tv[: n + 1, j]))
            for l in range(ntau):
                if l <= j:
                    s += abs(W.wf[j, l]) * sn[l] * mn[J + l - j]
                if l >= j:
                    s += abs(W.wb[j, l]) * sn[l] * mn[l - j]
            out["Jtv"].append(s)
    return {k: np.array(v) for k, v in out.items()}


def assert_blocks_close(got, ref, scale, name, rtol=RTOL):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    d = bnorm(got - ref)
    bad = np.nonzero(d > rtol * np.maximum(scale, 1e-300))[0]
    assert bad.size == 0, f"{name}: blocks {bad[:8]} exceed {rtol} x scale (worst ratio " \
                          f"{(d / np.maximum(scale, 1e-300)).max():.3e})"
    gn = np.linalg.norm(ref.ravel())
    if gn > 0:
        rel = np.linalg.norm((got - ref).ravel()) / gn
        assert rel <= rtol, f"{name}: global relative error {rel:.3e} > {rtol}"


def row_scales(N, ntau, n, m, cr, wn, wm, wfull):
    """Rounding scales of one batch row's three blocks (the bar of R14 for a single output):
    sum over terms of |weight| * ||Q||_F * ||P||_F."""
    nrm = lambda x: np.linalg.norm(x.reshape(len(x), -1), axis=1)
    ret, les, stv = nrm(cr["ret"]), nrm(cr["les"]), nrm(cr["stv"]) if ntau else None
    col, row = nrm(cr["col"]), nrm(cr["row"])
    g_ir = np.concatenate([col, row[m + 1:n + 1]])
    s_ir = np.sum(np.abs(wn[:n + 1]) * ret[:n + 1] * g_ir)
    g_il = np.concatenate([row[:m], [np.linalg.norm(cr["rdiag"])]])
    s_il = np.sum(np.abs(wm[:m + 1]) * les[:m + 1] * g_il)
    s_tv = np.sum(np.abs(wfull) * stv * nrm(cr["tv"])[::-1]) if ntau else 0.0
    return s_ir, s_il, s_tv


def batch_item(kbe, cr, n, m, wn, wm, wfull, flags):
    """A kbe.BatchItem on the device from host cross arrays (synth.batch_cross's keys)."""
    c = lambda a: to_dev(np.ascontiguousarray(a))
    th = cr["stv"].shape[0] > 0
    return kbe.BatchItem(n=n, m=m, sig_ret=c(cr["ret"]), sig_les=c(cr["les"]), col=c(cr["col"]),
                         row=c(cr["row"]), rdiag=c(cr["rdiag"]), wn=c(wn), wm=c(wm),
                         sig_tv=c(cr["stv"]) if th else None, tv=c(cr["tv"]) if th else None,
                         wtau=c(wfull) if th else None, flags=flags)
