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


def scales(kp, rd, tv, mat, sig, W: oracle.Weights, n, ms, js, greater=False):
    """Sum over terms of |c| ||Q||_F ||P||_F for outputs IR(m), IL(m), Itv(m) (m in ms) and Jtv(j)
    (j in js): the rounding-error scale of each output block.  greater: the greater form, whose
    I^R also reads D(s,m) = G^>(s,m) - G^<(s,m) (kp[s][m] below the diagonal, rdiag[m] on it,
    kp[m][s] above it) and whose I^< reads Sigma^R + Sigma^< in place of Sigma^<."""
    ret, les, stv = sig
    rn, ln = bnorm(ret), bnorm(les)
    if greater:
        ln = ln + rn
    w = W.w
    out = {"IR": [], "IL": [], "Itv": [], "Jtv": []}
    ntau = 0 if tv is None else tv.shape[1]
    J = ntau - 1
    for m in ms:
        col = bnorm(kp[: m + 1, m])                # G^<(s,m) for s <= m
        rowb = bnorm(kp[m, : n + 1])               # kp[m][s]
        sR = np.sum(np.abs(w[n, : m + 1]) * rn[: m + 1] * col)
        sR += np.sum(np.abs(w[n, m + 1: n + 1]) * rn[m + 1: n + 1] * rowb[m + 1: n + 1])
        if greater:  # the D part: rowb[s] for s < m, rdiag[m], kp[s][m] for s > m
            lower = bnorm(kp[m + 1: n + 1, m])
            sR += np.sum(np.abs(w[n, :m]) * rn[:m] * rowb[:m])
            sR += abs(w[n, m]) * rn[m] * bnorm(rd[m]) if m <= n else 0.0
            sR += np.sum(np.abs(w[n, m + 1: n + 1]) * rn[m + 1: n + 1] * lower)
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


def vjp_scales(kp, rd, tv, mat, sig, W: oracle.Weights, n, m0, m1, cot, flags):
    """Rounding scales of the adjoint's gradient blocks (the bar of R14 applied to the VJP): for
    every gradient block, the sum over the forward terms that read its block of |c| times the
    norms of the term's other factor and of the cotangent of the term's output.  Returns a dict
    with the keys of the gradient arrays: kp [nt, nt], rdiag [nt], tv [nt, ntau], mat [ntau],
    ret [n+1], les [n+1], stv [ntau]."""
    nt = rd.shape[0]
    ntau = 0 if tv is None else tv.shape[1]
    J = ntau - 1
    ret, les, stv = sig
    nk = bnorm(kp[:, :nt])
    nr = bnorm(rd)
    ntv = bnorm(tv) if ntau else np.zeros((nt, 0))
    nmat = bnorm(mat) if ntau else np.zeros(0)
    nret, nles = bnorm(ret), bnorm(les)
    nstv = bnorm(stv) if ntau else np.zeros(0)
    cIR, cIL, cIt, cJ = (bnorm(c) if c is not None else None for c in cot)
    greater = bool(flags & oracle.F_GREATER)
    S = {"kp": np.zeros((nt, nt)), "rdiag": np.zeros(nt), "tv": np.zeros((nt, ntau)),
         "mat": np.zeros(ntau), "ret": np.zeros(n + 1), "les": np.zeros(n + 1),
         "stv": np.zeros(ntau)}
    w = np.abs(W.w)
    s_all = np.arange(n + 1)
    for m in range(m0, m1):
        o = m - m0
        if flags & oracle.F_IR:
            a = w[n, : n + 1]
            c = cIR[o]
            # G^<(s,m): kp[s][m] for s <= m, kp[m][s] for s > m
            P = np.where(s_all <= m, nk[: n + 1, m], nk[m, : n + 1])
            S["ret"] += a * P * c
            S["kp"][: m + 1, m] += a[: m + 1] * nret[: m + 1] * c
            S["kp"][m, m + 1: n + 1] += a[m + 1:] * nret[m + 1:] * c
            if greater:  # D(s,m): kp[s][m] (s > m), rdiag[m] (s = m), kp[m][s] (s < m)
                D = np.where(s_all > m, nk[: n + 1, m], nk[m, : n + 1])
                D[m] = nr[m]
                S["ret"] += a * D * c
                S["kp"][m + 1: n + 1, m] += a[m + 1:] * nret[m + 1:] * c
                S["kp"][m, :m] += a[:m] * nret[:m] * c
                S["rdiag"][m] += a[m] * nret[m] * c
        if flags & oracle.F_IL:
            b = w[m, : m + 1]
            c = cIL[o]
            nQ = nles[: m + 1] + (nret[: m + 1] if greater else 0.0)
            P = np.append(nk[m, :m], nr[m])  # G^R(m,s): kp[m][s] for s < m, rdiag[m] at s = m
            S["les"][: m + 1] += b * P * c
            if greater:
                S["ret"][: m + 1] += b * P * c
            S["kp"][m, :m] += b[:m] * nQ[:m] * c
            S["rdiag"][m] += b[m] * nQ[m] * c
        if (flags & oracle.F_ITV) and ntau:
            c = cIt[o]
            S["tv"][m, ::-1] += np.abs(W.wfull) * nstv * c
            S["stv"] += np.abs(W.wfull) * ntv[m, ::-1] * c
    if (flags & oracle.F_JTV) and ntau:
        a = w[n, : n + 1]
        S["tv"][: n + 1] += (a * nret)[:, None] * cJ[None, :]
        S["ret"] += a * (ntv[: n + 1] * cJ[None, :]).sum(axis=1)
        for j in range(ntau):
            for l in range(ntau):
                if l <= j:
                    c, k = abs(W.wf[j, l]), J + l - j
                    S["stv"][l] += c * nmat[k] * cJ[j]
                    S["mat"][k] += c * nstv[l] * cJ[j]
                if l >= j:
                    c, k = abs(W.wb[j, l]), l - j
                    S["stv"][l] += c * nmat[k] * cJ[j]
                    S["mat"][k] += c * nstv[l] * cJ[j]
    return S


def sigma_vjp_scales(kp, rd, tv, u, n, gsig):
    """Rounding scales of the Sigma-row adjoint's gradient blocks.  Each entry of the gradient is a
    short sum of products 2 u_i u_j g x y of a cotangent entry and two G entries; the Hadamard
    product obeys ||g o x o y||_F <= ||g||_F ||x||_F ||y||_F, so per block the scale is the sum of
    those norm products over the self-energy entries that read it."""
    G = oracle.Green(kp, rd, tv)
    nt = rd.shape[0]
    ntau = tv.shape[1]
    J = ntau - 1
    u2 = 4.0 * np.max(np.abs(u)) ** 2
    gret, gles, gstv = gsig
    S_kp, S_rd, S_tv = np.zeros((nt, nt)), np.zeros(nt), np.zeros((nt, ntau))
    nb = lambda x: np.linalg.norm(x)
    for s in range(n + 1):
        L, Lt = oracle.les_block(G, n, s), oracle.les_block(G, s, n)
        Gg, Gt = oracle.gtr_block(G, n, s), oracle.gtr_block(G, s, n)
        g = nb(gret[s]) + nb(gles[s])
        b = u2 * g * (nb(L) + nb(Gt) + nb(Gg) + nb(Lt)) ** 2
        S_kp[n, s] += b
        S_kp[s, n] += b
        if s == n:
            S_rd[n] += b
    for l in range(ntau):
        b = u2 * nb(gstv[l]) * (nb(tv[n, l]) + nb(tv[n, J - l])) ** 2
        S_tv[n, l] += b
        S_tv[n, J - l] += b
    return S_kp, S_rd, S_tv


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
