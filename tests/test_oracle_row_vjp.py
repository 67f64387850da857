"""Pins for oracle.collision_row_vjp, the adjoint of one row's integrals.

  * Exact adjoint identities: the row integrals are linear in the self-energy blocks (G blocks
    fixed) and linear in the Green's-function blocks (Sigma fixed), so for any directions
    Re<cot, J dX> = Re<gX, dX> must hold to rounding, with J dX computed by the pinned forward
    oracle.collision_row.
  * Agreement with the full-system adjoint oracle.collision_vjp restricted to one column m, for
    rows cut from a full system: the row's gradient blocks are the full gradients at the blocks
    the row reads (kp column m, kp row m, rdiag[m], tv row m, and the self-energy row).
  * Output subsets: a block no selected output reads gets a zero gradient.
"""
import numpy as np
import pytest

import oracle
import synth

FL = oracle.F_IR | oracle.F_IL | oracle.F_ITV


def _rdot(a, b):
    return float(np.sum((np.conj(a) * b).real))


def _row_case(N, n, m, ntau, seed):
    rng = np.random.default_rng(seed)
    cm = lambda *s: rng.normal(size=s + (N, N)) + 1j * rng.normal(size=s + (N, N))
    sig = (cm(n + 1), cm(n + 1), cm(ntau))
    blocks = dict(col=cm(m + 1), row=cm(n + 1), rdg=cm(1)[0], tvm=cm(ntau))
    wn, wm, wf = rng.uniform(0.1, 1.0, n + 1), rng.uniform(0.1, 1.0, m + 1), rng.uniform(0.1, 1.0, ntau)
    cot = (cm(1)[0], cm(1)[0], cm(1)[0])
    return sig, blocks, wn, wm, wf, cot, cm


def _fwd(N, ntau, n, m, sig, b, wn, wm, wf, flags):
    return oracle.collision_row(N, ntau, n, m, sig, b["col"], b["row"], b["rdg"],
                                b["tvm"] if ntau else None, wn, wm, wf if ntau else None, flags)


@pytest.mark.parametrize("N,n,m,ntau,flags", [(1, 5, 2, 4, FL), (3, 9, 0, 5, FL), (3, 9, 9, 5, FL),
                                               (4, 6, 3, 0, oracle.F_IR | oracle.F_IL),
                                               (2, 7, 4, 6, oracle.F_IL), (5, 0, 0, 3, FL)])
def test_adjoint_identities(N, n, m, ntau, flags):
    sig, b, wn, wm, wf, cot, cm = _row_case(N, n, m, ntau, 10 * N + n + m)
    g = oracle.collision_row_vjp(N, ntau, n, m, sig, b["col"], b["row"], b["rdg"], b["tvm"], wn, wm,
                                 wf, cot, flags)
    g_ret, g_les, g_stv, g_col, g_row, g_rdg, g_tv = g
    # Sigma direction (G blocks fixed)
    dS = (cm(n + 1), cm(n + 1), cm(ntau))
    out = _fwd(N, ntau, n, m, dS, b, wn, wm, wf, flags)
    lhs = sum(_rdot(c, o) for c, o in zip(cot, out))
    rhs = _rdot(g_ret, dS[0]) + _rdot(g_les, dS[1]) + _rdot(g_stv, dS[2])
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)
    # Green's-function direction (Sigma fixed)
    dB = dict(col=cm(m + 1), row=cm(n + 1), rdg=cm(1)[0], tvm=cm(ntau))
    out = _fwd(N, ntau, n, m, sig, dB, wn, wm, wf, flags)
    lhs = sum(_rdot(c, o) for c, o in zip(cot, out))
    rhs = (_rdot(g_col, dB["col"]) + _rdot(g_row, dB["row"]) + _rdot(g_rdg, dB["rdg"]) +
           _rdot(g_tv, dB["tvm"]))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_unread_blocks_get_zero_gradient():
    N, n, m, ntau = 3, 8, 4, 5
    sig, b, wn, wm, wf, cot, _ = _row_case(N, n, m, ntau, 3)
    g_ret, g_les, g_stv, g_col, g_row, g_rdg, g_tv = oracle.collision_row_vjp(
        N, ntau, n, m, sig, b["col"], b["row"], b["rdg"], b["tvm"], wn, wm, wf, cot, FL)
    assert not g_les[m + 1:].any() and not g_row[m].any()
    g = oracle.collision_row_vjp(N, ntau, n, m, sig, b["col"], b["row"], b["rdg"], b["tvm"], wn, wm,
                                 wf, cot, oracle.F_ITV)
    for x in g[:2] + g[3:6]:
        assert not np.any(x)
    assert np.any(g[2]) and np.any(g[6])


@pytest.mark.parametrize("N,nt,ntau", [(2, 12, 6), (3, 9, 0)])
def test_matches_full_system_adjoint(N, nt, ntau):
    t, order = synth.grid(70 + N, nt, 0.02, 0.08, 3, 6)
    kp = synth.kp(70 + N, N, t)
    rd = synth.rdiag(N, nt)
    tv = synth.tv(70 + N, N, ntau, t)
    mat = synth.mat(70 + N, N, ntau)
    G = oracle.Green(kp, rd, tv, mat)
    W = oracle.Weights.build(t, order, 3.0 if ntau else None, ntau, 5)
    flags = oracle.F_IR | oracle.F_IL | (oracle.F_ITV if ntau else 0)
    rng = np.random.default_rng(N)
    for n, m in [(nt - 1, 0), (nt - 1, nt - 1), (nt - 1, nt // 2), (nt // 2, 2), (0, 0)]:
        sig = synth.sigma_row(9 + n, N, n, ntau, t)
        cm = lambda: rng.normal(size=(1, N, N)) + 1j * rng.normal(size=(1, N, N))
        cot = (cm(), cm(), cm(), np.zeros((ntau, N, N), np.complex128))
        gkp, grd, gtv, _, gret, gles, gstv = oracle.collision_vjp(G, sig, W, n, m, m + 1, cot, flags)
        r = oracle.collision_row_vjp(N, ntau, n, m, sig, kp[:m + 1, m], kp[m, :n + 1], rd[m],
                                     tv[m] if ntau else np.zeros((0, N, N)), W.w[n, :n + 1],
                                     W.w[m, :m + 1], W.wfull if ntau else None,
                                     tuple(c[0] for c in cot[:3]), flags)
        g_ret, g_les, g_stv, g_col, g_row, g_rdg, g_tv = r
        tol = lambda x: 1e-13 * (np.abs(x).max() + 1e-300)
        np.testing.assert_allclose(g_ret, gret, atol=tol(gret), rtol=0)
        np.testing.assert_allclose(g_les, gles, atol=tol(gles), rtol=0)
        np.testing.assert_allclose(g_col, gkp[:m + 1, m], atol=tol(gkp), rtol=0)
        want_row = gkp[m, :n + 1].copy()
        want_row[m] = 0  # kp[m][m] is the row's column block, not its row block
        np.testing.assert_allclose(g_row, want_row, atol=tol(gkp), rtol=0)
        np.testing.assert_allclose(g_rdg, grd[m], atol=tol(grd), rtol=0)
        if ntau:
            np.testing.assert_allclose(g_stv, gstv, atol=tol(gstv), rtol=0)
            np.testing.assert_allclose(g_tv, gtv[m], atol=tol(gtv), rtol=0)
        # nothing outside the blocks the row reads
        gkp[:m + 1, m] = 0
        gkp[m, :n + 1] = 0
        assert not gkp.any()
