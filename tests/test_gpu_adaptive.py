"""The adaptive propagation on the GPU (kbe_propagate_adaptive) against the oracle
(oracle/adaptive.py): the controller's decisions (grid, Adams orders, iteration counts, history
orders) against the oracle's own run, the solution against the oracle replaying the GPU's
decisions on the same grid, tolerance proportionality against a closed form, and the
Hubbard-chain workload's shape (8 sites, U = 1, beta = 10, 256 tau points, pulse on site 0) over a
shortened run with conservation and the oracle on the first steps."""
import numpy as np
import pytest
import torch
from scipy.special import erf

import synth
from oracle import adaptive as ad
from oracle import equilibrium as oeq
from oracle import propagate as op

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def problem(N, ntau, beta, rho0=None):
    h0 = synth.tight_binding(N)
    mat, rho = synth.free_thermal(h0, beta, ntau)
    P = op.Problem(t=np.zeros(1), order=np.zeros(1, np.int32), h0=h0, ntau=ntau, beta=beta,
                   mat=mat, rho0=(rho if rho0 is None else rho0) if not ntau else None)
    return h0, mat, P


def run_gpu(kbe, P, U, A, **kw):
    return kbe.propagate_adaptive(P.h0, U, A, kw.pop("t_end"), ntau=P.ntau, beta=P.beta,
                                  mat=P.mat, rho0=P.rho0, **kw)


CASES = [dict(N=2, ntau=6, beta=2.0, U=1.0, A=0.7, t_end=0.8, rtol=1e-5, atol=1e-8),
         dict(N=3, ntau=0, beta=2.0, U=1.5, A=0.5, t_end=0.6, rtol=1e-6, atol=1e-9),
         dict(N=4, ntau=5, beta=1.0, U=0.8, A=1.0, t_end=0.5, rtol=1e-4, atol=1e-7),
         # low orders and at most one fixed-point correction per step (rejections by the
         # convergence test as well as by the error test)
         dict(N=3, ntau=4, beta=1.5, U=1.2, A=0.9, t_end=0.5, rtol=1e-4, atol=1e-7, qmax=3,
              kmax=4, maxcor=1)]


@pytest.mark.parametrize("case", CASES,
                         ids=lambda c: f"N{c['N']}_ntau{c['ntau']}" + ("_q3k4m1" if "qmax" in c else ""))
def test_adaptive_matches_oracle(gpu, case):
    kbe = gpu
    c = dict(case)
    N, ntau, beta, U, A = c.pop("N"), c.pop("ntau"), c.pop("beta"), c.pop("U"), c.pop("A")
    h0, mat, P = problem(N, ntau, beta)
    _print("adaptive", N, ntau, c)
    g = run_gpu(kbe, P, U, A, capacity=512, **c)
    _print("  gpu: %d steps, %d rejected, orders %s" % (len(g["t"]) - 1, g["rejected"],
                                                         np.bincount(g["q"][1:])))
    ctl = ad.Controls(t_end=c["t_end"], rtol=c["rtol"], atol=c["atol"], nt_max=512,
                      qmax=c.get("qmax", 12), kmax=c.get("kmax", 10), maxcor=c.get("maxcor", 3))
    orc = ad.Adaptive(P, ctl)
    d_own = orc.run(U, A).numpy()
    own = orc.trace
    _print("  oracle: %d steps, %d rejected" % (len(own), orc.rejected))
    # the decisions: the same integer choices (steps, rejections, orders, iteration counts,
    # history orders); the step sizes are continuous functions of the error norms, which the two
    # sides round differently (~1e-13 relative, raised to 1/(q+1) and carried from step to step),
    # so the grids agree to that: 1e-8
    assert len(own) == len(g["t"]) - 1
    assert g["rejected"] == orc.rejected
    np.testing.assert_allclose(g["t"][1:], [x["t"] for x in own], rtol=1e-8, atol=0)
    assert list(g["q"][1:]) == [x["q"] for x in own]
    assert list(g["m"][1:]) == [x["m"] for x in own]
    assert g["ks"] == [x["ks"] for x in own]
    # the solution: the oracle replaying the GPU's decisions on the GPU's grid
    rep = ad.Adaptive(P, ctl)
    d = rep.run(U, A, replay=g["replay"]).numpy()
    kp_ref, tv_ref = rep.storage()
    nt = len(g["t"])
    kp = g["G"].kp[:nt, :nt].cpu().numpy()
    err = np.linalg.norm(kp - kp_ref) / np.linalg.norm(kp_ref)
    _print("  kp relative error %.3e" % err)
    assert err < 1e-12
    if ntau:
        tv = g["G"].tv[:nt].cpu().numpy()
        assert np.linalg.norm(tv - tv_ref) < 1e-12 * np.linalg.norm(tv_ref)
    dg = g["dens"].cpu().numpy()
    assert np.abs(dg - d).max() < 1e-12
    # on the oracle's own grid (shifted by up to 1e-8 relative) the densities move by |dn/dt| dt
    assert np.abs(d - d_own).max() < 1e-8
    tr = dg.sum(axis=1)
    assert np.abs(tr - tr[0]).max() < 1e-13 * max(1.0, abs(tr[0]))


def test_adaptive_tolerance_proportionality(gpu):
    """A single orbital with the pulse alone: G^<(t_m, t_end) = i rho exp(i(phi(t_end) - phi(t_m)))
    with phi the integral of h(t) (an erf); the error falls with rtol (atol = rtol / 1000)."""
    kbe = gpu
    h0, A, rho, T_end = 0.3, 0.8, 0.6, 4.0
    errs, steps = [], []
    for rtol in (1e-4, 1e-6, 1e-8):
        g = kbe.propagate_adaptive(np.array([[h0]]), 0.0, A, T_end, rho0=np.array([[rho]]),
                                   capacity=2048, rtol=rtol, atol=rtol * 1e-3)
        t = g["t"]
        s2 = np.sqrt(2.0)
        phi = h0 * t + A * np.sqrt(np.pi / 2) * (erf((t - 2.0) / s2) - erf(-2.0 / s2))
        exact = 1j * rho * np.exp(1j * (phi[-1] - phi))
        kp = g["G"].kp[: len(t), len(t) - 1, 0, 0].cpu().numpy()
        errs.append(np.abs(kp - exact).max())
        steps.append(len(t))
        _print("rtol %g: %d steps, error %.3e" % (rtol, len(t), errs[-1]))
    assert steps[0] < steps[1] < steps[2]
    assert errs[0] > errs[1] > errs[2]
    for e, rtol in zip(errs, (1e-4, 1e-6, 1e-8)):
        assert e < 100 * rtol


def test_adaptive_hubbard_workload_short(gpu):
    """The adaptive workload's shape over a shortened run: 8-site chain, U = 1, beta = 10, 256 tau
    points, the interacting equilibrium at half filling as the initial state, pulse on site 0,
    rtol 1e-6: finite, conserving, the order and the steps varying, and the first 6 steps against
    the oracle replaying them."""
    kbe = gpu
    N, ntau, beta, U, A = 8, 256, 10.0, 1.0, 1.0
    h0, _, P = problem(N, ntau, beta)
    P.mat, _ = oeq.solve(h0, U, U / 2, beta, ntau)
    g = run_gpu(kbe, P, U, A, capacity=1024, t_end=3.0, rtol=1e-6, atol=1e-10)
    d = g["dens"].cpu().numpy()
    t = g["t"]
    _print("hubbard short: %d steps, %d rejected, h from %.2e to %.2e, orders %s" % (
        len(t) - 1, g["rejected"], np.diff(t).min(), np.diff(t).max(), np.bincount(g["q"][1:])))
    assert np.all(np.isfinite(d))
    tr = d.sum(axis=1)
    assert np.abs(tr - tr[0]).max() < 1e-12 * tr[0]
    assert len(set(g["q"][1:])) >= 3 and np.diff(t).max() > 10 * np.diff(t).min()
    rep = ad.Adaptive(P, ad.Controls(t_end=3.0, rtol=1e-6, atol=1e-10, nt_max=16))
    rep.run(U, A, replay=g["replay"][:7])
    kp_ref, tv_ref = rep.storage()
    kp = g["G"].kp[:7, :7].cpu().numpy()
    assert np.linalg.norm(kp - kp_ref) < 1e-12 * np.linalg.norm(kp_ref)
    assert np.linalg.norm(g["G"].tv[:7].cpu().numpy() - tv_ref) < 1e-12 * np.linalg.norm(tv_ref)


def test_adaptive_capacity_exhausted(gpu):
    """A grid that runs out of points before t_end: KBE_ESTEP with the accepted steps, which are
    those of a run with room to spare (the same decisions, the same solution bit for bit)."""
    kbe = gpu
    h0, mat, P = problem(2, 6, 2.0)
    full = run_gpu(kbe, P, 1.0, 0.7, capacity=512, t_end=0.8, rtol=1e-5, atol=1e-8)
    cap = 12
    assert len(full["t"]) > cap
    with pytest.raises(kbe.KBEError, match="KBE_ESTEP") as ex:
        run_gpu(kbe, P, 1.0, 0.7, capacity=cap, t_end=0.8, rtol=1e-5, atol=1e-8)
    part = ex.value.partial
    assert ex.value.status == kbe.KBE_ESTEP and part is not None
    assert len(part["t"]) == cap
    assert np.array_equal(part["t"], full["t"][:cap])
    assert np.array_equal(part["q"], full["q"][:cap]) and part["ks"] == full["ks"][:cap - 1]
    kp_p = part["G"].kp[:cap, :cap].cpu().numpy()
    kp_f = full["G"].kp[:cap, :cap].cpu().numpy()
    assert np.array_equal(kp_p, kp_f)
    assert np.array_equal(part["dens"].cpu().numpy(), full["dens"][:cap].cpu().numpy())


def test_adaptive_rejects_bad_controls(gpu):
    """Argument errors are reported before any launch."""
    kbe = gpu
    h0, mat, P = problem(2, 0, 2.0)
    for bad in (dict(qmax=13), dict(kmax=1), dict(maxcor=0), dict(rtol=0.0), dict(h_first=-1.0)):
        with pytest.raises(kbe.KBEError, match="KBE_EINVAL"):
            run_gpu(kbe, P, 1.0, 0.7, capacity=16, t_end=0.5, **bad)


def test_adaptive_converges_to_a_fine_fixed_grid(gpu):
    """An interacting system (4-site chain, U = 1, pulse) without the oracle: the adaptive
    densities at t_end approach those of the fixed-grid propagation (a separate propagator, on a
    uniform grid of 1500 steps with sixth-order rules and five fixed-point iterations, whose own
    error is far below the tolerances) as the tolerance tightens."""
    kbe = gpu
    N, U, A, T = 4, 1.0, 0.8, 3.0
    h0 = synth.tight_binding(N)
    _, rho = synth.free_thermal(h0, 2.0, 0)
    nt = 1501
    t = np.linspace(0.0, T, nt)
    order = np.full(nt, 6, np.int32)
    ref = kbe.Propagation(t, order, h0, ntau=0, rho0=rho, iters=5)
    d_ref = ref.run(torch.full((N,), U, dtype=torch.float64, device="cuda:0"), A).cpu().numpy()[-1]
    errs = []
    for rtol in (1e-5, 1e-7, 1e-9):
        g = kbe.propagate_adaptive(h0, U, A, T, rho0=rho, capacity=2048, rtol=rtol,
                                   atol=rtol * 1e-3)
        d = g["dens"].cpu().numpy()[-1]
        errs.append(np.abs(d - d_ref).max())
        _print("rtol %g: %d steps, |n(T) - n_ref(T)| = %.2e" % (rtol, len(g["t"]) - 1, errs[-1]))
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] < 1e-3 and errs[2] < 1e-7
