"""The interacting equilibrium initial state on the GPU (kbe_equilibrium) against the oracle
(oracle/equilibrium.py): element-wise parity of G^M on the same inputs, from one orbital to the
largest orbital count and from a few tau points to the propagation workload's 256; the free
function without interaction; the iteration limit reported as KBE_ECONV with the last iterate;
repeatability; and the property the state exists for: a propagation on the GPU started from it
stays stationary, while one started from the free state does not."""
import numpy as np
import pytest
import torch

import synth
from oracle import equilibrium as eq

pytestmark = pytest.mark.gpu

# both sides stop once the largest change is below 1e-13; with mixing 1/2 the iterates then sit
# within a few 1e-13 of the fixed point, and the two eigensolvers differ in rounding
TOL = 2e-11


def _print(*a):
    print(*a, flush=True)


def chain(N, onsite=None):
    h = synth.tight_binding(N)
    if onsite is not None:
        h = h + np.diag(onsite)
    return h


CASES = [
    # the Hubbard atom at half filling
    dict(h0=np.zeros((1, 1)), u=1.0, mu=0.5, beta=2.0, ntau=33),
    # an asymmetric chain away from half filling, few tau points, site-dependent u
    dict(h0=chain(3, [0.3, -0.1, 0.2]), u=[1.0, 0.7, 1.2], mu=0.4, beta=2.0, ntau=9),
    dict(h0=chain(5, [0.2, 0.0, -0.3, 0.1, 0.0]), u=1.3, mu=0.2, beta=4.0, ntau=65),
    # the largest orbital count; 4 and 12 (the register-tiled convolution covers multiples of 4)
    dict(h0=chain(16), u=0.8, mu=0.4, beta=3.0, ntau=33),
    dict(h0=chain(4, [0.1, 0.0, -0.2, 0.3]), u=1.0, mu=0.6, beta=3.0, ntau=20),
    dict(h0=chain(12), u=[0.5 + 0.05 * i for i in range(12)], mu=0.3, beta=2.5, ntau=17),
    # the smallest tau grids (the two end points; three points)
    dict(h0=chain(2), u=1.0, mu=0.5, beta=1.0, ntau=2),
    dict(h0=chain(6, [0.1] * 6), u=0.9, mu=0.2, beta=2.0, ntau=3),
    # the propagation workload: 8 sites, U = 1, beta = 10, 256 tau points, half filling
    dict(h0=chain(8), u=1.0, mu=0.5, beta=10.0, ntau=256),
]


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"N{c['h0'].shape[0]}_ntau{c['ntau']}")
def test_equilibrium_matches_oracle(gpu, c):
    kbe = gpu
    _print("equilibrium", c["h0"].shape[0], c["ntau"], c["beta"])
    mat, info = kbe.equilibrium(c["h0"], c["u"], c["mu"], c["beta"], c["ntau"])
    G, oinfo = eq.solve(c["h0"], c["u"], c["mu"], c["beta"], c["ntau"])
    _print("  gpu", info, "oracle", oinfo)
    m = mat.cpu().numpy()
    assert info["change"] < 1e-13
    assert abs(info["iterations"] - oinfo["iterations"]) <= 2
    assert np.abs(m.imag).max() == 0
    np.testing.assert_allclose(m.real, G.real, atol=TOL, rtol=0)


def test_no_interaction_is_the_free_function(gpu):
    kbe = gpu
    h0 = chain(6, [0.1, -0.2, 0.0, 0.3, 0.0, -0.1])
    mat, info = kbe.equilibrium(h0, 0.0, 0.3, 5.0, 41)
    # the first iteration re-diagonalises the same matrix from the starting eigenvectors: the
    # free function again, to rounding
    assert info["iterations"] == 1 and info["change"] < 1e-15
    ref = eq.free_matsubara(h0 - 0.3 * np.eye(6), 5.0, 41)
    np.testing.assert_allclose(mat.cpu().numpy().real, ref, atol=1e-14, rtol=0)


def test_iteration_limit_reports_the_last_iterate(gpu):
    kbe = gpu
    h0 = chain(4)
    with pytest.raises(kbe.KBEError) as ex:
        kbe.equilibrium(h0, 1.0, 0.5, 4.0, 33, maxit=3)
    assert ex.value.status == kbe.KBE_ECONV
    mat, info = ex.value.partial
    assert info["iterations"] == 3 and info["change"] >= 1e-13
    G, oinfo = eq.solve(h0, 1.0, 0.5, 4.0, 33, maxit=3)
    assert oinfo["iterations"] == 3
    np.testing.assert_allclose(mat.cpu().numpy().real, G.real, atol=1e-12, rtol=0)


def test_repeatable(gpu):
    kbe = gpu
    h0 = chain(7, [0.1] * 7)
    a, _ = kbe.equilibrium(h0, 1.1, 0.3, 6.0, 100)
    b, _ = kbe.equilibrium(h0, 1.1, 0.3, 6.0, 100)
    assert torch.equal(a, b)


def test_propagation_from_the_equilibrium_is_stationary(gpu):
    """Adaptive propagation without a pulse: the equal-time density matrix G^<(t,t) stays at its
    initial value from the equilibrium, and moves away from the free state's."""
    kbe = gpu
    N, U, beta, ntau = 4, 1.0, 4.0, 64
    h0 = chain(N, [0.2, -0.1, 0.0, 0.1])
    mu = 0.4
    mat, _ = kbe.equilibrium(h0, U, mu, beta, ntau)
    free = torch.as_tensor(eq.free_matsubara(h0 - mu * np.eye(N), beta, ntau).astype(np.complex128))

    def drift(m):
        r = kbe.propagate_adaptive(h0, U, 0.0, 4.0, ntau=ntau, beta=beta, mat=m, capacity=1024,
                                   rtol=1e-8, atol=1e-10, kmax=10)
        n = len(r["t"])
        d = torch.diagonal(r["G"].kp[:n, :n], dim1=0, dim2=1).permute(2, 0, 1)  # G^<(t_n,t_n)
        return n - 1, float((d - d[0]).abs().max())

    steps_eq, d_eq = drift(mat)
    steps_free, d_free = drift(free.to(mat.device))
    _print("  equilibrium: %d steps, drift %.2e; free: %d steps, drift %.2e"
           % (steps_eq, d_eq, steps_free, d_free))
    assert d_eq < 1e-6
    assert d_free > 1e-3


def test_strong_coupling_does_not_converge(gpu):
    """At U = 20 the mixed iteration does not settle (the oracle's change is still 0.7 after 40
    iterations): KBE_ECONV, with a finite last iterate and its change."""
    kbe = gpu
    with pytest.raises(kbe.KBEError) as ex:
        kbe.equilibrium(chain(4), 20.0, 10.0, 4.0, 33, maxit=40)
    assert ex.value.status == kbe.KBE_ECONV
    mat, info = ex.value.partial
    assert info["iterations"] == 40 and info["change"] > 1e-3
    assert torch.isfinite(mat.real).all()
