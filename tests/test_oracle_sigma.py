"""Pins for the oracle's second-Born self-energy (Eq. SE with a local interaction)."""
import json
import os

import numpy as np
import pytest

import oracle
from tests.helpers import pack_kp, random_symmetric_full

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _green_from_full(les, gtr, tv=None):
    ret = gtr - les
    kp = pack_kp(les, ret)
    nt = les.shape[0]
    rdiag = np.array([ret[a, a] for a in range(nt)])
    return oracle.Green(kp, rdiag, tv)


def brute_force_se(les_ab, gtr_ab, les_ba, gtr_ba, U4):
    """Eq. SE with a general four-index U: Sigma^<>_ij = U_ifde U^Ex_jabc G^<>_fb G^<>_ea G^><_cd."""
    UEx = 2 * np.transpose(U4, (0, 2, 1, 3)) - U4  # U^Ex_jabc = 2 U_jbac - U_jabc
    s_les = np.einsum("ifde,jabc,fb,ea,cd->ij", U4, UEx, les_ab, les_ab, gtr_ba)
    s_gtr = np.einsum("ifde,jabc,fb,ea,cd->ij", U4, UEx, gtr_ab, gtr_ab, les_ba)
    return s_les, s_gtr


def local_u4(u):
    N = len(u)
    U4 = np.zeros((N, N, N, N))
    for i in range(N):
        U4[i, i, i, i] = u[i]
    return U4


@pytest.mark.parametrize("N", [1, 2, 3])
def test_local_reduction_matches_general_formula(N):
    rng = np.random.default_rng(10 + N)
    nt = 5
    les, gtr = random_symmetric_full(rng, N, nt)
    G = _green_from_full(les, gtr)
    u = rng.uniform(0.5, 2.0, size=N)
    U4 = local_u4(u)
    for a in range(nt):
        for b in range(nt):
            s_les, s_gtr = oracle.sigma_pair(G, u, a, b)
            r_les, r_gtr = brute_force_se(les[a, b], gtr[a, b], les[b, a], gtr[b, a], U4)
            np.testing.assert_allclose(s_les, r_les, rtol=1e-13, atol=1e-13)
            np.testing.assert_allclose(s_gtr, r_gtr, rtol=1e-13, atol=1e-13)


def test_mixed_component_matches_general_formula():
    rng = np.random.default_rng(5)
    N, nt, ntau = 3, 4, 7
    les, gtr = random_symmetric_full(rng, N, nt)
    tv = rng.normal(size=(nt, ntau, N, N)) + 1j * rng.normal(size=(nt, ntau, N, N))
    G = _green_from_full(les, gtr, tv)
    u = rng.uniform(0.5, 2.0, size=N)
    UEx = 2 * np.transpose(local_u4(u), (0, 2, 1, 3)) - local_u4(u)
    n = nt - 1
    _, _, stv = oracle.sigma_row(G, u, n)
    J = ntau - 1
    for l in range(ntau):
        gmix = tv[n, l]
        gbar = tv[n, J - l].conj().T  # G^[(tau_l, t) = G^](t, beta - tau_l)^dagger
        ref = np.einsum("ifde,jabc,fb,ea,cd->ij", local_u4(u), UEx, gmix, gmix, gbar)
        np.testing.assert_allclose(stv[l], ref, rtol=1e-13, atol=1e-13)


def test_symmetry_inherited():
    rng = np.random.default_rng(3)
    N, nt = 3, 6
    les, gtr = random_symmetric_full(rng, N, nt)
    G = _green_from_full(les, gtr)
    u = rng.uniform(0.5, 2.0, size=N)
    for a in range(nt):
        for b in range(nt):
            l_ab, g_ab = oracle.sigma_pair(G, u, a, b)
            l_ba, g_ba = oracle.sigma_pair(G, u, b, a)
            np.testing.assert_allclose(l_ab.conj().T, -l_ba, rtol=1e-13, atol=1e-13)
            np.testing.assert_allclose(g_ab.conj().T, -g_ba, rtol=1e-13, atol=1e-13)


def test_quadratic_in_u_exactly():
    rng = np.random.default_rng(4)
    N, nt, ntau = 2, 5, 5
    les, gtr = random_symmetric_full(rng, N, nt)
    tv = rng.normal(size=(nt, ntau, N, N)) + 1j * rng.normal(size=(nt, ntau, N, N))
    G = _green_from_full(les, gtr, tv)
    u = rng.uniform(0.5, 2.0, size=N)
    r1 = oracle.sigma_row(G, u, nt - 1)
    r2 = oracle.sigma_row(G, 2 * u, nt - 1)
    for x, y in zip(r1, r2):
        assert np.array_equal(4 * x, y)  # powers of two: exact in floating point


def test_row_mode_consistent_with_pairs():
    rng = np.random.default_rng(6)
    N, nt = 2, 6
    les, gtr = random_symmetric_full(rng, N, nt)
    G = _green_from_full(les, gtr)
    u = np.array([1.0, 0.6])
    n = 4
    ret, les_row, _ = oracle.sigma_row(G, u, n)
    for s in range(n + 1):
        l, g = oracle.sigma_pair(G, u, n, s)
        np.testing.assert_array_equal(les_row[s], l)
        np.testing.assert_array_equal(ret[s], g - l)


def test_hand_calculation_one_orbital():
    fx = json.load(open(os.path.join(GOLDEN, "sigma_2b_N1_hand.json")))
    kp = np.zeros((2, 2, 1, 1), np.complex128)
    for key, (re, im) in fx["kp"].items():
        kp[int(key[0]), int(key[1]), 0, 0] = re + 1j * im
    rdiag = np.full((2, 1, 1), complex(*fx["rdiag"]))
    G = oracle.Green(kp, rdiag)
    u = np.array([fx["u"]])
    les, gtr = oracle.sigma_pair(G, u, 1, 0)
    ret, _, _ = oracle.sigma_row(G, u, 1)
    e = fx["expected"]
    assert abs(les[0, 0] - complex(*e["sigma_les_10"])) < 1e-14
    assert abs(gtr[0, 0] - complex(*e["sigma_gtr_10"])) < 1e-14
    assert abs(ret[0, 0, 0] - complex(*e["sigma_ret_10"])) < 1e-14


def test_full_mode_agrees_with_rows_and_symmetry():
    """oracle.sigma_full against the pinned row function at every row (lower triangle, rdiag, tv)
    and, above the diagonal, against the inherited symmetry Sigma^<(t,t') = -Sigma^<(t',t)^dagger
    of the row values (which holds for inputs with G's symmetry)."""
    rng = np.random.default_rng(21)
    N, nt, ntau = 2, 6, 4
    les, gtr = random_symmetric_full(rng, N, nt)
    tv = rng.normal(size=(nt, ntau, N, N)) + 1j * rng.normal(size=(nt, ntau, N, N))
    G = _green_from_full(les, gtr, tv)
    u = np.array([0.8, 1.3])
    kp, rd, stv = oracle.sigma_full(G, u)
    for n in range(nt):
        ret, les_row, tv_row = oracle.sigma_row(G, u, n)
        for s in range(n):
            np.testing.assert_array_equal(kp[n, s], ret[s])
            np.testing.assert_allclose(kp[s, n], -les_row[s].conj().T, rtol=1e-13, atol=1e-13)
        np.testing.assert_array_equal(kp[n, n], les_row[n])
        np.testing.assert_array_equal(rd[n], ret[n])
        np.testing.assert_array_equal(stv[n], tv_row)
