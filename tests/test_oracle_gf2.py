"""Pins for the oracle's second-Born self-energy with a general four-index interaction (Eq. SE).

Each pin is fixed independently of the order in which the oracle's einsum contracts the indices:
  * a six-fold loop over the indices, written out in plain Python (tiny N, general U);
  * the same six-fold loop in plain C (oracle.c, orc_gf2_block) at 8 and 16 orbitals, the sizes
    the GPU kernels run, general U and an eight-fold symmetric one;
  * a rank-one U, for which the sum collapses to products of bilinear forms (closed form);
  * a local U, where Eq. SE reduces to the local second-Born formula of the C oracle, which has
    its own pins (hand calculation, brute force);
  * the anti-Hermitian symmetry Sigma^<>(t,t')^dagger = -Sigma^<>(t',t) inherited from G for a
    real U with the eight-fold symmetry of two-electron integrals in chemists' notation;
  * exact quadratic scaling in U (powers of two).
"""
import itertools

import numpy as np
import pytest

import oracle
from tests.helpers import pack_kp, random_symmetric_full


def _cmat(rng, N):
    return rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))


def _loops(U, A, C):
    """Eq. SE as six nested sums per (i, j), with Uex_jabc = 2 U_jbac - U_jabc written inline."""
    N = A.shape[0]
    out = np.zeros((N, N), np.complex128)
    for i, j in itertools.product(range(N), repeat=2):
        acc = 0j
        for f, d, e, a, b, c in itertools.product(range(N), repeat=6):
            ex = 2.0 * U[j, b, a, c] - U[j, a, b, c]
            acc += U[i, f, d, e] * ex * A[f, b] * A[e, a] * C[c, d]
        out[i, j] = acc
    return out


def sym8(rng, N):
    """A real U with (ij|kl) = (ji|kl) = (ij|lk) = (kl|ij) and the products of these."""
    U0 = rng.normal(size=(N,) * 4)
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
             (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    return sum(np.transpose(U0, p) for p in perms) / 8


@pytest.mark.parametrize("N", [1, 2, 3])
def test_matches_six_fold_loops(N):
    rng = np.random.default_rng(100 + N)
    U = rng.normal(size=(N,) * 4)          # no symmetry at all
    A, C = _cmat(rng, N), _cmat(rng, N)
    np.testing.assert_allclose(oracle.gf2_block(U, A, C), _loops(U, A, C), rtol=1e-13,
                               atol=1e-13 * np.abs(_loops(U, A, C)).max())


@pytest.mark.parametrize("N,sym", [(8, False), (16, False), (16, True)])
def test_matches_six_fold_loops_in_c(N, sym):
    """At full size: each entry within 1e-13 of its rounding scale, the six-fold sum of the
    magnitudes of its terms."""
    rng = np.random.default_rng(150 + N + sym)
    U = sym8(rng, N) if sym else rng.normal(size=(N,) * 4)
    A, C = _cmat(rng, N), _cmat(rng, N)
    got = oracle.gf2_block(U, A, C)
    ref = oracle.gf2_block_loops(U, A, C)
    scale = np.einsum("ifde,jabc,fb,ea,cd->ij", np.abs(U), np.abs(oracle.uex(U)), np.abs(A),
                      np.abs(A), np.abs(C), optimize="optimal")
    assert np.all(np.abs(got - ref) <= 1e-13 * scale)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_c_loops_match_python_loops():
    """The C six-fold loop against the Python one (tiny N, general U): the same sum written twice,
    so a transposed index in either shows."""
    rng = np.random.default_rng(160)
    U = rng.normal(size=(3,) * 4)
    A, C = _cmat(rng, 3), _cmat(rng, 3)
    ref = _loops(U, A, C)
    np.testing.assert_allclose(oracle.gf2_block_loops(U, A, C), ref, rtol=1e-13,
                               atol=1e-13 * np.abs(ref).max())


def test_uex_definition():
    rng = np.random.default_rng(7)
    U = rng.normal(size=(3,) * 4)
    X = oracle.uex(U)
    for j, a, b, c in itertools.product(range(3), repeat=4):
        assert X[j, a, b, c] == 2.0 * U[j, b, a, c] - U[j, a, b, c]


@pytest.mark.parametrize("N", [2, 5, 16])
def test_rank_one_closed_form(N):
    """U_ifde = x_i y_f z_d w_e: Uex_jabc = x_j (2 y_b z_a - y_a z_b) w_c and
    Sigma_ij = x_i x_j (wCz) [2 (y^T A y)(w^T A z) - (y^T A z)(w^T A y)]."""
    rng = np.random.default_rng(200 + N)
    x, y, z, w = (rng.normal(size=N) for _ in range(4))
    U = np.einsum("i,f,d,e->ifde", x, y, z, w)
    A, C = _cmat(rng, N), _cmat(rng, N)
    q = lambda u, M, v: u @ M @ v
    ref = np.outer(x, x) * q(w, C, z) * (2 * q(y, A, y) * q(w, A, z) - q(y, A, z) * q(w, A, y))
    np.testing.assert_allclose(oracle.gf2_block(U, A, C), ref, rtol=1e-12,
                               atol=1e-12 * np.abs(ref).max())


def _green(rng, N, nt, ntau):
    les, gtr = random_symmetric_full(rng, N, nt)
    ret = gtr - les
    kp = pack_kp(les, ret)
    rdiag = np.array([ret[a, a] for a in range(nt)])
    tv = (rng.normal(size=(nt, ntau, N, N)) + 1j * rng.normal(size=(nt, ntau, N, N))
          if ntau else None)
    return oracle.Green(kp, rdiag, tv), les, gtr


@pytest.mark.parametrize("N", [1, 2, 3])
def test_local_u_reduces_to_local_second_born(N):
    rng = np.random.default_rng(300 + N)
    nt, ntau = 5, 6
    G, _, _ = _green(rng, N, nt, ntau)
    u = rng.uniform(0.5, 2.0, size=N)
    U = np.zeros((N,) * 4)
    for i in range(N):
        U[i, i, i, i] = u[i]
    for n in (0, 2, nt - 1):
        got = oracle.sigma_gf2_row(G, U, n)
        want = oracle.sigma_row(G, u, n)
        for g, r in zip(got, want):
            np.testing.assert_allclose(g, r, rtol=1e-13, atol=1e-13 * (np.abs(r).max() + 1e-300))


def test_blocks_are_read_through_the_storage_symmetries():
    """les_block / gtr_block give back the full G^< and G^> the storage was packed from."""
    rng = np.random.default_rng(8)
    G, les, gtr = _green(rng, 2, 5, 0)
    for a, b in itertools.product(range(5), repeat=2):
        np.testing.assert_allclose(oracle.les_block(G, a, b), les[a, b], rtol=0, atol=1e-15)
        np.testing.assert_allclose(oracle.gtr_block(G, a, b), gtr[a, b], rtol=0, atol=1e-14)


@pytest.mark.parametrize("N", [2, 3, 4])
def test_symmetry_inherited_for_eightfold_u(N):
    rng = np.random.default_rng(400 + N)
    nt = 5
    _, les, gtr = _green(rng, N, nt, 0)
    U = sym8(rng, N)
    for a, b in itertools.product(range(nt), repeat=2):
        for A_ab, C_ba, A_ba, C_ab in ((les[a, b], gtr[b, a], les[b, a], gtr[a, b]),
                                       (gtr[a, b], les[b, a], gtr[b, a], les[a, b])):
            s_ab = oracle.gf2_block(U, A_ab, C_ba)
            s_ba = oracle.gf2_block(U, A_ba, C_ab)
            np.testing.assert_allclose(s_ab.conj().T, -s_ba, rtol=1e-12,
                                       atol=1e-12 * np.abs(s_ab).max())


def test_quadratic_in_u_exactly():
    rng = np.random.default_rng(9)
    G, _, _ = _green(rng, 3, 4, 4)
    U = rng.normal(size=(3,) * 4)
    for x, y in zip(oracle.sigma_gf2_row(G, U, 3), oracle.sigma_gf2_row(G, 2.0 * U, 3)):
        assert np.array_equal(4.0 * x, y)
