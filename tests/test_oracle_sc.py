"""Pins of the oracle's determinant algebra against brute force, closed forms
and LAPACK special cases (no GPU)."""
import math

import numpy as np
import pytest

import synth_inputs
from oracle import cd as ocd
from oracle import fci


def random_integrals(N, seed, naux=None):
    naux = naux or 3 * N
    return synth_inputs.ab_initio(N, naux, seed)


@pytest.mark.parametrize("N,na,nb", [(3, 1, 1), (4, 2, 1), (4, 2, 2), (5, 2, 2)])
def test_slater_condon_matches_second_quantization(N, na, nb):
    """Every entry of eq. (entry) equals <I|H|J> from applying each term of
    eq. (general-ham) with Jordan-Wigner signs (brute force)."""
    h, eri = random_integrals(N, 11 + N + na)
    Hsc, B1 = fci.dense_H(h, eri, N, na, nb)
    Hbf, B2 = fci.dense_H_second_quantized(h, eri, N, na, nb)
    assert B1 == B2
    np.testing.assert_allclose(Hsc, Hbf, rtol=0, atol=1e-13)


def test_planted_sign_error_is_caught():
    """A flipped exchange sign in the double element breaks the brute-force pin
    (guards the pin itself)."""
    N, na, nb = 4, 2, 2
    h, eri = random_integrals(N, 5)
    Hbf, _ = fci.dense_H_second_quantized(h, eri, N, na, nb)
    orig = fci.double_element

    def wrong(eri_, N_, x, p, q, r, s):
        sign, y = fci.apply_ops(x, [("c", r), ("c", s), ("a", q), ("a", p)])
        if sign == 0:
            return None, 0.0
        return y, sign * (fci.vphys(eri_, N_, r, s, p, q) + fci.vphys(eri_, N_, r, s, q, p))

    fci.double_element = wrong
    try:
        Hw, _ = fci.dense_H(h, eri, N, na, nb)
    finally:
        fci.double_element = orig
    assert np.max(np.abs(Hw - Hbf)) > 1e-3


@pytest.mark.parametrize("N,na,nb", [(6, 3, 3), (7, 3, 2)])
def test_hermitian_and_conserving(N, na, nb):
    h, eri = random_integrals(N, 3 + N)
    H, B = fci.dense_H(h, eri, N, na, nb)
    assert len(B) == math.comb(N, na) * math.comb(N, nb)
    np.testing.assert_array_equal(H, H.T)
    for a, b in B[:20]:
        for (a2, b2), _ in fci.column(h, eri, N, a, b):
            assert bin(a2).count("1") == na and bin(b2).count("1") == nb


@pytest.mark.parametrize("N,na,nb", [(6, 3, 3), (8, 3, 2), (12, 4, 4), (24, 6, 6)])
def test_column_size_closed_form(N, na, nb):
    h, eri = random_integrals(N, 1, naux=4)
    a, b = ocd.aufbau(h, na, nb)
    ka, kb, v = ocd.column(h, eri, a, b)
    assert len(ka) == fci.column_size(N, na, nb)
    assert len(set(zip(ka.tolist(), kb.tolist()))) == len(ka)
    if N <= 12:
        assert len(fci.column(h, eri, N, a, b)) == len(ka)


def test_column_size_survey_numbers():
    # counts for the two synthetic ab initio workloads (24 and 36 orbitals)
    assert fci.column_size(24, 6, 6) == 16471
    assert fci.column_size(36, 8, 8) == 71793


@pytest.mark.parametrize("N,na,nb,seed", [(8, 3, 3, 0), (10, 4, 3, 1), (12, 5, 5, 2)])
def test_cpp_column_matches_python(N, na, nb, seed):
    h, eri = random_integrals(N, seed)
    a_s, b_s = synth_inputs.random_dets(N, na, nb, 3, seed)
    for a, b in zip(a_s.tolist(), b_s.tolist()):
        py = {k: v for k, v in fci.column(h, eri, N, a, b)}
        ka, kb, v = ocd.column(h, eri, a, b)
        cp = {(int(x), int(y)): float(z) for x, y, z in zip(ka, kb, v)}
        assert set(py) == set(cp)
        for k in py:
            assert abs(py[k] - cp[k]) <= 1e-13, k


def test_two_site_hubbard_closed_form():
    for U in (0.5, 4.0, 10.0):
        h, eri = fci.hubbard_integrals((2,), 1.0, U)
        E0, _, _ = fci.ground_state_dense(h, eri, 2, 1, 1)
        assert abs(E0 - (U - math.sqrt(U * U + 16.0)) / 2.0) < 1e-13


def _free_fermion(dims, t, na, nb):
    eps = [0.0]
    for L in dims:
        if L == 2:
            lv = [-t, t]
        else:
            lv = [-2 * t * math.cos(2 * math.pi * m / L) for m in range(L)]
        eps = [e + x for e in eps for x in lv]
    eps.sort()
    return sum(eps[:na]) + sum(eps[:nb])


@pytest.mark.parametrize("dims,na,nb", [((6,), 3, 3), ((2, 3), 3, 2), ((2, 4), 2, 2)])
def test_free_fermions(dims, na, nb):
    h, eri = fci.hubbard_integrals(dims, 1.0, 0.0)
    L = int(np.prod(dims))
    E0, _, _ = fci.ground_state_dense(h, eri, L, na, nb)
    assert abs(E0 - _free_fermion(dims, 1.0, na, nb)) < 1e-12


def test_no_interaction_equals_orbital_sum():
    N, na, nb = 7, 3, 2
    h, _ = random_integrals(N, 9)
    eri = np.zeros((N,) * 4)
    E0, _, _ = fci.ground_state_dense(h, eri, N, na, nb)
    w = np.linalg.eigvalsh(h)
    assert abs(E0 - (w[:na].sum() + w[:nb].sum())) < 1e-12


def test_atomic_limit():
    for dims, na, nb in (((6,), 3, 3), ((2, 3), 4, 3)):
        L = int(np.prod(dims))
        h, eri = fci.hubbard_integrals(dims, 0.0, 3.0)
        E0, _, _ = fci.ground_state_dense(h, eri, L, na, nb)
        assert abs(E0 - 3.0 * max(0, na + nb - L)) < 1e-13


def test_4x4_levels_from_paper():
    rows = [l.split() for l in open("tests/golden/hubbard_4x4_levels.txt") if not l.startswith("#")]
    neg, zero, pos, deg = map(int, rows[0])
    h, _ = fci.hubbard_integrals((4, 4), 1.0, 0.0)
    w = np.linalg.eigvalsh(h)
    assert (np.sum(w < -1e-12), np.sum(abs(w) <= 1e-12), np.sum(w > 1e-12)) == (neg, zero, pos)
    assert math.comb(zero, 3) ** 2 == deg
    # U = 0 half filling: -24 (sum of the 8 lowest levels, twice)
    assert abs(2 * np.sort(w)[:8].sum() + 24.0) < 1e-12


def test_lanczos_matches_dense():
    h, eri = fci.hubbard_integrals((8,), 1.0, 4.0)
    E_dense, _, _ = fci.ground_state_dense(h, eri, 8, 4, 4)
    E_lan, _, _ = fci.ground_state_lanczos(h, eri, 8, 4, 4)
    assert abs(E_dense - E_lan) < 1e-10
