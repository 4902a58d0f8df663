"""Pins of the oracle's reduced density matrices and orbital gradient (no GPU)."""
import numpy as np
import pytest
import scipy.linalg

import synth_inputs
from oracle import fci


@pytest.fixture(scope="module")
def system():
    N, na, nb = 5, 2, 2
    h, eri = synth_inputs.ab_initio(N, 15, 21)
    E0, v0, B = fci.ground_state_dense(h, eri, N, na, nb)
    g1, g2 = fci.rdm12(B, v0, N)
    return N, na, nb, h, eri, E0, v0, B, g1, g2


def test_rdm_invariants(system):
    N, na, nb, h, eri, E0, v0, B, g1, g2 = system
    n = na + nb
    assert abs(np.trace(g1) - n) < 1e-12
    assert abs(np.einsum("pprr->", g2) - n * (n - 1)) < 1e-11
    np.testing.assert_allclose(g1, g1.T, atol=1e-13)
    np.testing.assert_allclose(g2, g2.transpose(2, 3, 0, 1), atol=1e-13)
    np.testing.assert_allclose(g2, g2.transpose(1, 0, 3, 2), atol=1e-13)
    w = np.linalg.eigvalsh(g1)
    assert w.min() > -1e-12 and w.max() < 2 + 1e-12
    # partial trace: sum_r Gamma_pqrr = (n - 1) gamma_pq
    np.testing.assert_allclose(np.einsum("pqrr->pq", g2), (n - 1) * g1, atol=1e-11)


def test_rdm_energy_is_rayleigh_quotient(system):
    N, na, nb, h, eri, E0, v0, B, g1, g2 = system
    assert abs(fci.energy_from_rdms(h, eri, g1, g2) - E0) < 1e-11
    # also for a non-eigenvector (random sparse vector)
    rng = np.random.default_rng(4)
    c = rng.normal(size=len(B)) * (rng.random(len(B)) < 0.5)
    H, _ = fci.dense_H(h, eri, N, na, nb)
    G1, G2 = fci.rdm12(B, c, N)
    assert abs(fci.energy_from_rdms(h, eri, G1, G2) - c @ H @ c / (c @ c)) < 1e-11


def _images(p, q, r, s):
    return {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
            (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}


def test_rdm_gradient_by_finite_difference(system):
    """E(c fixed) is linear in (h, eri), so central differences are exact up to
    rounding: dE/dh_pq = gamma_pq, and for a perturbation of all eight images of
    (pq|rs) together dE = 1/2 sum over the images of Gamma."""
    N, na, nb, h, eri, E0, v0, B, g1, g2 = system
    eps = 1e-3  # any step is exact for a linear function; this one keeps rounding ~1e-12

    def E(hh, ee):
        H, _ = fci.dense_H(hh, ee, N, na, nb)
        return v0 @ H @ v0

    for (p, q) in ((0, 0), (1, 3), (4, 2)):
        d = np.zeros_like(h)
        d[p, q] = d[q, p] = 1.0
        fd = (E(h + eps * d, eri) - E(h - eps * d, eri)) / (2 * eps)
        assert abs(fd - (g1[p, q] + (g1[q, p] if p != q else 0.0))) < 1e-9
    for idx in ((0, 0, 1, 1), (0, 1, 2, 3), (4, 3, 1, 0), (2, 2, 2, 2)):
        d = np.zeros_like(eri)
        ims = _images(*idx)
        for im in ims:
            d[im] = 1.0
        fd = (E(h, eri + eps * d) - E(h, eri - eps * d)) / (2 * eps)
        assert abs(fd - 0.5 * sum(g2[im] for im in ims)) < 1e-9


def test_orbital_gradient_by_finite_difference(system):
    """kappa = 2 (F - F^T) is dE/dK at U = exp(K) = I with the RDMs held fixed."""
    N, na, nb, h, eri, E0, v0, B, g1, g2 = system
    kap = fci.orbital_gradient(h, eri, g1, g2)
    rng = np.random.default_rng(8)
    for _ in range(3):
        K = rng.normal(size=(N, N))
        K = K - K.T
        eps = 1e-5

        def E(t):
            U = scipy.linalg.expm(t * K)
            hh, ee = fci.rotate_integrals(h, eri, U)
            return fci.energy_from_rdms(hh, ee, g1, g2)

        fd = (E(eps) - E(-eps)) / (2 * eps)
        pred = sum(K[p, q] * kap[p, q] for p in range(N) for q in range(p))
        assert abs(fd - pred) < 1e-7 * max(1.0, abs(pred))
    # at the exact FCI ground state of the full orbital space the energy is
    # invariant under rotations of the orbitals, so kappa vanishes
    assert np.max(np.abs(kap)) < 1e-9


def test_cpp_rdm_matches_brute_force(system):
    """The C++ operator-application RDMs equal the Python brute force, for the
    ground state and for a random sparse vector."""
    from oracle import cd as ocd

    N, na, nb, h, eri, E0, v0, B, g1, g2 = system
    ka = np.array([k[0] for k in B], np.uint64)
    kb = np.array([k[1] for k in B], np.uint64)
    G1, G2 = ocd.rdm12(N, ka, kb, v0)
    np.testing.assert_allclose(G1, g1, atol=1e-13)
    np.testing.assert_allclose(G2, g2, atol=1e-13)
    rng = np.random.default_rng(11)
    c = rng.normal(size=len(B)) * (rng.random(len(B)) < 0.4)
    keep = c != 0.0
    P1, P2 = fci.rdm12([B[i] for i in range(len(B)) if keep[i]], c[keep], N)
    Q1, Q2 = ocd.rdm12(N, ka[keep], kb[keep], c[keep])
    np.testing.assert_allclose(Q1, P1, atol=1e-13)
    np.testing.assert_allclose(Q2, P2, atol=1e-13)
    # the support energy equals the Rayleigh quotient of the dense matrix
    H, _ = fci.dense_H(h, eri, N, na, nb)
    cv = np.where(keep, c, 0.0)
    assert abs(ocd.support_energy(h, eri, ka[keep], kb[keep], c[keep]) - cv @ H @ cv / (cv @ cv)) < 1e-12
