"""Pins of the OptOrbFCI oracle (Sec. 3.4, Algorithm 4) against what the
mathematics fixes: the gradient of P4 against central differences of P4
itself, the polar factor against its defining properties, the invariance of
the FCI energy under rotations of the whole orbital space (M = N), the
monotone decrease of the outer energies, and the variational bound by the
FCI energy of the full M-orbital space."""
import numpy as np

import synth_inputs
from oracle import fci
from oracle import optorb as oo


def _random_u(M, N, seed):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((M, M)))
    return Q[:, :N]


def test_gradient_matches_differences():
    M, N, na, nb = 6, 4, 2, 1
    h, eri = synth_inputs.ab_initio(M, 18, 71)
    U = _random_u(M, N, 1)
    h2, e2 = oo.rotated(h, eri, U)
    E, v, basis = fci.ground_state_dense(h2, e2, N, na, nb)
    g1, g2 = fci.rdm12(basis, v, N)
    # P4 at U equals the FCI energy there (E = sum h' gamma + 1/2 sum eri' Gamma)
    assert abs(oo.p4(h, eri, U, g1, g2) - E) < 1e-11
    G = oo.p4_grad(h, eri, U, g1, g2)
    eps = 1e-5
    rng = np.random.default_rng(2)
    for _ in range(6):
        a, i = int(rng.integers(M)), int(rng.integers(N))
        D = np.zeros_like(U)
        D[a, i] = eps
        fd = (oo.p4(h, eri, U + D, g1, g2) - oo.p4(h, eri, U - D, g1, g2)) / (2 * eps)
        assert abs(fd - G[a, i]) < 1e-7 * max(1.0, abs(G[a, i])), (a, i, fd, G[a, i])


def test_polar_factor():
    rng = np.random.default_rng(3)
    U = _random_u(7, 3, 4)
    P = rng.standard_normal((3, 3))
    P = P @ P.T + 3 * np.eye(3)  # symmetric positive definite
    assert np.allclose(oo.orth(U @ P), U, atol=1e-13)
    X = rng.standard_normal((7, 3))
    Y = oo.orth(X)
    assert np.allclose(Y.T @ Y, np.eye(3), atol=1e-13)
    # X = Y S with S symmetric positive definite
    S = Y.T @ X
    assert np.allclose(S, S.T, atol=1e-12) and np.all(np.linalg.eigvalsh(0.5 * (S + S.T)) > 0)


def test_full_space_rotations_leave_the_energy():
    """M = N: every U is a rotation of the whole space.  The exact ground state
    rotated is another state of the same space, so P4 >= E0 = P4(U0): the
    orbital problem is stationary at the start (Riemannian gradient zero, the
    generalised Brillouin condition) and every outer energy is the same."""
    M = N = 4
    na, nb = 2, 2
    h, eri = synth_inputs.ab_initio(M, 12, 72)
    U0 = _random_u(M, N, 5)
    E, U, vals = oo.optorb(h, eri, N, na, nb, U0=U0, max_outer=4, energy_tol=-1.0)
    assert len(E) == 4
    assert np.max(np.abs(E - E[0])) < 1e-10
    assert np.allclose(U.T @ U, np.eye(N), atol=1e-12)
    h2, e2 = oo.rotated(h, eri, U0)
    E0, v, basis = fci.ground_state_dense(h2, e2, N, na, nb)
    g1, g2 = fci.rdm12(basis, v, N)
    assert np.linalg.norm(oo.riemannian(U0, oo.p4_grad(h, eri, U0, g1, g2))) < 1e-9
    assert np.max(np.abs(U - U0)) < 1e-8


def test_outer_energies_decrease_to_a_bound():
    M, N, na, nb = 6, 4, 2, 2
    h, eri = synth_inputs.ab_initio(M, 18, 73)
    E, U, vals = oo.optorb(h, eri, N, na, nb, max_outer=8, max_inner=60)
    assert len(E) >= 3
    assert np.all(np.diff(E) <= 1e-12), E
    assert E[-1] < E[0] - 1e-4
    E_full = np.linalg.eigvalsh(fci.dense_H(h, eri, M, na, nb)[0])[0]
    assert E[-1] >= E_full - 1e-10
    assert np.allclose(U.T @ U, np.eye(N), atol=1e-12)
    # each orbital problem ends at or below the energy it started from
    assert np.all(vals <= E[:len(vals)] + 1e-12)
