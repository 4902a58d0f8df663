"""Pins of the momentum-space Hubbard oracle (Sec. 4.1.1 HubbardK, Sec.
5.1.3): its spectrum against the real-space model (the eigenvalues do not
depend on the single-particle basis; a wrong sign, normalisation or
dispersion shows up in them), Hermiticity, momentum conservation of every
entry, the 4 x 4 level structure and degenerate block the paper states, and
the multi-state solver on it converging to LAPACK."""
import os

import numpy as np
import pytest

from oracle import fci
from oracle import hubbard_k as hk
from oracle import xcdfci as oxc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("dims,na,nb,U", [((4,), 2, 2, 4.0), ((2, 2), 2, 1, 3.0), ((2, 3), 2, 2, 4.0),
                                          ((3,), 2, 1, 5.0), ((5,), 3, 2, 2.0), ((2, 2, 2), 2, 2, 6.0)])
def test_spectrum_matches_real_space(dims, na, nb, U):
    t = 1.0
    Hk, _ = hk.dense_H(dims, t, U, na, nb)
    assert np.max(np.abs(Hk - Hk.T)) < 1e-14
    h, eri = fci.hubbard_integrals(dims, t, U)
    Hr, _ = fci.dense_H(h, eri, h.shape[0], na, nb)
    assert np.max(np.abs(np.linalg.eigvalsh(Hk) - np.linalg.eigvalsh(Hr))) < 1e-11


def test_entries_conserve_momentum():
    dims, t, U = (2, 3), 1.0, 4.0
    ks = hk.momenta(dims)

    def total(a, b):
        tot = [0] * len(dims)
        for s in (a, b):
            for p in fci.occ(s):
                tot = [(x + y) % d for x, y, d in zip(tot, ks[p], dims)]
        return tuple(tot)

    for a, b in fci.basis(6, 2, 2)[::7]:
        for key, v in hk.apply_H(dims, t, U, a, b).items():
            if v != 0.0:
                assert total(*key) == total(a, b)


def test_4x4_levels_and_degenerate_block():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "hubbard_4x4_levels.txt")) if not l.startswith("#")]
    neg, zero, pos, block = (int(x) for x in rows[0])
    eps = hk.levels((4, 4), 1.0)
    assert (int(np.sum(eps < -1e-12)), int(np.sum(np.abs(eps) <= 1e-12)), int(np.sum(eps > 1e-12))) == (neg, zero, pos)
    assert len(hk.lowest_strings(eps, 8)) ** 2 == block
    assert len(hk.lowest_strings(eps, 7)) == 15 and len(hk.lowest_strings(eps, 5)) == 1


def _total(dims, a, b):
    ks = hk.momenta(dims)
    tot = [0] * len(dims)
    for s in (a, b):
        for p in fci.occ(s):
            tot = [(x + y) % d for x, y, d in zip(tot, ks[p], dims)]
    return tuple(tot)


def test_start_and_solver_converge():
    """Ground states from the degenerate start (Sec. 5.1.3), by the solver
    with the momentum columns (one state: Alg. 1).  The start's block must
    reach the ground state's momentum sector; it does on these lattices (on
    2 x 4 with 3 + 3 electrons it does not: the block's lowest state lies in
    another sector than the doubly degenerate ground state)."""
    t, U = 1.0, 4.0
    for dims, na, nb in (((2, 3), 3, 3), ((6,), 2, 2), ((2, 2), 2, 2)):
        Hk, B = hk.dense_H(dims, t, U, na, nb)
        E0 = np.linalg.eigvalsh(Hk)[0]
        keys, C0 = hk.degenerate_start(dims, t, U, na, nb)
        x = oxc.xcdfci_run(None, None, keys, C0, max_steps=60000, dx_tol=1e-12,
                           column=lambda k: hk.column(dims, t, U, *k))
        assert x.steps < 60000
        assert abs(x.energies[-1][0] - E0) < 1e-8, (dims, x.energies[-1], E0)


def test_momentum_sectors_are_invariant():
    """H conserves total momentum, so a state built in some sectors stays in
    them: every determinant the solver stores has a total momentum of its
    start (why a start must reach the wanted states)."""
    dims, t, U, na, nb = (2, 3), 1.0, 4.0, 3, 3
    keys, C0 = hk.degenerate_start(dims, t, U, na, nb)
    sectors = {_total(dims, *k) for k in keys}
    x = oxc.xcdfci_run(None, None, keys, C0, max_steps=300, column=lambda k: hk.column(dims, t, U, *k))
    assert all(_total(dims, *k) in sectors for k in x.C)
