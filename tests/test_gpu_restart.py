"""Restart from a stored wavefunction (cdfci_load), the compression threshold
setter and the memory-budget search (cdfci_step_search) through the C ABI.

Bars: after a reload b equals H c over the stored set (1e-10 absolute
against sums over the oracle's columns, sampled, and against the original
context's maintained b, which agrees to rounding); the recomputed energy
equals the original context's exact c^T H c / c^T c to 1e-12 relative;
runs continued from a checkpoint converge to the oracle's ground energy
(1e-8 Ha)."""
import numpy as np
import pytest

import synth_inputs
from oracle import cd as ocd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2605_04483_amd as api

    return api


def _exact_b(h, eri, cmap, key):
    ka, kb, v = ocd.column(h, eri, *key)
    return sum(x * cmap.get((int(a), int(b)), 0.0) for a, b, x in zip(ka, kb, v))


def test_reload_rebuilds_b_and_the_energy(api):
    N, na, nb = 12, 4, 4
    h, eri = synth_inputs.ab_initio(N, 36, 51)
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 18)
    api.cdfci_step(ctx, 1, 3000)
    ka, kb, c, b = api.cdfci_export(ctx)
    E1 = api.cdfci_energy(ctx, exact=1)
    nz = c != 0.0
    ctx2 = api.cdfci_init(h, eri, na, nb, table_slots=1 << 18)
    api.cdfci_load(ctx2, ka[nz], kb[nz], c[nz])
    ka2, kb2, c2, b2 = api.cdfci_export(ctx2)
    assert abs(api.cdfci_energy(ctx2) - E1) <= 1e-12 * abs(E1)
    assert abs(api.cdfci_energy(ctx2, exact=1) - E1) <= 1e-12 * abs(E1)
    one = {(int(a), int(x)): (cc, bb) for a, x, cc, bb in zip(ka, kb, c, b)}
    two = {(int(a), int(x)): (cc, bb) for a, x, cc, bb in zip(ka2, kb2, c2, b2)}
    assert set(two) <= set(one)
    assert set(k for k in one if one[k][0] != 0.0) <= set(two)
    assert max(abs(two[k][0] - one[k][0]) for k in two) == 0.0
    assert max(abs(two[k][1] - one[k][1]) for k in two) <= 1e-10
    cmap = {k: v[0] for k, v in two.items() if v[0] != 0.0}
    rng = np.random.default_rng(1)
    keys = list(two)
    for i in rng.choice(len(keys), 20, replace=False):
        assert abs(two[keys[i]][1] - _exact_b(h, eri, cmap, keys[i])) <= 1e-10
    ctx.close()
    ctx2.close()


def test_reload_with_a_threshold_keeps_b_exact_on_the_stored_set(api):
    N, na, nb = 12, 4, 4
    h, eri = synth_inputs.ab_initio(N, 36, 51)
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 18)
    api.cdfci_step(ctx, 1, 3000)
    ka, kb, c, _ = api.cdfci_export(ctx)
    nz = c != 0.0
    occ0 = len(ka)
    api.cdfci_set_threshold(ctx, 1e-4)
    api.cdfci_load(ctx, ka[nz], kb[nz], c[nz])
    ka2, kb2, c2, b2 = api.cdfci_export(ctx)
    assert np.count_nonzero(nz) <= len(ka2) < occ0
    cmap = {(int(a), int(x)): cc for a, x, cc in zip(ka[nz], kb[nz], c[nz])}
    rng = np.random.default_rng(2)
    for i in rng.choice(len(ka2), 30, replace=False):
        key = (int(ka2[i]), int(kb2[i]))
        assert abs(b2[i] - _exact_b(h, eri, cmap, key)) <= 1e-10
    ctx.close()


def test_continued_run_converges(api):
    N, na, nb = 8, 4, 3
    h, eri = synth_inputs.ab_initio(N, 24, 31)
    E0 = ocd.ground_energy(h, eri, na, nb)
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 14)
    api.cdfci_step(ctx, 1, 500)
    ka, kb, c, _ = api.cdfci_export(ctx)
    ctx.close()
    nz = c != 0.0
    ctx2 = api.cdfci_init(h, eri, na, nb, table_slots=1 << 14, dx_threshold=1e-12)
    api.cdfci_load(ctx2, ka[nz], kb[nz], c[nz])
    st = api.cdfci_step(ctx2, 1, 200000)
    assert st["stopped"] == 1
    assert abs(api.cdfci_energy(ctx2, exact=1) - E0) < 1e-8
    # the multicoordinate step after a reload, then a reload of a context
    # that holds the multicoordinate state, continued by single steps
    api.cdfci_load(ctx2, ka[nz], kb[nz], c[nz])
    st = api.cdfci_step(ctx2, 64, 5000)
    assert abs(api.cdfci_energy(ctx2, exact=1) - E0) < 1e-8
    api.cdfci_load(ctx2, ka[nz], kb[nz], c[nz])
    st = api.cdfci_step(ctx2, 1, 200000)
    assert st["stopped"] == 1
    assert abs(api.cdfci_energy(ctx2, exact=1) - E0) < 1e-8
    ctx2.close()


def test_load_argument_errors(api):
    N, na, nb = 6, 3, 2
    h, eri = synth_inputs.ab_initio(N, 18, 11)
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 10)
    good = (0b000111, 0b000011)
    for ka, kb, c in [([0b001111], [0b000011], [1.0]),  # alpha count
                      ([0b000111], [1 << 6 | 1], [1.0]),  # orbital beyond N
                      ([good[0], good[0]], [good[1], good[1]], [1.0, 2.0]),  # repeated key
                      ([good[0]], [good[1]], [0.0]),  # zero vector
                      ([good[0]], [good[1]], [np.nan])]:
        with pytest.raises(api.CDFCIError) as e:
            api.cdfci_load(ctx, ka, kb, c)
        assert e.value.code == -1
    api.cdfci_load(ctx, [good[0]], [good[1]], [2.0])  # recovers from the rejected repeat
    assert api.cdfci_step(ctx, 1, 10)["steps"] == 10
    with pytest.raises(api.CDFCIError):
        api.cdfci_set_threshold(ctx, -1.0)
    ctx.close()


def test_search_keeps_the_table_within_budget(api):
    """N = 10, 5 + 5 (63,504 determinants) in 2^14 slots (12,943 entries at the
    0.79 load): at tau = 0 the table fills; the search raises tau instead, and
    the energy keeps falling."""
    N, na, nb = 10, 5, 5
    h, eri = synth_inputs.ab_initio(N, 30, 61)
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 14)
    with pytest.raises(api.CDFCIError) as e:
        api.cdfci_step(ctx, 1, 20000)
    assert e.value.code == -3
    ctx.close()
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 14)
    E_start = api.cdfci_energy(ctx)
    st, tau = api.cdfci_step_search(ctx, 20000, chunk=1000, fill=0.9, growth=10.0, tau0=1e-6)
    assert st["steps"] == 20000
    assert tau > 0.0
    assert st["occupied"] <= 0.79 * (1 << 14)
    E = api.cdfci_energy(ctx, exact=1)
    assert E < E_start
    assert E >= ocd.ground_energy(h, eri, na, nb) - 1e-9
    ctx.close()


def test_reload_on_a_lattice_context(api):
    """Restart of a real-space Hubbard context (Neel subspace start) from a
    checkpoint of an earlier run, continued to the ground energy."""
    from oracle import fci

    dims, na, nb, t, U = (2, 3), 3, 3, 1.0, 4.0
    h, eri = fci.hubbard_integrals(dims, t, U)
    E0 = ocd.ground_energy(h, eri, na, nb)
    ctx = api.cdfci_init_hubbard(dims, t, U, na, nb, table_slots=1 << 12)
    api.cdfci_step(ctx, 1, 300)
    ka, kb, c, _ = api.cdfci_export(ctx)
    nz = c != 0.0
    ctx.close()
    ctx = api.cdfci_init_hubbard(dims, t, U, na, nb, table_slots=1 << 12, dx_threshold=1e-12)
    api.cdfci_load(ctx, ka[nz], kb[nz], c[nz])
    st = api.cdfci_step(ctx, 1, 300000)
    assert st["stopped"] == 1
    assert abs(api.cdfci_energy(ctx, exact=1) - E0) < 1e-8
    ctx.close()


def test_fcidump_input(api):
    """The golden two-site Hubbard FCIDUMP through cdfci_read_fcidump into
    both solvers: ground energy (U - sqrt(U^2 + 16 t^2)) / 2 at t = 1, U = 4
    (the closed form of Sec. 2.2) and, with two states and a shift, the
    two lowest eigenvalues of the 4-determinant space (LAPACK)."""
    import os

    from oracle import fci

    path = os.path.join(os.path.dirname(__file__), "golden", "hubbard_dimer.FCIDUMP")
    h, eri, na, nb, ecore = api.read_fcidump(path)
    E0 = (4.0 - np.sqrt(32.0)) / 2
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 8, init_kind=2, dx_threshold=1e-14)
    api.cdfci_step(ctx, 1, 10000)
    assert abs(api.cdfci_energy(ctx, exact=1) + ecore - E0) < 1e-12
    ctx.close()
    H, _ = fci.dense_H(h, eri, 2, na, nb)
    w = np.linalg.eigvalsh(H)
    x = api.cdfci_xinit(h, eri, na, nb, 2, shift=5.0, table_slots=1 << 8, dx_threshold=1e-14)
    api.cdfci_xstep(x, 20000)
    assert np.max(np.abs(api.cdfci_xenergies(x) - w[:2])) < 1e-10
    x.close()
