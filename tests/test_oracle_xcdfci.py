"""Pins of the multi-state oracle (xCDFCI, Algorithm 3) against things it does
not compute itself: Algorithm 1's serial oracle (one state), the objective
f(C) = ||H + C C^T||_F^2 evaluated from its definition on a dense H, LAPACK's
lowest eigenvalues, and the maintained S = C^T C, Q = C^T H C, B = H C
recomputed from the stored rows."""
import numpy as np
import pytest

import synth_inputs
from oracle import cd as ocd
from oracle import fci
from oracle import xcdfci as oxc


def test_single_state_is_algorithm_1():
    """n = 1: the step eta g is Algorithm 1's step in c_i, so selections,
    energies and the stored vector match the C++ serial oracle."""
    h, eri = synth_inputs.ab_initio(8, 24, 7)
    keys, c0 = ocd.init_single(h, eri, 4, 3)
    K = 150
    orc = ocd.cd_run(h, eri, keys, c0, max_steps=K)
    x = oxc.xcdfci_run(h, eri, keys, c0[:, None], max_steps=K)
    checked = 0
    for s in range(K):
        g = (int(orc.sel_a[s]), int(orc.sel_b[s]))
        assert x.selections[s] == g, s
        assert abs(x.energies[s, 0] - orc.E[s]) <= 1e-11 * abs(orc.E[s]), s
        checked += 1
        if orc.gap[s] < 1e-9:
            break
    assert checked >= 100


def _dense_f(H, C):
    M = H + C @ C.T
    return float(np.sum(M * M))


def test_line_search_coefficients_match_the_objective():
    """h(eta) = f(C + eta e_i g) - f(C) with g = G_i = (4 H C + 4 C C^T C)_i,
    from dense matrices, equals the quartic with the w coefficients."""
    N, na, nb = 4, 2, 2
    h, eri = synth_inputs.ab_initio(N, 12, 5)
    H, basis = fci.dense_H(h, eri, N, na, nb)
    rng = np.random.default_rng(3)
    n = 3
    C = rng.standard_normal((len(basis), n))
    S = C.T @ C
    for i in (0, 7, 20):
        g = 4.0 * (H @ C)[i] + 4.0 * C[i] @ S
        w1, w2, w3, w4 = oxc.w_coeffs(C[i], (H @ C)[i], g, S, H[i, i])
        for eta in (-0.3, -0.05, 0.02, 0.11):
            D = np.zeros_like(C)
            D[i] = g
            ref = _dense_f(H, C + eta * D) - _dense_f(H, C)
            quart = w4 * eta**4 + w3 * eta**3 + w2 * eta**2 + w1 * eta
            assert abs(quart - ref) <= 1e-10 * max(1.0, abs(ref)), (i, eta, quart, ref)


@pytest.mark.parametrize("system,n", [("abinitio6", 3), ("ring6", 2)])
def test_converges_to_the_lowest_eigenvalues(system, n):
    """The ring needs a shift (sigma = U + 1) for a second negative eigenvalue
    on its Neel subspace; energies are reported with sigma added back."""
    shift = 0.0
    if system == "ring6":
        h, eri = fci.hubbard_integrals((6,), 1.0, 4.0)
        na = nb = 3
        D0 = ocd.neel((6,), na, nb)
        shift = 5.0
    else:
        h, eri = synth_inputs.ab_initio(6, 18, 11)
        na = nb = 3
        D0 = ocd.aufbau(h, na, nb)
    N = h.shape[0]
    H, _ = fci.dense_H(h, eri, N, na, nb)
    E = np.linalg.eigvalsh(H)[:n]
    keys, C0 = oxc.initial_rows(h, eri, D0, n)
    x = oxc.xcdfci_run(h, eri, keys, C0, max_steps=60000, dx_tol=1e-12, shift=shift)
    assert x.steps < 60000
    assert np.max(np.abs(x.energies[-1] - E)) < 1e-8, (x.energies[-1], E)


def test_maintained_matrices_and_subspace_start():
    """S, Q and B as maintained equal C^T C, C^T H C and H C recomputed from
    the stored rows (tau = 0).  The start rows are the reference determinant
    and, among the determinants the dense H connects to it, those of lowest
    diagonal (checked by brute force over the dense matrix)."""
    N, na, nb = 6, 3, 3
    h, eri = synth_inputs.ab_initio(N, 18, 11)
    H, basis = fci.dense_H(h, eri, N, na, nb)
    index = {k: i for i, k in enumerate(basis)}
    n = 3
    D0 = ocd.aufbau(h, na, nb)
    keys, C0 = oxc.initial_rows(h, eri, D0, n)
    i0 = index[D0]
    assert keys[0] == D0 and len(set(keys)) == n
    conn = [j for j in range(len(basis)) if j != i0 and H[j, i0] != 0.0]
    chosen = [index[k] for k in keys[1:]]
    assert all(H[j, i0] != 0.0 for j in chosen)
    worst = max(H[j, j] for j in chosen)
    assert all(H[j, j] >= worst for j in conn if j not in chosen)
    assert np.array_equal(C0, np.eye(n))
    x = oxc.xcdfci_run(h, eri, keys, C0, max_steps=400)
    Cm = np.zeros((len(basis), n))
    for k, row in x.C.items():
        Cm[index[k]] = row
    assert np.max(np.abs(x.S - Cm.T @ Cm)) < 1e-10 * np.max(np.abs(x.S))
    assert np.max(np.abs(x.Q - Cm.T @ H @ Cm)) < 1e-10 * np.max(np.abs(x.Q))
    HC = H @ Cm
    for k, row in x.B.items():
        assert np.max(np.abs(row - HC[index[k]])) < 1e-10, k
