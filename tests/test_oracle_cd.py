"""Pins of the oracle's line search, Algorithm 1 and Algorithm 2 against dense
LAPACK results, exact identities and brute force (no GPU)."""
import math

import numpy as np
import pytest

import synth_inputs
from oracle import cd as ocd
from oracle import fci
from oracle import linesearch as ols
from oracle import mcdfci as omc


# ---------------------------------------------------------------- line search

def _grid_argmin(v1, v2, v3):
    # brute force: fine grid around the critical points, then local refinement
    roots = np.roots([4.0, 3 * v3, 2 * v2, v1]).real
    lo, hi = roots.min() - 1.0, roots.max() + 1.0
    xs = np.linspace(lo, hi, 200001)
    ys = ols.h_of(xs, v1, v2, v3)
    return xs[np.argmin(ys)]


def test_line_search_random_cubics():
    rng = np.random.default_rng(0)
    n3 = 0
    for _ in range(300):
        c_i, b_i, H_ii, mu = rng.normal(size=4) * np.array([1.0, 3.0, 5.0, 1.0])
        mu = abs(mu) + 0.1
        v3, v2, v1 = ols.quartic_coeffs(c_i, b_i, H_ii, mu)
        e_py = ols.argmin_quartic(v1, v2, v3)
        e_cpp = ocd.line_search(v1, v2, v3)
        # both are stationary points
        for e in (e_py, e_cpp):
            dh = 4 * e**3 + 3 * v3 * e**2 + 2 * v2 * e + v1
            scale = 4 * abs(e) ** 3 + 3 * abs(v3) * e * e + 2 * abs(v2 * e) + abs(v1)
            assert abs(dh) <= 1e-12 * scale
        assert abs(e_py - e_cpp) <= 1e-10 * max(1.0, abs(e_py))
        # global minimum: no grid point is lower
        eg = _grid_argmin(v1, v2, v3)
        assert ols.h_of(e_cpp, v1, v2, v3) <= ols.h_of(eg, v1, v2, v3) + 1e-12
        if np.all(np.abs(np.roots([4.0, 3 * v3, 2 * v2, v1]).imag) < 1e-12):
            n3 += 1
    assert n3 > 20  # the three-real-root branch was exercised


def test_outer_root_rule():
    """With three real roots the minimiser is the outer root farther from the
    middle one (Appendix A); h(x3) - h(x1) = (16/3) s d^3, d = (x3-x1)/2,
    s = x2 - (x1+x3)/2."""
    for x1, x2, x3 in ((-2.0, 0.3, 1.0), (-1.0, -0.7, 3.0), (-0.5, 0.1, 0.4)):
        # h' = 4 (x-x1)(x-x2)(x-x3) = 4x^3 + 3 v3 x^2 + 2 v2 x + v1
        v3 = -4.0 * (x1 + x2 + x3) / 3.0
        v2 = 2.0 * (x1 * x2 + x1 * x3 + x2 * x3)
        v1 = -4.0 * x1 * x2 * x3
        e = ocd.line_search(v1, v2, v3)
        far = x1 if abs(x1 - x2) > abs(x3 - x2) else x3
        assert abs(e - far) < 1e-12
        d, s = (x3 - x1) / 2, x2 - (x1 + x3) / 2
        diff = ols.h_of(x3, v1, v2, v3) - ols.h_of(x1, v1, v2, v3)
        assert abs(diff - 16.0 / 3.0 * s * d**3) < 1e-10


# ---------------------------------------------------------------- Algorithm 1

def _ring8():
    h, eri = fci.hubbard_integrals((8,), 1.0, 4.0)
    return h, eri


def test_cd_ring8_converges_to_dense():
    h, eri = _ring8()
    E0 = ocd.ground_energy(h, eri, 4, 4)
    E_dense = fci.ground_state_dense(*fci.hubbard_integrals((2, 4), 1.0, 4.0), 8, 2, 2)[0]
    assert abs(ocd.ground_energy(*fci.hubbard_integrals((2, 4), 1.0, 4.0), 2, 2) - E_dense) < 1e-10
    keys, c0 = ocd.init_subspace(h, eri, ocd.neel((8,), 4, 4))
    r = ocd.cd_run(h, eri, keys, c0, max_steps=500000, dx_tol=1e-10)
    assert abs(r.energy - E0) < 1e-8
    assert r.energy >= E0 - 1e-12
    assert np.all(np.diff(r.E[r.E.size // 2:]) < 1e-9)  # settled


@pytest.mark.parametrize("system", ["ring8", "abinitio8"])
def test_cd_invariants_against_dense(system):
    """After K steps: stored b = H c, mu = c.c, alpha = c.Hc (dense products)."""
    if system == "ring8":
        h, eri = _ring8()
        N, na, nb = 8, 4, 4
        keys, c0 = ocd.init_subspace(h, eri, ocd.neel((8,), 4, 4))
    else:
        N, na, nb = 8, 3, 3
        h, eri = synth_inputs.ab_initio(N, 24, 7)
        keys, c0 = ocd.init_single(h, eri, na, nb)
    H, B = fci.dense_H(h, eri, N, na, nb)
    index = {k: i for i, k in enumerate(B)}
    for K in (1, 7, 300):
        r = ocd.cd_run(h, eri, keys, c0, max_steps=K, export=True)
        c = np.zeros(len(B))
        bst = {}
        for a, b, cv, bv in zip(r.keys_a, r.keys_b, r.c, r.b):
            c[index[(int(a), int(b))]] = cv
            bst[(int(a), int(b))] = bv
        Hc = H @ c
        for k, bv in bst.items():
            assert abs(bv - Hc[index[k]]) < 1e-11
        assert abs(r.mu - c @ c) < 1e-12 * max(1.0, c @ c)
        assert abs(r.alpha - c @ Hc) < 1e-11 * max(1.0, abs(c @ Hc))


def test_cd_objective_monotone():
    h, eri = synth_inputs.ab_initio(8, 24, 7)
    keys, c0 = ocd.init_single(h, eri, 3, 3)
    fs = []
    for K in range(1, 40):
        r = ocd.cd_run(h, eri, keys, c0, max_steps=K, trajectory=False)
        fs.append(2 * r.alpha + r.mu**2)
    assert np.all(np.diff(fs) <= 1e-10)


def test_cd_abinitio_converges_to_dense():
    N, na, nb = 8, 3, 3
    h, eri = synth_inputs.ab_initio(N, 24, 7)
    E0, _, _ = fci.ground_state_dense(h, eri, N, na, nb)
    keys, c0 = ocd.init_single(h, eri, na, nb)
    r = ocd.cd_run(h, eri, keys, c0, max_steps=200000, dx_tol=1e-11)
    assert abs(r.energy - E0) < 1e-8


def test_cd_first_step_is_argmax_and_line_search():
    """Step 1 reproduced by hand from dense H: the chosen coordinate maximises
    |4 (Hc)_j + 4 mu c_j| over the initial column, and eta minimises the quartic."""
    N, na, nb = 8, 3, 3
    h, eri = synth_inputs.ab_initio(N, 24, 7)
    H, B = fci.dense_H(h, eri, N, na, nb)
    index = {k: i for i, k in enumerate(B)}
    keys, c0 = ocd.init_single(h, eri, na, nb)
    c = np.zeros(len(B))
    c[index[keys[0]]] = c0[0]
    mu = c @ c
    g = np.abs(4 * H @ c + 4 * mu * c)
    cand = [k for k, v in fci.column(h, eri, N, *keys[0]) if v != 0.0]
    best = max(cand, key=lambda k: (g[index[k]], -k[1], -k[0]))
    r = ocd.cd_run(h, eri, keys, c0, max_steps=1)
    assert (int(r.sel_a[0]), int(r.sel_b[0])) == best
    i = index[best]
    v3, v2, v1 = ols.quartic_coeffs(c[i], (H @ c)[i], H[i, i], mu)
    assert abs(r.eta[0] - ols.argmin_quartic(v1, v2, v3)) < 1e-12


# ---------------------------------------------------------------- Algorithm 2

def test_mcdfci_step_energy_is_reduced_eigenvalue():
    """After one multicoordinate step the Rayleigh quotient equals lambda_min of
    Q^T H Q built from dense H (independent of the maintained b, alpha)."""
    N, na, nb = 8, 3, 3
    h, eri = synth_inputs.ab_initio(N, 24, 7)
    H, B = fci.dense_H(h, eri, N, na, nb)
    index = {k: i for i, k in enumerate(B)}
    keys, c0 = ocd.init_single(h, eri, na, nb)
    for m in (4, 16):
        st = omc.mcdfci_run(h, eri, keys, c0, m, max_steps=2)
        # rebuild step 2 from the state after step 1
        st1 = omc.mcdfci_run(h, eri, keys, c0, m, max_steps=1)
        c = np.zeros(len(B))
        for k, v in st1.c.items():
            c[index[k]] = v
        I = [index[k] for k in st.selections[1]]
        rest = c.copy()
        rest[I] = 0.0
        nu = np.linalg.norm(rest)
        Q = np.zeros((len(B), len(I) + 1))
        Q[:, 0] = rest / nu
        for t, i in enumerate(I):
            Q[i, t + 1] = 1.0
        lam = np.linalg.eigvalsh(Q.T @ H @ Q)[0]
        assert abs(st.energies[1] - lam) < 1e-10


def test_mcdfci_full_space_one_step():
    """m = dim with one electron per spin: the first column reaches every
    determinant, nu = 0 after selecting them all, and one step returns E0."""
    N, na, nb = 4, 1, 1
    h, eri = synth_inputs.ab_initio(N, 12, 3)
    E0, _, B = fci.ground_state_dense(h, eri, N, na, nb)
    keys, c0 = ocd.init_single(h, eri, na, nb)
    st = omc.mcdfci_run(h, eri, keys, c0, len(B), max_steps=2)
    assert len(st.selections[0]) == len(B)
    assert abs(st.energies[0] - E0) < 1e-12


@pytest.mark.parametrize("m", [4, 16])
def test_mcdfci_converges_to_dense(m):
    N, na, nb = 8, 3, 3
    h, eri = synth_inputs.ab_initio(N, 24, 7)
    E0 = ocd.ground_energy(h, eri, na, nb)
    keys, c0 = ocd.init_single(h, eri, na, nb)
    st = omc.mcdfci_run(h, eri, keys, c0, m, max_steps=10000 // m, dx_tol=1e-12)
    assert abs(st.energy - E0) < 1e-8
    assert np.all(np.array(st.energies) >= E0 - 1e-12)  # variational


def test_mcdfci_keeps_the_spin_flip_parity_of_a_closed_chosen_set():
    """With n_alpha = n_beta, H commutes with the spin flip P (alpha string <->
    beta string).  A step whose chosen set is closed under P maps a state of
    one P-parity to that parity, and a first step whose reduced eigenvector has
    no weight on the start (gamma = 0) leaves the start's parity altogether.
    Here (8 orbitals, 4+4, m = 64) the first step lands in the odd sector while
    the ground state is even; every later chosen set is closed under P, so the
    run stays odd and approaches the lowest odd eigenvalue, not E0.  Checked
    against the dense H split by parity (LAPACK on each sector)."""
    N, n = 8, 4
    h, eri = synth_inputs.ab_initio(N, 24, 1)
    H, B = fci.dense_H(h, eri, N, n, n)
    index = {k: i for i, k in enumerate(B)}
    flip = np.array([index[(b, a)] for (a, b) in B])
    assert np.max(np.abs(H[np.ix_(flip, flip)] - H)) < 1e-12
    # orthonormal bases of the even and odd sectors
    pairs = [(i, int(flip[i])) for i in range(len(B)) if i <= flip[i]]
    even = np.zeros((len(B), len(pairs)))
    odd_pairs = [(i, j) for i, j in pairs if i != j]
    odd = np.zeros((len(B), len(odd_pairs)))
    for t, (i, j) in enumerate(pairs):
        even[[i, j], t] = 1.0 / np.sqrt(2.0) if i != j else 1.0
    for t, (i, j) in enumerate(odd_pairs):
        odd[i, t], odd[j, t] = 1.0 / np.sqrt(2.0), -1.0 / np.sqrt(2.0)
    E0 = np.linalg.eigvalsh(H)[0]
    e_even = np.linalg.eigvalsh(even.T @ H @ even)[0]
    e_odd = np.linalg.eigvalsh(odd.T @ H @ odd)[0]
    assert abs(e_even - E0) < 1e-10 and e_odd > E0 + 1e-2
    keys, c0 = ocd.init_single(h, eri, n, n)
    st = omc.mcdfci_run(h, eri, keys, c0, 64, max_steps=150)
    assert st.gammas[0] < 1e-10
    for I in st.selections:
        assert {(b, a) for a, b in I} == set(I)
    x = np.zeros(len(B))
    for k, v in st.c.items():
        x[index[k]] = v
    x /= np.linalg.norm(x)
    assert np.linalg.norm(even.T @ x) < 1e-11
    assert np.all(np.array(st.energies) >= e_odd - 1e-10)
    assert st.energy - e_odd < 1e-5


@pytest.mark.parametrize("na,nb,tau", [(4, 3, 0.0), (4, 4, 1e-3)])
def test_cd_multithreaded_equals_serial(na, nb, tau):
    """The OpenMP form of Algorithm 1 (the all-core CPU baseline) follows the
    serial oracle bit for bit: same choices, steps, energies and stored set."""
    N = 10
    h, eri = synth_inputs.ab_initio(N, 30, 5)
    keys, c0 = ocd.init_single(h, eri, na, nb)
    a = ocd.cd_run(h, eri, keys, c0, tau=tau, max_steps=400)
    for threads in (1, 3, 8):
        b = ocd.cd_run_mt(h, eri, keys, c0, threads, tau=tau, max_steps=400)
        assert np.array_equal(a.E, b.E) and np.array_equal(a.eta, b.eta)
        assert np.array_equal(a.sel_a, b.sel_a) and np.array_equal(a.sel_b, b.sel_b)
        assert (a.nstored, a.elements, a.mu, a.alpha) == (b.nstored, b.elements, b.mu, b.alpha)
