"""GPU parity of the RDM reverse pass (gamma, Gamma, kappa, energy) against
the CPU oracle, called through the C ABI.  Bars: gamma and Gamma element by
element to 1e-12 absolute (entries are O(1) sums of products of normalised
coefficients, accumulated in FP64 in a different order), kappa to 1e-10
relative to its largest entry (an N^5 contraction), energies to 1e-11 Ha; the
top-n support bit-exact as a set."""
import numpy as np
import pytest
import scipy.linalg

import synth_inputs
from oracle import cd as ocd
from oracle import fci

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2605_04483_amd as api

    return api


def _ranked(ka, kb, c):
    """Indices of the entries with c != 0 ordered by |c| descending, equal
    |c| by the smaller (beta, alpha) key: the documented support order."""
    nz = np.nonzero(c != 0.0)[0]
    order = np.lexsort((ka[nz], kb[nz], -np.abs(c[nz])))
    return nz[order]


def _compare(api, ctx, h, eri, ka, kb, c, top_n, gE, N):
    g1o, g2o = ocd.rdm12(N, ka, kb, c)
    energy, dh, deri, kap = api.cdfci_rdm_backward(ctx, gE, top_n)
    assert np.max(np.abs(dh - gE * g1o)) < 1e-12
    assert np.max(np.abs(deri - 0.5 * gE * g2o)) < 1e-12
    kap_o = gE * fci.orbital_gradient(h, eri, g1o, g2o)
    assert np.max(np.abs(kap - kap_o)) < 1e-10 * max(1.0, np.max(np.abs(kap_o)))
    E_o = ocd.support_energy(h, eri, ka, kb, c)
    assert abs(energy[0] - E_o) < 1e-11, (energy, E_o)
    assert abs(energy[1] - E_o) < 1e-11, (energy, E_o)
    return energy, dh, deri, kap


@pytest.mark.parametrize("mode", ["single", "multi"])
def test_rdm_full_support_matches_oracle(api, mode):
    """8 orbitals, 3+3 electrons, every stored nonzero coefficient."""
    N = 8
    h, eri = synth_inputs.ab_initio(N, 24, 7)
    ctx = api.cdfci_init(h, eri, 3, 3, table_slots=1 << 14)
    if mode == "single":
        api.cdfci_step(ctx, 1, 300)
    else:
        api.cdfci_step(ctx, 8, 40)
    ka, kb, c, _ = api.cdfci_export(ctx)
    _compare(api, ctx, h, eri, ka, kb, c, 0, 0.7, N)
    ctx.close()


@pytest.mark.parametrize("system,top_n", [("abinitio8", 40), ("abinitio8", 1), ("ring8", 30),
                                          ("ring8", 100000)])
def test_rdm_top_n_support(api, system, top_n):
    """The support is the documented top-n set (ties in |c| are frequent on
    the symmetric ring) and its RDMs match the oracle's on that set."""
    if system == "ring8":
        N = 8
        h, eri = fci.hubbard_integrals((8,), 1.0, 4.0)
        ctx = api.cdfci_init_hubbard((8,), 1.0, 4.0, 4, 4, table_slots=1 << 14)
        api.cdfci_step(ctx, 16, 30)
    else:
        N = 8
        h, eri = synth_inputs.ab_initio(N, 24, 7)
        ctx = api.cdfci_init(h, eri, 3, 3, table_slots=1 << 14)
        api.cdfci_step(ctx, 1, 500)
    ka, kb, c, _ = api.cdfci_export(ctx)
    idx = _ranked(ka, kb, c)[:top_n]
    sa, sb, sc, _ = api.cdfci_export(ctx, top_n=top_n)
    assert len(sa) == len(idx)
    assert set(zip(sa.tolist(), sb.tolist())) == set(zip(ka[idx].tolist(), kb[idx].tolist()))
    _compare(api, ctx, h, eri, ka[idx], kb[idx], c[idx], top_n, 1.0, N)
    ctx.close()


def test_rdm_gradients_by_finite_difference(api):
    """dh and deri against central differences of the oracle's support energy
    (a path that never forms an RDM), and kappa against differences of the
    same energy with rotated integrals U = exp(eps K)."""
    N = 6
    h, eri = synth_inputs.ab_initio(N, 18, 11)
    ctx = api.cdfci_init(h, eri, 3, 2, table_slots=1 << 12)
    api.cdfci_step(ctx, 1, 200)
    ka, kb, c, _ = api.cdfci_export(ctx)
    energy, dh, deri, kap = api.cdfci_rdm_backward(ctx, 1.0, 0)
    rng = np.random.default_rng(3)
    eps = 1e-3  # E is linear in (h, eri): the central difference is exact up to rounding
    d = rng.normal(size=(N, N))
    d = d + d.T
    fd = (ocd.support_energy(h + eps * d, eri, ka, kb, c) -
          ocd.support_energy(h - eps * d, eri, ka, kb, c)) / (2 * eps)
    assert abs(fd - np.sum(dh * d)) < 1e-9
    de = rng.normal(size=(N, N, N, N))
    de = (de + de.transpose(1, 0, 2, 3) + de.transpose(0, 1, 3, 2) + de.transpose(1, 0, 3, 2))
    de = de + de.transpose(2, 3, 0, 1)
    fd = (ocd.support_energy(h, eri + eps * de, ka, kb, c) -
          ocd.support_energy(h, eri - eps * de, ka, kb, c)) / (2 * eps)
    assert abs(fd - np.sum(deri * de)) < 1e-8
    K = rng.normal(size=(N, N))
    K = K - K.T
    e2 = 1e-5

    def E(t):
        hh, ee = fci.rotate_integrals(h, eri, scipy.linalg.expm(t * K))
        return ocd.support_energy(hh, ee, ka, kb, c)

    fd = (E(e2) - E(-e2)) / (2 * e2)
    pred = sum(K[p, q] * kap[p, q] for p in range(N) for q in range(p))
    assert abs(fd - pred) < 1e-7 * max(1.0, abs(pred))
    ctx.close()


def test_rdm_n24_sampled_and_invariants(api):
    """24 orbitals, 6+6 electrons (16,471-entry columns): after 200
    multicoordinate steps of k = 64, the top 2000 determinants match the
    oracle element by element; the full support (every nonzero c) satisfies
    Tr gamma = n, sum_pr Gamma_pprr = n (n - 1), the symmetries of Gamma, and
    the two energy evaluations agree."""
    N, na, nb = 24, 6, 6
    h, eri = synth_inputs.ab_initio(N, 72, synth_inputs.CONFIG_SEEDS["abinitio_n24"])
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 27, z_threshold=5e-5)
    api.cdfci_step(ctx, 64, 200)
    ka, kb, c, _ = api.cdfci_export(ctx)
    idx = _ranked(ka, kb, c)[:2000]
    _compare(api, ctx, h, eri, ka[idx], kb[idx], c[idx], 2000, 1.0, N)
    energy, dh, deri, kap = api.cdfci_rdm_backward(ctx, 1.0, 0)
    n = na + nb
    G = 2.0 * deri
    assert abs(np.trace(dh) - n) < 1e-10
    assert abs(np.einsum("pprr->", G) - n * (n - 1)) < 1e-9
    assert np.max(np.abs(G - G.transpose(2, 3, 0, 1))) < 1e-13
    assert np.max(np.abs(G - G.transpose(1, 0, 3, 2))) < 1e-13
    assert np.max(np.abs(dh - dh.T)) < 1e-14
    assert abs(energy[0] - energy[1]) < 1e-10 * abs(energy[0])
    assert abs(energy[0] - fci.energy_from_rdms(h, eri, dh, G)) < 1e-10 * abs(energy[0])
    assert abs(kap + kap.T).max() < 1e-12
    ctx.close()


def test_autograd_support_energy(api):
    import torch

    from paper_2605_04483_amd import autograd as ag

    N = 6
    h, eri = synth_inputs.ab_initio(N, 18, 11)
    ctx = api.cdfci_init(h, eri, 3, 2, table_slots=1 << 12)
    api.cdfci_step(ctx, 1, 200)
    ht = torch.tensor(h, requires_grad=True)
    et = torch.tensor(eri, requires_grad=True)
    E = ag.support_energy(ctx, ht, et)
    (2.5 * E).backward()
    energy, dh, deri, _ = api.cdfci_rdm_backward(ctx, 2.5, 0)
    # separate calls: FP64 atomics may add in another order
    assert abs(E.item() - energy[0]) < 1e-12
    assert np.max(np.abs(ht.grad.numpy() - dh)) < 1e-12
    assert np.max(np.abs(et.grad.numpy() - deri)) < 1e-12
    ctx.close()


def test_make_rdm12_convention(api):
    """make_rdm1 / make_rdm12 (the spin-summed RDMs in the PySCF FCI solver
    convention the reverse pass follows) against the oracle's RDMs of the
    exported state, and E = sum h gamma + 1/2 sum (pq|rs) Gamma."""
    N = 8
    h, eri = synth_inputs.ab_initio(N, 24, 7)
    ctx = api.cdfci_init(h, eri, 4, 3, table_slots=1 << 14)
    api.cdfci_step(ctx, 1, 400)
    ka, kb, c, _ = api.cdfci_export(ctx)
    g1o, g2o = ocd.rdm12(N, ka, kb, c)
    g1 = api.make_rdm1(ctx)
    d1, d2 = api.make_rdm12(ctx)
    assert np.max(np.abs(g1 - g1o)) < 1e-12 and np.max(np.abs(d1 - g1o)) < 1e-12
    assert np.max(np.abs(d2 - g2o)) < 1e-12
    E = float(np.sum(h * d1) + 0.5 * np.sum(eri * d2))
    assert abs(E - api.cdfci_energy(ctx, exact=1)) < 1e-10
    ctx.close()


def _sym8(rng, N):
    """A random tensor with the 8-fold symmetry of (pq|rs)."""
    X = rng.normal(size=(N, N, N, N))
    X = X + X.transpose(1, 0, 2, 3)
    X = X + X.transpose(0, 1, 3, 2)
    return X + X.transpose(2, 3, 0, 1)


def test_rdm_reverse_pass_at_the_benchmark_size(api):
    """The benchmark's reverse pass: 24 orbitals, 6+6, tau = 5e-5, 2^28 slots,
    the state after 10^6 single-coordinate iterations, top 10^6 determinants
    by |c| (every nonzero c: about 3e5).  The top 2000 match the oracle
    element by element; on the whole support the invariants hold, the two
    energy evaluations agree, and dE/dh, dE/d(pq|rs) equal central
    differences (steps 1e-3 and 1e-6) of the support energy c^T H c / c^T c
    evaluated by a second context holding the same c under the perturbed
    integrals (get_column-based exact energy, not the RDMs)."""
    N, na, nb = 24, 6, 6
    h, eri = synth_inputs.ab_initio(N, 72, synth_inputs.CONFIG_SEEDS["abinitio_n24"])
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 28, z_threshold=5e-5)
    for _ in range(100):
        api.cdfci_step(ctx, 1, 10000)
    ka, kb, c, _ = api.cdfci_export(ctx, top_n=1_000_000)
    assert 100_000 < len(ka) < 1_000_000
    assert np.all(c != 0.0)
    idx = _ranked(ka, kb, c)[:2000]
    _compare(api, ctx, h, eri, ka[idx], kb[idx], c[idx], 2000, 1.0, N)
    energy, dh, deri, kap = api.cdfci_rdm_backward(ctx, 1.0, 1_000_000)
    ctx.close()
    n = na + nb
    G = 2.0 * deri
    assert abs(np.trace(dh) - n) < 1e-10
    assert abs(np.einsum("pprr->", G) - n * (n - 1)) < 1e-8
    # partial trace: sum_r Gamma_pqrr = (n - 1) gamma_pq
    assert np.max(np.abs(np.einsum("pqrr->pq", G) - (n - 1) * dh)) < 1e-9
    assert np.max(np.abs(G - G.transpose(2, 3, 0, 1))) < 1e-13
    assert np.max(np.abs(dh - dh.T)) < 1e-14
    assert abs(energy[0] - energy[1]) < 1e-10 * abs(energy[0])
    assert abs(energy[0] - fci.energy_from_rdms(h, eri, dh, G)) < 1e-10 * abs(energy[0])
    assert abs(kap + kap.T).max() < 1e-12
    rng = np.random.default_rng(24)
    Dh = rng.normal(size=(N, N))
    Dh = Dh + Dh.T
    De = _sym8(rng, N) * 0.05

    def support_energy(hh, ee):
        x = api.cdfci_init(hh, ee, na, nb, table_slots=1 << 28, z_threshold=5e-5)
        api.cdfci_load(x, ka, kb, c)
        e = api.cdfci_energy(x, exact=1)
        x.close()
        return e

    assert abs(support_energy(h, eri) - energy[1]) < 1e-10 * abs(energy[1])
    for eps, bar in ((1e-3, 1e-6), (1e-6, 1e-3)):
        fd_h = (support_energy(h + eps * Dh, eri) - support_energy(h - eps * Dh, eri)) / (2 * eps)
        assert abs(fd_h - np.sum(dh * Dh)) < bar * max(1.0, abs(fd_h)), (eps, fd_h, np.sum(dh * Dh))
        fd_e = (support_energy(h, eri + eps * De) - support_energy(h, eri - eps * De)) / (2 * eps)
        assert abs(fd_e - np.sum(deri * De)) < bar * max(1.0, abs(fd_e)), (eps, fd_e, np.sum(deri * De))
