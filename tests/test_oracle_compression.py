"""Pins of the oracle's compression rule (Sec. 3.1: with a threshold tau, an
increment eta H_ji of b_j is dropped when c_j = 0 and |eta H_ji| < tau, and a
determinant not yet stored is stored only by an increment that is kept; Alg. 2
applies the same rule to every contribution eta_i H_ji of a multicoordinate
step).  Checked without the oracle's own bookkeeping, from a dense H built by
the Python Slater-Condon rules and the trajectory (chosen coordinates, steps)
the oracle reports:

* every stored j with c_j != 0 has b_j = (H c)_j (its b was recalculated when j
  was chosen and no later increment of it is dropped);
* every stored j with c_j = 0 has |b_j - (H c)_j| at most (number of
  increments to j) * tau (each dropped increment is smaller than tau), and so
  has every determinant that is not stored, whose (H c)_j consists of dropped
  increments only;
* the stored set is exactly the start (c^(0), its column), the chosen
  coordinates and every j that received one increment of size >= tau;
* a tau above every increment stores nothing beyond the start and the chosen
  coordinates.

Planted mistakes (the comparison turned strict, the c_j != 0 clause dropped,
a determinant stored by a dropped increment) are compiled from edited copies
of the oracle's source in a temporary directory and must each break one of
the pins.  No GPU."""
import importlib.util
import os
import subprocess
import sys

import numpy as np
import pytest

import synth_inputs
from oracle import cd as ocd
from oracle import fci
from oracle import mcdfci as omc
from oracle import xcdfci as oxc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N, NA, NB, NAUX, SEED = 8, 3, 3, 24, 7


@pytest.fixture(scope="module")
def system():
    h, eri = synth_inputs.ab_initio(N, NAUX, SEED)
    H, B = fci.dense_H(h, eri, N, NA, NB)
    index = {k: i for i, k in enumerate(B)}
    keys, c0 = ocd.init_single(h, eri, NA, NB)
    return h, eri, H, B, index, keys, c0


def _start_set(H, index, B, keys):
    s = set(keys)
    for k in keys:
        s |= {B[j] for j in np.nonzero(H[:, index[k]])[0]}
    return s


def _cd_violations(sysd, r, tau):
    """Pins of a single-coordinate run r (exported state and trajectory)."""
    h, eri, H, B, index, keys, c0 = sysd
    bad = []
    c = np.zeros(len(B))
    stored = {}
    for a, b, cv, bv in zip(r.keys_a, r.keys_b, r.c, r.b):
        k = (int(a), int(b))
        c[index[k]] = cv
        stored[k] = bv
    Hc = H @ c
    # increments per determinant: eta_t H_{j, I_t} for j != I_t
    nincr = np.zeros(len(B), np.int64)
    big = np.zeros(len(B), bool)
    chosen = set()
    for t in range(r.steps):
        I = (int(r.sel_a[t]), int(r.sel_b[t]))
        chosen.add(I)
        col = H[:, index[I]].copy()
        col[index[I]] = 0.0
        nz = col != 0.0
        nincr += nz
        big |= nz & (np.abs(r.eta[t] * col) >= tau)
    for k, bv in stored.items():
        j = index[k]
        if c[j] != 0.0:
            if abs(bv - Hc[j]) > 1e-11 * max(1.0, abs(Hc[j])):
                bad.append(("exact b for c != 0", k, bv, Hc[j]))
        elif abs(bv - Hc[j]) > nincr[j] * tau + 1e-12:
            bad.append(("dropped increments bound", k, bv, Hc[j], nincr[j]))
    for j, k in enumerate(B):
        if k not in stored and abs(Hc[j]) > nincr[j] * tau + 1e-12:
            bad.append(("unstored bound", k, Hc[j], nincr[j]))
    expect = _start_set(H, index, B, keys) | chosen | {B[j] for j in np.nonzero(big)[0]}
    if set(stored) != expect:
        bad.append(("stored set", len(set(stored) - expect), len(expect - set(stored))))
    return bad


def _exact_tau(sysd, r0):
    """A tau equal, bit for bit, to |eta_0 H_{j*, I_0}| for an alpha-beta double
    j* of the first column (its entry is one integral, so the Python and C++
    rules give the same double)."""
    h, eri, H, B, index, keys, c0 = sysd
    I0 = (int(r0.sel_a[0]), int(r0.sel_b[0]))
    ka, kb, v = ocd.column(h, eri, *I0)
    best = None
    for a, b, x in zip(ka.tolist(), kb.tolist(), v.tolist()):
        if x == 0.0 or bin(a ^ I0[0]).count("1") != 2 or bin(b ^ I0[1]).count("1") != 2:
            continue
        if (a, b) in _start_set(H, index, B, keys):
            continue
        val = abs(r0.eta[0] * x)
        if best is None or val > best[0]:
            best = (val, (a, b))
    return best


def test_cd_compression_pins_hold(system):
    h, eri, H, B, index, keys, c0 = system
    r = ocd.cd_run(h, eri, keys, c0, tau=2e-3, max_steps=400, export=True)
    assert _cd_violations(system, r, 2e-3) == []
    # the rule was exercised: some increments were dropped, some stored new entries
    assert 0 < r.nstored < len(B)
    r_all = ocd.cd_run(h, eri, keys, c0, tau=0.0, max_steps=400, export=True)
    assert r_all.nstored > r.nstored


def test_cd_compression_huge_tau_stores_nothing_new(system):
    h, eri, H, B, index, keys, c0 = system
    r = ocd.cd_run(h, eri, keys, c0, tau=1e30, max_steps=200, export=True)
    chosen = {(int(a), int(b)) for a, b in zip(r.sel_a, r.sel_b)}
    stored = {(int(a), int(b)) for a, b in zip(r.keys_a, r.keys_b)}
    assert stored == _start_set(H, index, B, keys) | chosen
    assert _cd_violations(system, r, 1e30) == []


def test_cd_compression_threshold_is_inclusive(system):
    """tau equal to an increment of the first step: that increment is kept
    (|eta H_ji| >= tau) and stores its determinant."""
    h, eri, H, B, index, keys, c0 = system
    r0 = ocd.cd_run(h, eri, keys, c0, max_steps=1)
    tau, jstar = _exact_tau(system, r0)
    r = ocd.cd_run(h, eri, keys, c0, tau=tau, max_steps=1, export=True)
    stored = {(int(a), int(b)) for a, b in zip(r.keys_a, r.keys_b)}
    assert jstar in stored
    assert _cd_violations(system, r, tau) == []


# ---------------------------------------------------------------- planted mistakes

_RULE = "      if (cj != 0.0 || fabs(delta) >= tau) {\n        if (it == wf.end()) it = wf.emplace(e.k, Val{}).first;\n"
PLANTS = {
    "strict": (_RULE, _RULE.replace(">= tau", "> tau")),
    "no_cj_clause": (_RULE, _RULE.replace("cj != 0.0 || ", "")),
    "store_dropped": (_RULE, "      if (it == wf.end()) it = wf.emplace(e.k, Val{}).first;\n"
                             "      if (cj != 0.0 || fabs(delta) >= tau) {\n"),
}


def _planted_lib(tmp_path, name):
    src = open(os.path.join(ROOT, "oracle", "cd_serial.cpp")).read()
    old, new = PLANTS[name]
    assert src.count(old) == 1
    path = os.path.join(str(tmp_path), f"liboracle_{name}.so")
    cpp = os.path.join(str(tmp_path), f"cd_{name}.cpp")
    open(cpp, "w").write(src.replace(old, new))
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-o", path, cpp, "-lquadmath"], check=True)
    return ocd.bind(path)


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_cd_planted_mistakes_break_a_pin(system, tmp_path, name):
    h, eri, H, B, index, keys, c0 = system
    L = _planted_lib(tmp_path, name)
    r0 = ocd.cd_run(h, eri, keys, c0, max_steps=1)
    tau_eq, _ = _exact_tau(system, r0)
    found = False
    for tau, K in ((tau_eq, 1), (tau_eq, 60), (2e-3, 400)):
        r = ocd.cd_run(h, eri, keys, c0, tau=tau, max_steps=K, export=True, library=L)
        if _cd_violations(system, r, tau):
            found = True
            break
    assert found, name


# ---------------------------------------------------------------- Algorithm 2

def _mcd_violations(sysd, st, tau):
    h, eri, H, B, index, keys, c0 = sysd
    bad = []
    c = np.zeros(len(B))
    for k, v in st.c.items():
        c[index[k]] = v
    Hc = H @ c
    stored = set(st.c) | set(st.b)
    # bound on the dropped part: each increment is scaled by the later gammas
    bound = np.zeros(len(B))
    big = np.zeros(len(B), bool)
    chosen = set()
    for I, eta, gam in zip(st.selections, st.etas, st.gammas):
        bound *= abs(gam)
        Iidx = [index[i] for i in I]
        chosen |= set(I)
        for i, e in zip(Iidx, eta):
            col = H[:, i].copy()
            col[i] = 0.0
            nz = col != 0.0
            bound += nz * tau
            big |= nz & (np.abs(e * col) >= tau)
    for k in stored:
        j = index[k]
        bv = st.b.get(k, 0.0)
        if c[j] != 0.0:
            if abs(bv - Hc[j]) > 1e-10 * max(1.0, abs(Hc[j])):
                bad.append(("exact b for c != 0", k, bv, Hc[j]))
        elif abs(bv - Hc[j]) > bound[j] + 1e-11:
            bad.append(("dropped increments bound", k, bv, Hc[j]))
    for j, k in enumerate(B):
        if k not in stored and abs(Hc[j]) > bound[j] + 1e-11:
            bad.append(("unstored bound", k, Hc[j]))
    expect = _start_set(H, index, B, keys) | chosen | {B[j] for j in np.nonzero(big)[0]}
    if stored != expect:
        bad.append(("stored set", len(stored - expect), len(expect - stored)))
    return bad


def _mcd_module(name, old, new):
    src = open(os.path.join(ROOT, "oracle", "mcdfci.py")).read()
    assert src.count(old) == 1
    spec = importlib.util.spec_from_loader(f"oracle._planted_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), f"<planted {name}>", "exec"), mod.__dict__)
    return mod


_MRULE = "                if c.get(j, 0.0) != 0.0 or abs(delta) >= tau:\n                    b[j] = b.get(j, 0.0) + delta\n"
MPLANTS = {
    "strict": _MRULE.replace(">= tau", "> tau"),
    "no_cj_clause": _MRULE.replace("c.get(j, 0.0) != 0.0 or ", ""),
    "store_dropped": "                b.setdefault(j, 0.0)\n" + _MRULE,
}


@pytest.mark.parametrize("m", [4, 16])
def test_mcd_compression_pins_hold(system, m):
    h, eri, H, B, index, keys, c0 = system
    st = omc.mcdfci_run(h, eri, keys, c0, m, tau=2e-3, max_steps=40)
    assert _mcd_violations(system, st, 2e-3) == []
    full = omc.mcdfci_run(h, eri, keys, c0, m, tau=0.0, max_steps=40)
    assert len(set(full.c) | set(full.b)) > len(set(st.c) | set(st.b))


@pytest.mark.parametrize("name", sorted(MPLANTS))
def test_mcd_planted_mistakes_break_a_pin(system, name):
    h, eri, H, B, index, keys, c0 = system
    mod = _mcd_module(name, _MRULE, MPLANTS[name])
    first = omc.mcdfci_run(h, eri, keys, c0, 4, max_steps=1)
    # tau equal to the largest first-step increment onto a determinant outside the start
    start = _start_set(H, index, B, keys)
    incs = []
    for i, e in zip(first.selections[0], first.etas[0]):
        ka, kb, v = ocd.column(h, eri, *i)
        for a, b, x in zip(ka.tolist(), kb.tolist(), v.tolist()):
            if x != 0.0 and (a, b) not in start and bin(a ^ i[0]).count("1") == 2 \
                    and bin(b ^ i[1]).count("1") == 2:
                incs.append(abs(e * x))
    tau_eq = max(incs)
    found = False
    for tau, K in ((tau_eq, 1), (2e-3, 40)):
        st = mod.mcdfci_run(h, eri, keys, c0, 4, tau=tau, max_steps=K)
        if _mcd_violations(system, st, tau):
            found = True
            break
    assert found, name


# ---------------------------------------------------------------- Algorithm 3

def test_xcd_compression_pins_hold(system):
    """Several states: a row increment eta H_ji g is kept iff C_j != 0 or
    |eta H_ji| ||g||_inf >= tau; rows with C_j != 0 then hold B_j = (H C)_j."""
    h, eri, H, B, index, keys, c0 = system
    nst, tau = 2, 2e-3
    xkeys, C0 = oxc.initial_rows(h, eri, ocd.aufbau(h, NA, NB), nst)
    r = oxc.xcdfci_run(h, eri, xkeys, C0, tau=tau, max_steps=300)
    C = np.zeros((len(B), nst))
    for k, v in r.C.items():
        C[index[k]] = v
    HC = H @ C
    big = np.zeros(len(B), bool)
    chosen = set()
    for i, eta, gi in zip(r.selections, r.eta, r.ginf):
        chosen.add(i)
        col = H[:, index[i]].copy()
        col[index[i]] = 0.0
        big |= (col != 0.0) & (np.abs(eta * col) * gi >= tau)
    for k in r.C:
        j = index[k]
        if np.any(C[j] != 0.0):
            assert np.max(np.abs(r.B[k] - HC[j])) <= 1e-10 * max(1.0, np.max(np.abs(HC[j])))
    start = set(xkeys)
    for k in xkeys:
        start |= {B[j] for j in np.nonzero(H[:, index[k]])[0]}
    expect = start | chosen | {B[j] for j in np.nonzero(big)[0]}
    assert set(r.C) == expect
    assert len(expect) < len(B)
