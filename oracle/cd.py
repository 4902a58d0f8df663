"""ctypes driver for the serial CD oracle (cd_serial.cpp) and the initial-vector
rules.  Test infrastructure only.

Initial vectors (Alg. 1 starts from a given c^(0) with b^(0) = H c^(0)):
* ab initio: the aufbau determinant (the n_alpha / n_beta orbitals with the
  lowest h_pp, ties to the lower index) with c^(0) = sqrt(-H_00) e_0, the
  exact minimiser of f along e_0 (needs H_00 < 0, since the objective has
  nonzero minimisers only for a negative eigenvalue, Sec. 2.3);
* lattice models: a Neel-type determinant (alpha on the even-coordinate-sum
  sublattice, beta on the rest, both filled in ascending site order) and
  c^(0) = sqrt(-lambda) v from the lowest eigenpair of H restricted to that
  determinant and its column -- the real-space counterpart of the paper's
  subspace initialisation for the Hubbard model (Sec. 5.1.3).  The sign of v
  makes its component on the Neel determinant non-negative.
"""
import ctypes
import os

import numpy as np

from . import fci

_lib = None


def bind(path):
    """Load a build of cd_serial.cpp from `path` and declare its signatures."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    up = ctypes.POINTER(ctypes.c_uint64)
    ip = ctypes.POINTER(ctypes.c_int64)
    L.oracle_line_search.restype = ctypes.c_double
    L.oracle_line_search.argtypes = [ctypes.c_double] * 3
    L.oracle_entry.restype = ctypes.c_double
    L.oracle_entry.argtypes = [ctypes.c_int, dp, dp] + [ctypes.c_uint64] * 4
    L.oracle_column.restype = ctypes.c_int64
    L.oracle_column.argtypes = [ctypes.c_int, dp, dp, ctypes.c_uint64, ctypes.c_uint64,
                                ctypes.c_int64, up, up, dp]
    L.oracle_cd_run_mt.restype = ctypes.c_int
    L.oracle_cd_run_mt.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, up, up, dp, ctypes.c_double,
                                   ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, up,
                                   up, dp, ip, dp, dp, ip, ip]
    L.oracle_cd_run.restype = ctypes.c_int
    L.oracle_cd_run.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, up, up, dp,
                                ctypes.c_double, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, dp, up, up, dp, dp, ip, dp, dp, ip, ip,
                                ctypes.c_int64, up, up, dp, dp]
    return L


def lib():
    global _lib
    if _lib is None:
        from .build import LIB, build

        if not os.path.exists(LIB):
            build()
        _lib = bind(LIB)
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t)) if a is not None else None


def line_search(v1, v2, v3):
    return lib().oracle_line_search(v1, v2, v3)


def column(h, eri, a, b):
    """get_column of (a, b): arrays (ka, kb, vals), diagonal first."""
    N = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    cap = fci.column_size(N, bin(int(a)).count("1"), bin(int(b)).count("1"))
    ka = np.zeros(cap, np.uint64)
    kb = np.zeros(cap, np.uint64)
    v = np.zeros(cap)
    n = lib().oracle_column(N, _p(h, ctypes.c_double), _p(eri, ctypes.c_double), int(a), int(b),
                            cap, _p(ka, ctypes.c_uint64), _p(kb, ctypes.c_uint64),
                            _p(v, ctypes.c_double))
    assert n >= 0
    return ka[:n], kb[:n], v[:n]


def entry(h, eri, bra, ket):
    N = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    return lib().oracle_entry(N, _p(h, ctypes.c_double), _p(eri, ctypes.c_double),
                              int(bra[0]), int(bra[1]), int(ket[0]), int(ket[1]))


# ---------------------------------------------------------------------------
# initial vectors


def aufbau(h, na, nb):
    order = sorted(range(h.shape[0]), key=lambda p: (h[p, p], p))
    a = sum(1 << p for p in order[:na])
    b = sum(1 << p for p in order[:nb])
    return a, b


def neel(dims, na, nb):
    dims = tuple(int(d) for d in dims)
    L = int(np.prod(dims))
    even = [s for s in range(L) if sum(np.unravel_index(s, dims)) % 2 == 0]
    odd = [s for s in range(L) if sum(np.unravel_index(s, dims)) % 2 == 1]
    a_sites = (even + odd)[:na]
    rest = [s for s in range(L) if s not in a_sites]
    b_sites = (rest + a_sites)[:nb]
    return sum(1 << s for s in a_sites), sum(1 << s for s in b_sites)


def init_single(h, eri, na, nb):
    """Aufbau determinant with c = sqrt(-H_00)."""
    a, b = aufbau(h, na, nb)
    H00 = fci.diagonal(h, eri, h.shape[0], a, b)
    if not H00 < 0:
        raise ValueError("H_00 >= 0: no negative rank-one minimiser along e_0")
    return [(a, b)], np.array([np.sqrt(-H00)])


def init_subspace(h, eri, D0):
    """sqrt(-lambda) v for the lowest eigenpair of H on {D0} + column(D0)."""
    N = h.shape[0]
    ka, kb, v = column(h, eri, *D0)
    keys = [(int(ka[0]), int(kb[0]))] + [(int(x), int(y)) for x, y, z in zip(ka[1:], kb[1:], v[1:])
                                         if z != 0.0]
    n = len(keys)
    Hs = np.zeros((n, n))
    for j, kj in enumerate(keys):
        for i, ki in enumerate(keys):
            Hs[i, j] = fci.entry(h, eri, N, ki, kj)
    w, V = np.linalg.eigh(Hs)
    if not w[0] < 0:
        raise ValueError("lowest subspace eigenvalue is not negative")
    vec = V[:, 0]
    if vec[0] < 0:
        vec = -vec
    return keys, np.sqrt(-w[0]) * vec


# ---------------------------------------------------------------------------
# Algorithm 1


class CDResult:
    pass


def cd_run(h, eri, init_keys, init_c, tau=0.0, max_steps=1000, theta=0.9, dx_tol=0.0,
           trajectory=True, export=False, library=None):
    """Algorithm 1 from c^(0) = sum init_c[t] e_{init_keys[t]}.  `library` is
    a build bound by bind() (default: the oracle's own build)."""
    N = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    ia = np.array([k[0] for k in init_keys], np.uint64)
    ib = np.array([k[1] for k in init_keys], np.uint64)
    ic = np.ascontiguousarray(init_c, dtype=np.float64)
    T = max_steps if trajectory else 0
    tE = np.zeros(T) if trajectory else None
    ta = np.zeros(T, np.uint64) if trajectory else None
    tb = np.zeros(T, np.uint64) if trajectory else None
    te = np.zeros(T) if trajectory else None
    tg = np.zeros(T) if trajectory else None
    steps = np.zeros(1, np.int64)
    mu = np.zeros(1)
    al = np.zeros(1)
    nst = np.zeros(1, np.int64)
    nel = np.zeros(1, np.int64)
    cap = 0
    oa = ob = oc = ov = None
    L = library if library is not None else lib()

    def call(cap, oa, ob, oc, ov):
        return L.oracle_cd_run(N, _p(h, ctypes.c_double), _p(eri, ctypes.c_double), len(ia),
                               _p(ia, ctypes.c_uint64), _p(ib, ctypes.c_uint64),
                               _p(ic, ctypes.c_double), tau, max_steps, theta, dx_tol,
                               _p(tE, ctypes.c_double), _p(ta, ctypes.c_uint64),
                               _p(tb, ctypes.c_uint64), _p(te, ctypes.c_double),
                               _p(tg, ctypes.c_double), _p(steps, ctypes.c_int64),
                               _p(mu, ctypes.c_double), _p(al, ctypes.c_double),
                               _p(nst, ctypes.c_int64), _p(nel, ctypes.c_int64), cap,
                               _p(oa, ctypes.c_uint64), _p(ob, ctypes.c_uint64),
                               _p(oc, ctypes.c_double), _p(ov, ctypes.c_double))

    rc = call(cap, oa, ob, oc, ov)
    if rc != 0:
        raise RuntimeError(f"oracle_cd_run failed: {rc}")
    if export:
        cap = int(nst[0])
        oa = np.zeros(cap, np.uint64)
        ob = np.zeros(cap, np.uint64)
        oc = np.zeros(cap)
        ov = np.zeros(cap)
        rc = call(cap, oa, ob, oc, ov)
        assert rc == 0
    r = CDResult()
    n = int(steps[0])
    r.steps = n
    r.mu = float(mu[0])
    r.alpha = float(al[0])
    r.energy = r.alpha / r.mu
    r.nstored = int(nst[0])
    r.elements = int(nel[0])
    if trajectory:
        r.E = tE[:n]
        r.sel_a = ta[:n]
        r.sel_b = tb[:n]
        r.eta = te[:n]
        r.gap = tg[:n]
    if export:
        r.keys_a, r.keys_b, r.c, r.b = oa, ob, oc, ov
    return r


def cd_run_mt(h, eri, init_keys, init_c, threads, tau=0.0, max_steps=1000, theta=0.9, dx_tol=0.0,
              trajectory=True):
    """Algorithm 1 on `threads` host threads (OpenMP); the same trajectory as
    cd_run, bit for bit.  For the CPU timing baseline."""
    N = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    ia = np.array([k[0] for k in init_keys], np.uint64)
    ib = np.array([k[1] for k in init_keys], np.uint64)
    ic = np.ascontiguousarray(init_c, dtype=np.float64)
    T = max_steps if trajectory else 0
    tE = np.zeros(T) if trajectory else None
    ta = np.zeros(T, np.uint64) if trajectory else None
    tb = np.zeros(T, np.uint64) if trajectory else None
    te = np.zeros(T) if trajectory else None
    steps = np.zeros(1, np.int64)
    mu = np.zeros(1)
    al = np.zeros(1)
    nst = np.zeros(1, np.int64)
    nel = np.zeros(1, np.int64)
    rc = lib().oracle_cd_run_mt(N, _p(h, ctypes.c_double), _p(eri, ctypes.c_double), len(ia),
                                _p(ia, ctypes.c_uint64), _p(ib, ctypes.c_uint64), _p(ic, ctypes.c_double),
                                tau, max_steps, theta, dx_tol, int(threads), _p(tE, ctypes.c_double),
                                _p(ta, ctypes.c_uint64), _p(tb, ctypes.c_uint64), _p(te, ctypes.c_double),
                                _p(steps, ctypes.c_int64), _p(mu, ctypes.c_double), _p(al, ctypes.c_double),
                                _p(nst, ctypes.c_int64), _p(nel, ctypes.c_int64))
    if rc != 0:
        raise RuntimeError(f"oracle_cd_run_mt failed: {rc}")
    r = CDResult()
    n = int(steps[0])
    r.steps = n
    r.mu = float(mu[0])
    r.alpha = float(al[0])
    r.energy = r.alpha / r.mu
    r.nstored = int(nst[0])
    r.elements = int(nel[0])
    if trajectory:
        r.E, r.sel_a, r.sel_b, r.eta = tE[:n], ta[:n], tb[:n], te[:n]
    return r


def sparse_H(h, eri, na, nb):
    """scipy CSR FCI matrix from the C++ get_column (nonzeros only)."""
    import scipy.sparse as sp

    N = h.shape[0]
    B = fci.basis(N, na, nb)
    index = {k: i for i, k in enumerate(B)}
    rows, cols, vals = [], [], []
    for j, (a, b) in enumerate(B):
        ka, kb, v = column(h, eri, a, b)
        nz = v != 0.0
        for x, y, z in zip(ka[nz].tolist(), kb[nz].tolist(), v[nz].tolist()):
            rows.append(index[(x, y)])
            cols.append(j)
            vals.append(z)
    n = len(B)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n)), B


def ground_energy(h, eri, na, nb, dense_max=3000):
    """E0 by LAPACK eigh (dimension <= dense_max) else ARPACK Lanczos."""
    import scipy.sparse.linalg as sla

    H, B = sparse_H(h, eri, na, nb)
    if len(B) <= dense_max:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    w = sla.eigsh(H, k=1, which="SA", tol=1e-14, return_eigenvectors=False)
    return float(w[0])


def rdm12(N, keys_a, keys_b, c):
    """Spin-summed 1- and 2-RDMs (chemist order) of the normalised vector c
    over the given determinants, from the C++ operator-application oracle."""
    L = lib()
    if not hasattr(L, "_rdm_bound"):
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_rdm12.restype = ctypes.c_int
        L.oracle_rdm12.argtypes = [ctypes.c_int, ctypes.c_int64, up, up, dp, dp, dp]
        L.oracle_support_energy.restype = ctypes.c_double
        L.oracle_support_energy.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int64, up, up, dp]
        L._rdm_bound = True
    ka = np.ascontiguousarray(keys_a, dtype=np.uint64)
    kb = np.ascontiguousarray(keys_b, dtype=np.uint64)
    cc = np.ascontiguousarray(c, dtype=np.float64)
    g1 = np.zeros((N, N))
    g2 = np.zeros((N, N, N, N))
    rc = L.oracle_rdm12(N, len(cc), _p(ka, ctypes.c_uint64), _p(kb, ctypes.c_uint64),
                        _p(cc, ctypes.c_double), _p(g1, ctypes.c_double), _p(g2, ctypes.c_double))
    assert rc == 0
    return g1, g2


def support_energy(h, eri, keys_a, keys_b, c):
    """c^T H c / c^T c restricted to the given determinants."""
    rdm12(1, np.zeros(1, np.uint64), np.zeros(1, np.uint64), np.ones(1))  # binds the symbols
    L = lib()
    N = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    ka = np.ascontiguousarray(keys_a, dtype=np.uint64)
    kb = np.ascontiguousarray(keys_b, dtype=np.uint64)
    cc = np.ascontiguousarray(c, dtype=np.float64)
    return L.oracle_support_energy(N, _p(h, ctypes.c_double), _p(eri, ctypes.c_double), len(cc),
                                   _p(ka, ctypes.c_uint64), _p(kb, ctypes.c_uint64),
                                   _p(cc, ctypes.c_double))
