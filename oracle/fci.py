"""Plain, slow FCI reference (test infrastructure only; see oracle/__init__.py).

Conventions (chosen where the paper leaves them open):

* A determinant is a pair of occupation strings (a, b): bit p of `a` set means
  spatial orbital p holds a spin-up electron, likewise `b` for spin-down.
* Spin-orbital order is all alpha orbitals 0..N-1 followed by all beta
  orbitals N..2N-1, and |a, b> = prod_{P ascending} a^dagger_P |0> with the
  smallest index leftmost.  The fermionic phase of any operator string is then
  obtained by applying the operators one at a time (Jordan-Wigner counting).
* Two-electron integrals are chemist (pq|rs); the physicist tensor of
  eq. (general-ham) is v_pqrs = (pr|qs) (Sec. 2.2, eqs. (1int)-(2int)).
* Excitation operators, the ket J being the determinant whose column is built
  (get_column, Sec. 4.1.1):  single  a^dagger_r a_p;  double
  a^dagger_r a^dagger_s a_q a_p.  The Slater-Condon entry (Sec. 2.3,
  eq. (entry)) is the phase of that operator on J times
    single: h_rp + sum_{k in occ(J)} (v_rkpk - v_rkkp)
    double: v_rspq - v_rsqp
  with v restricted to matching spins.
"""
import itertools
import math

import numpy as np

# ---------------------------------------------------------------------------
# bit strings and operator application


def occ(s):
    """Sorted list of set bit positions of a Python int."""
    out = []
    p = 0
    while s:
        if s & 1:
            out.append(p)
        s >>= 1
        p += 1
    return out


def to_spinorb(a, b, N):
    """Spin-orbital occupation integer: alpha at bits 0..N-1, beta at N..2N-1."""
    return int(a) | (int(b) << N)


def from_spinorb(x, N):
    mask = (1 << N) - 1
    return x & mask, (x >> N) & mask


def apply_ops(x, ops):
    """Apply operators right-to-left: ops is a list [(kind, P), ...] written as
    the operator string reads (leftmost first); kind 'c' creates, 'a'
    annihilates.  Returns (sign, x') or (0, None) if the result vanishes."""
    sign = 1
    for kind, P in reversed(ops):
        below = bin(x & ((1 << P) - 1)).count("1")
        occupied = (x >> P) & 1
        if kind == "a":
            if not occupied:
                return 0, None
            x ^= 1 << P
        else:
            if occupied:
                return 0, None
            x |= 1 << P
        if below & 1:
            sign = -sign
    return sign, x


def vphys(eri, N, P, Q, R, S):
    """Physicist v_PQRS = <PQ|RS> = (PR|QS) over spin-orbitals (spins must match)."""
    if (P >= N) != (R >= N) or (Q >= N) != (S >= N):
        return 0.0
    return eri[P % N, R % N, Q % N, S % N]


def hone(h, N, P, Q):
    if (P >= N) != (Q >= N):
        return 0.0
    return h[P % N, Q % N]


# ---------------------------------------------------------------------------
# Slater-Condon entries (eq. (entry))


def diagonal(h, eri, N, a, b):
    """H_{J,J} = sum_{P in occ} h_PP + 1/2 sum_{P,Q in occ} (v_PQPQ - v_PQQP)."""
    oc = occ(to_spinorb(a, b, N))
    e = sum(hone(h, N, P, P) for P in oc)
    two = 0.0
    for P in oc:
        for Q in oc:
            two += vphys(eri, N, P, Q, P, Q) - vphys(eri, N, P, Q, Q, P)
    return e + 0.5 * two


def single_element(h, eri, N, x, p, r):
    """<I|H|J> for I proportional to a^dagger_r a_p J (spin-orbital indices)."""
    sign, y = apply_ops(x, [("c", r), ("a", p)])
    if sign == 0:
        return None, 0.0
    val = hone(h, N, r, p)
    for k in occ(x):
        val += vphys(eri, N, r, k, p, k) - vphys(eri, N, r, k, k, p)
    return y, sign * val


def double_element(eri, N, x, p, q, r, s):
    """<I|H|J> for I proportional to a^dagger_r a^dagger_s a_q a_p J."""
    sign, y = apply_ops(x, [("c", r), ("c", s), ("a", q), ("a", p)])
    if sign == 0:
        return None, 0.0
    val = vphys(eri, N, r, s, p, q) - vphys(eri, N, r, s, q, p)
    return y, sign * val


def entry(h, eri, N, bra, ket):
    """H_{bra, ket} for determinants given as (a, b) pairs (get_entry)."""
    x = to_spinorb(*ket, N)
    y = to_spinorb(*bra, N)
    d = x ^ y
    nd = bin(d).count("1")
    if nd == 0:
        return diagonal(h, eri, N, *ket)
    if nd == 2:
        p = occ(d & x)[0]
        r = occ(d & y)[0]
        return single_element(h, eri, N, x, p, r)[1]
    if nd == 4:
        p, q = occ(d & x)
        r, s = occ(d & y)
        return double_element(eri, N, x, p, q, r, s)[1]
    return 0.0


def column(h, eri, N, a, b, keep_zeros=True):
    """get_column(D): list of ((a', b'), H_{D', D}) -- the diagonal first, then
    every single and double excitation of D.  Exact zeros are kept unless
    keep_zeros is False."""
    x = to_spinorb(a, b, N)
    out = [((int(a), int(b)), diagonal(h, eri, N, a, b))]
    ns = 2 * N
    oc = occ(x)
    vi = [P for P in range(ns) if not (x >> P) & 1]
    for p in oc:
        for r in vi:
            if (p >= N) != (r >= N):
                continue
            y, v = single_element(h, eri, N, x, p, r)
            out.append((from_spinorb(y, N), v))
    for p, q in itertools.combinations(oc, 2):
        for r, s in itertools.combinations(vi, 2):
            # spin must be conserved: the multiset of spins of (p, q) equals (r, s)
            if sorted([p >= N, q >= N]) != sorted([r >= N, s >= N]):
                continue
            y, v = double_element(eri, N, x, p, q, r, s)
            out.append((from_spinorb(y, N), v))
    if not keep_zeros:
        out = [out[0]] + [kv for kv in out[1:] if kv[1] != 0.0]
    return out


def column_size(N, na, nb):
    """Closed-form number of entries get_column enumerates (diagonal included)."""
    va, vb = N - na, N - nb
    return (1 + na * va + nb * vb + math.comb(na, 2) * math.comb(va, 2)
            + math.comb(nb, 2) * math.comb(vb, 2) + na * va * nb * vb)


# ---------------------------------------------------------------------------
# basis and dense matrices


def strings(N, n):
    return [sum(1 << p for p in c) for c in itertools.combinations(range(N), n)]


def basis(N, na, nb):
    """All determinants of the FCI space (Sec. 2.1), alpha-major order."""
    return [(a, b) for a in strings(N, na) for b in strings(N, nb)]


def dense_H(h, eri, N, na, nb):
    """Dense H from get_column of every determinant."""
    B = basis(N, na, nb)
    index = {k: i for i, k in enumerate(B)}
    H = np.zeros((len(B), len(B)))
    for j, (a, b) in enumerate(B):
        for key, v in column(h, eri, N, a, b):
            H[index[key], j] += v
    return H, B


def dense_H_second_quantized(h, eri, N, na, nb):
    """Dense H by applying every term of eq. (general-ham) with Jordan-Wigner
    signs: sum_PQ h_PQ a+_P a_Q + 1/2 sum_PQRS v_PQRS a+_P a+_Q a_S a_R."""
    B = basis(N, na, nb)
    index = {to_spinorb(a, b, N): i for i, (a, b) in enumerate(B)}
    ns = 2 * N
    H = np.zeros((len(B), len(B)))
    terms = []
    for P in range(ns):
        for Q in range(ns):
            c = hone(h, N, P, Q)
            if c != 0.0:
                terms.append((c, [("c", P), ("a", Q)]))
    for P in range(ns):
        for Q in range(ns):
            for R in range(ns):
                for S in range(ns):
                    c = vphys(eri, N, P, Q, R, S)
                    if c != 0.0:
                        terms.append((0.5 * c, [("c", P), ("c", Q), ("a", S), ("a", R)]))
    for j, (a, b) in enumerate(B):
        x = to_spinorb(a, b, N)
        for c, ops in terms:
            sgn, y = apply_ops(x, ops)
            if sgn:
                H[index[y], j] += sgn * c
    return H, B


def sparse_H(h, eri, N, na, nb):
    """scipy CSR H built column by column (nonzeros only)."""
    import scipy.sparse as sp

    B = basis(N, na, nb)
    index = {k: i for i, k in enumerate(B)}
    rows, cols, vals = [], [], []
    for j, (a, b) in enumerate(B):
        for key, v in column(h, eri, N, a, b, keep_zeros=False):
            rows.append(index[key])
            cols.append(j)
            vals.append(v)
    n = len(B)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n)), B


def ground_state_dense(h, eri, N, na, nb):
    """(E0, v0, basis) from LAPACK eigh on the dense FCI matrix."""
    H, B = dense_H(h, eri, N, na, nb)
    w, V = np.linalg.eigh(H)
    return w[0], V[:, 0], B


def ground_state_lanczos(h, eri, N, na, nb, tol=1e-13):
    """(E0, v0, basis) from ARPACK Lanczos on the sparse FCI matrix."""
    import scipy.sparse.linalg as sla

    H, B = sparse_H(h, eri, N, na, nb)
    w, V = sla.eigsh(H, k=1, which="SA", tol=tol)
    return w[0], V[:, 0], B


# ---------------------------------------------------------------------------
# model Hamiltonians


def hubbard_bonds(dims):
    """Distinct unordered nearest-neighbour pairs of a periodic orthogonal
    lattice (site index row-major over dims); a direction of length 2 gives a
    single bond, a direction of length 1 none."""
    dims = tuple(int(d) for d in dims)
    L = int(np.prod(dims))
    bonds = set()
    for site in range(L):
        coord = np.unravel_index(site, dims)
        for ax, n in enumerate(dims):
            if n < 2:
                continue
            nb = list(coord)
            nb[ax] = (nb[ax] + 1) % n
            other = int(np.ravel_multi_index(nb, dims))
            if other != site:
                bonds.add((min(site, other), max(site, other)))
    return sorted(bonds)


def hubbard_integrals(dims, t, U):
    """Hubbard model (Sec. 2.2) as integrals: h_ij = -t on each bond,
    (ii|ii) = U, everything else zero."""
    L = int(np.prod(dims))
    h = np.zeros((L, L))
    for i, j in hubbard_bonds(dims):
        h[i, j] = h[j, i] = -t
    eri = np.zeros((L, L, L, L))
    for i in range(L):
        eri[i, i, i, i] = U
    return h, eri


# ---------------------------------------------------------------------------
# reduced density matrices of a (sparse) wavefunction


def rdm12(keys, coeffs, N):
    """Spin-summed 1-RDM gamma[p, q] = sum_s <a+_{ps} a_{qs}> and 2-RDM
    Gamma[p, q, r, s] = sum_{s,t} <a+_{ps} a+_{rt} a_{st} a_{qs}> (chemist
    index order, so E = sum h*gamma + 1/2 sum (pq|rs) Gamma), obtained by
    applying each operator string to every determinant of the support.
    The vector is normalised first."""
    c = np.asarray(coeffs, dtype=np.float64)
    c = c / np.linalg.norm(c)
    index = {to_spinorb(a, b, N): i for i, (a, b) in enumerate(keys)}
    X = [to_spinorb(a, b, N) for (a, b) in keys]
    g1 = np.zeros((N, N))
    g2 = np.zeros((N, N, N, N))
    for j, x in enumerate(X):
        cj = c[j]
        if cj == 0.0:
            continue
        for sp in (0, N):
            for p in range(N):
                for q in range(N):
                    sgn, y = apply_ops(x, [("c", p + sp), ("a", q + sp)])
                    if sgn and y in index:
                        g1[p, q] += c[index[y]] * sgn * cj
        for s1 in (0, N):
            for s2 in (0, N):
                for p in range(N):
                    for r in range(N):
                        for s in range(N):
                            for q in range(N):
                                sgn, y = apply_ops(x, [("c", p + s1), ("c", r + s2),
                                                       ("a", s + s2), ("a", q + s1)])
                                if sgn and y in index:
                                    g2[p, q, r, s] += c[index[y]] * sgn * cj
    return g1, g2


def energy_from_rdms(h, eri, g1, g2):
    """E = sum_pq h_pq gamma_pq + 1/2 sum_pqrs (pq|rs) Gamma_pqrs."""
    return float(np.sum(h * g1) + 0.5 * np.sum(eri * g2))


def generalized_fock(h, eri, g1, g2):
    """F_pq = sum_r h_pr gamma_rq + sum_rst (pr|st) Gamma_qrst."""
    return h @ g1 + np.einsum("prst,qrst->pq", eri, g2)


def orbital_gradient(h, eri, g1, g2):
    """kappa = 2 (F - F^T): derivative of E(U = exp(K)) at K = 0 with the RDMs
    held fixed, for the rotated integrals h' = U^T h U and the matching
    transform of (pq|rs), as entry K_pq of an antisymmetric generator."""
    F = generalized_fock(h, eri, g1, g2)
    return 2.0 * (F - F.T)


def rotate_integrals(h, eri, U):
    """h' = U^T h U, (pq|rs)' = sum U_ap U_bq U_cr U_ds (ab|cd)."""
    h2 = U.T @ h @ U
    e2 = np.einsum("abcd,ap,bq,cr,ds->pqrs", eri, U, U, U, U, optimize=True)
    return h2, e2
