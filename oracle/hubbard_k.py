"""Momentum-space Hubbard model (the paper's HubbardK Hamiltonian of Sec.
4.1.1: the Hubbard model of Sec. 2.2 written in the Bloch orbitals of the
periodic lattice) and the degenerate-subspace start of Sec. 5.1.3.  Test
infrastructure only.

Orbital k is the row-major index of a momentum vector (k_1, .., k_D),
k_d in [0, dims_d).  One-body energies
    eps_k = sum_d e_d(k_d),  e_d = -2t cos(2 pi k_d / dims_d) for dims_d >= 3,
                                   -t cos(pi k_d)            for dims_d = 2,
                                   0                         for dims_d = 1
(a direction of length 2 has one bond, as in the real-space model), and
    H = sum_{k,s} eps_k n_{k s} + (U / L) sum_{k,p,q} a+_{k+q up} a_{k up} a+_{p-q dn} a_{p dn}
(the Fourier transform of U sum_i n_{i up} n_{i dn}); momentum sums are
componentwise mod dims.  Spin-orbital order: all up orbitals, then all down
ones.  Every term is applied to the determinant with fci.apply_ops, so the
matrix is the operator's, term by term.

Start (Sec. 5.1.3): the determinants of lowest one-body energy (the Fermi
shell filled in every possible way when it is degenerate), H on them, and
its lowest eigenpairs.
"""
import itertools
import math

import numpy as np

from . import fci


def momenta(dims):
    return list(itertools.product(*[range(d) for d in dims]))


def index(dims, k):
    i = 0
    for d, kd in zip(dims, k):
        i = i * d + kd
    return i


def levels(dims, t):
    eps = []
    for k in momenta(dims):
        e = 0.0
        for d, kd in zip(dims, k):
            if d == 2:
                e += -t * math.cos(math.pi * kd)
            elif d >= 3:
                e += -2.0 * t * math.cos(2.0 * math.pi * kd / d)
        eps.append(e)
    return np.array(eps)


def apply_H(dims, t, U, a, b):
    """H e_(a,b) as a dict {(a', b'): value}."""
    dims = tuple(dims)
    L = int(np.prod(dims))
    eps = levels(dims, t)
    x = fci.to_spinorb(a, b, L)
    out = {}
    d = sum(eps[p] for p in fci.occ(a)) + sum(eps[p] for p in fci.occ(b))
    ks = momenta(dims)
    for k in ks:
        for p in ks:
            for q in ks:
                kq = index(dims, tuple((k[i] + q[i]) % dims[i] for i in range(len(dims))))
                pq = index(dims, tuple((p[i] - q[i]) % dims[i] for i in range(len(dims))))
                ops = [("c", kq), ("a", index(dims, k)), ("c", L + pq), ("a", L + index(dims, p))]
                sgn, y = fci.apply_ops(x, ops)
                if sgn:
                    key = fci.from_spinorb(y, L)
                    out[key] = out.get(key, 0.0) + sgn * U / L
    out[(a, b)] = out.get((a, b), 0.0) + d
    return out


def dense_H(dims, t, U, na, nb):
    L = int(np.prod(dims))
    B = fci.basis(L, na, nb)
    idx = {k: i for i, k in enumerate(B)}
    H = np.zeros((len(B), len(B)))
    for j, (a, b) in enumerate(B):
        for key, v in apply_H(dims, t, U, a, b).items():
            H[idx[key], j] += v
    return H, B


def column(dims, t, U, a, b):
    """(alpha keys, beta keys, values) of the nonzero column of (a, b), the
    diagonal first (the form the oracle's solvers take)."""
    col = apply_H(dims, t, U, a, b)
    keys = [(a, b)] + sorted(k for k, v in col.items() if k != (a, b) and v != 0.0)
    return (np.array([k[0] for k in keys], dtype=np.uint64), np.array([k[1] for k in keys], dtype=np.uint64),
            np.array([col[k] for k in keys]))


def lowest_strings(eps, n):
    """All occupation strings of n electrons with the lowest one-body energy."""
    order = sorted(range(len(eps)), key=lambda k: eps[k])
    if n == 0:
        return [0]
    e_f = eps[order[n - 1]]
    below = [k for k in order if eps[k] < e_f - 1e-12]
    shell = [k for k in order if abs(eps[k] - e_f) <= 1e-12]
    base = sum(1 << k for k in below)
    return sorted(base | sum(1 << k for k in combo) for combo in itertools.combinations(shell, n - len(below)))


def degenerate_start(dims, t, U, na, nb, n_states=1, shift=0.0):
    """Keys of the degenerate lowest configurations and C^(0) (m x n):
    column k = sqrt(-(lambda_k - shift)) v_k for the n lowest eigenpairs of H
    on them, signed so that the first largest-magnitude entry is positive."""
    eps = levels(dims, t)
    keys = [(a, b) for a in lowest_strings(eps, na) for b in lowest_strings(eps, nb)]
    pos = {k: i for i, k in enumerate(keys)}
    Hs = np.zeros((len(keys), len(keys)))
    for j, (a, b) in enumerate(keys):
        for key, v in apply_H(dims, t, U, a, b).items():
            if key in pos:
                Hs[pos[key], j] += v
    w, V = np.linalg.eigh(Hs - shift * np.eye(len(keys)))
    if len(keys) < n_states or not w[n_states - 1] < 0:
        raise ValueError("degenerate block too small or not negative")
    C0 = np.zeros((len(keys), n_states))
    for k in range(n_states):
        v = V[:, k]
        if v[int(np.argmax(np.abs(v)))] < 0:
            v = -v
        C0[:, k] = np.sqrt(-w[k]) * v
    return keys, C0
