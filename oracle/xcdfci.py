"""Serial coordinate descent for several low-lying states, xCDFCI (Sec. 3.3,
Algorithm 3; line search in Appendix A).  Test infrastructure only: columns
come from the C++ oracle's get_column, the subspace eigenproblem and the
(K+1)-dimensional pencil from LAPACK (numpy / scipy).

C holds n = K + 1 columns (one per state), stored by rows: C_j is the row of
determinant j.  B = H C, S = C^T C and Q = C^T H C (n x n).  One iteration:
1. i = argmax over the candidates of ||G_j||_inf with G = 4 B + 4 C S
   (candidates: the column of the previous coordinate plus that coordinate;
   ties to the smaller (beta, alpha) key).
2. With g = G_i, the step C <- C + eta e_i g minimises
   h(eta) = f(C + eta e_i g) - f(C) = w4 eta^4 + w3 eta^3 + w2 eta^2 + w1 eta,
       w1 = ||g||^2,
       w2 = 2 H_ii ||g||^2 + 2 (C_i . g)^2 + 2 ||C_i||^2 ||g||^2 + 2 g S g^T,
       w3 = 4 ||g||^2 (C_i . g),   w4 = ||g||^4
   (reading: the appendix prints w1 = 4 ||g||^2, but with G = 4B + 4CS the
   slope of h at 0 is <G, e_i g> = ||g||^2, which is also what the single
   state case reduces to; the other three coefficients are as printed).
   eta is the argmin of the monic quartic h / w4 by the Algorithm 1 rule.
3. S <- S + eta (C_i^T g + g^T C_i) + eta^2 g^T g,
   Q <- Q + eta (B_i^T g + g^T B_i) + eta^2 H_ii g^T g   (pre-step rows;
   the products are outer products, n x n),
   C_i <- C_i + eta g,
   B_j <- B_j + eta H_ji g over the column of i, with the compression rule
   per contribution row: update B_j iff C_j != 0 or |eta H_ji| ||g||_inf >= tau,
   then B_i = sum_j H_ji C_j recomputed.
4. Energies: the generalised eigenvalues of the pencil (Q, S), ascending;
   damped accumulator d of the step norm |eta| ||g||_2.
With n = 1 every step is the step of Algorithm 1 (eta g is its step in c_i).

Shift: the objective needs E_0 <= ... <= E_K < 0 (Sec. 2.3).  An optional
constant sigma replaces H by H - sigma I (every diagonal element, the
subspace matrix included); the eigenvectors are unchanged and the reported
energies add sigma back.

Initial C (Sec. 4.1.3, the excited-state solver): D_1 is the reference
determinant and D_2 .. D_n the determinants of lowest diagonal H_jj among
those connected to it (H_j,D1 != 0), each chosen from the ones not yet taken
(reading: equal H_jj ordered by the smaller (beta, alpha) key); column k of
C^(0) is the unit vector at D_k, B^(0) = H C^(0).  S and Q come from the
stored rows, and the first coordinate, which the paper leaves open, is the
argmax of ||G_j||_inf over every stored entry.
"""
import numpy as np
import scipy.linalg

from . import cd as cdmod
from . import fci


# relative window within which a followed pick counts as tying the maximum
FOLLOW_REL = 1e-13


def _order_key(k):
    return (k[1], k[0])


def initial_rows(h, eri, D0, n_states):
    """Keys D_1 .. D_n of the start and C^(0) restricted to them (the n x n
    identity)."""
    N = h.shape[0]
    ka, kb, v = cdmod.column(h, eri, *D0)
    d0 = (int(ka[0]), int(kb[0]))
    conn = [(int(x), int(y)) for x, y, z in zip(ka[1:], kb[1:], v[1:]) if z != 0.0]
    conn.sort(key=lambda k: (fci.diagonal(h, eri, N, k[0], k[1]), _order_key(k)))
    keys = [d0] + conn[: n_states - 1]
    if len(keys) < n_states:
        raise ValueError("fewer connected determinants than states")
    return keys, np.eye(n_states)


def w_coeffs(Ci, Bi, g, S, Hii):
    """Coefficients (w1, w2, w3, w4) of h(eta) = f(C + eta e_i g) - f(C)."""
    gg = float(g @ g)
    cg = float(Ci @ g)
    w1 = gg
    w2 = 2.0 * Hii * gg + 2.0 * cg * cg + 2.0 * float(Ci @ Ci) * gg + 2.0 * float(g @ S @ g)
    w3 = 4.0 * gg * cg
    w4 = gg * gg
    return w1, w2, w3, w4


def pencil_energies(Q, S):
    """Ascending generalised eigenvalues of (Q, S)."""
    return np.sort(scipy.linalg.eigh(Q, S, eigvals_only=True))


class XCDResult:
    pass


def xcdfci_run(h, eri, init_keys, C0, tau=0.0, max_steps=100, theta=0.9, dx_tol=0.0, shift=0.0, column=None,
               follow=None):
    """column (optional): key -> (alpha keys, beta keys, values) with the
    diagonal first, for Hamiltonians not given by integrals (h, eri unused).
    follow (optional): selections to take where the argmax is tied, i.e.
    where follow[step] has ||G||_inf within a relative FOLLOW_REL of the largest
    (another run's choice among equals); the first step where it is not is
    recorded in follow_failed."""
    n = C0.shape[1]
    colcache = {}

    def col(k):
        # column of H - shift I (the diagonal entry comes first)
        r = colcache.get(k)
        if r is None:
            ka, kb, v = column(k) if column is not None else cdmod.column(h, eri, k[0], k[1])
            r = [((int(x), int(y)), float(z) - (shift if e == 0 else 0.0))
                 for e, (x, y, z) in enumerate(zip(ka, kb, v))]
            colcache[k] = r
            if len(colcache) > 200000:
                colcache.clear()
        return r

    zero = np.zeros(n)
    C = {}
    B = {}
    for k, row in zip(init_keys, C0):
        C[k] = C.get(k, zero) + row
    for k, row in zip(init_keys, C0):
        for j, Hj in col(k):
            if Hj == 0.0:
                continue
            B[j] = B.get(j, zero) + Hj * row
            C.setdefault(j, zero.copy())
    keys0 = list(C.keys())
    Cm = np.array([C[k] for k in keys0], dtype=np.longdouble)
    Bm = np.array([B.get(k, zero) for k in keys0], dtype=np.longdouble)
    S = Cm.T @ Cm
    Q = Cm.T @ Bm

    def grad_row(k, S64):
        return 4.0 * B.get(k, zero) + 4.0 * C.get(k, zero) @ S64

    S64 = np.array(S, dtype=np.float64)
    # first coordinate: argmax over every stored entry
    cand = set(C.keys())
    energies, selections, gaps, etas, ginfs = [], [], [], [], []
    d = 0.0
    follow_failed = None
    for step in range(max_steps):
        S64 = np.array(S, dtype=np.float64)
        gn = {j: float(np.max(np.abs(grad_row(j, S64)))) for j in cand}
        order = sorted(cand, key=lambda j: (-gn[j], _order_key(j)))
        i = order[0]
        if follow is not None and step < len(follow) and follow_failed is None:
            # a pick of the device's is followed only where it ties the
            # maximum up to rounding (the values of both sides may differ in
            # their last bits): spin-flip images and lattice symmetries give
            # exact ties, anything farther apart is a different selection
            f = follow[step]
            if f in gn and gn[f] >= gn[i] * (1.0 - FOLLOW_REL):
                i = f
            else:
                follow_failed = step
        gaps.append((gn[order[0]] - gn[order[1]]) / gn[order[0]] if len(order) > 1 and gn[order[0]] > 0 else 1.0)
        Ci = C.get(i, zero).copy()
        Bi = B.get(i, zero).copy()
        g = 4.0 * Bi + 4.0 * Ci @ S64
        Hii = dict(col(i))[i]
        w1, w2, w3, w4 = w_coeffs(Ci, Bi, g, S64, Hii)
        eta = 0.0 if w4 == 0.0 else cdmod.line_search(w1 / w4, w2 / w4, w3 / w4)
        gL = g.astype(np.longdouble)
        CiL, BiL = Ci.astype(np.longdouble), Bi.astype(np.longdouble)
        etaL = np.longdouble(eta)
        S = S + etaL * (np.outer(CiL, gL) + np.outer(gL, CiL)) + etaL * etaL * np.outer(gL, gL)
        Q = Q + etaL * (np.outer(BiL, gL) + np.outer(gL, BiL)) + etaL * etaL * np.longdouble(Hii) * np.outer(gL, gL)
        C[i] = Ci + eta * g
        ginf = float(np.max(np.abs(g)))
        newcand = {i}
        for j, Hj in col(i):
            if Hj == 0.0 or j == i:
                continue
            newcand.add(j)
            cj = C.get(j)
            if (cj is not None and np.any(cj != 0.0)) or abs(eta * Hj) * ginf >= tau:
                B[j] = B.get(j, zero) + (eta * Hj) * g
                C.setdefault(j, zero.copy())
        B[i] = sum((Hj * C.get(j, zero) for j, Hj in col(i)), zero.copy())
        step_norm = abs(eta) * float(np.sqrt(g @ g))
        d = step_norm if step == 0 else theta * d + (1.0 - theta) * step_norm
        energies.append(shift + pencil_energies(np.array(Q, dtype=np.float64), np.array(S, dtype=np.float64)))
        selections.append(i)
        etas.append(eta)
        ginfs.append(ginf)
        cand = newcand
        if d < dx_tol:
            break
    r = XCDResult()
    r.follow_failed = follow_failed
    r.energies = np.array(energies)
    r.selections = selections
    r.gaps = np.array(gaps)
    r.eta = np.array(etas)
    r.ginf = np.array(ginfs)  # ||g||_inf of each step's row update
    r.S = np.array(S, dtype=np.float64)
    r.Q = np.array(Q, dtype=np.float64)
    r.C = C
    r.B = B
    r.steps = len(energies)
    return r
