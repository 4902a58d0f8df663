"""OptOrbFCI: orbital optimisation around FCI (Sec. 3.4, eq. (subopt),
Algorithm 4).  Test infrastructure only.

Given integrals h, (pq|rs) over M orbitals, the N orbitals of the FCI space
are the columns of U (M x N, U^T U = I).  Outer iteration l:
1. integrals in the current orbitals: h' = U^T h U and the four-index
   transform of (pq|rs);
2. the FCI ground state in them (here LAPACK on the dense matrix) and its
   energy E^(l);
3. its spin-summed RDMs gamma, Gamma (chemist order, E = sum h' gamma +
   1/2 sum (pq|rs)' Gamma, as in the reverse pass);
4. the orbital problem (subopt) with the RDMs held fixed,
       P4(U) = sum h_pq U_pp' U_qq' gamma_p'q'
               + 1/2 sum (pq|rs) U_pp' U_qq' U_rr' U_ss' Gamma_p'q'r's',
   by projected gradient steps U <- orth(U - t_k grad P4(U)) (eq. (projBB))
   with Barzilai-Borwein step sizes alternating between their two forms.

Readings (the paper gives the method, not these constants):
* orth(X) is the polar factor X (X^T X)^(-1/2), the matrix with orthonormal
  columns nearest to X;
* grad P4 is the Euclidean gradient in U; s = U_k - U_(k-1),
  y = grad_k - grad_(k-1); t_k = <s,s>/|<s,y>| for odd k, |<s,y>|/<y,y> for
  even k, t_0 = step0 (also whenever <s,y> = 0);
* the orbital problem stops when the Riemannian gradient
  grad - U sym(U^T grad) has Frobenius norm <= grad_tol or after max_inner
  steps, and returns its iterate of lowest P4 (so that E^(l+1) <= P4(U^(l+1))
  <= P4(U^(l)) = E^(l): the FCI energy in the new orbitals is at most that of
  the old wavefunction carried over);
* the outer loop stops when |E^(l) - E^(l-1)| <= energy_tol or after
  max_outer solves;
* U^(0) = the identity columns of the N orbitals of lowest h_pp (ties: the
  lower index).
"""
import numpy as np

from . import fci


def transform(eri, U, positions=(0, 1, 2, 3)):
    """Contract the given index positions of eri with U (one at a time)."""
    out = eri
    for pos in positions:
        out = np.moveaxis(np.tensordot(out, U, axes=([pos], [0])), -1, pos)
    return out


def rotated(h, eri, U):
    return U.T @ h @ U, transform(eri, U)


def p4(h, eri, U, g1, g2):
    """P4(U) of eq. (subopt) with the RDMs fixed."""
    h2, e2 = rotated(h, eri, U)
    return float(np.sum(h2 * g1) + 0.5 * np.sum(e2 * g2))


def p4_grad(h, eri, U, g1, g2):
    """Euclidean gradient of P4 in U: the one-body term twice (h and gamma
    symmetric), the two-body term summed over the four positions U enters."""
    g = h @ U @ (g1 + g1.T)
    for pos in range(4):
        others = [q for q in range(4) if q != pos]
        W = transform(eri, U, others)  # every index but `pos` rotated
        # contract W over the three rotated indices with Gamma's matching ones
        g = g + 0.5 * np.tensordot(np.moveaxis(W, pos, 0), np.moveaxis(g2, pos, 0),
                                   axes=([1, 2, 3], [1, 2, 3]))
    return g


def orth(X):
    w, V = np.linalg.eigh(X.T @ X)
    return X @ (V @ np.diag(w ** -0.5) @ V.T)


def riemannian(U, G):
    S = U.T @ G
    return G - U @ (0.5 * (S + S.T))


def initial_u(h, N):
    M = h.shape[0]
    order = sorted(range(M), key=lambda p: (h[p, p], p))[:N]
    U = np.zeros((M, N))
    for j, p in enumerate(sorted(order)):
        U[p, j] = 1.0
    return U


def solve_orbitals(h, eri, U, g1, g2, max_inner=100, grad_tol=1e-8, step0=1e-2):
    best, best_val = U, p4(h, eri, U, g1, g2)
    G = p4_grad(h, eri, U, g1, g2)
    U_prev = G_prev = None
    for k in range(max_inner):
        if np.linalg.norm(riemannian(U, G)) <= grad_tol:
            break
        t = step0
        if U_prev is not None:
            s, y = U - U_prev, G - G_prev
            sy = abs(float(np.sum(s * y)))
            if sy > 0.0:
                t = float(np.sum(s * s)) / sy if k % 2 == 1 else sy / float(np.sum(y * y))
        U_prev, G_prev = U, G
        U = orth(U - t * G)
        G = p4_grad(h, eri, U, g1, g2)
        val = p4(h, eri, U, g1, g2)
        if val < best_val:
            best, best_val = U, val
    return best, best_val


def optorb(h, eri, N, na, nb, U0=None, max_outer=20, max_inner=100, energy_tol=1e-8, grad_tol=1e-8,
           step0=1e-2):
    """Returns (energies E^(l), final U, P4 values of the orbital problems)."""
    U = initial_u(h, N) if U0 is None else np.array(U0, dtype=np.float64)
    energies, p4s = [], []
    for l in range(max_outer):
        h2, e2 = rotated(h, eri, U)
        E, v, basis = fci.ground_state_dense(h2, e2, N, na, nb)
        energies.append(float(E))
        if l > 0 and abs(energies[-1] - energies[-2]) <= energy_tol:
            break
        if l == max_outer - 1:
            break
        g1, g2 = fci.rdm12(basis, v, N)
        U, val = solve_orbitals(h, eri, U, g1, g2, max_inner, grad_tol, step0)
        p4s.append(val)
    return np.array(energies), U, np.array(p4s)
