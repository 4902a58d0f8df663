"""Serial multicoordinate descent, mCDFCI (Sec. 3.2, Algorithm 2).  Test
infrastructure only; columns come from the C++ oracle's get_column and the
(m+1)-dimensional eigenproblem from LAPACK (numpy.linalg.eigh).

Per step, in the order Algorithm 2 lists:
1. I = the m candidates with the largest |4 b_i + 4 mu c_i| (ties: smaller
   (b, a) as an unsigned 128-bit number), candidates being the union of the
   previous step's columns (eq. (choose-I)).
2. With nu = ||c - E_I c_I|| and c~ = (c - E_I c_I)/nu, Q = [c~, E_I] has
   orthonormal columns and A = Q^T H Q is
       A_00 = (alpha - 2 c_I.b_I + c_I.H_II.c_I) / nu^2,
       A_0I = (b_I - H_II c_I) / nu,        A_II = H_II,
   formed from the maintained b and alpha.  The reduced problem
   min_z ||A + z z^T||_F^2 is solved by z = sqrt(-lambda) v for the lowest
   eigenpair (lambda, v) of A, with the sign fixed by z_0 >= 0.  From
   z = [nu gamma; gamma c_I + eta] (eq. (def-z)) follow gamma and eta.  If
   nu = 0 the c~ column is dropped, gamma = 1 and eta = z_I - c_I.
3. c <- gamma c + E_I eta;  b <- gamma b + H_{:,I} eta with the compression
   rule applied per contribution (update b_j if c_j != 0 or |eta_i H_ji| >= tau).
4. b_i = sum_j H_ji c_j recomputed for i in I.
5. mu <- gamma^2 mu + 2 gamma eta.c_I + eta.eta,
   alpha <- gamma^2 alpha + 2 gamma eta.b_I + eta.H_II.eta (pre-step c_I, b_I),
   energy alpha/mu, damped accumulator of ||eta||_2.
"""
import numpy as np

from . import cd as cdmod


def _order_key(k):
    return (k[1], k[0])


class MCDState:
    pass


def mcdfci_run(h, eri, init_keys, init_c, m, tau=0.0, max_steps=100, theta=0.9, dx_tol=0.0):
    colcache = {}

    def col(k):
        r = colcache.get(k)
        if r is None:
            ka, kb, v = cdmod.column(h, eri, k[0], k[1])
            r = [((int(x), int(y)), float(z)) for x, y, z in zip(ka, kb, v)]
            colcache[k] = r
            if len(colcache) > 200000:
                colcache.clear()
        return r

    c = {}
    b = {}
    for k, v in zip(init_keys, init_c):
        c[k] = c.get(k, 0.0) + float(v)
    cand = set()
    for k, v in zip(init_keys, init_c):
        for j, Hj in col(k):
            if Hj == 0.0:
                continue
            b[j] = b.get(j, 0.0) + float(v) * Hj
            cand.add(j)
    mu = sum(x * x for x in c.values())
    alpha = sum(c[k] * b.get(k, 0.0) for k in c)
    d = 0.0
    energies = []
    selections = []
    gaps = []
    etas = []
    gammas = []
    for step in range(max_steps):
        g = {j: abs(4.0 * b.get(j, 0.0) + 4.0 * mu * c.get(j, 0.0)) for j in cand}
        order = sorted(cand, key=lambda j: (-g[j], _order_key(j)))
        I = order[:m]
        # relative gap between the last chosen and the first left-out gradient
        if len(order) > m and g[order[m - 1]] > 0.0:
            gaps.append((g[order[m - 1]] - g[order[m]]) / g[order[m - 1]])
        else:
            gaps.append(1.0)
        mm = len(I)
        cI = np.array([c.get(i, 0.0) for i in I])
        bI = np.array([b.get(i, 0.0) for i in I])
        cols = [dict(col(i)) for i in I]
        HII = np.array([[cols[j].get(I[i], 0.0) for j in range(mm)] for i in range(mm)])
        Iset = set(I)
        nu2 = sum(v * v for k, v in c.items() if k not in Iset)
        nu = np.sqrt(nu2)
        if nu > 0.0:
            A = np.zeros((mm + 1, mm + 1))
            A[0, 0] = (alpha - 2.0 * cI @ bI + cI @ HII @ cI) / nu2
            A[0, 1:] = A[1:, 0] = (bI - HII @ cI) / nu
            A[1:, 1:] = HII
            w, V = np.linalg.eigh(A)
            lam, v = w[0], V[:, 0]
            if v[0] < 0:
                v = -v
            z = np.sqrt(max(-lam, 0.0)) * v
            gamma = z[0] / nu
            eta = z[1:] - gamma * cI
        else:
            w, V = np.linalg.eigh(HII)
            lam, v = w[0], V[:, 0]
            z = np.sqrt(max(-lam, 0.0)) * v
            if z @ cI < 0:
                z = -z
            gamma = 1.0
            eta = z - cI
        # update c and b
        for k in list(c.keys()):
            c[k] *= gamma
        for k in list(b.keys()):
            b[k] *= gamma
        for i, e in zip(I, eta):
            c[i] = c.get(i, 0.0) + e
        newcand = set(I)
        for idx, i in enumerate(I):
            for j, Hj in col(i):
                if Hj == 0.0:
                    continue
                newcand.add(j)
                delta = eta[idx] * Hj
                if c.get(j, 0.0) != 0.0 or abs(delta) >= tau:
                    b[j] = b.get(j, 0.0) + delta
        for i in I:
            b[i] = sum(Hj * c.get(j, 0.0) for j, Hj in col(i))
        mu = gamma * gamma * mu + 2.0 * gamma * (eta @ cI) + eta @ eta
        alpha = gamma * gamma * alpha + 2.0 * gamma * (eta @ bI) + eta @ HII @ eta
        nrm = float(np.linalg.norm(eta))
        d = nrm if step == 0 else theta * d + (1.0 - theta) * nrm
        energies.append(alpha / mu)
        selections.append(list(I))
        etas.append(np.array(eta, dtype=np.float64))
        gammas.append(float(gamma))
        cand = newcand
        if d < dx_tol:
            break
    st = MCDState()
    st.c, st.b, st.mu, st.alpha = c, b, mu, alpha
    st.energies = np.array(energies)
    st.selections = selections
    st.gaps = np.array(gaps)
    st.etas = etas        # per step: eta (aligned with selections)
    st.gammas = gammas    # per step: gamma
    st.energy = alpha / mu
    return st
