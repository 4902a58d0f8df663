"""Exact line search of CDFCI (Sec. 3.1, eq. (choose-alpha); Appendix A).

Test infrastructure only.  h(eta) = f(c + eta e_i) - f(c)
                                  = eta^4 + v3 eta^3 + v2 eta^2 + v1 eta
with v3 = 4 c_i, v2 = 2 H_ii + 4 c_i^2 + 2 mu, v1 = 4 b_i + 4 mu c_i.
The minimiser is, by definition, the critical point (real root of the cubic
h'(eta) = 4 eta^3 + 3 v3 eta^2 + 2 v2 eta + v1) with the smallest h; ties go
to the smaller |eta|.
"""
import numpy as np


def quartic_coeffs(c_i, b_i, H_ii, mu):
    return 4.0 * c_i, 2.0 * H_ii + 4.0 * c_i * c_i + 2.0 * mu, 4.0 * b_i + 4.0 * mu * c_i


def h_of(eta, v1, v2, v3):
    return eta**4 + v3 * eta**3 + v2 * eta**2 + v1 * eta


def argmin_quartic(v1, v2, v3, newton_iters=8):
    roots = np.roots([4.0, 3.0 * v3, 2.0 * v2, v1])
    cands = []
    for r in roots:
        if abs(r.imag) <= 1e-7 * max(1.0, abs(r.real)):
            x = float(r.real)
            for _ in range(newton_iters):  # polish on the cubic
                f = 4 * x**3 + 3 * v3 * x**2 + 2 * v2 * x + v1
                fp = 12 * x**2 + 6 * v3 * x + 2 * v2
                if fp == 0.0:
                    break
                dx = f / fp
                x -= dx
                if abs(dx) <= 1e-16 * max(abs(x), 1e-300):
                    break
            cands.append(x)
    best = None
    for x in cands:
        key = (h_of(x, v1, v2, v3), abs(x))
        if best is None or key < best[0]:
            best = (key, x)
    return best[1]
