"""Seeded synthetic inputs shared by the oracle and the device path.

This module only draws random numbers and lays them out; it contains none of
the coordinate-descent method's arithmetic.  Both sides of every parity test
receive the same arrays from here.

Ab initio integrals: a symmetric one-body matrix h (orbital energies sorted in
[-20, 2] Ha on the diagonal, N(0, 0.1) couplings off it) and a chemist-notation
two-body tensor (pq|rs) = sum_L L^L_pq L^L_rs from a decaying symmetric factor
L.  The tensor is assembled once over canonical index pairs and mirrored so
that all eight index images are bitwise equal.

Hubbard: lattice specifications only (shape, t, U, electron counts); each side
builds its own hopping list from the shape.
"""
import numpy as np

__all__ = ["ab_initio", "hubbard_batch_specs", "random_dets", "CONFIG_SEEDS"]

# seeds used by the named workloads (recorded so runs are reproducible)
CONFIG_SEEDS = {"abinitio_n24": 2024, "abinitio_n36": 3636, "hubbard_batch": 256}


def _pair_index(N):
    idx = np.zeros((N, N), dtype=np.int64)
    k = 0
    for p in range(N):
        for q in range(p + 1):
            idx[p, q] = idx[q, p] = k
            k += 1
    return idx, k


def ab_initio(N, naux, seed):
    """Return (h, eri) as float64 arrays of shape (N, N) and (N, N, N, N).

    h_pp: Uniform(-20, 2) sorted ascending; h_pq = h_qp ~ N(0, 0.1) for p != q.
    L^L_pq = L^L_qp ~ N(0, 1) * exp(-|p - q| / 4) * 0.3 (drawn for p <= q).
    eri[p, q, r, s] = (pq|rs) = sum_L L^L_pq L^L_rs, bitwise 8-fold symmetric.
    """
    rng = np.random.default_rng(seed)
    h = np.zeros((N, N))
    h[np.diag_indices(N)] = np.sort(rng.uniform(-20.0, 2.0, size=N))
    off = rng.normal(0.0, 0.1, size=(N, N))
    iu = np.triu_indices(N, 1)
    h[iu] = off[iu]
    h[(iu[1], iu[0])] = off[iu]

    pidx, npair = _pair_index(N)
    P, Q = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    decay = np.exp(-np.abs(P - Q) / 4.0) * 0.3
    Ltri = np.zeros((naux, npair))
    for L in range(naux):
        g = rng.normal(0.0, 1.0, size=(N, N)) * decay
        for p in range(N):
            for q in range(p + 1):
                Ltri[L, pidx[p, q]] = g[q, p]  # draw for q <= p
    M = Ltri.T @ Ltri
    M = np.triu(M) + np.triu(M, 1).T  # bitwise symmetric in (pq) <-> (rs)
    eri = M[pidx[:, :, None, None], pidx[None, None, :, :]]
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)


SHAPES = [(2, 4), (3, 4), (4, 4), (2, 8), (3, 5)]


def hubbard_batch_specs(count, seed, shapes=SHAPES, umin=2.0, umax=10.0, t=1.0):
    """Specs for a batch of periodic Hubbard lattices at half filling.

    Each spec is a dict {dims, t, U, n_alpha, n_beta}; n_alpha = ceil(L/2),
    n_beta = floor(L/2) for L sites.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        dims = shapes[int(rng.integers(len(shapes)))]
        U = float(rng.uniform(umin, umax))
        L = int(np.prod(dims))
        out.append({"dims": tuple(dims), "t": t, "U": U,
                    "n_alpha": (L + 1) // 2, "n_beta": L // 2})
    return out


def random_dets(N, na, nb, count, seed):
    """`count` random (alpha, beta) occupation strings as uint64 arrays."""
    rng = np.random.default_rng(seed)
    a = np.zeros(count, dtype=np.uint64)
    b = np.zeros(count, dtype=np.uint64)
    for i in range(count):
        for arr, n in ((a, na), (b, nb)):
            occ = rng.choice(N, size=n, replace=False)
            v = 0
            for p in occ:
                v |= 1 << int(p)
            arr[i] = np.uint64(v)
    return a, b
