"""Writes hubbard_batch256.txt: the oracle's ground-state energies of every
2x4 and 3x4 lattice of the seeded 256-lattice benchmark batch (periodic
Hubbard, t = 1, half filling, U ~ U[2, 10]).  Calls only the oracle: the
Hamiltonian is assembled from the oracle's get_column (hopping part once per
shape, the on-site part U * (number of doubly occupied sites) added per
instance) and its lowest eigenvalue taken by LAPACK (2x4, dimension 4900) or
ARPACK Lanczos (3x4, dimension 853,776) to a residual of 1e-13.

Usage: python tests/golden/make_hubbard_batch256.py  (a few minutes per 3x4)
"""
import os
import sys

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth_inputs  # noqa: E402
from oracle import cd as ocd  # noqa: E402
from oracle import fci  # noqa: E402


def hopping_and_double_occupancy(dims, na, nb):
    h, eri = fci.hubbard_integrals(dims, 1.0, 0.0)
    T, basis = ocd.sparse_H(h, eri, na, nb)
    docc = np.array([bin(a & b).count("1") for a, b in basis], dtype=np.float64)
    return T, docc


def main():
    specs = synth_inputs.hubbard_batch_specs(256, synth_inputs.CONFIG_SEEDS["hubbard_batch"])
    out = os.path.join(HERE, "hubbard_batch256.txt")
    cache = {}
    lines = ["# Oracle ground-state energies of the 2x4 and 3x4 lattices of the seeded 256-lattice batch",
             "# (synth_inputs.hubbard_batch_specs(256, seed 256)); written by make_hubbard_batch256.py",
             "# columns: index  dims  n_alpha  n_beta  U  E0"]
    for i, s in enumerate(specs):
        if s["dims"] not in ((2, 4), (3, 4)):
            continue
        key = (s["dims"], s["n_alpha"], s["n_beta"])
        if key not in cache:
            cache[key] = hopping_and_double_occupancy(*key)
        T, docc = cache[key]
        H = (T + sp.diags(s["U"] * docc)).tocsr()
        if H.shape[0] <= 5000:
            E0 = float(np.linalg.eigvalsh(H.toarray())[0])
        else:
            E0 = float(sla.eigsh(H, k=1, which="SA", tol=1e-13, return_eigenvectors=False)[0])
        dims = "x".join(str(d) for d in s["dims"])
        lines.append(f"{i} {dims} {s['n_alpha']} {s['n_beta']} {s['U']!r} {E0!r}")
        print(lines[-1], flush=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
