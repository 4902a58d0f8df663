"""CPU oracle for the coordinate-descent FCI hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import, call, link or execute anything in this directory.  The product
path (the HIP library and its Python binding) never touches it.

Contents
--------
fci.py        determinant basis, Slater-Condon entries written out from the
              operator definition (Sec. 2.2, eq. (entry)), brute-force second
              quantization (eq. (general-ham)), dense / Lanczos ground states,
              spin-summed 1-/2-RDMs and the orbital-rotation gradient.
linesearch.py exact line search of the quartic h(eta) (Sec. 3.1, Appendix A).
mcdfci.py     serial multicoordinate descent (Alg. 2) with numpy/LAPACK for the
              (m+1)-dimensional eigenproblem.
xcdfci.py     serial coordinate descent for several states (Alg. 3).
hubbard_k.py  momentum-space Hubbard model (HubbardK) by operator application,
              the degenerate-subspace start.
optorb.py     OptOrbFCI outer loop (Alg. 4): rotated integrals, P4 and its
              gradient, polar factor, alternating Barzilai-Borwein steps.
cd_serial.cpp serial single-coordinate descent (Alg. 1), fp64 values with
              __float128 scalars mu, alpha; std::unordered_map storage.  Built
              into liboracle_cd.so by build.py and driven through cd.py.

Parity pins (tests/test_oracle_*.py) tie these to closed forms, LAPACK special
cases, brute force and the paper's printed Hubbard energies.
"""
