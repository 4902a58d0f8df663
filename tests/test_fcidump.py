"""FCIDUMP input (Sec. 4.1.1: molecular Hamiltonians are read from FCIDUMP
files, with an optional truncation threshold on the integrals).  Host code of
the library, so these run without a GPU.

Pins: the two-site Hubbard model written as a FCIDUMP (golden file, t = 1,
U = 4, one electron of each spin) has the closed-form ground energy
(U - sqrt(U^2 + 16 t^2)) / 2 (Sec. 2.2); synthetic integrals written out with
only their unique 8-fold images read back bit-exact."""
import os

import numpy as np
import pytest

import synth_inputs
from oracle import fci

import paper_2605_04483_amd as api

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hubbard_dimer.FCIDUMP")


def _write(path, h, eri, nelec, ms2, ecore, fortran=False, header_lines=1):
    N = h.shape[0]
    fmt = (lambda v: f"{v!r}".replace("e", "D")) if fortran else repr
    with open(path, "w") as f:
        if header_lines == 1:
            f.write(f"&FCI NORB={N},NELEC={nelec},MS2={ms2},ORBSYM={','.join(['1'] * N)},ISYM=1,/\n")
        else:
            f.write(f" &FCI NORB={N},\n  NELEC={nelec}, MS2={ms2},\n  ORBSYM={','.join(['1'] * N)},\n ISYM=1\n &END\n")
        for i in range(N):
            for j in range(i + 1):
                for k in range(N):
                    for l in range(k + 1):
                        if i * (i + 1) // 2 + j >= k * (k + 1) // 2 + l and eri[i, j, k, l] != 0.0:
                            f.write(f"{fmt(float(eri[i, j, k, l]))} {i + 1} {j + 1} {k + 1} {l + 1}\n")
        for i in range(N):
            for j in range(i + 1):
                if h[i, j] != 0.0:
                    f.write(f"{fmt(float(h[i, j]))} {i + 1} {j + 1} 0 0\n")
        for i in range(N):
            f.write(f"{fmt(-1.0 - i)} {i + 1} 0 0 0\n")  # orbital energies: ignored
        f.write(f"{fmt(float(ecore))} 0 0 0 0\n")


def test_golden_hubbard_dimer_closed_form():
    h, eri, na, nb, ecore = api.read_fcidump(GOLDEN)
    assert (na, nb, ecore) == (1, 1, 0.0)
    H, _ = fci.dense_H(h, eri, 2, na, nb)
    t, U = 1.0, 4.0
    assert abs(np.linalg.eigvalsh(H)[0] - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-14
    hh, ee = fci.hubbard_integrals((2,), t, U)
    assert np.array_equal(h, hh) and np.array_equal(eri, ee)


@pytest.mark.parametrize("fortran,header_lines,nelec,ms2", [(False, 1, 6, 0), (True, 4, 7, 1), (False, 4, 5, -3)])
def test_round_trip_is_bit_exact(tmp_path, fortran, header_lines, nelec, ms2):
    N = 6
    h, eri = synth_inputs.ab_initio(N, 18, 41)
    p = tmp_path / "x.FCIDUMP"
    _write(p, h, eri, nelec, ms2, 3.25, fortran, header_lines)
    h2, eri2, na, nb, ecore = api.read_fcidump(p)
    assert (na, nb) == ((nelec + ms2) // 2, (nelec - ms2) // 2)
    assert ecore == 3.25
    assert np.array_equal(h2, h)
    assert np.array_equal(eri2, eri)


def test_threshold_drops_small_integrals(tmp_path):
    N = 5
    h, eri = synth_inputs.ab_initio(N, 15, 42)
    p = tmp_path / "x.FCIDUMP"
    _write(p, h, eri, 4, 0, -1.5)
    tau = 1e-2
    h2, eri2, _, _, ecore = api.read_fcidump(p, threshold=tau)
    assert np.array_equal(h2, np.where(np.abs(h) < tau, 0.0, h))
    assert np.array_equal(eri2, np.where(np.abs(eri) < tau, 0.0, eri))
    assert ecore == -1.5
    assert np.count_nonzero(eri2) < np.count_nonzero(eri)


def test_malformed_inputs(tmp_path):
    with pytest.raises(api.CDFCIError):
        api.read_fcidump(tmp_path / "missing.FCIDUMP")
    bad = {
        "no_header": "1.0 1 1 1 1\n",
        "odd_spin": "&FCI NORB=2,NELEC=3,MS2=0 /\n",
        "index_range": "&FCI NORB=2,NELEC=2 /\n1.0 3 1 1 1\n",
        "short_line": "&FCI NORB=2,NELEC=2 /\n1.0 1 1\n",
        "too_many_electrons": "&FCI NORB=2,NELEC=6 /\n",
    }
    for name, text in bad.items():
        p = tmp_path / name
        p.write_text(text)
        with pytest.raises(api.CDFCIError) as e:
            api.read_fcidump(p)
        assert e.value.code == -1, name
    p = tmp_path / "big"
    p.write_text("&FCI NORB=64,NELEC=2 /\n")
    with pytest.raises(api.CDFCIError) as e:
        api.read_fcidump(p)
    assert e.value.code == -2
