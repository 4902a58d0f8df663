"""The C-ABI library loads and exports every entry point include/cdfci.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

from paper_2605_04483_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "cdfci.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cdfci_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("cdfci_init", "cdfci_step", "cdfci_energy", "cdfci_rdm_backward", "cdfci_column",
                 "cdfci_entry", "cdfci_export", "cdfci_free", "cdfci_init_hubbard"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    for name in declared_symbols():
        assert hasattr(L, name), name
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert bound == set(declared_symbols())


def test_struct_layouts(tmp_path):
    """Every field of the ctypes mirrors sits at the offset the C compiler
    gives it in include/cdfci.h."""
    import subprocess

    structs = {"cdfci_opts": _lib.cdfci_opts, "cdfci_stats": _lib.cdfci_stats,
               "cdfci_hubbard_spec": _lib.cdfci_hubbard_spec, "cdfci_batch_opts": _lib.cdfci_batch_opts,
               "cdfci_batch_stats": _lib.cdfci_batch_stats, "cdfci_optorb_opts": _lib.cdfci_optorb_opts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cdfci.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        name, field, value = line.split()
        cls = structs[name]
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(value), (name, field, got, value)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())


def test_strerror_without_gpu():
    L = _lib.load()
    assert L.cdfci_strerror(-3).decode().startswith("hash table full")
    assert L.cdfci_strerror(0).decode() == "ok"


def test_every_declared_error_code_has_its_own_message():
    """Each CDFCI_ERR_* of include/cdfci.h is mirrored in the binding and
    has a message of its own (no code falls through to "unknown error")."""
    text = open(os.path.join(ROOT, "include", "cdfci.h")).read()
    codes = dict(re.findall(r"#define (CDFCI_ERR_[A-Z_]+) (-\d+)", text))
    assert len(codes) >= 9
    L = _lib.load()
    msgs = set()
    for name, value in codes.items():
        assert getattr(_lib, name) == int(value), name
        m = L.cdfci_strerror(int(value)).decode()
        assert m != "unknown error", name
        msgs.add(m)
    assert len(msgs) == len(codes)


def test_host_side_argument_errors_without_gpu():
    """Argument checks that return before any device call."""
    L = _lib.load()
    ctx = ctypes.c_void_p()
    opts = _lib.cdfci_opts()
    # too many orbitals -> UNSUPPORTED before touching the device
    h = (ctypes.c_double * 1)()
    rc = L.cdfci_init(h, h, 64, 1, 1, ctypes.byref(opts), ctypes.byref(ctx))
    assert rc == _lib.CDFCI_ERR_UNSUPPORTED
    rc = L.cdfci_init(None, None, 4, 1, 1, ctypes.byref(opts), ctypes.byref(ctx))
    assert rc == _lib.CDFCI_ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert L.cdfci_workspace_size(24, 6, 6, ctypes.byref(opts), ctypes.byref(n)) == 0
    assert n.value == (1 << 22) * 32


def test_batch_argument_errors_without_gpu():
    """Every Hubbard spec is checked before the batch touches the device."""
    L = _lib.load()
    out = ctypes.c_void_p()
    opts = _lib.cdfci_batch_opts()
    sp = (_lib.cdfci_hubbard_spec * 2)()
    for s, dims in zip(sp, ((2, 4, 1), (8, 8, 1))):
        s.dims[:] = list(dims)
        s.ndim = 2
        s.n_alpha, s.n_beta, s.t, s.U = 4, 4, 1.0, 4.0
    assert L.cdfci_init_hubbard_batch(sp, 2, ctypes.byref(opts), ctypes.byref(out)) == _lib.CDFCI_ERR_UNSUPPORTED
    assert L.cdfci_init_hubbard_batch(sp, 0, ctypes.byref(opts), ctypes.byref(out)) == _lib.CDFCI_ERR_INVALID_ARG
    sp[1].dims[:] = [2, 4, 1]
    sp[1].ndim = 0
    assert L.cdfci_init_hubbard_batch(sp, 2, ctypes.byref(opts), ctypes.byref(out)) == _lib.CDFCI_ERR_INVALID_ARG
    sp[1].ndim = 2
    sp[1].n_alpha = 9
    assert L.cdfci_init_hubbard_batch(sp, 2, ctypes.byref(opts), ctypes.byref(out)) == _lib.CDFCI_ERR_UNSUPPORTED
    assert not out.value
