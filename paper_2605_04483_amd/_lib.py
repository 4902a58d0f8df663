"""ctypes declarations of the C ABI in include/cdfci.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdfci.so")

CDFCI_OK = 0
CDFCI_ERR_INVALID_ARG = -1
CDFCI_ERR_UNSUPPORTED = -2
CDFCI_ERR_TABLE_FULL = -3
CDFCI_ERR_NOT_NEGATIVE = -4
CDFCI_ERR_HIP = -5
CDFCI_ERR_BARRIER = -6
CDFCI_ERR_WORKSPACE = -7
CDFCI_ERR_NUMERIC = -8
CDFCI_ERR_INTERNAL = -9


class cdfci_opts(ctypes.Structure):
    _fields_ = [
        ("table_slots", ctypes.c_uint64),
        ("load_factor", ctypes.c_double),
        ("z_threshold", ctypes.c_double),
        ("dx_damping", ctypes.c_double),
        ("dx_threshold", ctypes.c_double),
        ("energy_shift", ctypes.c_double),
        ("init_kind", ctypes.c_int),
        ("grid_blocks", ctypes.c_int),
        ("block_threads", ctypes.c_int),
        ("reserved0", ctypes.c_int),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
    ]


class cdfci_stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64),
        ("total_steps", ctypes.c_int64),
        ("elements", ctypes.c_int64),
        ("inserts", ctypes.c_int64),
        ("probes", ctypes.c_int64),
        ("atomics", ctypes.c_int64),
        ("occupied", ctypes.c_uint64),
        ("max_probe", ctypes.c_int32),
        ("stopped", ctypes.c_int32),
        ("energy", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class cdfci_hubbard_spec(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int * 3),
        ("ndim", ctypes.c_int),
        ("n_alpha", ctypes.c_int),
        ("n_beta", ctypes.c_int),
        ("reserved", ctypes.c_int),
        ("t", ctypes.c_double),
        ("U", ctypes.c_double),
    ]


class cdfci_batch_opts(ctypes.Structure):
    _fields_ = [
        ("table_slots", ctypes.c_uint64),
        ("max_table_slots", ctypes.c_uint64),
        ("memory_budget", ctypes.c_uint64),
        ("load_factor", ctypes.c_double),
        ("z_threshold", ctypes.c_double),
        ("dx_damping", ctypes.c_double),
        ("dx_threshold", ctypes.c_double),
        ("chunk_steps", ctypes.c_int64),
        ("launches_per_graph", ctypes.c_int),
        ("waves", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class cdfci_batch_stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64),
        ("elements", ctypes.c_int64),
        ("running", ctypes.c_int32),
        ("stopped", ctypes.c_int32),
        ("failed", ctypes.c_int32),
        ("graph_replays", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("seconds", ctypes.c_double),
        ("peak_bytes", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class cdfci_optorb_opts(ctypes.Structure):
    _fields_ = [
        ("n_active", ctypes.c_int),
        ("max_outer", ctypes.c_int),
        ("max_inner", ctypes.c_int),
        ("k", ctypes.c_int),
        ("have_u", ctypes.c_int),
        ("reserved", ctypes.c_int),
        ("cd_steps", ctypes.c_int64),
        ("cd_dx_threshold", ctypes.c_double),
        ("energy_tol", ctypes.c_double),
        ("grad_tol", ctypes.c_double),
        ("step0", ctypes.c_double),
        ("z_threshold", ctypes.c_double),
        ("table_slots", ctypes.c_uint64),
        ("top_n", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
    ]


# (name, restype, argtypes) for every exported symbol of include/cdfci.h
_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_UP = ctypes.POINTER(ctypes.c_uint64)
_I64P = ctypes.POINTER(ctypes.c_int64)
_CTXP = ctypes.POINTER(ctypes.c_void_p)
_OPTP = ctypes.POINTER(cdfci_opts)
_STP = ctypes.POINTER(cdfci_stats)

SIGNATURES = [
    ("cdfci_workspace_size", ctypes.c_int,
     [ctypes.c_int, ctypes.c_int, ctypes.c_int, _OPTP, ctypes.POINTER(ctypes.c_size_t)]),
    ("cdfci_init", ctypes.c_int, [_DP, _DP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _OPTP, _CTXP]),
    ("cdfci_init_hubbard", ctypes.c_int,
     [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
      ctypes.c_int, _OPTP, _CTXP]),
    ("cdfci_step", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, _STP]),
    ("cdfci_step_trace", ctypes.c_int, [_P, ctypes.c_int64, _DP, _UP, _UP, _DP, _STP]),
    ("cdfci_step_energies", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, _DP, _STP]),
    ("cdfci_energy", ctypes.c_int, [_P, ctypes.c_int, _DP]),
    ("cdfci_rdm_backward", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int64, _DP, _DP, _DP, _DP]),
    ("cdfci_column", ctypes.c_int, [_P, _UP, _UP, _DP, ctypes.c_int64, _I64P]),
    ("cdfci_column_noalloc", ctypes.c_int, [_P, _UP, _UP, _DP, ctypes.c_int64, _I64P]),
    ("cdfci_entry", ctypes.c_int, [_P, _UP, _UP, _DP]),
    ("cdfci_export", ctypes.c_int, [_P, ctypes.c_int64, _UP, _DP, _DP, ctypes.c_int64, _I64P]),
    ("cdfci_phase_times", ctypes.c_int, [_P, _DP]),
    ("cdfci_load", ctypes.c_int, [_P, _UP, _DP, ctypes.c_int64]),
    ("cdfci_random_access_rates", ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, _DP]),
    ("cdfci_set_timing", ctypes.c_int, [_P, ctypes.c_int]),
    ("cdfci_mc_phase_times", ctypes.c_int, [_P, _DP, _I64P]),
    ("cdfci_mc_select_stats", ctypes.c_int, [_P, _I64P]),
    ("cdfci_mc_candidates", ctypes.c_int, [_P, _UP, _DP, _DP, _DP, ctypes.c_int64, _I64P, _DP]),
    ("cdfci_mc_selection", ctypes.c_int, [_P, _UP, _DP, ctypes.c_int64, _I64P]),
    ("cdfci_set_threshold", ctypes.c_int, [_P, ctypes.c_double]),
    ("cdfci_step_search", ctypes.c_int,
     [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double, _DP, _STP]),
    ("cdfci_free", ctypes.c_int, [_P]),
    ("cdfci_init_hubbard_batch", ctypes.c_int,
     [ctypes.POINTER(cdfci_hubbard_spec), ctypes.c_int, ctypes.POINTER(cdfci_batch_opts), _CTXP]),
    ("cdfci_step_batch", ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(cdfci_batch_stats)]),
    ("cdfci_batch_results", ctypes.c_int, [_P, _DP, _I64P, ctypes.POINTER(ctypes.c_int)]),
    ("cdfci_batch_trace", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, _DP, _UP, _UP]),
    ("cdfci_batch_context", ctypes.c_int, [_P, ctypes.c_int, _CTXP]),
    ("cdfci_free_batch", ctypes.c_int, [_P]),
    ("cdfci_tune_k", ctypes.c_int,
     [_P, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double, ctypes.c_int,
      ctypes.POINTER(ctypes.c_int), _DP]),
    ("cdfci_tune_batch", ctypes.c_int,
     [_P, _I64P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, _DP, ctypes.c_int, ctypes.c_int64,
      _I64P, ctypes.POINTER(ctypes.c_int), _DP]),
    ("cdfci_batch_tables", ctypes.c_int, [_P, _UP]),
    ("cdfci_xinit", ctypes.c_int,
     [_DP, _DP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _OPTP, _CTXP]),
    ("cdfci_xinit_hubbard", ctypes.c_int,
     [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
      ctypes.c_int, ctypes.c_int, ctypes.c_double, _OPTP, _CTXP]),
    ("cdfci_xinit_hubbard_k", ctypes.c_int,
     [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
      ctypes.c_int, ctypes.c_int, ctypes.c_double, _OPTP, _CTXP]),
    ("cdfci_xstep", ctypes.c_int, [_P, ctypes.c_int64, _DP, _UP, _UP, _STP]),
    ("cdfci_xenergies", ctypes.c_int, [_P, _DP]),
    ("cdfci_xmatrices", ctypes.c_int, [_P, _DP, _DP]),
    ("cdfci_xexport", ctypes.c_int, [_P, _UP, _DP, _DP, ctypes.c_int64, _I64P]),
    ("cdfci_xfree", ctypes.c_int, [_P]),
    ("cdfci_optorb", ctypes.c_int,
     [_DP, _DP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(cdfci_optorb_opts), _DP, _DP, _DP,
      ctypes.POINTER(ctypes.c_int)]),
    ("cdfci_read_fcidump", ctypes.c_int,
     [ctypes.c_char_p, ctypes.c_double, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
      ctypes.POINTER(ctypes.c_int), _DP, _DP, _DP]),
    ("cdfci_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("cdfci_last_error", ctypes.c_char_p, []),
]

_lib = None


def load():
    """Load libcdfci.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_2605_04483_amd/build.py "
                "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
