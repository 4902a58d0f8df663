"""MI355X-native coordinate-descent FCI (CDFCI) hot path.

The solver lives in the HIP library libcdfci.so (built from csrc/ for gfx950);
this package is its Python binding: `api` mirrors include/cdfci.h entry point
by entry point.  Importing the package does not load the library; the first
call does, and fails loudly if it has not been built.
"""
from .api import (Batch, live_objects, CDFCIError, Context, cdfci_batch_context, cdfci_batch_results, cdfci_batch_tables, cdfci_batch_trace,
                  cdfci_column, cdfci_column_noalloc, cdfci_energy, cdfci_entry, cdfci_export, cdfci_free, cdfci_free_batch,
                  cdfci_load, cdfci_mc_candidates, cdfci_mc_selection, cdfci_random_access_rates, cdfci_set_threshold, cdfci_set_timing, cdfci_mc_phase_times, cdfci_mc_select_stats, cdfci_step_search, cdfci_init, cdfci_init_hubbard, cdfci_init_hubbard_batch, cdfci_phase_times,
                  cdfci_rdm_backward, cdfci_step, cdfci_step_batch, cdfci_step_energies, cdfci_step_trace,
                  cdfci_strerror, cdfci_tune_batch, cdfci_tune_k, cdfci_workspace_size, cdfci_xenergies,
                  cdfci_xexport, cdfci_xfree, cdfci_xinit, cdfci_xinit_hubbard, cdfci_xinit_hubbard_k, cdfci_xmatrices, cdfci_xstep,
                  make_opts, make_rdm1, make_rdm12, read_fcidump, XContext, cdfci_optorb)

__all__ = ["Batch", "live_objects", "CDFCIError", "Context", "cdfci_batch_context", "cdfci_batch_results", "cdfci_batch_tables", "cdfci_batch_trace",
           "cdfci_column", "cdfci_column_noalloc", "cdfci_energy", "cdfci_entry", "cdfci_export", "cdfci_free", "cdfci_free_batch",
           "cdfci_load", "cdfci_mc_candidates", "cdfci_mc_selection", "cdfci_random_access_rates", "cdfci_set_threshold", "cdfci_set_timing", "cdfci_mc_phase_times", "cdfci_mc_select_stats", "cdfci_step_search", "cdfci_init", "cdfci_init_hubbard", "cdfci_init_hubbard_batch", "cdfci_phase_times",
           "cdfci_rdm_backward", "cdfci_step", "cdfci_step_batch", "cdfci_step_energies", "cdfci_step_trace",
           "cdfci_strerror", "cdfci_tune_batch", "cdfci_tune_k", "cdfci_workspace_size", "cdfci_xenergies",
           "cdfci_xexport", "cdfci_xfree", "cdfci_xinit", "cdfci_xinit_hubbard", "cdfci_xinit_hubbard_k", "cdfci_xmatrices", "cdfci_xstep",
           "make_opts", "make_rdm1", "make_rdm12", "read_fcidump", "XContext", "cdfci_optorb"]
