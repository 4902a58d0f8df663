/*
 * cdfci.h -- C ABI of the MI355X (gfx950) coordinate-descent FCI library.
 *
 * The library minimises f(c) = ||H + c c^T||_F^2 over the coefficients of a
 * sparse determinant expansion (paper Sec. 2.3, eq. (optimization)); its
 * minimisers are +-sqrt(-E0) v0 for the lowest eigenpair of H when E0 < 0.
 * H is the second-quantised Hamiltonian of eq. (general-ham), given by a
 * one-body matrix h and chemist two-body integrals (pq|rs), or by a periodic
 * Hubbard lattice (Sec. 2.2).  The coefficient vector c and the residual
 * b = H c are held together in a device-resident open-addressing hash table
 * keyed by 128-bit determinants.
 *
 * Determinant keys: a pair of 64-bit occupation strings {alpha, beta}; bit p
 * of the alpha word set means spatial orbital (or site) p holds a spin-up
 * electron.  Spin-orbital order for fermionic phases is all alpha orbitals
 * then all beta orbitals, each ascending; at most 63 spatial orbitals.
 *
 * Conventions for every entry point:
 *   - return value 0 = success, negative = CDFCI_ERR_* (never an exception);
 *     cdfci_strerror() gives text, cdfci_last_error() the last HIP message;
 *   - pointers are host pointers unless said otherwise; the library copies
 *     what it needs and never keeps a caller pointer past the call;
 *   - one context belongs to one HIP stream and is not re-entrant: calls on
 *     the same context must not overlap.
 */
#ifndef CDFCI_H
#define CDFCI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define CDFCI_OK 0
#define CDFCI_ERR_INVALID_ARG -1   /* bad sizes / null pointers / state */
#define CDFCI_ERR_UNSUPPORTED -2   /* N > 63, n > N, or a mode not built */
#define CDFCI_ERR_TABLE_FULL -3    /* hash table passed its occupancy limit (Sec. 4.1.2) */
#define CDFCI_ERR_NOT_NEGATIVE -4  /* starting energy >= 0: f has no nonzero minimiser (Sec. 2.3) */
#define CDFCI_ERR_HIP -5           /* a HIP runtime call failed */
#define CDFCI_ERR_BARRIER -6       /* a device-wide barrier exceeded its spin limit */
#define CDFCI_ERR_WORKSPACE -7     /* caller workspace too small */
#define CDFCI_ERR_NUMERIC -8       /* a multicoordinate step produced a non-finite value */
#define CDFCI_ERR_INTERNAL -9      /* an internal consistency check failed (cdfci_last_error says which) */

typedef struct cdfci_ctx cdfci_ctx; /* opaque, library-owned */

/* Options.  A zero-initialised struct gives the defaults noted per field. */
typedef struct {
  uint64_t table_slots;  /* hash slots (power of two); 0 = 2^22 */
  double load_factor;    /* max stored entries / slots before TABLE_FULL; 0 = 0.79 (Sec. 4.3) */
  double z_threshold;    /* compression threshold tau on b updates (Sec. 3.1); default 0 */
  double dx_damping;     /* theta of the damped step accumulator (Sec. 4.1.3); 0 = 0.9 */
  double dx_threshold;   /* stop when the accumulator falls below this; 0 = never */
  double energy_shift;   /* sigma: the solver minimises f for H - sigma I, which needs a
                            negative lowest eigenvalue (Sec. 2.3, eq. (optimization)); every
                            reported energy adds sigma back, the stored b is (H - sigma I) c
                            and alpha = c^T (H - sigma I) c; 0 = no shift */
  int init_kind;         /* c^(0): 0 = model default (1 for integrals, 2 for lattices);
                            1 = lowest-h_pp (aufbau) determinant with c = sqrt(-H_00);
                            2 = Neel determinant + sqrt(-lambda) times the lowest eigenvector
                            of H on it and the nonzero entries of its column */
  int grid_blocks;       /* workgroups of the single-coordinate persistent kernel; 0 = auto */
  int block_threads;     /* threads per workgroup of the single-coordinate kernel (64..256,
                            multiple of 64); 0 = 128 when the column gives every lane one
                            entry with one workgroup per compute unit, else 256 */
  int reserved0;
  void* workspace;          /* optional caller-owned device memory for the hash table and
                               buffers (e.g. a torch tensor); NULL = library allocates */
  size_t workspace_bytes;   /* size of `workspace` */
  void* stream;             /* hipStream_t to enqueue on; NULL = default stream */
} cdfci_opts;

/* Per-call statistics (Sec. 4.1.3 report quantities). */
typedef struct {
  int64_t steps;          /* coordinate-descent iterations done by this call */
  int64_t total_steps;    /* iterations since init */
  int64_t elements;       /* Hamiltonian entries enumerated (zeros included) */
  int64_t inserts;        /* new determinants stored */
  int64_t probes;         /* table slots inspected by the column scatters of k > 1 steps */
  int64_t atomics;        /* FP64 atomic b updates issued by those scatters */
  uint64_t occupied;      /* determinants in the table */
  int32_t max_probe;      /* longest probe sequence seen */
  int32_t stopped;        /* 1 if the damped accumulator fell below dx_threshold */
  double energy;          /* alpha / mu after the call */
  double dx;              /* damped accumulator d */
  double mu, alpha;       /* c^T c and c^T H c (maintained) */
  double seconds;         /* device time of the call */
} cdfci_stats;

/* Device bytes the context needs for the given sizes and options. */
int cdfci_workspace_size(int n_orb, int n_alpha, int n_beta, const cdfci_opts* opts, size_t* bytes);

/* Create a context for an integral Hamiltonian (Sec. 2.2 eq. (general-ham),
 * Sec. 4.1.1 HamiltonianMolecule).  h: n_orb*n_orb row-major, symmetric.
 * eri: n_orb^4 row-major chemist (pq|rs), eri[((p*N+q)*N+r)*N+s], with the
 * 8-fold permutational symmetry.  Each may be a host or a device pointer (an
 * exception to the host-pointer convention); both are copied, the caller
 * keeps ownership.  Builds c^(0) per opts->init_kind and b^(0) = H c^(0)
 * exactly (Alg. 1).  opts->energy_shift sigma is applied as h - (sigma / n) I
 * with n = n_alpha + n_beta, which on the n-electron space is H - sigma I;
 * CDFCI_ERR_NOT_NEGATIVE if the start still has no negative energy. */
int cdfci_init(const double* h, const double* eri, int n_orb, int n_alpha, int n_beta,
               const cdfci_opts* opts, cdfci_ctx** out);

/* Create a context for a periodic Hubbard lattice (Sec. 2.2): dims[0..ndim)
 * sites per direction (row-major site index), hopping -t on each distinct
 * nearest-neighbour pair (a direction of length 2 gives one bond), on-site
 * repulsion U. */
int cdfci_init_hubbard(const int* dims, int ndim, double t, double U, int n_alpha, int n_beta,
                       const cdfci_opts* opts, cdfci_ctx** out);

/* Run up to nsteps iterations and stop early if the damped step accumulator
 * drops below dx_threshold (Sec. 4.1.3).  k == 1: single-coordinate descent
 * (Alg. 1, Sec. 3.1).  1 < k <= 1024: multicoordinate descent (Alg. 2,
 * Sec. 3.2): the k candidates of largest |4 b_i + 4 mu c_i| from the previous
 * step's columns, the step (gamma, eta) from the lowest eigenpair of the
 * (k+1)-dimensional Q^T H Q, c <- gamma c + E_I eta, b <- gamma b + H_{:,I} eta.
 * Steps with different k may be mixed on one context.  k > 1 needs
 * table_slots <= 2^31 (candidate lists hold 32-bit slot ids), else
 * CDFCI_ERR_UNSUPPORTED.  Enqueued on the context's stream; returns after
 * completion.  out may be NULL. */
int cdfci_step(cdfci_ctx* ctx, int k, int64_t nsteps, cdfci_stats* out);

/* Like cdfci_step and also records the energy alpha/mu after every iteration
 * into energy (host, length nsteps). */
int cdfci_step_energies(cdfci_ctx* ctx, int k, int64_t nsteps, double* energy, cdfci_stats* out);

/* Like cdfci_step (k == 1 only) and also records, per iteration, the energy,
 * the chosen determinant and the step size into host arrays of length nsteps
 * (any may be NULL).  For parity tests. */
int cdfci_step_trace(cdfci_ctx* ctx, int64_t nsteps, double* energy, uint64_t* sel_alpha,
                     uint64_t* sel_beta, double* eta, cdfci_stats* out);

/* Energy estimate.  exact = 0: the maintained Rayleigh quotient alpha/mu
 * (get_variational_energy, Sec. 4.1.2).  exact = 1: recomputed
 * c^T H c / c^T c by applying H to the stored c on the device. */
int cdfci_energy(cdfci_ctx* ctx, int exact, double* energy);

/* Reverse pass of E = c^T H c / c^T c with c held fixed, the energy of the
 * variational objective of Sec. 3.4 eq. (subopt) at U = I, whose 1- and 2-RDMs
 * feed the orbital optimisation (Alg. 4).  The wavefunction is the top_n
 * stored determinants by |c| (equal |c| ordered by the smaller key; top_n <= 0
 * or above the count: every entry with c != 0), normalised.  Outputs, host,
 * any may be NULL:
 *   energy[0]    = sum h gamma + 1/2 sum (pq|rs) Gamma, energy[1] = the same
 *                  quotient evaluated directly from Hamiltonian entries;
 *   dh[p*N+q]    = grad_E * gamma_pq,  gamma_pq = sum_s <a+_ps a_qs>;
 *   deri[pqrs]   = grad_E * Gamma_pqrs / 2 (N^4 doubles),
 *                  Gamma_pqrs = sum_st <a+_ps a+_rt a_st a_qs> (chemist order);
 *   kappa[p*N+q] = grad_E * 2 (F_pq - F_qp), F_pq = sum_r h_pr gamma_rq
 *                  + sum_rst (pr|st) Gamma_qrst: the derivative of E(h', eri')
 *                  with h' = U^T h U, U = exp(K), K = -K^T, in K_pq (p > q).
 * gamma and Gamma are the derivatives of E in each tensor element (the
 * symmetric images of one integral each get their own share).  c is not
 * changed.  CDFCI_ERR_INVALID_ARG if no stored c is nonzero;
 * CDFCI_ERR_UNSUPPORTED if more than 4096 entries share the |c| at the top_n
 * boundary.  Device memory used: two N^4 arrays plus a table of the support. */
int cdfci_rdm_backward(cdfci_ctx* ctx, double grad_E, int64_t top_n, double* energy, double* dh,
                       double* deri, double* kappa);

/* get_column (Sec. 4.1.1): every (D', H_{D',D}) for D' = D and all single and
 * double excitations of D, in the library's enumeration order with the
 * diagonal first and exact zeros kept.  keys: 2*cap uint64 (alpha, beta
 * interleaved), vals: cap doubles.  *count = number of entries; if it
 * exceeds cap nothing is written and CDFCI_ERR_INVALID_ARG is returned. */
int cdfci_column(cdfci_ctx* ctx, const uint64_t key[2], uint64_t* keys, double* vals, int64_t cap,
                 int64_t* count);

/* get_column for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result as cdfci_column, staged through a fixed device array of the
 * library instead of per-call buffers, so the call makes no hipMalloc,
 * hipFree or other allocating call.  keys (2*cap uint64) and vals (cap
 * doubles) may be host or device pointers.  Limit: columns of at most
 * 262144 entries (6 MiB of staging per GPU, held until the process ends);
 * a larger column gives CDFCI_ERR_UNSUPPORTED with *count set.  Every call on
 * one GPU shares that staging array: calls that overlap on one GPU (other
 * contexts or threads) race and must be serialised by the caller. */
int cdfci_column_noalloc(cdfci_ctx* ctx, const uint64_t key[2], uint64_t* keys, double* vals, int64_t cap,
                         int64_t* count);

/* get_entry (Sec. 4.1.1): H_{k1,k2} by the Slater-Condon rules, eq. (entry). */
int cdfci_entry(cdfci_ctx* ctx, const uint64_t k1[2], const uint64_t k2[2], double* value);

/* Copy the stored determinants out: keys 2*cap uint64 (alpha, beta), c and b
 * values (true scale).  top_n > 0 keeps the top_n by |c| among the entries
 * with c != 0, chosen as cdfci_rdm_backward chooses its support (in no
 * particular order); top_n <= 0 keeps every stored entry.  *count = entries
 * available; at most cap are written. */
int cdfci_export(cdfci_ctx* ctx, int64_t top_n, uint64_t* keys, double* c, double* b, int64_t cap,
                 int64_t* count);

/* Profiling aid: device seconds that workgroup 0 of the single-coordinate
 * kernel has spent, since init, in its four phases: [0] choose-and-step
 * (H_DD, line search), [1] column scatter, [2] waiting at the device-wide
 * barrier, [3] combining the partial results.  seconds: 4 doubles.  The
 * timers are compiled into the kernel only with -DCDFCI_PHASE_TIMING;
 * otherwise CDFCI_ERR_UNSUPPORTED. */
int cdfci_phase_times(cdfci_ctx* ctx, double* seconds);

/* Inspection of the multicoordinate step (Alg. 2, eq. (choose-I)), for
 * parity tests.  Both need the context to be in the multicoordinate state
 * (its last step had k > 1), else CDFCI_ERR_INVALID_ARG.
 *
 * cdfci_mc_candidates: the candidates the next k > 1 step chooses from (the
 * stored determinants of the last step's columns and its chosen set, each
 * once), in no particular order.  keys 2*cap uint64 (alpha, beta); g, cv, bv
 * cap doubles each: the selection key |4 b^ + 4 mu c^| exactly as the
 * selection forms it, and the stored c^ and b^, where c = s c^ and b = s b^
 * with the lazy scale s of the multicoordinate state; mu_scale[0] = mu,
 * mu_scale[1] = s.  Any output may be NULL; *count = candidates, at most cap
 * written.  The state is not changed.
 *
 * cdfci_mc_selection: the chosen set of the last k > 1 step (in the
 * selection's internal order) and its step eta (true scale): keys 2*cap
 * uint64, eta cap doubles (may be NULL); *count = its size. */
int cdfci_mc_candidates(cdfci_ctx* ctx, uint64_t* keys, double* g, double* cv, double* bv, int64_t cap,
                        int64_t* count, double* mu_scale);
int cdfci_mc_selection(cdfci_ctx* ctx, uint64_t* keys, double* eta, int64_t cap, int64_t* count);

/* Measurement aid: the rates of the memory operations a column scatter is
 * made of, each alone over uniformly random slots of a table of table_slots
 * 32-byte slots (allocated for the call, on the current device), n_ops
 * operations per run, best of three timed runs: rates[0] 16-byte key
 * gathers/s, rates[1] gather + plain 8-byte read-modify-write/s, rates[2]
 * gather + agent-scope FP64 atomic add/s, rates[3] returning 32-bit atomic
 * ORs into a one-bit-per-slot bitmap/s, rates[4] bytes/s of a 1 GiB device
 * copy (read + write).  These are the ceilings the hash probes and atomics
 * of the solver are compared with. */
int cdfci_random_access_rates(uint64_t table_slots, int64_t n_ops, double* rates);

/* Measurement aid: with timing on (cdfci_set_timing; switching it resets the
 * sums), every multicoordinate step records HIP events on the context's
 * stream between its phases, and cdfci_mc_phase_times returns the summed
 * device seconds of [0] selection (begin, radix passes, gather), [1] H_II,
 * [2] the launch of the reduced eigenproblem, whose other workgroups run the
 * probe half of the column scatter, [3] the apply half of the scatter, [4]
 * finish and rescale, [5] the probe half alone (from its first
 * workgroup's start to its last one's end, device wall clock) and [6] the
 * reduced problem's workgroup alone (device wall clock) (7 doubles), and in
 * *steps (may be NULL) the steps timed. */
int cdfci_set_timing(cdfci_ctx* ctx, int on);
int cdfci_mc_phase_times(cdfci_ctx* ctx, double* seconds, int64_t* steps);

/* Measurement aid: running totals of the multicoordinate selections since
 * the context's multicoordinate state was created (4 int64, host): [0]
 * selections, [1] candidate positions holding a slot (a determinant reached
 * from several chosen columns counted once per column), [2] distinct slots
 * ranked exactly (those whose key is at least the bound the repeats allow),
 * [3] selections whose bound held fewer than k distinct determinants
 * (never expected; such a selection stops the run with CDFCI_ERR_INTERNAL).
 * Reads device state (synchronises the context's stream).  CDFCI_ERR_INVALID_ARG before
 * the first k > 1 step. */
int cdfci_mc_select_stats(cdfci_ctx* ctx, int64_t* counts);

/* Restart (Sec. 4.1.3: checkpoints for termination and restart from stored
 * wavefunctions).  Replaces the context's state by the wavefunction
 * c = sum_i cv[i] e_{key i}: keys 2*count uint64 (alpha, beta) and cv count
 * doubles, host, as cdfci_export writes them (entries with c = 0 may be
 * left out).  The table is cleared, the entries stored, and b = H c rebuilt:
 * the stored set is the given entries plus every determinant j with some
 * |H_ji c_i| >= z_threshold (every connected one when it is 0), and each
 * stored b_j is the full sum over the given entries.  mu = c.c and
 * alpha = c.b are recomputed in double-double, the iteration count and the
 * damped accumulator restart from zero, and the first coordinate is the
 * stored entry of largest |4 b_j + 4 mu c_j| (as after init).  A context
 * left by CDFCI_ERR_TABLE_FULL may be reloaded.  CDFCI_ERR_INVALID_ARG for a
 * key outside the context's orbitals or electron counts, a repeated key, a
 * non-finite coefficient or an all-zero c; CDFCI_ERR_TABLE_FULL if the set
 * does not fit. */
int cdfci_load(cdfci_ctx* ctx, const uint64_t* keys, const double* cv, int64_t count);

/* Set the compression threshold tau of later steps and loads (Sec. 3.1). */
int cdfci_set_threshold(cdfci_ctx* ctx, double tau);

/* Single-coordinate iterations within a memory budget (the z_threshold_search
 * option of the paper's solver input, Sec. 4.3).  Steps run in chunks of
 * `chunk` iterations, fewer if needed so that one chunk cannot add more than
 * the (1 - fill) share of the limit (an iteration stores at most one column);
 * when the stored entries exceed fill * load_factor * table_slots after a
 * chunk, the entries with c != 0 are kept, tau becomes
 * tau0 (if it was 0) or tau * growth, and the state is rebuilt from them by
 * cdfci_load, raising tau again until the rebuilt set fits.  Stops after
 * nsteps iterations or at dx_threshold.  *tau_out (may be NULL) gets the final
 * tau; out (may be NULL) sums steps, elements, inserts and seconds over the
 * call, the other fields are those after the last chunk.  fill in (0, 1],
 * growth > 1, tau0 > 0; CDFCI_ERR_TABLE_FULL if even tau > 1e3 leaves too
 * many entries. */
int cdfci_step_search(cdfci_ctx* ctx, int64_t nsteps, int64_t chunk, double fill, double growth, double tau0,
                      double* tau_out, cdfci_stats* out);

int cdfci_free(cdfci_ctx* ctx);

/* ---- Batches of periodic Hubbard lattices (Sec. 2.2, Alg. 1) ----------------
 * Many independent instances of uneven size advance together in one
 * persistent kernel: one wavefront holds one instance at a time (a Hubbard
 * column has at most 1 + 2 * bonds entries) and waves take instances from a
 * queue; the host replays a captured HIP graph of such launches until every
 * instance of the current wave has stopped or used its step budget.
 *
 * Memory: each instance gets a table sized to its FCI dimension (the smallest
 * power of two >= dimension / load_factor, at least 2^10, capped by
 * max_table_slots if that is set and by the memory budget), so no instance
 * can fill its table below the budget.  A scheduler keeps the tables of the
 * resident instances within memory_budget: a call runs the instances that
 * still have work in waves, admitting instances in index order while their
 * tables fit and evicting instances that have no work left in the call
 * (stopped or failed ones are released with their results kept; running ones
 * are checkpointed to host memory as their (key, c) list and restarted later
 * by the rule of cdfci_load: b rebuilt exactly, the step accumulator reset).
 * Each instance is an ordinary context created as by cdfci_init_hubbard
 * (Neel determinant plus subspace start); while it is resident it can be
 * inspected with cdfci_energy, cdfci_export and the like through
 * cdfci_batch_context. */
typedef struct {
  int dims[3];   /* sites per direction (row-major site index); entries past ndim ignored */
  int ndim;      /* 1..3; at most 63 sites and 64 distinct bonds */
  int n_alpha, n_beta;
  int reserved;
  double t, U;   /* hopping -t on each distinct nearest-neighbour pair, on-site U */
} cdfci_hubbard_spec;

typedef struct cdfci_batch cdfci_batch; /* opaque, library-owned */

typedef struct {
  uint64_t table_slots;      /* per instance (power of two); 0 = sized from the FCI dimension
                                (see above) */
  uint64_t max_table_slots;  /* cap of the automatic size; 0 = none (only the budget) */
  uint64_t memory_budget;    /* bytes of instance tables resident at once; 0 = 85% of the
                                device memory free at creation */
  double load_factor;        /* 0 = 0.79 */
  double z_threshold;        /* tau, as in cdfci_opts */
  double dx_damping;         /* 0 = 0.9 */
  double dx_threshold;       /* per-instance stopping rule; 0 = never */
  int64_t chunk_steps;       /* steps an instance runs per visit of a wave; 0 = 1024 */
  int launches_per_graph;    /* persistent launches captured in the replayed graph; 0 = 4 */
  int waves;                 /* wavefronts per launch; 0 = one per instance (at most 8192) */
  void* stream;              /* hipStream_t; NULL = a stream of the batch's own */
} cdfci_batch_opts;

typedef struct {
  int64_t steps;           /* iterations this call, summed over instances */
  int64_t elements;        /* column entries enumerated this call (nonzero hops + diagonal) */
  int32_t running;         /* instances that used their whole budget */
  int32_t stopped;         /* instances stopped by dx_threshold (now or before) */
  int32_t failed;          /* instances with an error (table full) */
  int32_t graph_replays;
  int32_t rounds;          /* waves of resident instances the scheduler ran */
  int32_t restarts;        /* instances restored from a checkpoint in this call */
  double seconds;          /* device time of the call */
  double peak_bytes;       /* largest table bytes resident at once in this call */
} cdfci_batch_stats;

/* Create count instances (count >= 1).  Specs are checked and table sizes
 * planned here; instances are created when the scheduler first admits them,
 * and an instance whose start fails (e.g. CDFCI_ERR_NOT_NEGATIVE) is marked
 * failed with that code. */
int cdfci_init_hubbard_batch(const cdfci_hubbard_spec* specs, int count, const cdfci_batch_opts* opts,
                             cdfci_batch** out);

/* Advance every instance by up to max_steps iterations (fewer if it stops or
 * fails); returns after completion.  out may be NULL. */
int cdfci_step_batch(cdfci_batch* batch, int64_t max_steps, cdfci_batch_stats* out);

/* Per instance (host arrays of length count, any may be NULL): energy
 * alpha/mu, iterations since init, status 1 = stopped by dx_threshold,
 * 0 = still running, negative = CDFCI_ERR_* of that instance. */
int cdfci_batch_results(cdfci_batch* batch, double* energy, int64_t* steps, int* status);

/* Advance only `instance` by up to nsteps iterations, recording per iteration
 * the energy and the chosen determinant (host arrays of length nsteps, any may
 * be NULL).  The instance is admitted if it is not resident (evicting others
 * as a call of cdfci_step_batch would).  For parity tests. */
int cdfci_batch_trace(cdfci_batch* batch, int instance, int64_t nsteps, double* energy,
                      uint64_t* sel_alpha, uint64_t* sel_beta);

/* Borrow the context of one resident instance (owned by the batch: do not
 * free it, do not step it while the batch runs; a later batch call may evict
 * it).  CDFCI_ERR_INVALID_ARG if the instance is not resident. */
int cdfci_batch_context(cdfci_batch* batch, int instance, cdfci_ctx** ctx);

/* Table slots planned for each instance (host array of length count). */
int cdfci_batch_tables(cdfci_batch* batch, uint64_t* slots);

int cdfci_free_batch(cdfci_batch* batch);

/* ---- Autotuning -------------------------------------------------------------
 * Both tuners measure real work on the live state and keep it: the trial steps
 * are ordinary steps (they move the state toward the minimiser). */

/* Pick the number of coordinates per step among ks[0..nk) (each 1..1024) by
 * the energy decrease per device-second.  Trials of about seconds_per_trial
 * each run in `rounds` rounds, forward then backward through ks, so that the
 * slowing convergence weighs on every candidate alike.  *best_k gets the
 * winner; rates (nk doubles, may be NULL) the mean decrease in Ha/s. */
int cdfci_tune_k(cdfci_ctx* ctx, const int* ks, int nk, double seconds_per_trial, int rounds, int* best_k,
                 double* rates);

/* Pick a batch's hash load factor, chunk_steps and launches_per_graph among
 * the candidate lists by aggregate iterations per second of wall time over
 * steps_per_trial iterations per instance each (the whole batch, so the
 * trade of a lower load factor, shorter probes against larger tables and
 * fewer resident instances per wave, is measured as it is paid).  A new load
 * factor re-plans every table: resident instances are checkpointed and
 * restarted at their new size.  The winners become the batch's settings.
 * lfs may be NULL (nlf = 0: the load factor is kept); best_* may be NULL. */
int cdfci_tune_batch(cdfci_batch* batch, const int64_t* chunks, int nc, const int* launches, int nl,
                     const double* lfs, int nlf, int64_t steps_per_trial, int64_t* best_chunk,
                     int* best_launches, double* best_lf);

/* ---- Several low-lying states: xCDFCI (Sec. 3.3, Alg. 3) ---------------------
 * Minimises f(C) = ||H - sigma I + C C^T||_F^2 over C with n = K + 1 columns
 * (1 <= n <= 8).  At a minimiser the column space of C is the span of the n
 * lowest eigenvectors of H; the energies are the eigenvalues of the pencil
 * (C^T H C, C^T C).  C and B = (H - sigma I) C live in a device hash table
 * keyed by determinant, one row of n doubles each; S = C^T C and
 * Q = C^T (H - sigma I) C are maintained in double-double precision.  One
 * iteration takes the row i of largest ||G_i||_inf, G = 4 B + 4 C S, among
 * the previous coordinate's column and that coordinate itself, and sets
 * C_i <- C_i + eta G_i with eta the exact minimiser of the quartic
 * f(C + eta e_i G_i) (Appendix A; the slope coefficient is ||G_i||^2), then
 * updates B over column i under the compression rule of Sec. 3.1 (z_threshold)
 * and recalculates B_i.
 *
 * sigma (shift) must make the n lowest eigenvalues of H - sigma I negative,
 * which f needs (Sec. 2.3); reported energies add it back.  Start (Sec. 4.1.3,
 * excited-state solver): D_1 = the reference determinant, D_2 .. D_n the
 * determinants of lowest diagonal H_jj among those connected to D_1
 * (H_j,D1 != 0; equal H_jj ordered by the smaller (beta, alpha) key), column
 * k of C^(0) the unit vector at D_k, B^(0) = (H - sigma I) C^(0); the first
 * coordinate is the stored row of largest ||G_j||_inf.  The reference is the
 * aufbau determinant (lowest h_pp; opts->init_kind == 2: the alternating
 * chain pattern as in cdfci_init), or the Neel determinant for lattices.
 * Only table_slots, load_factor, z_threshold, dx_damping, dx_threshold and
 * stream of opts are used.  CDFCI_ERR_UNSUPPORTED if fewer than n - 1
 * determinants are connected to D_1. */
typedef struct cdfci_xctx cdfci_xctx; /* opaque, library-owned */

int cdfci_xinit(const double* h, const double* eri, int n_orb, int n_alpha, int n_beta, int n_states,
                double shift, const cdfci_opts* opts, cdfci_xctx** out);

/* The same for a periodic Hubbard lattice (as cdfci_init_hubbard). */
int cdfci_xinit_hubbard(const int* dims, int ndim, double t, double U, int n_alpha, int n_beta,
                        int n_states, double shift, const cdfci_opts* opts, cdfci_xctx** out);

/* The same solver for the Hubbard model in momentum space (the paper's
 * HubbardK Hamiltonian, Sec. 4.1.1): orbital k is the row-major index of a
 * momentum vector on the periodic lattice dims[0..ndim), one-body energy
 * eps_k = sum_d -2t cos(2 pi k_d / dims_d) (-t cos(pi k_d) for a direction of
 * length 2, whose two sites share one bond; 0 for length 1), and the on-site
 * term (U/L) sum_{k,p,q} a+_{k+q up} a_{k up} a+_{p-q dn} a_{p dn}.  A column
 * holds the diagonal and the momentum-conserving pair moves, at most
 * 1 + n_alpha n_beta (L - 1) entries.  Start (Sec. 5.1.3): every
 * configuration of lowest one-body energy (the Fermi shell filled in all
 * ways), H - sigma I on them and its n lowest eigenpairs, column k of C^(0)
 * = sqrt(-(lambda_k - sigma)) v_k with its first largest-magnitude entry
 * positive.  H conserves total momentum, so the iteration never leaves the
 * sectors of that start.  With n_states = 1 this is Alg. 1 from the paper's
 * start.  CDFCI_ERR_UNSUPPORTED if the block has fewer than n or more than
 * 2048 configurations; CDFCI_ERR_NOT_NEGATIVE if a wanted eigenvalue of
 * H - sigma I on it is not negative. */
int cdfci_xinit_hubbard_k(const int* dims, int ndim, double t, double U, int n_alpha, int n_beta,
                          int n_states, double shift, const cdfci_opts* opts, cdfci_xctx** out);

/* Run up to nsteps iterations (one persistent cooperative launch, one
 * device-wide barrier per iteration) and stop early when
 * the damped accumulator of |eta| ||G_i||_2 falls below dx_threshold.  Host
 * traces, any may be NULL: energies (nsteps * n, the pencil's eigenvalues
 * after each iteration, ascending), sel_alpha / sel_beta (nsteps, the row
 * updated).  out may be NULL; its energy field is the lowest energy, mu and
 * alpha are trace(S) and trace(Q). */
int cdfci_xstep(cdfci_xctx* x, int64_t nsteps, double* energies, uint64_t* sel_alpha, uint64_t* sel_beta,
                cdfci_stats* out);

/* Current energies (n doubles, ascending, shift added back). */
int cdfci_xenergies(cdfci_xctx* x, double* energies);

/* The maintained S = C^T C and Q = C^T (H - sigma I) C (n*n row-major each,
 * rounded to double; either may be NULL). */
int cdfci_xmatrices(cdfci_xctx* x, double* S, double* Q);

/* Every stored determinant: keys 2*cap uint64 (alpha, beta), C and B rows
 * (n doubles each, cap*n), in no particular order.  *count = entries stored;
 * at most cap are written. */
int cdfci_xexport(cdfci_xctx* x, uint64_t* keys, double* C, double* B, int64_t cap, int64_t* count);

int cdfci_xfree(cdfci_xctx* x);

/* ---- Orbital optimisation: OptOrbFCI (Sec. 3.4, Alg. 4) ---------------------
 * Chooses N orbitals out of M (the columns of U, M x N, U^T U = I) that
 * minimise the FCI ground energy in the N-orbital space.  Outer iteration l:
 * integrals in the current orbitals (h' = U^T h U, four-index transform of
 * (pq|rs) on the device), the FCI ground state by coordinate descent
 * (cdfci_init + cdfci_step with k coordinates per step, then
 * cdfci_rdm_backward for the 1- and 2-RDM of the top_n support), energy
 * E^(l) = sum h' gamma + 1/2 sum (pq|rs)' Gamma, then the orbital problem of
 * eq. (subopt) with the RDMs fixed, P4(U), by projected steps
 * U <- orth(U - t_k grad P4(U)) (eq. (projBB)): orth the polar factor,
 * grad the Euclidean gradient, t_0 = step0 and then Barzilai-Borwein sizes
 * <s,s>/|<s,y>| and |<s,y>|/<y,y> in turn (s, y: differences of U and of
 * grad).  The orbital problem stops at a Riemannian gradient norm
 * <= grad_tol or after max_inner steps and keeps its iterate of lowest P4;
 * the outer loop stops when |E^(l) - E^(l-1)| <= energy_tol (a negative
 * value: never) or after max_outer solves. */
typedef struct {
  int n_active;            /* N: orbitals of the FCI space, 1..min(M, 63) */
  int max_outer;           /* FCI solves at most; 0 = 20 */
  int max_inner;           /* projected steps per orbital problem at most; 0 = 100 */
  int k;                   /* coordinates per CD step of each solve (1..1024); 0 = 1 */
  int have_u;              /* 1: U holds the start (orthonormalised first); 0: the identity
                              columns of the N orbitals of lowest h_pp, in orbital order */
  int reserved;
  int64_t cd_steps;        /* CD iterations per solve at most; 0 = 10^6 */
  double cd_dx_threshold;  /* stopping rule of each solve (Sec. 4.1.3); 0 = 1e-10 */
  double energy_tol;       /* 0 = 1e-8 */
  double grad_tol;         /* 0 = 1e-8 */
  double step0;            /* 0 = 1e-2 */
  double z_threshold;      /* tau of the solves */
  uint64_t table_slots;    /* per solve; 0 = 2^22 */
  int64_t top_n;           /* RDM support (0: every c != 0) */
  void* stream;            /* hipStream_t; NULL = default stream */
} cdfci_optorb_opts;

/* h (M x M), eri (M^4, chemist, 8-fold symmetric): host.  U: host M x N
 * row-major, the start when have_u, on return the orbitals of the last
 * solve.  energies and p4_values (may be NULL): host, max_outer doubles;
 * energies[l] = E^(l), p4_values[l] = P4 at the end of orbital problem l
 * (an upper bound of E^(l+1)).  *n_outer = solves done.  Errors of the
 * solves are passed on. */
int cdfci_optorb(const double* h, const double* eri, int n_basis, int n_alpha, int n_beta,
                 const cdfci_optorb_opts* opts, double* U, double* energies, double* p4_values, int* n_outer);

/* ---- FCIDUMP input (Sec. 4.1.1) ---------------------------------------------
 * Read a FCIDUMP file (namelist header "&FCI NORB=, NELEC=, MS2=, ..." closed
 * by "&END" or "/", then lines "value i j k l" with 1-based indices: (ij|kl)
 * for i,j,k,l > 0, h_ij for k = l = 0, the core energy for all zero; lines
 * with only i > 0 are ignored).  Host code only, no device work.
 * n_alpha = (NELEC + MS2) / 2, n_beta = (NELEC - MS2) / 2.  Integrals with
 * |value| < threshold are dropped (the paper's integral truncation; the core
 * energy is always kept).  h (n_orb^2), eri (n_orb^4, chemist, all 8 images
 * filled) and ecore are host buffers the caller sizes from a first call with
 * all three NULL, which reads the header only.  CDFCI_ERR_INVALID_ARG for an
 * unreadable file or a malformed header or line, CDFCI_ERR_UNSUPPORTED for
 * NORB > 63. */
int cdfci_read_fcidump(const char* path, double threshold, int* n_orb, int* n_alpha, int* n_beta, double* h,
                       double* eri, double* ecore);

const char* cdfci_strerror(int code);
const char* cdfci_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CDFCI_H */
