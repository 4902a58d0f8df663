"""Thin Python binding of include/cdfci.h.  Argument marshalling only: every
step of the solver runs in the HIP library; PyTorch supplies device memory (the
hash-table workspace) and the stream."""
import ctypes
import weakref

import numpy as np

from . import _lib
from ._lib import cdfci_batch_opts, cdfci_batch_stats, cdfci_hubbard_spec, cdfci_opts, cdfci_stats


class CDFCIError(RuntimeError):
    def __init__(self, code, where):
        L = _lib.load()
        msg = L.cdfci_strerror(code).decode()
        last = L.cdfci_last_error().decode()
        super().__init__(f"{where}: {msg} ({code})" + (f" [{last}]" if last else ""))
        self.code = code


# every library object this module has opened and not yet closed
_live = weakref.WeakSet()


def live_objects():
    """Number of contexts and batches opened through this module and still open."""
    return sum(1 for o in list(_live) if getattr(o, "handle", None) and not isinstance(o, _BorrowedContext))


def _check(rc, where):
    if rc != 0:
        raise CDFCIError(rc, where)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def make_opts(table_slots=1 << 22, load_factor=0.79, z_threshold=0.0, dx_damping=0.9,
              dx_threshold=0.0, energy_shift=0.0, init_kind=0, grid_blocks=0, block_threads=0,
              workspace=None, stream=None):
    o = cdfci_opts()
    o.table_slots = int(table_slots)
    o.load_factor = float(load_factor)
    o.z_threshold = float(z_threshold)
    o.dx_damping = float(dx_damping)
    o.dx_threshold = float(dx_threshold)
    o.energy_shift = float(energy_shift)
    o.init_kind = int(init_kind)
    o.grid_blocks = int(grid_blocks)
    o.block_threads = int(block_threads)
    if workspace is not None:
        o.workspace = ctypes.c_void_p(int(workspace.data_ptr()))
        o.workspace_bytes = int(workspace.numel() * workspace.element_size())
    if stream is not None:
        o.stream = ctypes.c_void_p(int(stream))
    return o


def cdfci_workspace_size(n_orb, n_alpha, n_beta, opts):
    n = ctypes.c_size_t(0)
    _check(_lib.load().cdfci_workspace_size(n_orb, n_alpha, n_beta, ctypes.byref(opts),
                                            ctypes.byref(n)), "cdfci_workspace_size")
    return n.value


def _torch_workspace(n_orb, n_alpha, n_beta, opts):
    """Allocate the table workspace with torch and bind torch's current stream."""
    import torch

    nbytes = cdfci_workspace_size(n_orb, n_alpha, n_beta, opts)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    opts.workspace = ctypes.c_void_p(int(ws.data_ptr()))
    opts.workspace_bytes = nbytes
    if not opts.stream:
        opts.stream = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    return ws


class Context:
    """Owns a cdfci_ctx (and the torch workspace that backs its table)."""

    def __init__(self, handle, workspace, N, na, nb):
        self.handle = handle
        self.workspace = workspace
        self.N, self.na, self.nb = N, na, nb
        self.integrals = None
        _live.add(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if self.handle:
            _lib.load().cdfci_free(self.handle)
            self.handle = None
            self.workspace = None


def _integral_arg(x):
    """(pointer, keep-alive, host copy) of an integral array: a float64 torch
    tensor on the GPU is passed as a device pointer, anything else as a
    contiguous float64 host array."""
    if type(x).__module__.startswith("torch"):
        import torch

        if x.is_cuda:
            t = x.detach().to(torch.float64).contiguous()
            return ctypes.cast(ctypes.c_void_p(t.data_ptr()), ctypes.POINTER(ctypes.c_double)), t, t
        x = x.detach().numpy()
    a = np.ascontiguousarray(x, dtype=np.float64)
    return _dp(a), a, a


def cdfci_init(h, eri, n_alpha, n_beta, use_torch_workspace=True, **kw):
    """Context for integrals h (N x N) and eri (N^4, chemist): numpy arrays,
    CPU tensors or float64 tensors on the GPU (passed as device pointers)."""
    L = _lib.load()
    hp, hk, href = _integral_arg(h)
    ep, ek, eref = _integral_arg(eri)
    N = int(hk.shape[0])
    assert tuple(hk.shape) == (N, N) and tuple(ek.shape) == (N, N, N, N)
    opts = make_opts(**kw)
    ws = _torch_workspace(N, n_alpha, n_beta, opts) if use_torch_workspace else None
    ctx = ctypes.c_void_p()
    _check(L.cdfci_init(hp, ep, N, n_alpha, n_beta, ctypes.byref(opts), ctypes.byref(ctx)), "cdfci_init")
    c = Context(ctx, ws, N, n_alpha, n_beta)
    c.integrals = (href, eref)  # what the context was created from (checked by autograd)
    return c


def cdfci_init_hubbard(dims, t, U, n_alpha, n_beta, use_torch_workspace=True, **kw):
    L = _lib.load()
    d = (ctypes.c_int * len(dims))(*[int(x) for x in dims])
    N = int(np.prod(dims))
    opts = make_opts(**kw)
    ws = _torch_workspace(N, n_alpha, n_beta, opts) if use_torch_workspace else None
    ctx = ctypes.c_void_p()
    _check(L.cdfci_init_hubbard(d, len(dims), float(t), float(U), n_alpha, n_beta,
                                ctypes.byref(opts), ctypes.byref(ctx)), "cdfci_init_hubbard")
    return Context(ctx, ws, N, n_alpha, n_beta)


def cdfci_step(ctx, k=1, nsteps=1):
    st = cdfci_stats()
    _check(_lib.load().cdfci_step(ctx.handle, int(k), int(nsteps), ctypes.byref(st)), "cdfci_step")
    return st.as_dict()


def cdfci_step_trace(ctx, nsteps):
    E = np.zeros(nsteps)
    a = np.zeros(nsteps, np.uint64)
    b = np.zeros(nsteps, np.uint64)
    eta = np.zeros(nsteps)
    st = cdfci_stats()
    _check(_lib.load().cdfci_step_trace(ctx.handle, int(nsteps), _dp(E), _up(a), _up(b), _dp(eta),
                                        ctypes.byref(st)), "cdfci_step_trace")
    n = st.steps
    return {"energy": E[:n], "sel_alpha": a[:n], "sel_beta": b[:n], "eta": eta[:n],
            "stats": st.as_dict()}


def cdfci_step_energies(ctx, k, nsteps):
    E = np.zeros(max(int(nsteps), 1))
    st = cdfci_stats()
    _check(_lib.load().cdfci_step_energies(ctx.handle, int(k), int(nsteps), _dp(E), ctypes.byref(st)),
           "cdfci_step_energies")
    return E[:st.steps], st.as_dict()


def cdfci_energy(ctx, exact=0):
    e = ctypes.c_double(0.0)
    _check(_lib.load().cdfci_energy(ctx.handle, int(exact), ctypes.byref(e)), "cdfci_energy")
    return e.value


def cdfci_rdm_backward(ctx, grad_E=1.0, top_n=0, want_eri=True):
    """Returns (energy[2], dh, deri or None, kappa); see include/cdfci.h."""
    N = ctx.N
    energy = np.zeros(2)
    dh = np.zeros((N, N))
    deri = np.zeros((N, N, N, N)) if want_eri else None
    kap = np.zeros((N, N))
    _check(_lib.load().cdfci_rdm_backward(ctx.handle, float(grad_E), int(top_n), _dp(energy), _dp(dh),
                                          _dp(deri) if deri is not None else None, _dp(kap)),
           "cdfci_rdm_backward")
    return energy, dh, deri, kap


def make_rdm1(ctx, top_n=0):
    """Spin-summed 1-RDM gamma[p, q] = sum_s <a+_ps a_qs> of the normalised
    top_n support (the reverse pass at grad_E = 1)."""
    _, dh, _, _ = cdfci_rdm_backward(ctx, 1.0, top_n, want_eri=False)
    return dh


def make_rdm12(ctx, top_n=0):
    """(gamma, Gamma): Gamma[p, q, r, s] = sum_st <a+_ps a+_rt a_st a_qs>
    (chemist order, E = sum h gamma + 1/2 sum (pq|rs) Gamma)."""
    _, dh, deri, _ = cdfci_rdm_backward(ctx, 1.0, top_n)
    return dh, 2.0 * deri


def cdfci_column(ctx, key):
    L = _lib.load()
    k = np.array([int(key[0]), int(key[1])], dtype=np.uint64)
    cnt = ctypes.c_int64(0)
    rc = L.cdfci_column(ctx.handle, _up(k), None, None, 0, ctypes.byref(cnt))
    n = cnt.value
    if n <= 0:
        _check(rc, "cdfci_column")
    keys = np.zeros(2 * n, np.uint64)
    vals = np.zeros(n)
    _check(L.cdfci_column(ctx.handle, _up(k), _up(keys), _dp(vals), n, ctypes.byref(cnt)),
           "cdfci_column")
    return keys[0::2].copy(), keys[1::2].copy(), vals


def cdfci_column_noalloc(ctx, key, keys_out=None, vals_out=None):
    """get_column through the no-allocation entry point.  keys_out (uint64,
    2*n) and vals_out (float64, n) may be given (numpy arrays or contiguous
    device tensors); else host arrays are made here.  Returns
    (keys_alpha, keys_beta, vals) for host outputs, else the count."""
    L = _lib.load()
    k = np.array([int(key[0]), int(key[1])], dtype=np.uint64)
    cnt = ctypes.c_int64(0)
    if keys_out is None:
        rc = L.cdfci_column_noalloc(ctx.handle, _up(k), None, None, 0, ctypes.byref(cnt))
        n = cnt.value
        if n <= 0 or rc not in (0, -1):
            _check(rc, "cdfci_column_noalloc")
        keys = np.zeros(2 * n, np.uint64)
        vals = np.zeros(n)
        _check(L.cdfci_column_noalloc(ctx.handle, _up(k), _up(keys), _dp(vals), n, ctypes.byref(cnt)),
               "cdfci_column_noalloc")
        return keys[0::2].copy(), keys[1::2].copy(), vals

    def ptr(x, t):
        if isinstance(x, np.ndarray):
            return x.ctypes.data_as(ctypes.POINTER(t)), x.size
        return ctypes.cast(ctypes.c_void_p(int(x.data_ptr())), ctypes.POINTER(t)), x.numel()

    kp, nk = ptr(keys_out, ctypes.c_uint64)
    vp, nv = ptr(vals_out, ctypes.c_double)
    _check(L.cdfci_column_noalloc(ctx.handle, _up(k), kp, vp, min(nk // 2, nv), ctypes.byref(cnt)),
           "cdfci_column_noalloc")
    return cnt.value


def cdfci_entry(ctx, bra, ket):
    k1 = np.array([int(bra[0]), int(bra[1])], dtype=np.uint64)
    k2 = np.array([int(ket[0]), int(ket[1])], dtype=np.uint64)
    v = ctypes.c_double(0.0)
    _check(_lib.load().cdfci_entry(ctx.handle, _up(k1), _up(k2), ctypes.byref(v)), "cdfci_entry")
    return v.value


def cdfci_export(ctx, top_n=0):
    L = _lib.load()
    cnt = ctypes.c_int64(0)
    _check(L.cdfci_export(ctx.handle, int(top_n), None, None, None, 0, ctypes.byref(cnt)),
           "cdfci_export")
    n = cnt.value
    keys = np.zeros(2 * max(n, 1), np.uint64)
    c = np.zeros(max(n, 1))
    b = np.zeros(max(n, 1))
    _check(L.cdfci_export(ctx.handle, int(top_n), _up(keys), _dp(c), _dp(b), n, ctypes.byref(cnt)),
           "cdfci_export")
    return keys[0:2 * n:2].copy(), keys[1:2 * n:2].copy(), c[:n], b[:n]


def cdfci_mc_candidates(ctx):
    """Candidates of the coming multicoordinate selection: dict with keys_alpha,
    keys_beta, g (the selection key as the device forms it), c_hat, b_hat,
    mu and the lazy scale s (c = s c_hat)."""
    L = _lib.load()
    cnt = ctypes.c_int64(0)
    _check(L.cdfci_mc_candidates(ctx.handle, None, None, None, None, 0, ctypes.byref(cnt), None),
           "cdfci_mc_candidates")
    n = cnt.value
    m = max(n, 1)
    keys = np.zeros(2 * m, np.uint64)
    g, c, b = np.zeros(m), np.zeros(m), np.zeros(m)
    ms = np.zeros(2)
    _check(L.cdfci_mc_candidates(ctx.handle, _up(keys), _dp(g), _dp(c), _dp(b), n, ctypes.byref(cnt),
                                 _dp(ms)), "cdfci_mc_candidates")
    return {"keys_alpha": keys[0:2 * n:2].copy(), "keys_beta": keys[1:2 * n:2].copy(), "g": g[:n],
            "c_hat": c[:n], "b_hat": b[:n], "mu": float(ms[0]), "scale": float(ms[1])}


def cdfci_mc_selection(ctx):
    """Chosen set of the last multicoordinate step: (keys_alpha, keys_beta, eta)."""
    L = _lib.load()
    cnt = ctypes.c_int64(0)
    _check(L.cdfci_mc_selection(ctx.handle, None, None, 0, ctypes.byref(cnt)), "cdfci_mc_selection")
    n = cnt.value
    keys = np.zeros(2 * max(n, 1), np.uint64)
    eta = np.zeros(max(n, 1))
    _check(L.cdfci_mc_selection(ctx.handle, _up(keys), _dp(eta), n, ctypes.byref(cnt)), "cdfci_mc_selection")
    return keys[0:2 * n:2].copy(), keys[1:2 * n:2].copy(), eta[:n]


def cdfci_random_access_rates(table_slots=1 << 28, n_ops=18_379_008):
    """Ceilings of the scatter's memory operations on random slots (see include/cdfci.h)."""
    r = np.zeros(5)
    _check(_lib.load().cdfci_random_access_rates(int(table_slots), int(n_ops), _dp(r)), "cdfci_random_access_rates")
    return {"gather16_per_s": r[0], "gather_rmw8_per_s": r[1], "gather_atomic_f64_per_s": r[2],
            "bitmap_or_ret_per_s": r[3], "copy_bytes_per_s": r[4], "table_slots": int(table_slots),
            "n_ops": int(n_ops)}


def cdfci_set_timing(ctx, on=True):
    _check(_lib.load().cdfci_set_timing(ctx.handle, int(bool(on))), "cdfci_set_timing")


def cdfci_mc_phase_times(ctx):
    """Summed device seconds per phase of the timed multicoordinate steps."""
    t = np.zeros(7)
    n = ctypes.c_int64(0)
    _check(_lib.load().cdfci_mc_phase_times(ctx.handle, _dp(t), ctypes.byref(n)), "cdfci_mc_phase_times")
    return {"select": t[0], "hii": t[1], "eigen_probe": t[2], "apply": t[3], "finish": t[4], "probe": t[5],
            "solve": t[6], "steps": n.value}


def cdfci_mc_select_stats(ctx):
    """Running totals of the multicoordinate selections (see include/cdfci.h)."""
    v = np.zeros(4, np.int64)
    _check(_lib.load().cdfci_mc_select_stats(ctx.handle, v.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
           "cdfci_mc_select_stats")
    return {"selections": int(v[0]), "positions": int(v[1]), "kept": int(v[2]), "fallbacks": int(v[3])}


def cdfci_load(ctx, keys_alpha, keys_beta, c):
    """Restart from a stored wavefunction (keys and c as cdfci_export returns)."""
    ka = np.asarray(keys_alpha, dtype=np.uint64)
    kb = np.asarray(keys_beta, dtype=np.uint64)
    keys = np.ascontiguousarray(np.stack([ka, kb], axis=1).reshape(-1))
    cv = np.ascontiguousarray(c, dtype=np.float64)
    assert len(ka) == len(kb) == len(cv)
    _check(_lib.load().cdfci_load(ctx.handle, _up(keys), _dp(cv), len(cv)), "cdfci_load")


def cdfci_set_threshold(ctx, tau):
    _check(_lib.load().cdfci_set_threshold(ctx.handle, float(tau)), "cdfci_set_threshold")


def cdfci_step_search(ctx, nsteps, chunk=10000, fill=0.9, growth=10.0, tau0=1e-6):
    """Returns (stats, final tau)."""
    st = cdfci_stats()
    tau = ctypes.c_double(0.0)
    _check(_lib.load().cdfci_step_search(ctx.handle, int(nsteps), int(chunk), float(fill), float(growth),
                                         float(tau0), ctypes.byref(tau), ctypes.byref(st)), "cdfci_step_search")
    return st.as_dict(), tau.value


def cdfci_phase_times(ctx):
    t = np.zeros(4)
    _check(_lib.load().cdfci_phase_times(ctx.handle, _dp(t)), "cdfci_phase_times")
    return {"step": t[0], "scatter": t[1], "barrier": t[2], "combine": t[3]}


def cdfci_free(ctx):
    ctx.close()


def cdfci_strerror(code):
    return _lib.load().cdfci_strerror(int(code)).decode()


# ---------------------------------------------------------------- Hubbard batches

class _BorrowedContext(Context):
    """An instance context owned by a batch (never freed from Python)."""

    def close(self):
        self.handle = None


class Batch:
    """Owns a cdfci_batch."""

    def __init__(self, handle, specs):
        self.handle = handle
        self.specs = specs
        self.count = len(specs)
        _live.add(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if self.handle:
            _lib.load().cdfci_free_batch(self.handle)
            self.handle = None


def cdfci_init_hubbard_batch(specs, table_slots=0, max_table_slots=0, memory_budget=0, load_factor=0.0,
                             z_threshold=0.0, dx_damping=0.0, dx_threshold=0.0, chunk_steps=0,
                             launches_per_graph=0, waves=0):
    """specs: sequence of dicts {dims, t, U, n_alpha, n_beta}."""
    L = _lib.load()
    arr = (cdfci_hubbard_spec * len(specs))()
    for i, sp in enumerate(specs):
        dims = tuple(int(x) for x in sp["dims"])
        assert 1 <= len(dims) <= 3
        arr[i].dims[:] = list(dims) + [1] * (3 - len(dims))
        arr[i].ndim = len(dims)
        arr[i].n_alpha = int(sp["n_alpha"])
        arr[i].n_beta = int(sp["n_beta"])
        arr[i].t = float(sp["t"])
        arr[i].U = float(sp["U"])
    o = cdfci_batch_opts()
    o.table_slots = int(table_slots)
    o.max_table_slots = int(max_table_slots)
    o.memory_budget = int(memory_budget)
    o.load_factor = float(load_factor)
    o.z_threshold = float(z_threshold)
    o.dx_damping = float(dx_damping)
    o.dx_threshold = float(dx_threshold)
    o.chunk_steps = int(chunk_steps)
    o.launches_per_graph = int(launches_per_graph)
    o.waves = int(waves)
    h = ctypes.c_void_p()
    _check(L.cdfci_init_hubbard_batch(arr, len(specs), ctypes.byref(o), ctypes.byref(h)),
           "cdfci_init_hubbard_batch")
    return Batch(h, list(specs))


def cdfci_step_batch(batch, max_steps):
    st = cdfci_batch_stats()
    _check(_lib.load().cdfci_step_batch(batch.handle, int(max_steps), ctypes.byref(st)), "cdfci_step_batch")
    return st.as_dict()


def cdfci_batch_results(batch):
    n = batch.count
    E = np.zeros(n)
    steps = np.zeros(n, np.int64)
    status = np.zeros(n, np.int32)
    _check(_lib.load().cdfci_batch_results(batch.handle, _dp(E), steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           status.ctypes.data_as(ctypes.POINTER(ctypes.c_int))),
           "cdfci_batch_results")
    return E, steps, status


def cdfci_batch_trace(batch, instance, nsteps):
    E = np.zeros(max(int(nsteps), 1))
    a = np.zeros(max(int(nsteps), 1), np.uint64)
    b = np.zeros(max(int(nsteps), 1), np.uint64)
    before = cdfci_batch_results(batch)[1][instance]
    _check(_lib.load().cdfci_batch_trace(batch.handle, int(instance), int(nsteps), _dp(E), _up(a), _up(b)),
           "cdfci_batch_trace")
    done = int(cdfci_batch_results(batch)[1][instance] - before)
    return {"energy": E[:done], "sel_alpha": a[:done], "sel_beta": b[:done]}


def cdfci_batch_context(batch, instance):
    h = ctypes.c_void_p()
    _check(_lib.load().cdfci_batch_context(batch.handle, int(instance), ctypes.byref(h)), "cdfci_batch_context")
    sp = batch.specs[instance]
    return _BorrowedContext(h, None, int(np.prod(sp["dims"])), int(sp["n_alpha"]), int(sp["n_beta"]))


def cdfci_free_batch(batch):
    batch.close()


# ---------------------------------------------------------------- autotuning

def cdfci_tune_k(ctx, ks=(64, 256, 1024), seconds_per_trial=0.05, rounds=2):
    """Returns (best_k, {k: Ha/s})."""
    arr = (ctypes.c_int * len(ks))(*[int(k) for k in ks])
    rates = np.zeros(len(ks))
    best = ctypes.c_int(0)
    _check(_lib.load().cdfci_tune_k(ctx.handle, arr, len(ks), float(seconds_per_trial), int(rounds),
                                    ctypes.byref(best), _dp(rates)), "cdfci_tune_k")
    return best.value, dict(zip((int(k) for k in ks), rates.tolist()))


def cdfci_tune_batch(batch, chunks=(256, 1024, 4096), launches=(1, 4, 16), load_factors=(),
                     steps_per_trial=20000):
    """Returns (best_chunk, best_launches, best_load_factor)."""
    ca = (ctypes.c_int64 * len(chunks))(*[int(c) for c in chunks])
    la = (ctypes.c_int * len(launches))(*[int(x) for x in launches])
    lf = np.ascontiguousarray(load_factors, dtype=np.float64)
    bc = ctypes.c_int64(0)
    bl = ctypes.c_int(0)
    blf = ctypes.c_double(0.0)
    _check(_lib.load().cdfci_tune_batch(batch.handle, ca, len(chunks), la, len(launches),
                                        _dp(lf) if len(lf) else None, len(lf), int(steps_per_trial),
                                        ctypes.byref(bc), ctypes.byref(bl), ctypes.byref(blf)),
           "cdfci_tune_batch")
    return bc.value, bl.value, blf.value


def cdfci_batch_tables(batch):
    """Table slots planned for each instance."""
    out = np.zeros(batch.count, np.uint64)
    _check(_lib.load().cdfci_batch_tables(batch.handle, _up(out)), "cdfci_batch_tables")
    return out


# ---------------------------------------------------------------- several states (xCDFCI)

class XContext:
    """Owns a cdfci_xctx (n_states columns of C and of B = (H - shift) C)."""

    def __init__(self, handle, N, na, nb, n_states, shift):
        self.handle = handle
        self.N, self.na, self.nb = N, na, nb
        self.n_states = n_states
        self.shift = shift
        _live.add(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if self.handle:
            _lib.load().cdfci_xfree(self.handle)
            self.handle = None


def _torch_stream(opts):
    if not opts.stream:
        import torch

        opts.stream = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))


def cdfci_xinit(h, eri, n_alpha, n_beta, n_states, shift=0.0, **kw):
    L = _lib.load()
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    N = h.shape[0]
    assert h.shape == (N, N) and eri.shape == (N, N, N, N)
    opts = make_opts(**kw)
    _torch_stream(opts)
    x = ctypes.c_void_p()
    _check(L.cdfci_xinit(_dp(h), _dp(eri), N, int(n_alpha), int(n_beta), int(n_states), float(shift),
                         ctypes.byref(opts), ctypes.byref(x)), "cdfci_xinit")
    return XContext(x, N, n_alpha, n_beta, int(n_states), float(shift))


def cdfci_xinit_hubbard(dims, t, U, n_alpha, n_beta, n_states, shift=0.0, **kw):
    L = _lib.load()
    d = (ctypes.c_int * len(dims))(*[int(v) for v in dims])
    N = int(np.prod(dims))
    opts = make_opts(**kw)
    _torch_stream(opts)
    x = ctypes.c_void_p()
    _check(L.cdfci_xinit_hubbard(d, len(dims), float(t), float(U), int(n_alpha), int(n_beta), int(n_states),
                                 float(shift), ctypes.byref(opts), ctypes.byref(x)), "cdfci_xinit_hubbard")
    return XContext(x, N, n_alpha, n_beta, int(n_states), float(shift))


def cdfci_xinit_hubbard_k(dims, t, U, n_alpha, n_beta, n_states=1, shift=0.0, **kw):
    """Momentum-space Hubbard model with the degenerate-subspace start."""
    L = _lib.load()
    d = (ctypes.c_int * len(dims))(*[int(v) for v in dims])
    N = int(np.prod(dims))
    opts = make_opts(**kw)
    _torch_stream(opts)
    x = ctypes.c_void_p()
    _check(L.cdfci_xinit_hubbard_k(d, len(dims), float(t), float(U), int(n_alpha), int(n_beta), int(n_states),
                                   float(shift), ctypes.byref(opts), ctypes.byref(x)), "cdfci_xinit_hubbard_k")
    return XContext(x, N, n_alpha, n_beta, int(n_states), float(shift))


def cdfci_xstep(x, nsteps, trace=False):
    """Returns stats, or (energies[steps, n], sel_alpha, sel_beta, stats) with trace."""
    st = cdfci_stats()
    L = _lib.load()
    if not trace:
        _check(L.cdfci_xstep(x.handle, int(nsteps), None, None, None, ctypes.byref(st)), "cdfci_xstep")
        return st.as_dict()
    m = max(int(nsteps), 1)
    E = np.zeros((m, x.n_states))
    a = np.zeros(m, np.uint64)
    b = np.zeros(m, np.uint64)
    _check(L.cdfci_xstep(x.handle, int(nsteps), _dp(E), _up(a), _up(b), ctypes.byref(st)), "cdfci_xstep")
    n = st.steps
    return E[:n], a[:n], b[:n], st.as_dict()


def cdfci_xenergies(x):
    E = np.zeros(x.n_states)
    _check(_lib.load().cdfci_xenergies(x.handle, _dp(E)), "cdfci_xenergies")
    return E


def cdfci_xmatrices(x):
    n = x.n_states
    S = np.zeros((n, n))
    Q = np.zeros((n, n))
    _check(_lib.load().cdfci_xmatrices(x.handle, _dp(S), _dp(Q)), "cdfci_xmatrices")
    return S, Q


def cdfci_xexport(x):
    """Returns (alpha keys, beta keys, C rows [m, n], B rows [m, n])."""
    L = _lib.load()
    cnt = ctypes.c_int64(0)
    _check(L.cdfci_xexport(x.handle, None, None, None, 0, ctypes.byref(cnt)), "cdfci_xexport")
    m = cnt.value
    n = x.n_states
    keys = np.zeros(2 * max(m, 1), np.uint64)
    C = np.zeros((max(m, 1), n))
    B = np.zeros((max(m, 1), n))
    _check(L.cdfci_xexport(x.handle, _up(keys), _dp(C), _dp(B), m, ctypes.byref(cnt)), "cdfci_xexport")
    m = min(m, cnt.value)
    return keys[0:2 * m:2].copy(), keys[1:2 * m:2].copy(), C[:m], B[:m]


def cdfci_xfree(x):
    x.close()


# ---------------------------------------------------------------- FCIDUMP input

def read_fcidump(path, threshold=0.0):
    """Returns (h [N, N], eri [N, N, N, N] chemist, n_alpha, n_beta, ecore)."""
    L = _lib.load()
    N, na, nb = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    p = str(path).encode()
    _check(L.cdfci_read_fcidump(p, float(threshold), ctypes.byref(N), ctypes.byref(na), ctypes.byref(nb),
                                None, None, None), "cdfci_read_fcidump")
    n = N.value
    h = np.zeros((n, n))
    eri = np.zeros((n, n, n, n))
    ecore = ctypes.c_double(0.0)
    _check(L.cdfci_read_fcidump(p, float(threshold), ctypes.byref(N), ctypes.byref(na), ctypes.byref(nb),
                                _dp(h), _dp(eri), ctypes.byref(ecore)), "cdfci_read_fcidump")
    return h, eri, na.value, nb.value, ecore.value


# ---------------------------------------------------------------- orbital optimisation (OptOrbFCI)

def cdfci_optorb(h, eri, n_active, n_alpha, n_beta, U0=None, max_outer=20, max_inner=100, k=1,
                 cd_steps=1000000, cd_dx_threshold=1e-10, energy_tol=1e-8, grad_tol=1e-8, step0=1e-2,
                 z_threshold=0.0, table_slots=1 << 22, top_n=0):
    """Returns (energies E^(l), final U [M, N], P4 values of the orbital problems)."""
    L = _lib.load()
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    M = h.shape[0]
    o = _lib.cdfci_optorb_opts()
    o.n_active = int(n_active)
    o.max_outer = int(max_outer)
    o.max_inner = int(max_inner)
    o.k = int(k)
    o.have_u = 0 if U0 is None else 1
    o.cd_steps = int(cd_steps)
    o.cd_dx_threshold = float(cd_dx_threshold)
    o.energy_tol = float(energy_tol)
    o.grad_tol = float(grad_tol)
    o.step0 = float(step0)
    o.z_threshold = float(z_threshold)
    o.table_slots = int(table_slots)
    o.top_n = int(top_n)
    import torch

    o.stream = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    U = np.zeros((M, int(n_active))) if U0 is None else np.array(U0, dtype=np.float64)
    U = np.ascontiguousarray(U)
    E = np.zeros(max(1, int(max_outer)))
    P = np.zeros(max(1, int(max_outer)))
    n = ctypes.c_int(0)
    _check(L.cdfci_optorb(_dp(h), _dp(eri), M, int(n_alpha), int(n_beta), ctypes.byref(o), _dp(U), _dp(E), _dp(P),
                          ctypes.byref(n)), "cdfci_optorb")
    return E[:n.value], U, P[:max(0, n.value - 1)]
