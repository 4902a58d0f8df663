"""Benchmark of the coordinate-descent FCI hot path on one MI355X.

Headline workload (`value`): synthetic ab initio Hamiltonian, 24 spatial
orbitals, 6 alpha + 6 beta electrons, 72 auxiliary vectors (seed 2024), hash
table of 2^28 slots, single-coordinate CDFCI (Alg. 1) for 10^6 iterations in
total (warmup + timed) with compression threshold tau = 5e-5 (at tau = 0 the
2^28-slot table reaches its 0.79 load limit after about 4.6e5 iterations).
One benchmark step = one cdfci_step call of --iters iterations (each: select,
line search, enumerate the 16471-entry column, Slater-Condon, probe, scatter,
recalculate b_i).  `value` = enumerated column entries per second.

Further blocks on the same JSON line (skipped with --no-extra):
  batched_vs_plain  the same N = 24 system from a fresh start with the
                    multicoordinate step (k picked by the autotuner), timed to
                    the energy the plain run reached;
  mcd_n36           N = 36, 8+8, naux 108, 2^30 slots, tau 5e-5: elements/s and
                    ms per step for k = 64, 256, 1024; k = 1 for a fixed wall time,
                    then the autotuned multicoordinate step timed to that energy;
  hubbard_batch     256 periodic lattices from {2x4, 3x4, 4x4, 2x8, 3x5}, half
                    filling, U ~ [2, 10], in one persistent kernel under a
                    replayed graph (autotuned), against the single-instance
                    path on a sample of the same instances;
  rdm               RDM reverse pass on the top 10^6 determinants of the
                    headline run's final state;
  xcdfci            several low-lying states (Alg. 3) on the headline system:
                    4 states, 2^26-slot table, tau = 5e-5, iterations/s and
                    entries/s of the persistent multi-state kernel, with the
                    multi-state oracle timed on its first iterations;
  hubbard_k         the paper's 4x4 momentum-space Hubbard case (U/t = 4,
                    8+8, degenerate-subspace start): iterations/s and the
                    energy after 2e5 iterations against the exact value the
                    paper quotes;
  optorb            OptOrbFCI (Alg. 4) on the headline integrals: 12 of the 24
                    orbitals, 4a+4b, 3 outer iterations of 20000 CD steps and
                    up to 30 projected steps each; seconds per outer iteration.

--copy-probe runs only a device copy of known size (for calibrating the HBM
byte counters of a profiler run) and exits.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_ELEMENT = 40
COUNTERS = os.path.join(ROOT, "profiles", "k_cd1_abinitio_n24_hbm_counters.md")
# k_cd1 is compiled from csrc/device.h and the part of csrc/cdfci.hip up to the
# end of the kernel (the multicoordinate, reverse-pass and batch code follows it)
K_CD1_END = b"// Adds the step count after the persistent kernel"


def sources_sha256():
    """sha256 of device.h followed by cdfci.hip up to the end of k_cd1."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2605_04483_amd/csrc/device.h"), "rb") as f:
        h.update(f.read())
    with open(os.path.join(ROOT, "paper_2605_04483_amd/csrc/cdfci.hip"), "rb") as f:
        src = f.read()
    end = src.find(K_CD1_END)
    h.update(src if end < 0 else src[:end])
    return h.hexdigest()


def measured_traffic_per_element():
    """HBM bytes per column entry of k_cd1 from the committed counter runs,
    or None when the kernel sources changed since they were taken."""
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_element:\s*([0-9.]+)", text)
    s = re.search(r"sources_sha256:\s*([0-9a-f]{64})", text)
    if not m or not s or s.group(1) != sources_sha256():
        return None
    return float(m.group(1))


def cpu_baseline_xcdfci(synth_inputs, tau, steps=20):
    """The multi-state oracle (one core) on the first iterations of the
    xcdfci block's run."""
    from oracle import cd as ocd
    from oracle import xcdfci as oxc

    N, na, nb, n = 24, 6, 6, 4
    h, eri = synth_inputs.ab_initio(N, 72, synth_inputs.CONFIG_SEEDS["abinitio_n24"])
    keys, C0 = oxc.initial_rows(h, eri, ocd.aufbau(h, na, nb), n)
    t0 = time.perf_counter()
    orc = oxc.xcdfci_run(h, eri, keys, C0, tau=tau, max_steps=steps)
    t_cpu = time.perf_counter() - t0
    return {"value": orc.steps / t_cpu, "unit": "iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {steps} iterations from the same start (set-up included)"}


def cpu_baseline(h, eri, na, nb, seconds_target=15.0):
    """Serial oracle (C++, one core) on the same workload from the same start:
    elements/s over a bounded number of iterations."""
    from oracle import cd as ocd
    from oracle import fci

    keys, c0 = ocd.init_single(h, eri, na, nb)
    n_col = fci.column_size(h.shape[0], na, nb)
    t = time.perf_counter()
    r = ocd.cd_run(h, eri, keys, c0, max_steps=200, trajectory=False)
    dt = time.perf_counter() - t
    iters = max(200, int(200 * seconds_target / max(dt, 1e-3)))
    t = time.perf_counter()
    r = ocd.cd_run(h, eri, keys, c0, max_steps=iters, trajectory=False)
    dt = time.perf_counter() - t
    return {"value": r.steps * n_col / dt, "unit": "H elements/s", "cores": 1, "kind": "oracle",
            "sample": f"first {r.steps} iterations of the same run (serial C++ oracle, "
                      f"{dt:.1f} s), iters/s = {r.steps / dt:.1f}"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batched_vs_plain(api, h, eri, na, nb, args, E_plain, t_plain, n_col):
    """Multicoordinate descent from a fresh start until it reaches E_plain."""
    t0 = time.perf_counter()
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << args.table_log2, z_threshold=args.tau)
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    best_k, rates = api.cdfci_tune_k(ctx, (64, 256, 1024), seconds_per_trial=0.05, rounds=2)
    E = api.cdfci_energy(ctx)
    steps = 0
    elements = 0
    while E > E_plain and time.perf_counter() - t0 < args.mc_limit:
        st = api.cdfci_step(ctx, best_k, 20)
        steps += st["steps"]
        elements += st["elements"]
        E = st["energy"]
        if st["stopped"]:
            break
    t_mc = time.perf_counter() - t0
    ctx.close()
    return {"plain_seconds": t_plain, "plain_energy": E_plain,
            "batched_seconds": t_mc, "batched_energy": E, "reached": bool(E <= E_plain),
            "speedup": t_plain / t_mc if E <= E_plain else None,
            "k": best_k, "tune_rates_Ha_per_s": rates, "batched_steps_after_tuning": steps,
            "batched_elements_per_s_after_tuning": elements / max(t_mc, 1e-9),
            "init_seconds": t_init,
            "note": "both from their own fresh init; tuning trials count toward the batched time"}


def mcd_n36(api, synth_inputs, args):
    N, na, nb = 36, 8, 8
    h, eri = synth_inputs.ab_initio(N, 108, synth_inputs.CONFIG_SEEDS["abinitio_n36"])
    out = {"workload": "ab initio N=36 8a+8b naux=108 seed=3636, 2^30-slot table, tau=5e-5",
           "column_entries": 71793}
    import torch

    for k in ((args.n36_k,) if args.n36_k else (64, 256, 1024)):
        ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 30, z_threshold=5e-5)
        api.cdfci_step(ctx, k, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = api.cdfci_step(ctx, k, args.n36_steps)
        wall = time.perf_counter() - t0
        out[f"k{k}"] = {"ms_per_step": 1e3 * wall / max(1, st["steps"]),
                        "elements_per_s": st["elements"] / wall,
                        "coordinate_updates_per_s": st["steps"] * k / wall,
                        "energy": st["energy"]}
        ctx.close()
        log(f"n36 k={k}: {out[f'k{k}']}")
    if args.n36_k:
        return out
    # plain single-coordinate descent for a fixed wall time, then the
    # multicoordinate step (k autotuned) from its own fresh start, timed to the
    # energy the plain run reached
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 30, z_threshold=5e-5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    while time.perf_counter() - t0 < args.n36_plain_seconds:
        st = api.cdfci_step(ctx, 1, 20000)
        iters += st["steps"]
    t_plain = time.perf_counter() - t0
    E_plain = st["energy"]
    out["k1"] = {"iters_per_s": iters / t_plain, "elements_per_s": iters * 71793 / t_plain,
                 "seconds": t_plain, "energy": E_plain}
    ctx.close()
    log(f"n36 plain: {out['k1']}")
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << 30, z_threshold=5e-5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best_k, rates = api.cdfci_tune_k(ctx, (64, 256, 1024), seconds_per_trial=0.05, rounds=2)
    E = api.cdfci_energy(ctx)
    while E > E_plain and time.perf_counter() - t0 < 3 * t_plain:
        st = api.cdfci_step(ctx, best_k, 10)
        E = st["energy"]
        if st["stopped"]:
            break
    t_mc = time.perf_counter() - t0
    ctx.close()
    out["batched_vs_plain"] = {"plain_seconds": t_plain, "plain_energy": E_plain, "batched_seconds": t_mc,
                               "batched_energy": E, "reached": bool(E <= E_plain), "k": best_k,
                               "speedup": t_plain / t_mc if E <= E_plain else None,
                               "tune_rates_Ha_per_s": rates}
    log(f"n36 batched vs plain: {out['batched_vs_plain']}")
    return out


def hubbard_batch(api, synth_inputs, args):
    specs = synth_inputs.hubbard_batch_specs(256, synth_inputs.CONFIG_SEEDS["hubbard_batch"])
    t0 = time.perf_counter()
    B = api.cdfci_init_hubbard_batch(specs, dx_threshold=1e-10)
    t_init = time.perf_counter() - t0
    chunk, launches, lf = api.cdfci_tune_batch(B, chunks=(512, 2048), launches=(2, 8), load_factors=(0.5, 0.79),
                                               steps_per_trial=4000)
    t0 = time.perf_counter()
    st = api.cdfci_step_batch(B, args.batch_steps)
    wall = time.perf_counter() - t0
    E, steps, status = api.cdfci_batch_results(B)
    B.close()
    # the single-instance path on a sample of the same instances, one after another
    plain_steps, plain_wall = 0, 0.0
    seen = set()
    for sp in specs:
        if sp["dims"] in seen:
            continue
        seen.add(sp["dims"])
        ctx = api.cdfci_init_hubbard(sp["dims"], sp["t"], sp["U"], sp["n_alpha"], sp["n_beta"],
                                     table_slots=1 << 22)
        t1 = time.perf_counter()
        s1 = api.cdfci_step(ctx, 1, 20000)
        plain_wall += time.perf_counter() - t1
        plain_steps += s1["steps"]
        ctx.close()
    plain_rate = plain_steps / plain_wall
    shapes = {}
    for sp in specs:
        shapes[str(sp["dims"])] = shapes.get(str(sp["dims"]), 0) + 1
    return {"instances": len(specs), "shapes": shapes, "init_seconds": t_init,
            "chunk_steps": chunk, "launches_per_graph": launches,
            "budget_per_instance": args.batch_steps,
            "iters_per_s": st["steps"] / wall, "elements_per_s": st["elements"] / wall,
            "wall_seconds": wall, "graph_replays": st["graph_replays"],
            "stopped": int((status == 1).sum()), "failed": int((status < 0).sum()),
            "plain_single_instance_iters_per_s": plain_rate,
            "batched_over_plain": (st["steps"] / wall) / plain_rate,
            "plain_sample": f"{len(seen)} instances (one per shape), 20000 iterations each, run one after another"}


def xcdfci_block(api, synth_inputs, args):
    import torch

    N, na, nb, n = 24, 6, 6, 4
    h, eri = synth_inputs.ab_initio(N, 72, synth_inputs.CONFIG_SEEDS["abinitio_n24"])
    n_col = 16471
    x = api.cdfci_xinit(h, eri, na, nb, n, table_slots=1 << 26, z_threshold=args.tau)
    api.cdfci_xstep(x, 2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = api.cdfci_xstep(x, args.xcd_iters)
    wall = time.perf_counter() - t0
    E = api.cdfci_xenergies(x)
    x.close()
    # bytes per column entry: key (16) + C and B rows read (16 n) + B row written (8 n)
    per_entry = 16 + 24 * n
    out = {"workload": f"ab initio N=24 6a+6b naux=72 seed=2024, {n} states, 2^26-slot table, tau={args.tau}",
           "iterations": st["steps"], "iters_per_s": st["steps"] / wall,
           "elements_per_s": st["steps"] * n_col / wall, "us_per_iter": 1e6 * wall / max(1, st["steps"]),
           "device_seconds": st["seconds"], "energies": E.tolist(), "occupied": st["occupied"],
           "algorithmic_bytes_per_entry": per_entry,
           "achieved_GBs": per_entry * st["steps"] * n_col / st["seconds"] / 1e9}
    return out


def hubbard_k_block(api, args):
    import torch

    x = api.cdfci_xinit_hubbard_k((4, 4), 1.0, 4.0, 8, 8, 1, table_slots=1 << 24)
    E_start = float(api.cdfci_xenergies(x)[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = api.cdfci_xstep(x, args.hubk_iters)
    wall = time.perf_counter() - t0
    E = float(api.cdfci_xenergies(x)[0])
    x.close()
    exact = -13.62185  # 4x4, U/t = 4, 8+8: exact diagonalisation value quoted in Sec. 5.1.3
    return {"workload": "4x4 periodic Hubbard in momentum space, t=1, U=4, 8a+8b, 400-configuration start, "
                        "2^24-slot table", "iterations": st["steps"], "iters_per_s": st["steps"] / wall,
            "elements_per_s": st["elements"] / wall, "us_per_iter": 1e6 * wall / max(1, st["steps"]),
            "energy_start": E_start, "energy": E, "error_vs_exact": E - exact, "occupied": st["occupied"]}


def optorb_block(api, synth_inputs, args):
    h, eri = synth_inputs.ab_initio(24, 72, synth_inputs.CONFIG_SEEDS["abinitio_n24"])
    t0 = time.perf_counter()
    E, U, P = api.cdfci_optorb(h, eri, 12, 4, 4, max_outer=3, max_inner=30, cd_steps=20000, energy_tol=-1.0,
                               table_slots=1 << 22)
    wall = time.perf_counter() - t0
    return {"workload": "ab initio N=24 naux=72 seed=2024 integrals, 12 active orbitals, 4a+4b, "
                        "3 outer iterations x (20000 CD steps + RDMs + <= 30 projected steps)",
            "energies": E.tolist(), "p4": P.tolist(), "seconds": wall, "seconds_per_outer": wall / len(E)}


def rdm_block(api, ctx, n_col):
    top_n = 1_000_000
    ka, _, _, _ = api.cdfci_export(ctx, top_n=top_n)
    n_sup = len(ka)
    t0 = time.perf_counter()
    energy, dh, deri, kap = api.cdfci_rdm_backward(ctx, 1.0, top_n)
    wall = time.perf_counter() - t0
    return {"top_n": top_n, "support": n_sup, "seconds": wall,
            "pair_visits_per_s": n_sup * n_col / wall, "energy_rdm": energy[0],
            "energy_direct": energy[1], "note": "wall time of cdfci_rdm_backward incl. host copies of "
                                                "gamma, Gamma (24^4) and kappa"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=95)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--iters", type=int, default=10000, help="CD iterations per benchmark step")
    ap.add_argument("--table-log2", type=int, default=28)
    ap.add_argument("--tau", type=float, default=5e-5)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--mc-limit", type=float, default=60.0)
    ap.add_argument("--n36-steps", type=int, default=8)
    ap.add_argument("--n36-plain-seconds", type=float, default=20.0)
    ap.add_argument("--batch-steps", type=int, default=100000)
    ap.add_argument("--xcd-iters", type=int, default=20000)
    ap.add_argument("--hubk-iters", type=int, default=200000)
    ap.add_argument("--only", choices=("n36", "hubbard", "rdm", "xcd", "optorb", "hubk"), default=None,
                    help="diagnostic: run one extra block alone (for profiler runs) and print it")
    ap.add_argument("--n36-k", type=int, default=0, help="with --only n36: a single k")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU layout is a design "
              "(sharding the hash table by key), not an executable path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2605_04483_amd as api
    import synth_inputs

    torch.cuda.set_device(0)
    if args.copy_probe:
        # 1 GiB read + 1 GiB write, the reference for FETCH_SIZE / WRITE_SIZE
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 8}), flush=True)
        return
    if args.only == "n36":
        print(json.dumps({"mcd_n36": mcd_n36(api, synth_inputs, args)}), flush=True)
        return
    if args.only == "hubbard":
        print(json.dumps({"hubbard_batch": hubbard_batch(api, synth_inputs, args)}), flush=True)
        return
    if args.only == "hubk":
        print(json.dumps({"hubbard_k": hubbard_k_block(api, args)}), flush=True)
        return
    if args.only == "optorb":
        print(json.dumps({"optorb": optorb_block(api, synth_inputs, args)}), flush=True)
        return
    if args.only == "xcd":
        blk = xcdfci_block(api, synth_inputs, args)
        if not args.no_cpu:
            blk["cpu_baseline"] = cpu_baseline_xcdfci(synth_inputs, args.tau)
        print(json.dumps({"xcdfci": blk}), flush=True)
        return
    N, na, nb, naux = 24, 6, 6, 72
    seed = synth_inputs.CONFIG_SEEDS["abinitio_n24"]
    h, eri = synth_inputs.ab_initio(N, naux, seed)
    n_col = 16471
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << args.table_log2, z_threshold=args.tau,
                         grid_blocks=args.grid)
    torch.cuda.synchronize()
    tw = time.perf_counter()
    for _ in range(args.warmup):
        api.cdfci_step(ctx, 1, args.iters)
    torch.cuda.synchronize()
    warm_wall = time.perf_counter() - tw
    kernel_s = 0.0
    iters = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = api.cdfci_step(ctx, 1, args.iters)
        kernel_s += st["seconds"]
        iters += st["steps"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"plain: {iters} iterations in {wall:.2f} s, E = {st['energy']:.10f}")
    elements = iters * n_col
    value = elements / wall
    achieved = BYTES_PER_ELEMENT * elements / kernel_s / 1e9
    per_el = measured_traffic_per_element()
    out = {
        "metric": "H elements/s + CD iters/s to 1e-5 Ha, batched vs plain, 1 MI355X",
        "value": value,
        "unit": "H elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ab initio N=24 6a+6b naux=72 seed=2024, 2^28-slot table, "
                               "single-coordinate CDFCI, 1e6 iterations",
                   "iters_per_step": args.iters, "tau": args.tau,
                   "column_entries": n_col},
        "cd_iters_per_s": iters / wall,
        "energy": st["energy"],
        "occupied": st["occupied"],
        "total_iterations": st["total_steps"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (per_el * args.iters * n_col) if per_el is not None else None,
                     "kernel": "k_cd1", "avg_launch_ms": 1e3 * kernel_s / args.steps,
                     "algorithmic_bytes_per_launch": BYTES_PER_ELEMENT * args.iters * n_col},
    }
    if args.only == "rdm":
        print(json.dumps({"rdm": rdm_block(api, ctx, n_col)}), flush=True)
        ctx.close()
        return
    if not args.no_extra:
        try:
            out["rdm"] = rdm_block(api, ctx, n_col)
            log(f"rdm: {out['rdm']}")
        except Exception as e:  # reported, not fatal
            out["rdm"] = {"error": str(e)}
    ctx.close()
    if not args.no_extra:
        for name, fn in (("batched_vs_plain",
                          lambda: batched_vs_plain(api, h, eri, na, nb, args, st["energy"], warm_wall + wall,
                                                   n_col)),
                         ("mcd_n36", lambda: mcd_n36(api, synth_inputs, args)),
                         ("xcdfci", lambda: xcdfci_block(api, synth_inputs, args)),
                         ("optorb", lambda: optorb_block(api, synth_inputs, args)),
                         ("hubbard_k", lambda: hubbard_k_block(api, args)),
                         ("hubbard_batch", lambda: hubbard_batch(api, synth_inputs, args))):
            try:
                out[name] = fn()
                log(f"{name}: done")
            except Exception as e:
                out[name] = {"error": str(e)}
                log(f"{name}: error {e}")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(h, eri, na, nb)
        if isinstance(out.get("xcdfci"), dict) and "error" not in out["xcdfci"]:
            out["xcdfci"]["cpu_baseline"] = cpu_baseline_xcdfci(synth_inputs, args.tau)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
