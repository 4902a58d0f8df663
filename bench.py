"""Benchmark of the coordinate-descent FCI hot path on one MI355X.

Workload: synthetic ab initio Hamiltonian, 24 spatial orbitals, 6 alpha + 6
beta electrons, 72 auxiliary vectors (seed 2024), hash table of 2^28 slots,
single-coordinate CDFCI (Alg. 1) for 10^6 iterations in total (warmup + timed)
with compression threshold tau = 5e-5 (at tau = 0 the 2^28-slot table reaches
its 0.79 load limit after about 4.6e5 iterations).  One benchmark step = one
cdfci_step call of --iters iterations (each: select, line search, enumerate the
16471-entry column, Slater-Condon, probe, scatter, recalculate b_i).

--copy-probe runs only a device copy of known size (for calibrating the HBM
byte counters of a profiler run) and exits.

Prints one JSON line: H elements/s (enumerated column entries per second,
zeros included) as `value`, plus CD iterations/s, the HBM roofline of the
persistent kernel (40 algorithmic bytes per element: a 32-byte slot read and
an 8-byte b write) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_ELEMENT = 40


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
    N, na, nb, naux = 24, 6, 6, 72
    seed = synth_inputs.CONFIG_SEEDS["abinitio_n24"]
    h, eri = synth_inputs.ab_initio(N, naux, seed)
    n_col = 16471
    ctx = api.cdfci_init(h, eri, na, nb, table_slots=1 << args.table_log2, z_threshold=args.tau,
                         grid_blocks=args.grid)
    for _ in range(args.warmup):
        api.cdfci_step(ctx, 1, args.iters)
    torch.cuda.synchronize()
    kernel_s = 0.0
    iters = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = api.cdfci_step(ctx, 1, args.iters)
        kernel_s += st["seconds"]
        iters += st["steps"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    elements = iters * n_col
    value = elements / wall
    achieved = BYTES_PER_ELEMENT * elements / kernel_s / 1e9
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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_cd1", "avg_launch_ms": 1e3 * kernel_s / args.steps},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(h, eri, na, nb)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
