"""Throughput of the ranking / H·x / Lanczos hot path on one MI355X.

Workload (default): periodic Hubbard chain, L = 14 sites, t = 1, U = 4, sector
(N_up, N_dn) = (7, 7) with 3432^2 = 11,778,624 states, fp64 vectors, Lanczos
from a seeded random unit start vector.  A step is one Lanczos step: the
on-the-fly H·x (unrank both halves, staggered rank of every hop target,
fermion signs, gather x) fused with u = H v_j - beta v_{j-1} and the alpha
partials, then alpha, w = u - alpha v_j, beta.  `value` is steps per second,
i.e. full H·x products per second; `granks_per_s` counts the ranked hop
targets.  All inputs are synthetic and resident in HBM before timing.

    python bench.py [--gpus 1] [--steps 200] [--warmup 10] [--no-cpu]

Prints one JSON line.  Only one GPU is used; --gpus above 1 is rejected.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Granks/s and Hubbard H·v/s, learned+batched vs plain trie, same GPU"
HBM_PEAK_GBS = 8000.0
L, U, NUP, NDN, SEED = 14, 4.0, 7, 7, 2


def chain_bonds(L):
    return [(i, (i + 1) % L, 1.0) for i in range(L)]


def hops_per_product(L, nu, nd):
    """Number of ranked hop targets in one product over the (nu, nd) sector:
    for each spin, each periodic bond whose two sites differ hops once.  Pairs
    (site i occupied, site i+1 empty or vice versa) over all half patterns:
    2 * C(L-2, n-1) configurations per bond and spin half."""
    cu, cd = math.comb(L, nu), math.comb(L, nd)
    per_up = L * 2 * math.comb(L - 2, nu - 1)
    per_dn = L * 2 * math.comb(L - 2, nd - 1)
    return per_up * cd + per_dn * cu


def cpu_baseline(budget_s: float):
    """The oracle's H·x (tuple terms, Eq. Talpha2, bisection ranks; plain C,
    one thread) on a contiguous block of rows, scaled to products per second."""
    from oracle import hamiltonian as OH
    import synth
    st = OH.sector(L, NUP, NDN)
    tl = OH.terms(L, chain_bonds(L), U)
    x = synth.start_vector(SEED, st.size)
    rows = 20000
    t0 = time.perf_counter()
    OH.apply(st, tl, x, row_range=(0, rows))
    dt = time.perf_counter() - t0
    rows = int(min(st.size, max(rows, rows * budget_s / max(dt, 1e-9))))
    t0 = time.perf_counter()
    OH.apply(st, tl, x, row_range=(0, rows))
    dt = time.perf_counter() - t0
    rate = rows / dt / st.size
    return {"value": rate, "unit": "H·v/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle H·x over rows 0..{rows - 1} of {st.size} ({dt:.1f} s, 1 thread), "
                      f"scaled to whole products"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--k", type=int, default=0, help="half-pattern chunk width (0 = automatic)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--G", type=int, default=-1,
                    help="fixed launch shape: alpha_up blocks per tile (0 = alpha_dn-stationary kernel); "
                         "implies --no-tune")
    ap.add_argument("--block", type=int, default=512, help="tile-kernel block size with --G")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the H·x product (and one plain copy of x for counter calibration); "
                         "for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the path is built and measured on a single "
              "MI355X (see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2203_04158_amd as mbr
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    h = mbr.hubbard_create(L, chain_bonds(L), [(NUP, NDN)], U=[U] * L, precision=mbr.F64, k=args.k)
    if args.G >= 0:
        cfg = mbr.hubbard_get_config(h)
        mbr.hubbard_set_config(h, k=cfg["k"], G=args.G, block=args.block)
    elif not args.no_tune:
        mbr.hubbard_autotune(h, reps=5)
    launch_cfg = mbr.hubbard_get_config(h)
    dim = h.dim
    v0 = torch.from_numpy(synth.start_vector(SEED, dim)).to(dev)

    if args.kernel_only:
        x = v0.clone()
        y = torch.empty_like(x)
        for _ in range(args.kernel_reps):
            mbr.hubbard_apply(h, x, y)
        y.copy_(x)  # plain copy of dim fp64 values: known traffic for calibration
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": True, "dim": dim, "launch": launch_cfg}), flush=True)
        return

    # warm-up: graph capture, caches, clocks
    if args.warmup > 0:
        lzw = mbr.lanczos_create(h, args.warmup, use_graph=True)
        mbr.lanczos_start(lzw, v0)
        mbr.lanczos_step(lzw, args.warmup)
        torch.cuda.synchronize()
        del lzw

    lz = mbr.lanczos_create(h, args.steps, use_graph=True)
    mbr.lanczos_start(lz, v0)
    mbr.lanczos_step(lz, 1)          # builds both step graphs before timing
    mbr.lanczos_step(lz, 1)
    mbr.lanczos_start(lz, v0)        # restart the recurrence from v0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mbr.lanczos_step(lz, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    e0, nsteps = mbr.lanczos_result(lz)

    # dominant kernel: the H·x product, timed with HIP events on this stream
    x = v0.clone()
    y = torch.empty_like(x)
    mbr.hubbard_apply(h, x, y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.kernel_reps):
        mbr.hubbard_apply(h, x, y)
    ev1.record()
    torch.cuda.synchronize()
    hv_ms = ev0.elapsed_time(ev1) / args.kernel_reps
    alg_bytes = 16.0 * dim  # x read once + y written once, fp64
    achieved = alg_bytes / (hv_ms * 1e-3) / 1e9

    steps = args.steps
    ms_per_step = elapsed * 1e3 / steps
    value = steps / elapsed
    hops = hops_per_product(L, NUP, NDN)
    gold = os.path.join(ROOT, "tests", "golden", "hubbard_chain_L14.json")
    e_ref = json.load(open(gold))["e0_exact"] if os.path.exists(gold) else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "H·v/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "hubbard_chain_L14_U4_sector7x7_lanczos_fp64",
                   "L": L, "t": 1.0, "U": U, "sector": [NUP, NDN], "dim": dim,
                   "lanczos_steps": steps, "ranker": "staggered halves",
                   "start_vector_seed": SEED,
                   "launch": {k: launch_cfg[k] for k in ("k", "G", "block", "tiles")}},
        "granks_per_s": value * hops / 1e9,
        "hops_per_product": hops,
        "hv_kernel_ms": hv_ms,
        "e0": float(e0[0]),
        "e0_rel_err_vs_oracle": (abs(e0[0] - e_ref) / abs(e_ref)) if e_ref else None,
        "lanczos_steps_done": int(nsteps[0]),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "hv_kernel (plain H·x)", "alg_bytes_per_launch": alg_bytes},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
