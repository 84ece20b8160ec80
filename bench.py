"""Throughput of the ranking / H·x / Lanczos hot path on one MI355X.

Headline workload: periodic Hubbard chain, L = 14 sites, t = 1, U = 4, sector
(N_up, N_dn) = (7, 7) with 3432^2 = 11,778,624 states, fp64 vectors, Lanczos
from a seeded random unit start vector.  A step is one Lanczos step: the
on-the-fly H·x (unrank both halves, staggered rank of every hop target,
fermion signs, gather x) fused with u = H v_j - beta v_{j-1} and the alpha
partials, then alpha, w = u - alpha v_j, beta.  `value` is Lanczos steps per
second; `hv_per_s` is plain H·x products per second and `granks_per_s` the
ranked hop targets per second of the step.  All inputs are synthetic and
resident in HBM before timing.

The other workloads of the path are measured after the headline (kernel time
by HIP events on the launch stream, every result checked for exactness or
against stored oracle energies):
  staggered    sector M=24, N=12; 2^22 uniform member queries; k = 8
  unrank       list gathers and list-free spin unrank, 2^24 indices
  staggered64  M=64, N=32 with 64-bit patterns and ranks; 2^22 queries
  trie         M=32, N=16 with >= 6 of orbitals 0-7 occupied (66,110,671
               states); 2^24 queries, 90% members and 10% non-members; k = 4, 8
  learned      learned index vs its search without the network vs trie vs
               spin-product staggered rank on the (7,7) chain sector as 28-bit
               patterns, and on M = 32 with 8 + 8 particles (165,636,900 states)
  chain        the headline chain with fp32 vectors (fp64 dot products), with
               and without reorthogonalisation, against fp64 at equal policy
  batched      Anderson impurity model (12 sites, U = 8, eps_d = -4), all 169
               sectors, 150 steps: batched graph-captured vs per-sector
               launches, each with fp32 and fp64 vectors, full
               reorthogonalisation; and both batched forms without it
  operator     generic term-tuple H·x on the momentum-space Hubbard ring, L = 14,
               (7,7), total momentum 0, trie ranks
  ceiling      measured ceilings: a plain copy, and random 4-byte gathers
               (independent and 4-deep chains) at footprints of 1 MB to 4 GB
               and from LDS
  sweep        (by name only) the ranking microbenchmark of Sec. V.A: M = 28,
               N = 1..27, sorted queries, bisection / combinadics / staggered /
               trie at R = 4, 8, 12

    python bench.py [--gpus 1] [--steps 200] [--warmup 10] [--no-cpu] [--rows all|none|a,b]

Prints one compact JSON line on stdout (headline, roofline, CPU baseline and a
short summary per workload); the full record of every workload goes to
stderr as one line starting with "[bench] detail".  Only one GPU is used;
--gpus above 1 is rejected.
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
ROWS = ("staggered", "unrank", "staggered64", "trie", "learned", "chain", "batched", "operator", "ceiling")
EXTRA_ROWS = ("sweep",)   # run only when asked for by name


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


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s: float):
    """The oracle's plain gather-form H·x with bisection ranks (the baseline
    method of Sec. V.B, fp64, plain C) on the headline workload, on one thread
    and on every host thread this process may use, each over a bounded block
    of rows scaled to whole products; Lanczos steps/s adds the step's vector
    work (two dot products, three vector updates) timed with numpy.  Also the
    oracle's bisection and combinadics ranks of the staggered row's workload
    (M = 24, N = 12, 2^22 member queries), unsorted and sorted."""
    from oracle import hamiltonian as OH
    from oracle import combinatorics as OC
    import synth
    threads = len(os.sched_getaffinity(0))
    st = OH.sector(L, NUP, NDN)
    x = synth.start_vector(SEED, st.size)
    bonds = chain_bonds(L)

    def rate(nt, share):
        rows = 20000 * nt
        t0 = time.perf_counter()
        OH.apply_bisect(st, L, bonds, U, None, x, row_range=(0, rows), threads=nt)
        dt = time.perf_counter() - t0
        rows = int(min(st.size, max(rows, rows * share / max(dt, 1e-9))))
        t0 = time.perf_counter()
        OH.apply_bisect(st, L, bonds, U, None, x, row_range=(0, rows), threads=nt)
        dt = time.perf_counter() - t0
        return rows / dt / st.size, rows, dt

    hv1, rows1, dt1 = rate(1, 0.35 * budget_s)
    hvn, rowsn, dtn = rate(threads, 0.35 * budget_s)
    w, u, q = x.copy(), x * 0.5, x * 0.25
    t0 = time.perf_counter()
    a = float(np.dot(q, u))
    u -= a * q
    u -= 0.5 * w
    b = float(np.sqrt(np.dot(u, u)))
    w[:] = u / b
    t_vec = time.perf_counter() - t0
    sec = OC.sector_enumerate(24, OC.constraints(24, 12))
    qr = sec[synth.uniform_indices(1, 1 << 22, sec.size)]
    qs = np.sort(qr)
    ranks = {}
    for meth in ("bisect", "cns"):
        for order, qq in (("unsorted", qr), ("sorted", qs)):
            for nt in (1, threads):
                t0 = time.perf_counter()
                OC.rank_batch_threads(sec, qq, meth, nt)
                ranks[f"{meth}_{order}_{nt}t"] = round(qq.size / (time.perf_counter() - t0) / 1e9, 4)
    return {"value": 1.0 / (1.0 / hvn + t_vec), "unit": "Lanczos steps/s", "cores": threads, "kind": "oracle",
            "sample": f"plain bisection gather-form H·x (oracle, fp64) over rows 0..{rowsn - 1} on {threads} "
                      f"threads ({dtn:.1f} s) and 0..{rows1 - 1} on 1 ({dt1:.1f} s) of {st.size}, scaled "
                      f"to whole products, plus the step's vector work (numpy, {t_vec * 1e3:.0f} ms)",
            "hv_per_s_1t": hv1, "hv_per_s_all": hvn, "steps_per_s_1t": 1.0 / (1.0 / hv1 + t_vec),
            "cpu": _cpu_model(), "nproc": os.cpu_count(), "rank_Granks_m24_n12_2e22": ranks}


# --------------------------------------------------------------------------- helpers
def time_launches(torch, fn, reps: int) -> float:
    """Average milliseconds of fn() over reps back-to-back calls, by HIP events
    recorded on torch's current stream, which is the stream the binding
    launches on."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def hbm_roofline(bytes_per_launch: float, ms: float, kernel: str) -> dict:
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel": kernel, "alg_bytes_per_launch": bytes_per_launch}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_hv_rows_and_rank.md")
L2_BYTES = 4 << 20       # L2 of one XCD
GRANULE = 64             # bytes of the smallest HBM access a random gather costs


def traffic_for(key: str):
    """HBM bytes per launch of kernel `key` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE record in profiles/ (scaled by the plain-copy calibration stored
    with it), or None when there is no record or the kernel's source file has
    changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        if not line.startswith("traffic-record "):
            continue
        f = dict(kv.split("=", 1) for kv in line.split()[1:])
        if f.get("kernel") != key:
            continue
        src = os.path.join(ROOT, f["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != f["sha256"]:
            return None
        return (float(f["fetch_kib"]) * float(f["fetch_scale"])
                + float(f["write_kib"]) * float(f["write_scale"])) * 1024.0
    return None


def full_mask(M):
    return (1 << M) - 1


def member_queries(torch, mbr, sector, seed, n):
    """n members drawn uniformly by index (SplitMix64 draw mod size) and their
    indices, as device tensors (patterns via the sector's unrank table)."""
    import synth
    idx = torch.from_numpy(synth.uniform_indices(seed, n, sector.size).astype(np.int32)).cuda()
    return mbr.unrank_batch(sector, idx), idx


# --------------------------------------------------------------------------- rows
def row_staggered(torch, mbr, reps):
    """Staggered rank (Fig. fastrank), M = 24, N = 12, k = 8, 2^22 queries."""
    M, N, k, nq = 24, 12, 8, 1 << 22
    s = mbr.sector_build(M, [(full_mask(M), N, N)])
    q, idx = member_queries(torch, mbr, s, 1, nq)
    r = mbr.build_staggered_tables(M, N, k)
    out = torch.empty(nq, dtype=torch.int32, device="cuda")
    ms = time_launches(torch, lambda: mbr.rank_batch(r, q, out=out), reps)
    exact = bool(torch.equal(out, idx))
    roof = hbm_roofline(8.0 * nq, ms, "rank_staggered_kernel (4 B in, 4 B out per query)")
    roof["traffic"] = traffic_for("rank_staggered_kernel<unsignedint,unsignedint,true,4,unsignedint>")
    # cold: each launch follows a 1 GB copy that evicts the L2s and the
    # last-level cache, so queries and table come from HBM (median of 10)
    scrub = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    scrub2 = torch.empty_like(scrub)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cold = []
    for _ in range(10):
        scrub2.copy_(scrub)
        e0.record()
        mbr.rank_batch(r, q, out=out)
        e1.record()
        torch.cuda.synchronize()
        cold.append(e0.elapsed_time(e1))
    del scrub, scrub2
    cold_ms = float(np.median(cold))
    cold_res = {"kernel_ms": cold_ms, "value": nq / (cold_ms * 1e-3) / 1e9,
                "roofline": hbm_roofline(8.0 * nq, cold_ms, "rank_staggered_kernel, cold caches")}
    # steady state: 2^28 queries (the 2^22 above, 64 times over; 2 GB moved
    # per launch, far beyond the caches)
    big_q = q.repeat(64)
    big_out = torch.empty(big_q.numel(), dtype=torch.int32, device="cuda")
    ms_big = time_launches(torch, lambda: mbr.rank_batch(r, big_q, out=big_out), 5)
    stress = {"queries": big_q.numel(), "kernel_ms": ms_big, "value": big_q.numel() / (ms_big * 1e-3) / 1e9,
              "exact": bool(torch.equal(big_out, idx.repeat(64))),
              "roofline": hbm_roofline(8.0 * big_q.numel(), ms_big, "rank_staggered_kernel, 2^28 queries")}
    del big_q, big_out
    # the rank-side autotuner's pick of k for this sector and these queries
    rt, tune = mbr.rank_autotune(s, mbr.RANKER_STAGGERED, q, reps=reps)
    ms_t = time_launches(torch, lambda: mbr.rank_batch(rt, q, out=out), reps)
    autotuned = {"k": tune["k"], "candidates_timed": tune["tried"], "kernel_ms": ms_t,
                 "value": nq / (ms_t * 1e-3) / 1e9, "exact": bool(torch.equal(out, idx))}
    return {"workload": "sector M=24 N=12 (2,704,156 states), 2^22 uniform member queries, k=8",
            "value": nq / (ms * 1e-3) / 1e9, "unit": "Granks/s", "kernel_ms": ms, "exact": exact,
            "roofline": roof, "cold_after_1GB_copy": cold_res, "stress_2e28": stress, "autotuned": autotuned}


def row_unrank(torch, mbr, reps):
    """Unrank (Sec. II, Eq. unrank) of 2^24 uniform indices: through the stored
    list (a random gather per query) in the M=24 N=12 sector and in the L=14
    (7,7) spin sector, and without a list in the spin sectors L=14 (7,7) and
    L=16 (8,8) (both halves from LDS, Eq. rankupdown inverted).  Checked by
    ranking the patterns back (staggered or spin-resolved ranks)."""
    import synth
    nq = 1 << 24
    h14 = (1 << 14) - 1
    res = {"workload": "2^24 uniform indices per case; list gathers in M=24 N=12 (2,704,156 states, "
                       "10.8 MB list) and L=14 (7,7) (11,778,624 states, 47 MB); list-free spin unrank "
                       "in L=14 (7,7) and L=16 (8,8) (165,636,900 states)"}
    for name, M, cons, ranker in (
            ("list_m24_n12", 24, [(full_mask(24), 12, 12)], lambda: mbr.build_staggered_tables(24, 12, 8)),
            ("list_chain_7x7", 28, [(full_mask(28), 14, 14), (h14, 7, 7), (h14 << 14, 7, 7)],
             lambda: mbr.build_spin_ranker(14, 7, 7, 7))):
        s = mbr.sector_build(M, cons)
        idx = torch.from_numpy(synth.uniform_indices(40 + M, nq, s.size).astype(np.int32)).cuda()
        out = torch.empty(nq, dtype=torch.int32, device="cuda")
        ms = time_launches(torch, lambda: mbr.unrank_batch(s, idx, out=out), reps)
        exact = bool(torch.equal(mbr.rank_batch(ranker(), out), idx))
        res[name] = {"value": nq / (ms * 1e-3) / 1e9, "unit": "Gunranks/s", "kernel_ms": ms, "exact": exact,
                     "roofline": hbm_roofline(8.0 * nq, ms, "unrank_kernel (4 B index in, 4 B pattern out; "
                                              "the list gather comes on top)")}
        del s
    for name, L_, nu, nd in (("spin_chain_7x7", 14, 7, 7), ("spin_l16_8x8", 16, 8, 8)):
        r = mbr.build_spin_ranker(L_, nu, nd, 8)
        total = math.comb(L_, nu) * math.comb(L_, nd)
        idx = torch.from_numpy(synth.uniform_indices(50 + L_, nq, total).astype(np.int32)).cuda()
        out = torch.empty(nq, dtype=torch.int32, device="cuda")
        ms = time_launches(torch, lambda: mbr.unrank_spin_batch(r, idx, out=out), reps)
        exact = bool(torch.equal(mbr.rank_batch(r, out), idx))
        res[name] = {"value": nq / (ms * 1e-3) / 1e9, "unit": "Gunranks/s", "kernel_ms": ms, "exact": exact,
                     "roofline": hbm_roofline(8.0 * nq, ms, "unrank_spin_kernel (4 B index in, 4 B pattern out)")}
    return res


def row_staggered64(torch, mbr, reps):
    """64-bit patterns and ranks: M = 64, N = 32 (C(64,32) = 1.83e18 states, no
    list can hold them); 2^22 queries; with 8-byte entries the rows members
    reach fit LDS at k = 4 (35 KB) and k = 5 (56 KB) but not at k = 8
    (278 KB) or 16 (40 MB), which are read through the caches.  Checked by
    agreement of the four tables and by the range of the ranks."""
    import synth
    M, N, nq = 64, 32, 1 << 22
    base = synth.random_subset_patterns(64, 1 << 18, M, N)
    q = torch.from_numpy(np.tile(base, nq // base.size).view(np.int64)).cuda()
    res = {"workload": "M=64 N=32, 2^22 queries (2^18 distinct uniform 32-subsets), 64-bit ranks"}
    outs = {}
    for k in (4, 5, 8, 16):
        r = mbr.build_staggered_tables(M, N, k, width_bits=64)
        out = torch.empty(nq, dtype=torch.int64, device="cuda")
        ms = time_launches(torch, lambda: mbr.rank_batch64(r, q, out=out), reps)
        outs[k] = out
        roof = hbm_roofline(16.0 * nq, ms, f"rank_staggered_kernel, 64-bit (8 B in, 8 B out per query), k={k}")
        res[f"k{k}"] = {"value": nq / (ms * 1e-3) / 1e9, "unit": "Granks/s", "kernel_ms": ms,
                        "table_bytes": int(r.info().bytes), "roofline": roof}
        del r
    ranks = outs[8].cpu().numpy().view(np.uint64)
    res["exact"] = (bool(torch.equal(outs[4], outs[8])) and bool(torch.equal(outs[5], outs[8]))
                    and bool(torch.equal(outs[8], outs[16]))
                    and bool((ranks < np.uint64(math.comb(M, N))).all()))
    return res


def row_trie(torch, mbr, reps):
    """Trie rank + membership (Fig. trielookup, safe lookup of Sec. IV) on the
    RAS-like sector M = 32, N = 16, >= 6 of orbitals 0-7 occupied."""
    import synth
    M, nq = 32, 1 << 24
    nm = nq // 10
    s = mbr.sector_build(M, [(full_mask(M), 16, 16), (0xFF, 6, 8)])
    mem, idx = member_queries(torch, mbr, s, 3, nq - nm)
    pool = synth.random_subset_patterns(33, nm + nm // 4, M, 16)
    non = pool[np.bitwise_count(pool & np.uint64(0xFF)) <= 5][:nm]
    assert non.size == nm
    perm = torch.from_numpy(synth.shuffle_positions(34, nq)).cuda()
    q = torch.cat([mem, torch.from_numpy(non.astype(np.uint32).view(np.int32)).cuda()])[perm].contiguous()
    want = torch.cat([idx, torch.full((nm,), -1, dtype=torch.int32, device="cuda")])[perm]
    out = torch.empty(nq, dtype=torch.int32, device="cuda")
    res = {"workload": "M=32 N=16, >=6 of orbitals 0-7 occupied (66,110,671 states); 2^24 queries, "
                       "90% members by uniform index, 10% non-members",
           "n_states": s.size}
    for k in (4, 8):
        r = mbr.build_trie(s, k)
        info = r.info()
        ms = time_launches(torch, lambda: mbr.rank_batch(r, q, out=out), reps)
        exact = bool(torch.equal(out, want))
        # algorithmic bytes per query: the query in and the rank out, plus
        # two 64-B HBM granules, one for the leaf level and one for the
        # membership read of the state list (the levels above are small
        # enough to stay in LDS or L2)
        per_q = 8.0 + 2 * GRANULE
        roof = hbm_roofline(per_q * nq, ms, f"trie_rank_kernel ({per_q:.0f} B per query: 8 B stream + "
                                            f"2 random {GRANULE}-B granules)")
        roof["traffic"] = traffic_for(f"trie_rank_kernel<unsignedint>@k{k}")
        # context: one granule for every dependent gather into an array that
        # neither LDS nor an XCD's L2 holds (at k = 8 also level 2, 9.4 MB)
        ent, lds_lv = mbr.trie_level_entries(r)
        far = [l for l in range(len(ent)) if l >= lds_lv and 4 * ent[l] > L2_BYTES]
        gathers = len(far) + (1 if 4 * s.size > L2_BYTES else 0)
        roof["frac_counting_every_far_level"] = (8.0 + GRANULE * gathers) * nq / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
        roof["far_gathers_per_query"] = gathers
        res[f"k{k}"] = {"value": nq / (ms * 1e-3) / 1e9, "unit": "Granks/s", "kernel_ms": ms,
                        "exact": exact, "levels": info.levels, "lds_levels": lds_lv,
                        "level_bytes": [4 * e for e in ent], "trie_bytes": int(info.bytes),
                        "overhead_f": info.bytes / 4 / s.size, "roofline": roof}
        del r
    # the bitmap trie (records {base, bitmap}, membership from the bitmaps):
    # 8 B stream + one 64-B granule for the one level beyond L2 (k = 8)
    for k in (4, 8):
        r = mbr.build_bitmap_trie(s, k)
        ms = time_launches(torch, lambda: mbr.rank_batch(r, q, out=out), reps)
        recs, rbytes, lds_lv = mbr.bitmap_trie_levels(r)
        res[f"bitmap_k{k}"] = {"value": nq / (ms * 1e-3) / 1e9, "unit": "Granks/s", "kernel_ms": ms,
                               "exact": bool(torch.equal(out, want)), "bytes": int(r.info().bytes),
                               "overhead_f": r.info().bytes / 4 / s.size, "records": recs,
                               "record_bytes": rbytes, "lds_levels": lds_lv,
                               "roofline": hbm_roofline(136.0 * nq, ms, "bt_rank_kernel at the packed trie's "
                                                                        "136 B per query")}
        res[f"bitmap_k{k}"]["roofline"]["traffic"] = traffic_for(f"bt_rank_kernel<unsignedint>@k{k}")
        del r
    # a plain copy of the 64 MB query array: known bytes, to calibrate the
    # hardware traffic counters of the kernels above in the same run
    qc = q.clone()
    del qc
    # the learned ranker's search without its network, on the same queries
    r = mbr.build_sampled_ranker(s)
    ms = time_launches(torch, lambda: mbr.rank_batch(r, q, out=out), reps)
    res["sampled_search_no_net"] = {"value": nq / (ms * 1e-3) / 1e9, "unit": "Granks/s", "kernel_ms": ms,
                                    "exact": bool(torch.equal(out, want)), "table_bytes": int(r.info().bytes),
                                    "levels": r.info().levels}
    return res


def row_learned(torch, mbr, reps, big: bool):
    """Learned index (network prediction, max-error window, exact search) against
    the packed trie, and on the spin-product sector also against the
    spin-resolved staggered rank, on 2^24 uniform member queries."""
    out = {}
    nq = 1 << 24
    cases = [("chain_7x7_28bit", 28, [(0x3FFF, 7, 7), (0x3FFF << 14, 7, 7)], (14, 7, 7))]
    if big:
        cases.append(("m32_8x8", 32, [(0xFFFF, 8, 8), (0xFFFF0000, 8, 8)], None))
    for name, M, cons, spin in cases:
        s = mbr.sector_build(M, cons)
        q, idx = member_queries(torch, mbr, s, 4, nq)
        res = {"n_states": s.size}
        trie = mbr.build_trie(s, 8)
        t0 = time.perf_counter()
        # the window search is forced (max_window above any window) so that the
        # learned path itself is timed, whatever its windows
        lr_ = mbr.learned_train(s, trie, epochs=8, batch=4096, lr=2e-3, seed=4,
                                samples_per_epoch=min(s.size, 1 << 22), max_window=1 << 31)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        res["learned_train_s"] = train_s
        res["learned_stats"] = mbr.learned_stats(lr_)
        if name == cases[0][0]:
            # stage 1 alone on the matrix cores: the network's forward pass over
            # the 2^24 queries (one kernel; it rounds the fp32 parameters to
            # bf16 as it loads them), timed by HIP events on its stream
            params = torch.from_numpy(mbr.learned_params(lr_)).cuda()
            yq = torch.empty(nq, dtype=torch.float32, device="cuda")
            mlp_ms = time_launches(torch, lambda: mbr.mlp_forward(params, q, out=yq), reps)
            flops = 12416.0 * nq
            res["mlp_forward"] = {"ms": mlp_ms, "roofline": {
                "bound": "mfma", "achieved": flops / (mlp_ms * 1e-3) / 1e12, "peak": 2500.0,
                "unit": "TFLOP/s", "frac": flops / (mlp_ms * 1e-3) / 1e12 / 2500.0,
                "kernel": "mlp_forward_kernel (12,416 flop per query, bf16 MFMA, fp32 accumulation)"}}
        res["learned_train"] = ("8 epochs x min(N_s, 2^22) samples, batch 4096, Adam lr 2e-3, seed 4; "
                                "2^b leaves, about 4 members per leaf, at most 2^12")
        # the same search without the network: the whole list is the window
        rankers = [("trie_k8", trie), ("learned", lr_), ("sampled_search_no_net", mbr.build_sampled_ranker(s)),
                   ("bitmap_trie_k8", mbr.build_bitmap_trie(s, 8))]
        if spin is not None:
            rankers.append(("spin_staggered", mbr.build_spin_ranker(*spin, k=7)))
        ranked = torch.empty(nq, dtype=torch.int32, device="cuda")
        for rn, r in rankers:
            ms = time_launches(torch, lambda: mbr.rank_batch(r, q, out=ranked), reps)
            res[rn] = {"value": nq / (ms * 1e-3) / 1e9, "unit": "Granks/s", "kernel_ms": ms,
                       "exact": bool(torch.equal(ranked, idx))}
        out[name] = res
        del rankers, lr_, trie, s, q, idx
    return out


def row_sweep(torch, mbr, reps):
    """The ranking microbenchmark of Sec. V.A on the GPU: M = 28 orbitals and
    every sector N = 1..27; 2^22 queries per sector drawn uniformly with
    replacement and ordered by value (as the paper does); bisection,
    combinadics ranking (Fig. algr), staggered lookup and trie lookup at
    R = 4, 8, 12.  Kernel time per lookup, exactness, and the trie's memory
    overhead f = trie bytes / (4 N_s); the bitmap trie at R = 4, 8 beside them."""
    import synth
    M, nq = 28, 1 << 22
    ranked = torch.empty(nq, dtype=torch.int32, device="cuda")
    methods = (["bisect", "cns"] + [f"staggered_k{k}" for k in (4, 8, 12)] + [f"trie_k{k}" for k in (4, 8, 12)]
               + [f"bitmap_k{k}" for k in (4, 8)])
    ns = {m: [] for m in methods}
    f = {f"trie_k{k}": [] for k in (4, 8, 12)}
    f.update({f"bitmap_k{k}": [] for k in (4, 8)})
    exact = True
    sizes = []
    for N in range(1, M):
        s = mbr.sector_build(M, [(full_mask(M), N, N)])
        sizes.append(s.size)
        idx = torch.from_numpy(np.sort(synth.uniform_indices(100 + N, nq, s.size)).astype(np.int32)).cuda()
        q = mbr.unrank_batch(s, idx)
        for m in methods:
            if m == "bisect":
                r = mbr.build_bisect_ranker(s)
            elif m == "cns":
                r = mbr.build_cns_ranker(M, N)
            elif m.startswith("staggered"):
                r = mbr.build_staggered_tables(M, N, int(m.split("_k")[1]))
            elif m.startswith("bitmap"):
                r = mbr.build_bitmap_trie(s, int(m.split("_k")[1]))
                f[m].append(r.info().bytes / 4 / s.size)
            else:
                r = mbr.build_trie(s, int(m.split("_k")[1]))
                f[m].append(r.info().bytes / 4 / s.size)
            ms = time_launches(torch, lambda: mbr.rank_batch(r, q, out=ranked), reps)
            exact = exact and bool(torch.equal(ranked, idx))
            ns[m].append(ms * 1e6 / nq)
            del r
        del s, q, idx
        print(f"[bench] sweep N={N} done", file=sys.stderr, flush=True)
    return {"workload": "M=28, N=1..27, 2^22 sorted uniform queries per sector",
            "n_states": sizes, "ns_per_lookup": ns, "trie_overhead_f": f, "exact": exact,
            "half_filled_granks_per_s": {m: 1.0 / ns[m][13] for m in methods}}


def row_operator(torch, mbr, reps):
    """Generic term-tuple H·x (Eq. H -> tuples by App. A, gather form of
    Eq. Talpha2) on the momentum-space Hubbard ring of Sec. V.C: L = 14
    momenta per spin (M = 28), U = 4, sector (7,7) with total momentum 0,
    ranked by a trie (the sector is irregular: no closed-form rank).  The
    interaction has L^3 momentum-conserving terms."""
    import synth
    L, U, K = 14, 4.0, 0
    M = 2 * L
    t = np.zeros((M, M))
    for k in range(L):
        t[k, k] = t[L + k, L + k] = 2.0 * math.cos(2 * math.pi * k / L)   # -eps_k
    cl = [(L + k1, k2, L + (k1 + k2 - k3) % L, k3, 4.0 * U / L)
          for k1 in range(L) for k2 in range(L) for k3 in range(L)]
    terms = mbr.terms_from_hamiltonian(M, t, cl)
    cons = [(0x3FFF, 7, 7), (0x3FFF << 14, 7, 7)]
    sec = mbr.sector_build_mod(M, cons, list(range(L)) * 2, L, K)
    res = {"workload": f"momentum-space Hubbard ring L={L}, U={U}, sector (7,7) K={K} "
                       f"({sec.size:,} states), {len(terms)} tuples",
           "n_states": sec.size, "n_terms": len(terms)}
    x = torch.from_numpy(2 * synth.uniform01(6, sec.size) - 1).cuda()
    ys = {}
    for k in (7, 14):
        r = mbr.build_trie(sec, k)
        op = mbr.operator_create(sec, r, terms)
        y = torch.empty_like(x)
        ms = time_launches(torch, lambda: mbr.operator_apply(op, x, y), reps)
        ys[k] = y
        res[f"trie_k{k}"] = {"value": 1e3 / ms, "unit": "H·v/s", "kernel_ms": ms,
                             "term_checks_per_s": len(terms) * sec.size / (ms * 1e-3),
                             "trie_bytes": int(r.info().bytes)}
        del op, r
    res["exact"] = bool(torch.equal(ys[7], ys[14]))  # two trie layouts, identical sums
    # ground state of the K = 0 sector by the operator's fp64 Lanczos; the
    # real-space chain's E0 (stored oracle value) is the minimum over K
    r = mbr.build_trie(sec, 14)
    op = mbr.operator_create(sec, r, terms)
    v0 = torch.from_numpy(synth.start_vector(7, sec.size)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, nst, _, _ = mbr.operator_lanczos(op, v0, 200)
    dt = time.perf_counter() - t0
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "hubbard_chain_L14.json")))["e0_exact"]
    res["lanczos"] = {"steps": nst, "value": nst / dt, "unit": "Lanczos steps/s", "e0_K0": e0,
                      "e0_real_space_oracle": gold, "rel_diff": abs(e0 - gold) / abs(gold)}
    return res


def row_batched(torch, mbr, steps: int):
    """Anderson impurity model, all 169 sectors, `steps` Lanczos steps:
    batched graph-captured steps against per-sector launches, each with fp32
    vectors (fp64 dot products) and with fp64 vectors, all with full
    reorthogonalisation (equal policy), so that batching and precision each
    show their own gain; and the two batched forms without
    reorthogonalisation (three-term recurrence).  Energies against the stored
    oracle values."""
    import synth
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "anderson_12.json")))
    Ls = 12
    eps = [g["eps_d"]] + g["eps_bath"]
    Us = [g["U"]] + [0.0] * (Ls - 1)
    bonds = [(0, l + 1, -float(v)) for l, v in enumerate(g["V"])]  # +V (c+_0 c_l + h.c.)
    sectors = [(nu, nd) for nu in range(Ls + 1) for nd in range(Ls + 1)]
    res = {"workload": "Anderson impurity, 1 + 11 bath sites, U=8, eps_d=-4, all 169 sectors "
                       f"(16,777,216 states), {steps} steps"}
    hv = {}
    for name, prec, batched, reorth in (("batched_fp32", mbr.F32, True, True),
                                        ("batched_fp64", mbr.F64, True, True),
                                        ("per_sector_fp32", mbr.F32, False, True),
                                        ("per_sector_fp64", mbr.F64, False, True),
                                        ("batched_fp32_no_reorth", mbr.F32, True, False),
                                        ("batched_fp64_no_reorth", mbr.F64, True, False)):
        h = mbr.hubbard_create(Ls, bonds, sectors, U=Us, eps=eps, precision=prec)
        shape = mbr.hubbard_autotune(h, reps=3)   # (k, G, block) for this Hamiltonian and precision
        v0 = torch.from_numpy(synth.start_vector(5, h.dim)).cuda()
        lz = mbr.lanczos_create(h, steps, reorth=reorth, batched=batched, use_graph=True)
        mbr.lanczos_start(lz, v0)
        mbr.lanczos_step(lz, 2)
        mbr.lanczos_start(lz, v0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mbr.lanczos_step(lz, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        e0, nst = mbr.lanczos_result(lz)
        worst = max(abs(e0[i] - g["e0"][f"{nu},{nd}"]) / max(1.0, abs(g["e0"][f"{nu},{nd}"]))
                    for i, (nu, nd) in enumerate(sectors))
        res[name] = {"value": steps / dt, "unit": "Lanczos steps/s", "ms_per_step": dt * 1e3 / steps,
                     "reorth": reorth, "e0": float(e0.min()), "worst_rel_err_vs_oracle": worst,
                     "launch": {kk: shape[kk] for kk in ("k", "G", "block", "tuned_ms")}}
        del lz
        torch.cuda.synchronize()
        if batched and reorth:
            x = torch.zeros(h.dim, dtype=torch.float32 if prec == mbr.F32 else torch.float64,
                            device="cuda")
            x.copy_(v0)
            y = torch.empty_like(x)
            hv_ms = time_launches(torch, lambda: mbr.hubbard_apply(h, x, y), 20)
            tsz = 4 if prec == mbr.F32 else 8
            hv[name.split("_")[1]] = {"kernel_ms": hv_ms, "hv_per_s": 1e3 / hv_ms, "launch": shape,
                                      "roofline": hbm_roofline(2.0 * tsz * h.dim, hv_ms,
                                                               f"H·x over all 169 sectors ({2 * tsz} B per row)")}
            # every launch shape of the product, for the record
            shapes = {}
            for G in (-2, -1, 0, 1, 2, 4):
                try:
                    mbr.hubbard_set_config(h, shape["k"], G, 512)
                except mbr.MbrError:
                    continue
                shapes[f"G{G}"] = time_launches(torch, lambda: mbr.hubbard_apply(h, x, y), 10)
            mbr.hubbard_set_config(h, shape["k"], shape["G"], shape["block"])
            hv[name.split("_")[1]]["ms_by_G"] = shapes
            del x, y
        del h
        torch.cuda.synchronize()
    res["hv"] = hv
    v = {k: res[k]["value"] for k in res if isinstance(res[k], dict) and "value" in res[k]}
    res["gain_batching_fp32"] = v["batched_fp32"] / v["per_sector_fp32"]
    res["gain_batching_fp64"] = v["batched_fp64"] / v["per_sector_fp64"]
    res["gain_fp32_batched"] = v["batched_fp32"] / v["batched_fp64"]
    res["gain_fp32_per_sector"] = v["per_sector_fp32"] / v["per_sector_fp64"]
    res["gain_fp32_no_reorth"] = v["batched_fp32_no_reorth"] / v["batched_fp64_no_reorth"]
    res["gain_both"] = v["batched_fp32"] / v["per_sector_fp64"]
    return res


def row_chain(torch, mbr, steps: int):
    """The headline chain (L = 14, (7,7)) with the precisions of the mixed form:
    fp64 vectors without reorthogonalisation (the headline), fp32 vectors with
    fp64 dot products without it, and both with full reorthogonalisation;
    ground energy against the oracle's."""
    import synth
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "hubbard_chain_L14.json")))["e0_exact"]
    res = {"workload": f"chain L=14 U=4 (7,7), {steps} steps, start vector seed {SEED}"}
    for name, prec, reorth in (("fp64", mbr.F64, False), ("fp32", mbr.F32, False),
                               ("fp64_reorth", mbr.F64, True), ("fp32_reorth", mbr.F32, True)):
        h = mbr.hubbard_create(L, chain_bonds(L), [(NUP, NDN)], U=[U] * L, precision=prec)
        mbr.hubbard_autotune(h, reps=5)
        shape = mbr.hubbard_get_config(h)
        v0 = torch.from_numpy(synth.start_vector(SEED, h.dim)).cuda()
        lz = mbr.lanczos_create(h, steps, reorth=reorth, use_graph=True)
        mbr.lanczos_start(lz, v0)
        mbr.lanczos_step(lz, 2)
        mbr.lanczos_start(lz, v0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mbr.lanczos_step(lz, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        e0, _ = mbr.lanczos_result(lz)
        res[name] = {"value": steps / dt, "unit": "Lanczos steps/s", "ms_per_step": dt * 1e3 / steps,
                     "e0": float(e0[0]), "rel_err_vs_oracle": abs(e0[0] - gold) / abs(gold),
                     "launch": {kk: shape[kk] for kk in ("k", "G", "block")}}
        if not reorth:
            x = torch.zeros(h.dim, dtype=torch.float32 if prec == mbr.F32 else torch.float64, device="cuda")
            x.copy_(v0)
            y = torch.empty_like(x)
            res[name]["hv_kernel_ms"] = time_launches(torch, lambda: mbr.hubbard_apply(h, x, y), 20)
            del x, y
        del lz, h
        torch.cuda.synchronize()
    # the plain trie inside H·x: every hop target's 28-bit pattern ranked by a
    # packed trie over the sector (k = 7, four levels), same sums
    for k in (7, 14):
        ht = mbr.hubbard_create(L, chain_bonds(L), [(NUP, NDN)], U=[U] * L, rank_kind=mbr.RANK_TRIE, k=k)
        v0 = torch.from_numpy(synth.start_vector(SEED, ht.dim)).cuda()
        x = v0.clone()
        y = torch.empty_like(x)
        ms = time_launches(torch, lambda: mbr.hubbard_apply(ht, x, y), 10)
        lz = mbr.lanczos_create(ht, steps, use_graph=True)
        mbr.lanczos_start(lz, v0)
        mbr.lanczos_step(lz, 2)
        mbr.lanczos_start(lz, v0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mbr.lanczos_step(lz, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        e0, _ = mbr.lanczos_result(lz)
        res[f"trie_k{k}"] = {"value": steps / dt, "unit": "Lanczos steps/s", "hv_kernel_ms": ms,
                             "hv_per_s": 1e3 / ms, "rel_err_vs_oracle": abs(e0[0] - gold) / abs(gold)}
        del lz, ht, x, y
        torch.cuda.synchronize()
    res["gain_fp32"] = res["fp32"]["value"] / res["fp64"]["value"]
    res["gain_fp32_reorth"] = res["fp32_reorth"]["value"] / res["fp64_reorth"]["value"]
    res["staggered_vs_trie_hv"] = res["trie_k7"]["hv_kernel_ms"] / res["fp64"]["hv_kernel_ms"]
    return res


def row_ceiling(torch, mbr, reps):
    """Measured ceilings for the rooflines: a plain copy of 1 GB (read + write),
    and 2^24 random 4-byte gathers from tables of 1 MB to 4 GB, independent
    (depth 1) and as 4-deep dependent chains like a trie walk, and from a
    64 KB table staged in LDS.  Gathers are reported per second and as HBM
    bandwidth counting one 64-byte granule per gather."""
    nq = 1 << 24
    gen = torch.Generator(device="cuda")
    gen.manual_seed(60)
    idx = torch.randint(0, 1 << 30, (nq,), dtype=torch.int32, device="cuda", generator=gen)
    out = torch.empty(nq, dtype=torch.int32, device="cuda")
    res = {"workload": "2^24 random 4-byte gathers per launch; tables of uniform random entries"}
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ms = time_launches(torch, lambda: b.copy_(a), reps)
    res["copy_1GB"] = {"kernel_ms": ms, "GBs": 2.0 * a.numel() * 4 / (ms * 1e-3) / 1e9}
    del a, b
    for lg in (18, 20, 22, 24, 26, 28, 30):
        tab = torch.randint(0, 1 << 30, (1 << lg,), dtype=torch.int32, device="cuda", generator=gen)
        for depth in (1, 4):
            ms = time_launches(torch, lambda: mbr.probe_gather(tab, idx, depth=depth, out=out), reps)
            g = nq * depth / (ms * 1e-3)
            res[f"{(4 << lg) >> 20}MB_d{depth}"] = {"kernel_ms": ms, "Ggathers_s": g / 1e9,
                                                   "granule_GBs": g * GRANULE / 1e9}
        del tab
        torch.cuda.synchronize()
    tab = torch.randint(0, 1 << 30, (1 << 14,), dtype=torch.int32, device="cuda", generator=gen)
    for depth in (1, 4):
        ms = time_launches(torch, lambda: mbr.probe_gather(tab, idx, depth=depth, lds=True, out=out), reps)
        res[f"lds64KB_d{depth}"] = {"kernel_ms": ms, "Ggathers_s": nq * depth / (ms * 1e-3) / 1e9}
    return res


# --------------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rows", default="all", help="extra workloads: all (" + ",".join(ROWS) + "), none, "
                                                  "or a comma list that may also name " + ",".join(EXTRA_ROWS))
    ap.add_argument("--no-big", action="store_true", help="skip the 165.6M-state learned-index sector")
    ap.add_argument("--k", type=int, default=0, help="half-pattern chunk width (0 = automatic)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--G", type=int, default=None,
                    help="fixed launch shape: alpha_up blocks per tile (0 = alpha_dn-stationary kernel, "
                         "-1 = flat kernel, -2 = block kernel for C_dn > 512); implies --no-tune")
    ap.add_argument("--block", type=int, default=512, help="tile-kernel block size with --G")
    ap.add_argument("--kernel-only", nargs="?", const="chain", choices=("chain", "anderson"),
                    help="only the H·x product of the headline chain (or of the impurity model over all "
                         "169 sectors, fp32) and one plain copy of x for counter calibration; for "
                         "hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the path is built and measured on a single MI355X "
              "(across GPUs, ranking would split the queries, a large sector its alpha_up blocks "
              "with one x exchange per H·x, and the batched impurity model whole sectors)",
              file=sys.stderr)
        sys.exit(2)
    rows = [] if args.rows == "none" else (list(ROWS) if args.rows == "all" else args.rows.split(","))
    for r in rows:
        if r not in ROWS + EXTRA_ROWS:
            ap.error(f"unknown row {r!r}")

    import torch
    import paper_2203_04158_amd as mbr
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.kernel_only == "anderson":
        g = json.load(open(os.path.join(ROOT, "tests", "golden", "anderson_12.json")))
        Ls = 12
        ha = mbr.hubbard_create(Ls, [(0, l + 1, -float(v)) for l, v in enumerate(g["V"])],
                                [(nu, nd) for nu in range(Ls + 1) for nd in range(Ls + 1)],
                                U=[g["U"]] + [0.0] * (Ls - 1), eps=[g["eps_d"]] + g["eps_bath"], precision=mbr.F32)
        if args.G is not None:
            cfg = mbr.hubbard_get_config(ha)
            mbr.hubbard_set_config(ha, k=args.k or cfg["k"], G=args.G, block=args.block)
        x = torch.from_numpy(synth.start_vector(5, ha.dim)).to(device=dev, dtype=torch.float32)
        y = torch.empty_like(x)
        for _ in range(args.kernel_reps):
            mbr.hubbard_apply(ha, x, y)
        y.copy_(x)  # plain copy of dim fp32 values: known traffic for calibration
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": "anderson", "dim": ha.dim, "launch": mbr.hubbard_get_config(ha)}),
              flush=True)
        return
    h = mbr.hubbard_create(L, chain_bonds(L), [(NUP, NDN)], U=[U] * L, precision=mbr.F64, k=args.k)
    if args.G is not None:
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
    del lz

    # dominant kernel: the H·x product, timed with HIP events on this stream
    x = v0.clone()
    y = torch.empty_like(x)
    hv_ms = time_launches(torch, lambda: mbr.hubbard_apply(h, x, y), args.kernel_reps)
    alg_bytes = 16.0 * dim  # x read once + y written once, fp64
    hv_kernel_name = {0: "hv_rows_kernel<double,false,4,true>", -2: "hv_block_kernel<double,false,true>"}
    kname = hv_kernel_name.get(launch_cfg["G"])
    roof = hbm_roofline(alg_bytes, hv_ms, f"{(kname or 'H·x kernel').split('<')[0]} (plain H·x)")
    roof["traffic"] = traffic_for(kname) if kname else None
    # context: with the up-hop gathers counted (8 B per hop changing alpha_up;
    # down-hop sources come from the row staged in LDS) the bytes that must
    # cross L2 per product
    up_hops = L * 2 * math.comb(L - 2, NUP - 1) * math.comb(L, NDN)
    roof["alg_bytes_with_up_gathers"] = alg_bytes + 8.0 * up_hops
    roof["achieved_with_up_gathers"] = roof["alg_bytes_with_up_gathers"] / (hv_ms * 1e-3) / 1e9

    steps = args.steps
    ms_per_step = elapsed * 1e3 / steps
    value = steps / elapsed
    hops = hops_per_product(L, NUP, NDN)
    gold = os.path.join(ROOT, "tests", "golden", "hubbard_chain_L14.json")
    e_ref = json.load(open(gold))["e0_exact"] if os.path.exists(gold) else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Lanczos steps/s",
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
        "hv_per_s": 1e3 / hv_ms,
        "hv_kernel_ms": hv_ms,
        "granks_per_s": value * hops / 1e9,
        # Ritz value after `steps` steps against the converged oracle energy
        # (converges by about 150 steps; the chain row runs 200)
        "ritz_rel_gap_vs_oracle_e0": (abs(e0[0] - e_ref) / abs(e_ref)) if e_ref else None,
        "lanczos_steps_done": int(nsteps[0]),
        "roofline": roof,
    }
    del h, x, y
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    extra = {}
    for r in rows:
        t0 = time.perf_counter()
        if r == "staggered":
            extra[r] = row_staggered(torch, mbr, 50)
        elif r == "unrank":
            extra[r] = row_unrank(torch, mbr, 20)
        elif r == "staggered64":
            extra[r] = row_staggered64(torch, mbr, 20)
        elif r == "trie":
            extra[r] = row_trie(torch, mbr, 20)
        elif r == "learned":
            extra[r] = row_learned(torch, mbr, 20, big=not args.no_big)
        elif r == "chain":
            extra[r] = row_chain(torch, mbr, 200)
        elif r == "batched":
            extra[r] = row_batched(torch, mbr, 150)
        elif r == "operator":
            extra[r] = row_operator(torch, mbr, 5)
        elif r == "ceiling":
            extra[r] = row_ceiling(torch, mbr, 10)
        elif r == "sweep":
            extra[r] = row_sweep(torch, mbr, 10)
        extra[r]["wall_s"] = time.perf_counter() - t0
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        print(f"[bench] row {r} done in {extra[r]['wall_s']:.1f} s", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    if extra:
        out["rows"] = summarize(extra)   # last, so that a tail of the line holds every workload
    print("[bench] detail " + json.dumps({"headline": out, "rows": extra}), file=sys.stderr, flush=True)
    line = _round(out)
    line["roofline"].pop("kernel", None)
    if "cpu_baseline" in line:
        line["cpu_baseline"].pop("rank_Granks_m24_n12_2e22", None)
        line["cpu_baseline"]["sample"] = (f"plain bisection gather-form H·x (oracle, fp64) on rows of the headline "
                                          f"sector, {line['cpu_baseline']['cores']} threads, scaled to whole products")
    print(json.dumps(line, separators=(",", ":")), flush=True)


def _round(v, digits: int = 4):
    """Floats to `digits` significant digits, for a short line."""
    if isinstance(v, float):
        return float(f"{v:.{digits}g}") if math.isfinite(v) else v
    if isinstance(v, dict):
        return {k: _round(x, digits) for k, x in v.items()}
    if isinstance(v, list):
        return [_round(x, digits) for x in v]
    return v


def summarize(extra: dict) -> dict:
    """One short entry per workload for the JSON line (the full records go to
    stderr): throughput, roofline fraction and exactness, short keys."""
    s = {}
    r3 = lambda d, keys: {k: d[k]["value"] for k in keys if k in d}  # noqa: E731
    if "staggered" in extra:
        e = extra["staggered"]
        s["cfg1_stag"] = {"Grk_s": e["value"], "frac": e["roofline"]["frac"], "exact": e["exact"],
                          "2e28_frac": e["stress_2e28"]["roofline"]["frac"]}
        if "autotuned" in e:
            s["cfg1_stag"]["tuned_k"] = e["autotuned"]["k"]
    if "unrank" in extra:
        e = extra["unrank"]
        s["unrank_G_s"] = {k: e[k]["value"] for k in ("list_chain_7x7", "spin_chain_7x7") if k in e}
    if "staggered64" in extra:
        s["m64_stag_Grk_s"] = {k: extra["staggered64"][k]["value"] for k in ("k5", "k8")}
    if "trie" in extra:
        e = extra["trie"]
        s["cfg3"] = {k: [e[k]["value"], e[k]["roofline"]["frac"]] for k in ("k8", "bitmap_k8") if k in e}
        s["cfg3"]["k4"] = e["k4"]["value"]
        s["cfg3"]["no_net"] = e["sampled_search_no_net"]["value"]
        s["cfg3"]["exact"] = all(e[k]["exact"] for k in ("k4", "k8", "bitmap_k4", "bitmap_k8") if k in e)
    if "learned" in extra:
        for name, r in extra["learned"].items():
            if isinstance(r, dict) and "learned" in r:
                t = r3(r, ("learned", "sampled_search_no_net", "trie_k8", "bitmap_trie_k8", "spin_staggered"))
                t["exact"] = all(r[k]["exact"] for k in ("learned", "sampled_search_no_net", "trie_k8",
                                                         "bitmap_trie_k8") if k in r)
                if "mlp_forward" in r:
                    t["mlp_frac"] = r["mlp_forward"]["roofline"]["frac"]
                s["cfg4_" + ("chain" if "chain" in name else "8x8")] = t
    if "chain" in extra:
        e = extra["chain"]
        s["cfg2_steps_s"] = {k: e[k]["value"] for k in ("fp64", "fp32", "fp64_reorth", "fp32_reorth",
                                                        "trie_k14")}
        s["cfg2_fp32_err"] = e["fp32"]["rel_err_vs_oracle"]
        s["cfg2_hv_ms"] = {"stag": e["fp64"]["hv_kernel_ms"], "trie_k14": e["trie_k14"]["hv_kernel_ms"]}
    if "batched" in extra:
        e = extra["batched"]
        s["cfg5_steps_s"] = {k: e[k]["value"] for k in e if isinstance(e[k], dict) and "value" in e[k]}
        s["cfg5_err"] = max(e[k]["worst_rel_err_vs_oracle"] for k in e
                            if isinstance(e[k], dict) and "worst_rel_err_vs_oracle" in e[k])
        s["cfg5_hv"] = {k: [v["kernel_ms"], v["roofline"]["frac"]] for k, v in e["hv"].items()}
    if "operator" in extra:
        s["kring_hv_s"] = extra["operator"]["trie_k14"]["value"]
    if "ceiling" in extra:
        e = extra["ceiling"]
        s["ceil_GBs"] = {"copy": e["copy_1GB"]["GBs"], "g4MB": e["4MB_d1"]["granule_GBs"],
                         "g256MB": e["256MB_d1"]["granule_GBs"], "g4GB": e["4096MB_d1"]["granule_GBs"]}
    if "sweep" in extra:
        s["sweep_n14_Grk_s"] = extra["sweep"]["half_filled_granks_per_s"]
        s["sweep_exact"] = extra["sweep"]["exact"]
    return s


if __name__ == "__main__":
    main()
