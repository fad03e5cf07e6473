"""Benchmark of the BCFW hot path on one MI355X.

Workload: m = n = 4096 points from the seeded 8-Gaussian RGB mixture, cost
stored in FP32 (64 MiB), uniform a, b, penalty weights w in {0.1, 1, 10},
ELS step, uniform sampling.  One benchmark "step" is one pass of the hot
path: m block updates (sample, gradient row, LMO, line search, update of t_i
and r) followed by the gap sweep and the stop test read back on the host.
Inputs are resident in HBM before timing starts.

Prints one JSON line: block-updates/s over the timed passes (all three w),
the chain kernel's roofline figures, the time to reach gap 1e-6 from the
initial plan for each w, and the CPU oracle's rate on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_GFLOPS = 78600.0      # MI355X dense FP64 vector
FP32_PEAK_GFLOPS = 157300.0     # MI355X dense FP32 vector
CSRC = os.path.join(ROOT, "paper_2103_05857_amd", "csrc")
KERNELS_SRC = [os.path.join(CSRC, f) for f in ("srot_kernels.hip", "srot_device.h", "srot_screen.hip")]
FUSED_SRC = [os.path.join(CSRC, f) for f in ("srot_team.hip", "srot_kernels.hip", "srot_device.h")]
PROFILE = os.path.join(ROOT, "profiles", "chain_gap_stored_f32_m4096_n4096.md")
SWEEP_PROFILE = os.path.join(ROOT, "profiles", "gap_sweep_stored_f32_m16384_n16384.md")
FUSED_PROFILE = os.path.join(ROOT, "profiles", "chain_gap_fused_m32768_n32768.md")


def profile_counters(profile, sources, kernel_prefix):
    """Per-dispatch counters of a kernel from a committed rocprofv3 summary,
    or None when the summary is absent or its kernels changed since."""
    import hashlib
    import re
    try:
        text = open(profile).read()
        blob = json.loads(re.findall(r"```json\n(.*?)\n```", text, flags=re.S)[-1])
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in sources)).hexdigest()[:16]
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("kernels_sha256") != sha:
        return None
    for name, v in blob["per_dispatch"].items():
        if name.startswith(kernel_prefix):
            return dict(v, fetch_scale=blob.get("fetch_scale"), write_scale=blob.get("write_scale"))
    return None


def fp32_counted_flops(c):
    """FP32 flops of one dispatch from the VALU instruction counters."""
    if not c or "SQ_INSTS_VALU_FMA_F32" not in c:
        return None
    return 64.0 * (2.0 * c["SQ_INSTS_VALU_FMA_F32"] + c["SQ_INSTS_VALU_ADD_F32"] + c["SQ_INSTS_VALU_MUL_F32"])


def fp64_counted_flops(c):
    """FP64 flops of one dispatch from the VALU instruction counters (64 lanes
    per instruction, an FMA counting two)."""
    if not c or "SQ_INSTS_VALU_FMA_F64" not in c:
        return None
    return 64.0 * (2.0 * c["SQ_INSTS_VALU_FMA_F64"] + c["SQ_INSTS_VALU_ADD_F64"] + c["SQ_INSTS_VALU_MUL_F64"])


def counter_traffic(kernel_prefix, profile=PROFILE, grid=None):
    """HBM bytes per dispatch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel factors), or
    None when the summary is absent or the kernel source changed since."""
    import hashlib
    import re
    try:
        text = open(profile).read()
        blob = json.loads(re.findall(r"```json\n(.*?)\n```", text, flags=re.S)[-1])
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNELS_SRC)).hexdigest()[:16]
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("kernels_sha256") != sha:
        return None
    for name, v in blob["per_dispatch"].items():
        if name.startswith(kernel_prefix) and (grid is None or name.endswith(f"[grid {grid}]")):
            fetch = v.get("fetch_kib", v.get("FETCH_SIZE"))
            write = v.get("write_kib", v.get("WRITE_SIZE"))
            if fetch is None or write is None:
                return None
            return 1024.0 * (fetch * blob["fetch_scale"] + write * blob["write_scale"])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed passes per penalty weight")
    ap.add_argument("--warmup", type=int, default=3, help="untimed passes per penalty weight")
    ap.add_argument("--m", type=int, default=4096)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--weights", type=str, default="0.1,1,10")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ttg", action="store_true", help="skip the time-to-gap solves")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--sections", type=str, default="sweep,fw,variants,batched,diff,fused",
                    help="extra workloads after the stored-cost one: sweep, fw, variants, batched, diff, fused")
    ap.add_argument("--sweep-n", type=int, default=16384)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--seq-sample", type=int, default=64,
                    help="problems of the batch solved one by one for the sequential baseline")
    ap.add_argument("--fused-n", type=int, default=32768)
    ap.add_argument("--fused-seconds", type=float, default=60.0,
                    help="time cap of the fused-cost solve")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the BCFW chain does not shard across GPUs); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2103_05857_amd import inputs as I
    from paper_2103_05857_amd import srot as S

    dev = torch.device("cuda:0")
    m, n = args.m, args.n
    weights = [float(x) for x in args.weights.split(",")]
    d = I.problem_mixture(0, m, n, cost_dtype=np.float32)
    C = torch.from_numpy(d["C"]).to(dev)
    a = torch.from_numpy(d["a"]).to(dev)
    b = torch.from_numpy(d["b"]).to(dev)
    torch.cuda.synchronize()

    total_updates = 0
    total_s = 0.0
    chain_ms = []          # event-timed srot_step(m) launches (sample + chain kernel)
    gap_ms = []            # event-timed gap sweeps (gap kernel + final reduction)
    nnz_rows = []
    screen_stats = {}
    ttg = {}
    for w in weights:
        sol = S.Solver(a, b, C=C, w=w, seed=0, eps=1e-6, max_passes=1, gap_every=1)
        stream = torch.cuda.current_stream()
        for _ in range(args.warmup):
            S.srot_step(sol.h, m)
            S.srot_gap(sol.h)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        evg = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        out5 = torch.empty(5, dtype=torch.float64, device=dev)
        t0 = time.perf_counter()
        for p in range(args.steps):
            ev[p][0].record(stream)
            S.srot_step(sol.h, m)            # one pass of m block updates
            ev[p][1].record(stream)
            S.srot_gap_async(sol.h, out5)    # gap sweep
            evg[p].record(stream)
            evg[p].synchronize()
            _ = out5[0].item()               # stop-test readback
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        total_updates += args.steps * m
        total_s += dt
        chain_ms += [e0.elapsed_time(e1) for e0, e1 in ev]
        gap_ms += [ev[p][1].elapsed_time(evg[p]) for p in range(args.steps)]
        st = S.srot_chain_stats(sol.h)      # the last timed pass
        screen_stats[str(w)] = dict(full_row_lmo=st[0], support_reread=st[1], steps=m)
        T, _ = sol.plan()
        nnz_rows.append(float((T > 0).sum().item()) / m)
        sol.close()
        del T
        if not args.no_ttg:
            sol = S.Solver(a, b, C=C, w=w, seed=0, eps=1e-6, max_passes=5000, gap_every=1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            status, (g, f, D), passes = sol.solve()
            torch.cuda.synchronize()
            ttg[str(w)] = dict(seconds=time.perf_counter() - t1, passes=passes, gap=g, f=f,
                               converged=(status == S.SROT_OK))
            sol.close()

    value = total_updates / total_s
    ms_per_step = 1000.0 * total_s / (args.steps * len(weights))
    chain_avg_ms = float(np.mean(chain_ms))
    # algorithmic bytes per block step: the FP32 cost row (4n) plus the sparse
    # plan row read and written (int32 index + FP64 value, nnz + 1 entries);
    # one srot_step(m) launch runs m of them
    nnz = float(np.mean(nnz_rows))
    bytes_per_step = 4.0 * n + 24.0 * (nnz + 1.0)
    achieved = bytes_per_step * m / (chain_avg_ms * 1e-3) / 1e9
    traffic = counter_traffic("srot::chain_screened_kernel<16, false, 0>")
    roofline = dict(kernel="chain_screened_kernel<16,f32>", bound="hbm", achieved=achieved,
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, bytes_per_launch=bytes_per_step * m, launch_ms=chain_avg_ms,
                    us_per_block_update=1000.0 * chain_avg_ms / m)
    # the once-per-pass gap sweep streams the whole cost: 4mn bytes of C, the
    # plan's support (12 bytes per nonzero), a, b and the per-row outputs
    gap_avg_ms = float(np.median(gap_ms))
    gap_bytes = 4.0 * m * n + 12.0 * nnz * m + 8.0 * (3 * m + n)
    gap_achieved = gap_bytes / (gap_avg_ms * 1e-3) / 1e9
    gap_sweep = dict(kernel="gap_stream_kernel<f32,2,2> + gap_final_kernel", bound="hbm",
                     achieved=gap_achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                     frac=gap_achieved / HBM_PEAK_GBS, bytes_per_launch=gap_bytes,
                     launch_ms=gap_avg_ms,
                     traffic=counter_traffic("srot::gap_stream_kernel<0, 2, 2, false, false>"))

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(d, m, weights[min(1, len(weights) - 1)], args.cpu_seconds)

    out = {
        "metric": "BCFW block-updates/sec + C-stream GB/s (% HBM peak); time-to-gap 1e-6 vs plain",
        "value": value, "unit": "block-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (FP32-stored cost)", "data": "synthetic",
        "config": {"workload": f"bcfw_stored_f32_mixture_m{m}_n{n}", "m": m, "n": n,
                   "weights": weights, "cost": "squared Euclidean, stored FP32",
                   "step": "one pass = m block updates + gap sweep + stop test"},
        "roofline": roofline,
        "c_stream": {"chain_GBps": achieved, "chain_frac": achieved / HBM_PEAK_GBS,
                     "gap_sweep": gap_sweep},
        "cpu_baseline": cpu,
        "time_to_gap_1e-6": ttg,
        "mean_row_nnz": nnz,
        "screened_lmo_last_pass": screen_stats,
    }
    sections = [x for x in args.sections.split(",") if x]
    if "sweep" in sections:
        out["gap_sweep_1GiB"] = bench_sweep(args)
    if "fw" in sections:
        out["full_fw"] = bench_fw(args, C, a, b)
    if "variants" in sections:
        out["variants_time_to_gap_1e-6"] = bench_variants(args, C, a, b)
    if "batched" in sections:
        out["batched"] = bench_batched(args)
    if "diff" in sections:
        out["differentiation"] = bench_diff(args)
    if "fused" in sections:
        out["fused"] = bench_fused(args)
    print(json.dumps(out))


def bench_sweep(args):
    """The per-pass gap sweep on a cost larger than the 256 MB Infinity Cache:
    m = n = 16384 mixture points, FP32 stored cost (1 GiB), after one pass of
    block steps from the initial plan; sweep plus final-sum kernel time from
    HIP events around srot_gap_async on the solver's stream (a device
    destination: no copy)."""
    import torch
    from paper_2103_05857_amd import inputs as I
    from paper_2103_05857_amd import srot as S
    dev = torch.device("cuda:0")
    n = args.sweep_n
    d = I.problem_mixture(0, n, n, with_cost=False)
    X = torch.from_numpy(d["X"]).to(dev).double()
    Y = torch.from_numpy(d["Y"]).to(dev).double()
    C = torch.empty(n, n, dtype=torch.float32, device=dev)
    for i0 in range(0, n, 2048):
        C[i0:i0 + 2048] = ((X[i0:i0 + 2048, None, :] - Y[None, :, :]) ** 2).sum(-1).float()
    del X, Y
    a = torch.from_numpy(d["a"]).to(dev)
    b = torch.from_numpy(d["b"]).to(dev)
    sol = S.Solver(a, b, C=C, w=1.0, seed=0)
    stream = torch.cuda.current_stream()
    # one pass of block steps on the stored 16384-column rows (the team chain)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    S.srot_step(sol.h, n)
    c1.record(stream)
    c1.synchronize()
    chain_us = 1000.0 * c0.elapsed_time(c1) / n
    out5 = torch.empty(5, dtype=torch.float64, device=dev)
    for _ in range(3):
        S.srot_gap_async(sol.h, out5)
    torch.cuda.synchronize()
    ms = []
    for _ in range(10):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        S.srot_gap_async(sol.h, out5)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    T, _ = sol.plan()
    nnz = int((T > 0).sum().item())
    del T
    sol.close()
    t = float(np.median(ms)) * 1e-3
    # algorithmic bytes: the cost once (4 m n), the plan's support (index +
    # value, 12 B per nonzero), r, b, a and the per-row outputs
    byts = 4.0 * n * n + 12.0 * nnz + 8.0 * (3 * n + 3 * n)
    # full FW (Alg. A.1) on the same cost: one sweep launch per iteration
    fw = S.Solver(a, b, C=C, w=1.0, seed=0)
    S.srot_fw_steps(fw.h, 3)
    torch.cuda.synchronize()
    f0 = torch.cuda.Event(enable_timing=True)
    f1 = torch.cuda.Event(enable_timing=True)
    iters = 20
    f0.record(stream)
    S.srot_fw_steps(fw.h, iters)
    f1.record(stream)
    f1.synchronize()
    fw_s = f0.elapsed_time(f1) * 1e-3 / iters
    Tf, _ = fw.plan()
    fw_nnz = int((Tf > 0).sum().item())
    del Tf
    fw.close()
    fw_bytes = 4.0 * n * n + 24.0 * fw_nnz + 8.0 * (3 * n + 4 * n)
    return {"workload": f"gap sweep, m=n={n} FP32 stored cost (1 GiB), after one pass",
            "kernel": "gap_stream_kernel<f32,4,1,rotated> + gap_final_kernel", "bound": "hbm",
            "us": t * 1e6, "bytes": byts, "achieved": byts / t / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": byts / t / 1e9 / HBM_PEAK_GBS,
            "traffic": counter_traffic("srot::gap_stream_kernel<0, 4, 1, false, true>", SWEEP_PROFILE,
                                       grid=512 * 256),
            "chain_us_per_block_update_first_pass": chain_us,
            "full_fw": {"workload": f"full FW, m=n={n}, FP32 stored cost (1 GiB), w=1, ELS, iterations 4-23",
                        "us_per_iteration": fw_s * 1e6, "bytes_per_iteration": fw_bytes,
                        "achieved": fw_bytes / fw_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": fw_bytes / fw_s / 1e9 / HBM_PEAK_GBS}}


def bench_fw(args, C, a, b):
    """Full Frank-Wolfe (Alg. A.1) on the stored-cost workload (w = 1): the
    time of one iteration (gap sweep, vertex column sums, line search,
    update) from HIP events around srot_fw_steps, and its stream rate."""
    import torch
    from paper_2103_05857_amd import srot as S
    m, n = C.shape
    sol = S.Solver(a, b, C=C, w=1.0, seed=0)
    S.srot_fw_steps(sol.h, 5)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    iters = 100
    e0.record(stream)
    S.srot_fw_steps(sol.h, iters)
    e1.record(stream)
    e1.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / iters
    g, f, D = sol.gap()
    T, _ = sol.plan()
    nnz = int((T > 0).sum().item())
    del T
    sol.close()
    # per iteration: the cost streamed once (4mn), the plan's support read and
    # written (24 B per nonzero), the vertex indices, r, b and s
    byts = 4.0 * m * n + 24.0 * nnz + 4.0 * m + 8.0 * 4 * n
    return {"workload": f"full FW, m=n={m}, FP32 stored cost, w=1, ELS", "us_per_iteration": t * 1e6,
            "bytes_per_iteration": byts, "achieved": byts / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": byts / t / 1e9 / HBM_PEAK_GBS, "gap_after_105_iterations": g}


def bench_variants(args, C, a, b):
    """Time to gap 1e-6 from the initial plan on the stored-cost workload
    (w = 1, gap every pass): plain BCFW (Alg. 1) with uniform and with
    per-pass permutation sampling, the away-step (Alg. A.2) and pairwise
    (Alg. A.3) block steps, gap-adaptive sampling (Alg. A.4, global update
    every pass) and full FW (Alg. A.1, gap at every iteration; "passes"
    counts its iterations)."""
    import torch
    from paper_2103_05857_amd import srot as S
    out = {}

    def run(sol, variant):
        if variant is None or variant == "perm":
            return sol.solve()
        if variant == "fw":
            return S.srot_fw_solve(sol.h)    # passes = FW iterations
        if variant == "ga":
            return S.srot_solve_ga(sol.h, 0.0, 1)
        return S.srot_solve_variant(sol.h, variant)

    for name, variant in (("bcfw", None), ("bcfw_permutation", "perm"), ("away", S.SROT_STEP_AWAY),
                          ("pairwise", S.SROT_STEP_PAIRWISE), ("gap_adaptive", "ga"), ("full_fw", "fw")):
        sampling = S.SROT_PERMUTE if variant == "perm" else S.SROT_UNIFORM
        # untimed: one pass (iteration) on a handle of its own, so that the
        # timed solve does not pay for the first use of its kernels
        warm = S.Solver(a, b, C=C, w=1.0, seed=0, eps=1e-6, max_passes=1, sampling=sampling)
        run(warm, variant)
        warm.close()
        sol = S.Solver(a, b, C=C, w=1.0, seed=0, eps=1e-6, max_passes=2000, sampling=sampling)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, (g, f, D), passes = run(sol, variant)
        torch.cuda.synchronize()
        out[name] = dict(seconds=time.perf_counter() - t0, passes=passes, gap=g, f=f,
                         converged=(st == S.SROT_OK))
        sol.close()
    return out


def bench_batched(args):
    """512 problems, m and n each log-uniform in [64, 4096], mixture palettes,
    FP32 stored cost, uniform weights, w = 1, every problem to gap 1e-6: one
    batched graph launch (autotuned tile shapes) against the single-problem
    solver run on the problems one after another (a sample, extrapolated by
    block updates)."""
    import torch
    from paper_2103_05857_amd import inputs as I
    from paper_2103_05857_amd import srot as S
    dev = torch.device("cuda:0")
    count = args.batch_count
    ms, ns = I.batched_sizes(0, count)
    Cs, As, Bs = [], [], []
    for p in range(count):
        d = I.batched_problem(0, p, int(ms[p]), int(ns[p]))
        X = torch.from_numpy(d["X"]).to(dev).double()
        Y = torch.from_numpy(d["Y"]).to(dev).double()
        Cs.append(((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1).float())
        As.append(torch.from_numpy(d["a"]).to(dev))
        Bs.append(torch.from_numpy(d["b"]).to(dev))
    torch.cuda.synchronize()
    opts = dict(w=1.0, eps=1e-6, max_passes=20000, seed=0)
    t0 = time.perf_counter()
    bs = S.BatchSolver(Cs, As, Bs, tune=True, **opts)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    # the first solve starts the largest problems first; later solves start
    # the previous solve's longest-running problems first
    t0 = time.perf_counter()
    bs.solve()
    first_s = time.perf_counter() - t0
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        st, out3, passes, status = bs.solve()
        times.append(time.perf_counter() - t0)
    tiles, tune_ms = bs.tiles()
    bs.close()
    # the same batch initialised again: tiles from the tuning cache
    t0 = time.perf_counter()
    bs2 = S.BatchSolver(Cs, As, Bs, tune=True, **opts)
    torch.cuda.synchronize()
    init_warm_s = time.perf_counter() - t0
    tiles2, _ = bs2.tiles()
    bs2.close()
    solve_s = float(np.median(times))
    # the straggler (most block steps) and its floor: the same problem alone
    # on the single-problem solver, which picks its fastest chain
    sp = int(np.argmax(passes * ms))
    sol = S.Solver(As[sp], Bs[sp], C=Cs[sp], **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, sp_passes = sol.solve()
    floor_s = time.perf_counter() - t0
    sp_kind = S.srot_chain_stats(sol.h)[2]
    sol.close()
    straggler = {"problem": sp, "m": int(ms[sp]), "n": int(ns[sp]), "passes": int(passes[sp]),
                 "batch_tile": "x".join(str(int(v)) for v in tiles[sp]),
                 "batch_us_per_block_update": 1e3 * float(tune_ms[sp]) if tune_ms[sp] > 0 else None,
                 "alone_seconds": floor_s, "alone_passes": int(sp_passes), "alone_chain_kind": int(sp_kind),
                 "alone_us_per_block_update": 1e6 * floor_s / (sp_passes * int(ms[sp])),
                 "batch_wall_over_floor": solve_s / floor_s}
    updates = int((passes * ms).sum())
    # cost bytes streamed: a row of 4n bytes per block step, 4mn per gap sweep
    cbytes = float((passes * ms * 4 * ns).sum() + (passes * 4 * ms * ns).sum())
    seq_s, seq_updates = 0.0, 0
    k = min(args.seq_sample, count)
    for p in range(k):
        sol = S.Solver(As[p], Bs[p], C=Cs[p], **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, np1 = sol.solve()
        seq_s += time.perf_counter() - t0
        seq_updates += np1 * int(ms[p])
        sol.close()
    seq_rate = seq_updates / seq_s
    uniq, cnt = np.unique(tiles, axis=0, return_counts=True)
    return {
        "workload": f"{count} problems, m,n log-uniform in [64,4096], FP32 stored cost, w=1, gap<=1e-6",
        "converged": int((status == 0).sum()), "seconds": solve_s, "first_solve_seconds": first_s,
        "block_updates": updates, "block_updates_per_s": updates / solve_s,
        "c_stream_GBps": cbytes / solve_s / 1e9, "c_stream_frac_hbm": cbytes / solve_s / 1e9 / HBM_PEAK_GBS,
        "passes_mean": float(passes.mean()), "passes_max": int(passes.max()),
        "init_and_autotune_s": init_s, "init_cached_tiles_s": init_warm_s,
        "cached_tiles_match": bool(np.array_equal(tiles, tiles2)), "straggler": straggler,
        "tiles": {f"{a}x{b}x{c}": int(n_) for (a, b, c), n_ in zip(uniq.tolist(), cnt.tolist())},
        "sequential": {"sample_problems": k, "seconds": seq_s, "block_updates_per_s": seq_rate,
                       "extrapolated_seconds_all": updates / seq_rate},
        "speedup_vs_sequential": (updates / seq_rate) / solve_s,
    }


def bench_diff(args):
    """Differentiation: m = n = 4096 mixture points (fused squared-Euclidean
    cost), w = 1, V = optimal value solved to gap 1e-6; forward alone against
    forward plus backward (dX, dY, da, db through srot_backward)."""
    import torch
    from paper_2103_05857_amd import inputs as I
    from paper_2103_05857_amd.autograd import semi_relaxed_ot
    dev = torch.device("cuda:0")
    d = I.problem_mixture(0, 4096, 4096, with_cost=False)
    X0 = torch.from_numpy(d["X"]).to(dev)
    Y0 = torch.from_numpy(d["Y"]).to(dev)
    a0 = torch.from_numpy(d["a"]).to(dev)
    b0 = torch.from_numpy(d["b"]).to(dev)
    fwd, both = [], []
    for rep in range(3):
        X = X0.clone().requires_grad_(True)
        Y = Y0.clone().requires_grad_(True)
        a = a0.clone().requires_grad_(True)
        b = b0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        V = semi_relaxed_ot(a, b, X=X, Y=Y, w=1.0, eps=1e-6, max_passes=5000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        V.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwd.append(t1 - t0)
        both.append(t2 - t0)
    return {"workload": "m=n=4096 mixture points, fused cost, w=1, V solved to gap 1e-6",
            "forward_s": float(np.median(fwd)), "forward_backward_s": float(np.median(both)),
            "backward_s": float(np.median(np.array(both) - np.array(fwd)))}


def bench_fused(args):
    """Fused on-the-fly cost: m = n = 32768 mixture points (the cost, 4 GiB in
    FP32, is never stored), a uniform, b ~ Dirichlet(1), w = 1, run to gap
    1e-5 or the time cap.  Rooflines against the FP64 vector peak (the chain
    and the sweep evaluate every cost entry in FP64): algorithmic flops per
    launch over the event-timed launch, with the counted flops and the VALU
    share from the committed rocprofv3 summary."""
    import torch
    from paper_2103_05857_amd import inputs as I
    from paper_2103_05857_amd import srot as S
    dev = torch.device("cuda:0")
    n = args.fused_n
    d = I.problem_mixture(0, n, n, dirichlet_b=True, with_cost=False)
    X = torch.from_numpy(d["X"]).to(dev)
    Y = torch.from_numpy(d["Y"]).to(dev)
    a = torch.from_numpy(d["a"]).to(dev)
    b = torch.from_numpy(d["b"]).to(dev)
    sol = S.Solver(a, b, X=X, Y=Y, w=1.0, seed=0, eps=1e-5)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    hist = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    out5 = torch.empty(5, dtype=torch.float64, device=dev)
    step_ms, gap_ms = [], []
    t0 = time.perf_counter()
    g = float("inf")
    passes = 0
    while time.perf_counter() - t0 < args.fused_seconds:
        e0.record(stream)
        S.srot_step(sol.h, n)
        e1.record(stream)
        S.srot_gap_async(sol.h, out5)
        e2.record(stream)
        e2.synchronize()
        g = float(out5[0].item())
        step_ms.append(e0.elapsed_time(e1))
        gap_ms.append(e1.elapsed_time(e2))
        passes += 1
        hist.append((passes, g))
        if g <= 1e-5:
            break
    wall = time.perf_counter() - t0
    kind = S.srot_chain_stats(sol.h)[2]
    sol.close()
    launch_ms = float(np.median(step_ms))
    sweep_ms = float(np.median(gap_ms))
    # one launch = n block steps; per step n cost evaluations of 10 FP64
    # flops (three differences, a product and two FMAs for the squared
    # distance, an FMA for + w r_j); the sweep screens all m n entries once
    # with the same 10 flops in FP32 (exact FP64 values only for the few
    # columns near each row's minimum)
    chain_flops = 10.0 * n * n
    sweep_flops = 10.0 * n * n
    cc = profile_counters(FUSED_PROFILE, FUSED_SRC, "srot::chain_team_kernel<2, false>")
    cs = profile_counters(FUSED_PROFILE, FUSED_SRC, "srot::gap_sweep_kernel<2, 1, 4")

    def valu_share(c):
        if not c or not c.get("SQ_WAVE_CYCLES"):
            return None
        return c["SQ_ACTIVE_INST_VALU"] / c["SQ_WAVE_CYCLES"]

    chain_ach = chain_flops / (launch_ms * 1e-3) / 1e9
    sweep_ach = sweep_flops / (sweep_ms * 1e-3) / 1e9
    roofline = dict(kernel="chain_team_kernel<sqeuclid>", bound="valu", achieved=chain_ach,
                    peak=FP64_PEAK_GFLOPS, unit="GFLOP/s (FP64)", frac=chain_ach / FP64_PEAK_GFLOPS,
                    flops_per_launch=chain_flops, launch_ms=launch_ms,
                    counted_flops_per_launch=fp64_counted_flops(cc),
                    valu_active_share_of_wave_cycles=valu_share(cc),
                    note="latency-bound: one record exchange between the team's workgroups per block step")
    sweep = dict(kernel="gap_sweep_kernel<sqeuclid> (FP32 screen) + gap_final_kernel", bound="valu",
                 achieved=sweep_ach, peak=FP32_PEAK_GFLOPS, unit="GFLOP/s (FP32)", frac=sweep_ach / FP32_PEAK_GFLOPS,
                 flops_per_launch=sweep_flops, launch_ms=sweep_ms,
                 counted_fp32_flops_per_launch=fp32_counted_flops(cs),
                 counted_fp64_flops_per_launch=fp64_counted_flops(cs),
                 valu_active_share_of_wave_cycles=valu_share(cs))
    return {"workload": f"m=n={n} mixture points, fused squared-Euclidean cost, b~Dirichlet(1), w=1, "
                        f"to gap 1e-5 (cap {args.fused_seconds:.0f} s)",
            "chain_kind": kind, "passes": passes, "gap": g, "converged": bool(g <= 1e-5), "seconds": wall,
            "us_per_block_update": 1000.0 * launch_ms / n, "block_updates_per_s": n / (launch_ms * 1e-3),
            "roofline": roofline, "gap_sweep": sweep,
            "gap_history": hist[:: max(1, len(hist) // 10)]}


def host_cpu():
    """Logical CPUs and model name of the host the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(d, m, w, seconds):
    """The FP64 oracle, single thread, on the same workload and the same
    block-index stream as the GPU: whole passes (m block steps + gap) until
    the gap reaches 1e-6 or about `seconds` of CPU time (value = block
    updates per second over that run), then the small configuration
    (m = n = 256 uniform points, FP64 cost, w = 1) run in full: 500 passes."""
    from oracle import oracle as O
    from paper_2103_05857_amd import inputs as I
    P = O.Problem(d["a"], d["b"], w, C=d["C"].astype(np.float64))
    st = O.State(P)
    t0 = time.perf_counter()
    passes, g = 0, float("inf")
    while time.perf_counter() - t0 < seconds and passes < 2000:
        O.bcfw_steps(P, st, I.philox_uniform_indices(0, passes * m, m, m), trace=False)
        g = O.gap(P, st.T)["g"]
        passes += 1
        if g <= 1e-6:
            break
    dt = time.perf_counter() - t0
    c1 = I.problem_uniform_c1(0, 256, 256)
    P1 = O.Problem(c1["a"], c1["b"], 1.0, C=c1["C"])
    s1 = O.State(P1)
    t1 = time.perf_counter()
    for p in range(500):
        O.bcfw_steps(P1, s1, I.philox_uniform_indices(0, p * 256, 256, 256), trace=False)
    g1 = O.gap(P1, s1.T)["g"]
    c1_s = time.perf_counter() - t1
    return dict(value=passes * m / dt, unit="block-updates/s", cores=1, kind="oracle",
                sample=f"{passes} passes of the {m} x {m} stored-cost workload at w={w} "
                       f"({'reached gap 1e-6' if g <= 1e-6 else f'stopped at the {seconds:.0f} s cap'}, "
                       f"gap {g:.3e}), {dt:.1f} s, single-threaded FP64 C oracle, same index stream as the GPU",
                time_to_gap_1e6_s=(dt if g <= 1e-6 else None), passes=passes,
                small_config_500_passes_s=c1_s, small_config_gap=g1, host=host_cpu())


if __name__ == "__main__":
    main()
