"""Benchmark: CG-SENSE on one MI355X, reported as E^H E applies per second.

Workload (default): 160 independent 2D slices of 256x256 with 12 coils and
their own sensitivity maps, variable-density mask R=4 with 24 centre lines,
30 CG iterations per solve, complex64 storage with fp64 inner products.
One step = one full solve of the batch (E^H y, CG init, 30 x [fused E^H E
with the p update, x/r update], finish).  Inputs are seeded synthetic
phantoms, coil maps, mask and noise, resident in HBM before timing.

Prints one JSON line with the metric, the roofline of the dominant kernel
(the fused E^H E launch, timed with HIP events on its stream inside the
timed region) and the FP64 oracle timed on the host for a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# HBM traffic of the fused kernel comes from rocprofv3 FETCH_SIZE/WRITE_SIZE
# runs recorded under profiles/; it is reported only while the kernel sources
# still hash to what was measured.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cgsense_256x256_c12_b160_k30.traffic.json")
EHE_SOURCES = ["kernels_ehe.hip", "fft_engine.hpp", "dft_small.hpp", "cplx.hpp", "bufio.hpp", "xcd.hpp",
               "lengths.hpp", "reduce.hpp", "kernels.hpp", "cg_scalar.hpp"]


def measured_traffic(kernel_key):
    import hashlib

    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except OSError:
        return None
    h = hashlib.sha256()
    for name in rec.get("kernel_sources", EHE_SOURCES):
        path = os.path.join(ROOT, "paper_1807_11830_amd", "csrc", name)
        if os.path.exists(path):
            h.update(name.encode())
            with open(path, "rb") as f:
                h.update(f.read())
    if h.hexdigest() != rec.get("kernel_sources_sha256"):
        return None
    k = rec.get("kernels", {}).get(kernel_key)
    return None if k is None else k["traffic_bytes"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=160)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--maps-storage", default="c64", choices=["c64", "bf16", "fp16"])
    ap.add_argument("--workload", default="cgsense", choices=["cgsense", "serving", "precision", "autograd3d", "paper", "small"],
                    help="cgsense (default, the metric's workload); the others print their own line")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--no-context", action="store_true",
                    help="skip the context figures (copy peak, torch.fft E^H E, serving and other workloads)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving and other-workload summaries only (profiling runs)")
    return ap.parse_args()


def make_inputs(w, B, dev):
    import torch

    from paper_1807_11830_amd import synth

    n, C = w.n, w.ncoils
    mask = w.mask_array()
    # per-slice maps: 16 distinct rotations, cycled over the batch (every
    # slice still owns its own buffer in HBM)
    uniq = min(B, 16)
    maps_u = np.stack([synth.coil_maps2d(n, C, rotation=2.0 * np.pi * i / (uniq * C))
                       for i in range(uniq)]).astype(np.complex64)
    maps = torch.empty((B, C, n, n), dtype=torch.complex64, device=dev)
    mu = torch.from_numpy(maps_u).to(dev)
    for b in range(B):
        maps[b].copy_(mu[b % uniq])
    imgs = torch.from_numpy(np.stack([synth.phantom2d(n, seed=synth.SEED_PHANTOM + b)
                                      for b in range(B)]).astype(np.complex64)).to(dev)
    return maps, imgs, mask, maps_u[0]


def host_info():
    """What the host offers: logical CPUs, the CPUs this process may use,
    OMP_NUM_THREADS and the CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "affinity_cpus": affinity,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "cpu_model": model}


def cpu_baseline(w, maps0, mask, y0, target_s):
    """The FP64 oracle's CG-SENSE on the workload's slices, on the host.

    Every host thread solves its own slice (whole solves: E^H y, then K
    iterations of the composed E^H(E p), fp64 throughout), one OpenMP thread
    each, so all cores work; K is chosen so one round takes about target_s/4.
    The rate counts K applies per solve, like the GPU value.  Reported: the
    median over 3 rounds, and one slice alone on one thread."""
    import concurrent.futures as cf
    import statistics

    import oracle

    hi = host_info()
    threads = int(hi["omp_num_threads"] or hi["affinity_cpus"])
    threads = max(1, min(threads, hi["affinity_cpus"]))
    maps0 = maps0.astype(np.complex128)
    y0 = y0.astype(np.complex128)[None]

    def solve(k):
        oracle.set_threads(1)
        oracle.cg(y0, maps0, mask, k)

    # single thread: one slice alone, two iterations to size the rounds
    solve(1)  # library load
    t0 = time.perf_counter()
    solve(2)
    t1 = time.perf_counter() - t0
    per_apply = t1 / 2.5  # E^H y costs about half an apply
    k = max(1, int(round((target_s / 4) / per_apply - 0.5)))
    t0 = time.perf_counter()
    solve(k)
    t_single = time.perf_counter() - t0
    rounds = []
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for _ in range(3):
            t0 = time.perf_counter()
            list(ex.map(solve, [k] * threads))
            rounds.append(time.perf_counter() - t0)
    med = statistics.median(rounds)
    return dict(value=threads * k / med, unit="applies/s", cores=threads, kind="oracle",
                single_thread_applies_per_s=k / t_single, host=hi,
                sample=f"{threads} concurrent whole solves of one {w.n}x{w.n} slice with {w.ncoils} coils "
                       f"(E^H y + {k} CG iterations, E^H E composed as E^H(E p), fp64), one OpenMP thread "
                       f"each; median of 3 rounds ({', '.join(f'{r:.1f}' for r in rounds)} s); "
                       f"single thread {k} iterations in {t_single:.1f} s")


def copy_peak(dev):
    """Device-to-device copy of 1 GiB on the same GPU (read + write rate)."""
    import torch

    src = torch.ones(1 << 27, dtype=torch.complex64, device=dev)  # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    cms = ev0.elapsed_time(ev1) / 5
    del src, dst
    return {"ms": cms, "gbs_read_plus_write": 2 * (1 << 30) / cms / 1e6}


def library_fft_ehe(maps, imgs, mask, reps=5):
    """E^H E of the same batch written with torch.fft (rocFFT) for reference:
    composed (centred 2D transforms of every coil image, mask, inverse,
    conjugate coil sum) and in the readout-decoupled form (1D transforms
    along y only).  Times in ms per apply of the whole batch."""
    import torch

    dev = imgs.device
    m = torch.from_numpy(mask.astype(np.float32)).to(dev)
    n = imgs.shape[-2]
    mu = torch.roll(m, -(n // 2)) / n  # uncentred mask / ny

    def composed():
        u = maps * imgs[:, None]
        k = torch.fft.fftshift(torch.fft.fft2(torch.fft.ifftshift(u, dim=(-2, -1)), norm="ortho"), dim=(-2, -1))
        k = k * m[:, None]
        v = torch.fft.fftshift(torch.fft.ifft2(torch.fft.ifftshift(k, dim=(-2, -1)), norm="ortho"), dim=(-2, -1))
        return (maps.conj() * v).sum(1)

    def hybrid():
        u = torch.fft.fft(maps * imgs[:, None], dim=-2) * mu[:, None]
        return (maps.conj() * torch.fft.ifft(u, dim=-2, norm="forward")).sum(1)

    out = {}
    for name, f in (("composed", composed), ("readout_decoupled", hybrid)):
        f()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            f()
        ev1.record()
        torch.cuda.synchronize()
        out[name + "_ms"] = ev0.elapsed_time(ev1) / reps
    torch.cuda.empty_cache()
    return out


def serving_summary(n_requests=512, factor=0.9):
    """The serving workload at one arrival rate: 512 seeded requests (own
    maps, image and noise each), Poisson arrivals at factor x the measured
    one-at-a-time rate; p50/p99 latency and solves/s of the engine (HBM
    budget) and of one solve at a time."""
    from paper_1807_11830_amd.serving import EngineExecutor, InputBank, Scheduler, SerialExecutor, make_requests

    bank = InputBank()
    t0 = time.perf_counter()
    reqs0 = make_requests(n_requests, rate=1.0)
    bank.prepare(reqs0)
    log(f"serving: {n_requests} requests' inputs ({bank.nbytes() / 2**30:.2f} GiB) in "
        f"{time.perf_counter() - t0:.1f} s")
    ser = SerialExecutor(bank)
    Scheduler(ser).run(make_requests(48, rate=1e9))  # warm plans and graphs
    mu = Scheduler(ser).run(make_requests(96, rate=1e9)).throughput
    reqs = make_requests(n_requests, rate=factor * mu)
    ex = EngineExecutor(bank, 200 << 30, max_slots=128)
    Scheduler(ex).run(make_requests(32, rate=1e9))
    se = Scheduler(ex).run(reqs)
    ex.close()
    reqs = make_requests(n_requests, rate=factor * mu)
    ss = Scheduler(ser).run(reqs)
    ser.close()
    bank.close()
    res = {"workload": f"serving_{n_requests}req_n128-320_c8-32_r2-4_k25", "arrival_factor": factor,
           "one_at_a_time_rate": mu, "inputs": "per request (own seeded maps, image, noise)",
           "engine": {"p50_ms": se.p50 * 1e3, "p99_ms": se.p99 * 1e3, "solves_per_s": se.throughput,
                      "max_inflight": se.max_inflight, "budget": "HBM (200 GiB)"},
           "one_at_a_time": {"p50_ms": ss.p50 * 1e3, "p99_ms": ss.p99 * 1e3, "solves_per_s": ss.throughput}}
    log(f"serving: x{factor} engine p50 {se.p50 * 1e3:.2f} p99 {se.p99 * 1e3:.2f} ms {se.throughput:.0f}/s; "
        f"one at a time p50 {ss.p50 * 1e3:.2f} p99 {ss.p99 * 1e3:.2f} ms {ss.throughput:.0f}/s")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(slices are independent: shard the batch across processes instead)", file=sys.stderr)
        sys.exit(2)
    {"cgsense": run_cgsense, "serving": run_serving, "precision": run_precision,
     "autograd3d": run_autograd3d, "paper": run_paper, "small": run_small}[args.workload](args)


def run_serving(args):
    """512 requests (sizes 128-320, 8-32 coils, R 2-4, 25 iterations) with
    Poisson arrivals at 0.5/0.9/1.5 x the one-at-a-time solve rate: p50/p99
    latency and solves/s of the batching engine vs one solve at a time."""
    import torch

    from paper_1807_11830_amd.serving import (EngineExecutor, InputBank, Scheduler, SerialExecutor,
                                              make_requests)

    bank = InputBank()
    log("serving: preparing inputs")
    probe = make_requests(96, rate=1e9)
    bank.prepare(probe)
    bank.prepare(make_requests(args.requests, rate=1.0))
    # warm up plans/graphs, then measure the one-at-a-time rate
    ser = SerialExecutor(bank)
    Scheduler(ser).run(make_requests(48, rate=1e9))
    st0 = Scheduler(ser).run(probe)
    mu = st0.throughput
    log(f"serving: one-at-a-time {mu:.1f} solves/s")
    budgets = {"hbm": 200 << 30, "cap256MB": 256 << 20}
    runs = []
    for f in (0.5, 0.9, 1.5):
        reqs = make_requests(args.requests, rate=f * mu)
        for bname, budget in budgets.items():
            ex = EngineExecutor(bank, budget, max_slots=128)
            Scheduler(ex).run(make_requests(32, rate=1e9))  # warm the plan pool
            stats = Scheduler(ex).run(reqs)
            ex.close()
            runs.append(dict(rate_factor=f, executor="engine", budget=bname, p50_ms=stats.p50 * 1e3,
                             p99_ms=stats.p99 * 1e3, solves_per_s=stats.throughput,
                             max_inflight=stats.max_inflight, steps=stats.steps))
            log(f"serving: x{f} engine[{bname}] p50 {stats.p50*1e3:.2f} ms p99 {stats.p99*1e3:.2f} ms "
                f"{stats.throughput:.1f}/s inflight<={stats.max_inflight}")
        reqs = make_requests(args.requests, rate=f * mu)
        stats = Scheduler(ser).run(reqs)
        runs.append(dict(rate_factor=f, executor="one-at-a-time", p50_ms=stats.p50 * 1e3,
                         p99_ms=stats.p99 * 1e3, solves_per_s=stats.throughput))
        log(f"serving: x{f} serial p50 {stats.p50*1e3:.2f} ms p99 {stats.p99*1e3:.2f} ms {stats.throughput:.1f}/s")
    # capacity: all requests present at t = 0
    burst = make_requests(args.requests, rate=1e9)
    ex = EngineExecutor(bank, budgets["hbm"], max_slots=128)
    Scheduler(ex).run(make_requests(32, rate=1e9))
    stats = Scheduler(ex).run(burst)
    ex.close()
    runs.append(dict(rate_factor="burst", executor="engine", budget="hbm", p50_ms=stats.p50 * 1e3,
                     p99_ms=stats.p99 * 1e3, solves_per_s=stats.throughput,
                     max_inflight=stats.max_inflight, steps=stats.steps))
    log(f"serving: burst engine p50 {stats.p50*1e3:.2f} ms p99 {stats.p99*1e3:.2f} ms {stats.throughput:.1f}/s "
        f"inflight<={stats.max_inflight}")
    burst = make_requests(args.requests, rate=1e9)
    stats = Scheduler(ser).run(burst)
    runs.append(dict(rate_factor="burst", executor="one-at-a-time", p50_ms=stats.p50 * 1e3,
                     p99_ms=stats.p99 * 1e3, solves_per_s=stats.throughput))
    log(f"serving: burst serial p50 {stats.p50*1e3:.2f} ms p99 {stats.p99*1e3:.2f} ms {stats.throughput:.1f}/s")
    ser.close()
    key = [r for r in runs if r["rate_factor"] == 0.9 and r.get("budget") == "hbm"][0]
    print(json.dumps({"metric": "served recon p99 latency (Poisson arrivals at 0.9 x one-at-a-time rate)",
                      "value": key["p99_ms"], "unit": "ms", "n_gpus": 1, "higher_is_better": False,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "serving_512req_n128-320_c8-32_r2-4_k25",
                                 "requests": args.requests, "one_at_a_time_solves_per_s": mu},
                      "runs": runs}), flush=True)


VALU_PEAK_TFLOPS = 78.6  # fp32 FMA without packed instructions: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz


def precision_roofline(st, n, C, B, K, launch_s):
    """Both bounds of one fused CG launch over B slices of n x n with C coils
    in storage st: HBM bytes (maps once in st, x, r, p, q read and written in
    complex64, averaged over the K launches of a solve) and fp32 flops
    (C forward/inverse n-point transform pairs at 5 n log2 n each per column,
    plus 16 flops per element and coil for the coil products and the mask)."""
    import math

    nvox = n * n
    sb = 8 if st == "c64" else 4
    by = B * nvox * (sb * C + (8 * 3 + (K - 1) * 8 * 8) / K)
    fl = B * nvox * C * (10 * math.log2(n) + 16)
    t_hbm = by / (HBM_PEAK_GBS * 1e9)
    t_alu = fl / (VALU_PEAK_TFLOPS * 1e12)
    bound = "hbm" if t_hbm >= t_alu else "alu"
    return {"avg_launch_us": launch_s * 1e6, "bytes": round(by), "flops": round(fl),
            "hbm_time_us": t_hbm * 1e6, "alu_time_us": t_alu * 1e6, "bound": bound,
            "frac": max(t_hbm, t_alu) / launch_s, "achieved_gbs": by / launch_s / 1e9,
            "achieved_tflops": fl / launch_s / 1e12}


def precision_result(batches, storages, reps=5):
    """Per batch size and storage: seconds per solve, applies/s, the fused CG
    launch against both bounds, and for 16-bit storage the relative L2
    difference from the GPU complex64 result (max over slices) and the
    speed-up over complex64 (storages must start with "c64")."""
    import torch

    from paper_1807_11830_amd import sense, synth

    w = synth.PREC_384
    K, n, C = w.iters, w.n, w.ncoils
    dev = torch.device("cuda:0")
    res = {}
    for B in batches:
        imgs, maps, mask = synth.slice_inputs(w, B, per_slice_maps=True)
        maps_t = torch.from_numpy(maps.astype(np.complex64)).to(dev)
        imgs_t = torch.from_numpy(imgs.astype(np.complex64)).to(dev)
        del imgs, maps
        with sense.Plan(maps_t, mask, batch=B) as p0:
            y = p0.E(imgs_t)
        noise = synth.complex_noise((B, C, n, n)).astype(np.complex64) * mask[None, None, :, None]
        y += torch.from_numpy(noise).to(dev)
        del noise
        out = {}
        xs = {}
        for st in storages:
            with sense.Plan(maps_t, mask, batch=B, maps_storage=st, kspace_storage=st) as plan:
                ys = sense.to_storage(y, st)
                plan.cg(ys, K)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    plan.cg(ys, K, sync=False)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps
                xs[st] = plan.cg(ys, K).x.clone()
                # per-launch times of the fused CG launch (group launch + combine)
                plan.set_profiling(True)
                plan.cg(ys, K, sync=False)
                torch.cuda.synchronize()
                n_l, ms_l = plan.profile()
                plan.set_profiling(False)
                launch_s = ms_l / 1e3 / max(n_l, 1)
                out[st] = {"solve_ms": dt * 1e3, "applies_per_s": B * K / dt, "coil_groups": plan.coil_groups()[0],
                           "fused_launch": precision_roofline(st, n, C, B, K, launch_s)}
                del ys
            log(f"precision: B={B} {st} {dt*1e3:.2f} ms/solve, fused launch {launch_s*1e6:.1f} us, "
                f"frac {out[st]['fused_launch']['frac']:.3f}")
        for st in storages[1:]:
            d = xs[st] - xs["c64"]
            out[st]["rel_l2_vs_gpu_c64_max_over_slices"] = float(
                (torch.linalg.vector_norm(d.reshape(B, -1), dim=1)
                 / torch.linalg.vector_norm(xs["c64"].reshape(B, -1), dim=1)).max())
            out[st]["speedup_vs_c64"] = out["c64"]["solve_ms"] / out[st]["solve_ms"]
            log(f"precision: B={B} {st} {out[st]}")
        res[f"batch{B}"] = out
        del maps_t, imgs_t, y, xs
        torch.cuda.empty_cache()
    return res


def run_precision(args):
    """384x384, 32 coils, VD R=4, 40 iterations: maps and k-space in c64 /
    bf16 / fp16 storage (fp32 arithmetic, fp64 reductions), at the workload's
    batch of 8 slices (whose BF16 working set fits the 256 MB memory-side
    cache) and at 48 slices (which does not); solves/s, both roofline bounds
    of the fused CG launch, and the relative L2 difference of each 16-bit
    result from the GPU complex64 result over all slices.  The errors against
    the FP64 oracle are the parity test's (tests/test_gpu_precision.py)."""
    from paper_1807_11830_amd import synth

    w = synth.PREC_384
    K = w.iters
    res = precision_result((w.batch, 48), ("c64", "bf16", "fp16"))
    print(json.dumps({"metric": "E^H E applies/s by storage precision (CG-SENSE, 40 iterations)",
                      "value": res[f"batch{w.batch}"]["bf16"]["applies_per_s"], "unit": "applies/s", "n_gpus": 1,
                      "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": w.name, "slices": w.batch, "iters": K}, "variants": res}), flush=True)


def small_result(steps, warmup):
    """One 64x64 slice, 4 coils, 20 CG iterations: microseconds per solve as
    the plan runs it by default (two eager launches: the x rows of E^H y,
    then the rest of E^H y and the whole loop in one workgroup), with graphs
    switched off (the same launches), and with the coils forced into the
    workspace's fill split (one fused launch per iteration, replayed from
    the solve's HIP graph)."""
    import torch

    from paper_1807_11830_amd import sense, synth

    w = synth.SMALL_64
    dev = torch.device("cuda:0")
    imgs, maps, mask = synth.slice_inputs(w, 1)
    maps_t = torch.from_numpy(maps.astype(np.complex64)).to(dev)
    out = {}
    with sense.Plan(maps_t, mask) as plan:
        y = plan.E(torch.from_numpy(imgs.astype(np.complex64)).to(dev))
        x = torch.empty((1, w.n, w.n), dtype=torch.complex64, device=dev)
        gdef, gmax = plan.coil_groups()
        # the default (one coil group at this size) and the fill split forced
        for mode in ("default", "graphs_off", f"graph_G{gmax}"):
            plan.set_graphs(mode != "graphs_off")
            plan.set_coil_groups(gmax if mode.endswith(f"_G{gmax}") else gdef)
            for _ in range(max(warmup, 1)):
                plan.cg(y, w.iters, out=x, sync=False)
            torch.cuda.synchronize()
            reps = steps
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.cg(y, w.iters, out=x, sync=False)
            torch.cuda.synchronize()
            out[mode] = (time.perf_counter() - t0) / reps * 1e6
            log(f"small: {mode} {out[mode]:.1f} us per solve")
    return out


def run_small(args):
    """The small-solve latency (small_result) as its own bench line."""
    from paper_1807_11830_amd import synth

    w = synth.SMALL_64
    out = small_result(args.steps, args.warmup)
    print(json.dumps({"metric": "CG-SENSE solve latency (64x64, 4 coils, 20 iterations)", "value": out["default"],
                      "unit": "us", "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
                      "data": "synthetic", "config": {"workload": w.name},
                      "us_per_solve": out}), flush=True)


def run_paper(args):
    """The paper's reconstruction workload (Section "Performance comparison
    with other frameworks"): 16 frames of 160x160 with 8 coils, fully sampled
    Cartesian k-space; the Eq. (1) reconstruction (E^H at full sampling) and
    the root-sum-of-squares reconstruction, each timed over 100 runs."""
    import torch

    from paper_1807_11830_amd import sense, synth

    n, C, B, reps = 160, 8, 16, 100
    dev = torch.device("cuda:0")
    full = np.ones(n, np.uint8)
    maps = torch.from_numpy(synth.coil_maps2d(n, C).astype(np.complex64)).to(dev)
    imgs = torch.from_numpy(np.stack([synth.phantom2d(n, seed=synth.SEED_PHANTOM + f)
                                      for f in range(B)]).astype(np.complex64)).to(dev)
    out = {}
    with sense.Plan(maps, full, batch=B) as plan:
        y = plan.E(imgs)
        x = torch.empty_like(imgs)
        img = torch.empty((B, n, n), dtype=torch.float32, device=dev)
        for name, f, nbytes in (("eq1_EH", lambda: plan.EH(y, out=x), 8 * n * n * (B * C + C + B)),
                                ("rss", lambda: plan.rss(y, out=img), 8 * n * n * B * C + 4 * n * n * B)):
            for _ in range(10):
                f()
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            for _ in range(reps):
                f()
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / reps
            out[name] = {"ms": ms, "algorithmic_bytes": nbytes, "achieved_gbs": nbytes / ms / 1e6}
            log(f"paper: {name} {ms * 1e3:.1f} us per 16-frame reconstruction ({nbytes / ms / 1e6:.0f} GB/s)")
    print(json.dumps({"metric": "reconstructions/s (16 frames 160x160, 8 coils, fully sampled)",
                      "value": 1e3 / out["rss"]["ms"], "unit": "RSS reconstructions/s", "n_gpus": 1,
                      "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "paper_16x160x160_c8_full", "frames": B, "coils": C},
                      "results": out}), flush=True)


def autograd3d_result(reps=10):
    """256x256x128 volume, 16 coils, (ky, kz) mask R=6 with a 32x32 centre:
    E forward plus its backward (E^H of a fixed upstream gradient) through
    torch.autograd; also the whole step of the loss ||E x - y||^2, whose
    elementwise residual and square run in torch, the pair with compact
    k-space, and a 10-iteration 3D CG solve."""
    import torch

    from paper_1807_11830_amd import sense, synth
    from paper_1807_11830_amd.autograd import sense_E

    nx, ny, nz, C = 256, 256, 128, 16
    dev = torch.device("cuda:0")
    log("autograd3d: inputs")
    mask = synth.mask_variable_density_2d(ny, nz, 6.0, (32, 32))
    maps = torch.from_numpy(synth.coil_maps3d(nx, ny, nz, C).astype(np.complex64)).to(dev)
    x_true = torch.from_numpy(synth.phantom3d(nx, ny, nz).astype(np.complex64)[None]).to(dev)
    with sense.Plan(maps, mask) as plan:
        y = plan.E(x_true)
        x = torch.zeros_like(x_true, requires_grad=True)
        g = y.clone()  # upstream gradient of the forward output

        def fwd_bwd():
            sense_E(x, plan).backward(g)
            x.grad = None

        def loss_step():
            r = sense_E(x, plan) - y
            torch.view_as_real(r).square().sum().backward()
            x.grad = None

        def timed(f):
            for _ in range(2):
                f()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                f()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        dt = timed(fwd_bwd)
        dt_loss = timed(loss_step)
    # the same pair with compact k-space (sampled (ky, kz) lines only), and
    # 3D CG-SENSE iterations on the compact data
    with sense.Plan(maps, mask, kspace_compact=True) as plan:
        g = plan.E(x_true)

        def fwd_bwd_compact():
            sense_E(x, plan).backward(g)
            x.grad = None

        dt_c = timed(fwd_bwd_compact)
        nlines = plan.nlines
        xs = torch.empty_like(x_true)
        K = 10
        plan.cg(g, K, out=xs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            plan.cg(g, K, out=xs, sync=False)
        torch.cuda.synchronize()
        dt_cg = (time.perf_counter() - t0) / 3
    nvox = nx * ny * nz
    nbytes = 8 * nvox * (2 * C + 1) * 2
    nbytes_c = 2 * (8 * nvox * (C + 1) + 8 * C * nlines * nx)
    log(f"autograd3d: 3D CG {dt_cg * 1e3:.2f} ms per {K}-iteration solve (compact k-space)")
    log(f"autograd3d: fwd+bwd {dt * 1e3:.2f} ms ({nbytes / dt / 1e9:.0f} GB/s algorithmic), "
        f"loss step {dt_loss * 1e3:.2f} ms, compact k-space fwd+bwd {dt_c * 1e3:.2f} ms "
        f"({nbytes_c / dt_c / 1e9:.0f} GB/s algorithmic)")
    del maps, x_true, x, g, xs
    torch.cuda.empty_cache()
    return {"ms_per_step": dt * 1e3, "algorithmic_bytes": nbytes, "achieved_gbs": nbytes / dt / 1e9,
            "loss_step_ms": dt_loss * 1e3,
            "compact_kspace": {"ms_per_step": dt_c * 1e3, "algorithmic_bytes": nbytes_c,
                               "achieved_gbs": nbytes_c / dt_c / 1e9},
            "cg3d": {"iters": K, "ms_per_solve": dt_cg * 1e3}}


def run_autograd3d(args):
    """The 3D workload (autograd3d_result) as its own bench line: E forward
    plus its backward through torch.autograd, per second."""
    r = autograd3d_result()
    dt = r.pop("ms_per_step") / 1e3
    print(json.dumps({"metric": "forward+backward of E per second (3D, autograd)", "value": 1.0 / dt,
                      "unit": "fwd+bwd/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
                      "data": "synthetic", "ms_per_step": dt * 1e3,
                      "config": {"workload": "autograd3d_256x256x128_c16_r6", "coils": 16}, **r}), flush=True)


def run_cgsense(args):
    import torch

    from paper_1807_11830_amd import sense, synth

    w = synth.SLICE_256
    B, K = args.batch, args.iters
    dev = torch.device("cuda:0")
    log(f"bench: building inputs ({B} slices {w.n}x{w.n}, {w.ncoils} coils)")
    maps, imgs, mask, maps0 = make_inputs(w, B, dev)
    plan = sense.Plan(maps, mask, batch=B, maps_storage=args.maps_storage)
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.SEED_NOISE)
    y = plan.E(imgs)
    noise = 1e-3 * torch.complex(torch.randn(y.shape, generator=gen, device=dev),
                                 torch.randn(y.shape, generator=gen, device=dev))
    y += noise * torch.from_numpy(mask.astype(np.float32)).to(dev)[None, None, :, None]
    x = torch.empty_like(imgs)
    torch.cuda.synchronize()
    del noise

    log(f"bench: warmup {args.warmup}")
    plan.set_profiling(True)
    for _ in range(args.warmup):
        plan.cg(y, K, out=x, sync=False)
    torch.cuda.synchronize()
    plan.profile()
    # one untimed pass of the timed length creates the plan's timing events,
    # so no event is created inside the timed region
    for _ in range(args.steps):
        plan.cg(y, K, out=x, sync=False)
    torch.cuda.synchronize()
    plan.profile()
    # the timed steps: whole solves launched on the plan's stream with HIP
    # events around every fused launch, so the throughput and the fused
    # launch's average duration come from the same launches
    log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.cg(y, K, out=x, sync=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_l, ms_l = plan.profile()
    plan.set_profiling(False)
    # the same steps replayed from each solve's captured HIP graph (the
    # serving path's form), reported beside them
    for _ in range(2):
        plan.cg(y, K, out=x, sync=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.cg(y, K, out=x, sync=False)
    torch.cuda.synchronize()
    dt_graph = time.perf_counter() - t0
    res = plan.cg(y, K, out=x)
    assert int(res.iters.min()) == K, res.iters

    nvox = w.n * w.n
    C = w.ncoils
    avg_s = ms_l / 1e3 / max(n_l, 1)
    # fused CG launch k: reads S (C values); k = 0 reads p and r and writes
    # q; k >= 1 also finishes iteration k-1, reading x, r, p, q and writing
    # x, r, p, q.  Averaged over the K launches of a solve.
    sbytes = 8 if args.maps_storage == "c64" else 4
    bytes_launch = B * nvox * (sbytes * C + (8 * 3 + (K - 1) * 8 * 8) / K)
    achieved = bytes_launch / avg_s / 1e9
    applies = B * K * args.steps
    log(f"bench: {dt * 1e3 / args.steps:.2f} ms/step, fused launch avg {avg_s * 1e6:.1f} us "
        f"({achieved:.0f} GB/s)")

    # the metric's unit alone: standalone E^H E apply, (C+2) complex vectors
    plan.set_profiling(True)
    p = imgs
    q = torch.empty_like(p)
    for _ in range(20):
        plan.EHE(p, out=q)
    torch.cuda.synchronize()
    n_a, ms_a = plan.profile()
    plan.set_profiling(False)
    apply_s = ms_a / 1e3 / max(n_a, 1)
    apply_bytes = B * nvox * (sbytes * C + 16)
    log(f"bench: standalone apply {apply_s * 1e6:.1f} us ({apply_bytes / apply_s / 1e9:.0f} GB/s)")

    out = {
        "metric": "E^H E applies/s (CG-SENSE, 256x256, 12 coils, R=4, 30 iterations)",
        "value": applies / dt,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "slices": B, "iters": K, "maps": "per-slice",
                   "maps_storage": args.maps_storage, "kspace_storage": "c64",
                   "inner_products": "f64", "nx": w.n, "ny": w.n, "coils": C},
        "roofline": {"bound": "hbm", "kernel": "ehe2d_kernel (fused CG iteration: x, r, p updates + E^H E)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     # counters were taken for the complex64-maps instantiation only
                     "traffic": measured_traffic("sense::ehe2d_kernel<256, 0, true, false, true>")
                     if args.maps_storage == "c64" else None,
                     "avg_launch_us": avg_s * 1e6, "launches": n_l,
                     "bytes_per_launch": round(bytes_launch)},
        "ehe_apply": {"avg_launch_us": apply_s * 1e6, "bytes_per_launch": apply_bytes,
                      "achieved_gbs": apply_bytes / apply_s / 1e9,
                      "applies_per_s": B / apply_s},
        "graph_replay": {"ms_per_step": dt_graph * 1e3 / args.steps, "applies_per_s": applies / dt_graph,
                         "note": "same steps, each solve replayed from its captured HIP graph"},
    }
    if not args.no_context:
        out["copy_1gib"] = copy_peak(dev)
        # the same launch against the copy rate measured in this run
        out["roofline"]["copy_peak_gbs"] = out["copy_1gib"]["gbs_read_plus_write"]
        out["roofline"]["frac_of_copy"] = achieved / out["copy_1gib"]["gbs_read_plus_write"]
        log(f"bench: 1 GiB copy {out['copy_1gib']['ms']:.3f} ms "
            f"({out['copy_1gib']['gbs_read_plus_write']:.0f} GB/s read+write)")
        lib = library_fft_ehe(maps, imgs, mask)
        lib["note"] = "same batch, torch.fft (rocFFT), context only"
        lib["hip_apply_ms"] = apply_s * 1e3
        out["library_fft_ehe"] = lib
        log(f"bench: torch.fft E^H E {lib}")
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        y0 = y[0].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(w, maps0, mask, y0, args.cpu_seconds)
        log(f"bench: cpu baseline {out['cpu_baseline']['value']:.2f} applies/s on "
            f"{out['cpu_baseline']['cores']} threads")
    plan.close()
    del maps, imgs, y, x, p, q
    torch.cuda.empty_cache()
    if not (args.no_context or args.no_serving):
        out["serving"] = serving_summary()
        out["other_workloads"] = other_workloads_summary()
    print(json.dumps(out), flush=True)


def other_workloads_summary():
    """Context for the default line: the other configurations at reduced
    repetition counts (their own --workload lines give the full runs).  A
    failure here is recorded in the line instead of suppressing it."""
    from paper_1807_11830_amd import synth

    bp = synth.PREC_384.batch
    res = {}
    for name, f in (("small_64x64_c4_k20_us_per_solve", lambda: small_result(100, 5)),
                    ("precision_384x384_c32_b8_k40", lambda: precision_result((bp,), ("c64", "bf16"), reps=3)[f"batch{bp}"]),
                    ("autograd3d_256x256x128_c16", lambda: autograd3d_result(reps=5))):
        t0 = time.perf_counter()
        try:
            res[name] = f()
        except Exception as e:  # context only: the metric's line still prints, with the error
            res[name] = {"error": f"{type(e).__name__}: {e}"}
        log(f"bench: {name} in {time.perf_counter() - t0:.1f} s")
    return res


if __name__ == "__main__":
    main()
