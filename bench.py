"""Benchmark: minimum cut of a 256x256x128 6-connected volume on one GPU.

One step = one cold-start solve of the whole hot path through the C ABI on the
largest single-GPU workload (a segmentation-shaped volume, 8.4 M voxels):
chain-prox sweeps of the three families (one launch), the product-space
Douglas-Rachford averaging step, the FP64 certificate checks and the cut
readout, run until the certificate is below 1e-3 (exact for the 2^-8-dyadic
data).  Inputs are generated once and resident in HBM before the timed region.

Prints one JSON line.  `value` is voxel-sweeps per second over the timed
steps (voxels x chain families x sweep launches / wall time).  `roofline`
rates the dominant kernel, the three-family sweep launch, by its event-timed
launches (HIP events on the solve's stream, in the last timed step) against
HBM bandwidth: 36 algorithmic bytes per voxel per launch (z_j, a_j read and
q_j written for each family) plus 12 on the launches that write edge duals.
`traffic` is the counter-measured HBM bytes per launch from the committed
profile, reported only while the sweep sources match the profile's hash.
Other objects: the 1024x1024 image (two-set form) with its own roofline, the
learned warm start and dual reuse (time to the exact cut, cold against warm),
the 8-connected image, alpha-expansion, the mixed BCD loop, and the batched
solve of 64 uneven grids.  `cpu_baseline` times the CPU oracle (FP64) on a
bounded number of iterations of the same volume, on one thread and on all the
host's threads, and checks the GPU cut against the oracle's max-flow energy.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "chain-prox voxel-sweeps/s (%HBM peak); time-to-exact-cut cold vs warm start"
HBM_PEAK_GBS = 8000.0
VOL_BYTES_VALUE = 36.0  # per voxel and sweep launch of the three families (values only)
VOL_BYTES_DUALS = 12.0  # added on the launches that also write the edge duals
IMG_BYTES_PER_VOXEL_SWEEP = 16.0  # two-set DR: 32 B per voxel-iteration over two sweeps
IMG_BYTES_DUALS = 4.0
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "volume3d_256x256x128_sweep_traffic.md")
IMG_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "image2d_1024_sweep_traffic.md")
SWEEP_SOURCES = ["chain.hpp", "lean.hpp", "piece.hpp", "sweeps.hip", "launch.hpp"]


def sweep_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_1503_01563_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "paper_1503_01563_amd", "build.py"), "rb") as fh:  # compiler flags
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_PROFILE):
    """HBM bytes per sweep launch from a committed counter summary, or None
    when the sweep kernels changed since the counters were taken."""
    import re
    try:
        text = open(path).read()
    except OSError:
        return None
    m_hash = re.search(r"sweep sources sha256\[:16\]: `([0-9a-f]+)`", text)
    m_val = re.search(r"HBM bytes per sweep launch: `([0-9.eE+]+)`", text)
    if not m_hash or not m_val or m_hash.group(1) != sweep_sources_hash():
        return None
    return float(m_val.group(1))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--check-every", type=int, default=4)
    ap.add_argument("--seed", type=int, default=3000, help="seed of the volume")
    ap.add_argument("--image-seed", type=int, default=2000)
    ap.add_argument("--size", type=int, default=1024, help="side of the image workload")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="approximate CPU time of each oracle baseline leg (one thread, all threads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also run the all-core oracle to its certificate on the volume (minutes)")
    ap.add_argument("--warm-grids", type=int, default=64,
                    help="held-out 512x512 grids for the cold vs warm-start comparison (0: skip)")
    ap.add_argument("--no-image", dest="image", action="store_false",
                    help="skip the 1024x1024 image section")
    ap.add_argument("--no-grid8", dest="grid8", action="store_false",
                    help="skip the 8-connected version of the image")
    ap.add_argument("--no-multilabel", dest="multilabel", action="store_false",
                    help="skip the alpha-expansion (multi-label) section")
    ap.add_argument("--no-batched", dest="batched", action="store_false",
                    help="skip the section solving 64 uneven grids in one batch")
    ap.add_argument("--no-mixed", dest="mixed", action="store_false",
                    help="skip the section comparing the mixed BCD-then-splitting loop")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, copy 256 MiB device to device (a reference "
                         "kernel for the HBM byte counters of a profiler run)")
    return ap.parse_args()


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_threads():
    """Threads of the all-core leg: OMP_NUM_THREADS when set (the host's
    share), else every CPU the process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(w, a, gpu_res, budget_s, full=False):
    """The oracle (FP64 product-space DR, unchanged) on a bounded number of
    iterations of the same volume, on one thread and on all threads, plus
    its max-flow energy for the exactness check."""
    import oracle
    oracle.build(force=False)
    n = w.size
    r = w.ndim
    nproc, model = cpu_info()
    threads = cpu_threads()
    legs = {}
    for name, th in (("single_thread", 1), ("all_threads", threads)):
        t0 = time.perf_counter()
        oracle.dr_solve(w, a, max_iters=1, gap_tol=0, threads=th)
        per_iter = time.perf_counter() - t0
        iters = max(1, min(60, int(budget_s / max(per_iter, 1e-6))))
        t0 = time.perf_counter()
        res = oracle.dr_solve(w, a, max_iters=iters, gap_tol=0, threads=th)
        dt = time.perf_counter() - t0
        legs[name] = {"threads": oracle.threads_used(th), "iters": res["iters"], "seconds": dt,
                      "voxel_sweeps_per_s": n * r * res["iters"] / dt, "ms_per_iter": 1e3 * dt / res["iters"]}
    t0 = time.perf_counter()
    e_star, _, _ = oracle.mincut(w, a, "dinic")
    dt_flow = time.perf_counter() - t0
    allc = legs["all_threads"]
    out = {
        "value": allc["voxel_sweeps_per_s"],
        "unit": "voxel-sweeps/s",
        "cores": allc["threads"],
        "kind": "oracle",
        "sample": "FP64 product-space DR (certificate every iteration) on the same 256x256x128 volume: "
                  "%d iterations on %d threads (%.1f s), %d on one thread (%.1f s); Dinic max-flow %.1f s"
                  % (allc["iters"], allc["threads"], allc["seconds"], legs["single_thread"]["iters"],
                     legs["single_thread"]["seconds"], dt_flow),
        "single_thread": legs["single_thread"],
        "all_threads": allc,
        "nproc": nproc,
        "cpu_model": model,
        "maxflow_energy": e_star,
        "maxflow_seconds": dt_flow,
        "gpu_energy_exact": bool(gpu_res.energy == e_star),
        "to_certificate_estimate_s": gpu_res.iters * allc["ms_per_iter"] / 1e3,
        "to_certificate_note": "the oracle runs the same iteration; estimate = GPU iterations to the "
                               "certificate x all-thread seconds per oracle iteration",
    }
    if full:
        t0 = time.perf_counter()
        res = oracle.dr_solve(w, a, max_iters=3000, gap_tol=1e-3, threads=threads)
        out["to_certificate"] = {"iters": res["iters"], "seconds": time.perf_counter() - t0,
                                 "threads": allc["threads"], "certified": res["status"] == 0,
                                 "energy": res["energy"]}
    return out


def timed_solves(wt, at, steps, warmup, check_every):
    """`warmup` untimed solves, then `steps` timed ones (the last with per-launch
    events); returns (results, wall seconds of the timed region, per-step walls)."""
    import torch

    from paper_1503_01563_amd import mc
    torch.cuda.synchronize()
    for _ in range(warmup):
        mc.tv_solve(wt, at, max_iters=3000, check_every=check_every)
    torch.cuda.synchronize()
    results, walls = [], []
    t0 = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        results.append(mc.tv_solve(wt, at, max_iters=3000, check_every=check_every, profile=k == steps - 1))
        walls.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    return results, time.perf_counter() - t0, walls


def roofline(prof, n, bytes_value, bytes_duals, kernel, traffic):
    """Rate of the dominant kernel: the sweep launches of one profiled solve
    that write values only (algorithmic bytes over their event-timed device
    time); the launches that also write edge duals (certificate iterations)
    are reported beside it."""
    launches = max(prof.sweep_launches, 1)
    dual_launches = min(prof.dual_sweep_launches, launches)
    value_launches = max(launches - dual_launches, 1)
    value_s = max(prof.sweep_ms - prof.dual_sweep_ms, 1e-9) / 1e3
    achieved = n * bytes_value * value_launches / value_s / 1e9
    dual_s = prof.dual_sweep_ms / 1e3
    return {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_unit": "HBM bytes per value launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
        "kernel": kernel,
        "avg_launch_us": 1e6 * value_s / value_launches,
        "bytes_per_launch": n * bytes_value,
        "launches": value_launches,
        "dual_launches": dual_launches,
        "dual_avg_launch_us": 1e6 * dual_s / dual_launches if dual_launches else None,
        "dual_bytes_per_launch": n * (bytes_value + bytes_duals),
        "dual_achieved": n * (bytes_value + bytes_duals) * dual_launches / dual_s / 1e9 if dual_launches and dual_s > 0 else None,
    }


def progress(msg, t0=[None]):
    """One line per finished section on stderr (the JSON line alone goes to stdout)."""
    now = time.time()
    if t0[0] is None:
        t0[0] = now
    print("bench: %s (%.1f s)" % (msg, now - t0[0]), file=sys.stderr, flush=True)


def main():
    args = parse()
    progress("start")
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1503_01563_amd import gen

    dev = torch.device("cuda:0")
    w, a = gen.config_volume3d(args.seed)
    wt = torch.from_numpy(w).to(dev)
    at = [torch.from_numpy(x).to(dev) for x in a]
    n = w.size
    r = w.ndim
    results, dt, walls = timed_solves(wt, at, args.steps, args.warmup, args.check_every)
    progress("volume: %d timed solves" % args.steps)
    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    sweeps = sum(r * n * res.sweep_launches for res in results)  # voxel-sweeps actually run
    last = results[-1]  # the step whose sweep launches carry events
    out = {
        "metric": METRIC,
        "value": sweeps / dt,
        "unit": "voxel-sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "volume %dx%dx%d (WxHxD) 6-connected, noisy ellipsoids, lambda=1.5, dyadic 2^-8, seed %d"
                        % (w.shape[2], w.shape[1], w.shape[0], args.seed),
            "solver": "product-space Douglas-Rachford (r = 3), cold start, certificate every %d iterations"
                      % args.check_every,
            "stop": "certificate < 1e-3",
        },
        "time_to_exact_cut_ms": 1e3 * float(np.median(walls)),
        "device_ms_median": float(np.median([q.ms for q in results])),
        "iters": last.iters,
        "certified": all(res.converged for res in results),
        "energy": last.energy,
        "roofline": roofline(last, n, VOL_BYTES_VALUE, VOL_BYTES_DUALS,
                             "k_stream3<false> (value launches: rows, columns and depth chains of the volume "
                             "in streamed pieces; the dual launches are k_stream3<true>)",
                             measured_traffic(TRAFFIC_PROFILE)),
    }
    if args.image:
        out["image2d"] = image2d_section(args.image_seed, (args.size, args.size), args.check_every)
        progress("image2d")
    if args.warm_grids > 0:
        out["warm_start"] = warm_start_section(args.warm_grids)
        progress("warm start")
        out["dual_reuse"] = dual_reuse_section()
        progress("dual reuse")
    if args.grid8:
        out["grid8"] = grid8_section(args.image_seed, (args.size, args.size))
        progress("grid8")
    if args.multilabel:
        out["alpha_expansion"] = alpha_expansion_section()
        progress("alpha expansion")
    if args.mixed:
        out["mixed_outer_loop"] = mixed_outer_loop_section(args.image_seed)
        progress("mixed outer loop")
    if args.batched:
        out["batched"] = batched_section()
        progress("batched")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a, last, args.cpu_seconds, full=args.cpu_full)
        progress("cpu baseline")
    print(json.dumps(out))


def image2d_section(seed, shape, check_every, steps=5):
    """The 1024x1024 segmentation-shaped image in the two-set form: time to the
    exact cut and the rate of its row and column sweep launches."""
    import numpy as np
    import torch

    from paper_1503_01563_amd import gen
    dev = torch.device("cuda:0")
    w, a = gen.config_image2d(seed, shape=shape)
    wt = torch.from_numpy(w).to(dev)
    at = [torch.from_numpy(x).to(dev) for x in a]
    results, dt, walls = timed_solves(wt, at, steps, 1, check_every)
    last = results[-1]
    n = w.size
    return {
        "workload": "image2d %dx%d 4-connected, noisy ellipses, lambda=2, dyadic 2^-8, seed %d"
                    % (shape[0], shape[1], seed),
        "solver": "two-set Douglas-Rachford, cold start, certificate every %d iterations" % check_every,
        "time_to_exact_cut_ms": 1e3 * float(np.median(walls)),
        "iters": last.iters,
        "certified": all(q.converged for q in results),
        "energy": last.energy,
        "voxel_sweeps_per_s": sum(n * q.sweep_launches for q in results) / dt,
        "roofline": roofline(last, n, IMG_BYTES_PER_VOXEL_SWEEP, IMG_BYTES_DUALS,
                             "k_sweep<ModeRows2> + k_sweep<ModeCols2> (row and column sweeps)",
                             measured_traffic(IMG_TRAFFIC_PROFILE)),
    }


def grid8_section(seed, shape, repeats=3):
    """The same image with 8-connectivity (rows, columns, two zig-zag chain
    families in the product space): time to the exact cut."""
    import numpy as np
    import torch

    from paper_1503_01563_amd import gen, mc
    dev = torch.device("cuda:0")
    w, a = gen.ellipse_grid8(shape, seed)
    wt = torch.from_numpy(w).to(dev)
    at = [torch.from_numpy(x).to(dev) for x in a]
    mc.tv_solve(wt, at, max_iters=3000, check_every=4)
    times, res = [], None
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = mc.tv_solve(wt, at, max_iters=3000, check_every=4)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    prof = mc.tv_solve(wt, at, max_iters=3000, check_every=4, profile=True)  # per-launch events, untimed
    n = w.size
    return {
        "workload": "image2d %dx%d 8-connected (diagonal weights lambda/sqrt 2), seed %d" % (shape[0], shape[1], seed),
        "time_to_exact_cut_ms": 1e3 * float(np.median(times)),
        "iters": res.iters,
        "certified": res.converged,
        "energy": res.energy,
        "chain_voxel_sweeps_per_s": n * 4 * res.iters / float(np.median(times)),
        "avg_sweep_launch_us": 1e3 * prof.sweep_ms / max(1, prof.sweep_launches),
    }


def alpha_expansion_section(seed=6000, shape=(288, 384), n_labels=16, repeats=3):
    """Multi-label stand-in for the paper's 384 x 288 stereo task: alpha-expansion
    (truncated linear V, T = 2) from all-0 labels, every move an exact cut."""
    import numpy as np
    import torch

    from paper_1503_01563_amd import gen, mc
    dev = torch.device("cuda:0")
    data, lam, true = gen.stereo_labels(shape, seed, n_labels=n_labels)
    dt = torch.from_numpy(data).to(dev)
    lt = [torch.from_numpy(x).to(dev) for x in lam]
    zeros = torch.zeros(shape, dtype=torch.int32, device=dev)
    labels = zeros.clone()
    mc.alpha_expansion(dt, lt, labels, mc.V_TRUNC_LINEAR, 2.0)  # warm-up
    times, res = [], None
    for _ in range(repeats):
        labels = zeros.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = mc.alpha_expansion(dt, lt, labels, mc.V_TRUNC_LINEAR, 2.0)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    # one run each: every move from a cold start, and overlapping-piece sweeps
    def once(**kw):
        lab = zeros.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = mc.alpha_expansion(dt, lt, lab, mc.V_TRUNC_LINEAR, 2.0, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r
    t_cold, r_cold = once(warm=False)
    t_piece, _ = once(whole_chains=False)
    return {
        "workload": "stereo-like %dx%d, %d labels, truncated linear T=2, seed %d" % (shape[1], shape[0], n_labels,
                                                                                      seed),
        "sweeps": "whole chains (one lane per chain)",
        "moves_start": "each move from the same label's previous move (dual reuse), certificate every 2 iterations",
        "time_ms": 1e3 * float(np.median(times)),
        "time_ms_cold_moves": 1e3 * t_cold,
        "dr_iters_cold_moves": int(r_cold.dr_iters),
        "time_ms_piece_sweeps": 1e3 * t_piece,
        "cycles": res.cycles,
        "moves": res.moves,
        "moves_skipped_unchanged": res.skipped,
        "accepted": res.accepted,
        "dr_iters": int(res.dr_iters),
        "energy0": res.energy0,
        "energy": res.energy,
        "all_moves_certified": res.uncertified == 0,
        "local_minimum": res.converged,
        "label_error_vs_truth": float((labels.cpu().numpy() != true).mean()),
    }


def mixed_outer_loop_section(seed=2000, repeats=3):
    """Time to the exact cut of MC_VARIANT_BCD_DR (16 BCD iterations, then the
    splitting from BCD's dual blocks) beside the plain splitting, on the bench
    image and on an iid integer grid."""
    import numpy as np
    import torch

    from paper_1503_01563_amd import gen, mc
    dev = torch.device("cuda:0")
    out = {}
    for name, (w, a) in (("image2d_1024", gen.config_image2d(seed)), ("iid_512", gen.config_warm(130000))):
        wt = torch.from_numpy(w).to(dev)
        at = [torch.from_numpy(x).to(dev) for x in a]
        row = {}
        for vname, var in (("splitting", mc.VARIANT_AUTO), ("bcd_then_splitting", mc.VARIANT_BCD_DR)):
            mc.tv_solve(wt, at, max_iters=6000, check_every=4, variant=var)
            times, res = [], None
            for _ in range(repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = mc.tv_solve(wt, at, max_iters=6000, check_every=4, variant=var)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            row[vname] = {"time_to_exact_cut_ms": 1e3 * float(np.median(times)), "iters": res.iters,
                          "certified": res.converged, "energy": res.energy}
        out[name] = row
    return out


BATCH_BYTES_PER_ITER = 32  # per voxel and two-set iteration: rows z, a -> q1; columns q1, z, w, a -> z'


def batched_section(seed=4000, count=64, repeats=3):
    """64 uneven integer grids (H, W uniform in [128, 1024]) solved together by
    mc_tv_solve_batched: per-grid time to the exact cut (device time from the
    start of the solve to the check that certified the grid), for the replayed
    graph of per-phase launches and for one persistent launch per check
    period.  roofline: the sweeps' algorithmic bytes (32 B per voxel and
    iteration over each grid's iterations) over the whole solve's device time
    -- a lower bound of the sweep kernels' rate, since the solve time also
    holds the checks."""
    import numpy as np
    import torch

    from paper_1503_01563_amd import gen, mc
    dev = torch.device("cuda:0")
    grids = gen.config_batch(seed, count)
    ws = [torch.from_numpy(w).to(dev) for w, _ in grids]
    As = [[torch.from_numpy(x).to(dev) for x in a] for _, a in grids]
    sizes = [w.size for w, _ in grids]
    mc.tv_solve_batched(ws, As, max_iters=3000, check_every=8)  # tunes the work items for this shape

    def design(persistent):
        runs = [mc.tv_solve_batched(ws, As, max_iters=3000, check_every=8, persistent=persistent)
                for _ in range(repeats)]
        r = runs[-1]
        total_ms = float(np.median([np.max(q.ms) for q in runs]))
        algo = float(sum(it * n for it, n in zip(r.iters, sizes))) * BATCH_BYTES_PER_ITER
        achieved = algo / (total_ms * 1e-3) / 1e9
        return {
            "p50_ms": float(np.median([np.percentile(q.ms, 50) for q in runs])),
            "p99_ms": float(np.median([np.percentile(q.ms, 99) for q in runs])),
            "max_ms": total_ms,
            "max_iters": int(max(r.iters)),
            "all_certified": all(q.converged for q in runs),
            "energies": list(r.energy),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_batch_rows + k_batch_cols (whole-solve rate)",
                         "bytes_per_voxel_iteration": BATCH_BYTES_PER_ITER},
        }

    graph = design(False)
    pers = design(True)
    same = graph.pop("energies") == pers.pop("energies")
    return {
        "workload": "%d integer grids, H and W uniform in [128, 1024] (%d voxels), seed %d"
                    % (count, sum(sizes), seed),
        "check_every": 8,
        "items_per_sweep": int(mc.tv_solve_batched(ws, As, max_iters=3000, check_every=8).items),
        "graph_replay": graph,
        "persistent": pers,
        "same_energies": same,
        "p50_ms": graph["p50_ms"],
        "p99_ms": graph["p99_ms"],
        "all_certified": graph["all_certified"] and pers["all_certified"],
    }


def dual_reuse_section(frames=8, shape=(512, 512), frac=0.02):
    """Time to exact cut over a sequence of related problems (an integer grid
    with 2 % of its unaries redrawn per frame), cold against reusing the
    previous frame's dual."""
    from paper_1503_01563_amd import gen, warmstart
    rows = warmstart.sequence_compare(gen.edit_sequence(shape, 7000, frames, frac=frac))
    rows = rows[1:]  # frame 0 has no predecessor
    return {
        "workload": "%d frames of a %dx%d integer grid, %.0f%% of the unaries redrawn per frame"
                    % (frames - 1, shape[0], shape[1], 100 * frac),
        "cold_ms_total": float(sum(r["cold_ms"] for r in rows)),
        "warm_ms_total": float(sum(r["warm_ms"] for r in rows)),
        "cold_iters_total": int(sum(r["cold_iters"] for r in rows)),
        "warm_iters_total": int(sum(r["warm_iters"] for r in rows)),
        "all_certified": all(r["cold_ok"] and r["warm_ok"] for r in rows),
        "same_energy": all(r["cold_energy"] == r["warm_energy"] for r in rows),
        "note": "warm state from the previous frame's row duals (row prox of its final state), "
                "re-clipped to the new weights, plus its primal",
    }


def warm_start_section(n_grids):
    """Time to exact cut, cold vs learned warm start, on held-out 512x512 grids."""
    import numpy as np

    from paper_1503_01563_amd import warmstart
    params, c = warmstart.load_params()
    seeds = range(warmstart.TEST_SEED0, warmstart.TEST_SEED0 + n_grids)
    rows = warmstart.compare(params, c, seeds, repeats=3)
    cold_ms = [r["cold_ms"] for r in rows]
    warm_ms = [r["warm_ms"] for r in rows]
    return {
        "workload": "%d held-out 512x512 integer grids (w in [-20,20], a in [0,10]), seeds %d.."
                    % (n_grids, warmstart.TEST_SEED0),
        "c": c,
        "cold_ms_median": float(np.median(cold_ms)),
        "warm_ms_median": float(np.median(warm_ms)),
        "cold_ms_total": float(np.sum(cold_ms)),
        "warm_ms_total": float(np.sum(warm_ms)),
        "cold_iters_total": int(sum(r["cold_iters"] for r in rows)),
        "warm_iters_total": int(sum(r["warm_iters"] for r in rows)),
        "all_certified": all(r["cold_ok"] and r["warm_ok"] for r in rows),
        "same_energy": all(r["cold_energy"] == r["warm_energy"] for r in rows),
        "note": "warm time includes network inference and the warm state",
    }


if __name__ == "__main__":
    main()
