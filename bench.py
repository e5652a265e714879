"""Throughput of the fused difference-free CPF-LBM step on one MI355X.

Workload: Rayleigh-Taylor instability on a 128 x 512 x 128 lattice
(8,388,608 nodes), heavy fluid on top (At = 0.5), single-mode perturbation
of amplitude 0.05 Lx, Re = 256, W = 4, sigma = 5e-5, periodic in x and z,
no-slip walls in y, Courant number 0.997; FP32 collision with the
populations stored in HBM as FP16 deviations (synthetic initial fields).
A step is the fused update (propagation, moments, both collisions, store)
of the whole lattice: one launch over the tiles that touch no wall and one
over the two wall slabs (plus the FP64 phase-mass bookkeeping every 10
steps); the reported value is MLUPS = nodes x steps / (seconds x 1e6), timed
with HIP events on the solver's stream with the state resident in HBM, and
the roofline figure divides the algorithmic bytes of a step by that step
time. The same run reports the BF16- and FP32-storage rates and the rate of
the finite-difference-normal comparison scheme (Sec. 3.4: grad phi by
central differences of a stored phi field, a second pass per step) in the
same storage mode, and the rate of the same step on the D3Q27 lattice
(224 instead of 160 algorithmic bytes per update in FP16 storage).
"roofline" also carries the bandwidth of a plain 1 GiB streaming copy on
the same GPU (probe_copy, include/probe.h: half read, half write, as the
step) and the step's fraction of it. "workloads" gives the rates of the
static droplet (32^3, FP64 and FP16), the rising bubble (128 x 128 x 256,
walls on all faces) and the Taylor-Green breakup (256^3) in FP16 and FP32.
"horizons" runs those three problems over their configured horizons (20k,
30k and 40k steps; FP16 and FP32 storage) with the observables of the
paper's Sec. 3: Rayleigh-Taylor spike and bubble fronts, the bubble's
centroid and rise velocity, the Taylor-Green fragment count and kinetic
energy, and the phase-mass drift of each (paper_2407_12263_amd/runs.py).

The "surrogate" object covers the learned part on the emulsion workload
(256^3 periodic, 200 droplets, random solenoidal velocity): the coarse-grid
U-Net is trained on the GPU from solver trajectories of held-out seeds
(32 trajectories x 65 snapshots by default), then a test seed is run for
1024 steps by the plain solver and by each surrogate schedule; it reports
wall time, speedup, phi relative L2 error against the plain run, fallbacks,
the same schedules with a persistence predictor, and the error floor of the
fine-grid reconstruction. Its "unet_roofline" object gives the network's
forward time on the 128^3 coarse grid (HIP events) against the dense BF16
MFMA peak, the training-step time, and beside them the oracle's forward
(FP64 NumPy) on a 64^3 sample, FLOP-scaled to one 128^3 forward, and its
training step on 32^3 scaled to 128^3. Its "coupling" object gives the wall
time of the transfer operations of a surrogate cycle (snapshot, base copy,
checks, level-set push with the solver rebuild) beside the coupling
oracle's round at the same 256^3 / 128^3 size.

Prints ONE JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline; surrogate-vs-LBM speedup at φ L2 err ≤1e-2"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2407_12263_amd/csrc/lbm_kernels.hpp", "paper_2407_12263_amd/csrc/lbm.hip"]
COUNTERS_FILE = "profiles/step_kernel_rayleigh_taylor_128x512x128_fp16.counters.txt"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(launch_bytes_alg: float):
    """HBM bytes per step (FETCH_SIZE and WRITE_SIZE of the step's launches,
    calibrated on a plain copy) from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, COUNTERS_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_step"])
    except (KeyError, ValueError):
        return None


def time_solver(sol, steps: int, warmup: int):
    import torch
    sol.step(warmup)
    torch.cuda.synchronize()
    stream = sol.stream
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        start.record(stream)
        sol.step(steps)
        end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3  # seconds


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


WORKLOADS = {
    # the paper's other test problems at the sizes of their configurations
    "static_droplet_32": (lambda inputs: inputs.static_droplet(), ("fp64", "fp16")),
    "rising_bubble_128x128x256": (lambda inputs: inputs.rising_bubble(), ("fp16", "fp32")),
    "taylor_green_256": (lambda inputs: inputs.taylor_green_breakup(), ("fp16", "fp32")),
}


def workload_rates(steps: int, warmup: int) -> dict:
    """MLUPS and the algorithmic-byte fraction of the HBM peak for the static
    droplet (32^3 periodic), the rising bubble (128 x 128 x 256, walls on all
    faces) and the Taylor-Green breakup (256^3 periodic), timed as the main
    workload."""
    import torch
    from paper_2407_12263_amd import inputs, lbm
    out = {}
    for name, (mk, precs) in WORKLOADS.items():
        w = mk(inputs)
        for prec in precs:
            print(f"[bench] {w.name} storage={prec} steps={steps}", file=sys.stderr, flush=True)
            sol = lbm.Solver(dict(w.params(), precision=prec), w.phi0, w.u0, w.p0)
            secs = time_solver(sol, steps, warmup)
            gbs = lbm.BYTES_PER_LU[prec] * w.N * steps / secs / 1e9
            out[f"{name}_{prec}"] = dict(mlups=round(w.N * steps / secs / 1e6, 1),
                                         ms_per_step=round(secs * 1e3 / steps, 5),
                                         grid=[w.nx, w.ny, w.nz], walls=list(w.wall),
                                         achieved_gbs=round(gbs, 1),
                                         hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
            del sol
            torch.cuda.synchronize()
    return out


def cpu_baseline(w, steps: int = 2):
    """The FP64 CPU oracle, untuned, on the full lattice of the same workload
    for a few steps (bounded sample), on all host threads and then one step
    on one thread; returns (MLUPS, threads, seconds, single-thread MLUPS)."""
    import oracle
    oracle.build(force=False)
    P = oracle.OracleParams(**w.params())
    o = oracle.Oracle(P, w.phi0, w.u0, w.p0)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    o.step(1)
    dt1 = time.perf_counter() - t1
    oracle.set_num_threads(threads)
    del o
    return w.N * steps / dt / 1e6, threads, dt, w.N / dt1 / 1e6


def unet_cpu_baseline(n: int = 64):
    """The oracle's U-Net forward (FP64 NumPy, untuned) once on an n^3 grid
    with random weights (bounded sample); returns (GFLOP/s, threads, seconds,
    FLOP of the sample)."""
    import numpy as np
    from oracle import surrogate_oracle as so
    ch = (16, 32, 48, 64)
    rng = np.random.default_rng(0)
    layers = so.unet_layers(ch)
    params = [(rng.standard_normal((27, co, ci)) * 0.05, np.zeros(co)) for _, ci, co, _ in layers]
    x = rng.standard_normal((n, n, n, 16))
    lev = lambda name: 0 if name == "out" else int(name[3:-1])
    flop = sum(2 * 27 * ci * co * (n >> lev(name)) ** 3 for name, ci, co, _ in layers)
    t0 = time.perf_counter()
    so.unet_forward(x, params, ch)
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = 1
    return flop / dt / 1e9, threads, dt, flop


def train_cpu_baseline(n: int = 32):
    """The oracle's training step (U-Net forward, MSE, backward, Adam; FP64
    NumPy, untuned) once on an n^3 grid; returns seconds."""
    import numpy as np
    from oracle import surrogate_oracle as so
    ch = (16, 32, 48, 64)
    rng = np.random.default_rng(0)
    params = [(rng.standard_normal((27, co, ci)) * 0.05, np.zeros(co))
              for _, ci, co, _ in so.unet_layers(ch)]
    x = rng.standard_normal((n, n, n, 16))
    t0 = time.perf_counter()
    out, cache = so.unet_forward(x, params, ch)
    _, dout = so.mse(out, np.zeros_like(out), np.ones(5))
    grads = so.unet_backward(dout, params, ch, cache)
    for (w, _), (gw, _) in zip(params, grads):
        so.adam(w, np.zeros_like(w), np.zeros_like(w), gw, 1)
    return time.perf_counter() - t0


def coupling_cpu_baseline(n: int = 256):
    """The coupling oracle's round at the full size (fine n^3, coarse
    (n/2)^3): coarsen, level-set prolongation with mass restoration,
    features and checks (FP64 NumPy); returns seconds."""
    import numpy as np
    from oracle import coupling_oracle as co
    rng = np.random.default_rng(0)
    shp = (n, n, n)
    phi, u, p = rng.random(shp), 0.02 * rng.standard_normal((3,) + shp), 4e-4 * rng.standard_normal(shp)
    scale = np.array([1.0, 0.02, 0.02, 0.02, 4e-4] + [1.0] * 11)
    t0 = time.perf_counter()
    s0 = co.coarsen(phi, u, p, scale)
    co.checks(co.features(s0))
    co.prolong_update(s0, s0, scale, 4.0, phi, u, p)
    return time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--storage", default="fp16", choices=["fp16", "bf16", "fp32", "fp64"])
    ap.add_argument("--secondary", default="bf16,fp32,fp16+fd,fp16+q27",
                    help="comma list of extra runs: storage mode, '+fd' for the "
                         "finite-difference-normal comparison scheme, '+q27' for D3Q27")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate-accelerated emulsion runs")
    ap.add_argument("--surrogate-trajectories", type=int, default=32,
                    help="training trajectories of 64 windows (32 -> 2080 snapshots)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the droplet, rising-bubble and Taylor-Green rates")
    ap.add_argument("--no-horizons", action="store_true",
                    help="skip the runs of the 3D test problems over their horizons")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the step would shard by z-slabs with one halo exchange per step)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_12263_amd import inputs, lbm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lbm.load_library()

    w = inputs.rayleigh_taylor()  # 128 x 512 x 128, Re = 256, At = 0.5
    results = {}
    modes = [args.storage] + [m for m in args.secondary.split(",") if m and m != args.storage]
    def parse_mode(mode):
        parts = mode.split("+")
        return parts[0], int("fd" in parts[1:]), 27 if "q27" in parts[1:] else 19

    for mode in modes:
        prec, fd, q = parse_mode(mode)
        print(f"[bench] {w.name} storage={prec} normal_fd={fd} lattice=D3Q{q} "
              f"warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)
        sol = lbm.Solver(dict(w.params(), precision=prec, normal_fd=fd, lattice=q), w.phi0, w.u0,
                         w.p0)
        secs = time_solver(sol, args.steps, args.warmup)
        d = sol.diagnostics()
        ok = all(map(lambda v: v == v, [d["sum_phi"], d["umax"]]))
        results[mode] = dict(seconds=secs, ms_per_step=secs * 1e3 / args.steps,
                             mlups=w.N * args.steps / secs / 1e6, finite=ok,
                             sum_phi=d["sum_phi"], umax=d["umax"])
        del sol
        torch.cuda.synchronize()

    main_r = results[args.storage]
    bpl = lbm.BYTES_PER_LU[args.storage]
    launch_bytes = bpl * w.N
    launch_s = main_r["seconds"] / args.steps
    achieved = launch_bytes / launch_s / 1e9
    traffic = measured_traffic(launch_bytes)
    from paper_2407_12263_amd import probe
    print("[bench] streaming copy probe, 1 GiB", file=sys.stderr, flush=True)
    copy = probe.copy_bandwidth()
    line = {
        "metric": METRIC,
        "value": round(main_r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name} rayleigh-taylor At=0.5 Re=256 W=4 c=0.997",
                   "grid": [w.nx, w.ny, w.nz], "nodes": w.N, "storage": args.storage,
                   "walls": "y", "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes_per_step": launch_bytes,
                     "kernel": "step_kernel (fused propagate+moments+collide+store; interior "
                               "and wall-slab launches)",
                     "copy_gbs": copy["copy_gbs"],
                     "frac_of_copy": round(achieved / copy["copy_gbs"], 4),
                     "copy_probe": copy},
        # the comparison scheme (fd) moves more than the difference-free
        # step's bytes per node, so its fraction is an effective rate at
        # those bytes
        "secondary": {m: {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 5),
                          ("effective_hbm_frac" if parse_mode(m)[1] else "hbm_frac"):
                              round((lbm.BYTES_PER_LU_Q27 if parse_mode(m)[2] == 27
                                     else lbm.BYTES_PER_LU)[parse_mode(m)[0]] * w.N
                                    / (r["seconds"] / args.steps) / 1e9 / HBM_PEAK_GBS, 4)}
                      for m, r in results.items() if m != args.storage},
        "checks": {m: {"finite": r["finite"], "sum_phi": r["sum_phi"], "umax": r["umax"]}
                   for m, r in results.items()},
    }
    if not args.no_workloads:
        line["workloads"] = workload_rates(args.steps, args.warmup)
    if not args.no_horizons:
        from paper_2407_12263_amd import runs
        print("[bench] horizons: Rayleigh-Taylor 20k, rising bubble 30k, Taylor-Green 40k steps",
              file=sys.stderr, flush=True)
        line["horizons"] = runs.horizons(log=lambda *a: print(*a, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline: oracle FP64, {args.cpu_steps} steps on the full lattice",
              file=sys.stderr, flush=True)
        mlups, threads, dt, mlups1 = cpu_baseline(w, args.cpu_steps)
        line["cpu_baseline"] = {"value": round(mlups, 3), "unit": "MLUPS", "cores": threads,
                                "kind": "oracle", "cpu_model": cpu_model(),
                                "sample": f"{args.cpu_steps} steps of the full {w.nx}x{w.ny}x{w.nz} "
                                          f"lattice in FP64 ({dt:.1f} s)",
                                "single_thread_value": round(mlups1, 3)}
    if not args.no_surrogate:
        from paper_2407_12263_amd import accel
        print(f"[bench] surrogate: emulsion 256^3, {args.surrogate_trajectories} training "
              "trajectories", file=sys.stderr, flush=True)
        try:
            line["surrogate"] = accel.surrogate_benchmark(
                train_seeds=tuple(range(1000, 1000 + args.surrogate_trajectories)),
                log=lambda *a: print(*a, file=sys.stderr, flush=True))
        except Exception as e:  # the main metric is still reported
            line["surrogate"] = {"error": f"{type(e).__name__}: {e}"}
        ur = line["surrogate"].get("unet_roofline")
        if ur and not args.no_cpu_baseline:
            print("[bench] cpu baseline: oracle U-Net forward on 64^3", file=sys.stderr, flush=True)
            gflops, threads, dt, flop = unet_cpu_baseline(64)
            ur["cpu_baseline"] = {"value": round(ur["flop_per_forward"] / (gflops * 1e9) * 1e3, 1),
                                  "unit": "ms per forward (FLOP-scaled)", "gflops": round(gflops, 2),
                                  "cores": threads, "kind": "oracle",
                                  "sample": f"one forward pass on a 64^3 grid in FP64 "
                                            f"({flop / 1e9:.1f} GFLOP, {dt:.1f} s)"}
            dt = train_cpu_baseline(32)
            ur["train_cpu_baseline"] = {"value": round(dt * 64 * 1e3, 1),
                                        "unit": "ms per training step (scaled by points)",
                                        "cores": threads, "kind": "oracle",
                                        "sample": f"one training step on a 32^3 grid in FP64 "
                                                  f"({dt:.1f} s), x 64 for 128^3"}
        cpl = line["surrogate"].get("coupling")
        if cpl and not args.no_cpu_baseline:
            print("[bench] cpu baseline: coupling oracle at 256^3", file=sys.stderr, flush=True)
            dt = coupling_cpu_baseline(256)
            cpl["cpu_baseline"] = {"value": round(dt * 1e3, 1), "unit": "ms per round",
                                   "kind": "oracle",
                                   "sample": "coarsen, features, checks and level-set "
                                             "prolongation at 256^3 / 128^3 in FP64, once"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
