#!/usr/bin/env python3
"""Throughput of the sparse-tile D3Q19 lattice Boltzmann step on one MI355X.

Workload: D3Q19 BGK quasi-compressible, FP64 PDFs, 256^3 periodic box filled
with seeded overlapping solid spheres (radius 4-12) down to porosity 0.3,
tau = 0.7, body force 1e-6 along x, 4x4x4 tiles (``--model incompressible``:
the paper's incompressible model, Eqs. 4 and 6, on the same workload).  A step is one full time step
(gather propagation + bounce-back + collision) over every non-empty tile;
inputs are resident in HBM before timing starts.

Prints one JSON line: MLUPS over non-solid nodes (the paper's counting,
Sec. 4.2), the roofline of the step kernel (algorithmic bytes 2*q*s_d per
non-solid node per step, Eq. 10, over the HIP-event-timed launch duration)
and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0  # dense BF16 MFMA, MI355X
METRIC = "D3Q19 sparse MLUPS & % HBM peak; time-to-steady-state, warm vs cold, FP32 vs FP64"
SD = {"f64": 8, "f32": 4, "f16": 2}
MODEL_NAME = {"quasi-compressible": "quasi-compressible", "incompressible": "incompressible"}


def model_name(args):
    return "%s %s" % (args.collision.upper(), MODEL_NAME[args.model])


def workload(args):
    from paper_1703_08015_amd import inputs
    if args.geometry == "spheres":
        mask, phi = inputs.spheres_3d(args.n, args.porosity, 4.0, 12.0, seed=args.seed)
        desc = ("D3Q19 %s, %d^3 periodic, overlapping solid spheres r 4-12 to porosity %.2f "
                "(seed %d), tau %.2f, g %.0e along x, 4x4x4 tiles" % (model_name(args), args.n, args.porosity,
                                                                     args.seed, args.tau, args.g))
    elif args.geometry == "vessel":
        mask, phi = inputs.vessel_tree(args.n, 0.08, seed=args.seed)
        desc = ("D3Q19 %s, %d^3 periodic, bifurcating vessel tree r 20->6 (5 generations, "
                "fluid fraction >= 0.08, seed %d), tau %.2f, g %.0e along x, 4x4x4 tiles"
                % (model_name(args), args.n, args.seed, args.tau, args.g))
    elif args.geometry == "channel2d":  # D2Q9: walls at y = 0 and n-1, periodic in x, discs r 3-6 to porosity 0.6
        mask, phi = inputs.channel_2d(args.n, args.n, porosity=0.6, seed=args.seed, max_tries=20_000_000)
        desc = ("D2Q9 %s, %d^2 channel (walls at y = 0 and %d, periodic in x), non-overlapping solid discs r 3-6 "
                "to porosity %.4f (seed %d), tau %.2f, g %.0e along x, 16x16 tiles"
                % (model_name(args), args.n, args.n - 1, phi, args.seed, args.tau, args.g))
    elif args.geometry == "cavity":  # the paper's dense workload: a closed box with a moving lid
        mask, phi = np.zeros((args.n,) * 3, bool), 1.0
        desc = ("D3Q19 %s, %d^3 lid-driven cavity (walls on every face, the +y face moving at %g along x), "
                "tau %.2f, no body force, 4x4x4 tiles" % (model_name(args), args.n, args.lid_u, args.tau))
    else:  # dense sanity point
        mask, phi = np.zeros((args.n,) * 3, bool), 1.0
        desc = "D3Q19 %s, %d^3 fully fluid periodic box, tau %.2f, 4x4x4 tiles" % (model_name(args), args.n,
                                                                                  args.tau)
    return mask, phi, desc


def traffic_for(kernel_name, workload_key):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None.  Returns (bytes, note):
    the figure is recorded, not measured in this run."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        table = json.load(fh)
    rec = table.get(kernel_name, {}).get(workload_key)
    if not rec:
        return None
    src = b""
    for rel in rec.get("source_files", []):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            src += fh.read()
    if not src or rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    note = "recorded %s in profiles/traffic.json from rocprofv3 FETCH_SIZE and WRITE_SIZE runs of the same kernel " \
           "source (L2 misses, including those the MALL serves: an upper bound on HBM bytes)" % rec.get("date", "")
    return rec.get("bytes_per_launch"), note


def step_kernel_key(args):
    """Name of the timed step kernel and the workload key of its traffic record."""
    inc = args.model == "incompressible"
    if args.geometry == "channel2d":
        kernel = "k_step<D2Q9,16x16,%s%s%s%s>" % (args.storage, ",incompressible" if inc else "",
                                                  ",single-copy" if args.pattern == "single-copy" else "",
                                                  ",mrt" if args.collision == "mrt" else "")
        return kernel, "%s_%d_%s_generic_%s" % (args.geometry, args.n, args.storage, args.order)
    kernel = "%s<D3Q19,4x4x4,%s%s%s%s%s>" % ("k_step" if args.kernel == "generic" else "k_step19", args.storage,
                                             ",shuffle" if args.kernel == "shuffle" else "",
                                           ",incompressible" if inc else "",
                                           ",single-copy" if args.pattern == "single-copy" else "",
                                           ",mrt" if args.collision == "mrt" else "")
    wkey = "%s_%d_%s_%s_%s_%s_tpb%d" % (args.geometry, args.n, args.storage,
                                        "scalar" if args.kernel == "auto" else args.kernel, args.order,
                                        "nt" if args.store in ("auto", "nontemporal") else "regular",
                                        args.tiles_per_block or 4)
    return kernel, wkey


def step_setup(args):
    """Body force, periodicity, moving lid, lattice and tile of the step workload."""
    if args.geometry == "cavity":
        return [0.0, 0.0, 0.0], (0, 0, 0), (1, 1, (args.lid_u, 0.0, 0.0)), 19, (4, 4, 4)
    if args.geometry == "channel2d":
        return [args.g, 0.0, 0.0], (1, 0, 0), None, 9, (16, 16, 1)
    return [args.g, 0.0, 0.0], (1, 1, 1), None, 19, (4, 4, 4)


def record_traffic(args, argv):
    """Store the HBM bytes per launch of the step kernel in profiles/traffic.json.

    Input: two rocprofv3 runs of this same command line (without
    --record-traffic), one with ``--pmc FETCH_SIZE`` and one with
    ``--pmc WRITE_SIZE``, written with ``-o run --output-format csv`` into the
    two given folders.  The counters are calibrated on the copy reference of
    the same runs (a fill of --copy-gib GiB, which reads nothing, then copies
    that read and write --copy-gib GiB each), so each counter is scaled by
    true bytes / counted bytes of that kernel.  Runs on the host only."""
    import csv
    fetch_dir, write_dir = args.record_traffic
    if args.copy_gib <= 0:
        raise SystemExit("--record-traffic needs the copy reference (--copy-gib > 0) in the profiled runs")
    kernel, wkey = step_kernel_key(args)
    csv_name = kernel.split("<")[0]

    def values(d, name):
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            return [float(r["Counter_Value"]) for r in csv.DictReader(fh) if r["Kernel_Name"] == name]

    true_kib = args.copy_gib * (1 << 20)
    fc, wc = values(fetch_dir, COPY_KERNEL), values(write_dir, COPY_KERNEL)
    if not fc or not wc:
        raise SystemExit("no %s dispatches in the counter runs" % COPY_KERNEL)
    f_scale, w_scale = true_kib / (sum(fc) / len(fc)), true_kib / (sum(wc) / len(wc))
    fk, wk = values(fetch_dir, csv_name), values(write_dir, csv_name)
    if not fk or not wk:
        raise SystemExit("no %s dispatches in the counter runs" % csv_name)
    fb = sum(fk) / len(fk) * 1024 * f_scale
    wb = sum(wk) / len(wk) * 1024 * w_scale
    generic = args.kernel == "generic" or args.geometry == "channel2d"
    files = ["paper_1703_08015_amd/csrc/%s" % ("kernels.hip" if generic else "step19.hip"),
             "paper_1703_08015_amd/csrc/device.h"]
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in files)
    cmd = " ".join(["python3", "bench.py"] + argv)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    table.setdefault(kernel, {})[wkey] = {
        "bytes_per_launch": int(round(fb + wb)), "fetch_bytes": int(round(fb)), "write_bytes": int(round(wb)),
        "fetch_scale": round(f_scale, 5), "write_scale": round(w_scale, 5),
        "fetch_kib_per_dispatch_raw": round(sum(fk) / len(fk), 1),
        "write_kib_per_dispatch_raw": round(sum(wk) / len(wk), 1),
        "dispatches": [len(fk), len(wk)],
        "source_sha256": hashlib.sha256(src).hexdigest(), "source_files": files,
        "date": time.strftime("%Y-%m-%d", time.gmtime(os.path.getmtime(os.path.join(fetch_dir,
                                                                                 "run_counter_collection.csv")))),
        "commands": ["rocprofv3 --pmc %s -T -d %s -o run --output-format csv -- %s" % (c, d, cmd)
                     for c, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir))]}
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    print(json.dumps({"kernel": kernel, "workload": wkey, "fetch_bytes": int(round(fb)), "write_bytes": int(round(wb)),
                      "fetch_scale": round(f_scale, 5), "write_scale": round(w_scale, 5)}))


def _cpu_model():
    """The host CPU as /proc/cpuinfo reports it: the model name plus the x86
    family / model / stepping numbers (a virtualised host may print only the
    vendor's brand in the name), and lscpu's model name if it differs."""
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    info.setdefault(k.strip(), v.strip())
    except OSError:
        return "unknown"
    name = info.get("model name", "unknown")
    out = "%s (family %s, model %s, stepping %s, %s MHz)" % (name, info.get("cpu family", "?"), info.get("model", "?"),
                                                           info.get("stepping", "?"), info.get("cpu MHz", "?"))
    try:
        import subprocess
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in r.stdout.splitlines():
            if line.startswith("Model name:"):
                ls = line.split(":", 1)[1].strip()
                if ls and ls != name:
                    out += "; lscpu: " + ls
    except (OSError, subprocess.SubprocessError):
        pass
    return out


def cpu_baseline(mask, args):
    """The FP64 oracle on the same geometry: all host cores for a bounded
    number of steps (about 10-30 s of CPU work at the default 160), and one
    thread for a few steps."""
    from oracle import dense
    dense.build()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = dense.INCOMPRESSIBLE if args.model == "incompressible" else dense.QUASI
    # the library's default D3Q19 MRT rates (s_e, s_eps, s_q, s_pi, s_m)
    mrt = (1.19, 1.4, 1.2, 1.4, 1.98) if args.collision == "mrt" else None
    g, per, lid, q, _ = step_setup(args)
    if q == 9:
        mrt = (1.64, 1.54, 1.9, 1.0, 1.0) if args.collision == "mrt" else None
    f = dense.init(q, mask, model=model)
    if lid is not None:
        lid = (lid[0], lid[1], lid[2], 1.0)  # rho_w: rho0 = 1 here, and 1 in the incompressible model
    t0 = time.perf_counter()
    dense.step(q, mask, f, args.tau, g, args.cpu_steps, periodic=per, nthreads=cores, model=model, mrt=mrt, lid=lid)
    dt = time.perf_counter() - t0
    one = max(1, args.cpu_steps // 16)
    t1 = time.perf_counter()
    dense.step(q, mask, f, args.tau, g, one, periodic=per, nthreads=1, model=model, mrt=mrt, lid=lid)
    dt1 = time.perf_counter() - t1
    nf = int((~mask).sum())
    return {"value": nf * args.cpu_steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": "%d steps of the full %d^%d geometry (%d non-solid nodes), FP64 dense C oracle, OpenMP, "
                      "%.1f s" % (args.cpu_steps, args.n, 2 if q == 9 else 3, nf, dt),
            "single_thread_mlups": nf * one / dt1 / 1e6, "single_thread_steps": one, "cpu_model": _cpu_model()}


COPY_KERNEL = "k_copy16"  # lbm_device_copy's kernel, as rocprofv3 -T names it


class CopyReference:
    """Achievable HBM bandwidth of the library's own device copy
    (lbm_device_copy: one 16-byte non-temporal load and store per thread, a
    grid covering the buffer) over buffers of ``gib`` GiB each, timed with HIP
    events on the current stream; the same kernel calibrates the rocprofv3
    byte counters.

    ``launch`` queues copies for at least ``min_seconds`` without waiting for
    them, so that the step's warm-up launches queue right behind them and the
    GPU is never idle in between; ``result`` reads the events afterwards.  The
    GPU's clock and power control needs about 100 ms of sustained memory
    traffic to settle: a step launched after a quiet spell runs up to 9%
    slower for its first few dozen launches (per-launch HIP-event profile:
    309 us, then 325-337 us around launches 10-20, back to 307 us by launch
    60; flat at 306-310 us right after 100 ms of copies)."""

    def __init__(self, torch, lbm, gib):
        self.torch, self.lbm = torch, lbm
        self.n = int(gib * (1 << 30)) // 8
        self.src = torch.ones(self.n, dtype=torch.float64, device="cuda")
        self.dst = torch.empty_like(self.src)

    def launch(self, min_seconds=0.2):
        t = self.torch
        e0, e1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        t.cuda.synchronize()
        e0.record()
        for _ in range(3):
            self.lbm.device_copy(self.dst, self.src)
        e1.record()
        t.cuda.synchronize()
        self.reps = max(10, int(min_seconds / (e0.elapsed_time(e1) / 3 * 1e-3)) + 1)
        self.e0, self.e1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        self.e0.record()
        for _ in range(self.reps):
            self.lbm.device_copy(self.dst, self.src)
        self.e1.record()

    def result(self):
        t = self.torch
        t.cuda.synchronize()
        ms = self.e0.elapsed_time(self.e1) / self.reps
        assert bool((self.dst[:: max(self.n // 4096, 1)] == 1.0).all()), "device copy lost data"
        n = self.n
        del self.src, self.dst
        t.cuda.empty_cache()
        return {"kernel": "lbm_device_copy", "bytes_read": 8 * n, "bytes_written": 8 * n, "ms": round(ms, 4),
                "reps": self.reps, "gbs": round(16 * n / (ms * 1e-3) / 1e9, 1)}


def _progress(tag):
    def f(steps, done, worst):
        print("[%s] %d steps, %d converged, worst residual %.3e" % (tag, steps, done, worst), file=sys.stderr,
              flush=True)
    return f


def _rel_l2(a, b):
    return float(((a - b) ** 2).sum().sqrt() / (b ** 2).sum().sqrt())


def mode_autotune(args, torch, lbm):
    """The autotuner on the step workload (--geometry, --storage): every
    candidate tile shape, step kernel, workgroup size and launch mode timed
    with HIP events (--steps after --warmup), fresh (no cache)."""
    from paper_1703_08015_amd import autotune
    mask, phi, desc = workload(args)
    g, per, lid, q, tile = step_setup(args)
    if lid is not None or q != 19:
        raise SystemExit("--mode autotune runs the D3Q19 step workloads without a lid")
    best = autotune.autotune(mask, periodic=per, lattice=19, storage=args.storage, tau=args.tau, g=tuple(g),
                             steps=args.steps, warmup=args.warmup, cache_path=None, refresh=True)
    trials = sorted(best.pop("trials"), key=lambda t: t.get("ms_per_step", 1e9))
    for t in trials:
        t["tile"] = "x".join(str(a) for a in t["tile"])
    return {"metric": "autotuner trials, ms per step", "unit": "MLUPS", "higher_is_better": True,
            "value": round(best["mlups"], 1), "dtype": args.storage, "data": "synthetic",
            "config": {"workload": desc}, "best": {k: v for k, v in best.items() if k != "cached"},
            "trials": trials}


def mode_steady(args, torch, lbm):
    """Time to steady state (residual < tol over check-interval steps) of the
    workload for FP64 and FP32 storage, and the FP32 steady velocity error
    against the FP64 one."""
    mask, phi, desc = workload(args)
    tiles = lbm.Tiles(mask, (4, 4, 4), (1, 1, 1))
    out = {"metric": "time to steady state (residual < %g)" % args.tol, "unit": "s", "higher_is_better": False,
           "data": "synthetic", "config": {"workload": desc, "n_fluid": tiles.info["n_fluid"],
                                           "check_every": args.check_every}, "runs": {}}
    fields = {}
    for st in ("f64", "f32"):
        s = lbm.Solver(tiles, lattice=19, storage=st, tau=args.tau, g=(args.g, 0.0, 0.0), graph_steps=args.check_every,
                       f16_scale_log2=args.f16_scale_log2, model=args.model, collision=args.collision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.init()
        steps, res = s.run_to_steady(tol=args.tol, check_every=args.check_every, max_steps=args.max_steps,
                                     progress=_progress("steady " + st))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        fields[st] = s.moments()
        out["runs"][st] = {"steps": int(steps[0]), "seconds": round(wall, 3), "residual": float(res[0]),
                           "mlups": round(tiles.info["n_fluid"] * max(int(steps[0]), 0) / wall / 1e6, 1)}
        del s
    fl = torch.from_numpy(~mask).cuda()
    u64, u32 = fields["f64"][1][:, fl], fields["f32"][1][:, fl]
    out["f32_vs_f64_u_rel_l2"] = _rel_l2(u32, u64)
    out["f32_vs_f64_rho_max_abs"] = float((fields["f32"][0][fl] - fields["f64"][0][fl]).abs().max())
    out["value"] = out["runs"]["f64"]["seconds"]
    out["f32_speedup"] = round(out["runs"]["f64"]["seconds"] / out["runs"]["f32"]["seconds"], 3)
    return out


def mode_vessel(args, torch, lbm):
    """Vessel-tree geometry: FP64 / FP32-offset / FP16-offset runs of a fixed
    number of steps; rho and u error of the offset forms against FP64."""
    from paper_1703_08015_amd import inputs
    mask, phi = inputs.vessel_tree(args.n, 0.08, seed=args.seed)
    tiles = lbm.Tiles(mask, (4, 4, 4), (1, 1, 1))
    desc = ("D3Q19 %s, %d^3 periodic, bifurcating vessel tree r 20->6 (5 generations, fluid "
            "fraction %.4f, seed %d), tau %.2f, g %.0e along x, %d steps from rest"
            % (model_name(args), args.n, phi, args.seed, args.tau, args.g, args.vessel_steps))
    out = {"metric": "offset-storage error vs FP64 and MLUPS", "unit": "MLUPS", "higher_is_better": True,
           "data": "synthetic", "config": {"workload": desc, "n_fluid": tiles.info["n_fluid"],
                                           "n_ftiles": tiles.info["n_ftiles"], "phi_t": round(tiles.info["phi_t"], 4),
                                           "f16_scale_log2": args.f16_scale_log2}, "runs": {}}
    fl = torch.from_numpy(~mask).cuda()
    ref = None
    for st in ("f64", "f32", "f16"):
        s = lbm.Solver(tiles, lattice=19, storage=st, tau=args.tau, g=(args.g, 0.0, 0.0),
                       f16_scale_log2=args.f16_scale_log2, model=args.model, collision=args.collision)
        s.init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.vessel_steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r, u = s.moments()
        run = {"mlups": round(tiles.info["n_fluid"] * args.vessel_steps / wall / 1e6, 1),
               "algorithmic_gbs": round(tiles.info["n_fluid"] * 38 * SD[st] * args.vessel_steps / wall / 1e9, 1)}
        if ref is None:
            ref = (r[fl].clone(), u[:, fl].clone())
        else:
            run["u_rel_l2_vs_f64"] = _rel_l2(u[:, fl], ref[1])
            run["rho_max_abs_vs_f64"] = float((r[fl] - ref[0]).abs().max())
        out["runs"][st] = run
        del s, r, u
    out["value"] = out["runs"]["f64"]["mlups"]
    return out


def batch_masks(count, seed):
    from paper_1703_08015_amd import inputs
    specs = inputs.batch_specs(count, seed=seed)
    masks = [inputs.porous_cube(sp)[0] for sp in specs]
    return specs, masks


def mode_batch(args, torch, lbm):
    """Batch of porous cubes (uneven sizes) in one concatenated tile list,
    run to steady state with converged samples dropped from the step."""
    t0 = time.perf_counter()
    specs, masks = batch_masks(args.batch, args.seed + 1000)
    tiles = lbm.Tiles.concat([lbm.Tiles(m) for m in masks])
    t_geom = time.perf_counter() - t0
    s = lbm.Solver(tiles, lattice=19, storage=args.storage, tau=args.tau, persistent=1, graph_steps=args.check_every,
                   f16_scale_log2=args.f16_scale_log2)
    s.set_sample_force(np.array([sp["g"] for sp in specs]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.init()
    steps, res = s.run_to_steady(tol=args.tol, check_every=args.check_every, max_steps=args.max_steps,
                                 progress=_progress("batch"))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    fluid = np.array([int((~m).sum()) for m in masks])
    done = steps > 0
    updates = int((fluid * np.where(done, steps, args.max_steps)).sum())
    desc = ("%d periodic porous cubes, edge uniform over 32..96 step 4, overlapping spheres r 4-12 to porosity "
            "U[0.2, 0.8], |g| = 1e-6 in a uniform direction, tau %.2f, %s storage, residual < %g every %d steps"
            % (args.batch, args.tau, args.storage, args.tol, args.check_every))
    return {"metric": "batched time to steady state", "value": round(wall, 3), "unit": "s", "higher_is_better": False,
            "data": "synthetic", "dtype": args.storage,
            "config": {"workload": desc, "n_samples": len(masks), "n_nodes": tiles.info["n_nodes"],
                       "n_fluid": tiles.info["n_fluid"], "n_ftiles": tiles.info["n_ftiles"]},
            "converged": int(done.sum()), "steps_min": int(steps[done].min()) if done.any() else None,
            "steps_median": int(np.median(steps[done])) if done.any() else None,
            "steps_max": int(steps[done].max()) if done.any() else None,
            "node_updates": updates, "mlups": round(updates / wall / 1e6, 1), "geometry_seconds": round(t_geom, 1)}


def unet_flops(n, levels=4, base=24, in_ch=8, out_ch=12):
    """Dense FLOPs of one U-Net forward pass on an n^3 grid: 2*27*cin*cout per
    voxel and 3x3x3 convolution, 2*8*cin*cout per coarse voxel of a 2x2x2
    transposed convolution, 2*cin*cout per voxel of the 1x1x1 head."""
    C = [base * 2 ** l for l in range(levels)]
    vox = float(n) ** 3
    f, cin = 0.0, in_ch
    for l in range(levels):
        v = vox / 8 ** l
        f += 2 * 27 * cin * C[l] * v + 2 * 27 * C[l] * C[l] * v
        cin = C[l]
    for l in range(levels - 2, -1, -1):
        v = vox / 8 ** l
        f += 2 * 8 * C[l + 1] * C[l] * (v / 8) + 2 * 27 * 2 * C[l] * C[l] * v + 2 * 27 * C[l] * C[l] * v
    return f + 2 * C[0] * ((out_ch + 7) // 8 * 8) * vox


def mode_unet(args, torch, lbm):
    """Throughput of the warm-start network's kernels: one forward pass and one
    training step (forward, backward, Adam) per sample size, HIP events on the
    current stream, against the dense BF16 MFMA peak."""
    from paper_1703_08015_amd import inputs, warmstart
    net = warmstart.make_net(levels=4, base=24, seed=args.seed)
    out = {}
    for n in (64, 128):
        m, _ = inputs.spheres_3d(n, 0.5, 4.0, 12.0, seed=args.seed + 1)
        sm = warmstart.Sample(torch, m, (args.g, 0.0, 0.0))
        x = warmstart.encode(torch, sm)
        dout = torch.zeros(sm.shape + (8,), dtype=torch.bfloat16, device="cuda")

        def timed(fn, reps):
            for _ in range(2):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        def train_step():
            net.forward_mixed(x, sm.dir)
            net.zero_grad()
            net.backward_mixed(dout, 8, sm.dir)
            net.adam_step(1e-6)

        fwd = timed(lambda: net.forward_mixed(x, sm.dir), 10)
        trn = timed(train_step, 5)
        F = unet_flops(n)
        out["%d^3" % n] = {"forward_ms": round(fwd, 3), "forward_tflops": round(F / fwd / 1e9, 1),
                           "train_step_ms": round(trn, 3), "train_tflops": round(3 * F / trn / 1e9, 1),
                           "gflop_forward": round(F / 1e9, 1)}
    big = out["128^3"]
    return {"metric": "U-Net forward throughput (warm-start network)", "unit": "TFLOP/s",
            "value": big["forward_tflops"], "higher_is_better": True, "dtype": "bf16 (fp32 accumulate)",
            "data": "synthetic",
            "config": {"workload": "U-Net 4 levels x 24 base channels, %d parameters, on 128^3 and 64^3 porous "
                                   "cubes (distance input), batch 1" % net.n_params()},
            "roofline": {"bound": "mfma", "achieved": big["forward_tflops"], "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(big["forward_tflops"] / BF16_PEAK_TFLOPS, 4),
                         "traffic": None},
            "sizes": out}


def mode_warmstart(args, torch, lbm):
    """Train the U-Net on steady states of the porous-cube batch (every cube;
    those whose edge is not a multiple of 8 tiled twice per axis, an exact
    periodic image), then compare warm and cold starts to the same residual
    on held-out 128^3 porous samples, and measure steps against the error of
    the starting fields on the first few of them."""
    from paper_1703_08015_amd import inputs, warmstart
    t0 = time.perf_counter()
    specs = inputs.batch_specs(args.batch, seed=args.seed + 1000)
    masks = [inputs.porous_cube(sp)[0] for sp in specs]
    data, steps, _ = warmstart.steady_dataset(torch, masks, [sp["g"] for sp in specs], tau=args.tau,
                                              progress=_progress("data"))
    data = [warmstart.training_view(torch, sm) for sm in data]
    t_data = time.perf_counter() - t0
    out_scale = warmstart.make_targets(torch, data, args.tau)
    net = warmstart.make_net(levels=4, base=24, seed=args.seed, out_scale=out_scale)
    t1 = time.perf_counter()
    hist = warmstart.train(torch, net, data, epochs=args.epochs, lr=args.lr,
                           progress=lambda ep, l: print("[train] epoch %d loss %.4e" % (ep, l), file=sys.stderr,
                                                        flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del data
    torch.cuda.empty_cache()
    rng = np.random.default_rng(args.seed + 5000)
    tests = []
    for k in range(args.test_samples):
        phi = float(rng.uniform(0.3, 0.7))
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        m, _ = inputs.spheres_3d(128, phi, 4.0, 12.0, seed=args.seed + 5000 + k)
        tests.append(warmstart.Sample(torch, m, (1e-6 * d).tolist()))
    rows = []
    for k, sm in enumerate(tests):
        r = warmstart.evaluate(torch, net, [sm], args.tau, fp64_cold=True)[0]
        print("[eval] sample %d cold f64 %d steps %.2fs, cold %d steps %.2fs, warm %d steps %.2fs, pred err %.3f, "
              "agree %.1e (vs f64 %.1e)%s"
              % (k, r["cold_f64_steps"], r["cold_f64_s"], r["cold_steps"], r["cold_s"], r["warm_steps"], r["warm_s"],
                 r["prediction_u_rel_l2"], r["warm_vs_cold_u_rel_l2"], r["warm_vs_cold_f64_u_rel_l2"],
                 " (fell back)" if r["fell_back"] else ""), file=sys.stderr, flush=True)
        rows.append(r)
    curves = []
    for k, sm in enumerate(tests[:args.curve_samples]):
        cold, pts = warmstart.error_curve(torch, net, sm, args.tau)
        print("[curve] sample %d cold %d steps; %s" % (k, cold["cold_steps"], ", ".join(
            "err %.3g -> %d steps" % (p["start_u_rel_l2"], p["steps"]) for p in pts)), file=sys.stderr, flush=True)
        curves.append(dict(sample=k, **cold, points=pts))
    cold_s = sum(r["cold_s"] for r in rows)
    warm_s = sum(r["warm_s"] for r in rows)
    return {"metric": "time to steady state, warm vs cold start", "unit": "s", "higher_is_better": False,
            "value": round(warm_s, 3), "data": "synthetic", "dtype": "f32 (solver), bf16 (network)",
            "config": {"workload": "%d held-out 128^3 periodic porous samples (spheres r 4-12, porosity U[0.3, 0.7], "
                                   "|g| 1e-6 random direction), tau %.2f, FP32 LBM to residual %g" %
                                   (args.test_samples, args.tau, args.tol),
                       "network": "U-Net 4 levels, 24 base channels, %d parameters" % net.n_params(),
                       "training": "%d porous cubes (edges 32..96; edges not a multiple of 8 tiled twice per "
                                   "axis), %d epochs, Adam lr %g" % (len(specs), args.epochs, args.lr)},
            "cold_seconds": round(cold_s, 3), "warm_seconds_incl_inference": round(warm_s, 3),
            "speedup": round(cold_s / warm_s, 3) if warm_s > 0 else None,
            "cold_f64_seconds": round(sum(r["cold_f64_s"] for r in rows), 3),
            "speedup_vs_cold_f64": round(sum(r["cold_f64_s"] for r in rows) / warm_s, 3) if warm_s > 0 else None,
            "warm_vs_cold_f64_u_rel_l2_max": float(np.max([r["warm_vs_cold_f64_u_rel_l2"] for r in rows])),
            "labels_seconds_in_warm": round(sum(r["labels_s"] for r in rows), 3),
            "inference_seconds_in_warm": round(sum(r["inference_s"] for r in rows), 3),
            "cold_steps_mean": float(np.mean([r["cold_steps"] for r in rows])),
            "warm_steps_mean": float(np.mean([r["warm_steps"] for r in rows])),
            "prediction_u_rel_l2_mean": float(np.mean([r["prediction_u_rel_l2"] for r in rows])),
            "prediction_u_rel_l2_best_scale_mean": float(np.mean([r["prediction_u_rel_l2_best_scale"]
                                                                  for r in rows])),
            "prediction_best_scale_mean": float(np.mean([r["prediction_best_scale"] for r in rows])),
            "warm_vs_cold_u_rel_l2_max": float(np.max([r["warm_vs_cold_u_rel_l2"] for r in rows])),
            "fallbacks": int(sum(r["fell_back"] for r in rows)),
            "train_loss_first_last": [hist[0], hist[-1]], "data_seconds": round(t_data, 1),
            "train_seconds": round(t_train, 1), "rows": rows, "error_curves": curves}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f64", choices=["f64", "f32", "f16"])
    ap.add_argument("--geometry", default="spheres", choices=["spheres", "vessel", "dense", "cavity", "channel2d"])
    ap.add_argument("--lid-u", type=float, default=0.05, help="lid velocity of --geometry cavity")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--porosity", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tau", type=float, default=0.7)
    ap.add_argument("--g", type=float, default=1e-6)
    ap.add_argument("--tiles-per-block", type=int, default=0)
    ap.add_argument("--order", default="morton", choices=["morton", "rowmajor"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "generic", "scalar", "shuffle"])
    ap.add_argument("--store", default="auto", choices=["auto", "regular", "nontemporal"])
    ap.add_argument("--f16-scale-log2", type=int, default=22)
    ap.add_argument("--cpu-steps", type=int, default=160)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--model", default="quasi-compressible", choices=["quasi-compressible", "incompressible"],
                    help="fluid model of the collision (modes step, steady and vessel)")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "mrt"],
                    help="collision operator: BGK (Eq. 2) or MRT (Eq. 8, published default rates) "
                         "(modes step, steady and vessel)")
    ap.add_argument("--pattern", default="two-copy", choices=["two-copy", "single-copy"],
                    help="PDF buffers: the paper's two copies, or one copy updated in place (step mode)")
    ap.add_argument("--mode", default="step",
                    choices=["step", "steady", "vessel", "batch", "warmstart", "unet", "autotune"])
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--test-samples", type=int, default=16)
    ap.add_argument("--curve-samples", type=int, default=4,
                    help="warmstart mode: held-out samples on which steps are measured against the start error")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--max-steps", type=int, default=200000)
    ap.add_argument("--vessel-steps", type=int, default=5000)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--copy-gib", type=float, default=4.0,
                    help="size of the device copy reference (read + write each this many GiB); 0 = skip")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="host only: store the step kernel's HBM bytes from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this command line in profiles/traffic.json")
    argv = sys.argv[1:]
    args = ap.parse_args()
    if args.mode == "step" and args.geometry == "channel2d" and args.n == 256:
        args.n = 4096  # a D2Q9 domain large enough to hide launch gaps
    if args.record_traffic:
        k = argv.index("--record-traffic")
        record_traffic(args, argv[:k] + argv[k + 3:])
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sparse-tile step is built and timed on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1703_08015_amd import lbm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.mode in ("batch", "warmstart", "unet") and (args.model != "quasi-compressible" or args.collision != "bgk"):
        print("--model and --collision apply to the step, steady and vessel modes only", file=sys.stderr)
        sys.exit(2)
    if args.mode != "step" and args.pattern != "two-copy":
        print("--pattern applies to the step mode only", file=sys.stderr)
        sys.exit(2)
    if args.mode != "step":
        if args.mode == "vessel" and args.n == 256:
            args.n = 448
        if args.mode in ("batch", "warmstart"):
            args.tau = 0.8 if args.tau == 0.7 else args.tau
            args.storage = "f32" if args.storage == "f64" else args.storage
        res = {"steady": mode_steady, "vessel": mode_vessel, "batch": mode_batch, "autotune": mode_autotune,
               "warmstart": mode_warmstart, "unet": mode_unet}[args.mode](args, torch, lbm)
        res["n_gpus"] = 1
        print(json.dumps(res), flush=True)
        return
    mask, phi, desc = workload(args)
    g, per, lid, q, tile = step_setup(args)
    tiles = lbm.Tiles(mask, tile, per)
    info = tiles.info
    solver = lbm.Solver(tiles, lattice=q, storage=args.storage, tau=args.tau, g=g,
                        tiles_per_block=args.tiles_per_block, f16_scale_log2=args.f16_scale_log2,
                        tile_order=args.order, step_kernel=args.kernel, store_policy=args.store, model=args.model,
                        pattern=args.pattern, collision=args.collision)
    if lid is not None:
        solver.set_lid(*lid)
    solver.init()
    # the copy reference runs right before the step's warm-up, which queues
    # behind it on the same stream with no idle gap
    copy = CopyReference(torch, lbm, args.copy_gib) if args.copy_gib > 0 else None
    if copy:
        copy.launch()
    solver.step(args.warmup)
    torch.cuda.synchronize()

    stream = solver.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    solver.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = ev0.elapsed_time(ev1) / args.steps

    copy_ref = copy.result() if copy else None
    # the state must still be physical after the timed steps
    tot = solver.reduce()[0]
    if not np.all(np.isfinite(tot)):
        raise RuntimeError("non-finite state after the timed steps")

    nf = info["n_fluid"]
    sd = SD[args.storage]
    mlups = nf * args.steps / wall / 1e6
    alg_bytes = nf * 2 * q * sd  # Eq. (10) per non-solid node, per launch
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    # D3Q19 on 4x4x4 tiles runs the scalar-mask kernel unless the generic one is asked for
    kernel, wkey = step_kernel_key(args)
    traffic, traffic_note = traffic_for(kernel, wkey) or (None, None)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {
            "workload": desc,
            "n_fluid": nf, "n_ftiles": info["n_ftiles"], "n_tiles": info["n_tiles"],
            "phi": round(info["phi"], 4), "phi_t": round(info["phi_t"], 4),
            "tiles_ratio": round(info["tiles_ratio"], 4), "bytes_per_fluid_node": 2 * q * SD[args.storage],
            "storage": args.storage, "tiles_per_block": args.tiles_per_block or 4,
            "tile_order": args.order, "step_kernel": args.kernel, "store_policy": args.store,
            "fluid_model": args.model, "pattern": args.pattern, "collision": args.collision,
            "workspace_bytes": solver.workspace.numel(),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "traffic_source": traffic_note,
            # measured overhead over the algorithmic bytes (the paper's Delta^B, Table 5)
            "delta_b": round(traffic / alg_bytes - 1.0, 4) if traffic else None,
            "kernel": kernel, "algorithmic_bytes_per_launch": alg_bytes, "launch_ms": round(launch_ms, 5),
        },
        "bu_eq43": round(mlups * 1e6 * 2 * q * sd / (HBM_PEAK_GBS * 1e9), 4),
    }
    if copy_ref:
        out["copy_reference"] = copy_ref
        out["roofline"]["frac_of_copy"] = round(achieved / copy_ref["gbs"], 4)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mask, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
