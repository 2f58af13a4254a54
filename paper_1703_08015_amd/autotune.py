"""Autotuner for the sparse-tile step: tile shape x workgroup size x launch mode.

Each candidate builds its own tiling and solver through the C ABI, runs a
warm-up, then times ``steps`` steps with HIP events on the solver's stream;
the fastest candidate wins.  Results are cached in a JSON file keyed by the
lattice, storage form, relaxation time and a hash of the geometries, so a
geometry is tuned once.
"""
import hashlib
import json
import os
import time

import numpy as np

from . import lbm

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lbm_autotune.json")


def candidates(lattice=19, batched=False):
    """Configurations tried for a lattice.  A batch that drops converged
    samples needs the scalar-mask kernel (4x4x4 or 4x4x8 tiles)."""
    if lattice == 9:
        return [dict(tile=(16, 16, 1), tiles_per_block=4, persistent=0, step_kernel="generic")]
    out = []
    for tpb in (1, 2, 4, 8):
        for persistent in (0, 1):
            out.append(dict(tile=(4, 4, 4), tiles_per_block=tpb, persistent=persistent, step_kernel="scalar"))
    for tpb in (1, 4):  # coalesced own loads, in-tile sources from other lanes
        out.append(dict(tile=(4, 4, 4), tiles_per_block=tpb, persistent=0, step_kernel="shuffle"))
    # 4x4x8 tiles on the scalar-mask kernel (each tile two 4x4x4 wavefronts)
    for tpb in (2, 4, 8):
        for persistent in (0, 1):
            out.append(dict(tile=(4, 4, 8), tiles_per_block=tpb, persistent=persistent, step_kernel="scalar"))
    if not batched:
        for tpb in (1, 4):
            out.append(dict(tile=(4, 4, 8), tiles_per_block=tpb, persistent=0, step_kernel="generic"))
    return out


def geometry_key(masks, periodic, lattice, storage, tau):
    h = hashlib.sha256()
    for m in masks:
        m = np.ascontiguousarray(np.asarray(m).astype(np.uint8))
        h.update(np.array(m.shape, np.int64).tobytes())
        h.update(m.tobytes())
    h.update(repr((tuple(periodic), lattice, storage, float(tau))).encode())
    return h.hexdigest()


def _time_candidate(torch, masks, periodic, cand, lattice, storage, tau, g, steps, warmup):
    parts = [lbm.Tiles(m, cand["tile"], periodic) for m in masks]
    tiles = parts[0] if len(parts) == 1 else lbm.Tiles.concat(parts)
    s = lbm.Solver(tiles, lattice=lattice, storage=storage, tau=tau, g=g, tiles_per_block=cand["tiles_per_block"],
                   persistent=cand["persistent"], step_kernel=cand["step_kernel"])
    s.init()
    # at least `warmup` steps and 0.1 s of them: the host tiling before each
    # candidate leaves the GPU idle, and the clock and power control needs
    # about that long of sustained load to settle
    t0 = time.perf_counter()
    s.step(warmup)
    torch.cuda.synchronize()
    while time.perf_counter() - t0 < 0.1:
        s.step(max(warmup, 10))
        torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    n_fluid = tiles.info["n_fluid"]
    del s
    return ms, n_fluid


def autotune(masks, periodic=(1, 1, 1), lattice=19, storage="f64", tau=0.7, g=(0.0, 0.0, 0.0), steps=30,
             warmup=5, cache_path=DEFAULT_CACHE, batched=None, refresh=False):
    """Return the fastest configuration for the geometries ``masks`` (one mask
    or a list of masks run as one batch) as a dict with the keys of
    ``candidates`` plus ``ms_per_step``, ``mlups`` and the full ``trials``."""
    import torch

    if isinstance(masks, np.ndarray):
        masks = [masks]
    if batched is None:
        batched = len(masks) > 1
    key = geometry_key(masks, periodic, lattice, storage, tau)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if not refresh and key in cache:
        best = dict(cache[key])
        best["tile"] = tuple(best["tile"])
        best["cached"] = True
        return best
    trials = []
    for cand in candidates(lattice, batched):
        try:
            ms, nf = _time_candidate(torch, masks, periodic, cand, lattice, storage, tau, g, steps, warmup)
        except lbm.LbmError as e:  # e.g. a periodic axis the tile shape does not divide
            trials.append(dict(cand, error=str(e)))
            continue
        trials.append(dict(cand, ms_per_step=ms, mlups=nf / (ms * 1e-3) / 1e6))
    ok = [t for t in trials if "ms_per_step" in t]
    if not ok:
        raise RuntimeError("no candidate configuration ran: %s" % trials)
    best = dict(min(ok, key=lambda t: t["ms_per_step"]))
    best["trials"] = trials
    if cache_path:
        cache[key] = dict(best, tile=list(best["tile"]))
        os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    best["cached"] = False
    return best
