"""Parity at the full workload sizes, in the launch configuration that bench.py
times, on sampled outputs.

At these sizes the dense oracle cannot step the whole domain in a test, but
it can compute any single node's state after K steps: that depends only on
the node's (2K+1)^3 neighbourhood (Eq. 1 pulls from x - c_i, Eq. 2 collides
locally).  Each case draws a seeded random macroscopic state (rho, u) from
the input generator, initialises the GPU solver with it (Eq. 3) and runs
K = 2 steps.  For every sampled fluid node the oracle initialises a 5^3 crop
of the same (rho, u) (periodic wrap; the crops laid side by side along x in
one non-periodic domain, so that a crop's centre depends only on its own
crop) and runs the same K steps; the crop's centre is compared with the GPU's
exported state there.  No oracle input comes from the GPU.  The samples
include nodes on the domain faces, where the periodic wrap crosses tile rows.

* 256^3 spheres at porosity 0.3, FP64 (the step that bench.py times): within
  1e-12 relative, element by element.
* 448^3 vessel tree: FP64 within 1e-12; FP32 offsets within 1e-5 of the
  node's largest offset (FP32 arithmetic and the rounding of the stored
  state are ~1e-7 of it); FP16 offsets (scale 2^22) within 2^-8 of the
  node's largest offset (their own rounding, 2^-11 of each stored offset,
  summed over the 19 values that enter a node's moments, through two
  steps).
* the 512-sample batch, FP32 offsets, persistent kernel with graph replay and
  per-sample forces: sampled nodes of six samples, FP32 bar.
* a 640^3 box at porosity 0.95, FP64: 4.7e9 PDF entries per copy, past the
  2^32 that the scalar-mask kernel addresses, so the solver runs the generic
  kernel with 64-bit entries (asking for the scalar-mask kernel is refused).
Each bar is shown to be tight: the oracle's run with a 5% larger relaxation
time, and for FP64 and FP32 also its run without the body force, fall outside
it.  A CPU test checks the crop construction against a whole-domain oracle
run.
"""
import sys

import numpy as np
import pytest

from oracle import dense
from paper_1703_08015_amd import inputs, lbm

Q = 19
K = 2  # steps; crops of edge 2K + 1
E = 2 * K + 1


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module", autouse=True)
def _built():
    dense.build()


def _sample_nodes(mask, n, seed):
    """n random fluid nodes plus fluid nodes on each of the six domain faces; (N, 3) as z, y, x."""
    rng = np.random.default_rng(seed)
    fl = np.flatnonzero(~mask)
    pick = [np.stack(np.unravel_index(rng.choice(fl, size=min(n, fl.size), replace=False), mask.shape), 1)]
    for ax in range(3):
        for side in (0, mask.shape[ax] - 1):
            face = np.take(~mask, side, axis=ax)
            idx = np.flatnonzero(face)
            if idx.size == 0:
                continue
            sel = rng.choice(idx, size=min(64, idx.size), replace=False)
            a, b = np.unravel_index(sel, face.shape)
            pick.append(np.insert(np.stack([a, b], 1), ax, side, axis=1))
    return np.unique(np.concatenate(pick), axis=0)


def _crop_index(nodes, shape):
    """Flat indices (E^3, N) of each node's E^3 neighbourhood, wrapped periodically."""
    nz, ny, nx = shape
    d = np.arange(-K, K + 1)
    dz, dy, dx = [v.reshape(-1, 1) for v in np.meshgrid(d, d, d, indexing="ij")]
    z = (nodes[None, :, 0] + dz) % nz
    y = (nodes[None, :, 1] + dy) % ny
    x = (nodes[None, :, 2] + dx) % nx
    return (z * ny + y) * nx + x


def _lay_out(vals, n):
    """(C, E^3 * N) gathered values to crops side by side along x: (C, E, E, E * N)."""
    c = vals.shape[0]
    return vals.reshape(c, E, E, E, n).transpose(0, 1, 2, 4, 3).reshape(c, E, E, E * n)


def _oracle(mask, rho, u, idx, tau, g):
    """The oracle's state after K steps from f_eq(rho, u), at the centres of the crops: (Q, N)."""
    n = idx.shape[1]
    flat = idx.reshape(-1)
    mc = _lay_out(mask.reshape(1, -1)[:, flat], n)[0]
    rc = _lay_out(rho.reshape(1, -1)[:, flat], n)[0]
    uc = _lay_out(u.reshape(3, -1)[:, flat], n)
    f = dense.init(Q, mc, rho=rc, u=uc)
    out = dense.step(Q, mc, f, tau, g, K, periodic=0, nthreads=8)
    return out[:, K, K, K::E]


def _bar(want, storage):
    """Allowed |GPU - oracle| per entry after K steps of the given storage form."""
    if storage == "f64":
        return 1e-12 * np.abs(want)
    node_max = np.max(np.abs(want - dense.lattice(Q)[1][:, None]), axis=0, keepdims=True)  # offsets, rho0 = 1
    return (1e-5 if storage == "f32" else 2.0 ** -8) * node_max + 2.0 ** -46


def _check(got, mask, rho, u, idx, tau, g, storage, what):
    want = _oracle(mask, rho, u, idx, tau, g)
    bar = _bar(want, storage)
    err = np.abs(got - want)
    _log(what, storage, "nodes", got.shape[1], "max error / bar", float(np.max(err / bar)))
    assert np.all(err <= bar), what
    # the bar is tight: a 5% larger relaxation time falls outside it, and in FP64 and FP32 so does a run
    # without the body force
    assert np.any(np.abs(got - _oracle(mask, rho, u, idx, 1.05 * tau, g)) > bar), what
    if storage != "f16":
        assert np.any(np.abs(got - _oracle(mask, rho, u, idx, tau, (0.0, 0.0, 0.0))) > bar), what


def _gpu_centres(torch, f_flat, idx):
    """The GPU state at the crop centres: f_flat is the (Q, nodes) export of one sample."""
    centre = idx[(E ** 3) // 2]
    return f_flat[:, torch.from_numpy(centre).to(f_flat.device)].cpu().numpy()


def _run_single(torch, mask, storage, tau, g, seed, drho, umax, **kw):
    tiles = lbm.Tiles(mask, (4, 4, 4), (1, 1, 1))
    s = lbm.Solver(tiles, lattice=Q, storage=storage, tau=tau, g=g, f16_scale_log2=22, **kw)
    rho, u = inputs.random_macro(mask, seed=seed, drho=drho, umax=umax)
    s.init(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    s.step(K)
    f = s.pdfs_export()
    torch.cuda.synchronize()
    del s
    return f.reshape(Q, -1), rho, u


def test_crops_reproduce_the_whole_domain_run():
    """CPU: K oracle steps on every node's crop equal K whole-domain periodic oracle steps."""
    mask = inputs.spheres_3d((12, 10, 9), 0.6, rmin=2, rmax=3, seed=21)[0]
    rho, u = inputs.random_macro(mask, seed=22)
    g, tau = (2e-5, -1e-5, 3e-6), 0.7
    whole = dense.step(Q, mask, dense.init(Q, mask, rho=rho, u=u), tau, g, K, periodic=7)
    nodes = np.argwhere(~mask)
    got = _oracle(mask, rho, u, _crop_index(nodes, mask.shape), tau, g)
    assert np.array_equal(got, whole[:, nodes[:, 0], nodes[:, 1], nodes[:, 2]])
    s = _sample_nodes(mask, 10, seed=23)
    assert all(np.any(s[:, a] == 0) and np.any(s[:, a] == mask.shape[a] - 1) for a in range(3))


@pytest.mark.gpu
def test_spheres_256_fp64(torch):
    mask, _ = inputs.spheres_3d(256, 0.3, 4.0, 12.0, seed=0)
    g, tau = (1e-6, 0.0, 0.0), 0.7
    _log("fullsize spheres 256^3 fp64")
    f, rho, u = _run_single(torch, mask, "f64", tau, g, seed=11, drho=0.01, umax=0.02, tiles_per_block=0,
                            tile_order="morton", step_kernel="auto", store_policy="auto")
    idx = _crop_index(_sample_nodes(mask, 20000, seed=12), mask.shape)
    _check(_gpu_centres(torch, f, idx), mask, rho, u, idx, tau, g, "f64", "spheres 256^3")


@pytest.fixture(scope="module")
def vessel():
    return inputs.vessel_tree(448, 0.08, seed=0)[0]


@pytest.mark.gpu
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_vessel_448(torch, vessel, storage):
    mask = vessel
    g, tau = (1e-5, 0.0, 0.0), 0.7
    _log("fullsize vessel 448^3", storage)
    f, rho, u = _run_single(torch, mask, storage, tau, g, seed=13, drho=2e-3, umax=4e-3)
    idx = _crop_index(_sample_nodes(mask, 20000, seed=14), mask.shape)
    _check(_gpu_centres(torch, f, idx), mask, rho, u, idx, tau, g, storage, "vessel 448^3")


@pytest.mark.gpu
def test_batch_512_persistent_graph(torch):
    specs = inputs.batch_specs(512, seed=1000)
    masks = [inputs.porous_cube(sp)[0] for sp in specs]
    _log("fullsize batch of 512, nodes", sum(m.size for m in masks))
    tiles = lbm.Tiles.concat([lbm.Tiles(m) for m in masks])
    tau = 0.8
    s = lbm.Solver(tiles, lattice=Q, storage="f32", tau=tau, persistent=1, graph_steps=K, f16_scale_log2=22)
    s.set_sample_force(np.array([sp["g"] for sp in specs]))
    fields = [inputs.random_macro(m, seed=2000 + k, drho=2e-3, umax=4e-3) for k, m in enumerate(masks)]
    rho_all = np.concatenate([r.ravel() for r, _ in fields])
    u_all = np.concatenate([v.reshape(-1) for _, v in fields])  # per sample [3][nodes]
    s.init(torch.from_numpy(rho_all).cuda(), torch.from_numpy(u_all).cuda())
    del rho_all, u_all
    s.step(K)  # one replay of the captured K-step graph
    f = s.pdfs_export()
    torch.cuda.synchronize()
    offs = np.concatenate([[0], np.cumsum([Q * m.size for m in masks])])
    rng = np.random.default_rng(15)
    for k in sorted(rng.choice(len(masks), size=6, replace=False)):
        m = masks[k]
        fk = f[offs[k]:offs[k] + Q * m.size].reshape(Q, m.size)
        idx = _crop_index(_sample_nodes(m, 3000, seed=16 + int(k)), m.shape)
        rho, u = fields[k]
        _check(_gpu_centres(torch, fk, idx), m, rho, u, idx, tau, specs[k]["g"], "f32",
               "batch sample %d (edge %d)" % (k, specs[k]["edge"]))


@pytest.mark.gpu
def test_past_2_to_the_32_entries_fp64(torch):
    mask, _ = inputs.spheres_3d(640, 0.95, 4.0, 12.0, seed=3)
    tiles = lbm.Tiles(mask, (4, 4, 4), (1, 1, 1))
    assert tiles.info["n_fluid"] * Q > 2 ** 32
    g, tau = (1e-5, 0.0, 0.0), 0.7
    _log("fullsize 640^3 past 2^32 entries, fluid nodes", tiles.info["n_fluid"])
    with pytest.raises(lbm.LbmError) as e:
        lbm.Solver(tiles, lattice=Q, storage="f64", tau=tau, g=g, step_kernel="scalar")
    assert e.value.code == lbm.LBM_ERR_UNSUPPORTED
    torch.cuda.empty_cache()
    f, rho, u = _run_single(torch, mask, "f64", tau, g, seed=17, drho=2e-3, umax=4e-3)
    idx = _crop_index(_sample_nodes(mask, 20000, seed=18), mask.shape)
    _check(_gpu_centres(torch, f, idx), mask, rho, u, idx, tau, g, "f64", "640^3")
