"""Parity at the full workload sizes, in the launch configuration that bench.py
times, on sampled outputs.

At these sizes the dense oracle cannot step the whole domain in a test, but
it can compute any single node's update: one step of a node depends only on
the post-collision state of its 3x3x3 neighbourhood (Eq. 1 pulls from
x - c_i, Eq. 2 collides locally).  So each case runs the GPU solver, exports
the state f_n, steps once more on the GPU and exports f_{n+1}; for every
sampled fluid node the oracle steps a 3x3x3 crop of f_n (periodic wrap, the
crops laid side by side along x in one non-periodic domain, so that a crop's
centre reads only its own crop) and the crop's centre is compared with the
GPU's f_{n+1} there.  The samples include nodes on the domain faces, where
the periodic wrap crosses tile rows.

* 256^3 spheres at porosity 0.3, FP64, from a random macroscopic state: within
  1e-12 relative, element by element.
* 448^3 vessel tree, 300 steps from rest, FP64 within 1e-12; FP32 offsets within
  1e-5 of the node's largest offset (FP32 arithmetic and rounding are ~1e-7 of
  it, a dropped force term ~1e-2); FP16 offsets (scale 2^22) within their own
  rounding, 2^-10 of the value, plus the same FP32 term.
* the 512-sample batch, FP32 offsets, persistent kernel with graph replay and
  per-sample forces, 200 steps from rest: sampled nodes of six samples, FP32 bar.
Each bar is also shown to be tight: the oracle's step without the body force
lies outside it.  A CPU test checks the crop construction itself against a
whole-domain oracle step.
"""
import sys

import numpy as np
import pytest

from oracle import dense
from paper_1703_08015_amd import inputs, lbm

Q = 19


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


def _as_torch_cpu(f):
    import torch
    return torch.from_numpy(np.ascontiguousarray(f))


_D = np.array([(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])


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
            coords = np.insert(np.stack([a, b], 1), ax, side, axis=1)
            pick.append(coords)
    return np.unique(np.concatenate(pick), axis=0)


def _neighbour_index(nodes, shape):
    """Flat indices (27, N) of each node's 3x3x3 neighbourhood, wrapped periodically."""
    nz, ny, nx = shape
    z = (nodes[None, :, 0] + _D[:, None, 0]) % nz
    y = (nodes[None, :, 1] + _D[:, None, 1]) % ny
    x = (nodes[None, :, 2] + _D[:, None, 2]) % nx
    return (z * ny + y) * nx + x


def _crops(f_flat, mask, idx):
    """Crops laid side by side along x: f (q, 3, 3, 3N) and mask (3, 3, 3N); f_flat is a (q, nodes) tensor."""
    import torch
    n = idx.shape[1]
    ti = torch.from_numpy(idx.reshape(-1)).to(f_flat.device)
    fc = f_flat[:, ti].reshape(Q, 3, 3, 3, n).permute(0, 1, 2, 4, 3).reshape(Q, 3, 3, 3 * n)
    mc = mask.reshape(-1)[idx.reshape(-1)].reshape(3, 3, 3, n).transpose(0, 1, 3, 2).reshape(3, 3, 3 * n)
    return fc.cpu().numpy(), mc


def _oracle_centres(fc, mc, tau, g):
    out = dense.step(Q, mc, fc, tau, g, 1, periodic=0, nthreads=8)
    return out[:, 1, 1, 1::3]


def _one_step_pair(torch, s, shape):
    """(f_n, f_{n+1}) as (q, nodes) tensors, exported around one more GPU step."""
    fa = s.pdfs_export()
    s.step(1)
    fb = s.pdfs_export()
    torch.cuda.synchronize()
    n = int(np.prod(shape))
    return fa.reshape(Q, n), fb.reshape(Q, n)


def _bar(want, storage, scale_log2=22):
    """Allowed |GPU - oracle| per entry for one step of the given storage form."""
    if storage == "f64":
        return 1e-12 * np.abs(want)
    dw = want - dense.lattice(Q)[1][:, None]  # offsets from the rest state, rho0 = 1
    bar = 1e-5 * np.max(np.abs(dw), axis=0, keepdims=True)
    if storage == "f16":
        bar = bar + 2.0 ** -10 * np.abs(dw) + 2.0 ** -(scale_log2 + 24)
    return bar


def _check(got, fc, mc, tau, g, storage, what):
    want = _oracle_centres(fc, mc, tau, g)
    bar = _bar(want, storage)
    err = np.abs(got - want)
    _log(what, storage, "nodes", got.shape[1], "max error / bar", np.max(err / bar))
    assert np.all(err <= bar)
    # the bar is tight enough to see the body force of a single step
    no_force = _oracle_centres(fc, mc, tau, (0.0, 0.0, 0.0))
    assert np.any(np.abs(got - no_force) > bar)


def test_crops_reproduce_the_whole_domain_step():
    """CPU: one oracle step of every node's crop equals one whole-domain periodic oracle step."""
    mask = inputs.spheres_3d((12, 10, 9), 0.6, rmin=2, rmax=3, seed=21)[0]
    f = inputs.random_pdfs(Q, mask, seed=22)
    g, tau = (2e-5, -1e-5, 3e-6), 0.7
    whole = dense.step(Q, mask, f, tau, g, 1, periodic=7)
    nodes = np.argwhere(~mask)
    idx = _neighbour_index(nodes, mask.shape)
    fc, mc = _crops(_as_torch_cpu(f.reshape(Q, -1)), mask, idx)
    got = _oracle_centres(fc, mc, tau, g)
    assert np.array_equal(got, whole[:, nodes[:, 0], nodes[:, 1], nodes[:, 2]])
    # and the face samples lie on the faces
    s = _sample_nodes(mask, 10, seed=23)
    assert all(np.any(s[:, a] == 0) and np.any(s[:, a] == mask.shape[a] - 1) for a in range(3))


@pytest.mark.gpu
def test_spheres_256_fp64_random_state(torch):
    mask, _ = inputs.spheres_3d(256, 0.3, 4.0, 12.0, seed=0)
    g, tau = (1e-6, 0.0, 0.0), 0.7
    _log("fullsize spheres 256^3 fp64")
    tiles = lbm.Tiles(mask, (4, 4, 4), (1, 1, 1))
    s = lbm.Solver(tiles, lattice=Q, storage="f64", tau=tau, g=g, tiles_per_block=0, f16_scale_log2=22,
                   tile_order="morton", step_kernel="auto", store_policy="auto")
    rho, u = inputs.random_macro(mask, seed=11)
    s.init(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    del rho, u
    s.step(20)
    fa, fb = _one_step_pair(torch, s, mask.shape)
    nodes = _sample_nodes(mask, 20000, seed=12)
    idx = _neighbour_index(nodes, mask.shape)
    fc, mc = _crops(fa, mask, idx)
    got = fb[:, torch.from_numpy(idx[13]).cuda()].cpu().numpy()  # offset (0, 0, 0) is entry 13
    _check(got, fc, mc, tau, g, "f64", "spheres 256^3")


@pytest.fixture(scope="module")
def vessel():
    mask, _ = inputs.vessel_tree(448, 0.08, seed=0)
    return mask, lbm.Tiles(mask, (4, 4, 4), (1, 1, 1))


@pytest.mark.gpu
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_vessel_448_from_rest(torch, vessel, storage):
    mask, tiles = vessel
    g, tau = (1e-6, 0.0, 0.0), 0.7
    _log("fullsize vessel 448^3", storage)
    s = lbm.Solver(tiles, lattice=Q, storage=storage, tau=tau, g=g, f16_scale_log2=22)
    s.init()
    s.step(300)
    fa, fb = _one_step_pair(torch, s, mask.shape)
    nodes = _sample_nodes(mask, 20000, seed=13)
    idx = _neighbour_index(nodes, mask.shape)
    fc, mc = _crops(fa, mask, idx)
    got = fb[:, torch.from_numpy(idx[13]).cuda()].cpu().numpy()
    del fa, fb
    _check(got, fc, mc, tau, g, storage, "vessel 448^3")


@pytest.mark.gpu
def test_batch_512_persistent_graph(torch):
    specs = inputs.batch_specs(512, seed=1000)
    masks = [inputs.porous_cube(sp)[0] for sp in specs]
    _log("fullsize batch of 512, nodes", sum(m.size for m in masks))
    tiles = lbm.Tiles.concat([lbm.Tiles(m) for m in masks])
    tau = 0.8
    s = lbm.Solver(tiles, lattice=Q, storage="f32", tau=tau, persistent=1, graph_steps=100, f16_scale_log2=22)
    s.set_sample_force(np.array([sp["g"] for sp in specs]))
    s.init()
    s.step(200)
    fa = s.pdfs_export()
    s.step(1)
    fb = s.pdfs_export()
    torch.cuda.synchronize()
    offs = np.concatenate([[0], np.cumsum([Q * m.size for m in masks])])
    rng = np.random.default_rng(14)
    for k in sorted(rng.choice(len(masks), size=6, replace=False)):
        m = masks[k]
        n = m.size
        a = fa[offs[k]:offs[k] + Q * n].reshape(Q, n)
        b = fb[offs[k]:offs[k] + Q * n].reshape(Q, n)
        nodes = _sample_nodes(m, 3000, seed=15 + int(k))
        idx = _neighbour_index(nodes, m.shape)
        fc, mc = _crops(a, m, idx)
        got = b[:, torch.from_numpy(idx[13]).cuda()].cpu().numpy()
        _check(got, fc, mc, tau, specs[k]["g"], "f32", "batch sample %d (edge %d)" % (k, specs[k]["edge"]))
