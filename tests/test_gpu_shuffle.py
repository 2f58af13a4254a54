"""The shuffle form of the D3Q19 step (step_kernel="shuffle"): coalesced own
loads, in-tile sources taken from other lanes (DPP row shifts, ds_bpermute),
neighbour sources gathered.  It performs the same arithmetic on the same
values as the scalar-mask gather, so every result must be bit-identical to
it; pure streaming must equal the oracle exactly and FP64 PDFs stay within
1e-12 of the oracle after 1000 steps."""
import math
import sys

import numpy as np
import pytest

from oracle import dense
from paper_1703_08015_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _geoms():
    yield "spheres_periodic", inputs.spheres_3d(24, 0.4, rmin=2, rmax=5, seed=1)[0], (1, 1, 1)
    yield "ragged", inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=2, periodic=(1, 0, 0))[0], (1, 0, 0)
    yield "dense", np.zeros((12, 8, 16), bool), (1, 1, 1)


def _run(torch, mask, per, steps, f0=None, rho=None, u=None, **kw):
    s = lbm.Solver(lbm.Tiles(mask, (4, 4, 4), per), lattice=19, **kw)
    if f0 is not None:
        s.pdfs_import(torch.from_numpy(f0).cuda())
    else:
        s.init(None if rho is None else torch.from_numpy(rho).cuda(), None if u is None else torch.from_numpy(u).cuda())
    s.step(steps)
    f = s.pdfs_export().cpu().numpy()
    torch.cuda.synchronize()
    return f


@pytest.mark.parametrize("tpb", [1, 2, 4, 8])
def test_permutation_bitexact(torch, tpb):
    """tau = +inf, g = 0: only streaming and bounce-back, GPU == oracle exactly."""
    for name, mask, per in _geoms():
        _log("shuffle permutation", tpb, name, mask.shape)
        f0 = inputs.random_pdfs(19, mask, seed=31)
        f = _run(torch, mask, per, 5, f0=f0, tau=math.inf, g=(0, 0, 0), step_kernel="shuffle", tiles_per_block=tpb)
        assert np.array_equal(f, dense.step(19, mask, f0, math.inf, [0, 0, 0], 5, periodic=per)), name


@pytest.mark.parametrize("storage,scale", [("f32", 0), ("f16", 12)])
def test_offset_permutation_bitexact(torch, storage, scale):
    mask = inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=2, periodic=(1, 0, 0))[0]
    _, w, _ = dense.lattice(19)
    rng = np.random.default_rng(17)
    off = rng.uniform(-1e-3, 1e-3, size=(19,) + mask.shape)
    if storage == "f32":
        off = off.astype(np.float32).astype(np.float64)
    else:
        off = (off * 2.0 ** scale).astype(np.float16).astype(np.float64) / 2.0 ** scale
    f0 = w[:, None, None, None] + off
    f0[:, mask] = 0.0
    f = _run(torch, mask, (1, 0, 0), 6, f0=f0, tau=math.inf, g=(0, 0, 0), storage=storage, f16_scale_log2=scale,
             step_kernel="shuffle")
    assert np.array_equal(f, dense.step(19, mask, f0, math.inf, [0, 0, 0], 6, periodic=(1, 0, 0)))


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("model", ["quasi-compressible", "incompressible"])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_equals_gather_bitwise(torch, storage, model, collision):
    """Random state, force along all axes: the shuffle form gives the gather
    form's bits after 40 steps (every storage form, model and collision)."""
    for name, mask, per in _geoms():
        rho, u = inputs.random_macro(mask, seed=32)
        kw = dict(tau=0.7, g=(2e-5, -1e-5, 3e-6), storage=storage, f16_scale_log2=16, model=model,
                  collision=collision, rho0=1.3 if model == "incompressible" else 1.0)
        a = _run(torch, mask, per, 40, rho=rho, u=u, step_kernel="scalar", **kw)
        b = _run(torch, mask, per, 40, rho=rho, u=u, step_kernel="shuffle", **kw)
        assert np.array_equal(a, b), (name, storage, model, collision)


@pytest.mark.parametrize("persistent,graph_steps", [(0, 0), (1, 0), (1, 7)])
def test_batch_launch_modes_equal_gather(torch, persistent, graph_steps):
    """A batch with per-sample forces and a frozen sample: direct, list and
    persistent launches with graph replay give the gather form's bits."""
    masks = [inputs.spheres_3d(n, 0.5, rmin=2, rmax=4, seed=40 + n)[0] for n in (16, 20, 12)]
    forces = np.array([[1e-5, 0, 0], [0, -2e-6, 3e-6], [1e-6, 1e-6, 1e-6]])
    out = {}
    for kernel in ("scalar", "shuffle"):
        t = lbm.Tiles.concat([lbm.Tiles(m) for m in masks])
        s = lbm.Solver(t, lattice=19, tau=0.8, storage="f32", persistent=persistent, graph_steps=graph_steps,
                       step_kernel=kernel)
        s.set_sample_force(forces)
        s.init()
        s.step(10)
        s.set_active([1, 0, 1])
        s.step(11)
        out[kernel] = s.pdfs_export().cpu().numpy()
    assert np.array_equal(out["scalar"], out["shuffle"])


def test_fp64_1000_steps_vs_oracle(torch):
    """FP64 PDFs within 1e-12 relative of the oracle after 1000 steps."""
    mask = inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=9, periodic=(1, 0, 0))[0]
    g = (2e-5, -1e-5, 3e-6)
    rho, u = inputs.random_macro(mask, seed=10)
    f = _run(torch, mask, (1, 0, 0), 1000, rho=rho, u=u, tau=0.7, g=g, step_kernel="shuffle")
    want = dense.step(19, mask, dense.init(19, mask, rho=rho, u=u), 0.7, g, 1000, periodic=(1, 0, 0), nthreads=8)
    fl = ~mask
    assert np.max(np.abs(f - want)[:, fl] / np.abs(want)[:, fl]) <= 1e-12


def test_single_copy_is_refused(torch):
    mask = inputs.spheres_3d(16, 0.5, rmin=2, rmax=4, seed=1)[0]
    with pytest.raises(lbm.LbmError) as e:
        lbm.Solver(lbm.Tiles(mask), lattice=19, tau=0.8, step_kernel="shuffle", pattern="single-copy")
    assert e.value.code == lbm.LBM_ERR_UNSUPPORTED
