"""GPU parity of the incompressible BGK model (Eqs. 4 and 6) against the CPU
oracle, through the C ABI.

The states are built around a reference density of 1.3, where the two fluid
models differ at first order, so a kernel that ignored the model switch
would fail every bar here (checked explicitly against the quasi-compressible
oracle).  Bars: FP64 PDFs within 1e-12 relative after 1000 steps on both
step kernels, both lattices and both 3D tile shapes; bit-exact batches,
persistent grids and graph replays against single runs; FP32/FP16 offsets
against the FP64 oracle.
"""
import math
import sys

import numpy as np
import pytest

from oracle import dense
from paper_1703_08015_amd import inputs, lbm

pytestmark = pytest.mark.gpu

INC = dense.INCOMPRESSIBLE
RHO0 = 1.3


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _macro(mask, seed, q):
    rho, u = inputs.random_macro(mask, seed=seed)
    rho = rho + (RHO0 - 1.0)
    if q == 9:
        u[2] = 0.0
    return rho, u


def _run(torch, mask, q, tau, g, steps, per, rho=None, u=None, tile=None, kernel="auto", storage="f64",
         f16_scale_log2=20, tpb=0):
    tile = tile or ((16, 16, 1) if q == 9 else (4, 4, 4))
    s = lbm.Solver(lbm.Tiles(mask, tile, per), lattice=q, storage=storage, tau=tau, g=g, rho0=RHO0,
                   tiles_per_block=tpb, step_kernel=kernel, f16_scale_log2=f16_scale_log2, model="incompressible")
    s.init(None if rho is None else torch.from_numpy(rho).cuda(), None if u is None else torch.from_numpy(u).cuda())
    s.step(steps)
    f = s.pdfs_export().cpu().numpy()
    r, v = s.moments()
    torch.cuda.synchronize()
    return f, r.cpu().numpy(), v.cpu().numpy(), s


CASES = [
    # (name, q, tile, kernel)
    ("d2q9_channel", 9, (16, 16, 1), "generic"),
    ("d3q19_scalar", 19, (4, 4, 4), "scalar"),
    ("d3q19_generic", 19, (4, 4, 4), "generic"),
    ("d3q19_tall_tiles", 19, (4, 4, 8), "generic"),
]


def _geometry(name, q):
    if q == 9:
        return inputs.channel_2d(48, 37, porosity=0.7, seed=31)[0], (1, 0, 0), (2e-5, -1e-5, 0.0)
    if name == "d3q19_tall_tiles":
        return inputs.spheres_3d((16, 12, 24), 0.45, rmin=2, rmax=5, seed=32)[0], (1, 1, 1), (1e-5, 0.0, -3e-6)
    return (inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=33, periodic=(1, 0, 0))[0], (1, 0, 0),
            (2e-5, -1e-5, 3e-6))


@pytest.mark.parametrize("name,q,tile,kernel", CASES)
def test_fp64_1000_steps(torch, name, q, tile, kernel):
    mask, per, g = _geometry(name, q)
    rho, u = _macro(mask, 34, q)
    _log("incompressible fp64", name, mask.shape, tile, kernel)
    f, r, v, _ = _run(torch, mask, q, 0.7, g, 1000, per, rho=rho, u=u, tile=tile, kernel=kernel)
    f0 = dense.init(q, mask, rho=rho, u=u, model=INC)
    want = dense.step(q, mask, f0, 0.7, g, 1000, periodic=per, nthreads=8, model=INC)
    fl = ~mask
    assert np.max(np.abs(f - want)[:, fl] / np.abs(want)[:, fl]) <= 1e-12
    rw, uw = dense.moments(q, mask, want, g, model=INC)
    assert np.max(np.abs(r - rw)) <= 1e-13
    assert np.max(np.abs(v - uw)) <= 1e-9 * np.max(np.abs(uw))
    # the quasi-compressible model gives a different state from the same start
    other = dense.step(q, mask, dense.init(q, mask, rho=rho, u=u), 0.7, g, 1000, periodic=per, nthreads=8)
    assert np.max(np.abs(f - other)[:, fl]) > 1e-6


@pytest.mark.parametrize("q", [9, 19])
def test_init_and_moments(torch, q):
    mask, per, g = _geometry("d2q9_channel" if q == 9 else "d3q19_scalar", q)
    rho, u = _macro(mask, 35, q)
    f, r, v, _ = _run(torch, mask, q, 0.9, g, 0, per, rho=rho, u=u)
    want = dense.init(q, mask, rho=rho, u=u, model=INC)
    assert np.max(np.abs(f - want)) <= 4e-16
    rw, uw = dense.moments(q, mask, want, g, model=INC)
    assert np.max(np.abs(r - rw)) <= 1e-15 and np.max(np.abs(v - uw)) <= 1e-15
    assert np.all(f[:, mask] == 0) and np.all(r[mask] == 0) and np.all(v[:, mask] == 0)


def test_reduce_and_residual(torch):
    """Mass, the momentum of the incompressible model (sum of u) and the
    residual, against math.fsum of the oracle's fields; the momentum grows by
    N g per step in a fully periodic box."""
    mask = np.zeros((8, 12, 16), bool)
    g = (1e-5, 0.0, -2e-6)
    rho, u = _macro(mask, 36, 19)
    s = lbm.Solver(lbm.Tiles(mask), lattice=19, tau=0.75, g=g, rho0=RHO0, model="incompressible")
    s.init(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    tot0 = s.reduce()[0]
    s.step(10)
    r1, u1 = [x.cpu().numpy() for x in s.moments()]
    tot = s.reduce()[0]
    assert math.isclose(tot[0], math.fsum(r1.ravel()), rel_tol=1e-13)
    assert math.isclose(tot[0], tot0[0], rel_tol=1e-13)
    for k in range(3):
        assert math.isclose(tot[1 + k], math.fsum(u1[k].ravel()), rel_tol=1e-11, abs_tol=1e-15)
        assert math.isclose(tot[1 + k], tot0[1 + k] + 10 * mask.size * g[k], rel_tol=1e-11, abs_tol=1e-13)
    ri, ui = dense.moments(19, mask, dense.init(19, mask, rho=rho, u=u, model=INC), g, model=INC)
    want = math.sqrt(math.fsum(((u1 - ui) ** 2).ravel()) / math.fsum((u1 ** 2).ravel()))
    assert math.isclose(s.residual()[0], want, rel_tol=1e-12)


@pytest.mark.parametrize("kernel", ["generic", "scalar"])
@pytest.mark.parametrize("storage,tol", [("f32", 2e-5), ("f16", 2e-2)])
def test_offset_storage_error_vs_fp64(torch, storage, tol, kernel):
    """FP32 / FP16 offsets f_i - w_i rho0 with FP32 arithmetic: velocity error
    against the FP64 oracle after 1000 steps from rest at rho0 = 1.3."""
    mask = inputs.spheres_3d(32, 0.3, seed=8)[0]
    g = (1e-6, 0.0, 0.0)
    _, _, v, _ = _run(torch, mask, 19, 0.7, g, 1000, (1, 1, 1), kernel=kernel, storage=storage, f16_scale_log2=22)
    want = dense.step(19, mask, dense.init(19, mask, rho0=RHO0, model=INC), 0.7, g, 1000, periodic=7, nthreads=8,
                      model=INC)
    _, uw = dense.moments(19, mask, want, g, model=INC)
    fl = ~mask
    err = np.linalg.norm((v - uw)[:, fl]) / np.linalg.norm(uw[:, fl])
    _log("incompressible offsets", storage, kernel, "velocity rel-L2 error after 1000 steps:", err)
    assert err <= tol


@pytest.mark.parametrize("tpb", [1, 2, 8])
def test_launch_shapes_agree(torch, tpb):
    """Every workgroup size of the scalar-mask step gives the same bits."""
    mask, per, g = _geometry("d3q19_scalar", 19)
    rho, u = _macro(mask, 37, 19)
    a = _run(torch, mask, 19, 0.8, g, 20, per, rho=rho, u=u, tpb=4)[0]
    b = _run(torch, mask, 19, 0.8, g, 20, per, rho=rho, u=u, tpb=tpb)[0]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("persistent,graph_steps", [(0, 0), (1, 0), (1, 5)])
def test_batch_equals_each_sample_alone(torch, persistent, graph_steps):
    """A concatenated batch (per-sample g), also on the persistent grid with
    graph replay, reproduces each sample's single run bit for bit."""
    specs = [(16, 0.5, (1e-5, 2e-6, 0.0), 41), (24, 0.35, (0.0, -3e-6, 4e-6), 42), (12, 0.7, (-2e-6, 0.0, 1e-6), 43)]
    masks = [inputs.spheres_3d(e, p, rmin=2, rmax=5, seed=sd)[0] for e, p, _, sd in specs]
    singles = []
    for m, (_, _, g, _) in zip(masks, specs):
        s = lbm.Solver(lbm.Tiles(m), lattice=19, tau=0.8, g=g, rho0=RHO0, model="incompressible")
        s.init()
        s.step(25)
        singles.append(s.pdfs_export().cpu().numpy().ravel())
    tb = lbm.Tiles.concat([lbm.Tiles(m) for m in masks])
    s = lbm.Solver(tb, lattice=19, tau=0.8, rho0=RHO0, model="incompressible", persistent=persistent,
                   graph_steps=graph_steps)
    s.set_sample_force(np.array([sp[2] for sp in specs]))
    s.init()
    for _ in range(5):
        s.step(5)
        torch.cuda.synchronize()
    f = s.pdfs_export().cpu().numpy()
    o = 0
    for m, want in zip(masks, singles):
        n = 19 * m.size
        assert np.array_equal(f[o:o + n], want)
        o += n
