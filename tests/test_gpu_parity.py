"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: bit-exact where no arithmetic happens (pure streaming with tau = +inf
and g = 0, checkpoint export/import, the tiling), FP64 PDFs within 1e-12
relative after 1000 steps (also on a crop of the benchmark geometry), FP64
reductions against math.fsum of the oracle's fields after the same steps.  Shapes span several tiles with ragged (padded) edges.
"""
import math
import os
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


def _tiles(mask, q, tile=None, periodic=(1, 1, 1)):
    if tile is None:
        tile = (16, 16, 1) if q == 9 else (4, 4, 4)
    return lbm.Tiles(mask, tile, periodic)


def _gpu_run(torch, mask, q, tau, g, steps, periodic, f0=None, rho=None, u=None, storage="f64", tile=None,
             tpb=0, f16_scale_log2=20, kernel="auto", order="morton"):
    t = _tiles(mask, q, tile, periodic)
    s = lbm.Solver(t, lattice=q, storage=storage, tau=tau, g=g, tiles_per_block=tpb,
                   f16_scale_log2=f16_scale_log2, step_kernel=kernel, tile_order=order)
    if f0 is not None:
        s.pdfs_import(torch.from_numpy(f0).cuda())
    else:
        s.init(None if rho is None else torch.from_numpy(rho).cuda(), None if u is None else torch.from_numpy(u).cuda())
    s.step(steps)
    f = s.pdfs_export().cpu().numpy()
    r, v = s.moments()
    torch.cuda.synchronize()
    return f, r.cpu().numpy(), v.cpu().numpy(), s


def _geoms(q):
    """(name, mask, periodic) with several tiles and ragged padded edges."""
    if q == 9:
        yield "channel64", inputs.channel_2d(64, 64, seed=0)[0], (1, 0, 0)
        yield "ragged", inputs.channel_2d(48, 37, porosity=0.7, seed=3)[0], (1, 0, 0)
    else:
        yield "spheres_periodic", inputs.spheres_3d(24, 0.4, rmin=2, rmax=5, seed=1)[0], (1, 1, 1)
        yield "ragged", inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=2, periodic=(1, 0, 0))[0], (1, 0, 0)


KERNELS = [(9, "generic", "rowmajor"), (9, "generic", "morton"), (19, "generic", "rowmajor"),
           (19, "generic", "morton"), (19, "scalar", "morton"), (19, "scalar", "rowmajor")]


@pytest.mark.parametrize("q,kernel,order", KERNELS)
def test_permutation_mode_bitexact(torch, q, kernel, order):
    """tau = +inf, g = 0: the step only moves values, so GPU == oracle exactly."""
    for name, mask, per in _geoms(q):
        _log("permutation", q, kernel, order, name, mask.shape)
        f0 = inputs.random_pdfs(q, mask, seed=21)
        f, _, _, _ = _gpu_run(torch, mask, q, math.inf, (0, 0, 0), 7, per, f0=f0, kernel=kernel, order=order)
        want = dense.step(q, mask, f0, math.inf, [0, 0, 0], 7, periodic=per)
        assert np.array_equal(f, want), name


@pytest.mark.parametrize("kernel", ["generic", "scalar"])
@pytest.mark.parametrize("tpb", [1, 2, 8])
def test_permutation_mode_bitexact_launch_shapes(torch, tpb, kernel):
    """Every workgroup size of the D3Q19 step visits every tile exactly once."""
    mask = inputs.spheres_3d((28, 20, 16), 0.5, rmin=2, rmax=5, seed=5)[0]
    f0 = inputs.random_pdfs(19, mask, seed=22)
    f, _, _, _ = _gpu_run(torch, mask, 19, math.inf, (0, 0, 0), 3, (1, 1, 1), f0=f0, tpb=tpb, kernel=kernel)
    assert np.array_equal(f, dense.step(19, mask, f0, math.inf, [0, 0, 0], 3, periodic=7))


def _tall_geoms():
    yield "periodic", inputs.spheres_3d((16, 12, 24), 0.45, rmin=2, rmax=5, seed=6)[0], (1, 1, 1)
    # z = 13 pads the last tile row to z = 16 with solid; walls on y and z
    yield "ragged", inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=2, periodic=(1, 0, 0))[0], (1, 0, 0)


@pytest.mark.parametrize("kernel", ["generic", "scalar"])
@pytest.mark.parametrize("tpb", [1, 4])
def test_permutation_mode_bitexact_tall_tiles(torch, kernel, tpb):
    """4x4x8 tiles: the generic kernel, and the scalar-mask kernel running each
    tile as two 4x4x4 halves (one wavefront each)."""
    for name, mask, per in _tall_geoms():
        _log("tall tiles permutation", kernel, tpb, name, mask.shape)
        f0 = inputs.random_pdfs(19, mask, seed=23)
        f, _, _, _ = _gpu_run(torch, mask, 19, math.inf, (0, 0, 0), 5, per, f0=f0, tile=(4, 4, 8), kernel=kernel,
                              tpb=tpb)
        assert np.array_equal(f, dense.step(19, mask, f0, math.inf, [0, 0, 0], 5, periodic=per)), name


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_tall_tiles_scalar_equals_4x4x4(torch, storage):
    """The scalar-mask kernel does the same arithmetic per node whatever the
    tile shape, so 4x4x8 tiles give the 4x4x4 tiles' bits after 30 steps
    from a random state with a force (all storage forms).  (The generic
    kernel groups the collision's operations differently: it agrees with both
    to rounding, as the oracle tests show.)"""
    for name, mask, per in _tall_geoms():
        rho, u = inputs.random_macro(mask, seed=24)
        kw = dict(rho=rho, u=u, storage=storage, f16_scale_log2=16, kernel="scalar")
        a, _, _, _ = _gpu_run(torch, mask, 19, 0.7, (2e-5, -1e-5, 3e-6), 30, per, tile=(4, 4, 4), **kw)
        b, _, _, _ = _gpu_run(torch, mask, 19, 0.7, (2e-5, -1e-5, 3e-6), 30, per, tile=(4, 4, 8), **kw)
        assert np.array_equal(a, b), (name, storage)


def test_fp64_1000_steps_tall_tiles_scalar(torch):
    """FP64 PDFs within 1e-12 of the oracle after 1000 steps, 4x4x8 tiles on
    the scalar-mask kernel, random state and force."""
    mask = inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=9, periodic=(1, 0, 0))[0]
    g = (2e-5, -1e-5, 3e-6)
    rho, u = inputs.random_macro(mask, seed=10)
    f, _, _, _ = _gpu_run(torch, mask, 19, 0.7, g, 1000, (1, 0, 0), rho=rho, u=u, kernel="scalar", tile=(4, 4, 8))
    want = dense.step(19, mask, dense.init(19, mask, rho=rho, u=u), 0.7, g, 1000, periodic=(1, 0, 0), nthreads=8)
    fl = ~mask
    assert np.max(np.abs(f - want)[:, fl] / np.abs(want)[:, fl]) <= 1e-12


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def test_fp64_1000_steps_channel_2d(torch):
    """D2Q9 64x64 channel with discs, tau 0.8, g = 1e-6 in x, 1000 steps."""
    mask, _ = inputs.channel_2d(64, 64, seed=0)
    g = (1e-6, 0.0, 0.0)
    f, r, u, _ = _gpu_run(torch, mask, 9, 0.8, g, 1000, (1, 0, 0))
    f0 = dense.init(9, mask)
    want = dense.step(9, mask, f0, 0.8, g, 1000, periodic=(1, 0, 0))
    fl = ~mask
    assert np.max(np.abs(f - want)[:, fl] / np.abs(want)[:, fl]) <= 1e-12
    rw, uw = dense.moments(9, mask, want, g)
    assert _rel(u, uw) <= 1e-9 and np.max(np.abs(r - rw)) <= 1e-13


@pytest.mark.parametrize("kernel", ["generic", "scalar"])
@pytest.mark.parametrize("case", ["spheres_periodic", "ragged_random_state"])
def test_fp64_1000_steps_3d(torch, case, kernel):
    """D3Q19 porous crops: from rest with g (tau 0.7), and from a random state."""
    if case == "spheres_periodic":
        mask = inputs.spheres_3d(32, 0.3, seed=8)[0]
        per, rho, u, g = (1, 1, 1), None, None, (1e-6, 0.0, 0.0)
    else:
        mask = inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=9, periodic=(1, 0, 0))[0]
        per, g = (1, 0, 0), (2e-5, -1e-5, 3e-6)
        rho, u = inputs.random_macro(mask, seed=10)
    f, r, v, _ = _gpu_run(torch, mask, 19, 0.7, g, 1000, per, rho=rho, u=u, kernel=kernel)
    f0 = dense.init(19, mask, rho=rho, u=u)
    want = dense.step(19, mask, f0, 0.7, g, 1000, periodic=per, nthreads=8)
    fl = ~mask
    assert np.max(np.abs(f - want)[:, fl] / np.abs(want)[:, fl]) <= 1e-12
    rw, uw = dense.moments(19, mask, want, g)
    assert _rel(v, uw) <= 1e-9


@pytest.mark.parametrize("q", [9, 19])
def test_init_and_moments_match_oracle(torch, q):
    mask = inputs.channel_2d(48, 37, seed=3)[0] if q == 9 else inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5,
                                                                                  seed=2, periodic=(1, 0, 0))[0]
    rho, u = inputs.random_macro(mask, seed=11)
    if q == 9:
        u[2] = 0.0
    g = (3e-6, -2e-6, 0.0 if q == 9 else 1e-6)
    f, r, v, _ = _gpu_run(torch, mask, q, 0.9, g, 0, (1, 0, 0), rho=rho, u=u)
    want = dense.init(q, mask, rho=rho, u=u)
    assert np.max(np.abs(f - want)) <= 4e-16
    rw, uw = dense.moments(q, mask, want, g)
    assert np.max(np.abs(r - rw)) <= 1e-15 and np.max(np.abs(v - uw)) <= 1e-15
    assert np.all(r[mask] == 0) and np.all(v[:, mask] == 0) and np.all(f[:, mask] == 0)


def test_reduce_and_residual(torch):
    mask = inputs.spheres_3d(24, 0.4, rmin=2, rmax=5, seed=12)[0]
    g = (1e-5, 0.0, -2e-6)
    t = _tiles(mask, 19)
    s = lbm.Solver(t, lattice=19, tau=0.75, g=g)
    rho, u = inputs.random_macro(mask, seed=13)
    s.init(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    tot0 = s.reduce()[0]
    s.step(10)
    r1, u1 = [x.cpu().numpy() for x in s.moments()]
    tot = s.reduce()[0]
    assert math.isclose(tot[0], math.fsum(r1.ravel()), rel_tol=1e-13)
    for k in range(3):
        assert math.isclose(tot[1 + k], math.fsum((r1 * u1[k]).ravel()), rel_tol=1e-11, abs_tol=1e-15)
    assert math.isclose(tot[0], tot0[0], rel_tol=1e-13)  # mass is conserved
    # residual against the velocity recorded at init
    res = s.residual()[0]
    ri, ui = dense.moments(19, mask, dense.init(19, mask, rho=rho, u=u), g)
    fl = ~mask
    want = math.sqrt(math.fsum(((u1 - ui)[:, fl] ** 2).ravel()) / math.fsum((u1[:, fl] ** 2).ravel()))
    assert math.isclose(res, want, rel_tol=1e-12)
    s.step(3)
    r2, u2 = [x.cpu().numpy() for x in s.moments()]
    want2 = math.sqrt(math.fsum(((u2 - u1)[:, fl] ** 2).ravel()) / math.fsum((u2[:, fl] ** 2).ravel()))
    assert math.isclose(s.residual()[0], want2, rel_tol=1e-12)
    # fixed-order reductions repeat exactly
    assert np.array_equal(s.reduce(), s.reduce())


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_reduce_and_residual_vs_oracle(torch, storage):
    """lbm_reduce and lbm_residual against math.fsum of the oracle's own
    fields after the same 10 steps (mass and momentum per Eq. 5, residual over
    the non-solid nodes), with nothing taken from the GPU's moments.

    FP64: the states agree to the parity bar, so the sums agree to 1e-13
    (mass) and 1e-11 (momentum).  FP32 offsets: each stored offset rounds to
    2^-24 of its magnitude; over q = 19 values, 10 steps and N_f nodes the
    worst case, all errors of one sign, moves the mass by
    N_f * 10 * 19 * 2^-23 * max|f - w rho0| (a factor 2 for the FP32
    arithmetic), and the momentum by as much; the residual, a ratio of norms
    of velocity differences of about 1e-2, is held to 1e-4 relative."""
    mask = inputs.spheres_3d(24, 0.4, rmin=2, rmax=5, seed=12)[0]
    g = (1e-5, 0.0, -2e-6)
    tau, steps = 0.75, 10
    t = _tiles(mask, 19)
    s = lbm.Solver(t, lattice=19, tau=tau, g=g, storage=storage)
    rho, u = inputs.random_macro(mask, seed=13)
    s.init(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    s.step(steps)
    tot = s.reduce()[0]
    res = s.residual()[0]
    f0 = dense.init(19, mask, rho=rho, u=u)
    f1 = dense.step(19, mask, f0, tau, list(g), steps, periodic=7)
    r0, u0 = dense.moments(19, mask, f0, g)
    r1, u1 = dense.moments(19, mask, f1, g)
    fl = ~mask
    mass = math.fsum(r1[fl])
    mom = [math.fsum((r1 * u1[k])[fl]) for k in range(3)]
    want_res = math.sqrt(math.fsum(((u1 - u0)[:, fl] ** 2).ravel()) / math.fsum((u1[:, fl] ** 2).ravel()))
    if storage == "f64":
        bar_m, bar_p, bar_r = 1e-13 * mass, 1e-11 * max(abs(v) for v in mom), 1e-12
    else:
        _, w, _ = dense.lattice(19)
        dmax = float(np.max(np.abs(f0 - w[:, None, None, None])[:, fl]))
        bar_m = bar_p = int(fl.sum()) * steps * 19 * 2.0 ** -23 * dmax
        bar_r = 1e-4
    _log("reduce vs oracle", storage, "mass", tot[0] - mass, "bar", bar_m,
         "momentum", [tot[1 + k] - mom[k] for k in range(3)], "bar", bar_p, "residual", res, want_res)
    assert abs(tot[0] - mass) <= bar_m
    for k in range(3):
        assert abs(tot[1 + k] - mom[k]) <= bar_p
    assert abs(res - want_res) <= bar_r * want_res


def _sphere256_crop():
    """A 64^3 crop of the 256^3 porosity-0.3 sphere packing (seed 0, radii
    4-12) that the step benchmark runs.  The tests run it periodic along x,
    the force direction, and closed on y and z (positions outside the crop
    count as solid): a crop closed on every axis settles towards a
    hydrostatic state with no flow (mean |u| 1e-8 after 1000 steps, against
    9e-6 with x periodic), where velocity errors measure only cancellation."""
    mask, _ = inputs.spheres_3d(256, 0.3, 4.0, 12.0, seed=0)
    return np.ascontiguousarray(mask[:64, :64, :64])


@pytest.mark.parametrize("kernel", ["generic", "scalar"])
def test_fp64_1000_steps_sphere256_crop(torch, kernel):
    """FP64 PDFs within 1e-12 of the oracle after 1000 steps on a crop of the
    benchmark geometry (tau 0.7, g 1e-6 along x, from rest)."""
    mask = _sphere256_crop()
    g = (1e-6, 0.0, 0.0)
    _log("sphere256 crop fp64", kernel, "porosity", float((~mask).mean()))
    f, _, v, _ = _gpu_run(torch, mask, 19, 0.7, g, 1000, (1, 0, 0), kernel=kernel)
    want = dense.step(19, mask, dense.init(19, mask), 0.7, g, 1000, periodic=(1, 0, 0), nthreads=8)
    fl = ~mask
    err = np.max(np.abs(f - want)[:, fl] / np.abs(want)[:, fl])
    _log("sphere256 crop fp64", kernel, "max rel PDF error", err)
    assert err <= 1e-12
    _, uw = dense.moments(19, mask, want, g)
    assert _rel(v, uw) <= 1e-9


def test_f32_1000_steps_sphere256_crop(torch):
    """FP32 offsets on the same crop: velocity rel-L2 against the FP64 oracle
    within the 2e-5 bar of the offset forms."""
    mask = _sphere256_crop()
    g = (1e-6, 0.0, 0.0)
    _, _, v, _ = _gpu_run(torch, mask, 19, 0.7, g, 1000, (1, 0, 0), storage="f32")
    want = dense.step(19, mask, dense.init(19, mask), 0.7, g, 1000, periodic=(1, 0, 0), nthreads=8)
    _, uw = dense.moments(19, mask, want, g)
    fl = ~mask
    err = np.linalg.norm((v - uw)[:, fl]) / np.linalg.norm(uw[:, fl])
    _log("sphere256 crop f32 velocity rel-L2", err)
    assert err <= 2e-5


def test_checkpoint_resume_bitexact(torch):
    mask = inputs.spheres_3d(24, 0.35, rmin=2, rmax=6, seed=14)[0]
    g = (1e-6, 0, 0)
    t = _tiles(mask, 19)
    a = lbm.Solver(t, lattice=19, tau=0.7, g=g)
    a.init()
    a.step(40)
    fa = a.pdfs_export()
    b = lbm.Solver(t, lattice=19, tau=0.7, g=g)
    b.init()
    b.step(20)
    ck = b.pdfs_export().clone()
    c = lbm.Solver(t, lattice=19, tau=0.7, g=g)
    c.pdfs_import(ck)
    c.step(20)
    assert torch.equal(fa, c.pdfs_export())
    assert a.step_count == 40 and c.step_count == 20


def test_degenerate_geometries(torch):
    # all solid: no tiles, every call succeeds and fields are zero
    mask = np.ones((8, 8, 8), bool)
    f, r, v, s = _gpu_run(torch, mask, 19, 0.7, (1e-6, 0, 0), 3, (1, 1, 1))
    assert s.tiles.info["n_ftiles"] == 0 and not f.any() and not r.any()
    # a single fluid node bounces everything back: f* stays the same closed form
    mask = np.ones((8, 8, 8), bool)
    mask[3, 5, 2] = False
    f0 = inputs.random_pdfs(19, mask, seed=15)
    f, _, _, _ = _gpu_run(torch, mask, 19, 0.8, (1e-6, 2e-6, 0), 4, (1, 1, 1), f0=f0)
    want = dense.step(19, mask, f0, 0.8, [1e-6, 2e-6, 0], 4, periodic=7)
    assert np.max(np.abs(f - want)) <= 1e-15
    # fully fluid periodic box
    mask = np.zeros((8, 12, 16), bool)
    rho, u = inputs.random_macro(mask, seed=16)
    f, _, _, _ = _gpu_run(torch, mask, 19, 0.6, (1e-5, 0, 0), 50, (1, 1, 1), rho=rho, u=u)
    want = dense.step(19, mask, dense.init(19, mask, rho=rho, u=u), 0.6, [1e-5, 0, 0], 50, periodic=7)
    assert np.max(np.abs(f - want) / np.abs(want)) <= 1e-13


def test_step_before_init_is_an_error(torch):
    t = _tiles(inputs.spheres_3d(16, 0.5, rmin=2, rmax=4, seed=1)[0], 19)
    s = lbm.Solver(t, lattice=19, tau=0.7)
    with pytest.raises(lbm.LbmError) as e:
        s.step(1)
    assert e.value.code == lbm.LBM_ERR_STATE


@pytest.mark.parametrize("kernel", ["generic", "scalar"])
@pytest.mark.parametrize("storage,scale", [("f32", 0), ("f16", 12)])
def test_offset_storage_permutation_bitexact(torch, storage, scale, kernel):
    """Pure streaming moves stored offsets unchanged; with PDFs whose offsets
    are representable in the storage type, GPU == oracle exactly."""
    q = 19
    mask = inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=2, periodic=(1, 0, 0))[0]
    _, w, _ = dense.lattice(q)
    rng = np.random.default_rng(17)
    off = rng.uniform(-1e-3, 1e-3, size=(q,) + mask.shape)
    if storage == "f32":
        off = off.astype(np.float32).astype(np.float64)
    else:
        off = (off * 2.0 ** scale).astype(np.float16).astype(np.float64) / 2.0 ** scale
    f0 = w[:, None, None, None] + off
    f0[:, mask] = 0.0
    f, _, _, _ = _gpu_run(torch, mask, q, math.inf, (0, 0, 0), 6, (1, 0, 0), f0=f0, storage=storage,
                          f16_scale_log2=scale, kernel=kernel)
    want = dense.step(q, mask, f0, math.inf, [0, 0, 0], 6, periodic=(1, 0, 0))
    assert np.array_equal(f, want)


@pytest.mark.parametrize("kernel", ["generic", "scalar"])
@pytest.mark.parametrize("storage,tol", [("f32", 2e-5), ("f16", 2e-2)])
def test_offset_storage_error_vs_fp64(torch, storage, tol, kernel):
    """FP32 / FP16-offset storage with FP32 arithmetic: velocity error against
    the FP64 oracle after 1000 steps (D3Q19 periodic porous crop)."""
    mask = inputs.spheres_3d(32, 0.3, seed=8)[0]
    g = (1e-6, 0.0, 0.0)
    _, _, v, _ = _gpu_run(torch, mask, 19, 0.7, g, 1000, (1, 1, 1), storage=storage, f16_scale_log2=22,
                          kernel=kernel)
    want = dense.step(19, mask, dense.init(19, mask), 0.7, g, 1000, periodic=7, nthreads=8)
    _, uw = dense.moments(19, mask, want, g)
    fl = ~mask
    err = np.linalg.norm((v - uw)[:, fl]) / np.linalg.norm(uw[:, fl])
    _log("offset storage", storage, "velocity rel-L2 error after 1000 steps:", err)
    assert err <= tol


@pytest.mark.parametrize("storage,kernel", [("f64", "scalar"), ("f32", "scalar"), ("f16", "scalar"),
                                            ("f64", "generic")])
def test_step_writes_every_fluid_entry(torch, storage, kernel):
    """The whole workspace starts as 0xFF bytes (NaN in FP64, FP32 and FP16):
    init must write every non-solid entry of one copy and each step every
    non-solid entry of the other, and nothing may rely on zeroed scratch."""
    mask = inputs.spheres_3d(24, 0.45, rmin=2, rmax=5, seed=21)[0]
    t = _tiles(mask, 19)
    kw = dict(lattice=19, storage=storage, tau=0.8, g=(1e-6, 0, 0), step_kernel=kernel, f16_scale_log2=20)
    n = lbm.workspace_bytes(t, **kw)
    ws = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    s = lbm.Solver(t, workspace=ws, **kw)
    s.init()
    fl = torch.from_numpy(~mask).cuda()
    for _ in range(3):
        f = s.pdfs_export()
        assert bool(torch.isfinite(f[:, fl]).all()), "an entry was never written"
        s.step(1)
    assert np.all(np.isfinite(s.reduce()))


def test_batch_persistent_graph_writes_every_fluid_entry(torch):
    parts = [_tiles(inputs.spheres_3d(n, 0.5, rmin=2, rmax=4, seed=30 + n)[0], 19) for n in (16, 20)]
    t = lbm.Tiles.concat(parts)
    kw = dict(lattice=19, storage="f32", tau=0.8, persistent=1, graph_steps=3)
    n = lbm.workspace_bytes(t, **kw)
    ws = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    s = lbm.Solver(t, workspace=ws, **kw)
    s.set_sample_force(np.array([[1e-6, 0, 0], [0, 1e-6, 0]]))
    s.init()
    s.step(7)
    tot = s.reduce()
    assert np.all(np.isfinite(tot)) and tot.shape == (2, 4)


def test_nonfinite_state_is_reported(torch):
    mask = inputs.spheres_3d(16, 0.5, rmin=2, rmax=4, seed=22)[0]
    t = _tiles(mask, 19)
    s = lbm.Solver(t, lattice=19, tau=0.8, g=(1e-6, 0, 0))
    s.init()
    f = s.pdfs_export().clone()
    z, y, x = [int(v[0]) for v in np.nonzero(~mask)]
    f[3, z, y, x] = float("nan")
    s.pdfs_import(f)
    for call in (s.reduce, s.residual):
        with pytest.raises(lbm.LbmError) as e:
            call()
        assert e.value.code == lbm.LBM_ERR_NONFINITE
    s.init()  # a fresh start clears the state
    assert np.all(np.isfinite(s.reduce()))
