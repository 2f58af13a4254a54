"""The single-copy (in-place) PDF pattern on the GPU, through the C ABI.

Every step of the single copy does the arithmetic of the two-copy step on
the same values, so the two patterns must agree bit for bit: PDF exports,
moments, reductions and residuals after odd and even step counts (the two
layouts of the single copy), on both step kernels, both lattices, all
storage forms and both fluid models.  The two-copy path is itself pinned to
the oracle; the single copy is also checked against the oracle directly
(pure streaming bit-exact, FP64 within 1e-12 after 1001 steps), for
batches on the persistent grid with graph replay, for the active-set rule and
for a workspace that starts as NaN bytes.
"""
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


CASES = [
    # (name, q, tile, kernel, storage, model)
    ("d3q19_scalar_f64", 19, (4, 4, 4), "scalar", "f64", "quasi-compressible"),
    ("d3q19_scalar_f32", 19, (4, 4, 4), "scalar", "f32", "quasi-compressible"),
    ("d3q19_scalar_f16", 19, (4, 4, 4), "scalar", "f16", "quasi-compressible"),
    ("d3q19_scalar_f64_inc", 19, (4, 4, 4), "scalar", "f64", "incompressible"),
    ("d3q19_generic_f64", 19, (4, 4, 4), "generic", "f64", "quasi-compressible"),
    ("d3q19_tall_f32", 19, (4, 4, 8), "generic", "f32", "quasi-compressible"),
    ("d2q9_f64", 9, (16, 16, 1), "generic", "f64", "quasi-compressible"),
    ("d2q9_f16_inc", 9, (16, 16, 1), "generic", "f16", "incompressible"),
]


def _geometry(q, tile):
    if q == 9:
        return inputs.channel_2d(48, 37, porosity=0.7, seed=51)[0], (1, 0, 0), (2e-5, -1e-5, 0.0)
    if tile == (4, 4, 8):
        return inputs.spheres_3d((16, 12, 24), 0.45, rmin=2, rmax=5, seed=52)[0], (1, 1, 1), (1e-5, 0.0, -3e-6)
    return (inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=53, periodic=(1, 0, 0))[0], (1, 0, 0),
            (2e-5, -1e-5, 3e-6))


def _solver(mask, q, tile, per, g, pattern, **kw):
    return lbm.Solver(lbm.Tiles(mask, tile, per), lattice=q, tau=0.7, g=g, f16_scale_log2=18, pattern=pattern, **kw)


def _state(torch, s):
    f = s.pdfs_export()
    r, u = s.moments()
    torch.cuda.synchronize()
    return f.cpu().numpy(), r.cpu().numpy(), u.cpu().numpy(), s.reduce(), s.residual()


@pytest.mark.parametrize("name,q,tile,kernel,storage,model", CASES)
def test_single_copy_equals_two_copy(torch, name, q, tile, kernel, storage, model):
    mask, per, g = _geometry(q, tile)
    rho, u = inputs.random_macro(mask, seed=54)
    if q == 9:
        u[2] = 0.0
    kw = dict(step_kernel=kernel, storage=storage, model=model)
    a = _solver(mask, q, tile, per, g, "two-copy", **kw)
    b = _solver(mask, q, tile, per, g, "single-copy", **kw)
    for s in (a, b):
        s.init(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    done = 0
    for n in (0, 1, 1, 3, 2, 7):
        a.step(n)
        b.step(n)
        done += n
        _log("single copy", name, "after", done, "steps")
        sa, sb = _state(torch, a), _state(torch, b)
        for x, y in zip(sa, sb):
            assert np.array_equal(x, y), (name, done)
    assert a.step_count == b.step_count == done


def test_pure_streaming_bitexact_against_oracle(torch):
    """tau = +inf, g = 0: the in-place steps only move values."""
    mask = inputs.spheres_3d((20, 22, 13), 0.5, rmin=2, rmax=5, seed=55, periodic=(1, 0, 0))[0]
    f0 = inputs.random_pdfs(19, mask, seed=56)
    for kernel in ("scalar", "generic"):
        for n in (1, 4, 7):
            s = lbm.Solver(lbm.Tiles(mask, (4, 4, 4), (1, 0, 0)), lattice=19, tau=math.inf, step_kernel=kernel,
                           pattern="single-copy")
            s.pdfs_import(torch.from_numpy(f0).cuda())
            s.step(n)
            got = s.pdfs_export().cpu().numpy()
            assert np.array_equal(got, dense.step(19, mask, f0, math.inf, [0, 0, 0], n, periodic=(1, 0, 0))), (kernel, n)


def test_fp64_1001_steps_against_oracle(torch):
    mask = inputs.spheres_3d(32, 0.3, seed=8)[0]
    g = (1e-6, 0.0, 0.0)
    rho, u = inputs.random_macro(mask, seed=57)
    s = lbm.Solver(lbm.Tiles(mask), lattice=19, tau=0.7, g=g, pattern="single-copy")
    s.init(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    s.step(1001)
    f = s.pdfs_export().cpu().numpy()
    want = dense.step(19, mask, dense.init(19, mask, rho=rho, u=u), 0.7, g, 1001, periodic=7, nthreads=8)
    fl = ~mask
    assert np.max(np.abs(f - want)[:, fl] / np.abs(want)[:, fl]) <= 1e-12


def _batch(torch, pattern, **kw):
    specs = [(16, 0.5, (1e-5, 2e-6, 0.0), 61), (24, 0.35, (0.0, -3e-6, 4e-6), 62), (12, 0.7, (-2e-6, 0.0, 1e-6), 63)]
    masks = [inputs.spheres_3d(e, p, rmin=2, rmax=5, seed=sd)[0] for e, p, _, sd in specs]
    tb = lbm.Tiles.concat([lbm.Tiles(m) for m in masks])
    s = lbm.Solver(tb, lattice=19, tau=0.8, storage="f32", pattern=pattern, **kw)
    s.set_sample_force(np.array([sp[2] for sp in specs]))
    s.init()
    return s


@pytest.mark.parametrize("persistent,graph_steps", [(0, 0), (1, 0), (1, 5), (0, 4)])
def test_batch_matches_two_copy(torch, persistent, graph_steps):
    """Batches on the persistent grid and with graph replay (odd and even
    graph lengths, eager work between replays), with a sample frozen after an
    even number of steps and read while the others are in the other layout."""
    a = _batch(torch, "two-copy", persistent=persistent, graph_steps=graph_steps)
    b = _batch(torch, "single-copy", persistent=persistent, graph_steps=graph_steps)
    for k in range(4):
        a.step(5)
        b.step(5)
        torch.cuda.synchronize()
        assert np.array_equal(a.pdfs_export().cpu().numpy(), b.pdfs_export().cpu().numpy()), k
    # 20 steps done: the single copy is in layout 0 and may change its active set
    for s in (a, b):
        s.set_active(np.array([1, 0, 1], np.uint8))
    a.step(3)
    b.step(3)  # odd: active samples in layout 1, the frozen one in layout 0
    for x, y in zip(_state(torch, a), _state(torch, b)):
        assert np.array_equal(x, y)
    with pytest.raises(lbm.LbmError) as e:
        b.set_active(np.array([1, 1, 1], np.uint8))
    assert e.value.code == lbm.LBM_ERR_STATE
    b.set_active(np.array([1, 0, 1], np.uint8))  # an unchanged set is always allowed
    a.step(1)
    b.step(1)
    for s in (a, b):
        s.set_active(np.array([1, 1, 1], np.uint8))
    a.step(6)
    b.step(6)
    for x, y in zip(_state(torch, a), _state(torch, b)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("storage,kernel", [("f64", "scalar"), ("f16", "scalar"), ("f32", "generic")])
def test_steps_write_every_fluid_entry(torch, storage, kernel):
    """The workspace starts as 0xFF bytes (NaN in every storage form): init
    must write every non-solid entry, and every in-place step must leave the
    state complete in both layouts."""
    mask = inputs.spheres_3d(24, 0.45, rmin=2, rmax=5, seed=64)[0]
    t = lbm.Tiles(mask)
    kw = dict(lattice=19, storage=storage, tau=0.8, g=(1e-6, 0, 0), step_kernel=kernel, f16_scale_log2=20,
              pattern="single-copy")
    n = lbm.workspace_bytes(t, **kw)
    ws = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    s = lbm.Solver(t, workspace=ws, **kw)
    s.init()
    fl = torch.from_numpy(~mask).cuda()
    for _ in range(4):
        f = s.pdfs_export()
        assert bool(torch.isfinite(f[:, fl]).all()), "an entry was never written"
        s.step(1)
    assert np.all(np.isfinite(s.reduce()))


def test_checkpoint_resume_across_layouts(torch):
    """An export taken in layout 1 (odd step count) resumes bit-exactly."""
    mask = inputs.spheres_3d(24, 0.35, rmin=2, rmax=6, seed=65)[0]
    t = lbm.Tiles(mask)
    a = lbm.Solver(t, lattice=19, tau=0.7, g=(1e-6, 0, 0), pattern="single-copy")
    a.init()
    a.step(41)
    fa = a.pdfs_export()
    b = lbm.Solver(t, lattice=19, tau=0.7, g=(1e-6, 0, 0), pattern="single-copy")
    b.init()
    b.step(21)
    ck = b.pdfs_export().clone()
    c = lbm.Solver(t, lattice=19, tau=0.7, g=(1e-6, 0, 0), pattern="single-copy")
    c.pdfs_import(ck)
    c.step(20)
    assert torch.equal(fa, c.pdfs_export())
