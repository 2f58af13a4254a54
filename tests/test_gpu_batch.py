"""Batched runs on the GPU: a concatenated tile list of uneven samples gives
exactly the per-sample results, converged samples can leave the active list,
the persistent grid and captured HIP graphs give the same bits as plain
launches (replayed several times with eager work in between)."""
import math

import numpy as np
import pytest

from paper_1703_08015_amd import inputs, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _samples():
    specs = [dict(edge=16, porosity=0.5, g=(1e-5, 2e-6, 0.0), seed=1),
             dict(edge=24, porosity=0.35, g=(0.0, -3e-6, 4e-6), seed=2),
             dict(edge=12, porosity=0.7, g=(-2e-6, 0.0, 1e-6), seed=3)]
    masks = [inputs.spheres_3d(s["edge"], s["porosity"], rmin=2, rmax=5, seed=s["seed"])[0] for s in specs]
    return specs, masks


def _single(torch, mask, g, steps, **kw):
    s = lbm.Solver(lbm.Tiles(mask), lattice=19, tau=0.8, g=g, **kw)
    s.init()
    s.step(steps)
    return s.pdfs_export().cpu().numpy().ravel()


def _batch(masks, specs, **kw):
    tb = lbm.Tiles.concat([lbm.Tiles(m) for m in masks])
    s = lbm.Solver(tb, lattice=19, tau=0.8, **kw)
    s.set_sample_force(np.array([sp["g"] for sp in specs]))
    s.init()
    return s


def _split(f, masks):
    out, o = [], 0
    for m in masks:
        n = 19 * m.size
        out.append(f[o:o + n])
        o += n
    return out


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_equals_each_sample_alone(torch, storage):
    specs, masks = _samples()
    s = _batch(masks, specs, storage=storage)
    s.step(25)
    parts = _split(s.pdfs_export().cpu().numpy(), masks)
    for sp, m, got in zip(specs, masks, parts):
        assert np.array_equal(got, _single(torch, m, sp["g"], 25, storage=storage))


def test_deactivated_sample_is_frozen(torch):
    specs, masks = _samples()
    s = _batch(masks, specs)
    s.step(7)  # odd count: the frozen state must survive the copy swap
    frozen = _split(s.pdfs_export().cpu().numpy(), masks)[1].copy()
    s.set_active([1, 0, 1])
    s.step(10)
    parts = _split(s.pdfs_export().cpu().numpy(), masks)
    assert np.array_equal(parts[1], frozen)
    assert np.array_equal(parts[0], _single(torch, masks[0], specs[0]["g"], 17))
    assert np.array_equal(parts[2], _single(torch, masks[2], specs[2]["g"], 17))
    s.set_active([1, 1, 1])
    s.step(3)
    parts = _split(s.pdfs_export().cpu().numpy(), masks)
    assert np.array_equal(parts[0], _single(torch, masks[0], specs[0]["g"], 20))


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("graph_steps", [0, 5, 4])
def test_persistent_and_graphs_match_plain_launches(torch, persistent, graph_steps):
    specs, masks = _samples()
    ref = _batch(masks, specs)
    ref.step(40)
    want = ref.pdfs_export()
    s = _batch(masks, specs, persistent=persistent, graph_steps=graph_steps)
    for k in range(4):  # replays separated by eager work and synchronisation
        s.step(10)
        r, u = s.moments()
        torch.cuda.synchronize()
        assert torch.isfinite(u).all()
    assert torch.equal(s.pdfs_export(), want)
    # with a sample switched off the same graphs keep working
    s.set_active([1, 0, 1])
    ref.set_active([1, 0, 1])
    s.step(15)
    ref.step(15)
    assert torch.equal(s.pdfs_export(), ref.pdfs_export())


def test_run_to_steady_deactivates_converged_samples(torch):
    specs, masks = _samples()
    s = _batch(masks, specs, graph_steps=50, persistent=1)
    steps, res = s.run_to_steady(tol=1e-6, check_every=50, max_steps=40000)
    assert np.all(steps > 0), (steps, res)
    assert np.all(res < 1e-6)
    # each sample reached the same steady state it reaches alone
    for k, (sp, m) in enumerate(zip(specs, masks)):
        one = lbm.Solver(lbm.Tiles(m), lattice=19, tau=0.8, g=sp["g"])
        one.init()
        st1, _ = one.run_to_steady(tol=1e-6, check_every=50, max_steps=40000)
        assert st1[0] == steps[k]


def test_autotuner_picks_a_timed_candidate_and_caches(torch, tmp_path):
    from paper_1703_08015_amd import autotune
    m = inputs.spheres_3d(32, 0.4, rmin=2, rmax=6, seed=4)[0]
    cache = str(tmp_path / "tune.json")
    best = autotune.autotune(m, tau=0.7, storage="f32", steps=5, warmup=2, cache_path=cache)
    assert not best["cached"] and best["ms_per_step"] > 0
    timed = [t for t in best["trials"] if "ms_per_step" in t]
    assert len(timed) == len(autotune.candidates(19))
    assert best["ms_per_step"] == min(t["ms_per_step"] for t in timed)
    again = autotune.autotune(m, tau=0.7, storage="f32", cache_path=cache)
    assert again["cached"] and again["tile"] == best["tile"] and again["tiles_per_block"] == best["tiles_per_block"]
    # a batch only considers configurations that can drop converged samples
    specs, masks = _samples()
    bb = autotune.autotune(masks, tau=0.8, steps=3, warmup=1, cache_path=cache)
    assert bb["tile"] == (4, 4, 4) and bb["step_kernel"] == "scalar"


@pytest.mark.parametrize("persistent,graph_steps", [(0, 0), (1, 5)])
def test_tall_tile_batch_on_scalar_kernel(torch, persistent, graph_steps):
    """4x4x8 tiles on the scalar-mask kernel (two wavefronts per tile): a batch
    with per-sample forces, direct or persistent launches with graph replay,
    and a sample frozen half way, gives the bits of each sample run alone on
    4x4x4 tiles."""
    specs = [dict(edge=16, porosity=0.5, g=(1e-5, 2e-6, 0.0), seed=1),
             dict(edge=24, porosity=0.35, g=(0.0, -3e-6, 4e-6), seed=2),
             dict(edge=8, porosity=0.7, g=(-2e-6, 0.0, 1e-6), seed=3)]
    masks = [inputs.spheres_3d(sp["edge"], sp["porosity"], rmin=2, rmax=5, seed=sp["seed"])[0] for sp in specs]
    tb = lbm.Tiles.concat([lbm.Tiles(m, (4, 4, 8)) for m in masks])
    s = lbm.Solver(tb, lattice=19, tau=0.8, step_kernel="scalar", persistent=persistent, graph_steps=graph_steps)
    s.set_sample_force(np.array([sp["g"] for sp in specs]))
    s.init()
    s.step(12)
    s.set_active([1, 0, 1])
    s.step(8)
    parts = _split(s.pdfs_export().cpu().numpy(), masks)
    for k, (sp, m, got) in enumerate(zip(specs, masks, parts)):
        want = _single(torch, m, sp["g"], 12 if k == 1 else 20)
        assert np.array_equal(got, want), k
