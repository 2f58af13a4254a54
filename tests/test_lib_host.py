"""Host-side checks of liblbm (no GPU needed): the library loads, exports
every function ``include/lbm.h`` declares, its tiling equals the NumPy tiling
oracle bit for bit, its lattice equals the oracle's, and host-side argument
validation reports the documented error codes."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import dense
from oracle import tiles as otiles
from paper_1703_08015_amd import inputs, lbm


def test_library_exports_every_declared_symbol():
    names = lbm.header_functions()
    assert len(names) >= 20
    L = lbm.lib()
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("q", [9, 19])
def test_lattice_matches_oracle(q):
    c, w, opp = lbm.lattice(q)
    c2, w2, opp2 = dense.lattice(q)
    assert np.array_equal(c, c2) and np.array_equal(w, w2) and np.array_equal(opp, opp2)


def _masks():
    yield "channel", inputs.channel_2d(64, 64, seed=0)[0], (16, 16, 1), (1, 0, 0)
    yield "channel_ragged", inputs.channel_2d(48, 37, porosity=0.7, seed=3)[0], (16, 16, 1), (1, 0, 0)
    yield "spheres", inputs.spheres_3d(32, 0.3, seed=1)[0], (4, 4, 4), (1, 1, 1)
    yield "spheres_ragged", inputs.spheres_3d((21, 18, 13), 0.5, rmin=2, rmax=5, seed=2,
                                             periodic=(0, 0, 0))[0], (4, 4, 4), (0, 0, 0)
    yield "spheres_tall", inputs.spheres_3d((16, 12, 24), 0.4, rmin=2, rmax=5, seed=4)[0], (4, 4, 8), (1, 1, 1)
    yield "vessel", inputs.vessel_tree(64, 0.08, r_root=5, r_leaf=2, seed=5)[0], (4, 4, 4), (1, 1, 1)


@pytest.mark.parametrize("name,mask,tile,periodic", list(_masks()), ids=lambda v: v if isinstance(v, str) else "")
def test_tiles_bitexact_vs_oracle(name, mask, tile, periodic):
    t = lbm.Tiles(mask, tile, periodic)
    e = t.export()
    o = otiles.tile(mask, tile, periodic)
    for k in ("tile_map", "tile_coord", "nbr", "fluid"):
        assert np.array_equal(e[k], o[k]), k
    i = t.info
    assert i["n_ftiles"] == o["n_ftiles"] and i["n_fluid"] == o["n_fluid"] and i["n_tiles"] == o["n_tiles"]
    assert i["phi"] == o["phi"] and math.isclose(i["phi_t"], o["phi_t"], rel_tol=1e-15)
    assert i["alpha_m"] == o["alpha_m"]
    assert tuple(i["grid"]) == tuple(o["grid"])


@settings(max_examples=80, deadline=None, derandomize=True)
@given(st.data())
def test_tiles_random_masks_bitexact(data):
    """Random masks of random shape, solid fraction and periodicity, for every
    tile shape: the library's tiling equals the oracle's bit for bit (periodic
    axes are drawn as multiples of the tile edge, as the library requires)."""
    tile = data.draw(st.sampled_from([(4, 4, 4), (4, 4, 8), (16, 16, 1)]))
    per = tuple(data.draw(st.booleans()) for _ in range(3))
    shape = []
    for a in range(3):
        if tile == (16, 16, 1) and a == 2:
            shape.append(1)
            continue
        hi = 40 if tile[a] == 16 else 14
        n = data.draw(st.integers(1, hi))
        if per[a]:
            n = -(-n // tile[a]) * tile[a]
        shape.append(n)
    density = data.draw(st.floats(0.0, 1.0))
    seed = data.draw(st.integers(0, 2 ** 31))
    mask = np.random.default_rng(seed).random(shape[::-1]) < density  # (nz, ny, nx)
    t = lbm.Tiles(mask, tile, per)
    e, o = t.export(), otiles.tile(mask, tile, per)
    for k in ("tile_map", "tile_coord", "nbr", "fluid"):
        assert np.array_equal(e[k], o[k]), k
    assert t.info["n_fluid"] == o["n_fluid"] and t.info["n_ftiles"] == o["n_ftiles"]
    assert t.info["alpha_m"] == o["alpha_m"]


def test_tiles_concat_offsets_rows():
    a = inputs.spheres_3d(16, 0.5, rmin=2, rmax=4, seed=1)[0]
    b = inputs.spheres_3d((8, 12, 16), 0.5, rmin=2, rmax=4, seed=2)[0]
    ta, tb = lbm.Tiles(a), lbm.Tiles(b)
    tc = lbm.Tiles.concat([ta, tb])
    ea, eb, ec = ta.export(), tb.export(), tc.export()
    na = ta.info["n_ftiles"]
    assert tc.info["n_samples"] == 2 and tc.info["n_ftiles"] == na + tb.info["n_ftiles"]
    assert np.array_equal(ec["nbr"][:27 * na], ea["nbr"])
    assert np.array_equal(ec["nbr"][27 * na:], np.where(eb["nbr"] < 0, -1, eb["nbr"] + na))
    assert np.array_equal(ec["fluid"], np.concatenate([ea["fluid"], eb["fluid"]]))
    assert np.array_equal(ec["tile_map"], np.concatenate([ea["tile_map"],
                                                          np.where(eb["tile_map"] < 0, -1, eb["tile_map"] + na)]))


def test_tiling_errors():
    with pytest.raises(lbm.LbmError) as e:
        lbm.Tiles(np.zeros((4, 4, 6), bool), (4, 4, 4), (1, 0, 0))
    assert e.value.code == lbm.LBM_ERR_SHAPE
    with pytest.raises(lbm.LbmError) as e:
        lbm.Tiles(np.zeros((4, 4, 8), bool), (8, 8, 8), (1, 1, 1))
    assert e.value.code == lbm.LBM_ERR_UNSUPPORTED
    t = lbm.Tiles(np.ones((8, 8, 8), bool))
    assert t.info["n_ftiles"] == 0 and t.info["n_fluid"] == 0


@pytest.mark.parametrize("kw,code", [
    (dict(tau=0.5), lbm.LBM_ERR_ARG),
    (dict(tau=0.2), lbm.LBM_ERR_ARG),
    (dict(tau=float("nan")), lbm.LBM_ERR_ARG),
    (dict(tau=-math.inf), lbm.LBM_ERR_ARG),
    (dict(rho0=0.0), lbm.LBM_ERR_ARG),
    (dict(g=(float("inf"), 0, 0)), lbm.LBM_ERR_ARG),
    (dict(storage=7), lbm.LBM_ERR_ARG),
    (dict(f16_scale_log2=40), lbm.LBM_ERR_ARG),
    (dict(lattice=9), lbm.LBM_ERR_UNSUPPORTED),
    (dict(tiles_per_block=3), lbm.LBM_ERR_UNSUPPORTED),
    (dict(tile_order=5), lbm.LBM_ERR_ARG),
    (dict(step_kernel=9), lbm.LBM_ERR_ARG),
    (dict(model=2), lbm.LBM_ERR_ARG),
    (dict(model=-1), lbm.LBM_ERR_ARG),
    (dict(pattern=2), lbm.LBM_ERR_ARG),
    (dict(collision=5), lbm.LBM_ERR_ARG),
    (dict(collision="mrt", mrt_rates=(2.5, 0, 0, 0, 0)), lbm.LBM_ERR_ARG),
    (dict(collision="mrt", mrt_rates=(1.2, -1.0, 0, 0, 0)), lbm.LBM_ERR_ARG),
    (dict(collision="mrt", tiles_per_block=2), lbm.LBM_ERR_UNSUPPORTED),
    (dict(collision="mrt", store_policy="regular"), lbm.LBM_ERR_UNSUPPORTED),
])
def test_param_validation(kw, code):
    t = lbm.Tiles(inputs.spheres_3d(16, 0.5, rmin=2, rmax=4, seed=1)[0])
    with pytest.raises(lbm.LbmError) as e:
        lbm.workspace_bytes(t, **kw)
    assert e.value.code == code


def test_workspace_size_counts_fluid_nodes_only():
    m = inputs.spheres_3d(32, 0.3, seed=1)[0]
    t = lbm.Tiles(m)
    for storage, sd in (("f64", 8), ("f32", 4), ("f16", 2)):
        n = lbm.workspace_bytes(t, storage=storage, tau=0.7)
        pdf = 2 * 19 * sd * t.info["n_fluid"]
        # two copies of the fluid nodes' PDFs (each tile region padded to 128 bytes), the FP64
        # residual reference velocity (24 bytes per fluid node) and under 200 bytes of tables per
        # tile (FP16: 256 more, the region bases of the step)
        nft = t.info["n_ftiles"]
        tables = 200 + (256 if storage == "f16" else 0)
        assert pdf < n < pdf + 24 * t.info["n_fluid"] + (2 * 128 + tables) * nft + 8192
    assert lbm.workspace_bytes(t, tau=math.inf) > 0


def test_single_copy_workspace_holds_one_pdf_copy():
    """The single-copy pattern needs exactly one PDF copy less."""
    m = inputs.spheres_3d(32, 0.3, seed=1)[0]
    t = lbm.Tiles(m)
    for storage, sd in (("f64", 8), ("f32", 4), ("f16", 2)):
        two = lbm.workspace_bytes(t, storage=storage, tau=0.7)
        one = lbm.workspace_bytes(t, storage=storage, tau=0.7, pattern="single-copy")
        copy = two - one
        # one copy: the fluid nodes' PDFs, each tile region padded to 128 bytes, the copy to 256
        assert 19 * sd * t.info["n_fluid"] <= copy <= 19 * sd * t.info["n_fluid"] + 128 * t.info["n_ftiles"] + 256


def test_autotune_candidates_and_key():
    from paper_1703_08015_amd import autotune
    c19 = autotune.candidates(19)
    assert any(c["tile"] == (4, 4, 8) for c in c19) and any(c["persistent"] for c in c19)
    # a batch that drops converged samples needs the scalar-mask step (either form, either tile shape)
    cb = autotune.candidates(19, batched=True)
    assert all(c["step_kernel"] in ("scalar", "shuffle") for c in cb) and any(c["tile"] == (4, 4, 8) for c in cb)
    m = np.zeros((8, 8, 8), bool)
    k1 = autotune.geometry_key([m], (1, 1, 1), 19, "f64", 0.7)
    m2 = m.copy()
    m2[0, 0, 0] = True
    assert k1 != autotune.geometry_key([m2], (1, 1, 1), 19, "f64", 0.7)
    assert k1 != autotune.geometry_key([m], (1, 1, 1), 19, "f32", 0.7)


def test_library_exports_every_nn_symbol():
    from paper_1703_08015_amd import nn
    names = nn.header_functions()
    assert len(names) >= 10
    L = lbm.lib()
    for n in names:
        assert hasattr(L, n), n


def test_components_bitexact_vs_oracle():
    from oracle import invariants
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(6):
        shape = tuple(int(v) for v in rng.integers(2, 10, size=3))
        cases.append((19, rng.random(shape) < rng.uniform(0.3, 0.7), int(rng.integers(0, 8))))
        cases.append((9, rng.random((1,) + shape[1:]) < rng.uniform(0.3, 0.7), int(rng.integers(0, 4))))
    m, _ = inputs.spheres_3d(32, 0.5, 2.0, 4.0, seed=2)
    cases.append((19, m, 7))
    for q, mask, periodic in cases:
        for axis in range(-1, 2 if q == 9 else 3):
            lab, n = lbm.components(mask, q, axis, periodic)
            ref, nref = invariants.components(mask, q, axis, periodic)
            assert n == nref and np.array_equal(lab, ref.astype(np.int32)), (q, mask.shape, periodic, axis)


def test_components_errors():
    m = np.zeros((4, 4, 4), bool)
    for kw, code in [(dict(lattice=27), lbm.LBM_ERR_UNSUPPORTED), (dict(axis=3), lbm.LBM_ERR_ARG),
                     (dict(axis=-2), lbm.LBM_ERR_ARG), (dict(lattice=9), lbm.LBM_ERR_ARG),
                     (dict(periodic=8), lbm.LBM_ERR_ARG)]:
        with pytest.raises(lbm.LbmError) as e:
            lbm.components(m, **kw)
        assert e.value.code == code, kw
    lab, n = lbm.components(np.ones((3, 3, 3), bool))
    assert n == 0 and np.all(lab == -1)
