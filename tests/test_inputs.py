"""The seeded input generators (CPU): deterministic per seed, report the
porosity they produce, stop at the target, keep the structure they promise
(channel walls, periodic wrap, fluid inside vessels), and the batch
specification follows its stated ranges."""
import numpy as np
import pytest

from paper_1703_08015_amd import inputs


def test_channel_2d_deterministic_walls_and_porosity():
    a, pa = inputs.channel_2d(96, 80, porosity=0.65, seed=7)
    b, pb = inputs.channel_2d(96, 80, porosity=0.65, seed=7)
    c, _ = inputs.channel_2d(96, 80, porosity=0.65, seed=8)
    assert np.array_equal(a, b) and pa == pb and not np.array_equal(a, c)
    assert a.shape == (1, 80, 96)
    assert a[0, 0].all() and a[0, -1].all()  # walls
    assert np.isclose(pa, 1.0 - a.mean(), rtol=0, atol=1e-15)
    assert 0.6 < pa <= 0.65  # stops at the first placement that reaches the target
    # without discs only the two walls are solid
    free, _ = inputs.channel_2d(96, 80, discs=False)
    assert free.sum() == 2 * 96


def test_channel_2d_discs_do_not_overlap():
    """Discs keep a gap: every solid connected blob away from the walls is one disc."""
    from scipy import ndimage
    m, _ = inputs.channel_2d(128, 64, porosity=0.7, rmin=3, rmax=5, seed=2)
    inner = m[0, 1:-1].copy()
    lab, n = ndimage.label(inner)
    sizes = ndimage.sum(inner, lab, range(1, n + 1))
    assert n > 10
    assert sizes.max() <= np.pi * (5 + 1) ** 2  # no blob larger than one disc of the largest radius


def test_spheres_3d_deterministic_porosity_and_wrap():
    a, pa = inputs.spheres_3d((24, 20, 16), 0.5, rmin=3, rmax=5, seed=4)
    b, pb = inputs.spheres_3d((24, 20, 16), 0.5, rmin=3, rmax=5, seed=4)
    assert np.array_equal(a, b) and pa == pb
    assert a.shape == (16, 20, 24)
    assert np.isclose(pa, 1.0 - a.mean(), rtol=0, atol=1e-15) and 0.4 < pa <= 0.5
    # periodic: the solid fraction near opposite faces is alike, and spheres cross the faces
    assert a[:, :, 0].any() and a[:, :, -1].any()
    np_, _ = inputs.spheres_3d((24, 20, 16), 0.5, rmin=3, rmax=5, seed=4, periodic=(0, 0, 0))
    assert not np.array_equal(np_, a)


def test_vessel_tree_is_sparse_fluid_in_solid():
    m, phi = inputs.vessel_tree(64, 0.05, r_root=5, r_leaf=2, seed=5)
    m2, phi2 = inputs.vessel_tree(64, 0.05, r_root=5, r_leaf=2, seed=5)
    assert np.array_equal(m, m2) and phi == phi2
    assert np.isclose(phi, 1.0 - m.mean(), rtol=0, atol=1e-15) and phi >= 0.05
    # fluid is tubular: most fluid nodes have fluid neighbours along some axis
    fl = ~m
    nb = sum(np.roll(fl, s, a) for a in range(3) for s in (-1, 1))
    assert (nb[fl] >= 2).mean() > 0.95


def test_batch_specs_ranges():
    specs = inputs.batch_specs(200, seed=3)
    assert specs == inputs.batch_specs(200, seed=3)
    edges = {s["edge"] for s in specs}
    assert edges <= set(range(32, 97, 4)) and len(edges) > 10
    phis = np.array([s["porosity"] for s in specs])
    assert phis.min() >= 0.2 and phis.max() <= 0.8
    g = np.array([s["g"] for s in specs])
    assert np.allclose(np.linalg.norm(g, axis=1), 1e-6)
    assert abs(g.mean(axis=0)).max() < 3e-7  # directions spread over the sphere
    assert len({s["seed"] for s in specs}) == 200


@pytest.mark.parametrize("seed", [0, 1])
def test_random_fields_are_seeded(seed):
    mask = inputs.spheres_3d(12, 0.6, rmin=2, rmax=3, seed=1)[0]
    f1, f2 = inputs.random_pdfs(19, mask, seed=seed), inputs.random_pdfs(19, mask, seed=seed)
    assert np.array_equal(f1, f2) and np.all(f1[:, mask] == 0) and np.all(f1[:, ~mask] > 0)
    r1, u1 = inputs.random_macro(mask, seed=seed)
    r2, u2 = inputs.random_macro(mask, seed=seed)
    assert np.array_equal(r1, r2) and np.array_equal(u1, u2)
