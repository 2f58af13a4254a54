"""lbm_project_invariants against the FP64 oracle projection: D3Q19 sphere
packings (periodic, walled, odd extents, many components, diagonal-only
contacts), D2Q9, the all-solid no-op; solid entries untouched; repeated
calls reuse the scratch; the result carries none of the exact invariants."""
import zlib

import numpy as np
import pytest

from oracle import invariants
from paper_1703_08015_amd import inputs, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _cases():
    cavity, _ = inputs.spheres_3d(24, 0.5, 2.0, 4.0, seed=4)
    cavity[2:7, 2:7, 2:7] = True
    cavity[3:6, 3:6, 3:6] = False
    dense, _ = inputs.spheres_3d(32, 0.3, 1.5, 3.0, seed=8)  # many small pores
    walled, _ = inputs.spheres_3d((20, 12, 16), 0.55, 2.0, 4.0, seed=5, periodic=(False, False, False))
    odd, _ = inputs.spheres_3d((13, 9, 11), 0.55, 2.0, 3.0, seed=6)
    diagonal, _ = inputs.spheres_3d(12, 0.5, 1.5, 3.0, seed=3)  # nodes touching only diagonally
    flat = np.random.default_rng(3).random((1, 36, 40)) < 0.5
    return [("cavity24", 19, cavity, 7), ("dense32", 19, dense, 7), ("walled", 19, walled, 0),
            ("odd", 19, odd, 7), ("diagonal12", 19, diagonal, 7), ("d2q9", 9, flat, 3), ("d2q9_walled", 9, flat, 0)]


def _fields(name, q, mask):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    rho = np.where(mask, 7.0, 1.0 + 0.01 * rng.normal(size=mask.shape))
    u = np.where(mask[None], 7.0, 0.01 * rng.normal(size=(3,) + mask.shape))
    if q == 9:
        u[2] = np.where(mask, 7.0, 0.0)
    return rho, u


@pytest.mark.parametrize("name,q,mask,periodic", _cases(), ids=[c[0] for c in _cases()])
def test_projection_matches_oracle(torch, name, q, mask, periodic):
    rho, u = _fields(name, q, mask)
    inv = lbm.Invariants(mask, q, periodic=[bool(periodic >> a & 1) for a in range(3)])
    assert inv.count == invariants.components(mask, q, -1, periodic)[1]
    print(name, "components", inv.count, flush=True)
    for iterations in (1, 8):
        ref_r, ref_u = invariants.project(mask, rho, u, q, rho0=1.0, periodic=periodic, iterations=iterations)
        for call in range(2):
            r_d = torch.from_numpy(rho.copy()).cuda()
            u_d = torch.from_numpy(u.copy()).cuda()
            inv.project(r_d, u_d, rho0=1.0, iterations=iterations)
            torch.cuda.synchronize()
            r_h, u_h = r_d.cpu().numpy(), u_d.cpu().numpy()
            fl = ~mask
            assert np.all(r_h[mask] == 7.0) and np.all(u_h[:, mask] == 7.0), "solid entries changed"
            assert np.abs(r_h[fl] - ref_r[fl]).max() <= 1e-13
            assert np.abs(u_h[:, fl] - ref_u[:, fl]).max() <= 1e-14 * np.abs(ref_u[:, fl]).max()
            if q == 9:
                assert np.all(u_h[2][fl] == 0.0)


def test_projected_momentum_carries_no_invariant(torch):
    """Against the exact invariant basis (dense null space of the link
    operator) of a packing with diagonal-only contacts."""
    mask, _ = inputs.spheres_3d(12, 0.5, 1.5, 3.0, seed=3)
    basis = invariants.invariant_basis(mask, 19)
    rho, u = _fields("basis", 19, mask)
    inv = lbm.Invariants(mask, 19)
    r_d = torch.from_numpy(rho.copy()).cuda()
    u_d = torch.from_numpy(u.copy()).cuda()
    inv.project(r_d, u_d)
    torch.cuda.synchronize()
    r_h, u_h = r_d.cpu().numpy(), u_d.cpu().numpy()
    j = (np.where(mask, 0.0, r_h)[None] * np.where(mask[None], 0.0, u_h)).transpose(1, 2, 3, 0).ravel()
    raw = (np.where(mask, 0.0, rho)[None] * np.where(mask[None], 0.0, u)).transpose(1, 2, 3, 0).ravel()
    assert np.abs(basis.T @ raw).max() > 1e-3 * np.linalg.norm(raw)
    assert np.abs(basis.T @ j).max() <= 1e-14 * np.linalg.norm(j)


def test_projection_of_rest_and_all_solid(torch):
    mask, _ = inputs.spheres_3d(16, 0.5, 2.0, 4.0, seed=1)
    inv = lbm.Invariants(mask, 19)
    r = torch.from_numpy(np.where(mask, 0.0, 1.0)).cuda()
    u = torch.zeros((3,) + mask.shape, dtype=torch.float64, device="cuda")
    inv.project(r, u)
    torch.cuda.synchronize()
    assert torch.equal(r.cpu(), torch.from_numpy(np.where(mask, 0.0, 1.0))) and not u.any()
    solid = np.ones((8, 8, 8), bool)
    inv0 = lbm.Invariants(solid, 19)
    assert inv0.count == 0
    r0 = torch.full((8, 8, 8), 3.0, dtype=torch.float64, device="cuda")
    u0 = torch.full((3, 8, 8, 8), 3.0, dtype=torch.float64, device="cuda")
    inv0.project(r0, u0)
    torch.cuda.synchronize()
    assert bool((r0 == 3.0).all()) and bool((u0 == 3.0).all())


def test_projection_argument_errors(torch):
    mask, _ = inputs.spheres_3d(8, 0.5, 2.0, 3.0, seed=1)
    inv = lbm.Invariants(mask, 19)
    r = torch.ones(mask.shape, dtype=torch.float64, device="cuda")
    u = torch.zeros((3,) + mask.shape, dtype=torch.float64, device="cuda")
    for kw in (dict(iterations=0), dict(iterations=1001), dict(rho0=0.0)):
        with pytest.raises(lbm.LbmError) as e:
            inv.project(r, u, **kw)
        assert e.value.code == lbm.LBM_ERR_ARG


@pytest.mark.parametrize("name,q,mask,periodic", _cases(), ids=[c[0] for c in _cases()])
def test_device_components_match_oracle(torch, name, q, mask, periodic):
    """lbm_components_device: the oracle's labels (first-appearance numbering)
    bit for bit, for every link set (all links and each axis alone)."""
    solid = torch.from_numpy(np.ascontiguousarray(mask.astype(np.uint8))).cuda()
    for axis in range(-1, 2 if q == 9 else 3):
        lab, count = lbm.components_device(solid, q, axis, periodic)
        want, wcount = invariants.components(mask, q, axis, periodic)
        print(name, "axis", axis, "components", count, flush=True)
        assert count == wcount
        assert np.array_equal(lab.cpu().numpy(), want)


def test_device_components_large_packing(torch):
    """A 128^3 packing with many pores: device labels equal the host's."""
    mask, _ = inputs.spheres_3d(128, 0.3, 2.0, 6.0, seed=12)
    lab_h, count_h = lbm.components(mask, 19, -1, 7)
    solid = torch.from_numpy(np.ascontiguousarray(mask.astype(np.uint8))).cuda()
    for _ in range(2):  # scratch reuse across calls
        lab, count = lbm.components_device(solid, 19, -1, 7)
        assert count == count_h and np.array_equal(lab.cpu().numpy(), lab_h)
    print("128^3 packing components", count_h, flush=True)


def test_device_invariants_project_like_host(torch):
    """Invariants built from a device mask carry the host mask's labels bit
    for bit, and project to the oracle's fields within the bars above (the
    per-component sums are FP64 atomics in no fixed order, so two
    projections agree only to rounding)."""
    mask, _ = inputs.spheres_3d(24, 0.5, 2.0, 4.0, seed=4)
    rho, u = _fields("device", 19, mask)
    ref_r, ref_u = invariants.project(mask, rho, u, 19, rho0=1.0, periodic=7, iterations=8)
    fl = ~mask
    labels = []
    for src in (mask, torch.from_numpy(np.ascontiguousarray(mask.astype(np.uint8))).cuda()):
        inv = lbm.Invariants(src, 19)
        labels.append((inv.labels.cpu().numpy(), inv.count))
        r_d, u_d = torch.from_numpy(rho.copy()).cuda(), torch.from_numpy(u.copy()).cuda()
        inv.project(r_d, u_d, rho0=1.0, iterations=8)
        r_h, u_h = r_d.cpu().numpy(), u_d.cpu().numpy()
        assert np.abs(r_h[fl] - ref_r[fl]).max() <= 1e-13
        assert np.abs(u_h[:, fl] - ref_u[:, fl]).max() <= 1e-14 * np.abs(ref_u[:, fl]).max()
    assert labels[0][1] == labels[1][1] and np.array_equal(labels[0][0], labels[1][0])
