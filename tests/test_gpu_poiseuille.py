"""Channel flow on the GPU against the exact discrete Poiseuille profile.

Between half-way bounce-back walls with Guo forcing, the steady velocity of
the fluid rows j = 1..N is u_j = g/(2 nu)(N^2/4 - y_j^2) + g(16 lam^2 - 3)/(8 lam),
y_j = j - (N+1)/2, lam = tau - 1/2, nu = lam/3: the closed form that pins the
oracle (tests/test_oracle_pins.py).  Here the GPU step reaches it: the 64x64
D2Q9 channel without discs (16x16 tiles, generic kernel) and a D3Q19 channel
on the scalar-mask kernel, both run with captured graphs; the FP32 offset
form within the bar of the FP32 form.
"""
import numpy as np
import pytest

from paper_1703_08015_amd import inputs, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _closed_form(N, tau, g):
    lam = tau - 0.5
    y = np.arange(1, N + 1) - (N + 1) / 2.0
    return g / (2 * lam / 3.0) * (N * N / 4.0 - y * y) + g * (16 * lam * lam - 3) / (8 * lam)


def _profile(u, N):
    """Mean u_x over each fluid row y = 1..N (the profile is uniform along x and z)."""
    ux = u[0]
    return np.array([ux[:, j, :].mean() for j in range(1, N + 1)]), ux


@pytest.mark.parametrize("tau", [0.8, 0.6])
def test_d2q9_channel_64(torch, tau):
    mask, _ = inputs.channel_2d(64, 64, discs=False, seed=0)
    N, g = 62, 1e-6
    s = lbm.Solver(lbm.Tiles(mask, (16, 16, 1), (1, 0, 0)), lattice=9, tau=tau, g=(g, 0, 0), graph_steps=2000)
    s.init()
    steps, res = s.run_to_steady(tol=1e-13, check_every=2000, max_steps=600_000)
    assert steps[0] > 0, "did not reach the residual"
    _, u = [x.cpu().numpy() for x in s.moments()]
    prof, ux = _profile(u, N)
    want = _closed_form(N, tau, g)
    assert np.max(np.abs(prof - want)) <= 1e-9 * want.max()
    # uniform along the channel, no transverse flow
    assert np.max(np.abs(ux[:, 1:N + 1, :] - prof[None, :, None])) <= 1e-12 * want.max()
    assert np.max(np.abs(u[1])) <= 1e-12 * want.max()


# FP32 offsets: the bar of the FP32 form (velocity within 1e-3 of the FP64 answer); measured 5.1e-5, the
# rounding floor of FP32 offsets at g = 1e-6
@pytest.mark.parametrize("storage,tol", [("f64", 1e-9), ("f32", 1e-3)])
def test_d3q19_channel_scalar_kernel(torch, storage, tol):
    N, tau, g = 32, 0.8, 1e-6
    mask = np.zeros((8, N + 2, 8), bool)
    mask[:, 0, :] = True
    mask[:, N + 1, :] = True
    s = lbm.Solver(lbm.Tiles(mask, (4, 4, 4), (1, 0, 1)), lattice=19, tau=tau, g=(g, 0, 0), storage=storage,
                   graph_steps=1000, step_kernel="scalar")
    s.init()
    s.step(40_000)  # about 38 e-folds of the slowest mode, N^2 / (pi^2 nu) steps each
    _, u = [x.cpu().numpy() for x in s.moments()]
    prof, _ = _profile(u, N)
    want = _closed_form(N, tau, g)
    err = np.max(np.abs(prof - want)) / want.max()
    print("D3Q19 channel", storage, "max error relative to u_max:", err)
    assert err <= tol
