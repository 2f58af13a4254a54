"""Pins of the oracle's moving wall (the lid of a driven cavity), on the CPU.

* Plane Couette flow between a fixed wall and the moving lid: with half-way
  bounce-back both walls sit half a node beyond the last fluid rows, and the
  exact discrete steady state is the linear profile u_x = U (j + 1/2) / N, for
  BGK at any tau and for MRT with the even moments at 1/tau and any odd rates
  (no force, so no slip term), with uniform density; the same mirrored for a
  lid on the other face.  Unequal even rates leave it off the line by O(U^2).
* A tangential lid adds equal and opposite terms on the two diagonal links
  of every lid node, so a closed cavity keeps its mass to rounding while it
  gains momentum in the lid's direction.
A wrong sign, weight or face fails the profile.
"""
import math

import numpy as np
import pytest

from oracle import dense


@pytest.fixture(scope="module", autouse=True)
def _built():
    dense.build()


def _couette(q, N, tau, U, side, model=dense.QUASI, mrt=None, rho0=1.0):
    """Run to steady state: 40 decay times of the slowest shear mode."""
    shape = (1, N, 2) if q == 9 else (2, N, 2)
    mask = np.zeros(shape, bool)
    per = (1, 0, 0) if q == 9 else (1, 0, 1)
    f = dense.init(q, mask, rho0=rho0, model=model)
    rho_w = rho0 if model == dense.QUASI else 1.0
    lid = (1, side, (U, 0.0, 0.0), rho_w)
    nu = (tau - 0.5) / 3
    steps = int(40 * N * N / (math.pi ** 2 * nu))
    f = dense.step(q, mask, f, tau, [0, 0, 0], steps, periodic=per, model=model, mrt=mrt, lid=lid)
    rho, u = dense.moments(q, mask, f, [0, 0, 0], model=model)
    return u[0, 0, :, 0], rho, u


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_couette_profile_is_exact(q, tau):
    N, U = 10, 1e-3
    ux, rho, u = _couette(q, N, tau, U, side=1)
    j = np.arange(N)
    assert np.max(np.abs(ux - U * (j + 0.5) / N)) <= 1e-10 * U
    assert np.max(np.abs(u[1])) <= 1e-10 * U and np.ptp(rho) <= 1e-13


@pytest.mark.parametrize("q", [9, 19])
def test_couette_lid_on_the_low_face_and_other_collisions(q):
    N, U = 8, -2e-3
    j = np.arange(N)
    ux, _, _ = _couette(q, N, 0.8, U, side=0)
    assert np.max(np.abs(ux - U * (N - j - 0.5) / N)) <= 1e-10 * abs(U)
    # two relaxation times (even moments at 1/tau, odd ones free): exact
    ux, _, _ = _couette(q, N, 0.8, U, side=1, mrt=[1.25, 1.25, 1.6, 1.25, 1.6])
    assert np.max(np.abs(ux - U * (j + 0.5) / N)) <= 1e-10 * abs(U)
    # unequal even rates: off the line by O(U^2) relative (measured 1.1e-9 here), shrinking 4x per halving of U
    devs = []
    for uu in (U, U / 2):
        ux, _, _ = _couette(q, N, 0.8, uu, side=1, mrt=[1.3, 1.1, 1.5, 1.7, 1.2])
        devs.append(np.max(np.abs(ux - uu * (j + 0.5) / N)) / abs(uu))
    assert devs[0] < 1e-8 and 3.5 < devs[0] / devs[1] < 4.5
    ux, _, _ = _couette(q, N, 0.8, U, side=1, model=dense.INCOMPRESSIBLE, rho0=1.3)
    assert np.max(np.abs(ux - U * (j + 0.5) / N)) <= 1e-10 * abs(U)


@pytest.mark.parametrize("q", [9, 19])
def test_closed_cavity_keeps_mass_and_gains_momentum(q):
    n = 12
    shape = (1, n, n) if q == 9 else (n, n, n)
    mask = np.zeros(shape, bool)
    f = dense.init(q, mask)
    m0 = math.fsum(f.ravel())
    U = 0.05
    f = dense.step(q, mask, f, 0.6, [0, 0, 0], 300, periodic=0, lid=(1, 1, (U, 0.0, 0.0), 1.0))
    rho, u = dense.moments(q, mask, f, [0, 0, 0])
    assert abs(math.fsum(f.ravel()) - m0) <= 1e-13 * m0
    px = math.fsum((rho * u[0]).ravel())
    assert px > 0  # dragged along +x by the lid
    # the top row moves with the lid, the bottom row much less
    assert u[0][..., n - 1, :].mean() > 5 * abs(u[0][..., 0, :].mean())


def test_lid_needs_a_non_periodic_axis():
    mask = np.zeros((1, 8, 8), bool)
    with pytest.raises(ValueError):
        dense.step(9, mask, dense.init(9, mask), 0.8, [0, 0, 0], 1, periodic=(1, 1, 0), lid=(1, 1, (1e-3, 0, 0), 1.0))
