"""Pins of the oracle's incompressible BGK model, Eqs. (4) and (6), against
facts the mathematics fixes (no GPU involved).

The model differs from the quasi-compressible one only in where the density
enters: the equilibrium is rho w_i plus a velocity polynomial with no density
factor, the velocity is the first moment itself (reference density 1), and
the Guo force density is g.  The tests below are chosen so that a density
factor left in any of these places, a dropped half-force shift or a wrong
coefficient fails one of them:

* moment identities of the equilibrium and of the source term (rho != 1);
* exact reduction to the quasi-compressible collision at unit density;
* exact linear shift: adding s w_i to every PDF adds s w_i to the result after
  any number of steps (the dynamics see the density only through its
  gradients); the quasi-compressible model breaks this, which the test checks
  too, so it discriminates;
* total momentum grows by g per fluid node per step (not rho g);
* the exact discrete Poiseuille profile at reference densities 1 and 1.3;
* the shear-wave decay rate nu k^2.
"""
import math

import numpy as np
import pytest

from oracle import dense
from paper_1703_08015_amd import inputs

INC, QC = dense.INCOMPRESSIBLE, dense.QUASI


@pytest.fixture(scope="module", autouse=True)
def _built():
    dense.build()


def _dims(q):
    return 2 if q == 9 else 3


def _vec(rng, d, lo, hi):
    v = np.zeros(3)
    v[:d] = rng.uniform(lo, hi, d)
    return v


@pytest.mark.parametrize("q", [9, 19])
def test_equilibrium_moments(q):
    """Eq. (4): sum f_eq = rho, sum c f_eq = u, sum cc f_eq = rho/3 I + u u."""
    c, w, _ = dense.lattice(q)
    d = _dims(q)
    rng = np.random.default_rng(21)
    for _ in range(20):
        rho = rng.uniform(0.5, 1.5)
        u = _vec(rng, d, -0.1, 0.1)
        fe = dense.feq(q, rho, u, model=INC)
        assert math.isclose(math.fsum(fe), rho, rel_tol=1e-15)
        for a in range(d):
            assert math.isclose(math.fsum(fe * c[:, a]), u[a], rel_tol=1e-14, abs_tol=1e-17)
            for b in range(d):
                want = rho * (a == b) / 3.0 + u[a] * u[b]
                assert math.isclose(math.fsum(fe * c[:, a] * c[:, b]), want, rel_tol=1e-14, abs_tol=1e-16)
        # the velocity-independent part is rho w_i, as in Eq. (3) at u = 0
        assert np.array_equal(dense.feq(q, rho, np.zeros(3), model=INC), rho * w)


@pytest.mark.parametrize("q", [9, 19])
def test_guo_moments(q):
    """Source with force density g: sum F = 0, sum c F = g, sum cc F = u g + g u,
    whatever rho is."""
    c, w, _ = dense.lattice(q)
    d = _dims(q)
    rng = np.random.default_rng(22)
    for _ in range(20):
        rho = rng.uniform(0.5, 1.5)
        u = _vec(rng, d, -0.1, 0.1)
        g = _vec(rng, d, -1e-3, 1e-3)
        F = dense.guo(q, rho, u, g, model=INC)
        assert abs(math.fsum(F)) < 1e-18
        for a in range(d):
            assert math.isclose(math.fsum(F * c[:, a]), g[a], rel_tol=1e-13, abs_tol=1e-19)
            for b in range(d):
                want = u[a] * g[b] + g[a] * u[b]
                assert math.isclose(math.fsum(F * c[:, a] * c[:, b]), want, rel_tol=1e-12, abs_tol=1e-19)
        assert np.array_equal(F, dense.guo(q, 1.0, u, g, model=QC))


@pytest.mark.parametrize("q", [9, 19])
def test_collision_adds_g_and_keeps_equilibrium(q):
    """One collision: mass unchanged, first moment gains g; at g = 0 the
    equilibrium of any (rho, u) is a fixed point."""
    c, w, _ = dense.lattice(q)
    d = _dims(q)
    rng = np.random.default_rng(23)
    for tau in (0.51, 0.7, 1.0, 1.9):
        f = w * rng.uniform(0.8, 1.4, q)
        g = _vec(rng, d, -1e-4, 1e-4)
        out = dense.collide(q, f, tau, g, model=INC)
        assert math.isclose(math.fsum(out), math.fsum(f), rel_tol=1e-15)
        for a in range(d):
            assert math.isclose(math.fsum(out * c[:, a]), math.fsum(f * c[:, a]) + g[a],
                                rel_tol=1e-12, abs_tol=1e-17)
        u = _vec(rng, d, -0.05, 0.05)
        fe = dense.feq(q, 1.3, u, model=INC)
        assert np.allclose(dense.collide(q, fe, tau, np.zeros(3), model=INC), fe, rtol=1e-15, atol=0)


@pytest.mark.parametrize("q", [9, 19])
def test_reduces_to_quasi_compressible_at_unit_density(q):
    """At rho = 1 Eqs. (4) and (6) are Eqs. (3) and (5): equilibria and source
    agree exactly, and so does a collision of a state whose sum is 1."""
    c, w, _ = dense.lattice(q)
    d = _dims(q)
    rng = np.random.default_rng(24)
    for _ in range(10):
        u = _vec(rng, d, -0.1, 0.1)
        g = _vec(rng, d, -1e-3, 1e-3)
        assert np.allclose(dense.feq(q, 1.0, u, model=INC), dense.feq(q, 1.0, u, model=QC), rtol=1e-15, atol=1e-17)
        assert np.array_equal(dense.guo(q, 1.0, u, g, model=INC), dense.guo(q, 1.0, u, g, model=QC))
        # w_i + a zero-sum perturbation: rho = 1 to rounding
        p = rng.uniform(-1e-3, 1e-3, q)
        p -= p.mean()
        f = w + p * w
        f[0] += 1.0 - math.fsum(f)
        a = dense.collide(q, f, 0.8, g, model=INC)
        b = dense.collide(q, f, 0.8, g, model=QC)
        assert np.max(np.abs(a - b)) < 1e-15


def _sphere_mask(n=12):
    m, _ = inputs.spheres_3d(n, 0.6, rmin=2, rmax=4, seed=27)
    return m


def _disc_mask():
    m, _ = inputs.channel_2d(32, 32, porosity=0.7, seed=25)
    return m


@pytest.mark.parametrize("q", [9, 19])
def test_uniform_density_shift_is_carried_exactly(q):
    """Linearity in the density: f(t; f0 + s w) = f(t; f0) + s w on every
    fluid node, for any geometry and force -- the incompressible dynamics see
    rho only through its gradients, and bounce-back maps s w_i onto itself.
    The quasi-compressible model does not have this property (u = j/rho)."""
    mask = _disc_mask() if q == 9 else _sphere_mask()
    per = (1, 0, 0) if q == 9 else 7
    c, w, _ = dense.lattice(q)
    fl = ~mask
    f0 = inputs.random_pdfs(q, mask, seed=26, lo=0.02, hi=0.06)
    g = np.array([2e-5, -1e-5, 0.0 if q == 9 else 1e-5])
    s = 0.37
    shift = np.zeros_like(f0)
    shift[:, fl] = (s * w)[:, None]
    gaps = {}
    for model in (INC, QC):
        a = dense.step(q, mask, f0, 0.75, g, 6, periodic=per, model=model)
        b = dense.step(q, mask, f0 + shift, 0.75, g, 6, periodic=per, model=model)
        gaps[model] = np.max(np.abs((b - a - shift)[:, fl]))
    assert gaps[INC] < 1e-14
    assert gaps[QC] > 1e-6


@pytest.mark.parametrize("q", [9, 19])
def test_momentum_grows_by_nodes_times_g(q):
    """Fully periodic, no solids: the total of u (the momentum at reference
    density 1) grows by N g per step, N the number of nodes, whatever rho is."""
    shape = (1, 16, 12) if q == 9 else (6, 8, 10)
    mask = np.zeros(shape, bool)
    rho, u = inputs.random_macro(mask, seed=28)
    rho = rho + 0.4
    if q == 9:
        u[2] = 0.0
    g = np.array([3e-5, -1e-5, 0.0 if q == 9 else 2e-5])
    f = dense.init(q, mask, rho=rho, u=u, model=INC)
    r0, u0 = dense.moments(q, mask, f, g, model=INC)
    # the stored state at t = 0 is f_eq(rho, u): its moments read rho and u - g/2
    assert np.allclose(r0, rho, rtol=1e-15, atol=0)
    assert np.allclose(u0, u - 0.5 * g[:, None, None, None], rtol=0, atol=1e-16)
    N = mask.size
    M = math.fsum(r0.ravel())
    P0 = np.array([math.fsum(u0[a].ravel()) for a in range(3)])
    t = 7
    f = dense.step(q, mask, f, 0.9, g, t, periodic=7, model=INC)
    r1, u1 = dense.moments(q, mask, f, g, model=INC)
    P1 = np.array([math.fsum(u1[a].ravel()) for a in range(3)])
    assert math.isclose(math.fsum(r1.ravel()), M, rel_tol=1e-14)
    assert np.allclose(P1, P0 + t * N * g, rtol=0, atol=1e-13 * N)


def _steady_channel(q, N, tau, g, rho0, tol=2e-11, chunk=2000, max_steps=400000):
    ny = N + 2
    shape = (1, ny, 2) if q == 9 else (2, ny, 2)
    mask = np.zeros(shape, bool)
    mask[:, 0, :] = True
    mask[:, ny - 1, :] = True
    periodic = (1, 0, 0) if q == 9 else (1, 0, 1)
    f = dense.init(q, mask, rho0=rho0, model=INC)
    gv = np.array([g, 0.0, 0.0])
    prev = None
    for _ in range(max_steps // chunk):
        f = dense.step(q, mask, f, tau, gv, chunk, periodic=periodic, model=INC)
        rho, u = dense.moments(q, mask, f, gv, model=INC)
        ux = u[0, 0, 1:N + 1, 0]
        if prev is not None and np.max(np.abs(ux - prev)) <= tol * np.max(np.abs(ux)):
            return ux, rho[~mask]
        prev = ux
    raise AssertionError("channel did not reach steady state")


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("tau,rho0", [(0.8, 1.0), (0.5 + math.sqrt(3) / 4, 1.3), (0.6, 1.3)])
def test_poiseuille_exact_discrete_profile(q, tau, rho0):
    """Steady channel flow equals the exact discrete solution of half-way
    bounce-back with Guo forcing, u_j = g/(2 nu)(N^2/4 - y_j^2) + g(16 lam^2 - 3)/(8 lam),
    lam = tau - 1/2, nu = lam/3: the incompressible state at uniform density
    rho0 is the unit-density state plus (rho0 - 1) w_i, so the profile does
    not depend on rho0, and the density stays uniform."""
    N, g = 12, 1e-6
    ux, rho = _steady_channel(q, N, tau, g, rho0)
    lam = tau - 0.5
    y = np.arange(1, N + 1) - (N + 1) / 2.0
    want = g / (2 * lam / 3.0) * (N * N / 4.0 - y * y) + g * (16 * lam * lam - 3) / (8 * lam)
    assert np.max(np.abs(ux - want)) <= 1e-10 * np.max(np.abs(want))
    # uniform density; its mean moves only by accumulated rounding over ~1e5 steps
    assert np.ptp(rho) < 1e-14
    assert abs(rho.mean() - rho0) < 1e-11


@pytest.mark.parametrize("q", [9, 19])
def test_shear_wave_decay_rate(q):
    """Fully periodic, g = 0, u_x = U sin(k y) at reference density 1.3: the
    amplitude decays at nu k^2 (nu = (tau - 1/2)/3), approached as O(k^2)."""
    tau, U, rho0 = 0.8, 1e-4, 1.3
    nu = (tau - 0.5) / 3
    devs = []
    for L in (16, 32):
        shape = (1, L, 2) if q == 9 else (2, L, 2)
        mask = np.zeros(shape, bool)
        y = np.arange(L)
        k = 2 * math.pi / L
        u = np.zeros((3,) + shape)
        u[0] = U * np.sin(k * y)[None, :, None]
        f = dense.init(q, mask, rho=np.full(shape, rho0), u=u, model=INC)
        t1, t2 = int(0.2 / (nu * k * k)), int(0.7 / (nu * k * k))
        amps = []
        f = dense.step(q, mask, f, tau, [0, 0, 0], t1, periodic=7, model=INC)
        amps.append(np.dot(dense.moments(q, mask, f, [0, 0, 0], model=INC)[1][0, 0, :, 0], np.sin(k * y)) * 2 / L)
        f = dense.step(q, mask, f, tau, [0, 0, 0], t2 - t1, periodic=7, model=INC)
        amps.append(np.dot(dense.moments(q, mask, f, [0, 0, 0], model=INC)[1][0, 0, :, 0], np.sin(k * y)) * 2 / L)
        devs.append(abs(math.log(amps[0] / amps[1]) / (t2 - t1) / (nu * k * k) - 1))
    assert devs[1] < 0.01
    assert devs[1] < devs[0] / 3


def test_unknown_model_is_rejected():
    with pytest.raises(ValueError):
        dense.feq(19, 1.0, np.zeros(3), model=2)
