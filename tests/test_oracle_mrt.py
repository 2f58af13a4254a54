"""Pins of the oracle's MRT collision (Eq. 8), on the CPU.

The paper does not print its MRT matrix; the oracle uses the published
orthogonal bases (Lallemand & Luo 2000 for D2Q9, d'Humieres et al. 2002 for
D3Q19).  Pinned by facts independent of how the oracle builds them:

* rows orthogonal, with the published squared norms;
* M f_eq equals the published closed-form equilibrium moments (both fluid
  models);
* every rate equal to 1/tau gives the BGK collision;
* mass is conserved and momentum gains the force density, whatever the rates;
* shear waves decay at nu k^2 with nu from tau alone;
* channel flow: the exact discrete profile of bounce-back walls with an odd
  rate set through Lambda = (1/s_nu - 1/2)(1/s_odd - 1/2), a parabola with slip
  g (16 Lambda - 3) / (24 nu), zero at Lambda = 3/16, for arbitrary even rates.
A wrong row, class or rate assignment fails one of these.
"""
import math

import numpy as np
import pytest

from oracle import dense

INC, QC = dense.INCOMPRESSIBLE, dense.QUASI
RATES = [1.19, 1.4, 1.2, 1.4, 1.98]  # s_e, s_eps, s_q, s_pi, s_m (the published D3Q19 set)


@pytest.fixture(scope="module", autouse=True)
def _built():
    dense.build()


def test_bases_are_orthogonal_with_published_norms():
    norms = {9: [9, 36, 36, 6, 12, 6, 12, 4, 4],
             19: [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]}
    for q in (9, 19):
        M, cls = dense.mrt_matrix(q)
        G = M @ M.T
        assert np.array_equal(G, np.diag(norms[q]).astype(float))
        assert np.array_equal(M, np.round(M))  # integer entries
        c, _, _ = dense.lattice(q)
        # density and momentum rows are 1 and the velocity components
        cons = [k for k in range(q) if dense.MRT_CLASSES[cls[k]] == "conserved"]
        rows = {tuple(M[k]) for k in cons}
        assert rows == {tuple(np.ones(q))} | {tuple(c[:, a].astype(float)) for a in range(2 if q == 9 else 3)}
        # five shear-stress rows in 3D (two in 2D), all second order in c
        nu = [k for k in range(q) if dense.MRT_CLASSES[cls[k]] == "nu"]
        assert len(nu) == (2 if q == 9 else 5)


def test_every_moment_is_even_or_odd_in_c():
    """Each row of both bases takes equal values on opposite velocities (even moments: density, energies, stresses)
    or opposite values (odd: momentum, heat fluxes, third-order terms), and the odd rows vanish on the rest
    direction; so M f splits into pair sums and differences."""
    for q in (9, 19):
        M, _ = dense.mrt_matrix(q)
        _, _, opp = dense.lattice(q)
        even = [np.array_equal(M[k], M[k][opp]) for k in range(q)]
        odd = [np.array_equal(M[k], -M[k][opp]) for k in range(q)]
        assert all(e != o for e, o in zip(even, odd))
        assert sum(odd) == (4 if q == 9 else 9)  # j and q along each axis, plus the three m rows in 3D
        assert all(M[k][0] == 0 for k in range(q) if odd[k])
        # the pair form reproduces M f
        rng = np.random.default_rng(q)
        f = rng.random(q)
        pairs = [i for i in range(1, q) if i < opp[i]]
        s, d = f[pairs] + f[opp[pairs]], f[pairs] - f[opp[pairs]]
        mf = np.array([(M[k][0] * f[0] if even[k] else 0.0) + M[k][pairs] @ (s if even[k] else d) for k in range(q)])
        assert np.allclose(mf, M @ f, rtol=1e-14, atol=1e-14)


def _published_eq(q, rho, u, d):
    """Closed-form equilibrium moments of the two bases, with d the density of
    the velocity terms (rho or 1)."""
    ux, uy, uz = u
    uu = ux * ux + uy * uy + uz * uz
    if q == 9:
        return np.array([rho, -2 * rho + 3 * d * uu, rho - 3 * d * uu, d * ux, -d * ux, d * uy, -d * uy,
                         d * (ux * ux - uy * uy), d * ux * uy])
    pxx = d * (3 * ux * ux - uu)
    pww = d * (uy * uy - uz * uz)
    return np.array([rho, -11 * rho + 19 * d * uu, 3 * rho - 5.5 * d * uu, d * ux, -2 / 3 * d * ux, d * uy,
                     -2 / 3 * d * uy, d * uz, -2 / 3 * d * uz, pxx, -0.5 * pxx, pww, -0.5 * pww, d * ux * uy,
                     d * uy * uz, d * ux * uz, 0.0, 0.0, 0.0])


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("model", [QC, INC])
def test_equilibrium_moments_are_the_published_ones(q, model):
    M, _ = dense.mrt_matrix(q)
    rng = np.random.default_rng(71)
    for _ in range(10):
        rho = rng.uniform(0.6, 1.4)
        u = np.zeros(3)
        u[:2 if q == 9 else 3] = rng.uniform(-0.1, 0.1, 2 if q == 9 else 3)
        m = M @ dense.feq(q, rho, u, model=model)
        want = _published_eq(q, rho, u, rho if model == QC else 1.0)
        assert np.allclose(m, want, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("model", [QC, INC])
def test_equal_rates_give_bgk(q, model):
    _, w, _ = dense.lattice(q)
    rng = np.random.default_rng(72)
    for tau in (0.55, 0.8, 1.7):
        f = w * rng.uniform(0.8, 1.3, q)
        g = rng.uniform(-1e-4, 1e-4, 3)
        if q == 9:
            g[2] = 0.0
        s = 1.0 / tau
        a = dense.collide(q, f, tau, g, model=model, mrt=[s] * 5)
        b = dense.collide(q, f, tau, g, model=model)
        assert np.max(np.abs(a - b)) < 1e-15


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("model", [QC, INC])
def test_collision_conserves_mass_and_adds_force(q, model):
    c, w, _ = dense.lattice(q)
    rng = np.random.default_rng(73)
    for _ in range(5):
        f = w * rng.uniform(0.8, 1.3, q)
        g = rng.uniform(-1e-4, 1e-4, 3)
        if q == 9:
            g[2] = 0.0
        rates = rng.uniform(0.6, 1.9, 5)
        out = dense.collide(q, f, 0.7, g, model=model, mrt=rates)
        rho = math.fsum(f)
        d = rho if model == QC else 1.0
        assert math.isclose(math.fsum(out), rho, rel_tol=1e-15)
        for a in range(3):
            assert math.isclose(math.fsum(out * c[:, a]), math.fsum(f * c[:, a]) + d * g[a], rel_tol=1e-12,
                                abs_tol=1e-17)
        # an equilibrium is a fixed point without force
        u = np.zeros(3)
        u[:2] = rng.uniform(-0.05, 0.05, 2)
        fe = dense.feq(q, 1.2, u, model=model)
        assert np.allclose(dense.collide(q, fe, 0.7, np.zeros(3), model=model, mrt=rates), fe, rtol=1e-14, atol=0)


@pytest.mark.parametrize("q", [9, 19])
def test_shear_wave_decays_with_tau_only(q):
    tau, U = 0.8, 1e-4
    nu = (tau - 0.5) / 3
    devs = []
    for L in (16, 32):
        shape = (1, L, 2) if q == 9 else (2, L, 2)
        mask = np.zeros(shape, bool)
        y = np.arange(L)
        k = 2 * math.pi / L
        u = np.zeros((3,) + shape)
        u[0] = U * np.sin(k * y)[None, :, None]
        f = dense.init(q, mask, rho=np.ones(shape), u=u)
        t1, t2 = int(0.2 / (nu * k * k)), int(0.7 / (nu * k * k))
        amps = []
        for n in (t1, t2 - t1):
            f = dense.step(q, mask, f, tau, [0, 0, 0], n, periodic=7, mrt=[1.5, 1.1, 1.3, 0.9, 1.7])
            amps.append(np.dot(dense.moments(q, mask, f, [0, 0, 0])[1][0, 0, :, 0], np.sin(k * y)) * 2 / L)
        devs.append(abs(math.log(amps[0] / amps[1]) / (t2 - t1) / (nu * k * k) - 1))
    assert devs[1] < 0.01
    assert devs[1] < devs[0] / 3


def _steady_channel(q, N, tau, g, mrt, tol=2e-11, chunk=2000, max_steps=600000):
    ny = N + 2
    shape = (1, ny, 2) if q == 9 else (2, ny, 2)
    mask = np.zeros(shape, bool)
    mask[:, 0, :] = True
    mask[:, ny - 1, :] = True
    per = (1, 0, 0) if q == 9 else (1, 0, 1)
    f = dense.init(q, mask)
    gv = np.array([g, 0.0, 0.0])
    prev = None
    for _ in range(max_steps // chunk):
        f = dense.step(q, mask, f, tau, gv, chunk, periodic=per, mrt=mrt)
        _, u = dense.moments(q, mask, f, gv)
        ux = u[0, 0, 1:N + 1, 0]
        if prev is not None and np.max(np.abs(ux - prev)) <= tol * np.max(np.abs(ux)):
            return ux
        prev = ux
    raise AssertionError("channel did not reach steady state")


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("tau,lam", [(0.8, 3 / 16), (1.4, 3 / 16), (0.8, 0.3)])
def test_poiseuille_depends_on_lambda_only(q, tau, lam):
    """Odd rates s_q = s_m = 1/(Lambda/(tau - 1/2) + 1/2), even rates unrelated
    to tau: u_j = g/(2 nu)(N^2/4 - y_j^2) + g(16 Lambda - 3)/(24 nu)."""
    N, g = 12, 1e-6
    lp = tau - 0.5
    s_odd = 1.0 / (lam / lp + 0.5)
    ux = _steady_channel(q, N, tau, g, [1.3, 1.1, s_odd, 1.7, s_odd])
    nu = lp / 3
    y = np.arange(1, N + 1) - (N + 1) / 2.0
    want = g / (2 * nu) * (N * N / 4.0 - y * y) + g * (16 * lam - 3) / (24 * nu)
    assert np.max(np.abs(ux - want)) <= 1e-8 * np.max(np.abs(want))
