"""Pins of the FP64 dense oracle against facts fixed by the paper and by the
mathematics of the lattice Boltzmann method (no GPU involved).

Each test targets a mistake that could hide in the oracle: a wrong weight or
velocity (isotropy sums), a wrong equilibrium coefficient (moment identities),
a wrong forcing term (Guo moments), a wrong propagation or bounce-back
(library np.roll, permutation structure, exact discrete Poiseuille profile),
and a wrong viscosity (shear-wave decay, second-order convergence).
"""
import math

import numpy as np
import pytest

from oracle import dense
from paper_1703_08015_amd import inputs


@pytest.fixture(scope="module", autouse=True)
def _built():
    dense.build()


def _dims(q):
    return 2 if q == 9 else 3


@pytest.mark.parametrize("q", [9, 19])
def test_lattice_isotropy(q):
    """Velocity set + weights: the moment sums of an isotropic lattice
    (sum w = 1, odd moments 0, second moment delta/3, fourth moment
    (dd + dd + dd)/9) -- these fix the weights uniquely for the set."""
    c, w, opp = dense.lattice(q)
    d = _dims(q)
    assert len(set(map(tuple, c))) == q
    assert np.all(np.abs(c) <= 1) and np.all(c[:, d:] == 0)
    assert np.all(w > 0)
    assert math.isclose(math.fsum(w), 1.0, rel_tol=0, abs_tol=1e-15)
    cf = c[:, :d].astype(float)
    for a in range(d):
        assert abs(np.dot(w, cf[:, a])) < 1e-16
        for b in range(d):
            assert math.isclose(np.dot(w, cf[:, a] * cf[:, b]), (a == b) / 3.0, abs_tol=1e-15)
            for g in range(d):
                assert abs(np.dot(w, cf[:, a] * cf[:, b] * cf[:, g])) < 1e-16
                for e in range(d):
                    want = ((a == b) * (g == e) + (a == g) * (b == e) + (a == e) * (b == g)) / 9.0
                    got = np.dot(w, cf[:, a] * cf[:, b] * cf[:, g] * cf[:, e])
                    assert math.isclose(got, want, abs_tol=1e-15)
    for i in range(q):
        assert np.array_equal(c[opp[i]], -c[i])
    assert c[0].tolist() == [0, 0, 0]
    # counts of face / edge directions quoted in Sec. 3.1.1.2 (q_s, q_d)
    nz = (np.abs(c).sum(axis=1))
    assert (nz == 1).sum() == (4 if q == 9 else 6)
    assert (nz == 2).sum() == (4 if q == 9 else 12)


@pytest.mark.parametrize("q", [9, 19])
def test_equilibrium_moments(q):
    """Eq. (3): sum f_eq = rho, sum c f_eq = rho u, sum cc f_eq = rho/3 I + rho u u."""
    c, w, _ = dense.lattice(q)
    d = _dims(q)
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.5, 1.5)
        u = np.zeros(3)
        u[:d] = rng.uniform(-0.1, 0.1, d)
        fe = dense.feq(q, rho, u)
        assert math.isclose(math.fsum(fe), rho, rel_tol=1e-15)
        for a in range(d):
            assert math.isclose(math.fsum(fe * c[:, a]), rho * u[a], abs_tol=1e-16)
            for b in range(d):
                want = rho * ((a == b) / 3.0 + u[a] * u[b])
                assert math.isclose(math.fsum(fe * c[:, a] * c[:, b]), want, rel_tol=1e-14, abs_tol=1e-16)


@pytest.mark.parametrize("q", [9, 19])
def test_guo_moments(q):
    """Guo source: sum F = 0, sum c F = rho g, sum cc F = rho (u g + g u)."""
    c, w, _ = dense.lattice(q)
    d = _dims(q)
    rng = np.random.default_rng(2)
    for _ in range(20):
        rho = rng.uniform(0.5, 1.5)
        u = np.zeros(3)
        g = np.zeros(3)
        u[:d] = rng.uniform(-0.1, 0.1, d)
        g[:d] = rng.uniform(-1e-3, 1e-3, d)
        F = dense.guo(q, rho, u, g)
        assert abs(math.fsum(F)) < 1e-18
        for a in range(d):
            assert math.isclose(math.fsum(F * c[:, a]), rho * g[a], rel_tol=1e-13, abs_tol=1e-19)
            for b in range(d):
                want = rho * (u[a] * g[b] + g[a] * u[b])
                assert math.isclose(math.fsum(F * c[:, a] * c[:, b]), want, rel_tol=1e-12, abs_tol=1e-19)


@pytest.mark.parametrize("q", [9, 19])
def test_collision_conserves_mass_and_adds_force(q):
    """Eqs. (2), (7) with forcing: mass is unchanged, first moment gains rho g,
    and the equilibrium is a fixed point when g = 0."""
    c, w, _ = dense.lattice(q)
    d = _dims(q)
    rng = np.random.default_rng(3)
    for tau in (0.51, 0.7, 1.0, 1.9):
        f = w * rng.uniform(0.8, 1.2, q)
        g = np.zeros(3)
        g[:d] = rng.uniform(-1e-4, 1e-4, d)
        out = dense.collide(q, f, tau, g)
        rho = math.fsum(f)
        assert math.isclose(math.fsum(out), rho, rel_tol=1e-15)
        for a in range(d):
            assert math.isclose(math.fsum(out * c[:, a]), math.fsum(f * c[:, a]) + rho * g[a],
                                rel_tol=1e-12, abs_tol=1e-17)
        u = np.zeros(3)
        u[:d] = rng.uniform(-0.05, 0.05, d)
        fe = dense.feq(q, 1.1, u)
        assert np.allclose(dense.collide(q, fe, tau, np.zeros(3)), fe, rtol=1e-15, atol=0)


def _disc_mask():
    m, _ = inputs.channel_2d(32, 32, porosity=0.7, seed=5)
    return m


def _sphere_mask(n=16):
    m, _ = inputs.spheres_3d(n, 0.6, rmin=2, rmax=4, seed=7)
    return m


@pytest.mark.parametrize("q", [9, 19])
def test_permutation_mode_periodic_is_roll(q):
    """tau = +inf, g = 0, no solids, all periodic: one step is a pure shift of
    each direction by c_i -- exactly numpy.roll."""
    shape = (1, 12, 10) if q == 9 else (6, 5, 4)
    mask = np.zeros(shape, bool)
    c, _, _ = dense.lattice(q)
    f = inputs.random_pdfs(q, mask, seed=11)
    out = dense.step(q, mask, f, math.inf, [0, 0, 0], 1, periodic=7)
    for i in range(q):
        want = np.roll(f[i], shift=(c[i][2], c[i][1], c[i][0]), axis=(0, 1, 2))
        assert np.array_equal(out[i], want)


@pytest.mark.parametrize("q", [9, 19])
def test_permutation_mode_with_solids_is_bijection(q):
    """With solids, pure streaming + bounce-back moves every stored fluid value
    to exactly one slot: the multiset of values is preserved exactly, and two
    steps with opposite... (values are unique, so equality of sorted arrays
    proves a permutation)."""
    mask = _disc_mask() if q == 9 else _sphere_mask()
    f = inputs.random_pdfs(q, mask, seed=12)
    fl = ~mask
    out = dense.step(q, mask, f, math.inf, [0, 0, 0], 3, periodic=(1, 0, 0) if q == 9 else 7)
    a = np.sort(f[:, fl].ravel())
    b = np.sort(out[:, fl].ravel())
    assert np.unique(a).size == a.size
    assert np.array_equal(a, b)


def test_bounce_back_single_obstacle():
    """A fluid node next to a lone solid node receives its own reversed value
    in the direction pointing away from the obstacle (half-way bounce-back)."""
    q = 19
    c, _, opp = dense.lattice(q)
    mask = np.zeros((5, 5, 5), bool)
    mask[2, 2, 2] = True
    f = inputs.random_pdfs(q, mask, seed=13)
    out = dense.step(q, mask, f, math.inf, [0, 0, 0], 1, periodic=7)
    for i in range(1, q):
        # node x whose source x - c_i is the solid node
        x = np.array([2, 2, 2]) + c[i]
        z, y, xx = x[2], x[1], x[0]
        assert out[i, z, y, xx] == f[opp[i], z, y, xx]


@pytest.mark.parametrize("q", [9, 19])
def test_first_step_from_rest(q):
    """From rest (f* = w_i everywhere) every fluid node of any geometry sees
    the uniform state after propagation, because bounce-back of w_i returns
    w_opp(i) = w_i; so after one step all fluid nodes hold the same values."""
    mask = _disc_mask() if q == 9 else _sphere_mask()
    c, w, _ = dense.lattice(q)
    g = np.array([1e-6, -2e-6, 0.0 if q == 9 else 3e-6])
    f0 = dense.init(q, mask)
    out = dense.step(q, mask, f0, 0.8, g, 1, periodic=(1, 0, 0) if q == 9 else 7)
    want = dense.collide(q, w, 0.8, g)
    fl = ~mask
    for i in range(q):
        assert np.all(out[i][fl] == want[i])
        assert np.all(f0[i][fl] == w[i])


@pytest.mark.parametrize("q", [9, 19])
def test_mass_conserved_each_step(q):
    mask = _disc_mask() if q == 9 else _sphere_mask()
    fl = ~mask
    f = inputs.random_pdfs(q, mask, seed=14, lo=0.02, hi=0.06)
    g = np.array([1e-5, 2e-5, 0.0 if q == 9 else -1e-5])
    m0 = math.fsum(f[:, fl].ravel())
    for _ in range(5):
        f = dense.step(q, mask, f, 0.7, g, 1, periodic=(1, 0, 0) if q == 9 else 7)
        m = math.fsum(f[:, fl].ravel())
        assert abs(m - m0) / m0 < 2 * q * 2.2e-16
        assert np.all(f[:, mask] == 0)


@pytest.mark.parametrize("q", [9, 19])
def test_momentum_grows_by_mass_times_g(q):
    """Fully periodic, no solids: total momentum P(t) = P(0) + t M g."""
    shape = (1, 16, 12) if q == 9 else (6, 8, 10)
    mask = np.zeros(shape, bool)
    rho, u = inputs.random_macro(mask, seed=15)
    if q == 9:
        u[2] = 0.0
    g = np.array([3e-5, -1e-5, 0.0 if q == 9 else 2e-5])
    f = dense.init(q, mask, rho=rho, u=u)
    r0, u0 = dense.moments(q, mask, f, g)
    M = math.fsum(r0.ravel())
    P0 = np.array([math.fsum((r0 * u0[a]).ravel()) for a in range(3)])
    t = 7
    f = dense.step(q, mask, f, 0.9, g, t, periodic=7)
    r1, u1 = dense.moments(q, mask, f, g)
    P1 = np.array([math.fsum((r1 * u1[a]).ravel()) for a in range(3)])
    assert math.isclose(math.fsum(r1.ravel()), M, rel_tol=1e-14)
    assert np.allclose(P1, P0 + t * M * g, rtol=0, atol=1e-13 * M)


def _channel(q, N, width=2):
    """Straight channel: solid rows y = 0 and y = N+1, fluid rows 1..N,
    periodic in x (and z for D3Q19)."""
    ny = N + 2
    shape = (1, ny, width) if q == 9 else (width, ny, width)
    mask = np.zeros(shape, bool)
    mask[:, 0, :] = True
    mask[:, ny - 1, :] = True
    periodic = (1, 0, 0) if q == 9 else (1, 0, 1)
    return mask, periodic


def _steady_channel(q, N, tau, g, tol=2e-11, chunk=2000, max_steps=400000):
    mask, periodic = _channel(q, N)
    f = dense.init(q, mask)
    gv = np.array([g, 0.0, 0.0])
    prev = None
    for _ in range(max_steps // chunk):
        f = dense.step(q, mask, f, tau, gv, chunk, periodic=periodic)
        _, u = dense.moments(q, mask, f, gv)
        ux = u[0, 0, 1:N + 1, 0]
        if prev is not None and np.max(np.abs(ux - prev)) <= tol * np.max(np.abs(ux)):
            return ux, u, mask
        prev = ux
    raise AssertionError("channel did not reach steady state")


def discrete_poiseuille(N, tau, g):
    """Exact steady velocity of the half-way bounce-back channel with Guo
    forcing: u_j = g/(2 nu) (N^2/4 - y_j^2) + g (16 lam^2 - 3)/(8 lam), with
    y_j = j - (N+1)/2, lam = tau - 1/2, nu = lam/3 -- a parabola with a
    uniform slip that vanishes at lam^2 = 3/16."""
    lam = tau - 0.5
    nu = lam / 3.0
    y = np.arange(1, N + 1) - (N + 1) / 2.0
    return g / (2 * nu) * (N * N / 4.0 - y * y) + g * (16 * lam * lam - 3) / (8 * lam)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("tau", [0.6, 0.8, 0.5 + math.sqrt(3) / 4, 1.3])
def test_poiseuille_exact_discrete_profile(q, tau):
    """Steady channel flow matches the exact discrete closed form to rounding
    (which pins bounce-back placement, the Guo half-force velocity and the
    viscosity (tau - 1/2)/3 of Eq. (2) together)."""
    N, g = 12, 1e-6
    ux, u, mask = _steady_channel(q, N, tau, g)
    want = discrete_poiseuille(N, tau, g)
    assert np.max(np.abs(ux - want)) <= 1e-10 * np.max(np.abs(want))
    # transverse velocity vanishes, profile uniform along the channel
    assert np.max(np.abs(u[1][~mask])) < 1e-10 * np.max(np.abs(want))
    cols = u[0][:, 1:N + 1, :]  # (nz, N, nx): every column carries the same profile
    assert np.max(np.abs(cols - ux[None, :, None])) <= 1e-13 * np.max(np.abs(want))


def test_poiseuille_exact_wall_point_has_no_slip():
    """At tau = 1/2 + sqrt(3)/4 the slip term vanishes: the profile equals the
    continuum parabola with walls half-way between nodes."""
    q, N, g = 9, 10, 1e-6
    tau = 0.5 + math.sqrt(3) / 4
    ux, _, _ = _steady_channel(q, N, tau, g)
    nu = (tau - 0.5) / 3
    y = np.arange(1, N + 1) - (N + 1) / 2.0
    cont = g / (2 * nu) * (N * N / 4.0 - y * y)
    assert np.max(np.abs(ux - cont)) <= 1e-10 * cont.max()


def test_poiseuille_second_order_convergence():
    """Relative L2 error against the continuum parabola falls as 1/N^2."""
    q, tau, g = 9, 0.8, 1e-6
    nu = (tau - 0.5) / 3
    errs = []
    Ns = [8, 16, 32]
    for N in Ns:
        ux, _, _ = _steady_channel(q, N, tau, g)
        y = np.arange(1, N + 1) - (N + 1) / 2.0
        cont = g / (2 * nu) * (N * N / 4.0 - y * y)
        errs.append(np.linalg.norm(ux - cont) / np.linalg.norm(cont))
    orders = [math.log(errs[k] / errs[k + 1], 2) for k in range(len(Ns) - 1)]
    assert all(1.9 < o < 2.1 for o in orders), orders


@pytest.mark.parametrize("q", [9, 19])
def test_shear_wave_decay_rate(q):
    """Fully periodic, g = 0, u_x = U sin(k y): the amplitude decays as
    exp(-nu k^2 t) with nu = (tau - 1/2)/3; the measured rate approaches nu k^2
    as the wave is resolved (discrete corrections are O(k^2))."""
    tau, U = 0.8, 1e-4
    nu = (tau - 0.5) / 3
    devs = []
    for L in (16, 32):
        shape = (1, L, 2) if q == 9 else (2, L, 2)
        mask = np.zeros(shape, bool)
        y = np.arange(L)
        k = 2 * math.pi / L
        rho = np.ones(shape)
        u = np.zeros((3,) + shape)
        u[0] = U * np.sin(k * y)[None, :, None]
        f = dense.init(q, mask, rho=rho, u=u)
        amps = []
        t1, t2 = int(0.2 / (nu * k * k)), int(0.7 / (nu * k * k))
        f = dense.step(q, mask, f, tau, [0, 0, 0], t1, periodic=7)
        _, uu = dense.moments(q, mask, f, [0, 0, 0])
        amps.append(np.dot(uu[0, 0, :, 0], np.sin(k * y)) * 2 / L)
        f = dense.step(q, mask, f, tau, [0, 0, 0], t2 - t1, periodic=7)
        _, uu = dense.moments(q, mask, f, [0, 0, 0])
        amps.append(np.dot(uu[0, 0, :, 0], np.sin(k * y)) * 2 / L)
        rate = math.log(amps[0] / amps[1]) / (t2 - t1)
        devs.append(abs(rate / (nu * k * k) - 1))
    assert devs[1] < 0.01
    assert devs[1] < devs[0] / 3
