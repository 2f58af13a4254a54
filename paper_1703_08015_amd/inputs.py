"""Seeded synthetic geometries and fields.

This module only draws inputs: solid masks shaped like the porous media and
vessel geometries the paper measures on (random sphere arrays, a vessel tree,
a 2D channel with obstacles) and random PDF fields for permutation checks.
It holds none of the lattice Boltzmann arithmetic and imports nothing from the
solver, so the GPU path and the CPU oracle can both be fed from it.

Conventions: masks are bool arrays (nz, ny, nx), True = solid; a node is
inside a sphere/disc/cylinder iff its squared distance to the centre (axis)
is <= r^2, measured with the minimum image on periodic axes.  Random numbers
come from ``numpy.random.default_rng(seed)``.
"""
import numpy as np


def _wrap_delta(d, n, periodic):
    if periodic:
        return (d + n / 2.0) % n - n / 2.0
    return d


def _box(center, r, n, periodic):
    lo = int(np.floor(center - r)) - 1
    hi = int(np.ceil(center + r)) + 2
    idx = np.arange(lo, hi)
    if periodic:
        if hi - lo >= n:
            idx = np.arange(n)
        else:
            idx = np.mod(idx, n)
    else:
        idx = idx[(idx >= 0) & (idx < n)]
    return idx


def _stamp_ball(solid, center, r, periodic):
    """Mark nodes within distance r of center (x, y, z); return newly solid count."""
    nz, ny, nx = solid.shape
    n = (nx, ny, nz)
    ix = _box(center[0], r, nx, periodic[0])
    iy = _box(center[1], r, ny, periodic[1])
    iz = _box(center[2], r, nz, periodic[2])
    if ix.size == 0 or iy.size == 0 or iz.size == 0:
        return 0
    dx = _wrap_delta(ix - center[0], n[0], periodic[0])
    dy = _wrap_delta(iy - center[1], n[1], periodic[1])
    dz = _wrap_delta(iz - center[2], n[2], periodic[2])
    inside = (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2) <= r * r
    sub = solid[np.ix_(iz, iy, ix)]
    new = int((inside & ~sub).sum())
    solid[np.ix_(iz, iy, ix)] = sub | inside
    return new


def channel_2d(nx=64, ny=64, porosity=0.6, rmin=3.0, rmax=6.0, seed=0, discs=True,
               max_tries=200000):
    """2D channel: solid walls at y = 0 and y = ny-1, periodic in x, plus
    non-overlapping solid discs of radius U[rmin, rmax] drawn until the
    porosity (fluid fraction of all nodes) first drops to <= ``porosity``.
    Returns (mask (1, ny, nx), achieved porosity)."""
    solid = np.zeros((1, ny, nx), bool)
    solid[0, 0, :] = True
    solid[0, ny - 1, :] = True
    rng = np.random.default_rng(seed)
    total = nx * ny
    n_solid = int(solid.sum())
    tries = 0
    # placed discs bucketed on a grid of cells at least 2 rmax + 1 wide, so a
    # candidate is tested against the discs of the 3x3 cells around it only
    # (the same acceptance rule as testing all of them)
    cell = 2.0 * rmax + 1.0
    ncx, ncy = max(1, int(nx // cell)), max(1, int(ny // cell))
    wx, wy = nx / ncx, ny / ncy
    buckets = {}
    while discs and (total - n_solid) / total > porosity and tries < max_tries:
        tries += 1
        r = rng.uniform(rmin, rmax)
        cx = rng.uniform(0, nx)
        cy = rng.uniform(1 + r, ny - 2 - r)
        ok = True
        bx, by = int(cx // wx) % ncx, min(int(cy // wy), ncy - 1)
        near = {((bx + dx) % ncx, by + dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1) if 0 <= by + dy < ncy}
        for key in near:
            for (px, py, pr) in buckets.get(key, ()):
                ddx = _wrap_delta(cx - px, nx, True)
                if ddx * ddx + (cy - py) ** 2 < (r + pr + 1.0) ** 2:
                    ok = False
                    break
            if not ok:
                break
        if not ok:
            continue
        buckets.setdefault((bx, by), []).append((cx, cy, r))
        sub = solid[0:1]
        n_solid += _stamp_ball(sub, (cx, cy, 0.0), r, (True, False, False))
    return solid, (total - n_solid) / total


def spheres_3d(n, porosity, rmin=4.0, rmax=12.0, seed=0, periodic=(True, True, True)):
    """Overlapping solid spheres with radius U[rmin, rmax] and uniform centres,
    added until the porosity first drops to <= ``porosity``.
    ``n`` is an int (cube) or (nx, ny, nz).  Returns (mask, achieved porosity)."""
    if np.isscalar(n):
        n = (int(n),) * 3
    nx, ny, nz = n
    solid = np.zeros((nz, ny, nx), bool)
    rng = np.random.default_rng(seed)
    total = nx * ny * nz
    n_solid = 0
    while (total - n_solid) / total > porosity:
        r = rng.uniform(rmin, rmax)
        c = (rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz))
        n_solid += _stamp_ball(solid, c, r, periodic)
    return solid, (total - n_solid) / total


def _stamp_capsule(fluid, p0, p1, r, periodic):
    """Mark nodes within distance r of the segment p0-p1 as fluid."""
    nz, ny, nx = fluid.shape
    n = (nx, ny, nz)
    lo = np.minimum(p0, p1) - r
    hi = np.maximum(p0, p1) + r
    idx = []
    for a in range(3):
        ii = np.arange(int(np.floor(lo[a])) - 1, int(np.ceil(hi[a])) + 2)
        if periodic[a]:
            ii = np.arange(n[a]) if ii.size >= n[a] else ii
        else:
            ii = ii[(ii >= 0) & (ii < n[a])]
        idx.append(ii)
    if any(i.size == 0 for i in idx):
        return
    X = idx[0][None, None, :].astype(np.float64)
    Y = idx[1][None, :, None].astype(np.float64)
    Z = idx[2][:, None, None].astype(np.float64)
    d = p1 - p0
    L2 = float(d @ d)
    # parameter of the closest point on the segment, on unwrapped coordinates
    t = ((X - p0[0]) * d[0] + (Y - p0[1]) * d[1] + (Z - p0[2]) * d[2]) / max(L2, 1e-12)
    t = np.clip(t, 0.0, 1.0)
    dx = X - (p0[0] + t * d[0])
    dy = Y - (p0[1] + t * d[1])
    dz = Z - (p0[2] + t * d[2])
    inside = dx * dx + dy * dy + dz * dz <= r * r
    wi = [np.mod(i, n[a]) if periodic[a] else i for a, i in enumerate(idx)]
    sub = fluid[np.ix_(wi[2], wi[1], wi[0])]
    fluid[np.ix_(wi[2], wi[1], wi[0])] = sub | inside


def _rotate_away(v, angle, rng):
    """Unit vector at ``angle`` from unit vector v, in a random plane."""
    a = rng.normal(size=3)
    a -= (a @ v) * v
    a /= np.linalg.norm(a)
    return np.cos(angle) * v + np.sin(angle) * a


def vessel_tree(n=448, fluid_fraction=0.08, generations=5, r_root=20.0, r_leaf=6.0, seed=0,
                periodic=(True, True, True), max_trees=200):
    """Vessel-like sparse geometry: seeded trees of bifurcating cylinders
    (capsules), radius shrinking geometrically from ``r_root`` to ``r_leaf``
    over ``generations`` generations, segment length U[6, 10] * r, branching
    half-angle U[25, 45] degrees.  Trees are planted until the fluid fraction
    first reaches >= ``fluid_fraction``.  Fluid inside the vessels, solid
    elsewhere.  Returns (mask, achieved porosity)."""
    if np.isscalar(n):
        n = (int(n),) * 3
    nx, ny, nz = n
    fluid = np.zeros((nz, ny, nx), bool)
    rng = np.random.default_rng(seed)
    ratio = (r_leaf / r_root) ** (1.0 / max(generations - 1, 1))
    total = nx * ny * nz
    for _ in range(max_trees):
        root = np.array([rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)])
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        stack = [(root, v, r_root, 0)]
        while stack:
            p, v, r, gen = stack.pop()
            length = rng.uniform(6.0, 10.0) * r
            q = p + length * v
            _stamp_capsule(fluid, p, q, r, periodic)
            if gen + 1 < generations:
                for _k in range(2):
                    ang = np.deg2rad(rng.uniform(25.0, 45.0))
                    stack.append((q, _rotate_away(v, ang, rng), r * ratio, gen + 1))
        if fluid.sum() / total >= fluid_fraction:
            break
    return ~fluid, float(fluid.sum()) / total


def batch_specs(count=512, seed=1000, edge_min=32, edge_max=96, step=4, phi_min=0.2, phi_max=0.8,
                g_mag=1e-6):
    """Per-sample specifications of a batch of porous cubes: edge uniform over
    {edge_min, edge_min+step, ..., edge_max}, target porosity U[phi_min, phi_max],
    force of magnitude ``g_mag`` with a direction uniform on the sphere, and a
    geometry seed."""
    rng = np.random.default_rng(seed)
    edges = np.arange(edge_min, edge_max + 1, step)
    out = []
    for k in range(count):
        e = int(rng.choice(edges))
        phi = float(rng.uniform(phi_min, phi_max))
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        out.append(dict(edge=e, porosity=phi, g=(g_mag * d).tolist(), seed=int(seed * 1000 + k)))
    return out


def porous_cube(spec, rmin=4.0, rmax=12.0):
    """Geometry of one ``batch_specs`` entry (periodic sphere packing)."""
    return spheres_3d(spec["edge"], spec["porosity"], rmin, rmax, seed=spec["seed"])


def random_pdfs(q, mask, seed=0, lo=0.01, hi=0.1):
    """Random positive post-collision PDFs f[q, z, y, x] (solid entries 0)."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(lo, hi, size=(q,) + mask.shape)
    f[:, np.asarray(mask, bool)] = 0.0
    return f


def random_macro(mask, seed=0, drho=0.01, umax=0.02):
    """Random density around 1 and velocity fields (rho[z,y,x], u[3,z,y,x])."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-drho, drho, size=mask.shape)
    u = rng.uniform(-umax, umax, size=(3,) + mask.shape)
    m = np.asarray(mask, bool)
    rho[m] = 0.0
    u[:, m] = 0.0
    return rho, u
