"""FP64 NumPy oracle of the conserved quantities of the discrete LBM dynamics
and of the projection that gives a warm-start (rho, u) the values a start
from rest has.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The step of Sec. 2 (BGK collision, Eq. 5, with the Guo body force; pull
streaming with half-way bounce-back at solid nodes) keeps two families of
linear functionals of the post-collision state f*:

* mass: the sum of f* over every set of fluid nodes joined by lattice links;

* staggered momentum: L_beta(f*) = sum_x beta(x) . j(x), j = sum_i c_i f*_i,
  for every field beta in the null space N of the link operator
      (A beta)_link = c . beta(x + c) + c . beta(x)
  (one row per fluid-fluid link).  Collision keeps j at each node and the
  force adds rho*g; streaming moves c_i f_i to x + c_i, where the row of A
  says c.beta(x+c) = -c.beta(x); bounce-back keeps the node and negates c.
  Both flip the sign of each term, so
      L_beta(t+1) = -L_beta(t) + sum_x beta(x) . g rho(x),
  never damped.  beta_k = (-1)^{x_k} on a set joined by links with c_k != 0
  is one such field; where fluid nodes touch only diagonally there are more.

A start from rest has j = 0 (every L_beta = 0) and rho0 per node.  A start
f* = f_eq(rho, u) has j = rho u and keeps its own L_beta, so it settles into a
different long-time state unless rho u is first made orthogonal to N.  The
link operator  T = (3/2) A^T W A,  W = diag(w_i),
    (T j)(x) = 3 sum_{i: x + c_i fluid} w_i c_i [c_i . (j(x) + j(x + c_i))] / 2,
is symmetric positive semi-definite with null space exactly N, so its range is
orthogonal to N.  It is the identity on smooth fields in the bulk
(3 sum_i w_i c_i c_i = I) with eigenvalues in [0, 1], hence the Richardson
iteration j <- j + T(rho u - j) from j = 0 stays orthogonal to N after any
number of sweeps and converges to the orthogonal projection of rho u.

Arrays: mask (nz, ny, nx) bool (True = solid), rho (nz, ny, nx),
u (3, nz, ny, nx) with u[0] the x component.  Labels are int64, -1 on solid
nodes, components numbered by first appearance in x-fastest scan order.
Periodic bits: 1 = x, 2 = y, 4 = z; a non-periodic edge is a wall.
"""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from . import dense


def _canonical(labels):
    """Renumber components 0,1,... by first appearance in scan order."""
    flat = labels.ravel()
    out = np.full(flat.shape, -1, np.int64)
    seen = {}
    for i in np.flatnonzero(flat >= 0):
        lab = flat[i]
        if lab not in seen:
            seen[lab] = len(seen)
        out[i] = seen[lab]
    return out.reshape(labels.shape), len(seen)


def _links(mask, q, periodic):
    """Yield (i, c_i, source index, target index) for every fluid-fluid link
    along direction i (both orientations of a link appear, once each)."""
    nz, ny, nx = mask.shape
    c, _, _ = dense.lattice(q)
    fluid = ~mask
    idx = np.arange(mask.size).reshape(mask.shape)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for i, ci in enumerate(c):
        if not ci.any():
            continue
        tx, ty, tz = x + ci[0], y + ci[1], z + ci[2]
        ok = fluid.copy()
        for t, n, bit in ((tx, nx, 1), (ty, ny, 2), (tz, nz, 4)):
            if not (periodic & bit):
                ok &= (t >= 0) & (t < n)
        tx, ty, tz = tx % nx, ty % ny, tz % nz
        ok &= fluid[tz, ty, tx]
        yield i, ci, idx[ok], idx[tz, ty, tx][ok]


def components(mask, q, axis=-1, periodic=7):
    """Connected fluid components under the links of the D2Q9 / D3Q19
    lattice that join two fluid nodes; with axis k in {0, 1, 2} only links
    with c_k != 0 count.  Returns (labels, count)."""
    mask = np.asarray(mask, bool)
    rows, cols = [], []
    for _, ci, a, b in _links(mask, q, periodic):
        if axis >= 0 and ci[axis] == 0:
            continue
        rows.append(a)
        cols.append(b)
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    graph = coo_matrix((np.ones(rows.size), (rows, cols)), shape=(mask.size, mask.size))
    _, lab = connected_components(graph, directed=False)
    lab = np.where((~mask).ravel(), lab, -1).reshape(mask.shape)
    return _canonical(lab)


def staggered_momentum(mask, rho, u, labels, count, axis):
    """Per component of the c_k != 0 links: sum of (-1)^{x_k} rho u_k (one
    member of the invariant family), and the component mass."""
    nz, ny, nx = mask.shape
    coord = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")[2 - axis]
    sign = np.where(coord % 2 == 0, 1.0, -1.0)
    on = labels >= 0
    s = np.bincount(labels[on], weights=(sign * rho * u[axis])[on], minlength=count)
    m = np.bincount(labels[on], weights=rho[on], minlength=count)
    return s, m


def link_matrix(mask, q, periodic=7):
    """The link operator A as a sparse matrix: one row per undirected
    fluid-fluid link, columns 3*node + k over all nodes."""
    mask = np.asarray(mask, bool)
    _, _, opp = dense.lattice(q)
    rows, cols, vals = [], [], []
    r = 0
    for i, ci, a, b in _links(mask, q, periodic):
        if i > opp[i]:
            continue  # the opposite direction describes the same links
        m = a.size
        for k in range(3):
            if ci[k] == 0:
                continue
            rows += [np.arange(r, r + m)] * 2
            cols += [3 * a + k, 3 * b + k]
            vals += [np.full(m, float(ci[k]))] * 2
        r += m
    if not rows:
        return coo_matrix((0, 3 * mask.size)).tocsr()
    return coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(r, 3 * mask.size)).tocsr()


def invariant_basis(mask, q, periodic=7):
    """Orthonormal basis (columns, shape (3*nodes, d)) of the null space of A
    restricted to fluid nodes, by dense eigen-decomposition of A^T A (small
    geometries only).  Each column reshaped to (nz, ny, nx, 3) is a beta."""
    mask = np.asarray(mask, bool)
    A = link_matrix(mask, q, periodic)
    fluid_cols = np.flatnonzero(np.repeat((~mask).ravel(), 3))
    if q == 9:
        fluid_cols = fluid_cols[fluid_cols % 3 != 2]  # no z momentum in 2D
    G = (A.T @ A)[fluid_cols][:, fluid_cols].toarray()
    w, v = np.linalg.eigh(G)
    null = v[:, w < 1e-9]
    out = np.zeros((3 * mask.size, null.shape[1]))
    out[fluid_cols] = null
    return out


def link_operator(mask, j, q, periodic=7):
    """(T j)(x) = 3 sum_{i: x + c_i fluid} w_i c_i [c_i . (j(x) + j(x + c_i))] / 2
    on fluid nodes, 0 on solid ones; j has shape (3, nz, ny, nx)."""
    mask = np.asarray(mask, bool)
    _, w, _ = dense.lattice(q)
    flat = np.asarray(j, np.float64).reshape(3, -1)
    out = np.zeros_like(flat)
    for i, ci, a, b in _links(mask, q, periodic):
        s = (ci[:, None] * (flat[:, a] + flat[:, b])).sum(axis=0) / 2.0
        np.add.at(out, (slice(None), a), 3.0 * w[i] * ci[:, None] * s[None, :])
    return out.reshape(np.shape(j))


def project(mask, rho, u, q, rho0=1.0, periodic=7, iterations=8):
    """Rescale rho so that every lattice-connected component holds rho0 per
    node, then replace rho u by `iterations` Richardson sweeps
    j <- j + T(rho u - j) from j = 0, and return (rho, j / rho)."""
    mask = np.asarray(mask, bool)
    rho = np.where(mask, 0.0, np.asarray(rho, np.float64))
    u = np.where(mask[None], 0.0, np.asarray(u, np.float64))
    lab, n = components(mask, q, -1, periodic)
    on = lab >= 0
    mass = np.bincount(lab[on], weights=rho[on], minlength=n)
    nodes = np.bincount(lab[on], minlength=n)
    scale = np.zeros(rho.shape)
    scale[on] = (rho0 * nodes / mass)[lab[on]]
    rho = rho * scale
    target = rho[None] * u
    j = np.zeros_like(u)
    for _ in range(iterations):
        j = j + link_operator(mask, target - j, q, periodic)
    safe = np.where(mask, 1.0, rho)
    return rho, np.where(mask[None], 0.0, j / safe[None])
