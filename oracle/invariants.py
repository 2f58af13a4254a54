"""FP64 NumPy oracle of the conserved quantities of the discrete LBM dynamics
and of the projection that gives a warm-start (rho, u) the values a start
from rest has.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The step of Sec. 2 (BGK collision, Eq. 5, with the Guo body force; pull
streaming with half-way bounce-back at solid nodes) conserves, besides the
mass of every set of fluid nodes joined by lattice links, one staggered
momentum per axis:

  collision keeps rho and j = sum_i c_i f_i at each node and the force adds
  exactly rho*g; a population with c_ik != 0 either moves one node along k or
  bounces back with c_ik negated, and both flip the sign of (-1)^{x_k} c_ik f_i.
  Hence, for every set A of fluid nodes that no link with c_k != 0 leaves,

      S_k(A, t+1) = -S_k(A, t) + g_k * sum_{x in A} (-1)^{x_k} rho(x),
      S_k(A, t)   =  sum_{x in A} (-1)^{x_k} j_k(x, t)

  (an even periodic extent keeps the parity consistent across the wrap).
  The long-time state is a period-2 cycle whose staggered part is set by
  S_k(A, 0): a start from rest has S_k = 0 and mass rho0 * |A|.  A start
  f* = f_eq(rho, u) has j = rho*u, so a prediction reaches the same long-time
  state only after its mass per component is rescaled and its staggered
  momentum per component is removed.

Arrays: mask (nz, ny, nx) bool (True = solid), rho (nz, ny, nx),
u (3, nz, ny, nx) with u[0] the x component.  Labels are int64, -1 on solid
nodes, components numbered by first appearance in x-fastest scan order.
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


def components(mask, q, axis=-1, periodic=7):
    """Connected fluid components under the links of the D2Q9 / D3Q19
    lattice that join two fluid nodes; with axis k in {0, 1, 2} only links
    with c_k != 0 count.  Returns (labels, count)."""
    mask = np.asarray(mask, bool)
    nz, ny, nx = mask.shape
    c, _, _ = dense.lattice(q)
    fluid = ~mask
    idx = np.arange(mask.size).reshape(mask.shape)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rows, cols = [], []
    for ci in c:
        if not ci.any() or (axis >= 0 and ci[axis] == 0):
            continue
        tx, ty, tz = x + ci[0], y + ci[1], z + ci[2]
        ok = fluid.copy()
        for t, n, bit in ((tx, nx, 1), (ty, ny, 2), (tz, nz, 4)):
            if not (periodic & bit):
                ok &= (t >= 0) & (t < n)
        tx, ty, tz = tx % nx, ty % ny, tz % nz
        ok &= fluid[tz, ty, tx]
        rows.append(idx[ok])
        cols.append(idx[tz, ty, tx][ok])
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    graph = coo_matrix((np.ones(rows.size), (rows, cols)), shape=(mask.size, mask.size))
    _, lab = connected_components(graph, directed=False)
    lab = np.where(fluid.ravel(), lab, -1).reshape(mask.shape)
    return _canonical(lab)


def staggered_momentum(mask, rho, u, labels, count, axis):
    """S_k per component: sum of (-1)^{x_k} rho u_k, and the component mass."""
    nz, ny, nx = mask.shape
    coord = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")[2 - axis]
    sign = np.where(coord % 2 == 0, 1.0, -1.0)
    on = labels >= 0
    s = np.bincount(labels[on], weights=(sign * rho * u[axis])[on], minlength=count)
    m = np.bincount(labels[on], weights=rho[on], minlength=count)
    return s, m


def project(mask, rho, u, q, rho0=1.0, periodic=7):
    """Rescale rho so that every lattice-connected component holds rho0 per
    node, then subtract from u_k, per component of the c_k != 0 links, the
    staggered field (-1)^{x_k} S_k / M that carries its staggered momentum."""
    mask = np.asarray(mask, bool)
    nz, ny, nx = mask.shape
    rho = np.where(mask, 0.0, np.asarray(rho, np.float64))
    u = np.where(mask[None], 0.0, np.asarray(u, np.float64))
    lab, n = components(mask, q, -1, periodic)
    on = lab >= 0
    mass = np.bincount(lab[on], weights=rho[on], minlength=n)
    nodes = np.bincount(lab[on], minlength=n)
    scale = np.zeros(rho.shape)
    scale[on] = (rho0 * nodes / mass)[lab[on]]
    rho = rho * scale
    u = u.copy()
    dims = 2 if q == 9 else 3
    for k in range(dims):
        labk, nk = components(mask, q, k, periodic)
        s, m = staggered_momentum(mask, rho, u, labk, nk, k)
        coord = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")[2 - k]
        sign = np.where(coord % 2 == 0, 1.0, -1.0)
        onk = labk >= 0
        u[k][onk] -= (sign * (s / m)[labk])[onk]
    return rho, u
