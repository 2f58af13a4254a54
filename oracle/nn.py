"""FP64 NumPy oracle of the warm-start network's layer operations.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Arrays are
channels-last, shaped (nz, ny, nx, C).  Definitions:

  conv3(x, w, b)[z,y,x,n]  = b[n] + sum_{t,c} x[(z+dz)%nz, (y+dy)%ny, (x+dx)%nx, c] w[n,t,c]
                              with t = (dz+1)*9 + (dy+1)*3 + (dx+1)    (circular padding)
  up2(x, w, b)[2z+az, 2y+ay, 2x+ax, n] = b[n] + sum_c x[z,y,x,c] w[n,a,c],  a = az*4 + ay*2 + ax
  maxpool2(x)[z,y,x,c]     = max over the 2x2x2 block at (2z, 2y, 2x); the winner is the
                              first maximum in the order a = az*4 + ay*2 + ax
  dense(x, w, b)           = x @ w.T + b                                   (1x1x1 convolution)

conv3_at, up2_at and maxpool2_at evaluate the same definitions at chosen
voxels only, for checks on grids too large to evaluate whole.

and their gradients (backward data and weights), written as the adjoints of
these linear maps.
"""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import dijkstra

OFFS = [((t // 9) - 1, ((t // 3) % 3) - 1, (t % 3) - 1) for t in range(27)]  # (dz, dy, dx)
CORNERS = [((a >> 2) & 1, (a >> 1) & 1, a & 1) for a in range(8)]  # (az, ay, ax)


def _shifted(x, dz, dy, dx):
    """s[z,y,x] = x[(z+dz)%nz, (y+dy)%ny, (x+dx)%nx]."""
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(0, 1, 2))


def conv3(x, w, b=None):
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (dz, dy, dx) in enumerate(OFFS):
        y += _shifted(x, dz, dy, dx) @ w[:, t, :].T
    return y if b is None else y + b


def conv3_at(x, w, b, nodes):
    """conv3(x, w, b) at the voxels nodes[k] = (z, y, x) only: shape (K, n_out)."""
    nz, ny, nx, _ = x.shape
    z, y_, x_ = nodes[:, 0], nodes[:, 1], nodes[:, 2]
    y = np.zeros((len(nodes), w.shape[0]))
    for t, (dz, dy, dx) in enumerate(OFFS):
        y += x[(z + dz) % nz, (y_ + dy) % ny, (x_ + dx) % nx, :] @ w[:, t, :].T
    return y if b is None else y + b


def conv3_backward(x, w, dy):
    """(dx, dw, db) of conv3 for output gradient dy."""
    dx = np.zeros(x.shape)
    dw = np.zeros(w.shape)
    for t, (dz, dy_, dx_) in enumerate(OFFS):
        # y gathers x at +offset, so dx scatters dy back at -offset
        dx += _shifted(dy @ w[:, t, :], -dz, -dy_, -dx_)
        dw[:, t, :] = np.einsum("zyxn,zyxc->nc", dy, _shifted(x, dz, dy_, dx_))
    return dx, dw, dy.sum(axis=(0, 1, 2))


def up2(x, w, b=None):
    nz, ny, nx, _ = x.shape
    y = np.zeros((2 * nz, 2 * ny, 2 * nx, w.shape[0]))
    for a, (az, ay, ax) in enumerate(CORNERS):
        y[az::2, ay::2, ax::2, :] = x @ w[:, a, :].T
    return y if b is None else y + b


def up2_at(x, w, b, nodes):
    """up2(x, w, b) at the fine voxels nodes[k] = (z, y, x) only: shape (K, n_out)."""
    a = (nodes[:, 0] & 1) * 4 + (nodes[:, 1] & 1) * 2 + (nodes[:, 2] & 1)
    xs = x[nodes[:, 0] // 2, nodes[:, 1] // 2, nodes[:, 2] // 2, :]
    y = np.einsum("kc,knc->kn", xs, np.transpose(w, (1, 0, 2))[a])
    return y if b is None else y + b


def up2_backward(x, w, dy):
    dx = np.zeros(x.shape)
    dw = np.zeros(w.shape)
    for a, (az, ay, ax) in enumerate(CORNERS):
        g = dy[az::2, ay::2, ax::2, :]
        dx += g @ w[:, a, :]
        dw[:, a, :] = np.einsum("zyxn,zyxc->nc", g, x)
    return dx, dw, dy.sum(axis=(0, 1, 2))


def maxpool2(x):
    nz, ny, nx, c = x.shape
    blocks = np.stack([x[az::2, ay::2, ax::2, :] for (az, ay, ax) in CORNERS], axis=0)
    arg = np.argmax(blocks, axis=0)  # first maximum in corner order
    return blocks.max(axis=0), arg.astype(np.uint8)


def maxpool2_at(x, nodes):
    """maxpool2(x)[0] at the coarse voxels nodes[k] = (z, y, x) only: shape (K, C)."""
    z, y, x_ = 2 * nodes[:, 0], 2 * nodes[:, 1], 2 * nodes[:, 2]
    return np.max(np.stack([x[z + az, y + ay, x_ + ax, :] for (az, ay, ax) in CORNERS]), axis=0)


def maxpool2_backward(arg, dy):
    nz, ny, nx, c = dy.shape
    dx = np.zeros((2 * nz, 2 * ny, 2 * nx, c))
    for a, (az, ay, ax) in enumerate(CORNERS):
        dx[az::2, ay::2, ax::2, :] = np.where(arg == a, dy, 0.0)
    return dx


def dense(x, w, b=None):
    y = x @ w.T
    return y if b is None else y + b


def dense_backward(x, w, dy):
    return dy @ w, np.einsum("zyxn,zyxc->nc", dy, x), dy.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


def relu_backward(y, dy):
    return np.where(y > 0, dy, 0.0)


def masked_mse(pred, target, solid):
    """Sum over non-solid voxels of the squared error, and its gradient."""
    on = (~np.asarray(solid, bool))[..., None]
    d = np.where(on, pred - target, 0.0)
    return float((d * d).sum()), 2.0 * d


def adam(p, m, v, g, lr, b1, b2, eps, step):
    """Adam (Kingma & Ba) with bias correction; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# D3Q19 link offsets (faces and edges) and their lengths
LINKS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
         if 0 < abs(dx) + abs(dy) + abs(dz) <= 2]


def distance(solid, periodic=7):
    """Length of the shortest path over D3Q19 links (1 for faces, sqrt(2) for
    edges) from every node to the nearest solid node (multi-source Dijkstra);
    inf where no solid node is reachable.  solid: (nz, ny, nx) bool."""
    solid = np.asarray(solid, bool)
    nz, ny, nx = solid.shape
    idx = np.arange(solid.size).reshape(solid.shape)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rows, cols, w = [], [], []
    for dx, dy, dz in LINKS:
        tx, ty, tz = x + dx, y + dy, z + dz
        ok = np.ones(solid.shape, bool)
        for t, n, bit in ((tx, nx, 1), (ty, ny, 2), (tz, nz, 4)):
            if not (periodic & bit):
                ok &= (t >= 0) & (t < n)
        rows.append(idx[ok])
        cols.append(idx[tz % nz, ty % ny, tx % nx][ok])
        w.append(np.full(int(ok.sum()), np.sqrt(abs(dx) + abs(dy) + abs(dz))))
    graph = coo_matrix((np.concatenate(w), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(solid.size, solid.size)).tocsr()
    sources = np.flatnonzero(solid.ravel())
    if sources.size == 0:
        return np.full(solid.shape, np.inf)
    return dijkstra(graph, directed=True, indices=sources, min_only=True).reshape(solid.shape)


def encode_geometry(solid, dist, scale, cap):
    """(nz, ny, nx, 8): solid flag, s = min(dist * scale, cap) and s^2 on
    non-solid nodes, zeros elsewhere."""
    solid = np.asarray(solid, bool)
    v = np.where(solid, 0.0, np.minimum(np.asarray(dist) * scale, cap))
    out = np.zeros(solid.shape + (8,))
    out[..., 0] = solid
    out[..., 1] = v
    out[..., 2] = v * v
    return out
