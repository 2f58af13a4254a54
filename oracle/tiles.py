"""NumPy oracle of the tiling of a solid mask (arXiv 1703.08015, Sec. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper covers the geometry with a uniform mesh of a-edge tiles starting at
node (0, 0), extends it with solid nodes where the size is not divisible by a,
and drops tiles that hold only solid nodes; the two-copy method keeps a
``tileMap`` with the index of each non-empty tile and -1 for empty ones, used
to find the neighbour tiles during propagation.

Readings where the paper is silent:
  * padding goes at the high end of each non-periodic axis; a periodic axis
    whose size is not a multiple of the tile edge is an error;
  * non-empty tiles are numbered in row-major order of tile coordinates with
    tx fastest;
  * the neighbour row of a tile has 27 entries, k = (dx+1) + 3(dy+1) + 9(dz+1)
    for dx, dy, dz in {-1, 0, 1}, wrapped on periodic axes, -1 for a position
    outside a non-periodic axis or an empty tile;
  * node l = lx + ax*(ly + ay*lz) of a tile is bit (l % 64) of fluid word
    l // 64 (set = non-solid);
  * alpha_M, "the ratio of allocated ghost buffers to all possible ghost
    buffers" (Sec. 3.1.1.2), counts the faces of non-empty tiles: a face
    buffer is needed where the tile across the face is non-empty, and every
    face of a non-empty tile is a possible one.  Faces are those of the axes
    along which the lattice has more than one node.
"""
import numpy as np


class TilingError(ValueError):
    pass


def tile(mask, tile_edges, periodic):
    """Tile a solid mask.

    mask        bool/uint8 array (nz, ny, nx), nonzero = solid
    tile_edges  (ax, ay, az)
    periodic    (px, py, pz) booleans
    Returns a dict of NumPy arrays and statistics.
    """
    mask = np.asarray(mask).astype(bool)
    n = [mask.shape[2], mask.shape[1], mask.shape[0]]  # nx, ny, nz
    a = list(tile_edges)
    pad = []
    for ax in range(3):
        if periodic[ax] and n[ax] % a[ax]:
            raise TilingError("periodic axis %d of size %d is not a multiple of %d" % (ax, n[ax], a[ax]))
        pad.append((-n[ax]) % a[ax])
    padded = np.pad(mask, ((0, pad[2]), (0, pad[1]), (0, pad[0])), constant_values=True)
    npad = [n[i] + pad[i] for i in range(3)]
    T = [npad[i] // a[i] for i in range(3)]
    fluid = ~padded
    # blocks[tz, ty, tx, lz, ly, lx]
    blocks = fluid.reshape(T[2], a[2], T[1], a[1], T[0], a[0]).transpose(0, 2, 4, 1, 3, 5)
    has = blocks.any(axis=(3, 4, 5))
    tz, ty, tx = np.nonzero(has)
    nft = tz.size
    tile_map = np.full(T[2] * T[1] * T[0], -1, np.int32)
    flat = (tz * T[1] + ty) * T[0] + tx
    tile_map[flat] = np.arange(nft, dtype=np.int32)
    coord = np.stack([tx, ty, tz], axis=1).astype(np.int32)

    nbr = np.full((nft, 27), -1, np.int32)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                k = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
                c = [tx + dx, ty + dy, tz + dz]
                ok = np.ones(nft, bool)
                for ax in range(3):
                    if periodic[ax]:
                        c[ax] = np.mod(c[ax], T[ax])
                    else:
                        ok &= (c[ax] >= 0) & (c[ax] < T[ax])
                        c[ax] = np.clip(c[ax], 0, T[ax] - 1)
                idx = (c[2] * T[1] + c[1]) * T[0] + c[0]
                nbr[:, k] = np.where(ok, tile_map[idx], -1)

    ntn = a[0] * a[1] * a[2]
    if ntn % 64:
        raise TilingError("tile of %d nodes is not a multiple of 64" % ntn)
    words = ntn // 64
    bits = blocks[tz, ty, tx].reshape(nft, ntn)  # node order lz, ly, lx -> l = lx + ax*(ly + ay*lz)
    weights = (np.uint64(1) << np.arange(64, dtype=np.uint64))
    fl = np.zeros((nft, words), np.uint64)
    for w in range(words):
        sub = bits[:, 64 * w:64 * (w + 1)].astype(np.uint64)
        fl[:, w] = (sub * weights).sum(axis=1, dtype=np.uint64)

    # alpha_M: non-empty face neighbours (slots 13 -+ 1, 3, 9 of the row)
    faces = shared = 0
    for ax, step in ((0, 1), (1, 3), (2, 9)):
        if npad[ax] > 1:
            shared += int((nbr[:, 13 - step] >= 0).sum() + (nbr[:, 13 + step] >= 0).sum())
            faces += 2 * nft

    n_nodes = n[0] * n[1] * n[2]
    n_f = int((~mask).sum())
    return dict(
        tile_map=tile_map, tile_coord=coord.reshape(-1), nbr=nbr.reshape(-1), fluid=fl.reshape(-1),
        grid=np.array(npad, np.int32), tgrid=np.array(T, np.int32),
        n_tiles=int(T[0] * T[1] * T[2]), n_ftiles=int(nft), n_fluid=n_f, n_nodes=n_nodes,
        phi=n_f / n_nodes, phi_t=(n_f / (nft * ntn)) if nft else 0.0,
        tiles_ratio=(T[0] * T[1] * T[2] / nft) if nft else float("inf"),
        alpha_m=(shared / faces) if faces else 0.0,
    )
