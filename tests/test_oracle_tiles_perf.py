"""Pins of the NumPy tiling oracle (brute force over tiny masks) and of the
overhead model (the paper's Table 1 and printed constants)."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import perfmodel as pm
from oracle import tiles

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_overheads.json")


def brute_tiles(mask, a, periodic):
    """Pure-Python loops over every node and tile: the tiling of Sec. 3."""
    nz, ny, nx = mask.shape
    n = [nx, ny, nz]
    npad = [((n[i] + a[i] - 1) // a[i]) * a[i] for i in range(3)]
    T = [npad[i] // a[i] for i in range(3)]

    def solid(x, y, z):
        if x >= nx or y >= ny or z >= nz:
            return True
        return bool(mask[z, y, x])

    order = []
    for tz in range(T[2]):
        for ty in range(T[1]):
            for tx in range(T[0]):
                any_fluid = False
                for lz in range(a[2]):
                    for ly in range(a[1]):
                        for lx in range(a[0]):
                            if not solid(tx * a[0] + lx, ty * a[1] + ly, tz * a[2] + lz):
                                any_fluid = True
                if any_fluid:
                    order.append((tx, ty, tz))
    index = {c: k for k, c in enumerate(order)}
    tmap = []
    for tz in range(T[2]):
        for ty in range(T[1]):
            for tx in range(T[0]):
                tmap.append(index.get((tx, ty, tz), -1))
    nbr = []
    fluid = []
    ntn = a[0] * a[1] * a[2]
    for (tx, ty, tz) in order:
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    c = [tx + dx, ty + dy, tz + dz]
                    ok = True
                    for ax in range(3):
                        if c[ax] < 0 or c[ax] >= T[ax]:
                            if periodic[ax]:
                                c[ax] %= T[ax]
                            else:
                                ok = False
                    nbr.append(index.get(tuple(c), -1) if ok else -1)
        words = [0] * (ntn // 64)
        for lz in range(a[2]):
            for ly in range(a[1]):
                for lx in range(a[0]):
                    l = lx + a[0] * (ly + a[1] * lz)
                    if not solid(tx * a[0] + lx, ty * a[1] + ly, tz * a[2] + lz):
                        words[l // 64] |= 1 << (l % 64)
        fluid.extend(words)
    return tmap, [c for t in order for c in t], nbr, fluid


CASES = [
    ((4, 4, 4), (1, 1, 1), (8, 12, 8)),
    ((4, 4, 4), (0, 1, 0), (9, 8, 7)),
    ((4, 4, 4), (0, 0, 0), (5, 5, 5)),
    ((16, 16, 1), (1, 0, 0), (32, 35, 1)),
    ((4, 4, 8), (1, 1, 1), (8, 8, 16)),
]


@pytest.mark.parametrize("a,periodic,shape", CASES)
@pytest.mark.parametrize("seed", [0, 1])
def test_tiles_match_brute_force(a, periodic, shape, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    mask = rng.random((nz, ny, nx)) < 0.8
    mask[rng.random((nz, ny, nx)) < 0.5] = True  # sparse fluid, some empty tiles
    t = tiles.tile(mask, a, periodic)
    tmap, coord, nbr, fluid = brute_tiles(mask, a, periodic)
    assert t["tile_map"].tolist() == tmap
    assert t["tile_coord"].tolist() == coord
    assert t["nbr"].tolist() == nbr
    assert [int(v) for v in t["fluid"]] == fluid
    nf = sum(bin(v).count("1") for v in fluid)
    assert nf == int((~mask).sum()) == t["n_fluid"]


@pytest.mark.parametrize("a,periodic,shape", CASES)
def test_alpha_m_brute_force(a, periodic, shape):
    """alpha_M from tile coordinates alone: for each non-empty tile and each
    face along an axis with more than one node, whether the tile across the
    face (wrapped on periodic axes) holds a non-solid node."""
    rng = np.random.default_rng(3)
    nx, ny, nz = shape
    mask = rng.random((nz, ny, nx)) < 0.6
    t = tiles.tile(mask, a, periodic)
    tmap, coord, _, _ = brute_tiles(mask, a, periodic)
    n = (nx, ny, nz)
    T = [-(-n[k] // a[k]) for k in range(3)]
    occupied = set(tuple(coord[3 * j:3 * j + 3]) for j in range(len(coord) // 3))
    faces = shared = 0
    for c in occupied:
        for ax in range(3):
            if T[ax] * a[ax] <= 1:
                continue
            for s in (-1, 1):
                faces += 1
                o = list(c)
                o[ax] += s
                if periodic[ax]:
                    o[ax] %= T[ax]
                elif not 0 <= o[ax] < T[ax]:
                    continue
                shared += tuple(o) in occupied
    assert t["alpha_m"] == shared / faces


def test_alpha_m_closed_forms():
    """A fluid box closed on every axis with T tiles per axis: 1 - 1/T (the
    2 of the 2T faces per tile row that lie on the box); periodic: 1; an
    isolated tile: 0; a 2D lattice counts the x and y faces only."""
    for T in (1, 2, 3, 5):
        t = tiles.tile(np.zeros((4 * T,) * 3, bool), (4, 4, 4), (0, 0, 0))
        assert t["alpha_m"] == pytest.approx(1.0 - 1.0 / T, abs=1e-15)
    assert tiles.tile(np.zeros((8, 12, 16), bool), (4, 4, 4), (1, 1, 1))["alpha_m"] == 1.0
    m = np.ones((12, 12, 12), bool)
    m[5, 6, 4] = False
    assert tiles.tile(m, (4, 4, 4), (1, 1, 1))["alpha_m"] == 0.0
    # 2D: 3 x 2 tiles of 16 x 16, periodic in x, closed in y: both x faces of
    # every tile are shared, one of its two y faces
    t = tiles.tile(np.zeros((1, 32, 48), bool), (16, 16, 1), (1, 0, 0))
    assert t["alpha_m"] == pytest.approx((6 * 2 + 6 * 1) / (6 * 4), abs=1e-15)


def test_tiles_edge_cases():
    a = (4, 4, 4)
    # all solid: no tiles
    t = tiles.tile(np.ones((8, 8, 8), bool), a, (1, 1, 1))
    assert t["n_ftiles"] == 0 and np.all(t["tile_map"] == -1)
    # one fluid node: one tile, self-neighbour on a periodic 1-tile axis
    m = np.ones((4, 8, 8), bool)
    m[1, 2, 3] = False
    t = tiles.tile(m, a, (1, 1, 1))
    assert t["n_ftiles"] == 1 and t["tile_coord"].tolist() == [0, 0, 0]
    assert int(t["fluid"][0]) == 1 << (3 + 4 * 2 + 16 * 1)
    row = t["nbr"].reshape(-1, 27)[0]
    assert row[13] == 0 and row[(0 + 1) + 3 * 1 + 9 * 0] == 0  # z wraps onto itself (Tz = 1)
    # non-divisible periodic axis
    with pytest.raises(tiles.TilingError):
        tiles.tile(np.zeros((4, 4, 6), bool), a, (1, 0, 0))
    # non-divisible non-periodic axis is padded with solid
    t = tiles.tile(np.zeros((4, 4, 6), bool), a, (0, 0, 0))
    assert t["grid"].tolist() == [8, 4, 4] and t["n_ftiles"] == 2
    assert int(t["fluid"][1]) == sum(1 << (x + 4 * y + 16 * z) for x in range(2) for y in range(4) for z in range(4))


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def _geom(lat):
    return (19, 4, 3) if lat == "D3Q19" else (9, 16, 2)


def _printed_within(fn, lo_args, hi_args, printed, digits):
    """The printed value (rounded to ``digits``) lies in the model's range when
    each input varies over its own rounding interval (the model is monotone in
    each input, so the interval ends bound it)."""
    vals = [fn(*args) for args in (lo_args, hi_args)]
    half = 0.5 * 10.0 ** (-digits)
    return min(vals) - half - 1e-12 <= printed <= max(vals) + half + 1e-12


@pytest.mark.parametrize("row", _golden()["table1"], ids=lambda r: r["case"])
def test_table1_rows(row):
    """Table 1: every overhead estimate follows from (phi, phi_t, alpha_M),
    printed to two digits, with s_d = 8, s_t = 2 and 4-byte indices."""
    lat = row["lattice"]
    q, a, d = _geom(lat)
    e = 0.005
    phi, pt, al = row["phi"], row["phi_t"], row["alpha_m"]
    assert round(pm.cm_memory(q, 8), 2) == row["dm_cm"]
    assert round(pm.cm_bandwidth(q, 8), 2) == row["db_cm"]
    assert _printed_within(lambda p: pm.fia_memory(q, 8, p), (phi - e,), (phi + e,), row["dm_fia"], 2)
    assert _printed_within(lambda p: pm.fia_bandwidth(q, 8, p), (phi - e,), (phi + e,), row["db_fia"], 3)
    assert _printed_within(lambda p: pm.t2c_bandwidth(q, 8, a, d, p), (pt - e,), (pt + e,), row["db_t2c"], 3)
    assert _printed_within(lambda p: pm.tgb_bandwidth(lat, 8, a, d, p), (pt - e,), (pt + e,), row["db_tgb"], 3)
    # the tiles ratio is not printed per case; Sec. 3.1.1.1 bounds it to (2.3, 8.6)
    assert _printed_within(lambda p, r: pm.t2c_memory(q, 8, a, d, p, r), (pt + e, 2.3), (pt - e, 8.6),
                           row["dm_t2c"], 2)
    assert _printed_within(lambda p, al_: pm.tgb_memory(lat, 8, a, d, p, al_), (pt + e, al - e), (pt - e, al + e),
                           row["dm_tgb"], 2)


def test_printed_constants():
    g = _golden()["constants"]
    # Eq. (24) written as (A + B * ratio)/phi_t - 1: A = 2 + s_t/M_node, B = s_ti/(n_tn M_node)
    for key, (q, a, d) in (("eq25_d2q9_16", (9, 16, 2)), ("eq26_d3q19_4", (19, 4, 3))):
        A = 2 + 2 / pm.m_node(q, 8)
        B = 4 / (pm.n_tn(a, d) * pm.m_node(q, 8))
        assert round(A, 3) == g[key][0] and round(B, 5) == g[key][1]
        # and the full function agrees with that linear form, Eq. (25)/(26)
        for pt, r in ((0.8, 3.0), (0.5, 7.0)):
            assert abs(pm.t2c_memory(q, 8, a, d, pt, r) - ((A + B * r) / pt - 1)) < 1e-12
    for key, lat in (("eq31_d2q9_16", "D2Q9"), ("eq32_d3q19_4", "D3Q19")):
        q, a, d = _geom(lat)
        A = 1 + (2 + pm.c_gbi(lat) * 4 / pm.n_tn(a, d)) / pm.m_node(q, 8)
        B = 2 * pm.c_gb(lat) / a
        assert round(A, 3) == g[key][0] and round(B, 3) == g[key][1]
        for pt, al in ((0.9, 0.95), (0.6, 0.8)):
            assert abs(pm.tgb_memory(lat, 8, a, d, pt, al) - ((A + B * al) / pt - 1)) < 1e-12
    for lat in ("D2Q9", "D3Q19"):
        q, a, d = _geom(lat)
        assert round(pm.t2c_bandwidth(q, 8, a, d, 1.0), 4) == g["db_t2c_times_phit"][lat]
        assert round(pm.tgb_bandwidth(lat, 8, a, d, 1.0), 4) == g["db_tgb_times_phit"][lat]
    for lat, (num, den) in g["c_gb"].items():
        assert abs(pm.c_gb(lat) - num / den) < 1e-15
    for lat, v in g["c_gbi"].items():
        assert pm.c_gbi(lat) == v


def test_transaction_and_bu_examples():
    g = _golden()
    c = g["coarctation"]
    assert round(c["non_solid_nodes"] * pm.b_node(19, 8) / 32) == c["min_transactions_32B"]
    h = g["bu_headline"]
    # the implied GTX Titan peak: 6 GB GDDR5 at 3.004 GHz effective x2, 384-bit bus
    peak = 3.004e9 * 2 * 384 / 8
    assert round(pm.bandwidth_utilisation(h["mlups"], 19, h["s_d"], peak), 3) == h["bu"]
