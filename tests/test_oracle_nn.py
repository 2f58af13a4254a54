"""Pins of the FP64 NumPy layer oracle: library routines (scipy.ndimage
correlate in wrap mode), finite differences of every backward pass, adjoint
identities, and the closed-form first Adam step."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import nn

rng = np.random.default_rng(42)


def test_conv3_is_wrapped_correlation():
    x = rng.normal(size=(5, 6, 4, 3))
    w = rng.normal(size=(2, 27, 3))
    b = rng.normal(size=2)
    y = nn.conv3(x, w, b)
    for n in range(2):
        want = np.full(x.shape[:3], b[n])
        for c in range(3):
            k = w[n, :, c].reshape(3, 3, 3)  # (dz, dy, dx) kernel, correlation
            want += ndimage.correlate(x[..., c], k, mode="wrap")
        assert np.allclose(y[..., n], want, rtol=1e-12, atol=1e-12)


def test_up2_places_each_corner():
    x = rng.normal(size=(2, 3, 2, 4))
    w = rng.normal(size=(3, 8, 4))
    y = nn.up2(x, w)
    assert y.shape == (4, 6, 4, 3)
    for a, (az, ay, ax) in enumerate(nn.CORNERS):
        assert np.allclose(y[1 * 2 + az, 2 * 2 + ay, 1 * 2 + ax], x[1, 2, 1] @ w[:, a, :].T)


def test_maxpool_brute_force():
    x = rng.normal(size=(4, 2, 6, 3))
    y, arg = nn.maxpool2(x)
    for z in range(2):
        for yy in range(1):
            for xx in range(3):
                for c in range(3):
                    blk = [x[2 * z + az, 2 * yy + ay, 2 * xx + ax, c] for (az, ay, ax) in nn.CORNERS]
                    assert y[z, yy, xx, c] == max(blk) and arg[z, yy, xx, c] == int(np.argmax(blk))


def _fd_check(f, backward, args, k, eps=1e-6):
    """d/dtheta <f(args), r> by central differences against backward()."""
    y = f(*args)
    r = rng.normal(size=y.shape)
    grads = backward(r)
    base = [a.copy() for a in args]
    d = rng.normal(size=base[k].shape)
    p = [a.copy() for a in base]
    m = [a.copy() for a in base]
    p[k] = p[k] + eps * d
    m[k] = m[k] - eps * d
    fd = (np.sum(f(*p) * r) - np.sum(f(*m) * r)) / (2 * eps)
    an = np.sum(grads[k] * d)
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)


def test_conv3_gradients_match_finite_differences():
    x = rng.normal(size=(3, 4, 5, 2))
    w = rng.normal(size=(3, 27, 2))
    b = rng.normal(size=3)
    f = lambda x_, w_, b_: nn.conv3(x_, w_, b_)
    bw = lambda r: nn.conv3_backward(x, w, r)
    for k in range(3):
        _fd_check(f, bw, [x, w, b], k)


def test_up2_gradients_match_finite_differences():
    x = rng.normal(size=(2, 3, 2, 3))
    w = rng.normal(size=(2, 8, 3))
    b = rng.normal(size=2)
    f = lambda x_, w_, b_: nn.up2(x_, w_, b_)
    bw = lambda r: nn.up2_backward(x, w, r)
    for k in range(3):
        _fd_check(f, bw, [x, w, b], k)


def test_dense_and_maxpool_gradients():
    x = rng.normal(size=(2, 2, 4, 5))
    w = rng.normal(size=(3, 5))
    b = rng.normal(size=3)
    for k in range(3):
        _fd_check(lambda x_, w_, b_: nn.dense(x_, w_, b_), lambda r: nn.dense_backward(x, w, r), [x, w, b], k)
    xp = rng.normal(size=(4, 4, 2, 2))  # continuous values: no ties
    _, arg = nn.maxpool2(xp)
    _fd_check(lambda x_: nn.maxpool2(x_)[0], lambda r: (nn.maxpool2_backward(arg, r),), [xp], 0)


def test_up2_is_adjoint_of_strided_gather():
    """<up2(x), y> = <x, G(y)> with G(y)[v] = sum_a y[2v + a] w_a (the backward data map)."""
    x = rng.normal(size=(2, 2, 3, 4))
    w = rng.normal(size=(5, 8, 4))
    y = rng.normal(size=(4, 4, 6, 5))
    gx, _, _ = nn.up2_backward(x, w, y)
    assert np.isclose(np.sum(nn.up2(x, w) * y), np.sum(x * gx), rtol=1e-12)


def test_masked_mse_and_relu():
    p = rng.normal(size=(2, 3, 2, 4))
    t = rng.normal(size=(2, 3, 2, 4))
    solid = rng.random((2, 3, 2)) < 0.4
    loss, g = nn.masked_mse(p, t, solid)
    assert np.isclose(loss, ((p - t) ** 2)[~solid].sum())
    assert np.all(g[solid] == 0)
    y = nn.relu(p)
    assert np.all(nn.relu_backward(y, t)[p <= 0] == 0)


def test_adam_first_step_moves_by_lr_times_sign():
    g = rng.normal(size=50)
    p0 = rng.normal(size=50)
    p, m, v = nn.adam(p0, np.zeros(50), np.zeros(50), g, lr=1e-3, b1=0.9, b2=0.999, eps=0.0, step=1)
    assert np.allclose(p, p0 - 1e-3 * np.sign(g), rtol=0, atol=1e-15)


def _chamfer_closed_form(a, b, c):
    """Cost of offset (a, b, c) with unit axis steps and sqrt(2) diagonal
    steps in a plane: each diagonal step replaces two axis steps, and at most
    min(floor((a+b+c)/2), b+c) of them fit (a >= b >= c >= 0)."""
    a, b, c = sorted((abs(a), abs(b), abs(c)), reverse=True)
    k = min((a + b + c) // 2, b + c)
    return (a + b + c) - (2 - np.sqrt(2)) * k


def test_distance_from_one_solid_node_has_the_closed_form():
    n = 9
    solid = np.zeros((n, n, n), bool)
    solid[4, 4, 4] = True
    d = nn.distance(solid, periodic=0)
    for z in range(n):
        for y in range(n):
            for x in range(n):
                assert np.isclose(d[z, y, x], _chamfer_closed_form(x - 4, y - 4, z - 4), rtol=0, atol=1e-12)
    # periodic: the minimum image
    dp = nn.distance(solid, periodic=7)
    assert np.isclose(dp[0, 0, 0], _chamfer_closed_form(4, 4, 4))
    assert np.isclose(dp[8, 0, 4], _chamfer_closed_form(4, 4, 0))


def test_distance_is_zero_on_solid_and_one_lipschitz_along_links():
    solid = rng.random((6, 7, 8)) < 0.1
    d = nn.distance(solid)
    assert np.all(d[solid] == 0) and np.all(d[~solid] >= 1)
    for dx, dy, dz in nn.LINKS:
        sh = np.roll(d, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        assert np.all(np.abs(sh - d) <= np.sqrt(abs(dx) + abs(dy) + abs(dz)) + 1e-12)
    assert np.all(np.isinf(nn.distance(np.zeros((3, 3, 3), bool))))


def test_layers_at_chosen_voxels_equal_the_whole_grid():
    """conv3_at, up2_at and maxpool2_at are the whole-grid layers read at chosen voxels, wrap included."""
    x = rng.normal(size=(6, 4, 8, 3))
    w = rng.normal(size=(5, 27, 3))
    b = rng.normal(size=5)
    nodes = np.argwhere(np.ones(x.shape[:3], bool))
    full = nn.conv3(x, w, b)
    assert np.allclose(nn.conv3_at(x, w, b, nodes), full[nodes[:, 0], nodes[:, 1], nodes[:, 2]], rtol=1e-13,
                       atol=1e-13)
    wu = rng.normal(size=(2, 8, 3))
    fine = nn.up2(x, wu, b[:2])
    fn = np.argwhere(np.ones(fine.shape[:3], bool))
    assert np.allclose(nn.up2_at(x, wu, b[:2], fn), fine[fn[:, 0], fn[:, 1], fn[:, 2]], rtol=1e-13, atol=1e-13)
    pooled, _ = nn.maxpool2(x)
    pn = np.argwhere(np.ones(pooled.shape[:3], bool))
    assert np.array_equal(nn.maxpool2_at(x, pn), pooled[pn[:, 0], pn[:, 1], pn[:, 2]])
