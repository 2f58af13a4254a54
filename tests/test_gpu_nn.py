"""GPU layer kernels of the warm-start network against the FP64 NumPy
oracle.  Inputs and weights are rounded to BF16 first, so the differences
left are FP32 accumulation order and the BF16 rounding of outputs."""
import numpy as np
import pytest

from oracle import nn as onn
from paper_1703_08015_amd import nn

pytestmark = pytest.mark.gpu
rng = np.random.default_rng(7)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def bf(a):
    """Round to the nearest BF16 value (ties to even), as float64."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def dev(torch, a, dtype=None):
    dtype = dtype or torch.bfloat16
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.float().cpu().numpy().astype(np.float64)


def close(got, want, rel=1.5e-2):
    scale = max(np.max(np.abs(want)), 1e-30)
    err = np.max(np.abs(got - want)) / scale
    assert err <= rel, err


GRID = (4, 5, 6)  # (nz, ny, nx): 120 voxels, not a multiple of the 64-row tile


def rows_of(shape):
    return (shape[2], shape[1], shape[0])


@pytest.mark.parametrize("cin,cout,relu", [(8, 24, True), (24, 48, False), (48, 24, True), (16, 8, False)])
def test_conv3_forward_backward(torch, cin, cout, relu):
    x = bf(rng.normal(size=GRID + (cin,)))
    w = bf(rng.normal(size=(cout, 27, cin)) * 0.1)
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    y = torch.empty(GRID + (cout,), dtype=torch.bfloat16, device="cuda")
    nn.forward(nn.CONV3, nn.IDENT, rows_of(GRID), 27, cin, cout, dev(torch, x), cin, dev(torch, w), y, cout,
               bias=dev(torch, b, torch.float32), relu=relu)
    want = onn.conv3(x, w, b)
    if relu:
        want = onn.relu(want)
    close(host(y), want)
    # backward data and weights for an output gradient dy
    dy = bf(rng.normal(size=GRID + (cout,)))
    wt = torch.empty((cin, 27, cout), dtype=torch.bfloat16, device="cuda")
    nn.backward_weights(nn.CONV3, 27, cin, cout, dev(torch, w), wt)
    dx = torch.empty(GRID + (cin,), dtype=torch.bfloat16, device="cuda")
    nn.forward(nn.CONV3, nn.IDENT, rows_of(GRID), 27, cout, cin, dev(torch, dy), cout, wt, dx, cin)
    gx, gw, gb = onn.conv3_backward(x, w, dy)
    close(host(dx), gx)
    dw = torch.zeros((cout, 27, cin), dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    nn.wgrad(nn.CONV3, nn.IDENT, rows_of(GRID), 27, cin, cout, dev(torch, x), cin, dev(torch, dy), cout, dw, db)
    close(host(dw), gw, 2e-5)
    close(host(db), gb, 2e-5)


@pytest.mark.parametrize("grid,cin,cout,relu", [
    ((34, 36, 68), 24, 24, True),   # partial 8x8x4 bricks on every axis
    ((32, 32, 64), 8, 24, False),   # the first layer: 8 input channels
    ((32, 32, 64), 48, 24, True),   # decoder: concatenated skip and upsampled halves
    ((16, 32, 64), 64, 96, True),   # two 32-channel chunks, three 32-column groups
    ((16, 32, 64), 24, 64, False),  # 24-channel chunk with four 16-column groups
    ((16, 32, 64), 48, 48, True),   # one 48-channel chunk, three 16-column groups
    ((16, 32, 64), 48, 64, False),  # one 48-channel chunk, four 16-column groups
    ((36, 64, 64), 48, 24, True),   # 640 bricks, a partial brick along x
])
def test_conv3_brick_kernel(torch, grid, cin, cout, relu):
    """Grids with at least 256 8x8x4 bricks run the LDS-halo kernel; the data
    gradient through the flipped weights takes the same path."""
    x = bf(rng.normal(size=grid + (cin,)))
    w = bf(rng.normal(size=(cout, 27, cin)) * 0.1)
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    y = torch.empty(grid + (cout,), dtype=torch.bfloat16, device="cuda")
    nn.forward(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, dev(torch, x), cin, dev(torch, w), y, cout,
               bias=dev(torch, b, torch.float32), relu=relu)
    want = onn.conv3(x, w, b)
    if relu:
        want = onn.relu(want)
    close(host(y), want)
    dy = bf(rng.normal(size=grid + (cout,)))
    wt = torch.empty((cin, 27, cout), dtype=torch.bfloat16, device="cuda")
    nn.backward_weights(nn.CONV3, 27, cin, cout, dev(torch, w), wt)
    dx = torch.empty(grid + (cin,), dtype=torch.bfloat16, device="cuda")
    nn.forward(nn.CONV3, nn.IDENT, rows_of(grid), 27, cout, cin, dev(torch, dy), cout, wt, dx, cin)
    gx, _, _ = onn.conv3_backward(x, w, dy)
    close(host(dx), gx)


def test_conv3_wgrad_large_grid_split(torch):
    """Voxel counts far above one workgroup's chunk exercise the split reduction."""
    g = (24, 20, 16)
    x = bf(rng.normal(size=g + (24,)))
    dy = bf(rng.normal(size=g + (24,)))
    dw = torch.zeros((24, 27, 24), dtype=torch.float32, device="cuda")
    nn.wgrad(nn.CONV3, nn.IDENT, rows_of(g), 27, 24, 24, dev(torch, x), 24, dev(torch, dy), 24, dw)
    _, gw, _ = onn.conv3_backward(x, np.zeros((24, 27, 24)), dy)
    close(host(dw), gw, 2e-5)


@pytest.mark.parametrize("grid,cin,cout", [
    ((66, 62, 70), 24, 24),   # partial 8x4x4 bricks on every axis, 24-channel level
    ((64, 64, 64), 8, 24),    # the first layer: 8 input channels
    ((64, 64, 64), 48, 24),   # decoder: concatenated skip and upsampled halves
    ((64, 64, 64), 24, 48),   # second level, three 16-column fragments
    ((64, 64, 64), 48, 48),   # three output-channel tiles
])
def test_conv3_wgrad_brick_kernel(torch, grid, cin, cout):
    """Grids of at least 2048 8x4x4 bricks take the weight gradient that
    stages each brick's input halo and output gradient in LDS once for all 27
    taps; against the oracle's dW (FP32 sums over 2.6-2.9e5 voxels)."""
    x = bf(rng.normal(size=grid + (cin,)))
    dy = bf(rng.normal(size=grid + (cout,)))
    dw = torch.zeros((cout, 27, cin), dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    nn.wgrad(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, dev(torch, x), cin, dev(torch, dy), cout, dw, db)
    _, gw, gb = onn.conv3_backward(x, np.zeros((cout, 27, cin)), dy)
    close(host(dw), gw, 2e-5)
    close(host(db), gb, 2e-5)
    # with a workspace: per-block partial sums added in a fixed order, the same
    # result to rounding and identical from run to run
    n = nn.wgrad_workspace(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, cin, cout)
    assert n > 0
    ws = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    runs = []
    for _ in range(2):
        dw2 = torch.zeros((cout, 27, cin), dtype=torch.float32, device="cuda")
        nn.wgrad(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, dev(torch, x), cin, dev(torch, dy), cout, dw2,
                 ws=ws)
        runs.append(host(dw2))
    close(runs[0], gw, 2e-5)
    assert np.array_equal(runs[0], runs[1])
    with pytest.raises(Exception):
        nn.wgrad(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, dev(torch, x), cin, dev(torch, dy), cout, dw2,
                 ws=ws[: n - 1])


@pytest.mark.parametrize("grid,cin,cout,relu,gated", [
    ((16, 16, 16), 96, 96, True, False),   # the coarse levels: 128 blocks, 81 K steps
    ((8, 8, 8), 192, 96, False, True),     # 16 blocks, 162 K steps
    ((12, 10, 6), 64, 48, True, True),     # a grid thinner than a brick, ragged row count
])
def test_split_k_forward(torch, grid, cin, cout, relu, gated):
    """With a workspace, small grids split K over blocks: FP32 partial sums
    added in a fixed order with bias, ReLU and gate; against the oracle,
    identical from run to run, and close to the unsplit kernel."""
    x = bf(rng.normal(size=grid + (cin,)))
    w = bf(rng.normal(size=(cout, 27, cin)) * 0.05)
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    gate = bf(rng.normal(size=grid + (cout,)))
    want = onn.conv3(x, w, b)
    if relu:
        want = onn.relu(want)
    if gated:
        want = np.where(gate > 0, want, 0.0)
    n = nn.forward_workspace(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, cin, cout)
    assert n > 0
    ws = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    X, W, B, Gt = dev(torch, x), dev(torch, w), dev(torch, b, torch.float32), dev(torch, gate)
    kw = dict(gate=Gt, ldg=cout, gate_channels=cout) if gated else {}
    outs = []
    for w_s in (ws, ws, None):
        y = torch.empty(grid + (cout,), dtype=torch.bfloat16, device="cuda")
        nn.forward(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, X, cin, W, y, cout, bias=B, relu=relu, ws=w_s,
                   **kw)
        outs.append(y)
    torch.cuda.synchronize()
    for y in outs:
        close(host(y), want)
    assert torch.equal(outs[0].view(torch.int16), outs[1].view(torch.int16))
    if gated:
        assert not host(outs[0])[gate <= 0].any()
    with pytest.raises(nn.LbmError):
        nn.forward(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, X, cin, W, outs[0], cout, ws=ws[: n - 1])


@pytest.mark.parametrize("grid,cin,cout", [
    ((16, 16, 16), 96, 96),   # the coarse levels: few bricks, several channel tiles
    ((18, 22, 28), 48, 48),   # partial bricks on every axis
])
def test_conv3_wgrad_brick_small_grid_with_workspace(torch, grid, cin, cout):
    """With a workspace the brick weight gradient also takes small grids (at
    least 128 brick-run x channel-tile blocks); against the oracle's dW."""
    x = bf(rng.normal(size=grid + (cin,)))
    dy = bf(rng.normal(size=grid + (cout,)))
    n = nn.wgrad_workspace(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, cin, cout)
    assert n > 0
    ws = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    dw = torch.zeros((cout, 27, cin), dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    nn.wgrad(nn.CONV3, nn.IDENT, rows_of(grid), 27, cin, cout, dev(torch, x), cin, dev(torch, dy), cout, dw, db, ws=ws)
    _, gw, gb = onn.conv3_backward(x, np.zeros((cout, 27, cin)), dy)
    close(host(dw), gw, 2e-5)
    close(host(db), gb, 2e-5)


def test_thin_grids_avoid_bricks(torch):
    """A grid thinner than a brick along x (4 voxels) has enough bricks for
    both brick kernels but a halo that wraps past one period; the forward pass
    and the weight gradient take the generic kernels and match the oracle."""
    grid = (128, 64, 4)
    x = bf(rng.normal(size=grid + (24,)))
    w = bf(rng.normal(size=(24, 27, 24)) * 0.1)
    y = torch.empty(grid + (24,), dtype=torch.bfloat16, device="cuda")
    nn.forward(nn.CONV3, nn.IDENT, rows_of(grid), 27, 24, 24, dev(torch, x), 24, dev(torch, w), y, 24)
    close(host(y), onn.conv3(x, w, np.zeros(24)))
    dy = bf(rng.normal(size=grid + (24,)))
    _, gw, _ = onn.conv3_backward(x, np.zeros((24, 27, 24)), dy)
    n = nn.wgrad_workspace(nn.CONV3, nn.IDENT, rows_of(grid), 27, 24, 24, 24, 24)
    for ws in (None, torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")):
        dw = torch.zeros((24, 27, 24), dtype=torch.float32, device="cuda")
        nn.wgrad(nn.CONV3, nn.IDENT, rows_of(grid), 27, 24, 24, dev(torch, x), 24, dev(torch, dy), 24, dw, ws=ws)
        close(host(dw), gw, 2e-5)


@pytest.mark.parametrize("cin,cout", [(48, 24), (16, 8)])
def test_up2_forward_backward(torch, cin, cout):
    coarse = (2, 3, 2)
    fine = tuple(2 * v for v in coarse)
    x = bf(rng.normal(size=coarse + (cin,)))
    w = bf(rng.normal(size=(cout, 8, cin)) * 0.2)
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    # output written into the second half of a concatenation buffer
    cat = torch.zeros(fine + (2 * cout,), dtype=torch.bfloat16, device="cuda")
    nn.forward(nn.IDENT, nn.SCATTER2, rows_of(coarse), 8, cin, cout, dev(torch, x), cin, dev(torch, w), cat, 2 * cout,
               bias=dev(torch, b, torch.float32), y_offset=cout)
    close(host(cat)[..., cout:], onn.up2(x, w, b))
    assert not host(cat)[..., :cout].any()
    dyc = bf(rng.normal(size=fine + (2 * cout,)))
    dy = dyc[..., cout:]
    wt = torch.empty((cin, 8, cout), dtype=torch.bfloat16, device="cuda")
    nn.backward_weights(nn.SCATTER2, 8, cin, cout, dev(torch, w), wt)
    dx = torch.empty(coarse + (cin,), dtype=torch.bfloat16, device="cuda")
    nn.forward(nn.GATHER2, nn.IDENT, rows_of(coarse), 8, cout, cin, dev(torch, dyc), 2 * cout, wt, dx, cin,
               x_offset=cout)
    gx, gw, gb = onn.up2_backward(x, w, dy)
    close(host(dx), gx)
    dw = torch.zeros((cout, 8, cin), dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    nn.wgrad(nn.IDENT, nn.SCATTER2, rows_of(coarse), 8, cin, cout, dev(torch, x), cin, dev(torch, dyc), 2 * cout, dw,
             db, dy_offset=cout)
    close(host(dw), gw, 2e-5)
    close(host(db), gb, 2e-5)


@pytest.mark.parametrize("kind", ["dense", "up2", "gather2"])
def test_generic_wgrad_with_workspace(torch, kind):
    """The weight gradient of the 1x1, transposed (2x2x2 stride 2) and
    pooling-stride layers with a workspace: partial sums of up to 2048 blocks
    per tile added in two fixed-order passes; against the oracle, identical
    from run to run, and close to the atomic-add path."""
    if kind == "dense":
        src, dst, taps, rows, cin, cout = nn.IDENT, nn.IDENT, 1, (64, 64, 32), 24, 16
        x = bf(rng.normal(size=rows + (cin,)))
        dy = bf(rng.normal(size=rows + (cout,)))
        want = onn.dense_backward(x, np.zeros((cout, cin)), dy)[1][:, None, :]
    elif kind == "up2":
        src, dst, taps, rows, cin, cout = nn.IDENT, nn.SCATTER2, 8, (16, 16, 16), 48, 24
        x = bf(rng.normal(size=rows + (cin,)))
        dy = bf(rng.normal(size=tuple(2 * v for v in rows) + (cout,)))
        want = onn.up2_backward(x, np.zeros((cout, 8, cin)), dy)[1]
    else:
        src, dst, taps, rows, cin, cout = nn.GATHER2, nn.IDENT, 8, (16, 16, 16), 24, 48
        x = bf(rng.normal(size=tuple(2 * v for v in rows) + (cin,)))
        dy = bf(rng.normal(size=rows + (cout,)))
        # the pooling-stride layer is the transposed layer's backward-data pass:
        # its weight gradient is the transposed layer's, with x and dy swapped
        want = np.transpose(onn.up2_backward(dy, np.zeros((cin, 8, cout)), x)[1], (2, 1, 0))
    grid = (rows[2], rows[1], rows[0])
    n = nn.wgrad_workspace(src, dst, grid, taps, cin, cout, cin, cout)
    assert n > 0
    ws = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    X, DY = dev(torch, x), dev(torch, dy)
    runs = []
    want_db = dy.reshape(-1, cout).sum(axis=0)  # every output row once
    for w_s in (ws, ws, None):
        dw = torch.zeros((cout, taps, cin), dtype=torch.float32, device="cuda")
        db = torch.zeros(cout, dtype=torch.float32, device="cuda")
        nn.wgrad(src, dst, grid, taps, cin, cout, X, cin, DY, cout, dw, db, ws=w_s)
        runs.append(host(dw))
        close(host(db), want_db, 2e-5)
    close(runs[0], want, 2e-5)
    assert np.array_equal(runs[0], runs[1])
    close(runs[2], want, 2e-5)


@pytest.mark.parametrize("coarse,cin,cout", [
    ((6, 5, 7), 192, 96),    # 6 K steps held in registers, two column tiles, taps spread over blocks
    ((20, 18, 34), 48, 24),  # 256-row blocks, ragged last block
    ((9, 8, 10), 96, 48),    # 3 K steps
])
def test_up2_forward_sizes(torch, coarse, cin, cout):
    """The transposed convolution's forward kernel (A fragments held across its
    8 taps, double-buffered tap weights, tile stored through LDS) against the
    oracle, written into the second half of a concatenation buffer."""
    fine = tuple(2 * v for v in coarse)
    x = bf(rng.normal(size=coarse + (cin,)))
    w = bf(rng.normal(size=(cout, 8, cin)) * 0.1)
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    cat = torch.zeros(fine + (2 * cout,), dtype=torch.bfloat16, device="cuda")
    nn.forward(nn.IDENT, nn.SCATTER2, rows_of(coarse), 8, cin, cout, dev(torch, x), cin, dev(torch, w), cat, 2 * cout,
               bias=dev(torch, b, torch.float32), y_offset=cout)
    close(host(cat)[..., cout:], onn.up2(x, w, b))
    assert not host(cat)[..., :cout].any()


def test_backward_weights_batch(torch):
    """Several layers' backward-data weights in one launch equal the one-layer
    calls bit for bit (3x3x3, transposed and 1x1 layers of different sizes)."""
    specs = [(nn.CONV3, 27, 24, 48), (nn.SCATTER2, 8, 96, 48), (nn.IDENT, 1, 24, 16), (nn.CONV3, 27, 8, 24),
             (nn.CONV3, 27, 192, 192)]
    jobs, want = [], []
    for mode, taps, cin, cout in specs:
        w = dev(torch, bf(rng.normal(size=(cout, taps, cin))))
        a = torch.empty((cin, taps, cout), dtype=torch.bfloat16, device="cuda")
        b = torch.empty_like(a)
        nn.backward_weights(mode, taps, cin, cout, w, a)
        jobs.append((mode, taps, cin, cout, w, b))
        want.append(a)
    nn.backward_weights_batch(jobs)
    torch.cuda.synchronize()
    for (_, _, _, _, _, b), a in zip(jobs, want):
        assert torch.equal(a.view(torch.int16), b.view(torch.int16))
    with pytest.raises(nn.LbmError):
        nn.backward_weights_batch([(nn.CONV3, 8, 24, 24, jobs[0][4], jobs[0][5])])


@pytest.mark.parametrize("coarse,cin,cout", [
    ((9, 7, 6), 16, 48),    # one input fragment, three output fragments (the largest LDS tiles)
    ((6, 5, 11), 32, 48),   # two input fragments, three output fragments
    ((8, 8, 8), 192, 96),   # four input tiles of 48 channels, three output tiles of 32
])
def test_up2_wgrad_shapes(torch, coarse, cin, cout):
    """The transposed convolution's weight and bias gradients (one wavefront
    per tap) on ragged row counts and every tile shape, with and without a
    workspace, against the oracle."""
    fine = tuple(2 * v for v in coarse)
    x = bf(rng.normal(size=coarse + (cin,)))
    dy = bf(rng.normal(size=fine + (cout,)))
    _, gw, gb = onn.up2_backward(x, np.zeros((cout, 8, cin)), dy)
    n = nn.wgrad_workspace(nn.IDENT, nn.SCATTER2, rows_of(coarse), 8, cin, cout, cin, cout)
    assert n > 0
    for ws in (None, torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")):
        dw = torch.zeros((cout, 8, cin), dtype=torch.float32, device="cuda")
        db = torch.zeros(cout, dtype=torch.float32, device="cuda")
        nn.wgrad(nn.IDENT, nn.SCATTER2, rows_of(coarse), 8, cin, cout, dev(torch, x), cin, dev(torch, dy), cout, dw, db,
                 ws=ws)
        close(host(dw), gw, 2e-5)
        close(host(db), gb, 2e-5)


def test_head_dense_fp32_and_backward(torch):
    x = bf(rng.normal(size=GRID + (24,)))
    w = np.zeros((8, 1, 24))
    w[:4] = bf(rng.normal(size=(4, 1, 24)))
    b = np.zeros(8)
    b[:4] = rng.normal(size=4).astype(np.float32)
    out = torch.empty(GRID + (4,), dtype=torch.float32, device="cuda")
    nn.forward(nn.IDENT, nn.IDENT, rows_of(GRID), 1, 24, 4, dev(torch, x), 24, dev(torch, w), out, 4,
               bias=dev(torch, b, torch.float32), y_fp32=True)
    close(host(out), onn.dense(x, w[:4, 0], b[:4]), 1e-5)
    dy = np.zeros(GRID + (8,))
    dy[..., :4] = bf(rng.normal(size=GRID + (4,)))
    dw = torch.zeros((8, 1, 24), dtype=torch.float32, device="cuda")
    db = torch.zeros(8, dtype=torch.float32, device="cuda")
    nn.wgrad(nn.IDENT, nn.IDENT, rows_of(GRID), 1, 24, 8, dev(torch, x), 24, dev(torch, dy), 8, dw, db)
    gx, gw, gb = onn.dense_backward(x, w[:, 0], dy)
    close(host(dw)[:, 0], gw, 2e-5)
    close(host(db), gb, 2e-5)
    wt = torch.empty((24, 1, 8), dtype=torch.bfloat16, device="cuda")
    nn.backward_weights(nn.IDENT, 1, 24, 8, dev(torch, w), wt)
    dx = torch.empty(GRID + (24,), dtype=torch.bfloat16, device="cuda")
    nn.forward(nn.IDENT, nn.IDENT, rows_of(GRID), 1, 8, 24, dev(torch, dy), 8, wt, dx, 24)
    close(host(dx), gx)


def test_maxpool_relu_mse_adam(torch):
    coarse = (2, 2, 3)
    fine = tuple(2 * v for v in coarse)
    x = bf(rng.normal(size=fine + (16,)))
    y = torch.empty(coarse + (16,), dtype=torch.bfloat16, device="cuda")
    arg = torch.empty(coarse + (16,), dtype=torch.uint8, device="cuda")
    nn.maxpool2(rows_of(coarse), 16, dev(torch, x), 16, y, 16, arg)
    wy, warg = onn.maxpool2(x)
    assert np.array_equal(host(y), wy) and np.array_equal(arg.cpu().numpy(), warg)
    dy = bf(rng.normal(size=coarse + (16,)))
    base = bf(rng.normal(size=fine + (16,)))
    dx = dev(torch, base)
    nn.maxpool2_backward(rows_of(coarse), 16, dev(torch, dy), 16, arg, dx, 16, accumulate=True)
    close(host(dx), base + onn.maxpool2_backward(warg, dy), 1e-2)
    nn.maxpool2_backward(rows_of(coarse), 16, dev(torch, dy), 16, arg, dx, 16)
    assert np.array_equal(host(dx), onn.maxpool2_backward(warg, dy))
    # relu backward
    yv = bf(rng.normal(size=(40, 8)))
    g = bf(rng.normal(size=(40, 8)))
    gd = dev(torch, g)
    nn.relu_backward(40, 8, dev(torch, yv), 8, gd, 8)
    assert np.array_equal(host(gd), onn.relu_backward(yv, g))
    # masked MSE
    pred = rng.normal(size=(50, 4)).astype(np.float32)
    targ = rng.normal(size=(50, 4)).astype(np.float32)
    solid = (rng.random(50) < 0.3).astype(np.uint8)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    dp = torch.empty((50, 8), dtype=torch.bfloat16, device="cuda")
    nn.mse(50, 4, dev(torch, pred, torch.float32), dev(torch, targ, torch.float32), dev(torch, solid, torch.uint8),
           0.5, dp, 8, loss)
    wl, wg = onn.masked_mse(pred.astype(np.float64), targ.astype(np.float64), solid.astype(bool))
    assert np.isclose(float(loss.item()), wl, rtol=1e-5)
    close(host(dp)[:, :4], 0.5 * wg, 1e-2)
    assert not host(dp)[:, 4:].any()
    # Adam (FP32) against the FP64 definition
    p0 = rng.normal(size=300).astype(np.float32)
    gr = rng.normal(size=300).astype(np.float32)
    P, M, V = [dev(torch, a, torch.float32) for a in (p0, np.zeros(300), np.zeros(300))]
    G = dev(torch, gr, torch.float32)
    p16 = torch.empty(300, dtype=torch.bfloat16, device="cuda")
    pp, mm, vv = p0.astype(np.float64), np.zeros(300), np.zeros(300)
    for step in (1, 2, 3):
        nn.adam(P, M, V, G, p16, 1e-2, step)
        pp, mm, vv = onn.adam(pp, mm, vv, gr.astype(np.float64), 1e-2, 0.9, 0.999, 1e-8, step)
    assert np.allclose(host(P), pp, rtol=1e-5, atol=1e-6)
    assert np.array_equal(host(p16), bf(host(P)))


@pytest.mark.parametrize("channels,ld,off", [(24, 48, 0), (24, 48, 24), (16, 16, 0), (12, 12, 0), (8, 20, 4)])
def test_pool_and_relu_paths(torch, channels, ld, off):
    """Max pooling, its backward and the ReLU backward on both kernel forms:
    whole 16-byte channel groups (channels, row stride and offset multiples of
    8) and the element-wise fallback (12 channels; stride 20).  Inputs are
    ReLU outputs, so ties at 0 are common: the first corner wins, as in the
    oracle, and the results are exact."""
    coarse = (3, 5, 4)
    fine = tuple(2 * v for v in coarse)
    xf = np.zeros(fine + (ld,))
    xf[..., off:off + channels] = np.maximum(bf(rng.normal(size=fine + (channels,))), 0.0)
    y = torch.zeros(coarse + (channels,), dtype=torch.bfloat16, device="cuda")
    arg = torch.empty(coarse + (channels,), dtype=torch.uint8, device="cuda")
    nn.maxpool2(rows_of(coarse), channels, dev(torch, xf), ld, y, channels, arg, x_offset=off)
    wy, warg = onn.maxpool2(xf[..., off:off + channels])
    assert np.array_equal(host(y), wy) and np.array_equal(arg.cpu().numpy(), warg)
    dy = bf(rng.normal(size=coarse + (channels,)))
    base = bf(rng.normal(size=fine + (ld,)))
    dx = dev(torch, base)
    nn.maxpool2_backward(rows_of(coarse), channels, dev(torch, dy), channels, arg, dx, ld, accumulate=True,
                         dx_offset=off)
    want = base.copy()
    want[..., off:off + channels] = bf(base[..., off:off + channels] + onn.maxpool2_backward(warg, dy))
    assert np.array_equal(host(dx), want)
    g = bf(rng.normal(size=fine + (ld,)))
    gd = dev(torch, g)
    n = int(np.prod(fine))
    nn.relu_backward(n, channels, dev(torch, xf), ld, gd, ld, y_offset=off, dy_offset=off)
    want = g.copy()
    want[..., off:off + channels] = onn.relu_backward(xf[..., off:off + channels], g[..., off:off + channels])
    assert np.array_equal(host(gd), want)


@pytest.mark.parametrize("src,grid,taps,cin,cout,gate_ch,ldg,goff", [
    (nn.CONV3, (4, 5, 6), 27, 24, 48, 24, 48, 0),     # generic kernel, the skip half of a concat gradient
    (nn.CONV3, (4, 5, 6), 27, 16, 24, 24, 32, 8),     # generic kernel, gate rows wider than the output
    (nn.IDENT, (4, 5, 6), 1, 16, 24, 24, 24, 0),      # 1x1 (the head's backward-data pass)
    (nn.GATHER2, (2, 3, 3), 8, 24, 48, 48, 48, 0),    # a transposed conv's backward-data pass
    (nn.CONV3, (32, 36, 68), 27, 24, 24, 24, 24, 0),  # brick kernel, partial bricks
    (nn.CONV3, (32, 32, 64), 27, 48, 48, 24, 48, 0),  # brick kernel, gate on half the channels
])
def test_gate_equals_relu_backward(torch, src, grid, taps, cin, cout, gate_ch, ldg, goff):
    """A gated forward pass writes exactly what the ungated pass followed by
    lbm_nn_relu_backward on its first gate_ch channels writes (bit for bit):
    the fused ReLU derivative of the backward-data passes."""
    fine = tuple(2 * v for v in grid) if src == nn.GATHER2 else grid
    x = bf(rng.normal(size=fine + (cin,)))
    w = bf(rng.normal(size=(cout, taps, cin)) * 0.1)
    gate = bf(rng.normal(size=grid + (ldg,)))
    gate[..., goff] = 0.0  # exact zeros close the gate too
    y0 = torch.empty(grid + (cout,), dtype=torch.bfloat16, device="cuda")
    y1 = torch.empty_like(y0)
    X, W, Gt = dev(torch, x), dev(torch, w), dev(torch, gate)
    nn.forward(src, nn.IDENT, rows_of(grid), taps, cin, cout, X, cin, W, y0, cout)
    nn.forward(src, nn.IDENT, rows_of(grid), taps, cin, cout, X, cin, W, y1, cout, gate=Gt, ldg=ldg,
               gate_channels=gate_ch, gate_offset=goff)
    n = int(np.prod(grid))
    nn.relu_backward(n, gate_ch, Gt, ldg, y0, cout, y_offset=goff)
    torch.cuda.synchronize()
    a, b = y0.cpu(), y1.cpu()
    assert torch.equal(a.view(torch.int16), b.view(torch.int16))
    assert (host(y1)[..., :gate_ch][gate[..., goff:goff + gate_ch] <= 0] == 0).all()
    with pytest.raises(nn.LbmError):
        nn.forward(src, nn.IDENT, rows_of(grid), taps, cin, cout, X, cin, W, y1, cout, gate=Gt, ldg=ldg,
                   gate_channels=cout + 8)


def test_force_mix(torch):
    y = rng.normal(size=(30, 12)).astype(np.float32)
    d = np.array([0.36, -0.48, 0.8])
    p = torch.empty((30, 4), dtype=torch.float32, device="cuda")
    nn.mix(dev(torch, y, torch.float32), d, p)
    want = sum(d[j] * y[:, 4 * j:4 * j + 4].astype(np.float64) for j in range(3))
    close(host(p), want, 1e-6)
    dp = np.zeros((30, 8))
    dp[:, :4] = bf(rng.normal(size=(30, 4)))
    dy = torch.empty((30, 16), dtype=torch.bfloat16, device="cuda")
    nn.mix_backward(dev(torch, dp), 8, d, dy, 16)
    hdy = host(dy)
    for j in range(3):
        close(hdy[:, 4 * j:4 * j + 4], d[j] * dp[:, :4], 1e-2)
    assert not hdy[:, 12:].any()


def test_encode_decode(torch):
    solid = (rng.random(GRID) < 0.4).astype(np.uint8)
    x = torch.empty(GRID + (8,), dtype=torch.bfloat16, device="cuda")
    d = np.array([0.6, -0.8, 0.0])
    nn.encode_input(dev(torch, solid, torch.uint8), d, x)
    hx = host(x)
    assert np.array_equal(hx[..., 0], solid.astype(float))
    assert np.allclose(hx[solid == 0][:, 1:4], bf(d)) and not hx[solid == 1][:, 1:].any()
    pred = rng.normal(size=GRID + (4,)).astype(np.float32)
    rho = torch.empty(GRID, dtype=torch.float64, device="cuda")
    u = torch.empty((3,) + GRID, dtype=torch.float64, device="cuda")
    scratch = torch.empty(2, dtype=torch.float64, device="cuda")
    nn.decode_output(dev(torch, pred, torch.float32), dev(torch, solid, torch.uint8), 1.0, 1e-3, rho, u, scratch)
    r, uu = rho.cpu().numpy(), u.cpu().numpy()
    fl = solid == 0
    assert np.isclose(r[fl].sum(), fl.sum(), rtol=1e-12) and np.all(r[~fl] == 0)
    want_u = np.moveaxis(pred[..., 1:].astype(np.float64) * 1e-3, -1, 0)
    assert np.allclose(uu[:, fl], want_u[:, fl], rtol=1e-12) and not uu[:, ~fl].any()
    raw = 1.0 + 1e-3 * pred[..., 0].astype(np.float64)
    assert np.allclose(r[fl], raw[fl] - raw[fl].mean() + 1.0, rtol=1e-12)


def _oracle_unet(net, x, dout):
    """The same network from the FP64 oracle layers, rounding activations and
    activation gradients to BF16 where the GPU stores them.  Returns the
    output and the gradient of every parameter (in net.params order)."""
    L, C = net.L, net.C
    P = lambda p: p.p.cpu().numpy().astype(np.float64)
    W = lambda p: bf(P(p))
    A = {}
    src = x
    for l in range(L):
        (w1, b1), (w2, b2) = net.enc[l]
        if l > 0:
            A["pool", l], A["arg", l] = onn.maxpool2(A["cat", l - 1])
            src = A["pool", l]
        A["in", l] = src
        A["e1", l] = bf(onn.relu(onn.conv3(src, W(w1), P(b1))))
        A["cat", l] = bf(onn.relu(onn.conv3(A["e1", l], W(w2), P(b2))))
    below = A["cat", L - 1]
    for k, l in enumerate(range(L - 2, -1, -1)):
        uw, ub = net.up[k]
        (w1, b1), (w2, b2) = net.dec[k]
        A["below", l] = below
        A["up", l] = bf(onn.up2(below, W(uw), P(ub)))
        A["catfull", l] = np.concatenate([A["cat", l], A["up", l]], axis=-1)
        A["d1", l] = bf(onn.relu(onn.conv3(A["catfull", l], W(w1), P(b1))))
        A["d2", l] = bf(onn.relu(onn.conv3(A["d1", l], W(w2), P(b2))))
        below = A["d2", l]
    hw, hb = net.head
    out = onn.dense(below, W(hw)[:, 0], P(hb))[..., :net.out_ch]
    grads = {}
    g_below, grads["hw"], grads["hb"] = onn.dense_backward(below, W(hw)[:, 0], dout)
    g_below = bf(g_below)
    gcat = {}
    for l in range(0, L - 1):
        idx = L - 2 - l
        uw, ub = net.up[idx]
        (w1, b1), (w2, b2) = net.dec[idx]
        g = bf(onn.relu_backward(A["d2", l], g_below))
        gx, grads["dec", idx, 1, "w"], grads["dec", idx, 1, "b"] = onn.conv3_backward(A["d1", l], W(w2), g)
        g = bf(onn.relu_backward(A["d1", l], bf(gx)))
        gx, grads["dec", idx, 0, "w"], grads["dec", idx, 0, "b"] = onn.conv3_backward(A["catfull", l], W(w1), g)
        gx = bf(gx)
        gcat[l] = gx[..., :C[l]]
        gup = gx[..., C[l]:]
        gb_, grads["up", idx, "w"], grads["up", idx, "b"] = onn.up2_backward(A["below", l], W(uw), gup)
        g_below = bf(gb_)
    gcat[L - 1] = g_below
    for l in range(L - 1, -1, -1):
        (w1, b1), (w2, b2) = net.enc[l]
        g = bf(onn.relu_backward(A["cat", l], gcat[l]))
        gx, grads["enc", l, 1, "w"], grads["enc", l, 1, "b"] = onn.conv3_backward(A["e1", l], W(w2), g)
        g = bf(onn.relu_backward(A["e1", l], bf(gx)))
        gx, grads["enc", l, 0, "w"], grads["enc", l, 0, "b"] = onn.conv3_backward(A["in", l], W(w1), g)
        if l > 0:
            gcat[l - 1] = bf(gcat[l - 1] + onn.maxpool2_backward(A["arg", l], bf(gx)))
    order = []
    for l in range(L):
        for j in range(2):
            order += [grads["enc", l, j, "w"], grads["enc", l, j, "b"]]
    for k in range(L - 1):
        order += [grads["up", k, "w"], grads["up", k, "b"]]
    for k in range(L - 1):
        for j in range(2):
            order += [grads["dec", k, j, "w"], grads["dec", k, j, "b"]]
    order += [grads["hw"][:, None, :], grads["hb"]]
    return out, order


def test_unet_forward_and_gradients_match_oracle(torch):
    from paper_1703_08015_amd.unet import UNet
    # inputs from a generator of their own, so that they do not depend on what
    # the other tests drew: on some draws a BF16 rounding or ReLU decision near
    # a tie goes the other way on the two sides (FP32 against FP64 sums), and
    # the flip carries down the backward chain (worst gradient deviation 0 to
    # 0.1 of its maximum over nine draws, 1e-4 or less on most)
    r = np.random.default_rng(100)
    net = UNet(levels=3, base=8, seed=3)
    g = (8, 8, 8)
    x = np.zeros(g + (8,))
    x[..., :4] = bf(r.normal(size=g + (4,)))
    out = net.forward(dev(torch, x))
    dout = np.zeros(g + (8,))
    dout[..., :4] = bf(r.normal(size=g + (4,)))
    net.zero_grad()
    net.backward(dev(torch, dout))
    torch.cuda.synchronize()
    want_out, want_grads = _oracle_unet(net, x, dout)
    close(host(out), want_out, 2e-2)
    assert len(want_grads) == len(net.params)
    for k, (p, wg) in enumerate(zip(net.params, want_grads)):
        got = host(p.g)
        assert got.shape == wg.shape, k
        close(got, wg, 6e-2)


@pytest.mark.parametrize("periodic", [7, 0, 5])
def test_distance_and_geometry_encoding(torch, periodic):
    from paper_1703_08015_amd import inputs
    solid, _ = inputs.spheres_3d((20, 12, 16), 0.55, 2.0, 4.0, seed=11,
                                 periodic=tuple(bool(periodic >> a & 1) for a in range(3)))
    solid[0, :3, :3] = True  # a few isolated bits near an edge
    want = onn.distance(solid, periodic)
    sd = torch.from_numpy(solid.astype(np.uint8)).cuda()
    dist = torch.empty(solid.shape, dtype=torch.float32, device="cuda")
    tmp = torch.empty_like(dist)
    nn.distance(sd, dist, tmp, sweeps=64, periodic=periodic)
    got = dist.cpu().numpy().astype(np.float64)
    fin = np.isfinite(want)
    assert np.allclose(got[fin], want[fin], rtol=1e-6, atol=1e-6)
    assert np.all(got[~fin] >= 1e29)
    # too few sweeps leave far nodes unreached, never below the true distance
    nn.distance(sd, dist, tmp, sweeps=2, periodic=periodic)
    few = dist.cpu().numpy().astype(np.float64)
    assert np.all(few[fin] >= want[fin] - 1e-5) and np.all(few[want <= 2.0] <= want[want <= 2.0] + 1e-5)
    nn.distance(sd, dist, tmp, sweeps=64, periodic=periodic)
    x = torch.empty(solid.shape + (8,), dtype=torch.bfloat16, device="cuda")
    nn.encode_geometry(sd, dist, 0.25, 3.0, x)
    ref = onn.encode_geometry(solid, np.where(fin, want, 1e30), 0.25, 3.0)
    close(host(x), bf(ref), rel=1e-2)
    assert np.all(host(x)[..., 3:] == 0)


def test_unet_side_stream_weight_gradients_bit_exact(torch):
    """Weight gradients on the side stream, overlapping the backward-data
    passes, give the same bits as the one-stream order, over two backward
    passes in a row (the second reusing every buffer of the first).  Bias
    gradients add one FP32 atomic per block and column, in whatever order the
    blocks finish, so they agree to the rounding of that sum."""
    from paper_1703_08015_amd.unet import UNet
    g = (32, 32, 64)
    x = torch.from_numpy(bf(rng.normal(size=g + (8,)))).to(torch.bfloat16).cuda()
    douts = [torch.from_numpy(bf(rng.normal(size=g + (8,)) * 0.1)).to(torch.bfloat16).cuda() for _ in range(2)]
    grads = {}
    for overlap in (False, True):
        net = UNet(levels=4, base=24, seed=5)
        net.overlap, net.overlap_min_voxels = overlap, 0
        got = []
        for d in douts:
            net.forward(x)
            net.zero_grad()
            net.backward(d)
            got.append([p.g.clone() for p in net.params])
        torch.cuda.synchronize()
        grads[overlap] = got
    shapes = [p.p.dim() for p in net.params]
    for a, b in zip(grads[False], grads[True]):
        for k, (ga, gb) in enumerate(zip(a, b)):
            if shapes[k] > 1:
                assert torch.equal(ga, gb), k
            else:
                scale = float(ga.abs().max()) + 1e-30
                assert float((ga - gb).abs().max()) <= 1e-4 * scale, k
