"""The warm-start network at its full size, in the configuration bench.py
times: the 4-level, 24-base U-Net with the force-linear head at 128^3.

* Every layer kernel the forward pass launches, at the grid, channel counts,
  strides and buffer offsets it has in the network (17 convolutions and
  up-samplings, 3 poolings, the head), on seeded random BF16 inputs, the
  network's BF16 weights and seeded FP32 biases, against the FP64 layer
  oracle on sampled voxels (2,000 per layer, all voxels where a grid has
  fewer).  BF16 outputs are within their rounding, 2^-8 of the value, plus
  1e-4 of the layer's largest output for FP32 accumulation order; pooling is
  exact; the FP32 head output within 1e-5 of its largest value.
* Circular padding, stride-2 pooling and stride-2 up-sampling make the
  network commute with shifts by multiples of 8 voxels (2^(levels-1)): the
  output of the shifted input is the shifted output, bit for bit, which
  checks every kernel's indexing over the whole grid.
"""
import sys

import numpy as np
import pytest

from oracle import nn as onn
from paper_1703_08015_amd import inputs, nn, warmstart

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def run(torch):
    """One forward pass at 128^3: the network, the input and the pass's activations."""
    net = warmstart.make_net(levels=4, base=24, seed=0)
    # biases start at zero; give them seeded values so that every bias path is checked
    gen = torch.Generator().manual_seed(5)
    for p in net.params:
        if p.b16 is None:
            p.p.copy_((torch.randn(p.p.shape, generator=gen) * 0.05).to(p.p.device))
    m, _ = inputs.spheres_3d(128, 0.5, 4.0, 12.0, seed=1)
    sm = warmstart.Sample(torch, m, (1e-6, 0.0, 0.0))
    x = warmstart.encode(torch, sm)
    mixed = net.forward_mixed(x, sm.dir).clone()
    torch.cuda.synchronize()
    return net, x, sm, mixed


def _h(t):
    return t.float().cpu().numpy().astype(np.float64)


def _nodes(shape, n, seed):
    rng = np.random.default_rng(seed)
    size = int(np.prod(shape))
    flat = np.arange(size) if size <= n else rng.choice(size, size=n, replace=False)
    return np.stack(np.unravel_index(flat, shape), 1)


def _at(a, nodes):
    return a[nodes[:, 0], nodes[:, 1], nodes[:, 2]]


def _check_bf16(got, want, what):
    bar = 2.0 ** -8 * np.abs(want) + 1e-4 * np.max(np.abs(want))
    _log(what, "max error / bar", float(np.max(np.abs(got - want) / bar)))
    assert np.all(np.abs(got - want) <= bar), what
    assert np.max(np.abs(want)) > 0, what


def _bf(a):
    """Round to the nearest BF16 value (ties to even), as float64."""
    a32 = np.asarray(a, np.float32)
    b = a32.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def test_every_layer_kernel_on_sampled_voxels(torch, run):
    net = run[0]
    L, C = net.L, net.C
    grids = [tuple(128 >> l for _ in range(3)) for l in range(L)]
    rng = np.random.default_rng(31)
    bf16 = dict(dtype=torch.bfloat16, device="cuda")

    def rnd(shape):
        return _bf(rng.normal(size=shape))

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(**bf16)

    def rows(g):
        return (g[2], g[1], g[0])

    W = lambda p: _h(p.b16)  # noqa: E731
    B = lambda p: _h(p.p)  # noqa: E731

    def conv(l, cin, cout, w, b, ld_in, width, what):
        """A 3x3x3 layer on level l: input ld_in wide, output written at offset 0 of a width-wide buffer."""
        g = grids[l]
        x = rnd(g + (ld_in,))
        y = torch.zeros(g + (width,), **bf16)
        nn.forward(nn.CONV3, nn.IDENT, rows(g), 27, cin, cout, dev(x), ld_in, w.b16, y, width, bias=b.p, relu=True)
        nodes = _nodes(g, 2000, seed=int(rng.integers(1 << 30)))
        _check_bf16(_at(_h(y), nodes)[:, :cout], onn.relu(onn.conv3_at(x[..., :cin], W(w), B(b), nodes)), what)

    for l in range(L):
        (w1, b1), (w2, b2) = net.enc[l]
        cin = net.in_ch if l == 0 else C[l - 1]
        conv(l, cin, C[l], w1, b1, cin, C[l], "enc %d conv 1" % l)
        conv(l, C[l], C[l], w2, b2, C[l], 2 * C[l] if l < L - 1 else C[l], "enc %d conv 2" % l)
        if l > 0:
            # pooling reads the skip half of the level above's concatenation buffer
            src = rnd(grids[l - 1] + (2 * C[l - 1],))
            pool = torch.empty(grids[l] + (C[l - 1],), **bf16)
            arg = torch.empty(grids[l] + (C[l - 1],), dtype=torch.uint8, device="cuda")
            nn.maxpool2(rows(grids[l]), C[l - 1], dev(src), 2 * C[l - 1], pool, C[l - 1], arg)
            nodes = _nodes(grids[l], 2000, seed=400 + l)
            assert np.array_equal(_at(_h(pool), nodes), onn.maxpool2_at(src[..., :C[l - 1]], nodes)), "pool %d" % l
    for k, l in enumerate(range(L - 2, -1, -1)):
        uw, ub = net.up[k]
        (w1, b1), (w2, b2) = net.dec[k]
        below = rnd(grids[l + 1] + (C[l + 1],))
        cat = torch.zeros(grids[l] + (2 * C[l],), **bf16)
        nn.forward(nn.IDENT, nn.SCATTER2, rows(grids[l + 1]), 8, C[l + 1], C[l], dev(below), C[l + 1], uw.b16, cat,
                   2 * C[l], bias=ub.p, y_offset=C[l])
        nodes = _nodes(grids[l], 2000, seed=500 + l)
        hc = _h(cat)
        _check_bf16(_at(hc, nodes)[:, C[l]:], onn.up2_at(below, W(uw), B(ub), nodes), "up to level %d" % l)
        assert not np.any(_at(hc, nodes)[:, :C[l]]), "up to level %d wrote the skip half" % l
        conv(l, 2 * C[l], C[l], w1, b1, 2 * C[l], C[l], "dec %d conv 1" % l)
        conv(l, C[l], C[l], w2, b2, C[l], C[l], "dec %d conv 2" % l)
    # the FP32 head (1x1x1) and the force-direction mix of its three 4-channel groups
    hw, hb = net.head
    oc = net.out_ch
    below = rnd(grids[0] + (C[0],))
    out = torch.empty(grids[0] + (oc,), dtype=torch.float32, device="cuda")
    nn.forward(nn.IDENT, nn.IDENT, rows(grids[0]), 1, C[0], oc, dev(below), C[0], hw.b16, out, oc, bias=hb.p,
               y_fp32=True)
    nodes = _nodes(grids[0], 2000, seed=600)
    want = onn.dense(_at(below, nodes), W(hw).reshape(hw.p.shape[0], -1)[:oc], B(hb)[:oc])
    err = np.max(np.abs(_at(_h(out), nodes) - want)) / np.max(np.abs(want))
    _log("head max error / max output", err)
    assert err <= 1e-5
    d = np.array([0.36, -0.48, 0.8])
    mixed = torch.empty(grids[0] + (4,), dtype=torch.float32, device="cuda")
    nn.mix(out, d, mixed)
    gm = _at(_h(mixed), nodes)
    mix = sum(d[j] * _at(_h(out), nodes)[:, 4 * j:4 * j + 4] for j in range(3))
    assert np.max(np.abs(gm - mix)) <= 1e-6 * np.max(np.abs(mix))


def test_shift_by_eight_commutes(torch, run):
    net, x, sm, mixed = run
    for shift in [(8, 0, 0), (0, 8, 0), (0, 0, 8), (24, 40, 64)]:
        xs = torch.roll(x, shifts=shift, dims=(0, 1, 2)).contiguous()
        ys = net.forward_mixed(xs, sm.dir)
        want = torch.roll(mixed, shifts=shift, dims=(0, 1, 2))
        torch.cuda.synchronize()
        diff = float((ys - want).abs().max())
        _log("shift", shift, "max |difference|", diff)
        assert torch.equal(ys, want), shift
