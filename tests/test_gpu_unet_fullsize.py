"""The warm-start network at its full size, in the configuration bench.py
times: the 4-level, 24-base U-Net with the force-linear head on a 128^3
porous sample's geometry encoding.

* Every layer of one forward pass against the FP64 layer oracle, on sampled
  voxels: the layer's own BF16 input as the GPU holds it after the pass, the
  BF16 weights and FP32 biases, and the oracle's layer evaluated at the
  sampled voxels (2,000 per layer, all voxels where a grid has fewer).  BF16
  outputs are within their rounding, 2^-8 of the value, plus 1e-4 of the
  layer's largest output for FP32 accumulation order; pooling is exact; the
  FP32 head output within 1e-5 of its largest value.
* Circular padding, stride-2 pooling and stride-2 up-sampling make the
  network commute with shifts by multiples of 8 voxels (2^(levels-1)): the
  output of the shifted input is the shifted output, bit for bit, which
  checks every kernel's indexing over the whole grid.
"""
import sys

import numpy as np
import pytest

from oracle import nn as onn
from paper_1703_08015_amd import inputs, warmstart

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


def test_every_layer_on_sampled_voxels(torch, run):
    net, x, sm, mixed = run
    _, A, grids = net._cache
    L, C = net.L, net.C
    W = lambda p: _h(p.b16)  # noqa: E731
    B = lambda p: _h(p.p)  # noqa: E731
    src = _h(x)
    for l in range(L):
        nodes = _nodes(grids[l], 2000, seed=100 + l)
        (w1, b1), (w2, b2) = net.enc[l]
        if l > 0:
            prev = _h(A["cat", l - 1])[..., :C[l - 1]]
            assert np.array_equal(_at(_h(A["pool", l]), nodes), onn.maxpool2_at(prev, nodes)), "pool %d" % l
            src = _h(A["pool", l])
        e1 = _h(A["e1", l])
        _check_bf16(_at(e1, nodes), onn.relu(onn.conv3_at(src, W(w1), B(b1), nodes)), "enc %d conv 1" % l)
        cat = _h(A["cat", l])
        _check_bf16(_at(cat, nodes)[:, :C[l]], onn.relu(onn.conv3_at(e1, W(w2), B(b2), nodes)), "enc %d conv 2" % l)
    below = _h(A["cat", L - 1])
    for k, l in enumerate(range(L - 2, -1, -1)):
        nodes = _nodes(grids[l], 2000, seed=200 + l)
        uw, ub = net.up[k]
        (w1, b1), (w2, b2) = net.dec[k]
        cat = _h(A["cat", l])
        _check_bf16(_at(cat, nodes)[:, C[l]:], onn.up2_at(below, W(uw), B(ub), nodes), "up to level %d" % l)
        d1 = _h(A["d1", l])
        _check_bf16(_at(d1, nodes), onn.relu(onn.conv3_at(cat, W(w1), B(b1), nodes)), "dec %d conv 1" % l)
        d2 = _h(A["d2", l])
        _check_bf16(_at(d2, nodes), onn.relu(onn.conv3_at(d1, W(w2), B(b2), nodes)), "dec %d conv 2" % l)
        below = d2
    # the FP32 head (1x1x1) and the force-direction mix of its three 4-channel groups
    nodes = _nodes(grids[0], 2000, seed=300)
    hw, hb = net.head
    oc = net.out_ch
    want = onn.dense(_at(below, nodes), W(hw).reshape(hw.p.shape[0], -1)[:oc], B(hb)[:oc])
    got = _at(_h(A["out"]), nodes)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    _log("head max error / max output", err)
    assert err <= 1e-5
    mix = sum(sm.dir[j] * want[:, 4 * j:4 * j + 4] for j in range(3))
    gm = _at(_h(mixed), nodes)
    assert np.max(np.abs(gm - mix)) <= 1e-5 * np.max(np.abs(mix))


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
