"""lbm_components_device_noalloc, the entry point for callers that cannot
allocate: through the C ABI it must return exactly the labels and count of
lbm_components_device (which takes its scratch from the caller) on two calls
in a row, the second on a smaller grid, and refuse a grid whose scratch would
exceed the fixed array."""
import ctypes

import numpy as np
import pytest

from paper_1703_08015_amd import inputs, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _case(torch, mask, q, periodic):
    solid = torch.from_numpy(np.ascontiguousarray(mask.astype(np.uint8))).cuda()
    want, wcount = lbm.components_device(solid, q, -1, periodic)
    labels = torch.full(tuple(solid.shape) if solid.dim() == 3 else (1,) + tuple(solid.shape), 7,
                        dtype=torch.int32, device="cuda")
    count = lbm.components_device_noalloc(solid, labels, q, -1, periodic)
    torch.cuda.synchronize()
    return want.cpu().numpy(), wcount, labels.cpu().numpy(), count


def test_noalloc_equals_allocating_entry_point_twice(torch):
    big = inputs.spheres_3d(96, 0.5, rmin=3, rmax=8, seed=5)[0]        # 884,736 nodes
    small = inputs.spheres_3d((20, 18, 13), 0.45, rmin=2, rmax=4, seed=6, periodic=(1, 0, 1))[0]
    for name, mask, per in (("96^3 packing", big, (1, 1, 1)), ("20x18x13 walled in y", small, (1, 0, 1))):
        print("noalloc components:", name, mask.shape, flush=True)
        want, wcount, got, count = _case(torch, mask, 19, per)
        assert count == wcount, name
        assert np.array_equal(got.reshape(want.shape), want), name


def test_noalloc_d2q9_and_limit(torch):
    chan = inputs.channel_2d(64, 64, seed=0)[0]
    print("noalloc components: D2Q9 channel", chan.shape, flush=True)
    want, wcount, got, count = _case(torch, chan, 9, (1, 0, 0))
    assert count == wcount and np.array_equal(got.reshape(want.shape), want)
    # a grid past the fixed scratch is refused before any launch
    cap = lbm.components_noalloc_max_scratch()
    assert cap == 1 << 22
    shape = np.array([256, 256, 64], np.int32)  # 4,194,304 nodes
    assert lbm.lib().lbm_components_device_scratch(lbm._np_ptr(shape)) > cap
    solid = torch.zeros((64, 256, 256), dtype=torch.uint8, device="cuda")
    labels = torch.empty_like(solid, dtype=torch.int32)
    with pytest.raises(lbm.LbmError) as e:
        lbm.components_device_noalloc(solid, labels, 19, -1, (1, 1, 1))
    assert e.value.code == lbm.LBM_ERR_ARG
