import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


_GPU = None


def _gpu_available():
    global _GPU
    if _GPU is None:
        try:
            import torch
            _GPU = bool(torch.cuda.is_available())
        except Exception:
            _GPU = False
    return _GPU


def pytest_collection_modifyitems(config, items):
    for item in items:
        if "gpu" in item.keywords and not _gpu_available():
            item.add_marker(pytest.mark.skip(reason="no GPU visible"))
