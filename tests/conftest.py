import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libipm.so")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    oracle.load()
    return oracle


def parity(got, ref):
    """Normwise relative L1 error per conserved variable, over cells and modes
    (arrays [cells][m][N])."""
    import numpy as np
    got = np.asarray(got)
    ref = np.asarray(ref)
    num = np.abs(got - ref).sum(axis=(0, 2))
    den = np.abs(ref).sum(axis=(0, 2))
    return num / np.maximum(den, 1e-300)


@pytest.fixture(scope="session")
def gpu_ctx():
    """A libipm context on cuda:0 ordered on torch's current stream."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_09238_amd import binding
    torch.cuda.init()
    ctx = binding.Context(device=0, stream=torch.cuda.current_stream().cuda_stream)
    yield ctx
    ctx.close()
