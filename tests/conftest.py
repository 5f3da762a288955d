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


# Per-mode bounds use the variable's mean scale as a floor: the dual solves
# stop on an absolute tolerance (the sum over variables of the Euclidean norm
# of the gradient below tau), so each moment of a cell carries an absolute
# error of order tau whatever its own size, and a mode whose content is
# below a thousandth of the variable's mean has no relative precision of
# its own to test.
MODE_FLOOR = 1e-3


def parity_stats(got, ref):
    """Three error measures of moments [cells][m][N] against a reference:
    - norm: normwise relative L1 per variable over all cells and modes;
    - elem: per (variable, mode) the largest error over cells divided by the
      largest |mode 0| of that variable (element by element);
    - mode: per (variable, mode) the L1 error over cells divided by the L1
      of that mode, floored at MODE_FLOOR times the L1 of mode 0."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    d = np.abs(got - ref)
    scale0 = np.maximum(np.abs(ref[:, :, 0]).max(axis=0), 1e-300)  # [m]
    elem = d.max(axis=0) / scale0[:, None]                          # [m][N]
    l1 = np.abs(ref).sum(axis=0)                                    # [m][N]
    mode = d.sum(axis=0) / np.maximum(np.maximum(l1, MODE_FLOOR * l1[:, :1]), 1e-300)
    return {"norm": parity(got, ref), "elem": elem, "mode": mode}


# Inexact Newton (stored inverse Hessians): both sides stop on the same tau
# but at different points of its ball, so a mode whose content sits near the
# floor can differ by a few 1e-9 of the variable's mean (measured up to
# 1.3e-8): the per-mode bound of those forms is 1e-7, their norm and element
# bounds stay at 1e-8.
INEXACT_MODE_TOL = 1e-7


def check_parity(got, ref, tol, what="", mode_tol=None):
    """Assert the norm and element measures of parity_stats are <= tol and the
    per-mode measure <= mode_tol (default tol); print them."""
    import numpy as np
    st = parity_stats(got, ref)
    print("  parity %s: norm %.2e  elem %.2e  mode %.2e" % (
        what, st["norm"].max(), st["elem"].max(), st["mode"].max()), flush=True)
    for k in ("norm", "elem", "mode"):
        t = tol if (k != "mode" or mode_tol is None) else mode_tol
        bad = np.argwhere(~(st[k] <= t))
        assert bad.size == 0, (what, k, t, bad[:8].tolist(), st[k].max())
    return st


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
