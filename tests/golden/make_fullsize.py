"""Write the full-size oracle references of the GPU parity tests (test
infrastructure: calls only the CPU oracle and the seeded input recipe).

    python tests/golden/make_fullsize.py [sod|bump|batch ...]

Each file holds the oracle's moments at a deterministic sample of cells, the
sample's cell indices and the run's step record:

- fullsize_sod8192_t014.npz: the 1D Euler Sod tube at its full size (8192
  cells, degree 9, 20 Gauss-Legendre nodes, Euler entropy, Rusanov, CFL 0.5)
  over its whole trajectory to t_end = 0.14 (Alg. 1 time loop), every 8th
  cell;
- fullsize_bump512_2steps.npz: the 2D Euler bump on the periodic 512 x 512
  grid (two uncertainties, total degree 5, 8 x 8 nodes) after 2 time steps:
  every cell of the 32 x 32 block around the bump centre and 512 seeded
  cells elsewhere;
- fullsize_batch64_2steps.npz: every problem of the 64-problem batch (three
  uncertainties, per-cell degrees 1-4 from the seeded recipe, 5^3 nodes)
  after 2 time steps: per problem the 8 cells nearest the bump centre and 16
  seeded cells, moments [cell][4][35] with modes above a cell's degree zero.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1912_09238_amd import workloads as W  # noqa: E402


def _oracle(spec, **kw):
    return oracle.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd), **kw)


def sample_bump512(n=512):
    """Cells of the 32 x 32 block around the centre, then 512 seeded others."""
    iy, ix = np.meshgrid(np.arange(n // 2 - 16, n // 2 + 16), np.arange(n // 2 - 16, n // 2 + 16),
                         indexing="ij")
    core = (iy * n + ix).reshape(-1)
    rng = np.random.default_rng(512)
    rest = np.setdiff1d(rng.choice(n * n, size=700, replace=False), core)[:512]
    return np.sort(np.concatenate([core, rest]))


def sample_batch(spec):
    """8 cells nearest the bump centre and 16 seeded cells of one problem."""
    xc, yc = W.cell_centres(spec)
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    d2 = ((X - spec["ic"]["cx"]) ** 2 + (Y - spec["ic"]["cy"]) ** 2).reshape(-1)
    near = np.argsort(d2, kind="stable")[:8]
    rng = np.random.default_rng(spec["seed"])
    rest = np.setdiff1d(rng.choice(d2.size, size=40, replace=False), near)[:16]
    return np.sort(np.concatenate([near, rest]))


def make_sod():
    spec = W.sod()
    o = _oracle(spec)
    info = o.run()
    assert info["status"] == 0 and info["done"] == 1, info
    cells = np.arange(0, spec["nx"], 8)
    np.savez_compressed(os.path.join(HERE, "fullsize_sod8192_t014.npz"), cells=cells,
                        moments=o.moments()[cells], steps=info["steps"], t=info["t"],
                        newton_iters=info["newton_iters"])


def make_bump():
    spec = W.bump2d()
    o = _oracle(spec)
    info = o.step(2)
    assert info["status"] == 0 and info["steps"] == 2, info
    cells = sample_bump512()
    np.savez_compressed(os.path.join(HERE, "fullsize_bump512_2steps.npz"), cells=cells,
                        moments=o.moments()[cells], steps=info["steps"], t=info["t"])


def make_batch():
    out = {}
    for k, spec in enumerate(W.batch_problems(count=64)):
        o = _oracle(spec, cell_degree=W.cell_degrees(spec))
        info = o.step(2)
        assert info["status"] == 0 and info["steps"] == 2, (k, info)
        cells = sample_batch(spec)
        out["cells%02d" % k] = cells
        out["moments%02d" % k] = o.moments()[cells]
        out["t%02d" % k] = info["t"]
        print("batch problem %d: %d cells, t = %.6g" % (k, o.cells, info["t"]), flush=True)
        del o
    np.savez_compressed(os.path.join(HERE, "fullsize_batch64_2steps.npz"), **out)


if __name__ == "__main__":
    oracle.build()
    todo = sys.argv[1:] or ["sod", "bump", "batch"]
    for name in todo:
        t0 = time.perf_counter()
        {"sod": make_sod, "bump": make_bump, "batch": make_batch}[name]()
        print("%s: %.1f s" % (name, time.perf_counter() - t0), flush=True)
