"""GPU: batched stepping of several problems (one launch per kernel shape per
step, replayed from device graphs) against stepping each problem alone, and
the autotuner.  Batching changes no arithmetic, so the comparison is bitwise;
one mixed batch is also compared with the oracle."""
import sys

import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W

from .conftest import check_parity, parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed_specs():
    """1D and 2D, IPM and one-shot, uniform and per-cell degrees, small and
    workgroup-per-cell Newton kernels."""
    rng = np.random.default_rng(7)
    a = W.burgers_shock(nx=120, degree=4, qpd=10, t_end=0.0)
    b = W.sod(nx=300, degree=9, qpd=20, t_end=0.0)
    c = W.bump2d(n=12, degree=2, qpd=3, p=3, t_end=0.0, v1_spread=0.2)
    c["ny"] = 9
    cd_c = rng.integers(0, 3, size=c["nx"] * c["ny"]).astype(np.int8)
    d = W.bump2d(n=10, degree=5, qpd=8, t_end=0.0)
    d["ny"] = 6
    e = W.steady_inflow(nx=60, one_shot=1)
    e["steady_eps"] = 0.0  # run a fixed number of pseudo-time steps
    return [(a, None, False), (b, None, False), (c, cd_c, False), (d, None, False), (e, None, True)]


def _make(ctx, spec, cd, dirichlet):
    from paper_1912_09238_amd import binding
    nodes, _ = binding.quadrature(spec["p"], spec["quad_per_dim"])
    kw = {}
    if cd is not None:
        kw["cell_degree"] = cd
    if dirichlet:
        kw["dirichlet"] = W.dirichlet_nodal(spec, nodes)
    return ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes), **kw)


def test_batched_steps_equal_single_problem_steps(gpu_ctx):
    specs = _mixed_specs()
    _say("gpu case: batch of %d mixed problems vs one by one" % len(specs))
    alone = []
    for spec, cd, dl in specs:
        pid = _make(gpu_ctx, spec, cd, dl)
        gpu_ctx.step(pid, 3, wait=True)   # odd start: the batch below mixes step parities
        gpu_ctx.step(pid, 14, wait=True)
        alone.append(gpu_ctx.moments(pid))
        gpu_ctx.release(pid)
    ids = [_make(gpu_ctx, spec, cd, dl) for spec, cd, dl in specs]
    gpu_ctx.step(ids[1], 3, wait=True)    # problem b runs 3 steps ahead
    gpu_ctx.step([i for k, i in enumerate(ids) if k != 1], 3, wait=True)
    gpu_ctx.step(ids, 5, wait=True)       # builds the batch plan
    gpu_ctx.step(ids, 6, wait=True)       # reuses it
    gpu_ctx.step(ids[0], 1, wait=True)    # invalidates it for the others
    gpu_ctx.step(ids[1:], 1, wait=True)
    gpu_ctx.step(ids, 2, wait=True)
    infos = gpu_ctx.step(ids, 0, wait=True)
    for k, pid in enumerate(ids):
        assert infos[k]["status"] == 0, infos[k]
        assert infos[k]["steps"] == 17, infos[k]
        got = gpu_ctx.moments(pid)
        assert np.array_equal(got, alone[k]), (k, np.max(np.abs(got - alone[k])))
        gpu_ctx.release(pid)


def test_batch_matches_oracle(gpu_ctx, orc):
    specs = _mixed_specs()[:4]
    _say("gpu case: batch of 4 vs oracle")
    ids = [_make(gpu_ctx, spec, cd, dl) for spec, cd, dl in specs]
    gpu_ctx.step(ids, 10, wait=True)
    for (spec, cd, _), pid in zip(specs, ids):
        kw = {} if cd is None else {"cell_degree": cd}
        o = orc.Oracle(spec, ic_fn=lambda nd, s=spec: W.ic_nodal(s, nd), **kw)
        o.step(10)
        err = parity(gpu_ctx.moments(pid), o.moments())
        _say("  %s parity %s" % (spec["name"], np.array2string(err, precision=2)))
        assert np.all(err <= 1e-10), err
        check_parity(gpu_ctx.moments(pid), o.moments(), 1e-10)
        gpu_ctx.release(pid)


def test_autotune_changes_no_result(gpu_ctx):
    from paper_1912_09238_amd import binding
    specs = _mixed_specs()
    _say("gpu case: autotune on a mixed batch")
    ids = [_make(gpu_ctx, spec, cd, dl) for spec, cd, dl in specs]
    tuned = gpu_ctx.autotune(ids, steps_per_candidate=1)  # 2 real steps per candidate
    assert tuned >= 1
    done = gpu_ctx.step(ids, 0, wait=True)[0]["steps"]
    gpu_ctx.step(ids, 5, wait=True)
    got = [gpu_ctx.moments(i) for i in ids]
    for i in ids:
        gpu_ctx.release(i)
    # the same steps in a fresh context with the default launch shapes
    ref_ctx = binding.Context(device=0)
    try:
        rids = [_make(ref_ctx, spec, cd, dl) for spec, cd, dl in specs]
        ref_ctx.step(rids, done + 5, wait=True)
        for k, pid in enumerate(rids):
            assert np.array_equal(ref_ctx.moments(pid), got[k]), k
    finally:
        ref_ctx.close()
