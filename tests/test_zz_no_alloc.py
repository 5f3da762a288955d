"""ipm_step_static (the batched step for callers that cannot allocate) against
ipm_step on the same problems: identical moments, duals and step records, on
two calls in a row (the second with fewer, smaller problems), and the size
limit of its fixed scratch reported as an argument error."""
import sys

import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_09238_amd import binding
    torch.cuda.init()
    c = binding.Context(device=0, stream=torch.cuda.current_stream().cuda_stream)
    yield c
    c.close()


def _specs(kind):
    if kind == "mix":
        out = []
        for k, n in enumerate((20, 28, 12)):
            s = W.bump2d(n=n, degree=4, qpd=5, p=3, center=(0.4 + 0.05 * k, 0.55), v1_spread=0.2)
            s["seed"] = 100 + k
            out.append((s, W.cell_degrees(s)))
        out.append((W.sod(nx=300, degree=9, qpd=20), None))
        return out
    s = W.bump2d(n=10, degree=4, qpd=5, p=3, center=(0.5, 0.45), v1_spread=0.2)
    s["seed"] = 7
    return [(s, W.cell_degrees(s))]


def _setup(ctx, specs):
    from paper_1912_09238_amd import binding
    ids = []
    for s, cd in specs:
        nodes, _ = binding.quadrature(s["p"], s["quad_per_dim"])
        kw = {"cell_degree": cd} if cd is not None else {}
        ids.append(ctx.set_problem(s, ic_nodal=W.ic_nodal(s, nodes), **kw))
    return ids


@pytest.mark.parametrize("kind,steps", [("mix", 7), ("small", 5)])
def test_static_step_equals_step(ctx, kind, steps):
    specs = _specs(kind)
    _say("gpu case: ipm_step_static %s, %d problems, %d steps" % (kind, len(specs), steps))
    ref_ids = _setup(ctx, specs)
    ref_info = ctx.step(ref_ids, steps, wait=True)
    ref = [(ctx.moments(i), ctx.dual(i)) for i in ref_ids]
    for i in ref_ids:
        ctx.release(i)
    ids = _setup(ctx, specs)
    # two calls: the first uploads the launch parameters, the second reuses them
    ctx.step_static(ids, steps - 2, wait=False)
    info = ctx.step_static(ids, 2, wait=True)
    got = [(ctx.moments(i), ctx.dual(i)) for i in ids]
    for i in ids:
        ctx.release(i)
    for a, b, ia, ib in zip(got, ref, info, ref_info):
        assert ia["status"] == 0 and ib["status"] == 0
        assert ia["steps"] == ib["steps"] == steps
        assert ia["t"] == ib["t"] and ia["newton_iters"] == ib["newton_iters"]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_static_step_rejects_plans_beyond_its_scratch(ctx):
    from paper_1912_09238_amd import binding
    s = W.burgers_shock(nx=4, degree=2, qpd=4, t_end=0.0)
    nodes, _ = binding.quadrature(1, 4)
    ic = W.ic_nodal(s, nodes)
    _say("gpu case: ipm_step_static size limit")
    ids = [ctx.set_problem(s, ic_nodal=ic) for _ in range(480)]
    try:
        with pytest.raises(binding.IpmError) as e:
            ctx.step_static(ids, 1, wait=True)
        assert e.value.code == -1 and "static scratch" in str(e.value)
        # a list that fits still steps
        info = ctx.step_static(ids[:8], 1, wait=True)
        assert all(i["status"] == 0 and i["steps"] == 1 for i in info)
    finally:
        for i in ids:
            ctx.release(i)
