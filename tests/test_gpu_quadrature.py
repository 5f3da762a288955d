"""GPU parity on Clenshaw-Curtis tensor and sparse grids (the rules of the
paper's three-uncertainty study, Sec. 7) through the C ABI."""
import sys

import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W

from .conftest import check_parity, parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(ctx, orc, spec, steps):
    from paper_1912_09238_amd import binding
    nodes, _ = binding.quadrature(spec["p"], spec["quad_per_dim"], spec["quad_rule"])
    _say("gpu case: %s rule=%s param=%d degree=%d Q=%d cells=%d steps=%d" % (
        spec["name"], spec["quad_rule"], spec["quad_per_dim"], spec["degree"], len(nodes),
        spec["nx"] * spec.get("ny", 1), steps))
    pid = ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))
    info = ctx.step(pid, steps, wait=True)[0]
    got = ctx.moments(pid)
    ctx.release(pid)
    o = orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd))
    oinfo = o.step(steps)
    assert info["status"] == 0 and oinfo["status"] == 0
    assert info["steps"] == oinfo["steps"]
    err = parity(got, o.moments())
    _say("  parity %s" % np.array2string(err, precision=2))
    assert np.all(err <= 1e-10), err
    check_parity(got, o.moments(), 1e-10)


def test_sod_tensor_clenshaw_curtis(gpu_ctx, orc):
    spec = W.sod(nx=250, degree=9, qpd=17)
    spec["quad_rule"] = "cc"
    _run(gpu_ctx, orc, spec, 20)


@pytest.mark.parametrize("level,degree", [(2, 1), (5, 2)])
def test_three_uncertainties_on_sparse_grids(gpu_ctx, orc, level, degree):
    """The paper's sparse-grid runs: order 1 on 25 nodes, order 2 on 441."""
    spec = W.bump2d(n=12, degree=degree, qpd=level, p=3, v1_spread=0.2)
    spec.update(quad_rule="cc_sparse", ny=10)
    _run(gpu_ctx, orc, spec, 5)


def test_sparse_grid_order3_loses_definiteness(gpu_ctx, orc):
    """Order 3 on the 25-node sparse grid: negative weights make the dual
    Hessian indefinite at set-up, on both sides."""
    from paper_1912_09238_amd import binding
    spec = W.bump2d(n=8, degree=3, qpd=2, p=3, v1_spread=0.2)
    spec["quad_rule"] = "cc_sparse"
    nodes, _ = binding.quadrature(3, 2, "cc_sparse")
    _say("gpu case: sparse level 2, degree 3 (indefinite Hessian)")
    with pytest.raises(binding.IpmError) as e:
        gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))
    assert e.value.code == -5
    assert orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd)).info["status"] & 8


def test_quadrature_rule_arguments(gpu_ctx):
    from paper_1912_09238_amd import binding
    spec = W.sod(nx=16, degree=2, qpd=12)
    spec["quad_rule"] = "cc_sparse"  # level 12 is out of range
    with pytest.raises(binding.IpmError) as e:
        gpu_ctx.set_problem(spec, ic_moments=np.zeros((16, 3, 3)))
    assert e.value.code == -1
