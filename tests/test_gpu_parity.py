"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  FP64 form: normwise relative L1 error per conserved
variable (over cells and modes) <= 1e-10."""
import math
import sys

import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W

from .conftest import check_parity, parity

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run_both(ctx, orc, spec, steps, cell_degree=None, dirichlet=False):
    from paper_1912_09238_amd import binding
    nodes, _ = binding.quadrature(spec["p"], spec["quad_per_dim"])
    kw = {}
    okw = {}
    if dirichlet:
        kw["dirichlet"] = W.dirichlet_nodal(spec, nodes)
        okw["dirichlet_fn"] = lambda nd: W.dirichlet_nodal(spec, nd)
    if cell_degree is not None:
        kw["cell_degree"] = cell_degree
        okw["cell_degree"] = cell_degree
    _say("gpu case: %s nx=%d ny=%d M=%d qpd=%d steps=%d" % (
        spec["name"], spec["nx"], spec.get("ny", 1), spec["degree"], spec["quad_per_dim"], steps))
    pid = ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes), **kw)
    info = ctx.step(pid, steps, wait=True)[0]
    got = ctx.moments(pid)
    gl = ctx.dual(pid)
    ctx.release(pid)
    o = orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd), **okw)
    oinfo = o.step(steps)
    return info, got, gl, oinfo, o


def _check(info, got, oinfo, o, tol=TOL):
    assert info["status"] == 0, info
    assert oinfo["status"] == 0, oinfo
    assert info["steps"] == oinfo["steps"]
    assert abs(info["t"] - oinfo["t"]) <= 1e-14 * max(1.0, abs(oinfo["t"]))
    err = parity(got, o.moments())
    _say("  parity per variable: %s  newton gpu=%d oracle=%d" % (
        np.array2string(err, precision=2), info["newton_iters"], oinfo["newton_iters"]))
    assert np.all(err <= tol), err
    check_parity(got, o.moments(), tol)


def test_burgers_shock_full_run(gpu_ctx, orc):
    spec = W.burgers_shock()
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 100)
    assert info["done"] == 1 and oinfo["steps"] == 9
    _check(info, got, oinfo, o)
    assert abs(info["newton_iters"] - oinfo["newton_iters"]) <= 0.02 * oinfo["newton_iters"]


@pytest.mark.parametrize("nx,steps", [(250, 30), (37, 12), (1, 3)])
def test_sod_small_ragged(gpu_ctx, orc, nx, steps):
    spec = W.sod(nx=nx, degree=9, qpd=20)
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, steps)
    _check(info, got, oinfo, o)


def test_sod_full_size_first_steps(gpu_ctx, orc):
    spec = W.sod()  # 8192 cells, degree 9, 20 nodes: the throughput workload
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 6)
    _check(info, got, oinfo, o)


@pytest.mark.parametrize("degree,qpd", [(0, 1), (2, 3), (4, 8), (6, 7)])
def test_sod_degrees(gpu_ctx, orc, degree, qpd):
    spec = W.sod(nx=64, degree=degree, qpd=qpd, t_end=0.05)
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 400)
    assert info["done"] == 1
    _check(info, got, oinfo, o)


@pytest.mark.parametrize("entropy", ["quadratic", "log_barrier"])
def test_burgers_entropies(gpu_ctx, orc, entropy):
    spec = W.burgers_shock(nx=90, degree=6, qpd=12, t_end=0.02)
    spec["entropy"] = entropy
    if entropy == "quadratic":
        spec["ic"] = dict(kind="shock1d", left=2.0, right=1.0, shift=0.0, spread=1.0)
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 1000)
    _check(info, got, oinfo, o)


def test_euler2d_periodic(gpu_ctx, orc):
    spec = W.bump2d(n=20, degree=2, qpd=4, t_end=0.05)
    spec["ny"] = 14
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 100)
    _check(info, got, oinfo, o)


def test_euler2d_three_uncertainties_uneven_degrees(gpu_ctx, orc):
    spec = W.bump2d(n=12, degree=2, qpd=3, p=3, t_end=0.03, v1_spread=0.2)
    spec["ic"]["cx"], spec["ic"]["cy"] = 0.45, 0.6
    rng = np.random.default_rng(1912)
    cd = rng.integers(0, 3, size=spec["nx"] * spec["ny"]).astype(np.int8)
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 100, cell_degree=cd)
    _check(info, got, oinfo, o)


@pytest.mark.parametrize("one_shot", [0, 1])
def test_steady_dirichlet_one_shot(gpu_ctx, orc, one_shot):
    spec = W.steady_inflow(one_shot=one_shot)
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 5000, dirichlet=True)
    assert info["done"] == 1 and info["residual"] <= 1e-10
    _check(info, got, oinfo, o)
    want = np.zeros(5)
    want[0], want[1] = 1.0, 0.2 / math.sqrt(3.0)
    assert np.max(np.abs(got[:, 0, :] - want)) < 5e-8


def test_deterministic_bitwise(gpu_ctx):
    from paper_1912_09238_amd import binding
    spec = W.sod(nx=512, degree=9, qpd=20)
    nodes, _ = binding.quadrature(1, 20)
    outs = []
    for _ in range(2):
        _say("gpu case: determinism sod nx=512")
        pid = gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))
        gpu_ctx.step(pid, 25, wait=True)
        outs.append(gpu_ctx.moments(pid))
        gpu_ctx.release(pid)
    assert np.array_equal(outs[0], outs[1])


def test_checkpoint_resume_bitwise(gpu_ctx):
    from paper_1912_09238_amd import binding
    spec = W.sod(nx=300, degree=5, qpd=8, t_end=0.0)
    nodes, _ = binding.quadrature(1, 8)
    ic = W.ic_nodal(spec, nodes)
    _say("gpu case: checkpoint/resume sod nx=300")
    a = gpu_ctx.set_problem(spec, ic_nodal=ic)
    gpu_ctx.step(a, 20, wait=True)
    full = gpu_ctx.moments(a)
    gpu_ctx.release(a)
    b = gpu_ctx.set_problem(spec, ic_nodal=ic)
    gpu_ctx.step(b, 10, wait=True)
    mom, lam = gpu_ctx.moments(b), gpu_ctx.dual(b)
    gpu_ctx.release(b)
    c = gpu_ctx.set_problem(spec, ic_moments=mom, ic_dual=lam)
    gpu_ctx.step(c, 10, wait=True)
    resumed = gpu_ctx.moments(c)
    gpu_ctx.release(c)
    assert np.array_equal(full, resumed)


def test_errors_are_reported(gpu_ctx):
    from paper_1912_09238_amd import binding
    spec = W.burgers_shock(nx=16)
    nodes, _ = binding.quadrature(1, 10)
    bad = dict(spec, cfl=-1.0)
    with pytest.raises(binding.IpmError) as e:
        gpu_ctx.set_problem(bad, ic_nodal=W.ic_nodal(spec, nodes))
    assert e.value.code == -1
    # initial state outside the log-barrier's domain
    out_of_range = dict(spec, u_plus=11.0)
    with pytest.raises(binding.IpmError) as e:
        gpu_ctx.set_problem(out_of_range, ic_nodal=W.ic_nodal(spec, nodes))
    assert e.value.code == -4
    with pytest.raises(binding.IpmError):
        gpu_ctx.step(12345, 1)


def test_newton_failure_is_sticky(gpu_ctx, orc):
    from paper_1912_09238_amd import binding
    spec = W.sod(nx=64, degree=5, qpd=8)
    spec["max_newton"] = 1
    spec["tau"] = 1e-14
    nodes, _ = binding.quadrature(1, 8)
    _say("gpu case: newton failure")
    with pytest.raises(binding.IpmError):
        # the initial dual cannot converge in one iteration to 1e-14
        gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))


# ---- cells of more than 64 unknowns: workgroup-per-cell Newton kernel

def test_euler2d_degree5_large_cells(gpu_ctx, orc):
    # N = 21, n = 84 unknowns per cell, 8 x 8 nodes: the 2D throughput workload's cell size
    spec = W.bump2d(n=16, degree=5, qpd=8, t_end=0.0)
    spec["ny"] = 12
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 8)
    _check(info, got, oinfo, o)


def test_euler2d_three_uncertainties_degree4_uneven(gpu_ctx, orc):
    # N = 35, n = 140 at degree 4, 5^3 nodes; per-cell degrees 0..4 (n = 4 .. 140)
    spec = W.bump2d(n=10, degree=4, qpd=5, p=3, t_end=0.0, v1_spread=0.2)
    spec["ny"] = 7
    rng = np.random.default_rng(1912)
    cd = rng.integers(0, 5, size=spec["nx"] * spec["ny"]).astype(np.int8)
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 5, cell_degree=cd)
    _check(info, got, oinfo, o)


def test_burgers_two_uncertainties_degree11(gpu_ctx, orc):
    # m = 1, N = 78 unknowns, 12 x 12 nodes, log-barrier entropy
    spec = W.burgers_shock(nx=40, degree=11, qpd=12, t_end=0.03)
    spec["p"] = 2
    info, got, _, oinfo, o = _run_both(gpu_ctx, orc, spec, 200)
    assert info["done"] == 1
    _check(info, got, oinfo, o)


def test_large_cells_with_three_variables_are_rejected(gpu_ctx):
    from paper_1912_09238_amd import binding
    spec = W.sod(nx=8, degree=4, qpd=5)
    spec["p"] = 3  # N = 35, n = 105 > 64 with m = 3
    nodes, _ = binding.quadrature(3, 5)
    with pytest.raises(binding.IpmError) as e:
        gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))
    assert e.value.code == -1
