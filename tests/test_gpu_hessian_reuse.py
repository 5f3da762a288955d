"""GPU: inexact-Hessian Newton (stored inverse Hessians reused while they
contract the dual residual) against the exact-Newton oracle.  The dual still
stops at tau, so the moments agree within the dual tolerance's reach rather
than bit for bit: normwise relative L1 per variable <= 1e-8 over these runs,
and E / Var within the precision form's 1e-4."""
import sys

import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W

from .conftest import INEXACT_MODE_TOL, check_parity, parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(ctx, orc, spec, steps):
    from paper_1912_09238_amd import binding
    nodes, _ = binding.quadrature(spec["p"], spec["quad_per_dim"])
    _say("gpu case: hessian reuse %s n=%dx%d p=%d degree=%d precision=%s steps=%d" % (
        spec["name"], spec["nx"], spec["ny"], spec["p"], spec["degree"],
        spec.get("precision", "fp64"), steps))
    pid = ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))
    info = ctx.step(pid, steps, wait=True)[0]
    got = ctx.moments(pid)
    ctx.release(pid)
    ref = dict(spec)
    ref.pop("hessian_reuse")
    ref.pop("precision", None)
    o = orc.Oracle(ref, ic_fn=lambda nd: W.ic_nodal(ref, nd))
    oinfo = o.step(steps)
    assert info["status"] == 0 and oinfo["status"] == 0
    assert info["steps"] == oinfo["steps"]
    want = o.moments()
    err = parity(got, want)
    rel = lambda a, b: float(np.abs(a - b).sum() / np.abs(b).sum())
    e = rel(got[:, :, 0], want[:, :, 0])
    v = rel(np.sum(got[:, :, 1:] ** 2, axis=2), np.sum(want[:, :, 1:] ** 2, axis=2))
    _say("  parity %s  E %.2e Var %.2e  newton gpu=%d oracle=%d" % (
        np.array2string(err, precision=2), e, v, info["newton_iters"], oinfo["newton_iters"]))
    assert np.all(err <= 1e-8), err
    check_parity(got, want, 1e-8, mode_tol=INEXACT_MODE_TOL)
    assert e <= 1e-4 and v <= 1e-4


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_reuse_2d_bump_84_unknowns(gpu_ctx, orc, precision):
    spec = W.bump2d(n=24, degree=5, qpd=8, p=2)
    spec.update(ny=18, hessian_reuse=1, precision=precision)
    _run(gpu_ctx, orc, spec, 15)


def test_reuse_three_uncertainties_140_unknowns(gpu_ctx, orc):
    spec = W.bump2d(n=8, degree=4, qpd=5, p=3, v1_spread=0.2)
    spec.update(ny=6, hessian_reuse=1)
    _run(gpu_ctx, orc, spec, 6)


@pytest.mark.parametrize("level,precision", [(1, "fp64"), (2, "fp64"), (2, "bf16")])
def test_reuse_uneven_degrees(gpu_ctx, orc, level, precision):
    """Per-cell degrees 1..4 (16, 40, 80 and 140 unknowns), 125 nodes: the
    16-unknown class runs on the workgroup kernel, the 40-unknown class on
    the 64-lane register-row kernel (inverse reuse only at level 2); each
    cell keeps its inverse in its class's slot."""
    spec = W.bump2d(n=10, degree=4, qpd=5, p=3, v1_spread=0.2)
    spec.update(ny=7, hessian_reuse=level, precision=precision)
    cd = np.random.default_rng(11).integers(1, 5, size=70).astype(np.int8)
    from paper_1912_09238_amd import binding
    nodes, _ = binding.quadrature(3, 5)
    _say("gpu case: hessian reuse %d (%s), uneven degrees 1..4, p=3, 70 cells, 6 steps" % (
        level, precision))
    pid = gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes), cell_degree=cd)
    info = gpu_ctx.step(pid, 6, wait=True)[0]
    got = gpu_ctx.moments(pid)
    gpu_ctx.release(pid)
    ref = dict(spec)
    ref.pop("hessian_reuse")
    ref.pop("precision")
    o = orc.Oracle(ref, ic_fn=lambda nd: W.ic_nodal(ref, nd), cell_degree=cd)
    oinfo = o.step(6)
    assert info["status"] == 0 and oinfo["status"] == 0
    err = parity(got, o.moments())
    _say("  parity %s" % np.array2string(err, precision=2))
    assert np.all(err <= 1e-8), err
    check_parity(got, o.moments(), 1e-8, mode_tol=INEXACT_MODE_TOL)


@pytest.mark.parametrize("case", ["sod_n30", "burgers_n5", "burgers_n10", "bump_n24", "bump_n40"])
def test_reuse_small_kernels(gpu_ctx, orc, case):
    """Register-row kernels: 32-lane groups with DPP broadcasts (Sod, 30
    unknowns; 2D, 24), 16-lane groups (Burgers degree 9), LDS broadcasts
    (Burgers degree 4, 8-lane groups; 2D degree 3, 40 unknowns in 64-lane
    groups); hessian_reuse = 2 extends the inverse reuse to them."""
    if case == "sod_n30":
        spec, steps = W.sod(nx=250, degree=9, qpd=20), 40
    elif case == "burgers_n5":
        spec, steps = W.burgers_shock(nx=200, degree=4, qpd=10), 9
    elif case == "burgers_n10":
        spec, steps = W.burgers_shock(nx=150, degree=9, qpd=14), 8
    elif case == "bump_n24":
        spec, steps = W.bump2d(n=20, degree=2, qpd=6, p=2), 12
        spec["ny"] = 14
    else:
        spec, steps = W.bump2d(n=16, degree=3, qpd=6, p=2), 10
        spec["ny"] = 13
    spec["hessian_reuse"] = 2
    _run(gpu_ctx, orc, spec, steps)


def test_reuse_small_kernel_sod_full_size(gpu_ctx, orc):
    """The Sod workload at its full size (8192 cells, 30 unknowns)."""
    spec = W.sod()
    spec["hessian_reuse"] = 2
    _run(gpu_ctx, orc, spec, 6)


def test_reuse_one_shot_steady(gpu_ctx, orc):
    """One-shot (one Newton step per pseudo-time step, from the stored
    inverse while it halves the residual) reaches the same steady state as
    the exact one-shot oracle."""
    from paper_1912_09238_amd import binding
    spec = W.steady_inflow(nx=100, degree=4, qpd=10, eps=1e-10, one_shot=1)
    spec["hessian_reuse"] = 2
    nodes, _ = binding.quadrature(1, 10)
    _say("gpu case: hessian reuse, one-shot steady inflow to eps 1e-10")
    pid = gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes),
                              dirichlet=W.dirichlet_nodal(spec, nodes))
    info = gpu_ctx.step(pid, 20000, wait=True)[0]
    got = gpu_ctx.moments(pid)
    gpu_ctx.release(pid)
    ref = dict(spec)
    ref.pop("hessian_reuse")
    o = orc.Oracle(ref, ic_fn=lambda nd: W.ic_nodal(ref, nd),
                   dirichlet_fn=lambda nd: W.dirichlet_nodal(ref, nd))
    oinfo = o.step(20000)
    _say("  steps gpu=%d oracle=%d" % (info["steps"], oinfo["steps"]))
    assert info["status"] == 0 and info["done"] == 1
    assert oinfo["status"] == 0 and oinfo["done"] == 1
    err = parity(got, o.moments())
    _say("  parity %s" % np.array2string(err, precision=2))
    assert np.all(err <= 1e-7), err
    check_parity(got, o.moments(), 1e-7, mode_tol=INEXACT_MODE_TOL)


def test_reuse_small_batched_equals_alone(gpu_ctx):
    """Small-kernel classes in a batch (Sod and Burgers, uneven degrees)
    give the same bits as stepping alone."""
    from paper_1912_09238_amd import binding
    a = W.sod(nx=300, degree=9, qpd=20)
    b = W.burgers_shock(nx=180, degree=6, qpd=10)
    c = W.sod(nx=200, degree=9, qpd=20)
    for x in (a, b, c):
        x["hessian_reuse"] = 2
    cds = [None, None, np.random.default_rng(2).integers(2, 10, size=200).astype(np.int8)]
    _say("gpu case: hessian reuse, small kernels, three problems batched vs alone")

    def make(spec, cd):
        nodes, _ = binding.quadrature(1, spec["quad_per_dim"])
        kw = {"cell_degree": cd} if cd is not None else {}
        return gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes), **kw)
    alone = []
    for spec, cd in zip((a, b, c), cds):
        pid = make(spec, cd)
        gpu_ctx.step(pid, 9, wait=True)
        alone.append(gpu_ctx.moments(pid))
        gpu_ctx.release(pid)
    ids = [make(spec, cd) for spec, cd in zip((a, b, c), cds)]
    gpu_ctx.step(ids, 4, wait=True)
    gpu_ctx.step(ids, 5, wait=True)
    for k, pid in enumerate(ids):
        assert np.array_equal(gpu_ctx.moments(pid), alone[k]), k
        gpu_ctx.release(pid)


def test_reuse_batched_equals_alone(gpu_ctx):
    from paper_1912_09238_amd import binding
    a = W.bump2d(n=12, degree=5, qpd=8, p=2)
    a.update(ny=10, hessian_reuse=1, precision="bf16")
    b = W.bump2d(n=8, degree=4, qpd=5, p=3, v1_spread=0.2)
    b.update(ny=9, hessian_reuse=1)
    specs = [a, b]
    _say("gpu case: hessian reuse, two problems batched vs alone")

    def make(spec):
        nodes, _ = binding.quadrature(spec["p"], spec["quad_per_dim"])
        return gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))
    alone = []
    for spec in specs:
        pid = make(spec)
        gpu_ctx.step(pid, 7, wait=True)
        alone.append(gpu_ctx.moments(pid))
        gpu_ctx.release(pid)
    ids = [make(spec) for spec in specs]
    gpu_ctx.step(ids, 7, wait=True)
    for k, pid in enumerate(ids):
        assert np.array_equal(gpu_ctx.moments(pid), alone[k]), k
        gpu_ctx.release(pid)


@pytest.mark.parametrize("level,precision,p", [(1, "fp64", 2), (2, "bf16", 2), (2, "fp64", 3)])
def test_reuse_with_adaptive_levels(gpu_ctx, orc, level, precision, p):
    """Inverse reuse with levels that move every step (each cell keeps one
    slot of the largest class's size; a level change retires its inverse),
    against the exact-Newton adaptive oracle: the levels agree in all but a
    few cells (a decision at a threshold may flip within the dual
    tolerance), E and Var within the precision form's 1e-4, and the moments
    within 1e-8 where every level agrees."""
    from paper_1912_09238_amd import binding
    if p == 2:
        spec = W.bump2d(n=24, degree=5, qpd=8, p=2)
        spec.update(ny=20, adapt=1, min_degree=1, delta_lo=1e-8, delta_hi=1e-4)
    else:
        spec = W.bump2d(n=12, degree=4, qpd=5, p=3, v1_spread=0.2)
        spec.update(ny=10, adapt=1, min_degree=1, delta_lo=1e-6, delta_hi=1e-4)
    spec.update(hessian_reuse=level, precision=precision)
    nodes, _ = binding.quadrature(p, spec["quad_per_dim"])
    _say("gpu case: hessian reuse %d (%s) with adaptive levels, p=%d, %d cells, 8 steps" % (
        level, precision, p, spec["nx"] * spec["ny"]))
    pid = gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))
    info = gpu_ctx.step(pid, 8, wait=True)[0]
    got, lv = gpu_ctx.moments(pid), gpu_ctx.degrees(pid)
    gpu_ctx.release(pid)
    ref = dict(spec)
    ref.pop("hessian_reuse")
    ref.pop("precision")
    o = orc.Oracle(ref, ic_fn=lambda nd: W.ic_nodal(ref, nd))
    oinfo = o.step(8)
    assert info["status"] == 0 and oinfo["status"] == 0
    want, olv = o.moments(), o.degrees()
    moved = int(np.sum(olv != olv.max()))
    flips = int(np.sum(lv != olv))
    rel = lambda a, b: float(np.abs(a - b).sum() / np.abs(b).sum())
    e = rel(got[:, :, 0], want[:, :, 0])
    v = rel(np.sum(got[:, :, 1:] ** 2, axis=2), np.sum(want[:, :, 1:] ** 2, axis=2))
    _say("  levels below the top: %d, differing: %d  E %.2e Var %.2e" % (moved, flips, e, v))
    assert moved > 10 and flips <= max(2, lv.size // 100)
    assert e <= 1e-4 and v <= 1e-4
    if flips == 0:
        err = parity(got, want)
        assert np.all(err <= 1e-8), err
        check_parity(got, want, 1e-8, mode_tol=INEXACT_MODE_TOL)


def test_reuse_stricter_contraction(gpu_ctx, orc):
    """reuse_theta = 0.1: stale steps must cut the residual tenfold."""
    spec = W.bump2d(n=16, degree=5, qpd=8, p=2)
    spec.update(ny=12, hessian_reuse=1, reuse_theta=0.1)
    _run(gpu_ctx, orc, spec, 10)


@pytest.mark.parametrize("bad", [dict(hessian_reuse=3), dict(hessian_reuse=-1),
                                 dict(hessian_reuse=1, reuse_theta=1.0),
                                 dict(hessian_reuse=1, reuse_theta=-0.1)])
def test_reuse_argument_errors(gpu_ctx, bad):
    from paper_1912_09238_amd import binding
    spec = W.bump2d(n=8, degree=5, qpd=8, p=2)
    spec.update(bad)
    nodes, _ = binding.quadrature(2, 8)
    with pytest.raises(binding.IpmError) as e:
        gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))
    assert e.value.code == -1
