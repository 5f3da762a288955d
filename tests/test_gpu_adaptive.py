"""GPU parity of dynamic adaptivity (Sec. 5, Alg. ad-IPM) through the C ABI:
levels bitwise equal to the oracle's after every checked step, moments
within the FP64 bound (normwise relative L1 per variable <= 1e-10), the
batched path bitwise equal to stepping alone, and the argument checks."""
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


def _adaptive(spec, lo, hi, dmin):
    s = dict(spec)
    s.update(adapt=1, min_degree=dmin, delta_lo=lo, delta_hi=hi)
    return s


def _make(ctx, spec, cd=None, dirichlet=False):
    from paper_1912_09238_amd import binding
    nodes, _ = binding.quadrature(spec["p"], spec["quad_per_dim"])
    kw = {"cell_degree": cd} if cd is not None else {}
    if dirichlet:
        kw["dirichlet"] = W.dirichlet_nodal(spec, nodes)
    return ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes), **kw)


def _compare(ctx, orc, spec, chunks, cd=None, dirichlet=False):
    """Step GPU and oracle side by side; after each chunk of steps compare
    the levels (bitwise) and the moments."""
    _say("gpu case: adaptive %s nx=%d ny=%d M=%d qpd=%d p=%d one_shot=%d retard=%s chunks=%s" % (
        spec["name"], spec["nx"], spec.get("ny", 1), spec["degree"], spec["quad_per_dim"],
        spec["p"], spec.get("one_shot", 0), spec.get("retard", ()), chunks))
    pid = _make(ctx, spec, cd, dirichlet)
    kw = {"cell_degree": cd} if cd is not None else {}
    if dirichlet:
        kw["dirichlet_fn"] = lambda nd: W.dirichlet_nodal(spec, nd)
    o = orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd), **kw)
    moved = 0
    prev = o.degrees()
    try:
        for k in chunks:
            info = ctx.step(pid, k, wait=True)[0]
            oinfo = o.step(k)
            assert info["status"] == 0, info
            assert oinfo["status"] == 0, oinfo
            assert info["steps"] == oinfo["steps"]
            assert info["retard_stage"] == oinfo["retard_stage"]
            dg, od = ctx.degrees(pid), o.degrees()
            assert np.array_equal(dg, od), np.nonzero(dg != od)
            moved += int(np.sum(od != prev))
            prev = od
            err = parity(ctx.moments(pid), o.moments())
            _say("  step %d: levels %s  parity %s" % (
                info["steps"], np.bincount(od, minlength=spec["degree"] + 1),
                np.array2string(err, precision=2)))
            assert np.all(err <= TOL), err
            check_parity(ctx.moments(pid), o.moments(), TOL)
    finally:
        ctx.release(pid)
    return moved, info, oinfo


def test_adaptive_sod(gpu_ctx, orc):
    spec = _adaptive(W.sod(nx=250, degree=9, qpd=20), 2e-5, 2e-4, 2)
    moved, info, oinfo = _compare(gpu_ctx, orc, spec, [1, 4, 15, 20])
    assert moved > 200
    assert abs(info["newton_iters"] - oinfo["newton_iters"]) <= 0.02 * oinfo["newton_iters"]


def test_adaptive_sod_full_size(gpu_ctx, orc):
    spec = _adaptive(W.sod(), 2e-5, 2e-4, 2)  # 8192 cells, levels 2..9
    moved, _, _ = _compare(gpu_ctx, orc, spec, [3, 5])
    assert moved > 8000


def test_adaptive_burgers_full_run(gpu_ctx, orc):
    spec = _adaptive(W.burgers_shock(nx=200, degree=4, qpd=10), 1e-6, 1e-4, 1)
    moved, info, _ = _compare(gpu_ctx, orc, spec, [2, 100])
    assert info["done"] == 1 and info["steps"] == 9 and moved > 100


def test_adaptive_2d_p2(gpu_ctx, orc):
    spec = _adaptive(W.bump2d(n=24, degree=5, qpd=8, p=2), 1e-8, 1e-4, 1)
    spec["ny"] = 20  # ragged: 480 cells
    moved, _, _ = _compare(gpu_ctx, orc, spec, [2, 4, 6])
    assert moved > 400


def test_adaptive_2d_p3_workgroup_classes(gpu_ctx, orc):
    """p = 3: level 3 (80 unknowns) runs on the workgroup-per-cell kernel;
    initial levels drawn at random."""
    spec = _adaptive(W.bump2d(n=16, degree=4, qpd=5, p=3, v1_spread=0.2), 1e-6, 1e-4, 1)
    cd = np.random.default_rng(3).integers(1, 5, size=256).astype(np.int8)
    moved, _, _ = _compare(gpu_ctx, orc, spec, [1, 3, 6], cd=cd)
    assert moved > 100


@pytest.mark.parametrize("entropy", ["log_barrier", "quadratic"])
def test_adaptive_one_shot_with_retardation(gpu_ctx, orc, entropy):
    """Alg. adosIPM on the steady inflow test: one Newton step per cell and
    pseudo-time step over work lists, levels capped at 1 until the residual
    reaches 3e-3 (about step 230, inside the transient, which then raises
    cells again), then up to 4; run to the steady stop."""
    spec = W.steady_inflow(nx=100, degree=4, qpd=10, eps=1e-10, one_shot=1)
    spec.update(entropy=entropy, adapt=1, min_degree=1, delta_lo=1e-6, delta_hi=5e-2,
                retard=((1, 3e-3), (4, 0.0)))
    moved, info, oinfo = _compare(gpu_ctx, orc, spec, [1, 30, 200, 5, 5, 5, 5, 5000],
                                  dirichlet=True)
    assert info["done"] == 1 and info["retard_stage"] == 1 and moved > 50


def test_adaptive_one_shot_2d_p3(gpu_ctx, orc):
    """Adaptive one-shot in 2D with three uncertainties (workgroup kernel
    class at level 3), random initial levels."""
    spec = _adaptive(W.bump2d(n=16, degree=4, qpd=5, p=3, v1_spread=0.2), 1e-6, 1e-4, 1)
    spec["one_shot"] = 1
    cd = np.random.default_rng(4).integers(1, 5, size=256).astype(np.int8)
    moved, _, _ = _compare(gpu_ctx, orc, spec, [1, 2, 5], cd=cd)
    assert moved > 100


def test_adaptive_batched_equals_alone(gpu_ctx):
    specs = [(_adaptive(W.sod(nx=300, degree=9, qpd=20, t_end=0.0), 2e-5, 2e-4, 2), None),
             (_adaptive(W.burgers_shock(nx=150, degree=4, qpd=10, t_end=0.0), 1e-6, 1e-4, 1),
              None),
             (W.sod(nx=200, degree=5, qpd=8, t_end=0.0), None),
             (_adaptive(dict(W.bump2d(n=12, degree=4, qpd=5, p=3, v1_spread=0.2), one_shot=1),
                        1e-6, 1e-4, 1), None)]
    _say("gpu case: adaptive batch of %d problems vs one by one" % len(specs))
    alone = []
    for spec, cd in specs:
        pid = _make(gpu_ctx, spec, cd)
        gpu_ctx.step(pid, 17, wait=True)
        alone.append((gpu_ctx.moments(pid), gpu_ctx.degrees(pid)))
        gpu_ctx.release(pid)
    ids = [_make(gpu_ctx, spec, cd) for spec, cd in specs]
    gpu_ctx.step(ids[0], 1, wait=True)  # mixed step parities in the batch
    gpu_ctx.step(ids, 6, wait=True)
    gpu_ctx.step(ids, 10, wait=True)
    gpu_ctx.step(ids[1:], 1, wait=True)
    for k, pid in enumerate(ids):
        assert np.array_equal(gpu_ctx.moments(pid), alone[k][0]), k
        assert np.array_equal(gpu_ctx.degrees(pid), alone[k][1]), k
        gpu_ctx.release(pid)


@pytest.mark.parametrize("bad", [dict(min_degree=0), dict(min_degree=10),
                                 dict(delta_lo=1e-3, delta_hi=1e-4), dict(quad_per_dim=9),
                                 dict(retard=((2, 1e-4), (9, 0.0))),  # no steady_eps
                                 dict(steady_eps=1e-8, retard=((5, 1e-4), (3, 0.0))),
                                 dict(steady_eps=1e-8, retard=((1, 1e-4), (9, 0.0))),
                                 dict(steady_eps=1e-8, adapt=0, retard=((2, 1e-4), (9, 0.0)))])
def test_adaptive_argument_errors(gpu_ctx, bad):
    from paper_1912_09238_amd import binding
    spec = _adaptive(W.sod(nx=16, degree=9, qpd=20), 2e-5, 2e-4, 2)
    spec.update(bad)
    with pytest.raises(binding.IpmError) as e:
        _make(gpu_ctx, spec)
    assert e.value.code == -1
