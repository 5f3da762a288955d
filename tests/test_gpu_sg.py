"""GPU: the stochastic-Galerkin baseline -- the analytic SG flux of Burgers'
equation (App. A) against the oracle and against the kinetic flux, and the
realizability check of SG gas states -- through the C ABI."""
import sys

import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W

from .conftest import check_parity, parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sg_burgers(qpd, flux, nx=300, M=9, bc="outflow"):
    spec = W.burgers_shock(nx=nx, degree=M, qpd=qpd, u_minus=0.0, u_plus=0.0, t_end=0.0)
    spec.update(entropy="quadratic", flux=flux, bc=(bc, bc, "outflow", "outflow"))
    spec["ic"] = dict(kind="shock1d", left=2.0, right=1.0, shift=0.0, spread=1.0)
    return spec


def _make(ctx, spec):
    from paper_1912_09238_amd import binding
    nodes, _ = binding.quadrature(spec["p"], spec["quad_per_dim"])
    return ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes))


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_analytic_sg_flux_vs_oracle(gpu_ctx, orc, bc):
    spec = _sg_burgers(15, "sg_analytic", bc=bc)  # N = 10
    _say("gpu case: analytic SG flux, Burgers nx=300 M=9 qpd=15 bc=%s, 40 steps" % bc)
    pid = _make(gpu_ctx, spec)
    info = gpu_ctx.step(pid, 40, wait=True)[0]
    got = gpu_ctx.moments(pid)
    gpu_ctx.release(pid)
    o = orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd))
    oinfo = o.step(40)
    assert info["status"] == 0 and oinfo["status"] == 0
    assert info["steps"] == oinfo["steps"] == 40
    err = parity(got, o.moments())
    _say("  parity %s" % np.array2string(err, precision=2))
    assert np.all(err <= 1e-10), err
    check_parity(got, o.moments(), 1e-10)


def test_analytic_equals_kinetic_flux_on_the_gpu(gpu_ctx):
    """Exactness of the kinetic LF flux at ceil((3M+1)/2) = 14 nodes (M = 9)."""
    _say("gpu case: analytic vs kinetic LF flux, Burgers nx=300 M=9 qpd=14, 30 steps")
    out = []
    for flux in ("lf", "sg_analytic"):
        pid = _make(gpu_ctx, _sg_burgers(14, flux))
        info = gpu_ctx.step(pid, 30, wait=True)[0]
        assert info["status"] == 0
        out.append(gpu_ctx.moments(pid))
        gpu_ctx.release(pid)
    assert np.max(np.abs(out[0] - out[1])) < 1e-12


def test_sg_sod_realizability(gpu_ctx, orc):
    """Degree 2: the SG projection has a node with negative density or
    pressure, reported at set-up as on the oracle; degree 9 with 11 nodes
    runs, in parity with the oracle."""
    from paper_1912_09238_amd import binding
    bad = W.sod(nx=200, degree=2, qpd=4, t_end=0.14, entropy="quadratic")
    _say("gpu case: SG Sod degree 2 (inadmissible at set-up)")
    with pytest.raises(binding.IpmError) as e:
        _make(gpu_ctx, bad)
    assert e.value.code == -4
    assert orc.Oracle(bad, ic_fn=lambda nd: W.ic_nodal(bad, nd)).info["status"] & 2
    good = W.sod(nx=200, degree=9, qpd=11, t_end=0.14, entropy="quadratic")
    _say("gpu case: SG Sod degree 9 qpd 11 to t_end")
    pid = _make(gpu_ctx, good)
    gpu_ctx.step(pid, 1000, wait=True)
    info = gpu_ctx.query(pid)
    got = gpu_ctx.moments(pid)
    gpu_ctx.release(pid)
    o = orc.Oracle(good, ic_fn=lambda nd: W.ic_nodal(good, nd))
    oinfo = o.run()
    assert info["status"] == 0 and info["done"] == 1 and info["steps"] == oinfo["steps"]
    err = parity(got, o.moments())
    _say("  parity %s" % np.array2string(err, precision=2))
    assert np.all(err <= 1e-10), err
    check_parity(got, o.moments(), 1e-10)


@pytest.mark.parametrize("bad", [dict(entropy="log_barrier", u_minus=0.5, u_plus=2.5),
                                 dict(degree=16, quad_per_dim=25),
                                 dict(bc=("dirichlet", "outflow", "outflow", "outflow")),
                                 dict(adapt=1, min_degree=1, delta_lo=1e-6, delta_hi=1e-4)])
def test_analytic_flux_argument_errors(gpu_ctx, bad):
    from paper_1912_09238_amd import binding
    spec = _sg_burgers(15, "sg_analytic", nx=16)
    spec.update(bad)
    with pytest.raises(binding.IpmError) as e:
        from paper_1912_09238_amd import binding as B
        nodes, _ = B.quadrature(spec["p"], spec["quad_per_dim"])
        kw = {}
        if spec["bc"][0] == "dirichlet":
            kw["dirichlet"] = np.zeros((4, nodes.shape[0], 1))
        gpu_ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes), **kw)
    assert e.value.code == -1
