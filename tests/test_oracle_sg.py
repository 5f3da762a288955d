"""Pins of the oracle's stochastic-Galerkin pieces: the analytic SG flux of
Burgers' equation (App. A, eq:numFluxAnalytic) and the inadmissibility of SG
gas states with non-positive density or pressure."""
import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W

from . import refs


def _sg_burgers(qpd, flux, nx=40, M=4, bc="outflow"):
    spec = W.burgers_shock(nx=nx, degree=M, qpd=qpd, u_minus=0.0, u_plus=0.0, t_end=0.0)
    spec.update(entropy="quadratic", flux=flux, bc=(bc, bc, "outflow", "outflow"))
    spec["ic"] = dict(kind="shock1d", left=2.0, right=1.0, shift=0.0, spread=1.0)
    return spec


def _oracle(orc, spec):
    return orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd))


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_analytic_flux_equals_kinetic_flux_iff_rule_is_exact(orc, bc):
    """App. A: with Lax-Friedrichs the kinetic flux integrates polynomials of
    degree 3M, so it equals the analytic flux when Gauss-Legendre has
    ceil((3M+1)/2) = 7 points (M = 4), and not with 6."""
    for qpd, exact in ((7, True), (6, False)):
        a = _oracle(orc, _sg_burgers(qpd, "lf", bc=bc))
        b = _oracle(orc, _sg_burgers(qpd, "sg_analytic", bc=bc))
        ia, ib = a.step(12), b.step(12)
        assert ia["status"] == 0 and ib["status"] == 0
        err = np.max(np.abs(a.moments() - b.moments()))
        if exact:
            assert err < 1e-13
        else:
            assert err > 1e-8


def test_analytic_flux_equals_triple_product_reference(orc):
    """Independent SG solver (numpy triple products, its own quadrature)."""
    M = 4
    o = _oracle(orc, _sg_burgers(6, "sg_analytic", M=M))  # the node count only sets dt
    C = refs.triple_products(M)
    uh = o.moments()[:, 0, :].copy()
    for s in range(10):
        info = o.step(1)
        want = refs.sg_burgers_lf_step(uh, 6.0 / 40, info["dt"], C)
        got = o.moments()[:, 0, :]
        assert np.max(np.abs(got - want)) < 1e-12, s
        uh = got.copy()


def test_sg_gas_states_with_negative_density_or_pressure_are_inadmissible(orc):
    u, _, _, ok = orc.closure("quadratic", 3, np.array([1.0, 0.0, 2.5]))
    assert ok and np.array_equal(u, [1.0, 0.0, 2.5])
    assert not orc.closure("quadratic", 3, np.array([-0.1, 0.0, 2.5]))[3]   # rho < 0
    assert not orc.closure("quadratic", 3, np.array([1.0, 3.0, 2.5]))[3]    # p < 0
    assert not orc.closure("quadratic", 4, np.array([1.0, 2.0, 2.0, 2.5]))[3]
    assert orc.closure("quadratic", 1, np.array([-5.0]))[3]  # Burgers: any state


def test_sg_sod_fails_where_the_projection_undershoots(orc):
    """The SG expansion of the uncertain Sod interface oscillates in xi
    (Gibbs); at low degree a node sees a negative density or pressure and the
    run is flagged inadmissible at set-up.  At degree 9 with 11 nodes it runs
    to t_end."""
    bad = W.sod(nx=200, degree=2, qpd=4, t_end=0.14, entropy="quadratic")
    assert _oracle(orc, bad).info["status"] & 2
    good = W.sod(nx=200, degree=9, qpd=11, t_end=0.14, entropy="quadratic")
    o = _oracle(orc, good)
    info = o.run()
    assert info["status"] == 0 and info["done"] == 1
