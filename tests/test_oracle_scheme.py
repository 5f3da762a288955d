"""Pins of the oracle's full step (Sec. 3.1 eq:momentIterationFunction in the
quadrature form eq:momentUpQuadrature, Algs. 1 and 2) against special cases,
invariants and independent references."""
import math

import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W

from . import refs


def _oracle(orc, spec, **kw):
    return orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd), **kw)


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("qpd,exact", [(7, True), (6, False)])
def test_quadratic_entropy_burgers_equals_analytic_sg_flux(orc, qpd, exact):
    """SG = IPM with quadratic entropy; the kinetic LF flux equals the
    analytic triple-product flux of App. A when the rule integrates degree 3M
    exactly (Gauss-Legendre: qpd >= (3M+1)/2), and not below."""
    M = 4
    spec = W.burgers_shock(nx=40, degree=M, qpd=qpd, u_minus=0.0, u_plus=0.0)
    spec["entropy"] = "quadratic"
    spec["ic"] = dict(kind="shock1d", left=2.0, right=1.0, shift=0.0, spread=1.0)
    o = _oracle(orc, spec)
    C = refs.triple_products(M)
    u0 = o.moments()[:, 0, :]
    info = o.step(1)
    assert info["status"] == 0
    want = refs.sg_burgers_lf_step(u0, 6.0 / 40, info["dt"], C)
    err = np.max(np.abs(o.moments()[:, 0, :] - want))
    if exact:
        assert err < 1e-12
    else:
        assert err > 1e-6


# ---------------------------------------------------------------- P2
def test_single_basis_function_is_deterministic_fv_burgers(orc):
    spec = W.burgers_shock(nx=120, degree=0, qpd=1, t_end=0.05)
    o = _oracle(orc, spec)
    info = o.run()
    assert info["status"] == 0
    u0 = W.ic_nodal(spec, np.zeros((1, 1)))[:, 0, :]  # the single node is xi = 0
    ref, k = refs.fv_burgers_lf(u0, 6.0 / 120, 0.5, t_end=0.05)
    assert k == info["steps"]
    assert np.max(np.abs(o.moments()[:, 0, 0] - ref[:, 0])) < 1e-9


def test_single_basis_function_is_deterministic_fv_sod(orc):
    spec = W.sod(nx=200, degree=0, qpd=1, t_end=0.1)
    o = _oracle(orc, spec)
    info = o.run()
    assert info["status"] == 0
    U0 = W.ic_nodal(spec, np.zeros((1, 1)))
    ref, k = refs.fv_euler_rusanov(U0, 1.0 / 200, 0.5, t_end=0.1)
    assert k == info["steps"]
    assert np.max(np.abs(o.moments()[:, :, 0] - ref[:, 0, :])) < 1e-9


# ---------------------------------------------------------------- P3
@pytest.mark.parametrize("case", ["burgers", "sod"])
def test_n_equals_q_is_coupled_collocation(orc, case):
    """With N = Q (p = 1) Phi is square and the IPM nodal values evolve as Q
    deterministic FV solves sharing one time step, for any entropy."""
    if case == "burgers":
        spec = W.burgers_shock(nx=60, degree=5, qpd=6, t_end=0.01)
        spec["x0"], spec["x1"] = -1.0, 2.0
        dx = 3.0 / 60
    else:
        spec = W.sod(nx=80, degree=3, qpd=4, t_end=0.05, spread=0.1)
        dx = 1.0 / 80
    spec["tau"] = 1e-12
    o = _oracle(orc, spec)
    nod0 = W.ic_nodal(spec, o.nodes)
    info = o.run()
    assert info["status"] == 0
    # with a square Phi the nodal values of the final moments are Phi uhat
    _, _, Phi = o.tables()
    got = np.einsum("qi,cai->cqa", Phi, o.moments())
    if case == "burgers":
        ref, k = refs.fv_burgers_lf(nod0[:, :, 0], dx, 0.5, t_end=spec["t_end"])
        got = got[:, :, 0]
    else:
        ref, k = refs.fv_euler_rusanov(nod0, dx, 0.5, t_end=spec["t_end"])
    assert k == info["steps"]
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-9


# ---------------------------------------------------------------- P2, P3 in 2D
def _bump_nonsquare(degree, qpd, p, bc):
    """2D Euler bump on a non-square grid (30 x 20 cells on [0,1] x [0,0.5]:
    dx = 1/30 != dy = 1/40), off-centre, moving with v = (1, 0.5), with a
    deterministic amplitude so that the single node xi = 0 sees a bump."""
    spec = W.bump2d(n=30, degree=degree, qpd=qpd, p=p, t_end=0.08, center=(0.62, 0.38),
                    amp0=0.5)
    spec["ny"], spec["y1"], spec["bc"] = 20, 0.5, bc
    spec["tau"] = 1e-12
    return spec


BC2D = [("periodic",) * 4, ("periodic", "periodic", "outflow", "outflow"),
        ("outflow", "outflow", "periodic", "periodic")]


@pytest.mark.parametrize("bc", BC2D)
def test_single_basis_function_is_deterministic_fv_euler2d(orc, bc):
    """N = 1 in 2D (degree 0, one node at xi = 0): the unsplit five-point
    update (reading C14 of Sec. 3.1 eq:momentIterationFunction on a
    Cartesian grid) with per-face Rusanov fluxes and the 2D time step
    dt = CFL / (a_x/dx + a_y/dy) (reading C9) is the deterministic finite-volume
    scheme of an independent NumPy solver: same step count, states to 1e-12.
    The grid has dx != dy and the flow v_x != v_y, so exchanging dx and dy in
    the update or the time step, or taking v_x for v_y in the y flux, moves the
    reference by 2e-2 to 7e-2 and fails the pin."""
    spec = _bump_nonsquare(0, 1, 2, bc)
    o = _oracle(orc, spec)
    info = o.run()
    assert info["status"] == 0
    U0 = W.ic_nodal(spec, np.zeros((1, 2))).reshape(20, 30, 1, 4)
    ref, k = refs.fv_euler2d(U0, 1.0 / 30, 0.5 / 20, 0.5, bc, t_end=0.08)
    assert k == info["steps"] and k > 10
    got = o.moments()[:, :, 0].reshape(20, 30, 4)
    assert np.max(np.abs(got - ref[:, :, 0, :])) < 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("bc", BC2D[:2])
def test_n_equals_q_is_coupled_collocation_euler2d(orc, bc):
    """N = Q in 2D (one uncertainty, degree 3, 4 Gauss nodes): Phi is square,
    so the nodal values of the IPM moments evolve as four deterministic 2D
    solves sharing one time step (the largest speed over all of them), for
    the Euler entropy; same non-square grid and flow as the N = 1 pin."""
    spec = _bump_nonsquare(3, 4, 1, bc)
    o = _oracle(orc, spec)
    nod0 = W.ic_nodal(spec, o.nodes)
    info = o.run()
    assert info["status"] == 0
    _, _, Phi = o.tables()
    got = np.einsum("qi,cai->cqa", Phi, o.moments()).reshape(20, 30, 4, 4)
    ref, k = refs.fv_euler2d(nod0.reshape(20, 30, 4, 4), 1.0 / 30, 0.5 / 20, 0.5, bc,
                             t_end=0.08)
    assert k == info["steps"]
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-11


# ---------------------------------------------------------------- P6
def test_conservation_up_to_boundary_flux_sod(orc):
    spec = W.sod(nx=64, degree=4, qpd=8, spread=0.05)
    spec["x0"], spec["x1"] = 0.3, 0.7
    o = _oracle(orc, spec)
    nod = o.nodal()  # ansatz of the converged IC dual, used by the first step
    _, w, Phi = o.tables()
    h_lam = np.einsum("q,cqa,qi->ai", w, nod, Phi)  # sum_j h(lambda_j)
    u0 = o.moments().sum(0)
    assert np.max(np.abs(h_lam - u0)) <= o.cells * 1e-10
    info = o.step(1)
    f_left, _ = refs.euler_flux_1d(nod[0])
    f_right, _ = refs.euler_flux_1d(nod[-1])
    G = np.einsum("q,qa,qi->ai", w, f_right - f_left, Phi)
    got = o.moments().sum(0) - h_lam
    want = -info["dt"] / (0.4 / 64) * G
    assert np.max(np.abs(got - want)) < 1e-12 * (1 + np.max(np.abs(want)))


def test_conservation_periodic_2d(orc):
    spec = W.bump2d(n=12, degree=2, qpd=4, t_end=0.03)
    o = _oracle(orc, spec)
    tot0 = o.moments().sum(0)
    info = o.run()
    assert info["status"] == 0 and info["steps"] >= 3
    drift = np.abs(o.moments().sum(0) - tot0)
    assert np.max(drift) <= info["steps"] * o.cells * 1e-10


# ---------------------------------------------------------------- P7
def test_log_barrier_run_stays_realizable(orc):
    spec = W.burgers_shock()
    o = _oracle(orc, spec)
    info = o.run()
    assert info["status"] == 0 and info["steps"] == 9 and abs(info["t"] - 0.01) < 1e-15
    nod = o.nodal()
    assert nod.min() > spec["u_minus"] and nod.max() < spec["u_plus"]
    assert 0.2 < info["newton_iters"] / info["cell_updates"] < 1.5


# ---------------------------------------------------------------- P9
@pytest.mark.parametrize("one_shot", [0, 1])
def test_steady_state_is_closed_form(orc, one_shot):
    spec = W.steady_inflow(one_shot=one_shot)
    o = _oracle(orc, spec, dirichlet_fn=lambda nd: W.dirichlet_nodal(spec, nd))
    info = o.run(5000)
    assert info["status"] == 0 and info["residual"] <= 1e-10
    want = np.zeros(o.N)
    want[0], want[1] = 1.0, 0.2 / math.sqrt(3.0)
    assert np.max(np.abs(o.moments()[:, 0, :] - want[None, :])) < 5e-8
    if one_shot:
        assert info["newton_iters"] == info["cell_updates"]


def test_one_shot_equals_ipm_for_quadratic_entropy(orc):
    # quadratic entropy: one Newton step solves the dual exactly, so one-shot
    # and classical IPM coincide step by step (Sec. 4 with the SG closure)
    spec = W.burgers_shock(nx=64, degree=4, qpd=8, t_end=0.05)
    spec["entropy"] = "quadratic"
    spec["ic"] = dict(kind="shock1d", left=2.0, right=1.0, shift=0.0, spread=1.0)
    a = _oracle(orc, spec)
    spec1 = dict(spec, one_shot=1)
    b = _oracle(orc, spec1)
    ia, ib = a.run(), b.run()
    assert ia["status"] == 0 and ib["status"] == 0 and ia["steps"] == ib["steps"]
    assert np.max(np.abs(a.moments() - b.moments())) < 1e-12


# ---------------------------------------------------------------- P10
def test_expectation_and_variance_vs_brute_force_collocation(orc):
    """IPM E and Var against 10^4 black-box deterministic solves (midpoint
    samples of xi): a closure + discretisation error, loose bound."""
    spec = W.burgers_shock(nx=100, degree=4, qpd=10, t_end=0.05)
    o = _oracle(orc, spec)
    info = o.run()
    assert info["status"] == 0
    S = 10000
    xi = -1 + (np.arange(S) + 0.5) * 2.0 / S
    u0 = W.ic_nodal(spec, xi[:, None])[:, :, 0]
    u, _ = refs.fv_burgers_lf(u0, 6.0 / 100, 0.5, t_end=0.05, shared_dt=False)
    E_sc, V_sc = u.mean(1), u.var(1)
    uh = o.moments()[:, 0, :]
    E, V = uh[:, 0], np.sum(uh[:, 1:] ** 2, axis=1)
    errE = np.sum(np.abs(E - E_sc)) / np.sum(np.abs(E_sc))
    errV = np.sum(np.abs(V - V_sc)) / np.sum(np.abs(V_sc))
    assert errE < 1e-2 and errV < 0.25, (errE, errV)


# ---------------------------------------------------------------- P11
def test_sod_mean_density_vs_exact_riemann(orc):
    spec = W.sod(nx=400, degree=4, qpd=8, t_end=0.14)
    o = _oracle(orc, spec)
    info = o.run()
    assert info["status"] == 0
    xc = (np.arange(400) + 0.5) / 400
    xg, wg = np.polynomial.legendre.leggauss(40)
    mean = np.zeros(400)
    for xi, wi in zip(xg, wg):
        sol, pstar, ustar = refs.exact_riemann(xc, 0.14, 0.5 + 0.05 * xi, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
        mean += 0.5 * wi * sol[:, 0]
    assert abs(pstar - 0.30313) < 1e-4 and abs(ustar - 0.92745) < 1e-4
    err = np.sum(np.abs(o.moments()[:, 0, 0] - mean)) / np.sum(mean)
    assert err < 2e-2, err
