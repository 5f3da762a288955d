"""Pins of the oracle's dynamic adaptivity (Sec. 5, eq:errorIndicator,
eq:adaptiveFVUpdate, Alg. ad-IPM) against special cases and an independent
stochastic-Galerkin reference."""
import math

import numpy as np

from paper_1912_09238_amd import workloads as W

from . import refs


def _oracle(orc, spec, **kw):
    return orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd), **kw)


def test_adaptive_without_level_changes_equals_static(orc):
    """Thresholds that never fire (no indicator is below -1 or above +inf):
    the adaptive run is the static run with the same per-cell degrees,
    bit for bit."""
    rng = np.random.default_rng(5)
    spec = W.sod(nx=60, degree=5, qpd=8, t_end=0.05, spread=0.1)
    deg = rng.integers(2, 6, size=60).astype(np.int8)
    a = _oracle(orc, spec, cell_degree=deg)
    a.step(12)
    spec_ad = dict(spec, adapt=1, min_degree=1, delta_lo=-1.0, delta_hi=math.inf)
    b = _oracle(orc, spec_ad, cell_degree=deg)
    b.step(12)
    assert np.array_equal(a.moments(), b.moments())
    assert np.array_equal(b.degrees(), deg)


def _sg_levels(uh, deg, lo, hi, dmin, dmax):
    """eq:errorIndicator by orthonormality (p = 1): the indicator at level d
    is the energy of mode d over the energy of modes 0..d."""
    out = deg.copy()
    for c in range(uh.shape[0]):
        d = int(deg[c])
        num = uh[c, d] ** 2
        den = float(np.sum(uh[c, :d + 1] ** 2))
        s = num / den
        if s < lo and d > dmin:
            out[c] = d - 1
        elif s > hi and d < dmax:
            out[c] = d + 1
    return out


def test_adaptive_sg_burgers_equals_triple_product_reference(orc):
    """Quadratic entropy (stochastic Galerkin, lambda = uhat) with levels
    moving every step: the oracle equals an independent SG solver with the
    analytic triple-product Lax-Friedrichs flux (App. A), levels from the
    indicator by orthonormality, every cell's state at its own level, and the
    update projected on the new level (eq:adaptiveFVUpdate)."""
    M, qpd, nx, steps = 4, 7, 40, 15
    lo, hi, dmin = 1e-6, 1e-3, 1
    spec = W.burgers_shock(nx=nx, degree=M, qpd=qpd, u_minus=0.0, u_plus=0.0)
    spec["entropy"] = "quadratic"
    spec["ic"] = dict(kind="shock1d", left=2.0, right=1.0, shift=0.0, spread=1.0)
    spec.update(adapt=1, min_degree=dmin, delta_lo=lo, delta_hi=hi, t_end=0.0)
    o = _oracle(orc, spec)
    uh = o.moments()[:, 0, :].copy()
    deg = np.full(nx, M, dtype=np.int8)
    C = refs.triple_products(M)
    x, _ = np.polynomial.legendre.leggauss(qpd)
    P = np.stack([math.sqrt(2 * i + 1) * np.polynomial.legendre.legval(x, np.eye(M + 1)[i])
                  for i in range(M + 1)], axis=1)  # [Q][N]
    dx = 6.0 / nx
    changed = 0
    for s in range(steps):
        new = _sg_levels(uh, deg, lo, hi, dmin, M)
        changed += int(np.sum(new != deg))
        a = np.max(np.abs(uh @ P.T))
        dt = 0.5 * dx / a
        un = refs.sg_burgers_lf_step(uh, dx, dt, C)
        for c in range(nx):
            un[c, new[c] + 1:] = 0.0
        info = o.step(1)
        assert info["status"] == 0
        assert abs(info["dt"] - dt) <= 1e-13 * dt
        assert np.array_equal(o.degrees(), new), s
        got = o.moments()[:, 0, :]
        assert np.max(np.abs(got - un)) < 1e-12, s
        uh, deg = got.copy(), new
    assert changed > 20  # the levels did move
    assert deg.min() == dmin and deg.max() == M


def test_adaptive_sod_conserves_mean_and_refines_at_waves(orc):
    """Every level keeps mode 0, so the adaptive scheme conserves the mean
    state (the waves stay inside the tube); cells away from the waves drop to
    the lowest level and the cells at the uncertain shock and contact keep
    high levels."""
    spec = W.sod(nx=200, degree=6, qpd=8, t_end=0.08, spread=0.05)
    spec.update(adapt=1, min_degree=1, delta_lo=2e-5, delta_hi=2e-4)
    o = _oracle(orc, spec)
    m0 = o.moments()[:, :, 0].sum(axis=0)
    info = o.run()
    assert info["status"] == 0 and info["done"] == 1
    m1 = o.moments()[:, :, 0].sum(axis=0)
    # boundary fluxes of the undisturbed states: momentum gains t (p_L - p_R) / dx;
    # each step may move the means by the dual tolerance (the old-moment term
    # is the ansatz h(lambda))
    want = m0 + np.array([0.0, 0.08 * (1.0 - 0.1) * 200, 0.0])
    assert np.max(np.abs(m1 - want)) <= info["steps"] * 200 * 1e-10
    deg = o.degrees()
    assert deg[:40].max() == 1 and deg[-30:].max() == 1  # undisturbed states
    assert deg.max() >= 4
    # modes above each cell's level are zero
    mom = o.moments()
    for c in range(200):
        assert np.all(mom[c, :, deg[c] + 1:] == 0.0)


def _steady_sg(nx=100, one_shot=1, retard=()):
    spec = W.steady_inflow(nx=nx, degree=4, qpd=10, eps=1e-10, one_shot=one_shot)
    spec.update(entropy="quadratic", adapt=1, min_degree=1, delta_lo=1e-6, delta_hi=5e-2,
                retard=retard)
    return spec


def _steady_oracle(orc, spec):
    return orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd),
                      dirichlet_fn=lambda nd: W.dirichlet_nodal(spec, nd))


def test_retarded_adaptive_one_shot_reaches_the_closed_form_steady_state(orc):
    """Alg. adosIPM on the steady inflow test with the quadratic entropy: the
    steady state is uhat = (1, 0.2/sqrt(3), 0, ...) in every cell at any
    level >= 1.  Stage 0 caps the levels at 1 until the residual reaches
    1e-4; without the cap the transient raises cells to level 4."""
    want = np.zeros(5)
    want[0], want[1] = 1.0, 0.2 / math.sqrt(3.0)
    for retard, capped in (((), False), (((1, 1e-4), (4, 0.0)), True)):
        o = _steady_oracle(orc, _steady_sg(retard=retard))
        top, stage0_top, stage_seen = 0, 0, set()
        while True:
            info = o.step(1)
            lv = int(o.degrees().max())
            top = max(top, lv)
            stage_seen.add(info["retard_stage"])
            if info["retard_stage"] == 0:
                stage0_top = max(stage0_top, lv)
            if info["done"] or info["steps"] > 5000:
                break
        assert info["status"] == 0 and info["done"] == 1
        assert np.max(np.abs(o.moments()[:, 0, :] - want)) < 5e-8
        if capped:
            assert stage_seen == {0, 1} and info["retard_stage"] == 1 and stage0_top == 1
        else:
            assert top == 4


def test_single_full_stage_equals_no_retardation(orc):
    """A schedule of one stage capped at the full degree is no schedule."""
    a = _steady_oracle(orc, _steady_sg(nx=60))
    b = _steady_oracle(orc, _steady_sg(nx=60, retard=((4, 0.0),)))
    ia, ib = a.step(400), b.step(400)
    assert ia["steps"] == ib["steps"]
    assert np.array_equal(a.moments(), b.moments())
    assert np.array_equal(a.degrees(), b.degrees())


def test_adaptive_one_shot_sg_equals_triple_product_reference(orc):
    """With the quadratic entropy one Newton step solves the dual exactly, so
    the adaptive one-shot (Alg. adosIPM without a cap) follows the same
    independent SG solver as the adaptive IPM."""
    M, qpd, nx, steps = 4, 7, 40, 12
    lo, hi, dmin = 1e-6, 1e-3, 1
    spec = W.burgers_shock(nx=nx, degree=M, qpd=qpd, u_minus=0.0, u_plus=0.0)
    spec["entropy"] = "quadratic"
    spec["ic"] = dict(kind="shock1d", left=2.0, right=1.0, shift=0.0, spread=1.0)
    spec.update(adapt=1, min_degree=dmin, delta_lo=lo, delta_hi=hi, t_end=0.0, one_shot=1)
    o = _oracle(orc, spec)
    uh = o.moments()[:, 0, :].copy()
    deg = np.full(nx, M, dtype=np.int8)
    C = refs.triple_products(M)
    x, _ = np.polynomial.legendre.leggauss(qpd)
    P = np.stack([math.sqrt(2 * i + 1) * np.polynomial.legendre.legval(x, np.eye(M + 1)[i])
                  for i in range(M + 1)], axis=1)
    dx = 6.0 / nx
    for s in range(steps):
        new = _sg_levels(uh, deg, lo, hi, dmin, M)
        dt = 0.5 * dx / np.max(np.abs(uh @ P.T))
        un = refs.sg_burgers_lf_step(uh, dx, dt, C)
        for c in range(nx):
            un[c, new[c] + 1:] = 0.0
        info = o.step(1)
        assert info["status"] == 0
        assert np.array_equal(o.degrees(), new), s
        got = o.moments()[:, 0, :]
        assert np.max(np.abs(got - un)) < 1e-12, s
        uh, deg = got.copy(), new
