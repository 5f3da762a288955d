"""Pins of the oracle's per-cell dual problem (Sec. 3.1 eq:L,
eq:dualIterationFunction, eq:tauCrit): derivatives by finite differences,
the dual round trip, and the stochastic-Galerkin special case."""
import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W


def _oracle(orc, spec):
    return orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd))


SPECS = {
    "burgers_logbarrier": lambda: W.burgers_shock(nx=4, degree=4, qpd=10),
    "sod_euler": lambda: W.sod(nx=4, degree=5, qpd=8),
    "euler2d": lambda: W.bump2d(n=2, degree=2, qpd=4),
}


def _sample_dual(o, rng, scale=0.3):
    """A dual vector near an admissible state: the IC dual of a cell plus a
    random perturbation of the higher modes, decaying with the mode index and
    scaled per conserved variable; redrawn until the ansatz is admissible."""
    base = o.dual()[0].copy()
    for _ in range(100):
        lam = base.copy()
        amp = scale * (0.1 + 0.2 * np.abs(base[:, :1]))
        lam[:, 1:] += amp * rng.normal(size=lam[:, 1:].shape) / np.arange(1, o.N)[None, :]
        if o.moments_of_dual(lam)[1]:
            return lam
    raise RuntimeError("no admissible sample")


@pytest.mark.parametrize("name", list(SPECS))
def test_gradient_and_hessian_are_derivatives_of_L(orc, name):
    o = _oracle(orc, SPECS[name]())
    rng = np.random.default_rng(1)
    lam = _sample_dual(o, rng, scale=0.1)
    uhat = o.moments()[0]
    L, g, H, ok = o.dual_cost(lam, uhat)
    assert ok
    n = o.m * o.N
    gf = np.zeros(n)
    Hf = np.zeros((n, n))
    flat = lam.reshape(-1)
    for k in range(n):
        h = 1e-5
        lp, lm = flat.copy(), flat.copy()
        lp[k] += h
        lm[k] -= h
        Lp, gp, _, _ = o.dual_cost(lp.reshape(lam.shape), uhat, hessian=False)
        Lm, gm, _, _ = o.dual_cost(lm.reshape(lam.shape), uhat, hessian=False)
        gf[k] = (Lp - Lm) / (2 * h)
        Hf[:, k] = (gp.reshape(-1) - gm.reshape(-1)) / (2 * h)
    assert np.max(np.abs(gf - g.reshape(-1))) < 1e-6 * (1 + np.max(np.abs(g)))
    assert np.max(np.abs(Hf - H)) < 1e-5 * np.max(np.abs(H))
    assert np.allclose(H, H.T, atol=1e-12 * np.max(np.abs(H)))
    assert np.linalg.eigvalsh(H).min() > 0


@pytest.mark.parametrize("name", list(SPECS))
def test_dual_round_trip(orc, name):
    # uhat = h(lam*)  =>  the dual solve recovers lam* (unique minimiser) and h(lam) = uhat
    o = _oracle(orc, SPECS[name]())
    rng = np.random.default_rng(2)
    for trial in range(3):
        lam_star = _sample_dual(o, rng, scale=0.5)
        uhat, ok = o.moments_of_dual(lam_star)
        assert ok
        lam0 = o.dual()[1 % o.cells].copy()  # start from another cell's dual
        lam, st, its = o.dual_solve(uhat, lam0)
        assert st == 0 and its > 0
        _, g, _, _ = o.dual_cost(lam, uhat, hessian=False)
        assert np.sum(np.sqrt(np.sum(g * g, axis=1))) < 1e-10  # eq:tauCrit
        assert np.max(np.abs(lam - lam_star)) < 1e-7 * (1 + np.max(np.abs(lam_star)))
        u2, _ = o.moments_of_dual(lam)
        assert np.max(np.abs(u2 - uhat)) < 1e-10


def test_converged_dual_takes_no_newton_step(orc):
    o = _oracle(orc, SPECS["sod_euler"]())
    lam0 = o.dual()[2]
    lam, st, its = o.dual_solve(o.moments()[2], lam0)
    assert st == 0 and its == 0 and np.array_equal(lam, lam0)


@pytest.mark.parametrize("m_eq", ["burgers1d", "euler1d"])
def test_quadratic_entropy_dual_is_the_moment_vector(orc, m_eq):
    # quadratic entropy: u_s = Lambda and H = Phi^T W Phi = I, so one Newton step
    # from any start lands on lambda = uhat (the SG closure, Sec. 3.1)
    spec = W.burgers_shock(nx=3, degree=4, qpd=7) if m_eq == "burgers1d" else W.sod(nx=3, degree=4, qpd=7)
    spec["entropy"] = "quadratic"
    o = _oracle(orc, spec)
    rng = np.random.default_rng(4)

    def sample():
        if m_eq == "burgers1d":
            return rng.normal(size=(o.m, o.N))
        # gas: a physical mean state with small higher modes, so that every
        # node stays admissible (SG gas states must have rho, p > 0)
        u = 0.01 * rng.normal(size=(o.m, o.N))
        u[:, 0] = (1.0, 0.1, 2.5)
        return u

    uhat = sample()
    lam, st, its = o.dual_solve(uhat, sample(), one_shot=True)
    assert st == 0 and its == 1
    assert np.max(np.abs(lam - uhat)) < 1e-13 * (1 + np.max(np.abs(uhat)))
    lam2, st2, its2 = o.dual_solve(uhat, sample())
    assert st2 == 0 and its2 == 1


def test_newton_failure_is_reported(orc):
    spec = W.sod(nx=3, degree=5, qpd=8)
    spec["max_newton"] = 1
    spec["tau"] = 1e-15
    o = _oracle(orc, spec)
    rng = np.random.default_rng(9)
    lam_star = _sample_dual(o, rng, scale=0.5)
    uhat, _ = o.moments_of_dual(lam_star)
    _, st, its = o.dual_solve(uhat, o.dual()[0])
    assert st & orc.STATUS["newton"]
