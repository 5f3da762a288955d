"""Pins of the oracle's closures u_s = (grad s)^-1, grad u_s and s_* (Sec. 2
eq:ansatz, Sec. 3.1; App. B): finite differences, the Legendre-Fenchel
identity, the entropy-gradient round trip, and the paper's printed Euler
ansatz under the reading of its exponent."""
import numpy as np
import pytest

GAMMA = 1.4


def _rand_euler_state(rng, d):
    rho = rng.uniform(0.2, 3.0)
    v = rng.uniform(-1.5, 1.5, size=d)
    p = rng.uniform(0.1, 3.0)
    E = p / (GAMMA - 1) + 0.5 * rho * v @ v
    return np.concatenate([[rho], rho * v, [E]])


CASES = [("quadratic", 1), ("quadratic", 3), ("log_barrier", 1), ("euler", 3), ("euler", 4)]


def _lam_samples(orc, ent, m, rng, k=8):
    out = []
    for _ in range(k):
        if ent == "euler":
            u = _rand_euler_state(rng, m - 2)
            lam, ok = orc.entropy_grad(ent, m, u, gamma=GAMMA)
            assert ok
        elif ent == "log_barrier":
            lam = rng.uniform(-6, 6, size=1)
        elif m >= 3:  # quadratic entropy of a gas: the dual is the state, physical
            lam = _rand_euler_state(rng, m - 2)
        else:
            lam = rng.normal(size=m)
        out.append(lam)
    return out


@pytest.mark.parametrize("ent,m", CASES)
def test_jacobian_and_sstar_gradient_by_finite_differences(orc, ent, m):
    rng = np.random.default_rng(3)
    um, up = 0.8, 12.2
    for lam in _lam_samples(orc, ent, m, rng):
        u, J, ss, ok = orc.closure(ent, m, lam, gamma=GAMMA, um=um, up=up)
        assert ok
        Jfd = np.zeros((m, m))
        gfd = np.zeros(m)
        for b in range(m):
            h = 1e-6 * max(1.0, abs(lam[b]))
            lp, lm_ = lam.copy(), lam.copy()
            lp[b] += h
            lm_[b] -= h
            up_, _, sp, _ = orc.closure(ent, m, lp, gamma=GAMMA, um=um, up=up)
            um_, _, sm, _ = orc.closure(ent, m, lm_, gamma=GAMMA, um=um, up=up)
            Jfd[:, b] = (up_ - um_) / (2 * h)
            gfd[b] = (sp - sm) / (2 * h)
        scale = np.max(np.abs(J)) + 1e-300
        assert np.max(np.abs(J - Jfd)) / scale < 1e-7
        assert np.max(np.abs(gfd - u)) / (np.max(np.abs(u)) + 1e-300) < 1e-7  # grad s_* = u_s
        assert np.allclose(J, J.T, rtol=0, atol=1e-12 * scale)
        assert np.all(np.linalg.eigvalsh(J) > 0)


@pytest.mark.parametrize("ent,m", CASES)
def test_fenchel_identity_and_round_trip(orc, ent, m):
    # s(u_s(L)) + s_*(L) = L . u_s(L)   and   grad s(u_s(L)) = L
    rng = np.random.default_rng(5)
    um, up = 0.8, 12.2
    for lam in _lam_samples(orc, ent, m, rng):
        u, J, ss, ok = orc.closure(ent, m, lam, gamma=GAMMA, um=um, up=up)
        s = orc.entropy(ent, m, u, gamma=GAMMA, um=um, up=up)
        assert abs(s + ss - lam @ u) < 1e-10 * (1 + abs(lam @ u))
        lam2, ok2 = orc.entropy_grad(ent, m, u, gamma=GAMMA, um=um, up=up)
        assert ok2
        assert np.max(np.abs(lam2 - lam)) < 1e-9 * (1 + np.max(np.abs(lam)))


def test_entropy_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(7)
    for m in (3, 4):
        u = _rand_euler_state(rng, m - 2)
        lam, ok = orc.entropy_grad("euler", m, u, gamma=GAMMA)
        for a in range(m):
            h = 1e-6 * abs(u[a]) + 1e-7
            up_, um_ = u.copy(), u.copy()
            up_[a] += h
            um_[a] -= h
            fd = (orc.entropy("euler", m, up_, gamma=GAMMA) - orc.entropy("euler", m, um_, gamma=GAMMA)) / (2 * h)
            assert abs(fd - lam[a]) < 1e-6 * (1 + abs(lam[a]))
    # E-derivative is -rho/eps (the printed form is a garbled reciprocal)
    u = np.array([0.7, 0.3, -0.2, 2.0])
    eps = u[3] - (u[1] ** 2 + u[2] ** 2) / (2 * u[0])
    lam, _ = orc.entropy_grad("euler", 4, u, gamma=GAMMA)
    assert abs(lam[3] + u[0] / eps) < 1e-14


def test_euler_ansatz_matches_printed_formulas_up_to_shift(orc):
    # App. B prints alpha(L) with -2 L4 gamma in the exponent; the inverse of the
    # printed gradient needs +2 L4 gamma, i.e. alpha_printed(L) = rho(L1 + 2 gamma).
    rng = np.random.default_rng(11)
    for _ in range(5):
        u0 = _rand_euler_state(rng, 2)
        L, _ = orc.entropy_grad("euler", 4, u0, gamma=GAMMA)
        L1, L2, L3, L4 = L
        alpha = np.exp((L2 ** 2 + L3 ** 2 - 2 * L1 * L4 - 2 * L4 * GAMMA) / (2 * L4 * (1 - GAMMA))) * (-L4) ** (1 / (1 - GAMMA))
        shifted = np.array([L1 + 2 * GAMMA, L2, L3, L4])
        u, _, _, ok = orc.closure("euler", 4, shifted, gamma=GAMMA)
        assert ok
        assert abs(u[0] - alpha) < 1e-12 * alpha
        assert abs(u[1] + L2 * alpha / L4) < 1e-12 * (1 + abs(u[1]))
        assert abs(u[2] + L3 * alpha / L4) < 1e-12 * (1 + abs(u[2]))
        assert abs(u[3] + alpha * (-L2 ** 2 - L3 ** 2 + 2 * L4) / (2 * L4 ** 2)) < 1e-12 * u[3]
        # and the unshifted closure inverts the entropy gradient exactly
        v, _, _, _ = orc.closure("euler", 4, L, gamma=GAMMA)
        assert np.max(np.abs(v - u0)) < 1e-12 * np.max(np.abs(u0))


def test_euler_domain_and_log_barrier_saturation(orc):
    _, _, _, ok = orc.closure("euler", 3, np.array([0.0, 0.0, 0.5]), gamma=GAMMA)
    assert not ok  # Lambda_E >= 0 is outside the closure's domain
    for L in (-800.0, -40.0, 0.0, 40.0, 800.0):
        u, J, ss, ok = orc.closure("log_barrier", 1, np.array([L]), um=0.8, up=12.2)
        assert ok and 0.8 <= u[0] <= 12.2 and J[0, 0] >= 0 and np.isfinite(ss)


def test_sstar_of_euler_is_scaled_density(orc):
    rng = np.random.default_rng(2)
    u0 = _rand_euler_state(rng, 1)
    L, _ = orc.entropy_grad("euler", 3, u0, gamma=GAMMA)
    u, _, ss, _ = orc.closure("euler", 3, L, gamma=GAMMA)
    assert abs(ss - (GAMMA - 1) * u0[0]) < 1e-13
