"""Pin of the oracle's IPM trajectories with a non-quadratic entropy and
N < Q: the discrete total entropy never increases.

Why it must hold (Sec. 2-3): the IPM ansatz u(lambda(uhat)) minimises the
quadrature entropy <s(u)>_Q over all nodal states with the moments uhat (its
dual problem is eq:L); the kinetic update moves every quadrature node by the
deterministic scheme, whose numerical flux (Lax-Friedrichs, Rusanov) is
entropy stable at CFL 0.5, so with periodic boundaries sum_j s(u~_jq) <=
sum_j s(u_jq) node by node; the updated moments are those of u~, so the next
ansatz has at most the entropy of u~.  Hence E_n = dx sum_j <s(u_j^n)>_Q is
non-increasing up to the dual tolerance (the ansatz matches its moments to
tau).  A dropped term, a wrong sign or a wrong index in the closure, the
dual solve, the flux or the update breaks it.  The entropies are evaluated
here from their definitions, on the oracle's nodal ansatz, with numpy's
Gauss-Legendre weights."""
import numpy as np

from paper_1912_09238_amd import workloads as W

GAMMA = W.GAMMA


def _weights(qpd):
    _, w = np.polynomial.legendre.leggauss(qpd)
    return w / 2.0


def _log_barrier(u, um, up):
    return (u - um) * np.log(u - um) + (up - u) * np.log(up - u)


def _euler_entropy(U):
    # -rho S with S = ln(p rho^-gamma) / (gamma - 1), the physical entropy
    rho, mom, E = U[..., 0], U[..., 1], U[..., 2]
    p = (GAMMA - 1.0) * (E - 0.5 * mom * mom / rho)
    return -rho * np.log(p * rho ** (-GAMMA)) / (GAMMA - 1.0)


def _history(orc, spec, steps, s_of_nodal):
    o = orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd))
    w = _weights(spec["quad_per_dim"])
    hist = [float(np.sum(s_of_nodal(o.nodal()) * w[None, :]))]
    for _ in range(steps):
        info = o.step(1)
        assert info["status"] == 0, info
        hist.append(float(np.sum(s_of_nodal(o.nodal()) * w[None, :])))
    return np.array(hist)


def test_total_entropy_decays_burgers_log_barrier(orc):
    spec = W.burgers_shock(nx=120, degree=4, qpd=10, t_end=0.0)
    spec["bc"] = ("periodic",) * 4
    um, up = spec["u_minus"], spec["u_plus"]
    hist = _history(orc, spec, 40, lambda U: _log_barrier(U[..., 0], um, up))
    inc = np.diff(hist)
    assert np.all(inc <= 1e-9 * abs(hist[0])), inc.max()
    assert hist[-1] < hist[0] - 1e-3 * abs(hist[0])  # the shocks dissipate


def test_total_entropy_decays_sod_euler(orc):
    spec = W.sod(nx=150, degree=5, qpd=8, t_end=0.0, spread=0.1)
    spec["bc"] = ("periodic",) * 4
    hist = _history(orc, spec, 40, _euler_entropy)
    inc = np.diff(hist)
    assert np.all(inc <= 1e-9 * abs(hist[0])), inc.max()
    assert hist[-1] < hist[0]


def test_total_entropy_decays_euler_2d(orc):
    """Two uncertainties on the periodic square (tensor weights are products
    of the 1D weights, whatever the node order)."""
    spec = W.bump2d(n=16, degree=3, qpd=5, p=2)
    w1 = _weights(5)
    w2 = np.outer(w1, w1).ravel()

    def s2(U):
        rho, mx, my, E = U[..., 0], U[..., 1], U[..., 2], U[..., 3]
        p = (GAMMA - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)
        return -rho * np.log(p * rho ** (-GAMMA)) / (GAMMA - 1.0)

    o = orc.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd))
    hist = [float(np.sum(s2(o.nodal()) * w2[None, :]))]
    for _ in range(20):
        assert o.step(1)["status"] == 0
        hist.append(float(np.sum(s2(o.nodal()) * w2[None, :])))
    inc = np.diff(hist)
    assert np.all(inc <= 1e-9 * abs(hist[0])), inc.max()
    assert hist[-1] < hist[0]
