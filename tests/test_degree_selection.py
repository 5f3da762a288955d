"""Static per-cell degree selection by the smoothness indicator
(eq:errorIndicator): oracle pins from closed forms, and the library's host
routine against the oracle on the batching workload's initial data."""
import math

import numpy as np
import pytest

from paper_1912_09238_amd import workloads as W


def _nodes(orc, p, qpd):
    return orc.quadrature(p, qpd)[0]


def test_indicator_of_a_linear_field_is_closed_form(orc):
    # u = a + b xi on [-1, 1]: u_1 = u, the only degree-1 mode is b/sqrt(3),
    # so S_1 = (b^2/3) / (a^2 + b^2/3) and every higher level adds nothing
    a, b = 2.0, 0.6
    x = _nodes(orc, 1, 6)[:, 0]
    S = orc.indicator(1, 4, 6, a + b * x)
    assert S[0] == pytest.approx((b * b / 3) / (a * a + b * b / 3), rel=1e-13)
    assert np.all(np.abs(S[1:]) < 1e-28)


def test_indicator_of_a_quadratic_in_the_second_variable(orc):
    # u = 1 + c P2(xi2), P2 = (3 x^2 - 1)/2: one degree-2 mode c/sqrt(5)
    c = 0.3
    nd = _nodes(orc, 2, 4)
    u = 1.0 + c * 0.5 * (3 * nd[:, 1] ** 2 - 1)
    S = orc.indicator(2, 3, 4, u)
    assert abs(S[0]) < 1e-28
    assert S[1] == pytest.approx((c * c / 5) / (1 + c * c / 5), rel=1e-12)
    assert abs(S[2]) < 1e-28


def test_selection_takes_the_highest_level_above_threshold(orc):
    # an odd cubic has no degree-2 part: S_2 = 0 but S_3 > 0 -> level 3
    x = _nodes(orc, 1, 6)[:, 0]
    ic = np.zeros((4, 6, 1))
    ic[0, :, 0] = 1.0                        # constant        -> 1
    ic[1, :, 0] = 1.0 + 0.5 * x              # linear          -> 1
    ic[2, :, 0] = 1.0 + 0.1 * x ** 3         # odd cubic       -> 3
    p4 = (35 * x ** 4 - 30 * x ** 2 + 3) / 8
    ic[3, :, 0] = 1.0 + 0.05 * p4            # S_4 = (0.05^2/9)/(1 + 0.05^2/9) -> 4
    deg = orc.select_degrees(1, 4, 6, ic, delta_hi=1e-4)
    assert deg.tolist() == [1, 1, 3, 4]
    S4 = orc.indicator(1, 4, 6, ic[3, :, 0])[3]
    assert S4 == pytest.approx((0.05 ** 2 / 9) / (1 + 0.05 ** 2 / 9), rel=1e-11)
    S = orc.indicator(1, 4, 6, ic[2, :, 0])
    assert abs(S[1]) < 1e-28 and S[2] > 1e-4


def test_library_selection_matches_oracle(orc):
    from paper_1912_09238_amd import binding
    # the batch workload's density is linear in xi_1 at t = 0: level 1 everywhere
    for spec in W.batch_problems(count=2, sides=(32, 48)):
        nodes, _ = binding.quadrature(3, spec["quad_per_dim"])
        ic = W.ic_nodal(spec, nodes)
        got = binding.select_degrees(3, 4, spec["quad_per_dim"], ic, 1e-4)
        want = orc.select_degrees(3, 4, spec["quad_per_dim"], ic, 1e-4)
        assert np.array_equal(got, want)
        assert np.all(got == 1)
    # an uncertain interface (Sod, x0 = 0.5 + 0.05 xi) needs high levels near x0 only
    spec = W.sod(nx=400, degree=9, qpd=20)
    nodes, _ = binding.quadrature(1, 20)
    ic = W.ic_nodal(spec, nodes)
    got = binding.select_degrees(1, 9, 20, ic, 1e-4)
    want = orc.select_degrees(1, 9, 20, ic, 1e-4)
    assert np.array_equal(got, want)
    xc = (np.arange(400) + 0.5) / 400
    assert np.all(got[np.abs(xc - 0.5) > 0.06] == 1)
    assert np.all(got[np.abs(xc - 0.5) < 0.04] >= 2)


def test_library_selection_rejects_inexact_quadrature():
    from paper_1912_09238_amd import binding
    with pytest.raises(binding.IpmError):
        binding.select_degrees(1, 4, 4, np.ones((2, 4, 1)))
