"""Pins of the oracle's quadrature and basis (Sec. 2, eq:numberBasisFcts;
App. A table A) against library routines, closed forms and the paper's
stated counts."""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10, 17, 20, 33, 64])
def test_gauss_legendre_matches_numpy(orc, n):
    x, w = orc.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(x - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-13


@pytest.mark.parametrize("p,qpd", [(1, 10), (2, 4), (3, 3)])
def test_tensor_rule_is_exact_for_monomials(orc, p, qpd):
    # <xi^k> under U(-1,1) is 1/(k+1) for even k, 0 for odd k; exact to 2 qpd - 1 per dim
    nodes, w = orc.quadrature(p, qpd)
    assert abs(w.sum() - 1.0) < 1e-14
    for ks in np.ndindex(*([2 * qpd] * p)):
        want = np.prod([0.0 if k % 2 else 1.0 / (k + 1) for k in ks])
        got = np.sum(w * np.prod(nodes ** np.array(ks)[None, :], axis=1))
        assert abs(got - want) < 1e-13, ks


def test_basis_counts_and_golden(orc):
    for p in range(1, 4):
        for M in range(0, 10):
            assert orc.num_basis(p, M) == math.comb(M + p, p)
            idx = orc.multi_indices(p, M)
            assert idx.shape == (math.comb(M + p, p), p)
            assert len({tuple(r) for r in idx}) == idx.shape[0]
            assert np.all(idx.sum(1) <= M)
    facts = json.load(open(GOLDEN))
    for rec in facts["basis_counts"]:
        assert orc.num_basis(rec["p"], rec["degree"]) == rec["N"], rec["cite"]


def test_multi_index_order_is_graded_prefix(orc):
    # total degree ascending; lower degree sets are prefixes of higher ones
    for p in (1, 2, 3):
        full = orc.multi_indices(p, 6)
        assert np.all(np.diff(full.sum(1)) >= 0)
        for M in range(6):
            sub = orc.multi_indices(p, M)
            assert np.array_equal(full[: sub.shape[0]], sub)
    assert orc.multi_indices(2, 2).tolist() == [[0, 0], [1, 0], [0, 1], [2, 0], [1, 1], [0, 2]]


def test_basis_is_scaled_legendre_1d(orc):
    x = np.linspace(-1, 1, 41)
    Phi = orc.basis_eval(1, 7, x[:, None])
    for i in range(8):
        c = np.zeros(i + 1)
        c[i] = 1.0
        ref = math.sqrt(2 * i + 1) * np.polynomial.legendre.legval(x, c)
        assert np.max(np.abs(Phi[:, i] - ref)) < 1e-12


@pytest.mark.parametrize("p,M,qpd", [(1, 9, 10), (2, 5, 8), (3, 4, 5), (2, 3, 4)])
def test_basis_orthonormal_under_quadrature(orc, p, M, qpd):
    nodes, w = orc.quadrature(p, qpd)
    Phi = orc.basis_eval(p, M, nodes)
    G = Phi.T @ (w[:, None] * Phi)
    assert np.max(np.abs(G - np.eye(Phi.shape[1]))) < 1e-12
    # tensor structure: phi_i(xi) = prod of 1D scaled Legendre factors
    idx = orc.multi_indices(p, M)
    for i in (0, len(idx) // 2, len(idx) - 1):
        ref = np.ones(nodes.shape[0])
        for k in range(p):
            c = np.zeros(idx[i, k] + 1)
            c[-1] = 1.0
            ref *= math.sqrt(2 * idx[i, k] + 1) * np.polynomial.legendre.legval(nodes[:, k], c)
        assert np.max(np.abs(Phi[:, i] - ref)) < 1e-12
