"""Pins of the oracle's determinant machinery: LU inverse, Sherman-Morrison, Woodbury."""
import itertools

import numpy as np
import pytest


def _cofactor_det(A):
    n = len(A)
    if n == 1:
        return A[0][0]
    return sum((-1) ** j * A[0][j] * _cofactor_det([row[:j] + row[j + 1:] for row in A[1:]])
               for j in range(n))


def test_inverse_and_logdet_against_library(orc):
    rng = np.random.default_rng(0)
    for n in [1, 2, 3, 5, 8, 17, 40]:
        A = rng.normal(size=(n, n))
        B, la, sg = orc.inverse(A)
        np.testing.assert_allclose(B @ A, np.eye(n), atol=1e-10 * np.linalg.cond(A))
        s_np, la_np = np.linalg.slogdet(A)
        assert abs(la - la_np) < 1e-12 * max(1.0, abs(la_np))
        assert sg == int(s_np)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_determinant_against_cofactor_expansion(orc, n):
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n))
    _, la, sg = orc.inverse(A)
    d = _cofactor_det(A.tolist())
    assert abs(sg * np.exp(la) - d) < 1e-12 * max(1.0, abs(d))


def test_sherman_morrison_ratio_and_update(orc):
    rng = np.random.default_rng(1)
    for n in range(1, 9):
        A = rng.normal(size=(n, n))
        B, la, sg = orc.inverse(A)
        for k in range(n):
            v = rng.normal(size=n)
            R = v @ B[:, k]
            A2 = A.copy()
            A2[k] = v
            d1 = _cofactor_det(A.tolist()) if n <= 4 else np.linalg.det(A)
            d2 = _cofactor_det(A2.tolist()) if n <= 4 else np.linalg.det(A2)
            assert abs(R - d2 / d1) < 1e-12 * max(1.0, abs(R)) * np.linalg.cond(A)
            B2 = orc.sherman_morrison(B, k, v, R)
            np.testing.assert_allclose(B2 @ A2, np.eye(n), atol=1e-11 * np.linalg.cond(A2))


def test_chain_of_updates_matches_fresh_inverse(orc):
    rng = np.random.default_rng(2)
    n = 12
    A = rng.normal(size=(n, n))
    B, _, _ = orc.inverse(A)
    for step in range(60):
        k = int(rng.integers(n))
        v = rng.normal(size=n)
        R = v @ B[:, k]
        if abs(R) < 0.05:
            continue
        B = orc.sherman_morrison(B, k, v, R)
        A[k] = v
    Bf, _, _ = orc.inverse(A)
    np.testing.assert_allclose(B, Bf, atol=1e-9 * np.linalg.cond(A))


def test_woodbury_equals_sherman_morrison_chain(orc):
    rng = np.random.default_rng(3)
    n = 10
    for m in range(1, n + 1):
        A = rng.normal(size=(n, n))
        B, _, _ = orc.inverse(A)
        rows = rng.permutation(n)[:m]
        V = rng.normal(size=(m, n))
        Bw = orc.woodbury(A, B, rows, V)
        Bs, As = B.copy(), A.copy()
        for q, k in enumerate(rows):
            R = V[q] @ Bs[:, k]
            Bs = orc.sherman_morrison(Bs, k, V[q], R)
            As[k] = V[q]
        np.testing.assert_allclose(Bw, Bs, atol=1e-9 * np.linalg.cond(As))
        np.testing.assert_allclose(Bw @ As, np.eye(n), atol=1e-9 * np.linalg.cond(As))
