"""Pins for the oracle's per-bin 2x2 complex solve (the E-field
reconstruction step of section 2; reading: channel c sees
V_c = sum_p H[c][p] E_p, p in {theta, phi}).

Checked against exact Gaussian-rational arithmetic with fractions.Fraction
on small-integer systems, a residual bound on random systems, and the
singular-bin policy.
"""
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import oracle as O


class Q:
    """Exact complex rational a + bi."""

    def __init__(self, a, b=0):
        self.a, self.b = F(a), F(b)

    def __add__(s, o):
        return Q(s.a + o.a, s.b + o.b)

    def __sub__(s, o):
        return Q(s.a - o.a, s.b - o.b)

    def __mul__(s, o):
        return Q(s.a * o.a - s.b * o.b, s.a * o.b + s.b * o.a)

    def __truediv__(s, o):
        d = o.a * o.a + o.b * o.b
        return Q((s.a * o.a + s.b * o.b) / d, (s.b * o.a - s.a * o.b) / d)

    def c(self):
        return complex(float(self.a), float(self.b))


def exact_solve(h, x):
    # Gaussian elimination with exact arithmetic on the 2x2 system h e = x
    a, b, c, d = h[0][0], h[0][1], h[1][0], h[1][1]
    if a.a != 0 or a.b != 0:
        m = c / a
        d2 = d - m * b
        x2 = x[1] - m * x[0]
        e1 = x2 / d2
        e0 = (x[0] - b * e1) / a
    else:
        # swap rows
        m = a / c
        b2 = b - m * d
        x2 = x[0] - m * x[1]
        e1 = x2 / b2
        e0 = (x[1] - d * e1) / c
    return [e0, e1]


def test_exact_rational_small_integer_systems():
    r = np.random.default_rng(11)
    n_done = 0
    while n_done < 200:
        hi = r.integers(-9, 10, size=(2, 2, 2))
        xi = r.integers(-9, 10, size=(2, 2))
        h = [[Q(hi[i, j, 0], hi[i, j, 1]) for j in range(2)] for i in range(2)]
        x = [Q(xi[i, 0], xi[i, 1]) for i in range(2)]
        det = h[0][0] * h[1][1] - h[0][1] * h[1][0]
        if det.a == 0 and det.b == 0:
            continue
        ref = [q.c() for q in exact_solve(h, x)]
        hc = np.array([[h[i][j].c() for j in range(2)] for i in range(2)])
        xc = np.array([x[i].c() for i in range(2)])
        e, sing = O.solve2(hc, xc, 1e-12)
        assert not sing
        kappa = np.sum(np.abs(hc) ** 2) / abs(det.c())
        scale = max(abs(ref[0]), abs(ref[1]), 1e-300)
        assert np.max(np.abs(e - np.array(ref))) <= 10 * 2.0 ** -52 * kappa * scale
        n_done += 1


def test_residual_random_systems():
    r = np.random.default_rng(12)
    for _ in range(500):
        h = r.standard_normal((2, 2)) + 1j * r.standard_normal((2, 2))
        x = r.standard_normal(2) + 1j * r.standard_normal(2)
        e, sing = O.solve2(h, x)
        assert not sing
        res = h @ e - x
        assert np.linalg.norm(res) <= 8 * 2.0 ** -52 * np.linalg.norm(h) * np.linalg.norm(e) + 1e-300
        # orientation: H is [channel][component]; a transposed H would fail this
        assert np.allclose(e, np.linalg.solve(h, x), rtol=1e-12, atol=0)


def test_singular_policy():
    h = np.array([[0.0, 1.0 + 1j], [0.0, 2.0 - 1j]])          # theta column zero: det = 0
    e, sing = O.solve2(h, np.array([1.0, 2.0]), 1e-12)
    assert sing and np.all(e == 0)
    # just above the threshold: solved
    eps = 1e-10
    h2 = np.array([[1.0, 1.0], [1.0, 1.0 + eps]])
    e2, s2 = O.solve2(h2, np.array([1.0, 1.0]), 1e-12)
    assert not s2
    assert np.allclose(h2 @ e2, [1.0, 1.0], atol=1e-5)
    # just below the threshold: treated as singular
    h3 = np.array([[1.0, 1.0], [1.0, 1.0 + 1e-13]])
    _, s3 = O.solve2(h3, np.array([1.0, 1.0]), 1e-12)
    assert s3
