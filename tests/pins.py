"""Pins for the j2d5pt oracle: checks against facts the mathematics fixes.

Each check takes ``run(u, coeffs, T) -> u_T`` (the FP64 oracle, or a planted
mutant of it) and raises AssertionError when the result disagrees with an
independent statement of what the update must produce.  None of them retypes
the oracle's floating-point loop:

* exact rational brute force on tiny grids (dyadic weights keep every
  intermediate exactly representable in FP64, so the float result must equal
  the exact one bit for bit);
* one-hot weights: the T-step result is a pure shift of the input toward the
  neighbour whose weight is 1, which fixes the orientation of N/S/E/W;
* a single interior cell: a scalar affine recurrence with a geometric-series
  closed form;
* discrete sine modes: eigenvectors of the update with a closed-form
  eigenvalue (symmetric weights), and the weighted variant that is an
  eigenvector only for the right orientation (asymmetric weights);
* invariants: constant preservation, linearity, maximum principle, mirror
  and transpose symmetry, the semigroup property.

Geometry (Listing 1 of the paper, x = column j, y = row i):
W = (i, j-1), E = (i, j+1), S = (i-1, j), N = (i+1, j).  Coefficients are
ordered (c, n, s, e, w).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from paper_2306_03336_amd import inputs

EPS64 = np.finfo(np.float64).eps


def _exact_steps(u, coeffs, T):
    """T steps in exact rational arithmetic, written from the neighbour definition."""
    rows, cols = len(u) - 2, len(u[0]) - 2
    c, n, s, e, w = (Fraction(x) for x in coeffs)
    cur = [[Fraction(x) for x in row] for row in u]
    for _ in range(T):
        nxt = [row[:] for row in cur]
        for i in range(1, rows + 1):
            for j in range(1, cols + 1):
                nxt[i][j] = (c * cur[i][j] + n * cur[i + 1][j] + s * cur[i - 1][j]
                             + e * cur[i][j + 1] + w * cur[i][j - 1])
        cur = nxt
    return cur


def check_exact_rational(run, rng=None):
    rng = np.random.default_rng(11) if rng is None else rng
    cases = [
        # (rows, cols, T, coeffs): every product and partial sum of these stays exact in FP64
        (3, 4, 12, (0.5, 0.125, 0.125, 0.125, 0.125)),
        (5, 7, 15, (0.5, 0.125, 0.125, 0.125, 0.125)),
        (8, 10, 10, (0.5, 0.25, 0.125, 0.0625, 0.0625)),
        (6, 9, 10, (0.0625, 0.5, 0.0625, 0.125, 0.25)),
        (1, 6, 11, (0.25, 0.125, 0.0625, 0.5, 0.0625)),
        (7, 1, 11, (0.25, 0.5, 0.0625, 0.125, 0.0625)),
    ]
    for rows, cols, T, coeffs in cases:
        u = rng.integers(0, 256, size=(rows + 2, cols + 2)).astype(np.float64)
        got = run(u, coeffs, T)
        want = _exact_steps(u.tolist(), coeffs, T)
        for i in range(rows + 2):
            for j in range(cols + 2):
                assert Fraction(float(got[i, j])) == want[i][j], (rows, cols, T, coeffs, i, j)


def check_one_hot_shift(run, rng=None):
    rng = np.random.default_rng(12) if rng is None else rng
    rows, cols, T = 9, 13, 5
    u = rng.random((rows + 2, cols + 2))
    I = np.arange(1, rows + 1)[:, None]
    J = np.arange(1, cols + 1)[None, :]
    expect = {
        "c": u[1:rows + 1, 1:cols + 1],
        # N = (i+1, j): the field moves up by one row per step; the bottom halo row feeds in
        "n": u[np.minimum(I + T, rows + 1), J],
        "s": u[np.maximum(I - T, 0), J],
        "e": u[I, np.minimum(J + T, cols + 1)],
        "w": u[I, np.maximum(J - T, 0)],
    }
    for k, name in enumerate("cnsew"):
        coeffs = [0.0] * 5
        coeffs[k] = 1.0
        got = run(u, coeffs, T)
        assert np.array_equal(got[1:rows + 1, 1:cols + 1], expect[name]), name


def check_single_cell(run, rng=None):
    rng = np.random.default_rng(13) if rng is None else rng
    for _ in range(4):
        c, n, s, e, w = rng.uniform(0.05, 0.6, size=5)
        u = np.zeros((3, 3))
        u[1, 1] = rng.uniform(-2, 2)
        hN, hS, hE, hW = rng.uniform(-1, 1, size=4)
        u[2, 1], u[0, 1], u[1, 2], u[1, 0] = hN, hS, hE, hW
        u[0, 0] = u[0, 2] = u[2, 0] = u[2, 2] = 1e300  # corners: never read
        T = 25
        b = n * hN + s * hS + e * hE + w * hW
        want = c ** T * u[1, 1] + b * (1 - c ** T) / (1 - c)
        got = run(u, (c, n, s, e, w), T)[1, 1]
        assert abs(got - want) <= 64 * EPS64 * max(1.0, abs(want)), (got, want)


def _sine_lambda(coeffs, rows, cols, p, q):
    c, n, s, e, w = coeffs
    return c + 2 * math.sqrt(n * s) * math.cos(math.pi * p / (rows + 1)) + \
        2 * math.sqrt(e * w) * math.cos(math.pi * q / (cols + 1))


def check_sine_modes(run):
    sym = [(0.2, 0.2, 0.2, 0.2, 0.2), (0.36, 0.22, 0.22, 0.1, 0.1), (0.1, 0.05, 0.05, 0.4, 0.4)]
    for rows, cols, p, q, T in [(31, 45, 1, 1, 120), (64, 48, 2, 5, 60), (1, 33, 1, 3, 80),
                                (17, 1, 4, 1, 80), (20, 20, 20, 1, 30)]:
        for coeffs in sym:
            u0 = inputs.sine_grid(rows, cols, p, q)
            lam = _sine_lambda(coeffs, rows, cols, p, q)
            # Rounding excites the other modes; keep lam^T >= 0.1 so none of them can outgrow
            # this one by more than 10x, which keeps the relative check tight.
            Tc = max(1, min(T, int(math.log(0.1) / math.log(abs(lam))) if abs(lam) < 1 else T))
            got = run(u0, coeffs, Tc)
            want = u0 * lam ** Tc
            den = np.max(np.abs(want[1:-1, 1:-1]))
            err = np.max(np.abs(got[1:-1, 1:-1] - want[1:-1, 1:-1])) / den
            assert err < 1e-12, (rows, cols, p, q, coeffs, Tc, err)


def check_asymmetric_mode(run):
    """rho^i sigma^j sin(pi p i/(N+1)) sin(pi q j/(M+1)), rho = sqrt(s/n), sigma = sqrt(w/e).

    It is an eigenvector with eigenvalue c + 2 sqrt(ns) cos(.) + 2 sqrt(ew) cos(.) only when
    N is (i+1, j) and E is (i, j+1); swapping either pair breaks it.
    """
    for rows, cols, T, coeffs in [(20, 28, 50, (0.3, 0.25, 0.1, 0.05, 0.3)),
                                  (12, 9, 40, (0.1, 0.05, 0.4, 0.3, 0.15))]:
        c, n, s, e, w = coeffs
        rho, sig = math.sqrt(s / n), math.sqrt(w / e)
        for p, q in [(1, 1), (3, 2)]:
            u0 = inputs.sine_grid(rows, cols, p, q)
            i = np.arange(rows + 2, dtype=np.float64)[:, None]
            j = np.arange(cols + 2, dtype=np.float64)[None, :]
            u0 = u0 * rho ** i * sig ** j
            lam = _sine_lambda(coeffs, rows, cols, p, q)
            got = run(u0, coeffs, T)
            want = u0 * lam ** T
            den = np.max(np.abs(want[1:-1, 1:-1]))
            err = np.max(np.abs(got[1:-1, 1:-1] - want[1:-1, 1:-1])) / den
            assert err < 1e-12, (rows, cols, coeffs, p, q, err)


def check_constant(run):
    u = inputs.empty_grid(12, 17, halo=1.0)
    u[1:-1, 1:-1] = 1.0
    got = run(u, inputs.EQUAL_WEIGHTS, 40)
    assert np.array_equal(got, u)  # 0.2 + 0.2 + 0.2 + 0.2 + 0.2 == 1 exactly, in this order
    u = inputs.empty_grid(7, 5, halo=-3.25)
    u[1:-1, 1:-1] = -3.25
    got = run(u, (0.5, 0.125, 0.125, 0.125, 0.125), 40)
    assert np.array_equal(got, u)
    coeffs = inputs.dirichlet_weights(7)
    u = inputs.empty_grid(10, 10, halo=2.0)
    u[1:-1, 1:-1] = 2.0
    T = 200
    got = run(u, coeffs, T)
    assert np.max(np.abs(got - 2.0)) <= 2.0 * 6 * T * EPS64


def check_linearity(run):
    rng = np.random.default_rng(14)
    coeffs = inputs.dirichlet_weights(3)
    a = inputs.uniform_grid(15, 11, rng)
    b = inputs.uniform_grid(15, 11, rng)
    T = 30
    lhs = run(2.5 * a - 0.75 * b, coeffs, T)
    rhs = 2.5 * run(a, coeffs, T) - 0.75 * run(b, coeffs, T)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def check_max_principle(run):
    coeffs = inputs.dirichlet_weights(4)
    u = inputs.uniform_grid(16, 19, 5, halo=0.25)
    lo, hi = float(u[:, :21].min()), float(u[:, :21].max())
    got = run(u, coeffs, 60)[1:-1, 1:-1]
    assert got.min() >= lo - 1e-15 and got.max() <= hi + 1e-15


def check_symmetry(run):
    rng = np.random.default_rng(15)
    c, n, s, e, w = coeffs = (0.31, 0.27, 0.05, 0.22, 0.15)
    u = inputs.uniform_grid(11, 14, rng, halo=0.0)
    u[0, :] = rng.random(16)
    u[-1, :] = rng.random(16)
    u[:, 0] = rng.random(13)
    u[:, -1] = rng.random(13)
    T = 20
    base = run(u, coeffs, T)
    flipped = run(np.ascontiguousarray(u[::-1, :]), (c, s, n, e, w), T)[::-1, :]
    assert np.max(np.abs(flipped - base)) < 1e-14
    mirrored = run(np.ascontiguousarray(u[:, ::-1]), (c, n, s, w, e), T)[:, ::-1]
    assert np.max(np.abs(mirrored - base)) < 1e-14
    transposed = run(np.ascontiguousarray(u.T), (c, e, w, n, s), T).T
    assert np.max(np.abs(transposed - base)) < 1e-14


def check_semigroup(run):
    coeffs = inputs.dirichlet_weights(6)
    u = inputs.uniform_grid(13, 21, 8, halo=0.5)
    whole = run(u, coeffs, 37)
    split = run(run(u, coeffs, 16), coeffs, 21)
    assert np.array_equal(whole, split)


ALL_CHECKS = [check_exact_rational, check_one_hot_shift, check_single_cell, check_sine_modes,
              check_asymmetric_mode, check_constant, check_linearity, check_max_principle,
              check_symmetry, check_semigroup]
