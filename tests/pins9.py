"""Pins for the j2d9pt (3 x 3 box) oracle: checks against facts the mathematics fixes.

Each check takes ``run(u, coeffs, T) -> u_T`` (the FP64 box oracle, or a
planted mutant of it) and raises AssertionError when the result disagrees with
an independent statement of what the update must produce.  None of them retypes
the oracle's floating-point loop:

* exact rational brute force on tiny grids, written as a sum over the nine
  (row offset, column offset) pairs of the block (dyadic weights and integer
  inputs keep every FP64 intermediate exact, so the float result must equal the
  exact one bit for bit);
* one-hot weights: T steps with a single weight of 1 move the field by T cells
  along that weight's offset, diagonals included, until the path meets the
  fixed halo ring -- which fixes the orientation of all nine weights;
* a 1 x 1 interior: a scalar affine recurrence whose constant term is the
  weighted sum of all eight halo cells around it (corners included);
* sine modes of the symmetric box (eigenvalue
  c + 2 n cos a + 2 e cos b + 4 d cos a cos b) and, for separable weights
  a(di) b(dj), the weighted mode rho^i sigma^j sin sin that is an eigenvector
  only for the right orientation of both axes;
* invariants: constant preservation, linearity, the semigroup property, row
  and column mirror and transpose symmetry, and the reduction to the 5-point
  stencil when the corner weights are zero (checked exactly on dyadic data).

Weight order (sw, s, se, w, c, e, nw, n, ne): rows i-1, i, i+1 (S to N), each
column j-1, j, j+1 (W to E).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from paper_2306_03336_amd import inputs

EPS64 = np.finfo(np.float64).eps

# (row offset, column offset) of each weight, in the weight order.
OFFSETS = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 0), (0, 1), (1, -1), (1, 0), (1, 1)]
NAMES = ["sw", "s", "se", "w", "c", "e", "nw", "n", "ne"]


def _exact_steps(u, coeffs, T):
    """T steps in exact rational arithmetic: each interior cell becomes the weighted sum of its 3 x 3 block."""
    rows, cols = len(u) - 2, len(u[0]) - 2
    wts = {off: Fraction(x) for off, x in zip(OFFSETS, coeffs)}
    cur = [[Fraction(x) for x in row] for row in u]
    for _ in range(T):
        nxt = [row[:] for row in cur]
        for i in range(1, rows + 1):
            for j in range(1, cols + 1):
                nxt[i][j] = sum(wt * cur[i + di][j + dj] for (di, dj), wt in wts.items())
        cur = nxt
    return cur


def check_exact_rational(run, rng=None):
    rng = np.random.default_rng(21) if rng is None else rng
    cases = [
        # (rows, cols, T, coeffs): dyadic weights, 8-bit integers; every product and partial sum stays exact
        (3, 4, 8, (0.0625, 0.125, 0.03125, 0.125, 0.25, 0.125, 0.0625, 0.125, 0.09375)),
        (5, 7, 9, (0.125, 0.0625, 0.0625, 0.0625, 0.25, 0.125, 0.0625, 0.125, 0.125)),
        (1, 6, 9, (0.25, 0.03125, 0.0625, 0.125, 0.125, 0.03125, 0.125, 0.0625, 0.1875)),
        (7, 1, 9, (0.03125, 0.25, 0.0625, 0.125, 0.125, 0.0625, 0.1875, 0.03125, 0.125)),
        (6, 5, 7, (0.5, 0.0, 0.0, 0.25, 0.0, 0.0, 0.0, 0.0, 0.25)),
    ]
    for rows, cols, T, coeffs in cases:
        u = rng.integers(0, 256, size=(rows + 2, cols + 2)).astype(np.float64)
        got = run(u, coeffs, T)
        want = _exact_steps(u.tolist(), coeffs, T)
        for i in range(rows + 2):
            for j in range(cols + 2):
                assert Fraction(float(got[i, j])) == want[i][j], (rows, cols, T, coeffs, i, j)


def check_one_hot_shift(run, rng=None):
    """Weight (di, dj) = 1: cell (i, j) after T steps holds u(i + t di, j + t dj), t the number of steps the
    path stays inside the interior (a halo cell, once reached, never changes)."""
    rng = np.random.default_rng(22) if rng is None else rng
    rows, cols, T = 9, 13, 5
    u = rng.random((rows + 2, cols + 2))
    for q, (di, dj) in enumerate(OFFSETS):
        coeffs = [0.0] * 9
        coeffs[q] = 1.0
        got = run(u, coeffs, T)
        for i in range(1, rows + 1):
            for j in range(1, cols + 1):
                t = T
                for s in range(1, T + 1):
                    ii, jj = i + s * di, j + s * dj
                    if ii in (0, rows + 1) or jj in (0, cols + 1):
                        t = s
                        break
                assert got[i, j] == u[i + t * di, j + t * dj], (NAMES[q], i, j)


def check_single_cell(run, rng=None):
    rng = np.random.default_rng(23) if rng is None else rng
    for _ in range(4):
        k = rng.uniform(0.02, 0.2, size=9)
        u = rng.uniform(-1, 1, size=(3, 3))
        u[1, 1] = rng.uniform(-2, 2)
        T = 25
        c = k[4]
        b = sum(k[q] * u[1 + di, 1 + dj] for q, (di, dj) in enumerate(OFFSETS) if (di, dj) != (0, 0))
        want = c ** T * u[1, 1] + b * (1 - c ** T) / (1 - c)
        got = run(u, tuple(k), T)[1, 1]
        assert abs(got - want) <= 64 * EPS64 * max(1.0, abs(want)), (got, want)


def _box_lambda(c, n, e, d, rows, cols, p, q):
    a = math.pi * p / (rows + 1)
    b = math.pi * q / (cols + 1)
    return c + 2 * n * math.cos(a) + 2 * e * math.cos(b) + 4 * d * math.cos(a) * math.cos(b)


def check_sine_modes(run):
    """Symmetric box (n = s, e = w, four equal corners d): sin(pi p i/(N+1)) sin(pi q j/(M+1)) is an
    eigenvector (the halo, corners included, is zero on it)."""
    sym = [(0.2, 0.1, 0.1, 0.05), (0.36, 0.12, 0.06, 0.035), (0.1, 0.05, 0.3, 0.0625)]
    for rows, cols, p, q, T in [(31, 45, 1, 1, 120), (64, 48, 2, 5, 60), (1, 33, 1, 3, 80),
                                (17, 1, 4, 1, 80), (20, 20, 20, 1, 30)]:
        for c, n, e, d in sym:
            coeffs = (d, n, d, e, c, e, d, n, d)
            u0 = inputs.sine_grid(rows, cols, p, q)
            lam = _box_lambda(c, n, e, d, rows, cols, p, q)
            Tc = max(1, min(T, int(math.log(0.1) / math.log(abs(lam))) if abs(lam) < 1 else T))
            got = run(u0, coeffs, Tc)
            want = u0 * lam ** Tc
            den = np.max(np.abs(want[1:-1, 1:-1]))
            err = np.max(np.abs(got[1:-1, 1:-1] - want[1:-1, 1:-1])) / den
            assert err < 1e-12, (rows, cols, p, q, (c, n, e, d), Tc, err)


def check_asymmetric_mode(run):
    """Separable weights k(di, dj) = a(di) b(dj): with rho = sqrt(a(-1)/a(1)), sigma = sqrt(b(-1)/b(1)),
    rho^i sigma^j sin(pi p i/(N+1)) sin(pi q j/(M+1)) is an eigenvector with eigenvalue
    (a0 + 2 sqrt(a(-1) a(1)) cos) (b0 + 2 sqrt(b(-1) b(1)) cos) only when row offset +1 is row i+1 and column
    offset +1 is column j+1; swapping either pair (or any corner pair) breaks it."""
    for rows, cols, T, (a, b) in [(20, 28, 50, ((0.1, 0.5, 0.4), (0.15, 0.6, 0.25))),
                                  (12, 9, 40, ((0.45, 0.35, 0.2), (0.05, 0.55, 0.4)))]:
        coeffs = tuple(a[di + 1] * b[dj + 1] for di, dj in OFFSETS)
        rho, sig = math.sqrt(a[0] / a[2]), math.sqrt(b[0] / b[2])
        for p, q in [(1, 1), (3, 2)]:
            u0 = inputs.sine_grid(rows, cols, p, q)
            i = np.arange(rows + 2, dtype=np.float64)[:, None]
            j = np.arange(cols + 2, dtype=np.float64)[None, :]
            u0 = u0 * rho ** i * sig ** j
            lam = (a[1] + 2 * math.sqrt(a[0] * a[2]) * math.cos(math.pi * p / (rows + 1))) * \
                  (b[1] + 2 * math.sqrt(b[0] * b[2]) * math.cos(math.pi * q / (cols + 1)))
            got = run(u0, coeffs, T)
            want = u0 * lam ** T
            den = np.max(np.abs(want[1:-1, 1:-1]))
            err = np.max(np.abs(got[1:-1, 1:-1] - want[1:-1, 1:-1])) / den
            assert err < 1e-12, (rows, cols, coeffs, p, q, err)


def check_constant(run):
    dy = (0.0625, 0.125, 0.0625, 0.125, 0.25, 0.125, 0.0625, 0.125, 0.0625)  # sums to 1 exactly in any order
    u = inputs.empty_grid(12, 17, halo=1.0)
    u[1:-1, 1:-1] = 1.0
    assert np.array_equal(run(u, dy, 40), u)
    u = inputs.empty_grid(7, 5, halo=-3.25)
    u[1:-1, 1:-1] = -3.25
    assert np.array_equal(run(u, dy, 40), u)
    coeffs = inputs.box_weights(7)
    u = inputs.empty_grid(10, 10, halo=2.0)
    u[1:-1, 1:-1] = 2.0
    T = 200
    got = run(u, coeffs, T)
    assert np.max(np.abs(got - 2.0)) <= 2.0 * 10 * T * EPS64


def check_linearity(run):
    rng = np.random.default_rng(24)
    coeffs = inputs.box_weights(3)
    a = inputs.uniform_grid(15, 11, rng)
    b = inputs.uniform_grid(15, 11, rng)
    T = 30
    lhs = run(2.5 * a - 0.75 * b, coeffs, T)
    rhs = 2.5 * run(a, coeffs, T) - 0.75 * run(b, coeffs, T)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def check_max_principle(run):
    coeffs = inputs.box_weights(4)
    u = inputs.uniform_grid(16, 19, 5, halo=0.25)
    lo, hi = float(u[:, :21].min()), float(u[:, :21].max())
    got = run(u, coeffs, 60)[1:-1, 1:-1]
    assert got.min() >= lo - 1e-15 and got.max() <= hi + 1e-15


def _permute(coeffs, fn):
    """Weights of the stencil seen through a map of offsets: new weight at fn(off) = old weight at off."""
    out = [0.0] * 9
    for q, off in enumerate(OFFSETS):
        out[OFFSETS.index(fn(off))] = coeffs[q]
    return tuple(out)


def check_symmetry(run):
    rng = np.random.default_rng(25)
    coeffs = tuple(rng.dirichlet(np.ones(9)))
    u = inputs.uniform_grid(11, 14, rng, halo=0.0)
    u[0, :] = rng.random(16)
    u[-1, :] = rng.random(16)
    u[:, 0] = rng.random(13)
    u[:, -1] = rng.random(13)
    T = 20
    base = run(u, coeffs, T)
    flipped = run(np.ascontiguousarray(u[::-1, :]), _permute(coeffs, lambda o: (-o[0], o[1])), T)[::-1, :]
    assert np.max(np.abs(flipped - base)) < 1e-14
    mirrored = run(np.ascontiguousarray(u[:, ::-1]), _permute(coeffs, lambda o: (o[0], -o[1])), T)[:, ::-1]
    assert np.max(np.abs(mirrored - base)) < 1e-14
    transposed = run(np.ascontiguousarray(u.T), _permute(coeffs, lambda o: (o[1], o[0])), T).T
    assert np.max(np.abs(transposed - base)) < 1e-14


def check_semigroup(run):
    coeffs = inputs.box_weights(6)
    u = inputs.uniform_grid(13, 21, 8, halo=0.5)
    whole = run(u, coeffs, 37)
    split = run(run(u, coeffs, 16), coeffs, 21)
    assert np.array_equal(whole, split)


def check_corners_matter(run):
    """A field that is zero except one halo corner: after one step with only that corner's weight set, just
    the interior cell diagonally next to it holds weight x corner."""
    rows, cols, T = 6, 6, 1
    for q, (di, dj) in enumerate(OFFSETS):
        if di == 0 or dj == 0:
            continue
        u = inputs.empty_grid(rows, cols)
        # the halo corner the weight reads for the nearest interior corner cell
        ci = 0 if di < 0 else rows + 1
        cj = 0 if dj < 0 else cols + 1
        u[ci, cj] = 1.0
        coeffs = [0.0] * 9
        coeffs[q] = 0.5
        got = run(u, coeffs, T)
        ii, jj = ci - di, cj - dj  # the interior cell next to that corner
        assert got[ii, jj] == 0.5, (NAMES[q], got[ii, jj])
        inner = got[1:-1, 1:-1].copy()
        inner[ii - 1, jj - 1] = 0.0
        assert not np.any(inner), NAMES[q]


ALL_CHECKS = [check_exact_rational, check_one_hot_shift, check_single_cell, check_sine_modes,
              check_asymmetric_mode, check_constant, check_linearity, check_max_principle,
              check_symmetry, check_semigroup, check_corners_matter]
