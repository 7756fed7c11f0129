"""Pins for the j3d7pt (3-D seven-point) oracle: checks against facts the mathematics fixes.

Each check takes ``run(u, coeffs, T) -> u_T`` (the FP64 3-D oracle, or a planted mutant of it) on arrays of
shape (depth + 2, rows + 2, pitch) and raises AssertionError when the result disagrees with an independent
statement of what the update must produce.  None of them retypes the oracle's floating-point loop:

* exact rational brute force on tiny grids, written as a sum over the seven (plane, row, column) offsets
  (dyadic weights and integer inputs keep every FP64 intermediate exact, so the float result must equal the
  exact one bit for bit);
* one-hot weights: T steps with a single weight of 1 move the field T cells along that weight's offset until
  the path meets the fixed halo shell -- which fixes the orientation of all seven weights;
* a 1 x 1 x 1 interior: a scalar affine recurrence whose constant term is the weighted sum of its six halo
  neighbours;
* sine modes (eigenvalue c + 2n cos a + 2e cos b + 2t cos g for n = s, e = w, t = b) and the weighted mode
  rho^i sigma^j tau^z sin sin sin, an eigenvector only for the right orientation of all three axes;
* planes decouple without t and b: each plane then follows the j2d5pt update on its own;
* invariants: constants, linearity, the semigroup property, the maximum principle, mirror symmetry of each
  axis (weights swapped accordingly).

Weight order (c, n, s, e, w, t, b): N = row i+1, S = row i-1, E = column j+1, W = column j-1, T = plane z+1,
B = plane z-1.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from paper_2306_03336_amd import inputs

EPS64 = np.finfo(np.float64).eps

# (plane, row, column) offset of each weight, in the weight order.
OFFSETS = [(0, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (1, 0, 0), (-1, 0, 0)]
NAMES = ["c", "n", "s", "e", "w", "t", "b"]


def _exact_steps(u, coeffs, T):
    """T steps in exact rational arithmetic: each interior cell becomes the weighted sum over the seven offsets."""
    depth, rows, cols = len(u) - 2, len(u[0]) - 2, len(u[0][0]) - 2
    wts = [(off, Fraction(x)) for off, x in zip(OFFSETS, coeffs)]
    cur = [[[Fraction(x) for x in row] for row in plane] for plane in u]
    for _ in range(T):
        nxt = [[row[:] for row in plane] for plane in cur]
        for z in range(1, depth + 1):
            for i in range(1, rows + 1):
                for j in range(1, cols + 1):
                    nxt[z][i][j] = sum(wt * cur[z + dz][i + di][j + dj] for (dz, di, dj), wt in wts)
        cur = nxt
    return cur


def check_exact_rational(run, rng=None):
    rng = np.random.default_rng(31) if rng is None else rng
    cases = [
        # (depth, rows, cols, T, coeffs): dyadic weights summing to 1, 8-bit integers: exact in FP64
        (3, 4, 5, 8, (0.25, 0.125, 0.0625, 0.125, 0.1875, 0.125, 0.125)),
        (2, 3, 6, 9, (0.0625, 0.25, 0.125, 0.0625, 0.125, 0.25, 0.125)),
        (5, 1, 3, 9, (0.125, 0.0625, 0.25, 0.125, 0.0625, 0.1875, 0.1875)),
        (1, 5, 2, 9, (0.1875, 0.125, 0.125, 0.25, 0.0625, 0.1875, 0.0625)),
    ]
    for depth, rows, cols, T, coeffs in cases:
        u = rng.integers(0, 256, size=(depth + 2, rows + 2, cols + 2)).astype(np.float64)
        got = run(u, coeffs, T)
        want = _exact_steps(u.tolist(), coeffs, T)
        for z in range(depth + 2):
            for i in range(rows + 2):
                for j in range(cols + 2):
                    assert Fraction(float(got[z, i, j])) == want[z][i][j], (depth, rows, cols, T, z, i, j)


def check_one_hot_shift(run, rng=None):
    rng = np.random.default_rng(32) if rng is None else rng
    depth, rows, cols, T = 6, 7, 9, 4
    u = rng.random((depth + 2, rows + 2, cols + 2))
    Z = np.arange(1, depth + 1)[:, None, None]
    I = np.arange(1, rows + 1)[None, :, None]
    J = np.arange(1, cols + 1)[None, None, :]
    Zb, Ib, Jb = np.broadcast_arrays(Z, I, J)
    for q, (dz, di, dj) in enumerate(OFFSETS):
        coeffs = [0.0] * 7
        coeffs[q] = 1.0
        got = run(u, coeffs, T)[1:-1, 1:-1, 1:-1]
        # the path stays interior for t steps, then sits on the halo shell, whose value never changes
        zz = np.clip(Zb + T * dz, 0, depth + 1)
        ii = np.clip(Ib + T * di, 0, rows + 1)
        jj = np.clip(Jb + T * dj, 0, cols + 1)
        assert np.array_equal(got, u[zz, ii, jj]), NAMES[q]


def check_single_cell(run, rng=None):
    rng = np.random.default_rng(33) if rng is None else rng
    for _ in range(4):
        k = rng.uniform(0.03, 0.25, size=7)
        u = rng.uniform(-1, 1, size=(3, 3, 3))
        u[1, 1, 1] = rng.uniform(-2, 2)
        for z, i, j in [(0, 0, 0), (0, 2, 2), (2, 0, 2), (2, 2, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]:
            u[z, i, j] = 1e300  # edges and corners of the shell: never read
        T = 20
        c = k[0]
        b = sum(k[q] * u[1 + dz, 1 + di, 1 + dj] for q, (dz, di, dj) in enumerate(OFFSETS) if q > 0)
        want = c ** T * u[1, 1, 1] + b * (1 - c ** T) / (1 - c)
        got = run(u, tuple(k), T)[1, 1, 1]
        assert abs(got - want) <= 64 * EPS64 * max(1.0, abs(want)), (got, want)


def check_sine_modes(run):
    for (depth, rows, cols, r, p, q, T) in [(9, 11, 13, 1, 1, 1, 40), (6, 14, 10, 2, 3, 1, 30), (1, 17, 9, 1, 2, 4, 30),
                                            (12, 1, 8, 3, 1, 2, 30)]:
        for c, n, e, t in [(0.4, 0.1, 0.1, 0.1), (0.1, 0.05, 0.3, 0.1), (0.2, 0.2, 0.1, 0.1)]:
            coeffs = (c, n, n, e, e, t, t)
            u0 = inputs.sine_grid3(depth, rows, cols, r, p, q)
            lam = (c + 2 * n * math.cos(math.pi * p / (rows + 1)) + 2 * e * math.cos(math.pi * q / (cols + 1))
                   + 2 * t * math.cos(math.pi * r / (depth + 1)))
            Tc = max(1, min(T, int(math.log(0.1) / math.log(abs(lam))) if abs(lam) < 1 else T))
            got = run(u0, coeffs, Tc)
            want = u0 * lam ** Tc
            den = np.max(np.abs(want[1:-1, 1:-1, 1:-1]))
            err = np.max(np.abs(got[1:-1, 1:-1, 1:-1] - want[1:-1, 1:-1, 1:-1])) / den
            assert err < 1e-12, (depth, rows, cols, (c, n, e, t), err)


def check_asymmetric_mode(run):
    """rho^i sigma^j tau^z sin sin sin with rho = sqrt(s/n), sigma = sqrt(w/e), tau = sqrt(b/t) is an eigenvector,
    eigenvalue c + 2 sqrt(ns) cos + 2 sqrt(ew) cos + 2 sqrt(tb) cos, only for the right orientation of each axis."""
    for depth, rows, cols, T, coeffs in [(8, 12, 10, 30, (0.3, 0.2, 0.05, 0.04, 0.16, 0.2, 0.05)),
                                         (10, 7, 9, 25, (0.1, 0.05, 0.3, 0.2, 0.05, 0.06, 0.24))]:
        c, n, s, e, w, t, b = coeffs
        rho, sig, tau = math.sqrt(s / n), math.sqrt(w / e), math.sqrt(b / t)
        u0 = inputs.sine_grid3(depth, rows, cols, 1, 1, 1)
        z = np.arange(depth + 2, dtype=np.float64)[:, None, None]
        i = np.arange(rows + 2, dtype=np.float64)[None, :, None]
        j = np.arange(cols + 2, dtype=np.float64)[None, None, :]
        u0 = u0 * rho ** i * sig ** j * tau ** z
        lam = (c + 2 * math.sqrt(n * s) * math.cos(math.pi / (rows + 1)) + 2 * math.sqrt(e * w) *
               math.cos(math.pi / (cols + 1)) + 2 * math.sqrt(t * b) * math.cos(math.pi / (depth + 1)))
        got = run(u0, coeffs, T)
        want = u0 * lam ** T
        den = np.max(np.abs(want[1:-1, 1:-1, 1:-1]))
        err = np.max(np.abs(got[1:-1, 1:-1, 1:-1] - want[1:-1, 1:-1, 1:-1])) / den
        assert err < 1e-12, (coeffs, err)


def check_planes_decouple(run):
    """With t = b = 0 the planes do not interact: each must follow the 2-D five-point update of its own plane,
    checked against an exact rational j2d5pt written here from the neighbour definition."""
    rng = np.random.default_rng(34)
    depth, rows, cols, T = 3, 5, 6, 6
    coeffs = (0.25, 0.125, 0.1875, 0.3125, 0.125, 0.0, 0.0)
    u = rng.integers(0, 256, size=(depth + 2, rows + 2, cols + 2)).astype(np.float64)
    got = run(u, coeffs, T)
    c, n, s, e, w = (Fraction(x) for x in coeffs[:5])
    for z in range(1, depth + 1):
        cur = [[Fraction(x) for x in row] for row in u[z].tolist()]
        for _ in range(T):
            nxt = [row[:] for row in cur]
            for i in range(1, rows + 1):
                for j in range(1, cols + 1):
                    nxt[i][j] = (c * cur[i][j] + n * cur[i + 1][j] + s * cur[i - 1][j] + e * cur[i][j + 1]
                                 + w * cur[i][j - 1])
            cur = nxt
        for i in range(rows + 2):
            for j in range(cols + 2):
                assert Fraction(float(got[z, i, j])) == cur[i][j], (z, i, j)


def check_constant(run):
    dy = (0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125)  # sums to 1 exactly in any order
    u = inputs.empty_grid3(5, 6, 7, halo=1.0)
    u[1:-1, 1:-1, 1:-1] = 1.0
    assert np.array_equal(run(u, dy, 30), u)
    coeffs = inputs.weights7(7)
    u = inputs.empty_grid3(6, 5, 4, halo=2.0)
    u[1:-1, 1:-1, 1:-1] = 2.0
    T = 100
    got = run(u, coeffs, T)
    assert np.max(np.abs(got - 2.0)) <= 2.0 * 8 * T * EPS64


def check_linearity(run):
    rng = np.random.default_rng(35)
    coeffs = inputs.weights7(3)
    a = inputs.uniform_grid3(5, 7, 6, rng)
    b = inputs.uniform_grid3(5, 7, 6, rng)
    T = 20
    lhs = run(2.5 * a - 0.75 * b, coeffs, T)
    rhs = 2.5 * run(a, coeffs, T) - 0.75 * run(b, coeffs, T)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def check_max_principle(run):
    coeffs = inputs.weights7(4)
    u = inputs.uniform_grid3(6, 8, 7, 5, halo=0.25)
    lo, hi = float(u.min()), float(u.max())
    got = run(u, coeffs, 40)[1:-1, 1:-1, 1:-1]
    assert got.min() >= lo - 1e-15 and got.max() <= hi + 1e-15


def check_symmetry(run):
    rng = np.random.default_rng(36)
    c, n, s, e, w, t, b = coeffs = tuple(rng.dirichlet(np.ones(7)))
    u = rng.random((6, 7, 8))  # random halo shell too
    T = 12
    base = run(u, coeffs, T)
    fz = run(np.ascontiguousarray(u[::-1]), (c, n, s, e, w, b, t), T)[::-1]
    assert np.max(np.abs(fz - base)) < 1e-14
    fi = run(np.ascontiguousarray(u[:, ::-1]), (c, s, n, e, w, t, b), T)[:, ::-1]
    assert np.max(np.abs(fi - base)) < 1e-14
    fj = run(np.ascontiguousarray(u[:, :, ::-1]), (c, n, s, w, e, t, b), T)[:, :, ::-1]
    assert np.max(np.abs(fj - base)) < 1e-14


def check_semigroup(run):
    coeffs = inputs.weights7(6)
    u = inputs.uniform_grid3(5, 9, 11, 8, halo=0.5)
    whole = run(u, coeffs, 23)
    split = run(run(u, coeffs, 9), coeffs, 14)
    assert np.array_equal(whole, split)


ALL_CHECKS = [check_exact_rational, check_one_hot_shift, check_single_cell, check_sine_modes,
              check_asymmetric_mode, check_planes_decouple, check_constant, check_linearity, check_max_principle,
              check_symmetry, check_semigroup]
