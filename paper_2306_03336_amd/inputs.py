"""Seeded synthetic inputs for the j2d5pt, j2d9pt and j3d7pt workloads.

This module only draws numbers and lays them out; it holds none of the
stencil's arithmetic.  Both the GPU tests/benchmark and the CPU oracle take
their inputs from here, so the two sides always see the same bytes.

Layout: a 2-D array of shape (rows + 2, pitch), row-major.  The interior is
``[1:rows+1, 1:cols+1]``; the one-cell ring around it is the Dirichlet halo;
columns beyond ``cols + 1`` (pitch padding) are zero and never read.

Coefficient order: j2d5pt (c, n, s, e, w); j2d9pt, the 3 x 3 box, (sw, s, se,
w, c, e, nw, n, ne) -- rows i-1, i, i+1, each west to east; j3d7pt (c, n, s,
e, w, t, b) -- t for plane z+1, b for plane z-1.

3-D layout (j3d7pt): an array of shape (depth + 2, rows + 2, pitch), plane z,
row i, column j; interior ``[1:depth+1, 1:rows+1, 1:cols+1]``; the one-cell
shell around it is the Dirichlet halo.

Recipes (all with ``numpy.random.default_rng``, PCG64):

* ``uniform_grid(rows, cols, seed, halo)``: interior ~ U[0, 1) drawn row by
  row with ``rng.random((rows, cols))``; halo cells set to ``halo``.
* ``dirichlet_weights(seed)``: ``rng.dirichlet(ones(5))`` -- five non-negative
  weights summing to 1 (up to the rounding of the draw), used as drawn.
* ``box_weights(seed)``: ``rng.dirichlet(ones(9))`` -- the same for the nine
  weights of the box.
* ``weights7(seed)``: ``rng.dirichlet(ones(7))`` -- the seven of j3d7pt.
* ``uniform_grid3(depth, rows, cols, seed, halo)``: interior ~ U[0, 1) drawn
  as ``rng.random((depth, rows, cols))``; halo shell set to ``halo``.
* ``workload(name)``: the named configurations below draw, from
  ``default_rng(seed)``, first the weights (when they are random) and then the
  interior.
* ``batched_set(seed=5)``: 64 problems; from ``default_rng(seed)`` in this
  order: sides ``clip(rint(exp(U(ln 128, ln 3072))), 128, 3072)``, step counts
  ``integers(100, 2001)``, weights per problem; dtype alternates FP64 (even
  index) / FP32 (odd index); each field is drawn from its own child seed of
  ``SeedSequence(seed).spawn(64)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EQUAL_WEIGHTS = (0.2, 0.2, 0.2, 0.2, 0.2)
EQUAL_WEIGHTS9 = (1.0 / 9,) * 9


def empty_grid(rows: int, cols: int, halo: float = 0.0, pitch: int | None = None,
               dtype=np.float64) -> np.ndarray:
    """A grid whose interior is zero and whose halo ring is ``halo``."""
    if rows < 1 or cols < 1:
        raise ValueError("rows and cols must be >= 1")
    pitch = cols + 2 if pitch is None else int(pitch)
    if pitch < cols + 2:
        raise ValueError("pitch must be >= cols + 2")
    g = np.zeros((rows + 2, pitch), dtype=dtype)
    g[0, :cols + 2] = halo
    g[rows + 1, :cols + 2] = halo
    g[:, 0] = halo
    g[:, cols + 1] = halo
    return g


def uniform_grid(rows: int, cols: int, seed, halo: float = 0.0, pitch: int | None = None,
                 dtype=np.float64) -> np.ndarray:
    """Interior ~ U[0, 1) from ``default_rng(seed)``; the draw is made in FP64."""
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    g = empty_grid(rows, cols, halo, pitch, np.float64)
    g[1:rows + 1, 1:cols + 1] = rng.random((rows, cols))
    return g.astype(dtype, copy=False)


def sine_grid(rows: int, cols: int, p: int = 1, q: int = 1, halo: float = 0.0,
              pitch: int | None = None, dtype=np.float64) -> np.ndarray:
    """Interior sin(pi p i / (rows+1)) * sin(pi q j / (cols+1)), i, j counted from 1."""
    g = empty_grid(rows, cols, halo, pitch, np.float64)
    i = np.arange(1, rows + 1, dtype=np.float64)[:, None]
    j = np.arange(1, cols + 1, dtype=np.float64)[None, :]
    g[1:rows + 1, 1:cols + 1] = np.sin(math.pi * p * i / (rows + 1)) * np.sin(math.pi * q * j / (cols + 1))
    return g.astype(dtype, copy=False)


def empty_grid3(depth: int, rows: int, cols: int, halo: float = 0.0, pitch: int | None = None,
                dtype=np.float64) -> np.ndarray:
    """A 3-D grid whose interior is zero and whose halo shell is ``halo``."""
    if depth < 1 or rows < 1 or cols < 1:
        raise ValueError("depth, rows and cols must be >= 1")
    pitch = cols + 2 if pitch is None else int(pitch)
    if pitch < cols + 2:
        raise ValueError("pitch must be >= cols + 2")
    g = np.zeros((depth + 2, rows + 2, pitch), dtype=dtype)
    g[:, :, :cols + 2] = halo
    g[1:depth + 1, 1:rows + 1, 1:cols + 1] = 0
    return g


def uniform_grid3(depth: int, rows: int, cols: int, seed, halo: float = 0.0, pitch: int | None = None,
                  dtype=np.float64) -> np.ndarray:
    """Interior ~ U[0, 1) from ``default_rng(seed)``, drawn in FP64 plane by plane."""
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    g = empty_grid3(depth, rows, cols, halo, pitch, np.float64)
    g[1:depth + 1, 1:rows + 1, 1:cols + 1] = rng.random((depth, rows, cols))
    return g.astype(dtype, copy=False)


def sine_grid3(depth: int, rows: int, cols: int, r: int = 1, p: int = 1, q: int = 1,
               pitch: int | None = None, dtype=np.float64) -> np.ndarray:
    """Interior sin(pi r z/(depth+1)) sin(pi p i/(rows+1)) sin(pi q j/(cols+1)), counted from 1; zero halo."""
    g = empty_grid3(depth, rows, cols, 0.0, pitch, np.float64)
    z = np.arange(1, depth + 1, dtype=np.float64)[:, None, None]
    i = np.arange(1, rows + 1, dtype=np.float64)[None, :, None]
    j = np.arange(1, cols + 1, dtype=np.float64)[None, None, :]
    g[1:depth + 1, 1:rows + 1, 1:cols + 1] = (np.sin(math.pi * r * z / (depth + 1)) *
                                              np.sin(math.pi * p * i / (rows + 1)) *
                                              np.sin(math.pi * q * j / (cols + 1)))
    return g.astype(dtype, copy=False)


def weights7(seed) -> tuple:
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(7))
    return tuple(float(x) for x in w)


def dirichlet_weights(seed) -> tuple:
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(5))
    return tuple(float(x) for x in w)


def box_weights(seed) -> tuple:
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(9))
    return tuple(float(x) for x in w)


@dataclass
class Workload:
    """One named configuration: the grid, the coefficients and the step count."""
    name: str
    rows: int
    cols: int
    T: int
    dtype: str               # "f64" or "f32": the precision the GPU path computes in
    coeffs: tuple
    halo: float
    seed: int
    weights: str = "equal"   # "equal" or "dirichlet"
    note: str = ""
    pts: int = 5             # 5: j2d5pt; 9: j2d9pt (the 3 x 3 box)

    @property
    def cell_updates(self) -> int:
        return self.rows * self.cols * self.T

    def grid(self, pitch: int | None = None, dtype=np.float64) -> np.ndarray:
        """The FP64 initial grid (draws the weights first when they are random)."""
        rng = np.random.default_rng(self.seed)
        if self.weights == "dirichlet":
            rng.dirichlet(np.ones(self.pts))
        return uniform_grid(self.rows, self.cols, rng, self.halo, pitch, dtype)


def _mk(name, rows, cols, T, dtype, weights, halo, seed, note=""):
    pts = 9 if name.startswith("j2d9pt") else 5
    if weights == "dirichlet":
        coeffs = box_weights(seed) if pts == 9 else dirichlet_weights(seed)
    else:
        coeffs = EQUAL_WEIGHTS9 if pts == 9 else EQUAL_WEIGHTS
    return Workload(name, rows, cols, T, dtype, coeffs, halo, seed, weights, note, pts)


WORKLOADS = {
    w.name: w for w in [
        _mk("j2d5pt_256x256_f64_T16", 256, 256, 16, "f64", "equal", 0.0, 1,
            "small case: every tile and a ragged edge, oracle in well under a second"),
        _mk("j2d5pt_2048x2048_f64_T10000", 2048, 2048, 10000, "f64", "dirichlet", 0.0, 2,
            "whole grid resident on chip"),
        _mk("j2d5pt_8192x8192_f64_T1000", 8192, 8192, 1000, "f64", "equal", 1.0, 3,
            "larger than on-chip memory: tile-serial sweep"),
        _mk("j2d5pt_3072x3072_f32_T2000", 3072, 3072, 2000, "f32", "equal", 0.0, 4,
            "precision pair, FP32 half: resident"),
        _mk("j2d5pt_3072x3072_f64_T2000", 3072, 3072, 2000, "f64", "equal", 0.0, 4,
            "precision pair, FP64 half (same input): larger than on-chip memory, tile-serial sweep"),
        _mk("j2d5pt_16384x16384_f32_T2000", 16384, 16384, 2000, "f32", "equal", 0.0, 4,
            "precision pair, FP32 half: tile-serial sweep"),
        _mk("j2d5pt_16384x16384_f64_T2000", 16384, 16384, 2000, "f64", "equal", 0.0, 4,
            "precision pair, FP64 half (same input): tile-serial sweep; the largest single-GPU FP64 run"),
        _mk("j2d9pt_256x256_f64_T16", 256, 256, 16, "f64", "dirichlet", 0.25, 6,
            "3 x 3 box, small case: every tile and a ragged edge"),
        _mk("j2d9pt_2048x2048_f64_T10000", 2048, 2048, 10000, "f64", "dirichlet", 0.0, 7,
            "3 x 3 box, two big tiles (its register tiles are smaller than j2d5pt's)"),
        _mk("j2d9pt_8192x8192_f64_T1000", 8192, 8192, 1000, "f64", "dirichlet", 1.0, 8,
            "3 x 3 box, larger than on-chip memory: tile-serial sweep"),
        _mk("j2d9pt_8192x8192_f32_T1000", 8192, 8192, 1000, "f32", "dirichlet", 1.0, 8,
            "3 x 3 box, FP32 (same input as the FP64 run): tile-serial sweep"),
    ]
}


@dataclass
class Workload3:
    """A named j3d7pt configuration (3-D grid, seven coefficients, step count)."""
    name: str
    depth: int
    rows: int
    cols: int
    T: int
    dtype: str
    coeffs: tuple
    halo: float
    seed: int
    note: str = ""
    pts: int = 7

    @property
    def cell_updates(self) -> int:
        return self.depth * self.rows * self.cols * self.T

    def grid(self, pitch: int | None = None, dtype=np.float64) -> np.ndarray:
        """The FP64 initial grid (the weights are drawn first from the same generator)."""
        rng = np.random.default_rng(self.seed)
        rng.dirichlet(np.ones(7))
        return uniform_grid3(self.depth, self.rows, self.cols, rng, self.halo, pitch, dtype)


def _mk3(name, depth, rows, cols, T, dtype, halo, seed, note=""):
    return Workload3(name, depth, rows, cols, T, dtype, weights7(seed), halo, seed, note)


WORKLOADS3 = {
    w.name: w for w in [
        _mk3("j3d7pt_256x256x256_f64_T30", 256, 256, 256, 30, "f64", 0.5, 9,
             "3-D seven-point, 128 MiB: several z-blocks per column"),
        _mk3("j3d7pt_512x512x512_f64_T60", 512, 512, 512, 60, "f64", 0.0, 10,
             "3-D seven-point, 1 GiB FP64: far larger than the chip"),
        _mk3("j3d7pt_512x512x512_f32_T60", 512, 512, 512, 60, "f32", 0.0, 10,
             "3-D seven-point, FP32 (same input as the FP64 run)"),
    ]
}


def workload(name: str):
    if name in WORKLOADS3:
        return WORKLOADS3[name]
    return WORKLOADS[name]


@dataclass
class BatchProblem:
    index: int
    side: int
    T: int
    dtype: str
    coeffs: tuple
    field_seed: np.random.SeedSequence = field(repr=False)
    halo: float = 0.0

    @property
    def cell_updates(self) -> int:
        return self.side * self.side * self.T

    def grid(self, pitch: int | None = None) -> np.ndarray:
        return uniform_grid(self.side, self.side, np.random.default_rng(self.field_seed),
                            self.halo, pitch, np.float64)


def batched_set(seed: int = 5, count: int = 64, lo: int = 128, hi: int = 3072,
                t_lo: int = 100, t_hi: int = 2000) -> list:
    """The batched workload: ``count`` square grids of uneven sizes and step counts."""
    rng = np.random.default_rng(seed)
    sides = np.clip(np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))), lo, hi).astype(int)
    steps = rng.integers(t_lo, t_hi + 1, size=count)
    weights = [dirichlet_weights(rng) for _ in range(count)]
    children = np.random.SeedSequence(seed).spawn(count)
    return [BatchProblem(k, int(sides[k]), int(steps[k]), "f64" if k % 2 == 0 else "f32",
                         weights[k], children[k]) for k in range(count)]
