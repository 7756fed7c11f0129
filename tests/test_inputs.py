"""The seeded input generators: reproducible bytes, valid weights, workload shapes."""
import numpy as np

from paper_2306_03336_amd import inputs


def test_uniform_grid_reproducible_and_laid_out():
    a = inputs.uniform_grid(30, 17, 3, halo=1.0, pitch=24)
    b = inputs.uniform_grid(30, 17, 3, halo=1.0, pitch=24)
    assert a.tobytes() == b.tobytes()
    assert a.shape == (32, 24)
    assert np.all(a[0, :19] == 1.0) and np.all(a[31, :19] == 1.0)
    assert np.all(a[:, 0] == 1.0) and np.all(a[:, 18] == 1.0)
    assert np.all(a[:, 19:] == 0.0)
    inner = a[1:31, 1:18]
    assert inner.min() >= 0.0 and inner.max() < 1.0
    assert not np.array_equal(inner, inputs.uniform_grid(30, 17, 4)[1:31, 1:18])


def test_dirichlet_weights():
    for seed in range(20):
        w = inputs.dirichlet_weights(seed)
        assert len(w) == 5 and min(w) >= 0.0
        assert abs(sum(w) - 1.0) <= 4 * np.finfo(np.float64).eps


def test_named_workloads():
    w = inputs.workload("j2d5pt_256x256_f64_T16")
    assert (w.rows, w.cols, w.T, w.coeffs, w.halo) == (256, 256, 16, inputs.EQUAL_WEIGHTS, 0.0)
    w2 = inputs.workload("j2d5pt_2048x2048_f64_T10000")
    assert w2.weights == "dirichlet" and abs(sum(w2.coeffs) - 1) < 1e-15
    assert inputs.workload("j2d5pt_8192x8192_f64_T1000").halo == 1.0
    g = w.grid()
    assert g.shape == (258, 258) and g.dtype == np.float64
    assert np.array_equal(g, w.grid())


def test_batched_set_ranges():
    probs = inputs.batched_set(5)
    assert len(probs) == 64
    assert all(128 <= p.side <= 3072 for p in probs)
    assert all(100 <= p.T <= 2000 for p in probs)
    assert [p.dtype for p in probs[:4]] == ["f64", "f32", "f64", "f32"]
    assert all(abs(sum(p.coeffs) - 1) < 1e-15 for p in probs)
    again = inputs.batched_set(5)
    assert [(p.side, p.T, p.coeffs) for p in probs] == [(p.side, p.T, p.coeffs) for p in again]
    small = min(probs, key=lambda p: p.side)
    assert np.array_equal(small.grid(), small.grid())
    total = sum(p.cell_updates for p in probs)
    assert 1e10 < total < 1e12
