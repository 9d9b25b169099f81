"""Host checks of the accuracy figures (paper_2012_04011_amd/accuracy.py)."""

import math

import numpy as np

from paper_2012_04011_amd import accuracy as A
from paper_2012_04011_amd import workloads as W


def _nodes(g, d):
    n, lo, hi = g["n"][d], g["lo"][d], g["hi"][d]
    per = (g["periodic_mask"] >> d) & 1
    return lo + np.arange(n) * ((hi - lo) / (n if per else n - 1))


def test_multilinear_sampling_is_exact_on_multilinear_functions():
    """Multilinear interpolation reproduces any function that is affine in
    each of x, y, v separately (products included); on theta the coarse
    nodes of a 2x-coarsened periodic axis are fine nodes, so any function of
    theta is copied."""
    fine, coarse = W.car_grid(23, 19, 11, 16), W.car_grid(9, 7, 5, 8)
    x, y, v, th = (_nodes(fine, d) for d in range(4))
    X, Y, Vv, TH = x[:, None, None, None], y[None, :, None, None], v[None, None, :, None], th[None, None, None, :]
    f = lambda X, Y, Vv, TH: 0.3 + 0.7 * X - 0.2 * Y + 1.1 * Vv + 0.05 * X * Y * Vv + np.sin(3 * TH) * (1 + X)
    Vf = f(X, Y, Vv, TH)
    xc, yc, vc, thc = (_nodes(coarse, d) for d in range(4))
    exact = f(xc[:, None, None, None], yc[None, :, None, None], vc[None, None, :, None], thc[None, None, None, :])
    S = A.sample_multilinear(Vf, fine, coarse)
    assert S.shape == tuple(coarse["n"])
    np.testing.assert_allclose(S, exact, rtol=0, atol=1e-12)


def test_multilinear_sampling_between_periodic_nodes():
    """Half-way between theta nodes the value is the mean of the two, also
    across the wrap from the last node to the first."""
    fine = {"n": (3, 3, 3, 4), "lo": (0, 0, 0, 0.0), "hi": (2, 2, 2, 4.0), "periodic_mask": 8}
    at = {"n": (3, 3, 3, 4), "lo": (0, 0, 0, 0.5), "hi": (2, 2, 2, 4.5), "periodic_mask": 8}
    V = np.broadcast_to(np.array([1.0, 2.0, 4.0, 8.0]), (3, 3, 3, 4)).copy()
    S = A.sample_multilinear(V, fine, at)
    np.testing.assert_allclose(S[0, 0, 0], [1.5, 3.0, 6.0, 4.5], rtol=0, atol=1e-15)


def test_precision_metrics_counts():
    g = W.car_grid(5, 5, 3, 4)
    tol = 1e-4 * 10.0 / 4
    ref = np.full(g["n"], 2.0)
    ref[0, 0, 0, 0] = 0.5       # in the band
    ref[1, 0, 0, 0] = -0.5 * tol  # next to the zero level set
    ref[2, 0, 0, 0] = 0.3
    V = ref.copy()
    V[0, 0, 0, 0] += 3 * tol     # band error
    V[1, 0, 0, 0] = 0.25 * tol   # flip within tol of the zero set
    V[2, 0, 0, 0] = -0.1         # flip far from it
    m = A.precision_metrics(V, ref, g)
    assert math.isclose(m["tol"], tol)
    assert m["flips"] == 2 and m["flips_outside"] == 1
    assert math.isclose(m["max_band"], 0.4) and math.isclose(m["max_all"], 0.4)
    c = A.consistency_metrics(V, g, ref, g)
    assert c["flips"] == 2 and c["flips_beyond_2dx"] == 0 and math.isclose(c["max_all"], 0.4)
