"""Post-processing of the resolution study (Sec. 3.2, 3.4): the pieces that
need no GPU, checked against closed forms."""

import numpy as np


def _an():
    from paper_2101_11107_amd import analysis
    return analysis


def test_similarity_index_closed_forms():
    """Eq. (11) with the factor 1/2: identical or uniformly scaled fields give
    1 (the speed term is normalized per field), opposite fields 0, orthogonal
    fields of equal normalized speed 1/2, a zero vector cos = 0."""
    an = _an()
    rng = np.random.default_rng(0)
    u = rng.normal(size=(50, 3))
    assert np.allclose(an.similarity_index_points(u, u), 1.0)
    assert np.allclose(an.similarity_index_points(u, 2.5 * u), 1.0)
    assert np.allclose(an.similarity_index_points(u, -u), 0.0)
    a = np.array([[1.0, 0, 0], [0, 2.0, 0]])
    b = np.array([[0, 1.0, 0], [0, 0, 2.0]])
    assert np.allclose(an.similarity_index_points(a, b), 0.5)
    z = np.array([[1.0, 0, 0], [0, 0, 0]])
    w = np.array([[1.0, 0, 0], [0, 1.0, 0]])
    si = an.similarity_index_points(z, w)
    assert np.isclose(si[0], 1.0) and np.isclose(si[1], 0.5 * (1.0 - 1.0))


def test_trilinear_is_exact_for_linear_fields():
    an = _an()
    nz, ny, nx = 7, 6, 9
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    A = np.array([[0.3, -1.2, 0.7], [2.0, 0.1, -0.4], [-0.5, 0.9, 1.1]])
    c = np.array([0.2, -0.3, 0.5])
    dense = np.stack([A[k, 0] * xx + A[k, 1] * yy + A[k, 2] * zz + c[k] for k in range(3)], axis=-1)
    p = np.random.default_rng(1).uniform([0, 0, 0], [nx - 1, ny - 1, nz - 1], size=(200, 3))
    got = an.trilinear(dense, p)
    ref = p @ A.T + c
    assert np.max(np.abs(got - ref)) < 1e-12
    # the nodes themselves
    q = np.array([[3, 2, 4], [0, 0, 0], [nx - 1, ny - 1, nz - 1]], float)
    assert np.allclose(an.trilinear(dense, q), q @ A.T + c)


def test_plane_points_and_periodicity():
    an = _an()
    mask = np.zeros((4, 5, 6), np.uint8)
    mask[1:3, 1:4, 2:5] = 1
    pts = an.plane_points(mask, "x", 3)
    assert len(pts) == 2 * 3 and np.all(pts[:, 0] == 3)
    pts = an.plane_points(mask, "z", 0)
    assert len(pts) == 0
    # a periodic probe signal has no change from cycle to cycle; a decaying
    # start-up transient shows shrinking changes
    t = np.arange(400)
    per = np.zeros((400, 1, 4))
    per[:, 0, 1] = 1.0 + 0.5 * np.sin(2 * np.pi * t / 100)
    assert max(an.periodicity(per, 100)) < 1e-12
    dec = per.copy()
    dec[:, 0, 1] += np.exp(-t / 60.0)
    ch = an.periodicity(dec, 100)
    assert len(ch) == 3 and ch[0] > ch[1] > ch[2] > 0
