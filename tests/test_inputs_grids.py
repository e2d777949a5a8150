"""The paper's two grid families (Section 5), as generated for the tests and
the benchmark: point counts against the M columns of Tables 5.1 and 5.3, and
the geometry of the polar grid."""
import numpy as np
import pytest

from nudft_inputs import make_grid_problem, polar_points

# Table 5.3 (polar grid, beta = 0.6): M for n = 32 .. 512
POLAR_M = {32: 2397, 64: 11620, 128: 54373, 256: 249074, 512: 1122019}
# Table 5.1 (random grid): M = 1.5 N
RANDOM_M = {32: 1536, 64: 6144, 128: 24576, 256: 98304, 512: 393216}


@pytest.mark.parametrize("n", sorted(POLAR_M))
def test_polar_point_count_matches_table(n):
    assert polar_points(n, 0.6).shape == (POLAR_M[n], 2)


@pytest.mark.parametrize("n", sorted(RANDOM_M))
def test_random_point_count_matches_table(n):
    pr = make_grid_problem("random", n, 1)
    assert pr.M == RANDOM_M[n]
    assert np.all((pr.points >= 0) & (pr.points < 1))


def test_polar_geometry():
    n = 64
    pts = polar_points(n, 0.6)
    assert np.all((pts >= 0) & (pts < 1))
    assert tuple(pts[0]) == (0.5, 0.5)
    d = pts[1:] - 0.5
    r = np.hypot(d[:, 0], d[:, 1])
    # every radius is (sqrt 2 / 2) p / n for an integer p in 1..n-1
    p = r / (np.sqrt(2) / 2) * n
    assert np.allclose(p, np.round(p), atol=1e-9)
    assert p.min() > 0.5 and p.max() < n - 0.5
    # the rings inside the inscribed circle (r < 1/2) are complete: n_t points
    nt = int(np.ceil(0.6 * n * np.log2(n)))
    full = np.round(p[r < 0.5 - 1e-12]).astype(int)
    counts = np.bincount(full)
    assert set(counts[counts > 0]) == {nt}
    # angles of ring 1 are q / n_t turns
    ring = d[np.round(p).astype(int) == 1]
    t = np.sort(np.mod(np.arctan2(ring[:, 1], ring[:, 0]) / (2 * np.pi), 1.0))
    assert np.allclose(t, np.arange(nt) / nt, atol=1e-12)


def test_grid_problems_are_seeded():
    a = make_grid_problem("random", 32, 5)
    b = make_grid_problem("random", 32, 5)
    assert np.array_equal(a.points, b.points) and np.array_equal(a.c_true, b.c_true)
    c = make_grid_problem("polar", 32, 5)
    assert np.array_equal(c.points, polar_points(32, 0.6))
