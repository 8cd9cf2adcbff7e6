"""Pins of the periodic 2D grid transfers of the FAS oracle (``oracle.fas``:
``restrict``, ``prolong``).  The paper defers its transfers to earlier work
(Sec. 6, "standard" FAS); the reading is nodal nesting (coarse node I on fine
node 2I, the nesting of the Cauchy error of Sec. 6.1), 9-point full weighting
and bilinear interpolation.  These pins hold for that reading and fail for a
wrong weight, a wrong offset of the nesting or a wrong periodic wrap:

* the Fourier symbol of full weighting (a closed form of the separable
  stencil (1/4)[1 2 1] in each direction), on modes with a random phase, so
  that a shifted nesting fails;
* single-node impulses, interior and across the periodic seam, against the
  stencil values by hand;
* bilinear interpolation reproduces bilinear fields exactly away from the seam
  and copies the coarse values onto the fine nodes 2I;
* full weighting is one quarter of the transpose of bilinear interpolation
  (the variational pair in 2D), as matrices built column by column.
"""
import numpy as np
import pytest

from oracle.fas import prolong, restrict


@pytest.mark.parametrize("n", [8, 16, 32])
def test_full_weighting_fourier_symbol(n):
    """R cos(a i + b j + phi) at coarse node (I, J) equals
    ((1 + cos a)/2)((1 + cos b)/2) cos(2 a I + 2 b J + phi)."""
    rng = np.random.default_rng(n)
    j, i = np.mgrid[0:n, 0:n]
    J, I = np.mgrid[0:n // 2, 0:n // 2]
    for p, q in [(1, 0), (0, 1), (1, 2), (3, 1), (n // 2 - 1, 2), (n // 4, n // 4)]:
        a, b = 2 * np.pi * p / n, 2 * np.pi * q / n
        phi = rng.uniform(0, 2 * np.pi)
        f = np.cos(a * i + b * j + phi)
        want = 0.25 * (1 + np.cos(a)) * (1 + np.cos(b)) * np.cos(2 * a * I + 2 * b * J + phi)
        assert np.abs(restrict(f) - want).max() < 1e-14


def test_full_weighting_impulses_by_hand():
    """A unit value at one fine node reaches the coarse nodes with the weights
    4/16 (same node), 2/16 (edge neighbour) and 1/16 (corner neighbour),
    including across the periodic seam."""
    n = 8
    cases = [
        ((2, 2), {(1, 1): 4 / 16}),                                  # on coarse node (1, 1)
        ((2, 3), {(1, 1): 2 / 16, (1, 2): 2 / 16}),                   # between two in x
        ((3, 2), {(1, 1): 2 / 16, (2, 1): 2 / 16}),                   # between two in y
        ((3, 3), {(1, 1): 1 / 16, (1, 2): 1 / 16, (2, 1): 1 / 16, (2, 2): 1 / 16}),
        ((0, 7), {(0, 3): 2 / 16, (0, 0): 2 / 16}),                   # x seam
        ((7, 7), {(3, 3): 1 / 16, (3, 0): 1 / 16, (0, 3): 1 / 16, (0, 0): 1 / 16}),  # corner seam
    ]
    for (fj, fi), want in cases:
        f = np.zeros((n, n))
        f[fj, fi] = 1.0
        c = restrict(f)
        exp = np.zeros((n // 2, n // 2))
        for (cj, ci), w in want.items():
            exp[cj, ci] = w
        assert np.array_equal(c, exp), (fj, fi)


def test_full_weighting_constants_and_mean():
    """Constants are kept, and so is the grid mean: every fine node hands a total
    weight of 4/16 to the coarse nodes, and there is one coarse node per four
    fine nodes."""
    rng = np.random.default_rng(3)
    assert np.array_equal(restrict(np.full((16, 16), 2.5)), np.full((8, 8), 2.5))
    f = rng.standard_normal((16, 16))
    assert abs(restrict(f).mean() - f.mean()) < 1e-15


def test_bilinear_interpolation_exact_on_bilinear_fields():
    """P of the coarse samples of a + b x + c y + d x y equals the field at every
    fine node whose interpolation stencil does not cross the seam, and the fine
    nodes 2I carry the coarse values unchanged."""
    n = 16
    rng = np.random.default_rng(5)
    a, b, c, d = rng.standard_normal(4)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    f = a + b * x + c * y + d * x * y
    cf = f[::2, ::2].copy()
    p = prolong(cf)
    assert np.array_equal(p[::2, ::2], cf)
    inner = np.s_[: n - 1, : n - 1]   # the last fine row / column interpolates across the seam
    assert np.abs(p[inner] - f[inner]).max() < 1e-12


def test_bilinear_interpolation_by_hand_at_the_seam():
    """A unit coarse value spreads to its fine node (1), the four edge
    midpoints (1/2) and the four cell centres (1/4), wrapping periodically."""
    c = np.zeros((4, 4))
    c[0, 0] = 1.0
    p = prolong(c)
    want = np.zeros((8, 8))
    want[0, 0] = 1.0
    for j, i in [(0, 1), (0, 7), (1, 0), (7, 0)]:
        want[j, i] = 0.5
    for j, i in [(1, 1), (1, 7), (7, 1), (7, 7)]:
        want[j, i] = 0.25
    assert np.array_equal(p, want)


@pytest.mark.parametrize("n", [8, 16])
def test_full_weighting_is_quarter_transpose_of_bilinear(n):
    """As matrices (built from unit vectors), R = P^T / 4."""
    m = n // 2
    P = np.zeros((n * n, m * m))
    for k in range(m * m):
        e = np.zeros(m * m)
        e[k] = 1.0
        P[:, k] = prolong(e.reshape(m, m)).ravel()
    R = np.zeros((m * m, n * n))
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        R[:, k] = restrict(e.reshape(n, n)).ravel()
    assert np.array_equal(R, P.T / 4.0)


def test_transfers_act_on_leading_axes_independently():
    """Stacks of fields (the unknown vector g, shape (c, n, n)) are transferred
    component by component."""
    rng = np.random.default_rng(9)
    g = rng.standard_normal((5, 16, 16))
    assert np.array_equal(restrict(g), np.stack([restrict(x) for x in g]))
    gc = rng.standard_normal((5, 8, 8))
    assert np.array_equal(prolong(gc), np.stack([prolong(x) for x in gc]))
