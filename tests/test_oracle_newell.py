"""Pins of the oracle's demag tensor against facts fixed outside the oracle.

Each pin uses mathematics independent of the oracle's own formulas:
* the trace identity N_xx + N_yy + N_zz = 1 of a cuboid's self term;
* Aharoni's closed-form demagnetising factor of a rectangular prism
  (J. Appl. Phys. 83, 3432 (1998)), a formula unrelated to Newell's f;
* a brute-force 6-D Gauss-Legendre average of the point-dipole kernel over the
  source and the target cell (no tent reduction), valid for separated cells;
* the point-dipole limit far away;
* prism consistency: a uniformly magnetised block of cells must see, on
  average, the self demag factor of one big cell of the same shape.
"""

import numpy as np
import pytest

from oracle import newell, fields


def aharoni_Dz(a, b, c):
    """Aharoni's demagnetising factor along z of a 2a x 2b x 2c prism."""
    r = np.sqrt(a * a + b * b + c * c)
    ab = np.sqrt(a * a + b * b)
    bc = np.sqrt(b * b + c * c)
    ac = np.sqrt(a * a + c * c)
    s = ((b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
         + b / (2 * c) * np.log((ab + a) / (ab - a))
         + a / (2 * c) * np.log((ab + b) / (ab - b))
         + c / (2 * a) * np.log((bc - b) / (bc + b))
         + c / (2 * b) * np.log((ac - a) / (ac + a))
         + 2 * np.arctan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return s / np.pi


def aharoni_factors(Lx, Ly, Lz):
    """(Dx, Dy, Dz) of an Lx x Ly x Lz prism by axis permutation."""
    return (aharoni_Dz(Ly / 2, Lz / 2, Lx / 2), aharoni_Dz(Lz / 2, Lx / 2, Ly / 2),
            aharoni_Dz(Lx / 2, Ly / 2, Lz / 2))


def box_average_dipole(R, d, npts=8):
    """-(1/(4 pi V)) Int_target Int_source K(r_t - r_s): plain 6-D
    Gauss-Legendre over both boxes; needs well-separated cells."""
    xi, w = np.polynomial.legendre.leggauss(npts)
    out = np.zeros(6)
    pts = [0.5 * dd * xi for dd in d]
    ws = [0.5 * dd * w for dd in d]
    # difference of two independent box points, axis by axis
    diffs, wdiff = [], []
    for a in range(3):
        t = (pts[a][:, None] - pts[a][None, :]).ravel()
        ww = (ws[a][:, None] * ws[a][None, :]).ravel()
        diffs.append(t)
        wdiff.append(ww)
    ux = R[0] + diffs[0][:, None, None]
    uy = R[1] + diffs[1][None, :, None]
    uz = R[2] + diffs[2][None, None, :]
    W = wdiff[0][:, None, None] * wdiff[1][None, :, None] * wdiff[2][None, None, :]
    r2 = ux * ux + uy * uy + uz * uz
    inv5 = 1.0 / (r2 * r2 * np.sqrt(r2))
    V = d[0] * d[1] * d[2]
    comps = [3 * ux * ux - r2, 3 * uy * uy - r2, 3 * uz * uz - r2, 3 * ux * uy, 3 * ux * uz,
             3 * uy * uz]
    for c in range(6):
        out[c] = np.sum(W * comps[c] * inv5)
    return -out / (4 * np.pi * V)


@pytest.mark.parametrize("d", [(1.0, 1.0, 1.0), (2.0, 1.0, 0.3), (5e-9, 5e-9, 5e-9),
                               (1.0, 1.0, 10.0), (3.0, 7.0, 2.0)])
def test_self_term_trace_is_one(d):
    N = newell.newell_tensor(0.0, 0.0, 0.0, *d)[:, 0]
    assert abs(N[0] + N[1] + N[2] - 1.0) < 1e-13
    assert np.all(np.abs(N[3:]) < 1e-15)


def test_cube_self_term_one_third():
    N = newell.newell_tensor(0.0, 0.0, 0.0, 2e-9, 2e-9, 2e-9)[:, 0]
    assert np.allclose(N[:3], 1.0 / 3.0, atol=1e-14)


@pytest.mark.parametrize("d", [(2.0, 1.0, 0.3), (5.0, 3.0, 1.0), (1.0, 1.0, 10.0),
                               (1.0, 4.0, 2.5)])
def test_self_term_matches_aharoni(d):
    N = newell.newell_tensor(0.0, 0.0, 0.0, *d)[:, 0]
    D = aharoni_factors(*d)
    assert np.allclose(N[:3], D, rtol=0, atol=1e-12)


@pytest.mark.parametrize("cells,d", [((2, 1, 0), (1.0, 1.0, 1.0)),
                                     ((3, -2, 1), (1.0, 1.0, 1.0)),
                                     ((-2, 3, -2), (1.0, 1.3, 0.8)),
                                     ((4, 1, -3), (1.0, 1.0, 1.0)),
                                     ((0, 3, 0), (2.0, 1.0, 1.0))])
def test_newell_matches_box_average_near(cells, d):
    """Newell closed form (near band) against brute-force box averaging."""
    R = np.array(cells, dtype=float) * np.array(d)
    N = newell.newell_tensor(*R, *d)[:, 0]
    Q = box_average_dipole(R, d, npts=10)
    assert np.max(np.abs(N - Q)) < 1e-7 * np.max(np.abs(Q))


@pytest.mark.parametrize("cells", [(7, 2, 1), (-12, 5, 0), (20, -9, 3), (45, 10, -1)])
def test_octant_far_band_matches_box_average(cells):
    """The oracle's far-field quadrature (tent form) against the 6-D rule."""
    d = (5e-9, 5e-9, 5e-9)
    c = np.abs(np.array(cells))
    octo = newell.octant_tensor(c[0] + 1, c[1] + 1, c[2] + 1, *d)[:, c[2], c[1], c[0]]
    sgn = np.sign(cells)
    sgn[sgn == 0] = 1
    par = np.prod(np.where(newell.PARITY < 0, sgn[None, :], 1), axis=1)
    R = np.array(cells, dtype=float) * np.array(d)
    Q = box_average_dipole(R, d, npts=6)
    assert np.max(np.abs(octo * par - Q)) < 1e-9 * np.max(np.abs(Q))


def test_far_field_tends_to_point_dipole():
    d = (5e-9, 5e-9, 5e-9)
    X, Y, Z = 150 * d[0], 60 * d[1], 20 * d[2]
    N = newell.quadrature_tensor(X, Y, Z, *d, 3)[:, 0]
    P = newell.point_dipole_tensor(X, Y, Z, *d)
    assert np.max(np.abs(N - P)) < 1e-7 * np.max(np.abs(P))


def test_near_far_continuity_at_switch():
    """Just inside and just outside the switch radius both methods describe
    the same integral."""
    d = (1.0, 1.0, 1.0)
    R = (5.0, 3.0, 1.0)   # |R| = 5.9 < 6: Newell band
    a = newell.newell_tensor(*R, *d)[:, 0]
    b = newell.quadrature_tensor(*R, *d, 6)[:, 0]
    assert np.max(np.abs(a - b)) < 1e-10 * np.max(np.abs(a))


def test_full_tensor_symmetries():
    T = newell.full_tensor(5, 4, 3, 1.0, 1.2, 0.7)
    flipped = T[:, ::-1, ::-1, ::-1]
    for c in range(6):
        sign = np.prod(newell.PARITY[c])
        assert np.allclose(flipped[c], sign * T[c], atol=1e-16)


@pytest.mark.parametrize("shape,mode", [((4, 2, 1), "direct"), ((3, 3, 3), "direct"),
                                        ((24, 12, 2), "fft"), ((64, 20, 2), "fft")])
def test_prism_consistency_uniform_block(shape, mode):
    """Mean demag field of a uniformly magnetised block equals -Ms D m with D
    the Aharoni factor of the whole block (exercises near and far bands)."""
    d = (5e-9, 5e-9, 5e-9)
    nx, ny, nz = shape
    P = fields.Problem(nx, ny, nz, *d, Ms=8e5, A=0.0, demag=mode)
    D = aharoni_factors(nx * d[0], ny * d[1], nz * d[2])
    for axis in range(3):
        m = np.zeros((3, nz, ny, nx))
        m[axis] = 1.0
        H = P.h_demag(m)
        mean = H.reshape(3, -1).mean(axis=1) / (-8e5)
        expect = np.zeros(3)
        expect[axis] = D[axis]
        assert np.max(np.abs(mean - expect)) < 2e-11, (axis, mean, expect)


def test_uniform_cube_one_third():
    for n in (2, 3):
        P = fields.Problem(n, n, n, 2e-9, 2e-9, 2e-9, Ms=1e6, A=0.0, demag="direct")
        m = np.zeros((3, n, n, n))
        m[2] = 1.0
        H = P.h_demag(m)
        assert abs(H[2].mean() / -1e6 - 1.0 / 3.0) < 1e-13
