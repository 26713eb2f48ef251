"""Cell-averaged demagnetisation tensor of a regular cuboid grid (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper (Sec. 3) states that the demagnetisation field on the regular cuboid
grid is evaluated as an FFT-accelerated convolution but does not print the
kernel.  The kernel used here is the standard one: the demag tensor N(r_i - r_j)
averaged over target cell i and source cell j of uniformly magnetised cuboids,
so that the demag field is

    H_d(r_i) = -Ms * sum_j N(r_i - r_j) m_j .

Definition (one integral, two evaluation methods):

    N_ab(R) = -1/(4 pi V) * Int_{[-d,d]^3} K_ab(R + t) prod_c (d_c - |t_c|) dt,
    K_ab(u) = (3 u_a u_b - delta_ab |u|^2) / |u|^5,

the source/target box convolution written as a tent weight.

* Near field, |R| < R_SW * h (h = largest cell edge): the closed form of
  Newell, Williams & Dunlop (JGR 98, 9551, 1993), i.e. the 27-point second
  difference of their functions f (diagonal) and g (off-diagonal).  It is
  evaluated here in x87 extended precision (64-bit mantissa) to tame its
  cancellation, which grows like (R/h)^6.
* Far field, |R| >= R_SW * h: Gauss-Legendre quadrature of the tent-weighted
  integral above, splitting every axis at t = 0 (where the tent has its kink),
  with the order chosen by distance (6 points per half-axis below 16 h, 4 below
  40 h, 3 beyond; relative error below 1e-11 in all three bands).  The integrand is smooth there, so the rule converges
  geometrically.

Reading (the paper is silent on the kernel): the near/far split and the
quadrature far field are this implementation's choice; they replace the
usual point-dipole far field, which is only accurate to O((h/R)^4).

Symmetry: N_aa is even in each of X, Y, Z; N_xy is odd in X and Y, even in Z;
N_xz is odd in X and Z; N_yz is odd in Y and Z.  The tensor is therefore
computed on the non-negative octant of offsets and mirrored.

Component order everywhere: (xx, yy, zz, xy, xz, yz).
"""

import numpy as np
from numpy.polynomial.legendre import leggauss

R_SW = 6.0          # Newell closed form strictly below R_SW * h
QUAD_R6 = 16.0      # 6-point (per half-axis) rule strictly below this many h
QUAD_R4 = 40.0      # 4-point rule strictly below this many h, 3-point beyond

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")


# ---------------------------------------------------------------------------
# Newell closed form (near field)
# ---------------------------------------------------------------------------

def _as_ld(x, y, z):
    """Broadcast to writable 1-D-or-more extended-precision arrays."""
    arrs = np.broadcast_arrays(*(np.atleast_1d(np.asarray(a, dtype=np.longdouble))
                                 for a in (x, y, z)))
    return tuple(np.array(a) for a in arrs)


def newell_f(x, y, z):
    """Newell's auxiliary function f(x, y, z) for the diagonal entries.

    f is even in each argument; it is evaluated on |x|, |y|, |z|.  A term
    whose argument has a vanishing denominator carries a vanishing prefactor
    and is dropped.
    """
    x, y, z = _as_ld(x, y, z)
    x, y, z = np.abs(x), np.abs(y), np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = (2 * x2 - y2 - z2) * R / 6
    rxz = np.sqrt(x2 + z2)
    m = rxz > 0
    out[m] += y[m] / 2 * (z2[m] - x2[m]) * np.arcsinh(y[m] / rxz[m])
    rxy = np.sqrt(x2 + y2)
    m = rxy > 0
    out[m] += z[m] / 2 * (y2[m] - x2[m]) * np.arcsinh(z[m] / rxy[m])
    m = (x * R) > 0
    out[m] -= x[m] * y[m] * z[m] * np.arctan(y[m] * z[m] / (x[m] * R[m]))
    return out


def newell_g(x, y, z):
    """Newell's auxiliary function g(x, y, z) for the off-diagonal entry xy.

    g is odd in x and in y and even in z: it is evaluated on absolute values
    and multiplied by sign(x) sign(y).
    """
    x, y, z = _as_ld(x, y, z)
    sgn = np.sign(x) * np.sign(y)
    x, y, z = np.abs(x), np.abs(y), np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = -x * y * R / 3
    rxy = np.sqrt(x2 + y2)
    m = rxy > 0
    out[m] += x[m] * y[m] * z[m] * np.arcsinh(z[m] / rxy[m])
    ryz = np.sqrt(y2 + z2)
    m = ryz > 0
    out[m] += y[m] / 6 * (3 * z2[m] - y2[m]) * np.arcsinh(x[m] / ryz[m])
    rxz = np.sqrt(x2 + z2)
    m = rxz > 0
    out[m] += x[m] / 6 * (3 * z2[m] - x2[m]) * np.arcsinh(y[m] / rxz[m])
    m = (z * R) > 0
    out[m] -= z[m] ** 3 / 6 * np.arctan(x[m] * y[m] / (z[m] * R[m]))
    m = (y * R) > 0
    out[m] -= z[m] * y2[m] / 2 * np.arctan(x[m] * z[m] / (y[m] * R[m]))
    m = (x * R) > 0
    out[m] -= z[m] * x2[m] / 2 * np.arctan(y[m] * z[m] / (x[m] * R[m]))
    return sgn * out


def _second_difference(fun, X, Y, Z, dx, dy, dz):
    """27-point stencil: sum over eps in {-1,0,1}^3 of c(ex)c(ey)c(ez) fun(...),
    with c(0) = 2 and c(+-1) = -1, divided by 4 pi dx dy dz."""
    acc = np.zeros(np.broadcast(X, Y, Z).shape, dtype=np.longdouble)
    c = {-1: -1, 0: 2, 1: -1}
    for ex in (-1, 0, 1):
        for ey in (-1, 0, 1):
            for ez in (-1, 0, 1):
                w = c[ex] * c[ey] * c[ez]
                acc += w * fun(X + ex * dx, Y + ey * dy, Z + ez * dz)
    return acc / (4 * np.pi * np.longdouble(dx) * np.longdouble(dy) * np.longdouble(dz))


def newell_tensor(X, Y, Z, dx, dy, dz):
    """Closed-form Newell tensor at physical offsets (X, Y, Z).

    Returns an array [6, ...] in component order (xx, yy, zz, xy, xz, yz),
    float64 (computed in extended precision).  Diagonal entries use f with the
    axes permuted, off-diagonal ones use g with the axes permuted.
    """
    L = np.longdouble
    X, Y, Z = _as_ld(X, Y, Z)
    dx, dy, dz = L(dx), L(dy), L(dz)
    f, g = newell_f, newell_g
    sd = _second_difference
    nxx = sd(lambda a, b, c: f(a, b, c), X, Y, Z, dx, dy, dz)
    nyy = sd(lambda a, b, c: f(b, a, c), X, Y, Z, dx, dy, dz)
    nzz = sd(lambda a, b, c: f(c, b, a), X, Y, Z, dx, dy, dz)
    nxy = sd(lambda a, b, c: g(a, b, c), X, Y, Z, dx, dy, dz)
    nxz = sd(lambda a, b, c: g(a, c, b), X, Y, Z, dx, dy, dz)
    nyz = sd(lambda a, b, c: g(b, c, a), X, Y, Z, dx, dy, dz)
    return np.stack([nxx, nyy, nzz, nxy, nxz, nyz]).astype(np.float64)


# ---------------------------------------------------------------------------
# Quadrature of the same integral (far field)
# ---------------------------------------------------------------------------

def _half_axis_rule(n, d):
    """Nodes and tent-weighted weights on [-d, 0] U [0, d] for one axis."""
    xi, w = leggauss(n)
    t_pos = 0.5 * d * (xi + 1.0)
    w_pos = 0.5 * d * w
    t = np.concatenate([-t_pos, t_pos])
    ww = np.concatenate([w_pos, w_pos]) * (d - np.abs(t))
    return t, ww


def quadrature_tensor(X, Y, Z, dx, dy, dz, n):
    """Tent-weighted Gauss-Legendre quadrature of N(R) with n points per
    half-axis (2n per axis).  X, Y, Z are 1-D arrays of equal length."""
    X = np.atleast_1d(np.asarray(X, dtype=np.float64))
    Y = np.atleast_1d(np.asarray(Y, dtype=np.float64))
    Z = np.atleast_1d(np.asarray(Z, dtype=np.float64))
    tx, wx = _half_axis_rule(n, dx)
    ty, wy = _half_axis_rule(n, dy)
    tz, wz = _half_axis_rule(n, dz)
    out = np.zeros((6, X.size))
    V = dx * dy * dz
    for a in range(tx.size):
        ux = X + tx[a]
        for b in range(ty.size):
            uy = Y + ty[b]
            for c in range(tz.size):
                uz = Z + tz[c]
                w = wx[a] * wy[b] * wz[c]
                r2 = ux * ux + uy * uy + uz * uz
                inv5 = 1.0 / (r2 * r2 * np.sqrt(r2))
                out[0] += w * (3 * ux * ux - r2) * inv5
                out[1] += w * (3 * uy * uy - r2) * inv5
                out[2] += w * (3 * uz * uz - r2) * inv5
                out[3] += w * (3 * ux * uy) * inv5
                out[4] += w * (3 * ux * uz) * inv5
                out[5] += w * (3 * uy * uz) * inv5
    return -out / (4 * np.pi * V)


def point_dipole_tensor(X, Y, Z, dx, dy, dz):
    """Point-dipole limit -(V/4 pi)(3 R R^T - R^2 I)/R^5 (far-field check)."""
    X, Y, Z = (np.asarray(a, dtype=np.float64) for a in (X, Y, Z))
    V = dx * dy * dz
    r2 = X * X + Y * Y + Z * Z
    inv5 = 1.0 / (r2 * r2 * np.sqrt(r2))
    k = -V / (4 * np.pi) * inv5
    return np.stack([k * (3 * X * X - r2), k * (3 * Y * Y - r2), k * (3 * Z * Z - r2),
                     k * 3 * X * Y, k * 3 * X * Z, k * 3 * Y * Z])


# ---------------------------------------------------------------------------
# Tensor on all offsets of a grid
# ---------------------------------------------------------------------------

def octant_tensor(nx, ny, nz, dx, dy, dz):
    """N at offsets (i dx, j dy, k dz), 0 <= i < nx, 0 <= j < ny, 0 <= k < nz.

    Returns float64 [6, nz, ny, nx].  Near field: Newell closed form; far
    field: quadrature (see module docstring).
    """
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = (i * dx).ravel()
    Y = (j * dy).ravel()
    Z = (k * dz).ravel()
    h = max(dx, dy, dz)
    r2 = X * X + Y * Y + Z * Z
    out = np.zeros((6, X.size))
    near = r2 < (R_SW * h) ** 2
    if near.any():
        out[:, near] = newell_tensor(X[near], Y[near], Z[near], dx, dy, dz)
    far = ~near
    for n, lo, hi in ((6, R_SW, QUAD_R6), (4, QUAD_R6, QUAD_R4), (3, QUAD_R4, np.inf)):
        sel = far & (r2 >= (lo * h) ** 2) & (r2 < (hi * h) ** 2)
        if sel.any():
            out[:, sel] = quadrature_tensor(X[sel], Y[sel], Z[sel], dx, dy, dz, n)
    return out.reshape(6, nz, ny, nx)


# parity of each component in (X, Y, Z): +1 even, -1 odd
PARITY = np.array([
    [1, 1, 1],     # xx
    [1, 1, 1],     # yy
    [1, 1, 1],     # zz
    [-1, -1, 1],   # xy
    [-1, 1, -1],   # xz
    [1, -1, -1],   # yz
])


def full_tensor(nx, ny, nz, dx, dy, dz):
    """N on all offsets -(n-1)..(n-1) per axis.

    Returns float64 [6, 2nz-1, 2ny-1, 2nx-1]; index (k, j, i) holds the offset
    (i-(nx-1), j-(ny-1), k-(nz-1)) in cells.
    """
    octo = octant_tensor(nx, ny, nz, dx, dy, dz)
    out = np.zeros((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
    ii = np.arange(-(nx - 1), nx)
    jj = np.arange(-(ny - 1), ny)
    kk = np.arange(-(nz - 1), nz)
    for c in range(6):
        px, py, pz = PARITY[c]
        sx = np.where(ii < 0, px, 1)
        sy = np.where(jj < 0, py, 1)
        sz = np.where(kk < 0, pz, 1)
        block = octo[c][np.abs(kk)][:, np.abs(jj)][:, :, np.abs(ii)]
        out[c] = block * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return out


def tensor_matrix(N6):
    """3x3 symmetric matrix view of a [6, ...] tensor array: [3, 3, ...]."""
    xx, yy, zz, xy, xz, yz = N6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])
