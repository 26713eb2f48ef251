"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and lays out field schedules; it holds
none of the method's arithmetic and imports neither the oracle nor the HIP
binding.  Both sides of every parity check receive the arrays made here.

Recipe (the stand-ins for the paper's Standard Problem #1 workload of Sec. 4
and the other synthetic workloads):

* RNG: numpy ``default_rng(14052728 + c)`` (PCG64) for workload c.
* "random unit vectors": N(0,1)^3 per cell drawn in (z, y, x, component)
  order and normalised; returned as structure of arrays [3, nz, ny, nx].
* "uniform + noise": normalise(direction + amp * N(0,1)^3), same draw order.
* fields in mT mean mu0 H, so 1 mT = 1e-3 / mu0 A/m with mu0 = 4 pi 1e-7.
"""

import numpy as np

MU0 = 4e-7 * np.pi
SEED_BASE = 14052728
MT = 1e-3 / MU0            # A/m per mT


def rng_for(workload):
    return np.random.default_rng(SEED_BASE + int(workload))


def random_unit(nx, ny, nz, rng):
    v = rng.standard_normal((nz, ny, nx, 3))
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    return np.ascontiguousarray(np.moveaxis(v, -1, 0))


def uniform_with_noise(direction, nx, ny, nz, amp, rng):
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    v = d[None, None, None, :] + amp * rng.standard_normal((nz, ny, nx, 3))
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    return np.ascontiguousarray(np.moveaxis(v, -1, 0))


def tilted(deg_from_x_toward_y):
    a = np.deg2rad(deg_from_x_toward_y)
    return np.array([np.cos(a), np.sin(a), 0.0])


def loop_fields(h_max_mT, step_mT, direction):
    """Down from +h_max to -h_max, then back up to +h_max (both ends once
    per branch), in A/m, [n, 3]."""
    n = int(round(2 * h_max_mT / step_mT))
    down = h_max_mT - step_mT * np.arange(n + 1)
    up = -h_max_mT + step_mT * np.arange(1, n + 1)
    amp = np.concatenate([down, up]) * MT
    return amp[:, None] * np.asarray(direction, dtype=np.float64)[None, :]


PERMALLOY = dict(Ms=8.0e5, A=1.3e-11, Ku=500.0, u=(1.0, 0.0, 0.0))


def workload(c):
    """Dict describing synthetic workload c (grid, material, m0, fields)."""
    rng = rng_for(c)
    if c == 0:
        nx, ny, nz, d = 32, 16, 1, 5e-9
        m0 = random_unit(nx, ny, nz, rng)
        h = tilted(1.0)
        fields = np.array([0.0, 4, 8, 12, 16, 20])[:, None] * MT * h[None, :]
        return dict(name="film 32x16x1, 5 nm cells, random start, 0..20 mT",
                    n=(nx, ny, nz), d=(d, d, d), m0=m0, fields=fields, tol=1e-6,
                    **PERMALLOY)
    if c == 1:
        nx, ny, nz, d = 400, 200, 4, 5e-9
        m0 = uniform_with_noise((1, 0, 0), nx, ny, nz, 1e-3, rng)
        fields = loop_fields(50.0, 1.0, tilted(1.0))
        return dict(name="SP1-like film 400x200x4, 5 nm cells, +-50 mT loop",
                    n=(nx, ny, nz), d=(d, d, d), m0=m0, fields=fields, tol=1e-6,
                    **PERMALLOY)
    if c == 2:
        nx = ny = nz = 128
        d = 2e-9
        m0 = random_unit(nx, ny, nz, rng)
        a = np.deg2rad(2.0)
        h = np.array([np.sin(a), 0.0, np.cos(a)])
        fields = np.arange(0, 201, 20.0)[:, None] * MT * h[None, :]
        return dict(name="cube 128^3, 2 nm cells, random start, 0..200 mT",
                    n=(nx, ny, nz), d=(d, d, d), m0=m0, fields=fields, tol=1e-6,
                    Ms=1.0e6, A=1.5e-11, Ku=5e4, u=(0.0, 0.0, 1.0))
    if c == 4:
        nx, ny, nz, d = 200, 100, 2, 5e-9
        ku = 500.0 * (1.0 + 0.1 * rng.standard_normal((nz, ny, nx)))
        m0 = uniform_with_noise((1, 0, 0), nx, ny, nz, 1e-3, rng)
        fields = -np.arange(0, 6, 1.0)[:, None] * MT * tilted(1.0)[None, :]
        return dict(name="film 200x100x2, 5 nm cells, per-cell Ku map",
                    n=(nx, ny, nz), d=(d, d, d), m0=m0, fields=fields, tol=1e-6,
                    Ms=8.0e5, A=1.3e-11, Ku=ku, u=(1.0, 0.0, 0.0))
    raise ValueError("unknown workload %r" % (c,))


def batched_platelets(n_samples=64, c=3):
    """Uneven thin platelets: nx in U{64..256}, ny in U{32..128}, nz in U{1,2},
    5 nm cells, Ku in U(0, 2e3) along x, field angle in U(0, 90) degrees,
    start along the field plus 1e-3 noise, +-40 mT loop in 2 mT steps."""
    rng = rng_for(c)
    nx = rng.integers(64, 257, size=n_samples)
    ny = rng.integers(32, 129, size=n_samples)
    nz = rng.integers(1, 3, size=n_samples)
    ku = rng.uniform(0.0, 2e3, size=n_samples)
    psi = rng.uniform(0.0, 90.0, size=n_samples)
    out = []
    for s in range(n_samples):
        h = tilted(psi[s])
        m0 = uniform_with_noise(h, int(nx[s]), int(ny[s]), int(nz[s]), 1e-3, rng)
        out.append(dict(n=(int(nx[s]), int(ny[s]), int(nz[s])), d=(5e-9,) * 3, m0=m0,
                        fields=loop_fields(40.0, 2.0, h), Ms=8.0e5, A=1.3e-11,
                        Ku=float(ku[s]), u=(1.0, 0.0, 0.0), tol=1e-6))
    return out


def sp1_loop(edge="long", cell=10e-9, step_mT=1.0):
    """Standard Problem 1 stand-in loop (Sec. 4): a 2000 x 1000 x 20 nm
    permalloy film (Ms 8e5 A/m, A 1.3e-11 J/m, Ku 500 J/m^3 along the long
    edge x), field along the long edge tilted 1 degree toward y ("long") or
    along the short edge tilted 1 degree toward x ("short"), +-50 mT loop in
    step_mT steps, start along the field with 1e-3 noise.  Seeds: 10 (long
    edge), 11 (short edge), plus 2 for 5 nm cells."""
    deg = {"long": 1.0, "short": 89.0}[edge]
    n = (int(round(2e-6 / cell)), int(round(1e-6 / cell)), int(round(20e-9 / cell)))
    rng = rng_for((10 if edge == "long" else 11) + (2 if cell < 7.5e-9 else 0))
    h = tilted(deg)
    m0 = uniform_with_noise(h, *n, 1e-3, rng)
    return dict(name="SP1 %s edge, %g nm cells, %g mT steps" % (edge, cell * 1e9, step_mT),
                n=n, d=(cell,) * 3, m0=m0, fields=loop_fields(50.0, step_mT, h), h=h,
                tol=1e-6, **PERMALLOY)
