"""Pins of the oracle's field terms and energy (closed forms, brute force)."""

import numpy as np
import pytest

from oracle import fields

MU0 = 4e-7 * np.pi


def random_unit(shape, seed):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((3,) + shape)
    return m / np.linalg.norm(m, axis=0)


def test_demag_fft_equals_direct_sum():
    P = fields.Problem(9, 6, 3, 5e-9, 4e-9, 3e-9, Ms=8e5, A=1.3e-11)
    m = random_unit((3, 6, 9), 3)
    a = P.h_demag_direct(m)
    b = P.h_demag_fft(m)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_demag_fft_threaded_equals_direct_sum():
    """The multi-threaded FFT (scipy.fft workers) gives the same convolution."""
    P = fields.Problem(9, 6, 3, 5e-9, 4e-9, 3e-9, Ms=8e5, A=1.3e-11, fft_workers=4)
    m = random_unit((3, 6, 9), 3)
    a = P.h_demag_direct(m)
    b = P.h_demag_fft(m)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_demag_direct_by_explicit_pair_loop():
    """The dense matrix against a literal double loop over cell pairs."""
    nx, ny, nz = 3, 2, 2
    d = (5e-9, 5e-9, 3e-9)
    P = fields.Problem(nx, ny, nz, *d, Ms=8e5, A=0.0, demag="direct")
    m = random_unit((nz, ny, nx), 4)
    from oracle import newell
    H = np.zeros_like(m)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for kk in range(nz):
                    for jj in range(ny):
                        for ii in range(nx):
                            R = ((i - ii) * d[0], (j - jj) * d[1], (k - kk) * d[2])
                            N6 = newell.newell_tensor(*R, *d)[:, 0]
                            M = newell.tensor_matrix(N6)
                            H[:, k, j, i] += -8e5 * M @ m[:, kk, jj, ii]
    assert np.max(np.abs(H - P.h_demag(m))) < 1e-12 * np.max(np.abs(H))


def test_exchange_uniform_is_zero():
    P = fields.Problem(6, 5, 3, 5e-9, 5e-9, 5e-9, Ms=8e5, A=1.3e-11)
    m = np.zeros((3, 3, 5, 6))
    m[:] = np.array([0.6, 0.0, 0.8])[:, None, None, None]
    assert np.max(np.abs(P.h_exchange(m))) < 1e-9


def test_exchange_helix_closed_form():
    """m = (cos kx, sin kx, 0): interior H_ex = -(4A/(mu0 Ms dx^2))(1 - cos k dx) m;
    the two end cells miss one neighbour."""
    nx, dx = 20, 5e-9
    Ms, A = 8e5, 1.3e-11
    k = 0.3 / dx
    x = np.arange(nx) * dx
    m = np.zeros((3, 1, 1, nx))
    m[0, 0, 0] = np.cos(k * x)
    m[1, 0, 0] = np.sin(k * x)
    P = fields.Problem(nx, 1, 1, dx, dx, dx, Ms=Ms, A=A)
    H = P.h_exchange(m)
    pref = 2 * A / (MU0 * Ms * dx * dx)
    interior = -2 * pref * (1 - np.cos(k * dx)) * m[:, 0, 0, 1:-1]
    assert np.allclose(H[:, 0, 0, 1:-1], interior, rtol=1e-12, atol=1e-6)
    # end cell 0 only sees cell 1
    end0 = pref * (m[:, 0, 0, 1] - m[:, 0, 0, 0])
    assert np.allclose(H[:, 0, 0, 0], end0, rtol=1e-12, atol=1e-6)


def test_exchange_anisotropic_spacing():
    """Variation only along z, with dz != dx: only the z bonds contribute,
    each divided by dz^2."""
    Ms, A, dz = 8e5, 1.3e-11, 3e-9
    m = np.zeros((3, 3, 2, 2))
    th = np.array([0.0, 0.2, 0.5])
    m[0] = np.cos(th)[:, None, None]
    m[2] = np.sin(th)[:, None, None]
    P = fields.Problem(2, 2, 3, 5e-9, 4e-9, dz, Ms=Ms, A=A)
    H = P.h_exchange(m)
    pref = 2 * A / (MU0 * Ms * dz * dz)
    mid = pref * (m[:, 0] + m[:, 2] - 2 * m[:, 1])
    assert np.allclose(H[:, 1], mid, rtol=1e-12, atol=1e-6)


def test_anisotropy_and_zeeman_closed_form():
    Ms, Ku = 8e5, 500.0
    u = np.array([1.0, 2.0, 2.0]) / 3.0
    m = random_unit((1, 2, 2), 7)
    P = fields.Problem(2, 2, 1, 5e-9, 5e-9, 5e-9, Ms=Ms, A=0.0, Ku=Ku, u=u,
                       H_ext=(10.0, -20.0, 30.0))
    H = P.h_anisotropy(m)
    for j in range(2):
        for i in range(2):
            mm = m[:, 0, j, i]
            assert np.allclose(H[:, 0, j, i], 2 * Ku / (MU0 * Ms) * (mm @ u) * u, rtol=1e-14)
    assert np.allclose(P.h_zeeman(m)[:, 0, 1, 1], [10.0, -20.0, 30.0])
    # anisotropy energy -V sum Ku (m.u)^2
    E = P.energy_terms(m)
    assert abs(E[2] - (-P.V * Ku * np.sum(np.einsum("c...,c->...", m, u) ** 2))) < 1e-30


def test_ku_map_per_cell():
    Ms = 8e5
    Ku = np.array([[[100.0, 200.0], [300.0, 400.0]]])
    m = random_unit((1, 2, 2), 9)
    P = fields.Problem(2, 2, 1, 5e-9, 5e-9, 5e-9, Ms=Ms, A=0.0, Ku=Ku)
    H = P.h_anisotropy(m)
    assert np.allclose(H[0], 2 * Ku / (MU0 * Ms) * m[0], rtol=1e-14)
    assert np.all(H[1:] == 0)


def test_exchange_energy_bond_form():
    """-1/2 mu0 Ms V sum m.H_ex equals A V sum_bonds |m_j - m_i|^2/Delta^2."""
    d = (5e-9, 4e-9, 3e-9)
    A = 1.3e-11
    m = random_unit((3, 4, 5), 11)
    P = fields.Problem(5, 4, 3, *d, Ms=8e5, A=A)
    e = P.energy_terms(m)[1]
    V = d[0] * d[1] * d[2]
    bonds = (np.sum((m[:, :, :, 1:] - m[:, :, :, :-1]) ** 2) / d[0] ** 2
             + np.sum((m[:, :, 1:] - m[:, :, :-1]) ** 2) / d[1] ** 2
             + np.sum((m[:, 1:] - m[:, :-1]) ** 2) / d[2] ** 2)
    assert abs(e - A * V * bonds) < 1e-12 * abs(e)


@pytest.mark.parametrize("mode", ["direct", "fft"])
def test_energy_gradient_consistency(mode):
    """dU along a tangent perturbation equals -mu0 Ms V H_eff . dm (eq. (5))."""
    nx, ny, nz = 6, 4, 2
    P = fields.Problem(nx, ny, nz, 5e-9, 5e-9, 5e-9, Ms=8e5, A=1.3e-11, Ku=500.0,
                       H_ext=(1e4, -3e3, 2e3), demag=mode)
    m = random_unit((nz, ny, nx), 5)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(m.shape)
    v -= np.sum(v * m, axis=0) * m           # tangent
    H = P.heff(m)
    slope = -8e5 * MU0 * P.V * np.sum(H * v)
    h = 1e-6

    def E(t):
        mm = m + t * v
        mm /= np.linalg.norm(mm, axis=0)
        return P.energy(mm)
    fd = (E(h) - E(-h)) / (2 * h)
    assert abs(fd - slope) < 1e-6 * abs(slope)


def test_demag_energy_positive_and_symmetric_operator():
    """The demag operator is symmetric negative semi-definite: U_d >= 0 and
    a . D b = b . D a."""
    P = fields.Problem(5, 4, 2, 5e-9, 5e-9, 5e-9, Ms=8e5, A=0.0, demag="direct")
    a = random_unit((2, 4, 5), 1)
    b = random_unit((2, 4, 5), 2)
    assert abs(np.sum(a * P.h_demag(b)) - np.sum(b * P.h_demag(a))) < 1e-9 * 8e5
    assert P.energy_terms(a)[0] > 0
