"""Effective field and energy of a finite-difference micromagnet (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper minimises the total free energy U(m) of the normalised magnetisation
(Sec. 2) and defines the effective field as H_eff = -(1/(mu0 Ms)) dU/dm
(eq. (5)).  Its experiments (Sec. 4) use a regular cuboid grid, exchange
constant A, uniaxial anisotropy constant K with easy axis u and a uniform
external field; the demagnetisation field is an FFT convolution (Sec. 3).
The paper names these terms without writing them out; the plain
finite-difference definitions below are the standard ones:

  demag       H_d,i  = -Ms sum_j N(r_i - r_j) m_j             (N: see newell)
  exchange    H_ex,i = 2A/(mu0 Ms) sum_{j in nb(i)} (m_j - m_i)/Delta_ij^2
              six face neighbours; a neighbour outside the body is omitted
              (free / Neumann boundary -- reading, the paper is silent)
  anisotropy  H_an,i = 2 Ku_i/(mu0 Ms) (m_i . u) u
  Zeeman      H_z    = H_ext
  energy      U = -mu0 Ms V sum_i m_i . ( (H_d + H_ex + H_an)_i / 2 + H_ext )
              i.e. U_an = -V sum_i Ku_i (m_i . u)^2 (reading: the constant
              K V is dropped, which changes neither fields nor minimisers),
              U_ex = A V sum_bonds |m_j - m_i|^2 / Delta^2.

Conventions: mu0 = 4 pi 1e-7 (the pre-2019 exact value); SI units, fields in
A/m, energies in J; arrays are [3, nz, ny, nx] (structure of arrays, x
fastest) for vector fields and [nz, ny, nx] for a per-cell Ku map.
"""

import numpy as np

from . import newell

MU0 = 4e-7 * np.pi
DIRECT_MAX_CELLS = 1024   # dense direct demag sum up to this many cells


class Problem:
    """A grid, a material and an external field.

    Parameters follow the paper's Sec. 4 notation: Ms (A/m), A (J/m),
    Ku (J/m^3; scalar or per-cell map [nz, ny, nx]), easy axis u, H_ext (A/m).
    ``demag`` chooses the demag evaluation: 'direct' (O(N^2) sum with the
    tensor of every offset), 'fft' (zero-padded FFT convolution of the same
    tensor) or 'auto' (direct up to DIRECT_MAX_CELLS cells).
    ``fft_workers`` > 1 runs the FFTs of the convolution with scipy.fft on
    that many threads (the same transforms; results agree to rounding).
    """

    def __init__(self, nx, ny, nz, dx, dy, dz, Ms, A, Ku=0.0, u=(1.0, 0.0, 0.0),
                 H_ext=(0.0, 0.0, 0.0), demag="auto", include_demag=True, fft_workers=1):
        self.n = (int(nx), int(ny), int(nz))
        self.d = (float(dx), float(dy), float(dz))
        self.V = float(dx) * float(dy) * float(dz)
        self.Ms = float(Ms)
        self.A = float(A)
        self.Ku = np.asarray(Ku, dtype=np.float64)
        u = np.asarray(u, dtype=np.float64)
        self.u = u / np.linalg.norm(u)
        self.H_ext = np.asarray(H_ext, dtype=np.float64).reshape(3)
        self.include_demag = include_demag
        self.fft_workers = int(fft_workers)
        ncell = nx * ny * nz
        if demag == "auto":
            demag = "direct" if ncell <= DIRECT_MAX_CELLS else "fft"
        self.demag_mode = demag
        self._N = None
        self._D = None
        self._Nhat = None

    # -- demag ------------------------------------------------------------
    @property
    def tensor(self):
        """N on every offset, [6, 2nz-1, 2ny-1, 2nx-1] (see newell)."""
        if self._N is None:
            self._N = newell.full_tensor(*self.n, *self.d)
        return self._N

    def _dense(self):
        """Dense [3N, 3N] matrix of sum_j N(r_i - r_j) . m_j, built from the
        tensor (Ms is applied at evaluation, so it may change afterwards)."""
        if self._D is None:
            nx, ny, nz = self.n
            k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
            i, j, k = i.ravel(), j.ravel(), k.ravel()
            oi = i[:, None] - i[None, :] + (nx - 1)
            oj = j[:, None] - j[None, :] + (ny - 1)
            ok = k[:, None] - k[None, :] + (nz - 1)
            M = newell.tensor_matrix(self.tensor)          # [3, 3, offsets...]
            ncell = i.size
            D = np.zeros((3, ncell, 3, ncell))
            for a in range(3):
                for b in range(3):
                    D[a, :, b, :] = M[a, b][ok, oj, oi]
            self._D = D.reshape(3 * ncell, 3 * ncell)
        return self._D

    def h_demag_direct(self, m):
        """H_d,i = -Ms sum_j N(r_i - r_j) m_j by the plain O(N^2) sum."""
        shape = m.shape
        return -self.Ms * (self._dense() @ m.reshape(-1)).reshape(shape)

    def _ffts(self):
        """(rfftn, irfftn): numpy's, or scipy's on fft_workers threads."""
        if self.fft_workers > 1:
            import scipy.fft as sf
            w = self.fft_workers
            return (lambda a, **k: sf.rfftn(a, workers=w, **k),
                    lambda a, **k: sf.irfftn(a, workers=w, **k))
        return np.fft.rfftn, np.fft.irfftn

    def h_demag_fft(self, m):
        """The same convolution, zero-padded to 2n per axis (1 if n = 1) and
        evaluated with an FFT (Sec. 3: FFT-accelerated convolution)."""
        rfftn, irfftn = self._ffts()
        nx, ny, nz = self.n
        Q = tuple(2 * n if n > 1 else 1 for n in (nz, ny, nx))
        if self._Nhat is None:
            K = np.zeros((6,) + Q)
            Nf = self.tensor
            def emb(n, q):
                idx = np.arange(q)
                off = np.where(idx < n, idx, idx - q)
                ok = np.abs(off) <= n - 1
                return off + (n - 1), ok
            iz, okz = emb(nz, Q[0])
            iy, oky = emb(ny, Q[1])
            ix, okx = emb(nx, Q[2])
            mask = okz[:, None, None] & oky[None, :, None] & okx[None, None, :]
            for c in range(6):
                blk = Nf[c][np.ix_(iz, iy, ix)]
                K[c] = np.where(mask, blk, 0.0)
            self._Nhat = rfftn(K, axes=(1, 2, 3))
        Mh = rfftn(m, s=Q, axes=(1, 2, 3))
        T = newell.tensor_matrix(self._Nhat)
        H = np.empty_like(m)
        for a in range(3):
            acc = T[a, 0] * Mh[0] + T[a, 1] * Mh[1] + T[a, 2] * Mh[2]
            H[a] = -self.Ms * irfftn(acc, s=Q, axes=(0, 1, 2))[:nz, :ny, :nx]
        return H

    def h_demag(self, m):
        if not self.include_demag:
            return np.zeros_like(m)
        if self.demag_mode == "direct":
            return self.h_demag_direct(m)
        return self.h_demag_fft(m)

    # -- local terms ---------------------------------------------------------
    def h_exchange(self, m):
        """Six-neighbour exchange field with free boundaries."""
        H = np.zeros_like(m)
        pref = 2.0 * self.A / (MU0 * self.Ms)
        for axis, delta in ((3, self.d[0]), (2, self.d[1]), (1, self.d[2])):
            if m.shape[axis] < 2:
                continue
            lo = [slice(None)] * 4
            hi = [slice(None)] * 4
            lo[axis] = slice(0, -1)
            hi[axis] = slice(1, None)
            lo, hi = tuple(lo), tuple(hi)
            diff = (m[hi] - m[lo]) / (delta * delta)
            H[lo] += diff        # cell i gains (m_{i+1} - m_i)
            H[hi] -= diff        # cell i+1 gains (m_i - m_{i+1})
        return pref * H

    def h_anisotropy(self, m):
        """Uniaxial anisotropy field 2 Ku/(mu0 Ms) (m . u) u."""
        mu = np.einsum("c...,c->...", m, self.u)
        pref = 2.0 * self.Ku / (MU0 * self.Ms)
        return (pref * mu)[None] * self.u.reshape(3, 1, 1, 1)

    def h_zeeman(self, m):
        return np.broadcast_to(self.H_ext.reshape(3, 1, 1, 1), m.shape).copy()

    # -- totals --------------------------------------------------------------
    def field_terms(self, m):
        """Dict of the four field terms for magnetisation m [3, nz, ny, nx]."""
        return {"demag": self.h_demag(m), "exchange": self.h_exchange(m),
                "anisotropy": self.h_anisotropy(m), "zeeman": self.h_zeeman(m)}

    def heff(self, m):
        """Effective field of eq. (5): the sum of the four terms."""
        t = self.field_terms(m)
        return t["demag"] + t["exchange"] + t["anisotropy"] + t["zeeman"]

    def energy_terms(self, m, terms=None):
        """(U_demag, U_exchange, U_anisotropy, U_zeeman) in J."""
        if terms is None:
            terms = self.field_terms(m)
        k = -MU0 * self.Ms * self.V
        dot = lambda H: float(np.sum(m * H))
        return (0.5 * k * dot(terms["demag"]), 0.5 * k * dot(terms["exchange"]),
                0.5 * k * dot(terms["anisotropy"]), k * dot(terms["zeeman"]))

    def energy(self, m):
        """Total free energy U(m) of Sec. 2."""
        return float(sum(self.energy_terms(m)))
