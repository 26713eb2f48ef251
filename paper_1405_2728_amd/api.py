"""Python binding of the minimiser library (argument marshalling only).

Every method maps one-to-one onto a function of include/mm.h; all work runs
in the HIP kernels of libmmbb.so.  Magnetisation and field arguments are
torch tensors on a ROCm device, float64, contiguous, with 3*nx*ny*nz
elements in [3][nz][ny][nx] order.  PyTorch supplies device memory and the
stream only.
"""

import ctypes as C

import numpy as np

from . import _lib

MM_FP64 = _lib.MM_FP64
MM_MIXED = _lib.MM_MIXED


class MMError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("%s (%d): %s" % (_lib.STATUS.get(code, "?"), code, message))
        self.code = code


def _dev_ptr(t, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must live on the GPU" % name)
    if t.dtype != torch.float64:
        raise ValueError("%s must be float64" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if n is not None and t.numel() != n:
        raise ValueError("%s must have %d elements, has %d" % (name, n, t.numel()))
    return C.c_void_p(t.data_ptr())


def _d3(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))
    return (C.c_double * 3)(*a.tolist())


class Context:
    """One library context (mm_create) on the current torch stream."""

    def __init__(self, prec="fp64", n_samples=1, stream=None):
        import torch
        self._lib = _lib.load()
        p = {"fp64": MM_FP64, "mixed": MM_MIXED}[prec]
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        handle = C.c_void_p()
        rc = self._lib.mm_create(C.byref(handle), p, int(n_samples), C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise MMError(rc, "mm_create failed")
        self._h = handle
        self.prec = prec
        self.n_samples = int(n_samples)
        self._shape = [None] * self.n_samples

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers ----------------------------------------------------------
    def _check(self, rc, allow_positive=False):
        if rc < 0 or (rc > 0 and not allow_positive):
            msg = self._lib.mm_last_error(self._h)
            raise MMError(rc, msg.decode() if msg else "")
        return rc

    def _n3(self, sample):
        nx, ny, nz = self._shape[sample]
        return 3 * nx * ny * nz

    def _new_field(self, sample):
        import torch
        nx, ny, nz = self._shape[sample]
        return torch.empty((3, nz, ny, nx), dtype=torch.float64, device="cuda")

    # -- set-up -------------------------------------------------------------
    def set_geometry(self, sample, nx, ny, nz, dx, dy, dz):
        self._check(self._lib.mm_set_geometry(self._h, sample, nx, ny, nz, dx, dy, dz))
        self._shape[sample] = (int(nx), int(ny), int(nz))

    def set_material(self, sample, Ms, A, Ku=0.0, u=(1.0, 0.0, 0.0), ku_map=None):
        ptr = None
        if ku_map is not None:
            nx, ny, nz = self._shape[sample]
            ptr = _dev_ptr(ku_map, nx * ny * nz, "ku_map")
        self._check(self._lib.mm_set_material(self._h, sample, Ms, A, Ku, _d3(u), ptr))

    def set_field(self, sample, H):
        self._check(self._lib.mm_set_field(self._h, sample, _d3(H)))

    def reset(self, sample):
        self._check(self._lib.mm_reset(self._h, sample))

    def set_option(self, key, value):
        self._check(self._lib.mm_set_option(self._h, key.encode(), float(value)))

    # -- evaluation -----------------------------------------------------------
    def heff(self, sample, m, out=None):
        n = self._n3(sample)
        if out is None:
            out = self._new_field(sample)
        self._check(self._lib.mm_heff(self._h, sample, _dev_ptr(m, n, "m"), _dev_ptr(out, n, "H")))
        return out

    def heff_static(self, sample, m, out):
        """mm_heff_static: the effective field with the library's fixed
        scratch array (no allocation by the library; out is the caller's)."""
        n = self._n3(sample)
        self._check(self._lib.mm_heff_static(self._h, sample, _dev_ptr(m, n, "m"),
                                             _dev_ptr(out, n, "H")))
        return out

    def field_terms(self, sample, m):
        n = self._n3(sample)
        hd, hex_, han = (self._new_field(sample) for _ in range(3))
        self._check(self._lib.mm_field_terms(self._h, sample, _dev_ptr(m, n, "m"),
                                             _dev_ptr(hd, n), _dev_ptr(hex_, n),
                                             _dev_ptr(han, n)))
        return hd, hex_, han

    def energy(self, sample, m):
        E = C.c_double()
        terms = (C.c_double * 4)()
        self._check(self._lib.mm_energy(self._h, sample, _dev_ptr(m, self._n3(sample), "m"),
                                        C.byref(E), terms))
        return E.value, tuple(terms)

    def mean(self, sample, m):
        out = (C.c_double * 3)()
        self._check(self._lib.mm_mean(self._h, sample, _dev_ptr(m, self._n3(sample), "m"), out))
        return np.array(out[:])

    # -- minimiser ------------------------------------------------------------
    def minimize_step(self, sample, m, info=True):
        si = _lib.StepInfo()
        self._check(self._lib.mm_minimize_step(self._h, sample, _dev_ptr(m, self._n3(sample), "m"),
                                               C.byref(si) if info else None))
        if not info:
            return None
        return {"tau": si.tau, "torque": si.torque, "energy": si.energy, "k": si.k}

    def minimize_to_tol(self, sample, m, tol=1e-6, max_iter=100000):
        r = _lib.MinResult()
        rc = self._check(self._lib.mm_minimize_to_tol(self._h, sample,
                                                      _dev_ptr(m, self._n3(sample), "m"),
                                                      float(tol), int(max_iter), C.byref(r)),
                         allow_positive=True)
        return {"status": rc, "converged": rc == 0, "iters": r.iters,
                "heff_evals": r.heff_evals, "torque": r.torque, "energy": r.energy}

    def minimize_continue(self, sample, m, tol=1e-6, max_iter=100000):
        """Continue the context's run on m (mm_minimize_continue); max_iter
        caps the run's total update count."""
        r = _lib.MinResult()
        rc = self._check(self._lib.mm_minimize_continue(self._h, sample,
                                                        _dev_ptr(m, self._n3(sample), "m"),
                                                        float(tol), int(max_iter), C.byref(r)),
                         allow_positive=True)
        return {"status": rc, "converged": rc == 0, "iters": r.iters,
                "heff_evals": r.heff_evals, "torque": r.torque, "energy": r.energy}

    def state_save(self, sample):
        """Checkpoint of the sample's run (mm_state_save) as bytes; m is not
        part of it."""
        n = C.c_int64()
        self._check(self._lib.mm_state_bytes(self._h, sample, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self._lib.mm_state_save(self._h, sample, buf, n.value))
        return buf.raw

    def state_load(self, sample, blob):
        """Restore a checkpoint written by state_save (mm_state_load)."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        self._check(self._lib.mm_state_load(self._h, sample, buf, len(blob)))

    def last_step(self, sample):
        """tau of the most recent update, torque and energy of the most
        recent evaluation and its index k (mm_last_step)."""
        si = _lib.StepInfo()
        self._check(self._lib.mm_last_step(self._h, sample, C.byref(si)))
        return {"tau": si.tau, "torque": si.torque, "energy": si.energy, "k": si.k}

    def hysteresis_sweep(self, ms, H, tol=1e-6, max_iter=100000):
        """ms: list of n_samples magnetisation tensors; H: [n_samples, n_fields, 3]
        (A/m).  Returns (<m> [S, F, 3], iters [S, F], status)."""
        H = np.ascontiguousarray(np.asarray(H, dtype=np.float64))
        if H.ndim == 2:
            H = H[None]
        S, F = H.shape[0], H.shape[1]
        if S != self.n_samples or len(ms) != S:
            raise ValueError("need one magnetisation and one field list per sample")
        ptrs = (C.c_void_p * S)(*[_dev_ptr(m, self._n3(k), "m").value for k, m in enumerate(ms)])
        mavg = np.zeros((S, F, 3))
        iters = np.zeros((S, F), dtype=np.int64)
        rc = self._check(self._lib.mm_hysteresis_sweep(
            self._h, ptrs, H.ctypes.data_as(C.POINTER(C.c_double)), F, float(tol), int(max_iter),
            mavg.ctypes.data_as(C.POINTER(C.c_double)),
            iters.ctypes.data_as(C.POINTER(C.c_int64))), allow_positive=True)
        return mavg, iters, rc

    # -- derivatives ------------------------------------------------------------
    def hessvec(self, sample, m, v, out=None):
        """Riemannian Hessian of U at m applied to the tangent field v."""
        n = self._n3(sample)
        if out is None:
            out = self._new_field(sample)
        self._check(self._lib.mm_hessvec(self._h, sample, _dev_ptr(m, n, "m"), _dev_ptr(v, n, "v"),
                                         _dev_ptr(out, n, "out")))
        return out

    def adjoint_solve(self, sample, m, rhs, tol=1e-10, max_iter=10000, out=None):
        """Adjoint field lam with Hess(m) lam = P rhs (conjugate gradients).
        Returns (lam, iterations, relative residual, status)."""
        n = self._n3(sample)
        if out is None:
            out = self._new_field(sample)
        it = C.c_int64()
        res = C.c_double()
        rc = self._check(self._lib.mm_adjoint_solve(
            self._h, sample, _dev_ptr(m, n, "m"), _dev_ptr(rhs, n, "rhs"), _dev_ptr(out, n, "lam"),
            float(tol), int(max_iter), C.byref(it), C.byref(res)), allow_positive=True)
        return out, it.value, res.value, rc

    def param_grads(self, sample, m, lam, ku=True):
        """Implicit gradients: dict with "A", "Ms" (floats), "H_ext" (3
        floats) and "Ku" (map [nz, ny, nx] or None)."""
        import torch
        n = self._n3(sample)
        dA = C.c_double()
        dMs = C.c_double()
        dH = (C.c_double * 3)()
        dKu = None
        if ku:
            nx, ny, nz = self._shape[sample]
            dKu = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
        self._check(self._lib.mm_param_grads(
            self._h, sample, _dev_ptr(m, n, "m"), _dev_ptr(lam, n, "lam"), C.byref(dA),
            C.byref(dMs), dH, _dev_ptr(dKu, n // 3, "dKu") if ku else None))
        return {"A": dA.value, "Ms": dMs.value, "H_ext": np.array(dH[:]), "Ku": dKu}

    def energy_grads(self, sample, m):
        """Derivatives of U at m: dict with "m" (tensor), "Ku" (tensor), "Ms",
        "A" (floats) and "H_ext" (3 floats)."""
        import torch
        n = self._n3(sample)
        nx, ny, nz = self._shape[sample]
        dm = self._new_field(sample)
        dku = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
        sc = (C.c_double * 5)()
        self._check(self._lib.mm_energy_grads(self._h, sample, _dev_ptr(m, n, "m"),
                                              _dev_ptr(dm, n), _dev_ptr(dku, n // 3), sc))
        return {"m": dm, "Ku": dku, "Ms": sc[0], "A": sc[1], "H_ext": np.array(sc[2:5])}

    def counters(self, sample):
        e = C.c_int64()
        i = C.c_int64()
        self._check(self._lib.mm_counters(self._h, sample, C.byref(e), C.byref(i)))
        return e.value, i.value

    def rows_per_block(self, sample):
        r = C.c_int()
        self._check(self._lib.mm_rows_per_block(self._h, sample, C.byref(r)))
        return r.value

    def yz_variant(self, sample):
        r = C.c_int()
        self._check(self._lib.mm_yz_variant(self._h, sample, C.byref(r)))
        return r.value

    # -- timing ---------------------------------------------------------------
    def profile(self, kernels=None):
        """Time the named kernels (None or [] stops; "all" times every
        kernel) with HIP events."""
        mask = 0
        if kernels == "all":
            mask = (1 << 30) - 1
        elif kernels:
            k = 0
            while True:
                name = self._lib.mm_kernel_name(k)
                if name is None:
                    break
                if name.decode() in kernels:
                    mask |= 1 << k
                k += 1
        self._check(self._lib.mm_profile(self._h, mask))

    def profile_read(self):
        out = {}
        k = 0
        while True:
            name = self._lib.mm_kernel_name(k)
            if name is None:
                break
            ms = C.c_double()
            n = C.c_int64()
            self._check(self._lib.mm_profile_read(self._h, k, C.byref(ms), C.byref(n)))
            out[name.decode()] = (ms.value, n.value)
            k += 1
        return out

    def kernel_bytes(self, sample):
        out = {}
        k = 0
        while True:
            name = self._lib.mm_kernel_name(k)
            if name is None:
                break
            b = C.c_double()
            self._check(self._lib.mm_kernel_bytes(self._h, sample, k, C.byref(b)))
            out[name.decode()] = b.value
            k += 1
        return out


def supported(prec, nx, ny, nz):
    p = {"fp64": MM_FP64, "mixed": MM_MIXED}[prec]
    return bool(_lib.load().mm_supported(p, nx, ny, nz))
