"""mm_heff_static (the allocation-free effective field) against mm_heff.

Both run the same kernels on the same input; only the memory holding the
convolution's spectrum differs (the library's fixed per-GPU array instead of
the sample's buffers), so the fields must agree bit for bit.  Two calls in a
row, the second on a smaller grid (the array keeps the first call's
contents), on the thin-film path and the full 3-D path, in FP64 and in the
mixed form; a grid whose spectrum exceeds the array is rejected.
"""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1405_2728_amd import _build
    _build.ensure_built()
    return torch


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_static_heff_equals_heff(torch_cuda, prec):
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    # film (17.2 MB spectrum in FP64), then smaller thin and 3-D grids
    grids = [(400, 200, 4), (100, 50, 2), (64, 48, 8)]
    ctx = Context(prec, n_samples=len(grids))
    fields = []
    for k, n in enumerate(grids):
        ctx.set_geometry(k, *n, 5e-9, 5e-9, 4e-9)
        ctx.set_material(k, 8e5, 1.3e-11, 2e3, (0.6, 0.8, 0.0))
        ctx.set_field(k, (1e4, -2e3, 5e2))
        rng = np.random.default_rng(70 + k)
        fields.append(torch.tensor(synth.random_unit(*n, rng), device="cuda"))
    for k, n in enumerate(grids):
        say("case heff_static", prec, n)
        m = fields[k]
        ref = ctx.heff(k, m)
        out = torch.full_like(m, float("nan"))
        ctx.heff_static(k, m, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), float((out - ref).abs().max())
    # the film again after the smaller grids (array holds their data)
    out = torch.full_like(fields[0], float("nan"))
    ctx.heff_static(0, fields[0], out)
    assert torch.equal(out, ctx.heff(0, fields[0]))
    ctx.close()


def test_static_heff_rejects_oversized_grid(torch_cuda):
    torch = torch_cuda
    from paper_1405_2728_amd import Context
    from paper_1405_2728_amd.api import MMError
    n = (256, 256, 16)          # 3-D path: spectra of ~50 + ~100 MB
    ctx = Context("fp64")
    ctx.set_geometry(0, *n, 2e-9, 2e-9, 2e-9)
    ctx.set_material(0, 8e5, 1.3e-11, 0.0, (1, 0, 0))
    m = torch.zeros((3, n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
    m[0] = 1.0
    out = torch.zeros_like(m)
    with pytest.raises(MMError) as e:
        ctx.heff_static(0, m, out)
    assert e.value.code == -1 and "bytes of scratch" in str(e.value)
    assert torch.count_nonzero(out) == 0
    ctx.close()
