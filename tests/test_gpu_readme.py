"""The usage example of README.md runs as written: it relaxes the
400 x 200 x 4 film from +x at +50 mT (1 degree toward y) to the tolerance."""

import os
import re

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with open(os.path.join(ROOT, "README.md")) as f:
        blocks = re.findall(r"```python\n(.*?)```", f.read(), re.S)
    assert len(blocks) == 1
    print("case README example", flush=True)
    ns = {}
    exec(compile(blocks[0], "README.md", "exec"), ns)
    r, H, m = ns["r"], ns["H"], ns["m"]
    print("  ", r, flush=True)
    assert r["converged"] and r["torque"] < 1e-6
    assert bool(torch.isfinite(H).all())
    norm = (m * m).sum(0).sqrt()
    assert float((norm - 1).abs().max()) < 1e-12
    assert float(m[0].mean()) > 0.9
