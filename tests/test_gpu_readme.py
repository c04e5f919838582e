"""The usage example of README.md runs as written (tube, plane, box and the
gradient through the adjoint) and gives finite, physical results."""
import os
import re

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    import torch
    assert torch.cuda.is_available()
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert len(blocks) == 1
    env = {}
    exec(compile(blocks[0], "README.md", "exec"), env)
    fields, f2d, f3d = env["fields"], env["f2d"], env["f3d"]
    assert np.isfinite(fields).all() and (fields[5] > 0).all()      # e > 0 along the tube
    assert np.isfinite(f2d).all() and np.isfinite(f3d).all()
    grads = [float(env[k].grad) for k in ("tau", "P_L", "n_L")]
    assert all(np.isfinite(g) for g in grads) and grads[1] != 0.0
