"""The Python example in README.md runs as written (on cuda:0) and does
what it says: a batch of two views into maps, and a split in place."""
import os
import re

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_python_example_runs():
    import torch

    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert len(blocks) == 1
    env = {}
    exec(compile(blocks[0], "README.md", "exec"), env)
    torch.cuda.synchronize()
    assert int(env["status"].item()) == 0
    assert int(env["count"].item()) == env["N"]          # an all-zero mask splits nothing
    assert torch.isfinite(env["maps"]).all()
    assert (env["maps"] == 0).all()                      # black images: no edges
