"""The Python examples of README.md run as written on the GPU (a solve with a snapshot and
a checkpoint file restarted bit for bit; a served stream of 200 requests)."""
import os
import re

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_examples_run(gpu, tmp_path, monkeypatch):
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert len(blocks) >= 2
    monkeypatch.chdir(tmp_path)  # the checkpoint file goes here
    scope = {}
    for i, block in enumerate(blocks):
        print("README python block %d" % i, flush=True)
        exec(compile(block, "README.md python block %d" % i, "exec"), scope)
    assert (tmp_path / "half.npz").exists()
