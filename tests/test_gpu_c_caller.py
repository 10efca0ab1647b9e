"""The C ABI used from plain C (no Python, no torch): the example program's
fields equal the Python binding's bit for bit, and its monitors match."""
import os
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEMO = os.path.join(ROOT, "paper_0809_3098_amd", "examples", "cavity_step_demo")


def test_c_caller_matches_python_binding(tmp_path):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0809_3098_amd.cavity as cm
    assert os.path.exists(DEMO), "build the library first (it builds the C example)"
    n, re, steps = 64, 1000.0, 20
    print(f"[c caller] n={n} re={re} steps={steps}", flush=True)
    out = tmp_path / "fields.bin"
    res = subprocess.run([DEMO, str(n), repr(re), str(steps), str(out)], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    words = res.stdout.split()
    got = np.fromfile(out, dtype=np.float64).reshape(2, n, n)
    c = cm.Cavity(cm.Params(n=n, re=re))
    st = c.step(steps)[0]
    psi, omega, _, _ = c.fields()
    c.close()
    assert np.array_equal(got[0], psi) and np.array_equal(got[1], omega)
    assert int(words[1]) == steps and float(words[7]) == st["ke"]
