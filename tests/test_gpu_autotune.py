"""The autotuner picks launch configurations and sweep schedules by timing
them on the device, caches them, and leaves results correct."""
import json
import os

import numpy as np
import pytest

from mixed_models import mixed_tolerances, rejects, rel
from oracle.cavity_oracle import CavityOracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0809_3098_amd.cavity as cav
    return cav


def test_autotune_single_then_cached(cm, tmp_path):
    n, re = 257, 2000.0
    cache = str(tmp_path / "tune.jsonl")
    print(f"[autotune] n={n}", flush=True)
    # solves to 1e-11: ten steps from rest leave psi small, and the 1e-11 bar
    # then needs a tolerance below the default (see the six-cavity test in
    # test_gpu_batch)
    c = cm.Cavity(cm.Params(n=n, re=re, poisson_tol=1e-11))
    c.step(2, want_stats=False)
    before = c.fields()
    t1 = c.autotune(0, cache)
    after = c.fields()
    # tuning measures on scratch buffers only
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    lines = [json.loads(l) for l in open(cache)]
    assert len(lines) == 1 and lines[0]["key"].endswith(f"n={n}|prec=0|solver=0|batch=0")
    t2 = c.autotune(0, cache)          # cache hit: same answer, no new line
    assert t1 == t2
    assert len(open(cache).readlines()) == 1
    c.step(8, want_stats=False)
    psi, omega, _, _ = c.fields()
    c.close()
    ref = CavityOracle(n, re)
    ref.step(10)
    ep = np.max(np.abs(psi - ref.psi)) / np.max(np.abs(ref.psi))
    ew = np.max(np.abs(omega - ref.omega)) / np.max(np.abs(ref.omega))
    assert ep <= 1e-11 and ew <= 1e-11, (ep, ew, t1)


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_mixed_and_batch(cm, tmp_path, precision):
    members = [(5000.0, 128), (10000.0, 256)]
    cache = str(tmp_path / "tune.jsonl")
    print(f"[autotune batch] precision={precision}", flush=True)
    # FP64: solves to 1e-11 (see the note on few-step runs in test_gpu_batch)
    tol = 1e-11 if precision == 0 else 1e-10
    c = cm.Cavity([cm.Params(n=n, re=re, precision=precision, poisson_tol=tol)
                   for re, n in members])
    c.step(1, want_stats=False)
    c.autotune(0, cache)
    c.autotune(1, cache)
    tb = c.autotune(-1, cache)
    assert tb["sweeps_per_launch"] >= 1
    keys = [json.loads(l)["key"] for l in open(cache)]
    assert len(keys) == 3 and keys[2].endswith("batch=128,256,")
    st = c.step(3)
    assert all(s["status"] == 0 and s["step"] == 4 for s in st)
    psi, omega, _, _ = c.fields(0)
    c.close()
    if precision == 0:
        ref = CavityOracle(128, 5000.0)
        ref.step(4)
        ep, ew = rel(psi, ref.psi), rel(omega, ref.omega)
        print(f"  psi {ep:.3e} omega {ew:.3e}")
        assert ep <= 1e-11 and ew <= 1e-11, (ep, ew)
    else:
        # the precision design's tolerances (see test_gpu_mixed), which reject
        # a run that stores omega in FP32
        (rpsi, romega, _), tol, _, bad = mixed_tolerances(128, 5000.0, 4)
        ep, ew = rel(psi, rpsi), rel(omega, romega)
        print(f"  psi {ep:.3e} (tol {tol['psi']:.3e}) omega {ew:.3e} (tol {tol['omega']:.3e})")
        assert rejects(tol, bad, ("psi", "omega"))
        assert ep <= tol["psi"] and ew <= tol["omega"], (ep, ew, tol)
