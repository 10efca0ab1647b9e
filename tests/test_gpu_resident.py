"""The resident solve (CAVITY_EXEC_RESIDENT): one launch per Poisson solve,
tiles kept on chip, halos swapped with the neighbouring tiles every round.

* Exactness of the halo exchange: a solve stopped by its sweep limit reports
  how many sweeps it made; psi equals the oracle's four-colour sweep applied
  that many times (1e-13 relative), on grids of several tiles in both tile
  shapes of the resident kernel and ragged against them.
* Converged solves meet the same error bound as the per-launch path.
* Time steps agree with the FP64 oracle to 1e-11 and with the per-launch
  path to within the solve tolerance.
* A cavity the resident kernel does not take (mixed precision) still runs.
"""
import numpy as np
import pytest

from mixed_models import mixed_tolerances, rejects
from oracle.cavity_oracle import CavityOracle, poisson_solve, sor_four_colour_sweep
from paper_0809_3098_amd import inputs

pytestmark = pytest.mark.gpu

PARITY = 1e-11


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0809_3098_amd.cavity as cav
    return cav


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("n,limit", [(64, 12), (200, 20), (600, 40), (777, 50)])
def test_sweep_limited_solve_equals_oracle_sweeps(cm, n, limit):
    print(f"[resident sweeps] n={n} limit={limit}", flush=True)
    relax = 1.7
    omega = inputs.random_field(n, seed=300 + n)
    c = cm.Cavity(cm.Params(n=n, re=1000.0, sor_omega=relax, poisson_max_sweeps=limit))
    c.set_exec(cm.CAVITY_EXEC_RESIDENT)
    psi, info = c.poisson(0, omega, allow_noconv=True)
    c.close()
    sweeps = info["sweeps"]
    print(f"  sweeps={sweeps} status={info['status']}")
    assert sweeps >= limit and info["status"] == cm.CAVITY_ENOCONV
    ref = np.zeros((n, n))
    for _ in range(sweeps):
        ref = sor_four_colour_sweep(ref, omega, relax)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(psi - ref)) <= 1e-13 * scale, np.max(np.abs(psi - ref)) / scale
    assert np.all(psi[0, :] == 0) and np.all(psi[-1, :] == 0)
    assert np.all(psi[:, 0] == 0) and np.all(psi[:, -1] == 0)


@pytest.mark.parametrize("n", [97, 513, 1024])
def test_converged_resident_solve(cm, n):
    print(f"[resident converged] n={n}", flush=True)
    omega = inputs.random_field(n, seed=11 * n, scale=0.02)
    c = cm.Cavity(cm.Params(n=n, re=1000.0, poisson_tol=1e-10))
    c.set_exec(cm.CAVITY_EXEC_RESIDENT)
    psi, info = c.poisson(0, omega)
    c.close()
    ref = poisson_solve(omega)
    inv = float(np.max(np.abs(poisson_solve(np.ones((n, n))))))
    err = np.max(np.abs(psi - ref))
    bound = 1.02 * inv * info["resid_inf"] + 1e-14 * np.max(np.abs(ref))
    print(f"  sweeps={info['sweeps']} resid={info['resid_inf']:.3e} err={err:.3e}")
    assert info["status"] == 0
    assert info["resid_inf"] <= 1e-10 or info["floor_limited"] == 1
    assert err <= bound, (err, bound, info)


@pytest.mark.parametrize("n,re,steps", [(64, 1000.0, 100), (1024, 1.0e4, 20)])
def test_resident_steps_match_oracle_and_stream(cm, n, re, steps):
    print(f"[resident steps] n={n} re={re} steps={steps}", flush=True)
    out = {}
    for mode in ("resident", "stream"):
        c = cm.Cavity(cm.Params(n=n, re=re, poisson_tol=1e-10))
        c.set_exec(cm.CAVITY_EXEC_RESIDENT if mode == "resident" else cm.CAVITY_EXEC_STREAM)
        st = c.step(steps)[0]
        out[mode] = c.fields()[:2] + (st,)
        c.close()
    ref = CavityOracle(n, re, workers=-1)
    ref.step(steps)
    psi, omega, st = out["resident"]
    ep, ew = _rel(psi, ref.psi), _rel(omega, ref.omega)
    print(f"  resident psi_rel={ep:.3e} omega_rel={ew:.3e} sweeps/step={st['sweeps_last_step']} "
          f"stream sweeps/step={out['stream'][2]['sweeps_last_step']}")
    assert ep <= PARITY and ew <= PARITY, (ep, ew)
    assert st["status"] == 0
    assert _rel(psi, out["stream"][0]) <= PARITY


def test_resident_mode_runs_other_cavities_as_stream(cm):
    print("[resident fallback]", flush=True)
    n, steps = 130, 5
    # the FP64 cavity solves to 1e-11 for the 1e-11 bar after a few steps from
    # rest (see the six-cavity test in test_gpu_batch)
    members = [cm.Params(n=n, re=2000.0, poisson_tol=1e-11),
               cm.Params(n=n, re=2.0e4, precision=cm.CAVITY_MIXED)]
    c = cm.Cavity(members)
    c.set_exec(cm.CAVITY_EXEC_RESIDENT)
    assert c.exec_mode() == cm.CAVITY_EXEC_RESIDENT
    stats = c.step(steps)
    assert all(s["status"] == 0 for s in stats)
    p64, w64 = c.fields(0)[:2]
    p32, w32 = c.fields(1)[:2]
    c.close()
    # the FP64 cavity (resident) at parity, the mixed one (per launch) within
    # the precision design's tolerances (see test_gpu_mixed)
    ref = CavityOracle(n, 2000.0)
    ref.step(steps)
    assert _rel(p64, ref.psi) <= PARITY and _rel(w64, ref.omega) <= PARITY
    (rpsi, romega, _), tol, _, bad = mixed_tolerances(n, 2.0e4, steps)
    assert rejects(tol, bad, ("psi", "omega"))
    assert _rel(p32, rpsi) <= tol["psi"] and _rel(w32, romega) <= tol["omega"]
