"""Full-size and maximum-size cases, in the launch configuration the bench uses.

* 4096 x 4096, Re = 3e4, noise start, one step: FP64 multigrid and mixed
  SOR (the configuration of that workload) against the FP64 oracle.  After a
  single step psi is still small (max 6e-5) and each of the five solves may
  leave an error of ||A^-1|| * tol in psi, so the comparison uses that bound
  (||A^-1||_inf computed by the oracle, the residual reported by the GPU);
  omega inherits the psi error through Thom's wall formula (2 / h^2), and the
  mixed path adds 4 times the error of the precision design's CPU model
  (``mixed_models.MixedModel``: eq. (Lwn) in FP32) for psi and omega.  Here
  the solver-tolerance term through Thom's 2 / h^2 (about 1e-3) exceeds what
  storing omega in FP32 would cost (about 4e-4), so this one-step check
  cannot see that defect; the mixed tests with discriminating tolerances are
  in test_gpu_mixed (including the 1024^2 cavity).
* The largest grid the library accepts (16385 x 16385): a solve stopped by
  its sweep limit is checked at sample nodes -- centre, next to a wall, next
  to a corner -- against the oracle's four-colour sweeps on a window around
  each sample; after k sweeps a node depends only on nodes within 4k of it.
"""
import numpy as np
import pytest

from mixed_models import FACTOR, mixed_tolerances
from oracle.cavity_oracle import CavityOracle, poisson_solve, sor_four_colour_sweep
from paper_0809_3098_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0809_3098_amd.cavity as cav
    return cav


@pytest.fixture(scope="module")
def ref4096():
    n, re = 4096, 3.0e4
    w0 = inputs.noise_omega0(n, 1e-3, 0)
    ref = CavityOracle(n, re, omega0=w0, workers=-1)
    ref.step(1)
    inv = float(np.max(np.abs(poisson_solve(np.ones((n, n)), workers=-1))))
    return n, re, w0, ref, inv


def _run(cm, n, re, w0, precision, solver):
    c = cm.Cavity(cm.Params(n=n, re=re, poisson_tol=1e-10, precision=precision), omega0=[w0])
    if solver:
        c.set_tuning(solver=solver)
    st = c.step(1)[0]
    psi, omega = c.fields()[:2]
    c.close()
    return psi, omega, st


def _check(psi, omega, ref, inv, resid, extra_w=0.0, extra_psi=0.0):
    h = ref.h
    bpsi = 5.5 * inv * resid + 1e-14 * np.max(np.abs(ref.psi)) + extra_psi
    bw = 2.0 / (h * h) * bpsi + extra_w + 1e-12 * np.max(np.abs(ref.omega))
    ep = np.max(np.abs(psi - ref.psi))
    ew = np.max(np.abs(omega - ref.omega))
    print(f"  |dpsi|={ep:.3e} (bound {bpsi:.3e})  |domega|={ew:.3e} (bound {bw:.3e})")
    assert ep <= bpsi and ew <= bw, (ep, bpsi, ew, bw)


def test_cavity4096_one_step_fp64_multigrid(cm, ref4096):
    n, re, w0, ref, inv = ref4096
    print(f"[4096 fp64 multigrid] n={n} re={re}", flush=True)
    psi, omega, st = _run(cm, n, re, w0, cm.CAVITY_FP64, cm.CAVITY_SOLVER_MG)
    assert st["status"] == 0
    _check(psi, omega, ref, inv, 1e-10)


def test_cavity4096_one_step_mixed_sor(cm, ref4096):
    n, re, w0, ref, inv = ref4096
    print(f"[4096 mixed sor] n={n} re={re}", flush=True)
    psi, omega, st = _run(cm, n, re, w0, cm.CAVITY_MIXED, 0)
    assert st["status"] == 0
    _, _, model, _ = mixed_tolerances(n, re, 1, ("noise", 1e-3, 0))
    extra_psi = FACTOR * model["psi"] * np.max(np.abs(ref.psi))
    extra_w = FACTOR * model["omega"] * np.max(np.abs(ref.omega))
    _check(psi, omega, ref, inv, 1e-10, extra_w, extra_psi)


def test_largest_grid_sampled_sweeps(cm):
    n, relax = 16385, 1.7
    print(f"[largest grid] n={n}", flush=True)
    omega = inputs.random_field(n, seed=5)
    # no extrapolation history (5 * levels fields of 2 GiB each at this size):
    # the test takes no time step
    c = cm.Cavity(cm.Params(n=n, re=1000.0, sor_omega=relax, poisson_max_sweeps=12,
                            warm_start=cm.CAVITY_WARM_PREVIOUS))
    c.set_tuning(check_every=2 * c.tuning()["sweeps_per_launch"])
    psi, info = c.poisson(0, omega, allow_noconv=True)
    c.close()
    k = info["sweeps"]
    print(f"  sweeps={k}")
    assert k >= 12
    rad = 4 * k + 4
    for (j, i) in ((n // 2, n // 2), (n // 3, 2), (n - 3, n - 3)):
        j0 = max(0, (j - rad) // 2 * 2)
        i0 = max(0, (i - rad) // 2 * 2)
        j1 = min(n, j + rad + 1)
        i1 = min(n, i + rad + 1)
        # the window's own edge is held fixed: a domain wall (psi = 0) where it
        # is one, else beyond the reach of the sample node
        win = np.zeros((j1 - j0, i1 - i0))
        w = omega[j0:j1, i0:i1]
        for _ in range(k):
            win = sor_four_colour_sweep(win, w, relax, h=1.0 / (n - 1))
        got = psi[j, i]
        want = win[j - j0, i - i0]
        assert abs(got - want) <= 1e-13 * max(1e-300, np.max(np.abs(win))), (j, i, got, want)
