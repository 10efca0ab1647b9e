"""GPU parity of the compact Poisson solve (Sec. 3, eqs. stream_4O, SequationFinal).

Every call goes through the C ABI (ctypes binding of libcavity.so).

* Fixed sweep counts: the HIP four-colour SOR after k sweeps equals the
  oracle's four-colour sweep applied k times (same ordering, same relaxation),
  to rounding.  Sizes are ragged against the tile size and span many tiles,
  so the halo logic of the temporally blocked kernel is exercised.
* Every compiled FP64 tile configuration, the same way; every FP32 one
  through a converged mixed-precision solve.
* Converged solves: |psi_gpu - psi*| <= ||A^-1||_inf * ||r_gpu||_inf, where psi*
  is the oracle's exact discrete solution, ||A^-1||_inf is computed by the
  oracle (max of the solution for unit vorticity) and ||r_gpu|| is the final
  residual max-norm the GPU reports (<= tolerance).
"""
import numpy as np
import pytest

from oracle.cavity_oracle import poisson_solve, sor_four_colour_sweep
from paper_0809_3098_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cav_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0809_3098_amd.cavity as cav
    return cav


def _inv_norm(n):
    return float(np.max(np.abs(poisson_solve(np.ones((n, n))))))


# (n, sweeps): up to 2048 nodes a side the default tiles are 84 x 54 with 5
# sweeps per launch (launch pairs of 10 sweeps)
@pytest.mark.parametrize("n,sweeps", [(5, 10), (33, 10), (64, 20), (97, 10), (330, 10),
                                      (400, 20), (1024, 10)])
def test_fixed_sweeps_match_oracle_four_colour_sweeps(cav_mod, n, sweeps):
    print(f"[fixed sweeps] n={n} sweeps={sweeps}", flush=True)
    relax = 1.7
    omega = inputs.random_field(n, seed=100 + n)
    c = cav_mod.Cavity(cav_mod.Params(n=n, re=1000.0, sor_omega=relax,
                                      poisson_max_sweeps=sweeps))
    # check after every launch pair, so the sweep limit stops at `sweeps`
    c.set_tuning(check_every=2 * c.tuning()["sweeps_per_launch"])
    psi, info = c.poisson(0, omega, allow_noconv=True)
    c.close()
    assert info["sweeps"] == sweeps
    ref = np.zeros((n, n))
    for _ in range(sweeps):
        ref = sor_four_colour_sweep(ref, omega, relax)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(psi - ref)) <= 1e-13 * scale, np.max(np.abs(psi - ref)) / scale
    assert np.all(psi[0, :] == 0) and np.all(psi[-1, :] == 0)
    assert np.all(psi[:, 0] == 0) and np.all(psi[:, -1] == 0)


# every compiled FP64 sweep configuration (tile x, tile y, sweeps per launch,
# threads), in the XCD-banded tile order
F64_CONFIGS = [(32, 32, 1, 256), (32, 32, 2, 256), (64, 32, 2, 512), (64, 64, 1, 1024),
               (64, 64, 2, 1024), (64, 64, 3, 1024), (64, 64, 2, 512), (64, 64, 4, 512),
               (64, 64, 4, 1024), (64, 64, 4, 768), (96, 64, 2, 1024), (96, 64, 3, 1024),
               (92, 50, 4, 1024), (84, 54, 5, 1024)]


@pytest.mark.parametrize("cfg", F64_CONFIGS)
def test_every_fp64_tile_config_matches_oracle_sweeps(cav_mod, cfg):
    """Two launch pairs, the second ending in a checking launch (wider halo):
    ragged against every tile shape, with tile counts that are not multiples
    of the eight XCDs."""
    tx, ty, s, nt = cfg
    n, relax = 777, 1.6
    sweeps = 4 * s
    print(f"[tile config] {cfg} n={n} sweeps={sweeps}", flush=True)
    omega = inputs.random_field(n, seed=7)
    c = cav_mod.Cavity(cav_mod.Params(n=n, re=1000.0, sor_omega=relax,
                                      poisson_max_sweeps=sweeps))
    c.set_tuning(tile_x=tx, tile_y=ty, sweeps_per_launch=s, threads=nt, xcd_bands=1,
                 check_every=2 * s)
    psi, info = c.poisson(0, omega, allow_noconv=True)
    c.close()
    assert info["sweeps"] == sweeps
    ref = np.zeros((n, n))
    for _ in range(sweeps):
        ref = sor_four_colour_sweep(ref, omega, relax)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(psi - ref)) <= 1e-13 * scale, np.max(np.abs(psi - ref)) / scale


F32_CONFIGS = [(32, 32, 1, 256), (32, 32, 2, 256), (64, 32, 2, 512), (64, 64, 2, 512),
               (64, 64, 2, 1024), (64, 64, 4, 1024), (64, 64, 6, 1024), (96, 64, 3, 1024),
               (96, 96, 3, 1024), (88, 56, 5, 1024), (64, 64, 4, 512), (64, 64, 6, 512)]


@pytest.mark.parametrize("cfg", F32_CONFIGS)
def test_every_fp32_tile_config_converges_to_oracle(cav_mod, cfg):
    """Mixed precision: the FP32 correction sweeps of each configuration
    drive the FP64-refined solve to the tolerance, and the result meets the
    error bound against the oracle's exact solution."""
    tx, ty, s, nt = cfg
    n = 777
    print(f"[fp32 tile config] {cfg} n={n}", flush=True)
    omega = inputs.random_field(n, seed=9, scale=0.02)
    c = cav_mod.Cavity(cav_mod.Params(n=n, re=1000.0, poisson_tol=1e-10, precision=1))
    c.set_tuning(tile_x32=tx, tile_y32=ty, sweeps_per_launch32=s, threads32=nt, xcd_bands=1)
    psi, info = c.poisson(0, omega)
    c.close()
    ref = poisson_solve(omega)
    err = np.max(np.abs(psi - ref))
    bound = 1.02 * _inv_norm(n) * info["resid_inf"] + 1e-14 * np.max(np.abs(ref))
    assert info["status"] == 0
    assert info["resid_inf"] <= 1e-10 or info["floor_limited"] == 1
    assert err <= bound, (err, bound, info)


def _converged_case(cav_mod, n, omega, precision, tol=1e-10):
    c = cav_mod.Cavity(cav_mod.Params(n=n, re=1000.0, poisson_tol=tol, precision=precision))
    psi, info = c.poisson(0, omega)
    c.close()
    ref = poisson_solve(omega)
    err = np.max(np.abs(psi - ref))
    bound = 1.02 * _inv_norm(n) * info["resid_inf"] + 1e-14 * np.max(np.abs(ref))
    return psi, ref, info, err, bound


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n", [17, 64, 130, 513])
def test_converged_solve_random_vorticity(cav_mod, n, precision):
    print(f"[converged random] n={n} precision={precision}", flush=True)
    omega = inputs.random_field(n, seed=7 * n, scale=0.02)
    psi, ref, info, err, bound = _converged_case(cav_mod, n, omega, precision)
    assert info["status"] == 0
    assert info["resid_inf"] <= 1e-10 or info["floor_limited"] == 1
    assert err <= bound, (err, bound, info)


@pytest.mark.parametrize("precision", [0, 1])
def test_converged_solve_full_size_discrete_eigenfunction(cav_mod, precision):
    """psi = sin(pi x) sin(pi y) is an exact discrete solution for a known omega."""
    n = 1024
    print(f"[eigenfunction] n={n} precision={precision}", flush=True)
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    mode = np.sin(np.pi * X) * np.sin(np.pi * Y)
    mode[0, :] = mode[-1, :] = mode[:, 0] = mode[:, -1] = 0.0
    c1 = np.cos(np.pi * h)
    lam = (8.0 * 2 * c1 + 4.0 * c1 * c1 - 20.0) / (6.0 * h * h)
    beta = (8.0 + 4.0 * c1) / 12.0
    omega = -lam / beta * mode * 1e-3          # psi of order 1e-3, like the cavity
    psi, ref, info, err, bound = _converged_case(cav_mod, n, omega, precision)
    assert np.max(np.abs(ref - 1e-3 * mode)) <= 1e-15
    assert info["status"] == 0
    assert err <= bound, (err, bound, info)


def test_converged_solve_lid_like_rhs(cav_mod):
    """The vorticity of the first stage of an impulsively started lid."""
    n = 1024
    print(f"[lid-like] n={n}", flush=True)
    omega = np.zeros((n, n))
    h = 1.0 / (n - 1)
    omega[-1, 1:-1] = -2.0 / h
    omega[-2, 1:-1] = -0.05 / h
    psi, ref, info, err, bound = _converged_case(cav_mod, n, omega, 0)
    assert info["status"] == 0
    assert err <= bound, (err, bound, info)
