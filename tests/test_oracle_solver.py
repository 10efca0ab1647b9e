"""Pins of the oracle's boundary conditions, operators and full time step.

* Thom's formula (Sec. 3.1) is exact when psi is quadratic in the wall-normal
  coordinate with the wall's psi = 0 and tangential velocity (0, or U on the
  lid).
* Eqs. (vel) and (Lwn) are central differences: exact for quadratic psi and
  omega (the advection products) and cubic omega (the diffusion term).
* The full step keeps psi = 0 on all walls bit for bit, is mirror symmetric
  (U -> -U reflects x -> 1-x), scales exactly under U -> 2U, and converges at
  second order in h on nested grids for a smooth flow.
"""
import numpy as np
import pytest

from oracle.cavity_oracle import (CavityOracle, diagnostics, mesh_spacing, thom_walls,
                                  transport_rhs, velocity)


def _nodes(n):
    h = mesh_spacing(n)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    return h, X, Y


# --------------------------------------------------------------------- Thom
def test_thom_exact_for_quadratic_wall_profiles():
    n = 21
    h, X, Y = _nodes(n)
    U = 1.7
    omega = np.full((n, n), 123.0)
    # bottom: psi = 0.3 y^2 -> omega = -psi_yy = -0.6
    w = thom_walls(omega, 0.3 * Y**2, h, U)
    np.testing.assert_allclose(w[0, 1:-1], -0.6, rtol=1e-12)
    # lid: psi = U (y-1) - 0.4 (y-1)^2, psi_y(1) = U -> omega = +0.8
    w = thom_walls(omega, U * (Y - 1) - 0.4 * (Y - 1) ** 2, h, U)
    np.testing.assert_allclose(w[-1, 1:-1], 0.8, rtol=1e-10)
    # left: psi = -0.25 x^2 -> omega = 0.5 ; right: psi = 0.7 (x-1)^2 -> -1.4
    w = thom_walls(omega, -0.25 * X**2, h, U)
    np.testing.assert_allclose(w[1:-1, 0], 0.5, rtol=1e-12)
    w = thom_walls(omega, 0.7 * (X - 1) ** 2, h, U)
    np.testing.assert_allclose(w[1:-1, -1], -1.4, rtol=1e-12)
    # corners are 0 and interior untouched
    assert w[0, 0] == w[0, -1] == w[-1, 0] == w[-1, -1] == 0.0
    assert np.all(w[1:-1, 1:-1] == 123.0)


# ------------------------------------------------------------ central diffs
def test_velocity_and_transport_rhs_exact_on_polynomials():
    n = 17
    h, X, Y = _nodes(n)
    U = 1.0
    nu = 0.37
    psi = 0.5 * X**2 - 0.3 * X * Y + 0.8 * Y**2 + 0.1 * X
    omega = 1.5 * X**2 + 0.4 * X * Y - 0.9 * Y**2 + 2.0 * Y + 0.2 * Y**3
    u_ex = -0.3 * X + 1.6 * Y                      # psi_y
    v_ex = -(1.0 * X - 0.3 * Y + 0.1)              # -psi_x
    wx = 3.0 * X + 0.4 * Y
    wy = 0.4 * X - 1.8 * Y + 2.0 + 0.6 * Y**2
    lap = 3.0 - 1.8 + 1.2 * Y
    u, v = velocity(psi, h, U)
    np.testing.assert_allclose(u[1:-1, 1:-1], u_ex[1:-1, 1:-1], atol=1e-12)
    np.testing.assert_allclose(v[1:-1, 1:-1], v_ex[1:-1, 1:-1], atol=1e-12)
    L = transport_rhs(omega, psi, h, nu)
    L_ex = -u_ex * wx - v_ex * (0.4 * X - 1.8 * Y + 2.0) + nu * lap
    # omega_y of the cubic term is not exact under a central difference:
    # (y+h)^3 - (y-h)^3 = 6 y^2 h + 2 h^3, i.e. an extra 0.2 h^2 in wy
    L_ex = L_ex - v_ex * (0.6 * Y**2 + 0.2 * h**2)
    np.testing.assert_allclose(L, L_ex[1:-1, 1:-1], rtol=0, atol=1e-10)
    # wall velocities
    assert np.all(u[-1, 1:-1] == U) and u[-1, 0] == 0 and u[-1, -1] == 0
    assert np.all(u[0, :] == 0) and np.all(v[:, 0] == 0) and np.all(v[:, -1] == 0)


# ------------------------------------------------------------------ step
def test_initial_state_from_rest():
    n = 33
    U = 1.3
    o = CavityOracle(n, 400.0, u_lid=U)
    h = o.h
    assert np.all(o.psi == 0.0)
    np.testing.assert_allclose(o.omega[-1, 1:-1], -2.0 * U / h, rtol=1e-15)
    assert np.all(o.omega[:-1, :] == 0.0)
    assert o.omega[-1, 0] == 0.0 and o.omega[-1, -1] == 0.0
    assert o.dt == pytest.approx(0.5 * h / U)
    assert o.nu == pytest.approx(U / 400.0)


def test_walls_of_psi_stay_zero_bit_exact():
    o = CavityOracle(33, 1000.0)
    for _ in range(5):
        o.step(4)
        p = o.psi
        assert np.all(p[0, :] == 0.0) and np.all(p[-1, :] == 0.0)
        assert np.all(p[:, 0] == 0.0) and np.all(p[:, -1] == 0.0)
        assert o.omega[0, 0] == o.omega[-1, -1] == 0.0


def test_mirror_symmetry():
    n, re, steps = 33, 500.0, 30
    a = CavityOracle(n, re, u_lid=1.0)
    b = CavityOracle(n, re, u_lid=-1.0)
    a.step(steps)
    b.step(steps)
    sp = np.max(np.abs(a.psi))
    sw = np.max(np.abs(a.omega))
    assert np.max(np.abs(b.psi + a.psi[:, ::-1])) <= 1e-13 * sp
    assert np.max(np.abs(b.omega + a.omega[:, ::-1])) <= 1e-13 * sw
    assert sp > 1e-3


def test_power_of_two_velocity_scaling_is_exact():
    # U -> 2U doubles nu (Re fixed) and halves dt (CFL fixed); the discrete
    # solution at step k is then exactly twice the U = 1 one.
    n, re, steps = 25, 700.0, 12
    a = CavityOracle(n, re, u_lid=1.0)
    b = CavityOracle(n, re, u_lid=2.0)
    assert b.dt * 2 == a.dt
    a.step(steps)
    b.step(steps)
    assert np.array_equal(b.psi, 2.0 * a.psi)
    assert np.array_equal(b.omega, 2.0 * a.omega)


def _smooth_omega0(n):
    """-laplacian of 0.1 sin^2(pi x) sin^2(pi y) (a no-slip-compatible psi)."""
    h, X, Y = _nodes(n)
    sx, sy = np.sin(np.pi * X), np.sin(np.pi * Y)
    return -0.2 * np.pi**2 * (np.cos(2 * np.pi * X) * sy**2 + np.cos(2 * np.pi * Y) * sx**2)


def test_second_order_grid_convergence_smooth_flow():
    T, dt, nu = 0.1, 1e-3, 0.01
    out = {}
    for n in (17, 33, 65, 129, 257):
        o = CavityOracle(n, 1.0, u_lid=0.0, dt=dt, nu=nu, omega0=_smooth_omega0(n))
        o.step(int(round(T / dt)))
        out[n] = (o.psi, o.omega)
    rp, rw = out[257]
    ep, ew = [], []
    for n in (17, 33, 65, 129):
        s = 256 // (n - 1)
        ep.append(np.max(np.abs(out[n][0] - rp[::s, ::s])))
        ew.append(np.max(np.abs(out[n][1] - rw[::s, ::s])))
    op = [np.log2(ep[k] / ep[k + 1]) for k in range(3)]
    ow = [np.log2(ew[k] / ew[k + 1]) for k in range(3)]
    assert all(1.8 < p < 2.4 for p in op), (ep, op)
    assert all(1.8 < p < 2.4 for p in ow[1:]), (ew, ow)


def test_diagnostics_definitions():
    n = 11
    h = mesh_spacing(n)
    z = np.zeros((n, n))
    one = np.ones((n, n))
    d = diagnostics(z, 0.5 * one, z, 3.0 * one, h, 1.0, 0.25)
    assert d["res_psi"] == pytest.approx(0.5 * n * n / n)
    assert d["res_omega"] == pytest.approx(3.0 * n)
    assert d["domega_inf_over_dt"] == pytest.approx(12.0)
    # uniform flow u = 2 (psi = 2 y): KE = 0.5 h^2 (n-2)^2 * 4
    _, X, Y = _nodes(n)
    d = diagnostics(z, 2.0 * Y, z, z, h, 1.0, 1.0)
    assert d["ke"] == pytest.approx(0.5 * h * h * (n - 2) ** 2 * 4.0)


def test_time_convergence_of_cavity_step():
    """Fixed grid, shrinking dt: the stage combination is consistent.

    Every stage inherits the previous stage's wall vorticity before Thom's
    formula refreshes it, so the coupled scheme converges at first order in
    dt (the interior-only SSPRK combination alone is fourth order, pinned by
    the ODE tests).  A wrong stage coefficient would make the scheme
    inconsistent: errors would stop shrinking with dt.
    """
    n, T, nu = 17, 0.1, 0.01
    dts = [4e-3, 2e-3, 1e-3, 5e-4]
    ref_dt = 1.25e-4
    runs = {}
    for dt in dts + [ref_dt]:
        o = CavityOracle(n, 1.0, u_lid=1.0, dt=dt, nu=nu, omega0=_smooth_omega0(n))
        o.step(int(round(T / dt)))
        runs[dt] = o.omega
    e = [np.max(np.abs(runs[d] - runs[ref_dt])) for d in dts]
    orders = [np.log2(e[k] / e[k + 1]) for k in range(len(dts) - 1)]
    assert all(0.9 < p < 1.6 for p in orders), (e, orders)
