"""Pins of the oracle's compact Poisson solve (Sec. 3, eqs. stream_4O, SequationFinal).

Independent evidence that the DST-based solve computes the solution of the
paper's compact equations:

* brute force: a dense matrix assembled node by node from the relaxation
  formula's fixed point and solved with LAPACK;
* the paper's own lexicographic relaxation, run to convergence;
* polynomial exactness (the compact scheme is exact for psi of degree <= 5
  with omega = -laplacian(psi));
* fourth-order convergence to the continuous solution psi = sin(pi x) sin(pi y);
* the discrete eigenfunction sin(p pi x) sin(q pi y).
"""
import numpy as np
import pytest

from oracle.cavity_oracle import (compact_eigenvalues, compact_operator, mesh_spacing,
                                  poisson_residual, poisson_rhs, poisson_solve,
                                  sor_four_colour_sweep, sor_lexicographic)


def _nodes(n):
    h = mesh_spacing(n)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")   # X[j, i] = x_i, Y[j, i] = y_j
    return h, X, Y


def _dense_solve(omega):
    """Assemble the compact system node by node and solve it densely.

    Unknowns: psi at interior nodes.  At a fixed point of eq. (SequationFinal)
    (5a/3) psi_P - A - C = B with the A, B, C, a, b, c of Sec. 3, b = c = 1/h^2.
    Wall psi are zero (Sec. 3.1) and drop out.
    """
    n = omega.shape[0]
    h = mesh_spacing(n)
    b = c = 1.0 / h**2
    a = b + c
    m = n - 2
    idx = lambda j, i: (j - 1) * m + (i - 1)
    M = np.zeros((m * m, m * m))
    r = np.zeros(m * m)
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            row = idx(j, i)
            coeffs = {
                (j, i): 5.0 * a / 3.0,
                (j, i + 1): -b + 2.0 * a / 12.0, (j, i - 1): -b + 2.0 * a / 12.0,
                (j + 1, i): -c + 2.0 * a / 12.0, (j - 1, i): -c + 2.0 * a / 12.0,
                (j + 1, i + 1): -a / 12.0, (j + 1, i - 1): -a / 12.0,
                (j - 1, i + 1): -a / 12.0, (j - 1, i - 1): -a / 12.0,
            }
            for (jj, ii), v in coeffs.items():
                if 1 <= jj <= n - 2 and 1 <= ii <= n - 2:
                    M[row, idx(jj, ii)] += v
            r[row] = (omega[j, i + 1] + omega[j + 1, i] + 8.0 * omega[j, i]
                      + omega[j, i - 1] + omega[j - 1, i]) / 12.0
    psi = np.zeros((n, n))
    psi[1:-1, 1:-1] = np.linalg.solve(M, r).reshape(m, m)
    return psi


@pytest.mark.parametrize("n", [5, 9, 12])
def test_dst_solve_matches_dense_brute_force(n):
    rng = np.random.default_rng(n)
    omega = rng.standard_normal((n, n))
    ref = _dense_solve(omega)
    got = poisson_solve(omega)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.all(got[0, :] == 0) and np.all(got[-1, :] == 0)
    assert np.all(got[:, 0] == 0) and np.all(got[:, -1] == 0)


@pytest.mark.parametrize("beta", [1.0, 1.5])
def test_dst_solve_matches_paper_lexicographic_relaxation(beta):
    n = 17
    rng = np.random.default_rng(7)
    omega = rng.standard_normal((n, n))
    ref, sweeps = sor_lexicographic(omega, beta, tol=1e-15)
    assert sweeps < 100000
    got = poisson_solve(omega)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(got))


def test_four_colour_relaxation_converges_to_same_solution():
    n = 17
    rng = np.random.default_rng(3)
    omega = rng.standard_normal((n, n))
    psi = np.zeros((n, n))
    for _ in range(400):
        psi = sor_four_colour_sweep(psi, omega, 1.6)
    got = poisson_solve(omega)
    assert np.max(np.abs(psi - got)) <= 1e-12 * np.max(np.abs(got))


@pytest.mark.parametrize("ny,nx,hgiven", [(9, 9, None), (7, 12, 0.05)])
def test_four_colour_sweep_is_pointwise_relaxation_in_colour_order(ny, nx, hgiven):
    """Brute force: loop node by node over the four groups, updating in place
    (also on a rectangular window with a given spacing)."""
    h = mesh_spacing(nx) if hgiven is None else hgiven
    b = c = 1.0 / h**2
    a = b + c
    rng = np.random.default_rng(11)
    omega = rng.standard_normal((ny, nx))
    psi0 = rng.standard_normal((ny, nx))
    if hgiven is None:
        psi0[0, :] = psi0[-1, :] = psi0[:, 0] = psi0[:, -1] = 0.0
    beta = 1.7
    P = psi0.copy()
    for (pi, pj) in ((0, 0), (1, 0), (0, 1), (1, 1)):
        for j in range(1, ny - 1):
            for i in range(1, nx - 1):
                if i % 2 != pi or j % 2 != pj:
                    continue
                A = b * (P[j, i + 1] + P[j, i - 1]) + c * (P[j + 1, i] + P[j - 1, i])
                B = (omega[j, i + 1] + omega[j + 1, i] + 8 * omega[j, i]
                     + omega[j, i - 1] + omega[j - 1, i]) / 12
                C = a / 12 * (P[j + 1, i + 1] - 2 * P[j + 1, i] + P[j + 1, i - 1]
                              - 2 * P[j, i + 1] - 2 * P[j, i - 1]
                              + P[j - 1, i + 1] - 2 * P[j - 1, i] + P[j - 1, i - 1])
                P[j, i] = 3 / 5 * beta / a * (A + B + C) + (1 - beta) * P[j, i]
    got = sor_four_colour_sweep(psi0, omega, beta, h=hgiven)
    assert np.max(np.abs(got - P)) <= 1e-13 * np.max(np.abs(P))


def test_windowed_sweeps_reproduce_full_grid_sweeps():
    """After k sweeps a node depends only on nodes within 4k of it (each of
    the four colour passes reaches one node further).  Sweeps on an
    even-aligned window with the full grid's spacing then give the full
    grid's values at the sample node; a window four nodes short of that reach
    does not, by far more than the tolerance (the reach is not overstated
    by much, so the check has teeth)."""
    n, k, beta = 121, 5, 1.7
    rng = np.random.default_rng(17)
    omega = rng.standard_normal((n, n))
    full = np.zeros((n, n))
    for _ in range(k):
        full = sor_four_colour_sweep(full, omega, beta)
    h = mesh_spacing(n)

    def windowed(j, i, rad):
        j0, i0 = max(0, (j - rad) // 2 * 2), max(0, (i - rad) // 2 * 2)
        j1, i1 = min(n, j + rad + 1), min(n, i + rad + 1)
        win = np.zeros((j1 - j0, i1 - i0))
        for _ in range(k):
            win = sor_four_colour_sweep(win, omega[j0:j1, i0:i1], beta, h=h)
        return win[j - j0, i - i0]

    for (j, i) in ((60, 60), (40, 2), (n - 3, n - 3), (1, 77)):
        assert abs(windowed(j, i, 4 * k + 4) - full[j, i]) <= 1e-13 * np.max(np.abs(full))
    assert abs(windowed(61, 61, 4 * k - 4) - full[61, 61]) > 1e-11 * np.max(np.abs(full))


def _poly_case(n, which):
    h, X, Y = _nodes(n)
    if which == "deg4":
        psi = X * (1 - X) * Y * (1 - Y)
        omega = 2.0 * (X * (1 - X) + Y * (1 - Y))          # -laplacian(psi)
    else:  # degree 5, no symmetry
        g = X * (1 - X) * Y * (1 - Y)
        s = X + 2 * Y
        # laplacian(g s) = s lap(g) + 2 grad g . grad s  (lap s = 0)
        lap_g = -2.0 * (Y * (1 - Y) + X * (1 - X))
        gx = (1 - 2 * X) * Y * (1 - Y)
        gy = X * (1 - X) * (1 - 2 * Y)
        psi = g * s
        omega = -(s * lap_g + 2.0 * (gx * 1.0 + gy * 2.0))
    return h, psi, omega


@pytest.mark.parametrize("which", ["deg4", "deg5"])
@pytest.mark.parametrize("n", [9, 33])
def test_polynomial_exactness(which, n):
    h, psi_exact, omega = _poly_case(n, which)
    got = poisson_solve(omega)
    assert np.max(np.abs(got - psi_exact)) <= 2e-14 * np.max(np.abs(psi_exact)) * n


def test_fourth_order_convergence_to_continuous_solution():
    errs = []
    ns = [17, 33, 65, 129]
    for n in ns:
        h, X, Y = _nodes(n)
        psi = np.sin(np.pi * X) * np.sin(np.pi * Y)
        omega = 2.0 * np.pi**2 * psi
        errs.append(np.max(np.abs(poisson_solve(omega) - psi)))
    orders = [np.log2(errs[k] / errs[k + 1]) for k in range(len(ns) - 1)]
    for p in orders:
        assert 3.9 < p < 4.1, (errs, orders)
    # second-order would be ~ (pi h)^2/12 ~ 3e-3 at n = 17: far above this
    assert errs[0] < 1e-5


@pytest.mark.parametrize("p,q", [(1, 1), (2, 5), (7, 3)])
def test_discrete_eigenfunction(p, q):
    n = 33
    h, X, Y = _nodes(n)
    mode = np.sin(p * np.pi * X) * np.sin(q * np.pi * Y)
    mode[0, :] = mode[-1, :] = mode[:, 0] = mode[:, -1] = 0.0
    # the operator applied node by node reproduces the closed-form eigenvalue
    lam = compact_eigenvalues(n)[q - 1, p - 1]
    applied = compact_operator(mode, h)
    assert np.max(np.abs(applied - lam * mode[1:-1, 1:-1])) <= 1e-12 * abs(lam)
    # B(mode) = beta_pq * mode with beta_pq = (8 + 2 c_p + 2 c_q)/12, so the
    # vorticity -lam/beta_pq * mode has exactly `mode` as its stream function.
    cp, cq = np.cos(p * np.pi * h), np.cos(q * np.pi * h)
    beta = (8 + 2 * cp + 2 * cq) / 12
    omega = -lam / beta * mode
    assert np.max(np.abs(poisson_rhs(omega) - beta * omega[1:-1, 1:-1])) <= 1e-12 * abs(lam)
    got = poisson_solve(omega)
    assert np.max(np.abs(got - mode)) <= 1e-13


def test_residual_of_solution_is_at_rounding_level():
    n = 65
    rng = np.random.default_rng(5)
    omega = rng.standard_normal((n, n))
    h = mesh_spacing(n)
    psi = poisson_solve(omega)
    r = poisson_residual(psi, omega, h)
    scale = np.max(np.abs(poisson_rhs(omega)))
    assert np.max(np.abs(r)) <= 1e-11 * scale


def test_default_relaxation_beats_both_classical_values():
    """The relaxation the library takes for converged solves, 5/8 of the way
    from the 5-point optimum 2/(1 + sin pi h) to Young's value for the
    compact operator's Jacobi radius mu = 0.8 cos pi h + 0.2 cos^2 pi h,
    needs fewer four-colour sweeps to reduce the residual 1e10 than either of
    them (the four-colour order of the 9-point stencil is not consistently
    ordered, so neither classical value is optimal)."""
    n = 65
    h = mesh_spacing(n)
    rng = np.random.default_rng(1)
    omega = np.zeros((n, n))
    omega[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    omega[-1, :] = -2.0 / h
    c = np.cos(np.pi * h)
    mu = 0.8 * c + 0.2 * c * c
    w5 = 2.0 / (1.0 + np.sin(np.pi * h))
    w9 = 2.0 / (1.0 + np.sqrt(1.0 - mu * mu))

    def sweeps(relax):
        p = np.zeros((n, n))
        r0 = np.max(np.abs(poisson_residual(p, omega, h)))
        for k in range(1, 5000):
            p = sor_four_colour_sweep(p, omega, relax)
            if np.max(np.abs(poisson_residual(p, omega, h))) <= 1e-10 * r0:
                return k
        return 5000

    k5, k9, km = sweeps(w5), sweeps(w9), sweeps(w5 - 0.625 * (w5 - w9))
    assert km < k5 and km < k9, (km, k5, k9)
