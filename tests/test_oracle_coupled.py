"""Pins of the oracle's coupled mode: a fixed number of relaxation sweeps of
eq. (SequationFinal) per stage instead of a solve of the stream equation.

* In the limit of many over-relaxed sweeps the coupled step is the solved
  step (the relaxation's fixed point is the compact equation's solution).
* A few under-relaxed sweeps per stage, checked against the same step built
  here from a dense-matrix statement of the four-colour relaxation (the
  compact operator assembled column by column from unit vectors, each colour
  updated as one projected Richardson step), warm-started from the psi of
  the stage before, as the coupled reading prescribes.
* Mirror symmetry (U -> -U reflects x -> 1 - x) holds for odd n, where the
  reflection maps every colour class onto itself.
"""
import numpy as np

from oracle.cavity_oracle import (CavityOracle, compact_operator, mesh_spacing, poisson_rhs,
                                  ssprk54_step, thom_walls, transport_rhs)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_many_sweeps_reach_the_solved_step():
    n, re, steps = 17, 100.0, 6
    solved = CavityOracle(n, re)
    solved.step(steps)
    coupled = CavityOracle(n, re, fixed_sweeps=150)
    coupled.step(steps)
    assert _rel(coupled.psi, solved.psi) < 1e-12
    assert _rel(coupled.omega, solved.omega) < 1e-12
    few = CavityOracle(n, re, fixed_sweeps=1, beta=0.5)
    few.step(steps)
    assert _rel(few.psi, solved.psi) > 1e-4  # the coupled mode is a different scheme


def _dense_sweeps(psi, omega, beta, sweeps):
    """Four-colour relaxation as dense linear algebra on the interior unknowns."""
    n = psi.shape[0]
    h = mesh_spacing(n)
    m = n - 2
    M = np.zeros((m * m, m * m))
    for k in range(m * m):
        e = np.zeros((n, n))
        e[1:-1, 1:-1].flat[k] = 1.0
        M[:, k] = compact_operator(e, h).ravel()
    rhs = poisson_rhs(omega).ravel()
    jj, ii = np.meshgrid(np.arange(1, n - 1), np.arange(1, n - 1), indexing="ij")
    scale = beta * 3.0 / (5.0 * (2.0 / (h * h)))   # beta * 3 / (5 a), a = 2 / h^2
    x = psi[1:-1, 1:-1].ravel().copy()
    for _ in range(sweeps):
        for ci, cj in ((0, 0), (1, 0), (0, 1), (1, 1)):
            sel = ((ii % 2 == ci) & (jj % 2 == cj)).ravel()
            x = x + np.where(sel, scale * (M @ x + rhs), 0.0)
    out = np.zeros((n, n))
    out[1:-1, 1:-1] = x.reshape(m, m)
    return out


def test_coupled_step_matches_dense_statement():
    n, re, steps, sweeps, beta = 7, 50.0, 3, 2, 0.7
    o = CavityOracle(n, re, fixed_sweeps=sweeps, beta=beta)
    h, U, nu, dt = o.h, o.u_lid, o.nu, o.dt
    state = (o.omega.copy(), o.psi.copy())

    def rhs(y):
        return transport_rhs(y[0], y[1], h, nu)

    def combine(ys, ks):
        w = np.zeros_like(ys[0][1][0])
        inner = sum(a * y[0][1:-1, 1:-1] for a, y in ys) + sum(b * k for b, k in ks)
        w[1:-1, 1:-1] = inner
        return w

    def finish(w_new, y_in):
        w = w_new.copy()
        edge = np.ones((n, n), bool)
        edge[1:-1, 1:-1] = False
        w[edge] = y_in[0][edge]            # walls carried from the input stage
        psi = _dense_sweeps(y_in[1], w, beta, sweeps)
        return (thom_walls(w, psi, h, U), psi)

    for _ in range(steps):
        state = ssprk54_step(state, rhs, dt, combine, finish)
    o.step(steps)
    assert _rel(o.psi, state[1]) < 1e-13
    assert _rel(o.omega, state[0]) < 1e-13


def test_coupled_mirror_symmetry_odd_n():
    n, re, steps = 15, 400.0, 5
    a = CavityOracle(n, re, u_lid=1.0, fixed_sweeps=3, beta=0.5)
    b = CavityOracle(n, re, u_lid=-1.0, fixed_sweeps=3, beta=0.5)
    a.step(steps)
    b.step(steps)
    assert np.max(np.abs(b.psi + a.psi[:, ::-1])) <= 1e-13 * np.max(np.abs(a.psi))
    assert np.max(np.abs(b.omega + a.omega[:, ::-1])) <= 1e-13 * np.max(np.abs(a.omega))
