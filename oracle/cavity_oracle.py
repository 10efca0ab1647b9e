"""FP64 CPU oracle for the driven-lid-cavity time step.

TEST INFRASTRUCTURE ONLY.  Nothing on the GPU product path imports, calls or
links this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, tables or
helpers with the HIP library; both sides receive their inputs as plain arrays.

What it computes follows N. Cardoso and P. Bicudo, "Time dependent simulation
of the Driven Lid Cavity at High Reynolds Number" (arXiv:0809.3098):

* Sec. 2, eqs. (vort0), (stream0), (str), (vortfinal): vorticity-stream
  function form, u = psi_y, v = -psi_x, laplacian(psi) = -omega.
* Sec. 3, eq. (Lwn): central-difference right-hand side L(omega).
* Sec. 3, eqs. (SSPRK54_1)-(SSPRK54_5): the five-stage, fourth-order SSPRK
  integrator in Shu-Osher form.
* Sec. 3, eqs. (stream_4O), (SequationFinal) and the A, B, C, a, b, c
  definitions that follow it: the fourth-order compact stream equation.  The
  oracle does not iterate: it solves that linear system exactly (to rounding)
  by diagonalising the compact nine-point operator with the type-I discrete
  sine transform.  ``sor_lexicographic`` is the paper's relaxation written out
  for tiny grids, used only to show that both solve the same equations.
* Sec. 3, eq. (vel): velocities from psi.
* Sec. 3.1: wall conditions (psi = 0 on every wall) and Thom's formula for the
  wall vorticity.
* Sec. 3.2, eqs. (resS), (resV): the RES_psi and RES_omega monitors.

Grid convention: an n x n node array indexed ``[j, i]``; x_i = i*h (column
index, fastest), y_j = j*h (row index), h = 1/(n-1); walls at i or j equal to
0 and n-1; the moving lid is the top row j = n-1 (Sec. 3, driven-cavity
figure and boundary conditions).

Readings of the paper taken here:

* alpha_21 is printed as 0.555626506348765, which makes the stage-2
  coefficients sum to 0.999997; a Shu-Osher stage must be a convex combination
  summing to one, so alpha_21 = 1 - alpha_20 = 0.555629506348765.
* c_10 is printed to 11 digits; the value used is the one that satisfies the
  first-order condition given the other printed coefficients, to 15 digits:
  0.391752226571890.
* Stage order (the algorithm figure is missing): every stage combines interior
  nodes only; the new stage inherits the wall vorticity of the stage it was
  computed from, then psi is solved for the new vorticity and Thom's formula
  refreshes the walls.  This costs five Poisson solves per step.
* Corners: two Thom formulas meet there; no stencil reads a corner vorticity,
  so it is set to 0.
* n is the number of nodes per side including walls, so h = 1/(n-1).
* nu = |U| * L / Re with L = 1 (Sec. 3.2 parameter list).
* Time step: dt = cfl * h / |U| unless given.
* RES normalisation 1/N uses N = nodes per side, sum over all n^2 nodes.
* Kinetic energy (not in the paper): KE = 0.5 h^2 sum over interior (u^2+v^2).
"""

from __future__ import annotations

import numpy as np
import scipy.fft

__all__ = [
    "SSPRK54_PRINTED",
    "SSPRK54",
    "mesh_spacing",
    "poisson_rhs",
    "compact_operator",
    "compact_eigenvalues",
    "poisson_solve",
    "thom_walls",
    "velocity",
    "transport_rhs",
    "ssprk54_step",
    "sor_lexicographic",
    "sor_four_colour_sweep",
    "poisson_residual",
    "diagnostics",
    "CavityOracle",
]

# ---------------------------------------------------------------------------
# SSPRK(5,4) coefficients, Sec. 3, eqs. (SSPRK54_1)-(SSPRK54_5).
# Stage k:  y_k = sum_l alpha_kl y_l + dt * sum_l beta_kl L(y_l).
# ---------------------------------------------------------------------------

#: The coefficients exactly as printed in the paper.
SSPRK54_PRINTED = {
    "c10": 0.39175222657,
    "a20": 0.444370493651235, "a21": 0.555626506348765, "b21": 0.368410593050371,
    "a30": 0.620101851488403, "a32": 0.379898148511597, "b32": 0.251891774271694,
    "a40": 0.178079954393132, "a43": 0.821920045606868, "b43": 0.544974750228521,
    "a52": 0.517231671970585, "a53": 0.096059710526147, "b53": 0.063692468666290,
    "a54": 0.386708617503269, "b54": 0.226007483236906,
}

#: The coefficients used: the printed ones with the two readings applied
#: (alpha_21 = 1 - alpha_20; c_10 from the first-order condition).
SSPRK54 = dict(SSPRK54_PRINTED)
SSPRK54["a21"] = 0.555629506348765
SSPRK54["c10"] = 0.391752226571890


def mesh_spacing(n: int) -> float:
    """h = 1/(n-1) for n nodes per side on the unit square (Sec. 3.2)."""
    if n < 3:
        raise ValueError("need at least 3 nodes per side")
    return 1.0 / (n - 1)


# ---------------------------------------------------------------------------
# Compact fourth-order stream equation, Sec. 3, eq. (stream_4O) and
# eq. (SequationFinal) with its A, B, C, a, b, c (square grid: dx = dy = h).
# At a fixed point of the relaxation, psi = (3/(5a)) (A + B + C); rearranged,
#   A + C - (5a/3) psi = -B,
# and with b = c = 1/h^2, a = 2/h^2 the left side is the nine-point operator
#   (4 (E+W+N+S) + (NE+NW+SE+SW) - 20 P) / (6 h^2).
# ---------------------------------------------------------------------------

def poisson_rhs(omega: np.ndarray) -> np.ndarray:
    """B of Sec. 3 (the vorticity term of the relaxation formula) on interior nodes.

    B = (omega_E + omega_N + 8 omega_P + omega_W + omega_S) / 12.  Wall
    vorticity enters for nodes next to a wall; corners never do.
    Returns an (n-2, n-2) array.
    """
    w = omega
    return (w[1:-1, 2:] + w[2:, 1:-1] + 8.0 * w[1:-1, 1:-1]
            + w[1:-1, :-2] + w[:-2, 1:-1]) / 12.0


def compact_operator(psi: np.ndarray, h: float) -> np.ndarray:
    """A + C - (5a/3) psi of Sec. 3 on interior nodes (square grid).

    A = b (psi_E + psi_W) + c (psi_N + psi_S);
    C = (a/12) (psi_NE - 2 psi_N + psi_NW - 2 psi_E - 2 psi_W + psi_SE
                - 2 psi_S + psi_SW);
    written here term by term from those definitions with b = c = 1/h^2.
    """
    b = c = 1.0 / (h * h)
    a = b + c
    P = psi[1:-1, 1:-1]
    E, W = psi[1:-1, 2:], psi[1:-1, :-2]
    N, S = psi[2:, 1:-1], psi[:-2, 1:-1]
    NE, NW = psi[2:, 2:], psi[2:, :-2]
    SE, SW = psi[:-2, 2:], psi[:-2, :-2]
    A = b * (E + W) + c * (N + S)
    C = (a / 12.0) * (NE - 2.0 * N + NW - 2.0 * E - 2.0 * W + SE - 2.0 * S + SW)
    return A + C - (5.0 * a / 3.0) * P


def compact_eigenvalues(n: int) -> np.ndarray:
    """Eigenvalues of the compact operator on sin(p pi x) sin(q pi y), [q-1, p-1].

    For psi = sin(p pi x_i) sin(q pi y_j) (zero on the walls), with
    c_p = cos(p pi h): E+W+N+S = 2 (c_p + c_q) psi and NE+NW+SE+SW = 4 c_p c_q
    psi, so the operator returns lambda_pq psi with
    lambda_pq = (8 (c_p + c_q) + 4 c_p c_q - 20) / (6 h^2).
    """
    h = mesh_spacing(n)
    k = np.arange(1, n - 1, dtype=np.float64)
    cp = np.cos(k * np.pi * h)
    cx = cp[None, :]
    cy = cp[:, None]
    return (8.0 * (cx + cy) + 4.0 * cx * cy - 20.0) / (6.0 * h * h)


def poisson_solve(omega: np.ndarray, workers: int | None = None) -> np.ndarray:
    """Exact (to rounding) solution of the compact stream equation for psi.

    Solves  A + C - (5a/3) psi = -B(omega)  on interior nodes with psi = 0 on
    every wall (Sec. 3.1), i.e. the fixed point the relaxation of
    eq. (SequationFinal) converges to, for any relaxation parameter.  The
    operator is diagonal in the type-I sine basis, so
    psi_hat = -B_hat / lambda_pq.
    """
    n = omega.shape[0]
    if omega.shape != (n, n):
        raise ValueError("omega must be square")
    rhs = poisson_rhs(omega)
    lam = compact_eigenvalues(n)
    rh = scipy.fft.dstn(rhs, type=1, workers=workers)
    ph = -rh / lam
    inner = scipy.fft.idstn(ph, type=1, workers=workers)
    psi = np.zeros_like(omega, dtype=np.float64)
    psi[1:-1, 1:-1] = inner
    return psi


def poisson_residual(psi: np.ndarray, omega: np.ndarray, h: float) -> np.ndarray:
    """Residual A + B + C - (5a/3) psi of the compact equation (omega units)."""
    return compact_operator(psi, h) + poisson_rhs(omega)


# ---------------------------------------------------------------------------
# Boundary conditions, Sec. 3.1.
# ---------------------------------------------------------------------------

def thom_walls(omega: np.ndarray, psi: np.ndarray, h: float, u_lid: float) -> np.ndarray:
    """Return a copy of omega whose walls hold Thom's wall vorticity.

    Bottom (j = 0):    omega = -2 psi[1, i] / h^2
    Top, lid (j=n-1):  omega = -2 psi[n-2, i] / h^2 - 2 U / h
    Left (i = 0):      omega = -2 psi[j, 1] / h^2
    Right (i = n-1):   omega = -2 psi[j, n-2] / h^2
    Corners: 0 (two formulas meet there and no stencil reads them).
    On a square grid the paper's dx/dy labelling of these four lines is
    immaterial.
    """
    out = np.array(omega, dtype=np.float64, copy=True)
    h2 = h * h
    out[0, 1:-1] = -2.0 * psi[1, 1:-1] / h2
    out[-1, 1:-1] = -2.0 * psi[-2, 1:-1] / h2 - 2.0 * u_lid / h
    out[1:-1, 0] = -2.0 * psi[1:-1, 1] / h2
    out[1:-1, -1] = -2.0 * psi[1:-1, -2] / h2
    out[0, 0] = out[0, -1] = out[-1, 0] = out[-1, -1] = 0.0
    return out


def velocity(psi: np.ndarray, h: float, u_lid: float):
    """u, v on all nodes: eq. (vel) inside, wall values of Sec. 3.1 on walls.

    u = (psi[j+1,i] - psi[j-1,i]) / (2h),  v = -(psi[j,i+1] - psi[j,i-1]) / (2h)
    Walls: u = U on the lid nodes (corners excluded), 0 elsewhere; v = 0.
    """
    u = np.zeros_like(psi, dtype=np.float64)
    v = np.zeros_like(psi, dtype=np.float64)
    u[1:-1, 1:-1] = (psi[2:, 1:-1] - psi[:-2, 1:-1]) / (2.0 * h)
    v[1:-1, 1:-1] = -(psi[1:-1, 2:] - psi[1:-1, :-2]) / (2.0 * h)
    u[-1, 1:-1] = u_lid
    return u, v


def transport_rhs(omega: np.ndarray, psi: np.ndarray, h: float, nu: float) -> np.ndarray:
    """L(omega) of eq. (Lwn) on interior nodes, with u, v from eq. (vel).

    L = -u (w_E - w_W)/(2h) - v (w_N - w_S)/(2h)
        + nu ((w_E - 2 w_P + w_W)/h^2 + (w_N - 2 w_P + w_S)/h^2)
    Returns an (n-2, n-2) array.
    """
    u = (psi[2:, 1:-1] - psi[:-2, 1:-1]) / (2.0 * h)
    v = -(psi[1:-1, 2:] - psi[1:-1, :-2]) / (2.0 * h)
    wP = omega[1:-1, 1:-1]
    wE, wW = omega[1:-1, 2:], omega[1:-1, :-2]
    wN, wS = omega[2:, 1:-1], omega[:-2, 1:-1]
    adv = -u * (wE - wW) / (2.0 * h) - v * (wN - wS) / (2.0 * h)
    dif = nu * ((wE - 2.0 * wP + wW) / (h * h) + (wN - 2.0 * wP + wS) / (h * h))
    return adv + dif


# ---------------------------------------------------------------------------
# SSPRK(5,4) in Shu-Osher form, eqs. (SSPRK54_1)-(SSPRK54_5).
# ---------------------------------------------------------------------------

def ssprk54_step(y0, rhs, dt, combine, finish, coef=None):
    """One SSPRK(5,4) step, stage by stage as in eqs. (SSPRK54_1)-(SSPRK54_5).

    rhs(y)                 -> L(y)
    combine(ys, ks)        -> sum(a*y for a, y in ys) + sum(b*k for b, k in ks)
    finish(y_new, y_input) -> the stage value after any per-stage constraint
                              (identity for an ODE; Poisson + walls for the
                              cavity).
    L(omega^(3)) is evaluated once and used by both stage 4 and stage 5.
    """
    c = SSPRK54 if coef is None else coef
    k0 = rhs(y0)
    y1 = finish(combine([(1.0, y0)], [(c["c10"] * dt, k0)]), y0)
    k1 = rhs(y1)
    y2 = finish(combine([(c["a20"], y0), (c["a21"], y1)], [(c["b21"] * dt, k1)]), y1)
    k2 = rhs(y2)
    y3 = finish(combine([(c["a30"], y0), (c["a32"], y2)], [(c["b32"] * dt, k2)]), y2)
    k3 = rhs(y3)
    y4 = finish(combine([(c["a40"], y0), (c["a43"], y3)], [(c["b43"] * dt, k3)]), y3)
    k4 = rhs(y4)
    y5 = finish(combine([(c["a52"], y2), (c["a53"], y3), (c["a54"], y4)],
                        [(c["b53"] * dt, k3), (c["b54"] * dt, k4)]), y4)
    return y5


# ---------------------------------------------------------------------------
# Relaxation of eq. (SequationFinal), for cross-checks on tiny grids.
# ---------------------------------------------------------------------------

def sor_lexicographic(omega: np.ndarray, beta: float, psi0: np.ndarray | None = None,
                      tol: float = 1e-13, max_sweeps: int = 100000):
    """The paper's SOR for the compact stream equation, pure-Python loops.

    Eq. (SequationFinal): psi_new = (3/5)(beta/a)(A + B + C) + (1 - beta) psi_old
    with A, B, C evaluated using already-updated values at (i-1, .) and
    (i, j-1) and old values at (i+1, .) and (i, j+1): nodes are visited with
    i (x) in the outer loop and j (y) in the inner loop, updating in place.
    Stops when the largest change in a sweep is below ``tol`` times the
    largest |psi|.  For tiny grids only (n <= 33).
    Returns (psi, sweeps).
    """
    n = omega.shape[0]
    h = mesh_spacing(n)
    b = c = 1.0 / (h * h)
    a = b + c
    psi = np.zeros((n, n)) if psi0 is None else np.array(psi0, dtype=np.float64, copy=True)
    P = psi.tolist()          # P[j][i]
    W = np.asarray(omega, dtype=np.float64).tolist()
    for sweep in range(1, max_sweeps + 1):
        dmax = 0.0
        pmax = 0.0
        for i in range(1, n - 1):
            for j in range(1, n - 1):
                A = b * (P[j][i + 1] + P[j][i - 1]) + c * (P[j + 1][i] + P[j - 1][i])
                B = (W[j][i + 1] + W[j + 1][i] + 8.0 * W[j][i] + W[j][i - 1] + W[j - 1][i]) / 12.0
                C = (a / 12.0) * (P[j + 1][i + 1] - 2.0 * P[j + 1][i] + P[j + 1][i - 1]
                                  - 2.0 * P[j][i + 1] - 2.0 * P[j][i - 1]
                                  + P[j - 1][i + 1] - 2.0 * P[j - 1][i] + P[j - 1][i - 1])
                new = 0.6 * (beta / a) * (A + B + C) + (1.0 - beta) * P[j][i]
                d = abs(new - P[j][i])
                if d > dmax:
                    dmax = d
                P[j][i] = new
                if abs(new) > pmax:
                    pmax = abs(new)
        if dmax <= tol * max(pmax, 1e-300):
            return np.array(P), sweep
    return np.array(P), max_sweeps


def sor_four_colour_sweep(psi: np.ndarray, omega: np.ndarray, relax: float,
                          h: float | None = None) -> np.ndarray:
    """One relaxation sweep of eq. (SequationFinal) in four-colour order.

    The paper visits nodes lexicographically; a parallel machine cannot.  In
    the four-colour order, nodes are grouped by (i mod 2, j mod 2) and the
    groups are visited as (0,0), (1,0), (0,1), (1,1); no two nodes of a group
    share a nine-point stencil, so each group is updated from the values left
    by the groups before it.  Within one group every node receives the
    update of eq. (SequationFinal) with relaxation parameter ``relax``.  The
    fixed point is the same linear system's solution.  Returns a new array.

    ``h`` defaults to the spacing of an n x n grid of the unit square; giving
    it lets the sweep run on a window cut from a larger grid (the window's
    edge nodes are held fixed, and its origin must have even indices so that
    the colours are the global ones).
    """
    ny, nx = psi.shape
    if h is None:
        h = mesh_spacing(nx)
    b = c = 1.0 / (h * h)
    a = b + c
    p = np.array(psi, dtype=np.float64, copy=True)
    Bv = np.zeros((ny, nx))
    Bv[1:-1, 1:-1] = poisson_rhs(omega)
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    inner = (ii > 0) & (ii < nx - 1) & (jj > 0) & (jj < ny - 1)
    for (pi, pj) in ((0, 0), (1, 0), (0, 1), (1, 1)):
        m = inner & (ii % 2 == pi) & (jj % 2 == pj)
        js, is_ = np.nonzero(m)
        A = b * (p[js, is_ + 1] + p[js, is_ - 1]) + c * (p[js + 1, is_] + p[js - 1, is_])
        C = (a / 12.0) * (p[js + 1, is_ + 1] - 2.0 * p[js + 1, is_] + p[js + 1, is_ - 1]
                          - 2.0 * p[js, is_ + 1] - 2.0 * p[js, is_ - 1]
                          + p[js - 1, is_ + 1] - 2.0 * p[js - 1, is_] + p[js - 1, is_ - 1])
        p[js, is_] = 0.6 * (relax / a) * (A + Bv[js, is_] + C) + (1.0 - relax) * p[js, is_]
    return p


# ---------------------------------------------------------------------------
# Monitors, Sec. 3.2 eqs. (resS), (resV); kinetic energy (not in the paper).
# ---------------------------------------------------------------------------

def diagnostics(psi_old, psi_new, omega_old, omega_new, h, u_lid, dt):
    """RES_psi, RES_omega (eqs. resS/resV), max|d omega|/dt and kinetic energy."""
    n = psi_new.shape[0]
    res_psi = float(np.sum(np.abs(psi_new - psi_old)) / n)
    res_omega = float(np.sum(np.abs(omega_new - omega_old)) / n)
    domega = float(np.max(np.abs(omega_new - omega_old)) / dt)
    u, v = velocity(psi_new, h, u_lid)
    ke = float(0.5 * h * h * np.sum(u[1:-1, 1:-1] ** 2 + v[1:-1, 1:-1] ** 2))
    return {"res_psi": res_psi, "res_omega": res_omega,
            "domega_inf_over_dt": domega, "ke": ke}


# ---------------------------------------------------------------------------
# The time stepper.
# ---------------------------------------------------------------------------

class CavityOracle:
    """Driven-lid cavity integrated with SSPRK(5,4), exact Poisson per stage.

    Parameters follow Sec. 3.2: unit square, lid speed ``u_lid`` on the top
    wall, Re = |U| L / nu with L = 1.  ``omega0`` (n x n, walls included) is the
    initial vorticity (default zero); psi is solved from it and the walls are
    then set by Thom's formula, so the stored pair is always consistent.
    ``nu`` overrides the viscosity derived from Re (used for U = 0 tests).

    ``fixed_sweeps`` > 0 selects the coupled reading of eq. (SequationFinal):
    instead of solving the stream equation, every stage relaxes psi with
    exactly that many four-colour sweeps of parameter ``beta`` (Sec. 4 gives
    beta between 0.8 and 0.1), starting from the psi of the stage before it.
    ``beta`` defaults to 2 / (1 + sin(pi h)).  The initial psi is still the
    exact solution for ``omega0``.
    """

    def __init__(self, n: int, re: float, u_lid: float = 1.0, dt: float | None = None,
                 cfl: float = 0.5, omega0: np.ndarray | None = None,
                 nu: float | None = None, workers: int | None = None,
                 fixed_sweeps: int = 0, beta: float | None = None):
        self.n = int(n)
        self.h = mesh_spacing(self.n)
        self.u_lid = float(u_lid)
        self.re = float(re)
        self.nu = abs(self.u_lid) / self.re if nu is None else float(nu)
        if dt is None:
            if self.u_lid == 0.0:
                raise ValueError("dt must be given when u_lid == 0")
            dt = cfl * self.h / abs(self.u_lid)
        self.dt = float(dt)
        self.workers = workers
        self.fixed_sweeps = int(fixed_sweeps)
        self.beta = (2.0 / (1.0 + np.sin(np.pi * self.h))) if beta is None else float(beta)
        w = np.zeros((n, n)) if omega0 is None else np.array(omega0, dtype=np.float64, copy=True)
        self.psi = poisson_solve(w, workers)
        self.omega = thom_walls(w, self.psi, self.h, self.u_lid)
        self.t = 0.0
        self.steps = 0
        self.last_diag = None

    # stage helpers -------------------------------------------------------
    def _rhs(self, state):
        omega, psi = state
        return transport_rhs(omega, psi, self.h, self.nu)

    @staticmethod
    def _combine(ys, ks):
        omega = np.zeros_like(ys[0][1][0])
        acc = None
        for a, (w, _) in ys:
            term = a * w[1:-1, 1:-1]
            acc = term if acc is None else acc + term
        for bcoef, k in ks:
            acc = acc + bcoef * k
        omega[1:-1, 1:-1] = acc
        return omega

    def _finish(self, omega_new, state_in):
        w_in, _ = state_in
        w = omega_new
        # the new stage inherits the input stage's wall vorticity ...
        w[0, :] = w_in[0, :]
        w[-1, :] = w_in[-1, :]
        w[:, 0] = w_in[:, 0]
        w[:, -1] = w_in[:, -1]
        # ... psi is solved for it (or, in the coupled mode, relaxed from the
        # input stage's psi), then Thom refreshes the walls.
        if self.fixed_sweeps > 0:
            psi = state_in[1]
            for _ in range(self.fixed_sweeps):
                psi = sor_four_colour_sweep(psi, w, self.beta)
        else:
            psi = poisson_solve(w, self.workers)
        return (thom_walls(w, psi, self.h, self.u_lid), psi)

    def step(self, nsteps: int = 1, diagnostics_every: int = 0):
        """Advance ``nsteps`` SSPRK(5,4) steps; returns the last diagnostics."""
        for s in range(nsteps):
            state0 = (self.omega, self.psi)
            w1, p1 = ssprk54_step(state0, self._rhs, self.dt, self._combine, self._finish)
            if diagnostics_every and ((s + 1) % diagnostics_every == 0 or s + 1 == nsteps):
                self.last_diag = diagnostics(self.psi, p1, self.omega, w1, self.h,
                                             self.u_lid, self.dt)
            self.omega, self.psi = w1, p1
            self.steps += 1
            self.t += self.dt
        return self.last_diag

    def fields(self):
        """psi, omega, u, v (copies), all n x n indexed [j, i]."""
        u, v = velocity(self.psi, self.h, self.u_lid)
        return self.psi.copy(), self.omega.copy(), u, v
