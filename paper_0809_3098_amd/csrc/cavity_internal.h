// Internal interface between the host runtime (cavity_runtime.cpp) and the
// HIP kernels (cavity_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cav {

// States of a Poisson solve, kept in device memory (PoissonCtl::state).
enum SolveState : int {
  SOLVE_RUN = 0,        // still sweeping
  SOLVE_CONVERGED = 1,  // residual max-norm <= tolerance
  SOLVE_FLOOR = 2,      // stagnated at the rounding floor above the tolerance
  SOLVE_NOCONV = 3,     // sweep limit reached
  SOLVE_NONFINITE = 4   // NaN or Inf met in the residual
};

// Device-resident control block of one cavity's Poisson solve.  Every sweep
// launch reads `state` first and returns at once unless it is SOLVE_RUN, so
// the host may enqueue more sweeps than needed without waiting.  The block
// that finishes a checking launch last (ticket) takes the decision.
struct alignas(128) PoissonCtl {
  unsigned long long rbits;   // max |g - psi| of the running check, as bits
  unsigned long long pbits;   // max |psi| of the running check, as bits
  unsigned int ticket;        // blocks of the running check that are done
  int state;                  // SolveState
  int phase;                  // 0 = over-relaxation, 1 = Gauss-Seidel polish
  int polish_left;            // polish checks still allowed
  double relax;               // relaxation parameter the next sweeps use
  double relax_sor;           // the over-relaxation value
  double tol_hat;             // tolerance in units of (g - psi)
  double best;                // best residual of the current phase
  double last;                // residual of the last check (units of g - psi)
  double psimax;              // max |psi| at the last check
  long long sweeps;           // sweeps done in this solve
  long long best_at;          // sweep count at which `best` was set
  long long max_sweeps;
  long long stall_window;     // sweeps without halving that mean stagnation
  long long sweeps_per_check; // sweeps between two checks
  int floor_limited;
  int pad0;
};

// Tile configuration of the temporally blocked four-colour sweep.
struct SorConfig {
  int tx, ty;      // output tile (nodes)
  int s;           // sweeps per launch
  int xcd_bands;   // 1: remap blocks so each XCD owns a band of tile rows
};

// ---- launches (all enqueue on `st`, return hipError_t) --------------------

// omega walls <- Thom(psi); corners <- 0.
hipError_t launch_thom(const double* psi, double* omega, int n, int pitch, double h,
                       double u_lid, hipStream_t st);

// F = 0.025 h^2 (w_E + w_W + w_N + w_S + 8 w_P) on interior nodes, 0 on walls.
hipError_t launch_poisson_rhs(const double* omega, double* F, int n, int pitch, double h,
                              hipStream_t st);

// Fused transport right-hand side and SSPRK stage combination on interior
// nodes:  out = a0*w0 + a1*win + ax*wx + b*L(win; psi);  walls of out <- win.
// With p_out != nullptr also  p_out = pa*wp + pb*win + pl*L(win; psi)
// (p_out may alias wp).  Null w0 / wx mean a0 / ax terms are absent.
struct StageArgs {
  double a0, a1, ax, b;       // out coefficients (b includes dt)
  double pa, pb, pl;          // p_out coefficients (pl includes dt)
  double nu, h;
};
hipError_t launch_stage(const double* psi, const double* w0, const double* win,
                        const double* wx, double* out, const double* wp, double* p_out,
                        int n, int pitch, const StageArgs& a, hipStream_t st);

// Reset a solve's control block (a kernel, so it can live in a graph).
hipError_t launch_ctl_reset(PoissonCtl* ctl, double relax, double tol_hat,
                            long long max_sweeps, long long stall_window,
                            long long sweeps_per_check, hipStream_t st);

// One launch of `cfg.s` four-colour sweeps, psi_in -> psi_out (ping-pong).
// check != 0: also the residual of the result and the solve decision.
hipError_t launch_sor64(const SorConfig& cfg, const double* psi_in, double* psi_out,
                        const double* F, int n, int pitch, PoissonCtl* ctl, int check,
                        hipStream_t st);
hipError_t launch_sor32(const SorConfig& cfg, const float* d_in, float* d_out, const float* R,
                        int n, int pitch, PoissonCtl* ctl, double relax, hipStream_t st);

// Mixed precision: FP64 residual r = g(psi) - psi into R32 (as float), zero
// d32, reduce max |r| and take the solve decision.
hipError_t launch_resid64(const double* psi, const double* F, float* R32, float* d32, int n,
                          int pitch, PoissonCtl* ctl, hipStream_t st);
// psi64 += d32 on interior nodes and count the inner sweeps (skipped once
// the solve has stopped).
hipError_t launch_refine(double* psi, const float* d32, int n, int pitch, PoissonCtl* ctl,
                         int inner_sweeps, hipStream_t st);

// Diagnostics: per-block partial sums, then a fixed-order final sum.
// out[0] = sum |psi1 - psi0|, out[1] = sum |w1 - w0|, out[2] = max |w1 - w0|,
// out[3] = sum over interior of u^2 + v^2.
hipError_t launch_diag(const double* psi0, const double* psi1, const double* w0,
                       const double* w1, int n, int pitch, double h, double* partial,
                       int npartial, double* out, hipStream_t st);
int diag_partials(int n);

// u, v from psi (eq. vel) with wall values; dense n*n outputs.
hipError_t launch_velocity(const double* psi, int n, int pitch, double h, double u_lid,
                           double* u, double* v, hipStream_t st);

// Pitched <-> dense copies and fills.
hipError_t launch_fill(double* a, int n, int pitch, double value, hipStream_t st);
hipError_t launch_fill32(float* a, int n, int pitch, float value, hipStream_t st);
hipError_t launch_copy_in(const double* dense, double* pitched, int n, int pitch,
                          hipStream_t st);
hipError_t launch_copy_out(const double* pitched, double* dense, int n, int pitch,
                           hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, int n, int pitch, hipStream_t st);
// interior nodes of dst <- src, walls of dst <- 0 (warm starts must have psi = 0 walls)
hipError_t launch_copy_interior(const double* src, double* dst, int n, int pitch,
                                hipStream_t st);

}  // namespace cav
