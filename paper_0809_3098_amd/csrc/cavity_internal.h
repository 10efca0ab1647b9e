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
// the host may enqueue more sweeps than needed without waiting.  A checking
// launch leaves per-block maxima; a one-block decision kernel that follows it
// on the stream (or a block of the batched kernel after a grid barrier)
// reduces them and takes the decision.
struct alignas(128) PoissonCtl {
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
  double floor_ulps;          // > 0: a residual within this many ulps of max |psi| is the
                              // rounding floor and stops the solve (floor-limited)
  int gs_open;                // 1: relax with 1 (Gauss-Seidel) until the first check
  int floor_limited;
  int werror;                 // 1: a wait of a resident solve timed out
  // Totals over every solve since the handle was created (never reset by a
  // solve), read by the host once per call.
  long long total_sweeps;
  int total_floor;            // solves that stopped at the rounding floor
  int total_noconv;           // solves that hit the sweep limit
  int total_nonfinite;        // solves that met NaN / Inf
  int total_solves;
};

// One cavity of a persistent batched solve (device-resident descriptor).
struct BatchMember {
  double* psi;
  double* psi_b;
  const double* F;
  PoissonCtl* ctl;
  double* part;        // two doubles per tile
  float* R32;
  float* d32a;
  float* d32b;
  int n, pitch;
  int tiles_x, tiles;  // tiles of this cavity in the batch's tile shape
  int tile0;           // first tile of this cavity in the batch tile list
  int pad;
};

// Grid barrier state and error flag of the persistent kernels.  Barrier
// generations only grow, across launches too: `epoch` is the generation the
// last launch ended with, `go` the last generation released by block 0.
// Arrival flags live in a separate array, one 128-byte line per block.
struct alignas(128) BatchCtl {
  unsigned int epoch;
  unsigned int go;
  int error;           // 1: a barrier wait timed out (blocks not co-resident)
  int pad;
};
constexpr int kMaxBatchGrid = 4096;        // blocks of a persistent launch
constexpr int kFlagStride = 32;            // words between two arrival flags

// Decision exchange of a resident solve (one per cavity).  Slot c % 2 holds
// the decision of residual check c once tag[c % 2] == c + 1.
struct alignas(128) ResidentCtl {
  unsigned int tag[2];
  int state[2];
  double relax[2];
  int error;           // 1: a wait timed out (blocks not co-resident)
  int pad;
};

// Tile configuration of the temporally blocked four-colour sweep.
struct SorConfig {
  int tx, ty;      // output tile (nodes)
  int s;           // sweeps per launch
  int nt;          // threads per block
  int xcd_bands;   // 1: remap blocks so each XCD owns a band of tile rows
};

// Whether (tx, ty, s, nt) is one of the compiled sweep kernels.
bool sor_config_supported(const SorConfig& c, bool fp32);
// Whether a resident solve exists for this tile shape and fits the device
// with one co-resident block per tile.
bool resident_supported(const SorConfig& c, int n, int device);
// Arrival flags of a resident solve: one 128-byte line per tile.
size_t resident_flag_bytes(int n);
// Upper bound on the blocks of any sweep launch (smallest tile) and of the
// residual kernel: sizes the partial-maximum array.
int sor_max_blocks(int n);
int resid_blocks(int n);

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
// psi32 != nullptr: L is evaluated in FP32 from that shadow of psi (mixed).
hipError_t launch_stage(const double* psi, const float* psi32, const double* w0,
                        const double* win, const double* wx, double* out, const double* wp,
                        double* p_out, int n, int pitch, const StageArgs& a, hipStream_t st);

// Reset a solve's control block (a kernel, so it can live in a graph).
// gs_steps: if not null and at least two steps are on file there (the count of
// an extrapolated warm start), the solve opens with Gauss-Seidel sweeps
// (relaxation 1) and switches to `relax` at its first check after a sweep.
hipError_t launch_ctl_reset(PoissonCtl* ctl, double relax, double tol_hat,
                            long long max_sweeps, long long stall_window,
                            long long sweeps_per_check, hipStream_t st, double floor_ulps = 0.0,
                            const long long* gs_steps = nullptr);

// One launch of `cfg.s` four-colour sweeps, psi_in -> psi_out (ping-pong).
// check != 0: also the residual of the result and the solve decision.
// `part` holds two doubles per block for the check's partial maxima.
hipError_t launch_sor64(const SorConfig& cfg, const double* psi_in, double* psi_out,
                        const double* F, int n, int pitch, PoissonCtl* ctl, double* part,
                        int check, hipStream_t st);
hipError_t launch_sor32(const SorConfig& cfg, const float* d_in, float* d_out, const float* R,
                        int n, int pitch, PoissonCtl* ctl, double relax, hipStream_t st);
// A whole FP64 solve in one launch, one block per tile kept resident: tiles
// exchange halos through psi / psi_b with their neighbours each round of S
// sweeps; every rounds_per_check rounds the tile residuals are reduced and
// block 0 decides (the decision takes effect two rounds later).  The result
// ends in psi.  flags and rctl are cleared by this call; part needs 4 doubles
// per tile.  Fails with hipErrorInvalidConfiguration when the tiles cannot be
// co-resident.
hipError_t launch_sor64_resident(const SorConfig& cfg, double* psi, double* psi_b,
                                 const double* F, int n, int pitch, PoissonCtl* ctl,
                                 double* part, unsigned int* flags, ResidentCtl* rctl,
                                 int rounds_per_check, long long spin_ticks, int device,
                                 hipStream_t st);

// Persistent batched solves: every member's Poisson solve runs in one launch;
// blocks sweep the batch's tile list round by round with grid barriers in
// between and decide each member's stop in device memory.  The grid must be
// co-resident (see batch_grid); barrier waits are bounded by spin_ticks of the
// 100 MHz wall clock and set BatchCtl::error when exceeded.
// FP64: pairs_per_check launch-pairs of cfg.s sweeps between checks.
hipError_t launch_batch64(const SorConfig& cfg, const BatchMember* mem, int count,
                          int total_tiles, int pairs_per_check, BatchCtl* bc,
                          unsigned int* flags, int grid, long long spin_ticks, hipStream_t st);
// Mixed: rounds of FP64 residual, inner_pairs FP32 launch-pairs (the last
// pair Gauss-Seidel) and FP64 refinement.
hipError_t launch_batch_mixed(const SorConfig& cfg32, const BatchMember* mem, int count,
                              int total_tiles, int inner_pairs, BatchCtl* bc,
                              unsigned int* flags, int grid, long long spin_ticks,
                              hipStream_t st);
// Largest co-resident grid for the batched kernel of this configuration.
int batch_grid(const SorConfig& cfg, bool mixed, int device);
bool batch_config_supported(const SorConfig& cfg, bool mixed);

// Mixed precision: FP64 residual r = g(psi) - psi into R32 (as float), zero
// d32, reduce max |r| and take the solve decision.
// sweeps_done: sweeps since the previous check, added to the solve's count.
hipError_t launch_resid64(const double* psi, const double* F, float* R32, float* d32, int n,
                          int pitch, PoissonCtl* ctl, double* part, hipStream_t st,
                          long long sweeps_done = 0);

// Multigrid: residual in vorticity units, restriction to the next coarser
// level (also zeroing its iterate), prolongation-and-correct, and a sweep
// launch with an explicit relaxation parameter (no residual check).
// (FP64 for the FP64 solver; FP32 for the correction cycles of mixed mode.)
hipError_t launch_mg_residual(const double* psi, const double* F, double* r, int n, int pitch,
                              double h, const PoissonCtl* ctl, hipStream_t st);
hipError_t launch_mg_residual(const float* psi, const float* F, float* r, int n, int pitch,
                              double h, const PoissonCtl* ctl, hipStream_t st);
hipError_t launch_mg_restrict(const double* r, int nf, int pitchf, double* Fc, double* Ec,
                              double* Ecb, int nc, int pitchc, const PoissonCtl* ctl,
                              hipStream_t st);
hipError_t launch_mg_restrict(const float* r, int nf, int pitchf, float* Fc, float* Ec,
                              float* Ecb, int nc, int pitchc, const PoissonCtl* ctl,
                              hipStream_t st);
hipError_t launch_mg_prolong(const double* Ec, int nc, int pitchc, double* psi, int nf,
                             int pitchf, const PoissonCtl* ctl, hipStream_t st);
hipError_t launch_mg_prolong(const float* Ec, int nc, int pitchc, float* psi, int nf,
                             int pitchf, const PoissonCtl* ctl, hipStream_t st);
// The coarse end of a V-cycle in one block: levels n[0] > n[1] > ... (the
// first with at most mg_fuse_max() nodes a side, down to the coarsest), nu
// smoothing sweeps (relaxation 1) before and after each coarse correction,
// coarse_sweeps sweeps with coarse_relax on the coarsest level; E (in and out,
// interior written) and F are level n[0]'s pitched arrays.  Same arithmetic,
// so the same bits, as the per-level launches.
int mg_fuse_max();
hipError_t launch_mg_fused(double* E, const double* F, int pitch, const int* n, int levels,
                           int nu, int coarse_sweeps, double coarse_relax, const PoissonCtl* ctl,
                           hipStream_t st);
hipError_t launch_mg_fused(float* E, const float* F, int pitch, const int* n, int levels, int nu,
                           int coarse_sweeps, double coarse_relax, const PoissonCtl* ctl,
                           hipStream_t st);
hipError_t launch_sor64_relax(const SorConfig& cfg, const double* psi_in, double* psi_out,
                              const double* F, int n, int pitch, PoissonCtl* ctl, double relax,
                              hipStream_t st);
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
// Zero `bytes` (a multiple of 4) with a kernel (graph-safe, unlike memset).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
// b = (float)a over the whole pitched array.
hipError_t launch_shadow(const double* a, float* b, int n, int pitch, hipStream_t st);
hipError_t launch_copy_in(const double* dense, double* pitched, int n, int pitch,
                          hipStream_t st);
hipError_t launch_copy_out(const double* pitched, double* dense, int n, int pitch,
                           hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, int n, int pitch, hipStream_t st);
// interior nodes of dst <- src, walls of dst <- 0 (warm starts must have psi = 0 walls)
hipError_t launch_copy_interior(const double* src, double* dst, int n, int pitch,
                                hipStream_t st);

// Start of a stage's Poisson solve extrapolated from the same stage of the last
// `levels` steps (2 <= levels <= 8), after filing the previous stage's psi in
// the history (5 * levels pitched fields, fstride doubles apart); *count =
// steps completed since the history was emptied, advanced by launch_warm_tick.
// wtab: device table, row L (kWarmCols doubles) = the weights for L steps on file.
constexpr int kWarmCols = 8;
hipError_t launch_warm(double* psi, double* hist, size_t fstride, int n, int pitch, int stage,
                       int levels, const long long* count, const double* wtab, hipStream_t st);
hipError_t launch_warm_tick(long long* count, hipStream_t st);

// Allocation-free Poisson solve: the largest grid it takes, the size of its
// device scratch array, and that array's address on the current device
// (looked up with hipGetSymbolAddress on the first call per device).
int noalloc_max_n();
size_t noalloc_bytes();
hipError_t noalloc_scratch(void** out);

}  // namespace cav
