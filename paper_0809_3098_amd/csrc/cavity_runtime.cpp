// Host runtime and C ABI of the driven-lid-cavity time stepper.
//
// Sequencing of a time step (N. Cardoso and P. Bicudo, arXiv:0809.3098,
// Sec. 3): five SSPRK(5,4) stages (eqs. SSPRK54_1-5).  Each stage
//   1. evaluates L(omega) of eq. (Lwn) with u, v of eq. (vel) and forms the
//      stage's interior vorticity; the stage keeps the wall vorticity of the
//      stage it was computed from;
//   2. assembles the right-hand side of the compact stream equation and
//      relaxes psi by four-colour SOR (eq. SequationFinal) until the residual
//      max-norm is below the tolerance;
//   3. refreshes the wall vorticity from psi by Thom's formula (Sec. 3.1).
// The work is enqueued on one HIP stream.  A Poisson solve's stopping
// decision lives in device memory, so sweeps are enqueued in chunks and the
// host only reads the decision once per chunk.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/cavity.h"
#include "cavity_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// SSPRK(5,4) Shu-Osher coefficients, Sec. 3 eqs. (SSPRK54_1)-(SSPRK54_5).
// alpha_21 is printed as 0.555626506348765, which leaves the stage-2
// coefficients summing to 0.999997; a Shu-Osher stage is a convex
// combination, so alpha_21 = 1 - alpha_20 is used.  c_10 is printed to 11
// digits; the 15-digit value satisfying the first-order condition with the
// other coefficients is used.
constexpr double kC10 = 0.391752226571890;
constexpr double kA20 = 0.444370493651235, kA21 = 0.555629506348765, kB21 = 0.368410593050371;
constexpr double kA30 = 0.620101851488403, kA32 = 0.379898148511597, kB32 = 0.251891774271694;
constexpr double kA40 = 0.178079954393132, kA43 = 0.821920045606868, kB43 = 0.544974750228521;
constexpr double kA52 = 0.517231671970585, kA53 = 0.096059710526147, kB53 = 0.063692468666290;
constexpr double kA54 = 0.386708617503269, kB54 = 0.226007483236906;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// One level of the multigrid hierarchy (level 0 is the cavity's own grid).
struct MgLevel {
  int n = 0, pitch = 0;
  double h = 0;
  double* E = nullptr;   // iterate (level 0: psi)
  double* Eb = nullptr;  // ping-pong partner (level 0: psi_b)
  double* F = nullptr;   // right-hand side, pre-scaled by 0.3 h^2
  double* r = nullptr;   // residual in vorticity units (not on the coarsest level)
};

// FP32 counterpart for the correction cycles of mixed precision (level 0:
// E = d32a, Eb = d32b, F = R32).
struct MgLevel32 {
  int n = 0, pitch = 0;
  double h = 0;
  float* E = nullptr;
  float* Eb = nullptr;
  float* F = nullptr;
  float* r = nullptr;
};

constexpr int kMgCoarsest = 9;     // levels stop at n <= 9
constexpr int kMgCoarseSweeps = 24;  // relaxation sweeps on the coarsest level
constexpr double kMgCoarseRelax = 1.5;

struct Member {
  cavity_params p{};
  int n = 0, pitch = 0;
  bool mixed = false;
  double h = 0, nu = 0, dt = 0, u_lid = 0, tol = 0, relax = 0;
  long long max_sweeps = 0, stall_window = 0;
  // device fields (pitched)
  double* w[4] = {nullptr, nullptr, nullptr, nullptr};  // w[0] = omega^n
  double* psi = nullptr;       // current psi (solve result always lands here)
  double* psi_b = nullptr;     // ping-pong partner
  double* psi_prev = nullptr;  // psi^n for the monitors; scratch between steps
  double* F = nullptr;
  float* R32 = nullptr;
  float* d32a = nullptr;
  float* d32b = nullptr;
  float* psi32 = nullptr;      // mixed: FP32 shadow of psi for the transport stencil
  cav::PoissonCtl* ctl = nullptr;
  double* part = nullptr;      // per-block partial maxima of a residual check
  unsigned int* rflags = nullptr;     // resident solve: per-tile round flags
  cav::ResidentCtl* rctl = nullptr;   // resident solve: decision exchange
  double* diag_partial = nullptr;
  double* diag_out = nullptr;
  int diag_np = 0;
  cav::SorConfig cfg64{64, 64, 2, 1024, 0};
  cav::SorConfig cfg32{64, 64, 2, 1024, 0};
  int pairs_per_check = 1;  // FP64: launch pairs between residual checks
  int inner_sweeps = 0;     // mixed: FP32 sweeps per refinement round
  int solver = CAVITY_SOLVER_SOR;
  int fixed = 0;            // > 0: sweeps per stage solve of the coupled mode
  // Start of each stage's solve: 1 = the previous stage's psi; >= 2 = the
  // extrapolation through that many steps' solutions of the same stage, kept
  // in hist (5 * warm pitched fields, hist_stride doubles apart; stage k's
  // slot r at (k - 1) * warm + r) with the count of steps on file in warm_cnt.
  int warm = 1;
  int warm_deg = 0;          // degree of the polynomial through the warm steps on file
  double* hist = nullptr;
  size_t hist_stride = 0;
  long long* warm_cnt = nullptr;
  double* warm_w = nullptr;  // device: row L = weights for L steps on file (L <= warm)
  std::vector<MgLevel> mg;  // multigrid hierarchy (allocated for every cavity)
  std::vector<MgLevel32> mg32;  // FP32 hierarchy (mixed cavities)
  // host-side state
  long long step = 0;
  double t = 0;
  long long sweeps_total = 0, sweeps_step = 0;
  double est_sweeps = 0;  // running estimate of sweeps per solve
  // sweeps of the last solve of each stage of a step (index 1..5): a stage's
  // count repeats from step to step far better than consecutive stages'
  double est_stage[6] = {0, 0, 0, 0, 0, 0};
  int floor_step = 0;
  int status_step = CAVITY_OK;
  double last_resid = 0;
};

// Forget the sweep estimates (a new schedule or relaxation changes them).
void reset_estimates(Member& m) {
  m.est_sweeps = 0;
  for (double& e : m.est_stage) e = 0;
}

}  // namespace

struct cavity_s {
  int count = 0;
  int device = 0;
  hipStream_t st = nullptr;
  bool poisoned = false;
  std::vector<Member> m;
  cav::PoissonCtl* host_ctl = nullptr;  // pinned readback of every member's ctl
  double* host_diag = nullptr;          // pinned readback, 4 per member
  // ---- execution of the Poisson solves
  int exec = CAVITY_EXEC_STREAM;
  bool mixed = false;                   // batch precision (all members agree)
  cav::SorConfig bcfg64{64, 64, 3, 768, 0};
  cav::SorConfig bcfg32{64, 64, 4, 1024, 0};
  int b_ppc = 1;                        // FP64: launch-pairs per check
  int b_inner_pairs = 1;                // mixed: FP32 launch-pairs per round
  int total_tiles = 0;
  int grid = 0;
  cav::BatchMember* d_mem = nullptr;    // device descriptors (workspace)
  cav::BatchCtl* d_bc = nullptr;        // grid barrier (workspace)
  unsigned int* d_flags = nullptr;      // grid-barrier arrival flags (workspace)
  cav::BatchCtl* host_bc = nullptr;     // pinned readback
  std::vector<cav::BatchMember> h_mem;
  std::vector<cav::PoissonCtl> last_tot;  // totals at the previous readback
  double* w0_base = nullptr;            // member 0's initial w[0]: step parity
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipStream_t cap_st = nullptr;         // private stream graphs are recorded on
  // Concurrent stream steps of several cavities: one stream per cavity
  // (default priority), forked from and joined back to st by events.  While
  // `fanned` is set, each cavity's work goes to its own stream.
  std::vector<hipStream_t> mst;
  std::vector<hipEvent_t> mev;
  hipEvent_t fork_ev = nullptr;
  bool fanned = false;
};

namespace {

#define HIP_TRY(h, expr)                                                         \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      if (h) (h)->poisoned = true;                                               \
      return fail(CAVITY_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    }                                                                            \
  } while (0)

// The stream cavity k's work goes to: its own while a step is fanned out,
// else the handle's.
hipStream_t member_stream(const cavity_s* h, int k) { return h->fanned ? h->mst[k] : h->st; }

// Enqueues made in its lifetime go to stream s (every enqueue helper uses
// h->st).
struct StreamScope {
  cavity_s* h;
  hipStream_t saved;
  StreamScope(cavity_s* h_, hipStream_t s) : h(h_), saved(h_->st) { h->st = s; }
  ~StreamScope() { h->st = saved; }
};

// Row pitch of every field, in nodes: a multiple of 32, so even and, for odd
// n, at least n + 1 (the sweep kernels load node pairs x, x + 1 with x even).
int pitch_of(int n) { return (n + 31) / 32 * 32; }

// Residual-check spacing (FP64) and inner sweeps per refinement round
// (mixed), rounded to whole launch pairs of the current kernels.
void set_schedule(Member& m, int check_every, int inner) {
  const int u64 = 2 * m.cfg64.s;
  m.pairs_per_check = std::max(1, (check_every + u64 - 1) / u64);
  const int u32 = 2 * m.cfg32.s;
  m.inner_sweeps = std::max(u32, (inner + u32 - 1) / u32 * u32);
}

// Validation and derived quantities (Sec. 3.2: Re = |U| L / nu, L = 1).
int derive(const cavity_params& p, Member& m) {
  if (p.n < 5 || p.n > 16385) return fail(CAVITY_EINVAL, "n = %d outside [5, 16385]", p.n);
  if (p.resume != 0 && p.resume != 1) return fail(CAVITY_EINVAL, "resume must be 0 or 1");
  if (p.resume && (!p.omega0 || !p.psi0))
    return fail(CAVITY_EINVAL, "resume = 1 needs both omega0 and psi0");
  if (p.precision != CAVITY_FP64 && p.precision != CAVITY_MIXED)
    return fail(CAVITY_EINVAL, "precision = %d is not CAVITY_FP64 or CAVITY_MIXED", p.precision);
  if (p.warm_start < 0 || p.warm_start > CAVITY_WARM_LEVELS_MAX)
    return fail(CAVITY_EINVAL, "warm_start = %d outside [0, %d]", p.warm_start,
                CAVITY_WARM_LEVELS_MAX);
  if (p.fixed_sweeps > 0 && p.warm_start > CAVITY_WARM_PREVIOUS)
    return fail(CAVITY_EINVAL, "warm_start extrapolation needs converged solves "
                               "(fixed_sweeps = 0)");
  if (p.fixed_sweeps < 0 || p.fixed_sweeps > (1 << 24))
    return fail(CAVITY_EINVAL, "fixed_sweeps = %d outside [0, 2^24]", p.fixed_sweeps);
  if (p.fixed_sweeps > 0 && p.precision != CAVITY_FP64)
    return fail(CAVITY_EINVAL, "fixed_sweeps needs precision CAVITY_FP64");
  const double vals[] = {p.re, p.u_lid, p.nu, p.dt, p.cfl, p.poisson_tol, p.sor_omega};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(CAVITY_EINVAL, "non-finite parameter");
  m.p = p;
  m.n = p.n;
  m.pitch = pitch_of(p.n);
  m.mixed = p.precision == CAVITY_MIXED;
  m.h = 1.0 / (p.n - 1);
  m.u_lid = p.u_lid;
  if (p.nu > 0) {
    m.nu = p.nu;
  } else {
    if (!(p.re > 0)) return fail(CAVITY_EINVAL, "re must be > 0 (got %g)", p.re);
    m.nu = std::fabs(p.u_lid) / p.re;
  }
  if (p.dt > 0) {
    m.dt = p.dt;
  } else {
    if (p.u_lid == 0) return fail(CAVITY_EINVAL, "dt must be > 0 when u_lid == 0");
    const double cfl = p.cfl > 0 ? p.cfl : 0.5;
    m.dt = cfl * m.h / std::fabs(p.u_lid);
  }
  m.fixed = p.fixed_sweeps;
  m.warm = p.warm_start != CAVITY_WARM_DEFAULT ? p.warm_start
           : p.fixed_sweeps > 0              ? CAVITY_WARM_PREVIOUS
           : p.precision == CAVITY_MIXED     ? CAVITY_WARM_LEVELS_MIXED
                                             : CAVITY_WARM_LEVELS_FP64;
  // FP64: the interpolating polynomial; mixed: a least-squares fit of degree at
  // most 5 (1024^2, Re 3e4, 1000 steps: 95.7 Mcell-steps/s with 8 steps and
  // degree 5, 93.1 with degree 4, 85.4 interpolating 6 steps, 60.3 with degree
  // 3; in FP64 the fits were slower: 25.9 with 8 steps and degree 5 against
  // 30.5 interpolating 7)
  m.warm_deg = m.warm < 2 ? 0 : m.mixed ? std::min(m.warm - 1, (int)CAVITY_WARM_DEGREE_MIXED)
                                        : m.warm - 1;
  m.tol = p.poisson_tol > 0 ? p.poisson_tol : 1e-10;
  m.max_sweeps = p.poisson_max_sweeps > 0 ? p.poisson_max_sweeps : 200LL * p.n;
  if (p.sor_omega > 0) {
    if (!(p.sor_omega < 2.0)) return fail(CAVITY_EINVAL, "sor_omega must lie in (0, 2)");
    m.relax = p.sor_omega;
  } else if (p.fixed_sweeps > 0) {
    // the coupled mode takes its parameter literally; unset, the classical
    // optimum for the 5-point operator (the oracle's default too)
    m.relax = 2.0 / (1.0 + std::sin(M_PI * m.h));
  } else {
    // Converged solves, where the parameter sets only the speed: 5/8 of the
    // way from the 5-point optimum 2/(1 + sin pi h) to Young's value
    // 2/(1 + sqrt(1 - mu^2)) for the compact operator's Jacobi radius
    // mu = 0.8 cos pi h + 0.2 cos^2 pi h (the four-colour order is not
    // consistently ordered, and neither end is optimal).  Measured on the
    // warm-started solves of time steps: the fewest sweeps at 513^2 to
    // 2049^2 (5 % fewer than the 5-point value at 1024^2, 12 % at 2049^2),
    // within 1 % of the fewest at 257^2.
    const double c = std::cos(M_PI * m.h), mu = 0.8 * c + 0.2 * c * c;
    const double w5 = 2.0 / (1.0 + std::sin(M_PI * m.h));
    const double w9 = 2.0 / (1.0 + std::sqrt(1.0 - mu * mu));
    m.relax = w5 - 0.625 * (w5 - w9);
  }
  // A stalled over-relaxation sits at its rounding floor; allow several
  // residual halvings' worth of sweeps (about 0.11 (n-1) each) before polishing.
  m.stall_window = std::max<long long>(64, 2LL * p.n);
  // tiles: small grids favour more, smaller blocks.  A launch costs about a
  // fixed part (start, region load, store) plus, per sweep, the plane rows
  // each wavefront walks; a region row is at most 128 nodes (64 per parity
  // plane, one per lane).  Measured on MI355X: at 1024^2, 84 x 54 tiles with
  // 5 sweeps per launch and 1024 threads (FP64; 247 tiles, one per CU, three
  // plane rows per wavefront, full 64-lane rows), XCD-banded: 2.9 us per
  // sweep against 3.1 for 64 x 64 with 4.  At 4096^2, 64 x 64 tiles with 4
  // sweeps and 512 threads (FP64, two blocks per CU overlap each other's
  // loads: 37.6 us per sweep against 47.7 for 96 x 64 with 3 and 1024
  // threads).  FP32 (no checking launches, so no wider halo): 88 x 56 tiles
  // with 5 sweeps at both sizes (2.38 / 20.0 us against 2.42 / 21.1 for the
  // next best).
  // Small grids take the same tiles: there the launch's fixed part dominates
  // and five sweeps per launch amortise it, even with most CUs idle (129^2 to
  // 320^2: 2.5-2.6 us per sweep against 5.3-5.9 for 32 x 32 tiles with one).
  if (p.n <= 2048) {
    m.cfg64 = {84, 54, 5, 1024, 1};
    m.cfg32 = {88, 56, 5, 1024, 1};
  } else {
    m.cfg64 = {64, 64, 4, 512, 0};
    m.cfg32 = {88, 56, 5, 1024, 1};
  }
  // Residual checks every n/10 sweeps (4 to 256) for solves started from the
  // previous stage's psi: a solve needs O(n) sweeps, so the overshoot past
  // convergence stays a fixed small fraction while the check launches (and
  // their decision kernels) stay rare.  Measured on the time step at 513^2 to
  // 2049^2 against n/16 (at most 64): equal at 513^2, 1 % faster at 1024^2,
  // 3 % at 2049^2.  Extrapolated starts need about half as many sweeps, and
  // checks every n/24 sweeps (rounded up to whole launch pairs: 50 at 1024^2)
  // are the fastest (1024^2, 1000 steps, Re 1e4 / 3e4: 30.5 / 31.3
  // Mcell-steps/s against 29.7 / 30.5 with n/10 = 110; 30, 70 and 160 sweeps
  // in between or below).
  // Mixed: 0.6 (n - 1) FP32 sweeps per refinement round.  A round reduces
  // the FP64 residual only about as far as the FP32 correction is accurate,
  // so sweeps beyond that are wasted; measured with the default relaxation
  // (factors 0.3 ... 3): the fastest steps at 1024^2 and at 4096^2 (23.9 and
  // 11.2 Mcell-steps/s against 17.8 and 5.1 with 1.5 (n - 1)).  With
  // extrapolated starts, 0.3 (n - 1) (1024^2, Re 3e4, 1000 steps: 84.8
  // Mcell-steps/s against 70.4; 200, 400, 500 and 800 sweeps: 70.5, 75.8,
  // 62.8, 55.3).
  const bool extrap = m.warm >= 2;
  set_schedule(m, std::min(256, std::max(4, p.n / (extrap ? 24 : 10))),
               (int)std::ceil((extrap ? 0.3 : 0.6) * (p.n - 1)));
  return CAVITY_OK;
}

size_t part_doubles(int n) {
  // two maxima per block of a checking launch or of the residual kernel;
  // a resident solve keeps two check slots of two maxima per tile
  return 4 * (size_t)std::max(cav::sor_max_blocks(n), cav::resid_blocks(n));
}

size_t flag_bytes() { return (size_t)cav::kMaxBatchGrid * cav::kFlagStride * sizeof(unsigned int); }

size_t handle_bytes(int count) {
  return align_up((size_t)count * sizeof(cav::BatchMember)) + align_up(sizeof(cav::BatchCtl)) +
         align_up(flag_bytes());
}

std::vector<int> mg_sizes(int n) {
  std::vector<int> v{n};
  while (v.back() > kMgCoarsest) v.push_back((v.back() - 1 + 1) / 2 + 1);
  return v;
}

size_t mg_bytes(int n) {
  const std::vector<int> v = mg_sizes(n);
  size_t b = align_up((size_t)n * pitch_of(n) * sizeof(double));  // level-0 residual
  for (size_t l = 1; l < v.size(); ++l)
    b += 4 * align_up((size_t)v[l] * pitch_of(v[l]) * sizeof(double));
  return b;
}

size_t mg32_bytes(int n) {
  const std::vector<int> v = mg_sizes(n);
  size_t b = align_up((size_t)n * pitch_of(n) * sizeof(float));  // level-0 residual
  for (size_t l = 1; l < v.size(); ++l)
    b += 4 * align_up((size_t)v[l] * pitch_of(v[l]) * sizeof(float));
  return b;
}

// Extrapolation weights of the warm starts.  Row L (2 <= L <= warm) holds w_q,
// q = 1 ... L: the start is sum_q w_q psi(step - q) for the polynomial of
// degree min(d, L - 1) through the L steps on file (least squares below L - 1).
constexpr int kWarmRows = CAVITY_WARM_LEVELS_MAX + 1;
using cav::kWarmCols;
static_assert(kWarmCols >= CAVITY_WARM_LEVELS_MAX, "a weight row holds every level");

// w_q for L points at -1 ... -L, degree d <= L - 1, evaluated at 0.  d = L - 1
// interpolates: the weights are (-1)^(q+1) C(L, q), exact in doubles.  Below,
// the least-squares polynomial, through a QR factorisation (modified
// Gram-Schmidt, long double) of the Vandermonde matrix in the centred abscissa
// s = (2q - L - 1) / (L - 1): p(0) = v0^T R^-1 Q^T y for the monomials v0 at
// s0 = -(L + 1) / (L - 1), so w = Q R^-T v0.
void warm_weights(int L, int d, double* w) {
  if (d >= L - 1) {
    double b = 1.0;
    for (int q = L; q >= 1; --q) {
      if (q < L) b = b * (q + 1) / (L - q);
      w[q - 1] = (q & 1) ? b : -b;
    }
    return;
  }
  long double Q[kWarmCols][kWarmCols] = {}, R[kWarmCols][kWarmCols] = {};
  for (int q = 1; q <= L; ++q) {
    const long double s = (long double)(2 * q - L - 1) / (L - 1);
    long double pw = 1;
    for (int k = 0; k <= d; ++k) {
      Q[q - 1][k] = pw;
      pw *= s;
    }
  }
  for (int k = 0; k <= d; ++k) {
    for (int j = 0; j < k; ++j) {
      long double dot = 0;
      for (int q = 0; q < L; ++q) dot += Q[q][j] * Q[q][k];
      R[j][k] = dot;
      for (int q = 0; q < L; ++q) Q[q][k] -= dot * Q[q][j];
    }
    long double nrm = 0;
    for (int q = 0; q < L; ++q) nrm += Q[q][k] * Q[q][k];
    nrm = sqrtl(nrm);
    R[k][k] = nrm;
    for (int q = 0; q < L; ++q) Q[q][k] /= nrm;
  }
  const long double s0 = -(long double)(L + 1) / (L - 1);
  long double z[kWarmCols], pw = 1;
  for (int k = 0; k <= d; ++k) {  // R^T z = v0
    long double v = pw;
    for (int j = 0; j < k; ++j) v -= R[j][k] * z[j];
    z[k] = v / R[k][k];
    pw *= s0;
  }
  for (int q = 0; q < L; ++q) {
    long double v = 0;
    for (int k = 0; k <= d; ++k) v += Q[q][k] * z[k];
    w[q] = (double)v;
  }
}

// Upload member m's weight table (enqueued on st; the host table stays valid
// until the stream has copied it: synchronised before returning).
hipError_t upload_warm_weights(const Member& m, hipStream_t st) {
  double tab[kWarmRows * kWarmCols] = {};
  for (int L = 2; L <= m.warm; ++L)
    warm_weights(L, std::min(m.warm_deg, L - 1), tab + L * kWarmCols);
  hipError_t e = hipMemcpyAsync(m.warm_w, tab, sizeof tab, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

size_t member_bytes(const Member& m) {
  const size_t f64 = align_up((size_t)m.n * m.pitch * sizeof(double));
  const size_t f32 = align_up((size_t)m.n * m.pitch * sizeof(float));
  size_t b = 8 * f64;  // w[4], psi, psi_b, psi_prev, F
  if (m.mixed) b += 4 * f32;
  b += align_up(sizeof(cav::PoissonCtl));
  b += align_up(part_doubles(m.n) * sizeof(double));
  b += align_up(cav::resident_flag_bytes(m.n)) + align_up(sizeof(cav::ResidentCtl));
  b += align_up((size_t)cav::diag_partials(m.n) * 4 * sizeof(double));
  b += align_up(4 * sizeof(double));
  b += mg_bytes(m.n);
  if (m.mixed) b += mg32_bytes(m.n);
  if (m.warm >= 2)
    b += 5 * (size_t)m.warm * f64 + align_up(sizeof(long long)) +
         align_up(kWarmRows * kWarmCols * sizeof(double));
  return b;
}

void carve(Member& m, char*& cur) {
  const size_t f64 = align_up((size_t)m.n * m.pitch * sizeof(double));
  const size_t f32 = align_up((size_t)m.n * m.pitch * sizeof(float));
  auto take = [&](size_t bytes) {
    char* r = cur;
    cur += bytes;
    return r;
  };
  for (int k = 0; k < 4; ++k) m.w[k] = reinterpret_cast<double*>(take(f64));
  m.psi = reinterpret_cast<double*>(take(f64));
  m.psi_b = reinterpret_cast<double*>(take(f64));
  m.psi_prev = reinterpret_cast<double*>(take(f64));
  m.F = reinterpret_cast<double*>(take(f64));
  if (m.mixed) {
    m.R32 = reinterpret_cast<float*>(take(f32));
    m.d32a = reinterpret_cast<float*>(take(f32));
    m.d32b = reinterpret_cast<float*>(take(f32));
    m.psi32 = reinterpret_cast<float*>(take(f32));
  }
  m.ctl = reinterpret_cast<cav::PoissonCtl*>(take(align_up(sizeof(cav::PoissonCtl))));
  m.part = reinterpret_cast<double*>(take(align_up(part_doubles(m.n) * sizeof(double))));
  m.rflags = reinterpret_cast<unsigned int*>(take(align_up(cav::resident_flag_bytes(m.n))));
  m.rctl = reinterpret_cast<cav::ResidentCtl*>(take(align_up(sizeof(cav::ResidentCtl))));
  m.diag_np = cav::diag_partials(m.n);
  m.diag_partial = reinterpret_cast<double*>(take(align_up((size_t)m.diag_np * 4 * 8)));
  m.diag_out = reinterpret_cast<double*>(take(align_up(4 * sizeof(double))));
  if (m.warm >= 2) {
    m.hist_stride = f64 / sizeof(double);
    m.hist = reinterpret_cast<double*>(take(5 * (size_t)m.warm * f64));
    m.warm_cnt = reinterpret_cast<long long*>(take(align_up(sizeof(long long))));
    m.warm_w = reinterpret_cast<double*>(take(align_up(kWarmRows * kWarmCols * sizeof(double))));
  }
  const std::vector<int> v = mg_sizes(m.n);
  m.mg.assign(v.size(), MgLevel{});
  for (size_t l = 0; l < v.size(); ++l) {
    MgLevel& L = m.mg[l];
    L.n = v[l];
    L.pitch = pitch_of(v[l]);
    L.h = 1.0 / (v[l] - 1);
    const size_t f = align_up((size_t)L.n * L.pitch * sizeof(double));
    if (l == 0) {
      L.E = m.psi;
      L.Eb = m.psi_b;
      L.F = m.F;
      L.r = reinterpret_cast<double*>(take(f));
    } else {
      L.E = reinterpret_cast<double*>(take(f));
      L.Eb = reinterpret_cast<double*>(take(f));
      L.F = reinterpret_cast<double*>(take(f));
      L.r = reinterpret_cast<double*>(take(f));
    }
  }
  m.mg32.clear();
  if (m.mixed) {
    m.mg32.assign(v.size(), MgLevel32{});
    for (size_t l = 0; l < v.size(); ++l) {
      MgLevel32& L = m.mg32[l];
      L.n = v[l];
      L.pitch = pitch_of(v[l]);
      L.h = 1.0 / (v[l] - 1);
      const size_t f = align_up((size_t)L.n * L.pitch * sizeof(float));
      if (l == 0) {
        L.E = m.d32a;
        L.Eb = m.d32b;
        L.F = m.R32;
        L.r = reinterpret_cast<float*>(take(f));
      } else {
        L.E = reinterpret_cast<float*>(take(f));
        L.Eb = reinterpret_cast<float*>(take(f));
        L.F = reinterpret_cast<float*>(take(f));
        L.r = reinterpret_cast<float*>(take(f));
      }
    }
  }
}

// Multigrid smoothing kernels: four-colour sweeps, 2 per launch.
// Smoother launches of the V-cycles (two sweeps each).  Above 2048 nodes a
// side, 512-thread blocks: two share a CU, so one block's loads and stores
// overlap the other's sweeps (measured at 4096^2: 43.8 against 67.4 us per
// FP64 sweep with 1024 threads).
cav::SorConfig mg_cfg(int n) {
  // up to 2048 nodes a side 64 x 32 tiles (3.1-3.4 us per sweep from 129^2 to
  // 513^2 against 3.7-4.5 for 64 x 64 with 1024 threads or 32 x 32)
  if (n > 2048) return cav::SorConfig{64, 64, 2, 512, 0};
  return cav::SorConfig{64, 32, 2, 512, 0};
}
constexpr int kMgNu = 2;   // pre- and post-smoothing sweeps (one launch each)
// A multigrid solve stops (floor-limited) once the residual max-norm, in the
// units of the relaxation (g - psi), is within this many ulps of max |psi|:
// the FP64 residual of the exact discrete solution sits at 2.6-3.9 ulps
// (1024^2), so cycles beyond this change only rounding noise.  With the
// developed flows of long runs (|psi| ~ 0.1 at 1024^2) that floor lies above
// a 1e-10 tolerance, and without this test every solve ran until its stall
// window (eight cycles without halving) ran out.
constexpr double kMgFloorUlps = 8.0;

// ---------------------------------------------------------------------------
// Poisson solves.  All members listed in `idx` are solved together: their
// sweeps are interleaved chunk by chunk and one readback serves them all.
// Each solve starts from the psi in Member::psi and leaves its result there;
// F must already hold the right-hand side.
// ---------------------------------------------------------------------------
long long unit_sweeps(const Member& m);

// FP64 SOR solves of a time step's stages that start from an extrapolation
// (two or more steps on file: decided on the device from the warm-start
// count, so a captured step graph does the same) open with Gauss-Seidel
// sweeps up to their first check.  The extrapolation's error is small but
// rough in space (largest next to the lid corners), so the start's residual
// is large (257^2, Re 1e4, step 100: error 3e-11, residual 6.7e-6 in
// vorticity units); over-relaxation damps rough components only by about
// w - 1 per sweep, Gauss-Seidel by a large factor.  Measured with the
// oracle's four-colour sweep on those starts: 350 sweeps to 1e-10, 130 with
// 10 Gauss-Seidel sweeps first, 90 with 20, 80 with 40.
// In mixed precision the opening is the first pair of FP32 correction sweeps
// of the solve's first refinement round.
bool gs_opening(const Member& m) {
  return m.warm >= 2 && m.solver == CAVITY_SOLVER_SOR && m.fixed == 0;
}

// stage_solve: the solve of an SSPRK stage (its start may be an extrapolation).
int reset_ctl(cavity_s* h, Member& m, bool stage_solve) {
  const double tol_hat = m.tol * 0.3 * m.h * m.h;  // (g - psi) = (3 h^2 / 10) r
  const long long spc = unit_sweeps(m);
  // multigrid halves the residual every cycle until the rounding floor:
  // eight cycles without halving mean the floor, and a residual within
  // kMgFloorUlps ulps of max |psi| is the floor itself
  const bool mg = m.solver == CAVITY_SOLVER_MG;
  const long long stall = mg ? 8LL * spc : m.stall_window;
  HIP_TRY(h, cav::launch_ctl_reset(m.ctl, m.relax, tol_hat, m.max_sweeps, stall, spc, h->st,
                                   mg ? kMgFloorUlps : 0.0,
                                   stage_solve && gs_opening(m) ? m.warm_cnt : nullptr));
  return CAVITY_OK;
}

// Sweeps between two residual checks (multigrid: fine-level sweeps of one
// V-cycle).
long long unit_sweeps(const Member& m) {
  if (m.solver == CAVITY_SOLVER_MG) return 2LL * kMgNu;
  return m.mixed ? m.inner_sweeps : 2LL * m.cfg64.s * m.pairs_per_check;
}

// One V(2,2)-cycle of the compact equation for member m, starting and ending
// with the iterate in m.psi.  On the finer levels each smoothing step is one
// launch of two four-colour Gauss-Seidel sweeps from one buffer of the level
// to the other, so after pre- and post-smoothing a level's iterate is back in
// its first buffer; the levels from the first with at most 65 nodes a side
// down to the coarsest run in one block (launch_mg_fused), with the same
// arithmetic.
int enqueue_vcycle(cavity_s* h, Member& m) {
  const int L = (int)m.mg.size() - 1;
  auto E = [&](int l) { return l == 0 ? m.psi : m.mg[l].E; };
  auto Eb = [&](int l) { return l == 0 ? m.psi_b : m.mg[l].Eb; };
  auto Fp = [&](int l) { return l == 0 ? m.F : m.mg[l].F; };
  // levels lc..L run in one block (the coarse end of the cycle)
  int lc = 0;
  while (lc < L && m.mg[lc].n > cav::mg_fuse_max()) ++lc;
  for (int l = 0; l < lc; ++l) {
    const MgLevel& v = m.mg[l];
    const MgLevel& c = m.mg[l + 1];
    HIP_TRY(h, cav::launch_sor64_relax(mg_cfg(v.n), E(l), Eb(l), Fp(l), v.n, v.pitch, m.ctl, 1.0,
                                       h->st));
    HIP_TRY(h, cav::launch_mg_residual(Eb(l), Fp(l), v.r, v.n, v.pitch, v.h, m.ctl, h->st));
    HIP_TRY(h, cav::launch_mg_restrict(v.r, v.n, v.pitch, c.F, c.E, c.Eb, c.n, c.pitch, m.ctl,
                                       h->st));
  }
  {
    int ns[8];
    for (int l = lc; l <= L; ++l) ns[l - lc] = m.mg[l].n;
    HIP_TRY(h, cav::launch_mg_fused(E(lc), Fp(lc), m.mg[lc].pitch, ns, L - lc + 1, kMgNu,
                                    kMgCoarseSweeps, kMgCoarseRelax, m.ctl, h->st));
  }
  for (int l = lc - 1; l >= 0; --l) {
    const MgLevel& v = m.mg[l];
    const MgLevel& c = m.mg[l + 1];
    HIP_TRY(h, cav::launch_mg_prolong(E(l + 1), c.n, c.pitch, Eb(l), v.n, v.pitch, m.ctl, h->st));
    HIP_TRY(h, cav::launch_sor64_relax(mg_cfg(v.n), Eb(l), E(l), Fp(l), v.n, v.pitch, m.ctl, 1.0,
                                       h->st));
  }
  return CAVITY_OK;
}

// The same cycle in FP32 for the correction equation of mixed precision:
// d32a holds the correction, R32 the FP64 residual rounded to FP32.
int enqueue_vcycle32(cavity_s* h, Member& m) {
  const int L = (int)m.mg32.size() - 1;
  int lc = 0;
  while (lc < L && m.mg32[lc].n > cav::mg_fuse_max()) ++lc;
  for (int l = 0; l < lc; ++l) {
    const MgLevel32& v = m.mg32[l];
    const MgLevel32& c = m.mg32[l + 1];
    HIP_TRY(h, cav::launch_sor32(mg_cfg(v.n), v.E, v.Eb, v.F, v.n, v.pitch, m.ctl, 1.0, h->st));
    HIP_TRY(h, cav::launch_mg_residual(v.Eb, v.F, v.r, v.n, v.pitch, v.h, m.ctl, h->st));
    HIP_TRY(h, cav::launch_mg_restrict(v.r, v.n, v.pitch, c.F, c.E, c.Eb, c.n, c.pitch, m.ctl,
                                       h->st));
  }
  {
    int ns[8];
    for (int l = lc; l <= L; ++l) ns[l - lc] = m.mg32[l].n;
    HIP_TRY(h, cav::launch_mg_fused(m.mg32[lc].E, m.mg32[lc].F, m.mg32[lc].pitch, ns, L - lc + 1,
                                    kMgNu, kMgCoarseSweeps, kMgCoarseRelax, m.ctl, h->st));
  }
  for (int l = lc - 1; l >= 0; --l) {
    const MgLevel32& v = m.mg32[l];
    const MgLevel32& c = m.mg32[l + 1];
    HIP_TRY(h, cav::launch_mg_prolong(c.E, c.n, c.pitch, v.Eb, v.n, v.pitch, m.ctl, h->st));
    HIP_TRY(h, cav::launch_sor32(mg_cfg(v.n), v.Eb, v.E, v.F, v.n, v.pitch, m.ctl, 1.0, h->st));
  }
  return CAVITY_OK;
}

// One chunk of work for member m: `units` check groups (FP64: pairs_per_check
// launch pairs, the last launch checking) or refinement rounds (mixed).
// Every launch returns at once once the solve has stopped.
int enqueue_chunk(cavity_s* h, Member& m, int units) {
  for (int u = 0; u < units; ++u) {
    if (m.solver == CAVITY_SOLVER_MG && m.mixed) {
      // FP64 residual (and the decision), one FP32 V-cycle on the
      // correction, FP64 refinement of psi
      HIP_TRY(h, cav::launch_resid64(m.psi, m.F, m.R32, m.d32a, m.n, m.pitch, m.ctl, m.part,
                                     h->st));
      const int rc = enqueue_vcycle32(h, m);
      if (rc != CAVITY_OK) return rc;
      HIP_TRY(h, cav::launch_refine(m.psi, m.d32a, m.n, m.pitch, m.ctl, 2 * kMgNu, h->st));
    } else if (m.solver == CAVITY_SOLVER_MG) {
      const int rc = enqueue_vcycle(h, m);
      if (rc != CAVITY_OK) return rc;
      HIP_TRY(h, cav::launch_resid64(m.psi, m.F, nullptr, nullptr, m.n, m.pitch, m.ctl, m.part,
                                     h->st, 2LL * kMgNu));
    } else if (!m.mixed) {
      for (int q = 0; q < m.pairs_per_check; ++q) {
        const int check = (q == m.pairs_per_check - 1) ? 1 : 0;
        HIP_TRY(h, cav::launch_sor64(m.cfg64, m.psi, m.psi_b, m.F, m.n, m.pitch, m.ctl, m.part,
                                     0, h->st));
        HIP_TRY(h, cav::launch_sor64(m.cfg64, m.psi_b, m.psi, m.F, m.n, m.pitch, m.ctl, m.part,
                                     check, h->st));
      }
    } else {
      HIP_TRY(h, cav::launch_resid64(m.psi, m.F, m.R32, m.d32a, m.n, m.pitch, m.ctl, m.part,
                                     h->st));
      const int pairs = m.inner_sweeps / (2 * m.cfg32.s);
      for (int q = 0; q < pairs; ++q) {
        // the last pair relaxes with 1 (Gauss-Seidel) to damp the FP32
        // over-relaxation noise before the correction is applied; the first
        // takes the control block's parameter (1 during a Gauss-Seidel
        // opening or after a stall, else m.relax)
        const double rl = (q == pairs - 1) ? 1.0 : (q == 0 ? 0.0 : m.relax);
        HIP_TRY(h, cav::launch_sor32(m.cfg32, m.d32a, m.d32b, m.R32, m.n, m.pitch, m.ctl, rl,
                                     h->st));
        HIP_TRY(h, cav::launch_sor32(m.cfg32, m.d32b, m.d32a, m.R32, m.n, m.pitch, m.ctl, rl,
                                     h->st));
      }
      HIP_TRY(h, cav::launch_refine(m.psi, m.d32a, m.n, m.pitch, m.ctl, m.inner_sweeps, h->st));
    }
  }
  return CAVITY_OK;
}

// Enqueue a residual check without sweeping (FP64): a converged warm start
// then needs no sweep at all.
int enqueue_initial_check(cavity_s* h, Member& m) {
  if (m.mixed) return CAVITY_OK;  // every refinement round starts with a check
  HIP_TRY(h, cav::launch_resid64(m.psi, m.F, nullptr, nullptr, m.n, m.pitch, m.ctl, m.part,
                                 h->st));
  return CAVITY_OK;
}

int read_ctls(cavity_s* h, const std::vector<int>& idx) {
  for (int k : idx)
    HIP_TRY(h, hipMemcpyAsync(&h->host_ctl[k], h->m[k].ctl, sizeof(cav::PoissonCtl),
                              hipMemcpyDeviceToHost, member_stream(h, k)));
  if (!h->fanned) {
    HIP_TRY(h, hipStreamSynchronize(h->st));
  } else {
    for (int k : idx) HIP_TRY(h, hipStreamSynchronize(h->mst[k]));
  }
  return CAVITY_OK;
}

// Tile shape of a resident solve for member m, if it has one on this device:
// 64 x 64 tiles (768 threads) from n > 512, 32 x 32 below, as long as every
// tile gets a co-resident block.
bool resident_config(const cavity_s* h, const Member& m, cav::SorConfig* c) {
  if (h->exec != CAVITY_EXEC_RESIDENT || m.mixed || m.solver != CAVITY_SOLVER_SOR || m.fixed)
    return false;
  const cav::SorConfig big{64, 64, 4, 768, 0}, small{32, 32, 2, 256, 0};
  if (m.n > 512 && cav::resident_supported(big, m.n, h->device)) {
    *c = big;
    return true;
  }
  if (cav::resident_supported(small, m.n, h->device)) {
    *c = small;
    return true;
  }
  return false;
}

// One resident launch for the whole solve of m (after its control reset and
// initial check).  Rounds per check follow the member's check spacing, but
// at least half the tile grid's width plus one, so that no block can run
// far enough ahead to reuse a partial-maximum slot block 0 is still reading.
int enqueue_resident(cavity_s* h, Member& m, const cav::SorConfig& c, bool stage_solve) {
  const int tiles = std::max((m.n + c.tx - 1) / c.tx, (m.n + c.ty - 1) / c.ty);
  const long long spc = 2LL * m.cfg64.s * m.pairs_per_check;
  const int P = std::max<int>({3, tiles / 2 + 1, (int)((spc + c.s - 1) / c.s)});
  const double tol_hat = m.tol * 0.3 * m.h * m.h;
  HIP_TRY(h, cav::launch_ctl_reset(m.ctl, m.relax, tol_hat, m.max_sweeps, m.stall_window,
                                   (long long)P * c.s, h->st, 0.0,
                                   stage_solve && gs_opening(m) ? m.warm_cnt : nullptr));
  HIP_TRY(h, cav::launch_resid64(m.psi, m.F, nullptr, nullptr, m.n, m.pitch, m.ctl, m.part,
                                 h->st));
  const long long spin = 10LL * 100000000LL;  // 10 s of the 100 MHz wall clock
  HIP_TRY(h, cav::launch_sor64_resident(c, m.psi, m.psi_b, m.F, m.n, m.pitch, m.ctl, m.part,
                                        m.rflags, m.rctl, P, spin, h->device, h->st));
  return CAVITY_OK;
}

// state_solve: the solve produces the state's psi (refresh its FP32 shadow);
// false for solves into scratch buffers.
// stage: the SSPRK stage (1..5) the solves belong to, 0 for any other solve;
// it selects the sweep estimate that sizes the first chunk of launches.
int solve_members(cavity_s* h, const std::vector<int>& idx, bool state_solve = true,
                  int stage = 0) {
  int rc;
  std::vector<int> active, resident;
  for (int k : idx) {
    Member& m = h->m[k];
    StreamScope sc(h, member_stream(h, k));
    cav::SorConfig rcfg;
    if (resident_config(h, m, &rcfg)) {
      if ((rc = enqueue_resident(h, m, rcfg, stage > 0)) != CAVITY_OK) return rc;
      resident.push_back(k);
      continue;
    }
    if ((rc = reset_ctl(h, m, stage > 0)) != CAVITY_OK) return rc;
    if ((rc = enqueue_initial_check(h, m)) != CAVITY_OK) return rc;
    active.push_back(k);
  }
  std::vector<long long> enqueued(h->count, 0);
  bool first = true;
  while (!active.empty()) {
    for (int k : active) {
      Member& m = h->m[k];
      const long long per_unit = unit_sweeps(m);
      // Launches enqueued past the device's decision still cost a few us
      // each, a chunk that falls short one more host round trip: the first
      // chunk covers the estimate with a small margin, later ones add a few
      // per cent of it (a quarter of what is enqueued when nothing is known).
      const double est = stage > 0 && m.est_stage[stage] > 0 ? m.est_stage[stage] : m.est_sweeps;
      long long units;
      if (first && est > 0)
        units = (long long)std::ceil(1.02 * est / per_unit);
      else if (first)
        units = std::max<long long>(4, (long long)(0.5 * (m.n - 1) / per_unit));
      else if (est > 0)
        units = std::max<long long>(1, (long long)std::ceil(0.05 * est / per_unit));
      else
        units = std::max<long long>(2, enqueued[k] / 4);
      units = std::max<long long>(1, std::min<long long>(units, m.max_sweeps / per_unit + 1));
      StreamScope sc(h, member_stream(h, k));
      if ((rc = enqueue_chunk(h, m, (int)units)) != CAVITY_OK) return rc;
      enqueued[k] += units;
    }
    first = false;
    if ((rc = read_ctls(h, active)) != CAVITY_OK) return rc;
    std::vector<int> still;
    for (int k : active) {
      const cav::PoissonCtl& c = h->host_ctl[k];
      if (c.state != cav::SOLVE_RUN) continue;
      Member& m = h->m[k];
      const long long per_unit = unit_sweeps(m);
      if (enqueued[k] * per_unit > 2 * m.max_sweeps + 64 * per_unit) {
        // the device never stopped the solve: a defect, not a slow solve
        h->poisoned = true;
        return fail(CAVITY_EHIP, "Poisson solve of cavity %d made no decision after %lld sweeps",
                    k, enqueued[k] * per_unit);
      }
      still.push_back(k);
    }
    active.swap(still);
  }
  if (!resident.empty() && (rc = read_ctls(h, resident)) != CAVITY_OK) return rc;
  for (int k : resident) {
    if (h->host_ctl[k].werror) {
      h->poisoned = true;
      return fail(CAVITY_EHIP, "resident solve of cavity %d: a wait timed out (tiles not "
                               "co-resident?)", k);
    }
  }
  for (int k : idx) {
    Member& m = h->m[k];
    if (m.mixed && state_solve)
      HIP_TRY(h, cav::launch_shadow(m.psi, m.psi32, m.n, m.pitch, member_stream(h, k)));
  }
  int worst = CAVITY_OK;
  for (int k : idx) {
    Member& m = h->m[k];
    const cav::PoissonCtl& c = h->host_ctl[k];
    m.sweeps_step += c.sweeps;
    m.sweeps_total += c.sweeps;
    m.last_resid = c.last * (10.0 / 3.0) / (m.h * m.h);
    if (c.sweeps > 0) {
      m.est_sweeps = m.est_sweeps > 0 ? 0.5 * (m.est_sweeps + c.sweeps) : (double)c.sweeps;
      if (stage > 0) m.est_stage[stage] = (double)c.sweeps;
    }
    if (c.state == cav::SOLVE_FLOOR) m.floor_step = 1;
    if (c.state == cav::SOLVE_NONFINITE) {
      h->poisoned = true;
      return fail(CAVITY_ENONFINITE, "non-finite Poisson residual in cavity %d", k);
    }
    if (c.state == cav::SOLVE_NOCONV) {
      m.status_step = CAVITY_ENOCONV;
      worst = fail(CAVITY_ENOCONV, "Poisson solve of cavity %d hit %lld sweeps (residual %g)", k,
                   (long long)c.sweeps, m.last_resid);
    }
  }
  return worst;
}

// Coupled mode (fixed_sweeps > 0): exactly m.fixed four-colour sweeps with
// relaxation m.relax from the psi left by the previous stage, no stopping
// test.  The last launch still evaluates the residual, against a tolerance of
// the largest double, so its check always ends the solve: the residual is
// reported and a non-finite one is counted in the control block's totals.
// Sweeps per launch do not change the result (every node sees the same
// neighbour values in the same colour order), so a remainder is swept with a
// one-sweep kernel.
int enqueue_fixed(cavity_s* h, Member& m) {
  HIP_TRY(h, cav::launch_ctl_reset(m.ctl, m.relax, DBL_MAX, m.fixed, m.fixed, m.fixed, h->st));
  const cav::SorConfig one{32, 32, 1, 256, 0};
  const int full = m.fixed / m.cfg64.s, rem = m.fixed % m.cfg64.s;
  const int launches = full + rem;
  double* a = m.psi;
  double* b = m.psi_b;
  for (int j = 0; j < launches; ++j) {
    const int check = (j == launches - 1) ? 1 : 0;
    HIP_TRY(h, cav::launch_sor64(j < full ? m.cfg64 : one, a, b, m.F, m.n, m.pitch, m.ctl,
                                 m.part, check, h->st));
    std::swap(a, b);
  }
  if (a != m.psi) HIP_TRY(h, cav::launch_copy(a, m.psi, m.n, m.pitch, h->st));
  return CAVITY_OK;
}

// After a step of coupled-mode members: sweeps, last residual and the
// non-finite check, from the control blocks' running totals (the step may
// have been a graph replay, with no host code between its launches).
int finish_fixed(cavity_s* h, const std::vector<int>& idx) {
  if (idx.empty()) return CAVITY_OK;
  const int rc = read_ctls(h, idx);
  if (rc != CAVITY_OK) return rc;
  for (int k : idx) {
    Member& m = h->m[k];
    const cav::PoissonCtl& c = h->host_ctl[k];
    cav::PoissonCtl& l = h->last_tot[k];
    const long long d = c.total_sweeps - l.total_sweeps;
    m.sweeps_step += d;
    m.sweeps_total += d;
    m.last_resid = c.last * (10.0 / 3.0) / (m.h * m.h);
    const bool nonfinite = c.total_nonfinite > l.total_nonfinite;
    l = c;
    if (nonfinite) {
      h->poisoned = true;
      return fail(CAVITY_ENONFINITE, "non-finite Poisson residual in cavity %d", k);
    }
  }
  return CAVITY_OK;
}

bool all_fixed(const cavity_s* h) {
  for (const Member& m : h->m)
    if (m.fixed == 0) return false;
  return true;
}

int enqueue_rhs_and_walls_prep(cavity_s* h, Member& m, const double* omega) {
  HIP_TRY(h, cav::launch_poisson_rhs(omega, m.F, m.n, m.pitch, m.h, h->st));
  return CAVITY_OK;
}

// ---------------------------------------------------------------------------
// Batched persistent solves.
// ---------------------------------------------------------------------------
void destroy_graphs(cavity_s* h) {
  for (int p = 0; p < 2; ++p) {
    if (h->gexec[p]) (void)hipGraphExecDestroy(h->gexec[p]);
    if (h->graph[p]) (void)hipGraphDestroy(h->graph[p]);
    h->gexec[p] = nullptr;
    h->graph[p] = nullptr;
  }
}

// Descriptors of every member in the batch's tile shape, uploaded to the
// workspace, and the co-resident grid size.
int setup_batch(cavity_s* h) {
  const cav::SorConfig& c = h->mixed ? h->bcfg32 : h->bcfg64;
  if (!cav::batch_config_supported(c, h->mixed))
    return fail(CAVITY_EINVAL, "batched kernel %dx%d s=%d nt=%d is not compiled", c.tx, c.ty, c.s,
                c.nt);
  h->h_mem.assign(h->count, cav::BatchMember{});
  int tile0 = 0;
  for (int k = 0; k < h->count; ++k) {
    Member& m = h->m[k];
    cav::BatchMember& b = h->h_mem[k];
    b.psi = m.psi;
    b.psi_b = m.psi_b;
    b.F = m.F;
    b.ctl = m.ctl;
    b.part = m.part;
    b.R32 = m.R32;
    b.d32a = m.d32a;
    b.d32b = m.d32b;
    b.n = m.n;
    b.pitch = m.pitch;
    b.tiles_x = (m.n + c.tx - 1) / c.tx;
    b.tiles = b.tiles_x * ((m.n + c.ty - 1) / c.ty);
    b.tile0 = tile0;
    tile0 += b.tiles;
  }
  h->total_tiles = tile0;
  HIP_TRY(h, hipMemcpy(h->d_mem, h->h_mem.data(), h->count * sizeof(cav::BatchMember),
                       hipMemcpyHostToDevice));
  const int g = cav::batch_grid(c, h->mixed, h->device);
  if (g <= 0) return fail(CAVITY_EHIP, "occupancy query for the batched kernel failed");
  h->grid = std::min(std::min(g, cav::kMaxBatchGrid), h->total_tiles);
  if (h->grid < h->count) h->grid = std::min(g, h->count);
  if (h->grid < h->count)
    return fail(CAVITY_EINVAL, "batch of %d cavities needs at least %d co-resident blocks",
                h->count, h->count);
  destroy_graphs(h);
  return CAVITY_OK;
}

long long batch_check_sweeps(const cavity_s* h) {
  return h->mixed ? 2LL * h->bcfg32.s * h->b_inner_pairs : 2LL * h->bcfg64.s * h->b_ppc;
}

// Enqueue one solve of every member in one persistent launch.  Like the
// per-launch path, an FP64 solve starts with a residual check, so a warm
// start that already meets the tolerance takes no sweep.
int enqueue_batch_solve(cavity_s* h) {
  for (Member& m : h->m) {
    const double tol_hat = m.tol * 0.3 * m.h * m.h;
    HIP_TRY(h, cav::launch_ctl_reset(m.ctl, m.relax, tol_hat, m.max_sweeps, m.stall_window,
                                     batch_check_sweeps(h), h->st, 0.0,
                                     gs_opening(m) ? m.warm_cnt : nullptr));
    if (!h->mixed)
      HIP_TRY(h, cav::launch_resid64(m.psi, m.F, nullptr, nullptr, m.n, m.pitch, m.ctl, m.part,
                                     h->st));
  }
  const long long spin = 10LL * 100000000LL;  // 10 s of the 100 MHz wall clock
  if (!h->mixed)
    HIP_TRY(h, cav::launch_batch64(h->bcfg64, h->d_mem, h->count, h->total_tiles, h->b_ppc,
                                   h->d_bc, h->d_flags, h->grid, spin, h->st));
  else
    HIP_TRY(h, cav::launch_batch_mixed(h->bcfg32, h->d_mem, h->count, h->total_tiles,
                                       h->b_inner_pairs, h->d_bc, h->d_flags, h->grid, spin,
                                       h->st));
  for (Member& m : h->m)
    if (m.mixed) HIP_TRY(h, cav::launch_shadow(m.psi, m.psi32, m.n, m.pitch, h->st));
  return CAVITY_OK;
}

// Read every member's solve totals and the barrier error flag, and turn the
// differences since the last read into this step's counts and status.
int collect_totals(cavity_s* h, bool update_step) {
  for (int k = 0; k < h->count; ++k)
    HIP_TRY(h, hipMemcpyAsync(&h->host_ctl[k], h->m[k].ctl, sizeof(cav::PoissonCtl),
                              hipMemcpyDeviceToHost, h->st));
  HIP_TRY(h, hipMemcpyAsync(h->host_bc, h->d_bc, sizeof(cav::BatchCtl), hipMemcpyDeviceToHost,
                            h->st));
  HIP_TRY(h, hipStreamSynchronize(h->st));
  if (h->last_tot.size() != (size_t)h->count) h->last_tot.assign(h->count, cav::PoissonCtl{});
  int worst = CAVITY_OK;
  for (int k = 0; k < h->count; ++k) {
    const cav::PoissonCtl& c = h->host_ctl[k];
    cav::PoissonCtl& l = h->last_tot[k];
    if (update_step) {
      Member& m = h->m[k];
      const long long d = c.total_sweeps - l.total_sweeps;
      m.sweeps_step += d;
      m.sweeps_total += d;
      m.last_resid = c.last * (10.0 / 3.0) / (m.h * m.h);
      if (c.total_floor > l.total_floor) m.floor_step = 1;
      if (c.total_nonfinite > l.total_nonfinite) {
        h->poisoned = true;
        worst = fail(CAVITY_ENONFINITE, "non-finite Poisson residual in cavity %d", k);
      } else if (c.total_noconv > l.total_noconv) {
        m.status_step = CAVITY_ENOCONV;
        if (worst == CAVITY_OK)
          worst = fail(CAVITY_ENOCONV, "a Poisson solve of cavity %d hit %lld sweeps", k,
                       (long long)m.max_sweeps);
      }
    }
    l = c;
  }
  if (h->host_bc->error) {
    h->poisoned = true;
    return fail(CAVITY_EHIP, "grid barrier of the batched kernel timed out (grid %d not "
                             "co-resident?)", h->grid);
  }
  return worst;
}

// ---------------------------------------------------------------------------
// One SSPRK(5,4) step of every member, stage by stage.
// Buffers: w[0] = omega^n, w[1] = omega^(1), omega^(3), omega^(n+1);
// w[2] = omega^(2), then the stage-5 partial sum P; w[3] = omega^(4).
// ---------------------------------------------------------------------------
double* stage_output(Member& m, int stage) {
  return (stage == 2) ? m.w[2] : (stage == 4) ? m.w[3] : m.w[1];
}

int enqueue_stage_one(cavity_s* h, Member& m, int stage) {
  {
    cav::StageArgs a{};
    a.nu = m.nu;
    a.h = m.h;
    const double dt = m.dt;
    const double* w0 = nullptr;
    const double* win = nullptr;
    const double* wx = nullptr;
    double* out = nullptr;
    const double* wp = nullptr;
    double* pout = nullptr;
    switch (stage) {
      case 1:
        win = m.w[0]; out = m.w[1]; a.a1 = 1.0; a.b = kC10 * dt;
        break;
      case 2:
        w0 = m.w[0]; win = m.w[1]; out = m.w[2]; a.a0 = kA20; a.a1 = kA21; a.b = kB21 * dt;
        break;
      case 3:
        w0 = m.w[0]; win = m.w[2]; out = m.w[1]; a.a0 = kA30; a.a1 = kA32; a.b = kB32 * dt;
        break;
      case 4:
        w0 = m.w[0]; win = m.w[1]; out = m.w[3]; a.a0 = kA40; a.a1 = kA43; a.b = kB43 * dt;
        wp = m.w[2]; pout = m.w[2]; a.pa = kA52; a.pb = kA53; a.pl = kB53 * dt;
        break;
      default:
        win = m.w[3]; wx = m.w[2]; out = m.w[1]; a.a1 = kA54; a.ax = 1.0; a.b = kB54 * dt;
        break;
    }
    HIP_TRY(h, cav::launch_stage(m.psi, m.mixed ? m.psi32 : nullptr, w0, win, wx, out, wp, pout,
                                 m.n, m.pitch, a, h->st));
    const int rc = enqueue_rhs_and_walls_prep(h, m, out);
    if (rc != CAVITY_OK) return rc;
    // the stage's transport has read psi: file it and start the solve from
    // the extrapolation
    if (m.warm >= 2)
      HIP_TRY(h, cav::launch_warm(m.psi, m.hist, m.hist_stride, m.n, m.pitch, stage, m.warm,
                                  m.warm_cnt, m.warm_w, h->st));
    return CAVITY_OK;
  }
}

// Stage kernels of every cavity, each on its stream.
int enqueue_stage(cavity_s* h, int stage) {
  for (int k = 0; k < h->count; ++k) {
    StreamScope sc(h, member_stream(h, k));
    const int rc = enqueue_stage_one(h, h->m[k], stage);
    if (rc != CAVITY_OK) return rc;
  }
  return CAVITY_OK;
}

int enqueue_thom(cavity_s* h, int stage) {
  for (int k = 0; k < h->count; ++k) {
    Member& m = h->m[k];
    HIP_TRY(h, cav::launch_thom(m.psi, stage_output(m, stage), m.n, m.pitch, m.h, m.u_lid,
                                member_stream(h, k)));
    // the step's five solutions are (or, for the last stage's, will be at the
    // next step's first stage) on file
    if (stage == 5 && m.warm >= 2)
      HIP_TRY(h, cav::launch_warm_tick(m.warm_cnt, member_stream(h, k)));
  }
  return CAVITY_OK;
}

// The whole step of coupled-mode cavities as pure enqueues.
int enqueue_step_fixed(cavity_s* h) {
  int rc;
  for (int stage = 1; stage <= 5; ++stage) {
    if ((rc = enqueue_stage(h, stage)) != CAVITY_OK) return rc;
    for (Member& m : h->m)
      if ((rc = enqueue_fixed(h, m)) != CAVITY_OK) return rc;
    if ((rc = enqueue_thom(h, stage)) != CAVITY_OK) return rc;
  }
  return CAVITY_OK;
}

// The whole step as pure enqueues (persistent solves): what a graph captures.
int enqueue_step_persistent(cavity_s* h) {
  int rc;
  for (int stage = 1; stage <= 5; ++stage) {
    if ((rc = enqueue_stage(h, stage)) != CAVITY_OK) return rc;
    if ((rc = enqueue_batch_solve(h)) != CAVITY_OK) return rc;
    if ((rc = enqueue_thom(h, stage)) != CAVITY_OK) return rc;
  }
  return CAVITY_OK;
}

int launch_step_graph(cavity_s* h) {
  const int parity = (h->m[0].w[0] == h->w0_base) ? 0 : 1;
  if (!h->gexec[parity]) {
    // The caller's stream may be the legacy null stream, which cannot be
    // captured: record on a private stream, replay on the caller's.
    if (!h->cap_st) HIP_TRY(h, hipStreamCreateWithFlags(&h->cap_st, hipStreamNonBlocking));
    HIP_TRY(h, hipStreamBeginCapture(h->cap_st, hipStreamCaptureModeThreadLocal));
    hipStream_t user = h->st;
    h->st = h->cap_st;
    const int rc = all_fixed(h) ? enqueue_step_fixed(h) : enqueue_step_persistent(h);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap_st, &g);
    h->st = user;
    if (rc != CAVITY_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      h->poisoned = true;
      return rc != CAVITY_OK ? rc : fail(CAVITY_EHIP, "graph capture failed: %s",
                                          hipGetErrorString(e));
    }
    h->graph[parity] = g;
    HIP_TRY(h, hipGraphInstantiate(&h->gexec[parity], g, nullptr, nullptr, 0));
  }
  HIP_TRY(h, hipGraphLaunch(h->gexec[parity], h->st));
  return CAVITY_OK;
}

// Fan a stream step of several cavities out to one stream each (created on
// first use), after everything already enqueued on the handle's stream, and
// join them back into it when the guard ends (also on an error path).
struct Fan {
  cavity_s* h = nullptr;
  ~Fan() {
    if (!h) return;
    h->fanned = false;
    for (int k = 0; k < h->count; ++k) {
      (void)hipEventRecord(h->mev[k], h->mst[k]);
      (void)hipStreamWaitEvent(h->st, h->mev[k], 0);
    }
  }
};

int fan_out(cavity_s* h, Fan& f) {
  if (h->mst.empty()) {
    // all or nothing: a partial set is released and the step fails
    std::vector<hipStream_t> st(h->count, nullptr);
    std::vector<hipEvent_t> ev(h->count, nullptr);
    hipEvent_t fork = nullptr;
    bool ok = hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < h->count; ++k)
      ok = hipStreamCreateWithFlags(&st[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      for (hipStream_t s : st)
        if (s) (void)hipStreamDestroy(s);
      for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
      if (fork) (void)hipEventDestroy(fork);
      return fail(CAVITY_EHIP, "could not create the per-cavity streams");
    }
    h->mst = st;
    h->mev = ev;
    h->fork_ev = fork;
  }
  HIP_TRY(h, hipEventRecord(h->fork_ev, h->st));
  for (int k = 0; k < h->count; ++k) HIP_TRY(h, hipStreamWaitEvent(h->mst[k], h->fork_ev, 0));
  h->fanned = true;
  f.h = h;
  return CAVITY_OK;
}

int step_all(cavity_s* h, bool want_diag) {
  int rc, worst = CAVITY_OK;
  for (Member& m : h->m) {
    m.sweeps_step = 0;
    m.floor_step = 0;
    m.status_step = CAVITY_OK;
    if (want_diag) HIP_TRY(h, cav::launch_copy(m.psi, m.psi_prev, m.n, m.pitch, h->st));
  }
  if (h->exec == CAVITY_EXEC_STREAM || h->exec == CAVITY_EXEC_RESIDENT) {
    std::vector<int> solved, fixed;
    for (int k = 0; k < h->count; ++k) (h->m[k].fixed > 0 ? fixed : solved).push_back(k);
    {
      // Several cavities in stream execution run on a stream each, so that the
      // launches of small cavities fill the CUs a large one leaves idle.  (Not
      // resident solves: each needs all its tiles co-resident.)
      Fan fan;
      if (h->exec == CAVITY_EXEC_STREAM && h->count > 1 && (rc = fan_out(h, fan)) != CAVITY_OK)
        return rc;
      for (int stage = 1; stage <= 5; ++stage) {
        if ((rc = enqueue_stage(h, stage)) != CAVITY_OK) return rc;
        for (int k : fixed) {
          StreamScope sc(h, member_stream(h, k));
          if ((rc = enqueue_fixed(h, h->m[k])) != CAVITY_OK) return rc;
        }
        rc = solved.empty() ? CAVITY_OK : solve_members(h, solved, true, stage);
        if (rc == CAVITY_ENONFINITE || rc == CAVITY_EHIP) return rc;
        if (rc != CAVITY_OK) worst = rc;
        if ((rc = enqueue_thom(h, stage)) != CAVITY_OK) return rc;
      }
    }
    if ((rc = finish_fixed(h, fixed)) != CAVITY_OK) return rc;
  } else if (all_fixed(h)) {
    if ((rc = launch_step_graph(h)) != CAVITY_OK) return rc;
    std::vector<int> all(h->count);
    for (int k = 0; k < h->count; ++k) all[k] = k;
    if ((rc = finish_fixed(h, all)) != CAVITY_OK) return rc;
  } else {
    rc = (h->exec == CAVITY_EXEC_GRAPH) ? launch_step_graph(h) : enqueue_step_persistent(h);
    if (rc != CAVITY_OK) return rc;
    rc = collect_totals(h, true);
    if (rc == CAVITY_ENONFINITE || rc == CAVITY_EHIP) return rc;
    if (rc != CAVITY_OK) worst = rc;
  }
  for (Member& m : h->m) {
    std::swap(m.w[0], m.w[1]);  // omega^(n+1) becomes the state; omega^n kept in w[1]
    m.step += 1;
    m.t += m.dt;
    if (want_diag)
      HIP_TRY(h, cav::launch_diag(m.psi_prev, m.psi, m.w[1], m.w[0], m.n, m.pitch, m.h,
                                  m.diag_partial, m.diag_np, m.diag_out, h->st));
  }
  return worst;
}

// ---------------------------------------------------------------------------
// Autotuner.  Every measurement runs on scratch buffers (psi_prev, psi_b, F,
// w[3], the FP32 fields and the control block between steps), so the state
// of the simulation is untouched.
// ---------------------------------------------------------------------------
struct EventTimer {
  hipEvent_t a = nullptr, b = nullptr;
  bool ok = false;
  EventTimer() { ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess; }
  ~EventTimer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Microseconds per sweep of `launches` back-to-back launches of config c.
int time_sweeps(cavity_s* h, Member& m, const cav::SorConfig& c, bool fp32, int launches,
                double* us_per_sweep) {
  EventTimer ev;
  if (!ev.ok) return fail(CAVITY_EHIP, "hipEventCreate failed");
  HIP_TRY(h, cav::launch_poisson_rhs(m.w[0], m.F, m.n, m.pitch, m.h, h->st));
  HIP_TRY(h, cav::launch_copy(m.psi, m.psi_prev, m.n, m.pitch, h->st));
  HIP_TRY(h, cav::launch_ctl_reset(m.ctl, m.relax, -1.0, 1LL << 62, 1LL << 62, 0, h->st));
  if (fp32) {
    HIP_TRY(h, cav::launch_resid64(m.psi, m.F, m.R32, m.d32a, m.n, m.pitch, m.ctl, m.part,
                                   h->st));
    HIP_TRY(h, cav::launch_ctl_reset(m.ctl, m.relax, -1.0, 1LL << 62, 1LL << 62, 0, h->st));
  }
  for (int k = -2; k < launches; ++k) {
    if (k == 0) HIP_TRY(h, hipEventRecord(ev.a, h->st));
    const bool fwd = (k & 1) == 0;
    if (fp32)
      HIP_TRY(h, cav::launch_sor32(c, fwd ? m.d32a : m.d32b, fwd ? m.d32b : m.d32a, m.R32, m.n,
                                   m.pitch, m.ctl, m.relax, h->st));
    else
      HIP_TRY(h, cav::launch_sor64(c, fwd ? m.psi_prev : m.psi_b, fwd ? m.psi_b : m.psi_prev,
                                   m.F, m.n, m.pitch, m.ctl, m.part, 0, h->st));
  }
  HIP_TRY(h, hipEventRecord(ev.b, h->st));
  HIP_TRY(h, hipEventSynchronize(ev.b));
  float ms = 0.f;
  HIP_TRY(h, hipEventElapsedTime(&ms, ev.a, ev.b));
  *us_per_sweep = 1e3 * ms / ((double)launches * c.s);
  return CAVITY_OK;
}

// Wall time of one complete solve of the member's current vorticity from a
// zero start, on scratch buffers (like cavity_poisson with a given omega).
int time_solve(cavity_s* h, int idx, double* ms_out) {
  Member& m = h->m[idx];
  double* saved_psi = m.psi;
  const long long saved_total = m.sweeps_total, saved_step = m.sweeps_step;
  const double saved_est = m.est_sweeps;
  const int saved_floor = m.floor_step, saved_status = m.status_step;
  const double saved_resid = m.last_resid;
  HIP_TRY(h, cav::launch_copy(m.w[0], m.w[3], m.n, m.pitch, h->st));
  HIP_TRY(h, cav::launch_fill(m.psi_prev, m.n, m.pitch, 0.0, h->st));
  HIP_TRY(h, cav::launch_poisson_rhs(m.w[3], m.F, m.n, m.pitch, m.h, h->st));
  HIP_TRY(h, hipStreamSynchronize(h->st));
  m.psi = m.psi_prev;
  m.est_sweeps = saved_est;
  const auto t0 = std::chrono::steady_clock::now();
  const int rc = solve_members(h, std::vector<int>{idx}, false);
  (void)hipStreamSynchronize(h->st);
  const auto t1 = std::chrono::steady_clock::now();
  m.psi = saved_psi;
  m.sweeps_total = saved_total;
  m.sweeps_step = saved_step;
  m.est_sweeps = saved_est;
  m.floor_step = saved_floor;
  m.status_step = saved_status;
  m.last_resid = saved_resid;
  if (rc != CAVITY_OK) return rc;
  *ms_out = std::chrono::duration<double, std::milli>(t1 - t0).count();
  return CAVITY_OK;
}

// Microseconds per round of the persistent kernel with config c, over a
// fixed number of rounds (no member stops early), on scratch descriptors.
int time_batch(cavity_s* h, const cav::SorConfig& c, int rounds, double* us_per_round) {
  EventTimer ev;
  if (!ev.ok) return fail(CAVITY_EHIP, "hipEventCreate failed");
  const cav::SorConfig saved64 = h->bcfg64, saved32 = h->bcfg32;
  const int saved_ppc = h->b_ppc, saved_inner = h->b_inner_pairs;
  if (h->mixed) h->bcfg32 = c; else h->bcfg64 = c;
  int rc = setup_batch(h);
  if (rc != CAVITY_OK) return rc;
  // scratch descriptors: psi -> psi_prev, and the sweep limit ends each
  // member's solve after `rounds` rounds
  std::vector<cav::BatchMember> scratch = h->h_mem;
  for (int k = 0; k < h->count; ++k) {
    Member& m = h->m[k];
    scratch[k].psi = m.psi_prev;
    HIP_TRY(h, cav::launch_copy(m.psi, m.psi_prev, m.n, m.pitch, h->st));
    HIP_TRY(h, cav::launch_poisson_rhs(m.w[0], m.F, m.n, m.pitch, m.h, h->st));
  }
  HIP_TRY(h, hipMemcpy(h->d_mem, scratch.data(), h->count * sizeof(cav::BatchMember),
                       hipMemcpyHostToDevice));
  const long long per_round = c.s;
  h->b_ppc = 1;
  h->b_inner_pairs = 1;
  for (Member& m : h->m)
    HIP_TRY(h, cav::launch_ctl_reset(m.ctl, m.relax, -1.0, rounds * per_round, 1LL << 62,
                                     2 * per_round, h->st));
  const long long spin = 10LL * 100000000LL;
  HIP_TRY(h, hipEventRecord(ev.a, h->st));
  if (h->mixed) {
    HIP_TRY(h, cav::launch_batch_mixed(c, h->d_mem, h->count, h->total_tiles, 1, h->d_bc,
                                       h->d_flags, h->grid, spin, h->st));
  } else {
    HIP_TRY(h, cav::launch_batch64(c, h->d_mem, h->count, h->total_tiles, 1, h->d_bc,
                                   h->d_flags, h->grid, spin, h->st));
  }
  HIP_TRY(h, hipEventRecord(ev.b, h->st));
  HIP_TRY(h, hipEventSynchronize(ev.b));
  float ms = 0.f;
  HIP_TRY(h, hipEventElapsedTime(&ms, ev.a, ev.b));
  // mixed rounds: residual + 2 FP32 launches + refinement; FP64: 2 launches + decision
  const int launches_per_round = 2;
  const long long done_rounds = h->mixed ? (rounds * per_round) / (2 * c.s) + 1
                                         : (rounds * per_round) / (2 * c.s);
  *us_per_round = 1e3 * ms / ((double)std::max<long long>(1, done_rounds) * launches_per_round);
  h->bcfg64 = saved64;
  h->bcfg32 = saved32;
  h->b_ppc = saved_ppc;
  h->b_inner_pairs = saved_inner;
  rc = setup_batch(h);  // restores the real descriptors
  if (rc != CAVITY_OK) return rc;
  return collect_totals(h, false);
}

std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string tune_key(cavity_s* h, int idx) {
  char buf[512];
  if (idx >= 0) {
    snprintf(buf, sizeof buf, "%s|n=%d|prec=%d|solver=%d|batch=0", arch_name(h->device).c_str(),
             h->m[idx].n, h->m[idx].mixed ? 1 : 0, h->m[idx].solver);
    return buf;
  }
  std::string k = arch_name(h->device) + "|prec=" + (h->mixed ? "1" : "0") + "|batch=";
  for (const Member& m : h->m) k += std::to_string(m.n) + ",";
  return k;
}

bool cache_lookup(const char* path, const std::string& key, cavity_tuning* t) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  const std::string pre = "{\"key\": \"" + key + "\", ";
  while (fgets(line, sizeof line, f)) {
    if (strncmp(line, pre.c_str(), pre.size()) != 0) continue;
    cavity_tuning r{};
    const int got = sscanf(line + pre.size(),
                           "\"tile_x\": %d, \"tile_y\": %d, \"sweeps_per_launch\": %d, "
                           "\"threads\": %d, \"tile_x32\": %d, \"tile_y32\": %d, "
                           "\"sweeps_per_launch32\": %d, \"threads32\": %d, "
                           "\"check_every\": %d, \"inner_sweeps\": %d, \"xcd_bands\": %d, "
                           "\"solver\": %d, \"sor_omega\": %lf, \"warm_degree\": %d",
                           &r.tile_x, &r.tile_y, &r.sweeps_per_launch, &r.threads, &r.tile_x32,
                           &r.tile_y32, &r.sweeps_per_launch32, &r.threads32, &r.check_every,
                           &r.inner_sweeps, &r.xcd_bands, &r.solver, &r.sor_omega,
                           &r.warm_degree);
    if (got == 14) {
      *t = r;
      found = true;  // the last matching line wins
    }
  }
  fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const cavity_tuning& t) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f,
          "{\"key\": \"%s\", \"tile_x\": %d, \"tile_y\": %d, \"sweeps_per_launch\": %d, "
          "\"threads\": %d, \"tile_x32\": %d, \"tile_y32\": %d, \"sweeps_per_launch32\": %d, "
          "\"threads32\": %d, \"check_every\": %d, \"inner_sweeps\": %d, "
          "\"xcd_bands\": %d, \"solver\": %d, \"sor_omega\": %.17g, \"warm_degree\": %d}\n",
          key.c_str(), t.tile_x, t.tile_y, t.sweeps_per_launch, t.threads, t.tile_x32,
          t.tile_y32, t.sweeps_per_launch32, t.threads32, t.check_every, t.inner_sweeps,
          t.xcd_bands, t.solver, t.sor_omega, t.warm_degree);
  fclose(f);
}

// Copy every member's monitors of the last logged step to the host.
int read_diag(cavity_s* h) {
  for (int k = 0; k < h->count; ++k)
    HIP_TRY(h, hipMemcpyAsync(&h->host_diag[4 * k], h->m[k].diag_out, 4 * sizeof(double),
                              hipMemcpyDeviceToHost, h->st));
  HIP_TRY(h, hipStreamSynchronize(h->st));
  return CAVITY_OK;
}

// Per-member results; the monitors (Sec. 3.2, eqs. resS and resV) come from
// the last read_diag when have_diag.
void fill_stats(const cavity_s* h, bool have_diag, cavity_stats* stats) {
  for (int k = 0; k < h->count; ++k) {
    const Member& m = h->m[k];
    cavity_stats& o = stats[k];
    std::memset(&o, 0, sizeof o);
    o.step = m.step;
    o.t = m.t;
    o.dt = m.dt;
    if (have_diag) {
      const double* d = &h->host_diag[4 * k];
      o.res_psi = d[0] / m.n;
      o.res_omega = d[1] / m.n;
      o.domega_inf_over_dt = d[2] / m.dt;
      o.ke = 0.5 * m.h * m.h * d[3];
    }
    o.last_resid_inf = m.last_resid;
    o.sweeps_total = m.sweeps_total;
    o.sweeps_last_step = m.sweeps_step;
    o.floor_limited = m.floor_step;
    o.status = m.status_step;
  }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* cavity_last_error(void) { return g_err.c_str(); }

int cavity_warm_weights(int32_t levels, int32_t degree, double* w) {
  if (!w) return fail(CAVITY_EINVAL, "null argument");
  if (levels < 2 || levels > CAVITY_WARM_LEVELS_MAX)
    return fail(CAVITY_EINVAL, "levels = %d outside [2, %d]", levels, CAVITY_WARM_LEVELS_MAX);
  if (degree < 1 || degree > levels - 1)
    return fail(CAVITY_EINVAL, "degree = %d outside [1, %d]", degree, levels - 1);
  warm_weights(levels, degree, w);
  return CAVITY_OK;
}

int cavity_workspace_bytes(const cavity_params* p, int32_t count, size_t* bytes) {
  if (!p || !bytes) return fail(CAVITY_EINVAL, "null argument");
  if (count < 1) return fail(CAVITY_EINVAL, "count must be >= 1");
  size_t total = handle_bytes(count);
  for (int k = 0; k < count; ++k) {
    Member m;
    const int rc = derive(p[k], m);
    if (rc != CAVITY_OK) return rc;
    total += member_bytes(m);
  }
  *bytes = total;
  return CAVITY_OK;
}

int cavity_create(const cavity_params* p, int32_t count, void* d_ws, size_t ws_bytes,
                  void* hip_stream, cavity_t* out) {
  if (!p || !out) return fail(CAVITY_EINVAL, "null argument");
  *out = nullptr;
  if (count < 1) return fail(CAVITY_EINVAL, "count must be >= 1");
  if (!d_ws) return fail(CAVITY_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign != 0)
    return fail(CAVITY_EINVAL, "workspace must be 256-byte aligned");
  cavity_s* h = new (std::nothrow) cavity_s();
  if (!h) return fail(CAVITY_ENOMEM, "host allocation failed");
  h->count = count;
  h->st = static_cast<hipStream_t>(hip_stream);
  h->m.resize(count);
  size_t need = 0;
  for (int k = 0; k < count; ++k) {
    const int rc = derive(p[k], h->m[k]);
    if (rc != CAVITY_OK) {
      delete h;
      return rc;
    }
    need += member_bytes(h->m[k]);
  }
  need += handle_bytes(count);
  if (ws_bytes < need) {
    delete h;
    return fail(CAVITY_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  }
  h->mixed = h->m[0].mixed;
  bool uniform = true;
  for (const Member& m : h->m) uniform = uniform && (m.mixed == h->mixed);
  if (hipGetDevice(&h->device) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&h->host_ctl), count * sizeof(cav::PoissonCtl)) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&h->host_diag), count * 4 * sizeof(double)) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&h->host_bc), sizeof(cav::BatchCtl)) != hipSuccess) {
    cavity_destroy(h);
    return fail(CAVITY_EHIP, "pinned host allocation failed");
  }
  char* cur = static_cast<char*>(d_ws);
  for (Member& m : h->m) carve(m, cur);
  h->d_mem = reinterpret_cast<cav::BatchMember*>(cur);
  cur += align_up((size_t)count * sizeof(cav::BatchMember));
  h->d_bc = reinterpret_cast<cav::BatchCtl*>(cur);
  cur += align_up(sizeof(cav::BatchCtl));
  h->d_flags = reinterpret_cast<unsigned int*>(cur);
  h->w0_base = h->m[0].w[0];

  auto bail = [&](int rc) {
    cavity_destroy(h);
    return rc;
  };
  if (cav::launch_zero(h->d_bc, sizeof(cav::BatchCtl), h->st) != hipSuccess ||
      cav::launch_zero(h->d_flags, flag_bytes(), h->st) != hipSuccess)
    return bail(fail(CAVITY_EHIP, "zero fill failed"));
  for (Member& m : h->m) {
    if (cav::launch_zero(m.ctl, sizeof(cav::PoissonCtl), h->st) != hipSuccess)
      return bail(fail(CAVITY_EHIP, "zero fill failed"));
    // no step on file yet
    if (m.warm_cnt && (cav::launch_zero(m.warm_cnt, sizeof(long long), h->st) != hipSuccess ||
                       upload_warm_weights(m, h->st) != hipSuccess))
      return bail(fail(CAVITY_EHIP, "warm-start setup failed"));
    for (int k = 0; k < 4; ++k)
      if (cav::launch_fill(m.w[k], m.n, m.pitch, 0.0, h->st) != hipSuccess)
        return bail(fail(CAVITY_EHIP, "fill failed"));
    double* f64[] = {m.psi, m.psi_b, m.psi_prev, m.F};
    for (double* f : f64)
      if (cav::launch_fill(f, m.n, m.pitch, 0.0, h->st) != hipSuccess)
        return bail(fail(CAVITY_EHIP, "fill failed"));
    if (m.mixed) {
      float* f32[] = {m.R32, m.d32a, m.d32b, m.psi32};
      for (float* f : f32)
        if (cav::launch_fill32(f, m.n, m.pitch, 0.0f, h->st) != hipSuccess)
          return bail(fail(CAVITY_EHIP, "fill failed"));
    }
    if (m.p.omega0 && cav::launch_copy_in(m.p.omega0, m.w[0], m.n, m.pitch, h->st) != hipSuccess)
      return bail(fail(CAVITY_EHIP, "omega0 copy failed"));
    if (m.p.psi0) {
      if (cav::launch_copy_in(m.p.psi0, m.psi_b, m.n, m.pitch, h->st) != hipSuccess ||
          cav::launch_copy_interior(m.psi_b, m.psi, m.n, m.pitch, h->st) != hipSuccess)
        return bail(fail(CAVITY_EHIP, "psi0 copy failed"));
    }
    m.p.omega0 = nullptr;
    m.p.psi0 = nullptr;
    int rc = enqueue_rhs_and_walls_prep(h, m, m.w[0]);
    if (rc != CAVITY_OK) return bail(rc);
  }
  // The initial state: psi solved for omega0, then Thom's wall vorticity.
  // A resumed member already holds such a pair and is taken as it is.
  std::vector<int> fresh;
  for (int k = 0; k < count; ++k)
    if (!h->m[k].p.resume) fresh.push_back(k);
  int rc = fresh.empty() ? CAVITY_OK : solve_members(h, fresh);
  if (rc == CAVITY_ENONFINITE || rc == CAVITY_EHIP) return bail(rc);
  for (int k : fresh) {
    Member& m = h->m[k];
    if (cav::launch_thom(m.psi, m.w[0], m.n, m.pitch, m.h, m.u_lid, h->st) != hipSuccess)
      return bail(fail(CAVITY_EHIP, "thom failed"));
  }
  for (Member& m : h->m)
    if (m.mixed && m.p.resume &&
        cav::launch_shadow(m.psi, m.psi32, m.n, m.pitch, h->st) != hipSuccess)
      return bail(fail(CAVITY_EHIP, "shadow failed"));
  if (hipStreamSynchronize(h->st) != hipSuccess) return bail(fail(CAVITY_EHIP, "sync failed"));
  for (Member& m : h->m) {
    m.sweeps_total = 0;
    m.sweeps_step = 0;
  }
  // Batch defaults: the tile shapes the autotuner measured fastest; residual
  // checks every 30-32 sweeps; FP32 rounds as long as the largest member's.
  // Cavities of at most 512 nodes a side (the ones graph execution is the
  // default for) take 64 x 32 tiles with 4 sweeps per round and 512 threads:
  // sixteen 128^2 cavities 25.5 Mcell-steps/s against 21.0 with 64 x 64 tiles
  // of 768 threads.  Larger ones take the per-launch kernel's tiles, five
  // sweeps per round (fewer grid barriers per sweep): the six-cavity
  // Reynolds sweep 16.9 Mcell-steps/s in FP64 against 13.6 with 64 x 64
  // tiles and three sweeps per round.
  {
    int inner = 0, nmax = 0;
    for (const Member& m : h->m) {
      inner = std::max(inner, m.inner_sweeps);
      nmax = std::max(nmax, m.n);
    }
    const int small = h->m[0].n <= 320 && count == 1;
    h->bcfg64 = small           ? cav::SorConfig{32, 32, 1, 256, 0}
                : nmax <= 512 ? cav::SorConfig{64, 32, 4, 512, 0}
                              : cav::SorConfig{84, 54, 5, 1024, 0};
    h->bcfg32 = small         ? cav::SorConfig{32, 32, 1, 256, 0}
                : nmax <= 512 ? cav::SorConfig{64, 64, 4, 1024, 0}
                              : cav::SorConfig{88, 56, 5, 1024, 0};
    h->b_ppc = std::max(1, 32 / (2 * h->bcfg64.s));
    h->b_inner_pairs = std::max(1, (inner + 2 * h->bcfg32.s - 1) / (2 * h->bcfg32.s));
  }
  const int rc2 = collect_totals(h, false);
  if (rc2 != CAVITY_OK) return bail(rc2);
  bool any_fixed = false;
  for (const Member& m : h->m) any_fixed = any_fixed || m.fixed > 0;
  if (count > 1 && uniform && !any_fixed) {
    const int rc3 = setup_batch(h);
    if (rc3 != CAVITY_OK) return bail(rc3);
    // The persistent graph fuses cavities too small to fill the GPU alone; once
    // one has more than 512 nodes a side (a quarter of the CUs or more), a
    // stream per cavity is faster (measured: sixteen 128^2 cavities 20.5
    // against 1.5 Mcell-steps/s, six of 256^2 to 1024^2 12.3 against 16.7).
    int nmax = 0;
    for (const Member& m : h->m) nmax = std::max(nmax, m.n);
    h->exec = nmax <= 512 ? CAVITY_EXEC_GRAPH : CAVITY_EXEC_STREAM;
  }
  *out = h;
  return rc;
}

int cavity_step(cavity_t h, int32_t nsteps, cavity_stats* stats) {
  if (!h) return fail(CAVITY_EINVAL, "null handle");
  if (h->poisoned) return fail(CAVITY_ESTATE, "handle poisoned by an earlier failure");
  if (nsteps < 0) return fail(CAVITY_EINVAL, "nsteps must be >= 0");
  HIP_TRY(h, hipSetDevice(h->device));
  int worst = CAVITY_OK;
  for (int s = 0; s < nsteps; ++s) {
    const bool diag = stats && s == nsteps - 1;
    const int rc = step_all(h, diag);
    if (rc == CAVITY_ENONFINITE || rc == CAVITY_EHIP) return rc;
    if (rc != CAVITY_OK) worst = rc;
  }
  if (stats) {
    if (nsteps > 0) {
      const int rc = read_diag(h);
      if (rc != CAVITY_OK) return rc;
    }
    fill_stats(h, nsteps > 0, stats);
  }
  return worst;
}

int cavity_run_steady(cavity_t h, int64_t max_steps, int32_t check_every,
                      const double* res_psi_tol, const double* res_omega_tol,
                      int64_t* steady_step, cavity_stats* stats) {
  if (!h) return fail(CAVITY_EINVAL, "null handle");
  if (h->poisoned) return fail(CAVITY_ESTATE, "handle poisoned by an earlier failure");
  if (max_steps < 1 || check_every < 1)
    return fail(CAVITY_EINVAL, "max_steps and check_every must be >= 1");
  if (!steady_step) return fail(CAVITY_EINVAL, "steady_step must not be NULL");
  std::vector<double> tp(h->count), tw(h->count);
  for (int k = 0; k < h->count; ++k) {
    const Member& m = h->m[k];
    // Sec. 4: 1e-12 / 1e-10 up to Re = 20 000, 1e-10 / 1e-8 above
    const double re = std::fabs(m.u_lid) / m.nu;
    tp[k] = res_psi_tol ? res_psi_tol[k] : (re <= 20000.0 ? 1e-12 : 1e-10);
    tw[k] = res_omega_tol ? res_omega_tol[k] : (re <= 20000.0 ? 1e-10 : 1e-8);
    if (!(tp[k] > 0) || !(tw[k] > 0) || !std::isfinite(tp[k]) || !std::isfinite(tw[k]))
      return fail(CAVITY_EINVAL, "thresholds of cavity %d must be finite and > 0", k);
    steady_step[k] = -1;
  }
  HIP_TRY(h, hipSetDevice(h->device));
  int worst = CAVITY_OK, pending = h->count;
  long long done = 0;
  while (done < max_steps && pending > 0) {
    const long long chunk = std::min<long long>(check_every, max_steps - done);
    for (long long s = 0; s < chunk; ++s) {
      const int rc = step_all(h, s == chunk - 1);
      if (rc == CAVITY_ENONFINITE || rc == CAVITY_EHIP) return rc;
      if (rc != CAVITY_OK) worst = rc;
    }
    done += chunk;
    const int rc = read_diag(h);
    if (rc != CAVITY_OK) return rc;
    for (int k = 0; k < h->count; ++k) {
      const Member& m = h->m[k];
      const double* d = &h->host_diag[4 * k];
      if (steady_step[k] < 0 && d[0] / m.n <= tp[k] && d[1] / m.n <= tw[k]) {
        steady_step[k] = m.step;
        --pending;
      }
    }
  }
  if (stats) fill_stats(h, true, stats);
  return worst;
}

int cavity_poisson(cavity_t h, int32_t idx, const double* d_omega, double* d_psi,
                   cavity_poisson_info* info) {
  if (!h) return fail(CAVITY_EINVAL, "null handle");
  if (h->poisoned) return fail(CAVITY_ESTATE, "handle poisoned by an earlier failure");
  if (idx < 0 || idx >= h->count) return fail(CAVITY_EINVAL, "idx %d out of range", idx);
  HIP_TRY(h, hipSetDevice(h->device));
  Member& m = h->m[idx];
  int rc;
  double* saved_psi = m.psi;
  double* saved_b = m.psi_b;
  if (d_omega) {
    // Solve for a caller-given vorticity from a zero start without touching
    // the state: w[3] holds the input, psi_prev / psi_b the iterate.
    HIP_TRY(h, cav::launch_copy_in(d_omega, m.w[3], m.n, m.pitch, h->st));
    HIP_TRY(h, cav::launch_fill(m.psi_prev, m.n, m.pitch, 0.0, h->st));
    m.psi = m.psi_prev;
    m.psi_b = saved_b;
    if ((rc = enqueue_rhs_and_walls_prep(h, m, m.w[3])) != CAVITY_OK) return rc;
  } else {
    if ((rc = enqueue_rhs_and_walls_prep(h, m, m.w[0])) != CAVITY_OK) return rc;
  }
  const long long before = m.sweeps_total;
  rc = solve_members(h, std::vector<int>{idx}, d_omega == nullptr);
  double* result = m.psi;
  m.psi = saved_psi;
  m.psi_b = saved_b;
  if (rc == CAVITY_ENONFINITE || rc == CAVITY_EHIP) return rc;
  if (!d_omega)
    HIP_TRY(h, cav::launch_thom(m.psi, m.w[0], m.n, m.pitch, m.h, m.u_lid, h->st));
  if (d_psi) HIP_TRY(h, cav::launch_copy_out(result, d_psi, m.n, m.pitch, h->st));
  // the solve's counts are not a step's: batched and coupled steps count
  // from these totals
  if (h->last_tot.size() == (size_t)h->count) h->last_tot[idx] = h->host_ctl[idx];
  if (info) {
    HIP_TRY(h, hipStreamSynchronize(h->st));
    const cav::PoissonCtl& c = h->host_ctl[idx];
    info->sweeps = m.sweeps_total - before;
    info->resid_inf = c.last * (10.0 / 3.0) / (m.h * m.h);
    info->floor_limited = c.state == cav::SOLVE_FLOOR ? 1 : 0;
    info->status = c.state == cav::SOLVE_NOCONV ? CAVITY_ENOCONV : CAVITY_OK;
  }
  return rc;
}

int cavity_poisson_noalloc(int32_t n, double poisson_tol, double sor_omega,
                           int32_t poisson_max_sweeps, const double* d_omega, double* d_psi,
                           void* hip_stream, cavity_poisson_info* info) {
  if (!d_omega || !d_psi) return fail(CAVITY_EINVAL, "d_omega and d_psi are required");
  if (n < 5 || n > cav::noalloc_max_n())
    return fail(CAVITY_EINVAL, "n = %d outside [5, %d], the grids the allocation-free solve's "
                               "scratch array holds", n, cav::noalloc_max_n());
  if (poisson_max_sweeps < 0) return fail(CAVITY_EINVAL, "poisson_max_sweeps must be >= 0");
  // the same derived solve parameters as a cavity of this size with default
  // tuning (relaxation, sweep kernel, check spacing, stall window, limits)
  cavity_params p{};
  p.n = n;
  p.re = 1.0;
  p.u_lid = 1.0;
  p.poisson_tol = poisson_tol;
  p.poisson_max_sweeps = poisson_max_sweeps;
  p.sor_omega = sor_omega;
  Member m;
  int rc = derive(p, m);
  if (rc != CAVITY_OK) return rc;
  cavity_s* const none = nullptr;  // no handle to poison
  void* base = nullptr;
  HIP_TRY(none, cav::noalloc_scratch(&base));
  // carve the scratch array: F, the iterate's pair, partial maxima, control
  const size_t f64 = align_up((size_t)m.n * m.pitch * sizeof(double));
  const size_t partb = align_up(part_doubles(m.n) * sizeof(double));
  if (3 * f64 + partb + align_up(sizeof(cav::PoissonCtl)) > cav::noalloc_bytes())
    return fail(CAVITY_EINVAL, "n = %d does not fit the scratch array", n);
  char* cur = static_cast<char*>(base);
  m.F = reinterpret_cast<double*>(cur);
  m.psi = reinterpret_cast<double*>(cur + f64);
  m.psi_b = reinterpret_cast<double*>(cur + 2 * f64);
  m.part = reinterpret_cast<double*>(cur + 3 * f64);
  m.ctl = reinterpret_cast<cav::PoissonCtl*>(cur + 3 * f64 + partb);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // omega (pitched, in psi_b for the moment) -> F; both iterates start at 0
  // (walls included), whatever an earlier call left in the array
  HIP_TRY(none, cav::launch_copy_in(d_omega, m.psi_b, m.n, m.pitch, st));
  HIP_TRY(none, cav::launch_poisson_rhs(m.psi_b, m.F, m.n, m.pitch, m.h, st));
  HIP_TRY(none, cav::launch_fill(m.psi, m.n, m.pitch, 0.0, st));
  HIP_TRY(none, cav::launch_fill(m.psi_b, m.n, m.pitch, 0.0, st));
  const double tol_hat = m.tol * 0.3 * m.h * m.h;
  const long long spc = unit_sweeps(m);
  HIP_TRY(none, cav::launch_ctl_reset(m.ctl, m.relax, tol_hat, m.max_sweeps, m.stall_window, spc,
                                      st));
  HIP_TRY(none, cav::launch_resid64(m.psi, m.F, nullptr, nullptr, m.n, m.pitch, m.ctl, m.part,
                                    st));
  // chunks of check groups until the device's decision stops the solve; the
  // decision is read into host stack memory
  cav::PoissonCtl c{};
  long long enqueued = 0;
  for (;;) {
    long long units = enqueued == 0 ? std::max<long long>(4, (long long)(0.5 * (m.n - 1) / spc))
                                    : std::max<long long>(2, enqueued / 4);
    units = std::max<long long>(1, std::min<long long>(units, m.max_sweeps / spc + 1));
    for (long long u = 0; u < units; ++u) {
      for (int q = 0; q < m.pairs_per_check; ++q) {
        const int check = (q == m.pairs_per_check - 1) ? 1 : 0;
        HIP_TRY(none, cav::launch_sor64(m.cfg64, m.psi, m.psi_b, m.F, m.n, m.pitch, m.ctl,
                                        m.part, 0, st));
        HIP_TRY(none, cav::launch_sor64(m.cfg64, m.psi_b, m.psi, m.F, m.n, m.pitch, m.ctl,
                                        m.part, check, st));
      }
    }
    enqueued += units;
    HIP_TRY(none, hipMemcpyAsync(&c, m.ctl, sizeof c, hipMemcpyDeviceToHost, st));
    HIP_TRY(none, hipStreamSynchronize(st));
    if (c.state != cav::SOLVE_RUN) break;
    if (enqueued * spc > 2 * m.max_sweeps + 64 * spc)
      return fail(CAVITY_EHIP, "allocation-free Poisson solve made no decision after %lld "
                               "sweeps", enqueued * spc);
  }
  HIP_TRY(none, cav::launch_copy_out(m.psi, d_psi, m.n, m.pitch, st));
  HIP_TRY(none, hipStreamSynchronize(st));
  const double resid = c.last * (10.0 / 3.0) / (m.h * m.h);
  if (info) {
    info->sweeps = c.sweeps;
    info->resid_inf = resid;
    info->floor_limited = c.state == cav::SOLVE_FLOOR ? 1 : 0;
    info->status = c.state == cav::SOLVE_NOCONV ? CAVITY_ENOCONV : CAVITY_OK;
  }
  if (c.state == cav::SOLVE_NONFINITE)
    return fail(CAVITY_ENONFINITE, "non-finite residual in the allocation-free Poisson solve");
  if (c.state == cav::SOLVE_NOCONV)
    return fail(CAVITY_ENOCONV, "allocation-free Poisson solve hit %lld sweeps (residual %g)",
                (long long)c.sweeps, resid);
  return CAVITY_OK;
}

int cavity_fields(cavity_t h, int32_t idx, double* d_psi, double* d_omega, double* d_u,
                  double* d_v) {
  if (!h) return fail(CAVITY_EINVAL, "null handle");
  if (h->poisoned) return fail(CAVITY_ESTATE, "handle poisoned by an earlier failure");
  if (idx < 0 || idx >= h->count) return fail(CAVITY_EINVAL, "idx %d out of range", idx);
  if ((d_u == nullptr) != (d_v == nullptr))
    return fail(CAVITY_EINVAL, "u and v must be requested together");
  HIP_TRY(h, hipSetDevice(h->device));
  Member& m = h->m[idx];
  if (d_psi) HIP_TRY(h, cav::launch_copy_out(m.psi, d_psi, m.n, m.pitch, h->st));
  if (d_omega) HIP_TRY(h, cav::launch_copy_out(m.w[0], d_omega, m.n, m.pitch, h->st));
  if (d_u) HIP_TRY(h, cav::launch_velocity(m.psi, m.n, m.pitch, m.h, m.u_lid, d_u, d_v, h->st));
  return CAVITY_OK;
}

int cavity_relax(cavity_t h, int32_t idx, int32_t sweeps, int32_t arith, double* d_psi_out,
                 int64_t* done) {
  if (!h) return fail(CAVITY_EINVAL, "null handle");
  if (h->poisoned) return fail(CAVITY_ESTATE, "handle poisoned by an earlier failure");
  if (idx < 0 || idx >= h->count) return fail(CAVITY_EINVAL, "idx %d out of range", idx);
  if (sweeps < 0) return fail(CAVITY_EINVAL, "sweeps must be >= 0");
  if (arith != 0 && arith != 1) return fail(CAVITY_EINVAL, "arith must be 0 or 1");
  Member& m = h->m[idx];
  if (arith == 1 && (!m.mixed || d_psi_out))
    return fail(CAVITY_EINVAL, "arith 1 needs a CAVITY_MIXED cavity and no psi output");
  HIP_TRY(h, hipSetDevice(h->device));
  // Scratch: psi_prev / psi_b hold the iterate, F the right-hand side.  The
  // control block is reset with an unreachable tolerance so that no launch
  // returns early.
  HIP_TRY(h, cav::launch_poisson_rhs(m.w[0], m.F, m.n, m.pitch, m.h, h->st));
  HIP_TRY(h, cav::launch_ctl_reset(m.ctl, m.relax, -1.0, 1LL << 62, 1LL << 62, 0, h->st));
  const int per = arith ? m.cfg32.s : m.cfg64.s;
  const int launches = (sweeps + 2 * per - 1) / (2 * per) * 2;
  if (arith == 0) {
    HIP_TRY(h, cav::launch_copy(m.psi, m.psi_prev, m.n, m.pitch, h->st));
    for (int k = 0; k < launches; k += 2) {
      HIP_TRY(h, cav::launch_sor64(m.cfg64, m.psi_prev, m.psi_b, m.F, m.n, m.pitch, m.ctl,
                                   m.part, 0, h->st));
      HIP_TRY(h, cav::launch_sor64(m.cfg64, m.psi_b, m.psi_prev, m.F, m.n, m.pitch, m.ctl,
                                   m.part, 0, h->st));
    }
    if (d_psi_out) HIP_TRY(h, cav::launch_copy_out(m.psi_prev, d_psi_out, m.n, m.pitch, h->st));
  } else {
    HIP_TRY(h, cav::launch_resid64(m.psi, m.F, m.R32, m.d32a, m.n, m.pitch, m.ctl, m.part,
                                   h->st));
    HIP_TRY(h, cav::launch_ctl_reset(m.ctl, m.relax, -1.0, 1LL << 62, 1LL << 62, 0, h->st));
    for (int k = 0; k < launches; k += 2) {
      HIP_TRY(h, cav::launch_sor32(m.cfg32, m.d32a, m.d32b, m.R32, m.n, m.pitch, m.ctl, m.relax,
                                   h->st));
      HIP_TRY(h, cav::launch_sor32(m.cfg32, m.d32b, m.d32a, m.R32, m.n, m.pitch, m.ctl, m.relax,
                                   h->st));
    }
  }
  if (done) *done = (int64_t)launches * per;
  return CAVITY_OK;
}

int cavity_get_tuning(cavity_t h, int32_t idx, cavity_tuning* t) {
  if (!h || !t) return fail(CAVITY_EINVAL, "null argument");
  if (idx == -1) {
    std::memset(t, 0, sizeof *t);
    t->tile_x = h->bcfg64.tx;
    t->tile_y = h->bcfg64.ty;
    t->sweeps_per_launch = h->bcfg64.s;
    t->threads = h->bcfg64.nt;
    t->tile_x32 = h->bcfg32.tx;
    t->tile_y32 = h->bcfg32.ty;
    t->sweeps_per_launch32 = h->bcfg32.s;
    t->threads32 = h->bcfg32.nt;
    t->check_every = (int32_t)(2LL * h->bcfg64.s * h->b_ppc);
    t->inner_sweeps = 2 * h->bcfg32.s * h->b_inner_pairs;
    t->xcd_bands = 0;
    t->sor_omega = 0.0;
    return CAVITY_OK;
  }
  if (idx < 0 || idx >= h->count) return fail(CAVITY_EINVAL, "idx %d out of range", idx);
  const Member& m = h->m[idx];
  std::memset(t, 0, sizeof *t);
  t->tile_x = m.cfg64.tx;
  t->tile_y = m.cfg64.ty;
  t->sweeps_per_launch = m.cfg64.s;
  t->threads = m.cfg64.nt;
  t->tile_x32 = m.cfg32.tx;
  t->tile_y32 = m.cfg32.ty;
  t->sweeps_per_launch32 = m.cfg32.s;
  t->threads32 = m.cfg32.nt;
  t->check_every = (int32_t)(2LL * m.cfg64.s * m.pairs_per_check);
  t->inner_sweeps = m.inner_sweeps;
  t->xcd_bands = m.cfg64.xcd_bands;
  t->solver = m.solver;
  t->sor_omega = m.relax;
  t->warm_degree = m.warm >= 2 ? m.warm_deg : 0;
  return CAVITY_OK;
}

int cavity_set_tuning(cavity_t h, int32_t idx, const cavity_tuning* t) {
  if (!h || !t) return fail(CAVITY_EINVAL, "null argument");
  if (idx == -1) {
    const cav::SorConfig c64{t->tile_x, t->tile_y, t->sweeps_per_launch, t->threads, 0};
    const cav::SorConfig c32{t->tile_x32, t->tile_y32, t->sweeps_per_launch32, t->threads32, 0};
    if (!cav::batch_config_supported(c64, false) || !cav::batch_config_supported(c32, true))
      return fail(CAVITY_EINVAL, "batched kernel configuration is not compiled");
    if (t->check_every < 1 || t->inner_sweeps < 1)
      return fail(CAVITY_EINVAL, "check_every and inner_sweeps must be >= 1");
    h->bcfg64 = c64;
    h->bcfg32 = c32;
    h->b_ppc = std::max(1, (t->check_every + 2 * c64.s - 1) / (2 * c64.s));
    h->b_inner_pairs = std::max(1, (t->inner_sweeps + 2 * c32.s - 1) / (2 * c32.s));
    if (h->exec != CAVITY_EXEC_STREAM) {
      HIP_TRY(h, hipSetDevice(h->device));
      return setup_batch(h);
    }
    destroy_graphs(h);
    return CAVITY_OK;
  }
  if (idx < 0 || idx >= h->count) return fail(CAVITY_EINVAL, "idx %d out of range", idx);
  destroy_graphs(h);
  const cav::SorConfig c64{t->tile_x, t->tile_y, t->sweeps_per_launch, t->threads, t->xcd_bands};
  const cav::SorConfig c32{t->tile_x32, t->tile_y32, t->sweeps_per_launch32, t->threads32,
                           t->xcd_bands};
  if (!cav::sor_config_supported(c64, false))
    return fail(CAVITY_EINVAL, "FP64 sweep kernel %dx%d s=%d nt=%d xcd=%d is not compiled",
                c64.tx, c64.ty, c64.s, c64.nt, c64.xcd_bands);
  if (!cav::sor_config_supported(c32, true))
    return fail(CAVITY_EINVAL, "FP32 sweep kernel %dx%d s=%d nt=%d xcd=%d is not compiled",
                c32.tx, c32.ty, c32.s, c32.nt, c32.xcd_bands);
  if (t->check_every < 1 || t->inner_sweeps < 1)
    return fail(CAVITY_EINVAL, "check_every and inner_sweeps must be >= 1");
  if (!(t->sor_omega > 0.0 && t->sor_omega < 2.0))
    return fail(CAVITY_EINVAL, "sor_omega must lie in (0, 2)");
  if (t->solver != CAVITY_SOLVER_SOR && t->solver != CAVITY_SOLVER_MG)
    return fail(CAVITY_EINVAL, "unknown solver %d", t->solver);
  Member& m = h->m[idx];
  if (t->solver == CAVITY_SOLVER_MG && h->exec != CAVITY_EXEC_STREAM)
    return fail(CAVITY_EINVAL, "the multigrid solver runs in stream execution");
  if (t->solver == CAVITY_SOLVER_MG && m.fixed > 0)
    return fail(CAVITY_EINVAL, "fixed_sweeps runs the SOR solver only");
  if (t->warm_degree < 0 || (t->warm_degree > 0 && (m.warm < 2 || t->warm_degree >= m.warm)))
    return fail(CAVITY_EINVAL, "warm_degree %d outside [1, %d]", t->warm_degree, m.warm - 1);
  if (t->warm_degree > 0 && t->warm_degree != m.warm_deg) {
    m.warm_deg = t->warm_degree;
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, upload_warm_weights(m, h->st));
  }
  m.solver = t->solver;
  m.cfg64 = c64;
  m.cfg32 = c32;
  m.relax = t->sor_omega;
  set_schedule(m, t->check_every, t->inner_sweeps);
  reset_estimates(m);
  destroy_graphs(h);  // captured launches carry the old configuration and relaxation
  return CAVITY_OK;
}

int cavity_autotune(cavity_t h, int32_t idx, const char* cache_path, cavity_tuning* chosen) {
  if (!h) return fail(CAVITY_EINVAL, "null handle");
  if (h->poisoned) return fail(CAVITY_ESTATE, "handle poisoned by an earlier failure");
  if (idx < -1 || idx >= h->count) return fail(CAVITY_EINVAL, "idx %d out of range", idx);
  HIP_TRY(h, hipSetDevice(h->device));
  int rc;
  const std::string key = tune_key(h, idx);
  cavity_tuning t{};
  if (cache_lookup(cache_path, key, &t)) {
    if ((rc = cavity_set_tuning(h, idx, &t)) != CAVITY_OK) return rc;
    if (chosen) *chosen = t;
    return CAVITY_OK;
  }
  if ((rc = cavity_get_tuning(h, idx, &t)) != CAVITY_OK) return rc;
  struct Cand { int tx, ty, s, nt, xcd; };
  static const std::vector<Cand> k64 = {{32, 32, 1, 256, 0}, {32, 32, 2, 256, 0}, {64, 32, 2, 512, 0},
                             {64, 32, 3, 512, 0},  {64, 32, 4, 512, 0},  {64, 64, 3, 512, 0},
                             {64, 64, 3, 768, 0},  {64, 64, 4, 768, 0},
                             {64, 64, 1, 1024, 0}, {64, 64, 2, 1024, 0}, {64, 64, 3, 1024, 0},
                             {64, 64, 2, 512, 0},  {64, 64, 4, 512, 0},  {64, 64, 4, 1024, 0},
                             {96, 64, 2, 1024, 0},
                             {96, 64, 3, 1024, 0}, {92, 50, 4, 1024, 0},
                             {84, 54, 5, 1024, 0}};
  static const std::vector<Cand> k32 = {{32, 32, 1, 256, 0}, {32, 32, 2, 256, 0}, {64, 32, 2, 512, 0},
                             {64, 64, 2, 512, 0}, {64, 64, 2, 1024, 0}, {64, 64, 4, 1024, 0},
                             {64, 64, 6, 1024, 0}, {96, 64, 3, 1024, 0}, {96, 96, 3, 1024, 0},
                             {88, 56, 5, 1024, 0}, {64, 64, 4, 512, 0},  {64, 64, 6, 512, 0}};
  if (idx >= 0) {
    Member& m = h->m[idx];
    // 1. tile shape, sweeps per launch and tile order, by sweep time
    for (int pass = 0; pass < (m.mixed ? 2 : 1); ++pass) {
      const bool fp32 = pass == 1;
      double best = 1e300;
      cav::SorConfig bc = fp32 ? m.cfg32 : m.cfg64;
      const long long cells = (long long)m.n * m.n;
      const int launches = (int)std::max<long long>(8, std::min<long long>(400, 40000000LL / cells));
      for (const Cand& c0 : (fp32 ? k32 : k64)) {
        for (int xcd = 0; xcd < 2; ++xcd) {
          const cav::SorConfig c{c0.tx, c0.ty, c0.s, c0.nt, xcd};
          if (!cav::sor_config_supported(c, fp32)) continue;
          double us = 0;
          if ((rc = time_sweeps(h, m, c, fp32, launches + (launches & 1), &us)) != CAVITY_OK)
            return rc;
          if (us < best) {
            best = us;
            bc = c;
          }
        }
      }
      if (fp32) m.cfg32 = bc; else m.cfg64 = bc;
    }
    // 2. sweep schedule, by the time of complete solves of the current state
    const int u64 = 2 * m.cfg64.s;
    const int u32 = 2 * m.cfg32.s;
    int best_ce = 2 * m.cfg64.s * m.pairs_per_check, best_in = m.inner_sweeps;
    double best_ms = 1e300;
    if (m.solver == CAVITY_SOLVER_MG) {
      // multigrid checks after every V-cycle; nothing to schedule
    } else if (!m.mixed) {
      for (int ce : {8, 16, 32, 64, 128}) {
        if (ce < u64) continue;
        set_schedule(m, ce, best_in);
        double ms = 0;
        if ((rc = time_solve(h, idx, &ms)) != CAVITY_OK) return rc;
        if (ms < best_ms) {
          best_ms = ms;
          best_ce = ce;
        }
      }
    } else {
      for (double f : {0.3, 0.45, 0.6, 0.8, 1.0}) {
        const int in = std::max(u32, (int)std::ceil(f * (m.n - 1)));
        set_schedule(m, best_ce, in);
        double ms = 0;
        if ((rc = time_solve(h, idx, &ms)) != CAVITY_OK) return rc;
        if (ms < best_ms) {
          best_ms = ms;
          best_in = in;
        }
      }
    }
    set_schedule(m, best_ce, best_in);
    reset_estimates(m);
    destroy_graphs(h);
    if ((rc = cavity_get_tuning(h, idx, &t)) != CAVITY_OK) return rc;
  } else {
    // batched kernel: tile shape by the time per persistent round
    const bool mixed = h->mixed;
    double best = 1e300;
    cav::SorConfig bc = mixed ? h->bcfg32 : h->bcfg64;
    for (const Cand& c0 : (mixed ? k32 : k64)) {
      const cav::SorConfig c{c0.tx, c0.ty, c0.s, c0.nt, 0};
      if (!cav::batch_config_supported(c, mixed)) continue;
      double us = 0;
      if ((rc = time_batch(h, c, 48 * 2, &us)) != CAVITY_OK) return rc;
      const double per_sweep = us / c.s;
      if (per_sweep < best) {
        best = per_sweep;
        bc = c;
      }
    }
    if (mixed) h->bcfg32 = bc; else h->bcfg64 = bc;
    h->b_ppc = std::max(1, 32 / (2 * h->bcfg64.s));
    int inner = 0;
    for (const Member& m : h->m) inner = std::max(inner, m.inner_sweeps);
    h->b_inner_pairs = std::max(1, (inner + 2 * h->bcfg32.s - 1) / (2 * h->bcfg32.s));
    if ((rc = setup_batch(h)) != CAVITY_OK) return rc;
    if ((rc = cavity_get_tuning(h, -1, &t)) != CAVITY_OK) return rc;
  }
  if ((rc = collect_totals(h, false)) != CAVITY_OK) return rc;
  cache_store(cache_path, key, t);
  if (chosen) *chosen = t;
  return CAVITY_OK;
}

int cavity_get_exec(cavity_t h, int32_t* mode) {
  if (!h || !mode) return fail(CAVITY_EINVAL, "null argument");
  *mode = h->exec;
  return CAVITY_OK;
}

int cavity_set_exec(cavity_t h, int32_t mode) {
  if (!h) return fail(CAVITY_EINVAL, "null handle");
  if (h->poisoned) return fail(CAVITY_ESTATE, "handle poisoned by an earlier failure");
  if (mode != CAVITY_EXEC_STREAM && mode != CAVITY_EXEC_PERSISTENT && mode != CAVITY_EXEC_GRAPH &&
      mode != CAVITY_EXEC_RESIDENT)
    return fail(CAVITY_EINVAL, "unknown execution mode %d", mode);
  HIP_TRY(h, hipSetDevice(h->device));
  if (mode == CAVITY_EXEC_RESIDENT) {
    // nothing to prepare: eligible solves launch resident, the rest stream
  } else if (mode == CAVITY_EXEC_GRAPH && all_fixed(h)) {
    // coupled mode: the step has no decision to wait for, the graph holds
    // the per-launch kernels as they are
    const int rc = collect_totals(h, false);
    if (rc != CAVITY_OK) return rc;
  } else if (mode != CAVITY_EXEC_STREAM) {
    for (const Member& m : h->m) {
      if (m.mixed != h->mixed)
        return fail(CAVITY_EINVAL, "batched execution needs one precision for all cavities");
      if (m.solver != CAVITY_SOLVER_SOR)
        return fail(CAVITY_EINVAL, "batched execution runs the SOR solver only");
      if (m.fixed > 0)
        return fail(CAVITY_EINVAL, "fixed_sweeps runs in stream or graph execution, with every "
                                   "cavity of the handle in the coupled mode for graphs");
    }
    int rc = setup_batch(h);
    if (rc != CAVITY_OK) return rc;
    rc = collect_totals(h, false);
    if (rc != CAVITY_OK) return rc;
  }
  destroy_graphs(h);
  h->exec = mode;
  return CAVITY_OK;
}

int cavity_destroy(cavity_t h) {
  if (!h) return CAVITY_OK;
  destroy_graphs(h);
  if (h->cap_st) (void)hipStreamDestroy(h->cap_st);
  for (hipStream_t st : h->mst)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : h->mev)
    if (ev) (void)hipEventDestroy(ev);
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->host_bc) (void)hipHostFree(h->host_bc);
  if (h->host_ctl) (void)hipHostFree(h->host_ctl);
  if (h->host_diag) (void)hipHostFree(h->host_diag);
  delete h;
  return CAVITY_OK;
}

}  // extern "C"
