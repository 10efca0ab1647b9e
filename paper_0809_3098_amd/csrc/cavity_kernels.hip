// HIP kernels of the driven-lid-cavity time step, written for gfx950 (MI355X).
//
// Method: N. Cardoso and P. Bicudo, arXiv:0809.3098, Sec. 3.  Field arrays
// are pitched row-major [j][i] (x fastest); walls at i, j in {0, n-1}; the
// lid is row n-1.  h = 1/(n-1) on the unit square.
//
// Stencil work here is bandwidth- or LDS-bound, not a dense contraction, so
// no matrix cores are used.  Wavefronts are 64 lanes; blocks are 256 threads.

#include <float.h>
#include <math.h>

#include "cavity_internal.h"

namespace cav {

namespace {

constexpr int kBlock = 256;
constexpr int kPolishChecks = 2;   // checks of Gauss-Seidel polish before giving up

// ---------------------------------------------------------------------------
// Block reductions (wavefront shuffles, then LDS across the four waves).
// ---------------------------------------------------------------------------
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Max over the block of two non-negative values; result valid in thread 0.
__device__ inline void block_max2(double& a, double& b) {
  __shared__ double red[2][kBlock / 64];
  a = wave_max(a);
  b = wave_max(b);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      a = fmax(a, red[0][w]);
      b = fmax(b, red[1][w]);
    }
  }
}

// NaN-aware magnitude: NaN maps to +Inf so that a max never drops it.
__device__ inline double mag(double r) {
  r = fabs(r);
  return (r != r) ? (double)INFINITY : r;
}

// The decision of a Poisson solve after one residual check (see PoissonCtl).
// r is max |g - psi| in the units of the relaxation formula.
__device__ void decide(PoissonCtl* c, double r, double pm, long long sweeps_done) {
  c->sweeps += sweeps_done;
  c->last = r;
  c->psimax = pm;
  int st = SOLVE_RUN;
  if (!(r <= DBL_MAX)) {
    st = SOLVE_NONFINITE;
  } else if (r <= c->tol_hat) {
    st = SOLVE_CONVERGED;
  } else {
    if (r < 0.5 * c->best) {
      c->best = r;
      c->best_at = c->sweeps;
    }
    if (c->phase == 0) {
      if (c->sweeps - c->best_at >= c->stall_window) {
        // Over-relaxation no longer reduces the residual: its rounding noise
        // is the floor.  Gauss-Seidel sweeps (relaxation 1) damp that noise.
        c->phase = 1;
        c->relax = 1.0;
        c->best = r;
        c->best_at = c->sweeps;
        c->polish_left = kPolishChecks;
      }
    } else if (--c->polish_left <= 0) {
      st = SOLVE_FLOOR;
      c->floor_limited = 1;
    }
    if (st == SOLVE_RUN && c->sweeps >= c->max_sweeps) st = SOLVE_NOCONV;
  }
  c->state = st;
}

// Thread 0 of every block of a checking launch: publish the block maxima;
// the last block to arrive reduces them and decides.
__device__ void finish_check(PoissonCtl* ctl, double rmax, double pmax, long long sweeps_done) {
  atomicMax(&ctl->rbits, (unsigned long long)__double_as_longlong(rmax));
  atomicMax(&ctl->pbits, (unsigned long long)__double_as_longlong(pmax));
  __threadfence();
  const unsigned int nblocks = gridDim.x * gridDim.y;
  const unsigned int t = atomicAdd(&ctl->ticket, 1u);
  if (t == nblocks - 1) {
    __threadfence();
    const double r = __longlong_as_double((long long)atomicAdd(&ctl->rbits, 0ull));
    const double pm = __longlong_as_double((long long)atomicAdd(&ctl->pbits, 0ull));
    ctl->rbits = 0ull;
    ctl->pbits = 0ull;
    ctl->ticket = 0u;
    decide(ctl, r, pm, sweeps_done);
  }
}

// ---------------------------------------------------------------------------
// Temporally blocked four-colour relaxation of eq. (SequationFinal).
//
// For a square grid the relaxation formula is, in correction form,
//   psi_P <- psi_P + w (g_P - psi_P),
//   g_P = 0.2 (E + W + N + S) + 0.05 (NE + NW + SE + SW) + F_P,
//   F_P = (3/(5a)) B_P = 0.025 h^2 (w_E + w_W + w_N + w_S + 8 w_P),
// which equals (3/5)(w/a)(A + B + C) + (1 - w) psi_P.  Colours are the parity
// classes (i mod 2, j mod 2) visited (0,0), (1,0), (0,1), (1,1); no two nodes
// of a class share a nine-point stencil.
//
// A block loads an output tile plus a halo of H = 4S + 2 nodes of psi and F
// into LDS, runs S sweeps (4S colour passes) there, and writes the tile.  A
// node's value after colour pass k is exact when every node within
// Chebyshev distance k of it was loaded, so pass k only updates nodes at
// least k from the region edge, and after 4S passes the tile and its first
// ring are exact: the tile's residual can be evaluated in LDS as well.
// LDS holds each field as four parity planes, so all reads of a colour pass
// are unit-stride across lanes.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY, int S>
struct SorGeom {
  static_assert(TX % 2 == 0 && TY % 2 == 0, "tile sizes must be even");
  static constexpr int H = 4 * S + 2;
  static constexpr int RX = TX + 2 * H;
  static constexpr int RY = TY + 2 * H;
  static constexpr int RXH = RX / 2;
  static constexpr int RYH = RY / 2;
  static constexpr int PLANE = RXH * RYH;
  static constexpr size_t LDS = 2ull * 4ull * PLANE * sizeof(T);
  static_assert(LDS <= 163840, "tile does not fit in 160 KiB of LDS");
};

template <typename T>
__device__ inline T fma_t(T a, T b, T c) { return fma(a, b, c); }
template <>
__device__ inline float fma_t<float>(float a, float b, float c) { return fmaf(a, b, c); }

template <typename T, int TX, int TY, int S, bool CHECK>
__global__ __launch_bounds__(kBlock) void k_sor(const T* __restrict__ pin, T* __restrict__ pout,
                                                const T* __restrict__ F, int n, int pitch,
                                                PoissonCtl* __restrict__ ctl, int tiles_x,
                                                int xcd_bands, double relax_arg) {
  using G = SorGeom<T, TX, TY, S>;
  __shared__ T sp[4 * G::PLANE];
  __shared__ T sf[4 * G::PLANE];
  if (ctl->state != SOLVE_RUN) return;
  const T w = (T)(relax_arg > 0.0 ? relax_arg : ctl->relax);

  const int nb = gridDim.x;
  int tile = blockIdx.x;
  if (xcd_bands && (nb & 7) == 0) tile = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int tyi = tile / tiles_x;
  const int txi = tile - tyi * tiles_x;
  const int x0 = txi * TX - G::H;  // region origin, even
  const int y0 = tyi * TY - G::H;
  const int tid = threadIdx.x;

  // Region load: rows of RX nodes, coalesced along x.
  for (int idx = tid; idx < G::RX * G::RY; idx += kBlock) {
    const int ly = idx / G::RX;
    const int lx = idx - ly * G::RX;
    const int gx = x0 + lx, gy = y0 + ly;
    T v = T(0), f = T(0);
    if ((unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n) {
      const size_t g = (size_t)gy * pitch + gx;
      v = pin[g];
      f = F[g];
    }
    const int o = (((ly & 1) << 1) | (lx & 1)) * G::PLANE + (ly >> 1) * G::RXH + (lx >> 1);
    sp[o] = v;
    sf[o] = f;
  }
  __syncthreads();

  const int lxd0 = 1 - x0, lxd1 = n - 2 - x0;  // domain interior in local coordinates
  const int lyd0 = 1 - y0, lyd1 = n - 2 - y0;
  const int lane = tid & 63, wave = tid >> 6;
  const T c4 = T(0.2), cd = T(0.05);

#pragma unroll 1
  for (int k = 1; k <= 4 * S; ++k) {
    const int c = (k - 1) & 3;
    const int cx = c & 1, cy = c >> 1;
    const int lxlo = max(k, lxd0), lxhi = min(G::RX - 1 - k, lxd1);
    const int lylo = max(k, lyd0), lyhi = min(G::RY - 1 - k, lyd1);
    const int a0 = (lxlo - cx + 1) >> 1, a1 = (lxhi - cx) >> 1;
    const int b0 = (lylo - cy + 1) >> 1, b1 = (lyhi - cy) >> 1;
    T* own = sp + (cy * 2 + cx) * G::PLANE;
    const T* ew = sp + (cy * 2 + (1 - cx)) * G::PLANE;
    const T* ns = sp + ((1 - cy) * 2 + cx) * G::PLANE;
    const T* dg = sp + ((1 - cy) * 2 + (1 - cx)) * G::PLANE;
    const T* ff = sf + (cy * 2 + cx) * G::PLANE;
    for (int bb = b0 + wave; bb <= b1; bb += kBlock / 64) {
      for (int aa = a0 + lane; aa <= a1; aa += 64) {
        const int o = bb * G::RXH + aa;
        const int oE = o + cx;                 // E at oE, W at oE - 1
        const int oN = o + cy * G::RXH;        // N at oN, S at oN - RXH
        const int oNE = oN + cx;               // NE, NW = oNE - 1, SE, SW one row down
        const T s4 = (ew[oE] + ew[oE - 1]) + (ns[oN] + ns[oN - G::RXH]);
        const T sd = (dg[oNE] + dg[oNE - 1]) + (dg[oNE - G::RXH] + dg[oNE - G::RXH - 1]);
        const T p = own[o];
        const T g = fma_t(c4, s4, fma_t(cd, sd, ff[o]));
        own[o] = fma_t(w, g - p, p);
      }
    }
    __syncthreads();
  }

  // Write the tile; with CHECK also its residual max |g - psi| and max |psi|.
  double rmax = 0.0, pmax = 0.0;
  for (int idx = tid; idx < TX * TY; idx += kBlock) {
    const int ty = idx / TX;
    const int lx = G::H + (idx - ty * TX);
    const int ly = G::H + ty;
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx < 1 || gx > n - 2 || gy < 1 || gy > n - 2) continue;
    const int cx = lx & 1, cy = ly & 1;
    const int o = (ly >> 1) * G::RXH + (lx >> 1);
    const T p = sp[(cy * 2 + cx) * G::PLANE + o];
    pout[(size_t)gy * pitch + gx] = p;
    if (CHECK) {
      const T* ew = sp + (cy * 2 + (1 - cx)) * G::PLANE;
      const T* ns = sp + ((1 - cy) * 2 + cx) * G::PLANE;
      const T* dg = sp + ((1 - cy) * 2 + (1 - cx)) * G::PLANE;
      const int oE = o + cx, oN = o + cy * G::RXH, oNE = oN + cx;
      const T s4 = (ew[oE] + ew[oE - 1]) + (ns[oN] + ns[oN - G::RXH]);
      const T sd = (dg[oNE] + dg[oNE - 1]) + (dg[oNE - G::RXH] + dg[oNE - G::RXH - 1]);
      const T g = fma_t(c4, s4, fma_t(cd, sd, sf[(cy * 2 + cx) * G::PLANE + o]));
      rmax = fmax(rmax, mag((double)(g - p)));
      pmax = fmax(pmax, mag((double)p));
    }
  }
  if (CHECK) {
    block_max2(rmax, pmax);
    if (tid == 0) finish_check(ctl, rmax, pmax, 2ll * S);
  }
}

// ---------------------------------------------------------------------------
// Transport right-hand side, eq. (Lwn) with eq. (vel), and the SSPRK stage.
// ---------------------------------------------------------------------------
__device__ inline double transport(const double* __restrict__ psi, const double* __restrict__ w,
                                   size_t p, int pitch, double inv2h, double invh2, double nu) {
  const double u = (psi[p + pitch] - psi[p - pitch]) * inv2h;
  const double v = -(psi[p + 1] - psi[p - 1]) * inv2h;
  const double wP = w[p], wE = w[p + 1], wW = w[p - 1], wN = w[p + pitch], wS = w[p - pitch];
  const double adv = -u * ((wE - wW) * inv2h) - v * ((wN - wS) * inv2h);
  const double dif = nu * (((wE - 2.0 * wP + wW) + (wN - 2.0 * wP + wS)) * invh2);
  return adv + dif;
}

__global__ __launch_bounds__(kBlock) void k_stage(const double* __restrict__ psi,
                                                  const double* __restrict__ w0,
                                                  const double* __restrict__ win,
                                                  const double* __restrict__ wx, double* out,
                                                  const double* wp, double* p_out, int n,
                                                  int pitch, StageArgs a) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n || j >= n) return;
  const size_t p = (size_t)j * pitch + i;
  if (i == 0 || j == 0 || i == n - 1 || j == n - 1) {
    out[p] = win[p];  // the new stage inherits the input stage's wall vorticity
    return;
  }
  const double inv2h = 0.5 / a.h;
  const double invh2 = 1.0 / (a.h * a.h);
  const double L = transport(psi, win, p, pitch, inv2h, invh2, a.nu);
  const double wi = win[p];
  double v = a.a1 * wi;
  if (w0) v = fma(a.a0, w0[p], v);
  if (wx) v = fma(a.ax, wx[p], v);
  out[p] = fma(a.b, L, v);
  if (p_out) p_out[p] = fma(a.pl, L, fma(a.pa, wp[p], a.pb * wi));
}

// ---------------------------------------------------------------------------
// Poisson right-hand side and Thom's wall vorticity.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_poisson_rhs(const double* __restrict__ w,
                                                        double* __restrict__ F, int n, int pitch,
                                                        double cF) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n || j >= n) return;
  const size_t p = (size_t)j * pitch + i;
  if (i == 0 || j == 0 || i == n - 1 || j == n - 1) {
    F[p] = 0.0;
    return;
  }
  F[p] = cF * (((w[p + 1] + w[p - 1]) + (w[p + pitch] + w[p - pitch])) + 8.0 * w[p]);
}

__global__ __launch_bounds__(kBlock) void k_thom(const double* __restrict__ psi,
                                                 double* __restrict__ w, int n, int pitch,
                                                 double h2, double two_u_over_h) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int m = n - 2;
  if (t == 0) {
    w[0] = 0.0;
    w[n - 1] = 0.0;
    w[(size_t)(n - 1) * pitch] = 0.0;
    w[(size_t)(n - 1) * pitch + n - 1] = 0.0;
  }
  if (t >= 4 * m) return;
  const int side = t / m;
  const int k = 1 + (t - side * m);
  if (side == 0) {         // bottom, j = 0
    w[k] = -2.0 * psi[(size_t)pitch + k] / h2;
  } else if (side == 1) {  // lid, j = n-1
    w[(size_t)(n - 1) * pitch + k] = -2.0 * psi[(size_t)(n - 2) * pitch + k] / h2 - two_u_over_h;
  } else if (side == 2) {  // left, i = 0
    w[(size_t)k * pitch] = -2.0 * psi[(size_t)k * pitch + 1] / h2;
  } else {                 // right, i = n-1
    w[(size_t)k * pitch + n - 1] = -2.0 * psi[(size_t)k * pitch + n - 2] / h2;
  }
}

// ---------------------------------------------------------------------------
// Control-block reset and the mixed-precision refinement kernels.
// ---------------------------------------------------------------------------
__global__ void k_ctl_reset(PoissonCtl* c, double relax, double tol_hat, long long max_sweeps,
                            long long stall_window, long long sweeps_per_check) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  c->rbits = 0ull;
  c->pbits = 0ull;
  c->ticket = 0u;
  c->state = SOLVE_RUN;
  c->phase = 0;
  c->polish_left = 0;
  c->relax = relax;
  c->relax_sor = relax;
  c->tol_hat = tol_hat;
  c->best = (double)INFINITY;
  c->last = (double)INFINITY;
  c->psimax = 0.0;
  c->sweeps = 0;
  c->best_at = 0;
  c->max_sweeps = max_sweeps;
  c->stall_window = stall_window;
  c->sweeps_per_check = sweeps_per_check;
  c->floor_limited = 0;
}

// r = g(psi) - psi in FP64 on interior nodes, reduced to max |r| for the solve
// decision; with R32 != nullptr also stored as float for the FP32 correction
// solve, whose correction d32 then starts from zero.
__global__ __launch_bounds__(kBlock) void k_resid64(const double* __restrict__ psi,
                                                    const double* __restrict__ F,
                                                    float* __restrict__ R32,
                                                    float* __restrict__ d32, int n, int pitch,
                                                    PoissonCtl* __restrict__ ctl) {
  if (ctl->state != SOLVE_RUN) return;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  double rmax = 0.0, pmax = 0.0;
  if (i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) {
    const size_t p = (size_t)j * pitch + i;
    const double s4 = (psi[p + 1] + psi[p - 1]) + (psi[p + pitch] + psi[p - pitch]);
    const double sd = (psi[p + pitch + 1] + psi[p + pitch - 1]) +
                      (psi[p - pitch + 1] + psi[p - pitch - 1]);
    const double g = fma(0.2, s4, fma(0.05, sd, F[p]));
    const double r = g - psi[p];
    if (R32) {
      R32[p] = (float)r;
      d32[p] = 0.0f;
    }
    rmax = mag(r);
    pmax = mag(psi[p]);
  }
  block_max2(rmax, pmax);
  if (threadIdx.x == 0) finish_check(ctl, rmax, pmax, 0ll);
}

__global__ __launch_bounds__(kBlock) void k_refine(double* __restrict__ psi,
                                                   const float* __restrict__ d32, int n,
                                                   int pitch, PoissonCtl* __restrict__ ctl,
                                                   int inner_sweeps) {
  if (ctl->state != SOLVE_RUN) return;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) ctl->sweeps += inner_sweeps;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i < 1 || i > n - 2 || j < 1 || j > n - 2) return;
  const size_t p = (size_t)j * pitch + i;
  psi[p] += (double)d32[p];
}

// ---------------------------------------------------------------------------
// Diagnostics (Sec. 3.2 eqs. resS, resV; kinetic energy).  Deterministic:
// fixed grid of blocks, fixed-order partial sums, then one block sums them.
// ---------------------------------------------------------------------------
constexpr int kDiagBlocks = 512;

__global__ __launch_bounds__(kBlock) void k_diag_partial(const double* __restrict__ psi0,
                                                         const double* __restrict__ psi1,
                                                         const double* __restrict__ w0,
                                                         const double* __restrict__ w1, int n,
                                                         int pitch, double inv2h,
                                                         double* __restrict__ partial) {
  double s_psi = 0.0, s_w = 0.0, m_w = 0.0, s_ke = 0.0;
  const long long total = (long long)n * n;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < total;
       t += (long long)gridDim.x * kBlock) {
    const int j = (int)(t / n);
    const int i = (int)(t - (long long)j * n);
    const size_t p = (size_t)j * pitch + i;
    s_psi += fabs(psi1[p] - psi0[p]);
    const double dw = fabs(w1[p] - w0[p]);
    s_w += dw;
    m_w = fmax(m_w, mag(dw));
    if (i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) {
      const double u = (psi1[p + pitch] - psi1[p - pitch]) * inv2h;
      const double v = -(psi1[p + 1] - psi1[p - 1]) * inv2h;
      s_ke = fma(u, u, fma(v, v, s_ke));
    }
  }
  __shared__ double red[4][kBlock];
  red[0][threadIdx.x] = s_psi;
  red[1][threadIdx.x] = s_w;
  red[2][threadIdx.x] = m_w;
  red[3][threadIdx.x] = s_ke;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + s]);
      red[3][threadIdx.x] += red[3][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_diag_final(const double* __restrict__ partial,
                                                       int np, double* __restrict__ out) {
  __shared__ double red[4][kBlock];
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int k = threadIdx.x; k < np; k += kBlock) {
    a += partial[4 * k + 0];
    b += partial[4 * k + 1];
    c = fmax(c, partial[4 * k + 2]);
    d += partial[4 * k + 3];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  red[3][threadIdx.x] = d;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + s]);
      red[3][threadIdx.x] += red[3][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Velocity output (eq. vel, Sec. 3.1 wall values) and layout helpers.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_velocity(const double* __restrict__ psi, int n,
                                                     int pitch, double inv2h, double u_lid,
                                                     double* __restrict__ u,
                                                     double* __restrict__ v) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n || j >= n) return;
  const size_t d = (size_t)j * n + i;
  if (i == 0 || j == 0 || i == n - 1 || j == n - 1) {
    u[d] = (j == n - 1 && i > 0 && i < n - 1) ? u_lid : 0.0;
    v[d] = 0.0;
    return;
  }
  const size_t p = (size_t)j * pitch + i;
  u[d] = (psi[p + pitch] - psi[p - pitch]) * inv2h;
  v[d] = -(psi[p + 1] - psi[p - 1]) * inv2h;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* a, int n, int pitch, T value) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= pitch || j >= n) return;
  a[(size_t)j * pitch + i] = value;
}

// mode 0: dense -> pitched; 1: pitched -> dense; 2: pitched -> pitched;
// 3: pitched -> pitched interior only, walls of dst <- 0.
__global__ __launch_bounds__(kBlock) void k_copy(const double* __restrict__ src,
                                                 double* __restrict__ dst, int n, int pitch,
                                                 int mode) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n || j >= n) return;
  const size_t d = (size_t)j * n + i;
  const size_t p = (size_t)j * pitch + i;
  if (mode == 0) {
    dst[p] = src[d];
  } else if (mode == 1) {
    dst[d] = src[p];
  } else if (mode == 2) {
    dst[p] = src[p];
  } else {
    const bool wall = (i == 0 || j == 0 || i == n - 1 || j == n - 1);
    dst[p] = wall ? 0.0 : src[p];
  }
}

inline dim3 grid2d(int nx, int ny) { return dim3((nx + 63) / 64, (ny + 3) / 4); }

// ---------------------------------------------------------------------------
// Tile-configuration dispatch of the sweep kernels.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY, int S>
hipError_t sor_launch(const T* pin, T* pout, const T* F, int n, int pitch, PoissonCtl* ctl,
                      int check, int xcd_bands, double relax, hipStream_t st) {
  const int tx = (n + TX - 1) / TX, ty = (n + TY - 1) / TY;
  const dim3 grid(tx * ty);
  if (check)
    hipLaunchKernelGGL((k_sor<T, TX, TY, S, true>), grid, dim3(kBlock), 0, st, pin, pout, F, n,
                       pitch, ctl, tx, xcd_bands, relax);
  else
    hipLaunchKernelGGL((k_sor<T, TX, TY, S, false>), grid, dim3(kBlock), 0, st, pin, pout, F, n,
                       pitch, ctl, tx, xcd_bands, relax);
  return hipGetLastError();
}

#define CAV_SOR_CONFIGS(X) \
  X(64, 64, 1)             \
  X(64, 64, 2)             \
  X(64, 64, 3)             \
  X(64, 32, 2)             \
  X(32, 32, 1)             \
  X(32, 32, 2)             \
  X(96, 48, 2)

template <typename T>
hipError_t sor_dispatch(const SorConfig& c, const T* pin, T* pout, const T* F, int n, int pitch,
                        PoissonCtl* ctl, int check, double relax, hipStream_t st) {
#define CAV_TRY(TX_, TY_, S_)                                                            \
  if (c.tx == TX_ && c.ty == TY_ && c.s == S_)                                           \
    return sor_launch<T, TX_, TY_, S_>(pin, pout, F, n, pitch, ctl, check, c.xcd_bands, \
                                       relax, st);
  CAV_SOR_CONFIGS(CAV_TRY)
#undef CAV_TRY
  return hipErrorInvalidValue;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers.
// ---------------------------------------------------------------------------
hipError_t launch_thom(const double* psi, double* omega, int n, int pitch, double h, double u_lid,
                       hipStream_t st) {
  const int m = 4 * (n - 2);
  hipLaunchKernelGGL(k_thom, dim3((m + kBlock - 1) / kBlock), dim3(kBlock), 0, st, psi, omega, n,
                     pitch, h * h, 2.0 * u_lid / h);
  return hipGetLastError();
}

hipError_t launch_poisson_rhs(const double* omega, double* F, int n, int pitch, double h,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_poisson_rhs, grid2d(n, n), dim3(kBlock), 0, st, omega, F, n, pitch,
                     0.025 * h * h);
  return hipGetLastError();
}

hipError_t launch_stage(const double* psi, const double* w0, const double* win, const double* wx,
                        double* out, const double* wp, double* p_out, int n, int pitch,
                        const StageArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_stage, grid2d(n, n), dim3(kBlock), 0, st, psi, w0, win, wx, out, wp,
                     p_out, n, pitch, a);
  return hipGetLastError();
}

hipError_t launch_ctl_reset(PoissonCtl* ctl, double relax, double tol_hat, long long max_sweeps,
                            long long stall_window, long long sweeps_per_check, hipStream_t st) {
  hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st, ctl, relax, tol_hat, max_sweeps,
                     stall_window, sweeps_per_check);
  return hipGetLastError();
}

hipError_t launch_sor64(const SorConfig& cfg, const double* psi_in, double* psi_out,
                        const double* F, int n, int pitch, PoissonCtl* ctl, int check,
                        hipStream_t st) {
  return sor_dispatch<double>(cfg, psi_in, psi_out, F, n, pitch, ctl, check, 0.0, st);
}

hipError_t launch_sor32(const SorConfig& cfg, const float* d_in, float* d_out, const float* R,
                        int n, int pitch, PoissonCtl* ctl, double relax, hipStream_t st) {
  return sor_dispatch<float>(cfg, d_in, d_out, R, n, pitch, ctl, 0, relax, st);
}

hipError_t launch_resid64(const double* psi, const double* F, float* R32, float* d32, int n,
                          int pitch, PoissonCtl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_resid64, grid2d(n, n), dim3(kBlock), 0, st, psi, F, R32, d32, n, pitch,
                     ctl);
  return hipGetLastError();
}

hipError_t launch_refine(double* psi, const float* d32, int n, int pitch, PoissonCtl* ctl,
                         int inner_sweeps, hipStream_t st) {
  hipLaunchKernelGGL(k_refine, grid2d(n, n), dim3(kBlock), 0, st, psi, d32, n, pitch, ctl,
                     inner_sweeps);
  return hipGetLastError();
}

int diag_partials(int n) {
  (void)n;
  return kDiagBlocks;
}

hipError_t launch_diag(const double* psi0, const double* psi1, const double* w0, const double* w1,
                       int n, int pitch, double h, double* partial, int npartial, double* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_diag_partial, dim3(npartial), dim3(kBlock), 0, st, psi0, psi1, w0, w1, n,
                     pitch, 0.5 / h, partial);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kBlock), 0, st, partial, npartial, out);
  return hipGetLastError();
}

hipError_t launch_velocity(const double* psi, int n, int pitch, double h, double u_lid,
                           double* u, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_velocity, grid2d(n, n), dim3(kBlock), 0, st, psi, n, pitch, 0.5 / h,
                     u_lid, u, v);
  return hipGetLastError();
}

hipError_t launch_fill(double* a, int n, int pitch, double value, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<double>, grid2d(pitch, n), dim3(kBlock), 0, st, a, n, pitch, value);
  return hipGetLastError();
}

hipError_t launch_fill32(float* a, int n, int pitch, float value, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<float>, grid2d(pitch, n), dim3(kBlock), 0, st, a, n, pitch, value);
  return hipGetLastError();
}

hipError_t launch_copy_in(const double* dense, double* pitched, int n, int pitch,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_copy, grid2d(n, n), dim3(kBlock), 0, st, dense, pitched, n, pitch, 0);
  return hipGetLastError();
}

hipError_t launch_copy_out(const double* pitched, double* dense, int n, int pitch,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_copy, grid2d(n, n), dim3(kBlock), 0, st, pitched, dense, n, pitch, 1);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int n, int pitch, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, grid2d(n, n), dim3(kBlock), 0, st, src, dst, n, pitch, 2);
  return hipGetLastError();
}

hipError_t launch_copy_interior(const double* src, double* dst, int n, int pitch,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_copy, grid2d(n, n), dim3(kBlock), 0, st, src, dst, n, pitch, 3);
  return hipGetLastError();
}

}  // namespace cav
