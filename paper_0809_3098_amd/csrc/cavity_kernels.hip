// HIP kernels of the driven-lid-cavity time step, written for gfx950 (MI355X).
//
// Method: N. Cardoso and P. Bicudo, arXiv:0809.3098, Sec. 3.  Field arrays
// are pitched row-major [j][i] (x fastest); walls at i, j in {0, n-1}; the
// lid is row n-1.  h = 1/(n-1) on the unit square.
//
// Stencil work here is bound by memory bandwidth, by on-chip data movement
// or by synchronisation, never a dense contraction, so no matrix cores are
// used.  Wavefronts are 64 lanes; the elementwise kernels use 256-thread
// blocks, the sweep kernels 256 to 1024 threads (one tile per block).

#include <float.h>
#include <math.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "cavity_internal.h"

namespace cav {

namespace {

constexpr int kBlock = 256;
constexpr int kPolishChecks = 2;   // checks of Gauss-Seidel polish before giving up

// ---------------------------------------------------------------------------
// Block reductions (wavefront shuffles, then LDS across the waves).
// ---------------------------------------------------------------------------
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Max over the block of two non-negative values; result valid in thread 0.
template <int NT>
__device__ inline void block_max2(double& a, double& b) {
  __shared__ double red[2][NT / 64];
  a = wave_max(a);
  b = wave_max(b);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; ++w) {
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
// A block loads an output tile plus a halo of H = 4S + 2 nodes of psi into
// LDS, runs S sweeps (4S colour passes) there, and writes the tile.  A node's
// value after colour pass k is exact when every node within Chebyshev
// distance k of it was loaded, so pass k only updates nodes at least k from
// the region edge, and after 4S passes the tile and its first ring are exact:
// the tile's residual can be evaluated in LDS as well.  LDS holds psi as four
// parity planes, so all reads of a colour pass are unit-stride across lanes.
//
// Each thread owns one column (lane) of a strip of K rows in every plane; the
// values of its own nodes and their right-hand sides F live in registers, so
// a colour pass reads only neighbours from LDS: one read of the lane's own
// column per neighbour row, the other-side column from the adjacent lane by
// a DPP wavefront shift, and walking up the strip reuses the row below.
// ---------------------------------------------------------------------------
// HX = 2 widens the halo by the ring that the tile's residual reads: after
// 4S passes the nodes at least 4S from the region edge are exact, which is
// all a launch that only sweeps needs (H = 4S); evaluating the residual of
// the tile needs its first ring exact too (H = 4S + 2, even for the parity
// planes).
template <typename T, int TX, int TY, int S, int NT, int HX>
struct SorGeom {
  static_assert(TX % 2 == 0 && TY % 2 == 0, "tile sizes must be even");
  static_assert(NT % 64 == 0, "whole wavefronts");
  static_assert(HX == 0 || HX == 2, "halo extra is 0 or 2");
  static constexpr int H = 4 * S + HX;
  static constexpr int RX = TX + 2 * H;
  static constexpr int RY = TY + 2 * H;
  static constexpr int RXH = RX / 2;
  static constexpr int RYH = RY / 2;
  static constexpr int PLANE = RXH * RYH;
  static constexpr int NW = NT / 64;               // wavefronts
  static constexpr int K = (RYH + NW - 1) / NW;    // plane rows per wavefront
  // LDS: one pad row, the four parity planes, then enough rows that a strip
  // may read one row below its first and one above its last row without a
  // bounds test (those values are never used), and at least 64 slots that
  // take the stores of lanes beyond a plane row.
  static constexpr int BASE = RXH;
  static constexpr int TAIL_ROWS = (NW * K + 1 - RYH) > 0 ? (NW * K + 1 - RYH) : 0;
  static constexpr int SINK = BASE + 4 * PLANE;
  static constexpr int TAIL = TAIL_ROWS * RXH > 64 ? TAIL_ROWS * RXH : 64;
  static constexpr int SLOTS = SINK + TAIL;
  static constexpr size_t LDS = (size_t)SLOTS * sizeof(T);
  static_assert(LDS <= 163840, "tile does not fit in 160 KiB of LDS");
  static_assert(RXH <= 64, "a plane row must fit one wavefront");
};

// Value held by the lane one to the left (DPP wave_shr:1) or one to the right
// (wave_shl:1); the lane without a source receives 0.
template <int CTRL>
__device__ inline double lane_shift(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline float lane_shift(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
constexpr int kDppShr1 = 0x138;  // from lane - 1
constexpr int kDppShl1 = 0x130;  // from lane + 1

template <typename T>
__device__ inline T fma_t(T a, T b, T c) { return fma(a, b, c); }
template <>
__device__ inline float fma_t<float>(float a, float b, float c) { return fmaf(a, b, c); }

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

// The relaxation target of eq. (SequationFinal) in correction form for one
// node of x-parity CX (see the sweep comment above):
//   g = 0.2 (E + W + N + S) + 0.05 (NE + NW + SE + SW) + F.
// Its E / W and diagonal neighbours come in pairs: one node in this lane
// (e, dn, ds) and one in the adjacent lane, which holds the same kind of node
// for its own column.  So the lane's share
//   q = e + 0.25 (dn + ds)
// and the adjacent lane's q, fetched by one wavefront shift, give
//   g = 0.2 ((q + q_adjacent) + (sn + ss)) + F,
// the same sum (0.25 = 0.05 / 0.2 is exact) with one shifted value per node
// instead of three.  For CX = 0 the other-side column is the left lane's, for
// CX = 1 the right lane's.
template <int CX, typename T>
__device__ __forceinline__ T gs_target(T e, T sn, T ss, T dn, T ds, T f) {
  constexpr int kOther = CX == 0 ? kDppShr1 : kDppShl1;
  const T q = fma_t(T(0.25), dn + ds, e);
  return fma_t(T(0.2), (q + lane_shift<kOther>(q)) + (sn + ss), f);
}

// The rows of colour C in a thread's strip that pass k updates (row r while
// k <= ky[r]); xs / xd: the N / S and diagonal neighbour values of the row
// beyond the strip (from LDS), used by the row visited last.  (A second copy
// of the loop without the row tests, for strips that lie inside the pass,
// doubled the vector instructions per sweep: the compiler copied the register
// arrays between the two versions.)
template <typename T, int K, int C>
__device__ __forceinline__ void strip_rows(T (&pv)[4][K], const T (&fv)[4][K], T xs, T xd, T wl,
                                           int k, const int (&ky)[K]) {
  constexpr int cx = C & 1, cy = C >> 1;
  constexpr int EW = cy * 2 + (1 - cx), NS = (1 - cy) * 2 + cx, DG = (1 - cy) * 2 + (1 - cx);
  if (cy == 0) {
    // rows K-1 down to 0; row r's N-side neighbours are in row r of the
    // y-parity-1 planes, its S-side ones in row r - 1 (LDS for r = 0)
    T sN = pv[NS][K - 1], dN = pv[DG][K - 1];
#pragma unroll
    for (int r = K - 1; r >= 0; --r) {
      const T sS = r > 0 ? pv[NS][r - 1] : xs;
      const T dS = r > 0 ? pv[DG][r - 1] : xd;
      if (k <= ky[r]) {  // wave-uniform
        const T p = pv[C][r];
        pv[C][r] = fma_t(wl, gs_target<cx>(pv[EW][r], sN, sS, dN, dS, fv[C][r]) - p, p);
      }
      sN = sS;
      dN = dS;
    }
  } else {
    // rows 0 up to K-1; row r's S-side neighbours are in row r of the
    // y-parity-0 planes, its N-side ones in row r + 1 (LDS for r = K - 1)
    T sS = pv[NS][0], dS = pv[DG][0];
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const T sN = r + 1 < K ? pv[NS][r + 1] : xs;
      const T dN = r + 1 < K ? pv[DG][r + 1] : xd;
      if (k <= ky[r]) {  // wave-uniform
        const T p = pv[C][r];
        pv[C][r] = fma_t(wl, gs_target<cx>(pv[EW][r], sN, sS, dN, dS, fv[C][r]) - p, p);
      }
      sS = sN;
      dS = dN;
    }
  }
}

// The last pass of a launch in which a node takes part.  Pass k (1 ... 4S)
// updates the domain's interior nodes at least k nodes from the region's edge
// (everything within distance k of such a node was loaded, so its value after
// the pass is exact): a node at local (x, y) while k <= min(x, RX - 1 - x)
// and k <= min(y, RY - 1 - y), a node outside the domain's interior never.
// kx: per lane, for its x-parity 0 and 1 columns; ky: per plane row r of the
// strip, for y-parity 0 and 1 (wave-uniform, scalar registers); kyall: the
// last pass in which the strip has a row of that y-parity.  Computed once per
// launch, they leave each pass one comparison per lane and per row.
template <int K>
struct PassLimits {
  int kx[2];
  int ky[2][K];
  int kyall[2];
};

template <typename T, int TX, int TY, int S, int NT, int HX>
__device__ __forceinline__ PassLimits<SorGeom<T, TX, TY, S, NT, HX>::K> pass_limits(
    int lxd0, int lxd1, int lyd0, int lyd1, int lane, int b0) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  PassLimits<G::K> lim;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int x = 2 * lane + c;
    lim.kx[c] = (x >= lxd0 && x <= lxd1) ? min(x, G::RX - 1 - x) : -1;
    lim.kyall[c] = -1;
#pragma unroll
    for (int r = 0; r < G::K; ++r) {
      const int y = 2 * (b0 + r) + c;
      lim.ky[c][r] = (y >= lyd0 && y <= lyd1) ? min(y, G::RY - 1 - y) : -1;
      lim.kyall[c] = max(lim.kyall[c], lim.ky[c][r]);
    }
  }
  return lim;
}

// One colour pass C (parity class (C & 1, C >> 1)) of pass number k over the
// nodes this thread owns.  sp points at the first plane.
//
// Thread (wave q, lane l) owns the nodes x = 2l, 2l + 1 and y = 2b, 2b + 1 for
// the K plane rows b = b0 ... b0 + K - 1 of its strip: a 2 x 2K block holding
// all four colours, kept in pv.  The owner is the only thread that updates a
// node, so pv is always current, and a node's eight neighbours are
//   * E / W: the other-x-parity node of the same row, in pv, and the same
//     colour in the adjacent lane (DPP wavefront shift);
//   * N / S: the other-y-parity nodes of rows b and b -/+ 1, in pv except the
//     row beyond the strip's end;
//   * diagonals: as N / S in the fourth colour, with the lane shift.
// Only that row beyond the strip (below its first row for cy = 0, above its
// last for cy = 1) crosses to another wavefront: its owner publishes it in
// LDS, and the caller reads it once per pair of passes (xs: the N / S
// neighbour plane's value, xd: the diagonal plane's).  After updating colour
// C a strip therefore publishes one row: its first for cy = 0 (read by the
// strip below in the cy = 1 passes), its last for cy = 1 (read by the strip
// above in the next sweep's cy = 0 passes).  Passes 0 and 1 read only what
// passes 2 and 3 of the previous sweep published, passes 2 and 3 only what
// passes 0 and 1 published, so a barrier after passes 1 and 3 orders every
// exchange and also keeps each published row from being overwritten while
// still read.
//
// The row that needs the value from LDS is visited last: top-down for
// cy = 0, bottom-up for cy = 1, so the LDS read's latency hides behind the
// other rows' updates.
//
// Lanes outside the pass relax with 0 (they keep their value) so the pass
// has no divergent branch; rows outside it are skipped (wave-uniform).  Only
// the edge nodes of the region lack a neighbour (cx = 0: lane 0; cx = 1: the
// last column; the first and last plane rows), and no pass updates them.
template <typename T, int TX, int TY, int S, int NT, int HX, int C>
__device__ __forceinline__ void colour_pass(T* sp, T (&pv)[4][SorGeom<T, TX, TY, S, NT, HX>::K],
                                            const T (&fv)[4][SorGeom<T, TX, TY, S, NT, HX>::K],
                                            int k,
                                            const PassLimits<SorGeom<T, TX, TY, S, NT, HX>::K>& lim,
                                            int lane, int b0, T w, T xs, T xd) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  constexpr int K = G::K;
  constexpr int cx = C & 1, cy = C >> 1;
  const T wl = (k <= lim.kx[cx]) ? w : T(0);
  if (k <= lim.kyall[cy]) {  // wave-uniform
    strip_rows<T, K, C>(pv, fv, xs, xd, wl, k, lim.ky[cy]);
    // publish the strip's boundary row of colour C (lanes beyond a plane row
    // store to the sink)
    constexpr int rp = cy == 0 ? 0 : K - 1;
    if (b0 + rp < G::RYH) {
      const int o = lane < G::RXH ? C * G::PLANE + (b0 + rp) * G::RXH + lane
                                  : G::SINK - G::BASE + lane;
      sp[o] = pv[C][rp];
    }
  }
  if (C == 1 || C == 3) __syncthreads();
}

// Residual of colour C over the tile's own interior nodes after the sweeps:
// max |g - psi| and max |psi| accumulated into rmax / pmax.  Same neighbour
// values and the same arithmetic as the update, no stores; called after the
// sweeps' final barrier, when every published boundary row is current.
template <typename T, int TX, int TY, int S, int NT, int HX, int C>
__device__ __forceinline__ void residual_pass(const T* pl,
                                              const T (&pv)[4][SorGeom<T, TX, TY, S, NT, HX>::K],
                                              const T (&fv)[4][SorGeom<T, TX, TY, S, NT, HX>::K],
                                              int lxd0, int lxd1, int lyd0, int lyd1, int lane,
                                              int b0, double& rmax, double& pmax) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  constexpr int K = G::K;
  constexpr int cx = C & 1, cy = C >> 1;
  constexpr int EW = cy * 2 + (1 - cx), NS = (1 - cy) * 2 + cx, DG = (1 - cy) * 2 + (1 - cx);
  const int lxlo = max(G::H, lxd0), lxhi = min(G::H + TX - 1, lxd1);
  const int lylo = max(G::H, lyd0), lyhi = min(G::H + TY - 1, lyd1);
  const int a0 = (lxlo - cx + 1) >> 1, a1 = (lxhi - cx) >> 1;
  const int r_lo = max((lylo - cy + 1) >> 1, b0) - b0;
  const int r_hi = min((lyhi - cy) >> 1, b0 + K - 1) - b0;
  if (r_lo > r_hi) return;
  const int ic = min(lane, G::RXH - 1);
  const bool lane_in = lane >= a0 && lane <= a1;
  T sS, dS, bN = T(0), bdN = T(0);
  if (cy == 0) {
    sS = pl[NS * G::PLANE + (b0 - 1) * G::RXH + ic];
    dS = pl[DG * G::PLANE + (b0 - 1) * G::RXH + ic];
  } else {
    sS = pv[NS][0];
    dS = pv[DG][0];
    bN = pl[NS * G::PLANE + (b0 + K) * G::RXH + ic];
    bdN = pl[DG * G::PLANE + (b0 + K) * G::RXH + ic];
  }
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const T sN = cy == 0 ? pv[NS][r] : (r + 1 < K ? pv[NS][r + 1] : bN);
    const T dN = cy == 0 ? pv[DG][r] : (r + 1 < K ? pv[DG][r + 1] : bdN);
    if (r >= r_lo && r <= r_hi) {  // wave-uniform
      const T p = pv[C][r];
      const T g = gs_target<cx>(pv[EW][r], sN, sS, dN, dS, fv[C][r]);
      if (lane_in) {
        rmax = fmax(rmax, mag((double)(g - p)));
        pmax = fmax(pmax, mag((double)p));
      }
    }
    sS = sN;
    dS = dN;
  }
}

// Device-coherent 8-byte accesses: agent-scope relaxed atomics, which the
// compiler emits as loads and stores with the device-scope cache bit, so a
// value stored on one XCD is seen by a load on another without writing back
// or invalidating whole L2 caches.
template <typename T>
__device__ inline T coh_load(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void coh_store(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Device-coherent 16-byte accesses of a pair of doubles: buffer loads and
// stores with the device-scope cache bit (sc1), through a buffer resource
// over the whole array (records beyond it read 0 and are not written, so a
// wrong offset cannot fault).  One instruction per pair instead of two
// 8-byte atomics.
constexpr int kCacheSc1 = 16;                  // cache-policy bit sc1
constexpr int kBufferDword3 = 0x00020000;      // raw buffer, 32-bit data format
__device__ inline __amdgpu_buffer_rsrc_t coh_buffer(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                           (int)min(bytes, (size_t)0x7fffffff), kBufferDword3);
}
__device__ inline double2 coh_load_pair(__amdgpu_buffer_rsrc_t r, size_t index) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(
                                         r, (int)(index * sizeof(double)), 0, kCacheSc1));
}
__device__ inline void coh_store_pair(__amdgpu_buffer_rsrc_t r, size_t index, double a, double b) {
  double2 v;
  v.x = a;
  v.y = b;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r,
                                         (int)(index * sizeof(double)), 0, kCacheSc1);
}

// Wait until this wavefront's global loads and stores have completed (and its
// device-scope stores are visible device-wide): s_waitcnt vmcnt(0).
__device__ inline void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// s_waitcnt lgkmcnt(0) (vmcnt and expcnt left at their maxima): every LDS
// and scalar memory read of this wavefront has returned.
constexpr int kWaitLgkm0 = 0xC07F;

// Phases of a tile, shared by the per-launch, batched and resident kernels.
// Region coordinates: x0, y0 is the global position of local (0, 0), even.

// psi of the region into the LDS planes, in pairs of nodes (x even, x odd)
// coalesced along x; the global loads of CHUNK pairs per thread are issued
// before their LDS stores (all of them by default; fewer keep fewer values
// live).  RING skips the pairs inside the tile (their LDS values are kept).
template <typename T, int TX, int TY, int S, int NT, int HX, bool RING, int CHUNK = 0,
          bool COHERENT = false>
__device__ __forceinline__ void region_to_lds(const T* __restrict__ pin, int n, int pitch, int x0,
                                              int y0, T* pl, int tid) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  using T2 = typename Pair<T>::type;
  constexpr int RXP = G::RX / 2;
  constexpr int NPAIR = RXP * G::RY;
  constexpr int NL = (NPAIR + NT - 1) / NT;
  constexpr int CH = (CHUNK > 0 && CHUNK < NL) ? CHUNK : NL;
  static_assert(!COHERENT || std::is_same<T, double>::value, "coherent tiles are FP64");
  const __amdgpu_buffer_rsrc_t crs = coh_buffer(pin, (size_t)n * pitch * sizeof(T));
#pragma unroll
  for (int q0 = 0; q0 < NL; q0 += CH) {
    T2 lv[CH];
    bool st[CH], zy[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int idx = tid + (q0 + j) * NT;
      lv[j].x = lv[j].y = T(0);
      zy[j] = false;
      const int ly = idx / RXP;
      const int lx = 2 * (idx - ly * RXP);
      st[j] = q0 + j < NL && idx < NPAIR &&
              !(RING && lx >= G::H && lx < G::H + TX && ly >= G::H && ly < G::H + TY);
      if (st[j]) {
        const int gx = x0 + lx, gy = y0 + ly;
        if ((unsigned)gy < (unsigned)n && (unsigned)gx < (unsigned)n) {
          const size_t g = (size_t)gy * pitch + gx;
          if constexpr (COHERENT) {
            // the same pair load with the device-scope bit (FP64 only)
            lv[j] = coh_load_pair(crs, g);
            zy[j] = gx + 1 >= n;
          } else {
            // One 16-byte load per pair, even for the last pair of an odd
            // grid: gx is even and the pitch even and above n - 1, so gx + 1
            // is still inside the row; that node lies beyond the grid and is
            // replaced by 0 when the pair is stored.  (A second, narrower
            // load in another branch would write the same registers, and a
            // select here would use the value: either makes the next load
            // wait for this one.)
            lv[j] = *reinterpret_cast<const T2*>(pin + g);
            zy[j] = gx + 1 >= n;
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int idx = tid + (q0 + j) * NT;
      if (st[j]) {
        const int ly = idx / RXP;
        const int o = ((ly & 1) << 1) * G::PLANE + (ly >> 1) * G::RXH + (idx - ly * RXP);
        pl[o] = lv[j].x;
        pl[o + G::PLANE] = zy[j] ? T(0) : lv[j].y;
      }
    }
  }
}

// Right-hand side of the owned nodes, straight into registers: the nodes of
// x parity 0 and 1 at one lane and row are neighbours in memory, so one pair
// load serves colours (0, cy) and (1, cy).
template <typename T, int TX, int TY, int S, int NT, int HX>
__device__ __forceinline__ void rhs_to_regs(const T* __restrict__ F, int n, int pitch, int x0,
                                            int y0, int lane, int b0,
                                            T (&fv)[4][SorGeom<T, TX, TY, S, NT, HX>::K]) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  using T2 = typename Pair<T>::type;
  // one pair load per lane and row, as for psi (gx + 1 stays inside the
  // pitch); rhs_zero_beyond clears the node beyond an odd grid afterwards
  const int gx = x0 + 2 * lane;
#pragma unroll
  for (int cy = 0; cy < 2; ++cy) {
#pragma unroll
    for (int r = 0; r < G::K; ++r) {
      const int gy = y0 + 2 * (b0 + r) + cy;
      T2 f;
      f.x = f.y = T(0);
      if (lane < G::RXH && b0 + r < G::RYH && (unsigned)gy < (unsigned)n &&
          (unsigned)gx < (unsigned)n)
        f = *reinterpret_cast<const T2*>(F + (size_t)gy * pitch + gx);
      fv[2 * cy][r] = f.x;
      fv[2 * cy + 1][r] = f.y;
    }
  }
}

// psi of the owned nodes straight into registers, one pair load per lane and
// row as for F (coalesced along x: a wavefront reads one plane row pair of
// the region); nodes outside the grid, and the node beyond an odd grid's last
// column, are 0.  COHERENT loads carry the device-scope bit (persistent
// kernels, whose tiles other blocks wrote in this launch).
template <typename T, int TX, int TY, int S, int NT, int HX, bool COHERENT>
__device__ __forceinline__ void psi_to_regs(const T* __restrict__ pin, int n, int pitch, int x0,
                                            int y0, int lane, int b0,
                                            T (&pv)[4][SorGeom<T, TX, TY, S, NT, HX>::K]) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  using T2 = typename Pair<T>::type;
  static_assert(!COHERENT || std::is_same<T, double>::value, "coherent tiles are FP64");
  const __amdgpu_buffer_rsrc_t crs = coh_buffer(pin, (size_t)n * pitch * sizeof(T));
  const int gx = x0 + 2 * lane;
#pragma unroll
  for (int cy = 0; cy < 2; ++cy) {
#pragma unroll
    for (int r = 0; r < G::K; ++r) {
      const int gy = y0 + 2 * (b0 + r) + cy;
      T2 f;
      f.x = f.y = T(0);
      if (lane < G::RXH && b0 + r < G::RYH && (unsigned)gy < (unsigned)n &&
          (unsigned)gx < (unsigned)n) {
        const size_t g = (size_t)gy * pitch + gx;
        if constexpr (COHERENT)
          f = coh_load_pair(crs, g);
        else
          f = *reinterpret_cast<const T2*>(pin + g);
      }
      pv[2 * cy][r] = f.x;
      pv[2 * cy + 1][r] = f.y;
    }
  }
}

// The rows of a strip that the neighbouring strips read before any pass has
// published them: its last row of the y-parity-1 planes (read by the strip
// above in passes 0 and 1) and its first row of the y-parity-0 planes (read
// by the strip below in passes 2 and 3).  Rows that no pass ever updates (a
// wall, nodes outside the grid) keep these values.
template <typename T, int TX, int TY, int S, int NT, int HX>
__device__ __forceinline__ void publish_strip_edges(T* pl, int lane, int b0,
                                                    const T (&pv)[4][SorGeom<T, TX, TY, S, NT, HX>::K]) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  constexpr int K = G::K;
  if (lane >= G::RXH) return;  // lanes beyond a plane row own no node
  if (b0 + K - 1 < G::RYH) {
    const int o = (b0 + K - 1) * G::RXH + lane;
    pl[2 * G::PLANE + o] = pv[2][K - 1];
    pl[3 * G::PLANE + o] = pv[3][K - 1];
  }
  if (b0 < G::RYH) {
    const int o = b0 * G::RXH + lane;
    pl[o] = pv[0][0];
    pl[G::PLANE + o] = pv[1][0];
  }
}

// The right-hand side of the node beyond an odd grid (x = n, in the pitch
// padding) to 0.  Called once the following loads are issued too: using the
// values earlier would make those loads wait.
template <typename T, int TX, int TY, int S, int NT, int HX>
__device__ __forceinline__ void rhs_zero_beyond(int n, int x0, int lane,
                                                T (&fv)[4][SorGeom<T, TX, TY, S, NT, HX>::K]) {
  if (x0 + 2 * lane + 1 < n) return;
#pragma unroll
  for (int cy = 0; cy < 2; ++cy) {
#pragma unroll
    for (int r = 0; r < SorGeom<T, TX, TY, S, NT, HX>::K; ++r) fv[2 * cy + 1][r] = T(0);
  }
}

// The owned nodes' psi from the LDS planes; RING refreshes only the nodes
// outside the tile.
template <typename T, int TX, int TY, int S, int NT, int HX, bool RING>
__device__ __forceinline__ void lds_to_regs(const T* pl, int lane, int b0,
                                            T (&pv)[4][SorGeom<T, TX, TY, S, NT, HX>::K]) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int r = 0; r < G::K; ++r) {
      const int lx = 2 * lane + (c & 1), ly = 2 * (b0 + r) + (c >> 1);
      const bool in = lane < G::RXH && b0 + r < G::RYH;
      const bool inner = lx >= G::H && lx < G::H + TX && ly >= G::H && ly < G::H + TY;
      if (!RING) {
        pv[c][r] = in ? pl[c * G::PLANE + (b0 + r) * G::RXH + lane] : T(0);
      } else if (in && !inner) {
        pv[c][r] = pl[c * G::PLANE + (b0 + r) * G::RXH + lane];
      }
    }
  }
}

// S sweeps = 4S colour passes over the region.  The rows beyond the strip
// are read from LDS once per pair of passes, right after the barrier that
// makes them current: below the strip, the y-parity-1 planes (2 and 3) for
// passes 0 and 1; above it, the y-parity-0 planes (0 and 1) for passes 2 and
// 3.  Neither pass of a pair writes the planes the pair reads.  (The padding
// rows keep both reads inside LDS; their values are used only for rows
// inside a pass.)
template <typename T, int TX, int TY, int S, int NT, int HX>
__device__ __forceinline__ void tile_sweeps(T* pl, T (&pv)[4][SorGeom<T, TX, TY, S, NT, HX>::K],
                                            const T (&fv)[4][SorGeom<T, TX, TY, S, NT, HX>::K],
                                            int lxd0, int lxd1, int lyd0, int lyd1, int lane,
                                            int b0, T w) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  const int ic = min(lane, G::RXH - 1);
  const T* below = pl + (b0 - 1) * G::RXH + ic;
  const T* above = pl + (b0 + G::K) * G::RXH + ic;
  const PassLimits<G::K> lim = pass_limits<T, TX, TY, S, NT, HX>(lxd0, lxd1, lyd0, lyd1, lane, b0);
#pragma unroll 1
  for (int s = 0; s < S; ++s) {
    const int k = 4 * s;
    const T l2 = below[2 * G::PLANE], l3 = below[3 * G::PLANE];
    colour_pass<T, TX, TY, S, NT, HX, 0>(pl, pv, fv, k + 1, lim, lane, b0, w, l2, l3);
    colour_pass<T, TX, TY, S, NT, HX, 1>(pl, pv, fv, k + 2, lim, lane, b0, w, l3, l2);
    const T u0 = above[0], u1 = above[G::PLANE];
    colour_pass<T, TX, TY, S, NT, HX, 2>(pl, pv, fv, k + 3, lim, lane, b0, w, u0, u1);
    colour_pass<T, TX, TY, S, NT, HX, 3>(pl, pv, fv, k + 4, lim, lane, b0, w, u1, u0);
  }
}

// Write the owned tile nodes, a pair (x even, x odd) per store where both
// are interior nodes of the domain.
template <typename T, int TX, int TY, int S, int NT, int HX, bool COHERENT = false>
__device__ __forceinline__ void tile_to_global(T* __restrict__ pout, int n, int pitch, int x0,
                                               int y0, int lane, int b0,
                                               const T (&pv)[4][SorGeom<T, TX, TY, S, NT, HX>::K]) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  using T2 = typename Pair<T>::type;
  static_assert(!COHERENT || std::is_same<T, double>::value, "coherent tiles are FP64");
  const __amdgpu_buffer_rsrc_t crs = coh_buffer(pout, (size_t)n * pitch * sizeof(T));
#pragma unroll
  for (int cy = 0; cy < 2; ++cy) {
#pragma unroll
    for (int r = 0; r < G::K; ++r) {
      const int b = b0 + r;
      const int lx = 2 * lane, ly = 2 * b + cy;
      // both nodes of the pair are in the tile or neither (H and TX even)
      if (lane >= G::RXH || b >= G::RYH) continue;
      if (lx < G::H || lx >= G::H + TX || ly < G::H || ly >= G::H + TY) continue;
      const int gx = x0 + lx, gy = y0 + ly;
      if (gy < 1 || gy > n - 2) continue;
      const bool in0 = gx >= 1 && gx <= n - 2;
      const bool in1 = gx + 1 <= n - 2;  // gx + 1 >= 1 always
      const size_t g = (size_t)gy * pitch + gx;
      if constexpr (COHERENT) {
        if (in0 && in1) {
          coh_store_pair(crs, g, pv[2 * cy][r], pv[2 * cy + 1][r]);
        } else {
          if (in0) coh_store(pout + g, pv[2 * cy][r]);
          if (in1) coh_store(pout + g + 1, pv[2 * cy + 1][r]);
        }
      } else if (in0 && in1) {
        // streaming store: the next launch reads psi from the memory side
        // anyway, and the kernel's end then has fewer lines to write back
        typedef T V2 __attribute__((ext_vector_type(2)));
        V2 v;
        v.x = pv[2 * cy][r];
        v.y = pv[2 * cy + 1][r];
        __builtin_nontemporal_store(v, reinterpret_cast<V2*>(pout + g));
      } else if (in0) {
        pout[g] = pv[2 * cy][r];
      } else if (in1) {
        pout[g + 1] = pv[2 * cy + 1][r];
      }
    }
  }
}

// Residual max |g - psi| and max |psi| over the tile (valid in thread 0).
template <typename T, int TX, int TY, int S, int NT, int HX>
__device__ __forceinline__ void tile_residual(const T* pl,
                                              const T (&pv)[4][SorGeom<T, TX, TY, S, NT, HX>::K],
                                              const T (&fv)[4][SorGeom<T, TX, TY, S, NT, HX>::K],
                                              int lxd0, int lxd1, int lyd0, int lyd1, int lane,
                                              int b0, double& rmax, double& pmax) {
  rmax = 0.0;
  pmax = 0.0;
  residual_pass<T, TX, TY, S, NT, HX, 0>(pl, pv, fv, lxd0, lxd1, lyd0, lyd1, lane, b0, rmax, pmax);
  residual_pass<T, TX, TY, S, NT, HX, 1>(pl, pv, fv, lxd0, lxd1, lyd0, lyd1, lane, b0, rmax, pmax);
  residual_pass<T, TX, TY, S, NT, HX, 2>(pl, pv, fv, lxd0, lxd1, lyd0, lyd1, lane, b0, rmax, pmax);
  residual_pass<T, TX, TY, S, NT, HX, 3>(pl, pv, fv, lxd0, lxd1, lyd0, lyd1, lane, b0, rmax, pmax);
  block_max2<NT>(rmax, pmax);
}

// One tile of S sweeps, shared by the per-launch kernel and the persistent
// batched kernel.  sp is the block's LDS.  With CHECK the block-wide maxima
// of |g - psi| and |psi| over the tile are returned in thread 0's rmax / pmax.
// run = false (block-uniform) ends the tile once its loads are done, before
// any sweep or store, and returns false: a caller whose go-ahead is itself a
// memory read passes it here so that its latency overlaps the region loads.
template <typename T, int TX, int TY, int S, int NT, int HX, bool COH = false>
__device__ __forceinline__ bool sor_tile(const T* __restrict__ pin, T* __restrict__ pout,
                                         const T* __restrict__ F, int n, int pitch, int tile,
                                         int tiles_x, T w, T* sp, bool CHECK, double& rmax_out,
                                         double& pmax_out, bool run = true) {
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  constexpr int K = G::K;
  T* const pl = sp + G::BASE;  // first parity plane
  const int tyi = tile / tiles_x;
  const int txi = tile - tyi * tiles_x;
  const int x0 = txi * TX - G::H;  // region origin, even
  const int y0 = tyi * TY - G::H;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the wavefront index is uniform: keeping it in a scalar register makes the
  // per-row range tests of the colour passes scalar branches
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int b0 = wave * K;         // first owned row of every plane
  T fv[4][K];
  T pv[4][K];
  rhs_to_regs<T, TX, TY, S, NT, HX>(F, n, pitch, x0, y0, lane, b0, fv);
  if constexpr (std::is_same<T, double>::value) {
    // FP64: psi of the owned nodes straight into registers (all loads in
    // flight before the first use); only the strip edges the neighbouring
    // strips read go through LDS (measured: 146 -> 120 us per launch of the
    // 4096^2 sweep, unchanged at 1024^2)
    psi_to_regs<T, TX, TY, S, NT, HX, COH>(pin, n, pitch, x0, y0, lane, b0, pv);
    rhs_zero_beyond<T, TX, TY, S, NT, HX>(n, x0, lane, fv);
    if (x0 + 2 * lane + 1 >= n) {
#pragma unroll
      for (int r = 0; r < K; ++r) {
        pv[1][r] = T(0);
        pv[3][r] = T(0);
      }
    }
    publish_strip_edges<T, TX, TY, S, NT, HX>(pl, lane, b0, pv);
    __syncthreads();
    if (!run) return false;
  } else {
    // FP32: the region through LDS (measured 4 % faster than the direct
    // loads at 1024^2 and 4096^2: 11.4 against 11.8 us, 98.7 against
    // 103.7 us per launch)
    region_to_lds<T, TX, TY, S, NT, HX, false, 0, COH>(pin, n, pitch, x0, y0, pl, tid);
    rhs_zero_beyond<T, TX, TY, S, NT, HX>(n, x0, lane, fv);
    __syncthreads();
    if (!run) return false;
    lds_to_regs<T, TX, TY, S, NT, HX, false>(pl, lane, b0, pv);
  }
  const int lxd0 = 1 - x0, lxd1 = n - 2 - x0;  // domain interior in local coordinates
  const int lyd0 = 1 - y0, lyd1 = n - 2 - y0;
  // Every LDS and scalar read issued so far has arrived before the passes
  // start: otherwise the waits the compiler places inside the pass loop
  // cover them on every iteration, and each pass would wait for its own
  // boundary-row reads at its start instead of at the row that uses them.
  __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
  tile_sweeps<T, TX, TY, S, NT, HX>(pl, pv, fv, lxd0, lxd1, lyd0, lyd1, lane, b0, w);
  tile_to_global<T, TX, TY, S, NT, HX, COH>(pout, n, pitch, x0, y0, lane, b0, pv);
  double rmax = 0.0, pmax = 0.0;
  if (CHECK)
    tile_residual<T, TX, TY, S, NT, HX>(pl, pv, fv, lxd0, lxd1, lyd0, lyd1, lane, b0, rmax, pmax);
  rmax_out = rmax;
  pmax_out = pmax;
  return true;
}

template <typename T, int TX, int TY, int S, int NT, bool CHECK>
__global__ __launch_bounds__(NT) void k_sor(const T* __restrict__ pin, T* __restrict__ pout,
                                            const T* __restrict__ F, int n, int pitch,
                                            PoissonCtl* __restrict__ ctl, double* __restrict__ part,
                                            int tiles_x, int xcd_bands, double relax_arg) {
  constexpr int HX = CHECK ? 2 : 0;
  using G = SorGeom<T, TX, TY, S, NT, HX>;
  __shared__ T sp[G::SLOTS];
  // A launch enqueued after its solve stopped returns without a sweep or a
  // store.  The state is read first but tested only after the region loads
  // (inside sor_tile), so its latency overlaps theirs: vector loads, which
  // complete in order with the region's, where a scalar load would be waited
  // for together with the kernel arguments before the first region load.
  const bool run = coh_load(&ctl->state) == SOLVE_RUN;
  const T w = (T)(relax_arg > 0.0 ? relax_arg : coh_load(&ctl->relax));
  // XCD bands: blocks are dealt to the eight XCDs in turn (block b to XCD
  // b mod 8), so XCD x gets a contiguous band of tiles, nb / 8 of them plus
  // one for the first nb mod 8 XCDs; neighbouring tiles then share an L2.
  const int nb = gridDim.x;
  int tile = blockIdx.x;
  if (xcd_bands) {
    const int q = nb >> 3, r = nb & 7, x = blockIdx.x & 7;
    tile = x * q + min(x, r) + (blockIdx.x >> 3);
  }
  double rmax = 0.0, pmax = 0.0;
  if (!sor_tile<T, TX, TY, S, NT, HX>(pin, pout, F, n, pitch, tile, tiles_x, w, sp, CHECK, rmax,
                                      pmax, run))
    return;
  // A checking launch only leaves its per-block maxima; k_decide, the next
  // launch on the stream, reduces them.  The kernel boundary orders the
  // stores, so no block pays for a device-wide release fence.
  if (CHECK && threadIdx.x == 0) {
    part[2 * blockIdx.x] = rmax;
    part[2 * blockIdx.x + 1] = pmax;
  }
}

// The decision of a Poisson solve after one residual check (see PoissonCtl).
// r is max |g - psi| in the units of the relaxation formula.
__device__ void decide(PoissonCtl* c, double r, double pm, long long sweeps_done) {
  c->sweeps += sweeps_done;
  c->total_sweeps += sweeps_done;
  c->last = r;
  c->psimax = pm;
  // an opening of Gauss-Seidel sweeps ends at the first check after a sweep
  if (c->gs_open && c->sweeps > 0) {
    c->gs_open = 0;
    c->relax = c->relax_sor;
  }
  int st = SOLVE_RUN;
  if (!(r <= DBL_MAX)) {
    st = SOLVE_NONFINITE;
  } else if (r <= c->tol_hat) {
    st = SOLVE_CONVERGED;
  } else if (c->floor_ulps > 0.0 && r <= c->floor_ulps * DBL_EPSILON * pm) {
    // The residual is at the rounding level of psi itself: no iteration can
    // lower it further (multigrid reaches it in a few cycles).
    st = SOLVE_FLOOR;
    c->floor_limited = 1;
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
  if (st != SOLVE_RUN) {
    c->total_solves += 1;
    if (st == SOLVE_FLOOR) c->total_floor += 1;
    if (st == SOLVE_NOCONV) c->total_noconv += 1;
    if (st == SOLVE_NONFINITE) c->total_nonfinite += 1;
  }
  c->state = st;
}

// The decision after a checking launch of nb blocks (one block).  A solve
// that had already stopped launched no sweep, and its partial maxima are
// stale: it is left alone.
// sweeps_done < 0 counts the control block's sweeps per check.
__global__ __launch_bounds__(256) void k_decide(PoissonCtl* __restrict__ ctl,
                                                const double* __restrict__ part, int nb,
                                                long long sweeps_done) {
  if (ctl->state != SOLVE_RUN) return;
  double r = 0.0, p = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) {
    r = fmax(r, part[2 * k]);
    p = fmax(p, part[2 * k + 1]);
  }
  block_max2<256>(r, p);
  if (threadIdx.x == 0) decide(ctl, r, p, sweeps_done < 0 ? ctl->sweeps_per_check : sweeps_done);
}

// ---------------------------------------------------------------------------
// Persistent batched Poisson solves (several cavities of uneven size, one
// launch).  The tile list concatenates every member's tiles; block b sweeps
// tiles b, b + G, ... of each round.  A round is one launch-equivalent of the
// per-launch path (S sweeps, psi_in -> psi_out), so results are bitwise those
// of the per-launch path with the same tile shape and check spacing.
// ---------------------------------------------------------------------------
__device__ inline int load_state(const PoissonCtl* c) {
  return __hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier.  Every block stores the new generation in its own arrival
// flag (one 128-byte line each, so arrivals never contend); the threads of
// block 0 wait for all flags in parallel and then release the generation in
// `go`, which the other blocks wait for.  Waits poll with relaxed atomic
// loads and order memory with one fence after the wait succeeds: an acquire
// on every poll would invalidate caches that blocks still computing rely on.
// Returns false (and sets bc->error) if a wait exceeds spin_ticks of the
// 100 MHz wall clock, so a grid that is not co-resident ends with an error
// instead of hanging.
__device__ bool grid_sync(BatchCtl* bc, unsigned int* flags, unsigned int nb, unsigned int& gen,
                          long long spin_ticks) {
  __shared__ int s_ok;
  wait_vm();  // this wavefront's stores have reached L2 before block 0's release
  __syncthreads();
  gen += 1u;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&flags[blockIdx.x * kFlagStride], gen, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  int ok = 1;
  if (blockIdx.x == 0) {
    const long long t0 = wall_clock64();
    for (unsigned int b = threadIdx.x; b < nb && ok; b += blockDim.x) {
      while (__hip_atomic_load(&flags[b * kFlagStride], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT) != gen) {
        __builtin_amdgcn_s_sleep(1);
        if (__hip_atomic_load(&bc->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            wall_clock64() - t0 > spin_ticks) {
          ok = 0;
          break;
        }
      }
    }
    ok = __syncthreads_and(ok);
    if (threadIdx.x == 0) {
      if (ok) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(&bc->go, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(&bc->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  } else if (threadIdx.x == 0) {
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(&bc->go, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != gen) {
      __builtin_amdgcn_s_sleep(1);
      if (__hip_atomic_load(&bc->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          wall_clock64() - t0 > spin_ticks) {
        __hip_atomic_store(&bc->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
  }
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// The same barrier for kernels whose cross-block data all move through
// device-scope loads and stores: every wavefront waits for its own stores,
// and no block writes back or invalidates an L2 cache.
__device__ bool grid_sync_coh(BatchCtl* bc, unsigned int* flags, unsigned int nb,
                              unsigned int& gen, long long spin_ticks) {
  __shared__ int s_ok;
  wait_vm();
  __syncthreads();
  gen += 1u;
  if (threadIdx.x == 0) coh_store(&flags[blockIdx.x * kFlagStride], gen);
  int ok = 1;
  if (blockIdx.x == 0) {
    const long long t0 = wall_clock64();
    for (unsigned int b = threadIdx.x; b < nb && ok; b += blockDim.x) {
      while (coh_load(&flags[b * kFlagStride]) != gen) {
        __builtin_amdgcn_s_sleep(1);
        if (coh_load(&bc->error) != 0 || wall_clock64() - t0 > spin_ticks) {
          ok = 0;
          break;
        }
      }
    }
    ok = __syncthreads_and(ok);
    if (threadIdx.x == 0) {
      if (ok)
        coh_store(&bc->go, gen);
      else
        coh_store(&bc->error, 1);
    }
  } else if (threadIdx.x == 0) {
    const long long t0 = wall_clock64();
    while (coh_load(&bc->go) != gen) {
      __builtin_amdgcn_s_sleep(1);
      if (coh_load(&bc->error) != 0 || wall_clock64() - t0 > spin_ticks) {
        coh_store(&bc->error, 1);
        ok = 0;
        break;
      }
    }
  }
  if (threadIdx.x == 0) s_ok = ok;
  __syncthreads();
  return s_ok != 0;
}

// The generation every block starts a launch with, and the record of the
// one it ended with (block 0, after the last barrier every block passed).
__device__ inline unsigned int batch_epoch(const BatchCtl* bc) {
  return __hip_atomic_load(&bc->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void batch_end(BatchCtl* bc, unsigned int gen) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(&bc->epoch, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int member_of(const BatchMember* mem, int count, int t) {
  int k = 0;
  while (k + 1 < count && t >= mem[k + 1].tile0) ++k;
  return k;
}

// Any member still solving?  Read by thread 0, broadcast through LDS.
__device__ bool any_running(const BatchMember* mem, int count) {
  __shared__ int s_any;
  if (threadIdx.x == 0) {
    int any = 0;
    for (int k = 0; k < count; ++k) any |= (load_state(mem[k].ctl) == SOLVE_RUN);
    s_any = any;
  }
  __syncthreads();
  const int r = s_any;
  __syncthreads();
  return r != 0;
}

// Block k reduces member k's partial maxima and takes its decision.
template <int NT>
__device__ void batch_decide(const BatchMember* mem, int count, long long sweeps_done) {
  if ((int)blockIdx.x >= count) return;
  const BatchMember& m = mem[blockIdx.x];
  if (load_state(m.ctl) != SOLVE_RUN) return;
  double r = 0.0, p = 0.0;
  for (int q = threadIdx.x; q < m.tiles; q += NT) {
    r = fmax(r, coh_load(&m.part[2 * q]));
    p = fmax(p, coh_load(&m.part[2 * q + 1]));
  }
  block_max2<NT>(r, p);
  if (threadIdx.x == 0) {
    decide(m.ctl, r, p, sweeps_done < 0 ? m.ctl->sweeps_per_check : sweeps_done);
    // what the other blocks read of the decision, device-coherent
    coh_store(&m.ctl->state, m.ctl->state);
    coh_store(&m.ctl->relax, m.ctl->relax);
  }
}

template <int TX, int TY, int S, int NT>
__global__ __launch_bounds__(NT) void k_batch64(const BatchMember* __restrict__ mem, int count,
                                                int total_tiles, int pairs_per_check,
                                                BatchCtl* __restrict__ bc,
                                                unsigned int* __restrict__ flags,
                                                long long spin_ticks) {
  using G = SorGeom<double, TX, TY, S, NT, 2>;  // rounds may check
  __shared__ double sp[G::SLOTS];
  const unsigned int nb = gridDim.x;
  unsigned int gen = batch_epoch(bc);
  while (any_running(mem, count)) {
    for (int r = 0; r < 2 * pairs_per_check; ++r) {
      const bool fwd = (r & 1) == 0;
      const bool check = (r == 2 * pairs_per_check - 1);
      for (int t = blockIdx.x; t < total_tiles; t += nb) {
        const BatchMember& m = mem[member_of(mem, count, t)];
        if (load_state(m.ctl) != SOLVE_RUN) continue;
        const int lt = t - m.tile0;
        const double w = coh_load(&m.ctl->relax);
        const double* pin = fwd ? m.psi : m.psi_b;
        double* pout = fwd ? m.psi_b : m.psi;
        double rmax = 0.0, pmax = 0.0;
        // one inlined tile body for both kinds of round; psi moves between
        // blocks through device-scope loads and stores, so the barrier needs
        // no cache write-back or invalidation
        sor_tile<double, TX, TY, S, NT, 2, true>(pin, pout, m.F, m.n, m.pitch, lt, m.tiles_x, w,
                                                 sp, check, rmax, pmax);
        if (check && threadIdx.x == 0) {
          coh_store(&m.part[2 * lt], rmax);
          coh_store(&m.part[2 * lt + 1], pmax);
        }
        __syncthreads();
      }
      if (!grid_sync_coh(bc, flags, nb, gen, spin_ticks)) return;
    }
    batch_decide<NT>(mem, count, -1);
    if (!grid_sync_coh(bc, flags, nb, gen, spin_ticks)) return;
  }
  batch_end(bc, gen);
}

template <int TX, int TY, int S, int NT>
__global__ __launch_bounds__(NT) void k_batch_mixed(const BatchMember* __restrict__ mem,
                                                    int count, int total_tiles, int inner_pairs,
                                                    BatchCtl* __restrict__ bc,
                                                    unsigned int* __restrict__ flags,
                                                    long long spin_ticks) {
  using G = SorGeom<float, TX, TY, S, NT, 0>;  // correction sweeps never check
  __shared__ float sp[G::SLOTS];
  const unsigned int nb = gridDim.x;
  unsigned int gen = batch_epoch(bc);
  for (;;) {
    // FP64 residual of psi on every tile; the correction starts from zero.
    for (int t = blockIdx.x; t < total_tiles; t += nb) {
      const BatchMember& m = mem[member_of(mem, count, t)];
      if (load_state(m.ctl) != SOLVE_RUN) continue;
      const int lt = t - m.tile0;
      const int tyi = lt / m.tiles_x, txi = lt - tyi * m.tiles_x;
      double rmax = 0.0, pmax = 0.0;
      for (int q = threadIdx.x; q < TX * TY; q += NT) {
        const int i = txi * TX + q % TX, j = tyi * TY + q / TX;
        if (i < 1 || i > m.n - 2 || j < 1 || j > m.n - 2) continue;
        const size_t p = (size_t)j * m.pitch + i;
        const double* psi = m.psi;
        const int pt = m.pitch;
        const double s4 = (psi[p + 1] + psi[p - 1]) + (psi[p + pt] + psi[p - pt]);
        const double sd = (psi[p + pt + 1] + psi[p + pt - 1]) + (psi[p - pt + 1] + psi[p - pt - 1]);
        const double r = fma(0.2, s4, fma(0.05, sd, m.F[p])) - psi[p];
        m.R32[p] = (float)r;
        m.d32a[p] = 0.0f;
        rmax = fmax(rmax, mag(r));
        pmax = fmax(pmax, mag(psi[p]));
      }
      block_max2<NT>(rmax, pmax);
      if (threadIdx.x == 0) {
        m.part[2 * lt] = rmax;
        m.part[2 * lt + 1] = pmax;
      }
      __syncthreads();
    }
    if (!grid_sync(bc, flags, nb, gen, spin_ticks)) return;
    batch_decide<NT>(mem, count, 0);
    if (!grid_sync(bc, flags, nb, gen, spin_ticks)) return;
    if (!any_running(mem, count)) {
      batch_end(bc, gen);
      return;
    }
    // FP32 correction sweeps; the last pair relaxes with 1, the first with the
    // control block's parameter (1 during a Gauss-Seidel opening), the others
    // over-relax.
    for (int r = 0; r < 2 * inner_pairs; ++r) {
      const bool fwd = (r & 1) == 0;
      for (int t = blockIdx.x; t < total_tiles; t += nb) {
        const BatchMember& m = mem[member_of(mem, count, t)];
        if (load_state(m.ctl) != SOLVE_RUN) continue;
        const float w = (r >= 2 * (inner_pairs - 1)) ? 1.0f
                        : (r < 2)                    ? (float)m.ctl->relax
                                                     : (float)m.ctl->relax_sor;
        double rm = 0.0, pm = 0.0;
        sor_tile<float, TX, TY, S, NT, 0>(fwd ? m.d32a : m.d32b, fwd ? m.d32b : m.d32a, m.R32,
                                          m.n, m.pitch, t - m.tile0, m.tiles_x, w, sp, false, rm,
                                          pm);
        __syncthreads();
      }
      if (!grid_sync(bc, flags, nb, gen, spin_ticks)) return;
    }
    // FP64 refinement psi += d, and the sweep count.
    for (int t = blockIdx.x; t < total_tiles; t += nb) {
      const BatchMember& m = mem[member_of(mem, count, t)];
      if (load_state(m.ctl) != SOLVE_RUN) continue;
      const int lt = t - m.tile0;
      const int tyi = lt / m.tiles_x, txi = lt - tyi * m.tiles_x;
      for (int q = threadIdx.x; q < TX * TY; q += NT) {
        const int i = txi * TX + q % TX, j = tyi * TY + q / TX;
        if (i < 1 || i > m.n - 2 || j < 1 || j > m.n - 2) continue;
        const size_t p = (size_t)j * m.pitch + i;
        m.psi[p] += (double)m.d32a[p];
      }
      if (lt == 0 && threadIdx.x == 0) {
        const long long done = 2LL * S * inner_pairs;
        m.ctl->sweeps += done;
        m.ctl->total_sweeps += done;
      }
    }
    if (!grid_sync(bc, flags, nb, gen, spin_ticks)) return;
  }
}

// ---------------------------------------------------------------------------
// Resident FP64 solve: one launch per Poisson solve, one block per tile for
// the whole solve.  A block keeps its tile's psi in LDS and the psi and F of
// the nodes it owns in registers, so a round of S sweeps only reloads the
// halo ring: the neighbours' tiles of the previous round, published through
// the ping-pong pair (round r writes buffer (r + 1) % 2).  A block starts
// round r once its (up to eight) neighbours have published round r - 1;
// since a block publishes only after reading, two buffers suffice.  At the
// start of every P-th round each block evaluates the residual of the state
// after the previous round (its tile and the freshly loaded first ring are
// exact) and leaves its maxima; one round later block 0 waits for every
// block, reduces them and decides; one round after that every block applies
// the decision.  The solve thus stops two rounds after the check that ended
// it, the same in every block.
//
// Everything exchanged between blocks (tiles, flags, maxima, decisions) is
// stored and loaded with device-scope 8-byte accesses; a block publishes a
// round by waiting for its own stores (s_waitcnt in every wavefront) and
// then storing its flag, so no block writes back or invalidates an L2 cache.
// Waits poll with relaxed loads and are bounded by the wall clock: a grid
// that is not co-resident ends with werror instead of hanging.
// ---------------------------------------------------------------------------
__device__ inline bool resident_failed(const ResidentCtl* rc, long long t0, long long spin) {
  return coh_load(&rc->error) != 0 || wall_clock64() - t0 > spin;
}
__device__ inline void resident_fail(ResidentCtl* rc, PoissonCtl* ctl) {
  coh_store(&rc->error, 1);
  coh_store(&ctl->werror, 1);
}

template <int TX, int TY, int S, int NT>
__global__ __launch_bounds__(NT) void k_sor_resident(double* __restrict__ bufa,
                                                     double* __restrict__ bufb,
                                                     const double* __restrict__ F, int n,
                                                     int pitch, int tiles_x, int tiles_y,
                                                     PoissonCtl* __restrict__ ctl,
                                                     double* __restrict__ part,
                                                     unsigned int* __restrict__ flags,
                                                     ResidentCtl* __restrict__ rc, int P,
                                                     long long spin_ticks) {
  using G = SorGeom<double, TX, TY, S, NT, 0>;
  constexpr int K = G::K;
  __shared__ double sp[G::SLOTS];
  __shared__ int s_go;
  __shared__ double s_w;
  // No block writes the control block before every block has published a
  // round, so every block reads the same starting state here.
  if (ctl->state != SOLVE_RUN) return;
  double* const pl = sp + G::BASE;
  const int ntiles = tiles_x * tiles_y;
  int tile = blockIdx.x;
  if ((ntiles & 7) == 0) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
  const int tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
  const int x0 = txi * TX - G::H, y0 = tyi * TY - G::H;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int b0 = wave * K;
  const int lxd0 = 1 - x0, lxd1 = n - 2 - x0, lyd0 = 1 - y0, lyd1 = n - 2 - y0;
  // thread t < 9 (t != 4) watches neighbour t of the 3 x 3 tiles around this one
  int nbr = -1;
  if (tid < 9 && tid != 4) {
    const int nx = txi + tid % 3 - 1, ny = tyi + tid / 3 - 1;
    if (nx >= 0 && nx < tiles_x && ny >= 0 && ny < tiles_y) nbr = ny * tiles_x + nx;
  }
  double fv[4][K], pv[4][K];
  double w = ctl->relax;
  region_to_lds<double, TX, TY, S, NT, 0, false>(bufa, n, pitch, x0, y0, pl, tid);
  rhs_to_regs<double, TX, TY, S, NT, 0>(F, n, pitch, x0, y0, lane, b0, fv);
  rhs_zero_beyond<double, TX, TY, S, NT, 0>(n, x0, lane, fv);
  __syncthreads();
  lds_to_regs<double, TX, TY, S, NT, 0, false>(pl, lane, b0, pv);
  int r = 0;
  bool stopped = false;
  for (;; ++r) {
    // Values the round's addresses derive from, re-materialised every round:
    // without this the compiler hoists every per-thread address of the ring
    // load, the refresh and the store out of the loop and runs out of
    // registers.
    int tid_r = tid, lane_r = lane;
    asm volatile("" : "+v"(tid_r), "+v"(lane_r));
    if (r > 0) {
      // the neighbours have published round r - 1
      int ok = 1;
      if (nbr >= 0) {
        const long long t0 = wall_clock64();
        while (coh_load(&flags[nbr * kFlagStride]) < (unsigned int)r) {
          __builtin_amdgcn_s_sleep(1);
          if (resident_failed(rc, t0, spin_ticks)) {
            ok = 0;
            break;
          }
        }
      }
      if (!__syncthreads_and(ok)) {
        if (tid == 0) resident_fail(rc, ctl);
        break;
      }
      region_to_lds<double, TX, TY, S, NT, 0, true, 2, true>((r & 1) ? bufb : bufa, n, pitch, x0,
                                                            y0, pl, tid_r);
      __syncthreads();
      lds_to_regs<double, TX, TY, S, NT, 0, true>(pl, lane_r, b0, pv);
      // residual of the state after round r - 1 (check c = r / P - 1)
      if (r % P == 0) {
        double rm, pm;
        tile_residual<double, TX, TY, S, NT, 0>(pl, pv, fv, lxd0, lxd1, lyd0, lyd1, lane_r, b0,
                                                rm, pm);
        if (tid == 0) {
          const int slot = (r / P - 1) & 1;
          coh_store(&part[2 * (slot * ntiles + tile)], rm);
          coh_store(&part[2 * (slot * ntiles + tile) + 1], pm);
        }
      }
      // block 0 decides check c = (r - 1) / P - 1 once every block has
      // published the round that evaluated it
      if (blockIdx.x == 0 && r % P == 1 && r > P) {
        const int slot = ((r - 1) / P - 1) & 1;
        int ok2 = 1;
        const long long t0 = wall_clock64();
        for (int b = tid; b < ntiles && ok2; b += NT) {
          while (coh_load(&flags[b * kFlagStride]) < (unsigned int)r) {
            __builtin_amdgcn_s_sleep(1);
            if (resident_failed(rc, t0, spin_ticks)) {
              ok2 = 0;
              break;
            }
          }
        }
        if (!__syncthreads_and(ok2)) {
          if (tid == 0) resident_fail(rc, ctl);
          break;
        }
        double rr = 0.0, pp = 0.0;
        for (int q = tid; q < ntiles; q += NT) {
          rr = fmax(rr, coh_load(&part[2 * (slot * ntiles + q)]));
          pp = fmax(pp, coh_load(&part[2 * (slot * ntiles + q) + 1]));
        }
        block_max2<NT>(rr, pp);
        if (tid == 0) {
          decide(ctl, rr, pp, ctl->sweeps_per_check);
          coh_store(&rc->state[slot], ctl->state);
          coh_store(&rc->relax[slot], ctl->relax);
          wait_vm();
          coh_store(&rc->tag[slot], (unsigned int)((r - 1) / P));
        }
      }
      // every block applies decision c = (r - 2) / P - 1
      if (r % P == 2 && r > P + 1) {
        const unsigned int want = (unsigned int)((r - 2) / P);
        const int slot = (int)(want - 1) & 1;
        if (tid == 0) {
          int ok3 = 1;
          const long long t0 = wall_clock64();
          while (coh_load(&rc->tag[slot]) != want) {
            __builtin_amdgcn_s_sleep(1);
            if (resident_failed(rc, t0, spin_ticks)) {
              ok3 = 0;
              break;
            }
          }
          if (ok3) {
            s_go = coh_load(&rc->state[slot]) == SOLVE_RUN ? 1 : 0;
            s_w = coh_load(&rc->relax[slot]);
          } else {
            resident_fail(rc, ctl);
            s_go = -1;
          }
        }
        __syncthreads();
        const int go = s_go;
        w = s_w;
        __syncthreads();
        if (go < 0) break;
        if (go == 0) {
          stopped = true;
          break;
        }
      }
    }
    tile_sweeps<double, TX, TY, S, NT, 0>(pl, pv, fv, lxd0, lxd1, lyd0, lyd1, lane_r, b0, w);
    tile_to_global<double, TX, TY, S, NT, 0, true>((r & 1) ? bufa : bufb, n, pitch, x0, y0,
                                                   lane_r, b0, pv);
    wait_vm();
    __syncthreads();
    if (tid == 0) coh_store(&flags[tile * kFlagStride], (unsigned int)(r + 1));
  }
  if (!stopped) return;
  // Rounds 0 .. r - 1 are done and the last one sits in buffer r % 2; the
  // result belongs in psi.  The decision counted the sweeps up to its check,
  // two rounds before the stop.
  if (r & 1) tile_to_global<double, TX, TY, S, NT, 0>(bufa, n, pitch, x0, y0, lane, b0, pv);
  if (blockIdx.x == 0 && tid == 0) {
    ctl->sweeps += 2LL * S;
    ctl->total_sweeps += 2LL * S;
  }
}


// ---------------------------------------------------------------------------
// Geometric multigrid for the compact stream equation (coarse levels are the
// same compact operator rediscretised on a coarser grid).  A level with m
// intervals (h = 1/m) coarsens to ceil(m/2) intervals; for odd m the grids
// are not nested, so transfers work in physical coordinates: prolongation is
// bilinear interpolation, restriction its transpose scaled by (h_f/h_c)^2.
// With x_i = i/m_f and X_I = I/m_c the hat weight of coarse node I at fine
// node i is 1 - |i m_c - I m_f| / m_f, evaluated exactly in integers; on
// nested levels these are the usual bilinear and full-weighting stencils.
// Every kernel returns at once when the solve has stopped.
// ---------------------------------------------------------------------------
// The per-node arithmetic of the transfer and residual steps, shared by the
// per-level kernels and the fused coarse cycle so that both give the same
// bits.  Arrays are row-major with the given pitch (global or LDS).

// r = (g - psi) / (0.3 h^2) at interior node p: the residual of the compact
// equation in vorticity units.
template <typename T>
__device__ __forceinline__ T mg_residual_at(const T* psi, const T* F, size_t p, int pitch,
                                            T inv03h2) {
  const T s4 = (psi[p + 1] + psi[p - 1]) + (psi[p + pitch] + psi[p - pitch]);
  const T sd = (psi[p + pitch + 1] + psi[p + pitch - 1]) + (psi[p - pitch + 1] + psi[p - pitch - 1]);
  const T g = fma_t(T(0.2), s4, fma_t(T(0.05), sd, F[p]));
  return (g - psi[p]) * inv03h2;
}

// The restricted residual at interior coarse node (I, J) (before the
// scaling): the transpose of bilinear interpolation in physical coordinates.
template <typename T>
__device__ __forceinline__ T mg_restrict_at(const T* r, int nf, int pitchf, int nc, int I,
                                            int J) {
  const long long mf = nf - 1, mc = nc - 1;
  const int i0 = max(1, (int)(((I - 1) * mf) / mc) + 1);
  const int i1 = min(nf - 2, (int)(((I + 1) * mf + mc - 1) / mc) - 1);
  const int j0 = max(1, (int)(((J - 1) * mf) / mc) + 1);
  const int j1 = min(nf - 2, (int)(((J + 1) * mf + mc - 1) / mc) - 1);
  const T invmf = T(1) / (T)mf;
  T sum = T(0);
  for (int j = j0; j <= j1; ++j) {
    const long long dj = (long long)j * mc - (long long)J * mf;
    const T wy = (T)(mf - (dj < 0 ? -dj : dj)) * invmf;
    if (wy <= T(0)) continue;
    T row = T(0);
    for (int i = i0; i <= i1; ++i) {
      const long long di = (long long)i * mc - (long long)I * mf;
      const T wx = (T)(mf - (di < 0 ? -di : di)) * invmf;
      if (wx > T(0)) row = fma_t(wx, r[(size_t)j * pitchf + i], row);
    }
    sum = fma_t(wy, row, sum);
  }
  return sum;
}

// The bilinear interpolation of the coarse correction at interior fine node
// (i, j).
template <typename T>
__device__ __forceinline__ T mg_prolong_at(const T* Ec, int nc, int pitchc, int nf, int i, int j) {
  const long long mf = nf - 1, mc = nc - 1;
  const int I = (int)(((long long)i * mc) / mf);
  const int J = (int)(((long long)j * mc) / mf);
  const T ti = (T)((long long)i * mc - (long long)I * mf) / (T)mf;
  const T tj = (T)((long long)j * mc - (long long)J * mf) / (T)mf;
  const size_t c = (size_t)J * pitchc + I;
  const T lo = fma_t(ti, Ec[c + 1] - Ec[c], Ec[c]);
  const T hi = fma_t(ti, Ec[c + pitchc + 1] - Ec[c + pitchc], Ec[c + pitchc]);
  return fma_t(tj, hi - lo, lo);
}

// The four-colour relaxation of one node, the same arithmetic as the sweep
// kernel (gs_target with the lane share of each side written out): the E-
// and W-side shares fma(0.25, NE + SE, E) and fma(0.25, NW + SW, W) summed,
// then psi <- psi + w (g - psi).
template <typename T>
__device__ __forceinline__ T mg_relax_at(const T* psi, const T* F, size_t p, int pitch, T w) {
  const T qe = fma_t(T(0.25), psi[p + pitch + 1] + psi[p - pitch + 1], psi[p + 1]);
  const T qw = fma_t(T(0.25), psi[p + pitch - 1] + psi[p - pitch - 1], psi[p - 1]);
  const T g = fma_t(T(0.2), (qe + qw) + (psi[p + pitch] + psi[p - pitch]), F[p]);
  const T v = psi[p];
  return fma_t(w, g - v, v);
}

// r = (g - psi) / (0.3 h^2): the residual of the compact equation in
// vorticity units (zero on walls).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_residual(const T* __restrict__ psi,
                                                        const T* __restrict__ F,
                                                        T* __restrict__ r, int n, int pitch,
                                                        T inv03h2,
                                                        const PoissonCtl* __restrict__ ctl) {
  if (ctl->state != SOLVE_RUN) return;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n || j >= n) return;
  const size_t p = (size_t)j * pitch + i;
  if (i == 0 || j == 0 || i == n - 1 || j == n - 1) {
    r[p] = T(0);
    return;
  }
  r[p] = mg_residual_at(psi, F, p, pitch, inv03h2);
}

// Coarse right-hand side F_c = 0.3 h_c^2 R r and a zero coarse iterate (both
// ping-pong buffers, walls included).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_restrict(const T* __restrict__ r, int nf,
                                                        int pitchf, T* __restrict__ Fc,
                                                        T* __restrict__ Ec,
                                                        T* __restrict__ Ecb, int nc,
                                                        int pitchc, T scale,
                                                        const PoissonCtl* __restrict__ ctl) {
  if (ctl->state != SOLVE_RUN) return;
  const int I = blockIdx.x * 64 + (threadIdx.x & 63);
  const int J = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (I >= nc || J >= nc) return;
  const size_t pc = (size_t)J * pitchc + I;
  Ec[pc] = T(0);
  Ecb[pc] = T(0);
  if (I == 0 || J == 0 || I == nc - 1 || J == nc - 1) {
    Fc[pc] = T(0);
    return;
  }
  Fc[pc] = scale * mg_restrict_at(r, nf, pitchf, nc, I, J);
}

// psi_f += P E_c (bilinear interpolation of the coarse correction).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_prolong(const T* __restrict__ Ec, int nc,
                                                       int pitchc, T* __restrict__ psi,
                                                       int nf, int pitchf,
                                                       const PoissonCtl* __restrict__ ctl) {
  if (ctl->state != SOLVE_RUN) return;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i < 1 || j < 1 || i > nf - 2 || j > nf - 2) return;
  psi[(size_t)j * pitchf + i] += mg_prolong_at(Ec, nc, pitchc, nf, i, j);
}

// ---------------------------------------------------------------------------
// The coarse end of a V-cycle in one block: every level from the first one
// with at most kMgFuseMax nodes a side down to the coarsest and back, with
// all iterates, right-hand sides and residuals in LDS (dense, pitch n).  On
// these grids a per-level launch does almost no work, so the launches'
// fixed cost was most of a V-cycle's time; here the levels are separated by
// block barriers instead.  Each step is the per-level kernels' arithmetic
// (shared device functions) and the relaxation sweeps update the colours in
// place in the same order as the sweep kernel, so the cycle gives the same
// bits as the per-level launches.  F of the first level is read from its
// global array, its iterate E read and written back there (walls stay 0).
// ---------------------------------------------------------------------------
constexpr int kMgFuseMax = 65;
constexpr int kMgFuseThreads = 256;
constexpr int kMgFuseLevels = 6;
// nodes of every level below a 65-node level (65, 33, 17, 9), each level
// holding E, F and the residual: 3 x 5684 values (136 KiB in FP64)
constexpr int kMgFuseNodes = 65 * 65 + 33 * 33 + 17 * 17 + 9 * 9;

struct MgFusedArgs {
  int levels;                     // levels in the block, finest first
  int n[kMgFuseLevels];           // nodes per side
  double inv03h2[kMgFuseLevels];  // residual scale 1 / (0.3 h^2)
  double scale[kMgFuseLevels];    // restriction scale onto level l (l >= 1)
  int nu;                         // sweeps before and after the coarse correction
  int coarse_sweeps;
  double coarse_relax;
};

template <typename T>
__device__ __forceinline__ void mg_block_sweeps(T* E, const T* F, int n, int sweeps, T w) {
  for (int s = 0; s < sweeps; ++s) {
    for (int c = 0; c < 4; ++c) {
      const int cx = c & 1, cy = c >> 1;
      // the interior nodes of parity (cx, cy): i = i0, i0 + 2, ... <= n - 2
      const int i0 = cx == 0 ? 2 : 1, j0 = cy == 0 ? 2 : 1;
      const int nx = (n - 2 - i0) / 2 + 1, ny = (n - 2 - j0) / 2 + 1;
      for (int q = threadIdx.x; q < nx * ny; q += kMgFuseThreads) {
        const int j = j0 + 2 * (q / nx), i = i0 + 2 * (q - (q / nx) * nx);
        const size_t p = (size_t)j * n + i;
        E[p] = mg_relax_at(E, F, p, n, w);
      }
      __syncthreads();
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kMgFuseThreads) void k_mg_fused(T* __restrict__ Eg,
                                                             const T* __restrict__ Fg, int pitch,
                                                             MgFusedArgs a,
                                                             const PoissonCtl* __restrict__ ctl) {
  __shared__ T mg_lds[3 * kMgFuseNodes];
  if (ctl->state != SOLVE_RUN) return;
  T* E[kMgFuseLevels];
  T* F[kMgFuseLevels];
  T* R[kMgFuseLevels];
  {
    T* cur = mg_lds;
    for (int l = 0; l < a.levels; ++l) {
      const int sz = a.n[l] * a.n[l];
      E[l] = cur;
      F[l] = cur + sz;
      R[l] = cur + 2 * sz;
      cur += 3 * sz;
    }
  }
  const int n0 = a.n[0];
  for (int q = threadIdx.x; q < n0 * n0; q += kMgFuseThreads) {
    const int j = q / n0, i = q - j * n0;
    E[0][q] = Eg[(size_t)j * pitch + i];
    F[0][q] = Fg[(size_t)j * pitch + i];
  }
  __syncthreads();
  const int L = a.levels - 1;
  for (int l = 0; l < L; ++l) {
    const int n = a.n[l], nc = a.n[l + 1];
    mg_block_sweeps(E[l], F[l], n, a.nu, T(1.0));
    const T inv = (T)a.inv03h2[l];
    for (int q = threadIdx.x; q < n * n; q += kMgFuseThreads) {
      const int j = q / n, i = q - j * n;
      R[l][q] = (i == 0 || j == 0 || i == n - 1 || j == n - 1)
                    ? T(0)
                    : mg_residual_at(E[l], F[l], (size_t)q, n, inv);
    }
    __syncthreads();
    const T sc = (T)a.scale[l + 1];
    for (int q = threadIdx.x; q < nc * nc; q += kMgFuseThreads) {
      const int J = q / nc, I = q - J * nc;
      E[l + 1][q] = T(0);
      F[l + 1][q] = (I == 0 || J == 0 || I == nc - 1 || J == nc - 1)
                        ? T(0)
                        : sc * mg_restrict_at(R[l], n, n, nc, I, J);
    }
    __syncthreads();
  }
  mg_block_sweeps(E[L], F[L], a.n[L], a.coarse_sweeps, (T)a.coarse_relax);
  for (int l = L - 1; l >= 0; --l) {
    const int n = a.n[l], nc = a.n[l + 1];
    for (int q = threadIdx.x; q < n * n; q += kMgFuseThreads) {
      const int j = q / n, i = q - j * n;
      if (i >= 1 && j >= 1 && i <= n - 2 && j <= n - 2)
        E[l][q] += mg_prolong_at(E[l + 1], nc, nc, n, i, j);
    }
    __syncthreads();
    mg_block_sweeps(E[l], F[l], n, a.nu, T(1.0));
  }
  for (int q = threadIdx.x; q < n0 * n0; q += kMgFuseThreads) {
    const int j = q / n0, i = q - j * n0;
    if (i >= 1 && j >= 1 && i <= n0 - 2 && j <= n0 - 2) Eg[(size_t)j * pitch + i] = E[0][q];
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

// The same operator in FP32 arithmetic, from an FP32 shadow of psi and the
// FP64 vorticity rounded to FP32 (mixed precision).
__device__ inline float transport32(const float* __restrict__ psi, const double* __restrict__ w,
                                    size_t p, int pitch, float inv2h, float invh2, float nu) {
  const float u = (psi[p + pitch] - psi[p - pitch]) * inv2h;
  const float v = -(psi[p + 1] - psi[p - 1]) * inv2h;
  const float wP = (float)w[p], wE = (float)w[p + 1], wW = (float)w[p - 1];
  const float wN = (float)w[p + pitch], wS = (float)w[p - pitch];
  const float adv = -u * ((wE - wW) * inv2h) - v * ((wN - wS) * inv2h);
  const float dif = nu * (((wE - 2.0f * wP + wW) + (wN - 2.0f * wP + wS)) * invh2);
  return adv + dif;
}

// psi32 == nullptr: L in FP64 from psi; otherwise L in FP32 from psi32.
// The stage combination is FP64 either way.
__global__ __launch_bounds__(kBlock) void k_stage(const double* __restrict__ psi,
                                                  const float* __restrict__ psi32,
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
  const double L = psi32 ? (double)transport32(psi32, win, p, pitch, (float)inv2h, (float)invh2,
                                               (float)a.nu)
                         : transport(psi, win, p, pitch, inv2h, invh2, a.nu);
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
                            long long stall_window, long long sweeps_per_check,
                            double floor_ulps, const long long* gs_steps) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int gs_open = (gs_steps && *gs_steps >= 2) ? 1 : 0;
  c->state = SOLVE_RUN;
  c->phase = 0;
  c->polish_left = 0;
  c->gs_open = gs_open;
  c->relax = gs_open ? 1.0 : relax;
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
  c->floor_ulps = floor_ulps;
  c->floor_limited = 0;
  c->werror = 0;
}

// r = g(psi) - psi in FP64 on interior nodes, reduced to max |r| for the solve
// decision; with R32 != nullptr also stored as float for the FP32 correction
// solve, whose correction d32 then starts from zero.  A block of 256 threads
// takes a tile of 64 x 16 interior nodes; a thread takes four consecutive rows
// of one column and loads the six rows of psi they touch once (all loads
// issued together); the block's two maxima go to the partial array (one pair
// per block), which k_decide reduces.
constexpr int kResidTileX = 64, kResidTileY = 16;

inline dim3 resid_grid(int n) {
  return dim3((n - 2 + kResidTileX - 1) / kResidTileX, (n - 2 + kResidTileY - 1) / kResidTileY);
}

__global__ __launch_bounds__(kBlock) void k_resid64(const double* __restrict__ psi,
                                                    const double* __restrict__ F,
                                                    float* __restrict__ R32,
                                                    float* __restrict__ d32, int n, int pitch,
                                                    const PoissonCtl* __restrict__ ctl,
                                                    double* __restrict__ part) {
  if (ctl->state != SOLVE_RUN) return;
  double rmax = 0.0, pmax = 0.0;
  const int i = 1 + blockIdx.x * kResidTileX + (threadIdx.x & 63);
  const int j0 = 1 + blockIdx.y * kResidTileY + 4 * (threadIdx.x >> 6);
  if (i <= n - 2 && j0 <= n - 2) {
    // rows j0 - 1 ... j0 + 4 (those inside the grid), columns i - 1, i, i + 1
    double w[6], c[6], e[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const int j = j0 - 1 + r;
      const size_t q = (size_t)min(j, n - 1) * pitch + i;
      w[r] = psi[q - 1];
      c[r] = psi[q];
      e[r] = psi[q + 1];
    }
#pragma unroll
    for (int r = 1; r <= 4; ++r) {
      const int j = j0 - 1 + r;
      if (j > n - 2) break;
      const size_t p = (size_t)j * pitch + i;
      const double s4 = (e[r] + w[r]) + (c[r + 1] + c[r - 1]);
      const double sd = (e[r + 1] + w[r + 1]) + (e[r - 1] + w[r - 1]);
      const double g = fma(0.2, s4, fma(0.05, sd, F[p]));
      const double res = g - c[r];
      if (R32) {
        R32[p] = (float)res;
        d32[p] = 0.0f;
      }
      rmax = fmax(rmax, mag(res));
      pmax = fmax(pmax, mag(c[r]));
    }
  }
  // per-block maxima only; k_decide follows on the stream
  block_max2<kBlock>(rmax, pmax);
  if (threadIdx.x == 0) {
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * b] = rmax;
    part[2 * b + 1] = pmax;
  }
}

__global__ __launch_bounds__(kBlock) void k_refine(double* __restrict__ psi,
                                                   const float* __restrict__ d32, int n,
                                                   int pitch, PoissonCtl* __restrict__ ctl,
                                                   int inner_sweeps) {
  if (ctl->state != SOLVE_RUN) return;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    ctl->sweeps += inner_sweeps;
    ctl->total_sweeps += inner_sweeps;
  }
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
  // block b takes rows b, b + gridDim.x, ...; its threads stride along a row
  for (int j = blockIdx.x; j < n; j += gridDim.x) {
    for (int i = threadIdx.x; i < n; i += kBlock) {
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

__global__ __launch_bounds__(kBlock) void k_zero(unsigned int* p, size_t words) {
  for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < words;
       k += (size_t)gridDim.x * kBlock)
    p[k] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_shadow(const double* __restrict__ a,
                                                   float* __restrict__ b, int n, int pitch) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= pitch || j >= n) return;
  const size_t p = (size_t)j * pitch + i;
  b[p] = (float)a[p];
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

// Starting value of a stage's Poisson solve from the same stage's solutions of
// the last `levels` steps.  hist holds `levels` slots per stage (stage k,
// slot r at hist + ((k - 1) * levels + r) * fstride); step q's solution of
// stage k sits in slot q mod levels.  *count is the number of steps completed
// since the history was last emptied.  On entry psi holds the solution of the
// stage before (stage 5 of the previous step when stage == 1): it is filed
// first, then replaced, if at least two earlier steps of this stage are on
// file, by the value at the current step of the polynomial through them:
// sum over q of w_q times the solution q steps back, with the weights of row
// L = min(steps on file, levels) of wtab (kWarmCols doubles per row; for the
// interpolating polynomial w_q = (-1)^(q+1) C(L, q)).  The solve that follows
// converges to the same tolerance from any start; a start whose error is
// O(dt^L) instead of O(dt) saves the sweeps that would remove the difference.
// Interior nodes only (psi = 0 on walls in every slot).

__global__ __launch_bounds__(kBlock) void k_warm(double* __restrict__ psi,
                                                 double* __restrict__ hist, size_t fstride,
                                                 int n, int pitch, int stage, int levels,
                                                 const long long* __restrict__ count,
                                                 const double* __restrict__ wtab) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i < 1 || j < 1 || i >= n - 1 || j >= n - 1) return;
  const long long s = *count;
  const size_t p = (size_t)j * pitch + i;
  const double cur = psi[p];
  if (stage > 1)
    hist[((size_t)(stage - 2) * levels + (int)(s % levels)) * fstride + p] = cur;
  else if (s >= 1)
    hist[((size_t)4 * levels + (int)((s - 1) % levels)) * fstride + p] = cur;
  const int L = (int)(s < levels ? s : levels);
  if (L < 2) return;
  const double* hk = hist + (size_t)(stage - 1) * levels * fstride + p;
  const double* w = wtab + L * kWarmCols;
  double g = 0.0;
  for (int q = L; q >= 1; --q)  // oldest point first
    g = fma(w[q - 1], hk[(size_t)((s - q) % levels) * fstride], g);
  psi[p] = g;
}

// One more step is on file (after the step's last stage).
__global__ void k_warm_tick(long long* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *count += 1;
}


// ---------------------------------------------------------------------------
// Tile-configuration dispatch of the sweep kernels.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY, int S, int NT>
hipError_t sor_launch(const T* pin, T* pout, const T* F, int n, int pitch, PoissonCtl* ctl,
                      double* part, int check, int xcd_bands, double relax, hipStream_t st) {
  // the tile loads read node pairs (x even, x + 1): the pitch must be even
  // and hold x = n for odd n
  if ((pitch & 1) || pitch < n + (n & 1)) return hipErrorInvalidValue;
  const int tx = (n + TX - 1) / TX, ty = (n + TY - 1) / TY;
  const dim3 grid(tx * ty);
  if (check) {
    // residual checks are FP64 only (FP32 sweeps relax a correction whose
    // residual the FP64 kernels evaluate), so FP32 tiles need not fit the
    // checking launch's wider halo
    if constexpr (std::is_same<T, double>::value) {
      hipLaunchKernelGGL((k_sor<T, TX, TY, S, NT, true>), grid, dim3(NT), 0, st, pin, pout, F,
                         n, pitch, ctl, part, tx, xcd_bands, relax);
      hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, st, ctl, part, (int)grid.x, -1LL);
    } else {
      return hipErrorInvalidValue;
    }
  } else
    hipLaunchKernelGGL((k_sor<T, TX, TY, S, NT, false>), grid, dim3(NT), 0, st, pin, pout, F, n,
                       pitch, ctl, part, tx, xcd_bands, relax);
  return hipGetLastError();
}

// (tile x, tile y, sweeps per launch, threads per block) instantiated for FP64
// and FP32; the autotuner chooses among them.
#define CAV_SOR_CONFIGS_F64(X) \
  X(32, 32, 1, 256)            \
  X(32, 32, 2, 256)            \
  X(64, 32, 2, 512)            \
  X(64, 64, 1, 1024)           \
  X(64, 64, 2, 1024)           \
  X(64, 64, 3, 1024)           \
  X(64, 64, 2, 512)            \
  X(64, 64, 4, 512)            \
  X(64, 64, 4, 1024)           \
  X(64, 64, 4, 768)            \
  X(96, 64, 2, 1024)           \
  X(96, 64, 3, 1024)           \
  X(92, 50, 4, 1024)           \
  X(84, 54, 5, 1024)

#define CAV_SOR_CONFIGS_F32(X) \
  X(32, 32, 1, 256)            \
  X(32, 32, 2, 256)            \
  X(64, 32, 2, 512)            \
  X(64, 64, 2, 512)            \
  X(64, 64, 2, 1024)           \
  X(64, 64, 4, 1024)           \
  X(64, 64, 6, 1024)           \
  X(96, 64, 3, 1024)           \
  X(96, 96, 3, 1024)           \
  X(88, 56, 5, 1024)           \
  X(64, 64, 4, 512)            \
  X(64, 64, 6, 512)

template <typename T>
hipError_t sor_dispatch(const SorConfig& c, const T* pin, T* pout, const T* F, int n, int pitch,
                        PoissonCtl* ctl, double* part, int check, double relax, hipStream_t st);

#define CAV_TRY(TX_, TY_, S_, NT_)                                                         \
  if (c.tx == TX_ && c.ty == TY_ && c.s == S_ && c.nt == NT_)                              \
    return sor_launch<T, TX_, TY_, S_, NT_>(pin, pout, F, n, pitch, ctl, part, check,      \
                                            c.xcd_bands, relax, st);
#define CAV_HAS(TX_, TY_, S_, NT_) \
  if (c.tx == TX_ && c.ty == TY_ && c.s == S_ && c.nt == NT_) return true;

template <>
hipError_t sor_dispatch<double>(const SorConfig& c, const double* pin, double* pout,
                                const double* F, int n, int pitch, PoissonCtl* ctl, double* part,
                                int check, double relax, hipStream_t st) {
  using T = double;
  CAV_SOR_CONFIGS_F64(CAV_TRY)
  return hipErrorInvalidValue;
}

template <>
hipError_t sor_dispatch<float>(const SorConfig& c, const float* pin, float* pout, const float* F,
                               int n, int pitch, PoissonCtl* ctl, double* part, int check,
                               double relax, hipStream_t st) {
  using T = float;
  CAV_SOR_CONFIGS_F32(CAV_TRY)
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

hipError_t launch_stage(const double* psi, const float* psi32, const double* w0,
                        const double* win, const double* wx, double* out, const double* wp,
                        double* p_out, int n, int pitch, const StageArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_stage, grid2d(n, n), dim3(kBlock), 0, st, psi, psi32, w0, win, wx, out,
                     wp, p_out, n, pitch, a);
  return hipGetLastError();
}

hipError_t launch_ctl_reset(PoissonCtl* ctl, double relax, double tol_hat, long long max_sweeps,
                            long long stall_window, long long sweeps_per_check, hipStream_t st,
                            double floor_ulps, const long long* gs_steps) {
  hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st, ctl, relax, tol_hat, max_sweeps,
                     stall_window, sweeps_per_check, floor_ulps, gs_steps);
  return hipGetLastError();
}

hipError_t launch_sor64(const SorConfig& cfg, const double* psi_in, double* psi_out,
                        const double* F, int n, int pitch, PoissonCtl* ctl, double* part,
                        int check, hipStream_t st) {
  return sor_dispatch<double>(cfg, psi_in, psi_out, F, n, pitch, ctl, part, check, 0.0, st);
}

hipError_t launch_sor32(const SorConfig& cfg, const float* d_in, float* d_out, const float* R,
                        int n, int pitch, PoissonCtl* ctl, double relax, hipStream_t st) {
  return sor_dispatch<float>(cfg, d_in, d_out, R, n, pitch, ctl, nullptr, 0, relax, st);
}

bool sor_config_supported(const SorConfig& c, bool fp32) {
  if (c.xcd_bands != 0 && c.xcd_bands != 1) return false;
  if (fp32) {
    CAV_SOR_CONFIGS_F32(CAV_HAS)
  } else {
    CAV_SOR_CONFIGS_F64(CAV_HAS)
  }
  return false;
}

int sor_max_blocks(int n) { return ((n + 31) / 32) * ((n + 31) / 32); }



#define CAV_BATCH_CONFIGS_F64(X) \
  X(32, 32, 1, 256)              \
  X(64, 32, 2, 512)              \
  X(64, 64, 2, 512)              \
  X(64, 64, 3, 512)              \
  X(64, 32, 3, 512)              \
  X(64, 32, 4, 512)              \
  X(64, 64, 3, 768)              \
  X(64, 64, 4, 512)              \
  X(84, 54, 5, 1024)

#define CAV_BATCH_CONFIGS_F32(X) \
  X(32, 32, 1, 256)              \
  X(64, 32, 2, 512)              \
  X(64, 64, 2, 1024)             \
  X(64, 64, 4, 1024)             \
  X(96, 64, 3, 1024)             \
  X(88, 56, 5, 1024)

bool batch_config_supported(const SorConfig& c, bool mixed) {
  if (c.xcd_bands != 0) return false;
  if (mixed) {
    CAV_BATCH_CONFIGS_F32(CAV_HAS)
  } else {
    CAV_BATCH_CONFIGS_F64(CAV_HAS)
  }
  return false;
}

template <typename K>
int occupancy_grid(K kernel, int nt, int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  return per_cu * cus;
}

int batch_grid(const SorConfig& c, bool mixed, int device) {
#define CAV_GRID64(TX_, TY_, S_, NT_)                                    \
  if (!mixed && c.tx == TX_ && c.ty == TY_ && c.s == S_ && c.nt == NT_) \
    return occupancy_grid(k_batch64<TX_, TY_, S_, NT_>, NT_, device);
#define CAV_GRID32(TX_, TY_, S_, NT_)                                   \
  if (mixed && c.tx == TX_ && c.ty == TY_ && c.s == S_ && c.nt == NT_) \
    return occupancy_grid(k_batch_mixed<TX_, TY_, S_, NT_>, NT_, device);
  CAV_BATCH_CONFIGS_F64(CAV_GRID64)
  CAV_BATCH_CONFIGS_F32(CAV_GRID32)
#undef CAV_GRID64
#undef CAV_GRID32
  return 0;
}

hipError_t launch_batch64(const SorConfig& c, const BatchMember* mem, int count, int total_tiles,
                          int pairs_per_check, BatchCtl* bc, unsigned int* flags, int grid,
                          long long spin_ticks, hipStream_t st) {
#define CAV_L64(TX_, TY_, S_, NT_)                                                              \
  if (c.tx == TX_ && c.ty == TY_ && c.s == S_ && c.nt == NT_) {                                 \
    hipLaunchKernelGGL((k_batch64<TX_, TY_, S_, NT_>), dim3(grid), dim3(NT_), 0, st, mem, count, \
                       total_tiles, pairs_per_check, bc, flags, spin_ticks);                    \
    return hipGetLastError();                                                                   \
  }
  CAV_BATCH_CONFIGS_F64(CAV_L64)
#undef CAV_L64
  return hipErrorInvalidValue;
}

hipError_t launch_batch_mixed(const SorConfig& c, const BatchMember* mem, int count,
                              int total_tiles, int inner_pairs, BatchCtl* bc, unsigned int* flags,
                              int grid, long long spin_ticks, hipStream_t st) {
#define CAV_L32(TX_, TY_, S_, NT_)                                                          \
  if (c.tx == TX_ && c.ty == TY_ && c.s == S_ && c.nt == NT_) {                             \
    hipLaunchKernelGGL((k_batch_mixed<TX_, TY_, S_, NT_>), dim3(grid), dim3(NT_), 0, st, mem, \
                       count, total_tiles, inner_pairs, bc, flags, spin_ticks);             \
    return hipGetLastError();                                                               \
  }
  CAV_BATCH_CONFIGS_F32(CAV_L32)
#undef CAV_L32
  return hipErrorInvalidValue;
}

int resid_blocks(int n) {
  const dim3 g = resid_grid(n);
  return (int)(g.x * g.y);
}

hipError_t launch_resid64(const double* psi, const double* F, float* R32, float* d32, int n,
                          int pitch, PoissonCtl* ctl, double* part, hipStream_t st,
                          long long sweeps_done) {
  const dim3 g = resid_grid(n);
  const int blocks = (int)(g.x * g.y);
  hipLaunchKernelGGL(k_resid64, g, dim3(kBlock), 0, st, psi, F, R32, d32, n, pitch, ctl, part);
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, st, ctl, part, blocks, sweeps_done);
  return hipGetLastError();
}

template <typename T>
hipError_t mg_residual(const T* psi, const T* F, T* r, int n, int pitch, double h,
                       const PoissonCtl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_mg_residual<T>, grid2d(n, n), dim3(kBlock), 0, st, psi, F, r, n, pitch,
                     (T)(1.0 / (0.3 * h * h)), ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t mg_restrict(const T* r, int nf, int pitchf, T* Fc, T* Ec, T* Ecb, int nc, int pitchc,
                       const PoissonCtl* ctl, hipStream_t st) {
  const double hc = 1.0 / (nc - 1);
  const double ratio = (double)(nc - 1) / (double)(nf - 1);
  hipLaunchKernelGGL(k_mg_restrict<T>, grid2d(nc, nc), dim3(kBlock), 0, st, r, nf, pitchf, Fc, Ec,
                     Ecb, nc, pitchc, (T)(0.3 * hc * hc * ratio * ratio), ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t mg_prolong(const T* Ec, int nc, int pitchc, T* psi, int nf, int pitchf,
                      const PoissonCtl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_mg_prolong<T>, grid2d(nf, nf), dim3(kBlock), 0, st, Ec, nc, pitchc, psi,
                     nf, pitchf, ctl);
  return hipGetLastError();
}

hipError_t launch_mg_residual(const double* psi, const double* F, double* r, int n, int pitch,
                              double h, const PoissonCtl* ctl, hipStream_t st) {
  return mg_residual<double>(psi, F, r, n, pitch, h, ctl, st);
}
hipError_t launch_mg_residual(const float* psi, const float* F, float* r, int n, int pitch,
                              double h, const PoissonCtl* ctl, hipStream_t st) {
  return mg_residual<float>(psi, F, r, n, pitch, h, ctl, st);
}
hipError_t launch_mg_restrict(const double* r, int nf, int pitchf, double* Fc, double* Ec,
                              double* Ecb, int nc, int pitchc, const PoissonCtl* ctl,
                              hipStream_t st) {
  return mg_restrict<double>(r, nf, pitchf, Fc, Ec, Ecb, nc, pitchc, ctl, st);
}
hipError_t launch_mg_restrict(const float* r, int nf, int pitchf, float* Fc, float* Ec,
                              float* Ecb, int nc, int pitchc, const PoissonCtl* ctl,
                              hipStream_t st) {
  return mg_restrict<float>(r, nf, pitchf, Fc, Ec, Ecb, nc, pitchc, ctl, st);
}
hipError_t launch_mg_prolong(const double* Ec, int nc, int pitchc, double* psi, int nf, int pitchf,
                             const PoissonCtl* ctl, hipStream_t st) {
  return mg_prolong<double>(Ec, nc, pitchc, psi, nf, pitchf, ctl, st);
}
hipError_t launch_mg_prolong(const float* Ec, int nc, int pitchc, float* psi, int nf, int pitchf,
                             const PoissonCtl* ctl, hipStream_t st) {
  return mg_prolong<float>(Ec, nc, pitchc, psi, nf, pitchf, ctl, st);
}

template <typename T>
hipError_t mg_fused(T* E, const T* F, int pitch, const int* n, int levels, int nu,
                    int coarse_sweeps, double coarse_relax, const PoissonCtl* ctl, hipStream_t st) {
  if (levels < 1 || levels > kMgFuseLevels || n[0] > kMgFuseMax) return hipErrorInvalidValue;
  MgFusedArgs a{};
  a.levels = levels;
  int nodes = 0;
  for (int l = 0; l < levels; ++l) {
    a.n[l] = n[l];
    const double h = 1.0 / (n[l] - 1);
    a.inv03h2[l] = 1.0 / (0.3 * h * h);
    if (l > 0) {
      const double ratio = (double)(n[l] - 1) / (double)(n[l - 1] - 1);
      a.scale[l] = 0.3 * h * h * ratio * ratio;
    }
    nodes += n[l] * n[l];
  }
  a.nu = nu;
  a.coarse_sweeps = coarse_sweeps;
  a.coarse_relax = coarse_relax;
  if (nodes > kMgFuseNodes) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mg_fused<T>, dim3(1), dim3(kMgFuseThreads), 0, st, E, F, pitch, a, ctl);
  return hipGetLastError();
}

int mg_fuse_max() { return kMgFuseMax; }

hipError_t launch_mg_fused(double* E, const double* F, int pitch, const int* n, int levels,
                           int nu, int coarse_sweeps, double coarse_relax, const PoissonCtl* ctl,
                           hipStream_t st) {
  return mg_fused<double>(E, F, pitch, n, levels, nu, coarse_sweeps, coarse_relax, ctl, st);
}
hipError_t launch_mg_fused(float* E, const float* F, int pitch, const int* n, int levels, int nu,
                           int coarse_sweeps, double coarse_relax, const PoissonCtl* ctl,
                           hipStream_t st) {
  return mg_fused<float>(E, F, pitch, n, levels, nu, coarse_sweeps, coarse_relax, ctl, st);
}

hipError_t launch_sor64_relax(const SorConfig& cfg, const double* psi_in, double* psi_out,
                              const double* F, int n, int pitch, PoissonCtl* ctl, double relax,
                              hipStream_t st) {
  return sor_dispatch<double>(cfg, psi_in, psi_out, F, n, pitch, ctl, nullptr, 0, relax, st);
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

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 4;
  const int blocks = (int)std::min<size_t>(1024, (words + kBlock - 1) / kBlock);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(kBlock), 0, st, static_cast<unsigned int*>(p),
                     words);
  return hipGetLastError();
}

hipError_t launch_shadow(const double* a, float* b, int n, int pitch, hipStream_t st) {
  hipLaunchKernelGGL(k_shadow, grid2d(pitch, n), dim3(kBlock), 0, st, a, b, n, pitch);
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

hipError_t launch_warm(double* psi, double* hist, size_t fstride, int n, int pitch, int stage,
                       int levels, const long long* count, const double* wtab, hipStream_t st) {
  hipLaunchKernelGGL(k_warm, grid2d(n, n), dim3(kBlock), 0, st, psi, hist, fstride, n, pitch,
                     stage, levels, count, wtab);
  return hipGetLastError();
}

hipError_t launch_warm_tick(long long* count, hipStream_t st) {
  hipLaunchKernelGGL(k_warm_tick, dim3(1), dim3(64), 0, st, count);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Scratch memory of the allocation-free Poisson solve (cavity_poisson_noalloc):
// a file-scope device array that each device holds for the life of the
// process.  Host code never passes the array's name to a kernel (in host code
// it is a host-side stand-in, not a device address): noalloc_scratch returns
// the address hipGetSymbolAddress gives for the current device, looked up
// once per device.
// ---------------------------------------------------------------------------
constexpr int kNoAllocMaxN = 1024;
// three pitched FP64 fields of the largest grid (right-hand side and the
// iterate's ping-pong pair; pitch(1024) = 1024), then 64 KiB for the partial
// maxima of the residual checks and the control block
constexpr size_t kNoAllocFieldBytes = (size_t)kNoAllocMaxN * kNoAllocMaxN * sizeof(double);
constexpr size_t kNoAllocBytes = 3 * kNoAllocFieldBytes + 64 * 1024;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

int noalloc_max_n() { return kNoAllocMaxN; }
size_t noalloc_bytes() { return kNoAllocBytes; }

hipError_t noalloc_scratch(void** out) {
  static std::mutex mu;
  static void* ptr[kNoAllocMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return hipSuccess;
}

// Tile shapes of the resident solve.
#define CAV_RESIDENT_CONFIGS(X) \
  X(64, 64, 4, 768)             \
  X(32, 32, 2, 256)

size_t resident_flag_bytes(int n) {
  return (size_t)sor_max_blocks(n) * kFlagStride * sizeof(unsigned int);
}

namespace {
template <int TX, int TY, int S, int NT>
int resident_capacity(int device) {
  return occupancy_grid(k_sor_resident<TX, TY, S, NT>, NT, device);
}
}  // namespace

bool resident_supported(const SorConfig& c, int n, int device) {
#define CAV_RES_FITS(TX_, TY_, S_, NT_)                                                \
  if (c.tx == TX_ && c.ty == TY_ && c.s == S_ && c.nt == NT_)                          \
    return ((n + TX_ - 1) / TX_) * ((n + TY_ - 1) / TY_) <=                            \
           resident_capacity<TX_, TY_, S_, NT_>(device);
  CAV_RESIDENT_CONFIGS(CAV_RES_FITS)
#undef CAV_RES_FITS
  return false;
}

hipError_t launch_sor64_resident(const SorConfig& c, double* psi, double* psi_b, const double* F,
                                 int n, int pitch, PoissonCtl* ctl, double* part,
                                 unsigned int* flags, ResidentCtl* rctl, int rounds_per_check,
                                 long long spin_ticks, int device, hipStream_t st) {
  if (!resident_supported(c, n, device) || rounds_per_check < 3)
    return hipErrorInvalidConfiguration;
  hipError_t e = launch_zero(flags, resident_flag_bytes(n), st);
  if (e != hipSuccess) return e;
  if ((e = launch_zero(rctl, sizeof(ResidentCtl), st)) != hipSuccess) return e;
#define CAV_RES_LAUNCH(TX_, TY_, S_, NT_)                                                    \
  if (c.tx == TX_ && c.ty == TY_ && c.s == S_ && c.nt == NT_) {                            \
    const int tx = (n + TX_ - 1) / TX_, ty = (n + TY_ - 1) / TY_;                          \
    hipLaunchKernelGGL((k_sor_resident<TX_, TY_, S_, NT_>), dim3(tx * ty), dim3(NT_), 0, st, \
                       psi, psi_b, F, n, pitch, tx, ty, ctl, part, flags, rctl,            \
                       rounds_per_check, spin_ticks);                                      \
    return hipGetLastError();                                                              \
  }
  CAV_RESIDENT_CONFIGS(CAV_RES_LAUNCH)
#undef CAV_RES_LAUNCH
  return hipErrorInvalidConfiguration;
}

}  // namespace cav
