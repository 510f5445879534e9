// Pass kernels of the iterative Fourier-transform hologram loop.
//
// Every kernel is one HBM pass over the [H][W] complex64 field: a row pass
// (1D FFT of each row, the contiguous axis) or a column pass (1D FFT of each
// column through padded LDS tiles), with the pointwise steps of the method
// fused into the load and store sides so that no separate elementwise pass
// exists:
//
//   Gerchberg-Saxton (Sec. 7.3, HoloGenAlgGSCuda; Gerchberg & Saxton 1972):
//     k_gs_row_start  phi0 -> SLM constraint -> * Q1 -> row FFT
//     k_gs_col        column FFT -> NMSE partial, amplitude replacement
//                     -> inverse column FFT          (replay plane)
//     k_gs_row        inverse row FFT -> * conj(Q1) -> SLM constraint
//                     [-> phase / level output] -> * Q1 -> row FFT
//   One-Step Phase-Retrieval (Sec. 7.3, HoloGenAlgOSPRCuda; Cable et al. 2004):
//     k_ospr_a        T e^{i theta} (ifftshift on load) -> inverse row FFT
//     k_ospr_b        inverse column FFT -> binarise Re -> levels -> column FFT
//     k_ospr_c        row FFT -> |.|^2 accumulated (fftshift on store) [-> NMSE]
//   Propagation (Fourier / single-FFT Fresnel):
//     k_prop_row, k_prop_col
//   Gradient-descent hologram (multi-plane NMSE loss, Wirtinger gradient, Adam):
//     k_grad_rows     START: phi -> Q1_j exp(i phi) -> row FFT, every plane
//     k_gs_col        column FFT -> loss partial, dL/dconj(U) -> inverse column FFT
//                     (one launch over every plane of every problem)
//     k_grad_rows     ADJ: inverse row FFT -> 2 Im(conj(V_j) G_j) summed over
//                     the planes in registers [-> gradient out] [-> Adam step
//                     on phi] [-> START of the next state]
//
// Conventions.  The field is row-major [H][W] complex64 (float2).  The forward
// transform uses exp(-2 pi i ...) and is unnormalised; inverse transforms
// inside the loops are left unscaled because every constraint that follows
// them (phase-only projection, quantiser, sign test) is invariant to a
// positive scale.  Q1 = q_y[y] q_x[x] is the Fresnel source chirp (tables of
// H + W entries); a null q_y selects a Fourier hologram.
//
// Launch shape.  A row team is one wavefront when T = 64, so its row index is
// wave-uniform and lives in a scalar register; teams past the last row load a
// valid row and skip their stores, so no per-element branch exists.  Column
// workgroups are mapped so that each XCD gets a contiguous range of column
// tiles: the C * 8-byte row segments of neighbouring tiles share 128-byte
// lines, and keeping them on one XCD lets that XCD's L2 serve them.
#pragma once

#include "fft_core.hpp"
#include "sizes.hpp"

#include <type_traits>

namespace hg {

constexpr float TWO_PI_F = 6.28318530717958647692f;

// Device-side scalars computed once per call (see k_stats_final).
struct Scalars {
  float a;          // N_px / sum(I): intensity normaliser of the replay field
  float b;          // N_px / sum(T^2): normaliser of the target intensity
  double denom;     // N_px^2 sum(T^4) / sum(T^2)^2 = N_px^2 sum (T_I / sum T_I)^2
  double sum_t2, sum_t4, sum_a2;
  float g;          // 2 a / denom: dNMSE/dI = g (a I - b T^2) for the gradient pass
  float c;          // sqrt(sum I / sum T^2): the target scale of a signal window
};

// SLM constraint shared by the GS kernels.
struct SlmConstraint {
  const float2* __restrict__ lvl_tab;  // exp(i 2 pi l / L), FP64-built; null = continuous
  int levels;
  float inv_delta;                     // L / (2 pi)
  double inv_delta_f64;                // L / (2 pi) for the one-off quantisation of phi0
  float2 half_step;                    // exp(i pi / L): rotates decision boundaries onto axes
  int amplitude;                       // amplitude-only SLM: nearest non-negative real value
  float amp_scale;                     // amplitude output of a loop state: 1 / (H W) undoes
                                       // the two unscaled inverse transforms
};

// ---------------------------------------------------------------------------
// SLM-plane constraint
// ---------------------------------------------------------------------------
// floor(angle / (pi/4)) of a non-zero vector, angle taken in [0, 2 pi),
// without branches: fold the lower half-plane onto the upper one (angle - pi),
// then the second quadrant onto the first (angle - pi/2), then compare the two
// coordinates (angle >= pi/4).  Each boundary goes to the higher sector, as
// floor() does: the upper half is y > 0 or (y == 0 and x > 0), the first
// quadrant of it x > 0, and the upper octant v >= u.
__device__ __forceinline__ int octant(float x, float y) {
  const bool upper = (y > 0.0f) | ((y == 0.0f) & (x > 0.0f));
  const float x1 = upper ? x : -x, y1 = upper ? y : -y;
  const bool second = !(x1 > 0.0f);
  const float u = second ? y1 : x1, v = second ? -x1 : y1;
  return (upper ? 0 : 4) + (second ? 2 : 0) + (v >= u ? 1 : 0);
}

// Level of a complex value: floor(mod(atan2(Im, Re), 2 pi) / Delta + 1/2) mod L.
// For L in {2, 4, 8} the value is first rotated by Delta/2, which puts the
// decision boundaries on the axes and diagonals, and the level is read from
// signs and magnitude comparisons; other L use atan2.  G = 0 has level 0.
__device__ __forceinline__ int quant_level(float2 g, const SlmConstraint& slm) {
  if (slm.levels == 8 || slm.levels == 4 || slm.levels == 2) {
    if (g.x == 0.0f && g.y == 0.0f) return 0;
    const float2 r = cmul(g, slm.half_step);
    const int o = octant(r.x, r.y);
    return slm.levels == 8 ? o : (slm.levels == 4 ? (o >> 1) : (o >> 2));
  }
  float th = atan2f(g.y, g.x);
  if (th < 0.0f) th += TWO_PI_F;
  int l = (int)floorf(th * slm.inv_delta + 0.5f);
  return l >= slm.levels ? l - slm.levels : l;
}

// Level of a phase value in radians (any finite value), decided in FP64: the
// starting phase is an input, so its quantisation is made exactly as the
// definition states rather than in the precision of the loop.
__device__ __forceinline__ int quant_phase(float phi, int levels, double inv_delta) {
  long long l = (long long)floor((double)phi * inv_delta + 0.5) % levels;
  return (int)(l < 0 ? l + levels : l);
}

// Unit-modulus value G/|G| (G = 0 -> 1).
__device__ __forceinline__ float2 unit_of(float2 g) {
  const float n2 = cnorm(g);
  if (n2 > 0.0f) {
    const float s = rsqrtf(n2);
    return make_float2(g.x * s, g.y * s);
  }
  return make_float2(1.0f, 0.0f);
}

__device__ __forceinline__ float wrap_phase(float2 u) {
  float p = atan2f(u.y, u.x);
  if (p < 0.0f) p += TWO_PI_F;
  if (p >= TWO_PI_F) p -= TWO_PI_F;
  return p;
}

// ---------------------------------------------------------------------------
// addressing helpers
// ---------------------------------------------------------------------------
// Global loads and stores with a 32-bit unsigned byte offset from a base
// pointer: the base stays in scalar registers and the address needs no 64-bit
// arithmetic.  Every buffer the kernels touch is below 4 GiB.
template <class T>
__device__ __forceinline__ T ldg(const T* base, uint32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void stg(T* base, uint32_t i, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T)) = v;
}

// Field accesses of the GS-family passes of length N.  For N <= 1024 they
// carry the nontemporal hint: each pass reads and writes the field once, and
// on the tiled 1024^2 loop dropping the hint from any one of its four field
// accesses costs 11-19 % per iteration.  Longer passes use plain accesses: at
// 2048^2 the hint costs about 1 % (tiled), and in row order it made a column
// pass, whose 32-byte row segments neighbouring workgroups share through L2,
// 1.5x slower.  The propagation and OSPR passes use plain accesses.
template <int N>
__device__ __forceinline__ float2 ldg_field(const float2* base, uint32_t i) {
  if constexpr (N <= 1024) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f2v w = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(reinterpret_cast<const char*>(base) + i * 8u));
    return make_float2(w.x, w.y);
  } else {
    return ldg(base, i);
  }
}
template <int N>
__device__ __forceinline__ void stg_field(float2* base, uint32_t i, float2 v) {
  if constexpr (N <= 1024) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f2v w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<f2v*>(reinterpret_cast<char*>(base) + i * 8u));
  } else {
    stg(base, i, v);
  }
}

// The same for per-pixel float arrays that a pass streams once (the gradient
// row pass's phase, accumulator and Adam moments): the hint took 13 % off an
// Adam step of the three-plane 1024^2 problem.
template <int N>
__device__ __forceinline__ float ldg_f(const float* base, uint32_t i) {
  if constexpr (N <= 1024)
    return __builtin_nontemporal_load(reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + i * 4u));
  else
    return ldg(base, i);
}
template <int N>
__device__ __forceinline__ void stg_f(float* base, uint32_t i, float v) {
  if constexpr (N <= 1024)
    __builtin_nontemporal_store(v, reinterpret_cast<float*>(reinterpret_cast<char*>(base) + i * 4u));
  else
    stg(base, i, v);
}

// Keeps the loads issued above it above it: the scheduler would otherwise sink
// table loads into the first FFT stage, and with one wavefront per SIMD their
// latency would then stall the second stage instead of overlapping the field
// loads.
__device__ __forceinline__ void issue_loads_here() { __builtin_amdgcn_sched_barrier(0); }

// (i + s) mod n for 0 <= i, s < n
template <int NC>
__device__ __forceinline__ int wrap_add(int i, int s) {
  if constexpr ((NC & (NC - 1)) == 0) return (i + s) & (NC - 1);
  else { const int j = i + s; return j >= NC ? j - NC : j; }
}
__device__ __forceinline__ int wrap_add_rt(int i, int s, int n) {
  const int j = i + s;
  return j >= n ? j - n : j;
}

// ---------------------------------------------------------------------------
// launch-shape helpers
// ---------------------------------------------------------------------------
// Workgroup b of n runs on XCD b % 8; give XCD x the contiguous tile range
// [x * n/8, ...) so that neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = b & 7, local = b >> 3;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + local;
}

// ---------------------------------------------------------------------------
// Field layout of the Gerchberg-Saxton family (GS, multi-plane GS, gradient,
// angular-spectrum GS) and of OSPR between their row and column passes,
// chosen per plan:
//   ft = 0: row order, element (y, x) at y W + x;
//   ft > 0: column tiles of ft (a power of two and a multiple of the column
//           pass's tile width), stored one tile after another, each row by
//           row: (y, x) at ((x / ft) H + y) ft + x % ft, the width rounded up
//           to a multiple of ft (the padding is never read).
// Tiled, a column pass moves short contiguous runs of whole tiles instead of
// C * 8-byte row segments spread over the frame, and a row pass whose
// workgroup interleaves its rows across the lanes (RowTeam) moves whole
// lines.  A row kernel of length N is compiled for one tile width,
// RowTeam<RowCfg<N>>::FT (0: row order only); a plan is tiled when that
// width is a multiple of its column pass's.  Propagation and the
// single-pixel search keep row order.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr uint32_t field_width(uint32_t w, uint32_t ft) { return ft ? (w + ft - 1) / ft * ft : w; }

// Row and thread of a row-pass thread; rows are packed TEAMS to a workgroup.
// With a tiled field and teams that synchronise through s_barrier, groups of
// ft consecutive lanes take consecutive rows, so one access of a wavefront
// covers ft-wide tile pieces of several rows; otherwise team = thread / T.
template <class C>
struct RowTeam {
  using P = typename C::P;
  // Tile width of the tiled layout these row kernels take (0: none).  The
  // teams must interleave (s_barrier exchanges) and every register slot must
  // lie a multiple of FT from t.  With one team (one row) per workgroup a
  // wavefront access covers FT-wide pieces of many tiles, whose lines the
  // workgroups of the neighbouring rows (on the same XCD) complete in L2.
  static constexpr int FT = C::FT;
  static_assert(FT == 0 || (!C::WAVE_SYNC && (FT & (FT - 1)) == 0 && P::T % FT == 0 &&
                            Layout<P, true, false>::STRIDE % FT == 0 && Layout<P, false, true>::STRIDE % FT == 0 &&
                            Layout<P, false, false>::STRIDE % FT == 0),
                "tile width unusable with this row shape");
  int t, team, y;
  bool live;
  // ft: the field's tile width, 0 or FT
  __device__ __forceinline__ RowTeam(int H, int ft = 0) {
    if (FT && ft) {
      team = (threadIdx.x / FT) % C::TEAMS;
      t = threadIdx.x % FT + FT * (threadIdx.x / (FT * C::TEAMS));
    } else {
      team = threadIdx.x / P::T;
      t = threadIdx.x % P::T;
    }
    // Tiled: neighbouring workgroups (whose rows share the field's cache
    // lines when a tile row is narrower than a line) go to one XCD.
    const int blk = (FT && ft) ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    int row = blk * C::TEAMS + team;
    if constexpr (!FT && P::T == 64) row = __builtin_amdgcn_readfirstlane(row);
    live = row < H;
    y = live ? row : H - 1;
  }
};

// Offsets of one thread's elements of row y in the field: the element at x
// (a register slot's position, a compile-time distance x - t from t, a
// multiple of FT) lies at base + (x - t) step.
struct RowField {
  uint32_t base, step;
  int t;
  template <int N, int FT>
  __device__ __forceinline__ static RowField make(int t, int y, int H, int ft) {
    if (FT && ft) return {(((uint32_t)t / FT) * (uint32_t)H + (uint32_t)y) * FT + (uint32_t)t % FT, (uint32_t)H, t};
    return {(uint32_t)y * N + (uint32_t)t, 1u, t};
  }
  __device__ __forceinline__ uint32_t at(int x) const { return base + (uint32_t)(x - t) * step; }
};

// Offsets of one column of a column pass: element y at base + y step (ft:
// the field's tile width or 0).
struct ColField {
  uint32_t base, step;
  __device__ __forceinline__ ColField(uint32_t x, int W, int H, int ft) {
    if (ft) {
      const uint32_t l = __builtin_ctz(ft);
      base = ((x >> l) * (uint32_t)H << l) + (x & (ft - 1));
      step = ft;
    } else {
      base = x;
      step = (uint32_t)W;
    }
  }
  __device__ __forceinline__ uint32_t at(int y) const { return base + (uint32_t)y * step; }
};

// Wavefront then workgroup sum of one float per thread, fixed order.
template <int THREADS>
__device__ __forceinline__ float block_sum(float v, float* red) {
  static_assert(THREADS % 64 == 0, "whole wavefronts");
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  constexpr int NW = THREADS / 64;
  if constexpr (NW == 1) {
    return v;
  } else {
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float s = 0.0f;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < NW; ++i) s += red[i];
    }
    return s;
  }
}

extern __shared__ float2 hg_dyn_lds[];

// ---------------------------------------------------------------------------
// LDS layout of a pass kernel: the teams' exchange regions, then the twiddle
// images when they are too large for registers (see PassTwiddles), then (row
// kernels) one table of N complex values such as the Fresnel chirp q_x when it
// is shared through LDS (see RowTable).
// ---------------------------------------------------------------------------
// Every kernel of a length shares one LDS reservation, sized by the twiddle
// needs of the kernels that run both transform orders; one-order kernels
// must fit inside it.
template <class P, int THREADS>
constexpr bool tw_fits_reservation() {
  constexpr int both = PassTwiddles<P, THREADS, true, true>::LDS_WORDS;
  return PassTwiddles<P, THREADS, true, false>::LDS_WORDS <= both &&
         PassTwiddles<P, THREADS, false, true>::LDS_WORDS <= both;
}

template <int N>
struct RowLds {
  using C = RowCfg<N>;
  using P = typename C::P;
  static_assert(tw_fits_reservation<P, C::THREADS>(), "one-order twiddles exceed the LDS reservation");
  // a team's exchange region, padded so that the teams sharing a wavefront
  // start on different LDS banks: 8 mod 16 complex values where tiled rows
  // interleave two teams across the lanes (1024-point SLM pass 8.26 -> 7.88 us
  // against 4 mod 16; 0, 12 mod 16 as slow as 4), else 4 mod 16
  static constexpr int TEAM_OFF = C::FT ? 8 : 4;
  static constexpr int TEAM = lds_len(N) + (TEAM_OFF + 16 - lds_len(N) % 16) % 16;
  static constexpr int TWF = C::TEAMS * TEAM;
  static constexpr int TAB = TWF + PassTwiddles<P, C::THREADS, true, true>::LDS_WORDS;
  // a per-column table is shared through LDS only when a thread's share of it
  // would take more than 16 registers (RowTable)
  static constexpr bool TABLE_IN_LDS = P::REGS > 16;
  static constexpr int WORDS = TAB + (TABLE_IN_LDS ? N : 0);
};
template <class CC>
struct ColLdsOf {
  using C = CC;
  using P = typename C::P;
  static_assert(tw_fits_reservation<P, C::THREADS>(), "one-order twiddles exceed the LDS reservation");
  static constexpr int TWF = C::C * lds_len(P::N);
  static constexpr int WORDS = TWF + PassTwiddles<P, C::THREADS, true, true>::LDS_WORDS;
};
template <int N>
using ColLds = ColLdsOf<ColCfg<N>>;

// Column configuration of the single-hologram (WIDE = false) or batched
// (WIDE = true) GS-family column passes.
template <int N, bool WIDE>
using ColCfgSel = std::conditional_t<WIDE, ColCfgWide<N>, ColCfg<N>>;

// Per-column sums of a column pass in an order that does not depend on how
// many columns share a workgroup, so that single and batched launches give
// bitwise the same error values: a fixed pairwise tree over the team's
// threads t within blocks of BT consecutive t (wavefront shuffles), then the
// blocks added in order.  BT = 64 / (the widest column count of the length),
// so that a block always lies inside one wavefront.
template <int N>
struct ColSum {
  static constexpr int CMAX = ColCfgWide<N>::C > ColCfg<N>::C ? ColCfgWide<N>::C : ColCfg<N>::C;
  static constexpr int T = ColCfg<N>::P::T;
  static constexpr int BT = (64 / CMAX) < T ? (64 / CMAX) : T;
  static constexpr int BLOCKS = T / BT;
  static_assert(BT >= 1 && T % BT == 0, "column-sum blocks must tile the team");
};

// One float per thread of column c, team thread t -> the column's total in
// the thread with t == 0 (others: unspecified).  red: C * BLOCKS floats.
template <int N, class CC>
__device__ __forceinline__ float column_sum(float v, int c, int t, float* red) {
  using S = ColSum<N>;
  static_assert(CC::C * S::BT <= 64, "a block must lie inside one wavefront");
#pragma unroll
  for (int off = CC::C; off < CC::C * S::BT; off <<= 1) v += __shfl_xor(v, off, 64);
  if constexpr (S::BLOCKS == 1) {
    return v;
  } else {
    if (t % S::BT == 0) red[c * S::BLOCKS + t / S::BT] = v;
    __syncthreads();
    float s = 0.0f;
    if (t == 0) {
#pragma unroll
      for (int b = 0; b < S::BLOCKS; ++b) s += red[c * S::BLOCKS + b];
    }
    return s;
  }
}

// The same for doubles (signal-window sums).
template <int N, class CC>
__device__ __forceinline__ double column_sum_f64(double v, int c, int t, double* red) {
  using S = ColSum<N>;
  static_assert(CC::C * S::BT <= 64, "a block must lie inside one wavefront");
#pragma unroll
  for (int off = CC::C; off < CC::C * S::BT; off <<= 1) v += __shfl_xor(v, off, 64);
  if constexpr (S::BLOCKS == 1) {
    return v;
  } else {
    if (t % S::BT == 0) red[c * S::BLOCKS + t / S::BT] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0) {
#pragma unroll
      for (int b = 0; b < S::BLOCKS; ++b) s += red[c * S::BLOCKS + b];
    }
    __syncthreads();
    return s;
  }
}

// Per-column table of a row pass (the Fresnel chirp q_x), read at the
// positions of layout L.  With at most 16 register slots per thread, each
// thread loads its own entries straight from global memory together with the
// field; larger layouts share one LDS copy per workgroup, visible after the
// caller's barrier.
template <int N, class L>
struct RowTable {
  using P = typename RowCfg<N>::P;
  static constexpr bool IN_REGS = !RowLds<N>::TABLE_IN_LDS;
  static constexpr bool USES_LDS = !IN_REGS;
  float2 r[IN_REGS ? P::REGS : 1];
  __device__ __forceinline__ void begin(const float2* src, int t) {
    if constexpr (IN_REGS) for_layout<L>(t, [&](int s, int x) { r[s] = src[x]; });
    else lds_fill<RowCfg<N>::THREADS, N>(hg_dyn_lds + RowLds<N>::TAB, src);
  }
  __device__ __forceinline__ float2 at(int s, int x) const {
    if constexpr (IN_REGS) return r[s];
    else return hg_dyn_lds[RowLds<N>::TAB + x];
  }
};

// A second per-column table of a row pass (the next plane's chirp in the
// gradient row pass): registers when they fit, else read from global memory
// where it is used (the LDS table region holds the first table).
template <int N, class L>
struct RowTableDirect {
  using P = typename RowCfg<N>::P;
  static constexpr bool IN_REGS = P::REGS <= 16;
  float2 r[IN_REGS ? P::REGS : 1];
  const float2* src;
  __device__ __forceinline__ void begin(const float2* s, int t) {
    src = s;
    if constexpr (IN_REGS) for_layout<L>(t, [&](int i, int x) { r[i] = s[x]; });
  }
  __device__ __forceinline__ float2 at(int i, int x) const {
    if constexpr (IN_REGS) return r[i];
    else return src[x];
  }
};

// A per-column table read from global memory where it is used.
struct RowTableGlobal {
  const float2* src;
  __device__ __forceinline__ void begin(const float2* s, int) { src = s; }
  __device__ __forceinline__ float2 at(int, int x) const { return src[x]; }
};

// ===========================================================================
// Propagation passes: out = post * Sh_out(FFT2(Sh_in(pre * in))), separable
// pre/post tables and cyclic shifts (Fourier: none; Fresnel: chirps + centring).
// ===========================================================================
struct PropRowArgs {
  const float2* in;
  float2* out;
  int H;
  int sx_in, sx_out;
  const float2* pre_y;  // null -> no pre-multiply
  const float2* pre_x;
  const float2* tw;     // twiddle image, forward radix order
  const float2* twr;    // twiddle image, reversed order (== tw for palindromic plans)
};

template <int N, int DIR>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_prop_row(PropRowArgs a) {
  using C = RowCfg<N>;
  using P = typename C::P;
  using LL = RowLds<N>;
  using L0 = Layout<P, false, false>;
  using L1 = Layout<P, false, true>;
  const RowTeam<C> rt(a.H);
  const int t = rt.t;
  LdsView<1> lds{hg_dyn_lds + rt.team * LL::TEAM};
  float2 v[P::REGS];
  const uint32_t row = (uint32_t)rt.y * N;
  for_layout<L0>(t, [&](int s, int x) { v[s] = ldg(a.in, row + wrap_add<N>(x, a.sx_in)); });
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, true, false>;
  TW tw;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  // the pre-multiply table: each thread's entries in registers, or shared
  // through LDS when they would take more than 16 registers
  float2 pre[LL::TABLE_IN_LDS ? 1 : P::REGS];
  if constexpr (LL::TABLE_IN_LDS) {
    if (a.pre_y) lds_fill<C::THREADS, N>(hg_dyn_lds + LL::TAB, a.pre_x);
  } else {
    if (a.pre_y) for_layout<L0>(t, [&](int s, int x) { pre[s] = a.pre_x[wrap_add<N>(x, a.sx_in)]; });
  }
  if constexpr (LL::TABLE_IN_LDS || TW::USES_LDS) __syncthreads();
  if (a.pre_y) {
    const float2 py = a.pre_y[rt.y];
    for_layout<L0>(t, [&](int s, int x) {
      const float2 q = LL::TABLE_IN_LDS ? hg_dyn_lds[LL::TAB + wrap_add<N>(x, a.sx_in)] : pre[LL::TABLE_IN_LDS ? 0 : s];
      v[s] = cmul(v[s], cmul(py, q));
    });
  }
  tw.template run<false, DIR, C::WAVE_SYNC>(v, t, lds);
  if (rt.live) for_layout<L1>(t, [&](int s, int k) { stg(a.out, row + wrap_add<N>(k, a.sx_out), v[s]); });
}

struct PropColArgs {
  float2* io;
  int W;
  int sy_in, sy_out;
  const float2* post_y;  // null -> no post-multiply
  const float2* post_x;
  float scale;
  const float2* tw;
  const float2* twr;
};

template <int N, int DIR>
__global__ __launch_bounds__(ColCfg<N>::THREADS) void k_prop_col(PropColArgs a) {
  using C = ColCfg<N>;
  using P = typename C::P;
  using LL = ColLds<N>;
  using L0 = Layout<P, false, false>;
  using L1 = Layout<P, false, true>;
  const int c = threadIdx.x % C::C, t = threadIdx.x / C::C;
  const int col = xcd_tile(blockIdx.x, gridDim.x) * C::C + c;
  const bool live = col < a.W;
  const uint32_t x = live ? col : a.W - 1;
  LdsView<C::C> lds{hg_dyn_lds + c};
  float2 v[P::REGS];
  for_layout<L0>(t, [&](int s, int y) { v[s] = ldg(a.io, (uint32_t)wrap_add<N>(y, a.sy_in) * a.W + x); });
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, true, false>;
  TW tw;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  if constexpr (TW::USES_LDS) __syncthreads();
  tw.template run<false, DIR, C::WAVE_SYNC>(v, t, lds);
  if (live) {
    const float2 px = a.post_y ? ldg(a.post_x, x) : make_float2(1.f, 0.f);
    for_layout<L1>(t, [&](int s, int k) {
      k = wrap_add<N>(k, a.sy_out);
      float2 z = v[s];
      if (a.post_y) z = cmul(z, cmul(ldg(a.post_y, k), px));
      stg(a.io, (uint32_t)k * a.W + x, cscale(z, a.scale));
    });
  }
}

// ===========================================================================
// Gerchberg-Saxton
// ===========================================================================
struct GsRowArgs {
  float2* field;
  const float* phase0;      // start kernel only: starting phase [H][W]
  const float* illum;       // SLM amplitude A [H][W]; null -> 1
  int H;
  const float2* q1y;        // Fresnel source chirp; null -> Fourier
  const float2* q1x;
  SlmConstraint slm;
  float* phase_out;         // non-null on the pass that produces the output state
  uint8_t* levels_out;
  const float2* tw;
  const float2* twr;
  // General pass only: when q_out_set, the SLM field leaves for the next
  // replay plane through the chirp qo (null -> Fourier plane) instead of Q1.
  int q_out_set;
  const float2* qoy;
  const float2* qox;
  uint32_t px;              // batch: pixels per hologram (row-order arrays)
  uint32_t fpx;             // batch: field elements per hologram
  int ft;                   // field layout (RowTeam, RowField)
  // Batch item blockIdx.y of a launch over a stack of same-shape holograms
  // (gridDim.y items; the illumination is shared).
  __device__ __forceinline__ void select_item() {
    const uint32_t off = blockIdx.y * px;
    field += blockIdx.y * fpx;
    if (phase0) phase0 += off;
    if (phase_out) phase_out += off;
    if (levels_out) levels_out += off;
  }
};

// SLM-constraint variants of the steady-state row pass.
enum { GS_CONT = 0, GS_QATAN = 1, GS_Q2 = 2, GS_Q4 = 4, GS_Q8 = 8, GS_AMP = 16 };
__host__ __device__ constexpr int gs_mode_index(int mode) {
  return mode == GS_CONT ? 0 : mode == GS_QATAN ? 1 : mode == GS_Q2 ? 2 : mode == GS_Q4 ? 3 : mode == GS_Q8 ? 4 : 5;
}

// Output of one SLM state: phase and level (phase-only SLMs) or the amplitude
// u.x scaled by amp (amplitude-only SLMs; level 0).
__device__ __forceinline__ void write_state(const GsRowArgs& a, uint32_t idx, float2 u, int level, float amp = 1.0f) {
  if (a.slm.amplitude) {
    if (a.phase_out) stg(a.phase_out, idx, u.x * amp);
    if (a.levels_out) stg(a.levels_out, idx, (uint8_t)0);
  } else if (a.slm.lvl_tab) {
    if (a.phase_out) stg(a.phase_out, idx, (float)level * (TWO_PI_F / (float)a.slm.levels));
    if (a.levels_out) stg(a.levels_out, idx, (uint8_t)level);
  } else {
    if (a.phase_out) stg(a.phase_out, idx, wrap_phase(u));
    if (a.levels_out) stg(a.levels_out, idx, (uint8_t)0);
  }
}

// phi0 -> H_0 = A exp(i C(phi0)) -> Q1 H_0 -> row FFT.  Runs once per call.
template <int N>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_gs_row_start(GsRowArgs a) {
  a.select_item();
  using C = RowCfg<N>;
  using P = typename C::P;
  using LL = RowLds<N>;
  using L0 = Layout<P, false, false>;
  using L1 = Layout<P, false, true>;
  const RowTeam<C> rt(a.H, a.ft);
  const int t = rt.t;
  LdsView<1> lds{hg_dyn_lds + rt.team * LL::TEAM};
  float2 v[P::REGS];
  const uint32_t row = (uint32_t)rt.y * N;
  float ph[P::REGS];
  for_layout<L0>(t, [&](int s, int x) { ph[s] = ldg(a.phase0, row + x); });
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, true, false>;
  using QX = RowTable<N, L0>;
  TW tw;
  QX qx;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  if (a.q1y) qx.begin(a.q1x, t);
  if constexpr (TW::USES_LDS || QX::USES_LDS) __syncthreads();
  const float2 qy = a.q1y ? a.q1y[rt.y] : make_float2(1.f, 0.f);
  const bool out = rt.live && (a.phase_out || a.levels_out);
  for_layout<L0>(t, [&](int s, int x) {
    float2 u;
    int level = 0;
    if (a.slm.amplitude) {
      u = make_float2(fmaxf(ph[s], 0.0f), 0.0f);   // the starting amplitude, constrained
    } else if (a.slm.lvl_tab) {
      level = quant_phase(ph[s], a.slm.levels, a.slm.inv_delta_f64);
      u = a.slm.lvl_tab[level];
    } else {
      float sn, cs;
      sincosf(ph[s], &sn, &cs);
      u = make_float2(cs, sn);
    }
    if (out) write_state(a, row + x, u, level);
    float2 h = a.illum ? cscale(u, ldg(a.illum, row + x)) : u;
    if (a.q1y) h = cmul(h, cmul(qy, qx.at(s, x)));
    v[s] = h;
  });
  tw.template run<false, -1, C::WAVE_SYNC>(v, t, lds);
  const RowField f = RowField::make<N, RowTeam<C>::FT>(t, rt.y, a.H, a.ft);
  if (rt.live) for_layout<L1>(t, [&](int s, int x) { stg_field<N>(a.field, f.at(x), v[s]); });
}

// exp(i o pi / 4) for an octant index o in [0, 8), from the index bits: the
// odd octants start from (1 + i)/sqrt(2), bit 1 turns by pi/2, bit 2 by pi.
__device__ __forceinline__ float2 octant_value(int o) {
  const bool odd = o & 1, quarter = o & 2, half = o & 4;
  const float bx = odd ? HG_SQRT1_2 : 1.0f, by = odd ? HG_SQRT1_2 : 0.0f;
  const float x = quarter ? -by : bx, y = quarter ? bx : by;
  return half ? make_float2(-x, -y) : make_float2(x, y);
}

template <int MODE>
__device__ __forceinline__ float2 slm_constrain(float2 g, const SlmConstraint& slm, int& level) {
  if constexpr (MODE == GS_CONT) {
    level = 0;
    return unit_of(g);
  } else if constexpr (MODE == GS_AMP) {
    // amplitude-only SLM: the nearest non-negative real value
    level = 0;
    return make_float2(fmaxf(g.x, 0.0f), 0.0f);
  } else if constexpr (MODE == GS_QATAN) {
    level = quant_level(g, slm);
    return slm.lvl_tab[level];
  } else {
    // L in {2, 4, 8}: octant of G exp(i pi / L); octant o <-> level o / (8 / L)
    const float2 r = cmul(g, slm.half_step);
    const int o = octant(r.x, r.y);
    constexpr int SHIFT = MODE == GS_Q8 ? 0 : (MODE == GS_Q4 ? 1 : 2);
    const bool zero = (g.x == 0.0f) & (g.y == 0.0f);
    level = zero ? 0 : (o >> SHIFT);
    return octant_value(level << SHIFT);
  }
}

// Runtime-selected constraint for the general row pass.
__device__ __forceinline__ float2 slm_constrain_rt(float2 g, const SlmConstraint& slm, int& level) {
  if (slm.amplitude) return slm_constrain<GS_AMP>(g, slm, level);
  if (!slm.lvl_tab) return slm_constrain<GS_CONT>(g, slm, level);
  if (slm.levels == 8) return slm_constrain<GS_Q8>(g, slm, level);
  if (slm.levels == 4) return slm_constrain<GS_Q4>(g, slm, level);
  if (slm.levels == 2) return slm_constrain<GS_Q2>(g, slm, level);
  return slm_constrain<GS_QATAN>(g, slm, level);
}

// Row pass of a GS iteration: inverse row FFT -> conj(Q1) -> constraint -> Q1
// -> row FFT.  The inverse runs the radices in reversed order so that its
// last-stage register layout is the first-stage layout of the forward
// transform.  MODE >= 0 with FRES fixed is the steady-state kernel (no
// illumination, no outputs); MODE < 0 takes the mode, the Fresnel flag, the
// illumination and the output arrays at run time (the pass that produces the
// returned state, and illuminated runs).  MP (MODE >= 0): the steady-state
// step of multi-plane GS, whose field leaves through the next plane's chirp
// (qoy, qox; null for a Fourier plane) and arrives through this plane's (q1y,
// q1x; null likewise), both tables loaded with the field.
template <int N, int MODE, bool FRES, bool MP = false>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_gs_row(GsRowArgs a) {
  a.select_item();
  using C = RowCfg<N>;
  using P = typename C::P;
  using LL = RowLds<N>;
  using LI = Layout<P, true, false>;   // first stage of the reversed (inverse) run
  using LF = Layout<P, false, false>;  // == last stage of the reversed run
  using L1 = Layout<P, false, true>;
  static_assert(LF::R == Layout<P, true, true>::R, "layout mismatch");
  constexpr bool GENERAL = MODE < 0;
  const RowTeam<C> rt(a.H, a.ft);
  const int t = rt.t;
  LdsView<1> lds{hg_dyn_lds + rt.team * LL::TEAM};
  float2 v[P::REGS];
  const uint32_t row = (uint32_t)rt.y * N;
  const bool fres = (GENERAL || MP) ? (a.q1y != nullptr) : FRES;
  const RowField f = RowField::make<N, RowTeam<C>::FT>(t, rt.y, a.H, a.ft);
  for_layout<LI>(t, [&](int s, int x) { v[s] = ldg_field<N>(a.field, f.at(x)); });
  // general pass: the illumination and an outgoing chirp are loaded with the
  // field, not where they are used after the transform
  float ill[GENERAL ? P::REGS : 1];
  if constexpr (GENERAL) {
    if (a.illum) for_layout<LF>(t, [&](int s, int x) { ill[s] = ldg(a.illum, row + x); });
  }
  issue_loads_here();
  // the general and multi-plane passes hold more registers: twiddles in
  // registers only where they are few
  using TW = PassTwiddles<P, C::THREADS, true, true, !GENERAL && !MP>;
  using QX = RowTable<N, LF>;
  using QO = RowTableDirect<N, LF>;
  TW tw;
  QX qx;
  QO qo;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  if (fres) qx.begin(a.q1x, t);
  if constexpr (MP) {
    if (a.qoy) qo.begin(a.qox, t);
  } else if constexpr (GENERAL) {
    if (a.q_out_set && a.qoy) qo.begin(a.qox, t);
  }
  // this row's chirp values load with the tables, not after the transform,
  // whose barriers would hold them back until the pointwise step needs them
  const float2 qy = fres ? a.q1y[rt.y] : make_float2(1.f, 0.f);
  const float2 qoy_row = ((MP || GENERAL) && a.qoy) ? a.qoy[rt.y] : make_float2(1.f, 0.f);
  if constexpr (TW::USES_LDS || QX::USES_LDS) __syncthreads();
  tw.template run<true, +1, C::WAVE_SYNC>(v, t, lds);
  if constexpr (MP) {
    const bool fres_out = a.qoy != nullptr;
    const float2 qoy = qoy_row;
    for_layout<LF>(t, [&](int s, int x) {
      float2 g = v[s];
      if (fres) g = cmulconj(g, cmul(qy, qx.at(s, x)));
      int level;
      const float2 u = slm_constrain<MODE>(g, a.slm, level);
      v[s] = fres_out ? cmul(u, cmul(qoy, qo.at(s, x))) : u;
    });
  } else if constexpr (!GENERAL) {
    for_layout<LF>(t, [&](int s, int x) {
      float2 g = v[s];
      float2 q;
      if constexpr (FRES) {
        q = cmul(qy, qx.at(s, x));
        g = cmulconj(g, q);
      }
      int level;
      float2 u = slm_constrain<MODE>(g, a.slm, level);
      if constexpr (FRES) u = cmul(u, q);
      v[s] = u;
    });
  } else {
    const bool out = rt.live && (a.phase_out || a.levels_out);
    const bool fres_out = a.q_out_set ? (a.qoy != nullptr) : fres;
    const float2 qoy = a.q_out_set ? qoy_row : qy;
    for_layout<LF>(t, [&](int s, int x) {
      float2 g = v[s];
      float2 q = make_float2(1.f, 0.f);
      if (fres) {
        q = cmul(qy, qx.at(s, x));
        g = cmulconj(g, q);
      }
      int level;
      float2 u = slm_constrain_rt(g, a.slm, level);
      if (out) write_state(a, row + x, u, level, a.slm.amp_scale);
      if (a.illum) u = cscale(u, ill[s]);
      if (a.q_out_set && fres_out) q = cmul(qoy, qo.at(s, x));
      v[s] = fres_out ? cmul(u, q) : u;
    });
  }
  tw.template run<false, -1, C::WAVE_SYNC>(v, t, lds);
  if (rt.live) for_layout<L1>(t, [&](int s, int x) { stg_field<N>(a.field, f.at(x), v[s]); });
}

struct GsColArgs {
  float2* field;
  int W;
  int H;
  const float* target;        // target amplitude in FFT order, tiled [tile][ky][C] (k_tile_target)
  const Scalars* sc;
  float* partials;            // one float per workgroup for this state; null -> no NMSE
  const float2* tw;
  const float2* twr;
  // signal window (k_gs_col<N, MODE, true>): per state the three sums
  // [3][workgroups] of the windowed error (see k_gs_col)
  double* wpartials;
  // batch strides of item blockIdx.y: field elements (tiled layout),
  // tiled-target floats, Scalars, partial floats
  uint32_t px, target_stride, sc_stride, partial_stride;
  int ft;                     // field layout (ColField)
  // (offsets in 64 bits: a batch of multi-plane problems can span more than
  // 2^32 target and partial-sum floats while its fields stay below that)
  __device__ __forceinline__ void select_item() {
    const size_t b = blockIdx.y;
    field += b * px;
    target += b * target_stride;
    sc += b * sc_stride;
    if (partials) partials += b * partial_stride;
  }
};

// Replay-plane pass of one state.  Column FFT -> R (the forward FFT2 of the
// SLM field completes here); NMSE partial sum(d^2), d = a |R|^2 - b T^2; then
//   COL_NMSE:    nothing more (last state of a call: no write-back);
//   COL_REPLACE: R' = T R / |R| (Gerchberg-Saxton amplitude replacement);
//   COL_GRAD:    R' = dL/dconj(R) = g d R (Wirtinger derivative of the NMSE);
// -> inverse column FFT (unscaled: with the inverse row FFT of the next pass
// it is the adjoint F^H of the forward FFT2) -> field.
// WIN (COL_NMSE, COL_REPLACE): a signal window, marked by negative values of
// the tiled target (k_tile_target).  Inside, R' = c T R / |R| with the target
// scale c; outside, R is kept.  The error is measured inside only, where sum I
// is not known in advance, so each workgroup writes three sums instead of one,
// with x = a |R|^2 and y = b T^2 (b from the window's sum T^2):
// sum x, sum x^2 and sum x y, in FP64 (k_window_nmse_reduce combines them).
//
// The error sums are per column (column_sum: an order independent of C), at
// partials[column] (window: wpartials[j][column], j < 3), so that the single
// (WIDE = false) and batched (WIDE = true) column configurations give bitwise
// the same values.
enum { COL_NMSE = 0, COL_REPLACE = 1, COL_GRAD = 2 };
template <int N, int MODE, bool WIN = false, bool WIDE = false>
__global__ __launch_bounds__((ColCfgSel<N, WIDE>::THREADS)) void k_gs_col(GsColArgs a) {
  static_assert(!WIN || MODE != COL_GRAD, "no signal window in the gradient pass");
  a.select_item();
  using C = ColCfgSel<N, WIDE>;
  using P = typename C::P;
  using LL = ColLdsOf<C>;
  using L0 = Layout<P, false, false>;
  using L1 = Layout<P, false, true>;
  using LB = Layout<P, true, true>;
  static_assert(LB::R == L0::R, "layout mismatch");
  constexpr bool BACK = MODE != COL_NMSE;
  const int c = threadIdx.x % C::C, t = threadIdx.x / C::C;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int col = tile * C::C + c;
  const bool live = col < a.W;
  const uint32_t x = live ? col : a.W - 1;
  LdsView<C::C> lds{hg_dyn_lds + c};
  float2 v[P::REGS];
  const ColField f(x, a.W, N, a.ft);
  for_layout<L0>(t, [&](int s, int y) { v[s] = ldg_field<N>(a.field, f.at(y)); });
  float tgt[P::REGS];
  const uint32_t tbase = (uint32_t)tile * N * C::C + c;
  for_layout<L1>(t, [&](int s, int ky) { tgt[s] = ldg(a.target, tbase + (uint32_t)ky * C::C); });
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, true, BACK>;
  TW tw;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  // the error scalars are read here, not after the transform, so that their
  // load does not wait behind its barriers
  const bool nm = WIN ? (a.wpartials != nullptr) : (a.partials != nullptr);
  const bool scaled = nm || MODE == COL_GRAD;
  const float sa = scaled ? a.sc->a : 0.f;
  const float sb = scaled ? a.sc->b : 0.f;
  const float sg = MODE == COL_GRAD ? a.sc->g : 0.f;
  const float sc_win = WIN ? a.sc->c : 0.f;
  if constexpr (TW::USES_LDS) __syncthreads();
  tw.template run<false, -1, C::WAVE_SYNC>(v, t, lds);
  float acc = 0.f;
  double w1 = 0.0, w2 = 0.0, w3 = 0.0;
  if constexpr (WIN) {
    const float sc = sc_win;
    for_layout<L1>(t, [&](int s, int) {
      const float2 R = v[s];
      const float tv = tgt[s];
      if (tv >= 0.0f) {
        const float I = cnorm(R);
        const double x = (double)(I * sa), y = (double)(tv * tv * sb);
        w1 += x;
        w2 = fma(x, x, w2);
        w3 = fma(x, y, w3);
        if constexpr (MODE == COL_REPLACE) {
          const float ct = tv * sc;
          const float k = ct * rsqrtf(I);
          v[s] = I > 0.0f ? make_float2(R.x * k, R.y * k) : make_float2(ct, 0.0f);
        }
      }
    });
  } else {
    for_layout<L1>(t, [&](int s, int) {
      const float2 R = v[s];
      const float tv = tgt[s];
      const float I = cnorm(R);
      const float d = fmaf(I, sa, -(tv * tv * sb));
      acc = fmaf(d, d, acc);
      if constexpr (MODE == COL_REPLACE) {
        const float k = tv * rsqrtf(I);
        v[s] = I > 0.0f ? make_float2(R.x * k, R.y * k) : make_float2(tv, 0.0f);
      } else if constexpr (MODE == COL_GRAD) {
        const float k = sg * d;
        v[s] = make_float2(R.x * k, R.y * k);
      }
    });
  }
  if constexpr (BACK) {
    tw.template run<true, +1, C::WAVE_SYNC>(v, t, lds);
    if (live) for_layout<LB>(t, [&](int s, int y) { stg_field<N>(a.field, f.at(y), v[s]); });
  }
  // The error's column sums run last, while the field stores drain: the
  // replaced values do not depend on them, and their barrier and shuffles
  // would otherwise sit between the two transforms.
  const uint32_t slot = (uint32_t)tile * C::C + c;   // the column's partial
  if constexpr (WIN) {
    if (nm) {
      __shared__ double wred[C::C * ColSum<N>::BLOCKS];
      if (!live) w1 = w2 = w3 = 0.0;
      w1 = column_sum_f64<N, C>(w1, c, t, wred);
      w2 = column_sum_f64<N, C>(w2, c, t, wred);
      w3 = column_sum_f64<N, C>(w3, c, t, wred);
      if (t == 0) {
        const uint32_t slots = gridDim.x * C::C;
        a.wpartials[slot] = w1;
        a.wpartials[slots + slot] = w2;
        a.wpartials[2 * slots + slot] = w3;
      }
    }
  } else if (nm) {
    __shared__ float red[C::C * ColSum<N>::BLOCKS];
    const float s = column_sum<N, C>(live ? acc : 0.0f, c, t, red);
    if (t == 0) a.partials[slot] = s;
  }
}

// ===========================================================================
// Gradient-descent hologram optimisation: adjoint row pass
// ===========================================================================
// Row passes of the gradient method: every plane of one state in one pass, the
// sum over planes in registers (problem blockIdx.y of a batch).
constexpr int GRAD_MAX_PLANES = 16;
enum { GRAD_START = 0, GRAD_ADJ = 1, GRAD_ADJ_NEXT = 2 };
struct GradRowArgs {
  float2* field;           // [planes] fields of the problem, fpx elements apart:
                           // in (ADJ): outputs of the COL_GRAD passes;
                           // out (START, ADJ_NEXT): forward row passes of the next state
  int ft;                  // their layout (RowField)
  float* phase;            // SLM phase phi [H][W]; updated in place by the Adam step
  int H;
  int planes;
  const float2* q1y[GRAD_MAX_PLANES];   // source chirp of each plane; null -> Fourier plane
  const float2* q1x[GRAD_MAX_PLANES];
  float* grad_out;         // dL/dphi; may be null
  float* m;                // Adam moments [H][W]; null -> no update
  float* v;
  float lr, beta1, beta2, eps;
  float bc1, bc2;          // 1 - beta1^t, 1 - beta2^t
  const float2* tw;
  const float2* twr;
  uint32_t px;             // batch: pixels per problem (row-order arrays)
  uint32_t fpx;            // field elements per plane
};
// The arrays of problem blockIdx.y of a launch over a batch of same-shape
// problems.  (Kept apart from the arguments: the per-plane chirp pointers
// are indexed at run time and must stay in the kernel-argument segment.)
struct GradItem {
  float2* field;
  float *phase, *grad_out, *m, *v;
  __device__ __forceinline__ explicit GradItem(const GradRowArgs& a) {
    const size_t off = (size_t)blockIdx.y * a.px;
    field = a.field + (size_t)blockIdx.y * a.planes * a.fpx;
    phase = a.phase + off;
    grad_out = a.grad_out ? a.grad_out + off : nullptr;
    m = a.m ? a.m + off : nullptr;
    v = a.v ? a.v + off : nullptr;
  }
};

// ADJ: for each plane j, inverse row FFT (completes G_j = F^H dL/dconj(U_j))
// -> V_j = Q1_j exp(i phi) recomputed from phi rather than stored -> g +=
// 2 Im(conj(V_j) G_j), planes in order; then the gradient is written out
// and/or one Adam step updates phi.  The phase is loaded with the first
// plane's field and exp(i phi) formed once for all planes; the moments are
// loaded after the last plane's transform.
// START, and ADJ_NEXT after the above: the forward evaluation of every plane
// from the phase held (updated by Adam, or as it was): Q1_j exp(i phi) -> row
// FFT -> field j (the arithmetic of k_gs_row_start on a continuous phase).
// A state thus costs one row pass and one column launch over all planes.
template <int N, int MODE>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_grad_rows(GradRowArgs a) {
  const GradItem it(a);
  using C = RowCfg<N>;
  using P = typename C::P;
  using LL = RowLds<N>;
  using LI = Layout<P, true, false>;   // first stage of the reversed (inverse) run
  using LF = Layout<P, false, false>;  // its last stage == first of the forward run
  using L1 = Layout<P, false, true>;   // last stage of the forward run
  constexpr bool ADJ = MODE != GRAD_START;
  constexpr bool FWD = MODE != GRAD_ADJ;
  const RowTeam<C> rt(a.H, a.ft);
  const int t = rt.t;
  const bool live = rt.live;
  LdsView<1> lds{hg_dyn_lds + rt.team * LL::TEAM};
  float2 v[P::REGS];
  const uint32_t row = (uint32_t)rt.y * N;
  const RowField f = RowField::make<N, RowTeam<C>::FT>(t, rt.y, a.H, a.ft);
  if constexpr (ADJ) for_layout<LI>(t, [&](int s, int x) { v[s] = ldg_field<N>(it.field, f.at(x)); });
  float ph[P::REGS], g[ADJ ? P::REGS : 1], mm[ADJ ? P::REGS : 1], vv[ADJ ? P::REGS : 1];
  const bool adam = ADJ && it.m != nullptr;
  for_layout<LF>(t, [&](int s, int x) { ph[s] = ldg_f<N>(it.phase, row + x); });
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, FWD, ADJ, false>;
  // Each plane's chirp row table: loaded into registers before the plane's
  // transform where a thread holds at most 8 values, below 1024 threads
  // (1024-point rows, 3-plane batch: 27.0 ms per 100 steps against 28.7 read
  // at the point of use); elsewhere read where it is used (from L2), since
  // 2 REGS more live registers through the plane loops spill there.
  using QT = std::conditional_t<(P::REGS <= 8 && C::THREADS < 1024), RowTableDirect<N, LF>, RowTableGlobal>;
  TW tw;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  if constexpr (TW::USES_LDS) __syncthreads();
  float2 e[P::REGS];   // exp(i phi), formed once for every plane
  for_layout<LF>(t, [&](int s, int) {
    float sn, cs;
    sincosf(ph[s], &sn, &cs);
    e[s] = make_float2(cs, sn);
  });
  if constexpr (ADJ) {
#pragma unroll
    for (int s = 0; s < P::REGS; ++s) g[s] = 0.0f;
#pragma unroll 1
    for (int j = 0; j < a.planes; ++j) {
      const float2* qy_j = a.q1y[j];
      QT qx;
      if (qy_j) qx.begin(a.q1x[j], t);
      const float2 qy = qy_j ? qy_j[rt.y] : make_float2(1.f, 0.f);
      tw.template run<true, +1, C::WAVE_SYNC>(v, t, lds);
      for_layout<LF>(t, [&](int s, int x) {
        float2 V = e[s];
        if (qy_j) V = cmul(V, cmul(qy, qx.at(s, x)));
        const float2 G = v[s];
        g[s] = fmaf(2.0f, fmaf(V.x, G.y, -(V.y * G.x)), g[s]);
      });
      if (j + 1 < a.planes) {
        const float2* fj = it.field + (size_t)(j + 1) * a.fpx;
        for_layout<LI>(t, [&](int s, int x) { v[s] = ldg_field<N>(fj, f.at(x)); });
      }
    }
    // the moments are needed only now (loaded earlier, they would hold
    // registers through every plane's transform)
    if (adam)
      for_layout<LF>(t, [&](int s, int x) {
        mm[s] = ldg_f<N>(it.m, row + x);
        vv[s] = ldg_f<N>(it.v, row + x);
      });
    for_layout<LF>(t, [&](int s, int x) {
      const uint32_t i = row + x;
      if (it.grad_out && live) stg_f<N>(it.grad_out, i, g[s]);
      if (adam) {
        const float m1 = fmaf(a.beta1, mm[s], (1.0f - a.beta1) * g[s]);
        const float v1 = fmaf(a.beta2, vv[s], (1.0f - a.beta2) * g[s] * g[s]);
        const float phn = ph[s] - a.lr * (m1 / a.bc1) / (sqrtf(v1 / a.bc2) + a.eps);
        if (live) {
          stg_f<N>(it.m, i, m1);
          stg_f<N>(it.v, i, v1);
          stg_f<N>(it.phase, i, phn);
        }
        if constexpr (FWD) {
          float sn, cs;
          sincosf(phn, &sn, &cs);
          e[s] = make_float2(cs, sn);
        }
      }
    });
  }
  if constexpr (FWD) {
#pragma unroll 1
    for (int j = 0; j < a.planes; ++j) {
      const float2* qy_j = a.q1y[j];
      QT qx;
      if (qy_j) qx.begin(a.q1x[j], t);
      const float2 qy = qy_j ? qy_j[rt.y] : make_float2(1.f, 0.f);
      for_layout<LF>(t, [&](int s, int x) {
        float2 h = e[s];
        if (qy_j) h = cmul(h, cmul(qy, qx.at(s, x)));
        v[s] = h;
      });
      tw.template run<false, -1, C::WAVE_SYNC>(v, t, lds);
      float2* fj = it.field + (size_t)j * a.fpx;
      if (live) for_layout<L1>(t, [&](int s, int x) { stg_field<N>(fj, f.at(x), v[s]); });
    }
  }
}

// ===========================================================================
// Angular-spectrum propagation: T(ky, kx) = exp(2 pi i z sqrt(1/lambda^2 - s)),
// s = fx^2 + fy^2, on the SLM's own grid (no evanescent components: the plan
// requires pitch > lambda / sqrt 2).  The phase, up to 2 pi z / lambda, is far
// beyond FP32; it is split as
//   k z - pi lambda z fy^2 - pi lambda z fx^2 - delta,
//   delta = pi lambda^3 z s^2 / (1 + r)^2,  r = sqrt(1 - lambda^2 s),
// where the first three are FP64-built per-axis tables (exp(i k z) folded
// into the row table) and delta, at most a few radians, is evaluated in FP32
// from s without cancellation.
// ===========================================================================
struct AsTransfer {
  const float2* ty;   // exp(i k z) exp(-i pi lambda z fy^2), FFT order [H]
  const float2* tx;   // exp(-i pi lambda z fx^2), FFT order [W]
  float lam2;         // lambda^2
  float c3;           // pi lambda^3 z
  float inv_hp, inv_wp;  // 1 / (H p), 1 / (W p)
  int H, W;
  // transfer at FFT indices (ky, kx); conjugate when CONJ
  template <bool CONJ>
  __device__ __forceinline__ float2 at(int ky, int kx) const {
    const float fy = (float)(ky < (H + 1) / 2 ? ky : ky - H) * inv_hp;
    const float fx = (float)(kx < (W + 1) / 2 ? kx : kx - W) * inv_wp;
    const float sq = fmaf(fy, fy, fx * fx);
    const float r = sqrtf(fmaf(-lam2, sq, 1.0f));
    const float onep = 1.0f + r;
    const float delta = c3 * sq * sq / (onep * onep);
    float sn, cs;
    sincosf(delta, &sn, &cs);
    const float2 t = cmul(cmul(ty[ky], tx[kx]), make_float2(cs, -sn));
    return CONJ ? make_float2(t.x, -t.y) : t;
  }
};

struct AsColArgs {
  float2* io;          // row-transformed field; the column pass finishes the transfer
  int W;
  int ft;              // field layout (ColField): 0 for propagation
  AsTransfer tr;
  float scale;         // applied on store (1 / (H W) for hg_propagate, 1 in the GS loop)
  const float2* tw;
  const float2* twr;
};

// Column FFT -> * T (or conj T, DIR = -1) -> inverse column FFT.
template <int N, int DIR>
__global__ __launch_bounds__(ColCfg<N>::THREADS) void k_as_col(AsColArgs a) {
  using C = ColCfg<N>;
  using P = typename C::P;
  using LL = ColLds<N>;
  using L0 = Layout<P, false, false>;
  using L1 = Layout<P, false, true>;
  using LB = Layout<P, true, true>;
  const int c = threadIdx.x % C::C, t = threadIdx.x / C::C;
  const int col = xcd_tile(blockIdx.x, gridDim.x) * C::C + c;
  const bool live = col < a.W;
  const uint32_t x = live ? col : a.W - 1;
  LdsView<C::C> lds{hg_dyn_lds + c};
  float2 v[P::REGS];
  const ColField f(x, a.W, N, a.ft);
  for_layout<L0>(t, [&](int s, int y) { v[s] = ldg_field<N>(a.io, f.at(y)); });
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, true, true>;
  TW tw;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  if constexpr (TW::USES_LDS) __syncthreads();
  tw.template run<false, -1, C::WAVE_SYNC>(v, t, lds);
  for_layout<L1>(t, [&](int s, int ky) { v[s] = cmul(v[s], a.tr.template at<(DIR < 0)>(ky, (int)x)); });
  tw.template run<true, +1, C::WAVE_SYNC>(v, t, lds);
  if (live) for_layout<LB>(t, [&](int s, int y) { stg_field<N>(a.io, f.at(y), cscale(v[s], a.scale)); });
}

struct AsRowArgs {
  float2* field;
  int H;
  int ft;                // field layout (RowField)
  const float* target;   // target amplitude [H][W], centred = natural order on this grid
  const Scalars* sc;
  float* partials;       // one float per workgroup; null -> no NMSE
  const float2* tw;
  const float2* twr;
};

// Replay pass of GS on the angular-spectrum model: inverse row FFT (R on the
// SLM grid) -> NMSE partial -> REPLACE: T R / |R| -> row FFT -> field.
template <int N, bool REPLACE>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_as_row(AsRowArgs a) {
  using C = RowCfg<N>;
  using P = typename C::P;
  using LL = RowLds<N>;
  using LI = Layout<P, true, false>;
  using LF = Layout<P, false, false>;
  using L1 = Layout<P, false, true>;
  __shared__ float red[C::THREADS / 64];
  const RowTeam<C> rt(a.H, a.ft);
  const int t = rt.t;
  LdsView<1> lds{hg_dyn_lds + rt.team * LL::TEAM};
  float2 v[P::REGS];
  const uint32_t row = (uint32_t)rt.y * N;
  const RowField f = RowField::make<N, RowTeam<C>::FT>(t, rt.y, a.H, a.ft);
  for_layout<LI>(t, [&](int s, int x) { v[s] = ldg_field<N>(a.field, f.at(x)); });
  float tg[P::REGS];
  for_layout<LF>(t, [&](int s, int x) { tg[s] = ldg(a.target, row + x); });
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, true, true>;
  TW tw;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  if constexpr (TW::USES_LDS) __syncthreads();
  tw.template run<true, +1, C::WAVE_SYNC>(v, t, lds);
  const bool nm = a.partials != nullptr;
  const float sa = nm ? a.sc->a : 0.f, sb = nm ? a.sc->b : 0.f;
  float acc = 0.f;
  for_layout<LF>(t, [&](int s, int) {
    const float2 R = v[s];
    const float tv = tg[s];
    const float I = cnorm(R);
    const float d = fmaf(I, sa, -(tv * tv * sb));
    acc = fmaf(d, d, acc);
    if constexpr (REPLACE) {
      const float k = tv * rsqrtf(I);
      v[s] = I > 0.0f ? make_float2(R.x * k, R.y * k) : make_float2(tv, 0.0f);
    }
  });
  if (nm) {
    const float sum = block_sum<C::THREADS>(rt.live ? acc : 0.0f, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = sum;
  }
  if constexpr (REPLACE) {
    tw.template run<false, -1, C::WAVE_SYNC>(v, t, lds);
    if (rt.live) for_layout<L1>(t, [&](int s, int x) { stg_field<N>(a.field, f.at(x), v[s]); });
  }
}

// ===========================================================================
// OSPR
// ===========================================================================
struct OsprRowArgs {
  float2* field;
  int H;
  int ft;                  // field layout between the passes (RowField)
  const float* target;     // centred amplitude [H][W]
  const float* theta;      // centred subframe phase [H][W] (pass A)
  const float* theta_next; // pass C with NEXT: the next subframe's phase (its pass A)
  float* intensity;        // centred accumulator / output [H][W] (pass C)
  int first, last;
  float inv_nsub;
  const Scalars* sc;
  float* partials;         // pass C of the last subframe: NMSE partials
  const float2* tw;
  const float2* twr;
};

// Pass A: E = T exp(i theta) read through ifftshift -> inverse row FFT.
template <int N>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_ospr_a(OsprRowArgs a) {
  using C = RowCfg<N>;
  using P = typename C::P;
  using LL = RowLds<N>;
  using L0 = Layout<P, false, false>;
  using L1 = Layout<P, false, true>;
  const RowTeam<C> rt(a.H, a.ft);
  const int t = rt.t;
  LdsView<1> lds{hg_dyn_lds + rt.team * LL::TEAM};
  float2 v[P::REGS];
  const uint32_t srow = (uint32_t)wrap_add_rt(rt.y, a.H / 2, a.H) * N;
  float th[P::REGS], am[P::REGS];
  for_layout<L0>(t, [&](int s, int x) {
    const uint32_t i = srow + wrap_add<N>(x, N / 2);
    th[s] = ldg(a.theta, i);
    am[s] = ldg(a.target, i);
  });
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, true, false>;
  TW tw;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  if constexpr (TW::USES_LDS) __syncthreads();
  for_layout<L0>(t, [&](int s, int) {
    float sn, cs;
    sincosf(th[s], &sn, &cs);
    v[s] = make_float2(am[s] * cs, am[s] * sn);
  });
  tw.template run<false, +1, C::WAVE_SYNC>(v, t, lds);
  const RowField f = RowField::make<N, RowTeam<C>::FT>(t, rt.y, a.H, a.ft);
  if (rt.live) for_layout<L1>(t, [&](int s, int x) { stg(a.field, f.at(x), v[s]); });
}

struct OsprColArgs {
  float2* field;
  int W;
  int ft;              // field layout between the passes (ColField)
  uint8_t* levels;     // [H][W] of this subframe, natural SLM order; may be null
  uint8_t* levels_im;  // pairs: [H][W] of the subframe binarised from Im G; may be null
  const float2* tw;
  const float2* twr;
};

// Pass B: inverse column FFT -> h = sign(Re G) -> level -> forward column FFT of h.
// The hologram is real, so its column transform is conjugate-symmetric,
// Z[H-y] = conj Z[y]: only the rows y <= H/2 are stored (pass C's row pairs
// take the rest from them).
// PAIR: two subframes from one G, h_re = sign(Re G) and h_im = sign(Im G), and
// the column FFT of the complex field h_re + i h_im carries both (pass C and
// k_ospr_pair_finish separate their intensities); all rows are stored.
template <int N, bool PAIR>
__global__ __launch_bounds__(ColCfgOspr<N>::THREADS) void k_ospr_b(OsprColArgs a) {
  using C = ColCfgOspr<N>;
  using P = typename C::P;
  using LL = ColLdsOf<C>;
  using LI = Layout<P, true, false>;
  using LF = Layout<P, false, false>;
  using L2 = Layout<P, false, true>;
  const int c = threadIdx.x % C::C, t = threadIdx.x / C::C;
  const int col = xcd_tile(blockIdx.x, gridDim.x) * C::C + c;
  const bool live = col < a.W;
  const uint32_t x = live ? col : a.W - 1;
  LdsView<C::C> lds{hg_dyn_lds + c};
  float2 v[P::REGS];
  const ColField f(x, a.W, N, a.ft);
  for_layout<LI>(t, [&](int s, int y) { v[s] = ldg(a.field, f.at(y)); });
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, true, true>;
  TW tw;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  if constexpr (TW::USES_LDS) __syncthreads();
  tw.template run<true, +1, C::WAVE_SYNC>(v, t, lds);
  const bool wl = live && a.levels;
  const bool wl_im = PAIR && live && a.levels_im;
  for_layout<LF>(t, [&](int s, int y) {
    const bool neg = !(v[s].x >= 0.0f);
    if (wl) stg(a.levels, (uint32_t)y * a.W + x, (uint8_t)(neg ? 1 : 0));
    float im = 0.0f;
    if constexpr (PAIR) {
      const bool neg_im = !(v[s].y >= 0.0f);
      if (wl_im) stg(a.levels_im, (uint32_t)y * a.W + x, (uint8_t)(neg_im ? 1 : 0));
      im = neg_im ? -1.0f : 1.0f;
    }
    v[s] = make_float2(neg ? -1.0f : 1.0f, im);
  });
  tw.template run<false, -1, C::WAVE_SYNC>(v, t, lds);
  if (live)
    for_layout<L2>(t, [&](int s, int y) {
      if (PAIR || y <= N / 2) stg(a.field, f.at(y), v[s]);
    });
}

// (N/2 - k) mod N: the centred position of frequency -k of an N-point row.
template <int NC>
__device__ __forceinline__ int centred_neg(int k) {
  const int j = NC / 2 - k;
  return j < 0 ? j + NC : j;
}

// Pass C: row FFT -> |.|^2 -> accumulate into the centred intensity (fftshift on
// store); the last subframe scales by 1/N_sub and adds the NMSE partials.
// NEXT: the same rows then run pass A of the next subframe (T exp(i theta_next)
// -> inverse row FFT -> field), so a subframe after the first costs two
// passes.  Its phase and the target are loaded after pass C's transform,
// while the intensity is accumulated (loaded with the field, they held
// registers through the transform: 4.5 % slower at 2048^2).
// HALF (a real hologram, whose pass B stored the rows y <= H/2): a team takes
// the row pair (y, H - y), y = 0..H/2.  Row H - y of the 2D transform is
// F[H-y][k] = conj F[y][-k], so one row transform gives both intensity rows,
// |F[H-y][k]|^2 = |F[y][-k]|^2 (centred: position (H - r, N - c) mod (H, N)
// mirrors (r, c)); with NEXT the team then runs pass A of both rows.  Rows 0
// and H/2 pair with themselves.  The running intensity is kept for row y
// only; the last subframe (not NEXT) writes the mirror row too.
template <int N, bool NEXT, bool HALF>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_ospr_c(OsprRowArgs a) {
  using C = RowCfg<N>;
  using P = typename C::P;
  using LL = RowLds<N>;
  using L0 = Layout<P, false, false>;
  using L1 = Layout<P, false, true>;
  __shared__ float red[C::THREADS / 64];
  const RowTeam<C> rt(HALF ? a.H / 2 + 1 : a.H, a.ft);
  const int t = rt.t;
  // the mirror row (HALF), and whether it is another row than y
  const int ym = HALF && rt.y != 0 ? a.H - rt.y : rt.y;
  const bool two = HALF && ym != rt.y;
  constexpr int RM = HALF ? P::REGS : 1;
  LdsView<1> lds{hg_dyn_lds + rt.team * LL::TEAM};
  float2 v[P::REGS];
  const RowField f = RowField::make<N, RowTeam<C>::FT>(t, rt.y, a.H, a.ft);
  for_layout<L0>(t, [&](int s, int x) { v[s] = ldg(a.field, f.at(x)); });
  const uint32_t orow = (uint32_t)wrap_add_rt(rt.y, a.H / 2, a.H) * N;
  const uint32_t orow_m = (uint32_t)wrap_add_rt(ym, a.H / 2, a.H) * N;
  const bool nm = !NEXT && a.last && a.partials;
  // The mirror row's loads are issued with row y's where registers allow
  // (at most 8 values per thread, below 1024 threads); elsewhere after the
  // transform that needs them.  The mirror row's running intensity is never
  // read: it equals row y's bitwise (the same additions in the same order
  // from zero), so only the last subframe writes it, from row y's.
  constexpr bool EARLY_M = C::THREADS < 1024 && P::REGS <= 8;
  float prev[P::REGS], tg[P::REGS], tg_m[RM];
  auto load_acc_mirror = [&]() {
    for_layout<L1>(t, [&](int s, int k) {
      tg_m[s] = nm && two ? ldg(a.target, orow_m + centred_neg<N>(k)) : 0.0f;
    });
  };
  for_layout<L1>(t, [&](int s, int k) {
    const uint32_t i = orow + wrap_add<N>(k, N / 2);
    prev[s] = a.first ? 0.0f : ldg(a.intensity, i);
    tg[s] = nm ? ldg(a.target, i) : 0.0f;
  });
  if constexpr (HALF && !NEXT && EARLY_M) load_acc_mirror();
  issue_loads_here();
  using TW = PassTwiddles<P, C::THREADS, true, false, !NEXT>;
  TW tw;
  tw.begin(a.tw, a.twr, hg_dyn_lds + LL::TWF, t);
  if constexpr (TW::USES_LDS) __syncthreads();
  tw.template run<false, -1, C::WAVE_SYNC>(v, t, lds);
  if constexpr (HALF && !NEXT && !EARLY_M) load_acc_mirror();
  float th[NEXT ? P::REGS : 1], am[NEXT ? P::REGS : 1];
  float th_m[NEXT ? RM : 1], am_m[NEXT ? RM : 1];
  auto load_mirror = [&]() {
    for_layout<L0>(t, [&](int s, int x) {
      const uint32_t im = orow_m + wrap_add<N>(x, N / 2);
      th_m[s] = ldg(a.theta_next, im);
      am_m[s] = ldg(a.target, im);
    });
  };
  if constexpr (NEXT) {
    for_layout<L0>(t, [&](int s, int x) {
      const uint32_t i = orow + wrap_add<N>(x, N / 2);
      th[s] = ldg(a.theta_next, i);
      am[s] = ldg(a.target, i);
    });
    if constexpr (HALF && EARLY_M) load_mirror();
  }
  float acc = 0.f;
  const float sa = nm ? a.sc->a : 0.f;
  const float sb = nm ? a.sc->b : 0.f;
  for_layout<L1>(t, [&](int s, int k) {
    const float e = cnorm(v[s]);
    float I = e + prev[s];
    if (!NEXT && a.last) {
      I *= a.inv_nsub;
      const float d = fmaf(I, sa, -(tg[s] * tg[s] * sb));
      acc = fmaf(d, d, acc);
    }
    if (rt.live) stg(a.intensity, orow + wrap_add<N>(k, N / 2), I);
    if constexpr (HALF && !NEXT) {
      if (a.last) {
        const float d = fmaf(I, sa, -(tg_m[s] * tg_m[s] * sb));
        if (two) acc = fmaf(d, d, acc);
      }
      if (rt.live && two) stg(a.intensity, orow_m + centred_neg<N>(k), I);
    }
  });
  if (a.partials) {
    const float s = block_sum<C::THREADS>(rt.live ? acc : 0.0f, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
  }
  if constexpr (NEXT) {
    for_layout<L0>(t, [&](int s, int) {
      float sn, cs;
      sincosf(th[s], &sn, &cs);
      v[s] = make_float2(am[s] * cs, am[s] * sn);
    });
    tw.template run<false, +1, C::WAVE_SYNC>(v, t, lds);
    if (rt.live) for_layout<L1>(t, [&](int s, int x) { stg(a.field, f.at(x), v[s]); });
    if constexpr (HALF) {
      // every team transforms (the exchanges' barriers span the workgroup);
      // only a distinct mirror row is stored
      if constexpr (!EARLY_M) load_mirror();
      for_layout<L0>(t, [&](int s, int) {
        float sn, cs;
        sincosf(th_m[s], &sn, &cs);
        v[s] = make_float2(am_m[s] * cs, am_m[s] * sn);
      });
      tw.template run<false, +1, C::WAVE_SYNC>(v, t, lds);
      const RowField fm = RowField::make<N, RowTeam<C>::FT>(t, ym, a.H, a.ft);
      if (rt.live && two) for_layout<L1>(t, [&](int s, int x) { stg(a.field, fm.at(x), v[s]); });
    }
  }
}

// ---------------------------------------------------------------------------
// per-length kernel table (one translation unit per length fills it in)
// ---------------------------------------------------------------------------
struct RowKernels {
  void (*prop_fwd)(PropRowArgs);
  void (*prop_inv)(PropRowArgs);
  void (*gs_start)(GsRowArgs);
  void (*gs_row[6][2])(GsRowArgs);   // steady state [gs_mode_index][Fresnel]
  void (*gs_row_general)(GsRowArgs); // outputs / illumination / any mode
  void (*gs_row_mp[5])(GsRowArgs);   // multi-plane steady state [gs_mode_index]
  void (*ospr_a)(OsprRowArgs);
  void (*ospr_c)(OsprRowArgs);
  void (*ospr_ca)(OsprRowArgs);   // pass C, then the next subframe's pass A
  void (*ospr_c_half)(OsprRowArgs);    // the same over row pairs (real holograms)
  void (*ospr_ca_half)(OsprRowArgs);
  void (*grad_rows[3])(GradRowArgs);   // [GRAD_START, GRAD_ADJ, GRAD_ADJ_NEXT]
  void (*as_row)(AsRowArgs);
  void (*as_row_nmse)(AsRowArgs);
  int teams, threads;
  size_t lds;
  int ft;          // RowTeam<RowCfg<N>>::FT
};
// The GS-family column passes of the batched configuration (ColCfgWide).
struct ColWideKernels {
  void (*gs_col)(GsColArgs);
  void (*gs_col_nmse)(GsColArgs);
  void (*grad_col)(GsColArgs);
  int cols, threads;     // cols = 0: the length has no batched configuration
  size_t lds;
};
struct ColKernels {
  void (*prop_fwd)(PropColArgs);
  void (*prop_inv)(PropColArgs);
  void (*gs_col)(GsColArgs);
  void (*gs_col_nmse)(GsColArgs);
  void (*gs_col_win)(GsColArgs);        // signal window
  void (*gs_col_win_nmse)(GsColArgs);
  void (*grad_col)(GsColArgs);
  void (*ospr_b)(OsprColArgs);
  void (*ospr_b_pair)(OsprColArgs);
  void (*as_fwd)(AsColArgs);
  void (*as_inv)(AsColArgs);
  int cols, threads;
  size_t lds;
  int ospr_cols, ospr_threads;   // OSPR's column pass (ColCfgOspr)
  size_t ospr_lds;
};
struct LengthEntry {
  int n;
  RowKernels row;
  ColKernels col;
  ColWideKernels col_wide;
  // twiddle images (FP64 values) for the row / column launch shapes, in
  // forward and reversed radix order; sizes in complex entries
  int row_tw_len[2], col_tw_len[2];
  void (*row_tw)(int rev, double* re, double* im);
  void (*col_tw)(int rev, double* re, double* im);
};

template <class P>
void twiddle_image_either(int rev, double* re, double* im) {
  if (rev) twiddle_image<P, true>(re, im);
  else twiddle_image<P, false>(re, im);
}

template <int N>
LengthEntry make_length_entry() {
  LengthEntry e;
  e.n = N;
  e.row.prop_fwd = k_prop_row<N, -1>;
  e.row.prop_inv = k_prop_row<N, +1>;
  e.row.gs_start = k_gs_row_start<N>;
  e.row.gs_row[5][0] = k_gs_row<N, GS_AMP, false>;
  e.row.gs_row[5][1] = k_gs_row<N, GS_AMP, true>;
  e.row.gs_row[0][0] = k_gs_row<N, GS_CONT, false>;
  e.row.gs_row[0][1] = k_gs_row<N, GS_CONT, true>;
  e.row.gs_row[1][0] = k_gs_row<N, GS_QATAN, false>;
  e.row.gs_row[1][1] = k_gs_row<N, GS_QATAN, true>;
  e.row.gs_row[2][0] = k_gs_row<N, GS_Q2, false>;
  e.row.gs_row[2][1] = k_gs_row<N, GS_Q2, true>;
  e.row.gs_row[3][0] = k_gs_row<N, GS_Q4, false>;
  e.row.gs_row[3][1] = k_gs_row<N, GS_Q4, true>;
  e.row.gs_row[4][0] = k_gs_row<N, GS_Q8, false>;
  e.row.gs_row[4][1] = k_gs_row<N, GS_Q8, true>;
  e.row.gs_row_general = k_gs_row<N, -1, false>;
  e.row.gs_row_mp[0] = k_gs_row<N, GS_CONT, false, true>;
  e.row.gs_row_mp[1] = k_gs_row<N, GS_QATAN, false, true>;
  e.row.gs_row_mp[2] = k_gs_row<N, GS_Q2, false, true>;
  e.row.gs_row_mp[3] = k_gs_row<N, GS_Q4, false, true>;
  e.row.gs_row_mp[4] = k_gs_row<N, GS_Q8, false, true>;
  e.row.ospr_a = k_ospr_a<N>;
  e.row.ospr_c = k_ospr_c<N, false, false>;
  e.row.ospr_ca = k_ospr_c<N, true, false>;
  e.row.ospr_c_half = k_ospr_c<N, false, true>;
  e.row.ospr_ca_half = k_ospr_c<N, true, true>;
  e.row.grad_rows[GRAD_START] = k_grad_rows<N, GRAD_START>;
  e.row.grad_rows[GRAD_ADJ] = k_grad_rows<N, GRAD_ADJ>;
  e.row.grad_rows[GRAD_ADJ_NEXT] = k_grad_rows<N, GRAD_ADJ_NEXT>;
  e.row.as_row = k_as_row<N, true>;
  e.row.as_row_nmse = k_as_row<N, false>;
  e.row.teams = RowCfg<N>::TEAMS;
  e.row.threads = RowCfg<N>::THREADS;
  e.row.lds = sizeof(float2) * RowLds<N>::WORDS;
  e.row.ft = RowTeam<RowCfg<N>>::FT;
  e.col = {k_prop_col<N, -1>, k_prop_col<N, +1>, k_gs_col<N, COL_REPLACE>, k_gs_col<N, COL_NMSE>,
           k_gs_col<N, COL_REPLACE, true>, k_gs_col<N, COL_NMSE, true>, k_gs_col<N, COL_GRAD>, k_ospr_b<N, false>, k_ospr_b<N, true>, k_as_col<N, +1>, k_as_col<N, -1>,
           ColCfg<N>::C, ColCfg<N>::THREADS, sizeof(float2) * ColLds<N>::WORDS,
           ColCfgOspr<N>::C, ColCfgOspr<N>::THREADS, sizeof(float2) * ColLdsOf<ColCfgOspr<N>>::WORDS};
  if constexpr (ColCfgWide<N>::DEFINED) {
    using CW = ColCfgWide<N>;
    e.col_wide = {k_gs_col<N, COL_REPLACE, false, true>, k_gs_col<N, COL_NMSE, false, true>,
                  k_gs_col<N, COL_GRAD, false, true>, CW::C, CW::THREADS,
                  sizeof(float2) * ColLdsOf<CW>::WORDS};
  } else {
    e.col_wide = {nullptr, nullptr, nullptr, 0, 0, 0};
  }
  using PR = typename RowCfg<N>::P;
  using PC = typename ColCfg<N>::P;
  e.row_tw_len[0] = TwRegs<PR, false>::TOTAL * PR::T;
  e.row_tw_len[1] = TwRegs<PR, true>::TOTAL * PR::T;
  e.col_tw_len[0] = TwRegs<PC, false>::TOTAL * PC::T;
  e.col_tw_len[1] = TwRegs<PC, true>::TOTAL * PC::T;
  e.row_tw = twiddle_image_either<PR>;
  e.col_tw = twiddle_image_either<PC>;
  return e;
}

}  // namespace hg
