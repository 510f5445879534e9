// Transform lengths compiled into the library and the launch shape of each.
//
// A row pass gives every row (length W, the contiguous axis) to a team of T
// threads and packs TEAMS rows into one workgroup.  FT is the column tile
// width of the tiled field layout the GS-family row kernels of that length
// take (0: row order only; a plan is tiled when its column pass's tile width
// divides FT).  A column pass gives every
// column (length H) to a team and packs C adjacent columns into one
// workgroup, so each global access covers C * 8 contiguous bytes per row.
// Teams of at most 64 threads that do not straddle a wavefront exchange data
// through LDS with wavefront-level ordering only; wider teams use s_barrier.
#pragma once

#include "fft_core.hpp"

namespace hg {

template <int N> struct RowCfg;
template <int N> struct ColCfg;

#define HG_ROW_CFG(N_, TEAMS_, T_, FT_, ...)                              \
  template <> struct RowCfg<N_> {                                        \
    using P = Plan<N_, T_, __VA_ARGS__>;                                 \
    static constexpr int TEAMS = TEAMS_;                                 \
    static constexpr int FT = FT_;                                       \
    static constexpr int THREADS = TEAMS_ * T_;                          \
    static constexpr bool WAVE_SYNC = (T_ <= 64) && (64 % T_ == 0);      \
  };
#define HG_COL_CFG(N_, C_, T_, ...)                                       \
  template <> struct ColCfg<N_> {                                        \
    using P = Plan<N_, T_, __VA_ARGS__>;                                 \
    static constexpr int C = C_;                                         \
    static constexpr int THREADS = C_ * T_;                              \
    static constexpr bool WAVE_SYNC = (C_ * T_ <= 64);                   \
  };

// The shapes of lengths 512, 1024, 1080, 1280, 1536, 1920, 2048, 2160, 3840,
// 4096 and 8192 were chosen by timing the GS loop on MI355X over candidate team sizes, radix
// orders and column tile widths (single holograms and same-shape batches;
// paper_2006_10509_amd/autotune.py automates the search); the rest are
// untuned defaults.  The tiled GS layout took a 1024^2 iteration from 21.8
// to 20.1 us and is level at 2048^2; rows of 64-thread teams cannot
// interleave and keep row order, and so does 1920 x 1080, where tiles
// measured 3-6 % slower.  Wider column tiles (C = 8: 64-byte row segments)
// win where the frame still gives every CU a tile.
// Tuned with paper_2006_10509_amd/autotune.py on MI355X (Fourier, L = 4, us
// per hologram-iteration): 1080 x 1920 in batches of 8, rows of 1920 as one
// 256-thread team in the order 8·3·5·16: 30.3 -> 22.9 (a single hologram at
// Fresnel L = 8: 56.7 -> 42.8 us per iteration); 2160 x 3840, one hologram:
// rows 1 x 256 (16·5·16·3), columns 2 x 256 (16·3·5·3·3): 139.6 -> 113.0;
// 1024 x 1280 in batches of 8, rows of 1280 on tiles of 2: 21.4 -> 12.2;
// 1536 x 2048, one hologram, columns of 1536 as two 256-thread teams:
// 45.5 -> 41.4.  A single 1080 x 1920 hologram found nothing better than
// 1 % (38.6 -> 38.3, other radix orders).
// 4096^2 (Fresnel, L = 8, us per iteration): rows of 512-thread teams
// (8·8·8·8, twiddles in registers) on tiles of 4 with one-column 512-thread
// column workgroups 206; two 128-thread teams (16·16·16) 322; two 256-thread
// teams with two-column 256-thread columns 241; tiles of 8: 230.
// 8192^2: one 1024-thread row per workgroup in the palindromic order
// 8·8·2·8·8 (22 twiddles in registers), tiles of 4: 1214; tiles of 2: 1382
// (the row pass rewrites 1.76x its bytes: eight workgroups share every line),
// 8 and 16: 1254 and 1262; row order 1530 (the column pass then reads 2.6x
// its bytes: eight workgroups share every line of 8192 rows, more than the
// L2 holds); 8·8·8·8·2 (twiddles read from memory) on tiles of 2: 1416;
// 512-thread row teams: 1190-1254.
//          N     rows/WG  T    FT  radices
HG_ROW_CFG(16,    64,     4,  0,   4, 4)
HG_ROW_CFG(32,    32,     8,  0,   4, 2, 4)
HG_ROW_CFG(64,    32,     8,  0,   8, 8)
HG_ROW_CFG(128,   16,    16,  0,   8, 2, 8)
HG_ROW_CFG(256,   16,    16,  0,   16, 16)
HG_ROW_CFG(512,   2,    64,  0,   8, 8, 8)
HG_ROW_CFG(1024,   2,   128,  4,   8, 4, 4, 8)
HG_ROW_CFG(2048,   1,   256,  8,   8, 4, 2, 4, 8)
HG_ROW_CFG(4096,   1,   512,  4,   8, 8, 8, 8)
HG_ROW_CFG(24,    32,     8,  0,   8, 3)
HG_ROW_CFG(60,    16,    16,  0,   4, 3, 5)
HG_ROW_CFG(90,    16,    16,  0,   2, 3, 3, 5)
HG_ROW_CFG(120,   16,    16,  0,   8, 3, 5)
HG_ROW_CFG(1080,   4,    64,  0,   8, 3, 3, 3, 5)
HG_ROW_CFG(1920,   1,   256,  0,   8, 3, 5, 16)
HG_ROW_CFG(1280,   2,   128,  2,   16, 5, 16)
HG_ROW_CFG(1536,   2,   128,  0,   8, 8, 8, 3)
HG_ROW_CFG(2160,   4,   144,  0,   16, 3, 3, 3, 5)
HG_ROW_CFG(3840,   1,   256,  0,   16, 5, 16, 3)
HG_ROW_CFG(8192,   1,  1024,  4,   8, 8, 2, 8, 8)

//          N     cols/WG  T    radices
HG_COL_CFG(16,    16,     4,   4, 4)
HG_COL_CFG(32,    16,     8,   4, 2, 4)
HG_COL_CFG(64,    16,     8,   8, 8)
HG_COL_CFG(128,   16,    16,   8, 2, 8)
HG_COL_CFG(256,    8,    16,   16, 16)
HG_COL_CFG(512,   8,    64,   8, 8, 8)
HG_COL_CFG(1024,   2,   128,   8, 4, 4, 8)
HG_COL_CFG(2048,   2,   128,   16, 8, 16)
HG_COL_CFG(4096,   1,   512,   8, 8, 8, 8)
HG_COL_CFG(24,    16,     8,   8, 3)
HG_COL_CFG(60,    16,    16,   4, 3, 5)
HG_COL_CFG(90,    16,    16,   2, 3, 3, 5)
HG_COL_CFG(120,   16,    16,   8, 3, 5)
HG_COL_CFG(1080,   8,   120,   8, 3, 3, 3, 5)
HG_COL_CFG(1920,   4,    64,   16, 8, 3, 5)
HG_COL_CFG(1280,   4,   128,   16, 5, 16)
HG_COL_CFG(1536,   2,   256,   8, 8, 8, 3)
HG_COL_CFG(2160,   2,   256,   16, 3, 5, 3, 3)
HG_COL_CFG(3840,   2,   256,   16, 16, 3, 5)
HG_COL_CFG(8192,   2,   256,   8, 8, 8, 16)

// Wider column workgroups for launches over a batch of holograms, where the
// GPU holds several workgroups of every CU's share: same teams (T, radices,
// hence the same twiddle images) as ColCfg<N>, C columns per workgroup.
// Lengths without one use ColCfg<N> for batches too.
template <int N> struct ColCfgWide { static constexpr bool DEFINED = false; static constexpr int C = 0; };
#define HG_COL_WIDE(N_, C_)                                               \
  template <> struct ColCfgWide<N_> {                                    \
    using P = typename ColCfg<N_>::P;                                    \
    static constexpr bool DEFINED = true;                                \
    static constexpr int C = C_;                                         \
    static constexpr int THREADS = C_ * P::T;                            \
    static constexpr bool WAVE_SYNC = (C_ * P::T <= 64);                 \
  };
// 1024^2 in batches of 8: 10.9 us per hologram-iteration with four columns
// per workgroup against 11.9 with two (a single hologram: 19.9 against 18.7).
HG_COL_WIDE(1024, 4)

// Columns per workgroup of OSPR's column pass (binarisation between the two
// transforms, no error sums), with the teams of ColCfg<N>: ColCfg<N>'s unless
// specialised.  At 2048 the GS passes are faster with two columns (2048^2 GS
// 57.3 -> 56.6 us per iteration; a batch of 16 at Fourier L = 4: 32.2 ->
// 30.5 ms) and OSPR's pass B with four (22.1 -> 16.9 us).
template <int N> struct ColCfgOspr {
  using P = typename ColCfg<N>::P;
  static constexpr int C = ColCfg<N>::C;
  static constexpr int THREADS = ColCfg<N>::THREADS;
  static constexpr bool WAVE_SYNC = ColCfg<N>::WAVE_SYNC;
};
#define HG_COL_OSPR(N_, C_)                                               \
  template <> struct ColCfgOspr<N_> {                                    \
    using P = typename ColCfg<N_>::P;                                    \
    static constexpr int C = C_;                                         \
    static constexpr int THREADS = C_ * P::T;                            \
    static constexpr bool WAVE_SYNC = (C_ * P::T <= 64);                 \
  };
HG_COL_OSPR(2048, 4)

// X-macro over every compiled length (used for host dispatch tables).
#define HG_FOR_EACH_LENGTH(X) \
  X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) \
  X(24) X(60) X(90) X(120) X(1080) X(1920) \
  X(1280) X(1536) X(2160) X(3840) X(8192)

}  // namespace hg
