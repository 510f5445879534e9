// Per-call statistics and the deterministic NMSE reduction (host TU only).
//
// The paper's Normaliser provides vector normalisation (Sec. 7.3); here the
// energy normalisation of the error metric needs sum T^2 and sum T^4 of the
// target and sum A^2 of the illumination once per call, and the per-workgroup
// partial sums of every state are combined in a fixed order so that the
// reported NMSE is bitwise reproducible.
#pragma once

#include "kernels.hpp"

namespace hg {

// Target amplitude rearranged once per call for the column pass: FFT order
// (T_f[ky][kx] = T[(ky + H/2) % H][(kx + W/2) % W]) and tiled so that the C
// columns of one column workgroup form one contiguous [ky][c] block.  With a
// signal window (centred, nonzero inside), pixels outside it get -1: the
// windowed column pass reads the sign as the window.
__global__ __launch_bounds__(256) void k_tile_target(const float* __restrict__ target, float* __restrict__ tiled,
                                                     int H, int W, int C, uint32_t total,
                                                     const uint8_t* __restrict__ window = nullptr) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= total) return;
  const int c = i % C;
  const int ky = (i / C) % H;
  const int tile = i / (C * H);
  const int x = tile * C + c;
  float v = 0.0f;
  if (x < W) {
    const int ys = wrap_add_rt(ky, H / 2, H);
    const int xs = wrap_add_rt(x, W / 2, W);
    v = target[(size_t)ys * W + xs];
    if (window && window[(size_t)ys * W + xs] == 0) v = -1.0f;
  }
  tiled[i] = v;
}


// ===========================================================================
// Per-call statistics and the deterministic NMSE reduction
// ===========================================================================
constexpr int STATS_THREADS = 256;
constexpr int STATS_MAX_BLOCKS = 512;

template <int THREADS>
__device__ __forceinline__ double block_sum_f64(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Three block sums at once, each through the same tree as block_sum_f64 (so
// each equals what block_sum_f64 gives for it) with one set of barriers.
// red: 3 * THREADS doubles.
template <int THREADS>
__device__ __forceinline__ void block_sum3_f64_tree(double& v0, double& v1, double& v2, double* red) {
  red[threadIdx.x] = v0;
  red[THREADS + threadIdx.x] = v1;
  red[2 * THREADS + threadIdx.x] = v2;
  __syncthreads();
#pragma unroll
  for (int s = THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      red[THREADS + threadIdx.x] += red[THREADS + threadIdx.x + s];
      red[2 * THREADS + threadIdx.x] += red[2 * THREADS + threadIdx.x + s];
    }
    __syncthreads();
  }
  v0 = red[0];
  v1 = red[THREADS];
  v2 = red[2 * THREADS];
  __syncthreads();
}

// sum T^2, sum T^4, sum A^2 per workgroup (FP64), fixed order; with a
// signal window (same order as the target, nonzero inside) the target sums
// run over the window only.
__global__ __launch_bounds__(STATS_THREADS) void k_stats_partial(const float* __restrict__ target,
                                                                 const float* __restrict__ illum,
                                                                 size_t n, double* __restrict__ part,
                                                                 const uint8_t* __restrict__ window = nullptr) {
  __shared__ double red[STATS_THREADS];
  double t2 = 0.0, t4 = 0.0, a2 = 0.0;
  for (size_t i = (size_t)blockIdx.x * STATS_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * STATS_THREADS) {
    const double tv = (window && window[i] == 0) ? 0.0 : (double)target[i];
    const double q = tv * tv;
    t2 += q;
    t4 += q * q;
    if (illum) {
      const double av = (double)illum[i];
      a2 += av * av;
    }
  }
  t2 = block_sum_f64<STATS_THREADS>(t2, red);
  t4 = block_sum_f64<STATS_THREADS>(t4, red);
  a2 = block_sum_f64<STATS_THREADS>(a2, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 3 + 0] = t2;
    part[blockIdx.x * 3 + 1] = t4;
    part[blockIdx.x * 3 + 2] = a2;
  }
}

// Combine the partials; sum I follows from Parseval: a2_scale sum A^2 for a
// GS state (|H| = A; a2_scale = N_px through one unnormalised FFT2, N_px^2
// through the unnormalised angular-spectrum round trip), or the given
// intensity_sum (N_px^2 for an OSPR average of +-1 holograms).
__global__ __launch_bounds__(STATS_THREADS) void k_stats_final(const double* __restrict__ part, int nblk, size_t n,
                                                               int has_illum, double intensity_sum, double a2_scale,
                                                               Scalars* __restrict__ sc, int unit_target_scale = 0) {
  __shared__ double red[STATS_THREADS];
  double t2 = 0.0, t4 = 0.0, a2 = 0.0;
  for (int i = threadIdx.x; i < nblk; i += STATS_THREADS) {
    t2 += part[i * 3 + 0];
    t4 += part[i * 3 + 1];
    a2 += part[i * 3 + 2];
  }
  t2 = block_sum_f64<STATS_THREADS>(t2, red);
  t4 = block_sum_f64<STATS_THREADS>(t4, red);
  a2 = block_sum_f64<STATS_THREADS>(a2, red);
  if (threadIdx.x == 0) {
    const double npx = (double)n;
    if (!has_illum) a2 = npx;
    const double s_i = intensity_sum > 0.0 ? intensity_sum : a2_scale * a2;
    sc->sum_t2 = t2;
    sc->sum_t4 = t4;
    sc->sum_a2 = a2;
    sc->a = (float)(npx / s_i);
    sc->b = (float)(npx / t2);
    sc->denom = npx * npx * t4 / (t2 * t2);
    sc->g = (float)(2.0 * (npx / s_i) / sc->denom);
    // the target scale of a signal window; 1 where the target is imposed as
    // given (an amplitude-only SLM, whose field energy is not fixed)
    sc->c = unit_target_scale ? 1.0f : (float)sqrt(s_i / t2);
  }
}

// Windowed NMSE of state blockIdx.x from the three per-workgroup sums of the
// windowed column pass (sum x, sum x^2, sum x y; x = a I, y = b T^2, so that
// sum_M y = N_px and sum_M y^2 = denom):
//   NMSE = sum_M (x / S1 - y / N_px)^2 / sum_M (y / N_px)^2
//        = 1 + (S2 / S1^2 - 2 S3 / (S1 N_px)) N_px^2 / denom,
// 1 when no light reaches the window (S1 = 0).  Fixed order, FP64.
__global__ __launch_bounds__(STATS_THREADS) void k_window_nmse_reduce(const double* __restrict__ wpartials, int nwg,
                                                                      const Scalars* __restrict__ sc, size_t npx,
                                                                      float* __restrict__ nmse) {
  __shared__ double red[STATS_THREADS];
  const double* p = wpartials + (size_t)blockIdx.x * 3 * nwg;
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int i = threadIdx.x; i < nwg; i += STATS_THREADS) {
    s1 += p[i];
    s2 += p[nwg + i];
    s3 += p[2 * nwg + i];
  }
  s1 = block_sum_f64<STATS_THREADS>(s1, red);
  s2 = block_sum_f64<STATS_THREADS>(s2, red);
  s3 = block_sum_f64<STATS_THREADS>(s3, red);
  if (threadIdx.x == 0) {
    const double n = (double)npx;
    const double e = s1 > 0.0 ? 1.0 + (s2 / (s1 * s1) - 2.0 * s3 / (s1 * n)) * n * n / sc->denom : 1.0;
    nmse[blockIdx.x] = (float)e;
  }
}

// nmse[k] = sum_wg partials[k][wg] / denom, one workgroup per state, fixed
// order; blockIdx.y selects the batch item (partials, Scalars and nmse
// advance by partial_stride, 1 and nmse_stride).
__global__ __launch_bounds__(STATS_THREADS) void k_nmse_reduce(const float* __restrict__ partials, int nwg,
                                                               const Scalars* __restrict__ sc,
                                                               float* __restrict__ nmse, size_t partial_stride,
                                                               size_t nmse_stride) {
  __shared__ double red[STATS_THREADS];
  partials += blockIdx.y * partial_stride;
  sc += blockIdx.y;
  nmse += blockIdx.y * nmse_stride;
  const float* p = partials + (size_t)blockIdx.x * nwg;
  double s = 0.0;
  for (int i = threadIdx.x; i < nwg; i += STATS_THREADS) s += (double)p[i];
  s = block_sum_f64<STATS_THREADS>(s, red);
  if (threadIdx.x == 0) nmse[blockIdx.x] = (float)(s / sc->denom);
}

// nmse[b] = sum_wg partials[b][wg] / denom of plane (first + b) % planes: the
// steps of a plane-by-plane multi-plane loop, one workgroup per step;
// blockIdx.y selects the problem of a batch (partials, Scalars and nmse
// advance by partial_stride, planes and nmse_stride).
__global__ __launch_bounds__(STATS_THREADS) void k_nmse_reduce_planes(const float* __restrict__ partials, int nwg,
                                                                      const Scalars* __restrict__ sc, int planes,
                                                                      int first, float* __restrict__ nmse,
                                                                      size_t partial_stride, size_t nmse_stride) {
  __shared__ double red[STATS_THREADS];
  partials += blockIdx.y * partial_stride;
  sc += blockIdx.y * (size_t)planes;
  nmse += blockIdx.y * nmse_stride;
  const float* p = partials + (size_t)blockIdx.x * nwg;
  double s = 0.0;
  for (int i = threadIdx.x; i < nwg; i += STATS_THREADS) s += (double)p[i];
  s = block_sum_f64<STATS_THREADS>(s, red);
  if (threadIdx.x == 0) nmse[blockIdx.x] = (float)(s / sc[(first + (int)blockIdx.x) % planes].denom);
}

// loss[k] = sum_j (sum_wg partials[k][b][j][wg]) / denom_j: the summed NMSE
// of the `planes` replay planes of state k of problem b = blockIdx.y, one
// workgroup per state and problem, fixed order.  The partials of state k
// start k state_stride floats in, those of problem b b problem_stride floats
// further; its Scalars and losses lie at the given strides.
__global__ __launch_bounds__(STATS_THREADS) void k_loss_reduce(const float* __restrict__ partials, int nwg,
                                                               int planes, const Scalars* __restrict__ sc,
                                                               float* __restrict__ loss, size_t problem_stride,
                                                               size_t state_stride, size_t loss_stride) {
  __shared__ double red[STATS_THREADS];
  partials += blockIdx.y * problem_stride + blockIdx.x * state_stride;
  sc += blockIdx.y * (size_t)planes;
  loss += blockIdx.y * loss_stride;
  double total = 0.0;
  for (int j = 0; j < planes; ++j) {
    const float* p = partials + (size_t)j * nwg;
    double s = 0.0;
    for (int i = threadIdx.x; i < nwg; i += STATS_THREADS) s += (double)p[i];
    s = block_sum_f64<STATS_THREADS>(s, red);
    total += s / sc[j].denom;
  }
  if (threadIdx.x == 0) loss[blockIdx.x] = (float)total;
}

// OSPR pairs, after the last pass C: S (centred) holds sum_n |H_n|^2 with
// H_n = FFT2(h_re + i h_im) of real +-1 holograms.  Since |FFT2 h_re(k)|^2 +
// |FFT2 h_im(k)|^2 = (|H(k)|^2 + |H(-k)|^2) / 2, the mean over the 2N real
// subframes is I(k) = (S(k) + S(-k)) * scale with scale = 1 / (4 N).  -k is
// the mirrored pixel ((H - y) % H, (W - x) % W) in centred order.  In place:
// every mirror pair is read and written by the thread of its first pixel.
// With partials, also the NMSE partial sums against T^2 (as pass C does).
constexpr int PAIR_THREADS = 256;
constexpr int PAIR_MAX_BLOCKS = 1024;
__global__ __launch_bounds__(PAIR_THREADS) void k_ospr_pair_finish(float* __restrict__ intensity,
                                                                   const float* __restrict__ target, int H, int W,
                                                                   float scale, const Scalars* __restrict__ sc,
                                                                   float* __restrict__ partials) {
  __shared__ double red[PAIR_THREADS];
  const size_t n = (size_t)H * W;
  const float sa = partials ? sc->a : 0.0f;
  const float sb = partials ? sc->b : 0.0f;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * PAIR_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * PAIR_THREADS) {
    const int y = (int)(i / W), x = (int)(i % W);
    const size_t j = (size_t)((H - y) % H) * W + (size_t)((W - x) % W);
    if (j < i) continue;
    const float v = (intensity[i] + intensity[j]) * scale;
    intensity[i] = v;
    if (j != i) intensity[j] = v;
    if (partials) {
      const float ti = target[i], di = fmaf(v, sa, -(ti * ti * sb));
      acc += (double)di * di;
      if (j != i) {
        const float tj = target[j], dj = fmaf(v, sa, -(tj * tj * sb));
        acc += (double)dj * dj;
      }
    }
  }
  if (partials) {
    acc = block_sum_f64<PAIR_THREADS>(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = (float)acc;
  }
}

}  // namespace hg
