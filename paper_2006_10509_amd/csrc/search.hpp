// Single-pixel search over an L-level phase hologram: direct binary search
// and simulated annealing with a rank-one update of the replay field (the
// paper's HoloGenAlgDSCuda, HoloGenAlgSACuda and FFTUpdaterCuda, Sec. 7.3).
// Host translation unit only.
//
// Changing the level of SLM pixel p = (py, px) from l to c changes the
// hologram by delta = A (w_c - w_l) at p alone (w_l = exp(2 pi i l / L)), so
// the replay field R = FFT2(Q1 H) changes by
//   dR(u) = Q1(p) delta exp(-2 pi i (uy py / H + ux px / W))
// at every replay pixel u: one pass over R instead of a transform.  With
// d(u) = a |R(u)|^2 - b T(u)^2 (the NMSE summand of the GS passes; a and b
// stay fixed because |H| = A keeps sum |R|^2 = N_px sum A^2) the error change is
//   dE = sum_u s(u) (2 d(u) + s(u)),  s(u) = a (2 Re(conj(R(u)) dR(u)) + |dR(u)|^2),
// accumulated in FP64.  A trial runs as two launches: k_search_trial applies
// the previous trial's update to R when it was accepted (so an accepted change
// costs no pass of its own) and sums dE for this trial; k_search_decide, one
// workgroup, takes the decision and records it.
#pragma once

#include "reduce.hpp"

namespace hg {

constexpr int SEARCH_THREADS = 256;
constexpr int SEARCH_MAX_BLOCKS = 1024;

// Decision state carried from one trial to the next (device memory).
struct SearchState {
  double e;        // current sum of d^2 (NMSE = e / denom)
  int pending;     // the last trial was accepted and R does not include it yet
  int py, px;      // its pixel
  float2 c;        // its Q1(p) * delta
};

// Everything a trial needs to know.
struct SearchArgs {
  float2* replay;              // R [H][W], FFT order
  const float* t2;             // T^2 in FFT order [H][W]
  uint8_t* levels;             // hologram level map [H][W]
  const int32_t* trials;       // [n][2]: pixel index, candidate level
  const float* temperature;    // [n] or null (direct search)
  const float* uniform;        // [n] or null
  const float2* lvl_tab;       // exp(2 pi i l / L)
  const float2* q1y;           // Fresnel source chirp or null
  const float2* q1x;
  const float2* unit_y;        // exp(-2 pi i k / H), k < H
  const float2* unit_x;        // exp(-2 pi i k / W), k < W
  const Scalars* sc;
  SearchState* state;
  double* partials;            // one per workgroup of k_search_trial
  uint8_t* accepted;           // [n] or null
  float* nmse;                 // [n + 1] or null
  int H, W;
  int L;                       // number of levels
  // A trial whose pixel or level is out of range is a rejected no-op, so a
  // bad trial list cannot send a kernel outside its buffers.
  __device__ __forceinline__ bool valid(int p, int cand) const {
    return p >= 0 && p < H * W && cand >= 0 && cand < L;
  }
};

__device__ __forceinline__ float2 search_delta(const SearchArgs& a, int p, int cand) {
  if (!a.valid(p, cand)) return make_float2(0.0f, 0.0f);
  const int old = a.levels[p];
  if (old >= a.L) return make_float2(0.0f, 0.0f);   // a level map entry out of range: no move
  const float2 wc = a.lvl_tab[cand], wl = a.lvl_tab[old];
  float2 c = make_float2(wc.x - wl.x, wc.y - wl.y);
  if (a.q1y) c = cmul(c, cmul(a.q1y[p / a.W], a.q1x[p % a.W]));
  return c;
}

// T^2 in FFT order from the centred target amplitude.
__global__ __launch_bounds__(256) void k_search_target(const float* __restrict__ target, float* __restrict__ t2,
                                                       int H, int W) {
  const size_t n = (size_t)H * W;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const int y = (int)(i / W), x = (int)(i % W);
    const float t = target[(size_t)wrap_add_rt(y, H / 2, H) * W + wrap_add_rt(x, W / 2, W)];
    t2[i] = t * t;
  }
}

// Phase of a level map, as the input of the transform that builds R.
__global__ __launch_bounds__(256) void k_search_phase(const uint8_t* __restrict__ levels, float* __restrict__ phase,
                                                      size_t n, float delta) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    phase[i] = (float)levels[i] * delta;
}

// Sum of d^2 over R (FP64), one partial per workgroup.
__global__ __launch_bounds__(SEARCH_THREADS) void k_search_error(SearchArgs a) {
  __shared__ double red[SEARCH_THREADS];
  const size_t n = (size_t)a.H * a.W;
  const float sa = a.sc->a, sb = a.sc->b;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * SEARCH_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * SEARCH_THREADS) {
    const float d = fmaf(cnorm(a.replay[i]), sa, -(a.t2[i] * sb));
    acc += (double)d * d;
  }
  acc = block_sum_f64<SEARCH_THREADS>(acc, red);
  if (threadIdx.x == 0) a.partials[blockIdx.x] = acc;
}

__global__ __launch_bounds__(SEARCH_THREADS) void k_search_start(SearchArgs a, int nb) {
  __shared__ double red[SEARCH_THREADS];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += SEARCH_THREADS) s += a.partials[i];
  s = block_sum_f64<SEARCH_THREADS>(s, red);
  if (threadIdx.x == 0) {
    a.state->e = s;
    a.state->pending = 0;
    if (a.nmse) a.nmse[0] = (float)(s / a.sc->denom);
  }
}

// Trial k: apply the pending update, then sum dE of moving pixel p_k to its
// candidate level.
__global__ __launch_bounds__(SEARCH_THREADS) void k_search_trial(SearchArgs a, int k) {
  __shared__ double red[SEARCH_THREADS];
  const size_t n = (size_t)a.H * a.W;
  const int p = a.trials[2 * k], cand = a.trials[2 * k + 1];
  const bool ok = a.valid(p, cand);
  const int py = ok ? p / a.W : 0, px = ok ? p % a.W : 0;
  const float2 c = search_delta(a, p, cand);
  const SearchState st = *a.state;
  const float sa = a.sc->a, sb = a.sc->b;
  const float c2 = cnorm(c);
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * SEARCH_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * SEARCH_THREADS) {
    const uint32_t uy = (uint32_t)(i / a.W), ux = (uint32_t)(i % a.W);
    float2 r = a.replay[i];
    if (st.pending) {
      const float2 w = cmul(a.unit_y[(uy * (uint32_t)st.py) % (uint32_t)a.H],
                            a.unit_x[(ux * (uint32_t)st.px) % (uint32_t)a.W]);
      r = cadd(r, cmul(st.c, w));
      a.replay[i] = r;
    }
    const float2 w = cmul(a.unit_y[(uy * (uint32_t)py) % (uint32_t)a.H], a.unit_x[(ux * (uint32_t)px) % (uint32_t)a.W]);
    const float2 dr = cmul(c, w);
    const float d = fmaf(cnorm(r), sa, -(a.t2[i] * sb));
    const float s = sa * fmaf(2.0f, fmaf(r.x, dr.x, r.y * dr.y), c2);
    acc += (double)s * (double)fmaf(2.0f, d, s);
  }
  acc = block_sum_f64<SEARCH_THREADS>(acc, red);
  if (threadIdx.x == 0) a.partials[blockIdx.x] = acc;
}

// Decision of trial k (one workgroup): direct search accepts dE < 0; with a
// temperature the Metropolis rule also accepts u_k < exp(-dNMSE / temp_k).
__global__ __launch_bounds__(SEARCH_THREADS) void k_search_decide(SearchArgs a, int k, int nb) {
  __shared__ double red[SEARCH_THREADS];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += SEARCH_THREADS) s += a.partials[i];
  s = block_sum_f64<SEARCH_THREADS>(s, red);
  if (threadIdx.x == 0) {
    const int p = a.trials[2 * k], cand = a.trials[2 * k + 1];
    const bool valid = a.valid(p, cand) && a.levels[p] < a.L;
    bool ok = valid && s < 0.0;
    if (valid && !ok && a.temperature) {
      const double dn = s / a.sc->denom;
      ok = (double)a.uniform[k] < exp(-dn / (double)a.temperature[k]);
    }
    SearchState* st = a.state;
    st->pending = ok ? 1 : 0;
    if (ok) {
      st->py = p / a.W;
      st->px = p % a.W;
      st->c = search_delta(a, p, cand);
      st->e += s;
      a.levels[p] = (uint8_t)cand;
    }
    if (a.accepted) a.accepted[k] = ok ? 1 : 0;
    if (a.nmse) a.nmse[k + 1] = (float)(st->e / a.sc->denom);
  }
}

}  // namespace hg
