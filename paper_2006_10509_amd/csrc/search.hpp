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
// accumulated in FP64.  A trial is one launch (k_search_step).  Every
// workgroup of trial k first decides trial k - 1 itself: it adds that trial's
// per-workgroup parts of dE in workgroup order, so all workgroups reach the
// same sum and decision, and workgroup 0 records it.  It then applies that
// move to R when it was accepted (an accepted change costs no pass of its
// own) and sums its part of trial k's dE.  The parts and the decision state
// alternate between two buffers, so no workgroup reads what another writes in
// the same launch; k_search_finish decides the last trial.
#pragma once

#include "reduce.hpp"

namespace hg {

constexpr int SEARCH_THREADS = 256;
constexpr int SEARCH_MAX_BLOCKS = 1024;

// State handed from the launch of trial k - 1 to that of trial k (two
// alternating copies in device memory).
struct SearchState {
  double e;        // sum of d^2 before the decision of trial k - 1 (NMSE = e / denom)
  int has_prev;    // trial k - 1 exists (k > 0)
  int valid;       // it is in range (pixel, candidate and the pixel's old level)
  int py, px;      // its pixel (valid trials only)
  float2 c;        // its Q1(p) * delta; zero for a trial out of range
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
  SearchState* state;          // [2]
  double* partials;            // [2][SEARCH_MAX_BLOCKS]: one per workgroup of k_search_step
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

// Change of R's coefficient at pixel p when its level goes from old to cand
// (zero for a trial out of range, or a level map entry out of range).
__device__ __forceinline__ float2 search_delta(const SearchArgs& a, int p, int cand, int old) {
  if (!a.valid(p, cand) || old >= a.L) return make_float2(0.0f, 0.0f);
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
    a.state[0].e = s;
    a.state[0].has_prev = 0;
    if (a.nmse) a.nmse[0] = (float)(s / a.sc->denom);
  }
}

// Decision of trial j from its nb per-workgroup parts of dE (every thread of
// the workgroup gets it): direct search accepts dE < 0; with a temperature
// the Metropolis rule also accepts u_j < exp(-dNMSE / temp_j); a trial out of
// range is rejected.  Workgroup 0 records the decision.
__device__ __forceinline__ bool search_decide(const SearchArgs& a, int j, int nb, bool valid, double* red, double& s) {
  const double* part = a.partials + (size_t)(j & 1) * SEARCH_MAX_BLOCKS;
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += SEARCH_THREADS) v += part[i];
  s = block_sum_f64<SEARCH_THREADS>(v, red);
  const int p = a.trials[2 * j], cand = a.trials[2 * j + 1];
  bool ok = valid && s < 0.0;
  if (valid && !ok && a.temperature) {
    const double dn = s / a.sc->denom;
    ok = (double)a.uniform[j] < exp(-dn / (double)a.temperature[j]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (ok) a.levels[p] = (uint8_t)cand;
    if (a.accepted) a.accepted[j] = ok ? 1 : 0;
  }
  return ok;
}

// Trial k: decide trial k - 1, apply its move to R when accepted, sum this
// workgroup's part of dE of moving pixel p_k to its candidate level.
__global__ __launch_bounds__(SEARCH_THREADS) void k_search_step(SearchArgs a, int k) {
  __shared__ double red[SEARCH_THREADS];
  const SearchState st = a.state[k & 1];
  const int nb = (int)gridDim.x;
  // trial k - 1
  bool moved = false;
  int pp = -1, pcand = 0;
  double e = st.e;
  if (st.has_prev) {
    pp = a.trials[2 * (k - 1)];
    pcand = a.trials[2 * (k - 1) + 1];
    double s;
    moved = search_decide(a, k - 1, nb, st.valid != 0, red, s);
    if (moved) e += s;
    if (a.nmse && blockIdx.x == 0 && threadIdx.x == 0) a.nmse[k] = (float)(e / a.sc->denom);
  }
  // trial k: the old level of its pixel is trial k - 1's candidate when that
  // move of the same pixel was accepted (workgroup 0 may be writing it to the
  // level map during this launch), else the map's entry
  const int p = a.trials[2 * k], cand = a.trials[2 * k + 1];
  const bool ok = a.valid(p, cand);
  const int old = ok ? ((moved && p == pp) ? pcand : (int)a.levels[p]) : 0;
  const int py = ok ? p / a.W : 0, px = ok ? p % a.W : 0;
  const float2 c = search_delta(a, p, cand, old);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SearchState nx;
    nx.e = e;
    nx.has_prev = 1;
    nx.valid = ok && old < a.L;
    nx.py = py;
    nx.px = px;
    nx.c = c;
    a.state[(k + 1) & 1] = nx;
  }
  const float sa = a.sc->a, sb = a.sc->b;
  const float c2 = cnorm(c);
  double acc = 0.0;
  const size_t n = (size_t)a.H * a.W;
  for (size_t i = (size_t)blockIdx.x * SEARCH_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * SEARCH_THREADS) {
    const uint32_t uy = (uint32_t)(i / a.W), ux = (uint32_t)(i % a.W);
    float2 r = a.replay[i];
    if (moved) {
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
  if (threadIdx.x == 0) a.partials[(size_t)(k & 1) * SEARCH_MAX_BLOCKS + blockIdx.x] = acc;
}

// Decision of the last trial (n > 0) of a call, one workgroup.
__global__ __launch_bounds__(SEARCH_THREADS) void k_search_finish(SearchArgs a, int n, int nb) {
  __shared__ double red[SEARCH_THREADS];
  const SearchState st = a.state[n & 1];
  double s;
  const bool moved = search_decide(a, n - 1, nb, st.valid != 0, red, s);
  if (a.nmse && threadIdx.x == 0) a.nmse[n] = (float)((moved ? st.e + s : st.e) / a.sc->denom);
}

}  // namespace hg
