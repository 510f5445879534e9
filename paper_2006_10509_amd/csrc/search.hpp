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
// accumulated in FP64.  Two trials share one launch (k_search_step): the
// pass over R sums the parts of dE of trial k and of trial k + 1 in both of
// its possible contexts, after trial k rejected (on R) and after trial k
// accepted (on R + dR_k, formed in registers exactly as the update that
// would have been stored).  Every workgroup of the next launch first decides
// the two pending trials itself: it adds their per-workgroup parts in
// workgroup order, trial k + 1's from the context trial k's decision
// selects, so all workgroups reach the same sums and decisions, and
// workgroup 0 records them.  It then applies the accepted moves to R (an
// accepted change costs no pass of its own) and sums its parts of the next
// two trials.  Every value and every FP64 sum is the one a launch per trial
// would form, so decisions and errors do not depend on the pairing.  The
// parts and the decision state alternate between two buffers, so no
// workgroup reads what another writes in the same launch; k_search_finish
// decides the last pending trials.
#pragma once

#include "reduce.hpp"

namespace hg {

constexpr int SEARCH_THREADS = 256;
constexpr int SEARCH_MAX_BLOCKS = 1024;

// One trial evaluated by a launch: its pixel and its change of R's
// coefficient, Q1(p) * delta (zero for a trial out of range).
struct SearchMove {
  int valid;       // in range (pixel, candidate and the pixel's old level)
  int py, px;      // its pixel (valid trials only)
  float2 c;
};

// State handed from the launch of trials k, k + 1 to the next launch (two
// alternating copies in device memory).
struct SearchState {
  double e;        // sum of d^2 before the decision of trial k (NMSE = e / denom)
  int pending;     // trials evaluated by the previous launch and not yet decided: 0, 1 or 2
  int first;       // index k of the first of them
  SearchMove m0;   // trial k
  SearchMove m1r;  // trial k + 1 after trial k rejected
  SearchMove m1a;  // trial k + 1 after trial k accepted
};

// Partial sums of a launch: [2 alternating buffers][3 sums][workgroups], the
// sums being dE of trial k, of trial k + 1 after k rejected, after k accepted.
constexpr int SEARCH_SUMS = 3;

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
  double* partials;            // [2][SEARCH_SUMS][SEARCH_MAX_BLOCKS]: per workgroup of k_search_step
  uint8_t* accepted;           // [n] or null
  float* nmse;                 // [n + 1] or null
  int H, W;
  // rows of R the search keeps and updates: H/2 + 1 when the hologram is real
  // (binary levels, Fourier plane: R(-u) = conj R(u), so the rows y <= H/2
  // hold all of R), else H
  int hh;
  uint32_t hmask, wmask;       // H - 1, W - 1 for a power of two, else 0
  uint32_t wshift;             // log2 W when wmask is set
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

// HALF (a.hh < a.H): pixel (uy, ux) of a kept row 0 < uy < H/2 stands for
// itself and its mirror (H - uy, -ux mod W), which has the same |R| and the
// same change of |R|^2 under any move; rows 0 and H/2 hold their own mirrors.
// The mirror's T^2 index, or -1 when the pixel has no separate mirror.
template <bool HALF>
__device__ __forceinline__ int search_mirror(const SearchArgs& a, uint32_t uy, uint32_t ux) {
  if (!HALF || uy == 0 || 2 * uy == (uint32_t)a.H) return -1;
  return (int)(((uint32_t)a.H - uy) * (uint32_t)a.W + (ux == 0 ? 0u : (uint32_t)a.W - ux));
}

// Sum of d^2 over R (FP64), one partial per workgroup.
template <bool HALF>
__global__ __launch_bounds__(SEARCH_THREADS) void k_search_error(SearchArgs a) {
  __shared__ double red[SEARCH_THREADS];
  const size_t n = (size_t)a.hh * a.W;
  const float sa = a.sc->a, sb = a.sc->b;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * SEARCH_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * SEARCH_THREADS) {
    const float nr = cnorm(a.replay[i]);
    const float d = fmaf(nr, sa, -(a.t2[i] * sb));
    acc += (double)d * d;
    if constexpr (HALF) {
      const int im = search_mirror<HALF>(a, (uint32_t)(i / a.W), (uint32_t)(i % a.W));
      if (im >= 0) {
        const float dm = fmaf(nr, sa, -(a.t2[im] * sb));
        acc += (double)dm * dm;
      }
    }
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
    a.state[0].pending = 0;
    a.state[0].first = 0;
    if (a.nmse) a.nmse[0] = (float)(s / a.sc->denom);
  }
}

// Decision of trial j whose error change is s: direct search accepts
// dE < 0; with a temperature the Metropolis rule also accepts
// u_j < exp(-dNMSE / temp_j); a trial out of range is rejected.  Workgroup 0
// records the decision.
__device__ __forceinline__ bool search_decide(const SearchArgs& a, int j, bool valid, double s) {
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

// The decisions of the pending trials of state st from the nb per-workgroup
// parts of their sums in partial buffer buf (all three sums are read and
// reduced together; every thread of the workgroup gets them): mv0, mv1
// receive the accepted moves in order, e the error after them; the NMSE
// after each trial is recorded.  (kp, kl) pairs are the accepted moves' new
// levels, newest last, for the old-level lookup of the following trials
// (workgroup 0 may be writing them to the level map during this launch).
struct SearchDecided {
  SearchMove mv0, mv1;   // the accepted moves in order (n_moves of them)
  int n_moves;
  int kp0, kl0, kp1, kl1;  // (pixel, new level) of the accepted moves, newest last
  double e;
};
__device__ __forceinline__ SearchDecided search_decide_pending(const SearchArgs& a, const SearchState& st, int buf,
                                                               int nb, double* red) {
  SearchDecided d;
  d.n_moves = 0;
  d.kp0 = d.kp1 = -1;
  d.kl0 = d.kl1 = 0;
  d.mv0 = d.mv1 = st.m0;
  d.e = st.e;
  if (st.pending == 0) return d;
  const double* part = a.partials + (size_t)buf * SEARCH_SUMS * SEARCH_MAX_BLOCKS;
  const bool two = st.pending == 2;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int i = threadIdx.x; i < nb; i += SEARCH_THREADS) {
    v0 += part[i];
    if (two) {
      v1 += part[SEARCH_MAX_BLOCKS + i];
      v2 += part[2 * SEARCH_MAX_BLOCKS + i];
    }
  }
  block_sum3_f64_tree<SEARCH_THREADS>(v0, v1, v2, red);
  const int j0 = st.first;
  const bool ok0 = search_decide(a, j0, st.m0.valid != 0, v0);
  if (ok0) {
    d.e += v0;
    d.mv0 = st.m0;
    d.n_moves = 1;
    d.kp0 = a.trials[2 * j0];
    d.kl0 = a.trials[2 * j0 + 1];
  }
  if (a.nmse && blockIdx.x == 0 && threadIdx.x == 0) a.nmse[j0 + 1] = (float)(d.e / a.sc->denom);
  if (two) {
    const SearchMove m1 = ok0 ? st.m1a : st.m1r;
    const double s1 = ok0 ? v2 : v1;
    const bool ok1 = search_decide(a, j0 + 1, m1.valid != 0, s1);
    if (ok1) {
      d.e += s1;
      if (ok0) {
        d.mv1 = m1;
      } else {
        d.mv0 = m1;
      }
      d.n_moves += 1;
      d.kp1 = a.trials[2 * (j0 + 1)];
      d.kl1 = a.trials[2 * (j0 + 1) + 1];
    }
    if (a.nmse && blockIdx.x == 0 && threadIdx.x == 0) a.nmse[j0 + 2] = (float)(d.e / a.sc->denom);
  }
  return d;
}

// Current level of pixel p (in range): the newest of the decided new levels,
// else the level map's entry.
__device__ __forceinline__ int search_level(const SearchArgs& a, const SearchDecided& d, int p) {
  if (d.kp1 == p) return d.kl1;
  if (d.kp0 == p) return d.kl0;
  return (int)a.levels[p];
}

__device__ __forceinline__ SearchMove search_move(const SearchArgs& a, int p, int cand, int old) {
  SearchMove m;
  const bool ok = a.valid(p, cand);
  m.valid = ok && old < a.L;
  m.py = ok ? p / a.W : 0;
  m.px = ok ? p % a.W : 0;
  m.c = search_delta(a, p, cand, old);
  return m;
}

// exp(-2 pi i (uy py / H + ux px / W)), the coefficient's pattern at replay
// pixel u (the products stay below 2^32: H, W <= 8192).
__device__ __forceinline__ uint32_t search_mod(uint32_t v, uint32_t n, uint32_t mask) {
  return mask ? (v & mask) : v % n;
}
__device__ __forceinline__ float2 search_wave_x(const SearchArgs& a, uint32_t ux, const SearchMove& m) {
  return a.unit_x[search_mod(ux * (uint32_t)m.px, (uint32_t)a.W, a.wmask)];
}
__device__ __forceinline__ float2 search_wave(const SearchArgs& a, uint32_t uy, const SearchMove& m, float2 wx) {
  return cmul(a.unit_y[search_mod(uy * (uint32_t)m.py, (uint32_t)a.H, a.hmask)], wx);
}

// Part of dE of adding dr = c w to r (pixel error d): s (2 d + s).
__device__ __forceinline__ double search_de(float2 r, float2 dr, float c2, float d, float sa) {
  const float s = sa * fmaf(2.0f, fmaf(r.x, dr.x, r.y * dr.y), c2);
  return (double)s * (double)fmaf(2.0f, d, s);
}
// The same with the pixel's mirror (error dm), whose change conj(dr) of
// conj(r) gives the same s: s (2 d + s) + s (2 dm + s).
__device__ __forceinline__ double search_de_pair(float2 r, float2 dr, float c2, float d, float dm, float sa) {
  const float s = sa * fmaf(2.0f, fmaf(r.x, dr.x, r.y * dr.y), c2);
  return (double)s * (double)fmaf(2.0f, d, s) + (double)s * (double)fmaf(2.0f, dm, s);
}

// Trials k and k + 1 (k + 1 < n, else trial k alone): decide the previous
// launch's pending trials, apply the accepted moves to R, sum this
// workgroup's parts of dE of trial k and of trial k + 1 in both contexts.
// HALF: the pass runs over the kept rows only (search_mirror).
template <bool HALF>
__global__ __launch_bounds__(SEARCH_THREADS) void k_search_step(SearchArgs a, int k, int n) {
  __shared__ double red[3 * SEARCH_THREADS];
  const int buf = (k >> 1) & 1;
  const SearchState st = a.state[buf];
  const int nb = (int)gridDim.x;
  const uint32_t npx = (uint32_t)a.hh * (uint32_t)a.W;
  const uint32_t i0 = blockIdx.x * SEARCH_THREADS + threadIdx.x, stride = gridDim.x * SEARCH_THREADS;
  // This thread's first elements of R and T^2 do not depend on the pending
  // decisions: their loads go out before the decisions, whose partial-sum
  // reads and reductions then overlap them.
  // (indices clamped into the frame: the loads are unconditional, and the
  // loop below uses only the elements that exist)
  constexpr uint32_t PF = 4;
  const uint32_t last = npx - 1;
  const float2 rp0 = a.replay[min(i0, last)], rp1 = a.replay[min(i0 + stride, last)];
  const float2 rp2 = a.replay[min(i0 + 2 * stride, last)], rp3 = a.replay[min(i0 + 3 * stride, last)];
  const float tp0 = a.t2[min(i0, last)], tp1 = a.t2[min(i0 + stride, last)];
  const float tp2 = a.t2[min(i0 + 2 * stride, last)], tp3 = a.t2[min(i0 + 3 * stride, last)];
  const SearchDecided dec = search_decide_pending(a, st, buf ^ 1, nb, red);
  // trial k
  const int p0 = a.trials[2 * k], cand0 = a.trials[2 * k + 1];
  const int old0 = a.valid(p0, cand0) ? search_level(a, dec, p0) : 0;
  const SearchMove m0 = search_move(a, p0, cand0, old0);
  // trial k + 1 after trial k rejected / accepted
  const bool two = k + 1 < n;
  SearchMove m1r, m1a;
  if (two) {
    const int p1 = a.trials[2 * (k + 1)], cand1 = a.trials[2 * (k + 1) + 1];
    const bool ok1 = a.valid(p1, cand1);
    const int old1r = ok1 ? search_level(a, dec, p1) : 0;
    const int old1a = ok1 ? (a.valid(p0, cand0) && p1 == p0 ? cand0 : old1r) : 0;
    m1r = search_move(a, p1, cand1, old1r);
    m1a = search_move(a, p1, cand1, old1a);
  } else {
    m1r.valid = 0;
    m1r.py = m1r.px = 0;
    m1r.c = make_float2(0.0f, 0.0f);
    m1a = m1r;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SearchState nx;
    nx.e = dec.e;
    nx.pending = two ? 2 : 1;
    nx.first = k;
    nx.m0 = m0;
    nx.m1r = m1r;
    nx.m1a = m1a;
    a.state[buf ^ 1] = nx;
  }
  const float sa = a.sc->a, sb = a.sc->b;
  const float c0 = cnorm(m0.c), c1r = cnorm(m1r.c), c1a = cnorm(m1a.c);
  double acc0 = 0.0, acc1r = 0.0, acc1a = 0.0;
  // When the stride is a multiple of W every element of this thread lies in
  // one column: the column factors of the patterns are loaded once.
  const bool one_col = stride % (uint32_t)a.W == 0;
  const uint32_t ux0 = search_mod(i0, (uint32_t)a.W, a.wmask);
  float2 xv0 = make_float2(0.0f, 0.0f), xv1 = xv0, x0 = xv0, x1 = xv0;
  if (one_col) {
    if (dec.n_moves > 0) xv0 = search_wave_x(a, ux0, dec.mv0);
    if (dec.n_moves > 1) xv1 = search_wave_x(a, ux0, dec.mv1);
    x0 = search_wave_x(a, ux0, m0);
    if (two) x1 = search_wave_x(a, ux0, m1r);  // m1r and m1a share the pixel
  }
  // per element: apply the accepted moves, sum the parts of dE (the first
  // PF elements from the registers loaded above)
  uint32_t j = 0;
  for (uint32_t i = i0; i < npx; i += stride, ++j) {
    float2 r;
    float t2raw;
    if (j < PF) {
      r = j == 0 ? rp0 : j == 1 ? rp1 : j == 2 ? rp2 : rp3;
      t2raw = j == 0 ? tp0 : j == 1 ? tp1 : j == 2 ? tp2 : tp3;
    } else {
      r = a.replay[i];
      t2raw = a.t2[i];
    }
    const uint32_t uy = a.wmask ? i >> a.wshift : i / (uint32_t)a.W;
    const uint32_t ux = one_col ? ux0 : search_mod(i, (uint32_t)a.W, a.wmask);
    if (dec.n_moves > 0) {
      r = cadd(r, cmul(dec.mv0.c, search_wave(a, uy, dec.mv0, one_col ? xv0 : search_wave_x(a, ux, dec.mv0))));
      if (dec.n_moves > 1)
        r = cadd(r, cmul(dec.mv1.c, search_wave(a, uy, dec.mv1, one_col ? xv1 : search_wave_x(a, ux, dec.mv1))));
      a.replay[i] = r;
    }
    const float t2 = t2raw * sb;
    const float d = fmaf(cnorm(r), sa, -t2);
    const float2 dr0 = cmul(m0.c, search_wave(a, uy, m0, one_col ? x0 : search_wave_x(a, ux, m0)));
    if constexpr (HALF) {
      const int im = search_mirror<HALF>(a, uy, ux);
      if (im >= 0) {
        const float t2m = a.t2[im] * sb;
        const float dm = fmaf(cnorm(r), sa, -t2m);
        acc0 += search_de_pair(r, dr0, c0, d, dm, sa);
        if (two) {
          const float2 w1 = search_wave(a, uy, m1r, one_col ? x1 : search_wave_x(a, ux, m1r));
          acc1r += search_de_pair(r, cmul(m1r.c, w1), c1r, d, dm, sa);
          const float2 ra = cadd(r, dr0);
          const float na = cnorm(ra);
          acc1a += search_de_pair(ra, cmul(m1a.c, w1), c1a, fmaf(na, sa, -t2), fmaf(na, sa, -t2m), sa);
        }
        continue;
      }
    }
    acc0 += search_de(r, dr0, c0, d, sa);
    if (two) {
      const float2 w1 = search_wave(a, uy, m1r, one_col ? x1 : search_wave_x(a, ux, m1r));
      acc1r += search_de(r, cmul(m1r.c, w1), c1r, d, sa);
      const float2 ra = cadd(r, dr0);
      acc1a += search_de(ra, cmul(m1a.c, w1), c1a, fmaf(cnorm(ra), sa, -t2), sa);
    }
  }
  double* part = a.partials + (size_t)buf * SEARCH_SUMS * SEARCH_MAX_BLOCKS;
  block_sum3_f64_tree<SEARCH_THREADS>(acc0, acc1r, acc1a, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = acc0;
    if (two) {
      part[SEARCH_MAX_BLOCKS + blockIdx.x] = acc1r;
      part[2 * SEARCH_MAX_BLOCKS + blockIdx.x] = acc1a;
    }
  }
}

// Decisions of the last pending trials of a call (n > 0), one workgroup.
__global__ __launch_bounds__(SEARCH_THREADS) void k_search_finish(SearchArgs a, int n, int nb) {
  __shared__ double red[3 * SEARCH_THREADS];
  // the last step launch (first trial k = 2 ((n - 1) / 2)) read state and
  // wrote its partial sums in buffer (k / 2) & 1, and its state in the other
  const int k = ((n - 1) / 2) * 2;
  const int buf = (k >> 1) & 1;
  search_decide_pending(a, a.state[buf ^ 1], buf, nb, red);
}

}  // namespace hg
