// Device building blocks of the Stockham autosort FFT used by every pass.
//
// The paper delegates its transforms to cuFFT behind FFTHandlerCuda (Sec. 2;
// Sec. 7.3).  Here the transform is written out for gfx950: one transform of
// length N is carried by a team of T threads; each thread holds its share of
// the sequence in registers, every radix-R stage is a set of R-point DFTs done
// in registers, and the data moves between stages through LDS in Stockham
// (self-sorting) order, so no bit-reversal pass exists.  The twiddles a thread
// needs are evaluated on the host in FP64, rounded to FP32 and laid out per
// thread (twiddle_image); each thread loads them into registers once per
// kernel with coalesced loads, before the field arrives, so no table access
// sits between stages.
//
// Stage s with radix R and Ns = product of the radices before it: butterfly j
// (0 <= j < N/R) takes x[j + r N/R], r < R, multiplies by w^(r k) with
// k = j mod Ns and w = exp(-+2 pi i / (Ns R)), does an R-point DFT and writes
// output r to (j - k) R + k + r Ns (Stockham 1966; Van Loan 1992, Sec. 1.7).
// Butterflies are dealt to the team's threads round-robin: thread t takes
// j = t + m T.  The first stage therefore reads x[t + m T + r N/R0] and the last
// stage leaves X[t + m T + r N/R_last] in registers, both unit-stride across
// threads, so the global loads and stores around a transform coalesce.
// Running the radices in reversed order leaves the layout the forward order
// starts from, which lets a kernel chain an inverse and a forward transform
// (or the reverse) with a pointwise step between them and no extra exchange.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

// ---------------------------------------------------------------------------
// complex helpers (float2: .x real, .y imaginary)
//
// Every sum of two products is written with an explicit fmaf: left to the
// compiler, a*b + c*d may be contracted as fma(a, b, c*d) or fma(c, d, a*b)
// depending on the surrounding code, so the same arithmetic in two kernels
// (a loop's start pass and its steady-state pass, say) could round
// differently.  With the contraction fixed here, a state computed by any
// sequence of calls is bitwise the same.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmulconj(float2 a, float2 b) {  // a * conj(b)
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cnorm(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }

// multiply by DIR * i  (DIR = -1: forward kernel exp(-...), +1: inverse)
template <int DIR> __device__ __forceinline__ float2 mul_dir_i(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// exact constants of the small DFTs
#define HG_SQRT1_2 0.70710678118654752440f
#define HG_COS_PI_8 0.92387953251128675613f
#define HG_SIN_PI_8 0.38268343236508977173f
#define HG_SIN_PI_3 0.86602540378443864676f
#define HG_COS_2PI_5 0.30901699437494742410f
#define HG_COS_4PI_5 (-0.80901699437494742410f)
#define HG_SIN_2PI_5 0.95105651629515357212f
#define HG_SIN_4PI_5 0.58778525229247312917f

// ---------------------------------------------------------------------------
// R-point DFTs in registers, natural order in and out
// ---------------------------------------------------------------------------
template <int DIR> __device__ __forceinline__ void dft2(float2* a) {
  float2 t = a[1];
  a[1] = csub(a[0], t);
  a[0] = cadd(a[0], t);
}

template <int DIR> __device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = mul_dir_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int DIR> __device__ __forceinline__ void dft4(float2* a) { dft4<DIR>(a[0], a[1], a[2], a[3]); }

// w8^1 and w8^3 with w8 = exp(DIR 2 pi i / 8)
template <int DIR> __device__ __forceinline__ float2 mul_w8_1(float2 a) {
  return DIR < 0 ? make_float2(HG_SQRT1_2 * (a.x + a.y), HG_SQRT1_2 * (a.y - a.x))
                 : make_float2(HG_SQRT1_2 * (a.x - a.y), HG_SQRT1_2 * (a.x + a.y));
}
template <int DIR> __device__ __forceinline__ float2 mul_w8_3(float2 a) {
  return DIR < 0 ? make_float2(HG_SQRT1_2 * (a.y - a.x), -HG_SQRT1_2 * (a.x + a.y))
                 : make_float2(-HG_SQRT1_2 * (a.x + a.y), HG_SQRT1_2 * (a.x - a.y));
}

template <int DIR> __device__ __forceinline__ void dft8(float2* a) {
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  float2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  o1 = mul_w8_1<DIR>(o1);
  o2 = mul_dir_i<DIR>(o2);
  o3 = mul_w8_3<DIR>(o3);
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

// w16^m, m in {1,2,3,4,6,9}
template <int DIR, int M> __device__ __forceinline__ float2 mul_w16(float2 a) {
  constexpr float s = (float)DIR;
  if constexpr (M == 0) return a;
  else if constexpr (M == 1) return cmul(a, make_float2(HG_COS_PI_8, s * HG_SIN_PI_8));
  else if constexpr (M == 2) return mul_w8_1<DIR>(a);
  else if constexpr (M == 3) return cmul(a, make_float2(HG_SIN_PI_8, s * HG_COS_PI_8));
  else if constexpr (M == 4) return mul_dir_i<DIR>(a);
  else if constexpr (M == 6) return mul_w8_3<DIR>(a);
  else  // M == 9: angle 9 pi / 8
    return cmul(a, make_float2(-HG_COS_PI_8, -s * HG_SIN_PI_8));
}

template <int DIR> __device__ __forceinline__ void dft16(float2* a) {
  // n = n2 + 4 n1, k = k1 + 4 k2: inner 4-point DFTs over n1, twiddle w16^(n2 k1),
  // outer 4-point DFTs over n2.
  float2 b[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 x0 = a[n2], x1 = a[n2 + 4], x2 = a[n2 + 8], x3 = a[n2 + 12];
    dft4<DIR>(x0, x1, x2, x3);
    b[n2 * 4 + 0] = x0; b[n2 * 4 + 1] = x1; b[n2 * 4 + 2] = x2; b[n2 * 4 + 3] = x3;
  }
  b[1 * 4 + 1] = mul_w16<DIR, 1>(b[1 * 4 + 1]);
  b[1 * 4 + 2] = mul_w16<DIR, 2>(b[1 * 4 + 2]);
  b[1 * 4 + 3] = mul_w16<DIR, 3>(b[1 * 4 + 3]);
  b[2 * 4 + 1] = mul_w16<DIR, 2>(b[2 * 4 + 1]);
  b[2 * 4 + 2] = mul_w16<DIR, 4>(b[2 * 4 + 2]);
  b[2 * 4 + 3] = mul_w16<DIR, 6>(b[2 * 4 + 3]);
  b[3 * 4 + 1] = mul_w16<DIR, 3>(b[3 * 4 + 1]);
  b[3 * 4 + 2] = mul_w16<DIR, 6>(b[3 * 4 + 2]);
  b[3 * 4 + 3] = mul_w16<DIR, 9>(b[3 * 4 + 3]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 y0 = b[k1], y1 = b[4 + k1], y2 = b[8 + k1], y3 = b[12 + k1];
    dft4<DIR>(y0, y1, y2, y3);
    a[k1] = y0; a[k1 + 4] = y1; a[k1 + 8] = y2; a[k1 + 12] = y3;
  }
}

template <int DIR> __device__ __forceinline__ void dft3(float2* a) {
  float2 t = cadd(a[1], a[2]);
  float2 d = mul_dir_i<DIR>(cscale(csub(a[1], a[2]), HG_SIN_PI_3));
  float2 m = make_float2(a[0].x - 0.5f * t.x, a[0].y - 0.5f * t.y);
  a[0] = cadd(a[0], t);
  a[1] = cadd(m, d);
  a[2] = csub(m, d);
}

template <int DIR> __device__ __forceinline__ void dft5(float2* a) {
  float2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
  float2 d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
  float2 b1 = make_float2(a[0].x + HG_COS_2PI_5 * t1.x + HG_COS_4PI_5 * t2.x,
                          a[0].y + HG_COS_2PI_5 * t1.y + HG_COS_4PI_5 * t2.y);
  float2 b2 = make_float2(a[0].x + HG_COS_4PI_5 * t1.x + HG_COS_2PI_5 * t2.x,
                          a[0].y + HG_COS_4PI_5 * t1.y + HG_COS_2PI_5 * t2.y);
  float2 e1 = mul_dir_i<DIR>(make_float2(fmaf(HG_SIN_2PI_5, d1.x, HG_SIN_4PI_5 * d2.x),
                                         fmaf(HG_SIN_2PI_5, d1.y, HG_SIN_4PI_5 * d2.y)));
  float2 e2 = mul_dir_i<DIR>(make_float2(fmaf(HG_SIN_4PI_5, d1.x, -(HG_SIN_2PI_5 * d2.x)),
                                         fmaf(HG_SIN_4PI_5, d1.y, -(HG_SIN_2PI_5 * d2.y))));
  a[0] = cadd(a[0], cadd(t1, t2));
  a[1] = cadd(b1, e1);
  a[4] = csub(b1, e1);
  a[2] = cadd(b2, e2);
  a[3] = csub(b2, e2);
}

template <int R, int DIR> __device__ __forceinline__ void dft(float2* a) {
  static_assert(R == 2 || R == 3 || R == 4 || R == 5 || R == 8 || R == 16, "unsupported radix");
  if constexpr (R == 2) dft2<DIR>(a);
  else if constexpr (R == 3) dft3<DIR>(a);
  else if constexpr (R == 4) dft4<DIR>(a);
  else if constexpr (R == 5) dft5<DIR>(a);
  else if constexpr (R == 8) dft8<DIR>(a);
  else dft16<DIR>(a);
}

// ---------------------------------------------------------------------------
// compile-time transform plan
// ---------------------------------------------------------------------------
template <int N_, int T_, int... Rs>
struct Plan {
  static constexpr int N = N_;
  static constexpr int T = T_;
  static constexpr int S = sizeof...(Rs);
  static constexpr int R[S] = {Rs...};

  // radix of stage s when the stages run in forward (REV = false) or reversed order
  static constexpr int radix(int s, bool rev) { return rev ? R[S - 1 - s] : R[s]; }
  static constexpr int ns(int s, bool rev) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= radix(i, rev);
    return p;
  }
  static constexpr int rounds(int s, bool rev) { return (N / radix(s, rev) + T - 1) / T; }
  static constexpr bool full(int s, bool rev) { return (N / radix(s, rev)) % T == 0; }
  static constexpr int regs_() {
    int m = 0;
    for (int s = 0; s < S; ++s) {
      int a = radix(s, false) * rounds(s, false);
      int b = radix(s, true) * rounds(s, true);
      m = a > m ? a : m;
      m = b > m ? b : m;
    }
    return m;
  }
  static constexpr int REGS = regs_();
  static constexpr bool palindrome_() {
    for (int s = 0; s < S; ++s)
      if (R[s] != R[S - 1 - s]) return false;
    return true;
  }
  // reversed order has the same stages, so both directions share twiddles
  static constexpr bool PALINDROME = palindrome_();
  static constexpr int product_() {
    int p = 1;
    for (int s = 0; s < S; ++s) p *= R[s];
    return p;
  }
  static_assert(product_() == N, "radices must multiply to N");
  static_assert(S >= 2, "at least two stages (one LDS exchange) per transform");
  static_assert(T <= 1024, "team too large");
};

// LDS padding: one spare complex slot every 2^PAD_LOG slots keeps the strided
// Stockham writes off a single bank.
constexpr int PAD_LOG = 4;
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> PAD_LOG); }
__host__ __device__ constexpr int lds_len(int n) { return lds_pad(n - 1) + 1; }

// Addressing of one team's LDS region: element i lives at base[lds_pad(i) * MUL].
template <int MUL>
struct LdsView {
  float2* base;
  __device__ __forceinline__ float2& at(int i) const { return base[lds_pad(i) * MUL]; }
  // Distance in float2 elements between at(i) and at(i + d) when d is a
  // multiple of the padding period, or when i and i + d lie in one padding
  // block: then it does not depend on i.
  __host__ __device__ static constexpr int padded_span(int d) {
    return (d % (1 << PAD_LOG) == 0 ? d + (d >> PAD_LOG) : d) * MUL;
  }
};

// Synchronisation between exchange phases.  A team inside one wavefront only
// needs the wavefront's LDS operations ordered; a wider team needs s_barrier.
template <bool WAVE_SYNC> __device__ __forceinline__ void team_sync() {
  if constexpr (WAVE_SYNC) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Register layout of the first stage (LAST = false) or the output of the last
// stage (LAST = true) of a run in the given order: slot m * R + r holds element
// t + m T + r N / R.
template <class P, bool REV, bool LAST> struct Layout {
  static constexpr int s = LAST ? P::S - 1 : 0;
  static constexpr int R = P::radix(s, REV);
  static constexpr int ROUNDS = P::rounds(s, REV);
  static constexpr bool FULL = P::full(s, REV);
  static constexpr int STRIDE = P::N / R;
  __device__ __forceinline__ static bool valid(int t, int m) { return FULL || (t + m * P::T < STRIDE); }
  __device__ __forceinline__ static int index(int t, int m, int r) { return t + m * P::T + r * STRIDE; }
};

// Visit every (register slot, element index) pair of a layout.
template <class L, class F>
__device__ __forceinline__ void for_layout(int t, F&& f) {
#pragma unroll
  for (int m = 0; m < L::ROUNDS; ++m)
#pragma unroll
    for (int r = 0; r < L::R; ++r)
      if (L::valid(t, m)) f(m * L::R + r, L::index(t, m, r));
}

// ---------------------------------------------------------------------------
// per-thread twiddles: stage s needs w^(r k), r = 1..R-1, for the k of each
// butterfly the thread owns; when T is a multiple of Ns all of a thread's
// butterflies in that stage share k.  Register slot i of thread t is read from
// a twiddle image laid out [i][t] (built on the host by twiddle_image), so
// every twiddle load is one unit-stride, coalesced wavefront load; indexing a
// plain exp(-2 pi i m / N) table by r k would be a gather over dozens of cache
// lines per instruction.
// ---------------------------------------------------------------------------
template <class P, bool REV>
struct TwRegs {
  static constexpr int sets(int s) {
    return P::ns(s, REV) == 1 ? 0 : ((P::T % P::ns(s, REV) == 0) ? 1 : P::rounds(s, REV));
  }
  static constexpr int offset(int s) {
    int o = 0;
    for (int i = 0; i < s; ++i) o += sets(i) * (P::radix(i, REV) - 1);
    return o;
  }
  static constexpr int TOTAL = offset(P::S);
  float2 w[TOTAL > 0 ? TOTAL : 1];

  __device__ __forceinline__ void load(const float2* __restrict__ img, int t) {
#pragma unroll
    for (int i = 0; i < TOTAL; ++i) w[i] = img[i * P::T + t];
  }
  __device__ __forceinline__ float2 at(int i, int) const { return w[i]; }
};

// The same twiddle image read from LDS at the point of use (one copy per
// workgroup, shared by all its teams; see stage_compute).
template <class P, bool REV>
struct TwLds {
  static constexpr int sets(int s) { return TwRegs<P, REV>::sets(s); }
  static constexpr int offset(int s) { return TwRegs<P, REV>::offset(s); }
  static constexpr int TOTAL = TwRegs<P, REV>::TOTAL;
  const float2* img;
  __device__ __forceinline__ float2 at(int i, int t) const { return img[i * P::T + t]; }
};

// Host: the twiddle image of order REV, TOTAL * T entries, slot i of thread t
// at [i * T + t]: exp(-2 pi i r k / (Ns R)) evaluated in FP64.
template <class P, bool REV>
void twiddle_image(double* re, double* im) {
  using TW = TwRegs<P, REV>;
  for (int s = 0; s < P::S; ++s) {
    const int R = P::radix(s, REV), NS = P::ns(s, REV);
    for (int set = 0; set < TW::sets(s); ++set)
      for (int r = 1; r < R; ++r)
        for (int t = 0; t < P::T; ++t) {
          const int k = (t + set * P::T) % NS;
          const long long m = (long long)r * k;               // angle = -2 pi m / (NS R)
          const double a = -2.0 * 3.14159265358979323846 * (double)(m % (NS * R)) / (double)(NS * R);
          const int i = TW::offset(s) + set * (R - 1) + r - 1;
          re[i * P::T + t] = __builtin_cos(a);
          im[i * P::T + t] = __builtin_sin(a);
        }
  }
}

// One radix stage in registers: twiddle then R-point DFTs.
template <class P, int S_, bool REV, int DIR, class TW>
__device__ __forceinline__ void stage_compute(float2* v, int t, const TW& tw) {
  constexpr int R = P::radix(S_, REV);
  constexpr int NS = P::ns(S_, REV);
  constexpr int NR = P::N / R;
  constexpr int ROUNDS = P::rounds(S_, REV);
  constexpr bool SHARED = (NS > 1) && (P::T % NS == 0);
  constexpr int OFF = TW::offset(S_);
#pragma unroll
  for (int m = 0; m < ROUNDS; ++m) {
    const int j = t + m * P::T;
    if (P::full(S_, REV) || j < NR) {
      if constexpr (NS > 1) {
        const int set = SHARED ? 0 : m;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 w = tw.at(OFF + set * (R - 1) + r - 1, t);
          v[m * R + r] = DIR < 0 ? cmul(v[m * R + r], w) : cmulconj(v[m * R + r], w);
        }
      }
      dft<R, DIR>(&v[m * R]);
    }
  }
}

// Move stage S_ outputs to the inputs of stage S_+1 through LDS.
template <class P, int S_, bool REV, bool WAVE_SYNC, int MUL>
__device__ __forceinline__ void stage_exchange(float2* v, int t, LdsView<MUL> lds) {
  constexpr int R = P::radix(S_, REV);
  constexpr int NS = P::ns(S_, REV);
  constexpr int NR = P::N / R;
  constexpr int ROUNDS = P::rounds(S_, REV);
  constexpr int R2 = P::radix(S_ + 1, REV);
  constexpr int NR2 = P::N / R2;
  constexpr int ROUNDS2 = P::rounds(S_ + 1, REV);
  // Where the padded distance between two slots does not depend on the
  // thread (strides that are multiples of the padding period, or a run of R
  // inside one padding block), the slots are addressed from one base pointer
  // with constant offsets instead of one padded index each.
  constexpr int PERIOD = 1 << PAD_LOG;
  constexpr bool W_SLOTS = NS % PERIOD == 0 || (NS == 1 && PERIOD % R == 0);
  constexpr bool W_ROUNDS = W_SLOTS && P::T % NS == 0 && (P::T * R) % PERIOD == 0;
  constexpr bool R_SLOTS = NR2 % PERIOD == 0;
  constexpr bool R_ROUNDS = R_SLOTS && P::T % PERIOD == 0;
  using LV = LdsView<MUL>;
  float2* const w0 = W_ROUNDS ? &lds.at((t - t % NS) * R + t % NS) : nullptr;
#pragma unroll
  for (int m = 0; m < ROUNDS; ++m) {
    const int j = t + m * P::T;
    if (P::full(S_, REV) || j < NR) {
      if constexpr (W_ROUNDS) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          w0[LV::padded_span(m * P::T * R) + LV::padded_span(r * NS)] = v[m * R + r];
      } else {
        const int k = j % NS;
        const int base = (j - k) * R + k;
        if constexpr (W_SLOTS) {
          float2* p = &lds.at(base);
#pragma unroll
          for (int r = 0; r < R; ++r) p[LV::padded_span(r * NS)] = v[m * R + r];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) lds.at(base + r * NS) = v[m * R + r];
        }
      }
    }
  }
  team_sync<WAVE_SYNC>();
  const float2* const r0 = R_ROUNDS ? &lds.at(t) : nullptr;
#pragma unroll
  for (int m = 0; m < ROUNDS2; ++m) {
    const int j = t + m * P::T;
    if (P::full(S_ + 1, REV) || j < NR2) {
      if constexpr (R_ROUNDS) {
#pragma unroll
        for (int r = 0; r < R2; ++r) v[m * R2 + r] = r0[LV::padded_span(m * P::T + r * NR2)];
      } else if constexpr (R_SLOTS) {
        const float2* p = &lds.at(j);
#pragma unroll
        for (int r = 0; r < R2; ++r) v[m * R2 + r] = p[LV::padded_span(r * NR2)];
      } else {
#pragma unroll
        for (int r = 0; r < R2; ++r) v[m * R2 + r] = lds.at(j + r * NR2);
      }
    }
  }
  team_sync<WAVE_SYNC>();
}

template <class P, int S_, bool REV, int DIR, bool WAVE_SYNC, int MUL, class TW>
__device__ __forceinline__ void run_from(float2* v, int t, LdsView<MUL> lds, const TW& tw) {
  stage_compute<P, S_, REV, DIR>(v, t, tw);
  if constexpr (S_ + 1 < P::S) {
    stage_exchange<P, S_, REV, WAVE_SYNC, MUL>(v, t, lds);
    run_from<P, S_ + 1, REV, DIR, WAVE_SYNC, MUL>(v, t, lds, tw);
  }
}

// Full transform of the team's sequence.  On entry v holds the first-stage
// layout of order REV, on exit the last-stage layout.  tw must have been
// loaded for order REV (or for either order when the plan is a palindrome).
template <class P, bool REV, int DIR, bool WAVE_SYNC, int MUL, class TW>
__device__ __forceinline__ void fft_run(float2* v, int t, LdsView<MUL> lds, const TW& tw) {
  run_from<P, 0, REV, DIR, WAVE_SYNC, MUL>(v, t, lds, tw);
}

// Twiddle registers for running order REV: the forward set when the plan is a
// palindrome (both orders have identical stages).
template <class P, bool REV>
using TwFor = TwRegs<P, P::PALINDROME ? false : REV>;

// LDS twiddles for order REV (the forward image serves both orders of a palindrome).
template <class P, bool REV>
using TwLdsFor = TwLds<P, P::PALINDROME ? false : REV>;

// Twiddle registers worth holding for a whole transform: up to 16 complex
// values (32 VGPRs), or more while twiddles and data together take at most 40
// complex values (80 VGPRs; e.g. 22 twiddles beside 8 data values at 8192, or
// beside 16 in the 2048-point column pass, whose LDS then holds the data
// alone: OSPR's 2048^2 column pass 23.1 -> 17.0 us).  Larger sets stay in
// LDS and are read at each use, since holding them would push the
// transform's registers into AGPR spills.
constexpr int TW_REG_MAX = 16;
constexpr int TW_DATA_REG_MAX = 40;

// Whether the kernels of plan P that run both transform orders hold their
// twiddles in registers (PassTwiddles with DATA_REGS), so that no LDS is
// reserved for twiddle images at this length.
template <class P>
constexpr bool tw_both_in_regs() {
  constexpr int f = TwRegs<P, false>::TOTAL, r = TwRegs<P, true>::TOTAL;
  return (f <= TW_REG_MAX && r <= TW_REG_MAX) || f + (P::PALINDROME ? 0 : r) + P::REGS <= TW_DATA_REG_MAX;
}

// Full transform of order REV with twiddles from the workgroup's LDS image:
// copied into registers once when the set is small, else read where used.
template <class P, bool REV, int DIR, bool WAVE_SYNC, int MUL>
__device__ __forceinline__ void fft_run_lds_tw(float2* v, int t, LdsView<MUL> lds, const float2* img) {
  if constexpr (TwFor<P, REV>::TOTAL <= TW_REG_MAX) {
    TwFor<P, REV> tw;
    tw.load(img, t);
    fft_run<P, REV, DIR, WAVE_SYNC>(v, t, lds, tw);
  } else {
    fft_run<P, REV, DIR, WAVE_SYNC>(v, t, lds, TwLdsFor<P, REV>{img});
  }
}

// Words of LDS taken by the twiddle images a kernel running both orders needs.
template <class P>
constexpr int tw_lds_len() {
  return TwRegs<P, false>::TOTAL * P::T + (P::PALINDROME ? 0 : TwRegs<P, true>::TOTAL * P::T);
}

// Copy N_ complex values from global memory to LDS with every thread of the
// workgroup (unit stride, coalesced).  Each thread issues its loads in batches
// of 8 before writing any of them, so a batch costs one memory round trip.
// The caller synchronises afterwards.
template <int THREADS, int N_>
__device__ __forceinline__ void lds_fill(float2* dst, const float2* __restrict__ src) {
  constexpr int PER = (N_ + THREADS - 1) / THREADS, B = 8;
#pragma unroll
  for (int b = 0; b < PER; b += B) {
    float2 tmp[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int i = (b + j) * THREADS + (int)threadIdx.x;
      if (b + j < PER && i < N_) tmp[j] = src[i];
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int i = (b + j) * THREADS + (int)threadIdx.x;
      if (b + j < PER && i < N_) dst[i] = tmp[j];
    }
  }
}

// Twiddle images above this many complex words are not copied into LDS: the
// transform reads them from the global image (a few hundred KiB at most,
// resident in L2) where it uses them, leaving the LDS to the data.
constexpr int TW_LDS_MAX_WORDS = 8704;

// Twiddles of one pass kernel for the transform orders it runs (USE_F: the
// forward radix order, USE_R: the reversed one).  When every set it needs
// fits in registers (IN_REGS below), each thread loads its own
// entries from the global twiddle image straight into registers: coalesced
// loads that go out with the kernel's data loads and need neither LDS nor a
// barrier.  Larger sets are copied into the workgroup's LDS at `lds_img`
// (visible after the caller's barrier) and read from there, unless they
// exceed TW_LDS_MAX_WORDS: those are read from the global image itself.
template <class P, int THREADS, bool USE_F, bool USE_R, bool DATA_REGS = true>
struct PassTwiddles {
  static constexpr bool PAL = P::PALINDROME;
  static constexpr bool NEED_F = USE_F || (USE_R && PAL);  // a palindrome runs both orders on the forward set
  static constexpr bool NEED_R = USE_R && !PAL;
  static constexpr int LEN_F = TwRegs<P, false>::TOTAL * P::T;
  static constexpr int LEN_R = TwRegs<P, true>::TOTAL * P::T;
  // every set needed within TW_REG_MAX, or (DATA_REGS: kernels whose other
  // registers leave room) all of them with the data within TW_DATA_REG_MAX
  static constexpr int REG_WORDS = (NEED_F ? TwRegs<P, false>::TOTAL : 0) + (NEED_R ? TwRegs<P, true>::TOTAL : 0);
  static constexpr bool IN_REGS = ((!NEED_F || TwRegs<P, false>::TOTAL <= TW_REG_MAX) &&
                                   (!NEED_R || TwRegs<P, true>::TOTAL <= TW_REG_MAX)) ||
                                  (DATA_REGS && REG_WORDS + P::REGS <= TW_DATA_REG_MAX);
  static constexpr int IMAGE_WORDS = (NEED_F ? LEN_F : 0) + (NEED_R ? LEN_R : 0);
  // Both orders' images: the LDS a launch of this length reserves is sized by
  // the kernels that run both orders, so a kernel running one order must take
  // the global path whenever those do.
  static constexpr int FULL_WORDS = LEN_F + (PAL ? 0 : LEN_R);
  // read at the point of use from the global image (also where the length's
  // other kernels hold their twiddles in registers and reserve no LDS)
  static constexpr bool IN_GLOBAL = !IN_REGS && (FULL_WORDS > TW_LDS_MAX_WORDS || tw_both_in_regs<P>());
  // true when begin() writes LDS and the caller must barrier before run()
  static constexpr bool USES_LDS = !IN_REGS && !IN_GLOBAL;
  // LDS words the twiddles take (0 in register and global modes)
  static constexpr int LDS_WORDS = USES_LDS ? IMAGE_WORDS : 0;

  TwRegs<P, false> f;
  TwRegs<P, true> r;
  const float2* img_f = nullptr;
  const float2* img_r = nullptr;

  __device__ __forceinline__ void begin(const float2* tw, const float2* twr, float2* lds_img, int t) {
    if constexpr (IN_REGS) {
      if constexpr (NEED_F) f.load(tw, t);
      if constexpr (NEED_R) r.load(twr, t);
    } else if constexpr (IN_GLOBAL) {
      img_f = tw;
      img_r = twr;
    } else {
      float2* rimg = lds_img + (NEED_F ? LEN_F : 0);
      if constexpr (NEED_F) lds_fill<THREADS, LEN_F>(lds_img, tw);
      if constexpr (NEED_R) lds_fill<THREADS, LEN_R>(rimg, twr);
      img_f = lds_img;
      img_r = rimg;
    }
  }

  // Full transform of order REV (see fft_run).
  template <bool REV, int DIR, bool WAVE_SYNC, int MUL>
  __device__ __forceinline__ void run(float2* v, int t, LdsView<MUL> lds) const {
    static_assert(REV ? USE_R : USE_F, "order not loaded");
    constexpr bool OWN_R = REV && !PAL;
    if constexpr (IN_REGS) {
      if constexpr (OWN_R) fft_run<P, true, DIR, WAVE_SYNC>(v, t, lds, r);
      else fft_run<P, REV, DIR, WAVE_SYNC>(v, t, lds, f);
    } else {
      fft_run_lds_tw<P, REV, DIR, WAVE_SYNC>(v, t, lds, OWN_R ? img_r : img_f);
    }
  }
};

}  // namespace hg
