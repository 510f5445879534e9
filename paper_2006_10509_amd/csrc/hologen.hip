// Host runtime of libhologen: plan creation (FP64 tables rounded to FP32),
// argument validation, workspace layout and the launch sequences of
// hg_propagate, hg_gs_iterate and hg_ospr.
//
// The plan plays the part of the paper's AlgorithmCuda base object, which
// keeps the problem's images and parameters and the handles to their device
// copies (Sec. 7.3; Sec. 4, Algorithm Interface); here the large images stay
// caller-owned device buffers and the plan keeps only small constant tables.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hologen.h"
#include "reduce.hpp"
#include "search.hpp"

using namespace hg;

namespace {

thread_local hg_status g_last_status = HG_OK;
thread_local std::string g_last_detail;
thread_local std::string g_error_text;

hg_status fail(hg_status s, const std::string& detail) {
  g_last_status = s;
  g_last_detail = detail;
  return s;
}

const char* status_text(hg_status s) {
  switch (s) {
    case HG_OK: return "success";
    case HG_ERR_INVALID_ARGUMENT: return "invalid argument";
    case HG_ERR_UNSUPPORTED_SIZE: return "unsupported transform size";
    case HG_ERR_OUT_OF_MEMORY: return "out of device memory";
    case HG_ERR_DEVICE: return "device error";
    case HG_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

// ---------------------------------------------------------------------------
// per-length kernel tables (each filled in by its own translation unit)
// ---------------------------------------------------------------------------
}  // namespace

#define HG_DECL_ENTRY(N) namespace hg { const LengthEntry* length_entry_##N(); }
HG_FOR_EACH_LENGTH(HG_DECL_ENTRY)

namespace {

#define HG_ENTRY_PTR(N) hg::length_entry_##N(),

const LengthEntry* find_length(int n) {
  static const LengthEntry* const table[] = {HG_FOR_EACH_LENGTH(HG_ENTRY_PTR)};
  for (const LengthEntry* e : table)
    if (e->n == n) return e;
  return nullptr;
}

bool smooth_235(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

template <class K>
hipError_t allow_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

hipError_t prepare_kernels(const LengthEntry* e) {
  hipError_t err = hipSuccess;
  auto chk = [&](hipError_t x) { if (x != hipSuccess && err == hipSuccess) err = x; };
  chk(allow_lds(e->row.prop_fwd, e->row.lds));
  chk(allow_lds(e->row.prop_inv, e->row.lds));
  chk(allow_lds(e->row.gs_start, e->row.lds));
  for (auto& mode : e->row.gs_row)
    for (auto k : mode) chk(allow_lds(k, e->row.lds));
  chk(allow_lds(e->row.gs_row_general, e->row.lds));
  for (auto k : e->row.gs_row_mp) chk(allow_lds(k, e->row.lds));
  chk(allow_lds(e->row.ospr_a, e->row.lds));
  chk(allow_lds(e->row.ospr_c, e->row.lds));
  chk(allow_lds(e->row.ospr_ca, e->row.lds));
  chk(allow_lds(e->row.ospr_c_half, e->row.lds));
  chk(allow_lds(e->row.ospr_ca_half, e->row.lds));
  chk(allow_lds(e->col.prop_fwd, e->col.lds));
  chk(allow_lds(e->col.prop_inv, e->col.lds));
  chk(allow_lds(e->col.gs_col, e->col.lds));
  chk(allow_lds(e->col.gs_col_nmse, e->col.lds));
  chk(allow_lds(e->col.gs_col_win, e->col.lds));
  chk(allow_lds(e->col.gs_col_win_nmse, e->col.lds));
  if (e->col_wide.cols) {
    chk(allow_lds(e->col_wide.gs_col, e->col_wide.lds));
    chk(allow_lds(e->col_wide.gs_col_nmse, e->col_wide.lds));
    chk(allow_lds(e->col_wide.grad_col, e->col_wide.lds));
  }
  chk(allow_lds(e->col.ospr_b, e->col.ospr_lds));
  chk(allow_lds(e->col.ospr_b_pair, e->col.ospr_lds));
  for (auto k : e->row.grad_rows) chk(allow_lds(k, e->row.lds));
  chk(allow_lds(e->col.grad_col, e->col.lds));
  chk(allow_lds(e->row.as_row, e->row.lds));
  chk(allow_lds(e->row.as_row_nmse, e->row.lds));
  chk(allow_lds(e->col.as_fwd, e->col.lds));
  chk(allow_lds(e->col.as_inv, e->col.lds));
  return err;
}

constexpr int kNmseChunk = 128;   // states reduced per k_nmse_reduce launch
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

std::vector<float2> to_f32(const std::vector<double>& re, const std::vector<double>& im) {
  std::vector<float2> out(re.size());
  for (size_t i = 0; i < re.size(); ++i) out[i] = make_float2((float)re[i], (float)im[i]);
  return out;
}

// A twiddle image (FP64 values from the length's kernel table) rounded to FP32.
template <class F>
std::vector<float2> twiddle_table(int len, F&& fill) {
  std::vector<double> re(len > 0 ? len : 1, 1.0), im(len > 0 ? len : 1, 0.0);
  if (len > 0) fill(re.data(), im.data());
  return to_f32(re, im);
}

// 1D quadratic phase exp(i pi ((j - n/2) pitch)^2 / (lambda z)) times `scale`, optionally conjugated.
std::vector<float2> chirp(int n, double pitch, double lambda_z, std::complex<double> scale, bool conj) {
  std::vector<double> re(n), im(n);
  for (int j = 0; j < n; ++j) {
    double c = (double)(j - n / 2) * pitch;
    double ph = M_PI * c * c / lambda_z;
    std::complex<double> v = std::polar(1.0, conj ? -ph : ph) * scale;
    re[j] = v.real();
    im[j] = v.imag();
  }
  return to_f32(re, im);
}

}  // namespace

struct hg_plan_s {
  hg_plan_desc desc;
  const LengthEntry* row;   // kernels for rows (length = width)
  const LengthEntry* col;   // kernels for columns (length = height)
  // twiddle images of the row kernels (length width) and column kernels
  // (length height), forward and reversed radix order
  float2* tw_row[2] = {nullptr, nullptr};
  float2* tw_col[2] = {nullptr, nullptr};
  float2* q1y = nullptr;    // Fresnel source chirp
  float2* q1x = nullptr;
  // Fresnel propagation tables: forward pre = Q1, post = c Q2;
  // inverse pre = conj(Q2)/c, post = conj(Q1)
  float2* fwd_post_y = nullptr;
  float2* fwd_post_x = nullptr;
  float2* inv_pre_y = nullptr;
  float2* inv_pre_x = nullptr;
  float2* inv_post_y = nullptr;
  float2* inv_post_x = nullptr;
  float2* lvl_tab = nullptr;
  float2* as_ty = nullptr;   // angular spectrum: exp(i k z) exp(-i pi lambda z fy^2) [H]
  float2* as_tx = nullptr;   //                   exp(-i pi lambda z fx^2) [W]
  float as_lam2 = 0.f, as_c3 = 0.f, as_inv_hp = 0.f, as_inv_wp = 0.f;
  float2* unit_y = nullptr;  // exp(-2 pi i k / H), k < H: single-pixel replay updates
  float2* unit_x = nullptr;  // exp(-2 pi i k / W), k < W
  int levels = 0;           // quantiser levels used by GS (0 = continuous)
  int row_blocks = 0, col_blocks = 0;
  // batched column configuration: used when wide_ok (W a multiple of its
  // column count, which also divides the field's tile width)
  bool wide_ok = false;
  int col_blocks_wide = 0;
  int ospr_col_blocks = 0;   // workgroups of OSPR's column pass
  int ospr_pair_blocks = 0;  // workgroups of OSPR's pass C over row pairs
  // per-column error partials of one state: the padded width of the widest
  // column configuration
  int col_slots = 0;
  int ft = 0;              // GS-family field layout: 0 row order, else column tile width
  size_t ws_bytes = 0;     // workspace of one hologram (ws_layout(p, 1).total)
  std::vector<void*> allocations;
  // diagnostics: event pairs around launches of one kernel kind
  int timed_kernel = 0;
  int timed_repeats = 1;
  std::vector<hipEvent_t> ev_start, ev_stop;
  size_t ev_used = 0;
  int64_t timed_runs = 0;
  hipError_t ev_error = hipSuccess;
};

namespace {

hg_status upload(hg_plan p, const std::vector<float2>& host, float2** dst) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, host.size() * sizeof(float2));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? HG_ERR_OUT_OF_MEMORY : HG_ERR_DEVICE,
                std::string("hipMalloc of plan table: ") + hipGetErrorString(e));
  }
  p->allocations.push_back(d);
  e = hipMemcpy(d, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(HG_ERR_DEVICE, std::string("hipMemcpy of plan table: ") + hipGetErrorString(e));
  *dst = static_cast<float2*>(d);
  return HG_OK;
}

void free_plan(hg_plan p) {
  for (void* d : p->allocations) (void)hipFree(d);
  for (hipEvent_t e : p->ev_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->ev_stop) (void)hipEventDestroy(e);
  delete p;
}

// Launch helper.  When `kind` is the timed kernel: with one repeat the launch
// goes through hipExtLaunchKernel with a start/stop event pair stamped from
// the dispatch itself; with R > 1 repeats the kernel is launched R times back
// to back between two hipEventRecord calls (see hg_timing_begin).
template <class A>
void launch(hg_plan p, int kind, hipStream_t s, void (*kernel)(A), dim3 blocks, int threads, size_t lds, A& args) {
  if (p->timed_kernel != kind || p->ev_error != hipSuccess) {
    hipLaunchKernelGGL(kernel, blocks, dim3(threads), lds, s, args);
    return;
  }
  if (p->ev_used == p->ev_start.size()) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      p->ev_error = e;
      hipLaunchKernelGGL(kernel, blocks, dim3(threads), lds, s, args);
      return;
    }
    p->ev_start.push_back(a);
    p->ev_stop.push_back(b);
  }
  hipEvent_t a = p->ev_start[p->ev_used], b = p->ev_stop[p->ev_used];
  hipError_t e = hipSuccess;
  if (p->timed_repeats == 1) {
    void* argv[] = {&args};
    e = hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), blocks, dim3(threads), argv, lds, s, a, b, 0);
  } else {
    e = hipEventRecord(a, s);
    for (int r = 0; e == hipSuccess && r < p->timed_repeats; ++r) {
      hipLaunchKernelGGL(kernel, blocks, dim3(threads), lds, s, args);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, s);
  }
  if (e != hipSuccess) {
    p->ev_error = e;
    return;
  }
  ++p->ev_used;
  p->timed_runs += p->timed_repeats;
}

hg_status validate_desc(const hg_plan_desc* d) {
  if (!d) return fail(HG_ERR_INVALID_ARGUMENT, "desc is NULL");
  for (int n : {d->width, d->height}) {
    if (n < 2 || n > 8192) return fail(HG_ERR_INVALID_ARGUMENT, "width/height must be in [2, 8192]");
    if (!smooth_235(n)) return fail(HG_ERR_UNSUPPORTED_SIZE, "width/height must be of the form 2^a 3^b 5^c");
    if (!find_length(n))
      return fail(HG_ERR_UNSUPPORTED_SIZE, "no transform of length " + std::to_string(n) + " is compiled into the library");
  }
  if (d->propagation != HG_FOURIER && d->propagation != HG_FRESNEL && d->propagation != HG_ANGULAR)
    return fail(HG_ERR_INVALID_ARGUMENT, "propagation must be HG_FOURIER, HG_FRESNEL or HG_ANGULAR");
  if (d->propagation == HG_FRESNEL) {
    for (double v : {d->wavelength, d->pixel_pitch, d->distance})
      if (!std::isfinite(v) || !(v > 0.0))
        return fail(HG_ERR_INVALID_ARGUMENT, "Fresnel wavelength, pixel_pitch and distance must be finite and > 0");
  }
  if (d->propagation == HG_ANGULAR) {
    if (!(std::isfinite(d->wavelength) && d->wavelength > 0.0 && std::isfinite(d->pixel_pitch) &&
          d->pixel_pitch > 0.0 && std::isfinite(d->distance)))
      return fail(HG_ERR_INVALID_ARGUMENT,
                  "angular-spectrum wavelength and pixel_pitch must be finite and > 0, distance finite");
    if (!(d->wavelength < std::sqrt(2.0) * d->pixel_pitch))
      return fail(HG_ERR_INVALID_ARGUMENT, "angular spectrum needs pixel_pitch > wavelength / sqrt(2) "
                                           "(no evanescent components on the grid)");
  }
  switch (d->modulation) {
    case HG_PHASE:
      if (d->levels != 0) return fail(HG_ERR_INVALID_ARGUMENT, "levels must be 0 for HG_PHASE");
      break;
    case HG_PHASE_QUANTISED:
      if (d->levels < 2 || d->levels > 256)
        return fail(HG_ERR_INVALID_ARGUMENT, "levels must be in [2, 256] for HG_PHASE_QUANTISED");
      break;
    case HG_BINARY_PHASE:
      if (d->levels != 2) return fail(HG_ERR_INVALID_ARGUMENT, "levels must be 2 for HG_BINARY_PHASE");
      break;
    case HG_AMPLITUDE:
      if (d->levels != 0) return fail(HG_ERR_INVALID_ARGUMENT, "levels must be 0 for HG_AMPLITUDE");
      break;
    default:
      return fail(HG_ERR_INVALID_ARGUMENT,
                  "modulation must be HG_PHASE, HG_PHASE_QUANTISED, HG_BINARY_PHASE or HG_AMPLITUDE");
  }
  return HG_OK;
}

AsTransfer as_transfer(hg_plan p) {
  AsTransfer t{};
  t.ty = p->as_ty;
  t.tx = p->as_tx;
  t.lam2 = p->as_lam2;
  t.c3 = p->as_c3;
  t.inv_hp = p->as_inv_hp;
  t.inv_wp = p->as_inv_wp;
  t.H = p->desc.height;
  t.W = p->desc.width;
  return t;
}

hg_status launch_status(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return HG_OK;
}

// Workspace of `batch` same-shape holograms: fields [batch] complex64 in the
// GS layout |
// Scalars [batch] | stats | NMSE partials [batch][kNmseChunk][workgroups] |
// tiled targets [batch][tiles][H][C].  batch = 1 is the single-call layout.
struct WsLayout {
  size_t sc, stats, partials, target, wpartials, total;
  size_t partial_stride, target_stride;   // floats per batch item
};

// Complex elements of one field in the plan's GS-family layout.
size_t field_elems(hg_plan p) {
  return (size_t)field_width((uint32_t)p->desc.width, (uint32_t)p->ft) * (size_t)p->desc.height;
}

WsLayout ws_layout(hg_plan p, int batch) {
  const size_t n = field_elems(p);
  const int nwg = p->row_blocks > p->col_slots ? p->row_blocks : p->col_slots;
  WsLayout L{};
  L.partial_stride = (size_t)kNmseChunk * nwg;
  L.target_stride = (size_t)p->col_slots * p->desc.height;
  L.sc = align_up((size_t)batch * n * sizeof(float2));
  L.stats = L.sc + align_up((size_t)batch * sizeof(Scalars));
  L.partials = L.stats + align_up((size_t)STATS_MAX_BLOCKS * 3 * sizeof(double));
  L.target = L.partials + align_up((size_t)batch * L.partial_stride * sizeof(float));
  L.wpartials = L.target + align_up((size_t)batch * L.target_stride * sizeof(float));
  // signal window (one hologram): three FP64 sums per column workgroup and state
  L.total = L.wpartials + align_up((size_t)kNmseChunk * 3 * p->col_slots * sizeof(double));
  return L;
}

struct Workspace {
  float2* field;
  Scalars* sc;
  double* stats;
  float* partials;
  float* target;      // target amplitude tiled for the column pass (k_tile_target)
  double* wpartials;  // signal-window error sums
};

Workspace carve(hg_plan p, void* ws, int batch = 1) {
  const WsLayout L = ws_layout(p, batch);
  char* b = static_cast<char*>(ws);
  return {reinterpret_cast<float2*>(b), reinterpret_cast<Scalars*>(b + L.sc),
          reinterpret_cast<double*>(b + L.stats), reinterpret_cast<float*>(b + L.partials),
          reinterpret_cast<float*>(b + L.target), reinterpret_cast<double*>(b + L.wpartials)};
}

size_t npix(hg_plan p) { return (size_t)p->desc.width * (size_t)p->desc.height; }

int stats_blocks(size_t n) {
  size_t b = (n + (size_t)STATS_THREADS * 16 - 1) / ((size_t)STATS_THREADS * 16);
  if (b < 1) b = 1;
  if (b > (size_t)STATS_MAX_BLOCKS) b = STATS_MAX_BLOCKS;
  return (int)b;
}

void enqueue_stats(hg_plan p, const Workspace& w, const float* target, const float* illum, double intensity_sum,
                   Scalars* out, hipStream_t s, const uint8_t* window = nullptr, int unit_target_scale = 0) {
  const size_t n = npix(p);
  const int nb = stats_blocks(n);
  // sum I of a GS state: N_px sum A^2 after the unnormalised FFT2; the
  // angular-spectrum replay pass sees H W times the unitary field, N_px^2 sum A^2
  const double a2_scale = p->desc.propagation == HG_ANGULAR ? (double)n * (double)n : (double)n;
  hipLaunchKernelGGL(k_stats_partial, dim3(nb), dim3(STATS_THREADS), 0, s, target, illum, n, w.stats, window);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(STATS_THREADS), 0, s, (const double*)w.stats, nb, n, illum ? 1 : 0,
                     intensity_sum, a2_scale, out, unit_target_scale);
}

// Column-pass configuration of a GS-family launch over `batch` holograms or
// problems: the batched one (ColCfgWide) when the length has one that fits
// the plan, else the single-hologram one.  Both write the error partials of
// a state per column (slots = padded width) in the same order.
struct ColLaunch {
  void (*gs_col)(GsColArgs);
  void (*gs_col_nmse)(GsColArgs);
  void (*grad_col)(GsColArgs);
  int cols, blocks, threads;
  size_t lds;
  int slots() const { return cols * blocks; }
};

ColLaunch col_launch(hg_plan p, int batch) {
  if (batch > 1 && p->wide_ok) {
    const ColWideKernels& w = p->col->col_wide;
    return {w.gs_col, w.gs_col_nmse, w.grad_col, w.cols, p->col_blocks_wide, w.threads, w.lds};
  }
  const ColKernels& c = p->col->col;
  return {c.gs_col, c.gs_col_nmse, c.grad_col, c.cols, p->col_blocks, c.threads, c.lds};
}

// Workspace of the gradient method for `batch` problems of `planes` replay
// planes each: fields [batch][planes] | Scalars [batch][planes] | stats |
// loss partials [kNmseChunk states][batch][planes][column workgroups] | tiled
// targets [batch][planes].  batch = 1 is the single-problem layout.  The
// fields, scalars, partials and targets of (problem b, plane j) are item
// b planes + j of the column launch over every plane of every problem.
struct GradLayout {
  size_t sc, stats, partials, target, target_stride, total;
  size_t state_stride;     // floats of loss partials per state
};

GradLayout grad_layout(hg_plan p, int planes, int batch = 1) {
  GradLayout g{};
  g.state_stride = (size_t)batch * planes * p->col_slots;
  g.sc = align_up((size_t)batch * planes * field_elems(p) * sizeof(float2));
  g.stats = g.sc + align_up((size_t)batch * planes * sizeof(Scalars));
  g.partials = g.stats + align_up((size_t)STATS_MAX_BLOCKS * 3 * sizeof(double));
  g.target = g.partials + align_up((size_t)kNmseChunk * g.state_stride * sizeof(float));
  g.target_stride = align_up((size_t)p->col_slots * p->desc.height * sizeof(float));
  g.total = g.target + (size_t)batch * planes * g.target_stride;
  return g;
}

// Workspace of multi-plane GS for `batch` problems of `planes` replay planes:
// fields [batch] | Scalars [batch][planes] | stats | NMSE partials
// [batch][kNmseChunk steps][column workgroups] | tiled targets
// [batch][planes].
struct MpLayout {
  size_t sc, stats, partials, target, target_stride, total;
  size_t partial_stride;   // floats of NMSE partials per problem
};

MpLayout mp_layout(hg_plan p, int planes, int batch = 1) {
  MpLayout g{};
  g.partial_stride = (size_t)kNmseChunk * p->col_slots;
  g.sc = align_up((size_t)batch * field_elems(p) * sizeof(float2));
  g.stats = g.sc + align_up((size_t)batch * planes * sizeof(Scalars));
  g.partials = g.stats + align_up((size_t)STATS_MAX_BLOCKS * 3 * sizeof(double));
  g.target = g.partials + align_up((size_t)batch * g.partial_stride * sizeof(float));
  g.target_stride = align_up((size_t)p->col_slots * p->desc.height * sizeof(float));
  g.total = g.target + (size_t)batch * planes * g.target_stride;
  return g;
}

constexpr int kMaxPlanes = 16;

hg_status validate_planes(const hg_plan* planes, int n_planes) {
  if (!planes) return fail(HG_ERR_INVALID_ARGUMENT, "planes is NULL");
  if (n_planes < 1 || n_planes > kMaxPlanes) return fail(HG_ERR_INVALID_ARGUMENT, "n_planes must be in 1..16");
  for (int j = 0; j < n_planes; ++j) {
    if (!planes[j]) return fail(HG_ERR_INVALID_ARGUMENT, "planes[" + std::to_string(j) + "] is NULL");
    if (planes[j]->desc.propagation == HG_ANGULAR)
      return fail(HG_ERR_INVALID_ARGUMENT, "planes must be HG_FOURIER or HG_FRESNEL plans");
    if (planes[j]->desc.width != planes[0]->desc.width || planes[j]->desc.height != planes[0]->desc.height)
      return fail(HG_ERR_INVALID_ARGUMENT, "all planes must have the same width and height");
  }
  return HG_OK;
}

// One gradient evaluation per step for `steps` steps (Adam when m != null),
// then, when final_loss, the loss of the state the last step leaves.
// loss[k] receives the summed NMSE of state k (nullable).
// `batch` problems side by side (grid.y = problem): problem b uses
// target_amp + b P H W, phase / grad / m / v + b H W and loss + b loss_stride,
// and its arithmetic is exactly that of a single-problem call.  A state is
// one column launch over every plane of every problem (item b P + j) and one
// row pass over every problem that handles all its planes.
hg_status grad_run(const hg_plan* planes, int P, int batch, const float* target_amp, float* phase, float* grad,
                   float* m, float* v, int steps, int first_step, float lr, float beta1, float beta2, float eps,
                   float* loss, size_t loss_stride, bool final_loss, void* workspace, hipStream_t stream) {
  hg_plan p0 = planes[0];
  const int W = p0->desc.width, H = p0->desc.height;
  const size_t n = npix(p0);
  const int items = batch * P;
  const GradLayout L = grad_layout(p0, P, batch);
  char* ws = static_cast<char*>(workspace);
  float2* field = reinterpret_cast<float2*>(ws);
  Scalars* sc = reinterpret_cast<Scalars*>(ws + L.sc);
  double* stats = reinterpret_cast<double*>(ws + L.stats);
  float* partials = reinterpret_cast<float*>(ws + L.partials);
  const RowKernels& rk = p0->row->row;
  const ColLaunch cl = col_launch(p0, items);
  const int cols = cl.cols;
  const uint32_t tiled_n = (uint32_t)cl.slots() * H;
  const int nb = stats_blocks(n);
  for (int i = 0; i < items; ++i) {
    const float* ti = target_amp + (size_t)i * n;
    float* tiled = reinterpret_cast<float*>(ws + L.target + (size_t)i * L.target_stride);
    hipLaunchKernelGGL(k_tile_target, dim3((tiled_n + 255) / 256), dim3(256), 0, stream, ti, tiled, H, W, cols,
                       tiled_n);
    hipLaunchKernelGGL(k_stats_partial, dim3(nb), dim3(STATS_THREADS), 0, stream, ti, (const float*)nullptr, n,
                       stats);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(STATS_THREADS), 0, stream, (const double*)stats, nb, n, 0,
                       (double)n * (double)n, (double)n, sc + i);
  }
  const dim3 rows(p0->row_blocks, batch), tiles(cl.blocks, items);
  GsColArgs ca{};
  ca.ft = p0->ft;
  ca.field = field;
  ca.W = W;
  ca.H = H;
  ca.tw = p0->tw_col[0];
  ca.twr = p0->tw_col[1];
  ca.px = (uint32_t)field_elems(p0);
  ca.target = reinterpret_cast<const float*>(ws + L.target);
  ca.target_stride = (uint32_t)(L.target_stride / sizeof(float));
  ca.sc = sc;
  ca.sc_stride = 1;
  ca.partial_stride = (uint32_t)cl.slots();
  GradRowArgs ga{};
  ga.px = (uint32_t)n;
  ga.fpx = (uint32_t)field_elems(p0);
  ga.ft = p0->ft;
  ga.field = field;
  ga.phase = phase;
  ga.H = H;
  ga.planes = P;
  for (int j = 0; j < P; ++j) {
    const bool fres = planes[j]->desc.propagation == HG_FRESNEL;
    ga.q1y[j] = fres ? planes[j]->q1y : nullptr;
    ga.q1x[j] = fres ? planes[j]->q1x : nullptr;
  }
  ga.grad_out = grad;
  ga.m = m;
  ga.v = v;
  ga.lr = lr;
  ga.beta1 = beta1;
  ga.beta2 = beta2;
  ga.eps = eps;
  ga.tw = p0->tw_row[0];
  ga.twr = p0->tw_row[1];
  const bool backward = grad || m;
  const int states = steps + (final_loss ? 1 : 0);
  hipLaunchKernelGGL(rk.grad_rows[GRAD_START], rows, dim3(rk.threads), rk.lds, stream, ga);
  int chunk0 = 0;
  for (int k = 0; k < states; ++k) {
    const bool is_step = k < steps;
    ca.partials = loss ? partials + (size_t)(k - chunk0) * L.state_stride : nullptr;
    if (is_step && backward) {
      if (m) {
        const int t = first_step + k;
        ga.bc1 = (float)(1.0 - std::pow((double)beta1, (double)t));
        ga.bc2 = (float)(1.0 - std::pow((double)beta2, (double)t));
      }
      hipLaunchKernelGGL(cl.grad_col, tiles, dim3(cl.threads), cl.lds, stream, ca);
      // the next state's forward evaluation (from the phase this pass leaves)
      // runs in the same pass when another state follows
      const int mode = k + 1 < states ? GRAD_ADJ_NEXT : GRAD_ADJ;
      hipLaunchKernelGGL(rk.grad_rows[mode], rows, dim3(rk.threads), rk.lds, stream, ga);
    } else if (loss) {
      hipLaunchKernelGGL(cl.gs_col_nmse, tiles, dim3(cl.threads), cl.lds, stream, ca);
    }
    if (loss && (k - chunk0 == kNmseChunk - 1 || k == states - 1)) {
      hipLaunchKernelGGL(k_loss_reduce, dim3(k - chunk0 + 1, batch), dim3(STATS_THREADS), 0, stream,
                         (const float*)partials, cl.slots(), P, (const Scalars*)sc, loss + chunk0,
                         (size_t)P * cl.slots(), L.state_stride, loss_stride);
      chunk0 = k + 1;
    }
  }
  return launch_status("gradient launch");
}

// Gerchberg-Saxton on the angular-spectrum model (one hologram).  Four passes
// per iteration: column FFT * T inverse column FFT; replay row pass (inverse
// row FFT -> NMSE, T R / |R| -> row FFT); column FFT * conj T inverse column
// FFT; SLM row pass (the Fourier-type GS row pass).
hg_status gs_run_angular(hg_plan p, const float* target_amp, const float* illumination, float* phase,
                         uint8_t* levels, float* nmse, int32_t iterations, void* workspace, hipStream_t stream) {
  const int W = p->desc.width, H = p->desc.height;
  Workspace w = carve(p, workspace, 1);
  const RowKernels& rk = p->row->row;
  const ColKernels& ck = p->col->col;
  GsRowArgs ra{};
  ra.ft = p->ft;
  ra.field = w.field;
  ra.illum = illumination;
  ra.H = H;
  ra.slm.lvl_tab = p->lvl_tab;
  ra.slm.levels = p->levels;
  ra.slm.inv_delta = p->levels ? (float)((double)p->levels / (2.0 * M_PI)) : 0.0f;
  ra.slm.inv_delta_f64 = p->levels ? (double)p->levels / (2.0 * M_PI) : 0.0;
  ra.slm.half_step = p->levels ? make_float2((float)std::cos(M_PI / p->levels), (float)std::sin(M_PI / p->levels))
                               : make_float2(1.0f, 0.0f);
  ra.tw = p->tw_row[0];
  ra.twr = p->tw_row[1];
  AsColArgs ca{};
  ca.ft = p->ft;
  ca.io = w.field;
  ca.W = W;
  ca.tr = as_transfer(p);
  ca.scale = 1.0f;
  ca.tw = p->tw_col[0];
  ca.twr = p->tw_col[1];
  AsRowArgs xa{};
  xa.ft = p->ft;
  xa.field = w.field;
  xa.H = H;
  xa.target = target_amp;
  xa.sc = w.sc;
  xa.tw = p->tw_row[0];
  xa.twr = p->tw_row[1];
  const int mode = p->levels == 0 ? GS_CONT
                 : (p->levels == 2 || p->levels == 4 || p->levels == 8) ? p->levels : GS_QATAN;
  void (*gs_row_hot)(GsRowArgs) = rk.gs_row[gs_mode_index(mode)][0];
  if (nmse) enqueue_stats(p, w, target_amp, illumination, 0.0, w.sc, stream);
  const dim3 rows(p->row_blocks), tiles(p->col_blocks);
  ra.phase0 = phase;
  ra.phase_out = iterations == 0 ? phase : nullptr;
  ra.levels_out = iterations == 0 ? levels : nullptr;
  hipLaunchKernelGGL(rk.gs_start, rows, dim3(rk.threads), rk.lds, stream, ra);
  int chunk0 = 0;
  for (int k = 0; k <= iterations; ++k) {
    const bool last = k == iterations;
    if (last && !nmse) break;
    hipLaunchKernelGGL(ck.as_fwd, tiles, dim3(ck.threads), ck.lds, stream, ca);
    xa.partials = nmse ? w.partials + (size_t)(k - chunk0) * p->row_blocks : nullptr;
    hipLaunchKernelGGL(last ? rk.as_row_nmse : rk.as_row, rows, dim3(rk.threads), rk.lds, stream, xa);
    if (nmse && (k - chunk0 == kNmseChunk - 1 || last)) {
      hipLaunchKernelGGL(k_nmse_reduce, dim3(k - chunk0 + 1, 1), dim3(STATS_THREADS), 0, stream,
                         (const float*)w.partials, p->row_blocks, (const Scalars*)w.sc, nmse + chunk0, (size_t)0,
                         (size_t)0);
      chunk0 = k + 1;
    }
    if (last) break;
    hipLaunchKernelGGL(ck.as_inv, tiles, dim3(ck.threads), ck.lds, stream, ca);
    ra.phase_out = k == iterations - 1 ? phase : nullptr;
    ra.levels_out = k == iterations - 1 ? levels : nullptr;
    void (*gs_row)(GsRowArgs) = (illumination || ra.phase_out) ? rk.gs_row_general : gs_row_hot;
    hipLaunchKernelGGL(gs_row, rows, dim3(rk.threads), rk.lds, stream, ra);
  }
  return launch_status("hg_gs_iterate launch");
}

// Gerchberg-Saxton on `batch` same-shape holograms stacked along the slowest
// axis (batch = 1: one hologram).  Every pass is one launch over all items
// (grid.y = batch item), so a batch of small holograms fills the GPU.
hg_status gs_run(hg_plan p, int batch, const float* target_amp, const float* illumination, float* phase,
                 uint8_t* levels, float* nmse, int32_t iterations, void* workspace, hipStream_t stream,
                 const uint8_t* window = nullptr) {
  const int W = p->desc.width, H = p->desc.height;
  const size_t n = npix(p);
  const WsLayout L = ws_layout(p, batch);
  Workspace w = carve(p, workspace, batch);
  const RowKernels& rk = p->row->row;
  const ColKernels& ck = p->col->col;

  GsRowArgs ra{};
  ra.ft = p->ft;
  ra.field = w.field;
  ra.illum = illumination;
  ra.H = H;
  ra.px = (uint32_t)n;
  ra.fpx = (uint32_t)field_elems(p);
  if (p->desc.propagation == HG_FRESNEL) {
    ra.q1y = p->q1y;
    ra.q1x = p->q1x;
  }
  ra.slm.lvl_tab = p->lvl_tab;
  ra.slm.levels = p->levels;
  ra.slm.inv_delta = p->levels ? (float)((double)p->levels / (2.0 * M_PI)) : 0.0f;
  ra.slm.inv_delta_f64 = p->levels ? (double)p->levels / (2.0 * M_PI) : 0.0;
  ra.slm.half_step = p->levels ? make_float2((float)std::cos(M_PI / p->levels), (float)std::sin(M_PI / p->levels))
                               : make_float2(1.0f, 0.0f);
  ra.tw = p->tw_row[0];
  ra.twr = p->tw_row[1];
  // amplitude-only SLM: its field energy changes between states, so the
  // error comes from the exact three-sum column pass (the windowed one, with
  // every pixel inside and the target imposed as given)
  const bool amplitude = p->desc.modulation == HG_AMPLITUDE;
  ra.slm.amplitude = amplitude ? 1 : 0;
  ra.slm.amp_scale = (float)(1.0 / (double)n);
  const bool exact = window != nullptr || amplitude;

  const ColLaunch cl = col_launch(p, exact ? 1 : batch);
  const int cols = cl.cols;
  const uint32_t tiled_n = (uint32_t)cl.slots() * H;
  for (int b = 0; b < batch; ++b)
    hipLaunchKernelGGL(k_tile_target, dim3((tiled_n + 255) / 256), dim3(256), 0, stream, target_amp + (size_t)b * n,
                       w.target + (size_t)b * L.target_stride, H, W, cols, tiled_n, window);

  GsColArgs ca{};
  ca.ft = p->ft;
  ca.field = w.field;
  ca.W = W;
  ca.H = H;
  ca.target = w.target;
  ca.sc = w.sc;
  ca.tw = p->tw_col[0];
  ca.twr = p->tw_col[1];
  ca.px = (uint32_t)field_elems(p);
  ca.target_stride = (uint32_t)L.target_stride;
  ca.sc_stride = 1;
  ca.partial_stride = (uint32_t)L.partial_stride;

  const int mode = amplitude ? GS_AMP : p->levels == 0 ? GS_CONT
                 : (p->levels == 2 || p->levels == 4 || p->levels == 8) ? p->levels : GS_QATAN;
  // steady-state kernel unless the pass needs illumination or produces outputs
  void (*gs_row_hot)(GsRowArgs) = rk.gs_row[gs_mode_index(mode)][p->desc.propagation == HG_FRESNEL ? 1 : 0];

  // a window needs its target scale even without the error trace
  if (nmse || exact)
    for (int b = 0; b < batch; ++b)
      enqueue_stats(p, w, target_amp + (size_t)b * n, illumination, 0.0, w.sc + b, stream, window,
                    amplitude ? 1 : 0);
  void (*col_hot)(GsColArgs) = exact ? ck.gs_col_win : cl.gs_col;
  void (*col_last)(GsColArgs) = exact ? ck.gs_col_win_nmse : cl.gs_col_nmse;

  const dim3 rows(p->row_blocks, batch), tiles(cl.blocks, batch);
  ra.phase0 = phase;
  ra.phase_out = iterations == 0 ? phase : nullptr;
  ra.levels_out = iterations == 0 ? levels : nullptr;
  hipLaunchKernelGGL(rk.gs_start, rows, dim3(rk.threads), rk.lds, stream, ra);

  int chunk0 = 0;  // first state of the pending reduction chunk
  for (int k = 0; k <= iterations; ++k) {
    const bool last = k == iterations;
    if (last && !nmse) break;
    ca.partials = (nmse && !exact) ? w.partials + (size_t)(k - chunk0) * cl.slots() : nullptr;
    ca.wpartials = (nmse && exact) ? w.wpartials + (size_t)(k - chunk0) * 3 * cl.slots() : nullptr;
    if (last) {
      hipLaunchKernelGGL(col_last, tiles, dim3(cl.threads), cl.lds, stream, ca);
    } else {
      launch(p, HG_KERNEL_GS_REPLAY, stream, col_hot, tiles, cl.threads, cl.lds, ca);
    }
    if (nmse && (k - chunk0 == kNmseChunk - 1 || last)) {
      if (exact)
        hipLaunchKernelGGL(k_window_nmse_reduce, dim3(k - chunk0 + 1), dim3(STATS_THREADS), 0, stream,
                           (const double*)w.wpartials, cl.slots(), (const Scalars*)w.sc, n, nmse + chunk0);
      else
        hipLaunchKernelGGL(k_nmse_reduce, dim3(k - chunk0 + 1, batch), dim3(STATS_THREADS), 0, stream,
                           (const float*)w.partials, cl.slots(), (const Scalars*)w.sc, nmse + chunk0,
                           L.partial_stride, (size_t)iterations + 1);
      chunk0 = k + 1;
    }
    if (last) break;
    ra.phase_out = k == iterations - 1 ? phase : nullptr;
    ra.levels_out = k == iterations - 1 ? levels : nullptr;
    void (*gs_row)(GsRowArgs) = (illumination || ra.phase_out) ? rk.gs_row_general : gs_row_hot;
    launch(p, HG_KERNEL_GS_SLM, stream, gs_row, rows, rk.threads, rk.lds, ra);
  }
  return launch_status("hg_gs_iterate launch");
}

// Workspace of hg_gs_iterate_noalloc: one static array per device, so that
// the call needs no allocation.  In host code `scratch` names a host-side
// stand-in, never the device array: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address reaches kernels.
static __device__ __align__(256) unsigned char scratch[HG_NOALLOC_WORKSPACE_MAX];

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Device address of the current device's scratch array (nullptr and a status
// on failure).
hg_status device_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HG_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(HG_ERR_DEVICE, "device index out of range");
  std::call_once(g_scratch_once[dev], [dev] {
    void* ptr = nullptr;
    const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = err;
    g_scratch_ptr[dev] = err == hipSuccess ? ptr : nullptr;
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
    return fail(HG_ERR_DEVICE, std::string("hipGetSymbolAddress of the static workspace: ") +
                                   hipGetErrorString(g_scratch_err[dev]));
  *out = g_scratch_ptr[dev];
  return HG_OK;
}

hg_status gs_validate(hg_plan p, const float* target_amp, const float* phase, int32_t iterations, void* workspace) {
  if (!p) return fail(HG_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (!target_amp) return fail(HG_ERR_INVALID_ARGUMENT, "target_amp is NULL");
  if (!phase) return fail(HG_ERR_INVALID_ARGUMENT, "phase is NULL");
  if (!workspace) return fail(HG_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (iterations < 0) return fail(HG_ERR_INVALID_ARGUMENT, "iterations must be >= 0");
  return HG_OK;
}

// Multi-plane GS on `batch` same-shape problems (batch 1: hg_gs_multiplane).
// Problem b takes target_amp + b P N, phase and levels + b N and nmse + b (P
// iterations + P); its field, Scalars, partial sums and tiled targets lie at
// the item strides of mp_layout, and every pass is one launch over all
// problems (gridDim.y), with the wide column configuration where there is one.
hg_status multiplane_run(const hg_plan* planes, int32_t n_planes, int32_t batch, const float* target_amp,
                         const float* illumination, float* phase, uint8_t* levels, float* nmse, int32_t iterations,
                         void* workspace, hipStream_t stream, const char* what) {
  hg_status st = validate_planes(planes, n_planes);
  if (st != HG_OK) return st;
  st = gs_validate(planes[0], target_amp, phase, iterations, workspace);
  if (st != HG_OK) return st;
  if (batch < 1 || batch > 65535) return fail(HG_ERR_INVALID_ARGUMENT, "batch must be in 1..65535");
  if ((size_t)batch * field_elems(planes[0]) > (size_t)UINT32_MAX)
    return fail(HG_ERR_INVALID_ARGUMENT, "batch * height * (padded) width must be below 2^32");
  for (int j = 1; j < n_planes; ++j)
    if (planes[j]->desc.modulation != planes[0]->desc.modulation || planes[j]->levels != planes[0]->levels)
      return fail(HG_ERR_INVALID_ARGUMENT, "all planes must have the same modulation and levels");
  if (planes[0]->desc.modulation == HG_AMPLITUDE)
    return fail(HG_ERR_INVALID_ARGUMENT, std::string(what) + " takes phase-only plans");
  const int P = n_planes;
  hg_plan p0 = planes[0];
  const int W = p0->desc.width, H = p0->desc.height;
  const size_t n = npix(p0);
  const MpLayout L = mp_layout(p0, P, batch);
  char* ws = static_cast<char*>(workspace);
  float2* field = reinterpret_cast<float2*>(ws);
  Scalars* sc = reinterpret_cast<Scalars*>(ws + L.sc);
  double* stats = reinterpret_cast<double*>(ws + L.stats);
  float* partials = reinterpret_cast<float*>(ws + L.partials);
  const RowKernels& rk = p0->row->row;
  const ColLaunch cl = col_launch(p0, batch);
  const int slots = cl.slots();   // per-column error partials of one step
  const uint32_t tiled_n = (uint32_t)slots * H;
  const int nb = stats_blocks(n);
  const size_t steps_total = (size_t)iterations * P + P;   // nmse entries per problem
  for (int b = 0; b < batch; ++b)
    for (int j = 0; j < P; ++j) {
      const float* tj = target_amp + ((size_t)b * P + j) * n;
      float* tiled = reinterpret_cast<float*>(ws + L.target + ((size_t)b * P + j) * L.target_stride);
      hipLaunchKernelGGL(k_tile_target, dim3((tiled_n + 255) / 256), dim3(256), 0, stream, tj, tiled, H, W, cl.cols,
                         tiled_n);
      if (nmse) {
        hipLaunchKernelGGL(k_stats_partial, dim3(nb), dim3(STATS_THREADS), 0, stream, tj, illumination, n, stats);
        hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(STATS_THREADS), 0, stream, (const double*)stats, nb, n,
                           illumination ? 1 : 0, 0.0, (double)n, sc + (size_t)b * P + j);
      }
    }
  auto chirp_of = [&](int j, const float2*& qy, const float2*& qx) {
    const bool fres = planes[j]->desc.propagation == HG_FRESNEL;
    qy = fres ? planes[j]->q1y : nullptr;
    qx = fres ? planes[j]->q1x : nullptr;
  };
  GsRowArgs ra{};
  ra.ft = p0->ft;
  ra.field = field;
  ra.illum = illumination;
  ra.H = H;
  ra.px = (uint32_t)n;
  ra.fpx = (uint32_t)field_elems(p0);
  ra.slm.lvl_tab = p0->lvl_tab;
  ra.slm.levels = p0->levels;
  ra.slm.inv_delta = p0->levels ? (float)((double)p0->levels / (2.0 * M_PI)) : 0.0f;
  ra.slm.inv_delta_f64 = p0->levels ? (double)p0->levels / (2.0 * M_PI) : 0.0;
  ra.slm.half_step = p0->levels ? make_float2((float)std::cos(M_PI / p0->levels), (float)std::sin(M_PI / p0->levels))
                                : make_float2(1.0f, 0.0f);
  ra.tw = p0->tw_row[0];
  ra.twr = p0->tw_row[1];
  GsColArgs ca{};
  ca.ft = p0->ft;
  ca.field = field;
  ca.W = W;
  ca.H = H;
  ca.tw = p0->tw_col[0];
  ca.twr = p0->tw_col[1];
  ca.px = (uint32_t)field_elems(p0);
  ca.target_stride = (uint32_t)((size_t)P * L.target_stride / sizeof(float));
  ca.sc_stride = (uint32_t)P;
  ca.partial_stride = (uint32_t)L.partial_stride;
  const dim3 rows(p0->row_blocks, batch), tiles(cl.blocks, batch);
  const int mp_mode = gs_mode_index(p0->levels == 0 ? GS_CONT
                                    : (p0->levels == 2 || p0->levels == 4 || p0->levels == 8) ? p0->levels
                                                                                                : GS_QATAN);

  chirp_of(0, ra.q1y, ra.q1x);
  ra.phase0 = phase;
  ra.phase_out = iterations == 0 ? phase : nullptr;
  ra.levels_out = iterations == 0 ? levels : nullptr;
  hipLaunchKernelGGL(rk.gs_start, rows, dim3(rk.threads), rk.lds, stream, ra);
  const int steps = iterations * P;
  int chunk0 = 0;
  auto flush = [&](int upto) {   // reduce the partials of steps chunk0..upto
    hipLaunchKernelGGL(k_nmse_reduce_planes, dim3(upto - chunk0 + 1, batch), dim3(STATS_THREADS), 0, stream,
                       (const float*)partials, slots, (const Scalars*)sc, P, chunk0, nmse + chunk0,
                       L.partial_stride, steps_total);
    chunk0 = upto + 1;
  };
  for (int s = 0; s < steps; ++s) {
    const int j = s % P;
    ca.target = reinterpret_cast<const float*>(ws + L.target + (size_t)j * L.target_stride);
    ca.sc = sc + j;
    ca.partials = nmse ? partials + (size_t)(s - chunk0) * slots : nullptr;
    hipLaunchKernelGGL(cl.gs_col, tiles, dim3(cl.threads), cl.lds, stream, ca);
    if (nmse && s - chunk0 == kNmseChunk - 1) flush(s);
    chirp_of(j, ra.q1y, ra.q1x);
    ra.q_out_set = 1;
    chirp_of((j + 1) % P, ra.qoy, ra.qox);
    ra.phase_out = s == steps - 1 ? phase : nullptr;
    ra.levels_out = s == steps - 1 ? levels : nullptr;
    // steady-state variant unless the step needs illumination or produces outputs
    void (*row)(GsRowArgs) =
        (illumination || ra.phase_out || ra.levels_out) ? rk.gs_row_general : rk.gs_row_mp[mp_mode];
    hipLaunchKernelGGL(row, rows, dim3(rk.threads), rk.lds, stream, ra);
  }
  if (nmse) {
    // the final state at every plane: its start pass for that plane's chirp, then an NMSE-only pass
    GsRowArgs fa = ra;
    fa.q_out_set = 0;
    fa.phase0 = phase;
    fa.phase_out = nullptr;
    fa.levels_out = nullptr;
    for (int j = 0; j < P; ++j) {
      const int s = steps + j;
      chirp_of(j, fa.q1y, fa.q1x);
      hipLaunchKernelGGL(rk.gs_start, rows, dim3(rk.threads), rk.lds, stream, fa);
      ca.target = reinterpret_cast<const float*>(ws + L.target + (size_t)j * L.target_stride);
      ca.sc = sc + j;
      ca.partials = partials + (size_t)(s - chunk0) * slots;
      hipLaunchKernelGGL(cl.gs_col_nmse, tiles, dim3(cl.threads), cl.lds, stream, ca);
      if (s - chunk0 == kNmseChunk - 1 || j == P - 1) flush(s);
    }
  }
  return launch_status((std::string(what) + " launch").c_str());
}

}  // namespace

// ===========================================================================
// C ABI (the only symbols the library exports)
// ===========================================================================
#pragma GCC visibility push(default)
extern "C" {

const char* hg_error(hg_status s) {
  g_error_text = status_text(s);
  if (s != HG_OK && s == g_last_status && !g_last_detail.empty()) g_error_text += ": " + g_last_detail;
  return g_error_text.c_str();
}

int32_t hg_length_supported(int32_t n) { return find_length(n) ? 1 : 0; }

hg_status hg_plan_create(const hg_plan_desc* desc, hg_plan* out) {
  if (!out) return fail(HG_ERR_INVALID_ARGUMENT, "out is NULL");
  hg_status st = validate_desc(desc);
  if (st != HG_OK) return st;
  st = HG_OK;
  hg_plan p = new hg_plan_s();
  p->desc = *desc;
  const int W = desc->width, H = desc->height;
  p->row = find_length(W);
  p->col = find_length(H);
  hipError_t e = prepare_kernels(p->row);
  if (e == hipSuccess) e = prepare_kernels(p->col);
  if (e != hipSuccess) {
    free_plan(p);
    return fail(HG_ERR_DEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  }
  for (int rev = 0; rev < 2 && st == HG_OK; ++rev) {
    st = upload(p, twiddle_table(p->row->row_tw_len[rev], [&](double* re, double* im) { p->row->row_tw(rev, re, im); }),
                &p->tw_row[rev]);
    if (st == HG_OK)
      st = upload(p, twiddle_table(p->col->col_tw_len[rev], [&](double* re, double* im) { p->col->col_tw(rev, re, im); }),
                  &p->tw_col[rev]);
  }
  if (st == HG_OK && desc->propagation == HG_FRESNEL) {
    const double lz = desc->wavelength * desc->distance;
    const double pitch = desc->pixel_pitch;
    const double py_out = lz / ((double)H * pitch), px_out = lz / ((double)W * pitch);
    const double kz = 2.0 * M_PI * std::fmod(desc->distance / desc->wavelength, 1.0);
    const std::complex<double> pref = std::polar(1.0, kz) / std::complex<double>(0.0, lz) * (pitch * pitch);
    const std::complex<double> one(1.0, 0.0);
    st = upload(p, chirp(H, pitch, lz, one, false), &p->q1y);
    if (st == HG_OK) st = upload(p, chirp(W, pitch, lz, one, false), &p->q1x);
    if (st == HG_OK) st = upload(p, chirp(H, py_out, lz, pref, false), &p->fwd_post_y);
    if (st == HG_OK) st = upload(p, chirp(W, px_out, lz, one, false), &p->fwd_post_x);
    if (st == HG_OK) st = upload(p, chirp(H, py_out, lz, one / pref, true), &p->inv_pre_y);
    if (st == HG_OK) st = upload(p, chirp(W, px_out, lz, one, true), &p->inv_pre_x);
    if (st == HG_OK) st = upload(p, chirp(H, pitch, lz, one, true), &p->inv_post_y);
    if (st == HG_OK) st = upload(p, chirp(W, pitch, lz, one, true), &p->inv_post_x);
  }
  if (desc->modulation == HG_PHASE_QUANTISED || desc->modulation == HG_BINARY_PHASE) {
    p->levels = desc->levels;
    if (st == HG_OK) {
      std::vector<double> re(p->levels), im(p->levels);
      for (int l = 0; l < p->levels; ++l) {
        re[l] = std::cos(2.0 * M_PI * l / p->levels);
        im[l] = std::sin(2.0 * M_PI * l / p->levels);
      }
      st = upload(p, to_f32(re, im), &p->lvl_tab);
    }
  }
  if (st == HG_OK && desc->propagation == HG_ANGULAR) {
    const double lam = desc->wavelength, pitch = desc->pixel_pitch, z = desc->distance;
    const double kz = 2.0 * M_PI * std::fmod(z / lam, 1.0);
    for (int axis = 0; axis < 2 && st == HG_OK; ++axis) {
      const int m = axis == 0 ? H : W;
      std::vector<double> re(m), im(m);
      for (int k = 0; k < m; ++k) {
        const double f = (double)(k < (m + 1) / 2 ? k : k - m) / ((double)m * pitch);
        const double ph = std::fmod(-M_PI * lam * z * f * f, 2.0 * M_PI) + (axis == 0 ? kz : 0.0);
        re[k] = std::cos(ph);
        im[k] = std::sin(ph);
      }
      st = upload(p, to_f32(re, im), axis == 0 ? &p->as_ty : &p->as_tx);
    }
    p->as_lam2 = (float)(lam * lam);
    p->as_c3 = (float)(M_PI * lam * lam * lam * z);
    p->as_inv_hp = (float)(1.0 / ((double)H * pitch));
    p->as_inv_wp = (float)(1.0 / ((double)W * pitch));
  }
  for (int axis = 0; axis < 2 && st == HG_OK; ++axis) {
    const int m = axis == 0 ? H : W;
    std::vector<double> re(m), im(m);
    for (int k = 0; k < m; ++k) {
      re[k] = std::cos(2.0 * M_PI * k / m);
      im[k] = -std::sin(2.0 * M_PI * k / m);
    }
    st = upload(p, to_f32(re, im), axis == 0 ? &p->unit_y : &p->unit_x);
  }
  if (st != HG_OK) {
    free_plan(p);
    return st;
  }
  p->row_blocks = (H + p->row->row.teams - 1) / p->row->row.teams;
  p->col_blocks = (W + p->col->col.cols - 1) / p->col->col.cols;
  p->ospr_col_blocks = (W + p->col->col.ospr_cols - 1) / p->col->col.ospr_cols;
  p->ospr_pair_blocks = (H / 2 + 1 + p->row->row.teams - 1) / p->row->row.teams;
  // Tiled where the row kernels are compiled for a tile width that the column
  // passes' widths divide (whole-line accesses on both passes); row order
  // elsewhere.
  p->ft = p->row->row.ft != 0 && p->row->row.ft % p->col->col.cols == 0 &&
                  p->row->row.ft % p->col->col.ospr_cols == 0
              ? p->row->row.ft
              : 0;
  const size_t n = (size_t)W * H;
  {
    const int cw = p->col->col_wide.cols;
    p->wide_ok = cw > 0 && W % cw == 0 && (p->ft == 0 || p->ft % cw == 0);
    p->col_blocks_wide = cw > 0 ? W / cw : 0;
    p->col_slots = p->col_blocks * p->col->col.cols;
    if (cw > 0) p->col_slots = std::max(p->col_slots, (W + cw - 1) / cw * cw);
  }
  p->ws_bytes = ws_layout(p, 1).total;
  *out = p;
  return HG_OK;
}

hg_status hg_plan_destroy(hg_plan plan) {
  if (plan) free_plan(plan);
  return HG_OK;
}

size_t hg_workspace_bytes(hg_plan plan) { return plan ? plan->ws_bytes : 0; }

hg_status hg_propagate(hg_plan p, const void* in_c64, void* out_c64, int32_t direction, void* workspace,
                       hipStream_t stream) {
  (void)workspace;
  if (!p) return fail(HG_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (!in_c64 || !out_c64) return fail(HG_ERR_INVALID_ARGUMENT, "in/out is NULL");
  if (direction != HG_FORWARD && direction != HG_INVERSE)
    return fail(HG_ERR_INVALID_ARGUMENT, "direction must be HG_FORWARD or HG_INVERSE");
  const int W = p->desc.width, H = p->desc.height;
  const bool fres = p->desc.propagation == HG_FRESNEL;
  const bool fwd = direction == HG_FORWARD;
  PropRowArgs ra{};
  ra.in = static_cast<const float2*>(in_c64);
  ra.out = static_cast<float2*>(out_c64);
  ra.H = H;
  ra.tw = p->tw_row[0];
  ra.twr = p->tw_row[1];
  PropColArgs ca{};
  ca.io = static_cast<float2*>(out_c64);
  ca.W = W;
  ca.tw = p->tw_col[0];
  ca.twr = p->tw_col[1];
  ca.scale = fwd ? 1.0f : (float)(1.0 / ((double)W * (double)H));
  if (fres) {
    ra.sx_in = ra.sx_out = W / 2;
    ca.sy_in = ca.sy_out = H / 2;
    if (fwd) {
      ra.pre_y = p->q1y; ra.pre_x = p->q1x;
      ca.post_y = p->fwd_post_y; ca.post_x = p->fwd_post_x;
    } else {
      ra.pre_y = p->inv_pre_y; ra.pre_x = p->inv_pre_x;
      ca.post_y = p->inv_post_y; ca.post_x = p->inv_post_x;
    }
  }
  const RowKernels& rk = p->row->row;
  const ColKernels& ck = p->col->col;
  if (p->desc.propagation == HG_ANGULAR) {
    // row FFT -> column FFT * T (conj T back) inverse column FFT, 1/(H W) -> inverse row FFT
    PropRowArgs r1 = ra;
    launch(p, HG_KERNEL_PROP_ROW, stream, rk.prop_fwd, p->row_blocks, rk.threads, rk.lds, r1);
    AsColArgs ac{};
    ac.io = static_cast<float2*>(out_c64);
    ac.W = W;
    ac.tr = as_transfer(p);
    ac.scale = (float)(1.0 / ((double)W * (double)H));
    ac.tw = p->tw_col[0];
    ac.twr = p->tw_col[1];
    launch(p, HG_KERNEL_PROP_COL, stream, fwd ? ck.as_fwd : ck.as_inv, p->col_blocks, ck.threads, ck.lds, ac);
    PropRowArgs r2 = ra;
    r2.in = static_cast<const float2*>(out_c64);
    launch(p, HG_KERNEL_PROP_ROW, stream, rk.prop_inv, p->row_blocks, rk.threads, rk.lds, r2);
    return launch_status("hg_propagate launch");
  }
  launch(p, HG_KERNEL_PROP_ROW, stream, fwd ? rk.prop_fwd : rk.prop_inv, p->row_blocks, rk.threads, rk.lds, ra);
  launch(p, HG_KERNEL_PROP_COL, stream, fwd ? ck.prop_fwd : ck.prop_inv, p->col_blocks, ck.threads, ck.lds, ca);
  return launch_status("hg_propagate launch");
}

hg_status hg_gs_iterate(hg_plan p, const float* target_amp, const float* illumination, float* phase,
                        uint8_t* levels, float* nmse, int32_t iterations, void* workspace, hipStream_t stream) {
  const hg_status st = gs_validate(p, target_amp, phase, iterations, workspace);
  if (st != HG_OK) return st;
  if (p->desc.modulation == HG_AMPLITUDE) {
    if (illumination) return fail(HG_ERR_INVALID_ARGUMENT, "an HG_AMPLITUDE plan takes no illumination");
    if (p->desc.propagation == HG_ANGULAR)
      return fail(HG_ERR_INVALID_ARGUMENT, "HG_AMPLITUDE needs an HG_FOURIER or HG_FRESNEL plan");
  }
  if (p->desc.propagation == HG_ANGULAR)
    return gs_run_angular(p, target_amp, illumination, phase, levels, nmse, iterations, workspace, stream);
  return gs_run(p, 1, target_amp, illumination, phase, levels, nmse, iterations, workspace, stream);
}

hg_status hg_gs_iterate_window(hg_plan p, const float* target_amp, const uint8_t* window, const float* illumination,
                               float* phase, uint8_t* levels, float* nmse, int32_t iterations, void* workspace,
                               hipStream_t stream) {
  const hg_status st = gs_validate(p, target_amp, phase, iterations, workspace);
  if (st != HG_OK) return st;
  if (!window) return fail(HG_ERR_INVALID_ARGUMENT, "window is NULL");
  if (p->desc.modulation == HG_AMPLITUDE)
    return fail(HG_ERR_INVALID_ARGUMENT, "hg_gs_iterate_window takes phase-only plans");
  if (p->desc.propagation == HG_ANGULAR)
    return fail(HG_ERR_INVALID_ARGUMENT, "hg_gs_iterate_window takes HG_FOURIER or HG_FRESNEL plans");
  return gs_run(p, 1, target_amp, illumination, phase, levels, nmse, iterations, workspace, stream, window);
}

hg_status hg_gs_iterate_noalloc(hg_plan p, const float* target_amp, const float* illumination, float* phase,
                                uint8_t* levels, float* nmse, int32_t iterations, hipStream_t stream) {
  if (!p) return fail(HG_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (!target_amp) return fail(HG_ERR_INVALID_ARGUMENT, "target_amp is NULL");
  if (!phase) return fail(HG_ERR_INVALID_ARGUMENT, "phase is NULL");
  if (iterations < 0) return fail(HG_ERR_INVALID_ARGUMENT, "iterations must be >= 0");
  if (p->ws_bytes > (size_t)HG_NOALLOC_WORKSPACE_MAX)
    return fail(HG_ERR_UNSUPPORTED_SIZE, "the plan needs " + std::to_string(p->ws_bytes) +
                                             " bytes of workspace, above HG_NOALLOC_WORKSPACE_MAX (" +
                                             std::to_string((size_t)HG_NOALLOC_WORKSPACE_MAX) + ")");
  void* ws = nullptr;
  const hg_status sst = device_scratch(&ws);
  if (sst != HG_OK) return sst;
  return hg_gs_iterate(p, target_amp, illumination, phase, levels, nmse, iterations, ws, stream);
}

size_t hg_workspace_bytes_batched(hg_plan plan, int32_t batch) {
  if (!plan || batch < 1) return 0;
  return ws_layout(plan, batch).total;
}

hg_status hg_gs_iterate_batched(hg_plan p, int32_t batch, const float* target_amp, const float* illumination,
                                float* phase, uint8_t* levels, float* nmse, int32_t iterations, void* workspace,
                                hipStream_t stream) {
  const hg_status st = gs_validate(p, target_amp, phase, iterations, workspace);
  if (st != HG_OK) return st;
  if (batch < 1 || batch > 65535) return fail(HG_ERR_INVALID_ARGUMENT, "batch must be in 1..65535");
  if (p->desc.propagation == HG_ANGULAR)
    return fail(HG_ERR_INVALID_ARGUMENT, "hg_gs_iterate_batched takes HG_FOURIER or HG_FRESNEL plans");
  if (p->desc.modulation == HG_AMPLITUDE)
    return fail(HG_ERR_INVALID_ARGUMENT, "hg_gs_iterate_batched takes phase-only plans");
  if ((size_t)batch * field_elems(p) > (size_t)UINT32_MAX)
    return fail(HG_ERR_INVALID_ARGUMENT, "batch * height * (width rounded up to a multiple of 4) must be below 2^32");
  return gs_run(p, batch, target_amp, illumination, phase, levels, nmse, iterations, workspace, stream);
}

hg_status hg_ospr(hg_plan p, const float* target_amp, const float* sub_phase, int32_t n_sub, uint8_t* holograms,
                  float* intensity, float* nmse, void* workspace, hipStream_t stream) {
  if (!p) return fail(HG_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (p->desc.propagation != HG_FOURIER) return fail(HG_ERR_INVALID_ARGUMENT, "hg_ospr needs a HG_FOURIER plan");
  if (!target_amp || !sub_phase || !intensity)
    return fail(HG_ERR_INVALID_ARGUMENT, "target_amp, sub_phase and intensity are required");
  if (!workspace) return fail(HG_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (n_sub < 1) return fail(HG_ERR_INVALID_ARGUMENT, "n_sub must be >= 1");
  const int W = p->desc.width, H = p->desc.height;
  const size_t n = npix(p);
  Workspace w = carve(p, workspace);
  const RowKernels& rk = p->row->row;
  const ColKernels& ck = p->col->col;
  if (nmse) enqueue_stats(p, w, target_amp, nullptr, (double)n * (double)n, w.sc, stream);

  OsprRowArgs ra{};
  ra.ft = p->ft;
  ra.field = w.field;
  ra.H = H;
  ra.target = target_amp;
  ra.intensity = intensity;
  ra.inv_nsub = (float)(1.0 / (double)n_sub);
  ra.sc = w.sc;
  ra.tw = p->tw_row[0];
  ra.twr = p->tw_row[1];
  OsprColArgs ca{};
  ca.ft = p->ft;
  ca.field = w.field;
  ca.W = W;
  ca.tw = p->tw_col[0];
  ca.twr = p->tw_col[1];
  // pass A of subframe 0; after that each pass C also runs the next pass A
  ra.theta = sub_phase;
  launch(p, HG_KERNEL_OSPR_A, stream, rk.ospr_a, p->row_blocks, rk.threads, rk.lds, ra);
  for (int s = 0; s < n_sub; ++s) {
    ra.first = s == 0;
    ra.last = s == n_sub - 1;
    ra.partials = (ra.last && nmse) ? w.partials : nullptr;
    ra.theta_next = ra.last ? nullptr : sub_phase + (size_t)(s + 1) * n;
    ca.levels = holograms ? holograms + (size_t)s * n : nullptr;
    launch(p, HG_KERNEL_OSPR_B, stream, ck.ospr_b, p->ospr_col_blocks, ck.ospr_threads, ck.ospr_lds, ca);
    launch(p, HG_KERNEL_OSPR_C, stream, ra.last ? rk.ospr_c_half : rk.ospr_ca_half, p->ospr_pair_blocks,
           rk.threads, rk.lds, ra);
  }
  if (nmse)
    hipLaunchKernelGGL(k_nmse_reduce, dim3(1), dim3(STATS_THREADS), 0, stream, (const float*)w.partials,
                       p->ospr_pair_blocks, (const Scalars*)w.sc, nmse, (size_t)0, (size_t)0);
  return launch_status("hg_ospr launch");
}

hg_status hg_ospr_pairs(hg_plan p, const float* target_amp, const float* sub_phase, int32_t n_pairs,
                        uint8_t* holograms, float* intensity, float* nmse, void* workspace, hipStream_t stream) {
  if (!p) return fail(HG_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (p->desc.propagation != HG_FOURIER) return fail(HG_ERR_INVALID_ARGUMENT, "hg_ospr_pairs needs a HG_FOURIER plan");
  if (!target_amp || !sub_phase || !intensity)
    return fail(HG_ERR_INVALID_ARGUMENT, "target_amp, sub_phase and intensity are required");
  if (!workspace) return fail(HG_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (n_pairs < 1) return fail(HG_ERR_INVALID_ARGUMENT, "n_pairs must be >= 1");
  const int W = p->desc.width, H = p->desc.height;
  const size_t n = npix(p);
  Workspace w = carve(p, workspace);
  const RowKernels& rk = p->row->row;
  const ColKernels& ck = p->col->col;
  if (nmse) enqueue_stats(p, w, target_amp, nullptr, (double)n * (double)n, w.sc, stream);

  OsprRowArgs ra{};
  ra.ft = p->ft;
  ra.field = w.field;
  ra.H = H;
  ra.target = target_amp;
  ra.intensity = intensity;
  ra.sc = w.sc;
  ra.tw = p->tw_row[0];
  ra.twr = p->tw_row[1];
  OsprColArgs ca{};
  ca.ft = p->ft;
  ca.field = w.field;
  ca.W = W;
  ca.tw = p->tw_col[0];
  ca.twr = p->tw_col[1];
  ra.theta = sub_phase;
  launch(p, HG_KERNEL_OSPR_A, stream, rk.ospr_a, p->row_blocks, rk.threads, rk.lds, ra);
  for (int s = 0; s < n_pairs; ++s) {
    const bool final_pair = s == n_pairs - 1;
    ra.first = s == 0;
    ra.last = 0;        // sums only: the finish kernel averages and scores
    ra.partials = nullptr;
    ra.theta_next = final_pair ? nullptr : sub_phase + (size_t)(s + 1) * n;
    ca.levels = holograms ? holograms + (size_t)(2 * s) * n : nullptr;
    ca.levels_im = holograms ? holograms + (size_t)(2 * s + 1) * n : nullptr;
    launch(p, HG_KERNEL_OSPR_B, stream, ck.ospr_b_pair, p->ospr_col_blocks, ck.ospr_threads, ck.ospr_lds, ca);
    launch(p, HG_KERNEL_OSPR_C, stream, final_pair ? rk.ospr_c : rk.ospr_ca, p->row_blocks, rk.threads, rk.lds, ra);
  }
  // one partial per block: at most PAIR_MAX_BLOCKS, and never more than the
  // workspace's partial buffer holds (kNmseChunk x workgroups of a pass)
  const size_t cap = ws_layout(p, 1).partial_stride;
  size_t nb = (n + PAIR_THREADS - 1) / PAIR_THREADS;
  if (nb > (size_t)PAIR_MAX_BLOCKS) nb = PAIR_MAX_BLOCKS;
  if (nb > cap) nb = cap;
  hipLaunchKernelGGL(k_ospr_pair_finish, dim3((unsigned)nb), dim3(PAIR_THREADS), 0, stream, intensity, target_amp, H, W,
                     (float)(1.0 / (4.0 * n_pairs)), (const Scalars*)w.sc, nmse ? w.partials : nullptr);
  if (nmse)
    hipLaunchKernelGGL(k_nmse_reduce, dim3(1), dim3(STATS_THREADS), 0, stream, (const float*)w.partials, (int)nb,
                       (const Scalars*)w.sc, nmse, (size_t)0, (size_t)0);
  return launch_status("hg_ospr_pairs launch");
}

size_t hg_search_workspace_bytes(hg_plan plan) {
  if (!plan) return 0;
  const size_t n = npix(plan);
  return align_up(n * sizeof(float2)) + 2 * align_up(n * sizeof(float)) + align_up(sizeof(Scalars)) +
         align_up((size_t)STATS_MAX_BLOCKS * 3 * sizeof(double)) +
         align_up(2 * SEARCH_SUMS * SEARCH_MAX_BLOCKS * sizeof(double)) + align_up(2 * sizeof(SearchState));
}

hg_status hg_pixel_search(hg_plan p, const float* target_amp, uint8_t* levels, const int32_t* trials,
                          int32_t n_trials, const float* temperature, const float* uniform, uint8_t* accepted,
                          float* nmse, void* workspace, hipStream_t stream) {
  if (!p) return fail(HG_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (!p->lvl_tab || p->levels < 2)
    return fail(HG_ERR_INVALID_ARGUMENT, "hg_pixel_search needs a HG_PHASE_QUANTISED or HG_BINARY_PHASE plan");
  if (p->desc.propagation == HG_ANGULAR)
    return fail(HG_ERR_INVALID_ARGUMENT, "hg_pixel_search takes HG_FOURIER or HG_FRESNEL plans");
  if (!target_amp || !levels) return fail(HG_ERR_INVALID_ARGUMENT, "target_amp and levels are required");
  if (n_trials < 0) return fail(HG_ERR_INVALID_ARGUMENT, "n_trials must be >= 0");
  if (n_trials > 0 && !trials) return fail(HG_ERR_INVALID_ARGUMENT, "trials is NULL");
  if ((temperature == nullptr) != (uniform == nullptr))
    return fail(HG_ERR_INVALID_ARGUMENT, "temperature and uniform must both be given (annealing) or both be NULL");
  if (!workspace) return fail(HG_ERR_INVALID_ARGUMENT, "workspace is NULL");
  const int W = p->desc.width, H = p->desc.height;
  const size_t n = npix(p);
  char* b = static_cast<char*>(workspace);
  float2* replay = reinterpret_cast<float2*>(b);
  size_t off = align_up(n * sizeof(float2));
  float* t2 = reinterpret_cast<float*>(b + off);
  off += align_up(n * sizeof(float));
  float* phase = reinterpret_cast<float*>(b + off);
  off += align_up(n * sizeof(float));
  Scalars* sc = reinterpret_cast<Scalars*>(b + off);
  off += align_up(sizeof(Scalars));
  double* stats = reinterpret_cast<double*>(b + off);
  off += align_up((size_t)STATS_MAX_BLOCKS * 3 * sizeof(double));
  double* partials = reinterpret_cast<double*>(b + off);
  off += align_up(2 * SEARCH_SUMS * SEARCH_MAX_BLOCKS * sizeof(double));
  SearchState* state = reinterpret_cast<SearchState*>(b + off);

  Workspace w{replay, sc, stats, nullptr, nullptr};
  enqueue_stats(p, w, target_amp, nullptr, (double)n * (double)n, sc, stream);
  const unsigned gb = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_search_target, dim3(gb), dim3(256), 0, stream, target_amp, t2, H, W);
  hipLaunchKernelGGL(k_search_phase, dim3(gb), dim3(256), 0, stream, (const uint8_t*)levels, phase, n,
                     (float)(2.0 * M_PI / p->levels));
  // R = FFT2(Q1 H): the GS start pass (row transforms) and a forward column pass
  const RowKernels& rk = p->row->row;
  const ColKernels& ck = p->col->col;
  GsRowArgs ra{};
  ra.field = replay;
  ra.phase0 = phase;
  ra.H = H;
  if (p->desc.propagation == HG_FRESNEL) {
    ra.q1y = p->q1y;
    ra.q1x = p->q1x;
  }
  ra.slm.lvl_tab = p->lvl_tab;
  ra.slm.levels = p->levels;
  ra.slm.inv_delta = (float)((double)p->levels / (2.0 * M_PI));
  ra.slm.inv_delta_f64 = (double)p->levels / (2.0 * M_PI);
  ra.tw = p->tw_row[0];
  ra.twr = p->tw_row[1];
  hipLaunchKernelGGL(rk.gs_start, dim3(p->row_blocks), dim3(rk.threads), rk.lds, stream, ra);
  PropColArgs ca{};
  ca.io = replay;
  ca.W = W;
  ca.scale = 1.0f;
  ca.tw = p->tw_col[0];
  ca.twr = p->tw_col[1];
  hipLaunchKernelGGL(ck.prop_fwd, dim3(p->col_blocks), dim3(ck.threads), ck.lds, stream, ca);

  SearchArgs sa{};
  sa.replay = replay;
  sa.t2 = t2;
  sa.levels = levels;
  sa.trials = trials;
  sa.temperature = temperature;
  sa.uniform = uniform;
  sa.lvl_tab = p->lvl_tab;
  sa.q1y = ra.q1y;
  sa.q1x = ra.q1x;
  sa.unit_y = p->unit_y;
  sa.unit_x = p->unit_x;
  sa.sc = sc;
  sa.state = state;
  sa.partials = partials;
  sa.accepted = accepted;
  sa.nmse = nmse;
  sa.H = H;
  sa.W = W;
  sa.hmask = (H & (H - 1)) == 0 ? (uint32_t)(H - 1) : 0u;
  sa.wmask = (W & (W - 1)) == 0 ? (uint32_t)(W - 1) : 0u;
  sa.wshift = sa.wmask ? (uint32_t)__builtin_ctz((unsigned)W) : 0u;
  sa.L = p->levels;
  // A binary hologram on a Fourier plane is real (levels +-1), so R is
  // conjugate-symmetric and the search keeps the rows y <= H/2 of it.
  const bool half = p->desc.propagation == HG_FOURIER && p->levels == 2 && H % 2 == 0;
  sa.hh = half ? H / 2 + 1 : H;
  const size_t n_kept = (size_t)sa.hh * W;
  const int nb =
      (int)std::min<size_t>((n_kept + SEARCH_THREADS * 4 - 1) / (SEARCH_THREADS * 4), SEARCH_MAX_BLOCKS);
  hipLaunchKernelGGL(half ? k_search_error<true> : k_search_error<false>, dim3(nb), dim3(SEARCH_THREADS), 0, stream,
                     sa);
  hipLaunchKernelGGL(k_search_start, dim3(1), dim3(SEARCH_THREADS), 0, stream, sa, nb);
  for (int k = 0; k < n_trials; k += 2)
    hipLaunchKernelGGL(half ? k_search_step<true> : k_search_step<false>, dim3(nb), dim3(SEARCH_THREADS), 0, stream,
                       sa, k, (int)n_trials);
  if (n_trials > 0)
    hipLaunchKernelGGL(k_search_finish, dim3(1), dim3(SEARCH_THREADS), 0, stream, sa, n_trials, nb);
  return launch_status("hg_pixel_search launch");
}

size_t hg_multiplane_workspace_bytes(hg_plan plan, int32_t n_planes) {
  return hg_multiplane_workspace_bytes_batched(plan, n_planes, 1);
}

size_t hg_multiplane_workspace_bytes_batched(hg_plan plan, int32_t n_planes, int32_t batch) {
  if (!plan || n_planes < 1 || n_planes > kMaxPlanes || batch < 1 || batch > 65535) return 0;
  return mp_layout(plan, n_planes, batch).total;
}

hg_status hg_gs_multiplane(const hg_plan* planes, int32_t n_planes, const float* target_amp,
                            const float* illumination, float* phase, uint8_t* levels, float* nmse,
                            int32_t iterations, void* workspace, hipStream_t stream) {
  return multiplane_run(planes, n_planes, 1, target_amp, illumination, phase, levels, nmse, iterations, workspace,
                        stream, "hg_gs_multiplane");
}

hg_status hg_gs_multiplane_batched(const hg_plan* planes, int32_t n_planes, int32_t batch,
                                    const float* target_amp, const float* illumination, float* phase,
                                    uint8_t* levels, float* nmse, int32_t iterations, void* workspace,
                                    hipStream_t stream) {
  return multiplane_run(planes, n_planes, batch, target_amp, illumination, phase, levels, nmse, iterations,
                        workspace, stream, "hg_gs_multiplane_batched");
}


size_t hg_grad_workspace_bytes(hg_plan plan, int32_t n_planes) {
  return hg_grad_workspace_bytes_batched(plan, n_planes, 1);
}

size_t hg_grad_workspace_bytes_batched(hg_plan plan, int32_t n_planes, int32_t batch) {
  if (!plan || n_planes < 1 || n_planes > kMaxPlanes || batch < 1 || batch > 65535) return 0;
  return grad_layout(plan, n_planes, batch).total;
}

namespace {

hg_status grad_validate(const hg_plan* planes, int32_t n_planes, int32_t batch, const float* target_amp,
                        void* workspace) {
  hg_status st = validate_planes(planes, n_planes);
  if (st != HG_OK) return st;
  if (!target_amp) return fail(HG_ERR_INVALID_ARGUMENT, "target_amp is NULL");
  if (!workspace) return fail(HG_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (batch < 1 || batch > 65535) return fail(HG_ERR_INVALID_ARGUMENT, "batch must be in 1..65535");
  if ((size_t)batch * n_planes > 65535) return fail(HG_ERR_INVALID_ARGUMENT, "batch * n_planes must be <= 65535");
  if ((size_t)batch * n_planes * field_elems(planes[0]) > (size_t)UINT32_MAX)
    return fail(HG_ERR_INVALID_ARGUMENT, "batch * n_planes * height * (padded) width must be below 2^32");
  return HG_OK;
}

hg_status grad_eval(const hg_plan* planes, int32_t n_planes, int32_t batch, const float* target_amp,
                    const float* phase, float* grad, float* loss, void* workspace, hipStream_t stream) {
  hg_status st = grad_validate(planes, n_planes, batch, target_amp, workspace);
  if (st != HG_OK) return st;
  if (!phase) return fail(HG_ERR_INVALID_ARGUMENT, "phase is NULL");
  if (!grad && !loss) return HG_OK;
  // one evaluation: the phase is only read (no Adam state); one loss per problem
  return grad_run(planes, n_planes, batch, target_amp, const_cast<float*>(phase), grad, nullptr, nullptr,
                  grad ? 1 : 0, 1, 0.f, 0.f, 0.f, 0.f, loss, 1, grad == nullptr, workspace, stream);
}

hg_status grad_adam(const hg_plan* planes, int32_t n_planes, int32_t batch, const float* target_amp, float* phase,
                    float* adam_m, float* adam_v, int32_t steps, int32_t first_step, float lr, float beta1,
                    float beta2, float eps, float* loss, void* workspace, hipStream_t stream) {
  hg_status st = grad_validate(planes, n_planes, batch, target_amp, workspace);
  if (st != HG_OK) return st;
  if (!phase || !adam_m || !adam_v) return fail(HG_ERR_INVALID_ARGUMENT, "phase/adam_m/adam_v is NULL");
  if (steps < 0) return fail(HG_ERR_INVALID_ARGUMENT, "steps must be >= 0");
  if (first_step < 1) return fail(HG_ERR_INVALID_ARGUMENT, "first_step must be >= 1");
  if (!(std::isfinite(lr) && lr > 0.f)) return fail(HG_ERR_INVALID_ARGUMENT, "lr must be finite and > 0");
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
    return fail(HG_ERR_INVALID_ARGUMENT, "beta1 and beta2 must be in [0, 1)");
  if (!(std::isfinite(eps) && eps > 0.f)) return fail(HG_ERR_INVALID_ARGUMENT, "eps must be finite and > 0");
  if (steps == 0 && !loss) return HG_OK;
  return grad_run(planes, n_planes, batch, target_amp, phase, nullptr, adam_m, adam_v, steps, first_step, lr, beta1,
                  beta2, eps, loss, (size_t)steps + 1, loss != nullptr, workspace, stream);
}

}  // namespace

hg_status hg_grad(const hg_plan* planes, int32_t n_planes, const float* target_amp, const float* phase, float* grad,
                  float* loss, void* workspace, hipStream_t stream) {
  return grad_eval(planes, n_planes, 1, target_amp, phase, grad, loss, workspace, stream);
}

hg_status hg_grad_batched(const hg_plan* planes, int32_t n_planes, int32_t batch, const float* target_amp,
                          const float* phase, float* grad, float* loss, void* workspace, hipStream_t stream) {
  return grad_eval(planes, n_planes, batch, target_amp, phase, grad, loss, workspace, stream);
}

hg_status hg_grad_adam(const hg_plan* planes, int32_t n_planes, const float* target_amp, float* phase, float* adam_m,
                       float* adam_v, int32_t steps, int32_t first_step, float lr, float beta1, float beta2, float eps,
                       float* loss, void* workspace, hipStream_t stream) {
  return grad_adam(planes, n_planes, 1, target_amp, phase, adam_m, adam_v, steps, first_step, lr, beta1, beta2, eps,
                   loss, workspace, stream);
}

hg_status hg_grad_adam_batched(const hg_plan* planes, int32_t n_planes, int32_t batch, const float* target_amp,
                               float* phase, float* adam_m, float* adam_v, int32_t steps, int32_t first_step,
                               float lr, float beta1, float beta2, float eps, float* loss, void* workspace,
                               hipStream_t stream) {
  return grad_adam(planes, n_planes, batch, target_amp, phase, adam_m, adam_v, steps, first_step, lr, beta1, beta2,
                   eps, loss, workspace, stream);
}

hg_status hg_timing_begin(hg_plan p, int32_t kernel, int32_t repeats) {
  if (!p) return fail(HG_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (kernel < HG_KERNEL_GS_REPLAY || kernel > HG_KERNEL_PROP_COL)
    return fail(HG_ERR_INVALID_ARGUMENT, "unknown kernel id");
  if (repeats < 1 || repeats > 1000) return fail(HG_ERR_INVALID_ARGUMENT, "repeats must be in 1..1000");
  p->timed_kernel = kernel;
  p->timed_repeats = repeats;
  p->ev_used = 0;
  p->timed_runs = 0;
  p->ev_error = hipSuccess;
  return HG_OK;
}

hg_status hg_timing_end(hg_plan p, double* total_ms, int64_t* launches) {
  if (!p) return fail(HG_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (!total_ms || !launches) return fail(HG_ERR_INVALID_ARGUMENT, "total_ms/launches is NULL");
  const size_t used = p->ev_used;
  const int64_t runs = p->timed_runs;
  const hipError_t pending = p->ev_error;
  p->timed_kernel = 0;
  p->timed_repeats = 1;
  p->ev_used = 0;
  p->timed_runs = 0;
  p->ev_error = hipSuccess;
  if (pending != hipSuccess) return fail(HG_ERR_DEVICE, std::string("timing events: ") + hipGetErrorString(pending));
  double sum = 0.0;
  if (used) {
    hipError_t e = hipEventSynchronize(p->ev_stop[used - 1]);
    if (e != hipSuccess) return fail(HG_ERR_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
    for (size_t i = 0; i < used; ++i) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, p->ev_start[i], p->ev_stop[i]);
      if (e != hipSuccess) return fail(HG_ERR_DEVICE, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
      sum += ms;
    }
  }
  *total_ms = sum;
  *launches = runs;
  return HG_OK;
}

}  // extern "C"
#pragma GCC visibility pop
