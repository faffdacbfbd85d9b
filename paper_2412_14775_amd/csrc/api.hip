// api.hip -- the C ABI of librfi (declared in include/rfi.h): argument
// validation, plan construction, kernel launch on the caller's stream, error
// reporting.  Every argument check runs before any HIP call, so invalid input
// is rejected without touching a device.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/rfi.h"
#include "internal.h"
#include "plan.h"

struct rfi_plan {
  rfi_params p;
  int device;
  int64_t n_streams;
  int64_t n_groups;  // channel groups: n_streams / block_f
  int32_t nW;
  int32_t n_seg;
  size_t sample_bytes;
  void *state;  // device, n_groups * sizeof(rfi::StateRec) bytes, ADAPTIVE only
  size_t state_bytes;
  uint64_t uid;  // rfi::plan_uid
  int n_cu;      // compute units of `device`
};

namespace {

thread_local std::string g_error;
std::atomic<uint64_t> g_next_plan_uid{1};

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int ok() { return RFI_OK; }

int hip_fail(hipError_t e, const char *what) {
  return fail(RFI_ERR_DEVICE, "%s: %s (%s)", what, hipGetErrorString(e), hipGetErrorName(e));
}

// Makes `device` current for the lifetime of the guard and restores the previous one.
class DeviceGuard {
 public:
  explicit DeviceGuard(int device) {
    err_ = hipGetDevice(&prev_);
    if (err_ == hipSuccess && prev_ != device) err_ = hipSetDevice(device);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
  }
  hipError_t error() const { return err_; }

 private:
  int prev_ = 0;
  hipError_t err_ = hipSuccess;
};

bool finite(float x) { return std::isfinite(x); }

int validate(const rfi_params *p) {
  if (p == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "params is NULL");
  if (p->n_stations < 1) return fail(RFI_ERR_INVALID_ARGUMENT, "n_stations must be >= 1 (got %d)", p->n_stations);
  const int64_t N = p->n_stations;
  if ((int64_t)p->n_baselines != N * (N + 1) / 2)
    return fail(RFI_ERR_INVALID_ARGUMENT, "n_baselines must be N(N+1)/2 = %lld for N = %d (got %d)",
                (long long)(N * (N + 1) / 2), p->n_stations, p->n_baselines);
  if (p->n_channels < 1) return fail(RFI_ERR_INVALID_ARGUMENT, "n_channels must be >= 1 (got %d)", p->n_channels);
  if (p->block_m < 2) return fail(RFI_ERR_INVALID_ARGUMENT, "block_m must be >= 2 (got %d)", p->block_m);
  if (p->n_samples < 1 || p->n_samples % p->block_m != 0)
    return fail(RFI_ERR_INVALID_ARGUMENT, "n_samples (%d) must be a positive multiple of block_m (%d)",
                p->n_samples, p->block_m);
  if (p->vis_format != RFI_VIS_CF32 && p->vis_format != RFI_VIS_CF16)
    return fail(RFI_ERR_INVALID_ARGUMENT, "vis_format must be RFI_VIS_CF32 or RFI_VIS_CF16 (got %d)", p->vis_format);
  const int64_t sb = p->vis_format == RFI_VIS_CF32 ? 32 : 16;
  if ((int64_t)p->n_samples * sb >= (int64_t)1 << 31)
    return fail(RFI_ERR_INVALID_ARGUMENT, "n_samples * %lld bytes per sample must be < 2^31", (long long)sb);
  if (p->block_f < 1 || p->n_channels % p->block_f != 0)
    return fail(RFI_ERR_INVALID_ARGUMENT, "block_f (%d) must be >= 1 and divide n_channels (%d)", p->block_f,
                p->n_channels);
  if (!(finite(p->sk_d) && p->sk_d > 0.0f)) return fail(RFI_ERR_INVALID_ARGUMENT, "sk_d must be finite and > 0");
  if (std::isnan(p->sk_low) || std::isnan(p->sk_high) || !(p->sk_low < p->sk_high))
    return fail(RFI_ERR_INVALID_ARGUMENT, "need sk_low < sk_high (got %g, %g)", p->sk_low, p->sk_high);
  if (!(p->ds_gamma >= 0.0f && p->ds_gamma <= 1.0f))
    return fail(RFI_ERR_INVALID_ARGUMENT, "ds_gamma must be in [0, 1] (got %g)", p->ds_gamma);
  if (!(finite(p->eps) && p->eps >= 0.0f)) return fail(RFI_ERR_INVALID_ARGUMENT, "eps must be finite and >= 0");
  if (p->options & ~(uint32_t)(RFI_OPT_NO_SK | RFI_OPT_NO_DS | RFI_OPT_ADAPTIVE | RFI_OPT_PAPER_MIXED))
    return fail(RFI_ERR_INVALID_ARGUMENT, "unknown option bits 0x%x", p->options);
  if (p->options & RFI_OPT_ADAPTIVE) {
    if (!(finite(p->kappa_sk) && p->kappa_sk >= 0.0f && finite(p->kappa_ds) && p->kappa_ds >= 0.0f))
      return fail(RFI_ERR_INVALID_ARGUMENT, "kappa_sk and kappa_ds must be finite and >= 0");
    if (p->n_warm < 0) return fail(RFI_ERR_INVALID_ARGUMENT, "n_warm must be >= 0");
  }
  if (p->block_f != 1 && p->block_f != 2 && p->block_f != 4)
    return fail(RFI_ERR_UNSUPPORTED, "block_f must be 1, 2 or 4 (got %d)", p->block_f);
  if ((int64_t)p->block_f * p->n_samples * sb >= (int64_t)1 << 31)
    return fail(RFI_ERR_INVALID_ARGUMENT, "block_f * n_samples * bytes per sample must be < 2^31");
  if ((p->options & RFI_OPT_PAPER_MIXED) &&
      rfi::kernel_for(p->block_m, p->block_f, p->vis_format == RFI_VIS_CF32 ? rfi::FMT_CF32 : rfi::FMT_CF16,
                      true) != rfi::kWindows)
    return fail(RFI_ERR_UNSUPPORTED,
                "RFI_OPT_PAPER_MIXED needs complex64 storage and a window M = K S (K <= 8, S a power of two, F S <= 64)");
  return RFI_OK;
}

// Waves per stream: split short, few streams over up to 4 waves of a block
// (window-aligned segments) so that small arrays still fill the GPU.
int choose_segments(const rfi_params &p, int64_t n_streams) {
  int n_seg = 1;
  const rfi::KernelKind kind =
      rfi::kernel_for(p.block_m, p.block_f, p.vis_format == RFI_VIS_CF32 ? rfi::FMT_CF32 : rfi::FMT_CF16,
                      (p.options & RFI_OPT_PAPER_MIXED) != 0);
  if (kind != rfi::kTiled && kind != rfi::kLong) return 1;  // only these kernels split a stream
  const int64_t target_waves = 64 * 1024;
  while (n_seg < rfi::kWavesPerBlock && n_streams * n_seg < target_waves &&
         p.n_samples % (2 * n_seg * p.block_m) == 0 && p.n_samples / (2 * n_seg) >= 256)
    n_seg *= 2;
  return n_seg;
}

// Zeroes n 32-bit words with vector stores.  rfi_state_reset uses this kernel rather than
// hipMemsetAsync so that a caller may capture the reset in a graph: memset nodes have given
// wrong results on replays after the first, kernel nodes have not.
__global__ void __launch_bounds__(256) zero_words(uint32_t *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

}  // namespace

uint64_t rfi::plan_uid(const rfi_plan *plan) { return plan->uid; }

size_t rfi::plan_stats_bytes(const rfi_plan *plan) { return (size_t)plan->n_groups * plan->nW * 3 * sizeof(float); }

int rfi::set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

extern "C" {

void rfi_params_default(rfi_params *p) {
  if (p == nullptr) return;
  std::memset(p, 0, sizeof *p);
  p->block_m = 64;
  p->vis_format = RFI_VIS_CF32;
  p->sk_d = 1.0f;
  p->sk_low = 0.5f;
  p->sk_high = 2.0f;
  p->ds_gamma = 0.4f;
  p->eps = 1.0f / 8388608.0f;  // 2^-23
  p->kappa_sk = 3.0f;
  p->kappa_ds = 3.0f;
  p->n_warm = 0;
  p->block_f = 1;
}

int rfi_plan_create(const rfi_params *params, int device, rfi_plan **out) {
  if (out == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (int rc = validate(params)) return rc;
  if (device < 0) return fail(RFI_ERR_INVALID_ARGUMENT, "device must be >= 0 (got %d)", device);
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device >= count) return fail(RFI_ERR_INVALID_ARGUMENT, "device %d does not exist (%d devices)", device, count);

  rfi_plan *plan = new (std::nothrow) rfi_plan{};
  if (plan == nullptr) return fail(RFI_ERR_OUT_OF_MEMORY, "host allocation of the plan failed");
  plan->p = *params;
  plan->uid = g_next_plan_uid.fetch_add(1);
  plan->device = device;
  e = hipDeviceGetAttribute(&plan->n_cu, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) {
    delete plan;
    return hip_fail(e, "hipDeviceGetAttribute(multiprocessor count)");
  }
  plan->n_streams = (int64_t)params->n_baselines * params->n_channels;
  plan->n_groups = plan->n_streams / params->block_f;
  plan->nW = params->n_samples / params->block_m;
  plan->sample_bytes = params->vis_format == RFI_VIS_CF32 ? 32 : 16;
  plan->n_seg = choose_segments(*params, plan->n_streams);
  if (params->options & RFI_OPT_ADAPTIVE) {
    DeviceGuard g(device);
    if (g.error() != hipSuccess) {
      delete plan;
      return hip_fail(g.error(), "hipSetDevice");
    }
    plan->state_bytes = (size_t)plan->n_groups * sizeof(rfi::StateRec);
    e = hipMalloc(&plan->state, plan->state_bytes);
    if (e != hipSuccess) {
      delete plan;
      (void)hipGetLastError();
      return fail(RFI_ERR_OUT_OF_MEMORY, "hipMalloc of %zu state bytes: %s", plan->state_bytes, hipGetErrorString(e));
    }
    e = hipMemset(plan->state, 0, plan->state_bytes);
    if (e != hipSuccess) {
      (void)hipFree(plan->state);
      delete plan;
      return hip_fail(e, "hipMemset(state)");
    }
  }
  *out = plan;
  return ok();
}

int rfi_screen(rfi_plan *plan, const void *vis, float *avg, float *weight, uint8_t *flags, float *stats,
               void *hip_stream) {
  if (plan == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (vis == nullptr || avg == nullptr || weight == nullptr)
    return fail(RFI_ERR_INVALID_ARGUMENT, "vis, avg and weight must not be NULL");
  if (reinterpret_cast<uintptr_t>(vis) % 16 != 0) return fail(RFI_ERR_INVALID_ARGUMENT, "vis must be 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(avg) % 16 != 0) return fail(RFI_ERR_INVALID_ARGUMENT, "avg must be 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(weight) % 4 != 0 || (stats && reinterpret_cast<uintptr_t>(stats) % 4 != 0))
    return fail(RFI_ERR_INVALID_ARGUMENT, "weight and stats must be 4-byte aligned");
  const rfi_params &p = plan->p;
  rfi::ScreenArgs a{};
  a.vis = static_cast<const uint8_t *>(vis);
  a.avg = avg;
  a.weight = weight;
  a.flags = flags;
  a.stats = stats;
  a.state = static_cast<rfi::StateRec *>(plan->state);
  a.n_groups = plan->n_groups;
  a.F = p.block_f;
  a.T = p.n_samples;
  a.M = p.block_m;
  a.nW = plan->nW;
  a.n_seg = plan->n_seg;
  a.seg_samples = p.n_samples / plan->n_seg;
  a.seg_windows = a.seg_samples / p.block_m;
  const double W = (double)p.block_m * p.block_f;
  a.pre = (float)((W * (double)p.sk_d + 1.0) / (W - 1.0));
  a.Wf = (float)W;
  a.invW = (float)(1.0 / W);
  a.Mt = (float)p.block_m;
  a.eps = p.eps;
  a.s_low = p.sk_low;
  a.s_high = p.sk_high;
  a.gamma = p.ds_gamma;
  a.kappa_sk = p.kappa_sk;
  a.kappa_ds = p.kappa_ds;
  a.n_warm = p.n_warm;
  a.options = p.options;
  a.invT = (float)(1.0 / (double)p.n_samples);
  a.n_cu = plan->n_cu;

  DeviceGuard g(plan->device);
  if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
  hipError_t e = rfi::launch_screen(p.vis_format, a, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "screen kernel launch");
  return ok();
}

int rfi_destroy(rfi_plan *plan) {
  if (plan == nullptr) return ok();
  int rc = RFI_OK;
  if (plan->state != nullptr) {
    DeviceGuard g(plan->device);
    hipError_t e = hipFree(plan->state);
    if (e != hipSuccess) rc = hip_fail(e, "hipFree(state)");
  }
  delete plan;
  return rc;
}

const char *rfi_last_error(void) { return g_error.c_str(); }

int rfi_plan_footprint(const rfi_plan *plan, size_t *bytes) {
  if (plan == nullptr || bytes == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "plan and bytes must not be NULL");
  const size_t S = (size_t)plan->n_streams;
  const size_t vis = S * (size_t)plan->p.n_samples * plan->sample_bytes;
  const size_t out = S * (8 * sizeof(float) + sizeof(float)) + (size_t)plan->n_groups * plan->nW;
  *bytes = plan->state_bytes + vis + out;
  return ok();
}

size_t rfi_state_bytes(const rfi_plan *plan) { return plan ? plan->state_bytes : 0; }

int rfi_state_get(rfi_plan *plan, void *host_dst, size_t bytes) {
  if (plan == nullptr || host_dst == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "plan and host_dst must not be NULL");
  if (plan->state == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "plan has no adaptive state");
  if (bytes != plan->state_bytes) return fail(RFI_ERR_INVALID_ARGUMENT, "bytes must be %zu", plan->state_bytes);
  DeviceGuard g(plan->device);
  if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
  hipError_t e = hipMemcpy(host_dst, plan->state, bytes, hipMemcpyDeviceToHost);
  return e == hipSuccess ? ok() : hip_fail(e, "hipMemcpy(state -> host)");
}

int rfi_state_set(rfi_plan *plan, const void *host_src, size_t bytes) {
  if (plan == nullptr || host_src == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "plan and host_src must not be NULL");
  if (plan->state == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "plan has no adaptive state");
  if (bytes != plan->state_bytes) return fail(RFI_ERR_INVALID_ARGUMENT, "bytes must be %zu", plan->state_bytes);
  DeviceGuard g(plan->device);
  if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
  hipError_t e = hipMemcpy(plan->state, host_src, bytes, hipMemcpyHostToDevice);
  return e == hipSuccess ? ok() : hip_fail(e, "hipMemcpy(host -> state)");
}

int rfi_state_reset(rfi_plan *plan, void *hip_stream) {
  if (plan == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (plan->state == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "plan has no adaptive state");
  DeviceGuard g(plan->device);
  if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
  const size_t words = plan->state_bytes / 4;
  const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_words, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<uint32_t *>(plan->state), words);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ok() : hip_fail(e, "state reset launch");
}

size_t rfi_probe_sink_floats(size_t bytes) {
  (void)bytes;
  return rfi::probe_sink_floats();
}

int rfi_probe_read(const void *src, size_t bytes, float *sink, void *hip_stream) {
  if (src == nullptr || sink == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "src and sink must not be NULL");
  if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0)
    return fail(RFI_ERR_INVALID_ARGUMENT, "bytes and src must be multiples of 16");
  hipError_t e = rfi::launch_probe_read(src, bytes, sink, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? ok() : hip_fail(e, "probe_read launch");
}

int rfi_probe_copy(void *dst, const void *src, size_t bytes, void *hip_stream) {
  if (src == nullptr || dst == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "src and dst must not be NULL");
  if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
    return fail(RFI_ERR_INVALID_ARGUMENT, "bytes, src and dst must be multiples of 16");
  hipError_t e = rfi::launch_probe_copy(dst, src, bytes, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? ok() : hip_fail(e, "probe_copy launch");
}

int rfi_probe_half_sums(uint32_t *mismatches, void *hip_stream) {
  if (mismatches == nullptr) return fail(RFI_ERR_INVALID_ARGUMENT, "mismatches must not be NULL");
  hipError_t e = rfi::launch_probe_half_sums(mismatches, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? ok() : hip_fail(e, "probe_half_sums launch");
}

}  // extern "C"
