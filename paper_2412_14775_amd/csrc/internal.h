// Internal declarations shared by the C-ABI layer (api.hip) and the kernels
// (screen.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rfi {

// Adaptive state record, one per channel group (64 bytes; layout is part of the ABI): the
// exact count of clean windows and the float64 running mean and sum of squared deviations
// of (tau, r_re, r_im).  A float32 state drifts from the float64 one by about 1e-5 (mean)
// and 1e-4 (M2) relative after 1e5 integrations of 48 windows, which the 1e-5 tolerance
// does not allow; each integration's own moments stay float32 (at most T / 2 windows).
struct StateRec {
  uint64_t n;
  double mean[3];
  double m2[3];
  uint64_t reserved;
};
static_assert(sizeof(StateRec) == 64, "state record is 64 bytes");

// Launch arguments of the screen kernels (passed by value as the kernel argument).
struct ScreenArgs {
  const uint8_t *vis;   // [streams][T] samples of `sample_bytes` each
  float *avg;           // [streams][8]
  float *weight;        // [streams]
  uint8_t *flags;       // [streams][nW] or null
  float *stats;         // [streams][nW][3] or null
  StateRec *state;      // [groups] adaptive state or null
  int64_t n_groups;     // B * C / F: channel groups (= streams when F = 1)
  int32_t F;            // channels per window (1, 2 or 4)
  int32_t T;            // samples per stream
  int32_t M;            // window length in time samples
  int32_t nW;           // windows per group = T / M
  int32_t n_seg;        // waves per group (1, 2 or 4)
  int32_t seg_samples;  // samples per wave segment = T / n_seg
  int32_t seg_windows;  // windows per wave segment = seg_samples / M
  float pre;            // (W d + 1) / (W - 1), W = M F
  float Wf;             // W as float
  float invW;           // 1 / W
  float Mt;             // M as float (time samples of a window, per channel)
  float eps;
  float s_low, s_high, gamma;
  float kappa_sk, kappa_ds;
  int32_t n_warm;
  uint32_t options;
  float invT;
  int32_t n_cu;         // compute units of the device (sizes the persistent tiled launch)
};


enum : int { FMT_CF32 = 0, FMT_CF16 = 1 };
constexpr uint32_t kOptPaperMixed = 8u;  // RFI_OPT_PAPER_MIXED

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kMaxTiledLog2M = 12;  // tiled kernels exist for M = 2 .. 4096

// The kernel that screens windows of M samples x F channels in storage format `fmt`:
// tiled (F = 1, M a power of two <= 4096); windowed (runs of C <= 8 samples per lane,
// ceil(M / C) F <= 64 lanes per window) when its layout is exact, when the long kernel does
// not apply, or when the layout fills at least kPadOverLong of its lane slots; long (F = 1,
// M more than half a step: 128 complex64 / 256 complex-half samples); otherwise (F > 1,
// windows wider than 64 lanes) the wide-window kernel, a window over several steps of one
// channel chunk each (F = 4 with runs within 32 lanes: two channels' runs per step).  The paper's mixed precision exists only in the windowed kernel on exact
// layouts with complex64 storage (kNone elsewhere).  The tiled and long kernels may split a
// stream into window-aligned segments (one wave each).
enum KernelKind { kTiled, kWindows, kLong, kWide, kNone };
KernelKind kernel_for(int M, int F, int fmt, bool mixed);

// Samples per lane of the wide-window kernel's chunks (64 C samples of one channel's run).
int wide_chunk(int M, int fmt);
// Samples per lane of its two-runs-per-step form (F = 4, runs within 32 lanes), or 0.
int wide_pairs_chunk(int M, int fmt);

// Lane layout of the windowed kernel: C samples per lane, padded (pad) or exact, and the
// share of its lane slots that hold samples.  C = 0: the windowed kernel does not apply.
struct WindowsLayout {
  int C;
  bool pad;
  double share;
};
WindowsLayout windows_layout(int M, int F, int fmt, bool mixed);
constexpr int kPadMaxC32 = 5;            // padded complex64 layouts: at most 5 samples per lane
constexpr double kPadOverLong = 0.75;    // padded layouts this full go before the long kernel

// Kernel selection (kernel_for).  Returns hipErrorInvalidValue when no kernel matches.
hipError_t launch_screen(int fmt, const ScreenArgs &a, hipStream_t stream);
bool tiled_supports(int M);

// Records the thread's last error (read back by rfi_last_error) and returns `code`.
int set_error(int code, const char *fmt, ...);

hipError_t launch_probe_read(const void *src, size_t bytes, float *sink, hipStream_t stream);
hipError_t launch_probe_copy(void *dst, const void *src, size_t bytes, hipStream_t stream);
size_t probe_sink_floats();
// Check of the complex-half sums against conversion + float32 add: one count per binary16
// value (kHalfSumsValues entries of `bad`), each over kHalfSumsOthers second operands.
constexpr int kHalfSumsValues = 65536;
constexpr int kHalfSumsOthers = 1024;
hipError_t launch_probe_half_sums(uint32_t *bad, hipStream_t stream);

}  // namespace rfi
