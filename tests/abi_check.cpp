// Host-side exercise of librfi's C ABI for the sanitizer test (no GPU needed): every
// argument check, error strings, the hyperparameter helpers on odd inputs.  Prints
// "ALL OK" when every expectation holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"
#include "rfi.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond);    \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static rfi_params good() {
  rfi_params p;
  rfi_params_default(&p);
  p.n_stations = 4;
  p.n_baselines = 10;
  p.n_channels = 16;
  p.n_samples = 256;
  p.block_m = 16;
  return p;
}

// Which kernel screens which window shape (rfi::kernel_for): the plan's segment choice and the
// launch both follow it.
static void kernel_choice() {
  using namespace rfi;
  const int c32 = FMT_CF32, c16 = FMT_CF16;
  EXPECT(kernel_for(2, 1, c32, false) == kTiled && kernel_for(64, 1, c16, false) == kTiled);
  EXPECT(kernel_for(4096, 1, c32, false) == kTiled);
  EXPECT(kernel_for(8192, 1, c32, false) == kLong && kernel_for(8192, 1, c16, false) == kLong);
  EXPECT(kernel_for(10, 2, c16, false) == kWindows && kernel_for(5, 4, c32, false) == kWindows);
  EXPECT(kernel_for(20, 1, c32, false) == kWindows && kernel_for(3, 1, c16, false) == kWindows);
  EXPECT(kernel_for(64, 2, c32, false) == kWindows && kernel_for(384, 1, c32, false) == kWindows);
  EXPECT(kernel_for(300, 1, c32, false) == kWindows && kernel_for(300, 1, c16, false) == kWindows);  // 5 x 60 lanes
  EXPECT(kernel_for(600, 1, c16, false) == kLong && kernel_for(3000, 1, c16, false) == kLong);
  EXPECT(kernel_for(513, 1, c16, false) == kLong && kernel_for(321, 1, c32, false) == kLong);  // > 64 runs of 8 / 5
  // padded runs fill at least 3/4 of their lane slots: before the long kernel
  EXPECT(kernel_for(500, 1, c16, false) == kWindows && kernel_for(257, 1, c16, false) == kWindows);
  EXPECT(kernel_for(131, 1, c32, false) == kWindows && kernel_for(131, 1, c16, false) == kWindows);
  EXPECT(kernel_for(67, 1, c32, false) == kWindows && kernel_for(127, 1, c16, false) == kWindows);
  EXPECT(kernel_for(100, 1, c32, false) == kWindows && kernel_for(15, 2, c16, false) == kWindows);
  EXPECT(kernel_for(61, 1, c32, false) == kWindows && kernel_for(61, 1, c16, false) == kWindows);
  EXPECT(kernel_for(8192, 2, c32, false) == kWide && kernel_for(300, 2, c16, false) == kWide);  // > 64 lanes
  EXPECT(kernel_for(129, 4, c16, false) == kWide && kernel_for(200, 4, c32, false) == kWide);
  EXPECT(kernel_for(256, 2, c16, false) == kWindows && kernel_for(257, 2, c16, false) == kWide);
  // chunks of 64 C samples: 300 = 5 x 60 lanes (94 %), 8192 = 16 chunks of 512, 129 on 64 x 4
  EXPECT(wide_chunk(300, c16) == 5 && wide_chunk(8192, c16) == 8 && wide_chunk(129, c16) == 4);
  EXPECT(wide_chunk(200, c32) == 4 && wide_chunk(8192, c32) == 4 && wide_chunk(257, c32) == 3);
  EXPECT(wide_chunk(1000, c16) == 8 && wide_chunk(600, c16) == 5);
  // two runs per step (F = 4): the fewest samples per lane that fit a run in 32 lanes
  EXPECT(wide_pairs_chunk(129, c16) == 5 && wide_pairs_chunk(200, c16) == 7 && wide_pairs_chunk(256, c16) == 8);
  EXPECT(wide_pairs_chunk(257, c16) == 0 && wide_pairs_chunk(100, c16) == 0);
  EXPECT(wide_pairs_chunk(81, c32) == 3 && wide_pairs_chunk(100, c32) == 4 && wide_pairs_chunk(129, c32) == 0);
  EXPECT(kernel_for(100, 4, c32, false) == kWide && kernel_for(81, 4, c32, false) == kWide);
  // lane layouts: (samples per lane, padded, share of lane slots)
  const WindowsLayout l100 = windows_layout(100, 1, c16, false), l100b = windows_layout(100, 1, c32, false);
  EXPECT(l100.C == 7 && l100.pad && l100.share > 0.89 && l100.share < 0.90);   // 15 runs on 16 lanes
  EXPECT(l100b.C == 4 && l100b.pad && l100b.share == 25.0 / 32.0);            // complex64: C <= 5 padded
  EXPECT(windows_layout(10, 2, c16, false).C == 5 && !windows_layout(10, 2, c16, false).pad);
  EXPECT(windows_layout(48, 1, c32, false).C == 6 && !windows_layout(48, 1, c32, false).pad);
  EXPECT(windows_layout(50, 1, c16, false).C == 7 && windows_layout(61, 1, c16, false).C == 8);
  EXPECT(windows_layout(100, 1, c32, true).C == 0 && windows_layout(10, 2, c32, true).C == 5);
  EXPECT(kernel_for(1000, 2, c16, false) == kWide);
  EXPECT(kernel_for(10, 2, c32, true) == kWindows && kernel_for(64, 1, c32, true) == kWindows);
  EXPECT(kernel_for(10, 2, c16, true) == kNone && kernel_for(1024, 1, c32, true) == kNone);
  EXPECT(kernel_for(100, 1, c32, true) == kNone);  // mixed precision: whole power-of-two lane groups only
}

int main() {
  kernel_choice();
  rfi_plan *plan = reinterpret_cast<rfi_plan *>(0x1);
  EXPECT(rfi_plan_create(nullptr, 0, &plan) == RFI_ERR_INVALID_ARGUMENT && plan == nullptr);
  EXPECT(std::strlen(rfi_last_error()) > 0);
  rfi_params p = good();
  EXPECT(rfi_plan_create(&p, 0, nullptr) == RFI_ERR_INVALID_ARGUMENT);
  struct Bad { void (*mutate)(rfi_params &); int code; };
  const Bad bad[] = {
      {[](rfi_params &q) { q.n_stations = 0; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.n_stations = 70000; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.n_baselines = 11; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.block_m = 0; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.n_samples = -16; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.vis_format = -1; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.sk_d = -1.0f; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.sk_low = NAN; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.ds_gamma = NAN; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.eps = NAN; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.options = 0xffffffffu; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.options = RFI_OPT_ADAPTIVE; q.kappa_ds = INFINITY; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.block_f = 0; }, RFI_ERR_INVALID_ARGUMENT},
      {[](rfi_params &q) { q.block_f = 16; }, RFI_ERR_UNSUPPORTED},
      {[](rfi_params &q) { q.options = RFI_OPT_PAPER_MIXED; q.vis_format = RFI_VIS_CF16; }, RFI_ERR_UNSUPPORTED},
      {[](rfi_params &q) { q.options = RFI_OPT_PAPER_MIXED; q.block_m = 100; q.n_samples = 500; }, RFI_ERR_UNSUPPORTED},
  };
  for (const Bad &b : bad) {
    rfi_params q = good();
    b.mutate(q);
    rfi_plan *out = reinterpret_cast<rfi_plan *>(0x1);
    EXPECT(rfi_plan_create(&q, 0, &out) == b.code && out == nullptr);
  }
  // a valid plan on a machine without a GPU: a device error, never a crash
  rfi_plan *out = nullptr;
  const int rc = rfi_plan_create(&p, 0, &out);
  EXPECT(rc == RFI_OK || rc == RFI_ERR_DEVICE || rc == RFI_ERR_INVALID_ARGUMENT);
  if (rc == RFI_OK) rfi_destroy(out);
  EXPECT(rfi_screen(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_destroy(nullptr) == RFI_OK);
  size_t bytes = 0;
  EXPECT(rfi_plan_footprint(nullptr, &bytes) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_state_bytes(nullptr) == 0);
  EXPECT(rfi_state_get(nullptr, nullptr, 0) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_state_set(nullptr, nullptr, 0) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_state_reset(nullptr, nullptr) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_probe_read(nullptr, 16, nullptr, nullptr) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_probe_copy(nullptr, nullptr, 16, nullptr) == RFI_ERR_INVALID_ARGUMENT);
  // serving: configuration and request checks
  rfi_server *srv = reinterpret_cast<rfi_server *>(0x1);
  rfi_server_config cfg{0, 0, 1, 1, 0};
  EXPECT(rfi_server_create(&cfg, &srv) == RFI_ERR_INVALID_ARGUMENT && srv == nullptr);
  cfg.n_slots = 4;
  cfg.hbm_budget = 0;
  EXPECT(rfi_server_create(&cfg, &srv) == RFI_ERR_INVALID_ARGUMENT);
  cfg.hbm_budget = 1;
  cfg.max_graphs = -1;
  EXPECT(rfi_server_create(&cfg, &srv) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_server_create(nullptr, &srv) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_server_submit(nullptr, nullptr) == RFI_ERR_INVALID_ARGUMENT);
  int32_t n = -1;
  EXPECT(rfi_server_poll(nullptr, nullptr, 0, &n, 0.0) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_server_drain(nullptr, 0.0) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_server_get_stats(nullptr, nullptr) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_server_destroy(nullptr) == RFI_OK);
  EXPECT(rfi_server_now(nullptr) == 0.0);
  // hyperparameter helpers
  double m, v, s;
  EXPECT(rfi_sk_null_moments(20, 2.0f, &m, &v, &s) == RFI_OK && std::fabs(m - 1.0) < 1e-9 && v > 0 && s > 0);
  EXPECT(rfi_sk_null_moments(1, 1.0f, &m, &v, &s) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_sk_null_moments(16, NAN, &m, &v, &s) == RFI_ERR_INVALID_ARGUMENT);
  float lo, hi, g, d;
  EXPECT(rfi_thresholds_from_pfa(20, 2.0f, 0.05, 0.05, &lo, &hi, &g) == RFI_OK && lo < 1 && hi > 1 && g > 0 && g < 1);
  EXPECT(rfi_thresholds_from_pfa(20, 2.0f, 1.0, 0.05, &lo, &hi, &g) == RFI_ERR_INVALID_ARGUMENT);
  std::vector<float> st(3 * 1000);
  for (int i = 0; i < 1000; ++i) {
    st[3 * i] = 0.5f + (i % 37) * 0.03f;
    st[3 * i + 1] = (i % 11) * 0.02f;
    st[3 * i + 2] = i % 3 ? NAN : 0.0f;
  }
  EXPECT(rfi_calibrate_from_stats(st.data(), 1000, 20, 2.0f, 0.05, 0.05, &d, &lo, &hi, &g) == RFI_OK && d > 0);
  EXPECT(rfi_calibrate_from_stats(st.data(), 1, 20, 2.0f, 0.05, 0.05, &d, &lo, &hi, &g) == RFI_ERR_INVALID_ARGUMENT);
  EXPECT(rfi_calibrate_from_stats(nullptr, 10, 20, 2.0f, 0.05, 0.05, &d, &lo, &hi, &g) == RFI_ERR_INVALID_ARGUMENT);
  std::vector<float> nan(30, NAN);
  EXPECT(rfi_calibrate_from_stats(nan.data(), 10, 20, 2.0f, 0.05, 0.05, &d, &lo, &hi, &g) == RFI_ERR_INVALID_ARGUMENT);
  if (failures == 0) std::printf("ALL OK\n");
  return failures == 0 ? 0 : 1;
}
