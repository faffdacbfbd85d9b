// screen.hip -- gfx950 kernels of the online energy + polarisation RFI screen
// (arXiv 2412.14775, Section 2, Tables 1-2).
//
// One pass over the visibilities, bound by HBM bandwidth:
//   * each wave owns one stream (baseline, channel) or a window-aligned segment
//     of it, and walks it in 8 KiB steps;
//   * a step is read with fully coalesced 16-byte buffer loads (lane l takes
//     16-byte piece i*64 + l) and transposed through a per-wave LDS tile, so
//     that afterwards each lane holds K consecutive time samples (K = 4 for
//     complex64 storage, 8 for complex-half storage).  The LDS slot of piece p
//     is p ^ (((p >> 3) ^ (p >> 6)) & 7): both the coalesced writes and the
//     transposed 16-byte reads hit distinct banks;
//   * per sample: Stokes I, Q, U, V (eq. IQUV); y = |I|^2, z = |I| (Table 1
//     groups 1-2); p = |(q, u, v)| + eps and the unit vector (Table 2 groups 1-3)
//     for the real and the imaginary parts -- all in FP32, with the hardware
//     sqrt and reciprocal;
//   * window sums (Table 1 groups 3-4, Table 2 group 4) accumulate serially in
//     each lane and, when a window spans several lanes, with a DPP butterfly
//     whose result every lane of the window holds;
//   * each lane also sums its raw samples of the window; when the window's
//     flag is known the partial is added to the lane's stream accumulator only
//     if the window is clean, so no sample is kept in registers;
//   * at the end of the stream one cross-lane reduction gives the masked sum
//     and the count of clean samples: average = sum / count, weight = count / T.
// No atomics: every reduction has a fixed order, so results are bitwise
// reproducible run to run.

#include "internal.h"

namespace rfi {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kPieces = 8;                    // 16-byte pieces per lane per step
constexpr int kTilePieces = kWave * kPieces;  // 8 KiB per wave per step
constexpr int kRsrcWord3 = 0x00020000;        // raw buffer, 32-bit data format
// Cache policy of the visibility loads: non-temporal (every byte is read exactly
// once, so it should not displace anything in L2 / the infinity cache).
constexpr int kLoadStreaming = 2;

__device__ __forceinline__ int lds_slot(int p) { return p ^ (((p >> 3) ^ (p >> 6)) & 7); }

// Orders this wave's LDS accesses (the tile is private to the wave).
__device__ __forceinline__ void wave_lds_order() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of G lanes; every lane of a group receives the same
// (bitwise identical) total.  Levels 4 and 8 use the mirror patterns, valid
// because after the previous levels the partner's value is already uniform
// over its quad / half-row.
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (G >= 2) v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  if constexpr (G >= 4) v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  if constexpr (G >= 8) v += dpp_mov<0x141>(v);  // row_half_mirror: other quad
  if constexpr (G >= 16) v += dpp_mov<0x140>(v); // row_mirror: other half-row
  if constexpr (G >= 32) v += __shfl_xor(v, 16);
  if constexpr (G >= 64) v += __shfl_xor(v, 32);
  return v;
}

// Running (count, mean, sum of squared deviations) of the three statistics.
struct Moments {
  float n;
  float m[3];
  float s[3];
};

__device__ __forceinline__ void moments_push(Moments &a, float x0, float x1, float x2) {
  a.n += 1.0f;
  const float inv = 1.0f / a.n;
  const float x[3] = {x0, x1, x2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float d = x[k] - a.m[k];
    a.m[k] += d * inv;
    a.s[k] += d * (x[k] - a.m[k]);
  }
}

// Pairwise merge of Chan, Golub & LeVeque (1979).
__device__ __forceinline__ Moments moments_merge(const Moments &a, const Moments &b) {
  const float n = a.n + b.n;
  if (n == 0.0f) return a;
  const float fb = b.n / n;
  const float cross = a.n * b.n / n;
  Moments r;
  r.n = n;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float d = b.m[k] - a.m[k];
    r.m[k] = a.m[k] + d * fb;
    r.s[k] = a.s[k] + b.s[k] + d * d * cross;
  }
  return r;
}

__device__ __forceinline__ Moments moments_shfl_xor(const Moments &a, int mask) {
  Moments b;
  b.n = __shfl_xor(a.n, mask);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    b.m[k] = __shfl_xor(a.m[k], mask);
    b.s[k] = __shfl_xor(a.s[k], mask);
  }
  return b;
}

struct Thresholds {
  float s_low, s_high, g_re, g_im;
};

// Per-stream thresholds: plan values, or from the running null statistics.
__device__ __forceinline__ Thresholds stream_thresholds(const ScreenArgs &a, int64_t stream) {
  Thresholds t{a.s_low, a.s_high, a.gamma, a.gamma};
  if (a.state != nullptr) {
    const StateRec *st = reinterpret_cast<const StateRec *>(a.state) + stream;
    const uint32_t n = st->n;
    const uint32_t warm = a.n_warm > 2 ? (uint32_t)a.n_warm : 2u;
    if (n >= warm) {
      const float inv = 1.0f / (float)(n - 1);
      const float sd0 = sqrtf(st->m2[0] * inv);
      const float sd1 = sqrtf(st->m2[1] * inv);
      const float sd2 = sqrtf(st->m2[2] * inv);
      t.s_low = st->mean[0] - a.kappa_sk * sd0;
      t.s_high = st->mean[0] + a.kappa_sk * sd0;
      t.g_re = st->mean[1] + a.kappa_ds * sd1;
      t.g_im = st->mean[2] + a.kappa_ds * sd2;
    }
  }
  return t;
}

// One sample: Stokes (eq. IQUV) and the per-sample terms of Tables 1 and 2,
// added to the window sums ws = (S1, S2, sum q^, u^, v^ of Re, of Im) and the
// raw sums wr.  x = (xx_re, xx_im, xy_re, xy_im, yx_re, yx_im, yy_re, yy_im).
__device__ __forceinline__ void accumulate_sample(float ws[8], float wr[8], const float x[8],
                                                  float eps) {
  const float Ir = x[0] + x[6], Ii = x[1] + x[7];
  const float Qr = x[0] - x[6], Qi = x[1] - x[7];
  const float Ur = x[2] + x[4], Ui = x[3] + x[5];
  const float Vr = x[5] - x[3], Vi = x[2] - x[4];  // V = j (xy - yx)
  const float y = Ir * Ir + Ii * Ii;
  ws[0] += hw_sqrt(y);
  ws[1] += y;
  const float rr = hw_rcp(hw_sqrt(Qr * Qr + Ur * Ur + Vr * Vr) + eps);
  ws[2] += Qr * rr;
  ws[3] += Ur * rr;
  ws[4] += Vr * rr;
  const float ri = hw_rcp(hw_sqrt(Qi * Qi + Ui * Ui + Vi * Vi) + eps);
  ws[5] += Qi * ri;
  ws[6] += Ui * ri;
  ws[7] += Vi * ri;
#pragma unroll
  for (int k = 0; k < 8; ++k) wr[k] += x[k];
}

// Per-stream running results of a wave.  A window covers F adjacent channels
// of one baseline (F = 1: a single channel), each with its own masked sum.
template <int F>
struct StreamAcc {
  float sum[F][8];  // masked raw sums per channel (lane partials)
  float kept;       // clean time samples (lane partial; the same for the F channels)
  Moments mom;      // statistics of clean windows (adaptive state)
};

// Statistics and flag of one window from its totals; flag / stats written by
// the window's leader lane; raw partials folded in when the window is clean.
template <int F>
__device__ __forceinline__ void finish_window(const ScreenArgs &a, const Thresholds &th,
                                              const float tot[8], const float (*wr)[8],
                                              int64_t out_index, bool valid, bool leader,
                                              StreamAcc<F> &acc) {
  const float tau = a.pre * (a.Wf * tot[1] / (tot[0] * tot[0] + a.eps) - 1.0f);
  const float r_re = sqrtf(tot[2] * tot[2] + tot[3] * tot[3] + tot[4] * tot[4]) * a.invW;
  const float r_im = sqrtf(tot[5] * tot[5] + tot[6] * tot[6] + tot[7] * tot[7]) * a.invW;
  uint32_t bits = (!(tau >= th.s_low) ? 1u : 0u) | (tau > th.s_high ? 2u : 0u) |
                  (!(r_re <= th.g_re) ? 4u : 0u) | (!(r_im <= th.g_im) ? 8u : 0u);
  if (a.options & 1u) bits &= ~3u;
  if (a.options & 2u) bits &= ~12u;
  const bool clean = valid && bits == 0u;
  if (clean) {
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int k = 0; k < 8; ++k) acc.sum[f][k] += wr[f][k];
  }
  if (valid && leader) {
    if (clean) {
      acc.kept += a.Mt;
      if (a.state != nullptr) moments_push(acc.mom, tau, r_re, r_im);
    }
    if (a.flags != nullptr) a.flags[out_index] = (uint8_t)bits;
    if (a.stats != nullptr) {
      float *s = a.stats + out_index * 3;
      s[0] = tau;
      s[1] = r_re;
      s[2] = r_im;
    }
  }
}

constexpr int kXfer = 4 * 8 + 8;  // per-wave LDS record: sums of up to 4 channels, kept, moments

// End of a stream group: reduce the wave's partials, combine the segments
// (waves of one block), write average, weight and the adaptive state.
template <int F>
__device__ __forceinline__ void finish_stream(const ScreenArgs &a, StreamAcc<F> &acc, int64_t group,
                                              int seg, bool active, int wave, int lane,
                                              float (*xfer)[kXfer]) {
#pragma unroll
  for (int f = 0; f < F; ++f)
#pragma unroll
    for (int k = 0; k < 8; ++k) acc.sum[f][k] = group_sum<64>(acc.sum[f][k]);
  acc.kept = group_sum<64>(acc.kept);
  if (a.state != nullptr) {
#pragma unroll
    for (int mask = 1; mask < kWave; mask <<= 1)
      acc.mom = moments_merge(acc.mom, moments_shfl_xor(acc.mom, mask));
  }
  if (a.n_seg > 1) {  // uniform over the block
    constexpr int o = 8 * F;
    if (lane == 0) {
#pragma unroll
      for (int f = 0; f < F; ++f)
#pragma unroll
        for (int k = 0; k < 8; ++k) xfer[wave][8 * f + k] = acc.sum[f][k];
      xfer[wave][o] = acc.kept;
      xfer[wave][o + 1] = acc.mom.n;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        xfer[wave][o + 2 + k] = acc.mom.m[k];
        xfer[wave][o + 5 + k] = acc.mom.s[k];
      }
    }
    __syncthreads();
    if (seg == 0) {
      for (int s = 1; s < a.n_seg; ++s) {
        const float *x = xfer[wave + s];
#pragma unroll
        for (int f = 0; f < F; ++f)
#pragma unroll
          for (int k = 0; k < 8; ++k) acc.sum[f][k] += x[8 * f + k];
        acc.kept += x[o];
        Moments b;
        b.n = x[o + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          b.m[k] = x[o + 2 + k];
          b.s[k] = x[o + 5 + k];
        }
        acc.mom = moments_merge(acc.mom, b);
      }
    }
  }
  if (!active || seg != 0 || lane != 0) return;
  const float inv = acc.kept > 0.0f ? 1.0f / acc.kept : 0.0f;
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const int64_t stream = group * F + f;
    f32x4 *out = reinterpret_cast<f32x4 *>(a.avg + stream * 8);
    out[0] = f32x4{acc.sum[f][0] * inv, acc.sum[f][1] * inv, acc.sum[f][2] * inv, acc.sum[f][3] * inv};
    out[1] = f32x4{acc.sum[f][4] * inv, acc.sum[f][5] * inv, acc.sum[f][6] * inv, acc.sum[f][7] * inv};
    a.weight[stream] = acc.kept * a.invT;
  }
  if (a.state != nullptr && acc.mom.n > 0.0f) {
    StateRec *st = reinterpret_cast<StateRec *>(a.state) + group;
    StateRec r = *st;
    Moments old;
    old.n = (float)r.n;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      old.m[k] = r.mean[k];
      old.s[k] = r.m2[k];
    }
    const Moments nw = moments_merge(old, acc.mom);
    r.n += (uint32_t)acc.mom.n;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      r.mean[k] = nw.m[k];
      r.m2[k] = nw.s[k];
    }
    *st = r;
  }
}

// The tiled kernel, for power-of-two window lengths M = 2^LOG2M.
template <int FMT, int LOG2M>
__global__ void __launch_bounds__(kBlock) screen_tiled(const ScreenArgs a) {
  constexpr int K = FMT == FMT_CF32 ? 4 : 8;    // samples per lane per step
  constexpr int SB = FMT == FMT_CF32 ? 32 : 16; // bytes per sample
  constexpr int SPI = kWave * K;                // samples per step
  constexpr int M = 1 << LOG2M;
  constexpr bool LOCAL = M <= K;                // windows do not cross lanes
  constexpr int LPW = LOCAL ? 1 : (M / K < kWave ? M / K : kWave);  // lanes per window
  constexpr int IPW = M > SPI ? M / SPI : 1;    // steps per window

  __shared__ u32x4 tile[kWavesPerBlock][kTilePieces];
  __shared__ float xfer[kWavesPerBlock][kXfer];

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int64_t unit = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  const int64_t stream = unit / a.n_seg;
  const int seg = (int)(unit - stream * a.n_seg);
  const bool active = stream < a.n_groups;

  StreamAcc<1> acc{};
  if (active) {
    const Thresholds th = stream_thresholds(a, stream);
    const uint8_t *base = a.vis + (stream * a.T + (int64_t)seg * a.seg_samples) * SB;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(base), (short)0, a.seg_samples * SB, kRsrcWord3);
    const int n_steps = (a.seg_samples + SPI - 1) / SPI;
    const int64_t out_base = stream * a.nW + (int64_t)seg * a.seg_windows;
    u32x4 *my_tile = tile[wave];

    u32x4 buf[kPieces];
    auto issue = [&](int step) {
#pragma unroll
      for (int i = 0; i < kPieces; ++i)
        buf[i] = __builtin_bit_cast(
            u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                       rsrc, (unsigned)(step * SPI * SB + (i * kWave + lane) * 16), 0, kLoadStreaming));
    };

    float ws[8] = {}, wr[1][8] = {};
    issue(0);
    for (int step = 0; step < n_steps; ++step) {
      wave_lds_order();
#pragma unroll
      for (int i = 0; i < kPieces; ++i) my_tile[lds_slot(i * kWave + lane)] = buf[i];
      wave_lds_order();
      if (step + 1 < n_steps) issue(step + 1);

#pragma unroll
      for (int j = 0; j < K; ++j) {
        float x[8];
        if constexpr (FMT == FMT_CF32) {
          const f32x4 lo = __builtin_bit_cast(f32x4, my_tile[lds_slot(kPieces * lane + 2 * j)]);
          const f32x4 hi = __builtin_bit_cast(f32x4, my_tile[lds_slot(kPieces * lane + 2 * j + 1)]);
          x[0] = lo[0]; x[1] = lo[1]; x[2] = lo[2]; x[3] = lo[3];
          x[4] = hi[0]; x[5] = hi[1]; x[6] = hi[2]; x[7] = hi[3];
        } else {
          const f16x8 h = __builtin_bit_cast(f16x8, my_tile[lds_slot(kPieces * lane + j)]);
#pragma unroll
          for (int k = 0; k < 8; ++k) x[k] = (float)h[k];
        }
        accumulate_sample(ws, wr[0], x, a.eps);
        if constexpr (LOCAL) {
          if ((j + 1) % M == 0) {
            const int w = (step * SPI + lane * K) / M + j / M;
            finish_window<1>(a, th, ws, wr, out_base + w, w < a.seg_windows, true, acc);
#pragma unroll
            for (int k = 0; k < 8; ++k) ws[k] = wr[0][k] = 0.0f;
          }
        }
      }
      if constexpr (!LOCAL) {
        if ((step + 1) % IPW == 0) {
          float tot[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) tot[k] = group_sum<LPW>(ws[k]);
          const int w = ((step + 1 - IPW) * SPI + lane * K) / M;
          finish_window<1>(a, th, tot, wr, out_base + w, w < a.seg_windows, lane % LPW == 0, acc);
#pragma unroll
          for (int k = 0; k < 8; ++k) ws[k] = wr[0][k] = 0.0f;
        }
      }
    }
  }
  finish_stream<1>(a, acc, stream, seg, active, wave, lane, xfer);
}

// Any window length (M >= 2, including M that is not a power of two) and
// time x frequency windows of F = 1, 2 or 4 adjacent channels: one wave per
// channel group, one lane per window, samples read directly.  Slower than the
// tiled kernel; used for the shapes the tiled kernel does not cover.
template <int FMT, int F>
__global__ void __launch_bounds__(kBlock) screen_generic(const ScreenArgs a) {
  constexpr int SB = FMT == FMT_CF32 ? 32 : 16;
  __shared__ float xfer[kWavesPerBlock][kXfer];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int64_t group = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  const bool active = group < a.n_groups;
  StreamAcc<F> acc{};
  if (active) {
    const Thresholds th = stream_thresholds(a, group);
    const uint8_t *base = a.vis + group * F * (int64_t)a.T * SB;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(base), (short)0, F * a.T * SB, kRsrcWord3);
    for (int w = lane; w < a.nW; w += kWave) {
      float ws[8] = {}, wr[F][8] = {};
#pragma unroll
      for (int f = 0; f < F; ++f) {
        for (int t = 0; t < a.M; ++t) {
          const unsigned off = (unsigned)((f * a.T + w * a.M + t) * SB);
          float x[8];
          if constexpr (FMT == FMT_CF32) {
            const f32x4 lo = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, kLoadStreaming));
            const f32x4 hi = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off + 16, 0, kLoadStreaming));
            x[0] = lo[0]; x[1] = lo[1]; x[2] = lo[2]; x[3] = lo[3];
            x[4] = hi[0]; x[5] = hi[1]; x[6] = hi[2]; x[7] = hi[3];
          } else {
            const f16x8 h = __builtin_bit_cast(f16x8, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, kLoadStreaming));
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = (float)h[k];
          }
          accumulate_sample(ws, wr[f], x, a.eps);
        }
      }
      finish_window<F>(a, th, ws, wr, group * a.nW + w, true, true, acc);
    }
  }
  finish_stream<F>(a, acc, group, 0, active, wave, lane, xfer);
}

template <int FMT, int LOG2M>
hipError_t launch_tiled(const ScreenArgs &a, hipStream_t stream) {
  const int64_t units = a.n_groups * a.n_seg;
  const int64_t blocks = (units + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((screen_tiled<FMT, LOG2M>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, a);
  return hipGetLastError();
}

template <int FMT>
hipError_t dispatch_tiled(int log2m, const ScreenArgs &a, hipStream_t stream) {
  switch (log2m) {
    case 1: return launch_tiled<FMT, 1>(a, stream);
    case 2: return launch_tiled<FMT, 2>(a, stream);
    case 3: return launch_tiled<FMT, 3>(a, stream);
    case 4: return launch_tiled<FMT, 4>(a, stream);
    case 5: return launch_tiled<FMT, 5>(a, stream);
    case 6: return launch_tiled<FMT, 6>(a, stream);
    case 7: return launch_tiled<FMT, 7>(a, stream);
    case 8: return launch_tiled<FMT, 8>(a, stream);
    case 9: return launch_tiled<FMT, 9>(a, stream);
    case 10: return launch_tiled<FMT, 10>(a, stream);
    case 11: return launch_tiled<FMT, 11>(a, stream);
    case 12: return launch_tiled<FMT, 12>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int FMT>
hipError_t launch_generic(const ScreenArgs &a, hipStream_t stream) {
  const int64_t blocks = (a.n_groups + kWavesPerBlock - 1) / kWavesPerBlock;
  const dim3 grid((unsigned)blocks), block(kBlock);
  switch (a.F) {
    case 1: hipLaunchKernelGGL((screen_generic<FMT, 1>), grid, block, 0, stream, a); break;
    case 2: hipLaunchKernelGGL((screen_generic<FMT, 2>), grid, block, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((screen_generic<FMT, 4>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int ilog2_exact(int m) {
  int l = 0;
  while ((1 << l) < m) ++l;
  return (1 << l) == m ? l : -1;
}

// ----------------------------------------------------------------------------- probes

constexpr int kProbeBlocks = 4096;

__global__ void __launch_bounds__(kBlock) probe_read_kernel(const u32x4 *src, size_t n16, float *sink) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  u32x4 acc = {0u, 0u, 0u, 0u};
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const u32x4 v0 = __builtin_nontemporal_load(src + i);
    const u32x4 v1 = __builtin_nontemporal_load(src + i + stride);
    const u32x4 v2 = __builtin_nontemporal_load(src + i + 2 * stride);
    const u32x4 v3 = __builtin_nontemporal_load(src + i + 3 * stride);
    acc ^= v0 ^ v1 ^ v2 ^ v3;
  }
  for (; i < n16; i += stride) acc ^= __builtin_nontemporal_load(src + i);
  unsigned x = acc[0] ^ acc[1] ^ acc[2] ^ acc[3];
  for (int m = 1; m < kWave; m <<= 1) x ^= __shfl_xor(x, m);
  if ((threadIdx.x % kWave) == 0)
    sink[(size_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave] = __builtin_bit_cast(float, x);
}

__global__ void __launch_bounds__(kBlock) probe_copy_kernel(u32x4 *dst, const u32x4 *src, size_t n16) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

int tiled_samples_per_lane(int fmt) { return fmt == FMT_CF32 ? 4 : 8; }

bool tiled_supports(int M) {
  const int l = ilog2_exact(M);
  return l >= 1 && l <= kMaxTiledLog2M;
}

hipError_t launch_screen(int fmt, const ScreenArgs &a, hipStream_t stream) {
  const int l = ilog2_exact(a.M);
  const bool tiled = a.F == 1 && l >= 1 && l <= kMaxTiledLog2M;
  if (fmt == FMT_CF32) return tiled ? dispatch_tiled<FMT_CF32>(l, a, stream) : launch_generic<FMT_CF32>(a, stream);
  if (fmt == FMT_CF16) return tiled ? dispatch_tiled<FMT_CF16>(l, a, stream) : launch_generic<FMT_CF16>(a, stream);
  return hipErrorInvalidValue;
}

size_t probe_sink_floats() { return (size_t)kProbeBlocks * kWavesPerBlock; }

hipError_t launch_probe_read(const void *src, size_t bytes, float *sink, hipStream_t stream) {
  hipLaunchKernelGGL(probe_read_kernel, dim3(kProbeBlocks), dim3(kBlock), 0, stream,
                     static_cast<const u32x4 *>(src), bytes / 16, sink);
  return hipGetLastError();
}

hipError_t launch_probe_copy(void *dst, const void *src, size_t bytes, hipStream_t stream) {
  hipLaunchKernelGGL(probe_copy_kernel, dim3(kProbeBlocks), dim3(kBlock), 0, stream,
                     static_cast<u32x4 *>(dst), static_cast<const u32x4 *>(src), bytes / 16);
  return hipGetLastError();
}

}  // namespace rfi
