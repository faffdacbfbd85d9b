// screen.hip -- gfx950 kernels of the online energy + polarisation RFI screen
// (arXiv 2412.14775, Section 2, Tables 1-2).
//
// Five kernels share the per-sample and per-window code below (kernel_for picks one):
//   screen_tiled       time-only windows of M = 2^k <= 4096 samples (the hot path);
//   screen_windows     windows of M = K S samples x F channels (non-power-of-two M and
//                      the paper's time x frequency windows), optionally in the
//                      paper's mixed precision (Tables 3-4);
//   screen_long        time-only windows of more than half a step, edges anywhere;
//   screen_wide        time x frequency windows wider than 64 lanes of runs of 8
//                      samples, a window over several steps of one channel each;
//   screen_wide_pairs  the same over four channels whose runs fit 32 lanes, two
//                      channels per step.
//
// screen_tiled, one pass over the visibilities, bound by HBM bandwidth:
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
// reproducible run to run (the same plan, shape and device: a persistent launch that
// splits a channel group between two waves adds their partial sums in its own order).

#include <algorithm>

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

// Running (count, mean, sum of squared deviations) of the three statistics over one
// integration's clean windows (float32 sums; the count is exact).
struct Moments {
  uint32_t n;
  float m[3];
  float s[3];
};

__device__ __forceinline__ void moments_push(Moments &a, float x0, float x1, float x2) {
  a.n += 1u;
  const float inv = 1.0f / (float)a.n;
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
  const uint32_t n = a.n + b.n;
  if (n == 0u) return a;
  const float fb = (float)b.n / (float)n;
  const float cross = (float)a.n * fb;
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
  b.n = (uint32_t)__shfl_xor((int)a.n, mask);
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
    const StateRec &st = a.state[stream];
    const uint64_t n = st.n;
    const uint64_t warm = a.n_warm > 2 ? (uint64_t)a.n_warm : 2u;
    if (n >= warm) {  // float64 like the state; the comparisons are float32
      const double inv = 1.0 / (double)(n - 1);
      const double sd0 = sqrt(st.m2[0] * inv);
      const double sd1 = sqrt(st.m2[1] * inv);
      const double sd2 = sqrt(st.m2[2] * inv);
      t.s_low = (float)(st.mean[0] - (double)a.kappa_sk * sd0);
      t.s_high = (float)(st.mean[0] + (double)a.kappa_sk * sd0);
      t.g_re = (float)(st.mean[1] + (double)a.kappa_ds * sd1);
      t.g_im = (float)(st.mean[2] + (double)a.kappa_ds * sd2);
    }
  }
  return t;
}

// The integration's moments b merged into the stream's state (Chan, Golub & LeVeque), in
// float64 with the exact count: n' = n + n_b, mean' = mean + delta n_b / n',
// M2' = M2 + M2_b + delta^2 n n_b / n'.
__device__ __forceinline__ void state_merge(StateRec *st, const Moments &b) {
  StateRec r = *st;
  const double fb = (double)b.n / (double)(r.n + b.n);
  const double cross = (double)r.n * fb;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double d = (double)b.m[k] - r.mean[k];
    r.mean[k] += d * fb;
    r.m2[k] += (double)b.s[k] + d * d * cross;
  }
  r.n += b.n;
  *st = r;
}

// x into the running sum s; FIRST: s is still empty and takes x itself (the same value as
// 0 + x, without the zero)
template <bool FIRST>
__device__ __forceinline__ void add_to(float &s, float x) {
  if constexpr (FIRST)
    s = x;
  else
    s += x;
}

// Per-sample terms of Tables 1 and 2 from one sample's Stokes parameters (eq. IQUV),
// added to the window sums ws = (S1, S2, sum q^, u^, v^ of Re, of Im).
template <bool FIRST = false>
__device__ __forceinline__ void accumulate_stokes(float ws[8], float Ir, float Ii, float Qr, float Qi,
                                                  float Ur, float Ui, float Vr, float Vi, float eps) {
  const float y = Ir * Ir + Ii * Ii;
  add_to<FIRST>(ws[0], hw_sqrt(y));
  add_to<FIRST>(ws[1], y);
  const float rr = hw_rcp(hw_sqrt(Qr * Qr + Ur * Ur + Vr * Vr) + eps);
  add_to<FIRST>(ws[2], Qr * rr);
  add_to<FIRST>(ws[3], Ur * rr);
  add_to<FIRST>(ws[4], Vr * rr);
  const float ri = hw_rcp(hw_sqrt(Qi * Qi + Ui * Ui + Vi * Vi) + eps);
  add_to<FIRST>(ws[5], Qi * ri);
  add_to<FIRST>(ws[6], Ui * ri);
  add_to<FIRST>(ws[7], Vi * ri);
}

// One sample: Stokes parameters and the per-sample terms into ws, the sample itself
// into the raw sums wr.  x = (xx_re, xx_im, xy_re, xy_im, yx_re, yx_im, yy_re, yy_im).
template <bool FIRST = false>
__device__ __forceinline__ void accumulate_sample(float ws[8], float wr[8], const float x[8],
                                                  float eps) {
  accumulate_stokes<FIRST>(ws, x[0] + x[6], x[1] + x[7], x[0] - x[6], x[1] - x[7], x[2] + x[4], x[3] + x[5],
                           x[5] - x[3], x[2] - x[4], eps);  // I, Q, U, V = j (xy - yx)
#pragma unroll
  for (int k = 0; k < 8; ++k) add_to<FIRST>(wr[k], x[k]);
}

// Sums and differences of binary16 halves of 32-bit words (half 0 = the low one) in
// float32 with one rounding, by v_fma_mix_f32, which takes binary16 operands converted
// exactly: mix_add<SA, SB>(a, b) == (float)a_SA + (float)b_SB bit for bit, and so on.
template <int SA, int SB>
__device__ __forceinline__ float mix_add(uint32_t a, uint32_t b) {
  float d;
  asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[%3,0,%4] op_sel_hi:[1,0,1]" : "=v"(d) : "v"(a), "v"(b), "n"(SA), "n"(SB));
  return d;
}
template <int SA, int SB>
__device__ __forceinline__ float mix_sub(uint32_t a, uint32_t b) {  // a_SA - b_SB
  float d;
  asm("v_fma_mix_f32 %0, %2, -1.0, %1 op_sel:[%4,0,%3] op_sel_hi:[1,0,1]" : "=v"(d) : "v"(a), "v"(b), "n"(SA), "n"(SB));
  return d;
}
template <int SA>
__device__ __forceinline__ float mix_acc(float acc, uint32_t a) {  // acc + a_SA
  asm("v_fma_mix_f32 %0, %1, 1.0, %0 op_sel:[%2,0,0] op_sel_hi:[1,0,0]" : "+v"(acc) : "v"(a), "n"(SA));
  return acc;
}
template <int SA>
__device__ __forceinline__ float mix_cvt(uint32_t a) {  // a_SA (0 + a_SA)
  float d;
  asm("v_fma_mix_f32 %0, %1, 1.0, 0 op_sel:[%2,0,0] op_sel_hi:[1,0,0]" : "=v"(d) : "v"(a), "n"(SA));
  return d;
}
template <bool FIRST, int SA>
__device__ __forceinline__ void mix_add_to(float &s, uint32_t a) {
  if constexpr (FIRST)
    s = mix_cvt<SA>(a);
  else
    s = mix_acc<SA>(s, a);
}

// accumulate_sample for a complex-half sample as it sits in memory (words xx, xy, yx,
// yy; real part in the low half), without separate conversions: the same float32
// results bit for bit, with 8 fewer VALU operations per sample.
template <bool FIRST = false>
__device__ __forceinline__ void accumulate_sample_h(float ws[8], float wr[8], u32x4 h, float eps) {
  accumulate_stokes<FIRST>(ws, mix_add<0, 0>(h.x, h.w), mix_add<1, 1>(h.x, h.w), mix_sub<0, 0>(h.x, h.w),
                           mix_sub<1, 1>(h.x, h.w), mix_add<0, 0>(h.y, h.z), mix_add<1, 1>(h.y, h.z),
                           mix_sub<1, 1>(h.z, h.y), mix_sub<0, 0>(h.y, h.z), eps);
  mix_add_to<FIRST, 0>(wr[0], h.x);
  mix_add_to<FIRST, 1>(wr[1], h.x);
  mix_add_to<FIRST, 0>(wr[2], h.y);
  mix_add_to<FIRST, 1>(wr[3], h.y);
  mix_add_to<FIRST, 0>(wr[4], h.z);
  mix_add_to<FIRST, 1>(wr[5], h.z);
  mix_add_to<FIRST, 0>(wr[6], h.w);
  mix_add_to<FIRST, 1>(wr[7], h.w);
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
__device__ __forceinline__ void mixed_statistics(const ScreenArgs &a, const float tot[8], float &tau, float &r_re,
                                                 float &r_im);

template <int F, bool MIXED = false>
__device__ __forceinline__ void finish_window(const ScreenArgs &a, const Thresholds &th,
                                              const float tot[8], const float (*wr)[8],
                                              int64_t out_index, bool valid, bool leader,
                                              StreamAcc<F> &acc, uint8_t *lds_flags = nullptr,
                                              int64_t lds_first = 0) {
  float tau, r_re, r_im;
  if constexpr (MIXED) {
    mixed_statistics(a, tot, tau, r_re, r_im);
  } else {
    // hardware reciprocal and square root (1 ulp), as per sample: a correctly rounded
    // division and sqrt cost about a quarter of a window's finish, which the windowed
    // complex-half kernels feel (2 %)
    tau = a.pre * (a.Wf * tot[1] * hw_rcp(tot[0] * tot[0] + a.eps) - 1.0f);
    r_re = hw_sqrt(tot[2] * tot[2] + tot[3] * tot[3] + tot[4] * tot[4]) * a.invW;
    r_im = hw_sqrt(tot[5] * tot[5] + tot[6] * tot[6] + tot[7] * tot[7]) * a.invW;
  }
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
    if (a.flags != nullptr) {
      if (lds_flags != nullptr)  // held in LDS (persistent tiled kernel), index from lds_first
        lds_flags[out_index - lds_first] = (uint8_t)bits;
      else
        a.flags[out_index] = (uint8_t)bits;
    }
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
                                              float (*xfer)[kXfer], float *lds_out = nullptr,
                                              int64_t lds_first = 0) {
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
      xfer[wave][o + 1] = __uint_as_float(acc.mom.n);
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
        b.n = __float_as_uint(x[o + 1]);
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
  if (F == 1 && lds_out != nullptr) {
    float *o = lds_out + (group - lds_first) * 9;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = acc.sum[0][k] * inv;
    o[8] = acc.kept * a.invT;
    if (a.state != nullptr && acc.mom.n > 0u) state_merge(a.state + group, acc.mom);
    return;
  }
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const int64_t stream = group * F + f;
    f32x4 *out = reinterpret_cast<f32x4 *>(a.avg + stream * 8);
    out[0] = f32x4{acc.sum[f][0] * inv, acc.sum[f][1] * inv, acc.sum[f][2] * inv, acc.sum[f][3] * inv};
    out[1] = f32x4{acc.sum[f][4] * inv, acc.sum[f][5] * inv, acc.sum[f][6] * inv, acc.sum[f][7] * inv};
    a.weight[stream] = acc.kept * a.invT;
  }
  if (a.state != nullptr && acc.mom.n > 0u) state_merge(a.state + group, acc.mom);
}

// The tiled kernel, for power-of-two window lengths M = 2^LOG2M.  One wave per stream
// segment; or, PERSIST, block b screens the whole streams [b U, (b + 1) U) (wave w every
// fourth of them from b U + w) and keeps their flags, averages and weights in LDS until the
// last is done, then writes them in one pass: bytes written back to HBM while the reads
// stream cost many times their size, written after them hardly anything (the averages and
// weights, 36 bytes a stream, +0.8-1.1 % held back).
template <int FMT, int LOG2M, bool PERSIST>
__global__ void __launch_bounds__(kBlock) screen_tiled(const ScreenArgs a, int U, int hold_avg) {
  constexpr int K = FMT == FMT_CF32 ? 4 : 8;    // samples per lane per step
  constexpr int SB = FMT == FMT_CF32 ? 32 : 16; // bytes per sample
  constexpr int SPI = kWave * K;                // samples per step
  constexpr int M = 1 << LOG2M;
  constexpr bool LOCAL = M <= K;                // windows do not cross lanes
  constexpr int LPW = LOCAL ? 1 : (M / K < kWave ? M / K : kWave);  // lanes per window
  constexpr int IPW = M > SPI ? M / SPI : 1;    // steps per window

  __shared__ u32x4 tile[kWavesPerBlock][kTilePieces];
  __shared__ float xfer[kWavesPerBlock][kXfer];
  extern __shared__ __align__(16) uint8_t block_flags[];  // PERSIST: U nW flag bytes, then 9 floats a stream

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int64_t first = PERSIST ? (int64_t)blockIdx.x * U : 0;  // the block's streams (PERSIST)
  const int64_t last = PERSIST ? min(first + (int64_t)U, a.n_groups) : 0;
  for (int64_t unit = PERSIST ? first + wave : (int64_t)blockIdx.x * kWavesPerBlock + wave;;
       unit += kWavesPerBlock) {
    const int64_t stream = PERSIST ? unit : unit / a.n_seg;
    const int seg = PERSIST ? 0 : (int)(unit - stream * a.n_seg);
    const bool active = stream < (PERSIST ? last : a.n_groups);
    if (PERSIST && !active) break;

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
                         rsrc, (unsigned)(step * SPI * SB) + (unsigned)((i * kWave + lane) * 16), 0, kLoadStreaming));
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
          if constexpr (FMT == FMT_CF32) {
            const f32x4 lo = __builtin_bit_cast(f32x4, my_tile[lds_slot(kPieces * lane + 2 * j)]);
            const f32x4 hi = __builtin_bit_cast(f32x4, my_tile[lds_slot(kPieces * lane + 2 * j + 1)]);
            const float x[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            accumulate_sample(ws, wr[0], x, a.eps);
          } else {
            accumulate_sample_h(ws, wr[0], my_tile[lds_slot(kPieces * lane + j)], a.eps);
          }
          if constexpr (LOCAL) {
            if ((j + 1) % M == 0) {
              const int w = (step * SPI + lane * K) / M + j / M;
              finish_window<1>(a, th, ws, wr, out_base + w, w < a.seg_windows, true, acc,
                               PERSIST ? block_flags : nullptr, first * a.nW);
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
            finish_window<1>(a, th, tot, wr, out_base + w, w < a.seg_windows, lane % LPW == 0, acc,
                             PERSIST ? block_flags : nullptr, first * a.nW);
#pragma unroll
            for (int k = 0; k < 8; ++k) ws[k] = wr[0][k] = 0.0f;
          }
        }
      }
    }
    finish_stream<1>(a, acc, stream, seg, active, wave, lane, xfer,
                     PERSIST && hold_avg ? reinterpret_cast<float *>(block_flags + ((U * a.nW + 15) & ~15)) : nullptr,
                     first);
    if (!PERSIST) break;
  }
  if constexpr (PERSIST) {
    __syncthreads();
    if (a.flags != nullptr) {
      const int64_t base = first * a.nW, n = (last - first) * a.nW;
      for (int64_t i = threadIdx.x; i < n; i += kBlock) a.flags[base + i] = block_flags[i];
    }
    const float *bo = reinterpret_cast<const float *>(block_flags + ((U * a.nW + 15) & ~15));
    for (int64_t i = threadIdx.x; hold_avg && i < last - first; i += kBlock) {
      const float *o = bo + i * 9;
      f32x4 *out = reinterpret_cast<f32x4 *>(a.avg + (first + i) * 8);
      out[0] = f32x4{o[0], o[1], o[2], o[3]};
      out[1] = f32x4{o[4], o[5], o[6], o[7]};
      a.weight[first + i] = o[8];
    }
  }
}

// Windows of more than a quarter of a step of samples (K 64 / 4) of one channel, any
// such M: the window edges may fall anywhere inside a step, at most four per step.
// Same loads and LDS transpose as the tiled kernel; a step that lies inside the
// current window, or ends exactly where it does, is summed without per-sample tests.
// In a step with an edge inside it the lanes take runs of K + 1 samples that do not
// cross an edge: the first lanes the samples that close this window, the next ones
// each window that lies wholly in the step (up to three), the others those that open
// the next window (at most 62 lanes), so the step costs K + 1 sample slots instead of
// the 2 K of two masked passes over every lane, plus one wave reduction per window
// it closes.  Each lane adds its step sums plainly for kFold steps before folding them into
// the window sums, so no lane sums more than kFold K samples in a row whatever M is.
//
// MAXW: the most windows that lie wholly inside one step for this M (1 when 2 M > a step,
// 2 when 3 M > a step, else 3 above a quarter of a step): the edge step is unrolled for that
// many.  The launch takes only windows of more than half a step (MAXW = 1): every shorter
// length has a lane layout in the windowed kernel (runs of up to 8 samples, padded), which
// screens it 1-45 % faster than this kernel did (complex half M = 131-500 0.51-0.69 -> 0.73-0.80
// of the HBM peak, complex64 M = 67-193 0.62-0.80 -> 0.82-0.83).
template <int FMT, int MAXW>
__global__ void __launch_bounds__(kBlock) screen_long(const ScreenArgs a) {
  constexpr int K = FMT == FMT_CF32 ? 4 : 8;
  constexpr int SB = FMT == FMT_CF32 ? 32 : 16;
  constexpr int SPI = kWave * K;
  constexpr int kFold = 16;

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
                       rsrc, (unsigned)(step * SPI * SB) + (unsigned)((i * kWave + lane) * 16), 0, kLoadStreaming));
    };
    // sample t of the step (t = K lane + j in the plain steps), from the LDS tile
    auto sample = [&](int t, float ps[8], float pr[8]) {
      if constexpr (FMT == FMT_CF32) {
        const f32x4 lo = __builtin_bit_cast(f32x4, my_tile[lds_slot(2 * t)]);
        const f32x4 hi = __builtin_bit_cast(f32x4, my_tile[lds_slot(2 * t + 1)]);
        const float x[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        accumulate_sample(ps, pr, x, a.eps);
      } else {
        accumulate_sample_h(ps, pr, my_tile[lds_slot(t)], a.eps);
      }
    };

    float ps[8] = {}, pr[8] = {};      // plain sums since the last fold
    float ss[8] = {}, sr[1][8] = {};   // the current window's sums
    int since_fold = 0;
    auto fold = [&]() {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        ss[k] += ps[k];
        sr[0][k] += pr[k];
        ps[k] = pr[k] = 0.0f;
      }
      since_fold = 0;
    };
    int w = 0;                  // current window, counted from the segment start
    int w_end = a.M;            // one past its last sample, from the segment start
    issue(0);
    for (int step = 0; step < n_steps; ++step) {
      wave_lds_order();
#pragma unroll
      for (int i = 0; i < kPieces; ++i) my_tile[lds_slot(i * kWave + lane)] = buf[i];
      wave_lds_order();
      if (step + 1 < n_steps) issue(step + 1);

      auto close_window = [&]() {            // window w ends in this step: reduce, finish
        fold();
        float tot[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) tot[k] = group_sum<kWave>(ss[k]);
        finish_window<1>(a, th, tot, sr, out_base + w, w < a.seg_windows, lane == 0, acc);
#pragma unroll
        for (int k = 0; k < 8; ++k) ss[k] = sr[0][k] = 0.0f;
        ++w;
        w_end += a.M;
      };
      const int n1 = w_end - step * SPI;     // samples of the step in window w (uniform)
      if (n1 >= SPI) {                       // the step lies inside the window, or ends it
#pragma unroll
        for (int j = 0; j < K; ++j) sample(lane * K + j, ps, pr);
        if (n1 == SPI) close_window();
      } else {
        // Pieces of the step: 0, the last n1 samples of window w; 1 .. nw, windows that lie
        // wholly in the step (nw <= MAXW); nw + 1, the first
        // samples of the window that goes on into the next step.  Each piece gets lanes
        // with runs of C samples, in order.
        constexpr int C = K + 1;
        const int nw = (SPI - n1) / a.M;       // uniform
        int piece = -1, lo = SPI, hi = SPI;    // lanes past the last piece take nothing
        int lanes_before = 0;
#pragma unroll
        for (int p = 0; p < MAXW + 2; ++p) {
          const int start = p == 0 ? 0 : min(n1 + (p - 1) * a.M, SPI);
          const int end = p == 0 ? n1 : (p <= nw ? n1 + p * a.M : SPI);
          const int lanes = (end - start + C - 1) / C;
          if (lane >= lanes_before && lane < lanes_before + lanes) {
            piece = p;
            lo = start + (lane - lanes_before) * C;
            hi = min(lo + C, end);
          }
          lanes_before += lanes;
        }
        float cs[8] = {}, cr[8] = {};
#pragma unroll
        for (int j = 0; j < C; ++j)
          if (lo + j < hi) sample(lo + j, cs, cr);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          ps[k] += piece == 0 ? cs[k] : 0.0f;
          pr[k] += piece == 0 ? cr[k] : 0.0f;
        }
        close_window();
#pragma unroll
        for (int p = 1; p <= MAXW; ++p) {
          if (p <= nw) {                       // window w lies in piece p (uniform)
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              ss[k] = piece == p ? cs[k] : 0.0f;
              sr[0][k] = piece == p ? cr[k] : 0.0f;
            }
            close_window();
          }
        }
        if (w < a.seg_windows) {               // piece nw + 1 opens the next window
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            ps[k] = piece == nw + 1 ? cs[k] : 0.0f;
            pr[k] = piece == nw + 1 ? cr[k] : 0.0f;
          }
        }
      }
      if (++since_fold == kFold) fold();
    }
  }
  finish_stream<1>(a, acc, stream, seg, active, wave, lane, xfer);
}

// ----------------------------------------------------------------------------- paper's mixed precision
// Tables 3-4: per-sample groups and the SK moments in FP32; the sums of the unit
// vectors, their squares, r and its comparison, and the SK ratio and its
// comparison in FP16 (every FP16 operation rounds its result to binary16; FP32
// inputs are converted first).

__device__ __forceinline__ float round16(float x) { return (float)(_Float16)x; }

// As accumulate_sample, but the unit-vector sums (Table 2 group 4) accumulate in FP16.
__device__ __forceinline__ void accumulate_sample_mixed(float ws[8], float wr[8], const float x[8], float eps) {
  const float Ir = x[0] + x[6], Ii = x[1] + x[7];
  const float Qr = x[0] - x[6], Qi = x[1] - x[7];
  const float Ur = x[2] + x[4], Ui = x[3] + x[5];
  const float Vr = x[5] - x[3], Vi = x[2] - x[4];
  const float y = Ir * Ir + Ii * Ii;
  ws[0] += hw_sqrt(y);
  ws[1] += y;
  const float rr = hw_rcp(hw_sqrt(Qr * Qr + Ur * Ur + Vr * Vr) + eps);
  const float ri = hw_rcp(hw_sqrt(Qi * Qi + Ui * Ui + Vi * Vi) + eps);
  ws[2] = round16(ws[2] + round16(Qr * rr));
  ws[3] = round16(ws[3] + round16(Ur * rr));
  ws[4] = round16(ws[4] + round16(Vr * rr));
  ws[5] = round16(ws[5] + round16(Qi * ri));
  ws[6] = round16(ws[6] + round16(Ui * ri));
  ws[7] = round16(ws[7] + round16(Vi * ri));
#pragma unroll
  for (int k = 0; k < 8; ++k) wr[k] += x[k];
}

// One butterfly level of the window sums v[0..7] over aligned groups of lanes (the partner
// of each lane by the DPP control CTRL, or lane ^ XOR when CTRL is 0).  Sums R16 .. 7 round
// each addition to binary16 (the paper's mixed precision: R16 = 2, else 8 for none).
template <int CTRL, int XOR, int R16>
__device__ __forceinline__ void group_level8(float v[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float o = CTRL != 0 ? dpp_mov<CTRL>(v[e]) : __shfl_xor(v[e], XOR);
    v[e] = e >= R16 ? round16(v[e] + o) : v[e] + o;
  }
}

// The eight window sums over aligned groups of L lanes, L a run-time power of two (uniform):
// one branch per level rather than per sum and level.  Every lane of a group receives the
// same totals, as group_sum gives them.
template <int R16>
__device__ __forceinline__ void group_sum8_rt(float v[8], int L) {
  if (L >= 2) group_level8<0xB1, 0, R16>(v);
  if (L >= 4) group_level8<0x4E, 0, R16>(v);
  if (L >= 8) group_level8<0x141, 0, R16>(v);
  if (L >= 16) group_level8<0x140, 0, R16>(v);
  if (L >= 32) group_level8<0, 16, R16>(v);
  if (L >= 64) group_level8<0, 32, R16>(v);
}

// tau, r_re, r_im from window totals in the mixed precision.
__device__ __forceinline__ void mixed_statistics(const ScreenArgs &a, const float tot[8], float &tau, float &r_re,
                                                 float &r_im) {
  const float s12 = tot[0] * tot[0];                                   // group 6, FP32
  const float num = round16(round16(a.Wf) * round16(tot[1]));          // group 7, FP16
  const float den = round16(round16(s12) + 0.0009765625f);             //   eps = 2^-10
  const float ratio = round16(num / den);
  tau = round16(round16(a.pre) * round16(ratio - 1.0f));
  auto r16 = [&](float q, float u, float v) {
    float sq = round16(round16(q * q) + round16(u * u));               // group 5, FP16
    sq = round16(sq + round16(v * v));
    return round16(round16(sqrtf(sq)) / round16(a.Wf));                // group 6, FP16
  };
  r_re = r16(tot[2], tot[3], tot[4]);
  r_im = r16(tot[5], tot[6], tot[7]);
}

// Windows of M time samples x F channels on lane groups: each channel of a window is
// cut into S runs of C consecutive samples (C <= 8, F S <= 64), one lane per run, and a
// window owns L lanes, F S rounded up to a power of two; lane l = (j L + f S + s) owns run
// s of channel f of window j of the step, so a lane stays on one channel and keeps one
// masked sum.  A step covers 64 / L windows: for each channel a contiguous run of their
// samples, loaded coalesced (channel-major) into the wave's LDS tile and read back per
// lane, then summed over the L lanes of each window with a DPP butterfly.
//   PAD = false: M = C S exactly and F S = L (every lane holds C samples of its window);
//       the tile holds the step's pieces in load order.
//   PAD = true: any M with S = ceil(M / C); the last run of each channel holds
//       M - (S - 1) C samples and the L - F S lanes left over in each group neither read
//       nor add.  In the tile each channel of a window takes S C samples, the samples past
//       M are zeros (written once; a zero sample adds exactly zero to every window sum and
//       raw sum), so every lane reads C samples without tests.  Each lane's load offsets and
//       tile slots are fixed for the kernel and computed once; the step offset is a scalar.
//       The channel sums at the end are masked wave sums.
//   PERSIST = false: one wave per channel group.  PERSIST = true: a block screens a range of
//       groups and holds their flags, averages and weights in LDS until it is done (the
//       persistent branch at the end of the kernel).
template <int FMT, int C, int F, bool MIXED, bool PAD, bool PERSIST>
__global__ void __launch_bounds__(kBlock) screen_windows(const ScreenArgs a, int U) {
  constexpr int SB = FMT == FMT_CF32 ? 32 : 16;
  constexpr int PPS = SB / 16;                  // 16-byte pieces per sample
  constexpr int P = C * PPS;                    // pieces per lane per step (at most, PAD)
  constexpr int CH_PIECES = kWave * P / F;      // pieces of one channel per step (!PAD)
  constexpr int CH_SAMPLES = kWave * C / F;     // samples of one channel per step (!PAD)
  static_assert(!(MIXED && PAD), "the paper's mixed precision runs on whole lane groups");
  __shared__ u32x4 tile[kWavesPerBlock][kWave * P];
  extern __shared__ __align__(16) uint8_t block_flags[];  // PERSIST: flag bytes, then 9 floats a stream

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int S = PAD ? (a.M + C - 1) / C : a.M / C;   // lanes per channel of a window
  const int FS = F * S;                         // lanes that hold samples
  int L = FS;                                   // lanes per window
  if constexpr (PAD) L = FS > 1 ? 1 << (32 - __builtin_clz(FS - 1)) : 1;
  const int g = lane % L;
  const bool act = !PAD || g < FS;              // lane holds samples
  const int j = lane / L, f = act ? g / S : 0, s = act ? g % S : 0;
  const int wps = kWave / L;                    // windows per step
  const int ch_samples = PAD ? wps * a.M : CH_SAMPLES;    // samples of one channel per step
  const int ch_tile = PAD ? wps * S * C * PPS : CH_PIECES; // tile pieces of one channel
  const int n_steps = (a.nW + wps - 1) / wps;
  u32x4 *my_tile = tile[wave];

  // Piece i of a step is piece q = i 64 + lane of the step's F channel runs (channel-major),
  // q < n_load: its byte offset in the group (the step adds ch_samples SB as a scalar) and,
  // PAD, its tile slot (otherwise slot q).  Both are fixed for the kernel.  A piece past the
  // end of a channel (ragged last step) belongs to no valid window: past the group's buffer the
  // hardware bounds check returns zeros without a memory access; inside it (F > 1, the end of a
  // channel that is not the last) the last step leaves the piece unread.
  int voff[P], slot[PAD ? P : 1], tpos[F > 1 ? P : 1];
  const int n_load = F * ch_samples * PPS;      // !PAD: 64 P
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int q = i * kWave + lane;
    voff[i] = 0;
    if constexpr (F > 1) tpos[i] = 0;
    if constexpr (PAD) {
      slot[i] = -1;
      my_tile[i * kWave + lane] = u32x4{0u, 0u, 0u, 0u};  // the padding stays zero
    }
    if (q < n_load) {
      const int ch = q / (ch_samples * PPS), r = q - ch * ch_samples * PPS;
      const int t = r / PPS, h = r - t * PPS;  // sample of the channel run, half of it
      voff[i] = (ch * a.T + t) * SB + h * 16;  // < F T SB < 2^31
      if constexpr (F > 1) tpos[i] = t;
      if constexpr (PAD) {
        const int w = t / a.M, o = t - w * a.M;  // window of the step, sample of the window
        slot[i] = ch * ch_tile + (w * S * C + o) * PPS + h;
      }
    }
  }
  const int my_piece = act ? f * ch_tile + (j * S * C + s * C) * PPS : 0;

  // Steps [st0, st1) of channel group `group` into acc: flags and statistics of their windows
  // written (to LDS at lds_flags + (w - lds_w0) when lds_flags is set), raw sums of the clean
  // windows folded into this lane's channel sum.
  auto screen_steps = [&](int64_t group, int st0, int st1, StreamAcc<1> &acc, uint8_t *lds_flags,
                          int64_t lds_w0) {
    const Thresholds th = stream_thresholds(a, group);
    const uint8_t *base = a.vis + group * F * (int64_t)a.T * SB;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(base), (short)0, F * a.T * SB, kRsrcWord3);
    u32x4 buf[P] = {};                          // a piece the last step leaves unread keeps its old value
    auto issue = [&](int step) {
      const int soff = step * ch_samples * SB;
      const int room = step == n_steps - 1 ? a.T - step * ch_samples : ch_samples;  // uniform
#pragma unroll
      for (int i = 0; i < P; ++i)
        if ((!PAD || slot[i] >= 0) && (F == 1 || tpos[i] < room))
          buf[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[i], soff, kLoadStreaming));
    };
    issue(st0);
    for (int step = st0; step < st1; ++step) {
      wave_lds_order();
#pragma unroll
      for (int i = 0; i < P; ++i) {
        if constexpr (PAD) {
          if (slot[i] >= 0) my_tile[slot[i]] = buf[i];
        } else {
          my_tile[i * kWave + lane] = buf[i];
        }
      }
      wave_lds_order();
      if (step + 1 < st1) issue(step + 1);
      float ws[8] = {}, wr[8] = {};
#pragma unroll
      for (int k = 0; k < C; ++k) {
        if (!act) break;                        // PAD: a lane left over in its group
        if constexpr (FMT == FMT_CF32) {
          const f32x4 lo = __builtin_bit_cast(f32x4, my_tile[my_piece + 2 * k]);
          const f32x4 hi = __builtin_bit_cast(f32x4, my_tile[my_piece + 2 * k + 1]);
          const float x[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
          if constexpr (MIXED)
            accumulate_sample_mixed(ws, wr, x, a.eps);
          else if (!PAD && k == 0)              // every lane holds C samples: the first starts the sums
            accumulate_sample<true>(ws, wr, x, a.eps);
          else
            accumulate_sample(ws, wr, x, a.eps);
        } else {
          static_assert(!MIXED, "the paper's mixed precision takes complex64 input");
          if (!PAD && k == 0)
            accumulate_sample_h<true>(ws, wr, my_tile[my_piece + k], a.eps);
          else
            accumulate_sample_h(ws, wr, my_tile[my_piece + k], a.eps);
        }
      }
      group_sum8_rt<MIXED ? 2 : 8>(ws, L);     // ws now holds the window totals
      const int w = step * wps + j;
      const bool valid = w < a.nW;
      // one lane per window plays the leader of finish_window (kept count, moments, flag and
      // statistics); every lane folds its own raw partial into its own channel's sum
      const float wr1[1][8] = {{wr[0], wr[1], wr[2], wr[3], wr[4], wr[5], wr[6], wr[7]}};
      if constexpr (MIXED) {
        Thresholds t16{round16(th.s_low), round16(th.s_high), round16(th.g_re), round16(th.g_im)};
        finish_window<1, true>(a, t16, ws, wr1, group * a.nW + w, valid, g == 0, acc, lds_flags, lds_w0);
      } else {
        finish_window<1>(a, th, ws, wr1, group * a.nW + w, valid, g == 0, acc, lds_flags, lds_w0);
      }
    }
  };

  // The wave's results for one group, reduced over its lanes into lane 0: channel sums (F x 8),
  // kept count, moments.
  auto reduce_group = [&](const StreamAcc<1> &acc, float sums[F][8], float &kept, Moments &mom) {
    if constexpr (PAD) {                        // channel bits are not lane bits: masked wave sums
#pragma unroll
      for (int c = 0; c < F; ++c)
#pragma unroll
        for (int e = 0; e < 8; ++e) sums[c][e] = group_sum<64>(act && f == c ? acc.sum[0][e] : 0.0f);
    } else {                                    // skip the f bits of the lane index, then lane c S
#pragma unroll                                  // holds channel c
      for (int e = 0; e < 8; ++e) {
        float v = acc.sum[0][e];
        for (int m = 1; m < kWave; m <<= 1)
          if (m < S || m >= L) v += __shfl_xor(v, m);
#pragma unroll
        for (int c = 0; c < F; ++c) sums[c][e] = __shfl(v, c * S);
      }
    }
    kept = group_sum<64>(acc.kept);
    mom = acc.mom;
    if (a.state != nullptr) {
#pragma unroll
      for (int m = 1; m < kWave; m <<= 1) mom = moments_merge(mom, moments_shfl_xor(mom, m));
    }
  };

  // Average, weight and adaptive state of a whole group (lane 0's values); a persistent block
  // holds the averages and weights in LDS (hold, 9 floats per channel from group hold_first)
  // and writes them with its flags.
  auto write_group = [&](int64_t group, const float sums[F][8], float kept, const Moments &mom,
                         float *hold = nullptr, int64_t hold_first = 0) {
    const float inv = kept > 0.0f ? 1.0f / kept : 0.0f;
    if (hold != nullptr) {
#pragma unroll
      for (int c = 0; c < F; ++c) {
        float *o = hold + ((group - hold_first) * F + c) * 9;
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = sums[c][k] * inv;
        o[8] = kept * a.invT;
      }
      if (a.state != nullptr && mom.n > 0u) state_merge(a.state + group, mom);
      return;
    }
#pragma unroll
    for (int c = 0; c < F; ++c) {
      const int64_t stream = group * F + c;
      f32x4 *out = reinterpret_cast<f32x4 *>(a.avg + stream * 8);
      out[0] = f32x4{sums[c][0] * inv, sums[c][1] * inv, sums[c][2] * inv, sums[c][3] * inv};
      out[1] = f32x4{sums[c][4] * inv, sums[c][5] * inv, sums[c][6] * inv, sums[c][7] * inv};
      a.weight[stream] = kept * a.invT;
    }
    if (a.state != nullptr && mom.n > 0u) state_merge(a.state + group, mom);
  };

  if constexpr (!PERSIST) {                     // one wave per channel group
    const int64_t group = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    StreamAcc<1> acc{};
    if (group < a.n_groups) screen_steps(group, 0, n_steps, acc, nullptr, 0);
    float sums[F][8], kept;
    Moments mom;
    reduce_group(acc, sums, kept, mom);
    if (group < a.n_groups && lane == 0) write_group(group, sums, kept, mom);
  } else {
    // Block b screens the channel groups [first, last) = [b U, (b + 1) U), or with U = 0
    // [b n / G, (b + 1) n / G) (n groups, G blocks: the blocks differ by at most one group).  Its
    // waves take the groups in rounds of four, whole (wave w every fourth from first + w), and
    // split the steps of the last (last - first) mod 4 groups evenly, each a contiguous run of
    // them; a group split between waves leaves each a partial record (channel sums, kept count,
    // moments) in LDS, merged once the block is done.  The block's flags stay in LDS until then
    // and are written in one pass, after the reads.
    __shared__ float rec[2 * kWavesPerBlock][kXfer];
    __shared__ int64_t rec_group[2 * kWavesPerBlock];
    const int64_t nb = gridDim.x;
    const int64_t first = U > 0 ? (int64_t)blockIdx.x * U : (int64_t)blockIdx.x * a.n_groups / nb;
    const int64_t last = U > 0 ? min(first + U, a.n_groups) : ((int64_t)blockIdx.x + 1) * a.n_groups / nb;
    if (threadIdx.x < 2 * kWavesPerBlock) rec_group[threadIdx.x] = -1;
    __syncthreads();
    const int64_t most = U > 0 ? U : (a.n_groups + nb - 1) / nb;   // groups of the largest block
    float *hold = reinterpret_cast<float *>(block_flags + ((most * a.nW + 15) & ~15));
    const int64_t split0 = first + (last - first) / kWavesPerBlock * kWavesPerBlock;
    for (int64_t group = first + wave; group < split0; group += kWavesPerBlock) {
      StreamAcc<1> acc{};
      screen_steps(group, 0, n_steps, acc, block_flags, first * a.nW);
      float sums[F][8], kept;
      Moments mom;
      reduce_group(acc, sums, kept, mom);
      if (lane == 0) write_group(group, sums, kept, mom, hold, first);
    }
    const int64_t total = (last - split0) * n_steps;
    const int64_t s_end = total * (wave + 1) / kWavesPerBlock;
    int n_rec = 0;
    for (int64_t s0 = total * wave / kWavesPerBlock; s0 < s_end;) {
      const int64_t gi = s0 / n_steps;
      const int st0 = (int)(s0 - gi * n_steps);
      const int st1 = (int)min((int64_t)n_steps, st0 + (s_end - s0));
      const int64_t group = split0 + gi;
      StreamAcc<1> acc{};
      screen_steps(group, st0, st1, acc, block_flags, first * a.nW);
      float sums[F][8], kept;
      Moments mom;
      reduce_group(acc, sums, kept, mom);
      if (st0 == 0 && st1 == n_steps) {         // the whole group in this wave
        if (lane == 0) write_group(group, sums, kept, mom, hold, first);
      } else if (lane == 0) {                   // at most two per wave: its first and its last group
        const int r = 2 * wave + n_rec;
#pragma unroll
        for (int c = 0; c < F; ++c)
#pragma unroll
          for (int e = 0; e < 8; ++e) rec[r][8 * c + e] = sums[c][e];
        rec[r][32] = kept;
        rec[r][33] = __uint_as_float(mom.n);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          rec[r][34 + k] = mom.m[k];
          rec[r][37 + k] = mom.s[k];
        }
        rec_group[r] = group;
      }
      if (!(st0 == 0 && st1 == n_steps)) ++n_rec;
      s0 += st1 - st0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {                     // groups split between waves: merge the records
      for (int r = 0; r < 2 * kWavesPerBlock; ++r) {
        const int64_t group = rec_group[r];
        if (group < 0) continue;
        float sums[F][8], kept = rec[r][32];
        Moments mom{__float_as_uint(rec[r][33]), {rec[r][34], rec[r][35], rec[r][36]}, {rec[r][37], rec[r][38], rec[r][39]}};
#pragma unroll
        for (int c = 0; c < F; ++c)
#pragma unroll
          for (int e = 0; e < 8; ++e) sums[c][e] = rec[r][8 * c + e];
        for (int q = r + 1; q < 2 * kWavesPerBlock; ++q) {
          if (rec_group[q] != group) continue;
#pragma unroll
          for (int c = 0; c < F; ++c)
#pragma unroll
            for (int e = 0; e < 8; ++e) sums[c][e] += rec[q][8 * c + e];
          kept += rec[q][32];
          const Moments b{__float_as_uint(rec[q][33]), {rec[q][34], rec[q][35], rec[q][36]}, {rec[q][37], rec[q][38], rec[q][39]}};
          mom = moments_merge(mom, b);
          rec_group[q] = -1;
        }
        write_group(group, sums, kept, mom, hold, first);
      }
    }
    __syncthreads();
    if (a.flags != nullptr) {
      const int64_t base = first * a.nW, n = (last - first) * a.nW;
      for (int64_t i = threadIdx.x; i < n; i += kBlock) a.flags[base + i] = block_flags[i];
    }
    for (int64_t i = threadIdx.x; i < (last - first) * F; i += kBlock) {  // stream first F + i
      const float *o = hold + i * 9;
      f32x4 *out = reinterpret_cast<f32x4 *>(a.avg + (first * F + i) * 8);
      out[0] = f32x4{o[0], o[1], o[2], o[3]};
      out[1] = f32x4{o[4], o[5], o[6], o[7]};
      a.weight[first * F + i] = o[8];
    }
  }
}

// Time x frequency windows wider than one lane group (F > 1 and F ceil(M / 8) > 64 runs): one
// wave per channel group.  A step is one chunk of one channel's run of a window, up to 64 C
// consecutive samples (C per lane), so a run of M samples takes R = ceil(M / (64 C)) steps and a
// window F R.  The chunk is loaded coalesced and transposed through the wave's LDS tile as in
// the tiled kernel; each step's buffer resource ends where the run does, so in the last chunk
// of a run the loads past its end return zeros with no memory access (a zero sample adds exactly
// zero to every window and raw sum).  A lane sums its C samples of a step, then adds those step
// sums into the window sums and into its channel's raw sums: no lane sums more than C + F R
// terms in a row.  After the window's last step: one wave reduction and the window finish.
template <int FMT, int C, int F>
__global__ void __launch_bounds__(kBlock) screen_wide(const ScreenArgs a) {
  constexpr int SB = FMT == FMT_CF32 ? 32 : 16;
  constexpr int PPS = SB / 16;                  // 16-byte pieces per sample
  constexpr int P = C * PPS;                    // pieces per lane per step
  constexpr int CHUNK = kWave * C;              // samples per step
  static_assert(F == 2 || F == 4, "wide windows span 2 or 4 channels");
  __shared__ u32x4 tile[kWavesPerBlock][kWave * P];
  __shared__ float xfer[kWavesPerBlock][kXfer];
  // eight pieces per lane: the tiled kernel's bank-conflict-free slots
  auto slot = [](int q) { return P == kPieces ? lds_slot(q) : q; };

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int64_t group = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  const bool active = group < a.n_groups;
  StreamAcc<F> acc{};
  if (active) {
    const Thresholds th = stream_thresholds(a, group);
    const uint8_t *gbase = a.vis + group * F * (int64_t)a.T * SB;
    const int R = (a.M + CHUNK - 1) / CHUNK;   // chunks per channel run
    u32x4 *my_tile = tile[wave];
    u32x4 buf[P];
    int lj = 0, lf = 0, lc = 0;                 // the next chunk to load: window, channel, chunk
    auto issue = [&]() {
      const int64_t start = (int64_t)lf * a.T + (int64_t)lj * a.M + (int64_t)lc * CHUNK;  // sample of the group
      const int len = min(CHUNK, a.M - lc * CHUNK);
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<uint8_t *>(gbase + start * SB), (short)0, len * SB, kRsrcWord3);
      // a run that does not start or end on a 128-byte line shares its first and last lines with
      // the runs before and after it in the channel, which come F R steps apart: the loads of
      // those pieces keep the default cache policy so the lines stay in L2 until the neighbour
      // run reads them (non-temporal, 300 x 2 in complex half read 1.2 % more than its bytes)
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const unsigned off = (unsigned)((i * kWave + lane) * 16);
        if (i == 0 || i == P - 1)
          buf[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
        else
          buf[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kLoadStreaming));
      }
      if (++lc == R) {
        lc = 0;
        if (++lf == F) {
          lf = 0;
          ++lj;
        }
      }
    };
    float ws[8] = {}, wr[F][8] = {};
    issue();
    for (int j = 0; j < a.nW; ++j) {
#pragma unroll
      for (int f = 0; f < F; ++f) {
        for (int c = 0; c < R; ++c) {
          wave_lds_order();
#pragma unroll
          for (int i = 0; i < P; ++i) my_tile[slot(i * kWave + lane)] = buf[i];
          wave_lds_order();
          if (lj < a.nW) issue();
          float ps[8], pr[8];
#pragma unroll
          for (int k = 0; k < C; ++k) {
            if constexpr (FMT == FMT_CF32) {
              const f32x4 lo = __builtin_bit_cast(f32x4, my_tile[slot(P * lane + 2 * k)]);
              const f32x4 hi = __builtin_bit_cast(f32x4, my_tile[slot(P * lane + 2 * k + 1)]);
              const float x[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
              if (k == 0)
                accumulate_sample<true>(ps, pr, x, a.eps);
              else
                accumulate_sample(ps, pr, x, a.eps);
            } else {
              if (k == 0)
                accumulate_sample_h<true>(ps, pr, my_tile[slot(P * lane + k)], a.eps);
              else
                accumulate_sample_h(ps, pr, my_tile[slot(P * lane + k)], a.eps);
            }
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            ws[k] += ps[k];
            wr[f][k] += pr[k];
          }
        }
      }
      float tot[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) tot[k] = group_sum<kWave>(ws[k]);
      finish_window<F>(a, th, tot, wr, group * a.nW + j, true, lane == 0, acc);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        ws[k] = 0.0f;
#pragma unroll
        for (int f = 0; f < F; ++f) wr[f][k] = 0.0f;
      }
    }
  }
  finish_stream<F>(a, acc, group, 0, active, wave, lane, xfer);
}

// Wide windows over four channels whose runs fit 32 lanes (M <= 32 C): a step holds the runs of
// two channels of a window, lanes [0, S) channel 2p and [S, 2S) channel 2p + 1 (S = ceil(M / C),
// p = 0, 1), so a window is two steps, fewer lanes stand idle than with one run per step (129 x 4:
// 52 of 64 lanes on runs of 5 where one run of 4 per step used 33), and a lane keeps the raw sums
// of two channels.  Each run takes S C tile slots; the slots past M stay zero (written once, never
// loaded), as do the lanes past 2 S.
template <int FMT, int C>
__global__ void __launch_bounds__(kBlock) screen_wide_pairs(const ScreenArgs a) {
  constexpr int SB = FMT == FMT_CF32 ? 32 : 16;
  constexpr int PPS = SB / 16;                  // 16-byte pieces per sample
  constexpr int P = C * PPS;                    // pieces per lane per step
  constexpr int F = 4;
  __shared__ u32x4 tile[kWavesPerBlock][kWave * P];

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int64_t group = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  const bool active = group < a.n_groups;
  const int S = (a.M + C - 1) / C;              // lanes per run, <= 32
  const int h = lane / S;                       // the lane's channel of the pair (2, 3, ...: idle)
  const bool act = h < 2;
  const int my_piece = act ? lane * C * PPS : 0;  // (h S + s) C PPS
  u32x4 *my_tile = tile[wave];
  // piece q = i 64 + lane of a step, q < 2 M PPS: run hq = q / (M PPS), piece r of it; its byte
  // offset in the group (the step adds the pair's channel and the window as a scalar) and its
  // tile slot, fixed for the kernel
  int voff[P], lslot[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int q = i * kWave + lane;
    my_tile[i * kWave + lane] = u32x4{0u, 0u, 0u, 0u};
    voff[i] = 0;
    lslot[i] = -1;
    if (q < 2 * a.M * PPS) {
      const int hq = q / (a.M * PPS), r = q - hq * a.M * PPS;
      voff[i] = hq * a.T * SB + r * 16;         // < 2 T SB
      lslot[i] = hq * S * C * PPS + r;
    }
  }
  StreamAcc<2> acc{};                           // acc.sum[p]: channel 2 p + h
  if (active) {
    const Thresholds th = stream_thresholds(a, group);
    const uint8_t *base = a.vis + group * F * (int64_t)a.T * SB;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(base), (short)0, F * a.T * SB, kRsrcWord3);
    u32x4 buf[P] = {};
    auto issue = [&](int j, int p) {            // channels 2 p, 2 p + 1 of window j
      const int soff = (2 * p * a.T + j * a.M) * SB;
#pragma unroll
      for (int i = 0; i < P; ++i)
        if (lslot[i] >= 0)
          buf[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[i], soff, kLoadStreaming));
    };
    float ws[8] = {}, wr[2][8] = {};
    issue(0, 0);
    for (int j = 0; j < a.nW; ++j) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        wave_lds_order();
#pragma unroll
        for (int i = 0; i < P; ++i)
          if (lslot[i] >= 0) my_tile[lslot[i]] = buf[i];
        wave_lds_order();
        if (p == 0)
          issue(j, 1);
        else if (j + 1 < a.nW)
          issue(j + 1, 0);
        float ps[8] = {}, pr[8] = {};
#pragma unroll
        for (int k = 0; k < C; ++k) {
          if (!act) break;
          if constexpr (FMT == FMT_CF32) {
            const f32x4 lo = __builtin_bit_cast(f32x4, my_tile[my_piece + 2 * k]);
            const f32x4 hi = __builtin_bit_cast(f32x4, my_tile[my_piece + 2 * k + 1]);
            const float x[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            accumulate_sample(ps, pr, x, a.eps);
          } else {
            accumulate_sample_h(ps, pr, my_tile[my_piece + k], a.eps);
          }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          ws[k] += ps[k];
          wr[p][k] += pr[k];
        }
      }
      float tot[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) tot[k] = group_sum<kWave>(ws[k]);
      finish_window<2>(a, th, tot, wr, group * a.nW + j, true, lane == 0, acc);
#pragma unroll
      for (int k = 0; k < 8; ++k) ws[k] = wr[0][k] = wr[1][k] = 0.0f;
    }
  }
  // channel 2 p + hh: masked wave sums of acc.sum[p] over the lanes of run hh
  float chan[F][8];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
      for (int e = 0; e < 8; ++e) chan[2 * p + hh][e] = group_sum<kWave>(act && h == hh ? acc.sum[p][e] : 0.0f);
  const float kept = group_sum<kWave>(acc.kept);
  Moments mom = acc.mom;
  if (a.state != nullptr) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) mom = moments_merge(mom, moments_shfl_xor(mom, m));
  }
  if (active && lane == 0) {
    const float inv = kept > 0.0f ? 1.0f / kept : 0.0f;
#pragma unroll
    for (int c = 0; c < F; ++c) {
      const int64_t stream = group * F + c;
      f32x4 *out = reinterpret_cast<f32x4 *>(a.avg + stream * 8);
      out[0] = f32x4{chan[c][0] * inv, chan[c][1] * inv, chan[c][2] * inv, chan[c][3] * inv};
      out[1] = f32x4{chan[c][4] * inv, chan[c][5] * inv, chan[c][6] * inv, chan[c][7] * inv};
      a.weight[stream] = kept * a.invT;
    }
    if (a.state != nullptr && mom.n > 0u) state_merge(a.state + group, mom);
  }
}

// Unused dynamic LDS that caps the complex64 tiled kernel at three blocks (12 waves) per CU
// (33 KiB static + 7.5 KiB > 160 KiB / 4).  Its registers alone would allow 16 waves; with fewer
// streams read at once the kernel streams 1-2 % faster.  The complex-half kernel is held at
// 12 waves by its registers already.
constexpr unsigned kCf32OccupancyPad = 7680;

// Blocks per CU of the complex-half tiled kernel, set by unused dynamic LDS (0: the four its
// registers and LDS allow; kCf32OccupancyPad: three; 22528 bytes: two), by log2 M.  Timed on
// 48 x 64 and 64 x 256 arrays with the variants alternating launch by launch: two blocks are
// 3-5 % faster than four at M = 8-64 and 1024-4096, three blocks 2-3 % faster at M = 4 and
// 128-512 (where two lose up to 4.5 %), four best at M = 2 (two: -6.5 %).  As with the
// complex64 kernel, fewer streams read at once suit HBM better, up to the point where too
// few loads are in flight.
constexpr unsigned kTiledCf16Pad[kMaxTiledLog2M + 1] = {0u, 0u, 7680u, 22528u, 22528u, 22528u, 22528u,
                                                        7680u, 7680u, 7680u, 22528u, 22528u, 22528u};

// The persistent complex64 tiled launch: three blocks per CU, each holding at most this many
// bytes of flags, averages and weights in LDS (33 KiB static + 19 KiB < 160 KiB / 3).  Complex64 with flags, one
// segment per stream: +1 % at M = 64, +4 % at M = 16.  Complex half lost 1-4 % in this form
// (more registers per loop) and keeps the one-stream-per-wave launch.
constexpr int kPersistBlocksPerCu = 3;

constexpr int64_t kPersistFlagBytes = 19456;

// Groups per block of a persistent launch of at most G blocks: ceil(n / G), rounded up to a
// multiple of the waves per block once that exceeds them, so that every wave of every block
// but the last screens the same number of groups and the waves end together (37 groups per
// block leave one wave in four a tenth group after the others).
inline int64_t balanced_share(int64_t n, int64_t G) {
  int64_t U = (n + G - 1) / G;
  if (U > kWavesPerBlock) U = (U + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock;
  return U;
}

template <int FMT, int LOG2M>
hipError_t launch_tiled(const ScreenArgs &a, hipStream_t stream) {
  if constexpr (FMT == FMT_CF32) {
    if (a.n_seg == 1 && a.flags != nullptr && a.n_cu > 0) {
      const int64_t G = (int64_t)a.n_cu * kPersistBlocksPerCu;
      const int64_t U = balanced_share(a.n_groups, G);
      if (U * a.nW <= kPersistFlagBytes) {   // and the averages too where they fit beside the flags
        const int hold_avg = ((U * a.nW + 15) & ~15) + U * 36 <= kPersistFlagBytes;
        const int64_t blocks = (a.n_groups + U - 1) / U;
        const unsigned lds = (unsigned)std::max<int64_t>(hold_avg ? ((U * a.nW + 15) & ~15) + U * 36 : U * a.nW,
                                                         kCf32OccupancyPad);
        hipLaunchKernelGGL((screen_tiled<FMT, LOG2M, true>), dim3((unsigned)blocks), dim3(kBlock), lds, stream,
                           a, (int)U, hold_avg);
        return hipGetLastError();
      }
    }
  }
  const int64_t units = a.n_groups * a.n_seg;
  const int64_t blocks = (units + kWavesPerBlock - 1) / kWavesPerBlock;
  const unsigned pad = FMT == FMT_CF32 ? kCf32OccupancyPad : kTiledCf16Pad[LOG2M];
  hipLaunchKernelGGL((screen_tiled<FMT, LOG2M, false>), dim3((unsigned)blocks), dim3(kBlock), pad, stream, a, 0, 0);
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

// Unused dynamic LDS that caps the complex-half long-window kernel at two blocks (8 waves)
// per CU (33 KiB static + 22 KiB > 160 KiB / 3) where edge steps are rare (M >= 2048): its
// plain steps then stream faster than at the three blocks its registers allow (M = 3072:
// 0.82 -> 0.87 of the HBM peak).  With frequent edges (M = 600-1000) three blocks are better
// (two: -16 to -18 %), and complex64 is the same either way.
constexpr unsigned kLongCf16RareEdgePad = 22528;

template <int FMT>
hipError_t launch_long(const ScreenArgs &a, hipStream_t stream) {
  const int64_t units = a.n_groups * a.n_seg;
  const int64_t blocks = (units + kWavesPerBlock - 1) / kWavesPerBlock;
  const unsigned pad = FMT == FMT_CF16 && a.M >= 2048 ? kLongCf16RareEdgePad : 0u;
  const int spi = kWave * (FMT == FMT_CF32 ? 4 : 8);
  if (2 * a.M <= spi) return hipErrorInvalidValue;  // kernel_for sends these to the windowed kernel
  hipLaunchKernelGGL((screen_long<FMT, 1>), dim3((unsigned)blocks), dim3(kBlock), pad, stream, a);
  return hipGetLastError();
}

template <int FMT, int C>
hipError_t launch_wide_c(const ScreenArgs &a, hipStream_t stream) {
  const int64_t blocks = (a.n_groups + kWavesPerBlock - 1) / kWavesPerBlock;
  const dim3 grid((unsigned)blocks), block(kBlock);
  switch (a.F) {
    case 2: hipLaunchKernelGGL((screen_wide<FMT, C, 2>), grid, block, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((screen_wide<FMT, C, 4>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int FMT, int C>
hipError_t launch_wide_pairs_c(const ScreenArgs &a, hipStream_t stream) {
  const int64_t blocks = (a.n_groups + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((screen_wide_pairs<FMT, C>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, a);
  return hipGetLastError();
}

template <int FMT>
hipError_t launch_wide(const ScreenArgs &a, hipStream_t stream) {
  if (a.F == 4) {                               // runs that fit 32 lanes: two channels per step
    switch (wide_pairs_chunk(a.M, FMT)) {
      case 0: break;
      case 3: if constexpr (FMT == FMT_CF32) return launch_wide_pairs_c<FMT, 3>(a, stream); break;
      case 4: if constexpr (FMT == FMT_CF32) return launch_wide_pairs_c<FMT, 4>(a, stream); break;
      case 5: if constexpr (FMT == FMT_CF16) return launch_wide_pairs_c<FMT, 5>(a, stream); break;
      case 6: if constexpr (FMT == FMT_CF16) return launch_wide_pairs_c<FMT, 6>(a, stream); break;
      case 7: if constexpr (FMT == FMT_CF16) return launch_wide_pairs_c<FMT, 7>(a, stream); break;
      case 8: if constexpr (FMT == FMT_CF16) return launch_wide_pairs_c<FMT, 8>(a, stream); break;
      default: return hipErrorInvalidValue;
    }
  }
  if constexpr (FMT == FMT_CF32) {
    switch (wide_chunk(a.M, FMT)) {
      case 2: return launch_wide_c<FMT, 2>(a, stream);
      case 3: return launch_wide_c<FMT, 3>(a, stream);
      case 4: return launch_wide_c<FMT, 4>(a, stream);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (wide_chunk(a.M, FMT)) {
      case 4: return launch_wide_c<FMT, 4>(a, stream);
      case 5: return launch_wide_c<FMT, 5>(a, stream);
      case 6: return launch_wide_c<FMT, 6>(a, stream);
      case 7: return launch_wide_c<FMT, 7>(a, stream);
      case 8: return launch_wide_c<FMT, 8>(a, stream);
      default: return hipErrorInvalidValue;
    }
  }
}

constexpr int kFourBlocksLds = 33024;  // LDS per block that leaves room for four (160 KiB / 5 < this)

template <int FMT, int C, bool MIXED, bool PAD, bool PERSIST>
hipError_t launch_windows_f(dim3 grid, unsigned lds, int U, const ScreenArgs &a, hipStream_t stream) {
  switch (a.F) {
    case 1: hipLaunchKernelGGL((screen_windows<FMT, C, 1, MIXED, PAD, PERSIST>), grid, dim3(kBlock), lds, stream, a, U); break;
    case 2: hipLaunchKernelGGL((screen_windows<FMT, C, 2, MIXED, PAD, PERSIST>), grid, dim3(kBlock), lds, stream, a, U); break;
    case 4: hipLaunchKernelGGL((screen_windows<FMT, C, 4, MIXED, PAD, PERSIST>), grid, dim3(kBlock), lds, stream, a, U); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int FMT, int C, bool MIXED, bool PAD>
hipError_t launch_windows_k(const ScreenArgs &a, hipStream_t stream) {
  // exact complex-half layouts of 5 or more samples per lane: at most four blocks per CU (unused
  // dynamic LDS past 160 KiB / 5): 1-2 % faster than the five their registers allow (10 x 2, 5 x 4,
  // M = 20, 48); padded layouts and runs of 3 are not
  constexpr int tile_bytes = kWavesPerBlock * kWave * C * (FMT == FMT_CF32 ? 2 : 1) * 16;
  constexpr unsigned pad = FMT == FMT_CF16 && !PAD && !MIXED && C >= 5 && tile_bytes < kFourBlocksLds
                               ? (unsigned)(kFourBlocksLds - tile_bytes) : 0u;
  // Exact layouts of at most 6 samples per lane with a flag array run persistent, each block's
  // flags, averages and weights held in LDS until its groups are done, at the most blocks per CU
  // (4, 3, 2) whose share fits beside the tile.  Complex64 (the paper's mixed form included): U groups per block, a
  // multiple of the four waves, so each wave screens whole groups (10 x 2 +5.5 %, 5 x 4 +5.1 %,
  // M = 20 +4.5 %, the mixed form +3.4 %, M = 48 +1.1 % over one wave per group; runs of 8 lose
  // 3 %).  Complex half, whose VALU-heavy waves run as fast as their CU lets them, needs the same
  // work on every CU: G = blocks per CU x CUs blocks of n / G groups, the steps of each block's
  // last (n / G) mod 4 groups split between its waves; at most three blocks per CU (four: 5 x 4
  // -4 %, 10 x 2 -0.5 to -0.9 %; two: 10 x 2 -2.5 %); and only where a group has at least 16 steps
  // (over one wave per group: 5 x 4 +6 to +8 %, 10 x 2 +0.7 to +2.5 %; M = 20 and 48, 8-10 steps
  // per group, lost 1-4 %).  Interleaved whole groups matter to complex64: contiguous runs of groups per wave cost
  // it 0.6-2 %.
  if constexpr (!PAD && C <= 6) {
    constexpr int rec_bytes = 2 * kWavesPerBlock * (kXfer * 4 + 8);
    const int L = a.F * (a.M / C), wps = kWave / L;
    const bool long_groups = (a.nW + wps - 1) / wps >= 16;
    for (int bpc = FMT == FMT_CF16 ? 3 : 4; bpc >= 2 && a.flags != nullptr && a.n_cu > 0 && (FMT == FMT_CF32 || long_groups); --bpc) {
      const int64_t G = std::min<int64_t>((int64_t)a.n_cu * bpc, a.n_groups);
      const int64_t U = FMT == FMT_CF32 ? balanced_share(a.n_groups, G) : 0;
      const int64_t blocks = U > 0 ? (a.n_groups + U - 1) / U : G;
      const int64_t most = U > 0 ? U : (a.n_groups + G - 1) / G;   // groups of the largest block
      const int64_t room = 163840 / bpc - 512 - tile_bytes - rec_bytes;
      const int64_t held = ((most * a.nW + 15) & ~15) + most * a.F * 36;   // flags, averages, weights
      if (held <= room) {
        const unsigned lds = (unsigned)std::max<int64_t>(held, (int64_t)pad);
        return launch_windows_f<FMT, C, MIXED, PAD, true>(dim3((unsigned)blocks), lds, (int)U, a, stream);
      }
    }
  }
  const int64_t blocks = (a.n_groups + kWavesPerBlock - 1) / kWavesPerBlock;
  return launch_windows_f<FMT, C, MIXED, PAD, false>(dim3((unsigned)blocks), pad, 0, a, stream);
}

// PAD (padded runs or partial lane groups) exists only outside the paper's mixed precision.
template <int FMT, int C, bool MIXED>
hipError_t launch_windows_p(bool pad, const ScreenArgs &a, hipStream_t stream) {
  if constexpr (MIXED)
    return pad ? hipErrorInvalidValue : launch_windows_k<FMT, C, true, false>(a, stream);
  else if constexpr (FMT == FMT_CF32 && C > kPadMaxC32)  // windows_layout never pads these
    return pad ? hipErrorInvalidValue : launch_windows_k<FMT, C, false, false>(a, stream);
  else
    return pad ? launch_windows_k<FMT, C, false, true>(a, stream) : launch_windows_k<FMT, C, false, false>(a, stream);
}

template <int FMT, bool MIXED>
hipError_t launch_windows(const WindowsLayout &w, const ScreenArgs &a, hipStream_t stream) {
  switch (w.C) {
    case 2: return launch_windows_p<FMT, 2, MIXED>(w.pad, a, stream);
    case 3: return launch_windows_p<FMT, 3, MIXED>(w.pad, a, stream);
    case 4: return launch_windows_p<FMT, 4, MIXED>(w.pad, a, stream);
    case 5: return launch_windows_p<FMT, 5, MIXED>(w.pad, a, stream);
    case 6: return launch_windows_p<FMT, 6, MIXED>(w.pad, a, stream);
    case 7: return launch_windows_p<FMT, 7, MIXED>(w.pad, a, stream);
    case 8: return launch_windows_p<FMT, 8, MIXED>(w.pad, a, stream);
    default: return hipErrorInvalidValue;
  }
}

int ilog2_exact(int m) {
  int l = 0;
  while ((1 << l) < m) ++l;
  return (1 << l) == m ? l : -1;
}

// ----------------------------------------------------------------------------- probes

constexpr int kProbeBlocks = 4096;
constexpr int kProbeChunk = 16384;  // bytes per wave per step

// Read-only probe with the screen's access pattern at its best: each wave streams
// contiguous 16 KiB steps of its own chunk with coalesced non-temporal 16-byte
// loads; the chunks of consecutive waves are adjacent.
__global__ void __launch_bounds__(kBlock) probe_read_kernel(const u32x4 *src, size_t n16, float *sink) {
  const int lane = threadIdx.x % kWave;
  const size_t waves = (size_t)gridDim.x * kWavesPerBlock;
  const size_t wave = (size_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  const size_t n_steps = (n16 * 16 + kProbeChunk - 1) / kProbeChunk;
  const uint8_t *base = reinterpret_cast<const uint8_t *>(src);
  const size_t total = n16 * 16;
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (size_t step = wave; step < n_steps; step += waves) {
    const size_t off = step * kProbeChunk;
    const size_t len = total - off < (size_t)kProbeChunk ? total - off : (size_t)kProbeChunk;
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(base + off), (short)0, (int)len, kRsrcWord3);
    u32x4 v[kProbeChunk / 1024];
#pragma unroll
    for (int i = 0; i < kProbeChunk / 1024; ++i)
      v[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, (i * kWave + lane) * 16, 0, kLoadStreaming));
#pragma unroll
    for (int i = 0; i < kProbeChunk / 1024; ++i) acc ^= v[i];
  }
  unsigned x = acc[0] ^ acc[1] ^ acc[2] ^ acc[3];
  for (int m = 1; m < kWave; m <<= 1) x ^= __shfl_xor(x, m);
  if (lane == 0) sink[wave] = __builtin_bit_cast(float, x);
}

__global__ void __launch_bounds__(kBlock) probe_copy_kernel(u32x4 *dst, const u32x4 *src, size_t n16) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

bool tiled_supports(int M) {
  const int l = ilog2_exact(M);
  return l >= 1 && l <= kMaxTiledLog2M;
}

// Samples per lane of the wide-window kernel: the C (complex half 4-8, complex64 2-4: at most
// eight 16-byte pieces per lane) whose chunks of 64 C samples fill the largest share of their
// lane slots over a run of M samples, M / (ceil(M / 64 C) 64 C); ties to the larger C.
int wide_chunk(int M, int fmt) {
  const int lo = fmt == FMT_CF32 ? 2 : 4, hi = fmt == FMT_CF32 ? 4 : 8;
  int best = hi;
  double best_share = 0.0;
  for (int C = hi; C >= lo; --C) {
    const int64_t chunk = (int64_t)kWave * C, slots = (M + chunk - 1) / chunk * chunk;
    const double share = (double)M / (double)slots;
    if (share > best_share + 1e-12) {
      best = C;
      best_share = share;
    }
  }
  return best;
}

// Samples per lane of the two-runs-per-step wide kernel (F = 4): ceil(M / 32), the fewest that
// fit a channel's run in 32 lanes, for complex half 5-8 (M = 129-256) and complex64 3-4
// (M = 65-128); 0 where it does not apply.
int wide_pairs_chunk(int M, int fmt) {
  const int C = (M + 31) / 32;
  const int lo = fmt == FMT_CF32 ? 3 : 5, hi = fmt == FMT_CF32 ? 4 : 8;
  return C >= lo && C <= hi ? C : 0;
}

WindowsLayout windows_layout(int M, int F, int fmt, bool mixed) {
  // Runs of C = 2..8 samples per lane, S = ceil(M / C) runs per channel, F S <= 64 lanes
  // rounded up to a power of two L: the layout that fills the largest share M F / (L C) of
  // its lane slots; among equals the largest C (fewer lanes per window, fewer window
  // reductions per sample).  An exact layout (M = C S and F S = L: share 1) runs without
  // padding; a padded one keeps per-piece offsets and slots in registers, which complex64
  // storage (two pieces per sample) affords up to C = kPadMaxC32.
  WindowsLayout best{0, false, 0.0};
  for (int C = 8; C >= 2; --C) {
    const int S = (M + C - 1) / C;
    const int FS = F * S;
    if (FS > kWave) continue;
    int L = 1;
    while (L < FS) L *= 2;
    const bool exact = S * C == M && FS == L;
    if (!exact && (mixed || (fmt == FMT_CF32 && C > kPadMaxC32))) continue;
    const double share = (double)M * F / ((double)L * C);
    if (share > best.share + 1e-12) best = WindowsLayout{C, !exact, share};
  }
  return best;
}

KernelKind kernel_for(int M, int F, int fmt, bool mixed) {
  if (mixed)  // the windowed kernel on whole lane groups, complex64 storage
    return fmt == FMT_CF32 && windows_layout(M, F, fmt, true).C > 0 ? kWindows : kNone;
  if (F == 1 && tiled_supports(M)) return kTiled;
  const WindowsLayout w = windows_layout(M, F, fmt, false);
  const bool long_ok = F == 1 && 2 * M > kWave * (fmt == FMT_CF32 ? 4 : 8);
  if (w.C > 0 && (!w.pad || !long_ok || w.share >= kPadOverLong)) return kWindows;
  if (long_ok) return kLong;
  return F > 1 ? kWide : kNone;  // every F = 1 length has one of the kernels above
}

hipError_t launch_screen(int fmt, const ScreenArgs &a, hipStream_t stream) {
  const bool cf32 = fmt == FMT_CF32;
  switch (kernel_for(a.M, a.F, fmt, (a.options & kOptPaperMixed) != 0)) {
    case kTiled: {
      const int l = ilog2_exact(a.M);
      return cf32 ? dispatch_tiled<FMT_CF32>(l, a, stream) : dispatch_tiled<FMT_CF16>(l, a, stream);
    }
    case kWindows: {
      const bool mixed = (a.options & kOptPaperMixed) != 0;
      const WindowsLayout w = windows_layout(a.M, a.F, fmt, mixed);
      if (mixed) return launch_windows<FMT_CF32, true>(w, a, stream);
      return cf32 ? launch_windows<FMT_CF32, false>(w, a, stream) : launch_windows<FMT_CF16, false>(w, a, stream);
    }
    case kLong: return cf32 ? launch_long<FMT_CF32>(a, stream) : launch_long<FMT_CF16>(a, stream);
    case kWide: return cf32 ? launch_wide<FMT_CF32>(a, stream) : launch_wide<FMT_CF16>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------------------- half sums check

__device__ __forceinline__ float cvt_f16_lo(uint32_t w) {  // binary16 in the low half -> float32
  float f;
  asm volatile("v_cvt_f32_f16 %0, %1" : "=v"(f) : "v"(w));
  return f;
}

__device__ __forceinline__ bool same_f32(float x, float y) {
  return (x != x && y != y) || __float_as_uint(x) == __float_as_uint(y);
}

// One thread per binary16 value a (65536 threads): every form of the complex-half sums
// (mix_add, mix_sub, mix_acc, both halves) against conversion by v_cvt_f32_f16 followed by
// a float32 add, for kHalfSumsOthers values b (signed zeros, subnormals, the largest finite
// values, infinities, a NaN, then pseudo-random bit patterns).  bad[a] counts differences.
__global__ void __launch_bounds__(kBlock) probe_half_sums_kernel(uint32_t *bad) {
#pragma clang fp contract(off)  // the references below are single roundings: no fused c + a
  const uint32_t a16 = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t special[] = {0x0000u, 0x8000u, 0x0001u, 0x8001u, 0x03ffu, 0x0400u, 0x3c00u, 0xbc00u,
                              0x7bffu, 0xfbffu, 0x7c00u, 0xfc00u, 0x7e00u, 0x3555u, 0xb555u, 0x1000u};
  uint32_t n = 0, x = 12345u;
  for (int i = 0; i < kHalfSumsOthers; ++i) {
    uint32_t b16;
    if (i < 16) {
      b16 = special[i];
    } else {
      x = x * 1664525u + 1013904223u;
      b16 = x >> 16;
    }
    const uint32_t A = a16 | (b16 << 16), B = b16 | (a16 << 16);  // a low, b high; and swapped
    const float fa = cvt_f16_lo(a16), fb = cvt_f16_lo(b16);
    const float c1 = fb * 3.0f, c2 = fa * 0.37f;
    n += !same_f32(mix_add<0, 0>(A, B), fa + fb);
    n += !same_f32(mix_add<1, 1>(A, B), fb + fa);
    n += !same_f32(mix_sub<0, 0>(A, B), fa - fb);
    n += !same_f32(mix_sub<1, 1>(A, B), fb - fa);
    n += !same_f32(mix_sub<0, 1>(A, A), fa - fb);
    n += !same_f32(mix_acc<0>(c1, A), c1 + fa);
    n += !same_f32(mix_acc<1>(c2, A), c2 + fb);
  }
  bad[a16] = n;
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

hipError_t launch_probe_half_sums(uint32_t *bad, hipStream_t stream) {
  hipLaunchKernelGGL(probe_half_sums_kernel, dim3(kHalfSumsValues / kBlock), dim3(kBlock), 0, stream, bad);
  return hipGetLastError();
}

}  // namespace rfi
