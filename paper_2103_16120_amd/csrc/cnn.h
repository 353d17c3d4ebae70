// Learned preconditioner network: 3x3 convolutions C_in -> 32 -> 32 -> 32 ->
// 32 -> 1 with ReLU between layers, BF16 weights and activations, float32
// accumulation on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Tensors are NHWC with 32 channels per pixel (64 B; unused channels are
// zero), natural [NY][NX] pixel order.  Padding on the sphere matches the
// elliptic operator: longitude periodic, the row beyond a pole is the polar
// row seen across the pole (shifted by NX/2).
//
// MFMA 16x16x32 operand layout (checked on the device): lane l holds
//   A[m = l%16][k = 8*(l/16) .. +7],  B[k = 8*(l/16) .. +7][n = l%16],
//   C[m = 4*(l/16) .. +3][n = l%16].
// A convolution is an implicit GEMM per tap: M = 16 output pixels, K = 32
// input channels, N = 16 output channels.
#pragma once

#include <type_traits>

#include "device.h"

namespace mpgcr {

constexpr int CNN_LAYERS = 5;
constexpr int TAPS = 9;             // tap t = (dy+1)*3 + (dx+1)
constexpr int WG_WAVES = 4;

struct ConvArgs {
  const __bf16* in;        // [B][ny][nx][CH]
  const __bf16* w;         // [TAPS][CH out][CH in]
  const __bf16* wpole;     // same layout: weights for taps that read across a pole
  const float* bias;       // [CH] or null
  __bf16* out;             // [B][ny][nx][CH] (bf16 output modes)
  float* out32;            // [B][ny][nx] channel 0 (float32 output mode)
  const __bf16* mask;      // multiply by (mask > 0), [B][ny][nx][CH], or null
  const int* active;       // [B]: images with 0 are skipped (output left as is), or null (all)
  int row_begin, row_end;  // rows computed (all: 0, ny)
  int pole_row;            // -1: taps use `w`, across-pole taps `wpole` only if wpole == w (forward);
                           // 0 or ny-1: the launch covers that polar row alone and its
                           // across-pole taps use `wpole`
  int nr;                  // rows per wave (a band of one 64-pixel column strip)
  int nx, ny, log2nx, batch;
};

// source pixel (row, column) read by output pixel (j, i) through tap (dy, dx)
__device__ __forceinline__ void sphere_src(int j, int i, int dy, int dx, int nx, int ny, int& jj, int& ii,
                                           bool& ghost) {
  jj = j + dy;
  ii = (i + dx) & (nx - 1);
  ghost = false;
  if (jj < 0) {
    jj = 0;
    ii = (ii + (nx >> 1)) & (nx - 1);
    ghost = true;
  } else if (jj >= ny) {
    jj = ny - 1;
    ii = (ii + (nx >> 1)) & (nx - 1);
    ghost = true;
  }
}

// orders the LDS accesses of one wave (the wave's lanes run in lockstep; the
// fences keep the compiler and the memory pipeline from reordering them)
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) {
  bf16x8 v;
  __builtin_memcpy(&v, __builtin_assume_aligned(p, 16), 16);
  return v;
}

// ---------------------------------------------------------------------------
// 3x3 convolution, 32 input channels, NT*16 output channels.
// OUT: 0 = bf16 NHWC (32 channels written), 1 = float32 channel 0 only.
//
// A wave owns a 64-pixel column strip over a band of `nr` consecutive rows
// and walks down it with the input rows held in registers: entering output
// row r it holds input rows r-1, r, r+1 (across a pole: the polar row
// shifted by NX/2), and once the taps on row r-1 are issued it loads row r+2
// into that row's registers, so each input pixel is fetched from the caches
// once per wave rather than once per tap.  A row is held as four
// 16-pixel fragments in the matrix-core operand layout plus one halo fragment
// (pixel i0-1 in the lanes of fragment pixel 0, pixel i0+64 in the lanes of
// fragment pixel 15).  The taps dx = -1 and +1 take the fragments shifted by
// one pixel across lanes (DPP row shifts within each 16-lane row; the lane
// that falls off a fragment takes its neighbour fragment's edge pixel
// through a row rotation, or the halo), so no tap is re-read.
//
// The matrix-core product is C[out channel][pixel] = W[out][in] X[in][pixel]:
// the weights are the A operand (16 output channels x 32 input channels,
// staged in LDS once per workgroup; each [tap][out channel] row is padded to
// 40 elements so the 16 lanes reading one 16-byte column hit distinct banks)
// and the input fragment the B operand, so a lane's result is four
// consecutive output channels of one pixel.  Accumulation starts from the
// bias and takes the taps in the order t = 0..8 for every output.  When the taps that read across a pole need
// other weights than the rest (the adjoint in the backward pass), the two
// polar rows are computed by launches of their own (`pole_row`) whose staged
// set takes those taps from `wpole`.  Outputs are stored by conv_store.
// ---------------------------------------------------------------------------
constexpr int CONV_NR = 16;             // rows per wave: a band of one 64-pixel column strip
constexpr int WROW = CH + 8;
constexpr int OROW = CH + 8;             // padded pixel row of the output tile

// DPP controls (16-lane rows): dst[i] = src[i-1] / src[i+1] within the row
// (the lane beyond the row keeps the `old` operand), and rotations by one
// lane either way
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHL1 = 0x101, DPP_ROW_ROR1 = 0x121, DPP_ROW_ROR15 = 0x12F;

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <int CTRL>
__device__ __forceinline__ bf16x8 dpp_upd(bf16x8 old, bf16x8 src) {
  const u32x4 o = __builtin_bit_cast(u32x4, old), s = __builtin_bit_cast(u32x4, src);
  u32x4 r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = (unsigned)__builtin_amdgcn_update_dpp((int)o[k], (int)s[k], CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(bf16x8, r);
}

template <int CTRL>
__device__ __forceinline__ bf16x8 dpp_mov(bf16x8 src) {
  const u32x4 s = __builtin_bit_cast(u32x4, src);
  u32x4 r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = (unsigned)__builtin_amdgcn_mov_dpp((int)s[k], CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(bf16x8, r);
}

struct ConvRow {
  bf16x8 v[4];   // pixels i0 + 16b + (lane % 16), channels 8*(lane/16) .. +7
  bf16x8 h;      // halo: pixel i0-1 in lanes with lane % 16 == 0, i0+64 with lane % 16 == 15
};

// fragment f of a row shifted by dx pixels: lane (m, k) = pixel 16f + m + dx
template <int DX>
__device__ __forceinline__ bf16x8 conv_shift(const ConvRow& x, int f) {
  if constexpr (DX == 0) return x.v[f];
  else if constexpr (DX < 0) return dpp_upd<DPP_ROW_SHR1>(f == 0 ? x.h : dpp_mov<DPP_ROW_ROR1>(x.v[f - 1]), x.v[f]);
  else return dpp_upd<DPP_ROW_SHL1>(f == 3 ? x.h : dpp_mov<DPP_ROW_ROR15>(x.v[f + 1]), x.v[f]);
}

// CIN: channels stored per input pixel (8 for the first layer's packed input,
// whose channels beyond are zero and not stored; else CH).
// stores a wave's output row strip.  acc[n][f]: lane holds output channels
// 16n + 4*(lane/16) .. +3 of pixel 16f + lane%16 (bias included); prow: the
// strip's first pixel.  OUT == 1: float32 channel 0; else bf16 NHWC through
// the wave's LDS tile (8-byte writes of four channels, 16-byte reads and
// stores of eight), with ReLU (forward hidden layers) or the mask mk (the
// tile reads' pixels 16u + lane/4, channels 8*(lane%4) .. +7).  The stores
// are nontemporal: a layer's output is read back by the next layer's pass
// over the whole batch, far beyond what the caches hold, and streaming
// stores measured 8% faster per forward pass.
template <int NT, int OUT, bool MASK>
__device__ __forceinline__ void conv_store(const ConvArgs& A, const f32x4 (&acc)[NT][4], __bf16* tile, long long prow,
                                           int lane, const bf16x8* mk) {
  static_assert(OUT == 1 || NT == 2, "bf16 outputs carry 32 channels");
  constexpr bool RELU = OUT == 0 && !MASK;
  const int ml = lane & 15;
  if constexpr (OUT == 1) {
    if (lane < 16) {
#pragma unroll
      for (int f = 0; f < 4; ++f) __builtin_nontemporal_store(acc[0][f][0], A.out32 + prow + 16 * f + ml);
    }
  } else {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int c0 = 16 * n + 4 * (lane >> 4);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        bf16x4 o;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float v = acc[n][f][q];
          if (RELU) v = fmaxf(v, 0.f);
          o[q] = (__bf16)v;
        }
        *(bf16x4*)&tile[(16 * f + ml) * OROW + c0] = o;
      }
    }
    wave_sync_lds();
    const int c8 = 8 * (lane & 3);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int px = 16 * u + (lane >> 2);
      bf16x8 v = *(const bf16x8*)&tile[px * OROW + c8];
      if constexpr (MASK) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (!((float)mk[u][c] > 0.f)) v[c] = (__bf16)0.f;
      }
      __builtin_nontemporal_store(v, (bf16x8*)(A.out + (prow + px) * CH + c8));
    }
    wave_sync_lds();   // the tile is rewritten by the next row's epilogue
  }
}

// MASK: the output is multiplied by (mask > 0) (A.mask: the backward pass's
// input gradients).  ReLU follows the hidden layers of the forward pass
// (bf16 output without a mask) and no other convolution.
template <int NT, int OUT, int CIN, bool MASK>
__global__ __launch_bounds__(256, 3) void k_conv(ConvArgs A) {
  __shared__ __attribute__((aligned(16))) __bf16 sw[TAPS * NT * 16 * WROW];
  __shared__ __attribute__((aligned(16))) __bf16 so[OUT == 0 ? WG_WAVES : 1][OUT == 0 ? 64 * OROW : 8];
  if (A.active && !A.active[blockIdx.y]) return;   // the whole workgroup: one image
  const int tid = threadIdx.x;
  // stage the weights of the NT*16 output channels, 16 bytes a thread; in a
  // polar-row launch the taps that read across the pole come from the
  // across-pole set
  for (int k = tid; k < TAPS * NT * 16 * 4; k += 256) {
    const int row = k >> 2, q = 8 * (k & 3);       // row = tap * (NT*16) + out channel
    const int t = row / (NT * 16), co = row - t * (NT * 16);
    const int dy = t / 3 - 1;
    const bool across = A.pole_row >= 0 && ((dy < 0 && A.pole_row == 0) || (dy > 0 && A.pole_row == A.ny - 1));
    *(bf16x8*)&sw[row * WROW + q] = ld8((across ? A.wpole : A.w) + (t * CH + co) * CH + q);
  }
  __syncthreads();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int spr = A.nx >> 6;                       // 64-pixel strips per row
  const int w = blockIdx.x * WG_WAVES + wave;      // wave within the image: strip w % spr, band w / spr
  const int r0 = A.row_begin + (w / spr) * A.nr;
  if (r0 >= A.row_end) return;
  const int r1 = min(r0 + A.nr, A.row_end);
  const int i0 = (w % spr) * 64;
  const int b = blockIdx.y;
  const long long npix = (long long)A.nx * A.ny;
  const __bf16* img = A.in + (long long)b * npix * CIN;
  const int kq = 8 * (lane >> 4);          // channel block of this lane (B operand)
  const bool kin = CIN == CH || kq < CIN;  // this lane's input channels are stored
  const int ml = lane & 15;
  const int hx = ml == 0 ? i0 - 1 : (ml == 15 ? i0 + 64 : i0 + ml);   // halo pixel of this lane
  auto load_row = [&](int rr, ConvRow& x) {
    int jj = rr, sh = 0;
    if (rr < 0) {
      jj = 0;
      sh = A.nx >> 1;
    } else if (rr >= A.ny) {
      jj = A.ny - 1;
      sh = A.nx >> 1;
    }
    const __bf16* row = img + (long long)jj * A.nx * CIN + kq;
#pragma unroll
    for (int f = 0; f < 4; ++f)
      x.v[f] = kin ? ld8(row + ((i0 + 16 * f + ml + sh) & (A.nx - 1)) * CIN) : bf16x8{};
    x.h = kin ? ld8(row + ((hx + sh) & (A.nx - 1)) * CIN) : bf16x8{};
  };
  __bf16* tile = so[OUT == 0 ? wave : 0];
  // this lane's biases: output channels 16n + 4*(lane/16) .. +3 (OUT == 1: channel 0)
  float bias[NT][4];
#pragma unroll
  for (int n = 0; n < NT; ++n)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int co = OUT == 1 ? 0 : 16 * n + 4 * (lane >> 4) + q;
      bias[n][q] = A.bias ? A.bias[co] : 0.f;
    }
  const int c8 = 8 * (lane & 3);   // output tile reads: pixels 16u + lane/4, channels c8 .. c8+7
  // output row r from input rows xs (r-1), xc (r), xn (r+1); once the taps
  // of xs are issued, xs receives row `next` (when `load`)
  auto compute = [&](int r, ConvRow& xs, const ConvRow& xc, const ConvRow& xn, int next, bool load) {
    f32x4 acc[NT][4];   // the bias, then taps t = 0..8
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[n][f] = f32x4{bias[n][0], bias[n][1], bias[n][2], bias[n][3]};
    const long long prow = (long long)b * npix + (long long)r * A.nx + i0;   // first pixel of the strip
    // the mask of the row's outputs, loaded ahead of the next row's loads so
    // that waiting for it does not wait for those
    bf16x8 mk[MASK ? 4 : 1];
    if constexpr (MASK) {
#pragma unroll
      for (int u = 0; u < 4; ++u) mk[u] = ld8(A.mask + (prow + 16 * u + (lane >> 2)) * CH + c8);
    }
    auto taps = [&](auto DY, const ConvRow& x) {
      constexpr int dy = decltype(DY)::value;
      auto tap = [&](auto DX) {
        constexpr int dx = decltype(DX)::value;
        constexpr int t = (dy + 1) * 3 + (dx + 1);
        bf16x8 wf[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) wf[n] = *(const bf16x8*)&sw[(t * NT * 16 + 16 * n + ml) * WROW + kq];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const bf16x8 fr = conv_shift<dx>(x, f);
#pragma unroll
          for (int n = 0; n < NT; ++n) acc[n][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[n], fr, acc[n][f], 0, 0, 0);
        }
      };
      tap(std::integral_constant<int, -1>{});
      tap(std::integral_constant<int, 0>{});
      tap(std::integral_constant<int, 1>{});
    };
    taps(std::integral_constant<int, -1>{}, xs);
    if (load) load_row(next, xs);
    taps(std::integral_constant<int, 0>{}, xc);
    taps(std::integral_constant<int, 1>{}, xn);
    conv_store<NT, OUT, MASK>(A, acc, tile, prow, lane, mk);
  };
  // three row buffers in rotation: output row r reads (r-1, r, r+1), and the
  // buffer of row r-1 receives row r+2 once row r's taps on it are issued
  ConvRow x0, x1, x2;
  load_row(r0 - 1, x0);
  load_row(r0, x1);
  load_row(r0 + 1, x2);
#pragma unroll 1
  for (int r = r0; r < r1; r += 3) {
    compute(r, x0, x1, x2, r + 2, r + 1 < r1);
    if (r + 1 >= r1) break;
    compute(r + 1, x1, x2, x0, r + 3, r + 2 < r1);
    if (r + 2 >= r1) break;
    compute(r + 2, x2, x0, x1, r + 4, r + 3 < r1);
  }
}

// The first layer's packed input stores 8 channels per pixel, so four taps
// share one K = 32 matrix-core step: lane row s (lanes 16s .. 16s+15) of the
// input operand holds tap t = 4g + s of tap group g (t = 9..11 are zero),
// loaded directly at the tap's source pixel, and the staged weights hold
// W[4g+s][out][0..7] at k = 8s .. 8s+7.  Three groups replace nine taps, and
// no operand is shifted across lanes.  A wave walks down its column strip as
// in k_conv, loading row r+1's operands while row r is computed.  Forward
// only (one weight set).
constexpr int TGROUPS = 3;

__global__ __launch_bounds__(256, 2) void k_conv_in8(ConvArgs A) {
  constexpr int CIN = 8;
  __shared__ __attribute__((aligned(16))) __bf16 sw[TGROUPS * CH * WROW];
  __shared__ __attribute__((aligned(16))) __bf16 so[WG_WAVES][64 * OROW];
  if (A.active && !A.active[blockIdx.y]) return;   // the whole workgroup: one image
  const int tid = threadIdx.x;
  for (int k = tid; k < TGROUPS * CH * 4; k += 256) {
    const int row = k >> 2, sl = k & 3;            // row = group * CH + out channel, sl = tap slot
    const int g = row / CH, co = row - g * CH, t = 4 * g + sl;
    *(bf16x8*)&sw[row * WROW + 8 * sl] = t < TAPS ? ld8(A.w + (t * CH + co) * CH) : bf16x8{};
  }
  __syncthreads();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int spr = A.nx >> 6;
  const int w = blockIdx.x * WG_WAVES + wave;      // wave within the image: strip w % spr, band w / spr
  const int r0 = A.row_begin + (w / spr) * A.nr;
  if (r0 >= A.row_end) return;
  const int r1 = min(r0 + A.nr, A.row_end);
  const int i0 = (w % spr) * 64;
  const int b = blockIdx.y;
  const long long npix = (long long)A.nx * A.ny;
  const __bf16* img = A.in + (long long)b * npix * CIN;
  const int sl = lane >> 4, ml = lane & 15;
  __bf16* tile = so[wave];
  float bias[2][4];
#pragma unroll
  for (int n = 0; n < 2; ++n)
#pragma unroll
    for (int q = 0; q < 4; ++q) bias[n][q] = A.bias ? A.bias[16 * n + 4 * sl + q] : 0.f;
  // operands of output row r: x[g][f] = tap 4g + sl at pixels 16f + ml of the strip
  auto load = [&](int r, bf16x8 (&x)[TGROUPS][4]) {
#pragma unroll
    for (int g = 0; g < TGROUPS; ++g) {
      const int t = 4 * g + sl;
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      int jj = r + dy, sh = 0;
      if (jj < 0) {
        jj = 0;
        sh = A.nx >> 1;
      } else if (jj >= A.ny) {
        jj = A.ny - 1;
        sh = A.nx >> 1;
      }
      const __bf16* row = img + (long long)jj * A.nx * CIN;
#pragma unroll
      for (int f = 0; f < 4; ++f)
        x[g][f] = t < TAPS ? ld8(row + ((i0 + 16 * f + ml + dx + sh) & (A.nx - 1)) * CIN) : bf16x8{};
    }
  };
  auto compute = [&](int r, const bf16x8 (&x)[TGROUPS][4]) {
    f32x4 acc[2][4];   // the bias, then tap groups 0..2
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[n][f] = f32x4{bias[n][0], bias[n][1], bias[n][2], bias[n][3]};
#pragma unroll
    for (int g = 0; g < TGROUPS; ++g) {
      bf16x8 wf[2];
#pragma unroll
      for (int n = 0; n < 2; ++n) wf[n] = *(const bf16x8*)&sw[(g * CH + 16 * n + ml) * WROW + 8 * sl];
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[n][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[n], x[g][f], acc[n][f], 0, 0, 0);
    }
    const long long prow = (long long)b * npix + (long long)r * A.nx + i0;
    conv_store<2, 0, false>(A, acc, tile, prow, lane, nullptr);
  };
  bf16x8 xa[TGROUPS][4], xb[TGROUPS][4];
  load(r0, xa);
#pragma unroll 1
  for (int r = r0; r < r1; r += 2) {
    if (r + 1 < r1) load(r + 1, xb);
    compute(r, xa);
    if (r + 1 >= r1) break;
    if (r + 2 < r1) load(r + 2, xa);
    compute(r + 1, xb);
  }
}

// The first two layers fused (inference: the first layer's output is not
// kept).  A wave walks down its column strip as in k_conv; entering output
// row r of the second layer it holds the first layer's outputs for rows r-1
// and r in registers and computes row r+1 of them in between: the first
// layer's taps are packed four to a K = 32 step as in k_conv_in8, for the
// strip's four 16-pixel fragments and a fifth whose lanes 0 and 15 of each
// lane row compute pixels i0-1 and i0+64 -- the halo the second layer's dx
// taps need, computed rather than fetched.  The first layer's result lane
// (pixel m, lane row g) holds its output channels 4g..4g+3 and 16+4g..16+4g+3,
// which is the second layer's input operand once the second layer's weights
// take their input channels in that order (k = 8g + j -> channel 4g + j for
// j < 4, 16 + 4g + j - 4 else).  Beyond a pole the first layer's output row is
// its polar row seen across the pole: the polar row computed at columns
// shifted by NX/2.  The intermediate activation never leaves the chip: the
// pass reads the packed input (16 B a pixel) and writes the second layer's
// output (64 B), against 16 + 64 + 64 + 64 B for the two layers apart.
__global__ __launch_bounds__(256, 2) void k_conv12(ConvArgs A, const __bf16* w2, const float* bias2) {
  constexpr int CIN = 8;
  __shared__ __attribute__((aligned(16))) __bf16 sw1[TGROUPS * CH * WROW];
  __shared__ __attribute__((aligned(16))) __bf16 sw2[TAPS * CH * WROW];
  __shared__ __attribute__((aligned(16))) __bf16 so[WG_WAVES][64 * OROW];
  if (A.active && !A.active[blockIdx.y]) return;   // the whole workgroup: one image
  const int tid = threadIdx.x;
  for (int k = tid; k < TGROUPS * CH * 4; k += 256) {
    const int row = k >> 2, sl = k & 3;            // row = group * CH + out channel, sl = tap slot
    const int g = row / CH, co = row - g * CH, t = 4 * g + sl;
    *(bf16x8*)&sw1[row * WROW + 8 * sl] = t < TAPS ? ld8(A.w + (t * CH + co) * CH) : bf16x8{};
  }
  for (int k = tid; k < TAPS * CH * CH; k += 256) {   // [tap][out][k]: input channel order of the fused operand
    const int row = k / CH, kk = k - row * CH;        // row = tap * CH + out channel
    const int g = kk >> 3, j = kk & 7;
    const int ci = j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
    sw2[row * WROW + kk] = w2[row * CH + ci];
  }
  __syncthreads();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int spr = A.nx >> 6;
  const int w = blockIdx.x * WG_WAVES + wave;      // wave within the image: strip w % spr, band w / spr
  const int r0 = A.row_begin + (w / spr) * A.nr;
  if (r0 >= A.row_end) return;
  const int r1 = min(r0 + A.nr, A.row_end);
  const int i0 = (w % spr) * 64;
  const int b = blockIdx.y;
  const long long npix = (long long)A.nx * A.ny;
  const __bf16* img = A.in + (long long)b * npix * CIN;
  const int sl = lane >> 4, ml = lane & 15;
  const int hx = ml == 0 ? i0 - 1 : (ml == 15 ? i0 + 64 : i0 + ml);   // halo fragment pixel of this lane
  __bf16* tile = so[wave];
  float bias1[2][4], bias2v[2][4];
#pragma unroll
  for (int n = 0; n < 2; ++n)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      bias1[n][q] = A.bias ? A.bias[16 * n + 4 * sl + q] : 0.f;
      bias2v[n][q] = bias2 ? bias2[16 * n + 4 * sl + q] : 0.f;
    }
  // first-layer operands of fragment f (4: the halo fragment) of row q, the
  // columns shifted by cs (NX/2 for a row beyond a pole)
  auto l1_load = [&](int q, int cs, int f, bf16x8 (&x)[TGROUPS]) {
    const int px = (f < 4 ? i0 + 16 * f + ml : hx) + cs;
#pragma unroll
    for (int g = 0; g < TGROUPS; ++g) {
      const int t = 4 * g + sl;
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      int jj = q + dy, sh = 0;
      if (jj < 0) {
        jj = 0;
        sh = A.nx >> 1;
      } else if (jj >= A.ny) {
        jj = A.ny - 1;
        sh = A.nx >> 1;
      }
      x[g] = t < TAPS ? ld8(img + ((long long)jj * A.nx + ((px + dx + sh) & (A.nx - 1))) * CIN) : bf16x8{};
    }
  };
  // the first layer's output row q (q = -1 and ny: across the pole) as the
  // second layer's input row; l1_start issues the loads of its first
  // fragment into xa, layer1 computes it
  auto l1_row = [&](int& q, int& cs) {
    cs = 0;
    if (q < 0) {
      q = 0;
      cs = A.nx >> 1;
    } else if (q >= A.ny) {
      q = A.ny - 1;
      cs = A.nx >> 1;
    }
  };
  auto l1_start = [&](int q, bf16x8 (&xa)[TGROUPS]) {
    int cs;
    l1_row(q, cs);
    l1_load(q, cs, 0, xa);
  };
  auto layer1 = [&](int q, bf16x8 (&xa)[TGROUPS], ConvRow& out) {
    int cs;
    l1_row(q, cs);
    bf16x8 xb[TGROUPS];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      bf16x8 (&x)[TGROUPS] = (f & 1) ? xb : xa;
      if (f + 1 < 5) l1_load(q, cs, f + 1, (f & 1) ? xa : xb);
      f32x4 acc[2];
#pragma unroll
      for (int n = 0; n < 2; ++n) acc[n] = f32x4{bias1[n][0], bias1[n][1], bias1[n][2], bias1[n][3]};
#pragma unroll
      for (int g = 0; g < TGROUPS; ++g)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const bf16x8 wf = *(const bf16x8*)&sw1[(g * CH + 16 * n + ml) * WROW + 8 * sl];
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf, x[g], acc[n], 0, 0, 0);
        }
      bf16x8 o;
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) o[4 * n + qq] = (__bf16)fmaxf(acc[n][qq], 0.f);
      if (f < 4) out.v[f] = o;
      else out.h = o;
    }
  };
  // second-layer output row r from first-layer rows xs (r-1) and xc (r);
  // row r+1 is computed into xn after the taps on xs and xc are issued
  auto compute = [&](int r, const ConvRow& xs, const ConvRow& xc, ConvRow& xn) {
    f32x4 acc[2][4];
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[n][f] = f32x4{bias2v[n][0], bias2v[n][1], bias2v[n][2], bias2v[n][3]};
    auto taps = [&](auto DY, const ConvRow& x) {
      constexpr int dy = decltype(DY)::value;
      auto tap = [&](auto DX) {
        constexpr int dx = decltype(DX)::value;
        constexpr int t = (dy + 1) * 3 + (dx + 1);
        bf16x8 wf[2];
#pragma unroll
        for (int n = 0; n < 2; ++n) wf[n] = *(const bf16x8*)&sw2[(t * CH + 16 * n + ml) * WROW + 8 * sl];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const bf16x8 fr = conv_shift<dx>(x, f);
#pragma unroll
          for (int n = 0; n < 2; ++n) acc[n][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[n], fr, acc[n][f], 0, 0, 0);
        }
      };
      tap(std::integral_constant<int, -1>{});
      tap(std::integral_constant<int, 0>{});
      tap(std::integral_constant<int, 1>{});
    };
    bf16x8 xa[TGROUPS];
    l1_start(r + 1, xa);
    taps(std::integral_constant<int, -1>{}, xs);
    taps(std::integral_constant<int, 0>{}, xc);
    layer1(r + 1, xa, xn);
    taps(std::integral_constant<int, 1>{}, xn);
    const long long prow = (long long)b * npix + (long long)r * A.nx + i0;
    conv_store<2, 0, false>(A, acc, tile, prow, lane, nullptr);
  };
  ConvRow x0, x1, x2;
  {
    bf16x8 xa[TGROUPS];
    l1_start(r0 - 1, xa);
    layer1(r0 - 1, xa, x0);
    l1_start(r0, xa);
    layer1(r0, xa, x1);
  }
#pragma unroll 1
  for (int r = r0; r < r1; r += 3) {
    compute(r, x0, x1, x2);
    if (r + 1 >= r1) break;
    compute(r + 1, x1, x2, x0);
    if (r + 2 >= r1) break;
    compute(r + 2, x2, x0, x1);
  }
}

// The last two layers fused (inference: the fourth layer's output is not
// kept).  A wave walks down its column strip holding the fourth layer's input
// rows (ConvRow plus a second halo: pixels i0-2 and i0+65 in the lanes of
// fragment pixels 0 and 15) and the fourth layer's output rows r-1, r, r+1.
// The fourth layer computes its output for the strip's four fragments by the
// DPP-shifted taps of k_conv and for a fifth fragment whose lanes 0 and 15
// compute pixels i0-1 and i0+64 (their dx taps read i0-2, i0-1, i0 and i0+63,
// i0+64, i0+65, all held), so the last layer's halo is computed rather than
// fetched.  Its result lane (pixel m, lane row g) holds channels 4g..4g+3 and
// 16+4g..16+4g+3, the last layer's input operand once the last layer's
// weights take their input channels in that order.  Beyond a pole the fourth
// layer's output row is its polar row computed at columns shifted by NX/2.
// The pass reads the fourth layer's input (64 B a pixel) and writes the
// float32 output (4 B), against 64 + 64 + 64 + 4 B for the two layers apart.
struct ConvRow2 {
  ConvRow x;
  bf16x8 h2;     // pixel i0-2 in lanes with lane % 16 == 0, i0+65 with lane % 16 == 15
};

__global__ __launch_bounds__(256, 2) void k_conv45(ConvArgs A, const __bf16* w5, const float* bias5) {
  __shared__ __attribute__((aligned(16))) __bf16 sw4[TAPS * CH * WROW];
  __shared__ __attribute__((aligned(16))) __bf16 sw5[TAPS * 16 * WROW];
  if (A.active && !A.active[blockIdx.y]) return;   // the whole workgroup: one image
  const int tid = threadIdx.x;
  for (int k = tid; k < TAPS * CH * 4; k += 256) {
    const int row = k >> 2, q = 8 * (k & 3);       // row = tap * CH + out channel
    *(bf16x8*)&sw4[row * WROW + q] = ld8(A.w + row * CH + q);
  }
  for (int k = tid; k < TAPS * 16 * CH; k += 256) {   // [tap][out][k]: input channel order of the fused operand
    const int row = k / CH, kk = k - row * CH;        // row = tap * 16 + out channel
    const int t = row >> 4, co = row & 15;
    const int g = kk >> 3, j = kk & 7;
    const int ci = j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
    sw5[row * WROW + kk] = w5[(t * CH + co) * CH + ci];
  }
  __syncthreads();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int spr = A.nx >> 6;
  const int w = blockIdx.x * WG_WAVES + wave;      // wave within the image: strip w % spr, band w / spr
  const int r0 = A.row_begin + (w / spr) * A.nr;
  if (r0 >= A.row_end) return;
  const int r1 = min(r0 + A.nr, A.row_end);
  const int i0 = (w % spr) * 64;
  const int b = blockIdx.y;
  const long long npix = (long long)A.nx * A.ny;
  const __bf16* img = A.in + (long long)b * npix * CH;
  const int kq = 8 * (lane >> 4), sl = lane >> 4, ml = lane & 15;
  const int hx = ml == 0 ? i0 - 1 : (ml == 15 ? i0 + 64 : i0 + ml);
  const int hx2 = ml == 0 ? i0 - 2 : (ml == 15 ? i0 + 65 : i0 + ml);
  float bias4[2][4], b5 = bias5 ? bias5[0] : 0.f;
#pragma unroll
  for (int n = 0; n < 2; ++n)
#pragma unroll
    for (int q = 0; q < 4; ++q) bias4[n][q] = A.bias ? A.bias[16 * n + 4 * sl + q] : 0.f;
  // the fourth layer's input row rr, columns shifted by cs
  auto load_row = [&](int rr, int cs, ConvRow2& x) {
    int jj = rr, sh = cs;
    if (rr < 0) {
      jj = 0;
      sh += A.nx >> 1;
    } else if (rr >= A.ny) {
      jj = A.ny - 1;
      sh += A.nx >> 1;
    }
    const __bf16* row = img + (long long)jj * A.nx * CH + kq;
#pragma unroll
    for (int f = 0; f < 4; ++f) x.x.v[f] = ld8(row + ((i0 + 16 * f + ml + sh) & (A.nx - 1)) * CH);
    x.x.h = ld8(row + ((hx + sh) & (A.nx - 1)) * CH);
    x.h2 = ld8(row + ((hx2 + sh) & (A.nx - 1)) * CH);
  };
  // the fourth layer's output row from its input rows xs, xc, xn, as the last
  // layer's input row
  auto layer4 = [&](const ConvRow2& xs, const ConvRow2& xc, const ConvRow2& xn, ConvRow& out) {
    // fragments F0 .. F0+NF-1 at a time (fewer accumulators live; the taps'
    // weights are read once per group)
    auto group = [&](auto F0_, auto NF_) {
      constexpr int F0 = decltype(F0_)::value, NF = decltype(NF_)::value;
      f32x4 acc[2][NF];
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[n][f] = f32x4{bias4[n][0], bias4[n][1], bias4[n][2], bias4[n][3]};
      auto taps = [&](auto DY, const ConvRow2& x) {
        constexpr int dy = decltype(DY)::value;
        auto tap = [&](auto DX) {
          constexpr int dx = decltype(DX)::value;
          constexpr int t = (dy + 1) * 3 + (dx + 1);
          bf16x8 wf[2];
#pragma unroll
          for (int n = 0; n < 2; ++n) wf[n] = *(const bf16x8*)&sw4[(t * CH + 16 * n + ml) * WROW + kq];
#pragma unroll
          for (int i = 0; i < NF; ++i) {
            const int f = F0 + i;
            bf16x8 fr;
            if (f < 4) fr = conv_shift<dx>(x.x, f);
            else if (dx == 0) fr = x.x.h;
            else if (dx < 0) fr = ml == 0 ? x.h2 : x.x.v[3];   // lane 0: i0-2; lane 15: i0+63
            else fr = ml == 15 ? x.h2 : x.x.v[0];                 // lane 0: i0; lane 15: i0+65
#pragma unroll
            for (int n = 0; n < 2; ++n) acc[n][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[n], fr, acc[n][i], 0, 0, 0);
          }
        };
        tap(std::integral_constant<int, -1>{});
        tap(std::integral_constant<int, 0>{});
        tap(std::integral_constant<int, 1>{});
      };
      taps(std::integral_constant<int, -1>{}, xs);
      taps(std::integral_constant<int, 0>{}, xc);
      taps(std::integral_constant<int, 1>{}, xn);
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        bf16x8 o;
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int q = 0; q < 4; ++q) o[4 * n + q] = (__bf16)fmaxf(acc[n][i][q], 0.f);
        if (F0 + i < 4) out.v[F0 + i] = o;
        else out.h = o;
      }
    };
    group(std::integral_constant<int, 0>{}, std::integral_constant<int, 3>{});
    __builtin_amdgcn_sched_barrier(0);   // keeps the groups' weight reads from being hoisted together
    group(std::integral_constant<int, 3>{}, std::integral_constant<int, 2>{});
    __builtin_amdgcn_sched_barrier(0);
  };
  // the fourth layer's output row q = -1 or ny (across the pole: the polar
  // row at columns shifted by NX/2), its input rows loaded into ys, yc, yn
  auto layer4_pole = [&](int q, ConvRow2& ys, ConvRow2& yc, ConvRow2& yn, ConvRow& out) {
    const int qp = q < 0 ? 0 : A.ny - 1, cs = A.nx >> 1;
    load_row(qp - 1, cs, ys);
    load_row(qp, cs, yc);
    load_row(qp + 1, cs, yn);
    layer4(ys, yc, yn, out);
  };
  // last layer, output row r from the fourth layer's rows as, ac, an
  auto layer5 = [&](int r, const ConvRow& as, const ConvRow& ac, const ConvRow& an) {
    f32x4 acc[1][4];
#pragma unroll
    for (int f = 0; f < 4; ++f) acc[0][f] = f32x4{b5, b5, b5, b5};
    auto taps = [&](auto DY, const ConvRow& x) {
      constexpr int dy = decltype(DY)::value;
      auto tap = [&](auto DX) {
        constexpr int dx = decltype(DX)::value;
        constexpr int t = (dy + 1) * 3 + (dx + 1);
        const bf16x8 wf = *(const bf16x8*)&sw5[(t * 16 + ml) * WROW + kq];
#pragma unroll
        for (int f = 0; f < 4; ++f)
          acc[0][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf, conv_shift<dx>(x, f), acc[0][f], 0, 0, 0);
      };
      tap(std::integral_constant<int, -1>{});
      tap(std::integral_constant<int, 0>{});
      tap(std::integral_constant<int, 1>{});
    };
    taps(std::integral_constant<int, -1>{}, as);
    taps(std::integral_constant<int, 0>{}, ac);
    taps(std::integral_constant<int, 1>{}, an);
    const long long prow = (long long)b * npix + (long long)r * A.nx + i0;
    conv_store<1, 1, false>(A, acc, nullptr, prow, lane, nullptr);
  };
  // fourth-layer output rows r-1, r (a0, a1) and input rows r, r+1 (x1, x2)
  ConvRow a0, a1, a2;
  ConvRow2 x0, x1, x2;
  if (r0 == 0) layer4_pole(-1, x0, x1, x2, a0);
  else {
    load_row(r0 - 2, 0, x0);
    load_row(r0 - 1, 0, x1);
    load_row(r0, 0, x2);
    layer4(x0, x1, x2, a0);
  }
  load_row(r0 - 1, 0, x0);
  load_row(r0, 0, x1);
  load_row(r0 + 1, 0, x2);
  layer4(x0, x1, x2, a1);
  // step r: input row r+2 into the buffer of row r-1, the fourth layer's row
  // r+1 into the buffer of row r-2, then the last layer's row r
  // (at the south pole the row r+1 beyond it; the input buffers are free then)
  auto step = [&](int r, ConvRow2& xs, ConvRow2& xc, ConvRow2& xn, const ConvRow& as, const ConvRow& ac, ConvRow& an) {
    if (r + 1 < A.ny) {
      load_row(r + 2, 0, xs);
      layer4(xc, xn, xs, an);
    } else {
      layer4_pole(r + 1, xs, xc, xn, an);
    }
    layer5(r, as, ac, an);
  };
#pragma unroll 1
  for (int r = r0; r < r1; r += 3) {
    step(r, x0, x1, x2, a0, a1, a2);
    if (r + 1 >= r1) break;
    step(r + 1, x1, x2, x0, a1, a2, a0);
    if (r + 2 >= r1) break;
    step(r + 2, x2, x0, x1, a2, a0, a1);
  }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients of a 3x3 convolution:
//   dW[t][co][ci] = sum_q dpre[q][co] * in[src_t(q)][ci],  db[co] = sum_q dpre[q][co]
// an implicit GEMM with M = co, N = ci and K = pixels.  Each wave walks
// `chunks` chunks of 32 pixels of one row, transposing the dpre and input
// blocks through wave-private LDS so the MFMA operands are 16-byte reads, and
// writes its partial sums; k_wgrad_reduce adds the partials in a fixed order.
// ---------------------------------------------------------------------------
constexpr int WG_Q = 32;                 // pixels per K chunk
constexpr int WG_LD = WG_Q + 8;          // padded LDS row (16-byte aligned)
constexpr int WG_PART = TAPS * CH * CH + CH;

struct WgradArgs {
  const __bf16* in;        // layer input [B][ny][nx][in_stride]
  const __bf16* dpre;      // gradient at the layer output before activation [B][ny][nx][CH]
  float* part;             // [nwaves][WG_PART]
  int nx, ny, log2nx, batch;
  int in_stride;           // channels stored per input pixel (8 or CH; channels beyond are zero)
  int chunks;              // 32-pixel chunks per wave
  long long total_chunks;
};

__global__ __launch_bounds__(256) void k_wgrad(WgradArgs A) {
  __shared__ __attribute__((aligned(16))) __bf16 sd[WG_WAVES][CH][WG_LD];
  __shared__ __attribute__((aligned(16))) __bf16 sa[WG_WAVES][CH][WG_LD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const long long gw = (long long)blockIdx.x * WG_WAVES + wave;
  const long long c0 = gw * A.chunks;
  float* part = A.part + gw * WG_PART;
  f32x4 acc[TAPS][2][2];
#pragma unroll
  for (int t = 0; t < TAPS; ++t)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[t][a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbias = 0.f;
  const int npix = A.nx * A.ny;
  const int chunks_per_image = npix / WG_Q;
  const int ql = lane >> 1, ch0 = 16 * (lane & 1);   // staging: pixel ql, channels ch0..ch0+15
  const int kq = 8 * (lane >> 4), ml = lane & 15;
  for (int c = 0; c < A.chunks; ++c) {
    const long long chunk = c0 + c;
    if (chunk >= A.total_chunks) break;      // uniform over the wave
    const int b = (int)(chunk / chunks_per_image);
    const int p0 = (int)(chunk % chunks_per_image) * WG_Q;
    const int j = p0 >> A.log2nx, i0 = p0 & (A.nx - 1);
    // dpre block, transposed to [co][q]
    {
      const __bf16* src = A.dpre + ((long long)b * npix + p0 + ql) * CH + ch0;
      const bf16x8 v0 = ld8(src), v1 = ld8(src + 8);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        sd[wave][ch0 + k][ql] = v0[k];
        sd[wave][ch0 + 8 + k][ql] = v1[k];
      }
    }
    wave_sync_lds();
    if (lane < CH) {
      float s = 0.f;
#pragma unroll 8
      for (int q = 0; q < WG_Q; ++q) s += (float)sd[wave][lane][q];
      dbias += s;
    }
    bf16x8 afr[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) afr[mt] = *(const bf16x8*)&sd[wave][16 * mt + ml][kq];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) {
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      int jj, ii;
      bool ghost;
      sphere_src(j, i0 + ql, dy, dx, A.nx, A.ny, jj, ii, ghost);
      const __bf16* src = A.in + ((long long)b * npix + (long long)jj * A.nx + ii) * A.in_stride + ch0;
      const bf16x8 v0 = ch0 < A.in_stride ? ld8(src) : bf16x8{};
      const bf16x8 v1 = ch0 + 8 < A.in_stride ? ld8(src + 8) : bf16x8{};
      wave_sync_lds();   // previous tap's reads of sa are complete
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        sa[wave][ch0 + k][ql] = v0[k];
        sa[wave][ch0 + 8 + k][ql] = v1[k];
      }
      wave_sync_lds();
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const bf16x8 bfr = *(const bf16x8*)&sa[wave][16 * nt + ml][kq];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
          acc[t][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[mt], bfr, acc[t][mt][nt], 0, 0, 0);
      }
    }
    wave_sync_lds();   // sd is rewritten by the next chunk
  }
  // partial sums: C lane layout co = 16 mt + 4*(lane/16) + r, ci = 16 nt + lane%16
#pragma unroll
  for (int t = 0; t < TAPS; ++t)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = 16 * mt + 4 * (lane >> 4) + r, ci = 16 * nt + ml;
          part[(t * CH + co) * CH + ci] = acc[t][mt][nt][r];
        }
  if (lane < CH) part[TAPS * CH * CH + lane] = dbias;
}

// grad[k] = sum over waves of part[w][k] in a fixed order, in two levels:
// segment sums (blockIdx.y = segment of the wave range), then their sum
constexpr int WG_SEG = 64;
__global__ void k_wgrad_reduce(const float* part, int nwaves, float* seg) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= WG_PART) return;
  const int per = (nwaves + WG_SEG - 1) / WG_SEG;
  const int w0 = blockIdx.y * per, w1 = min(nwaves, w0 + per);
  float s = 0.f;
  for (int w = w0; w < w1; ++w) s += part[(long long)w * WG_PART + k];
  seg[(long long)blockIdx.y * WG_PART + k] = s;
}
__global__ void k_wgrad_reduce2(const float* seg, float* grad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= WG_PART) return;
  float s = 0.f;
  for (int g = 0; g < WG_SEG; ++g) s += seg[(long long)g * WG_PART + k];
  grad[k] = s;
}

}  // namespace mpgcr
