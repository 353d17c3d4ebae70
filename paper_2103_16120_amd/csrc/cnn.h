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

#include "device.h"

namespace mpgcr {

constexpr int CNN_LAYERS = 5;
constexpr int TAPS = 9;             // tap t = (dy+1)*3 + (dx+1)
constexpr int CONV_MT = 4;          // 16-pixel M tiles per wave (64 pixels)
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
  int nx, ny, log2nx, batch;
  int relu;
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
// OUT: 0 = bf16 NHWC (32 channels written, the upper 16 zero when NT == 1),
//      1 = float32 channel 0 only.
// A workgroup covers CONV_SPW groups of four consecutive 64-pixel strips, one
// strip per wave at a time.  A wave first stages its strip's input -- the
// three rows j-1, j, j+1 (across a pole: the polar row shifted by NX/2) over
// pixels i0-1 .. i0+64, all stored channels -- in an LDS tile of its own, 16
// bytes a lane per load, so each input pixel is fetched from the caches once
// per row instead of once per tap; it then computes the strip two 16-pixel
// tiles at a time from the tile (the 18 input fragments of a tile pair are
// read before the MFMAs that use them).
// The four waves share the weight fragments staged in LDS once per workgroup;
// each [tap][out channel] row of 32 input channels is padded to 40 elements so
// that the 16 lanes reading one 16-byte column hit distinct banks.  When the
// taps that read across a pole need other weights than the rest (the adjoint
// in the backward pass), the two polar rows are computed by launches of their
// own (`pole_row`) whose staged set takes those taps from `wpole`, so the LDS
// holds one set of nine taps.  bf16 outputs go through a per-wave
// LDS tile so that each lane stores 16 contiguous bytes (8 channels of one
// pixel); the backward ReLU mask is applied there, 8 channels at a time.
// ---------------------------------------------------------------------------
constexpr int WROW = CH + 8;
constexpr int CONV_SPW = 4;              // strip groups per workgroup
constexpr int OROW = CH + 8;             // padded pixel row of the output tile
constexpr int SPX = 64 + 2;              // staged pixels per row: the strip and one on each side

// CIN: channels stored per input pixel (8 for the first layer's packed input,
// whose channels beyond are zero and not stored; else CH).
template <int NT, int OUT, int CIN>
__global__ __launch_bounds__(256) void k_conv(ConvArgs A) {
  __shared__ __attribute__((aligned(16))) __bf16 sw[TAPS * CH * WROW];
  __shared__ __attribute__((aligned(16))) __bf16 so[WG_WAVES][16 * OROW];
  __shared__ __attribute__((aligned(16))) __bf16 si[WG_WAVES][3 * SPX * CIN];   // [row][pixel][channel]
  if (A.active && !A.active[blockIdx.y]) return;   // the whole workgroup: one image
  const int tid = threadIdx.x;
  const int npix = A.nx * A.ny;
  const int spr = A.nx >> 6;                       // 64-pixel strips per row
  const long long s_first = (long long)A.row_begin * spr + (long long)blockIdx.x * CONV_SPW * WG_WAVES;
  const long long s_end = (long long)A.row_end * spr;
  // stage the weights, 16 bytes a thread; in a polar-row launch the taps that
  // read across the pole come from the across-pole set
  for (int k = tid; k < TAPS * CH * 4; k += 256) {
    const int row = k >> 2, q = 8 * (k & 3);
    const int dy = (row >> 5) / 3 - 1;             // row = tap * CH + out channel
    const bool across = A.pole_row >= 0 && ((dy < 0 && A.pole_row == 0) || (dy > 0 && A.pole_row == A.ny - 1));
    *(bf16x8*)&sw[row * WROW + q] = ld8((across ? A.wpole : A.w) + row * CH + q);
  }
  __syncthreads();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int b = blockIdx.y;
  const __bf16* img = A.in + (long long)b * npix * CIN;
  const int kq = 8 * (lane >> 4);          // channel block of this lane (A and B operands)
  const bool kin = CIN == CH || kq < CIN;  // this lane's input channels are stored
  const int ml = lane & 15;
  __bf16* tile = so[wave];
  __bf16* stage = si[wave];
  constexpr int CPP = CIN / 8;             // 16-byte chunks per staged pixel
  constexpr int NCH = 3 * SPX * CPP, NLD = (NCH + 63) / 64;
  // the staged input of a strip: rows j-1 .. j+1, pixels i0-1 .. i0+64; the
  // loads of the next strip are issued before the current strip's MFMAs and
  // written to the tile after them (one tile per wave, two syncs per strip)
  bf16x8 buf[NLD];
  auto fetch = [&](long long strip) {
    const int p0 = (int)(strip * 64);
    const int j = p0 >> A.log2nx, i0 = p0 & (A.nx - 1);
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int c = lane + 64 * u;
      if (c < NCH) {
        const int r = c / (SPX * CPP), rem = c - r * (SPX * CPP);
        const int px = rem / CPP, q = rem - px * CPP;
        int jj, ii;
        bool ghost;
        sphere_src(j, i0 - 1 + px, r - 1, 0, A.nx, A.ny, jj, ii, ghost);
        buf[u] = ld8(img + ((long long)jj * A.nx + ii) * CIN + 8 * q);
      }
    }
  };
  auto put = [&]() {
    wave_sync_lds();   // the previous strip's reads of the tile come first
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int c = lane + 64 * u;
      if (c < NCH) *(bf16x8*)&stage[c * 8] = buf[u];   // chunk c = (row, pixel, 16-byte channel block)
    }
    wave_sync_lds();
  };
  if (s_first + wave < s_end) {
    fetch(s_first + wave);
    put();
  }
#pragma unroll 1
  for (int g = 0; g < CONV_SPW; ++g) {
    const long long strip = s_first + g * WG_WAVES + wave;
    if (strip >= s_end) break;
    const int p0 = (int)(strip * 64);
    const long long next = strip + WG_WAVES;
    const bool more = g + 1 < CONV_SPW && next < s_end;
    if (more) fetch(next);
#pragma unroll 1
    for (int mt = 0; mt < CONV_MT; mt += 2) {
      bf16x8 a[2][TAPS];
#pragma unroll
      for (int t = 0; t < TAPS; ++t) {
        const int dy = t / 3 - 1, dx = t % 3 - 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int px = 16 * (mt + h) + ml + dx + 1;
          a[h][t] = kin ? *(const bf16x8*)&stage[((dy + 1) * SPX + px) * CIN + kq] : bf16x8{};
        }
      }
      f32x4 acc[2][NT];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[h][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < TAPS; ++t) {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const bf16x8 bw = *(const bf16x8*)&sw[(t * CH + 16 * n + ml) * WROW + kq];
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[h][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[h][t], bw, acc[h][n], 0, 0, 0);
        }
      }
      // epilogue: lane holds output channel co = 16n + ml of pixels 4*(lane/16) .. +3 of each tile
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const long long pt = (long long)b * npix + p0 + 16 * (mt + h);   // first pixel of the tile
        if (OUT == 1) {
          if (ml == 0) {
            const float bias = A.bias ? A.bias[0] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              float v = acc[h][0][r] + bias;
              if (A.relu) v = fmaxf(v, 0.f);
              A.out32[pt + 4 * (lane >> 4) + r] = v;
            }
          }
        } else {
#pragma unroll
          for (int n = 0; n < NT; ++n) {
            const int co = 16 * n + ml;
            const float bias = A.bias ? A.bias[co] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              float v = acc[h][n][r] + bias;
              if (A.relu) v = fmaxf(v, 0.f);
              tile[(4 * (lane >> 4) + r) * OROW + co] = (__bf16)v;
            }
          }
          if (NT == 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tile[(4 * (lane >> 4) + r) * OROW + 16 + ml] = (__bf16)0.f;
          }
          wave_sync_lds();
          // lane: pixel lane/4 of the tile, channels 8*(lane%4) .. +7
          const int px = lane >> 2, c8 = 8 * (lane & 3);
          bf16x8 v = *(const bf16x8*)&tile[px * OROW + c8];
          const long long o = (pt + px) * CH + c8;
          if (A.mask) {
            const bf16x8 mk = ld8(A.mask + o);
#pragma unroll
            for (int c = 0; c < 8; ++c)
              if (!((float)mk[c] > 0.f)) v[c] = (__bf16)0.f;
          }
          *(bf16x8*)(A.out + o) = v;
          wave_sync_lds();   // the tile is rewritten by the next tile's epilogue
        }
      }
    }
    if (more) put();
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
