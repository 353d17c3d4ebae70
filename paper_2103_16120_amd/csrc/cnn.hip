// Host side of the learned-preconditioner network (see cnn.h and the cnn_*
// declarations in include/mpgcr.h): parameter packing, forward pass, loss,
// backward pass and Adam, all on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mpgcr.h"
#include "cnn.h"
#include "cnn_internal.h"

using namespace mpgcr;

namespace {
thread_local std::string g_cnn_error;

int cfail(cnn_net* n, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (n) n->err = buf;
  else g_cnn_error = buf;
  return code;
}
}  // namespace

#define CHK(n, call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return cfail((n), GCR_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// parameter layout (float32, the reference layout): for each layer l,
// w_l [co][ci][3][3] then b_l [co]; shapes c_in->32->32->32->32->1
static void layer_shape(int c_in, int l, int& co, int& ci) {
  ci = l == 0 ? c_in : CH;
  co = l == CNN_LAYERS - 1 ? 1 : CH;
}

extern "C" int64_t cnn_param_count(int c_in) {
  if (c_in < 1 || c_in > CH) return -1;
  int64_t n = 0;
  for (int l = 0; l < CNN_LAYERS; ++l) {
    int co, ci;
    layer_shape(c_in, l, co, ci);
    n += (int64_t)co * ci * 9 + co;
  }
  return n;
}

// ---------------------------------------------------------------------------
// device kernels
// ---------------------------------------------------------------------------
struct PackW {
  const float* params;
  __bf16* wf;     // [layer][TAPS][CH][CH] forward: [t][co][ci]
  __bf16* wa;     // adjoint: [t'][ci][co] = w[co][ci][-t']
  __bf16* wp;     // adjoint across a pole: [t'][ci][co] = w[co][ci][(dy', -dx')]
  float* bias;    // [layer][CH]
  int c_in;
  long long off[CNN_LAYERS];
  int co[CNN_LAYERS], ci[CNN_LAYERS];
};

__global__ void k_pack_weights(PackW P) {
  const int l = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;   // over TAPS*CH*CH
  if (idx >= TAPS * CH * CH) return;
  const int t = idx / (CH * CH), a = (idx / CH) % CH, c = idx % CH;
  const int co_n = P.co[l], ci_n = P.ci[l];
  const float* w = P.params + P.off[l];
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  // forward: out channel a = co, in channel c = ci, tap t
  float vf = (a < co_n && c < ci_n) ? w[((a * ci_n + c) * 3 + (dy + 1)) * 3 + (dx + 1)] : 0.f;
  // adjoint: out channel a = ci, in channel c = co
  const int ty = -dy, tx = -dx;
  float va = (c < co_n && a < ci_n) ? w[((c * ci_n + a) * 3 + (ty + 1)) * 3 + (tx + 1)] : 0.f;
  float vp = (c < co_n && a < ci_n) ? w[((c * ci_n + a) * 3 + (dy + 1)) * 3 + (tx + 1)] : 0.f;
  const long long o = (long long)l * TAPS * CH * CH + idx;
  P.wf[o] = (__bf16)vf;
  P.wa[o] = (__bf16)va;
  P.wp[o] = (__bf16)vp;
  if (t == 0 && c == 0) P.bias[l * CH + a] = a < co_n ? w[(long long)co_n * ci_n * 9 + a] : 0.f;
}

// NCHW float32 [B][c_in][ny][nx] -> NHWC bf16 [B][ny][nx][stride], one pixel
// (four 16-byte stores) per thread
__global__ void k_pack_input(const float* in, __bf16* out, int c_in, long long npix, int batch, int stride) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= npix * batch) return;
  const long long b = k / npix, p = k % npix;
  bf16x8* dst = (bf16x8*)(out + k * stride);
  for (int q = 0; q < stride / 8; ++q) {
    bf16x8 v;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int ch = 8 * q + c;
      v[c] = (__bf16)(ch < c_in ? in[(b * c_in + ch) * npix + p] : 0.f);
    }
    dst[q] = v;
  }
}

// float32 [B][npix] -> NHWC bf16 channel 0 (others zero)
__global__ void k_pack_grad(const float* g, __bf16* out, long long n) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= n) return;
  bf16x8 v;
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = (__bf16)0.f;
  bf16x8* dst = (bf16x8*)(out + k * CH);
  dst[1] = v;
  dst[2] = v;
  dst[3] = v;
  v[0] = (__bf16)g[k];
  dst[0] = v;
}

// mean squared error: per-block partial sums of (y-t)^2 (fixed order) and
// dy = 2 (y - t) / n
__global__ void k_mse(const float* y, const float* t, float* dy, double* part, long long n) {
  __shared__ double red[256];
  double s = 0.0;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
    const float d = y[k] - t[k];
    dy[k] = 2.f * d / (float)n;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// fragment-layout gradients [t][co][ci] + db[co] -> reference layout
struct UnpackG {
  const float* g;      // [WG_PART] of one layer
  float* flat;         // destination: w [co][ci][3][3] then b
  int co, ci;
};
__global__ void k_unpack_grad(UnpackG U) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int nw = U.co * U.ci * 9;
  if (k < nw) {
    const int co = k / (U.ci * 9), ci = (k / 9) % U.ci, t = k % 9;
    U.flat[k] = U.g[(t * CH + co) * CH + ci];
  } else if (k < nw + U.co) {
    U.flat[k] = U.g[TAPS * CH * CH + (k - nw)];
  }
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
static int alloc_all(cnn_net* n) {
  hipError_t e = hipSuccess;
  auto A = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes ? bytes : 1);
    if (e == hipSuccess) n->allocs.push_back(*p);
  };
  const size_t npix = (size_t)n->nx * n->ny * n->max_batch;
  A((void**)&n->params, n->nparams * sizeof(float));
  A((void**)&n->grads, n->nparams * sizeof(float));
  A((void**)&n->adam_m, n->nparams * sizeof(float));
  A((void**)&n->adam_v, n->nparams * sizeof(float));
  A((void**)&n->wf, (size_t)CNN_LAYERS * TAPS * CH * CH * sizeof(__bf16));
  A((void**)&n->wa, (size_t)CNN_LAYERS * TAPS * CH * CH * sizeof(__bf16));
  A((void**)&n->wp, (size_t)CNN_LAYERS * TAPS * CH * CH * sizeof(__bf16));
  A((void**)&n->bias, (size_t)CNN_LAYERS * CH * sizeof(float));
  for (int l = 0; l < CNN_LAYERS; ++l) A((void**)&n->act[l], npix * (l == 0 ? n->in_stride : CH) * sizeof(__bf16));
  A((void**)&n->dbuf[0], npix * CH * sizeof(__bf16));
  A((void**)&n->dbuf[1], npix * CH * sizeof(__bf16));
  A((void**)&n->y, npix * sizeof(float));
  A((void**)&n->dy, npix * sizeof(float));
  n->wg_chunks = 32;
  n->wg_waves_max = (int)((npix / WG_Q + n->wg_chunks - 1) / n->wg_chunks);
  n->wg_waves_max = (n->wg_waves_max + WG_WAVES - 1) / WG_WAVES * WG_WAVES;
  A((void**)&n->wg_part, (size_t)n->wg_waves_max * WG_PART * sizeof(float));
  A((void**)&n->wg_sum, (size_t)WG_PART * sizeof(float));
  A((void**)&n->wg_seg, (size_t)WG_SEG * WG_PART * sizeof(float));
  A((void**)&n->loss_part, 1024 * sizeof(double));
  if (e != hipSuccess) return cfail(n, e == hipErrorOutOfMemory ? GCR_ENOMEM : GCR_EHIP, "allocation: %s",
                                    hipGetErrorString(e));
  if (hipHostMalloc((void**)&n->loss_host, 1024 * sizeof(double), 0) != hipSuccess)
    return cfail(n, GCR_ENOMEM, "pinned allocation failed");
  return GCR_OK;
}

static void free_all(cnn_net* n) {
  for (void* p : n->allocs) (void)hipFree(p);
  n->allocs.clear();
  if (n->loss_host) (void)hipHostFree(n->loss_host);
  n->loss_host = nullptr;
}

extern "C" int cnn_create(int32_t nx, int32_t ny, int32_t max_batch, int32_t c_in, void* stream, cnn_net** out) {
  if (out) *out = nullptr;
  if (!out) return cfail(nullptr, GCR_EINVAL, "cnn_create: NULL out");
  if (nx < 64 || nx > NXMAX || (nx & (nx - 1))) return cfail(nullptr, GCR_EINVAL, "nx must be a power of two in [64, 1024]");
  if (ny < 2 || ny > 4096) return cfail(nullptr, GCR_EINVAL, "ny must be in [2, 4096]");
  if (max_batch < 1 || max_batch > 4096) return cfail(nullptr, GCR_EINVAL, "max_batch must be in [1, 4096]");
  if (c_in < 1 || c_in > CH) return cfail(nullptr, GCR_EINVAL, "c_in must be in [1, 32]");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return cfail(nullptr, GCR_EHIP, "no HIP device available");
  cnn_net* n = new (std::nothrow) cnn_net();
  if (!n) return cfail(nullptr, GCR_ENOMEM, "host allocation failed");
  n->nx = nx;
  n->ny = ny;
  n->log2nx = 0;
  while ((1 << n->log2nx) < nx) ++n->log2nx;
  n->max_batch = max_batch;
  n->c_in = c_in;
  n->in_stride = c_in <= 8 ? 8 : CH;
  n->stream = (hipStream_t)stream;
  n->nparams = cnn_param_count(c_in);
  int rc = alloc_all(n);
  if (rc != GCR_OK) {
    g_cnn_error = n->err;
    free_all(n);
    delete n;
    return rc;
  }
  (void)hipMemsetAsync(n->params, 0, n->nparams * sizeof(float), n->stream);
  (void)hipMemsetAsync(n->adam_m, 0, n->nparams * sizeof(float), n->stream);
  (void)hipMemsetAsync(n->adam_v, 0, n->nparams * sizeof(float), n->stream);
  if (hipStreamSynchronize(n->stream) != hipSuccess) {
    free_all(n);
    delete n;
    return cfail(nullptr, GCR_EHIP, "initialisation failed");
  }
  *out = n;
  return GCR_OK;
}

extern "C" int cnn_destroy(cnn_net* n) {
  if (!n) return GCR_OK;
  (void)hipStreamSynchronize(n->stream);
  free_all(n);
  delete n;
  return GCR_OK;
}

static int pack_weights(cnn_net* n) {
  PackW P{};
  P.params = n->params;
  P.wf = n->wf;
  P.wa = n->wa;
  P.wp = n->wp;
  P.bias = n->bias;
  P.c_in = n->c_in;
  long long off = 0;
  for (int l = 0; l < CNN_LAYERS; ++l) {
    layer_shape(n->c_in, l, P.co[l], P.ci[l]);
    P.off[l] = off;
    off += (long long)P.co[l] * P.ci[l] * 9 + P.co[l];
  }
  hipLaunchKernelGGL(k_pack_weights, dim3((TAPS * CH * CH + 255) / 256, CNN_LAYERS), dim3(256), 0, n->stream, P);
  CHK(n, hipGetLastError());
  return GCR_OK;
}

extern "C" int cnn_set_params(cnn_net* n, const float* host, int64_t count) {
  if (!n || !host) return GCR_EINVAL;
  if (count != n->nparams) return cfail(n, GCR_EINVAL, "expected %lld parameters", (long long)n->nparams);
  CHK(n, hipMemcpyAsync(n->params, host, count * sizeof(float), hipMemcpyHostToDevice, n->stream));
  CHK(n, hipMemsetAsync(n->adam_m, 0, count * sizeof(float), n->stream));
  CHK(n, hipMemsetAsync(n->adam_v, 0, count * sizeof(float), n->stream));
  n->adam_t = 0;
  int rc = pack_weights(n);
  if (rc != GCR_OK) return rc;
  CHK(n, hipStreamSynchronize(n->stream));
  return GCR_OK;
}

extern "C" int cnn_get_params(cnn_net* n, float* host, int64_t count) {
  if (!n || !host) return GCR_EINVAL;
  if (count != n->nparams) return cfail(n, GCR_EINVAL, "expected %lld parameters", (long long)n->nparams);
  CHK(n, hipMemcpyAsync(host, n->params, count * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  CHK(n, hipStreamSynchronize(n->stream));
  return GCR_OK;
}

static ConvArgs conv_args(const cnn_net* n, int batch) {
  ConvArgs A{};
  A.nx = n->nx;
  A.ny = n->ny;
  A.log2nx = n->log2nx;
  A.batch = batch;
  A.row_begin = 0;
  A.row_end = n->ny;
  A.pole_row = -1;
  A.nr = CONV_NR;
  return A;
}

static dim3 conv_grid(const cnn_net* n, int batch, int rows, int nr) {
  const long long waves = (long long)(n->nx / 64) * ((rows + nr - 1) / nr);
  return dim3((unsigned)((waves + WG_WAVES - 1) / WG_WAVES), batch);
}

// A over all rows; when the across-pole taps need their own weights
// (A.wpole != A.w), the interior rows and each polar row are separate launches
template <int NT, int OUT, int CIN, bool MASK>
static void launch_conv_m(const cnn_net* n, int batch, ConvArgs A, hipStream_t st) {
  if (A.wpole == A.w) {
    hipLaunchKernelGGL((k_conv<NT, OUT, CIN, MASK>), conv_grid(n, batch, n->ny, A.nr), dim3(256), 0, st, A);
    return;
  }
  if (n->ny > 2) {
    ConvArgs I = A;
    I.row_begin = 1;
    I.row_end = n->ny - 1;
    hipLaunchKernelGGL((k_conv<NT, OUT, CIN, MASK>), conv_grid(n, batch, n->ny - 2, I.nr), dim3(256), 0, st, I);
  }
  for (int pr : {0, n->ny - 1}) {
    ConvArgs P = A;
    P.row_begin = pr;
    P.row_end = pr + 1;
    P.pole_row = pr;
    hipLaunchKernelGGL((k_conv<NT, OUT, CIN, MASK>), conv_grid(n, batch, 1, P.nr), dim3(256), 0, st, P);
  }
}

// the forward layers (no mask)
template <int NT, int OUT, int CIN = CH>
static void launch_conv(const cnn_net* n, int batch, ConvArgs A, hipStream_t st) {
  launch_conv_m<NT, OUT, CIN, false>(n, batch, A, st);
}

// forward from act[0] (already packed) to y (float32 [B][npix]); `keep`:
// every activation is written (training); else the first two layers run
// fused when the input is packed 8 channels a pixel (act[1] is not written)
// and the last two run fused (act[4] is not written)
int cnn_forward_packed(cnn_net* n, int batch, float* y, hipStream_t st, const int* active, bool keep) {
  for (int l = 0; l < CNN_LAYERS; ++l) {
    ConvArgs A = conv_args(n, batch);
    A.active = active;
    A.in = n->act[l];
    A.w = n->wf + (size_t)l * TAPS * CH * CH;
    A.wpole = A.w;
    A.bias = n->bias + l * CH;
    if (l < CNN_LAYERS - 1) {
      A.out = n->act[l + 1];
      if (l == 0 && n->in_stride == 8 && !keep) {
        A.out = n->act[2];
        hipLaunchKernelGGL(k_conv12, conv_grid(n, batch, n->ny, A.nr), dim3(256), 0, st, A,
                           (const __bf16*)(n->wf + (size_t)TAPS * CH * CH), (const float*)(n->bias + CH));
        ++l;
      } else if (l == 0 && n->in_stride == 8) {
        hipLaunchKernelGGL(k_conv_in8, conv_grid(n, batch, n->ny, A.nr), dim3(256), 0, st, A);
      } else if (l == CNN_LAYERS - 2 && !keep) {   // the last two layers fused
        A.out32 = y;
        hipLaunchKernelGGL(k_conv45, conv_grid(n, batch, n->ny, A.nr), dim3(256), 0, st, A,
                           (const __bf16*)(n->wf + (size_t)(CNN_LAYERS - 1) * TAPS * CH * CH),
                           (const float*)(n->bias + (CNN_LAYERS - 1) * CH));
        break;
      } else {
        launch_conv<2, 0>(n, batch, A, st);
      }
    } else {
      A.out32 = y;
      launch_conv<1, 1>(n, batch, A, st);
    }
  }
  CHK(n, hipGetLastError());
  return GCR_OK;
}

static int check_batch(cnn_net* n, int batch) {
  if (!n) return GCR_EINVAL;
  if (batch < 1 || batch > n->max_batch) return cfail(n, GCR_EINVAL, "batch must be in [1, %d]", n->max_batch);
  return GCR_OK;
}

extern "C" int cnn_forward(cnn_net* n, int32_t batch, const float* in, float* out) {
  int rc = check_batch(n, batch);
  if (rc != GCR_OK) return rc;
  if (!in || !out) return cfail(n, GCR_EINVAL, "NULL tensor");
  const long long npix = (long long)n->nx * n->ny;
  hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((npix * batch + 255) / 256)), dim3(256), 0, n->stream, in,
                     n->act[0], n->c_in, npix, batch, n->in_stride);
  return cnn_forward_packed(n, batch, out, n->stream, nullptr, false);
}

// the forward pass of training: every activation kept for the backward pass
static int forward_keep(cnn_net* n, int batch, const float* in, float* out) {
  const long long npix = (long long)n->nx * n->ny;
  hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((npix * batch + 255) / 256)), dim3(256), 0, n->stream, in,
                     n->act[0], n->c_in, npix, batch, n->in_stride);
  return cnn_forward_packed(n, batch, out, n->stream, nullptr, true);
}

// gradients of sum(dyv * net) w.r.t. all parameters into n->grads (reference layout)
static int backward(cnn_net* n, int batch, const float* dyv) {
  const long long npix = (long long)n->nx * n->ny;
  const long long tot = npix * batch;
  hipLaunchKernelGGL(k_pack_grad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, n->stream, dyv, n->dbuf[0], tot);
  long long off[CNN_LAYERS];
  long long o = 0;
  for (int l = 0; l < CNN_LAYERS; ++l) {
    int co, ci;
    layer_shape(n->c_in, l, co, ci);
    off[l] = o;
    o += (long long)co * ci * 9 + co;
  }
  int cur = 0;
  for (int l = CNN_LAYERS - 1; l >= 0; --l) {
    // weight gradient of layer l: input act[l], gradient at its output dbuf[cur]
    WgradArgs W{};
    W.in = n->act[l];
    W.in_stride = l == 0 ? n->in_stride : CH;
    W.dpre = n->dbuf[cur];
    W.part = n->wg_part;
    W.nx = n->nx;
    W.ny = n->ny;
    W.log2nx = n->log2nx;
    W.batch = batch;
    W.chunks = n->wg_chunks;
    W.total_chunks = tot / WG_Q;
    const int waves = (int)((W.total_chunks + W.chunks - 1) / W.chunks);
    const int blocks = (waves + WG_WAVES - 1) / WG_WAVES;
    hipLaunchKernelGGL(k_wgrad, dim3(blocks), dim3(256), 0, n->stream, W);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((WG_PART + 255) / 256, WG_SEG), dim3(256), 0, n->stream,
                       (const float*)n->wg_part, waves, n->wg_seg);
    hipLaunchKernelGGL(k_wgrad_reduce2, dim3((WG_PART + 255) / 256), dim3(256), 0, n->stream, (const float*)n->wg_seg,
                       n->wg_sum);
    UnpackG U{};
    U.g = n->wg_sum;
    U.flat = n->grads + off[l];
    layer_shape(n->c_in, l, U.co, U.ci);
    hipLaunchKernelGGL(k_unpack_grad, dim3((U.co * U.ci * 9 + U.co + 255) / 256), dim3(256), 0, n->stream, U);
    if (l == 0) break;
    // gradient at the input of layer l, masked by the ReLU of layer l-1
    ConvArgs A = conv_args(n, batch);
    A.in = n->dbuf[cur];
    A.w = n->wa + (size_t)l * TAPS * CH * CH;
    A.wpole = n->wp + (size_t)l * TAPS * CH * CH;
    A.bias = nullptr;
    A.out = n->dbuf[cur ^ 1];
    A.mask = n->act[l];
    launch_conv_m<2, 0, CH, true>(n, batch, A, n->stream);
    cur ^= 1;
  }
  CHK(n, hipGetLastError());
  return GCR_OK;
}

extern "C" int cnn_gradients(cnn_net* n, int32_t batch, const float* in, const float* dy, float* grads_host) {
  int rc = check_batch(n, batch);
  if (rc != GCR_OK) return rc;
  if (!in || !dy || !grads_host) return cfail(n, GCR_EINVAL, "NULL tensor");
  if ((rc = forward_keep(n, batch, in, n->y)) != GCR_OK) return rc;
  if ((rc = backward(n, batch, dy)) != GCR_OK) return rc;
  CHK(n, hipMemcpyAsync(grads_host, n->grads, n->nparams * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  CHK(n, hipStreamSynchronize(n->stream));
  return GCR_OK;
}

extern "C" int cnn_train_step(cnn_net* n, int32_t batch, const float* in, const float* target, float lr,
                              double* loss) {
  int rc = check_batch(n, batch);
  if (rc != GCR_OK) return rc;
  if (!in || !target) return cfail(n, GCR_EINVAL, "NULL tensor");
  if (!(lr > 0.f) || !std::isfinite(lr)) return cfail(n, GCR_EINVAL, "lr must be finite and > 0");
  if ((rc = forward_keep(n, batch, in, n->y)) != GCR_OK) return rc;
  const long long tot = (long long)n->nx * n->ny * batch;
  const int lb = 256;
  hipLaunchKernelGGL(k_mse, dim3(lb), dim3(256), 0, n->stream, (const float*)n->y, target, n->dy, n->loss_part, tot);
  if ((rc = backward(n, batch, n->dy)) != GCR_OK) return rc;
  n->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)n->adam_t), c2 = 1.f - powf(b2, (float)n->adam_t);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n->nparams + 255) / 256)), dim3(256), 0, n->stream, n->params,
                     (const float*)n->grads, n->adam_m, n->adam_v, (long long)n->nparams, lr, b1, b2, 1e-8f, c1, c2);
  if ((rc = pack_weights(n)) != GCR_OK) return rc;
  if (loss) {
    CHK(n, hipMemcpyAsync(n->loss_host, n->loss_part, lb * sizeof(double), hipMemcpyDeviceToHost, n->stream));
    CHK(n, hipStreamSynchronize(n->stream));
    double s = 0.0;
    for (int i = 0; i < lb; ++i) s += n->loss_host[i];
    *loss = s / (double)tot;
  }
  return GCR_OK;
}

extern "C" const char* cnn_last_error(const cnn_net* n) { return n ? n->err.c_str() : g_cnn_error.c_str(); }
