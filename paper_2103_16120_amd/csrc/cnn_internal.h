// Host-side state of a learned-preconditioner network, shared by the network
// API (cnn.hip) and the solver, which runs inference on its own stream.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mpgcr.h"

struct cnn_net {
  int nx = 0, ny = 0, log2nx = 0, max_batch = 0, c_in = 0;
  int64_t nparams = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<void*> allocs;
  // parameters, reference layout (float32): per layer w [co][ci][3][3], b [co]
  float* params = nullptr;
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int adam_t = 0;
  // packed bf16 weight fragments [layer][tap][32][32]: forward, adjoint,
  // adjoint across a pole; biases [layer][32]
  __bf16* wf = nullptr;
  __bf16* wa = nullptr;
  __bf16* wp = nullptr;
  float* bias = nullptr;
  // activations [B][ny][nx][32] bf16: act[0] is the packed input, act[l] the
  // input of layer l; two buffers for gradients flowing backwards.  The packed
  // input holds in_stride channels per pixel: 8 when c_in <= 8 (the rest of
  // the 32 the first layer's MFMA takes are zero, not stored), else 32.
  __bf16* act[5] = {};
  int in_stride = 32;
  __bf16* dbuf[2] = {};
  float* y = nullptr;        // network output [B][ny][nx]
  float* dy = nullptr;       // loss gradient [B][ny][nx]
  float* wg_part = nullptr;  // per-wave weight-gradient partials
  float* wg_sum = nullptr;
  float* wg_seg = nullptr;   // segment sums of the weight-gradient partials
  int wg_chunks = 0, wg_waves_max = 0;
  double* loss_part = nullptr;
  double* loss_host = nullptr;
};

// forward pass from the packed input act[0] to `y` on stream `st`; images b
// with active[b] == 0 are skipped (active: device array [batch], or null);
// keep: write every layer's activation (the backward pass reads them)
int cnn_forward_packed(cnn_net* n, int batch, float* y, hipStream_t st, const int* active = nullptr,
                       bool keep = false);
