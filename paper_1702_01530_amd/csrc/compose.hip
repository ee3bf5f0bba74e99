// Stereo-pair building on the device: the paper's post-processing of the two
// channels for a display (Section 3, Fig. 2: e.g. an anaglyph).  Both modes
// write 8-bit RGBA:
//   red-cyan anaglyph: red from the left eye, green and blue from the right eye;
//   side by side: the left eye's image followed by the right eye's, 2W x H.
// Display encoding of a linear value x: code = floor(255 * sqrt(clamp(x * exposure, 0, 1)) + 0.5),
// every step a correctly rounded FP32 operation (no contraction), alpha 255.

#include <hip/hip_runtime.h>

#include "rt_internal.h"

namespace srt {
namespace {

__device__ inline uint32_t encode(float x, float exposure) {
  float v = __fmul_rn(x, exposure);
  v = fminf(fmaxf(v, 0.0f), 1.0f);
  const float g = __fsqrt_rn(v);
  return uint32_t(floorf(__fadd_rn(__fmul_rn(255.0f, g), 0.5f)));
}

__global__ __launch_bounds__(256) void k_compose(const float* __restrict__ left, const float* __restrict__ right,
                                                 int W, int H, int mode, float exposure, uint32_t* __restrict__ out) {
  const int64_t n = int64_t(W) * H;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < (mode == RT_COMPOSE_SIDE_BY_SIDE ? 2 * n : n);
       i += int64_t(gridDim.x) * 256) {
    uint32_t r, g, b;
    int64_t o;
    if (mode == RT_COMPOSE_ANAGLYPH_RED_CYAN) {
      r = encode(left[3 * i + 0], exposure);
      g = encode(right[3 * i + 1], exposure);
      b = encode(right[3 * i + 2], exposure);
      o = i;
    } else {
      const int64_t row = i / (2 * W), col = i % (2 * W);
      const float* src = col < W ? left : right;
      const int64_t p = row * W + (col < W ? col : col - W);
      r = encode(src[3 * p + 0], exposure);
      g = encode(src[3 * p + 1], exposure);
      b = encode(src[3 * p + 2], exposure);
      o = i;
    }
    out[o] = r | (g << 8) | (b << 16) | (255u << 24);
  }
}

}  // namespace

hipError_t compose_stereo(const float* left, const float* right, int W, int H, int mode, float exposure,
                          uint8_t* out, hipStream_t s) {
  const int64_t n = int64_t(W) * H * (mode == RT_COMPOSE_SIDE_BY_SIDE ? 2 : 1);
  const unsigned grid = unsigned(std::min<int64_t>((n + 255) / 256, 4096));
  k_compose<<<grid, 256, 0, s>>>(left, right, W, H, mode, exposure, reinterpret_cast<uint32_t*>(out));
  return hipGetLastError();
}

}  // namespace srt
