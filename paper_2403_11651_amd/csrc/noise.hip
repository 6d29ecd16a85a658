// Uniform quantisation noise for the training proxy y_hat = y + u (Section
// II "Encoding": the latents are optimised through a differentiable proxy of
// the quantisation).  Counter-based: Philox4x32-10 (Salmon, Moraes, Dror and
// Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011), so every
// value depends only on (seed, iteration, stream id, index) and a captured
// graph draws fresh noise on every replay by reading the iteration from the
// device step counter.
#include "common.hpp"
#include "kernels.hpp"

namespace cc {

struct Philox4 {
  uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(Philox4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   // round multipliers
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   // key increments
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t lo0 = M0 * c.v[0], hi0 = __umulhi(M0, c.v[0]);
    const uint32_t lo1 = M1 * c.v[2], hi1 = __umulhi(M1, c.v[2]);
    c = Philox4{{hi1 ^ c.v[1] ^ k0, lo1, hi0 ^ c.v[3] ^ k1, lo0}};
  }
  return c;
}

__global__ __launch_bounds__(256) void noise_kernel(float* __restrict__ u, int64_t n, uint32_t k0, uint32_t k1,
                                                    const int32_t* __restrict__ step, uint32_t stream_id) {
  const uint32_t it = step ? (uint32_t)step[0] : 0u;
  const int64_t groups = (n + 3) / 4;
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < groups; g += (int64_t)gridDim.x * 256) {
    const Philox4 w = philox4x32_10(Philox4{{(uint32_t)g, (uint32_t)((uint64_t)g >> 32), it, stream_id}}, k0, k1);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = g * 4 + e;
      if (i < n) u[i] = (float)(w.v[e] >> 8) * 0x1p-24f - 0.5f;
    }
  }
}

}  // namespace cc
