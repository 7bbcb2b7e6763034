// Greedy distance-k colouring on the device (Sec. 2.1, probing paragraph).
//
// The sequential greedy colouring visits vertices by ascending key
// (priority, index) and gives each the smallest colour not held by an
// earlier-visited vertex within graph distance k.  Jones-Plassmann rounds
// produce the identical colouring in parallel: in every round a still
// uncoloured vertex whose key is the smallest among the uncoloured vertices of
// its distance-k ball takes the smallest colour absent from the coloured
// vertices of that ball.  All earlier-visited vertices of the ball are then
// coloured and no later one is, which is exactly the sequential situation.
// Ball minima and colour sets are formed by k rounds of neighbour propagation
// from a snapshot, so each round is deterministic.
#include "ldq_internal.h"

namespace ldq {

#define LDQ_CW 4   // 64-bit words of the colour-set bitmask (up to 256 colours)

struct JPState {
  unsigned long long *key;     // [2][n]   key of uncoloured vertices, ~0 for coloured
  unsigned long long *mask;    // [2][n][LDQ_CW]
};

__global__ void jp_seed_kernel(const int32_t *colour, const int32_t *prio, int64_t n, unsigned long long *key,
                               unsigned long long *mask) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = colour[i];
    const unsigned long long k =
        ((unsigned long long)(uint32_t)(prio ? prio[i] : (int32_t)i) << 32) | (unsigned long long)(uint32_t)i;
    key[i] = c < 0 ? k : ~0ull;
#pragma unroll
    for (int w = 0; w < LDQ_CW; ++w) mask[i * LDQ_CW + w] = (c >= 0 && c / 64 == w) ? (1ull << (c % 64)) : 0ull;
  }
}

__global__ void jp_propagate_kernel(const int32_t *rowptr, const int32_t *colind, int64_t n,
                                    const unsigned long long *key_in, const unsigned long long *mask_in,
                                    unsigned long long *key_out, unsigned long long *mask_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    unsigned long long k = key_in[i];
    unsigned long long m[LDQ_CW];
#pragma unroll
    for (int w = 0; w < LDQ_CW; ++w) m[w] = mask_in[i * LDQ_CW + w];
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int32_t j = colind[e];
      k = min(k, key_in[j]);
#pragma unroll
      for (int w = 0; w < LDQ_CW; ++w) m[w] |= mask_in[(int64_t)j * LDQ_CW + w];
    }
    key_out[i] = k;
#pragma unroll
    for (int w = 0; w < LDQ_CW; ++w) mask_out[i * LDQ_CW + w] = m[w];
  }
}

__global__ void jp_assign_kernel(int32_t *colour, const int32_t *prio, int64_t n, const unsigned long long *kmin,
                                 const unsigned long long *mask, int *remaining, int *overflow) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (colour[i] >= 0) continue;
    const unsigned long long k =
        ((unsigned long long)(uint32_t)(prio ? prio[i] : (int32_t)i) << 32) | (unsigned long long)(uint32_t)i;
    if (kmin[i] != k) continue;
    int c = -1;
    for (int w = 0; w < LDQ_CW && c < 0; ++w) {
      const unsigned long long free = ~mask[i * LDQ_CW + w];
      if (free) c = w * 64 + __ffsll((long long)free) - 1;
    }
    if (c < 0) {
      atomicMax(overflow, 1);
      continue;
    }
    colour[i] = c;
    atomicSub(remaining, 1);
  }
}

// One Jones-Plassmann round: seed from the current colours, k propagation
// steps, assignment.  key/mask hold two ping-pong copies.
hipError_t launch_jp_round(const int32_t *rowptr, const int32_t *colind, int64_t n, int k, const int32_t *prio,
                           int32_t *colour, unsigned long long *key, unsigned long long *mask, int *remaining,
                           int *overflow, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
  unsigned long long *ka = key, *kb = key + n;
  unsigned long long *ma = mask, *mb = mask + n * LDQ_CW;
  hipLaunchKernelGGL(jp_seed_kernel, dim3(blocks), dim3(256), 0, s, colour, prio, n, ka, ma);
  for (int step = 0; step < k; ++step) {
    hipLaunchKernelGGL(jp_propagate_kernel, dim3(blocks), dim3(256), 0, s, rowptr, colind, n, ka, ma, kb, mb);
    std::swap(ka, kb);
    std::swap(ma, mb);
  }
  hipLaunchKernelGGL(jp_assign_kernel, dim3(blocks), dim3(256), 0, s, colour, prio, n, ka, ma, remaining, overflow);
  return hipGetLastError();
}

}  // namespace ldq
