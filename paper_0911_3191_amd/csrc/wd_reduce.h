// Deterministic FP64 reductions: each workgroup reduces its per-site
// contributions (wavefront shuffles, then a fixed-order sum over the 4 waves
// of a 256-thread block) and writes one partial per component; a finalize
// pass sums the partials of one right-hand side in a fixed order.  No float
// atomics, so results are bitwise reproducible and do not depend on how many
// right-hand sides share a launch.
#pragma once

#include <hip/hip_runtime.h>

namespace wd {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxDot = 4;  // components per partial record

// Sum v[0..N) over the block; thread 0 writes out[0..N).  Every thread of
// the block must call it (inactive sites contribute zeros).  The LDS slots
// are shared by every call with the same N in a kernel, so the trailing
// barrier keeps a following call (the next right-hand side of a multi-RHS
// launch) from overwriting them before thread 0 has read this call's sums.
template <int N>
__device__ __forceinline__ void block_sum_store(double (&v)[N], double* out) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += __shfl_down(v[k], off, 64);
  __shared__ double sm[N][kWaves];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) sm[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (int)blockDim.x >> 6;  // 1, 2 or 4 waves
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double t = sm[k][0];
      if (nw == 2) t += sm[k][1];
      if (nw == 4) t = (sm[k][0] + sm[k][1]) + (sm[k][2] + sm[k][3]);
      out[k] = t;
    }
  }
  __syncthreads();
}

// Fixed-order sum of nb partial records (stride kMaxDot) into res[0..N).
// Called by all threads of one block; the result is valid in thread 0.  Ends
// with a barrier so that a second call may reuse the LDS slots at once.
template <int N>
__device__ __forceinline__ void sum_partials(const double* part, int nb, double (&res)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) res[k] = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock)
#pragma unroll
    for (int k = 0; k < N; ++k) res[k] += part[(int64_t)i * kMaxDot + k];
  __shared__ double sm[N][kBlock];
#pragma unroll
  for (int k = 0; k < N; ++k) sm[k][threadIdx.x] = res[k];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < N; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + w];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < N; ++k) res[k] = sm[k][0];
  __syncthreads();
}

}  // namespace wd
