// Bandwidth ceilings for the roofline of the lattice step: a streaming copy
// and the data movement of an even step without its arithmetic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "psclbm_probe.h"

namespace psclbm {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(256) k_stream_copy(const f4* __restrict__ src,
                                                     f4* __restrict__ dst, long long n) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

// Partner of array k: 0 stays, 2j-1 <-> 2j.
__host__ __device__ constexpr int partner(int k) { return k == 0 ? 0 : (k % 2 ? k + 1 : k - 1); }

template <int Q>
__global__ void __launch_bounds__(256) k_stream_swap(float* __restrict__ a, long long n) {
  const long long c = ((long long)blockIdx.x * 256 + threadIdx.x) * 2;
  if (c >= n) return;
  f2 v[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k)
    v[k] = __builtin_nontemporal_load(reinterpret_cast<const f2*>(a + k * n + c));
#pragma unroll
  for (int k = 0; k < Q; ++k)
    __builtin_nontemporal_store(v[k], reinterpret_cast<f2*>(a + partner(k) * n + c));
}

}  // namespace
}  // namespace psclbm

extern "C" {

int psclbm_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* hip_stream) {
  using namespace psclbm;
  if (!d_src || !d_dst || bytes == 0 || bytes % 16 != 0 ||
      ((uintptr_t)d_src % 16) != 0 || ((uintptr_t)d_dst % 16) != 0)
    return PSCLBM_EINVAL;
  const long long n = (long long)(bytes / 16);
  const long long blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffLL) return PSCLBM_EINVAL;
  k_stream_copy<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(hip_stream)>>>(
      static_cast<const f4*>(d_src), static_cast<f4*>(d_dst), n);
  return hip_ok(hipGetLastError());
}

int psclbm_stream_swap(float* d_a, long long n, int q, void* hip_stream) {
  using namespace psclbm;
  if (!d_a || n <= 0 || n % 2 != 0 || (q != 9 && q != 19) || ((uintptr_t)d_a % 8) != 0)
    return PSCLBM_EINVAL;
  const long long blocks = (n / 2 + 255) / 256;
  if (blocks > 0x7fffffffLL) return PSCLBM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (q == 9)
    k_stream_swap<9><<<(unsigned)blocks, 256, 0, s>>>(d_a, n);
  else
    k_stream_swap<19><<<(unsigned)blocks, 256, 0, s>>>(d_a, n);
  return hip_ok(hipGetLastError());
}

}  // extern "C"
