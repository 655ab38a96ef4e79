// ceilings.hip -- random-access ceilings of the device, measured by the
// benchmark beside the table kernels (a separate library, libck_ceilings.so;
// not part of the table's C ABI).
//
// Two access patterns bound the table's work:
//   * random line gathers: a lookup or a planner's bin view is one whole bin
//     line (128 bytes for 8-slot bins) at a random address;
//   * random 64-bit atomics: every bin a plan writes is claimed with one
//     atomicMin on its claim word at a random address.
// Both kernels draw their addresses in-kernel from a counter-based hash, so
// the only memory traffic is the pattern itself.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// a uniform index in [0, n) from a 64-bit draw (high word of the product)
__device__ __forceinline__ uint64_t below(uint64_t r, uint64_t n) { return __umul64hi(r, n); }

// LPL lanes per line, each loading 16 bytes: query q reads line
// below(mix64(seed ^ q), lines) whole.  Each lane folds what it read into a
// running XOR, written once per lane at the end (so the loads are live).
template <int LPL>
__global__ __launch_bounds__(256) void k_gather(const ulonglong2* __restrict__ buf,
                                                uint64_t lines, uint64_t n, uint64_t seed,
                                                uint64_t* __restrict__ out) {
  const uint32_t lane = threadIdx.x & (LPL - 1);
  const uint64_t gid = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPL;
  const uint64_t groups = (uint64_t)gridDim.x * blockDim.x / LPL;
  uint64_t acc = 0;
  for (uint64_t q = gid; q < n; q += groups) {
    const uint64_t line = below(mix64(seed ^ q), lines);
    const ulonglong2 v = buf[line * LPL + lane];
    acc ^= v.x ^ v.y;
  }
  out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// op i: atomicMin(&buf[below(mix64(seed ^ i), words)], mix64(i))
__global__ __launch_bounds__(256) void k_atomic_min(unsigned long long* __restrict__ buf,
                                                    uint64_t words, uint64_t n, uint64_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    atomicMin(&buf[below(mix64(seed ^ i), words)], (unsigned long long)mix64(i));
}

}  // namespace

extern "C" {

// Threads of the gather grid (the size of `out`, in 8-byte words).
uint64_t ckc_gather_threads() { return 256ull * 8192; }

// n random line reads of line_bytes (64 or 128) over buf[0, lines * line_bytes).
// `out` holds ckc_gather_threads() words.  Returns 0, or -1 for a bad argument.
int ckc_gather(const void* buf, uint64_t lines, uint32_t line_bytes, uint64_t n, uint64_t seed,
               uint64_t* out, void* stream) {
  if (!buf || !out || lines == 0) return -1;
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid(8192), block(256);
  if (line_bytes == 128)
    hipLaunchKernelGGL(k_gather<8>, grid, block, 0, s, (const ulonglong2*)buf, lines, n, seed,
                       out);
  else if (line_bytes == 64)
    hipLaunchKernelGGL(k_gather<4>, grid, block, 0, s, (const ulonglong2*)buf, lines, n, seed,
                       out);
  else
    return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// n random 64-bit atomicMin operations over buf[0, words).
int ckc_atomic_min(void* buf, uint64_t words, uint64_t n, uint64_t seed, void* stream) {
  if (!buf || words == 0) return -1;
  hipLaunchKernelGGL(k_atomic_min, dim3(8192), dim3(256), 0, (hipStream_t)stream,
                     (unsigned long long*)buf, words, n, seed);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
