// Read-only streaming probe: the HBM ceiling the Dslash is measured against.  Each workgroup is one
// wave that reads one 32 KiB chunk with 16-byte non-temporal loads (64 lanes x 16 B = 1 KiB per load
// instruction, all 32 loads of a lane issued before the first use, as the Dslash's link stream issues
// its loads) and folds the words with XOR into one word it writes back, so no load can be dropped.
#include "device.h"
#include "launch.h"

namespace stag {

constexpr int kProbeLoads = 32;  // 16-byte loads per lane: 32 KiB per workgroup

__global__ __launch_bounds__(kWave) void k_stream_read(const u4v* buf, unsigned* sink) {
  gptr<u4v> p = as_global<u4v>(buf) + (long)blockIdx.x * kProbeLoads * kWave + threadIdx.x;
  u4v w[kProbeLoads];
#pragma unroll
  for (int j = 0; j < kProbeLoads; ++j) w[j] = __builtin_nontemporal_load(p + j * kWave);
  unsigned x = 0u;
#pragma unroll
  for (int j = 0; j < kProbeLoads; ++j) x ^= w[j].x ^ w[j].y ^ w[j].z ^ w[j].w;
  // fold the wave to lane 0 and store one word per workgroup
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x ^= __shfl_xor(x, off, kWave);
  if (threadIdx.x == 0) sink[blockIdx.x] = x;
}

long stream_read_chunk_bytes() { return (long)kProbeLoads * kWave * 16; }

hipError_t launch_stream_read(const void* buf, long bytes, unsigned* sink, hipStream_t st) {
  const long chunk = stream_read_chunk_bytes();
  if (bytes <= 0 || bytes % chunk) return hipErrorInvalidValue;
  k_stream_read<<<(unsigned)(bytes / chunk), kWave, 0, st>>>(reinterpret_cast<const u4v*>(buf), sink);
  return hipGetLastError();
}

}  // namespace stag
