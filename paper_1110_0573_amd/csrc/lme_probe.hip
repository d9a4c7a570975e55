// lme_probe.hip -- LDS read-bandwidth probe, the peak against which the
// resident kernels' LDS traffic is placed.
//
// Every lane of every wave reads 16 bytes per instruction (ds_read_b128),
// a wave covering 1 KiB of consecutive addresses (no bank conflicts), in a
// loop whose address changes every iteration; the values are folded with
// XOR (one cheap VALU op per dword, far below the VALU rate) and written
// once so the loads cannot be removed.  Bytes read per launch =
// grid * 1024 * iters * 16.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int kProbeEntries = 4096;  // 64 KiB of LDS per workgroup

__global__ __launch_bounds__(1024) void lds_read_probe(int iters, uint32_t *sink) {
  __shared__ uint4 buf[kProbeEntries];
  const int t = threadIdx.x;
  for (int i = t; i < kProbeEntries; i += 1024)
    buf[i] = make_uint4(i, 3 * i + 1, 5 * i + 2, 7 * i + 3);
  __syncthreads();
  uint4 acc = make_uint4(0, 0, 0, 0);
  for (int it = 0; it < iters; ++it) {
    const uint4 v = buf[(t + it * 64) & (kProbeEntries - 1)];
    acc.x ^= v.x;
    acc.y ^= v.y;
    acc.z ^= v.z;
    acc.w ^= v.w;
  }
  const uint32_t r = acc.x ^ acc.y ^ acc.z ^ acc.w;
  if (r == 0x9e3779b9u) sink[blockIdx.x] = r;   // practically never: keeps the loads
}

}  // namespace

// Launches the probe: grid workgroups of 1024 threads, iters reads of 16
// bytes per thread.  sink: device uint32 [grid] (written only by chance).
extern "C" hipError_t lme_internal_probe_lds(int grid, int iters, uint32_t *sink, hipStream_t s) {
  if (grid < 1 || iters < 1 || !sink) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lds_read_probe, dim3(grid), dim3(1024), 0, s, iters, sink);
  return hipGetLastError();
}
