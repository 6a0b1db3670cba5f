// lb_probe.hip -- streaming probes: what a bandwidth-bound kernel can reach
// on this device. They are measurement tools for the roofline of the step's
// kernels, not part of the step.
//
//   kind 0  read:    every 16-byte chunk of src read once (a sum per lane is
//                    stored into the first 16 bytes of dst only when it
//                    equals -1.2345e30, which finite inputs of order one
//                    never give)
//   kind 1  write:   every 16-byte chunk of dst written once
//   kind 2  copy:    src -> dst in 16-byte chunks (one read and one write)
//   kind 3  collide: two components of 19 planes of N = nx ny nz floats; node
//                    n gathers plane i at n - c_i (D3Q19, periodic) from src
//                    and stores plane i at n in dst, as the fused step moves
//                    its populations (one read and one write per value)
//
// Workgroups are dealt to the 8 XCDs as contiguous ranges, as the step's
// streaming kernels deal them.
#include <hip/hip_runtime.h>

#include "lb_device.hpp"
#include "lb_internal.hpp"

namespace lbh {

constexpr int PRB = 256;

__device__ __forceinline__ uint32_t xcd_block(uint32_t per_xcd) {
  return (blockIdx.x % 8u) * per_xcd + blockIdx.x / 8u;
}

__global__ void __launch_bounds__(PRB)
k_probe_read(const float4* __restrict__ src, size_t n16, uint32_t per_xcd, float* __restrict__ sink) {
  const size_t t = size_t(xcd_block(per_xcd)) * PRB + threadIdx.x;
  if (t >= n16) return;
  const float4 v = src[t];
  const float s = v.x + v.y + v.z + v.w;
  if (s == -1.2345e30f) sink[threadIdx.x & 3u] = s;  // within the first chunk of dst
}

__global__ void __launch_bounds__(PRB)
k_probe_write(float4* __restrict__ dst, size_t n16, uint32_t per_xcd) {
  const size_t t = size_t(xcd_block(per_xcd)) * PRB + threadIdx.x;
  if (t >= n16) return;
  dst[t] = make_float4(float(t & 7), 1.0f, 2.0f, 3.0f);
}

__global__ void __launch_bounds__(PRB)
k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n16, uint32_t per_xcd) {
  const size_t t = size_t(xcd_block(per_xcd)) * PRB + threadIdx.x;
  if (t >= n16) return;
  dst[t] = src[t];
}

__global__ void __launch_bounds__(PRB)
k_probe_collide(const float* __restrict__ src, float* __restrict__ dst, uint32_t nx, uint32_t ny,
                uint32_t nz, uint32_t per_xcd) {
  const uint32_t n = xcd_block(per_xcd) * PRB + threadIdx.x;
  const uint32_t N = nx * ny * nz;
  if (n >= N) return;
  uint32_t x, y, z;
  node_xyz(n, nx, ny, x, y, z);
  Nbr nb(x, y, z, nx, ny, nz);
  float v[2][Q];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int i = 0; i < Q; ++i) v[k][i] = ld32(src + (size_t(k) * Q + i) * N, nb.pull(i));
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int i = 0; i < Q; ++i) st32(dst + (size_t(k) * Q + i) * N, n, v[k][i]);
}

}  // namespace lbh

using namespace lbh;

extern "C" int lb_probe_stream(int32_t kind, const void* src, void* dst, size_t bytes, int32_t nx,
                               int32_t ny, int32_t nz, int32_t reps, void* stream,
                               double* ms_per_launch) {
  if (!ms_per_launch || reps < 1 || kind < 0 || kind > 3) return LB_E_ARG;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  size_t n16 = bytes / 16;
  uint64_t N = 0;
  if (kind == 3) {
    if (nx < 1 || ny < 1 || nz < 1) return LB_E_ARG;
    N = uint64_t(nx) * ny * nz;
    // 32-bit offsets within one plane, as the step's kernels use them
    if (N * 4 > 0xFFFFFFFFull || N > 0x7FFFFFFFull) return LB_E_SHAPE;
    if (bytes < N * 2 * Q * 4) return LB_E_SHAPE;
  }
  if ((kind != 1 && !src) || !dst || (kind != 3 && n16 == 0)) return LB_E_ARG;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16) return LB_E_ARG;
  const uint64_t items = kind == 3 ? N : n16;
  const uint64_t blocks = (items + PRB - 1) / PRB;
  const uint32_t per_xcd = uint32_t((blocks + 7) / 8);
  const dim3 grid(8u * per_xcd), blk(PRB);
  float* sink = static_cast<float*>(dst);  // the read probe's sink (first 4 floats)
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LB_E_HIP;
  auto launch = [&]() {
    switch (kind) {
      case 0:
        hipLaunchKernelGGL(k_probe_read, grid, blk, 0, s, static_cast<const float4*>(src), n16,
                           per_xcd, sink);
        break;
      case 1:
        hipLaunchKernelGGL(k_probe_write, grid, blk, 0, s, static_cast<float4*>(dst), n16, per_xcd);
        break;
      case 2:
        hipLaunchKernelGGL(k_probe_copy, grid, blk, 0, s, static_cast<const float4*>(src),
                           static_cast<float4*>(dst), n16, per_xcd);
        break;
      default:
        hipLaunchKernelGGL(k_probe_collide, grid, blk, 0, s, static_cast<const float*>(src),
                           static_cast<float*>(dst), uint32_t(nx), uint32_t(ny), uint32_t(nz),
                           per_xcd);
    }
  };
  launch();  // warm-up
  hipError_t e = hipEventRecord(e0, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return LB_E_HIP;
  *ms_per_launch = double(ms) / reps;
  return LB_OK;
}
