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
//   kind 4  march:   the same planes moved as a step would move them if it
//                    also took the moments in its own sweep: a workgroup owns
//                    a column of FTX x FTY nodes and walks FZC z-planes. For
//                    plane z+1 it gathers the column's 2 x 19 pulled values
//                    and those of a one-node ring around the column, keeps the
//                    column's values in registers and puts the per-component
//                    sums s_k (the moments) into a ring of three planes in
//                    LDS; then it stores plane z as
//                      dst_{k,i}(n) = g_{k,i}(n) + 1e-3 sum_{j=1..18} j s_{1-k}(n + c_j)
//                    with g the gathered values of kind 3, so that each store
//                    waits for the sums of all 18 neighbours, as the
//                    Shan-Chen force does. nx must be a multiple of FTX and ny
//                    of FTY.
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

constexpr int FTX = 128, FTY = 8, FZC = 128;  // the fastest of the shapes tried at 512^3

__global__ void __launch_bounds__(FTX * FTY)
k_probe_march(const float* __restrict__ src, float* __restrict__ dst, uint32_t nx, uint32_t ny,
              uint32_t nz) {
  constexpr int NT = FTX * FTY, HX = FTX + 2, HY = FTY + 2, HN = HX * HY, NH = HN - NT;
  static_assert(NH <= NT, "one ring node per thread at most");
  __shared__ float sums[3][2][HN];
  const int t = int(threadIdx.x), tx = t % FTX, ty = t / FTX;
  const uint32_t ntx = nx / FTX, nty = ny / FTY;
  const uint32_t tile = blockIdx.x % (ntx * nty), chunk = blockIdx.x / (ntx * nty);
  const uint32_t x0 = (tile % ntx) * FTX, y0 = (tile / ntx) * FTY;
  const int z0 = int(chunk) * FZC, z1 = min(z0 + FZC, int(nz));
  const uint32_t N = nx * ny * nz;
  // the ring node of this thread, if any: frame rows 0 and HY-1, then columns 0 and HX-1
  int hx = 0, hy = 0;
  if (t < HX) {
    hx = t;
  } else if (t < 2 * HX) {
    hx = t - HX;
    hy = HY - 1;
  } else if (t < 2 * HX + FTY) {
    hy = t - 2 * HX + 1;
  } else {
    hx = HX - 1;
    hy = t - 2 * HX - FTY + 1;
  }
  const uint32_t gx = x0 + uint32_t(tx), gy = y0 + uint32_t(ty);
  const uint32_t rx = (x0 + nx + uint32_t(hx) - 1u) % nx, ry = (y0 + ny + uint32_t(hy) - 1u) % ny;
  float held[2][Q], cur[2][Q];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int i = 0; i < Q; ++i) held[k][i] = 0.0f;
  // trip counts are uniform over the workgroup: every thread reaches the barriers
  for (int z = z0 - 2; z < z1; ++z) {
    const uint32_t zn = uint32_t((z + 1 + 2 * int(nz)) % int(nz));  // plane z+1, periodic
    const int slot = (z + 1 + 3) % 3;                               // z + 1 >= -1
    {
      const Nbr nb(gx, gy, zn, nx, ny, nz);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          cur[k][i] = ld32(src + (size_t(k) * Q + i) * N, nb.pull(i));
          s += cur[k][i];
        }
        sums[slot][k][(ty + 1) * HX + tx + 1] = s;
      }
    }
    if (t < NH) {
      const Nbr nb(rx, ry, zn, nx, ny, nz);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < Q; ++i) s += ld32(src + (size_t(k) * Q + i) * N, nb.pull(i));
        sums[slot][k][hy * HX + hx] = s;
      }
    }
    __syncthreads();
    if (z >= z0) {
      const uint32_t n = gx + nx * (gy + ny * uint32_t(z));
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        float s = 0.0f;
#pragma unroll
        for (int j = 1; j < Q; ++j)
          s += float(j) * sums[(z + CZ[j] + 3) % 3][1 - k][(ty + 1 + CY[j]) * HX + tx + 1 + CX[j]];
#pragma unroll
        for (int i = 0; i < Q; ++i) st32(dst + (size_t(k) * Q + i) * N, n, held[k][i] + 1e-3f * s);
      }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int i = 0; i < Q; ++i) held[k][i] = cur[k][i];
    __syncthreads();
  }
}

}  // namespace lbh

using namespace lbh;

extern "C" int lb_probe_stream(int32_t kind, const void* src, void* dst, size_t bytes, int32_t nx,
                               int32_t ny, int32_t nz, int32_t reps, void* stream,
                               double* ms_per_launch) {
  if (!ms_per_launch || reps < 1 || kind < 0 || kind > 4) return LB_E_ARG;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  size_t n16 = bytes / 16;
  uint64_t N = 0;
  const bool planes = kind >= 3;
  if (planes) {
    if (nx < 1 || ny < 1 || nz < 1) return LB_E_ARG;
    N = uint64_t(nx) * ny * nz;
    // 32-bit offsets within one plane, as the step's kernels use them
    if (N * 4 > 0xFFFFFFFFull || N > 0x7FFFFFFFull) return LB_E_SHAPE;
    if (bytes < N * 2 * Q * 4) return LB_E_SHAPE;
    if (kind == 4 && (nx % FTX != 0 || ny % FTY != 0)) return LB_E_SHAPE;
  }
  if ((kind != 1 && !src) || !dst || (!planes && n16 == 0)) return LB_E_ARG;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16) return LB_E_ARG;
  const uint64_t items = planes ? N : n16;
  const uint64_t blocks = (items + PRB - 1) / PRB;
  const uint32_t per_xcd = uint32_t((blocks + 7) / 8);
  const dim3 grid(8u * per_xcd), blk(PRB);
  // kind 4: one workgroup per column tile and chunk of planes
  const uint32_t mblocks = kind == 4 ? uint32_t(nx / FTX) * uint32_t(ny / FTY) *
                                           uint32_t((nz + FZC - 1) / FZC)
                                     : 0u;
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
      case 3:
        hipLaunchKernelGGL(k_probe_collide, grid, blk, 0, s, static_cast<const float*>(src),
                           static_cast<float*>(dst), uint32_t(nx), uint32_t(ny), uint32_t(nz),
                           per_xcd);
        break;
      default:
        hipLaunchKernelGGL(k_probe_march, dim3(mblocks), dim3(FTX * FTY), 0, s,
                           static_cast<const float*>(src), static_cast<float*>(dst), uint32_t(nx),
                           uint32_t(ny), uint32_t(nz));
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
