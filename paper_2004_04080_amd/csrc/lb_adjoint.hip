// lb_adjoint.hip -- loss, checkpoints and the reverse-mode sweep.
//
// Loss of the differentiation study: L = sum over fluid nodes of
// |grad_lat phi|^2 with phi = psi_A - psi_B and grad_lat = 3 sum_i w_i (.) c_i.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "lb_device.hpp"
#include "lb_internal.hpp"

namespace lbh {

constexpr int ABLOCK = 256;

static inline uint32_t ablocks(uint64_t n) { return uint32_t((n + ABLOCK - 1) / ABLOCK); }

size_t adj_layout(const lb_params& p, size_t fbytes, AdjLayout& al) {
  al = AdjLayout();
  if (p.checkpoint_every <= 0) return 0;
  const size_t N = size_t(p.nx) * p.ny * p.nz;
  const size_t K = size_t(p.checkpoint_every);
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t off = 0;
  al.nckpt = int((size_t(p.max_record_steps) + K - 1) / K);
  al.ckpt = off;
  off += size_t(al.nckpt) * fbytes;
  al.seg = off;
  off += K * fbytes;
  const size_t lam = up(size_t(p.ncomp) * Q * N * sizeof(double));
  al.lam[0] = off;
  off += lam;
  al.lam[1] = off;
  off += lam;
  al.lam_a = off;
  off += up(size_t(p.ncomp) * 3 * N * sizeof(double));
  al.lam_psi = off;
  off += up(size_t(p.ncomp) * N * sizeof(double));
  al.lam_rho = off;
  off += up(size_t(p.ncomp) * N * sizeof(double));
  al.lam_j = off;
  off += up(3 * N * sizeof(double));
  al.grad = off;
  off += up(3 * N * sizeof(double));
  al.partials = off;
  off += up(size_t(RED_BLOCKS) * RED_N * sizeof(double));
  al.total = off;
  return off;
}

int record_checkpoint(lb_ctx* c) {
  const int64_t idx = c->rec_steps / c->P.checkpoint_every;
  if (idx >= c->al.nckpt) {
    c->err = "checkpoint storage exhausted";
    return LB_E_CAPACITY;
  }
  const hipError_t e = hipMemcpyAsync(aptr(c, c->al.ckpt + size_t(idx) * c->req.f), c->B.f[c->cur],
                                      c->req.f, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) {
    c->err = std::string("checkpoint copy: ") + hipGetErrorString(e);
    return LB_E_HIP;
  }
  return LB_OK;
}

// grad_lat phi on fluid nodes (0 elsewhere) and per-block partial sums of |grad|^2
template <typename real>
__global__ void __launch_bounds__(ABLOCK)
k_loss_grad(const real* __restrict__ psi, const uint16_t* __restrict__ owner, uint32_t nx,
            uint32_t ny, uint32_t nz, int ncomp, double* __restrict__ grad,
            double* __restrict__ partial) {
  const uint32_t N = nx * ny * nz;
  double acc = 0.0;
  for (uint32_t n = blockIdx.x * ABLOCK + threadIdx.x; n < N; n += gridDim.x * ABLOCK) {
    double g[3] = {0, 0, 0};
    if (!owner || owner[n] == 0) {
      uint32_t x, y, z;
      node_xyz(n, nx, ny, x, y, z);
      Nbr nb(x, y, z, nx, ny, nz);
      for (int i = 1; i < Q; ++i) {
        const uint32_t m = nb.push(i);
        const double phi = ncomp == 2 ? double(psi[m]) - double(psi[N + m]) : double(psi[m]);
        g[0] += 3.0 * WQ[i] * phi * CX[i];
        g[1] += 3.0 * WQ[i] * phi * CY[i];
        g[2] += 3.0 * WQ[i] * phi * CZ[i];
      }
      acc += g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    }
    if (grad)
      for (int d = 0; d < 3; ++d) grad[size_t(d) * N + n] = g[d];
  }
  __shared__ double sh[ABLOCK];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = ABLOCK / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(ABLOCK) k_sum_partials(const double* __restrict__ partial,
                                                         int nb, double* __restrict__ out) {
  __shared__ double sh[ABLOCK];
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += ABLOCK) a += partial[b];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = ABLOCK / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// dL/dphi(m) = sum over fluid n = m - c_i of 2 grad(n) . 3 w_i c_i
__global__ void __launch_bounds__(ABLOCK)
k_loss_seed(const double* __restrict__ grad, uint32_t nx, uint32_t ny, uint32_t nz,
            double* __restrict__ seedA, double* __restrict__ seedB) {
  const uint32_t m = blockIdx.x * ABLOCK + threadIdx.x;
  const uint32_t N = nx * ny * nz;
  if (m >= N) return;
  uint32_t x, y, z;
  node_xyz(m, nx, ny, x, y, z);
  Nbr nb(x, y, z, nx, ny, nz);
  double s = 0.0;
  for (int i = 1; i < Q; ++i) {
    const uint32_t n = nb.pull(i);
    s += 6.0 * WQ[i] * (CX[i] * grad[n] + CY[i] * grad[N + n] + CZ[i] * grad[2 * size_t(N) + n]);
  }
  if (seedA) seedA[m] = s;
  if (seedB) seedB[m] = -s;
}

hipError_t launch_loss(lb_ctx* c, double* L_dev, double* seedA, double* seedB) {
  const auto& g = c->geo;
  const uint16_t* own =
      c->has_solids ? static_cast<const uint16_t*>(c->B.owner[c->own_old]) : nullptr;
  double* grad = (seedA || seedB) ? reinterpret_cast<double*>(aptr(c, c->al.grad)) : nullptr;
  double* partial = reinterpret_cast<double*>(wptr(c, c->wl.partials));
  const int nb = int(std::min<uint64_t>(RED_BLOCKS, ablocks(g.N)));
  if (g.prec == LB_FP64)
    hipLaunchKernelGGL(k_loss_grad<double>, dim3(nb), dim3(ABLOCK), 0, c->stream,
                       static_cast<const double*>(c->B.rho), own, g.nx, g.ny, g.nz, g.ncomp, grad,
                       partial);
  else
    hipLaunchKernelGGL(k_loss_grad<float>, dim3(nb), dim3(ABLOCK), 0, c->stream,
                       static_cast<const float*>(c->B.rho), own, g.nx, g.ny, g.nz, g.ncomp, grad,
                       partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(ABLOCK), 0, c->stream, partial, nb, L_dev);
  if (grad)
    hipLaunchKernelGGL(k_loss_seed, dim3(ablocks(g.N)), dim3(ABLOCK), 0, c->stream, grad, g.nx,
                       g.ny, g.nz, seedA, g.ncomp == 2 ? seedB : nullptr);
  return hipGetLastError();
}

int backward(lb_ctx* c, const double*, const double*, double*, double*, double*) {
  c->err = "reverse mode not available";
  return LB_E_STATE;
}

}  // namespace lbh

using namespace lbh;

extern "C" {

int lb_loss(lb_ctx* c, double* L, double* dL_dpsiA, double* dL_dpsiB) {
  if (!c || !L) return LB_E_ARG;
  if ((dL_dpsiA || dL_dpsiB) && c->P.checkpoint_every <= 0) {
    c->err = "loss gradients need the adjoint buffer (checkpoint_every > 0)";
    return LB_E_STATE;
  }
  const uint16_t* own =
      c->has_solids ? static_cast<const uint16_t*>(c->B.owner[c->own_old]) : nullptr;
  hipError_t e = launch_density(c, c->B.f[c->cur]);
  if (e == hipSuccess && c->nparticles > 0) e = launch_fill_particles(c, own, false);
  if (e == hipSuccess && c->P.walls) e = launch_fill_walls(c, own);
  double* Ld = reinterpret_cast<double*>(wptr(c, c->wl.red_out));
  if (e == hipSuccess) e = launch_loss(c, Ld, dL_dpsiA, dL_dpsiB);
  if (e == hipSuccess) e = hipMemcpyAsync(L, Ld, sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->err = std::string("lb_loss: ") + hipGetErrorString(e);
    return LB_E_HIP;
  }
  return LB_OK;
}

int lb_backward(lb_ctx* c, const double* sA, const double* sB, double* dA0, double* dG,
                double dg[3]) {
  if (!c) return LB_E_ARG;
  return backward(c, sA, sB, dA0, dG, dg);
}

}  // extern "C"
