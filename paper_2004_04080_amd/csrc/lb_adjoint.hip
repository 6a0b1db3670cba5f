// lb_adjoint.hip -- loss, checkpoints and the reverse-mode sweep.
//
// Loss of the differentiation study: L = sum over fluid nodes of
// |grad_lat phi|^2 with phi = psi_A - psi_B and grad_lat = 3 sum_i w_i (.) c_i.
//
// Reverse mode of the step on a fixed geometry (static spheres, walls at
// rest, equal relaxation times). The step (Sec. 3.1, steps 1-8) maps the
// gathered populations f(t) to f(t+1):
//   rho_k = sum_i f_ki,  u = sum_k j_k / sum_k rho_k             (Eq. rho, vel, scvel)
//   psi_k = rho_k on fluid nodes; on frontier solids the w-weighted mean of
//           the fluid neighbours (Eq. soliddens)
//   a_k   = g - G s sum_i w_i psi_kbar(n + c_i) c_i              (Eq. shanchen)
//   f*_ki = (1 - omega) f_ki + (omega - 1) E_i(rho_k, u) + E_i(rho_k, u + a_k)   (Eq. lbsbgk)
//   f_ki(n, t+1) = f*_ki(n - c_i) if n - c_i is fluid, else f*_{k,opp(i)}(n)  (Eq. bgk2, bbv)
// with E_i(rho, v) = w_i rho (1 + 3 c_i.v + 4.5 (c_i.v)^2 - 1.5 v.v); a link
// to a solid at rest reflects without correction. Its adjoint, with mu(t) the
// derivative of L with respect to the gathered populations f(t):
//   lam*_ki(n) = mu_ki(n + c_i, t+1) if n + c_i is fluid, else mu_{k,opp(i)}(n, t+1)
//   mu_ki(n, t) = (1 - omega) lam*_ki + dL/drho_k + dL/dR + dL/dJ . c_i + lam_rho_k(n)
// where the middle terms come from the moments of lam* (see k_adj_collide)
// and lam_rho_k carries the pseudo-potential paths: the transpose of the
// Shan-Chen stencil (k_adj_psi) and of the frontier fill (k_adj_rho).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
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
  const size_t mu = up(size_t(p.ncomp) * Q * N * sizeof(double));
  al.mu[0] = off;
  off += mu;
  al.mu[1] = off;
  off += mu;
  al.lam_a = off;
  off += up(size_t(p.ncomp) * 3 * N * sizeof(double));
  al.lam_psi = off;
  off += up(size_t(p.ncomp) * N * sizeof(double));
  al.winv = off;
  off += up(N * sizeof(double));
  al.grad = off;
  off += up(3 * N * sizeof(double));
  al.partials = off;
  off += up(size_t(ablocks(N)) * 4 * sizeof(double));
  al.accum = off;
  off += up(4 * sizeof(double));
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

// ---------------------------------------------------------------------------
// Reverse sweep kernels
// ---------------------------------------------------------------------------
struct AdjArgs {
  const void* fin;         // forward state: pull-form populations before the step
  const void* psi;         // pseudo-potential of that state (fill included)
  const uint16_t* owner;   // the fixed map (nullptr: no solids)
  const double* mu_next;   // mu(t+1) [NC][Q][N]
  double* mu;              // mu(t)   [NC][Q][N]  (local part; k_adj_rho adds the rest)
  double* lam_a;           // [NC][3][N]
  double* partial;         // [gridDim][4]: dL/dG, dL/dg
  uint32_t nx, ny, nz, N;
  double Gs, s;            // G * sc_norm and sc_norm
  double g[3], rho0[2], omega;
};

__device__ __forceinline__ bool is_fluid(const uint16_t* owner, uint32_t n) {
  return !owner || owner[n] == 0;
}

// Deterministic per-block sum of 4 values into partial[blockIdx.x][4].
__device__ __forceinline__ void block_sum4(double v[4], double* __restrict__ partial) {
  __shared__ double sh[4][ABLOCK];
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int st = ABLOCK / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[size_t(blockIdx.x) * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

// Collision adjoint at each fluid node: recompute the forward moments and
// accelerations from the stored state, gather lam* from mu(t+1) along the
// streaming and bounce-back paths, and apply the transposed Jacobian of
// Eq. lbsbgk. With m0 = sum_i w_i lam_i, m1 = sum_i w_i lam_i c_i and
// M2 = sum_i w_i lam_i c_i c_i:
//   sum_i lam_i w_i P_i(v)      = m0 + 3 m1.v + 4.5 v.M2.v - 1.5 (v.v) m0
//   sum_i lam_i w_i grad P_i(v) = 3 m1 + 9 M2 v - 3 m0 v
template <typename real, int NC>
__global__ void __launch_bounds__(ABLOCK) k_adj_collide(const AdjArgs a) {
  const uint32_t n = blockIdx.x * ABLOCK + threadIdx.x;
  double part[4] = {0, 0, 0, 0};
  if (n < a.N && is_fluid(a.owner, n)) {
    const uint32_t N = a.N;
    uint32_t x, y, z;
    node_xyz(n, a.nx, a.ny, x, y, z);
    Nbr nb(x, y, z, a.nx, a.ny, a.nz);
    const real* fin = static_cast<const real*>(a.fin);
    const real* psi = static_cast<const real*>(a.psi);
    // forward: moments, mixture velocity, accelerations
    double rho[NC], J[3] = {0, 0, 0}, S[NC][3];
    for (int k = 0; k < NC; ++k) {
      double sum = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double v = double(fin[(size_t(k) * Q + i) * N + nb.pull(i)]);
        sum += v;
        J[0] += v * CX[i];
        J[1] += v * CY[i];
        J[2] += v * CZ[i];
      }
      rho[k] = a.rho0[k] + sum;
      S[k][0] = S[k][1] = S[k][2] = 0.0;
      if (NC == 2) {
        const real* pk = psi + size_t(NC - 1 - k) * N;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const double p = WQ[i] * double(pk[nb.push(i)]);
          S[k][0] += p * CX[i];
          S[k][1] += p * CY[i];
          S[k][2] += p * CZ[i];
        }
      }
    }
    double R = 0.0;
    for (int k = 0; k < NC; ++k) R += rho[k];
    const double u[3] = {J[0] / R, J[1] / R, J[2] / R};
    const double om = a.omega;
    double lam_u[3] = {0, 0, 0}, A[NC], la[NC][3];
    double lam[NC][Q];
    for (int k = 0; k < NC; ++k) {
      // lam*_ki: along the streaming path, or back along the link
      lam[k][0] = a.mu_next[(size_t(k) * Q) * N + n];
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const uint32_t m = nb.push(i);
        lam[k][i] = is_fluid(a.owner, m) ? a.mu_next[(size_t(k) * Q + i) * N + m]
                                         : a.mu_next[(size_t(k) * Q + OPP[i]) * N + n];
      }
      double m0 = 0, m1[3] = {0, 0, 0}, M2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double wl = WQ[i] * lam[k][i];
        const int c[3] = {CX[i], CY[i], CZ[i]};
        m0 += wl;
        for (int d = 0; d < 3; ++d) {
          m1[d] += wl * c[d];
          for (int e = 0; e < 3; ++e) M2[d][e] += wl * c[d] * c[e];
        }
      }
      double v[3];
      for (int d = 0; d < 3; ++d) v[d] = u[d] + a.g[d] - a.Gs * S[k][d];
      auto pm = [&](const double* q) {
        double qMq = 0.0, m1q = 0.0, qq = 0.0;
        for (int d = 0; d < 3; ++d) {
          m1q += m1[d] * q[d];
          qq += q[d] * q[d];
          for (int e = 0; e < 3; ++e) qMq += q[d] * M2[d][e] * q[e];
        }
        return m0 + 3.0 * m1q + 4.5 * qMq - 1.5 * qq * m0;
      };
      A[k] = (om - 1.0) * pm(u) + pm(v);
      for (int d = 0; d < 3; ++d) {
        double M2u = 0.0, M2v = 0.0;
        for (int e = 0; e < 3; ++e) {
          M2u += M2[d][e] * u[e];
          M2v += M2[d][e] * v[e];
        }
        const double gu = 3.0 * m1[d] + 9.0 * M2u - 3.0 * m0 * u[d];
        const double gv = 3.0 * m1[d] + 9.0 * M2v - 3.0 * m0 * v[d];
        la[k][d] = rho[k] * gv;
        lam_u[d] += rho[k] * ((om - 1.0) * gu + gv);
      }
    }
    // u = J / R
    const double lam_J[3] = {lam_u[0] / R, lam_u[1] / R, lam_u[2] / R};
    const double lam_R = -(lam_u[0] * u[0] + lam_u[1] * u[1] + lam_u[2] * u[2]) / R;
    for (int k = 0; k < NC; ++k) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        a.mu[(size_t(k) * Q + i) * N + n] = (1.0 - om) * lam[k][i] + A[k] + lam_R +
                                            lam_J[0] * CX[i] + lam_J[1] * CY[i] +
                                            lam_J[2] * CZ[i];
      for (int d = 0; d < 3; ++d) {
        a.lam_a[(size_t(k) * 3 + d) * N + n] = la[k][d];
        part[0] -= a.s * S[k][d] * la[k][d];   // da_k/dG = -s S_k
        part[1 + d] += la[k][d];               // da_k/dg = identity
      }
    }
  }
  block_sum4(part, a.partial);
}

// Transpose of the Shan-Chen stencil: psi_k(m) enters a_kbar(n) of every
// fluid n = m - c_i with the coefficient -G s w_i c_i.
template <int NC>
__global__ void __launch_bounds__(ABLOCK)
k_adj_psi(const double* __restrict__ lam_a, const uint16_t* __restrict__ owner, uint32_t nx,
          uint32_t ny, uint32_t nz, double Gs, double* __restrict__ lam_psi) {
  const uint32_t m = blockIdx.x * ABLOCK + threadIdx.x;
  const uint32_t N = nx * ny * nz;
  if (m >= N) return;
  uint32_t x, y, z;
  node_xyz(m, nx, ny, x, y, z);
  Nbr nb(x, y, z, nx, ny, nz);
  for (int k = 0; k < NC; ++k) {
    const int kb = NC - 1 - k;
    double acc = 0.0;
    if (NC == 2) {
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const uint32_t n = nb.pull(i);
        if (!is_fluid(owner, n)) continue;
        acc += WQ[i] * (CX[i] * lam_a[(size_t(kb) * 3) * N + n] +
                        CY[i] * lam_a[(size_t(kb) * 3 + 1) * N + n] +
                        CZ[i] * lam_a[(size_t(kb) * 3 + 2) * N + n]);
      }
    }
    lam_psi[size_t(k) * N + m] = -Gs * acc;
  }
}

// 1 / sum of w_i over the fluid neighbours of each solid node (0 when none
// and on fluid nodes): the normalisation of the frontier fill.
__global__ void __launch_bounds__(ABLOCK)
k_adj_fill_weights(const uint16_t* __restrict__ owner, uint32_t nx, uint32_t ny, uint32_t nz,
                   double* __restrict__ winv) {
  const uint32_t s = blockIdx.x * ABLOCK + threadIdx.x;
  const uint32_t N = nx * ny * nz;
  if (s >= N) return;
  double W = 0.0;
  if (!is_fluid(owner, s)) {
    uint32_t x, y, z;
    node_xyz(s, nx, ny, x, y, z);
    Nbr nb(x, y, z, nx, ny, nz);
    for (int i = 1; i < Q; ++i)
      if (is_fluid(owner, nb.push(i))) W += WQ[i];
  }
  winv[s] = W > 0.0 ? 1.0 / W : 0.0;
}

// Pseudo-potential paths into the density of each fluid node m: its own psi,
// and the fill of every frontier solid s = m - c_j, which weighs rho(m) with
// (1 + zeta_k) w_j / W(s). The sum is added to mu_ki(m) for every i.
template <int NC>
__global__ void __launch_bounds__(ABLOCK)
k_adj_rho(const double* __restrict__ lam_psi, const uint16_t* __restrict__ owner,
          const double* __restrict__ winv, uint32_t nx, uint32_t ny, uint32_t nz, double z0,
          double z1, double* __restrict__ mu) {
  const uint32_t m = blockIdx.x * ABLOCK + threadIdx.x;
  const uint32_t N = nx * ny * nz;
  if (m >= N || !is_fluid(owner, m)) return;
  uint32_t x, y, z;
  node_xyz(m, nx, ny, x, y, z);
  Nbr nb(x, y, z, nx, ny, nz);
  for (int k = 0; k < NC; ++k) {
    double lr = lam_psi[size_t(k) * N + m];
    if (owner) {
      const double zf = 1.0 + (k == 0 ? z0 : z1);
#pragma unroll
      for (int j = 1; j < Q; ++j) {
        const uint32_t s = nb.pull(j);
        if (owner[s] != 0) lr += zf * WQ[j] * winv[s] * lam_psi[size_t(k) * N + s];
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) mu[(size_t(k) * Q + i) * N + m] += lr;
  }
}

// Deterministic sum of the step's block partials into the running totals.
__global__ void __launch_bounds__(ABLOCK)
k_adj_accum(const double* __restrict__ partial, int nb, double* __restrict__ accum) {
  __shared__ double sh[4][ABLOCK];
  double v[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += ABLOCK)
    for (int c = 0; c < 4; ++c) v[c] += partial[size_t(b) * 4 + c];
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int st = ABLOCK / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) accum[threadIdx.x] += sh[threadIdx.x][0];
}

// dL/drho_A(n, 0) = sum_i w_i mu_Ai(n, 0): the initial populations are
// f_i = E_i(rho_A0, 0) = w_i rho_A0 on fluid nodes (Eq. LEQ with u = 0).
__global__ void __launch_bounds__(ABLOCK)
k_adj_init(const double* __restrict__ mu, const uint16_t* __restrict__ owner, uint32_t N,
           double* __restrict__ out) {
  const uint32_t n = blockIdx.x * ABLOCK + threadIdx.x;
  if (n >= N) return;
  double s = 0.0;
  if (is_fluid(owner, n))
#pragma unroll
    for (int i = 0; i < Q; ++i) s += WQ[i] * mu[size_t(i) * N + n];
  out[n] = s;
}

// One forward step on a fixed geometry from fin to fout, leaving the context's
// own state and the sphere accumulators alone (reverse-sweep recomputation).
static hipError_t forward_fixed(lb_ctx* c, const void* fin, void* fout, const uint16_t* own) {
  hipError_t e = launch_density(c, fin);
  if (e == hipSuccess && c->nparticles > 0) e = launch_fill_particles(c, own, false);
  if (e == hipSuccess && c->P.walls) e = launch_fill_walls(c, own);
  if (e == hipSuccess) e = launch_collide(c, fin, fout, own, false);
  return e;
}

static hipError_t psi_of(lb_ctx* c, const void* f, const uint16_t* own) {
  hipError_t e = launch_density(c, f);
  if (e == hipSuccess && c->nparticles > 0) e = launch_fill_particles(c, own, false);
  if (e == hipSuccess && c->P.walls) e = launch_fill_walls(c, own);
  return e;
}

template <int NC>
static hipError_t adj_rho(lb_ctx* c, const uint16_t* own, double* mu) {
  const auto& g = c->geo;
  const double z1 = NC == 2 ? c->P.zeta[1] : 0.0;
  hipLaunchKernelGGL(k_adj_rho<NC>, dim3(ablocks(g.N)), dim3(ABLOCK), 0, c->stream,
                     reinterpret_cast<const double*>(aptr(c, c->al.lam_psi)), own,
                     reinterpret_cast<const double*>(aptr(c, c->al.winv)), g.nx, g.ny, g.nz,
                     c->P.zeta[0], z1, mu);
  return hipGetLastError();
}

template <typename real, int NC>
static hipError_t adj_step(lb_ctx* c, const void* fin, const uint16_t* own, const double* mu_next,
                           double* mu) {
  const auto& g = c->geo;
  const auto& P = c->P;
  AdjArgs a;
  a.fin = fin;
  a.psi = c->B.rho;
  a.owner = own;
  a.mu_next = mu_next;
  a.mu = mu;
  a.lam_a = reinterpret_cast<double*>(aptr(c, c->al.lam_a));
  a.partial = reinterpret_cast<double*>(aptr(c, c->al.partials));
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.N = g.N;
  a.Gs = P.G * P.sc_norm;
  a.s = P.sc_norm;
  for (int d = 0; d < 3; ++d) a.g[d] = P.g[d];
  a.rho0[0] = P.rho0[0];
  a.rho0[1] = P.rho0[NC - 1];
  a.omega = 1.0 / P.tau[0];
  const dim3 grid(ablocks(g.N));
  hipLaunchKernelGGL((k_adj_collide<real, NC>), grid, dim3(ABLOCK), 0, c->stream, a);
  hipLaunchKernelGGL(k_adj_psi<NC>, grid, dim3(ABLOCK), 0, c->stream, a.lam_a, own, g.nx, g.ny,
                     g.nz, a.Gs, reinterpret_cast<double*>(aptr(c, c->al.lam_psi)));
  hipError_t e = adj_rho<NC>(c, own, mu);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_accum, dim3(1), dim3(ABLOCK), 0, c->stream, a.partial, int(grid.x),
                     reinterpret_cast<double*>(aptr(c, c->al.accum)));
  return hipGetLastError();
}

template <int NC>
static hipError_t adj_step_p(lb_ctx* c, const void* fin, const uint16_t* own,
                             const double* mu_next, double* mu) {
  return c->geo.prec == LB_FP64 ? adj_step<double, NC>(c, fin, own, mu_next, mu)
                                : adj_step<float, NC>(c, fin, own, mu_next, mu);
}

int backward(lb_ctx* c, const double* seedA, const double* seedB, double* dA0, double* dG,
             double* dg) {
  const auto& P = c->P;
  const auto& g = c->geo;
  if (!seedA || !dA0 || !dG || !dg) {
    c->err = "lb_backward: seedA, dL_drhoA0, dL_dG and dL_dg are required";
    return LB_E_ARG;
  }
  if (P.checkpoint_every <= 0 || c->rec_steps <= 0) {
    c->err = "lb_backward: no recorded steps (checkpoint_every > 0 and lb_step first)";
    return LB_E_STATE;
  }
  if (c->moving) {
    c->err = "lb_backward: moving spheres change the map; set particles_fixed";
    return LB_E_STATE;
  }
  if (P.walls && (P.wall_type[0] != 0 || P.wall_type[1] != 0)) {
    c->err = "lb_backward: open faces are not differentiated";
    return LB_E_STATE;
  }
  if (P.janus && c->nparticles > 0) {
    c->err = "lb_backward: Janus wetting is not differentiated";
    return LB_E_STATE;
  }
  if (g.ncomp == 2 && P.tau[0] != P.tau[1]) {
    c->err = "lb_backward: needs equal relaxation times";
    return LB_E_STATE;
  }
  if (P.walls)
    for (int d = 0; d < 3; ++d)
      if (P.wall_u_lo[d] != 0.0 || P.wall_u_hi[d] != 0.0) {
        c->err = "lb_backward: needs walls at rest";
        return LB_E_STATE;
      }
  const uint16_t* own =
      c->has_solids ? static_cast<const uint16_t*>(c->B.owner[c->own_old]) : nullptr;
  const size_t N = g.N, fb = c->req.f;
  const size_t mubytes = size_t(g.ncomp) * Q * N * sizeof(double);
  double* mu[2] = {reinterpret_cast<double*>(aptr(c, c->al.mu[0])),
                   reinterpret_cast<double*>(aptr(c, c->al.mu[1]))};
  double* lam_psi = reinterpret_cast<double*>(aptr(c, c->al.lam_psi));
  double* accum = reinterpret_cast<double*>(aptr(c, c->al.accum));
  auto fail_hip = [&](hipError_t e) {
    c->err = std::string("lb_backward: ") + hipGetErrorString(e);
    return LB_E_HIP;
  };
  hipError_t e = hipSuccess;
  for (int b = 0; b < 2 && e == hipSuccess; ++b) e = launch_zero(mu[b], mubytes, c->stream);
  if (e == hipSuccess)
    e = launch_zero(aptr(c, c->al.lam_a), size_t(g.ncomp) * 3 * N * sizeof(double), c->stream);
  if (e == hipSuccess) e = launch_zero(lam_psi, size_t(g.ncomp) * N * sizeof(double), c->stream);
  if (e == hipSuccess) e = launch_zero(accum, 4 * sizeof(double), c->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_adj_fill_weights, dim3(ablocks(N)), dim3(ABLOCK), 0, c->stream, own,
                       g.nx, g.ny, g.nz, reinterpret_cast<double*>(aptr(c, c->al.winv)));
    e = hipGetLastError();
  }
  // mu(T) from the seeds dL/dpsi(T)
  if (e == hipSuccess)
    e = hipMemcpyAsync(lam_psi, seedA, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && g.ncomp == 2 && seedB)
    e = hipMemcpyAsync(lam_psi + N, seedB, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  int cur = 0;
  if (e == hipSuccess) e = g.ncomp == 2 ? adj_rho<2>(c, own, mu[cur]) : adj_rho<1>(c, own, mu[cur]);
  if (e != hipSuccess) return fail_hip(e);

  const int64_t K = P.checkpoint_every, T = c->rec_steps;
  for (int64_t sidx = (T - 1) / K; sidx >= 0; --sidx) {
    const int64_t t0 = sidx * K, len = std::min<int64_t>(K, T - t0);
    auto seg = [&](int64_t j) { return aptr(c, c->al.seg + size_t(j) * fb); };
    e = hipMemcpyAsync(seg(0), aptr(c, c->al.ckpt + size_t(sidx) * fb), fb,
                       hipMemcpyDeviceToDevice, c->stream);
    for (int64_t j = 1; j < len && e == hipSuccess; ++j) e = forward_fixed(c, seg(j - 1), seg(j), own);
    for (int64_t j = len - 1; j >= 0 && e == hipSuccess; --j) {
      e = psi_of(c, seg(j), own);
      if (e == hipSuccess)
        e = g.ncomp == 2 ? adj_step_p<2>(c, seg(j), own, mu[cur], mu[1 - cur])
                         : adj_step_p<1>(c, seg(j), own, mu[cur], mu[1 - cur]);
      cur = 1 - cur;
    }
    if (e != hipSuccess) return fail_hip(e);
  }
  hipLaunchKernelGGL(k_adj_init, dim3(ablocks(N)), dim3(ABLOCK), 0, c->stream, mu[cur], own,
                     g.N, dA0);
  e = hipGetLastError();
  double acc[4] = {0, 0, 0, 0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(acc, accum, sizeof(acc), hipMemcpyDeviceToHost, c->stream);
  // leave the pseudo-potential of the current state as lb_step would
  if (e == hipSuccess) e = psi_of(c, c->B.f[c->cur], own);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_hip(e);
  *dG = acc[0];
  for (int d = 0; d < 3; ++d) dg[d] = acc[1 + d];
  return LB_OK;
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
