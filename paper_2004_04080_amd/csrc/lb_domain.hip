// lb_domain.hip -- average domain size of the phase field.
//
// The paper measures coarsening by L(t) = 2 pi int S(k) dk / int k S(k) dk
// (Sec. 4, Eq. Cluster_L_eq), with S(k) the structure factor of the
// order-parameter fluctuations phi' = phi - <phi>, phi = (rho_A - rho_B) /
// (rho_A + rho_B), averaged over spherical shells in Fourier space. Here:
//   1. phi on the fluid nodes (pull-gathered densities, 0 on solid nodes) and
//      block sums of phi and of the fluid count;
//   2. phi' = phi - <phi> on the fluid nodes;
//   3. a real-to-complex 3-D FFT in FP64 (rocFFT), unnormalised;
//   4. |phi'(k)|^2 / N binned into shells s = round(|k| / dk) (halves up, decided
//      in integers), dk = 2 pi / min(L),
//      s <= min(L) / 2, with the weight 2 for the modes the half spectrum
//      stands for twice; per-workgroup LDS bins, then FP64 atomics;
//   5. on the host: shell means S(s) and the ratio of the two sums.
// Wave vectors are k_d = 2 pi m_d / L_d with the integer frequencies m_d of
// the transform (|m_d| <= L_d / 2).
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "lb_device.hpp"
#include "lb_internal.hpp"

namespace lbh {

constexpr int DBLOCK = 256;
constexpr int DSHELL_BLOCKS = 2048;

struct DomainLayout {
  size_t x = 0, X = 0, partial = 0, bins = 0, counts = 0, fftwork = 0, total = 0;
  int nblocks = 0, nshell = 0;
};

static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

static DomainLayout domain_layout(const lb_ctx* c, size_t fft_work) {
  DomainLayout d;
  const auto& g = c->geo;
  const size_t N = g.N, M = size_t(g.nx / 2 + 1) * g.ny * g.nz;
  d.nblocks = int((N + DBLOCK - 1) / DBLOCK);
  d.nshell = int(std::min({g.nx, g.ny, g.nz}) / 2) + 1;
  size_t off = 0;
  d.x = off;
  off += up256(N * sizeof(double));
  d.X = off;
  off += up256(M * 2 * sizeof(double));
  d.partial = off;
  off += up256(size_t(d.nblocks) * 2 * sizeof(double));
  d.bins = off;
  off += up256(size_t(d.nshell) * sizeof(double));
  d.counts = off;
  off += up256(size_t(d.nshell) * sizeof(unsigned long long));
  d.fftwork = off;
  off += up256(fft_work);
  d.total = off;
  return d;
}

// phi on fluid nodes (0 elsewhere) and per-block sums of phi and the fluid count
template <typename real>
__global__ void __launch_bounds__(DBLOCK)
k_phi(const real* __restrict__ f, const uint16_t* __restrict__ owner, uint32_t nx, uint32_t ny,
      uint32_t nz, double r0a, double r0b, double* __restrict__ x, double* __restrict__ partial) {
  const uint32_t n = blockIdx.x * DBLOCK + threadIdx.x;
  const uint32_t N = nx * ny * nz;
  double phi = 0.0, one = 0.0;
  if (n < N && (!owner || owner[n] == 0)) {
    uint32_t xx, yy, zz;
    node_xyz(n, nx, ny, xx, yy, zz);
    Nbr nb(xx, yy, zz, nx, ny, nz);
    double s[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int i = 0; i < Q; ++i) s[k] += double(f[(size_t(k) * Q + i) * N + nb.pull(i)]);
    const double ra = r0a + s[0], rb = r0b + s[1];
    phi = (ra - rb) / (ra + rb);
    one = 1.0;
  }
  if (n < N) x[n] = phi;
  __shared__ double sh[2][DBLOCK];
  sh[0][threadIdx.x] = phi;
  sh[1][threadIdx.x] = one;
  __syncthreads();
  for (int st = DBLOCK / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * size_t(blockIdx.x)] = sh[0][0];
    partial[2 * size_t(blockIdx.x) + 1] = sh[1][0];
  }
}

// <phi> over the fluid nodes into partial[0] (one workgroup, fixed order)
__global__ void __launch_bounds__(DBLOCK) k_phi_mean(double* __restrict__ partial, int nb) {
  __shared__ double sh[2][DBLOCK];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += DBLOCK) {
    a += partial[2 * size_t(i)];
    b += partial[2 * size_t(i) + 1];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int st = DBLOCK / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[0] = sh[1][0] > 0.0 ? sh[0][0] / sh[1][0] : 0.0;
}

__global__ void __launch_bounds__(DBLOCK)
k_phi_center(double* __restrict__ x, const uint16_t* __restrict__ owner, uint32_t N,
             const double* __restrict__ mean) {
  const uint32_t n = blockIdx.x * DBLOCK + threadIdx.x;
  if (n >= N || (owner && owner[n] != 0)) return;
  x[n] -= *mean;
}

// Shell of a wave vector with integer frequencies (mx, my, mz): round-half-up
// of |k| / dk. With A = lcm(L_d) and a_d = A / L_d, |k| / dk = Lmin sqrt(q) / A
// with the integer q = sum_d (m_d a_d)^2, and the shell is the largest s >= 0
// with (2s - 1)^2 A^2 <= 4 Lmin^2 q, decided in 128-bit integers around a
// floating-point first guess (boxes of unequal sides have exact half-integral
// ratios, where floating point alone could round either way).
struct ShellGeom {
  uint64_t a[3], A, Lmin;
};
__device__ __forceinline__ int shell_of(int mx, int my, int mz, const ShellGeom& G) {
  using u128 = unsigned __int128;
  const uint64_t px = uint64_t(mx < 0 ? -mx : mx) * G.a[0];
  const uint64_t py = uint64_t(my < 0 ? -my : my) * G.a[1];
  const uint64_t pz = uint64_t(mz < 0 ? -mz : mz) * G.a[2];
  const u128 q = u128(px) * px + u128(py) * py + u128(pz) * pz;
  const u128 rhs = u128(4) * G.Lmin * G.Lmin * q;
  const u128 A2 = u128(G.A) * G.A;
  int64_t s = int64_t(floor(double(G.Lmin) * sqrt(double(q)) / double(G.A) + 0.5));
  if (s < 0) s = 0;
  if (u128(2 * s + 1) * u128(2 * s + 1) * A2 <= rhs) ++s;
  if (s > 0 && u128(2 * s - 1) * u128(2 * s - 1) * A2 > rhs) --s;
  return int(s);
}

// |X|^2 / N per shell over the half spectrum [nz][ny][nx/2 + 1]
__global__ void __launch_bounds__(DBLOCK)
k_shells(const double* __restrict__ X, uint32_t nx, uint32_t ny, uint32_t nz, int nshell,
         ShellGeom G, double invN, double* __restrict__ bins,
         unsigned long long* __restrict__ counts) {
  extern __shared__ double lds[];
  double* sb = lds;
  unsigned long long* sc = reinterpret_cast<unsigned long long*>(lds + nshell);
  for (int s = threadIdx.x; s < nshell; s += DBLOCK) {
    sb[s] = 0.0;
    sc[s] = 0ull;
  }
  __syncthreads();
  const uint32_t hx = nx / 2 + 1;
  const uint64_t M = uint64_t(hx) * ny * nz;
  for (uint64_t t = uint64_t(blockIdx.x) * DBLOCK + threadIdx.x; t < M;
       t += uint64_t(gridDim.x) * DBLOCK) {
    const uint32_t jx = uint32_t(t % hx);
    const uint64_t r = t / hx;
    const uint32_t jy = uint32_t(r % ny), jz = uint32_t(r / ny);
    const int mx = int(jx);
    const int my = jy <= ny / 2 ? int(jy) : int(jy) - int(ny);
    const int mz = jz <= nz / 2 ? int(jz) : int(jz) - int(nz);
    const int s = shell_of(mx, my, mz, G);
    if (s >= nshell) continue;
    // modes 0 < mx < nx/2 stand for mx and -mx
    const int w = (jx == 0 || 2 * jx == nx) ? 1 : 2;
    const double re = X[2 * t], im = X[2 * t + 1];
    atomicAdd(&sb[s], double(w) * (re * re + im * im) * invN);
    atomicAdd(&sc[s], (unsigned long long)w);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < nshell; s += DBLOCK) {
    if (sc[s] == 0ull) continue;
    unsafeAtomicAdd(&bins[s], sb[s]);
    atomicAdd(&counts[s], sc[s]);
  }
}

struct FftPlan {
  rocfft_plan plan = nullptr;
  rocfft_execution_info info = nullptr;
  size_t work = 0;
};

static std::once_flag g_fft_once;

static int fft_plan(lb_ctx* c, FftPlan*& out) {
  std::call_once(g_fft_once, [] { rocfft_setup(); });
  if (!c->fft) {
    auto* p = new FftPlan;
    const size_t len[3] = {c->geo.nx, c->geo.ny, c->geo.nz};
    if (rocfft_plan_create(&p->plan, rocfft_placement_notinplace,
                           rocfft_transform_type_real_forward, rocfft_precision_double, 3, len,
                           1, nullptr) != rocfft_status_success ||
        rocfft_plan_get_work_buffer_size(p->plan, &p->work) != rocfft_status_success ||
        rocfft_execution_info_create(&p->info) != rocfft_status_success) {
      if (p->plan) rocfft_plan_destroy(p->plan);
      delete p;
      c->err = "rocFFT plan creation failed";
      return LB_E_HIP;
    }
    c->fft = p;
  }
  out = static_cast<FftPlan*>(c->fft);
  return LB_OK;
}

void free_fft(lb_ctx* c) {
  if (!c->fft) return;
  auto* p = static_cast<FftPlan*>(c->fft);
  if (p->info) rocfft_execution_info_destroy(p->info);
  if (p->plan) rocfft_plan_destroy(p->plan);
  delete p;
  c->fft = nullptr;
}

}  // namespace lbh

using namespace lbh;

extern "C" {

int lb_domain_workspace(lb_ctx* c, size_t* bytes, int32_t* nshell) {
  if (!c || !bytes) return LB_E_ARG;
  if (c->geo.ncomp != 2) {
    c->err = "the domain size needs two components";
    return LB_E_STATE;
  }
  FftPlan* p = nullptr;
  const int rc = fft_plan(c, p);
  if (rc != LB_OK) return rc;
  const DomainLayout d = domain_layout(c, p->work);
  *bytes = d.total;
  if (nshell) *nshell = d.nshell;
  return LB_OK;
}

int lb_domain_size(lb_ctx* c, void* work, size_t work_bytes, double* L, double* S,
                   int32_t nshell) {
  if (!c || !work || !L) return LB_E_ARG;
  size_t need = 0;
  int32_t ns = 0;
  int rc = lb_domain_workspace(c, &need, &ns);
  if (rc != LB_OK) return rc;
  if (work_bytes < need) {
    c->err = "domain-size workspace too small (see lb_domain_workspace)";
    return LB_E_ARG;
  }
  if (S && nshell < ns) {
    c->err = "shell array shorter than the shell count";
    return LB_E_ARG;
  }
  FftPlan* p = nullptr;
  fft_plan(c, p);
  const DomainLayout d = domain_layout(c, p->work);
  const auto& g = c->geo;
  char* w = static_cast<char*>(work);
  double* x = reinterpret_cast<double*>(w + d.x);
  double* X = reinterpret_cast<double*>(w + d.X);
  double* partial = reinterpret_cast<double*>(w + d.partial);
  double* bins = reinterpret_cast<double*>(w + d.bins);
  auto* counts = reinterpret_cast<unsigned long long*>(w + d.counts);
  const uint16_t* own =
      c->has_solids ? static_cast<const uint16_t*>(c->B.owner[c->own_old]) : nullptr;
  hipStream_t s = c->stream;
  const dim3 grid(d.nblocks), blk(DBLOCK);
  if (g.prec == LB_FP64)
    hipLaunchKernelGGL(k_phi<double>, grid, blk, 0, s, static_cast<const double*>(c->B.f[c->cur]),
                       own, g.nx, g.ny, g.nz, c->P.rho0[0], c->P.rho0[1], x, partial);
  else
    hipLaunchKernelGGL(k_phi<float>, grid, blk, 0, s, static_cast<const float*>(c->B.f[c->cur]),
                       own, g.nx, g.ny, g.nz, c->P.rho0[0], c->P.rho0[1], x, partial);
  hipLaunchKernelGGL(k_phi_mean, dim3(1), blk, 0, s, partial, d.nblocks);
  hipLaunchKernelGGL(k_phi_center, grid, blk, 0, s, x, own, g.N, partial);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_zero(bins, size_t(d.nshell) * sizeof(double), s);
  if (e == hipSuccess)
    e = launch_zero(counts, size_t(d.nshell) * sizeof(unsigned long long), s);
  if (e != hipSuccess) {
    c->err = std::string("lb_domain_size: ") + hipGetErrorString(e);
    return LB_E_HIP;
  }
  void* in[1] = {x};
  void* outb[1] = {X};
  if (rocfft_execution_info_set_stream(p->info, s) != rocfft_status_success ||
      (p->work && rocfft_execution_info_set_work_buffer(p->info, w + d.fftwork, p->work) !=
                      rocfft_status_success) ||
      rocfft_execute(p->plan, in, outb, p->info) != rocfft_status_success) {
    c->err = "rocFFT execution failed";
    return LB_E_HIP;
  }
  const double dk = 2.0 * M_PI / double(std::min({g.nx, g.ny, g.nz}));
  const size_t lds = size_t(d.nshell) * (sizeof(double) + sizeof(unsigned long long));
  ShellGeom G;
  G.A = std::lcm(std::lcm(uint64_t(g.nx), uint64_t(g.ny)), uint64_t(g.nz));
  G.a[0] = G.A / g.nx;
  G.a[1] = G.A / g.ny;
  G.a[2] = G.A / g.nz;
  G.Lmin = std::min({g.nx, g.ny, g.nz});
  hipLaunchKernelGGL(k_shells, dim3(DSHELL_BLOCKS), blk, lds, s, X, g.nx, g.ny, g.nz, d.nshell,
                     G, 1.0 / double(g.N), bins, counts);
  std::vector<double> hb(d.nshell);
  std::vector<unsigned long long> hc(d.nshell);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(hb.data(), bins, hb.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hc.data(), counts, hc.size() * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    c->err = std::string("lb_domain_size: ") + hipGetErrorString(e);
    return LB_E_HIP;
  }
  double num = 0.0, den = 0.0;
  for (int k = 0; k < d.nshell; ++k) {
    const double mean = hc[k] ? hb[k] / double(hc[k]) : 0.0;
    if (S) S[k] = mean;
    if (k >= 1 && hc[k]) {
      num += mean;
      den += double(k) * dk * mean;
    }
  }
  *L = den > 0.0 ? 2.0 * M_PI * num / den : NAN;
  return LB_OK;
}

}  // extern "C"
