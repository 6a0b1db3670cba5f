// lb_noalloc.hip -- lb_observables_noalloc: the observables of the current
// state with their reduction scratch in a static device array, for callers
// that cannot allocate device memory.
//
// `scratch` holds the per-workgroup partial records of the fluid reduction
// (at most RED_BLOCKS of RED_N doubles), its final record and the sphere
// sums. Host code never passes the array's name to a kernel or a copy: in
// host code it is only a stand-in for the symbol. lb_init takes the array's
// device address once per device with hipGetSymbolAddress (with that device
// current) and every call uses that address. All calls on one device share
// the array; calls that overlap in time on one device race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lb_device.hpp"
#include "lb_internal.hpp"

namespace lbh {

constexpr int kSphereSums = 8;  // momentum[3], KE, rotational KE, sum |F_link|
constexpr size_t kScratchDoubles = size_t(RED_BLOCKS) * RED_N + RED_N + kSphereSums;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices] = {};

int noalloc_setup(lb_ctx* c) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    c->err = std::string("noalloc scratch: hipGetDevice: ") + hipGetErrorString(e);
    return LB_E_HIP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      c->err = std::string("noalloc scratch: hipGetSymbolAddress: ") + hipGetErrorString(e);
      return LB_E_HIP;
    }
    g_scratch[dev] = ptr;
  }
  c->noalloc_scratch = g_scratch[dev];
  return LB_OK;
}

// Sphere sums of the observables in a fixed order (one workgroup, strided
// over the spheres, then a tree): sum m v, sum m v^2 / 2, sum I w^2 / 2 and
// sum |F_link| of the last step. Every output is written, so nothing in the
// scratch needs clearing first.
constexpr int SBLOCK = 256;
__global__ void __launch_bounds__(SBLOCK)
k_sphere_sums(const double* __restrict__ ps, const double* __restrict__ acc, int np, double mass,
              double inertia, double* __restrict__ out) {
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int p = threadIdx.x; p < np; p += SBLOCK) {
    const double* S = ps + size_t(p) * PSTRIDE;
    const double vx = S[PS_V], vy = S[PS_V + 1], vz = S[PS_V + 2];
    const double wx = S[PS_W], wy = S[PS_W + 1], wz = S[PS_W + 2];
    v[0] += mass * vx;
    v[1] += mass * vy;
    v[2] += mass * vz;
    v[3] += 0.5 * mass * (vx * vx + vy * vy + vz * vz);
    v[4] += 0.5 * inertia * (wx * wx + wy * wy + wz * wz);
    v[5] += acc[size_t(p) * ASTRIDE + AC_FLABS];
  }
  __shared__ double sh[SBLOCK];
  for (int c = 0; c < 6; ++c) {
    sh[threadIdx.x] = v[c];
    __syncthreads();
    for (int s = SBLOCK / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
    __syncthreads();
  }
}

}  // namespace lbh

using namespace lbh;

extern "C" int lb_observables_noalloc(lb_ctx* c, lb_obs* o) {
  if (!c || !o) return LB_E_ARG;
  if (!c->noalloc_scratch) {
    c->err = "lb_observables_noalloc: no static scratch on this device";
    return LB_E_STATE;
  }
  const int nb = reduce_blocks(c);
  if (size_t(nb) * RED_N + RED_N + kSphereSums > kScratchDoubles) {
    c->err = "lb_observables_noalloc: the reduction needs more than its static scratch";
    return LB_E_CAPACITY;
  }
  double* part = static_cast<double*>(c->noalloc_scratch);
  double* red = part + size_t(RED_BLOCKS) * RED_N;
  double* sph = red + RED_N;
  int rc = current_psi(c);
  if (rc != LB_OK) return rc;
  hipError_t e = launch_reduce(c, part, red);
  if (e == hipSuccess && c->nparticles > 0) {
    hipLaunchKernelGGL(k_sphere_sums, dim3(1), dim3(SBLOCK), 0, c->stream, pstate(c), pacc(c),
                       c->nparticles, c->mass, c->inertia, sph);
    e = hipGetLastError();
  }
  double r[RED_N + kSphereSums] = {};
  int32_t flags[3] = {0, 0, 0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(r, red, (RED_N + (c->nparticles > 0 ? kSphereSums : 0)) * sizeof(double),
                       hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(flags, wptr(c, c->wl.flags), sizeof(flags), hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->err = std::string("lb_observables_noalloc: ") + hipGetErrorString(e);
    return LB_E_HIP;
  }
  obs_fluid(c, r, o);
  const double* s = r + RED_N;
  for (int d = 0; d < 3; ++d) o->particle_momentum[d] = s[d];
  o->particle_ke = s[3];
  o->particle_ke_rot = s[4];
  o->flink_abs = s[5];
  return obs_flags(c, r, flags, o);
}
