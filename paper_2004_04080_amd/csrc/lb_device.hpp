// lb_device.hpp -- lattice constants and device helpers of the gfx950 path.
//
// D3Q19 (Sec. 2.1 of the LBsoft paper): weights 1/3, 1/18, 1/36, c_s^2 = 1/3.
// The library's direction order groups the velocities by c_z so that the
// pull-gather of a z-plane reads the planes z+1, z and z-1 in three blocks:
//   0            rest
//   1..8         c_z =  0: +x -x +y -y (+x+y) (-x-y) (+x-y) (-x+y)
//   9..13        c_z = +1: (0,0) (+x) (-x) (+y) (-y)
//   14..18       c_z = -1: (0,0) (-x) (+x) (-y) (+y)
// so that opp(i) = i+5 for 9..13 and i-5 for 14..18.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbh {

constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 1, -1, 0, 0, 0, -1, 1, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 1, -1, -1, 1, 0, 0, 0, 1, -1, 0, 0, 0, -1, 1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 14, 15, 16, 17, 18, 9, 10, 11, 12, 13};
constexpr double W1 = 1.0 / 18.0, W2 = 1.0 / 36.0;
constexpr double WQ[Q] = {1.0 / 3.0, W1, W1, W1, W1, W2, W2, W2, W2, W1,
                          W2, W2, W2, W2, W1, W2, W2, W2, W2};

constexpr uint16_t OWN_WALL = 0xFFFF;   // owner value of a wall node
constexpr int PSTRIDE = 32;             // doubles per sphere in the state array
constexpr int ASTRIDE = 32;             // doubles per sphere in the accumulator array

// sphere state record (AoS, PSTRIDE doubles)
enum : int {
  PS_X = 0, PS_V = 3, PS_W = 6, PS_Q = 9, PS_FPREV = 13, PS_TPREV = 16,
  PS_XRA = 19,   // centre used for the map of the previous step M_{t-1}
  PS_XRB = 22,   // centre used for the map two steps back (kept in the record)
  PS_HAVEPREV = 25
};
// per-step accumulators (AoS, ASTRIDE doubles)
enum : int {
  AC_FLIQ = 0, AC_TLIQ = 3, AC_FLABS = 6, AC_FD = 8, AC_TD = 11, AC_FC = 14, AC_TC = 17,
  AC_FSC = 20, AC_TSC = 23, AC_FH = 26,
  AC_NEAR = 29   // 1 when another sphere's centre is closer than 2R + 1/2 (may share nodes)
};

// Periodic neighbour addressing of node (x, y, z): index of (x+dx, y+dy, z+dz)
// for dx, dy, dz in {-1, 0, 1}.
struct Nbr {
  uint32_t xs[3];
  uint32_t rows[3][3];  // [dy+1][dz+1] -> nx * (y' + ny * z')
  __device__ __forceinline__ Nbr(uint32_t x, uint32_t y, uint32_t z, uint32_t nx, uint32_t ny,
                                 uint32_t nz) {
    xs[0] = x == 0 ? nx - 1 : x - 1;
    xs[1] = x;
    xs[2] = x + 1 == nx ? 0 : x + 1;
    uint32_t ys[3] = {y == 0 ? ny - 1 : y - 1, y, y + 1 == ny ? 0 : y + 1};
    uint32_t zs[3] = {z == 0 ? nz - 1 : z - 1, z, z + 1 == nz ? 0 : z + 1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) rows[a][b] = nx * (ys[a] + ny * zs[b]);
  }
  // node n + c_i
  __device__ __forceinline__ uint32_t push(int i) const {
    return xs[CX[i] + 1] + rows[CY[i] + 1][CZ[i] + 1];
  }
  // node n - c_i
  __device__ __forceinline__ uint32_t pull(int i) const {
    return xs[1 - CX[i]] + rows[1 - CY[i]][1 - CZ[i]];
  }
};

// Periodic neighbour (x+cx, y+cy, z+cz) for offsets only known at run time,
// by plain arithmetic (indexing the Nbr tables with run-time offsets would
// force them out of registers).
__device__ __forceinline__ uint32_t nbr_dyn(uint32_t x, uint32_t y, uint32_t z, int cx, int cy,
                                            int cz, uint32_t nx, uint32_t ny, uint32_t nz) {
  int a = int(x) + cx, b = int(y) + cy, c = int(z) + cz;
  a = a < 0 ? a + int(nx) : (a >= int(nx) ? a - int(nx) : a);
  b = b < 0 ? b + int(ny) : (b >= int(ny) ? b - int(ny) : b);
  c = c < 0 ? c + int(nz) : (c >= int(nz) ? c - int(nz) : c);
  return uint32_t(a) + nx * (uint32_t(b) + ny * uint32_t(c));
}

// Element access base[idx] with a 32-bit index off a wave-uniform base. The
// byte offset stays 32-bit, so the access takes the scalar-base plus
// vector-offset address form with no 64-bit address arithmetic per lane.
// Callers keep every array addressed this way below 4 GiB per base.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     idx * uint32_t(sizeof(T)));
}
// Raw buffer access through a descriptor in scalar registers: the base of
// one array (uniform), its size in bytes and a 32-bit byte offset per lane.
// An offset at or past the size is out of range: the hardware drops such a
// store (gfx9 raw-buffer range check), which predicates a store without a
// branch or a change of the execution mask. kOffNone is out of range for every
// array here (a population plane holds at most 0xFFFFFFFC bytes).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
constexpr uint32_t kOffNone = 0xFFFFFFFFu;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), short(0), int(bytes), 0x00020000);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(off), 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, int(off), 0, 0);
}

template <typename T>
__device__ __forceinline__ void st32(T* base, uint32_t idx, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * uint32_t(sizeof(T))) = v;
}

// c_i . (x, y, z) for a direction known at compile time, from sign flips and
// adds only (a multiply by a zero component would not fold away in IEEE mode)
template <typename real>
__device__ __forceinline__ real cdot(int i, real x, real y, real z) {
  real s = real(0);
  bool have = false;
  if (CX[i]) { s = CX[i] > 0 ? x : -x; have = true; }
  if (CY[i]) { const real t = CY[i] > 0 ? y : -y; s = have ? s + t : t; have = true; }
  if (CZ[i]) { const real t = CZ[i] > 0 ? z : -z; s = have ? s + t : t; }
  return s;
}
// |c_i|^2 == 1: the direction has weight 1/18 (else 1/36, or 1/3 at rest)
constexpr bool axis_dir(int i) { return CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i] == 1; }

__device__ __forceinline__ void node_xyz(uint32_t n, uint32_t nx, uint32_t ny, uint32_t& x,
                                         uint32_t& y, uint32_t& z) {
  x = n % nx;
  uint32_t t = n / nx;
  y = t % ny;
  z = t / ny;
}

// Minimum image of a periodic displacement. |d| < L/2 needs no division and
// gives the same value as the general form (rint(d/L) is then zero).
__device__ __forceinline__ double min_image(double d, double L) {
  return fabs(d + d) < L ? d : d - L * rint(d / L);
}

__device__ __forceinline__ int wrap_int(int v, int L) {
  v %= L;
  return v < 0 ? v + L : v;
}

// Per-sphere sums of per-lane contributions, added with FP64 atomics into
// acc[pid * ASTRIDE + off + c], c < NV. Consecutive lanes that carry the same
// sphere id form a run (a wave covers consecutive nodes of one row, so the
// nodes of one sphere in it are mostly adjacent). A segmented inclusive scan
// over shifts 1, 2, 4, ..., which stops once no run is longer than the shift,
// leaves each run's total in its last lane; that lane issues the atomics, one
// per component. Lanes with pid < 0 contribute nothing. Every lane of the wave
// calls this.
template <int NV>
__device__ __forceinline__ void flush_runs(double* __restrict__ acc, int off, int pid,
                                           const double v[NV]) {
  const int lane = __lane_id();
  const int prev = __shfl_up(pid, 1);
  const uint64_t heads = __ballot(lane == 0 || prev != pid);
  if (!__ballot(pid >= 0)) return;
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int pos = lane - (63 - __clzll(heads & upto));  // position in the run
  double s[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) s[c] = v[c];
  for (int k = 1; k < 64; k <<= 1) {
    if (!__ballot(pid >= 0 && pos >= k)) break;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      const double t = __shfl_up(s[c], k);
      if (pos >= k) s[c] += t;
    }
  }
  const bool last = lane == 63 || (((heads >> lane) >> 1) & 1ull);
  if (pid >= 0 && last) {
    double* A = acc + size_t(pid) * ASTRIDE + off;
#pragma unroll
    for (int c = 0; c < NV; ++c) unsafeAtomicAdd(A + c, s[c]);
  }
}

}  // namespace lbh
