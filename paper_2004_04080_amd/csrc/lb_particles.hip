// lb_particles.hip -- sphere kernels of the gfx950 path (FP64 throughout).
//
// Map maintenance uses two owner maps in ping-pong: at step t the "old" map
// holds M_{t-1} = raster(x(t-1)) and the "new" one, cleared, is rasterised
// at x(t). One workgroup per sphere then walks its box and lists the frontier
// nodes and the node events of the step; the fill and event kernels run over
// those lists, one thread per entry. Per-sphere sums (destroyed and created
// nodes, frontier Shan-Chen force) are wave-level sums over runs of lanes of
// one sphere, added with FP64 atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lb_device.hpp"
#include "lb_internal.hpp"

namespace lbh {

constexpr int PBLOCK = 256;

struct Box {
  int lo[3], n[3];
  int total;
};

// Node box covering every node within R of a centre (Sec. 2.4 staircase sphere).
// A non-finite centre (a diverged run) gives an empty box.
__device__ __forceinline__ Box sphere_box(const double c[3], double R) {
  Box b;
  b.total = 1;
  for (int a = 0; a < 3; ++a) {
    if (!isfinite(c[a]) || fabs(c[a]) > 1e7) {
      b.total = 0;
      b.lo[a] = 0;
      b.n[a] = 0;
      continue;
    }
    b.lo[a] = int(floor(c[a] - R));
    b.n[a] = int(ceil(c[a] + R)) - b.lo[a] + 1;
    b.total *= b.n[a];
  }
  return b;
}

// Visit every node (x, y, z) of box b with the workgroup laid out as 16 x 16
// threads over (x, y), every thread walking all z: no divisions in the walk.
template <typename F>
__device__ __forceinline__ void for_box(const Box& b, F&& f) {
  static_assert(PBLOCK == 256, "16 x 16 thread layout");
  const int tx = int(threadIdx.x & 15u), ty = int(threadIdx.x >> 4);
  for (int k = 0; k < b.n[2]; ++k)
    for (int j = ty; j < b.n[1]; j += 16)
      for (int i = tx; i < b.n[0]; i += 16) f(b.lo[0] + i, b.lo[1] + j, b.lo[2] + k);
}

// periodic image in [0, L); box coordinates stray from [0, L) by at most R + 1
__device__ __forceinline__ int wrap_box(int v, int L) {
  return unsigned(v) < unsigned(L) ? v : (v < 0 && v >= -L ? v + L : (v >= L && v < 2 * L ? v - L : wrap_int(v, L)));
}

struct PArgs {
  uint16_t* own_new;
  const uint16_t* own_old;
  double* ps;
  double* acc;
  int32_t* flags;
  void* fin;         // post-collision populations of the previous step
  void* psi;
  int nx, ny, nz;
  uint32_t N;
  double L[3], invL[3];
  double R;
  double rho0[2];
  double zeta[2];
  double rho_fb[2];
  double Gs;
  int ncomp;
  int walls;
  int np;
  int janus;
  double janus_theta0, janus_width, janus_zeta[2];
};

// A list of nodes built per sphere: entries (node, payload), the count
// appended so far (cleared before each build) and the capacity.
struct NodeList {
  uint2* list;
  int32_t* count;
  uint32_t cap;
};

// LDS staging of list entries: a workgroup moves its entries to the list in
// blocks, so that the shared counter takes one atomic per block of entries.
template <int CAP>
struct Stage {
  uint2 e[CAP];
  int staged, base;
};

template <int CAP>
__device__ void stage_flush(Stage<CAP>& st, const NodeList& L) {
  if (threadIdx.x == 0) st.base = atomicAdd(L.count, st.staged);
  __syncthreads();
  for (int t = int(threadIdx.x); t < st.staged; t += PBLOCK)
    if (uint32_t(st.base + t) < L.cap) L.list[st.base + t] = st.e[t];
  __syncthreads();
  if (threadIdx.x == 0) st.staged = 0;
}

// the lanes with `put` append v, one LDS atomic per wave
template <int CAP>
__device__ __forceinline__ void stage_push(Stage<CAP>& st, bool put, uint2 v) {
  const uint64_t has = __ballot(put);
  if (!has) return;
  const int lane = __lane_id();
  int w = 0;
  if (lane == 0) w = atomicAdd(&st.staged, int(__popcll(has)));
  w = __shfl(w, 0);
  if (put) st.e[w + int(__popcll(has & ((1ull << lane) - 1ull)))] = v;
}

// walls + empty fluid
__global__ void k_map_reset(uint16_t* own, uint32_t nx, uint32_t ny, uint32_t nz, int walls) {
  const uint32_t n = blockIdx.x * PBLOCK + threadIdx.x;
  if (n >= nx * ny * nz) return;
  const uint32_t z = n / (nx * ny);
  own[n] = (walls && (z == 0 || z == nz - 1)) ? OWN_WALL : 0;
}

// wall planes z = 0 and z = nz - 1 of a cleared map
__global__ void k_wall_planes(uint16_t* own, uint32_t nx, uint32_t ny, uint32_t nz) {
  const uint32_t plane = nx * ny;
  const uint32_t t = blockIdx.x * PBLOCK + threadIdx.x;
  if (t >= 2 * plane) return;
  own[t < plane ? t : size_t(nz - 1) * plane + (t - plane)] = OWN_WALL;
}

// Lowest sphere index wins a node claimed by several spheres; walls stay walls.
__device__ __forceinline__ void claim(uint16_t* own, uint32_t n, uint16_t val) {
  uint32_t* word = reinterpret_cast<uint32_t*>(reinterpret_cast<uintptr_t>(own + n) & ~uintptr_t(3));
  const int shift = (reinterpret_cast<uintptr_t>(own + n) & 2) ? 16 : 0;
  uint32_t old = *word, assumed;
  do {
    assumed = old;
    const uint16_t cur = uint16_t((assumed >> shift) & 0xFFFFu);
    if (cur == OWN_WALL || (cur != 0 && cur <= val)) return;
    const uint32_t nw = (assumed & ~(0xFFFFu << shift)) | (uint32_t(val) << shift);
    old = atomicCAS(word, assumed, nw);
  } while (old != assumed);
}

// Staircase sphere: node n belongs to p when |minimg(r_n - x_p)|^2 < R^2.
// With near_flags, a sphere with no other centre within 2R + 1/2 (AC_NEAR,
// from k_pairs) shares no node with another sphere and writes its nodes with
// plain stores into the cleared map; the others claim theirs atomically.
__global__ void __launch_bounds__(PBLOCK) k_raster(PArgs a, int which, int near_flags) {
  const int p = blockIdx.x;
  const double* P = a.ps + size_t(p) * PSTRIDE;
  const double c[3] = {P[which], P[which + 1], P[which + 2]};
  const Box b = sphere_box(c, a.R);
  const double R2 = a.R * a.R;
  const bool alone = near_flags && a.acc[size_t(p) * ASTRIDE + AC_NEAR] == 0.0;
  if (which == PS_X && threadIdx.x == 0 && a.flags) {
    // speed limit of the moving-boundary scheme: at most half a node per step
    const double vmax = fmax(fabs(P[PS_V]), fmax(fabs(P[PS_V + 1]), fabs(P[PS_V + 2])));
    if (!(vmax <= 0.5)) atomicOr(a.flags, 1);
  }
  for_box(b, [&](int x, int y, int z) {
    const int wx = wrap_box(x, a.nx), wy = wrap_box(y, a.ny), wz = wrap_box(z, a.nz);
    if (a.walls && (wz == 0 || wz == a.nz - 1)) return;
    const double dx = min_image(wx - c[0], a.L[0]);
    const double dy = min_image(wy - c[1], a.L[1]);
    const double dz = min_image(wz - c[2], a.L[2]);
    if (dx * dx + dy * dy + dz * dz < R2) {
      const uint32_t n = uint32_t(wx) + a.nx * (uint32_t(wy) + a.ny * uint32_t(wz));
      if (alone) a.own_new[n] = uint16_t(p + 1);
      else claim(a.own_new, n, uint16_t(p + 1));
    }
  });
}

// Fluid-node destruction (Eq. distr) and creation (Eq. creat) between the map
// of the current populations (own_old) and the new map (own_new), one thread
// per entry of the event list. A destroyed node hands its bare momentum
// sum_k j_k to its new sphere; a created node gets f_eq(rho_bar_k, u_w) in
// the slots it gathers from, with rho_bar the w-weighted mean over the
// neighbours fluid in both maps, and the sphere it left loses the momentum
// sum_k rho_bar_k u_w. Both are summed per sphere into F_d, T_d, F_c, T_c
// (wave-segmented sums, then FP64 atomics; the accumulators are cleared at
// the start of the step).
//
// One node event: node n destroyed (fluid -> sphere `sphere`) or created
// (sphere `sphere` -> fluid); its momentum terms go to v (for sphere pid).
template <typename real, int NC>
__device__ __forceinline__ void event_one(const PArgs& a, uint32_t n, bool destroyed, int sphere,
                                          int& pid, double v[12]) {
  pid = sphere;
  const double* P = a.ps + size_t(pid) * PSTRIDE;
  uint32_t x, y, z;
  node_xyz(n, uint32_t(a.nx), uint32_t(a.ny), x, y, z);
  Nbr nb(x, y, z, uint32_t(a.nx), uint32_t(a.ny), uint32_t(a.nz));
  const double d[3] = {min_image(double(x) - P[PS_X], a.L[0]),
                       min_image(double(y) - P[PS_X + 1], a.L[1]),
                       min_image(double(z) - P[PS_X + 2], a.L[2])};
  real* fin = static_cast<real*>(a.fin);
  real* psi = static_cast<real*>(a.psi);
  const uint32_t N = a.N;
  if (destroyed) {
    double J[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double fv = double(fin[(size_t(k) * Q + i) * N + nb.pull(i)]);
        J[0] += fv * CX[i];
        J[1] += fv * CY[i];
        J[2] += fv * CZ[i];
      }
    v[0] = J[0];
    v[1] = J[1];
    v[2] = J[2];
    v[3] = d[1] * J[2] - d[2] * J[1];
    v[4] = d[2] * J[0] - d[0] * J[2];
    v[5] = d[0] * J[1] - d[1] * J[0];
  } else {
    const double wx_ = P[PS_W], wy_ = P[PS_W + 1], wz_ = P[PS_W + 2];
    const double uw[3] = {P[PS_V] + (wy_ * d[2] - wz_ * d[1]),
                          P[PS_V + 1] + (wz_ * d[0] - wx_ * d[2]),
                          P[PS_V + 2] + (wx_ * d[1] - wy_ * d[0])};
    double wsum = 0.0, s[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) s[k] = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const uint32_t m = nb.push(i);
      if (a.own_old[m] != 0 || a.own_new[m] != 0) continue;
      wsum += WQ[i];
#pragma unroll
      for (int k = 0; k < NC; ++k) s[k] += WQ[i] * double(psi[size_t(k) * N + m]);
    }
    const double uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      // deviation of the created density from rho0_k
      const double dr = wsum > 0.0 ? s[k] / wsum : a.rho_fb[k] - a.rho0[k];
      const double rb = a.rho0[k] + dr;
      tot += rb;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double cu = CX[i] * uw[0] + CY[i] * uw[1] + CZ[i] * uw[2];
        fin[(size_t(k) * Q + i) * N + nb.pull(i)] =
            real(WQ[i] * dr + WQ[i] * rb * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
      }
      psi[size_t(k) * N + n] = real(dr);
    }
    const double M[3] = {tot * uw[0], tot * uw[1], tot * uw[2]};
    v[6] = -M[0];
    v[7] = -M[1];
    v[8] = -M[2];
    v[9] = -(d[1] * M[2] - d[2] * M[1]);
    v[10] = -(d[2] * M[0] - d[0] * M[2]);
    v[11] = -(d[0] * M[1] - d[1] * M[0]);
  }
}

template <typename real, int NC>
__global__ void __launch_bounds__(PBLOCK) k_events_list(PArgs a, NodeList ev) {
  const uint32_t total = min(uint32_t(*ev.count), ev.cap);
  if (blockIdx.x == 0 && threadIdx.x == 0 && uint32_t(*ev.count) > ev.cap && a.flags)
    atomicOr(a.flags + 2, 1);  // list overflow (the capacity bound rules it out)
  const uint32_t nwaves = gridDim.x * (PBLOCK / 64);
  // whole waves step together through the list: flush_runs needs every lane
  for (uint32_t base = (blockIdx.x * PBLOCK + threadIdx.x) / 64 * 64; base < total;
       base += nwaves * 64) {
    const uint32_t e = base + __lane_id();
    int pid = -1;
    double v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = 0.0;
    if (e < total) {
      const uint2 en = ev.list[e];
      event_one<real, NC>(a, en.x, (en.y >> 31) != 0u, int(en.y & 0xFFFFu) - 1, pid, v);
    }
    flush_runs<12>(a.acc, AC_FD, pid, v);
  }
}

// Direction sets as bit masks over the 18 moving directions: axis and
// diagonal directions, and per axis those with c = +1 / -1 in each class.
constexpr uint32_t dir_set(int axis, int sign, int cls) {
  uint32_t m = 0;
  for (int i = 1; i < Q; ++i) {
    const int c = axis == 0 ? CX[i] : (axis == 1 ? CY[i] : CZ[i]);
    const bool ax = axis_dir(i);
    if ((sign == 0 || c == sign) && ((cls == 1) == ax)) m |= 1u << i;
  }
  return m;
}
constexpr uint32_t kAxisDirs = dir_set(0, 0, 1), kDiagDirs = dir_set(0, 0, 2);
constexpr uint32_t kPos1[3] = {dir_set(0, 1, 1), dir_set(1, 1, 1), dir_set(2, 1, 1)};
constexpr uint32_t kNeg1[3] = {dir_set(0, -1, 1), dir_set(1, -1, 1), dir_set(2, -1, 1)};
constexpr uint32_t kPos2[3] = {dir_set(0, 1, 2), dir_set(1, 1, 2), dir_set(2, 1, 2)};
constexpr uint32_t kNeg2[3] = {dir_set(0, -1, 2), dir_set(1, -1, 2), dir_set(2, -1, 2)};

// Lists of a sphere map, one workgroup per sphere over its box:
// * frontier: every node of the sphere with at least one fluid neighbour, as
//   (node, mask of the directions i with n + c_i fluid);
// * with ev.list set, the node events of the step from own_old to own_new:
//   (node, sphere + 1, bit 31 set for a destroyed node). A destroyed node is
//   listed by the sphere that takes it, a created one by the sphere that
//   leaves it; the box then also covers the sphere's previous centre (PS_XRA),
//   up to 4 nodes away (a sphere that moved further has raised the speed flag).
// The map holds sphere p around the centre at offset `which` of its record.
// Entries of one sphere sit together in each list. Along an axis shorter than
// the box, one period of the box is walked, so that no node is listed twice.
// CAP64: at most 64 registers (eight waves per SIMD). In FP64 the kernel
// runs beside a moments pass whose waves hold 64 registers each, and a wave
// of its own must fit in what one of them frees (side stream 9.2 -> 6.5 ms
// at 512^3 with 32,000 spheres); beside the FP32 pass it runs faster with
// the compiler's own register count (3.8 against 5.2 ms capped).
template <bool CAP64>
__global__ void __launch_bounds__(PBLOCK, CAP64 ? 8 : 1) k_sphere_lists(PArgs a, NodeList fl,
                                                                       NodeList ev, int which) {
  __shared__ Stage<1024> sf;
  __shared__ Stage<512> se;
  const bool events = ev.list != nullptr;
  const int p = blockIdx.x;
  const double* P = a.ps + size_t(p) * PSTRIDE;
  const double c[3] = {P[which], P[which + 1], P[which + 2]};
  Box b = sphere_box(c, a.R);
  if (events && b.total > 0) {
    const int L[3] = {a.nx, a.ny, a.nz};
    for (int d = 0; d < 3; ++d) {
      double dd = min_image(P[PS_XRA + d] - c[d], double(L[d]));
      dd = isfinite(dd) ? fmin(4.0, fmax(-4.0, dd)) : 0.0;
      const int lo = int(floor(c[d] + dd - a.R)), hi = int(ceil(c[d] + dd + a.R));
      const int nlo = min(b.lo[d], lo), nhi = max(b.lo[d] + b.n[d] - 1, hi);
      b.lo[d] = nlo;
      b.n[d] = nhi - nlo + 1;
    }
  }
  const int nb0 = min(b.n[0], a.nx), nb1 = min(b.n[1], a.ny), nb2 = min(b.n[2], a.nz);
  const uint16_t me = uint16_t(p + 1);
  const int tx = int(threadIdx.x & 15u), ty = int(threadIdx.x >> 4);
  const double deep2 = a.R > 1.5 ? (a.R - 1.5) * (a.R - 1.5) : -1.0;
  // Which map reads can decide anything: the sphere owns a node of a map
  // only inside its ball there (the raster's test, |d|^2 < R^2 off the wall
  // layers), so outside it the new map cannot hold this sphere; a destroyed
  // node is the sphere's now and was fluid, so it is not surely inside the
  // old ball; a created node is fluid now and was the sphere's, so it is
  // inside the old ball and not surely inside the new one. "Maybe" and
  // "surely" inside are FP32 tests of |d|^2 against R^2 +- eps2, where eps2
  // bounds the FP32 error of |d|^2 for a node within R + 1 of the centre:
  // coordinates and centre rounded to FP32 (each within L 2^-24), the
  // subtraction, the choice of periodic image next to L/2, the squares and
  // the sum (with a factor 2 to spare). The lists are those of reading every
  // node; only the reads that cannot change them are skipped.
  const double Lmax = fmax(a.L[0], fmax(a.L[1], a.L[2]));
  const double eps2 = 8.0 * (a.R + 1.0) * (Lmax + a.R + 1.0) * 0x1p-23;
  const float R2lo = float(a.R * a.R - eps2), R2hi = float(a.R * a.R + eps2);
  const float cnf[3] = {float(c[0]), float(c[1]), float(c[2])};
  const float cof[3] = {float(P[PS_XRA]), float(P[PS_XRA + 1]), float(P[PS_XRA + 2])};
  const float Lf[3] = {float(a.L[0]), float(a.L[1]), float(a.L[2])};
  auto dist2f = [&](uint32_t wx, uint32_t wy, uint32_t wz, const float* ctr) {
    float s2 = 0.0f;
    const uint32_t wc[3] = {wx, wy, wz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float v = float(wc[d]) - ctr[d];
      v = fabsf(v + v) < Lf[d] ? v : v - Lf[d] * rintf(v / Lf[d]);
      s2 += v * v;
    }
    return s2;
  };
  if (threadIdx.x == 0) sf.staged = se.staged = 0;
  // trip counts are uniform over the workgroup: every thread reaches the barriers
  for (int k = 0; k < nb2; ++k)
    for (int jb = 0; jb < nb1; jb += 16)
      for (int ib = 0; ib < nb0; ib += 16) {
        const int i = ib + tx, j = jb + ty;
        uint32_t n = 0, mask = 0, evc = 0;
        if (i < nb0 && j < nb1) {
          const uint32_t wx = uint32_t(wrap_box(b.lo[0] + i, a.nx));
          const uint32_t wy = uint32_t(wrap_box(b.lo[1] + j, a.ny));
          const uint32_t wz = uint32_t(wrap_box(b.lo[2] + k, a.nz));
          n = wx + uint32_t(a.nx) * (wy + uint32_t(a.ny) * wz);
          const bool wall = a.walls && (wz == 0 || wz == uint32_t(a.nz) - 1);
          const float n2 = dist2f(wx, wy, wz, cnf);
          const bool maybe_new = !wall && n2 < R2hi, sure_new = !wall && n2 < R2lo;
          bool maybe_old = false, sure_old = false;
          if (events) {
            const float o2 = dist2f(wx, wy, wz, cof);
            maybe_old = !wall && o2 < R2hi;
            sure_old = !wall && o2 < R2lo;
          }
          const bool moved = events && ((maybe_new && !sure_old) || (maybe_old && !sure_new));
          const uint16_t w = (maybe_new || moved) ? a.own_new[n] : uint16_t(0);
          // a node closer than R - 3/2 to the centre has every neighbour (at
          // most sqrt 2 away) inside the ball: none of them is fluid
          const double dx = min_image(double(wx) - c[0], a.L[0]);
          const double dy = min_image(double(wy) - c[1], a.L[1]);
          const double dz = min_image(double(wz) - c[2], a.L[2]);
          if (w == me && !(dx * dx + dy * dy + dz * dz < deep2)) {
            Nbr nbr(wx, wy, wz, uint32_t(a.nx), uint32_t(a.ny), uint32_t(a.nz));
#pragma unroll
            for (int d = 1; d < Q; ++d)
              if (a.own_new[nbr.push(d)] == 0) mask |= 1u << d;
          }
          if (moved) {
            const uint16_t o = a.own_old[n];
            if (o == 0 && w == me) evc = 0x80000000u | me;   // destroyed
            else if (w == 0 && o == me) evc = me;           // created
          }
        }
        __syncthreads();
        const int cf = sf.staged, ce = se.staged;  // the same values in every thread
        __syncthreads();
        if (cf > 1024 - PBLOCK) {  // room for one entry per thread
          stage_flush(sf, fl);
          __syncthreads();
        }
        if (ce > 512 - PBLOCK) {
          stage_flush(se, ev);
          __syncthreads();
        }
        stage_push(sf, mask != 0, make_uint2(n, mask));
        if (events) stage_push(se, evc != 0, make_uint2(n, evc));
      }
  __syncthreads();
  if (sf.staged > 0) stage_flush(sf, fl);
  if (events && se.staged > 0) stage_flush(se, ev);
}

// Virtual densities on the sphere frontier (Eq. soliddens) and the Shan-Chen
// force those nodes feel (Eq. shanchen2): a solid node of a sphere with at
// least one fluid neighbour takes the w-weighted mean of the pseudo-potential
// of those neighbours; with forces on, its force
// F = -G s sum_k psi_k(n) sum_{i: n+c_i fluid} w_i psi_kbar(n+c_i) c_i and the
// torque about the sphere centre are summed into F_SC, T_SC of its sphere.
// Wall nodes are left to the wall fill.
//
// The frontier nodes come from a list (k_sphere_lists), one thread per entry,
// so that the waves are full: walking every node of the box instead leaves
// most lanes of a wave idle, since a wave crossing a sphere holds a handful
// of its frontier nodes among fluid and interior nodes.
//
// One frontier node n of sphere o with fluid-neighbour mask `mask`: its
// virtual densities, and with forces on its Shan-Chen force and torque
// (v, for sphere pid).
template <typename real, int NC, bool JANUS>
__device__ __forceinline__ void fill_one(const PArgs& a, uint32_t n, uint32_t mask, uint16_t o,
                                         int& pid, double v[6]) {
  uint32_t x, y, z;
  node_xyz(n, uint32_t(a.nx), uint32_t(a.ny), x, y, z);
  Nbr nb(x, y, z, uint32_t(a.nx), uint32_t(a.ny), uint32_t(a.nz));
  real* psi = static_cast<real*>(a.psi);
  const uint32_t N = a.N;
  // weights over the fluid neighbours from the mask alone: sum w_i and
  // sum w_i c_i, axis (1/18) and diagonal (1/36) directions counted apart
  // (__popc is unsigned: counts are taken as int before differencing)
  auto cnt = [&](uint32_t set) { return int(__popc(mask & set)); };
  const double wsum = W1 * cnt(kAxisDirs) + W2 * cnt(kDiagDirs);
  double Ws[3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    Ws[d] = W1 * (cnt(kPos1[d]) - cnt(kNeg1[d])) + W2 * (cnt(kPos2[d]) - cnt(kNeg2[d]));
  // sum_i w_i psi_k(n + c_i) and sum_i w_i psi_k(n + c_i) c_i over the
  // fluid neighbours, in the storage precision, by weight class
  double sk[NC], gk[NC][3];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const real* pk = psi + size_t(k) * N;
    real s1 = 0, s2 = 0, g1[3] = {0, 0, 0}, g2[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const real pv = (mask & (1u << i)) ? pk[nb.push(i)] : real(0);
      const int c[3] = {CX[i], CY[i], CZ[i]};
      if (axis_dir(i)) s1 += pv;
      else s2 += pv;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (!c[d]) continue;
        if (axis_dir(i)) g1[d] += c[d] > 0 ? pv : -pv;
        else g2[d] += c[d] > 0 ? pv : -pv;
      }
    }
    sk[k] = W1 * double(s1) + W2 * double(s2);
    for (int d = 0; d < 3; ++d) gk[k][d] = W1 * double(g1[d]) + W2 * double(g2[d]);
  }
  double zeta[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) zeta[k] = a.zeta[k];
  if (JANUS) {
    // Janus wetting: angle from the sphere's body x axis, smooth switch
    const double* P = a.ps + size_t(o - 1) * PSTRIDE;
    const double q0 = P[PS_Q], q1 = P[PS_Q + 1], q2 = P[PS_Q + 2], q3 = P[PS_Q + 3];
    const double ax[3] = {q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3, 2 * (q1 * q2 + q0 * q3),
                          2 * (q1 * q3 - q0 * q2)};
    const double d[3] = {min_image(double(x) - P[PS_X], a.L[0]),
                         min_image(double(y) - P[PS_X + 1], a.L[1]),
                         min_image(double(z) - P[PS_X + 2], a.L[2])};
    const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double an = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    double cth = (d[0] * ax[0] + d[1] * ax[1] + d[2] * ax[2]) / (dn * an);
    cth = fmin(1.0, fmax(-1.0, cth));
    const double theta = acos(cth) * (180.0 / M_PI);
    double t = (a.janus_theta0 + 0.5 * a.janus_width - theta) / a.janus_width;
    t = fmin(1.0, fmax(0.0, t));
    const double S = 2.0 * t * t * (3.0 - 2.0 * t) - 1.0;
    zeta[0] = a.janus_zeta[0] * S;
    if (NC == 2) zeta[NC - 1] = -a.janus_zeta[1] * S;
  }
  double dv[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    dv[k] = zeta[k] * a.rho0[k] + (1.0 + zeta[k]) * sk[k] / wsum;
    psi[size_t(k) * N + n] = real(dv[k]);
  }
  if (NC == 2 && a.acc) {
    double F[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int kb = NC - 1 - k;
      const double pk = a.rho0[k] + dv[k];
      for (int c = 0; c < 3; ++c) F[c] -= a.Gs * pk * (a.rho0[kb] * Ws[c] + gk[kb][c]);
    }
    pid = int(o) - 1;
    const double* P = a.ps + size_t(pid) * PSTRIDE;
    double d[3] = {double(x) - P[PS_X], double(y) - P[PS_X + 1], double(z) - P[PS_X + 2]};
    for (int c = 0; c < 3; ++c) d[c] -= a.L[c] * rint(d[c] * a.invL[c]);
    v[0] = F[0];
    v[1] = F[1];
    v[2] = F[2];
    v[3] = d[1] * F[2] - d[2] * F[1];
    v[4] = d[2] * F[0] - d[0] * F[2];
    v[5] = d[0] * F[1] - d[1] * F[0];
  }
}

template <typename real, int NC, bool JANUS>
__global__ void __launch_bounds__(PBLOCK) k_fill_list(PArgs a, NodeList fl) {
  const uint32_t total = min(uint32_t(*fl.count), fl.cap);
  if (blockIdx.x == 0 && threadIdx.x == 0 && uint32_t(*fl.count) > fl.cap && a.flags)
    atomicOr(a.flags + 2, 1);  // list overflow (the capacity bound rules it out)
  const uint32_t nwaves = gridDim.x * (PBLOCK / 64);
  // whole waves step together through the list: flush_runs needs every lane
  for (uint32_t base = (blockIdx.x * PBLOCK + threadIdx.x) / 64 * 64; base < total;
       base += nwaves * 64) {
    const uint32_t e = base + __lane_id();
    int pid = -1;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (e < total) {
      const uint2 en = fl.list[e];
      fill_one<real, NC, JANUS>(a, en.x, en.y, a.own_new[en.x], pid, v);
    }
    if (NC == 2 && a.acc) flush_runs<6>(a.acc, AC_FSC, pid, v);
  }
}

// ---------------------------------------------------------------------------
// Hertz contacts (Eq. hertzpot, repulsive reading) through a uniform cell list.
// ---------------------------------------------------------------------------
struct CellArgs {
  const double* ps;
  double* acc;
  int32_t* count;
  int32_t* start;
  int32_t* ids;
  int nc[3];
  double cs[3];   // cell side
  double L[3];
  int np;
  double K, d0, rcap;
  int walls;
  double zlo, zhi;
  double R, lub_mu, lub_hn, lub_hcap;
};

// cell of one coordinate, clamped to [0, nc) in floating point before the
// conversion (a non-finite coordinate lands in cell 0)
__device__ __forceinline__ int cell_index(double x, double cs, int nc) {
  double q = floor(x / cs);
  q = q >= 0.0 ? q : 0.0;
  q = q <= double(nc - 1) ? q : double(nc - 1);
  return int(q);
}

__device__ __forceinline__ int cell_of(const CellArgs& a, const double* x) {
  int ci[3];
  for (int d = 0; d < 3; ++d) ci[d] = cell_index(x[d], a.cs[d], a.nc[d]);
  return ci[0] + a.nc[0] * (ci[1] + a.nc[1] * ci[2]);
}

__global__ void k_cell_count(CellArgs a) {
  const int p = blockIdx.x * PBLOCK + threadIdx.x;
  if (p >= a.np) return;
  atomicAdd(&a.count[cell_of(a, a.ps + size_t(p) * PSTRIDE)], 1);
}

// exclusive scan of count into start (single workgroup), then clear count;
// tiles of 32 consecutive cells per thread keep the serial rounds few. The
// workgroup is one wave per SIMD, so that it finds a compute unit at once
// while the density pass fills the chip.
constexpr int kScanThreads = 256;
__global__ void __launch_bounds__(kScanThreads) k_cell_scan(int32_t* count, int32_t* start,
                                                            int ncell) {
  constexpr int PER = 32, TILE = kScanThreads * PER;
  __shared__ int32_t wsum[kScanThreads / 64];
  __shared__ int32_t carry;
  const int lane = __lane_id(), wv = int(threadIdx.x) / 64;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ncell; base += TILE) {
    const int i0 = base + int(threadIdx.x) * PER;
    int32_t v[PER], t = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      v[j] = i0 + j < ncell ? count[i0 + j] : 0;
      t += v[j];
    }
    // inclusive scan of the thread totals within the wave, then over waves
    int incl = t;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(incl, off);
      if (lane >= off) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int before = carry;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    int run = before + incl - t;
#pragma unroll
    for (int j = 0; j < PER; ++j)
      if (i0 + j < ncell) {
        start[i0 + j] = run;
        count[i0 + j] = 0;
        run += v[j];
      }
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) carry = run;
    __syncthreads();
  }
  if (threadIdx.x == 0) start[ncell] = carry;
}

__global__ void k_cell_fill(CellArgs a) {
  const int p = blockIdx.x * PBLOCK + threadIdx.x;
  if (p >= a.np) return;
  const int c = cell_of(a, a.ps + size_t(p) * PSTRIDE);
  const int slot = atomicAdd(&a.count[c], 1);
  a.ids[a.start[c] + slot] = p;
}

// sort the ids of each cell so that the pair sums have a fixed order
__global__ void k_cell_sort(CellArgs a, int ncell) {
  const int c = blockIdx.x * PBLOCK + threadIdx.x;
  if (c >= ncell) return;
  const int b = a.start[c], e = a.start[c + 1];
  // A cell of side >= d0 holds a handful of non-overlapping spheres; a crowded
  // cell only arises from non-finite positions and is left unsorted so that
  // the quadratic insertion sort stays short.
  if (e - b > 64) return;
  for (int i = b + 1; i < e; ++i) {
    const int v = a.ids[i];
    int j = i - 1;
    while (j >= b && a.ids[j] > v) {
      a.ids[j + 1] = a.ids[j];
      --j;
    }
    a.ids[j + 1] = v;
  }
}

__device__ __forceinline__ double hertz_mag(double r, double K, double d0, double rcap) {
  if (r >= d0) return 0.0;
  const double h = d0 - fmax(r, rcap);
  return 2.5 * K * h * sqrt(h);
}

// The pair force on sphere p (centre xp, state record rp) from sphere q
// (centre xq, record rq), added to F: Hertz repulsion (Eq. hertzpot) and
// lubrication (Eq. libric) along the line of centres of the nearest periodic
// images; `near` is set when the centres are closer than 2R + 1/2 (the two
// may share nodes). The velocities are read from the records only for a pair
// within the lubrication range.
__device__ __forceinline__ void pair_term(const CellArgs& a, const double xp[3], const double* rp,
                                          const double xq[3], const double* rq, double F[3],
                                          bool& near) {
  const double d[3] = {min_image(xq[0] - xp[0], a.L[0]), min_image(xq[1] - xp[1], a.L[1]),
                       min_image(xq[2] - xp[2], a.L[2])};
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  near = near || !(r >= 2.0 * a.R + 0.5);
  const double mag = hertz_mag(r, a.K, a.d0, a.rcap);
  if (mag != 0.0)
    for (int e = 0; e < 3; ++e) F[e] -= mag * d[e] / r;
  const double h = r - 2.0 * a.R;
  if (a.lub_mu > 0.0 && h < a.lub_hn) {
    const double he = fmax(h, a.lub_hcap);
    const double* vp = rp + PS_V;
    const double* vq = rq + PS_V;
    double vn = 0.0;
    for (int e = 0; e < 3; ++e) vn += (vp[e] - vq[e]) * d[e] / r;
    const double fl =
        -6.0 * M_PI * a.lub_mu * 0.25 * a.R * a.R * (1.0 / he - 1.0 / a.lub_hn) * vn;
    for (int e = 0; e < 3; ++e) F[e] += fl * d[e] / r;
  }
}

// Mirror image of a sphere across each wall plane (the same Hertz law).
__device__ __forceinline__ void wall_term(const CellArgs& a, const double xp[3], double F[3]) {
  if (!a.walls) return;
  F[2] += hertz_mag(2.0 * (xp[2] - a.zlo), a.K, a.d0, a.rcap);
  F[2] -= hertz_mag(2.0 * (a.zhi - xp[2]), a.K, a.d0, a.rcap);
}

// One thread per sphere over the 27 neighbouring cells of the cell list.
__global__ void k_pairs(CellArgs a) {
  const int p = blockIdx.x * PBLOCK + threadIdx.x;
  if (p >= a.np) return;
  const double* rp = a.ps + size_t(p) * PSTRIDE;
  const double xp[3] = {rp[0], rp[1], rp[2]};
  int ci[3];
  for (int d = 0; d < 3; ++d) ci[d] = cell_index(xp[d], a.cs[d], a.nc[d]);
  double F[3] = {0, 0, 0};
  bool near = false;
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    // visit each neighbouring cell once, also when there are fewer than 3 cells
    lo[d] = a.nc[d] >= 3 ? -1 : 0;
    hi[d] = a.nc[d] >= 3 ? 1 : a.nc[d] - 1;
  }
  for (int dz = lo[2]; dz <= hi[2]; ++dz)
    for (int dy = lo[1]; dy <= hi[1]; ++dy)
      for (int dx = lo[0]; dx <= hi[0]; ++dx) {
        const int cx = wrap_int(ci[0] + dx, a.nc[0]), cy = wrap_int(ci[1] + dy, a.nc[1]),
                  cz = wrap_int(ci[2] + dz, a.nc[2]);
        const int c = cx + a.nc[0] * (cy + a.nc[1] * cz);
        for (int s = a.start[c]; s < a.start[c + 1]; ++s) {
          const int q = a.ids[s];
          if (q == p) continue;
          const double* rq = a.ps + size_t(q) * PSTRIDE;
          const double xq[3] = {rq[0], rq[1], rq[2]};
          pair_term(a, xp, rp, xq, rq, F, near);
        }
      }
  wall_term(a, xp, F);
  double* A = a.acc + size_t(p) * ASTRIDE;
  for (int e = 0; e < 3; ++e) A[AC_FH + e] = F[e];
  A[AC_NEAR] = near ? 1.0 : 0.0;
}

// Every pair at once, for a few spheres: one workgroup per sphere, each
// thread over at most kPairsPer others, whose centres it loads together
// before any arithmetic. The map update runs beside the density pass, whose
// gathers keep the memory system full and every dependent round trip long;
// the cell list costs five dependent kernels and a serial walk over 27 cells
// per thread, and a loop with one round trip per other sphere costs as much,
// while here the sum takes one round trip. The thread sums are added in a
// fixed order (a butterfly in each wave, then the waves in turn), so the
// forces are the same on every run; far pairs add exactly zero, so they are
// those of the cell list up to the order of the sums. The workgroup writes
// the sphere's whole accumulator record (zeros, the pair force and the near
// flag), which takes the place of the record clear of the cell-list path.
constexpr int kAllPairsMax = 1024;
constexpr int kPairsPer = kAllPairsMax / PBLOCK;
static_assert(kPairsPer * PBLOCK == kAllPairsMax, "spheres per thread");
static_assert(ASTRIDE <= 64, "one lane per accumulator entry");
__global__ void __launch_bounds__(PBLOCK) k_pairs_all(CellArgs a) {
  const int p = int(blockIdx.x);  // grid: one workgroup per sphere
  const int t = int(threadIdx.x), lane = __lane_id(), wv = t / 64;
  const double* rp = a.ps + size_t(p) * PSTRIDE;
  const double xp[3] = {rp[0], rp[1], rp[2]};
  double xq[kPairsPer][3];
#pragma unroll
  for (int j = 0; j < kPairsPer; ++j) {
    const int q = t + j * PBLOCK;
    const double* rq = a.ps + size_t(q < a.np ? q : p) * PSTRIDE;
#pragma unroll
    for (int d = 0; d < 3; ++d) xq[j][d] = rq[d];
  }
  double F[3] = {0, 0, 0};
  bool near = false;
#pragma unroll
  for (int j = 0; j < kPairsPer; ++j) {
    const int q = t + j * PBLOCK;
    if (q < a.np && q != p) pair_term(a, xp, rp, xq[j], a.ps + size_t(q) * PSTRIDE, F, near);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int e = 0; e < 3; ++e) F[e] += __shfl_xor(F[e], off);
  const bool wnear = __ballot(near) != 0ull;
  __shared__ double part[PBLOCK / 64][3];
  __shared__ int pnear[PBLOCK / 64];
  if (lane == 0) {
    for (int e = 0; e < 3; ++e) part[wv][e] = F[e];
    pnear[wv] = wnear ? 1 : 0;
  }
  __syncthreads();
  if (wv != 0) return;
  double G[3] = {0, 0, 0};
  int nr = 0;
  for (int w = 0; w < PBLOCK / 64; ++w) {
    for (int e = 0; e < 3; ++e) G[e] += part[w][e];
    nr |= pnear[w];
  }
  wall_term(a, xp, G);
  if (lane < ASTRIDE) {
    double v = 0.0;
    if (lane == AC_FH) v = G[0];
    if (lane == AC_FH + 1) v = G[1];
    if (lane == AC_FH + 2) v = G[2];
    if (lane == AC_NEAR) v = nr ? 1.0 : 0.0;
    a.acc[size_t(p) * ASTRIDE + lane] = v;
  }
}

// ---------------------------------------------------------------------------
// Newton-Euler update (Eq. lf) with the half-step fluid force average and
// Svanberg's implicit mid-step quaternion (Eq. quatder, svanimpl).
// ---------------------------------------------------------------------------
__device__ void quat_rate(const double q[4], const double w[3], double out[4]) {
  const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  // body-frame angular velocity w* = R(q)^T w with the (unnormalised) matrix R(q)
  const double R00 = q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3, R01 = 2 * (q1 * q2 - q0 * q3),
               R02 = 2 * (q1 * q3 + q0 * q2);
  const double R10 = 2 * (q1 * q2 + q0 * q3), R11 = q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3,
               R12 = 2 * (q2 * q3 - q0 * q1);
  const double R20 = 2 * (q1 * q3 - q0 * q2), R21 = 2 * (q2 * q3 + q0 * q1),
               R22 = q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3;
  const double bx = R00 * w[0] + R10 * w[1] + R20 * w[2];
  const double by = R01 * w[0] + R11 * w[1] + R21 * w[2];
  const double bz = R02 * w[0] + R12 * w[1] + R22 * w[2];
  out[0] = 0.5 * (-q1 * bx - q2 * by - q3 * bz);
  out[1] = 0.5 * (q0 * bx - q3 * by + q2 * bz);
  out[2] = 0.5 * (q3 * bx + q0 * by - q1 * bz);
  out[3] = 0.5 * (-q2 * bx + q1 * by + q0 * bz);
}

__global__ void k_integrate(double* ps, const double* acc, int np, double mass, double inertia,
                            double Lx, double Ly, double Lz, int rotate) {
  const int p = blockIdx.x * PBLOCK + threadIdx.x;
  if (p >= np) return;
  double* P = ps + size_t(p) * PSTRIDE;
  const double* A = acc + size_t(p) * ASTRIDE;
  if (P[PS_HAVEPREV] == 0.0)
    for (int e = 0; e < 3; ++e) {
      P[PS_FPREV + e] = A[AC_FLIQ + e];
      P[PS_TPREV + e] = A[AC_TLIQ + e];
    }
  const double L[3] = {Lx, Ly, Lz};
  double w[3];
  for (int e = 0; e < 3; ++e) {
    const double F = 0.5 * (P[PS_FPREV + e] + A[AC_FLIQ + e]) + A[AC_FD + e] + A[AC_FC + e] +
                     A[AC_FH + e] + A[AC_FSC + e];
    const double T = 0.5 * (P[PS_TPREV + e] + A[AC_TLIQ + e]) + A[AC_TD + e] + A[AC_TC + e] +
                     A[AC_TSC + e];
    P[PS_V + e] += F / mass;
    P[PS_XRB + e] = P[PS_XRA + e];
    P[PS_XRA + e] = P[PS_X + e];
    double x = fmod(P[PS_X + e] + P[PS_V + e], L[e]);
    if (x < 0) x += L[e];
    if (x >= L[e]) x -= L[e];
    P[PS_X + e] = x;
    if (rotate) P[PS_W + e] += T / inertia;
    w[e] = P[PS_W + e];
    P[PS_FPREV + e] = A[AC_FLIQ + e];
    P[PS_TPREV + e] = A[AC_TLIQ + e];
  }
  P[PS_HAVEPREV] = 1.0;
  if (!rotate) return;
  double q[4] = {P[PS_Q], P[PS_Q + 1], P[PS_Q + 2], P[PS_Q + 3]};
  double qd[4], qh[4], qn[4];
  quat_rate(q, w, qd);
  for (int c = 0; c < 4; ++c) qh[c] = q[c] + 0.5 * qd[c];
  for (int it = 0; it < 50; ++it) {
    quat_rate(qh, w, qn);
    double diff = 0.0;
    for (int c = 0; c < 4; ++c) diff = fmax(diff, fabs(qn[c] - qd[c]));
    for (int c = 0; c < 4; ++c) {
      qd[c] = qn[c];
      qh[c] = q[c] + 0.5 * qd[c];
    }
    if (diff <= 1e-14) break;
  }
  double nrm = 0.0;
  for (int c = 0; c < 4; ++c) {
    q[c] += qd[c];
    nrm += q[c] * q[c];
  }
  nrm = sqrt(nrm);
  for (int c = 0; c < 4; ++c) P[PS_Q + c] = q[c] / nrm;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Zero `bytes` bytes at p: 16-byte stores for the aligned body, single bytes
// for the edges. The step clears its buffers with this kernel rather than a
// memset: a caller may capture steps into a graph, and memset nodes have
// given wrong results on graph replays on this hardware.
__global__ void __launch_bounds__(PBLOCK) k_zero(unsigned char* __restrict__ p, size_t bytes) {
  const size_t head = (16u - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u;
  const size_t h = head < bytes ? head : bytes;
  const size_t body = (bytes - h) / 16;
  const size_t tid = size_t(blockIdx.x) * PBLOCK + threadIdx.x;
  const size_t nth = size_t(gridDim.x) * PBLOCK;
  uint4* q = reinterpret_cast<uint4*>(p + h);
  for (size_t i = tid; i < body; i += nth) q[i] = make_uint4(0u, 0u, 0u, 0u);
  const size_t done = h + body * 16;
  if (tid < h) p[tid] = 0;
  if (tid < bytes - done) p[done + tid] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((bytes / 16 + PBLOCK - 1) / PBLOCK, 4096);
  hipLaunchKernelGGL(k_zero, dim3(uint32_t(std::max<size_t>(blocks, 1))), dim3(PBLOCK), 0, s,
                     static_cast<unsigned char*>(p), bytes);
  return hipGetLastError();
}

static PArgs pargs(lb_ctx* c, uint16_t* own_new, const uint16_t* own_old) {
  PArgs a;
  a.own_new = own_new;
  a.own_old = own_old;
  a.ps = pstate(c);
  a.acc = pacc(c);
  a.flags = reinterpret_cast<int32_t*>(wptr(c, c->wl.flags));
  a.fin = c->B.f[c->cur];
  a.psi = c->B.rho;
  a.nx = int(c->geo.nx);
  a.ny = int(c->geo.ny);
  a.nz = int(c->geo.nz);
  a.N = c->geo.N;
  a.L[0] = c->geo.nx;
  a.L[1] = c->geo.ny;
  a.L[2] = c->geo.nz;
  for (int d = 0; d < 3; ++d) a.invL[d] = 1.0 / a.L[d];
  a.R = c->P.radius;
  a.ncomp = c->geo.ncomp;
  for (int k = 0; k < 2; ++k) {
    a.rho0[k] = c->P.rho0[k];
    a.zeta[k] = c->P.zeta[k];
    a.rho_fb[k] = c->P.rho_fallback[k];
  }
  a.Gs = c->P.G * c->P.sc_norm;
  a.walls = c->P.walls;
  a.np = c->nparticles;
  a.janus = c->P.janus;
  a.janus_theta0 = c->P.janus_theta0;
  a.janus_width = c->P.janus_width;
  a.janus_zeta[0] = c->P.janus_zeta[0];
  a.janus_zeta[1] = c->P.janus_zeta[1];
  return a;
}

hipError_t launch_raster_full(lb_ctx* c, uint16_t* owner) {
  const auto& g = c->geo;
  c->flist_map = nullptr;
  hipLaunchKernelGGL(k_map_reset, dim3((g.N + PBLOCK - 1) / PBLOCK), dim3(PBLOCK), 0, c->stream,
                     owner, g.nx, g.ny, g.nz, c->P.walls);
  if (c->nparticles > 0)
    hipLaunchKernelGGL(k_raster, dim3(c->nparticles), dim3(PBLOCK), 0, c->stream,
                       pargs(c, owner, owner), int(PS_X), 0);
  return hipGetLastError();
}

hipError_t launch_clear_accumulators(lb_ctx* c) {
  return launch_zero(pacc(c), size_t(c->nparticles) * ASTRIDE * sizeof(double), c->stream);
}

// On stream s: clear the per-step sphere accumulators, sum the Hertz and
// lubrication pair forces through the cell list (flagging spheres that may
// share nodes), rebuild the new map at the current centres, and list its
// frontier and the node events of the step. Independent of the populations,
// so it can run beside the density pass.
hipError_t launch_map_update(lb_ctx* c, hipStream_t s) {
  uint16_t* own_new = static_cast<uint16_t*>(c->B.owner[1 - c->own_old]);
  const uint16_t* own_old = static_cast<const uint16_t*>(c->B.owner[c->own_old]);
  const PArgs a = pargs(c, own_new, own_old);
  const dim3 gp(c->nparticles), bp(PBLOCK);
  // Hertz and lubrication pairs: all at once for a few spheres, else through
  // the cell list
  CellArgs ca;
  ca.ps = pstate(c);
  ca.acc = pacc(c);
  ca.count = reinterpret_cast<int32_t*>(wptr(c, c->wl.cell_count));
  ca.start = reinterpret_cast<int32_t*>(wptr(c, c->wl.cell_start));
  ca.ids = reinterpret_cast<int32_t*>(wptr(c, c->wl.cell_ids));
  int ncell = 1;
  for (int d = 0; d < 3; ++d) {
    ca.nc[d] = c->ncell[d];
    ncell *= c->ncell[d];
    ca.L[d] = d == 0 ? c->geo.nx : d == 1 ? c->geo.ny : c->geo.nz;
    ca.cs[d] = ca.L[d] / c->ncell[d];
  }
  ca.np = c->nparticles;
  ca.K = c->P.hertz_K;
  ca.d0 = c->P.hertz_d0;
  ca.rcap = c->P.hertz_rcap;
  ca.walls = c->P.walls;
  ca.zlo = 0.5;
  ca.zhi = c->geo.nz - 1.5;
  ca.R = c->P.radius;
  ca.lub_mu = c->P.lub_mu;
  ca.lub_hn = c->P.lub_hn;
  ca.lub_hcap = c->P.lub_hcap;
  hipError_t e;
  if (c->nparticles <= kAllPairsMax) {
    hipLaunchKernelGGL(k_pairs_all, gp, bp, 0, s, ca);
  } else {
    e = launch_zero(pacc(c), size_t(c->nparticles) * ASTRIDE * sizeof(double), s);
    if (e != hipSuccess) return e;
    e = launch_zero(ca.count, size_t(ncell) * sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    const dim3 gt((c->nparticles + PBLOCK - 1) / PBLOCK);
    hipLaunchKernelGGL(k_cell_count, gt, bp, 0, s, ca);
    hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(kScanThreads), 0, s, ca.count, ca.start, ncell);
    hipLaunchKernelGGL(k_cell_fill, gt, bp, 0, s, ca);
    hipLaunchKernelGGL(k_cell_sort, dim3((ncell + PBLOCK - 1) / PBLOCK), bp, 0, s, ca, ncell);
    hipLaunchKernelGGL(k_pairs, gt, bp, 0, s, ca);
  }
  // the new map: cleared, walls, spheres at the current centres
  e = launch_zero(own_new, size_t(c->geo.N) * sizeof(uint16_t), s);
  if (e != hipSuccess) return e;
  if (c->P.walls) {
    const uint32_t plane = c->geo.nx * c->geo.ny;
    hipLaunchKernelGGL(k_wall_planes, dim3((2 * plane + PBLOCK - 1) / PBLOCK), bp, 0, s, own_new,
                       c->geo.nx, c->geo.ny, c->geo.nz);
  }
  hipLaunchKernelGGL(k_raster, gp, bp, 0, s, a, int(PS_X), 1);
  e = launch_sphere_lists(c, own_new, own_old, int(PS_X), s);
  c->flist_map = e == hipSuccess ? own_new : nullptr;
  return e;
}

// Node creation and destruction between the two maps (after the density pass
// and the map update).
static NodeList frontier_list(lb_ctx* c) {
  NodeList fl;
  fl.list = reinterpret_cast<uint2*>(wptr(c, c->wl.flist));
  fl.count = reinterpret_cast<int32_t*>(wptr(c, c->wl.fcount));
  fl.cap = uint32_t(c->wl.fcap);
  return fl;
}

static NodeList event_list(lb_ctx* c) {
  NodeList ev;
  ev.list = reinterpret_cast<uint2*>(wptr(c, c->wl.elist));
  ev.count = reinterpret_cast<int32_t*>(wptr(c, c->wl.ecount));
  ev.cap = uint32_t(c->wl.ecap);
  return ev;
}

hipError_t launch_sphere_lists(lb_ctx* c, const uint16_t* owner, const uint16_t* owner_old,
                               int which, hipStream_t s) {
  const NodeList fl = frontier_list(c);
  NodeList ev = event_list(c);
  hipError_t e = launch_zero(fl.count, sizeof(int32_t), s);
  if (e == hipSuccess && owner_old) e = launch_zero(ev.count, sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  if (!owner_old) ev.list = nullptr;
  if (c->nparticles > 0) {
    const PArgs a = pargs(c, const_cast<uint16_t*>(owner), owner_old ? owner_old : owner);
    if (c->geo.prec == LB_FP64)
      hipLaunchKernelGGL(k_sphere_lists<true>, dim3(c->nparticles), dim3(PBLOCK), 0, s, a, fl,
                         ev, which);
    else
      hipLaunchKernelGGL(k_sphere_lists<false>, dim3(c->nparticles), dim3(PBLOCK), 0, s, a, fl,
                         ev, which);
  }
  return hipGetLastError();
}

hipError_t launch_events(lb_ctx* c) {
  uint16_t* own_new = static_cast<uint16_t*>(c->B.owner[1 - c->own_old]);
  const uint16_t* own_old = static_cast<const uint16_t*>(c->B.owner[c->own_old]);
  const PArgs a = pargs(c, own_new, own_old);
  const NodeList ev = event_list(c);
  if (ev.cap == 0) return hipSuccess;
  const dim3 grid(uint32_t(std::min<size_t>((c->wl.ecap + PBLOCK - 1) / PBLOCK, 1024))), bp(PBLOCK);
  const bool two = c->geo.ncomp == 2;
  if (c->geo.prec == LB_FP64) {
    if (two) hipLaunchKernelGGL((k_events_list<double, 2>), grid, bp, 0, c->stream, a, ev);
    else hipLaunchKernelGGL((k_events_list<double, 1>), grid, bp, 0, c->stream, a, ev);
  } else {
    if (two) hipLaunchKernelGGL((k_events_list<float, 2>), grid, bp, 0, c->stream, a, ev);
    else hipLaunchKernelGGL((k_events_list<float, 1>), grid, bp, 0, c->stream, a, ev);
  }
  return hipGetLastError();
}

hipError_t launch_fill_particles(lb_ctx* c, const uint16_t* owner, bool forces, bool list_ready) {
  if (!list_ready && c->flist_map != owner) {
    // the current map: rasterised around the centres of the last step
    const hipError_t e = launch_sphere_lists(c, owner, nullptr, int(PS_XRA), c->stream);
    if (e != hipSuccess) return e;
    c->flist_map = owner;
  }
  PArgs a = pargs(c, const_cast<uint16_t*>(owner), owner);
  if (!forces) a.acc = nullptr;  // psi only: leave the force terms alone
  const NodeList fl = frontier_list(c);
  if (fl.cap == 0) return hipSuccess;
  // enough waves to cover the list in a few passes
  const dim3 grid(uint32_t(std::min<size_t>((c->wl.fcap + PBLOCK - 1) / PBLOCK, 32768)));
  const bool two = c->geo.ncomp == 2, janus = c->P.janus != 0;
  const hipStream_t s = c->stream;
  if (c->geo.prec == LB_FP64) {
    if (two && janus) hipLaunchKernelGGL((k_fill_list<double, 2, true>), grid, dim3(PBLOCK), 0, s, a, fl);
    else if (two) hipLaunchKernelGGL((k_fill_list<double, 2, false>), grid, dim3(PBLOCK), 0, s, a, fl);
    else if (janus) hipLaunchKernelGGL((k_fill_list<double, 1, true>), grid, dim3(PBLOCK), 0, s, a, fl);
    else hipLaunchKernelGGL((k_fill_list<double, 1, false>), grid, dim3(PBLOCK), 0, s, a, fl);
  } else {
    if (two && janus) hipLaunchKernelGGL((k_fill_list<float, 2, true>), grid, dim3(PBLOCK), 0, s, a, fl);
    else if (two) hipLaunchKernelGGL((k_fill_list<float, 2, false>), grid, dim3(PBLOCK), 0, s, a, fl);
    else if (janus) hipLaunchKernelGGL((k_fill_list<float, 1, true>), grid, dim3(PBLOCK), 0, s, a, fl);
    else hipLaunchKernelGGL((k_fill_list<float, 1, false>), grid, dim3(PBLOCK), 0, s, a, fl);
  }
  return hipGetLastError();
}

hipError_t launch_integrate(lb_ctx* c) {
  hipLaunchKernelGGL(k_integrate, dim3((c->nparticles + PBLOCK - 1) / PBLOCK), dim3(PBLOCK), 0,
                     c->stream, pstate(c), pacc(c), c->nparticles, c->mass, c->inertia,
                     double(c->geo.nx), double(c->geo.ny), double(c->geo.nz), c->P.rotate);
  return hipGetLastError();
}

}  // namespace lbh
