// lb_fluid.hip -- fluid kernels of the gfx950 path.
//
// Storage: two population buffers f[k][i][n] (SoA, x fastest) holding the
// post-collision populations of the previous step in pull form: the value
// that streams into node n along c_i sits at slot (i, n - c_i). Solid nodes'
// slots carry the reflected values of the links that end on them, so the
// pull-gather needs no bounce-back branch. Values are deviations
// f_i - w_i rho0_k in the storage type `real` (float or double).
#include <hip/hip_runtime.h>

#include "lb_device.hpp"
#include "lb_internal.hpp"

namespace lbh {

constexpr int BLOCK = 256;

static inline uint32_t nblocks(uint64_t n) { return uint32_t((n + BLOCK - 1) / BLOCK); }
// target band width of the collide sweep, in workgroups per z-plane (16
// workgroups: 4,096 nodes, 8 rows of 512)
constexpr uint32_t kBandTarget = 16;

// ---------------------------------------------------------------------------
// Initial populations f_i = f_eq(rho0(n), u0(n)) (Eq. LEQ), written in pull form.
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(BLOCK)
k_init(real* __restrict__ f, const double* __restrict__ rho0, const double* __restrict__ u0,
       const uint16_t* __restrict__ owner, uint32_t first, uint32_t count, uint32_t nx,
       uint32_t ny, uint32_t nz, int ncomp, double r0a, double r0b) {
  const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
  if (t >= count) return;
  const uint32_t n = first + t, N = nx * ny * nz;
  if (owner && owner[n] != 0) return;
  uint32_t x, y, z;
  node_xyz(n, nx, ny, x, y, z);
  Nbr nb(x, y, z, nx, ny, nz);
  double ux = 0, uy = 0, uz = 0;
  if (u0) {
    ux = u0[3 * size_t(t)];
    uy = u0[3 * size_t(t) + 1];
    uz = u0[3 * size_t(t) + 2];
  }
  const double uu = ux * ux + uy * uy + uz * uz;
  for (int k = 0; k < ncomp; ++k) {
    const double r = rho0[size_t(k) * count + t];
    const double ref = k == 0 ? r0a : r0b;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
      const double dev = WQ[i] * (r - ref) + WQ[i] * r * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      f[(size_t(k) * Q + i) * N + nb.pull(i)] = real(dev);
    }
  }
}

// ---------------------------------------------------------------------------
// Moments of the pull-gathered populations: psi_k(n) - rho0_k = sum_i df_i.
// Written for every node; solid nodes get overwritten by the fill kernels.
// Each XCD sweeps one contiguous range of nodes, so that the lines a gather
// shifted by one node shares with the neighbouring workgroup stay in its L2.
// ---------------------------------------------------------------------------
template <typename real, int NC>
__global__ void __launch_bounds__(BLOCK)
k_density(const real* __restrict__ f, real* __restrict__ psi, uint32_t nx, uint32_t ny,
          uint32_t nz, uint32_t blocks_per_xcd) {
  const uint32_t b = (blockIdx.x % 8u) * blocks_per_xcd + blockIdx.x / 8u;
  const uint32_t n = b * BLOCK + threadIdx.x;
  const uint32_t N = nx * ny * nz;
  if (n >= N) return;
  uint32_t x, y, z;
  node_xyz(n, nx, ny, x, y, z);
  Nbr nb(x, y, z, nx, ny, nz);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const real* fk = f + size_t(k) * Q * N;
    real s = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) s += ld32(fk + size_t(i) * N, nb.pull(i));
    st32(psi + size_t(k) * N, n, s);
  }
}

struct CollideArgs {
  const void* fin;
  void* fout;
  const void* psi;
  const uint16_t* owner;
  const double* ps;   // sphere state records
  double* acc;        // sphere accumulators
  uint32_t nx, ny, nz, N;
  double Gs;          // G * sc_norm
  double g[3];
  double rho0[2];
  double inv_tau[2];
  double nu[2];       // c_s^2 (tau_k - 1/2)
  double omega;       // relaxation rate when the relaxation times are equal
  int equal_tau;
  double wall_lo[3], wall_hi[3];
  int wall_type[2];         // 0 moving wall, 1 pressure, 2 velocity, 3 equilibrium
  double wall_rho[2][2];    // [face][component]
  const double* ubnd;       // [2][nx*ny][3] mixture velocity one layer inside each face
  double L[3], invL[3];
  uint32_t blocks_per_xcd;  // workgroups per XCD (grid = 8 x blocks_per_xcd)
  uint32_t nblk;            // workgroups that hold nodes
  uint32_t band_w;          // workgroups per band and z-plane (0: whole planes)
  uint32_t plane_w;         // workgroups per z-plane
  uint32_t* counts;         // [k][i][N] store counts of the counting variant, else null
};

// Packed direction tables for a direction index that varies per lane:
// two bits (c + 1) per direction and axis.
constexpr uint64_t pack_dir(const int* c) {
  uint64_t v = 0;
  for (int i = 0; i < Q; ++i) v |= uint64_t(c[i] + 1) << (2 * i);
  return v;
}
constexpr uint64_t PCX = pack_dir(CX), PCY = pack_dir(CY), PCZ = pack_dir(CZ);
__device__ __forceinline__ int dir_c(uint64_t packed, int i) { return int((packed >> (2 * i)) & 3) - 1; }
// opposite direction in the library's order (1<->2, 3<->4, 5<->6, 7<->8, 9..13<->14..18)
__device__ __forceinline__ int dir_opp(int i) { return i <= 8 ? ((i - 1) ^ 1) + 1 : (i <= 13 ? i + 5 : i - 5); }

// ---------------------------------------------------------------------------
// Bounce-back of one link and its momentum exchange. Fluid node (x, y, z),
// with post-collision values fs_k = f*_ki and densities rho_k, has a solid
// neighbour s = n + c_i owned by o (a sphere id + 1, or the wall). The
// reflection of Eq. bbv / LADDFLBE with the surface velocity of Eq. UPI,
//   f*_ki - 2 w_i rho_k (u_w . c_i) / c_s^2,
// goes into slot (opp(i), s), the one n gathers next step; the link force of
// Eq. LADDFORCE, sum_k [2 f*_ki - 2 w_i rho_k (u_w . c_i)/c_s^2] c_i, with the
// constant part 2 w_i rho0_k c_i added in FP64, and its torque about the
// sphere centre (Eq. FORCEPARTEQ, TORQUEPARTEQ) are accumulated per lane in
// lv for sphere pid (flushed with atomics when a lane moves on to another
// sphere). u_w = v + w x (r_w - x_p) with r_w the link midpoint.
// ---------------------------------------------------------------------------
// Open face (Sec. 2.2): the population leaving fluid node n along c_i into
// the face layer returns along -c_i (full values; stored as deviations) as
//   pressure:     -f*_i + 2 w_i rho_w [1 + (u_w.c_i)^2/(2 cs^4) - u_w^2/(2 cs^2)]  (Eq. bbp)
//   velocity:      f*_i - 2 w_i rho_w (u_w.c_i)/cs^2                                (Eq. bbv)
//   equilibrium:   f_eq_{-i}(rho_w, u_w)
// with the face's density (pressure, equilibrium) or velocity (velocity,
// equilibrium) and the other extrapolated: X_w = X(n) + (X(n) - X(n'))/2,
// n' the next node inwards along z (X(n) alone if n' is solid).
template <typename real, int NC, bool COUNT>
__device__ void open_face(const CollideArgs& a, int face, int i, int j, uint32_t s, uint32_t x,
                          uint32_t y, uint32_t z, const real fs[NC], const real rho[NC],
                          const real u[3]) {
  const uint32_t N = a.N;
  real* __restrict__ fout = static_cast<real*>(a.fout);
  const real* __restrict__ psi = static_cast<const real*>(a.psi);
  const int cx = dir_c(PCX, i), cy = dir_c(PCY, i), cz = dir_c(PCZ, i);
  const double wi = (cx * cx + cy * cy + cz * cz == 1) ? W1 : W2;
  const uint32_t plane = a.nx * a.ny;
  const uint32_t n = x + a.nx * (y + a.ny * z);
  const uint32_t nin = face == 0 ? n + plane : n - plane;
  const bool ok = a.owner[nin] == 0;
  const int type = a.wall_type[face];
  const double* U = face == 0 ? a.wall_lo : a.wall_hi;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double w0 = wi * a.rho0[k];
    const double f = double(fs[k]) + w0;  // full post-collision value
    double r;
    if (type == 1) {
      const double* ui = a.ubnd + (size_t(face) * plane + (x + a.nx * y)) * 3;
      double uw[3];
      for (int d = 0; d < 3; ++d) {
        const double un = double(u[d]);
        uw[d] = ok ? un + 0.5 * (un - ui[d]) : un;
      }
      const double uc = uw[0] * cx + uw[1] * cy + uw[2] * cz;
      const double uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
      r = -f + 2.0 * wi * a.wall_rho[face][k] * (1.0 + 4.5 * uc * uc - 1.5 * uu);
    } else if (type == 2) {
      const double rn = double(rho[k]);
      const double rin = a.rho0[k] + double(psi[size_t(k) * N + nin]);
      const double rw = ok ? rn + 0.5 * (rn - rin) : rn;
      r = f - 6.0 * wi * rw * (U[0] * cx + U[1] * cy + U[2] * cz);
    } else {
      // f_eq along -c_i
      const double uc = -(U[0] * cx + U[1] * cy + U[2] * cz);
      const double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
      r = wi * a.wall_rho[face][k] * (1.0 + 3.0 * uc + 4.5 * uc * uc - 1.5 * uu);
    }
    st32(fout + (size_t(k) * Q + j) * N, s, real(r - w0));
    if (COUNT) atomicAdd(a.counts + (size_t(k) * Q + j) * N + s, 1u);
  }
}

template <typename real, int NC, bool COUNT>
__device__ __forceinline__ void link_one(const CollideArgs& a, int i, uint16_t o, uint32_t x,
                                         uint32_t y, uint32_t z, const real fs[NC],
                                         const real rho[NC], const real u[3], int& pid,
                                         double lv[7]) {
  const uint32_t N = a.N;
  real* __restrict__ fout = static_cast<real*>(a.fout);
  const int cx = dir_c(PCX, i), cy = dir_c(PCY, i), cz = dir_c(PCZ, i);
  const int j = dir_opp(i);
  const uint32_t s = nbr_dyn(x, y, z, cx, cy, cz, a.nx, a.ny, a.nz);
  const double wi = (cx * cx + cy * cy + cz * cz == 1) ? W1 : W2;
  double uwx, uwy, uwz, rwx = 0, rwy = 0, rwz = 0;
  int p = -1;
  if (o == OWN_WALL) {
    const bool lo = int(z) + cz == 0;
    if (a.wall_type[lo ? 0 : 1] != 0) {
      open_face<real, NC, COUNT>(a, lo ? 0 : 1, i, j, s, x, y, z, fs, rho, u);
      return;
    }
    uwx = lo ? a.wall_lo[0] : a.wall_hi[0];
    uwy = lo ? a.wall_lo[1] : a.wall_hi[1];
    uwz = lo ? a.wall_lo[2] : a.wall_hi[2];
  } else {
    p = int(o) - 1;
    const double* P = a.ps + size_t(p) * PSTRIDE;
    double d;
    d = double(x) + 0.5 * cx - P[PS_X];
    rwx = d - a.L[0] * rint(d * a.invL[0]);
    d = double(y) + 0.5 * cy - P[PS_X + 1];
    rwy = d - a.L[1] * rint(d * a.invL[1]);
    d = double(z) + 0.5 * cz - P[PS_X + 2];
    rwz = d - a.L[2] * rint(d * a.invL[2]);
    const double wx = P[PS_W], wy = P[PS_W + 1], wz = P[PS_W + 2];
    uwx = P[PS_V] + (wy * rwz - wz * rwy);
    uwy = P[PS_V + 1] + (wz * rwx - wx * rwz);
    uwz = P[PS_V + 2] + (wx * rwy - wy * rwx);
  }
  const real cw = real(6.0 * wi * (uwx * cx + uwy * cy + uwz * cz));
  double dev = 0.0;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const real corr = cw * rho[k];
    // the reflected slot lies in another row, usually one already written
    // back: a streaming store (measured 0.1 ms faster at 512^3 than a plain one)
    __builtin_nontemporal_store(fs[k] - corr, fout + (size_t(k) * Q + j) * N + s);
    if (COUNT) atomicAdd(a.counts + (size_t(k) * Q + j) * N + s, 1u);
    dev += double(real(2) * fs[k] - corr);
  }
  if (p < 0 || !a.acc) return;
  const double rho0sum = a.rho0[0] + (NC == 2 ? a.rho0[NC - 1] : 0.0);
  const double fl = 2.0 * wi * rho0sum + dev;  // F_link = fl c_i
  const double Fx = fl * cx, Fy = fl * cy, Fz = fl * cz;
  if (p != pid) {
    if (pid >= 0) {  // this lane's links touch another sphere: flush the first one
      double* acp = a.acc + size_t(pid) * ASTRIDE;
#pragma unroll
      for (int c = 0; c < 6; ++c) unsafeAtomicAdd(acp + AC_FLIQ + c, lv[c]);
      unsafeAtomicAdd(acp + AC_FLABS, lv[6]);
    }
    pid = p;
#pragma unroll
    for (int c = 0; c < 7; ++c) lv[c] = 0.0;
  }
  lv[0] += Fx;
  lv[1] += Fy;
  lv[2] += Fz;
  lv[3] += rwy * Fz - rwz * Fy;
  lv[4] += rwz * Fx - rwx * Fz;
  lv[5] += rwx * Fy - rwy * Fx;
  lv[6] += fabs(fl) * (wi == W1 ? 1.0 : 1.4142135623730951);
}

// Links of one wave, gathered in LDS so that every lane takes one link at a
// time instead of each lane walking its own (a wave would otherwise iterate
// as often as its busiest lane has links). The queues of a workgroup's waves
// are then processed as one list, in 64-entry chunks dealt to the waves, so
// the links fill as few waves as they need. Entries beyond a wave's capacity
// are left to their lanes (see k_collide).
constexpr int QW = 256;
// With 4-byte values every lane keeps all its post-collision values, indexed
// by (direction, lane), which costs one LDS store per value and no index
// arithmetic; 8-byte values are packed by link to stay within the LDS budget.
template <typename real>
constexpr bool kDenseLinks = sizeof(real) == 4;
template <typename real, int NC>
struct LinkQueue {
  uint32_t meta[QW];  // lane | direction << 6 | owner << 11
  real fs[NC][kDenseLinks<real> ? Q * 64 : QW];
  uint32_t x[64], y[64], z[64];
  real rho[NC][64];
  real u[3][64];
};

// ---------------------------------------------------------------------------
// The fused step, one thread per node: pull-gather (Eq. bgk2), moments and
// mixture velocity (Eq. rho, vel, scvel), Shan-Chen acceleration from the
// pseudo-potential of the neighbours (Eq. shanchen), EDM collision
// (Eq. lbsbgk) and store; then the bounce-back and momentum exchange of
// every link from a fluid node to a solid one (link_one).
//
// Collision in deviation form, with E_i(v) = w_i rho (3 c.v + 4.5 (c.v)^2 - 1.5 v.v):
//   df*_i = w_i drho + E_i(u + a) + (1 - omega)(df_i - w_i drho - E_i(u)),
// which regroups, per pair of opposite directions i and -i, into a part even
// in c_i and a part odd in c_i (o = 1 - omega, v = u + a):
//   df*_{+-i} = o df_{+-i} + w_i [S + 4.5 rho ((c.v)^2 - o (c.u)^2)]
//                          +- 3 w_i rho (c.v - o c.u),
//   S = omega drho - 1.5 rho (v.v - o u.u),
// so each pair costs one evaluation of the two parts.
// Every load of the node (map, gathers, pseudo-potential) is issued before
// any branch on the map. A solid node writes zeros into the slots that no
// link fills, so together with the reflections every slot of the output is
// written. Workgroups are dealt round-robin over the 8 XCDs; the block index
// is remapped so that each XCD sweeps its own y-bands of the box, each band
// through every z-plane (band_block), and neighbouring rows share that XCD's
// L2.
// ---------------------------------------------------------------------------
// Order in which an XCD sweeps its workgroups. The box is cut along y into
// bands of band_w workgroups per z-plane; the sweep takes one band through
// every z-plane before the next band. The rows at z - 1 and z + 1 of a row
// (its pseudo-potential neighbours, and the solid slots that its reflections
// fill) are then handled within a few hundred workgroups of it, while they
// still sit in the XCD's L2. Logical index s -> workgroup of nodes.
__device__ __forceinline__ uint32_t band_block(const CollideArgs& a, uint32_t s) {
  if (a.band_w == 0 || s >= a.nblk) return s;
  const uint32_t w = s % a.band_w, t = s / a.band_w;
  const uint32_t z = t % a.nz, band = t / a.nz;
  return z * a.plane_w + band * a.band_w + w;
}

// COUNT: the variant that also counts every population store in a.counts
// (one writer per slot of the output: the uniqueness of the reflected slots
// and the completeness of the solid nodes' zeros); selected at run time by
// lb_debug_count_writes, never by a step that does not ask for it.
template <typename real, int NC, bool SOLIDS, bool COUNT = false>
__global__ void __launch_bounds__(BLOCK) k_collide(const CollideArgs a) {
  const uint32_t b = band_block(a, (blockIdx.x % 8u) * a.blocks_per_xcd + blockIdx.x / 8u);
  const uint32_t n0 = b * BLOCK + threadIdx.x;
  const bool valid = n0 < a.N;
  const uint32_t N = a.N;
  const uint32_t n = valid ? n0 : N - 1;  // tail lanes mirror the last node and store nothing
  uint32_t x, y, z;
  node_xyz(n, a.nx, a.ny, x, y, z);
  Nbr nb(x, y, z, a.nx, a.ny, a.nz);
  const real* __restrict__ fin = static_cast<const real*>(a.fin);
  real* __restrict__ fout = static_cast<real*>(a.fout);
  const real* __restrict__ psi = static_cast<const real*>(a.psi);
  const int lane = __lane_id();

  // map: this node and the 18 neighbours; the wave's links are numbered
  uint32_t lmask = 0;
  bool fluid = valid;
  int qbase = 0, qtotal = 0;
  bool queued = true;
  __shared__ LinkQueue<real, NC> lqs[SOLIDS ? BLOCK / 64 : 1];
  LinkQueue<real, NC>& lq = lqs[SOLIDS ? threadIdx.x / 64 : 0];
  if (SOLIDS) {
    fluid = valid && ld32(a.owner, n) == 0;
    uint16_t ow[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      ow[i] = ld32(a.owner, nb.push(i));
      if (ow[i] != 0) lmask |= 1u << i;
    }
    const uint32_t lm = fluid ? lmask : 0u;
    const int cnt = __popc(lm);
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    qbase = incl - cnt;
    queued = qbase + cnt <= QW;
    // entries of lanes past the capacity stay with their lanes
    const uint64_t over = __ballot(!queued && cnt > 0);
    qtotal = over ? __shfl(qbase, __ffsll((unsigned long long)over) - 1) : __shfl(incl, 63);
    if (queued && lm) {
      int pos = qbase;
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (lm & (1u << i)) lq.meta[pos++] = uint32_t(lane) | uint32_t(i) << 6 | uint32_t(ow[i]) << 11;
    }
  }
  real f[NC][Q];
  // 4-byte values: every load of the node leaves at once (8-byte values
  // gather after the pseudo-potential sums, below)
  if constexpr (sizeof(real) == 4) {
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int i = 0; i < Q; ++i) f[k][i] = ld32(fin + (size_t(k) * Q + i) * N, nb.pull(i));
  }

  // Shan-Chen acceleration a_k = -G s sum_i w_i psi_kbar(n + c_i) c_i + g; the
  // rho0 part of psi cancels because every neighbour of a fluid node is fluid
  // or a frontier solid carrying a virtual density. Summed over pairs of
  // opposite directions, axis (w = 1/18) and diagonal (w = 1/36) terms apart.
  real ax[NC], ay[NC], az[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    ax[k] = real(a.g[0]);
    ay[k] = real(a.g[1]);
    az[k] = real(a.g[2]);
  }
  if (NC == 2) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const real* pk = psi + size_t(NC - 1 - k) * N;
      real s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0};
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        if (OPP[i] < i) continue;
        const real p = ld32(pk, nb.push(i)) - ld32(pk, nb.pull(i));
        const int c[3] = {CX[i], CY[i], CZ[i]};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (!c[d]) continue;
          if (axis_dir(i)) s1[d] += c[d] > 0 ? p : -p;
          else s2[d] += c[d] > 0 ? p : -p;
        }
      }
      const real gs = real(a.Gs);
      ax[k] -= gs * (real(W1) * s1[0] + real(W2) * s2[0]);
      ay[k] -= gs * (real(W1) * s1[1] + real(W2) * s2[1]);
      az[k] -= gs * (real(W1) * s1[2] + real(W2) * s2[2]);
    }
  }
  if constexpr (sizeof(real) == 8) {
    // 8-byte values: the pseudo-potential sums are complete (the empty asm
    // takes them as inputs and orders memory) before the 38 gathers leave, so
    // the 36 stencil loads and the gathered values are never in flight
    // together: 152 registers instead of 196, three waves per SIMD instead of
    // two (collide 22.58 -> 22.09 ms at 512^3 with 32,000 spheres, 17.99 ->
    // 17.34 ms without spheres, A/B on one box)
#pragma unroll
    for (int k = 0; k < NC; ++k) asm volatile("" ::"v"(ax[k]), "v"(ay[k]), "v"(az[k]) : "memory");
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int i = 0; i < Q; ++i) f[k][i] = ld32(fin + (size_t(k) * Q + i) * N, nb.pull(i));
  }

  // Solid lanes run the same arithmetic and store zeros through the same
  // store instructions as the fluid lanes, into slot 0 and the slots towards
  // solid neighbours; the slots towards fluid neighbours are left to the
  // reflections written by those neighbours. A wave that mixes fluid and
  // solid nodes thus issues every store once.
  const uint32_t smask = !valid ? 0u : (fluid ? 0x7FFFFu : (lmask | 1u));
  if (!fluid) lmask = 0;  // links are walked from fluid nodes only

  real drho[NC], rho[NC], jx[NC], jy[NC], jz[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    // momentum from differences of opposite populations: f_i and f_opp(i)
    // are close, so the differences (and their sums) carry few rounding errors
    real s = f[k][0], j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      s += f[k][i];
      if (OPP[i] < i) continue;
      const real d = f[k][i] - f[k][OPP[i]];
      const int c[3] = {CX[i], CY[i], CZ[i]};
#pragma unroll
      for (int e = 0; e < 3; ++e)
        if (c[e]) j[e] += c[e] > 0 ? d : -d;
    }
    drho[k] = (SOLIDS && !fluid) ? real(0) : s;
    rho[k] = real(a.rho0[k]) + s;
    jx[k] = j[0];
    jy[k] = j[1];
    jz[k] = j[2];
  }
  real ux, uy, uz;
  if (NC == 1) {
    const real ir = real(1) / rho[0];
    ux = jx[0] * ir;
    uy = jy[0] * ir;
    uz = jz[0] * ir;
  } else {
    const real t0 = real(a.inv_tau[0]), t1 = real(a.inv_tau[NC - 1]);
    const real id = real(1) / (rho[0] * t0 + rho[NC - 1] * t1);
    ux = (jx[0] * t0 + jx[NC - 1] * t1) * id;
    uy = (jy[0] * t0 + jy[NC - 1] * t1) * id;
    uz = (jz[0] * t0 + jz[NC - 1] * t1) * id;
  }
  real om;
  if (NC == 1 || a.equal_tau) {
    om = real(a.omega);
  } else {
    // mixture viscosity 1/nu_bar = sum_k (rho_k/rho)/nu_k; omega = 2 cs2/(2 nu_bar + cs2)
    const real rt = rho[0] + rho[NC - 1];
    const real inv_nu = (rho[0] / real(a.nu[0]) + rho[NC - 1] / real(a.nu[NC - 1])) / rt;
    const real nub = real(1) / inv_nu;
    om = real(2.0 / 3.0) / (real(2) * nub + real(1.0 / 3.0));
  }
  // A solid lane relaxes with omega = 0 from zero density deviation, velocity
  // and acceleration: each of its outputs is then 0 * f + 0 (f is a finite
  // value gathered from slots that every step writes), so it stores zeros
  // without a select per output.
  if (SOLIDS && !fluid) {
    ux = uy = uz = real(0);
    om = real(0);
  }
  const real omc = (SOLIDS && !fluid) ? real(0) : real(1) - om;
  const real ouu = omc * (ux * ux + uy * uy + uz * uz);
  // (1 - omega) c.u and (1 - omega)(c.u)^2 per pair, shared by the components
  real ocu[Q], ocu2[Q];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (OPP[i] < i) continue;
    const real cu = cdot(i, ux, uy, uz);
    ocu[i] = omc * cu;
    ocu2[i] = ocu[i] * cu;
  }
  const bool enq = SOLIDS && queued && lmask != 0;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const bool sl = SOLIDS && !fluid;
    const real vx = sl ? real(0) : ux + ax[k], vy = sl ? real(0) : uy + ay[k],
               vz = sl ? real(0) : uz + az[k];
    const real S = om * drho[k] - real(1.5) * rho[k] * ((vx * vx + vy * vy + vz * vz) - ouu);
    const real A = real(4.5) * rho[k], B = real(3) * rho[k];
    const real wS[2] = {real(W1) * S, real(W2) * S};
    const real wA[2] = {real(W1) * A, real(W2) * A};
    const real wB[2] = {real(W1) * B, real(W2) * B};
    real* fk = fout + size_t(k) * Q * N;
    auto put = [&](int i, real v) {
      // with spheres the store is predicated per lane and direction: by an
      // out-of-range offset, without a branch
      if (SOLIDS)
        buf_store(buf_rsrc(fk + size_t(i) * N, N * uint32_t(sizeof(real))),
                  ((smask >> i) & 1u) ? n * uint32_t(sizeof(real)) : kOffNone, v);
      else if (smask & (1u << i))
        st32(fk + size_t(i) * N, n, v);
      if (COUNT && ((smask >> i) & 1u)) atomicAdd(a.counts + (size_t(k) * Q + i) * N + n, 1u);
      // the link's post-collision value, for the lane that will take the link
      if (kDenseLinks<real>) {
        if (SOLIDS) lq.fs[k][i * 64 + lane] = v;
      } else if (enq && (lmask & (1u << i))) {
        lq.fs[k][qbase + __popc(lmask & ((1u << i) - 1u))] = v;
      }
    };
    put(0, omc * f[k][0] + real(1.0 / 3.0) * S);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (OPP[i] < i) continue;
      const int cls = axis_dir(i) ? 0 : 1;
      const real cv = cdot(i, vx, vy, vz);
      const real E = (cv * cv - ocu2[i]) * wA[cls] + wS[cls];
      const real D = (cv - ocu[i]) * wB[cls];
      put(i, omc * f[k][i] + (E + D));
      put(OPP[i], omc * f[k][OPP[i]] + (E - D));
    }
  }
  if (!SOLIDS) return;

  int pid = -1;
  double lv[7] = {0, 0, 0, 0, 0, 0, 0};
  lq.x[lane] = x;
  lq.y[lane] = y;
  lq.z[lane] = z;
#pragma unroll
  for (int k = 0; k < NC; ++k) lq.rho[k][lane] = rho[k];
  lq.u[0][lane] = ux;
  lq.u[1][lane] = uy;
  lq.u[2][lane] = uz;
  // The block's queues form one list: wave w takes its 64-entry chunks w,
  // w + W, ... (W waves per block), so a block's links fill as few waves as
  // they need and the other waves skip the link phase.
  constexpr int WPB = BLOCK / 64;
  __shared__ int qtot[WPB];
  if (lane == 0) qtot[threadIdx.x / 64] = qtotal;
  __syncthreads();
  int pre[WPB + 1];
  pre[0] = 0;
#pragma unroll
  for (int w = 0; w < WPB; ++w) pre[w + 1] = pre[w] + qtot[w];
  const int QB = pre[WPB];
  for (int E = int(threadIdx.x); E < QB; E += BLOCK) {
    int ws = 0;
#pragma unroll
    for (int w = 1; w < WPB; ++w) ws += E >= pre[w] ? 1 : 0;
    const int e = E - pre[ws];
    const LinkQueue<real, NC>& q = lqs[ws];
    const uint32_t m = q.meta[e];
    const int src = int(m & 63u), i = int((m >> 6) & 31u);
    const uint16_t o = uint16_t(m >> 11);
    real fs[NC], rk[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      fs[k] = q.fs[k][kDenseLinks<real> ? i * 64 + src : e];
      rk[k] = q.rho[k][src];
    }
    const real us[3] = {q.u[0][src], q.u[1][src], q.u[2][src]};
    link_one<real, NC, COUNT>(a, i, o, q.x[src], q.y[src], q.z[src], fs, rk, us, pid, lv);
  }
  if (!queued) {
    // past the wave's capacity: this lane walks its own links, reading back
    // the values it has just stored
    while (lmask) {
      const int i = __ffs(lmask) - 1;
      lmask &= lmask - 1u;
      real fs[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) fs[k] = ld32(fout + (size_t(k) * Q + i) * N, n);
      const uint32_t sn = nbr_dyn(x, y, z, dir_c(PCX, i), dir_c(PCY, i), dir_c(PCZ, i), a.nx,
                                  a.ny, a.nz);
      const real un[3] = {ux, uy, uz};
      link_one<real, NC, COUNT>(a, i, ld32(a.owner, sn), x, y, z, fs, rho, un, pid, lv);
    }
  }
  if (a.acc) flush_runs<7>(a.acc, AC_FLIQ, pid, lv);
}

// ---------------------------------------------------------------------------
// Virtual densities of wall frontier nodes (Eq. soliddens): the two wall
// layers take the w-weighted mean of their fluid neighbours.
// ---------------------------------------------------------------------------
template <typename real, int NC>
__global__ void __launch_bounds__(BLOCK)
k_fill_walls(real* __restrict__ psi, const uint16_t* __restrict__ owner, uint32_t nx,
             uint32_t ny, uint32_t nz, double z0a, double z0b, double r0a, double r0b) {
  const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t plane = nx * ny;
  if (t >= 2 * plane) return;
  const uint32_t x = t % nx, y = (t / nx) % ny, z = t < plane ? 0 : nz - 1;
  const uint32_t N = plane * nz;
  const uint32_t n = x + nx * (y + ny * z);
  Nbr nb(x, y, z, nx, ny, nz);
  double wsum = 0, s[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) s[k] = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const uint32_t m = nb.push(i);
    if (owner[m] != 0) continue;
    wsum += WQ[i];
#pragma unroll
    for (int k = 0; k < NC; ++k) s[k] += WQ[i] * double(psi[size_t(k) * N + m]);
  }
  if (wsum == 0.0) return;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double zeta = k == 0 ? z0a : z0b, ref = k == 0 ? r0a : r0b;
    psi[size_t(k) * N + n] = real(zeta * ref + (1.0 + zeta) * s[k] / wsum);
  }
}

// ---------------------------------------------------------------------------
// State transfer: post-streaming populations of the fluid nodes (full values).
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(BLOCK)
k_get_pop(const real* __restrict__ fki, const uint16_t* __restrict__ owner, uint32_t first,
          uint32_t count, uint32_t nx, uint32_t ny, uint32_t nz, int i, double ref,
          double* __restrict__ out) {
  const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
  if (t >= count) return;
  const uint32_t n = first + t;
  if (owner && owner[n] != 0) {
    out[t] = 0.0;
    return;
  }
  uint32_t x, y, z;
  node_xyz(n, nx, ny, x, y, z);
  Nbr nb(x, y, z, nx, ny, nz);
  out[t] = WQ[i] * ref + double(fki[nb.pull(i)]);
}

template <typename real>
__global__ void __launch_bounds__(BLOCK)
k_set_pop(real* __restrict__ fki, const uint16_t* __restrict__ owner, uint32_t first,
          uint32_t count, uint32_t nx, uint32_t ny, uint32_t nz, int i, double ref,
          const double* __restrict__ in) {
  const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
  if (t >= count) return;
  const uint32_t n = first + t;
  if (owner && owner[n] != 0) return;
  uint32_t x, y, z;
  node_xyz(n, nx, ny, x, y, z);
  Nbr nb(x, y, z, nx, ny, nz);
  fki[nb.pull(i)] = real(in[t] - WQ[i] * ref);
}

// Moments of a chunk of nodes: out [ncomp + 3][count] = rho_k, u (0 on solids).
template <typename real>
__global__ void __launch_bounds__(BLOCK)
k_get_fields(const real* __restrict__ f, const uint16_t* __restrict__ owner, uint32_t first,
             uint32_t count, uint32_t nx, uint32_t ny, uint32_t nz, int ncomp, double r0a,
             double r0b, double it0, double it1, double* __restrict__ out) {
  const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
  if (t >= count) return;
  const uint32_t n = first + t, N = nx * ny * nz;
  double rho[2] = {0, 0}, j[2][3] = {{0, 0, 0}, {0, 0, 0}};
  double u[3] = {0, 0, 0};
  if (!owner || owner[n] == 0) {
    uint32_t x, y, z;
    node_xyz(n, nx, ny, x, y, z);
    Nbr nb(x, y, z, nx, ny, nz);
    double num[3] = {0, 0, 0}, den = 0;
    for (int k = 0; k < ncomp; ++k) {
      double s = 0;
      for (int i = 0; i < Q; ++i) {
        const double v = double(f[(size_t(k) * Q + i) * N + nb.pull(i)]);
        s += v;
        j[k][0] += v * CX[i];
        j[k][1] += v * CY[i];
        j[k][2] += v * CZ[i];
      }
      rho[k] = (k == 0 ? r0a : r0b) + s;
      const double it = k == 0 ? it0 : it1;
      for (int c = 0; c < 3; ++c) num[c] += j[k][c] * it;
      den += rho[k] * it;
    }
    for (int c = 0; c < 3; ++c) u[c] = num[c] / den;
  }
  for (int k = 0; k < ncomp; ++k) out[size_t(k) * count + t] = rho[k];
  for (int c = 0; c < 3; ++c) out[size_t(ncomp + c) * count + t] = u[c];
}

template <typename real>
__global__ void __launch_bounds__(BLOCK)
k_get_psi(const real* __restrict__ psi, const uint16_t* __restrict__ owner, uint32_t first,
          uint32_t count, uint32_t nx, uint32_t ny, uint32_t nz, double ref,
          double* __restrict__ out) {
  const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
  if (t >= count) return;
  const uint32_t n = first + t;
  bool valid = true;
  if (owner && owner[n] != 0) {  // solid: valid only on the frontier
    uint32_t x, y, z;
    node_xyz(n, nx, ny, x, y, z);
    Nbr nb(x, y, z, nx, ny, nz);
    valid = false;
    for (int i = 1; i < Q; ++i) valid = valid || owner[nb.push(i)] == 0;
  }
  out[t] = valid ? ref + double(psi[n]) : 0.0;
}

__global__ void k_owner_to_int(const uint16_t* __restrict__ owner, uint32_t first,
                               uint32_t count, int32_t* __restrict__ out) {
  const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
  if (t >= count) return;
  const uint16_t o = owner ? owner[first + t] : 0;
  out[t] = o == OWN_WALL ? -1 : int32_t(o);
}

// ---------------------------------------------------------------------------
// Observables: deterministic two-level FP64 reduction over the fluid nodes.
// partial[b][*]: 0,1 sum drho_k; 2..4 momentum; 5,6 min drho_k; 7,8 max drho_k;
// 9 max |u|; 10 fluid nodes; 11 non-finite count; 12..14 sum over components
// of the force density F_k = -G s rho_k sum_i w_i psi_kbar(n + c_i) c_i + rho_k g
// (Eq. shanchen), from the pseudo-potential of the current state.
// ---------------------------------------------------------------------------
constexpr int RED_USED = 15;
template <typename real>
__global__ void __launch_bounds__(BLOCK)
k_reduce_partials(const real* __restrict__ f, const real* __restrict__ psi,
                  const uint16_t* __restrict__ owner, uint32_t nx, uint32_t ny, uint32_t nz,
                  int ncomp, double r0a, double r0b, double it0, double it1, double Gs, double gx,
                  double gy, double gz, double* __restrict__ partial) {
  const uint32_t N = nx * ny * nz;
  double v[RED_N];
  for (int c = 0; c < RED_N; ++c) v[c] = 0.0;
  v[5] = v[6] = 1e300;
  v[7] = v[8] = -1e300;
  for (uint32_t n = blockIdx.x * BLOCK + threadIdx.x; n < N; n += gridDim.x * BLOCK) {
    if (owner && owner[n] != 0) continue;
    uint32_t x, y, z;
    node_xyz(n, nx, ny, x, y, z);
    Nbr nb(x, y, z, nx, ny, nz);
    double num[3] = {0, 0, 0}, den = 0;
    for (int k = 0; k < ncomp; ++k) {
      double s = 0, j[3] = {0, 0, 0};
      for (int i = 0; i < Q; ++i) {
        const double d = double(f[(size_t(k) * Q + i) * N + nb.pull(i)]);
        s += d;
        j[0] += d * CX[i];
        j[1] += d * CY[i];
        j[2] += d * CZ[i];
      }
      v[k] += s;
      for (int c = 0; c < 3; ++c) v[2 + c] += j[c];
      v[5 + k] = fmin(v[5 + k], s);
      v[7 + k] = fmax(v[7 + k], s);
      if (!isfinite(s)) v[11] += 1.0;
      const double it = k == 0 ? it0 : it1;
      for (int c = 0; c < 3; ++c) num[c] += j[c] * it;
      const double rk = (k == 0 ? r0a : r0b) + s;
      den += rk * it;
      // force density; the psi reference cancels in the stencil because
      // every neighbour of a fluid node is fluid or a frontier solid
      double sc[3] = {0, 0, 0};
      if (ncomp == 2) {
        const real* pk = psi + size_t(1 - k) * N;
        for (int i = 1; i < Q; ++i) {
          const double w = double(pk[nb.push(i)]) * WQ[i];
          sc[0] += w * CX[i];
          sc[1] += w * CY[i];
          sc[2] += w * CZ[i];
        }
      }
      v[12] += rk * (gx - Gs * sc[0]);
      v[13] += rk * (gy - Gs * sc[1]);
      v[14] += rk * (gz - Gs * sc[2]);
    }
    const double ux = num[0] / den, uy = num[1] / den, uz = num[2] / den;
    v[9] = fmax(v[9], sqrt(ux * ux + uy * uy + uz * uz));
    v[10] += 1.0;
  }
  __shared__ double sh[BLOCK];
  for (int c = 0; c < RED_USED; ++c) {
    sh[threadIdx.x] = v[c];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        const double o = sh[threadIdx.x + s];
        double& m = sh[threadIdx.x];
        if (c == 5 || c == 6) m = fmin(m, o);
        else if (c == 7 || c == 8 || c == 9) m = fmax(m, o);
        else m += o;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[size_t(blockIdx.x) * RED_N + c] = sh[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(BLOCK) k_reduce_final(const double* __restrict__ partial,
                                                        int nb, double* __restrict__ out) {
  __shared__ double sh[BLOCK];
  for (int c = 0; c < RED_USED; ++c) {
    double acc = (c == 5 || c == 6) ? 1e300 : (c == 7 || c == 8 || c == 9) ? -1e300 : 0.0;
    for (int b = threadIdx.x; b < nb; b += BLOCK) {
      const double o = partial[size_t(b) * RED_N + c];
      if (c == 5 || c == 6) acc = fmin(acc, o);
      else if (c == 7 || c == 8 || c == 9) acc = fmax(acc, o);
      else acc += o;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        const double o = sh[threadIdx.x + s];
        double& m = sh[threadIdx.x];
        if (c == 5 || c == 6) m = fmin(m, o);
        else if (c == 7 || c == 8 || c == 9) m = fmax(m, o);
        else m += o;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline bool fp64(const lb_ctx* c) { return c->geo.prec == LB_FP64; }

hipError_t launch_init_populations(lb_ctx* c, const double* rho0, const double* u0,
                                   uint32_t first, uint32_t count) {
  const auto& g = c->geo;
  const uint16_t* own = c->has_solids ? static_cast<const uint16_t*>(c->B.owner[c->own_old]) : nullptr;
  if (fp64(c))
    hipLaunchKernelGGL(k_init<double>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<double*>(c->B.f[c->cur]), rho0, u0, own, first, count,
                       g.nx, g.ny, g.nz, g.ncomp, c->P.rho0[0], c->P.rho0[1]);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<float*>(c->B.f[c->cur]), rho0, u0, own, first, count,
                       g.nx, g.ny, g.nz, g.ncomp, c->P.rho0[0], c->P.rho0[1]);
  return hipGetLastError();
}

template <typename real>
static void density_t(lb_ctx* c, const void* f) {
  const auto& g = c->geo;
  const uint32_t bpx = (nblocks(g.N) + 7) / 8;
  const real* fr = static_cast<const real*>(f);
  real* psi = static_cast<real*>(c->B.rho);
  if (g.ncomp == 2)
    hipLaunchKernelGGL((k_density<real, 2>), dim3(8u * bpx), dim3(BLOCK), 0, c->stream, fr, psi,
                       g.nx, g.ny, g.nz, bpx);
  else
    hipLaunchKernelGGL((k_density<real, 1>), dim3(8u * bpx), dim3(BLOCK), 0, c->stream, fr, psi,
                       g.nx, g.ny, g.nz, bpx);
}

hipError_t launch_density(lb_ctx* c, const void* f) {
  if (fp64(c)) density_t<double>(c, f);
  else density_t<float>(c, f);
  return hipGetLastError();
}

template <typename real, int NC>
static void collide_t(lb_ctx* c, const CollideArgs& a) {
  dim3 grid(8u * a.blocks_per_xcd);
  if (c->has_solids && a.counts)
    hipLaunchKernelGGL((k_collide<real, NC, true, true>), grid, dim3(BLOCK), 0, c->stream, a);
  else if (c->has_solids)
    hipLaunchKernelGGL((k_collide<real, NC, true>), grid, dim3(BLOCK), 0, c->stream, a);
  else
    hipLaunchKernelGGL((k_collide<real, NC, false>), grid, dim3(BLOCK), 0, c->stream, a);
}

hipError_t launch_collide(lb_ctx* c, const void* fin, void* fout, const uint16_t* owner,
                          bool forces) {
  const auto& g = c->geo;
  const auto& P = c->P;
  CollideArgs a;
  a.fin = fin;
  a.fout = fout;
  a.psi = c->B.rho;
  a.owner = owner;
  a.ps = c->nparticles ? pstate(c) : nullptr;
  a.acc = (c->nparticles && forces) ? pacc(c) : nullptr;
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.N = g.N;
  a.Gs = P.G * P.sc_norm;
  for (int d = 0; d < 3; ++d) {
    a.g[d] = P.g[d];
    a.wall_lo[d] = P.wall_u_lo[d];
    a.wall_hi[d] = P.wall_u_hi[d];
  }
  for (int f = 0; f < 2; ++f) {
    a.wall_type[f] = P.walls ? P.wall_type[f] : 0;
    for (int k = 0; k < 2; ++k) a.wall_rho[f][k] = P.wall_rho[f][k];
  }
  a.ubnd = reinterpret_cast<const double*>(wptr(c, c->wl.ubnd));
  a.counts = forces ? c->write_counts : nullptr;  // not during the adjoint's recomputation
  a.L[0] = g.nx;
  a.L[1] = g.ny;
  a.L[2] = g.nz;
  for (int d = 0; d < 3; ++d) a.invL[d] = 1.0 / a.L[d];
  a.nblk = nblocks(g.N);
  a.blocks_per_xcd = (a.nblk + 7) / 8;
  // bands of at most kBandTarget workgroups per z-plane (the largest width
  // that divides the plane), when whole workgroups tile a z-plane; otherwise
  // plain plane order
  a.band_w = 0;
  a.plane_w = 0;
  if ((uint64_t(g.nx) * g.ny) % BLOCK == 0) {
    a.plane_w = uint32_t(uint64_t(g.nx) * g.ny / BLOCK);
    for (uint32_t w = std::min(kBandTarget, a.plane_w); w >= 1; --w)
      if (a.plane_w % w == 0) {
        a.band_w = w;
        break;
      }
  }
  const int kb = g.ncomp == 2 ? 1 : 0;
  a.rho0[0] = P.rho0[0];
  a.rho0[1] = P.rho0[kb];
  a.inv_tau[0] = 1.0 / P.tau[0];
  a.inv_tau[1] = 1.0 / P.tau[kb];
  a.nu[0] = (P.tau[0] - 0.5) / 3.0;
  a.nu[1] = (P.tau[kb] - 0.5) / 3.0;
  a.equal_tau = P.tau[0] == P.tau[kb];
  a.omega = 1.0 / P.tau[0];
  if (fp64(c)) {
    if (g.ncomp == 2) collide_t<double, 2>(c, a);
    else collide_t<double, 1>(c, a);
  } else {
    if (g.ncomp == 2) collide_t<float, 2>(c, a);
    else collide_t<float, 1>(c, a);
  }
  return hipGetLastError();
}

bool has_pressure_face(const lb_params& p) {
  return p.walls && (p.wall_type[0] == 1 || p.wall_type[1] == 1);
}

// Mixture velocity (Eq. scvel) of the nodes one layer inside each face layer,
// z = 2 and z = nz - 3, from the populations of the step (node events done).
template <typename real>
__global__ void __launch_bounds__(BLOCK)
k_face_velocity(const real* __restrict__ f, uint32_t nx, uint32_t ny, uint32_t nz, int ncomp,
                double r0a, double r0b, double it0, double it1, double* __restrict__ ubnd) {
  const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t plane = nx * ny;
  if (t >= 2 * plane) return;
  const int face = t < plane ? 0 : 1;
  const uint32_t xy = t - face * plane, x = xy % nx, y = xy / nx;
  const uint32_t z = face == 0 ? 2 : nz - 3;
  const uint32_t N = plane * nz;
  Nbr nb(x, y, z, nx, ny, nz);
  double num[3] = {0, 0, 0}, den = 0;
  for (int k = 0; k < ncomp; ++k) {
    double s = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      const double v = double(f[(size_t(k) * Q + i) * N + nb.pull(i)]);
      s += v;
      j[0] += v * CX[i];
      j[1] += v * CY[i];
      j[2] += v * CZ[i];
    }
    const double it = k == 0 ? it0 : it1;
    for (int d = 0; d < 3; ++d) num[d] += j[d] * it;
    den += ((k == 0 ? r0a : r0b) + s) * it;
  }
  for (int d = 0; d < 3; ++d) ubnd[size_t(t) * 3 + d] = num[d] / den;
}

hipError_t launch_face_velocity(lb_ctx* c, const void* f) {
  const auto& g = c->geo;
  const auto& P = c->P;
  const int kb = g.ncomp == 2 ? 1 : 0;
  double* ub = reinterpret_cast<double*>(wptr(c, c->wl.ubnd));
  const dim3 grid(nblocks(2ull * g.nx * g.ny));
  if (fp64(c))
    hipLaunchKernelGGL(k_face_velocity<double>, grid, dim3(BLOCK), 0, c->stream,
                       static_cast<const double*>(f), g.nx, g.ny, g.nz, g.ncomp, P.rho0[0],
                       P.rho0[kb], 1.0 / P.tau[0], 1.0 / P.tau[kb], ub);
  else
    hipLaunchKernelGGL(k_face_velocity<float>, grid, dim3(BLOCK), 0, c->stream,
                       static_cast<const float*>(f), g.nx, g.ny, g.nz, g.ncomp, P.rho0[0],
                       P.rho0[kb], 1.0 / P.tau[0], 1.0 / P.tau[kb], ub);
  return hipGetLastError();
}

hipError_t launch_fill_walls(lb_ctx* c, const uint16_t* owner) {
  const auto& g = c->geo;
  const auto& P = c->P;
  dim3 grid(nblocks(2ull * g.nx * g.ny));
  const double z1 = g.ncomp == 2 ? P.zeta[1] : 0.0, r1 = g.ncomp == 2 ? P.rho0[1] : 0.0;
  if (fp64(c)) {
    if (g.ncomp == 2)
      hipLaunchKernelGGL((k_fill_walls<double, 2>), grid, dim3(BLOCK), 0, c->stream,
                         static_cast<double*>(c->B.rho), owner, g.nx, g.ny, g.nz, P.zeta[0], z1, P.rho0[0], r1);
    else
      hipLaunchKernelGGL((k_fill_walls<double, 1>), grid, dim3(BLOCK), 0, c->stream,
                         static_cast<double*>(c->B.rho), owner, g.nx, g.ny, g.nz, P.zeta[0], z1, P.rho0[0], r1);
  } else {
    if (g.ncomp == 2)
      hipLaunchKernelGGL((k_fill_walls<float, 2>), grid, dim3(BLOCK), 0, c->stream,
                         static_cast<float*>(c->B.rho), owner, g.nx, g.ny, g.nz, P.zeta[0], z1, P.rho0[0], r1);
    else
      hipLaunchKernelGGL((k_fill_walls<float, 1>), grid, dim3(BLOCK), 0, c->stream,
                         static_cast<float*>(c->B.rho), owner, g.nx, g.ny, g.nz, P.zeta[0], z1, P.rho0[0], r1);
  }
  return hipGetLastError();
}

static const uint16_t* cur_owner(lb_ctx* c) {
  return c->has_solids ? static_cast<const uint16_t*>(c->B.owner[c->own_old]) : nullptr;
}

hipError_t launch_get_populations(lb_ctx* c, int k, int i, uint32_t first, uint32_t count,
                                  double* out) {
  const auto& g = c->geo;
  const size_t off = (size_t(k) * Q + i) * g.N;
  if (fp64(c))
    hipLaunchKernelGGL(k_get_pop<double>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<const double*>(c->B.f[c->cur]) + off, cur_owner(c), first, count,
                       g.nx, g.ny, g.nz, i, c->P.rho0[k], out);
  else
    hipLaunchKernelGGL(k_get_pop<float>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<const float*>(c->B.f[c->cur]) + off, cur_owner(c), first, count,
                       g.nx, g.ny, g.nz, i, c->P.rho0[k], out);
  return hipGetLastError();
}

hipError_t launch_set_populations(lb_ctx* c, int k, int i, uint32_t first, uint32_t count,
                                  const double* in) {
  const auto& g = c->geo;
  const size_t off = (size_t(k) * Q + i) * g.N;
  if (fp64(c))
    hipLaunchKernelGGL(k_set_pop<double>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<double*>(c->B.f[c->cur]) + off, cur_owner(c), first, count,
                       g.nx, g.ny, g.nz, i, c->P.rho0[k], in);
  else
    hipLaunchKernelGGL(k_set_pop<float>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<float*>(c->B.f[c->cur]) + off, cur_owner(c), first, count,
                       g.nx, g.ny, g.nz, i, c->P.rho0[k], in);
  return hipGetLastError();
}

hipError_t launch_get_fields(lb_ctx* c, uint32_t first, uint32_t count, double* out) {
  const auto& g = c->geo;
  const auto& P = c->P;
  const int kb = g.ncomp == 2 ? 1 : 0;
  if (fp64(c))
    hipLaunchKernelGGL(k_get_fields<double>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<const double*>(c->B.f[c->cur]), cur_owner(c), first, count,
                       g.nx, g.ny, g.nz, g.ncomp, P.rho0[0], P.rho0[kb], 1.0 / P.tau[0],
                       1.0 / P.tau[kb], out);
  else
    hipLaunchKernelGGL(k_get_fields<float>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<const float*>(c->B.f[c->cur]), cur_owner(c), first, count,
                       g.nx, g.ny, g.nz, g.ncomp, P.rho0[0], P.rho0[kb], 1.0 / P.tau[0],
                       1.0 / P.tau[kb], out);
  return hipGetLastError();
}

hipError_t launch_get_psi(lb_ctx* c, uint32_t first, uint32_t count, int comp, double* out) {
  const auto& g = c->geo;
  const size_t off = size_t(comp) * g.N;
  if (fp64(c))
    hipLaunchKernelGGL(k_get_psi<double>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<const double*>(c->B.rho) + off, cur_owner(c), first, count,
                       g.nx, g.ny, g.nz, c->P.rho0[comp], out);
  else
    hipLaunchKernelGGL(k_get_psi<float>, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream,
                       static_cast<const float*>(c->B.rho) + off, cur_owner(c), first, count,
                       g.nx, g.ny, g.nz, c->P.rho0[comp], out);
  return hipGetLastError();
}

hipError_t launch_owner_to_int(lb_ctx* c, const uint16_t* owner, uint32_t first,
                               uint32_t count, int32_t* out) {
  hipLaunchKernelGGL(k_owner_to_int, dim3(nblocks(count)), dim3(BLOCK), 0, c->stream, owner,
                     first, count, out);
  return hipGetLastError();
}

int reduce_blocks(const lb_ctx* c) { return int(std::min<uint64_t>(RED_BLOCKS, nblocks(c->geo.N))); }

hipError_t launch_reduce(lb_ctx* c, double* partial, double* out_dev) {
  const auto& g = c->geo;
  const auto& P = c->P;
  const int kb = g.ncomp == 2 ? 1 : 0;
  const int nb = reduce_blocks(c);
  const double Gs = P.G * P.sc_norm;
  if (fp64(c))
    hipLaunchKernelGGL(k_reduce_partials<double>, dim3(nb), dim3(BLOCK), 0, c->stream,
                       static_cast<const double*>(c->B.f[c->cur]),
                       static_cast<const double*>(c->B.rho), cur_owner(c), g.nx, g.ny, g.nz,
                       g.ncomp, P.rho0[0], P.rho0[kb], 1.0 / P.tau[0], 1.0 / P.tau[kb], Gs,
                       P.g[0], P.g[1], P.g[2], partial);
  else
    hipLaunchKernelGGL(k_reduce_partials<float>, dim3(nb), dim3(BLOCK), 0, c->stream,
                       static_cast<const float*>(c->B.f[c->cur]),
                       static_cast<const float*>(c->B.rho), cur_owner(c), g.nx, g.ny, g.nz,
                       g.ncomp, P.rho0[0], P.rho0[kb], 1.0 / P.tau[0], 1.0 / P.tau[kb], Gs,
                       P.g[0], P.g[1], P.g[2], partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(BLOCK), 0, c->stream, partial, nb, out_dev);
  return hipGetLastError();
}


}  // namespace lbh
