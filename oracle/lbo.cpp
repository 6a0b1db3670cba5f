// lbo.cpp -- reference oracle (TEST INFRASTRUCTURE ONLY).
//
// Plain, serial, FP64 implementation of the LBsoft time step for two
// Shan-Chen fluid components and rigid spheres, written from Sec. 2 of
// Bonaccorso et al. (arXiv 2004.04080) and the eight-step sequence of
// Sec. 3.1. It is slow on purpose: every step of the method is a separate
// loop over the whole box, in the paper's order, on full (not deviation)
// populations, with compensated (Neumaier) sums wherever many terms of both
// signs are added (the loss-of-significance remark of Sec. 3.1).
//
// Readings of the paper where it is silent, garbled or inconsistent are
// marked READING and listed in the design notes of the repository.
//
// Nothing here is shared with the HIP implementation. Only tests, the smoke
// check and the benchmark's CPU-baseline leg may load this library.

#include "lbo.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Scalar types: double for ordinary runs, Dual for forward-mode derivatives.
// ---------------------------------------------------------------------------
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() = default;
  Dual(double a) : v(a), d(0.0) {}  // NOLINT: implicit on purpose
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
inline Dual& operator-=(Dual& a, Dual b) { return a = a - b; }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }

// Neumaier's compensated summation.
template <class T>
struct NSum {
  T s = 0.0, c = 0.0;
  void add(T x) {
    T t = s + x;
    if (std::fabs(val(s)) >= std::fabs(val(x)))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  T get() const { return s + c; }
  void clear() { s = 0.0; c = 0.0; }
};

// ---------------------------------------------------------------------------
// D3Q19 lattice (Sec. 2.1): the rest vector, the six first neighbours and the
// twelve second neighbours; weights 1/3, 1/18, 1/36; c_s^2 = 1/3.
// The paper's numbering figure is not available; this order is the oracle's.
// ---------------------------------------------------------------------------
const int Q = 19;
const int CV[Q][3] = {{0, 0, 0},                                          //
                      {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},     //
                      {0, 0, 1},  {0, 0, -1},                             //
                      {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},    //
                      {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},    //
                      {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
const double WT[Q] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                      1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
const double CS2 = 1.0 / 3.0;

int find_opposite(int i) {
  for (int j = 0; j < Q; ++j)
    if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2]) return j;
  return -1;
}
struct OppTable {
  int o[Q];
  OppTable() {
    for (int i = 0; i < Q; ++i) o[i] = find_opposite(i);
  }
};
// index of the direction -c_i
inline int opposite(int i) {
  static const OppTable t;
  return t.o[i];
}

// Second-order equilibrium (Eq. LEQ): w_i rho (1 + u_i + q_i/2) with the
// dipole u_i = c_i.u / c_s^2 and quadrupole q_i = (c_ia c_ib - c_s^2 d_ab) u_a u_b / c_s^4.
template <class T>
T feq(int i, T rho, const T u[3]) {
  T cu = u[0] * double(CV[i][0]) + u[1] * double(CV[i][1]) + u[2] * double(CV[i][2]);
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  T dip = cu / CS2;
  T quad = (cu * cu - uu * CS2) / (CS2 * CS2);
  return rho * WT[i] * (1.0 + dip + quad * 0.5);
}

inline double minimg(double d, double L) { return d - L * std::nearbyint(d / L); }
inline double wrapc(double x, double L) {
  double r = std::fmod(x, L);
  if (r < 0) r += L;
  if (r >= L) r -= L;
  return r;
}
inline void cross(const double a[3], const double b[3], double out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

struct Particle {
  double x[3], v[3], w[3], q[4];
  double Fprev[3], Tprev[3];
  bool have_prev = false;
  // accumulators of the step in progress
  NSum<double> Fliq[3], Tliq[3], Fd[3], Td[3], Fc[3], Tc[3], FSC[3], TSC[3], flabs;
  double FH[3];
  // values of the last completed step (reported)
  double last[31];
};

// ---------------------------------------------------------------------------
// The simulation state. T is the type of the fluid fields.
// ---------------------------------------------------------------------------
template <class T>
struct Sim {
  lbo_params P;
  int64_t N = 0;
  int K = 1;
  T G = 0.0;
  T g[3] = {0.0, 0.0, 0.0};
  std::vector<T> f;         // [k][i][n], post-streaming populations f(t)
  std::vector<int> own;     // map of the previous step M_{t-1}
  std::vector<int32_t> nb;  // [n][i] neighbour node n + c_i (periodic wrap)
  std::vector<Particle> parts;
  double mass = 0.0, inertia = 0.0;
  int64_t tstep = 0;
  double ledger[16] = {0};  // observables 16..31 of the last step
  std::vector<T> fs, refl, fn;  // per-step work arrays [k][i][n]

  T& F(int k, int i, int64_t n) { return f[(int64_t(k) * Q + i) * N + n]; }
  int cx(int64_t n) const { return int(n % P.nx); }
  int cy(int64_t n) const { return int((n / P.nx) % P.ny); }
  int cz(int64_t n) const { return int(n / (int64_t(P.nx) * P.ny)); }
  int64_t idx(int x, int y, int z) const {
    x = ((x % P.nx) + P.nx) % P.nx;
    y = ((y % P.ny) + P.ny) % P.ny;
    z = ((z % P.nz) + P.nz) % P.nz;
    return x + int64_t(P.nx) * (y + int64_t(P.ny) * z);
  }
  bool is_wall_layer(int z) const { return P.walls && (z == 0 || z == P.nz - 1); }

  void setup(const lbo_params& p) {
    P = p;
    K = P.ncomp;
    N = int64_t(P.nx) * P.ny * P.nz;
    G = P.G;
    for (int a = 0; a < 3; ++a) g[a] = P.g[a];
    f.assign(size_t(K) * Q * N, T(0.0));
    own.assign(N, 0);
    nb.resize(size_t(N) * Q);
    for (int64_t n = 0; n < N; ++n) {
      for (int i = 0; i < Q; ++i)
        nb[n * Q + i] = int32_t(idx(cx(n) + CV[i][0], cy(n) + CV[i][1], cz(n) + CV[i][2]));
      if (is_wall_layer(cz(n))) own[n] = -1;
    }
    const double R = P.radius;
    mass = P.particle_density * 4.0 / 3.0 * M_PI * R * R * R;
    inertia = 0.4 * mass * R * R;
  }

  // Initial populations f_i = f_eq(rho0, u0) (u0 = 0 when absent).
  void init_fields(const T* rho0, const double* u0) {
    for (int64_t n = 0; n < N; ++n) {
      if (own[n] != 0) continue;
      T u[3] = {0.0, 0.0, 0.0};
      if (u0)
        for (int a = 0; a < 3; ++a) u[a] = u0[n * 3 + a];
      for (int k = 0; k < K; ++k)
        for (int i = 0; i < Q; ++i) F(k, i, n) = feq<T>(i, rho0[int64_t(k) * N + n], u);
    }
  }

  // Staircase spheres (Sec. 2.4): node n belongs to sphere p when its
  // minimum-image distance from the centre is strictly below R; the lowest
  // particle index wins where spheres overlap; wall layers stay walls.
  void raster(std::vector<int>& M) const {
    for (int64_t n = 0; n < N; ++n) M[n] = is_wall_layer(cz(n)) ? -1 : 0;
    const double R = P.radius, R2 = R * R;
    const double L[3] = {double(P.nx), double(P.ny), double(P.nz)};
    for (size_t p = 0; p < parts.size(); ++p) {
      const double* x = parts[p].x;
      int lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        lo[a] = int(std::floor(x[a] - R));
        hi[a] = int(std::ceil(x[a] + R));
      }
      for (int zz = lo[2]; zz <= hi[2]; ++zz)
        for (int yy = lo[1]; yy <= hi[1]; ++yy)
          for (int xx = lo[0]; xx <= hi[0]; ++xx) {
            int64_t n = idx(xx, yy, zz);
            if (M[n] != 0) continue;
            double d[3] = {minimg(cx(n) - x[0], L[0]), minimg(cy(n) - x[1], L[1]),
                           minimg(cz(n) - x[2], L[2])};
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < R2) M[n] = int(p) + 1;
          }
    }
  }

  void sep(int64_t n, const double* xp, double d[3]) const {
    d[0] = minimg(cx(n) - xp[0], P.nx);
    d[1] = minimg(cy(n) - xp[1], P.ny);
    d[2] = minimg(cz(n) - xp[2], P.nz);
  }

  // Hertz contact (Eq. hertzpot). READING: repulsive, with onset distance d0
  // and the force held constant below the capping distance rcap:
  // |F| = 5/2 K (d0 - max(r, rcap))^(3/2).
  double hertz_mag(double r) const {
    if (r >= P.hertz_d0) return 0.0;
    double h = P.hertz_d0 - std::max(r, P.hertz_rcap);
    return 2.5 * P.hertz_K * h * std::sqrt(h);
  }

  void hertz() {
    const double L[3] = {double(P.nx), double(P.ny), double(P.nz)};
    for (auto& pp : parts)
      for (int a = 0; a < 3; ++a) pp.FH[a] = 0.0;
    for (size_t p = 0; p < parts.size(); ++p)
      for (size_t q = p + 1; q < parts.size(); ++q) {
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = minimg(parts[q].x[a] - parts[p].x[a], L[a]);
        double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double mag = hertz_mag(r);
        if (mag != 0.0)
          for (int a = 0; a < 3; ++a) {
            parts[p].FH[a] -= mag * d[a] / r;
            parts[q].FH[a] += mag * d[a] / r;
          }
        // Lubrication (Eq. libric). READING: the printed scalar acts along the
        // unit vector r_pq / |r_pq| (r_pq = x_q - x_p), with the coefficient
        // lub_mu in place of the viscosity and the gap held at lub_hcap below
        // it; velocities at t - 1/2 (the latest known). It resists the
        // relative motion along the line of centres.
        const double h = r - 2.0 * P.radius;
        if (P.lub_mu > 0.0 && h < P.lub_hn) {
          const double he = std::max(h, P.lub_hcap);
          double vn = 0.0;
          for (int a = 0; a < 3; ++a) vn += (parts[p].v[a] - parts[q].v[a]) * d[a] / r;
          const double fl = -6.0 * M_PI * P.lub_mu * 0.25 * P.radius * P.radius *
                            (1.0 / he - 1.0 / P.lub_hn) * vn;
          for (int a = 0; a < 3; ++a) {
            parts[p].FH[a] += fl * d[a] / r;
            parts[q].FH[a] -= fl * d[a] / r;
          }
        }
      }
    // READING: with walls, each wall plane (halfway between the wall layer and
    // the first fluid layer) pushes a sphere like a mirror image sphere.
    if (P.walls) {
      const double zlo = 0.5, zhi = P.nz - 1.5;
      for (auto& pp : parts) {
        pp.FH[2] += hertz_mag(2.0 * (pp.x[2] - zlo));
        pp.FH[2] -= hertz_mag(2.0 * (zhi - pp.x[2]));
      }
    }
  }

  // Quaternion rotation matrix R(q) (space = R body) and the time derivative
  // q' = 1/2 Q(q) [0, w*] with w* = R^T w the body-frame angular velocity.
  static void qdot(const double q[4], const double w[3], double out[4]) {
    const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
    double Rm[3][3] = {{q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3, 2 * (q1 * q2 - q0 * q3),
                        2 * (q1 * q3 + q0 * q2)},
                       {2 * (q1 * q2 + q0 * q3), q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3,
                        2 * (q2 * q3 - q0 * q1)},
                       {2 * (q1 * q3 - q0 * q2), 2 * (q2 * q3 + q0 * q1),
                        q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3}};
    double ws[3];
    for (int a = 0; a < 3; ++a) ws[a] = Rm[0][a] * w[0] + Rm[1][a] * w[1] + Rm[2][a] * w[2];
    const double Qm[4][4] = {{q0, -q1, -q2, -q3}, {q1, q0, -q3, q2}, {q2, q3, q0, -q1},
                             {q3, -q2, q1, q0}};
    const double v4[4] = {0.0, ws[0], ws[1], ws[2]};
    for (int r = 0; r < 4; ++r) {
      double s = 0.0;
      for (int c = 0; c < 4; ++c) s += Qm[r][c] * v4[c];
      out[r] = 0.5 * s;
    }
  }

  // Rotational leap-frog with Svanberg's implicit mid-step quaternion
  // (Eq. lf, quatder, svanimpl). READING: start from q(t) + q'(q(t))/2,
  // iterate to |delta q'|_inf <= 1e-14 (at most 50 times), normalise q(t+1).
  static void rotate_q(double q[4], const double w[3]) {
    double qd[4], qh[4], qn[4];
    qdot(q, w, qd);
    for (int c = 0; c < 4; ++c) qh[c] = q[c] + 0.5 * qd[c];
    for (int it = 0; it < 50; ++it) {
      qdot(qh, w, qn);
      double diff = 0.0;
      for (int c = 0; c < 4; ++c) diff = std::max(diff, std::fabs(qn[c] - qd[c]));
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
    nrm = std::sqrt(nrm);
    for (int c = 0; c < 4; ++c) q[c] /= nrm;
  }

  // S1 quantities on the fluid nodes of map M: rho_k, j_k and the mixture
  // velocity u = sum_k j_k/tau_k / sum_k rho_k/tau_k (Eq. rho, vel, scvel).
  void moments(const std::vector<int>& M, std::vector<T>& rho, std::vector<T>& j,
               std::vector<T>& u) {
    rho.assign(size_t(K) * N, T(0.0));
    j.assign(size_t(K) * N * 3, T(0.0));
    u.assign(size_t(N) * 3, T(0.0));
    for (int64_t n = 0; n < N; ++n) {
      if (M[n] != 0) continue;
      T num[3] = {0.0, 0.0, 0.0}, den = 0.0;
      for (int k = 0; k < K; ++k) {
        T r = 0.0, jj[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
          T fi = F(k, i, n);
          r += fi;
          for (int a = 0; a < 3; ++a) jj[a] += fi * double(CV[i][a]);
        }
        rho[int64_t(k) * N + n] = r;
        for (int a = 0; a < 3; ++a) {
          j[(int64_t(k) * N + n) * 3 + a] = jj[a];
          num[a] += jj[a] / P.tau[k];
        }
        den += r / P.tau[k];
      }
      for (int a = 0; a < 3; ++a) u[n * 3 + a] = num[a] / den;
    }
  }

  // S4 (first half): pseudo-potential field psi_k = rho_k on fluid nodes and
  // the virtual density (Eq. soliddens) on solid nodes with a fluid neighbour.
  void fill(const std::vector<int>& M, const std::vector<T>& rho, std::vector<T>& rt) const {
    rt.assign(size_t(K) * N, T(0.0));
    for (int64_t n = 0; n < N; ++n) {
      if (M[n] == 0) {
        for (int k = 0; k < K; ++k) rt[int64_t(k) * N + n] = rho[int64_t(k) * N + n];
        continue;
      }
      double wsum = 0.0;
      for (int i = 1; i < Q; ++i)
        if (M[nb[n * Q + i]] == 0) wsum += WT[i];
      if (wsum == 0.0) continue;
      for (int k = 0; k < K; ++k) {
        T s = 0.0;
        for (int i = 1; i < Q; ++i) {
          int64_t m = nb[n * Q + i];
          if (M[m] == 0) s += rho[int64_t(k) * N + m] * WT[i];
        }
        rt[int64_t(k) * N + n] = (1.0 + zeta_at(M, n, k)) * s / wsum;
      }
    }
  }

  // Wetting constant of a solid node (Eq. soliddens). READING (Janus
  // particles, benchmark input "force shanchen angle/particel"): on a sphere
  // node at angle theta from the sphere's body x axis (first column of R(q)),
  // zeta_A = +janus_zeta[0] S(theta) and zeta_B = -janus_zeta[1] S(theta),
  // S = 2 t^2 (3 - 2t) - 1 with t = clamp((theta0 + width/2 - theta) / width,
  // 0, 1): +1 on the cap around the axis, -1 on the opposite side, a smooth
  // step across the band of the given width around theta0.
  double zeta_at(const std::vector<int>& M, int64_t n, int k) const {
    if (!P.janus || M[n] <= 0) return P.zeta[k];
    const Particle& pp = parts[M[n] - 1];
    const double* q = pp.q;
    const double ax[3] = {q[0] * q[0] + q[1] * q[1] - q[2] * q[2] - q[3] * q[3],
                          2 * (q[1] * q[2] + q[0] * q[3]), 2 * (q[1] * q[3] - q[0] * q[2])};
    double d[3];
    sep(n, pp.x, d);
    const double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double an = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    double c = (d[0] * ax[0] + d[1] * ax[1] + d[2] * ax[2]) / (dn * an);
    c = std::min(1.0, std::max(-1.0, c));
    const double theta = std::acos(c) * 180.0 / M_PI;
    double t = (P.janus_theta0 + 0.5 * P.janus_width - theta) / P.janus_width;
    t = std::min(1.0, std::max(0.0, t));
    const double S = 2.0 * t * t * (3.0 - 2.0 * t) - 1.0;
    return k == 0 ? P.janus_zeta[0] * S : -P.janus_zeta[1] * S;
  }

  // Open face (Sec. 2.2): the population that leaves fluid node n along c_i
  // into the face layer returns along -c_i as
  //   pressure:    -f*_i + 2 w_i rho_w [1 + (u_w.c_i)^2/(2 cs^4) - u_w^2/(2 cs^2)]  (Eq. bbp)
  //   velocity:     f*_i - 2 w_i rho_w (u_w.c_i)/cs^2                                (Eq. bbv)
  //   equilibrium:  f_eq_{-i}(rho_w, u_w)
  // with the given rho_w (pressure, equilibrium) or u_w (velocity,
  // equilibrium) and the other one extrapolated from the fluid:
  // X_w = X(n) + (X(n) - X(n')) / 2, n' the next node inwards along z.
  // READING: if n' is not fluid, X_w = X(n). The mixture velocity u of S1 is
  // extrapolated; densities per component. Momentum and mass that cross the
  // face go into the wall ledgers.
  void open_face(int face, int64_t n, int i, const std::vector<int>& M, const std::vector<T>& rho,
                 const std::vector<T>& u, const std::vector<T>& fs, std::vector<T>& refl,
                 NSum<double>* led_ml, NSum<double>* led_wall) const {
    const int type = P.wall_type[face];
    const double* U = face == 0 ? P.wall_u_lo : P.wall_u_hi;
    const int64_t inner = idx(cx(n), cy(n), cz(n) + (face == 0 ? 1 : -1));
    const bool ok = M[inner] == 0;
    T Fl[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < K; ++k) {
      const T fsi = fs[(int64_t(k) * Q + i) * N + n];
      T r;
      if (type == 1) {
        T uw[3];
        for (int a = 0; a < 3; ++a)
          uw[a] = ok ? u[n * 3 + a] + 0.5 * (u[n * 3 + a] - u[inner * 3 + a]) : u[n * 3 + a];
        const T uc = uw[0] * CV[i][0] + uw[1] * CV[i][1] + uw[2] * CV[i][2];
        const T uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
        r = -fsi + 2.0 * WT[i] * P.wall_rho[face][k] *
                       (1.0 + uc * uc / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
      } else if (type == 2) {
        const T rn = rho[int64_t(k) * N + n];
        const T rw = ok ? rn + 0.5 * (rn - rho[int64_t(k) * N + inner]) : rn;
        const double uc = U[0] * CV[i][0] + U[1] * CV[i][1] + U[2] * CV[i][2];
        r = fsi - 2.0 * WT[i] * rw * uc / CS2;
      } else {
        const T Ut[3] = {U[0], U[1], U[2]};
        r = feq<T>(opposite(i), T(P.wall_rho[face][k]), Ut);
      }
      refl[(int64_t(k) * Q + opposite(i)) * N + n] = r;
      for (int a = 0; a < 3; ++a) Fl[a] += (fsi + r) * double(CV[i][a]);
      led_ml[k].add(val(r - fsi));
    }
    for (int a = 0; a < 3; ++a) led_wall[a].add(val(Fl[a]));
  }

  bool frontier(const std::vector<int>& M, int64_t n) const {
    if (M[n] == 0) return false;
    for (int i = 1; i < Q; ++i)
      if (M[nb[n * Q + i]] == 0) return true;
    return false;
  }

  int step() {
    const bool moving = !parts.empty() && !P.particles_fixed;
    const double L[3] = {double(P.nx), double(P.ny), double(P.nz)};
    for (auto& pp : parts) {
      for (int a = 0; a < 3; ++a) {
        pp.Fliq[a].clear(); pp.Tliq[a].clear(); pp.Fd[a].clear(); pp.Td[a].clear();
        pp.Fc[a].clear(); pp.Tc[a].clear(); pp.FSC[a].clear(); pp.TSC[a].clear();
        pp.FH[a] = 0.0;
      }
      pp.flabs.clear();
    }
    NSum<double> led_md[2], led_mc[2], led_ml[2], led_body[3], led_sc[3], led_wall[3];

    // S1: moments on the fluid nodes of the previous map.
    std::vector<T> rho, j, u;
    moments(own, rho, j, u);

    // S2: new map and the fluid-node destruction / creation events.
    std::vector<int> own_new = own;
    if (moving) {
      for (auto& pp : parts)
        for (int a = 0; a < 3; ++a)
          if (std::fabs(pp.v[a]) > 0.5) return LBO_E_SPEED;
      raster(own_new);
      for (int64_t n = 0; n < N; ++n) {
        int o = own[n], w = own_new[n];
        if (o == 0 && w > 0) {
          // Destruction (Eq. distr): the node's momentum goes to the particle.
          // READING: the bare momentum sum_k j_k (equal to (rho_A+rho_B) u
          // for equal relaxation times).
          Particle& pp = parts[w - 1];
          double d[3], J[3], tq[3];
          sep(n, pp.x, d);
          for (int a = 0; a < 3; ++a) {
            J[a] = 0.0;
            for (int k = 0; k < K; ++k) J[a] += val(j[(int64_t(k) * N + n) * 3 + a]);
          }
          cross(d, J, tq);
          for (int a = 0; a < 3; ++a) {
            pp.Fd[a].add(J[a]);
            pp.Td[a].add(tq[a]);
          }
          for (int k = 0; k < K; ++k) led_md[k].add(val(rho[int64_t(k) * N + n]));
          for (int k = 0; k < K; ++k)
            for (int i = 0; i < Q; ++i) F(k, i, n) = 0.0;
        }
      }
      for (int64_t n = 0; n < N; ++n) {
        int o = own[n], w = own_new[n];
        if (o > 0 && w == 0) {
          // Creation (Eq. creat). READING: densities are the w-weighted mean
          // over the neighbours that are fluid in both maps.
          Particle& pp = parts[o - 1];
          double d[3], uw[3];
          sep(n, pp.x, d);
          cross(pp.w, d, uw);
          for (int a = 0; a < 3; ++a) uw[a] += pp.v[a];
          double wsum = 0.0;
          for (int i = 1; i < Q; ++i) {
            int64_t m = nb[n * Q + i];
            if (own[m] == 0 && own_new[m] == 0) wsum += WT[i];
          }
          T tot = 0.0;
          T ut[3] = {uw[0], uw[1], uw[2]};
          for (int k = 0; k < K; ++k) {
            T rb = P.rho_fallback[k];
            if (wsum > 0.0) {
              T s = 0.0;
              for (int i = 1; i < Q; ++i) {
                int64_t m = nb[n * Q + i];
                if (own[m] == 0 && own_new[m] == 0) s += rho[int64_t(k) * N + m] * WT[i];
              }
              rb = s / wsum;
            }
            for (int i = 0; i < Q; ++i) F(k, i, n) = feq<T>(i, rb, ut);
            rho[int64_t(k) * N + n] = rb;
            for (int a = 0; a < 3; ++a) j[(int64_t(k) * N + n) * 3 + a] = rb * uw[a];
            tot += rb;
            led_mc[k].add(val(rb));
          }
          for (int a = 0; a < 3; ++a) u[n * 3 + a] = uw[a];
          double Pm[3] = {val(tot) * uw[0], val(tot) * uw[1], val(tot) * uw[2]}, tq[3];
          cross(d, Pm, tq);
          for (int a = 0; a < 3; ++a) {
            pp.Fc[a].add(-Pm[a]);
            pp.Tc[a].add(-tq[a]);
          }
        }
      }
      // S3: pair forces.
      hertz();
    }

    // S4: pseudo-potential field with virtual solid densities, the fluid
    // Shan-Chen force (Eq. shanchen) and its reaction on frontier solid nodes
    // (Eq. shanchen2). READING: repulsive sign and the lattice-gradient
    // normalisation F_k = -G sc_norm rho_k sum_i w_i psi_kbar(n+c_i) c_i.
    std::vector<T> rt;
    fill(own_new, rho, rt);
    std::vector<T> acc(size_t(K) * N * 3, T(0.0));  // a_k = F_k / rho_k
    for (int64_t n = 0; n < N; ++n) {
      if (own_new[n] != 0) continue;
      for (int k = 0; k < K; ++k) {
        T s[3] = {0.0, 0.0, 0.0};
        if (K == 2) {
          const int kb = 1 - k;
          for (int i = 1; i < Q; ++i) {
            T r = rt[int64_t(kb) * N + nb[n * Q + i]] * WT[i];
            for (int a = 0; a < 3; ++a) s[a] += r * double(CV[i][a]);
          }
        }
        T rk = rho[int64_t(k) * N + n];
        for (int a = 0; a < 3; ++a) {
          T sc = -(G * P.sc_norm) * s[a];
          acc[(int64_t(k) * N + n) * 3 + a] = sc + g[a];
          led_sc[a].add(val(rk * sc));
          led_body[a].add(val(rk * g[a]));
        }
      }
    }
    if (K == 2) {
      for (int64_t n = 0; n < N; ++n) {
        if (own_new[n] <= 0 || !frontier(own_new, n)) continue;
        Particle& pp = parts[own_new[n] - 1];
        double Fs[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < K; ++k) {
          const int kb = 1 - k;
          double s[3] = {0.0, 0.0, 0.0};
          for (int i = 1; i < Q; ++i) {
            int64_t m = nb[n * Q + i];
            if (own_new[m] != 0) continue;
            for (int a = 0; a < 3; ++a) s[a] += WT[i] * val(rho[int64_t(kb) * N + m]) * CV[i][a];
          }
          for (int a = 0; a < 3; ++a) Fs[a] += -val(G) * P.sc_norm * val(rt[int64_t(k) * N + n]) * s[a];
        }
        double d[3], tq[3];
        sep(n, pp.x, d);
        cross(d, Fs, tq);
        for (int a = 0; a < 3; ++a) {
          pp.FSC[a].add(Fs[a]);
          pp.TSC[a].add(tq[a]);
        }
      }
    }

    // S5: two-component BGK collision with Exact-Difference-Method forcing
    // (Eq. lbsbgk): f* = f_eq(rho_k, u + a_k) + (1 - w_e)(f - f_eq(rho_k, u)).
    // READING: w_e = 2 c_s^2 / (2 nu_bar + c_s^2), the inverse of Eq. viscosity.
    fs.assign(size_t(K) * Q * N, T(0.0));
    for (int64_t n = 0; n < N; ++n) {
      if (own_new[n] != 0) continue;
      T we;
      if (K == 1) {
        we = 1.0 / P.tau[0];
      } else {
        T rtot = rho[n] + rho[N + n];
        T inv_nu = 0.0;
        for (int k = 0; k < 2; ++k) inv_nu += (rho[int64_t(k) * N + n] / rtot) / (CS2 * (P.tau[k] - 0.5));
        T nubar = 1.0 / inv_nu;
        we = 2.0 * CS2 / (2.0 * nubar + CS2);
      }
      const T* un = &u[n * 3];
      for (int k = 0; k < K; ++k) {
        T rk = rho[int64_t(k) * N + n];
        const T* ak = &acc[(int64_t(k) * N + n) * 3];
        T us[3] = {un[0] + ak[0], un[1] + ak[1], un[2] + ak[2]};
        for (int i = 0; i < Q; ++i)
          fs[(int64_t(k) * Q + i) * N + n] =
              feq<T>(i, rk, us) + (1.0 - we) * (F(k, i, n) - feq<T>(i, rk, un));
      }
    }

    // S6: halfway bounce-back at solid links with the moving-wall correction
    // (Eq. LADDFLBE, UPI) and the link momentum exchange (Eq. LADDFORCE).
    // READING: u_w = v_p + w_p x (r_w - x_p) with the particle velocities of
    // the previous half step; rho is the local component density.
    refl.assign(size_t(K) * Q * N, T(0.0));
    for (int64_t n = 0; n < N; ++n) {
      if (own_new[n] != 0) continue;
      for (int i = 1; i < Q; ++i) {
        int64_t s = nb[n * Q + i];
        int o = own_new[s];
        if (o == 0) continue;
        double uw[3], rw[3] = {0.0, 0.0, 0.0};
        Particle* pp = nullptr;
        if (o < 0) {
          const int face = cz(s) == 0 ? 0 : 1;
          const double* U = face == 0 ? P.wall_u_lo : P.wall_u_hi;
          for (int a = 0; a < 3; ++a) uw[a] = U[a];
          if (P.wall_type[face] != 0) {
            open_face(face, n, i, own_new, rho, u, fs, refl, led_ml, led_wall);
            continue;
          }
        } else {
          pp = &parts[o - 1];
          double r[3] = {cx(n) + 0.5 * CV[i][0], cy(n) + 0.5 * CV[i][1], cz(n) + 0.5 * CV[i][2]};
          for (int a = 0; a < 3; ++a) rw[a] = minimg(r[a] - pp->x[a], L[a]);
          cross(pp->w, rw, uw);
          for (int a = 0; a < 3; ++a) uw[a] += pp->v[a];
        }
        double ucw = uw[0] * CV[i][0] + uw[1] * CV[i][1] + uw[2] * CV[i][2];
        T Fl[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < K; ++k) {
          T corr = 2.0 * WT[i] * rho[int64_t(k) * N + n] * ucw / CS2;
          T fsi = fs[(int64_t(k) * Q + i) * N + n];
          refl[(int64_t(k) * Q + opposite(i)) * N + n] = fsi - corr;
          for (int a = 0; a < 3; ++a) Fl[a] += (2.0 * fsi - corr) * double(CV[i][a]);
          led_ml[k].add(-val(corr));
        }
        double Fv[3] = {val(Fl[0]), val(Fl[1]), val(Fl[2])};
        if (pp) {
          double tq[3];
          cross(rw, Fv, tq);
          for (int a = 0; a < 3; ++a) {
            pp->Fliq[a].add(Fv[a]);
            pp->Tliq[a].add(tq[a]);
          }
          pp->flabs.add(std::sqrt(Fv[0] * Fv[0] + Fv[1] * Fv[1] + Fv[2] * Fv[2]));
        } else {
          for (int a = 0; a < 3; ++a) led_wall[a].add(Fv[a]);
        }
      }
    }

    // S7: Newton-Euler update of the spheres, FP64 (Eq. lf with the
    // half-step force average). READING: the Shan-Chen reaction on the solid
    // frontier is part of the total; F_liq(-1/2) := F_liq(+1/2) at the first step.
    for (auto& pp : parts) {
      double Fl[3], Tl[3];
      for (int a = 0; a < 3; ++a) {
        Fl[a] = pp.Fliq[a].get();
        Tl[a] = pp.Tliq[a].get();
      }
      double* last = pp.last;
      for (int a = 0; a < 3; ++a) {
        last[0 + a] = pp.Fd[a].get();
        last[3 + a] = pp.Td[a].get();
        last[6 + a] = pp.Fc[a].get();
        last[9 + a] = pp.Tc[a].get();
        last[12 + a] = pp.FH[a];
        last[15 + a] = pp.FSC[a].get();
        last[18 + a] = pp.TSC[a].get();
        last[21 + a] = Fl[a];
        last[24 + a] = Tl[a];
      }
      last[27] = pp.flabs.get();
      if (!moving) continue;
      if (!pp.have_prev)
        for (int a = 0; a < 3; ++a) {
          pp.Fprev[a] = Fl[a];
          pp.Tprev[a] = Tl[a];
        }
      double Ft[3], Tt[3];
      for (int a = 0; a < 3; ++a) {
        NSum<double> sf, st;
        sf.add(0.5 * (pp.Fprev[a] + Fl[a]));
        sf.add(last[0 + a]);
        sf.add(last[6 + a]);
        sf.add(last[12 + a]);
        sf.add(last[15 + a]);
        st.add(0.5 * (pp.Tprev[a] + Tl[a]));
        st.add(last[3 + a]);
        st.add(last[9 + a]);
        st.add(last[18 + a]);
        Ft[a] = sf.get();
        Tt[a] = st.get();
      }
      for (int a = 0; a < 3; ++a) {
        pp.v[a] += Ft[a] / mass;
        pp.x[a] = wrapc(pp.x[a] + pp.v[a], L[a]);
      }
      if (P.rotate) {
        for (int a = 0; a < 3; ++a) pp.w[a] += Tt[a] / inertia;
        rotate_q(pp.q, pp.w);
      }
      for (int a = 0; a < 3; ++a) {
        pp.Fprev[a] = Fl[a];
        pp.Tprev[a] = Tl[a];
      }
      pp.have_prev = true;
    }

    // S8: pull streaming on the fluid nodes of the new map (Eq. bgk2, bb).
    fn.assign(size_t(K) * Q * N, T(0.0));
    for (int64_t n = 0; n < N; ++n) {
      if (own_new[n] != 0) continue;
      for (int i = 0; i < Q; ++i) {
        int64_t src = nb[n * Q + opposite(i)];  // n - c_i
        for (int k = 0; k < K; ++k) {
          int64_t o = (int64_t(k) * Q + i) * N;
          fn[o + n] = (own_new[src] == 0) ? fs[o + src] : refl[o + n];
        }
      }
    }
    f.swap(fn);
    own.swap(own_new);
    ++tstep;
    for (int k = 0; k < 2; ++k) {
      ledger[0 + k] = led_md[k].get();
      ledger[2 + k] = led_mc[k].get();
      ledger[4 + k] = led_ml[k].get();
    }
    for (int a = 0; a < 3; ++a) {
      ledger[6 + a] = led_body[a].get();
      ledger[9 + a] = led_sc[a].get();
      ledger[12 + a] = led_wall[a].get();
    }
    ledger[15] = double(tstep);
    return LBO_OK;
  }

  // Loss of the differentiation study: L = sum over fluid nodes of
  // |grad phi|^2, phi = psi_A - psi_B, grad = (1/c_s^2) sum_i w_i phi(n+c_i) c_i,
  // evaluated on the current state with the virtual densities of the current map.
  T loss() {
    std::vector<T> rho, j, u, rt;
    moments(own, rho, j, u);
    fill(own, rho, rt);
    NSum<T> L;
    for (int64_t n = 0; n < N; ++n) {
      if (own[n] != 0) continue;
      T gr[3] = {0.0, 0.0, 0.0};
      for (int i = 1; i < Q; ++i) {
        int64_t m = nb[n * Q + i];
        T phi = (K == 2) ? rt[m] - rt[N + m] : rt[m];
        for (int a = 0; a < 3; ++a) gr[a] += phi * (WT[i] * CV[i][a] / CS2);
      }
      L.add(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
    }
    return L.get();
  }

  int add_particles(int n, const double* x, const double* v, const double* w, const double* q) {
    const double L[3] = {double(P.nx), double(P.ny), double(P.nz)};
    for (int p = 0; p < n; ++p) {
      Particle pp;
      for (int a = 0; a < 3; ++a) {
        pp.x[a] = wrapc(x[3 * p + a], L[a]);
        pp.v[a] = v ? v[3 * p + a] : 0.0;
        pp.w[a] = w ? w[3 * p + a] : 0.0;
        pp.Fprev[a] = pp.Tprev[a] = pp.FH[a] = 0.0;
      }
      for (int c = 0; c < 4; ++c) pp.q[c] = q ? q[4 * p + c] : (c == 0 ? 1.0 : 0.0);
      std::fill(pp.last, pp.last + 31, 0.0);
      parts.push_back(pp);
    }
    // Nodes covered by the spheres become solid; their populations are dropped.
    std::vector<int> M(N);
    raster(M);
    for (int64_t m = 0; m < N; ++m)
      if (M[m] != 0 && own[m] == 0)
        for (int k = 0; k < K; ++k)
          for (int i = 0; i < Q; ++i) F(k, i, m) = 0.0;
    own.swap(M);
    return LBO_OK;
  }
};

bool valid(const lbo_params* p) {
  if (!p) return false;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
  if (p->ncomp != 1 && p->ncomp != 2) return false;
  for (int k = 0; k < p->ncomp; ++k)
    if (!(p->tau[k] > 0.5)) return false;
  if (p->walls && p->nz < 3) return false;
  if (p->janus && !(p->janus_width > 0.0)) return false;
  for (int f = 0; f < 2; ++f) {
    if (p->wall_type[f] < 0 || p->wall_type[f] > 3) return false;
    if (p->wall_type[f] != 0 && p->nz < 4) return false;
  }
  if (p->lub_mu < 0.0 || (p->lub_mu > 0.0 && !(p->lub_hn > p->lub_hcap && p->lub_hcap > 0.0)))
    return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface
// ---------------------------------------------------------------------------
extern "C" {

void* lbo_create(const lbo_params* p, const double* rho0, const double* u0) {
  if (!valid(p) || !rho0) return nullptr;
  auto* s = new Sim<double>();
  s->setup(*p);
  s->init_fields(rho0, u0);
  return s;
}

void lbo_destroy(void* s) { delete static_cast<Sim<double>*>(s); }

int lbo_add_particles(void* s, int32_t n, const double* x, const double* v, const double* w,
                      const double* q) {
  auto* S = static_cast<Sim<double>*>(s);
  if (n < 0 || (n > 0 && !x)) return LBO_E_ARG;
  return S->add_particles(n, x, v, w, q);
}

int lbo_step(void* s, int32_t nsteps) {
  auto* S = static_cast<Sim<double>*>(s);
  for (int t = 0; t < nsteps; ++t) {
    int rc = S->step();
    if (rc != LBO_OK) return rc;
  }
  return LBO_OK;
}

void lbo_lattice(int32_t* c, double* w) {
  for (int i = 0; i < Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = CV[i][a];
    w[i] = WT[i];
  }
}

void lbo_get_f(const void* s, double* out) {
  auto* S = static_cast<const Sim<double>*>(s);
  std::memcpy(out, S->f.data(), S->f.size() * sizeof(double));
}

void lbo_set_f(void* s, const double* in) {
  auto* S = static_cast<Sim<double>*>(s);
  std::memcpy(S->f.data(), in, S->f.size() * sizeof(double));
}

void lbo_get_rho(const void* s, double* out) {
  auto* S = const_cast<Sim<double>*>(static_cast<const Sim<double>*>(s));
  std::vector<double> rho, j, u;
  S->moments(S->own, rho, j, u);
  std::memcpy(out, rho.data(), rho.size() * sizeof(double));
}

void lbo_get_psi(const void* s, double* out) {
  auto* S = const_cast<Sim<double>*>(static_cast<const Sim<double>*>(s));
  std::vector<double> rho, j, u, rt;
  S->moments(S->own, rho, j, u);
  S->fill(S->own, rho, rt);
  std::memcpy(out, rt.data(), rt.size() * sizeof(double));
}

void lbo_get_u(const void* s, double* out) {
  auto* S = const_cast<Sim<double>*>(static_cast<const Sim<double>*>(s));
  std::vector<double> rho, j, u;
  S->moments(S->own, rho, j, u);
  std::memcpy(out, u.data(), u.size() * sizeof(double));
}

void lbo_get_owner(const void* s, int32_t* out) {
  auto* S = static_cast<const Sim<double>*>(s);
  for (int64_t n = 0; n < S->N; ++n) out[n] = S->own[n];
}

void lbo_set_owner(void* s, const int32_t* in) {
  auto* S = static_cast<Sim<double>*>(s);
  for (int64_t n = 0; n < S->N; ++n) S->own[n] = in[n];
}

int32_t lbo_num_particles(const void* s) {
  return int32_t(static_cast<const Sim<double>*>(s)->parts.size());
}

void lbo_get_particles(const void* s, double* out) {
  auto* S = static_cast<const Sim<double>*>(s);
  for (size_t p = 0; p < S->parts.size(); ++p) {
    const Particle& pp = S->parts[p];
    double* o = out + p * LBO_PREC;
    for (int a = 0; a < 3; ++a) {
      o[0 + a] = pp.x[a];
      o[3 + a] = pp.v[a];
      o[6 + a] = pp.w[a];
      o[13 + a] = pp.Fprev[a];
      o[16 + a] = pp.Tprev[a];
    }
    for (int c = 0; c < 4; ++c) o[9 + c] = pp.q[c];
    for (int r = 0; r < 28; ++r) o[19 + r] = pp.last[r];
    o[47] = S->mass;
    o[48] = S->inertia;
    o[49] = pp.have_prev ? 1.0 : 0.0;
  }
}

void lbo_set_particle_state(void* s, const double* in) {
  auto* S = static_cast<Sim<double>*>(s);
  for (size_t p = 0; p < S->parts.size(); ++p) {
    Particle& pp = S->parts[p];
    const double* o = in + p * LBO_PREC;
    for (int a = 0; a < 3; ++a) {
      pp.x[a] = o[0 + a];
      pp.v[a] = o[3 + a];
      pp.w[a] = o[6 + a];
      pp.Fprev[a] = o[13 + a];
      pp.Tprev[a] = o[16 + a];
    }
    for (int c = 0; c < 4; ++c) pp.q[c] = o[9 + c];
    pp.have_prev = o[49] != 0.0;
  }
}

void lbo_observables(const void* s, double* out) {
  auto* S = const_cast<Sim<double>*>(static_cast<const Sim<double>*>(s));
  std::vector<double> rho, j, u;
  S->moments(S->own, rho, j, u);
  const int64_t N = S->N;
  NSum<double> mass[2], mom[3];
  double rmin[2] = {1e300, 1e300}, rmax[2] = {-1e300, -1e300}, umax = 0.0;
  int64_t nfl = 0;
  for (int64_t n = 0; n < N; ++n) {
    if (S->own[n] != 0) continue;
    ++nfl;
    for (int k = 0; k < S->K; ++k) {
      double r = rho[int64_t(k) * N + n];
      mass[k].add(r);
      rmin[k] = std::min(rmin[k], r);
      rmax[k] = std::max(rmax[k], r);
      for (int a = 0; a < 3; ++a) mom[a].add(j[(int64_t(k) * N + n) * 3 + a]);
    }
    double uu = std::sqrt(u[n * 3] * u[n * 3] + u[n * 3 + 1] * u[n * 3 + 1] + u[n * 3 + 2] * u[n * 3 + 2]);
    umax = std::max(umax, uu);
  }
  std::fill(out, out + LBO_NOBS, 0.0);
  for (int k = 0; k < S->K; ++k) {
    out[0 + k] = mass[k].get();
    out[5 + k] = rmin[k];
    out[7 + k] = rmax[k];
  }
  for (int a = 0; a < 3; ++a) out[2 + a] = mom[a].get();
  out[9] = umax;
  out[10] = double(nfl);
  NSum<double> pm[3], ke, kr;
  for (auto& pp : S->parts) {
    double v2 = 0.0, w2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      pm[a].add(S->mass * pp.v[a]);
      v2 += pp.v[a] * pp.v[a];
      w2 += pp.w[a] * pp.w[a];
    }
    ke.add(0.5 * S->mass * v2);
    kr.add(0.5 * S->inertia * w2);
  }
  for (int a = 0; a < 3; ++a) out[11 + a] = pm[a].get();
  out[14] = ke.get();
  out[15] = kr.get();
  for (int r = 0; r < 16; ++r) out[16 + r] = S->ledger[r];
  // Physical fluid momentum (Sec. 2.3, the velocity that follows Eq. lbsbgk
  // with the exact-difference forcing): sum_k j_k + F_k / 2 on every fluid
  // node, with the force density F_k of Eq. shanchen (pseudo-potential of the
  // current map, virtual densities on frontier solids) plus rho_k g.
  std::vector<double> rt;
  S->fill(S->own, rho, rt);
  NSum<double> ph[3];
  for (int64_t n = 0; n < N; ++n) {
    if (S->own[n] != 0) continue;
    for (int k = 0; k < S->K; ++k) {
      double s[3] = {0.0, 0.0, 0.0};
      if (S->K == 2)
        for (int i = 1; i < Q; ++i) {
          const double r = rt[int64_t(1 - k) * N + S->nb[n * Q + i]] * WT[i];
          for (int a = 0; a < 3; ++a) s[a] += r * CV[i][a];
        }
      const double rk = rho[int64_t(k) * N + n];
      for (int a = 0; a < 3; ++a) {
        ph[a].add(j[(int64_t(k) * N + n) * 3 + a]);
        ph[a].add(0.5 * (-(S->G * S->P.sc_norm) * rk * s[a] + rk * S->g[a]));
      }
    }
  }
  for (int a = 0; a < 3; ++a) out[32 + a] = ph[a].get();
  // sum over the spheres of sum over links of |F_link| of the last step
  NSum<double> fl;
  for (auto& pp : S->parts) fl.add(pp.last[27]);
  out[35] = fl.get();
}

void lbo_test_rotate(double* q, const double* w, int32_t nsteps) {
  for (int t = 0; t < nsteps; ++t) Sim<double>::rotate_q(q, w);
}

double lbo_loss(const void* s) {
  auto* S = const_cast<Sim<double>*>(static_cast<const Sim<double>*>(s));
  return S->loss();
}

int lbo_loss_tangent(const lbo_params* p, const double* rho0, int32_t np, const double* x,
                     int32_t nsteps, double dG, const double* dg, const double* drhoA,
                     double* L, double* dL) {
  if (!valid(p) || !rho0 || (np > 0 && (!x || !p->particles_fixed))) return LBO_E_ARG;
  Sim<Dual> S;
  S.setup(*p);
  S.G = Dual(p->G, dG);
  for (int a = 0; a < 3; ++a) S.g[a] = Dual(p->g[a], dg ? dg[a] : 0.0);
  std::vector<Dual> r0(size_t(S.K) * S.N);
  for (int64_t m = 0; m < int64_t(r0.size()); ++m) {
    double d = (drhoA && m < S.N) ? drhoA[m] : 0.0;
    r0[m] = Dual(rho0[m], d);
  }
  S.init_fields(r0.data(), nullptr);
  if (np > 0) S.add_particles(np, x, nullptr, nullptr, nullptr);
  for (int t = 0; t < nsteps; ++t) {
    int rc = S.step();
    if (rc != LBO_OK) return rc;
  }
  Dual l = S.loss();
  *L = l.v;
  *dL = l.d;
  return LBO_OK;
}

int lbo_psi_tangent(const lbo_params* p, const double* rho0, int32_t np, const double* x,
                    int32_t nsteps, double dG, const double* dg, const double* drhoA,
                    double* psi, double* dpsi) {
  if (!valid(p) || !rho0 || !psi || !dpsi || (np > 0 && (!x || !p->particles_fixed)))
    return LBO_E_ARG;
  Sim<Dual> S;
  S.setup(*p);
  S.G = Dual(p->G, dG);
  for (int a = 0; a < 3; ++a) S.g[a] = Dual(p->g[a], dg ? dg[a] : 0.0);
  std::vector<Dual> r0(size_t(S.K) * S.N);
  for (int64_t m = 0; m < int64_t(r0.size()); ++m) {
    double d = (drhoA && m < S.N) ? drhoA[m] : 0.0;
    r0[m] = Dual(rho0[m], d);
  }
  S.init_fields(r0.data(), nullptr);
  if (np > 0) S.add_particles(np, x, nullptr, nullptr, nullptr);
  for (int t = 0; t < nsteps; ++t) {
    int rc = S.step();
    if (rc != LBO_OK) return rc;
  }
  // the pseudo-potential of the final state, as the loss sees it
  std::vector<Dual> rho, j, u, rt;
  S.moments(S.own, rho, j, u);
  S.fill(S.own, rho, rt);
  for (size_t m = 0; m < rt.size(); ++m) {
    psi[m] = rt[m].v;
    dpsi[m] = rt[m].d;
  }
  return LBO_OK;
}

}  // extern "C"
