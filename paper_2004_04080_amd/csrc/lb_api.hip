// lb_api.hip -- host runtime behind the C interface of include/lbhip.h.
//
// Validation runs on the host before any device call. A step is a fixed
// sequence of kernel launches on the context's stream (no host
// synchronisation inside lb_step):
//   [moving, side stream] clear accumulators, unraster, raster, Hertz pairs
//   density (pull-gather moments)                      -> psi
//   [moving] wait for the side stream; node events
//   [spheres] frontier fill + Shan-Chen on solids; [walls] wall fill
//   collide (SC + EDM + store + moving bounce-back + link momentum exchange)
//   [moving] integrate; swap buffers and maps
// The side stream (default priority) lets the latency-bound map update run
// beside the bandwidth-bound density pass; it is joined through an event
// before anything reads the new map or the accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "lb_device.hpp"
#include "lb_internal.hpp"

using namespace lbh;

namespace {

thread_local std::string g_last_error;

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int fail(lb_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_last_error = msg;
  return code;
}

#define HIPCHK(c, expr)                                                          \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(c, LB_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool is_finite(double v) { return std::isfinite(v); }

int validate(const lb_params* p, std::string& why) {
  if (!p) { why = "params is NULL"; return LB_E_ARG; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "box sizes must be >= 1"; return LB_E_ARG; }
  const uint64_t N = uint64_t(p->nx) * p->ny * p->nz;
  if (N > (uint64_t(1) << 31) - 1) { why = "box has more than 2^31-1 nodes"; return LB_E_SHAPE; }
  if (p->walls != 0 && p->walls != 1) { why = "walls must be 0 or 1"; return LB_E_ARG; }
  if (p->walls && p->nz < 3) { why = "walls need nz >= 3"; return LB_E_ARG; }
  if (p->ncomp != 1 && p->ncomp != 2) { why = "ncomp must be 1 or 2"; return LB_E_ARG; }
  for (int k = 0; k < p->ncomp; ++k) {
    if (!is_finite(p->tau[k]) || !(p->tau[k] > 0.5)) { why = "tau must be > 1/2"; return LB_E_ARG; }
    if (!is_finite(p->rho0[k])) { why = "rho0 must be finite"; return LB_E_ARG; }
  }
  if (!is_finite(p->G) || !is_finite(p->sc_norm)) { why = "G and sc_norm must be finite"; return LB_E_ARG; }
  for (int d = 0; d < 3; ++d)
    if (!is_finite(p->g[d]) || !is_finite(p->wall_u_lo[d]) || !is_finite(p->wall_u_hi[d])) {
      why = "g and wall velocities must be finite";
      return LB_E_ARG;
    }
  if (p->precision != LB_FP32 && p->precision != LB_FP64) { why = "bad precision"; return LB_E_ARG; }
  if (p->janus != 0 && p->janus != 1) { why = "janus must be 0 or 1"; return LB_E_ARG; }
  for (int f = 0; f < 2; ++f) {
    const int t = p->wall_type[f];
    if (t < 0 || t > 3) { why = "wall_type must be 0..3"; return LB_E_ARG; }
    if (t != 0 && (!p->walls || p->nz < 4)) {
      why = "open faces need walls = 1 and nz >= 4";
      return LB_E_ARG;
    }
    if (t == 1 || t == 3)
      for (int k = 0; k < p->ncomp; ++k)
        if (!(p->wall_rho[f][k] > 0.0) || !is_finite(p->wall_rho[f][k])) {
          why = "wall_rho must be finite and > 0 on pressure and equilibrium faces";
          return LB_E_ARG;
        }
  }
  if (p->janus && !(p->janus_width > 0.0 && is_finite(p->janus_width) &&
                    is_finite(p->janus_theta0) && is_finite(p->janus_zeta[0]) &&
                    is_finite(p->janus_zeta[1]))) {
    why = "janus needs a finite width > 0, angle and constants";
    return LB_E_ARG;
  }
  if (!(p->lub_mu >= 0.0) || !is_finite(p->lub_mu) ||
      (p->lub_mu > 0.0 && !(p->lub_hcap > 0.0 && p->lub_hn > p->lub_hcap && is_finite(p->lub_hn)))) {
    why = "lubrication needs lub_mu >= 0 and 0 < lub_hcap < lub_hn";
    return LB_E_ARG;
  }
  // kernels address one population plane [k][i][*] with 32-bit byte offsets
  if (N * (p->precision == LB_FP64 ? 8u : 4u) > 0xFFFFFFFFull) {
    why = "one population plane (nodes x element size) exceeds 4 GiB";
    return LB_E_SHAPE;
  }
  if (p->max_particles < 0 || p->max_particles > 65534) {
    why = "max_particles must be in [0, 65534]";
    return LB_E_ARG;
  }
  if (p->max_particles > 0) {
    const double Lmin = std::min({p->nx, p->ny, p->nz});
    if (!(p->radius > 0.0) || !(p->radius < 0.5 * Lmin)) {
      why = "radius must be in (0, min box size / 2)";
      return LB_E_ARG;
    }
    if (!(p->particle_density > 0.0) || !is_finite(p->particle_density)) {
      why = "particle_density must be > 0";
      return LB_E_ARG;
    }
    if (!(p->hertz_K >= 0.0) || !(p->hertz_rcap >= 0.0) || !(p->hertz_d0 >= p->hertz_rcap) ||
        !is_finite(p->hertz_d0)) {
      why = "Hertz parameters need K >= 0 and d0 >= rcap >= 0";
      return LB_E_ARG;
    }
    for (int k = 0; k < p->ncomp; ++k)
      if (!is_finite(p->zeta[k]) || !is_finite(p->rho_fallback[k])) {
        why = "zeta and rho_fallback must be finite";
        return LB_E_ARG;
      }
  }
  if (p->checkpoint_every < 0 || p->max_record_steps < 0) {
    why = "checkpoint_every and max_record_steps must be >= 0";
    return LB_E_ARG;
  }
  if (p->checkpoint_every > 0 && p->max_record_steps == 0) {
    why = "recording needs max_record_steps > 0";
    return LB_E_ARG;
  }
  return LB_OK;
}

bool has_solids(const lb_params& p) { return p.walls || p.max_particles > 0; }

void compute_sizes(const lb_params& p, lb_sizes& s, WorkLayout& wl, AdjLayout& al,
                   int ncell[3]) {
  const size_t N = size_t(p.nx) * p.ny * p.nz;
  const size_t es = p.precision == LB_FP64 ? 8 : 4;
  s.f = align_up(size_t(p.ncomp) * Q * N * es);
  s.rho = align_up(size_t(p.ncomp) * N * es);
  s.owner = has_solids(p) ? align_up(N * 2) : 0;
  s.particles = align_up(size_t(p.max_particles) * (PSTRIDE + ASTRIDE) * sizeof(double));
  cell_dims(p, ncell);
  s.work = work_layout(p, wl, ncell[0] * ncell[1] * ncell[2]);
  s.adjoint = adj_layout(p, s.f, al);
}

const uint16_t* owner_now(lb_ctx* c) {
  return c->has_solids ? static_cast<const uint16_t*>(c->B.owner[c->own_old]) : nullptr;
}

hipEvent_t ev_get(lb_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// HIP events around the kernels of one phase of a step (only while timing).
struct Phase {
  lb_ctx* c;
  int ph;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Phase(lb_ctx* ctx, int phase, hipStream_t stream = nullptr)
      : c(ctx), ph(phase), s(stream ? stream : ctx->stream) {
    if (c->timing && (a = ev_get(c)) != nullptr) (void)hipEventRecord(a, s);
  }
  ~Phase() {
    if (!a) return;
    hipEvent_t b = ev_get(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->ev_open.push_back({ph, {a, b}});
  }
};

// Collect the elapsed times of the recorded event pairs (synchronises).
int harvest(lb_ctx* c, bool keep) {
  if (c->ev_open.empty()) return LB_OK;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LB_E_HIP;
  for (auto& e : c->ev_open) {
    float ms = 0.0f;
    if (keep && hipEventElapsedTime(&ms, e.second.first, e.second.second) == hipSuccess) {
      c->phase_ms[e.first] += ms;
      c->phase_n[e.first] += 1;
    }
    c->ev_pool.push_back(e.second.first);
    c->ev_pool.push_back(e.second.second);
  }
  c->ev_open.clear();
  return LB_OK;
}

uint32_t chunk_nodes(lb_ctx* c, int per_node) {
  return uint32_t(std::max<size_t>(1, c->wl.staging_n / size_t(per_node)));
}

}  // namespace

namespace lbh {

void cell_dims(const lb_params& p, int ncell[3]) {
  const int L[3] = {p.nx, p.ny, p.nz};
  // the neighbouring cells must hold every sphere within the Hertz range, the
  // lubrication range and 2R + 1/2 (spheres that may share nodes)
  double side = std::max({1.0, p.hertz_d0, 2.0 * p.radius + 0.5});
  if (p.lub_mu > 0.0) side = std::max(side, 2.0 * p.radius + p.lub_hn);
  for (int d = 0; d < 3; ++d) ncell[d] = std::max(1, int(std::floor(L[d] / side)));
  if (p.max_particles == 0) ncell[0] = ncell[1] = ncell[2] = 1;
}

size_t work_layout(const lb_params& p, WorkLayout& wl, int ncell_total) {
  const size_t N = size_t(p.nx) * p.ny * p.nz;
  size_t off = 0;
  wl.flags = off;
  off = align_up(off + 64 * sizeof(int32_t));
  wl.partials = off;
  off = align_up(off + size_t(RED_BLOCKS) * RED_N * sizeof(double));
  wl.red_out = off;
  off = align_up(off + RED_N * sizeof(double));
  wl.cell_count = off;
  off = align_up(off + size_t(ncell_total) * sizeof(int32_t));
  wl.cell_start = off;
  off = align_up(off + size_t(ncell_total + 1) * sizeof(int32_t));
  wl.cell_ids = off;
  off = align_up(off + size_t(std::max(p.max_particles, 1)) * sizeof(int32_t));
  wl.staging_n = 5 * std::min<size_t>(N, size_t(1) << 20);
  wl.staging = off;
  off = align_up(off + wl.staging_n * sizeof(double));
  wl.ubnd = off;
  if (has_pressure_face(p)) off = align_up(off + 2 * size_t(p.nx) * p.ny * 3 * sizeof(double));
  // Frontier list: a sphere owns only nodes closer than R to its centre, and
  // the unit cubes around those nodes lie inside the ball of radius R + 1, so
  // a sphere owns fewer than 4/3 pi (R + 1)^3 nodes.
  wl.fcount = off;
  off = align_up(off + sizeof(int32_t));
  const double rr = std::max(p.radius, 0.0) + 1.0;
  const size_t per = size_t(std::ceil(4.0 / 3.0 * M_PI * rr * rr * rr));
  wl.fcap = std::min(N, size_t(std::max(p.max_particles, 0)) * per);
  wl.fcap = std::min<size_t>(wl.fcap, 0xFFFFFFFFu);
  wl.flist = off;
  off = align_up(off + wl.fcap * 2 * sizeof(uint32_t));
  // Event list: a sphere's created nodes are nodes it owned, its destroyed
  // nodes nodes it owns now, so at most twice the bound above per sphere.
  wl.ecount = off;
  off = align_up(off + sizeof(int32_t));
  wl.ecap = std::min(N, 2 * size_t(std::max(p.max_particles, 0)) * per);
  wl.ecap = std::min<size_t>(wl.ecap, 0xFFFFFFFFu);
  wl.elist = off;
  off = align_up(off + wl.ecap * 2 * sizeof(uint32_t));
  wl.total = off;
  return off;
}

}  // namespace lbh

extern "C" {

const char* lb_version(void) { return "lbhip 1.0 (gfx950)"; }

const char* lb_strerror(int s) {
  switch (s) {
    case LB_OK: return "ok";
    case LB_E_ARG: return "invalid argument";
    case LB_E_SHAPE: return "buffer or box size mismatch";
    case LB_E_OVERLAP: return "spheres overlap each other or a wall";
    case LB_E_CAPACITY: return "capacity exceeded";
    case LB_E_NONFINITE: return "non-finite value in the fluid";
    case LB_E_PARTICLE_SPEED: return "a sphere moved more than half a node in one step";
    case LB_E_HIP: return "HIP runtime error";
    case LB_E_STATE: return "call not valid in the current state";
    default: return "unknown status";
  }
}

const char* lb_last_error(const lb_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

int lb_lattice(int32_t* c, double* w) {
  if (!c || !w) return LB_E_ARG;
  for (int i = 0; i < Q; ++i) {
    c[3 * i] = CX[i];
    c[3 * i + 1] = CY[i];
    c[3 * i + 2] = CZ[i];
    w[i] = WQ[i];
  }
  return LB_OK;
}

int lb_required_sizes(const lb_params* p, lb_sizes* out) {
  std::string why;
  const int rc = validate(p, why);
  if (rc != LB_OK) return fail(nullptr, rc, why);
  if (!out) return fail(nullptr, LB_E_ARG, "out is NULL");
  WorkLayout wl;
  AdjLayout al;
  int nc[3];
  compute_sizes(*p, *out, wl, al, nc);
  return LB_OK;
}

int lb_init(const lb_params* p, const lb_buffers* b, const double* rho0, const double* u0,
            void* stream, lb_ctx** out) {
  std::string why;
  int rc = validate(p, why);
  if (rc != LB_OK) return fail(nullptr, rc, why);
  if (!b || !rho0 || !out) return fail(nullptr, LB_E_ARG, "buffers, rho0 and out are required");
  lb_sizes req;
  WorkLayout wl;
  AdjLayout al;
  int nc[3];
  compute_sizes(*p, req, wl, al, nc);
  struct Need { void* ptr; size_t have, need; const char* name; };
  const Need needs[] = {{b->f[0], b->bytes.f, req.f, "f[0]"},
                        {b->f[1], b->bytes.f, req.f, "f[1]"},
                        {b->rho, b->bytes.rho, req.rho, "rho"},
                        {b->owner[0], b->bytes.owner, req.owner, "owner[0]"},
                        {b->owner[1], b->bytes.owner, req.owner, "owner[1]"},
                        {b->particles, b->bytes.particles, req.particles, "particles"},
                        {b->work, b->bytes.work, req.work, "work"},
                        {b->adjoint, b->bytes.adjoint, req.adjoint, "adjoint"}};
  for (const auto& n : needs) {
    if (n.need == 0) continue;
    if (!n.ptr) return fail(nullptr, LB_E_ARG, std::string("buffer ") + n.name + " is NULL");
    if (n.have < n.need)
      return fail(nullptr, LB_E_SHAPE, std::string("buffer ") + n.name + " is too small");
    if (reinterpret_cast<uintptr_t>(n.ptr) % 16 != 0)
      return fail(nullptr, LB_E_ARG, std::string("buffer ") + n.name + " is not 16-byte aligned");
  }
  const size_t N = size_t(p->nx) * p->ny * p->nz;
  for (size_t k = 0; k < size_t(p->ncomp) * N; ++k)
    if (!is_finite(rho0[k]) || !(rho0[k] > 0.0))
      return fail(nullptr, LB_E_ARG, "initial densities must be finite and > 0");

  lb_ctx* c = new lb_ctx();
  c->P = *p;
  if (p->ncomp == 1) {
    c->P.tau[1] = c->P.tau[0];
    c->P.rho0[1] = c->P.rho0[0];
    c->P.zeta[1] = c->P.zeta[0];
    c->P.rho_fallback[1] = c->P.rho_fallback[0];
  }
  c->req = req;
  c->B = *b;
  c->stream = static_cast<hipStream_t>(stream);
  c->geo = Geometry{uint32_t(p->nx), uint32_t(p->ny), uint32_t(p->nz), uint32_t(N), p->ncomp,
                    p->precision, size_t(p->precision == LB_FP64 ? 8 : 4)};
  c->wl = wl;
  c->al = al;
  c->has_solids = has_solids(*p);
  if (noalloc_setup(c) != LB_OK) {
    g_last_error = c->err;
    delete c;
    return LB_E_HIP;
  }
  for (int d = 0; d < 3; ++d) c->ncell[d] = nc[d];
  const double R = p->radius;
  c->mass = p->particle_density * 4.0 / 3.0 * M_PI * R * R * R;
  c->inertia = 0.4 * c->mass * R * R;
  auto bad = [&](int code) {
    g_last_error = c->err;
    delete c;
    return code;
  };
  if (hipMemsetAsync(c->B.f[0], 0, req.f, c->stream) != hipSuccess ||
      hipMemsetAsync(c->B.f[1], 0, req.f, c->stream) != hipSuccess ||
      hipMemsetAsync(c->B.rho, 0, req.rho, c->stream) != hipSuccess ||
      hipMemsetAsync(c->B.work, 0, req.work, c->stream) != hipSuccess ||
      (req.particles && hipMemsetAsync(c->B.particles, 0, req.particles, c->stream) != hipSuccess)) {
    c->err = "hipMemsetAsync failed during init";
    return bad(LB_E_HIP);
  }
  if (c->has_solids) {
    if (launch_raster_full(c, static_cast<uint16_t*>(c->B.owner[0])) != hipSuccess ||
        launch_raster_full(c, static_cast<uint16_t*>(c->B.owner[1])) != hipSuccess) {
      c->err = "map initialisation failed";
      return bad(LB_E_HIP);
    }
  }
  // initial populations, staged through the work buffer in chunks
  const int per = p->ncomp + (u0 ? 3 : 0);
  const uint32_t chunk = chunk_nodes(c, per);
  double* stage = reinterpret_cast<double*>(wptr(c, c->wl.staging));
  std::vector<double> host(size_t(chunk) * per);
  for (uint32_t first = 0; first < N; first += chunk) {
    const uint32_t cnt = uint32_t(std::min<size_t>(chunk, N - first));
    for (int k = 0; k < p->ncomp; ++k)
      std::memcpy(&host[size_t(k) * cnt], rho0 + size_t(k) * N + first, cnt * sizeof(double));
    if (u0) std::memcpy(&host[size_t(p->ncomp) * cnt], u0 + 3 * size_t(first), 3 * cnt * sizeof(double));
    if (hipMemcpyAsync(stage, host.data(), size_t(cnt) * per * sizeof(double),
                       hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        launch_init_populations(c, stage, u0 ? stage + size_t(p->ncomp) * cnt : nullptr, first,
                                cnt) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      c->err = "initial population upload failed";
      return bad(LB_E_HIP);
    }
  }
  *out = c;
  return LB_OK;
}

int lb_num_particles(const lb_ctx* c) { return c ? c->nparticles : 0; }

namespace {

// A coordinate taken into [0, L): fmod leaves (-L, L), and a tiny negative
// value plus L rounds to L itself, which is wrapped again.
double wrap_coord(double v, double L) {
  double r = std::fmod(v, L);
  if (r < 0) r += L;
  if (r >= L) r -= L;
  return r;
}

// Checks of a set of sphere records before they are rasterised: records
// [P0, P1) of st are new; each must stay clear of the wall layers, and no two
// centres may be closer than 2R unless both are old (hash grid of cell side
// 2R). Returns LB_OK or the status, with the reason in why.
int check_placement(const lb_ctx* c, const std::vector<double>& st, int P0, int P1,
                    std::string& why) {
  const double L[3] = {double(c->geo.nx), double(c->geo.ny), double(c->geo.nz)};
  const double R = c->P.radius;
  if (c->P.walls)
    for (int p = P0; p < P1; ++p) {
      const double z = st[size_t(p) * PSTRIDE + PS_X + 2];
      if (z - R < 0.5 || z + R > L[2] - 1.5) {
        why = "a sphere reaches a wall layer";
        return LB_E_OVERLAP;
      }
    }
  const double side = 2.0 * R;
  int nc[3];
  for (int d = 0; d < 3; ++d) nc[d] = std::max(1, int(L[d] / side));
  std::unordered_map<int64_t, std::vector<int>> grid;
  auto key = [&](const int ci[3]) {
    return (int64_t(ci[2]) * nc[1] + ci[1]) * nc[0] + ci[0];
  };
  for (int p = 0; p < P1; ++p) {
    const double* r = &st[size_t(p) * PSTRIDE];
    int ci[3];
    for (int d = 0; d < 3; ++d) ci[d] = std::min(nc[d] - 1, int(r[PS_X + d] / L[d] * nc[d]));
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int cj[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
          for (int d = 0; d < 3; ++d) cj[d] = ((cj[d] % nc[d]) + nc[d]) % nc[d];
          auto it = grid.find(key(cj));
          if (it == grid.end()) continue;
          for (int q2 : it->second) {
            if (p < P0 && q2 < P0) continue;
            const double* s = &st[size_t(q2) * PSTRIDE];
            double d2 = 0;
            for (int d = 0; d < 3; ++d) {
              double dd = r[PS_X + d] - s[PS_X + d];
              dd -= L[d] * std::nearbyint(dd / L[d]);
              d2 += dd * dd;
            }
            if (d2 < side * side) {
              why = "sphere centres closer than 2R";
              return LB_E_OVERLAP;
            }
          }
        }
    auto& cell = grid[key(ci)];
    if (std::find(cell.begin(), cell.end(), p) == cell.end()) cell.push_back(p);
  }
  return LB_OK;
}

}  // namespace

int lb_add_particles(lb_ctx* c, int32_t n, const double* x, const double* v, const double* w,
                     const double* q) {
  if (!c) return LB_E_ARG;
  if (n < 0 || (n > 0 && !x)) return fail(c, LB_E_ARG, "bad sphere arrays");
  if (c->step != 0) return fail(c, LB_E_STATE, "spheres can only be added before the first step");
  if (n == 0) return LB_OK;
  if (c->nparticles + n > c->P.max_particles)
    return fail(c, LB_E_CAPACITY, "more spheres than max_particles");
  const double L[3] = {double(c->geo.nx), double(c->geo.ny), double(c->geo.nz)};
  // host copy of the existing records plus the new ones
  const int P0 = c->nparticles, P1 = P0 + n;
  std::vector<double> st(size_t(P1) * PSTRIDE, 0.0);
  if (P0 > 0)
    HIPCHK(c, hipMemcpy(st.data(), pstate(c), size_t(P0) * PSTRIDE * sizeof(double),
                        hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) {
    double* r = &st[size_t(P0 + i) * PSTRIDE];
    for (int d = 0; d < 3; ++d) {
      if (!is_finite(x[3 * i + d]) || (v && !is_finite(v[3 * i + d])) ||
          (w && !is_finite(w[3 * i + d])))
        return fail(c, LB_E_ARG, "non-finite sphere position or velocity");
      const double xv = wrap_coord(x[3 * i + d], L[d]);
      r[PS_X + d] = r[PS_XRA + d] = r[PS_XRB + d] = xv;
      r[PS_V + d] = v ? v[3 * i + d] : 0.0;
      r[PS_W + d] = w ? w[3 * i + d] : 0.0;
    }
    double qn = 0;
    for (int e = 0; e < 4; ++e) {
      r[PS_Q + e] = q ? q[4 * i + e] : (e == 0 ? 1.0 : 0.0);
      qn += r[PS_Q + e] * r[PS_Q + e];
    }
    if (!is_finite(qn) || !(qn > 0.0)) return fail(c, LB_E_ARG, "bad sphere quaternion");
  }
  std::string why;
  const int rc = check_placement(c, st, P0, P1, why);
  if (rc != LB_OK) return fail(c, rc, why);
  HIPCHK(c, hipMemcpy(pstate(c) + size_t(P0) * PSTRIDE, &st[size_t(P0) * PSTRIDE],
                      size_t(n) * PSTRIDE * sizeof(double), hipMemcpyHostToDevice));
  c->nparticles = P1;
  c->moving = !c->P.particles_fixed;
  HIPCHK(c, launch_raster_full(c, static_cast<uint16_t*>(c->B.owner[0])));
  HIPCHK(c, launch_raster_full(c, static_cast<uint16_t*>(c->B.owner[1])));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LB_OK;
}

int lb_step(lb_ctx* c, int32_t nsteps) {
  if (!c) return LB_E_ARG;
  if (nsteps < 0) return fail(c, LB_E_ARG, "nsteps < 0");
  for (int32_t s = 0; s < nsteps; ++s) {
    if (c->P.checkpoint_every > 0) {
      if (c->rec_steps >= c->P.max_record_steps)
        return fail(c, LB_E_CAPACITY, "more steps than max_record_steps while recording");
      if (c->rec_steps % c->P.checkpoint_every == 0) {
        const int rc = record_checkpoint(c);
        if (rc != LB_OK) return rc;
      }
    }
    void* fin = c->B.f[c->cur];
    void* fout = c->B.f[1 - c->cur];
    const bool moving = c->moving && c->nparticles > 0;
    if (moving) {
      // map update and pair forces on the side stream, beside the density pass
      if (!c->side) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
      }
      HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
      HIPCHK(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
      {
        Phase ph(c, 1, c->side);
        HIPCHK(c, launch_map_update(c, c->side));
      }
      HIPCHK(c, hipEventRecord(c->ev_join, c->side));
    }
    {
      Phase ph(c, 0);
      HIPCHK(c, launch_density(c, fin));
    }
    const uint16_t* own = owner_now(c);
    if (c->nparticles > 0 && !moving) HIPCHK(c, launch_clear_accumulators(c));
    if (moving) {
      HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
      Phase ph(c, 1);
      HIPCHK(c, launch_events(c));
      own = static_cast<const uint16_t*>(c->B.owner[1 - c->own_old]);
    }
    if (has_pressure_face(c->P)) HIPCHK(c, launch_face_velocity(c, fin));
    if (c->nparticles > 0 || c->P.walls) {
      Phase ph(c, 2);
      if (c->nparticles > 0) HIPCHK(c, launch_fill_particles(c, own, true, moving));
      if (c->P.walls) HIPCHK(c, launch_fill_walls(c, own));
    }
    {
      Phase ph(c, 3);
      HIPCHK(c, launch_collide(c, fin, fout, own));
    }
    if (c->moving) {
      Phase ph(c, 4);
      HIPCHK(c, launch_integrate(c));
      c->own_old = 1 - c->own_old;
    }
    c->cur = 1 - c->cur;
    ++c->step;
    if (c->P.checkpoint_every > 0) ++c->rec_steps;
  }
  return LB_OK;
}

namespace {
struct StateHeader {
  char magic[8];  // "LBSTATE1"
  int32_t nx, ny, nz, ncomp, precision, walls, nparticles, reserved;
  int64_t step;
  uint64_t f_bytes, owner_bytes, particle_bytes;
};
constexpr char kStateMagic[8] = {'L', 'B', 'S', 'T', 'A', 'T', 'E', '1'};

void state_parts(const lb_ctx* c, int np, uint64_t& fb, uint64_t& ob, uint64_t& pb) {
  fb = c->req.f;
  ob = c->has_solids ? uint64_t(c->geo.N) * sizeof(uint16_t) : 0;
  pb = uint64_t(np) * PSTRIDE * sizeof(double);
}
}  // namespace

int lb_state_bytes(const lb_ctx* c, size_t* bytes) {
  if (!c || !bytes) return LB_E_ARG;
  uint64_t fb, ob, pb;
  state_parts(c, c->nparticles, fb, ob, pb);
  *bytes = sizeof(StateHeader) + fb + 2 * ob + pb;
  return LB_OK;
}

int lb_get_state(lb_ctx* c, void* blob, size_t bytes) {
  size_t need = 0;
  if (!c || !blob || lb_state_bytes(c, &need) != LB_OK) return LB_E_ARG;
  if (bytes < need) return fail(c, LB_E_ARG, "state buffer too small (see lb_state_bytes)");
  StateHeader h;
  std::memcpy(h.magic, kStateMagic, sizeof(h.magic));
  h.nx = int32_t(c->geo.nx);
  h.ny = int32_t(c->geo.ny);
  h.nz = int32_t(c->geo.nz);
  h.ncomp = c->geo.ncomp;
  h.precision = c->geo.prec;
  h.walls = c->P.walls;
  h.nparticles = c->nparticles;
  h.reserved = 0;
  h.step = c->step;
  state_parts(c, c->nparticles, h.f_bytes, h.owner_bytes, h.particle_bytes);
  char* out = static_cast<char*>(blob);
  std::memcpy(out, &h, sizeof(h));
  out += sizeof(h);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(out, c->B.f[c->cur], h.f_bytes, hipMemcpyDeviceToHost));
  out += h.f_bytes;
  if (h.owner_bytes) {
    HIPCHK(c, hipMemcpy(out, c->B.owner[c->own_old], h.owner_bytes, hipMemcpyDeviceToHost));
    out += h.owner_bytes;
    HIPCHK(c, hipMemcpy(out, c->B.owner[1 - c->own_old], h.owner_bytes, hipMemcpyDeviceToHost));
    out += h.owner_bytes;
  }
  if (h.particle_bytes)
    HIPCHK(c, hipMemcpy(out, pstate(c), h.particle_bytes, hipMemcpyDeviceToHost));
  return LB_OK;
}

int lb_set_state(lb_ctx* c, const void* blob, size_t bytes) {
  if (!c || !blob || bytes < sizeof(StateHeader)) return LB_E_ARG;
  StateHeader h;
  std::memcpy(&h, blob, sizeof(h));
  if (std::memcmp(h.magic, kStateMagic, sizeof(h.magic)) != 0)
    return fail(c, LB_E_ARG, "not a state blob");
  if (h.nx != int32_t(c->geo.nx) || h.ny != int32_t(c->geo.ny) || h.nz != int32_t(c->geo.nz) ||
      h.ncomp != c->geo.ncomp || h.precision != c->geo.prec || h.walls != c->P.walls)
    return fail(c, LB_E_SHAPE, "state blob of another box, component count, precision or walls");
  if (h.nparticles < 0 || h.nparticles > c->P.max_particles)
    return fail(c, LB_E_CAPACITY, "state blob holds more spheres than max_particles");
  uint64_t fb, ob, pb;
  state_parts(c, h.nparticles, fb, ob, pb);
  if (h.f_bytes != fb || h.owner_bytes != ob || h.particle_bytes != pb ||
      bytes < sizeof(h) + fb + 2 * ob + pb)
    return fail(c, LB_E_ARG, "state blob sizes do not match this context");
  const char* in = static_cast<const char*>(blob) + sizeof(h);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->B.f[c->cur], in, fb, hipMemcpyHostToDevice));
  in += fb;
  if (ob) {
    HIPCHK(c, hipMemcpy(c->B.owner[c->own_old], in, ob, hipMemcpyHostToDevice));
    in += ob;
    HIPCHK(c, hipMemcpy(c->B.owner[1 - c->own_old], in, ob, hipMemcpyHostToDevice));
    in += ob;
  }
  c->flist_map = nullptr;
  if (pb) HIPCHK(c, hipMemcpy(pstate(c), in, pb, hipMemcpyHostToDevice));
  c->nparticles = h.nparticles;
  c->moving = h.nparticles > 0 && !c->P.particles_fixed;
  c->step = h.step;
  c->rec_steps = 0;
  HIPCHK(c, hipMemset(wptr(c, c->wl.flags), 0, 16 * sizeof(int32_t)));
  return LB_OK;
}

int lb_debug_count_writes(lb_ctx* c, void* counts) {
  if (!c) return LB_E_ARG;
  if (counts && !c->has_solids)
    return fail(c, LB_E_STATE, "store counting needs walls or spheres (bounce-back links)");
  if (reinterpret_cast<uintptr_t>(counts) % 4 != 0)
    return fail(c, LB_E_ARG, "counts must be 4-byte aligned");
  c->write_counts = static_cast<uint32_t*>(counts);
  return LB_OK;
}

int lb_sync(lb_ctx* c) {
  if (!c) return LB_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LB_OK;
}

}  // extern "C"

namespace lbh {

// Pseudo-potential of the current state on its map: moments, then the
// virtual densities of the frontier (the sphere fill leaves the force
// accumulators alone).
int current_psi(lb_ctx* c) {
  HIPCHK(c, launch_density(c, c->B.f[c->cur]));
  const uint16_t* own = c->has_solids ? static_cast<const uint16_t*>(c->B.owner[c->own_old])
                                      : nullptr;
  if (c->nparticles > 0) HIPCHK(c, launch_fill_particles(c, own, false));
  if (c->P.walls) HIPCHK(c, launch_fill_walls(c, own));
  return LB_OK;
}

// The fluid part of lb_obs from the reduction results r (layout of
// k_reduce_partials), after clearing the whole record.
void obs_fluid(const lb_ctx* c, const double* r, lb_obs* o) {
  std::memset(o, 0, sizeof(*o));
  o->step = c->step;
  o->fluid_nodes = int64_t(r[10]);
  for (int k = 0; k < c->geo.ncomp; ++k) {
    o->mass[k] = r[10] * c->P.rho0[k] + r[k];
    o->rho_min[k] = c->P.rho0[k] + r[5 + k];
    o->rho_max[k] = c->P.rho0[k] + r[7 + k];
  }
  for (int d = 0; d < 3; ++d) {
    o->momentum[d] = r[2 + d];
    o->phys_momentum[d] = r[2 + d] + 0.5 * r[12 + d];
  }
  o->u_max = r[9];
  o->nparticles = c->nparticles;
}

// The flags of lb_obs (work-buffer flags and the non-finite count of r) and
// the status they make lb_observables return.
int obs_flags(lb_ctx* c, const double* r, const int32_t* flags, lb_obs* o) {
  o->flags = (flags[0] ? 1 : 0) | (r[11] > 0 || !std::isfinite(r[0]) ? 2 : 0) | (flags[2] ? 4 : 0);
  if (o->flags & 1) return fail(c, LB_E_PARTICLE_SPEED, "sphere speed exceeded 1/2 per step");
  if (o->flags & 2) return fail(c, LB_E_NONFINITE, "non-finite populations");
  if (o->flags & 4) return fail(c, LB_E_CAPACITY, "frontier list overflow");
  return LB_OK;
}

}  // namespace lbh

extern "C" {

int lb_observables(lb_ctx* c, lb_obs* o) {
  if (!c || !o) return LB_E_ARG;
  double* red = reinterpret_cast<double*>(wptr(c, c->wl.red_out));
  // the force density of the physical momentum needs the pseudo-potential
  const int rc = current_psi(c);
  if (rc != LB_OK) return rc;
  HIPCHK(c, launch_reduce(c, reinterpret_cast<double*>(wptr(c, c->wl.partials)), red));
  double r[RED_N];
  int32_t flags[3];
  HIPCHK(c, hipMemcpyAsync(r, red, sizeof(r), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(flags, wptr(c, c->wl.flags), sizeof(flags), hipMemcpyDeviceToHost,
                           c->stream));
  std::vector<double> st(size_t(c->nparticles) * PSTRIDE), ac(size_t(c->nparticles) * ASTRIDE);
  if (c->nparticles) {
    HIPCHK(c, hipMemcpyAsync(st.data(), pstate(c), st.size() * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ac.data(), pacc(c), ac.size() * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  obs_fluid(c, r, o);
  // particle sums with Neumaier compensation
  auto nsum = [&](auto get) {
    double s = 0, comp = 0;
    for (int p = 0; p < c->nparticles; ++p) {
      const double x = get(&st[size_t(p) * PSTRIDE]);
      const double t = s + x;
      comp += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
      s = t;
    }
    return s + comp;
  };
  for (int d = 0; d < 3; ++d)
    o->particle_momentum[d] = nsum([&](const double* P) { return c->mass * P[PS_V + d]; });
  o->particle_ke = nsum([&](const double* P) {
    return 0.5 * c->mass * (P[PS_V] * P[PS_V] + P[PS_V + 1] * P[PS_V + 1] + P[PS_V + 2] * P[PS_V + 2]);
  });
  o->particle_ke_rot = nsum([&](const double* P) {
    return 0.5 * c->inertia * (P[PS_W] * P[PS_W] + P[PS_W + 1] * P[PS_W + 1] + P[PS_W + 2] * P[PS_W + 2]);
  });
  {
    double s = 0, comp = 0;
    for (int p = 0; p < c->nparticles; ++p) {
      const double x = ac[size_t(p) * ASTRIDE + AC_FLABS];
      const double t = s + x;
      comp += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
      s = t;
    }
    o->flink_abs = s + comp;
  }
  return obs_flags(c, r, flags, o);
}

int lb_get_fields(lb_ctx* c, double* rho, double* u) {
  if (!c || !rho) return LB_E_ARG;
  const int nc = c->geo.ncomp, per = nc + 3;
  const uint32_t N = c->geo.N, chunk = chunk_nodes(c, per);
  double* stage = reinterpret_cast<double*>(wptr(c, c->wl.staging));
  std::vector<double> h(size_t(chunk) * per);
  for (uint32_t first = 0; first < N; first += chunk) {
    const uint32_t cnt = std::min(chunk, N - first);
    HIPCHK(c, launch_get_fields(c, first, cnt, stage));
    HIPCHK(c, hipMemcpyAsync(h.data(), stage, size_t(cnt) * per * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < nc; ++k)
      std::memcpy(rho + size_t(k) * N + first, &h[size_t(k) * cnt], cnt * sizeof(double));
    if (u)
      for (uint32_t t = 0; t < cnt; ++t)
        for (int d = 0; d < 3; ++d) u[3 * size_t(first + t) + d] = h[size_t(nc + d) * cnt + t];
  }
  return LB_OK;
}

int lb_get_psi(lb_ctx* c, double* psi) {
  if (!c || !psi) return LB_E_ARG;
  const int rc = current_psi(c);
  if (rc != LB_OK) return rc;
  const uint32_t N = c->geo.N, chunk = chunk_nodes(c, 1);
  double* stage = reinterpret_cast<double*>(wptr(c, c->wl.staging));
  for (int k = 0; k < c->geo.ncomp; ++k)
    for (uint32_t first = 0; first < N; first += chunk) {
      const uint32_t cnt = std::min(chunk, N - first);
      HIPCHK(c, launch_get_psi(c, first, cnt, k, stage));
      HIPCHK(c, hipMemcpyAsync(psi + size_t(k) * N + first, stage, cnt * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
  return LB_OK;
}

int lb_get_populations(lb_ctx* c, double* f) {
  if (!c || !f) return LB_E_ARG;
  const uint32_t N = c->geo.N, chunk = chunk_nodes(c, 1);
  double* stage = reinterpret_cast<double*>(wptr(c, c->wl.staging));
  for (int k = 0; k < c->geo.ncomp; ++k)
    for (int i = 0; i < Q; ++i)
      for (uint32_t first = 0; first < N; first += chunk) {
        const uint32_t cnt = std::min(chunk, N - first);
        HIPCHK(c, launch_get_populations(c, k, i, first, cnt, stage));
        HIPCHK(c, hipMemcpyAsync(f + (size_t(k) * Q + i) * N + first, stage,
                                 cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
      }
  return LB_OK;
}

int lb_set_populations(lb_ctx* c, const double* f) {
  if (!c || !f) return LB_E_ARG;
  const uint32_t N = c->geo.N, chunk = chunk_nodes(c, 1);
  double* stage = reinterpret_cast<double*>(wptr(c, c->wl.staging));
  for (int k = 0; k < c->geo.ncomp; ++k)
    for (int i = 0; i < Q; ++i)
      for (uint32_t first = 0; first < N; first += chunk) {
        const uint32_t cnt = std::min(chunk, N - first);
        HIPCHK(c, hipMemcpyAsync(stage, f + (size_t(k) * Q + i) * N + first,
                                 cnt * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, launch_set_populations(c, k, i, first, cnt, stage));
        HIPCHK(c, hipStreamSynchronize(c->stream));
      }
  return LB_OK;
}

int lb_get_owner(lb_ctx* c, int32_t* owner) {
  if (!c || !owner) return LB_E_ARG;
  const uint32_t N = c->geo.N, chunk = chunk_nodes(c, 1);
  int32_t* stage = reinterpret_cast<int32_t*>(wptr(c, c->wl.staging));
  for (uint32_t first = 0; first < N; first += chunk) {
    const uint32_t cnt = std::min(chunk, N - first);
    HIPCHK(c, launch_owner_to_int(c, owner_now(c), first, cnt, stage));
    HIPCHK(c, hipMemcpyAsync(owner + first, stage, cnt * sizeof(int32_t), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return LB_OK;
}

int lb_get_particles(lb_ctx* c, double* rec) {
  if (!c || (!rec && c->nparticles)) return LB_E_ARG;
  const int np = c->nparticles;
  if (np == 0) return LB_OK;
  std::vector<double> st(size_t(np) * PSTRIDE), ac(size_t(np) * ASTRIDE);
  HIPCHK(c, hipMemcpyAsync(st.data(), pstate(c), st.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(ac.data(), pacc(c), ac.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int p = 0; p < np; ++p) {
    const double* S = &st[size_t(p) * PSTRIDE];
    const double* A = &ac[size_t(p) * ASTRIDE];
    double* o = rec + size_t(p) * LB_PREC;
    std::memset(o, 0, LB_PREC * sizeof(double));
    for (int d = 0; d < 3; ++d) {
      o[LB_P_X + d] = S[PS_X + d];
      o[LB_P_V + d] = S[PS_V + d];
      o[LB_P_W + d] = S[PS_W + d];
      o[LB_P_FPREV + d] = S[PS_FPREV + d];
      o[LB_P_TPREV + d] = S[PS_TPREV + d];
      o[LB_P_FD + d] = A[AC_FD + d];
      o[LB_P_TD + d] = A[AC_TD + d];
      o[LB_P_FC + d] = A[AC_FC + d];
      o[LB_P_TC + d] = A[AC_TC + d];
      o[LB_P_FH + d] = A[AC_FH + d];
      o[LB_P_FSC + d] = A[AC_FSC + d];
      o[LB_P_TSC + d] = A[AC_TSC + d];
      o[LB_P_FLIQ + d] = A[AC_FLIQ + d];
      o[LB_P_TLIQ + d] = A[AC_TLIQ + d];
    }
    for (int e = 0; e < 4; ++e) o[LB_P_Q + e] = S[PS_Q + e];
    o[LB_P_FLABS] = A[AC_FLABS];
    o[LB_P_MASS] = c->mass;
    o[LB_P_INERTIA] = c->inertia;
    o[LB_P_HAVEPREV] = S[PS_HAVEPREV];
  }
  return LB_OK;
}

int lb_set_particles(lb_ctx* c, const double* rec) {
  if (!c || (!rec && c->nparticles)) return LB_E_ARG;
  const int np = c->nparticles;
  if (np == 0) return LB_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<double> st(size_t(np) * PSTRIDE);
  HIPCHK(c, hipMemcpy(st.data(), pstate(c), st.size() * sizeof(double), hipMemcpyDeviceToHost));
  const double L[3] = {double(c->geo.nx), double(c->geo.ny), double(c->geo.nz)};
  const bool before_first_step = c->step == 0;
  for (int p = 0; p < np; ++p) {
    double* S = &st[size_t(p) * PSTRIDE];
    const double* o = rec + size_t(p) * LB_PREC;
    double qn = 0;
    for (int e = 0; e < 4; ++e) qn += o[LB_P_Q + e] * o[LB_P_Q + e];
    bool finite = is_finite(qn) && is_finite(o[LB_P_HAVEPREV]);
    for (int d = 0; d < 3; ++d)
      finite = finite && is_finite(o[LB_P_X + d]) && is_finite(o[LB_P_V + d]) &&
               is_finite(o[LB_P_W + d]) && is_finite(o[LB_P_FPREV + d]) &&
               is_finite(o[LB_P_TPREV + d]);
    if (!finite) return fail(c, LB_E_ARG, "non-finite value in a sphere record");
    if (!(qn > 0.0)) return fail(c, LB_E_ARG, "bad sphere quaternion");
    for (int d = 0; d < 3; ++d) {
      const double xv = wrap_coord(o[LB_P_X + d], L[d]);
      if (before_first_step) {
        S[PS_X + d] = S[PS_XRA + d] = S[PS_XRB + d] = xv;
      } else if (xv != S[PS_X + d]) {
        // a moved sphere frees and covers nodes, which needs the node
        // events of a step (or a whole state, lb_set_state)
        return fail(c, LB_E_STATE, "sphere positions can only change before the first step");
      }
      S[PS_V + d] = o[LB_P_V + d];
      S[PS_W + d] = o[LB_P_W + d];
      S[PS_FPREV + d] = o[LB_P_FPREV + d];
      S[PS_TPREV + d] = o[LB_P_TPREV + d];
    }
    for (int e = 0; e < 4; ++e) S[PS_Q + e] = o[LB_P_Q + e];
    S[PS_HAVEPREV] = o[LB_P_HAVEPREV] != 0.0 ? 1.0 : 0.0;
  }
  if (before_first_step) {
    std::string why;
    const int rc = check_placement(c, st, 0, np, why);
    if (rc != LB_OK) return fail(c, rc, why);
  }
  HIPCHK(c, hipMemcpy(pstate(c), st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice));
  if (before_first_step) {
    // the fluid nodes of the new map start from the populations of lb_init
    // (no population was ever stepped); nodes that become solid are dropped
    HIPCHK(c, launch_raster_full(c, static_cast<uint16_t*>(c->B.owner[0])));
    HIPCHK(c, launch_raster_full(c, static_cast<uint16_t*>(c->B.owner[1])));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LB_OK;
}

int lb_timing(lb_ctx* c, int enable) {
  if (!c) return LB_E_ARG;
  // starting drops what was recorded before; stopping keeps it for lb_timing_read
  if (harvest(c, enable == 0) != LB_OK)
    return fail(c, LB_E_HIP, "timing: stream synchronisation failed");
  if (enable != 0)
    for (int p = 0; p < LB_NPHASE; ++p) {
      c->phase_ms[p] = 0.0;
      c->phase_n[p] = 0;
    }
  c->timing = enable != 0;
  return LB_OK;
}

int lb_timing_read(lb_ctx* c, double ms[LB_NPHASE], int64_t count[LB_NPHASE]) {
  if (!c || !ms || !count) return LB_E_ARG;
  if (harvest(c, true) != LB_OK) return fail(c, LB_E_HIP, "timing: stream synchronisation failed");
  for (int p = 0; p < LB_NPHASE; ++p) {
    ms[p] = c->phase_ms[p];
    count[p] = c->phase_n[p];
  }
  return LB_OK;
}

void lb_free(lb_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->side) (void)hipStreamSynchronize(c->side);
  harvest(c, false);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->side) (void)hipStreamDestroy(c->side);
  free_fft(c);
  delete c;
}

}  // extern "C"
