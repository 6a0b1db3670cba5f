// lb_internal.hpp -- host-side context and launch interface shared by the
// translation units of liblbhip (not installed, not part of the C interface).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbhip.h"

namespace lbh {

// Scratch layout inside the caller's work buffer (byte offsets).
struct WorkLayout {
  size_t flags = 0;        // int32[16]: 0 speed exceeded, 1 non-finite
  size_t partials = 0;     // double[RED_BLOCKS][RED_N]
  size_t red_out = 0;      // double[RED_N]
  size_t cell_count = 0;   // int32[ncell]
  size_t cell_start = 0;   // int32[ncell + 1]
  size_t cell_ids = 0;     // int32[P]
  size_t staging = 0;      // double[staging_n]
  size_t staging_n = 0;
  size_t ubnd = 0;         // double[2][nx*ny][3]: mixture velocity next to open faces
  size_t fcount = 0;       // int32: entries appended to the frontier list
  size_t flist = 0;        // uint2[fcap]: frontier nodes of the sphere map (node, mask)
  size_t fcap = 0;
  size_t ecount = 0;       // int32: entries appended to the event list
  size_t elist = 0;        // uint2[ecap]: node events of a moving step (node, code)
  size_t ecap = 0;
  size_t total = 0;
};

constexpr int RED_BLOCKS = 1024;
constexpr int RED_N = 16;

// Adjoint buffer layout (byte offsets), present when checkpoint_every > 0.
struct AdjLayout {
  size_t ckpt = 0;         // checkpoints: nckpt population buffers
  int nckpt = 0;
  size_t seg = 0;          // segment states: checkpoint_every population buffers
  size_t mu[2] = {0, 0};   // adjoint of the gathered populations (ping-pong), FP64 [ncomp][19][N]
  size_t lam_a = 0;        // FP64 [ncomp][3][N]: adjoint of the Shan-Chen acceleration
  size_t lam_psi = 0;      // FP64 [ncomp][N]: adjoint of the pseudo-potential
  size_t winv = 0;         // FP64 [N]: 1 / (sum of w_i over fluid neighbours) of frontier solids
  size_t grad = 0;         // FP64 [3][N]: loss gradient scratch
  size_t partials = 0;     // double[blocks][4] of one reverse step
  size_t accum = 0;        // double[4]: dL/dG, dL/dg
  size_t total = 0;
};

struct Geometry {
  uint32_t nx, ny, nz, N;
  int ncomp;
  int prec;      // LB_FP32 / LB_FP64
  size_t esize;  // bytes per stored real
};

}  // namespace lbh

struct lb_ctx {
  lb_params P;
  lb_sizes req;
  lb_buffers B;
  hipStream_t stream = nullptr;
  // second stream for the map update and pair forces of moving spheres, which
  // overlap the density pass (default priority; joined before the node events)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  void* fft = nullptr;  // FFT plan of the domain-size measure, made on first use
  // the owner map the frontier list was built for (null: none); every write
  // of a map other than the map update, which rebuilds the list, clears it
  const void* flist_map = nullptr;
  lbh::Geometry geo;
  lbh::WorkLayout wl;
  lbh::AdjLayout al;
  int cur = 0;        // population buffer holding the post-collision state f*(t-1)
  int own_old = 0;    // owner map holding the map of the current populations
  int nparticles = 0;
  int64_t step = 0;
  bool has_solids = false;  // walls or spheres present
  bool moving = false;      // spheres present and not fixed
  int ncell[3] = {1, 1, 1};
  double mass = 0.0, inertia = 0.0;
  // recording for the adjoint
  int64_t rec_steps = 0;
  // phase timing (HIP events on the context's stream)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_open;
  double phase_ms[LB_NPHASE] = {};
  int64_t phase_n[LB_NPHASE] = {};
  std::string err;
  // static scratch of lb_observables_noalloc on the context's device
  void* noalloc_scratch = nullptr;
  // caller's [ncomp][19][N] counters of lb_debug_count_writes (null: off)
  uint32_t* write_counts = nullptr;
};

namespace lbh {

size_t work_layout(const lb_params& p, WorkLayout& wl, int ncell_total);
size_t adj_layout(const lb_params& p, size_t fbytes, AdjLayout& al);
void cell_dims(const lb_params& p, int ncell[3]);

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_init_populations(lb_ctx* c, const double* rho0_dev, const double* u0_dev,
                                   uint32_t first, uint32_t count);
hipError_t launch_density(lb_ctx* c, const void* f);
// forces = false leaves the sphere accumulators alone (recomputation in the reverse sweep)
hipError_t launch_collide(lb_ctx* c, const void* fin, void* fout, const uint16_t* owner,
                          bool forces = true);
hipError_t launch_fill_walls(lb_ctx* c, const uint16_t* owner);
// mixture velocity of the second fluid layer inside each pressure face
hipError_t launch_face_velocity(lb_ctx* c, const void* f);
bool has_pressure_face(const lb_params& p);
hipError_t launch_get_populations(lb_ctx* c, int k, int i, uint32_t first, uint32_t count,
                                  double* out);
hipError_t launch_set_populations(lb_ctx* c, int k, int i, uint32_t first, uint32_t count,
                                  const double* in);
hipError_t launch_get_fields(lb_ctx* c, uint32_t first, uint32_t count, double* out);
hipError_t launch_get_psi(lb_ctx* c, uint32_t first, uint32_t count, int comp, double* out);
// observables of the current state: reduce_blocks(c) partial records of RED_N
// doubles into `partial`, the final RED_N doubles into out_dev
int reduce_blocks(const lb_ctx* c);
hipError_t launch_reduce(lb_ctx* c, double* partial, double* out_dev);
// pseudo-potential of the current state on its map (moments and fills)
int current_psi(lb_ctx* c);
// lb_obs from the reduction results: the fluid part (clears the record first),
// then the flags and the status they make the call return
void obs_fluid(const lb_ctx* c, const double* r, lb_obs* o);
int obs_flags(lb_ctx* c, const double* r, const int32_t* flags, lb_obs* o);
// device address of the static scratch of the allocation-free entry point
// on the current device, taken once per device (LB_OK or LB_E_HIP)
int noalloc_setup(lb_ctx* c);
hipError_t launch_owner_to_int(lb_ctx* c, const uint16_t* owner, uint32_t first,
                               uint32_t count, int32_t* out);

// particles
hipError_t launch_raster_full(lb_ctx* c, uint16_t* owner);   // walls + all spheres at x
hipError_t launch_map_update(lb_ctx* c, hipStream_t s);  // clear, unraster, raster, pairs
// zero bytes at p on stream s with a fill kernel (graph-capture safe)
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_events(lb_ctx* c);                     // node creation / destruction
// frontier list of the sphere map `owner`, whose spheres sit around the
// centres at record offset `which`, on stream s; with owner_old set, also
// the list of node events from owner_old to owner
hipError_t launch_sphere_lists(lb_ctx* c, const uint16_t* owner, const uint16_t* owner_old,
                               int which, hipStream_t s);
// virtual densities (and with forces on, F_SC and T_SC) of the frontier of
// `owner`; builds the list of the current map first unless list_ready (the
// list of the new map, built by launch_map_update)
hipError_t launch_fill_particles(lb_ctx* c, const uint16_t* owner, bool forces,
                                 bool list_ready = false);
hipError_t launch_integrate(lb_ctx* c);
hipError_t launch_clear_accumulators(lb_ctx* c);

// adjoint
hipError_t launch_loss(lb_ctx* c, double* L_dev, double* seedA, double* seedB);
int backward(lb_ctx* c, const double* seedA, const double* seedB, double* dL_drhoA0,
             double* dL_dG, double* dL_dg);
int record_checkpoint(lb_ctx* c);

// domain size
void free_fft(lb_ctx* c);

inline char* wptr(lb_ctx* c, size_t off) { return static_cast<char*>(c->B.work) + off; }
inline char* aptr(lb_ctx* c, size_t off) { return static_cast<char*>(c->B.adjoint) + off; }
inline double* pstate(lb_ctx* c) { return static_cast<double*>(c->B.particles); }
inline double* pacc(lb_ctx* c) {
  return static_cast<double*>(c->B.particles) + size_t(c->P.max_particles) * 32;
}

}  // namespace lbh
