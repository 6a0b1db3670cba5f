/*
 * lbhip.h -- C interface of the MI355X (gfx950) implementation of the LBsoft
 * two-component lattice-Boltzmann + colloid time step.
 *
 * Method: Bonaccorso et al., "LBsoft: a parallel open-source software for
 * simulation of colloidal systems" (arXiv 2004.04080). One call of lb_step
 * advances the state by the eight-step particle sequence of Sec. 3.1:
 * moments (Eq. rho, vel, scvel), fluid-node destruction and creation
 * (Eq. distr, creat), Hertz contacts (Eq. hertzpot), virtual solid densities
 * and Shan-Chen forces (Eq. soliddens, shanchen, shanchen2), the EDM collision
 * (Eq. lbsbgk), moving halfway bounce-back with link momentum exchange
 * (Eq. LADDFLBE, UPI, LADDFORCE, FORCEPARTEQ, TORQUEPARTEQ), the rotational
 * leap-frog of the spheres (Eq. lf, quatder, svanimpl) and streaming (Eq. bgk2).
 *
 * Conventions
 *  - Node index n = x + nx*(y + ny*z); lattice units throughout.
 *  - Populations travel across the interface only as FP64 "post-streaming"
 *    values f^k_i(n, t) on fluid nodes, layout [k][i][n], direction order of
 *    lb_lattice(). Inside the library they are stored in FP32 or FP64 as
 *    deviations f_i - w_i rho0_k from the lattice weights.
 *  - Device buffers are allocated and owned by the caller (sizes from
 *    lb_required_sizes) and must outlive the context; the library never
 *    frees them. All device work is queued on the stream given to lb_init;
 *    calls marked "synchronises" wait for that stream.
 *  - Every call returns an lb_status (0 = success, < 0 = error); nothing
 *    throws across the interface. Parameter checks run on the host before
 *    any device work, so they need no GPU.
 *  - A context is not thread-safe; use one context per stream.
 */
#ifndef LBHIP_H
#define LBHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lb_status {
  LB_OK = 0,
  LB_E_ARG = -1,            /* invalid parameter or null pointer                      */
  LB_E_SHAPE = -2,          /* a buffer is smaller than required / size mismatch      */
  LB_E_OVERLAP = -3,        /* spheres overlap each other or a wall                   */
  LB_E_CAPACITY = -4,       /* more spheres than params.max_particles                 */
  LB_E_NONFINITE = -5,      /* a NaN or Inf appeared in the fluid                     */
  LB_E_PARTICLE_SPEED = -6, /* a sphere moved more than half a node in one step; the
                               state after that step is not meaningful               */
  LB_E_HIP = -7,            /* a HIP runtime call failed                              */
  LB_E_STATE = -8           /* call not valid in the current state                    */
} lb_status;

typedef enum lb_precision {
  LB_FP32 = 0, /* populations and fields in FP32 (deviations from w_i rho0_k)          */
  LB_FP64 = 1  /* populations and fields in FP64 (deviations from w_i rho0_k)          */
} lb_precision;

typedef struct lb_params {
  int32_t nx, ny, nz;       /* box; x and y are always periodic                       */
  int32_t walls;            /* 0: z periodic; 1: solid wall layers z = 0, z = nz-1    */
  double  wall_u_lo[3];     /* velocity of the z = 0 wall (Eq. bbv)                   */
  double  wall_u_hi[3];     /* velocity of the z = nz-1 wall                          */
  int32_t ncomp;            /* 1 or 2 fluid components                                */
  double  tau[2];           /* BGK relaxation times (> 1/2), Eq. viscosity            */
  double  G;                /* Shan-Chen coupling G_C, Eq. shanchen                   */
  double  sc_norm;          /* normalisation s of the Shan-Chen stencil:
                               F_k = -G s rho_k sum_i w_i psi_kbar(n + c_i) c_i.
                               s = 1 is the printed equation (repulsive sign)        */
  double  g[3];             /* body acceleration, force density rho_k g               */
  double  rho0[2];          /* deviation reference per component (e.g. 1.0)          */
  int32_t precision;        /* lb_precision                                           */
  int32_t max_particles;    /* capacity for spheres (0 = none), at most 65534         */
  double  radius;           /* sphere radius R (< min box size / 2)                   */
  double  particle_density; /* sphere mass m = density * 4/3 pi R^3, I = 2/5 m R^2    */
  double  hertz_K;          /* Hertz constant K, Eq. hertzpot                         */
  double  hertz_d0;         /* contact onset distance (e.g. 2R + 1)                   */
  double  hertz_rcap;       /* distance below which the contact force is capped      */
  double  zeta[2];          /* wetting constants zeta_ads, Eq. soliddens              */
  double  rho_fallback[2];  /* density of a created node that has no fluid neighbour  */
  int32_t rotate;           /* integrate the rotational motion (Eq. lf3, lf4)         */
  int32_t particles_fixed;  /* spheres are static obstacles (no map updates, no pair
                               forces, no integration); needed by lb_backward         */
  int32_t checkpoint_every; /* > 0: lb_step records a checkpoint every that many
                               steps so that lb_backward can run (see there)         */
  int32_t max_record_steps; /* number of steps lb_step may record (with checkpoints) */
  /* Janus wetting of the spheres (Sec. 4, benchmark input "force shanchen
   * angle/particel"): on a frontier node at angle theta (degrees) from the
   * sphere's body x axis, zeta of Eq. soliddens is +janus_zeta[0] S(theta) for
   * component A and -janus_zeta[1] S(theta) for B, S = 2t^2(3 - 2t) - 1 with
   * t = clamp((janus_theta0 + janus_width/2 - theta) / janus_width, 0, 1).
   * janus = 0 keeps the constant zeta[k]; walls always use zeta[k].        */
  int32_t janus;
  double  janus_theta0, janus_width, janus_zeta[2];
  /* Lubrication between spheres (Eq. libric), on when lub_mu > 0: for a gap
   * h = |r_ij| - 2R below lub_hn, F_i = -6 pi lub_mu R^2/4 (1/h - 1/lub_hn)
   * ((v_i - v_j) . e_ij) e_ij with e_ij = r_ij/|r_ij|, r_ij = x_j - x_i, and h
   * held at lub_hcap below it (benchmark input: 0.1, 0.67, 0.5). Added to the
   * pair force; velocities at t - 1/2.                                      */
  double  lub_mu, lub_hn, lub_hcap;
  /* Type of the two z faces when walls = 1, [0] at z = 0 and [1] at z = nz-1
   * (Sec. 2.2, Eq. bb, bbv, bbp; input directive "bound open ... type"):
   *   0 moving wall, Eq. bbv with the local density and wall_u_lo/hi;
   *   1 pressure: anti-bounce-back Eq. bbp with the density wall_rho[f][k]
   *     and the mixture velocity extrapolated from the fluid;
   *   2 velocity: Eq. bbv with wall_u_lo/hi and the density extrapolated;
   *   3 equilibrium: f_eq(wall_rho[f][k], wall_u) enters through the face.
   * Extrapolation: X_w = X(r_b) + (X(r_b) - X(r_b')) / 2, r_b the fluid node
   * next to the face and r_b' the next one inwards (X(r_b) alone when r_b' is
   * solid). Open faces need nz >= 4; the wall layers keep their virtual
   * densities (zeta) for the Shan-Chen force.                               */
  int32_t wall_type[2];
  double  wall_rho[2][2];
} lb_params;

/* Byte sizes of the caller-owned device buffers. */
typedef struct lb_sizes {
  size_t f;          /* one population buffer; two are needed (ping-pong)           */
  size_t rho;        /* pseudo-potential field psi_k(n), [ncomp][N]                 */
  size_t owner;      /* one owner map (uint16 per node); two are needed             */
  size_t particles;  /* FP64 particle state                                         */
  size_t work;       /* scratch: cell lists, reduction partials, staging, flags     */
  size_t adjoint;    /* checkpoints and adjoint fields (0 if checkpoint_every == 0) */
} lb_sizes;

/* Caller-owned device buffers and their allocated byte sizes. */
typedef struct lb_buffers {
  void*  f[2];
  void*  rho;
  void*  owner[2];
  void*  particles;
  void*  work;
  void*  adjoint;
  lb_sizes bytes;    /* allocated sizes; each must be >= lb_required_sizes()        */
} lb_buffers;

/* Observables of the current state (FP64): the statistics of Sec. 3 and the
 * output keys of App. C (masses, momenta, extrema, particle momentum and
 * energies). */
typedef struct lb_obs {
  int64_t step;          /* steps taken since lb_init                                 */
  int64_t fluid_nodes;   /* fluid nodes of the current map                            */
  double  mass[2];       /* sum over fluid nodes of rho_k                              */
  double  momentum[3];   /* bare momentum: sum over fluid nodes and components of
                            sum_i f_i c_i                                              */
  double  rho_min[2], rho_max[2];
  double  u_max;         /* max over fluid nodes of |u| (mixture velocity, Eq. scvel)  */
  double  particle_momentum[3];
  double  particle_ke;   /* sum 1/2 m v^2                                              */
  double  particle_ke_rot; /* sum 1/2 I w^2                                            */
  int32_t nparticles;
  int32_t flags;         /* bit 0: particle speed exceeded, bit 1: non-finite fluid,
                            bit 2: frontier list overflow (ruled out by its sizing)    */
  double  phys_momentum[3]; /* physical momentum (Sec. 2.3, after Eq. lbsbgk): the bare
                            momentum plus half the force density summed over the fluid,
                            F_k = Shan-Chen force (Eq. shanchen, virtual densities of the
                            current map on the frontier) + rho_k g                     */
  double  flink_abs;     /* sum over spheres and links of |F_link| (Eq. LADDFORCE) of
                            the last step: the scale of the particle force tolerances  */
} lb_obs;

/* Per-sphere record of lb_get_particles / lb_set_particles, FP64, in this order. */
#define LB_PREC 50
enum {
  LB_P_X = 0,        /* position x(t) [3]                                     */
  LB_P_V = 3,        /* velocity v(t - 1/2) [3]                               */
  LB_P_W = 6,        /* angular velocity w(t - 1/2), space frame [3]           */
  LB_P_Q = 9,        /* orientation quaternion q(t) [4]                        */
  LB_P_FPREV = 13,   /* fluid force F_liq(t - 1/2) [3]                         */
  LB_P_TPREV = 16,   /* fluid torque T_liq(t - 1/2) [3]                        */
  /* force terms of the last completed step: */
  LB_P_FD = 19, LB_P_TD = 22,   /* destroyed nodes (Eq. distr)                 */
  LB_P_FC = 25, LB_P_TC = 28,   /* created nodes (Eq. creat)                   */
  LB_P_FH = 31,                 /* Hertz contacts (Eq. hertzpot)               */
  LB_P_FSC = 34, LB_P_TSC = 37, /* Shan-Chen on frontier solids (Eq. shanchen2) */
  LB_P_FLIQ = 40, LB_P_TLIQ = 43, /* link momentum exchange (Eq. FORCEPARTEQ,
                                     TORQUEPARTEQ)                             */
  LB_P_FLABS = 46,   /* sum over links of |F_link|                             */
  LB_P_MASS = 47, LB_P_INERTIA = 48,
  LB_P_HAVEPREV = 49 /* 1 when FPREV/TPREV hold a previous half-step value     */
};

/* Infrastructure (no passage of the paper defines these): library version
 * string; a static description of a status code; the last error message of
 * a context (or of the last failed lb_init when ctx is NULL), owned by the
 * library and valid until the next call on that context. */
const char* lb_version(void);
const char* lb_strerror(int status);
const char* lb_last_error(const struct lb_ctx* ctx);

/* D3Q19 velocities c [19][3] and weights w [19] in the library's order
 * (Sec. 2.1). Host only. */
int lb_lattice(int32_t* c, double* w);

/* Device buffer sizes for params: the two population buffers of the
 * collide-stream sequence (Sec. 3.1; the pull form of Eq. bgk2, 2 x ncomp x
 * 19 values per node), the pseudo-potential field (Eq. shanchen), the two
 * owner maps of the moving-boundary scheme (Sec. 2.3), the sphere records
 * and accumulators, the work buffer (lists, reductions, staging) and, with
 * checkpoint_every > 0, the adjoint's checkpoints. Host only; validates
 * params. Errors: LB_E_ARG (null or invalid parameters), LB_E_SHAPE (box too
 * large: a population plane must stay below 4 GiB). */
int lb_required_sizes(const lb_params* params, lb_sizes* out);

/* Create a context on the caller's buffers and stream (hipStream_t, NULL =
 * default stream) and set f^k_i = f_eq(rho0_k(n), u0(n)) (Eq. LEQ).
 * rho0: host FP64 [ncomp][N]; u0: host FP64 [N][3] or NULL for rest.
 * Synchronises. Errors: LB_E_ARG, LB_E_SHAPE, LB_E_HIP. */
int lb_init(const lb_params* params, const lb_buffers* buffers, const double* rho0,
            const double* u0, void* hip_stream, struct lb_ctx** out);

/* Add n spheres of the common radius (Sec. 2.4): host FP64 centres x [n][3],
 * velocities v [n][3] (NULL = 0), angular velocities w [n][3] (NULL = 0),
 * quaternions q [n][4] (NULL = identity). Nodes inside a sphere become solid
 * and their populations are discarded. Allowed before the first step only.
 * Synchronises. Errors: LB_E_CAPACITY, LB_E_OVERLAP (centres closer than
 * 2R, or a sphere reaching a wall layer), LB_E_STATE, LB_E_HIP. */
int lb_add_particles(struct lb_ctx* ctx, int32_t n, const double* x, const double* v,
                     const double* w, const double* q);

/* Advance nsteps time steps (Sec. 3.1, eight-step sequence). Asynchronous on
 * the context's stream. With moving spheres the map update of each step runs
 * on a second stream that the context creates on first use (default
 * priority); it waits for the context's stream and is joined back into it
 * before the step goes on, so callers see one stream. A sphere faster than
 * 1/2 node per step is flagged and reported by the next synchronising call.
 * With checkpoint_every > 0 the steps are recorded for lb_backward
 * (LB_E_CAPACITY beyond max_record_steps).
 * Graph capture: a step issues only kernel launches and event records and
 * waits (buffers are cleared by a kernel, not a memset), so a caller may
 * capture lb_step on a non-default context stream into a HIP graph once the
 * context has stepped eagerly at least once (the side stream and its events
 * then exist). A graph of an even number of steps ends on the buffers it
 * starts from and may be replayed any number of times; the context's step
 * counter (lb_obs.step) advances when steps are captured, not when they are
 * replayed. Not with checkpoint_every > 0 or with per-phase timing on, whose
 * host-side records would not follow the replays.
 * Errors: LB_E_ARG, LB_E_HIP, LB_E_CAPACITY. */
int lb_step(struct lb_ctx* ctx, int32_t nsteps);

/* FP64 observables of the current state. Recomputes the pseudo-potential of
 * the current state for the force density (as lb_get_psi). Synchronises.
 * Errors: LB_E_PARTICLE_SPEED / LB_E_NONFINITE / LB_E_CAPACITY (node-list
 * overflow) when flagged (out is still filled). */
int lb_observables(struct lb_ctx* ctx, lb_obs* out);

/* lb_observables for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same outputs and errors, computed by the same kernels, with the
 * reduction partials and the sphere sums in a static device array of the
 * library (at most 1024 partial records of 16 doubles, its final record and
 * 8 sphere sums: about 131 KB, held on each device the library runs on until
 * the process ends) instead of the context's work buffer. It calls no
 * hipMalloc, hipFree or other allocating routine and allocates no host heap
 * memory. Every call on a device shares that device's array: calls that
 * overlap in time on one device (two streams, two threads) race and must not
 * be made. Errors as lb_observables, plus LB_E_CAPACITY if a reduction would
 * need more than the array holds (no box the library accepts does) and
 * LB_E_STATE if the array's address could not be taken at lb_init. The
 * sphere sums are added in another order than lb_observables adds them (a
 * fixed tree instead of a compensated serial sum), so they may differ in the
 * last bits. Synchronises. */
int lb_observables_noalloc(struct lb_ctx* ctx, lb_obs* out);

/* Moments of the current state on fluid nodes (0 on solid nodes), host FP64:
 * rho [ncomp][N] and mixture velocity u [N][3] (Eq. scvel; NULL to skip). Synchronises. */
int lb_get_fields(struct lb_ctx* ctx, double* rho, double* u);

/* Pseudo-potential psi_k(n) of the last step (fluid densities plus virtual
 * densities of frontier solids, Eq. soliddens), host FP64 [ncomp][N]. Synchronises. */
int lb_get_psi(struct lb_ctx* ctx, double* psi);

/* Post-streaming populations f^k_i(n, t), host FP64 [ncomp][19][N] (full
 * values, direction order of lb_lattice, 0 on solid nodes). Synchronises. */
int lb_get_populations(struct lb_ctx* ctx, double* f);
/* Replace the populations of the fluid nodes of the current map (same layout).
 * Values are rounded to the storage precision. Synchronises. */
int lb_set_populations(struct lb_ctx* ctx, const double* f);

/* Owner map of the current state: 0 fluid, p+1 node of sphere p, -1 wall;
 * host int32 [N]. Synchronises. */
int lb_get_owner(struct lb_ctx* ctx, int32_t* owner);

/* Sphere records (Sec. 2.4-2.5 particle state; LB_PREC doubles each), host
 * FP64 [nparticles][LB_PREC]. lb_set_particles writes v, w, q, FPREV, TPREV
 * and HAVEPREV of the existing spheres; every value must be finite and q
 * non-zero (LB_E_ARG). Before the first step it also takes new positions
 * (wrapped into the box), checks them like lb_add_particles (LB_E_OVERLAP)
 * and re-rasterises the map: nodes that a moved sphere frees keep the
 * populations they held before the spheres covered them (those of lb_init
 * unless lb_set_populations changed them). After the first step a position
 * that differs from the stored one is refused (LB_E_STATE): a moved sphere
 * needs the node events of a step; lb_set_state replaces a whole state.
 * Nothing is changed when a check fails. Synchronises. */
int lb_get_particles(struct lb_ctx* ctx, double* rec);
int lb_set_particles(struct lb_ctx* ctx, const double* rec);
int lb_num_particles(const struct lb_ctx* ctx);

/* Loss of the differentiation study on the current state:
 * L = sum over fluid nodes of |grad_lat phi|^2, phi = psi_A - psi_B,
 * grad_lat phi(n) = 3 sum_i w_i phi(n + c_i) c_i, psi with the virtual
 * densities of the current map. L to host; optionally dL/dpsi_k(n) into
 * device FP64 arrays dL_dpsiA, dL_dpsiB [N] (NULL to skip). Synchronises. */
int lb_loss(struct lb_ctx* ctx, double* L, double* dL_dpsiA, double* dL_dpsiB);

/* Reverse-mode derivative of a loss of the final pseudo-potential through
 * every recorded step, with checkpoint recomputation. Inputs: device FP64
 * seeds dL/dpsi_k(n) at the final state [N] each (dL_dpsiB may be NULL).
 * Outputs: device FP64 dL/drho0_A(n) [N] of the initial density of component
 * A (the state set by lb_init with u0 = 0), and host dL/dG and dL/dg[3].
 * Requires checkpoint_every > 0, equal relaxation times, no moving spheres
 * (particles_fixed or none) and zero wall velocities. Synchronises.
 * Errors: LB_E_STATE, LB_E_ARG, LB_E_HIP. */
int lb_backward(struct lb_ctx* ctx, const double* dL_dpsiA, const double* dL_dpsiB,
                double* dL_drhoA0, double* dL_dG, double dL_dg[3]);

/* Restart snapshot of the whole evolving state (the paper's restart files,
 * input directives of App. A): the populations as stored (storage precision,
 * pull form), both owner maps and the sphere records, behind a small header
 * (box, components, precision, walls, sphere count, step). The blob is
 * opaque, host memory owned by the caller; lb_state_bytes gives its size.
 * lb_get_state synchronises and copies the state out. lb_set_state
 * synchronises and replaces the state of a context created with the same
 * box, components, precision and walls and at least as many sphere slots;
 * the adjoint recording restarts empty. Errors: LB_E_ARG (NULL, short
 * buffer, bad header), LB_E_SHAPE (blob of another configuration),
 * LB_E_CAPACITY (more spheres than max_particles), LB_E_HIP. Populations that
 * are not finite are accepted and reported by lb_observables (flags bit 1). */
int lb_state_bytes(const struct lb_ctx* ctx, size_t* bytes);
int lb_get_state(struct lb_ctx* ctx, void* blob, size_t bytes);
int lb_set_state(struct lb_ctx* ctx, const void* blob, size_t bytes);

/* Average domain size of the phase field (Sec. 4, Eq. Cluster_L_eq):
 * L = 2 pi sum_s S(s) / sum_s k_s S(s) over the shells s = 1 .. min(L)/2 of
 * the structure factor S(k) = |phi'(k)|^2 / N of phi' = phi - <phi>,
 * phi = (rho_A - rho_B) / (rho_A + rho_B) on the fluid nodes of the current
 * state (0 on solids). Shell s holds the wave vectors k_d = 2 pi m_d / L_d
 * with round(|k| / dk) = s, dk = 2 pi / min(nx, ny, nz); S(s) is their mean.
 * Two components only. The transform runs in FP64 on the context's stream.
 * lb_domain_workspace gives the device workspace size in bytes and the shell
 * count (min(L)/2 + 1, shell 0 included); it creates the FFT plan on first
 * use (the only allocation, made by the FFT library; released by lb_free).
 * lb_domain_size takes a caller-owned device workspace of that size, writes
 * L to the host (NaN when phi' vanishes) and, unless S is NULL, the shell
 * means S(0..nshell-1) to a host array of nshell doubles. Synchronises.
 * Errors: LB_E_ARG (NULL, small workspace or array), LB_E_STATE (one
 * component), LB_E_HIP. */
int lb_domain_workspace(struct lb_ctx* ctx, size_t* bytes, int32_t* nshell);
int lb_domain_size(struct lb_ctx* ctx, void* work, size_t work_bytes, double* L, double* S,
                   int32_t nshell);

/* Streaming probes (measurement only, not part of the step): the time of a
 * plain bandwidth-bound kernel on this device, the ceiling against which the
 * step's kernels are read. kind 0 reads `bytes` of src (16-byte chunks; the
 * first 16 bytes of dst are only a sink that finite inputs of order one never
 * reach); kind 1
 * writes `bytes` of dst; kind 2 copies `bytes` from src to dst; kind 3 moves
 * two components of 19 FP32 planes of N = nx ny nz nodes in the pattern of
 * the fused step: plane i of node n is gathered from node n - c_i (D3Q19,
 * periodic) of src and stored at n in dst (src and dst each 2*19*N*4 bytes,
 * bytes >= that; one plane below 4 GiB). kind 4 moves the same planes as a
 * z-march that also takes the moments in its sweep (the pattern of a step
 * without a separate density pass, Sec. 3.1): workgroups own 128 x 8 columns
 * and walk 128 z-planes, gathering each plane for the column and a one-node
 * ring around it, and store dst_{k,i}(n) = g_{k,i}(n) + 1e-3 sum_{j=1..18} j
 * s_{1-k}(n + c_j), with g the values kind 3 stores and s_k(m) the sum over i
 * of g_{k,i}(m); nx a multiple of 128 and ny of 8 (else LB_E_SHAPE). Device
 * pointers, 16-byte aligned, owned by the caller. One untimed launch, then reps launches on `stream`
 * (hipStream_t) between HIP events; *ms_per_launch gets their mean.
 * Synchronises. Errors: LB_E_ARG, LB_E_SHAPE, LB_E_HIP. */
int lb_probe_stream(int32_t kind, const void* src, void* dst, size_t bytes, int32_t nx,
                    int32_t ny, int32_t nz, int32_t reps, void* stream, double* ms_per_launch);

/* Debugging the bounce-back (Sec. 3.1, steps 6 and 8: each reflected
 * population has exactly one writer): with counts non-NULL, every later
 * lb_step runs the collide variant that also adds 1 to counts[k][i][n]
 * (device uint32 [ncomp][19][N], zeroed and owned by the caller) for every
 * population it stores into slot (k, i, n) of the output buffer: the
 * post-collision values of fluid nodes, the zeros of solid nodes and every
 * reflection. After s steps every entry must be s. NULL switches it off.
 * Walls or spheres required (LB_E_STATE). Slower; for tests only. */
int lb_debug_count_writes(struct lb_ctx* ctx, void* counts);

/* Wait for all work queued by the context (infrastructure: synchronises the
 * context's stream; the side stream of the map update joins that stream
 * within every step). Errors: LB_E_ARG, LB_E_HIP. */
int lb_sync(struct lb_ctx* ctx);

/* Per-phase GPU timing with HIP events recorded on the context's stream around
 * the kernels of each phase of lb_step, the phases of the paper's step
 * sequence (Sec. 3.1) whose throughput the paper reports per lattice update
 * (Eq. glups). lb_timing(ctx, 1) clears the totals
 * and starts recording; lb_timing(ctx, 0) stops recording and keeps the
 * totals. lb_timing_read synchronises and returns the summed milliseconds
 * and interval counts per phase (phase 1 records the map update on the side
 * stream and the node events on the context's stream, two per step):
 * 0 moments (density), 1 sphere map/events/pairs, 2 virtual-density fills,
 * 3 collide-stream-bounce-back with the link momentum exchange,
 * 4 sphere integration. */
#define LB_NPHASE 5
int lb_timing(struct lb_ctx* ctx, int enable);
int lb_timing_read(struct lb_ctx* ctx, double ms[LB_NPHASE], int64_t count[LB_NPHASE]);

/* Destroy a context (infrastructure): releases the library's own objects
 * (streams, events, the FFT plan) but not the caller's buffers. NULL is
 * ignored. */
void lb_free(struct lb_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
