/*
 * sph.h -- C ABI of the MI355X (gfx950) SPH hot path.
 *
 * One simulation step follows the paper's simulation loop (arXiv 2511.15908,
 * Alg. 2 and Sec. 3.2): rigid-body particles are re-placed from their parent
 * transform, a uniform-grid spatial hash orders the particles (here a
 * counting sort by Morton cell slot with reorder and cell start/end tables),
 * soft-body spring
 * forces are applied, then the SPH density/pressure pass and the force pass of
 * Alg. 1 run over the neighbours, the point forces on each grabbed body are
 * reduced into a force and torque (Sec. 3.2, Sec. 3.3), and fluid and soft
 * particles are integrated with the semi-implicit Euler scheme (Eq. euler).
 * The body wrench is the haptic output of Fig. 1 / Sec. 3.3; the device pose
 * enters through sph_set_body_pose.
 *
 * Conventions for every call:
 *  - All functions return sph_status and never abort or throw.  Argument
 *    errors are reported before any device work is enqueued.  A HIP runtime
 *    failure returns SPH_ERR_DEVICE and sph_last_error() holds its text; after
 *    it the context only accepts sph_destroy (SPH_ERR_STATE otherwise).
 *  - Host pointers are plain C arrays owned by the caller and only read or
 *    written during the call.  The device workspace is one caller-allocated
 *    block (e.g. a torch uint8 tensor) borrowed by the context until
 *    sph_destroy; the library allocates no device memory of its own.
 *  - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; calls that return data to the host synchronise it.
 *  - One context per host thread; different contexts are independent.
 */
#ifndef SPH_H_
#define SPH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 1u

typedef struct sph_ctx sph_ctx;

typedef enum {
    SPH_OK = 0,
    SPH_ERR_ARG = 1,         /* invalid argument (null pointer, bad size, bad id, bad value) */
    SPH_ERR_WORKSPACE = 2,   /* workspace missing, misaligned (256 B) or smaller than sph_workspace_size */
    SPH_ERR_DEVICE = 3,      /* HIP runtime error; see sph_last_error */
    SPH_ERR_STATE = 4,       /* call not valid in the context's state (after a device error) */
    SPH_ERR_UNSTABLE = 5,    /* a particle velocity or position became non-finite or exceeded v_max */
    SPH_ERR_UNSUPPORTED = 6, /* precision/flag/geometry the library does not implement */
    SPH_ERR_CAPACITY = 7     /* a cell neighbourhood exceeded the candidate capacity (extreme compression);
                                the step that raised it and any enqueued after it used stale density and
                                force in the overflowing cells, so the state is undefined: from then on
                                sph_step returns this status without enqueuing, syncing calls report it
                                again, and only reads and sph_destroy remain useful */
} sph_status;

typedef enum { SPH_FP32 = 0, SPH_FP64 = 1 } sph_precision;

/* Particle types: each particle has a type (Sec. 3.2 unified framework). */
enum { SPH_FLUID = 0, SPH_SOFT = 1, SPH_BOUNDARY = 2 };

/* Alternative readings of points the paper leaves open (default 0). */
enum {
    SPH_FLAG_CLAMP_NEG_PRESSURE = 1u,   /* p = max(k (rho - rho0), 0) instead of Eq. pressure as printed */
    SPH_FLAG_BOUNDARY_SINGLE_TERM = 2u, /* fluid-boundary pressure term p_i/rho_i^2 once, not mirrored */
    SPH_FLAG_NO_BOUNDARY_VISCOSITY = 4u, /* no viscosity between fluid/soft and boundary particles */
    SPH_FLAG_UNIFIED_BOUNDARY = 8u       /* Sec. 3.2 typed particles: a boundary particle is an SPH particle
                                            with mass psi_b and a density and pressure of its own (Eq.
                                            density over all neighbours, Eq. pressure); the pair force then
                                            uses rho_b, p_b instead of the mirrored rho_i, p_i.  Flag 2 has
                                            no effect under it.  sph_read_field reports boundary rho and p. */
};

/* Fields readable with sph_read_field, all in original particle-id order. */
enum {
    SPH_FIELD_X = 0,        /* double[3n] positions after the last step (or init) */
    SPH_FIELD_V = 1,        /* double[3n] velocities after the last step (or init) */
    SPH_FIELD_RHO = 2,      /* double[n] density of the last step (fluid/soft; boundary 0, own rho_b with flag 8) */
    SPH_FIELD_PRESSURE = 3, /* double[n] pressure p = k (rho - rho0) of the last step */
    SPH_FIELD_FORCE = 4,    /* double[3n] total force of the last step: pair forces + m g + springs
                               (fluid/soft); reaction force of kinematic boundary particles; 0 static */
    SPH_FIELD_PSI = 5,      /* double[n] boundary volume mass psi_b = rho0 V_b (0 for fluid/soft) */
    SPH_FIELD_KEY = 6,      /* uint32[n] Morton cell key of the last neighbour search */
    SPH_FIELD_SPRING = 7    /* double[3n] spring force of the last step (soft; 0 otherwise) */
};

typedef struct {
    uint32_t abi_version;      /* must be SPH_ABI_VERSION */
    int32_t precision;         /* sph_precision of particle arithmetic; the wrench is always FP64 */
    uint32_t flags;            /* SPH_FLAG_* */
    uint32_t smoothing_window; /* K >= 1 samples in the rolling average (Sec. 3.3: some tens of cycles) */
    double h;                  /* smoothing length; kernel support is 2h (Eq. kernel) [m] */
    double rho0;               /* rest density (Eq. pressure) [kg/m^3] */
    double k_pressure;         /* pressure constant k (Eq. pressure) [m^2/s^2] */
    double nu;                 /* kinematic viscosity nu (Alg. 1) [m^2/s] */
    double gravity[3];         /* external acceleration, F_ext = m g (Alg. 1) [m/s^2] */
    double dt;                 /* time step (Eq. euler) [s] */
    double domain_lo[3];       /* uniform grid bounds [m]; particles outside use the edge cells */
    double domain_hi[3];
    double v_max;              /* |v| above this flags SPH_ERR_UNSTABLE; 0 = only non-finite */
    uint32_t max_probes;       /* capacity of density probe points (sph_set_probes), <= 2^20; 0 = none */
    uint32_t log_steps;        /* capacity of the per-step body log (sph_read_log), steps; 0 = none */
    uint32_t track_steps;      /* capacity of each body's pose track (sph_set_body_track); 0 = none */
    uint32_t reserved[5];      /* must be zero */
} sph_params;

typedef struct {               /* caller-owned host arrays, read only during sph_init */
    uint32_t n;                /* number of particles (all types) */
    const double *x;           /* [3n] initial positions (rounded to the run precision) */
    const double *v;           /* [3n] initial velocities */
    const double *mass;        /* [n] mass of fluid/soft particles and of the particles of free
                                  rigid bodies (their mass elements); ignored for other boundary
                                  particles */
    const uint8_t *type;       /* [n] SPH_FLUID / SPH_SOFT / SPH_BOUNDARY */
    const int32_t *object;     /* [n] object id of boundary particles (0..n_objects-1), -1 otherwise */
    uint32_t n_objects;        /* boundary objects */
    const uint8_t *object_kinematic; /* [n_objects] 0: static, 1: pose-driven (grabbed) body,
                                        2: free rigid body (Sec. 3.2 rigid bodies under the summed
                                        particle forces; grab/release below) */
    const double *object_pose0;      /* [7 n_objects] reference point c[3] and unit quaternion
                                        q[4] = (w,x,y,z) of each object; body-frame offsets are
                                        taken from x at this pose.  For a free rigid body the
                                        reference point is replaced by its particles' centre of
                                        mass (the body frame keeps q) */
    uint32_t n_springs;        /* soft-body springs (Sec. 3.2 mass-spring model) */
    const uint32_t *spring_ij; /* [2 n_springs] particle ids of the two ends (soft particles) */
    const double *spring_L0;   /* [n_springs] rest length [m] */
    const double *spring_k;    /* [n_springs] stiffness [N/m] */
    const double *spring_c;    /* [n_springs] damping along the spring [N s/m] */
} sph_scene;

typedef struct {               /* read-only facts about a context */
    uint32_t n, n_fluid, n_soft, n_boundary, n_body_particles, n_kinematic;
    uint32_t grid_dims[3], grid_bits;   /* cells per axis, Morton bits per axis */
    uint32_t cell_slots;                /* 2^(3 grid_bits) */
    uint32_t max_candidates;            /* per-cell neighbourhood capacity */
    uint64_t steps;                     /* steps taken */
    double cell_size;                   /* 2h (1 + 2^-10) */
} sph_info;

/*
 * Bytes of device workspace sph_init needs for these params and scene: the
 * particle state the simulation loop of Alg. 2 carries from step to step
 * (positions, velocities, types, body slots, spring table), the uniform-grid
 * hash of Alg. 2 (keys, sort buffers, cell start/end tables, Sec. 3.1), the
 * density/pressure and force arrays of Alg. 1 and the FP64 body tables
 * (Sec. 3.2, 3.3).  Host-only (no device work); SPH_ERR_ARG /
 * SPH_ERR_UNSUPPORTED as sph_init would report them.
 */
sph_status sph_workspace_size(const sph_params *params, const sph_scene *scene, size_t *bytes);

/*
 * Create a context: validate, copy the scene into the workspace (async on
 * hip_stream, the call synchronises before returning), compute boundary
 * volumes psi_b from the initial configuration and sort the particles once.
 * d_workspace: device pointer, 256-byte aligned, ws_bytes >= sph_workspace_size.
 */
sph_status sph_init(const sph_params *params, const sph_scene *scene, void *d_workspace,
                    size_t ws_bytes, void *hip_stream, sph_ctx **out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sph_init
 * with the workspace taken from a device array inside the library instead of
 * the caller's, SPH_STATIC_WORKSPACE_BYTES on each device the library runs on,
 * held until the process ends.  The array is on the calling thread's current
 * device; hip_stream must belong to that device.  Everything after init
 * (sph_step and the rest) is unchanged; sph_destroy hands the array back.
 * The array keeps the previous context's contents; init writes or clears
 * everything a step reads.  One such context per device at a time: a second
 * sph_init_static on a device whose array is held returns SPH_ERR_STATE (two
 * contexts on one array would overwrite each other's state); a scene whose
 * sph_workspace_size exceeds the array returns SPH_ERR_WORKSPACE.  No device
 * memory is allocated by this call or by any later call on the context.
 */
#define SPH_STATIC_WORKSPACE_BYTES (128u << 20)
sph_status sph_init_static(const sph_params *params, const sph_scene *scene, void *hip_stream, sph_ctx **out);

/*
 * Pose of a kinematic object from the haptic device (Sec. 3.3, Fig. 1):
 * reference point c, orientation q (w,x,y,z; normalised by the library),
 * linear velocity v and angular velocity w (world frame).  Enqueued on the
 * context's last stream; takes effect at the next step.  Between calls the
 * pose advances every step by c += v dt, q <- normalise(q + dt/2 (0,w) q).
 * Errors: SPH_ERR_ARG for a static or unknown object or a zero/non-finite q.
 */
sph_status sph_set_body_pose(sph_ctx *ctx, uint32_t object, const double c[3], const double q[4],
                             const double v[3], const double w[3]);

/*
 * Free rigid bodies (object_kinematic 2).  Mass m = sum of the body's particle
 * masses, inertia about their centre of mass from the same particles; each
 * step, after the wrench, the velocities take a semi-implicit Euler step in
 * binary64: v += dt (F/m + g), w += dt I_w^-1 (T - w x (I_w w)) with
 * I_w = R I R^T (Euler's equations), then the pose advances as for a
 * kinematic body.  There is no contact between rigid bodies or with the tank
 * (boundary-boundary pairs exert nothing).  sph_set_body_pose also sets the
 * state of a free body.
 * sph_grab_body: the body follows sph_set_body_pose (device-driven) until
 * sph_release_body hands it back to the integration; both keep the current
 * pose and velocities and restart the rolling average.  SPH_ERR_ARG for an
 * object that is not a free rigid body.
 * sph_get_body_state: current c, q, v, w of a kinematic or free body
 * (synchronises the stream).
 */
sph_status sph_grab_body(sph_ctx *ctx, uint32_t object);
sph_status sph_release_body(sph_ctx *ctx, uint32_t object);
sph_status sph_get_body_state(sph_ctx *ctx, uint32_t object, double c[3], double q[4], double v[3], double w[3]);

/*
 * Batches: independent scenes stepped together (one context, one launch per
 * kernel for all scenes).  params[k] and scenes[k] describe scene k exactly
 * as for sph_init; the scenes share precision, dt, gravity, v_max,
 * smoothing_window, log_steps, track_steps and max_probes.  Each scene
 * keeps its own h, grid, constants and flags.  In the context, particle ids,
 * object ids and spring ends of scene k follow those of scenes 0..k-1 (a
 * scene's particle i is id part0_k + i, part0_k = sum of the previous scenes'
 * n), and every call below works on those global ids.  sph_init is the batch
 * of one.
 */
sph_status sph_batch_workspace_size(const sph_params *params, const sph_scene *scenes, uint32_t n_scenes,
                                    size_t *bytes);
sph_status sph_batch_init(const sph_params *params, const sph_scene *scenes, uint32_t n_scenes, void *d_workspace,
                          size_t ws_bytes, void *hip_stream, sph_ctx **out);

/*
 * Per-step body log (params.log_steps > 0): every step appends, for each
 * kinematic or free body in kinematic-index order (ascending object id), 20
 * doubles: c[3], q[4], v[3], w[3] of the pose the step's forces saw, F[3],
 * T[3] (the wrench of sph_get_body_wrench, unsmoothed), and the record's step
 * number.  The log keeps the last log_steps steps.  sph_read_log copies the
 * kept steps, oldest first, as [steps][bodies][20] into out (n_doubles must
 * hold them), writes their number to n_steps, empties the log and
 * synchronises.
 */
sph_status sph_read_log(sph_ctx *ctx, double *out, size_t n_doubles, uint32_t *n_steps);

/*
 * Per-step probe log (params.log_steps > 0, params.max_probes > 0, at least
 * one kinematic or free body): every step also keeps the densities of the
 * current probe set (sph_set_probes) beside its body-log record.
 * sph_read_probe_log copies, for the steps sph_read_log would return (oldest
 * first), [steps][n_probes] densities into out (n_doubles must hold them) and
 * writes their number to n_steps; it does not empty the log, so call it
 * before sph_read_log, which empties both.  Steps taken under an earlier
 * probe set report that set's values.  Synchronises.  With no body, no
 * probes or no log it reports 0 steps.
 */
sph_status sph_read_probe_log(sph_ctx *ctx, double *out, size_t n_doubles, uint32_t *n_steps);

/*
 * Graph replay (enable != 0): sph_step launches a HIP graph of two captured
 * steps (captured at the first use, on that call's stream) instead of their
 * kernels one by one; an odd remainder runs as a plain step.  Needs a
 * non-default stream (SPH_ERR_ARG otherwise).  Poses, grab/release and
 * smoothing resets are plain stream work between replays; changing the probe
 * set or disabling drops the graph.  Profiling steps run without the graph.
 */
sph_status sph_set_graph(sph_ctx *ctx, int enable);

/*
 * Pose track of a kinematic (or grabbed) body: poses[k] = c[3], q[4], v[3],
 * w[3] for the k-th step from the next one on (n <= track_steps); the body
 * takes them one per step on the device (no host work per step, e.g. under
 * graph replay) and extrapolates from the last.  sph_set_body_pose ends a
 * track.  SPH_ERR_ARG for a static body, a free (released) body, n above the
 * capacity, a zero or non-finite entry.  The host array is copied; the call
 * synchronises.
 */
sph_status sph_set_body_track(sph_ctx *ctx, uint32_t object, uint32_t n, const double *poses);

/*
 * Enqueue n_steps full steps on hip_stream (no host synchronisation).  One
 * step is one pass of the simulation loop (Alg. 2): rigid placement (Sec.
 * 3.2), the spatial hash and its sorted order (Sec. 3.1, Alg. 2), spring
 * forces (Sec. 3.2), the density and pressure pass and the force pass of
 * Alg. 1 (Eqs. kernel, density, pressure), the reduction of the body
 * particles' forces into each body's force and torque (Sec. 3.2, 3.3) and
 * the semi-implicit Euler update (Eq. euler).  Errors raised on the device
 * (SPH_ERR_UNSTABLE, SPH_ERR_CAPACITY) surface at the next synchronising
 * call; SPH_ERR_STATE after a device error, SPH_ERR_CAPACITY after an overflow.
 */
sph_status sph_step(sph_ctx *ctx, uint32_t n_steps, void *hip_stream);

/*
 * Wrench exerted by the fluid and soft particles on a kinematic object
 * (gravity excluded), about its reference point c, world frame, binary64:
 * F [N], T [N m].  smoothed = 0: the last step's sample; 1: the mean of the
 * last min(K, steps since init or reset) samples (Sec. 3.3 rolling average).
 * Synchronises the stream; returns SPH_ERR_UNSTABLE / SPH_ERR_CAPACITY if a
 * step since the last check raised that condition (the values are still
 * written).
 */
sph_status sph_get_body_wrench(sph_ctx *ctx, uint32_t object, double F[3], double T[3], int smoothed);

/* Restart the rolling average of a kinematic object (grab or release). */
sph_status sph_reset_smoothing(sph_ctx *ctx, uint32_t object);

/*
 * Copy a field (SPH_FIELD_*, each defined beside its enum entry by the
 * equation it comes from: Eq. density, Eq. pressure, Alg. 1 forces, Eq. euler
 * state) into host_dst, in original particle-id order, converted to double
 * (keys as uint32); bytes must equal its size (SPH_ERR_ARG otherwise).
 * Synchronises and reports pending step errors like sph_synchronize (the
 * values are still written).
 */
sph_status sph_read_field(sph_ctx *ctx, int field, void *host_dst, size_t bytes);

/*
 * Neighbour lists N(i) = { j : |x_i - x_j| < 2h } (the support of Eq. kernel,
 * over which Alg. 1 sums; the integer decision is the canonical predicate of
 * the run precision) found by the last step's density pass, for checking (any
 * N, but it copies O(N * candidates) bytes to the host).  The extra output
 * total lets a caller size ids with a first call (ids = NULL, cap = 0).  counts[n] receives
 * |N(i)| for fluid, soft and kinematic-boundary particles (0 for static
 * boundary particles); ids receives the lists back to back in particle-id
 * order, each ascending, self included.  *total receives the total; ids is
 * only written when total <= cap.
 */
sph_status sph_debug_neighbors(sph_ctx *ctx, uint32_t *counts, uint32_t *ids, size_t cap,
                               size_t *total);

/* The same for the given particle ids only (counts[t] and lists in target order). */
sph_status sph_debug_neighbors_of(sph_ctx *ctx, uint32_t n_targets, const uint32_t *targets,
                                  uint32_t *counts, uint32_t *ids, size_t cap, size_t *total);

/*
 * Work counters accumulated on the device since init: out[0] neighbour pairs
 * of fluid/soft particles (self included), out[1] neighbour pairs of all
 * particles that receive forces (fluid, soft and kinematic boundary), out[2]
 * candidate pairs tested (64 lanes x candidates per wavefront), out[3]
 * wavefronts of the density pass, out[4] / out[5] wavefront iterations of the
 * density / force neighbour loops (each iteration serves up to 64 pairs).
 * Synchronises the stream.
 */
sph_status sph_get_stats(sph_ctx *ctx, uint64_t out[6]);

/* Facts about the context (sizes, grid). */
sph_status sph_get_info(const sph_ctx *ctx, sph_info *info);

/* Wait for the context's stream; report SPH_ERR_UNSTABLE / SPH_ERR_CAPACITY if raised. */
sph_status sph_synchronize(sph_ctx *ctx);

/*
 * Per-phase GPU timing with HIP events recorded on the step's stream.
 * sph_profile_begin(ctx, max_steps) arms it for the next max_steps steps;
 * sph_profile_begin_sampled(ctx, max_steps, every) records only on every
 * every-th of them (the first, the every+1-th, ...), so that the event
 * records (a few microseconds each, two per phase) weigh less on the steps
 * timed around them; every = 0 is SPH_ERR_ARG.  Steps with events run
 * eagerly, not as graph replays.  sph_profile_read synchronises and writes,
 * for each phase id 0..n_phases-1 (see sph_profile_phase_name), the summed
 * milliseconds and launch count over the steps that recorded events.  The
 * body placement runs inside the key launch, the springs inside the density
 * launch and the body wrench inside the integration launch, so their phases
 * ("place", "springs", "wrench") read 0.
 */
sph_status sph_profile_begin(sph_ctx *ctx, uint32_t max_steps);
sph_status sph_profile_begin_sampled(sph_ctx *ctx, uint32_t max_steps, uint32_t every);
sph_status sph_profile_read(sph_ctx *ctx, double *ms, uint32_t *launches, uint32_t n_phases);
const char *sph_profile_phase_name(uint32_t phase);

/*
 * Density probes: the density field of the fluid and soft particles at given
 * points (Sec. 3.4: density at grid points from particle proximity and the
 * smoothing kernel, reusing the uniform-grid hash),
 *   rho(p) = sum_{j fluid/soft, predicate(p, x_j)} m_j W(|p - x_j|),
 * evaluated every step on the state the force pass sees (after placement, before
 * integration).  points: [3n] host array; frame: [n] object id of a kinematic
 * body whose frame the point is given in (moves with the body), or -1 for world
 * coordinates.  n <= max_probes.  Replaces the previous set (the host arrays are
 * copied; the caller keeps ownership); the values read zero until the next
 * step.  SPH_ERR_ARG for n > max_probes, a non-finite point or a frame that is
 * not a kinematic object.  sph_read_probes copies the last step's values into
 * the caller's [n] doubles, n equal to the count last set, and synchronises;
 * it reports pending step errors like sph_synchronize.  The probe points are
 * rounded to the run precision; the support test is the particle-pair one.
 * In a batch a body-frame point samples its body's scene and a world point
 * scene 0.
 */
sph_status sph_set_probes(sph_ctx *ctx, uint32_t n, const double *points, const int32_t *frame);
sph_status sph_read_probes(sph_ctx *ctx, double *rho, uint32_t n);

/* Release the context (not the caller's workspace).  NULL is accepted. */
sph_status sph_destroy(sph_ctx *ctx);

const char *sph_status_string(sph_status s);
const char *sph_last_error(const sph_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H_ */
