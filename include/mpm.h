/*
 * mpm.h -- C ABI of the MI355X explicit MLS-MPM substep library (with the
 * standard-MPM and PB-MPM solver variants, see mpm_set_solver).
 *
 * The library advances a scene (or a batch of scenes, mpm_create_batch) of
 * the material point method of CRESSim-MPM (arXiv 2502.18437): per substep,
 * P2G scatter of mass, APIC
 * affine momentum and MLS stress (Sec. III-B, eq. mls_mpm_p2g_momentum_force),
 * a grid update with gravity, rigid-tool SDF contact with friction and drag
 * (Sec. IV-A, eq. v_correction) and sticky box walls (Sec. III-A, boundary
 * conditions), then a G2P gather of velocity, affine matrix C, deformation
 * gradient F and position (eqs. mls_mpm_g2p_momentum, mls_mpm_g2p_f,
 * mls_mpm_g2p_integration) -- Algorithm 1 of the paper.
 *
 * The call sequence mirrors the paper's object model (Sec. V-A): a scene is
 * created (SimulationFactory / Scene), particles and tools are set
 * (ParticleObject / Shape), mpm_step enqueues work and returns at once like
 * Scene::advance, and mpm_read_state blocks like Scene::fetchResults.
 *
 * Conventions for every call:
 *  - Return value: MPM_OK (0) or a negative MPM_E* code. mpm_last_error()
 *    gives a per-handle message for the most recent failure.
 *  - Units: SI (m, s, kg, Pa). The domain is [0, 1)^3 with n_grid^3 nodes at
 *    i * dx, dx = 1 / n_grid; y is up.
 *  - Arrays at the API are row-major per particle: x and v are (n, 3), C and
 *    F are (n, 3, 3) with element [a][b] at 9p + 3a + b, E is (n,).
 *  - `where` = MPM_HOST (0): the pointer is host memory; MPM_DEVICE (1): it is
 *    device memory on the handle's GPU. Device pointers must stay valid until
 *    the handle's stream has passed the call.
 *  - Ownership: the library owns every device buffer it allocates until
 *    mpm_destroy; the caller owns all arrays it passes; inputs are copied.
 *  - Asynchrony: mpm_set_particles, mpm_set_tool_sdf and mpm_step enqueue
 *    on the handle's stream and return without waiting. mpm_read_state,
 *    mpm_get_info and mpm_destroy synchronise the stream.
 *  - Deferred errors: errors detected on the device (MPM_EDOMAIN,
 *    MPM_ENONFINITE, MPM_EINVERTED) are sticky; they are returned by the next
 *    blocking call and stay set until the next mpm_set_particles.
 *  - Threading: one host thread per handle at a time.
 */
#ifndef MPM_H_
#define MPM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define MPM_OK 0
#define MPM_EINVAL (-1)     /* bad argument, NULL handle, size out of range */
#define MPM_ENOMEM (-2)     /* a device or host allocation failed */
#define MPM_EHIP (-3)       /* a HIP runtime call failed */
#define MPM_EDOMAIN (-4)    /* a particle's 3x3x3 stencil left the grid; that
                               particle is left unchanged */
#define MPM_ENONFINITE (-5) /* a particle's state is not finite; it is left
                               unchanged */
#define MPM_EINVERTED (-6)  /* det F <= 0 was seen in the stress evaluation */
#define MPM_ERANGE (-7)     /* a particle's P2G contribution exceeded the
                               fixed-point range of the grid accumulator
                               (|m v| beyond about 1000 m_p m/s); that particle
                               is left out of the P2G of that substep */
#define MPM_ETOOBIG (-8)    /* a size beyond a fixed maximum of an entry point
                               that allocates nothing (nothing was computed) */

/* Precedence when several device errors are pending:
 * MPM_ENONFINITE, then MPM_EDOMAIN, then MPM_ERANGE, then MPM_EINVERTED. */

#define MPM_HOST 0
#define MPM_DEVICE 1

#define MPM_MAX_TOOLS 8

/* Grid accumulation mode of the P2G scatter. Each particle's contributions
 * are rounded to fixed point (weights in units of 2^-22) and summed exactly
 * per block in LDS; the modes differ in the momentum units and in the global
 * sum over blocks. */
#define MPM_ACCUM_F32 0   /* momentum in 32-bit fields at a power-of-two unit
                             chosen per work item from the bound of its
                             particles' contributions (MLS-MPM; the other
                             solvers and push-out use the units of
                             MPM_ACCUM_FIXED), block sums added with FP32
                             atomics: fastest; the summation order of the
                             FP32 adds varies */
#define MPM_ACCUM_FIXED 1 /* momentum in 64-bit fields in units of 2^-40 of
                             the particle mass times 1 m/s, block sums added
                             with integer atomics: results
                             are bit-identical run to run, for any particle
                             order and re-binning schedule. A node's 32-bit
                             weight sum holds up to 1024 (about 1000 particles
                             per cell) */

/* Tool geometries (Sec. IV-A: one SDF per rigid shape). */
#define MPM_TOOL_NONE 0    /* removes the tool */
#define MPM_TOOL_CAPSULE 1 /* segment along the body x axis;
                              size = {half_length, radius, unused} */
#define MPM_TOOL_BOX 2     /* oriented box; size = half extents in body axes */
#define MPM_TOOL_PLANE 3   /* half space; body +y is the outward normal
                              through center; size unused */
/* Cutting and suturing geometries (Sec. IV-B, IV-C): */
#define MPM_TOOL_SLICER 4  /* blade: rectangle in the body x-y plane,
                              size = {half_width (x), half_height (y), unused};
                              its side is the sign of body z. Nodes within
                              `margin` (> 0, the fattened region) of it get the
                              contact law with normal +-body z on their own
                              side, so material is parted rather than pushed;
                              beyond the spine edge (body y > half_height) the
                              field is the distance to the spine and the
                              contact is sticky (relative velocity 0). The
                              cutting edge is the body -y edge. */
#define MPM_TOOL_SEGMENT 5 /* 1D line segment along body x (thread segment,
                              straight needle); size = {half_length,
                              thickness, unused} */
#define MPM_TOOL_ARC 6     /* 1D circular arc in the body x-y plane centred
                              on `center`, from angle -half_angle to
                              +half_angle about body +x (suture needle);
                              size = {radius, half_angle (rad, <= pi),
                              thickness}. For segments and arcs, nodes within
                              the thickness keep only the part of their
                              relative velocity along the curve tangent
                              (then friction and drag), unless separating. */

typedef struct mpm_handle mpm_handle;

/* Scene constants. */
typedef struct mpm_params {
  int32_t n_grid;          /* nodes per axis, 8 <= n_grid <= 1024; dx = 1/n_grid */
  float dt;                /* substep length in s, > 0 */
  float gravity[3];        /* m/s^2, e.g. {0, -9.8, 0} */
  int32_t wall_band;       /* nodes with an index < band or > n_grid-1-band
                              get v = 0 (sticky walls); 0 disables */
  float nu;                /* Poisson ratio, 0 <= nu < 0.5 */
  float E_default;         /* Young's modulus used when no per-particle E */
  int32_t accum_mode;      /* MPM_ACCUM_F32 or MPM_ACCUM_FIXED */
  int32_t tile;            /* transfer work tile edge in cells: 8 (one 8^3 grid block) or 4
                              (a quarter-edge sub-block, for small or sparse scenes); 0 = 8.
                              mpm_set_launch_config and mpm_autotune can change it */
  int32_t resort_interval; /* substeps between particle re-binning; 0 = default */
  int64_t max_particles;   /* capacity reserved at create, >= 0 */
} mpm_params;

/* One rigid tool. The pose is kinematic: during the k-th substep after the
 * mpm_set_tool_sdf call the centre is center + k * dt * lin_vel (the pose at
 * the start of that substep); the orientation stays fixed, and ang_vel only
 * enters the rigid velocity v_r = lin_vel + ang_vel x (x_I - centre) used by
 * the contact law. */
typedef struct mpm_tool {
  int32_t type;        /* MPM_TOOL_* */
  double center[3];    /* m */
  double quat[4];      /* body-to-world rotation (w, x, y, z); normalised */
  double size[3];      /* see MPM_TOOL_* */
  double lin_vel[3];   /* m/s */
  double ang_vel[3];   /* rad/s */
  float mu;            /* kinetic friction coefficient mu_k >= 0 */
  float drag;          /* drag factor c_d in [0, 1]: 1 = no drag, 0 = sticky */
  float margin;        /* contact when phi(x_I) < margin (fattened region) */
  int32_t push_out;    /* nonzero: particle push-out (Sec. IV-A, after the particle collisions of
                          Stomakhin et al. 2013). After each substep's position update a particle
                          inside the tool, phi(x) < 0 at the tool's pose of the next substep, moves
                          to the surface along the unit outward normal: x <- x - phi n. Solid tools
                          only (capsule, box, plane); ignored for the thin ones. v, C and F are
                          unchanged. Not differentiated: rollouts refuse such a tool. */
} mpm_tool;

/* Counters, valid after a blocking call. */
typedef struct mpm_info {
  int64_t n_particles;
  int64_t substeps;          /* substeps enqueued since mpm_create */
  int64_t resorts;           /* particle re-binnings since mpm_create */
  int64_t occupied_blocks;   /* grid blocks holding particles, last binning */
  int64_t active_blocks;     /* blocks the grid update visits, last binning */
  int64_t active_nodes;      /* nodes with mass > 0 in the last substep */
  int64_t n_inverted;        /* particle-substeps with det F <= 0 */
  int64_t n_domain;          /* particles found outside the grid */
  int64_t n_nonfinite;       /* particles with non-finite state */
  int64_t n_fallback;        /* particle-substeps that left their block's
                                tile and took the global-memory path */
  int64_t n_range;           /* particle-substeps refused by the range check */
  int32_t tile;             /* transfer work tile edge in use (4 or 8) */
  int32_t resort_interval;
  int32_t accum_mode;
  int32_t n_tools;
  int64_t rollouts;          /* rollouts recorded by mpm_rollout_forward since
                                mpm_create; mpm_rollout_backward always
                                differentiates the latest one */
} mpm_info;

/* Create a scene on the current HIP device (the paper's SimulationFactory
 * building a Scene, Sec. V-A: the simulation domain, time step, gravity,
 * boundary band and material defaults of Sec. III-A). `hip_stream` is a
 * hipStream_t cast to uint64_t (e.g. torch.cuda.current_stream().cuda_stream);
 * 0 makes the library create and own a stream. Allocates the dense n_grid^3
 * grid (two float4 arrays) and room for max_particles particles.
 * Errors: MPM_EINVAL (NULL pointers, out-of-range field), MPM_ENOMEM,
 * MPM_EHIP. On error *out is NULL. */
int mpm_create(const mpm_params* p, uint64_t hip_stream, mpm_handle** out);

/* Destroy the scene: synchronises its stream, frees every device buffer
 * and returns the pending device error, if any. NULL is a no-op (MPM_OK). */
int mpm_destroy(mpm_handle* h);

/* Replace the particle set (ParticleObject, Sec. V-A) with n particles.
 * x is required when n > 0; v = NULL means 0, C = NULL means 0, F = NULL
 * means I, E = NULL means E_default for every particle. mass and vol0 are the
 * per-particle mass and initial volume (> 0). Particles are identified by
 * their index 0..n-1 in these arrays; mpm_read_state returns them in this
 * order. Clears the deferred errors. The scene clock (substep counter) and
 * the tools are left as they are.
 * Errors: MPM_EINVAL (n < 0, n > max_particles, NULL x with n > 0,
 * mass or vol0 <= 0, bad where, a handle with several scenes), MPM_EHIP. */
int mpm_set_particles(mpm_handle* h, int64_t n, const float* x, const float* v,
                      const float* C, const float* F, const float* E,
                      float mass, float vol0, int32_t where);

/* Set, replace (or with type MPM_TOOL_NONE remove) tool `tool_id`
 * (0 <= tool_id < MPM_MAX_TOOLS): a rigid Shape of the scene (Sec. V-A)
 * described by its signed distance function, with the contact law of
 * Sec. IV-A (eq. v_correction) and the cutting and suturing geometries of
 * Sec. IV-B and IV-C. Its pose advances kinematically with its velocity
 * (Sec. V-C). Tools are applied to each grid node in id order, then the
 * walls. Errors: MPM_EINVAL (bad id, type, size <= 0 for
 * the used fields, non-finite values, mu < 0, drag outside [0, 1]). */
int mpm_set_tool_sdf(mpm_handle* h, int32_t tool_id, const mpm_tool* t);

/* Enqueue n_substeps substeps of Algorithm 1 and return without waiting for
 * them (Scene::advance, Sec. V-A). With adaptive re-binning on
 * (mpm_launch_config.rebin_drift > 0, the default) the host stays at most 8
 * substeps ahead of the device, so the call returns when the device is
 * within 8 substeps of the end. n_substeps = 0 is a no-op. Errors:
 * MPM_EINVAL (n_substeps < 0), MPM_EHIP (launch failure). */
int mpm_step(mpm_handle* h, int32_t n_substeps);

/* Block until the stream drains (Scene::fetchResults, Sec. V-A) and write
 * the particle state of Algorithm 1 (x, v, C, F; Sec. III-B) in the caller's
 * original particle order. NULL outputs are skipped.
 * Returns the pending device error, if any (the state is still written).
 * Errors: MPM_EINVAL (bad where), MPM_EHIP. */
int mpm_read_state(mpm_handle* h, float* x, float* v, float* C, float* F, int32_t where);

/* Synchronise and fill *info. Errors: MPM_EINVAL, MPM_EHIP. */
int mpm_get_info(mpm_handle* h, mpm_info* info);

/* Two-way coupling (Sec. IV-A): the impulse (N s) exerted on each tool by the
 * material during the most recent mpm_step call, i.e. minus the momentum the
 * tool's velocity correction gave the grid nodes, summed over its substeps.
 * out is (MPM_MAX_TOOLS + 1) x 3 doubles: rows 0..7 are the tools, row 8 the
 * walls. A host application applies row k to its rigid body for tool k.
 * Blocking. Errors: MPM_EINVAL (NULL), MPM_EHIP. */
int mpm_read_tool_impulses(mpm_handle* h, double* out);

/* Message of the most recent failure on this handle ("" if none). The
 * string is owned by the handle and valid until its next call. A NULL
 * handle gives the message of the last failed mpm_create. */
const char* mpm_last_error(const mpm_handle* h);

/* Fixed-corotated Kirchhoff stress (Stomakhin et al. 2012) of n deformation
 * gradients with the GPU's own polar decomposition:
 * tau = 2 mu (F - R) F^T + lambda (J - 1) J I, mu and lambda from E[i] and nu.
 * F and tau are (n, 3, 3) row-major, E is (n,); all host (where = MPM_HOST)
 * or all device memory. Synchronous. Diagnostic entry point for tests of the
 * constitutive step; the substep computes the same quantity in registers.
 * Errors: MPM_EINVAL, MPM_ENOMEM, MPM_EHIP. */
int mpm_eval_stress(int64_t n, const float* F, const float* E, float nu, float* tau,
                    int32_t where);

/* mpm_eval_stress without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc). Same arguments, layout and result as mpm_eval_stress
 * (bit for bit: the same kernel). Host inputs and outputs are staged
 * through a fixed device array of MPM_NOALLOC_MAX_PARTICLES x 19 floats
 * (about 5 MB), which the library holds on every GPU it runs on until the
 * process ends; device inputs and outputs are used in place. Runs on the
 * current device and the null stream; synchronous. Every call on one GPU
 * shares that array: calls that overlap on one GPU (several host threads)
 * race and must be serialised by the caller.
 * Errors: MPM_EINVAL (bad argument), MPM_ETOOBIG (n above
 * MPM_NOALLOC_MAX_PARTICLES; nothing is computed), MPM_EHIP. The message of
 * a failure is given by mpm_last_error(NULL). */
#define MPM_NOALLOC_MAX_PARTICLES 65536
int mpm_eval_stress_noalloc(int64_t n, const float* F, const float* E, float nu, float* tau,
                            int32_t where);

/* Per-kernel timing with HIP events on the handle's stream while enabled:
 * the transfer and grid kernels record theirs as part of their dispatch
 * (hipExtLaunchKernel), the binning pipeline between marker events. Kinds,
 * in order: 0 sort (binning pipeline), 1 p2g, 2 g2p2g (fused), 3 g2p, 4 grid
 * update. While timing, every substep launches its kernels one by one (no
 * graph replay). */
#define MPM_KERNEL_KINDS 5
typedef struct mpm_kernel_times {
  double total_ms[MPM_KERNEL_KINDS];
  int64_t launches[MPM_KERNEL_KINDS];
} mpm_kernel_times;

/* Enable (enable >= 1) or disable (0) event timing; enabling clears the
 * totals. enable = k > 1 times the transfer and grid kernels of every k-th
 * substep only (substep index divisible by k), a uniform sample that keeps
 * the events' own cost (a few microseconds per event on the stream) off the
 * other substeps; binning is timed at every re-binning. EINVAL for
 * enable < 0. */
int mpm_profile(mpm_handle* h, int32_t enable);
/* Synchronise and return the totals accumulated since timing was enabled. */
int mpm_profile_read(mpm_handle* h, mpm_kernel_times* out);

/* ------------------------------------------------------ launch configuration */
/* Positions a re-binning inside mpm_step sorts the particles by (the first
 * substep of a call always sorts the state in memory):
 *  - MPM_REBIN_ADVANCE: a G2P pass first writes v, C and the advanced x, F;
 *    the sort takes those positions and a P2G pass scatters from the written
 *    state, so no stencil leaves its tile in the first substep after it.
 *  - MPM_REBIN_IN_PLACE: the sort takes the positions in memory (those the
 *    next G2P reads) and the fused transfer goes on: no extra G2P and P2G
 *    passes and no v, C to permute, but particles that cross a block
 *    boundary in that substep scatter through global memory.
 *  - MPM_REBIN_AUTO: in place for MLS-MPM and standard MPM with
 *    resort_interval >= 4, else advance (fast scenes re-bin often; a PB-MPM
 *    step's passes all scatter from the advanced positions). */
#define MPM_REBIN_AUTO 0
#define MPM_REBIN_ADVANCE 1
#define MPM_REBIN_IN_PLACE 2

/* How mpm_step launches its kernels. Results do not depend on it beyond the
 * order of FP32 atomics (in MPM_ACCUM_FIXED mode not at all). */
typedef struct mpm_launch_config {
  int32_t resort_interval; /* substeps between particle re-binnings, >= 1 */
  int32_t transfer_wgs;    /* workgroups of the persistent transfer kernels, a multiple of 8 in [8, 65536] */
  int32_t graph_chunk;     /* runs of this many plain substeps (fused transfer + grid update) are
                              recorded once as a HIP graph and replayed; 0 = launch every kernel */
  int32_t rebin_mode;      /* MPM_REBIN_AUTO, MPM_REBIN_ADVANCE or MPM_REBIN_IN_PLACE */
  int32_t tile;            /* transfer work tile edge in cells: 8 (512-thread workgroups, a
                              10^3-node LDS tile) or 4 (128-thread workgroups, 6^3 nodes);
                              0 keeps the current one. A change re-bins the particles */
  int32_t rebin_drift;     /* adaptive re-binning: re-bin before resort_interval ends once the
                              particles outside their tiles (on the global-memory path) average
                              more than this many per million per substep since the last
                              re-binning (read without waiting, a few substeps late); 0 = off,
                              default 5000 */
} mpm_launch_config;

/* Read / replace the launch configuration (the defaults: resort_interval
 * from mpm_params or 256, the tile of mpm_params, two 8-cell-tile or eight
 * 4-cell-tile workgroups per compute unit, graph_chunk 8, MPM_REBIN_AUTO).
 * Errors: MPM_EINVAL (NULL, value out of range). */
int mpm_get_launch_config(const mpm_handle* h, mpm_launch_config* out);
int mpm_set_launch_config(mpm_handle* h, const mpm_launch_config* c);

/* Autotuner: times mpm_step(trial_substeps) on the current scene for each
 * candidate configuration (work tiles of 8 or 4 cells; re-binning every 1,
 * 2, 4, 8, 16, 32 or 64 substeps; 1 to 4 transfer workgroups per compute unit
 * for 8-cell tiles, 4 to 16 for 4-cell ones; graphs on or off),
 * restoring the particles, their order, the device status and the clock
 * before every trial, and keeps the fastest (written to *chosen if not
 * NULL). For each workgroup count and graph setting the intervals are tried
 * in increasing order, and a candidate over 3 times slower than the best so
 * far ends that run. These candidates use MPM_REBIN_AUTO; the fastest is
 * then also timed with the re-binning mode AUTO did not pick. The
 * configuration in use is timed first and kept unless the fastest candidate
 * beats it by more than 5% (both timed once more at the end; the better of
 * each one's two timings counts), since short trials cannot resolve smaller
 * differences. The scene is left as it was, except that the next mpm_step
 * re-bins and the tool impulses read zero. Blocking; at most 232 calls of
 * mpm_step (a warm-up and a timed call per timing). A trial shorter than the
 * longer intervals cannot tell them apart.
 * Errors: MPM_EINVAL (no particles, trial_substeps < 1), MPM_ENOMEM (it
 * needs a copy of the particle buffer), MPM_EHIP. */
int mpm_autotune(mpm_handle* h, int32_t trial_substeps, mpm_launch_config* chosen);

/* ------------------------------------------------------ batches of scenes */
/* A handle with n_scenes independent scenes that share the grid size, dt,
 * gravity, wall band, material constants and accumulation mode. Each
 * scene has its own particles, tools and n^3 grid. Every stage of mpm_step
 * runs once for all scenes: the scene is the leading part of the grid-block
 * id, so one launch per stage covers the batch and uneven particle counts
 * balance across the GPU. mpm_create is mpm_create_batch with n_scenes = 1;
 * the single-scene calls act on scene 0. max_particles is the capacity of
 * the whole batch. Differentiable rollouts need n_scenes = 1.
 * Errors: as mpm_create; MPM_EINVAL also for n_scenes < 1 or when
 * n_scenes x ceil(n_grid / 8)^3 x 512 grid nodes reach 2^31. */
int mpm_create_batch(const mpm_params* p, int32_t n_scenes, uint64_t hip_stream, mpm_handle** out);

/* Replace the particles of every scene: counts[n_scenes] particles per scene,
 * the arrays holding scene 0's particles, then scene 1's, and so on (layout,
 * `where` and NULL rules as mpm_set_particles). mass and vol0 apply to every
 * particle. mpm_read_state returns the state in the same order. Blocks the
 * calling thread when n_scenes > 1 (it uploads the scene offsets).
 * Errors: MPM_EINVAL (NULL counts, a negative count, total above
 * max_particles, mass or vol0 not positive), MPM_EHIP. */
int mpm_set_batch_particles(mpm_handle* h, const int64_t* counts, const float* x, const float* v, const float* C,
                            const float* F, const float* E, float mass, float vol0, int32_t where);

/* mpm_set_tool_sdf / mpm_set_tool_velocity_table / mpm_read_tool_impulses
 * for scene `scene` (0 <= scene < n_scenes; otherwise MPM_EINVAL). */
int mpm_set_scene_tool(mpm_handle* h, int32_t scene, int32_t tool_id, const mpm_tool* t);
int mpm_set_scene_tool_velocity_table(mpm_handle* h, int32_t scene, int32_t tool_id, int64_t n_rows,
                                      const double* table);
int mpm_read_scene_tool_impulses(mpm_handle* h, int32_t scene, double* out);

/* ------------------------------------------------------ scripted tool motion */
/* Per-substep linear velocities of tool `tool_id` (Sec. V: a shape's velocity
 * is set for every step). `table` is n_rows x 3 doubles in host memory,
 * copied. The tool is re-anchored at its current pose; during the j-th
 * substep from now it moves with row j (j < n_rows) and its centre is the
 * anchor plus dt times the sum of rows 0..j-1; afterwards lin_vel from
 * mpm_set_tool_sdf applies again. n_rows = 0 removes the table. Applies to
 * mpm_step and mpm_rollout_forward alike; a new mpm_set_tool_sdf clears it.
 * Errors: MPM_EINVAL (no such tool, NULL table, non-finite entry). */
int mpm_set_tool_velocity_table(mpm_handle* h, int32_t tool_id, int64_t n_rows, const double* table);

/* ------------------------------------------------------ solvers */
/* The three MPM solvers of Sec. III. Every one uses the quadratic B-spline
 * stencil, the grid, the tools and the walls of mpm_step; they differ in the
 * transfers, the material model and what one mpm_step "substep" is.
 *  MPM_SOLVER_MLS (default): MLS-MPM, Algorithm 1 (Sec. III-B): APIC
 *    transfers with the fixed-corotated stress folded into the affine
 *    momentum.
 *  MPM_SOLVER_PIC: standard MPM (Sec. III-A): PIC transfers; P2G adds the
 *    internal force -dt V0 tau grad N of the Neo-Hookean Kirchhoff stress
 *    tau = mu (F F^T - I) + lambda ln(J) I (eq. neo_hookean, J clamped to
 *    >= 1e-6 inside the logarithm); G2P gives v and the velocity gradient
 *    L = sum v_I grad N^T, which is stored where C is (mpm_read_state returns
 *    L as C); F <- (I + dt L) F.
 *  MPM_SOLVER_PB: PB-MPM (Sec. III-C): a substep is one step of length dt
 *    made of `iterations` transfer passes. Gravity is added to the particle
 *    velocities once per step; each pass projects C onto the co-rotational
 *    constraint (F* = (I + dt C) F, target beta R + (1 - beta) F* /
 *    det(F*)^(1/3) with R the rotation of F*, C <- (target F^-1 - I) / dt),
 *    scatters mass and APIC momentum without stress, runs the grid update
 *    without gravity (tools at the pose of the step, walls) and gathers v and
 *    C; after the last pass F <- (I + dt C) F and x <- x + dt v. The tool and
 *    wall impulses are those of the last pass. No stress model is used (E
 *    is ignored).
 * `iterations` (1..1024) and `beta` (in [0, 1]) are used by MPM_SOLVER_PB
 * only. Takes effect at the next mpm_step; the differentiable rollout
 * needs MPM_SOLVER_MLS.
 * Errors: MPM_EINVAL (NULL handle, unknown solver, iterations or beta out of
 * range for MPM_SOLVER_PB). */
#define MPM_SOLVER_MLS 0
#define MPM_SOLVER_PIC 1
#define MPM_SOLVER_PB 2
int mpm_set_solver(mpm_handle* h, int32_t solver, int32_t iterations, float beta);
/* Read the solver settings (any output may be NULL). Errors: MPM_EINVAL
 * (NULL handle). */
int mpm_get_solver(const mpm_handle* h, int32_t* solver, int32_t* iterations, float* beta);

/* ------------------------------------------------------ differentiable rollout
 * Reverse-mode gradients of a rollout (the paper targets learning with the
 * simulator, Sec. I and V). The rollout runs the same substep as mpm_step
 * (Algorithm 1 with the contact of Sec. IV) on a dense n^3 grid with the
 * particles in the caller's order, keeping a copy of the state every
 * `checkpoint_every` substeps; the reverse pass recomputes each segment from
 * its checkpoint and walks the substeps backwards through hand-written
 * adjoint kernels. With checkpoint_every = 1 every substep's grid is kept as
 * well and nothing is recomputed. Device memory: (n_substeps /
 * checkpoint_every + 4) particle states of 96 bytes per particle, plus
 * checkpoint_every more when checkpoint_every > 1; 60 bytes per grid node,
 * plus 32 bytes per node for each kept grid (n_substeps of them when
 * checkpoint_every = 1, else checkpoint_every during the reverse pass). */

/* Run n_substeps substeps from the current state and record the rollout.
 * theta (device, N floats, caller order) sets E_p = exp(theta_p) for the
 * rollout and afterwards; NULL keeps the current E. The particle state
 * afterwards is that after the rollout (mpm_read_state reads it). The tool
 * impulses are not recorded (they read zero). Not blocking.
 * Errors: MPM_EINVAL (no particles, n_substeps < 0, checkpoint_every < 1),
 * MPM_ENOMEM, MPM_EHIP; device errors are deferred as for mpm_step.
 * MPM_EINVAL also when the solver is not MPM_SOLVER_MLS or a tool has push_out on. */
int mpm_rollout_forward(mpm_handle* h, int32_t n_substeps, int32_t checkpoint_every, const float* theta);

/* Gradient of a scalar loss L through the recorded rollout. Inputs (device,
 * caller order, NULL = zero): xb, vb, Cb, Fb = dL/d(final x, v, C, F) with the
 * shapes of mpm_read_state. Outputs: theta_bar (device, N floats, required) =
 * dL/d theta_p with E_p = exp(theta_p); vel_bar (host, MPM_MAX_TOOLS x
 * n_substeps x 3 doubles, NULL to skip) = dL/d(linear velocity of tool q
 * during substep j of the rollout), which acts on the contact of that
 * substep and moves every later pose; xb0, vb0, Cb0, Fb0 (device, NULL to
 * skip) = dL/d(state at the rollout start). Contact sets, stencil cells and
 * clamps are held at the ones the forward pass took. The particle state is
 * not changed; the call may be repeated with other seeds. Blocking when
 * vel_bar is given. Errors: MPM_EINVAL (no recorded rollout: particles, tools,
 * tables or the clock changed since mpm_rollout_forward; NULL theta_bar),
 * MPM_ENOMEM, MPM_EHIP. */
int mpm_rollout_backward(mpm_handle* h, const float* xb, const float* vb, const float* Cb, const float* Fb,
                         float* theta_bar, double* vel_bar, float* xb0, float* vb0, float* Cb0, float* Fb0);

#ifdef __cplusplus
}
#endif

#endif /* MPM_H_ */
