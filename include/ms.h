/*
 * ms.h — C ABI of the MI355X batched rigid-body step library (libms).
 *
 * The library advances many independent rigid-body environments ("envs") by one or more
 * fixed time steps with a single fused HIP kernel on one GPU.  The capability follows the
 * GPU-parallel, heterogeneous simulation of ManiSkill3 (arXiv 2410.00425): every parallel env
 * is its own scene with its own object count and articulation (Sec. III-C, Heterogeneous GPU
 * Simulation), state stays resident on the GPU (Sec. III-B, GPU Parallelized Simulation and
 * Rendering), envs can be reset in part (App. C, PPO: partial resets) with per-env seeded
 * randomisation (App. B, Environment Setup and Domain Randomizations), and the solver runs a
 * fixed number of position / velocity iterations (App. E, Setup: 120 Hz, 4 position and 0
 * velocity iterations).  The paper does not state the contact and solver equations; the step
 * model this library implements is fixed by the oracle's documented reading (sequential-impulse
 * TGS/PGS with speculative contacts, patch friction: two tangent rows and a torsional row per
 * manifold; revolute and prismatic joints with a soft PD drive and position limits).
 *
 * Conventions: SI units, z up, quaternions (w, x, y, z), angular velocity in the world frame.
 * Body and joint indices inside descriptors are env-local.  All device pointers are
 * caller-owned (usually torch tensors) and must stay valid until the stream reaches the call.
 * Every call is stream-ordered and non-blocking unless stated otherwise; none synchronises
 * the device.  Argument and validation failures return a code synchronously and enqueue
 * nothing; the thread-local message is available from ms_last_error().
 * A batch is not thread-safe; distinct batches may be used from distinct threads.
 */
#ifndef MS_H
#define MS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MS_OK = 0,
    MS_E_INVALID_ARG = 1,  /* null pointer, bad size, bad index, bad descriptor */
    MS_E_NO_WORKSPACE = 2, /* workspace smaller than ms_query_batch_bytes() */
    MS_E_BUDGET = 3,       /* request exceeds the server's HBM budget */
    MS_E_DEVICE = 4,       /* a HIP runtime call failed */
    MS_E_CAPACITY = 5,     /* an env exceeds a kernel capacity (bodies, joints, LDS) */
    MS_E_STATE = 6         /* call not valid in the object's current state */
} ms_status;

enum { MS_SPHERE = 0, MS_CAPSULE = 1, MS_BOX = 2, MS_COMPOUND = 3 };
enum { MS_BODY_STATIC = 1 };            /* zero inverse mass and inertia; never integrated */
enum { MS_SOLVER_TGS = 0, MS_SOLVER_PGS = 1 };
enum { MS_JOINT_REVOLUTE = 0, MS_JOINT_PRISMATIC = 1 };

/* Per-env status bits written by the step (status[E], int32). */
enum {
    MS_STATUS_NONFINITE = 1,       /* a NaN/Inf appeared: the env keeps its pre-step state and is frozen */
    MS_STATUS_CONTACT_OVERFLOW = 2,/* more contact points than the env's capacity: the first ones in
                                      canonical pair order were kept */
    MS_STATUS_COLOR_OVERFLOW = 4   /* more than 64 colours: extra blocks were solved serially */
};
#define MS_STATUS_FROZEN_MASK 1

/* Limits of the fused kernel. */
#define MS_MAX_BODIES_PER_ENV 64
#define MS_MAX_JOINTS_PER_ENV 64
#define MS_MAX_BLOCKS_PER_ENV 256   /* joints + manifold capacity of one env */
#define MS_MAX_PARTS 4              /* primitive parts of one compound body */

/* One rigid body.  Shape dims: sphere (r, -, -); capsule (r, half_len, -) with its axis along
 * body-local z and half_len = half the cylinder length; box (hx, hy, hz) half-extents.
 * mass > 0 gives the mass; otherwise mass = density * volume.  The centre of mass is the shape
 * centre and the principal axes are the shape axes.  Compound (MS_COMPOUND): dims[0] holds the
 * index of the body's entry in the scene's compound table (an integer value); its mass and
 * inertia follow from its parts (see ms_compound_desc).  88 bytes, no padding. */
typedef struct {
    int32_t shape;
    int32_t flags;
    float dims[3];
    float mass;
    float density;
    float friction;
    float restitution;
    float pos[3];
    float quat[4];
    float linvel[3];
    float angvel[3];
} ms_body_desc;

/* One joint (the paper's articulations, Sec. III-F1, driven by PD joint-position controllers,
 * App. B, Controller / Action Space): revolute about the z axis of its joint frame, or prismatic
 * along it (App. A, Classic Control: the cart-pole's slider).  parent = -1 attaches the child to
 * the static world.  frame_* = (px, py, pz, qw, qx, qy, qz) in the body's local frame (the world
 * frame for parent = -1).  kp (N m / rad or N / m) and kd (N m s / rad or N s / m) define the PD
 * position drive toward `target` (rad or m); kp = kd = 0 disables the drive.  limited != 0 adds
 * one-sided limit rows at lower / upper (App. A, Locomotion: constrained joint limits).  Parent
 * and child never collide with each other.  92 bytes, no padding. */
typedef struct {
    int32_t parent;
    int32_t child;
    float frame_parent[7];
    float frame_child[7];
    float kp;
    float kd;
    float target;
    int32_t type;       /* MS_JOINT_REVOLUTE or MS_JOINT_PRISMATIC */
    int32_t limited;    /* != 0: position limits [lower, upper] */
    float lower;
    float upper;
} ms_joint_desc;

/* A compound body's shape: 1..MS_MAX_PARTS primitive parts (sphere, capsule or box with the
 * body dims' meaning) at poses (px, py, pz, qw, qx, qy, qz) in the body frame: the convex pieces
 * of a decomposed object (the paper's objects are convex-decomposed meshes, Sec. III-B and App.
 * B, Environment Setup).  Contacts: every pair of parts of the two bodies (each part against the
 * ground) runs the primitive narrowphase and keeps <= 4 points as its own manifold with its own
 * friction patch, in part order (A's parts outer).  Mass: uniform density over the parts, shared
 * by volume (overlaps count twice); inertia: each part's about its centre, rotated into the body
 * frame and moved to the origin (parallel axes), summed.  The body frame must be the principal
 * frame with the centre of mass at the origin: create rejects a compound whose centre of mass is
 * off the origin by more than 1e-4 of its extent or whose products of inertia exceed 1e-3 of its
 * largest moment.  Part quaternions must be unit to 1e-5.  180 bytes, no padding. */
typedef struct {
    int32_t n_children;
    int32_t shape[MS_MAX_PARTS];
    float dims[MS_MAX_PARTS][3];
    float pose[MS_MAX_PARTS][7];
} ms_compound_desc;

/* A batch of envs in compressed form: env e owns bodies [env_body_off[e], env_body_off[e+1]) and
 * joints [env_joint_off[e], env_joint_off[e+1]); compound bodies index the compound table, shared
 * by every env.  Host memory, copied during create. */
typedef struct {
    int32_t n_envs;
    const int32_t* env_body_off;   /* [n_envs + 1] */
    const ms_body_desc* bodies;    /* [env_body_off[n_envs]] */
    const int32_t* env_joint_off;  /* [n_envs + 1] */
    const ms_joint_desc* joints;   /* [env_joint_off[n_envs]] */
    int32_t n_compounds;                  /* entries of the compound table (0: none) */
    const ms_compound_desc* compounds;    /* [n_compounds] (may be null when n_compounds is 0) */
} ms_scene_desc;

/* Step parameters.  One step advances dt; TGS runs pos_iters substeps of one iteration each,
 * PGS runs one substep of pos_iters iterations; vel_iters velocity-only sweeps follow.  The
 * ground is the half-space z <= plane_z when plane_enabled != 0.  max_contacts_per_env <= 0
 * selects the default min(6 * n_dyn + 8, 384) contact points per env, max_manifolds_per_env <= 0
 * min(3 * n_dyn + 4, 192) manifolds (n_dyn: dynamic bodies of the env); pairs beyond them lose
 * their points and the env's status gets bit 2.  debug_export != 0 makes the step also write the last
 * step's pair list, contact points and colours (read with ms_get_contacts).
 * Cross-step warm start (warm_start != 0; the solver's iteration counts of App. E, Setup, assume
 * contacts that persist across steps): each step ends by caching, per env in the workspace, every
 * manifold's body pair, its friction patch's tangential impulse as a world vector and its twist
 * impulse, and every contact point's final normal impulse with its position in body B's frame at
 * the step start.  The next step starts each new point from the nearest cached point of the same
 * body pair closer than warm_radius (none beyond it), projects the cached tangential impulse on
 * the patch's new tangents, and applies these impulses in its first substep as well.  The cache
 * is part of the batch, not of ms_state_view: a step is then a function of the state and the
 * cache; ms_reset_envs and ms_reset_envs_random clear the listed envs' caches.  96 bytes. */
typedef struct {
    float dt;
    int32_t pos_iters;
    int32_t vel_iters;
    int32_t solver;
    float gravity[3];
    float plane_z;
    int32_t plane_enabled;
    float plane_friction;
    float plane_restitution;
    float contact_offset;
    float baumgarte;
    float max_depen_vel;
    float joint_baumgarte;
    float bounce_threshold;
    float lin_damping;
    float ang_damping;
    int32_t max_contacts_per_env;
    int32_t debug_export;
    int32_t joint_iters;
    int32_t max_manifolds_per_env;
    int32_t warm_start;   /* != 0: cross-step warm start from the contact cache (see below) */
    float warm_radius;    /* m: matching radius of the contact cache */
} ms_sim_params;

/* Caller-owned device buffers in structure-of-arrays form over all B bodies of the batch:
 * pos[3][B], quat[4][B], linvel[3][B], angvel[3][B] (float32, component-major) and status[E]. */
typedef struct {
    float* pos;
    float* quat;
    float* linvel;
    float* angvel;
    int32_t* status;
} ms_state_view;

/* Execution plan knobs.  lanes_per_env = 0 lets the library pick (autotuned or heuristic);
 * otherwise 1, 2, 4, 8, 16, 32 or 64 lanes of a 64-wide wavefront serve one env.  pack != 0
 * sorts envs by size class before tiling (heterogeneous batches).  launch_mode 0: a batch whose
 * tiles need several LDS sizes runs in one launch of workgroups of up to 4 wavefronts, each
 * workgroup holding a bin of tiles packed into half a CU's LDS; 1: one launch per LDS class
 * (concurrent streams).  Both give the same bits. */
typedef struct {
    int32_t lanes_per_env;
    int32_t pack;
    int32_t max_resident_groups; /* 0 = the device's resident capacity (class launches) */
    int32_t launch_mode;
} ms_plan;

typedef struct ms_batch ms_batch;

/* Device workspace bytes needed by a batch (state, parameters, joints, targets, tiles, contact
 * cache, debug).  The workspace is all the device memory a batch uses, so an HBM budget can be
 * checked before anything is allocated (Sec. III-B: GPU memory efficiency).  Host-only, never
 * touches the device.  Errors: MS_E_INVALID_ARG / MS_E_CAPACITY for invalid descriptors. */
ms_status ms_query_batch_bytes(const ms_sim_params* params, const ms_scene_desc* scene,
                               const ms_plan* plan, size_t* bytes);

/* Create a batch of independent, possibly heterogeneous envs (Sec. III-C, Heterogeneous GPU
 * Simulation: per-env object counts and articulations).
 * Validate the scene, lay out the workspace (caller-owned device memory of at least
 * ms_query_batch_bytes() bytes, 256-byte aligned) and upload the initial state on `hip_stream`
 * (NULL = the default stream).  The initial state is kept for ms_reset_envs(src = NULL).
 * Reconfiguration is a destroy + create. */
ms_status ms_create_batch(const ms_sim_params* params, const ms_scene_desc* scene,
                          const ms_plan* plan, void* dev_workspace, size_t ws_bytes,
                          void* hip_stream, ms_batch** out);

/* The batched physics step (Sec. III-B: all envs advanced in parallel on the GPU; App. E, Setup:
 * position iterations = TGS substeps).
 * Advance every env by n_steps steps (n_steps >= 1) in one fused launch.  dev_targets holds one
 * drive target per joint of the batch (float32 [total joints], device) and replaces the
 * descriptor targets for this and later calls; NULL keeps the current ones.  Envs with a frozen
 * status are skipped. */
ms_status ms_step(ms_batch* b, const float* dev_targets, int32_t n_steps, void* hip_stream);

/* Partial reset (App. C, PPO: partial resets).  Write state for the listed envs (int32 device
 * array of n_ids env ids, each in [0, E)) and clear their status (and their contact forces).
 * src = NULL restores the initial state; otherwise src holds full-batch SoA arrays (same shape
 * as ms_state_view) from which the listed envs' bodies are copied.  Ids outside [0, E) are
 * skipped and counted (ms_get_invalid_ids).  MS_E_INVALID_ARG for a null pointer or negative
 * n_ids (nothing enqueued). */
ms_status ms_reset_envs(ms_batch* b, const int32_t* dev_env_ids, int32_t n_ids,
                        const ms_state_view* src, void* hip_stream);

/* Randomised partial reset (App. C, PPO: partial resets; App. B, Environment Setup and Domain
 * Randomizations: initial joint positions drawn around a reference, object placement and yaw
 * drawn uniformly; Sec. III-G: per-env seeded randomness).  For each listed env (int32 device
 * array of n_ids ids), starting from the batch's initial state: every free dynamic body (the
 * child of no joint) moves by xy_half * (2u - 1) in x and in y and turns about the world z axis
 * through its centre by yaw_half * (2u - 1); every joint, in index order, takes the position
 * q0 = q_init + joint_sigma * N (q_init its position in the initial state, N an Irwin-Hall
 * standard normal deviate: the sum of 12 uniforms minus 6) and poses its child from its parent;
 * all velocities are zero, the status is cleared, the env's contact forces are zero, and with
 * targets_follow the joint's drive target becomes q0.  Random numbers: Philox4x32-10 under the
 * 64-bit key `seed` with counter (env id, count, purpose, index); body i uses block (1, i), joint
 * j blocks (0, 3j .. 3j + 2); u = the top 24 bits / 2^24.  `count` distinguishes successive
 * resets of one env.  Stream-ordered, no host synchronisation.  Errors (nothing enqueued):
 * MS_E_INVALID_ARG for a null pointer, negative n_ids, a noise scale that is negative or not
 * finite, or a batch whose envs do not order their joints parents first.  Ids outside [0, E) are
 * skipped and counted (ms_get_invalid_ids). */
typedef struct {
    float joint_sigma;      /* rad (revolute) or m (prismatic) */
    float xy_half;          /* m */
    float yaw_half;         /* rad */
    int32_t targets_follow; /* != 0: drive targets become the drawn joint positions */
} ms_reset_noise;
ms_status ms_reset_envs_random(ms_batch* b, const int32_t* dev_env_ids, int32_t n_ids, const ms_reset_noise* noise,
                               uint64_t seed, uint32_t count, void* hip_stream);

/* Target-delta joint position controller (App. B, Controller / Action Space): per joint,
 * target += clip(a, -1, 1) * (high - low) / 2 in float32.  dev_actions: float32 [J] (device);
 * dev_low / dev_high: float32 [J] per-joint bounds, or NULL to use the scalars low / high.
 * Stream-ordered.  MS_E_INVALID_ARG for null actions or a non-finite scalar bound in use. */
ms_status ms_apply_actions(ms_batch* b, const float* dev_actions, const float* dev_low, const float* dev_high, float low,
                           float high, void* hip_stream);

/* Copy the current drive targets, float32 [J], into caller-owned device memory.  Stream-ordered. */
ms_status ms_get_targets(ms_batch* b, float* dev_out, void* hip_stream);

/* Joint positions of the current state, float32 [J] (device, caller-owned): the twist angle
 * 2 atan2(q_rel.z, q_rel.w) of the child's joint frame relative to the parent's for a revolute
 * joint (the drive's angle, unwrapped into [-pi, pi]), the anchors' separation along the slide
 * axis for a prismatic one (App. B, Controller / Action Space: the controller's q_t).
 * Stream-ordered. */
ms_status ms_get_joint_positions(ms_batch* b, float* dev_out, void* hip_stream);

/* Contact-force readout for touch sensing (App. A, Dextrous Manipulation: touch sensors), kept on
 * the device.  ms_set_contact_forces(enable != 0) makes every later step of the batch accumulate,
 * per dynamic body, the net contact impulse of the step: for every substep, the final normal
 * impulses of the body's contact points and the two tangent impulses of its friction patches
 * (added on a manifold's side B, subtracted on side A; the body's manifolds in the solver's colour
 * order, a manifold's points before its patch), divided by dt.  Static bodies report zero.  A
 * launch of several steps keeps the last step's.  Frozen envs and steps that went non-finite give
 * zero.  Enabling zeroes the buffer; enabling and disabling
 * synchronise `hip_stream`.  ms_get_contact_forces copies float32 [3][B] (component-major, like
 * the state planes) into caller-owned device memory, stream-ordered; MS_E_STATE when not enabled.
 * Tuning trial steps (ms_tune_batch) overwrite the forces. */
ms_status ms_set_contact_forces(ms_batch* b, int32_t enable, void* hip_stream);
ms_status ms_get_contact_forces(ms_batch* b, float* dev_out, void* hip_stream);

/* Number of env ids outside [0, E) met by ms_reset_envs and ms_reset_envs_random since the last
 * clear (those ids were skipped).  Synchronises `hip_stream`; clear != 0 zeroes the count. */
ms_status ms_get_invalid_ids(ms_batch* b, int32_t* host_count, int32_t clear, void* hip_stream);

/* Copy the current state (all envs) into caller-owned device buffers (Sec. III-B: observations
 * stay on the GPU).  Stream-ordered device-to-device copies. */
ms_status ms_get_state(ms_batch* b, const ms_state_view* dst, void* hip_stream);

/* Body and joint offsets of the batch (host arrays of n_envs + 1 entries each), and totals. */
ms_status ms_get_layout(ms_batch* b, int32_t* host_env_body_off, int32_t* host_env_joint_off);
ms_status ms_get_sizes(ms_batch* b, int32_t* n_envs, int32_t* n_bodies, int32_t* n_joints);

/* Contact export of the last step of the last ms_step call (requires debug_export; synchronises
 * `hip_stream`).  Per env, in canonical pair order, host_pairs receives int32 records
 * {env, a, b, kept_points, decision} for every candidate pair (b = 0xFFFF is the ground plane;
 * decision is the narrowphase branch: the separating axis for box pairs, the parallel branch for
 * capsule pairs, the inside face for sphere-box; for a pair with a compound body, kept_points
 * sums its pairs of parts and decision is 64 + the first pair of parts with points, 63 if none).
 * host_points receives float records {px, py, pz, nx, ny, nz, s0, lambda_n} for every kept point
 * (world frame, normal from A to B, step-start separation, final normal impulse), and
 * host_manifolds float records {env, pair index within the env, colour, lambda_t1, lambda_t2,
 * lambda_twist, mu, r_twist} per manifold (a compound pair has one manifold per pair of parts
 * with points, in part order).  Buffers may be NULL (counts only); records beyond a *_cap are
 * dropped. */
ms_status ms_get_contacts(ms_batch* b, int32_t* host_pairs, int32_t pairs_cap, float* host_points,
                          int32_t points_cap, float* host_manifolds, int32_t manifolds_cap,
                          int32_t* n_pairs, int32_t* n_points, int32_t* n_manifolds, void* hip_stream);

/* Execution plan of a batch: number of env tiles, launch grid, LDS bytes per workgroup and the
 * lanes serving each env (host array of n_envs entries, may be NULL). */
ms_status ms_get_plan(ms_batch* b, int32_t* n_tiles, int32_t* grid, int32_t* lds_bytes,
                      int32_t* host_env_lanes);

/* LDS classes of the launch plan: *n_classes and, per class, int32 {tiles, LDS bytes per
 * workgroup, kernel variant (0 unconstrained, 1 two waves per SIMD, 2 and 3 the same two built
 * for tiles that hold one env on all 64 lanes; a class runs its one-env tiles with 2 or 3 and its
 * other tiles with 0 or 1, and the value reported is the first), lanes per env, first tile}
 * into host_classes (may be NULL).  With launch_mode 0 a plan of several classes runs as one
 * launch of bins; the classes still describe its tiles' LDS sizes, and ms_get_plan reports the
 * bins (grid = number of bins, LDS bytes per bin). */
ms_status ms_get_classes(ms_batch* b, int32_t* n_classes, int32_t* host_classes);

/* Autotuner (the batching pattern's project-written tuner of envs per workgroup and solver
 * tiling).  First the env tiling: for every group of envs that the planner gave the same lanes per
 * env (so 64 / lanes envs per wavefront), the whole batch is timed over trial_steps steps with
 * half and with twice as many lanes for that group, and a change is kept if it is at least 3 %
 * faster.  Then, for a batch that runs as one launch of bins, the bins' shape: at most 2, 3 or 4
 * tiles per bin packed into a quarter, a third or half of a CU's LDS (default: 4 in half), kept
 * if at least 3 % faster.  Then, when the batch runs as one launch per LDS class, each kernel
 * variant of every class is timed over trial_steps launches of that class alone and the
 * fastest kept (the bins launch has fixed builds).  The tiling never changes a result.  The
 * batch's state, status, contact cache and work counters are saved before and restored after (the
 * trial steps leave no trace; contact forces, if enabled, are overwritten).  Synchronises
 * `hip_stream`. */
ms_status ms_tune_batch(ms_batch* b, int32_t trial_steps, void* hip_stream);

/* Work counters accumulated by every step since the last reset, int64 [n_envs][16]: steps,
 * candidate pairs per shape kind (12 kinds: 3 * min + max of the two shapes for body pairs,
 * 9 + shape for plane pairs; sphere 0, capsule 1, box 2), contact points, manifolds, colours
 * (summed over steps).  host_stats may be NULL; reset != 0 zeroes the counters.  Synchronises
 * `hip_stream`. */
ms_status ms_get_stats(ms_batch* b, int64_t* host_stats, int32_t reset, void* hip_stream);

/* Free the batch's host-side record (the workspace stays the caller's).  Destroy its graphs first;
 * the caller must let the stream pass the batch's last launch before reusing the workspace. */
ms_status ms_destroy_batch(ms_batch* b);

/* Captured step sequences (Sec. "GPU Parallelized Simulation and Rendering": the step stays on
 * the GPU with minimal host overhead per step).  ms_graph_create records
 * n_launches consecutive ms_step(b, dev_targets, steps_per_launch) calls, including the fork /
 * join of LDS classes on side streams, into a HIP graph by stream capture on a private stream
 * and instantiates it; ms_graph_launch replays it on `hip_stream` (stream-ordered, no host
 * synchronisation).  The graph reads dev_targets (J floats, may be NULL) at replay time, so the
 * caller may rewrite that buffer between replays; it must stay valid while the graph exists.
 * The graph holds no memset nodes.  A graph belongs to its batch: destroy it before the batch.
 * ms_tune_batch re-plans the batch's tiles and ms_set_contact_forces switches its kernel build; a
 * graph captured before either replays the old launch, so ms_graph_launch then returns MS_E_STATE
 * (destroy the graph and capture again).
 * Errors: invalid arguments or a failed capture return a status and leave nothing behind. */
typedef struct ms_graph ms_graph;
ms_status ms_graph_create(ms_batch* b, const float* dev_targets, int32_t steps_per_launch, int32_t n_launches,
                          ms_graph** out);
ms_status ms_graph_launch(ms_graph* g, void* hip_stream);
ms_status ms_graph_destroy(ms_graph* g);

/* Fused step over several batches in one launch (the serving path): the env tiles of every
 * batch are merged into one work list, run as one launch of LDS-packed bins when they need
 * several LDS sizes (as ms_step does for one batch).  dev_targets (may be NULL) holds per-batch target
 * pointers as in ms_step.  dev_scratch is caller device memory of at least
 * ms_query_step_many_bytes() bytes (256-byte aligned) that receives the combined work list; it
 * must not be reused until the stream has passed this launch.  The batches must live on the
 * current device. */
ms_status ms_query_step_many_bytes(ms_batch* const* batches, int32_t n_batches, size_t* bytes);
ms_status ms_step_many(ms_batch* const* batches, const float* const* dev_targets, int32_t n_batches,
                       int32_t n_steps, void* dev_scratch, size_t scratch_bytes, void* hip_stream);

/* ms_step_many for callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): the same fused launch, with the
 * combined work list in a static device array of MS_STEP_MANY_NOALLOC_BYTES that the library
 * holds on each GPU it runs on until the process ends, instead of caller scratch.  The call
 * allocates nothing (no device, pinned or heap memory); the work list is uploaded from a static
 * host image.  Results are bit-identical to ms_step_many.  Limits: the work list (the size
 * ms_query_step_many_bytes reports) must fit MS_STEP_MANY_NOALLOC_BYTES and n_batches <= 4096,
 * else MS_E_CAPACITY and nothing is enqueued.  Every call on one GPU shares that GPU's array and
 * overwrites it completely: calls on one stream are ordered, but calls on different streams of
 * one GPU whose launches may overlap race on it (serialise them on one stream or use
 * ms_step_many).  The host part of concurrent calls is serialised by a lock. */
#define MS_STEP_MANY_NOALLOC_BYTES (4u << 20)
ms_status ms_step_many_noalloc(ms_batch* const* batches, const float* const* dev_targets, int32_t n_batches,
                               int32_t n_steps, void* hip_stream);

/* Serving (Sec. "GPU Parallelized Simulation and Rendering": all state stays on one GPU; Sec.
 * "Heterogeneous GPU Simulation": envs of different sizes share the GPU).  A server owns a
 * worker thread and a stream on the current device, and a caller-owned device arena of
 * arena_bytes (256-byte aligned) from which it carves, first fit, each admitted session's
 * workspace (ms_query_batch_bytes + its targets buffer) and a scratch reserve of scratch_bytes
 * for the fused work list (0: arena / 16, at most 16 MiB).
 *   ms_server_open    queues a session (a batch of envs, descriptors copied) for admission and
 *                     returns its id; sessions are admitted in arrival order as soon as their
 *                     block fits (HBM-budget admission; one that can never fit the arena is
 *                     rejected here with MS_E_BUDGET).
 *   ms_server_submit  queues a request of n_steps steps (host_targets: J floats or NULL =
 *                     keep); a session's requests run in submission order.
 *   ms_server_wait    blocks until the request is done, fills *info (may be NULL) and forgets
 *                     the request: wait on each request exactly once.
 *   ms_server_close   retires the session after its queued requests; its block is freed.
 *   ms_server_get_state  waits until the session is admitted and idle, then copies its state
 *                     on hip_stream as ms_get_state does.
 *   ms_server_drain   waits until every queued request has run and closed sessions are gone.
 *   ms_server_stats   int64 [8]: fused launches, batches summed over launches, env-steps, requests
 *                     done, sessions admitted, busy microseconds, peak arena bytes, sessions
 *                     rejected at admission.
 *   ms_server_destroy runs what is queued, stops the worker and frees everything.
 * Continuous batching: each worker iteration advances the head request of every admitted
 * session by the smallest remaining step count in one ms_step_many launch; requests arriving
 * meanwhile join the next iteration.  Times are seconds on ms_server_clock (monotonic).
 * The arena must stay valid until ms_server_destroy returns.  All calls are thread safe. */
typedef struct ms_server ms_server;
typedef struct {
    int64_t request, session;
    int32_t status, n_steps;
    double t_submit, t_start, t_done;   /* queued, first launch, completion observed */
    int32_t fused_batches;              /* sessions in the launch that completed it */
    int32_t pad;
} ms_request_info;
ms_status ms_server_create(void* dev_arena, size_t arena_bytes, size_t scratch_bytes, ms_server** out);
ms_status ms_server_open(ms_server* s, const ms_sim_params* params, const ms_scene_desc* scene, const ms_plan* plan,
                         int64_t* session);
ms_status ms_server_submit(ms_server* s, int64_t session, int32_t n_steps, const float* host_targets,
                           int64_t* request);
ms_status ms_server_wait(ms_server* s, int64_t request, ms_request_info* info);
ms_status ms_server_close(ms_server* s, int64_t session);
ms_status ms_server_get_state(ms_server* s, int64_t session, const ms_state_view* dst, void* hip_stream);
ms_status ms_server_drain(ms_server* s);
ms_status ms_server_stats(ms_server* s, int64_t* host_stats);
ms_status ms_server_destroy(ms_server* s);
double ms_server_clock(void);

/* Measurement helper, not part of the step: launches n_waves 64-lane wavefronts on hip_stream
 * that run `iters` rounds of 8 independent float32 chains, each round one multiply and one add
 * per chain (no fused or packed forms, the instruction kinds of the step's arithmetic), and
 * write one float per lane to dev_out [n_waves * 64] (device memory, caller-owned).  FLOP per
 * launch = 16 * iters * 64 * n_waves; timing the launch gives the FP32 vector rate that code
 * of this kind can reach.  MS_E_INVALID_ARG for a null pointer or a non-positive size. */
ms_status ms_peak_fp32(float* dev_out, int n_waves, int iters, void* hip_stream);

/* Measurement helper of the per-phase clock build (libms built with -DMS_PHASE_CLOCK; the default
 * build returns MS_E_STATE): wave-cycles spent by the batch's wavefronts in each phase of the step
 * since the last reset, int64 [16]: load, pose + bounding boxes, broadphase, narrowphase + rows,
 * contact cache, colouring, block lists, gravity + warm start, bias + joint prep, joint-wave warm
 * start, sweeps, force sums, integration, velocity + restitution passes, guard + exports, store.
 * Synchronises `hip_stream`; reset != 0 zeroes the counters. */
ms_status ms_get_phase_clocks(ms_batch* b, int64_t* host_cycles, int32_t reset, void* hip_stream);

/* Thread-local message of the last non-OK status returned on this thread. */
const char* ms_last_error(void);

/* Library version string. */
const char* ms_version(void);

/* Host-only consistency check of the kernel's LDS layout and pair indexing for every supported
 * env size and of the packing of tiles into bins; returns 0 when consistent.  Touches no device. */
int ms_selfcheck(void);

#ifdef __cplusplus
}
#endif

#endif /* MS_H */
