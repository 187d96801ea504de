/*
 * pkmi.h -- C ABI of the MI355X (gfx950) batched Levenberg-Marquardt
 * inverse-kinematics library (PyRoki, arXiv 2505.03728).
 *
 * The problem solved per (target, seed) pair is the paper's IK formulation
 * (Sec. IV-A: a robot, a joint pose cost, joint limit and joint
 * regularisation costs) minimised with Levenberg-Marquardt (Sec. III-A) over
 * the weighted residuals of Sec. III-C.
 *
 * Conventions for every entry point:
 *  - Return value: PK_OK (0) or a negative PK_E* code; pk_last_error() gives
 *    a message.  No C++ exception crosses this boundary.
 *  - "device" pointers are HIP device memory owned by the caller (e.g. the
 *    data of a torch tensor) and must stay valid until the work enqueued on
 *    `stream` has finished.  "host" pointers are read before the call
 *    returns.
 *  - Batched arrays are structure-of-arrays: a [planes][N] array stores
 *    plane i of problem p at index i*N + p.  Every float is FP32.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *    stream) unless stated otherwise.  A context is not thread-safe.
 *  - The library allocates device memory only in pk_create, pk_robot_upload,
 *    pk_seeder_create and when a solve needs a larger workspace than any
 *    earlier call (the workspace grows, never shrinks).
 */
#ifndef PKMI_H
#define PKMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pk_ctx pk_ctx;

/* Return codes. */
#define PK_OK 0
#define PK_EINVAL (-1)        /* null pointer, bad size, malformed tree      */
#define PK_EUNSUPPORTED (-2)  /* size above a library limit, variant absent  */
#define PK_ENOMEM (-3)        /* device allocation failed                    */
#define PK_EHIP (-4)          /* a HIP runtime call or launch failed          */
#define PK_ENOTFOUND (-5)     /* unknown robot or seeder id                  */

/* Per-problem status (low byte) and flag bits. */
#define PK_CONVERGED 0        /* every EE within tol_pos / tol_rot           */
#define PK_MAX_ITERS 1        /* iteration budget spent, not within tolerance */
#define PK_STALLED 2          /* a step was rejected with lambda at lambda_max */
#define PK_NONFINITE 3        /* NaN/Inf in the seed or target: left untouched */
#define PK_TARGET_SOLVED 4    /* ended by target_exit: another problem of its
                                 target met the tolerance in the same pass    */
#define PK_FLAG_FP64 0x100    /* some Cholesky pivot fell below pivot_rel times
                                 the largest diagonal and the step was re-solved
                                 in FP64                                      */

#define PK_EE_POSE 0          /* full SE(3) target: 7 values p, quat (wxyz)  */
#define PK_EE_POSITION 1      /* position-only target: 3 values              */

#define PK_MAX_JOINTS 64          /* variables (non-fixed joints) per robot      */
#define PK_MAX_TREE_JOINTS 128    /* joints of a description, fixed ones included */
#define PK_MAX_EES 8
#define PK_MAX_DEVICES 64         /* devices the allocation-free entry point serves */
#define PK_NOALLOC_MAX_PROBLEMS (1 << 20)  /* problems per pk_ik_solve_noalloc call  */

/* Kernel variants for pk_lm_options.variant. */
#define PK_VARIANT_AUTO 0     /* pick by robot shape and the autotune table  */
#define PK_VARIANT_LANE 1     /* one problem per lane; star-of-chains robots  */
#define PK_VARIANT_WAVE 2     /* one problem per 64-lane wavefront; any tree:
                                 the path-pair layout where it applies, else
                                 the lane-per-joint layout                    */
#define PK_VARIANT_WAVE_JOINT 3  /* one problem per wavefront, lane-per-joint
                                    layout forced (any tree)                 */

/* Joint kinds (Sec. III-B: fixed, revolute and prismatic joints). */
#define PK_JOINT_REVOLUTE 0   /* rotation by q about the axis                 */
#define PK_JOINT_PRISMATIC 1  /* translation by q (metres) along the axis       */
#define PK_JOINT_FIXED 2      /* no variable                                    */

/* Robot description (host memory, FP64; rounded to FP32 on upload).
 * Joints in topological order (parent[j] < j, -1 = the base).
 * Forward kinematics (Sec. III-B, T_base<-i = FK(q)_i):
 *   revolute:  p_j = p_parent + R_parent offset_j,
 *              R_j = R_parent Rot(mount_quat_j) Rot(axis_j, q_j);
 *   prismatic: R_j = R_parent Rot(mount_quat_j),
 *              p_j = p_parent + R_parent offset_j + R_j axis_j q_j;
 *   fixed:     R_j = R_parent Rot(mount_quat_j), p_j = p_parent + R_parent offset_j.
 * EE k is fixed to joint ee_joint[k] by (ee_offset[k], ee_quat[k]).
 * A mimic joint (mimic_joint[j] >= 0) is revolute or prismatic but follows
 * its driver: q_j = mimic_multiplier[j] * q_driver + mimic_offset[j]; its
 * Jacobian column adds into the driver's.  The driver must be a non-fixed,
 * non-mimic joint, and every EE below a mimic joint must be below its
 * driver too (so the structure of J^T J is that of the tree).
 * The problem's variables are the joints that are neither fixed nor mimic,
 * in index order: every [n][N] joint array (seeds, joints, q_rest) has n =
 * that count, the value pk_robot_info reports.  Fixed joints are folded into
 * their neighbours on upload (their limits are ignored, as are a mimic
 * joint's); an EE needs a non-fixed ancestor. */
typedef struct {
    int32_t n_joints;            /* 1..PK_MAX_TREE_JOINTS, at most PK_MAX_JOINTS non-fixed */
    const int32_t *parent;       /* [n]                                       */
    const double *mount_quat;    /* [n][4] wxyz, normalised on upload          */
    const double *offset;        /* [n][3] metres, in the parent frame         */
    const double *axis;          /* [n][3] unit joint axis after the mount     */
    const double *lower;         /* [n] radians                                */
    const double *upper;         /* [n] radians, >= lower                      */
    int32_t n_ee;                /* 1..PK_MAX_EES                              */
    const int32_t *ee_joint;     /* [m]                                       */
    const double *ee_offset;     /* [m][3]                                    */
    const double *ee_quat;       /* [m][4] wxyz                               */
    const int32_t *ee_kind;      /* [m] PK_EE_POSE or PK_EE_POSITION           */
    const int32_t *joint_type;   /* [n] PK_JOINT_*, or NULL = all revolute      */
    const int32_t *mimic_joint;  /* [n] driver joint index or -1; NULL = none   */
    const double *mimic_multiplier; /* [n] (read where mimic_joint >= 0)       */
    const double *mimic_offset;  /* [n]                                        */
} pk_tree;

/* Residual weights (Sec. III-C: the costs are weighted residuals and LM
 * minimises the sum of their squares):
 *   pose EE:     [w_pos * rho ; w_rot * phi],  [rho; phi] = log(T_target^-1 T_ee)
 *   position EE: w_pos * (p_ee - p_target)
 *   limit:       w_limit * (max(0, q - upper) + max(0, lower - q))
 *   rest:        w_rest * (q - q_rest)
 * q_rest: device [n] or NULL for (lower + upper) / 2. */
typedef struct {
    float w_pos, w_rot, w_limit, w_rest;
    const float *q_rest;
} pk_cost_weights;

/* Levenberg-Marquardt controls.  A trial step solves
 * (J^T J + lambda * diag(max(J^T J_jj, damping_floor))) delta = -J^T r;
 * it is accepted iff the cost strictly decreases, then
 * lambda = max(lambda / nu_down, lambda_min), else
 * lambda = min(lambda * nu_up, lambda_max) (a rejection with lambda already
 * at lambda_max ends the problem as PK_STALLED).  Every trial counts as one
 * iteration.  With early_exit, a problem stops as soon as every EE is within
 * tol_pos (metres) and, for pose EEs, tol_rot (radians); the test is
 * inclusive and runs at the seed and after every accepted step.
 * target_exit (with early_exit): a problem also ends, as PK_TARGET_SOLVED, in
 * the pass in which another problem of its target meets the tolerance, when
 * the two run side by side: in one run of consecutive lanes of the per-lane
 * kernel's wavefront (K consecutive problems of a target share a wavefront
 * when K divides 64, and each 64-problem block of a target when 64 divides
 * K).  A target's success and first iteration at tolerance are those of the
 * run without it; its best-of-K pick is among the problems that met the
 * tolerance by then.  Honoured by pk_ik_solve (and its allocation-free form)
 * and by pk_ik_solve_seeded's single-launch passes; the per-wavefront kernels
 * (one problem per wavefront), resumed problems, pk_ik_solve_mixed and
 * pk_ik_beam ignore it. */
typedef struct {
    int32_t max_iters;
    float lambda0, nu_up, nu_down, lambda_min, lambda_max;
    int32_t early_exit;
    float tol_pos, tol_rot;
    float damping_floor;         /* e.g. 1e-6                                 */
    float pivot_rel;             /* FP64 re-solve below this pivot ratio (1e-6) */
    int32_t variant;             /* PK_VARIANT_*                              */
    int32_t target_exit;         /* 0/1, see above                            */
} pk_lm_options;

/* A batch: T targets, K seeds each, N = T*K problems; problem p uses target
 * p / K.
 * targets (device): per EE k in order, 7 planes (px,py,pz,qw,qx,qy,qz) for a
 *   pose EE or 3 planes (px,py,pz) for a position EE, each plane T floats:
 *   total (sum of widths) * T floats.  Quaternions are normalised on use.
 * seeds (device): [n][N] joint values. */
typedef struct {
    int64_t n_targets;
    int32_t K;
    const float *targets;
    const float *seeds;
} pk_ik_problem;

/* Outputs (device).  Only `joints` is required; any other pointer may be
 * NULL.  Errors are measured at the returned joints: pos_err = |p_ee - p_t|,
 * rot_err = rotation angle of R_t^T R_ee (0 for position EEs).
 * best_*: per target, the seed chosen among its K problems: if any meets the
 * tolerance, the lowest total cost among those, else the lowest pose-only
 * residual sum of squares; ties go to the lower seed index.
 * trace_*: state after each of the first trace_iters iterations (debug). */
typedef struct {
    float *joints;               /* [n][N]                                    */
    float *pos_err;              /* [m][N]                                    */
    float *rot_err;              /* [m][N]                                    */
    float *cost;                 /* [N] final sum of squared residuals        */
    int32_t *iters;              /* [N] trials performed                      */
    int32_t *accepts;            /* [N] accepted trials                       */
    int32_t *status;             /* [N] PK_CONVERGED.. | PK_FLAG_FP64          */
    int32_t *iters_to_tol;       /* [N] first iteration within tolerance, -1   */
    int32_t *best_index;         /* [T] seed index k of the chosen problem     */
    float *best_joints;          /* [n][T]                                    */
    int32_t *target_success;     /* [T] 1 if some seed met the tolerance        */
    int32_t trace_iters;         /* 0..64                                      */
    float *trace_q;              /* [trace_iters][n][N]                        */
    int32_t *trace_accept;       /* [trace_iters][N]                           */
    float *pose_cost;            /* [N] pose-only residual sum of squares (the
                                    best-of-K key of targets no seed solved)   */
} pk_ik_outputs;

/* Context on one device (ordinal as seen by HIP).  Allocates the context's
 * device-side tables. */
int pk_create(pk_ctx **out, int device_ordinal);
int pk_destroy(pk_ctx *ctx);
/* Message of the last failed call on ctx (never NULL; ctx may be NULL). */
const char *pk_last_error(pk_ctx *ctx);

/* Copies the tree to the device (FP32) and returns its id.  Validates shape,
 * parent order, unit axes (within 1e-3; renormalised), limits, joint kinds
 * and EE references; folds fixed joints.  The per-lane kernel
 * (PK_VARIANT_LANE) serves single chains of 2 to 10 joints (revolute or
 * prismatic) ending in one EE and the star of 4 chains x 4 revolute joints
 * with 4 position EEs; other robots, and robots with mimic joints, run on
 * the per-wavefront kernel (PK_VARIANT_LANE is unsupported for them).  The
 * per-wavefront kernel gives each (joint, EE path) pair a lane -- a joint
 * shared by several root-to-EE paths gets one lane per path -- when the
 * robot has no mimic joints, at most 16 levels and at most 64 such pairs
 * (the path-pair layout); otherwise each joint gets one lane.
 * Synchronous. */
int pk_robot_upload(pk_ctx *ctx, const pk_tree *tree, int32_t *robot_id);
/* n variables (joints neither fixed nor mimic), m EEs, target floats per target (sum of EE widths), residual rows
 * (6 per pose EE, 3 per position EE, then n limit and n rest rows), and the
 * star shape used by the per-lane kernel (chains = 0 if not a star). */
int pk_robot_info(pk_ctx *ctx, int32_t robot_id, int32_t *n, int32_t *m,
                  int32_t *target_floats, int32_t *rows, int32_t *chains,
                  int32_t *chain_len);

/* Forward kinematics (Sec. III-B) for N configurations q [n][N] (device).
 * ee_pose [m][7][N]: position and unit quaternion (wxyz, w >= 0).
 * joint_frames (optional) [n][12][N]: R_j row-major (9) then p_j (3), for
 * the joints that are variables. */
int pk_fk(pk_ctx *ctx, int32_t robot_id, int64_t N, const float *q, float *ee_pose,
          float *joint_frames, void *stream);

/* Residual vector and analytic Jacobian at q (debug / parity entry point).
 * r [rows][N], J [rows][n][N] (row order as in pk_robot_info), problem p
 * uses target p / K from the targets layout of pk_ik_problem. */
int pk_residual_jacobian(pk_ctx *ctx, int32_t robot_id, int64_t N, int32_t K,
                         const float *targets, const float *q,
                         const pk_cost_weights *w, float *r, float *J, void *stream);

/* Batched LM IK (the hot path): FK, residuals, analytic Jacobian, damped
 * normal equations, per-problem Cholesky (FP64 re-solve on a small pivot),
 * accept/reject and the lambda update, then best-of-K when requested. */
int pk_ik_solve(pk_ctx *ctx, int32_t robot_id, const pk_ik_problem *problem,
                const pk_cost_weights *w, const pk_lm_options *opt,
                const pk_ik_outputs *out, void *stream);

/* pk_ik_solve without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as pk_ik_solve; the
 * scratch that best-of-K needs when the caller passes no cost, pose_cost or
 * status buffer (12 bytes per problem) comes from a 12 MiB device array that
 * the library holds on each GPU until the process ends, instead of the
 * context's grow-only workspace.  The caller still owns every input and
 * output.  Limit: T*K <= PK_NOALLOC_MAX_PROBLEMS, else PK_EUNSUPPORTED before
 * anything is launched.  All calls on one GPU (every context on it) share the
 * array, which keeps the last call's contents: calls that overlap in time on
 * one GPU (different streams, or different threads) race, so the caller
 * serialises them (one stream, or events).  Asynchronous on `stream`. */
int pk_ik_solve_noalloc(pk_ctx *ctx, int32_t robot_id, const pk_ik_problem *problem,
                        const pk_cost_weights *w, const pk_lm_options *opt,
                        const pk_ik_outputs *out, void *stream);

/* ------------------------------------------------------- mixed batches
 * Several groups of problems (different robots, shapes, weights) solved
 * together: per group, persistent LM launches whose wavefronts pop work
 * items from a device queue, at most iters_per_launch iterations per launch
 * with the problem state kept in HBM, and a compaction of the unfinished
 * problems between launches (problems that exit early free their lanes).
 * The launch chain of all groups is captured into one hipGraph (a branch per
 * group, so groups run concurrently) and replayed on later calls with the
 * same buffers.  Per-problem results equal those of pk_ik_solve with the same
 * inputs and options.  Traces are not supported here. */
typedef struct {
    int32_t robot_id;
    pk_ik_problem problem;
    pk_cost_weights weights;
    pk_ik_outputs out;
} pk_ik_group;

#define PK_MAX_GROUPS 16
#define PK_SCHED_SINGLE 0
#define PK_SCHED_PER_GROUP 1

typedef struct {
    int32_t iters_per_launch;    /* k; 0 = all iterations in one launch        */
    int32_t waves_per_cu;        /* persistent grid = waves_per_cu x CUs wavefronts */
    int32_t use_graph;           /* 1 = capture / replay a hipGraph             */
    int32_t workgroup_size;      /* threads per workgroup: 64, 128 or 256 (each
                                    wavefront pops its own work items); 0 = 64  */
    int32_t mode;                /* PK_SCHED_SINGLE: every group in ONE persistent
                                    launch per round, its wavefronts popping
                                    (group, problem range) items from one device
                                    queue (at most 8 groups; robots with at most 16
                                    tree levels and 4 EEs); PK_SCHED_PER_GROUP: each
                                    group's persistent launches on a stream of its
                                    own, the groups running concurrently         */
    int32_t variant[PK_MAX_GROUPS];  /* per group: lanes per problem, PK_VARIANT_LANE (1)
                                        or PK_VARIANT_WAVE (64); PK_VARIANT_AUTO = the
                                        options' choice                          */
} pk_sched_options;              /* k and waves_per_cu zero = the autotuned entry if any */

/* Asynchronous on `stream`.  sched may be NULL (graph on, autotuned or
 * default schedule).  All groups share the options (one iteration budget). */
int pk_ik_solve_mixed(pk_ctx *ctx, int32_t n_groups, const pk_ik_group *groups,
                      const pk_lm_options *opt, const pk_sched_options *sched, void *stream);
/* Times every candidate schedule (both modes x k in {1, 2, 5, 10, 25, all} x
 * wavefronts per CU in {2, 4, 8, 16} x, in single mode, workgroup sizes {64, 128,
 * 256} that fit the LDS x, for each group whose robot the per-lane kernel
 * supports, one or 64 lanes per problem; graph on) on these groups, stores the fastest in the
 * context's table under the batch's key (the groups' robot classes: variables
 * n, EEs m, EE kind; the iteration budget, early exit and variant options;
 * the GPU architecture, e.g. gfx950) and returns it.  When the environment
 * variable PK_AUTOTUNE_TABLE names a file, the table is written there as JSON
 * (pk_create reads that file into every new context).  Runs the solve several
 * times (the outputs hold the last run).  Synchronous. */
int pk_autotune_mixed(pk_ctx *ctx, int32_t n_groups, const pk_ik_group *groups,
                      const pk_lm_options *opt, pk_sched_options *best, float *best_ms,
                      void *stream);
/* The context's autotune table as JSON: {"format": "pkmi-autotune-1",
 * "entries": [{"key", "k", "waves_per_cu", "workgroup_size", "variants",
 * "ms"}, ...]}, one entry per line.  Synchronous host file I/O. */
int pk_autotune_save(pk_ctx *ctx, const char *path);
/* Adds (or replaces) the entries of a file written by pk_autotune_save;
 * *entries (optional) = entries read.  PK_ENOTFOUND if the file cannot be
 * read. */
int pk_autotune_load(pk_ctx *ctx, const char *path, int32_t *entries);
/* The table's entry for this batch's key (what pk_ik_solve_mixed uses when k
 * and waves_per_cu are zero); PK_ENOTFOUND if there is none. */
int pk_autotune_lookup(pk_ctx *ctx, int32_t n_groups, const pk_ik_group *groups,
                       const pk_lm_options *opt, pk_sched_options *found, float *ms);

/* ---------------------------------------------------------------- seeder
 * Learned seeder: an MLP (BF16 matrix-core GEMMs, FP32 accumulation) from an
 * EE pose target to K joint-space seeds, trained on (FK(q), q) pairs with
 * the min-over-seeds loss  L = mean_b min_k |qhat_{b,k} - q_b|^2  and Adam
 * (beta 0.9 / 0.999, eps 1e-8, bias-corrected).  Input encoding:
 * [p / reach, unit quaternion with w >= 0], reach = sum of link and EE
 * offset lengths.  Hidden layers Linear + SiLU, linear output.  Robots with
 * one pose EE only.  The seeds feed pk_ik_solve (LM refinement), with plain
 * random-seed LM as the fallback. */

/* init (host, optional, FP32): per layer W [out][in] then b [out], layers in
 * order, in = 7 for the first layer, out = n*K for the last; init_count must
 * equal pk_seeder_param_count.  NULL = all zeros.  Synchronous. */
int pk_seeder_create(pk_ctx *ctx, int32_t robot_id, int32_t K, int32_t hidden, int32_t depth,
                     const float *init, int64_t init_count, int32_t *seeder_id);
int pk_seeder_param_count(pk_ctx *ctx, int32_t seeder_id, int64_t *count);
/* Copies (synchronously, in the init layout) the parameters (which = 0), the
 * gradients of the last step (1) or Adam's first (2) / second (3) moments. */
int pk_seeder_get(pk_ctx *ctx, int32_t seeder_id, int32_t which, float *host_out, int64_t count);
/* Network output y [B][n*K] (device) for encoded inputs x [B][7] (device).
 * Hidden widths 128, 256 and 512 with n*K <= 128 run as one fused kernel
 * (activations kept on chip); other shapes layer by layer. */
int pk_seeder_forward(pk_ctx *ctx, int32_t seeder_id, const float *x, int64_t B, float *y,
                      void *stream);
/* The same output computed layer by layer with the training pass's GEMMs
 * (activations through HBM); for checking the fused inference pass. */
int pk_seeder_forward_layers(pk_ctx *ctx, int32_t seeder_id, const float *x, int64_t B, float *y,
                             void *stream);
/* Loss (device scalar, optional) and parameter gradients for one batch of
 * encoded inputs x [B][7] and joints q [B][n] (device); B a multiple of 128. */
int pk_seeder_grad(pk_ctx *ctx, int32_t seeder_id, const float *x, const float *q, int64_t B,
                   float *loss, void *stream);
/* Training on q_train [n][S] (device); targets are FK(q).  Epoch e visits
 * samples in the order perm[e*S .. e*S+S) (device int32, or NULL for index
 * order) in S / batch steps of `batch` (a multiple of 128) samples.
 * loss_log (device, optional): one mean loss per step.  Synchronous at exit. */
int pk_seeder_train(pk_ctx *ctx, int32_t seeder_id, const float *q_train, int64_t S,
                    int32_t batch, int32_t epochs, float lr, const int32_t *perm,
                    float *loss_log, void *stream);
/* K seeds per target for pose targets [7][T] (device, pk_ik_problem layout)
 * -> seeds [n][T*K] (device), clamped to the joint limits. */
int pk_seeder_infer(pk_ctx *ctx, int32_t seeder_id, const float *targets, int64_t T,
                    float *seeds, void *stream);
/* Learned seeds + LM refinement, with random-seed LM as the fallback:
 *   1. the seeder gives K seeds per target (pk_seeder_infer);
 *   2. LM with `refine` on the T*K problems, best-of-K per target;
 *   3. (restart_iters > 0) the K problems of each target that step 2 did not
 *      solve are listed on the device and LM is started again from their
 *      final joints (lambda back at lambda0, early exit as `refine`) for
 *      restart_iters iterations, best-of-K again;
 *   4. targets still unsolved are listed on the device and solved again from
 *      fallback_seeds [n][T*fallback_K] with `fallback`: all fallback_K seeds
 *      at once, or (fallback_chunk = c, 0 < c < fallback_K) in stages of c
 *      seeds, seeds k*c .. k*c+c-1 of a target run in stage k only if none of
 *      its earlier stages' problems converged.  Every fallback problem's LM is
 *      independent of the others, so the stages solve exactly the targets that
 *      one pass over all fallback_K seeds solves, and each run problem gives
 *      the same result; a target's pick is the best of the seeds it ran;
 *   5. per target the result of the pass that solved it.
 * Steps 3 and 4 run persistent launches over their lists (wavefronts pop
 * items from a device queue), so their cost follows the listed problems, not
 * T.  Asynchronous on `stream`; no host synchronisation inside. */
typedef struct {
    int32_t seeder_id;
    int32_t fallback_K;              /* 0 = no fallback                          */
    const float *fallback_seeds;     /* device [n][T*fallback_K]                 */
    pk_lm_options refine;            /* e.g. 10 iterations, early exit           */
    pk_lm_options fallback;          /* e.g. 30 iterations                       */
    int32_t refine_iters_per_launch; /* 0 = the refinement in one launch; k > 0 =
                                        k iterations per launch with the unfinished
                                        problems compacted in between (persistent
                                        kernel, hipGraph), as pk_ik_solve_mixed   */
    int32_t refine_blocks_per_cu;    /* persistent grid for k > 0: wavefronts per CU (0 = 4) */
    int32_t restart_iters;           /* step 3's iteration budget; 0 = no step 3    */
    int32_t persist_waves_per_cu;    /* grid of steps 3 and 4: wavefronts per CU (0 = 8) */
    int32_t fallback_chunk;          /* seeds per target per fallback stage (0 or
                                        >= fallback_K: one stage)                 */
} pk_seeded_options;

typedef struct {
    float *best_joints;              /* [n][T] required                          */
    int32_t *target_success;         /* [T]                                      */
    int32_t *source;                 /* [T] 0 learned seeds, 2 learned seeds after the
                                        restart, 1 fallback, -1 none               */
    int32_t *iters_to_tol;           /* [T] fewest LM iterations to tolerance over
                                        the succeeding pass's seeds (after a restart:
                                        refine.max_iters + the restart's), -1 if none */
    int32_t *refine_iters;           /* [T*K] optional counters of pass 2         */
    int32_t *refine_accepts;         /* [T*K]                                    */
    int32_t *fallback_iters;         /* [T*fallback_K] optional, 0 if not run      */
    int32_t *fallback_accepts;       /* [T*fallback_K]                           */
    int32_t *n_fallback;             /* device scalar: targets re-solved          */
    int32_t *restart_iters;          /* [T*K] optional counters of step 3, 0 if not
                                        restarted                                 */
    int32_t *restart_accepts;        /* [T*K]                                    */
    int32_t *n_restart;              /* device scalar: targets restarted          */
    int32_t *n_fallback_problems;    /* device scalar: fallback problems run      */
} pk_seeded_outputs;

int pk_ik_solve_seeded(pk_ctx *ctx, int32_t robot_id, int64_t n_targets, const float *targets,
                       const pk_cost_weights *w, const pk_seeded_options *opt,
                       const pk_seeded_outputs *out, void *stream);

/* Checkpoint of parameters, Adam moments and the step count (versioned
 * binary file).  Synchronous. */
int pk_seeder_save(pk_ctx *ctx, int32_t seeder_id, const char *path);
int pk_seeder_load(pk_ctx *ctx, int32_t seeder_id, const char *path);

/* ------------------------------------------------------------ IK-Beam
 * Beam search over LM (Sec. V-C, runtime analysis: 64 seeds, 6 iterations on
 * all of them, the 4 of lowest error kept for 10 more, the best returned).
 * Per target:
 *   1. stage 0: LM from each of its n_seeds seeds for iters0 iterations;
 *   2. the first `keep` of them in the survivor order below;
 *   3. stage 1: LM again from their stage-0 joints, lambda back at lambda0,
 *      for iters1 iterations;
 *   4. the first of the survivors' stage-1 results in the same order.
 * Survivor order: a seed within tolerance before one that is not; among those
 * within tolerance the lower total cost first, among the others the lower
 * pose-only residual sum of squares; a NaN value after every number; then
 * the lower seed index.  When no value is NaN its first element is the
 * best-of-K choice of pk_ik_solve.
 * The LM options apply to both stages except max_iters (iters0 / iters1).
 * seeds (device): [n][T*n_seeds], problem t*n_seeds + k is seed k of target t.
 * Asynchronous on `stream`; no host synchronisation inside.  Errors:
 * PK_EINVAL for a NULL required pointer or a schedule outside the ranges
 * below, PK_EUNSUPPORTED for T*n_seeds >= 2^31. */
typedef struct {
    int32_t n_seeds;                 /* 1..64 seeds per target                   */
    int32_t iters0;                  /* >= 0, stage-0 LM iterations (paper: 6)   */
    int32_t keep;                    /* 1..n_seeds survivors (paper: 4)          */
    int32_t iters1;                  /* >= 0, stage-1 LM iterations (paper: 10)  */
} pk_beam_schedule;

/* Outputs (device).  best_joints is required; every other pointer may be
 * NULL.  The stage arrays expose the intermediate results (parity checks,
 * debugging); without them the library keeps those in its own workspace. */
typedef struct {
    float *best_joints;              /* [n][T] the returned solution             */
    int32_t *best_index;             /* [T] its stage-0 seed index, 0..n_seeds-1  */
    int32_t *target_success;         /* [T] 1 if it meets the tolerance           */
    float *pos_err;                  /* [m][T] at best_joints                     */
    float *rot_err;                  /* [m][T]                                    */
    float *cost;                     /* [T] total cost at best_joints             */
    float *stage0_joints;            /* [n][T*n_seeds]                            */
    float *stage0_cost;              /* [T*n_seeds]                               */
    float *stage0_pose_cost;         /* [T*n_seeds] pose-only residual sum of squares */
    int32_t *stage0_status;          /* [T*n_seeds] PK_CONVERGED.. | flags         */
    int32_t *kept;                   /* [T][keep] survivors' seed indices, in order */
    float *stage1_joints;            /* [n][T*keep] problem t*keep + r: survivor r */
    float *stage1_cost;              /* [T*keep]                                  */
    float *stage1_pose_cost;         /* [T*keep]                                  */
    int32_t *stage1_status;          /* [T*keep]                                  */
} pk_beam_outputs;

int pk_ik_beam(pk_ctx *ctx, int32_t robot_id, int64_t n_targets, const float *targets,
               const float *seeds, const pk_cost_weights *w, const pk_lm_options *opt,
               const pk_beam_schedule *sched, const pk_beam_outputs *out, void *stream);

/* ------------------------------------------------- trajectory optimisation
 * LM over trajectories of T configurations (Sec. II: each configuration
 * interacts only with its temporal neighbours; Sec. III-C costs).  Per
 * trajectory the variables are q_0 .. q_{T-1} (n each, time-major) and the
 * weighted residual rows are
 *   start pose: log(T_start^-1 T_ee(q_0)) as in pk_cost_weights (w_pos, w_rot),
 *   goal pose:  the same at q_{T-1},
 *   limits:     w_limit (max(0, q - upper) + max(0, lower - q)) at every t,
 *   smoothness: w_smooth (q_t - q_{t-1}), t = 1 .. T-1,
 *   velocity:   w_vel max(0, |q_t - q_{t-1}| - vmax dt), t = 1 .. T-1,
 *   acceleration: w_acc (-q_{t-2} + 16 q_{t-1} - 30 q_t + 16 q_{t+1} - q_{t+2}) / (12 dt^2),
 *   jerk:       w_jerk (-q_{t-2} + 2 q_{t-1} - 2 q_{t+1} + q_{t+2}) / (2 dt^3),
 *               both t = 2 .. T-3 (five-point stencils).
 * The LM controller is pk_ik_solve's (pk_lm_options; success = both
 * endpoint poses within tol_pos / tol_rot).  J^T J is banded with
 * half-bandwidth 4n; it is formed and factored in FP64 (a pivot not above
 * pivot_rel times the largest damped diagonal rejects the step).  Robots: one chain of 4, 6, 7 or 10 joints (revolute or
 * prismatic, no mimic joints) with one pose EE; T >= 5 and T * n <= 256.
 * Asynchronous on `stream`.  Errors: PK_EINVAL (NULL pointer, bad sizes or
 * costs, w_vel != 0 without vmax), PK_EUNSUPPORTED (robot shape). */
typedef struct {
    int64_t B;                       /* trajectories                              */
    int32_t T;                       /* timesteps                                 */
    const float *start;              /* device [7][B]: p, quaternion wxyz          */
    const float *goal;               /* device [7][B]                              */
    const float *init;               /* device [B][T][n] initial trajectories      */
} pk_traj_problem;

typedef struct {
    float dt;                        /* seconds between configurations            */
    float w_pos, w_rot;              /* start / goal pose rows                    */
    float w_limit, w_smooth, w_vel, w_acc, w_jerk;
    const float *vmax;               /* device [n] velocity limits; NULL only with
                                        w_vel == 0 (no velocity rows), else PK_EINVAL */
} pk_traj_costs;

typedef struct {
    float *traj;                     /* [B][T][n] required                        */
    float *cost;                     /* [B] final sum of squared residuals        */
    int32_t *iters;                  /* [B]                                       */
    int32_t *accepts;                /* [B]                                       */
    int32_t *status;                 /* [B] PK_CONVERGED / PK_MAX_ITERS / PK_STALLED */
    float *pos_err;                  /* [2][B] start, goal                        */
    float *rot_err;                  /* [2][B]                                    */
} pk_traj_outputs;

int pk_traj_solve(pk_ctx *ctx, int32_t robot_id, const pk_traj_problem *problem,
                  const pk_traj_costs *costs, const pk_lm_options *opt,
                  const pk_traj_outputs *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PKMI_H */
