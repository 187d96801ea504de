// Internal host/device definitions of the MI355X batched-LM IK library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pkmi.h"

namespace pk {

// Joints are stored in "z-axis joint frames": frame j is the paper's joint
// frame R_j rotated by a fixed U_j that maps e_z onto the joint axis, so the
// joint rotation is always Rz(q_j).  Then one joint is
//   O_j = O_parent * G_j * Rz(q_j),   p_j = p_parent + O_parent * t_j,
// with G_j = U_parent^T R_mount,j U_j and t_j = U_parent^T offset_j, and the
// world joint axis is the third column of O_j.  The host computes G and t in
// FP64 from the FP64 tree and rounds them to FP32.
struct JointC {
    float G[9];        // row-major
    float t[3];
    float lo, hi, mid;
    int32_t parent;
    float Ut[9];       // U_j^T, to report the paper's R_j = O_j U_j^T
    int32_t depth;
    int32_t type;      // PK_JOINT_REVOLUTE or PK_JOINT_PRISMATIC (fixed joints are folded away)
    int32_t var;       // variable index, -1 for a mimic joint
    int32_t mimic_src; // mimic joint: its driver (a joint index), else -1
    float mimic_a, mimic_b;   // q = mimic_a * q_driver + mimic_b
    int32_t pad;       // 128 bytes per joint: every joint's fields keep the same alignment
};
static_assert(sizeof(JointC) == 128, "JointC is 128 bytes");

struct EEC {
    float G[9];        // U_e^T R_eeoff
    float t[3];        // U_e^T ee_offset
    int32_t joint;
    int32_t kind;      // PK_EE_POSE / PK_EE_POSITION
    int32_t tgt_off;   // first target plane of this EE
    int32_t row_off;   // first residual row of this EE
};

constexpr int PK_STEP_PIVOTS = 16;   // pivots per elimination step (LDS slots)
constexpr int PK_LANE_MAX_CHAIN = 10; // longest single chain the per-lane kernel serves
constexpr int PK_PATH_MAX_DEPTH = 16; // tree levels the path-pair wavefront kernel serves
constexpr uint8_t PK_PATH_NONE = 0xff;

// Path-pair layout of one problem on a 64-lane wavefront.  Lane l holds the
// pair (joint[l], path group[l]): every joint on the path from the root to EE
// k has a lane in group k, so a joint shared by several EE paths has one copy
// per path; a joint on no EE path has one lane with group -1.  Each copy holds
// the part of its joint's row of J^T J that its path's EE rows give; the
// owner copy (the one in the lowest-numbered path) also holds the limit and
// rest rows and, once the other copies are merged into it, the whole row.
struct PathC {
    int32_t ok;                    // the layout applies to this robot
    int32_t lanes;                 // lanes in use
    int32_t ncopy;                 // most copies of one joint, minus one
    uint32_t copy_depths;          // bit d: some joint at depth d has more than one copy
    uint8_t joint[64];             // lane -> joint
    int8_t group[64];              // lane -> EE path (-1: the joint is on no EE path)
    uint8_t owner[64];             // lane -> lane of its joint's owner copy
    uint8_t merge_step[64];        // owner lanes of shared joints: the step whose merge phase
                                   // adds the other copies' rows (PK_PATH_NONE: no merge)
    int8_t lane_ee[64];            // lane -> the EE whose joint it holds in that EE's path (-1)
    uint8_t anc[64][PK_PATH_MAX_DEPTH];   // [l][d]: lane of l's ancestor at depth d in l's path
                                          // (l itself at its depth and beyond, and for group -1)
    uint8_t copies[64][8];         // owner lanes: the other copies' lanes (PK_PATH_NONE-padded)
    uint32_t jump[64];             // byte k: lane of l's path ancestor 2^k levels up (l if none)
    uint64_t upd[64];              // bit s: at step s the pivot owned by l's path lies below l's joint
    uint32_t step_info[64];        // [s] bits 0-7: deepest pivot depth of step s; bits 8-15:
                                   // 1 + deepest depth merged at step s (0: no merge phase)
};

struct RobotC {
    int32_t n, m, tgt_floats, pose_rows;   // pose_rows = sum of EE row counts
    int32_t chains, chain_len, max_depth, prismatic;   // prismatic: count of prismatic joints
    uint64_t anc[PK_MAX_EES];              // bit j set iff joint j is an ancestor of EE k
    JointC j[PK_MAX_JOINTS];
    EEC e[PK_MAX_EES];
    float mid[PK_MAX_JOINTS];              // (lower + upper) / 2, the default rest pose
    uint64_t janc[PK_MAX_JOINTS];          // bit i set iff joint i is a proper ancestor of joint j
    uint64_t jdesc[PK_MAX_JOINTS];         // bit k set iff joint j is a proper ancestor of joint k
    uint8_t anc_at[PK_MAX_JOINTS][PK_MAX_JOINTS];   // [j][d]: ancestor of j at depth d (d <= depth j; j itself at its depth)
    // Elimination schedule of the tree factorization: step s removes the
    // joints step_joint[step_start[s] .. step_start[s+1]) (at most
    // PK_STEP_PIVOTS, none an ancestor of another, all their descendants
    // removed in earlier steps); joint j is pivot step_pos[j] of step step_of[j].
    int32_t nstep, pad2;
    // Variables: the joints that are not mimic joints (nv of them, in joint
    // order); the mimic joints, listed.
    int32_t nv, n_mimic;
    uint8_t mimic_list[PK_MAX_JOINTS];
    uint8_t step_start[PK_MAX_JOINTS + 1];
    uint8_t step_joint[PK_MAX_JOINTS];
    uint8_t step_of[PK_MAX_JOINTS];
    uint8_t step_pos[PK_MAX_JOINTS];
    PathC path;
};

// Uniform per-call data for the LM kernels (passed by value).
struct SolveParams {
    float w_pos, w_rot, w_limit, w_rest;
    float lambda0, nu_up, nu_down, lambda_min, lambda_max;
    float tol_pos, tol_rot, damping_floor, pivot_rel;
    int32_t max_iters, early_exit, K, trace_iters;
    int64_t N, T;
    const float *targets, *seeds, *q_rest;
    float *joints, *pos_err, *rot_err, *cost, *pose_cost;
    int32_t *iters, *accepts, *status, *iters_to_tol;
    float *trace_q;
    int32_t *trace_acc;
    // Optional active list: thread/wave i < *n_active (or N) solves problem
    // active[i] (or i).  Lets a launch sized for N run a device-chosen subset.
    const int32_t *active;
    const int32_t *n_active;
    // Resumable execution (persistent scheduler).  With st_state set, a
    // problem's LM state persists in HBM between launches: q in `joints`,
    // lambda in st_lambda, counters in iters/accepts/iters_to_tol and the
    // done/stalled/FP64 bits in st_state.  resume = 0 starts from the seeds;
    // each launch runs at most iter_budget more iterations.
    float *st_lambda;
    int32_t *st_state;
    int32_t resume;
    int32_t iter_budget;
    // Per-lane kernel: a problem started from its seed also ends once a
    // problem of its target in its run of consecutive lanes met the tolerance.
    int32_t target_exit;
    // Persistent launch: blocks pop work items (64 problems for the per-lane
    // kernel, 1 for the wave kernel) from *queue_head until none are left.
    int32_t *queue_head;
};

// st_state bits
#define PK_ST_DONE 0x10000
#define PK_ST_STALLED 0x20000

// Best-of-K outputs written by the per-lane kernel itself (its K problems of
// a target share a wavefront when K divides 64); NULL pointers are skipped.
struct BestOut {
    int32_t *index;
    float *joints;     // [n][T]
    int32_t *success;
};

// Launchers (defined next to their kernels).  Return hipSuccess or the
// launch error.
bool lane_variant_available(int chains, int chain_len, int kind);
// persist_blocks: grid size when P.queue_head is set (0 = one block per item).
// best (non-persistent launches without an active list, K dividing 64 only):
// best-of-K in the same launch.
hipError_t launch_lm_lane(const RobotC *dev_robot, const RobotC &host_robot,
                          const SolveParams &P, hipStream_t s, int persist_blocks = 0,
                          const BestOut *best = nullptr);
bool wave_variant_available(int n);
hipError_t launch_lm_wave(const RobotC *dev_robot, const RobotC &host_robot,
                          const SolveParams &P, hipStream_t s, int persist_blocks = 0);
bool path_variant_available(const RobotC &host_robot);
hipError_t launch_lm_path(const RobotC *dev_robot, const RobotC &host_robot,
                          const SolveParams &P, hipStream_t s, int persist_blocks = 0);
hipError_t launch_best_of_k(const SolveParams &P, int n, int32_t *best_index,
                            float *best_joints, int32_t *success, hipStream_t s);
hipError_t launch_fk(const RobotC *dev_robot, int64_t N, const float *q, float *ee_pose,
                     float *joint_frames, hipStream_t s);
hipError_t launch_residual_jacobian(const RobotC *dev_robot, int64_t N, int32_t K,
                                    const float *targets, const float *q,
                                    const SolveParams &w, float *r, float *J, hipStream_t s);

}  // namespace pk
