// Device-side description of a mixed batch for the single persistent LM
// launch (lm_mixed.hip), built on the host by the scheduler (sched.hip).
//
// A batch is up to PK_MAX_GROUPS groups; each group is one robot with its
// problems, weights, outputs and resumable state (SolveParams) and the device
// path that solves it.  One round of the launch chain runs every unfinished
// problem of every group for at most k more LM iterations: a plan kernel
// turns the groups' active-list sizes into a table of work items, the
// persistent kernel's wavefronts pop items from one queue, and a compaction
// kernel packs the problems that are still unfinished into the next round's
// active lists.
#pragma once

#include "pk_internal.hpp"

namespace pk {

// Device paths of the persistent kernel (one per (lanes per problem, robot
// class) instantiation).
enum MixedPath : int32_t {
    MIX_LANE_ARM = 0,     // one problem per lane, serial 7-joint arm, one pose EE
    MIX_LANE_HAND = 1,    // one problem per lane, 4 chains of 4 joints, 4 position EEs
    MIX_WAVE_16_4 = 2,    // one problem per wavefront, lane per joint, depth <= 16 levels, <= 4 EEs
    MIX_PATH_16_4 = 3,    // one problem per wavefront, lane per (joint, EE path) pair,
                          // depth <= 16 levels, <= 4 EEs
    MIX_WAVE_64_8 = 4,    // one problem per wavefront, any tree (<= 64 joints, 8 EEs)
    MIX_PATHS = 5
};

// Groups one persistent launch serves (its description travels by value as
// kernel arguments, which keeps every buffer pointer a global-memory pointer).
constexpr int PK_MIX_GROUPS = 8;

struct MixedGroup {
    const RobotC *rb;
    const float *qr;          // rest pose: the caller's, else the robot's mid-range table
    SolveParams P;            // buffers, weights, options, resumable state and this
                              // round's active list, budget and resume flag
    int32_t *list[2];         // active lists of alternate rounds
    int32_t *count;           // [2] active-list sizes
    int32_t path;             // MixedPath
    int32_t per_item;         // problems per work item: 64 (lane paths) or 1 (wavefront paths)
};

struct MixedArgs {
    int32_t n_groups;
    int32_t round;
    MixedGroup g[PK_MIX_GROUPS];            // in queue order
};

// LDS floats one wavefront needs on a path.
int mixed_lds_floats(int path);

// Enqueues one round on stream s: plan (work items per group into item_end,
// queue head reset), persistent solve (each problem at most P.iter_budget more
// iterations), and, unless it is the last round, compaction.  a holds this
// round's fields; item_end [PK_MIX_GROUPS] and head are device buffers;
// waves = persistent wavefronts in total; wg = threads per workgroup (64, 128
// or 256); lds_floats = per-wavefront LDS (the largest over the batch's
// paths); max_n = the largest group.
hipError_t launch_mixed_round(const MixedArgs &a, int32_t *item_end, int32_t *head, int max_n,
                              bool last, int waves, int wg, int lds_floats, hipStream_t s);

}  // namespace pk
