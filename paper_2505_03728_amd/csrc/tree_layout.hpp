// Host-side tables of the tree factorisation: the leaves-first elimination
// schedule and the path-pair layout (PathC) of the one-problem-per-wavefront
// LM kernel.  Used by pk_robot_upload, and by the CPU test of the layout,
// which solves random trees with these tables.
#pragma once

#include <string.h>

#include "pk_internal.hpp"

namespace pk {

// Elimination steps (R.nstep, step_start, step_joint, step_of, step_pos):
// joints by height (leaves 0, a parent one above its highest child),
// descending index within a height, at most PK_STEP_PIVOTS per step.  No
// joint of a step is an ancestor of another, and all their descendants fall
// in earlier steps.  Needs R.n and the parents.
inline void build_step_schedule(RobotC &R)
{
    const int n = R.n;
    int h[PK_MAX_JOINTS] = {0};
    int hmax = 0;
    for (int j = n - 1; j >= 0; --j) {
        const int par = R.j[j].parent;
        if (par >= 0 && h[par] < h[j] + 1) h[par] = h[j] + 1;
    }
    for (int j = 0; j < n; ++j) hmax = h[j] > hmax ? h[j] : hmax;
    int ns = 0, pos = 0;
    for (int lv = 0; lv <= hmax; ++lv) {
        int inlev = 0;
        for (int j = n - 1; j >= 0; --j) {
            if (h[j] != lv) continue;
            if (inlev % PK_STEP_PIVOTS == 0) R.step_start[ns++] = (uint8_t)pos;
            R.step_of[j] = (uint8_t)(ns - 1);
            R.step_pos[j] = (uint8_t)(inlev % PK_STEP_PIVOTS);
            R.step_joint[pos++] = (uint8_t)j;
            ++inlev;
        }
    }
    R.step_start[ns] = (uint8_t)pos;
    R.nstep = ns;
}

// Path-pair layout (PathC) of the wavefront kernel that gives each (joint,
// EE path) pair a lane.  Leaves R.path.ok = 0 when the robot does not fit it
// (mimic joints, more than PK_PATH_MAX_DEPTH levels, more than 64 pairs).
// Needs R's joints, EEs, ancestor sets and elimination schedule.
inline void build_path_layout(RobotC &R)
{
    PathC &Pc = R.path;
    memset(&Pc, 0, sizeof Pc);
    const int n = R.n, m = R.m;
    if (R.n_mimic > 0 || R.max_depth + 1 > PK_PATH_MAX_DEPTH) return;
    int lane_of[PK_MAX_JOINTS][PK_MAX_EES], own_lane[PK_MAX_JOINTS], og[PK_MAX_JOINTS];
    for (int j = 0; j < n; ++j) {
        own_lane[j] = og[j] = -1;
        for (int k = 0; k < PK_MAX_EES; ++k) lane_of[j][k] = -1;
    }
    int lanes = 0;
    for (int k = 0; k < m; ++k) {
        const int e = R.e[k].joint;
        for (int d = 0; d <= R.j[e].depth; ++d) {
            if (lanes >= 64) return;
            const int j = R.anc_at[e][d];
            lane_of[j][k] = lanes;
            Pc.joint[lanes] = (uint8_t)j;
            Pc.group[lanes] = (int8_t)k;
            ++lanes;
        }
    }
    for (int j = 0; j < n; ++j) {
        for (int k = 0; k < m && og[j] < 0; ++k)
            if (lane_of[j][k] >= 0) og[j] = k;
        if (og[j] >= 0) {
            own_lane[j] = lane_of[j][og[j]];
            continue;
        }
        if (lanes >= 64) return;   // a joint on no EE path: one lane of its own
        own_lane[j] = lanes;
        Pc.joint[lanes] = (uint8_t)j;
        Pc.group[lanes] = -1;
        ++lanes;
    }
    Pc.lanes = lanes;
    memset(Pc.merge_step, PK_PATH_NONE, sizeof Pc.merge_step);
    memset(Pc.copies, PK_PATH_NONE, sizeof Pc.copies);
    for (int l = 0; l < 64; ++l) {
        Pc.lane_ee[l] = -1;
        for (int d = 0; d < PK_PATH_MAX_DEPTH; ++d) Pc.anc[l][d] = (uint8_t)l;
    }
    for (int k = 0; k < m; ++k) Pc.lane_ee[lane_of[R.e[k].joint][k]] = (int8_t)k;
    uint32_t pdep[PK_MAX_JOINTS] = {0}, mdep[PK_MAX_JOINTS] = {0};
    for (int l = 0; l < lanes; ++l) {
        const int j = Pc.joint[l], k = Pc.group[l], dep = R.j[j].depth;
        Pc.owner[l] = (uint8_t)own_lane[j];
        if (k < 0) continue;
        for (int d = 0; d <= dep; ++d) Pc.anc[l][d] = (uint8_t)lane_of[R.anc_at[j][d]][k];
        for (int b = 0; b < 4; ++b) {
            const int d = dep - (1 << b);
            Pc.jump[l] |= (uint32_t)(d >= 0 ? lane_of[R.anc_at[j][d]][k] : l) << (8 * b);
        }
        // updates: the pivots owned by path k below joint j
        for (int i = 0; i < n; ++i)
            if (og[i] == k && ((R.janc[i] >> j) & 1ull)) Pc.upd[l] |= 1ull << R.step_of[i];
    }
    for (int i = 0; i < n; ++i)
        if (og[i] >= 0 && pdep[R.step_of[i]] < (uint32_t)R.j[i].depth) pdep[R.step_of[i]] = R.j[i].depth;
    int ncopy = 0;
    for (int j = 0; j < n; ++j) {
        if (og[j] < 0) continue;
        int c = 0;
        for (int k = og[j] + 1; k < m; ++k)
            if (lane_of[j][k] >= 0) Pc.copies[own_lane[j]][c++] = (uint8_t)lane_of[j][k];
        if (c == 0) continue;
        ncopy = c > ncopy ? c : ncopy;
        Pc.copy_depths |= 1u << R.j[j].depth;
        // The other copies take updates only from pivots of their own paths
        // below j; the merge follows the last of them.
        int ms = 0;
        for (int i = 0; i < n; ++i)
            if (((R.janc[i] >> j) & 1ull) && og[i] != og[j] && R.step_of[i] + 1 > ms) ms = R.step_of[i] + 1;
        Pc.merge_step[own_lane[j]] = (uint8_t)ms;
        if (mdep[ms] < (uint32_t)R.j[j].depth + 1) mdep[ms] = R.j[j].depth + 1;
    }
    Pc.ncopy = ncopy;
    for (int s = 0; s < R.nstep; ++s) Pc.step_info[s] = pdep[s] | (mdep[s] << 8);
    Pc.ok = 1;
}

}  // namespace pk
