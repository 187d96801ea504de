// Host-side context of the library (shared by the C-ABI source files).
#pragma once

#include <string>
#include <vector>

#include "pk_internal.hpp"

namespace pk {

struct RobotEntry {
    RobotC host;
    RobotC *dev = nullptr;
};

struct SeederState;
void seeder_free(SeederState *s);

}  // namespace pk

struct pk_ctx {
    int device = 0;
    std::string err;
    std::vector<pk::RobotEntry> robots;
    std::vector<pk::SeederState *> seeders;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *ws2 = nullptr;      // learned-seed pipeline workspace
    size_t ws2_bytes = 0;
    void *ws3 = nullptr;      // IK-Beam workspace
    size_t ws3_bytes = 0;
};

namespace pk {

// Records the message on ctx (or the global slot when ctx is NULL) and
// returns code.
int fail(pk_ctx *ctx, int code, const char *fmt, ...);
RobotEntry *robot_of(pk_ctx *ctx, int32_t id);
// Validates LM options and weights; fills P (everything but the buffers) and
// resolves the kernel variant.  Returns PK_OK or an error (message set).
int prepare_solve(pk_ctx *ctx, const RobotEntry &rb, const pk_cost_weights *w,
                  const pk_lm_options *o, SolveParams &P, int &variant);
// best: best-of-K in the LM launch itself (per-lane kernel only; see launch_lm_lane).
hipError_t launch_lm(const RobotEntry &rb, const SolveParams &P, int variant, hipStream_t s,
                     int persist_blocks = 0, const BestOut *best = nullptr);
void sched_free(pk_ctx *ctx);
// Reads the autotune table named by PK_AUTOTUNE_TABLE, if any, into ctx.
void sched_load_env(pk_ctx *ctx);
// The mixed scheduler on these groups (no argument checks beyond the
// per-group ones); used by the seeded pipeline's refinement.
int sched_run(pk_ctx *ctx, int n_groups, const pk_ik_group *groups, const pk_lm_options *opt,
              const pk_sched_options &sch, hipStream_t stream);
// Seeder inference into seeds [n][T*K] (device), asynchronous.
int seeder_infer_into(pk_ctx *ctx, int32_t seeder_id, const float *targets, int64_t T,
                      float *seeds, hipStream_t s, int32_t *K_out, int32_t *robot_out);

}  // namespace pk

#define PK_HIP(ctx, call)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::pk::fail(ctx, PK_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)
