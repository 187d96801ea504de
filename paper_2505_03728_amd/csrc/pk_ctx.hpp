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
};

namespace pk {

// Records the message on ctx (or the global slot when ctx is NULL) and
// returns code.
int fail(pk_ctx *ctx, int code, const char *fmt, ...);
RobotEntry *robot_of(pk_ctx *ctx, int32_t id);

}  // namespace pk

#define PK_HIP(ctx, call)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::pk::fail(ctx, PK_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)
