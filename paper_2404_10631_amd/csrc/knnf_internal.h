// knnf_internal.h -- host-runtime pieces shared by knnf_api.cpp and knnf_server.cpp.
#pragma once

#include <stdint.h>

#include "../../include/knnf.h"
#include "knnf_device.h"

namespace knnf {

// Record `st` and a formatted message as the calling thread's last error.
knnf_status set_error(knnf_status st, const char* fmt, ...);

// Frame checks of include/knnf.h (index is used in the message only).
knnf_status validate_frame(const knnf_frame* f, int index);

// Context default merged with an optional caller plan; validity check.
knnf_plan resolve_plan(const knnf_ctx* ctx, const knnf_plan* p);
bool plan_valid(const knnf_plan& p);

// Device-side description of a frame and its number of tiles under a plan.
FrameDesc desc_of(const knnf_frame& f);
uint32_t tiles_of(int H, int W, const knnf_plan& p);

// One launch over the given tile ranges, in the given order, on `stream`
// (persistent claim loop or one wavefront per task, as p.launch says).  Items must be validated.  The work table goes through one of the
// context's table slots (reused only after the launch that used it ended).
knnf_status launch_items(knnf_ctx* ctx, const WorkItem* items, int n, const knnf_plan& p,
                         void* stream);

// Device ordinal of a context.
int ctx_device(const knnf_ctx* ctx);

// KNNF_EDEVICE (and the message) once the context has failed, else KNNF_OK.
knnf_status ctx_status(const knnf_ctx* ctx);

// Mark the context failed (a server's HIP call failed on it).
void ctx_mark_failed(knnf_ctx* ctx, const char* what);

}  // namespace knnf
