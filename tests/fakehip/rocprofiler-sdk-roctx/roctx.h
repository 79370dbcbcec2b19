// Stand-in for the roctx marker API -- TEST INFRASTRUCTURE ONLY.  The fake
// runtime counts ranges so that the serving tests can check that every range
// the host runtime opens is closed.
#pragma once
#include <stdint.h>

typedef uint64_t roctx_range_id_t;

extern "C" {
void roctxMarkA(const char* message);
int roctxRangePushA(const char* message);
int roctxRangePop(void);
roctx_range_id_t roctxRangeStartA(const char* message);
void roctxRangeStop(roctx_range_id_t id);
}

namespace fakehip {
long roctx_started();     // ranges started (roctxRangeStartA)
long roctx_open();        // started minus stopped; negative if an id was stopped twice
long roctx_pushed();      // roctxRangePushA calls
int roctx_depth();        // push depth of the calling thread
bool roctx_saw(const char* substring);  // some started range's name contains it
}
