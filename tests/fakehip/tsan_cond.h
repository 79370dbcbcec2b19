// Forced include of the ThreadSanitizer build of the serving tests -- TEST
// INFRASTRUCTURE ONLY.  This libstdc++ implements steady-clock timed waits
// of std::condition_variable with pthread_cond_clockwait, which this
// compiler's ThreadSanitizer does not intercept: it would miss the unlock
// inside the wait and report false double locks and races.  Without the
// macro the library falls back to pthread_cond_timedwait, which it sees.
#pragma once
#include <bits/c++config.h>
#undef _GLIBCXX_USE_PTHREAD_COND_CLOCKWAIT
