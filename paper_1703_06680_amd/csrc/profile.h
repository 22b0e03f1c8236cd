// Optional per-phase GPU timing with HIP events (diagnostic).
//
// When enabled, every launch site calls mark(stream, "phase") just before it
// enqueues work; consecutive marks on a stream delimit one phase, whose
// duration (hipEventElapsedTime between the two events) is added to the
// phase's running total once the call has synchronised.  Disabled, mark() is
// a branch.  The recorder is process-global and not thread-safe: profile from
// one host thread.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ddm {
namespace prof {

bool enabled();
// Sets recording on or off and returns the previous setting (recording is
// switched off while a graph is captured).
bool swap_enabled(bool on);
void mark(hipStream_t s, const char *phase);
void end(hipStream_t s);
// Resolve the recorded events (the stream must have been synchronised).
void flush();

}  // namespace prof
}  // namespace ddm
