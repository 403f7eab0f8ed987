// ff_host.h -- host-side helpers shared by the C-ABI translation units:
// argument checks and HIP error capture.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ff.h"

namespace ffh {

inline bool aligned(const void *p, uintptr_t bytes)
{
    return (reinterpret_cast<uintptr_t>(p) % bytes) == 0;
}

// Remember the text of a HIP error for ff_last_error() (per host thread) and
// map it to a status: a missing gfx950 code object means the device is not
// supported, anything else is a runtime failure.
ff_status hip_failure(hipError_t err);

// Status of the launches just enqueued on this thread.
inline ff_status launch_status()
{
    const hipError_t err = hipGetLastError();
    return err == hipSuccess ? FF_OK : hip_failure(err);
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Ceiling division for non-negative values.
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

} // namespace ffh
