// ff_api.hip -- library-wide entry points: status strings, version, build
// information and the per-thread record of the last HIP error.
#include <cstdio>
#include <cstring>

#include "ff_host.h"

namespace {
thread_local char g_last_error[256] = "";
}

namespace ffh {

ff_status hip_failure(hipError_t err)
{
    std::snprintf(g_last_error, sizeof(g_last_error), "%s (%d): %s", hipGetErrorName(err),
                  static_cast<int>(err), hipGetErrorString(err));
    if (err == hipErrorNoBinaryForGpu || err == hipErrorInvalidDeviceFunction)
        return FF_ERR_UNSUPPORTED;
    return FF_ERR_HIP;
}

} // namespace ffh

extern "C" {

const char *ff_status_str(ff_status status)
{
    switch (status) {
    case FF_OK: return "FF_OK";
    case FF_ERR_NULL: return "FF_ERR_NULL";
    case FF_ERR_SIZE: return "FF_ERR_SIZE";
    case FF_ERR_ALIGN: return "FF_ERR_ALIGN";
    case FF_ERR_WORKSPACE: return "FF_ERR_WORKSPACE";
    case FF_ERR_UNSUPPORTED: return "FF_ERR_UNSUPPORTED";
    case FF_ERR_HIP: return "FF_ERR_HIP";
    case FF_ERR_ARG: return "FF_ERR_ARG";
    default: return "FF_ERR_UNKNOWN";
    }
}

int32_t ff_abi_version(void) { return FF_ABI_VERSION; }

#define FF_STRINGIFY_(x) #x
#define FF_STRINGIFY(x) FF_STRINGIFY_(x)

const char *ff_build_info(void)
{
    return "libff abi=" FF_STRINGIFY(FF_ABI_VERSION)
           "; target=gfx950"
           "; fp-contract=off"
           "; f32-denormals=preserve"
           "; f32-division=correctly-rounded"
           "; twoprod=fma(ff_mul,ff_div) dekker-split-4097(ff_mul_dekker)"
           "; add12=branch-free-6-op";
}

const char *ff_last_error(void) { return g_last_error; }

} // extern "C"
