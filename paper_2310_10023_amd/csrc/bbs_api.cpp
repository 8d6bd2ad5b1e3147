// Error reporting and version of the libbbs C ABI.
#include <string>

#include "bbs_internal.h"

namespace bbs {

namespace {
thread_local std::string g_last_error;
}

const char *last_error_cstr() { return g_last_error.c_str(); }

void set_error(const std::string &msg) { g_last_error = msg; }

bbs_status fail(bbs_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

bbs_status hip_fail(hipError_t e, const char *what)
{
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipGetLastError();
    set_error(msg);
    return e == hipErrorOutOfMemory ? BBS_ERR_OOM : BBS_ERR_DEVICE;
}

}  // namespace bbs

extern "C" const char *bbs_last_error(void) { return bbs::last_error_cstr(); }

extern "C" int32_t bbs_abi_version(void) { return BBS_ABI_VERSION; }
