// ldp_status.cpp -- status strings and version of the C ABI.
#include "../../include/ldp.h"

extern "C" {

const char *ldp_status_string(int status)
{
    switch (status) {
    case LDP_OK: return "ok";
    case LDP_ERR_INVALID_ARG: return "invalid argument";
    case LDP_ERR_HIP: return "HIP runtime error";
    case LDP_ERR_NO_MEMORY: return "out of memory or plan capacity";
    case LDP_ERR_UNSUPPORTED: return "unsupported size or configuration";
    case LDP_ERR_BUSY: return "resource busy";
    }
    return "unknown status";
}

int ldp_version(void) { return 1; }

}  // extern "C"
