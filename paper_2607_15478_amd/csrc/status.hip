// Status strings of the C ABI.
#include "common.h"

extern "C" const char* pardtw_status_string(pardtw_status status) {
    switch (status) {
        case PARDTW_OK: return "ok";
        case PARDTW_ERR_INVALID_ARG: return "invalid argument";
        case PARDTW_ERR_WORKSPACE: return "workspace missing or too small";
        case PARDTW_ERR_HIP: return "HIP runtime or launch error";
        case PARDTW_ERR_UNSUPPORTED: return "unsupported combination";
    }
    return "unknown status";
}
