// Status strings and version of the C ABI.
#include "common.hpp"

extern "C" const char* harp_status_str(harp_status s) {
    switch (s) {
        case HARP_OK: return "ok";
        case HARP_E_ARG: return "invalid argument";
        case HARP_E_DOMAIN: return "antenna pair closer than the model's inner radius r_min";
        case HARP_E_SINGULAR: return "exact zero pivot";
        case HARP_E_NOCONV: return "iterative refinement did not reach its tolerance";
        case HARP_E_HIP: return "HIP runtime error";
        case HARP_E_WORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

extern "C" int32_t harp_version(void) { return 100; }
