// Status strings of the DDHF C ABI.
#include "ddhf_internal.h"

extern "C" const char* ddhf_status_string(int status) {
    switch (status) {
        case DDHF_OK: return "ok";
        case DDHF_EINVAL: return "invalid argument";
        case DDHF_ENOSPACE: return "workspace too small";
        case DDHF_EHIP: return "HIP launch or runtime error";
        case DDHF_ETRUNC: return "result truncated";
        default: return "unknown status";
    }
}
