// Quantum-number block-sparse rotation (grouped small GEMMs).
#include <hip/hip_runtime.h>

#include <string>

#include "rot_internal.h"

namespace rot {

size_t blocked_workspace_bytes(const rot_blocked_problem* p) {
    (void)p;
    return 0;
}

rot_status blocked_validate(const rot_blocked_problem* p, std::string* why) {
    (void)p;
    *why = "rot_batch_blocked is not implemented yet";
    return ROT_ERR_UNSUPPORTED;
}

hipError_t rotate_blocked(const rot_blocked_problem* p, void* ws, size_t ws_bytes, hipStream_t stream) {
    (void)p; (void)ws; (void)ws_bytes; (void)stream;
    return hipErrorNotSupported;
}

}  // namespace rot
