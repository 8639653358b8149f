// Raw buffer descriptors on gfx950, shared by the kernels that address
// memory through them (gemm_bf16x3.hip, blocked.hip).
#pragma once

namespace rot {

// Dword 3 of a descriptor for untyped 32-bit data.  With stride 0 the
// hardware checks each access against num_records bytes: a load at or past
// it returns zero, a store there is dropped.
constexpr int kBufferFlags = 0x00020000;

}  // namespace rot
