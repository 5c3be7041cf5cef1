// Destination tile of a gather, shared by the plan (host) and the kernels.
#pragma once
#include <cstdint>

namespace fscc {

// A tile of at most 16 x 16 elements of one row-major destination block
// (leading dimension ld): elements k0 + r*ld + c for r < nr, c < nc.
struct GTile {
    int64_t k0;
    int32_t ld;
    int16_t nr, nc;
};

}  // namespace fscc
