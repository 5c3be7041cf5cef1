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

// How one term of a reorder reads its source over one destination tile of an
// affine traversal: element (r, c) of the tile takes
//   s0 >= 0:  (-1 if bit 62 of s0) * src[(s0 & ~bit62) + r*sa + c*sb]
//   s0 == RTERM_ZERO:   nothing (a structural zero over the whole tile)
//   s0 == RTERM_MAPPED: the term's per-element map (no affine form here)
struct RTerm {
    int64_t s0;
    int32_t sa, sb;
};
// A work unit of an affine traversal: rects [first, first + count) of the
// op's affine tiles, at most RUNIT_MAX_RECTS of them and RUNIT_MAX_ELEMS
// destination elements together, processed by one wave.
struct RUnit {
    int32_t first, count;
};
constexpr int RUNIT_MAX_RECTS = 8;
constexpr int RUNIT_MAX_ELEMS = 256;
constexpr int64_t RTERM_ZERO = -1;
constexpr int64_t RTERM_MAPPED = -2;
constexpr int64_t RTERM_NEG = (int64_t)1 << 62;

}  // namespace fscc
