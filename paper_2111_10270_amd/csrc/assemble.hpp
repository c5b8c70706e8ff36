// Device assembly of a batch from per-instance table images: one copy step
// ("segment") per table range, with the index shift that the instance's place
// in the batch needs.  Shared by the host planner and the copy kernel.
#pragma once
#include <cstdint>

namespace bddmma {

enum SegOp : int32_t {
    SEG_COPY = 0,     // dst[i] = src[i]
    SEG_ADD = 1,      // dst[i] = src[i] + a          (elem 4: int32, 8: int64)
    SEG_PADVAR = 2,   // dst[i] = src[i] == b ? c : src[i] + a   (elem 4)
    SEG_FILL = 3,     // dst[i] = a                   (elem 4 or 8; src unused)
};

struct Seg {
    uint64_t src, dst;   // byte addresses
    int64_t n;           // elements
    int32_t op, elem;    // SegOp, element bytes (1, 2, 4, 8)
    int64_t a, b, c;
    int64_t pad;
};
static_assert(sizeof(Seg) == 64, "Seg is 64 bytes");

// elements of one segment handled by one block of the copy kernel
constexpr int64_t kSegChunk = 16384;

}  // namespace bddmma
