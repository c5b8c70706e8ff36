// Solver hooks used by the serving pool (pool.cpp); not part of the C ABI.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "bddmma.h"

namespace bddmma {

// set the calling thread's bddmma_last_error message; returns code
int set_error(int code, const std::string &msg);

// Load into the fresh solver s (created, nothing loaded) the batch of the
// loaded single-instance solvers `parts` (same precision as s), each instance
// keeping the tiles it has alone.  slot_off[k]: first slot of instance k.
int solver_load_merged(bddmma_solver *s, const std::vector<const bddmma_solver *> &parts,
                       std::vector<int64_t> &slot_off);

int64_t solver_slots(const bddmma_solver *s);

// 32 or 64 for a loaded solver, 0 otherwise
int solver_precision(const bddmma_solver *s);

// Copy lambda and M of slots [src_off, src_off + n) of src to [dst_off,
// dst_off + n) of dst, ordered on dst's stream (both bound, equal precision).
int solver_copy_slots(bddmma_solver *dst, int64_t dst_off, const bddmma_solver *src, int64_t src_off, int64_t n);

// Terminated multipliers (lambda + omega M) and M of the instance whose slots
// start at slot_off in the bound batch s, in the pair order of `part` (that
// instance loaded alone); either output may be NULL.
int solver_instance_multipliers(bddmma_solver *s, int64_t slot_off, const bddmma_solver *part, double *lam,
                                double *mm);

}  // namespace bddmma
