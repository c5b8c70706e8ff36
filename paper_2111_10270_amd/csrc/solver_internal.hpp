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
// keeping the tiles it has alone.  Only the small tables are built on the
// host; the big ones are assembled on the device when the batch is bound with
// solver_bind_assembled.  slot_off[k]: first slot of instance k.
int solver_load_virtual(bddmma_solver *s, const std::vector<const bddmma_solver *> &parts,
                        std::vector<int64_t> &slot_off);

// Bind such a batch: its big tables are copied (with their index shifts) on
// the device from the member images (images[k]: device address of the image
// of parts[k], image_bytes[k] its size, as solver_image wrote it); scratch
// holds the copy descriptors.  Ordered on hip_stream; synchronises it.
int solver_bind_assembled(bddmma_solver *s, void *dev_ptr, size_t bytes, void *hip_stream,
                          const std::vector<const bddmma_solver *> &parts, const std::vector<uint64_t> &images,
                          const std::vector<uint64_t> &image_bytes, void *scratch, size_t scratch_bytes);

// Host image of a loaded single instance's tables, and its size.
int solver_image(const bddmma_solver *s, std::vector<uint8_t> &buf);
uint64_t solver_image_bytes(const bddmma_solver *s);

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

// Bind s to the library's static workspace (dev_ptr, bytes) on HIP device
// `device`; as bddmma_bind, and the solver remembers the device so that its
// later calls fail once another solver holds that device's array.
int solver_bind_static(bddmma_solver *s, void *dev_ptr, size_t bytes, void *hip_stream, int device);

// A pinned host buffer of `bytes` that s uses for its readbacks while it
// fits, owned by the caller (a serving pool lends one to its batches); no
// effect on a solver that already owns one.
void solver_lend_pinned(bddmma_solver *s, void *pin, size_t bytes);

// Whether s holds the static workspace of `device` (static_workspace.hip),
// and its release when s is destroyed.
bool static_workspace_held(const bddmma_solver *s, int device);
void static_workspace_forget(const bddmma_solver *s, int device);

}  // namespace bddmma
