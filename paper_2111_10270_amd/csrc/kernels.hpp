// Host-callable launchers of the solver's HIP kernels.  All pointers are
// device pointers inside the bound workspace; all launches go to `st`.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.hpp"

namespace bddmma {

// Sweep flavours: UPDATE runs the deferred parallel update of Alg. 1 while it
// sweeps; FIXED only records min-marginal differences at fixed multipliers.
enum SweepMode { MODE_UPDATE = 0, MODE_FIXED = 1 };

// LDS of one block of the wide kernel (all the BDD regions it holds)
constexpr int kWideBlockLds = 64 << 10;

struct DevProblem {
    const TileDesc *tiles;
    int64_t n_tiles;
    const int32_t *lists;              // tile ids of every TileList
    int64_t list_off[kNumLists + 1];
    int32_t list_first[kNumLists];     // first id of a list of consecutive ascending tile ids, else -1
    const uint32_t *layers;
    const uint32_t *child;
    const int32_t *pair_var;
    const int32_t *vptr;
    const int32_t *vslot;
    const uint16_t *code;              // [n_slots] source of each slot's averaged term
    const AvgBucket *gbuckets;         // variables averaged by the averaging kernel
    int32_t n_gbuckets;
    AvgBucketSet gbucket_set;          // the same descriptors, passed to the averaging kernel by value
    int64_t gblocks;
    const int32_t *gslot;
    const double *cost;
    int64_t n_vars, n_slots;
    void *scratch;          // per-tile scratch for tiles outside LDS (element type = precision)
    int lds_lane_elems;     // per-lane LDS elements of the largest LDS tile
    int wide_elems;         // LDS elements of the largest wide tile (2 * nodes + 2 * K)
    int wide_lanes;         // lanes per BDD of the wide kernel: 16, 32 or 64
    double *wide_part;      // [wide tiles * 64] per-BDD bound partials of the wide kernel
    // batches of independent instances (nullptr for a single ILP): instance
    // of every variable and tile, and the first variable of every instance
    const int32_t *var_inst;
    const int32_t *tile_inst;
    const int64_t *inst_var;
    const double *inst_tau;   // Alg. 2 zero threshold per instance (replaces tau)
    // fused averaging (layout.hpp; nullptr / 0 when the averaging kernel runs)
    const uint32_t *gmeta;    // [n_slots] entry, rank and |J_i| of slots of such variables
    const int32_t *gsrc;      // [n_g] slot of every entry
    void *gbuf;               // 2 x n_g values (element type = precision)
    int64_t n_g;
};

constexpr int kRedBlocks = 512;
constexpr int kResidualBlocks = 4096;   // blocks of launch_residual (partials in red)

// Weights of the averaged term: w1 = omega, w2 = omega / 2 in working precision.
template <typename T>
struct Omega {
    T w1, w2;
    double w64;   // omega itself (the averaged terms' weight omega/|J_i| is formed in FP64)
};

// One sweep over every tile.  dir 0 = ascending variables (Alg. 3), 1 =
// descending (Alg. 4).  MODE_UPDATE: on entry mm holds the previous sweep's M
// (read for the in-tile averaging), except at the slots of variables averaged
// by the averaging kernel, which hold their averaged term (launch_average runs
// right before); on exit mm holds this sweep's M everywhere.  With tile_lb !=
// nullptr each tile writes sum_lanes E^j + omega * sum min(M, 0).  MODE_FIXED
// writes M to mm without reading it or touching lam.
template <typename T>
void launch_sweep(const DevProblem &p, T *lam, T *mm, double *tile_lb, Omega<T> w, int dir, int mode, hipStream_t st);

// Persistent kernel: n_sweeps updating sweeps (directions dir0, dir0^1, ...)
// over the mixed register tiles of layer class ki in one cooperative launch,
// a grid-wide barrier between sweeps; sweep s writes its per-tile bound
// partials to lbpart + s * lb_stride.  Only for problems whose tiles all lie
// in that class and whose averaging is fused (or absent).  Returns 0, or -1
// when the launch is not possible (then nothing ran).
template <typename T>
int launch_persist(const DevProblem &p, int ki, T *lam, T *mm, double *lbpart, int64_t lb_stride, Omega<T> w,
                   int32_t n_sweeps, int32_t dir0, hipStream_t st);

// register-resident sweeps of the fast-path tiles of width class wi
template <typename T, int DIR, int W, bool UPD>
void launch_reg(const DevProblem &p, int wi, T *lam, T *mm, double *tile_lb, Omega<T> w, hipStream_t st);

// a_i = omega/|J_i| * sum_k M_ik (ascending row order) for the variables the
// sweep does not average itself; the term replaces M_ik at every slot of i.
// Nothing to do with fused averaging.
template <typename T>
void launch_average(const DevProblem &p, T *mm, double omega, hipStream_t st);

// fused averaging: the per-variable copy read by the next sweep (direction
// dir) from the differences in mm; needed before a run of sweeps whenever mm
// may have changed outside the sweeps (initialisation, state loads, rounding)
template <typename T>
void launch_gather_refresh(const DevProblem &p, const T *mm, int dir, hipStream_t st);

// bounds of n sweeps from their per-tile partials (row r of part, n_tiles
// each): out[r] = offset + sum of row r, in a fixed order
void launch_lb_many(const double *part, int64_t n_tiles, int64_t n, double offset, double *out, hipStream_t st);

// per-variable averaged terms of all variables into avg[n_vars] (state export)
template <typename T>
void launch_average_all(const DevProblem &p, const T *mm, T *avg, double omega, hipStream_t st);

// out[0] = offset + sum_t part[t] in a fixed order; scratch holds kRedBlocks doubles
void launch_reduce_sum(const double *part, int64_t n, double offset, double *scratch, double *out, hipStream_t st);

// lambda = c_i / |J_i|, M-bar = 0
template <typename T>
void launch_init(const DevProblem &p, T *lam, T *mm, hipStream_t st);

// lam += omega * mm on every slot
template <typename T>
void launch_terminate(const DevProblem &p, T *lam, const T *mm, T omega, hipStream_t st);

// per-tile energies in FP64 into tile_e at the dual-feasible multipliers
// lam + omega * mm - share[i] (share from launch_residual / _seg)
template <typename T>
void launch_cert(const DevProblem &p, const T *lam, const T *mm, double omega, const double *share, double *tile_e,
                 hipStream_t st);

// red[0] = sum_i max(r_i, 0), red[1] = max_i |r_i| with r_i = sum_j (lam + omega mm) - c_i;
// red holds 2 + 2 * kResidualBlocks doubles; share[i] = r_i / |J_i| ([n_vars + 1]
// doubles, share[n_vars] = 0)
template <typename T>
void launch_residual(const DevProblem &p, const T *lam, const T *mm, double omega, double *red, double *share,
                     hipStream_t st);

// counter[k] = number of variables of instance k with a zero / disagreeing
// min-marginal sign or a flag (counter[0..n_inst) is cleared first)
template <typename T>
void launch_conflicts(const DevProblem &p, const T *mm, double tau, const uint8_t *flag, int32_t *counter,
                      int64_t n_inst, hipStream_t st);

// one Alg. 2 perturbation of every variable; the random draw of variable i
// uses its index inside its instance
template <typename T>
void launch_perturb(const DevProblem &p, T *lam, const T *mm, double tau, double delta, uint64_t seed,
                    uint64_t round, int scale, const uint8_t *flag, hipStream_t st);

// xbest[i] = x[i] for the variables of instances k with take[k] != 0
void launch_take_x(const DevProblem &p, const uint8_t *x, uint8_t *xbest, const uint8_t *take, hipStream_t st);

// out[k] = offset[k] (0 if offset is null) + sum of part[seg[k] .. seg[k+1]) in a fixed order
void launch_seg_sum(const double *part, const int64_t *seg, int64_t n_seg, const double *offset, double *out,
                    hipStream_t st);

// per-instance objective sum_i cost_i x_i over [inst_var[k], inst_var[k+1]) in
// chunks of kObjChunk variables from the instance start: part[c] per chunk
// (chunk list from the host), then launch_seg_sum over each instance's chunks
constexpr int64_t kObjChunk = 1 << 12;
void launch_obj_chunks(const double *cost, const uint8_t *x, const int64_t *chunk_begin, int64_t n_chunks,
                       int64_t n_vars, double *part, hipStream_t st);

// per instance: pos[k] = sum max(r_i, 0), mx[k] = max |r_i| over its
// variables, in the objective's chunks (part_* hold one value per chunk);
// share[i] = r_i / |J_i| as launch_residual
template <typename T>
void launch_residual_seg(const DevProblem &p, const T *lam, const T *mm, double omega, const int64_t *chunk_begin,
                         int64_t n_chunks, const int64_t *seg, int64_t n_inst, double *part_pos, double *part_max,
                         double *pos, double *mx, double *share, hipStream_t st);

// x_i = [M_i. < 0] for variables in some subproblem (0 elsewhere)
template <typename T>
void launch_decode(const DevProblem &p, const T *mm, uint8_t *x, hipStream_t st);

// Original rows on the device, for the final exact check of a primal point.
struct DevRows {
    const int64_t *row_ptr;   // [n_rows + 1]
    const int32_t *col;       // [nnz]
    const int32_t *coef;      // [nnz] nonzero coefficients
    const int8_t *sense;      // [n_rows]
    const int64_t *rhs;       // [n_rows]
    int64_t n_rows;
    const int8_t *preset;     // [n_vars] presolved value (0/1) or -1 when decoded
    const int32_t *row_inst;  // [n_rows] instance of every row (batches), else nullptr
};

// full point: xfull[i] = preset[i] >= 0 ? preset[i] : xdec[i]
void launch_finalize_x(const DevRows &r, int64_t n_vars, const uint8_t *xdec, uint8_t *xfull, hipStream_t st);

// counter[k] = number of original rows of instance k xfull violates (int64
// arithmetic; counter[0..n_inst) is cleared first)
void launch_row_check(const DevRows &r, const uint8_t *xfull, int32_t *counter, int64_t n_inst, hipStream_t st);


// walk the BDDs of the instances k with only[k] != 0 (every BDD if only is
// null) with the 0-1 point x (x[n_vars] must be 0): counter[k] += number of
// BDDs of instance k that reject it, flag[i] = 1 for every variable of those
// BDDs (counter[0..n_inst) is cleared first)
void launch_check(const DevProblem &p, const uint8_t *x, uint8_t *flag, int32_t *counter, const uint8_t *only,
                  int64_t n_inst, hipStream_t st);

template <typename T>
void launch_fill(T *dst, T value, int64_t n, hipStream_t st);

// tables derived on the device at bind instead of uploaded: the variable of
// every pair slot (n_vars for padding slots) from the variable -> slot lists,
// and the instance of every variable from the instances' first variables
void launch_pair_var(const int32_t *vptr, const int32_t *vslot, int64_t n_vars, int64_t n_slots, int32_t *pair_var,
                     hipStream_t st);
void launch_var_inst(const int64_t *inst_var, int64_t n_inst, int64_t n_vars, int32_t *var_inst, hipStream_t st);

template <typename T>
void launch_copy(T *dst, const T *src, int64_t n, hipStream_t st);

}  // namespace bddmma
