// Host side of the solver: ILP validation, presolve, BDD compilation and the
// packing of BDDs into 64-lane tiles (see layout.hpp for the device layout).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "layout.hpp"

namespace bddmma {

struct Ilp {
    int64_t n_vars = 0, n_rows = 0;
    std::vector<double> cost;
    std::vector<int64_t> row_ptr;   // rows with columns sorted ascending, zero coefficients removed
    std::vector<int32_t> col;
    std::vector<int64_t> coef;
    std::vector<int8_t> sense;
    std::vector<int64_t> rhs;
    // independent instances of a batch: instance k owns variables
    // [inst_var[k], inst_var[k+1]) and rows [inst_row[k], inst_row[k+1]); a
    // single ILP is one instance
    std::vector<int64_t> inst_var, inst_row;
    int64_t n_inst() const { return (int64_t)inst_var.size() - 1; }
};

// Flat store of compiled BDDs, in ascending original row order.
struct BddSet {
    std::vector<int32_t> row;        // [B] original row id
    std::vector<int64_t> lay_off;    // [B+1] into lay_var / lay_width
    std::vector<int32_t> lay_var;    // [P] variable of each layer
    std::vector<int32_t> lay_width;  // [P] nodes of each layer
    std::vector<int64_t> node_off;   // [B+1] into child
    std::vector<uint32_t> child;     // [N] lo | hi << 16 (next-layer index or kTop / kBot)
    int64_t n_bdds() const { return (int64_t)row.size(); }
};

struct Packed {
    std::vector<TileDesc> tiles;
    std::vector<int32_t> lists;                  // tile ids of every TileList, concatenated
    std::vector<int64_t> list_off;               // [kNumLists + 1]
    std::vector<uint32_t> layers;     // layer table
    std::vector<uint32_t> child;      // node words
    std::vector<int32_t> pair_var;    // [S] variable per slot, n_vars for padding
    std::vector<int64_t> slot_of_pair;  // [P] canonical pair -> slot
    std::vector<int32_t> vptr;        // [V+1] variable -> its slots, ascending row order
    std::vector<int32_t> vslot;       // [P]
    std::vector<uint16_t> code;       // averaging codes (layout.hpp), one K*64 block per distinct tile pattern
    std::vector<int32_t> gvars;       // variables averaged by the averaging kernel, ascending
    std::vector<AvgBucket> gbuckets;  // the same variables bucketed by |J_i| (layout.hpp)
    std::vector<int32_t> gslot;       // bucket slot lists (ELL) / variable ids (CSR bucket)
    int64_t gblocks = 0;              // averaging blocks covering all buckets
    std::vector<uint32_t> gmeta;      // [S] fused averaging (layout.hpp); empty when the averaging kernel runs
    std::vector<int32_t> gsrc;        // slot of every entry of the per-variable copies
    int64_t n_slots = 0;
    int64_t scratch_elems = 0;        // device scratch elements for non-LDS tiles
    int max_lds_lane_elems = 0;       // per-lane LDS elements of the largest LDS tile
    int max_wide_elems = 0;           // LDS elements (2 * nodes + 2 * K) of the largest wide tile
    int max_layers = 0, max_width = 0;
    // batches: tiles are instance-pure and instance k owns tiles
    // [inst_tile[k], inst_tile[k+1]); the id arrays are filled for batches only
    std::vector<int64_t> inst_tile;
    std::vector<int32_t> tile_inst, var_inst, row_inst;
};

struct Problem {
    Ilp ilp;
    std::vector<int8_t> fixed;   // -1 free, else the presolved value
    std::vector<int32_t> deg;    // |J_i| over kept rows
    BddSet bdds;
    std::vector<int32_t> pair_var, pair_row;   // canonical pair order
    double lb_offset = 0.0;
    std::vector<double> inst_offset;   // lb_offset per instance
    int64_t n_nodes = 0, n_fixed = 0, n_free = 0;
};

// status codes mirror the C ABI
enum Status { ST_OK = 0, ST_INVALID = -1, ST_INFEASIBLE = -2, ST_NOMEM = -3 };

// Validate and normalise the CSR input.  Returns ST_OK or ST_INVALID (msg set).
int ingest_ilp(Ilp &out, int64_t n_vars, const double *costs, int64_t n_rows, const int64_t *row_ptr,
               const int32_t *col, const int32_t *coef, const int8_t *sense, const int64_t *rhs,
               std::string &msg);

// Instance boundaries of a batch (n_inst counts of variables and rows, in
// order); every row must reference variables of its own instance only.
int set_instances(Ilp &ilp, int64_t n_inst, const int64_t *inst_vars, const int64_t *inst_rows, std::string &msg);

// Presolve + compile every remaining row.  ST_OK / ST_INFEASIBLE / ST_INVALID.
int build_problem(Problem &p, std::string &msg);

// Host threads of ingestion, presolve, compilation and packing: at most n
// (clamped to 1..16, default 16), process-wide.  Results do not depend on it.
void set_host_thread_cap(int n);

// Pack the compiled BDDs into tiles.  lds_elem_budget: per-lane elements a tile
// may keep in LDS (0 disables LDS); lds_max_nodes > 0 additionally caps the
// nodes per lane of LDS tiles; fast selects the register-resident path for the
// tiles it can take; merge_bytes is the padding traffic per sweep a layer
// class may add to join a larger class (0: no merging); problems of at most
// small_tiles tiles sweep their width-2 tiles of one topology as mixed tiles
// (one launch per layer class); tiles outside the register classes with a
// layer of >= wide_min_width nodes (> 0) whose per-BDD LDS need fits in
// wide_lds_elems elements use the wide kernel (a group of lanes per BDD).
// ST_OK / ST_INVALID.
// fast also enables the in-tile averaging of variables with |J_i| <= 2.
int pack_problem(const Problem &p, int lds_elem_budget, int lds_max_nodes, bool fast, double merge_bytes,
                 int64_t small_tiles, int wide_lds_elems, int wide_min_width, int fuse_elem, Packed &out,
                 std::string &msg);

// Batch of independent instances assembled from their own single-instance
// results: the union problem is block-diagonal and every instance keeps the
// tiles, classes and averaging codes it has when solved alone (tile, slot,
// node, layer, code and scratch offsets are shifted; averaging buckets of equal
// degree are merged).  Instance k's slots form the range
// [slot_off[k], slot_off[k] + parts[k].pk->n_slots).  ST_OK / ST_INVALID.
struct Part {
    const Problem *p;
    const Packed *pk;
};
int merge_instances(const std::vector<Part> &parts, Problem &out, Packed &opk, std::vector<int64_t> &slot_off,
                    std::string &msg);

// ---- the same batch assembled on the device -----------------------------------
// Tables a solver uploads for its problem, in the order of the layout.
enum TableId {
    TB_PAIR_VAR, TB_VPTR, TB_VSLOT, TB_CODE, TB_GSLOT, TB_CHILD, TB_LAYERS, TB_COST,
    TB_RPTR, TB_RCOL, TB_RCOEF, TB_RSENSE, TB_RRHS, TB_PRESET, TB_VAR_INST, TB_ROW_INST, kNumTables
};
struct TableSet {
    uint64_t off[kNumTables];   // byte offsets from the base
    uint64_t bytes;             // total (images) / end of the last table
};

// Image of one instance's tables (what bind uploads for it alone; presolved
// values as the check kernel reads them, coefficients as int32), 256-byte
// aligned tables; no instance ids.
TableSet image_layout(const Problem &p, const Packed &pk);
void write_image(const Problem &p, const Packed &pk, const TableSet &ts, uint8_t *buf);

// Sizes of the big tables of a merged batch.
struct MergedSizes {
    int64_t pairs = 0, code = 0, gslot = 0, child = 0, layers = 0, nnz = 0;
};

// merge_instances without the big tables: tiles, lists, buckets, instance
// ranges and scalars exactly as merge_instances fills them; the tables listed
// in TableId (and the host-only pair maps) are left empty, their sizes in sz.
int merge_small(const std::vector<Part> &parts, Problem &out, Packed &opk, std::vector<int64_t> &slot_off,
                MergedSizes &sz, std::string &msg);

// Copy steps that write every TableId table of the merged batch (byte offsets
// dst.off from dst_base) from the instance images at img[k] (laid out by
// image_layout), giving exactly the tables merge_instances builds.
struct Seg;
void assembly_segments(const std::vector<Part> &parts, const std::vector<uint64_t> &img, uint64_t dst_base,
                       const TableSet &dst, std::vector<Seg> &out);

// ---- serial min-marginal averaging (ablation) ---------------------------------
// Tables of the variable-by-variable scheme: the compiled BDDs in their own
// order (not tiled), and a level schedule.  A variable's forward level is
// one more than the largest forward level of its predecessors in the BDDs
// that contain it (0 without predecessors); backward levels mirror this with
// successors.  Variables of one level share no BDD, so a level is one
// parallel step, and visiting levels in order visits every BDD's layers in
// order, as the sequential scheme does.
struct SerialTables {
    std::vector<uint32_t> child;     // [N] node words (next-layer index | index << 16, or kTop / kBot)
    std::vector<int32_t> pinfo;      // [4P] per pair: first node of its layer, layer width,
                                     //      first node of the next layer (-1: last layer), BDD
    std::vector<int32_t> bpair;      // [B+1] pair range of each BDD
    std::vector<int32_t> vptr, vpair;            // variable -> its pairs, ascending row order
    std::vector<int32_t> lf_ptr, lf_var;         // forward levels (CSR)
    std::vector<int32_t> lb_ptr, lb_var;         // backward levels (CSR)
    std::vector<int32_t> slot;       // [P] slot of each pair in the tile layout
};
int build_serial(const Problem &p, const Packed &pk, SerialTables &out, std::string &msg);

// ---- encoding of rows whose BDDs would be too wide --------------------------------
// A row  sum a_i x_i (sense) b  whose partial sums can take more than
// max_states values (min(2^k, sum |a_i| + 1) over its k nonzero terms) is
// replaced by a binary adder network over auxiliary variables appended after
// the original ones:
//  - a negative coefficient uses the complement xb_i of x_i (row x_i + xb_i = 1,
//    one complement per variable), so all weights w_i are positive and the
//    right-hand side becomes B = b + sum_{a_i < 0} |a_i|;
//  - column k adds the inputs whose weight has bit k set and the carry of
//    column k - 1 (its bits c_{k-1,j} with weights 2^j) into a sum bit s_k and
//    a carry C_k = (sum bits) div 2 written in binary:
//        sum inputs + sum_j 2^j c_{k-1,j} - s_k - sum_j 2^(j+1) c_{k,j} = 0,
//    with as many columns as the total weight needs;
//  - one row  sum_k 2^k s_k (sense) B  compares the sum with B; its most
//    significant bit gets the smallest variable id, so this BDD stays narrow.
// Every auxiliary value is determined by x, so the encoded rows admit exactly
// the points of the original row (extended by those values).  Auxiliary
// variables cost 0.  Rows within the limit are copied unchanged.  The weight
// sum of an encoded row must stay below 2^30 (ST_INVALID otherwise).
int encode_wide_rows(const Ilp &in, int64_t max_states, Ilp &out, int64_t &n_encoded, std::string &msg);

// Compile one row  sum a_h x_h (sense) b  over ascending variables into a
// reduced BDD appended to `out`.  Returns ST_OK, ST_INFEASIBLE or ST_INVALID.
int compile_row(const int32_t *var, const int64_t *a, int k, int sense, int64_t b, BddSet &out,
                std::string &msg);

}  // namespace bddmma
