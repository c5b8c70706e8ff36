// Device data layout shared by the host packer and the HIP kernels.
//
// Subproblem BDDs (Sec. 5, Def. "BDD") are grouped into tiles of 64 whole
// BDDs, one BDD per lane of a 64-wide wavefront.  Inside a tile everything is
// layer-major and lane-minor, so the 64 lanes of a wave touch 64 consecutive
// elements whenever they read or write the pair arrays:
//
//   pair slot (tile t, layer h, lane l) = tiles[t].pair_base + h * 64 + l
//
// Node structure: nodes of one layer are numbered 0..W_h-1 (W_h = tile-wide
// layer width).  A node's two successors (Sec. 5: s^0(v), s^1(v)) are stored as
// one 32-bit word, lo | hi << 16, each an index into the next layer or one of
// the terminal codes.  Tiles whose 64 BDDs share one topology store the words
// once (flag TILE_SHARED); other tiles store one word per (node, lane) at
// node_base + node * 64 + lane, node = layer offset + index.  BDDs shorter than
// the tile are padded with chain layers whose multiplier stays exactly 0, and
// partially filled tiles with such chains in every lane; both are neutral for
// every min-marginal, multiplier and energy.
#pragma once
#include <stdint.h>

namespace bddmma {

constexpr int kLanes = 64;
constexpr uint32_t kBot = 0xFFFFu;   // arc into the rejecting terminal
constexpr uint32_t kTop = 0xFFFEu;   // arc into the accepting terminal
constexpr int kMaxWidth = 65533;     // largest layer width encodable in 16 bits

constexpr uint16_t TILE_SHARED = 1;  // all lanes use the same node words
constexpr uint16_t TILE_GATHER = 2;  // some slot's variable is averaged inside the sweep from
                                     // the per-variable copy of the previous differences

struct TileDesc {
    uint32_t pair_base;     // first pair slot of the tile
    uint32_t node_base;     // first node word of the tile
    uint32_t layer_base;    // first entry of the tile's layer table
    uint32_t scratch_base;  // per-tile device scratch (shortest paths kept outside LDS)
    uint16_t K;             // layers (padded length)
    uint16_t nodes;         // nodes per lane = sum of the layer widths
    uint16_t flags;
    uint16_t pad0;
    uint32_t code_base;     // first averaging code of the tile (tiles with equal codes share them)
    uint32_t fast_base;     // fast-path tiles: first word of the register kernel's copy of the node words
};
static_assert(sizeof(TileDesc) == 32, "TileDesc is 32 bytes");

// layer table entry: node offset of the layer (low 16 bits) | width << 16
inline uint32_t layer_entry(uint32_t noff, uint32_t width) { return noff | (width << 16); }

// per-lane scratch elements a tile needs (lambda, averaged term, two distance arrays)
inline uint32_t lane_elems(uint32_t K, uint32_t nodes) { return 2u * K + 2u * nodes; }

// Register-resident fast path: shared tiles (one topology) with at most
// kKClass[last] layers and layers at most kWClass[last] wide use a fixed layer
// stride (node (h, q) at h * W + q, unused nodes have both arcs into the
// rejecting terminal) and are swept by kernels unrolled for a compile-time
// layer count KMAX and width W: a fast tile has exactly kKClass[ki] layers
// (shorter BDDs are padded with neutral chain layers, as in mixed tiles), so
// the kernels run without per-layer guards.  Their register kernel reads a second copy of
// the node words at fast_base in which the last layer's arcs into the
// accepting terminal point at node 0 of a virtual layer K (the terminal
// layer: node 0 = accept at distance 0), so every layer is handled alike.
constexpr int kNumKClasses = 20;
constexpr int kKClass[kNumKClasses] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 20, 24, 28, 32};
constexpr int kNumWClasses = 2;
constexpr int kWClass[kNumWClasses] = {2, 4};
// width-4 tiles deeper than 16 layers would need more than 170 VGPRs per lane
// (one wave per SIMD); they stay on the general kernels
constexpr bool fast_class_ok(int wi, int ki) { return kWClass[wi] * kKClass[ki] <= 64; }
// Mixed tiles (lanes of different topologies) of width <= 2 and at most 32
// layers run on the register kernel too, with per-lane node words in VGPRs
// (same fixed stride and layer classes, words at fast_base + node * 64 + lane).
constexpr bool mix_class_ok(int ki) { return kKClass[ki] <= 32; }

// Tile lists.  Every tile is in exactly one of the two *_ALL lists (shortest
// paths in LDS or in device scratch for the general kernels); tiles outside the
// fast path are also in the matching *_REST list; fast tiles are in the list of
// their (width class, layer class), mixed fast tiles (width 2) in that of their
// layer class.
enum TileList {
    LIST_GEN_LDS_ALL = 0,
    LIST_GEN_GLOB_ALL = 1,
    LIST_GEN_LDS_REST = 2,
    LIST_GEN_GLOB_REST = 3,
    LIST_FAST0 = 4,
    LIST_MIX0 = LIST_FAST0 + kNumKClasses * kNumWClasses,
    LIST_LONG_SH = LIST_MIX0 + kNumKClasses,   // width-2 tiles longer than every class, one topology
    LIST_LONG_MIX = LIST_LONG_SH + 1,          // the same, per-lane topologies
    LIST_WIDE = LIST_LONG_MIX + 1,             // wide tiles: a group of lanes per BDD, over its nodes
    kNumLists = LIST_WIDE + 1
};

// Wide tiles (a layer of at least wide_min_width nodes, kWideMinWidth by
// default) are swept by a group of 16, 32 or 64 lanes per BDD, spread over a
// layer's nodes; the BDD's distances to root and to top, multipliers and
// averaged terms (2 * nodes + 2 * K elements) and its node words sit in LDS.
// Mixed wide tiles carry a BDD-major copy of their node words at fast_base
// (lane l's node n at fast_base + l * nodes + n).
constexpr int kWideMinWidth = 4;
inline int fast_list(int wi, int ki) { return LIST_FAST0 + wi * kNumKClasses + ki; }
inline int mix_list(int ki) { return LIST_MIX0 + ki; }

// Long tiles (width <= 2, more layers than the largest class) run a
// chunked register kernel that keeps per-layer values in the tile's device
// scratch: 2 distances per layer at [(2h + q) * 64 + lane] and the averaged
// term at [(2K + h) * 64 + lane] (3K elements per lane, within lane_elems).

// Where a pair slot takes the averaged term a_i = omega/|J_i| * sum_k M_ik of
// its variable from (Alg. 1 deferred update).  Variables with |J_i| <= 2 whose
// pairs all lie in one tile are averaged inside the sweep from the tile's own
// previous min-marginal differences: code = offset (h * 64 + lane) of the
// partner slot in the tile, or kCodeSelf when |J_i| = 1 (padding slots too).
// All other variables are averaged by the averaging kernel, which stores the
// term per slot (kCodeGlobal).
constexpr uint16_t kCodeSelf = 0xFFFEu;
constexpr uint16_t kCodeGlobal = 0xFFFFu;

// Fused averaging of the variables with code kCodeGlobal (used when all of
// them lie in mixed register tiles, at most kGatherMaxDeg subproblems each, so
// that a slot reads at most kGatherOthers entries besides its own in one trip):
// instead of the averaging kernel, each sweep reads the previous sweep's
// differences of all slots of such a variable from a variable-major array
// (entries base .. base+|J_i|-1 in ascending row order) and writes its own
// difference into the other of two such arrays (forward sweeps read the
// first and write the second, backward sweeps the reverse).  Per slot of such
// a variable: gmeta = entry | rank << 24 | (|J_i| - 1) << 28, entry = base +
// rank, so one 32-bit word locates the whole block.
constexpr int kGatherOthers = 4;
constexpr int kGatherMaxDeg = kGatherOthers + 1;
// layer classes whose mixed tiles may use it: all in FP32; up to 24 layers in
// FP64, where the extra registers of the deeper classes would spill
constexpr bool fuse_class_ok(int elem, int layers) { return elem == 4 || layers <= 24; }
constexpr int64_t kGatherMaxEntries = int64_t(1) << 24;
inline uint32_t gather_meta(uint32_t entry, uint32_t rank, uint32_t deg)
{
    return entry | (rank << 24) | ((deg - 1u) << 28);
}

// Variables averaged by the averaging kernel are bucketed by |J_i|.  Buckets
// with deg <= kEllMaxDeg store the slots column-major (slot k of the bucket's
// variable i at base + k * count + i) so a thread reads its slots coalesced
// in one round; the last bucket (deg = 0) lists variables with more
// subproblems by id and uses the variable CSR.
constexpr int kEllMaxDeg = 16;
struct AvgBucket {
    int32_t deg;            // |J_i| of the bucket, 0 = CSR bucket
    int32_t count;          // variables in the bucket
    int32_t block_begin;    // first averaging block of the bucket
    int32_t pad;
    int64_t base;           // first entry in the bucket slot / id array
};
static_assert(sizeof(AvgBucket) == 24, "AvgBucket is 24 bytes");

// all buckets of a problem (at most one per degree up to kEllMaxDeg, plus the
// CSR bucket), small enough to travel as a kernel argument
struct AvgBucketSet {
    AvgBucket b[kEllMaxDeg + 1];
    int32_t n;
};

}  // namespace bddmma
