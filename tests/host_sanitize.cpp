// Host-side driver for a sanitizer build (AddressSanitizer + UBSan) of the
// solver's host code: ingestion, instance boundaries, presolve, BDD
// compilation and tile packing, on generated ILPs (random rows around a
// hidden point, wide knapsack rows, long rows, empty rows, batches) under
// every packing option, and batches assembled from instances packed alone
// (on the host, and through the device assembly's copy segments).
// Exits non-zero on the first inconsistency; the
// sanitizers abort on memory or undefined-behaviour errors.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "assemble.hpp"
#include "problem.hpp"

using namespace bddmma;

namespace {

struct Rng {   // SplitMix64 (Steele, Lea & Flood 2014)
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int64_t range(int64_t a, int64_t b) { return a + (int64_t)(next() % (uint64_t)(b - a + 1)); }
};

struct Csr {
    int64_t n_vars = 0;
    std::vector<double> cost;
    std::vector<int64_t> row_ptr{0};
    std::vector<int32_t> col, coef;
    std::vector<int8_t> sense;
    std::vector<int64_t> rhs;
    void row(const std::vector<int32_t> &c, const std::vector<int32_t> &a, int s, int64_t b)
    {
        col.insert(col.end(), c.begin(), c.end());
        coef.insert(coef.end(), a.begin(), a.end());
        row_ptr.push_back((int64_t)col.size());
        sense.push_back((int8_t)s);
        rhs.push_back(b);
    }
    int64_t n_rows() const { return (int64_t)sense.size(); }
};

// rows around a hidden 0/1 point (always feasible), some of them long or wide
Csr random_ilp(Rng &g, int64_t n, int64_t rows, int max_len, int max_coef)
{
    Csr c;
    c.n_vars = n;
    std::vector<int> x(n);
    for (auto &v : x) v = (int)g.range(0, 1);
    for (int64_t i = 0; i < n; ++i) c.cost.push_back((double)g.range(-40, 40) / 8.0);
    for (int64_t r = 0; r < rows; ++r) {
        const int k = (int)g.range(1, std::min<int64_t>(max_len, n));
        std::vector<int32_t> vs, a;
        std::vector<char> used(n, 0);
        while ((int)vs.size() < k) {
            const int32_t v = (int32_t)g.range(0, n - 1);
            if (used[v]) continue;
            used[v] = 1;
            vs.push_back(v);
            a.push_back((int32_t)(g.range(1, max_coef) * (g.range(0, 1) ? 1 : -1)));
        }
        int64_t lhs = 0;
        for (int q = 0; q < k; ++q) lhs += (int64_t)a[q] * x[vs[q]];
        const int s = (int)g.range(-1, 1);
        const int64_t slack = g.range(0, 2);
        c.row(vs, a, s, lhs + (s < 0 ? slack : s > 0 ? -slack : 0));
    }
    return c;
}

// <= rows of 2..6 variables with coefficients in [-3, 3] and slack 3..5 at a
// hidden point: flipping one variable moves a row by at most 3, so no row
// forces a variable and presolve keeps every row
Csr loose_ilp(Rng &g, int64_t n, int64_t rows)
{
    Csr c;
    c.n_vars = n;
    std::vector<int> x(n);
    for (auto &v : x) v = (int)g.range(0, 1);
    for (int64_t i = 0; i < n; ++i) c.cost.push_back((double)g.range(-40, 40) / 8.0);
    for (int64_t r = 0; r < rows; ++r) {
        const int k = (int)g.range(2, 6);
        std::vector<int32_t> vs, a;
        while ((int)vs.size() < k) {
            const int32_t v = (int32_t)g.range(0, n - 1);
            bool dup = false;
            for (int32_t u : vs) dup |= u == v;
            if (dup) continue;
            vs.push_back(v);
            a.push_back((int32_t)(g.range(1, 3) * (g.range(0, 1) ? 1 : -1)));
        }
        int64_t lhs = 0;
        for (int q = 0; q < k; ++q) lhs += (int64_t)a[q] * x[vs[q]];
        c.row(vs, a, -1, lhs + g.range(3, 5));
    }
    return c;
}

int fails = 0;

void check(bool ok, const char *what, int64_t seed)
{
    if (!ok) {
        std::fprintf(stderr, "FAIL %s (seed %lld)\n", what, (long long)seed);
        ++fails;
    }
}

void run(const Csr &c, const std::vector<int64_t> &iv, const std::vector<int64_t> &ir, int64_t seed)
{
    for (int variant = 0; variant < 5; ++variant) {
        Problem p;
        std::string msg;
        int rc = ingest_ilp(p.ilp, c.n_vars, c.cost.data(), c.n_rows(), c.row_ptr.data(), c.col.data(),
                            c.coef.data(), c.sense.data(), c.rhs.data(), msg);
        check(rc == ST_OK, "ingest", seed);
        if (rc != ST_OK) return;
        if (!iv.empty()) {
            rc = set_instances(p.ilp, (int64_t)iv.size(), iv.data(), ir.data(), msg);
            check(rc == ST_OK, "instances", seed);
            if (rc != ST_OK) return;
        }
        rc = build_problem(p, msg);
        check(rc == ST_OK, "build (rows are feasible by construction)", seed);
        if (rc != ST_OK) return;
        Packed pk;
        const bool fast = variant != 4;
        const int lds = variant == 3 ? 0 : 128;
        const double merge = variant == 1 ? 0.0 : 32.0 * (1 << 20);
        const int64_t small = variant == 2 ? 0 : 2048;
        rc = pack_problem(p, lds, 0, fast, merge, small, variant == 0 ? 0 : 16384, variant == 2 ? 3 : 16, variant == 1 ? 0 : 4 << (variant & 1),
                          pk, msg);
        check(rc == ST_OK, "pack", seed);
        if (rc != ST_OK) {
            std::fprintf(stderr, "  %s\n", msg.c_str());
            return;
        }
        // every pair has exactly one slot, slots carry their pair's variable
        const int64_t P = (int64_t)p.pair_var.size();
        check((int64_t)pk.slot_of_pair.size() == P, "slot map size", seed);
        std::vector<char> seen(pk.n_slots, 0);
        for (int64_t q = 0; q < P; ++q) {
            const int64_t s = pk.slot_of_pair[q];
            const bool in = s >= 0 && s < pk.n_slots;
            check(in, "slot in range", seed);
            if (!in) continue;
            check(!seen[s], "slot used once", seed);
            seen[s] = 1;
            check(pk.pair_var[s] == p.pair_var[q], "slot variable", seed);
        }
        check((int64_t)pk.inst_tile.size() == p.ilp.n_inst() + 1, "instance tile ranges", seed);
        // fused averaging: every kernel-averaged variable owns a contiguous
        // block of entries in ascending row order, each entry's slot points
        // back at it, and the slot's tile is flagged
        if (!pk.gmeta.empty()) {
            check((int64_t)pk.gmeta.size() == pk.n_slots, "gather meta size", seed);
            int64_t e = 0;
            for (int32_t v : pk.gvars) {
                const int32_t a = pk.vptr[v], deg = pk.vptr[v + 1] - a;
                check(deg >= 1 && deg <= kGatherMaxDeg, "gather degree", seed);
                for (int32_t r = 0; r < deg; ++r) {
                    const int32_t sl = pk.vslot[a + r];
                    check(e + r < (int64_t)pk.gsrc.size() && pk.gsrc[(size_t)(e + r)] == sl, "gather source", seed);
                    check(pk.gmeta[(size_t)sl] == gather_meta((uint32_t)(e + r), (uint32_t)r, (uint32_t)deg),
                          "gather meta", seed);
                    bool flagged = false, class_ok = false;
                    for (const TileDesc &d : pk.tiles)
                        if (sl >= (int64_t)d.pair_base && sl < (int64_t)d.pair_base + (int64_t)d.K * kLanes) {
                            flagged = (d.flags & TILE_GATHER) != 0;
                            class_ok = fuse_class_ok(4 << (variant & 1), d.K);
                        }
                    check(flagged, "gather tile flag", seed);
                    check(class_ok, "gather tile class", seed);
                }
                e += deg;
            }
            check(e == (int64_t)pk.gsrc.size(), "gather entries", seed);
        }
    }
}

template <class T>
bool same_vec(const std::vector<T> &a, const std::vector<T> &b)
{
    return a.size() == b.size() && (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(T)) == 0);
}

// ingestion, presolve, compilation and packing give the same tables on one
// host thread and on several (every threaded phase is reached: more than
// 16,384 BDDs for the parallel sort, more than 4,096 variables, rows and tiles)
void run_threads(const Csr &c, int64_t seed)
{
    Problem p[2];
    Packed pk[2];
    for (int k = 0; k < 2; ++k) {
        set_host_thread_cap(k == 0 ? 1 : 8);
        std::string msg;
        int rc = ingest_ilp(p[k].ilp, c.n_vars, c.cost.data(), c.n_rows(), c.row_ptr.data(), c.col.data(),
                            c.coef.data(), c.sense.data(), c.rhs.data(), msg);
        if (rc == ST_OK) rc = build_problem(p[k], msg);
        if (rc == ST_OK) rc = pack_problem(p[k], 128, 0, true, 32.0 * (1 << 20), 2048, 16384, 16, 4, pk[k], msg);
        check(rc == ST_OK, "threads: construction", seed);
        if (rc != ST_OK) {
            std::fprintf(stderr, "  %s\n", msg.c_str());
            set_host_thread_cap(16);
            return;
        }
    }
    set_host_thread_cap(16);
    const Ilp &a = p[0].ilp, &b = p[1].ilp;
    check(same_vec(a.row_ptr, b.row_ptr) && same_vec(a.col, b.col) && same_vec(a.coef, b.coef), "threads: ingest",
          seed);
    const BddSet &x = p[0].bdds, &y = p[1].bdds;
    check(same_vec(x.row, y.row) && same_vec(x.lay_off, y.lay_off) && same_vec(x.lay_var, y.lay_var) &&
              same_vec(x.lay_width, y.lay_width) && same_vec(x.node_off, y.node_off) && same_vec(x.child, y.child),
          "threads: BDDs", seed);
    check(same_vec(p[0].fixed, p[1].fixed) && same_vec(p[0].deg, p[1].deg) && same_vec(p[0].pair_var, p[1].pair_var) &&
              same_vec(p[0].pair_row, p[1].pair_row),
          "threads: pairs", seed);
    const Packed &u = pk[0], &v = pk[1];
    check(u.tiles.size() == v.tiles.size() &&
              (u.tiles.empty() || std::memcmp(u.tiles.data(), v.tiles.data(), u.tiles.size() * sizeof(TileDesc)) == 0),
          "threads: tiles", seed);
    check(same_vec(u.lists, v.lists) && same_vec(u.list_off, v.list_off) && same_vec(u.layers, v.layers) &&
              same_vec(u.child, v.child),
          "threads: lists, layers, node words", seed);
    check(same_vec(u.pair_var, v.pair_var) && same_vec(u.slot_of_pair, v.slot_of_pair) && same_vec(u.vptr, v.vptr) &&
              same_vec(u.vslot, v.vslot),
          "threads: slots", seed);
    check(same_vec(u.code, v.code) && same_vec(u.gvars, v.gvars) && same_vec(u.gslot, v.gslot) &&
              u.gbuckets.size() == v.gbuckets.size() &&
              (u.gbuckets.empty() ||
               std::memcmp(u.gbuckets.data(), v.gbuckets.data(), u.gbuckets.size() * sizeof(AvgBucket)) == 0) &&
              u.gblocks == v.gblocks && u.n_slots == v.n_slots,
          "threads: averaging tables", seed);
    check(x.n_bdds() > 16384 && p[0].ilp.n_vars > 4096 && (int64_t)u.tiles.size() > 4096 / 64,
          "threads: the case reaches every threaded phase", seed);
}

// host model of the device copy kernel (same semantics per segment)
void apply_segments(const std::vector<Seg> &segs)
{
    for (const Seg &g : segs)
        for (int64_t i = 0; i < g.n; ++i) switch (g.elem) {
            case 1:
                reinterpret_cast<uint8_t *>(g.dst)[i] =
                    g.op == SEG_FILL ? (uint8_t)g.a : reinterpret_cast<const uint8_t *>(g.src)[i];
                break;
            case 2:
                reinterpret_cast<uint16_t *>(g.dst)[i] =
                    g.op == SEG_FILL ? (uint16_t)g.a : reinterpret_cast<const uint16_t *>(g.src)[i];
                break;
            case 4: {
                int32_t v = g.op == SEG_FILL ? (int32_t)g.a : reinterpret_cast<const int32_t *>(g.src)[i];
                if (g.op == SEG_ADD) v += (int32_t)g.a;
                else if (g.op == SEG_PADVAR) v = v == (int32_t)g.b ? (int32_t)g.c : v + (int32_t)g.a;
                reinterpret_cast<int32_t *>(g.dst)[i] = v;
                break;
            }
            case 8: {
                int64_t v = g.op == SEG_FILL ? g.a : reinterpret_cast<const int64_t *>(g.src)[i];
                if (g.op == SEG_ADD) v += g.a;
                reinterpret_cast<int64_t *>(g.dst)[i] = v;
                break;
            }
            default: break;
            }
}

// The device assembly path: small tables from merge_small, big tables from
// the instances' images through the copy segments; both must equal what
// merge_instances builds on the host (the big tables are compared in a
// buffer poisoned beforehand, so every element must have been written).
void check_assembly(const std::vector<Part> &parts, const Problem &u, const Packed &o,
                    const std::vector<int64_t> &soff, int64_t seed)
{
    Problem us;
    Packed os;
    std::vector<int64_t> so;
    MergedSizes sz;
    std::string msg;
    int rc = merge_small(parts, us, os, so, sz, msg);
    check(rc == ST_OK, "assembly: merge_small", seed);
    if (rc != ST_OK) return;
    check(so == soff, "assembly: slot offsets", seed);
    auto eq = [](const void *a, const void *b, size_t n) { return n == 0 || std::memcmp(a, b, n) == 0; };
    check(os.tiles.size() == o.tiles.size() && eq(os.tiles.data(), o.tiles.data(), o.tiles.size() * sizeof(TileDesc)),
          "assembly: tiles", seed);
    check(os.lists == o.lists && os.list_off == o.list_off && os.inst_tile == o.inst_tile &&
              os.tile_inst == o.tile_inst && os.gblocks == o.gblocks && os.n_slots == o.n_slots &&
              os.scratch_elems == o.scratch_elems && os.max_lds_lane_elems == o.max_lds_lane_elems &&
              os.max_wide_elems == o.max_wide_elems,
          "assembly: small tables", seed);
    check(os.gbuckets.size() == o.gbuckets.size() &&
              eq(os.gbuckets.data(), o.gbuckets.data(), o.gbuckets.size() * sizeof(AvgBucket)),
          "assembly: buckets", seed);
    check(us.ilp.inst_var == u.ilp.inst_var && us.ilp.inst_row == u.ilp.inst_row &&
              us.inst_offset == u.inst_offset && us.lb_offset == u.lb_offset,
          "assembly: instance ranges", seed);
    check(sz.pairs == (int64_t)u.pair_var.size() && sz.code == (int64_t)o.code.size() &&
              sz.gslot == (int64_t)o.gslot.size() && sz.child == (int64_t)o.child.size() &&
              sz.layers == (int64_t)o.layers.size() && sz.nnz == (int64_t)u.ilp.col.size(),
          "assembly: sizes", seed);
    // images
    std::vector<std::vector<uint64_t>> img(parts.size());
    std::vector<uint64_t> base;
    for (size_t k = 0; k < parts.size(); ++k) {
        const TableSet ts = image_layout(*parts[k].p, *parts[k].pk);
        img[k].assign(ts.bytes / 8 + 1, 0);
        write_image(*parts[k].p, *parts[k].pk, ts, reinterpret_cast<uint8_t *>(img[k].data()));
        base.push_back((uint64_t)(uintptr_t)img[k].data());
    }
    // batch tables
    const int64_t V = u.ilp.n_vars, R = u.ilp.n_rows, nnz = (int64_t)u.ilp.col.size();
    const uint64_t bytes[kNumTables] = {(uint64_t)o.n_slots * 4, (uint64_t)(V + 1) * 4, u.pair_var.size() * 4,
                                        o.code.size() * 2, o.gslot.size() * 4, o.child.size() * 4,
                                        o.layers.size() * 4, (uint64_t)V * 8, (uint64_t)(R + 1) * 8,
                                        (uint64_t)nnz * 4, (uint64_t)nnz * 4, (uint64_t)R, (uint64_t)R * 8,
                                        (uint64_t)V, parts.size() > 1 ? (uint64_t)V * 4 : 0,
                                        parts.size() > 1 ? (uint64_t)R * 4 : 0};
    TableSet dst{};
    uint64_t at = 0;
    for (int t = 0; t < kNumTables; ++t) {
        dst.off[t] = at;
        at = (at + bytes[t] + 8 + 255) & ~uint64_t(255);
    }
    std::vector<uint64_t> buf(at / 8 + 1, 0xA5A5A5A5A5A5A5A5ull);
    uint8_t *b = reinterpret_cast<uint8_t *>(buf.data());
    std::vector<Seg> segs;
    assembly_segments(parts, base, (uint64_t)(uintptr_t)b, dst, segs);
    // every segment inside its table
    for (const Seg &g : segs) {
        bool in = false;
        for (int t = 0; t < kNumTables; ++t)
            in |= g.dst >= (uint64_t)(uintptr_t)(b + dst.off[t]) &&
                  g.dst + (uint64_t)g.n * g.elem <= (uint64_t)(uintptr_t)(b + dst.off[t]) + bytes[t];
        check(in, "assembly: segment inside one table", seed);
        if (!in) return;
    }
    apply_segments(segs);
    auto same = [&](int t, const void *ref, uint64_t n) {
        return n == bytes[t] && (n == 0 || std::memcmp(b + dst.off[t], ref, n) == 0);
    };
    std::vector<int32_t> coef32(u.ilp.coef.begin(), u.ilp.coef.end());
    std::vector<int8_t> pre((size_t)V);
    for (int64_t i = 0; i < V; ++i)
        pre[i] = u.fixed[i] >= 0 ? u.fixed[i] : u.deg[i] == 0 ? (int8_t)(u.ilp.cost[i] < 0.0 ? 1 : 0) : (int8_t)-1;
    check(same(TB_PAIR_VAR, o.pair_var.data(), o.pair_var.size() * 4), "assembly: pair_var", seed);
    check(same(TB_VPTR, o.vptr.data(), o.vptr.size() * 4), "assembly: vptr", seed);
    check(same(TB_VSLOT, o.vslot.data(), o.vslot.size() * 4), "assembly: vslot", seed);
    check(same(TB_CODE, o.code.data(), o.code.size() * 2), "assembly: code", seed);
    check(same(TB_GSLOT, o.gslot.data(), o.gslot.size() * 4), "assembly: gslot", seed);
    check(same(TB_CHILD, o.child.data(), o.child.size() * 4), "assembly: child", seed);
    check(same(TB_LAYERS, o.layers.data(), o.layers.size() * 4), "assembly: layers", seed);
    check(same(TB_COST, u.ilp.cost.data(), u.ilp.cost.size() * 8), "assembly: cost", seed);
    check(same(TB_RPTR, u.ilp.row_ptr.data(), u.ilp.row_ptr.size() * 8), "assembly: row_ptr", seed);
    check(same(TB_RCOL, u.ilp.col.data(), u.ilp.col.size() * 4), "assembly: col", seed);
    check(same(TB_RCOEF, coef32.data(), coef32.size() * 4), "assembly: coef", seed);
    check(same(TB_RSENSE, u.ilp.sense.data(), u.ilp.sense.size()), "assembly: sense", seed);
    check(same(TB_RRHS, u.ilp.rhs.data(), u.ilp.rhs.size() * 8), "assembly: rhs", seed);
    check(same(TB_PRESET, pre.data(), pre.size()), "assembly: preset", seed);
    if (parts.size() > 1) {
        check(same(TB_VAR_INST, o.var_inst.data(), o.var_inst.size() * 4), "assembly: var_inst", seed);
        check(same(TB_ROW_INST, o.row_inst.data(), o.row_inst.size() * 4), "assembly: row_inst", seed);
    }
}

// Batch assembled from instances packed alone (the serving pool's path):
// every instance keeps its tiles, slots and codes at shifted offsets, and the
// merged averaging buckets hold every kernel-averaged variable once with its
// slots in ascending row order.
void run_merge(const std::vector<Csr> &cs, int variant, int64_t seed)
{
    std::vector<Problem> ps(cs.size());
    std::vector<Packed> pks(cs.size());
    std::vector<Part> parts;
    std::string msg;
    for (size_t k = 0; k < cs.size(); ++k) {
        const Csr &c = cs[k];
        int rc = ingest_ilp(ps[k].ilp, c.n_vars, c.cost.data(), c.n_rows(), c.row_ptr.data(), c.col.data(),
                            c.coef.data(), c.sense.data(), c.rhs.data(), msg);
        if (rc == ST_OK) rc = build_problem(ps[k], msg);
        if (rc == ST_OK)
            rc = pack_problem(ps[k], variant == 3 ? 0 : 128, 0, variant != 4, variant == 1 ? 0.0 : 32.0 * (1 << 20),
                              variant == 2 ? 0 : 2048, variant == 0 ? 0 : 16384, variant == 2 ? 3 : 16, 8, pks[k],
                              msg);
        check(rc == ST_OK, "merge: instance alone", seed);
        if (rc != ST_OK) return;
        parts.push_back(Part{&ps[k], &pks[k]});
    }
    Problem u;
    Packed o;
    std::vector<int64_t> soff;
    int rc = merge_instances(parts, u, o, soff, msg);
    check(rc == ST_OK, "merge", seed);
    if (rc != ST_OK) {
        std::fprintf(stderr, "  %s\n", msg.c_str());
        return;
    }
    const int64_t V = u.ilp.n_vars;
    check(u.ilp.n_inst() == (int64_t)cs.size(), "merge: instance count", seed);
    int64_t voff = 0, poff = 0, toff = 0;
    for (size_t k = 0; k < cs.size(); ++k) {
        const Problem &p = ps[k];
        const Packed &pk = pks[k];
        check(u.ilp.inst_var[k] == voff, "merge: variable range", seed);
        for (size_t q = 0; q < p.pair_var.size(); ++q) {
            const int64_t s = o.slot_of_pair[poff + (int64_t)q];
            check(s == pk.slot_of_pair[q] + soff[k], "merge: slot of pair", seed);
            check(o.pair_var[s] == p.pair_var[q] + voff && u.pair_var[poff + q] == p.pair_var[q] + voff,
                  "merge: pair variable", seed);
        }
        for (int64_t sl = 0; sl < pk.n_slots; ++sl)
            if (pk.pair_var[sl] == (int32_t)p.ilp.n_vars)
                check(o.pair_var[soff[k] + sl] == (int32_t)V, "merge: padding slot", seed);
        for (size_t t = 0; t < pk.tiles.size(); ++t) {
            const TileDesc &a = pk.tiles[t], &b = o.tiles[toff + t];
            check(b.pair_base == a.pair_base + soff[k] && b.K == a.K && b.nodes == a.nodes && b.flags == a.flags,
                  "merge: tile", seed);
            for (uint32_t h = 0; h < a.K; ++h)
                check(o.layers[b.layer_base + h] == pk.layers[a.layer_base + h], "merge: layer table", seed);
            for (uint32_t q = 0; q < (uint32_t)a.K * kLanes; ++q)
                check(o.code[b.code_base + q] == pk.code[a.code_base + q], "merge: codes", seed);
            const uint32_t words = (uint32_t)a.nodes * ((a.flags & TILE_SHARED) ? 1u : (uint32_t)kLanes);
            for (uint32_t w = 0; w < words; ++w) {
                check(o.child[b.node_base + w] == pk.child[a.node_base + w], "merge: node words", seed);
                check(o.child[b.fast_base + w] == pk.child[a.fast_base + w], "merge: fast words", seed);
            }
            if (cs.size() > 1) check(o.tile_inst[toff + t] == (int32_t)k, "merge: tile instance", seed);
        }
        for (int l = 0; l < kNumLists; ++l) {
            int64_t n = 0;
            for (int64_t q = o.list_off[l]; q < o.list_off[l + 1]; ++q)
                n += o.lists[q] >= toff && o.lists[q] < toff + (int64_t)pk.tiles.size();
            check(n == pk.list_off[l + 1] - pk.list_off[l], "merge: list membership", seed);
        }
        check(o.inst_tile[k] == toff && o.inst_tile[k + 1] == toff + (int64_t)pk.tiles.size(),
              "merge: instance tiles", seed);
        voff += p.ilp.n_vars;
        poff += (int64_t)p.pair_var.size();
        toff += (int64_t)pk.tiles.size();
    }
    // buckets: every kernel-averaged variable exactly once, slots in row order
    std::vector<int> hits((size_t)V, 0);
    int32_t blocks = 0;
    for (const AvgBucket &b : o.gbuckets) {
        check(b.block_begin == blocks, "merge: bucket blocks", seed);
        blocks += (b.count + 255) / 256;
        for (int32_t i = 0; i < b.count; ++i) {
            int32_t v;
            if (b.deg == 0) {
                v = o.gslot[b.base + i];
            } else {
                v = o.pair_var[o.gslot[b.base + i]];
                check(o.vptr[v + 1] - o.vptr[v] == b.deg, "merge: bucket degree", seed);
                for (int k = 0; k < b.deg; ++k)
                    check(o.gslot[b.base + (int64_t)k * b.count + i] == o.vslot[o.vptr[v] + k], "merge: bucket slots",
                          seed);
            }
            if (v >= 0 && v < V) hits[v]++;
        }
    }
    check(blocks == o.gblocks, "merge: block count", seed);
    std::vector<int> want((size_t)V, 0);
    for (int32_t v : o.gvars) want[v] = 1;
    for (int64_t v = 0; v < V; ++v) check(hits[v] == want[v], "merge: averaged variables", seed);
    check_assembly(parts, u, o, soff, seed);
}

}  // namespace

int main()
{
    for (int64_t seed = 1; seed <= 40; ++seed) {
        Rng g{(uint64_t)seed * 0x2545F4914F6CDD1Dull};
        const int64_t n = g.range(1, 120);
        const int max_len = seed % 5 == 0 ? 70 : (int)g.range(1, 24);
        const int max_coef = seed % 7 == 0 ? 60 : 3;
        Csr c = random_ilp(g, n, g.range(0, 3 * n), max_len, max_coef);
        run(c, {}, {}, seed);
        // a batch of three copies of different instances
        Csr b;
        std::vector<int64_t> iv, ir;
        for (int k = 0; k < 3; ++k) {
            Rng h{(uint64_t)(seed * 7 + k)};
            Csr m = random_ilp(h, h.range(1, 60), h.range(0, 90), (int)h.range(1, 30), 3);
            for (size_t e = 0; e < m.col.size(); ++e) m.col[e] += (int32_t)b.n_vars;
            for (int64_t r = 0; r < m.n_rows(); ++r) {
                std::vector<int32_t> cs(m.col.begin() + m.row_ptr[r], m.col.begin() + m.row_ptr[r + 1]);
                std::vector<int32_t> as(m.coef.begin() + m.row_ptr[r], m.coef.begin() + m.row_ptr[r + 1]);
                b.row(cs, as, m.sense[r], m.rhs[r]);
            }
            b.cost.insert(b.cost.end(), m.cost.begin(), m.cost.end());
            b.n_vars += m.n_vars;
            iv.push_back(m.n_vars);
            ir.push_back(m.n_rows());
        }
        run(b, iv, ir, seed);
        std::vector<Csr> insts;
        for (int k = 0; k < (int)(seed % 4) + 1; ++k) {
            Rng h{(uint64_t)(seed * 13 + k)};
            const int64_t nk = h.range(0, 70);
            insts.push_back(random_ilp(h, nk, nk ? h.range(0, 2 * nk) : 0, seed % 6 == 0 ? 40 : (int)h.range(1, 22), 3));
        }
        run_merge(insts, (int)(seed % 5), seed);
    }
    {
        // enough rows for the threaded ingestion and compilation
        Rng h{4242};
        run(random_ilp(h, 3000, 6000, 6, 3), {}, {}, 4242);
    }
    {
        // one host thread against several
        Rng h{5151};
        run_threads(loose_ilp(h, 9000, 20000), 5151);
    }
    {
        // large enough for the threaded merge
        std::vector<Csr> big;
        for (int k = 0; k < 5; ++k) {
            Rng h{(uint64_t)(977 + k)};
            big.push_back(random_ilp(h, 2500 + 300 * k, 3500, 8, 3));
        }
        run_merge(big, 0, 977);
        run_merge(big, 4, 978);
    }
    std::printf("host checks: %d failures\n", fails);
    return fails ? 1 : 0;
}
