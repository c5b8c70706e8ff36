// Host-side driver for a sanitizer build (AddressSanitizer + UBSan) of the
// solver's host code: ingestion, instance boundaries, presolve, BDD
// compilation and tile packing, on generated ILPs (random rows around a
// hidden point, wide knapsack rows, long rows, empty rows, batches) under
// every packing option, and batches assembled from instances packed alone.
// Exits non-zero on the first inconsistency; the
// sanitizers abort on memory or undefined-behaviour errors.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

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
        rc = pack_problem(p, lds, 0, fast, merge, small, variant == 0 ? 0 : 16384, pk, msg);
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
                              variant == 2 ? 0 : 2048, variant == 0 ? 0 : 16384, pks[k], msg);
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
    std::printf("host checks: %d failures\n", fails);
    return fails ? 1 : 0;
}
