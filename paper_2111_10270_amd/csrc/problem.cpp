// ILP ingestion, presolve, BDD compilation and tile packing (host side).
//
// BDD compilation follows Sec. 5 (Defs. "BDD", "Constraint Set
// Correspondence"): one layer per variable of the row in ascending id order,
// two arcs per node, every root-to-accept path a feasible point.  Nodes start
// as partial sums of the assigned prefix, pruned by the interval of sums the
// remaining variables can still add; a bottom-up pass then removes nodes that
// cannot reach the accepting terminal and merges nodes with equal successor
// pairs, which gives the reduced (canonical) quasi-reduced BDD.  The paper only
// needs Def. "BDD"; reduction keeps the tiles small.
#include "problem.hpp"
#include "assemble.hpp"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <exception>
#include <thread>
#include <unordered_map>

namespace bddmma {

namespace {

uint64_t mix64(uint64_t h, uint64_t v)
{
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h * 0xFF51AFD7ED558CCDull;
}

bool sense_holds(int64_t v, int sense, int64_t b) { return sense < 0 ? v <= b : sense > 0 ? v >= b : v == b; }

std::atomic<int> g_thread_cap{16};

// host threads for construction work over `items` independent items: up to
// the cap (16 by default) and the hardware's threads, one below 4,096 items
int host_threads(int64_t items)
{
    unsigned hw = std::thread::hardware_concurrency();
    const unsigned cap = (unsigned)g_thread_cap.load(std::memory_order_relaxed);
    int n = (int)std::max(1u, std::min(hw ? hw : 1u, cap));
    return items < 4096 ? 1 : n;
}

// fn(t) for t in [0, n): t = 0 on the calling thread, the others on threads
// of their own.  An exception thrown on any of them (std::bad_alloc on a huge
// problem) is rethrown here once every thread has joined, so it reaches the
// caller's error handling instead of ending the process.
template <class F>
void run_threads(int n, F &&fn)
{
    if (n <= 1) {
        fn(0);
        return;
    }
    std::vector<std::exception_ptr> err((size_t)n);
    std::vector<std::thread> th;
    th.reserve((size_t)n - 1);
    try {
        for (int t = 1; t < n; ++t)
            th.emplace_back([&fn, &err, t] {
                try {
                    fn(t);
                } catch (...) {
                    err[(size_t)t] = std::current_exception();
                }
            });
        fn(0);
    } catch (...) {
        err[0] = std::current_exception();
    }
    for (auto &x : th) x.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// fn(t, begin, end) on nth contiguous ranges of [0, n), range t on thread t
template <class F>
void parallel_ranges(int64_t n, int nth, F &&fn)
{
    if (nth <= 1 || n < 2) {
        fn(0, (int64_t)0, n);
        return;
    }
    const int64_t chunk = (n + nth - 1) / nth;
    run_threads(nth, [&](int t) {
        const int64_t a = std::min<int64_t>(n, t * chunk), b = std::min<int64_t>(n, a + chunk);
        fn(t, a, b);
    });
}

// the result of std::sort(v, less) for a strict total order `less`: runs
// sorted on nth threads, then merged pairwise in parallel
template <class T, class L>
void parallel_sort(std::vector<T> &v, int nth, L less)
{
    const int64_t n = (int64_t)v.size();
    if (nth <= 1 || n < 16384) {
        std::sort(v.begin(), v.end(), less);
        return;
    }
    const int64_t chunk = (n + nth - 1) / nth;
    std::vector<int64_t> cut;
    for (int64_t a = 0; a < n; a += chunk) cut.push_back(a);
    cut.push_back(n);
    const int runs = (int)cut.size() - 1;
    parallel_ranges(runs, runs, [&](int, int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) std::sort(v.begin() + cut[r], v.begin() + cut[r + 1], less);
    });
    std::vector<T> tmp((size_t)n);
    while (cut.size() > 2) {
        std::vector<int64_t> next;
        const int pairs = ((int)cut.size() - 1 + 1) / 2;
        parallel_ranges(pairs, pairs, [&](int, int64_t a, int64_t b) {
            for (int64_t q = a; q < b; ++q) {
                const int64_t x0 = cut[2 * q], x1 = cut[std::min<size_t>(2 * q + 1, cut.size() - 1)],
                              x2 = cut[std::min<size_t>(2 * q + 2, cut.size() - 1)];
                std::merge(v.begin() + x0, v.begin() + x1, v.begin() + x1, v.begin() + x2, tmp.begin() + x0, less);
            }
        });
        for (size_t q = 0; q < cut.size(); q += 2) next.push_back(cut[q]);
        if (next.back() != n) next.push_back(n);
        cut.swap(next);
        v.swap(tmp);
    }
}

}  // namespace

void set_host_thread_cap(int n) { g_thread_cap.store(std::max(1, std::min(n, 16)), std::memory_order_relaxed); }

int ingest_ilp(Ilp &o, int64_t n_vars, const double *costs, int64_t n_rows, const int64_t *row_ptr,
               const int32_t *col, const int32_t *coef, const int8_t *sense, const int64_t *rhs,
               std::string &msg)
{
    if (n_vars < 0 || n_rows < 0 || n_vars > INT32_MAX - 1) { msg = "n_vars / n_rows out of range"; return ST_INVALID; }
    if (n_vars > 0 && !costs) { msg = "costs is NULL"; return ST_INVALID; }
    if (n_rows > 0 && (!row_ptr || !sense || !rhs)) { msg = "row arrays are NULL"; return ST_INVALID; }
    if (n_rows > 0 && row_ptr[0] != 0) { msg = "row_ptr[0] must be 0"; return ST_INVALID; }
    int64_t nnz = n_rows > 0 ? row_ptr[n_rows] : 0;
    if (nnz > 0 && (!col || !coef)) { msg = "col / coef are NULL"; return ST_INVALID; }
    o.n_vars = n_vars;
    o.n_rows = n_rows;
    o.inst_var = {0, n_vars};
    o.inst_row = {0, n_rows};
    o.cost.assign(costs, costs + n_vars);
    for (int64_t i = 0; i < n_vars; ++i)
        if (!(costs[i] == costs[i]) || costs[i] == __builtin_inf() || costs[i] == -__builtin_inf()) {
            msg = "cost " + std::to_string(i) + " is not finite";
            return ST_INVALID;
        }
    o.sense.assign(sense, sense + n_rows);
    o.rhs.assign(rhs, rhs + n_rows);
    // rows are checked, cleaned (zero coefficients dropped) and sorted by
    // column on several threads, in two passes over contiguous row ranges:
    // checks and counts, then entries written at their final place (and
    // repeated variables detected).  A range stops at its first bad row and
    // the lowest failing range reports, so the error is the first row in
    // order that fails the first pass, else the first with a repeated
    // variable.
    const int nth = host_threads(n_rows);
    const int64_t chunk = (n_rows + nth - 1) / std::max(1, nth);
    std::vector<std::string> err((size_t)nth);
    std::vector<char> bad((size_t)nth, 0);
    auto run = [&](auto &&body) {
        std::fill(bad.begin(), bad.end(), 0);
        auto one = [&](int t) {
            const int64_t r0 = std::min<int64_t>(n_rows, t * chunk), r1 = std::min<int64_t>(n_rows, r0 + chunk);
            for (int64_t r = r0; r < r1; ++r)
                if (!body(r, err[(size_t)t])) {
                    bad[(size_t)t] = 1;
                    return;
                }
        };
        run_threads(nth, one);
        for (int t = 0; t < nth; ++t)
            if (bad[(size_t)t]) {
                msg = err[(size_t)t];
                return false;
            }
        return true;
    };
    o.row_ptr.assign((size_t)n_rows + 1, 0);
    const bool counted = run([&](int64_t r, std::string &m) {
        if (row_ptr[r + 1] < row_ptr[r]) { m = "row_ptr decreases at row " + std::to_string(r); return false; }
        if (sense[r] < -1 || sense[r] > 1) { m = "sense must be -1, 0 or +1"; return false; }
        __int128 mag = 0;
        int64_t n = 0;
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n_vars) { m = "column out of range in row " + std::to_string(r); return false; }
            if (coef[e] == 0) continue;
            ++n;
            mag += coef[e] < 0 ? -(__int128)coef[e] : (__int128)coef[e];
        }
        __int128 rb = rhs[r] < 0 ? -(__int128)rhs[r] : (__int128)rhs[r];
        if (mag + rb > ((__int128)1 << 62)) { m = "row " + std::to_string(r) + ": coefficient sum too large"; return false; }
        o.row_ptr[r + 1] = n;
        return true;
    });
    if (!counted) return ST_INVALID;
    for (int64_t r = 0; r < n_rows; ++r) o.row_ptr[r + 1] += o.row_ptr[r];
    o.col.resize((size_t)o.row_ptr[n_rows]);
    o.coef.resize((size_t)o.row_ptr[n_rows]);
    const bool filled = run([&](int64_t r, std::string &m) {
        std::vector<std::pair<int32_t, int64_t>> ent;
        ent.reserve((size_t)(o.row_ptr[r + 1] - o.row_ptr[r]));
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
            if (coef[e] != 0) ent.emplace_back(col[e], (int64_t)coef[e]);
        std::sort(ent.begin(), ent.end());
        for (size_t q = 1; q < ent.size(); ++q)
            if (ent[q].first == ent[q - 1].first) { m = "variable repeated in row " + std::to_string(r); return false; }
        int64_t at = o.row_ptr[r];
        for (auto &pr : ent) {
            o.col[at] = pr.first;
            o.coef[at++] = pr.second;
        }
        return true;
    });
    return filled ? ST_OK : ST_INVALID;
}

int set_instances(Ilp &ilp, int64_t n_inst, const int64_t *inst_vars, const int64_t *inst_rows, std::string &msg)
{
    if (n_inst < 1 || !inst_vars || !inst_rows) { msg = "a batch needs n_inst >= 1 and both count arrays"; return ST_INVALID; }
    if (n_inst > INT32_MAX - 1) { msg = "too many instances"; return ST_INVALID; }
    ilp.inst_var.assign(1, 0);
    ilp.inst_row.assign(1, 0);
    for (int64_t k = 0; k < n_inst; ++k) {
        if (inst_vars[k] < 0 || inst_rows[k] < 0) { msg = "negative instance size"; return ST_INVALID; }
        ilp.inst_var.push_back(ilp.inst_var.back() + inst_vars[k]);
        ilp.inst_row.push_back(ilp.inst_row.back() + inst_rows[k]);
    }
    if (ilp.inst_var.back() != ilp.n_vars || ilp.inst_row.back() != ilp.n_rows) {
        msg = "instance sizes do not add up to n_vars / n_rows";
        return ST_INVALID;
    }
    for (int64_t k = 0; k < n_inst; ++k)
        for (int64_t r = ilp.inst_row[k]; r < ilp.inst_row[k + 1]; ++r)
            for (int64_t e = ilp.row_ptr[r]; e < ilp.row_ptr[r + 1]; ++e)
                if (ilp.col[e] < ilp.inst_var[k] || ilp.col[e] >= ilp.inst_var[k + 1]) {
                    msg = "row " + std::to_string(r) + " references a variable of another instance";
                    return ST_INVALID;
                }
    return ST_OK;
}

int compile_row(const int32_t *var, const int64_t *a_in, int k, int sense, int64_t b, BddSet &out,
                std::string &msg)
{
    thread_local std::vector<int64_t> A, slo, shi, cur, nxt;
    thread_local std::vector<std::vector<int64_t>> S;
    thread_local std::vector<std::vector<uint32_t>> W;   // raw child words per layer
    thread_local std::vector<std::vector<uint8_t>> alive;
    thread_local std::vector<std::vector<int32_t>> nid;
    thread_local std::vector<std::pair<uint64_t, int32_t>> keys;
    thread_local std::vector<std::pair<int32_t, int32_t>> reps;

    A.assign(a_in, a_in + k);
    if (sense > 0) {   // a.x >= b  <=>  -a.x <= -b
        for (auto &x : A) x = -x;
        b = -b;
        sense = -1;
    }
    slo.assign(k + 1, 0);
    shi.assign(k + 1, 0);
    for (int h = k - 1; h >= 0; --h) {
        slo[h] = slo[h + 1] + std::min<int64_t>(A[h], 0);
        shi[h] = shi[h + 1] + std::max<int64_t>(A[h], 0);
    }
    auto admissible = [&](int64_t s, int h) {
        if (sense < 0) return s + slo[h] <= b;
        return s + slo[h] <= b && b <= s + shi[h];
    };
    // a <= row is certain once even the largest completion stays within b; all
    // such partial sums of a layer have the same (all-accepting) future, so
    // they share one state, b - shi[h] (the reduction below would merge them
    // anyway; merging here keeps rows with huge weights, which have few
    // undecided sums per layer, from growing before the reduction)
    auto canon = [&](int64_t v, int h) {
        if (sense < 0 && h < k && v + shi[h] <= b) return b - shi[h];
        return v;
    };
    if (!admissible(0, 0)) return ST_INFEASIBLE;
    if ((int)S.size() < k + 1) { S.resize(k + 1); W.resize(k + 1); alive.resize(k + 1); nid.resize(k + 1); }
    S[0].assign(1, canon(0, 0));
    for (int h = 0; h < k; ++h) {
        // successors of layer h: s (zero-arc) and s + a_h (one-arc); both lists sorted
        const auto &s = S[h];
        auto &n = S[h + 1];
        n.clear();
        size_t i = 0, j = 0;
        const int64_t d = A[h];
        while (i < s.size() || j < s.size()) {
            int64_t v;
            if (j >= s.size() || (i < s.size() && s[i] <= s[j] + d)) v = s[i++];
            else v = s[j++] + d;
            v = canon(v, h + 1);
            if ((n.empty() || n.back() != v) && (h + 1 == k ? (sense < 0 ? v <= b : v == b) : admissible(v, h + 1)))
                n.push_back(v);
        }
        if (h + 1 < k && (int64_t)n.size() > kMaxWidth) {
            msg = "BDD layer wider than 65533 nodes";
            return ST_INVALID;
        }
        if (n.empty()) return ST_INFEASIBLE;
    }
    // arcs: index into the next layer, or the terminals after the last layer
    for (int h = 0; h < k; ++h) {
        const auto &s = S[h];
        W[h].resize(s.size());
        for (size_t q = 0; q < s.size(); ++q) {
            uint32_t c[2];
            for (int t = 0; t < 2; ++t) {
                int64_t v = canon(s[q] + (t ? A[h] : 0), h + 1);
                if (h + 1 == k) {
                    c[t] = std::binary_search(S[k].begin(), S[k].end(), v) ? kTop : kBot;
                } else {
                    auto it = std::lower_bound(S[h + 1].begin(), S[h + 1].end(), v);
                    c[t] = (it != S[h + 1].end() && *it == v) ? (uint32_t)(it - S[h + 1].begin()) : kBot;
                }
            }
            W[h][q] = c[0] | (c[1] << 16);
        }
    }
    // bottom-up: drop nodes that cannot reach the accepting terminal
    for (int h = k - 1; h >= 0; --h) {
        alive[h].assign(W[h].size(), 0);
        for (size_t q = 0; q < W[h].size(); ++q) {
            uint32_t c[2] = {W[h][q] & 0xFFFFu, W[h][q] >> 16};
            for (int t = 0; t < 2; ++t) {
                bool ok = c[t] == kTop || (c[t] != kBot && alive[h + 1][c[t]]);
                if (!ok) c[t] = kBot;
            }
            W[h][q] = c[0] | (c[1] << 16);
            alive[h][q] = (c[0] != kBot) || (c[1] != kBot);
        }
    }
    if (!alive[0][0]) return ST_INFEASIBLE;
    // bottom-up: merge nodes with equal successor pairs, ids in order of first appearance
    std::vector<int32_t> width(k);
    for (int h = k - 1; h >= 0; --h) {
        keys.clear();
        for (size_t q = 0; q < W[h].size(); ++q) {
            if (!alive[h][q]) continue;
            uint32_t c[2] = {W[h][q] & 0xFFFFu, W[h][q] >> 16};
            if (h + 1 < k)
                for (int t = 0; t < 2; ++t)
                    if (c[t] != kBot) c[t] = (uint32_t)nid[h + 1][c[t]];
            W[h][q] = c[0] | (c[1] << 16);
            keys.emplace_back(W[h][q], (int32_t)q);
        }
        std::sort(keys.begin(), keys.end());
        reps.clear();
        for (size_t q = 0; q < keys.size(); ++q)
            if (q == 0 || keys[q].first != keys[q - 1].first) reps.emplace_back(keys[q].second, (int32_t)q);
        std::sort(reps.begin(), reps.end());
        nid[h].assign(W[h].size(), -1);
        // group start position -> final id
        std::vector<int32_t> gid(keys.size());
        for (size_t r = 0; r < reps.size(); ++r) gid[reps[r].second] = (int32_t)r;
        int32_t g = -1;
        for (size_t q = 0; q < keys.size(); ++q) {
            if (q == 0 || keys[q].first != keys[q - 1].first) g = gid[q];
            nid[h][keys[q].second] = g;
        }
        width[h] = (int32_t)reps.size();
        // compact words into final order
        std::vector<uint32_t> words(reps.size());
        for (size_t r = 0; r < reps.size(); ++r) words[r] = W[h][reps[r].first];
        W[h].swap(words);
    }
    for (int h = 0; h < k; ++h) {
        out.lay_var.push_back(var[h]);
        out.lay_width.push_back(width[h]);
        out.child.insert(out.child.end(), W[h].begin(), W[h].end());
    }
    out.lay_off.push_back((int64_t)out.lay_var.size());
    out.node_off.push_back((int64_t)out.child.size());
    return ST_OK;
}

namespace {

struct PassResult {
    BddSet set;
    std::vector<std::pair<int32_t, int8_t>> forced;
    int status = ST_OK;
    std::string msg;
};

void compile_rows(const Ilp &ilp, const std::vector<int8_t> &fixed, int64_t r0, int64_t r1, PassResult &res)
{
    BddSet &o = res.set;
    o.lay_off.assign(1, 0);
    o.node_off.assign(1, 0);
    std::vector<int32_t> v;
    std::vector<int64_t> a;
    for (int64_t r = r0; r < r1; ++r) {
        v.clear();
        a.clear();
        int64_t b = ilp.rhs[r];
        for (int64_t e = ilp.row_ptr[r]; e < ilp.row_ptr[r + 1]; ++e) {
            int32_t c = ilp.col[e];
            if (fixed[c] >= 0) { b -= ilp.coef[e] * fixed[c]; continue; }
            v.push_back(c);
            a.push_back(ilp.coef[e]);
        }
        if (v.empty()) {
            if (!sense_holds(0, ilp.sense[r], b)) {
                res.status = ST_INFEASIBLE;
                res.msg = "row " + std::to_string(r) + " is violated by the fixed variables";
                return;
            }
            continue;
        }
        size_t l0 = o.lay_var.size(), n0 = o.child.size();
        int st = compile_row(v.data(), a.data(), (int)v.size(), ilp.sense[r], b, o, res.msg);
        if (st != ST_OK) {
            res.status = st;
            if (st == ST_INFEASIBLE) res.msg = "row " + std::to_string(r) + " has no feasible 0-1 point";
            else res.msg = "row " + std::to_string(r) + ": " + res.msg;
            return;
        }
        o.row.push_back((int32_t)r);
        // a layer without zero-arcs (one-arcs) forces its variable to 1 (0)
        size_t node = n0;
        for (size_t h = l0; h < o.lay_var.size(); ++h) {
            bool has0 = false, has1 = false;
            for (int32_t q = 0; q < o.lay_width[h]; ++q, ++node) {
                uint32_t w = o.child[node];
                has0 |= (w & 0xFFFFu) != kBot;
                has1 |= (w >> 16) != kBot;
            }
            if (!has0 || !has1) res.forced.emplace_back(o.lay_var[h], (int8_t)(has1 ? 1 : 0));
        }
    }
}

}  // namespace

int build_problem(Problem &p, std::string &msg)
{
    const Ilp &ilp = p.ilp;
    p.fixed.assign(ilp.n_vars, -1);
    const int nthreads = host_threads(ilp.n_rows);
    std::vector<PassResult> res;
    // Presolve by rounds: compile every row against the fixings known at the
    // start of the round, then apply all forced values; repeat until a round
    // forces nothing.  The fixed set is the closure of single-row implications,
    // so the order of rounds does not change it.
    for (;;) {
        res.assign(nthreads, PassResult());
        const int64_t chunk = (ilp.n_rows + nthreads - 1) / nthreads;
        run_threads(nthreads, [&](int t) {
            const int64_t r0 = std::min<int64_t>(ilp.n_rows, t * chunk), r1 = std::min<int64_t>(ilp.n_rows, r0 + chunk);
            compile_rows(ilp, p.fixed, r0, r1, res[(size_t)t]);
        });
        for (auto &r : res)
            if (r.status != ST_OK) { msg = r.msg; return r.status; }
        bool any = false;
        for (auto &r : res)
            for (auto &f : r.forced) {
                int8_t &cur = p.fixed[f.first];
                if (cur >= 0 && cur != f.second) {
                    msg = "variable " + std::to_string(f.first) + " is forced to both 0 and 1";
                    return ST_INFEASIBLE;
                }
                if (cur < 0) { cur = f.second; any = true; }
            }
        if (!any) break;
    }
    // concatenate the per-thread stores (each already in ascending row order),
    // every store copied to its final place by its own thread
    BddSet &B = p.bdds;
    B = BddSet();
    const size_t nres = res.size();
    std::vector<int64_t> bo(nres + 1, 0), lo(nres + 1, 0), no(nres + 1, 0);
    for (size_t r = 0; r < nres; ++r) {
        bo[r + 1] = bo[r] + (int64_t)res[r].set.row.size();
        lo[r + 1] = lo[r] + (int64_t)res[r].set.lay_var.size();
        no[r + 1] = no[r] + (int64_t)res[r].set.child.size();
    }
    B.row.resize((size_t)bo[nres]);
    B.lay_off.resize((size_t)bo[nres] + 1);
    B.node_off.resize((size_t)bo[nres] + 1);
    B.lay_var.resize((size_t)lo[nres]);
    B.lay_width.resize((size_t)lo[nres]);
    B.child.resize((size_t)no[nres]);
    B.lay_off[0] = 0;
    B.node_off[0] = 0;
    parallel_ranges((int64_t)nres, (int)nres, [&](int, int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            BddSet &s = res[(size_t)r].set;
            std::copy(s.row.begin(), s.row.end(), B.row.begin() + bo[r]);
            for (size_t j = 1; j < s.lay_off.size(); ++j) B.lay_off[(size_t)bo[r] + j] = lo[r] + s.lay_off[j];
            for (size_t j = 1; j < s.node_off.size(); ++j) B.node_off[(size_t)bo[r] + j] = no[r] + s.node_off[j];
            std::copy(s.lay_var.begin(), s.lay_var.end(), B.lay_var.begin() + lo[r]);
            std::copy(s.lay_width.begin(), s.lay_width.end(), B.lay_width.begin() + lo[r]);
            std::copy(s.child.begin(), s.child.end(), B.child.begin() + no[r]);
            s = BddSet();
        }
    });
    res.clear();
    const int64_t P = (int64_t)B.lay_var.size();
    p.deg.assign(ilp.n_vars, 0);
    p.pair_var.resize(P);
    p.pair_row.resize(P);
    parallel_ranges(B.n_bdds(), host_threads(B.n_bdds()), [&](int, int64_t a, int64_t b) {
        for (int64_t j = a; j < b; ++j)
            for (int64_t q = B.lay_off[j]; q < B.lay_off[j + 1]; ++q) {
                p.pair_var[q] = B.lay_var[q];
                p.pair_row[q] = B.row[j];
            }
    });
    {
        // |J_i|: each thread counts the pairs of its own variable range
        const int dt = host_threads(P);
        const int64_t V = ilp.n_vars, chunk = (V + dt - 1) / dt;
        parallel_ranges(dt, dt, [&](int t, int64_t, int64_t) {
            const int64_t v0 = std::min<int64_t>(V, t * chunk), v1 = std::min<int64_t>(V, v0 + chunk);
            std::vector<int32_t> cnt((size_t)(v1 - v0) + 1, 0);   // last entry absorbs other ranges
            const uint64_t span = (uint64_t)(v1 - v0);
            for (int64_t q = 0; q < P; ++q) {
                const uint64_t d = (uint64_t)((int64_t)B.lay_var[q] - v0);
                cnt[d < span ? d : span]++;
            }
            std::copy(cnt.begin(), cnt.end() - 1, p.deg.begin() + v0);
        });
    }
    p.lb_offset = 0.0;
    p.n_fixed = p.n_free = 0;
    p.inst_offset.assign((size_t)ilp.n_inst(), 0.0);
    for (int64_t k = 0; k < ilp.n_inst(); ++k)
        for (int64_t i = ilp.inst_var[k]; i < ilp.inst_var[k + 1]; ++i) {
            double c = 0.0;
            if (p.fixed[i] >= 0) {
                c = p.fixed[i] ? ilp.cost[i] : 0.0;
                p.n_fixed++;
            } else if (p.deg[i] == 0) {
                c = ilp.cost[i] < 0.0 ? ilp.cost[i] : 0.0;
                p.n_free++;
            }
            p.lb_offset += c;
            p.inst_offset[k] += c;
        }
    p.n_nodes = (int64_t)B.child.size();
    if (P >= INT32_MAX) { msg = "too many pairs"; return ST_INVALID; }
    return ST_OK;
}

namespace {

struct TilePlan {
    std::vector<int64_t> lanes;   // BDD ids, -1 for padding lanes
    bool shared = false;
    int K = 0;
    std::vector<int32_t> width;   // [K] layer widths of the tile layout
    int64_t first_row = 0;
    int wi = -1, ki = -1;         // fast-path class, -1 = general kernels only
    bool mix = false;             // fast path with per-lane topologies
    bool lng = false;             // chunked register kernel (width 2, K beyond the classes)
    bool wide = false;            // wide kernel (a group of lanes per BDD)
};

}  // namespace

int pack_problem(const Problem &p, int lds_elem_budget, int lds_max_nodes, bool fast, double merge_bytes,
                 int64_t small_tiles, int wide_lds_elems, int wide_min_width, int fuse_elem, Packed &o,
                 std::string &msg)
{
    const BddSet &B = p.bdds;
    const int64_t nb = B.n_bdds();
    const int64_t V = p.ilp.n_vars;
    auto k_of = [&](int64_t j) { return (int)(B.lay_off[j + 1] - B.lay_off[j]); };
    auto n_of = [&](int64_t j) { return (int64_t)(B.node_off[j + 1] - B.node_off[j]); };
    const int nth = host_threads(nb);
    std::vector<uint64_t> hash(nb);
    parallel_ranges(nb, nth, [&](int, int64_t a, int64_t b) {
        for (int64_t j = a; j < b; ++j) {
            uint64_t h = mix64(0, (uint64_t)k_of(j));
            for (int64_t q = B.lay_off[j]; q < B.lay_off[j + 1]; ++q) h = mix64(h, (uint64_t)B.lay_width[q]);
            for (int64_t q = B.node_off[j]; q < B.node_off[j + 1]; ++q) h = mix64(h, B.child[q]);
            hash[j] = h;
        }
    });
    // instance of every BDD (tiles never mix instances of a batch)
    const Ilp &ilp = p.ilp;
    const bool batch = ilp.n_inst() > 1;
    std::vector<int32_t> row_inst;
    if (batch) {
        row_inst.resize((size_t)ilp.n_rows);
        for (int64_t k = 0; k < ilp.n_inst(); ++k)
            for (int64_t r = ilp.inst_row[k]; r < ilp.inst_row[k + 1]; ++r) row_inst[r] = (int32_t)k;
    }
    auto inst_of = [&](int64_t j) { return batch ? row_inst[B.row[j]] : 0; };
    auto same_topology = [&](int64_t x, int64_t y) {
        if (inst_of(x) != inst_of(y)) return false;
        if (k_of(x) != k_of(y) || n_of(x) != n_of(y) || hash[x] != hash[y]) return false;
        return std::equal(B.lay_width.begin() + B.lay_off[x], B.lay_width.begin() + B.lay_off[x + 1],
                          B.lay_width.begin() + B.lay_off[y]) &&
               std::equal(B.child.begin() + B.node_off[x], B.child.begin() + B.node_off[x + 1],
                          B.child.begin() + B.node_off[y]);
    };
    std::vector<int64_t> order(nb);
    for (int64_t j = 0; j < nb; ++j) order[j] = j;
    parallel_sort(order, nth, [&](int64_t x, int64_t y) {
        if (inst_of(x) != inst_of(y)) return inst_of(x) < inst_of(y);
        if (k_of(x) != k_of(y)) return k_of(x) < k_of(y);
        if (n_of(x) != n_of(y)) return n_of(x) < n_of(y);
        if (hash[x] != hash[y]) return hash[x] < hash[y];
        return x < y;
    });
    std::vector<TilePlan> plans;
    std::vector<int64_t> mixed;
    for (int64_t s = 0; s < nb;) {
        int64_t e = s + 1;
        while (e < nb && same_topology(order[s], order[e])) ++e;
        int64_t len = e - s;
        int64_t full = len / kLanes, rem = len % kLanes;
        for (int64_t t = 0; t < full + (rem >= 16 ? 1 : 0); ++t) {
            TilePlan tp;
            tp.shared = true;
            for (int l = 0; l < kLanes; ++l) {
                int64_t q = s + t * kLanes + l;
                tp.lanes.push_back(q < e ? order[q] : -1);
            }
            plans.push_back(std::move(tp));
        }
        if (rem > 0 && rem < 16)
            for (int64_t q = s + full * kLanes; q < e; ++q) mixed.push_back(order[q]);
        s = e;
    }
    std::sort(mixed.begin(), mixed.end(), [&](int64_t x, int64_t y) {
        if (inst_of(x) != inst_of(y)) return inst_of(x) < inst_of(y);
        if (n_of(x) != n_of(y)) return n_of(x) < n_of(y);
        if (k_of(x) != k_of(y)) return k_of(x) < k_of(y);
        return x < y;
    });
    for (size_t s = 0; s < mixed.size();) {
        size_t e = s;
        while (e < mixed.size() && e - s < (size_t)kLanes && inst_of(mixed[e]) == inst_of(mixed[s])) ++e;
        TilePlan tp;
        for (int l = 0; l < kLanes; ++l) tp.lanes.push_back(s + l < e ? mixed[s + l] : -1);
        plans.push_back(std::move(tp));
        s = e;
    }
    // tile shapes
    const bool small = (int64_t)plans.size() <= small_tiles;
    for (auto &tp : plans) {
        int K = 0;
        tp.first_row = INT64_MAX;
        for (int64_t j : tp.lanes)
            if (j >= 0) {
                K = std::max(K, k_of(j));
                tp.first_row = std::min<int64_t>(tp.first_row, B.row[j]);
            }
        K = std::max(K, 1);
        tp.K = K;
        tp.width.assign(K, 1);
        for (int64_t j : tp.lanes)
            if (j >= 0)
                for (int h = 0; h < k_of(j); ++h)
                    tp.width[h] = std::max(tp.width[h], B.lay_width[B.lay_off[j] + h]);
        const int maxw = *std::max_element(tp.width.begin(), tp.width.end());
        for (int wi = 0; fast && tp.shared && wi < kNumWClasses && tp.wi < 0; ++wi)
            if (maxw <= kWClass[wi])
                for (int ki = 0; ki < kNumKClasses; ++ki)
                    if (K <= kKClass[ki] && fast_class_ok(wi, ki)) {
                        tp.wi = wi;
                        tp.ki = ki;
                        break;
                    }
        // small problems: width-2 tiles of one topology join the mixed tiles
        // (per-lane words), so each sweep needs one launch per layer class
        // instead of one per class and kind; the launches of a small problem
        // are latency-bound, so fewer of them beats cheaper lanes
        if (fast && tp.shared && small && maxw <= kWClass[0]) tp.shared = false;
        if (fast && !tp.shared && maxw <= kWClass[0])
            for (int ki = 0; ki < kNumKClasses; ++ki)
                if (K <= kKClass[ki] && mix_class_ok(ki)) {
                    tp.wi = 0;
                    tp.ki = ki;
                    tp.mix = true;
                    break;
                }
        if (fast && tp.wi < 0 && maxw <= kWClass[0] && K > kKClass[kNumKClasses - 1]) {
            tp.wi = 0;
            tp.lng = true;
            tp.mix = !tp.shared;
        }
        int64_t nodes = 0;
        for (int w : tp.width) nodes += w;
        if (K > 65535 || nodes > 65535) { msg = "a BDD has more than 65535 layers or nodes"; return ST_INVALID; }
        tp.wide = fast && tp.wi < 0 && wide_min_width > 0 && maxw >= wide_min_width && wide_lds_elems > 0 &&
                  2 * nodes + 2 * (int64_t)K <= (int64_t)wide_lds_elems;
    }
    // Fewer launches: inside a width class, the tiles of a layer class join
    // the next larger class present (padded to its layer count) while the
    // padding moves fewer bytes per sweep than a separate launch costs (a
    // small launch runs for about one wave lifetime at low occupancy):
    // merge_bytes, 0 = every class launches on its own.
    constexpr double kSlotBytes = 16.0;                // lambda and M read + written (FP32)
    for (int g = 0; g < kNumWClasses + 1; ++g) {
        // groups: shared tiles of each width class, then the mixed tiles
        const int wi = g < kNumWClasses ? g : 0;
        const bool mix = g == kNumWClasses;
        auto in_group = [&](const TilePlan &tp) { return tp.wi == wi && tp.mix == mix && !tp.lng; };
        int64_t cnt[kNumKClasses] = {0};
        for (auto &tp : plans)
            if (in_group(tp)) cnt[tp.ki]++;
        int into[kNumKClasses];
        for (int ki = 0; ki < kNumKClasses; ++ki) into[ki] = ki;
        for (;;) {
            int best = -1, best_to = -1;
            double best_cost = merge_bytes;
            for (int ki = 0; ki < kNumKClasses; ++ki) {
                if (!cnt[ki]) continue;
                int kj = ki + 1;
                while (kj < kNumKClasses && !cnt[kj]) ++kj;
                if (kj == kNumKClasses) break;
                const double cost = (double)cnt[ki] * (kKClass[kj] - kKClass[ki]) * kLanes * kSlotBytes;
                if (cost <= best_cost) {
                    best_cost = cost;
                    best = ki;
                    best_to = kj;
                }
            }
            if (best < 0 || merge_bytes <= 0.0) break;
            cnt[best_to] += cnt[best];
            cnt[best] = 0;
            for (int ki = 0; ki < kNumKClasses; ++ki)
                if (into[ki] == best) into[ki] = best_to;
        }
        for (auto &tp : plans)
            if (in_group(tp)) tp.ki = into[tp.ki];
    }
    // fast tiles: exactly the class's layer count (long tiles keep theirs),
    // fixed layer stride
    for (auto &tp : plans)
        if (tp.wi >= 0) {
            if (!tp.lng) tp.K = kKClass[tp.ki];
            tp.width.assign(tp.K, kWClass[tp.wi]);
        }
    auto tile_nodes = [](const TilePlan &tp) {
        int64_t n = 0;
        for (int w : tp.width) n += w;
        return n;
    };
    auto in_lds = [&](const TilePlan &tp) {
        if (tp.lng) return false;   // the chunked kernel keeps its values in device scratch
        const int64_t n = tile_nodes(tp);
        return lds_elem_budget > 0 && (int64_t)lane_elems(tp.K, (uint32_t)n) <= lds_elem_budget &&
               (lds_max_nodes <= 0 || n <= lds_max_nodes);
    };
    std::stable_sort(plans.begin(), plans.end(),
                     [&](const TilePlan &x, const TilePlan &y) { return x.first_row < y.first_row; });

    // emit
    o = Packed();
    std::vector<std::vector<int32_t>> lists(kNumLists);
    int64_t slots = 0, scratch = 0;
    // topology hash -> ((representative BDD, node base), width class) of emitted shared tiles
    std::unordered_multimap<uint64_t, std::pair<std::pair<int64_t, int64_t>, int>> topo_base;
    // place the node words of BDD j into the tile layout (stride 1: shared, 64: per lane)
    auto place = [&](int64_t j, const std::vector<uint32_t> &noff, int K, size_t base, size_t stride, int lane) {
        const int kj = j >= 0 ? k_of(j) : 0;
        int64_t src = j >= 0 ? B.node_off[j] : 0;
        for (int h = 0; h < K; ++h) {
            if (h < kj) {
                const int wj = B.lay_width[B.lay_off[j] + h];
                for (int q = 0; q < wj; ++q) {
                    uint32_t w = B.child[src++];
                    if (h == kj - 1 && kj < K) {   // accept -> padding chain
                        uint32_t lo = w & 0xFFFFu, hi = w >> 16;
                        if (lo == kTop) lo = 0;
                        if (hi == kTop) hi = 0;
                        w = lo | (hi << 16);
                    }
                    o.child[base + (size_t)(noff[h] + q) * stride + lane] = w;
                }
            } else {
                const uint32_t nxt = (h == K - 1) ? kTop : 0u;
                o.child[base + (size_t)noff[h] * stride + lane] = nxt | (nxt << 16);
            }
        }
    };
    for (auto &tp : plans) {
        const int32_t tid = (int32_t)o.tiles.size();
        TileDesc d{};
        d.pair_base = (uint32_t)slots;
        d.node_base = (uint32_t)o.child.size();
        d.layer_base = (uint32_t)o.layers.size();
        d.K = (uint16_t)tp.K;
        const int64_t nodes = tile_nodes(tp);
        d.nodes = (uint16_t)nodes;
        d.flags = tp.shared ? TILE_SHARED : 0;
        if (in_lds(tp)) {
            o.max_lds_lane_elems = std::max<int>(o.max_lds_lane_elems, (int)lane_elems(tp.K, (uint32_t)nodes));
            d.scratch_base = 0;
            lists[LIST_GEN_LDS_ALL].push_back(tid);
            if (tp.wi < 0 && !tp.wide) lists[LIST_GEN_LDS_REST].push_back(tid);
        } else {
            d.scratch_base = (uint32_t)scratch;
            scratch += (int64_t)kLanes * lane_elems(tp.K, (uint32_t)nodes);
            lists[LIST_GEN_GLOB_ALL].push_back(tid);
            if (tp.wi < 0 && !tp.wide) lists[LIST_GEN_GLOB_REST].push_back(tid);
        }
        if (tp.wide) {
            lists[LIST_WIDE].push_back(tid);
            o.max_wide_elems = std::max<int>(o.max_wide_elems, (int)(2 * nodes + 2 * tp.K));
        }
        if (tp.wi >= 0) {
            lists[tp.lng ? (tp.mix ? LIST_LONG_MIX : LIST_LONG_SH) : tp.mix ? mix_list(tp.ki) : fast_list(tp.wi, tp.ki)]
                .push_back(tid);
        }
        std::vector<uint32_t> noff(tp.K + 1, 0);
        for (int h = 0; h < tp.K; ++h) {
            noff[h + 1] = noff[h] + tp.width[h];
            o.layers.push_back(layer_entry(noff[h], tp.width[h]));
        }
        o.max_layers = std::max(o.max_layers, tp.K);
        for (int64_t j : tp.lanes)
            if (j >= 0)
                for (int h = 0; h < k_of(j); ++h) o.max_width = std::max(o.max_width, B.lay_width[B.lay_off[j] + h]);
        const size_t base = o.child.size();
        if (tp.shared) {
            // tiles of one topology share a single copy of the node words (and
            // hence the scalar-cache lines that hold them)
            const int64_t rep = tp.lanes[0];
            int64_t found = -1;
            auto range = topo_base.equal_range(hash[rep]);
            for (auto it = range.first; it != range.second; ++it)
                if (it->second.second == (int)tp.wi && same_topology(it->second.first.first, rep)) {
                    found = it->second.first.second;
                    break;
                }
            if (found >= 0) {
                d.node_base = (uint32_t)found;
            } else {
                // fast tiles: the standard words, then the register kernel's
                // copy whose last layer points accepting arcs at node 0
                const size_t copies = tp.wi >= 0 ? 2 : 1;
                o.child.resize(base + copies * (size_t)nodes, kBot | (kBot << 16));
                place(rep, noff, tp.K, base, 1, 0);
                if (tp.wi >= 0)
                    for (int64_t n = 0; n < nodes; ++n) {
                        uint32_t w = o.child[base + (size_t)n];
                        if ((int64_t)noff[tp.K - 1] <= n) {
                            uint32_t lo = w & 0xFFFFu, hi = w >> 16;
                            if (lo == kTop) lo = 0;
                            if (hi == kTop) hi = 0;
                            w = lo | (hi << 16);
                        }
                        o.child[base + (size_t)nodes + (size_t)n] = w;
                    }
                topo_base.emplace(hash[rep], std::make_pair(std::make_pair(rep, (int64_t)base), (int)tp.wi));
            }
            d.fast_base = tp.wi >= 0 ? d.node_base + (uint32_t)nodes : d.node_base;
        } else {
            const size_t copies = tp.wi >= 0 || tp.wide ? 2 : 1;
            const size_t per = (size_t)nodes * kLanes;
            o.child.resize(base + copies * per, kBot | (kBot << 16));
            for (int l = 0; l < kLanes; ++l) place(tp.lanes[l], noff, tp.K, base, kLanes, l);
            d.fast_base = d.node_base;
            if (tp.wide) {
                // BDD-major copy for the wide kernel
                for (int l = 0; l < kLanes; ++l)
                    for (int64_t n = 0; n < nodes; ++n)
                        o.child[base + per + (size_t)l * nodes + n] = o.child[base + (size_t)n * kLanes + l];
                d.fast_base = d.node_base + (uint32_t)per;
            }
            if (tp.wi >= 0) {
                // the register kernel's per-lane copy (accepting arcs of the last layer -> node 0)
                const size_t last = (size_t)noff[tp.K - 1] * kLanes;
                for (size_t n = 0; n < per; ++n) {
                    uint32_t w = o.child[base + n];
                    if (n >= last) {
                        uint32_t lo = w & 0xFFFFu, hi = w >> 16;
                        if (lo == kTop) lo = 0;
                        if (hi == kTop) hi = 0;
                        w = lo | (hi << 16);
                    }
                    o.child[base + per + n] = w;
                }
                d.fast_base = d.node_base + (uint32_t)per;
            }
        }
        o.tiles.push_back(d);
        slots += (int64_t)tp.K * kLanes;
        if (slots >= INT32_MAX || scratch >= (int64_t)UINT32_MAX || o.child.size() >= UINT32_MAX) {
            msg = "problem too large for 32-bit slot indices";
            return ST_INVALID;
        }
    }
    o.list_off.assign(kNumLists + 1, 0);
    for (int l = 0; l < kNumLists; ++l) {
        o.list_off[l + 1] = o.list_off[l] + (int64_t)lists[l].size();
        o.lists.insert(o.lists.end(), lists[l].begin(), lists[l].end());
    }
    // every arc must stay inside the tile: heads index the next layer, and only
    // the last layer may reach the accepting terminal
    for (const TileDesc &d : o.tiles) {
        const bool sh = (d.flags & TILE_SHARED) != 0;
        for (uint32_t h = 0; h < d.K; ++h) {
            const uint32_t le = o.layers[d.layer_base + h], noff = le & 0xFFFFu, W = le >> 16;
            const uint32_t Wn = h + 1 < d.K ? (o.layers[d.layer_base + h + 1] >> 16) : 0u;
            if (noff + W > d.nodes || (h + 1 < d.K && noff + W + Wn > d.nodes)) {
                msg = "internal error: inconsistent layer table";
                return ST_INVALID;
            }
            for (uint32_t q = 0; q < W; ++q)
                for (int l = 0; l < (sh ? 1 : kLanes); ++l) {
                    const uint32_t w = o.child[d.node_base + (sh ? (noff + q) : (size_t)(noff + q) * kLanes + l)];
                    for (uint32_t c : {w & 0xFFFFu, w >> 16}) {
                        const bool ok = c == kBot || (c == kTop ? h + 1 == d.K : (h + 1 < d.K && c < Wn));
                        if (!ok) {
                            msg = "internal error: BDD arc leaves its tile";
                            return ST_INVALID;
                        }
                    }
                }
        }
    }
    // the register kernel's copy: fixed stride W, heads below W, node 0 of the
    // virtual terminal layer only from the last layer; layer count = class
    for (int l = LIST_FAST0; l < LIST_WIDE; ++l) {
        const bool lng = l >= LIST_LONG_SH;
        const bool mix = lng ? l == LIST_LONG_MIX : l >= LIST_MIX0;
        const int wi = mix || lng ? 0 : (l - LIST_FAST0) / kNumKClasses;
        const int ki = lng ? -1 : mix ? l - LIST_MIX0 : (l - LIST_FAST0) % kNumKClasses;
        for (int32_t t : lists[l]) {
            const TileDesc &d = o.tiles[t];
            // long tiles keep 3K values per lane in their device scratch
            const bool ok = (lng ? d.K > kKClass[kNumKClasses - 1] &&
                                       3ull * d.K <= lane_elems(d.K, d.nodes) &&
                                       (uint64_t)d.scratch_base + 64ull * lane_elems(d.K, d.nodes) <=
                                           (uint64_t)scratch
                                 : d.K == kKClass[ki]) &&
                            (o.layers[d.layer_base] >> 16) == (uint32_t)kWClass[wi] &&
                            d.fast_base != d.node_base && ((d.flags & TILE_SHARED) != 0) == !mix &&
                            (lng || (mix ? mix_class_ok(ki) : fast_class_ok(wi, ki)));
            if (!ok) {
                msg = "internal error: fast-path tile does not match its kernel class";
                return ST_INVALID;
            }
        }
    }
    std::vector<char> on_fast(o.tiles.size(), 0);
    for (int l = LIST_FAST0; l < LIST_WIDE; ++l)
        for (int32_t t : lists[l]) on_fast[t] = 1;
    for (int32_t t : lists[LIST_WIDE]) {
        const TileDesc &d = o.tiles[t];
        const bool sh = (d.flags & TILE_SHARED) != 0;
        if (on_fast[t] || (!sh && (uint64_t)d.fast_base + 64ull * d.nodes > o.child.size()) ||
            (sh && d.fast_base != d.node_base) || 2 * d.nodes + 2 * d.K > o.max_wide_elems) {
            msg = "internal error: inconsistent wide tile";
            return ST_INVALID;
        }
    }
    for (size_t t = 0; t < o.tiles.size(); ++t) {
        const TileDesc &d = o.tiles[t];
        if (!on_fast[t]) continue;
        const uint32_t W = o.layers[d.layer_base] >> 16;
        const bool sh = (d.flags & TILE_SHARED) != 0;
        const uint32_t lanes = sh ? 1 : kLanes;
        if ((uint64_t)d.fast_base + (uint64_t)d.K * W * lanes > o.child.size()) {
            msg = "internal error: inconsistent fast-path words";
            return ST_INVALID;
        }
        for (uint32_t h = 0; h < d.K; ++h)
            for (uint32_t q = 0; q < W; ++q)
                for (uint32_t l = 0; l < lanes; ++l) {
                    const uint32_t w = o.child[d.fast_base + (h * W + q) * lanes + l];
                    for (uint32_t c : {w & 0xFFFFu, w >> 16})
                        if (!(c == kBot || (h + 1 < d.K ? c < W : c == 0))) {
                            msg = "internal error: fast-path arc out of range";
                            return ST_INVALID;
                        }
                }
    }
    // instance ranges of the tiles (tiles are sorted by first row, and the rows
    // of instance k precede those of instance k+1)
    o.inst_tile.assign(1, 0);
    o.tile_inst.clear();
    o.var_inst.clear();
    o.row_inst.clear();
    for (size_t t = 0; t < plans.size(); ++t) {
        int32_t k = 0;
        for (int64_t j : plans[t].lanes)
            if (j >= 0) {
                k = inst_of(j);
                break;
            }
        for (int64_t j : plans[t].lanes)
            if (j >= 0 && inst_of(j) != k) {
                msg = "internal error: a tile mixes instances";
                return ST_INVALID;
            }
        if (batch) o.tile_inst.push_back(k);
        while ((int64_t)o.inst_tile.size() <= (int64_t)k) o.inst_tile.push_back((int64_t)t);
        if ((int64_t)o.inst_tile.size() != (int64_t)k + 1) {
            msg = "internal error: tiles not ordered by instance";
            return ST_INVALID;
        }
    }
    while ((int64_t)o.inst_tile.size() <= ilp.n_inst()) o.inst_tile.push_back((int64_t)plans.size());
    if (batch) {
        o.row_inst = row_inst;
        o.var_inst.resize((size_t)V);
        for (int64_t k = 0; k < ilp.n_inst(); ++k)
            for (int64_t i = ilp.inst_var[k]; i < ilp.inst_var[k + 1]; ++i) o.var_inst[i] = (int32_t)k;
    }
    o.n_slots = slots;
    o.scratch_elems = scratch;
    // slots of every pair, and the padding variable id for unused slots
    const int64_t P = (int64_t)B.lay_var.size();
    o.pair_var.assign(slots, (int32_t)V);
    o.slot_of_pair.assign(P, -1);
    const int64_t n_plans = (int64_t)plans.size();
    parallel_ranges(n_plans, host_threads(n_plans), [&](int, int64_t a, int64_t b) {
        for (int64_t t = a; t < b; ++t) {
            const TilePlan &tp = plans[t];
            for (int l = 0; l < kLanes; ++l) {
                int64_t j = tp.lanes[l];
                if (j < 0) continue;
                for (int h = 0; h < k_of(j); ++h) {
                    int64_t slot = (int64_t)o.tiles[t].pair_base + (int64_t)h * kLanes + l;
                    int64_t pq = B.lay_off[j] + h;
                    o.pair_var[slot] = B.lay_var[pq];
                    o.slot_of_pair[pq] = slot;
                }
            }
        }
    });
    // variable -> slots in ascending row order (pairs are already in row
    // order): each thread owns a variable range and scans all pairs in order
    o.vptr.assign(V + 1, 0);
    for (int64_t i = 0; i < V; ++i) o.vptr[i + 1] = o.vptr[i] + p.deg[i];
    o.vslot.assign(P, 0);
    {
        const int vt = host_threads(P);
        const int64_t chunk = (V + vt - 1) / vt;
        parallel_ranges(vt, vt, [&](int t, int64_t, int64_t) {
            const int64_t v0 = std::min<int64_t>(V, t * chunk), v1 = std::min<int64_t>(V, v0 + chunk);
            const uint64_t span = (uint64_t)(v1 - v0);
            // write positions of the range's variables, plus one entry whose
            // writes (pairs of other ranges) land in a private dummy slot;
            // no branch on the variable
            std::vector<int64_t> fill((size_t)span + 1);
            for (int64_t v = v0; v < v1; ++v) fill[(size_t)(v - v0)] = o.vptr[v];
            int32_t dummy[1];
            for (int64_t q = 0; q < P; ++q) {
                const uint64_t d = (uint64_t)((int64_t)B.lay_var[q] - v0);
                const bool mine = d < span;
                int64_t &f = fill[mine ? d : span];
                int32_t *dst = mine ? o.vslot.data() + f : dummy;
                *dst = (int32_t)o.slot_of_pair[q];
                f += mine;
            }
        });
    }
    // source of every slot's averaged term
    std::vector<int32_t> tile_of_slot((size_t)slots);
    const int64_t n_tiles = (int64_t)o.tiles.size();
    parallel_ranges(n_tiles, host_threads(n_tiles), [&](int, int64_t a, int64_t b) {
        for (int64_t t = a; t < b; ++t)
            for (int64_t s = o.tiles[t].pair_base; s < (int64_t)o.tiles[t].pair_base + (int64_t)o.tiles[t].K * kLanes;
                 ++s)
                tile_of_slot[s] = (int32_t)t;
    });
    std::vector<uint16_t> code((size_t)slots, kCodeSelf);
    // a wide tile's BDDs run in different blocks, so no in-tile partner there
    std::vector<char> wide_tile(o.tiles.size(), 0);
    for (int32_t t : lists[LIST_WIDE]) wide_tile[t] = 1;
    o.gvars.clear();
    {
        // each thread codes a variable range (its slots are its own) and
        // lists its kernel-averaged variables; the lists join in order
        const int ct = host_threads(V);
        std::vector<std::vector<int32_t>> gv((size_t)ct);
        parallel_ranges(V, ct, [&](int t, int64_t v0, int64_t v1) {
            for (int64_t i = v0; i < v1; ++i) {
                const int32_t a = o.vptr[i], b = o.vptr[i + 1];
                if (a == b) continue;
                bool local = fast && b - a <= 2;
                if (local) {
                    const int32_t t2 = tile_of_slot[o.vslot[a]];
                    local = o.tiles[t2].K * kLanes < (int)kCodeSelf && tile_of_slot[o.vslot[b - 1]] == t2 &&
                            (b - a == 1 || !wide_tile[t2]);
                }
                if (!local) {
                    gv[(size_t)t].push_back((int32_t)i);
                    for (int32_t q = a; q < b; ++q) code[o.vslot[q]] = kCodeGlobal;
                } else if (b - a == 2) {
                    const int32_t base = (int32_t)o.tiles[tile_of_slot[o.vslot[a]]].pair_base;
                    code[o.vslot[a]] = (uint16_t)(o.vslot[a + 1] - base);
                    code[o.vslot[a + 1]] = (uint16_t)(o.vslot[a] - base);
                }
            }
        });
        for (auto &g : gv) o.gvars.insert(o.gvars.end(), g.begin(), g.end());
    }
    // bucket the kernel-averaged variables by |J_i|
    {
        std::vector<std::vector<int32_t>> by_deg(kEllMaxDeg + 1);
        for (int32_t v : o.gvars) {
            const int32_t d = o.vptr[v + 1] - o.vptr[v];
            by_deg[d <= kEllMaxDeg ? d : 0].push_back(v);
        }
        o.gbuckets.clear();
        o.gslot.clear();
        int32_t blocks = 0;
        for (int d = 1; d <= kEllMaxDeg + 1; ++d) {
            const int dd = d <= kEllMaxDeg ? d : 0;   // CSR bucket last
            const std::vector<int32_t> &vs = by_deg[dd];
            if (vs.empty()) continue;
            AvgBucket b{};
            b.deg = dd;
            b.count = (int32_t)vs.size();
            b.block_begin = blocks;
            b.base = (int64_t)o.gslot.size();
            if (dd == 0) {
                o.gslot.insert(o.gslot.end(), vs.begin(), vs.end());
            } else {
                o.gslot.resize(o.gslot.size() + (size_t)dd * vs.size());
                for (size_t i = 0; i < vs.size(); ++i)
                    for (int k = 0; k < dd; ++k)
                        o.gslot[b.base + (int64_t)k * b.count + (int64_t)i] = o.vslot[o.vptr[vs[i]] + k];
            }
            blocks += (b.count + 255) / 256;
            o.gbuckets.push_back(b);
        }
        o.gblocks = blocks;
    }
    // fused averaging (layout.hpp) when every kernel-averaged variable lies in
    // mixed register tiles of classes that support it at the value size
    // fuse_elem (0 = off) and has at most kGatherMaxDeg subproblems
    o.gmeta.clear();
    o.gsrc.clear();
    if (fuse_elem > 0 && !o.gvars.empty()) {
        std::vector<char> mixed(o.tiles.size(), 0);
        for (int ki = 0; ki < kNumKClasses; ++ki)
            if (fuse_class_ok(fuse_elem, kKClass[ki]))
                for (int32_t t : lists[mix_list(ki)]) mixed[t] = 1;
        bool ok = true;
        int64_t ne = 0;
        for (size_t k = 0; ok && k < o.gvars.size(); ++k) {
            const int32_t v = o.gvars[k], a = o.vptr[v], b = o.vptr[v + 1];
            ok = b - a <= kGatherMaxDeg;
            for (int32_t q = a; ok && q < b; ++q) ok = mixed[tile_of_slot[o.vslot[q]]] != 0;
            ne += b - a;
        }
        if (ok && ne < kGatherMaxEntries) {
            o.gmeta.assign((size_t)slots, 0u);
            o.gsrc.resize((size_t)ne);
            int64_t e = 0;
            for (int32_t v : o.gvars) {
                const int32_t a = o.vptr[v], deg = o.vptr[v + 1] - a;
                for (int32_t r = 0; r < deg; ++r) {
                    const int32_t sl = o.vslot[a + r];
                    o.gsrc[(size_t)(e + r)] = sl;
                    o.gmeta[(size_t)sl] = gather_meta((uint32_t)(e + r), (uint32_t)r, (uint32_t)deg);
                    o.tiles[tile_of_slot[sl]].flags |= TILE_GATHER;
                }
                e += deg;
            }
        }
    }
    // tiles with the same code pattern share one copy of it
    o.code.clear();
    std::unordered_multimap<uint64_t, uint32_t> code_seen;
    std::vector<uint64_t> code_hash((size_t)n_tiles);
    parallel_ranges(n_tiles, host_threads(n_tiles), [&](int, int64_t a, int64_t b) {
        for (int64_t t = a; t < b; ++t) {
            const size_t n = (size_t)o.tiles[t].K * kLanes;
            const uint16_t *blk = code.data() + o.tiles[t].pair_base;
            uint64_t h = mix64(0, n);
            for (size_t q = 0; q < n; ++q) h = mix64(h, blk[q]);
            code_hash[t] = h;
        }
    });
    for (int64_t t = 0; t < n_tiles; ++t) {
        TileDesc &d = o.tiles[t];
        const size_t n = (size_t)d.K * kLanes;
        const uint16_t *blk = code.data() + d.pair_base;
        const uint64_t h = code_hash[t];
        int64_t found = -1;
        auto range = code_seen.equal_range(h);
        for (auto it = range.first; it != range.second; ++it)
            if (it->second + n <= o.code.size() && std::equal(blk, blk + n, o.code.begin() + it->second)) {
                found = it->second;
                break;
            }
        if (found < 0) {
            found = (int64_t)o.code.size();
            o.code.insert(o.code.end(), blk, blk + n);
            code_seen.emplace(h, (uint32_t)found);
        }
        d.code_base = (uint32_t)found;
    }
    // partner offsets must point inside their own tile
    for (const TileDesc &d : o.tiles)
        for (uint32_t q = 0; q < (uint32_t)d.K * kLanes; ++q) {
            const uint16_t c = o.code[d.code_base + q];
            if (c < kCodeSelf && (uint32_t)c >= (uint32_t)d.K * kLanes) {
                msg = "internal error: averaging partner outside its tile";
                return ST_INVALID;
            }
        }
    return ST_OK;
}

namespace {

// offsets of every instance in each merged table (prefix sums)
struct MergeOff {
    int64_t v, r, nnz, p, s, t, c, l, k, sc, b;
};

int merge_offsets(const std::vector<Part> &parts, std::vector<MergeOff> &off, std::string &msg)
{
    const int64_t n = (int64_t)parts.size();
    off.assign((size_t)n + 1, MergeOff{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
    for (int64_t k = 0; k < n; ++k) {
        const Part &pt = parts[k];
        if (!pt.p || !pt.pk || pt.p->ilp.n_inst() != 1) {
            msg = "merge_instances: every part must be one compiled and packed instance";
            return ST_INVALID;
        }
        const Problem &p = *pt.p;
        const Packed &pk = *pt.pk;
        MergeOff o = off[k];
        o.v += p.ilp.n_vars;
        o.r += p.ilp.n_rows;
        o.nnz += (int64_t)p.ilp.col.size();
        o.p += (int64_t)p.pair_var.size();
        o.s += pk.n_slots;
        o.t += (int64_t)pk.tiles.size();
        o.c += (int64_t)pk.child.size();
        o.l += (int64_t)pk.layers.size();
        o.k += (int64_t)pk.code.size();
        o.sc += pk.scratch_elems;
        o.b += p.bdds.n_bdds();
        off[k + 1] = o;
    }
    const MergeOff &tot = off[n];
    if (tot.v >= INT32_MAX || tot.p >= INT32_MAX || tot.s >= INT32_MAX || tot.t >= INT32_MAX || tot.r >= INT32_MAX ||
        tot.c >= (int64_t)UINT32_MAX || tot.l >= (int64_t)UINT32_MAX || tot.k >= (int64_t)UINT32_MAX ||
        tot.sc >= (int64_t)UINT32_MAX) {
        msg = "batch too large for 32-bit indices";
        return ST_INVALID;
    }
    return ST_OK;
}

// averaging buckets of the batch: one per degree over all instances
// (variables in instance order), the CSR bucket last, as the packer orders
// them; at[d][k] = first entry of instance k in the merged bucket of degree d
struct BucketPlan {
    std::vector<AvgBucket> mb;
    std::vector<int64_t> of_deg;             // merged bucket of degree d, -1 if none
    std::vector<std::vector<int64_t>> at;
    int64_t gslot = 0;
    int32_t blocks = 0;
};

int bucket_plan(const std::vector<Part> &parts, BucketPlan &bp, std::string &msg)
{
    const int64_t n = (int64_t)parts.size();
    constexpr int kDegs = kEllMaxDeg + 1;
    bp.at.assign((size_t)kDegs, std::vector<int64_t>((size_t)n + 1, 0));
    for (int d = 0; d < kDegs; ++d)
        for (int64_t k = 0; k < n; ++k) {
            int64_t c = 0;
            for (const AvgBucket &bk : parts[k].pk->gbuckets)
                if (bk.deg == d) c += bk.count;
            bp.at[d][k + 1] = bp.at[d][k] + c;
        }
    bp.mb.clear();
    bp.of_deg.assign((size_t)kDegs, -1);
    bp.blocks = 0;
    bp.gslot = 0;
    for (int d = 1; d <= kEllMaxDeg + 1; ++d) {
        const int dd = d <= kEllMaxDeg ? d : 0;
        const int64_t count = bp.at[dd][n];
        if (count == 0) continue;
        if (count >= INT32_MAX) {
            msg = "batch too large for 32-bit indices";
            return ST_INVALID;
        }
        AvgBucket nb{};
        nb.deg = dd;
        nb.count = (int32_t)count;
        nb.block_begin = bp.blocks;
        nb.base = bp.gslot;
        bp.gslot += (int64_t)(dd ? dd : 1) * count;
        bp.blocks += (int32_t)((count + 255) / 256);
        bp.of_deg[dd] = (int64_t)bp.mb.size();
        bp.mb.push_back(nb);
    }
    return ST_OK;
}

int merge_impl(const std::vector<Part> &parts, Problem &P, Packed &O, std::vector<int64_t> &slot_off, bool big,
               MergedSizes *sz, std::string &msg)
{
    P = Problem();
    O = Packed();
    const int64_t n = (int64_t)parts.size();
    std::vector<MergeOff> off;
    int rc = merge_offsets(parts, off, msg);
    if (rc != ST_OK) return rc;
    const MergeOff &tot = off[n];
    const int64_t V = tot.v, S = tot.s;
    slot_off.resize((size_t)n);
    for (int64_t k = 0; k < n; ++k) slot_off[k] = off[k].s;
    const bool batch = n > 1;
    BucketPlan bp;
    if ((rc = bucket_plan(parts, bp, msg)) != ST_OK) return rc;
    const std::vector<AvgBucket> &mb = bp.mb;
    const std::vector<int64_t> &bucket_of_deg = bp.of_deg;
    const std::vector<std::vector<int64_t>> &at = bp.at;
    O.gblocks = bp.blocks;
    if (big) O.gslot.resize((size_t)bp.gslot);
    O.gbuckets = mb;
    // sizes
    Ilp &U = P.ilp;
    U.n_vars = V;
    U.n_rows = tot.r;
    if (big) {
        U.cost.resize((size_t)V);
        U.row_ptr.resize((size_t)tot.r + 1);
        U.row_ptr[0] = 0;
        U.col.resize((size_t)tot.nnz);
        U.coef.resize((size_t)tot.nnz);
        U.sense.resize((size_t)tot.r);
        U.rhs.resize((size_t)tot.r);
    }
    U.inst_var.resize((size_t)n + 1);
    U.inst_row.resize((size_t)n + 1);
    for (int64_t k = 0; k <= n; ++k) {
        U.inst_var[k] = off[k].v;
        U.inst_row[k] = off[k].r;
    }
    // the merged problem carries the row ids of its BDDs only: the diagrams
    // themselves live in the tiles' node words
    P.bdds.lay_off.assign(1, 0);
    P.bdds.node_off.assign(1, 0);
    P.inst_offset.resize((size_t)n);
    O.tiles.resize((size_t)tot.t);
    O.inst_tile.resize((size_t)n + 1);
    for (int64_t k = 0; k <= n; ++k) O.inst_tile[k] = off[k].t;
    if (batch) O.tile_inst.resize((size_t)tot.t);
    std::vector<int64_t> gv_off((size_t)n + 1, 0);
    for (int64_t k = 0; k < n; ++k) gv_off[k + 1] = gv_off[k] + (int64_t)parts[k].pk->gvars.size();
    if (big) {
        P.fixed.resize((size_t)V);
        P.deg.resize((size_t)V);
        P.bdds.row.resize((size_t)tot.b);
        P.pair_var.resize((size_t)tot.p);
        P.pair_row.resize((size_t)tot.p);
        O.layers.resize((size_t)tot.l);
        O.child.resize((size_t)tot.c);
        O.code.resize((size_t)tot.k);
        O.pair_var.resize((size_t)S);
        O.slot_of_pair.resize((size_t)tot.p);
        O.vptr.resize((size_t)V + 1);
        O.vptr[0] = 0;
        O.vslot.resize((size_t)tot.p);
        O.gvars.resize((size_t)gv_off[n]);
        if (batch) {
            O.var_inst.resize((size_t)V);
            O.row_inst.resize((size_t)tot.r);
        }
    } else if (sz) {
        sz->pairs = tot.p;
        sz->code = tot.k;
        sz->gslot = bp.gslot;
        sz->child = tot.c;
        sz->layers = tot.l;
        sz->nnz = tot.nnz;
    }
    // fill: every instance writes its own disjoint ranges
    auto fill = [&](int64_t k) {
        const Problem &p = *parts[k].p;
        const Packed &pk = *parts[k].pk;
        const Ilp &il = p.ilp;
        const MergeOff &o = off[k];
        const int32_t nv = (int32_t)il.n_vars;
        P.inst_offset[k] = p.lb_offset;
        std::vector<char> glob(pk.tiles.size(), 0);
        for (int64_t q = pk.list_off[LIST_GEN_GLOB_ALL]; q < pk.list_off[LIST_GEN_GLOB_ALL + 1]; ++q)
            glob[(size_t)pk.lists[q]] = 1;
        for (size_t t = 0; t < pk.tiles.size(); ++t) {
            TileDesc d = pk.tiles[t];
            d.pair_base += (uint32_t)o.s;
            d.node_base += (uint32_t)o.c;
            d.fast_base += (uint32_t)o.c;
            d.layer_base += (uint32_t)o.l;
            d.code_base += (uint32_t)o.k;
            if (glob[t]) d.scratch_base += (uint32_t)o.sc;
            O.tiles[o.t + t] = d;
        }
        if (batch) std::fill(O.tile_inst.begin() + o.t, O.tile_inst.begin() + off[k + 1].t, (int32_t)k);
        if (!big) return;
        std::copy(il.cost.begin(), il.cost.end(), U.cost.begin() + o.v);
        for (int64_t r = 0; r < il.n_rows; ++r) U.row_ptr[o.r + r + 1] = o.nnz + il.row_ptr[r + 1];
        std::transform(il.col.begin(), il.col.end(), U.col.begin() + o.nnz,
                       [&](int32_t c) { return (int32_t)(c + o.v); });
        std::copy(il.coef.begin(), il.coef.end(), U.coef.begin() + o.nnz);
        std::copy(il.sense.begin(), il.sense.end(), U.sense.begin() + o.r);
        std::copy(il.rhs.begin(), il.rhs.end(), U.rhs.begin() + o.r);
        std::copy(p.fixed.begin(), p.fixed.end(), P.fixed.begin() + o.v);
        std::copy(p.deg.begin(), p.deg.end(), P.deg.begin() + o.v);
        std::transform(p.bdds.row.begin(), p.bdds.row.end(), P.bdds.row.begin() + o.b,
                       [&](int32_t r) { return (int32_t)(r + o.r); });
        std::transform(p.pair_var.begin(), p.pair_var.end(), P.pair_var.begin() + o.p,
                       [&](int32_t v) { return (int32_t)(v + o.v); });
        std::transform(p.pair_row.begin(), p.pair_row.end(), P.pair_row.begin() + o.p,
                       [&](int32_t r) { return (int32_t)(r + o.r); });
        std::copy(pk.layers.begin(), pk.layers.end(), O.layers.begin() + o.l);
        std::copy(pk.child.begin(), pk.child.end(), O.child.begin() + o.c);
        std::copy(pk.code.begin(), pk.code.end(), O.code.begin() + o.k);
        std::transform(pk.pair_var.begin(), pk.pair_var.end(), O.pair_var.begin() + o.s,
                       [&](int32_t v) { return v == nv ? (int32_t)V : (int32_t)(v + o.v); });
        std::transform(pk.slot_of_pair.begin(), pk.slot_of_pair.end(), O.slot_of_pair.begin() + o.p,
                       [&](int64_t sl) { return sl + o.s; });
        for (int64_t i = 0; i < il.n_vars; ++i) O.vptr[o.v + i + 1] = (int32_t)(o.p + pk.vptr[i + 1]);
        std::transform(pk.vslot.begin(), pk.vslot.end(), O.vslot.begin() + o.p,
                       [&](int32_t sl) { return (int32_t)(sl + o.s); });
        std::transform(pk.gvars.begin(), pk.gvars.end(), O.gvars.begin() + gv_off[k],
                       [&](int32_t v) { return (int32_t)(v + o.v); });
        for (const AvgBucket &bk : pk.gbuckets) {
            const AvgBucket &m = mb[(size_t)bucket_of_deg[bk.deg]];
            const int32_t *src = pk.gslot.data() + bk.base;
            const int64_t a0 = at[bk.deg][k];
            if (bk.deg == 0) {
                for (int32_t i = 0; i < bk.count; ++i) O.gslot[m.base + a0 + i] = (int32_t)(src[i] + o.v);
            } else {
                for (int kk = 0; kk < bk.deg; ++kk)
                    for (int32_t i = 0; i < bk.count; ++i)
                        O.gslot[m.base + (int64_t)kk * m.count + a0 + i] =
                            (int32_t)(src[(int64_t)kk * bk.count + i] + o.s);
            }
        }
        if (batch) {
            std::fill(O.var_inst.begin() + o.v, O.var_inst.begin() + off[k + 1].v, (int32_t)k);
            std::fill(O.row_inst.begin() + o.r, O.row_inst.begin() + off[k + 1].r, (int32_t)k);
        }
    };
    {
        unsigned hw = std::thread::hardware_concurrency();
        const int64_t nth = std::min<int64_t>(n, (int64_t)std::max(1u, std::min(hw ? hw : 1u, 16u)));
        if (nth <= 1 || !big || tot.s < (1 << 16)) {
            for (int64_t k = 0; k < n; ++k) fill(k);
        } else {
            // instances in descending size order over the threads
            std::vector<int64_t> order((size_t)n);
            for (int64_t k = 0; k < n; ++k) order[k] = k;
            std::sort(order.begin(), order.end(),
                      [&](int64_t x, int64_t y) { return off[x + 1].s - off[x].s > off[y + 1].s - off[y].s; });
            std::atomic<int64_t> next{0};
            run_threads((int)nth, [&](int) {
                for (int64_t q; (q = next.fetch_add(1)) < n;) fill(order[q]);
            });
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        const Problem &p = *parts[k].p;
        const Packed &pk = *parts[k].pk;
        P.lb_offset += p.lb_offset;
        P.n_nodes += p.n_nodes;
        P.n_fixed += p.n_fixed;
        P.n_free += p.n_free;
        O.max_lds_lane_elems = std::max(O.max_lds_lane_elems, pk.max_lds_lane_elems);
        O.max_wide_elems = std::max(O.max_wide_elems, pk.max_wide_elems);
        O.max_layers = std::max(O.max_layers, pk.max_layers);
        O.max_width = std::max(O.max_width, pk.max_width);
    }
    // lists: each class's tiles, instance by instance
    O.list_off.assign(kNumLists + 1, 0);
    for (int l = 0; l < kNumLists; ++l) {
        for (int64_t k = 0; k < n; ++k) {
            const Packed &pk = *parts[k].pk;
            for (int64_t q = pk.list_off[l]; q < pk.list_off[l + 1]; ++q)
                O.lists.push_back((int32_t)(pk.lists[q] + off[k].t));
        }
        O.list_off[l + 1] = (int64_t)O.lists.size();
    }
    O.n_slots = S;
    O.scratch_elems = tot.sc;
    // every tile inside the merged tables
    for (const TileDesc &d : O.tiles) {
        const uint64_t n64 = (uint64_t)d.K * kLanes;
        const uint64_t words = (uint64_t)d.nodes * ((d.flags & TILE_SHARED) ? 1u : (uint64_t)kLanes);
        if ((uint64_t)d.pair_base + n64 > (uint64_t)S || (uint64_t)d.code_base + n64 > (uint64_t)tot.k ||
            (uint64_t)d.layer_base + d.K > (uint64_t)tot.l || (uint64_t)d.node_base + words > (uint64_t)tot.c ||
            (uint64_t)d.fast_base + words > (uint64_t)tot.c) {
            msg = "internal error: merged tile outside its tables";
            return ST_INVALID;
        }
    }
    if (big && O.vptr.back() != tot.p) {
        msg = "internal error: inconsistent merged slot tables";
        return ST_INVALID;
    }
    return ST_OK;
}

}  // namespace

int merge_instances(const std::vector<Part> &parts, Problem &P, Packed &O, std::vector<int64_t> &slot_off,
                    std::string &msg)
{
    return merge_impl(parts, P, O, slot_off, true, nullptr, msg);
}

int merge_small(const std::vector<Part> &parts, Problem &P, Packed &O, std::vector<int64_t> &slot_off,
                MergedSizes &sz, std::string &msg)
{
    return merge_impl(parts, P, O, slot_off, false, &sz, msg);
}

TableSet image_layout(const Problem &p, const Packed &pk)
{
    TableSet t{};
    uint64_t o = 0;
    auto take = [&](int id, uint64_t bytes) {
        t.off[id] = o;
        o = (o + std::max<uint64_t>(bytes, 1) + 255) & ~uint64_t(255);
    };
    const Ilp &il = p.ilp;
    take(TB_PAIR_VAR, (uint64_t)pk.n_slots * 4);
    take(TB_VPTR, (uint64_t)(il.n_vars + 1) * 4);
    take(TB_VSLOT, pk.vslot.size() * 4);
    take(TB_CODE, pk.code.size() * 2);
    take(TB_GSLOT, pk.gslot.size() * 4);
    take(TB_CHILD, pk.child.size() * 4);
    take(TB_LAYERS, pk.layers.size() * 4);
    take(TB_COST, (uint64_t)il.n_vars * 8);
    take(TB_RPTR, (uint64_t)(il.n_rows + 1) * 8);
    take(TB_RCOL, il.col.size() * 4);
    take(TB_RCOEF, il.coef.size() * 4);
    take(TB_RSENSE, (uint64_t)il.n_rows);
    take(TB_RRHS, (uint64_t)il.n_rows * 8);
    take(TB_PRESET, (uint64_t)il.n_vars);
    t.off[TB_VAR_INST] = t.off[TB_ROW_INST] = o;   // instance ids are not part of an image
    t.bytes = o;
    return t;
}

void write_image(const Problem &p, const Packed &pk, const TableSet &ts, uint8_t *buf)
{
    const Ilp &il = p.ilp;
    auto put = [&](int id, const void *src, size_t bytes) {
        if (bytes) std::memcpy(buf + ts.off[id], src, bytes);
    };
    put(TB_PAIR_VAR, pk.pair_var.data(), pk.pair_var.size() * 4);
    put(TB_VPTR, pk.vptr.data(), pk.vptr.size() * 4);
    put(TB_VSLOT, pk.vslot.data(), pk.vslot.size() * 4);
    put(TB_CODE, pk.code.data(), pk.code.size() * 2);
    put(TB_GSLOT, pk.gslot.data(), pk.gslot.size() * 4);
    put(TB_CHILD, pk.child.data(), pk.child.size() * 4);
    put(TB_LAYERS, pk.layers.data(), pk.layers.size() * 4);
    put(TB_COST, il.cost.data(), il.cost.size() * 8);
    put(TB_RPTR, il.row_ptr.data(), il.row_ptr.size() * 8);
    put(TB_RCOL, il.col.data(), il.col.size() * 4);
    int32_t *coef = reinterpret_cast<int32_t *>(buf + ts.off[TB_RCOEF]);
    for (size_t e = 0; e < il.coef.size(); ++e) coef[e] = (int32_t)il.coef[e];
    put(TB_RSENSE, il.sense.data(), il.sense.size());
    put(TB_RRHS, il.rhs.data(), il.rhs.size() * 8);
    int8_t *pre = reinterpret_cast<int8_t *>(buf + ts.off[TB_PRESET]);
    for (int64_t i = 0; i < il.n_vars; ++i)
        pre[i] = p.fixed[i] >= 0 ? p.fixed[i] : p.deg[i] == 0 ? (int8_t)(il.cost[i] < 0.0 ? 1 : 0) : (int8_t)-1;
}

void assembly_segments(const std::vector<Part> &parts, const std::vector<uint64_t> &img, uint64_t dst_base,
                       const TableSet &dst, std::vector<Seg> &out)
{
    out.clear();
    std::vector<MergeOff> off;
    std::string msg;
    BucketPlan bp;
    if (merge_offsets(parts, off, msg) != ST_OK || bucket_plan(parts, bp, msg) != ST_OK) return;
    const int64_t n = (int64_t)parts.size();
    const int64_t V = off[n].v;
    auto seg = [&](uint64_t src, int id, int64_t at_elem, int64_t cnt, int32_t op, int32_t elem, int64_t a = 0,
                   int64_t b = 0, int64_t c = 0) {
        if (cnt <= 0) return;
        Seg g{};
        g.src = src;
        g.dst = dst_base + dst.off[id] + (uint64_t)at_elem * (uint64_t)elem;
        g.n = cnt;
        g.op = op;
        g.elem = elem;
        g.a = a;
        g.b = b;
        g.c = c;
        out.push_back(g);
    };
    seg(0, TB_VPTR, 0, 1, SEG_FILL, 4, 0);
    seg(0, TB_RPTR, 0, 1, SEG_FILL, 8, 0);
    for (int64_t k = 0; k < n; ++k) {
        const Problem &p = *parts[k].p;
        const Packed &pk = *parts[k].pk;
        const Ilp &il = p.ilp;
        const TableSet ts = image_layout(p, pk);
        const uint64_t b = img[k];
        const MergeOff &o = off[k];
        seg(b + ts.off[TB_PAIR_VAR], TB_PAIR_VAR, o.s, pk.n_slots, SEG_PADVAR, 4, o.v, il.n_vars, V);
        seg(b + ts.off[TB_VPTR] + 4, TB_VPTR, o.v + 1, il.n_vars, SEG_ADD, 4, o.p);
        seg(b + ts.off[TB_VSLOT], TB_VSLOT, o.p, (int64_t)pk.vslot.size(), SEG_ADD, 4, o.s);
        seg(b + ts.off[TB_CODE], TB_CODE, o.k, (int64_t)pk.code.size(), SEG_COPY, 2);
        for (const AvgBucket &bk : pk.gbuckets) {
            const AvgBucket &m = bp.mb[(size_t)bp.of_deg[bk.deg]];
            const int64_t a0 = bp.at[bk.deg][k];
            const uint64_t src = b + ts.off[TB_GSLOT] + (uint64_t)bk.base * 4;
            if (bk.deg == 0)
                seg(src, TB_GSLOT, m.base + a0, bk.count, SEG_ADD, 4, o.v);
            else
                for (int kk = 0; kk < bk.deg; ++kk)
                    seg(src + (uint64_t)kk * bk.count * 4, TB_GSLOT, m.base + (int64_t)kk * m.count + a0, bk.count,
                        SEG_ADD, 4, o.s);
        }
        seg(b + ts.off[TB_CHILD], TB_CHILD, o.c, (int64_t)pk.child.size(), SEG_COPY, 4);
        seg(b + ts.off[TB_LAYERS], TB_LAYERS, o.l, (int64_t)pk.layers.size(), SEG_COPY, 4);
        seg(b + ts.off[TB_COST], TB_COST, o.v, il.n_vars, SEG_COPY, 8);
        seg(b + ts.off[TB_RPTR] + 8, TB_RPTR, o.r + 1, il.n_rows, SEG_ADD, 8, o.nnz);
        seg(b + ts.off[TB_RCOL], TB_RCOL, o.nnz, (int64_t)il.col.size(), SEG_ADD, 4, o.v);
        seg(b + ts.off[TB_RCOEF], TB_RCOEF, o.nnz, (int64_t)il.coef.size(), SEG_COPY, 4);
        seg(b + ts.off[TB_RSENSE], TB_RSENSE, o.r, il.n_rows, SEG_COPY, 1);
        seg(b + ts.off[TB_RRHS], TB_RRHS, o.r, il.n_rows, SEG_COPY, 8);
        seg(b + ts.off[TB_PRESET], TB_PRESET, o.v, il.n_vars, SEG_COPY, 1);
        if (n > 1) {
            seg(0, TB_VAR_INST, o.v, il.n_vars, SEG_FILL, 4, k);
            seg(0, TB_ROW_INST, o.r, il.n_rows, SEG_FILL, 4, k);
        }
    }
}

int build_serial(const Problem &p, const Packed &pk, SerialTables &o, std::string &msg)
{
    const BddSet &B = p.bdds;
    const int64_t nb = B.n_bdds(), P = (int64_t)B.lay_var.size(), N = (int64_t)B.child.size();
    const int64_t V = p.ilp.n_vars;
    if (N >= INT32_MAX || P >= INT32_MAX || (int64_t)pk.slot_of_pair.size() != P) {
        msg = "serial tables: problem too large or not packed";
        return ST_INVALID;
    }
    o = SerialTables();
    o.child = B.child;
    o.pinfo.resize((size_t)(4 * P));
    o.bpair.resize((size_t)nb + 1);
    for (int64_t b = 0; b < nb; ++b) {
        o.bpair[b] = (int32_t)B.lay_off[b];
        int64_t node = B.node_off[b];
        for (int64_t q = B.lay_off[b]; q < B.lay_off[b + 1]; ++q) {
            const int64_t w = B.lay_width[q];
            o.pinfo[4 * q + 0] = (int32_t)node;
            o.pinfo[4 * q + 1] = (int32_t)w;
            o.pinfo[4 * q + 2] = q + 1 < B.lay_off[b + 1] ? (int32_t)(node + w) : -1;
            o.pinfo[4 * q + 3] = (int32_t)b;
            node += w;
        }
        if (node != B.node_off[b + 1]) {
            msg = "serial tables: inconsistent layer widths";
            return ST_INVALID;
        }
    }
    o.bpair[nb] = (int32_t)P;
    o.vptr.assign((size_t)V + 1, 0);
    for (int64_t q = 0; q < P; ++q) o.vptr[B.lay_var[q] + 1]++;
    for (int64_t i = 0; i < V; ++i) o.vptr[i + 1] += o.vptr[i];
    o.vpair.resize((size_t)P);
    {
        std::vector<int32_t> fill(o.vptr.begin(), o.vptr.end() - 1);
        for (int64_t q = 0; q < P; ++q) o.vpair[fill[B.lay_var[q]]++] = (int32_t)q;   // pairs ascend in row order
    }
    // levels: predecessors have smaller ids (forward), successors larger ones
    std::vector<int32_t> lf((size_t)V, -1), lb((size_t)V, -1);
    auto first = [&](int64_t q) { return q == (int64_t)o.bpair[o.pinfo[4 * q + 3]]; };
    for (int64_t i = 0; i < V; ++i)
        for (int32_t t = o.vptr[i]; t < o.vptr[i + 1]; ++t) {
            const int64_t q = o.vpair[t];
            lf[i] = std::max(lf[i], first(q) ? 0 : lf[B.lay_var[q - 1]] + 1);
        }
    for (int64_t i = V - 1; i >= 0; --i)
        for (int32_t t = o.vptr[i]; t < o.vptr[i + 1]; ++t) {
            const int64_t q = o.vpair[t];
            lb[i] = std::max(lb[i], o.pinfo[4 * q + 2] < 0 ? 0 : lb[B.lay_var[q + 1]] + 1);
        }
    auto csr = [&](const std::vector<int32_t> &lev, std::vector<int32_t> &ptr, std::vector<int32_t> &var) {
        int32_t nl = 0;
        for (int32_t l : lev) nl = std::max(nl, l + 1);
        ptr.assign((size_t)nl + 1, 0);
        for (int32_t l : lev)
            if (l >= 0) ptr[l + 1]++;
        for (int32_t l = 0; l < nl; ++l) ptr[l + 1] += ptr[l];
        var.resize((size_t)ptr[nl]);
        std::vector<int32_t> f(ptr.begin(), ptr.end() - 1);
        for (int64_t i = 0; i < V; ++i)
            if (lev[i] >= 0) var[f[lev[i]]++] = (int32_t)i;
    };
    csr(lf, o.lf_ptr, o.lf_var);
    csr(lb, o.lb_ptr, o.lb_var);
    o.slot.resize((size_t)P);
    for (int64_t q = 0; q < P; ++q) o.slot[q] = (int32_t)pk.slot_of_pair[q];
    return ST_OK;
}

int encode_wide_rows(const Ilp &in, int64_t max_states, Ilp &o, int64_t &n_encoded, std::string &msg)
{
    if (max_states < 2) {
        msg = "max_states must be >= 2";
        return ST_INVALID;
    }
    const int64_t n = in.n_vars;
    n_encoded = 0;
    // which rows need the encoding
    std::vector<char> enc((size_t)in.n_rows, 0);
    for (int64_t r = 0; r < in.n_rows; ++r) {
        const int64_t k = in.row_ptr[r + 1] - in.row_ptr[r];
        __int128 mag = 0;
        for (int64_t e = in.row_ptr[r]; e < in.row_ptr[r + 1]; ++e) mag += in.coef[e] < 0 ? -in.coef[e] : in.coef[e];
        const bool few = k < 62 && ((int64_t)1 << k) <= max_states;
        enc[r] = !few && mag + 1 > (__int128)max_states;
        n_encoded += enc[r];
    }
    o = Ilp();
    o.cost = in.cost;
    o.row_ptr.assign(1, 0);
    int64_t nv = n;
    auto add_row = [&](const std::vector<std::pair<int32_t, int64_t>> &t, int sense, int64_t b) {
        std::vector<std::pair<int32_t, int64_t>> s(t);
        std::sort(s.begin(), s.end());
        for (auto &pr : s) {
            o.col.push_back(pr.first);
            o.coef.push_back(pr.second);
        }
        o.row_ptr.push_back((int64_t)o.col.size());
        o.sense.push_back((int8_t)sense);
        o.rhs.push_back(b);
    };
    auto new_var = [&]() {
        o.cost.push_back(0.0);
        return (int32_t)nv++;
    };
    std::vector<int32_t> comp((size_t)n, -1);   // complement of x_i, created on first use
    for (int64_t r = 0; r < in.n_rows; ++r) {
        std::vector<std::pair<int32_t, int64_t>> t;
        for (int64_t e = in.row_ptr[r]; e < in.row_ptr[r + 1]; ++e) t.emplace_back(in.col[e], in.coef[e]);
        if (!enc[r]) {
            add_row(t, in.sense[r], in.rhs[r]);
            continue;
        }
        // positive weights over x or its complement
        std::vector<std::pair<int32_t, int64_t>> w;
        int64_t B = in.rhs[r], total = 0;
        for (auto &pr : t) {
            if (pr.second > 0) {
                w.push_back(pr);
            } else {
                int32_t &c = comp[pr.first];
                if (c < 0) {
                    c = new_var();
                    add_row({{pr.first, 1}, {c, 1}}, 0, 1);
                }
                w.emplace_back(c, -pr.second);
                B += -pr.second;
            }
            total += w.back().second;
            if (total >= ((int64_t)1 << 30)) {
                msg = "row " + std::to_string(r) + ": weight sum too large to encode";
                return ST_INVALID;
            }
        }
        // L columns cover the total weight; the carry out of column k is at
        // most floor(sum_i (w_i mod 2^(k+1)) / 2^(k+1)), which is 0 after the
        // last column since the total is below 2^L
        int L = 1;
        while (((int64_t)1 << L) <= total) ++L;
        std::vector<int64_t> maxc((size_t)L);
        for (int k = 0; k < L; ++k) {
            int64_t low = 0;
            for (auto &pr : w) low += pr.second & (((int64_t)1 << (k + 1)) - 1);
            maxc[k] = low >> (k + 1);
        }
        // ids: sum bits from the most significant down, then carry bits
        std::vector<int32_t> sbit((size_t)L);
        for (int k = L - 1; k >= 0; --k) sbit[k] = new_var();
        std::vector<std::vector<int32_t>> cbits((size_t)L);
        for (int k = 0; k < L; ++k)
            for (int j = 0; ((int64_t)1 << j) <= maxc[k]; ++j) cbits[k].push_back(new_var());
        for (int k = 0; k < L; ++k) {
            std::vector<std::pair<int32_t, int64_t>> row;
            for (auto &pr : w)
                if ((pr.second >> k) & 1) row.emplace_back(pr.first, 1);
            if (k > 0)
                for (size_t j = 0; j < cbits[k - 1].size(); ++j) row.emplace_back(cbits[k - 1][j], (int64_t)1 << j);
            row.emplace_back(sbit[k], -1);
            for (size_t j = 0; j < cbits[k].size(); ++j) row.emplace_back(cbits[k][j], -((int64_t)1 << (j + 1)));
            add_row(row, 0, 0);
        }
        const int K = L;
        std::vector<std::pair<int32_t, int64_t>> cmp;
        for (int k = 0; k < K; ++k) cmp.emplace_back(sbit[k], (int64_t)1 << k);
        add_row(cmp, in.sense[r], B);
        if (maxc[K - 1] != 0) {
            msg = "internal error: adder network leaves a carry";
            return ST_INVALID;
        }
    }
    o.n_vars = nv;
    o.n_rows = (int64_t)o.sense.size();
    o.inst_var = {0, nv};
    o.inst_row = {0, o.n_rows};
    if (nv >= INT32_MAX) {
        msg = "encoding needs too many variables";
        return ST_INVALID;
    }
    return ST_OK;
}

}  // namespace bddmma
