// Serving pool: continuous batching of independent instances.  Instances are
// compiled on host worker threads, which then write each instance's table
// image and upload it into the pool's arena, each on a stream of its own,
// while the resident batch keeps running (when image space is free;
// otherwise the image goes up at admission); an instance whose upload is
// still running joins at a later step instead of holding the batch up.  The
// resident batch is the solver's batch (every step of the method runs in its
// kernels), re-assembled on the device from the member images whenever
// membership changes, with the members' dual state carried over device to
// device.
//
// Arena: [copy descriptors | member images | batch half A | batch half B].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "bddmma.h"
#include "solver_internal.hpp"

using namespace bddmma;

namespace {

enum ImgState { IMG_NONE = 0, IMG_UPLOADING = 1, IMG_RESIDENT = 2 };

struct Inst {
    int32_t state = BDDMMA_POOL_QUEUED;
    int32_t error = 0;
    int32_t iters = 0, n_iter = 0;
    int64_t steps = 0;
    double lb_free = NAN, lb_cert = NAN, res = NAN;
    size_t bytes = 0;
    int64_t n_vars = 0, n_pairs = 0;
    bddmma_solver *s = nullptr;     // the instance alone: loaded, never bound
    bddmma_solver *pre = nullptr;   // handed over loaded by the caller, not yet checked
    int64_t slot_off = -1;          // first slot in the resident batch (-1: not in it)
    uint64_t img_size = 0;          // bytes of its table image
    int64_t img_off = -1;           // image offset in the image region (-1: none)
    int img = IMG_NONE;
    std::vector<double> lam, mm;    // terminated multipliers and M at retirement
    int32_t rounded = 0, round_status = 0, rounds = 0;   // Alg. 2 at retirement
    double ub = NAN;
    std::vector<uint8_t> x;         // its point (round_status OK)
    // input, until compiled
    int64_t nv = 0, nr = 0;
    std::vector<double> cost;
    std::vector<int64_t> row_ptr, rhs;
    std::vector<int32_t> col, coef;
    std::vector<int8_t> sense;
};

constexpr double kNaN = std::numeric_limits<double>::quiet_NaN();
constexpr size_t kAsmBytes = 8u << 20;   // copy descriptors of one assembly
constexpr size_t kPoolPinBytes = 1u << 20; // pinned readback buffer lent to the batches

double ms_since(std::chrono::steady_clock::time_point t)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

}  // namespace

struct bddmma_pool {
    bddmma_options opt{};
    int32_t max_active = 1;
    bool keep_multipliers = true;
    bool round = false;             // Alg. 2 for retiring members
    std::mutex mu;
    std::condition_variable cv_job, cv_idle, cv_img;
    std::deque<Inst *> jobs;
    int64_t pending = 0;            // jobs queued or running (compilations and image uploads)
    bool stop = false;
    std::vector<std::thread> workers;
    std::map<int64_t, std::unique_ptr<Inst>> inst;   // by ticket (submission order)
    int64_t next_ticket = 1;
    std::vector<int64_t> members;   // tickets of the resident batch, in batch order
    bool changed = false;           // membership differs from the assembled batch
    char *arena = nullptr;
    char *asm_area = nullptr;       // copy descriptors
    char *img_area = nullptr;       // member images
    size_t img_cap = 0;
    std::map<uint64_t, uint64_t> img_free;   // free image blocks: offset -> bytes
    char *halves = nullptr;
    size_t half = 0;
    int side = 0;                   // arena half holding the assembled batch
    hipStream_t st = nullptr;       // the caller's stream: every batch launch
    void *pin = nullptr;            // pinned host buffer lent to every batch for its readbacks
    bddmma_solver *batch = nullptr;
    bool bound = false;
    bddmma_pool_counters cnt{};
};

namespace {

#define POOL_GUARD_BEGIN try {
#define POOL_GUARD_END                                                                            \
    }                                                                                             \
    catch (const std::bad_alloc &) { return set_error(BDDMMA_ERR_NO_MEMORY, "host allocation failed"); } \
    catch (const std::exception &ex) { return set_error(BDDMMA_ERR_INVALID_ARG, ex.what()); }            \
    catch (...) { return set_error(BDDMMA_ERR_INVALID_ARG, "unexpected error"); }

uint64_t img_blocks(uint64_t bytes) { return (std::max<uint64_t>(bytes, 1) + 255) & ~uint64_t(255); }

// first fit in the image region; -1 when nothing fits (lock held)
int64_t img_alloc(bddmma_pool *p, uint64_t bytes)
{
    bytes = img_blocks(bytes);
    for (auto it = p->img_free.begin(); it != p->img_free.end(); ++it)
        if (it->second >= bytes) {
            const uint64_t at = it->first, left = it->second - bytes;
            p->img_free.erase(it);
            if (left) p->img_free.emplace(at + bytes, left);
            return (int64_t)at;
        }
    return -1;
}

// return an instance's image space, merging free neighbours (lock held)
void img_release(bddmma_pool *p, Inst *in)
{
    in->img = IMG_NONE;
    if (in->img_off < 0) return;
    uint64_t at = (uint64_t)in->img_off, bytes = img_blocks(in->img_size);
    in->img_off = -1;
    auto nx = p->img_free.lower_bound(at);
    if (nx != p->img_free.end() && at + bytes == nx->first) {
        bytes += nx->second;
        nx = p->img_free.erase(nx);
    }
    if (nx != p->img_free.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == at) {
            pv->second += bytes;
            return;
        }
    }
    p->img_free.emplace(at, bytes);
}

// a compiled (or failed) instance becomes READY (FAILED); lock held
void settle(Inst *in, int rc, bddmma_solver *s)
{
    if (rc == BDDMMA_OK) {
        size_t bytes = 0;
        bddmma_stats stt{};
        rc = bddmma_workspace_bytes(s, &bytes);
        if (rc == BDDMMA_OK) rc = bddmma_get_stats(s, &stt);
        if (rc == BDDMMA_OK) {
            in->s = s;
            in->bytes = bytes;
            in->n_vars = stt.n_vars;
            in->n_pairs = stt.n_pairs;
            in->img_size = solver_image_bytes(s);
            in->state = BDDMMA_POOL_READY;
        }
    }
    if (rc != BDDMMA_OK) {
        bddmma_destroy(s);
        in->s = nullptr;
        in->state = BDDMMA_POOL_FAILED;
        in->error = rc;
    }
    in->cost = {};
    in->row_ptr = {};
    in->rhs = {};
    in->col = {};
    in->coef = {};
    in->sense = {};
}

// image space for a READY instance without one, if it fits now (lock held):
// the caller then uploads it
bool claim_image(bddmma_pool *p, Inst *in)
{
    if (!p->bound || in->state != BDDMMA_POOL_READY || in->img != IMG_NONE || in->img_size > p->img_cap) return false;
    const int64_t at = img_alloc(p, in->img_size);
    if (at < 0) return false;
    in->img_off = at;
    in->img = IMG_UPLOADING;
    return true;
}

// write the image of `in` into buf and upload it on `st` (no lock; the
// instance is UPLOADING, which keeps it and its image space in place)
int upload_image(bddmma_pool *p, Inst *in, hipStream_t st, std::vector<uint8_t> &buf)
{
    int rc = solver_image(in->s, buf);
    if (rc) return rc;
    if (!buf.empty() &&
        hipMemcpyAsync(p->img_area + in->img_off, buf.data(), buf.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        return set_error(BDDMMA_ERR_HIP, "image upload failed");
    if (hipStreamSynchronize(st) != hipSuccess) return set_error(BDDMMA_ERR_HIP, "image upload failed");
    return BDDMMA_OK;
}

void worker(bddmma_pool *p)
{
    hipStream_t up_st = nullptr;   // this worker's upload stream (default priority)
    std::vector<uint8_t> buf;      // image staging, reused
    for (;;) {
        Inst *in;
        {
            std::unique_lock<std::mutex> lk(p->mu);
            p->cv_job.wait(lk, [&] { return p->stop || !p->jobs.empty(); });
            if (p->stop) {
                lk.unlock();
                if (up_st) (void)hipStreamDestroy(up_st);
                return;
            }
            in = p->jobs.front();
            p->jobs.pop_front();
        }
        // a queued or uploading instance is neither released nor admitted,
        // and the pool joins its workers before freeing anything, so `in`
        // stays valid without the lock
        bool up = false;
        if (in->state == BDDMMA_POOL_QUEUED) {
            bddmma_solver *s = in->pre;
            int rc = BDDMMA_OK;
            if (s) {
                in->pre = nullptr;
                int64_t ni = 0;
                rc = bddmma_num_instances(s, &ni);
                if (!rc && ni != 1) rc = set_error(BDDMMA_ERR_INVALID_ARG, "a pool instance must be a single ILP");
                if (!rc && solver_precision(s) != p->opt.precision)
                    rc = set_error(BDDMMA_ERR_INVALID_ARG, "instance precision differs from the pool's");
            } else {
                rc = bddmma_create(&p->opt, &s);
                if (rc == BDDMMA_OK)
                    rc = bddmma_load_ilp(s, in->nv, in->cost.data(), in->nr, in->row_ptr.data(), in->col.data(),
                                         in->coef.data(), in->sense.data(), in->rhs.data());
            }
            std::lock_guard<std::mutex> lk(p->mu);
            settle(in, rc, s);
            up = claim_image(p, in);
        } else {
            up = true;   // an upload job: image space already claimed
        }
        if (up) {
            int rc = BDDMMA_OK;
            if (!up_st && hipStreamCreateWithFlags(&up_st, hipStreamNonBlocking) != hipSuccess) {
                up_st = nullptr;
                rc = set_error(BDDMMA_ERR_HIP, "upload stream creation failed");
            }
            if (!rc) rc = upload_image(p, in, up_st, buf);
            std::lock_guard<std::mutex> lk(p->mu);
            if (rc) img_release(p, in);   // admission uploads it again
            else in->img = IMG_RESIDENT;
            p->cv_img.notify_all();
        }
        std::lock_guard<std::mutex> lk(p->mu);
        if (--p->pending == 0) p->cv_idle.notify_all();
    }
}

// hand image uploads of READY instances to the workers while space is free
// (lock held)
void prefetch_images(bddmma_pool *p)
{
    for (auto &kv : p->inst) {
        Inst *in = kv.second.get();
        if (in->state != BDDMMA_POOL_READY || in->img != IMG_NONE) continue;
        if (!claim_image(p, in)) break;
        p->jobs.push_back(in);
        p->pending++;
        p->cv_job.notify_one();
    }
}

// Build the batch of the current members in the other arena half and carry
// the dual state of continuing members over.
int reassemble(bddmma_pool *p)
{
    std::vector<const bddmma_solver *> parts;
    std::vector<Inst *> mem;
    std::vector<uint64_t> img, img_bytes;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        for (int64_t t : p->members) {
            Inst *in = p->inst.at(t).get();
            mem.push_back(in);
            parts.push_back(in->s);
            img.push_back((uint64_t)(uintptr_t)(p->img_area + in->img_off));
            img_bytes.push_back(in->img_size);
        }
    }
    bddmma_options o = p->opt;
    o.rel_tol = 0.0;   // the pool applies the tolerance per member
    bddmma_solver *nb = nullptr;
    int rc = bddmma_create(&o, &nb);
    if (rc) return rc;
    if (p->pin) solver_lend_pinned(nb, p->pin, kPoolPinBytes);
    std::vector<int64_t> off;
    size_t need = 0;
    auto t0 = std::chrono::steady_clock::now();
    rc = solver_load_virtual(nb, parts, off);
    p->cnt.merge_ms += ms_since(t0);
    t0 = std::chrono::steady_clock::now();
    if (!rc) rc = bddmma_workspace_bytes(nb, &need);
    if (!rc && need > p->half) rc = set_error(BDDMMA_ERR_NO_MEMORY, "resident batch exceeds its half of the pool arena");
    if (!rc)
        rc = solver_bind_assembled(nb, p->halves + (size_t)(p->side ^ 1) * p->half, p->half, p->st, parts, img,
                                   img_bytes, p->asm_area, kAsmBytes);
    for (size_t k = 0; !rc && k < mem.size(); ++k)
        if (p->batch && mem[k]->slot_off >= 0)
            rc = solver_copy_slots(nb, off[k], p->batch, mem[k]->slot_off, solver_slots(mem[k]->s));
    if (!rc && hipStreamSynchronize(p->st) != hipSuccess) rc = set_error(BDDMMA_ERR_HIP, "pool stream synchronise failed");
    if (rc) {
        bddmma_destroy(nb);
        return rc;
    }
    bddmma_destroy(p->batch);
    p->batch = nb;
    p->side ^= 1;
    p->cnt.bind_ms += ms_since(t0);
    p->cnt.assemblies++;
    std::lock_guard<std::mutex> lk(p->mu);
    for (size_t k = 0; k < mem.size(); ++k) mem[k]->slot_off = off[k];
    p->changed = false;
    return BDDMMA_OK;
}

// Alg. 2 for the retiring members mem[ret[.]]: a batch of only them,
// assembled from their images in the free arena half with their state copied
// from the resident batch (which gives each the result of its solo run).
int round_members(bddmma_pool *p, const std::vector<Inst *> &mem, const std::vector<size_t> &ret)
{
    std::vector<const bddmma_solver *> parts;
    std::vector<uint64_t> img, img_bytes;
    std::vector<int64_t> voff(1, 0);
    for (size_t k : ret) {
        const Inst *in = mem[k];
        parts.push_back(in->s);
        img.push_back((uint64_t)(uintptr_t)(p->img_area + in->img_off));
        img_bytes.push_back(in->img_size);
        voff.push_back(voff.back() + in->n_vars);
    }
    bddmma_options o = p->opt;
    o.rel_tol = 0.0;
    bddmma_solver *rb = nullptr;
    int rc = bddmma_create(&o, &rb);
    if (rc) return rc;
    if (p->pin) solver_lend_pinned(rb, p->pin, kPoolPinBytes);
    std::vector<int64_t> off;
    size_t need = 0;
    rc = solver_load_virtual(rb, parts, off);
    if (!rc) rc = bddmma_workspace_bytes(rb, &need);
    if (!rc && need > p->half) rc = set_error(BDDMMA_ERR_NO_MEMORY, "rounding batch exceeds half of the pool arena");
    if (!rc)
        rc = solver_bind_assembled(rb, p->halves + (size_t)(p->side ^ 1) * p->half, p->half, p->st, parts, img,
                                   img_bytes, p->asm_area, kAsmBytes);
    for (size_t q = 0; !rc && q < ret.size(); ++q)
        rc = solver_copy_slots(rb, off[q], p->batch, mem[ret[q]]->slot_off, solver_slots(parts[q]));
    const size_t n = ret.size();
    std::vector<uint8_t> x((size_t)std::max<int64_t>(voff.back(), 1));
    std::vector<double> ub(n);
    std::vector<int32_t> rounds(n), status(n);
    if (!rc) rc = bddmma_batch_round(rb, x.data(), ub.data(), rounds.data(), status.data());
    bddmma_destroy(rb);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(p->mu);
    for (size_t q = 0; q < n; ++q) {
        Inst *in = mem[ret[q]];
        in->rounded = 1;
        in->round_status = status[q];
        in->rounds = rounds[q];
        if (status[q] == BDDMMA_OK) {
            in->ub = ub[q];
            in->x.assign(x.begin() + voff[q], x.begin() + voff[q + 1]);
        }
    }
    return BDDMMA_OK;
}

int enqueue(bddmma_pool *p, std::unique_ptr<Inst> in, int64_t *ticket)
{
    std::lock_guard<std::mutex> lk(p->mu);
    const int64_t t = p->next_ticket++;
    p->jobs.push_back(in.get());
    p->pending++;
    p->inst.emplace(t, std::move(in));
    *ticket = t;
    p->cv_job.notify_one();
    return BDDMMA_OK;
}

}  // namespace

extern "C" {

int bddmma_pool_create(const bddmma_options *opt, int32_t max_active, int32_t host_threads, int32_t flags,
                       bddmma_pool **out)
{
    POOL_GUARD_BEGIN
    if (!out) return set_error(BDDMMA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (max_active < 1) return set_error(BDDMMA_ERR_INVALID_ARG, "max_active must be >= 1");
    if (host_threads < 0) return set_error(BDDMMA_ERR_INVALID_ARG, "host_threads must be >= 0");
    if (flags & ~(BDDMMA_POOL_KEEP_MULTIPLIERS | BDDMMA_POOL_ROUND))
        return set_error(BDDMMA_ERR_INVALID_ARG, "unknown pool flags");
    bddmma_options o;
    if (opt) o = *opt;
    else bddmma_options_default(&o);
    // validate the options once, as bddmma_create does
    bddmma_solver *probe = nullptr;
    int rc = bddmma_create(&o, &probe);
    if (rc) return rc;
    bddmma_destroy(probe);
    std::unique_ptr<bddmma_pool> p(new bddmma_pool());
    p->opt = o;
    p->max_active = max_active;
    p->keep_multipliers = (flags & BDDMMA_POOL_KEEP_MULTIPLIERS) != 0;
    p->round = (flags & BDDMMA_POOL_ROUND) != 0;
    unsigned hw = std::thread::hardware_concurrency();
    int n = host_threads > 0 ? host_threads : (int)std::max(1u, std::min(hw ? hw : 1u, 8u));
    for (int i = 0; i < n; ++i) p->workers.emplace_back(worker, p.get());
    *out = p.release();
    return BDDMMA_OK;
    POOL_GUARD_END
}

int bddmma_pool_bind(bddmma_pool *p, void *dev_ptr, size_t bytes, void *hip_stream)
{
    if (!p) return set_error(BDDMMA_ERR_INVALID_ARG, "pool is NULL");
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->bound) return set_error(BDDMMA_ERR_STATE, "pool arena already bound");
    if (!dev_ptr) return set_error(BDDMMA_ERR_INVALID_ARG, "device pointer is NULL");
    if (((uintptr_t)dev_ptr) % 256) return set_error(BDDMMA_ERR_INVALID_ARG, "device pointer must be 256-byte aligned");
    if (bytes < kAsmBytes + 3 * 1024) return set_error(BDDMMA_ERR_NO_MEMORY, "pool arena too small");
    const size_t rest = bytes - kAsmBytes;
    const size_t img_cap = (rest / 3) & ~(size_t)255;
    const size_t half = ((rest - img_cap) / 2) & ~(size_t)255;
    p->arena = (char *)dev_ptr;
    p->asm_area = p->arena;
    p->img_area = p->arena + kAsmBytes;
    p->img_cap = img_cap;
    p->img_free.clear();
    p->img_free.emplace(0, img_cap);
    p->halves = p->img_area + img_cap;
    p->half = half;
    p->st = (hipStream_t)hip_stream;
    p->bound = true;
    if (!p->pin && hipHostMalloc(&p->pin, kPoolPinBytes, hipHostMallocDefault) != hipSuccess) {
        p->pin = nullptr;   // the batches then read back through pageable memory
        (void)hipGetLastError();
    }
    prefetch_images(p);
    return BDDMMA_OK;
}

int bddmma_pool_submit(bddmma_pool *p, int64_t n_vars, const double *costs, int64_t n_rows, const int64_t *row_ptr,
                       const int32_t *col, const int32_t *coef, const int8_t *sense, const int64_t *rhs,
                       int32_t n_iter, int64_t *ticket)
{
    POOL_GUARD_BEGIN
    if (!p || !ticket) return set_error(BDDMMA_ERR_INVALID_ARG, "NULL argument");
    if (n_iter < 1) return set_error(BDDMMA_ERR_INVALID_ARG, "n_iter must be >= 1");
    if (n_vars < 0 || n_rows < 0 || (n_vars > 0 && !costs) || !row_ptr || (n_rows > 0 && (!sense || !rhs)))
        return set_error(BDDMMA_ERR_INVALID_ARG, "bad ILP arrays");
    const int64_t nnz = row_ptr[n_rows];
    if (nnz < 0 || (nnz > 0 && (!col || !coef))) return set_error(BDDMMA_ERR_INVALID_ARG, "bad ILP arrays");
    std::unique_ptr<Inst> in(new Inst());
    in->n_iter = n_iter;
    in->nv = n_vars;
    in->nr = n_rows;
    in->cost.assign(costs, costs + n_vars);
    in->row_ptr.assign(row_ptr, row_ptr + n_rows + 1);
    in->col.assign(col, col + nnz);
    in->coef.assign(coef, coef + nnz);
    in->sense.assign(sense, sense + n_rows);
    in->rhs.assign(rhs, rhs + n_rows);
    return enqueue(p, std::move(in), ticket);
    POOL_GUARD_END
}

int bddmma_pool_submit_loaded(bddmma_pool *p, bddmma_solver *s, int32_t n_iter, int64_t *ticket)
{
    POOL_GUARD_BEGIN
    if (!p || !s || !ticket) {
        bddmma_destroy(s);
        return set_error(BDDMMA_ERR_INVALID_ARG, "NULL argument");
    }
    if (n_iter < 1) {
        bddmma_destroy(s);
        return set_error(BDDMMA_ERR_INVALID_ARG, "n_iter must be >= 1");
    }
    std::unique_ptr<Inst> in(new Inst());
    in->n_iter = n_iter;
    in->pre = s;
    return enqueue(p, std::move(in), ticket);
    POOL_GUARD_END
}

int bddmma_pool_wait_compiled(bddmma_pool *p)
{
    if (!p) return set_error(BDDMMA_ERR_INVALID_ARG, "pool is NULL");
    std::unique_lock<std::mutex> lk(p->mu);
    p->cv_idle.wait(lk, [&] { return p->pending == 0; });
    return BDDMMA_OK;
}

int bddmma_pool_step(bddmma_pool *p, int32_t iters, int32_t *n_active, int32_t *n_retired)
{
    POOL_GUARD_BEGIN
    if (!p) return set_error(BDDMMA_ERR_INVALID_ARG, "pool is NULL");
    if (!p->bound) return set_error(BDDMMA_ERR_STATE, "no pool arena bound");
    if (iters < 1) return set_error(BDDMMA_ERR_INVALID_ARG, "iters must be >= 1");
    if (n_active) *n_active = 0;
    if (n_retired) *n_retired = 0;
    std::vector<Inst *> fresh;   // admitted without an uploaded image: it goes up now
    auto ti = std::chrono::steady_clock::now();
    {
        // admission in submission order while the batch fits
        std::unique_lock<std::mutex> lk(p->mu);
        size_t used = 0;
        for (int64_t t : p->members) used += p->inst.at(t)->bytes;
        for (auto &kv : p->inst) {
            Inst *in = kv.second.get();
            if (in->state != BDDMMA_POOL_READY) continue;
            if (in->bytes > p->half || in->img_size > p->img_cap) {
                p->cv_img.wait(lk, [&] { return in->img != IMG_UPLOADING; });
                img_release(p, in);
                bddmma_destroy(in->s);
                in->s = nullptr;
                in->state = BDDMMA_POOL_FAILED;
                in->error = BDDMMA_ERR_NO_MEMORY;
                continue;
            }
            if ((int32_t)p->members.size() >= p->max_active || used + in->bytes > p->half) break;
            if (in->img == IMG_UPLOADING) continue;   // joins once its image is up
            if (in->img == IMG_NONE) {
                if (!claim_image(p, in)) break;
                fresh.push_back(in);
            }
            in->state = BDDMMA_POOL_ACTIVE;
            in->slot_off = -1;
            p->cnt.admitted++;
            used += in->bytes;
            p->members.push_back(kv.first);
            p->changed = true;
        }
        if (p->members.empty()) {
            bddmma_destroy(p->batch);
            p->batch = nullptr;
            p->changed = false;
            return BDDMMA_OK;
        }
    }
    int rc;
    std::vector<uint8_t> buf;
    for (Inst *in : fresh) {
        if ((rc = upload_image(p, in, p->st, buf))) return rc;
        std::lock_guard<std::mutex> lk(p->mu);
        in->img = IMG_RESIDENT;
    }
    p->cnt.image_ms += ms_since(ti);
    if ((p->changed || !p->batch) && (rc = reassemble(p))) return rc;
    std::vector<Inst *> mem;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        for (int64_t t : p->members) mem.push_back(p->inst.at(t).get());
    }
    // a step ends early where a member would otherwise run past its count
    int32_t run = iters;
    for (Inst *in : mem) run = std::min(run, in->n_iter - in->iters);
    auto t0 = std::chrono::steady_clock::now();
    if ((rc = bddmma_run_dual(p->batch, run, nullptr))) return rc;
    p->cnt.run_ms += ms_since(t0);
    t0 = std::chrono::steady_clock::now();
    const size_t n = p->members.size();
    std::vector<double> lbf(n), lbc(n, NAN), res(n, NAN);
    if ((rc = bddmma_batch_bounds(p->batch, lbf.data(), nullptr, nullptr))) return rc;   // lb_free only
    p->cnt.bounds_ms += ms_since(t0);
    p->cnt.steps++;
    std::vector<char> done(n, 0);
    for (size_t k = 0; k < n; ++k) {
        Inst *in = mem[k];
        const bool flat = p->opt.rel_tol > 0.0 && in->steps >= 1 &&
                          std::fabs(lbf[k] - in->lb_free) <= p->opt.rel_tol * std::max(1.0, std::fabs(lbf[k]));
        done[k] = in->iters + run >= in->n_iter || flat;
    }
    // the certified bound and the residual of the retiring members (one
    // certificate pass over the batch, only on steps where someone retires)
    if (std::find(done.begin(), done.end(), 1) != done.end()) {
        const auto tc = std::chrono::steady_clock::now();
        if ((rc = bddmma_batch_bounds(p->batch, nullptr, lbc.data(), res.data()))) return rc;
        p->cnt.bounds_ms += ms_since(tc);
    }
    t0 = std::chrono::steady_clock::now();
    for (size_t k = 0; k < n; ++k) {
        Inst *in = mem[k];
        if (done[k] && p->keep_multipliers) {
            std::vector<double> lam((size_t)in->n_pairs), mm((size_t)in->n_pairs);
            if ((rc = solver_instance_multipliers(p->batch, in->slot_off, in->s, lam.data(), mm.data()))) return rc;
            std::lock_guard<std::mutex> lk(p->mu);
            in->lam.swap(lam);
            in->mm.swap(mm);
        }
    }
    if (p->round) {
        std::vector<size_t> ret;
        for (size_t k = 0; k < n; ++k)
            if (done[k]) ret.push_back(k);
        if (!ret.empty()) {
            auto tr = std::chrono::steady_clock::now();
            if ((rc = round_members(p, mem, ret))) return rc;
            p->cnt.round_ms += ms_since(tr);
        }
    }
    std::lock_guard<std::mutex> lk(p->mu);
    std::vector<int64_t> keep;
    int32_t retired = 0;
    for (size_t k = 0; k < n; ++k) {
        Inst *in = mem[k];
        in->iters += run;
        in->steps++;
        in->lb_free = lbf[k];
        if (done[k]) {
            in->lb_cert = lbc[k];
            in->res = res[k];
        }
        if (done[k]) {
            in->state = BDDMMA_POOL_DONE;
            in->slot_off = -1;
            img_release(p, in);
            ++retired;
            p->changed = true;
        } else {
            keep.push_back(p->members[k]);
        }
    }
    p->members.swap(keep);
    p->cnt.retired += retired;
    p->cnt.retire_ms += ms_since(t0);
    // freed image space goes to the next instances waiting for admission
    if (retired) prefetch_images(p);
    if (n_active) *n_active = (int32_t)p->members.size();
    if (n_retired) *n_retired = retired;
    return BDDMMA_OK;
    POOL_GUARD_END
}

int bddmma_pool_poll(bddmma_pool *p, int64_t ticket, bddmma_pool_info *info)
{
    if (!p || !info) return set_error(BDDMMA_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->inst.find(ticket);
    if (it == p->inst.end()) return set_error(BDDMMA_ERR_INVALID_ARG, "unknown ticket");
    const Inst &in = *it->second;
    *info = bddmma_pool_info{};
    info->state = in.state;
    info->error = in.error;
    info->iters = in.iters;
    info->n_iter = in.n_iter;
    info->n_vars = in.n_vars;
    info->n_pairs = in.n_pairs;
    info->steps = in.steps;
    info->lb_free = in.steps ? in.lb_free : kNaN;
    info->lb_cert = in.steps ? in.lb_cert : kNaN;
    info->max_residual = in.steps ? in.res : kNaN;
    info->workspace_bytes = in.bytes;
    info->rounded = in.rounded;
    info->round_status = in.round_status;
    info->rounds = in.rounds;
    info->ub = in.ub;
    return BDDMMA_OK;
}

int bddmma_pool_primal(bddmma_pool *p, int64_t ticket, uint8_t *x_out)
{
    if (!p || !x_out) return set_error(BDDMMA_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->inst.find(ticket);
    if (it == p->inst.end()) return set_error(BDDMMA_ERR_INVALID_ARG, "unknown ticket");
    const Inst &in = *it->second;
    if (in.state != BDDMMA_POOL_DONE || !in.rounded || in.round_status != BDDMMA_OK)
        return set_error(BDDMMA_ERR_STATE, "no rounded point (retire with BDDMMA_POOL_ROUND and a converged Alg. 2)");
    std::copy(in.x.begin(), in.x.end(), x_out);
    return BDDMMA_OK;
}

int bddmma_pool_result(bddmma_pool *p, int64_t ticket, double *lambda, double *mm, int32_t *pair_var,
                       int32_t *pair_row)
{
    POOL_GUARD_BEGIN
    if (!p) return set_error(BDDMMA_ERR_INVALID_ARG, "pool is NULL");
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->inst.find(ticket);
    if (it == p->inst.end()) return set_error(BDDMMA_ERR_INVALID_ARG, "unknown ticket");
    const Inst &in = *it->second;
    if (in.state != BDDMMA_POOL_DONE) return set_error(BDDMMA_ERR_STATE, "instance not retired");
    if ((lambda || mm) && !p->keep_multipliers)
        return set_error(BDDMMA_ERR_STATE, "the pool keeps no multipliers (no BDDMMA_POOL_KEEP_MULTIPLIERS)");
    if (lambda) std::copy(in.lam.begin(), in.lam.end(), lambda);
    if (mm) std::copy(in.mm.begin(), in.mm.end(), mm);
    if (pair_var || pair_row) {
        std::vector<int32_t> pv((size_t)in.n_pairs), pr((size_t)in.n_pairs);
        int rc = bddmma_get_pairs(in.s, pv.data(), pr.data());
        if (rc) return rc;
        if (pair_var) std::copy(pv.begin(), pv.end(), pair_var);
        if (pair_row) std::copy(pr.begin(), pr.end(), pair_row);
    }
    return BDDMMA_OK;
    POOL_GUARD_END
}

int bddmma_pool_get_counters(bddmma_pool *p, bddmma_pool_counters *out)
{
    if (!p || !out) return set_error(BDDMMA_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(p->mu);
    *out = p->cnt;
    out->batch_capacity = p->half;
    out->image_capacity = p->img_cap;
    out->image_free = 0;
    for (auto &kv : p->img_free) out->image_free += kv.second;
    return BDDMMA_OK;
}

int bddmma_pool_release(bddmma_pool *p, int64_t ticket)
{
    if (!p) return set_error(BDDMMA_ERR_INVALID_ARG, "pool is NULL");
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->inst.find(ticket);
    if (it == p->inst.end()) return set_error(BDDMMA_ERR_INVALID_ARG, "unknown ticket");
    Inst &in = *it->second;
    if (in.state != BDDMMA_POOL_DONE && in.state != BDDMMA_POOL_FAILED)
        return set_error(BDDMMA_ERR_STATE, "only retired or failed instances can be released");
    bddmma_destroy(in.s);
    p->inst.erase(it);
    return BDDMMA_OK;
}

void bddmma_pool_destroy(bddmma_pool *p)
{
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->stop = true;
    }
    p->cv_job.notify_all();
    for (auto &w : p->workers) w.join();
    if (p->bound && p->st) (void)hipStreamSynchronize(p->st);
    bddmma_destroy(p->batch);
    for (auto &kv : p->inst) {
        bddmma_destroy(kv.second->s);
        bddmma_destroy(kv.second->pre);
    }
    if (p->pin) (void)hipHostFree(p->pin);
    delete p;
}

}  // extern "C"
