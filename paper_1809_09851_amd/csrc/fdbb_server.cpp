// Native request server (declared in include/fdbb_server.h): a scheduler
// thread admits queued requests in arrival order while a launch slot is free
// and their outputs fit in a device arena of the budget's size, packs them
// into one persistent batch launch per slot (a direct launch of the slot's
// plan, with the server's batch configuration and the LDS its list
// stages), and retires them when the slot's completion event fires.  Outputs
// live in the arena until the caller releases them.
#include "../../include/fdbb_server.h"

#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/fdbb.h"
#include "free_list.hpp"

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// After its last activity the scheduler polls for this long before it
// sleeps, so that a request arriving soon after is picked up at once.
constexpr int64_t kSpinNs = 200000;

size_t elem_size(int dtype) { return dtype == FDBB_F64 ? 8 : 4; }

// Output layout of a task: sizes in elements of each output slot, and the
// leading dimension the server gives them (n padded to 64 points).
struct OutShape {
    int64_t ld = 0;
    size_t bytes[3] = {0, 0, 0};
};

bool out_shape(const fdbb_task &t, OutShape *s)
{
    const int64_t D = t.dim, K = D + 2;
    const int64_t ld = std::max<int64_t>(64, (t.n + 63) / 64 * 64);
    const size_t es = elem_size(t.dtype);
    s->ld = ld;
    switch (t.op) {
    case FDBB_OP_CONS2PRIM:
    case FDBB_OP_PRIM2CONS:
    case FDBB_OP_CONS2CHAR:
    case FDBB_OP_CHAR2CONS:
    case FDBB_OP_ADJOINT:
    case FDBB_OP_ROE_AVERAGE:
    case FDBB_OP_FLUX_DIR: s->bytes[0] = (size_t)(K * ld) * es; return true;
    case FDBB_OP_FLUX: s->bytes[0] = (size_t)(K * D * ld) * es; return true;
    case FDBB_OP_RIEMANN: s->bytes[0] = (size_t)((2 * D + 1) * ld) * es; return true;
    case FDBB_OP_FLUX_JACOBIAN: s->bytes[0] = (size_t)(D * ld * K * K) * es; return true;
    case FDBB_OP_V_MAG2: s->bytes[0] = (size_t)ld * es; return true;
    case FDBB_OP_EOS:
        s->bytes[0] = (size_t)ld * es;
        s->bytes[1] = (size_t)ld * es;
        return true;
    case FDBB_OP_FUSED:
        s->bytes[0] = (size_t)(K * D * ld) * es;
        s->bytes[1] = (size_t)(D * ld * K * K) * es;
        s->bytes[2] = (size_t)((2 * D + 1) * ld) * es;
        return true;
    default: return false;
    }
}

// HBM bytes one task moves (inputs read once, outputs written once).
double moved_bytes(const fdbb_task &t)
{
    const double D = t.dim, K = D + 2, n = (double)t.n, es = (double)elem_size(t.dtype);
    double per = 0;
    switch (t.op) {
    case FDBB_OP_CONS2PRIM:
    case FDBB_OP_PRIM2CONS:
    case FDBB_OP_CONS2CHAR:
    case FDBB_OP_CHAR2CONS:
    case FDBB_OP_FLUX_DIR: per = 2 * K; break;
    case FDBB_OP_ADJOINT: per = K * K; break;
    case FDBB_OP_ROE_AVERAGE: per = 3 * K; break;
    case FDBB_OP_FLUX: per = K + K * D; break;
    case FDBB_OP_RIEMANN: per = K + 2 * D + 1; break;
    case FDBB_OP_FLUX_JACOBIAN: per = K + D * K * K; break;
    case FDBB_OP_V_MAG2: per = D + 2; break;
    case FDBB_OP_EOS: per = K + 2; break;
    case FDBB_OP_FUSED: per = K + K * D + D * K * K + 2 * D + 1; break;
    default: break;
    }
    return per * n * es;
}

// One device allocation of the budget's size, carved by a first-fit free
// list (free_list.hpp).
class Arena {
public:
    int init(size_t bytes)
    {
        list_.reset(bytes);
        if (hipMalloc(&base_, list_.size()) != hipSuccess) {
            base_ = nullptr;
            return FDBB_ENOMEM;
        }
        return FDBB_OK;
    }
    void release_all()
    {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
    }
    // offset of a block of `bytes`, or SIZE_MAX when nothing fits
    size_t alloc(size_t bytes) { return list_.alloc(bytes); }
    void free(size_t off, size_t bytes) { list_.release(off, bytes); }
    unsigned char *ptr(size_t off) const { return static_cast<unsigned char *>(base_) + off; }
    size_t used() const { return list_.used(); }
    size_t size() const { return list_.size(); }

private:
    void *base_ = nullptr;
    fdbb::FreeList list_;
};

struct Request {
    fdbb_task task;
    uint64_t tag;
    int64_t t_submit, t_admit = 0, t_done = 0;
    size_t off[3] = {SIZE_MAX, SIZE_MAX, SIZE_MAX};
    size_t bytes[3] = {0, 0, 0};
};

struct Slot {
    hipStream_t stream = nullptr;  // shared by every slot in single mode
    hipEvent_t done = nullptr;
    fdbb_batch_plan *plan = nullptr;
    std::vector<Request> batch;
    bool busy = false;
    int launch_rc = 0;
};

}  // namespace

struct fdbb_server {
    int device = 0;
    int mode = FDBB_SERVE_BATCHED;
    int max_batch = 64;
    double max_batch_bytes = 0;
    Arena arena;
    std::vector<Slot> slots;
    hipStream_t single_stream = nullptr;

    std::mutex mu;  // guards queue, completed, outputs, stats and the arena
    std::condition_variable cv;
    std::deque<Request> queue;
    std::deque<fdbb_completion> completed;
    std::unordered_map<uint64_t, Request> outstanding;  // completed, not yet released
    std::unordered_set<uint64_t> live;                  // tags submitted, not yet released
    fdbb_server_stats stats{};
    bool kick = false;  // set by submit and release: wakes a sleeping scheduler
    std::atomic<bool> stop{false};
    std::thread worker;
    std::string error;
};

namespace {

void fill_outputs(fdbb_server *s, Request &r)
{
    OutShape sh;
    out_shape(r.task, &sh);
    void *p[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < 3; ++k)
        if (r.bytes[k]) p[k] = s->arena.ptr(r.off[k]);
    r.task.out0 = p[0];
    r.task.out1 = p[1];
    r.task.out2 = p[2];
    r.task.ld_out0 = r.task.ld_out1 = r.task.ld_out2 = sh.ld;
}

// Admit, oldest first, what fits; returns false when the head of the queue
// is waiting for memory.  Caller holds s->mu.
bool take_batch(fdbb_server *s, std::vector<Request> &batch)
{
    double moved = 0;
    while (!s->queue.empty() && (int)batch.size() < s->max_batch) {
        Request &r = s->queue.front();
        const double m = moved_bytes(r.task);
        if (!batch.empty() && moved + m > s->max_batch_bytes) break;
        bool ok = true;
        for (int k = 0; k < 3 && ok; ++k) {
            if (!r.bytes[k]) continue;
            r.off[k] = s->arena.alloc(r.bytes[k]);
            if (r.off[k] == SIZE_MAX) ok = false;
        }
        if (!ok) {  // give back what this request got and wait for memory
            for (int k = 0; k < 3; ++k)
                if (r.bytes[k] && r.off[k] != SIZE_MAX) {
                    s->arena.free(r.off[k], r.bytes[k]);
                    r.off[k] = SIZE_MAX;
                }
            break;
        }
        fill_outputs(s, r);
        moved += m;
        batch.push_back(r);
        s->queue.pop_front();
    }
    s->stats.peak_arena_bytes = std::max<int64_t>(s->stats.peak_arena_bytes, (int64_t)s->arena.used());
    return !batch.empty();
}

int launch(fdbb_server *s, Slot &slot)
{
    std::vector<fdbb_task> tasks;
    tasks.reserve(slot.batch.size());
    for (const Request &r : slot.batch) tasks.push_back(r.task);
    int rc = FDBB_OK;
    if (s->mode == FDBB_SERVE_SINGLE || tasks.size() == 1) {
        for (const fdbb_task &t : tasks)
            if ((rc = fdbb_task_run(&t, slot.stream))) break;
    } else {
        rc = fdbb_batch_plan_update(slot.plan, tasks.data(), (int)tasks.size(), slot.stream);
        if (!rc) rc = fdbb_batch_exec(slot.plan, slot.stream, 0);
    }
    if (!rc && hipEventRecord(slot.done, slot.stream) != hipSuccess) rc = FDBB_EHIP;
    return rc;
}

void run_loop(fdbb_server *s)
{
    (void)hipSetDevice(s->device);
    // sleeps below are short; ask for them to be honoured to the microsecond
    (void)prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    int64_t last_active = now_ns();
    while (!s->stop.load(std::memory_order_relaxed)) {
        bool progressed = false, any_busy = false;
        // retire finished slots
        for (Slot &slot : s->slots) {
            if (!slot.busy) continue;
            const hipError_t q = hipEventQuery(slot.done);
            if (q == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            const int64_t t = now_ns();
            std::lock_guard<std::mutex> lock(s->mu);
            for (Request &r : slot.batch) {
                r.t_done = t;
                fdbb_completion c{};
                c.tag = r.tag;
                c.status = (q == hipSuccess && slot.launch_rc == FDBB_OK) ? FDBB_OK : FDBB_EHIP;
                c.out0 = r.task.out0, c.out1 = r.task.out1, c.out2 = r.task.out2;
                c.ld = r.task.ld_out0;
                c.t_submit_ns = r.t_submit, c.t_admit_ns = r.t_admit, c.t_done_ns = r.t_done;
                s->completed.push_back(c);
                s->outstanding.emplace(r.tag, r);
                s->stats.completed += 1;
            }
            slot.batch.clear();
            slot.busy = false;
            progressed = true;
        }
        // admit into free slots
        for (Slot &slot : s->slots) {
            if (slot.busy) continue;
            {
                std::lock_guard<std::mutex> lock(s->mu);
                if (s->queue.empty() || !take_batch(s, slot.batch)) break;
                const int64_t t = now_ns();
                for (Request &r : slot.batch) r.t_admit = t;
                s->stats.launches += 1;
            }
            slot.launch_rc = launch(s, slot);
            if (slot.launch_rc) {
                std::lock_guard<std::mutex> lock(s->mu);
                s->error = std::string("launch failed: ") + fdbb_last_error();
                s->stats.errors += 1;
            }
            slot.busy = true;  // the event (or its failure) retires the batch
            any_busy = true;
            progressed = true;
        }
        const int64_t now = now_ns();
        if (progressed || any_busy) {
            // launches in flight: poll their events without sleeping
            if (progressed) last_active = now;
            std::this_thread::yield();
            continue;
        }
        if (now - last_active < kSpinNs) {
            // recently active: a next arrival is likely soon
            std::this_thread::yield();
            continue;
        }
        // idle, or the queue head waits for memory: sleep until a
        // submission or a release (both notify), re-checking now and then
        std::unique_lock<std::mutex> lock(s->mu);
        s->cv.wait_for(lock, std::chrono::microseconds(500), [s] { return s->kick || s->stop.load(); });
        s->kick = false;
    }
}

}  // namespace

extern "C" {

int fdbb_server_create(int64_t budget_bytes, int slots, int max_batch, double max_batch_bytes, int mode,
                       fdbb_server **out)
{
    if (!out) return FDBB_EINVAL;
    *out = nullptr;
    if (budget_bytes <= 0 || slots < 1 || slots > 64 || max_batch < 1 || !(max_batch_bytes > 0) ||
        (mode != FDBB_SERVE_BATCHED && mode != FDBB_SERVE_SINGLE))
        return FDBB_EINVAL;
    fdbb_server *s = new fdbb_server();
    (void)hipGetDevice(&s->device);
    s->mode = mode;
    s->max_batch = mode == FDBB_SERVE_SINGLE ? 1 : max_batch;
    s->max_batch_bytes = max_batch_bytes;
    int rc = s->arena.init((size_t)budget_bytes);
    if (rc) {
        delete s;
        return rc;
    }
    if (mode == FDBB_SERVE_SINGLE && hipStreamCreateWithFlags(&s->single_stream, hipStreamNonBlocking) != hipSuccess) {
        fdbb_server_destroy(s);
        return FDBB_EHIP;
    }
    // Batched launches take the server's batch configuration (its grid sized
    // to this device) and reserve LDS for any task; each launch is direct,
    // with the LDS its own task list stages.
    int block = 0, ppt = 0, grid_per_cu = 0, nt = 0, cus = 0;
    if (mode == FDBB_SERVE_BATCHED) {
        fdbb_get_server_batch_config(&block, &ppt, &grid_per_cu, &nt);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess) {
            fdbb_server_destroy(s);
            return FDBB_EHIP;
        }
    }
    const int grid = cus * (grid_per_cu > 0 ? grid_per_cu : std::max(1, 2048 / std::max(1, block)));
    s->slots.resize(slots);
    for (Slot &slot : s->slots) {
        if (mode == FDBB_SERVE_SINGLE) slot.stream = s->single_stream;
        else if (hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking) != hipSuccess) {
            fdbb_server_destroy(s);
            return FDBB_EHIP;
        }
        if (hipEventCreateWithFlags(&slot.done, hipEventDisableTiming) != hipSuccess) {
            fdbb_server_destroy(s);
            return FDBB_EHIP;
        }
        if (mode == FDBB_SERVE_BATCHED &&
            (rc = fdbb_batch_plan_create(nullptr, 0, std::max(1, max_batch), block, ppt, grid, nt, &slot.plan))) {
            fdbb_server_destroy(s);
            return rc;
        }
    }
    s->worker = std::thread(run_loop, s);
    *out = s;
    return FDBB_OK;
}

int fdbb_server_submit(fdbb_server *s, const fdbb_task *task, uint64_t tag)
{
    if (!s || !task) return FDBB_EINVAL;
    Request r;
    r.task = *task;
    r.tag = tag;
    OutShape sh;
    if (!out_shape(r.task, &sh) || task->op == FDBB_OP_EIGENVECTORS || task->op == FDBB_OP_CHAR_APPLY)
        return FDBB_EINVAL;
    size_t total = 0;
    for (int k = 0; k < 3; ++k) {
        r.bytes[k] = sh.bytes[k];
        total += sh.bytes[k];
    }
    // validate now, so that errors reach the caller: the outputs get
    // placeholder addresses in a range no device allocation uses (above
    // 2^56), where they can only overlap each other, which they do not
    fdbb_task probe = r.task;
    const uintptr_t base = (uintptr_t)1 << 56;
    probe.out0 = sh.bytes[0] ? (void *)base : nullptr;
    probe.out1 = sh.bytes[1] ? (void *)(base + sh.bytes[0] + 4096) : nullptr;
    probe.out2 = sh.bytes[2] ? (void *)(base + sh.bytes[0] + sh.bytes[1] + 8192) : nullptr;
    probe.ld_out0 = probe.ld_out1 = probe.ld_out2 = sh.ld;
    if (const int rc = fdbb_task_check(&probe)) return rc;
    if (total > s->arena.size()) return FDBB_ENOMEM;
    r.t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lock(s->mu);
        if (!s->live.insert(tag).second) return FDBB_EINVAL;
        s->queue.push_back(r);
        s->stats.submitted += 1;
        s->kick = true;
    }
    s->cv.notify_one();
    return FDBB_OK;
}

int fdbb_server_poll(fdbb_server *s, fdbb_completion *out, int max, int *count)
{
    if (!s || (!out && max > 0) || !count) return FDBB_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    int k = 0;
    while (k < max && !s->completed.empty()) {
        out[k++] = s->completed.front();
        s->completed.pop_front();
    }
    *count = k;
    return FDBB_OK;
}

int fdbb_server_release(fdbb_server *s, uint64_t tag)
{
    if (!s) return FDBB_EINVAL;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->outstanding.find(tag);
        if (it == s->outstanding.end()) return FDBB_EINVAL;
        for (int k = 0; k < 3; ++k)
            if (it->second.bytes[k]) s->arena.free(it->second.off[k], it->second.bytes[k]);
        s->outstanding.erase(it);
        s->live.erase(tag);
        s->kick = true;
    }
    s->cv.notify_one();
    return FDBB_OK;
}

int fdbb_server_get_stats(fdbb_server *s, fdbb_server_stats *out)
{
    if (!s || !out) return FDBB_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->stats;
    out->arena_bytes = (int64_t)s->arena.used();
    out->queued = (int64_t)s->queue.size();
    return FDBB_OK;
}

int fdbb_server_destroy(fdbb_server *s)
{
    if (!s) return FDBB_OK;
    s->stop.store(true);
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (Slot &slot : s->slots) {
        if (slot.stream) (void)hipStreamSynchronize(slot.stream);
        if (slot.plan) fdbb_batch_plan_destroy(slot.plan);
        if (slot.done) (void)hipEventDestroy(slot.done);
        if (slot.stream && slot.stream != s->single_stream) (void)hipStreamDestroy(slot.stream);
    }
    if (s->single_stream) (void)hipStreamDestroy(s->single_stream);
    s->arena.release_all();
    delete s;
    return FDBB_OK;
}

}  // extern "C"
