// Serving loop for IRK step-solve requests (continuous batching on one GPU).
//
// Requests (operator, tableau, dt, number of steps, initial field) are
// queued FIFO and admitted as soon as a slot is free and their resident
// state -- the solver workspace (stage vectors, Krylov bases, multigrid
// hierarchies) plus two state fields -- fits in the caller's device arena.
// Admitted requests stay resident until their last step; every running
// request is a non-blocking step state machine on its slot's HIP streams,
// and one progress pass advances all of them, so requests that arrive while
// others run start as soon as memory and a slot free up and their kernels
// overlap on the device.  Slots (streams, events, pinned staging) are made
// when the server is created: admitting a request only enqueues work (the
// u0 copy, the context's table uploads) and a finished request is retired
// when an event behind all of its work has completed, so no progress pass
// waits for the device.  Arithmetic is exactly that of irk_step on the same
// problem (same kernels, deterministic reductions), so a request's result
// does not depend on what else is running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "irk_internal.h"
#include "mg_tiled.h"

namespace irk {
irk_status step_begin(irk_ctx *c, const double *u_n, double t_n, double dt, double tol, double *u_np1);
int step_poll(irk_ctx *c, irk_status *st, irk_stats *stats);
void *res_new(int nlanes, size_t upload);
void res_free(void *r);
size_t res_upload_need(int family, int s, const irk_operator *op, const irk_options *opt);
irk_status create_in_res(int family, int s, const irk_operator *op, const irk_options *opt, void *ws,
                         size_t ws_bytes, hipStream_t stream, void *res, irk_ctx **out);
irk_status record_all_done(irk_ctx *c, hipEvent_t ev);
void ctx_free(irk_ctx *c);
void *broker_create(int fp32);
void broker_destroy(void *b, int fp32);
int broker_flush(void *b, int fp32);
bool attach_broker(irk_ctx *c, void *fp32_broker, void *fp64_broker);
}  // namespace irk

namespace {

double now_s() {
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    return std::chrono::duration<double>(clk::now() - t0).count();
}

// First-fit allocator over the caller's device arena (256-byte granules,
// free blocks coalesced on release).
class Arena {
  public:
    void init(size_t base_bytes) {
        free_.clear();
        free_[0] = base_bytes;
        cap_ = base_bytes;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0;
};

// A slot: the Newton-level stream and the resource set (block streams,
// events, pinned staging) one admitted request runs on, made when the server
// is created so that admitting a request allocates nothing and waits for
// nothing.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t fin = nullptr;                 // behind all of a finishing request's work
    void *res = nullptr;
    bool busy = false;
};

// largest grid side and eigen-blocks a slot's staging and streams cover
constexpr int kSlotMaxSide = 16384;
constexpr int kSlotLanes = 3;                 // eigen-blocks of s <= 5
// pinned upload area: forcing tables 2 (nx + ny) and the exactly solved
// Poisson level's basis and eigenvalues
constexpr size_t kSlotUpload = (size_t)4 * kSlotMaxSide + (size_t)IRK_FDM_MAX * IRK_FDM_MAX + IRK_FDM_MAX;

struct Req {
    long id = 0;
    irk_request r;
    irk_request_info info;
    size_t ws_bytes = 0, field_bytes = 0, off = 0, total = 0;
    bool allocated = false;
    irk_ctx *ctx = nullptr;
    int slot = -1;
    hipStream_t stream = nullptr;             // the slot's stream
    hipEvent_t u0_ready = nullptr;            // recorded on the caller's stream at submit
    double *ua = nullptr, *ub = nullptr;      // resident state, ping-pong
    double t = 0.0, step_t0 = 0.0;
    irk_status final_status = IRK_OK;         // while finishing
};

}  // namespace

struct irk_server {
    unsigned char *arena = nullptr;
    // shared V-cycle brokers: the preconditioner V-cycles of all running
    // requests that wait at the same time run as shared launches
    void *brk32 = nullptr, *brk64 = nullptr;
    Arena alloc;
    int max_slots = 1;
    long next_id = 1;
    std::deque<Req *> queue;
    std::vector<Req *> running;
    std::vector<Req *> finishing;             // done stepping, waiting for their last copy
    std::map<long, Req *> finished;
    std::vector<Slot> slots;
    std::vector<double> step_ms;              // latency of every completed step
    int peak_running = 0;
    size_t peak_bytes = 0;
};

static size_t field_len(const irk_operator &op) {
    const size_t n = (size_t)op.nx * op.ny;
    return op.kind == IRK_OP_VSF_2D ? 2 * n : n;
}

// the request's slot, arena range and event are free again; its result is
// final
static void complete(irk_server *s, Req *q) {
    const irk_status st = q->final_status;
    q->info.status = st;
    q->info.state = st == IRK_OK ? IRK_REQ_DONE : IRK_REQ_FAILED;
    q->info.t_done = now_s();
    if (q->ctx) irk::ctx_free(q->ctx);
    q->ctx = nullptr;
    if (q->slot >= 0) s->slots[q->slot].busy = false;
    q->slot = -1;
    q->stream = nullptr;
    if (q->u0_ready) (void)hipEventDestroy(q->u0_ready);
    q->u0_ready = nullptr;
    if (q->allocated) s->alloc.release(q->off, q->total);
    q->allocated = false;
    s->finished[q->id] = q;
}

// A request is done stepping (or failed): its result copy and an event
// behind all of its work are enqueued, and it completes when that event has
// (progress polls it); nothing here waits for the device.
static void finish(irk_server *s, Req *q, irk_status st) {
    q->final_status = st;
    if (!q->ctx) {
        complete(s, q);
        return;
    }
    Slot &sl = s->slots[q->slot];
    if (st == IRK_OK && q->r.out &&
        hipMemcpyAsync(q->r.out, q->ua, q->field_bytes, hipMemcpyDeviceToDevice, q->stream) != hipSuccess)
        q->final_status = IRK_E_DEVICE;
    if (irk::record_all_done(q->ctx, sl.fin) != IRK_OK) {
        // the event could not be recorded: wait here instead
        (void)hipDeviceSynchronize();
        q->final_status = IRK_E_DEVICE;
        complete(s, q);
        return;
    }
    s->finishing.push_back(q);
}

static void poll_finishing(irk_server *s) {
    for (size_t k = 0; k < s->finishing.size();) {
        Req *q = s->finishing[k];
        const hipError_t e = hipEventQuery(s->slots[q->slot].fin);
        if (e == hipErrorNotReady) {
            ++k;
            continue;
        }
        if (e != hipSuccess) q->final_status = IRK_E_DEVICE;
        s->finishing.erase(s->finishing.begin() + k);
        complete(s, q);
    }
}

// admit the queue head if a slot and memory are available
static bool try_admit(irk_server *s) {
    if (s->queue.empty() || (int)s->running.size() >= s->max_slots) return false;
    int slot = -1;
    for (int k = 0; k < (int)s->slots.size() && slot < 0; ++k)
        if (!s->slots[k].busy) slot = k;
    if (slot < 0) return false;                   // every slot still finishing
    Req *q = s->queue.front();
    if (q->total > s->alloc.capacity()) {          // can never fit
        s->queue.pop_front();
        finish(s, q, IRK_E_NOMEM);
        return true;
    }
    size_t off = 0;
    if (!s->alloc.alloc(q->total, &off)) return false;   // FIFO: wait for memory
    s->queue.pop_front();
    q->off = off;
    q->allocated = true;
    q->info.t_admit = now_s();
    q->info.state = IRK_REQ_RUNNING;
    Slot &sl = s->slots[slot];
    sl.busy = true;
    q->slot = slot;
    q->stream = sl.stream;
    unsigned char *base = s->arena + off;
    q->ua = (double *)base;
    q->ub = (double *)(base + ((q->field_bytes + 255) & ~size_t(255)));
    unsigned char *ws = base + 2 * ((q->field_bytes + 255) & ~size_t(255));
    irk_status st = IRK_OK;
    // u0 is read after the work the caller had queued on its stream at
    // submit; everything below only enqueues on the slot's streams
    if (hipStreamWaitEvent(q->stream, q->u0_ready, 0) != hipSuccess) st = IRK_E_DEVICE;
    if (st == IRK_OK &&
        hipMemcpyAsync(q->ua, q->r.u0, q->field_bytes, hipMemcpyDeviceToDevice, q->stream) != hipSuccess)
        st = IRK_E_DEVICE;
    if (st == IRK_OK)
        st = irk::create_in_res(q->r.family, q->r.s, &q->r.op, q->r.use_options ? &q->r.opt : nullptr, ws,
                                q->ws_bytes, q->stream, sl.res, &q->ctx);
    if (st == IRK_OK) (void)irk::attach_broker(q->ctx, s->brk32, s->brk64);
    q->t = q->r.t0;
    if (st == IRK_OK) {
        q->step_t0 = now_s();
        st = irk::step_begin(q->ctx, q->ua, q->t, q->r.dt, q->r.tol, q->ub);
    }
    if (st != IRK_OK) {
        finish(s, q, st);
        return true;
    }
    s->running.push_back(q);
    s->peak_running = std::max(s->peak_running, (int)s->running.size());
    s->peak_bytes = std::max(s->peak_bytes, s->alloc.used());
    return true;
}

extern "C" irk_status irk_server_create(void *arena, size_t arena_bytes, int max_slots, irk_server **out) {
    if (!out || !arena || ((uintptr_t)arena & 255) != 0 || arena_bytes < 256 || max_slots < 1) return IRK_E_ARG;
    irk_server *s = new (std::nothrow) irk_server();
    if (!s) return IRK_E_NOMEM;
    s->arena = (unsigned char *)arena;
    s->alloc.init(arena_bytes & ~size_t(255));
    s->max_slots = max_slots;
    // every slot's streams, events and pinned staging, and the shared V-cycle
    // brokers, now: admission then allocates nothing
    const size_t upload = kSlotUpload;
    s->slots.resize(max_slots);
    bool ok = true;
    for (Slot &sl : s->slots) {
        ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&sl.fin, hipEventDisableTiming) == hipSuccess &&
             (sl.res = irk::res_new(kSlotLanes, upload)) != nullptr;
        if (!ok) break;
    }
    s->brk32 = ok ? irk::broker_create(1) : nullptr;
    s->brk64 = ok ? irk::broker_create(0) : nullptr;
    if (!ok || !s->brk32 || !s->brk64) {
        irk_server_destroy(s);
        return IRK_E_DEVICE;
    }
    *out = s;
    return IRK_OK;
}

extern "C" irk_status irk_server_submit(irk_server *s, const irk_request *r, long *id) {
    if (!s || !r || !id || !r->u0 || !r->out || r->nsteps < 1 || !(r->dt > 0)) return IRK_E_ARG;
    const size_t ws = irk_workspace_bytes((irk_family)r->family, r->s, &r->op, r->use_options ? &r->opt : nullptr);
    if (ws == 0) return IRK_E_ARG;
    // a slot's staging covers grids of side <= kSlotMaxSide
    if (r->op.nx > kSlotMaxSide || r->op.ny > kSlotMaxSide ||
        irk::res_upload_need(r->family, r->s, &r->op, r->use_options ? &r->opt : nullptr) > kSlotUpload)
        return IRK_E_ARG;
    Req *q = new (std::nothrow) Req();
    if (!q) return IRK_E_NOMEM;
    q->id = s->next_id++;
    q->r = *r;
    std::memset(&q->info, 0, sizeof(q->info));
    q->info.state = IRK_REQ_QUEUED;
    q->info.t_submit = now_s();
    q->ws_bytes = ws;
    q->field_bytes = field_len(r->op) * sizeof(double);
    q->total = 2 * ((q->field_bytes + 255) & ~size_t(255)) + ws;
    // (a request that can never fit fails at admission without reading u0)
    if (q->total <= s->alloc.capacity() &&
        (hipEventCreateWithFlags(&q->u0_ready, hipEventDisableTiming) != hipSuccess ||
         hipEventRecord(q->u0_ready, (hipStream_t)r->stream) != hipSuccess)) {
        if (q->u0_ready) (void)hipEventDestroy(q->u0_ready);
        delete q;
        return IRK_E_DEVICE;
    }
    s->queue.push_back(q);
    *id = q->id;
    return IRK_OK;
}

static void poll_running(irk_server *s);

extern "C" int irk_server_progress(irk_server *s) {
    if (!s) return -1;
    poll_finishing(s);
    while (try_admit(s)) {
    }
    poll_running(s);
    // V-cycles that requests left waiting in this pass run as shared
    // launches; the resumed lanes continue at the next poll
    irk::broker_flush(s->brk32, 1);
    irk::broker_flush(s->brk64, 0);
    return (int)s->running.size() + (int)s->queue.size() + (int)s->finishing.size();
}

static void poll_running(irk_server *s) {
    for (size_t k = 0; k < s->running.size();) {
        Req *q = s->running[k];
        irk_status st = IRK_OK;
        irk_stats stats;
        if (!irk::step_poll(q->ctx, &st, &stats)) {
            ++k;
            continue;
        }
        const double t1 = now_s();
        if (st == IRK_OK) {
            s->step_ms.push_back(1e3 * (t1 - q->step_t0));
            q->info.steps_done++;
            q->info.newton_its += stats.newton_its;
            q->info.krylov_its += stats.krylov_its;
            q->t += q->r.dt;
            std::swap(q->ua, q->ub);
            if (q->info.steps_done < q->r.nsteps) {
                q->step_t0 = t1;
                st = irk::step_begin(q->ctx, q->ua, q->t, q->r.dt, q->r.tol, q->ub);
                if (st == IRK_OK) {
                    ++k;
                    continue;
                }
            }
        }
        s->running.erase(s->running.begin() + k);
        finish(s, q, st);
        while (try_admit(s)) {
        }
    }
}

extern "C" irk_status irk_server_info(irk_server *s, long id, irk_request_info *info) {
    if (!s || !info) return IRK_E_ARG;
    auto it = s->finished.find(id);
    if (it != s->finished.end()) {
        *info = it->second->info;
        return IRK_OK;
    }
    for (Req *q : s->running)
        if (q->id == id) { *info = q->info; return IRK_OK; }
    for (Req *q : s->finishing)
        if (q->id == id) { *info = q->info; return IRK_OK; }
    for (Req *q : s->queue)
        if (q->id == id) { *info = q->info; return IRK_OK; }
    return IRK_E_ARG;
}

extern "C" irk_status irk_server_stats(irk_server *s, double *step_ms, int cap, int *nsteps, int *peak_running,
                                       size_t *peak_bytes) {
    if (!s) return IRK_E_ARG;
    const int n = (int)s->step_ms.size();
    if (nsteps) *nsteps = n;
    if (step_ms)
        for (int k = 0; k < n && k < cap; ++k) step_ms[k] = s->step_ms[k];
    if (peak_running) *peak_running = s->peak_running;
    if (peak_bytes) *peak_bytes = s->peak_bytes;
    return IRK_OK;
}

extern "C" void irk_server_destroy(irk_server *s) {
    if (!s) return;
    for (Req *q : s->running) finish(s, q, IRK_E_ARG);
    s->running.clear();
    for (const Slot &sl : s->slots)
        if (sl.busy && sl.fin) (void)hipEventSynchronize(sl.fin);
    poll_finishing(s);
    for (Req *q : s->queue) {
        if (q->u0_ready) (void)hipEventDestroy(q->u0_ready);
        delete q;
    }
    for (auto &kv : s->finished) delete kv.second;
    if (s->brk32) irk::broker_destroy(s->brk32, 1);
    if (s->brk64) irk::broker_destroy(s->brk64, 0);
    for (Slot &sl : s->slots) {
        if (sl.res) irk::res_free(sl.res);
        if (sl.stream) {
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
        }
        if (sl.fin) (void)hipEventDestroy(sl.fin);
    }
    delete s;
}
