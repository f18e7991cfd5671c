// Continuous-batching request loop (fpcg_server_* in fpcg.h).
//
// Requests carry host buffers.  A request is admitted when a stream slot is
// free and its device footprint fits the context's budget next to the
// requests already in flight; its inputs are staged through pinned memory,
// the detector runs on the slot's stream and the outputs come back through
// pinned memory.  Requests arriving while others run are admitted as slots
// and memory free up, so work of different requests overlaps on the device.
// Each channel is computed by its own workgroup in a fixed order, so a
// request's results do not depend on what else is in flight.
//
// The host copies between the caller's buffers and pinned staging run on two
// worker threads (one stages inputs and enqueues the device work in
// admission order, one copies results out), so the thread that polls only
// schedules.  A resident channel set keeps the block-Jacobi factor of each
// (L, operand format, work precision) it is served with: the first request
// stores it, later ones read it in place of the factorisation, also after
// the set's channels were replaced by their next realisation
// (fpcg_server_channels_update with keep_precond).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "fpcg_host.hpp"

using namespace fpcg;

namespace {

enum : int { Q_QUEUED = 0, Q_STAGING = 1, Q_RUNNING = 2, Q_COPYOUT = 3, Q_DONE = 4 };

// a kept block-Jacobi factor of a resident channel set
struct Pc {
    void* buf = nullptr;
    size_t bytes = 0;
    hipEvent_t ready = nullptr;   // recorded after the launch that stores it
    bool pending = false;         // a storing launch has been admitted
    bool valid = false;           // ... and was enqueued without error
};
using PcKey = std::tuple<int, int, int>;   // L, operand format, work precision

struct ChanSet {
    int64_t B = 0;
    int32_t Nbs = 0, K = 0, io_c64 = 0;
    void* dH = nullptr;
    double* dS = nullptr;
    size_t bytes = 0;
    int users = 0;          // queued or running requests reading it
    std::map<PcKey, Pc> pc;
};

struct Slot;

struct Req {
    uint64_t ticket = 0;
    fpcg_request r{};
    Plan plan;
    size_t bytes = 0;
    int state = Q_QUEUED;
    fpcg_status status = FPCG_OK;
    std::string msg;        // the failing call's message (workers keep their own last error)
    // set at admission for the staging worker
    Slot* slot = nullptr;
    const void* dH = nullptr;
    const double* dS = nullptr;
    Pc* pc = nullptr;
    int pc_mode = 0;        // 0, FPCG_PRECOND_STORE or FPCG_PRECOND_LOAD
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Req* req = nullptr;
    void* dbuf = nullptr;   // device: H | Y | sigma2 | xhat | labels | flags
    size_t dcap = 0;
    void* hbuf = nullptr;   // pinned staging, same layout
    size_t hcap = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t h, y, s2, x, lab, fl, total;
};

// slot buffer of a request; a request on a resident channel set has no H or
// sigma^2 segment (zero-length, at the Y offset)
Layout layout_of(const fpcg_request& r) {
    const size_t el = r.io_c64 ? 8 : 16;
    const bool resident = r.channels != 0;
    Layout L;
    size_t o = 0;
    L.h = o; o = resident ? o : align256(o + (size_t)r.B * r.Nbs * r.K * el);
    L.y = o; o = align256(o + (size_t)r.B * r.Nbs * r.R * el);
    L.s2 = o; o = resident ? o : align256(o + (size_t)r.B * 8);
    L.x = o; o = align256(o + (size_t)r.B * r.K * r.R * el);
    L.lab = o; o = align256(o + (size_t)r.B * r.K * r.R);
    L.fl = o; o = align256(o + (size_t)r.B * 4);
    L.total = o;
    return L;
}

void free_pc(Pc& p) {
    if (p.buf) (void)hipFree(p.buf);
    if (p.ready) (void)hipEventDestroy(p.ready);
    p = Pc{};
}

}  // namespace

struct fpcg_server {
    fpcg_ctx* ctx = nullptr;
    int cap = 0;
    std::vector<Slot> slots;
    std::deque<Req*> queue;
    std::unordered_map<uint64_t, Req*> reqs;
    size_t held = 0;   // device bytes of all slot buffers
    std::unordered_map<uint64_t, ChanSet> chans;
    size_t chan_bytes = 0;   // device bytes of the resident channel sets and their factors
    uint64_t next = 1, next_chan = 1;
    std::mutex mu;
    std::deque<Req*> in_jobs, out_jobs;
    std::condition_variable cv_in, cv_out, cv_progress;
    bool stop = false;
    std::thread in_worker, out_worker;
};

// the end of a request (under the lock): its slot and channel set are free
static void finish(fpcg_server* s, Req* rq, fpcg_status st) {
    if (st != FPCG_OK) {
        rq->status = st;
        rq->msg = fpcg_last_error();
    }
    rq->state = Q_DONE;
    if (rq->slot) rq->slot->req = nullptr;
    rq->slot = nullptr;
    if (rq->r.channels) s->chans[rq->r.channels].users--;
    s->cv_progress.notify_all();
}

// staging worker, outside the lock: inputs into pinned memory, the copy to the
// device, the launch (waiting for a kept factor's storing launch), the copy
// back to pinned memory and the slot's completion event
static fpcg_status stage_and_launch(fpcg_server* s, Req* rq, hipEvent_t pc_wait, hipEvent_t pc_record) {
    Slot& sl = *rq->slot;
    const fpcg_request& r = rq->r;
    const Layout L = layout_of(r);
    char* hb = static_cast<char*>(sl.hbuf);
    char* db = static_cast<char*>(sl.dbuf);
    const size_t el = r.io_c64 ? 8 : 16;
    const size_t nh = (size_t)r.B * r.Nbs * r.K * el, ny = (size_t)r.B * r.Nbs * r.R * el;
    if (!r.channels) std::memcpy(hb + L.h, r.H, nh);
    std::memcpy(hb + L.y, r.Y, ny);
    if (!r.channels) std::memcpy(hb + L.s2, r.sigma2, (size_t)r.B * 8);
    hipError_t e = hipMemcpyAsync(db, hb, L.x, hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) return fail(FPCG_E_DEVICE, "H2D copy: %s", hipGetErrorString(e));
    const void* dH = rq->dH ? rq->dH : static_cast<const void*>(db + L.h);
    const double* dS = rq->dS ? rq->dS : reinterpret_cast<const double*>(db + L.s2);
    fpcg_status st;
    if (rq->pc_mode) {
        if (pc_wait && hipStreamWaitEvent(sl.stream, pc_wait, 0) != hipSuccess)
            return fail(FPCG_E_DEVICE, "waiting for the stored factor failed");
        LaunchExtra ex;
        ex.n = r.B;
        if (rq->pc_mode == FPCG_PRECOND_STORE) ex.T_out = rq->pc->buf;
        else ex.T_in = rq->pc->buf;
        int form = s->ctx->launch_form;
        if (form == FPCG_LAUNCH_AUTO) {
            auto it = s->ctx->tuned.find(tune_key(rq->plan, r.R, r.io_c64));
            form = it != s->ctx->tuned.end() ? it->second : FPCG_LAUNCH_FUSED;
        }
        st = launch_detect_form(s->ctx, sl.stream, rq->plan, form, r.B, r.Nbs, r.K, r.R, dH, db + L.y, r.io_c64, dS,
                                r.qam_order, r.iters, db + L.x, reinterpret_cast<uint8_t*>(db + L.lab),
                                reinterpret_cast<uint32_t*>(db + L.fl), &ex);
        if (st == FPCG_OK && pc_record && hipEventRecord(pc_record, sl.stream) != hipSuccess)
            st = fail(FPCG_E_DEVICE, "recording the stored factor failed");
    } else {
        st = launch_detect(s->ctx, sl.stream, rq->plan, r.B, r.Nbs, r.K, r.R, dH, db + L.y, r.io_c64, dS,
                           r.qam_order, r.iters, db + L.x, reinterpret_cast<uint8_t*>(db + L.lab),
                           reinterpret_cast<uint32_t*>(db + L.fl));
    }
    if (st != FPCG_OK) return st;
    e = hipMemcpyAsync(hb + L.x, db + L.x, L.total - L.x, hipMemcpyDeviceToHost, sl.stream);
    if (e != hipSuccess) return fail(FPCG_E_DEVICE, "D2H copy: %s", hipGetErrorString(e));
    e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) return fail(FPCG_E_DEVICE, "event record: %s", hipGetErrorString(e));
    return FPCG_OK;
}

static void in_loop(fpcg_server* s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_in.wait(lk, [&] { return s->stop || !s->in_jobs.empty(); });
        if (s->in_jobs.empty()) break;   // stop, nothing left
        Req* rq = s->in_jobs.front();
        s->in_jobs.pop_front();
        hipEvent_t wait = nullptr, record = nullptr;
        if (rq->pc_mode == FPCG_PRECOND_LOAD) {
            if (!rq->pc->valid) {                     // its storing launch failed
                finish(s, rq, fail(FPCG_E_DEVICE, "request %llu: the kept factor was not stored",
                                   (unsigned long long)rq->ticket));
                continue;
            }
            wait = rq->pc->ready;
        } else if (rq->pc_mode == FPCG_PRECOND_STORE) {
            record = rq->pc->ready;
        }
        lk.unlock();
        const fpcg_status st = stage_and_launch(s, rq, wait, record);
        if (st != FPCG_OK) (void)hipStreamSynchronize(rq->slot->stream);
        lk.lock();
        if (rq->pc_mode == FPCG_PRECOND_STORE) {
            rq->pc->valid = st == FPCG_OK;
            rq->pc->pending = st == FPCG_OK;
        }
        if (st != FPCG_OK) finish(s, rq, st);
        else rq->state = Q_RUNNING;
        s->cv_progress.notify_all();
    }
}

static void out_loop(fpcg_server* s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_out.wait(lk, [&] { return s->stop || !s->out_jobs.empty(); });
        if (s->out_jobs.empty()) break;
        Req* rq = s->out_jobs.front();
        s->out_jobs.pop_front();
        lk.unlock();
        const Layout L = layout_of(rq->r);
        const char* hb = static_cast<const char*>(rq->slot->hbuf);
        const size_t el = rq->r.io_c64 ? 8 : 16;
        std::memcpy(rq->r.xhat, hb + L.x, (size_t)rq->r.B * rq->r.K * rq->r.R * el);
        std::memcpy(rq->r.labels, hb + L.lab, (size_t)rq->r.B * rq->r.K * rq->r.R);
        if (rq->r.flags) std::memcpy(rq->r.flags, hb + L.fl, (size_t)rq->r.B * 4);
        lk.lock();
        finish(s, rq, FPCG_OK);
    }
}

// the kept factor a request on a resident channel set uses (under the lock):
// stored by the first request of its (L, format, work) class, read by later
// ones; none where it would not fit the budget
static void pick_factor(fpcg_server* s, Req* rq) {
    const fpcg_request& r = rq->r;
    if (!r.channels || r.block_L <= 0) return;
    ChanSet& cs = s->chans[r.channels];
    const PcKey key(r.block_L, r.sched.gram_op, r.sched.work);
    auto it = cs.pc.find(key);
    if (it != cs.pc.end()) {                          // stored (or being stored): read it; after a failed store, store again
        Pc& p = it->second;
        rq->pc = &p;
        rq->pc_mode = p.pending ? FPCG_PRECOND_LOAD : FPCG_PRECOND_STORE;
        p.pending = true;
        return;
    }
    const size_t bytes = (size_t)r.B * r.K * r.block_L * (r.sched.work == FPCG_F64 ? 16 : 8);
    if (s->held + s->chan_bytes + bytes > s->ctx->budget) return;
    Pc p;
    if (hipMalloc(&p.buf, bytes) != hipSuccess || hipEventCreateWithFlags(&p.ready, hipEventDisableTiming) != hipSuccess) {
        free_pc(p);
        return;
    }
    p.bytes = bytes;
    p.pending = true;
    s->chan_bytes += bytes;
    Pc& kept = cs.pc[key] = p;
    rq->pc = &kept;
    rq->pc_mode = FPCG_PRECOND_STORE;
}

static fpcg_status retire_and_admit(fpcg_server* s) {
    // finished device work: its results go to the copy-out worker
    for (Slot& sl : s->slots) {
        Req* rq = sl.req;
        if (!rq || rq->state != Q_RUNNING) continue;
        hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
            finish(s, rq, fail(FPCG_E_DEVICE, "request %llu: %s", (unsigned long long)rq->ticket, hipGetErrorString(q)));
            continue;
        }
        rq->state = Q_COPYOUT;
        s->out_jobs.push_back(rq);
        s->cv_out.notify_one();
    }
    // admit in arrival order while a slot is free and the budget allows; the
    // budget covers every device buffer the server holds (slot buffers are
    // kept and reused, and grown only when a request needs more)
    while (!s->queue.empty()) {
        Req* rq = s->queue.front();
        const Layout L = layout_of(rq->r);
        Slot* pick = nullptr;
        for (Slot& sl : s->slots)   // a free slot that already fits: no allocation
            if (!sl.req && sl.dcap >= L.total) { pick = &sl; break; }
        if (!pick) {
            for (Slot& sl : s->slots)
                if (!sl.req) { pick = &sl; break; }
            if (!pick) break;                                      // every slot busy
            if (s->held + s->chan_bytes - pick->dcap + L.total > s->ctx->budget) {
                // release the buffers of the other idle slots, then try again
                for (Slot& sl : s->slots) {
                    if (sl.req || &sl == pick || !sl.dbuf) continue;
                    (void)hipFree(sl.dbuf);
                    (void)hipHostFree(sl.hbuf);
                    s->held -= sl.dcap;
                    sl.dbuf = nullptr; sl.hbuf = nullptr; sl.dcap = sl.hcap = 0;
                }
                if (s->held + s->chan_bytes - pick->dcap + L.total > s->ctx->budget) break;   // wait for running requests
            }
            if (pick->dbuf) (void)hipFree(pick->dbuf);
            if (pick->hbuf) (void)hipHostFree(pick->hbuf);
            s->held -= pick->dcap;
            pick->dbuf = nullptr; pick->hbuf = nullptr; pick->dcap = pick->hcap = 0;
            if (hipMalloc(&pick->dbuf, L.total) != hipSuccess ||
                hipHostMalloc(&pick->hbuf, L.total, hipHostMallocDefault) != hipSuccess) {
                if (pick->dbuf) (void)hipFree(pick->dbuf);
                pick->dbuf = nullptr; pick->hbuf = nullptr;
                s->queue.pop_front();
                finish(s, rq, fail(FPCG_E_NOMEM, "device/pinned allocation of %zu bytes failed", L.total));
                continue;
            }
            pick->dcap = pick->hcap = L.total;
            s->held += L.total;
        }
        s->queue.pop_front();
        pick->req = rq;
        rq->slot = pick;
        if (rq->r.channels) {
            const ChanSet& cs = s->chans[rq->r.channels];
            rq->dH = cs.dH;
            rq->dS = cs.dS;
        }
        pick_factor(s, rq);
        rq->state = Q_STAGING;
        s->in_jobs.push_back(rq);
        s->cv_in.notify_one();
    }
    return FPCG_OK;
}

extern "C" {

fpcg_status fpcg_server_create(fpcg_ctx* ctx, int32_t n_slots, int32_t queue_cap, fpcg_server** out) {
    clear_error();
    if (!ctx || !out) return fail(FPCG_E_INVAL, "NULL argument");
    if (n_slots < 1 || n_slots > 16) return fail(FPCG_E_INVAL, "n_slots=%d must be in [1, 16]", n_slots);
    if (queue_cap < 1) return fail(FPCG_E_INVAL, "queue_cap=%d must be >= 1", queue_cap);
    (void)hipSetDevice(ctx->device);
    fpcg_server* s = new fpcg_server();
    s->ctx = ctx;
    s->cap = queue_cap;
    s->slots.resize(n_slots);
    for (Slot& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            fpcg_server_destroy(s);
            return fail(FPCG_E_DEVICE, "stream/event creation failed");
        }
    }
    s->in_worker = std::thread(in_loop, s);
    s->out_worker = std::thread(out_loop, s);
    *out = s;
    return FPCG_OK;
}

fpcg_status fpcg_submit(fpcg_server* s, const fpcg_request* req, uint64_t* ticket) {
    clear_error();
    if (!s || !req || !ticket) return fail(FPCG_E_INVAL, "NULL argument");
    Plan plan;
    fpcg_status st = check_args(req->B, req->Nbs, req->K, req->R, req->qam_order, req->iters, req->block_L, &req->sched, &plan);
    if (st != FPCG_OK) return st;
    const bool resident = req->channels != 0;
    if (req->B > 0 && ((!resident && (!req->H || !req->sigma2)) || !req->Y || !req->xhat || !req->labels))
        return fail(FPCG_E_INVAL, "request buffers must be non-NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (resident) {
        auto it = s->chans.find(req->channels);
        if (it == s->chans.end())
            return fail(FPCG_E_INVAL, "unknown channel set %llu", (unsigned long long)req->channels);
        const ChanSet& c = it->second;
        if (c.B != req->B || c.Nbs != req->Nbs || c.K != req->K || c.io_c64 != req->io_c64)
            return fail(FPCG_E_INVAL, "request sizes do not match channel set %llu", (unsigned long long)req->channels);
    }
    const size_t bytes = layout_of(*req).total;
    if (bytes + s->chan_bytes > s->ctx->budget)
        return fail(FPCG_E_NOMEM, "request needs %zu bytes, budget %zu (%zu in channel sets)", bytes, s->ctx->budget,
                    s->chan_bytes);
    if ((int)s->queue.size() >= s->cap) return fail(FPCG_E_BUSY, "queue full (%d)", s->cap);
    Req* rq = new Req();
    rq->ticket = s->next++;
    rq->r = *req;
    rq->plan = plan;
    rq->bytes = bytes;
    s->reqs[rq->ticket] = rq;
    s->queue.push_back(rq);
    if (resident) s->chans[req->channels].users++;
    *ticket = rq->ticket;
    (void)hipSetDevice(s->ctx->device);
    return retire_and_admit(s);
}

fpcg_status fpcg_poll(fpcg_server* s, uint64_t ticket, int32_t* done) {
    clear_error();
    if (!s || !done) return fail(FPCG_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    (void)hipSetDevice(s->ctx->device);
    retire_and_admit(s);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(FPCG_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Req* rq = it->second;
    *done = rq->state == Q_DONE ? 1 : 0;
    if (rq->state == Q_DONE) {
        const fpcg_status st = rq->status;
        const std::string msg = rq->msg;
        s->reqs.erase(it);
        delete rq;
        return st == FPCG_OK ? st : fail(st, "%s", msg.c_str());
    }
    return FPCG_OK;
}

fpcg_status fpcg_drain(fpcg_server* s) {
    clear_error();
    if (!s) return fail(FPCG_E_INVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        retire_and_admit(s);
        bool busy = !s->queue.empty();
        for (Slot& sl : s->slots) busy |= sl.req != nullptr;
        if (!busy) return FPCG_OK;
        // the workers signal progress; device completions are polled
        s->cv_progress.wait_for(lk, std::chrono::microseconds(200));
    }
}

fpcg_status fpcg_server_channels(fpcg_server* s, int64_t B, int32_t Nbs, int32_t K, int32_t io_c64, const void* H,
                                 const double* sigma2, uint64_t* handle) {
    clear_error();
    if (!s || !handle) return fail(FPCG_E_INVAL, "NULL argument");
    if (B < 1 || B > 0x7fffffffLL || Nbs < 1 || K < 1) return fail(FPCG_E_INVAL, "bad channel-set sizes");
    if (!H || !sigma2) return fail(FPCG_E_INVAL, "H and sigma2 must be non-NULL");
    const size_t nh = (size_t)B * Nbs * K * (io_c64 ? 8 : 16), ns = (size_t)B * 8;
    std::lock_guard<std::mutex> lk(s->mu);
    (void)hipSetDevice(s->ctx->device);
    retire_and_admit(s);
    if (s->held + s->chan_bytes + nh + ns > s->ctx->budget) {
        // make room from idle slot buffers first
        for (Slot& sl : s->slots) {
            if (sl.req || !sl.dbuf) continue;
            (void)hipFree(sl.dbuf);
            (void)hipHostFree(sl.hbuf);
            s->held -= sl.dcap;
            sl.dbuf = nullptr; sl.hbuf = nullptr; sl.dcap = sl.hcap = 0;
        }
        if (s->held + s->chan_bytes + nh + ns > s->ctx->budget)
            return fail(FPCG_E_NOMEM, "channel set of %zu bytes does not fit the budget", nh + ns);
    }
    ChanSet c;
    c.B = B; c.Nbs = Nbs; c.K = K; c.io_c64 = io_c64 ? 1 : 0;
    if (hipMalloc(&c.dH, nh) != hipSuccess || hipMalloc((void**)&c.dS, ns) != hipSuccess) {
        if (c.dH) (void)hipFree(c.dH);
        return fail(FPCG_E_NOMEM, "device allocation of %zu bytes failed", nh + ns);
    }
    if (hipMemcpy(c.dH, H, nh, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.dS, sigma2, ns, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c.dH);
        (void)hipFree(c.dS);
        return fail(FPCG_E_DEVICE, "channel-set upload failed");
    }
    c.bytes = nh + ns;
    const uint64_t h = s->next_chan++;
    s->chans[h] = c;
    s->chan_bytes += c.bytes;
    *handle = h;
    return FPCG_OK;
}

fpcg_status fpcg_server_release(fpcg_server* s, uint64_t handle) {
    clear_error();
    if (!s) return fail(FPCG_E_INVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->chans.find(handle);
    if (it == s->chans.end()) return fail(FPCG_E_INVAL, "unknown channel set %llu", (unsigned long long)handle);
    (void)hipSetDevice(s->ctx->device);
    retire_and_admit(s);
    if (it->second.users > 0) return fail(FPCG_E_BUSY, "channel set %llu is in use", (unsigned long long)handle);
    (void)hipFree(it->second.dH);
    (void)hipFree(it->second.dS);
    s->chan_bytes -= it->second.bytes;
    for (auto& kv : it->second.pc) {
        s->chan_bytes -= kv.second.bytes;
        free_pc(kv.second);
    }
    s->chans.erase(it);
    return FPCG_OK;
}

fpcg_status fpcg_server_channels_update(fpcg_server* s, uint64_t handle, const void* H, const double* sigma2,
                                        int32_t keep_precond) {
    clear_error();
    if (!s) return fail(FPCG_E_INVAL, "NULL server");
    if (!H || !sigma2) return fail(FPCG_E_INVAL, "H and sigma2 must be non-NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->chans.find(handle);
    if (it == s->chans.end()) return fail(FPCG_E_INVAL, "unknown channel set %llu", (unsigned long long)handle);
    (void)hipSetDevice(s->ctx->device);
    retire_and_admit(s);
    ChanSet& c = it->second;
    if (c.users > 0) return fail(FPCG_E_BUSY, "channel set %llu is in use", (unsigned long long)handle);
    const size_t nh = (size_t)c.B * c.Nbs * c.K * (c.io_c64 ? 8 : 16), ns = (size_t)c.B * 8;
    if (hipMemcpy(c.dH, H, nh, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.dS, sigma2, ns, hipMemcpyHostToDevice) != hipSuccess)
        return fail(FPCG_E_DEVICE, "channel-set upload failed");
    if (!keep_precond) {
        for (auto& kv : c.pc) {
            s->chan_bytes -= kv.second.bytes;
            free_pc(kv.second);
        }
        c.pc.clear();
    }
    return FPCG_OK;
}

fpcg_status fpcg_server_stats(fpcg_server* s, int32_t* in_flight, int32_t* queued, size_t* bytes_held) {
    clear_error();
    if (!s) return fail(FPCG_E_INVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    int f = 0;
    for (Slot& sl : s->slots) f += sl.req != nullptr;
    if (in_flight) *in_flight = f;
    if (queued) *queued = (int32_t)s->queue.size();
    if (bytes_held) *bytes_held = s->held + s->chan_bytes;
    return FPCG_OK;
}

void fpcg_server_destroy(fpcg_server* s) {
    if (!s) return;
    if (s->in_worker.joinable()) (void)fpcg_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_in.notify_all();
    s->cv_out.notify_all();
    if (s->in_worker.joinable()) s->in_worker.join();
    if (s->out_worker.joinable()) s->out_worker.join();
    for (Slot& sl : s->slots) {
        if (sl.dbuf) (void)hipFree(sl.dbuf);
        if (sl.hbuf) (void)hipHostFree(sl.hbuf);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto& kv : s->chans) {
        if (kv.second.dH) (void)hipFree(kv.second.dH);
        if (kv.second.dS) (void)hipFree(kv.second.dS);
        for (auto& p : kv.second.pc) free_pc(p.second);
    }
    for (auto& kv : s->reqs) delete kv.second;
    delete s;
}

}  // extern "C"
