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
#include <hip/hip_runtime.h>

#include <cstring>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "fpcg_host.hpp"

using namespace fpcg;

namespace {

struct Req {
    uint64_t ticket = 0;
    fpcg_request r{};
    Plan plan;
    size_t in_bytes = 0, out_bytes = 0, bytes = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    fpcg_status status = FPCG_OK;
};

struct ChanSet {
    int64_t B = 0;
    int32_t Nbs = 0, K = 0, io_c64 = 0;
    void* dH = nullptr;
    double* dS = nullptr;
    size_t bytes = 0;
    int users = 0;          // queued or running requests reading it
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

}  // namespace

struct fpcg_server {
    fpcg_ctx* ctx = nullptr;
    int cap = 0;
    std::vector<Slot> slots;
    std::deque<Req*> queue;
    std::unordered_map<uint64_t, Req*> reqs;
    size_t held = 0;   // device bytes of all slot buffers
    std::unordered_map<uint64_t, ChanSet> chans;
    size_t chan_bytes = 0;   // device bytes of the resident channel sets
    uint64_t next = 1, next_chan = 1;
    std::mutex mu;
};

static fpcg_status retire_and_admit(fpcg_server* s) {
    // retire finished requests
    for (Slot& sl : s->slots) {
        if (!sl.req) continue;
        hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        Req* rq = sl.req;
        if (q != hipSuccess) {
            rq->status = fail(FPCG_E_DEVICE, "request %llu: %s", (unsigned long long)rq->ticket, hipGetErrorString(q));
        } else {
            const Layout L = layout_of(rq->r);
            const char* hb = static_cast<const char*>(sl.hbuf);
            const size_t el = rq->r.io_c64 ? 8 : 16;
            std::memcpy(rq->r.xhat, hb + L.x, (size_t)rq->r.B * rq->r.K * rq->r.R * el);
            std::memcpy(rq->r.labels, hb + L.lab, (size_t)rq->r.B * rq->r.K * rq->r.R);
            if (rq->r.flags) std::memcpy(rq->r.flags, hb + L.fl, (size_t)rq->r.B * 4);
        }
        rq->state = 2;
        if (rq->r.channels) s->chans[rq->r.channels].users--;
        sl.req = nullptr;
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
                rq->status = fail(FPCG_E_NOMEM, "device/pinned allocation of %zu bytes failed", L.total);
                rq->state = 2;
                if (rq->r.channels) s->chans[rq->r.channels].users--;
                continue;
            }
            pick->dcap = pick->hcap = L.total;
            s->held += L.total;
        }
        s->queue.pop_front();
        Slot& sl = *pick;
        char* hb = static_cast<char*>(sl.hbuf);
        char* db = static_cast<char*>(sl.dbuf);
        const fpcg_request& r = rq->r;
        const size_t el = r.io_c64 ? 8 : 16;
        const size_t nh = (size_t)r.B * r.Nbs * r.K * el, ny = (size_t)r.B * r.Nbs * r.R * el;
        const ChanSet* cs = r.channels ? &s->chans[r.channels] : nullptr;
        if (!cs) std::memcpy(hb + L.h, r.H, nh);
        std::memcpy(hb + L.y, r.Y, ny);
        if (!cs) std::memcpy(hb + L.s2, r.sigma2, (size_t)r.B * 8);
        hipError_t e = hipMemcpyAsync(db, hb, L.x, hipMemcpyHostToDevice, sl.stream);
        fpcg_status st = FPCG_OK;
        if (e != hipSuccess) st = fail(FPCG_E_DEVICE, "H2D copy: %s", hipGetErrorString(e));
        const void* dH = cs ? cs->dH : static_cast<const void*>(db + L.h);
        const double* dS = cs ? cs->dS : reinterpret_cast<const double*>(db + L.s2);
        if (st == FPCG_OK)
            st = launch_detect(s->ctx, sl.stream, rq->plan, r.B, r.Nbs, r.K, r.R, dH, db + L.y, r.io_c64, dS,
                               r.qam_order, r.iters, db + L.x, reinterpret_cast<uint8_t*>(db + L.lab),
                               reinterpret_cast<uint32_t*>(db + L.fl));
        if (st == FPCG_OK) {
            e = hipMemcpyAsync(hb + L.x, db + L.x, L.total - L.x, hipMemcpyDeviceToHost, sl.stream);
            if (e != hipSuccess) st = fail(FPCG_E_DEVICE, "D2H copy: %s", hipGetErrorString(e));
        }
        if (st == FPCG_OK) {
            e = hipEventRecord(sl.done, sl.stream);
            if (e != hipSuccess) st = fail(FPCG_E_DEVICE, "event record: %s", hipGetErrorString(e));
        }
        if (st != FPCG_OK) {
            rq->status = st;
            rq->state = 2;
            if (rq->r.channels) s->chans[rq->r.channels].users--;
            (void)hipStreamSynchronize(sl.stream);
            continue;
        }
        rq->state = 1;
        sl.req = rq;
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
    *done = rq->state == 2 ? 1 : 0;
    if (rq->state == 2) {
        fpcg_status st = rq->status;
        s->reqs.erase(it);
        delete rq;
        return st;
    }
    return FPCG_OK;
}

fpcg_status fpcg_drain(fpcg_server* s) {
    clear_error();
    if (!s) return fail(FPCG_E_INVAL, "NULL server");
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            (void)hipSetDevice(s->ctx->device);
            retire_and_admit(s);
            bool busy = !s->queue.empty();
            for (Slot& sl : s->slots) busy |= sl.req != nullptr;
            if (!busy) return FPCG_OK;
            for (Slot& sl : s->slots)
                if (sl.req) { (void)hipEventSynchronize(sl.done); break; }
        }
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
    s->chans.erase(it);
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
    (void)fpcg_drain(s);
    for (Slot& sl : s->slots) {
        if (sl.dbuf) (void)hipFree(sl.dbuf);
        if (sl.hbuf) (void)hipHostFree(sl.hbuf);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto& kv : s->chans) {
        if (kv.second.dH) (void)hipFree(kv.second.dH);
        if (kv.second.dS) (void)hipFree(kv.second.dS);
    }
    for (auto& kv : s->reqs) delete kv.second;
    delete s;
}

}  // extern "C"
