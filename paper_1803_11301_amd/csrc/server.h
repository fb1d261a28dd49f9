// server.h -- the product server: continuous batching of product requests
// over several HIP streams, admitted by device-memory footprint.
//
// One scheduler thread per server admits requests and sees them complete;
// each launch slot (a stream with its own workspace view) has a launcher
// thread that enqueues the slot's kernels, outside the server lock, so that
// the slots' launches (a dozen kernels for a product on the fused path) are
// issued side by side rather than one after another on the scheduler.
// Requests are queued by polymul_submit; whenever a slot is free, the
// admission policy of server_policy.h picks the next launch: waiting small
// products (by default at most 2^20 bits, up to 512 of them) together as one
// batched launch of k_batch, or one larger product through the
// single-product path.  Its workspace is carved out of the server's arena,
// one device allocation made at creation, so memory use never exceeds the
// budget and nothing is allocated while serving.  Launches on different
// slots overlap on the device; a slot is freed, and its arena range
// returned, when its completion event has fired.
//
// Included at the end of fpmul.hip (it uses the product and batch paths).
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "server_policy.h"

namespace {

struct SrvTicket {
    int state = 0;   // 0 waiting, 1 running, 2 done
    int rc = 0;
    std::string err;   // message of a failed launch
    uint64_t t_submit = 0, t_start = 0, t_done = 0;
};

struct SrvSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    polymul_ctx *view = nullptr;     // borrows the parent's tables and arena ranges
    BtDesc *host_desc = nullptr;     // pinned, max_batch entries
    bool busy = false;               // a plan is admitted on the slot
    bool go = false;                 // ... and waits for the launcher thread
    bool launched = false;           // ... and its kernels and `done` are enqueued
    fpmul_srv::Plan plan;
    std::thread launcher;
};

uint64_t srv_now_ns(std::chrono::steady_clock::time_point t0)
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0)
        .count();
}

// device bytes of one single-product launch (the four workspace buffers)
uint64_t srv_single_bytes(uint64_t lc) { return fpmul_plan::single_launch_bytes(lc); }

}  // namespace

struct polymul_server {
    polymul_ctx *ctx = nullptr;   // parent: device, tables, batch steps
    void *arena_base = nullptr;
    fpmul_srv::Arena arena;
    fpmul_srv::Policy policy;
    fpmul_srv::Footprint fp;
    std::vector<SrvSlot> slots;
    std::mutex m;
    std::condition_variable cv_work, cv_done, cv_launch;
    std::deque<fpmul_srv::Req> pending;
    std::unordered_map<uint64_t, SrvTicket> tickets;
    uint64_t next_ticket = 1;
    uint32_t busy = 0;
    bool stop = false;
    bool stop_launchers = false;
    std::thread th;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
};

static void srv_finish(polymul_server *S, SrvSlot &slot, int rc)
{
    const uint64_t t = srv_now_ns(S->t0);
    for (const auto &r : slot.plan.reqs) {
        auto it = S->tickets.find(r.ticket);   // a ticket is only released once it is done
        if (it == S->tickets.end()) continue;
        SrvTicket &tk = it->second;
        tk.state = 2;
        tk.rc = rc;
        if (rc) tk.err = g_err;
        tk.t_done = t;
    }
    S->arena.release(slot.plan.off, slot.plan.bytes);
    slot.busy = false;
    slot.launched = false;
    slot.plan.reqs.clear();
    S->busy--;
}

// enqueue the plan on the slot; returns the launch's result code
static int srv_launch(polymul_server *S, SrvSlot &slot)
{
    const fpmul_srv::Plan &p = slot.plan;
    polymul_ctx *v = slot.view;
    char *base = static_cast<char *>(S->arena_base) + p.off;
    hipStream_t s = slot.stream;
    int rc;
    if (!p.batch) {
        const fpmul_srv::Req &r = p.reqs[0];
        // four buffers of the words product_body asks for; never launch on a
        // reservation smaller than that (plan.h sizes both, and the CPU check
        // of tests/native/plan_check.cpp holds them together)
        const uint64_t words = r.fa ? fpmul_plan::ws_words_for(r.res_log2n)
                                    : fpmul_plan::product_ws_words(r.la, r.lb, v->large_field_log2n);
        if (4 * words * 8 > p.bytes)
            return fail(POLYMUL_EIO, "server reservation of " + std::to_string(p.bytes) + " bytes is smaller than the " +
                                         std::to_string(4 * words * 8) + " bytes of the product's workspace");
        for (int k = 0; k < 4; ++k) v->ws[k] = reinterpret_cast<uint64_t *>(base + (size_t)k * words * 8);
        v->ws_words = words;
        if (r.fa)
            rc = resident_body(v, r.fa, r.res_log2n, r.b, r.lb, r.out, r.la + r.lb - 1, s);
        else
            rc = product_body(v, r.a, r.la, r.b, r.lb, r.out, s);
    } else {
        const uint32_t count = (uint32_t)p.reqs.size();
        const size_t wsb = batch_ws_bytes(v, count, p.max_lc);
        for (uint32_t k = 0; k < count; ++k) {
            const fpmul_srv::Req &r = p.reqs[k];
            slot.host_desc[k] = BtDesc{r.a, r.b, r.out, r.la, r.lb};
        }
        BtDesc *ddesc = reinterpret_cast<BtDesc *>(base + wsb);
        hipError_t e = hipMemcpyAsync(ddesc, slot.host_desc, (size_t)count * sizeof(BtDesc), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return fail(POLYMUL_EIO, std::string("copy batch descriptors: ") + hipGetErrorString(e));
        v->bws = base;
        v->bws_bytes = wsb;
        rc = batch_body(v, count, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, ddesc,
                        p.max_lc, nullptr, s);
    }
    if (rc) return rc;
    HIP_TRY(hipEventRecord(slot.done, s));
    return 0;
}

// the launcher thread of one slot: enqueues each plan the scheduler admits on
// the slot, without holding the server lock
static void srv_launcher(polymul_server *S, SrvSlot *slot)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->m);
    for (;;) {
        S->cv_launch.wait(lk, [S, slot] { return slot->go || S->stop_launchers; });
        if (!slot->go) break;
        slot->go = false;
        lk.unlock();
        const int rc = srv_launch(S, *slot);
        // nothing of a failed launch runs past this point
        if (rc) (void)hipStreamSynchronize(slot->stream);
        lk.lock();
        if (rc) {
            srv_finish(S, *slot, rc);   // the message of this thread's failure
            S->cv_done.notify_all();
        } else {
            slot->launched = true;
        }
        S->cv_work.notify_all();
    }
}

static void srv_loop(polymul_server *S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->m);
    for (;;) {
        // completions (an event not yet recorded reads as complete: only the
        // launched slots are asked)
        for (SrvSlot &slot : S->slots) {
            if (!slot.busy || !slot.launched) continue;
            hipError_t q = hipEventQuery(slot.done);
            if (q == hipErrorNotReady) continue;
            srv_finish(S, slot, q == hipSuccess ? 0 : fail(POLYMUL_EIO, hipGetErrorString(q)));
            S->cv_done.notify_all();
        }
        // admissions
        for (SrvSlot &slot : S->slots) {
            if (slot.busy) continue;
            if (!fpmul_srv::next_plan(S->pending, S->arena, S->policy, S->fp, slot.plan)) break;
            slot.busy = true;
            S->busy++;
            const uint64_t t = srv_now_ns(S->t0);
            for (const auto &r : slot.plan.reqs) {
                auto it = S->tickets.find(r.ticket);
                if (it == S->tickets.end()) continue;
                it->second.state = 1;
                it->second.t_start = t;
            }
            slot.go = true;
            S->cv_launch.notify_all();
        }
        if (S->stop && S->pending.empty() && S->busy == 0) break;
        if (S->busy)
            S->cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            S->cv_work.wait(lk, [S] { return S->stop || !S->pending.empty(); });
    }
}

extern "C" {

int polymul_server_create(polymul_server **out, polymul_ctx *ctx, size_t hbm_budget_bytes, uint32_t max_slots)
{
    if (!out) return fail(POLYMUL_EINVAL, "server out pointer is null");
    *out = nullptr;
    if (!ctx) return fail(POLYMUL_EINVAL, "ctx is null");
    if (max_slots < 1 || max_slots > 64) return fail(POLYMUL_EINVAL, "max_slots must be in [1, 64]");
    if (hbm_budget_bytes < (1u << 20)) return fail(POLYMUL_EINVAL, "hbm_budget_bytes must be at least 1 MiB");
    DeviceGuard g(ctx->device);
    HIP_TRY(g.err);
    int rc;
    if ((rc = batch_steps_upload(ctx)) || (rc = set_lds_limits())) return rc;
    std::unique_ptr<polymul_server> S(new polymul_server());
    S->ctx = ctx;
    polymul_ctx *parent = ctx;
    S->fp.single = [](uint64_t lc) { return srv_single_bytes(lc); };
    S->fp.batch = [parent](uint32_t count, uint64_t max_lc) {
        return (uint64_t)batch_ws_bytes(parent, count, max_lc) +
               fpmul_srv::Arena::round((uint64_t)count * sizeof(BtDesc));
    };
    hipError_t e = hipMalloc(&S->arena_base, hbm_budget_bytes);
    if (e != hipSuccess) return fail(POLYMUL_ENOMEM, std::string("hipMalloc server arena: ") + hipGetErrorString(e));
    S->arena.reset(hbm_budget_bytes);
    S->slots.resize(max_slots);
    for (SrvSlot &slot : S->slots) {
        e = hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&slot.host_desc, (size_t)4096 * sizeof(BtDesc), hipHostMallocDefault);
        if (e != hipSuccess) break;
        slot.view = new polymul_ctx();
        slot.view->device = ctx->device;
        slot.view->tables = ctx->tables;
        slot.view->psteps = ctx->psteps;
        slot.view->bsteps = ctx->bsteps;
        slot.view->num_cu = ctx->num_cu;
        slot.view->tuned = ctx->tuned;
        slot.view->small_field_log2n = ctx->small_field_log2n;
        slot.view->large_field_log2n = M64_MAX_LOG2N + 1;   // the server admits m = 64 products only
        slot.view->borrowed = true;
    }
    if (e != hipSuccess) {
        for (SrvSlot &slot : S->slots) {
            if (slot.stream) (void)hipStreamDestroy(slot.stream);
            if (slot.done) (void)hipEventDestroy(slot.done);
            if (slot.host_desc) (void)hipHostFree(slot.host_desc);
            delete slot.view;
        }
        (void)hipFree(S->arena_base);
        return fail(POLYMUL_EIO, std::string("server streams: ") + hipGetErrorString(e));
    }
    polymul_server *raw = S.release();
    for (SrvSlot &slot : raw->slots) slot.launcher = std::thread(srv_launcher, raw, &slot);
    raw->th = std::thread(srv_loop, raw);
    *out = raw;
    return 0;
}

int polymul_server_destroy(polymul_server *S)
{
    if (!S) return 0;
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->th.joinable()) S->th.join();   // every admitted plan has completed
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stop_launchers = true;
    }
    S->cv_launch.notify_all();
    for (SrvSlot &slot : S->slots)
        if (slot.launcher.joinable()) slot.launcher.join();
    DeviceGuard g(S->ctx->device);
    for (SrvSlot &slot : S->slots) {
        if (slot.stream) (void)hipStreamSynchronize(slot.stream);
        if (slot.stream) (void)hipStreamDestroy(slot.stream);
        if (slot.done) (void)hipEventDestroy(slot.done);
        if (slot.host_desc) (void)hipHostFree(slot.host_desc);
        delete slot.view;   // borrowed buffers: nothing of its own to free
    }
    if (S->arena_base) (void)hipFree(S->arena_base);
    delete S;
    return 0;
}

int polymul_server_set_policy(polymul_server *S, uint64_t batch_limit_bits, uint32_t max_batch)
{
    if (!S) return fail(POLYMUL_EINVAL, "server is null");
    if (batch_limit_bits > POLYMUL_BATCH_MAX_PRODUCT_BITS || max_batch < 1 || max_batch > 4096)
        return fail(POLYMUL_EINVAL, "policy out of range");
    std::lock_guard<std::mutex> lk(S->m);
    if (S->next_ticket != 1) return fail(POLYMUL_EINVAL, "policy must be set before the first submit");
    S->policy.batch_limit_bits = batch_limit_bits;
    S->policy.max_batch = max_batch;
    return 0;
}

int polymul_submit(polymul_server *S, const uint64_t *a, uint64_t len_a, const uint64_t *b, uint64_t len_b,
                   uint64_t *out, uint64_t *ticket)
{
    if (!S || !ticket) return fail(POLYMUL_EINVAL, "server or ticket pointer is null");
    *ticket = 0;
    const bool empty = len_a == 0 || len_b == 0;
    if (!empty) {
        if (len_a > POLYMUL_SERVER_MAX_PRODUCT_BITS || len_b > POLYMUL_SERVER_MAX_PRODUCT_BITS ||
            len_a + len_b - 1 > POLYMUL_SERVER_MAX_PRODUCT_BITS)
            return fail(POLYMUL_EINVAL, "product length exceeds 2^37 bits");
        DeviceGuard g(S->ctx->device);
        HIP_TRY(g.err);
        int rc;
        if ((rc = check_dev_ptr(a, "a_bits")) || (rc = check_dev_ptr(b, "b_bits")) ||
            (rc = check_dev_ptr(out, "out")))
            return rc;
        const uint64_t lc = len_a + len_b - 1;
        const size_t ob = (size_t)((lc + 63) / 64) * 8;
        if (ranges_overlap(out, ob, a, (size_t)((len_a + 63) / 64) * 8) ||
            ranges_overlap(out, ob, b, (size_t)((len_b + 63) / 64) * 8))
            return fail(POLYMUL_EINVAL, "out overlaps an input");
        const uint64_t need = lc <= S->policy.batch_limit_bits ? S->fp.batch(1, lc) : S->fp.single(lc);
        if (fpmul_srv::Arena::round(need) > S->arena.size())
            return fail(POLYMUL_ENOMEM, "request needs " + std::to_string(need) + " bytes, more than the server budget");
    }
    {
        std::lock_guard<std::mutex> lk(S->m);
        const uint64_t id = S->next_ticket++;
        SrvTicket &tk = S->tickets[id];
        tk.t_submit = srv_now_ns(S->t0);
        if (empty) {
            tk.state = 2;
            tk.t_start = tk.t_done = tk.t_submit;
        } else {
            fpmul_srv::Req r;
            r.ticket = id;
            r.la = len_a;
            r.lb = len_b;
            r.a = a;
            r.b = b;
            r.out = out;
            S->pending.push_back(r);
        }
        *ticket = id;
    }
    S->cv_work.notify_all();
    return 0;
}

int polymul_submit_resident(polymul_server *S, const polymul_resident *res, const uint64_t *b, uint64_t len_b,
                            uint64_t *out, uint64_t *ticket)
{
    if (!S || !ticket || !res) return fail(POLYMUL_EINVAL, "server, resident operand or ticket pointer is null");
    *ticket = 0;
    if (res->device != S->ctx->device) return fail(POLYMUL_EINVAL, "resident operand is on another device");
    const bool empty = len_b == 0;
    if (!empty) {
        if (res->len_a + len_b - 1 > (1ull << res->log2n))
            return fail(POLYMUL_EINVAL, "product longer than the resident operand's transform");
        DeviceGuard g(S->ctx->device);
        HIP_TRY(g.err);
        int rc;
        if ((rc = check_dev_ptr(b, "b_bits")) || (rc = check_dev_ptr(out, "out"))) return rc;
        const uint64_t lc = res->len_a + len_b - 1;
        if (ranges_overlap(out, (size_t)((lc + 63) / 64) * 8, b, (size_t)((len_b + 63) / 64) * 8))
            return fail(POLYMUL_EINVAL, "out overlaps an input");
        const uint64_t need = S->fp.single(1ull << res->log2n);
        if (fpmul_srv::Arena::round(need) > S->arena.size())
            return fail(POLYMUL_ENOMEM, "request needs " + std::to_string(need) + " bytes, more than the server budget");
    }
    {
        std::lock_guard<std::mutex> lk(S->m);
        const uint64_t id = S->next_ticket++;
        SrvTicket &tk = S->tickets[id];
        tk.t_submit = srv_now_ns(S->t0);
        if (empty) {
            tk.state = 2;
            tk.t_start = tk.t_done = tk.t_submit;
        } else {
            fpmul_srv::Req r;
            r.ticket = id;
            r.la = res->len_a;
            r.lb = len_b;
            r.b = b;
            r.out = out;
            r.fa = res->vals;
            r.res_log2n = res->log2n;
            S->pending.push_back(r);
        }
        *ticket = id;
    }
    S->cv_work.notify_all();
    return 0;
}

int polymul_poll(polymul_server *S, uint64_t ticket, int *done)
{
    if (!S || !done) return fail(POLYMUL_EINVAL, "server or done pointer is null");
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(POLYMUL_EINVAL, "unknown ticket");
    *done = it->second.state == 2;
    if (*done && it->second.rc) return fail(it->second.rc, it->second.err);
    return 0;
}

// wait for a ticket, read its times, and forget it
static int srv_wait_release(polymul_server *S, uint64_t ticket, uint64_t *submit_ns, uint64_t *start_ns,
                            uint64_t *done_ns)
{
    std::unique_lock<std::mutex> lk(S->m);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(POLYMUL_EINVAL, "unknown ticket");
    // a rehash by another submit invalidates iterators but not the element's address
    const SrvTicket *tp = &it->second;
    S->cv_done.wait(lk, [tp] { return tp->state == 2; });
    const SrvTicket tk = *tp;
    S->tickets.erase(ticket);
    if (submit_ns) *submit_ns = tk.t_submit;
    if (start_ns) *start_ns = tk.t_start;
    if (done_ns) *done_ns = tk.t_done;
    if (tk.rc) return fail(tk.rc, tk.err);
    return 0;
}

int polymul_wait(polymul_server *S, uint64_t ticket)
{
    if (!S) return fail(POLYMUL_EINVAL, "server is null");
    return srv_wait_release(S, ticket, nullptr, nullptr, nullptr);
}

int polymul_wait_times(polymul_server *S, uint64_t ticket, uint64_t *submit_ns, uint64_t *start_ns,
                       uint64_t *done_ns)
{
    if (!S) return fail(POLYMUL_EINVAL, "server is null");
    return srv_wait_release(S, ticket, submit_ns, start_ns, done_ns);
}

int polymul_ticket_times(polymul_server *S, uint64_t ticket, uint64_t *submit_ns, uint64_t *start_ns,
                         uint64_t *done_ns)
{
    if (!S) return fail(POLYMUL_EINVAL, "server is null");
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(POLYMUL_EINVAL, "unknown ticket");
    if (submit_ns) *submit_ns = it->second.t_submit;
    if (start_ns) *start_ns = it->second.t_start;
    if (done_ns) *done_ns = it->second.t_done;
    return 0;
}

int polymul_server_tickets(polymul_server *S, uint64_t *count)
{
    if (!S || !count) return fail(POLYMUL_EINVAL, "server or count pointer is null");
    std::lock_guard<std::mutex> lk(S->m);
    *count = S->tickets.size();
    return 0;
}

}  // extern "C"
