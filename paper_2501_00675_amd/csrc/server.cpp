// Serving runtime: admission by slot and HBM footprint, continuous batching of
// level-synchronous steps, latency stamps (cos_server_* in cos.h).
//
// One scheduling thread owns all device work of a server.  A step is a replay
// of an instantiated graph (step-table upload, then the whole-graph and the
// streamed step kernels side by side) on the work stream, followed by an
// event; a host callback on a second stream waits for that event, so the
// callback never stands between two steps on the work stream.  Two step
// tables alternate so the thread can queue step k+1 while step k runs (stream
// order keeps every request's stages in sequence).  The callback, which must
// not call HIP, only marks the requests that finished in its step and wakes
// the thread.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "fused_plan.h"
#include "serve_sched.h"
#include "serve_types.h"

namespace cosdag {
namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum ReqState { RS_QUEUED, RS_ACTIVE, RS_DONE, RS_CANCELED, RS_FAILED };

struct Request {
    uint64_t ticket = 0;
    int bypassed = 0;  // later requests admitted ahead of this one (admit bounds it)
    const Graph *g = nullptr;
    const double *x = nullptr;
    double *out = nullptr;
    int32_t *out_exp = nullptr;
    int64_t S = 0;
    cos_precision p = COS_FP64;
    bool fused = false;
    bool table32 = false;    // streamed lookup request at binary32: its first stage copies the tables
    int section = SS_FUSED;  // ServeSection of its work
    FusedLayout flay;
    Workspace wlay;
    uint64_t footprint = 0, arena_off = 0;
    int slot = -1;
    int next_stage = 0, n_stages = 0;  // stages issued so far / in total
    int steps = 0;
    int64_t first_step = -1;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    ReqState state = RS_QUEUED;
    cos_status status = COS_EAGAIN;
};

struct StepBuf {
    StepTable *h_tab = nullptr;     // pinned
    StepTable *d_tab = nullptr;
    hipGraphExec_t exec = nullptr;         // rational-factor sections
    hipGraphExec_t exec_lookup = nullptr;  // all four sections
    hipEvent_t done = nullptr;             // recorded on the work stream after the step's graph
    bool busy = false;
    bool lookup = false;               // the step has lookup-factor work (replay exec_lookup)
    std::vector<Request *> finishing;  // requests whose last stage is in this step
    cos_step_record rec{};             // the step's trace record (t_done_ns set on completion)
    struct Server *srv = nullptr;
};

constexpr size_t kTraceKeep = 65536;  // unread step records kept

}  // namespace
}  // namespace cosdag

struct cos_server {
    cosdag::Request *dummy = nullptr;
};

namespace cosdag {
namespace {

struct Server : cos_server {
    int device = 0;
    uint64_t budget = 0;
    int max_slots = 0;
    std::vector<const Graph *> graphs;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::vector<Request *> slots;
    Arena arena{0};
    uint64_t next_ticket = 1;
    bool stop = false;
    int inflight = 0;
    cos_server_stats st{};
    // device
    hipStream_t stream = nullptr;     // every step, set-up copy and fill, in order
    hipStream_t cb_stream = nullptr;  // completion callbacks, each after its step's event, so that a
                                      // callback never holds back the next step on the work stream
    char *d_arena = nullptr;
    ServeReqDev *d_reqs = nullptr;
    std::vector<StepSetup> pending_setup;  // set-up of admitted requests not yet carried by a step
    StepBuf bufs[2];
    std::thread worker;

    std::deque<cos_step_record> trace;  // completed steps not read yet
    int64_t admissions = 0;         // requests admitted so far (their admission index)
    int64_t fail_admission_at = -1;  // test hook: this admission's set-up is made to fail

    ~Server();
    void run();
    StepSetup setup_entry(const Request *r) const;
    void fail_request(Request *r);
};

void step_done(void *p) {
    StepBuf *b = static_cast<StepBuf *>(p);
    Server *s = b->srv;
    const int64_t t = now_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Request *r : b->finishing) {
            if (r->state != RS_ACTIVE)
                continue;  // failed while this step was in flight
            r->t_done = t;
            r->state = RS_DONE;
            r->status = COS_OK;
            if (r->footprint)
                s->arena.release(r->arena_off, r->footprint);
            s->slots[r->slot] = nullptr;
            ++s->st.completed;
        }
        b->finishing.clear();
        b->rec.t_done_ns = t;
        s->trace.push_back(b->rec);
        if (s->trace.size() > kTraceKeep)
            s->trace.pop_front();
        b->busy = false;
        --s->inflight;
    }
    s->cv.notify_all();
}

uint32_t stage_items(const Request &r, int stage, uint32_t *n_rg, uint32_t *kind, uint32_t *level) {
    const Graph &g = *r.g;
    if (r.fused) {
        *kind = SK_FUSED;
        *level = 0;
        *n_rg = 1;
        return static_cast<uint32_t>((r.S + kWave - 1) / kWave);
    }
    if (r.table32) {
        if (stage == 0) {
            *kind = SK_TABLE32;
            *level = 0;
            *n_rg = 1;
            return static_cast<uint32_t>(static_cast<int64_t>(g.n_slots) * r.wlay.S_pad / kServeCombineTile);
        }
        --stage;
    }
    const int L = g.L;
    if (stage < L - 1) {  // interior level stage + 1
        const int l = stage + 1;
        *kind = SK_LEVEL;
        *level = static_cast<uint32_t>(l);
        *n_rg = static_cast<uint32_t>((g.levels[l - 1].w_dst + kServeLevelRowsPerItem - 1) / kServeLevelRowsPerItem);
        return *n_rg * static_cast<uint32_t>(r.wlay.S_pad / (kWave * kServeLevelK));
    }
    if (stage == L - 1) {
        *kind = SK_FINAL;
        *level = static_cast<uint32_t>(L);
        *n_rg = static_cast<uint32_t>(r.wlay.final_chunks);
        return *n_rg * static_cast<uint32_t>(r.wlay.S_pad / (kWave * kServeFinalK));
    }
    *kind = SK_COMBINE;
    *level = static_cast<uint32_t>(L);
    *n_rg = 1;
    return static_cast<uint32_t>((r.S + kServeCombineTile - 1) / kServeCombineTile);
}

// A newly admitted request's slot entry and exponent-row initial value (host
// only: the set-up kernel of the first step that includes the request writes
// them on the device).
StepSetup Server::setup_entry(const Request *r) const {
    const Graph &g = *r->g;
    StepSetup su{};
    su.slot = static_cast<uint32_t>(r->slot);
    ServeReqDev &d = su.req;
    d.row_ptr = g.d_row_ptr;
    d.edges = g.d_edges;
    d.edges32 = g.d_edges32;
    d.edgesL = g.d_edgesL;
    d.levels = g.d_levels;
    d.h16 = g.d_h16;
    d.x = r->x;
    d.out = r->out;
    d.out_exp = r->out_exp;
    d.ws = r->footprint ? d_arena + r->arena_off : nullptr;
    d.S = r->S;
    d.S_pad = r->fused ? 0 : r->wlay.S_pad;
    d.off_buf0 = r->wlay.off_buf0;
    d.off_buf1 = r->wlay.off_buf1;
    d.off_maxbits = r->wlay.off_maxbits;
    d.off_partial = r->wlay.off_partial;
    d.L = g.L;
    d.precision = r->p;
    d.rows_variant = rows_variant((g.max_width + kFusedWaves - 1) / kFusedWaves);
    d.final_chunks = r->wlay.final_chunks;
    d.n_slots = g.n_slots;
    d.t32 = r->table32 ? reinterpret_cast<float *>(d.ws + r->wlay.off_table32) : nullptr;
    d.off_red = static_cast<uint32_t>(r->flay.off_red);
    d.off_part = static_cast<uint32_t>(r->flay.off_part);
    // exponent rows: row 0 holds level 1's headroom 2^h_1 (binary16; else 0 = no
    // shift), rows 1..L start at zero for the levels' maxima
    if (!r->fused && is_rescaled(r->p)) {
        const int32_t h1 = r->p == COS_FP16_RESCALED && g.L >= 2 ? g.h16[1] : 0;
        su.fill = 1;
        su.row0 = h1 ? static_cast<uint32_t>(127 + h1) << 23 : 0u;
    }
    return su;
}

// Mark an active request failed and give back its slot and workspace (under the lock).
void Server::fail_request(Request *r) {
    r->state = RS_FAILED;
    r->status = COS_EDEVICE;
    r->t_done = now_ns();
    ++st.failed;
    if (r->footprint)
        arena.release(r->arena_off, r->footprint);
    slots[r->slot] = nullptr;
}

void Server::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        // ---- admission (host bookkeeping under the lock)
        const std::vector<Request *> admitted = admit(queue, slots, arena);
        std::vector<int64_t> admission_index;
        for (Request *r : admitted) {
            r->state = RS_ACTIVE;
            r->t_admit = now_ns();
            admission_index.push_back(admissions++);
        }

        // ---- set-up of the admitted requests (slot entry, exponent rows), carried by the next step, which
        // is the first to include them.  A request whose set-up fails fails alone.
        if (!admitted.empty()) {
            bool failed = false;
            for (size_t i = 0; i < admitted.size(); ++i) {
                if (admission_index[i] == fail_admission_at) {
                    fail_request(admitted[i]);
                    failed = true;
                } else {
                    pending_setup.push_back(setup_entry(admitted[i]));
                }
            }
            if (failed)
                cv.notify_all();
        }
        int active = 0;
        for (Request *r : slots)
            active += r != nullptr;
        st.max_active = std::max<int64_t>(st.max_active, active);
        st.peak_bytes = std::max<uint64_t>(st.peak_bytes, arena.used());

        // ---- next step, if a table is free and some request has a stage left
        StepBuf *b = nullptr;
        for (StepBuf &cand : bufs)
            if (!cand.busy) {
                b = &cand;
                break;
            }
        if (b && any_stage_left(slots)) {
            // whole-graph (fused) entries first, then level / final / combine entries
            StepTable &t = *b->h_tab;
            uint32_t n = 0, items[SS_COUNT] = {}, count[SS_COUNT] = {};
            compose_step(slots, SS_COUNT, [&](int section, Request *r) {
                StepEntry &e = t.e[n++];
                e.slot = static_cast<uint32_t>(r->slot);
                e.n_items = stage_items(*r, r->next_stage, &e.n_rg, &e.kind, &e.level);
                e.item_base = items[section];
                items[section] += e.n_items;
                ++count[section];
                if (r->first_step < 0)
                    r->first_step = st.steps;
                ++r->steps;
                if (r->next_stage + 1 == r->n_stages)
                    b->finishing.push_back(r);
            });
            for (auto &per_section : t.claimed)
                for (auto &c : per_section)
                    c.v = 0;
            t.n_setup = static_cast<uint32_t>(pending_setup.size());
            std::copy(pending_setup.begin(), pending_setup.end(), t.setup);
            pending_setup.clear();
            int64_t all_items = 0;
            for (uint32_t sec = 0; sec < SS_COUNT; ++sec) {
                t.n[sec] = count[sec];
                t.items[sec] = items[sec];
                all_items += items[sec];
            }
            b->lookup = count[SS_FUSED_LOOKUP] + count[SS_STREAMED_LOOKUP] > 0;
            b->rec = cos_step_record{st.steps, now_ns(), 0,
                                     static_cast<int32_t>(count[SS_FUSED] + count[SS_FUSED_LOOKUP]),
                                     static_cast<int32_t>(count[SS_STREAMED] + count[SS_STREAMED_LOOKUP]),
                                     all_items};
            b->busy = true;
            ++inflight;
            ++st.steps;
            st.items += all_items;
            st.max_step_requests = std::max<int64_t>(st.max_step_requests, n);
        } else {
            b = nullptr;
        }

        if (!b) {
            if (admitted.empty()) {
                if (stop && queue.empty() && inflight == 0) {
                    bool idle = true;
                    for (Request *r : slots)
                        idle &= r == nullptr;
                    if (idle)
                        break;
                }
                cv.wait(lk);
            }
            continue;
        }

        // ---- the step: one replay of the step graph, then the completion callback
        lk.unlock();
        hipError_t err = hipSuccess;
        {
            TimedLaunch tl(KK_SERVE, stream);
            err = hipGraphLaunch(b->lookup ? b->exec_lookup : b->exec, stream);
        }
        if (err == hipSuccess)
            err = hipEventRecord(b->done, stream);
        if (err == hipSuccess)
            err = hipStreamWaitEvent(cb_stream, b->done, 0);
        if (err == hipSuccess)
            err = hipLaunchHostFunc(cb_stream, step_done, b);
        lk.lock();
        if (err != hipSuccess) {
            // the device is unusable for this server: fail every active request (set-ups not yet
            // carried by a step belong to them)
            for (Request *r : slots)
                if (r)
                    fail_request(r);
            pending_setup.clear();
            b->finishing.clear();
            b->busy = false;
            --inflight;
            cv.notify_all();
        }
    }
}

Server::~Server() {
    for (StepBuf &b : bufs) {
        if (b.exec)
            (void)hipGraphExecDestroy(b.exec);
        if (b.exec_lookup)
            (void)hipGraphExecDestroy(b.exec_lookup);
        if (b.d_tab)
            (void)hipFree(b.d_tab);
        if (b.h_tab)
            (void)hipHostFree(b.h_tab);
        if (b.done)
            (void)hipEventDestroy(b.done);
    }
    if (d_reqs)
        (void)hipFree(d_reqs);
    if (d_arena)
        (void)hipFree(d_arena);
    if (stream)
        (void)hipStreamDestroy(stream);
    if (cb_stream)
        (void)hipStreamDestroy(cb_stream);
}

Server *server_of(cos_server *s) { return static_cast<Server *>(s); }

}  // namespace
}  // namespace cosdag

using namespace cosdag;

extern "C" cos_status cos_server_create(uint64_t hbm_budget, int32_t max_slots, cos_server **out) {
    if (!out)
        return fail(COS_EINVAL, "cos_server_create: out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > kServeMaxEntries)
        return fail(COS_EINVAL, "cos_server_create: max_slots must be in 1.." + std::to_string(kServeMaxEntries));
    try {
        auto s = std::make_unique<Server>();
        s->budget = hbm_budget;
        s->max_slots = max_slots;
        s->slots.assign(max_slots, nullptr);
        s->arena = Arena(hbm_budget);
        s->st.budget_bytes = hbm_budget;
        hipError_t err = hipGetDevice(&s->device);
        if (err == hipSuccess)
            err = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (err == hipSuccess)
            err = hipStreamCreateWithFlags(&s->cb_stream, hipStreamNonBlocking);
        if (err == hipSuccess && hbm_budget)
            err = hipMalloc(reinterpret_cast<void **>(&s->d_arena), hbm_budget);
        if (err == hipSuccess)
            err = hipMalloc(reinterpret_cast<void **>(&s->d_reqs), sizeof(ServeReqDev) * max_slots);
        for (StepBuf &b : s->bufs) {
            b.srv = s.get();
            if (err == hipSuccess)
                err = hipHostMalloc(reinterpret_cast<void **>(&b.h_tab), sizeof(StepTable), hipHostMallocDefault);
            if (err == hipSuccess)
                err = hipMalloc(reinterpret_cast<void **>(&b.d_tab), sizeof(StepTable));
            if (err == hipSuccess)
                err = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
            if (err == hipSuccess)
                err = serve_build_step_graph(b.d_tab, b.h_tab, s->d_reqs, false, &b.exec);
            if (err == hipSuccess)
                err = serve_build_step_graph(b.d_tab, b.h_tab, s->d_reqs, true, &b.exec_lookup);
        }
        if (err != hipSuccess)
            return hip_fail(err, "cos_server_create");
        Server *raw = s.get();
        raw->worker = std::thread([raw] { raw->run(); });
        *out = s.release();
        return COS_OK;
    } catch (const std::bad_alloc &) {
        return fail(COS_ENOMEM, "cos_server_create: host allocation failed");
    } catch (const std::exception &e) {
        return fail(COS_EDEVICE, std::string("cos_server_create: ") + e.what());
    }
}

extern "C" cos_status cos_server_add_graph(cos_server *h, const cos_graph *g, int32_t *gid) {
    if (!h || !g || !gid)
        return fail(COS_EINVAL, "cos_server_add_graph: NULL argument");
    Server *s = server_of(h);
    const Graph &G = graph_of(g);
    if (G.device != s->device)
        return fail(COS_EINVAL, "cos_server_add_graph: graph lives on another device");
    std::lock_guard<std::mutex> lk(s->mu);
    s->graphs.push_back(&G);
    *gid = static_cast<int32_t>(s->graphs.size() - 1);
    return COS_OK;
}

extern "C" cos_status cos_server_submit(cos_server *h, int32_t gid, const double *x_dev, int64_t S, cos_precision p,
                                        double *out_dev, int32_t *out_exp_dev, uint64_t *ticket) {
    if (!h || !x_dev || !out_dev || !ticket)
        return fail(COS_EINVAL, "cos_server_submit: NULL argument");
    if (p != COS_FP64 && p != COS_FP32_RESCALED && p != COS_FP32 && p != COS_FP16_RESCALED &&
        p != COS_BF16_RESCALED)
        return fail(COS_EINVAL, "cos_server_submit: unknown precision");
    if (S < 1 || S > INT32_MAX)
        return fail(COS_EINVAL, "cos_server_submit: S must be in 1..2^31-1");
    Server *s = server_of(h);
    auto r = std::make_unique<Request>();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (gid < 0 || gid >= static_cast<int32_t>(s->graphs.size()))
            return fail(COS_EINVAL, "cos_server_submit: unknown graph id");
        r->g = s->graphs[gid];
    }
    const Graph &g = *r->g;
    // the conditions cos_evaluate refuses for 16-bit storage
    if (check_precision_range(g, p, "cos_server_submit") != COS_OK)
        return COS_EINVAL;
    if (value_bytes(p) == 2 && g.path == COS_PATH_FUSED)
        return fail(COS_EINVAL, "cos_server_submit: 16-bit level storage runs on the streamed plan only");
    if (p == COS_FP16_RESCALED && g.h16.empty())
        return fail(COS_EINVAL, "cos_server_submit: binary16 storage needs rational factors with level row sums of "
                                "|a| below 2^110 (use COS_BF16_RESCALED or COS_FP32_RESCALED)");
    r->x = x_dev;
    r->out = out_dev;
    r->out_exp = out_exp_dev;
    r->S = S;
    r->p = p;
    // the same plan choice cos_evaluate makes for this graph (results are bit-identical to it)
    r->fused = g.path == COS_PATH_FUSED || (g.path == COS_PATH_AUTO && fused_fits(g, p));
    r->section = (r->fused ? SS_FUSED : SS_STREAMED) + (g.kind == FK_LOOKUP ? SS_FUSED_LOOKUP : 0);
    if (r->fused) {
        if (!fused_fits(g, p))
            return fail(COS_EINVAL, "cos_server_submit: fused plan requested but the graph does not fit in LDS");
        r->flay = fused_layout(g, p == COS_FP64 ? sizeof(double) : sizeof(float), p == COS_FP32_RESCALED, 1);
        r->n_stages = 1;
    } else {
        if (max_chunk(g, p) < S)
            return fail(COS_EINVAL, "cos_server_submit: S too large for one sweep; use cos_evaluate");
        r->table32 = uses_table32(g, p);
        r->wlay = layout_for_chunk(g, S, p, r->table32);
        r->footprint = r->wlay.bytes;
        r->n_stages = g.L + 1 + (r->table32 ? 1 : 0);
        if (r->footprint > s->budget)
            return fail(COS_ENOMEM, "cos_server_submit: the request's workspace (" + std::to_string(r->footprint) +
                                        " bytes) exceeds the server's HBM budget");
    }
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop)
            return fail(COS_EINVAL, "cos_server_submit: server is shutting down");
        r->ticket = s->next_ticket++;
        *ticket = r->ticket;
        s->queue.push_back(r.get());
        s->reqs.emplace(r->ticket, std::move(r));
        ++s->st.submitted;
    }
    s->cv.notify_all();
    return COS_OK;
}

namespace {
cos_status finish_poll(Server *s, std::unordered_map<uint64_t, std::unique_ptr<Request>>::iterator it,
                       cos_req_stats *out) {
    Request *r = it->second.get();
    if (out) {
        out->t_submit_ns = r->t_submit;
        out->t_admit_ns = r->t_admit;
        out->t_done_ns = r->t_done;
        out->status = r->status;
        out->steps = r->steps;
        out->first_step = r->first_step;
        out->footprint = static_cast<int64_t>(r->footprint);
    }
    if (r->state == RS_QUEUED || r->state == RS_ACTIVE)
        return COS_EAGAIN;
    const cos_status st = r->status;
    bool referenced = false;  // a failed request may still be listed by a step in flight
    for (const StepBuf &b : s->bufs)
        referenced |= std::find(b.finishing.begin(), b.finishing.end(), r) != b.finishing.end();
    if (!referenced)
        s->reqs.erase(it);
    return st;
}
}  // namespace

extern "C" cos_status cos_server_poll(cos_server *h, uint64_t ticket, cos_req_stats *stats) {
    if (!h)
        return fail(COS_EINVAL, "cos_server_poll: server is NULL");
    Server *s = server_of(h);
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return fail(COS_EINVAL, "cos_server_poll: unknown ticket");
    return finish_poll(s, it, stats);
}

extern "C" cos_status cos_server_wait(cos_server *h, uint64_t ticket, cos_req_stats *stats) {
    if (!h)
        return fail(COS_EINVAL, "cos_server_wait: server is NULL");
    Server *s = server_of(h);
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return fail(COS_EINVAL, "cos_server_wait: unknown ticket");
    Request *r = it->second.get();
    s->cv.wait(lk, [r] { return r->state != RS_QUEUED && r->state != RS_ACTIVE; });
    return finish_poll(s, s->reqs.find(ticket), stats);
}

extern "C" cos_status cos_server_cancel(cos_server *h, uint64_t ticket) {
    if (!h)
        return fail(COS_EINVAL, "cos_server_cancel: server is NULL");
    Server *s = server_of(h);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end())
            return fail(COS_EINVAL, "cos_server_cancel: unknown ticket");
        Request *r = it->second.get();
        if (r->state != RS_QUEUED)
            return r->state == RS_ACTIVE ? COS_EAGAIN : COS_OK;
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
        r->state = RS_CANCELED;
        r->status = COS_ECANCELED;
        r->t_done = now_ns();
        ++s->st.cancelled;
    }
    s->cv.notify_all();
    return COS_OK;
}

extern "C" cos_status cos_server_read_steps(cos_server *h, cos_step_record *out, int64_t cap, int64_t *n) {
    if (!h || !n)
        return fail(COS_EINVAL, "cos_server_read_steps: NULL argument");
    if (cap < 0 || (cap > 0 && !out))
        return fail(COS_EINVAL, "cos_server_read_steps: bad cap or out");
    Server *s = server_of(h);
    std::lock_guard<std::mutex> lk(s->mu);
    int64_t k = 0;
    while (k < cap && !s->trace.empty()) {
        out[k++] = s->trace.front();
        s->trace.pop_front();
    }
    *n = k;
    return COS_OK;
}

extern "C" cos_status cos_server_fail_admission(cos_server *h, int64_t admission_index) {
    if (!h)
        return fail(COS_EINVAL, "cos_server_fail_admission: server is NULL");
    if (admission_index < -1)
        return fail(COS_EINVAL, "cos_server_fail_admission: index must be >= -1");
    Server *s = server_of(h);
    std::lock_guard<std::mutex> lk(s->mu);
    s->fail_admission_at = admission_index;
    return COS_OK;
}

extern "C" cos_status cos_server_get_stats(cos_server *h, cos_server_stats *out) {
    if (!h || !out)
        return fail(COS_EINVAL, "cos_server_get_stats: NULL argument");
    Server *s = server_of(h);
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return COS_OK;
}

extern "C" cos_status cos_server_destroy(cos_server *h) {
    if (!h)
        return COS_OK;
    Server *s = server_of(h);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Request *r : s->queue) {
            r->state = RS_CANCELED;
            r->status = COS_ECANCELED;
            ++s->st.cancelled;
        }
        s->queue.clear();
    }
    s->cv.notify_all();
    if (s->worker.joinable())
        s->worker.join();
    hipError_t err = hipStreamSynchronize(s->stream);
    const hipError_t cb_err = hipStreamSynchronize(s->cb_stream);
    if (err == hipSuccess)
        err = cb_err;
    delete s;
    if (err != hipSuccess)
        return hip_fail(err, "cos_server_destroy");
    return COS_OK;
}
