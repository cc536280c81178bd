// Serving loop: continuous batching of filtered queries against one
// HBM-resident index.
//
// Requests (one query vector and its constraint pairs, copied at submit)
// wait in a bounded queue.  A scheduler thread owns `streams` batch slots;
// whenever a slot is free and requests wait, it takes the oldest ones (up
// to the batch cap, optionally waiting up to `batch_window_us` for a batch
// to fill), packs them into pinned host buffers, and enqueues on the slot's
// stream: host-to-device copies, one search call, device-to-host copies and
// an event.  Slots run concurrently, so copies and kernels of different
// batches overlap.  Finished slots are retired in completion order: each
// request's ids and distances go to a result queue with its latency (submit
// to the moment the scheduler sees the event complete).
//
// Admission: submit refuses (EBUSY) beyond `queue_slots` waiting requests
// and rejects non-finite query rows (EINVAL).  Device memory: the search
// workspaces of all batches in flight share `workspace_bytes`; a batch is
// sized to the largest count whose workspace (exact bytes of the search's
// own layout) fits what the batches in flight leave free, and waits for a
// retirement when not even one query fits.  A query's result does not
// depend on the batch it lands in: every search kernel is batch invariant.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "caps_internal.h"

namespace caps {

using Clock = std::chrono::steady_clock;

// Waiting requests, oldest first from `head`: query rows (d floats each),
// constraint pairs, and per request its ticket, submit time and number of
// constraints.  Flat arrays, so that submitting and batching allocate
// nothing per request; consumed entries are dropped once the head passes
// half of the arrays.
struct ReqQueue {
    std::vector<float> q;
    std::vector<int32_t> attr, val;
    std::vector<uint64_t> ticket;
    std::vector<Clock::time_point> t0;
    std::vector<int32_t> ncon;
    size_t head = 0, chead = 0;   // first waiting request and its first constraint
    size_t size() const { return ticket.size() - head; }
    bool empty() const { return size() == 0; }
    void compact(size_t d) {
        if (head == 0 || head * 2 < ticket.size()) return;
        ticket.erase(ticket.begin(), ticket.begin() + (ptrdiff_t)head);
        t0.erase(t0.begin(), t0.begin() + (ptrdiff_t)head);
        ncon.erase(ncon.begin(), ncon.begin() + (ptrdiff_t)head);
        q.erase(q.begin(), q.begin() + (ptrdiff_t)(head * d));
        attr.erase(attr.begin(), attr.begin() + (ptrdiff_t)chead);
        val.erase(val.begin(), val.begin() + (ptrdiff_t)chead);
        head = chead = 0;
    }
};

// Finished requests, oldest first from `head`: ticket, latency, status and
// k ids and distances each (flat, like the request queue).
struct DoneQueue {
    std::vector<uint64_t> ticket;
    std::vector<float> lat;
    std::vector<int32_t> status;
    std::vector<int32_t> ids;
    std::vector<float> dist;
    size_t head = 0;
    size_t size() const { return ticket.size() - head; }
    void compact(size_t k) {
        if (head == 0 || head * 2 < ticket.size()) return;
        ticket.erase(ticket.begin(), ticket.begin() + (ptrdiff_t)head);
        lat.erase(lat.begin(), lat.begin() + (ptrdiff_t)head);
        status.erase(status.begin(), status.begin() + (ptrdiff_t)head);
        ids.erase(ids.begin(), ids.begin() + (ptrdiff_t)(head * k));
        dist.erase(dist.begin(), dist.begin() + (ptrdiff_t)(head * k));
        head = 0;
    }
};

struct SrvSlot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    caps_status status = CAPS_OK;
    size_t ws_bytes = 0;                   // workspace reserved by the batch in flight
    std::vector<uint64_t> tickets;         // the batch in flight
    std::vector<Clock::time_point> t0s;
    float *hq = nullptr, *hdist = nullptr, *dq = nullptr, *ddist = nullptr;
    int32_t *hoff = nullptr, *hattr = nullptr, *hval = nullptr, *hids = nullptr;
    int32_t *doff = nullptr, *dattr = nullptr, *dval = nullptr, *dids = nullptr;
};

struct Server {
    const Index *ix = nullptr;
    caps_server_params p{};
    caps_search_params sp{};
    int32_t d = 0, k = 0, cap = 0;
    size_t inflight = 0;               // workspace bytes reserved by batches in flight (scheduler thread)
    std::mutex mu;
    std::condition_variable cv;        // new request / stop (scheduler side)
    std::condition_variable cv_done;   // a batch retired (drain side)
    ReqQueue pending;
    DoneQueue done;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, rejected = 0, failed = 0, batches = 0, batched = 0;
    std::vector<double> lat;
    Clock::time_point t_first{}, t_last{};
    bool have_first = false;
    std::string err;
    std::vector<SrvSlot> slots;
    std::thread worker;
};

static void retire(Server *S, SrvSlot &sl) {
    const Clock::time_point t = Clock::now();
    const size_t nb = sl.tickets.size(), k = (size_t)S->k;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        DoneQueue &D = S->done;
        for (size_t i = 0; i < nb; i++) {
            const double ms = std::chrono::duration<double, std::milli>(t - sl.t0s[i]).count();
            S->lat.push_back(ms);
            D.ticket.push_back(sl.tickets[i]);
            D.lat.push_back((float)ms);
            D.status.push_back(sl.status);
        }
        const size_t o = D.ids.size();
        if (sl.status == CAPS_OK) {
            D.ids.insert(D.ids.end(), sl.hids, sl.hids + nb * k);
            D.dist.insert(D.dist.end(), sl.hdist, sl.hdist + nb * k);
        } else {
            D.ids.resize(o + nb * k, -1);
            D.dist.resize(o + nb * k, 0.0f);
            S->failed += (int64_t)nb;
        }
        S->completed += (int64_t)nb;
        S->t_last = t;
    }
    S->cv_done.notify_all();
    S->inflight -= sl.ws_bytes;
    sl.ws_bytes = 0;
    sl.busy = false;
    sl.tickets.clear();
    sl.t0s.clear();
}

// Takes the oldest nb waiting requests into the slot's pinned buffers and
// ticket list (the caller holds the lock); returns their constraint count.
static int32_t take_batch(Server *S, SrvSlot &sl, size_t nb) {
    ReqQueue &P = S->pending;
    const size_t d = (size_t)S->d;
    memcpy(sl.hq, P.q.data() + P.head * d, sizeof(float) * nb * d);
    int32_t ncon = 0;
    sl.hoff[0] = 0;
    for (size_t i = 0; i < nb; i++) {
        ncon += P.ncon[P.head + i];
        sl.hoff[i + 1] = ncon;
    }
    if (ncon > 0) {
        memcpy(sl.hattr, P.attr.data() + P.chead, sizeof(int32_t) * (size_t)ncon);
        memcpy(sl.hval, P.val.data() + P.chead, sizeof(int32_t) * (size_t)ncon);
    }
    sl.tickets.assign(P.ticket.begin() + (ptrdiff_t)P.head, P.ticket.begin() + (ptrdiff_t)(P.head + nb));
    sl.t0s.assign(P.t0.begin() + (ptrdiff_t)P.head, P.t0.begin() + (ptrdiff_t)(P.head + nb));
    P.head += nb;
    P.chead += (size_t)ncon;
    P.compact(d);
    return ncon;
}

// Enqueues the packed batch on the slot's stream: copies in, the search,
// copies out, the completion event.
static void launch(Server *S, SrvSlot &sl, int32_t ncon) {
    const int32_t nb = (int32_t)sl.tickets.size(), d = S->d, k = S->k;
    caps_status s = CAPS_OK;
    hipError_t e = hipMemcpyAsync(sl.dq, sl.hq, sizeof(float) * (size_t)nb * d, hipMemcpyHostToDevice, sl.st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.doff, sl.hoff, sizeof(int32_t) * (size_t)(nb + 1), hipMemcpyHostToDevice, sl.st);
    if (e == hipSuccess && ncon > 0)
        e = hipMemcpyAsync(sl.dattr, sl.hattr, sizeof(int32_t) * (size_t)ncon, hipMemcpyHostToDevice, sl.st);
    if (e == hipSuccess && ncon > 0)
        e = hipMemcpyAsync(sl.dval, sl.hval, sizeof(int32_t) * (size_t)ncon, hipMemcpyHostToDevice, sl.st);
    if (e != hipSuccess) s = CAPS_EDEVICE;
    if (s == CAPS_OK)
        s = search(S->ix, &S->sp, sl.dq, nb, sl.doff, sl.dattr, sl.dval, ncon, sl.dids, sl.ddist, nullptr, nullptr,
                   nullptr, nullptr, sl.st);
    if (s == CAPS_OK) {
        e = hipMemcpyAsync(sl.hids, sl.dids, sizeof(int32_t) * (size_t)nb * k, hipMemcpyDeviceToHost, sl.st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.hdist, sl.ddist, sizeof(float) * (size_t)nb * k, hipMemcpyDeviceToHost, sl.st);
        if (e != hipSuccess) s = CAPS_EDEVICE;
    }
    if (s != CAPS_OK) {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->err.empty()) S->err = caps_last_error();
    }
    sl.status = s;
    sl.busy = true;
    if (hipEventRecord(sl.ev, sl.st) != hipSuccess) {
        // no event to wait for: the stream is in error, finish the batch now
        (void)hipStreamSynchronize(sl.st);
        sl.status = CAPS_EDEVICE;
        retire(S, sl);
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->batches++;
        S->batched += nb;
    }
}

// Largest batch of at most `want` queries whose search workspace fits the
// budget the batches in flight leave free (0: none fits); *ws receives its
// bytes.  Without a budget every batch fits.
static int32_t admit(Server *S, int32_t want, size_t *ws) {
    if (S->p.workspace_bytes <= 0) {
        *ws = 0;
        return want;
    }
    const size_t budget = (size_t)S->p.workspace_bytes;
    const size_t avail = budget > S->inflight ? budget - S->inflight : 0;
    if (search_workspace_bytes(S->ix, &S->sp, 1) > avail) return 0;
    int32_t lo = 1, hi = want;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (search_workspace_bytes(S->ix, &S->sp, mid) <= avail) lo = mid;
        else hi = mid - 1;
    }
    *ws = search_workspace_bytes(S->ix, &S->sp, lo);
    return lo;
}

static void run(Server *S) {
    (void)hipSetDevice(S->ix->device);
    const auto window = std::chrono::duration<double, std::micro>(S->p.batch_window_us);
    for (;;) {
        bool progressed = false, any_busy = false;
        for (auto &sl : S->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            if (q != hipSuccess) {   // the batch's copies or kernels failed: its buffers are not results
                sl.status = CAPS_EDEVICE;
                std::lock_guard<std::mutex> lk(S->mu);
                if (S->err.empty()) S->err = std::string("caps_server: ") + hipGetErrorString(q);
            }
            retire(S, sl);
            progressed = true;
        }
        SrvSlot *free_slot = nullptr;
        for (auto &sl : S->slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        bool taken = false, quit = false;
        int32_t ncon = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (free_slot && !S->pending.empty()) {
                const bool fill = S->p.batch_window_us > 0 && !S->stop &&
                                  (int32_t)S->pending.size() < S->cap &&
                                  Clock::now() - S->pending.t0[S->pending.head] < window;
                if (!fill) {
                    size_t ws = 0;
                    const int32_t nb = admit(S, (int32_t)std::min((size_t)S->cap, S->pending.size()), &ws);
                    if (nb > 0) {   // else wait for a batch in flight to free its workspace
                        ncon = take_batch(S, *free_slot, (size_t)nb);
                        free_slot->ws_bytes = ws;
                        S->inflight += ws;
                        taken = true;
                    }
                }
            }
            if (!taken && !progressed) {
                bool busy_now = false;
                for (auto &sl : S->slots) busy_now |= sl.busy;
                if (S->stop && S->pending.empty() && !busy_now) {
                    quit = true;
                } else {
                    // poll in-flight batches and the batch window at a fine grain,
                    // otherwise sleep until a request arrives
                    const bool fine = any_busy || !S->pending.empty();
                    S->cv.wait_for(lk, fine ? std::chrono::microseconds(10) : std::chrono::microseconds(2000));
                }
            }
        }
        if (quit) break;
        if (taken) launch(S, *free_slot, ncon);
    }
}

static void free_slot(SrvSlot &sl) {
    if (sl.st) (void)hipStreamSynchronize(sl.st);
    void *host[] = {sl.hq, sl.hdist, sl.hoff, sl.hattr, sl.hval, sl.hids};
    for (void *p : host)
        if (p) (void)hipHostFree(p);
    void *dev[] = {sl.dq, sl.ddist, sl.doff, sl.dattr, sl.dval, sl.dids};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
}

static void destroy(Server *S) {
    if (S->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv.notify_all();
        S->worker.join();
    }
    for (auto &sl : S->slots) free_slot(sl);
    delete S;
}

static caps_status enqueue(Server *S, const float *q, int32_t n_con, const int32_t *attr, const int32_t *val,
                           Clock::time_point t0, uint64_t *ticket) {
    bool wake = false;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            set_error("caps_server_submit: server is stopping");
            return CAPS_EINVAL;
        }
        ReqQueue &P = S->pending;
        if ((int32_t)P.size() >= S->p.queue_slots) {
            S->rejected++;
            set_error("caps_server_submit: queue full (%d waiting)", S->p.queue_slots);
            return CAPS_EBUSY;
        }
        const uint64_t tk = S->next_ticket++;
        if (ticket) *ticket = tk;
        if (!S->have_first) {
            S->t_first = t0;
            S->have_first = true;
        }
        S->submitted++;
        // the scheduler polls at a fine grain while requests wait: it needs a
        // wake-up only when the queue was empty (it may be in its long sleep)
        // or a full batch is ready
        wake = P.empty() || (int32_t)P.size() + 1 >= S->cap;
        P.q.insert(P.q.end(), q, q + S->d);
        if (n_con > 0) {
            P.attr.insert(P.attr.end(), attr, attr + n_con);
            P.val.insert(P.val.end(), val, val + n_con);
        }
        P.ticket.push_back(tk);
        P.t0.push_back(t0);
        P.ncon.push_back(n_con);
    }
    if (wake) S->cv.notify_one();
    return CAPS_OK;
}

}  // namespace caps

using namespace caps;

struct caps_server {
    Server *s;
};

extern "C" caps_status caps_server_create(const caps_index *idx, const caps_server_params *p, caps_server **out) {
    if (!idx || !p || !out) {
        set_error("caps_server_create: null argument");
        return CAPS_EINVAL;
    }
    *out = nullptr;
    const Index &ix = idx->ix;
    if (p->k < 1 || p->k > kMaxK || p->nprobe < 1 || p->nprobe > ix.b || p->mode < 0 || p->mode > 2 ||
        p->routing < 0 || p->routing > 1 || p->max_batch < 1 || p->max_batch > 65536 || p->streams < 1 ||
        p->streams > 8 || p->queue_slots < 1 || p->max_constraints < 0 || p->max_constraints > 64 ||
        !(p->batch_window_us >= 0.0) || p->workspace_bytes < 0 || (p->flags & ~(int32_t)CAPS_SEARCH_DISJUNCTIVE)) {
        set_error("caps_server_create: parameter out of range");
        return CAPS_EINVAL;
    }
    if (p->mode == 1 && ix.prec == CAPS_PREC_NONE) {
        set_error("caps_server_create: mode 1 needs an index with a low-precision copy");
        return CAPS_EINVAL;
    }
    if (p->routing == 1 && !ix.router) {
        set_error("caps_server_create: routing 1 needs a trained router");
        return CAPS_EINVAL;
    }
    Server *S = new Server;
    S->ix = &ix;
    S->p = *p;
    S->sp.k = p->k;
    S->sp.nprobe = p->nprobe;
    S->sp.rule = 0;
    S->sp.mode = p->mode;
    S->sp.rerank = p->rerank;
    S->sp.routing = p->routing;
    S->sp.flags = p->flags & CAPS_SEARCH_DISJUNCTIVE;   // (the budget is the server's own: not a sub-batch cap)
    S->d = ix.d;
    S->k = p->k;
    // batch cap: largest size whose search workspace fits the budget
    int32_t cap = p->max_batch;
    if (p->workspace_bytes > 0) {
        int32_t lo = 1, hi = p->max_batch;
        if (search_workspace_bytes(&ix, &S->sp, 1) > (size_t)p->workspace_bytes) {
            delete S;
            set_error("caps_server_create: workspace_bytes below one query's search workspace");
            return CAPS_EINVAL;
        }
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo + 1) / 2;
            if (search_workspace_bytes(&ix, &S->sp, mid) <= (size_t)p->workspace_bytes) lo = mid;
            else hi = mid - 1;
        }
        cap = lo;
    }
    S->cap = cap;
    const size_t mc = (size_t)std::max(1, cap * p->max_constraints);
    S->slots.resize((size_t)p->streams);
    hipError_t e = hipSetDevice(ix.device);
    for (auto &sl : S->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.hq, sizeof(float) * (size_t)cap * S->d, 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.hdist, sizeof(float) * (size_t)cap * S->k, 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.hoff, sizeof(int32_t) * (size_t)(cap + 1), 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.hattr, sizeof(int32_t) * mc, 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.hval, sizeof(int32_t) * mc, 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.hids, sizeof(int32_t) * (size_t)cap * S->k, 0);
        if (e == hipSuccess) e = hipMalloc((void **)&sl.dq, sizeof(float) * (size_t)cap * S->d);
        if (e == hipSuccess) e = hipMalloc((void **)&sl.ddist, sizeof(float) * (size_t)cap * S->k);
        if (e == hipSuccess) e = hipMalloc((void **)&sl.doff, sizeof(int32_t) * (size_t)(cap + 1));
        if (e == hipSuccess) e = hipMalloc((void **)&sl.dattr, sizeof(int32_t) * mc);
        if (e == hipSuccess) e = hipMalloc((void **)&sl.dval, sizeof(int32_t) * mc);
        if (e == hipSuccess) e = hipMalloc((void **)&sl.dids, sizeof(int32_t) * (size_t)cap * S->k);
    }
    if (e != hipSuccess) {
        set_error("caps_server_create: %s", hipGetErrorString(e));
        destroy(S);
        return e == hipErrorOutOfMemory ? CAPS_ENOMEM : CAPS_EDEVICE;
    }
    S->worker = std::thread(run, S);
    *out = new caps_server{S};
    return CAPS_OK;
}

extern "C" caps_status caps_server_submit(caps_server *srv, const float *q, int32_t n_con, const int32_t *con_attr,
                                          const int32_t *con_val, uint64_t *ticket) {
    if (!srv || !q || n_con < 0 || (n_con > 0 && (!con_attr || !con_val))) {
        set_error("caps_server_submit: bad arguments");
        return CAPS_EINVAL;
    }
    if (n_con > srv->s->p.max_constraints) {
        set_error("caps_server_submit: %d constraints, the server takes at most %d", n_con,
                  srv->s->p.max_constraints);
        return CAPS_EINVAL;
    }
    for (int32_t j = 0; j < srv->s->d; j++)
        if (!isfinite(q[j])) {
            set_error("caps_server_submit: query coordinate %d is not finite", j);
            return CAPS_EINVAL;
        }
    return enqueue(srv->s, q, n_con, con_attr, con_val, Clock::now(), ticket);
}

extern "C" caps_status caps_server_replay(caps_server *srv, const float *q, const int32_t *con_off,
                                          const int32_t *con_attr, const int32_t *con_val, int32_t n,
                                          const double *arrival_s, uint64_t *tickets) {
    if (!srv || n < 0 || (n > 0 && (!q || !con_off || !arrival_s)) ||
        (n > 0 && con_off[n] > con_off[0] && (!con_attr || !con_val))) {
        set_error("caps_server_replay: bad arguments");
        return CAPS_EINVAL;
    }
    Server *S = srv->s;
    const Clock::time_point start = Clock::now();
    for (int32_t i = 0; i < n; i++) {
        const int32_t lo = con_off[i], nc = con_off[i + 1] - con_off[i];
        if (lo < 0 || nc < 0 || nc > S->p.max_constraints) {
            set_error("caps_server_replay: request %d has bad constraint offsets or too many constraints", i);
            return CAPS_EINVAL;
        }
        for (int32_t j = 0; j < S->d; j++)
            if (!isfinite(q[(size_t)i * S->d + j])) {
                set_error("caps_server_replay: request %d has a non-finite coordinate", i);
                return CAPS_EINVAL;
            }
        const Clock::time_point at =
            start + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
        Clock::time_point now = Clock::now();
        if (at - now > std::chrono::microseconds(200)) std::this_thread::sleep_until(at - std::chrono::microseconds(100));
        while ((now = Clock::now()) < at) {
        }
        uint64_t tk = 0;
        const caps_status s = enqueue(S, q + (size_t)i * S->d, nc, con_attr + lo, con_val + lo, at, &tk);
        if (tickets) tickets[i] = s == CAPS_OK ? tk : 0;   // 0: refused (queue full)
        if (s != CAPS_OK && s != CAPS_EBUSY) return s;
    }
    return CAPS_OK;
}

extern "C" caps_status caps_server_poll(caps_server *srv, int32_t max, uint64_t *tickets, int32_t *ids, float *dist,
                                        float *latency_ms, int32_t *status, int32_t *n_done) {
    if (!srv || max < 0 || !n_done || (max > 0 && (!tickets || !ids || !dist))) {
        set_error("caps_server_poll: bad arguments");
        return CAPS_EINVAL;
    }
    Server *S = srv->s;
    std::lock_guard<std::mutex> lk(S->mu);
    DoneQueue &D = S->done;
    const size_t c = std::min((size_t)max, D.size()), k = (size_t)S->k, h = D.head;
    if (c > 0) {
        memcpy(tickets, D.ticket.data() + h, sizeof(uint64_t) * c);
        memcpy(ids, D.ids.data() + h * k, sizeof(int32_t) * c * k);
        memcpy(dist, D.dist.data() + h * k, sizeof(float) * c * k);
        if (latency_ms) memcpy(latency_ms, D.lat.data() + h, sizeof(float) * c);
        if (status) memcpy(status, D.status.data() + h, sizeof(int32_t) * c);
        D.head += c;
        D.compact(k);
    }
    *n_done = (int32_t)c;
    return CAPS_OK;
}

extern "C" caps_status caps_server_drain(caps_server *srv, double timeout_s) {
    if (!srv) {
        set_error("caps_server_drain: null server");
        return CAPS_EINVAL;
    }
    Server *S = srv->s;
    std::unique_lock<std::mutex> lk(S->mu);
    const bool ok = S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                        [S] { return S->completed == S->submitted; });
    if (!ok) {
        set_error("caps_server_drain: %lld of %lld requests still open after %.1f s",
                  (long long)(S->submitted - S->completed), (long long)S->submitted, timeout_s);
        return CAPS_EBUSY;
    }
    return CAPS_OK;
}

extern "C" caps_status caps_server_stats(caps_server *srv, caps_server_stats_t *out, int32_t reset) {
    if (!srv || !out) {
        set_error("caps_server_stats: null argument");
        return CAPS_EINVAL;
    }
    Server *S = srv->s;
    std::lock_guard<std::mutex> lk(S->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->failed = S->failed;
    out->batches = S->batches;
    out->mean_batch = S->batches ? (double)S->batched / (double)S->batches : 0.0;
    out->max_batch = S->cap;
    if (!S->lat.empty()) {
        std::vector<double> v = S->lat;
        std::sort(v.begin(), v.end());
        auto pct = [&](double f) {
            const size_t i = (size_t)std::min<double>((double)v.size() - 1, floor(f * (double)(v.size() - 1) + 0.5));
            return v[i];
        };
        double sum = 0.0;
        for (double x : v) sum += x;
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = v.back();
        out->mean_ms = sum / (double)v.size();
        const double span = std::chrono::duration<double>(S->t_last - S->t_first).count();
        out->qps = span > 0 ? (double)S->completed / span : 0.0;
    }
    if (reset) {
        S->submitted -= S->completed;
        S->completed = S->rejected = S->failed = S->batches = S->batched = 0;
        S->lat.clear();
        S->have_first = false;
    }
    return CAPS_OK;
}

extern "C" void caps_server_destroy(caps_server *srv) {
    if (!srv) return;
    destroy(srv->s);
    delete srv;
}
