// Serving runtime: continuous batching of gradient requests (see the serving
// section of include/shapegrad.h for the contract).
//
// One scheduler thread owns all device work.  Each turn it
//   1. admits queued requests in arrival order while a request slot is free and
//      the request's buffers fit the HBM budget (a request that does not fit
//      waits at the head of the queue, one whose session already has a request
//      in flight waits for that session's buffer);
//   2. polls the events of the batches in flight and completes their requests;
//   3. when a stream is free, forms a batch of admitted requests and enqueues
//      it on that stream: per request its p upload and stage (first slice
//      only), slices of its seeded field generation, one batched column-kernel
//      launch per kernel specialization covering slices of the requests'
//      blocks, and for requests whose last slice it holds the gradient copy;
//      then an event.
// With max_launch_us set, a batch takes work only up to that many estimated
// microseconds: a large request is split into slices over several batches of
// the same stream (so its stage, field generation and column blocks stay in
// stream order), and requests that arrive meanwhile are batched beside its
// later slices or run on the other streams instead of waiting for all of it.
// Clients never touch the device: serve_submit queues, serve_poll waits on a
// condition variable for the scheduler to publish the result.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <limits>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sg_scene.h"

using namespace sg;

namespace {

// cost model of a batch's device work: HBM bytes moved at 4.5 TB/s
constexpr double kBytesPerUs = 4.5e6;
constexpr int64_t kGenSlice = 1 << 16;      // field generation is sliced in multiples of this many samples
constexpr int64_t kFakeBlocks = 1000;       // fake-executor requests: work units of a request

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum ReqState { PENDING, ADMITTED, LAUNCHED, DONE, CANCELLED, FAILED };

struct Session;

struct Buf {                 // device buffers of one admitted request
    float2* e = nullptr;     // seeded field planes (allocated when a seeded request first needs them)
    float2* a = nullptr;
    double* p = nullptr;
    double* fval = nullptr;
    float4* bbox = nullptr;
    PrimRec* prec = nullptr;
    double* ztab = nullptr;
    uint32_t* code = nullptr;
    uint32_t* gcode = nullptr;
    double* grad = nullptr;
    unsigned long long* fx = nullptr;   // deterministic sessions: fixed-point accumulators
    double* h_p = nullptr;   // pinned
    double* h_grad = nullptr;
    bool fields = false;     // holds field planes (fake buffers: counted only)
    int64_t bytes = 0;       // counted against the budget while the buffer exists
    Session* owner = nullptr;
};

struct Session {
    uint32_t id = 0;
    sg_scene* scene = nullptr;      // null for fake sessions
    int64_t n_params = 0;
    int64_t stage_bytes = 0;        // staging, gradient and accumulators of one request
    int64_t field_bytes = 0;        // the seeded field planes of one request
    bool det = false;               // the scene's deterministic setting when the session opened
    std::vector<Buf*> free_bufs;    // idle buffers kept for the session's next requests
    std::vector<Buf*> all_bufs;
};

struct Req {
    uint64_t ticket = 0;
    Session* s = nullptr;
    std::vector<double> p, grad;
    uint64_t seed = 0;
    bool caller = false;            // fields from the caller's planes (ce, ca)
    const float2* ce[kMaxComp] = {};
    const float2* ca[kMaxComp] = {};
    double omega = 0;
    int state = PENDING;
    bool cancel = false;
    sg_status status = SG_OK;
    Buf* buf = nullptr;
    int64_t need = 0;               // bytes of its buffer this request uses
    sg_req_stats st{};
    // progress through sliced launches
    int64_t gen_n = 0, gen_done = 0;        // seeded field samples
    int64_t blocks = 0, blocks_done = 0;    // column-kernel blocks
    double block_bytes = 0.0;               // estimated HBM bytes per block
    bool staged = false;
    int lane = -1;                  // the stream its slices run on once one has been launched
};

struct Slice {                     // one request's share of a batch
    Req* r;
    int64_t g0, g1;                 // field samples generated
    int64_t b0, b1;                 // column blocks
    bool first, last;
};

struct Lane {                      // one stream and the batch in flight on it
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Slice> batch;
    bool busy = false;
    bool failed = false;
    int64_t fake_ready_ns = 0;
    KParams* d_plist = nullptr;     // device copies of the batch's launch parameters
    int* d_first = nullptr;
    KParams* h_plist = nullptr;     // pinned
    int* h_first = nullptr;
};

}  // namespace

struct sg_server {
    sg_ctx* ctx = nullptr;
    sg_server_opts opts{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stop = false;
    std::vector<std::unique_ptr<Session>> sessions;
    std::deque<Req*> pending;
    std::deque<Req*> ready;         // admitted, with slices left to launch
    std::unordered_map<uint64_t, Req*> reqs;
    uint64_t next_ticket = 1;
    int64_t bytes_used = 0;         // bytes of the requests admitted and not yet finished
    int64_t bytes_held = 0;         // bytes of every request buffer that exists (busy or idle)
    std::list<Buf*> idle;           // idle buffers, least recently released first
    int slots_used = 0;
    std::vector<Lane> lanes;
    int next_lane = 0;
    int64_t launches = 0, completed = 0, max_batch_seen = 0;
    int64_t fault_launch = -1;      // SG_FAULT_INJECT=launch:N
    int64_t fault_alloc = -1;       // SG_FAULT_INJECT=alloc:N: buffer allocations N, N+1, ... fail
    int64_t allocs = 0;
};

namespace {

void free_buf(Buf* b, bool fake) {
    if (fake) {
        delete b;
        return;
    }
    hipFree(b->e);
    hipFree(b->a);
    hipFree(b->p);
    hipFree(b->fval);
    hipFree(b->bbox);
    hipFree(b->prec);
    hipFree(b->ztab);
    hipFree(b->code);
    hipFree(b->gcode);
    hipFree(b->grad);
    hipFree(b->fx);
    if (b->h_p) hipHostFree(b->h_p);
    if (b->h_grad) hipHostFree(b->h_grad);
    delete b;
}

bool alloc_staging(sg_scene* sc, bool det, Buf* b) {
    const int64_t nfield = std::max<int64_t>(1, sc->nfield), n = std::max<int64_t>(1, sc->n_params);
    hipError_t e = hipMalloc((void**)&b->p, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&b->fval, nfield * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&b->bbox, std::max(1, sc->nprim) * sizeof(float4));
    if (e == hipSuccess) e = hipMalloc((void**)&b->prec, std::max(1, sc->nprim) * sizeof(PrimRec));
    if (e == hipSuccess) e = hipMalloc((void**)&b->ztab, (size_t)sc->ncomp * sc->nclass * sc->nw * 3 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&b->code, (size_t)sc->ncomp * sc->nw * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc((void**)&b->gcode, (size_t)sc->ncomp * ((sc->nw + kGroup - 1) / kGroup) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&b->grad, n * sizeof(double));
    if (e == hipSuccess && det) e = hipMalloc((void**)&b->fx, (3 * n + 1) * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_p, n * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_grad, n * sizeof(double));
    return e == hipSuccess;
}

bool alloc_fields(sg_scene* sc, Buf* b) {
    const int64_t cm = (int64_t)sc->ncomp * sc->plane;
    hipError_t e = hipMalloc((void**)&b->e, cm * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc((void**)&b->a, cm * sizeof(float2));
    if (e != hipSuccess) {
        hipFree(b->e);
        hipFree(b->a);
        b->e = b->a = nullptr;
    }
    return e == hipSuccess;
}

// fake results: grad_k = 2 p_k + (seed mod 1000)
void fake_result(Req* r) {
    r->grad.resize(r->s->n_params);
    for (int64_t k = 0; k < r->s->n_params; ++k) r->grad[k] = 2.0 * r->p[k] + (double)(r->seed % 1000);
}

void release(sg_server* v, Req* r) {
    if (r->buf) {
        r->s->free_bufs.push_back(r->buf);
        v->idle.push_back(r->buf);
        r->buf = nullptr;
    }
    v->bytes_used -= r->need;
    v->slots_used -= 1;
}

// Frees an idle buffer (its session's next request allocates a new one).
void drop_idle(sg_server* v, Buf* b) {
    Session* s = b->owner;
    s->free_bufs.erase(std::find(s->free_bufs.begin(), s->free_bufs.end(), b));
    s->all_bufs.erase(std::find(s->all_bufs.begin(), s->all_bufs.end(), b));
    v->idle.remove(b);
    v->bytes_held -= b->bytes;
    free_buf(b, v->opts.fake_executor != 0);
}

// The least recently released idle buffer other than `keep`, or null.
Buf* oldest_idle(sg_server* v, const Buf* keep) {
    for (Buf* b : v->idle)
        if (b != keep) return b;
    return nullptr;
}

// Frees least recently released idle buffers (never `keep`) until `extra`
// more bytes fit the budget; true if they fit.
bool make_room(sg_server* v, int64_t extra, const Buf* keep) {
    while (v->bytes_held + extra > v->opts.hbm_budget_bytes) {
        Buf* b = oldest_idle(v, keep);
        if (!b) return false;
        drop_idle(v, b);
    }
    return true;
}

// Gives buffer b (a new one when null) what a request of session s needs:
// staging, and the field planes for a seeded request.  False when the device
// is out of memory (or an injected allocation failure); b keeps what it had.
bool provide(sg_server* v, Session* s, Buf*& b, bool fields) {
    const bool inject = v->fault_alloc >= 0 && v->allocs >= v->fault_alloc;
    v->allocs++;
    if (inject) return false;
    const bool fake = v->opts.fake_executor != 0;
    Buf* nb = b;
    if (!nb) {
        nb = new Buf;
        nb->owner = s;
        if (!fake && !alloc_staging(s->scene, s->det, nb)) {
            free_buf(nb, false);
            return false;
        }
        nb->bytes = s->stage_bytes;
    }
    if (fields && !nb->fields) {
        if (!fake && !alloc_fields(s->scene, nb)) {
            if (!b) free_buf(nb, false);
            return false;
        }
        nb->fields = true;
        nb->bytes += s->field_bytes;
    }
    b = nb;
    return true;
}

void retire(sg_server* v, Req* r, int state, sg_status status) {
    r->state = state;
    r->status = status;
    r->st.done_ns = now_ns();
    v->cv_done.notify_all();
}

// Admit queued requests in arrival order while slots and budget allow.  The
// budget bounds every request buffer that exists: a session keeps its idle
// buffers for its next requests.  A session with a request in flight grows
// only into free budget; when none is left its next request waits for one of
// the session's own buffers (later requests of other sessions may pass it, up
// to kMaxPassed of them).  Only a session with nothing in flight frees the
// least recently released idle buffers of other sessions to make room, so a
// deep queue does not turn into a cycle of freeing and reallocating buffers
// (each free waits for the device).
constexpr int kMaxPassed = 64;
void admit(sg_server* v) {
    const bool fake = v->opts.fake_executor != 0;
    size_t i = 0;
    int passed = 0;
    while (i < v->pending.size()) {
        Req* r = v->pending[i];
        Session* s = r->s;
        if (v->slots_used >= v->opts.max_slots) return;
        const bool fields = !r->caller;
        // an idle buffer of the session, preferably one that already has what r needs
        Buf* b = nullptr;
        for (Buf* c : s->free_bufs)
            if (!b || (fields && c->fields && !b->fields)) b = c;
        const int64_t extra = !b ? s->stage_bytes + (fields ? s->field_bytes : 0)
                                 : ((fields && !b->fields) ? s->field_bytes : 0);
        if (extra > 0) {
            if (v->bytes_held + extra > v->opts.hbm_budget_bytes) {
                if (s->all_bufs.size() > s->free_bufs.size()) {
                    // its session has a request in flight: wait for that buffer
                    if (++passed > kMaxPassed) return;
                    ++i;
                    continue;
                }
                if (!make_room(v, extra, b)) return;   // busy buffers hold the budget
            }
            const bool had = b != nullptr;
            const int64_t before = had ? b->bytes : 0;
            if (!provide(v, s, b, fields)) {
                // device memory short: free every other idle buffer and try once more
                while (Buf* x = oldest_idle(v, b)) drop_idle(v, x);
                if (!provide(v, s, b, fields)) {
                    if (v->slots_used > 0) return;     // in-flight requests will free memory
                    // nothing runs that could free memory: the request cannot be served now
                    v->pending.erase(v->pending.begin() + (std::ptrdiff_t)i);
                    retire(v, r, FAILED, SG_E_NOMEM);
                    continue;
                }
            }
            if (!had) s->all_bufs.push_back(b);
            v->bytes_held += b->bytes - before;
        }
        auto it = std::find(s->free_bufs.begin(), s->free_bufs.end(), b);
        if (it != s->free_bufs.end()) {
            s->free_bufs.erase(it);
            v->idle.remove(b);
        }
        r->buf = b;
        r->need = s->stage_bytes + (fields ? s->field_bytes : 0);
        v->pending.erase(v->pending.begin() + (std::ptrdiff_t)i);
        v->bytes_used += r->need;
        v->slots_used += 1;
        r->state = ADMITTED;
        r->st.admit_ns = now_ns();
        // its work: field generation (seeded), then the column blocks
        if (fake) {
            r->blocks = kFakeBlocks;
            r->block_bytes = (double)s->stage_bytes / kFakeBlocks;
        } else {
            sg_scene* sc = s->scene;
            const KParams kp = column_params(sc);
            r->gen_n = fields ? (int64_t)sc->ncomp * sc->plane : 0;
            r->blocks = (int64_t)kp.ncomp * kp.tiles_u * kp.tiles_v * kp.nseg;
            r->block_bytes = 16.0 * (double)sc->ncomp * (double)sc->plane / (double)std::max<int64_t>(1, r->blocks);
        }
        v->ready.push_back(r);
    }
}

void drop_ready(sg_server* v, Req* r) {
    auto it = std::find(v->ready.begin(), v->ready.end(), r);
    if (it != v->ready.end()) v->ready.erase(it);
}

void finish_batch(sg_server* v, Lane& L, bool ok) {
    const int64_t t = now_ns();
    for (const Slice& c : L.batch) {
        Req* r = c.r;
        if (!ok) {
            drop_ready(v, r);
            r->state = FAILED;
            r->status = SG_E_DEVICE;
        } else if (c.last || r->cancel) {
            drop_ready(v, r);
            if (r->cancel) {
                r->state = CANCELLED;
                r->status = SG_E_CANCELLED;
            } else {
                if (v->opts.fake_executor) fake_result(r);
                else r->grad.assign(r->buf->h_grad, r->buf->h_grad + r->s->n_params);
                r->state = DONE;
                r->status = SG_OK;
                v->completed++;
            }
        } else {
            continue;       // more slices to come, on this lane
        }
        r->st.done_ns = t;
        release(v, r);
    }
    L.batch.clear();
    L.busy = false;
    L.failed = false;
}

// Takes work from the ready requests into lane li's batch, up to max_batch
// requests and (with max_launch_us) that many estimated microseconds: first
// every request, in arrival order, whose remaining work fits whole; then a
// slice of the oldest one that did not fit (at least a quarter of the budget,
// so a large request progresses while small ones keep arriving).  A sliced
// request stays at its place in the queue, tied to this lane.  Returns the
// number of slices.
int form_batch(sg_server* v, int li) {
    Lane& L = v->lanes[li];
    const double budget = v->opts.max_launch_us > 0 ? (double)v->opts.max_launch_us * kBytesPerUs
                                                    : std::numeric_limits<double>::infinity();
    double used = 0.0;
    std::vector<Req*> cancelled;
    Req* big = nullptr;
    auto remaining = [](const Req* r) {
        return 16.0 * (double)(r->gen_n - r->gen_done) + r->block_bytes * (double)(r->blocks - r->blocks_done);
    };
    for (Req* r : v->ready) {
        if (r->lane >= 0 && r->lane != li) continue;      // its slices run on another stream
        if (r->cancel && r->lane >= 0) {                  // sliced, cancelled, nothing of it in flight
            cancelled.push_back(r);
            continue;
        }
        if ((int)L.batch.size() + (big ? 1 : 0) >= v->opts.max_batch) break;
        const double need = remaining(r);
        if (need <= budget - used) {
            L.batch.push_back(Slice{r, r->gen_done, r->gen_n, r->blocks_done, r->blocks, !r->staged, true});
            used += need;
        } else if (!big) {
            big = r;
        }
    }
    if (big && (int)L.batch.size() < v->opts.max_batch) {
        Req* r = big;
        double room = std::max(budget - used, 0.25 * budget);
        Slice c{r, r->gen_done, r->gen_done, r->blocks_done, r->blocks_done, !r->staged, false};
        const int64_t grem = r->gen_n - r->gen_done, brem = r->blocks - r->blocks_done;
        int64_t g = 0, b = 0;
        if (grem > 0) {
            g = std::min(grem, std::max<int64_t>(kGenSlice, (int64_t)(room / 16.0) / kGenSlice * kGenSlice));
            room -= 16.0 * (double)g;
        }
        if (g == grem && room > 0.0)
            b = std::min<int64_t>(brem, (int64_t)(room / std::max(1.0, r->block_bytes)));
        if (g == 0 && b == 0) b = 1;                     // every slice makes progress
        c.g1 = c.g0 + g;
        c.b1 = c.b0 + b;
        c.last = c.g1 == r->gen_n && c.b1 == r->blocks;
        L.batch.push_back(c);
    }
    for (Req* r : cancelled) {
        drop_ready(v, r);
        retire(v, r, CANCELLED, SG_E_CANCELLED);
        release(v, r);
    }
    return (int)L.batch.size();
}

double slice_us(const Slice& c) {
    return (16.0 * (double)(c.g1 - c.g0) + c.r->block_bytes * (double)(c.b1 - c.b0)) / kBytesPerUs;
}

// Enqueue lane li's batch (device work only; called with the lock held).
bool launch_batch(sg_server* v, Lane& L, int li) {
    const int64_t t = now_ns();
    for (Slice& c : L.batch) {
        Req* r = c.r;
        if (c.first) {
            r->state = LAUNCHED;
            r->st.launch_ns = t;
            r->st.batch_size = (int32_t)L.batch.size();
            r->lane = li;
        }
        r->gen_done = c.g1;
        r->blocks_done = c.b1;
    }
    v->max_batch_seen = std::max<int64_t>(v->max_batch_seen, (int64_t)L.batch.size());
    const bool inject = (v->launches == v->fault_launch);
    v->launches++;
    if (v->opts.fake_executor) {
        double us = (double)v->opts.fake_us;
        for (const Slice& c : L.batch) us += slice_us(c);
        L.fake_ready_ns = t + (int64_t)(us * 1000.0);
        L.failed = inject;
        for (Slice& c : L.batch) c.r->staged = true;
        return true;
    }
    if (inject) {
        L.failed = true;
        return true;
    }
    hipStream_t st = L.stream;
    // per request: p and stage (first slice), field generation slices
    for (Slice& c : L.batch) {
        Req* r = c.r;
        sg_scene* sc = r->s->scene;
        Buf* b = r->buf;
        if (c.first) {
            std::memcpy(b->h_p, r->p.data(), r->s->n_params * sizeof(double));
            if (r->s->n_params &&
                hipMemcpyAsync(b->p, b->h_p, r->s->n_params * sizeof(double), hipMemcpyHostToDevice, st))
                return false;
            StageParams sp = stage_params(sc, b->p);
            sp.fval[0] = b->fval;
            sp.bbox[0] = b->bbox;
            sp.prec[0] = b->prec;
            if (!sc->static_w) {
                sp.ztab[0] = b->ztab;
                sp.code[0] = b->code;
                sp.gcode[0] = b->gcode;
            }
            sp.zero_ptr = b->grad;
            sp.zero_n = sc->n_params;
            if (launch_stage(sp, 1, st) != hipSuccess) return false;
            if (r->s->det && sc->n_params > 0 &&
                launch_fill(reinterpret_cast<double*>(b->fx), 0.0, 3 * sc->n_params + 1, st) != hipSuccess)
                return false;
            r->staged = true;
        }
        if (c.g1 > c.g0 && launch_fieldgen(b->e, b->a, c.g0, c.g1, r->seed, st) != hipSuccess) return false;
    }
    // one batched column launch per kernel specialization over the slices'
    // blocks; a group of g slices uses h_plist[g0, g0 + g) and the prefix
    // h_first[g0, g0 + g] (terminated by its total)
    const int nb = (int)L.batch.size();
    std::vector<bool> grouped(nb, false);
    int slot = 0;
    for (int i = 0; i < nb; ++i) {
        if (grouped[i] || L.batch[i].b1 == L.batch[i].b0) continue;
        const int tree = L.batch[i].r->s->scene->tree, var = L.batch[i].r->s->scene->variant;
        const int g0 = slot;
        int ng = 0;
        int64_t blocks = 0;
        for (int j = i; j < nb; ++j) {
            const Slice& c = L.batch[j];
            sg_scene* sc = c.r->s->scene;
            if (grouped[j] || c.b1 == c.b0 || sc->tree != tree || sc->variant != var) continue;
            grouped[j] = true;
            Req* r = c.r;
            Buf* b = r->buf;
            KParams kp = column_params(sc);
            kp.fval = b->fval;
            kp.bbox = b->bbox;
            kp.prec = b->prec;
            if (!sc->static_w) {
                kp.ztab = b->ztab;
                kp.code = b->code;
                kp.gcode = b->gcode;
            }
            kp.grad = b->grad;
            if (r->s->det && sc->n_params > 0) {
                kp.fx = b->fx;
                kp.fx_n = sc->n_params;
            }
            for (int cc = 0; cc < kMaxComp; ++cc) {
                const int k = std::min(cc, sc->ncomp - 1);
                kp.ef[cc] = r->caller ? r->ce[k] : b->e + (int64_t)k * sc->plane;
                kp.ea[cc] = r->caller ? r->ca[k] : b->a + (int64_t)k * sc->plane;
            }
            kp.two_omega = (float)(2.0 * r->omega);
            kp.block0 = (int32_t)c.b0;
            L.h_plist[g0 + ng] = kp;
            L.h_first[g0 + ng] = (int)blocks;
            blocks += c.b1 - c.b0;
            ++ng;
        }
        L.h_first[g0 + ng] = (int)blocks;
        if (hipMemcpyAsync(L.d_plist + g0, L.h_plist + g0, ng * sizeof(KParams), hipMemcpyHostToDevice, st)) return false;
        if (hipMemcpyAsync(L.d_first + g0, L.h_first + g0, (ng + 1) * sizeof(int), hipMemcpyHostToDevice, st))
            return false;
        if (launch_column_batch(tree, var, L.d_plist + g0, L.d_first + g0, ng, blocks, st) != hipSuccess) return false;
        slot = g0 + ng + 1;
    }
    for (const Slice& c : L.batch) {
        if (!c.last) continue;
        Req* r = c.r;
        if (r->s->det && r->s->n_params > 0 &&
            launch_fx_finish(r->buf->fx, r->s->n_params, r->buf->grad, st) != hipSuccess)
            return false;
        if (r->s->n_params &&
            hipMemcpyAsync(r->buf->h_grad, r->buf->grad, r->s->n_params * sizeof(double), hipMemcpyDeviceToHost, st))
            return false;
    }
    return hipEventRecord(L.done, st) == hipSuccess;
}

void scheduler(sg_server* v) {
    if (!v->opts.fake_executor) hipSetDevice(v->ctx->device);
    std::unique_lock<std::mutex> lk(v->mu);
    while (true) {
        admit(v);
        // completions
        bool any_busy = false;
        for (Lane& L : v->lanes) {
            if (!L.busy) continue;
            bool fin = false, ok = true;
            if (v->opts.fake_executor) {
                fin = now_ns() >= L.fake_ready_ns;
                ok = !L.failed;
            } else if (L.failed) {
                // a failed launch: wait for whatever reached the stream, then fail the batch
                fin = hipStreamQuery(L.stream) != hipErrorNotReady;
                ok = false;
            } else {
                const hipError_t q = hipEventQuery(L.done);
                fin = q != hipErrorNotReady;
                ok = q == hipSuccess;
            }
            if (fin) {
                finish_batch(v, L, ok);
                v->cv_done.notify_all();
            } else {
                any_busy = true;
            }
        }
        admit(v);
        // launches
        for (int k = 0; k < (int)v->lanes.size() && !v->ready.empty(); ++k) {
            const int li = (v->next_lane + k) % (int)v->lanes.size();
            Lane& L = v->lanes[li];
            if (L.busy) continue;
            if (form_batch(v, li) == 0) continue;
            L.busy = true;
            if (!launch_batch(v, L, li)) L.failed = true;
            any_busy = true;
            v->next_lane = (li + 1) % (int)v->lanes.size();
        }
        if (v->stop && v->pending.empty() && v->ready.empty() && !any_busy) break;
        if (any_busy) {
            // batches in flight: poll their events at a fine grain
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else if (!v->stop) {
            v->cv_work.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" sg_status sg_fieldgen(void* e_fwd, void* e_adj, int64_t n, uint64_t seed, void* stream) {
    if (!e_fwd || !e_adj || n < 0) return fail(SG_E_INVALID, "sg_fieldgen: bad arguments");
    if (n == 0) return SG_OK;
    HIP_OK(launch_fieldgen((float2*)e_fwd, (float2*)e_adj, 0, n, seed, (hipStream_t)stream));
    return SG_OK;
}

extern "C" sg_status sg_server_create(sg_ctx* ctx, const sg_server_opts* o, sg_server** out) {
    if (!o || !out) return fail(SG_E_INVALID, "sg_server_create: NULL argument");
    *out = nullptr;
    if (!o->fake_executor && !ctx) return fail(SG_E_INVALID, "sg_server_create: NULL ctx");
    int64_t budget = o->hbm_budget_bytes;
    if (budget == 0) {       // SG_HBM_BUDGET: bytes, optionally K / M / G (powers of 2^10)
        budget = int64_t(8) << 30;
        if (const char* b = std::getenv("SG_HBM_BUDGET")) {
            char* end = nullptr;
            const long long val = std::strtoll(b, &end, 10);
            int shift = 0;
            if (end && (*end == 'K' || *end == 'k')) shift = 10, ++end;
            else if (end && (*end == 'M' || *end == 'm')) shift = 20, ++end;
            else if (end && (*end == 'G' || *end == 'g')) shift = 30, ++end;
            if (end == b || !end || *end != '\0' || val <= 0 || val > (std::numeric_limits<int64_t>::max() >> shift))
                return fail(SG_E_INVALID, "sg_server_create: SG_HBM_BUDGET=\"%s\" is not a positive size", b);
            budget = (int64_t)val << shift;
        }
    }
    if (budget <= 0 || o->max_slots < 1 || o->max_batch < 1 || o->n_streams < 1 || o->n_streams > 8 ||
        o->fake_us < 0 || o->max_launch_us < 0)
        return fail(SG_E_INVALID, "sg_server_create: bad options");
    auto* v = new sg_server;
    v->ctx = ctx;
    v->opts = *o;
    v->opts.hbm_budget_bytes = budget;
    if (const char* fi = std::getenv("SG_FAULT_INJECT")) {
        if (std::strncmp(fi, "launch:", 7) == 0) v->fault_launch = std::atoll(fi + 7);
        if (std::strncmp(fi, "alloc:", 6) == 0) v->fault_alloc = std::atoll(fi + 6);
    }
    v->lanes.resize(o->n_streams);
    if (!o->fake_executor) {
        hipError_t e = hipSetDevice(ctx->device);
        for (Lane& L : v->lanes) {
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
            const size_t np = 2 * (size_t)o->max_batch + 2;
            if (e == hipSuccess) e = hipMalloc((void**)&L.d_plist, np * sizeof(KParams));
            if (e == hipSuccess) e = hipMalloc((void**)&L.d_first, (np + 1) * sizeof(int));
            if (e == hipSuccess) e = hipHostMalloc((void**)&L.h_plist, np * sizeof(KParams));
            if (e == hipSuccess) e = hipHostMalloc((void**)&L.h_first, (np + 1) * sizeof(int));
        }
        if (e != hipSuccess) {
            sg_server_destroy(v);
            return fail(SG_E_DEVICE, "sg_server_create: %s", hipGetErrorString(e));
        }
    }
    v->th = std::thread(scheduler, v);
    *out = v;
    return SG_OK;
}

extern "C" sg_status sg_server_destroy(sg_server* v) {
    if (!v) return fail(SG_E_INVALID, "NULL server");
    {
        std::lock_guard<std::mutex> lk(v->mu);
        v->stop = true;
        for (Req* r : v->pending) {
            r->state = CANCELLED;
            r->status = SG_E_CANCELLED;
        }
        v->pending.clear();
        // requests with nothing launched are cancelled; sliced ones finish
        // the slices in flight and are cancelled by the scheduler
        std::deque<Req*> keep;
        for (Req* r : v->ready) {
            if (r->lane >= 0) {
                r->cancel = true;
                keep.push_back(r);
                continue;
            }
            r->state = CANCELLED;
            r->status = SG_E_CANCELLED;
            release(v, r);
        }
        v->ready.swap(keep);
    }
    v->cv_work.notify_all();
    if (v->th.joinable()) v->th.join();
    v->cv_done.notify_all();
    for (auto& kv : v->reqs) delete kv.second;
    v->reqs.clear();
    for (auto& s : v->sessions)
        for (Buf* b : s->all_bufs) free_buf(b, v->opts.fake_executor != 0);
    if (!v->opts.fake_executor) {
        for (Lane& L : v->lanes) {
            if (L.stream) hipStreamDestroy(L.stream);
            if (L.done) hipEventDestroy(L.done);
            hipFree(L.d_plist);
            hipFree(L.d_first);
            if (L.h_plist) hipHostFree(L.h_plist);
            if (L.h_first) hipHostFree(L.h_first);
        }
    }
    delete v;
    return SG_OK;
}

static sg_status open_session(sg_server* v, sg_scene* sc, int64_t n_params, int64_t stage_bytes,
                              int64_t field_bytes, bool det, uint32_t* id) {
    std::lock_guard<std::mutex> lk(v->mu);
    auto s = std::make_unique<Session>();
    s->id = (uint32_t)v->sessions.size();
    s->scene = sc;
    s->n_params = n_params;
    s->stage_bytes = stage_bytes;
    s->field_bytes = field_bytes;
    s->det = det;
    *id = s->id;
    v->sessions.push_back(std::move(s));
    return SG_OK;
}

extern "C" sg_status serve_open_session(sg_server* v, sg_scene* sc, uint32_t* id) {
    if (!v || !sc || !id) return fail(SG_E_INVALID, "serve_open_session: NULL argument");
    if (v->opts.fake_executor) return fail(SG_E_INVALID, "fake-executor servers take fake sessions");
    if (sc->ctx->device != v->ctx->device) return fail(SG_E_INVALID, "scene on another device");
    bool det;
    {
        std::lock_guard<std::mutex> lk(sc->mu);
        det = sc->deterministic;
    }
    const int64_t stage = staging_bytes(sc) + (det ? 8 * (3 * std::max<int64_t>(1, sc->n_params) + 1) : 0);
    return open_session(v, sc, sc->n_params, stage, 16 * (int64_t)sc->ncomp * sc->plane, det, id);
}

extern "C" sg_status serve_open_fake_session(sg_server* v, int64_t n_params, int64_t bytes, uint32_t* id) {
    if (!v || !id) return fail(SG_E_INVALID, "serve_open_fake_session: NULL argument");
    if (!v->opts.fake_executor) return fail(SG_E_INVALID, "only fake-executor servers take fake sessions");
    if (n_params < 0 || bytes < 0) return fail(SG_E_INVALID, "bad sizes");
    return open_session(v, nullptr, n_params, bytes, 0, false, id);
}

static sg_status submit(sg_server* v, uint32_t sid, const double* p, uint64_t seed, const void* const* e_fwd,
                        const void* const* e_adj, double omega, uint64_t* ticket) {
    if (!v || !ticket) return fail(SG_E_INVALID, "serve_submit: NULL argument");
    const bool caller = e_fwd != nullptr || e_adj != nullptr;
    Req* r;
    {
        std::lock_guard<std::mutex> lk(v->mu);
        if (sid >= v->sessions.size()) return fail(SG_E_INVALID, "serve_submit: unknown session %u", sid);
        Session* s = v->sessions[sid].get();
        if (s->n_params > 0 && !p) return fail(SG_E_INVALID, "serve_submit: p is NULL");
        for (int64_t k = 0; k < s->n_params; ++k)
            if (!std::isfinite(p[k])) return fail(SG_E_INVALID, "serve_submit: p[%lld] not finite", (long long)k);
        if (!std::isfinite(omega)) return fail(SG_E_INVALID, "serve_submit: omega not finite");
        if (caller) {
            if (!s->scene) return fail(SG_E_INVALID, "serve_submit_fields: a fake session has no planes");
            if (!e_fwd || !e_adj) return fail(SG_E_INVALID, "serve_submit_fields: field pointer arrays are NULL");
            for (int c = 0; c < s->scene->ncomp; ++c)
                if (!e_fwd[c] || !e_adj[c]) return fail(SG_E_INVALID, "serve_submit_fields: field plane %d is NULL", c);
        }
        const int64_t need = s->stage_bytes + (caller ? 0 : s->field_bytes);
        if (need > v->opts.hbm_budget_bytes)
            return fail(SG_E_TOO_LARGE, "request needs %lld bytes, budget is %lld", (long long)need,
                        (long long)v->opts.hbm_budget_bytes);
        if (v->stop) return fail(SG_E_INVALID, "server is shutting down");
        r = new Req;
        r->ticket = v->next_ticket++;
        r->s = s;
        r->p.assign(p, p + s->n_params);
        r->seed = seed;
        r->caller = caller;
        if (caller)
            for (int c = 0; c < s->scene->ncomp; ++c) {
                r->ce[c] = (const float2*)e_fwd[c];
                r->ca[c] = (const float2*)e_adj[c];
            }
        r->omega = omega;
        r->st.submit_ns = now_ns();
        v->reqs[r->ticket] = r;
        v->pending.push_back(r);
        *ticket = r->ticket;
    }
    v->cv_work.notify_one();
    return SG_OK;
}

extern "C" sg_status serve_submit(sg_server* v, uint32_t sid, const double* p, uint64_t seed, double omega,
                                  uint64_t* ticket) {
    return submit(v, sid, p, seed, nullptr, nullptr, omega, ticket);
}

extern "C" sg_status serve_submit_fields(sg_server* v, uint32_t sid, const double* p, const void* const* e_fwd,
                                         const void* const* e_adj, double omega, uint64_t* ticket) {
    if (!e_fwd || !e_adj) return fail(SG_E_INVALID, "serve_submit_fields: field pointer arrays are NULL");
    return submit(v, sid, p, 0, e_fwd, e_adj, omega, ticket);
}

extern "C" sg_status serve_poll(sg_server* v, uint64_t ticket, double* grad_out, int64_t timeout_us,
                                sg_req_stats* stats) {
    if (!v) return fail(SG_E_INVALID, "serve_poll: NULL server");
    std::unique_lock<std::mutex> lk(v->mu);
    auto it = v->reqs.find(ticket);
    if (it == v->reqs.end()) return fail(SG_E_INVALID, "serve_poll: unknown ticket %llu", (unsigned long long)ticket);
    Req* r = it->second;
    auto final_state = [&] { return r->state == DONE || r->state == CANCELLED || r->state == FAILED; };
    if (!final_state()) {
        if (timeout_us < 0) v->cv_done.wait(lk, final_state);
        else if (timeout_us > 0) v->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), final_state);
    }
    if (!final_state()) return SG_EAGAIN;
    const sg_status st = r->status;
    if (st == SG_OK && r->s->n_params > 0) {
        if (!grad_out) return fail(SG_E_INVALID, "serve_poll: grad_out is NULL");
        std::memcpy(grad_out, r->grad.data(), r->s->n_params * sizeof(double));
    }
    if (stats) *stats = r->st;
    v->reqs.erase(it);
    delete r;
    if (st == SG_E_CANCELLED) return fail(SG_E_CANCELLED, "request %llu was cancelled", (unsigned long long)ticket);
    if (st == SG_E_NOMEM)
        return fail(st, "request %llu: no device memory for its buffers while nothing else ran",
                    (unsigned long long)ticket);
    if (st != SG_OK) return fail(st, "request %llu failed on the device", (unsigned long long)ticket);
    return SG_OK;
}

extern "C" sg_status serve_cancel(sg_server* v, uint64_t ticket) {
    if (!v) return fail(SG_E_INVALID, "serve_cancel: NULL server");
    std::lock_guard<std::mutex> lk(v->mu);
    auto it = v->reqs.find(ticket);
    if (it == v->reqs.end()) return fail(SG_E_INVALID, "serve_cancel: unknown ticket");
    Req* r = it->second;
    if (r->state == PENDING) {
        v->pending.erase(std::find(v->pending.begin(), v->pending.end(), r));
        r->state = CANCELLED;
        r->status = SG_E_CANCELLED;
    } else if (r->state == ADMITTED) {
        drop_ready(v, r);
        r->state = CANCELLED;
        r->status = SG_E_CANCELLED;
        release(v, r);
    } else if (r->state == LAUNCHED) {
        r->cancel = true;      // its slices in flight finish; no more are launched
    }
    v->cv_done.notify_all();
    v->cv_work.notify_one();
    return SG_OK;
}

extern "C" sg_status serve_counters(sg_server* v, int64_t* completed, int64_t* batches, int64_t* max_batch_seen,
                                    int64_t* bytes_in_use, int64_t* bytes_held) {
    if (!v) return fail(SG_E_INVALID, "NULL server");
    std::lock_guard<std::mutex> lk(v->mu);
    if (completed) *completed = v->completed;
    if (batches) *batches = v->launches;
    if (max_batch_seen) *max_batch_seen = v->max_batch_seen;
    if (bytes_in_use) *bytes_in_use = v->bytes_used;
    if (bytes_held) *bytes_held = v->bytes_held;
    return SG_OK;
}
