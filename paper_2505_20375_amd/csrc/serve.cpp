// Continuous-batching request server for CI solves.
//
// Requests (integrals, space, Davidson options) queue on submission; their
// host-side setup (string tables, transposed integrals) happens then.  Each
// tick
//   1. admits queued requests in FIFO order while the slot count and the
//      device-memory budget allow (the footprint is computed exactly from
//      the sizes the context will allocate),
//   2. launches the pending sigma products of every active request, each on
//      the request's own path and stream, so that they overlap on the
//      device,
//   3. advances every active request by one Davidson iteration and retires
//      the finished ones, releasing their memory for the next admissions.
//      Each active request owns a HIP stream; the iterations of different
//      requests run on host worker threads, so that one request's host work
//      and synchronisation round trips overlap the others' device work.
// Requests therefore join and leave between ticks while others are on the
// device; their vectors stay resident from admission to completion.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/stpci.h"
#include "../../include/stpci_serve.h"
#include "ctx.hpp"
#include "kernels.hpp"

using namespace stp;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum ReqState { QUEUED = 0, ACTIVE = 1, DONE = 2, FAILED = 3, CANCELLED = 4 };

struct Req {
    int id = 0;
    stpci_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;  // owned by the server's pool while active
    stpci_dav_opts opts{};
    int64_t footprint = 0;
    int state = QUEUED;
    stpci_status status = STPCI_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<double> energies, resid;
    int n_iter = 0;
    int64_t n_dets = 0;
    double nnz = 0;
    int sigma_vectors = 0;
    std::string err;
};

}  // namespace

struct stpci_server {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t budget = 0;
    int max_active = 0;
    int64_t used = 0, peak_used = 0;
    int peak_active = 0;
    int64_t ticks = 0, sigma_launches = 0;
    double t_admit = 0, t_sigma = 0, t_step = 0;   // wall seconds spent in the tick's three phases
    std::vector<std::unique_ptr<Req>> reqs;
    std::deque<int> queue;
    std::vector<int> active;
    std::vector<hipStream_t> free_streams;  // request streams not in use
    std::string err;
    ~stpci_server() {
        (void)hipSetDevice(device);
        for (auto& r : reqs) {
            stpci_destroy(r->ctx);
            if (r->stream) (void)hipStreamDestroy(r->stream);
        }
        for (hipStream_t st : free_streams) (void)hipStreamDestroy(st);
    }
};

// Hand a request's stream back to the pool once its work has drained.
static void release_stream(stpci_server* s, Req& q) {
    if (!q.stream) return;
    (void)hipStreamSynchronize(q.stream);
    s->free_streams.push_back(q.stream);
    q.stream = nullptr;
}

static int64_t store_bytes(const stpci_ctx* c) {
    DevSpace tmp{};
    tmp.sp = c->hs.sp;
    return (int64_t)pair_store_bytes(tmp, c->cplx);
}

// Device bytes a request holds while active: tables, integrals (with the
// FP32 or bfloat16 copies of the reduced-precision forms), the schedule of the row-tiled
// fallback kernel where the tile kernel does not apply, the Davidson
// vectors and workspace, and the sigma kernel's own workspace (the
// store-and-reduce workspace where it fits 1 GB, larger ones being sent to
// device atomics when the request is created, and the grouped kernel's
// items, counted as one per intermediate).
static int64_t footprint(const stpci_ctx* c, const stpci_dav_opts& o) {
    int64_t b = device_table_bytes(c, o.precision == STPCI_FP32) + dav_device_bytes(c, o);
    if (o.precision == STPCI_BF16 && select_kernel(c) == 4) {
        const int64_t npp = pair_mfma_npp(c->M * (c->M - 1) / 2);
        b += npp * npp * (c->cplx ? 3 : 1) * 2;   // the bfloat16 pair table
    }
    const int64_t eb = store_bytes(c);
    if (eb <= ((int64_t)1 << 30)) b += eb;
    if (o.precision != STPCI_BF16) b += c->hs.sp.npwork_dets * (int64_t)sizeof(GrpItem);
    return b;
}

// host threads that advance the active requests' Davidson iterations
constexpr int kWorkers = 8;

static stpci_status srv_err(stpci_server* s, stpci_status st, const std::string& m) {
    s->err = m;
    return st;
}

// The pending sigma products of several step-wise Davidson runs on one
// device, each on its context's own path and stream: the launches of all
// runs are issued back to back and overlap on the device.  (One launch over
// the intermediates of all runs, per kernel family, was slower: it sizes the
// workspace of every intermediate by the largest degree in the group and
// gives up each run's own kernel choice; 48 solves of 1e4 to 3e5
// determinants took 1.86 s that way against 1.75 s.)  st[i]: status of
// ctxs[i] (its error text in its stpci_last_error); ran[i]: its products were
// launched (contexts without pending products are skipped).
static void sigma_batch(stpci_ctx* const* ctxs, int n, std::vector<stpci_status>& st, std::vector<char>& ran,
                        int64_t* launches) {
    st.assign(n, STPCI_OK);
    ran.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        stpci_ctx* c = ctxs[i];
        const void* in;
        void* out;
        int nv;
        stpci_precision prec;
        if (!dav_pending(c, &in, &out, &nv, &prec)) continue;
        st[i] = sigma_impl(c, in, out, nv, prec);
        ran[i] = st[i] == STPCI_OK;
        if (ran[i]) {
            c->dav.products_ready = true;
            if (launches) ++*launches;
        }
    }
}

extern "C" {

stpci_status stpci_server_create(stpci_server** out, int hip_device, void* hip_stream, int64_t mem_budget_bytes,
                                 int max_active) {
    if (!out || hip_device < 0 || mem_budget_bytes <= 0 || max_active < 1) return STPCI_EINVAL;
    *out = nullptr;
    if (hipSetDevice(hip_device) != hipSuccess) return STPCI_EHIP;
    stpci_server* s = new (std::nothrow) stpci_server();
    if (!s) return STPCI_ENOMEM;
    s->device = hip_device;
    s->stream = (hipStream_t)hip_stream;
    s->budget = mem_budget_bytes;
    s->max_active = max_active;
    *out = s;
    return STPCI_OK;
}

void stpci_server_destroy(stpci_server* s) { delete s; }

const char* stpci_server_last_error(const stpci_server* s) { return s ? s->err.c_str() : "null server"; }

stpci_status stpci_server_submit(stpci_server* s, const stpci_request* r, int* id) {
    if (!s || !r || !id || !r->opts) return STPCI_EINVAL;
    std::unique_ptr<Req> q(new (std::nothrow) Req());
    if (!q) return STPCI_ENOMEM;
    stpci_status st = stpci_create(&q->ctx, s->device, (void*)s->stream);
    if (st) return srv_err(s, st, "context creation failed");
    if ((st = stpci_set_integrals(q->ctx, r->n_orb, r->scalar, r->spin_free, r->h, r->g, r->e_core)) ||
        (st = stpci_set_space(q->ctx, r->n_elec, r->n_sub, r->sub_size, r->win_lo, r->win_hi))) {
        std::string m = stpci_last_error(q->ctx);
        stpci_destroy(q->ctx);
        q->ctx = nullptr;
        return srv_err(s, st, m);
    }
    if (q->ctx->hs.sp.M != q->ctx->M) {
        stpci_destroy(q->ctx);
        q->ctx = nullptr;
        return srv_err(s, STPCI_EINVAL, "space and integrals cover different numbers of spin-orbitals");
    }
    q->opts = *r->opts;
    q->opts.guess_dev = nullptr;
    if (q->opts.k < 1 || q->opts.k > 16 || q->opts.k > q->ctx->hs.sp.ndets) {
        stpci_destroy(q->ctx);
        q->ctx = nullptr;
        return srv_err(s, STPCI_EINVAL, "k must be in [1, min(16, n_dets)]");
    }
    if (select_kernel(q->ctx) == 4 && store_bytes(q->ctx) > ((int64_t)1 << 30))
        (void)stpci_set_sigma_kernel(q->ctx, "pair_atomic");   // no workspace outside the footprint
    q->footprint = footprint(q->ctx, q->opts);
    if (q->footprint > s->budget) {
        stpci_destroy(q->ctx);
        q->ctx = nullptr;
        return srv_err(s, STPCI_ENOMEM, "request footprint exceeds the server's memory budget");
    }
    q->n_dets = q->ctx->hs.sp.ndets;
    q->nnz = q->ctx->hs.nnz;
    q->id = (int)s->reqs.size();
    q->t_submit = now_s();
    *id = q->id;
    s->queue.push_back(q->id);
    s->reqs.push_back(std::move(q));
    return STPCI_OK;
}

stpci_status stpci_server_cancel(stpci_server* s, int id) {
    if (!s || id < 0 || id >= (int)s->reqs.size()) return STPCI_EINVAL;
    Req& q = *s->reqs[id];
    if (q.state == QUEUED) {
        s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), id), s->queue.end());
    } else if (q.state == ACTIVE) {
        s->active.erase(std::remove(s->active.begin(), s->active.end(), id), s->active.end());
        s->used -= q.footprint;
    } else {
        return STPCI_OK;
    }
    q.state = CANCELLED;
    q.t_done = now_s();
    stpci_destroy(q.ctx);
    q.ctx = nullptr;
    release_stream(s, q);
    return STPCI_OK;
}

static stpci_status collect(Req& q) {
    const int k = q.opts.k;
    q.energies.assign(k, 0.0);
    q.resid.assign(k, 0.0);
    return dav_collect(q.ctx, q.energies.data(), q.resid.data(), nullptr, &q.n_iter);
}

static void retire(stpci_server* s, Req& q, stpci_status st) {
    q.status = st;
    q.state = (st == STPCI_OK || st == STPCI_ENOCONV) ? DONE : FAILED;
    if (q.ctx) {
        q.err = stpci_last_error(q.ctx);
        q.sigma_vectors = q.ctx->nsigma[0] + q.ctx->nsigma[1] + q.ctx->nsigma[2];
    }
    q.t_done = now_s();
    stpci_destroy(q.ctx);
    q.ctx = nullptr;
    release_stream(s, q);
    s->used -= q.footprint;
    s->active.erase(std::remove(s->active.begin(), s->active.end(), q.id), s->active.end());
}

stpci_status stpci_server_tick(stpci_server* s, int* n_active, int* n_finished) {
    if (!s) return STPCI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return srv_err(s, STPCI_EHIP, "hipSetDevice");
    int finished = 0;
    const double t0 = now_s();
    // 1. FIFO admission by slots and device-memory budget
    while (!s->queue.empty() && (int)s->active.size() < s->max_active) {
        Req& q = *s->reqs[s->queue.front()];
        if (s->used + q.footprint > s->budget) break;
        s->queue.pop_front();
        q.state = ACTIVE;
        q.t_admit = now_s();
        s->active.push_back(q.id);
        s->used += q.footprint;
        stpci_status st = STPCI_OK;
        if (s->free_streams.empty()) {
            hipStream_t ns = nullptr;
            if (hipStreamCreateWithFlags(&ns, hipStreamNonBlocking) != hipSuccess) st = STPCI_EHIP;
            else s->free_streams.push_back(ns);
        }
        if (!st) {
            q.stream = s->free_streams.back();
            s->free_streams.pop_back();
            q.ctx->stream = q.stream;
            st = dav_begin(q.ctx, &q.opts);
        }
        if (!st && q.opts.precision == STPCI_FP32) st = ensure32(q.ctx);
        if (st) {
            retire(s, q, st);
            ++finished;
        }
    }
    s->peak_used = std::max(s->peak_used, s->used);
    s->peak_active = std::max(s->peak_active, (int)s->active.size());
    const double t1 = now_s();
    // 2. pending sigma products of all active requests, each on its own
    // stream
    const std::vector<int> admitted(s->active);  // retire() edits the active list
    std::vector<stpci_ctx*> cs;
    for (int id : admitted) cs.push_back(s->reqs[id]->ctx);
    std::vector<stpci_status> bst;
    std::vector<char> ran;
    sigma_batch(cs.data(), (int)cs.size(), bst, ran, &s->sigma_launches);
    std::vector<int> stepped;
    for (size_t i = 0; i < admitted.size(); ++i) {
        Req& q = *s->reqs[admitted[i]];
        if (bst[i]) {
            retire(s, q, bst[i]);
            ++finished;
        } else if (ran[i]) {
            stepped.push_back(q.id);
        }
    }
    const double t2 = now_s();
    // 3. one Davidson iteration for every request whose products were
    // computed, on worker threads (each request on its own stream; a
    // request's state is touched by one thread only)
    std::sort(stepped.begin(), stepped.end());
    stepped.erase(std::unique(stepped.begin(), stepped.end()), stepped.end());
    stepped.erase(std::remove_if(stepped.begin(), stepped.end(),
                                 [&](int id) { return s->reqs[id]->state != ACTIVE; }),
                  stepped.end());
    const int ns = (int)stepped.size();
    std::vector<stpci_status> sts(ns, STPCI_OK);
    std::vector<int> fins(ns, 0);
    std::atomic<int> next{0};
    auto work = [&]() {
        if (hipSetDevice(s->device) != hipSuccess) {
            for (int i; (i = next.fetch_add(1)) < ns;) sts[i] = STPCI_EHIP;
            return;
        }
        for (int i; (i = next.fetch_add(1)) < ns;) {
            Req& q = *s->reqs[stepped[i]];
            sts[i] = dav_step_after_sigma(q.ctx, &fins[i]);
            if (!sts[i] && fins[i]) sts[i] = collect(q);
        }
    };
    const int nthreads = std::min(ns, kWorkers);
    std::vector<std::thread> pool;
    for (int t = 1; t < nthreads; ++t) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
    for (int i = 0; i < ns; ++i) {
        if (sts[i] || fins[i]) {
            retire(s, *s->reqs[stepped[i]], sts[i]);
            ++finished;
        }
    }
    ++s->ticks;
    const double t3 = now_s();
    s->t_admit += t1 - t0;
    s->t_sigma += t2 - t1;
    s->t_step += t3 - t2;
    if (n_active) *n_active = (int)s->active.size() + (int)s->queue.size();  // pending after the step
    if (n_finished) *n_finished = finished;
    return STPCI_OK;
}

stpci_status stpci_server_result(const stpci_server* s, int id, int* state, double* energies, double* resid,
                                 int* n_iter, double* t_submit, double* t_admit, double* t_done) {
    if (!s || id < 0 || id >= (int)s->reqs.size()) return STPCI_EINVAL;
    const Req& q = *s->reqs[id];
    if (state) *state = q.state;
    if (energies)
        for (size_t j = 0; j < q.energies.size(); ++j) energies[j] = q.energies[j];
    if (resid)
        for (size_t j = 0; j < q.resid.size(); ++j) resid[j] = q.resid[j];
    if (n_iter) *n_iter = q.n_iter;
    if (t_submit) *t_submit = q.t_submit;
    if (t_admit) *t_admit = q.t_admit;
    if (t_done) *t_done = q.t_done;
    return q.state == FAILED ? q.status : STPCI_OK;
}

stpci_status stpci_server_request_info(const stpci_server* s, int id, int64_t* n_dets, double* nnz_h,
                                       int64_t* footprint_bytes, int* sigma_vectors) {
    if (!s || id < 0 || id >= (int)s->reqs.size()) return STPCI_EINVAL;
    const Req& q = *s->reqs[id];
    if (n_dets) *n_dets = q.n_dets;
    if (nnz_h) *nnz_h = q.nnz;
    if (footprint_bytes) *footprint_bytes = q.footprint;
    if (sigma_vectors) *sigma_vectors = q.sigma_vectors;
    return STPCI_OK;
}

stpci_status stpci_server_phase_times(const stpci_server* s, double* admit_s, double* sigma_s, double* step_s) {
    if (!s) return STPCI_EINVAL;
    if (admit_s) *admit_s = s->t_admit;
    if (sigma_s) *sigma_s = s->t_sigma;
    if (step_s) *step_s = s->t_step;
    return STPCI_OK;
}

stpci_status stpci_server_stats(const stpci_server* s, int64_t* used_bytes, int64_t* peak_bytes, int* peak_active,
                                int64_t* ticks, int64_t* sigma_launches) {
    if (!s) return STPCI_EINVAL;
    if (used_bytes) *used_bytes = s->used;
    if (peak_bytes) *peak_bytes = s->peak_used;
    if (peak_active) *peak_active = s->peak_active;
    if (ticks) *ticks = s->ticks;
    if (sigma_launches) *sigma_launches = s->sigma_launches;
    return STPCI_OK;
}

// ---- step-wise Davidson: the server's steps as separate calls -------------

int64_t stpci_footprint_bytes(const stpci_ctx* c, const stpci_dav_opts* o) {
    if (!c || !o || !c->have_ints || !c->have_space || c->hs.sp.M != c->M) return -1;
    if (o->k < 1 || o->k > 16 || o->k > c->hs.sp.ndets) return -1;
    stpci_dav_opts oo = *o;
    // the extra root of a certified run or of the energy stop
    const bool extra = o->certify || (o->refine_tol_energy > 0.0 && o->precision != STPCI_FP64);
    if (extra && oo.k < 16 && oo.k < c->hs.sp.ndets) ++oo.k;
    return footprint(c, oo);
}

stpci_status stpci_dav_begin(stpci_ctx* c, const stpci_dav_opts* o) {
    if (!c || !o) return STPCI_EINVAL;
    if (c->host_only) return set_err(c, STPCI_ESTATE, "host-only context");
    stpci_status st = dav_begin(c, o);
    if (!st && o->precision == STPCI_FP32) st = ensure32(c);   // tables of the FP32 phase
    return st;
}

stpci_status stpci_dav_sigma_batched(stpci_ctx* const* ctxs, int n) {
    if (!ctxs || n < 1) return STPCI_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!ctxs[i]) return STPCI_EINVAL;
    stpci_ctx* lead = ctxs[0];
    for (int i = 0; i < n; ++i) {
        if (ctxs[i]->host_only) return set_err(ctxs[i], STPCI_ESTATE, "host-only context");
        if (ctxs[i]->device != lead->device)
            return set_err(ctxs[i], STPCI_EINVAL, "contexts of one batched call must share a device");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return set_err(ctxs[i], STPCI_EINVAL, "a context appears twice");
    }
    if (hipSetDevice(lead->device) != hipSuccess) return set_err(lead, STPCI_EHIP, "hipSetDevice");
    std::vector<stpci_status> st;
    std::vector<char> ran;
    sigma_batch(ctxs, n, st, ran, nullptr);
    for (int i = 0; i < n; ++i)
        if (st[i]) return st[i];   // the context's own error text is set
    return STPCI_OK;
}

stpci_status stpci_dav_finish_step(stpci_ctx* c, int* done) {
    if (!c || !done) return STPCI_EINVAL;
    *done = 0;
    DavState& D = c->dav;
    if (!D.active) return set_err(c, STPCI_ESTATE, "no step-wise Davidson run in progress");
    if (!D.products_ready)
        return set_err(c, STPCI_ESTATE, "the pending sigma products were not computed (stpci_dav_sigma_batched)");
    if (hipSetDevice(c->device) != hipSuccess) return set_err(c, STPCI_EHIP, "hipSetDevice");
    return dav_step_after_sigma(c, done);
}

stpci_status stpci_dav_result(stpci_ctx* c, double* energies, double* resid, void* vecs_dev, int* n_iter) {
    if (!c || !energies || !resid) return STPCI_EINVAL;
    if (!c->dav.done) return set_err(c, STPCI_ESTATE, "the Davidson run has not finished");
    if (hipSetDevice(c->device) != hipSuccess) return set_err(c, STPCI_EHIP, "hipSetDevice");
    return dav_collect(c, energies, resid, vecs_dev, n_iter);
}

}  // extern "C"
