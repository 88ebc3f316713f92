// Serving loop: continuous batching of source-term requests from many host
// callers into fused multi-request launches (ak_server_* in annkin.h).
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <memory>
#include <mutex>
#include <vector>

#include "annkin.h"
#include "ak_device.h"
#include "ak_internal.h"
#include "ak_sched.h"

namespace ak {

static size_t elem_size(int prec) { return prec == AK_FP64 ? 8 : 4; }

// Arena layout of one request: T[n], P[n], Y[NS][n], omega[NS][n], each
// array 256-byte aligned.
static size_t request_bytes(int prec, int ns, int64_t n)
{
    const size_t e = elem_size(prec);
    return 2 * Arena::round(e * n) + 2 * Arena::round(e * n * ns);
}

struct GpuExec {
    struct Slot {
        hipStream_t st = nullptr;
        std::vector<hipEvent_t> ev;      // per request of the batch: its copy-out done
        BatchDesc *d_desc[2] = {nullptr, nullptr};
        BatchDesc *h_desc[2] = {nullptr, nullptr};
        JitBatchDesc *d_jdesc = nullptr;   // requests of mechanism-compiled kernels
        JitBatchDesc *h_jdesc = nullptr;
        int nlaunch = 0;
        int rc = 0;
        bool busy = false;
        std::string what;                // the failed HIP call, if any
    };
    int device = 0;
    unsigned char *arena = nullptr;
    bool own_arena = true;           // false: the caller's buffer
    int max_req = 64;
    std::vector<Slot> slots;
    std::mutex mu;

    int init(int dev, size_t arena_bytes, int inflight, int max_requests, void *ext)
    {
        device = dev;
        max_req = max_requests;
        DeviceGuard g(dev);
        if (!g.ok) return set_error(AK_EDEVICE, "ak_server_create: cannot select device %d", dev);
        hipError_t e;
        if (ext) {
            // the caller's arena: device memory of this device, aligned
            hipPointerAttribute_t at{};
            e = hipPointerGetAttributes(&at, ext);
            if (e != hipSuccess || at.type != hipMemoryTypeDevice || at.device != dev) {
                (void)hipGetLastError();
                return set_error(AK_EINVAL, "ak_server_create: the arena is not device memory of "
                                            "device %d", dev);
            }
            if ((uintptr_t)ext % 256)
                return set_error(AK_EINVAL, "ak_server_create: the arena is not 256-byte aligned");
            arena = (unsigned char *)ext;
            own_arena = false;
        } else if ((e = hipMalloc((void **)&arena, arena_bytes)) != hipSuccess) {
            arena = nullptr;
            return set_error(AK_ENOMEM, "ak_server_create: arena of %zu bytes: %s", arena_bytes,
                             hipGetErrorString(e));
        }
        slots.resize(inflight);
        for (Slot &s : slots) {
            if ((e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking)) != hipSuccess)
                return hip_error(e, "ak_server_create: stream");
            s.ev.assign(max_requests, nullptr);
            for (hipEvent_t &ev : s.ev)
                if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
                    return hip_error(e, "ak_server_create: events");
            for (int p = 0; p < 2; ++p) {
                if ((e = hipMalloc((void **)&s.d_desc[p], sizeof(BatchDesc) * max_req)) !=
                        hipSuccess ||
                    (e = hipHostMalloc((void **)&s.h_desc[p], sizeof(BatchDesc) * max_req,
                                       hipHostMallocDefault)) != hipSuccess)
                    return set_error(AK_ENOMEM, "ak_server_create: descriptor tables: %s",
                                     hipGetErrorString(e));
            }
            if ((e = hipMalloc((void **)&s.d_jdesc, sizeof(JitBatchDesc) * max_req)) !=
                    hipSuccess ||
                (e = hipHostMalloc((void **)&s.h_jdesc, sizeof(JitBatchDesc) * max_req,
                                   hipHostMallocDefault)) != hipSuccess)
                return set_error(AK_ENOMEM, "ak_server_create: descriptor tables: %s",
                                 hipGetErrorString(e));
        }
        return AK_OK;
    }

    void destroy()
    {
        DeviceGuard g(device);
        for (Slot &s : slots) {
            if (s.st) (void)hipStreamSynchronize(s.st);
            for (int p = 0; p < 2; ++p) {
                if (s.d_desc[p]) (void)hipFree(s.d_desc[p]);
                if (s.h_desc[p]) (void)hipHostFree(s.h_desc[p]);
            }
            if (s.d_jdesc) (void)hipFree(s.d_jdesc);
            if (s.h_jdesc) (void)hipHostFree(s.h_jdesc);
            for (hipEvent_t ev : s.ev)
                if (ev) (void)hipEventDestroy(ev);
            if (s.st) (void)hipStreamDestroy(s.st);
        }
        slots.clear();
        if (arena && own_arena) (void)hipFree(arena);
        arena = nullptr;
    }

    // Enqueue copies in, one fused launch per precision, and per request its
    // copy out followed by its event.
    void *launch(const std::vector<Request *> &reqs)
    {
        Slot *s = nullptr;
        {
            std::lock_guard<std::mutex> g(mu);
            for (Slot &c : slots)
                if (!c.busy) {
                    c.busy = true;
                    s = &c;
                    break;
                }
        }
        if (!s) return nullptr;   // cannot happen: the scheduler bounds in-flight batches
        DeviceGuard g(device);
        s->rc = 0;
        s->nlaunch = 0;
        hipError_t e = hipSuccess;
        const char *step = "";
        auto ok = [&](hipError_t x) {
            if (x != hipSuccess && e == hipSuccess) {
                e = x;
                s->what = std::string(step) + ": " + hipGetErrorString(x);
            }
            return x == hipSuccess;
        };
        for (Request *r : reqs) {
            const size_t es = elem_size(r->prec);
            unsigned char *b = arena + r->arena_off;
            unsigned char *dT = b, *dP = dT + Arena::round(es * r->n);
            unsigned char *dY = dP + Arena::round(es * r->n);
            step = "copy in";
            ok(hipMemcpyAsync(dT, r->T, es * r->n, hipMemcpyHostToDevice, s->st));
            ok(hipMemcpyAsync(dP, r->P, es * r->n, hipMemcpyHostToDevice, s->st));
            ok(hipMemcpy2DAsync(dY, es * r->n, r->Y, es * r->ldY, es * r->n, r->ns,
                                hipMemcpyHostToDevice, s->st));
        }
        // Requests whose mechanism has compiled kernels for their precision:
        // one launch per (mechanism, precision), with the same kernel that
        // ak_eval_source runs, so that a request's result does not depend on
        // its batch.  All other requests: one fused launch of the table-driven
        // kernel per precision.
        std::vector<std::pair<const JitKernels *, std::vector<const Request *>>> groups;
        for (const Request *r : reqs) {
            const JitKernels *jk = &((const ak_mechanism *)r->mech)->jit[r->prec];
            if (!jk->src) continue;
            size_t gi = 0;
            while (gi < groups.size() && groups[gi].first != jk) ++gi;
            if (gi == groups.size()) groups.push_back({jk, {}});
            groups[gi].second.push_back(r);
        }
        if (!groups.empty()) {
            // descriptor table: the groups one after another, block offsets
            // counted within each group
            std::vector<int> first(groups.size() + 1, 0);
            std::vector<int64_t> gblocks(groups.size(), 0);
            int nj = 0;
            for (size_t gi = 0; gi < groups.size(); ++gi) {
                first[gi] = nj;
                const int block = groups[gi].first->block;
                for (const Request *r : groups[gi].second) {
                    const size_t es = elem_size(r->prec);
                    unsigned char *b = arena + r->arena_off;
                    JitBatchDesc &d = s->h_jdesc[nj++];
                    d.T = b;
                    d.P = b + Arena::round(es * r->n);
                    d.Y = b + 2 * Arena::round(es * r->n);
                    d.om = b + 2 * Arena::round(es * r->n) + Arena::round(es * r->n * r->ns);
                    d.ldY = d.ldO = d.n = r->n;
                    d.block_begin = gblocks[gi];
                    gblocks[gi] += (r->n + block - 1) / block;
                }
            }
            first[groups.size()] = nj;
            step = "descriptor table";
            ok(hipMemcpyAsync(s->d_jdesc, s->h_jdesc, sizeof(JitBatchDesc) * nj,
                              hipMemcpyHostToDevice, s->st));
            step = "compiled-kernel launch";
            for (size_t gi = 0; gi < groups.size(); ++gi) {
                const ak_mechanism *m = (const ak_mechanism *)groups[gi].second[0]->mech;
                ok(jit_batch_launch(*groups[gi].first, s->d_jdesc + first[gi],
                                    first[gi + 1] - first[gi], gblocks[gi], m->view.err,
                                    s->st));
                s->nlaunch++;
            }
        }
        for (int p = 0; p < 2; ++p) {
            const int prec = p == 0 ? AK_FP32 : AK_FP64;
            int nd = 0;
            int64_t blocks = 0;
            size_t lds = 0;
            int max_ns = 0;
            for (Request *r : reqs) {
                if (r->prec != prec) continue;
                const ak_mechanism *m = (const ak_mechanism *)r->mech;
                if (m->jit[r->prec].src) continue;
                const size_t es = elem_size(r->prec);
                unsigned char *b = arena + r->arena_off;
                BatchDesc &d = s->h_desc[p][nd++];
                d.m = m->view;
                d.T = b;
                d.P = b + Arena::round(es * r->n);
                d.Y = b + 2 * Arena::round(es * r->n);
                d.om = b + 2 * Arena::round(es * r->n) + Arena::round(es * r->n * r->ns);
                d.ldY = d.ldO = d.n = r->n;
                d.block_begin = blocks;
                blocks += (r->n + m->view.tile - 1) / m->view.tile;
                lds = std::max(lds, source_lds_bytes(m->ns, m->view.tile));
                max_ns = std::max(max_ns, m->ns);
            }
            if (!nd) continue;
            step = "descriptor table";
            ok(hipMemcpyAsync(s->d_desc[p], s->h_desc[p], sizeof(BatchDesc) * nd,
                              hipMemcpyHostToDevice, s->st));
            step = "fused launch";
            ok(source_batch_launch(prec == AK_FP64, s->d_desc[p], nd, blocks, lds, max_ns,
                                   s->st));
            s->nlaunch++;
        }
        for (size_t i = 0; i < reqs.size(); ++i) {
            const Request *r = reqs[i];
            const size_t es = elem_size(r->prec);
            unsigned char *dO = arena + r->arena_off + 2 * Arena::round(es * r->n) +
                                Arena::round(es * r->n * r->ns);
            step = "copy out";
            ok(hipMemcpy2DAsync(r->om, es * r->ldO, dO, es * r->n, es * r->n, r->ns,
                                hipMemcpyDeviceToHost, s->st));
            step = "event";
            ok(hipEventRecord(s->ev[i], s->st));
        }
        if (e != hipSuccess) s->rc = AK_EDEVICE;
        else s->what.clear();
        return s;
    }

    // Wait for request i of a batch; on failure *err says why (the text is
    // copied into the request, which outlives the server).
    int wait(void *token, size_t i, std::string *err)
    {
        if (!token) {
            *err = "no stream slot for the batch";
            return AK_EDEVICE;
        }
        Slot *s = (Slot *)token;
        DeviceGuard g(device);
        hipError_t e = hipEventSynchronize(s->ev[i]);
        if (e != hipSuccess) {
            *err = std::string("event wait: ") + hipGetErrorString(e);
            return AK_EDEVICE;
        }
        if (s->rc) *err = s->what;
        return s->rc;
    }

    int64_t launches(void *token) { return token ? ((Slot *)token)->nlaunch : 0; }

    void release(void *token)
    {
        if (!token) return;
        std::lock_guard<std::mutex> g(mu);
        ((Slot *)token)->busy = false;
    }
};

}  // namespace ak

using namespace ak;

struct ak_server {
    int device = 0;
    SchedConfig cfg;
    GpuExec exec;
    std::unique_ptr<Scheduler<GpuExec>> sched;
};

struct ak_request {
    Request r;
    ak_server *srv = nullptr;
};

extern "C" {

int ak_server_create(const ak_server_config *c, ak_server **out)
{
    if (!c || !out) return set_error(AK_EINVAL, "ak_server_create: null argument");
    *out = nullptr;
    SchedConfig cfg;
    if (c->arena && c->arena_bytes == 0)
        return set_error(AK_EINVAL, "ak_server_create: a caller arena needs arena_bytes > 0");
    cfg.arena_bytes = c->arena_bytes ? c->arena_bytes : ((size_t)1 << 30);
    cfg.max_inflight = c->max_inflight > 0 ? c->max_inflight : 3;
    cfg.max_batch_requests = c->max_batch_requests > 0 ? c->max_batch_requests : 64;
    cfg.max_batch_cells = c->max_batch_cells > 0 ? c->max_batch_cells : ((int64_t)1 << 16);
    cfg.small_cells = c->small_request_cells > 0 ? c->small_request_cells : 4096;
    cfg.batching = c->batching != 0;
    if (cfg.max_inflight > 16 || cfg.max_batch_requests > 4096)
        return set_error(AK_EINVAL, "ak_server_create: max_inflight <= 16, max_batch_requests <= 4096");
    ak_server *s = new (std::nothrow) ak_server();
    if (!s) return set_error(AK_ENOMEM, "ak_server_create: out of host memory");
    s->device = c->device;
    s->cfg = cfg;
    int rc = s->exec.init(c->device, cfg.arena_bytes, cfg.max_inflight, cfg.max_batch_requests,
                          c->arena);
    if (rc) {
        s->exec.destroy();
        delete s;
        return rc;
    }
    s->sched.reset(new Scheduler<GpuExec>(cfg, &s->exec));
    *out = s;
    return AK_OK;
}

int ak_server_submit(ak_server *s, const ak_mechanism *m, ak_precision prec, const void *T,
                     const void *P, const void *Y, int64_t ldY, int64_t n, void *omega,
                     int64_t ldO, ak_request **out)
{
    if (!s || !m || !out) return set_error(AK_EINVAL, "ak_server_submit: null argument");
    *out = nullptr;
    if (prec != AK_FP32 && prec != AK_FP64)
        return set_error(AK_EINVAL, "ak_server_submit: bad precision %d", (int)prec);
    if (n <= 0) return set_error(AK_EINVAL, "ak_server_submit: n_cells must be positive");
    if (!T || !P || !Y || !omega) return set_error(AK_EINVAL, "ak_server_submit: null buffer");
    if (ldY < n || ldO < n) return set_error(AK_EINVAL, "ak_server_submit: ldY or ldO < n_cells");
    if (m->device != s->device)
        return set_error(AK_EINVAL, "ak_server_submit: mechanism on device %d, server on %d",
                         m->device, s->device);
    if (m->pdep && !m->jit[prec].src)
        return set_error(AK_EUNSUPPORTED, "ak_server_submit: third-body and falloff reactions "
                                          "need the compiled kernel for this precision");
    ak_request *q = new (std::nothrow) ak_request();
    if (!q) return set_error(AK_ENOMEM, "ak_server_submit: out of host memory");
    q->srv = s;
    Request &r = q->r;
    r.mech = m;
    r.prec = prec;
    r.ns = m->ns;
    r.T = T;
    r.P = P;
    r.Y = Y;
    r.om = omega;
    r.ldY = ldY;
    r.ldO = ldO;
    r.n = n;
    r.bytes = request_bytes(prec, m->ns, n);
    const int rc = s->sched->submit(&r);
    if (rc) {
        delete q;
        return set_error(rc == -4 ? AK_E2BIG : AK_EINVAL,
                         rc == -4 ? "ak_server_submit: request of %lld cells exceeds the arena"
                                  : "ak_server_submit: server is shutting down (%lld cells)",
                         (long long)n);
    }
    *out = q;
    return AK_OK;
}

int ak_request_wait(ak_request *q, double timeout_s)
{
    if (!q) return set_error(AK_EINVAL, "ak_request_wait: null request");
    const int rc = Scheduler<GpuExec>::wait(&q->r, timeout_s);
    if (rc == -5) return set_error(AK_ETIMEDOUT, "ak_request_wait: timed out");
    if (rc == -6) return set_error(AK_ECANCELED, "ak_request_wait: request was cancelled");
    if (rc) {
        std::string why;
        {
            std::lock_guard<std::mutex> l(q->r.mu);
            why = q->r.error;
        }
        return set_error(rc, "ak_request_wait: request failed (%s)", why.c_str());
    }
    return AK_OK;
}

int ak_request_cancel(ak_request *q)
{
    if (!q) return set_error(AK_EINVAL, "ak_request_cancel: null request");
    return q->srv->sched->cancel(&q->r) == 0 ? AK_OK : 1;
}

int ak_request_free(ak_request *q)
{
    if (!q) return AK_OK;
    {
        std::lock_guard<std::mutex> l(q->r.mu);
        if (q->r.state < kDone)
            return set_error(AK_EINVAL, "ak_request_free: request still pending");
    }
    delete q;
    return AK_OK;
}

int ak_server_get_stats(ak_server *s, ak_server_stats *out)
{
    if (!s || !out) return set_error(AK_EINVAL, "ak_server_get_stats: null argument");
    SchedStats st = s->sched->stats();
    std::memset(out, 0, sizeof *out);
    out->submitted = st.submitted;
    out->completed = st.completed;
    out->cancelled = st.cancelled;
    out->failed = st.failed;
    out->batches = st.batches;
    out->launches = st.launches;
    out->cells = st.cells;
    out->queue_depth = (int64_t)s->sched->queue_depth();
    out->inflight = s->sched->inflight();
    out->arena_bytes = s->sched->arena_capacity();
    out->arena_used = s->sched->arena_used();
    out->p50_ms = percentile(st.latency, 50) * 1e3;
    out->p99_ms = percentile(st.latency, 99) * 1e3;
    double sum = 0, mx = 0;
    for (double v : st.latency) {
        sum += v;
        mx = std::max(mx, v);
    }
    out->mean_ms = st.latency.empty() ? 0.0 : sum / st.latency.size() * 1e3;
    out->max_ms = mx * 1e3;
    const double span = st.last_done - st.first_submit;
    out->cells_per_s = span > 0 ? st.cells / span : 0.0;
    return AK_OK;
}

int ak_server_reset_stats(ak_server *s)
{
    if (!s) return set_error(AK_EINVAL, "ak_server_reset_stats: null server");
    s->sched->reset_stats();
    return AK_OK;
}

int ak_server_destroy(ak_server *s)
{
    if (!s) return AK_OK;
    s->sched->shutdown();
    s->sched.reset();
    s->exec.destroy();
    delete s;
    return AK_OK;
}

}  // extern "C"
