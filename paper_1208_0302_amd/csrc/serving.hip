// Continuous-batching inversion service (the streaming use the paper aims at
// in Sec. 7: near real-time maps from a steady flow of observations).
//
// Requests (tiles of pixels, each with its own lines, bounds, genetic-
// algorithm settings and seed) are admitted in arrival order while their
// resident populations fit in a device-memory budget.  Every gs_step launch
// advances all resident requests together by up to K generations: one
// workgroup per pixel, the population resumed from HBM into LDS and stored
// back.  A request leaves as soon as it reaches its own generation count and
// its memory is returned, so later requests join the next launch.
//
// Every random number is a function of (request seed, request-local pixel id,
// generation, individual) and each pixel's arithmetic does not depend on what
// else is resident, so a request's result is bit-identical alone, in any mix,
// and to a single ga_invert call with the same settings.
#include <hip/hip_runtime.h>

#include <deque>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "genesis_common.h"
#include "scheduler.h"

namespace genesis {

struct ReqDesc {
    const float *obs, *sigma, *mu;
    uint16_t *genes;  // [npix][pop][9], session-owned
    float *fit;       // [npix][pop], session-owned
    float *best_params, *best_chi2;
    float *best_alpha;  // [npix], fill-fraction requests only
    int32_t *status;
    int64_t npix;
    int32_t generations;  // G of the request
    int32_t gen_done;     // generations completed before this launch, -1 = not started
    int32_t gen_to;       // generation to reach in this launch
    int32_t synth;        // GENESIS_SYNTH_NATIVE or GENESIS_SYNTH_FP16
    int32_t fill;         // 1: the fill-fraction merit of Sec. 5.2 (fc)
    int32_t pad_;
    DevLines<float> ls;
    DevLinesH lh;         // FP16 synthesis only
    Bounds b;
    GaConst ga;
    FillConst fc;         // fill-fraction requests only
};

}  // namespace genesis

using namespace genesis;

namespace {

__global__ __launch_bounds__(1024) void k_ga_advance(const ReqDesc *__restrict__ reqs,
                                                     const int64_t *__restrict__ first, int nreq)
{
    code_shift<GENESIS_PAD_ADVANCE>();
    extern __shared__ __align__(16) unsigned char smem[];
    // request of this workgroup: the last r with first[r] <= blockIdx.x
    const int64_t blk = blockIdx.x;
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= blk)
            lo = mid;
        else
            hi = mid - 1;
    }
    const ReqDesc &d = reqs[lo];
    const int64_t p = blk - first[lo];
    const int pop = d.ga.pop;
    const int L = d.ls.L;
    const GaLds<float> s = ga_lds<float>(smem, L, pop);
    const int tid = threadIdx.x;
    const bool active = tid < pop;
    // nu = 4L - 9, or 4L - 10 with the fill fraction as a tenth parameter
    const float inv_nu = (float)(1.0 / (4.0 * L - (d.fill ? GENESIS_NPAR + 1 : GENESIS_NPAR)));
    const bool finish = d.gen_to == d.generations;
    const double mu = d.mu ? (double)d.mu[p] : 1.0;
    FillPix<float> &fp = *reinterpret_cast<FillPix<float> *>(s.fill);

    if (tid == 0) {
        stage_box(d.b, d.ga.pixel_bounds, p, *s.box);
        if (d.fill)
            fill_setup(d.fc, d.ls.nlines, mu, fp);
    }
    float w2[4];
    int st = stage_pixel(d.obs + p * 4 * (int64_t)L, d.sigma + p * 4, L, s.obs, w2);
    if (st == 0 && d.ga.pixel_bounds)
        st = box_status(*s.box, d.synth == GENESIS_SYNTH_FP16);
    if (st == 0 && d.fill)
        st = fp.status;
    if (st != 0) {
        if (finish && tid == 0) {
            for (int j = 0; j < GENESIS_NPAR; ++j)
                d.best_params[p * GENESIS_NPAR + j] = NAN;
            d.best_chi2[p] = NAN;
            if (d.fill)
                d.best_alpha[p] = NAN;
            if (d.status)
                d.status[p] = st;
        }
        return;
    }
    const uint32_t pix = d.ga.pixel_base + (uint32_t)p;
    // a new request starts from generation 0; a resumed one from the
    // generation saved at the end of the previous launch (after its restart)
    GenState<float> gs;
    if (d.gen_done < 0) {
        gs = generation_zero(s, pop, tid, pix, p, d.ga);
    } else {
        gs = GenState<float>{d.gen_done, 0, false, true, 0.0f};
        if (active) {
            const int64_t row = p * pop + tid;
#pragma unroll
            for (int j = 0; j < GENESIS_NPAR; ++j)
                s.genes[j * pop + tid] = d.genes[row * GENESIS_NPAR + j];
            gs.f = d.fit[row];
            s.fit[tid] = gs.f;
        }
    }
    // the evaluation of the request's kind (uniform over the workgroup)
    if (d.synth == GENESIS_SYNTH_FP16 && d.fill) {
        generation_loop(s, pop, tid, pix, d.ga, d.generations, d.gen_to, nullptr, gs,
                        [&](const uint16_t *genes) -> float {
                            float al;
                            return evaluate_fill_h(genes, pop, tid, *s.box, mu, d.ls, d.lh, fp,
                                                   (float)d.fc.alpha_lo, (float)d.fc.alpha_hi,
                                                   s.obs, w2, inv_nu, al);
                        });
    } else if (d.synth == GENESIS_SYNTH_FP16) {
        generation_loop(s, pop, tid, pix, d.ga, d.generations, d.gen_to, nullptr, gs,
                        [&](const uint16_t *genes) -> float {
                            return evaluate_lds_h(genes, pop, tid, *s.box, mu, d.ls, d.lh, s.obs,
                                                  w2, inv_nu);
                        });
    } else if (d.fill) {
        generation_loop(s, pop, tid, pix, d.ga, d.generations, d.gen_to, nullptr, gs,
                        [&](const uint16_t *genes) -> float {
                            float al;
                            return evaluate_fill(genes, pop, tid, *s.box, mu, d.ls, fp,
                                                 (float)d.fc.alpha_lo, (float)d.fc.alpha_hi, s.obs,
                                                 w2, inv_nu, al);
                        });
    } else {
        generation_loop(s, pop, tid, pix, d.ga, d.generations, d.gen_to, nullptr, gs,
                        [&](const uint16_t *genes) -> float {
                            return evaluate_lds(genes, pop, tid, *s.box, mu, d.ls, s.obs, w2,
                                                inv_nu);
                        });
    }
    if (finish) {
        double par[GENESIS_NPAR];
        const int e = best_of(s, pop, gs, par);
        if (tid == 0) {
            for (int j = 0; j < GENESIS_NPAR; ++j)
                d.best_params[p * GENESIS_NPAR + j] = (float)par[j];
            d.best_chi2[p] = s.fit[e];
            if (d.fill) {
                // the best individual's alpha, as ga_invert finds it
                float al;
                if (d.synth == GENESIS_SYNTH_FP16) {
                    ModelH m;
                    model_setup(par, mu, m);
                    (void)chi2_fill_of_h(m, d.ls, d.lh, fp, (float)d.fc.alpha_lo,
                                         (float)d.fc.alpha_hi, s.obs, w2, inv_nu, al);
                } else {
                    Model<float> m;
                    model_setup(par, mu, m);
                    (void)chi2_fill_of(m, d.ls, fp, (float)d.fc.alpha_lo, (float)d.fc.alpha_hi,
                                       s.obs, w2, inv_nu, al);
                }
                d.best_alpha[p] = al;
            }
            if (d.status)
                d.status[p] = 0;
        }
    } else if (active) {
        const int64_t row = p * pop + tid;
        for (int j = 0; j < GENESIS_NPAR; ++j)
            d.genes[row * GENESIS_NPAR + j] = s.genes[gs.cur + j * pop + tid];
        d.fit[row] = gs.f;
    }
}

// What the session keeps per request beside the scheduler's bookkeeping.
struct Payload {
    ReqDesc desc{};
    hipEvent_t done_ev = nullptr;
};
using Req = SchedReq<Payload>;

struct Session {
    explicit Session(size_t budget, int gens) : sched(budget, gens) {}
    Scheduler<Payload> sched;
    int device = 0;
    // every launch of the session waits for the previous one, whatever stream
    // it came on, so memory freed stream-ordered after a launch is never
    // still in use by a kernel of an earlier step on another stream
    hipEvent_t last_ev = nullptr;
    bool last_valid = false;
    std::mutex mu;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t request_bytes(int64_t npix, int pop)
{
    return align256((size_t)npix * pop * GENESIS_NPAR * sizeof(uint16_t)) +
           align256((size_t)npix * pop * sizeof(float));
}

void free_population(Req &r, hipStream_t st)
{
    if (r.p.desc.genes)
        (void)hipFreeAsync(r.p.desc.genes, st);
    if (r.p.desc.fit)
        (void)hipFreeAsync(r.p.desc.fit, st);
    r.p.desc.genes = nullptr;
    r.p.desc.fit = nullptr;
}

}  // namespace

extern "C" {

int gs_create(size_t hbm_budget_bytes, int32_t gens_per_step, void **session)
{
    if (!session)
        return fail(ME_EINVAL, "session must not be NULL");
    if (gens_per_step < 1)
        return fail(ME_EINVAL, "gens_per_step must be >= 1");
    if (hbm_budget_bytes == 0)
        return fail(ME_EINVAL, "the memory budget must be positive");
    auto *s = new Session(hbm_budget_bytes, gens_per_step);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(ME_EHIP, "hipGetDevice failed");
    }
    if (hipEventCreateWithFlags(&s->last_ev, hipEventDisableTiming) != hipSuccess) {
        delete s;
        return fail(ME_EHIP, "hipEventCreate failed");
    }
    *session = s;
    return ME_OK;
}

}  // extern "C"

namespace {

int submit_impl(void *session, const float *obs, const float *sigma, const float *mu,
                int64_t npix, const me_line *lines, const me_grid *grids, int32_t nlines,
                const me_bounds *bounds, const ga_config *cfg, const me_fill *fill,
                float *best_params, float *best_alpha, float *best_chi2, int32_t *status,
                uint64_t *request_id)
{
    auto *s = static_cast<Session *>(session);
    if (!s || !request_id)
        return fail(ME_EINVAL, "session and request_id must not be NULL");
    auto r = std::make_shared<Req>();
    ReqDesc &d = r->p.desc;
    if (int rc = pack_lines(lines, grids, nlines, d.ls))
        return rc;
    if (int rc = pack_bounds(bounds, d.b))
        return rc;
    if (int rc = pack_ga(cfg, d.ga))
        return rc;
    d.synth = cfg->synth_precision;
    d.fill = fill ? 1 : 0;
    if (d.synth == GENESIS_SYNTH_FP16) {
        if (!(bounds->lo[5] >= 0.0 && bounds->hi[5] <= kHalfMaxDamping))
            return fail(ME_EINVAL, "FP16 synthesis needs damping bounds within [0, %g]",
                        kHalfMaxDamping);
        pack_lines_h(d.ls, d.lh);
    }
    if (fill) {
        if (int rc = pack_fill(fill, nlines, d.fc))
            return rc;
        if (!best_alpha)
            return fail(ME_EINVAL, "best_alpha must not be NULL");
    }
    if (npix < 1 || npix > kMaxGrid)
        return fail(ME_EINVAL, "npix must lie in [1, 2^30]");
    if (4 * d.ls.L <= GENESIS_NPAR + d.fill)
        return fail(ME_EINVAL, "need 4 L > %d wavelength samples for nu > 0",
                    GENESIS_NPAR + d.fill);
    if (ga_lds_bytes<float>(d.ls.L, cfg->pop) > kMaxLds)
        return fail(ME_ENOMEM, "L = %d, pop = %d exceed LDS", d.ls.L, cfg->pop);
    if (!obs || !sigma || !best_params || !best_chi2)
        return fail(ME_EINVAL, "NULL array argument");
    d.obs = obs;
    d.sigma = sigma;
    d.mu = mu;
    d.npix = npix;
    d.generations = cfg->generations;
    d.best_params = best_params;
    d.best_chi2 = best_chi2;
    d.best_alpha = fill ? best_alpha : nullptr;
    d.status = status;
    r->npix = npix;
    r->generations = cfg->generations;
    r->bytes = request_bytes(npix, cfg->pop);
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->bytes > s->sched.budget())
        return fail(ME_ENOMEM, "request needs %zu B, more than the whole budget %zu B", r->bytes,
                    s->sched.budget());
    if (hipEventCreateWithFlags(&r->p.done_ev, hipEventDisableTiming) != hipSuccess)
        return fail(ME_EHIP, "hipEventCreate failed");
    (void)s->sched.submit(r);
    *request_id = r->id;
    return ME_OK;
}

}  // namespace

extern "C" {

int gs_submit(void *session, const float *obs, const float *sigma, const float *mu, int64_t npix,
              const me_line *lines, const me_grid *grids, int32_t nlines,
              const me_bounds *bounds, const ga_config *cfg, float *best_params,
              float *best_chi2, int32_t *status, uint64_t *request_id)
{
    return submit_impl(session, obs, sigma, mu, npix, lines, grids, nlines, bounds, cfg, nullptr,
                       best_params, nullptr, best_chi2, status, request_id);
}

int gs_submit_fill(void *session, const float *obs, const float *sigma, const float *mu,
                   int64_t npix, const me_line *lines, const me_grid *grids, int32_t nlines,
                   const me_bounds *bounds, const ga_config *cfg, const me_fill *fill,
                   float *best_params, float *best_alpha, float *best_chi2, int32_t *status,
                   uint64_t *request_id)
{
    if (!fill)
        return fail(ME_EINVAL, "fill must not be NULL");
    return submit_impl(session, obs, sigma, mu, npix, lines, grids, nlines, bounds, cfg, fill,
                       best_params, best_alpha, best_chi2, status, request_id);
}

int gs_set_max_resident_pixels(void *session, int64_t max_pixels)
{
    auto *s = static_cast<Session *>(session);
    if (!s)
        return fail(ME_EINVAL, "session must not be NULL");
    if (max_pixels < 0)
        return fail(ME_EINVAL, "max_pixels must be >= 0");
    std::lock_guard<std::mutex> lk(s->mu);
    s->sched.set_max_pixels(max_pixels);
    return ME_OK;
}

int gs_step(void *session, void *stream)
{
    auto *s = static_cast<Session *>(session);
    if (!s)
        return fail(ME_EINVAL, "session must not be NULL");
    hipStream_t st = as_stream(stream);
    std::lock_guard<std::mutex> lk(s->mu);
    // order this step after the session's previous one (frees below are
    // stream-ordered on `st`)
    if (s->last_valid && hipStreamWaitEvent(st, s->last_ev, 0) != hipSuccess)
        return fail(ME_EHIP, "hipStreamWaitEvent failed");
    auto free_on_st = [st](Req &r) { free_population(r, st); };
    std::vector<Req *> res;
    const bool admitted_all = s->sched.plan(
        [st](Req &r) {
            ReqDesc &d = r.p.desc;
            const size_t gb = (size_t)d.npix * d.ga.pop * GENESIS_NPAR * sizeof(uint16_t);
            const size_t fb = (size_t)d.npix * d.ga.pop * sizeof(float);
            if (hipMallocAsync((void **)&d.genes, gb, st) != hipSuccess ||
                hipMallocAsync((void **)&d.fit, fb, st) != hipSuccess) {
                free_population(r, st);
                return false;
            }
            return true;
        },
        free_on_st, res);
    auto record_last = [&]() {
        if (hipEventRecord(s->last_ev, st) == hipSuccess)
            s->last_valid = true;
    };
    if (!admitted_all) {
        record_last();
        return fail(ME_ENOMEM, "device allocation for a queued request failed");
    }
    if (res.empty()) {
        record_last();
        return ME_OK;
    }
    // descriptors of this launch
    const int nreq = (int)res.size();
    std::vector<ReqDesc> descs(nreq);
    std::vector<int64_t> first(nreq + 1);
    int max_pop = 2;
    size_t lds = 0;
    first[0] = 0;
    for (int i = 0; i < nreq; ++i) {
        ReqDesc &d = res[i]->p.desc;
        d.gen_done = res[i]->gen_done;
        d.gen_to = res[i]->gen_to;
        descs[i] = d;
        first[i + 1] = first[i] + d.npix;
        max_pop = std::max(max_pop, d.ga.pop);
        lds = std::max(lds, ga_lds_bytes<float>(d.ls.L, d.ga.pop));
    }
    if (first[nreq] > kMaxGrid) {
        record_last();
        return fail(ME_EINVAL, "more than 2^30 resident pixels");
    }
    void *dbuf = nullptr;
    const size_t dbytes = align256(sizeof(ReqDesc) * nreq) + sizeof(int64_t) * (nreq + 1);
    if (hipMallocAsync(&dbuf, dbytes, st) != hipSuccess) {
        record_last();
        return fail(ME_ENOMEM, "descriptor allocation failed");
    }
    ReqDesc *d_descs = (ReqDesc *)dbuf;
    int64_t *d_first = (int64_t *)((char *)dbuf + align256(sizeof(ReqDesc) * nreq));
    if (hipMemcpyAsync(d_descs, descs.data(), sizeof(ReqDesc) * nreq, hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(d_first, first.data(), sizeof(int64_t) * (nreq + 1), hipMemcpyHostToDevice,
                       st) != hipSuccess) {
        (void)hipFreeAsync(dbuf, st);
        record_last();
        return fail(ME_EHIP, "descriptor upload failed");
    }
    hipLaunchKernelGGL(k_ga_advance, dim3((unsigned)first[nreq]), dim3(block_for_pop(max_pop)),
                       lds, st, d_descs, d_first, nreq);
    if (int rc = check_launch("gs_step")) {
        (void)hipFreeAsync(dbuf, st);
        record_last();
        return rc;
    }
    (void)hipFreeAsync(dbuf, st);
    // finished requests leave and return their memory
    s->sched.commit([st](Req &r) { (void)hipEventRecord(r.p.done_ev, st); }, free_on_st);
    record_last();
    return ME_OK;
}

int gs_poll(void *session, uint64_t request_id, int32_t *done)
{
    auto *s = static_cast<Session *>(session);
    if (!s || !done)
        return fail(ME_EINVAL, "session and done must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    Req *r = s->sched.find(request_id);
    if (!r)
        return fail(ME_EINVAL, "unknown request %llu", (unsigned long long)request_id);
    *done = 0;
    if (r->state == kDone)
        *done = hipEventQuery(r->p.done_ev) == hipSuccess ? 1 : 0;
    else if (r->state == kCancelled)
        *done = -1;
    return ME_OK;
}

int gs_cancel(void *session, uint64_t request_id)
{
    auto *s = static_cast<Session *>(session);
    if (!s)
        return fail(ME_EINVAL, "session must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->sched.cancel(request_id))
        return fail(ME_EINVAL, "unknown request %llu", (unsigned long long)request_id);
    return ME_OK;
}

int gs_release(void *session, uint64_t request_id)
{
    auto *s = static_cast<Session *>(session);
    if (!s)
        return fail(ME_EINVAL, "session must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    Req *r = s->sched.find(request_id);
    if (!r)
        return fail(ME_EINVAL, "unknown request %llu", (unsigned long long)request_id);
    if (r->state == kDone && hipEventQuery(r->p.done_ev) != hipSuccess)
        return fail(ME_EBUSY, "request %llu is still running on the device",
                    (unsigned long long)request_id);
    const bool ok = s->sched.release(request_id, [](Req &q) {
        if (q.p.done_ev)
            (void)hipEventDestroy(q.p.done_ev);
        q.p.done_ev = nullptr;
    });
    if (!ok)
        return fail(ME_EBUSY, "request %llu is queued or resident", (unsigned long long)request_id);
    return ME_OK;
}

int gs_stats(void *session, int64_t *queued, int64_t *resident, size_t *bytes_in_use)
{
    auto *s = static_cast<Session *>(session);
    if (!s)
        return fail(ME_EINVAL, "session must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued)
        *queued = (int64_t)s->sched.queued();
    if (resident)
        *resident = (int64_t)s->sched.resident();
    if (bytes_in_use)
        *bytes_in_use = s->sched.in_use();
    return ME_OK;
}

int gs_tracked(void *session, int64_t *n)
{
    auto *s = static_cast<Session *>(session);
    if (!s || !n)
        return fail(ME_EINVAL, "session and n must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *n = (int64_t)s->sched.tracked();
    return ME_OK;
}

int gs_destroy(void *session)
{
    auto *s = static_cast<Session *>(session);
    if (!s)
        return ME_OK;
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->sched.for_each_resident([](Req &r) { free_population(r, nullptr); });
        s->sched.for_each([](Req &r) {
            if (r.p.done_ev)
                (void)hipEventDestroy(r.p.done_ev);
            r.p.done_ev = nullptr;
        });
        if (s->last_ev)
            (void)hipEventDestroy(s->last_ev);
    }
    (void)hipDeviceSynchronize();
    delete s;
    return ME_OK;
}

}  // extern "C"
