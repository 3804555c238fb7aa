// C ABI of the DMK library (declarations and documentation in include/dmk.h).
// Every entry point converts internal failures into status codes; no C++
// exception crosses the boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "dmk_internal.h"

namespace dmk {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

void *dalloc(Plan *P, size_t bytes)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{DMK_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e)};
    }
    P->allocations.push_back(p);
    P->device_bytes += (int64_t)bytes;
    return p;
}

void plan_free_all(Plan *P)
{
    for (void *p : P->allocations) (void)hipFree(p);
    P->allocations.clear();
}

}  // namespace dmk

using namespace dmk;

namespace dmk {

// An eval reads and writes plan-owned workspace, so it must not overlap the
// previous eval on the same plan, whichever stream that one used: the new
// stream waits for the completion event of the last one, and the event is
// recorded again at the end.  Under stream capture the caller's graph orders
// the work itself, and events from outside the capture may not be waited on.
static bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    DMK_HIP(hipStreamIsCapturing(s, &st));
    return st != hipStreamCaptureStatusNone;
}

void begin_eval(Plan *P, hipStream_t s)
{
    if (P->ev_done && P->done_recorded && !capturing(s)) DMK_HIP(hipStreamWaitEvent(s, P->ev_done, 0));
}

void end_eval(Plan *P, hipStream_t s)
{
    if (P->ev_done && !capturing(s)) {
        DMK_HIP(hipEventRecord(P->ev_done, s));
        P->done_recorded = true;
    }
    P->last_stream = s;
}

void create_done_event(Plan *P) { DMK_HIP(hipEventCreateWithFlags(&P->ev_done, hipEventDisableTiming)); }
}  // namespace dmk

extern "C" {

const char *dmk_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// device buffers of one host call, freed when it returns
struct TempBufs {
    std::vector<void *> p;
    ~TempBufs()
    {
        for (void *x : p) (void)hipFree(x);
    }
    void *get(size_t bytes)
    {
        void *x = nullptr;
        DMK_HIP(hipMalloc(&x, std::max<size_t>(bytes, 1)));
        p.push_back(x);
        return x;
    }
};

// (p, n_f) pairs with compiled kernels, in increasing order
constexpr int kBuilt[][2] = {{9, 6}, {15, 10}, {18, 12}};

// c, n_f, p for tol: the parameter table's row (Table 1 plus 1e-5) when tol
// has one and nothing is overridden; otherwise c = opts->pswf_c or
// log(1/tol) (eq. pswfcvalue) and the search of Sec. 3.7 for n_f and p,
// rounded up to the smallest compiled pair.  A caller's p and/or n_f must
// name a compiled pair (the other member is taken from it).
Params choose_params(double tol, int dim, const dmk_opts &o)
{
    if (o.p < 0 || o.n_f < 0 || o.pswf_c < 0 || !std::isfinite(o.pswf_c))
        throw Error{DMK_ERR_ARG, "p, n_f and pswf_c must be >= 0"};
    if (o.pswf_c != 0 && (o.pswf_c < 2.0 || o.pswf_c > 40.0)) throw Error{DMK_ERR_ARG, "pswf_c must lie in [2, 40]"};
    Params prm;
    const bool row = params_for(tol, &prm, dim);
    auto built = [](int p, int nf) {
        for (const auto &b : kBuilt)
            if (b[0] == p && b[1] == nf) return true;
        return false;
    };
    if (row && !o.p && !o.n_f && !o.pswf_c) {
        if (!built(prm.p, prm.nf))
            throw Error{DMK_ERR_UNSUPPORTED, "tol " + std::to_string(tol) + " needs proxy order p = " +
                                                 std::to_string(prm.p) + ", not built (largest: 18, tol >= 1e-6)"};
        return prm;
    }
    const double c = o.pswf_c ? o.pswf_c : (row ? prm.c : std::log(1.0 / tol));
    int p = o.p, nf = o.n_f;
    if (!p || !nf) {
        if (p || nf) {  // one given: the compiled pair that has it
            for (const auto &b : kBuilt)
                if (b[0] == p || b[1] == nf) {
                    p = b[0];
                    nf = b[1];
                    break;
                }
        } else {
            Params sp;
            search_params(tol, c, &sp, nullptr, nullptr);
            for (const auto &b : kBuilt)
                if (b[0] >= sp.p && b[1] >= sp.nf) {
                    p = b[0];
                    nf = b[1];
                    break;
                }
            if (!p)
                throw Error{DMK_ERR_UNSUPPORTED, "tol " + std::to_string(tol) + " needs p = " + std::to_string(sp.p) +
                                                     ", n_f = " + std::to_string(sp.nf) +
                                                     "; kernels are built for p <= 18, n_f <= 12"};
        }
    }
    if (!built(p, nf))
        throw Error{DMK_ERR_UNSUPPORTED, "(p, n_f) = (" + std::to_string(p) + ", " + std::to_string(nf) +
                                             ") is not built; built pairs: (9, 6), (15, 10), (18, 12)"};
    prm.tol = tol;
    prm.c = c;
    prm.p = p;
    prm.nf = nf;
    prm.hw = 2.0 * M_PI / (3.0 + std::sqrt((double)dim));
    prm.nw = (int)std::ceil(c / prm.hw);
    return prm;
}

// Shared by dmk_plan and dmk_plan_batched: validates, builds tables, the
// forest of trees, lists and workspace.  poff: host offsets [nprob+1].
dmk_plan_t make_plan(int dim, dmk_kernel kernel, double tol, int32_t nprob, const int64_t *poff, const double *pts,
                     const dmk_opts *opts, void *stream, int64_t nsrc_st = -1)
{
    // nsrc_st >= 0: a plan of separate target sets; pts holds the union,
    // sources (the first nsrc_st points) then targets
    if (dim != 2 && dim != 3) throw Error{DMK_ERR_ARG, "dim must be 2 or 3"};
    if (kernel != DMK_LAPLACE && kernel != DMK_YUKAWA && kernel != DMK_POWER2) throw Error{DMK_ERR_ARG, "unknown kernel"};
    if (kernel == DMK_POWER2 && dim != 3) throw Error{DMK_ERR_UNSUPPORTED, "the 1/r^2 kernel is built for dim = 3"};
    if (!(tol > 0) || !std::isfinite(tol)) throw Error{DMK_ERR_ARG, "tol must be positive"};
    if (nprob < 1) throw Error{DMK_ERR_ARG, "nprob must be >= 1"};
    if (dim == 3 && nprob > 1 && kernel == DMK_YUKAWA)
        throw Error{DMK_ERR_UNSUPPORTED, "batches of 3-D Yukawa problems are not built (tables per problem)"};
    if (!poff) throw Error{DMK_ERR_ARG, "offsets is NULL"};
    if (poff[0] != 0) throw Error{DMK_ERR_ARG, "offsets[0] must be 0"};
    for (int32_t b = 0; b < nprob; ++b)
        if (poff[b + 1] < poff[b]) throw Error{DMK_ERR_ARG, "offsets must be non-decreasing"};
    const int64_t n = poff[nprob];
    if (n >= (int64_t(1) << 31)) throw Error{DMK_ERR_ARG, "n must satisfy 0 <= n < 2^31"};
    if (n > 0 && !pts) throw Error{DMK_ERR_ARG, "pts is NULL"};
    dmk_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (tol > 1e-2 || tol < 1e-12) throw Error{DMK_ERR_ARG, "tol must lie in [1e-12, 1e-2]"};
    const Params prm = choose_params(tol, dim, o);
    if (o.precision != DMK_FP64 && o.precision != DMK_MIXED) throw Error{DMK_ERR_ARG, "unknown precision"};
    if (o.precision == DMK_MIXED && tol < 1e-6 * (1 - 1e-9))
        throw Error{DMK_ERR_PRECISION, "mixed precision needs tol >= 1e-6"};
    // key layout: problem index above dim * kb Morton bits, 63 bits in all
    int pbits = 0;
    while ((int64_t(1) << pbits) < nprob) ++pbits;
    const int kbmax = (dim == 3) ? 21 : 31;
    const int kb = std::min(kbmax, (63 - pbits) / dim);
    const int dflt = (dim == 3) ? 20 : 30;
    if (o.leaf_max < 0 || o.max_depth < 0 || o.max_depth > kb) throw Error{DMK_ERR_ARG, "bad leaf_max/max_depth"};
    if (kernel == DMK_YUKAWA && !(o.lambda > 0 && std::isfinite(o.lambda)))
        throw Error{DMK_ERR_ARG, "the Yukawa kernel needs lambda > 0"};
    if ((o.flags & DMK_FLAG_LEVEL_LAUNCHES) && (o.flags & DMK_FLAG_QUEUE_LAUNCHES))
        throw Error{DMK_ERR_ARG, "DMK_FLAG_LEVEL_LAUNCHES and DMK_FLAG_QUEUE_LAUNCHES exclude each other"};
    auto *P = new Plan();
    try {
        P->dim = dim;
        P->kernel = kernel;
        P->lambda = o.lambda;
        P->nprob = nprob;
        P->poff.assign(poff, poff + nprob + 1);
        P->pbits = pbits;
        P->kb = kb;
        P->precision = o.precision;
        P->leaf_max = o.leaf_max ? o.leaf_max : 64;
        P->max_depth = o.max_depth ? o.max_depth : std::min(dflt, kb);
        P->flags = o.flags;
        P->queued = queue_schedule(dim, o.flags);
        P->n = n;
        build_tables(prm, &P->tab, dim, kernel == DMK_POWER2 ? 2 : 0);
        P->p = prm.p;
        P->nf = prm.nf;
        P->nw = prm.nw;
        hipStream_t s = (hipStream_t)stream;
        P->d_poff = (int64_t *)dalloc(P, (nprob + 1) * sizeof(int64_t));
        DMK_HIP(hipMemcpyAsync(P->d_poff, P->poff.data(), (nprob + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        upload_tables(P, s);
        build_tree(P, pts, s);
        if (nsrc_st >= 0) {
            P->st = true;
            P->nsrc = nsrc_st;
            split_roles(P, s);
        }
        build_lists(P, s);
        if (dim == 3) {  // unit change per problem: 1/(4 pi S_b) for the 1/r kernels, 1/S_b^2 for 1/r^2
            std::vector<double> sc(nprob);
            for (int b = 0; b < nprob; ++b)
                sc[b] = (kernel == DMK_POWER2) ? 1.0 / (P->pside[b] * P->pside[b]) : 1.0 / (4.0 * M_PI * P->pside[b]);
            P->d_pscale = (double *)dalloc(P, nprob * sizeof(double));
            DMK_HIP(hipMemcpy(P->d_pscale, sc.data(), nprob * sizeof(double), hipMemcpyHostToDevice));
        }
        if (kernel == DMK_YUKAWA && dim == 2) {
            if (P->nlevels > 32) throw Error{DMK_ERR_UNSUPPORTED, "Yukawa plans hold at most 32 levels"};
            for (int b = 0; b < nprob; ++b)
                if (o.lambda * P->pside[b] > 50.0)
                    throw Error{DMK_ERR_UNSUPPORTED, "lambda times a problem's extent must stay <= 50"};
            build_yukawa_tables(P, s);
        } else if (kernel == DMK_YUKAWA) {
            // lambda S: below 1e-3 the k -> 0 differences of the mollifier lose
            // digits (and the kernel is 1/r to that precision); above 1000 every
            // level's mollified kernel is zero and the direct sums carry all
            const double ls = o.lambda * P->pside[0];
            if (!(ls >= 1e-3 && ls <= 1000.0))
                throw Error{DMK_ERR_UNSUPPORTED, "lambda times the point set's extent must lie in [1e-3, 1000]"};
            if (P->nlevels > 32) throw Error{DMK_ERR_UNSUPPORTED, "Yukawa plans hold at most 32 levels"};
            build_yukawa3_tables(P, s);
        }
        alloc_workspace(P);
        count_work(P, s);
        create_done_event(P);
        if (P->flags & DMK_FLAG_BATCHED) {
            // default-priority streams only
            DMK_HIP(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
            DMK_HIP(hipStreamCreateWithFlags(&P->side_stream, hipStreamNonBlocking));
            DMK_HIP(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
            DMK_HIP(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming));
        }
    } catch (...) {
        plan_release(P);
        throw;
    }
    return reinterpret_cast<dmk_plan_t>(P);
}

}  // namespace

extern "C" {

dmk_status dmk_plan(int dim, dmk_kernel kernel, double tol, int64_t n, const double *pts, const dmk_opts *opts,
                    void *stream, dmk_plan_t *out)
{
    if (out) *out = nullptr;
    return guarded([&] {
        if (!out) throw Error{DMK_ERR_ARG, "out is NULL"};
        if (n < 0) throw Error{DMK_ERR_ARG, "n must satisfy 0 <= n < 2^31"};
        const int64_t off[2] = {0, n};
        *out = make_plan(dim, kernel, tol, 1, off, pts, opts, stream);
    });
}

dmk_status dmk_plan_targets(int dim, dmk_kernel kernel, double tol, int64_t nsrc, const double *src, int64_t ntgt,
                            const double *tgt, const dmk_opts *opts, void *stream, dmk_plan_t *out)
{
    if (out) *out = nullptr;
    return guarded([&] {
        if (!out) throw Error{DMK_ERR_ARG, "out is NULL"};
        if (dim != 3) throw Error{DMK_ERR_UNSUPPORTED, "separate target sets are built for dim = 3"};
        if (nsrc < 0 || ntgt < 0 || nsrc + ntgt >= (int64_t(1) << 31))
            throw Error{DMK_ERR_ARG, "need 0 <= nsrc, ntgt and nsrc + ntgt < 2^31"};
        if ((nsrc > 0 && !src) || (ntgt > 0 && !tgt)) throw Error{DMK_ERR_ARG, "src or tgt is NULL"};
        hipStream_t s = (hipStream_t)stream;
        const int64_t n = nsrc + ntgt;
        double *u = nullptr;  // the union on the device, sources first
        DMK_HIP(hipMalloc(&u, (size_t)std::max<int64_t>(n, 1) * 3 * sizeof(double)));
        try {
            if (nsrc) DMK_HIP(hipMemcpyAsync(u, src, (size_t)nsrc * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
            if (ntgt)
                DMK_HIP(hipMemcpyAsync(u + 3 * nsrc, tgt, (size_t)ntgt * 3 * sizeof(double), hipMemcpyDeviceToDevice,
                                       s));
            const int64_t off[2] = {0, n};
            *out = make_plan(dim, kernel, tol, 1, off, u, opts, stream, nsrc);
        } catch (...) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(u);
            throw;
        }
        DMK_HIP(hipStreamSynchronize(s));
        (void)hipFree(u);
    });
}

dmk_status dmk_plan_batched(int dim, dmk_kernel kernel, double tol, int32_t nprob, const int64_t *offsets,
                            const double *pts, const dmk_opts *opts, void *stream, dmk_plan_t *out)
{
    if (out) *out = nullptr;
    return guarded([&] {
        if (!out) throw Error{DMK_ERR_ARG, "out is NULL"};
        *out = make_plan(dim, kernel, tol, nprob, offsets, pts, opts, stream);
    });
}

dmk_status dmk_tune_leaf(int dim, dmk_kernel kernel, double tol, int32_t nprob, const int64_t *offsets,
                         const double *pts, const double *charges, const dmk_opts *opts, const int32_t *cand,
                         int32_t ncand, int32_t reps, void *stream, int32_t *best, double *ms)
{
    return guarded([&] {
        if (!cand || ncand < 1 || !best) throw Error{DMK_ERR_ARG, "candidates and best are required"};
        if (reps < 1) throw Error{DMK_ERR_ARG, "reps must be >= 1"};
        if (!offsets) throw Error{DMK_ERR_ARG, "offsets is NULL"};
        for (int32_t i = 0; i < ncand; ++i)
            if (cand[i] < 1) throw Error{DMK_ERR_ARG, "leaf capacities must be >= 1"};
        const int64_t n = offsets[nprob > 0 ? nprob : 0];
        if (n > 0 && !charges) throw Error{DMK_ERR_ARG, "charges is NULL"};
        dmk_opts o;
        std::memset(&o, 0, sizeof(o));
        if (opts) o = *opts;
        hipStream_t s = (hipStream_t)stream;
        double *pot = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        DMK_HIP(hipMalloc(&pot, (size_t)std::max<int64_t>(n, 1) * sizeof(double)));
        double bestms = 0.0;
        int32_t bi = -1;
        try {
            DMK_HIP(hipEventCreate(&e0));
            DMK_HIP(hipEventCreate(&e1));
            for (int32_t i = 0; i < ncand; ++i) {
                o.leaf_max = cand[i];
                dmk_plan_t h = make_plan(dim, kernel, tol, nprob, offsets, pts, &o, stream);
                Plan *P = reinterpret_cast<Plan *>(h);
                float t = 0.0f;
                try {
                    run_eval(P, charges, pot, nullptr, nullptr, s);  // warm-up (and graph capture)
                    DMK_HIP(hipEventRecord(e0, s));
                    for (int32_t r = 0; r < reps; ++r) run_eval(P, charges, pot, nullptr, nullptr, s);
                    DMK_HIP(hipEventRecord(e1, s));
                    DMK_HIP(hipEventSynchronize(e1));
                    DMK_HIP(hipEventElapsedTime(&t, e0, e1));
                } catch (...) {
                    (void)hipStreamSynchronize(s);
                    plan_release(P);
                    throw;
                }
                DMK_HIP(hipStreamSynchronize(s));
                plan_release(P);
                const double m = (double)t / reps;
                if (ms) ms[i] = m;
                if (bi < 0 || m < bestms) { bi = i; bestms = m; }
            }
        } catch (...) {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            (void)hipFree(pot);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipFree(pot);
        *best = cand[bi];
    });
}

dmk_status dmk_tune(int dim, dmk_kernel kernel, double tol, int32_t nprob, const int64_t *offsets, const double *pts,
                    const double *charges, const dmk_opts *opts, const int32_t *cand, int32_t ncand, int32_t reps,
                    void *stream, dmk_opts *best, double *ms, double *err)
{
    return guarded([&] {
        if (!cand || ncand < 1 || !best) throw Error{DMK_ERR_ARG, "candidates and best are required"};
        if (reps < 1) throw Error{DMK_ERR_ARG, "reps must be >= 1"};
        if (!offsets || nprob < 1) throw Error{DMK_ERR_ARG, "offsets and nprob >= 1 are required"};
        for (int32_t i = 0; i < ncand; ++i)
            if (cand[i] < 1) throw Error{DMK_ERR_ARG, "leaf capacities must be >= 1"};
        const int64_t n = offsets[nprob];
        if (n < 2 || !pts || !charges) throw Error{DMK_ERR_ARG, "at least two points, pts and charges are required"};
        dmk_opts o;
        std::memset(&o, 0, sizeof(o));
        if (opts) o = *opts;
        hipStream_t s = (hipStream_t)stream;
        // the pairs to try: the caller's, or every compiled pair from the coarsest
        const Params rule = choose_params(tol, dim, o);
        std::vector<std::pair<int, int>> pairs;
        if (o.p || o.n_f) pairs.push_back({rule.p, rule.nf});
        else
            for (const auto &b : kBuilt) pairs.push_back({b[0], b[1]});
        // accuracy gate: direct sums at evenly spaced sample targets
        const int ns = (int)std::min<int64_t>(256, n);
        std::vector<int64_t> tidx(ns);
        for (int k = 0; k < ns; ++k) tidx[k] = (int64_t)((k + 0.5) * (double)n / ns);
        TempBufs B;
        int64_t *d_tidx = (int64_t *)B.get(ns * sizeof(int64_t)), *d_off = (int64_t *)B.get((nprob + 1) * sizeof(int64_t));
        double *d_dir = (double *)B.get(ns * sizeof(double)), *pot = (double *)B.get(n * sizeof(double));
        DMK_HIP(hipMemcpyAsync(d_tidx, tidx.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice, s));
        DMK_HIP(hipMemcpyAsync(d_off, offsets, (nprob + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        direct_sample(dim, kernel, o.lambda, pts, charges, d_off, nprob, d_tidx, ns, d_dir, s);
        std::vector<double> dir(ns), hp(n);
        DMK_HIP(hipMemcpyAsync(dir.data(), d_dir, ns * sizeof(double), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipStreamSynchronize(s));
        double dnorm = 0.0;
        for (double v : dir) dnorm += v * v;
        dnorm = std::sqrt(std::max(dnorm, 1e-300));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        DMK_HIP(hipEventCreate(&e0));
        struct Ev {
            hipEvent_t &a, &b;
            ~Ev() { if (a) (void)hipEventDestroy(a); if (b) (void)hipEventDestroy(b); }
        } ev{e0, e1};
        DMK_HIP(hipEventCreate(&e1));
        // one plan: returns the sampled error, and the mean eval time if timed
        auto trial = [&](int leaf, int p, int nf, bool timed, double *t_ms) {
            dmk_opts q = o;
            q.leaf_max = leaf;
            q.p = p;
            q.n_f = nf;
            q.pswf_c = rule.c;
            dmk_plan_t h = make_plan(dim, kernel, tol, nprob, offsets, pts, &q, stream);
            Plan *P = reinterpret_cast<Plan *>(h);
            double e = 0.0;
            try {
                run_eval(P, charges, pot, nullptr, nullptr, s);  // warm-up (and graph capture)
                if (timed) {
                    float t = 0.0f;
                    DMK_HIP(hipEventRecord(e0, s));
                    for (int32_t r = 0; r < reps; ++r) run_eval(P, charges, pot, nullptr, nullptr, s);
                    DMK_HIP(hipEventRecord(e1, s));
                    DMK_HIP(hipEventSynchronize(e1));
                    DMK_HIP(hipEventElapsedTime(&t, e0, e1));
                    *t_ms = (double)t / reps;
                }
                DMK_HIP(hipMemcpyAsync(hp.data(), pot, n * sizeof(double), hipMemcpyDeviceToHost, s));
                DMK_HIP(hipStreamSynchronize(s));
            } catch (...) {
                (void)hipStreamSynchronize(s);
                plan_release(P);
                throw;
            }
            plan_release(P);
            for (int k = 0; k < ns; ++k) e += (hp[tidx[k]] - dir[k]) * (hp[tidx[k]] - dir[k]);
            return std::sqrt(e) / dnorm;
        };
        // the coarsest pair that meets tol, then the fastest leaf capacity;
        // if the winner misses tol (errors vary a little with n_s), the next pair
        size_t pi = 0;
        for (; pi + 1 < pairs.size(); ++pi)
            if (trial(cand[0], pairs[pi].first, pairs[pi].second, false, nullptr) <= tol) break;
        int bi = 0;
        double e_best = 0.0;
        for (;;) {
            double bt = 0.0;
            bi = -1;
            for (int32_t i = 0; i < ncand; ++i) {
                double t = 0.0;
                const double e = trial(cand[i], pairs[pi].first, pairs[pi].second, true, &t);
                if (ms) ms[i] = t;
                if (bi < 0 || t < bt) { bi = i; bt = t; e_best = e; }
            }
            if (e_best <= tol || pi + 1 >= pairs.size()) break;
            ++pi;
        }
        *best = o;
        best->leaf_max = cand[bi];
        best->p = pairs[pi].first;
        best->n_f = pairs[pi].second;
        best->pswf_c = rule.c;
        if (err) *err = e_best;
    });
}

dmk_status dmk_problem_info(dmk_plan_t plan, int32_t prob, double *center, double *side)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (prob < 0 || prob >= P->nprob) throw Error{DMK_ERR_ARG, "problem index out of range"};
        if (center)
            for (int d = 0; d < P->dim; ++d) center[d] = P->pcenter[(size_t)P->dim * prob + d];
        if (side) *side = P->pside[prob];
    });
}

dmk_status dmk_eval_parts(dmk_plan_t plan, const double *charges, double *far_part, double *near_part, void *stream)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (P->is_vol) throw Error{DMK_ERR_ARG, "a volume plan is evaluated with dmk_vol_eval"};
        if (P->nsrc > 0 && !charges) throw Error{DMK_ERR_ARG, "charges is NULL"};
        BusyGuard g(P);
        hipStream_t s = (hipStream_t)stream;
        begin_eval(P, s);
        run_eval(P, charges, nullptr, far_part, near_part, s);
        end_eval(P, s);
    });
}

dmk_status dmk_eval(dmk_plan_t plan, const double *charges, double *pot, void *stream)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (P->is_vol) throw Error{DMK_ERR_ARG, "a volume plan is evaluated with dmk_vol_eval"};
        if ((P->nsrc > 0 && !charges) || (P->ntgt > 0 && !pot)) throw Error{DMK_ERR_ARG, "charges or pot is NULL"};
        BusyGuard g(P);
        hipStream_t s = (hipStream_t)stream;
        begin_eval(P, s);
        run_eval(P, charges, pot, nullptr, nullptr, s);
        end_eval(P, s);
    });
}

dmk_status dmk_vol_plan(double tol, int32_t q, double rho_scale, int32_t min_level, int32_t max_level,
                        int32_t nfeat, const double *feat, dmk_density_fn density, void *ctx, const dmk_opts *opts,
                        void *stream, dmk_plan_t *out)
{
    return guarded([&] {
        if (!out) throw Error{DMK_ERR_ARG, "out is NULL"};
        *out = nullptr;
        *out = make_vol_plan(tol, q, rho_scale, min_level, max_level, nfeat, feat, density, ctx, opts, stream);
    });
}

dmk_status dmk_vol_info(dmk_plan_t plan, int64_t *nleaf, int64_t *npoints)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (!P->is_vol) throw Error{DMK_ERR_ARG, "not a volume plan"};
        if (nleaf) *nleaf = P->vol.nleaf;
        if (npoints) *npoints = P->n;
    });
}

dmk_status dmk_vol_leaves(dmk_plan_t plan, int32_t *level, int32_t *ijk)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (!P->is_vol) throw Error{DMK_ERR_ARG, "not a volume plan"};
        if (level) std::memcpy(level, P->vol.level.data(), P->vol.level.size() * sizeof(int32_t));
        if (ijk) std::memcpy(ijk, P->vol.ijk.data(), P->vol.ijk.size() * sizeof(int32_t));
    });
}

dmk_status dmk_vol_nodes(dmk_plan_t plan, double *xyz, void *stream)
{
    return guarded([&] {
        if (!plan || !xyz) throw Error{DMK_ERR_ARG, "NULL argument"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (!P->is_vol) throw Error{DMK_ERR_ARG, "not a volume plan"};
        vol_nodes(P, xyz, (hipStream_t)stream);
    });
}

dmk_status dmk_vol_eval(dmk_plan_t plan, const double *rho, double *u, double *far_part, double *near_part,
                        void *stream)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (!P->is_vol) throw Error{DMK_ERR_ARG, "not a volume plan (use dmk_eval)"};
        if (!rho) throw Error{DMK_ERR_ARG, "rho is NULL"};
        if (!u && !far_part && !near_part) throw Error{DMK_ERR_ARG, "no output requested"};
        BusyGuard g(P);
        hipStream_t s = (hipStream_t)stream;
        begin_eval(P, s);
        run_vol_eval(P, rho, u, far_part, near_part, s);
        end_eval(P, s);
    });
}

dmk_status dmk_plan_info(dmk_plan_t plan, dmk_plan_stats *st)
{
    return guarded([&] {
        if (!plan || !st) throw Error{DMK_ERR_ARG, "NULL argument"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        std::memset(st, 0, sizeof(*st));
        st->n = P->n;
        st->nbox = P->nbox;
        st->nlevels = P->nlevels;
        st->p = P->p;
        st->nf = P->nf;
        st->nw = P->nw;
        st->c = P->tab.prm.c;
        st->tol = P->tab.prm.tol;
        st->leaf_max = P->leaf_max;
        st->precision = P->precision;
        st->nleaf = P->nleaf;
        st->nfout = P->nfout;
        st->nfin = P->nfin;
        st->npairs = P->npairs;
        st->device_bytes = P->device_bytes;
        for (int d = 0; d < P->dim; ++d) st->center[d] = P->center[d];
        st->side = P->side;
        st->dim = P->dim;
        st->nprob = P->nprob;
        st->nsrc = P->nsrc;
        st->ntgt = P->ntgt;
        if (P->q_fail) DMK_HIP(hipMemcpy(&st->queue_timeouts, P->q_fail, sizeof(int32_t), hipMemcpyDeviceToHost));
    });
}

dmk_status dmk_export_tree(dmk_plan_t plan, int64_t *perm, int32_t *level, uint64_t *bkey, int64_t *parent,
                           int64_t *child0, int64_t *pstart, int64_t *pcount, uint8_t *flags, int64_t *colleague,
                           int32_t *ncoarse, int64_t *coarse)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        const int64_t n = P->n, nb = P->nbox;
        auto cp32to64 = [&](const int32_t *src, int64_t cnt, int64_t *dst) {
            if (!dst || cnt == 0) return;
            std::vector<int32_t> h(cnt);
            DMK_HIP(hipMemcpy(h.data(), src, cnt * sizeof(int32_t), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < cnt; ++i) dst[i] = h[i];
        };
        cp32to64(P->perm, n, perm);
        if (level) DMK_HIP(hipMemcpy(level, P->blevel, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (bkey) DMK_HIP(hipMemcpy(bkey, P->bkey, nb * sizeof(uint64_t), hipMemcpyDeviceToHost));
        cp32to64(P->parent, nb, parent);
        cp32to64(P->child0, nb, child0);
        cp32to64(P->pstart, nb, pstart);
        cp32to64(P->pcount, nb, pcount);
        if (flags) DMK_HIP(hipMemcpy(flags, P->bflags, nb, hipMemcpyDeviceToHost));
        const int64_t ncol = (P->dim == 3) ? 27 : 9, nco = (1 << P->dim) - 1;
        cp32to64(P->colleague, ncol * nb, colleague);
        if (ncoarse) DMK_HIP(hipMemcpy(ncoarse, P->ncoarse, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
        cp32to64(P->coarse, nco * nb, coarse);
    });
}

dmk_status dmk_export_near_lists(dmk_plan_t plan, int64_t *leaf_box, int64_t *offsets, int64_t *src_box)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        auto cp = [&](const int32_t *src, int64_t cnt, int64_t *dst) {
            if (!dst || cnt == 0) return;
            std::vector<int32_t> h(cnt);
            DMK_HIP(hipMemcpy(h.data(), src, cnt * sizeof(int32_t), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < cnt; ++i) dst[i] = h[i];
        };
        cp(P->l_leaf, P->nleaf, leaf_box);
        if (offsets) {
            if (P->nleaf == 0) offsets[0] = 0;
            else cp(P->nl_off, P->nleaf + 1, offsets);
        }
        cp(P->nl_src, P->nl_total, src_box);
    });
}

dmk_status dmk_copy_box_data(dmk_plan_t plan, int what, int64_t box, double *out)
{
    return guarded([&] {
        if (!plan || !out) throw Error{DMK_ERR_ARG, "NULL argument"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (box < 0 || box >= P->nbox) throw Error{DMK_ERR_ARG, "box out of range"};
        if (!P->has_workspace) throw Error{DMK_ERR_STATE, "the plan holds no eval workspace (DMK_FLAG_NO_WORKSPACE)"};
        const int64_t p3 = (P->dim == 3) ? (int64_t)P->p * P->p * P->p : (int64_t)P->p * P->p;
        int32_t slot = -1;
        const double *base = nullptr;
        const void *vbase = nullptr;
        if (what == 0) {
            DMK_HIP(hipMemcpy(&slot, P->proxy_slot + box, sizeof(int32_t), hipMemcpyDeviceToHost));
            vbase = P->proxy;
        } else if (what == 1) {
            DMK_HIP(hipMemcpy(&slot, P->local_slot + box, sizeof(int32_t), hipMemcpyDeviceToHost));
            vbase = P->local;
        } else {
            throw Error{DMK_ERR_ARG, "what must be 0 or 1"};
        }
        (void)base;
        if (slot < 0) throw Error{DMK_ERR_ARG, "box holds no such data"};
        if (P->last_stream) DMK_HIP(hipStreamSynchronize(P->last_stream));
        DMK_HIP(hipDeviceSynchronize());
        if (P->precision == DMK_FP64) {
            DMK_HIP(hipMemcpy(out, (const double *)vbase + (int64_t)slot * p3, p3 * sizeof(double),
                              hipMemcpyDeviceToHost));
        } else {
            std::vector<float> h(p3);
            DMK_HIP(hipMemcpy(h.data(), (const float *)vbase + (int64_t)slot * p3, p3 * sizeof(float),
                              hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < p3; ++i) out[i] = h[i];
        }
    });
}

dmk_status dmk_precompute_probe(double tol, int what, int64_t n, const double *x, double *out)
{
    return guarded([&] {
        if (n < 0 || (n > 0 && !out)) throw Error{DMK_ERR_ARG, "bad n or out"};
        if (what == 10) {  // parameter search: x[0] = c (0: log(1/tol)); out = c, n_f, p, errors
            if (n < 5) throw Error{DMK_ERR_ARG, "n >= 5 needed"};
            if (!(tol > 0 && tol < 1)) throw Error{DMK_ERR_ARG, "tol must lie in (0, 1)"};
            const double c = (x && x[0] > 0) ? x[0] : std::log(1.0 / tol);
            Params prm;
            double e_nf = 0.0, e_p = 0.0;
            search_params(tol, c, &prm, &e_nf, &e_p);
            out[0] = prm.c; out[1] = prm.nf; out[2] = prm.p; out[3] = e_nf; out[4] = e_p;
            return;
        }
        // what 12, 13, 14: the 1/r^2 tables, as what 1, 2, 3 for 1/r
        const int kind = (what >= 12 && what <= 14) ? 2 : 0;
        if (kind == 2) what -= 11;
        const int dim = (what >= 6) ? 2 : 3;
        Params prm;
        if (!params_for(tol, &prm, dim)) throw Error{DMK_ERR_UNSUPPORTED, "tolerance not in the table"};
        Tables t;
        build_tables(prm, &t, dim, kind);
        if (what == 9) {
            if (n < 4) throw Error{DMK_ERR_ARG, "n >= 4 needed"};
            out[0] = t.m0; out[1] = prm.nw; out[2] = prm.hw; out[3] = t.gdeg;
            return;
        }
        if (what == 4) {
            if (n < 4) throw Error{DMK_ERR_ARG, "n >= 4 needed"};
            out[0] = t.psi0; out[1] = t.c0; out[2] = t.c2; out[3] = t.lambda0;
            return;
        }
        if (what == 5) {
            if (n < 6) throw Error{DMK_ERR_ARG, "n >= 6 needed"};
            out[0] = prm.c; out[1] = prm.nf; out[2] = prm.p; out[3] = prm.nw; out[4] = prm.hw; out[5] = t.gdeg;
            return;
        }
        if (n > 0 && !x) throw Error{DMK_ERR_ARG, "x is NULL"};
        for (int64_t i = 0; i < n; ++i) {
            double v = NAN;
            if (what == 0) {
                v = pswf_eval(t, x[i]) / t.psi0;
            } else if (what == 1) {
                double u = 2.0 * x[i] - 1.0, b1 = 0.0, b2 = 0.0;
                for (int k = t.gdeg; k >= 1; --k) {
                    double b0 = t.gcheb[k] + 2.0 * u * b1 - b2;
                    b2 = b1;
                    b1 = b0;
                }
                v = t.gcheb[0] + u * b1 - b2;
            } else if (what == 2 || what == 3) {
                const int nf = (what == 2) ? t.nf : t.nw, nn = 2 * nf + 1;
                const std::vector<double> &w = (what == 2) ? t.wd0 : t.ww;
                long k2 = lround(x[i]);
                for (int m3 = 0; m3 <= nf && std::isnan(v); ++m3)
                    for (int m2 = -nf; m2 <= nf && std::isnan(v); ++m2)
                        for (int m1 = -nf; m1 <= nf; ++m1)
                            if ((long)(m1 * m1 + m2 * m2 + m3 * m3) == k2) {
                                v = (what == 2) ? w[((size_t)(m1 + nf) * (nf + 1) + m3) * nn + (m2 + nf)]
                                                : w[((size_t)m3 * nn + (m2 + nf)) * nn + (m1 + nf)];
                                break;
                            }
            } else if (what == 6 || what == 7) {
                const int nf = (what == 6) ? t.nf : t.nw, nh = nf + 1;
                const std::vector<double> &w = (what == 6) ? t.wd0 : t.ww;
                long k2 = lround(x[i]);
                for (int m2 = 0; m2 <= nf && std::isnan(v); ++m2)
                    for (int m1 = -nf; m1 <= nf; ++m1)
                        if ((long)(m1 * m1 + m2 * m2) == k2) {
                            v = w[(size_t)(m1 + nf) * nh + m2];
                            break;
                        }
            } else if (what == 8) {
                double u = 2.0 * x[i] * x[i] - 1.0, b1 = 0.0, b2 = 0.0;
                for (int k = t.gdeg; k >= 1; --k) {
                    double b0 = t.gcheb[k] + 2.0 * u * b1 - b2;
                    b2 = b1;
                    b1 = b0;
                }
                v = t.gcheb[0] + u * b1 - b2;
            } else {
                throw Error{DMK_ERR_ARG, "what must be 0..10 or 12..14"};
            }
            out[i] = v;
        }
    });
}

dmk_status dmk_stage_timing(dmk_plan_t plan, int enable)
{
    return guarded([&] {
        if (!plan) throw Error{DMK_ERR_ARG, "plan is NULL"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (P->last_stream) DMK_HIP(hipStreamSynchronize(P->last_stream));
        for (auto &r : P->pending) {
            P->event_pool.push_back(r.a);
            P->event_pool.push_back(r.b);
        }
        P->pending.clear();
        for (int i = 0; i < DMK_NSTAGES; ++i) {
            P->stage_ms[i] = 0.0;
            P->stage_launches[i] = 0;
        }
        P->timing = enable != 0;
    });
}

dmk_status dmk_stage_times(dmk_plan_t plan, double *ms, int64_t *launches, int nstages)
{
    return guarded([&] {
        if (!plan || nstages < 0) throw Error{DMK_ERR_ARG, "bad argument"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        if (P->last_stream) DMK_HIP(hipStreamSynchronize(P->last_stream));
        for (auto &r : P->pending) {
            float t = 0.0f;
            DMK_HIP(hipEventSynchronize(r.b));
            DMK_HIP(hipEventElapsedTime(&t, r.a, r.b));
            P->stage_ms[r.stage] += t;
            P->stage_launches[r.stage] += 1;
            P->event_pool.push_back(r.a);
            P->event_pool.push_back(r.b);
        }
        P->pending.clear();
        for (int i = 0; i < nstages && i < DMK_NSTAGES; ++i) {
            if (ms) ms[i] = P->stage_ms[i];
            if (launches) launches[i] = P->stage_launches[i];
        }
    });
}

dmk_status dmk_stage_work(dmk_plan_t plan, double *flops, double *bytes, int nstages)
{
    return guarded([&] {
        if (!plan || nstages < 0) throw Error{DMK_ERR_ARG, "bad argument"};
        Plan *P = reinterpret_cast<Plan *>(plan);
        double F[DMK_NSTAGES], B[DMK_NSTAGES];
        stage_work(P, F, B);
        for (int i = 0; i < nstages && i < DMK_NSTAGES; ++i) {
            if (flops) flops[i] = F[i];
            if (bytes) bytes[i] = B[i];
        }
    });
}

void dmk_plan_destroy(dmk_plan_t plan)
{
    if (!plan) return;
    Plan *P = reinterpret_cast<Plan *>(plan);
    if (P->last_stream) (void)hipStreamSynchronize(P->last_stream);
    (void)hipDeviceSynchronize();
    plan_release(P);
}

}  // extern "C"

namespace dmk {
// frees everything a plan holds (device memory, events, streams, graph)
void plan_release(Plan *P)
{
    for (auto &r : P->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : P->event_pool) (void)hipEventDestroy(e);
    if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    if (P->ev_done) (void)hipEventDestroy(P->ev_done);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    if (P->side_stream) (void)hipStreamDestroy(P->side_stream);
    plan_free_all(P);
    delete P;
}

}  // namespace dmk
