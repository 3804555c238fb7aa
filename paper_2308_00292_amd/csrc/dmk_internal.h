// Internal declarations of the gfx950 DMK library: plan layout, precomputed
// tables and error plumbing.  Not part of the C ABI (include/dmk.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <exception>
#include <new>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmk.h"

namespace dmk {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);

struct Error {
    dmk_status code;
    std::string msg;
};

#define DMK_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::dmk::Error{DMK_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// ------------------------------------------------------------- parameters
struct Params {
    double tol;
    double c;    // PSWF parameter
    int nf;      // plane-wave half width of D_l
    int p;       // Chebyshev order
    int nw;      // plane-wave half width of W_0
    double hw;   // plane-wave spacing of W_0 (root side 1)
};
bool params_for(double tol, Params *out, int dim = 3);
// Sec. 3.7 for tolerances off the table: the smallest n_f and p meeting tol
// for PSWF parameter c (errors of the chosen values returned if non-NULL).
void search_params(double tol, double c, Params *out, double *err_nf, double *err_p);

// Host-side tables, all FP64 (Step 1 of the algorithm).  In 2-D the
// plane-wave arrays are [m1][m2] with m2 >= 0, the weights are those of the
// log kernel's split (level-independent), and gcheb holds the smooth part m
// of its residual as a series in 2 (r/s_l)^2 - 1.
struct Tables {
    Params prm;
    int dim = 3;
    double m0 = 0.0;                       // 2-D: m(0), the r -> 0 value of the smooth part
    int p, nf, nn, nh, nw, nwn, nwh;
    double psi0, c0, c2, lambda0;
    std::vector<double> coef;              // PSWF Legendre coefficients (even k)
    std::vector<double> xcheb;             // p first-kind Chebyshev nodes
    std::vector<double> bary;              // barycentric weights of the nodes
    std::vector<double> c2p;               // [2][p][p] A_s[a][i] = l_a((x_i + s)/2)
    std::vector<double> epw;               // [nn][p][2] exp(-i pi m x_j / 3)
    std::vector<double> ew;                // [nwn][p][2] exp(-i hw m x_j / 2)
    std::vector<double> wd0;               // 3-D [nn][nh][nn] D_0 weights, half spectrum, [m1][m3][m2]; 2-D [nn][nh]
    std::vector<double> ww;                // 3-D [nwh][nwn][nwn] W_0 weights, [m3][m2][m1]; 2-D [nwn][nwh]
    std::vector<double> gcheb;             // Chebyshev coefficients of Phi(sqrt t)/sqrt t on [0,1]
    int gdeg;                              // degree kept for FP64 evaluation
    int gdeg32;                            // degree kept for FP32 evaluation
    int kind = 0;                          // 0: 1/r split (or 2-D); 2: 1/r^2 (gcheb: Phi2(sqrt t)/t; weights scale 4^l)
};
// kind: 0 for the 1/r-type splits (and every 2-D table), 2 for 1/r^2 in 3-D
void build_tables(const Params &prm, Tables *t, int dim = 3, int kind = 0);

// PSWF helpers exposed for the host-side self checks in the tests.
double pswf_eval(const Tables &t, double x);  // any real x
double pswf_phi(const Tables &t, double x);  // Phi(x) = (1/c_0) int_0^x psi, 1 beyond x = 1

// ------------------------------------------------------------------- plan
struct LevelLists {
    // offsets into the concatenated device lists, per level [nlevels+1]
    std::vector<int64_t> fout_off, fin_off, anc_off, leaf_off;
};

// Volume potential (continuous sources on a density-adaptive tree of q^3
// Chebyshev leaf grids; vol.hip).  The point machinery holds the box tree:
// its points are the leaf nodes, leaf capacity q^3, root fixed to the unit
// cube, so its leaves are exactly the volume leaves.
struct VolData {
    int q = 0;
    int64_t nleaf = 0;
    std::vector<int32_t> level, ijk;     // host leaf list, Morton order
    double tau_a = 0, sqL = 0, tpan_w = 1.0;  // sqL: lower end of the t-quadrature, x s_T
    int tpan_gl = 5;
    int split = 0;                       // 0: Gaussian split; 1: PSWF split (tol 1e-6)
    int nfit = 0;                        // PSWF split: fitted Gaussians of the residual
    std::vector<double> fit;             // [2][nfit]: t s_T, then w s_T
    double fit_err = 0;                  // max |fit error| on its sample grid, x 1/s_T
    double *d_fit = nullptr;
    int32_t *d_level = nullptr, *d_ijk = nullptr;
    int32_t *box2v = nullptr;            // [nbox] volume leaf of a leaf box, -1 otherwise
    int32_t *d_esrc = nullptr;           // [gather entries] volume leaf of each entry's source
    double *d_v1 = nullptr;              // [2][p][q] density -> parent proxy matrices
    float *f_v1 = nullptr;
    double *d_xq = nullptr, *d_bq = nullptr;     // leaf nodes and barycentric weights
    double *d_d2 = nullptr;              // [q][q] second derivative on the leaf nodes
    double *d_tgl = nullptr, *d_tglw = nullptr;  // Gauss-Legendre rule per log-t panel
    double *d_egl = nullptr, *d_eglw = nullptr;  // Gauss-Legendre rule of the 1-D Gaussian integrals
    double *ufar = nullptr, *unear = nullptr;    // [nleaf q^3], leaf-major
    // near-field tables: one q x q matrix per (per-axis offset class, Gaussian)
    // for a unit source box; d_pkey[e][4] holds, for gather-list entry e,
    // the first table row (Gaussian) of each axis' class (-1: pair pruned),
    // then flags: bit 0 ends a (y, z) group, bit 1 a z group, and the
    // entry's Gaussian count sits above bit 1
    int32_t *d_pkey = nullptr;
    int32_t *d_kng = nullptr;            // [nkey] Gaussians of the class
    int64_t *d_kbase = nullptr;          // [nkey] first Gaussian of the class
    double *d_gtab = nullptr;            // [ngauss][q][q]
    float *f_gtab = nullptr;             // FP32 copy for mixed-precision plans
    double *d_gw = nullptr;              // [ngauss] quadrature weight of the Gaussian
    int64_t nkey = 0, ngauss_tab = 0;
    // work counts gathered at plan time
    int64_t n_merge = 0;        // non-leaf children merged by the child->parent matrices
    int64_t n_pairs = 0;        // (source leaf, target leaf) pairs of the near field
    int64_t n_gauss = 0;        // Gaussians summed over those pairs
    int64_t n_gauss_passes = 0; // near-field mode-product passes times their Gaussians
};

struct Plan {
    // configuration
    bool is_vol = false;
    bool fixed_root = false;  // root = the unit cube centred at the origin
    VolData vol;
    int dim = 3, p = 0, nf = 0, nw = 0, precision = 0, leaf_max = 64, max_depth = 20;
    int kernel = DMK_LAPLACE;
    double lambda = 0.0;       // Yukawa parameter, input units
    uint64_t flags = 0;
    Tables tab;
    int64_t n = 0;
    double center[3] = {0, 0, 0}, side = 1.0;  // root cube of problem 0

    // independent problems (a forest: one tree per problem, boxes of all
    // problems interleaved level by level); a single point set is nprob = 1
    int32_t nprob = 1;
    int kb = 21, pbits = 0;               // key bits per axis, problem-id bits
    std::vector<int64_t> poff;            // host [nprob+1] point offsets
    std::vector<double> pcenter, pside;   // host [nprob][dim], [nprob]
    int64_t *d_poff = nullptr;            // device copies
    double *d_pcenter = nullptr, *d_pside = nullptr;
    double *d_pscale = nullptr;           // [nprob] 3-D unit change of each problem's potentials
    int32_t *bprob = nullptr;             // [nbox] problem of each box

    // sorted points
    double *X = nullptr, *Y = nullptr, *Z = nullptr;
    int32_t *perm = nullptr;
    uint64_t *keys = nullptr;

    // sources and targets.  A plan of separate target sets (st) builds its
    // tree on the union of nsrc sources (union input indices 0..nsrc-1) and
    // ntgt targets (nsrc..n-1), then keeps each set apart in tree order with
    // per-box ranges; otherwise both views alias the union arrays.
    bool st = false;
    int64_t nsrc = 0, ntgt = 0;
    double *Xs = nullptr, *Ys = nullptr, *Zs = nullptr;  // sources, tree order
    int32_t *sperm = nullptr, *sstart = nullptr, *scount = nullptr;
    double *Xt = nullptr, *Yt = nullptr, *Zt = nullptr;  // targets, tree order
    int32_t *tperm = nullptr, *tstart = nullptr, *tcount = nullptr;

    // boxes (level-major, Morton order within a level)
    int nlevels = 0;
    std::vector<int64_t> level_start;  // host [nlevels+1]
    int64_t nbox = 0;
    uint64_t *bkey = nullptr;
    int32_t *blevel = nullptr, *parent = nullptr, *child0 = nullptr;
    int32_t *pstart = nullptr, *pcount = nullptr;
    uint8_t *bflags = nullptr;  // bit0 leaf, bit1 fout, bit2 fin, bit3 terminal
    int32_t *colleague = nullptr;  // [nbox][3^dim]
    int32_t *anchor = nullptr;     // [nbox] nearest ancestor-or-self holding local values
    uint8_t *anc_read = nullptr;   // [nanc] 1 where a finer anchor reads the anchor's local values
    int32_t *ncoarse = nullptr, *coarse = nullptr;  // [nbox], [nbox][2^dim - 1]
    double *bcenter = nullptr;     // [nbox][dim]

    // work lists (device, concatenated by level) and slot maps
    LevelLists ll;
    int32_t *l_fout = nullptr, *l_fin = nullptr, *l_anc = nullptr, *l_leaf = nullptr;
    int32_t *anc_tbeg = nullptr;   // [nanc+1] offsets into anc_tgt
    int32_t *anc_tgt = nullptr;    // [nleaf points] targets grouped by the anchor of their leaf
    int32_t *proxy_slot = nullptr, *local_slot = nullptr, *psi_slot = nullptr;
    bool queued = false;           // upward pass and local values queue-fed (else one launch per level)
    int32_t *l_fout_up = nullptr;  // l_fout with the levels in reverse (finest first): the upward queue
    int32_t *q_fail = nullptr;     // waits of the queue-fed kernels that ran out of polls (sticky)
    int64_t nfout = 0, nfin = 0, nanc = 0, nleaf = 0, max_fin_level = 0, max_fout_level = 0;
    // sibling groups for the diagonal translation: per parent of F_in boxes,
    // the Psi slots of its 2^dim children and the Phi slots of the 4^dim
    // boxes of the block around them (-1 where absent); a root with F_in
    // forms a group of its own
    int32_t *oct_dst = nullptr;    // [noct][2^dim]
    int32_t *oct_src = nullptr;    // [noct][4^dim]
    int32_t *oct_level = nullptr;  // [noct] level of the children
    int32_t *oct_prob = nullptr;   // [noct] problem of the group
    int64_t noct = 0;

    // near (residual) lists in gather form over l_leaf order
    int32_t *nl_off = nullptr, *nl_src = nullptr;
    int32_t *nl_pre = nullptr;     // [nl_total + nleaf] running source-point counts per list (+ total)
    int32_t nl_max = 0;            // longest residual list (source boxes)
    int64_t nl_total = 0, npairs = 0;

    // device tables, FP64 and FP32 copies
    double *d_c2p = nullptr, *d_epw = nullptr, *d_ew = nullptr, *d_wd0 = nullptr,
           *d_ww = nullptr, *d_gcheb = nullptr, *d_gmono = nullptr, *d_xcheb = nullptr, *d_bary = nullptr;
    float *f_c2p = nullptr, *f_epw = nullptr, *f_wd0 = nullptr, *f_gcheb = nullptr, *f_gmono = nullptr,
          *f_xcheb = nullptr, *f_bary = nullptr;

    // eval workspace (element type: double for DMK_FP64, float for DMK_MIXED)
    double *qs = nullptr, *ufar = nullptr, *ures = nullptr, *rootscratch = nullptr;
    void *proxy = nullptr;   // [nfout][p^3]
    void *local = nullptr;   // [nanc][p^3]
    void *phi = nullptr;     // [max_fout_level][2][nh*nn*nn] planar
    void *psi = nullptr;     // [max_fin_level][2][nh*nn*nn] planar
    void *w0vals = nullptr;  // [nprob][p^d] W_0 values on the root grids
    int32_t *qctl = nullptr; // queue heads [4], then per-slot flags: upward [nfout], local [nanc]
    int64_t ws_bytes = 0;         // the workspace's size, each buffer rounded up to 256 bytes
    bool has_workspace = false;   // false for DMK_FLAG_NO_WORKSPACE plans

    // 2-D K_0(lambda r): tables per (problem, level), index b * nlevels + l,
    // for mu = lambda S_b 2^-l (lambda S_b: the problem's scaled parameter)
    double *y_wd64 = nullptr;  float *y_wd32 = nullptr;     // [ntab][nn*nh] D_l weights
    double *y_ww = nullptr;                                  // [nprob][nwn*nwh] W_0 weights
    double *y_cheb64 = nullptr; float *y_cheb32 = nullptr;  // [ntab][YDEG+1] smooth part M_l
    double *y_self = nullptr;                                // [ntab] M_l(0)
    double *y_lam = nullptr;                                 // [nprob] lambda S_b
    int y_deg = 0, y_deg32 = 0;

    // per-stage event timing (dmk_stage_timing / dmk_stage_times)
    struct Rec { int stage; hipEvent_t a, b; };
    bool timing = false;
    std::vector<Rec> pending;
    std::vector<hipEvent_t> event_pool;
    double stage_ms[DMK_NSTAGES] = {0};
    int64_t stage_launches[DMK_NSTAGES] = {0};

    // algorithmic work counts gathered at plan time
    int64_t n_anterp = 0;      // points anterpolated straight onto F_out parents
    int64_t n_merge = 0;       // F_out children merged by c2p
    int64_t n_shift_pairs = 0; // (F_in box, F_out colleague) pairs
    int64_t npairs_in = 0;     // residual pairs closer than the source box side
    int64_t nanc_tgt = 0;      // anchors with at least one target (blocks of the leaf stage that read values)

    // batched execution: graph of the eval core, capture and side streams
    hipStream_t cap_stream = nullptr, side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraphExec_t graph_exec = nullptr;

    std::vector<void *> allocations;
    int64_t device_bytes = 0;
    std::atomic<int> busy{0};
    hipStream_t last_stream = nullptr;
    // completion of the last eval (recorded on its stream): the next eval's
    // stream waits on it, because the workspace is plan-owned
    hipEvent_t ev_done = nullptr;
    bool done_recorded = false;
};

void *dalloc(Plan *P, size_t bytes);  // tracked device allocation
void plan_free_all(Plan *P);
void create_done_event(Plan *P);  // the completion event that orders evals on different streams
// Orders an eval after the plan's previous one (begin) and records its
// completion (end); both skip the event while the stream is being captured.
void begin_eval(Plan *P, hipStream_t s);
void end_eval(Plan *P, hipStream_t s);

// One eval at a time per plan (host side): a second concurrent call fails.
struct BusyGuard {
    Plan *P;
    explicit BusyGuard(Plan *p) : P(p)
    {
        int expect = 0;
        if (!P->busy.compare_exchange_strong(expect, 1))
            throw Error{DMK_ERR_STATE, "plan is in use by another dmk_eval"};
    }
    ~BusyGuard() { P->busy.store(0); }
};

// Runs f and turns every exception into a status code and a message.
template <typename F>
dmk_status guarded(F &&f)
{
    try {
        f();
        return DMK_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return DMK_ERR_NOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return DMK_ERR_STATE;
    } catch (...) {
        set_error("unknown failure");
        return DMK_ERR_STATE;
    }
}
void plan_release(Plan *P);  // device memory, events, streams, graph, then the Plan itself

void build_tree(Plan *P, const double *pts, hipStream_t s);
// the source and target views of a plan with separate target sets (after build_tree)
void split_roles(Plan *P, hipStream_t s);
void build_lists(Plan *P, hipStream_t s);
void upload_tables(Plan *P, hipStream_t s);
// one buffer of the eval workspace: the plan field that points to it, and its size
struct WsItem {
    void **ptr;
    size_t bytes;
};
// the schedule of the upward pass and the local values: queue-fed over all
// levels by default in 3-D, one launch per level by default in 2-D; the
// flags force either
inline bool queue_schedule(int dim, uint64_t flags)
{
    if (flags & DMK_FLAG_QUEUE_LAUNCHES) return true;
    if (flags & DMK_FLAG_LEVEL_LAUNCHES) return false;
    return dim == 3;
}
void workspace_layout(Plan *P, std::vector<WsItem> &items);
void workspace_layout2(Plan *P, std::vector<WsItem> &items);
// dalloc's the workspace (not for DMK_FLAG_NO_WORKSPACE point plans); sets ws_bytes
void alloc_workspace(Plan *P);
// far-field stages shared with the volume code (root window, plane waves,
// local values of the anchors); p = 18 only
void far_stages(Plan *P, hipStream_t s);
// volume potential: plan (host tree from the density callback, then the box
// tree, lists and tables) and evaluation
dmk_plan_t make_vol_plan(double tol, int32_t q, double rho_scale, int32_t min_level, int32_t max_level,
                         int32_t nfeat, const double *feat, dmk_density_fn density, void *ctx, const dmk_opts *opts,
                         void *stream);
void run_vol_eval(Plan *P, const double *rho, double *u, double *far_part, double *near_part, hipStream_t s);
void vol_nodes(Plan *P, double *xyz, hipStream_t s);
void vol_stage_work(const Plan *P, double *F, double *Bt);

void run_eval(Plan *P, const double *charges, double *pot, double *far_part, double *near_part,
              hipStream_t s);
void count_work(Plan *P, hipStream_t s);
void run_eval2(Plan *P, const double *charges, double *pot, double *far_part, double *near_part,
               hipStream_t s);
void build_yukawa_tables(Plan *P, hipStream_t s);   // 2-D K_0(lambda r)
void build_yukawa3_tables(Plan *P, hipStream_t s);  // 3-D e^{-lambda r}/(4 pi r)
void stage_work(const Plan *P, double *flops, double *bytes);
// direct sums u_i = sum_{j != i} K(r_ij) q_j (input units, each target's own
// problem) at the targets d_tidx[ntgt]; pts [n][dim] and q in input order
void direct_sample(int dim, int kernel, double lam, const double *pts, const double *q, const int64_t *d_off,
                   int nprob, const int64_t *d_tidx, int ntgt, double *d_out, hipStream_t s);

// Records HIP events around one stage launch when timing is enabled.
struct StageScope {
    Plan *P;
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr;
    hipEvent_t get()
    {
        if (!P->event_pool.empty()) {
            hipEvent_t e = P->event_pool.back();
            P->event_pool.pop_back();
            return e;
        }
        hipEvent_t e;
        DMK_HIP(hipEventCreate(&e));
        return e;
    }
    StageScope(Plan *p, hipStream_t st, int sg) : P(p), s(st), stage(sg)
    {
        if (P->timing) {
            a = get();
            DMK_HIP(hipEventRecord(a, s));
        }
    }
    ~StageScope() noexcept(false)
    {
        if (P->timing) {
            hipEvent_t b = get();
            DMK_HIP(hipEventRecord(b, s));
            P->pending.push_back({stage, a, b});
        }
    }
};

}  // namespace dmk
