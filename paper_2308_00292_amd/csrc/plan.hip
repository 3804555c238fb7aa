// Step 0 of the discrete DMK algorithm (Sec. 3.6) on the GPU: root cube,
// Morton keys, stable radix sort, the level-restricted adaptive octree
// (Sec. 3.3), colleagues, coarse neighbours, the flags F_leaf/F_out/F_in,
// per-level work lists and the residual interaction lists.
//
// Tree rules (each box refined into all 8 children):
//  (1) a box holding more than n_s points is refined (below the depth cap);
//  (2) level restriction -- leaves sharing a boundary point differ by at most
//      one level -- holds iff every refined box Q at level l has all its
//      level-l neighbour regions present, i.e. their parents are refined.
// The set of refined boxes is the smallest set closed under (1) and (2).  It
// is computed by one sweep from the finest level upward: the refined boxes of
// level l force the parents of their 27 neighbour regions at level l-1.
// Each box is identified by its Morton prefix; all lookups are binary
// searches in sorted prefix arrays, so the result does not depend on
// scheduling and is reproducible bit for bit.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>

#include "dmk_internal.h"

namespace dmk {

namespace {

constexpr int KB = 21;  // key bits per dimension
constexpr int TPB = 256;

__host__ __device__ inline uint64_t spread3(uint64_t v)
{
    // bit b of v -> bit 3b
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__host__ __device__ inline uint64_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return v;
}

// x is the most significant coordinate inside each 3-bit group
__host__ __device__ inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z)
{
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

__host__ __device__ inline void unmorton(uint64_t k, int64_t *c)
{
    c[0] = (int64_t)compact3(k >> 2);
    c[1] = (int64_t)compact3(k >> 1);
    c[2] = (int64_t)compact3(k);
}

__device__ inline int64_t lower_bound_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline int64_t find_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t i = lower_bound_u64(a, n, v);
    return (i < n && a[i] == v) ? i : -1;
}

// ---------------------------------------------------------------- kernels
__global__ void k_bbox_partial(const double *pts, int64_t n, double *part)
{
    __shared__ double red[7][TPB];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    double bad = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
        for (int d = 0; d < 3; ++d) {
            double v = pts[3 * i + d];
            if (!isfinite(v)) bad = 1.0;
            mn[d] = fmin(mn[d], v);
            mx[d] = fmax(mx[d], v);
        }
    for (int d = 0; d < 3; ++d) { red[d][threadIdx.x] = mn[d]; red[3 + d][threadIdx.x] = mx[d]; }
    red[6][threadIdx.x] = bad;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int d = 0; d < 3; ++d) {
                red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + s]);
                red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + s]);
            }
            red[6][threadIdx.x] = fmax(red[6][threadIdx.x], red[6][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) part[blockIdx.x * 7 + threadIdx.x] = red[threadIdx.x][0];
}

#pragma clang fp contract(off)
__global__ void k_keys(const double *pts, int64_t n, double cx, double cy, double cz, double side,
                       double *xn, uint64_t *keys, int32_t *idx)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    const double scale = 2097152.0;  // 2^21
    const double c[3] = {cx, cy, cz};
    uint64_t k[3];
    for (int d = 0; d < 3; ++d) {
        double x = (pts[3 * i + d] - c[d]) / side;
        xn[d * n + i] = x;
        double f = floor((x + 0.5) * scale);
        uint64_t kk = (f <= 0.0) ? 0ull : (uint64_t)f;
        if (kk > (1ull << KB) - 1ull) kk = (1ull << KB) - 1ull;
        k[d] = kk;
    }
    keys[i] = morton(k[0], k[1], k[2]);
    idx[i] = (int32_t)i;
}
#pragma clang fp contract(on)

__global__ void k_gather_points(const double *xn, const int32_t *perm, int64_t n, double *X, double *Y,
                                double *Z)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    X[i] = xn[j];
    Y[i] = xn[n + j];
    Z[i] = xn[2 * n + j];
}

// children of the refined prefixes of one level
__global__ void k_children(const uint64_t *ref, int64_t m, uint64_t *out)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= 8 * m) return;
    out[i] = (ref[i >> 3] << 3) | (uint64_t)(i & 7);
}

__device__ inline void prefix_range(const uint64_t *keys, int64_t n, uint64_t P, int l, int64_t *lo,
                                    int64_t *hi)
{
    if (l == 0) { *lo = 0; *hi = n; return; }
    int sh = 3 * (KB - l);
    *lo = lower_bound_u64(keys, n, P << sh);
    *hi = lower_bound_u64(keys, n, (P + 1) << sh);
}

__global__ void k_refine_flag(const uint64_t *ex, int64_t m, int l, const uint64_t *keys, int64_t n,
                              int ns, uint8_t *flag)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= m) return;
    int64_t a, b;
    prefix_range(keys, n, ex[i], l, &a, &b);
    flag[i] = (b - a > ns) ? 1 : 0;
}

// parents (level l-1) of the 27 level-l neighbour regions of each refined box
__global__ void k_balance_cands(const uint64_t *ref, int64_t m, int l, uint64_t *out)
{
    int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (t >= 27 * m) return;
    int64_t i = t / 27;
    int k = (int)(t % 27);
    int64_t c[3];
    unmorton(ref[i], c);
    int64_t d[3] = {k / 9 - 1, (k / 3) % 3 - 1, k % 3 - 1};
    int64_t lim = (int64_t)1 << l;
    uint64_t res = ~0ull;
    int64_t q[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        q[a] = c[a] + d[a];
        if (q[a] < 0 || q[a] >= lim) ok = false;
    }
    if (ok) res = morton((uint64_t)(q[0] >> 1), (uint64_t)(q[1] >> 1), (uint64_t)(q[2] >> 1));
    out[t] = res;
}

__global__ void k_box_fill(int l, int64_t b0, int64_t nb, const uint64_t *bkey_all, int64_t prev0,
                           int64_t nprev, int64_t next0, const uint64_t *ref, int64_t nref,
                           const uint64_t *keys, int64_t n, int ns, int32_t *blevel, int32_t *parent,
                           int32_t *child0, int32_t *pstart, int32_t *pcount, uint8_t *bflags,
                           double *bcenter)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nb) return;
    int64_t b = b0 + i;
    uint64_t P = bkey_all[b];
    blevel[b] = l;
    int64_t a, e;
    prefix_range(keys, n, P, l, &a, &e);
    pstart[b] = (int32_t)a;
    pcount[b] = (int32_t)(e - a);
    int64_t r = (nref > 0) ? find_u64(ref, nref, P) : -1;
    bool leaf = r < 0;
    child0[b] = leaf ? -1 : (int32_t)(next0 + 8 * r);
    parent[b] = (l == 0) ? -1 : (int32_t)(prev0 + find_u64(bkey_all + prev0, nprev, P >> 3));
    uint8_t f = leaf ? 1 : 0;
    if (!leaf && (e - a) > ns) f |= 2;
    bflags[b] = f;
    int64_t c[3];
    unmorton(P, c);
    double s = ldexp(1.0, -l);
    for (int d = 0; d < 3; ++d) bcenter[3 * b + d] = -0.5 + ((double)c[d] + 0.5) * s;
}

__global__ void k_colleagues(int l, int64_t b0, int64_t nb, const uint64_t *bkey_all, int32_t *col)
{
    int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (t >= 27 * nb) return;
    int64_t i = t / 27;
    int k = (int)(t % 27);
    int64_t c[3];
    unmorton(bkey_all[b0 + i], c);
    int64_t d[3] = {k / 9 - 1, (k / 3) % 3 - 1, k % 3 - 1};
    int64_t lim = (int64_t)1 << l;
    int32_t res = -1;
    int64_t q[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        q[a] = c[a] + d[a];
        if (q[a] < 0 || q[a] >= lim) ok = false;
    }
    if (ok) {
        int64_t f = find_u64(bkey_all + b0, nb, morton((uint64_t)q[0], (uint64_t)q[1], (uint64_t)q[2]));
        if (f >= 0) res = (int32_t)(b0 + f);
    }
    col[(b0 + i) * 27 + k] = res;
}

__global__ void k_flags2(int64_t nbox, const int32_t *col, const int32_t *parent, uint8_t *bflags)
{
    int64_t b = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (b >= nbox) return;
    uint8_t f = bflags[b];
    bool fin = false;
    for (int k = 0; k < 27; ++k) {
        int32_t j = col[b * 27 + k];
        if (j >= 0 && (bflags[j] & 2)) fin = true;
    }
    bool fout = f & 2;
    int32_t par = parent[b];
    bool term = !fout && (par < 0 || (bflags[par] & 2));
    f |= (fin ? 4 : 0) | (term ? 8 : 0);
    bflags[b] = f;  // bits 0-1 are only read by other threads, bits 2-3 only written here
}

__global__ void k_coarse(int l, int64_t b0, int64_t nb, const uint64_t *bkey_all, int64_t prev0,
                         int64_t nprev, const uint8_t *bflags, int32_t *ncoarse, int32_t *coarse)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nb) return;
    int64_t b = b0 + i;
    int cnt = 0;
    int32_t found[7];
    if (l > 0 && (bflags[b] & 1)) {
        uint64_t P = bkey_all[b];
        int64_t c[3];
        unmorton(P, c);
        int64_t lim = (int64_t)1 << l;
        for (int k = 0; k < 27; ++k) {
            int64_t d[3] = {k / 9 - 1, (k / 3) % 3 - 1, k % 3 - 1};
            int64_t q[3];
            bool ok = true;
            for (int a = 0; a < 3; ++a) {
                q[a] = c[a] + d[a];
                if (q[a] < 0 || q[a] >= lim) ok = false;
            }
            if (!ok) continue;
            uint64_t Q = morton((uint64_t)(q[0] >> 1), (uint64_t)(q[1] >> 1), (uint64_t)(q[2] >> 1));
            if (Q == (P >> 3)) continue;
            int64_t f = find_u64(bkey_all + prev0, nprev, Q);
            if (f < 0) continue;
            int32_t j = (int32_t)(prev0 + f);
            if (!(bflags[j] & 1)) continue;
            bool dup = false;
            for (int m = 0; m < cnt; ++m) dup |= (found[m] == j);
            if (!dup && cnt < 7) found[cnt++] = j;
        }
    }
    ncoarse[b] = cnt;
    for (int m = 0; m < 7; ++m) coarse[b * 7 + m] = (m < cnt) ? found[m] : -1;
}

// ------------------------------------------------------------ small helpers
template <typename T>
T *talloc(Plan *P, int64_t count)
{
    return (T *)dalloc(P, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
}

struct Scratch {  // temporary device buffers freed at the end of the plan build
    std::vector<void *> ptrs;
    template <typename T>
    T *get(int64_t count)
    {
        void *p = nullptr;
        DMK_HIP(hipMalloc(&p, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
        ptrs.push_back(p);
        return (T *)p;
    }
    ~Scratch()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + TPB - 1) / TPB); }

// sorted unique union of uint64 arrays (removes the ~0 sentinel)
int64_t sort_unique(Scratch &S, uint64_t *in, int64_t n, uint64_t **out, hipStream_t s)
{
    if (n == 0) { *out = S.get<uint64_t>(1); return 0; }
    uint64_t *sorted = S.get<uint64_t>(n);
    size_t tb = 0;
    DMK_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, in, sorted, (int)n, 0, 64, s));
    void *tmp = S.get<char>((int64_t)tb);
    DMK_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tb, in, sorted, (int)n, 0, 64, s));
    uint64_t *uniq = S.get<uint64_t>(n);
    int64_t *cnt = S.get<int64_t>(1);
    tb = 0;
    DMK_HIP(hipcub::DeviceSelect::Unique(nullptr, tb, sorted, uniq, cnt, (int)n, s));
    tmp = S.get<char>((int64_t)tb);
    DMK_HIP(hipcub::DeviceSelect::Unique(tmp, tb, sorted, uniq, cnt, (int)n, s));
    int64_t m = 0;
    DMK_HIP(hipMemcpyAsync(&m, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DMK_HIP(hipStreamSynchronize(s));
    if (m > 0) {
        uint64_t last = 0;
        DMK_HIP(hipMemcpy(&last, uniq + m - 1, sizeof(uint64_t), hipMemcpyDeviceToHost));
        if (last == ~0ull) m--;
    }
    *out = uniq;
    return m;
}

}  // namespace

void build_tree(Plan *P, const double *pts, hipStream_t s)
{
    const int64_t n = P->n;
    Scratch S;
    // ---- root cube from the bounding box
    double bb[7] = {0, 0, 0, 0, 0, 0, 0};
    if (n > 0) {
        int nb = (int)std::min<int64_t>(1024, (n + TPB - 1) / TPB);
        double *part = S.get<double>(7 * nb);
        hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(TPB), 0, s, pts, n, part);
        std::vector<double> h(7 * nb);
        DMK_HIP(hipMemcpyAsync(h.data(), part, 7 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipStreamSynchronize(s));
        for (int d = 0; d < 3; ++d) { bb[d] = h[d]; bb[3 + d] = h[3 + d]; }
        for (int b = 0; b < nb; ++b) {
            for (int d = 0; d < 3; ++d) {
                bb[d] = std::min(bb[d], h[7 * b + d]);
                bb[3 + d] = std::max(bb[3 + d], h[7 * b + 3 + d]);
            }
            bb[6] = std::max(bb[6], h[7 * b + 6]);
        }
        if (bb[6] != 0.0) throw Error{DMK_ERR_ARG, "non-finite point coordinate"};
    }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        P->center[d] = 0.5 * (bb[d] + bb[3 + d]);
        if (bb[3 + d] - bb[d] > ext) ext = bb[3 + d] - bb[d];
    }
    P->side = (ext > 0.0) ? ext * (1.0 + std::ldexp(1.0, -40)) : 1.0;

    // ---- keys, sort, sorted coordinates
    P->X = talloc<double>(P, n);
    P->Y = talloc<double>(P, n);
    P->Z = talloc<double>(P, n);
    P->perm = talloc<int32_t>(P, n);
    P->keys = talloc<uint64_t>(P, n);
    if (n > 0) {
        double *xn = S.get<double>(3 * n);
        uint64_t *k0 = S.get<uint64_t>(n);
        int32_t *i0 = S.get<int32_t>(n);
        hipLaunchKernelGGL(k_keys, dim3(nblk(n)), dim3(TPB), 0, s, pts, n, P->center[0], P->center[1],
                           P->center[2], P->side, xn, k0, i0);
        size_t tb = 0;
        DMK_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k0, P->keys, i0, P->perm, (int)n, 0, 63, s));
        void *tmp = S.get<char>((int64_t)tb);
        DMK_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, k0, P->keys, i0, P->perm, (int)n, 0, 63, s));
        hipLaunchKernelGGL(k_gather_points, dim3(nblk(n)), dim3(TPB), 0, s, xn, P->perm, n, P->X, P->Y, P->Z);
    }

    // ---- refinement by count
    const int maxd = P->max_depth;
    std::vector<uint64_t *> ref(maxd + 2, nullptr);
    std::vector<int64_t> nref(maxd + 2, 0);
    uint64_t *ex = S.get<uint64_t>(1);
    {
        uint64_t zero = 0;
        DMK_HIP(hipMemcpyAsync(ex, &zero, sizeof(uint64_t), hipMemcpyHostToDevice, s));
    }
    int64_t nex = 1;
    for (int l = 0; l < maxd && n > 0; ++l) {
        if (l > 0) {
            nex = 8 * nref[l - 1];
            ex = S.get<uint64_t>(nex);
            hipLaunchKernelGGL(k_children, dim3(nblk(nex)), dim3(TPB), 0, s, ref[l - 1], nref[l - 1], ex);
        }
        uint8_t *flag = S.get<uint8_t>(nex);
        hipLaunchKernelGGL(k_refine_flag, dim3(nblk(nex)), dim3(TPB), 0, s, ex, nex, l, P->keys, n,
                           P->leaf_max, flag);
        uint64_t *sel = S.get<uint64_t>(nex);
        int64_t *cnt = S.get<int64_t>(1);
        size_t tb = 0;
        DMK_HIP(hipcub::DeviceSelect::Flagged(nullptr, tb, ex, flag, sel, cnt, (int)nex, s));
        void *tmp = S.get<char>((int64_t)tb);
        DMK_HIP(hipcub::DeviceSelect::Flagged(tmp, tb, ex, flag, sel, cnt, (int)nex, s));
        int64_t m = 0;
        DMK_HIP(hipMemcpyAsync(&m, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipStreamSynchronize(s));
        ref[l] = sel;
        nref[l] = m;
        if (m == 0) break;
    }
    // ---- level restriction: finest refined level upward
    int lmax = -1;
    for (int l = 0; l < maxd; ++l)
        if (nref[l] > 0) lmax = l;
    for (int l = lmax; l >= 1; --l) {
        if (nref[l] == 0) continue;
        int64_t nc = 27 * nref[l];
        uint64_t *cand = S.get<uint64_t>(nc + nref[l - 1]);
        hipLaunchKernelGGL(k_balance_cands, dim3(nblk(nc)), dim3(TPB), 0, s, ref[l], nref[l], l, cand);
        if (nref[l - 1] > 0)
            DMK_HIP(hipMemcpyAsync(cand + nc, ref[l - 1], nref[l - 1] * sizeof(uint64_t),
                                   hipMemcpyDeviceToDevice, s));
        uint64_t *merged = nullptr;
        int64_t m = sort_unique(S, cand, nc + nref[l - 1], &merged, s);
        ref[l - 1] = merged;
        nref[l - 1] = m;
    }

    // ---- materialise boxes level by level
    std::vector<int64_t> lstart(1, 0);
    std::vector<int64_t> cnts;
    cnts.push_back(1);
    for (int l = 1; l <= maxd; ++l) {
        if (nref[l - 1] == 0) break;
        cnts.push_back(8 * nref[l - 1]);
    }
    P->nlevels = (int)cnts.size();
    for (int64_t c : cnts) lstart.push_back(lstart.back() + c);
    P->level_start = lstart;
    const int64_t nbox = lstart.back();
    P->nbox = nbox;
    P->bkey = talloc<uint64_t>(P, nbox);
    P->blevel = talloc<int32_t>(P, nbox);
    P->parent = talloc<int32_t>(P, nbox);
    P->child0 = talloc<int32_t>(P, nbox);
    P->pstart = talloc<int32_t>(P, nbox);
    P->pcount = talloc<int32_t>(P, nbox);
    P->bflags = talloc<uint8_t>(P, nbox);
    P->colleague = talloc<int32_t>(P, 27 * nbox);
    P->ncoarse = talloc<int32_t>(P, nbox);
    P->coarse = talloc<int32_t>(P, 7 * nbox);
    P->bcenter = talloc<double>(P, 3 * nbox);
    {
        uint64_t zero = 0;
        DMK_HIP(hipMemcpyAsync(P->bkey, &zero, sizeof(uint64_t), hipMemcpyHostToDevice, s));
    }
    for (int l = 1; l < P->nlevels; ++l)
        hipLaunchKernelGGL(k_children, dim3(nblk(cnts[l])), dim3(TPB), 0, s, ref[l - 1], nref[l - 1],
                           P->bkey + lstart[l]);
    for (int l = 0; l < P->nlevels; ++l) {
        int64_t prev0 = (l > 0) ? lstart[l - 1] : 0, nprev = (l > 0) ? cnts[l - 1] : 0;
        int64_t next0 = lstart[l + 1];
        hipLaunchKernelGGL(k_box_fill, dim3(nblk(cnts[l])), dim3(TPB), 0, s, l, lstart[l], cnts[l], P->bkey,
                           prev0, nprev, next0, ref[l], (l < maxd) ? nref[l] : (int64_t)0, P->keys, n,
                           P->leaf_max, P->blevel, P->parent, P->child0, P->pstart, P->pcount, P->bflags,
                           P->bcenter);
    }
    for (int l = 0; l < P->nlevels; ++l)
        hipLaunchKernelGGL(k_colleagues, dim3(nblk(27 * cnts[l])), dim3(TPB), 0, s, l, lstart[l], cnts[l],
                           P->bkey, P->colleague);
    hipLaunchKernelGGL(k_flags2, dim3(nblk(nbox)), dim3(TPB), 0, s, nbox, P->colleague, P->parent, P->bflags);
    for (int l = 0; l < P->nlevels; ++l) {
        int64_t prev0 = (l > 0) ? lstart[l - 1] : 0, nprev = (l > 0) ? cnts[l - 1] : 0;
        hipLaunchKernelGGL(k_coarse, dim3(nblk(cnts[l])), dim3(TPB), 0, s, l, lstart[l], cnts[l], P->bkey,
                           prev0, nprev, P->bflags, P->ncoarse, P->coarse);
    }
    DMK_HIP(hipGetLastError());
    DMK_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ lists
namespace {

__global__ void k_list_flags(int64_t nbox, const uint8_t *bflags, const int32_t *pcount, uint8_t *f_fout,
                             uint8_t *f_fin, uint8_t *f_leaf)
{
    int64_t b = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (b >= nbox) return;
    uint8_t f = bflags[b];
    bool ne = pcount[b] > 0;
    f_fout[b] = (f & 2) ? 1 : 0;
    f_fin[b] = (ne && (f & 4)) ? 1 : 0;
    f_leaf[b] = (ne && (f & 1)) ? 1 : 0;
}

// targets grouped by anchor: per leaf, its anchor's slot, and per anchor the
// number of targets
__global__ void k_leaf_keys(const int32_t *leaves, int64_t nleaf, const int32_t *anchor, const int32_t *local_slot,
                            const int32_t *pcount, int32_t *key, int32_t *ident, int32_t *anc_cnt)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nleaf) return;
    int32_t L = leaves[i];
    int32_t a = local_slot[anchor[L]];
    key[i] = a;
    ident[i] = L;
    atomicAdd(&anc_cnt[a], pcount[L]);
}

__global__ void k_leaf_counts(const int32_t *sorted_leaves, int64_t nleaf, const int32_t *pcount, int32_t *cnt)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < nleaf) cnt[i] = pcount[sorted_leaves[i]];
}

__global__ void k_fill_targets(const int32_t *sorted_leaves, int64_t nleaf, const int32_t *pstart,
                               const int32_t *pcount, const int32_t *pos, int32_t *tgt)
{
    int64_t i = blockIdx.x;
    if (i >= nleaf) return;
    int32_t L = sorted_leaves[i];
    for (int k = threadIdx.x; k < pcount[L]; k += TPB) tgt[pos[i] + k] = pstart[L] + k;
}

__global__ void k_slots(const int32_t *list, int64_t m, int32_t *slot)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < m) slot[list[i]] = (int32_t)i;
}

// parents of the non-empty F_in boxes of levels >= 1
__global__ void k_oct_flag(const int32_t *fin, int64_t m, const int32_t *parent, uint8_t *flag)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= m) return;
    int32_t P = parent[fin[i]];
    if (P >= 0) flag[P] = 1;
}

// sibling group of parent P: child k = (x y z bits) sits at cell k + (1,1,1)
// of the 4x4x4 block; cell g holds child ((g+1) & 1) of P's colleague at
// offset (g+1)/2 - 1 per axis
__global__ void k_oct_fill(const int32_t *octs, int64_t m, const int32_t *child0, const int32_t *col,
                           const uint8_t *bflags, const int32_t *blevel, const int32_t *proxy_slot,
                           const int32_t *psi_slot, int32_t *dst, int32_t *src, int32_t *lev)
{
    int64_t i = blockIdx.x;
    if (i >= m) return;
    const int32_t P = octs[i];
    const int t = threadIdx.x;
    if (t < 8) dst[i * 8 + t] = psi_slot[child0[P] + t];
    if (t == 0) lev[i] = blevel[P] + 1;
    if (t < 64) {
        const int g[3] = {t / 16, (t / 4) % 4, t % 4};
        int k = 0, c = 0;
        for (int a = 0; a < 3; ++a) {
            k = 3 * k + (g[a] + 1) / 2;      // colleague offset + 1
            c = 2 * c + ((g[a] + 1) & 1);   // child bit
        }
        int32_t C = col[(int64_t)P * 27 + k];
        int32_t v = -1;
        if (C >= 0 && child0[C] >= 0) {
            int32_t S = child0[C] + c;
            if (bflags[S] & 2) v = proxy_slot[S];
        }
        src[i * 64 + t] = v;
    }
}

// anchor of a box: itself if it holds points and has F_in, else its parent's
// anchor; the root is always an anchor.  One launch per level, top down.
__global__ void k_anchor(int64_t b0, int64_t nb, const int32_t *parent, const uint8_t *f_fin, int32_t *anchor)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nb) return;
    int64_t b = b0 + i;
    anchor[b] = (parent[b] < 0 || f_fin[b]) ? (int32_t)b : anchor[parent[b]];
}

// residual lists, gather form: for target leaf B, the terminal non-empty
// boxes among (a) the colleagues of B and of each of its ancestors and
// (b) the leaves one level finer that share a boundary point with B.
template <bool FILL>
__global__ void k_near_lists(const int32_t *leaves, int64_t nleaf, const int32_t *lstart_dev, int nlevels,
                             const uint64_t *bkey, const int32_t *blevel, const int32_t *parent,
                             const int32_t *col, const uint8_t *bflags, const int32_t *pcount,
                             int32_t *count, const int32_t *off, int32_t *src, int32_t *pre, int64_t *pairs)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nleaf) return;
    int32_t B = leaves[i];
    int cnt = 0;
    int64_t pr = 0;
    int32_t base = FILL ? off[i] : 0;
    // pre: running count of source points before each entry (FILL pass)
    for (int32_t A = B; A >= 0; A = parent[A])
        for (int k = 0; k < 27; ++k) {
            int32_t T = col[(int64_t)A * 27 + k];
            if (T >= 0 && (bflags[T] & 8) && pcount[T] > 0) {
                if (FILL) { src[base + cnt] = T; pre[base + i + cnt] = (int32_t)pr; }
                cnt++;
                pr += pcount[T];
            }
        }
    int l = blevel[B];
    if (l + 1 < nlevels) {
        int64_t c[3];
        unmorton(bkey[B], c);
        int64_t lim = (int64_t)1 << (l + 1);
        int64_t n1 = lstart_dev[l + 2] - lstart_dev[l + 1];
        const uint64_t *k1 = bkey + lstart_dev[l + 1];
        for (int r = 0; r < 64; ++r) {
            int64_t o[3] = {r / 16 - 1, (r / 4) % 4 - 1, r % 4 - 1};
            bool own = true, ok = true;
            int64_t q[3];
            for (int a = 0; a < 3; ++a) {
                if (o[a] < 0 || o[a] > 1) own = false;
                q[a] = 2 * c[a] + o[a];
                if (q[a] < 0 || q[a] >= lim) ok = false;
            }
            if (own || !ok) continue;
            int64_t f = find_u64(k1, n1, morton((uint64_t)q[0], (uint64_t)q[1], (uint64_t)q[2]));
            if (f < 0) continue;
            int32_t T = (int32_t)(lstart_dev[l + 1] + f);
            if ((bflags[T] & 1) && (bflags[T] & 8) && pcount[T] > 0) {
                if (FILL) { src[base + cnt] = T; pre[base + i + cnt] = (int32_t)pr; }
                cnt++;
                pr += pcount[T];
            }
        }
    }
    if (FILL) pre[base + i + cnt] = (int32_t)pr;  // total after the last entry (one extra slot per leaf)
    if (!FILL) {
        count[i] = cnt;
        pairs[i] = pr * pcount[B];
    }
}

int64_t select_indices(Scratch &S, const uint8_t *flag, int64_t first, int64_t count, int32_t *out,
                       hipStream_t s)
{
    if (count == 0) return 0;
    hipcub::CountingInputIterator<int32_t> it((int32_t)first);
    int64_t *cnt = S.get<int64_t>(1);
    size_t tb = 0;
    DMK_HIP(hipcub::DeviceSelect::Flagged(nullptr, tb, it, flag + first, out, cnt, (int)count, s));
    void *tmp = S.get<char>((int64_t)tb);
    DMK_HIP(hipcub::DeviceSelect::Flagged(tmp, tb, it, flag + first, out, cnt, (int)count, s));
    int64_t m = 0;
    DMK_HIP(hipMemcpyAsync(&m, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DMK_HIP(hipStreamSynchronize(s));
    return m;
}

}  // namespace

void build_lists(Plan *P, hipStream_t s)
{
    Scratch S;
    const int64_t nbox = P->nbox;
    const int L = P->nlevels;
    uint8_t *f_fout = S.get<uint8_t>(nbox), *f_fin = S.get<uint8_t>(nbox), *f_leaf = S.get<uint8_t>(nbox);
    hipLaunchKernelGGL(k_list_flags, dim3(nblk(nbox)), dim3(TPB), 0, s, nbox, P->bflags, P->pcount, f_fout, f_fin,
                       f_leaf);
    P->l_fout = talloc<int32_t>(P, nbox);
    P->l_fin = talloc<int32_t>(P, nbox);
    P->l_anc = talloc<int32_t>(P, nbox + 1);
    P->l_leaf = talloc<int32_t>(P, nbox);
    P->anchor = talloc<int32_t>(P, nbox);
    auto &ll = P->ll;
    ll.fout_off.assign(L + 1, 0);
    ll.fin_off.assign(L + 1, 0);
    ll.anc_off.assign(L + 1, 0);
    ll.leaf_off.assign(L + 1, 0);
    for (int l = 0; l < L; ++l) {
        int64_t b0 = P->level_start[l], nb = P->level_start[l + 1] - b0;
        ll.fout_off[l + 1] = ll.fout_off[l] + select_indices(S, f_fout, b0, nb, P->l_fout + ll.fout_off[l], s);
        ll.fin_off[l + 1] = ll.fin_off[l] + select_indices(S, f_fin, b0, nb, P->l_fin + ll.fin_off[l], s);
        ll.leaf_off[l + 1] = ll.leaf_off[l] + select_indices(S, f_leaf, b0, nb, P->l_leaf + ll.leaf_off[l], s);
        hipLaunchKernelGGL(k_anchor, dim3(nblk(nb)), dim3(TPB), 0, s, b0, nb, P->parent, f_fin, P->anchor);
    }
    // anchors: the root, then the non-empty F_in boxes of levels >= 1
    {
        int32_t zero = 0;
        DMK_HIP(hipMemcpyAsync(P->l_anc, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
        ll.anc_off[0] = 0;
        ll.anc_off[1] = (P->n > 0) ? 1 : 0;
        for (int l = 1; l < L; ++l) {
            int64_t m = ll.fin_off[l + 1] - ll.fin_off[l];
            if (m)
                DMK_HIP(hipMemcpyAsync(P->l_anc + ll.anc_off[l], P->l_fin + ll.fin_off[l], m * sizeof(int32_t),
                                       hipMemcpyDeviceToDevice, s));
            ll.anc_off[l + 1] = ll.anc_off[l] + m;
        }
    }
    P->nfout = ll.fout_off[L];
    P->nfin = ll.fin_off[L];
    P->nanc = ll.anc_off[L];
    P->nleaf = ll.leaf_off[L];
    P->max_fin_level = 0;
    P->max_fout_level = 0;
    for (int l = 0; l < L; ++l) {
        P->max_fin_level = std::max(P->max_fin_level, ll.fin_off[l + 1] - ll.fin_off[l]);
        P->max_fout_level = std::max(P->max_fout_level, ll.fout_off[l + 1] - ll.fout_off[l]);
    }
    P->proxy_slot = talloc<int32_t>(P, nbox);
    P->local_slot = talloc<int32_t>(P, nbox);
    P->psi_slot = talloc<int32_t>(P, nbox);
    DMK_HIP(hipMemsetAsync(P->proxy_slot, 0xff, nbox * sizeof(int32_t), s));
    DMK_HIP(hipMemsetAsync(P->local_slot, 0xff, nbox * sizeof(int32_t), s));
    DMK_HIP(hipMemsetAsync(P->psi_slot, 0xff, nbox * sizeof(int32_t), s));
    if (P->nfout)
        hipLaunchKernelGGL(k_slots, dim3(nblk(P->nfout)), dim3(TPB), 0, s, P->l_fout, P->nfout, P->proxy_slot);
    if (P->nanc)
        hipLaunchKernelGGL(k_slots, dim3(nblk(P->nanc)), dim3(TPB), 0, s, P->l_anc, P->nanc, P->local_slot);
    if (P->nfin)
        hipLaunchKernelGGL(k_slots, dim3(nblk(P->nfin)), dim3(TPB), 0, s, P->l_fin, P->nfin, P->psi_slot);

    // sibling groups for the diagonal translation (the root first, then the
    // parents level by level)
    {
        uint8_t *f_oct = S.get<uint8_t>(nbox);
        DMK_HIP(hipMemsetAsync(f_oct, 0, nbox, s));
        if (P->nfin)
            hipLaunchKernelGGL(k_oct_flag, dim3(nblk(P->nfin)), dim3(TPB), 0, s, P->l_fin, P->nfin, P->parent, f_oct);
        int32_t *octs = S.get<int32_t>(nbox + 1);
        int64_t m = select_indices(S, f_oct, 0, nbox, octs, s);
        int32_t root_psi = -1, root_phi = -1;
        if (nbox > 0) {
            DMK_HIP(hipMemcpyAsync(&root_psi, P->psi_slot, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            DMK_HIP(hipMemcpyAsync(&root_phi, P->proxy_slot, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            DMK_HIP(hipStreamSynchronize(s));
        }
        const int64_t r = (root_psi >= 0) ? 1 : 0;
        P->noct = m + r;
        P->oct_dst = talloc<int32_t>(P, std::max<int64_t>(P->noct, 1) * 8);
        P->oct_src = talloc<int32_t>(P, std::max<int64_t>(P->noct, 1) * 64);
        P->oct_level = talloc<int32_t>(P, std::max<int64_t>(P->noct, 1));
        if (r) {
            // the root's only colleague is itself: target cell (1,1,1) = 21
            std::vector<int32_t> d(8, -1), g(64, -1);
            d[0] = root_psi;
            g[21] = root_phi;
            int32_t l0 = 0;
            DMK_HIP(hipMemcpyAsync(P->oct_dst, d.data(), 8 * sizeof(int32_t), hipMemcpyHostToDevice, s));
            DMK_HIP(hipMemcpyAsync(P->oct_src, g.data(), 64 * sizeof(int32_t), hipMemcpyHostToDevice, s));
            DMK_HIP(hipMemcpyAsync(P->oct_level, &l0, sizeof(int32_t), hipMemcpyHostToDevice, s));
            DMK_HIP(hipStreamSynchronize(s));
        }
        if (m)
            hipLaunchKernelGGL(k_oct_fill, dim3((unsigned)m), dim3(64), 0, s, octs, m, P->child0, P->colleague,
                               P->bflags, P->blevel, P->proxy_slot, P->psi_slot, P->oct_dst + 8 * r,
                               P->oct_src + 64 * r, P->oct_level + r);
    }

    // targets grouped by the anchor of their leaf (leaf evaluation)
    {
        const int64_t nleaf = ll.leaf_off[L], nanc = ll.anc_off[L];
        P->anc_tbeg = talloc<int32_t>(P, nanc + 1);
        P->anc_tgt = talloc<int32_t>(P, std::max<int64_t>(P->n, 1));
        int32_t *cnt = S.get<int32_t>(nanc + 1);
        DMK_HIP(hipMemsetAsync(cnt, 0, (nanc + 1) * sizeof(int32_t), s));
        if (nleaf > 0) {
            int32_t *key = S.get<int32_t>(nleaf), *ident = S.get<int32_t>(nleaf);
            int32_t *skey = S.get<int32_t>(nleaf), *sleaf = S.get<int32_t>(nleaf);
            hipLaunchKernelGGL(k_leaf_keys, dim3(nblk(nleaf)), dim3(TPB), 0, s, P->l_leaf, nleaf, P->anchor,
                               P->local_slot, P->pcount, key, ident, cnt);
            size_t tb = 0;
            DMK_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key, skey, ident, sleaf, (int)nleaf, 0, 32, s));
            void *tmp = S.get<char>((int64_t)tb);
            DMK_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, skey, ident, sleaf, (int)nleaf, 0, 32, s));
            int32_t *lc = S.get<int32_t>(nleaf + 1), *pos = S.get<int32_t>(nleaf + 1);
            hipLaunchKernelGGL(k_leaf_counts, dim3(nblk(nleaf)), dim3(TPB), 0, s, sleaf, nleaf, P->pcount, lc);
            DMK_HIP(hipMemsetAsync(lc + nleaf, 0, sizeof(int32_t), s));
            tb = 0;
            DMK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, lc, pos, (int)nleaf + 1, s));
            tmp = S.get<char>((int64_t)tb);
            DMK_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, lc, pos, (int)nleaf + 1, s));
            hipLaunchKernelGGL(k_fill_targets, dim3((unsigned)nleaf), dim3(TPB), 0, s, sleaf, nleaf, P->pstart,
                               P->pcount, pos, P->anc_tgt);
        }
        size_t tb = 0;
        DMK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, P->anc_tbeg, (int)nanc + 1, s));
        void *tmp = S.get<char>((int64_t)tb);
        DMK_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt, P->anc_tbeg, (int)nanc + 1, s));
    }

    // near lists over the leaf order
    const int64_t nleaf = P->nleaf;
    int32_t *lsd = S.get<int32_t>(L + 2);
    {
        std::vector<int32_t> h(L + 2);
        for (int l = 0; l <= L; ++l) h[l] = (int32_t)P->level_start[l];
        h[L + 1] = h[L];
        DMK_HIP(hipMemcpyAsync(lsd, h.data(), (L + 2) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    P->nl_off = talloc<int32_t>(P, nleaf + 1);
    if (nleaf > 0) {
        int32_t *cnt = S.get<int32_t>(nleaf);
        int64_t *pairs = S.get<int64_t>(nleaf);
        hipLaunchKernelGGL(k_near_lists<false>, dim3(nblk(nleaf)), dim3(TPB), 0, s, P->l_leaf, nleaf, lsd, L, P->bkey,
                           P->blevel, P->parent, P->colleague, P->bflags, P->pcount, cnt, (const int32_t *)nullptr,
                           (int32_t *)nullptr, (int32_t *)nullptr, pairs);
        size_t tb = 0;
        DMK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, P->nl_off, (int)nleaf + 1, s));
        // exclusive sum over nleaf+1 entries needs a trailing zero in the input
        int32_t *cnt1 = S.get<int32_t>(nleaf + 1);
        DMK_HIP(hipMemcpyAsync(cnt1, cnt, nleaf * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        DMK_HIP(hipMemsetAsync(cnt1 + nleaf, 0, sizeof(int32_t), s));
        void *tmp = S.get<char>((int64_t)tb);
        DMK_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt1, P->nl_off, (int)nleaf + 1, s));
        int32_t total = 0;
        DMK_HIP(hipMemcpyAsync(&total, P->nl_off + nleaf, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        {
            int32_t *mx = S.get<int32_t>(1);
            size_t tbm = 0;
            DMK_HIP(hipcub::DeviceReduce::Max(nullptr, tbm, cnt, mx, (int)nleaf, s));
            void *tmpm = S.get<char>((int64_t)tbm);
            DMK_HIP(hipcub::DeviceReduce::Max(tmpm, tbm, cnt, mx, (int)nleaf, s));
            int32_t hmx = 0;
            DMK_HIP(hipMemcpyAsync(&hmx, mx, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            DMK_HIP(hipStreamSynchronize(s));
            if (hmx > 1024)
                throw Error{DMK_ERR_UNSUPPORTED, "a leaf's residual list exceeds 1024 source boxes"};
        }
        int64_t *psum = S.get<int64_t>(1);
        tb = 0;
        DMK_HIP(hipcub::DeviceReduce::Sum(nullptr, tb, pairs, psum, (int)nleaf, s));
        tmp = S.get<char>((int64_t)tb);
        DMK_HIP(hipcub::DeviceReduce::Sum(tmp, tb, pairs, psum, (int)nleaf, s));
        DMK_HIP(hipMemcpyAsync(&P->npairs, psum, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipStreamSynchronize(s));
        P->nl_total = total;
        P->nl_src = talloc<int32_t>(P, total);
        P->nl_pre = talloc<int32_t>(P, total + nleaf);
        hipLaunchKernelGGL(k_near_lists<true>, dim3(nblk(nleaf)), dim3(TPB), 0, s, P->l_leaf, nleaf, lsd, L, P->bkey,
                           P->blevel, P->parent, P->colleague, P->bflags, P->pcount, (int32_t *)nullptr,
                           (const int32_t *)P->nl_off, P->nl_src, P->nl_pre, (int64_t *)nullptr);
    } else {
        P->nl_src = talloc<int32_t>(P, 1);
        P->nl_pre = talloc<int32_t>(P, 1);
        DMK_HIP(hipMemsetAsync(P->nl_off, 0, sizeof(int32_t), s));
    }
    DMK_HIP(hipGetLastError());
    DMK_HIP(hipStreamSynchronize(s));
}

}  // namespace dmk
