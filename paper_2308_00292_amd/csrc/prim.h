// Device-wide primitives of the plan build: stable LSD radix sort of
// (key, value) pairs, exclusive prefix sums, stream compaction and
// reductions.  gfx950, 64-lane waves; plan-time code (the eval never calls
// these).  Temporary buffers come from the caller's allocator `S`, any type
// with `template <class T> T *get(int64_t count)` whose memory lives until
// the work enqueued on the stream has finished.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <type_traits>

namespace dmk {
namespace prim {

constexpr int kThreads = 256;          // threads per block
constexpr int kItems = 8;              // items per thread in a tile
constexpr int kTile = kThreads * kItems;
constexpr int kDigits = 256;           // 8-bit radix digits
constexpr int kWaves = kThreads / 64;

inline unsigned tiles(int64_t n) { return (unsigned)((n + kTile - 1) / kTile); }

// ------------------------------------------------------------- scans
// Block-wide exclusive scan of one int32 per thread (returns the block total).
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *lds_wave, int32_t &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t incl = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) lds_wave[wave] = incl;
    __syncthreads();
    int32_t before = 0;
    total = 0;
    for (int w = 0; w < kWaves; ++w) {
        const int32_t t = lds_wave[w];
        if (w < wave) before += t;
        total += t;
    }
    __syncthreads();
    return before + incl - v;
}

// Each block scans its tile in place order: out[i] = sum of in[tile start .. i-1];
// sums[block] = the tile's total.
__global__ void __launch_bounds__(kThreads) k_scan_tile(const int32_t *in, int32_t *out, int64_t n, int32_t *sums)
{
    __shared__ int32_t wsum[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int32_t v[kItems];
    int32_t run = 0;
    for (int k = 0; k < kItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        run += v[k];
    }
    int32_t total;
    int32_t ex = block_exclusive_scan(run, wsum, total);
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kThreads) k_scan_add(int32_t *out, int64_t n, const int32_t *offs)
{
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int32_t o = offs[blockIdx.x];
    for (int k = threadIdx.x; k < kTile; k += kThreads)
        if (base + k < n) out[base + k] += o;
}

// out[i] = in[0] + ... + in[i-1] for i < n (in and out may not alias).
template <class Alloc>
void exclusive_scan(Alloc &S, const int32_t *in, int32_t *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    const unsigned nb = tiles(n);
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kThreads), 0, s, in, out, n, (int32_t *)nullptr);
        return;
    }
    int32_t *sums = S.template get<int32_t>(nb);
    int32_t *offs = S.template get<int32_t>(nb);
    hipLaunchKernelGGL(k_scan_tile, dim3(nb), dim3(kThreads), 0, s, in, out, n, sums);
    exclusive_scan(S, sums, offs, nb, s);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kThreads), 0, s, out, n, offs);
}

// ------------------------------------------------------- radix sort
template <typename K>
__global__ void __launch_bounds__(kThreads) k_rs_hist(const K *keys, int64_t n, int shift, int32_t *hist)
{
    __shared__ int32_t h[kDigits];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int k = threadIdx.x; k < kTile; k += kThreads)
        if (base + k < n) atomicAdd(&h[(int)((keys[base + k] >> shift) & 0xff)], 1);
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];  // digit-major
}

// Scatters one tile stably: rounds of kThreads consecutive items; within a
// round the rank among equal digits comes from wave ballots (lower lanes)
// and the counts of lower waves, across rounds from a running count.
template <typename K, bool VALS>
__global__ void __launch_bounds__(kThreads) k_rs_scatter(const K *kin, const int32_t *vin, K *kout, int32_t *vout,
                                                         int64_t n, int shift, const int32_t *offs)
{
    __shared__ int32_t run[kDigits];
    __shared__ int32_t wcnt[kWaves][kDigits];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    run[threadIdx.x] = offs[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
        const bool live = i < n;
        K key = 0;
        int32_t val = 0;
        int dg = 0;
        if (live) {
            key = kin[i];
            if (VALS) val = vin[i];
            dg = (int)((key >> shift) & 0xff);
        }
        uint64_t match = __ballot(live);
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot(live && ((dg >> b) & 1));
            match &= ((dg >> b) & 1) ? bb : ~bb;
        }
        const int rank = __popcll(match & lt);
        const int cnt = __popcll(match);
        if (live && rank == cnt - 1) wcnt[wave][dg] = cnt;  // the group's last lane
        __syncthreads();
        if (live) {
            int32_t pos = run[dg] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][dg];
            kout[pos] = key;
            if (VALS) vout[pos] = val;
        }
        __syncthreads();
        int32_t add = 0;
        for (int w = 0; w < kWaves; ++w) {
            add += wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = 0;
        }
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

// Stable sort of n keys (and int32 values if vin) by bits [0, end_bit);
// results in kout / vout.  kin / vin are not modified.
template <class Alloc, typename K>
void sort_pairs(Alloc &S, const K *kin, K *kout, const int32_t *vin, int32_t *vout, int64_t n, int end_bit,
                hipStream_t s)
{
    static_assert(std::is_unsigned<K>::value, "unsigned keys");
    if (n <= 0) return;
    const int passes = std::max(1, (end_bit + 7) / 8);
    const unsigned nb = tiles(n);
    int32_t *hist = S.template get<int32_t>((int64_t)kDigits * nb);
    int32_t *offs = S.template get<int32_t>((int64_t)kDigits * nb);
    K *kalt = S.template get<K>(n);
    int32_t *valt = vin ? S.template get<int32_t>(n) : nullptr;
    const K *ksrc = kin;
    const int32_t *vsrc = vin;
    for (int p = 0; p < passes; ++p) {
        // the last pass lands in kout / vout
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        K *kdst = to_out ? kout : kalt;
        int32_t *vdst = to_out ? vout : valt;
        hipLaunchKernelGGL(k_rs_hist<K>, dim3(nb), dim3(kThreads), 0, s, ksrc, n, 8 * p, hist);
        exclusive_scan(S, hist, offs, (int64_t)kDigits * nb, s);
        if (vin)
            hipLaunchKernelGGL((k_rs_scatter<K, true>), dim3(nb), dim3(kThreads), 0, s, ksrc, vsrc, kdst, vdst, n,
                               8 * p, offs);
        else
            hipLaunchKernelGGL((k_rs_scatter<K, false>), dim3(nb), dim3(kThreads), 0, s, ksrc, vsrc, kdst, vdst, n,
                               8 * p, offs);
        ksrc = kdst;
        vsrc = vdst;
    }
}

// -------------------------------------------------------- compaction
__global__ void __launch_bounds__(kThreads) k_flag_i32(const uint8_t *flag, int64_t n, int32_t *f)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) f[i] = flag[i] ? 1 : 0;
}

template <typename K>
__global__ void __launch_bounds__(kThreads) k_flag_unique(const K *a, int64_t n, int32_t *f)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) f[i] = (i == 0 || a[i] != a[i - 1]) ? 1 : 0;
}

// items == nullptr: the selected item is first + i (a counting sequence)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_select(const T *items, T first, const int32_t *f, const int32_t *pos,
                                                     int64_t n, T *out, int64_t *count)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    if (f[i]) out[pos[i]] = items ? items[i] : (T)(first + (T)i);
    if (i == n - 1) *count = (int64_t)pos[i] + f[i];
}

inline unsigned blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kThreads - 1) / kThreads); }

// out = the items whose flag is set, in order; *d_count (device) their number.
template <class Alloc, typename T>
void select_flagged(Alloc &S, const T *items, T first, const uint8_t *flag, T *out, int64_t *d_count, int64_t n,
                    hipStream_t s)
{
    int32_t *f = S.template get<int32_t>(n);
    int32_t *pos = S.template get<int32_t>(n);
    hipLaunchKernelGGL(k_flag_i32, dim3(blocks(n)), dim3(kThreads), 0, s, flag, n, f);
    exclusive_scan(S, f, pos, n, s);
    hipLaunchKernelGGL(k_select<T>, dim3(blocks(n)), dim3(kThreads), 0, s, items, first, (const int32_t *)f,
                       (const int32_t *)pos, n, out, d_count);
}

// out = the distinct values of the sorted array a, in order; *d_count their number.
template <class Alloc, typename K>
void unique_sorted(Alloc &S, const K *a, K *out, int64_t *d_count, int64_t n, hipStream_t s)
{
    int32_t *f = S.template get<int32_t>(n);
    int32_t *pos = S.template get<int32_t>(n);
    hipLaunchKernelGGL(k_flag_unique<K>, dim3(blocks(n)), dim3(kThreads), 0, s, a, n, f);
    exclusive_scan(S, f, pos, n, s);
    hipLaunchKernelGGL(k_select<K>, dim3(blocks(n)), dim3(kThreads), 0, s, a, (K)0, (const int32_t *)f,
                       (const int32_t *)pos, n, out, d_count);
}

// -------------------------------------------------------- reductions
__global__ void __launch_bounds__(kThreads) k_max_i32(const int32_t *a, int64_t n, int32_t *res)
{
    __shared__ int32_t w[kWaves];
    int32_t m = INT32_MIN;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        m = max(m, a[i]);
    for (int d = 32; d > 0; d >>= 1) m = max(m, __shfl_xor(m, d, 64));
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kWaves; ++k) m = max(m, w[k]);
        atomicMax(res, m);
    }
}

__global__ void __launch_bounds__(kThreads) k_sum_i64(const int64_t *a, int64_t n, unsigned long long *res)
{
    __shared__ unsigned long long w[kWaves];
    unsigned long long t = 0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        t += (unsigned long long)a[i];
    for (int d = 32; d > 0; d >>= 1) t += __shfl_xor(t, d, 64);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kWaves; ++k) t += w[k];
        atomicAdd(res, t);
    }
}

__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }
__global__ void k_set_u64(unsigned long long *p, unsigned long long v) { *p = v; }

// *res = max of a[0..n) (n >= 1)
inline void reduce_max(const int32_t *a, int64_t n, int32_t *res, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, res, (int32_t)INT32_MIN);
    hipLaunchKernelGGL(k_max_i32, dim3(std::min<unsigned>(blocks(n), 1024)), dim3(kThreads), 0, s, a, n, res);
}

// *res = sum of the non-negative a[0..n)
inline void reduce_sum(const int64_t *a, int64_t n, int64_t *res, hipStream_t s)
{
    unsigned long long *r = reinterpret_cast<unsigned long long *>(res);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, r, 0ull);
    hipLaunchKernelGGL(k_sum_i64, dim3(std::min<unsigned>(blocks(n), 1024)), dim3(kThreads), 0, s, a, n, r);
}

}  // namespace prim
}  // namespace dmk
