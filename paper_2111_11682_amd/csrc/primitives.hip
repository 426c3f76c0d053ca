// Device-wide building blocks: exclusive scan, stable LSD radix sort, bin
// counting and fills.  Used by the layout (ingest) and by the banding step of
// the neighbour search; not on the per-rating SGD path.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.hpp"

namespace lshmf {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char* what)
{
    set_error("%s: %s", what, hipGetErrorString(e));
    return LSHMF_EDEVICE;
}

const char* last_error() { return g_err; }

// ------------------------------------------------------------------ fills
template <typename T>
__global__ void k_fill(T* p, int64_t n, T v)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        p[x] = v;
}

template <typename T>
static int fill(T* p, int64_t n, T v, hipStream_t s)
{
    if (n <= 0) return LSHMF_OK;
    int64_t blocks = ceil_div(n, 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    LSHMF_LAUNCHED("k_fill");
    return LSHMF_OK;
}

int fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) { return fill(p, n, v, s); }
int fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) { return fill(p, n, v, s); }
int fill_f32(float* p, int64_t n, float v, hipStream_t s) { return fill(p, n, v, s); }

// ------------------------------------------------------------------- scan
// One workgroup of 256 threads scans a tile of 1024 values (4 per thread).
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int64_t wave_incl_scan(int64_t v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int64_t y = __shfl_up(v, o, kWave);
        if (lane >= o) v += y;
    }
    return v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const int64_t* in, int64_t* out,
                                                            int64_t n, int64_t* sums)
{
    __shared__ int64_t wsum[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t local = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        local += v[k];
    }
    int64_t incl = wave_incl_scan(local);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    int64_t wprefix = 0;
    for (int w = 0; w < wave; ++w) wprefix += wsum[w];
    int64_t run = wprefix + incl - local;   // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) {
        int64_t tot = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) tot += wsum[w];
        sums[blockIdx.x] = tot;
    }
}

__global__ void k_scan_add(int64_t* out, int64_t n, const int64_t* offs)
{
    const int64_t x = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t y = x + (int64_t)k * kScanThreads;
        if (y < n) out[y] += offs[blockIdx.x];
    }
}

__global__ void k_set_total(int64_t* out, int64_t n, const int64_t* sums_scanned, int64_t nb)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = sums_scanned[nb];
}

size_t scan_tmp_elems(int64_t n)
{
    size_t tot = 0;
    while (n > 1) {
        const int64_t nb = ceil_div(n, kScanTile);
        tot += (size_t)nb + 1;
        n = nb;
    }
    return tot + 2;
}

int scan_excl(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s)
{
    if (n <= 0) {
        hipLaunchKernelGGL(k_fill<int64_t>, dim3(1), dim3(1), 0, s, out, (int64_t)1, (int64_t)0);
        LSHMF_LAUNCHED("k_fill(scan total)");
        return LSHMF_OK;
    }
    const int64_t nb = ceil_div(n, kScanTile);
    int64_t* sums = tmp;            // nb + 1 entries, scanned recursively in place
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, sums);
    LSHMF_LAUNCHED("k_scan_tile");
    if (nb == 1) {  // sums[0] is the total
        hipLaunchKernelGGL(k_set_total, dim3(1), dim3(1), 0, s, out, n, sums, (int64_t)0);
        LSHMF_LAUNCHED("k_set_total");
        return LSHMF_OK;
    }
    LSHMF_TRY(scan_excl(sums, sums, nb, tmp + nb + 1, s));
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, n, sums);
    LSHMF_LAUNCHED("k_scan_add");
    hipLaunchKernelGGL(k_set_total, dim3(1), dim3(1), 0, s, out, n, sums, nb);
    LSHMF_LAUNCHED("k_set_total");
    return LSHMF_OK;
}

// ------------------------------------------------------------- radix sort
// 8-bit digits; a tile of 4096 keys per 256-thread workgroup.
constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kRsBins = 256;

size_t radix_hist_elems(int64_t n) { return (size_t)ceil_div(n, kRsTile) * kRsBins + 1; }

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t* keys, int64_t n, int shift,
                                                        int64_t* hist, int64_t ntiles)
{
    __shared__ int cnt[kRsBins];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t x = base + (int64_t)k * kRsThreads + threadIdx.x;
        if (x < n) atomicAdd(&cnt[(keys[x] >> shift) & (kRsBins - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one tile.  Wave w ranks keys [w * 1024, (w + 1) * 1024) of
// the tile in rounds of 64: lanes with equal digits find each other with 8
// ballots, and a key's rank among its wave's equal digits is the wave's count
// so far plus the lanes below it.  The tile is then sorted by digit in LDS
// (digit start + earlier waves' counts + rank) and written out in that order,
// so a digit's keys of the tile go to consecutive addresses.
constexpr int kRsRounds = kRsTile / (kRsThreads / kWave) / kWave;  // rounds of 64 keys per wave

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t* kin, const uint32_t* vin,
                                                           uint64_t* kout, uint32_t* vout, int64_t n,
                                                           int shift, const int64_t* offs,
                                                           int64_t ntiles)
{
    constexpr int kWaves = kRsThreads / kWave;
    __shared__ uint64_t skey[kRsTile];
    __shared__ uint32_t sval[kRsTile];
    __shared__ int wcnt[kWaves][kRsBins];  // per wave: digit counts, then the digit's first slot
    __shared__ int lstart[kRsBins];        // first slot of each digit in the sorted tile
    __shared__ int wsum[kWaves];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * kRsTile;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    uint64_t key[kRsRounds];
    uint32_t val[kRsRounds];
    int rank[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t x = tile0 + (int64_t)wave * (kRsRounds * kWave) + r * kWave + lane;
        const bool valid = x < n;
        key[r] = valid ? kin[x] : 0ull;
        val[r] = valid ? vin[x] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t x = tile0 + (int64_t)wave * (kRsRounds * kWave) + r * kWave + lane;
        const bool valid = x < n;
        const int d = (int)((key[r] >> shift) & (kRsBins - 1));
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot(valid && ((d >> b) & 1));
            same &= ((d >> b) & 1) ? bal : ~bal;
        }
        const int below = __popcll(same & lt_mask);
        const int before = valid ? wcnt[wave][d] : 0;  // read by all lanes before the leader adds
        rank[r] = before + below;
        if (valid && below == 0) wcnt[wave][d] = before + __popcll(same);
    }
    __syncthreads();
    // thread tid = digit: the tile's count, its first slot (scan over digits)
    // and each wave's first slot within the digit
    int tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) tot += wcnt[w][tid];
    int incl = tot;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    int start = incl - tot;
    for (int w = 0; w < wave; ++w) start += wsum[w];
    lstart[tid] = start;
    int acc = start;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int c = wcnt[w][tid];
        wcnt[w][tid] = acc;
        acc += c;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t x = tile0 + (int64_t)wave * (kRsRounds * kWave) + r * kWave + lane;
        if (x < n) {
            const int d = (int)((key[r] >> shift) & (kRsBins - 1));
            const int pos = wcnt[wave][d] + rank[r];
            skey[pos] = key[r];
            sval[pos] = val[r];
        }
    }
    __syncthreads();
    const int64_t tile_n = n - tile0 < kRsTile ? n - tile0 : kRsTile;
    for (int p = tid; p < tile_n; p += kRsThreads) {
        const uint64_t k = skey[p];
        const int d = (int)((k >> shift) & (kRsBins - 1));
        const int64_t g = offs[(int64_t)d * ntiles + blockIdx.x] + (p - lstart[d]);
        kout[g] = k;
        vout[g] = sval[p];
    }
}

int radix_sort(uint64_t* keys[2], uint32_t* vals[2], int64_t n, int bits, int64_t* hist,
               int64_t* scan_tmp, hipStream_t s, int* result_index)
{
    int cur = 0;
    if (n > 1) {
        const int64_t ntiles = ceil_div(n, kRsTile);
        for (int shift = 0; shift < bits; shift += 8) {
            hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(kRsThreads), 0, s, keys[cur],
                               n, shift, hist, ntiles);
            LSHMF_LAUNCHED("k_rs_hist");
            LSHMF_TRY(scan_excl(hist, hist, ntiles * kRsBins, scan_tmp, s));
            hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(kRsThreads), 0, s,
                               keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1], n, shift, hist,
                               ntiles);
            LSHMF_LAUNCHED("k_rs_scatter");
            cur ^= 1;
        }
    }
    *result_index = cur;
    return LSHMF_OK;
}

// --------------------------------------------------------------- counting
// Up to kCountLds bins per window: every workgroup counts its share of the
// input in LDS (so the ratings of a popular item do not queue on one global
// counter) and adds its non-zero bins to the global counts.  Larger ranges
// (users, blocks) count with global atomics after merging runs of equal
// consecutive ids inside each wave (inputs grouped by user give one atomic
// per run).
constexpr int kCountLds = 16384;
constexpr int kCountThreads = 256;

__global__ __launch_bounds__(kCountThreads) void k_count_lds(const int32_t* idx, int64_t n, int64_t nbins,
                                                             unsigned long long* cnt)
{
    __shared__ uint32_t h[kCountLds];
    const int64_t lo = (int64_t)blockIdx.y * kCountLds;
    const int64_t width = nbins - lo < kCountLds ? nbins - lo : kCountLds;
    for (int x = threadIdx.x; x < width; x += kCountThreads) h[x] = 0;
    __syncthreads();
    for (int64_t x = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * kCountThreads) {
        const int64_t b = (int64_t)idx[x] - lo;
        if (b >= 0 && b < width) atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < width; x += kCountThreads)
        if (h[x]) atomicAdd(&cnt[lo + x], (unsigned long long)h[x]);
}

__global__ void k_count(const int32_t* idx, int64_t n, unsigned long long* cnt)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // whole waves step together so that every lane takes part in the ballots
    for (int64_t x0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x - lane; x0 < n; x0 += stride) {
        const int64_t x = x0 + lane;
        const bool valid = x < n;
        const int32_t v = valid ? idx[x] : -1;
        const int32_t prev = __shfl_up(v, 1, kWave);
        const bool head = valid && (lane == 0 || prev != v);
        const uint64_t heads = __ballot(head);
        const uint64_t vmask = __ballot(valid);     // a prefix of the wave
        if (head) {
            const uint64_t above = lane == kWave - 1 ? 0ull : heads >> (lane + 1) << (lane + 1);
            const int end = above ? __ffsll((unsigned long long)above) - 1 : 64 - __clzll((long long)vmask);
            atomicAdd(&cnt[v], (unsigned long long)(end - lane));
        }
    }
}

int count_bins(const int32_t* idx, int64_t n, int64_t* cnt, int64_t nbins, hipStream_t s)
{
    LSHMF_TRY(fill_i64(cnt, nbins, 0, s));
    if (n <= 0) return LSHMF_OK;
    if (nbins <= 4 * kCountLds) {
        int64_t blocks = ceil_div(n, 16 * kCountThreads);
        if (blocks > 512) blocks = 512;
        const unsigned windows = (unsigned)ceil_div(nbins, kCountLds);
        hipLaunchKernelGGL(k_count_lds, dim3((unsigned)blocks, windows), dim3(kCountThreads), 0, s, idx, n, nbins,
                           (unsigned long long*)cnt);
        LSHMF_LAUNCHED("k_count_lds");
        return LSHMF_OK;
    }
    int64_t blocks = ceil_div(n, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_count, dim3((unsigned)blocks), dim3(256), 0, s, idx, n,
                       (unsigned long long*)cnt);
    LSHMF_LAUNCHED("k_count");
    return LSHMF_OK;
}

}  // namespace lshmf
