// Ingest and layout of the training ratings.
//
// From the COO triplets this builds, all on the device:
//   * CSR by user (items ascending)   -- R(i) membership for Eq. (rr)
//   * CSC by item (users ascending)   -- the per-item sums of Eq. (item_hash)
//   * the stratified block stream     -- the SGD order (see sgd_epoch in lshmf.h)
//     with per-block ranges, item segments and, for every rating, the
//     previous rating of the same user inside its block (the only ordering
//     constraint between the waves that share a block)
//   * mu, b0_i, bh0_j: the "simple case" means of Sec. 3.2, exact integer sums
//     reduced and divided in FP64.
#include "common.hpp"

namespace lshmf {

__global__ void k_check_ids(const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n,
                            int32_t M, int32_t N, int32_t* err)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        if (u[x] < 0 || u[x] >= M || it[x] < 0 || it[x] >= N || rc[x] == 0 || rc[x] > 15)
            atomicOr(err, 1);
    }
}

// key = user * N + item  (CSR order)  or  item * M + user  (CSC order)
__global__ void k_keys_pair(const int32_t* major, const int32_t* minor, int64_t n, int64_t nminor,
                            uint64_t* keys, uint32_t* vals)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        keys[x] = (uint64_t)major[x] * (uint64_t)nminor + (uint64_t)minor[x];
        vals[x] = (uint32_t)x;
    }
}

struct StratKey {
    int64_t P, MP, NP;  // strata, ceil(M/P), ceil(N/P)
};

// Stream order: (stratum s, block b, item j, user i).  Users i = b mod P and
// items j = (b+s) mod P inside a block, so (s, b, j/P, i/P) orders the same.
__global__ void k_keys_stream(const int32_t* u, const int32_t* it, int64_t n, StratKey sk,
                              uint64_t* keys, uint32_t* vals)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = u[x], j = it[x];
        const int64_t rb = i % sk.P, cb = j % sk.P;
        const int64_t s = (cb - rb + sk.P) % sk.P;
        const uint64_t blk = (uint64_t)(s * sk.P + rb);
        keys[x] = ((blk * (uint64_t)sk.NP + (uint64_t)(j / sk.P)) * (uint64_t)sk.MP) + (uint64_t)(i / sk.P);
        vals[x] = (uint32_t)x;
    }
}

__device__ inline int64_t block_of(int64_t i, int64_t j, int64_t P)
{
    const int64_t rb = i % P, cb = j % P;
    return ((cb - rb + P) % P) * P + rb;
}

// After the stream sort: packed (user, code), item, block id, edge -> position.
__global__ void k_stream_fill(const uint32_t* order, const int32_t* u, const int32_t* it,
                              const uint8_t* rc, int64_t n, int64_t P, uint32_t* pk, int32_t* sj,
                              int32_t* blk_of_pos, int32_t* e2s)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = order[p];
        const int32_t i = u[e], j = it[e];
        pk[p] = ((uint32_t)i << 4) | (uint32_t)rc[e];
        sj[p] = j;
        blk_of_pos[p] = (int32_t)block_of(i, j, P);
        e2s[e] = (int32_t)p;
    }
}

// A segment starts where the block or the item changes.
__global__ void k_seg_flags(const int32_t* sj, const int32_t* blk_of_pos, int64_t n, int64_t* flag)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        flag[p] = (p == 0 || sj[p] != sj[p - 1] || blk_of_pos[p] != blk_of_pos[p - 1]) ? 1 : 0;
}

__global__ void k_seg_fill(const int32_t* sj, const int32_t* blk_of_pos, const int64_t* ex, int64_t n,
                           int32_t* seg_col, int64_t* seg_start)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const bool start = (p == 0 || sj[p] != sj[p - 1] || blk_of_pos[p] != blk_of_pos[p - 1]);
        if (start) {
            seg_col[ex[p]] = sj[p];
            seg_start[ex[p]] = p;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) seg_start[ex[n]] = n;
}

__global__ void k_blk_seg(const int64_t* blk_ptr, const int64_t* ex, int64_t nblk, int64_t n,
                          int64_t* blk_seg)
{
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b <= nblk;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = blk_ptr[b];
        blk_seg[b] = (p < n) ? ex[p] : ex[n];
    }
}

// Dependency order: (s, b, user i, item j); value = stream position.
__global__ void k_keys_dep(const int32_t* u, const int32_t* it, const int32_t* e2s, int64_t n,
                           StratKey sk, uint64_t* keys, uint32_t* vals)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = u[x], j = it[x];
        const uint64_t blk = (uint64_t)block_of(i, j, sk.P);
        keys[x] = ((blk * (uint64_t)sk.MP + (uint64_t)(i / sk.P)) * (uint64_t)sk.NP) + (uint64_t)(j / sk.P);
        vals[x] = (uint32_t)e2s[x];
    }
}

__global__ void k_dep_fill(const uint64_t* keys, const uint32_t* pos, int64_t n, int64_t NP,
                           const int32_t* blk_of_pos, const int64_t* blk_ptr, int32_t* dep)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = pos[x];
        int32_t d = -1;
        if (x > 0 && keys[x] / (uint64_t)NP == keys[x - 1] / (uint64_t)NP)
            d = (int32_t)((int64_t)pos[x - 1] - blk_ptr[blk_of_pos[p]]);
        dep[p] = d;
    }
}

// CSR / CSC payloads after their sorts.
__global__ void k_gather_pair(const uint32_t* order, const int32_t* other, const uint8_t* rc,
                              int64_t n, int32_t* out_idx, uint8_t* out_rc, const int32_t* e2s,
                              int32_t* out_spos)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = order[x];
        out_idx[x] = other[e];
        out_rc[x] = rc[e];
        if (out_spos) out_spos[x] = e2s[e];
    }
}

// ---------------------------------------------------------------- baselines
__global__ void k_sum_codes(const uint8_t* rc, int64_t n, unsigned long long* total)
{
    unsigned long long s = 0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        s += rc[x];
    // integer sums are exact and order-free
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_down(s, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(total, s);
}

__global__ void k_mu(const unsigned long long* total, int64_t n, int rscale, double* mu)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *mu = (double)(*total) / ((double)rscale * (double)n);
}

// One wave per row of a compressed matrix: b = mean(row)/rscale - mu (0 if empty).
__global__ void k_row_means(const int64_t* ptr, const uint8_t* rc, int64_t rows, int rscale,
                            const double* mu, float* out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t r = wave0; r < rows; r += nwaves) {
        const int64_t a = ptr[r], z = ptr[r + 1];
        unsigned long long s = 0;
        for (int64_t x = a + lane; x < z; x += kWave) s += rc[x];
        for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_down(s, o, kWave);
        if (lane == 0)
            out[r] = (z > a) ? (float)((double)s / ((double)rscale * (double)(z - a)) - *mu) : 0.0f;
    }
}

static unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 16384)
{
    int64_t b = ceil_div(n > 0 ? n : 1, threads);
    return (unsigned)(b > cap ? cap : b);
}

int ingest(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n,
           hipStream_t s)
{
    const lshmf_dims& d = c->d;
    const int64_t P = c->P;
    const StratKey sk{P, ceil_div(d.M, P), ceil_div(d.N, P)};
    int ri = 0;

    LSHMF_TRY(fill_i32(c->err, 2, 0, s));
    hipLaunchKernelGGL(k_check_ids, dim3(grid_for(n)), dim3(256), 0, s, u, it, rc, n, d.M, d.N, c->err);
    LSHMF_LAUNCHED("k_check_ids");
    int32_t herr = 0;
    LSHMF_HIP(hipMemcpyAsync(&herr, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LSHMF_HIP(hipStreamSynchronize(s));
    if (herr) {
        set_error("ingest: a rating has a user outside [0,%d), an item outside [0,%d) or a code "
                  "outside 1..15", d.M, d.N);
        return LSHMF_EINVAL;
    }

    // -- stratified block stream
    int32_t* e2s = c->csr_spos;       // reused: edge -> stream position (nnz int32)
    int32_t* blk_of_pos = c->seg_col; // reused until segments are written
    hipLaunchKernelGGL(k_keys_stream, dim3(grid_for(n)), dim3(256), 0, s, u, it, n, sk, c->sk[0], c->sv[0]);
    LSHMF_LAUNCHED("k_keys_stream");
    const int sbits = bits_for((uint64_t)(P * P) * (uint64_t)sk.NP * (uint64_t)sk.MP);
    LSHMF_TRY(radix_sort(c->sk, c->sv, n, sbits, c->hist, c->scan_tmp, s, &ri));
    // the dependency arrays below need e2s, and blk_of_pos lives in seg_col:
    // keep blk_of_pos in the cnt region instead (int64 sized, cast to int32)
    int32_t* bop = reinterpret_cast<int32_t*>(c->cnt);
    (void)blk_of_pos;
    hipLaunchKernelGGL(k_stream_fill, dim3(grid_for(n)), dim3(256), 0, s, c->sv[ri], u, it, rc, n, P,
                       c->pk, c->sj, bop, e2s);
    LSHMF_LAUNCHED("k_stream_fill");
    // block pointers
    LSHMF_TRY(count_bins(bop, n, c->blk_seg, P * P, s));       // blk_seg as a temporary
    LSHMF_TRY(scan_excl(c->blk_seg, c->blk_ptr, P * P, c->scan_tmp, s));
    // segments: flags in seg_start (int64, nnz+1 entries), scanned in place
    hipLaunchKernelGGL(k_seg_flags, dim3(grid_for(n)), dim3(256), 0, s, c->sj, bop, n, c->seg_start);
    LSHMF_LAUNCHED("k_seg_flags");
    int64_t* ex = reinterpret_cast<int64_t*>(c->sk[ri ^ 1]);  // free sort buffer, n+1 int64
    LSHMF_TRY(scan_excl(c->seg_start, ex, n, c->scan_tmp, s));
    hipLaunchKernelGGL(k_seg_fill, dim3(grid_for(n)), dim3(256), 0, s, c->sj, bop, ex, n, c->seg_col,
                       c->seg_start);
    LSHMF_LAUNCHED("k_seg_fill");
    hipLaunchKernelGGL(k_blk_seg, dim3(grid_for(P * P + 1)), dim3(256), 0, s, c->blk_ptr, ex, P * P, n,
                       c->blk_seg);
    LSHMF_LAUNCHED("k_blk_seg");
    // dependencies: previous rating of the same user inside the block
    hipLaunchKernelGGL(k_keys_dep, dim3(grid_for(n)), dim3(256), 0, s, u, it, e2s, n, sk, c->sk[0], c->sv[0]);
    LSHMF_LAUNCHED("k_keys_dep");
    LSHMF_TRY(radix_sort(c->sk, c->sv, n, sbits, c->hist, c->scan_tmp, s, &ri));
    hipLaunchKernelGGL(k_dep_fill, dim3(grid_for(n)), dim3(256), 0, s, c->sk[ri], c->sv[ri], n, sk.NP,
                       bop, c->blk_ptr, c->dep);
    LSHMF_LAUNCHED("k_dep_fill");

    // -- CSR by user, with the stream position of each rating
    hipLaunchKernelGGL(k_keys_pair, dim3(grid_for(n)), dim3(256), 0, s, u, it, n, (int64_t)d.N, c->sk[0], c->sv[0]);
    LSHMF_LAUNCHED("k_keys_pair(csr)");
    LSHMF_TRY(radix_sort(c->sk, c->sv, n, bits_for((uint64_t)d.M * (uint64_t)d.N), c->hist, c->scan_tmp, s, &ri));
    // e2s is read while csr_spos (the same memory) is written: stage e2s first
    int32_t* e2s_copy = reinterpret_cast<int32_t*>(c->sk[ri ^ 1]);
    LSHMF_HIP(hipMemcpyAsync(e2s_copy, e2s, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_gather_pair, dim3(grid_for(n)), dim3(256), 0, s, c->sv[ri], it, rc, n, c->csr_col,
                       c->csr_rc, e2s_copy, c->csr_spos);
    LSHMF_LAUNCHED("k_gather_pair(csr)");
    LSHMF_TRY(count_bins(u, n, c->cnt, d.M, s));
    LSHMF_TRY(scan_excl(c->cnt, c->row_ptr, d.M, c->scan_tmp, s));

    // -- CSC by item
    hipLaunchKernelGGL(k_keys_pair, dim3(grid_for(n)), dim3(256), 0, s, it, u, n, (int64_t)d.M, c->sk[0], c->sv[0]);
    LSHMF_LAUNCHED("k_keys_pair(csc)");
    LSHMF_TRY(radix_sort(c->sk, c->sv, n, bits_for((uint64_t)d.M * (uint64_t)d.N), c->hist, c->scan_tmp, s, &ri));
    hipLaunchKernelGGL(k_gather_pair, dim3(grid_for(n)), dim3(256), 0, s, c->sv[ri], u, rc, n, c->csc_row,
                       c->csc_rc, nullptr, nullptr);
    LSHMF_LAUNCHED("k_gather_pair(csc)");
    LSHMF_TRY(count_bins(it, n, c->cnt, d.N, s));
    LSHMF_TRY(scan_excl(c->cnt, c->col_ptr, d.N, c->scan_tmp, s));

    // -- baselines (Sec. 3.2, simple case), FP64
    unsigned long long* total = reinterpret_cast<unsigned long long*>(c->cnt);
    LSHMF_TRY(fill_i64(c->cnt, 1, 0, s));
    hipLaunchKernelGGL(k_sum_codes, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, rc, n, total);
    LSHMF_LAUNCHED("k_sum_codes");
    hipLaunchKernelGGL(k_mu, dim3(1), dim3(64), 0, s, total, n, d.rscale, c->t.mu);
    LSHMF_LAUNCHED("k_mu");
    hipLaunchKernelGGL(k_row_means, dim3(grid_for((int64_t)d.M * kWave)), dim3(256), 0, s, c->row_ptr,
                       c->csr_rc, (int64_t)d.M, d.rscale, c->t.mu, c->t.b0);
    LSHMF_LAUNCHED("k_row_means(users)");
    hipLaunchKernelGGL(k_row_means, dim3(grid_for((int64_t)d.N * kWave)), dim3(256), 0, s, c->col_ptr,
                       c->csc_rc, (int64_t)d.N, d.rscale, c->t.mu, c->t.bh0);
    LSHMF_LAUNCHED("k_row_means(items)");

    // largest block, for the LDS capacity check of the SGD kernel
    int64_t* hptr = new int64_t[P * P + 1];
    hipError_t e = hipMemcpyAsync(hptr, c->blk_ptr, sizeof(int64_t) * (P * P + 1), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete[] hptr;
        return hip_fail(e, "ingest: block pointers");
    }
    int64_t mx = 0;
    for (int64_t b = 0; b < P * P; ++b) mx = hptr[b + 1] - hptr[b] > mx ? hptr[b + 1] - hptr[b] : mx;
    delete[] hptr;
    c->max_block_nnz = mx;
    return LSHMF_OK;
}

}  // namespace lshmf
