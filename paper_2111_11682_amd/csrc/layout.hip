// Ingest and layout of the ratings.
//
// All on the device:
//   * the rating store (COO), which online updates append to;
//   * CSR by user (items ascending)   -- R(i) membership for Eq. (rr)
//   * CSC by item (users ascending)   -- the per-item sums of Eq. (item_hash)
//   * stratified streams              -- the SGD order (see sgd_epoch in lshmf.h)
//     with per-block ranges, item runs and, for every rating, its place in
//     the chain of the same user's ratings inside its block (the only
//     ordering constraint between the waves that share a block);
//   * mu, b0_i, bh0_j: the "simple case" means of Sec. 3.2, exact integer sums
//     reduced and divided in FP64.
#include <utility>

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

// A (user, item) pair given twice: adjacent equal keys after a sort by pair.
__global__ void k_dup_flags(const uint64_t* keys, int64_t n, int32_t* err)
{
    for (int64_t x = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        if (keys[x] == keys[x - 1]) atomicOr(err, 2);
}

// A batch pair (u, i) already in the store: binary search of i in the CSR
// row of u (users >= M_old have no row yet).
__global__ void k_in_store(const int32_t* u, const int32_t* it, int64_t n, int32_t M_old, const int64_t* row_ptr,
                           const int32_t* col, int32_t* err)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = u[x], j = it[x];
        if (i < 0 || i >= M_old || j < 0) continue;  // out-of-range ids are reported apart
        int64_t l = row_ptr[i], r = row_ptr[i + 1];
        while (l < r) {
            const int64_t m = (l + r) >> 1;
            if (col[m] < j) l = m + 1;
            else r = m;
        }
        if (l < row_ptr[i + 1] && col[l] == j) atomicOr(err, 4);
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
    int64_t P, MP, N, M;  // strata, ceil(M/P), items, users
};

// Stream order: (stratum s, block b, item rank, user rank), where a rank
// orders items (users) by decreasing degree within the stream's ratings, then
// id.  Heavy users come first in every item run, so the chains of their many
// ratings in a block start early.
__global__ void k_keys_stream(const int32_t* u, const int32_t* it, const int32_t* rank, const int32_t* urank,
                              int64_t n, StratKey sk, uint64_t* keys, uint32_t* vals)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = u[x], j = it[x];
        const int64_t rb = i % sk.P, cb = j % sk.P;
        const int64_t s = (cb - rb + sk.P) % sk.P;
        const uint64_t blk = (uint64_t)(s * sk.P + rb);
        keys[x] = ((blk * (uint64_t)sk.N + (uint64_t)rank[j]) * (uint64_t)sk.M) + (uint64_t)urank[i];
        vals[x] = (uint32_t)x;
    }
}

// Items (or users) by (degree in the stream desc, id asc): key = (n - deg) * 2^idbits + j.
__global__ void k_keys_rank(const int64_t* deg, int32_t N, int64_t n, int idbits, uint64_t* keys,
                            uint32_t* vals)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x) {
        keys[j] = ((uint64_t)(n - deg[j]) << idbits) | (uint64_t)j;
        vals[j] = (uint32_t)j;
    }
}

__global__ void k_rank_fill(const uint32_t* order, int32_t N, int32_t* rank)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < N;
         x += (int64_t)gridDim.x * blockDim.x)
        rank[order[x]] = (int32_t)x;
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

// Dependency order: (s, b, user i, item rank); value = stream position.
__global__ void k_keys_dep(const int32_t* u, const int32_t* it, const int32_t* rank, const int32_t* e2s,
                           int64_t n, StratKey sk, uint64_t* keys, uint32_t* vals)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = u[x], j = it[x];
        const uint64_t blk = (uint64_t)block_of(i, j, sk.P);
        keys[x] = ((blk * (uint64_t)sk.MP + (uint64_t)(i / sk.P)) * (uint64_t)sk.N) + (uint64_t)rank[j];
        vals[x] = (uint32_t)e2s[x];
    }
}

__device__ inline bool same_user_block(const uint64_t* keys, int64_t a, int64_t b, int64_t N)
{
    return keys[a] / (uint64_t)N == keys[b] / (uint64_t)N;
}

// A user with several ratings in a block gets a mailbox slot in that block:
// flag the first rating of each such chain (in (block, user, item rank) order).
__global__ void k_chain_flags(const uint64_t* keys, int64_t n, int64_t N, int64_t* flag)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const bool pred = x > 0 && same_user_block(keys, x, x - 1, N);
        const bool succ = x + 1 < n && same_user_block(keys, x, x + 1, N);
        flag[x] = (!pred && succ) ? 1 : 0;
    }
}

// dep[p]: local index (inside the block) of the previous rating of the same
// user, or -1.  link[p] drives the SGD kernel's hand-over of user rows
// between waves: bit 31 = a later rating of the user follows in the block,
// bit 30 = an earlier one precedes, bits 16..29 = position in the user's
// chain, bits 0..15 = the chain's mailbox slot in the block.
__global__ void k_dep_fill(const uint64_t* keys, const uint32_t* pos, int64_t n, int64_t N,
                           const int32_t* blk_of_pos, const int64_t* blk_ptr, const int64_t* ex, int32_t* dep,
                           uint32_t* link)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = pos[x];
        const int64_t blk = blk_of_pos[p];
        const bool pred = x > 0 && same_user_block(keys, x, x - 1, N);
        const bool succ = x + 1 < n && same_user_block(keys, x, x + 1, N);
        int64_t q = 0;
        while (x - q > 0 && same_user_block(keys, x - q, x - q - 1, N)) ++q;
        dep[p] = pred ? (int32_t)((int64_t)pos[x - 1] - blk_ptr[blk]) : -1;
        uint32_t lk = 0;
        if (pred || succ) {
            const int64_t slot = ex[x - q] - ex[blk_ptr[blk]];
            lk = (succ ? 0x80000000u : 0u) | (pred ? 0x40000000u : 0u) | ((uint32_t)q << 16) | (uint32_t)slot;
        }
        link[p] = lk;
    }
}

// mailbox slots used by each block
// Dispatch order of the blocks of each stratum: key (stratum, ratings desc,
// block id asc), so that a stratum's heaviest blocks start first.
__global__ void k_keys_blkorder(const int64_t* blk_ptr, int64_t P, int pb, uint64_t* keys, uint32_t* vals)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < P * P;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t st = (uint64_t)(x / P), b = (uint64_t)(x % P);
        const int64_t nnz = blk_ptr[x + 1] - blk_ptr[x];
        const uint64_t wgt = nnz > 0xFFFFFFFFLL ? 0xFFFFFFFFull : (uint64_t)nnz;
        keys[x] = (st << (32 + pb)) | ((0xFFFFFFFFull - wgt) << pb) | b;
        vals[x] = (uint32_t)b;
    }
}

// Per stratum, the blocks with more than kLightNnz ratings and the blocks with
// any: both come first in the dispatch order (ratings descending), so binary
// searches over it find where they end.
__global__ void k_heavy_count(const int64_t* blk_ptr, const int32_t* blk_order, int64_t P, int32_t* heavy)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < P; s += (int64_t)gridDim.x * blockDim.x) {
        for (int h = 0; h < 2; ++h) {
            const int64_t above = h == 0 ? kLightNnz : 0;
            int64_t lo = 0, hi = P;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                const int64_t b = s * P + blk_order[s * P + mid];
                if (blk_ptr[b + 1] - blk_ptr[b] > above) lo = mid + 1;
                else hi = mid;
            }
            heavy[h * P + s] = (int32_t)lo;
        }
    }
}

// The runs of the block at each dispatch position, read by the SGD kernel in
// one load instead of two dependent ones (dispatch order, then run range).
__global__ void k_block_runs(const int32_t* blk_order, const int64_t* blk_seg, int64_t P, int32_t* blk_run)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < P * P;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = (x / P) * P + blk_order[x];
        blk_run[2 * x] = (int32_t)blk_seg[b];
        blk_run[2 * x + 1] = (int32_t)(blk_seg[b + 1] - blk_seg[b]);
    }
}

__global__ void k_block_slots(const int64_t* blk_ptr, const int64_t* ex, int64_t nblk, int32_t* out)
{
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nblk;
         b += (int64_t)gridDim.x * blockDim.x)
        out[b] = (int32_t)(ex[blk_ptr[b + 1]] - ex[blk_ptr[b]]);
}

// CSR / CSC payloads after their sorts.
__global__ void k_gather_pair(const uint32_t* order, const int32_t* other, const uint8_t* rc,
                              int64_t n, int32_t* out_idx, uint8_t* out_rc)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = order[x];
        out_idx[x] = other[e];
        out_rc[x] = rc[e];
    }
}

// Fixed baselines of users / items first seen in an online batch: the mean
// of their batch ratings minus mu (existing ones keep theirs).
__global__ void k_sum_by_id(const int32_t* id, const uint8_t* rc, int64_t n, int32_t first,
                            unsigned long long* sum, unsigned long long* cnt)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = id[x];
        if (v >= first) {
            atomicAdd(&sum[v - first], (unsigned long long)rc[x]);
            atomicAdd(&cnt[v - first], 1ull);
        }
    }
}

__global__ void k_new_means(const unsigned long long* sum, const unsigned long long* cnt, int32_t count,
                            int rscale, const double* mu, float* out)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < count;
         x += (int64_t)gridDim.x * blockDim.x)
        out[x] = cnt[x] ? (float)((double)sum[x] / ((double)rscale * (double)cnt[x]) - *mu) : 0.0f;
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

// Largest block, most mailbox slots in a block and the number of item runs
// of a stream, for the SGD kernel's limits: stats[0..2] (zeroed before).
__global__ void k_stream_stats(const int64_t* blk_ptr, const int64_t* blk_seg, const int32_t* blk_slots,
                               int64_t nblk, int64_t* stats)
{
    unsigned long long mx = 0, msl = 0;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nblk;
         b += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long len = (unsigned long long)(blk_ptr[b + 1] - blk_ptr[b]);
        mx = len > mx ? len : mx;
        msl = (unsigned long long)blk_slots[b] > msl ? (unsigned long long)blk_slots[b] : msl;
    }
    atomicMax(reinterpret_cast<unsigned long long*>(stats), mx);
    atomicMax(reinterpret_cast<unsigned long long*>(stats + 1), msl);
    if (blockIdx.x == 0 && threadIdx.x == 0) stats[2] = blk_seg[nblk];
}

// Compressed rows after an online batch: row r of the merged copy holds the
// old row (rows r >= n_old are empty) and the batch's row, minor ids
// ascending.  new_ptr[r] = old_ptr[min(r, n_old)] + b_ptr[r].
__global__ void k_merged_ptr(const int64_t* old_ptr, int64_t n_old, const int64_t* b_ptr, int64_t n_new,
                             int64_t* new_ptr)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= n_new;
         r += (int64_t)gridDim.x * blockDim.x)
        new_ptr[r] = old_ptr[r < n_old ? r : n_old] + b_ptr[r];
}

// One wave per row: every element goes to its place in the merged row, found
// by a binary search in the other list (no pair is in both).
__global__ __launch_bounds__(256) void k_merge_rows(const int64_t* old_ptr, const int32_t* old_idx,
                                                    const uint8_t* old_rc, int64_t n_old, const int64_t* b_ptr,
                                                    const int32_t* b_idx, const uint8_t* b_rc, int64_t n_new,
                                                    const int64_t* new_ptr, int32_t* new_idx, uint8_t* new_rc)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t r = w0; r < n_new; r += nw) {
        const int64_t oa = old_ptr[r < n_old ? r : n_old];
        const int64_t oz = r < n_old ? old_ptr[r + 1] : oa;
        const int64_t ba = b_ptr[r], bz = b_ptr[r + 1];
        const int64_t base = new_ptr[r];
        for (int64_t x = oa + lane; x < oz; x += kWave) {
            const int32_t key = old_idx[x];
            int64_t l = ba, h = bz;
            while (l < h) {
                const int64_t m = (l + h) >> 1;
                if (b_idx[m] < key) l = m + 1;
                else h = m;
            }
            const int64_t dst = base + (x - oa) + (l - ba);
            new_idx[dst] = key;
            new_rc[dst] = old_rc[x];
        }
        for (int64_t y = ba + lane; y < bz; y += kWave) {
            const int32_t key = b_idx[y];
            int64_t l = oa, h = oz;
            while (l < h) {
                const int64_t m = (l + h) >> 1;
                if (old_idx[m] < key) l = m + 1;
                else h = m;
            }
            const int64_t dst = base + (y - ba) + (l - oa);
            new_idx[dst] = key;
            new_rc[dst] = b_rc[y];
        }
    }
}

static unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 16384)
{
    int64_t b = ceil_div(n > 0 ? n : 1, threads);
    return (unsigned)(b > cap ? cap : b);
}

int sync_status(lshmf_ctx* c, hipStream_t s)
{
    int32_t herr = 0;
    LSHMF_HIP(hipMemcpyAsync(&herr, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LSHMF_HIP(hipStreamSynchronize(s));
    if (herr) {
        set_error("an SGD dependency wait gave up after its spin limit (status word %#x): a broken hand-over, "
                  "the tables do not follow the stated order", herr);
        return LSHMF_EDEVICE;
    }
    return LSHMF_OK;
}

// Reads the input-check word c->err[1] (bit 0 ids or codes out of range, bit 1
// a pair given twice, bit 2 a pair already in the store) after a
// synchronisation; reports the SGD status word as sync_status does.
int input_status(lshmf_ctx* c, int32_t M, int32_t N, hipStream_t s)
{
    int32_t herr[2] = {0, 0};
    LSHMF_HIP(hipMemcpyAsync(herr, c->err, sizeof(herr), hipMemcpyDeviceToHost, s));
    LSHMF_HIP(hipStreamSynchronize(s));
    if (herr[1] & 1) {
        set_error("a rating has a user outside [0,%d), an item outside [0,%d) or a code outside 1..15", M, N);
        return LSHMF_EINVAL;
    }
    if (herr[1] & 2) {
        set_error("a (user, item) pair is given twice");
        return LSHMF_EINVAL;
    }
    if (herr[1] & 4) {
        set_error("a (user, item) pair of the batch is already in the store");
        return LSHMF_EINVAL;
    }
    if (herr[0]) {
        set_error("an SGD dependency wait gave up after its spin limit (status word %#x): a broken hand-over, "
                  "the tables do not follow the stated order", herr[0]);
        return LSHMF_EDEVICE;
    }
    return LSHMF_OK;
}

int launch_id_checks(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n, int32_t M,
                     int32_t N, hipStream_t s, bool check_pairs = false);

int check_ids(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n, int32_t M,
              int32_t N, hipStream_t s)
{
    LSHMF_TRY(launch_id_checks(c, u, it, rc, n, M, N, s));
    return input_status(c, M, N, s);
}

// Launches the input checks of n ratings into c->err[1] (cleared first):
// ids and codes in range; with check_pairs also no pair twice and none in
// the store (the online batch).  The caller reads the word with input_status
// after a synchronisation.
int launch_id_checks(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n, int32_t M,
                     int32_t N, hipStream_t s, bool check_pairs)
{
    int32_t* flag = c->err + 1;  // a word of its own: c->err[0] is the SGD status word
    LSHMF_TRY(fill_i32(flag, 1, 0, s));
    if (n <= 0) return LSHMF_OK;
    hipLaunchKernelGGL(k_check_ids, dim3(grid_for(n)), dim3(256), 0, s, u, it, rc, n, M, N, flag);
    LSHMF_LAUNCHED("k_check_ids");
    if (!check_pairs) return LSHMF_OK;
    // keys of out-of-range ids are garbage but stay inside the sort buffers
    hipLaunchKernelGGL(k_keys_pair, dim3(grid_for(n)), dim3(256), 0, s, u, it, n, (int64_t)N, c->sk[0], c->sv[0]);
    LSHMF_LAUNCHED("k_keys_pair(batch)");
    int ri = 0;
    LSHMF_TRY(radix_sort(c->sk, c->sv, n, bits_for((uint64_t)M * (uint64_t)N), c->hist, c->scan_tmp, s, &ri));
    hipLaunchKernelGGL(k_dup_flags, dim3(grid_for(n)), dim3(256), 0, s, c->sk[ri], n, flag);
    LSHMF_LAUNCHED("k_dup_flags(batch)");
    hipLaunchKernelGGL(k_in_store, dim3(grid_for(n)), dim3(256), 0, s, u, it, n, c->M, c->row_ptr, c->csr_col, flag);
    LSHMF_LAUNCHED("k_in_store");
    return LSHMF_OK;
}

// Compressed copy of n ratings by `major` (ptr over n_major rows, minor ids
// ascending inside a row).
int compress(lshmf_ctx* c, const int32_t* major, const int32_t* minor, const uint8_t* rc, int64_t n,
             int64_t n_major, int64_t n_minor, int64_t* ptr, int32_t* idx, uint8_t* rc_out, hipStream_t s,
             int32_t* dup_flag)
{
    int ri = 0;
    if (n > 0) {
        hipLaunchKernelGGL(k_keys_pair, dim3(grid_for(n)), dim3(256), 0, s, major, minor, n, n_minor, c->sk[0],
                           c->sv[0]);
        LSHMF_LAUNCHED("k_keys_pair");
        LSHMF_TRY(radix_sort(c->sk, c->sv, n, bits_for((uint64_t)n_major * (uint64_t)n_minor), c->hist,
                             c->scan_tmp, s, &ri));
        if (dup_flag) {
            hipLaunchKernelGGL(k_dup_flags, dim3(grid_for(n)), dim3(256), 0, s, c->sk[ri], n, dup_flag);
            LSHMF_LAUNCHED("k_dup_flags");
        }
        hipLaunchKernelGGL(k_gather_pair, dim3(grid_for(n)), dim3(256), 0, s, c->sv[ri], minor, rc, n, idx, rc_out);
        LSHMF_LAUNCHED("k_gather_pair");
    }
    LSHMF_TRY(count_bins(major, n, c->cnt, n_major, s));
    return scan_excl(c->cnt, ptr, n_major, c->scan_tmp, s);
}

// CSR and CSC of the store's c->nnz ratings over c->M users and c->N items.
// dup_flag: a word that gets bit 1 when a pair occurs twice (or NULL).
int build_compressed(lshmf_ctx* c, hipStream_t s, int32_t* dup_flag)
{
    LSHMF_TRY(compress(c, c->coo_i, c->coo_u, c->coo_rc, c->nnz, c->N, c->M, c->col_ptr, c->csc_row, c->csc_rc, s,
                       nullptr));
    return compress(c, c->coo_u, c->coo_i, c->coo_rc, c->nnz, c->M, c->N, c->row_ptr, c->csr_col, c->csr_rc, s,
                    dup_flag);
}

// CSR and CSC of the store grown by a batch, merged from the previous copies
// and the batch's own CSR and CSC (no pair in both) into the second buffers,
// which then become current: O(store) copying, no sort of the store.
int merge_compressed(lshmf_ctx* c, int32_t M_old, int32_t N_old, const int64_t* b_rptr, const int32_t* b_col,
                     const uint8_t* b_rrc, const int64_t* b_cptr, const int32_t* b_row, const uint8_t* b_crc,
                     hipStream_t s)
{
    const int64_t M = c->M, N = c->N;
    hipLaunchKernelGGL(k_merged_ptr, dim3(grid_for(M + 1)), dim3(256), 0, s, c->row_ptr, (int64_t)M_old, b_rptr, M,
                       c->row_ptr_alt);
    LSHMF_LAUNCHED("k_merged_ptr(rows)");
    hipLaunchKernelGGL(k_merge_rows, dim3(grid_for(M * kWave)), dim3(256), 0, s, c->row_ptr, c->csr_col, c->csr_rc,
                       (int64_t)M_old, b_rptr, b_col, b_rrc, M, c->row_ptr_alt, c->csr_col_alt, c->csr_rc_alt);
    LSHMF_LAUNCHED("k_merge_rows(rows)");
    hipLaunchKernelGGL(k_merged_ptr, dim3(grid_for(N + 1)), dim3(256), 0, s, c->col_ptr, (int64_t)N_old, b_cptr, N,
                       c->col_ptr_alt);
    LSHMF_LAUNCHED("k_merged_ptr(cols)");
    hipLaunchKernelGGL(k_merge_rows, dim3(grid_for(N * kWave)), dim3(256), 0, s, c->col_ptr, c->csc_row, c->csc_rc,
                       (int64_t)N_old, b_cptr, b_row, b_crc, N, c->col_ptr_alt, c->csc_row_alt, c->csc_rc_alt);
    LSHMF_LAUNCHED("k_merge_rows(cols)");
    std::swap(c->row_ptr, c->row_ptr_alt);
    std::swap(c->csr_col, c->csr_col_alt);
    std::swap(c->csr_rc, c->csr_rc_alt);
    std::swap(c->col_ptr, c->col_ptr_alt);
    std::swap(c->csc_row, c->csc_row_alt);
    std::swap(c->csc_rc, c->csc_rc_alt);
    return LSHMF_OK;
}

// The stratified stream of n ratings (u, it, rc) over the current M x N,
// laid out on the device; its block statistics follow into st.stats.  The
// stream is usable after stream_finish (a synchronisation later).
int build_stream_async(lshmf_ctx* c, Stream& st, const int32_t* u, const int32_t* it, const uint8_t* rc,
                       int64_t n, hipStream_t s)
{
    if (n > st.cap) {
        set_error("a stream of %lld ratings exceeds its capacity %lld", (long long)n, (long long)st.cap);
        return LSHMF_ECAPACITY;
    }
    st.n = st.max_block_nnz = st.max_block_slots = st.nseg = st.pending = 0;
    st.codes = false;
    if (n == 0) return LSHMF_OK;
    const int64_t P = c->P;
    const StratKey sk{P, ceil_div(c->M, P), c->N, c->M};
    const int sbits = bits_for((uint64_t)(P * P)) + bits_for((uint64_t)sk.N) + bits_for((uint64_t)sk.M);
    if (sbits > 64) {
        set_error("stream sort key of %d bits: too many strata, items and users for 64 bits", sbits);
        return LSHMF_ECAPACITY;
    }
    int ri = 0;

    // item order inside blocks, then user order inside item runs: degree
    // within these ratings desc, id asc
    const int idbits = bits_for((uint64_t)c->N);
    LSHMF_TRY(count_bins(it, n, c->cnt, c->N, s));
    hipLaunchKernelGGL(k_keys_rank, dim3(grid_for(c->N)), dim3(256), 0, s, c->cnt, c->N, n, idbits, c->sk[0],
                       c->sv[0]);
    LSHMF_LAUNCHED("k_keys_rank");
    LSHMF_TRY(radix_sort(c->sk, c->sv, c->N, idbits + bits_for((uint64_t)n + 1), c->hist, c->scan_tmp, s, &ri));
    hipLaunchKernelGGL(k_rank_fill, dim3(grid_for(c->N)), dim3(256), 0, s, c->sv[ri], c->N, c->irank);
    LSHMF_LAUNCHED("k_rank_fill");
    const int ubits = bits_for((uint64_t)c->M);
    LSHMF_TRY(count_bins(u, n, c->cnt, c->M, s));
    hipLaunchKernelGGL(k_keys_rank, dim3(grid_for(c->M)), dim3(256), 0, s, c->cnt, c->M, n, ubits, c->sk[0],
                       c->sv[0]);
    LSHMF_LAUNCHED("k_keys_rank(users)");
    LSHMF_TRY(radix_sort(c->sk, c->sv, c->M, ubits + bits_for((uint64_t)n + 1), c->hist, c->scan_tmp, s, &ri));
    hipLaunchKernelGGL(k_rank_fill, dim3(grid_for(c->M)), dim3(256), 0, s, c->sv[ri], c->M, c->urank);
    LSHMF_LAUNCHED("k_rank_fill(users)");

    // stream order and block ranges
    int32_t* bop = reinterpret_cast<int32_t*>(c->cnt);       // block of each stream position
    hipLaunchKernelGGL(k_keys_stream, dim3(grid_for(n)), dim3(256), 0, s, u, it, c->irank, c->urank, n, sk,
                       c->sk[0], c->sv[0]);
    LSHMF_LAUNCHED("k_keys_stream");
    LSHMF_TRY(radix_sort(c->sk, c->sv, n, sbits, c->hist, c->scan_tmp, s, &ri));
    hipLaunchKernelGGL(k_stream_fill, dim3(grid_for(n)), dim3(256), 0, s, c->sv[ri], u, it, rc, n, P, st.pk,
                       st.sj, bop, c->e2s);
    LSHMF_LAUNCHED("k_stream_fill");
    LSHMF_TRY(count_bins(bop, n, st.blk_seg, P * P, s));       // blk_seg as a temporary
    LSHMF_TRY(scan_excl(st.blk_seg, st.blk_ptr, P * P, c->scan_tmp, s));
    // item runs inside blocks
    hipLaunchKernelGGL(k_seg_flags, dim3(grid_for(n)), dim3(256), 0, s, st.sj, bop, n, st.seg_start);
    LSHMF_LAUNCHED("k_seg_flags");
    int64_t* ex = reinterpret_cast<int64_t*>(c->sk[ri ^ 1]);  // free sort buffer, n+1 int64
    LSHMF_TRY(scan_excl(st.seg_start, ex, n, c->scan_tmp, s));
    hipLaunchKernelGGL(k_seg_fill, dim3(grid_for(n)), dim3(256), 0, s, st.sj, bop, ex, n, st.seg_col,
                       st.seg_start);
    LSHMF_LAUNCHED("k_seg_fill");
    hipLaunchKernelGGL(k_blk_seg, dim3(grid_for(P * P + 1)), dim3(256), 0, s, st.blk_ptr, ex, P * P, n,
                       st.blk_seg);
    LSHMF_LAUNCHED("k_blk_seg");
    // each user's chain of ratings inside a block
    hipLaunchKernelGGL(k_keys_dep, dim3(grid_for(n)), dim3(256), 0, s, u, it, c->irank, c->e2s, n, sk,
                       c->sk[0], c->sv[0]);
    LSHMF_LAUNCHED("k_keys_dep");
    LSHMF_TRY(radix_sort(c->sk, c->sv, n, sbits, c->hist, c->scan_tmp, s, &ri));
    int64_t* chain = reinterpret_cast<int64_t*>(c->sk[ri ^ 1]);  // n+1 int64, scanned in place
    hipLaunchKernelGGL(k_chain_flags, dim3(grid_for(n)), dim3(256), 0, s, c->sk[ri], n, sk.N, chain);
    LSHMF_LAUNCHED("k_chain_flags");
    LSHMF_TRY(scan_excl(chain, chain, n, c->scan_tmp, s));
    hipLaunchKernelGGL(k_dep_fill, dim3(grid_for(n)), dim3(256), 0, s, c->sk[ri], c->sv[ri], n, sk.N, bop,
                       st.blk_ptr, chain, st.dep, st.link);
    LSHMF_LAUNCHED("k_dep_fill");
    hipLaunchKernelGGL(k_block_slots, dim3(grid_for(P * P)), dim3(256), 0, s, st.blk_ptr, chain, P * P,
                       st.blk_slots);
    LSHMF_LAUNCHED("k_block_slots");
    // blocks of each stratum, heaviest first (the order blocks are dispatched in)
    {
        const int pb = bits_for((uint64_t)P);
        hipLaunchKernelGGL(k_keys_blkorder, dim3(grid_for(P * P)), dim3(256), 0, s, st.blk_ptr, P, pb, c->sk[0],
                           c->sv[0]);
        LSHMF_LAUNCHED("k_keys_blkorder");
        int ro = 0;
        LSHMF_TRY(radix_sort(c->sk, c->sv, P * P, pb + 32 + pb, c->hist, c->scan_tmp, s, &ro));
        LSHMF_HIP(hipMemcpyAsync(st.blk_order, c->sv[ro], sizeof(int32_t) * P * P, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_heavy_count, dim3(grid_for(P)), dim3(256), 0, s, st.blk_ptr, st.blk_order, P, st.heavy);
        LSHMF_LAUNCHED("k_heavy_count");
        hipLaunchKernelGGL(k_block_runs, dim3(grid_for(P * P)), dim3(256), 0, s, st.blk_order, st.blk_seg, P,
                           st.blk_run);
        LSHMF_LAUNCHED("k_block_runs");
    }
    // zero tails: the SGD kernel reads a few records past a run's end
    LSHMF_TRY(fill_i32(reinterpret_cast<int32_t*>(st.pk) + n, kStreamPad, 0, s));
    LSHMF_TRY(fill_i32(reinterpret_cast<int32_t*>(st.link) + n, kStreamPad, 0, s));

    // largest block, most mailbox slots in a block and the run count
    LSHMF_TRY(fill_i64(st.stats, 4, 0, s));
    hipLaunchKernelGGL(k_stream_stats, dim3(grid_for(P * P, 256, 1024)), dim3(256), 0, s, st.blk_ptr, st.blk_seg,
                       st.blk_slots, P * P, st.stats);
    LSHMF_LAUNCHED("k_stream_stats");
    st.pending = n;
    return LSHMF_OK;
}

// After a synchronisation: the host copy of the stream's statistics (hstats,
// copied from st.stats) makes the stream usable.
void stream_finish(Stream& st, const int64_t* hstats)
{
    if (st.pending == 0) return;
    st.n = st.pending;
    st.pending = 0;
    st.max_block_nnz = hstats[0];
    st.max_block_slots = hstats[1];
    st.nseg = hstats[2];
    st.codes = false;
}

int build_stream(lshmf_ctx* c, Stream& st, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n,
                 hipStream_t s)
{
    LSHMF_TRY(build_stream_async(c, st, u, it, rc, n, s));
    if (n == 0) return LSHMF_OK;
    int64_t h[4] = {0, 0, 0, 0};
    LSHMF_HIP(hipMemcpyAsync(h, st.stats, sizeof(h), hipMemcpyDeviceToHost, s));
    LSHMF_HIP(hipMemcpyAsync(st.hcounts.data(), st.heavy, sizeof(int32_t) * st.hcounts.size(),
                             hipMemcpyDeviceToHost, s));
    LSHMF_TRY(sync_status(c, s));
    stream_finish(st, h);
    return LSHMF_OK;
}

// mu, b0_i, bh0_j of the simple case (Sec. 3.2) over the whole store.
int baselines_all(lshmf_ctx* c, hipStream_t s)
{
    if (c->d.model == LSHMF_PLAIN_MF) {  // rhat = u . v: no mean, no baselines
        LSHMF_TRY(fill_i64(reinterpret_cast<int64_t*>(c->t.mu), 1, 0, s));
        LSHMF_TRY(fill_f32(c->t.b0, c->M, 0.0f, s));
        return fill_f32(c->t.bh0, c->N, 0.0f, s);
    }
    const int64_t n = c->nnz;
    unsigned long long* total = reinterpret_cast<unsigned long long*>(c->cnt);
    LSHMF_TRY(fill_i64(c->cnt, 1, 0, s));
    hipLaunchKernelGGL(k_sum_codes, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, c->coo_rc, n, total);
    LSHMF_LAUNCHED("k_sum_codes");
    hipLaunchKernelGGL(k_mu, dim3(1), dim3(64), 0, s, total, n, c->d.rscale, c->t.mu);
    LSHMF_LAUNCHED("k_mu");
    hipLaunchKernelGGL(k_row_means, dim3(grid_for((int64_t)c->M * kWave)), dim3(256), 0, s, c->row_ptr,
                       c->csr_rc, (int64_t)c->M, c->d.rscale, c->t.mu, c->t.b0);
    LSHMF_LAUNCHED("k_row_means(users)");
    hipLaunchKernelGGL(k_row_means, dim3(grid_for((int64_t)c->N * kWave)), dim3(256), 0, s, c->col_ptr,
                       c->csc_rc, (int64_t)c->N, c->d.rscale, c->t.mu, c->t.bh0);
    LSHMF_LAUNCHED("k_row_means(items)");
    return LSHMF_OK;
}

// Baselines of ids in [first, first + count) from n batch ratings.
int baselines_new(lshmf_ctx* c, const int32_t* id, const uint8_t* rc, int64_t n, int32_t first, int32_t count,
                  float* out, hipStream_t s)
{
    if (count <= 0) return LSHMF_OK;
    if (c->d.model == LSHMF_PLAIN_MF) return fill_f32(out + first, count, 0.0f, s);
    unsigned long long* sum = reinterpret_cast<unsigned long long*>(c->cnt);
    unsigned long long* cn = sum + count;
    LSHMF_TRY(fill_i64(c->cnt, 2 * (int64_t)count, 0, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_sum_by_id, dim3(grid_for(n)), dim3(256), 0, s, id, rc, n, first, sum, cn);
        LSHMF_LAUNCHED("k_sum_by_id");
    }
    hipLaunchKernelGGL(k_new_means, dim3(grid_for(count)), dim3(256), 0, s, sum, cn, count, c->d.rscale, c->t.mu,
                       out + first);
    LSHMF_LAUNCHED("k_new_means");
    return LSHMF_OK;
}

int ingest(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n, hipStream_t s)
{
    LSHMF_TRY(fill_i32(c->err, 1, 0, s));  // the device status word starts healthy
    LSHMF_TRY(check_ids(c, u, it, rc, n, c->M, c->N, s));
    if (n > 0) {
        LSHMF_HIP(hipMemcpyAsync(c->coo_u, u, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        LSHMF_HIP(hipMemcpyAsync(c->coo_i, it, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        LSHMF_HIP(hipMemcpyAsync(c->coo_rc, rc, n, hipMemcpyDeviceToDevice, s));
    }
    c->nnz = n;
    LSHMF_TRY(build_compressed(c, s, c->err + 1));
    LSHMF_TRY(input_status(c, c->M, c->N, s));  // a pair given twice
    LSHMF_TRY(baselines_all(c, s));
    LSHMF_TRY(build_stream(c, c->train, c->coo_u, c->coo_i, c->coo_rc, n, s));
    c->train_stale = false;
    return LSHMF_OK;
}

}  // namespace lshmf
