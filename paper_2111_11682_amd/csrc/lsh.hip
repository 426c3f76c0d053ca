// simLSH neighbour search without the N x N similarity matrix (Sec. 4.1).
//
//   k_simlsh_acc    pre-sign sums acc[j][b] = sum_{i in col j} Psi(r_ij)(2 H_ib - 1)
//                   (Eq. item_hash).  Integer arithmetic, so the sums are exact
//                   and independent of the order of the atomic flushes.
//   k_simlsh_sign   Upsilon: bit b of item j is set iff acc[j][b] >= 0.
//   k_rpcos_*,      the two other families of the Sec. 5.3 comparison (sign
//   k_minhash_*     random projection, b-bit minwise hashing) filling the
//                   same signature layout.
//   k_band_keys     q band keys of p*G bits (p hashes ANDed per band).
//   k_bucket_*      one radix sort of (band, key) groups the items of every
//                   bucket; a bucket id per (band, item).
//   k_topk          per item: collision counts over its q buckets in an LDS
//                   hash table, the K most frequent partners by (count desc,
//                   id asc), seeded SplitMix64 supplement, ids ascending.
//   k_nbr_codes     per training rating (i, j): the rating code of user i for
//                   each neighbour JK[j][k] (0 if not rated), 4 bits per slot;
//                   this resolves R^K(i;j) and N^K(i;j) once for all epochs.
//   k_nbr_codes_rows  the same codes by user row through an LDS item map, for
//                   streams that hold most of the store.
#include "common.hpp"

namespace lshmf {

// ------------------------------------------------------------ projection
// A wave walks a chunk of CSC positions, one column segment at a time (the
// columns meeting the chunk, in order).  Lane (g, w) owns signature word w of
// the current 64-word slice (32 bits) and takes the positions p of the
// segment with p = start + g (mod R), R = 64 / Wd rating groups, Wd the
// slice's word count rounded up to a power of two.  Per rating it loads one
// word of H_i and adds Psi(r) to the counters of its set bits,
// S_t += Psi * bit_t; T sums Psi.  At the segment's end the R groups' counters
// are summed across the wave and one lane per word adds
// acc[j][32w + t] += 2 S_t - T = sum Psi (2 bit - 1) with integer atomics, so
// the sums are exact and independent of the order of the flushes (the
// counters wrap modulo 2^32; the exact total fits int32).  Summing before the
// atomics keeps a popular column's chunks to one atomic per bit each.
constexpr int kAccChunk = 1024;    // CSC positions per wave

__global__ __launch_bounds__(256) void k_simlsh_acc(const int64_t* col_ptr, const int32_t* row,
                                                    const uint8_t* rc, int64_t nnz, int32_t N,
                                                    const uint32_t* H, int words, int B, int psi_exp,
                                                    int wd_log2, int32_t* acc)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t p0 = wave * kAccChunk;
    if (p0 >= nnz) return;
    const int64_t p1 = p0 + kAccChunk < nnz ? p0 + kAccChunk : nnz;
    const int Wd = 1 << wd_log2;
    const int R = kWave >> wd_log2;
    const int grp = lane >> wd_log2;
    const int w = (int)blockIdx.y * kWave + (lane & (Wd - 1));
    const bool wok = w < words;
    // column containing p0: largest j with col_ptr[j] <= p0
    int32_t lo = 0, hi = N;  // invariant col_ptr[lo] <= p0 < col_ptr[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (col_ptr[mid] <= p0) lo = mid;
        else hi = mid;
    }
    int32_t j = lo;
    int64_t cs = p0;
    for (;;) {
        const int64_t cend = col_ptr[j + 1];
        const int64_t ce = cend < p1 ? cend : p1;
        uint32_t S[32];
#pragma unroll
        for (int t = 0; t < 32; ++t) S[t] = 0u;
        uint32_t T = 0u;
        int64_t p = cs + grp;
        int64_t i_next = p < ce ? row[p] : 0;
        uint32_t c_next = p < ce ? rc[p] : 0u;
        while (p < ce) {
            const int64_t i = i_next;
            const uint32_t code = c_next;
            const int64_t pn = p + R;
            if (pn < ce) {
                i_next = row[pn];
                c_next = rc[pn];
            }
            const uint32_t x = wok ? H[i * words + w] : 0u;
            uint32_t psi = 1u;
            for (int e = 0; e < psi_exp; ++e) psi *= code;
            T += psi;
#pragma unroll
            for (int t = 0; t < 32; ++t) S[t] += ((x >> t) & 1u) * psi;
            p = pn;
        }
        // sum the R groups: lanes with the same word differ in the bits above wd_log2
        for (int o = Wd; o < kWave; o <<= 1) {
#pragma unroll
            for (int t = 0; t < 32; ++t) S[t] += (uint32_t)__shfl_xor((int)S[t], o, kWave);
            T += (uint32_t)__shfl_xor((int)T, o, kWave);
        }
        if (grp == 0 && wok && T != 0u) {
            int32_t* a = acc + (int64_t)j * B + 32 * w;
#pragma unroll
            for (int t = 0; t < 32; ++t) {
                const int32_t v = (int32_t)(2u * S[t] - T);
                if (32 * w + t < B && v != 0) atomicAdd(a + t, v);
            }
        }
        if (ce >= p1) break;
        // next column with ratings (empty columns end where this one ends)
        do {
            ++j;
        } while (col_ptr[j + 1] <= ce);
        cs = ce;
    }
}

__global__ void k_simlsh_sign(const int32_t* acc, int32_t N, int B, int words, uint32_t* sig)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < (int64_t)N * words;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = x / words;
        const int w = (int)(x % words);
        uint32_t v = 0;
        for (int t = 0; t < 32; ++t) {
            const int b = w * 32 + t;
            if (b < B && acc[j * B + b] >= 0) v |= 1u << t;
        }
        sig[x] = v;
    }
}

// RP_cos (sign random projection for the cosine similarity, the family of
// the Sec. 5.3 comparison): acc[j][b] += r_ij g_ib in FP32.  The sign is an
// integer decided by floating point, so the order is fixed: one wave per
// (item, 64-bit slice), lane b sums the item's raters in CSC order (users
// ascending) with one fused multiply-add each, continuing the stored sum.
__global__ __launch_bounds__(256) void k_rpcos_acc(const int64_t* col_ptr, const int32_t* row, const uint8_t* rc,
                                                   int32_t N, const float* g, int B, float inv_s, float* acc)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int slices = (B + kWave - 1) / kWave;
    if (wave >= (int64_t)N * slices) return;
    const int64_t j = wave / slices;
    const int b = (int)(wave % slices) * kWave + lane;
    const int64_t a = col_ptr[j], z = col_ptr[j + 1];
    if (a == z) return;
    const bool ok = b < B;
    float s = ok ? acc[j * B + b] : 0.0f;
    for (int64_t p = a; p < z; ++p) {
        const float r = (float)rc[p] * inv_s;
        const float gv = ok ? g[(int64_t)row[p] * B + b] : 0.0f;
        s = __builtin_fmaf(r, gv, s);
    }
    if (ok) acc[j * B + b] = s;
}

__global__ void k_rpcos_sign(const float* acc, int32_t N, int B, int words, uint32_t* sig)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < (int64_t)N * words;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = x / words;
        const int w = (int)(x % words);
        uint32_t v = 0;
        for (int t = 0; t < 32; ++t) {
            const int b = w * 32 + t;
            if (b < B && acc[j * B + b] >= 0.0f) v |= 1u << t;
        }
        sig[x] = v;
    }
}

// minHash (b-bit minwise hashing of the rater sets): mins[j][h] = least random
// value v_ih over the raters of item j; integer minima are exact and order-free.
__global__ __launch_bounds__(256) void k_minhash_acc(const int64_t* col_ptr, const int32_t* row, int32_t N,
                                                     const uint32_t* v, int nh, uint32_t* mins)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int slices = (nh + kWave - 1) / kWave;
    if (wave >= (int64_t)N * slices) return;
    const int64_t j = wave / slices;
    const int h = (int)(wave % slices) * kWave + lane;
    const int64_t a = col_ptr[j], z = col_ptr[j + 1];
    if (a == z || h >= nh) return;
    uint32_t m = mins[j * nh + h];
    for (int64_t p = a; p < z; ++p) {
        const uint32_t x = v[(int64_t)row[p] * nh + h];
        m = x < m ? x : m;
    }
    mins[j * nh + h] = m;
}

// The G low bits of each minimum, hash h at bits [hG, (h+1)G) of the signature.
__global__ void k_minhash_sign(const uint32_t* mins, int32_t N, int nh, int G, int words, uint32_t* sig)
{
    const int B = nh * G;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < (int64_t)N * words;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = x / words;
        const int w = (int)(x % words);
        uint32_t v = 0;
        for (int t = 0; t < 32; ++t) {
            const int b = w * 32 + t;
            if (b < B && ((mins[j * nh + b / G] >> (b % G)) & 1u)) v |= 1u << t;
        }
        sig[x] = v;
    }
}

// --------------------------------------------------------------- banding
__global__ void k_band_keys(const uint32_t* sig, int32_t N, int words, int pG, int q, uint64_t* keys,
                            uint32_t* vals)
{
    const int64_t n = (int64_t)q * N;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(x / N);
        const int64_t j = x % N;
        const int off = t * pG;
        const int w0 = off >> 5, sh = off & 31;  // pG <= 56: three words suffice
        const uint32_t* r = sig + j * words;
        uint64_t v = r[w0];
        if (w0 + 1 < words) v |= (uint64_t)r[w0 + 1] << 32;
        v >>= sh;
        if (sh > 0 && w0 + 2 < words) v |= (uint64_t)r[w0 + 2] << (64 - sh);
        const uint64_t key = v & ((1ull << pG) - 1ull);
        keys[x] = ((uint64_t)t << pG) | key;
        vals[x] = (uint32_t)j;
    }
}

__global__ void k_bucket_flags(const uint64_t* keys, int64_t n, int64_t* flag)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        flag[x] = (x == 0 || keys[x] != keys[x - 1]) ? 1 : 0;
}

// bucket id of sorted position x is incl[x] - 1 = ex[x+1] - 1
__global__ void k_bucket_fill(const uint64_t* keys, const uint32_t* items, const int64_t* ex, int64_t n,
                              int32_t N, int pG, int32_t* bitem, int32_t* bbegin, int32_t* bpos)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t id = (int32_t)(ex[x + 1] - 1);
        const uint32_t j = items[x];
        const int64_t t = (int64_t)(keys[x] >> pG);
        bitem[x] = (int32_t)j;
        if (x == 0 || keys[x] != keys[x - 1]) bbegin[id] = (int32_t)x;
        bpos[t * N + j] = id;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) bbegin[ex[n]] = (int32_t)n;
}

// ------------------------------------------------------------------ top-K
constexpr int kTopkThreads = 256;
constexpr int kTabCap = 4096;              // LDS hash slots
constexpr int kRangeCap = kTabCap / 2;     // occurrences admitted per range
constexpr int kMaxK = 128;

__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t c)
{
    // SplitMix64 (Steele, Lea, Flood 2014): output c of the stream at `seed`
    uint64_t z = seed + c * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline uint32_t slot_hash(uint32_t x) { return (x * 2654435761u) >> 20; }  // 12 bits

// Bitonic sort of buf[0..n2) ascending, n2 a power of two, whole workgroup.
__device__ void bitonic_sort(uint64_t* buf, int n2)
{
    for (int k = 2; k <= n2; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int t = threadIdx.x; t < (n2 >> 1); t += blockDim.x) {
                const int i = 2 * jj * (t / jj) + (t % jj);
                const int l = i + jj;
                const bool up = (i & k) == 0;
                const uint64_t a = buf[i], b = buf[l];
                if ((a > b) == up) {
                    buf[i] = b;
                    buf[l] = a;
                }
            }
            __syncthreads();
        }
    }
}

__device__ inline int block_sum_int(int v, int* scratch)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    int tot = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) tot += scratch[w];
    return tot;
}

// One workgroup per item.  Candidate ids are processed in id ranges small
// enough that their occurrences fit the LDS table; a running best list of K
// (count desc, id asc) keys is merged with each range by a bitonic sort.
__global__ __launch_bounds__(kTopkThreads) void k_topk(const int32_t* bitem, const int32_t* bbegin,
                                                       const int32_t* bpos, int32_t N, int q, int K,
                                                       uint64_t seed_fill, int32_t* JK, int32_t j_first)
{
    __shared__ uint64_t buf[kTabCap];      // hash table (key | count) / sort buffer
    __shared__ uint64_t best[kMaxK];
    __shared__ int32_t chosen[kMaxK];
    __shared__ int red[kTopkThreads / kWave];
    __shared__ int nbest_s, nent_s;
    uint32_t* tkey = reinterpret_cast<uint32_t*>(buf);             // kTabCap keys
    uint32_t* tcnt = reinterpret_cast<uint32_t*>(buf) + kTabCap;   // kTabCap counts

    const int32_t j = j_first + blockIdx.x;
    if (j >= N) return;
    const int tid = threadIdx.x;
    if (tid == 0) nbest_s = 0;
    int32_t lo = 0, span = N;
    while (lo < N) {
        const int32_t hi = (int32_t)((int64_t)lo + span < N ? lo + span : N);
        // occurrences of ids in [lo, hi) over the q buckets of j
        int occ = 0;
        for (int t = 0; t < q; ++t) {
            const int32_t id = bpos[(int64_t)t * N + j];
            const int32_t a = bbegin[id], z = bbegin[id + 1];
            for (int32_t x = a + tid; x < z; x += kTopkThreads) {
                const int32_t c = bitem[x];
                occ += (c != j && c >= lo && c < hi);
            }
        }
        occ = block_sum_int(occ, red);
        if (occ > kRangeCap && hi - lo > 1) {
            span = (hi - lo) / 2;
            continue;
        }
        for (int x = tid; x < kTabCap; x += kTopkThreads) {
            tkey[x] = 0xFFFFFFFFu;
            tcnt[x] = 0;
        }
        __syncthreads();
        for (int t = 0; t < q; ++t) {
            const int32_t id = bpos[(int64_t)t * N + j];
            const int32_t a = bbegin[id], z = bbegin[id + 1];
            for (int32_t x = a + tid; x < z; x += kTopkThreads) {
                const uint32_t c = (uint32_t)bitem[x];
                if ((int32_t)c == j || (int32_t)c < lo || (int32_t)c >= hi) continue;
                uint32_t h = slot_hash(c) & (kTabCap - 1);
                while (true) {
                    const uint32_t old = atomicCAS(&tkey[h], 0xFFFFFFFFu, c);
                    if (old == 0xFFFFFFFFu || old == c) {
                        atomicAdd(&tcnt[h], 1u);
                        break;
                    }
                    h = (h + 1) & (kTabCap - 1);
                }
            }
        }
        __syncthreads();
        // extract (q - count, id) keys into registers, then into buf
        constexpr int kPer = kTabCap / kTopkThreads;
        uint64_t ent[kPer];
        int nmine = 0;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int x = tid + r * kTopkThreads;
            ent[r] = ~0ull;
            if (tkey[x] != 0xFFFFFFFFu) {
                ent[r] = ((uint64_t)(q - (int)tcnt[x]) << 32) | tkey[x];
                ++nmine;
            }
        }
        if (tid == 0) nent_s = 0;
        __syncthreads();
        int pos = nmine ? atomicAdd(&nent_s, nmine) : 0;
#pragma unroll
        for (int r = 0; r < kPer; ++r)
            if (ent[r] != ~0ull) buf[pos++] = ent[r];
        __syncthreads();
        const int nent = nent_s, nb = nbest_s;
        for (int x = tid; x < nb; x += kTopkThreads) buf[nent + x] = best[x];
        int n2 = 1;
        while (n2 < nent + nb) n2 <<= 1;
        for (int x = nent + nb + tid; x < n2; x += kTopkThreads) buf[x] = ~0ull;
        __syncthreads();
        if (n2 > 1) bitonic_sort(buf, n2);
        const int keep = (nent + nb) < K ? (nent + nb) : K;
        for (int x = tid; x < keep; x += kTopkThreads) best[x] = buf[x];
        __syncthreads();
        if (tid == 0) nbest_s = keep;
        __syncthreads();
        lo = hi;
    }
    // random supplement, ids ascending
    if (tid == 0) {
        int n = nbest_s;
        for (int x = 0; x < n; ++x) chosen[x] = (int32_t)(best[x] & 0xFFFFFFFFu);
        for (uint64_t a = 0; n < K; ++a) {
            const int32_t cand = (int32_t)(splitmix64(seed_fill, ((uint64_t)j << 32) + a + 1) % (uint64_t)N);
            bool dup = cand == j;
            for (int y = 0; y < n && !dup; ++y) dup = chosen[y] == cand;
            if (!dup) chosen[n++] = cand;
        }
        for (int x = 1; x < K; ++x) {  // insertion sort, K <= 128
            const int32_t v = chosen[x];
            int y = x - 1;
            while (y >= 0 && chosen[y] > v) {
                chosen[y + 1] = chosen[y];
                --y;
            }
            chosen[y + 1] = v;
        }
    }
    __syncthreads();
    for (int x = tid; x < K; x += kTopkThreads) JK[(int64_t)j * K + x] = chosen[x];
}

// -------------------------------------------------------- neighbour codes
// One wave per stream rating; lane L resolves slots L and L + 64 by binary
// search in the user's CSR row, then byte x of the record packs slots 2x
// (low nibble) and 2x+1 (high nibble).
__global__ __launch_bounds__(256) void k_nbr_codes(const uint32_t* pk, const int32_t* sj, int64_t n,
                                                   const int32_t* JK, int K, const int64_t* row_ptr,
                                                   const int32_t* csr_col, const uint8_t* csr_rc,
                                                   uint8_t* nib, int nstride)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t p = w0; p < n; p += nw) {
        const int64_t i = pk[p] >> 4;
        const int64_t j = sj[p];
        const int64_t a = row_ptr[i], z = row_ptr[i + 1];
        int code[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = lane + h * kWave;
            if (k < K) {
                const int32_t nb = JK[j * K + k];
                int64_t l = a, r = z;
                while (l < r) {
                    const int64_t m = (l + r) >> 1;
                    if (csr_col[m] < nb) l = m + 1;
                    else r = m;
                }
                code[h] = (l < z && csr_col[l] == nb) ? csr_rc[l] : 0;
            }
        }
        // byte `lane` packs slots 2*lane and 2*lane+1
        const int s0 = 2 * lane, s1 = 2 * lane + 1;
        const int lo0 = __shfl(code[0], s0 & 63, kWave), hi0 = __shfl(code[1], s0 & 63, kWave);
        const int lo1 = __shfl(code[0], s1 & 63, kWave), hi1 = __shfl(code[1], s1 & 63, kWave);
        const int c0 = s0 < 64 ? lo0 : hi0;
        const int c1 = s1 < 64 ? lo1 : hi1;
        if (lane < nstride) nib[p * nstride + lane] = (uint8_t)(c0 | (c1 << 4));
    }
}

// The same codes by user row, for a stream that holds the whole store.  The
// stream positions are sorted by user (stable, so ascending inside a user),
// which groups them as the CSR rows are grouped: user i's ratings take
// positions row_ptr[i] .. row_ptr[i+1] of the sorted list.  One workgroup
// takes one user row at a time: the row's rating codes are scattered into an
// LDS byte map indexed by item (N bytes), and every 4-byte word of every
// record of the row (8 slots) is resolved with 8 LDS reads, so a rating costs
// its K neighbour ids from L2 instead of K binary searches in HBM.
constexpr int kCodeMapMax = 65536;   // items an LDS byte map can hold
constexpr int kCodeUnroll = 4;       // records words in flight per thread

__global__ void k_keys_user(const uint32_t* pk, int64_t n, uint64_t* keys, uint32_t* vals)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        keys[p] = pk[p] >> 4;
        vals[p] = (uint32_t)p;
    }
}

__global__ __launch_bounds__(256) void k_nbr_codes_rows(const int64_t* row_ptr, const int32_t* csr_col,
                                                        const uint8_t* csr_rc, int32_t M, int32_t N,
                                                        const uint32_t* by_user, const int32_t* sj,
                                                        const int32_t* JK, int K, uint8_t* nib, int nstride)
{
    extern __shared__ uint32_t map_words[];
    uint8_t* map = reinterpret_cast<uint8_t*>(map_words);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int x = tid; x < (N + 3) / 4; x += nt) map_words[x] = 0;
    const int wpr = nstride / 4;               // 4-byte words per record
    const bool quads = (K & 3) == 0;           // JK rows 16-byte aligned
    // a thread's work items t = tid + m * nt as (record e, word w) = divmod(t, wpr)
    const int e0 = tid / wpr, w0 = tid - e0 * wpr;
    const int de = nt / wpr, dw = nt - de * wpr;
    for (int32_t i = blockIdx.x; i < M; i += gridDim.x) {
        const int64_t a = row_ptr[i];
        const int32_t deg = (int32_t)(row_ptr[i + 1] - a);
        __syncthreads();                       // the previous row's map is clear
        for (int32_t x = tid; x < deg; x += nt) map[csr_col[a + x]] = csr_rc[a + x];
        __syncthreads();
        int e = e0, w = w0;
        while (e < deg) {
            int ee[kCodeUnroll], ww[kCodeUnroll];
            uint32_t p[kCodeUnroll];
#pragma unroll
            for (int u = 0; u < kCodeUnroll; ++u) {
                ee[u] = e;
                ww[u] = w;
                p[u] = e < deg ? by_user[a + e] : 0u;
                e += de;
                w += dw;
                if (w >= wpr) {
                    w -= wpr;
                    ++e;
                }
            }
            int32_t j[kCodeUnroll];
#pragma unroll
            for (int u = 0; u < kCodeUnroll; ++u) j[u] = ee[u] < deg ? sj[p[u]] : 0;
#pragma unroll
            for (int u = 0; u < kCodeUnroll; ++u) {
                if (ee[u] >= deg) continue;
                const int32_t* jk = JK + (int64_t)j[u] * K;
                const int k0 = 8 * ww[u];
                uint32_t word = 0;
                if (quads && k0 + 8 <= K) {
                    const int4 q0 = *reinterpret_cast<const int4*>(jk + k0);
                    const int4 q1 = *reinterpret_cast<const int4*>(jk + k0 + 4);
                    word = (uint32_t)map[q0.x] | (uint32_t)map[q0.y] << 4 | (uint32_t)map[q0.z] << 8 |
                           (uint32_t)map[q0.w] << 12 | (uint32_t)map[q1.x] << 16 | (uint32_t)map[q1.y] << 20 |
                           (uint32_t)map[q1.z] << 24 | (uint32_t)map[q1.w] << 28;
                } else {
                    for (int h = 0; h < 8 && k0 + h < K; ++h) word |= (uint32_t)map[jk[k0 + h]] << (4 * h);
                }
                *reinterpret_cast<uint32_t*>(nib + (int64_t)p[u] * nstride + 4 * ww[u]) = word;
            }
        }
        __syncthreads();
        for (int32_t x = tid; x < deg; x += nt) map[csr_col[a + x]] = 0;
    }
}

// The same by user row for any item count: a row's (item, code) pairs sit in
// an LDS open-addressing table (linear probing on a Fibonacci hash of the item
// id, at most half full), so a slot costs a short probe sequence instead of a
// byte-map read.  Rows of up to kHashRow ratings take one table (a quarter
// full when they have at most kHashRow / 2).  A longer row is cut into chunks
// of kHashRow consecutive CSR entries: every chunk, in a workgroup of its own,
// resolves the slots whose items it holds for every record of the row and ORs
// them into the record (zeroed beforehand), so the row's cost is spread over
// its chunks' workgroups.
constexpr int kHashLg = 14;
constexpr int kHashCap = 1 << kHashLg;   // table entries (64 KB of LDS)
constexpr int kHashRow = kHashCap / 2;
constexpr int kHashThreads = 512;
constexpr uint32_t kHashEmpty = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t hash_code(const uint32_t* tab, uint32_t mask, int sh, int32_t item)
{
    uint32_t h = ((uint32_t)item * 2654435769u) >> sh;
    while (true) {
        const uint32_t e = tab[h];
        if (e == kHashEmpty) return 0u;
        if ((int32_t)(e >> 4) == item) return e & 15u;
        h = (h + 1) & mask;
    }
}

// Table of n CSR entries from `a` on (2^lg entries); the caller synchronises
// before (the table is free) and after (it is complete).
__device__ __forceinline__ void hash_fill(uint32_t* tab, int lg, const int32_t* csr_col, const uint8_t* csr_rc,
                                          int64_t a, int32_t n)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint32_t mask = (1u << lg) - 1u;
    for (int x = tid; x <= (int)mask; x += nt) tab[x] = kHashEmpty;
    __syncthreads();
    for (int32_t x = tid; x < n; x += nt) {  // items of a row are distinct: no key is inserted twice
        const int32_t it = csr_col[a + x];
        const uint32_t key = ((uint32_t)it << 4) | (uint32_t)csr_rc[a + x];
        uint32_t h = ((uint32_t)it * 2654435769u) >> (32 - lg);
        while (atomicCAS(&tab[h], kHashEmpty, key) != kHashEmpty) h = (h + 1) & mask;
    }
}

// Every 4-byte word of the records of the row's deg ratings (stream positions
// by_user[a ..]): the codes the table holds; stored, or ORed in when nonzero.
template <bool kOr>
__device__ __forceinline__ void hash_resolve(const uint32_t* tab, int lg, int64_t a, int32_t deg,
                                             const uint32_t* by_user, const int32_t* sj, const int32_t* JK, int K,
                                             uint8_t* nib, int nstride)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint32_t mask = (1u << lg) - 1u;
    const int sh = 32 - lg;
    const int wpr = nstride / 4;               // 4-byte words per record
    const bool quads = (K & 3) == 0;           // JK rows 16-byte aligned
    // a thread's work items t = tid + m * nt as (record e, word w) = divmod(t, wpr)
    int e = tid / wpr, w = tid - (tid / wpr) * wpr;
    const int de = nt / wpr, dw = nt - de * wpr;
    while (e < deg) {
        int ee[kCodeUnroll], ww[kCodeUnroll];
        uint32_t p[kCodeUnroll];
#pragma unroll
        for (int u = 0; u < kCodeUnroll; ++u) {
            ee[u] = e;
            ww[u] = w;
            p[u] = e < deg ? by_user[a + e] : 0u;
            e += de;
            w += dw;
            if (w >= wpr) {
                w -= wpr;
                ++e;
            }
        }
        int32_t j[kCodeUnroll];
#pragma unroll
        for (int u = 0; u < kCodeUnroll; ++u) j[u] = ee[u] < deg ? sj[p[u]] : 0;
#pragma unroll
        for (int u = 0; u < kCodeUnroll; ++u) {
            if (ee[u] >= deg) continue;
            const int32_t* jk = JK + (int64_t)j[u] * K;
            const int k0 = 8 * ww[u];
            int32_t nb[8];
            if (quads && k0 + 8 <= K) {
                const int4 q0 = *reinterpret_cast<const int4*>(jk + k0);
                const int4 q1 = *reinterpret_cast<const int4*>(jk + k0 + 4);
                nb[0] = q0.x; nb[1] = q0.y; nb[2] = q0.z; nb[3] = q0.w;
                nb[4] = q1.x; nb[5] = q1.y; nb[6] = q1.z; nb[7] = q1.w;
            } else {
                for (int h = 0; h < 8; ++h) nb[h] = k0 + h < K ? jk[k0 + h] : -1;
            }
            uint32_t word = 0;
#pragma unroll
            for (int h = 0; h < 8; ++h)
                if (nb[h] >= 0) word |= hash_code(tab, mask, sh, nb[h]) << (4 * h);
            uint32_t* dst = reinterpret_cast<uint32_t*>(nib + (int64_t)p[u] * nstride + 4 * ww[u]);
            if (!kOr) *dst = word;
            else if (word != 0u) atomicOr(dst, word);
        }
    }
}

// Rows of up to kHashRow ratings; a longer row gets its records zeroed and
// its id appended to long_rows (long_cnt[0] rows, long_cnt[1] the most
// ratings of one), in no particular order.
__global__ __launch_bounds__(kHashThreads) void k_nbr_codes_hash(const int64_t* row_ptr, const int32_t* csr_col,
                                                                 const uint8_t* csr_rc, int32_t M,
                                                                 const uint32_t* by_user, const int32_t* sj,
                                                                 const int32_t* JK, int K, uint8_t* nib,
                                                                 int nstride, unsigned long long* long_cnt,
                                                                 int32_t* long_rows)
{
    __shared__ uint32_t tab[kHashCap];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int wpr = nstride / 4;
    for (int32_t i = blockIdx.x; i < M; i += gridDim.x) {
        const int64_t a = row_ptr[i];
        const int32_t deg = (int32_t)(row_ptr[i + 1] - a);
        if (deg == 0) continue;                // the same for every thread of the block
        if (deg > kHashRow) {
            for (int64_t x = tid; x < (int64_t)deg * wpr; x += nt) {
                const int64_t e = x / wpr;
                *reinterpret_cast<uint32_t*>(nib + (int64_t)by_user[a + e] * nstride + 4 * (x - e * wpr)) = 0u;
            }
            if (tid == 0) {
                long_rows[atomicAdd(&long_cnt[0], 1ull)] = i;
                atomicMax(&long_cnt[1], (unsigned long long)deg);
            }
            continue;
        }
        int lg = 6;
        while (lg < kHashLg && (1 << lg) < 4 * deg) ++lg;
        __syncthreads();                       // the previous row's lookups are done
        hash_fill(tab, lg, csr_col, csr_rc, a, deg);
        __syncthreads();
        hash_resolve<false>(tab, lg, a, deg, by_user, sj, JK, K, nib, nstride);
    }
}

// The long rows' chunks: pair t = (row long_rows[t % L], chunk t / L).
__global__ __launch_bounds__(kHashThreads) void k_nbr_codes_long(const int64_t* row_ptr, const int32_t* csr_col,
                                                                 const uint8_t* csr_rc, const uint32_t* by_user,
                                                                 const int32_t* sj, const int32_t* JK, int K,
                                                                 uint8_t* nib, int nstride,
                                                                 const unsigned long long* long_cnt,
                                                                 const int32_t* long_rows)
{
    __shared__ uint32_t tab[kHashCap];
    const int64_t L = (int64_t)long_cnt[0];
    const int64_t chunks = ((int64_t)long_cnt[1] + kHashRow - 1) / kHashRow;
    for (int64_t t = blockIdx.x; t < L * chunks; t += gridDim.x) {
        const int32_t i = long_rows[t % L];
        const int64_t lo = (t / L) * kHashRow;
        const int64_t a = row_ptr[i];
        const int32_t deg = (int32_t)(row_ptr[i + 1] - a);
        if (lo >= deg) continue;               // the same for every thread of the block
        const int32_t n = deg - lo < kHashRow ? (int32_t)(deg - lo) : kHashRow;
        __syncthreads();                       // the previous chunk's lookups are done
        hash_fill(tab, kHashLg, csr_col, csr_rc, a + lo, n);
        __syncthreads();
        hash_resolve<true>(tab, kHashLg, a, deg, by_user, sj, JK, K, nib, nstride);
    }
}

__global__ void k_nbr_b0(const int32_t* JK, const float* bh0, int64_t n, float* out)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        out[x] = bh0[JK[x]];
}

static unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 16384)
{
    int64_t b = ceil_div(n > 0 ? n : 1, threads);
    return (unsigned)(b > cap ? cap : b);
}

// Adds the ratings of a CSC (col_ptr over c->N items) to the per-item hash
// state of the context's family: simLSH sums Psi(r)(2H-1) (R: bit strings
// H, ceil(B/32) words per user), RP_cos sums r g (R: B Gaussians per user),
// minHash minima (R: B/G random values per user).
int hash_add(lshmf_ctx* c, const int64_t* col_ptr, const int32_t* row, const uint8_t* rc, int64_t nnz,
             const void* R, hipStream_t s)
{
    if (nnz <= 0) return LSHMF_OK;
    const int fam = c->d.hash_family;
    if (fam == LSHMF_SIMLSH) {
        const int64_t waves = ceil_div(nnz, kAccChunk);
        const int slices = (c->words + kWave - 1) / kWave;
        const int in_slice = c->words < kWave ? c->words : kWave;
        const int wd_log2 = bits_for((uint64_t)in_slice);  // smallest power of two >= the slice's words
        hipLaunchKernelGGL(k_simlsh_acc, dim3((unsigned)ceil_div(waves * kWave, 256), (unsigned)slices), dim3(256), 0,
                           s, col_ptr, row, rc, nnz, c->N, static_cast<const uint32_t*>(R), c->words, c->B,
                           c->d.psi_exp, wd_log2, c->t.acc);
        LSHMF_LAUNCHED("k_simlsh_acc");
    } else if (fam == LSHMF_RPCOS) {
        const int64_t waves = (int64_t)c->N * ceil_div(c->B, kWave);
        hipLaunchKernelGGL(k_rpcos_acc, dim3((unsigned)ceil_div(waves * kWave, 256)), dim3(256), 0, s, col_ptr, row, rc,
                           c->N, static_cast<const float*>(R), c->B, 1.0f / (float)c->d.rscale,
                           reinterpret_cast<float*>(c->t.acc));
        LSHMF_LAUNCHED("k_rpcos_acc");
    } else {
        const int nh = c->B / c->d.G;
        const int64_t waves = (int64_t)c->N * ceil_div(nh, kWave);
        hipLaunchKernelGGL(k_minhash_acc, dim3((unsigned)ceil_div(waves * kWave, 256)), dim3(256), 0, s, col_ptr, row,
                           c->N, static_cast<const uint32_t*>(R), nh, reinterpret_cast<uint32_t*>(c->t.acc));
        LSHMF_LAUNCHED("k_minhash_acc");
    }
    return LSHMF_OK;
}

// Empty hash state of items [n0, n1): zero sums, or the all-ones minimum.
int hash_clear(lshmf_ctx* c, int64_t n0, int64_t n1, hipStream_t s)
{
    if (c->d.hash_family == LSHMF_MINHASH) {
        const int64_t nh = c->B / c->d.G;
        return fill_i32(c->t.acc + n0 * nh, (n1 - n0) * nh, -1, s);
    }
    return fill_i32(c->t.acc + n0 * c->B, (n1 - n0) * c->B, 0, s);
}

int signs(lshmf_ctx* c, hipStream_t s)
{
    const unsigned g = grid_for((int64_t)c->N * c->words);
    if (c->d.hash_family == LSHMF_SIMLSH) {
        hipLaunchKernelGGL(k_simlsh_sign, dim3(g), dim3(256), 0, s, c->t.acc, c->N, c->B, c->words, c->t.sig);
        LSHMF_LAUNCHED("k_simlsh_sign");
    } else if (c->d.hash_family == LSHMF_RPCOS) {
        hipLaunchKernelGGL(k_rpcos_sign, dim3(g), dim3(256), 0, s, reinterpret_cast<const float*>(c->t.acc), c->N,
                           c->B, c->words, c->t.sig);
        LSHMF_LAUNCHED("k_rpcos_sign");
    } else {
        hipLaunchKernelGGL(k_minhash_sign, dim3(g), dim3(256), 0, s, reinterpret_cast<const uint32_t*>(c->t.acc),
                           c->N, c->B / c->d.G, c->d.G, c->words, c->t.sig);
        LSHMF_LAUNCHED("k_minhash_sign");
    }
    return LSHMF_OK;
}

// Band keys and buckets over all c->N items, then the top-K lists and the
// neighbour baselines of items [j_first, j_first + count).
int neighbours_for(lshmf_ctx* c, int32_t j_first, int32_t count, uint64_t seed_fill, hipStream_t s)
{
    const lshmf_dims& d = c->d;
    if (d.K == 0) {  // no neighbour lists to find
        LSHMF_TRY(mark(c, 3, s));
        LSHMF_TRY(mark(c, 4, s));
        return LSHMF_OK;
    }
    const int64_t nq = (int64_t)d.q * c->N;
    hipLaunchKernelGGL(k_band_keys, dim3(grid_for(nq)), dim3(256), 0, s, c->t.sig, c->N, c->words, c->pG, d.q,
                       c->sk[0], c->sv[0]);
    LSHMF_LAUNCHED("k_band_keys");
    int ri = 0;
    LSHMF_TRY(radix_sort(c->sk, c->sv, nq, c->pG + bits_for((uint64_t)d.q), c->hist, c->scan_tmp, s, &ri));
    hipLaunchKernelGGL(k_bucket_flags, dim3(grid_for(nq)), dim3(256), 0, s, c->sk[ri], nq, c->cnt);
    LSHMF_LAUNCHED("k_bucket_flags");
    int64_t* ex = reinterpret_cast<int64_t*>(c->sk[ri ^ 1]);
    LSHMF_TRY(scan_excl(c->cnt, ex, nq, c->scan_tmp, s));
    hipLaunchKernelGGL(k_bucket_fill, dim3(grid_for(nq)), dim3(256), 0, s, c->sk[ri], c->sv[ri], ex, nq, c->N,
                       c->pG, c->bitem, c->bbegin, c->bpos);
    LSHMF_LAUNCHED("k_bucket_fill");
    LSHMF_TRY(mark(c, 3, s));
    for (int32_t j0 = 0; j0 < count; j0 += 65535) {
        const int32_t nj = count - j0 < 65535 ? count - j0 : 65535;
        hipLaunchKernelGGL(k_topk, dim3((unsigned)nj), dim3(kTopkThreads), 0, s, c->bitem, c->bbegin, c->bpos, c->N,
                           d.q, d.K, seed_fill, c->t.JK, j_first + j0);
        LSHMF_LAUNCHED("k_topk");
    }
    // fixed baselines of the neighbour slots (read once per item run by the SGD)
    const int64_t nk = (int64_t)count * d.K;
    if (nk > 0) {
        hipLaunchKernelGGL(k_nbr_b0, dim3(grid_for(nk)), dim3(256), 0, s, c->t.JK + (int64_t)j_first * d.K,
                           c->t.bh0, nk, c->nbr_b0 + (int64_t)j_first * d.K);
        LSHMF_LAUNCHED("k_nbr_b0");
    }
    LSHMF_TRY(mark(c, 4, s));
    return LSHMF_OK;
}

// Neighbour codes of every rating of a stream (R^K / N^K resolution).
int stream_codes(lshmf_ctx* c, Stream& st, hipStream_t s)
{
    if (st.n > 0 && c->d.K > 0) {
        if (st.n == c->nnz && c->N < (1 << 27)) {
            // the stream is the store (no pair twice), so its ratings of user i
            // are exactly CSR row i
            hipLaunchKernelGGL(k_keys_user, dim3(grid_for(st.n)), dim3(256), 0, s, st.pk, st.n, c->sk[0], c->sv[0]);
            LSHMF_LAUNCHED("k_keys_user");
            int ri = 0;
            LSHMF_TRY(radix_sort(c->sk, c->sv, st.n, bits_for((uint64_t)c->M), c->hist, c->scan_tmp, s, &ri));
            const unsigned grid = (unsigned)(c->M < 4096 ? (c->M > 0 ? c->M : 1) : 4096);
            if (c->N <= kCodeMapMax) {
                const size_t lds = sizeof(uint32_t) * (size_t)((c->N + 3) / 4);
                hipLaunchKernelGGL(k_nbr_codes_rows, dim3(grid), dim3(256), lds, s, c->row_ptr, c->csr_col,
                                   c->csr_rc, c->M, c->N, c->sv[ri], st.sj, c->t.JK, c->d.K, st.nib, c->nstride);
                LSHMF_LAUNCHED("k_nbr_codes_rows");
            } else {
                // item ids past the byte map's reach: hash tables, long rows in
                // chunks (their list and counters in the free counter buffer)
                unsigned long long* long_cnt = reinterpret_cast<unsigned long long*>(c->cnt);
                int32_t* long_rows = reinterpret_cast<int32_t*>(c->cnt + 2);
                LSHMF_TRY(fill_i64(c->cnt, 2, 0, s));
                hipLaunchKernelGGL(k_nbr_codes_hash, dim3(grid), dim3(kHashThreads), 0, s, c->row_ptr, c->csr_col,
                                   c->csr_rc, c->M, c->sv[ri], st.sj, c->t.JK, c->d.K, st.nib, c->nstride,
                                   long_cnt, long_rows);
                LSHMF_LAUNCHED("k_nbr_codes_hash");
                hipLaunchKernelGGL(k_nbr_codes_long, dim3(1024), dim3(kHashThreads), 0, s, c->row_ptr, c->csr_col,
                                   c->csr_rc, c->sv[ri], st.sj, c->t.JK, c->d.K, st.nib, c->nstride, long_cnt,
                                   long_rows);
                LSHMF_LAUNCHED("k_nbr_codes_long");
            }
        } else {
            hipLaunchKernelGGL(k_nbr_codes, dim3(grid_for(st.n * kWave, 256, 65536)), dim3(256), 0, s, st.pk,
                               st.sj, st.n, c->t.JK, c->d.K, c->row_ptr, c->csr_col, c->csr_rc, st.nib,
                               c->nstride);
            LSHMF_LAUNCHED("k_nbr_codes");
        }
    }
    st.codes = true;
    return LSHMF_OK;
}

// w, c of the old items after a rebuild of every list: a neighbour kept
// across the rebuild brings its values to its new slot, a new one starts at
// 0.  Both lists are sorted by id, so each lane finds its neighbour by binary
// search in the old row.  One wave per item.
__global__ __launch_bounds__(256) void k_remap_slots(const int32_t* JK_old, const float* W_old, const float* C_old,
                                                     const int32_t* JK_new, int32_t n_old, int K, float* W, float* C)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t j = w0; j < n_old; j += nw) {
        const int32_t* old = JK_old + j * K;
        for (int k = lane; k < K; k += kWave) {
            const int32_t n = JK_new[j * K + k];
            int l = 0, r = K;
            while (l < r) {
                const int m = (l + r) >> 1;
                if (old[m] < n) l = m + 1;
                else r = m;
            }
            const bool kept = l < K && old[l] == n;
            W[j * K + k] = kept ? W_old[j * K + l] : 0.0f;
            C[j * K + k] = kept ? C_old[j * K + l] : 0.0f;
        }
    }
}

// Every item's list searched again over the current signatures; W and C of
// items [0, n_old) follow their neighbour ids (the rows of newer items must
// already be zero).  The old lists and tables are kept in the arena.
int rebuild_lists(lshmf_ctx* c, int32_t n_old, uint64_t seed_fill, hipStream_t s)
{
    const int64_t nk = (int64_t)n_old * c->d.K;
    if (c->d.K == 0) return LSHMF_OK;
    if (nk > 0) {
        LSHMF_HIP(hipMemcpyAsync(c->old_jk, c->t.JK, sizeof(int32_t) * nk, hipMemcpyDeviceToDevice, s));
        LSHMF_HIP(hipMemcpyAsync(c->old_w, c->t.W, sizeof(float) * nk, hipMemcpyDeviceToDevice, s));
        LSHMF_HIP(hipMemcpyAsync(c->old_c, c->t.C, sizeof(float) * nk, hipMemcpyDeviceToDevice, s));
    }
    LSHMF_TRY(neighbours_for(c, 0, c->N, seed_fill, s));
    if (nk > 0) {
        hipLaunchKernelGGL(k_remap_slots, dim3(grid_for((int64_t)n_old * kWave)), dim3(256), 0, s, c->old_jk,
                           c->old_w, c->old_c, c->t.JK, n_old, c->d.K, c->t.W, c->t.C);
        LSHMF_LAUNCHED("k_remap_slots");
    }
    return LSHMF_OK;
}

int build_neighbours(lshmf_ctx* c, const void* R, uint64_t seed_fill, hipStream_t s)
{
    c->timed = false;
    LSHMF_TRY(mark(c, 0, s));
    LSHMF_TRY(hash_clear(c, 0, c->N, s));
    LSHMF_TRY(hash_add(c, c->col_ptr, c->csc_row, c->csc_rc, c->nnz, R, s));
    LSHMF_TRY(mark(c, 1, s));
    LSHMF_TRY(signs(c, s));
    LSHMF_TRY(mark(c, 2, s));
    LSHMF_TRY(neighbours_for(c, 0, c->N, seed_fill, s));
    LSHMF_TRY(stream_codes(c, c->train, s));
    LSHMF_TRY(mark(c, 5, s));
    return LSHMF_OK;
}

}  // namespace lshmf
