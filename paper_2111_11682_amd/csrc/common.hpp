// Internal declarations shared by the HIP sources of liblshmf.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "lshmf.h"

struct lshmf_ctx;

namespace lshmf {

constexpr int kWave = 64;
constexpr int kStreamPad = 64;  // zeroed records after the stream arrays (read-ahead of the SGD)
constexpr int kLightNnz = 64;   // SGD blocks with at most this many ratings run in teams

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

#define LSHMF_TRY(expr)                                   \
    do {                                                  \
        int st_ = (expr);                                 \
        if (st_ != LSHMF_OK) return st_;                  \
    } while (0)

#define LSHMF_HIP(expr)                                   \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return ::lshmf::hip_fail(e_, #expr); \
    } while (0)

#define LSHMF_LAUNCHED(name)                              \
    do {                                                  \
        hipError_t e_ = hipGetLastError();                \
        if (e_ != hipSuccess) return ::lshmf::hip_fail(e_, name); \
    } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int bits_for(uint64_t v)  // bits needed to represent values in [0, v)
{
    int b = 0;
    while (b < 64 && (v - 1) >> b) ++b;
    return b;
}

// ------------------------------------------------------- device primitives
// Exclusive prefix sum of n int64 values; out has n+1 entries, out[n] = total.
// in == out is allowed.  tmp must hold scan_tmp_elems(n) int64.
size_t scan_tmp_elems(int64_t n);
int scan_excl(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the low `bits` key bits.
// Input in keys[0]/vals[0]; the sorted pairs end in keys[r]/vals[r] where r
// is the returned index (0 or 1).  hist needs radix_hist_elems(n) int64.
size_t radix_hist_elems(int64_t n);
int radix_sort(uint64_t* keys[2], uint32_t* vals[2], int64_t n, int bits, int64_t* hist,
               int64_t* scan_tmp, hipStream_t s, int* result_index);

// Per-bin counts of idx[0..n) into cnt[0..nbins) (cnt zeroed by the call).
int count_bins(const int32_t* idx, int64_t n, int64_t* cnt, int64_t nbins, hipStream_t s);

// Synchronises s and reports the SGD status word c->err[0]: LSHMF_EDEVICE
// (with a message) when a dependency wait gave up, else LSHMF_OK.
int sync_status(lshmf_ctx* c, hipStream_t s);

// RMSE of n predictions against rating codes (Sec. 5.1), reduced in FP64 in a
// fixed order through kRmsePartials per-block partial sums kept in `partial`.
constexpr int kRmsePartials = 512;
int rmse_with(const float* pred, const uint8_t* rc, int64_t n, int rscale, double* partial, double* out,
              hipStream_t s);

// BF16 (round to nearest even) of n FP32 values.
int to_bf16_rows(const float* src, uint16_t* dst, int64_t n, hipStream_t s);

// BF16 copies (and bias snapshots) of every row after `core` phases of an
// online batch; see run_online.
int refresh_after_online(lshmf_ctx* c, int32_t M_old, int32_t N_old, uint32_t flags, hipStream_t s);

// Fills.
int fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s);
int fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
int fill_f32(float* p, int64_t n, float v, hipStream_t s);

}  // namespace lshmf

// ------------------------------------------------------------ the context
namespace lshmf {

// One stratified stream of ratings: the order an SGD pass visits them in.
// Stratum s runs blocks (b, (b+s) mod P) of users i mod P = b and items
// j mod P = (b+s) mod P; inside a block item runs go by decreasing degree
// (within the stream's own ratings, ties by id), users inside a run by
// decreasing degree too (ties by id).
struct Stream {
    int64_t cap = 0;           // ratings it can hold
    uint32_t* pk;              // cap + kStreamPad  (user << 4) | code
    int32_t* sj;               // cap               item
    int32_t* dep;              // cap               previous rating of the user in the block (local) or -1
    uint32_t* link;            // cap + kStreamPad  hand-over word (successor, predecessor, chain pos, slot)
    uint8_t* nib;              // (cap + kStreamPad) * nstride   neighbour codes
    int64_t* blk_ptr;          // P*P + 1
    int64_t* blk_seg;          // P*P + 1
    int32_t* seg_col;          // cap               item of each run
    int64_t* seg_start;        // cap + 1
    int32_t* blk_slots;        // P*P               mailbox slots per block
    int32_t* blk_order;        // P*P               dispatch order of each stratum's blocks: most ratings first
    int32_t* blk_run;          // 2 P*P             per stratum and dispatch position: the block's first run
                               //                   (segment) and its run count
    int32_t* heavy;            // 2P                per stratum: blocks with more than kLightNnz ratings, then
                               //                   blocks with any (both lead the dispatch order)
    std::vector<int32_t> hcounts;  // host copy of heavy (2P), read with the statistics
    int64_t n = 0;             // host copies after a build
    int64_t max_block_nnz = 0;
    int64_t max_block_slots = 0;
    int64_t nseg = 0;
    int64_t* stats;            // 4 (device) largest block, most slots, runs
    int64_t pending = 0;       // ratings laid out, statistics not read yet
    bool codes = false;        // nib valid for the current neighbour lists
};

}  // namespace lshmf

struct lshmf_ctx {
    lshmf_dims d;              // as created; M_cap, N_cap, nnz_cap resolved
    int32_t M, N;              // current users and items
    int64_t nnz;               // current ratings in the store
    int B;                     // hash bits G*p*q
    int words;                 // uint32 words per signature
    int pG;                    // band width in bits
    int P;                     // strata
    int nstride;               // bytes of neighbour codes per rating (K nibbles, padded)
    int64_t sort_n;            // capacity of the sort buffers

    lshmf_tables t;
    bool bound = false, ingested = false, neighbours = false;

    // rating store and its compressed copies (device)
    int32_t* coo_u;            // nnz_cap
    int32_t* coo_i;            // nnz_cap
    uint8_t* coo_rc;           // nnz_cap
    int64_t* row_ptr;          // M_cap+1   CSR by user
    int32_t* csr_col;          // nnz_cap   items, ascending per user
    uint8_t* csr_rc;           // nnz_cap
    int64_t* col_ptr;          // N_cap+1   CSC by item
    int32_t* csc_row;          // nnz_cap   users, ascending per item
    uint8_t* csc_rc;           // nnz_cap
    // second buffers of both: an online batch merges into them, then they swap
    int64_t* row_ptr_alt;
    int32_t* csr_col_alt;
    uint8_t* csr_rc_alt;
    int64_t* col_ptr_alt;
    int32_t* csc_row_alt;
    uint8_t* csc_rc_alt;

    lshmf::Stream train;       // all ratings of the store
    lshmf::Stream phase[3];    // online batch: new users / new items / the rest
    bool train_stale = false;  // the store grew since `train` was built

    // online batch scratch
    int32_t* bat_u;            // batch_cap  batch ratings grouped by phase
    int32_t* bat_i;
    uint8_t* bat_rc;
    int64_t* bcol_ptr;         // N_cap+1    CSC of the batch (hash sums, merge)
    int32_t* bcsc_row;         // batch_cap
    uint8_t* bcsc_rc;
    int64_t* brow_ptr;         // M_cap+1    CSR of the batch (merge)
    int32_t* bcsr_col;         // batch_cap
    uint8_t* bcsr_rc;

    // shared scratch
    int32_t* irank;            // N_cap   item order of the stream being built
    int32_t* urank;            // M_cap   user order of the stream being built
    int32_t* e2s;              // max(nnz_cap, batch_cap) rating -> stream position
    int64_t* cnt;              // counters / flags
    uint64_t* sk[2];           // sort keys
    uint32_t* sv[2];           // sort values
    int64_t* hist;             // radix histogram
    int64_t* scan_tmp;
    double* red;               // FP64 reduction partials
    float* trash;              // sink for loads/stores that must not touch a table
    float* nbr_b0;             // N_cap*K fixed baseline bh0 of each neighbour slot
    int32_t* bitem;            // q*N_cap  items sorted by (band, key)
    int32_t* bbegin;           // q*N_cap+1 bucket starts (by bucket id)
    int32_t* bpos;             // q*N_cap  bucket id of (band t, item j) at t*N + j
    int32_t* old_jk;           // N_cap*K  lists, w and c before a rebuild
    float* old_w;
    float* old_c;
    int32_t* err;              // device status words: [0] SGD waits, [1] input checks
    float* bu_s;               // M_cap  BF16 modes: snapshot of b that predict reads (refreshed with the copies)
    float* bv_s;               // N_cap  snapshot of bh

    // phase timing of the neighbour search (diagnostics)
    bool timing = false, timed = false;
    hipEvent_t ev[6] = {};
};

namespace lshmf {
// Records phase boundary k of the neighbour search when timing is on.
inline int mark(lshmf_ctx* c, int k, hipStream_t s)
{
    if (c->timing) {
        LSHMF_HIP(hipEventRecord(c->ev[k], s));
        if (k == 5) c->timed = true;
    }
    return LSHMF_OK;
}
}  // namespace lshmf
