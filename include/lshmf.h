/*
 * liblshmf -- LSH-aggregated neighbourhood matrix factorisation on MI355X.
 *
 * C ABI of the HIP library.  Every entry point is asynchronous on the
 * caller's HIP stream, returns LSHMF_OK (0) or a negative status, and never
 * lets a C++ exception cross the boundary.  lshmf_last_error() returns a
 * thread-local message for the last failure.
 *
 * Ownership: the caller owns all device memory.  The library allocates no
 * device memory at all; it carves its internal buffers out of one caller
 * supplied arena whose size lshmf_arena_bytes() reports.  Host memory is used
 * only for the opaque context object.  All pointers named d_* are device
 * pointers; layouts are row-major and dense unless stated otherwise.
 *
 * Notation follows the paper (arXiv 2111.11682, Table "symbols"):
 * M users (rows, set I), N items (columns, set J), F factor rank, K
 * neighbours per item, ratings r_ij.  Ratings travel as integer codes
 * rc = rscale * r (rscale 1: integer ratings 1..5; rscale 2: half-steps
 * 0.5..5.0), so rc is in 1..15.
 */
#ifndef LSHMF_H
#define LSHMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden visibility; only these names are exported. */
#pragma GCC visibility push(default)

typedef struct ihipStream_t* lshmf_stream_t; /* hipStream_t; NULL = default stream */

enum {
    LSHMF_OK = 0,
    LSHMF_EINVAL = -1,    /* bad dimensions, null pointer, id out of range   */
    LSHMF_ESTATE = -2,    /* call order violated (e.g. sgd before neighbours) */
    LSHMF_ECAPACITY = -3, /* arena too small or a block too large for LDS     */
    LSHMF_EDEVICE = -4    /* a HIP runtime error; message has its string      */
};

/* Storage modes.  LSHMF_BF16: FP32 masters of U, V, W, C plus BF16 copies
 * that predict reads.  LSHMF_BF16_U: the user rows are stored only in BF16
 * (table U16; U is not used and may be NULL) -- the SGD reads them as BF16,
 * computes in FP32 and writes them back rounded to nearest even, so each
 * rating moves 4F bytes of u instead of 8F; V, W, C keep FP32 masters and
 * BF16 copies as in LSHMF_BF16.  Inside an SGD block a user's row passes
 * from one rating to the next in FP32. */
enum { LSHMF_FP32 = 0, LSHMF_BF16 = 1, LSHMF_BF16_U = 2 };

/* Hash families of the neighbour search (Sec. 4.1 simLSH; RP_cos and minHash
 * are the two other LSH families of the top-K comparison in Sec. 5.3). */
enum { LSHMF_SIMLSH = 0, LSHMF_RPCOS = 1, LSHMF_MINHASH = 2 };

/* online_update flags */
enum { LSHMF_REBUILD_NBRS = 1 };

/* Models (Sec. 4.2): the neighbourhood model of Eq. (rr) -- with K = 0 it is
 * biased MF -- or plain MF, rhat = u_i . v_j with only U and V learned, the
 * model of Alg. CUSGD++ (requires K = 0; mu, b, bh, b0, bh0 stay zero). */
enum { LSHMF_NEIGHBOURHOOD = 0, LSHMF_PLAIN_MF = 1 };

typedef struct lshmf_dims {
    int32_t M, N;      /* users, items                                       */
    int32_t F;         /* rank of U (M x F) and V (N x F), 1..256            */
    int32_t K;         /* neighbours per item, 0..128, K <= N - 1; K = 0 is  */
                       /* biased MF without the neighbour term (no w, c)     */
    int32_t G, p, q;   /* G bits per hash, p hashes ANDed per band, q bands
                          ORed (Sec. 4.1 coarse- and fine-grained hashing);
                          B = G*p*q <= 8192 bits, band width p*G <= 56 and
                          p*G + ceil(log2 q) <= 64; minHash needs G <= 32    */
    int32_t rscale;    /* rating code scale, 1 or 2                          */
    int32_t psi_exp;   /* Psi(r) = rc^psi_exp in the hash sums (2: Psi = r^2) */
    int32_t n_strata;  /* P: users and items split into P blocks by id mod P */
    int32_t storage;   /* LSHMF_FP32; LSHMF_BF16: BF16 copies of U, V, W, C
                          for serving next to the FP32 masters; LSHMF_BF16_U:
                          U stored in BF16 only (see the storage modes)     */
    int32_t hash_family; /* LSHMF_SIMLSH, LSHMF_RPCOS or LSHMF_MINHASH       */
    int32_t model;     /* LSHMF_NEIGHBOURHOOD or LSHMF_PLAIN_MF              */
    int32_t reserved;  /* 0                                                  */
    int64_t nnz;       /* ratings of the initial training set                */
    /* Capacities for online learning (0: the initial size; batch_cap 0: no
     * online batches).  Tables and the arena are sized for them.            */
    int32_t M_cap, N_cap;
    int64_t nnz_cap;   /* ratings the store holds, training set + batches    */
    int64_t batch_cap; /* most ratings one online_update call takes          */
} lshmf_dims;

/* Learning rates alpha and regularisers lambda, in the order
 * (b_i, bh_j, u_i, v_j, w_j, c_j) of Eq. (sgd_update); the rate of epoch t is
 * alpha / (1 + beta * t^1.5), Eq. (learn_rate). */
typedef struct lshmf_hparams {
    float alpha[6];
    float lambda[6];
    float beta;
    int32_t reserved;
} lshmf_hparams;

/* Model tables: caller-owned device buffers, FP32, row-major, sized for the
 * capacities M_cap and N_cap (M, N below):
 *   U  [M*F]   V  [N*F]          factor rows u_i, v_j              (Eq. rr, part 4)
 *   bu [M]     bv [N]            learned deviations b_i, bh_j       (Eq. rr, part 1)
 *   W  [N*K]   C  [N*K]          explicit / implicit influence w_j, c_j, slot k
 *                                 refers to neighbour JK[j*K + k]    (Eq. rr, parts 2, 3)
 *   JK [N*K]   int32             top-K neighbours, ascending ids per row
 *   acc[N*B]   int32             per-item hash state, kept for online learning:
 *                                simLSH pre-sign sums (int32); RP_cos FP32 sums
 *                                (bit patterns); minHash minima (uint32, the
 *                                first N*B/G entries)
 *   sig[N*ceil(B/32)] uint32     simLSH signatures, bit b at word b/32, bit b%32
 *   b0 [M]     bh0 [N]           fixed baseline deviations of the "simple case"
 *   mu [1]     double            global mean
 * U, V, bu, bv, W, C are read and written by sgd_epoch; the caller initialises
 * them (the paper's Alg. CULSH-MF takes the initial values as input).
 *
 * Storage mode LSHMF_BF16 adds U16 [M*F], V16 [N*F], W16 [N*K], C16 [N*K]:
 * BF16 bit patterns (round to nearest even) of the FP32 tables above, which
 * stay the masters that SGD reads and writes.  Every call that changes a
 * master row also rewrites its BF16 copy before it returns (one conversion
 * pass over the tables after the SGD); predict reads the copies, and
 * snapshots of b and bh taken at the same moments (kept in the arena).  The
 * pointers are ignored in mode LSHMF_FP32.  With K = 0, W, C, JK, W16 and C16
 * hold nothing and may be NULL.  In mode LSHMF_BF16_U, U16 is the only copy of
 * the user rows (the caller initialises U16; U is ignored and may be NULL). */
typedef struct lshmf_tables {
    float* U;
    float* V;
    float* bu;
    float* bv;
    float* W;
    float* C;
    int32_t* JK;
    int32_t* acc;
    uint32_t* sig;
    float* b0;
    float* bh0;
    double* mu;
    uint16_t* U16;
    uint16_t* V16;
    uint16_t* W16;
    uint16_t* C16;
} lshmf_tables;

typedef struct lshmf_ctx lshmf_ctx; /* opaque, host memory */

/* Creates a context for the given dimensions (validated here). */
int lshmf_create(const lshmf_dims* dims, lshmf_ctx** out);
void lshmf_destroy(lshmf_ctx* ctx);

/* Device bytes the library needs for its layout and scratch buffers. */
int lshmf_arena_bytes(const lshmf_ctx* ctx, size_t* bytes);

/* Binds caller-owned tables and arena (device pointers, 256-byte aligned
 * arena).  The pointers must stay valid until the context is destroyed. */
int lshmf_bind(lshmf_ctx* ctx, const lshmf_tables* tables, void* d_arena, size_t arena_bytes);

/* Ingest and layout of the training ratings (COO, d_u[n], d_i[n], d_rc[n],
 * n <= dims.nnz_cap; resets the model to dims.M x dims.N): CSR by user, CSC
 * by item, the stratified block stream and the fixed baselines mu, b0, bh0
 * (Sec. 3.2, the "simple case" means, reduced in FP64).  Ids outside
 * [0,M) x [0,N), codes outside 1..15 and a (u, i) pair given twice (R holds
 * one value per pair, Sec. 3.1) give LSHMF_EINVAL after a stream
 * synchronisation, with nothing bound to the model. */
int lshmf_ingest(lshmf_ctx* ctx, const int32_t* d_u, const int32_t* d_i, const uint8_t* d_rc,
                 int64_t n, lshmf_stream_t stream);

/* LSH neighbours without the N x N similarity matrix (Sec. 4.1, Eq.
 * item_hash and Alg. CULSH): per-item hash state and B-bit signatures, q band
 * keys of p*G bits, bucket collisions counted per item, the K most frequent
 * partners (ties by smaller id), a seeded random supplement when fewer than
 * K exist (SplitMix64(seed_fill, j*2^32 + a + 1) mod N, a = 0, 1, ...), rows
 * stored by ascending id.  Also resolves, for every training rating (i, j),
 * which neighbours of j user i has rated.  With K = 0 only acc and sig are
 * computed.  Requires lshmf_ingest.
 *
 * d_rand holds the random draws of the family, one row per user (M rows;
 * online batches read rows up to M_new):
 *   LSHMF_SIMLSH   the strings H_i: ceil(B/32) uint32 words, bit b at word
 *                  b/32, bit b%32; acc = sum Psi(r) (2 H_i - 1), bit = [acc >= 0]
 *   LSHMF_RPCOS    B FP32 Gaussian directions g_i; acc = sum r g_i in FP32,
 *                  raters of an item in ascending user id, one fused
 *                  multiply-add each; bit = [acc >= 0]
 *   LSHMF_MINHASH  B/G uint32 random values v_i (a random order of the
 *                  users per hash); acc = minimum of v_i over the raters,
 *                  hash h = its G low bits at signature bits [hG, (h+1)G)
 */
int build_lsh_neighbours(lshmf_ctx* ctx, const void* d_rand, uint64_t seed_fill,
                         lshmf_stream_t stream);

/* The objective of Eq. (loss_r) on the current tables, in FP64:
 * d_loss[0] = sum over the training ratings of (r - rhat)^2 (rhat of Eq. rr
 * in FP32, squared and summed in FP64) + lambda_b |b|^2 + lambda_bh |bh|^2 +
 * lambda_u |U|^2 + lambda_v |V|^2 + lambda_w |W|^2 + lambda_c |C|^2, with
 * lambda from hp and the w, c norms over every stored slot.  The reduction
 * order is fixed, so the value is reproducible.  Requires
 * build_lsh_neighbours. */
int lshmf_loss(lshmf_ctx* ctx, const lshmf_hparams* hp, double* d_loss, lshmf_stream_t stream);

/* One SGD epoch t (0-based) over all training ratings in the stratified
 * order: stratum s = 0..P-1 runs the P blocks (b, (b+s) mod P) of users
 * i mod P = b and items j mod P = (b+s) mod P; inside a block, runs of one
 * item by decreasing item degree (ties by smaller id), and inside a run users
 * by decreasing user degree (ties by smaller id); degrees count the ratings
 * of the pass.  Each rating applies Eq.
 * (sgd_update) with the prediction of Eq. (rr), N(i) the complement of R(i)
 * (the CULSH-MF adjustment), and the residual baseline of the w-term fixed to
 * the simple-case means.  Results do not depend on how blocks are scheduled.
 * When d_loss_or_null is not NULL, the objective after the epoch is written
 * there as by lshmf_loss.  Requires build_lsh_neighbours. */
int sgd_epoch(lshmf_ctx* ctx, const lshmf_hparams* hp, int32_t epoch, double* d_loss_or_null,
              lshmf_stream_t stream);

/* Online learning (Sec. 4.3, Alg. "Online Learning") of a batch of n new
 * ratings (d_u, d_i, d_rc as for lshmf_ingest) that may bring new users
 * [M, M_new) and new items [N, N_new):
 *   - the saved hash state acc grows by the batch's terms (rows of new items
 *     start empty) and every signature is recomputed (Eq. item_hash);
 *   - existing items keep JK; each new item gets its top-K from the band
 *     collisions over all N_new items, exactly as build_lsh_neighbours.
 *     With flags & LSHMF_REBUILD_NBRS every item's list is searched again
 *     instead, and the w, c values of the existing items follow their
 *     neighbour ids: a neighbour kept by the new list brings its values to
 *     its new slot, a new neighbour starts at 0 (a periodic rebuild for long
 *     streams; the paper keeps the old lists);
 *   - mu and the existing b0, bh0 stay; a new id's fixed baseline is the mean
 *     of its batch ratings minus mu;
 *   - `passes` rounds of three SGD phases at the rate of epoch `epoch`, each
 *     phase over its own ratings in the stratified order of sgd_epoch: (A) new
 *     users on existing items update only b_i, u_i; (B) ratings on new items
 *     update only bh_j, v_j, w_j, c_j; (C) the rest update both sides; R(i)
 *     includes the batch.
 * The caller writes U rows [M, M_new) (U16 rows in mode LSHMF_BF16_U) and V
 * rows [N, N_new) before the call;
 * the library zeroes bu, bv, W, C of the new ids.  d_H holds M_new rows.
 * The batch joins the training set of later sgd_epoch calls.  Exceeding a
 * capacity, or a batch phase too large for one SGD block (raise n_strata),
 * gives LSHMF_ECAPACITY; ids outside [0,M_new) x [0,N_new), bad codes, a
 * pair given twice in the batch or already in the store give LSHMF_EINVAL;
 * all before any table or the store is touched.  d_rand as for
 * build_lsh_neighbours, M_new rows.  Requires build_lsh_neighbours. */
int online_update(lshmf_ctx* ctx, const int32_t* d_u, const int32_t* d_i, const uint8_t* d_rc, int64_t n,
                  int32_t M_new, int32_t N_new, const void* d_rand, uint64_t seed_fill,
                  const lshmf_hparams* hp, int32_t epoch, int32_t passes, uint32_t flags,
                  lshmf_stream_t stream);

/* ---- Serving loop: continuous batching of online updates and queries ----
 *
 * lshmf_serve replays a request log against the model in arrival order, the
 * way a server takes the online sparse stream that motivates Sec. 4.3:
 *   - an update request is one online_update call (its initial factor rows of
 *     new ids come from d_U0 / d_V0); one that exceeds batch_cap or the free
 *     store is refused (status LSHMF_ECAPACITY) and leaves the model as it is;
 *   - consecutive query requests that have arrived by the time the GPU can
 *     take them are merged into one predict launch of at most
 *     max_query_batch pairs (a larger single request is refused); a query
 *     sees exactly the updates that arrived before it, so the answers do not
 *     depend on how requests were merged;
 *   - payload uploads and result downloads run on a copy stream beside the
 *     compute stream, double-buffered in the caller's device staging area;
 *   - in storage mode LSHMF_BF16, predict reads only the BF16 copies and the
 *     bias snapshots, which an update rewrites in its last step: queries then
 *     run on a stream of their own (created and destroyed by the call, default
 *     priority) beside the hashing, neighbour and SGD phases of the next
 *     update, and only that last step waits for the queries that arrived
 *     before it.  In the other modes queries and updates share the compute
 *     stream.  Either way a query sees exactly the updates that arrived before
 *     it, so answers do not depend on the overlap;
 *   - an update's upload waits until the previous update no longer reads the
 *     staging.
 * Request times are seconds from the start of the call; the loop waits for
 * arrivals in real time (all zero: back to back).  Host payload arrays
 * should be pinned for the copies to overlap. */
enum { LSHMF_REQ_UPDATE = 0, LSHMF_REQ_QUERY = 1 };

typedef struct lshmf_request {
    int32_t kind;            /* LSHMF_REQ_UPDATE or LSHMF_REQ_QUERY                  */
    int32_t M_new, N_new;    /* update: users and items after the batch              */
    int32_t reserved;
    int64_t offset;          /* first element of the payload (h_u/h_i/h_rc or h_qu/h_qi/h_pred) */
    int64_t n;               /* ratings or query pairs                               */
    double arrival;          /* seconds from the start of the call                   */
} lshmf_request;

typedef struct lshmf_serve_io {
    const lshmf_request* req;  /* host, n_req entries, arrivals non-decreasing      */
    int64_t n_req;
    const int32_t* h_u;        /* host update payload                               */
    const int32_t* h_i;
    const uint8_t* h_rc;
    const int32_t* h_qu;       /* host query payload                                */
    const int32_t* h_qi;
    float* h_pred;             /* host, answers at each query request's offset      */
    const float* d_U0;         /* device, initial rows of new users [M_cap*F]       */
    const float* d_V0;         /* device, initial rows of new items [N_cap*F]       */
    const void* d_rand;        /* device, hash-family draws of M_cap users          */
    uint64_t seed_fill;
    lshmf_hparams hp;
    int32_t epoch, passes;     /* online_update's learning-rate epoch and passes    */
    int64_t max_query_batch;   /* pairs per predict launch                          */
    void* d_stage;             /* device staging, lshmf_serve_stage_bytes() bytes   */
    size_t stage_bytes;
    double* h_start;           /* host out: launch time of each request (s)         */
    double* h_done;            /* host out: time its result was complete (s)        */
    int32_t* h_status;         /* host out: LSHMF_OK or the refusal status          */
} lshmf_serve_io;

/* Device staging bytes lshmf_serve needs for max_query_batch pairs. */
int lshmf_serve_stage_bytes(const lshmf_ctx* ctx, int64_t max_query_batch, size_t* bytes);

/* Runs the loop until every request is answered or refused.  compute and
 * copy must be different streams (NULL is not allowed).  Returns the first
 * hard failure (a HIP error or LSHMF_ESTATE); refusals are per request. */
int lshmf_serve(lshmf_ctx* ctx, const lshmf_serve_io* io, lshmf_stream_t compute, lshmf_stream_t copy);

/* Eq. (rr) for n query pairs (d_u[x], d_i[x]) -> d_out[x] (FP32), with R(i)
 * the user's training items.  Ids out of range give NaN for that query. */
int predict(lshmf_ctx* ctx, const int32_t* d_u, const int32_t* d_i, int64_t n, float* d_out,
            lshmf_stream_t stream);

/* Storage mode LSHMF_BF16: rewrites every BF16 copy from the FP32 masters,
 * for a caller that edited the masters itself.  build_lsh_neighbours does
 * the same; in mode LSHMF_FP32 this does nothing. */
int lshmf_sync_storage(lshmf_ctx* ctx, lshmf_stream_t stream);

/* RMSE of predictions against rating codes (Sec. 5.1), reduced in FP64 in a
 * fixed order: d_out[0] = sqrt(sum (rc/rscale - pred)^2 / n). */
int lshmf_rmse(lshmf_ctx* ctx, const float* d_pred, const uint8_t* d_rc, int64_t n,
               double* d_out, lshmf_stream_t stream);

/* lshmf_rmse for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * context and no arena.  Same arguments and result as lshmf_rmse, with the
 * rating scale passed directly (rscale 1 or 2); the value is bit-identical
 * to lshmf_rmse's.  Its FP64 partial sums live in a fixed 4 KiB device array
 * of the library (512 partials, whatever n), one per GPU, held until the
 * process ends; the first call on a device looks up that device's copy.
 * It calls no allocating routine.  Calls on one GPU share the array:
 * calls that overlap in time on the same GPU (different streams, or
 * different host threads) race and may return wrong values; calls ordered on
 * one stream do not.  The stream must belong to the current device.
 * LSHMF_EINVAL for a NULL d_out, n < 0, NULL data with n > 0 or another
 * rscale. */
int lshmf_rmse_noalloc(const float* d_pred, const uint8_t* d_rc, int64_t n, int32_t rscale,
                       double* d_out, lshmf_stream_t stream);

/* Phase timing of build_lsh_neighbours (diagnostics).  While enabled, the
 * call records HIP events at its phase boundaries on its stream (the events
 * are created here; nothing else changes).  lshmf_lsh_phase_ms waits for the
 * last event and writes the milliseconds of the phases of the last call:
 * out[0] hash state (projection, minima), out[1] signatures, out[2] band keys
 * and buckets, out[3] top-K lists and neighbour baselines, out[4] neighbour
 * codes of the training ratings.  LSHMF_ESTATE if nothing was timed. */
int lshmf_set_timing(lshmf_ctx* ctx, int32_t enable);
int lshmf_lsh_phase_ms(lshmf_ctx* ctx, double* out);

/* Synchronises the stream and reports the device status word: LSHMF_OK, or
 * LSHMF_EDEVICE when an SGD dependency wait gave up after its spin limit (a
 * broken hand-over; the tables are then not those of the stated order).  The
 * library's own synchronising calls (lshmf_ingest, online_update,
 * lshmf_serve and sgd_epoch when it lays the stream out again) report it too. */
int lshmf_check(lshmf_ctx* ctx, lshmf_stream_t stream);

/* Read-only device pointers into the arena, for inspection and tests: the
 * stratified stream (pk = user << 4 | code, sj = item, dep = previous rating
 * of the same user in the block or -1, nib = K 4-bit neighbour codes per
 * rating, nstride bytes each), block and segment ranges, and the CSR / CSC
 * copies of the training set.  Valid after lshmf_ingest (nib after
 * build_lsh_neighbours) until the next lshmf_bind; after online_update the
 * stream describes the previous training set until the next sgd_epoch lays
 * out the grown one. */
typedef struct lshmf_layout {
    const uint32_t* pk;
    const int32_t* sj;
    const int32_t* dep;
    const uint8_t* nib;
    const int64_t* blk_ptr;   /* P*P + 1, block b of stratum s at s*P + b */
    const int64_t* blk_seg;   /* P*P + 1 */
    const int32_t* seg_col;
    const int64_t* seg_start;
    const int64_t* row_ptr;   /* M + 1 */
    const int32_t* csr_col;
    const uint8_t* csr_rc;
    const int64_t* col_ptr;   /* N + 1 */
    const int32_t* csc_row;
    const uint8_t* csc_rc;
    const int32_t* err;       /* device status word: 0 while healthy; bit 1 set if
                                 an SGD dependency wait hit its spin limit */
    int32_t nstride;
    int32_t P;
    int32_t M, N;             /* current users and items                     */
    int64_t nnz;              /* ratings in the store                        */
} lshmf_layout;

int lshmf_export_layout(const lshmf_ctx* ctx, lshmf_layout* out);

/* Thread-local message describing the last non-OK status. */
const char* lshmf_last_error(void);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif

#endif /* LSHMF_H */
