// Online learning (Sec. 4.3, Alg. "Online Learning"): a batch of new ratings,
// possibly from new users and on new items, is folded into a trained model
// without rebuilding the similarity structure of the existing items.
//
//   1. the saved hash state (simLSH pre-sign sums of Eq. item_hash, or the
//      RP_cos sums / minHash minima) of the items the batch touches grows by
//      the batch's terms, new items starting empty, and all signatures are
//      recomputed;
//   2. existing items keep their neighbour lists; each new item gets its
//      top-K from the band collisions over all items (with the rebuild flag,
//      every list is searched again and w, c follow their neighbour ids);
//   3. mu and the existing fixed baselines stay; a new user's or item's fixed
//      baseline is the mean of its batch ratings minus mu;
//   4. `passes` times, three SGD phases over the batch, each in the
//      stratified order of its own ratings: ratings of new users on existing
//      items update only the user side, ratings on new items only the item
//      side, the rest both sides.
// The caller writes the initial factor rows u_i, v_j of the new ids before
// the call; the library zeroes their b_i, bh_j, w_j, c_j.  Every refusal
// (ids, codes, repeated pairs, a phase too large for one SGD block) comes
// before the store, the tables or the training stream change.
#include "common.hpp"

namespace lshmf {

int launch_id_checks(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n, int32_t M,
                     int32_t N, hipStream_t s, bool check_pairs);
int input_status(lshmf_ctx* c, int32_t M, int32_t N, hipStream_t s);
int compress(lshmf_ctx* c, const int32_t* major, const int32_t* minor, const uint8_t* rc, int64_t n,
             int64_t n_major, int64_t n_minor, int64_t* ptr, int32_t* idx, uint8_t* rc_out, hipStream_t s,
             int32_t* dup_flag);
int merge_compressed(lshmf_ctx* c, int32_t M_old, int32_t N_old, const int64_t* b_rptr, const int32_t* b_col,
                     const uint8_t* b_rrc, const int64_t* b_cptr, const int32_t* b_row, const uint8_t* b_crc,
                     hipStream_t s);
int build_stream_async(lshmf_ctx* c, Stream& st, const int32_t* u, const int32_t* it, const uint8_t* rc,
                       int64_t n, hipStream_t s);
void stream_finish(Stream& st, const int64_t* hstats);
int baselines_new(lshmf_ctx* c, const int32_t* id, const uint8_t* rc, int64_t n, int32_t first, int32_t count,
                  float* out, hipStream_t s);
int hash_add(lshmf_ctx* c, const int64_t* col_ptr, const int32_t* row, const uint8_t* rc, int64_t nnz,
             const void* R, hipStream_t s);
int hash_clear(lshmf_ctx* c, int64_t n0, int64_t n1, hipStream_t s);
int signs(lshmf_ctx* c, hipStream_t s);
int neighbours_for(lshmf_ctx* c, int32_t j_first, int32_t count, uint64_t seed_fill, hipStream_t s);
int rebuild_lists(lshmf_ctx* c, int32_t n_old, uint64_t seed_fill, hipStream_t s);
int stream_codes(lshmf_ctx* c, Stream& st, hipStream_t s);
int sgd_fits(const lshmf_ctx* c, const Stream& st);
int run_sgd(lshmf_ctx* c, Stream& st, const lshmf_hparams* hp, int epoch, int upd, hipStream_t s);
int refresh_bf16(lshmf_ctx* c, int64_t m0, int64_t m1, int64_t n0, int64_t n1, hipStream_t s);
int refresh_bf16_touched(lshmf_ctx* c, const int64_t* b_rptr, const int64_t* b_cptr, hipStream_t s);

namespace {

// Phase of each batch rating: 0 new user on an existing item, 1 new item,
// 2 the rest.  Keys for a stable sort by phase, the phase also as int32 for
// counting.
__global__ void k_phase_keys(const int32_t* u, const int32_t* it, int64_t n, int32_t M_old, int32_t N_old,
                             uint64_t* keys, uint32_t* vals, int32_t* phase)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int ph = it[x] >= N_old ? 1 : (u[x] >= M_old ? 0 : 2);
        keys[x] = (uint64_t)ph;
        vals[x] = (uint32_t)x;
        phase[x] = ph;
    }
}

__global__ void k_gather3(const uint32_t* order, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n,
                          int32_t* ou, int32_t* oi, uint8_t* orc)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = order[x];
        ou[x] = u[e];
        oi[x] = it[e];
        orc[x] = rc[e];
    }
}

unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 16384)
{
    int64_t b = ceil_div(n > 0 ? n : 1, threads);
    return (unsigned)(b > cap ? cap : b);
}

}  // namespace

// Checks the batch (ids and codes in range, no pair twice, none in the
// store) and splits it into its three phases, each laid out as its own
// stratified stream over the grown id ranges M_new x N_new, then checks each
// against the SGD kernel's per-block limits.  Arena scratch only: the store,
// the tables and the training stream are not touched.  Two synchronisations:
// the check word with the phase sizes, then the three streams' statistics.
static int check_and_layout(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n,
                            int32_t M_new, int32_t N_new, hipStream_t s)
{
    const int32_t M_old = c->M, N_old = c->N;
    LSHMF_TRY(launch_id_checks(c, u, it, rc, n, M_new, N_new, s, true));
    int64_t cnt[3] = {0, 0, 0};
    if (n > 0) {
        int32_t* phase = c->e2s;
        hipLaunchKernelGGL(k_phase_keys, dim3(grid_for(n)), dim3(256), 0, s, u, it, n, M_old, N_old, c->sk[0],
                           c->sv[0], phase);
        LSHMF_LAUNCHED("k_phase_keys");
        int ri = 0;
        LSHMF_TRY(radix_sort(c->sk, c->sv, n, 2, c->hist, c->scan_tmp, s, &ri));
        hipLaunchKernelGGL(k_gather3, dim3(grid_for(n)), dim3(256), 0, s, c->sv[ri], u, it, rc, n, c->bat_u,
                           c->bat_i, c->bat_rc);
        LSHMF_LAUNCHED("k_gather3");
        LSHMF_TRY(count_bins(phase, n, c->cnt, 3, s));
        LSHMF_HIP(hipMemcpyAsync(cnt, c->cnt, sizeof(cnt), hipMemcpyDeviceToHost, s));
    }
    LSHMF_TRY(input_status(c, M_new, N_new, s));
    // the phase streams are laid out over the grown ranges
    c->M = M_new;
    c->N = N_new;
    int status = LSHMF_OK;
    int64_t stats[3][4] = {};
    int64_t off = 0;
    for (int k = 0; k < 3 && status == LSHMF_OK; ++k) {
        status = build_stream_async(c, c->phase[k], c->bat_u + off, c->bat_i + off, c->bat_rc + off, cnt[k], s);
        if (status == LSHMF_OK && cnt[k] > 0) {
            Stream& ph = c->phase[k];
            hipError_t e = hipMemcpyAsync(stats[k], ph.stats, sizeof(stats[k]), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ph.hcounts.data(), ph.heavy, sizeof(int32_t) * ph.hcounts.size(),
                                   hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) status = hip_fail(e, "hipMemcpyAsync(stream stats)");
        }
        off += cnt[k];
    }
    if (status == LSHMF_OK) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) status = hip_fail(e, "hipStreamSynchronize(phase streams)");
    }
    for (int k = 0; k < 3 && status == LSHMF_OK; ++k) {
        stream_finish(c->phase[k], stats[k]);
        status = sgd_fits(c, c->phase[k]);
    }
    if (status != LSHMF_OK) {
        c->M = M_old;
        c->N = N_old;
    }
    return status;
}

// BF16 copies and bias snapshots after an online batch: every row after a
// rebuild (w, c moved with their ids), else the rows the SGD changed (the
// batch's users and items, from the batch's CSR and CSC) and the new ids.
int refresh_after_online(lshmf_ctx* c, int32_t M_old, int32_t N_old, uint32_t flags, hipStream_t s)
{
    if (flags & LSHMF_REBUILD_NBRS) return refresh_bf16(c, 0, c->M, 0, c->N, s);
    LSHMF_TRY(refresh_bf16_touched(c, c->brow_ptr, c->bcol_ptr, s));
    return refresh_bf16(c, M_old, c->M, N_old, c->N, s);
}

// refresh = false leaves the BF16 copies and bias snapshots of the batch's
// rows to a later refresh_after_online (the serving loop orders it after the
// queries that must not see the batch).
int run_online(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n, int32_t M_new,
               int32_t N_new, const void* R, uint64_t seed_fill, const lshmf_hparams* hp, int epoch,
               int passes, uint32_t flags, hipStream_t s, bool refresh)
{
    const int32_t M_old = c->M, N_old = c->N;
    const int K = c->d.K;
    // every refusal comes before the model, the store or the training stream change
    LSHMF_TRY(check_and_layout(c, u, it, rc, n, M_new, N_new, s));
    // the model can no longer be trained or queried as before until this call succeeds
    c->neighbours = false;
    c->train_stale = true;
    c->train.codes = false;

    // append the batch to the rating store
    if (n > 0) {
        LSHMF_HIP(hipMemcpyAsync(c->coo_u + c->nnz, u, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        LSHMF_HIP(hipMemcpyAsync(c->coo_i + c->nnz, it, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        LSHMF_HIP(hipMemcpyAsync(c->coo_rc + c->nnz, rc, n, hipMemcpyDeviceToDevice, s));
    }
    // the batch's own CSC (hash sums, merge) and CSR (merge)
    LSHMF_TRY(compress(c, it, u, rc, n, N_new, M_new, c->bcol_ptr, c->bcsc_row, c->bcsc_rc, s, nullptr));
    LSHMF_TRY(compress(c, u, it, rc, n, M_new, N_new, c->brow_ptr, c->bcsr_col, c->bcsr_rc, s, nullptr));

    // 1. the saved hash state grows by the batch, by item, then signatures
    LSHMF_TRY(hash_clear(c, N_old, N_new, s));
    LSHMF_TRY(hash_add(c, c->bcol_ptr, c->bcsc_row, c->bcsc_rc, n, R, s));
    LSHMF_TRY(signs(c, s));

    // learned parameters of the new ids start at zero
    LSHMF_TRY(fill_f32(c->t.bu + M_old, M_new - M_old, 0.0f, s));
    LSHMF_TRY(fill_f32(c->t.bv + N_old, N_new - N_old, 0.0f, s));
    LSHMF_TRY(fill_f32(c->t.W + (int64_t)N_old * K, (int64_t)(N_new - N_old) * K, 0.0f, s));
    LSHMF_TRY(fill_f32(c->t.C + (int64_t)N_old * K, (int64_t)(N_new - N_old) * K, 0.0f, s));

    // 3. fixed baselines of the new ids (before the neighbour baselines read them)
    LSHMF_TRY(baselines_new(c, u, rc, n, M_old, M_new - M_old, c->t.b0, s));
    LSHMF_TRY(baselines_new(c, it, rc, n, N_old, N_new - N_old, c->t.bh0, s));

    // R(i) now includes the batch: merged, not sorted again
    c->nnz += n;
    LSHMF_TRY(merge_compressed(c, M_old, N_old, c->brow_ptr, c->bcsr_col, c->bcsr_rc, c->bcol_ptr, c->bcsc_row,
                               c->bcsc_rc, s));

    // 2. neighbour lists of the new items only, or of every item on a rebuild
    if (flags & LSHMF_REBUILD_NBRS) LSHMF_TRY(rebuild_lists(c, N_old, seed_fill, s));
    else if (N_new > N_old) LSHMF_TRY(neighbours_for(c, N_old, N_new - N_old, seed_fill, s));

    // 4. the three phases of the batch
    for (int k = 0; k < 3; ++k) LSHMF_TRY(stream_codes(c, c->phase[k], s));
    static const int kUpd[3] = {1, 2, 3};  // user side, item side, both
    for (int p = 0; p < passes; ++p)
        for (int k = 0; k < 3; ++k) LSHMF_TRY(run_sgd(c, c->phase[k], hp, epoch, kUpd[k], s));
    if (refresh) LSHMF_TRY(refresh_after_online(c, M_old, N_old, flags, s));
    c->neighbours = true;
    return LSHMF_OK;
}

}  // namespace lshmf
