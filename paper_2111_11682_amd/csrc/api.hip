// C ABI of liblshmf: validation, arena layout and the entry points declared
// in include/lshmf.h.  No C++ exception crosses this boundary.
#include <cstring>
#include <new>

#include "common.hpp"

namespace lshmf {
const char* last_error();
int ingest(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n, hipStream_t s);
int build_neighbours(lshmf_ctx* c, const void* R, uint64_t seed_fill, hipStream_t s);
int build_stream(lshmf_ctx* c, Stream& st, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n,
                 hipStream_t s);
int stream_codes(lshmf_ctx* c, Stream& st, hipStream_t s);
int run_sgd(lshmf_ctx* c, Stream& st, const lshmf_hparams* hp, int epoch, int upd, hipStream_t s);
int run_online(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n, int32_t M_new,
               int32_t N_new, const void* R, uint64_t seed_fill, const lshmf_hparams* hp, int epoch,
               int passes, uint32_t flags, hipStream_t s, bool refresh = true);
int run_loss(lshmf_ctx* c, const lshmf_hparams* hp, double* out, hipStream_t s);
int run_predict(lshmf_ctx* c, const int32_t* qu, const int32_t* qi, int64_t n, float* out, hipStream_t s);
int run_rmse(lshmf_ctx* c, const float* pred, const uint8_t* rc, int64_t n, double* out, hipStream_t s);
int refresh_bf16(lshmf_ctx* c, int64_t m0, int64_t m1, int64_t n0, int64_t n1, hipStream_t s);

namespace {

struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

void carve_stream(Carver& k, Stream& st, int64_t cap, int64_t P, int nstride)
{
    st.cap = cap;
    st.pk = k.take<uint32_t>(cap + kStreamPad);
    st.sj = k.take<int32_t>(cap);
    st.dep = k.take<int32_t>(cap);
    st.link = k.take<uint32_t>(cap + kStreamPad);
    st.nib = k.take<uint8_t>((size_t)(cap + kStreamPad) * nstride);
    st.blk_ptr = k.take<int64_t>(P * P + 1);
    st.blk_seg = k.take<int64_t>(P * P + 1);
    st.seg_col = k.take<int32_t>(cap);
    st.seg_start = k.take<int64_t>(cap + 1);
    st.blk_slots = k.take<int32_t>(P * P);
    st.blk_order = k.take<int32_t>(P * P);
    st.blk_run = k.take<int32_t>(2 * P * P);
    st.heavy = k.take<int32_t>(2 * P);
    st.hcounts.assign((size_t)(2 * P), 0);
    st.stats = k.take<int64_t>(4);
}

int64_t max3(int64_t a, int64_t b, int64_t c)
{
    const int64_t m = a > b ? a : b;
    return m > c ? m : c;
}

// One walk over the arena, used both to size it (base == nullptr) and to
// assign the regions.  Everything is sized for the capacities in c->d.
size_t carve(lshmf_ctx* c, char* base)
{
    const lshmf_dims& d = c->d;
    const int64_t nz = d.nnz_cap, bc = d.batch_cap, Mc = d.M_cap, Nc = d.N_cap, P = c->P;
    const int64_t nq = (int64_t)d.q * Nc;
    Carver k{base};
    c->coo_u = k.take<int32_t>(nz);
    c->coo_i = k.take<int32_t>(nz);
    c->coo_rc = k.take<uint8_t>(nz);
    c->row_ptr = k.take<int64_t>(Mc + 1);
    c->csr_col = k.take<int32_t>(nz);
    c->csr_rc = k.take<uint8_t>(nz);
    c->col_ptr = k.take<int64_t>(Nc + 1);
    c->csc_row = k.take<int32_t>(nz);
    c->csc_rc = k.take<uint8_t>(nz);
    // the second buffers are needed only when online batches grow the store
    const int64_t nz2 = bc > 0 ? nz : 0;
    c->row_ptr_alt = k.take<int64_t>(bc > 0 ? Mc + 1 : 0);
    c->csr_col_alt = k.take<int32_t>(nz2);
    c->csr_rc_alt = k.take<uint8_t>(nz2);
    c->col_ptr_alt = k.take<int64_t>(bc > 0 ? Nc + 1 : 0);
    c->csc_row_alt = k.take<int32_t>(nz2);
    c->csc_rc_alt = k.take<uint8_t>(nz2);
    carve_stream(k, c->train, nz, P, c->nstride);
    for (Stream& st : c->phase) carve_stream(k, st, bc, P, c->nstride);
    c->bat_u = k.take<int32_t>(bc);
    c->bat_i = k.take<int32_t>(bc);
    c->bat_rc = k.take<uint8_t>(bc);
    c->bcol_ptr = k.take<int64_t>(Nc + 1);
    c->bcsc_row = k.take<int32_t>(bc);
    c->bcsc_rc = k.take<uint8_t>(bc);
    c->brow_ptr = k.take<int64_t>(Mc + 1);
    c->bcsr_col = k.take<int32_t>(bc);
    c->bcsr_rc = k.take<uint8_t>(bc);
    c->irank = k.take<int32_t>(Nc);
    c->urank = k.take<int32_t>(Mc);
    c->e2s = k.take<int32_t>(nz > bc ? nz : bc);
    c->trash = k.take<float>(1024);
    const int64_t cn = max3(max3(2 * Mc, 2 * Nc, P * P), max3(nz, nq, bc), 4);
    c->cnt = k.take<int64_t>(cn + 2);
    c->sort_n = max3(max3(nz, nq, bc), max3(Nc, Mc, P * P), 0) + 2;
    c->sk[0] = k.take<uint64_t>(c->sort_n);
    c->sk[1] = k.take<uint64_t>(c->sort_n);
    c->sv[0] = k.take<uint32_t>(c->sort_n);
    c->sv[1] = k.take<uint32_t>(c->sort_n);
    const size_t hist_n = radix_hist_elems(c->sort_n);
    c->hist = k.take<int64_t>(hist_n);
    size_t scan_n = scan_tmp_elems((int64_t)hist_n);
    const size_t scan_n2 = scan_tmp_elems(c->sort_n);
    if (scan_n2 > scan_n) scan_n = scan_n2;
    c->scan_tmp = k.take<int64_t>(scan_n);
    c->red = k.take<double>(8192);
    c->bu_s = k.take<float>(Mc);
    c->bv_s = k.take<float>(Nc);
    c->nbr_b0 = k.take<float>((size_t)Nc * d.K);
    c->bitem = k.take<int32_t>(nq);
    c->bbegin = k.take<int32_t>(nq + 1);
    c->bpos = k.take<int32_t>(nq);
    const int64_t nk_old = Nc * (int64_t)d.K;  // a rebuild keeps the old lists, w and c here
    c->old_jk = k.take<int32_t>(nk_old);
    c->old_w = k.take<float>(nk_old);
    c->old_c = k.take<float>(nk_old);
    c->err = k.take<int32_t>(64);
    return (k.off + 255) & ~size_t(255);
}

int validate(const lshmf_dims* d)
{
    if (!d) {
        set_error("dims is NULL");
        return LSHMF_EINVAL;
    }
    const int64_t B = (int64_t)d->G * d->p * d->q;
    if (d->M < 1 || d->N < 2 || d->M >= (1 << 28)) {
        set_error("need 1 <= M < 2^28 and N >= 2 (M=%d N=%d)", d->M, d->N);
        return LSHMF_EINVAL;
    }
    if (d->F < 1 || d->F > 256) {
        set_error("F=%d outside 1..256", d->F);
        return LSHMF_EINVAL;
    }
    if (d->K < 0 || d->K > 128 || d->K > d->N - 1) {
        set_error("K=%d outside 0..min(128, N-1)", d->K);
        return LSHMF_EINVAL;
    }
    if (d->G < 1 || d->p < 1 || d->q < 1 || B > 8192 || (int64_t)d->G * d->p > 56 || d->q > 4096 ||
        d->G * d->p + bits_for((uint64_t)d->q) > 64) {
        set_error("hash shape G=%d p=%d q=%d: need G*p*q <= 8192, G*p <= 56, q <= 4096 and G*p + "
                  "ceil(log2 q) <= 64", d->G, d->p, d->q);
        return LSHMF_EINVAL;
    }
    if (d->hash_family != LSHMF_SIMLSH && d->hash_family != LSHMF_RPCOS && d->hash_family != LSHMF_MINHASH) {
        set_error("hash_family=%d is none of LSHMF_SIMLSH, LSHMF_RPCOS, LSHMF_MINHASH", d->hash_family);
        return LSHMF_EINVAL;
    }
    if ((d->model != LSHMF_NEIGHBOURHOOD && d->model != LSHMF_PLAIN_MF) || (d->model == LSHMF_PLAIN_MF && d->K != 0)) {
        set_error("model=%d: LSHMF_NEIGHBOURHOOD, or LSHMF_PLAIN_MF with K = 0 (K=%d)", d->model, d->K);
        return LSHMF_EINVAL;
    }
    if (d->hash_family == LSHMF_MINHASH && d->G > 32) {
        set_error("minHash keeps at most the 32 bits of a minimum per hash (G=%d)", d->G);
        return LSHMF_EINVAL;
    }
    if (d->rscale != 1 && d->rscale != 2) {
        set_error("rscale=%d must be 1 or 2", d->rscale);
        return LSHMF_EINVAL;
    }
    if (d->psi_exp < 1 || d->psi_exp > 4) {
        set_error("psi_exp=%d outside 1..4", d->psi_exp);
        return LSHMF_EINVAL;
    }
    // |acc| <= M * 15^psi_exp must fit int32
    double bound = (double)(d->M_cap > d->M ? d->M_cap : d->M);
    for (int e = 0; e < d->psi_exp; ++e) bound *= 15.0;
    if (bound >= 2147483647.0) {
        set_error("M * 15^psi_exp overflows the int32 hash sums");
        return LSHMF_EINVAL;
    }
    if (d->n_strata < 1 || d->n_strata > 4096) {
        set_error("n_strata=%d outside 1..4096", d->n_strata);
        return LSHMF_EINVAL;
    }
    if (d->storage != LSHMF_FP32 && d->storage != LSHMF_BF16 && d->storage != LSHMF_BF16_U) {
        set_error("storage=%d is none of LSHMF_FP32, LSHMF_BF16, LSHMF_BF16_U", d->storage);
        return LSHMF_EINVAL;
    }
    if (d->nnz < 0 || d->nnz >= ((int64_t)1 << 31)) {
        set_error("nnz=%lld outside [0, 2^31)", (long long)d->nnz);
        return LSHMF_EINVAL;
    }
    if (d->M_cap < 0 || d->N_cap < 0 || d->nnz_cap < 0 || d->batch_cap < 0) {
        set_error("negative capacity");
        return LSHMF_EINVAL;
    }
    if (d->M_cap >= (1 << 28) || d->nnz_cap >= ((int64_t)1 << 31) || d->batch_cap >= ((int64_t)1 << 31)) {
        set_error("capacities must stay below M_cap 2^28, nnz_cap and batch_cap 2^31");
        return LSHMF_EINVAL;
    }
    if ((d->M_cap && d->M_cap < d->M) || (d->N_cap && d->N_cap < d->N) || (d->nnz_cap && d->nnz_cap < d->nnz)) {
        set_error("a capacity is below its initial size (M_cap=%d M=%d N_cap=%d N=%d nnz_cap=%lld nnz=%lld)",
                  d->M_cap, d->M, d->N_cap, d->N, (long long)d->nnz_cap, (long long)d->nnz);
        return LSHMF_EINVAL;
    }
    return LSHMF_OK;
}

}  // namespace
}  // namespace lshmf

using namespace lshmf;

extern "C" {

int lshmf_create(const lshmf_dims* dims, lshmf_ctx** out)
{
    if (!out) {
        set_error("out is NULL");
        return LSHMF_EINVAL;
    }
    *out = nullptr;
    LSHMF_TRY(validate(dims));
    lshmf_ctx* c = new (std::nothrow) lshmf_ctx();
    if (!c) {
        set_error("out of host memory");
        return LSHMF_EINVAL;
    }
    c->d = *dims;
    if (c->d.M_cap == 0) c->d.M_cap = dims->M;
    if (c->d.N_cap == 0) c->d.N_cap = dims->N;
    if (c->d.nnz_cap == 0) c->d.nnz_cap = dims->nnz;
    c->M = dims->M;
    c->N = dims->N;
    c->nnz = 0;
    c->B = dims->G * dims->p * dims->q;
    c->words = (c->B + 31) / 32;
    c->pG = dims->G * dims->p;
    c->P = dims->n_strata;
    c->nstride = (((dims->K + 1) / 2) + 3) & ~3;
    carve(c, nullptr);
    *out = c;
    return LSHMF_OK;
}

void lshmf_destroy(lshmf_ctx* ctx)
{
    if (!ctx) return;
    for (hipEvent_t& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

int lshmf_set_timing(lshmf_ctx* ctx, int32_t enable)
{
    if (!ctx) {
        set_error("lshmf_set_timing: NULL context");
        return LSHMF_EINVAL;
    }
    if (enable && !ctx->ev[0])
        for (hipEvent_t& e : ctx->ev) LSHMF_HIP(hipEventCreate(&e));
    ctx->timing = enable != 0;
    ctx->timed = false;
    return LSHMF_OK;
}

int lshmf_lsh_phase_ms(lshmf_ctx* ctx, double* out)
{
    if (!ctx || !out) {
        set_error("lshmf_lsh_phase_ms: NULL argument");
        return LSHMF_EINVAL;
    }
    if (!ctx->timed) {
        set_error("lshmf_lsh_phase_ms: no timed neighbour search since timing was enabled");
        return LSHMF_ESTATE;
    }
    LSHMF_HIP(hipEventSynchronize(ctx->ev[5]));
    for (int k = 0; k < 5; ++k) {
        float ms = 0.0f;
        LSHMF_HIP(hipEventElapsedTime(&ms, ctx->ev[k], ctx->ev[k + 1]));
        out[k] = ms;
    }
    return LSHMF_OK;
}

int lshmf_arena_bytes(const lshmf_ctx* ctx, size_t* bytes)
{
    if (!ctx || !bytes) {
        set_error("NULL argument");
        return LSHMF_EINVAL;
    }
    lshmf_ctx tmp = *ctx;
    *bytes = carve(&tmp, nullptr);
    return LSHMF_OK;
}

int lshmf_bind(lshmf_ctx* ctx, const lshmf_tables* t, void* d_arena, size_t arena_bytes)
{
    if (!ctx || !t || !d_arena) {
        set_error("NULL argument");
        return LSHMF_EINVAL;
    }
    // with K = 0 the neighbour tables hold nothing and may be NULL
    const bool nbr = ctx->d.K > 0;
    if ((!t->U && ctx->d.storage != LSHMF_BF16_U) || !t->V || !t->bu || !t->bv || (nbr && (!t->W || !t->C || !t->JK)) || !t->acc || !t->sig ||
        !t->b0 || !t->bh0 || !t->mu) {
        set_error("a table pointer is NULL");
        return LSHMF_EINVAL;
    }
    if (ctx->d.storage != LSHMF_FP32 && (!t->U16 || !t->V16 || (nbr && (!t->W16 || !t->C16)))) {
        set_error("storage modes BF16 and BF16_U need the U16, V16, W16 and C16 tables");
        return LSHMF_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(d_arena) & 255) {
        set_error("arena must be 256-byte aligned");
        return LSHMF_EINVAL;
    }
    const size_t need = carve(ctx, nullptr);
    if (arena_bytes < need) {
        set_error("arena of %zu bytes, need %zu", arena_bytes, need);
        return LSHMF_ECAPACITY;
    }
    carve(ctx, static_cast<char*>(d_arena));
    ctx->t = *t;
    ctx->bound = true;
    ctx->ingested = ctx->neighbours = false;
    return LSHMF_OK;
}

int lshmf_ingest(lshmf_ctx* ctx, const int32_t* d_u, const int32_t* d_i, const uint8_t* d_rc, int64_t n,
                 lshmf_stream_t stream)
{
    if (!ctx || !ctx->bound) {
        set_error("context not bound");
        return LSHMF_ESTATE;
    }
    if (n < 0 || n > ctx->d.nnz_cap) {
        set_error("ingest: n=%lld outside [0, nnz_cap=%lld]", (long long)n, (long long)ctx->d.nnz_cap);
        return LSHMF_EINVAL;
    }
    if (n > 0 && (!d_u || !d_i || !d_rc)) {
        set_error("ingest: NULL rating array");
        return LSHMF_EINVAL;
    }
    ctx->ingested = ctx->neighbours = false;
    ctx->M = ctx->d.M;
    ctx->N = ctx->d.N;
    LSHMF_TRY(ingest(ctx, d_u, d_i, d_rc, n, reinterpret_cast<hipStream_t>(stream)));
    ctx->ingested = true;
    return LSHMF_OK;
}

int build_lsh_neighbours(lshmf_ctx* ctx, const void* d_rand, uint64_t seed_fill, lshmf_stream_t stream)
{
    if (!ctx || !ctx->ingested) {
        set_error("build_lsh_neighbours: ratings not ingested");
        return LSHMF_ESTATE;
    }
    if (!d_rand) {
        set_error("build_lsh_neighbours: the random draws are NULL");
        return LSHMF_EINVAL;
    }
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    LSHMF_TRY(build_neighbours(ctx, d_rand, seed_fill, s));
    LSHMF_TRY(refresh_bf16(ctx, 0, ctx->M, 0, ctx->N, s));
    ctx->neighbours = true;
    return LSHMF_OK;
}

// The training stream of the whole store, laid out again when online batches
// grew the store, with neighbour codes for the current lists.
static int ensure_train(lshmf_ctx* ctx, hipStream_t s)
{
    if (ctx->train_stale) {
        LSHMF_TRY(build_stream(ctx, ctx->train, ctx->coo_u, ctx->coo_i, ctx->coo_rc, ctx->nnz, s));
        ctx->train_stale = false;
    }
    if (!ctx->train.codes) LSHMF_TRY(stream_codes(ctx, ctx->train, s));
    return LSHMF_OK;
}

int lshmf_loss(lshmf_ctx* ctx, const lshmf_hparams* hp, double* d_loss, lshmf_stream_t stream)
{
    if (!ctx || !ctx->neighbours) {
        set_error("lshmf_loss: neighbours not built");
        return LSHMF_ESTATE;
    }
    if (!hp || !d_loss) {
        set_error("lshmf_loss: NULL argument");
        return LSHMF_EINVAL;
    }
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    LSHMF_TRY(ensure_train(ctx, s));
    return run_loss(ctx, hp, d_loss, s);
}

int sgd_epoch(lshmf_ctx* ctx, const lshmf_hparams* hp, int32_t epoch, double* d_loss_or_null,
              lshmf_stream_t stream)
{
    if (!ctx || !ctx->neighbours) {
        set_error("sgd_epoch: neighbours not built");
        return LSHMF_ESTATE;
    }
    if (!hp || epoch < 0) {
        set_error("sgd_epoch: bad hyper-parameters or epoch");
        return LSHMF_EINVAL;
    }
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    LSHMF_TRY(ensure_train(ctx, s));
    LSHMF_TRY(run_sgd(ctx, ctx->train, hp, epoch, 3, s));
    // the SGD writes only the FP32 masters; the BF16 copies follow in one pass
    LSHMF_TRY(refresh_bf16(ctx, 0, ctx->M, 0, ctx->N, s));
    return d_loss_or_null ? run_loss(ctx, hp, d_loss_or_null, s) : LSHMF_OK;
}

int lshmf_check(lshmf_ctx* ctx, lshmf_stream_t stream)
{
    if (!ctx || !ctx->bound) {
        set_error("lshmf_check: context not bound");
        return LSHMF_ESTATE;
    }
    return sync_status(ctx, reinterpret_cast<hipStream_t>(stream));
}

int online_update(lshmf_ctx* ctx, const int32_t* d_u, const int32_t* d_i, const uint8_t* d_rc, int64_t n,
                  int32_t M_new, int32_t N_new, const void* d_rand, uint64_t seed_fill, const lshmf_hparams* hp,
                  int32_t epoch, int32_t passes, uint32_t flags, lshmf_stream_t stream)
{
    if (!ctx || !ctx->neighbours) {
        set_error("online_update: neighbours not built");
        return LSHMF_ESTATE;
    }
    if (!hp || epoch < 0 || passes < 0 || !d_rand || n < 0 || (n > 0 && (!d_u || !d_i || !d_rc)) ||
        (flags & ~(uint32_t)LSHMF_REBUILD_NBRS)) {
        set_error("online_update: bad arguments");
        return LSHMF_EINVAL;
    }
    if (M_new < ctx->M || N_new < ctx->N) {
        set_error("online_update: M_new=%d, N_new=%d below the current %d x %d", M_new, N_new, ctx->M, ctx->N);
        return LSHMF_EINVAL;
    }
    if (M_new > ctx->d.M_cap || N_new > ctx->d.N_cap || n > ctx->d.batch_cap || ctx->nnz + n > ctx->d.nnz_cap) {
        set_error("online_update: %d x %d with %lld + %lld ratings exceeds the capacities %d x %d, batch %lld, "
                  "store %lld", M_new, N_new, (long long)ctx->nnz, (long long)n, ctx->d.M_cap, ctx->d.N_cap,
                  (long long)ctx->d.batch_cap, (long long)ctx->d.nnz_cap);
        return LSHMF_ECAPACITY;
    }
    return run_online(ctx, d_u, d_i, d_rc, n, M_new, N_new, d_rand, seed_fill, hp, epoch, passes, flags,
                      reinterpret_cast<hipStream_t>(stream));
}

int predict(lshmf_ctx* ctx, const int32_t* d_u, const int32_t* d_i, int64_t n, float* d_out,
            lshmf_stream_t stream)
{
    if (!ctx || !ctx->neighbours) {
        set_error("predict: neighbours not built");
        return LSHMF_ESTATE;
    }
    if (n < 0 || (n > 0 && (!d_u || !d_i || !d_out))) {
        set_error("predict: bad query arrays");
        return LSHMF_EINVAL;
    }
    return run_predict(ctx, d_u, d_i, n, d_out, reinterpret_cast<hipStream_t>(stream));
}

int lshmf_rmse(lshmf_ctx* ctx, const float* d_pred, const uint8_t* d_rc, int64_t n, double* d_out,
               lshmf_stream_t stream)
{
    if (!ctx || !ctx->bound) {
        set_error("lshmf_rmse: context not bound");
        return LSHMF_ESTATE;
    }
    if (n < 0 || !d_out || (n > 0 && (!d_pred || !d_rc))) {
        set_error("lshmf_rmse: bad arguments");
        return LSHMF_EINVAL;
    }
    return run_rmse(ctx, d_pred, d_rc, n, d_out, reinterpret_cast<hipStream_t>(stream));
}

int lshmf_sync_storage(lshmf_ctx* ctx, lshmf_stream_t stream)
{
    if (!ctx || !ctx->bound) {
        set_error("lshmf_sync_storage: context not bound");
        return LSHMF_ESTATE;
    }
    return refresh_bf16(ctx, 0, ctx->M, 0, ctx->N, reinterpret_cast<hipStream_t>(stream));
}

int lshmf_export_layout(const lshmf_ctx* ctx, lshmf_layout* out)
{
    if (!ctx || !out || !ctx->bound) {
        set_error("lshmf_export_layout: context not bound");
        return LSHMF_ESTATE;
    }
    const Stream& st = ctx->train;
    out->pk = st.pk;
    out->sj = st.sj;
    out->dep = st.dep;
    out->nib = st.nib;
    out->blk_ptr = st.blk_ptr;
    out->blk_seg = st.blk_seg;
    out->seg_col = st.seg_col;
    out->seg_start = st.seg_start;
    out->row_ptr = ctx->row_ptr;
    out->csr_col = ctx->csr_col;
    out->csr_rc = ctx->csr_rc;
    out->col_ptr = ctx->col_ptr;
    out->csc_row = ctx->csc_row;
    out->csc_rc = ctx->csc_rc;
    out->err = ctx->err;
    out->nstride = ctx->nstride;
    out->P = ctx->P;
    out->M = ctx->M;
    out->N = ctx->N;
    out->nnz = ctx->nnz;
    return LSHMF_OK;
}

const char* lshmf_last_error(void) { return lshmf::last_error(); }

}  // extern "C"
