/*
 * Plain FP64 CPU oracle for LSH-MF (arXiv 2111.11682).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
 * HIP path.  It is loaded by the tests, by the smoke check and by the CPU
 * baseline leg of the benchmark -- never by the product path.  It shares no
 * code, header, table or helper with the HIP library; the two only read the
 * same seeded inputs.
 *
 * Each function follows one passage of the paper and favours the plainest
 * formulation over speed:
 *   - simLSH coding ........................ Sec. 4.1, Eq. (item_hash)
 *   - coarse/fine banding, top-K ........... Sec. 4.1 "Coarse-grained and
 *                                            Fine-grained Hashing", Alg. CULSH
 *   - baseline means (the "simple case") ... Sec. 3.2, part (1) of Eq. (rr)
 *   - prediction ........................... Eq. (rr) with the CULSH-MF
 *                                            adjustment N(i) = J \ R(i)
 *   - SGD step ............................. Eq. (sgd_update)
 *   - learning-rate schedule ............... Eq. (learn_rate)
 *   - objective ............................ Eq. (loss_r)
 *   - RMSE ................................. Sec. 5.1
 *   - online update ........................ Sec. 4.3, Alg. "Online Learning"
 *   - neighbour-list rebuild with w, c
 *     following their neighbour ids ........ a reading (the paper keeps old
 *                                            lists; see orc_remap_slots)
 *   - RP_cos and minHash hash families ..... Sec. 5.3, the top-K comparison
 *                                            (Table of top-K methods)
 *
 * Readings where the paper is silent are documented next to the code that
 * takes them.  Random numbers: the user hash strings H_i and the initial
 * factors are inputs; the random supplement of the top-K list draws from
 * SplitMix64 (Steele, Lea, Flood 2014), written here from its definition.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* SplitMix64: output number c (c >= 1) of the stream started at `seed`.     */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + c * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* OpenMP threads of the parallel loops (timing on one thread or all).      */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* simLSH coding, Sec. 4.1 Eq. (item_hash).                                 */
/*   acc[j][b] = sum_{i rated j} Psi(r_ij) * Phi(H_i,b),  Phi(h) = 2h - 1     */
/*   sig[j][b] = Upsilon(acc[j][b]) = 1 if acc >= 0 else 0                    */
/* Psi(r) = rc^psi_exp with rc = rscale * r; a positive common factor does    */
/* not change any sign, so Psi on codes gives the same signature as Psi on r. */
/* Bits are LSB-first: bit b lives in word b/32 at position b%32.             */
/* ------------------------------------------------------------------------ */
static int64_t psi_of(int rc, int psi_exp)
{
    int64_t v = 1;
    for (int e = 0; e < psi_exp; ++e) v *= rc;
    return v;
}

static int hbit(const uint32_t* H, int words, int64_t i, int b)
{
    return (int)((H[i * words + b / 32] >> (b % 32)) & 1u);
}

/* acc[j][b] += Psi(r_ij) * Phi(H_i,b) over the given ratings (no reset).   */
/* The sums are integers, so their order does not matter: OpenMP threads    */
/* take disjoint ranges of bits b and each walks all ratings.               */
int orc_simlsh_add(int M, int N, int B, int64_t nnz, const int32_t* u, const int32_t* it,
                   const uint8_t* rc, const uint32_t* H, int psi_exp, int64_t* acc /* N*B */)
{
    if (M <= 0 || N <= 0 || B <= 0 || nnz < 0) return ORC_EINVAL;
    for (int64_t e = 0; e < nnz; ++e)
        if (u[e] < 0 || u[e] >= M || it[e] < 0 || it[e] >= N) return ORC_EINVAL;
    const int words = (B + 31) / 32;
#pragma omp parallel for schedule(dynamic, 1)
    for (int wd = 0; wd < words; ++wd) {
        const int b1 = (wd + 1) * 32 < B ? (wd + 1) * 32 : B;
        for (int64_t e = 0; e < nnz; ++e) {
            const int i = u[e], j = it[e];
            const int64_t w = psi_of(rc[e], psi_exp);
            for (int b = wd * 32; b < b1; ++b)
                acc[(int64_t)j * B + b] += w * (2 * hbit(H, words, i, b) - 1);
        }
    }
    return ORC_OK;
}

/* Upsilon: signature bit b of item j is 1 iff acc[j][b] >= 0. */
void orc_signs(int N, int B, const int64_t* acc, uint32_t* sig)
{
    const int words = (B + 31) / 32;
    memset(sig, 0, sizeof(uint32_t) * (size_t)N * words);
    for (int j = 0; j < N; ++j)
        for (int b = 0; b < B; ++b)
            if (acc[(int64_t)j * B + b] >= 0)
                sig[(int64_t)j * words + b / 32] |= 1u << (b % 32);
}

int orc_simlsh(int M, int N, int B, int64_t nnz, const int32_t* u, const int32_t* it,
               const uint8_t* rc, const uint32_t* H, int psi_exp,
               int64_t* acc /* N*B */, uint32_t* sig /* N*ceil(B/32) */)
{
    memset(acc, 0, sizeof(int64_t) * (size_t)(N > 0 ? N : 0) * (B > 0 ? B : 0));
    const int st = orc_simlsh_add(M, N, B, nnz, u, it, rc, H, psi_exp, acc);
    if (st != ORC_OK) return st;
    orc_signs(N, B, acc, sig);
    return ORC_OK;
}

/* Key of coarse band t: the p*G bits [t*p*G, (t+1)*p*G) of the signature,    */
/* i.e. p consecutive G-bit simLSH hashes that must all agree (AND).         */
uint64_t orc_band_key(const uint32_t* sig_row, int t, int G, int p)
{
    const int w = G * p;
    uint64_t key = 0;
    for (int x = 0; x < w; ++x) {
        const int b = t * w + x;
        key |= (uint64_t)((sig_row[b / 32] >> (b % 32)) & 1u) << x;
    }
    return key;
}

/* All band keys of every item: keys[j*q + t] = key_t(j). */
int orc_band_keys(int N, int B, int G, int p, int q, const uint32_t* sig, uint64_t* keys)
{
    if (G * p * q > B || G * p > 64) return ORC_EINVAL;
    const int words = (B + 31) / 32;
    for (int j = 0; j < N; ++j)
        for (int t = 0; t < q; ++t)
            keys[(int64_t)j * q + t] = orc_band_key(sig + (int64_t)j * words, t, G, p);
    return ORC_OK;
}

/* count_j(j') = number of bands t in [0,q) with key_t(j) == key_t(j').     */
/* Fine-grained hashing (OR over q bands) counts how often a pair collides. */
/* An item is not its own candidate: count_j(j) = 0.                        */
int orc_pair_counts(int N, int q, const uint64_t* keys, int j, int32_t* count /* N */)
{
    if (j < 0 || j >= N) return ORC_EINVAL;
    for (int jj = 0; jj < N; ++jj) {
        int c = 0;
        for (int t = 0; t < q; ++t)
            c += keys[(int64_t)j * q + t] == keys[(int64_t)jj * q + t];
        count[jj] = (jj == j) ? 0 : c;
    }
    return ORC_OK;
}

static int cmp_i32(const void* a, const void* b)
{
    const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Top-K by frequency, Sec. 4.1 and Alg. CULSH (the top-K search step):       */
/* candidates are the items sharing at least one band with j; take the K most */
/* frequent, ties by smaller id; if fewer than K exist, supplement with       */
/* random items x_a = SplitMix64(seed_fill, j*2^32 + a + 1) mod N, a = 0,1,..  */
/* skipping j and items already present.  The row is stored by id ascending;  */
/* that order is the slot order k of w_{j,k} and c_{j,k}.                      */
int orc_topk(int N, int B, int G, int p, int q, int K, const uint32_t* sig,
             uint64_t seed_fill, const int32_t* items, int n_items, int32_t* JK)
{
    if (K <= 0 || K > N - 1 || G * p * q > B || G * p > 64) return ORC_EINVAL;
    for (int x = 0; x < n_items; ++x)
        if (items[x] < 0 || items[x] >= N) return ORC_EINVAL;
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N * q);
    if (!keys) return ORC_ENOMEM;
    orc_band_keys(N, B, G, p, q, sig, keys);
    int status = ORC_OK;
    /* items are independent: one count vector per thread */
#pragma omp parallel
    {
        int32_t* count = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
        if (!count) {
#pragma omp atomic write
            status = ORC_ENOMEM;
        }
#pragma omp for schedule(dynamic, 16)
        for (int x = 0; x < n_items; ++x) {
            if (!count) continue;
            const int j = items[x];
            orc_pair_counts(N, q, keys, j, count);
            int32_t* row = JK + (int64_t)x * K;
            int n = 0;
            /* highest count first; within one count, ids ascending */
            for (int c = q; c >= 1 && n < K; --c)
                for (int jj = 0; jj < N && n < K; ++jj)
                    if (count[jj] == c) row[n++] = jj;
            for (uint64_t a = 0; n < K; ++a) {
                const int cand = (int)(orc_splitmix64(seed_fill, ((uint64_t)j << 32) + a + 1) % (uint64_t)N);
                int dup = (cand == j);
                for (int y = 0; y < n && !dup; ++y) dup = (row[y] == cand);
                if (!dup) row[n++] = cand;
            }
            qsort(row, (size_t)K, sizeof(int32_t), cmp_i32);
        }
        free(count);
    }
    free(keys);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Neighbour-list rebuild (a reading; the paper keeps the lists of existing  */
/* items, Sec. 4.3).  When the lists of all items are searched again, each  */
/* item's w and c values follow their neighbour ids: a neighbour kept       */
/* across the rebuild brings its w_{j,k}, c_{j,k} to its new slot, and a    */
/* slot whose neighbour is new starts at 0.  Rows j >= n_old are new items  */
/* and start at 0.  Lists are sorted by id, so the search is a merge.       */
/* ------------------------------------------------------------------------ */
int orc_remap_slots(int N, int n_old, int K, const int32_t* JK_old, const double* W_old,
                    const double* C_old, const int32_t* JK_new, double* W_new, double* C_new)
{
    if (K <= 0 || n_old < 0 || n_old > N) return ORC_EINVAL;
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < K; ++k) {
            double w = 0.0, c = 0.0;
            if (j < n_old) {
                const int n = JK_new[(int64_t)j * K + k];
                for (int k2 = 0; k2 < K; ++k2)
                    if (JK_old[(int64_t)j * K + k2] == n) {
                        w = W_old[(int64_t)j * K + k2];
                        c = C_old[(int64_t)j * K + k2];
                        break;
                    }
            }
            W_new[(int64_t)j * K + k] = w;
            C_new[(int64_t)j * K + k] = c;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The two other LSH families of the top-K comparison, Sec. 5.3.  Both fill */
/* the same signature layout as simLSH (B = G*p*q bits, hash h of band t at */
/* bits [(t*p + h)*G, (t*p + h + 1)*G)), so banding and top-K are shared.   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t j, i;
    int64_t idx;
} orc_colent;

static int cmp_col_user(const void* a, const void* b)
{
    const orc_colent* x = (const orc_colent*)a;
    const orc_colent* y = (const orc_colent*)b;
    if (x->j != y->j) return (x->j > y->j) - (x->j < y->j);
    return (x->i > y->i) - (x->i < y->i);
}

/* RP_cos: sign random projection for the cosine similarity (Charikar's     */
/* simHash, the hash simLSH is modelled on).  Item column x_j holds the      */
/* plain ratings r_ij; each of the B bits projects it on a Gaussian          */
/* direction g_.b:  acc[j][b] = sum_i r_ij g_ib,  bit b = [acc >= 0].        */
/* The sign is an integer decided by floating point, so this follows the    */
/* kernel's precision and order: FP32, one fused multiply-add per rating,   */
/* the raters of a column in ascending user id, continuing the stored sum   */
/* (an online batch adds its own raters of the column, ascending).          */
int orc_rpcos_add(int M, int N, int B, int64_t nnz, const int32_t* u, const int32_t* it,
                  const uint8_t* rc, int rscale, const float* g /* M*B */, float* acc /* N*B */)
{
    if (M <= 0 || N <= 0 || B <= 0 || nnz < 0 || rscale <= 0) return ORC_EINVAL;
    orc_colent* e = (orc_colent*)malloc(sizeof(orc_colent) * (size_t)(nnz > 0 ? nnz : 1));
    if (!e) return ORC_ENOMEM;
    for (int64_t x = 0; x < nnz; ++x) {
        if (u[x] < 0 || u[x] >= M || it[x] < 0 || it[x] >= N) { free(e); return ORC_EINVAL; }
        e[x].j = it[x]; e[x].i = u[x]; e[x].idx = x;
    }
    qsort(e, (size_t)nnz, sizeof(orc_colent), cmp_col_user);
    for (int64_t x = 0; x < nnz; ++x) {
        const float r = (float)rc[e[x].idx] / (float)rscale;   /* exact: rc <= 15, rscale 1 or 2 */
        float* a = acc + (int64_t)e[x].j * B;
        const float* gi = g + (int64_t)e[x].i * B;
        for (int b = 0; b < B; ++b) a[b] = fmaf(r, gi[b], a[b]);
    }
    free(e);
    return ORC_OK;
}

void orc_rpcos_signs(int N, int B, const float* acc, uint32_t* sig)
{
    const int words = (B + 31) / 32;
    memset(sig, 0, sizeof(uint32_t) * (size_t)N * words);
    for (int j = 0; j < N; ++j)
        for (int b = 0; b < B; ++b)
            if (acc[(int64_t)j * B + b] >= 0.0f) sig[(int64_t)j * words + b / 32] |= 1u << (b % 32);
}

/* minHash (Broder) for the Jaccard similarity of the rater sets, which the */
/* paper contrasts with simLSH in Sec. 4.1: hash h of item j is the least   */
/* random value v_ih over its raters (a random permutation of the users).   */
/* mins must start at 0xFFFFFFFF, the value of an item without raters;     */
/* adding ratings only lowers it, so an online batch continues it.          */
int orc_minhash_add(int M, int N, int nh, int64_t nnz, const int32_t* u, const int32_t* it,
                    const uint32_t* v /* M*nh */, uint32_t* mins /* N*nh */)
{
    if (M <= 0 || N <= 0 || nh <= 0 || nnz < 0) return ORC_EINVAL;
    for (int64_t x = 0; x < nnz; ++x) {
        const int i = u[x], j = it[x];
        if (i < 0 || i >= M || j < 0 || j >= N) return ORC_EINVAL;
        for (int h = 0; h < nh; ++h) {
            const uint32_t val = v[(int64_t)i * nh + h];
            if (val < mins[(int64_t)j * nh + h]) mins[(int64_t)j * nh + h] = val;
        }
    }
    return ORC_OK;
}

/* The G-bit hash is the lowest G bits of the minimum (b-bit minwise         */
/* hashing, Li and Konig 2010): hash h fills bits [h*G, (h+1)*G), LSB first. */
int orc_minhash_sig(int N, int nh, int G, const uint32_t* mins, uint32_t* sig)
{
    if (G < 1 || G > 32) return ORC_EINVAL;
    const int B = nh * G, words = (B + 31) / 32;
    memset(sig, 0, sizeof(uint32_t) * (size_t)N * words);
    for (int j = 0; j < N; ++j)
        for (int h = 0; h < nh; ++h)
            for (int x = 0; x < G; ++x) {
                const int b = h * G + x;
                if ((mins[(int64_t)j * nh + h] >> x) & 1u) sig[(int64_t)j * words + b / 32] |= 1u << (b % 32);
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Training set by user, R(i): rows sorted by item id (for membership tests). */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t j;
    int64_t i;
    int64_t idx;
} orc_edge;

static int cmp_user_item(const void* a, const void* b)
{
    const orc_edge* x = (const orc_edge*)a;
    const orc_edge* y = (const orc_edge*)b;
    if (x->i != y->i) return (x->i > y->i) - (x->i < y->i);
    return (x->j > y->j) - (x->j < y->j);
}

int orc_build_csr(int M, int64_t nnz, const int32_t* u, const int32_t* it, const uint8_t* rc,
                  int64_t* row_ptr /* M+1 */, int32_t* col /* nnz */, uint8_t* rcs /* nnz */)
{
    orc_edge* e = (orc_edge*)malloc(sizeof(orc_edge) * (size_t)(nnz > 0 ? nnz : 1));
    if (!e) return ORC_ENOMEM;
    for (int64_t x = 0; x < nnz; ++x) {
        if (u[x] < 0 || u[x] >= M) { free(e); return ORC_EINVAL; }
        e[x].i = u[x]; e[x].j = it[x]; e[x].idx = x;
    }
    qsort(e, (size_t)nnz, sizeof(orc_edge), cmp_user_item);
    for (int i = 0; i <= M; ++i) row_ptr[i] = 0;
    for (int64_t x = 0; x < nnz; ++x) {
        row_ptr[e[x].i + 1]++;
        col[x] = (int32_t)e[x].j;
        rcs[x] = rc[e[x].idx];
    }
    for (int i = 0; i < M; ++i) row_ptr[i + 1] += row_ptr[i];
    free(e);
    return ORC_OK;
}

typedef struct {
    int M;
    const int64_t* row_ptr;
    const int32_t* col;
    const uint8_t* rc;
} orc_csr;

/* rating code of (i, n) in the training set, or 0 if i did not rate n */
static int rated_code(const orc_csr* R, int i, int n)
{
    int64_t lo = R->row_ptr[i], hi = R->row_ptr[i + 1];
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (R->col[mid] < n) lo = mid + 1;
        else hi = mid;
    }
    return (lo < R->row_ptr[i + 1] && R->col[lo] == n) ? R->rc[lo] : 0;
}

/* ------------------------------------------------------------------------ */
/* Baselines, Sec. 3.2 part (1), the "simple case":                          */
/*   mu = mean rating; b0_i = mean of row i - mu; bh0_j = mean of col j - mu. */
/* A row or column with no rating gets 0.  These fixed baselines are the     */
/* b-bar used inside the residual (r_{i,j1} - b-bar_{i,j1}) of the w-term.    */
/* ------------------------------------------------------------------------ */
int orc_baselines(int M, int N, int64_t nnz, const int32_t* u, const int32_t* it,
                  const uint8_t* rc, int rscale, double* mu, double* b0 /* M */,
                  double* bh0 /* N */)
{
    if (nnz <= 0 || rscale <= 0) return ORC_EINVAL;
    double* su = (double*)calloc((size_t)M, sizeof(double));
    double* sj = (double*)calloc((size_t)N, sizeof(double));
    int64_t* cu = (int64_t*)calloc((size_t)M, sizeof(int64_t));
    int64_t* cj = (int64_t*)calloc((size_t)N, sizeof(int64_t));
    if (!su || !sj || !cu || !cj) { free(su); free(sj); free(cu); free(cj); return ORC_ENOMEM; }
    double tot = 0.0;
    for (int64_t e = 0; e < nnz; ++e) {
        const double r = (double)rc[e] / rscale;
        tot += r;
        su[u[e]] += r; cu[u[e]] += 1;
        sj[it[e]] += r; cj[it[e]] += 1;
    }
    *mu = tot / (double)nnz;
    for (int i = 0; i < M; ++i) b0[i] = cu[i] ? su[i] / (double)cu[i] - *mu : 0.0;
    for (int j = 0; j < N; ++j) bh0[j] = cj[j] ? sj[j] / (double)cj[j] - *mu : 0.0;
    free(su); free(sj); free(cu); free(cj);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Model state (all FP64).                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int M, N, F, K, rscale;
    double mu;
    double* U;    /* M*F */
    double* V;    /* N*F */
    double* bu;   /* M   learned b_i */
    double* bv;   /* N   learned bh_j */
    double* W;    /* N*K explicit influence, slot order of JK */
    double* C;    /* N*K implicit influence */
    const double* b0;   /* M fixed baseline deviations */
    const double* bh0;  /* N */
    const int32_t* JK;  /* N*K neighbour ids, ascending per row */
} orc_model;

/* Prediction, Eq. (rr), with N(i) taken as the complement of R(i) inside    */
/* S^K(j) (the CULSH-MF adjustment of Sec. 4.2).  A side with no members     */
/* contributes nothing (the |.|^(-1/2) factor of an empty set is not used).   */
double orc_predict_one(const orc_model* m, const orc_csr* R, int i, int j)
{
    double r = m->mu + m->bu[i] + m->bv[j];
    for (int f = 0; f < m->F; ++f) r += m->U[(int64_t)i * m->F + f] * m->V[(int64_t)j * m->F + f];
    int nR = 0;
    for (int k = 0; k < m->K; ++k) nR += rated_code(R, i, m->JK[(int64_t)j * m->K + k]) != 0;
    const int nN = m->K - nR;
    double sw = 0.0, sc = 0.0;
    for (int k = 0; k < m->K; ++k) {
        const int n = m->JK[(int64_t)j * m->K + k];
        const int code = rated_code(R, i, n);
        if (code) {
            const double resid = (double)code / m->rscale - (m->mu + m->b0[i] + m->bh0[n]);
            sw += resid * m->W[(int64_t)j * m->K + k];
        } else {
            sc += m->C[(int64_t)j * m->K + k];
        }
    }
    if (nR > 0) r += sw / sqrt((double)nR);
    if (nN > 0) r += sc / sqrt((double)nN);
    return r;
}

int orc_predict(const orc_model* m, const orc_csr* R, int64_t n, const int32_t* qu,
                const int32_t* qi, double* out)
{
    for (int64_t x = 0; x < n; ++x) {
        if (qu[x] < 0 || qu[x] >= m->M || qi[x] < 0 || qi[x] >= m->N) return ORC_EINVAL;
        out[x] = orc_predict_one(m, R, qu[x], qi[x]);
    }
    return ORC_OK;
}

/* RMSE over a held-out set, Sec. 5.1 (no clipping of predictions). */
double orc_rmse(int64_t n, const double* pred, const uint8_t* rc, int rscale)
{
    double s = 0.0;
    for (int64_t x = 0; x < n; ++x) {
        const double d = (double)rc[x] / rscale - pred[x];
        s += d * d;
    }
    return n ? sqrt(s / (double)n) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* One SGD step, Eq. (sgd_update), on rating (i, j, r).                       */
/* e = r - rhat from the pre-step state; every right-hand side uses the       */
/* pre-step values (simultaneous update).  w_{j,k} moves only for k in R^K,   */
/* c_{j,k} only for k in N^K; slots that are not touched are not decayed.     */
/* `upd` selects parameter groups: bit0 user side {b_i, u_i}, bit1 item side  */
/* {bh_j, v_j, w_j, c_j} (online learning freezes one side, Alg. Online).     */
/* ------------------------------------------------------------------------ */
typedef struct {
    double g[6];    /* learning rates of this epoch: b, bh, u, v, w, c */
    double lam[6];  /* regularisers:                 b, bh, u, v, w, c */
} orc_rates;

static void sgd_step(orc_model* m, const orc_csr* R, const orc_rates* h, int i, int j,
                     int code, int upd, int32_t* codes /* scratch K */, double* ubuf /* F */)
{
    const int F = m->F, K = m->K;
    double* u = m->U + (int64_t)i * F;
    double* v = m->V + (int64_t)j * F;
    double* w = m->W + (int64_t)j * K;
    double* c = m->C + (int64_t)j * K;
    const int32_t* nb = m->JK + (int64_t)j * K;

    int nR = 0;
    for (int k = 0; k < K; ++k) { codes[k] = rated_code(R, i, nb[k]); nR += codes[k] != 0; }
    const int nN = K - nR;
    const double sR = nR ? 1.0 / sqrt((double)nR) : 0.0;
    const double sN = nN ? 1.0 / sqrt((double)nN) : 0.0;

    const double rhat = orc_predict_one(m, R, i, j);
    const double e = (double)code / m->rscale - rhat;

    const double bi = m->bu[i], bj = m->bv[j];
    for (int f = 0; f < F; ++f) ubuf[f] = u[f];
    if (upd & 1) {
        m->bu[i] = bi + h->g[0] * (e - h->lam[0] * bi);
        for (int f = 0; f < F; ++f) u[f] = ubuf[f] + h->g[2] * (e * v[f] - h->lam[2] * ubuf[f]);
    }
    if (upd & 2) {
        m->bv[j] = bj + h->g[1] * (e - h->lam[1] * bj);
        for (int f = 0; f < F; ++f) v[f] = v[f] + h->g[3] * (e * ubuf[f] - h->lam[3] * v[f]);
        for (int k = 0; k < K; ++k) {
            if (codes[k]) {
                const double resid = (double)codes[k] / m->rscale - (m->mu + m->b0[i] + m->bh0[nb[k]]);
                w[k] += h->g[4] * (sR * e * resid - h->lam[4] * w[k]);
            } else {
                c[k] += h->g[5] * (sN * e - h->lam[5] * c[k]);
            }
        }
    }
}

/* A single step on one rating (tests of the update rule against the gradient). */
int orc_sgd_one(orc_model* m, const orc_csr* R, const orc_rates* h, int i, int j, int code, int upd)
{
    int32_t* codes = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m->K > 0 ? m->K : 1));
    double* ubuf = (double*)malloc(sizeof(double) * (size_t)(m->F > 0 ? m->F : 1));
    if (!codes || !ubuf) { free(codes); free(ubuf); return ORC_ENOMEM; }
    sgd_step(m, R, h, i, j, code, upd, codes, ubuf);
    free(codes);
    free(ubuf);
    return ORC_OK;
}

/* Learning rate of epoch t (0-based), Eq. (learn_rate): alpha/(1+beta t^1.5) */
void orc_rates_for_epoch(const double* alpha, const double* lam, double beta, int t, orc_rates* out)
{
    const double d = 1.0 + beta * pow((double)t, 1.5);
    for (int x = 0; x < 6; ++x) { out->g[x] = alpha[x] / d; out->lam[x] = lam[x]; }
}

/* ------------------------------------------------------------------------ */
/* Stratified epoch order.  Users split into P row blocks by i mod P, items   */
/* into P column blocks by j mod P.  Stratum s = 0..P-1 holds the P blocks    */
/* (b, (b+s) mod P); blocks of one stratum share no user and no item.  Inside */
/* a block ratings run item by item -- the column-resident order of Alg.      */
/* CULSH-MF -- with items taken by decreasing number of ratings in the pass  */
/* (ties by ascending id), and inside an item users by decreasing number of  */
/* ratings in the pass (ties by ascending id).  P = 1 is a serial order of   */
/* that algorithm.                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t s, b, rank, urank, idx;
} orc_sched;

static int cmp_sched(const void* a, const void* b)
{
    const orc_sched* x = (const orc_sched*)a;
    const orc_sched* y = (const orc_sched*)b;
    if (x->s != y->s) return (x->s > y->s) - (x->s < y->s);
    if (x->b != y->b) return (x->b > y->b) - (x->b < y->b);
    if (x->rank != y->rank) return (x->rank > y->rank) - (x->rank < y->rank);
    return (x->urank > y->urank) - (x->urank < y->urank);
}

/* order key of an item or a user: more ratings first, then smaller id */
static int64_t rank_key(const int64_t* deg, int64_t nnz, int id)
{
    return (nnz - deg[id]) * (int64_t)(1u << 31) + id;
}

/* order[x] = index into the COO arrays of the x-th rating of the epoch;      */
/* blk_ptr[s*P + b] .. blk_ptr[s*P + b + 1] delimit block b of stratum s.     */
int orc_schedule(int P, int64_t nnz, const int32_t* u, const int32_t* it,
                 int64_t* order /* nnz */, int64_t* blk_ptr /* P*P+1 */)
{
    if (P <= 0) return ORC_EINVAL;
    int32_t N = 0, M = 0;
    for (int64_t x = 0; x < nnz; ++x) {
        N = it[x] + 1 > N ? it[x] + 1 : N;
        M = u[x] + 1 > M ? u[x] + 1 : M;
    }
    int64_t* deg = (int64_t*)calloc((size_t)(N > 0 ? N : 1), sizeof(int64_t));
    int64_t* udeg = (int64_t*)calloc((size_t)(M > 0 ? M : 1), sizeof(int64_t));
    orc_sched* e = (orc_sched*)malloc(sizeof(orc_sched) * (size_t)(nnz > 0 ? nnz : 1));
    if (!e || !deg || !udeg) { free(e); free(deg); free(udeg); return ORC_ENOMEM; }
    for (int64_t x = 0; x < nnz; ++x) {
        deg[it[x]]++;
        udeg[u[x]]++;
    }
    for (int64_t x = 0; x < nnz; ++x) {
        const int64_t rb = u[x] % P, cb = it[x] % P;
        e[x].s = ((cb - rb) % P + P) % P;
        e[x].b = rb;
        e[x].rank = rank_key(deg, nnz, it[x]);
        e[x].urank = rank_key(udeg, nnz, u[x]);
        e[x].idx = x;
    }
    qsort(e, (size_t)nnz, sizeof(orc_sched), cmp_sched);
    for (int64_t x = 0; x <= (int64_t)P * P; ++x) blk_ptr[x] = 0;
    for (int64_t x = 0; x < nnz; ++x) {
        order[x] = e[x].idx;
        blk_ptr[e[x].s * P + e[x].b + 1]++;
    }
    for (int64_t x = 0; x < (int64_t)P * P; ++x) blk_ptr[x + 1] += blk_ptr[x];
    free(e);
    free(deg);
    free(udeg);
    return ORC_OK;
}

/* One epoch (Alg. CULSH-MF's inner loops) in the stratified order.           */
/* reverse_blocks runs the blocks of each stratum in descending b: the result */
/* must not change, since the blocks are independent.                          */
/* Strata [s0, s1) of that order: a bounded sample of an epoch (timing).   */
int orc_sgd_strata(orc_model* m, const orc_csr* R, const int32_t* u, const int32_t* it,
                   const uint8_t* rc, const int64_t* order, const int64_t* blk_ptr, int P, int s0,
                   int s1, const orc_rates* h, int reverse_blocks, int upd)
{
    int status = ORC_OK;
    if (s0 < 0 || s1 > P || s0 > s1) return ORC_EINVAL;
    for (int s = s0; s < s1; ++s) {
        /* the blocks of one stratum touch disjoint users and items */
#pragma omp parallel for schedule(dynamic, 1)
        for (int bb = 0; bb < P; ++bb) {
            const int b = reverse_blocks ? P - 1 - bb : bb;
            int32_t* codes = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m->K > 0 ? m->K : 1));
            double* ubuf = (double*)malloc(sizeof(double) * (size_t)(m->F > 0 ? m->F : 1));
            if (!codes || !ubuf) {
#pragma omp atomic write
                status = ORC_ENOMEM;
            } else {
                for (int64_t x = blk_ptr[(int64_t)s * P + b]; x < blk_ptr[(int64_t)s * P + b + 1]; ++x) {
                    const int64_t e = order[x];
                    sgd_step(m, R, h, u[e], it[e], rc[e], upd, codes, ubuf);
                }
            }
            free(codes);
            free(ubuf);
        }
    }
    return status;
}

int orc_sgd_epoch(orc_model* m, const orc_csr* R, int64_t nnz, const int32_t* u,
                  const int32_t* it, const uint8_t* rc, const int64_t* order,
                  const int64_t* blk_ptr, int P, const orc_rates* h, int reverse_blocks,
                  int upd)
{
    (void)nnz;
    return orc_sgd_strata(m, R, u, it, rc, order, blk_ptr, P, 0, P, h, reverse_blocks, upd);
}

/* Objective, Eq. (loss_r): squared training error plus the L2 penalties.     */
/* The w and c penalties sum over every stored slot of every item.            */
double orc_loss(const orc_model* m, const orc_csr* R, const double* lam)
{
    double s = 0.0;
    for (int i = 0; i < R->M; ++i)
        for (int64_t x = R->row_ptr[i]; x < R->row_ptr[i + 1]; ++x) {
            const double d = (double)R->rc[x] / m->rscale - orc_predict_one(m, R, i, R->col[x]);
            s += d * d;
        }
    double pb = 0, pbh = 0, pu = 0, pv = 0, pw = 0, pc = 0;
    for (int i = 0; i < m->M; ++i) pb += m->bu[i] * m->bu[i];
    for (int j = 0; j < m->N; ++j) pbh += m->bv[j] * m->bv[j];
    for (int64_t x = 0; x < (int64_t)m->M * m->F; ++x) pu += m->U[x] * m->U[x];
    for (int64_t x = 0; x < (int64_t)m->N * m->F; ++x) pv += m->V[x] * m->V[x];
    for (int64_t x = 0; x < (int64_t)m->N * m->K; ++x) { pw += m->W[x] * m->W[x]; pc += m->C[x] * m->C[x]; }
    return s + lam[0] * pb + lam[1] * pbh + lam[2] * pu + lam[3] * pv + lam[4] * pw + lam[5] * pc;
}
