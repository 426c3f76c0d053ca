// Prediction (Eq. rr), the FP64 RMSE and objective (Eq. loss_r) reductions,
// and the BF16 copies of the storage mode.
#include <cmath>

#include "common.hpp"
#include "wave.hpp"

namespace lshmf {

// BF16 copies of n FP32 values.
__global__ void k_to_bf16(const float* src, uint16_t* dst, int64_t n)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        dst[x] = to_bf16(src[x]);
}

int to_bf16_rows(const float* src, uint16_t* dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return LSHMF_OK;
    int64_t b = ceil_div(n, 256);
    if (b > 16384) b = 16384;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)b), dim3(256), 0, s, src, dst, n);
    LSHMF_LAUNCHED("k_to_bf16");
    return LSHMF_OK;
}

// Plain copies of n FP32 values (the bias snapshots that predict reads in the
// BF16 storage modes).
__global__ void k_copy_f32(const float* src, float* dst, int64_t n)
{
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        dst[x] = src[x];
}

static int copy_rows(const float* src, float* dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return LSHMF_OK;
    int64_t b = ceil_div(n, 256);
    if (b > 16384) b = 16384;
    hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)b), dim3(256), 0, s, src, dst, n);
    LSHMF_LAUNCHED("k_copy_f32");
    return LSHMF_OK;
}

// BF16 copies of the rows r < n_rows with ptr[r+1] > ptr[r] (the rows a batch
// touched) of up to two FP32 tables of `width` floats a row; a wave per row.
__global__ __launch_bounds__(256) void k_bf16_touched(const int64_t* ptr, int64_t n_rows, const float* a,
                                                      uint16_t* a16, int64_t wa, const float* b, uint16_t* b16,
                                                      int64_t wb, const float* bias, float* bias_s)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t r = w0; r < n_rows; r += nw) {
        if (ptr[r + 1] == ptr[r]) continue;
        if (bias && lane == 0) bias_s[r] = bias[r];
        for (int64_t k = lane; k < wa; k += kWave) a16[r * wa + k] = to_bf16(a[r * wa + k]);
        if (b)
            for (int64_t k = lane; k < wb; k += kWave) b16[r * wb + k] = to_bf16(b[r * wb + k]);
    }
}

// BF16 copies of the user rows with ratings in a batch (its CSR row_ptr over
// c->M users) and of the item rows with ratings in it (its CSC col_ptr).
int refresh_bf16_touched(lshmf_ctx* c, const int64_t* b_rptr, const int64_t* b_cptr, hipStream_t s)
{
    if (c->d.storage == LSHMF_FP32) return LSHMF_OK;
    const int64_t F = c->d.F, K = c->d.K, N = c->N, M = c->M;
    const int64_t wu = c->d.storage == LSHMF_BF16_U ? 0 : F;  // BF16_U: U16 is the master, only b is copied
    auto grid = [](int64_t rows) {
        int64_t b = ceil_div(rows > 0 ? rows * kWave : 1, 256);
        return (unsigned)(b > 16384 ? 16384 : b);
    };
    if (M > 0) {
        hipLaunchKernelGGL(k_bf16_touched, dim3(grid(M)), dim3(256), 0, s, b_rptr, M, c->t.U, c->t.U16, wu,
                           (const float*)nullptr, (uint16_t*)nullptr, (int64_t)0, (const float*)c->t.bu, c->bu_s);
        LSHMF_LAUNCHED("k_bf16_touched(users)");
    }
    if (N > 0) {
        hipLaunchKernelGGL(k_bf16_touched, dim3(grid(N)), dim3(256), 0, s, b_cptr, N, c->t.V, c->t.V16, F, c->t.W,
                           c->t.W16, K, (const float*)c->t.bv, c->bv_s);
        LSHMF_LAUNCHED("k_bf16_touched(items V,W)");
        hipLaunchKernelGGL(k_bf16_touched, dim3(grid(N)), dim3(256), 0, s, b_cptr, N, c->t.C, c->t.C16, K,
                           (const float*)nullptr, (uint16_t*)nullptr, (int64_t)0, (const float*)nullptr,
                           (float*)nullptr);
        LSHMF_LAUNCHED("k_bf16_touched(items C)");
    }
    return LSHMF_OK;
}

// BF16 copies of the rows [m0, m1) of U and [n0, n1) of V, W, C.
int refresh_bf16(lshmf_ctx* c, int64_t m0, int64_t m1, int64_t n0, int64_t n1, hipStream_t s)
{
    if (c->d.storage == LSHMF_FP32) return LSHMF_OK;
    const int64_t F = c->d.F, K = c->d.K;
    if (c->d.storage == LSHMF_BF16) LSHMF_TRY(to_bf16_rows(c->t.U + m0 * F, c->t.U16 + m0 * F, (m1 - m0) * F, s));
    LSHMF_TRY(copy_rows(c->t.bu + m0, c->bu_s + m0, m1 - m0, s));
    LSHMF_TRY(copy_rows(c->t.bv + n0, c->bv_s + n0, n1 - n0, s));
    LSHMF_TRY(to_bf16_rows(c->t.V + n0 * F, c->t.V16 + n0 * F, (n1 - n0) * F, s));
    LSHMF_TRY(to_bf16_rows(c->t.W + n0 * K, c->t.W16 + n0 * K, (n1 - n0) * K, s));
    return to_bf16_rows(c->t.C + n0 * K, c->t.C16 + n0 * K, (n1 - n0) * K, s);
}

// ---------------------------------------------------------------- predict
struct PredArgs {
    const int32_t* JK;
    const float* b0;
    const float* bh0;
    const double* mu;
    const void* U;    // float, or BF16 bits in storage mode BF16
    const void* V;
    const float* bu;
    const float* bv;
    const void* W;
    const void* C;
    const int64_t* row_ptr;
    const int32_t* csr_col;
    const uint8_t* csr_rc;
    int M, N, F, K;
    float inv_s;
};

__device__ inline float ld_tab(const float* p, int64_t x) { return p[x]; }
__device__ inline float ld_tab(const uint16_t* p, int64_t x) { return from_bf16(p[x]); }

// One wave per query: Eq. (rr) with R^K / N^K resolved by binary search of
// each neighbour in the user's training row.  T: storage type of U, V, W, C.
template <int FP, int KP, typename T>
__global__ __launch_bounds__(256) void k_predict(PredArgs a, const int32_t* qu, const int32_t* qi, int64_t n,
                                                 float* out)
{
    const T* U = static_cast<const T*>(a.U);
    const T* V = static_cast<const T*>(a.V);
    const T* W = static_cast<const T*>(a.W);
    const T* C = static_cast<const T*>(a.C);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    const float mu = (float)(*a.mu);
    const int F = a.F, K = a.K;
    for (int64_t x = w0; x < n; x += nw) {
        const int64_t i = qu[x], j = qi[x];
        if (i < 0 || i >= a.M || j < 0 || j >= a.N) {
            if (lane == 0) out[x] = __int_as_float(0x7fc00000);
            continue;
        }
        const int64_t ra = a.row_ptr[i], rz = a.row_ptr[i + 1];
        float part = 0.0f;
#pragma unroll
        for (int y = 0; y < FP; ++y) {
            const int f = lane + y * kWave;
            if (f < F) part += ld_tab(U, i * F + f) * ld_tab(V, j * F + f);
        }
        int code[KP];
        int nb[KP];
        int nR = 0;
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            const int k = lane + y * kWave;
            code[y] = 0;
            nb[y] = 0;
            if (k < K) {
                nb[y] = a.JK[j * K + k];
                int64_t l = ra, r = rz;
                while (l < r) {
                    const int64_t m = (l + r) >> 1;
                    if (a.csr_col[m] < nb[y]) l = m + 1;
                    else r = m;
                }
                code[y] = (l < rz && a.csr_col[l] == nb[y]) ? a.csr_rc[l] : 0;
            }
            nR += __popcll(__ballot(code[y] != 0));
        }
        const int nN = K - nR;
        const float sR = nR > 0 ? 1.0f / sqrtf((float)nR) : 0.0f;
        const float sN = nN > 0 ? 1.0f / sqrtf((float)nN) : 0.0f;
        const float base_i = mu + a.b0[i];
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            const int k = lane + y * kWave;
            if (k < K) {
                if (code[y]) part += ((float)code[y] * a.inv_s - base_i - a.bh0[nb[y]]) * ld_tab(W, j * K + k) * sR;
                else part += ld_tab(C, j * K + k) * sN;
            }
        }
        const float tot = wave_sum(part);
        if (lane == 0) out[x] = mu + a.bu[i] + a.bv[j] + tot;
    }
}

template <int FP, typename T>
static void launch_predict_t(const PredArgs& a, const int32_t* qu, const int32_t* qi, int64_t n, float* out,
                             unsigned grid, hipStream_t s)
{
    if (a.K <= kWave)
        hipLaunchKernelGGL((k_predict<FP, 1, T>), dim3(grid), dim3(256), 0, s, a, qu, qi, n, out);
    else
        hipLaunchKernelGGL((k_predict<FP, 2, T>), dim3(grid), dim3(256), 0, s, a, qu, qi, n, out);
}

template <int FP>
static void launch_predict_k(const PredArgs& a, bool bf, const int32_t* qu, const int32_t* qi, int64_t n,
                             float* out, unsigned grid, hipStream_t s)
{
    if (bf) launch_predict_t<FP, uint16_t>(a, qu, qi, n, out, grid, s);
    else launch_predict_t<FP, float>(a, qu, qi, n, out, grid, s);
}

int run_predict(lshmf_ctx* c, const int32_t* qu, const int32_t* qi, int64_t n, float* out, hipStream_t s)
{
    if (n <= 0) return LSHMF_OK;
    const lshmf_dims& d = c->d;
    const bool bf = d.storage != LSHMF_FP32;  // BF16 copies (BF16), or BF16 user rows and copies (BF16_U)
    PredArgs a{c->t.JK, c->t.b0, c->t.bh0, c->t.mu,
               bf ? (const void*)c->t.U16 : (const void*)c->t.U, bf ? (const void*)c->t.V16 : (const void*)c->t.V,
               bf ? c->bu_s : c->t.bu, bf ? c->bv_s : c->t.bv,
               bf ? (const void*)c->t.W16 : (const void*)c->t.W, bf ? (const void*)c->t.C16 : (const void*)c->t.C,
               c->row_ptr, c->csr_col, c->csr_rc, c->M, c->N, d.F, d.K, 1.0f / (float)d.rscale};
    int64_t blocks = ceil_div(n * kWave, 256);
    if (blocks > 65536) blocks = 65536;
    const int fp = (d.F + kWave - 1) / kWave;
    switch (fp) {
        case 1: launch_predict_k<1>(a, bf, qu, qi, n, out, (unsigned)blocks, s); break;
        case 2: launch_predict_k<2>(a, bf, qu, qi, n, out, (unsigned)blocks, s); break;
        case 3: launch_predict_k<3>(a, bf, qu, qi, n, out, (unsigned)blocks, s); break;
        default: launch_predict_k<4>(a, bf, qu, qi, n, out, (unsigned)blocks, s); break;
    }
    LSHMF_LAUNCHED("k_predict");
    return LSHMF_OK;
}

// ------------------------------------------------------------------- RMSE

__device__ inline double block_sum_f64(double v, double* scratch)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int x = 0; x < (int)(blockDim.x / kWave); ++x) t += scratch[x];
    return t;
}

__global__ __launch_bounds__(256) void k_sse_partial(const float* pred, const uint8_t* rc, int64_t n,
                                                     double inv_s, double* partial)
{
    __shared__ double scratch[256 / kWave];
    double s = 0.0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const double dlt = (double)rc[x] * inv_s - (double)pred[x];
        s += dlt * dlt;
    }
    const double t = block_sum_f64(s, scratch);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_sse_final(const double* partial, int nparts, int64_t n, double* out)
{
    __shared__ double scratch[256 / kWave];
    double s = 0.0;
    for (int x = threadIdx.x; x < nparts; x += blockDim.x) s += partial[x];
    const double t = block_sum_f64(s, scratch);
    if (threadIdx.x == 0) *out = n > 0 ? sqrt(t / (double)n) : 0.0;
}

// ------------------------------------------------------------------- loss
// Eq. (loss_r) in FP64: the squared error over the training ratings plus the
// six L2 penalties.  Every partial has a fixed owner and every sum a fixed
// order, so the value is reproducible bit for bit.
constexpr int kLossBlocks = 1024;
constexpr int kLossWaves = 4;

struct LossLam {
    float l[6];
};

struct LossArgs {
    const uint32_t* pk;
    const uint8_t* nib;
    const int32_t* seg_col;
    const int64_t* seg_start;
    const float* nbr_b0;
    const float* b0;
    const double* mu;
    const float* U;
    const uint16_t* U16;  // storage mode BF16_U: the user rows (U unused), else NULL
    const float* V;
    const float* bu;
    const float* bv;
    const float* W;
    const float* C;
    int64_t nseg;
    int F, K, nstride;
    float inv_s;
};

// One wave per item run (wave w of the grid takes runs w, w + waves, ...),
// the item state in registers; each rating's prediction (Eq. rr) in FP32,
// its squared error added in FP64 in stream order.
template <int FP, int KP>
__global__ __launch_bounds__(kLossWaves* kWave) void k_loss_sse(LossArgs a, double* partial)
{
    __shared__ double wsum[kLossWaves];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int64_t nw = (int64_t)gridDim.x * kLossWaves;
    const float mu = (float)(*a.mu);
    const int F = a.F, K = a.K;
    double acc = 0.0;
    for (int64_t seg = (int64_t)blockIdx.x * kLossWaves + wv; seg < a.nseg; seg += nw) {
        const int64_t j = a.seg_col[seg];
        const int64_t ea = a.seg_start[seg], ez = a.seg_start[seg + 1];
        float v[FP], w[KP], c[KP], bhn[KP];
#pragma unroll
        for (int x = 0; x < FP; ++x) {
            const int f = lane + x * kWave;
            v[x] = f < F ? a.V[j * F + f] : 0.0f;
        }
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            const int k = lane + y * kWave;
            w[y] = k < K ? a.W[j * K + k] : 0.0f;
            c[y] = k < K ? a.C[j * K + k] : 0.0f;
            bhn[y] = k < K ? a.nbr_b0[j * K + k] : 0.0f;
        }
        const float bh = a.bv[j];
        for (int64_t p = ea; p < ez; ++p) {
            const uint32_t pw = a.pk[p];
            const int64_t i = pw >> 4;
            const float r = (float)(pw & 15u) * a.inv_s;
            const float base_i = mu + a.b0[i];
            float part = 0.0f;
#pragma unroll
            for (int x = 0; x < FP; ++x) {
                const int f = lane + x * kWave;
                if (f < F) part += (a.U16 ? from_bf16(a.U16[i * F + f]) : a.U[i * F + f]) * v[x];
            }
            int code[KP];
            int nR = 0;
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                const int k = lane + y * kWave;
                const int byte = (lane >> 1) + y * (kWave / 2);
                code[y] = k < K ? (int)((a.nib[p * a.nstride + (byte < a.nstride ? byte : 0)] >> ((lane & 1) * 4)) & 15u)
                                : 0;
                nR += __popcll(__ballot(code[y] != 0));
            }
            const float sR = nR > 0 ? 1.0f / sqrtf((float)nR) : 0.0f;
            const float sN = K - nR > 0 ? 1.0f / sqrtf((float)(K - nR)) : 0.0f;
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                const int k = lane + y * kWave;
                if (k < K) part += code[y] ? ((float)code[y] * a.inv_s - base_i - bhn[y]) * w[y] * sR : c[y] * sN;
            }
            const float e = r - (mu + a.bu[i] + bh + wave_sum(part));
            acc += (double)e * (double)e;
        }
    }
    if (lane == 0) wsum[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int x = 0; x < kLossWaves; ++x) t += wsum[x];
        partial[blockIdx.x] = t;
    }
}

// Squared norms of the six tables (b, bh, U, V, W, C): block b owns a fixed
// grid-stride share of each and writes partial[t * blocks + b].
__global__ __launch_bounds__(256) void k_loss_norms(const float* bu, int64_t nb, const float* bv, int64_t nbh,
                                                    const float* U, const uint16_t* U16, int64_t nu, const float* V,
                                                    int64_t nv, const float* W, const float* C, int64_t nk,
                                                    double* partial)
{
    __shared__ double scratch[256 / kWave];
    const float* tab[6] = {bu, bv, U, V, W, C};
    const int64_t len[6] = {nb, nbh, nu, nv, nk, nk};
    for (int t = 0; t < 6; ++t) {
        double s = 0.0;
        for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < len[t];
             x += (int64_t)gridDim.x * blockDim.x) {
            const double v = (t == 2 && U16) ? (double)from_bf16(U16[x]) : (double)tab[t][x];
            s += v * v;
        }
        const double tot = block_sum_f64(s, scratch);
        if (threadIdx.x == 0) partial[(int64_t)t * gridDim.x + blockIdx.x] = tot;
        __syncthreads();
    }
}

// loss = sse + sum_t lambda_t |table_t|^2, every sum over blocks in block order.
__global__ __launch_bounds__(256) void k_loss_final(const double* partial, int blocks, LossLam lam, double* out)
{
    __shared__ double scratch[256 / kWave];
    double tot[7];
    for (int t = 0; t < 7; ++t) {
        double s = 0.0;
        for (int x = threadIdx.x; x < blocks; x += blockDim.x) s += partial[(int64_t)t * blocks + x];
        tot[t] = block_sum_f64(s, scratch);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double l = tot[0];
        for (int t = 0; t < 6; ++t) l += (double)lam.l[t] * tot[t + 1];
        *out = l;
    }
}

int run_loss(lshmf_ctx* c, const lshmf_hparams* hp, double* out, hipStream_t s)
{
    const lshmf_dims& d = c->d;
    const Stream& st = c->train;
    const uint16_t* u16 = d.storage == LSHMF_BF16_U ? c->t.U16 : nullptr;
    LossArgs a{st.pk, c->nstride > 0 ? st.nib : reinterpret_cast<const uint8_t*>(c->trash), st.seg_col,
               st.seg_start, c->nbr_b0, c->t.b0, c->t.mu, c->t.U, u16, c->t.V, c->t.bu, c->t.bv,
               d.K > 0 ? c->t.W : c->trash, d.K > 0 ? c->t.C : c->trash, st.n > 0 ? st.nseg : 0,
               d.F, d.K, c->nstride, 1.0f / (float)d.rscale};
    double* part = c->red;  // [0, B): squared errors; [(t+1)B, (t+2)B): norm t
    const dim3 grid(kLossBlocks), block(kLossWaves * kWave);
    const int fp = (d.F + kWave - 1) / kWave;
    const bool k2 = d.K > kWave;
#define LSHMF_LOSS(FPV)                                                                              \
    if (k2) hipLaunchKernelGGL((k_loss_sse<FPV, 2>), grid, block, 0, s, a, part);                    \
    else hipLaunchKernelGGL((k_loss_sse<FPV, 1>), grid, block, 0, s, a, part);
    switch (fp) {
        case 1: LSHMF_LOSS(1) break;
        case 2: LSHMF_LOSS(2) break;
        case 3: LSHMF_LOSS(3) break;
        default: LSHMF_LOSS(4) break;
    }
#undef LSHMF_LOSS
    LSHMF_LAUNCHED("k_loss_sse");
    const int64_t M = c->M, N = c->N, F = d.F, K = d.K;
    hipLaunchKernelGGL(k_loss_norms, grid, dim3(256), 0, s, c->t.bu, M, c->t.bv, N, c->t.U, u16, M * F, c->t.V,
                       N * F, a.W, a.C, K > 0 ? N * K : 0, part + kLossBlocks);
    LSHMF_LAUNCHED("k_loss_norms");
    LossLam lam;
    for (int t = 0; t < 6; ++t) lam.l[t] = hp->lambda[t];
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, part, kLossBlocks, lam, out);
    LSHMF_LAUNCHED("k_loss_final");
    return LSHMF_OK;
}

// The RMSE reduction with its kRmsePartials per-block partial sums in `partial`.
int rmse_with(const float* pred, const uint8_t* rc, int64_t n, int rscale, double* partial, double* out,
              hipStream_t s)
{
    hipLaunchKernelGGL(k_sse_partial, dim3(kRmsePartials), dim3(256), 0, s, pred, rc, n, 1.0 / (double)rscale,
                       partial);
    LSHMF_LAUNCHED("k_sse_partial");
    hipLaunchKernelGGL(k_sse_final, dim3(1), dim3(256), 0, s, partial, kRmsePartials, n, out);
    LSHMF_LAUNCHED("k_sse_final");
    return LSHMF_OK;
}

int run_rmse(lshmf_ctx* c, const float* pred, const uint8_t* rc, int64_t n, double* out, hipStream_t s)
{
    return rmse_with(pred, rc, n, c->d.rscale, c->red, out, s);
}

}  // namespace lshmf
