// Neighbourhood-MF SGD over the stratified block stream, prediction and the
// FP64 RMSE reduction.
//
// k_sgd_stratum (Alg. CULSH-MF, Eq. sgd_update with Eq. rr): one workgroup per
// block of the stratum, 8 waves.  A wave takes the next item segment of its
// block (a run of ratings of one item j), holds the item state {v_j, bh_j,
// w_j, c_j} in registers for the whole run -- the register-resident column
// state of the paper's kernel -- and streams the users' {u_i, b_i} from HBM.
// Lanes own features f = lane + 64x and neighbour slots k = lane + 64y, so
// u.v, the explicit w-sum and the implicit c-sum of Eq. (rr) fold into ONE
// 64-lane reduction.  Blocks of a stratum share no user and no item; inside a
// block, a rating waits (LDS flag) for the previous rating of the same user,
// which makes the result identical to running the block's ratings in order.
#include <cmath>

#include "common.hpp"

namespace lshmf {

constexpr int kSgdWaves = 8;
constexpr int kMaxBlockNnz = 1 << 16;   // LDS done-flags: 8 KB
constexpr int kSpinLimit = 1 << 24;     // bounded wait: a broken dependency ends the kernel

struct SgdArgs {
    const uint32_t* pk;
    const int32_t* dep;
    const uint8_t* nib;
    const int64_t* blk_ptr;
    const int64_t* blk_seg;
    const int32_t* seg_col;
    const int64_t* seg_start;
    const int32_t* JK;
    const float* b0;
    const float* bh0;
    const double* mu;
    float* U;
    float* V;
    float* bu;
    float* bv;
    float* W;
    float* C;
    int32_t* err;
    int F, K, P, nstride, s;
    float inv_s;
    float g[6], l[6];
};

__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <int FP, int KP>
__global__ __launch_bounds__(kSgdWaves* kWave) void k_sgd_stratum(SgdArgs a)
{
    __shared__ uint32_t done[kMaxBlockNnz / 32];
    __shared__ int next_seg;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t blk = (int64_t)a.s * a.P + blockIdx.x;
    const int64_t e0 = a.blk_ptr[blk], e1 = a.blk_ptr[blk + 1];
    const int64_t g0 = a.blk_seg[blk], g1 = a.blk_seg[blk + 1];
    const int nwords = (int)((e1 - e0 + 31) / 32);
    for (int x = threadIdx.x; x < nwords; x += blockDim.x) done[x] = 0;
    if (threadIdx.x == 0) next_seg = 0;
    __syncthreads();
    const float mu = (float)(*a.mu);
    const int F = a.F, K = a.K;
    while (true) {
        int g = 0;
        if (lane == 0) g = atomicAdd(&next_seg, 1);
        g = __shfl(g, 0, kWave);
        if (g >= g1 - g0) break;
        const int64_t seg = g0 + g;
        const int64_t j = a.seg_col[seg];
        const int64_t ea = a.seg_start[seg], ez = a.seg_start[seg + 1];

        float v[FP], w[KP], c[KP], bhn[KP];
#pragma unroll
        for (int x = 0; x < FP; ++x) {
            const int f = lane + x * kWave;
            v[x] = f < F ? a.V[j * F + f] : 0.0f;
        }
        float bh = a.bv[j];
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            const int k = lane + y * kWave;
            w[y] = c[y] = bhn[y] = 0.0f;
            if (k < K) {
                w[y] = a.W[j * K + k];
                c[y] = a.C[j * K + k];
                bhn[y] = a.bh0[a.JK[j * K + k]];
            }
        }

        for (int64_t e = ea; e < ez; ++e) {
            const int d = a.dep[e];
            if (d >= 0) {
                int spins = 0;
                while (!((__hip_atomic_load(&done[d >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >>
                          (d & 31)) & 1u)) {
                    if (++spins > kSpinLimit) {
                        if (lane == 0) atomicOr(a.err, 2);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            const uint32_t pk = a.pk[e];
            const int64_t i = pk >> 4;
            const float r = (float)(pk & 15u) * a.inv_s;
            float u[FP];
#pragma unroll
            for (int x = 0; x < FP; ++x) {
                const int f = lane + x * kWave;
                u[x] = f < F ? a.U[i * F + f] : 0.0f;
            }
            const float bi = a.bu[i];
            const float base_i = mu + a.b0[i];
            const uint8_t* nb = a.nib + e * a.nstride;
            int code[KP];
            int nR = 0;
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                const int k = lane + y * kWave;
                code[y] = k < K ? (nb[k >> 1] >> ((k & 1) * 4)) & 15 : 0;
                nR += __popcll(__ballot(code[y] != 0));
            }
            const int nN = K - nR;
            const float sR = nR > 0 ? 1.0f / sqrtf((float)nR) : 0.0f;
            const float sN = nN > 0 ? 1.0f / sqrtf((float)nN) : 0.0f;

            float part = 0.0f;
#pragma unroll
            for (int x = 0; x < FP; ++x) part += u[x] * v[x];
            float resid[KP];
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                const int k = lane + y * kWave;
                resid[y] = (float)code[y] * a.inv_s - base_i - bhn[y];
                if (k < K) part += code[y] ? resid[y] * w[y] * sR : c[y] * sN;
            }
            const float rhat = mu + bi + bh + wave_sum(part);
            const float err = r - rhat;

            if (lane == 0) a.bu[i] = bi + a.g[0] * (err - a.l[0] * bi);
            bh = bh + a.g[1] * (err - a.l[1] * bh);
#pragma unroll
            for (int x = 0; x < FP; ++x) {
                const int f = lane + x * kWave;
                if (f < F) {
                    a.U[i * F + f] = u[x] + a.g[2] * (err * v[x] - a.l[2] * u[x]);
                    v[x] = v[x] + a.g[3] * (err * u[x] - a.l[3] * v[x]);
                }
            }
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                const int k = lane + y * kWave;
                if (k < K) {
                    if (code[y]) w[y] += a.g[4] * (sR * err * resid[y] - a.l[4] * w[y]);
                    else c[y] += a.g[5] * (sN * err - a.l[5] * c[y]);
                }
            }
            // publish this rating's user-side writes to the other waves of the block
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) {
                const int64_t le = e - e0;
                __hip_atomic_fetch_or(&done[le >> 5], 1u << (le & 31), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
#pragma unroll
        for (int x = 0; x < FP; ++x) {
            const int f = lane + x * kWave;
            if (f < F) a.V[j * F + f] = v[x];
        }
        if (lane == 0) a.bv[j] = bh;
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            const int k = lane + y * kWave;
            if (k < K) {
                a.W[j * K + k] = w[y];
                a.C[j * K + k] = c[y];
            }
        }
    }
}

template <int FP, int KP>
static int launch_sgd(const SgdArgs& args, hipStream_t s)
{
    hipLaunchKernelGGL((k_sgd_stratum<FP, KP>), dim3((unsigned)args.P), dim3(kSgdWaves * kWave), 0, s, args);
    LSHMF_LAUNCHED("k_sgd_stratum");
    return LSHMF_OK;
}

template <int FP>
static int launch_sgd_k(const SgdArgs& args, hipStream_t s)
{
    return args.K <= kWave ? launch_sgd<FP, 1>(args, s) : launch_sgd<FP, 2>(args, s);
}

int run_sgd_epoch(lshmf_ctx* c, const lshmf_hparams* hp, int epoch, hipStream_t s)
{
    const lshmf_dims& d = c->d;
    if (c->max_block_nnz > kMaxBlockNnz) {
        set_error("sgd_epoch: a block holds %lld ratings, more than %d; raise n_strata",
                  (long long)c->max_block_nnz, kMaxBlockNnz);
        return LSHMF_ECAPACITY;
    }
    SgdArgs a;
    a.pk = c->pk;
    a.dep = c->dep;
    a.nib = c->nib;
    a.blk_ptr = c->blk_ptr;
    a.blk_seg = c->blk_seg;
    a.seg_col = c->seg_col;
    a.seg_start = c->seg_start;
    a.JK = c->t.JK;
    a.b0 = c->t.b0;
    a.bh0 = c->t.bh0;
    a.mu = c->t.mu;
    a.U = c->t.U;
    a.V = c->t.V;
    a.bu = c->t.bu;
    a.bv = c->t.bv;
    a.W = c->t.W;
    a.C = c->t.C;
    a.err = c->err;
    a.F = d.F;
    a.K = d.K;
    a.P = c->P;
    a.nstride = c->nstride;
    a.inv_s = 1.0f / (float)d.rscale;
    // Eq. (learn_rate): gamma_t = alpha / (1 + beta * t^1.5)
    const double den = 1.0 + (double)hp->beta * std::pow((double)epoch, 1.5);
    for (int x = 0; x < 6; ++x) {
        a.g[x] = (float)((double)hp->alpha[x] / den);
        a.l[x] = hp->lambda[x];
    }
    const int fp = (d.F + kWave - 1) / kWave;
    for (int st = 0; st < c->P; ++st) {
        a.s = st;
        switch (fp) {
            case 1: LSHMF_TRY(launch_sgd_k<1>(a, s)); break;
            case 2: LSHMF_TRY(launch_sgd_k<2>(a, s)); break;
            case 3: LSHMF_TRY(launch_sgd_k<3>(a, s)); break;
            default: LSHMF_TRY(launch_sgd_k<4>(a, s)); break;
        }
    }
    return LSHMF_OK;
}

// ---------------------------------------------------------------- predict
struct PredArgs {
    const int32_t* JK;
    const float* b0;
    const float* bh0;
    const double* mu;
    const float* U;
    const float* V;
    const float* bu;
    const float* bv;
    const float* W;
    const float* C;
    const int64_t* row_ptr;
    const int32_t* csr_col;
    const uint8_t* csr_rc;
    int M, N, F, K;
    float inv_s;
};

// One wave per query: Eq. (rr) with R^K / N^K resolved by binary search of
// each neighbour in the user's training row.
template <int FP, int KP>
__global__ __launch_bounds__(256) void k_predict(PredArgs a, const int32_t* qu, const int32_t* qi, int64_t n,
                                                 float* out)
{
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
            if (f < F) part += a.U[i * F + f] * a.V[j * F + f];
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
                if (code[y]) part += ((float)code[y] * a.inv_s - base_i - a.bh0[nb[y]]) * a.W[j * K + k] * sR;
                else part += a.C[j * K + k] * sN;
            }
        }
        const float tot = wave_sum(part);
        if (lane == 0) out[x] = mu + a.bu[i] + a.bv[j] + tot;
    }
}

template <int FP>
static void launch_predict_k(const PredArgs& a, const int32_t* qu, const int32_t* qi, int64_t n, float* out,
                             unsigned grid, hipStream_t s)
{
    if (a.K <= kWave)
        hipLaunchKernelGGL((k_predict<FP, 1>), dim3(grid), dim3(256), 0, s, a, qu, qi, n, out);
    else
        hipLaunchKernelGGL((k_predict<FP, 2>), dim3(grid), dim3(256), 0, s, a, qu, qi, n, out);
}

int run_predict(lshmf_ctx* c, const int32_t* qu, const int32_t* qi, int64_t n, float* out, hipStream_t s)
{
    if (n <= 0) return LSHMF_OK;
    const lshmf_dims& d = c->d;
    PredArgs a{c->t.JK, c->t.b0, c->t.bh0, c->t.mu, c->t.U, c->t.V, c->t.bu, c->t.bv, c->t.W, c->t.C,
               c->row_ptr, c->csr_col, c->csr_rc, d.M, d.N, d.F, d.K, 1.0f / (float)d.rscale};
    int64_t blocks = ceil_div(n * kWave, 256);
    if (blocks > 65536) blocks = 65536;
    const int fp = (d.F + kWave - 1) / kWave;
    switch (fp) {
        case 1: launch_predict_k<1>(a, qu, qi, n, out, (unsigned)blocks, s); break;
        case 2: launch_predict_k<2>(a, qu, qi, n, out, (unsigned)blocks, s); break;
        case 3: launch_predict_k<3>(a, qu, qi, n, out, (unsigned)blocks, s); break;
        default: launch_predict_k<4>(a, qu, qi, n, out, (unsigned)blocks, s); break;
    }
    LSHMF_LAUNCHED("k_predict");
    return LSHMF_OK;
}

// ------------------------------------------------------------------- RMSE
constexpr int kSseBlocks = 512;

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

int run_rmse(lshmf_ctx* c, const float* pred, const uint8_t* rc, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sse_partial, dim3(kSseBlocks), dim3(256), 0, s, pred, rc, n,
                       1.0 / (double)c->d.rscale, c->red);
    LSHMF_LAUNCHED("k_sse_partial");
    hipLaunchKernelGGL(k_sse_final, dim3(1), dim3(256), 0, s, c->red, kSseBlocks, n, out);
    LSHMF_LAUNCHED("k_sse_final");
    return LSHMF_OK;
}

}  // namespace lshmf
