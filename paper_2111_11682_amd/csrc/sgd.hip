// Neighbourhood-MF SGD over the stratified block stream (Alg. CULSH-MF,
// Eq. sgd_update with the prediction of Eq. rr).
//
// k_sgd_stratum: one workgroup per block of the stratum, kSgdWaves waves.
// Blocks of a stratum share no user and no item; inside a block a rating
// waits (LDS mailbox with sequence numbers) for the previous rating of the
// same user, which makes the result that of running the block's ratings in
// stream order.  The item state {v_j, bh_j, w_j, c_j} of a run stays in
// registers; lanes own features f = lane + 64x and neighbour slots
// k = lane + 64y.
//
// Group recurrence.  The ratings of one item run are taken G at a time.  With
// the decays a = 1 - gamma * lambda of Eq. (sgd_update) and the item state at
// the group's start, rating t of the group predicts
//     rhat_t = P_t + sum_{s<t} Q_ts e_s
//     P_t  = mu + b_i + a_b^t bh + a_v^t u_t.v
//            + sum_k x_tk (a_w^{n_k(t)} w_k  or  a_c^{m_k(t)} c_k)
//     Q_ts = g_b a_b^{t-1-s} + g_v a_v^{t-1-s} u_t.u_s
//            + sum_k x_tk x_sk g a^{n_k(t)-n_k(s)-1}   (slots on the same side)
// where x_tk is the neighbour coefficient of slot k for rating t
// (|R^K|^-1/2 (r - bbar) on an explicit slot, |N^K|^-1/2 on an implicit one),
// n_k(t) / m_k(t) count the group's earlier ratings with slot k explicit /
// implicit, and g, a are the rate and decay of w (explicit) or c (implicit).
// The Q_ts involve no error and no item state, so they are computed apart
// from the dependent chain; the errors then follow from the forward
// substitution e_t = r_t - P_t - sum_{s<t} Q_ts e_s, and the state moves to
// the group's end in closed form.  This is Eq. (sgd_update) in stream order,
// reassociated: the same values up to FP32 rounding.
//
// Roles.  The block's first runs, when long, each get a gang: helper waves
// load and prepare groups (user rows from HBM or the mailbox, neighbour
// coefficients, the Q_ts) into an LDS ring, and an item wave runs only the
// chain (P_t, the substitution, the state and user-row updates).  The other
// runs are taken one wave per run, doing both parts.
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "wave.hpp"

namespace lshmf {

constexpr int kSgdWaves = 16;
constexpr int kHelpers = 4;                      // helper waves of a gang
constexpr int kGangWaves = kHelpers + 1;
constexpr int kMaxGangs = 2;                     // gangs per block
constexpr int kGangMin = 48;                     // shortest run given a gang
constexpr int kMaxRingGroups = 8;                // groups in a gang's ring
constexpr int kSpinLimit = 1 << 24;              // bounded wait: a broken hand-over ends the kernel
constexpr int kMaxMailboxBytes = 150 * 1024;     // mailbox part of a block's dynamic LDS
constexpr int kMaxLdsBytes = 160 * 1024 - 256;   // all of it (static LDS aside)
static_assert(kMaxGangs * kGangWaves <= kSgdWaves, "every gang role needs a wave");
constexpr int kMaxChainPos = (1 << 14) - 1;      // link encoding limits
constexpr int kMaxSlots = (1 << 16) - 2;

struct SgdArgs {
    const uint8_t* nib;
    const int64_t* blk_ptr;
    const int64_t* blk_seg;
    const int32_t* seg_col;
    const int64_t* seg_start;
    const float* nbr_b0;
    const float* b0;
    const double* mu;
    float* U;
    float* V;
    float* bu;
    float* bv;
    float* W;
    float* C;
    float* trash;
    int32_t* err;
    int F, K, P, nstride, s, slots;
    int max_gangs;    // gangs the LDS holds (0: every run is taken by a single wave)
    int ring_groups;  // groups in each gang's ring
    int ring_off;     // float offset of the gang rings in dynamic LDS
    float inv_s;
    // Eq. (sgd_update) as decay and rate: theta <- a theta + g (e x); a frozen
    // side has a = 1, g = 0
    float a_u, g_u, a_bu, g_bu;                  // user side: u_i, b_i
    float a_w, a_c, g_w, g_c, inv_aw, inv_ac;    // item side: w_j, c_j
    float pav[9], pab[9];                        // a_v^t, a_b^t
    float pvi[8];                                // g_v a_v^-(t+1)
    float gvp[8], gbp[8];                        // g_v a_v^t, g_b a_b^t
};

__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }
__host__ __device__ constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) >> 1); }

// Floats of one ring group of a gang: G rating slots (u: F, x-tilde: K,
// x-acute: K, explicit-slot masks: 4 words), G headers (r - mu - b_i, b_i,
// user, hand-over word), the G x G matrix Q and the group-end decay powers
// of the w and c slots (2K).
__host__ __device__ inline int ring_mask_off(int F, int K) { return (F + 2 * K + 1) & ~1; }
__host__ __device__ inline int ring_slot_floats(int F, int K) { return ring_mask_off(F, K) + 4; }
__host__ __device__ inline int ring_group_floats(int F, int K, int G)
{
    return ((G * ring_slot_floats(F, K) + 4 * G + G * G + 2 * K) + 3) & ~3;
}

// Sums NP values (a power of two <= 64) over the wave at once: each of
// log2(NP) halving steps sends half of a lane's values to the partner lane
// and adds the other half it receives; lane l ends with the total of value
// l >> (6 - log2 NP).  Fixed association order.
template <int NP>
__device__ inline float batched_sum(float (&v)[NP], int lane)
{
    constexpr int LOG = ilog2c(NP);
#pragma unroll
    for (int st = 0; st < LOG; ++st) {
        const int m = 32 >> st;
        const int h = NP >> (st + 1);
        const bool up = (lane & m) != 0;
#pragma unroll
        for (int i = 0; i < NP / 2; ++i) {
            if (i < h) {
                const float keep = up ? v[h + i] : v[i];
                const float give = up ? v[i] : v[h + i];
                v[i] = keep + __shfl_xor(give, m, kWave);
            }
        }
    }
    float x = v[0];
#pragma unroll
    for (int m = 32 >> LOG; m >= 1; m >>= 1) x += __shfl_xor(x, m, kWave);
    return x;
}

// HBM inputs of one group, loaded a group ahead of use.  Lane t holds the
// scalars of rating t; rows and neighbour-code bytes are per rating.
template <int FP, int KP, int G>
struct GStage {
    float u[G][FP];
    uint32_t nb[(G + 3) / 4][KP];  // neighbour-code byte of rating t at byte t % 4
    uint32_t pw, lw;  // lane t: (user << 4) | code, hand-over word
    float bi, b0;     // lane t
};

// One rating prepared for the group solve: its (possibly handed-over) user
// row and the neighbour coefficients scaled for P (xt) and for Q and the
// state update (xa).
template <int FP, int KP>
struct Prepared {
    float u[FP];
    float xt[KP], xa[KP];
    uint32_t exm;  // bit y: this lane's slot k = lane + 64y is explicit for the rating
    __device__ bool ex(int y) const { return ((exm >> y) & 1u) != 0; }
};

template <int FP, int KP, int G>
__global__ __launch_bounds__(kSgdWaves* kWave) void k_sgd_stratum(SgdArgs a, const uint32_t* __restrict__ pk,
                                                                   const uint32_t* __restrict__ link)
{
    constexpr int NPAIR = G * (G - 1) / 2;
    constexpr int GP = FP + KP >= 3 ? 2 : 4;           // group of a wave that runs a whole run
    constexpr int NPAIRP = GP * (GP - 1) / 2;
    constexpr int NPP = pow2_at_least(NPAIRP + GP);    // its batched sum: pairs and P values
    // mailbox: slots + 1 rows (the last is a write sink) of F floats, b_i, sequence
    extern __shared__ float smem[];
    __shared__ int next_seg;
    const int F = a.F, K = a.K;
    const int dummy = a.slots;
    float* mb_u = smem;
    float* mb_b = smem + (size_t)(dummy + 1) * F;
    int* mb_seq = reinterpret_cast<int*>(mb_b + dummy + 1);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t blk = (int64_t)a.s * a.P + blockIdx.x;
    const int64_t g0 = a.blk_seg[blk], g1 = a.blk_seg[blk + 1];
    const int nsegs = (int)(g1 - g0);
    int ngang = 0;
    for (int k = 0; k < a.max_gangs && k < nsegs; ++k) {
        if (a.seg_start[g0 + k + 1] - a.seg_start[g0 + k] < kGangMin) break;
        ngang = k + 1;
    }
    const int RG = a.ring_groups;
    const int GS = ring_group_floats(F, K, G);
    const int RS = ring_slot_floats(F, K);
    const int gang_floats = RG * GS + 2 * kMaxRingGroups;
    float* rings = smem + a.ring_off;
    for (int x = threadIdx.x; x <= dummy; x += blockDim.x) mb_seq[x] = 0;
    for (int gi = 0; gi < ngang; ++gi) {
        int* fl = reinterpret_cast<int*>(rings + (size_t)gi * gang_floats + RG * GS);
        for (int x = threadIdx.x; x < 2 * kMaxRingGroups; x += blockDim.x) fl[x] = 0;  // ready[], done[]
    }
    if (threadIdx.x == 0) next_seg = ngang;
    __syncthreads();
    const float mu = (float)(*a.mu);
    const float inv_s = a.inv_s;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));  // wave-uniform
    bool dead = false;  // after one failed wait, later waits are skipped so the kernel ends

    // ---- shared pieces -------------------------------------------------------
    // HBM loads of the group of `cnt` ratings at stream positions p0..; no waits
    auto stage = [&](auto& S, int64_t p0, int cnt) {
        constexpr int GG = std::extent<decltype(S.u)>::value;
        S.pw = lane < cnt ? pk[p0 + lane] : 0u;
        S.lw = lane < cnt ? link[p0 + lane] : 0u;
        const int64_t il = S.pw >> 4;
        S.bi = a.bu[il];
        S.b0 = a.b0[il];
#pragma unroll
        for (int x = 0; x < (GG + 3) / 4; ++x)
#pragma unroll
            for (int y = 0; y < KP; ++y) S.nb[x][y] = 0u;
#pragma unroll
        for (int t = 0; t < GG; ++t) {
            const int64_t i = (uint32_t)__builtin_amdgcn_readlane((int)S.pw, t) >> 4;
#pragma unroll
            for (int x = 0; x < FP; ++x) {
                const int f = lane + x * kWave;
                S.u[t][x] = *(f < F ? a.U + i * F + f : a.trash + lane);
            }
            // positions past the run read the zero padding after the stream
            const uint8_t* nbp = a.nib + (p0 + t) * a.nstride;
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                const int byte = (lane >> 1) + y * (kWave / 2);
                S.nb[t >> 2][y] |= (uint32_t)nbp[byte < a.nstride ? byte : 0] << (8 * (t & 3));
            }
        }
    };
    // Waits for the hand-over of rating t's user (when an earlier rating of the
    // user in this block precedes it), then its row and b_i, and the
    // neighbour coefficients x of its slots.  Running decay powers of the
    // group (pw, pc: a^n before this rating; iw, ic: g a^-(n+1)) advance.
    float bhn[KP];
    auto prep = [&](const auto& S, int t, Prepared<FP, KP>& R, float& bi_out, float (&pw)[KP], float (&pc)[KP],
                    float (&iw)[KP], float (&ic)[KP]) {
        const uint32_t lw = (uint32_t)__builtin_amdgcn_readlane((int)S.lw, t);
        const bool has_pred = ((lw >> 30) & 1u) != 0;
        const int pslot = has_pred ? (int)(lw & 0xFFFFu) : dummy;
        if (has_pred) {
            const int want = (int)((lw >> 16) & 0x3FFFu);
            int spins = 0;
            while (!dead && __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                &mb_seq[pslot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) != want) {
                if (++spins > kSpinLimit) {
                    if (lane == 0) atomicOr(a.err, 2);
                    dead = true;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
#pragma unroll
        for (int x = 0; x < FP; ++x) {
            const int f = lane + x * kWave;
            const float mv = mb_u[f < F ? pslot * F + f : dummy * F];
            R.u[x] = f < F ? (has_pred ? mv : S.u[t][x]) : 0.0f;
        }
        const float bi_s = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, S.bi), t));
        const float b0_s = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, S.b0), t));
        bi_out = has_pred ? mb_b[pslot] : bi_s;
        const float base_i = mu + b0_s;
        int code[KP];
        int nR = 0;
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            const int k = lane + y * kWave;
            code[y] = k < K ? (int)((S.nb[t >> 2][y] >> (8 * (t & 3) + (lane & 1) * 4)) & 15u) : 0;
            nR += __popcll(__ballot(code[y] != 0));
        }
        const float sR = nR > 0 ? __builtin_amdgcn_rsqf((float)nR) : 0.0f;
        const float sN = K - nR > 0 ? __builtin_amdgcn_rsqf((float)(K - nR)) : 0.0f;
        R.exm = 0u;
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            const int k = lane + y * kWave;
            const bool ex = code[y] != 0;
            const bool im = !ex && k < K;
            const float x = ex ? ((float)code[y] * inv_s - base_i - bhn[y]) * sR : (im ? sN : 0.0f);
            R.exm |= (ex ? 1u : 0u) << y;
            R.xt[y] = x * (ex ? pw[y] : pc[y]);
            R.xa[y] = x * (ex ? iw[y] : ic[y]);
            pw[y] = ex ? pw[y] * a.a_w : pw[y];
            iw[y] = ex ? iw[y] * a.inv_aw : iw[y];
            pc[y] = im ? pc[y] * a.a_c : pc[y];
            ic[y] = im ? ic[y] * a.inv_ac : ic[y];
        }
    };
    // pair (t, s), s < t, of a group -> index t(t-1)/2 + s
    auto pair_part = [&](const Prepared<FP, KP>& T, const Prepared<FP, KP>& Sr, int t, int s) {
        float uu = 0.0f;
#pragma unroll
        for (int x = 0; x < FP; ++x) uu += T.u[x] * Sr.u[x];
        float q = a.gvp[t - 1 - s] * uu;
#pragma unroll
        for (int y = 0; y < KP; ++y) q += (T.ex(y) == Sr.ex(y)) ? T.xt[y] * Sr.xa[y] : 0.0f;
        return q;
    };
    // The chain of one group: the errors from P (lane t: r - mu - b_i - P_t, the
    // item-state part still to subtract) and the rows of Q, then the user rows
    // and the item state moved to the group's end.  Lane t of reff/bi/lw holds
    // rating t; cnt <= G ratings.
    float v[FP], w[KP], c[KP], bh = 0.0f;
    auto chain = [&](const auto& R, float pt_l, float reff_l, float bi_l, uint32_t user_l, uint32_t lw_l,
                     const auto& qrow, const float (&pwg)[KP], const float (&pcg)[KP], int cnt) {
        constexpr int GN = std::extent<std::remove_reference_t<decltype(R)>>::value;
        // lane t: e_t after the substitution
        float val = reff_l - a.pab[lane < GN ? lane : 0] * bh - pt_l;
        float e[GN];
#pragma unroll
        for (int s = 0; s < GN; ++s) {
            e[s] = 0.0f;
            if (s < cnt) {
                e[s] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, val), s));
                val -= lane > s ? qrow[s] * e[s] : 0.0f;
            }
        }
        // user rows from v_t, the item vector before rating t, then the state
        float vacc[FP], wacc[KP], cacc[KP];
#pragma unroll
        for (int x = 0; x < FP; ++x) vacc[x] = 0.0f;
#pragma unroll
        for (int y = 0; y < KP; ++y) wacc[y] = cacc[y] = 0.0f;
#pragma unroll
        for (int t = 0; t < GN; ++t) {
            if (t >= cnt) break;
            const int64_t i = (int64_t)__builtin_amdgcn_readlane((int)user_l, t);
            const uint32_t lw = (uint32_t)__builtin_amdgcn_readlane((int)lw_l, t);
            const bool has_succ = (lw >> 31) != 0;
            const int ws = has_succ ? (int)(lw & 0xFFFFu) : dummy;
            // wave-uniform destinations: the HBM row or a sink row
            float* urow = has_succ ? a.trash + kWave * FP : a.U + i * F;
            float* mrow = mb_u + ws * F;
            const float gu = a.g_u * e[t] * a.pav[t];
            const float gv = a.pvi[t] * e[t];
#pragma unroll
            for (int x = 0; x < FP; ++x) {
                const int f = lane + x * kWave;
                const float vt = v[x] + vacc[x];
                const float unew = a.a_u * R[t].u[x] + gu * vt;
                if (f < F) {
                    mrow[f] = unew;
                    urow[f] = unew;
                }
                vacc[x] += gv * R[t].u[x];
            }
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                const float d = e[t] * R[t].xa[y];
                wacc[y] += R[t].ex(y) ? d : 0.0f;
                cacc[y] += R[t].ex(y) ? 0.0f : d;
            }
        }
        const float pv = a.pav[cnt < GN ? cnt : GN];
#pragma unroll
        for (int x = 0; x < FP; ++x) v[x] = pv * (v[x] + vacc[x]);
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            w[y] = pwg[y] * (w[y] + wacc[y]);
            c[y] = pcg[y] * (c[y] + cacc[y]);
        }
        float bn = a.pab[cnt < GN ? cnt : GN] * bh;
#pragma unroll
        for (int t = 0; t < GN; ++t)
            if (t < cnt) bn += a.gbp[cnt - 1 - t] * e[t];
        bh = bn;
        // b_i of lane t's user to the mailbox or HBM, then the hand-over numbers
        const bool live = lane < cnt;
        const bool succ = live && (lw_l >> 31) != 0;
        const int ws = succ ? (int)(lw_l & 0xFFFFu) : dummy;
        const float bnew = a.a_bu * bi_l + a.g_bu * val;
        if (live) {
            mb_b[ws] = bnew;
            *(succ ? a.trash + 2 * kWave * FP + lane : a.bu + user_l) = bnew;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        if (succ)
            __hip_atomic_store(&mb_seq[ws], (int)((lw_l >> 16) & 0x3FFFu) + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto load_item = [&](int64_t j) {
#pragma unroll
        for (int x = 0; x < FP; ++x) {
            const int f = lane + x * kWave;
            v[x] = f < F ? a.V[j * F + f] : 0.0f;
        }
        bh = a.bv[j];
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            const int k = lane + y * kWave;
            w[y] = k < K ? a.W[j * K + k] : 0.0f;
            c[y] = k < K ? a.C[j * K + k] : 0.0f;
        }
    };
    auto load_bhn = [&](int64_t j) {
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            const int k = lane + y * kWave;
            bhn[y] = k < K ? a.nbr_b0[j * K + k] : 0.0f;
        }
    };
    auto store_item = [&](int64_t j) {
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
    };
    // the P-value of every rating of the group: dots with the group-start state
    auto p_parts = [&](const auto& R, auto& p) {
        constexpr int GN = std::extent<std::remove_reference_t<decltype(R)>>::value;
#pragma unroll
        for (int t = 0; t < GN; ++t) {
            float uv = 0.0f;
#pragma unroll
            for (int x = 0; x < FP; ++x) uv += R[t].u[x] * v[x];
            float q = a.pav[t] * uv;
#pragma unroll
            for (int y = 0; y < KP; ++y) q += R[t].xt[y] * (R[t].ex(y) ? w[y] : c[y]);
            p[t] = q;
        }
    };

    if (wv < ngang * kGangWaves) {
        // ---- a gang: helpers fill ring groups, the item wave consumes them
        const int gang = wv / kGangWaves, role = wv % kGangWaves;
        const int64_t seg = g0 + gang;
        const int64_t j = a.seg_col[seg];
        const int64_t ea = a.seg_start[seg];
        const int len = (int)(a.seg_start[seg + 1] - ea);
        const int ngroups = (len + G - 1) / G;
        float* ring = rings + (size_t)gang * gang_floats;
        int* ready = reinterpret_cast<int*>(ring + RG * GS);
        int* done = ready + kMaxRingGroups;
        if (role == 0) {
            // ---- item wave
            __builtin_amdgcn_s_setprio(3);
            load_item(j);
            for (int g = 0; g < ngroups; ++g) {
                const int cnt = len - g * G < G ? len - g * G : G;
                const int gs = g % RG;
                int spins = 0;
                while (!dead && __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                    &ready[gs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) != g + 1) {
                    if (++spins > kSpinLimit) {
                        if (lane == 0) atomicOr(a.err, 4);
                        dead = true;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                const float* base = ring + (size_t)gs * GS;
                Prepared<FP, KP> R[G];
#pragma unroll
                for (int t = 0; t < G; ++t) {
                    const float* d = base + t * RS;
                    const bool ok = t < cnt;
#pragma unroll
                    for (int x = 0; x < FP; ++x) {
                        const int f = lane + x * kWave;
                        const float uv = d[f < F ? f : 0];
                        R[t].u[x] = (ok && f < F) ? uv : 0.0f;
                    }
                    const uint64_t* eb = reinterpret_cast<const uint64_t*>(d + ring_mask_off(F, K));
                    R[t].exm = 0u;
#pragma unroll
                    for (int y = 0; y < KP; ++y) {
                        const int k = lane + y * kWave;
                        const float xt = d[F + (k < K ? k : 0)], xa = d[F + K + (k < K ? k : 0)];
                        const bool inb = ok && k < K;
                        R[t].xt[y] = inb ? xt : 0.0f;
                        R[t].xa[y] = inb ? xa : 0.0f;
                        R[t].exm |= (inb && ((eb[y] >> lane) & 1ull)) ? (1u << y) : 0u;
                    }
                }
                const int* hd = reinterpret_cast<const int*>(base + G * RS) + 4 * (lane < cnt ? lane : 0);
                const float reff_l = __int_as_float(hd[0]);
                const float bi_l = __int_as_float(hd[1]);
                const uint32_t user_l = (uint32_t)hd[2];
                const uint32_t lw_l = lane < cnt ? (uint32_t)hd[3] : 0u;
                const float* qb = base + G * RS + 4 * G + (lane < G ? lane : 0) * G;
                float qrow[G];
#pragma unroll
                for (int s = 0; s < G; ++s) qrow[s] = qb[s];
                float pwg[KP], pcg[KP];
                const float* pg = base + G * RS + 4 * G + G * G;
#pragma unroll
                for (int y = 0; y < KP; ++y) {
                    const int k = lane + y * kWave;
                    pwg[y] = k < K ? pg[k] : 1.0f;
                    pcg[y] = k < K ? pg[K + k] : 1.0f;
                }
                // the ring group is read: hand it back to its helper
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                if (lane == 0) __hip_atomic_store(&done[gs], g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                float p[G];
                p_parts(R, p);
                const float tot = batched_sum<G>(p, lane);
                const float pt_l = __shfl(tot, (lane < G ? lane : 0) << (6 - ilog2c(G)), kWave);
                chain(R, pt_l, reff_l, bi_l, user_l, lw_l, qrow, pwg, pcg, cnt);
            }
            __builtin_amdgcn_s_setprio(0);
            store_item(j);
        } else {
            // ---- helper h: groups h, h + H, ... of the run
            const int h = role - 1;
            load_bhn(j);
            GStage<FP, KP, G> SA;
            if (h < ngroups) stage(SA, ea + (int64_t)h * G, len - h * G < G ? len - h * G : G);
            for (int g = h; g < ngroups; g += kHelpers) {
                const int cnt = len - g * G < G ? len - g * G : G;
                const int gs = g % RG;
                GStage<FP, KP, G> SB;
                const int gn = g + kHelpers;
                if (gn < ngroups) stage(SB, ea + (int64_t)gn * G, len - gn * G < G ? len - gn * G : G);
                // the ring group's previous occupant must have been read
                if (g >= RG) {
                    int spins = 0;
                    while (!dead && __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                        &done[gs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) < g - RG + 1) {
                        if (++spins > kSpinLimit) {
                            if (lane == 0) atomicOr(a.err, 4);
                            dead = true;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                }
                float* base = ring + (size_t)gs * GS;
                float pw[KP], pc[KP], iw[KP], ic[KP];
#pragma unroll
                for (int y = 0; y < KP; ++y) {
                    pw[y] = pc[y] = 1.0f;
                    iw[y] = a.g_w * a.inv_aw;
                    ic[y] = a.g_c * a.inv_ac;
                }
                int* hdw = reinterpret_cast<int*>(base + G * RS);
                // Q: the pairs of the group, each added as soon as its later rating
                // is prepared (the earlier one is read back from the ring)
                // rows [1, TS) are summed first, rows [TS, G) second (fewer live registers)
                constexpr int TS = G > 6 ? 6 : G;
                constexpr int NQ1 = pow2_at_least(TS * (TS - 1) / 2);
                constexpr int NQ2 = pow2_at_least(NPAIR - TS * (TS - 1) / 2);
                float q[NQ1 > NQ2 ? NQ1 : NQ2];
                auto flush_pairs = [&](auto& qq, int first, int count) {
                    constexpr int NQ = std::extent<std::remove_reference_t<decltype(qq)>>::value;
                    const float tot = batched_sum<NQ>(qq, lane);
                    const int idx = first + (lane >> (6 - ilog2c(NQ)));
                    if ((lane & ((1 << (6 - ilog2c(NQ))) - 1)) == 0 && idx - first < count) {
                        int tq = 1;
                        while (tq * (tq + 1) / 2 <= idx) ++tq;
                        const int sq = idx - tq * (tq - 1) / 2;
                        base[G * RS + 4 * G + tq * G + sq] = tot + a.gbp[tq - 1 - sq];
                    }
                };
#pragma unroll
                for (int x = 0; x < NQ1; ++x) q[x] = 0.0f;
#pragma unroll
                for (int t = 0; t < G; ++t) {
                    if (t == TS) {
                        float q1[NQ1];
#pragma unroll
                        for (int x = 0; x < NQ1; ++x) q1[x] = q[x];
                        flush_pairs(q1, 0, TS * (TS - 1) / 2);
#pragma unroll
                        for (int x = 0; x < NQ2; ++x) q[x] = 0.0f;
                    }
                    if (t < cnt) {
                        Prepared<FP, KP> Rt;
                        float bi = 0.0f;
                        prep(SA, t, Rt, bi, pw, pc, iw, ic);
                        float* d = base + t * RS;
#pragma unroll
                        for (int x = 0; x < FP; ++x) {
                            const int f = lane + x * kWave;
                            if (f < F) d[f] = Rt.u[x];
                        }
#pragma unroll
                        for (int y = 0; y < KP; ++y) {
                            const int k = lane + y * kWave;
                            if (k < K) {
                                d[F + k] = Rt.xt[y];
                                d[F + K + k] = Rt.xa[y];
                            }
                            const uint64_t m = __ballot(Rt.ex(y));
                            if (lane == 0) reinterpret_cast<uint64_t*>(d + ring_mask_off(F, K))[y] = m;
                        }
                        if (lane == 0) {
                            const uint32_t pwv = (uint32_t)__builtin_amdgcn_readlane((int)SA.pw, t);
                            const float r = (float)(pwv & 15u) * inv_s;
                            hdw[4 * t + 0] = __float_as_int(r - (mu + bi));
                            hdw[4 * t + 1] = __float_as_int(bi);
                            hdw[4 * t + 2] = (int)(pwv >> 4);
                            hdw[4 * t + 3] = __builtin_amdgcn_readlane((int)SA.lw, t);
                        }
#pragma unroll
                        for (int s2 = 0; s2 < t; ++s2) {
                            const float* ds = base + s2 * RS;
                            const uint64_t* ebs = reinterpret_cast<const uint64_t*>(ds + ring_mask_off(F, K));
                            Prepared<FP, KP> Rs;
#pragma unroll
                            for (int x = 0; x < FP; ++x) {
                                const int f = lane + x * kWave;
                                const float uv = ds[f < F ? f : 0];
                                Rs.u[x] = f < F ? uv : 0.0f;
                            }
                            Rs.exm = 0u;
#pragma unroll
                            for (int y = 0; y < KP; ++y) {
                                const int k = lane + y * kWave;
                                const float xa = ds[F + K + (k < K ? k : 0)];
                                Rs.xa[y] = k < K ? xa : 0.0f;
                                Rs.xt[y] = 0.0f;
                                Rs.exm |= (k < K && ((ebs[y] >> lane) & 1ull)) ? (1u << y) : 0u;
                            }
                            const int pidx = t * (t - 1) / 2 + s2 - (t >= TS ? TS * (TS - 1) / 2 : 0);
                            q[pidx] = pair_part(Rt, Rs, t, s2);
                        }
                    }
                }
                float* pg = base + G * RS + 4 * G + G * G;
#pragma unroll
                for (int y = 0; y < KP; ++y) {
                    const int k = lane + y * kWave;
                    if (k < K) {
                        pg[k] = pw[y];
                        pg[K + k] = pc[y];
                    }
                }
                if (TS < G) {
                    float q2[NQ2];
#pragma unroll
                    for (int x = 0; x < NQ2; ++x) q2[x] = q[x];
                    flush_pairs(q2, TS * (TS - 1) / 2, NPAIR - TS * (TS - 1) / 2);
                } else {
                    float q1[NQ1];
#pragma unroll
                    for (int x = 0; x < NQ1; ++x) q1[x] = q[x];
                    flush_pairs(q1, 0, NPAIR);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                if (lane == 0) __hip_atomic_store(&ready[gs], g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                SA = SB;
            }
        }
    }

    // ---- the other runs: one wave per run, both parts
    while (true) {
        int gsel = 0;
        if (lane == 0) gsel = atomicAdd(&next_seg, 1);
        gsel = __builtin_amdgcn_readfirstlane(gsel);
        if (gsel >= nsegs) break;
        const int64_t seg = g0 + gsel;
        const int64_t j = a.seg_col[seg];
        const int64_t ea = a.seg_start[seg];
        const int len = (int)(a.seg_start[seg + 1] - ea);
        if (len > 4 * GP) __builtin_amdgcn_s_setprio(2);
        load_item(j);
        load_bhn(j);
        const int ngroups = (len + GP - 1) / GP;
        GStage<FP, KP, GP> SA;
        stage(SA, ea, len < GP ? len : GP);
        for (int g = 0; g < ngroups; ++g) {
            const int cnt = len - g * GP < GP ? len - g * GP : GP;
            GStage<FP, KP, GP> SB;
            const int gn = g + 1;
            if (gn < ngroups) stage(SB, ea + (int64_t)gn * GP, len - gn * GP < GP ? len - gn * GP : GP);
            Prepared<FP, KP> R[GP];
            float pw[KP], pc[KP], iw[KP], ic[KP];
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                pw[y] = pc[y] = 1.0f;
                iw[y] = a.g_w * a.inv_aw;
                ic[y] = a.g_c * a.inv_ac;
            }
            float bi_l = 0.0f;
            // pairs (Q) and P values, each added as soon as its rating is prepared
            float q[NPP];
#pragma unroll
            for (int x = 0; x < NPP; ++x) q[x] = 0.0f;
#pragma unroll
            for (int t = 0; t < GP; ++t) {
                if (t < cnt) {
                    float bi = 0.0f;
                    prep(SA, t, R[t], bi, pw, pc, iw, ic);
                    bi_l = lane == t ? bi : bi_l;
                    float uv = 0.0f;
#pragma unroll
                    for (int x = 0; x < FP; ++x) uv += R[t].u[x] * v[x];
                    float pp = a.pav[t] * uv;
#pragma unroll
                    for (int y = 0; y < KP; ++y) pp += R[t].xt[y] * (R[t].ex(y) ? w[y] : c[y]);
                    q[NPAIRP + t] = pp;
#pragma unroll
                    for (int s2 = 0; s2 < t; ++s2) q[t * (t - 1) / 2 + s2] = pair_part(R[t], R[s2], t, s2);
                } else {
#pragma unroll
                    for (int x = 0; x < FP; ++x) R[t].u[x] = 0.0f;
#pragma unroll
                    for (int y = 0; y < KP; ++y) R[t].xt[y] = R[t].xa[y] = 0.0f;
                    R[t].exm = 0u;
                }
            }
            const float tot = batched_sum<NPP>(q, lane);
            constexpr int SH = 6 - ilog2c(NPP);
            const int tl = lane < GP ? lane : 0;
            float qrow[GP];
#pragma unroll
            for (int s = 0; s < GP; ++s) {
                const int idx = s < tl ? tl * (tl - 1) / 2 + s : 0;
                const float qv = __shfl(tot, idx << SH, kWave);
                qrow[s] = s < tl ? qv + a.gbp[s < tl ? tl - 1 - s : 0] : 0.0f;
            }
            const float pt_l = __shfl(tot, (NPAIRP + tl) << SH, kWave);
            const uint32_t pwl = lane < cnt ? SA.pw : 0u;
            const float r = (float)(pwl & 15u) * inv_s;
            const float reff_l = r - (mu + bi_l);
            chain(R, pt_l, reff_l, bi_l, pwl >> 4, lane < cnt ? SA.lw : 0u, qrow, pw, pc, cnt);
            SA = SB;
        }
        __builtin_amdgcn_s_setprio(0);
        store_item(j);
    }
}

// Dynamic LDS of one block: the mailbox (slots + 1 rows of F floats, b_i and
// a sequence word) and the gang rings with their flags.
template <int G>
static size_t sgd_lds_bytes(const SgdArgs& args)
{
    const size_t gang = (size_t)args.ring_groups * ring_group_floats(args.F, args.K, G) + 2 * kMaxRingGroups;
    return ((size_t)args.ring_off + (size_t)args.max_gangs * gang) * sizeof(float);
}

template <int FP, int KP, int G>
static int launch_sgd(SgdArgs args, const uint32_t* pk, const uint32_t* link, hipStream_t s)
{
    // as many ring groups and gangs as fit beside the mailbox
    args.max_gangs = kMaxGangs;
    args.ring_groups = kMaxRingGroups;
    while (sgd_lds_bytes<G>(args) > (size_t)kMaxLdsBytes) {
        if (args.ring_groups > 4) args.ring_groups = 4;
        else if (args.max_gangs > 0) {
            --args.max_gangs;
            args.ring_groups = kMaxRingGroups;
        } else break;
    }
    if (args.max_gangs == 0) args.ring_groups = 1;
    const size_t lds = sgd_lds_bytes<G>(args);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sgd_stratum<FP, KP, G>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(k_sgd_stratum)");
    }
    hipLaunchKernelGGL((k_sgd_stratum<FP, KP, G>), dim3((unsigned)args.P), dim3(kSgdWaves * kWave), lds, s, args,
                       pk, link);
    LSHMF_LAUNCHED("k_sgd_stratum");
    return LSHMF_OK;
}

// Group size: 8 ratings where the rows are short, 4 where the registers of
// eight prepared ratings would not fit.
template <int FP>
static int launch_sgd_k(const SgdArgs& args, const uint32_t* pk, const uint32_t* link, hipStream_t s)
{
    if (args.K > kWave) return launch_sgd<FP, 2, 4>(args, pk, link, s);
    if constexpr (FP <= 1) return launch_sgd<FP, 1, 8>(args, pk, link, s);
    else return launch_sgd<FP, 1, 4>(args, pk, link, s);
}

// Can k_sgd_stratum run this stream: the mailbox of every block in LDS and
// its chain positions and slots inside the hand-over word's fields?
int sgd_fits(const lshmf_ctx* c, const Stream& st)
{
    const size_t lds = (size_t)(st.max_block_slots + 1) * (c->d.F + 2) * sizeof(float);
    if (st.max_block_slots > kMaxSlots || lds > (size_t)kMaxMailboxBytes || st.max_block_nnz > kMaxChainPos) {
        set_error("sgd: a block needs %lld mailbox slots (%zu bytes of LDS, limit %d) or holds %lld "
                  "ratings (limit %d); raise n_strata",
                  (long long)st.max_block_slots, lds, kMaxMailboxBytes, (long long)st.max_block_nnz, kMaxChainPos);
        return LSHMF_ECAPACITY;
    }
    return LSHMF_OK;
}

// One SGD pass over a stream; upd selects the parameter sides to update.
int run_sgd(lshmf_ctx* c, Stream& st, const lshmf_hparams* hp, int epoch, int upd, hipStream_t s)
{
    const lshmf_dims& d = c->d;
    if (st.n == 0) return LSHMF_OK;
    LSHMF_TRY(sgd_fits(c, st));
    SgdArgs a;
    // K = 0: no codes; the kernel's clamped code reads then land on the sink
    a.nib = c->nstride > 0 ? st.nib : reinterpret_cast<const uint8_t*>(c->trash);
    a.blk_ptr = st.blk_ptr;
    a.blk_seg = st.blk_seg;
    a.seg_col = st.seg_col;
    a.seg_start = st.seg_start;
    a.nbr_b0 = c->nbr_b0;
    a.b0 = c->t.b0;
    a.mu = c->t.mu;
    a.U = c->t.U;
    a.V = c->t.V;
    a.bu = c->t.bu;
    a.bv = c->t.bv;
    a.W = c->t.W;
    a.C = c->t.C;
    a.trash = c->trash;
    a.err = c->err;
    a.F = d.F;
    a.K = d.K;
    a.P = c->P;
    a.nstride = c->nstride;
    a.slots = (int)st.max_block_slots;
    a.inv_s = 1.0f / (float)d.rscale;
    a.ring_off = (int)(((st.max_block_slots + 1) * (d.F + 2) + 3) & ~3LL);
    a.max_gangs = kMaxGangs;
    a.ring_groups = kMaxRingGroups;
    // Eq. (learn_rate): gamma_t = alpha / (1 + beta * t^1.5); Eq. (sgd_update)
    // as theta <- (1 - gamma lambda) theta + gamma (e x).  Order of the six
    // groups: b_i, bh_j, u_i, v_j, w_j, c_j.
    const double den = 1.0 + (double)hp->beta * std::pow((double)epoch, 1.5);
    double g[6], dec[6];
    for (int x = 0; x < 6; ++x) {
        g[x] = (double)(float)((double)hp->alpha[x] / den);
        dec[x] = 1.0 - g[x] * (double)hp->lambda[x];
    }
    const bool usr = (upd & 1) != 0, itm = (upd & 2) != 0;
    if (d.model == LSHMF_PLAIN_MF) g[0] = g[1] = 0.0, dec[0] = dec[1] = 1.0;  // no biases to learn
    if (!usr) g[0] = g[2] = 0.0, dec[0] = dec[2] = 1.0;
    if (!itm) g[1] = g[3] = g[4] = g[5] = 0.0, dec[1] = dec[3] = dec[4] = dec[5] = 1.0;
    a.a_bu = (float)dec[0];
    a.g_bu = (float)g[0];
    a.a_u = (float)dec[2];
    a.g_u = (float)g[2];
    a.a_w = (float)dec[4];
    a.a_c = (float)dec[5];
    a.g_w = (float)g[4];
    a.g_c = (float)g[5];
    a.inv_aw = (float)(1.0 / dec[4]);
    a.inv_ac = (float)(1.0 / dec[5]);
    for (int t = 0; t <= 8; ++t) {
        a.pav[t] = (float)std::pow(dec[3], t);
        a.pab[t] = (float)std::pow(dec[1], t);
    }
    for (int t = 0; t < 8; ++t) {
        a.pvi[t] = (float)(g[3] * std::pow(dec[3], -(t + 1)));
        a.gvp[t] = (float)(g[3] * std::pow(dec[3], t));
        a.gbp[t] = (float)(g[1] * std::pow(dec[1], t));
    }
    const int fp = (d.F + kWave - 1) / kWave;
    for (int stratum = 0; stratum < c->P; ++stratum) {
        a.s = stratum;
        switch (fp) {
            case 1: LSHMF_TRY(launch_sgd_k<1>(a, st.pk, st.link, s)); break;
            case 2: LSHMF_TRY(launch_sgd_k<2>(a, st.pk, st.link, s)); break;
            case 3: LSHMF_TRY(launch_sgd_k<3>(a, st.pk, st.link, s)); break;
            default: LSHMF_TRY(launch_sgd_k<4>(a, st.pk, st.link, s)); break;
        }
    }
    return LSHMF_OK;
}

}  // namespace lshmf
