// Neighbourhood-MF SGD over the stratified block stream, prediction and the
// FP64 RMSE reduction.
//
// k_sgd_stratum (Alg. CULSH-MF, Eq. sgd_update with Eq. rr): one workgroup per
// block of the stratum, kSgdWaves waves.  A wave takes the next item run of
// its block (the ratings of one item j), holds the item state {v_j, bh_j, w_j,
// c_j} in registers for the whole run -- the register-resident column state
// of the paper's kernel -- and streams the users' {u_i, b_i} from HBM.  Lanes
// own features f = lane + 64x and neighbour slots k = lane + 64y, so u.v, the
// explicit w-sum and the implicit c-sum of Eq. (rr) fold into ONE 64-lane
// reduction.  The block's first run, when long, is split between an item
// wave that runs only the dependent update chain and helper waves that load
// and prepare the user side (a gang, below).  Blocks of a stratum
// share no user and no item; inside a block, a rating waits (LDS mailbox with
// sequence numbers) for the previous rating of the same user, which makes the
// result identical to running the block's ratings in order.
#include <cmath>

#include "common.hpp"
#include "wave.hpp"

namespace lshmf {

constexpr int kSgdWaves = 16;
constexpr int kGroup = 4;                        // ratings per pipeline stage
constexpr int kHelpers = 4;                      // helper waves of a gang
constexpr int kGangWaves = kHelpers + 2;         // item wave, helpers, writer wave
constexpr int kMaxGangs = 2;                     // gangs per block
// shortest segment given a gang: 48 ratings when a block can hold two gangs,
// 32 when its LDS holds one (measured on the ML-10M and Netflix shapes)
constexpr int kGangMin2 = 48;
constexpr int kGangMin1 = 32;
constexpr int kHG = 1;                           // ratings per helper pipeline stage
constexpr int kTeam = 4;                         // light blocks per team workgroup
constexpr int kIG = 8;                           // ratings per item-wave group
// ring slots of a gang: a power of two (slot = rating & (kRing - 1)) and a
// multiple of kHelpers, so that every slot belongs to one helper, and of kIG,
// so that no group wraps; at least 2 * kHG + 3 per helper, so that a helper
// can prepare two stages ahead of the item wave
constexpr int kRing = 64;
static_assert((kRing & (kRing - 1)) == 0 && kRing % kHelpers == 0 && kRing % kIG == 0 &&
                  kRing >= (2 * kHG + 3) * kHelpers,
              "ring size");
constexpr int kSpinLimit = 1 << 24;              // bounded wait: a broken hand-over ends the kernel
constexpr int kMaxMailboxBytes = 150 * 1024;     // mailbox part of a block's dynamic LDS
constexpr int kMaxLdsBytes = 160 * 1024 - 256;   // all of it (static LDS aside)
static_assert(kMaxGangs * kGangWaves <= kSgdWaves, "every gang role needs a wave");
static_assert(kSgdWaves % kTeam == 0, "team members take equal shares of the waves");
constexpr int kMaxChainPos = (1 << 14) - 1;      // link encoding limits
constexpr int kMaxSlots = (1 << 16) - 2;

struct SgdArgs {
    const uint8_t* nib;
    const int64_t* blk_ptr;
    const int32_t* blk_run;    // 2 P*P: first run and run count of the block at each dispatch position
    const int32_t* seg_col;
    const int64_t* seg_start;
    const float* nbr_b0;
    const float* b0;
    const double* mu;
    float* U;
    uint16_t* U16;    // storage mode BF16_U: the user rows in HBM are BF16 (U unused), else NULL
    float* V;
    float* bu;
    float* bv;
    float* W;
    float* C;
    float* trash;
    int32_t* err;
    int F, K, P, nstride, s, slots;
    int grid;         // workgroups of this stratum's launch
    int nh;           // heavy blocks of this stratum (the first nh workgroups run one each)
    int upd;          // bit 0: update the user side {b_i, u_i}; bit 1: the item side {bh_j, v_j, w_j, c_j}
    int max_gangs;    // gangs the LDS holds (0: every segment is run by a single wave)
    int gang_min;     // shortest segment given a gang
    int team;         // light blocks per team workgroup (1: every block has a workgroup of its own)
    int team_slots;   // mailbox slots of a team member (a light block has at most kLightNnz / 2)
    int team_floats;  // floats of LDS per team member
    int ring_off;     // float offset of the gang rings in dynamic LDS
    int ring_rs;      // floats per ring slot: u (64 FP), rw (64 KP), cn (64 KP), zero-padded
    float inv_s;
    float g[6], l[6];
};

// User-side HBM inputs of one group of ratings, loaded a group ahead of use.
// A user rated earlier in the same block is read from the block's LDS mailbox
// instead, when its rating is computed.
// One parameter update of Eq. (sgd_update), x + g (e q - l x), as the item wave
// and the writer wave of a gang both evaluate it: the writer replays the item
// wave's updates of v_j and must reach the same values bit for bit.
__device__ __forceinline__ float sgd_step(float x, float g, float e, float q, float l)
{
    return __builtin_fmaf(g, __builtin_fmaf(e, q, -(l * x)), x);
}

template <int FP, int KP>
struct Stage {
    float gu[kGroup][FP];
    float gbi[kGroup], b0[kGroup];
    uint32_t nb[kGroup][KP];  // raw neighbour-code bytes of this lane's slots
    uint32_t pk[kGroup];      // (user << 4) | code
    uint32_t lk[kGroup];      // hand-over word
};

// HBM inputs of kHG ratings of a helper wave, loaded a stage ahead of use.
template <int FP, int KP>
struct HStage {
    float u[kHG][FP];
    float bi[kHG], b0[kHG];
    uint32_t nb[kHG][KP];
    uint32_t pw[kHG], lw[kHG];
};

template <int FP, int KP, bool UB>
__global__ __launch_bounds__(kSgdWaves* kWave) void k_sgd_stratum(SgdArgs a, const uint32_t* __restrict__ pk,
                                                                   const uint32_t* __restrict__ link)
{
    // mailbox: slots + 1 rows (the last is a write sink) of F floats, b_i, sequence
    extern __shared__ float smem[];
    __shared__ int next_seg[kTeam];
    const int F = a.F, K = a.K;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));  // wave-uniform
    // The first a.nh workgroups run one block each (the heaviest, with
    // gangs); each later one runs a team of up to a.team light blocks, member m
    // on waves [m W, (m+1) W) with a mailbox of its own.  Blocks of a stratum
    // share no user and no item, so the members never interact.
    const int64_t sP = (int64_t)a.s * a.P;
    const int nh = a.team > 1 ? a.nh : a.P;
    const bool in_team = (int)blockIdx.x >= nh;
    const int member = in_team ? wv / (kSgdWaves / a.team) : 0;
    // dispatch position of this wave's block (-1: none for this member)
    int64_t xpos = (int64_t)blockIdx.x;
    if (in_team) {
        xpos = nh + ((int64_t)blockIdx.x - nh) * a.team + member;
        if (xpos >= a.P) xpos = -1;
    }
    const int dummy = in_team ? a.team_slots : a.slots;
    float* mb_u = smem + (in_team ? (size_t)member * a.team_floats : 0);
    float* mb_b = mb_u + (size_t)(dummy + 1) * F;
    int* mb_seq = reinterpret_cast<int*>(mb_b + dummy + 1);
    const int2 brun = xpos >= 0 ? *reinterpret_cast<const int2*>(a.blk_run + 2 * (sP + xpos)) : make_int2(0, 0);
    const int64_t g0 = brun.x;
    const int nsegs = brun.y;
    // The first segments of the block, while long, each get a gang: an item
    // wave that keeps the item state and runs only the dependent update chain,
    // fed through an LDS ring by helper waves that load and prepare the
    // user-side inputs of every rating.
    int ngang = 0;
    for (int k = 0; !in_team && k < a.max_gangs && k < nsegs; ++k) {
        if (a.seg_start[g0 + k + 1] - a.seg_start[g0 + k] < a.gang_min) break;
        ngang = k + 1;
    }
    const int RS = a.ring_rs;
    const int GS = kRing * (RS + 7) + 4;  // floats per gang: data, headers, ready, done, errors, count
    float* rings = smem + a.ring_off;
    if (!in_team) {
        for (int x = threadIdx.x; x <= dummy; x += blockDim.x) mb_seq[x] = 0;
        for (int gi = 0; gi < ngang; ++gi) {
            int* ready = reinterpret_cast<int*>(rings + (size_t)gi * GS + kRing * RS + kRing * 4);
            for (int x = threadIdx.x; x < 3 * kRing + 1; x += blockDim.x) ready[x] = 0;  // ready, done, err, count
        }
        if (threadIdx.x == 0) next_seg[0] = ngang;
    } else {
        // each member's waves clear its own sequence words
        const int wpm = kSgdWaves / a.team;
        for (int x = (int)threadIdx.x - member * wpm * kWave; x <= dummy; x += wpm * kWave) mb_seq[x] = 0;
        if (threadIdx.x < (unsigned)a.team) next_seg[threadIdx.x] = 0;
    }
    __syncthreads();
    const float mu = (float)(*a.mu);
    const float inv_s = a.inv_s;

    if (wv < ngang * kGangWaves) {
        // Ring protocol.  Helper h prepares ratings n = h, h + H, ... into
        // slot n & (kRing - 1) and sets ready; the item wave runs each group of kIG
        // ratings (the dependent chain of v_j, bh_j, w_j, c_j) and publishes
        // the group's errors; the writer wave then writes each u_i's new row
        // to the mailbox (the user rates again later in the block) or to HBM,
        // b_i, the hand-over sequence numbers and done.  A slot is reused by
        // the same helper kRing / H of its ratings later, once the slot's
        // previous rating is done.  The item wave waits only for ready slots
        // and the writer only for published errors, both of ratings the
        // helpers prepare without waiting on them, so every wait ends.
        const int gang = wv / kGangWaves, role = wv % kGangWaves;
        const int64_t seg = g0 + gang;
        const int64_t j = a.seg_col[seg];
        const int64_t ea = a.seg_start[seg];
        const int len = (int)(a.seg_start[seg + 1] - ea);
        float* rdata = rings + (size_t)gang * GS;
        int* rhdr = reinterpret_cast<int*>(rdata + kRing * RS);
        int* rready = rhdr + kRing * 4;
        int* rdone = rready + kRing;
        float* rerr = reinterpret_cast<float*>(rdone + kRing);
        int* rcount = reinterpret_cast<int*>(rerr + kRing);  // ratings whose errors are published
        if (role == 0) {
            // ---- item wave: Eq. (rr) and Eq. (sgd_update) in stream order
            __builtin_amdgcn_s_setprio(3);
            float v[FP], w[KP], c[KP];
#pragma unroll
            for (int x = 0; x < FP; ++x) {
                const int f = lane + x * kWave;
                v[x] = f < F ? a.V[j * F + f] : 0.0f;
            }
            float bh = a.bv[j];
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                const int k = lane + y * kWave;
                w[y] = k < K ? a.W[j * K + k] : 0.0f;
                c[y] = k < K ? a.C[j * K + k] : 0.0f;
            }
            bool dead = false;  // after one failed wait, later waits are skipped so the kernel ends
            // lane t < cnt checks slot (g0 + t): are all kIG inputs of the group there?
            auto group_ready = [&](int gs, int cnt) {
                const int sl = (gs + lane) & (kRing - 1);
                const int want = gs + lane + 1;
                const bool ok = lane >= cnt ||
                                __hip_atomic_load(&rready[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == want;
                return __ballot(!ok) == 0ull;
            };
            auto wait_group = [&](int gs, int cnt) {
                int spins = 0;
                while (!dead && !group_ready(gs, cnt)) {
                    if (++spins > kSpinLimit) {
                        if (lane == 0) atomicOr(a.err, 4);
                        dead = true;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
            };
            // Inputs of a group from the ring.  Two of them alternate, one
            // computed while the other is loaded, so nothing is copied.
            struct IBuf {
                float u[kIG][FP], rw[kIG][KP], cn[kIG][KP];
                float reff;  // lane t: r - mu - b_i of rating gs + t
            };
            // Slot sections are whole multiples of 64 floats, zero past F and
            // K, so every lane loads straight into its register (no selects:
            // the loads of a group issue back to back).
            auto load_group = [&](IBuf& B, int gs, int cnt) {
#pragma unroll
                for (int t = 0; t < kIG; ++t) {
                    const float* d = rdata + ((gs + t) & (kRing - 1)) * RS + lane;
#pragma unroll
                    for (int x = 0; x < FP; ++x) B.u[t][x] = d[x * kWave];
#pragma unroll
                    for (int y = 0; y < KP; ++y) {
                        B.rw[t][y] = d[(FP + y) * kWave];
                        B.cn[t][y] = d[(FP + KP + y) * kWave];
                    }
                }
                B.reff = __int_as_float(rhdr[((gs + (lane < cnt ? lane : 0)) & (kRing - 1)) * 4]);
            };
            // One group: Eq. (rr) and Eq. (sgd_update) of the item side for its
            // ratings in order, the next group's inputs loaded into N when they
            // are already there, then the group's errors published.  The rates
            // of a side that is not updated are zero, so its parameters keep
            // their values exactly.
            auto run_group = [&](IBuf& B, IBuf& N, int gs) {
                const int cnt = len - gs < kIG ? len - gs : kIG;
                const int gn = gs + kIG;
                const int cntn = len - gn < kIG ? len - gn : kIG;
                bool have_next = false;
                if (gn < len && group_ready(gn, cntn)) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                    load_group(N, gn, cntn);
                    have_next = true;
                }
                float errv = 0.0f;  // lane t: error of rating gs + t
#pragma unroll
                for (int t = 0; t < kIG; ++t) {
                    if (t >= cnt) break;
                    const float reff = __builtin_bit_cast(
                        float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, B.reff), t));
                    float part = 0.0f;
#pragma unroll
                    for (int x = 0; x < FP; ++x) part += B.u[t][x] * v[x];
#pragma unroll
                    for (int y = 0; y < KP; ++y) part += B.rw[t][y] * w[y] + B.cn[t][y] * c[y];
                    const float err = reff - (bh + wave_sum(part));
                    errv = lane == t ? err : errv;
#pragma unroll
                    for (int x = 0; x < FP; ++x) v[x] = sgd_step(v[x], a.g[3], err, B.u[t][x], a.l[3]);
                    bh = sgd_step(bh, a.g[1], err, 1.0f, a.l[1]);
#pragma unroll
                    for (int y = 0; y < KP; ++y) {
                        // an explicit slot has cn == 0; padding slots stay zero either way
                        const bool rs = B.cn[t][y] == 0.0f;
                        const float wn = sgd_step(w[y], a.g[4], err, B.rw[t][y], a.l[4]);
                        const float cnn = sgd_step(c[y], a.g[5], err, B.cn[t][y], a.l[5]);
                        w[y] = rs ? wn : w[y];
                        c[y] = rs ? c[y] : cnn;
                    }
                }
                // the group's errors, for the writer wave
                if (lane < cnt) rerr[(gs + lane) & (kRing - 1)] = errv;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                if (lane == 0) __hip_atomic_store(rcount, gs + cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (gn < len && !have_next) {
                    wait_group(gn, cntn);
                    load_group(N, gn, cntn);
                }
            };
            IBuf BA, BB;
            wait_group(0, len < kIG ? len : kIG);
            load_group(BA, 0, len < kIG ? len : kIG);
            for (int gs = 0;; gs += 2 * kIG) {
                run_group(BA, BB, gs);
                if (gs + kIG >= len) break;
                run_group(BB, BA, gs + kIG);
                if (gs + 2 * kIG >= len) break;
            }
            __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int x = 0; x < FP; ++x) {
                const int f = lane + x * kWave;
                if (f < F) {
                    a.V[j * F + f] = v[x];
                }
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
        } else if (role == kHelpers + 1) {
            // ---- writer wave: the user side of each rating from the item
            // wave's errors.  It replays v_j's updates (the same sgd_step on the
            // same values) to have v_j as it was before every rating.
            __builtin_amdgcn_s_setprio(2);
            float v[FP];
#pragma unroll
            for (int x = 0; x < FP; ++x) {
                const int f = lane + x * kWave;
                v[x] = f < F ? a.V[j * F + f] : 0.0f;
            }
            bool dead = false;
            for (int gs = 0; gs < len; gs += kIG) {
                const int cnt = len - gs < kIG ? len - gs : kIG;
                int spins = 0;
                while (!dead && __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                    rcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) < gs + cnt) {
                    if (++spins > kSpinLimit) {
                        if (lane == 0) atomicOr(a.err, 4);
                        dead = true;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                // lane t: error, b_i, user and hand-over word of rating gs + t
                const int sl_l = (gs + (lane < cnt ? lane : 0)) & (kRing - 1);
                const float errv = rerr[sl_l];
                const int* hd = rhdr + sl_l * 4;
                const float bi_v = __int_as_float(hd[1]);
                const int i_v = hd[2], lw_v = hd[3];
                // the group's u rows, all loads in flight at once (slots past
                // cnt hold stale values that are never used)
                float ug[kIG][FP];
#pragma unroll
                for (int t = 0; t < kIG; ++t) {
                    const float* d = rdata + ((gs + t) & (kRing - 1)) * RS + lane;
#pragma unroll
                    for (int x = 0; x < FP; ++x) ug[t][x] = d[x * kWave];
                }
#pragma unroll
                for (int t = 0; t < kIG; ++t) {
                    if (t >= cnt) break;
                    const float err =
                        __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, errv), t));
                    const int64_t i = (int64_t)__builtin_amdgcn_readlane(i_v, t);
                    const uint32_t lw = (uint32_t)__builtin_amdgcn_readlane(lw_v, t);
                    const bool has_succ = (lw >> 31) != 0;
                    const int ws = has_succ ? (int)(lw & 0xFFFFu) : dummy;
                    // wave-uniform destinations: the mailbox row of the user's
                    // next rating in the block, else the HBM row (FP32, or BF16
                    // with round to nearest even in storage mode BF16_U); the
                    // store that must not happen goes to a sink
                    float* urow = (has_succ || UB) ? a.trash + kWave * FP : a.U + i * F;
                    uint16_t* hrow = (!has_succ && UB) ? a.U16 + i * F
                                                          : reinterpret_cast<uint16_t*>(a.trash + 3 * kWave * FP);
                    float* mrow = mb_u + ws * F;
#pragma unroll
                    for (int x = 0; x < FP; ++x) {
                        const int f = lane + x * kWave;
                        const float uo = ug[t][x];
                        const float unew = sgd_step(uo, a.g[2], err, v[x], a.l[2]);
                        if (x < FP - 1 || f < F) {  // only the last pass has lanes past F
                            mrow[f] = unew;
                            if constexpr (UB) hrow[f] = to_bf16(unew);
                            else urow[f] = unew;
                        }
                        v[x] = sgd_step(v[x], a.g[3], err, uo, a.l[3]);
                    }
                }
                // b_i to the mailbox or HBM, then the hand-over sequence numbers
                // and the done flags (lane t: rating gs + t)
                const bool live = lane < cnt;
                const bool succ = live && ((uint32_t)lw_v >> 31) != 0;
                const int ws = succ ? (lw_v & 0xFFFF) : dummy;
                const float bnew = sgd_step(bi_v, a.g[0], errv, 1.0f, a.l[0]);
                if (live) {
                    mb_b[ws] = bnew;
                    *(succ ? a.trash + 2 * kWave * FP + lane : a.bu + i_v) = bnew;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                if (live) {
                    __hip_atomic_store(&mb_seq[ws], ((lw_v >> 16) & 0x3FFF) + 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_store(&rdone[(gs + lane) & (kRing - 1)], gs + lane + 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
            __builtin_amdgcn_s_setprio(0);
        } else {
            // ---- helper wave h: ratings n = h, h + H, ... of the segment
            const int h = role - 1;
            const int mcount = h < len ? (len - h + kHelpers - 1) / kHelpers : 0;
            bool dead = false;  // after one failed wait, later waits are skipped so the kernel ends
            float bhn[KP];
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                const int k = lane + y * kWave;
                bhn[y] = k < K ? a.nbr_b0[j * K + k] : 0.0f;
            }
            // HBM loads of kHG ratings (t0.. of the current word batch); no waits
            auto hstage = [&](HStage<FP, KP>& S, uint32_t pkv, uint32_t lkv, int mb, int t0, int nbw) {
#pragma unroll
                for (int t = 0; t < kHG; ++t) {
                    const int tt = t0 + t;
                    const bool valid = tt < nbw;
                    const uint32_t pw = (uint32_t)__builtin_amdgcn_readlane((int)pkv, tt & 63);
                    const uint32_t lw = (uint32_t)__builtin_amdgcn_readlane((int)lkv, tt & 63);
                    S.pw[t] = pw;
                    S.lw[t] = lw;
                    const int64_t i = valid ? (int64_t)(pw >> 4) : 0;
                    const int64_t pos = valid ? ea + h + (int64_t)kHelpers * (mb + tt) : ea;
                    if constexpr (UB) {
#pragma unroll
                        for (int x = 0; x < FP; ++x) {
                            const int f = lane + x * kWave;
                            S.u[t][x] = from_bf16(a.U16[f < F ? i * F + f : 0]);
                        }
                    } else {
#pragma unroll
                        for (int x = 0; x < FP; ++x) {
                            const int f = lane + x * kWave;
                            S.u[t][x] = *(f < F ? a.U + i * F + f : a.trash + lane);
                        }
                    }
                    S.bi[t] = a.bu[i];
                    S.b0[t] = a.b0[i];
                    const uint8_t* nbp = a.nib + pos * a.nstride;
#pragma unroll
                    for (int y = 0; y < KP; ++y) {
                        const int byte = (lane >> 1) + y * (kWave / 2);
                        S.nb[t][y] = nbp[byte < a.nstride ? byte : 0];
                    }
                }
            };
            // user-side inputs of each staged rating into the ring, in order
            auto hprep = [&](HStage<FP, KP>& S, int mb, int t0, int nbw) {
#pragma unroll
                for (int t = 0; t < kHG; ++t) {
                    const int tt = t0 + t;
                    if (tt >= nbw) break;
                    const int n = h + kHelpers * (mb + tt);
                    const int sl = n & (kRing - 1);
                    const uint32_t pw = S.pw[t], lw = S.lw[t];
                    // the slot's previous rating, n - kRing, must be done
                    if (n >= kRing) {
                        int spins = 0;
                        while (!dead && __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                            &rdone[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) < n - kRing + 1) {
                            if (++spins > kSpinLimit) {
                                if (lane == 0) atomicOr(a.err, 4);
                                dead = true;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                    }
                    // an earlier rating of the user in this block hands its row over
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
                    float u[FP];
#pragma unroll
                    for (int x = 0; x < FP; ++x) {
                        const int f = lane + x * kWave;
                        const float mv = mb_u[f < F ? pslot * F + f : dummy * F];
                        u[x] = f < F ? (has_pred ? mv : S.u[t][x]) : 0.0f;
                    }
                    const float bi = has_pred ? mb_b[pslot] : S.bi[t];
                    const float base_i = mu + S.b0[t];
                    int code[KP];
                    int nR = 0;
#pragma unroll
                    for (int y = 0; y < KP; ++y) {
                        const int k = lane + y * kWave;
                        code[y] = k < K ? (int)((S.nb[t][y] >> ((lane & 1) * 4)) & 15u) : 0;
                        nR += __popcll(__ballot(code[y] != 0));
                    }
                    const float sR = nR > 0 ? __builtin_amdgcn_rsqf((float)nR) : 0.0f;
                    const float sN = K - nR > 0 ? __builtin_amdgcn_rsqf((float)(K - nR)) : 0.0f;
                    // u (zero past F), then rw and cn (zero past K), 64 floats a section
                    float* d = rdata + sl * RS + lane;
#pragma unroll
                    for (int x = 0; x < FP; ++x) d[x * kWave] = u[x];
#pragma unroll
                    for (int y = 0; y < KP; ++y) {
                        const int k = lane + y * kWave;
                        const float resid = (float)code[y] * inv_s - base_i - bhn[y];
                        d[(FP + y) * kWave] = code[y] ? resid * sR : 0.0f;
                        d[(FP + KP + y) * kWave] = (k < K && !code[y]) ? sN : 0.0f;
                    }
                    const float r = (float)(pw & 15u) * inv_s;
                    if (lane == 0) {
                        int* hd = rhdr + sl * 4;
                        hd[0] = __float_as_int(r - (mu + bi));
                        hd[1] = __float_as_int(bi);
                        hd[2] = (int)(pw >> 4);
                        hd[3] = (int)lw;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                    if (lane == 0) __hip_atomic_store(&rready[sl], n + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            };
            HStage<FP, KP> SA, SB;
            for (int mb = 0; mb < mcount; mb += kWave) {
                const int nbw = mcount - mb < kWave ? mcount - mb : kWave;
                uint32_t pkv = 0u, lkv = 0u;
                if (lane < nbw) {
                    const int64_t pos = ea + h + (int64_t)kHelpers * (mb + lane);
                    pkv = pk[pos];
                    lkv = link[pos];
                }
                hstage(SA, pkv, lkv, mb, 0, nbw);
                for (int t0 = 0;; t0 += 2 * kHG) {
                    hstage(SB, pkv, lkv, mb, t0 + kHG, nbw);
                    hprep(SA, mb, t0, nbw);
                    if (t0 + kHG >= nbw) break;
                    hstage(SA, pkv, lkv, mb, t0 + 2 * kHG, nbw);
                    hprep(SB, mb, t0 + kHG, nbw);
                    if (t0 + 2 * kHG >= nbw) break;
                }
            }
        }
    }

    while (true) {
        int g = 0;
        if (lane == 0) g = atomicAdd(&next_seg[member], 1);
        g = __builtin_amdgcn_readfirstlane(g);
        if (g >= nsegs) break;
        const int64_t seg = g0 + g;
        const int64_t j = a.seg_col[seg];
        const int64_t ea = a.seg_start[seg], ez = a.seg_start[seg + 1];
        if (ez - ea > 4 * kGroup) __builtin_amdgcn_s_setprio(2);

        // item state, register resident for the whole segment
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
                bhn[y] = a.nbr_b0[j * K + k];
            }
        }

        // (user, code) and hand-over words of a group: one vector load each
        auto words = [&](uint32_t& px, uint32_t& lx, int64_t gb) {
            px = lane < kGroup ? pk[gb + lane] : 0u;
            lx = lane < kGroup ? link[gb + lane] : 0u;
        };
        // wait for an earlier rating of the same user, then load the inputs
        // HBM inputs of a group, loaded a group ahead; no waits here, so a
        // rating never waits on a hand-over meant for a later one
        auto stage = [&](Stage<FP, KP>& S, uint32_t px, uint32_t lx, int64_t gb) {
#pragma unroll
            for (int sl = 0; sl < kGroup; ++sl) {
                const uint32_t pw = (uint32_t)__builtin_amdgcn_readlane((int)px, sl);
                const uint32_t lw = (uint32_t)__builtin_amdgcn_readlane((int)lx, sl);
                S.pk[sl] = pw;
                S.lk[sl] = lw;
                const int64_t i = pw >> 4;
                // lanes past F read the sink row: every load is issued by all lanes
                if constexpr (UB) {
#pragma unroll
                    for (int x = 0; x < FP; ++x) {
                        const int f = lane + x * kWave;
                        const float gv = from_bf16(a.U16[f < F ? i * F + f : 0]);
                        S.gu[sl][x] = f < F ? gv : 0.0f;
                    }
                } else {
#pragma unroll
                    for (int x = 0; x < FP; ++x) {
                        const int f = lane + x * kWave;
                        const float gv = *(f < F ? a.U + i * F + f : a.trash + lane);
                        S.gu[sl][x] = f < F ? gv : 0.0f;   // lanes past F keep u = 0 (and so v = 0)
                    }
                }
                S.gbi[sl] = a.bu[i];
                S.b0[sl] = a.b0[i];
                const uint8_t* nbp = a.nib + (gb + sl) * a.nstride;
#pragma unroll
                for (int y = 0; y < KP; ++y) {
                    const int byte = (lane >> 1) + y * (kWave / 2);
                    S.nb[sl][y] = nbp[byte < a.nstride ? byte : 0];
                }
            }
        };
        // Eq. (rr) and Eq. (sgd_update) for the ratings of one group, in order;
        // then hand the updated user rows to later ratings of the same users
        auto compute = [&](Stage<FP, KP>& S, int64_t gb) {
            // are the hand-overs of the whole group there?  lane t checks rating gb + t
            uint32_t lwl = 0u;
#pragma unroll
            for (int sl = 0; sl < kGroup; ++sl) lwl = lane == sl ? S.lk[sl] : lwl;
            const bool hpl = lane < kGroup && gb + lane < ez && ((lwl >> 30) & 1u);
            const bool okl = !hpl || __hip_atomic_load(&mb_seq[lwl & 0xFFFFu], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP) == (int)((lwl >> 16) & 0x3FFFu);
            const bool ready = __ballot(!okl) == 0ull;
            float mrow[kGroup][FP], mbv[kGroup];
            if (ready) {
                // read every handed-over row of the group at once
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
#pragma unroll
                for (int sl = 0; sl < kGroup; ++sl) {
                    const uint32_t lw = S.lk[sl];
                    const int rs = (gb + sl < ez && ((lw >> 30) & 1u)) ? (int)(lw & 0xFFFFu) : dummy;
#pragma unroll
                    for (int x = 0; x < FP; ++x) {
                        const int f = lane + x * kWave;
                        mrow[sl][x] = mb_u[f < F ? rs * F + f : dummy * F];
                    }
                    mbv[sl] = mb_b[rs];
                }
            }
#pragma unroll
            for (int sl = 0; sl < kGroup; ++sl) {
                const bool valid = gb + sl < ez;
                const uint32_t lw = S.lk[sl];
                const bool has_pred = valid && ((lw >> 30) & 1u);
                const bool has_succ = valid && (lw >> 31);
                const int slot = (int)(lw & 0xFFFFu);
                const int64_t i = S.pk[sl] >> 4;
                const float r = (float)(S.pk[sl] & 15u) * inv_s;
                const float base_i = mu + S.b0[sl];
                int code[KP];
                float resid[KP];
                int nR = 0;
#pragma unroll
                for (int y = 0; y < KP; ++y) {
                    const int k = lane + y * kWave;
                    code[y] = k < K ? (int)((S.nb[sl][y] >> ((lane & 1) * 4)) & 15u) : 0;
                    resid[y] = (float)code[y] * inv_s - base_i - bhn[y];
                    nR += __popcll(__ballot(code[y] != 0));
                }
                const float sR = nR > 0 ? __builtin_amdgcn_rsqf((float)nR) : 0.0f;
                const float sN = K - nR > 0 ? __builtin_amdgcn_rsqf((float)(K - nR)) : 0.0f;
                // an earlier rating of the user in this block hands its row over
                if (has_pred && !ready) {
                    const int want = (int)((lw >> 16) & 0x3FFFu);
                    int spins = 0;
                    while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(&mb_seq[slot], __ATOMIC_RELAXED,
                                                                            __HIP_MEMORY_SCOPE_WORKGROUP)) != want) {
                        if (++spins > kSpinLimit) {
                            if (lane == 0) atomicOr(a.err, 2);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
#pragma unroll
                    for (int x = 0; x < FP; ++x) {
                        const int f = lane + x * kWave;
                        mrow[sl][x] = mb_u[f < F ? slot * F + f : dummy * F];
                    }
                    mbv[sl] = mb_b[slot];
                }
                float u[FP];
#pragma unroll
                for (int x = 0; x < FP; ++x) {
                    const int f = lane + x * kWave;
                    u[x] = has_pred ? (f < F ? mrow[sl][x] : 0.0f) : S.gu[sl][x];
                }
                const float bi = has_pred ? mbv[sl] : S.gbi[sl];
                // u.v + |R^K|^-1/2 sum resid*w + |N^K|^-1/2 sum c: one reduction
                float part = 0.0f;
#pragma unroll
                for (int x = 0; x < FP; ++x) part += u[x] * v[x];
#pragma unroll
                for (int y = 0; y < KP; ++y) {
                    const float t = code[y] ? resid[y] * w[y] * sR : c[y] * sN;
                    part += lane + y * kWave < K ? t : 0.0f;
                }
                const float err = r - (mu + bi + bh + wave_sum(part));
                // all right-hand sides from the pre-step state.  The last rating
                // of a user in the block writes HBM; earlier ones only the
                // mailbox.  Stores that must not happen go to sinks instead, so
                // every lane issues the same stores without branches.
                const bool to_hbm = valid && !has_succ;
                const int ws = has_succ ? slot : dummy;
                const float bnew = bi + a.g[0] * (err - a.l[0] * bi);
                float* bsink = a.trash + 2 * kWave * FP;
                *((lane == 0 && to_hbm) ? a.bu + i : bsink + lane) = bnew;
                mb_b[lane == 0 ? ws : dummy] = bnew;
                const float bh_new = bh + a.g[1] * (err - a.l[1] * bh);
                bh = valid ? bh_new : bh;
#pragma unroll
                for (int x = 0; x < FP; ++x) {
                    const int f = lane + x * kWave;
                    const float unew = u[x] + a.g[2] * (err * v[x] - a.l[2] * u[x]);
                    if constexpr (UB) {
                        uint16_t* hs = reinterpret_cast<uint16_t*>(a.trash + 3 * kWave * FP);
                        *((to_hbm && f < F) ? a.U16 + i * F + f : hs + f) = to_bf16(unew);
                    } else {
                        *((to_hbm && f < F) ? a.U + i * F + f : a.trash + kWave * FP + f) = unew;
                    }
                    mb_u[f < F ? ws * F + f : dummy * F] = unew;
                    const float vn = v[x] + a.g[3] * (err * u[x] - a.l[3] * v[x]);
                    v[x] = valid ? vn : v[x];
                }
#pragma unroll
                for (int y = 0; y < KP; ++y) {
                    const bool in_k = lane + y * kWave < K;
                    const float wn = w[y] + a.g[4] * (sR * err * resid[y] - a.l[4] * w[y]);
                    const float cn = c[y] + a.g[5] * (sN * err - a.l[5] * c[y]);
                    w[y] = (valid && in_k && code[y]) ? wn : w[y];
                    c[y] = (valid && in_k && !code[y]) ? cn : c[y];
                }
            }
            // the mailbox rows are written: publish their sequence numbers
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
            if (lane == 0) {
#pragma unroll
                for (int sl = 0; sl < kGroup; ++sl) {
                    const uint32_t lw = S.lk[sl];
                    const bool has_succ = gb + sl < ez && (lw >> 31);
                    const int ws = has_succ ? (int)(lw & 0xFFFFu) : dummy;
                    __hip_atomic_store(&mb_seq[ws], (int)((lw >> 16) & 0x3FFFu) + 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        };

        Stage<FP, KP> SA, SB;
        uint32_t pkA, lkA, pkB, lkB;
        if (ez - ea <= kGroup) {
            words(pkA, lkA, ea);
            stage(SA, pkA, lkA, ea);
            compute(SA, ea);
        } else {
            // inputs of group g+1 in flight while group g computes
            words(pkA, lkA, ea);
            words(pkB, lkB, ea + kGroup);
            stage(SA, pkA, lkA, ea);
            words(pkA, lkA, ea + 2 * kGroup);
            for (int64_t gb = ea;; gb += 2 * kGroup) {
                stage(SB, pkB, lkB, gb + kGroup);
                words(pkB, lkB, gb + 3 * kGroup);
                compute(SA, gb);
                if (gb + kGroup >= ez) break;
                stage(SA, pkA, lkA, gb + 2 * kGroup);
                words(pkA, lkA, gb + 4 * kGroup);
                compute(SB, gb + kGroup);
                if (gb + 2 * kGroup >= ez) break;
            }
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int x = 0; x < FP; ++x) {
            const int f = lane + x * kWave;
            if (f < F) {
                a.V[j * F + f] = v[x];
            }
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

// Lane passes over F features and K neighbour slots, as the kernel
// instantiations take them (K = 0 runs with one pass of zero slots).
static int fp_of(int F) { return (F + kWave - 1) / kWave; }
static int kp_of(int K) { return K > kWave ? 2 : 1; }

// Dynamic LDS of one block: the mailbox (slots + 1 rows of F floats, b_i and
// a sequence word) and the gang rings.
static size_t sgd_lds_bytes(const SgdArgs& args)
{
    const size_t gs = (size_t)kRing * (args.ring_rs + 7) + 4;
    const size_t one = ((size_t)args.ring_off + (size_t)args.max_gangs * gs) * sizeof(float);
    const size_t team = (size_t)args.team * (size_t)args.team_floats * sizeof(float);
    return one > team ? one : team;
}

template <int FP, int KP, bool UB>
static int launch_sgd(const SgdArgs& args, const uint32_t* pk, const uint32_t* link, hipStream_t s)
{
    const size_t lds = sgd_lds_bytes(args);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sgd_stratum<FP, KP, UB>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(k_sgd_stratum)");
    }
    hipLaunchKernelGGL((k_sgd_stratum<FP, KP, UB>), dim3((unsigned)args.grid), dim3(kSgdWaves * kWave), lds, s,
                       args, pk, link);
    LSHMF_LAUNCHED("k_sgd_stratum");
    return LSHMF_OK;
}

template <int FP>
static int launch_sgd_k(const SgdArgs& args, const uint32_t* pk, const uint32_t* link, hipStream_t s)
{
    // storage mode BF16_U has its own instantiation: the FP32 kernels stay as they are
    if (args.U16) return args.K <= kWave ? launch_sgd<FP, 1, true>(args, pk, link, s) : launch_sgd<FP, 2, true>(args, pk, link, s);
    return args.K <= kWave ? launch_sgd<FP, 1, false>(args, pk, link, s) : launch_sgd<FP, 2, false>(args, pk, link, s);
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
    a.blk_run = st.blk_run;
    a.seg_col = st.seg_col;
    a.seg_start = st.seg_start;
    a.nbr_b0 = c->nbr_b0;
    a.b0 = c->t.b0;
    a.mu = c->t.mu;
    a.U = c->t.U;
    a.U16 = d.storage == LSHMF_BF16_U ? c->t.U16 : nullptr;
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
    a.upd = upd;
    a.inv_s = 1.0f / (float)d.rscale;
    // gangs only where their rings fit beside the mailbox
    a.ring_off = (int)(((st.max_block_slots + 1) * (d.F + 2) + 3) & ~3LL);
    a.ring_rs = kWave * (fp_of(d.F) + 2 * kp_of(d.K));
    a.max_gangs = kMaxGangs;
    a.team = 1;
    a.team_slots = kLightNnz / 2;
    a.team_floats = (int)(((int64_t)(a.team_slots + 1) * (d.F + 2) + 3) & ~3LL);
    while (a.max_gangs > 0 && sgd_lds_bytes(a) > (size_t)kMaxLdsBytes) --a.max_gangs;
    a.gang_min = a.max_gangs >= 2 ? kGangMin2 : kGangMin1;
    // light blocks in teams where their mailboxes fit in the block's LDS
    for (int t = kTeam; t > 1 && a.team == 1; t /= 2) {
        a.team = t;
        if (sgd_lds_bytes(a) > (size_t)kMaxLdsBytes) a.team = 1;
    }
    // Eq. (learn_rate): gamma_t = alpha / (1 + beta * t^1.5)
    const double den = 1.0 + (double)hp->beta * std::pow((double)epoch, 1.5);
    for (int x = 0; x < 6; ++x) {
        a.g[x] = (float)((double)hp->alpha[x] / den);
        a.l[x] = hp->lambda[x];
    }
    // plain MF (Alg. CUSGD++'s model, rhat = u . v): no biases to learn; with
    // zero rates the bias updates leave b and bh exactly at their zero start
    if (d.model == LSHMF_PLAIN_MF) a.g[0] = a.g[1] = 0.0f;
    // a side that is not updated gets zero rates: x + 0 * (...) == x exactly
    if (!(upd & 1)) a.g[0] = a.g[2] = 0.0f;
    if (!(upd & 2)) a.g[1] = a.g[3] = a.g[4] = a.g[5] = 0.0f;
    const int fp = (d.F + kWave - 1) / kWave;
    const int P = c->P;
    for (int stratum = 0; stratum < P; ++stratum) {
        // workgroups: the heavy blocks one each, the other non-empty blocks in
        // teams; a stratum without ratings is not launched
        const int nh = st.hcounts[stratum], ne = st.hcounts[P + stratum];
        if (ne == 0) continue;
        a.s = stratum;
        a.nh = nh;
        a.grid = a.team > 1 ? nh + (ne - nh + a.team - 1) / a.team : ne;
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
