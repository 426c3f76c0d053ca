// Serving loop: replays a log of online updates (Sec. 4.3) and rating queries
// (Eq. rr) in arrival order with continuous batching of queries, admission
// against the preallocated capacities, and uploads / downloads on a copy
// stream beside the compute stream.  Host code only; every step of the work
// is one of the library's GPU entry points.
#include <chrono>
#include <deque>
#include <thread>

#include "common.hpp"

namespace lshmf {

int run_online(lshmf_ctx* c, const int32_t* u, const int32_t* it, const uint8_t* rc, int64_t n, int32_t M_new,
               int32_t N_new, const void* R, uint64_t seed_fill, const lshmf_hparams* hp, int epoch,
               int passes, uint32_t flags, hipStream_t s, bool refresh);

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct StageLayout {
    size_t upd_u, upd_i, upd_rc, q[2], bytes;
    size_t q_qi, q_out;  // offsets inside a query slot
};

StageLayout stage_layout(const lshmf_ctx* c, int64_t mqb)
{
    StageLayout L;
    const size_t bc = (size_t)c->d.batch_cap;
    size_t off = 0;
    L.upd_u = off;
    off += align256(bc * 4);
    L.upd_i = off;
    off += align256(bc * 4);
    L.upd_rc = off;
    off += align256(bc);
    L.q_qi = align256((size_t)mqb * 4);
    L.q_out = 2 * L.q_qi;
    const size_t qslot = 3 * L.q_qi;
    for (int k = 0; k < 2; ++k) {
        L.q[k] = off;
        off += qslot;
    }
    L.bytes = off;
    return L;
}

double seconds_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// One launched piece of work: requests [first, last] finish with ev[0]; its
// events go back to the pool only when it retires.
struct Work {
    int64_t first, last;
    hipEvent_t ev[3];
    int nev;
    int qslot;  // query staging slot, -1 for an update
};

}  // namespace
}  // namespace lshmf

using namespace lshmf;

extern "C" {

int lshmf_serve_stage_bytes(const lshmf_ctx* ctx, int64_t max_query_batch, size_t* bytes)
{
    if (!ctx || !bytes || max_query_batch < 1) {
        set_error("lshmf_serve_stage_bytes: bad arguments");
        return LSHMF_EINVAL;
    }
    *bytes = stage_layout(ctx, max_query_batch).bytes;
    return LSHMF_OK;
}

int lshmf_serve(lshmf_ctx* ctx, const lshmf_serve_io* io, lshmf_stream_t compute_, lshmf_stream_t copy_)
{
    if (!ctx || !ctx->neighbours) {
        set_error("lshmf_serve: neighbours not built");
        return LSHMF_ESTATE;
    }
    if (!io || !io->req || io->n_req < 0 || !io->h_start || !io->h_done || !io->h_status || !io->d_stage ||
        io->max_query_batch < 1 || !compute_ || !copy_ || compute_ == copy_) {
        set_error("lshmf_serve: bad arguments (two distinct streams, staging and outputs are required)");
        return LSHMF_EINVAL;
    }
    const StageLayout L = stage_layout(ctx, io->max_query_batch);
    if (io->stage_bytes < L.bytes || (reinterpret_cast<uintptr_t>(io->d_stage) & 255)) {
        set_error("lshmf_serve: staging of %zu bytes (256-byte aligned), need %zu", io->stage_bytes, L.bytes);
        return LSHMF_ECAPACITY;
    }
    const lshmf_request* R = io->req;
    for (int64_t r = 0; r < io->n_req; ++r) {
        const bool bad_kind = R[r].kind != LSHMF_REQ_UPDATE && R[r].kind != LSHMF_REQ_QUERY;
        const bool no_payload = R[r].n > 0 && (R[r].kind == LSHMF_REQ_UPDATE ? (!io->h_u || !io->h_i || !io->h_rc)
                                                                             : (!io->h_qu || !io->h_qi || !io->h_pred));
        if (bad_kind || R[r].n < 0 || R[r].offset < 0 || no_payload || (r > 0 && R[r].arrival < R[r - 1].arrival)) {
            set_error("lshmf_serve: request %lld is malformed or arrives before its predecessor", (long long)r);
            return LSHMF_EINVAL;
        }
    }
    const hipStream_t cs = reinterpret_cast<hipStream_t>(compute_);
    const hipStream_t ps = reinterpret_cast<hipStream_t>(copy_);
    char* stage = static_cast<char*>(io->d_stage);
    int32_t* su = reinterpret_cast<int32_t*>(stage + L.upd_u);
    int32_t* si = reinterpret_cast<int32_t*>(stage + L.upd_i);
    uint8_t* src = reinterpret_cast<uint8_t*>(stage + L.upd_rc);
    const int64_t F = ctx->d.F;

    // In storage mode BF16, queries read only the BF16 copies and bias
    // snapshots, which an update rewrites in its last step: queries then run
    // on a stream of their own beside the next update's hashing, neighbour
    // and SGD phases, and only that last step waits for them.  Other modes
    // read live tables, so queries and updates share the compute stream.
    const bool overlap = ctx->d.storage == LSHMF_BF16;
    hipStream_t qs = cs;
    constexpr int kEvents = 16;
    // events: a pool recycled as work retires, plus three markers that are
    // recorded again each time (a wait refers to the latest record)
    hipEvent_t pool[kEvents] = {};
    hipEvent_t mark[3] = {};
    hipError_t e0 = hipSuccess;
    for (int k = 0; k < kEvents && e0 == hipSuccess; ++k) {
        e0 = hipEventCreateWithFlags(&pool[k], hipEventDisableTiming);
        if (e0 != hipSuccess) pool[k] = nullptr;
    }
    for (int k = 0; k < 3 && e0 == hipSuccess; ++k) {
        e0 = hipEventCreateWithFlags(&mark[k], hipEventDisableTiming);
        if (e0 != hipSuccess) mark[k] = nullptr;
    }
    if (e0 == hipSuccess && overlap) {
        e0 = hipStreamCreateWithFlags(&qs, hipStreamNonBlocking);
        if (e0 != hipSuccess) qs = cs;
    }
    hipEvent_t visible = mark[0], qdone = mark[1], upd_fin = mark[2];
    auto release_all = [&]() {
        for (hipEvent_t x : pool)
            if (x) (void)hipEventDestroy(x);
        for (hipEvent_t x : mark)
            if (x) (void)hipEventDestroy(x);
        if (qs != cs) (void)hipStreamDestroy(qs);
    };
    if (e0 != hipSuccess) {
        release_all();
        return hip_fail(e0, "lshmf_serve set-up");
    }
    bool have_visible = false, have_qdone = false, have_upd = false;

    std::deque<hipEvent_t> free_ev(pool, pool + kEvents);
    std::deque<Work> inflight;
    bool qbusy[2] = {false, false};
    int status = LSHMF_OK;
    int64_t next = 0, retired = 0;
    const auto t0 = std::chrono::steady_clock::now();

    auto take_event = [&]() {
        hipEvent_t x = free_ev.front();
        free_ev.pop_front();
        return x;
    };
    auto refuse = [&](int64_t r, int st) {
        const double t = seconds_since(t0);
        io->h_start[r] = io->h_done[r] = t;
        io->h_status[r] = st;
        ++retired;
    };

    while (retired < io->n_req && status == LSHMF_OK) {
        bool progress = false;
        // retire finished work, whichever finished (queries may overtake an update)
        for (auto it = inflight.begin(); it != inflight.end();) {
            const hipError_t e = hipEventQuery(it->ev[0]);
            if (e == hipErrorNotReady) {
                ++it;
                continue;
            }
            if (e != hipSuccess) {
                status = hip_fail(e, "hipEventQuery");
                break;
            }
            const double t = seconds_since(t0);
            for (int64_t r = it->first; r <= it->last; ++r) io->h_done[r] = t;
            retired += it->last - it->first + 1;
            if (it->qslot >= 0) qbusy[it->qslot] = false;
            for (int k = 0; k < it->nev; ++k) free_ev.push_back(it->ev[k]);
            it = inflight.erase(it);
            progress = true;
        }
        if (status != LSHMF_OK) break;

        if (next < io->n_req && inflight.size() < 4 && free_ev.size() >= 3 && R[next].arrival <= seconds_since(t0)) {
            const lshmf_request& q = R[next];
            if (q.kind == LSHMF_REQ_UPDATE) {
                if (q.n > ctx->d.batch_cap || ctx->nnz + q.n > ctx->d.nnz_cap || q.M_new > ctx->d.M_cap ||
                    q.N_new > ctx->d.N_cap) {
                    refuse(next++, LSHMF_ECAPACITY);
                    continue;
                }
                if (q.M_new < ctx->M || q.N_new < ctx->N) {
                    refuse(next++, LSHMF_EINVAL);
                    continue;
                }
                // The update staging is rewritten only once the previous update's
                // kernels, the last readers of it, are done.
                hipEvent_t up = take_event(), fin = take_event();
                hipError_t e = hipSuccess;
                if (have_upd) e = hipStreamWaitEvent(ps, upd_fin, 0);
                if (e == hipSuccess && q.n > 0)
                    e = hipMemcpyAsync(su, io->h_u + q.offset, 4 * q.n, hipMemcpyHostToDevice, ps);
                if (e == hipSuccess && q.n > 0)
                    e = hipMemcpyAsync(si, io->h_i + q.offset, 4 * q.n, hipMemcpyHostToDevice, ps);
                if (e == hipSuccess && q.n > 0) e = hipMemcpyAsync(src, io->h_rc + q.offset, q.n, hipMemcpyHostToDevice, ps);
                if (e == hipSuccess) e = hipEventRecord(up, ps);
                if (e == hipSuccess) e = hipStreamWaitEvent(cs, up, 0);
                // initial factor rows of the new ids (Alg. "Online Learning" takes them as input)
                if (e == hipSuccess && q.M_new > ctx->M) {
                    if (ctx->d.storage == LSHMF_BF16_U) {  // the user rows live in BF16 only
                        if (to_bf16_rows(io->d_U0 + ctx->M * F, ctx->t.U16 + ctx->M * F, F * (q.M_new - ctx->M), cs) !=
                            LSHMF_OK)
                            e = hipErrorLaunchFailure;
                    } else {
                        e = hipMemcpyAsync(ctx->t.U + ctx->M * F, io->d_U0 + ctx->M * F,
                                           sizeof(float) * F * (q.M_new - ctx->M), hipMemcpyDeviceToDevice, cs);
                    }
                }
                if (e == hipSuccess && q.N_new > ctx->N)
                    e = hipMemcpyAsync(ctx->t.V + ctx->N * F, io->d_V0 + ctx->N * F,
                                       sizeof(float) * F * (q.N_new - ctx->N), hipMemcpyDeviceToDevice, cs);
                if (e != hipSuccess) {
                    free_ev.push_back(up);
                    free_ev.push_back(fin);
                    status = hip_fail(e, "lshmf_serve update upload");
                    break;
                }
                io->h_start[next] = seconds_since(t0);
                const int32_t M_old = ctx->M, N_old = ctx->N;
                const int st = run_online(ctx, su, si, src, q.n, q.M_new, q.N_new, io->d_rand, io->seed_fill, &io->hp,
                                          io->epoch, io->passes, 0u, cs, !overlap);
                if (st == LSHMF_EINVAL || st == LSHMF_ECAPACITY) {  // refused before anything changed
                    io->h_done[next] = seconds_since(t0);
                    io->h_status[next] = st;
                    ++retired;
                    ++next;
                    e = hipStreamSynchronize(ps);  // the upload is done before its events are reused
                    free_ev.push_back(up);
                    free_ev.push_back(fin);
                    if (e != hipSuccess) status = hip_fail(e, "hipStreamSynchronize(copy)");
                    continue;
                }
                if (st != LSHMF_OK) {
                    status = st;
                    break;
                }
                if (overlap) {
                    // the copies change only after the queries that came before this update
                    if (have_qdone) e = hipStreamWaitEvent(cs, qdone, 0);
                    int st2 = e == hipSuccess ? refresh_after_online(ctx, M_old, N_old, 0u, cs) : LSHMF_OK;
                    if (e == hipSuccess && st2 == LSHMF_OK) e = hipEventRecord(visible, cs);
                    if (st2 != LSHMF_OK) {
                        status = st2;
                        break;
                    }
                    have_visible = true;
                }
                if (e == hipSuccess) e = hipEventRecord(fin, cs);
                if (e == hipSuccess) e = hipEventRecord(upd_fin, cs);
                if (e != hipSuccess) {
                    status = hip_fail(e, "hipEventRecord");
                    break;
                }
                have_upd = true;
                io->h_status[next] = LSHMF_OK;
                inflight.push_back(Work{next, next, {fin, up}, 2, -1});
                ++next;
                progress = true;
            } else {
                if (q.n > io->max_query_batch) {
                    refuse(next++, LSHMF_ECAPACITY);
                    continue;
                }
                const int slot = qbusy[0] ? 1 : 0;
                if (qbusy[slot]) goto idle;  // both query slots in flight
                {
                    // merge the queries that have arrived, up to the batch limit
                    const double now = seconds_since(t0);
                    int64_t last = next, total = q.n;
                    while (last + 1 < io->n_req && R[last + 1].kind == LSHMF_REQ_QUERY && R[last + 1].arrival <= now &&
                           total + R[last + 1].n <= io->max_query_batch) {
                        ++last;
                        total += R[last].n;
                    }
                    char* base = stage + L.q[slot];
                    int32_t* qu = reinterpret_cast<int32_t*>(base);
                    int32_t* qi = reinterpret_cast<int32_t*>(base + L.q_qi);
                    float* out = reinterpret_cast<float*>(base + L.q_out);
                    hipEvent_t up = take_event(), ready = take_event(), fin = take_event();
                    hipError_t e = hipSuccess;
                    int64_t at = 0;
                    for (int64_t r = next; r <= last && e == hipSuccess; ++r) {
                        if (R[r].n == 0) continue;
                        e = hipMemcpyAsync(qu + at, io->h_qu + R[r].offset, 4 * R[r].n, hipMemcpyHostToDevice, ps);
                        if (e == hipSuccess)
                            e = hipMemcpyAsync(qi + at, io->h_qi + R[r].offset, 4 * R[r].n, hipMemcpyHostToDevice, ps);
                        at += R[r].n;
                    }
                    if (e == hipSuccess) e = hipEventRecord(up, ps);
                    if (e == hipSuccess) e = hipStreamWaitEvent(qs, up, 0);
                    // these queries see every update that arrived before them
                    if (e == hipSuccess && overlap && have_visible) e = hipStreamWaitEvent(qs, visible, 0);
                    if (e != hipSuccess) {
                        for (hipEvent_t x : {up, ready, fin}) free_ev.push_back(x);
                        status = hip_fail(e, "lshmf_serve query upload");
                        break;
                    }
                    const double ts = seconds_since(t0);
                    for (int64_t r = next; r <= last; ++r) {
                        io->h_start[r] = ts;
                        io->h_status[r] = LSHMF_OK;
                    }
                    const int st = predict(ctx, qu, qi, total, out, reinterpret_cast<lshmf_stream_t>(qs));
                    if (st != LSHMF_OK) {
                        for (hipEvent_t x : {up, ready, fin}) free_ev.push_back(x);
                        status = st;
                        break;
                    }
                    e = hipEventRecord(ready, qs);
                    if (e == hipSuccess && overlap) {
                        e = hipEventRecord(qdone, qs);
                        have_qdone = true;
                    }
                    if (e == hipSuccess) e = hipStreamWaitEvent(ps, ready, 0);
                    at = 0;
                    for (int64_t r = next; r <= last && e == hipSuccess; ++r) {
                        if (R[r].n > 0)
                            e = hipMemcpyAsync(io->h_pred + R[r].offset, out + at, 4 * R[r].n, hipMemcpyDeviceToHost,
                                               ps);
                        at += R[r].n;
                    }
                    if (e == hipSuccess) e = hipEventRecord(fin, ps);
                    if (e != hipSuccess) {
                        for (hipEvent_t x : {up, ready, fin}) free_ev.push_back(x);
                        status = hip_fail(e, "lshmf_serve answer download");
                        break;
                    }
                    qbusy[slot] = true;
                    inflight.push_back(Work{next, last, {fin, up, ready}, 3, slot});
                    next = last + 1;
                    progress = true;
                }
            }
        }
    idle:
        if (!progress) std::this_thread::yield();
    }
    // drain whatever is still queued, then release the events and the query stream
    hipError_t e1 = hipStreamSynchronize(cs);
    hipError_t e2 = hipStreamSynchronize(ps);
    hipError_t e3 = qs != cs ? hipStreamSynchronize(qs) : hipSuccess;
    release_all();
    if (status == LSHMF_OK && e1 != hipSuccess) status = hip_fail(e1, "hipStreamSynchronize(compute)");
    if (status == LSHMF_OK && e2 != hipSuccess) status = hip_fail(e2, "hipStreamSynchronize(copy)");
    if (status == LSHMF_OK && e3 != hipSuccess) status = hip_fail(e3, "hipStreamSynchronize(queries)");
    if (status == LSHMF_OK) status = sync_status(ctx, cs);  // an SGD wait that gave up
    return status;
}

}  // extern "C"
