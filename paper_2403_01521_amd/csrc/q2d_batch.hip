// Replica batches: R independent systems (own box, own particle count, the
// same alpha and SOE table) advanced by one random-batch step together.
//
// Every kernel family of the single-system step runs once for all replicas:
// the sort orders particles by (replica, z) and lays each replica out in
// whole segments of S particles (the tail padded with zero charges at the
// replica's top height), so a segment belongs to one replica; the kernels
// look the replica up from the segment (its modes, coefficients, 2 pi / A,
// j = i constant), and no carry crosses from one replica to the next.  Each
// replica samples its own P modes (Sec. 4.1, App. G) with its own Philox key.
//
// A step can be captured in a hipGraph whose sampler reads the step number
// from device memory and whose last node increments it, so replays advance
// the random batch like successive calls.  The launch shapes (segment
// length, sweep work-group split, aggregate chunks per wave) are tuned by
// timing candidates on the caller's data.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "q2d_internal.h"

using namespace q2d;

namespace {

constexpr double PI = 3.14159265358979323846;

__global__ void k_set_u64(uint64_t *a, uint64_t v) { a[0] = v; }
__global__ void k_inc_u64(uint64_t *a) { a[0] += 1; }

__global__ void k_batch_modes_out(const int32_t *modes, int R, int P, int p_pad, int32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)R * P) return;
    const int r = (int)(i / P), m = (int)(i % P);
    out[2 * i] = modes[(int64_t)r * 2 * p_pad + m];
    out[2 * i + 1] = modes[(int64_t)r * 2 * p_pad + p_pad + m];
}

bool valid_S(int S) { return S >= WAVE && S <= 512 && S % WAVE == 0; }

// launch shapes of a batch step (segment length, sweep split, aggregate
// chunks per wave; see Plan::cfg_split / cfg_cpw)
struct Config {
    int S, split, cpw;
};

bool valid_config(int S, int split, int cpw) {
    return valid_S(S) && (split == 1 || split == 2) && (cpw == 1 || cpw == 2 || cpw == 4);
}

// shapes a tune has chosen, per process
struct TuneKey {
    int device, R;
    int64_t ntot;
    int P, M, fp32;
    bool operator==(const TuneKey &o) const {
        return device == o.device && R == o.R && ntot == o.ntot && P == o.P && M == o.M &&
               fp32 == o.fp32;
    }
};
std::mutex tune_mu;
std::vector<std::pair<TuneKey, Config>> tune_cache;

bool tune_cache_get(const TuneKey &k, Config &c) {
    std::lock_guard<std::mutex> lock(tune_mu);
    for (const auto &e : tune_cache)
        if (e.first == k) {
            c = e.second;
            return true;
        }
    return false;
}

void tune_cache_put(const TuneKey &k, const Config &c) {
    std::lock_guard<std::mutex> lock(tune_mu);
    for (auto &e : tune_cache)
        if (e.first == k) {
            e.second = c;
            return;
        }
    tune_cache.push_back({k, c});
}

// padded offsets and the segment -> replica table for segment length S
q2d_status layout(Plan *p, int S) {
    const int R = p->R;
    p->h_poff.assign(R + 1, 0);
    std::vector<int32_t> seg;
    for (int r = 0; r < R; ++r) {
        const int64_t ns = (p->h_n[r] + S - 1) / S;
        p->h_poff[r + 1] = p->h_poff[r] + ns * S;
        for (int64_t k = 0; k < ns; ++k) seg.push_back(r);
    }
    p->Npad = p->h_poff[R];
    p->S_batch = S;
    if (p->Npad > ((int64_t)1 << 31) - 1) return Q2D_ECAPACITY;
    q2d_status st;
    if ((st = ensure(p, p->rep_poff, (size_t)(R + 1) * sizeof(int64_t))) != Q2D_OK) return st;
    if ((st = ensure(p, p->seg_rep, std::max<size_t>(seg.size(), 1) * sizeof(int32_t))) != Q2D_OK)
        return st;
    if (hipMemcpyAsync(p->rep_poff.p, p->h_poff.data(), (R + 1) * sizeof(int64_t),
                       hipMemcpyHostToDevice, p->stream) != hipSuccess)
        return Q2D_EDEVICE;
    if (!seg.empty() && hipMemcpyAsync(p->seg_rep.p, seg.data(), seg.size() * sizeof(int32_t),
                                       hipMemcpyHostToDevice, p->stream) != hipSuccess)
        return Q2D_EDEVICE;
    // the captured step (if any) belongs to the old layout
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    return hipStreamSynchronize(p->stream) == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

Config current_config(const Plan *p) {
    return Config{p->S_batch, p->cfg_split ? p->cfg_split : 1, p->cfg_cpw ? p->cfg_cpw : 2};
}

// A new shape: a new layout if S changes; any change drops a captured step
// (its kernels were recorded with the old shapes)
q2d_status apply_config(Plan *p, const Config &c) {
    const Config cur = current_config(p);
    p->cfg_split = c.split;
    p->cfg_cpw = c.cpw;
    if (c.S != cur.S || !p->h_poff.size()) return layout(p, c.S);
    if (c.split != cur.split || c.cpw != cur.cpw) {
        if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->graph_exec = nullptr;
        p->graph = nullptr;
    }
    return Q2D_OK;
}

// One step on p->stream (and the internal stream): sampling || sort, then the
// k != 0 passes || the k = 0 term, then the epilogue.
q2d_status batch_step(Plan *p, const void *pos, const void *q, int P, uint64_t seed,
                      uint64_t step, const uint64_t *step_dev, void *phi, void *F, double *E,
                      int32_t *modes_out) {
    q2d_status st;
    const int p_pad = ((P + WAVE - 1) / WAVE) * WAVE;
    tstart(p, 4);
    if (hipEventRecord(p->ev_fork, p->stream) != hipSuccess ||
        hipStreamWaitEvent(p->side, p->ev_fork, 0) != hipSuccess)
        return Q2D_EDEVICE;
    {
        SideScope side(p);
        if ((st = sample_modes_batch(p, P, seed, step, step_dev)) != Q2D_OK) return st;
        if (modes_out) {
            const int64_t n = (int64_t)p->R * P;
            k_batch_modes_out<<<(int)((n + 255) / 256), 256, 0, p->stream>>>(
                (const int32_t *)p->rb_modes.p, p->R, P, p_pad, modes_out);
        }
    }
    if (hipEventRecord(p->ev_modes, p->side) != hipSuccess) return Q2D_EDEVICE;
    int nch = 0;
    if ((st = sort_and_stage_batch(p, pos, q)) != Q2D_OK) return st;
    if (p->Npad > 0 && (st = k0_side(p, p->Npad)) != Q2D_OK) return st;
    if (hipStreamWaitEvent(p->stream, p->ev_modes, 0) != hipSuccess) return Q2D_EDEVICE;
    if (p->Npad > 0) {
        if ((st = kmodes_run(p, p->Npad, (const int32_t *)p->rb_modes.p, p->rb_coef.p, p_pad, 0, P,
                             &nch)) != Q2D_OK)
            return st;
        if (hipStreamWaitEvent(p->stream, p->ev_k0, 0) != hipSuccess) return Q2D_EDEVICE;
    }
    st = epilogue_batch(p, nch, phi, F, E);
    tstop(p, 4);
    return st;
}

q2d_status check_step_args(q2d_batch_t b, const void *pos, const void *q, int32_t P) {
    if (!b) return Q2D_EINVAL;
    if (b->Ntot > 0 && (!pos || !q)) return Q2D_EINVAL;
    if (P < 1) return Q2D_EINVAL;
    if (P > b->opts.p_max) return Q2D_ECAPACITY;
    if (hipSetDevice(b->device) != hipSuccess) return Q2D_EDEVICE;
    return Q2D_OK;
}

}  // namespace

extern "C" {

q2d_status q2d_batch_create(int32_t R, const double *boxes, const int64_t *n, double alpha,
                            int32_t M, const double *w, const double *s, const q2d_opts *opts,
                            void *stream, q2d_batch_t *out) {
    if (!out) return Q2D_EINVAL;
    *out = nullptr;
    if (R < 1 || R > 65536 || !boxes || !n || !opts) return Q2D_EINVAL;
    if (opts->p_max < 1) return Q2D_EINVAL;
    if (opts->sampler != Q2D_SAMPLER_METROPOLIS) return Q2D_EUNSUPPORTED;
    int64_t Ntot = 0;
    for (int r = 0; r < R; ++r) {
        const double Lx = boxes[3 * r], Ly = boxes[3 * r + 1], Lz = boxes[3 * r + 2];
        if (!(Lx > 0 && Ly > 0 && Lz > 0) || !std::isfinite(Lx) || !std::isfinite(Ly) ||
            !std::isfinite(Lz) || n[r] < 0)
            return Q2D_EINVAL;
        Ntot += n[r];
        if (Ntot > ((int64_t)1 << 31) - 1) return Q2D_ECAPACITY;
    }
    q2d_batch *p = new (std::nothrow) q2d_batch();
    if (!p) return Q2D_ENOMEM;
    q2d_opts o = *opts;
    o.n_max = std::max<int64_t>(Ntot, 1);
    q2d_status st = plan_init(p, boxes[0], boxes[1], boxes[2], alpha, 0.0, 0.0, M, w, s, &o, stream);
    if (st == Q2D_OK) {
        p->R = R;
        p->Ntot = Ntot;
        p->h_box.assign(boxes, boxes + 3 * R);
        p->h_n.assign(n, n + R);
        p->h_off.assign(R + 1, 0);
        for (int r = 0; r < R; ++r) p->h_off[r + 1] = p->h_off[r] + n[r];
        // per-replica lattice constants and the k = 0 prefactor
        p->h_H.assign(3 * R, 0.0);  // H, then room for the per-replica charge sums
        p->h_diag.assign(R, 0.0);
        std::vector<double> tpa(R);
        for (int r = 0; r < R; ++r) {
            box_constants(p, boxes[3 * r], boxes[3 * r + 1], &p->h_H[r], &p->h_diag[r]);
            tpa[r] = 2.0 * PI / (boxes[3 * r] * boxes[3 * r + 1]);
        }
        std::vector<int32_t> rep_of(std::max<int64_t>(Ntot, 1), 0);
        for (int r = 0; r < R; ++r)
            for (int64_t i = p->h_off[r]; i < p->h_off[r + 1]; ++i) rep_of[i] = r;
        struct Up {
            Buf *b;
            const void *h;
            size_t bytes;
        } ups[] = {{&p->rep_box, p->h_box.data(), p->h_box.size() * sizeof(double)},
                   {&p->rep_H, p->h_H.data(), p->h_H.size() * sizeof(double)},
                   {&p->rep_diag, p->h_diag.data(), p->h_diag.size() * sizeof(double)},
                   {&p->rep_tpa, tpa.data(), tpa.size() * sizeof(double)},
                   {&p->rep_of, rep_of.data(), rep_of.size() * sizeof(int32_t)},
                   {&p->rep_off, p->h_off.data(), p->h_off.size() * sizeof(int64_t)}};
        for (const Up &u : ups) {
            if ((st = ensure(p, *u.b, u.bytes)) != Q2D_OK) break;
            if (hipMemcpyAsync(u.b->p, u.h, u.bytes, hipMemcpyHostToDevice, p->stream) !=
                hipSuccess) {
                st = Q2D_EDEVICE;
                break;
            }
        }
        if (st == Q2D_OK) st = ensure(p, p->step_ctr, sizeof(uint64_t));
        if (st == Q2D_OK) st = layout(p, 256);
    }
    if (st != Q2D_OK) {
        plan_release(p);
        delete p;
        return st;
    }
    *out = p;
    return Q2D_OK;
}

q2d_status q2d_batch_destroy(q2d_batch_t b) {
    if (!b) return Q2D_EINVAL;
    plan_release(b);
    delete b;
    return Q2D_OK;
}

q2d_status q2d_batch_set_stream(q2d_batch_t b, void *stream) {
    if (!b) return Q2D_EINVAL;
    b->stream = (hipStream_t)stream;
    return Q2D_OK;
}

q2d_status q2d_batch_set_segment(q2d_batch_t b, int32_t S) {
    if (!b || !valid_S(S)) return Q2D_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return Q2D_EDEVICE;
    return layout(b, S);
}

q2d_status q2d_batch_info(q2d_batch_t b, int32_t *segment, int64_t *n_padded, double *H,
                          double *diag_rb) {
    if (!b) return Q2D_EINVAL;
    if (segment) *segment = b->S_batch;
    if (n_padded) *n_padded = b->Npad;
    for (int r = 0; r < b->R; ++r) {
        if (H) H[r] = b->h_H[r];
        if (diag_rb) diag_rb[r] = b->h_diag[r];
    }
    return Q2D_OK;
}

q2d_status q2d_batch_rbm_step(q2d_batch_t b, const void *pos, const void *q, int32_t P,
                              uint64_t seed, uint64_t step, void *phi, void *F, double *E,
                              int32_t *modes_out) {
    q2d_status st = check_step_args(b, pos, q, P);
    if (st != Q2D_OK) return st;
    return batch_step(b, pos, q, P, seed, step, nullptr, phi, F, E, modes_out);
}

q2d_status q2d_batch_set_config(q2d_batch_t b, int32_t S, int32_t split, int32_t agg_cpw) {
    if (!b || !valid_config(S, split, agg_cpw)) return Q2D_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return Q2D_EDEVICE;
    return apply_config(b, Config{S, split, agg_cpw});
}

q2d_status q2d_batch_get_config(q2d_batch_t b, int32_t *S, int32_t *split, int32_t *agg_cpw) {
    if (!b) return Q2D_EINVAL;
    const Config c = current_config(b);
    if (S) *S = c.S;
    if (split) *split = c.split;
    if (agg_cpw) *agg_cpw = c.cpw;
    return Q2D_OK;
}

// Coordinate descent over the launch shapes, each candidate timed on the
// caller's data (one untimed step sizes its scratch, then 3 timed steps):
// the segment length S in {64, 128, 256, 512}, then the sweep's work-group
// split {per direction, both directions}, then the aggregate pass's chunks per
// wave {1, 2, 4}, then S once more.  The result is cached for the process by
// (device, R, total N, P, M, precision); a later tune of the same shape
// applies it without timing.
q2d_status q2d_batch_tune(q2d_batch_t b, const void *pos, const void *q, int32_t P, uint64_t seed,
                          void *phi, void *F, double *E, int32_t *segment) {
    q2d_status st = check_step_args(b, pos, q, P);
    if (st != Q2D_OK) return st;
    const TuneKey key{b->device, b->R, b->Ntot, P, b->M, b->fp32 ? 1 : 0};
    Config best = current_config(b);
    if (tune_cache_get(key, best)) {
        if ((st = apply_config(b, best)) == Q2D_OK && segment) *segment = best.S;
        return st;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return Q2D_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return Q2D_EDEVICE;
    }
    const int saved_timing = b->timing;
    b->timing = 0;
    float best_ms = 1e30f;
    auto time_config = [&](const Config &c) -> q2d_status {
        q2d_status s2 = apply_config(b, c);
        if (s2 != Q2D_OK) return s2;
        if ((s2 = batch_step(b, pos, q, P, seed, 0, nullptr, phi, F, E, nullptr)) != Q2D_OK)
            return s2;
        (void)hipEventRecord(e0, b->stream);
        for (int k = 0; k < 3 && s2 == Q2D_OK; ++k)
            s2 = batch_step(b, pos, q, P, seed, 1 + k, nullptr, phi, F, E, nullptr);
        (void)hipEventRecord(e1, b->stream);
        float ms = 0.f;
        if (s2 != Q2D_OK) return s2;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return Q2D_EDEVICE;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        return Q2D_OK;
    };
    const int cand_S[] = {64, 128, 256, 512};
    const int cand_split[] = {1, 2};
    const int cand_cpw[] = {1, 2, 4};
    for (int round = 0; round < 2 && st == Q2D_OK; ++round) {
        for (int S : cand_S) {
            Config c = best;
            c.S = S;
            if (st == Q2D_OK) st = time_config(c);
        }
        if (round == 1) break;
        for (int sp : cand_split) {
            Config c = best;
            c.split = sp;
            if (st == Q2D_OK) st = time_config(c);
        }
        for (int cw : cand_cpw) {
            Config c = best;
            c.cpw = cw;
            if (st == Q2D_OK) st = time_config(c);
        }
    }
    b->timing = saved_timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == Q2D_OK) st = apply_config(b, best);
    if (st == Q2D_OK) {
        tune_cache_put(key, best);
        if (segment) *segment = best.S;
    }
    return st;
}

q2d_status q2d_batch_capture(q2d_batch_t b, const void *pos, const void *q, int32_t P,
                             uint64_t seed, uint64_t step0, void *phi, void *F, double *E) {
    q2d_status st = check_step_args(b, pos, q, P);
    if (st != Q2D_OK) return st;
    // an eager step first: every scratch buffer exists before capture
    if ((st = batch_step(b, pos, q, P, seed, step0, nullptr, phi, F, E, nullptr)) != Q2D_OK)
        return st;
    if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return Q2D_EDEVICE;
    k_set_u64<<<1, 1, 0, b->stream>>>((uint64_t *)b->step_ctr.p, step0);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return Q2D_EDEVICE;
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
    const hipStream_t user = b->stream;
    const int saved_timing = b->timing;
    b->timing = 0;
    b->stream = b->cap_stream;
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        b->stream = user;
        b->timing = saved_timing;
        return Q2D_EDEVICE;
    }
    st = batch_step(b, pos, q, P, seed, 0, (const uint64_t *)b->step_ctr.p, phi, F, E, nullptr);
    if (st == Q2D_OK) k_inc_u64<<<1, 1, 0, b->stream>>>((uint64_t *)b->step_ctr.p);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap_stream, &g);
    b->stream = user;
    b->timing = saved_timing;
    if (st != Q2D_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return st != Q2D_OK ? st : Q2D_EDEVICE;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        b->graph = nullptr;
        b->graph_exec = nullptr;
        return Q2D_EDEVICE;
    }
    return Q2D_OK;
}

q2d_status q2d_batch_replay(q2d_batch_t b, int32_t n_steps) {
    if (!b || n_steps < 0) return Q2D_EINVAL;
    if (!b->graph_exec) return Q2D_EUNSUPPORTED;
    if (hipSetDevice(b->device) != hipSuccess) return Q2D_EDEVICE;
    for (int i = 0; i < n_steps; ++i)
        if (hipGraphLaunch(b->graph_exec, b->stream) != hipSuccess) return Q2D_EDEVICE;
    return Q2D_OK;
}

q2d_status q2d_batch_check(q2d_batch_t b) {
    if (!b) return Q2D_EINVAL;
    return plan_check(b);
}

}  // extern "C"
