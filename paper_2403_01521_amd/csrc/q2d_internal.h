// Internal declarations of the q2d library (host plan, scratch, kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/q2d.h"

namespace q2d {

constexpr int WAVE = 64;
constexpr int MAX_PAIRS = 16;  // M <= 32 SOE terms (conjugate pairs)

// ----------------------------------------------------------------------------
// small complex helper used on host and device
// ----------------------------------------------------------------------------
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ inline cx<T> cadd(cx<T> a, cx<T> b) {
    return {a.re + b.re, a.im + b.im};
}

// e^{-beta t} for the spans tables of the segmented carry scans (FP64: the
// carries are built from them); one definition for the k != 0 and k = 0 passes
__device__ inline cx<double> span_decay(double br, double bi, double t) {
    double sn, cs;
    sincos(bi * t, &sn, &cs);
    const double m = exp(-br * t);
    return {m * cs, -m * sn};
}

// SOE pair representatives passed to kernels by value.
struct PairParams {
    int mh;                       // number of conjugate pairs used
    double beta_re[MAX_PAIRS];    // beta_l = alpha s_l, representative with Im > 0
    double beta_im[MAX_PAIRS];
    // k = 0 combine coefficients (eq. 32 / eq. dzphi_0), pair-summed (x2):
    double c0u_re[MAX_PAIRS], c0u_im[MAX_PAIRS];  // phi: coefficient of U
    double c0v_re[MAX_PAIRS], c0v_im[MAX_PAIRS];  // phi: coefficient of V
    double f0u_re[MAX_PAIRS], f0u_im[MAX_PAIRS];  // dz:  coefficient of U
    double f0v_re[MAX_PAIRS], f0v_im[MAX_PAIRS];  // dz:  coefficient of V
    // per-term SOE data for mode coefficients (all M terms)
    int m_all;
    double w_re[2 * MAX_PAIRS], w_im[2 * MAX_PAIRS];
    double b_re[2 * MAX_PAIRS], b_im[2 * MAX_PAIRS];   // beta of every term
    int rep_of[2 * MAX_PAIRS];                          // pair index if representative, else -1
};

// Philox4x32-10 (Salmon et al., SC'11): multipliers 0xD2511F53, 0xCD9E8D57,
// key increments 0x9E3779B9, 0xBB67AE85.
__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// uniform in (0, 1) from 53 bits of two words
__device__ inline double u53(uint32_t a, uint32_t b) {
    const uint64_t v = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return ((double)v + 0.5) * 0x1p-53;
}

// Number of real fields per mode in a coefficient table:
//   0 kx, 1 ky, 2 k, 3 omega, 4 ak, 5 akd, then per pair l: al.re al.im ald.re ald.im
inline int coef_fields(int mh) { return 6 + 4 * mh; }

// ----------------------------------------------------------------------------
// device scratch buffer that grows on demand
// ----------------------------------------------------------------------------
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

// A launcher's scratch needs: the buffers it ensures, in the order it ensures
// them (fixed capacity: building a list allocates nothing).
struct BufReq {
    Buf *b;
    size_t bytes;
};
struct Reqs {
    static constexpr int CAP = 32;
    BufReq r[CAP];
    int n = 0;
    bool overflow = false;
    void add(Buf &b, size_t bytes) {
        if (n < CAP)
            r[n++] = BufReq{&b, bytes};
        else
            overflow = true;
    }
};

// Allocation-free calls: while a plan holds an arena, ensure() hands out
// consecutive 256-byte pieces of it instead of allocating, and remembers the
// buffer each piece replaced; arena_restore() puts the plan's own buffers back
// when the call has been enqueued.
struct Arena {
    static constexpr int CAP = 48;
    char *base = nullptr;
    size_t cap = 0, off = 0;
    Buf *lent[CAP];
    Buf saved[CAP];
    int n = 0;
};
// bytes an arena hands out for the requests, in order (the rule of ensure():
// a buffer already lent with enough bytes is reused, else a new piece)
size_t arena_need(const Reqs &q);
void arena_restore(Arena &a);

struct Plan {
    int device = 0;
    hipStream_t stream = nullptr;
    // internal stream for work independent of the mode scans (mode sampling,
    // the k = 0 term), forked from and joined back into `stream` by events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_sorted = nullptr, ev_modes = nullptr, ev_k0 = nullptr;
    double Lx, Ly, Lz, alpha, rc, kc;
    int M = 0, mh = 0;
    q2d_opts opts{};
    bool fp32 = false;
    PairParams pp{};
    double H = 0, diag_exact = 0, diag_rb = 0, k0_self = 0, c_lin = 0;
    std::vector<double> soe_w, soe_s;  // the SOE table (2M re, im each)

    // exact-k half-lattice mode list (device) and its coefficient table
    int64_t n_exact = 0, n_exact_pad = 0;
    Buf exact_modes;  // int32 [2][n_exact_pad]
    Buf exact_coef;   // T [fields][n_exact_pad]

    // caller-given mode list (q2d_modes_eval)
    Buf user_modes;   // int32 [2][n_pad]
    Buf user_w;       // double [n_pad]
    Buf user_coef;    // T [fields][n_pad]

    // random-batch tables
    Buf rb_modes;     // int32 [2][p_pad]
    Buf rb_coef;      // T [fields][p_pad]
    Buf rb_work;      // sampler work arrays
    Buf iid_tab;      // i.i.d. sampler: cumulative tables (FP64), built at creation
    int iid_mxm = 0, iid_mym = 0;

    // sorting and sorted data
    Buf keys_a, keys_b, vals_a, vals_b, hist;
    Buf recs;                  // (x, y, z, q) records in input order, for the gather
    Buf s_ux, s_uy, s_z, s_q;  // sorted SoA
    int32_t *perm = nullptr;   // points into vals_a or vals_b after the sort
    // sources of the scans: sorted q unless set (the adjoint pass points it at s_g)
    const void *src = nullptr;
    Buf s_g;                   // sorted adjoint weights g (T)
    Buf fq;                    // field of the charges q per particle, sorted order (FP64 x 3)

    // k != 0 scans
    Buf spans;                 // FP64 complex W,G per (segment, pair)
    Buf agg;                   // aggregates / carries (both directions)
    Buf carry_tmp;             // per-range transfers of the carry scan
    // the next random-batch step's modes, sampled ahead on the internal stream
    // at the end of a q2d_rbm_step call; the next call swaps them in when it
    // asks for (spec_seed, spec_step, spec_P) on the same stream
    Buf sp_modes, sp_coef, sp_status;
    bool spec_ok = false;
    bool no_ahead = false;  // set once a step of this plan was captured into a graph
    uint64_t spec_seed = 0, spec_step = 0;
    int32_t spec_P = 0;
    hipStream_t spec_stream = nullptr;
    Buf outk;                  // per-chunk per-particle outputs (T x 4)

    // k = 0 scans (own carry scratch: they run concurrently with the k != 0 scans)
    Buf spans0, agg0, carry_tmp0;
    Buf phi0, fz0;             // FP64 per particle (sorted order)

    // epilogue and status
    Buf epart;
    Buf inv;                   // int32 inverse of perm (input index -> sorted index)
    bool inv_ready = false;    // inv already enqueued for the current call (side stream)
    Buf status;                // int32 device status word

    // short range: cell starts, per-row tile offsets, cell-sorted records,
    // per-tile energy partials
    Buf cell_start, row_tiles, cell_rec, tile_e;

    // replica batch (R > 0): R independent systems of fixed sizes in one plan.
    // Inputs are concatenated by replica; after the sort each replica occupies
    // a run of whole segments of S_batch particles (padding: zero charge at
    // the replica's top height).
    int R = 0;
    int S_batch = 512;
    int64_t Ntot = 0, Npad = 0;
    std::vector<double> h_box, h_H, h_diag;      // [R][3], [R], [R]
    std::vector<int64_t> h_n, h_off, h_poff;     // [R], [R+1], [R+1]
    Buf rep_box;      // double [R][3]
    Buf rep_H;        // double [R]
    Buf rep_diag;     // double [R]: random-batch j = i constant
    Buf rep_tpa;      // double [R]: 2 pi / A
    Buf rep_of;       // int32 [Ntot]: replica of each input particle
    Buf rep_off;      // int64 [R+1]: input offsets
    Buf rep_poff;     // int64 [R+1]: padded offsets
    Buf seg_rep;      // int32 [Npad / S_batch]
    Buf pperm;        // int32 [Npad]: input index of each padded position, -1 for padding
    Buf epart_rep;    // double [Npad / S_batch]: per-segment energy partials
    int64_t rep_mstride = 0, rep_cstride = 0;    // per-replica table strides at this P
    // captured step (hipGraph) reading its step number from step_ctr
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    Buf step_ctr;     // uint64 [1]

    // timing
    int timing = 0;  // bit mask of timed kernel families
    int timing_stride = 1;  // record on every timing_stride-th call only
    int64_t ncalls = 0;     // entry-point calls (counted at the call timer's start)
    // Q2D_SERIAL=1 at plan creation: the side-stream work runs on the caller's
    // stream (no overlap; for per-kernel profiles)
    bool serial = false;
    hipEvent_t ev[5][2]{};
    double t_ms[5]{};
    int64_t t_cnt[5]{};
    std::vector<hipEvent_t> pend_ev[5];
    // non-null during an allocation-free call
    Arena *arena = nullptr;
    // launch shapes of the k != 0 passes (0: the default): one work-group per
    // sweep direction (1) or both in one (2); 16-mode chunks per wave of the
    // FP32 aggregate pass (1, 2 or 4)
    int cfg_split = 0, cfg_cpw = 0;
};

// growth helper: ensure buffer holds at least `bytes`
q2d_status ensure(Plan *p, Buf &b, size_t bytes);

// scratch requests of the launchers (the same lists their own ensure() calls use)
void sort_reqs(Plan *p, int64_t N, Reqs &q);
void sampler_reqs(Plan *p, int P, Reqs &q);
void kmodes_reqs(Plan *p, int64_t N, int64_t n_modes, Reqs &q);
void k0_reqs(Plan *p, int64_t N, Reqs &q);
void inv_reqs(Plan *p, int64_t N, Reqs &q);
void epilogue_reqs(Plan *p, int64_t N, Reqs &q);
// bytes of the range-transfer scratch of a carry scan over ncols columns
size_t carry_tmp_bytes(int64_t ncols, int nseg);
// ensure every request of a list
q2d_status ensure_all(Plan *p, const Reqs &q);

// plan set-up shared by single systems and replica batches (q2d_api.hip)
q2d_status plan_init(Plan *p, double Lx, double Ly, double Lz, double alpha, double r_c,
                     double k_c, int32_t M, const double *w, const double *s, const q2d_opts *opts,
                     void *stream);
void plan_release(Plan *p);
// wait for the stream, read and clear the device status word
q2d_status plan_check(Plan *p);
// H and the random-batch j = i constant of a box for the plan's SOE table
void box_constants(const Plan *p, double Lx, double Ly, double *H, double *diag_rb);

// integer from the environment (tuning switches), dflt if unset
int env_int(const char *name, int dflt);

// timing helpers
void tstart(Plan *p, int which);
void tstop(Plan *p, int which);

// ----------------------------------------------------------------------------
// launchers (each enqueues on p->stream)
// ----------------------------------------------------------------------------
// validation + key staging + stable radix sort by z + gather of sorted SoA
q2d_status sort_and_stage(Plan *p, const void *pos, const void *q, int64_t N);
// stable LSD radix sort (8-bit digits, `passes` of them) of N uint32 keys in
// p->keys_a with values in p->vals_a (keys_b, vals_b, hist: scratch); returns
// where the sorted keys and values ended up
q2d_status radix_sort_u32(Plan *p, int64_t N, int passes, uint32_t **keys_out,
                          int32_t **vals_out);
// replica batches: sort by (replica, z) into the padded segment layout
q2d_status sort_and_stage_batch(Plan *p, const void *pos, const void *q);

// device coefficient tables for a list of modes
q2d_status build_mode_coefs(Plan *p, const int32_t *modes, int64_t n, int64_t n_pad,
                            const double *weights_dev, double weight_const, void *coef);

// cumulative tables of the i.i.d. mode sampler (host)
void iid_tables(double alpha, double Lx, double Ly, std::vector<double> &tab, int *mxm, int *mym);
// random-batch sampler: writes p->rb_modes and p->rb_coef for P modes
q2d_status sample_modes(Plan *p, int P, uint64_t seed, uint64_t step, int *status = nullptr);
// replica batches: P modes per replica ([r][2][p_pad], [r][fields][p_pad]);
// step is read from step_dev when it is not null (captured steps)
q2d_status sample_modes_batch(Plan *p, int P, uint64_t seed, uint64_t step,
                              const uint64_t *step_dev);

// k != 0 part over a mode table: per-particle outputs in n_chunks_out chunks
// of outk, to be summed
q2d_status kmodes_run(Plan *p, int64_t N, const int32_t *modes, const void *coef,
                      int64_t coef_stride, int64_t mode_off, int64_t n_modes, int *n_chunks_out);

// k = 0 term: writes p->phi0, p->fz0 (FP64, sorted order)
q2d_status k0_run(Plan *p, int64_t N);

// combine, unsort, energy
// inverse permutation of the current sort, on p->stream (single systems)
q2d_status launch_inv(Plan *p, int64_t N);
q2d_status epilogue(Plan *p, int64_t N, int n_chunks, double diag, bool with_k0, void *phi,
                    void *F, double *E);

// replica batches: combine, unsort (padding skipped), energy per replica
q2d_status epilogue_batch(Plan *p, int n_chunks, void *phi, void *F, double *E);

// adjoint: sorted copy of the caller's weights g into s_g
q2d_status gather_sources(Plan *p, const void *g, int64_t N);
// adjoint: keep the field of the current sources (charges q) in p->fq
q2d_status epilogue_field(Plan *p, int64_t N, int n_chunks);
// adjoint: with the outputs of the pass over sources g, write
//   dq = phi(g) (j = i constant, k = 0 and self terms included) and
//   dpos = -(g * field(q) + q * field(g)), unsorted
q2d_status epilogue_vjp(Plan *p, int64_t N, int n_chunks, double diag, void *dq, void *dpos);

// Enqueue on the plan's internal stream within a scope: the launchers use p->stream.
struct SideScope {
    Plan *p;
    hipStream_t saved;
    explicit SideScope(Plan *p_) : p(p_), saved(p_->stream) {
        if (!p->serial) p->stream = p->side;
    }
    ~SideScope() { p->stream = saved; }
};

// Extra work of a random-batch step on the internal stream: with modes
// sampled ahead (hit), their sampler status and the caller's mode copy; and
// the next step's modes sampled ahead after the k = 0 term (ahead).
struct SideExtra {
    bool hit = false;
    int32_t *modes_out = nullptr;
    int P = 0;
    bool ahead = false;
    uint64_t seed = 0, next_step = 0;
};

// the k = 0 term on the internal stream once the sorted data exist; the main
// stream must wait for ev_k0 before reading phi0 / fz0
q2d_status k0_side(Plan *p, int64_t N, const SideExtra *ex = nullptr);
// the modes of (seed, step) into sp_modes / sp_coef, sampler status into sp_status
q2d_status sample_modes_ahead(Plan *p, int P, uint64_t seed, uint64_t step);
// on p->stream: the sampled-ahead status bits into the plan's status word, and
// the modes of rb_modes into the caller's array
q2d_status ahead_hit_side(Plan *p, int P, int32_t *modes_out);

// short range
q2d_status short_range_run(Plan *p, const void *pos, const void *q, int64_t N, void *phi, void *F,
                           double *E);

}  // namespace q2d

// The opaque handles of the C ABI are the plan itself.
struct q2d_plan : public q2d::Plan {};
struct q2d_batch : public q2d::Plan {};
