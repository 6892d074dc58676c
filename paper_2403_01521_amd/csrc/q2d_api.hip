// C ABI of the library: plan set-up (host FP64 precomputation) and the entry
// points.  See include/q2d.h for the contract of every function.
//
// Host precomputation at plan creation ("Precomputation" of Alg. 1 and Alg. 2):
//  * the SOE table is checked and split into conjugate pairs;
//  * H = sum_{k != 0} exp(-k^2/(4 alpha^2)) (Sec. 4.1, eq. hk) by direct lattice sum;
//  * the exact-k half-lattice mode list 0 < |k| <= k_c with weights
//    2 (pi/A) exp(-k^2/(4 alpha^2)) (the k and -k terms are complex conjugates);
//  * the j = i constants D = (pi/A) sum_k e^{-k^2/4a^2} K_k(0) of the SOE
//    kernel, over |k| <= k_c (exact-k) and over the whole lattice (random batch);
//  * the k = 0 constants K_0(0) and the linear coefficient (2/sqrt(pi)) sum w_l/s_l.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <new>

#include "q2d_internal.h"

namespace q2d {

static size_t piece(size_t bytes) { return ((bytes ? bytes : 16) + 255) & ~(size_t)255; }

// an allocation-free call: lend b a piece of the arena (never allocates)
static q2d_status arena_take(Arena &a, Buf &b, size_t bytes) {
    int i = 0;
    while (i < a.n && a.lent[i] != &b) ++i;
    if (i < a.n && b.bytes >= bytes) return Q2D_OK;
    if (i == a.n) {
        if (a.n == Arena::CAP) return Q2D_ECAPACITY;
        a.lent[a.n] = &b;
        a.saved[a.n] = b;
        ++a.n;
    }
    const size_t sz = piece(bytes);
    if (a.off + sz > a.cap) return Q2D_ECAPACITY;
    b.p = a.base + a.off;
    b.bytes = sz;
    a.off += sz;
    return Q2D_OK;
}

size_t arena_need(const Reqs &q) {
    if (q.overflow) return ~(size_t)0;
    const Buf *seen[Reqs::CAP];
    size_t have[Reqs::CAP];
    int n = 0;
    size_t total = 0;
    for (int r = 0; r < q.n; ++r) {
        int i = 0;
        while (i < n && seen[i] != q.r[r].b) ++i;
        if (i < n && have[i] >= q.r[r].bytes) continue;
        if (i == n) seen[n++] = q.r[r].b;
        have[i] = piece(q.r[r].bytes);
        total += have[i];
    }
    return total;
}

void arena_restore(Arena &a) {
    for (int i = a.n - 1; i >= 0; --i) *a.lent[i] = a.saved[i];
    a.n = 0;
}

q2d_status ensure_all(Plan *p, const Reqs &q) {
    if (q.overflow) return Q2D_EINVAL;
    for (int r = 0; r < q.n; ++r) {
        const q2d_status st = ensure(p, *q.r[r].b, q.r[r].bytes);
        if (st != Q2D_OK) return st;
    }
    return Q2D_OK;
}

q2d_status ensure(Plan *p, Buf &b, size_t bytes) {
    if (p->arena) return arena_take(*p->arena, b, bytes);
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return Q2D_OK;
    if (b.p) {
        if (hipStreamSynchronize(p->stream) != hipSuccess) return Q2D_EDEVICE;
        if (p->side && hipStreamSynchronize(p->side) != hipSuccess) return Q2D_EDEVICE;
        // a captured step holds the old address: drop the graph (replay then
        // returns Q2D_EUNSUPPORTED until the next capture)
        if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->graph_exec = nullptr;
        p->graph = nullptr;
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    const size_t sz = (bytes + 255) & ~(size_t)255;
    if (hipMalloc(&b.p, sz) != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return Q2D_ENOMEM;
    }
    b.bytes = sz;
    return Q2D_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free step: one static array per device, held
// until the process ends.  Its host-side name is not a device address: host
// code uses only the address looked up once per device (with that device
// current) when a plan is created there.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[Q2D_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_DEVICES = 64;
std::mutex noalloc_mu;
bool noalloc_looked[NOALLOC_DEVICES];
char *noalloc_ptr[NOALLOC_DEVICES];
}  // namespace

// once per device, with that device current (plan creation)
static void noalloc_setup(int dev) {
    if (dev < 0 || dev >= NOALLOC_DEVICES) return;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (noalloc_looked[dev]) return;
    noalloc_looked[dev] = true;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr)
        noalloc_ptr[dev] = (char *)ptr;
    else
        (void)hipGetLastError();
}

static char *noalloc_base(int dev) {
    if (dev < 0 || dev >= NOALLOC_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    return noalloc_ptr[dev];
}

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return (v && *v) ? atoi(v) : dflt;
}

// calls are counted where every entry point starts its call timer; a call
// records its events only if it is a sampled one (every timing_stride-th)
static bool timing_on(const Plan *p, int which) {
    return (p->timing & (1 << which)) && p->ncalls % p->timing_stride == 0;
}

void tstart(Plan *p, int which) {
    if (which == 4) ++p->ncalls;
    if (!timing_on(p, which)) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, p->stream);
    p->pend_ev[which].push_back(e);
}

void tstop(Plan *p, int which) {
    if (!timing_on(p, which)) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, p->stream);
    p->pend_ev[which].push_back(e);
}

static void timing_flush(Plan *p) {
    for (int w = 0; w < 5; ++w) {
        auto &v = p->pend_ev[w];
        for (size_t i = 0; i + 1 < v.size(); i += 2) {
            float ms = 0.f;
            if (hipEventSynchronize(v[i + 1]) == hipSuccess &&
                hipEventElapsedTime(&ms, v[i], v[i + 1]) == hipSuccess) {
                p->t_ms[w] += ms;
                p->t_cnt[w] += 1;
            }
        }
        for (auto e : v) (void)hipEventDestroy(e);
        v.clear();
    }
}

static void free_buf(Buf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

}  // namespace q2d

using namespace q2d;
using cd = std::complex<double>;

namespace {

const double PI = 3.14159265358979323846;

// K_k(0) of the SOE pair kernel (eq. SOEphi at z = 0, Gaussian factor removed)
double soe_K0_at(double k, double alpha, const std::vector<cd> &w, const std::vector<cd> &s) {
    cd acc = 0.0;
    for (size_t l = 0; l < w.size(); ++l) {
        const cd b = alpha * s[l];
        acc += w[l] * (2.0 * b - 2.0 * k) / (b * b - k * k);
    }
    return (2.0 * alpha / (std::sqrt(PI) * k) * acc).real();
}

// Direct lattice sums of a box (Sec. 4.1, eq. hk; the j = i constants of the
// k != 0 modes): H = sum_{k != 0} e^{-k^2/4a^2}, and D = (pi/A) sum e^{-k^2/4a^2}
// K_k(0) over the whole lattice (random batch) and over 0 < |k| <= k_c (exact-k).
// Terms with e^{-k^2/4a^2} < 1e-18 are dropped.
void lattice_sums(double Lx, double Ly, double alpha, double k_c, const std::vector<cd> &wc,
                  const std::vector<cd> &sc, double *H, double *diag_rb, double *diag_exact) {
    const double A = Lx * Ly;
    const double kmax = 2.0 * alpha * std::sqrt(std::log(1e18));
    const int mxm = (int)std::ceil(kmax * Lx / (2 * PI)), mym = (int)std::ceil(kmax * Ly / (2 * PI));
    double gx = 0, gy = 0;
    for (int m = -mxm; m <= mxm; ++m) gx += std::exp(-std::pow(2 * PI * m / Lx, 2) / (4 * alpha * alpha));
    for (int m = -mym; m <= mym; ++m) gy += std::exp(-std::pow(2 * PI * m / Ly, 2) / (4 * alpha * alpha));
    *H = gx * gy - 1.0;
    double drb = 0.0, dex = 0.0;
    for (int mx = -mxm; mx <= mxm; ++mx)
        for (int my = -mym; my <= mym; ++my) {
            if (mx == 0 && my == 0) continue;
            const double kx = 2 * PI * mx / Lx, ky = 2 * PI * my / Ly;
            const double k2 = kx * kx + ky * ky;
            if (k2 > kmax * kmax) continue;
            const double k = std::sqrt(k2);
            const double t = std::exp(-k2 / (4 * alpha * alpha)) * soe_K0_at(k, alpha, wc, sc);
            drb += t;
            if (k_c > 0 && k2 <= k_c * k_c) dex += t;
        }
    *diag_rb = PI / A * drb;
    *diag_exact = 0.0;
    if (k_c > 0) {
        // exact-k terms beyond kmax (if k_c > kmax) are below 1e-18 of the first
        const int ex = (int)std::floor(k_c * Lx / (2 * PI)), ey = (int)std::floor(k_c * Ly / (2 * PI));
        if (k_c > kmax)
            for (int mx = -ex; mx <= ex; ++mx)
                for (int my = -ey; my <= ey; ++my) {
                    const double kx = 2 * PI * mx / Lx, ky = 2 * PI * my / Ly;
                    const double k2 = kx * kx + ky * ky;
                    if ((mx == 0 && my == 0) || k2 <= kmax * kmax || k2 > k_c * k_c) continue;
                    const double k = std::sqrt(k2);
                    dex += std::exp(-k2 / (4 * alpha * alpha)) * soe_K0_at(k, alpha, wc, sc);
                }
        *diag_exact = PI / A * dex;
    }
}

int first_error(int bits) {
    const int order[] = {Q2D_EOUTOFBOX, Q2D_ENONNEUTRAL, Q2D_ESAMPLER};
    for (int c : order)
        if (bits & (1 << c)) return c;
    return Q2D_OK;
}

__global__ void k_zero_status(int *st, double *qs) {
    st[0] = 0;
    qs[0] = 0.0;
    qs[1] = 0.0;
}

// caller's (mx, my) pairs and weights -> the [2][n_pad] mode table; a (0, 0)
// entry (no k != 0 mode) becomes (1, 0) with weight 0 so that it adds nothing
__global__ void k_user_modes(const int32_t *in, const double *w_in, int64_t n, int64_t n_pad,
                             int32_t *modes, double *w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    int32_t mx = 0, my = 0;
    double wt = 0.0;
    if (i < n) {
        mx = in[2 * i];
        my = in[2 * i + 1];
        wt = w_in[i];
    }
    if (mx == 0 && my == 0) {
        mx = 1;
        wt = 0.0;
    }
    modes[i] = mx;
    modes[n_pad + i] = my;
    w[i] = wt;
}

__global__ void k_modes_out(const int32_t *modes, int P, int p_pad, int32_t *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) {
        out[2 * i] = modes[i];
        out[2 * i + 1] = modes[p_pad + i];
    }
}

// error bits of a sampler run into the plan's status word (which kernels on
// the other stream may set at the same time)
__global__ void k_word_or(int *dst, const int *src) {
    if (*src) atomicOr(dst, *src);
}

// The two passes of the adjoint once the particles are sorted (and, for the
// random batch, the modes drawn): sources q keep their field in p->fq, then
// sources g give phi(g) and f(g), combined by the adjoint epilogue.
q2d_status vjp_passes(Plan *p, int64_t N, const int32_t *modes, const void *coef,
                      int64_t stride, int64_t n_modes, double diag, const void *g, void *dq,
                      void *dpos) {
    q2d_status st;
    int nch = 0;
    p->src = nullptr;
    if ((st = k0_side(p, N)) != Q2D_OK) return st;
    if (n_modes > 0 && (st = kmodes_run(p, N, modes, coef, stride, 0, n_modes, &nch)) != Q2D_OK)
        return st;
    if (hipStreamWaitEvent(p->stream, p->ev_k0, 0) != hipSuccess) return Q2D_EDEVICE;
    if ((st = epilogue_field(p, N, nch)) != Q2D_OK) return st;
    if ((st = gather_sources(p, g, N)) != Q2D_OK) return st;
    p->src = p->s_g.p;
    st = k0_side(p, N);
    if (st == Q2D_OK && n_modes > 0) st = kmodes_run(p, N, modes, coef, stride, 0, n_modes, &nch);
    p->src = nullptr;
    if (st != Q2D_OK) return st;
    if (hipStreamWaitEvent(p->stream, p->ev_k0, 0) != hipSuccess) return Q2D_EDEVICE;
    return epilogue_vjp(p, N, nch, diag, dq, dpos);
}

}  // namespace

namespace q2d {

q2d_status ahead_hit_side(Plan *p, int P, int32_t *modes_out) {
    k_word_or<<<1, 1, 0, p->stream>>>((int *)p->status.p, (const int *)p->sp_status.p);
    if (modes_out) {
        const int p_pad = ((P + WAVE - 1) / WAVE) * WAVE;
        k_modes_out<<<(P + 255) / 256, 256, 0, p->stream>>>((const int32_t *)p->rb_modes.p, P,
                                                            p_pad, modes_out);
    }
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

q2d_status k0_side(Plan *p, int64_t N, const SideExtra *ex) {
    if (hipEventRecord(p->ev_sorted, p->stream) != hipSuccess ||
        hipStreamWaitEvent(p->side, p->ev_sorted, 0) != hipSuccess)
        return Q2D_EDEVICE;
    q2d_status st = Q2D_OK;
    {
        SideScope side(p);
        if (ex && ex->hit) st = ahead_hit_side(p, ex->P, ex->modes_out);
        // the epilogue's inverse permutation, off the critical path
        if (st == Q2D_OK && !p->R && (st = launch_inv(p, N)) == Q2D_OK) p->inv_ready = true;
        if (st == Q2D_OK) st = k0_run(p, N);
        // the next step's modes: the main stream waits for ev_k0 before its
        // epilogue, so they are in place before the next call's first launch
        if (st == Q2D_OK && ex && ex->ahead)
            st = sample_modes_ahead(p, ex->P, ex->seed, ex->next_step);
    }
    if (st != Q2D_OK) return st;
    return hipEventRecord(p->ev_k0, p->side) == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

// Validation and host set-up of a plan (allocated by the caller); on failure
// the caller releases it with plan_release.
q2d_status plan_init(Plan *p, double Lx, double Ly, double Lz, double alpha, double r_c,
                     double k_c, int32_t M, const double *w, const double *s, const q2d_opts *opts,
                     void *stream) {
    if (!opts || !w || !s) return Q2D_EINVAL;
    if (!(Lx > 0 && Ly > 0 && Lz > 0 && alpha > 0) || !std::isfinite(Lx) || !std::isfinite(Ly) ||
        !std::isfinite(Lz) || !std::isfinite(alpha) || std::isnan(r_c) || std::isnan(k_c))
        return Q2D_EINVAL;
    if (M < 2 || M > 2 * MAX_PAIRS || (M % 2)) return Q2D_EINVAL;
    if (opts->precision != Q2D_FP64 && opts->precision != Q2D_FP32) return Q2D_EINVAL;
    if (opts->n_max <= 0 || opts->n_max > ((int64_t)1 << 31) - 1 || opts->p_max < 0 ||
        opts->thin < 0)
        return Q2D_EINVAL;
    if (opts->sampler != Q2D_SAMPLER_METROPOLIS && opts->sampler != Q2D_SAMPLER_IID)
        return Q2D_EINVAL;
    if (r_c > 0 && r_c > 0.5 * std::min(Lx, Ly)) return Q2D_EINVAL;
    // SOE table: conjugate-closed, Re s > 0, no real node
    std::vector<cd> wc(M), sc(M);
    for (int l = 0; l < M; ++l) {
        wc[l] = cd(w[2 * l], w[2 * l + 1]);
        sc[l] = cd(s[2 * l], s[2 * l + 1]);
        if (!std::isfinite(wc[l].real()) || !std::isfinite(wc[l].imag()) ||
            !std::isfinite(sc[l].real()) || !std::isfinite(sc[l].imag()))
            return Q2D_EINVAL;
        if (!(sc[l].real() > 0) || std::fabs(sc[l].imag()) <= 1e-12 * std::abs(sc[l]))
            return Q2D_EINVAL;
    }
    std::vector<int> partner(M, -1);
    for (int l = 0; l < M; ++l) {
        for (int j = 0; j < M; ++j) {
            if (j == l) continue;
            if (std::abs(sc[j] - std::conj(sc[l])) <= 1e-10 * std::abs(sc[l]) &&
                std::abs(wc[j] - std::conj(wc[l])) <= 1e-10 * std::abs(wc[l]) + 1e-300) {
                partner[l] = j;
                break;
            }
        }
        if (partner[l] < 0) return Q2D_EINVAL;
    }

    p->Lx = Lx;
    p->Ly = Ly;
    p->Lz = Lz;
    p->alpha = alpha;
    p->rc = r_c;
    p->kc = k_c;
    p->M = M;
    p->mh = M / 2;
    p->opts = *opts;
    if (p->opts.thin <= 0) p->opts.thin = 1;
    p->fp32 = opts->precision == Q2D_FP32;
    p->stream = (hipStream_t)stream;
    p->serial = env_int("Q2D_SERIAL", 0) != 0;
    if (hipGetDevice(&p->device) != hipSuccess) return Q2D_EDEVICE;
    noalloc_setup(p->device);
    if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_sorted, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_modes, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_k0, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return Q2D_EDEVICE;
    }

    // pair representatives (Im s > 0) and k = 0 combine coefficients
    PairParams &pp = p->pp;
    pp.mh = p->mh;
    pp.m_all = M;
    int r = 0;
    const double sqpi = std::sqrt(PI);
    for (int l = 0; l < M; ++l) {
        pp.w_re[l] = wc[l].real();
        pp.w_im[l] = wc[l].imag();
        pp.b_re[l] = alpha * sc[l].real();
        pp.b_im[l] = alpha * sc[l].imag();
        pp.rep_of[l] = -1;
        if (sc[l].imag() > 0) {
            if (r >= MAX_PAIRS) return Q2D_EINVAL;
            pp.rep_of[l] = r;
            pp.beta_re[r] = alpha * sc[l].real();
            pp.beta_im[r] = alpha * sc[l].imag();
            const cd ws = wc[l] / sqpi;
            const cd cu = 2.0 * ws / alpha;
            const cd cv = -2.0 * ws * (2.0 / sc[l]);
            const cd fu = -2.0 * ws * (sc[l] + 2.0 / sc[l]);
            const cd fv = 2.0 * ws * (2.0 * alpha);
            pp.c0u_re[r] = cu.real();
            pp.c0u_im[r] = cu.imag();
            pp.c0v_re[r] = cv.real();
            pp.c0v_im[r] = cv.imag();
            pp.f0u_re[r] = fu.real();
            pp.f0u_im[r] = fu.imag();
            pp.f0v_re[r] = fv.real();
            pp.f0v_im[r] = fv.imag();
            ++r;
        }
    }
    if (r != p->mh) return Q2D_EINVAL;
    cd clin = 0.0, k0s = 0.0;
    for (int l = 0; l < M; ++l) {
        clin += wc[l] / sc[l];
        k0s += wc[l] / (alpha * sqpi);
    }
    p->c_lin = 2.0 / sqpi * clin.real();
    p->k0_self = k0s.real();

    // lattice sums: H and the j = i constants
    lattice_sums(Lx, Ly, alpha, k_c, wc, sc, &p->H, &p->diag_rb, &p->diag_exact);
    p->soe_w.assign(w, w + 2 * M);
    p->soe_s.assign(s, s + 2 * M);
    const double A = Lx * Ly;
    q2d_status st = ensure(p, p->status, 64);
    if (st != Q2D_OK) return st;
    if (opts->sampler == Q2D_SAMPLER_IID && opts->p_max > 0) {
        std::vector<double> tab;
        iid_tables(alpha, Lx, Ly, tab, &p->iid_mxm, &p->iid_mym);
        if ((st = ensure(p, p->iid_tab, tab.size() * sizeof(double))) != Q2D_OK) return st;
        if (hipMemcpy(p->iid_tab.p, tab.data(), tab.size() * sizeof(double),
                      hipMemcpyHostToDevice) != hipSuccess)
            return Q2D_EDEVICE;
    }
    k_zero_status<<<1, 1, 0, p->stream>>>((int *)p->status.p, (double *)((char *)p->status.p + 16));

    // exact-k half-lattice mode table
    if (k_c > 0) {
        std::vector<int32_t> mxv, myv;
        std::vector<double> wt;
        const int ex = (int)std::floor(k_c * Lx / (2 * PI)), ey = (int)std::floor(k_c * Ly / (2 * PI));
        for (int mx = 0; mx <= ex; ++mx)
            for (int my = (mx == 0 ? 1 : -ey); my <= ey; ++my) {
                const double kx = 2 * PI * mx / Lx, ky = 2 * PI * my / Ly;
                const double k2 = kx * kx + ky * ky;
                if (k2 > k_c * k_c) continue;
                mxv.push_back(mx);
                myv.push_back(my);
                wt.push_back(2.0 * PI / A * std::exp(-k2 / (4 * alpha * alpha)));
            }
        p->n_exact = (int64_t)mxv.size();
        p->n_exact_pad = ((p->n_exact + WAVE - 1) / WAVE) * WAVE;
        if (p->n_exact > 0) {
            const int64_t np = p->n_exact_pad;
            std::vector<int32_t> m2(2 * np, 0);
            std::vector<double> w2(np, 0.0);
            for (int64_t i = 0; i < p->n_exact; ++i) {
                m2[i] = mxv[i];
                m2[np + i] = myv[i];
                w2[i] = wt[i];
            }
            Buf wbuf;
            const size_t tsz = p->fp32 ? sizeof(float) : sizeof(double);
            if ((st = ensure(p, p->exact_modes, m2.size() * sizeof(int32_t))) != Q2D_OK ||
                (st = ensure(p, p->exact_coef, (size_t)coef_fields(p->mh) * np * tsz)) != Q2D_OK ||
                (st = ensure(p, wbuf, w2.size() * sizeof(double))) != Q2D_OK) {
                free_buf(wbuf);
                return st;
            }
            if (hipMemcpyAsync(p->exact_modes.p, m2.data(), m2.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, p->stream) != hipSuccess ||
                hipMemcpyAsync(wbuf.p, w2.data(), w2.size() * sizeof(double),
                               hipMemcpyHostToDevice, p->stream) != hipSuccess) {
                free_buf(wbuf);
                return Q2D_EDEVICE;
            }
            st = build_mode_coefs(p, (const int32_t *)p->exact_modes.p, p->n_exact, np,
                                  (const double *)wbuf.p, 0.0, p->exact_coef.p);
            (void)hipStreamSynchronize(p->stream);
            free_buf(wbuf);
            if (st != Q2D_OK) return st;
        }
    }
    if (hipStreamSynchronize(p->stream) != hipSuccess) return Q2D_EDEVICE;
    return Q2D_OK;
}


// Wait for the plan's work and free everything it owns (not the struct).
void box_constants(const Plan *p, double Lx, double Ly, double *H, double *diag_rb) {
    const int M = p->M;
    std::vector<cd> wc(M), sc(M);
    for (int l = 0; l < M; ++l) {
        wc[l] = cd(p->soe_w[2 * l], p->soe_w[2 * l + 1]);
        sc[l] = cd(p->soe_s[2 * l], p->soe_s[2 * l + 1]);
    }
    double dex = 0.0;
    lattice_sums(Lx, Ly, p->alpha, 0.0, wc, sc, H, diag_rb, &dex);
}

void plan_release(Plan *p) {
    (void)hipSetDevice(p->device);
    (void)hipStreamSynchronize(p->stream);
    if (p->side) (void)hipStreamSynchronize(p->side);
    for (int w = 0; w < 5; ++w) {
        for (auto e : p->pend_ev[w]) (void)hipEventDestroy(e);
        p->pend_ev[w].clear();
    }
    Buf *bufs[] = {&p->exact_modes, &p->exact_coef, &p->rb_modes, &p->rb_coef, &p->rb_work,
                   &p->sp_modes, &p->sp_coef, &p->sp_status,
                   &p->iid_tab,
                   &p->user_modes, &p->user_w, &p->user_coef, &p->s_g, &p->fq,
                   &p->keys_a, &p->keys_b, &p->vals_a, &p->vals_b, &p->hist, &p->s_ux,
                   &p->s_uy, &p->s_z, &p->s_q, &p->spans, &p->agg, &p->carry_tmp, &p->outk, &p->spans0,
                   &p->agg0, &p->carry_tmp0, &p->phi0, &p->fz0, &p->epart, &p->inv, &p->status,
                   &p->cell_start, &p->row_tiles, &p->cell_rec, &p->tile_e, &p->rep_box,
                   &p->rep_H, &p->rep_diag, &p->rep_tpa, &p->rep_of, &p->rep_off, &p->rep_poff,
                   &p->seg_rep, &p->pperm, &p->epart_rep, &p->step_ctr, &p->recs};
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    for (Buf *b : bufs) free_buf(*b);
    for (hipEvent_t e : {p->ev_fork, p->ev_sorted, p->ev_modes, p->ev_k0})
        if (e) (void)hipEventDestroy(e);
    if (p->side) (void)hipStreamDestroy(p->side);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    p->side = nullptr;
    p->cap_stream = nullptr;
}


}  // namespace q2d

extern "C" {

const char *q2d_status_string(q2d_status st) {
    switch (st) {
        case Q2D_OK: return "ok";
        case Q2D_EINVAL: return "invalid argument";
        case Q2D_ENONNEUTRAL: return "system is not charge neutral";
        case Q2D_EOUTOFBOX: return "particle outside [0, Lz] in z or non-finite input";
        case Q2D_ENOMEM: return "out of memory";
        case Q2D_ECAPACITY: return "size exceeds the plan's capacity";
        case Q2D_EDEVICE: return "HIP runtime error";
        case Q2D_ESAMPLER: return "mode sampler found no non-zero proposal";
        case Q2D_EUNSUPPORTED: return "plan was created without support for this call";
        case Q2D_EDTYPE: return "element type differs from the plan's precision";
    }
    return "unknown status";
}

q2d_status q2d_plan_create(double Lx, double Ly, double Lz, double alpha, double r_c, double k_c,
                           int32_t M, const double *w, const double *s, const q2d_opts *opts,
                           void *stream, q2d_plan_t *out) {
    if (!out) return Q2D_EINVAL;
    *out = nullptr;
    q2d_plan *p = new (std::nothrow) q2d_plan();
    if (!p) return Q2D_ENOMEM;
    const q2d_status st = plan_init(p, Lx, Ly, Lz, alpha, r_c, k_c, M, w, s, opts, stream);
    if (st != Q2D_OK) {
        plan_release(p);
        delete p;
        return st;
    }
    *out = p;
    return Q2D_OK;
}

q2d_status q2d_plan_destroy(q2d_plan_t p) {
    if (!p) return Q2D_EINVAL;
    plan_release(p);
    delete p;
    return Q2D_OK;
}

q2d_status q2d_plan_set_stream(q2d_plan_t p, void *stream) {
    if (!p) return Q2D_EINVAL;
    p->stream = (hipStream_t)stream;
    p->spec_ok = false;
    return Q2D_OK;
}

q2d_status q2d_plan_info(q2d_plan_t p, q2d_info *info) {
    if (!p || !info) return Q2D_EINVAL;
    info->n_modes_exact = p->n_exact;
    info->M = p->M;
    info->H = p->H;
    info->diag_exact = p->diag_exact;
    info->diag_rb = p->diag_rb;
    info->soe_k0_self = p->k0_self;
    return Q2D_OK;
}

static q2d_status check_io(q2d_plan_t p, const void *pos, const void *q, int64_t N) {
    if (!p) return Q2D_EINVAL;
    if (N < 0) return Q2D_EINVAL;
    if (N > 0 && (!pos || !q)) return Q2D_EINVAL;
    if (N > p->opts.n_max) return Q2D_ECAPACITY;
    if (hipSetDevice(p->device) != hipSuccess) return Q2D_EDEVICE;
    return Q2D_OK;
}

q2d_status q2d_long_range(q2d_plan_t p, const void *pos, const void *q, int64_t N, void *phi,
                          void *F, double *E) {
    q2d_status st = check_io(p, pos, q, N);
    if (st != Q2D_OK) return st;
    if (!(p->kc > 0)) return Q2D_EUNSUPPORTED;
    tstart(p, 4);
    int nch = 0;
    if (N > 0) {
        if ((st = sort_and_stage(p, pos, q, N)) != Q2D_OK) return st;
        if ((st = k0_side(p, N)) != Q2D_OK) return st;
        if (p->n_exact > 0 &&
            (st = kmodes_run(p, N, (const int32_t *)p->exact_modes.p, p->exact_coef.p,
                             p->n_exact_pad, 0, p->n_exact, &nch)) != Q2D_OK)
            return st;
        if (hipStreamWaitEvent(p->stream, p->ev_k0, 0) != hipSuccess) return Q2D_EDEVICE;
    }
    st = epilogue(p, N, nch, p->diag_exact, true, phi, F, E);
    tstop(p, 4);
    return st;
}

// Whether work enqueued on the plan's stream now goes into a graph (a failed
// query counts as yes).  From the first such call on, the plan samples no
// modes ahead: a replay of the captured sampler writes the plan's mode
// buffers, one of which may hold modes sampled ahead for an eager call.
static bool capture_guard(Plan *p) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(p->stream, &cap) != hipSuccess) {
        (void)hipGetLastError();
        cap = hipStreamCaptureStatusActive;
    }
    if (cap == hipStreamCaptureStatusNone) return false;
    p->no_ahead = true;
    p->spec_ok = false;
    return true;
}

// The random-batch step after the argument checks (shared by q2d_rbm_step and
// its allocation-free variant).
static q2d_status rbm_step_body(q2d_plan_t p, const void *pos, const void *q, int64_t N,
                                int32_t P, uint64_t seed, uint64_t step, void *phi, void *F,
                                double *E, int32_t *modes_out) {
    q2d_status st;
    tstart(p, 4);
    const int p_pad = ((P + WAVE - 1) / WAVE) * WAVE;
    // Modes of this step sampled ahead by the previous call on this stream:
    // the main stream waited for that call's ev_k0, which follows them.
    SideExtra ex;
    ex.P = P;
    ex.modes_out = modes_out;
    const bool plain = !p->arena && !p->serial && !p->R && !capture_guard(p) && !p->no_ahead;
    ex.hit = plain && N > 0 && p->spec_ok && p->spec_seed == seed && p->spec_step == step &&
             p->spec_P == P && p->spec_stream == p->stream;
    ex.ahead = plain && N > 0;
    ex.seed = seed;
    ex.next_step = step + 1;
    if (ex.hit) {
        std::swap(p->rb_modes, p->sp_modes);
        std::swap(p->rb_coef, p->sp_coef);
    }
    if (plain) p->spec_ok = false;
    if (!ex.hit) {
        // the sampler runs on the side stream while the main stream sorts
        if (hipEventRecord(p->ev_fork, p->stream) != hipSuccess ||
            hipStreamWaitEvent(p->side, p->ev_fork, 0) != hipSuccess)
            return Q2D_EDEVICE;
        {
            SideScope side(p);
            if ((st = sample_modes(p, P, seed, step)) != Q2D_OK) return st;
            if (modes_out)
                k_modes_out<<<(P + 255) / 256, 256, 0, p->stream>>>(
                    (const int32_t *)p->rb_modes.p, P, p_pad, modes_out);
        }
        if (hipEventRecord(p->ev_modes, p->side) != hipSuccess) return Q2D_EDEVICE;
    }
    int nch = 0;
    if (N > 0) {
        if ((st = sort_and_stage(p, pos, q, N)) != Q2D_OK) return st;
        if ((st = k0_side(p, N, &ex)) != Q2D_OK) return st;
        if (ex.ahead) {
            p->spec_ok = true;
            p->spec_seed = seed;
            p->spec_step = step + 1;
            p->spec_P = P;
            p->spec_stream = p->stream;
        }
        if (!ex.hit && hipStreamWaitEvent(p->stream, p->ev_modes, 0) != hipSuccess)
            return Q2D_EDEVICE;
        if ((st = kmodes_run(p, N, (const int32_t *)p->rb_modes.p, p->rb_coef.p, p_pad, 0, P,
                             &nch)) != Q2D_OK)
            return st;
        if (hipStreamWaitEvent(p->stream, p->ev_k0, 0) != hipSuccess) return Q2D_EDEVICE;
    } else if (hipStreamWaitEvent(p->stream, p->ev_modes, 0) != hipSuccess) {
        return Q2D_EDEVICE;
    }
    st = epilogue(p, N, nch, p->diag_rb, true, phi, F, E);
    tstop(p, 4);
    return st;
}

static q2d_status check_rbm(q2d_plan_t p, const void *pos, const void *q, int64_t N, int32_t P) {
    q2d_status st = check_io(p, pos, q, N);
    if (st != Q2D_OK) return st;
    if (P < 1) return Q2D_EINVAL;
    if (p->opts.p_max <= 0) return Q2D_EUNSUPPORTED;
    if (P > p->opts.p_max) return Q2D_ECAPACITY;
    return Q2D_OK;
}

q2d_status q2d_rbm_step(q2d_plan_t p, const void *pos, const void *q, int64_t N, int32_t P,
                        uint64_t seed, uint64_t step, void *phi, void *F, double *E,
                        int32_t *modes_out) {
    const q2d_status st = check_rbm(p, pos, q, N, P);
    if (st != Q2D_OK) return st;
    return rbm_step_body(p, pos, q, N, P, seed, step, phi, F, E, modes_out);
}

// The allocation-free step: the same body with every scratch buffer of the
// call lent from the device's static array.  The requests are listed in the
// order the body ensures them (sampler, sort, inverse permutation and k = 0 on
// the internal stream, k != 0 passes, epilogue), so arena_need() is the exact
// number of bytes the call takes.
q2d_status q2d_rbm_step_noalloc(q2d_plan_t p, const void *pos, const void *q, int64_t N,
                                int32_t P, uint64_t seed, uint64_t step, void *phi, void *F,
                                double *E, int32_t *modes_out) {
    q2d_status st = check_rbm(p, pos, q, N, P);
    if (st != Q2D_OK) return st;
    char *base = noalloc_base(p->device);
    if (!base) return Q2D_EDEVICE;
    Reqs req;
    sampler_reqs(p, P, req);
    if (N > 0) {
        sort_reqs(p, N, req);
        inv_reqs(p, N, req);
        k0_reqs(p, N, req);
        kmodes_reqs(p, N, P, req);
        epilogue_reqs(p, N, req);
    }
    if (arena_need(req) > Q2D_NOALLOC_SCRATCH_BYTES) return Q2D_ECAPACITY;
    Arena a;
    a.base = base;
    a.cap = Q2D_NOALLOC_SCRATCH_BYTES;
    // timing events are not created inside this call
    const int timing = p->timing;
    p->timing = 0;
    p->arena = &a;
    st = rbm_step_body(p, pos, q, N, P, seed, step, phi, F, E, modes_out);
    p->arena = nullptr;
    p->timing = timing;
    arena_restore(a);
    if (st != Q2D_OK) {
        // work already enqueued on the internal stream ends before the
        // caller's stream goes on (the next call reuses the same memory)
        if (hipEventRecord(p->ev_k0, p->side) == hipSuccess)
            (void)hipStreamWaitEvent(p->stream, p->ev_k0, 0);
    }
    return st;
}

q2d_status q2d_long_range_vjp(q2d_plan_t p, const void *pos, const void *q, const void *g,
                              int64_t N, void *dq, void *dpos) {
    q2d_status st = check_io(p, pos, q, N);
    if (st != Q2D_OK) return st;
    if (N > 0 && !g) return Q2D_EINVAL;
    if (!(p->kc > 0)) return Q2D_EUNSUPPORTED;
    if (N == 0) return Q2D_OK;
    tstart(p, 4);
    if ((st = sort_and_stage(p, pos, q, N)) != Q2D_OK) return st;
    st = vjp_passes(p, N, (const int32_t *)p->exact_modes.p, p->exact_coef.p, p->n_exact_pad,
                    p->n_exact, p->diag_exact, g, dq, dpos);
    tstop(p, 4);
    return st;
}

q2d_status q2d_rbm_step_vjp(q2d_plan_t p, const void *pos, const void *q, const void *g,
                            int64_t N, int32_t P, uint64_t seed, uint64_t step, void *dq,
                            void *dpos) {
    q2d_status st = check_io(p, pos, q, N);
    if (st != Q2D_OK) return st;
    if (N > 0 && !g) return Q2D_EINVAL;
    if (P < 1) return Q2D_EINVAL;
    if (p->opts.p_max <= 0) return Q2D_EUNSUPPORTED;
    if (P > p->opts.p_max) return Q2D_ECAPACITY;
    if (N == 0) return Q2D_OK;
    (void)capture_guard(p);
    tstart(p, 4);
    const int p_pad = ((P + WAVE - 1) / WAVE) * WAVE;
    if (hipEventRecord(p->ev_fork, p->stream) != hipSuccess ||
        hipStreamWaitEvent(p->side, p->ev_fork, 0) != hipSuccess)
        return Q2D_EDEVICE;
    {
        SideScope side(p);
        if ((st = sample_modes(p, P, seed, step)) != Q2D_OK) return st;
    }
    if (hipEventRecord(p->ev_modes, p->side) != hipSuccess) return Q2D_EDEVICE;
    if ((st = sort_and_stage(p, pos, q, N)) != Q2D_OK) return st;
    if (hipStreamWaitEvent(p->stream, p->ev_modes, 0) != hipSuccess) return Q2D_EDEVICE;
    st = vjp_passes(p, N, (const int32_t *)p->rb_modes.p, p->rb_coef.p, p_pad, P, p->diag_rb, g,
                    dq, dpos);
    tstop(p, 4);
    return st;
}

q2d_status q2d_modes_eval(q2d_plan_t p, const void *pos, const void *q, int64_t N,
                          const int32_t *modes, const double *weights, int64_t n_modes, void *phi,
                          void *F, double *E) {
    q2d_status st = check_io(p, pos, q, N);
    if (st != Q2D_OK) return st;
    if (n_modes < 0 || (n_modes > 0 && (!modes || !weights)) || n_modes > ((int64_t)1 << 30))
        return Q2D_EINVAL;
    tstart(p, 4);
    int nch = 0;
    if (N > 0 && n_modes > 0) {
        const int64_t n_pad = ((n_modes + WAVE - 1) / WAVE) * WAVE;
        const size_t tsz = p->fp32 ? sizeof(float) : sizeof(double);
        if ((st = ensure(p, p->user_modes, (size_t)2 * n_pad * sizeof(int32_t))) != Q2D_OK ||
            (st = ensure(p, p->user_w, (size_t)n_pad * sizeof(double))) != Q2D_OK ||
            (st = ensure(p, p->user_coef, (size_t)coef_fields(p->mh) * n_pad * tsz)) != Q2D_OK)
            return st;
        k_user_modes<<<(int)((n_pad + 255) / 256), 256, 0, p->stream>>>(
            modes, weights, n_modes, n_pad, (int32_t *)p->user_modes.p, (double *)p->user_w.p);
        if ((st = build_mode_coefs(p, (const int32_t *)p->user_modes.p, n_modes, n_pad,
                                   (const double *)p->user_w.p, 0.0, p->user_coef.p)) != Q2D_OK)
            return st;
        if ((st = sort_and_stage(p, pos, q, N)) != Q2D_OK) return st;
        if ((st = kmodes_run(p, N, (const int32_t *)p->user_modes.p, p->user_coef.p, n_pad, 0,
                             n_modes, &nch)) != Q2D_OK)
            return st;
    } else if (N > 0) {
        if ((st = sort_and_stage(p, pos, q, N)) != Q2D_OK) return st;
    }
    st = epilogue(p, N, nch, 0.0, false, phi, F, E);
    tstop(p, 4);
    return st;
}

q2d_status q2d_short_range(q2d_plan_t p, const void *pos, const void *q, int64_t N, void *phi,
                           void *F, double *E) {
    q2d_status st = check_io(p, pos, q, N);
    if (st != Q2D_OK) return st;
    if (!(p->rc > 0)) return Q2D_EUNSUPPORTED;
    if (N == 0) return epilogue(p, 0, 0, 0.0, true, nullptr, nullptr, E);
    return short_range_run(p, pos, q, N, phi, F, E);
}

q2d_status q2d_plan_check(q2d_plan_t p) {
    if (!p) return Q2D_EINVAL;
    return plan_check(p);
}

}  // extern "C"

namespace q2d {

q2d_status plan_check(Plan *p) {
    if (hipSetDevice(p->device) != hipSuccess) return Q2D_EDEVICE;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return Q2D_EDEVICE;
    int bits = 0;
    if (hipMemcpy(&bits, p->status.p, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return Q2D_EDEVICE;
    k_zero_status<<<1, 1, 0, p->stream>>>((int *)p->status.p, (double *)((char *)p->status.p + 16));
    if (hipStreamSynchronize(p->stream) != hipSuccess) return Q2D_EDEVICE;
    return (q2d_status)first_error(bits);
}

}  // namespace q2d

extern "C" {

q2d_status q2d_plan_timing_enable(q2d_plan_t p, int32_t mask) {
    if (!p) return Q2D_EINVAL;
    timing_flush(p);
    for (int w = 0; w < 5; ++w) {
        p->t_ms[w] = 0;
        p->t_cnt[w] = 0;
    }
    p->timing = mask & 31;
    return Q2D_OK;
}

q2d_status q2d_plan_timing_stride(q2d_plan_t p, int32_t n) {
    if (!p || n < 1) return Q2D_EINVAL;
    p->timing_stride = n;
    p->ncalls = 0;
    return Q2D_OK;
}

q2d_status q2d_plan_timing_read(q2d_plan_t p, int32_t which, double *ms_total, int64_t *count) {
    if (!p || which < 0 || which > 4 || !ms_total || !count) return Q2D_EINVAL;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return Q2D_EDEVICE;
    timing_flush(p);
    *ms_total = p->t_ms[which];
    *count = p->t_cnt[which];
    return Q2D_OK;
}

}  // extern "C"
