// Fourier-mode tables: per-mode SOE coefficients and the random-batch sampler.
//
// Coefficients (Sec. 3.2, eq. SOEphi; App. E, eq. z-der).  For a mode k with
// |k| = k the pair kernel without its Gaussian factor is
//   K_k(z) = (2 alpha/(sqrt(pi) k)) sum_l w_l (2 beta_l e^{-kz} - 2k e^{-beta_l z}) / (beta_l^2 - k^2)
//          = a_k e^{-kz} + sum_l a_l e^{-beta_l z},   beta_l = alpha s_l,
// so with c_l = (2 alpha/(sqrt(pi) k)) w_l / (beta_l^2 - k^2):
//   a_k = Re sum_l 2 beta_l c_l,   a_l = -2 k c_l,
// and its derivative K'_k(z) = -k a_k e^{-kz} + sum_l (2 k beta_l c_l) e^{-beta_l z}.
// Conjugate SOE terms give conjugate scans for real inputs, so each pair is
// carried once with doubled coefficients (the sum of a term and its conjugate
// is twice its real part).
//
// Sampler (Sec. 4.1 and App. G): importance sampling of k != 0 from
// h(k) = exp(-k^2/(4 alpha^2))/H by an independence Metropolis chain whose
// proposal rounds a Gaussian draw m* ~ N(0, (alpha L)^2/(2 pi^2)) per axis;
// random numbers from Philox4x32-10.  Proposals are independent of the chain
// state, so they are drawn in parallel and only the accept/reject walk runs
// sequentially.
#include <cmath>

#include "q2d_internal.h"

namespace q2d {

namespace {

// Replica batches (boxes != null): work-group row blockIdx.y = replica r, with
// its own box, mode table (modes + r 2 n_pad) and coefficient table
// (coef + r nf n_pad), and weight (pi/A_r) H_r / P.
template <typename T>
__global__ __launch_bounds__(256) void k_mode_coefs(const int32_t *__restrict__ modes, int64_t n,
                                                    int64_t n_pad, const double *weights,
                                                    double weight_const, PairParams pp,
                                                    double alpha, double Lx, double Ly,
                                                    T *__restrict__ coef,
                                                    const double *__restrict__ boxes,
                                                    const double *__restrict__ rep_H, int P) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_pad) return;
    const int nf = 6 + 4 * pp.mh;
    if (boxes) {
        const int r = blockIdx.y;
        Lx = boxes[3 * r];
        Ly = boxes[3 * r + 1];
        weight_const = 3.14159265358979323846 / (Lx * Ly) * rep_H[r] / P;
        modes += (int64_t)r * 2 * n_pad;
        coef += (int64_t)r * nf * n_pad;
    }
    if (m >= n) {
        for (int f = 0; f < nf; ++f) coef[f * n_pad + m] = (T)0;
        return;
    }
    const double PI = 3.14159265358979323846;
    const double kx = 2.0 * PI * modes[m] / Lx;
    const double ky = 2.0 * PI * modes[n_pad + m] / Ly;
    const double k = sqrt(kx * kx + ky * ky);
    const double om = weights ? weights[m] : weight_const;
    const double pre = 2.0 * alpha / (sqrt(PI) * k);
    double ak = 0.0;
    for (int l = 0; l < pp.m_all; ++l) {
        const cx<double> b{pp.b_re[l], pp.b_im[l]};
        const cx<double> w{pp.w_re[l], pp.w_im[l]};
        cx<double> den = cmul(b, b);
        den.re -= k * k;
        // c = pre * w / den
        const double dd = den.re * den.re + den.im * den.im;
        const cx<double> wd{(w.re * den.re + w.im * den.im) / dd, (w.im * den.re - w.re * den.im) / dd};
        const cx<double> c{pre * wd.re, pre * wd.im};
        const cx<double> bc = cmul(b, c);
        ak += 2.0 * bc.re;
        const int r = pp.rep_of[l];
        if (r >= 0) {
            // pair representative: doubled a_l = -2 k c and doubled 2 k beta c
            coef[(6 + 4 * r + 0) * n_pad + m] = (T)(2.0 * (-2.0 * k * c.re));
            coef[(6 + 4 * r + 1) * n_pad + m] = (T)(2.0 * (-2.0 * k * c.im));
            coef[(6 + 4 * r + 2) * n_pad + m] = (T)(2.0 * (2.0 * k * bc.re));
            coef[(6 + 4 * r + 3) * n_pad + m] = (T)(2.0 * (2.0 * k * bc.im));
        }
    }
    coef[0 * n_pad + m] = (T)kx;
    coef[1 * n_pad + m] = (T)ky;
    coef[2 * n_pad + m] = (T)k;
    coef[3 * n_pad + m] = (T)om;
    coef[4 * n_pad + m] = (T)ak;
    coef[5 * n_pad + m] = (T)(-k * ak);
}

// proposal probability of one axis (App. G), as differences of erfc in the tails
__device__ inline double q_axis(int m, double aL) {
    const double PI = 3.14159265358979323846;
    const int am = m < 0 ? -m : m;
    if (am == 0) return erf(PI / (2.0 * aL));
    return 0.5 * (erfc(PI * (2 * am - 1) / (2.0 * aL)) - erfc(PI * (2 * am + 1) / (2.0 * aL)));
}

// target over proposal, unnormalised; 0 at m = (0, 0)
__device__ inline double mh_weight(int mx, int my, double alpha, double Lx, double Ly) {
    if (mx == 0 && my == 0) return 0.0;
    const double PI = 3.14159265358979323846;
    const double kx = 2.0 * PI * mx / Lx, ky = 2.0 * PI * my / Ly;
    const double h = exp(-(kx * kx + ky * ky) / (4.0 * alpha * alpha));
    return h / (q_axis(mx, alpha * Lx) * q_axis(my, alpha * Ly));
}

constexpr int SAMPLER_RESERVE = 64;
constexpr int SAMPLER_LDS = 2048;  // proposals staged in LDS for the walk

// Philox key of replica r of a batch: the batch seed advanced r times by the
// 64-bit golden-ratio increment (replica 0 draws exactly like one system)
__host__ __device__ inline uint64_t replica_seed(uint64_t seed, int r) {
    return seed + (uint64_t)r * 0x9E3779B97F4A7C15ull;
}

// One block per system: parallel proposals, then the sequential accept/reject
// walk.  Replica batches (boxes != null): block r uses replica r's box and
// seed and its own slices of the work arrays and of the mode table.
__global__ __launch_bounds__(1024) void k_sample(int P, int D, uint64_t seed, uint64_t step,
                                                 double alpha, double Lx, double Ly,
                                                 int32_t *__restrict__ prop,
                                                 double *__restrict__ wgt,
                                                 double *__restrict__ uacc,
                                                 int32_t *__restrict__ modes, int p_pad,
                                                 int *status, const double *__restrict__ boxes,
                                                 const uint64_t *__restrict__ step_dev) {
    const int n = SAMPLER_RESERVE + P * D;
    if (step_dev) step = step_dev[0];  // captured step: the number is read on the device
    if (boxes) {
        const int r = blockIdx.x;
        Lx = boxes[3 * r];
        Ly = boxes[3 * r + 1];
        seed = replica_seed(seed, r);
        prop += (int64_t)r * 2 * n;
        wgt += (int64_t)r * n;
        uacc += (int64_t)r * n;
        modes += (int64_t)r * 2 * p_pad;
    }
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t s0 = (uint32_t)step, s1 = (uint32_t)(step >> 32);
    const double PI = 3.14159265358979323846;
    const double sx = alpha * Lx / (PI * sqrt(2.0)), sy = alpha * Ly / (PI * sqrt(2.0));
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        uint32_t c[4] = {(uint32_t)e, s0, s1, 0u};
        philox10(c, k0, k1);
        const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
        const double R = sqrt(-2.0 * log(u1));
        const double n1 = R * cos(2.0 * PI * u2), n2 = R * sin(2.0 * PI * u2);
        const int mx = (int)floor(sx * n1 + 0.5), my = (int)floor(sy * n2 + 0.5);
        uint32_t a[4] = {(uint32_t)e, s0, s1, 1u};
        philox10(a, k0, k1);
        prop[2 * e] = mx;
        prop[2 * e + 1] = my;
        wgt[e] = mh_weight(mx, my, alpha, Lx, Ly);
        uacc[e] = u53(a[0], a[1]);
    }
    __syncthreads();
    // the sequential walk reads the proposals from LDS
    __shared__ int32_t lx[SAMPLER_LDS], ly[SAMPLER_LDS];
    __shared__ double lw[SAMPLER_LDS], lu[SAMPLER_LDS];
    const bool in_lds = n <= SAMPLER_LDS;
    if (in_lds) {
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            lx[e] = prop[2 * e];
            ly[e] = prop[2 * e + 1];
            lw[e] = wgt[e];
            lu[e] = uacc[e];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && in_lds) {
        int e0 = -1;
        for (int e = 0; e < SAMPLER_RESERVE; ++e)
            if (lx[e] != 0 || ly[e] != 0) {
                e0 = e;
                break;
            }
        if (e0 < 0) {
            atomicOr(status, 1 << Q2D_ESAMPLER);
            e0 = 0;
        }
        int cx_ = lx[e0], cy_ = ly[e0];
        double wc = lw[e0];
        for (int t = 1; t <= P * D; ++t) {
            const int e = e0 + t;
            if (lu[e] < lw[e] / wc) {
                cx_ = lx[e];
                cy_ = ly[e];
                wc = lw[e];
            }
            if (t % D == 0) {
                const int pidx = t / D - 1;
                modes[pidx] = cx_;
                modes[p_pad + pidx] = cy_;
            }
        }
    }
    if (threadIdx.x == 0 && !in_lds) {
        int e0 = -1;
        for (int e = 0; e < SAMPLER_RESERVE; ++e)
            if (prop[2 * e] != 0 || prop[2 * e + 1] != 0) {
                e0 = e;
                break;
            }
        if (e0 < 0) {
            atomicOr(status, 1 << Q2D_ESAMPLER);
            e0 = 0;
        }
        int cx_ = prop[2 * e0], cy_ = prop[2 * e0 + 1];
        double wc = wgt[e0];
        for (int t = 1; t <= P * D; ++t) {
            const int e = e0 + t;
            if (uacc[e] < wgt[e] / wc) {
                cx_ = prop[2 * e];
                cy_ = prop[2 * e + 1];
                wc = wgt[e];
            }
            if (t % D == 0) {
                const int pidx = t / D - 1;
                modes[pidx] = cx_;
                modes[p_pad + pidx] = cy_;
            }
        }
    }
    __syncthreads();
    // padding modes
    for (int i = P + threadIdx.x; i < p_pad; i += blockDim.x) {
        modes[i] = 0;
        modes[p_pad + i] = 0;
    }
}

// Exact i.i.d. draws from h(k) over k != 0 (the alternative to the chain of
// App. G).  h factorises into g_x(m_x) g_y(m_y) with g(m) = e^{-(pi m/(alpha L))^2};
// draw i inverts two cumulative tables with the two 53-bit uniforms of one
// Philox block (counter (i, step, stream 2)): m_x from its marginal given
// m != (0, 0) (weights g_x(m) (Z_y - [m = 0])), then m_y from g_y, or from g_y
// without m_y = 0 when m_x = 0.  tab = [cdf_x (2 mxm + 1)][cdf_y (2 mym + 1)]
// [cdf_y without 0 (2 mym + 1)].
__device__ inline int first_at_least(const double *c, int n, double u) {
    int lo = 0, hi = n - 1;  // c[n - 1] = 1 > u
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] >= u)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_sample_iid(int P, uint64_t seed, uint64_t step,
                                                    const double *__restrict__ tab, int mxm,
                                                    int mym, int32_t *__restrict__ modes,
                                                    int p_pad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p_pad) return;
    if (i >= P) {
        modes[i] = 0;
        modes[p_pad + i] = 0;
        return;
    }
    uint32_t c[4] = {(uint32_t)i, (uint32_t)step, (uint32_t)(step >> 32), 2u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const int nx = 2 * mxm + 1, ny = 2 * mym + 1;
    const int mx = first_at_least(tab, nx, u53(c[0], c[1])) - mxm;
    const double *cy = tab + nx + (mx == 0 ? ny : 0);
    const int my = first_at_least(cy, ny, u53(c[2], c[3])) - mym;
    modes[i] = mx;
    modes[p_pad + i] = my;
}

}  // namespace

// Cumulative tables of the i.i.d. sampler (host, FP64), in the layout
// k_sample_iid reads; axis ranges |m| <= mxm, mym cover g(m) >= 1e-18.
void iid_tables(double alpha, double Lx, double Ly, std::vector<double> &tab, int *mxm, int *mym) {
    const double PI = 3.14159265358979323846;
    const double kmax = 2.0 * alpha * std::sqrt(std::log(1e18));
    *mxm = (int)std::ceil(kmax * Lx / (2 * PI));
    *mym = (int)std::ceil(kmax * Ly / (2 * PI));
    auto g = [&](int m, double L) {
        const double t = PI * m / (alpha * L);
        return std::exp(-t * t);
    };
    double zy = 0.0;
    for (int m = -*mym; m <= *mym; ++m) zy += g(m, Ly);
    auto cumulate = [&](int mm, auto wfun) {
        const size_t b = tab.size();
        double run = 0.0;
        for (int m = -mm; m <= mm; ++m) {
            run += wfun(m);
            tab.push_back(run);
        }
        for (size_t j = b; j < tab.size(); ++j) tab[j] /= run;
    };
    tab.clear();
    cumulate(*mxm, [&](int m) { return g(m, Lx) * (m == 0 ? zy - 1.0 : zy); });
    cumulate(*mym, [&](int m) { return g(m, Ly); });
    cumulate(*mym, [&](int m) { return m == 0 ? 0.0 : g(m, Ly); });
}

q2d_status build_mode_coefs(Plan *p, const int32_t *modes, int64_t n, int64_t n_pad,
                            const double *weights_dev, double weight_const, void *coef) {
    if (n_pad <= 0) return Q2D_OK;
    const int nb = (int)((n_pad + 255) / 256);
    if (p->fp32)
        k_mode_coefs<float><<<nb, 256, 0, p->stream>>>(modes, n, n_pad, weights_dev, weight_const,
                                                       p->pp, p->alpha, p->Lx, p->Ly,
                                                       (float *)coef, nullptr, nullptr, 0);
    else
        k_mode_coefs<double><<<nb, 256, 0, p->stream>>>(modes, n, n_pad, weights_dev,
                                                        weight_const, p->pp, p->alpha, p->Lx,
                                                        p->Ly, (double *)coef, nullptr, nullptr, 0);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

void sampler_reqs(Plan *p, int P, Reqs &q) {
    const int p_pad = ((P + WAVE - 1) / WAVE) * WAVE;
    const size_t tsz = p->fp32 ? sizeof(float) : sizeof(double);
    if (p->opts.sampler != Q2D_SAMPLER_IID) {
        const int D = p->opts.thin > 0 ? p->opts.thin : 1;
        const int n = SAMPLER_RESERVE + P * D;
        q.add(p->rb_work, (size_t)n * (2 * sizeof(int32_t) + 2 * sizeof(double)));
    }
    q.add(p->rb_modes, (size_t)2 * p_pad * sizeof(int32_t));
    q.add(p->rb_coef, (size_t)coef_fields(p->mh) * p_pad * tsz);
}

q2d_status sample_modes(Plan *p, int P, uint64_t seed, uint64_t step, int *status) {
    const double PI = 3.14159265358979323846;
    Reqs req;
    sampler_reqs(p, P, req);
    q2d_status st;
    if ((st = ensure_all(p, req)) != Q2D_OK) return st;
    if (p->opts.sampler == Q2D_SAMPLER_IID) {
        const int p_pad = ((P + WAVE - 1) / WAVE) * WAVE;
        k_sample_iid<<<(p_pad + 255) / 256, 256, 0, p->stream>>>(
            P, seed, step, (const double *)p->iid_tab.p, p->iid_mxm, p->iid_mym,
            (int32_t *)p->rb_modes.p, p_pad);
        if (hipGetLastError() != hipSuccess) return Q2D_EDEVICE;
        return build_mode_coefs(p, (const int32_t *)p->rb_modes.p, P, p_pad, nullptr,
                                PI / (p->Lx * p->Ly) * p->H / P, p->rb_coef.p);
    }
    const int D = p->opts.thin > 0 ? p->opts.thin : 1;
    const int n = SAMPLER_RESERVE + P * D;
    const int p_pad = ((P + WAVE - 1) / WAVE) * WAVE;
    int32_t *prop = (int32_t *)p->rb_work.p;
    double *wgt = (double *)((char *)p->rb_work.p + (size_t)n * 2 * sizeof(int32_t));
    double *uacc = wgt + n;
    k_sample<<<1, 1024, 0, p->stream>>>(P, D, seed, step, p->alpha, p->Lx, p->Ly, prop, wgt, uacc,
                                         (int32_t *)p->rb_modes.p, p_pad,
                                         status ? status : (int *)p->status.p, nullptr, nullptr);
    if (hipGetLastError() != hipSuccess) return Q2D_EDEVICE;
    return build_mode_coefs(p, (const int32_t *)p->rb_modes.p, P, p_pad, nullptr,
                            PI / (p->Lx * p->Ly) * p->H / P, p->rb_coef.p);
}

__global__ void k_word_zero(int *a) { *a = 0; }

// The next step's modes, sampled ahead into the second buffers (swapped with
// rb_modes / rb_coef around the sampler, which also fills them), with its own
// status word: a step never asked for must not raise the plan's status.
q2d_status sample_modes_ahead(Plan *p, int P, uint64_t seed, uint64_t step) {
    q2d_status st;
    if ((st = ensure(p, p->sp_status, sizeof(int))) != Q2D_OK) return st;
    k_word_zero<<<1, 1, 0, p->stream>>>((int *)p->sp_status.p);
    std::swap(p->rb_modes, p->sp_modes);
    std::swap(p->rb_coef, p->sp_coef);
    st = sample_modes(p, P, seed, step, (int *)p->sp_status.p);
    std::swap(p->rb_modes, p->sp_modes);
    std::swap(p->rb_coef, p->sp_coef);
    return st;
}

q2d_status sample_modes_batch(Plan *p, int P, uint64_t seed, uint64_t step,
                              const uint64_t *step_dev) {
    const int D = p->opts.thin > 0 ? p->opts.thin : 1;
    const int n = SAMPLER_RESERVE + P * D;
    const int p_pad = ((P + WAVE - 1) / WAVE) * WAVE;
    const int nf = coef_fields(p->mh);
    const size_t tsz = p->fp32 ? sizeof(float) : sizeof(double);
    q2d_status st;
    if ((st = ensure(p, p->rb_work,
                     (size_t)p->R * n * (2 * sizeof(int32_t) + 2 * sizeof(double)))) != Q2D_OK)
        return st;
    if ((st = ensure(p, p->rb_modes, (size_t)p->R * 2 * p_pad * sizeof(int32_t))) != Q2D_OK)
        return st;
    if ((st = ensure(p, p->rb_coef, (size_t)p->R * nf * p_pad * tsz)) != Q2D_OK) return st;
    int32_t *prop = (int32_t *)p->rb_work.p;
    double *wgt = (double *)((char *)p->rb_work.p + (size_t)p->R * n * 2 * sizeof(int32_t));
    double *uacc = wgt + (size_t)p->R * n;
    const double *boxes = (const double *)p->rep_box.p;
    k_sample<<<p->R, 1024, 0, p->stream>>>(P, D, seed, step, p->alpha, 0.0, 0.0, prop, wgt, uacc,
                                            (int32_t *)p->rb_modes.p, p_pad, (int *)p->status.p,
                                            boxes, step_dev);
    const dim3 grid((p_pad + 255) / 256, p->R);
    if (p->fp32)
        k_mode_coefs<float><<<grid, 256, 0, p->stream>>>(
            (const int32_t *)p->rb_modes.p, P, p_pad, nullptr, 0.0, p->pp, p->alpha, 0.0, 0.0,
            (float *)p->rb_coef.p, boxes, (const double *)p->rep_H.p, P);
    else
        k_mode_coefs<double><<<grid, 256, 0, p->stream>>>(
            (const int32_t *)p->rb_modes.p, P, p_pad, nullptr, 0.0, p->pp, p->alpha, 0.0, 0.0,
            (double *)p->rb_coef.p, boxes, (const double *)p->rep_H.p, P);
    p->rep_mstride = 2 * (int64_t)p_pad;
    p->rep_cstride = (int64_t)nf * p_pad;
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

}  // namespace q2d
