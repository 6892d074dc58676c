// The k = 0 Fourier term, always evaluated exactly (SOE form) in FP64.
//
// Pair kernel (Sec. 3.2, eq. 32) and its derivative (App. E, eq. dzphi_0):
//   K_0(z)  = sum_l (w_l/sqrt(pi)) [2z/s_l + (1/alpha - 2z/s_l) e^{-beta_l z}]
//   K_0'(z) = sum_l (w_l/sqrt(pi)) [2/s_l - (s_l + 2/s_l - 2 alpha z) e^{-beta_l z}]
//   phi^0_i = -(2 pi/A) sum_j q_j K_0(|z_ij|)   (j = i included: K_0(0))
//   F^0_z,i = (2 pi/A) q_i sum_{j != i} q_j sgn(z_i - z_j) K_0'(|z_ij|)
// The kernels take the sources q_j as an array (the charges, or the adjoint
// weights) and store phi^0 and the field F^0_z,i / q_i.
// The z e^{-beta z} terms are split as z_ij e^{-beta z_ij} = z_i e^{..} - z_j e^{..}
// (j below i), so every term is a plain decayed scan of one of two real
// sources, q_j and q_j z_j; the linear terms are the beta = 0 scans (prefix
// sums).  Conjugate SOE terms are carried once with doubled coefficients.
//
// Layout: segments of S0 = 64 consecutive sorted particles (S0 divides every
// replica-batch segment, so no k = 0 segment straddles two replicas).  A lane
// works on one (segment, pair): a wave holds 64 / LG segments of LG pair
// lanes each (LG = 8 for up to 8 pairs, else 16), the segment's heights and
// sources staged in LDS and read as broadcasts.  The linear (beta = 0) terms
// ride along on pair lane 0.  Per-particle sums over the pairs use a register
// reduce-scatter inside each lane group (every LG steps, fixed order), so the
// results are deterministic.  Segment aggregates and carries use the same
// FP64 carry scan as the k != 0 modes.
#include "q2d_internal.h"

namespace q2d {

q2d_status carry_k0(Plan *p, int nseg, int S, int64_t N);

namespace {

constexpr int S0 = 64;
constexpr int ZP = S0 + 1;  // padded LDS rows: the segment groups hit distinct banks

// sum_{k <= ND} (-x)^k / k! by Horner in -x (x = ar + i ai)
template <int ND>
__device__ inline cx<double> expm_taylor(double ar, double ai) {
    constexpr double inv_fact[8] = {1.0,         1.0,         1.0 / 2,     1.0 / 6,
                                    1.0 / 24,    1.0 / 120,   1.0 / 720,   1.0 / 5040};
    double pr = inv_fact[ND], pi = 0.0;
#pragma unroll
    for (int k = ND - 1; k >= 0; --k) {
        const double nr = -(pr * ar - pi * ai), ni = -(pr * ai + pi * ar);
        pr = nr + inv_fact[k];
        pi = ni;
    }
    return {pr, pi};
}

// e^{-(br + i bi) t}.  Small arguments r = |ar| + |ai| (dense particles) use a
// Taylor polynomial whose remainder r^{n+1}/(n+1)! stays below 1e-17:
// degree 4 for r < 2^-10, degree 7 for r < 2^-6.
__device__ inline cx<double> cexpm64(double br, double bi, double t) {
    const double ar = br * t, ai = bi * t;
    const double r = fabs(ar) + fabs(ai);
    if (r < 0x1p-10) return expm_taylor<4>(ar, ai);
    if (r < 0x1p-6) return expm_taylor<7>(ar, ai);
    const double m = exp(-ar);
    double s, c;
    sincos(ai, &s, &c);
    return {m * c, -m * s};
}

// agg0 layout: [dir][seg][slot][input] complex double, slot mh = linear (beta 0)
__device__ inline int64_t a0_idx(int nseg, int ns, int dir, int seg, int slot, int inp) {
    return (((int64_t)dir * nseg + seg) * ns + slot) * 2 + inp;
}

template <typename T, int LG>
struct K0Lds {
    static constexpr int G = WAVE / LG;  // segments per wave
    T z[G][ZP], q[G][ZP];                // inputs in their own precision
    double ph[G][ZP], fz[G][ZP];
    double rb[G][LG][LG + 1];            // per-group reduction rows [step][pair lane]
    // pair coefficients: beta (re, im), then c0u, c0v, f0u, f0v (re, im) per pair
    double cf[10][MAX_PAIRS];
};

// the aggregate kernel's LDS: heights, sources and the pair exponents only
// (a third of the sweep's, so that it runs at its register-limited occupancy)
template <typename T, int LG>
struct K0AggLds {
    static constexpr int G = WAVE / LG;
    T z[G][ZP], q[G][ZP];
    double br[MAX_PAIRS], bi[MAX_PAIRS];
};

// the pair tables, copied with uniform indices (a lane-dependent index into
// the kernel-argument struct would compile to select chains over all entries)
template <typename T, int LG>
__device__ inline void k0_coefs(const PairParams &pp, K0Lds<T, LG> &L) {
    if (threadIdx.x == 0) {
        for (int l = 0; l < pp.mh; ++l) {
            L.cf[0][l] = pp.beta_re[l];
            L.cf[1][l] = pp.beta_im[l];
            L.cf[2][l] = pp.c0u_re[l];
            L.cf[3][l] = pp.c0u_im[l];
            L.cf[4][l] = pp.c0v_re[l];
            L.cf[5][l] = pp.c0v_im[l];
            L.cf[6][l] = pp.f0u_re[l];
            L.cf[7][l] = pp.f0u_im[l];
            L.cf[8][l] = pp.f0v_re[l];
            L.cf[9][l] = pp.f0v_im[l];
        }
    }
}

// heights and sources of the wave's segments (zero past N)
template <typename T, int G, typename LDS>
__device__ inline void k0_stage(const T *__restrict__ zs, const T *__restrict__ qs, int64_t N,
                                int seg0, LDS &L) {
    for (int e = threadIdx.x; e < G * S0; e += WAVE) {
        const int g = e / S0, j = e % S0;
        const int64_t i = (int64_t)(seg0 + g) * S0 + j;
        L.z[g][j] = i < N ? zs[i] : (T)0;
        L.q[g][j] = i < N ? qs[i] : (T)0;
    }
    __syncthreads();
}

// Sum v[t] over the LG pair lanes of a group; lane l of the group gets the sum
// for t = l.  Through LDS rows (a register butterfly with lane-dependent
// selects is turned by the compiler into dynamic indexing); the pair lanes are
// added in a fixed order.  The work-group is one wave.
template <int LG>
__device__ inline double group_sum(const double (&v)[LG], double (*rb)[LG + 1], int l) {
#pragma unroll
    for (int t = 0; t < LG; ++t) rb[t][l] = v[t];
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < LG; ++u) s += rb[l][u];
    __syncthreads();
    return s;
}

// Segment aggregates, and the spans of the k = 0 carry scan: W = e^{-beta
// (z_last - z_first)}, G = e^{-beta (z_first(next) - z_last)} per (segment,
// pair), the same values the k != 0 spans kernel forms for its segments.
template <typename T, int LG>
__global__ __launch_bounds__(WAVE) void k0_agg(const T *__restrict__ zs, const T *__restrict__ qs,
                                               int64_t N, int nseg, PairParams pp,
                                               cx<double> *__restrict__ agg,
                                               cx<double> *__restrict__ spans) {
    constexpr int G = K0AggLds<T, LG>::G;
    __shared__ K0AggLds<T, LG> L;
    const int g = threadIdx.x / LG, l = threadIdx.x % LG;
    const int seg0 = blockIdx.x * G, seg = seg0 + g;
    if (threadIdx.x == 0) {
        for (int k = 0; k < pp.mh; ++k) {
            L.br[k] = pp.beta_re[k];
            L.bi[k] = pp.beta_im[k];
        }
    }
    k0_stage<T, G>(zs, qs, N, seg0, L);
    if (seg >= nseg) return;
    const int n = (int)min((int64_t)S0, N - (int64_t)seg * S0);
    const int ns = pp.mh + 1;
    const T *z = L.z[g], *q = L.q[g];
    if (l < pp.mh) {
        const double br = L.br[l], bi = L.bi[l];
        const double zf = (double)z[0], zl = (double)z[n - 1];
        const double zn = seg + 1 < nseg ? (double)zs[(int64_t)(seg + 1) * S0] : zl;
        spans[((int64_t)seg * pp.mh + l) * 2] = span_decay(br, bi, zl - zf);
        spans[((int64_t)seg * pp.mh + l) * 2 + 1] = span_decay(br, bi, zn - zl);
        // forward: referenced to the segment's last particle; backward: to its first
        cx<double> fq{0, 0}, fz{0, 0}, bq{0, 0}, bz{0, 0}, e{1, 0};
        for (int j = 0; j < n; ++j) {
            const cx<double> d = j ? cexpm64(br, bi, z[j] - z[j - 1]) : cx<double>{1, 0};
            const double qz = q[j] * z[j];
            fq = cmul(fq, d);
            fz = cmul(fz, d);
            fq.re += q[j];
            fz.re += qz;
            e = cmul(e, d);
            bq.re += q[j] * e.re;
            bq.im += q[j] * e.im;
            bz.re += qz * e.re;
            bz.im += qz * e.im;
        }
        agg[a0_idx(nseg, ns, 0, seg, l, 0)] = fq;
        agg[a0_idx(nseg, ns, 0, seg, l, 1)] = fz;
        agg[a0_idx(nseg, ns, 1, seg, l, 0)] = bq;
        agg[a0_idx(nseg, ns, 1, seg, l, 1)] = bz;
    }
    if (l == 0) {
        double sq = 0, sz = 0;
        for (int j = 0; j < n; ++j) {
            sq += q[j];
            sz += q[j] * z[j];
        }
        agg[a0_idx(nseg, ns, 0, seg, pp.mh, 0)] = cx<double>{sq, 0};
        agg[a0_idx(nseg, ns, 0, seg, pp.mh, 1)] = cx<double>{sz, 0};
        agg[a0_idx(nseg, ns, 1, seg, pp.mh, 0)] = cx<double>{sq, 0};
        agg[a0_idx(nseg, ns, 1, seg, pp.mh, 1)] = cx<double>{sz, 0};
    }
}

template <typename T, int LG>
__global__ __launch_bounds__(WAVE) void k0_sweep(const T *__restrict__ zs,
                                                 const T *__restrict__ qs, int64_t N, int nseg,
                                                 PairParams pp, double c_lin, double k0_self,
                                                 double two_pi_over_A,
                                                 const cx<double> *__restrict__ agg,
                                                 double *__restrict__ phi0,
                                                 double *__restrict__ fz0,
                                                 const double *__restrict__ rep_tpa,
                                                 const int32_t *__restrict__ seg_rep,
                                                 int seg_div) {
    constexpr int G = K0Lds<T, LG>::G;
    __shared__ K0Lds<T, LG> L;
    const int g = threadIdx.x / LG, l = threadIdx.x % LG;
    const int seg0 = blockIdx.x * G, seg = seg0 + g;
    k0_coefs<T, LG>(pp, L);
    k0_stage<T, G>(zs, qs, N, seg0, L);
    const int n = seg < nseg ? (int)min((int64_t)S0, N - (int64_t)seg * S0) : 0;
    const int ns = pp.mh + 1;
    const bool act = n > 0 && l < pp.mh;
    const T *z = L.z[g], *q = L.q[g];
    // pair l (zero coefficients on idle lanes); the linear terms count on lane 0 only
    const int lc = act ? l : 0;
    const double br = L.cf[0][lc], bi = L.cf[1][lc];
    const double on = act ? 1.0 : 0.0;
    const cx<double> cu{on * L.cf[2][lc], on * L.cf[3][lc]};
    const cx<double> cv{on * L.cf[4][lc], on * L.cf[5][lc]};
    const cx<double> fu{on * L.cf[6][lc], on * L.cf[7][lc]};
    const cx<double> fv{on * L.cf[8][lc], on * L.cf[9][lc]};
    const double lw = (l == 0 && n > 0) ? c_lin : 0.0;
    const int sg = n > 0 ? seg : 0;
    // forward: U = sum_{j<i} q_j e^{..}, W = sum_{j<i} q_j z_j e^{..}, V = z_i U - W;
    // linear: Q, Z = sums of q and q z below
    cx<double> pq{0, 0}, pz{0, 0};
    if (act) {
        pq = agg[a0_idx(nseg, ns, 0, sg, l, 0)];
        pz = agg[a0_idx(nseg, ns, 0, sg, l, 1)];
    }
    double Q = n > 0 ? agg[a0_idx(nseg, ns, 0, sg, pp.mh, 0)].re : 0.0;
    double Z = n > 0 ? agg[a0_idx(nseg, ns, 0, sg, pp.mh, 1)].re : 0.0;
    for (int c0 = 0; c0 < S0; c0 += LG) {
        double vp[LG], vf[LG];
#pragma unroll
        for (int t = 0; t < LG; ++t) {
            const int j = c0 + t;
            vp[t] = vf[t] = 0.0;
            if (j < n) {
                const cx<double> d = j ? cexpm64(br, bi, z[j] - z[j - 1]) : cx<double>{1, 0};
                const cx<double> U = cmul(pq, d), W = cmul(pz, d);
                const cx<double> V{z[j] * U.re - W.re, z[j] * U.im - W.im};
                vp[t] = cu.re * U.re - cu.im * U.im + cv.re * V.re - cv.im * V.im +
                        lw * (z[j] * Q - Z);
                vf[t] = fu.re * U.re - fu.im * U.im + fv.re * V.re - fv.im * V.im + lw * Q;
                pq = cx<double>{U.re + q[j], U.im};
                pz = cx<double>{W.re + q[j] * z[j], W.im};
                Q += q[j];
                Z += q[j] * z[j];
            }
        }
        const double sp = group_sum<LG>(vp, L.rb[g], l);
        const double sf = group_sum<LG>(vf, L.rb[g], l);
        L.ph[g][c0 + l] = sp;
        L.fz[g][c0 + l] = sf;
    }
    // backward: U = sum_{j>i} q_j e^{..}, W = sum_{j>i} q_j z_j e^{..}, V = W - z_i U;
    // linear: Q, Z = sums above
    pq = pz = cx<double>{0, 0};
    if (act) {
        pq = agg[a0_idx(nseg, ns, 1, sg, l, 0)];
        pz = agg[a0_idx(nseg, ns, 1, sg, l, 1)];
    }
    Q = n > 0 ? agg[a0_idx(nseg, ns, 1, sg, pp.mh, 0)].re : 0.0;
    Z = n > 0 ? agg[a0_idx(nseg, ns, 1, sg, pp.mh, 1)].re : 0.0;
    for (int c0 = S0 - LG; c0 >= 0; c0 -= LG) {
        double vp[LG], vf[LG];
#pragma unroll
        for (int t = LG - 1; t >= 0; --t) {
            const int j = c0 + t;
            vp[t] = vf[t] = 0.0;
            if (j < n) {
                const cx<double> U = pq, W = pz;
                const cx<double> V{W.re - z[j] * U.re, W.im - z[j] * U.im};
                vp[t] = cu.re * U.re - cu.im * U.im + cv.re * V.re - cv.im * V.im +
                        lw * (Z - z[j] * Q);
                vf[t] = -(fu.re * U.re - fu.im * U.im + fv.re * V.re - fv.im * V.im) - lw * Q;
                Q += q[j];
                Z += q[j] * z[j];
                if (j) {
                    const cx<double> d = cexpm64(br, bi, z[j] - z[j - 1]);
                    pq = cmul(cx<double>{U.re + q[j], U.im}, d);
                    pz = cmul(cx<double>{W.re + q[j] * z[j], W.im}, d);
                }
            }
        }
        const double sp = group_sum<LG>(vp, L.rb[g], l);
        const double sf = group_sum<LG>(vf, L.rb[g], l);
        L.ph[g][c0 + l] += sp;
        L.fz[g][c0 + l] += sf;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < G * S0; e += WAVE) {
        const int gg = e / S0, j = e % S0, s = seg0 + gg;
        const int64_t i = (int64_t)s * S0 + j;
        if (s < nseg && i < N) {
            // replica batches: 2 pi / A of the replica holding this segment
            const double tpa = rep_tpa ? rep_tpa[seg_rep[s / seg_div]] : two_pi_over_A;
            phi0[i] = -tpa * (L.ph[gg][j] + (double)L.q[gg][j] * k0_self);
            fz0[i] = tpa * L.fz[gg][j];  // field: the target charge is applied later
        }
    }
}

}  // namespace

// aggregates, carries and sweep with LG pair lanes per segment
template <int LG>
static q2d_status k0_launch(Plan *p, int64_t N, int nseg, const void *qsrc, double tpa,
                            const double *rep_tpa, const int32_t *seg_rep, int seg_div) {
    const int nb = (nseg + K0Lds<float, LG>::G - 1) / K0Lds<float, LG>::G;
    cx<double> *agg = (cx<double> *)p->agg0.p;
    cx<double> *spans = (cx<double> *)p->spans0.p;
    if (p->fp32)
        k0_agg<float, LG><<<nb, WAVE, 0, p->stream>>>(
            (const float *)p->s_z.p, (const float *)qsrc, N, nseg, p->pp, agg, spans);
    else
        k0_agg<double, LG><<<nb, WAVE, 0, p->stream>>>(
            (const double *)p->s_z.p, (const double *)qsrc, N, nseg, p->pp, agg, spans);
    q2d_status st = carry_k0(p, nseg, S0, N);
    if (st != Q2D_OK) return st;
    if (p->fp32)
        k0_sweep<float, LG><<<nb, WAVE, 0, p->stream>>>(
            (const float *)p->s_z.p, (const float *)qsrc, N, nseg, p->pp, p->c_lin, p->k0_self,
            tpa, agg, (double *)p->phi0.p, (double *)p->fz0.p, rep_tpa, seg_rep, seg_div);
    else
        k0_sweep<double, LG><<<nb, WAVE, 0, p->stream>>>(
            (const double *)p->s_z.p, (const double *)qsrc, N, nseg, p->pp, p->c_lin, p->k0_self,
            tpa, agg, (double *)p->phi0.p, (double *)p->fz0.p, rep_tpa, seg_rep, seg_div);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

void k0_reqs(Plan *p, int64_t N, Reqs &q) {
    if (N <= 0) return;
    const int nseg = (int)((N + S0 - 1) / S0);
    const int mh = p->mh;
    q.add(p->spans0, (size_t)nseg * mh * 2 * sizeof(cx<double>));
    q.add(p->agg0, (size_t)2 * nseg * (mh + 1) * 2 * sizeof(cx<double>));
    q.add(p->phi0, (size_t)N * sizeof(double));
    q.add(p->fz0, (size_t)N * sizeof(double));
    q.add(p->carry_tmp0, carry_tmp_bytes((int64_t)(mh + 1) * 2, nseg));
}

q2d_status k0_run(Plan *p, int64_t N) {
    if (N <= 0) return Q2D_OK;
    tstart(p, 3);
    const int nseg = (int)((N + S0 - 1) / S0);
    const int mh = p->mh;
    q2d_status st;
    Reqs req;
    k0_reqs(p, N, req);
    if ((st = ensure_all(p, req)) != Q2D_OK) return st;
    const void *qsrc = p->src ? p->src : p->s_q.p;
    const double PI = 3.14159265358979323846;
    const double tpa = 2.0 * PI / (p->Lx * p->Ly);
    const double *rep_tpa = p->R ? (const double *)p->rep_tpa.p : nullptr;
    const int32_t *seg_rep = p->R ? (const int32_t *)p->seg_rep.p : nullptr;
    const int seg_div = p->R ? p->S_batch / S0 : 1;
    st = mh <= 8 ? k0_launch<8>(p, N, nseg, qsrc, tpa, rep_tpa, seg_rep, seg_div)
                 : k0_launch<16>(p, N, nseg, qsrc, tpa, rep_tpa, seg_rep, seg_div);
    if (st != Q2D_OK) return st;
    tstop(p, 3);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

}  // namespace q2d
