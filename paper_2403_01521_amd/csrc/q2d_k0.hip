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
// Layout: one thread per segment of S0 consecutive sorted particles holding
// all SOE pairs; segment aggregates and carries use the same FP64 carry scan
// as the k != 0 modes.
#include "q2d_internal.h"

namespace q2d {

q2d_status carry_k0(Plan *p, int nseg, int S, int64_t N);
q2d_status spans_k0(Plan *p, int nseg, int S, int64_t N);

namespace {

constexpr int S0 = 16;

__device__ inline cx<double> cexpm64(double br, double bi, double t) {
    const double ar = br * t, ai = bi * t;
    if (fabs(ar) + fabs(ai) < 0.015625) {
        double pr = 1.0 / 5040.0, pi = 0.0;
        const double cs[7] = {1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0, 1.0 / 6.0, 0.5, 1.0, 1.0};
#pragma unroll
        for (int n = 0; n < 7; ++n) {
            const double nr = -(pr * ar - pi * ai), ni = -(pr * ai + pi * ar);
            pr = nr + cs[n];
            pi = ni;
        }
        return {pr, pi};
    }
    const double m = exp(-ar);
    double s, c;
    sincos(ai, &s, &c);
    return {m * c, -m * s};
}

// agg0 layout: [dir][seg][slot][input] complex double, slot mh = linear (beta 0)
__device__ inline int64_t a0_idx(int nseg, int ns, int dir, int seg, int slot, int inp) {
    return (((int64_t)dir * nseg + seg) * ns + slot) * 2 + inp;
}

template <typename T>
__global__ __launch_bounds__(128) void k0_agg(const T *__restrict__ zs, const T *__restrict__ qs,
                                              int64_t N, int nseg, PairParams pp,
                                              cx<double> *__restrict__ agg) {
    const int seg = blockIdx.x * blockDim.x + threadIdx.x;
    if (seg >= nseg) return;
    const int64_t i0 = (int64_t)seg * S0;
    const int n = (int)min((int64_t)S0, N - i0);
    double z[S0], q[S0];
#pragma unroll
    for (int j = 0; j < S0; ++j) {
        z[j] = j < n ? (double)zs[i0 + j] : 0.0;
        q[j] = j < n ? (double)qs[i0 + j] : 0.0;
    }
    const int ns = pp.mh + 1;
    for (int l = 0; l < pp.mh; ++l) {
        const double br = pp.beta_re[l], bi = pp.beta_im[l];
        cx<double> fq{0, 0}, fz{0, 0}, bq{0, 0}, bz{0, 0}, e{1, 0};
#pragma unroll
        for (int j = 0; j < S0; ++j) {
            if (j < n) {
                const cx<double> d = j ? cexpm64(br, bi, z[j] - z[j - 1]) : cx<double>{1, 0};
                fq = cmul(fq, d);
                fz = cmul(fz, d);
                fq.re += q[j];
                fz.re += q[j] * z[j];
                e = cmul(e, d);
                bq.re += q[j] * e.re;
                bq.im += q[j] * e.im;
                bz.re += q[j] * z[j] * e.re;
                bz.im += q[j] * z[j] * e.im;
            }
        }
        agg[a0_idx(nseg, ns, 0, seg, l, 0)] = fq;
        agg[a0_idx(nseg, ns, 0, seg, l, 1)] = fz;
        agg[a0_idx(nseg, ns, 1, seg, l, 0)] = bq;
        agg[a0_idx(nseg, ns, 1, seg, l, 1)] = bz;
    }
    double sq = 0, sz = 0;
#pragma unroll
    for (int j = 0; j < S0; ++j) {
        sq += q[j];
        sz += q[j] * z[j];
    }
    agg[a0_idx(nseg, ns, 0, seg, pp.mh, 0)] = cx<double>{sq, 0};
    agg[a0_idx(nseg, ns, 0, seg, pp.mh, 1)] = cx<double>{sz, 0};
    agg[a0_idx(nseg, ns, 1, seg, pp.mh, 0)] = cx<double>{sq, 0};
    agg[a0_idx(nseg, ns, 1, seg, pp.mh, 1)] = cx<double>{sz, 0};
}

template <typename T>
__global__ __launch_bounds__(128) void k0_sweep(const T *__restrict__ zs,
                                                const T *__restrict__ qs, int64_t N, int nseg,
                                                PairParams pp, double c_lin, double k0_self,
                                                double two_pi_over_A,
                                                const cx<double> *__restrict__ agg,
                                                double *__restrict__ phi0,
                                                double *__restrict__ fz0,
                                                const double *__restrict__ rep_tpa,
                                                const int32_t *__restrict__ seg_rep,
                                                int seg_div) {
    const int seg = blockIdx.x * blockDim.x + threadIdx.x;
    if (seg >= nseg) return;
    // replica batches: 2 pi / A of the replica holding this segment
    if (rep_tpa) two_pi_over_A = rep_tpa[seg_rep[seg / seg_div]];
    const int64_t i0 = (int64_t)seg * S0;
    const int n = (int)min((int64_t)S0, N - i0);
    double z[S0], q[S0], ph[S0], fz[S0];
#pragma unroll
    for (int j = 0; j < S0; ++j) {
        z[j] = j < n ? (double)zs[i0 + j] : 0.0;
        q[j] = j < n ? (double)qs[i0 + j] : 0.0;
        ph[j] = 0.0;
        fz[j] = 0.0;
    }
    const int ns = pp.mh + 1;
    for (int l = 0; l < pp.mh; ++l) {
        const double br = pp.beta_re[l], bi = pp.beta_im[l];
        const cx<double> cu{pp.c0u_re[l], pp.c0u_im[l]}, cv{pp.c0v_re[l], pp.c0v_im[l]};
        const cx<double> fu{pp.f0u_re[l], pp.f0u_im[l]}, fv{pp.f0v_re[l], pp.f0v_im[l]};
        // forward: U = sum_{j<i} q_j e^{..}, W = sum_{j<i} q_j z_j e^{..}, V = z_i U - W
        cx<double> pq = agg[a0_idx(nseg, ns, 0, seg, l, 0)];
        cx<double> pz = agg[a0_idx(nseg, ns, 0, seg, l, 1)];
#pragma unroll
        for (int j = 0; j < S0; ++j) {
            if (j < n) {
                const cx<double> d = j ? cexpm64(br, bi, z[j] - z[j - 1]) : cx<double>{1, 0};
                const cx<double> U = cmul(pq, d), W = cmul(pz, d);
                const cx<double> V{z[j] * U.re - W.re, z[j] * U.im - W.im};
                ph[j] += cu.re * U.re - cu.im * U.im + cv.re * V.re - cv.im * V.im;
                fz[j] += fu.re * U.re - fu.im * U.im + fv.re * V.re - fv.im * V.im;
                pq = cx<double>{U.re + q[j], U.im};
                pz = cx<double>{W.re + q[j] * z[j], W.im};
            }
        }
        // backward: U = sum_{j>i} q_j e^{..}, W = sum_{j>i} q_j z_j e^{..}, V = W - z_i U
        pq = agg[a0_idx(nseg, ns, 1, seg, l, 0)];
        pz = agg[a0_idx(nseg, ns, 1, seg, l, 1)];
#pragma unroll
        for (int j = S0 - 1; j >= 0; --j) {
            if (j < n) {
                const cx<double> U = pq, W = pz;
                const cx<double> V{W.re - z[j] * U.re, W.im - z[j] * U.im};
                ph[j] += cu.re * U.re - cu.im * U.im + cv.re * V.re - cv.im * V.im;
                fz[j] -= fu.re * U.re - fu.im * U.im + fv.re * V.re - fv.im * V.im;
                if (j) {
                    const cx<double> d = cexpm64(br, bi, z[j] - z[j - 1]);
                    pq = cmul(cx<double>{U.re + q[j], U.im}, d);
                    pz = cmul(cx<double>{W.re + q[j] * z[j], W.im}, d);
                }
            }
        }
    }
    // linear terms (beta = 0): prefix sums of q and q z below and above
    double Qf = agg[a0_idx(nseg, ns, 0, seg, pp.mh, 0)].re;
    double Zf = agg[a0_idx(nseg, ns, 0, seg, pp.mh, 1)].re;
    double Qb = agg[a0_idx(nseg, ns, 1, seg, pp.mh, 0)].re;
    double Zb = agg[a0_idx(nseg, ns, 1, seg, pp.mh, 1)].re;
    double sq = 0, sz = 0;
#pragma unroll
    for (int j = 0; j < S0; ++j) {
        sq += q[j];
        sz += q[j] * z[j];
    }
    // Qb, Zb are the sums above the segment; add the segment's part above j
    double aq = sq, az = sz;
#pragma unroll
    for (int j = 0; j < S0; ++j) {
        if (j < n) {
            aq -= q[j];
            az -= q[j] * z[j];
            const double qa = Qb + aq, za = Zb + az;
            ph[j] += c_lin * ((z[j] * Qf - Zf) + (za - z[j] * qa));
            fz[j] += c_lin * (Qf - qa);
            Qf += q[j];
            Zf += q[j] * z[j];
        }
    }
#pragma unroll
    for (int j = 0; j < S0; ++j) {
        if (j < n) {
            phi0[i0 + j] = -two_pi_over_A * (ph[j] + q[j] * k0_self);
            fz0[i0 + j] = two_pi_over_A * fz[j];  // field: the target charge is applied later
        }
    }
}

}  // namespace

q2d_status k0_run(Plan *p, int64_t N) {
    if (N <= 0) return Q2D_OK;
    tstart(p, 3);
    const int nseg = (int)((N + S0 - 1) / S0);
    const int mh = p->mh;
    q2d_status st;
    if ((st = ensure(p, p->spans0, (size_t)nseg * mh * 2 * sizeof(cx<double>))) != Q2D_OK)
        return st;
    if ((st = ensure(p, p->agg0, (size_t)2 * nseg * (mh + 1) * 2 * sizeof(cx<double>))) != Q2D_OK)
        return st;
    if ((st = ensure(p, p->phi0, (size_t)N * sizeof(double))) != Q2D_OK) return st;
    if ((st = ensure(p, p->fz0, (size_t)N * sizeof(double))) != Q2D_OK) return st;
    if ((st = spans_k0(p, nseg, S0, N)) != Q2D_OK) return st;
    const int nb = (nseg + 127) / 128;
    const void *qsrc = p->src ? p->src : p->s_q.p;
    const double PI = 3.14159265358979323846;
    const double tpa = 2.0 * PI / (p->Lx * p->Ly);
    const double *rep_tpa = p->R ? (const double *)p->rep_tpa.p : nullptr;
    const int32_t *seg_rep = p->R ? (const int32_t *)p->seg_rep.p : nullptr;
    const int seg_div = p->R ? p->S_batch / S0 : 1;
    if (p->fp32)
        k0_agg<float><<<nb, 128, 0, p->stream>>>((const float *)p->s_z.p, (const float *)qsrc,
                                                  N, nseg, p->pp, (cx<double> *)p->agg0.p);
    else
        k0_agg<double><<<nb, 128, 0, p->stream>>>((const double *)p->s_z.p,
                                                   (const double *)qsrc, N, nseg, p->pp,
                                                   (cx<double> *)p->agg0.p);
    if ((st = carry_k0(p, nseg, S0, N)) != Q2D_OK) return st;
    if (p->fp32)
        k0_sweep<float><<<nb, 128, 0, p->stream>>>(
            (const float *)p->s_z.p, (const float *)qsrc, N, nseg, p->pp, p->c_lin,
            p->k0_self, tpa, (const cx<double> *)p->agg0.p, (double *)p->phi0.p,
            (double *)p->fz0.p, rep_tpa, seg_rep, seg_div);
    else
        k0_sweep<double><<<nb, 128, 0, p->stream>>>(
            (const double *)p->s_z.p, (const double *)qsrc, N, nseg, p->pp, p->c_lin,
            p->k0_self, tpa, (const cx<double> *)p->agg0.p, (double *)p->phi0.p,
            (double *)p->fz0.p, rep_tpa, seg_rep, seg_div);
    tstop(p, 3);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

}  // namespace q2d
