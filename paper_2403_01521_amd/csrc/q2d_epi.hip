// Epilogue: sum the parts of the long-range potential and force in sorted
// order, scatter them back to input order, and reduce the energy in FP64.
//   phi_i = sum_k phi^k_i + q_i D + phi^0_i - 2 alpha q_i / sqrt(pi)   (Sec. 2.2, eq. self)
// (the k = 0 and self terms are left out for a partial k-space sum)
//   F_i   = q_i (sum_k force parts) + F^0_i
//   E     = 1/2 sum_i q_i phi_i                                        (pair energy, Sec. 2.1)
// D is the configuration-independent j = i constant of the k != 0 modes.
// The energy is reduced in a fixed order (block tree, then one block over the
// block partials), so repeated calls give identical bits.
#include <algorithm>

#include "q2d_internal.h"

namespace q2d {

namespace {

constexpr int EPI_THREADS = 256;

// Combine in sorted order.  The result {phi, F_x, F_y, F_z} of particle i
// replaces chunk 0's entry i (each thread reads its own entries first), and
// k_unsort moves it to input order: random 16-byte reads instead of the
// partial-line writes of a scatter.
template <typename T>
__global__ __launch_bounds__(EPI_THREADS) void k_epi(int64_t N, int nchunks, T *__restrict__ outk,
                                                     const T *__restrict__ qs,
                                                     const double *__restrict__ phi0,
                                                     const double *__restrict__ fz0, double diag,
                                                     double self_c, double *__restrict__ epart) {
    __shared__ double red[EPI_THREADS];
    const int64_t i = (int64_t)blockIdx.x * EPI_THREADS + threadIdx.x;
    double e = 0.0;
    if (i < N) {
        double o0 = 0, o1 = 0, o2 = 0, o3 = 0;
        for (int c = 0; c < nchunks; ++c) {
            const T *o = outk + ((int64_t)c * N + i) * 4;
            o0 += (double)o[0];
            o1 += (double)o[1];
            o2 += (double)o[2];
            o3 += (double)o[3];
        }
        const double q = (double)qs[i];
        const double ph = o0 + q * diag + (phi0 ? phi0[i] : 0.0) - self_c * q;
        T *r = outk + i * 4;
        r[0] = (T)ph;
        r[1] = (T)(q * o1);
        r[2] = (T)(q * o2);
        r[3] = (T)(q * (o3 + (fz0 ? fz0[i] : 0.0)));
        e = q * ph;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int h = EPI_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) epart[blockIdx.x] = red[0];
}

// E = 1/2 sum of the block partials, by one whole work-group in a fixed order
__device__ inline void energy_block(const double *__restrict__ epart, int nparts,
                                    double *__restrict__ E) {
    __shared__ double red[EPI_THREADS];
    double s = 0.0;
    for (int b = threadIdx.x; b < nparts; b += EPI_THREADS) s += epart[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = EPI_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) E[0] = 0.5 * red[0];
}

// input order: particle o takes the combined result of its sorted slot inv[o];
// work-group 0 also reduces the energy (k_epi's partials are complete when
// this launch starts), which saves a launch
template <typename T>
__global__ __launch_bounds__(EPI_THREADS) void k_unsort(int64_t N, const T *__restrict__ res,
                                                        const int32_t *__restrict__ inv,
                                                        T *__restrict__ phi, T *__restrict__ F,
                                                        const double *__restrict__ epart,
                                                        int nparts, double *__restrict__ E) {
    const int64_t o = (int64_t)blockIdx.x * EPI_THREADS + threadIdx.x;
    if (o < N) {
        const T *r = res + (int64_t)inv[o] * 4;
        if (phi) phi[o] = r[0];
        if (F) {
            F[3 * o] = r[1];
            F[3 * o + 1] = r[2];
            F[3 * o + 2] = r[3];
        }
    }
    if (E && blockIdx.x == 0) energy_block(epart, nparts, E);
}

__global__ __launch_bounds__(EPI_THREADS) void k_inv(const int32_t *__restrict__ perm, int64_t N,
                                                     int32_t *__restrict__ inv) {
    const int64_t i = (int64_t)blockIdx.x * EPI_THREADS + threadIdx.x;
    if (i < N) inv[perm[i]] = (int32_t)i;
}

__global__ __launch_bounds__(EPI_THREADS) void k_energy(const double *__restrict__ epart,
                                                        int nparts, double *__restrict__ E) {
    energy_block(epart, nparts, E);
}

__global__ void k_set_zero(double *E) { E[0] = 0.0; }

// sum of the chunks' outputs for particle i (sorted order), in FP64
template <typename T>
__device__ inline void chunk_sum(const T *__restrict__ outk, int64_t N, int nchunks, int64_t i,
                                 double o[4]) {
    o[0] = o[1] = o[2] = o[3] = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        const T *v = outk + ((int64_t)c * N + i) * 4;
        o[0] += (double)v[0];
        o[1] += (double)v[1];
        o[2] += (double)v[2];
        o[3] += (double)v[3];
    }
}

// the field (force per unit target charge) of the current sources, sorted order
template <typename T>
__global__ __launch_bounds__(EPI_THREADS) void k_field(int64_t N, int nchunks,
                                                       const T *__restrict__ outk,
                                                       const double *__restrict__ fz0,
                                                       double *__restrict__ fq) {
    const int64_t i = (int64_t)blockIdx.x * EPI_THREADS + threadIdx.x;
    if (i >= N) return;
    double o[4];
    chunk_sum(outk, N, nchunks, i, o);
    fq[3 * i] = o[1];
    fq[3 * i + 1] = o[2];
    fq[3 * i + 2] = o[3] + fz0[i];
}

// Adjoint of phi(pos, q) for weights g (Sec. 2.2 pair sum, App. E forces):
// phi_i = sum_j G(r_i, r_j) q_j with G symmetric, so
//   dq_j   = sum_i g_i G(r_i, r_j)                    = phi(g)_j
//   dpos_k = sum_i g_i d phi_i / d r_k = -(g_k f(q)_k + q_k f(g)_k),
// f(s) being the field of the sources s (the force on a unit charge).
template <typename T>
__global__ __launch_bounds__(EPI_THREADS) void k_vjp(int64_t N, int nchunks,
                                                     const T *__restrict__ outk,
                                                     const T *__restrict__ qs,
                                                     const T *__restrict__ gs,
                                                     const double *__restrict__ phi0,
                                                     const double *__restrict__ fz0,
                                                     const double *__restrict__ fq,
                                                     const int32_t *__restrict__ perm,
                                                     double diag, double self_c,
                                                     T *__restrict__ dq, T *__restrict__ dpos) {
    const int64_t i = (int64_t)blockIdx.x * EPI_THREADS + threadIdx.x;
    if (i >= N) return;
    double o[4];
    chunk_sum(outk, N, nchunks, i, o);
    const double q = (double)qs[i], g = (double)gs[i];
    const int64_t orig = perm[i];
    if (dq) dq[orig] = (T)(o[0] + g * diag + phi0[i] - self_c * g);
    if (dpos) {
        dpos[3 * orig] = (T)(-(g * fq[3 * i] + q * o[1]));
        dpos[3 * orig + 1] = (T)(-(g * fq[3 * i + 1] + q * o[2]));
        dpos[3 * orig + 2] = (T)(-(g * fq[3 * i + 2] + q * (o[3] + fz0[i])));
    }
}

}  // namespace

void inv_reqs(Plan *p, int64_t N, Reqs &q) {
    if (N > 0) q.add(p->inv, (size_t)N * sizeof(int32_t));
}

// scratch of epilogue() (the inverse permutation only if it is not ready)
void epilogue_reqs(Plan *p, int64_t N, Reqs &q) {
    if (N <= 0) return;
    const int nb = (int)((N + EPI_THREADS - 1) / EPI_THREADS);
    const size_t tsz = p->fp32 ? sizeof(float) : sizeof(double);
    q.add(p->epart, (size_t)nb * sizeof(double));
    q.add(p->outk, (size_t)N * 4 * tsz);
    inv_reqs(p, N, q);
}

q2d_status epilogue(Plan *p, int64_t N, int n_chunks, double diag, bool with_k0, void *phi,
                    void *F, double *E) {
    if (N <= 0) {
        if (E) k_set_zero<<<1, 1, 0, p->stream>>>(E);
        return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
    }
    const int nb = (int)((N + EPI_THREADS - 1) / EPI_THREADS);
    q2d_status st;
    if ((st = ensure(p, p->epart, (size_t)nb * sizeof(double))) != Q2D_OK) return st;
    const double self_c = with_k0 ? 2.0 * p->alpha / sqrt(3.14159265358979323846) : 0.0;
    const double *phi0 = with_k0 ? (const double *)p->phi0.p : nullptr;
    const double *fz0 = with_k0 ? (const double *)p->fz0.p : nullptr;
    const bool out = phi || F;
    const bool need_inv = out && !p->inv_ready;
    // k_epi writes each particle's result over chunk 0 of outk: with no chunks
    // (no modes) the buffer may not exist yet; with chunks it already holds
    // n_chunks x N x 4 values and ensure() keeps it
    const size_t tsz = p->fp32 ? sizeof(float) : sizeof(double);
    if ((st = ensure(p, p->outk, (size_t)N * 4 * tsz)) != Q2D_OK) return st;
    p->inv_ready = false;
    if (need_inv && (st = launch_inv(p, N)) != Q2D_OK) return st;
    if (p->fp32)
        k_epi<float><<<nb, EPI_THREADS, 0, p->stream>>>(N, n_chunks, (float *)p->outk.p,
                                                        (const float *)p->s_q.p, phi0, fz0, diag,
                                                        self_c, (double *)p->epart.p);
    else
        k_epi<double><<<nb, EPI_THREADS, 0, p->stream>>>(N, n_chunks, (double *)p->outk.p,
                                                         (const double *)p->s_q.p, phi0, fz0,
                                                         diag, self_c, (double *)p->epart.p);
    const double *ep = (const double *)p->epart.p;
    if (out) {
        const int32_t *inv = (const int32_t *)p->inv.p;
        if (p->fp32)
            k_unsort<float><<<nb, EPI_THREADS, 0, p->stream>>>(N, (const float *)p->outk.p, inv,
                                                               (float *)phi, (float *)F, ep, nb, E);
        else
            k_unsort<double><<<nb, EPI_THREADS, 0, p->stream>>>(
                N, (const double *)p->outk.p, inv, (double *)phi, (double *)F, ep, nb, E);
    } else if (E) {
        k_energy<<<1, EPI_THREADS, 0, p->stream>>>(ep, nb, E);
    }
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

q2d_status launch_inv(Plan *p, int64_t N) {
    if (N <= 0) return Q2D_OK;
    Reqs req;
    inv_reqs(p, N, req);
    q2d_status st = ensure_all(p, req);
    if (st != Q2D_OK) return st;
    k_inv<<<(int)((N + EPI_THREADS - 1) / EPI_THREADS), EPI_THREADS, 0, p->stream>>>(
        p->perm, N, (int32_t *)p->inv.p);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

q2d_status epilogue_field(Plan *p, int64_t N, int n_chunks) {
    if (N <= 0) return Q2D_OK;
    q2d_status st = ensure(p, p->fq, (size_t)N * 3 * sizeof(double));
    if (st != Q2D_OK) return st;
    const int nb = (int)((N + EPI_THREADS - 1) / EPI_THREADS);
    if (p->fp32)
        k_field<float><<<nb, EPI_THREADS, 0, p->stream>>>(N, n_chunks, (const float *)p->outk.p,
                                                          (const double *)p->fz0.p,
                                                          (double *)p->fq.p);
    else
        k_field<double><<<nb, EPI_THREADS, 0, p->stream>>>(N, n_chunks, (const double *)p->outk.p,
                                                           (const double *)p->fz0.p,
                                                           (double *)p->fq.p);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

q2d_status epilogue_vjp(Plan *p, int64_t N, int n_chunks, double diag, void *dq, void *dpos) {
    if (N <= 0) return Q2D_OK;
    const int nb = (int)((N + EPI_THREADS - 1) / EPI_THREADS);
    const double self_c = 2.0 * p->alpha / sqrt(3.14159265358979323846);
    if (p->fp32)
        k_vjp<float><<<nb, EPI_THREADS, 0, p->stream>>>(
            N, n_chunks, (const float *)p->outk.p, (const float *)p->s_q.p,
            (const float *)p->s_g.p, (const double *)p->phi0.p, (const double *)p->fz0.p,
            (const double *)p->fq.p, p->perm, diag, self_c, (float *)dq, (float *)dpos);
    else
        k_vjp<double><<<nb, EPI_THREADS, 0, p->stream>>>(
            N, n_chunks, (const double *)p->outk.p, (const double *)p->s_q.p,
            (const double *)p->s_g.p, (const double *)p->phi0.p, (const double *)p->fz0.p,
            (const double *)p->fq.p, p->perm, diag, self_c, (double *)dq, (double *)dpos);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

namespace {

constexpr int EPB = 64;  // threads per segment in the batch epilogue

// Replica batches: one work-group per segment (a segment lies in one
// replica), padding skipped, the replica's j = i constant; the energy partial
// of each segment is reduced in a fixed order.
template <typename T>
__global__ __launch_bounds__(EPB) void k_epi_batch(int S, int64_t Npad, int nchunks,
                                                   const T *__restrict__ outk,
                                                   const T *__restrict__ qs,
                                                   const double *__restrict__ phi0,
                                                   const double *__restrict__ fz0,
                                                   const int32_t *__restrict__ pperm,
                                                   const int32_t *__restrict__ seg_rep,
                                                   const double *__restrict__ rep_diag,
                                                   double self_c, T *__restrict__ phi,
                                                   T *__restrict__ F,
                                                   double *__restrict__ epart) {
    __shared__ double red[EPB];
    const int seg = blockIdx.x;
    const double diag = rep_diag[seg_rep[seg]];
    double e = 0.0;
    for (int t = threadIdx.x; t < S; t += EPB) {
        const int64_t i = (int64_t)seg * S + t;
        const int32_t orig = pperm[i];
        if (orig < 0) continue;
        double o[4];
        chunk_sum(outk, Npad, nchunks, i, o);
        const double q = (double)qs[i];
        const double ph = o[0] + q * diag + phi0[i] - self_c * q;
        if (phi) phi[orig] = (T)ph;
        if (F) {
            F[3 * (int64_t)orig] = (T)(q * o[1]);
            F[3 * (int64_t)orig + 1] = (T)(q * o[2]);
            F[3 * (int64_t)orig + 2] = (T)(q * (o[3] + fz0[i]));
        }
        e += q * ph;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int h = EPB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) epart[seg] = red[0];
}

// E_r = 1/2 sum of replica r's segment partials, in segment order
__global__ __launch_bounds__(EPB) void k_energy_batch(const double *__restrict__ epart, int S,
                                                      const int64_t *__restrict__ poff, int R,
                                                      double *__restrict__ E) {
    __shared__ double red[EPB];
    const int r = blockIdx.x;
    const int64_t s0 = poff[r] / S, s1 = poff[r + 1] / S;
    double v = 0.0;
    for (int64_t s = s0 + threadIdx.x; s < s1; s += EPB) v += epart[s];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = EPB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) E[r] = 0.5 * red[0];
}

}  // namespace

q2d_status epilogue_batch(Plan *p, int n_chunks, void *phi, void *F, double *E) {
    const int64_t Npad = p->Npad;
    const int S = p->S_batch;
    const int nseg = (int)(Npad / S);
    q2d_status st = ensure(p, p->epart_rep, (size_t)std::max(nseg, 1) * sizeof(double));
    if (st != Q2D_OK) return st;
    const double self_c = 2.0 * p->alpha / sqrt(3.14159265358979323846);
    if (nseg > 0) {
        if (p->fp32)
            k_epi_batch<float><<<nseg, EPB, 0, p->stream>>>(
                S, Npad, n_chunks, (const float *)p->outk.p, (const float *)p->s_q.p,
                (const double *)p->phi0.p, (const double *)p->fz0.p, (const int32_t *)p->pperm.p,
                (const int32_t *)p->seg_rep.p, (const double *)p->rep_diag.p, self_c, (float *)phi,
                (float *)F, (double *)p->epart_rep.p);
        else
            k_epi_batch<double><<<nseg, EPB, 0, p->stream>>>(
                S, Npad, n_chunks, (const double *)p->outk.p, (const double *)p->s_q.p,
                (const double *)p->phi0.p, (const double *)p->fz0.p, (const int32_t *)p->pperm.p,
                (const int32_t *)p->seg_rep.p, (const double *)p->rep_diag.p, self_c,
                (double *)phi, (double *)F, (double *)p->epart_rep.p);
    }
    if (E)
        k_energy_batch<<<p->R, EPB, 0, p->stream>>>((const double *)p->epart_rep.p, S,
                                                   (const int64_t *)p->rep_poff.p, p->R, E);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

}  // namespace q2d
