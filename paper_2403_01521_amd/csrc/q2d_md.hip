// Charged walls and the Langevin update: the remaining steps of an RBSE2D
// molecular-dynamics step (Alg. 2: the particle-slab term; Sec. 4.3: the
// Langevin dynamics the random-batch forces drive).
//
// Particle-slab term (Sec. 2.4, Thm 2.7, eq. phionwallzero, eq. spectial).
// Walls at z = 0 and z = Lz with doubly periodic surface charge densities of
// cell Fourier coefficients sig(k) = int_cell sigma(rho) e^{-i k.rho} drho:
//   phi_ps(r) = (2 pi/A) Re sum_{k != 0} e^{i k.rho}/k [sb(k) e^{-k|z|} + st(k) e^{-k|z - Lz|}]
//               - (2 pi/A) [sb(0) |z| + st(0) |z - Lz|],
// F = -q grad phi_ps, E = sum_i q_i phi_ps(r_i) (the walls are external: no
// factor 1/2).  Uniform walls are the zero modes alone.  One thread per
// particle loops over the listed modes (shared by all threads); FP64
// arithmetic for both precisions (the term is O(N n_modes) and cheap).
//
// Langevin step (Sec. 4.3, eq. langevin) by the BAOAB splitting: stage 0 is
// B A O A from the forces at the current positions (half kick, half drift,
// the exact Ornstein-Uhlenbeck step of the friction and noise, half drift),
// then x, y wrap and z folds back between the walls by specular reflection;
// stage 1 is the closing half kick B with the forces at the new positions.
// Normal deviates: Philox4x32-10, key = seed, counter (particle, step, stream)
// with streams 3 (x, y) and 4 (z), Box-Muller on two 53-bit uniforms.
#include <algorithm>
#include <cmath>

#include "q2d_internal.h"

namespace q2d {

namespace {

struct SlabArgs {
    double Lx, Ly, Lz, tpa;  // tpa = 2 pi / A
    double s0b, s0t;         // zero modes (charge per cell)
    int n_modes;
};

template <typename T>
__global__ __launch_bounds__(256) void k_slab(const T *__restrict__ pos, const T *__restrict__ q,
                                              int64_t N, SlabArgs a,
                                              const int32_t *__restrict__ modes,
                                              const double *__restrict__ sb,
                                              const double *__restrict__ st, T *__restrict__ phi,
                                              T *__restrict__ F, double *__restrict__ part) {
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < N) {
        const double x = (double)pos[3 * i], y = (double)pos[3 * i + 1], z = (double)pos[3 * i + 2];
        const double qi = (double)q[i];
        const double zb = fabs(z), zt = fabs(z - a.Lz);
        const double gb = z > 0.0 ? 1.0 : (z < 0.0 ? -1.0 : 0.0);
        const double gt = z > a.Lz ? 1.0 : (z < a.Lz ? -1.0 : 0.0);
        double p = -a.tpa * (a.s0b * zb + a.s0t * zt);
        double dx = 0.0, dy = 0.0, dz = -a.tpa * (a.s0b * gb + a.s0t * gt);
        const double PI = 3.14159265358979323846;
        for (int m = 0; m < a.n_modes; ++m) {
            const double kx = 2.0 * PI * modes[2 * m] / a.Lx, ky = 2.0 * PI * modes[2 * m + 1] / a.Ly;
            const double k = sqrt(kx * kx + ky * ky);
            double s, c;
            sincos(kx * x + ky * y, &s, &c);
            const double eb = exp(-k * zb), et = exp(-k * zt);
            // u = sb eb + st et (complex); term = tpa e^{i k.rho} u / k
            const double ur = sb[2 * m] * eb + st[2 * m] * et;
            const double ui = sb[2 * m + 1] * eb + st[2 * m + 1] * et;
            const double tr = a.tpa * (c * ur - s * ui) / k, ti = a.tpa * (c * ui + s * ur) / k;
            p += tr;
            // d/dx Re(term) = Re(i kx term) = -kx Im(term)
            dx -= kx * ti;
            dy -= ky * ti;
            const double vr = sb[2 * m] * gb * eb + st[2 * m] * gt * et;
            const double vi = sb[2 * m + 1] * gb * eb + st[2 * m + 1] * gt * et;
            dz -= a.tpa * (c * vr - s * vi);
        }
        if (phi) phi[i] = (T)p;
        if (F) {
            F[3 * i] = (T)(-qi * dx);
            F[3 * i + 1] = (T)(-qi * dy);
            F[3 * i + 2] = (T)(-qi * dz);
        }
        e = qi * p;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_parts(const double *part, int n, double *E) {
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < n; b += 256) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) E[0] = red[0];
}

// two standard normals from one Philox block (Box-Muller)
__device__ inline void normal2(uint32_t i, uint64_t seed, uint64_t step, uint32_t stream,
                               double &n0, double &n1) {
    uint32_t c[4] = {i, (uint32_t)step, (uint32_t)(step >> 32), stream};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
    const double r = sqrt(-2.0 * log(u1));
    const double PI = 3.14159265358979323846;
    n0 = r * cos(2.0 * PI * u2);
    n1 = r * sin(2.0 * PI * u2);
}

struct LangevinArgs {
    double Lx, Ly, Lz, dt, gamma, kT;
    uint64_t seed, step;
    int stage;
};

template <typename T>
__global__ __launch_bounds__(256) void k_langevin(T *__restrict__ pos, T *__restrict__ mom,
                                                  const T *__restrict__ mass, int64_t N,
                                                  const T *__restrict__ F0, const T *__restrict__ F1,
                                                  const T *__restrict__ F2, LangevinArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    T p[3], f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p[d] = mom[3 * i + d];
        T s = 0;
        if (F0) s += F0[3 * i + d];
        if (F1) s += F1[3 * i + d];
        if (F2) s += F2[3 * i + d];
        f[d] = s;
    }
    const T h = (T)(0.5 * a.dt);
#pragma unroll
    for (int d = 0; d < 3; ++d) p[d] += h * f[d];
    if (a.stage == 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) mom[3 * i + d] = p[d];
        return;
    }
    const T m = mass ? mass[i] : (T)1;
    T r[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) r[d] = pos[3 * i + d] + h * p[d] / m;
    const T c1 = (T)exp(-a.gamma * a.dt / (double)m);
    const T c2 = (T)sqrt((double)m * a.kT * (1.0 - (double)c1 * (double)c1));
    double n[4];
    normal2((uint32_t)i, a.seed, a.step, 3u, n[0], n[1]);
    normal2((uint32_t)i, a.seed, a.step, 4u, n[2], n[3]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p[d] = c1 * p[d] + c2 * (T)n[d];
        r[d] += h * p[d] / m;
    }
    r[0] -= floor(r[0] / (T)a.Lx) * (T)a.Lx;
    r[1] -= floor(r[1] / (T)a.Ly) * (T)a.Ly;
    const T L2 = (T)(2.0 * a.Lz);
    const T zf = r[2] - floor(r[2] / L2) * L2;
    const bool odd = zf > (T)a.Lz;
    r[2] = odd ? L2 - zf : zf;
    p[2] = odd ? -p[2] : p[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pos[3 * i + d] = r[d];
        mom[3 * i + d] = p[d];
    }
}

template <typename T>
q2d_status slab_impl(Plan *p, const T *pos, const T *q, int64_t N, int32_t n_modes,
                     const int32_t *modes, const double *sb, const double *st, double s0b,
                     double s0t, T *phi, T *F, double *E) {
    const int nb = (int)((N + 255) / 256);
    q2d_status s = ensure(p, p->epart, (size_t)std::max(nb, 1) * sizeof(double));
    if (s != Q2D_OK) return s;
    SlabArgs a{p->Lx, p->Ly, p->Lz, 2.0 * 3.14159265358979323846 / (p->Lx * p->Ly), s0b, s0t,
               n_modes};
    if (N > 0)
        k_slab<T><<<nb, 256, 0, p->stream>>>(pos, q, N, a, modes, sb, st, phi, F,
                                             (double *)p->epart.p);
    if (E) k_sum_parts<<<1, 256, 0, p->stream>>>((const double *)p->epart.p, N > 0 ? nb : 0, E);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

}  // namespace

}  // namespace q2d

using namespace q2d;

extern "C" {

q2d_status q2d_slab(q2d_plan_t p, const void *pos, const void *q, int64_t N, int32_t n_modes,
                    const int32_t *modes, const double *sig_bot, const double *sig_top,
                    double sig0_bot, double sig0_top, void *phi, void *F, double *E) {
    if (!p || N < 0 || n_modes < 0) return Q2D_EINVAL;
    if (N > 0 && (!pos || !q)) return Q2D_EINVAL;
    if (n_modes > 0 && (!modes || !sig_bot || !sig_top)) return Q2D_EINVAL;
    if (!std::isfinite(sig0_bot) || !std::isfinite(sig0_top)) return Q2D_EINVAL;
    if (N > p->opts.n_max) return Q2D_ECAPACITY;
    if (hipSetDevice(p->device) != hipSuccess) return Q2D_EDEVICE;
    if (p->fp32)
        return slab_impl<float>(p, (const float *)pos, (const float *)q, N, n_modes, modes,
                                sig_bot, sig_top, sig0_bot, sig0_top, (float *)phi, (float *)F, E);
    return slab_impl<double>(p, (const double *)pos, (const double *)q, N, n_modes, modes,
                             sig_bot, sig_top, sig0_bot, sig0_top, (double *)phi, (double *)F, E);
}

q2d_status q2d_langevin_step(q2d_plan_t p, void *pos, void *mom, const void *mass, int64_t N,
                             const void *F0, const void *F1, const void *F2, double dt,
                             double gamma, double kT, uint64_t seed, uint64_t step,
                             int32_t stage) {
    if (!p || N < 0 || (stage != 0 && stage != 1)) return Q2D_EINVAL;
    if (N > 0 && (!mom || (stage == 0 && !pos))) return Q2D_EINVAL;
    if (!(dt > 0) || !(gamma >= 0) || !(kT >= 0) || !std::isfinite(dt) || !std::isfinite(gamma) ||
        !std::isfinite(kT))
        return Q2D_EINVAL;
    if (N > p->opts.n_max) return Q2D_ECAPACITY;
    if (N == 0) return Q2D_OK;
    if (hipSetDevice(p->device) != hipSuccess) return Q2D_EDEVICE;
    LangevinArgs a{p->Lx, p->Ly, p->Lz, dt, gamma, kT, seed, step, stage};
    const int nb = (int)((N + 255) / 256);
    if (p->fp32)
        k_langevin<float><<<nb, 256, 0, p->stream>>>((float *)pos, (float *)mom,
                                                     (const float *)mass, N, (const float *)F0,
                                                     (const float *)F1, (const float *)F2, a);
    else
        k_langevin<double><<<nb, 256, 0, p->stream>>>((double *)pos, (double *)mom,
                                                      (const double *)mass, N, (const double *)F0,
                                                      (const double *)F1, (const double *)F2, a);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

}  // extern "C"
