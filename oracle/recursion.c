/*
 * O3: the z-sorted O(N) recursion of Sec. 3.2, FP64, plain C (oracle).
 *
 * TEST INFRASTRUCTURE ONLY.  Not linked by the product library; loaded by the
 * test suite and the CPU-baseline leg of the benchmark through ctypes.
 *
 * For every Fourier mode k and every exponent beta in {k} U {alpha s_l}, the
 * pairwise sum S = sum_{j<i} q_i q_j e^{i k.rho_ij} e^{-beta z_ij} (eq. 33) is
 * evaluated after sorting by z with the coefficient recursion of eq. 35:
 *     A_1 = 0,  A_i = A_{i-1} e^{-beta (z_{i-1} - z_{i-2})} + q_{i-1} e^{-i k.rho_{i-1}},
 *     T_i = e^{-beta (z_i - z_{i-1})} A_i          (= sum_{j<i} b_j e^{-beta(z_i - z_j)})
 * and its mirror image for j > i (needed for per-particle potentials and the
 * two sums of App. E).  The mode's pair kernel K_k(z) = sum_beta c_beta e^{-beta z}
 * (the SOE form of (xi^+ + xi^-)/k, eq. SOEphi) and its derivative
 * K'_k(z) = sum_beta d_beta e^{-beta z} (eq. z-der) are then assembled per
 * particle:
 *     phi_i  += w_k Re( e^{i k.rho_i} C_i ),        C_i = sum_beta c_beta (T_i + B_i)
 *     F_rho  += w_k q_i k_vec Im( e^{i k.rho_i} C_i )
 *     F_z    -= w_k q_i Re( e^{i k.rho_i} D_i ),     D_i = sum_beta d_beta (T_i - B_i)
 * All M SOE terms are used individually (no pairing of conjugates) and each
 * mode enters with its own weight w_k, so a full-lattice mode list gives the
 * real total directly.
 *
 * The k = 0 term uses eq. 32 and eq. dzphi_0 with the same recursion on real
 * sources q_j, plus the first-moment recursion for z_ij e^{-beta z_ij}:
 *     Vh_i = e^{-beta D}(Vh_{i-1} + D A_{i-1}),  D = z_{i-1} - z_{i-2},
 *     V_i  = e^{-beta d}(Vh_i + d A_i),          d = z_i - z_{i-1},
 * and prefix sums of q_j and q_j z_j for the linear part.
 *
 * Pin: equal to the direct pair sums of O2 to rounding (tests).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double *g_sort_z;
static int cmp_z(const void *a, const void *b)
{
    int ia = *(const int *)a, ib = *(const int *)b;
    double za = g_sort_z[ia], zb = g_sort_z[ib];
    if (za < zb) return -1;
    if (za > zb) return 1;
    return (ia > ib) - (ia < ib);
}

/* Forward recursion (eq. 35) for one beta: out[n] = sum_{m<n} b[m] e^{-beta(z[n]-z[m])}
 * in sorted order. */
static void forward_T(int N, const double *z, const cplx *b, cplx beta, cplx *out)
{
    cplx A = 0.0;
    for (int n = 0; n < N; ++n) {
        if (n == 0) {
            out[0] = 0.0;
            continue;
        }
        if (n >= 2) A = A * cexp(-beta * (z[n - 1] - z[n - 2]));
        A += b[n - 1];
        out[n] = cexp(-beta * (z[n] - z[n - 1])) * A;
    }
}

/* Mirror recursion: out[n] = sum_{m>n} b[m] e^{-beta(z[m]-z[n])}. */
static void backward_B(int N, const double *z, const cplx *b, cplx beta, cplx *out)
{
    cplx A = 0.0;
    for (int n = N - 1; n >= 0; --n) {
        if (n == N - 1) {
            out[n] = 0.0;
            continue;
        }
        if (n <= N - 3) A = A * cexp(-beta * (z[n + 2] - z[n + 1]));
        A += b[n + 1];
        out[n] = cexp(-beta * (z[n + 1] - z[n])) * A;
    }
}

/*
 * Long-range SOE Ewald2D (k != 0 modes + k = 0 + self) for all particles.
 *   modes (mx[m], my[m]) with weight[m]; include_self_pair adds the j = i term
 *   of every k != 0 mode; diag adds q_i * diag to phi.
 * Outputs are in input order.  Returns 0 on success.
 */
int o3_long_range(int N, const double *x, const double *y, const double *z, const double *q,
                  double Lx, double Ly, double alpha, int M, const double *w_re,
                  const double *w_im, const double *s_re, const double *s_im, int nmodes,
                  const int *mx, const int *my, const double *weight, int include_self_pair,
                  double diag, int nthreads, double *phi, double *Fx, double *Fy, double *Fz)
{
    const double PI = 3.14159265358979323846;
    const double SQPI = sqrt(PI);
    const double A2 = Lx * Ly;
    if (N <= 0) return 0;
    int *ord = (int *)malloc(sizeof(int) * N);
    double *zs = (double *)malloc(sizeof(double) * N);
    double *xs = (double *)malloc(sizeof(double) * N);
    double *ys = (double *)malloc(sizeof(double) * N);
    double *qs = (double *)malloc(sizeof(double) * N);
    cplx *w = (cplx *)malloc(sizeof(cplx) * M);
    cplx *s = (cplx *)malloc(sizeof(cplx) * M);
    double *phs = (double *)calloc(N, sizeof(double));
    double *fxs = (double *)calloc(N, sizeof(double));
    double *fys = (double *)calloc(N, sizeof(double));
    double *fzs = (double *)calloc(N, sizeof(double));
    for (int i = 0; i < N; ++i) ord[i] = i;
    g_sort_z = z;
    qsort(ord, N, sizeof(int), cmp_z);
    for (int n = 0; n < N; ++n) {
        zs[n] = z[ord[n]];
        xs[n] = x[ord[n]];
        ys[n] = y[ord[n]];
        qs[n] = q[ord[n]];
    }
    for (int l = 0; l < M; ++l) {
        w[l] = w_re[l] + I * w_im[l];
        s[l] = s_re[l] + I * s_im[l];
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

    /* ---------------- k != 0 modes ---------------- */
#pragma omp parallel
    {
        cplx *b = (cplx *)malloc(sizeof(cplx) * N);
        cplx *T = (cplx *)malloc(sizeof(cplx) * N);
        cplx *B = (cplx *)malloc(sizeof(cplx) * N);
        cplx *C = (cplx *)malloc(sizeof(cplx) * N);
        cplx *D = (cplx *)malloc(sizeof(cplx) * N);
        double *lph = (double *)calloc(N, sizeof(double));
        double *lfx = (double *)calloc(N, sizeof(double));
        double *lfy = (double *)calloc(N, sizeof(double));
        double *lfz = (double *)calloc(N, sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m < nmodes; ++m) {
            double kx = 2.0 * PI * mx[m] / Lx, ky = 2.0 * PI * my[m] / Ly;
            double k = hypot(kx, ky);
            double om = weight[m];
            for (int n = 0; n < N; ++n) {
                b[n] = qs[n] * cexp(-I * (kx * xs[n] + ky * ys[n]));
                C[n] = 0.0;
                D[n] = 0.0;
            }
            /* coefficients of e^{-k z}: c_k = (2a/(sqrt(pi)k)) sum_l w_l 2 beta_l/(beta_l^2-k^2),
             * d_k = -(2a/sqrt(pi)) sum_l w_l 2 beta_l/(beta_l^2-k^2) */
            cplx ck = 0.0, dk = 0.0;
            cplx self_sum = 0.0;
            for (int l = 0; l < M; ++l) {
                cplx bl = alpha * s[l];
                cplx den = bl * bl - k * k;
                ck += 2.0 * alpha / (SQPI * k) * w[l] * 2.0 * bl / den;
                dk += -2.0 * alpha / SQPI * w[l] * 2.0 * bl / den;
            }
            self_sum += ck;
            forward_T(N, zs, b, (cplx)k, T);
            backward_B(N, zs, b, (cplx)k, B);
            for (int n = 0; n < N; ++n) {
                C[n] += creal(ck) * (T[n] + B[n]);
                D[n] += creal(dk) * (T[n] - B[n]);
            }
            for (int l = 0; l < M; ++l) {
                cplx bl = alpha * s[l];
                cplx den = bl * bl - k * k;
                cplx cl = -2.0 * alpha / (SQPI * k) * w[l] * 2.0 * k / den;
                cplx dl = 2.0 * alpha / SQPI * w[l] * 2.0 * bl / den;
                self_sum += cl;
                forward_T(N, zs, b, bl, T);
                backward_B(N, zs, b, bl, B);
                for (int n = 0; n < N; ++n) {
                    C[n] += cl * (T[n] + B[n]);
                    D[n] += dl * (T[n] - B[n]);
                }
            }
            for (int n = 0; n < N; ++n) {
                cplx e = cexp(I * (kx * xs[n] + ky * ys[n]));
                cplx ec = e * C[n];
                lph[n] += om * creal(ec);
                lfx[n] += om * qs[n] * kx * cimag(ec);
                lfy[n] += om * qs[n] * ky * cimag(ec);
                lfz[n] += -om * qs[n] * creal(e * D[n]);
                if (include_self_pair) lph[n] += om * qs[n] * creal(self_sum);
            }
        }
#pragma omp critical
        {
            for (int n = 0; n < N; ++n) {
                phs[n] += lph[n];
                fxs[n] += lfx[n];
                fys[n] += lfy[n];
                fzs[n] += lfz[n];
            }
        }
        free(b); free(T); free(B); free(C); free(D);
        free(lph); free(lfx); free(lfy); free(lfz);
    }

    /* ---------------- k = 0 (eq. 32, eq. dzphi_0) ---------------- */
    {
        double *Ql = (double *)malloc(sizeof(double) * N);  /* sum_{j<n} q_j */
        double *Zl = (double *)malloc(sizeof(double) * N);  /* sum_{j<n} q_j z_j */
        double qa = 0.0, za = 0.0, qtot = 0.0, ztot = 0.0;
        for (int n = 0; n < N; ++n) {
            Ql[n] = qa;
            Zl[n] = za;
            qa += qs[n];
            za += qs[n] * zs[n];
        }
        qtot = qa;
        ztot = za;
        cplx *Uf = (cplx *)malloc(sizeof(cplx) * N), *Vf = (cplx *)malloc(sizeof(cplx) * N);
        cplx *Ub = (cplx *)malloc(sizeof(cplx) * N), *Vb = (cplx *)malloc(sizeof(cplx) * N);
        double *p0 = (double *)calloc(N, sizeof(double));
        double *f0 = (double *)calloc(N, sizeof(double));
        double K0self = 0.0;
        for (int l = 0; l < M; ++l) {
            cplx bl = alpha * s[l];
            K0self += creal(w[l] / SQPI / alpha);
            /* forward: U_n = sum_{j<n} q_j e^{-b(z_n-z_j)}, V_n = sum_{j<n} q_j (z_n-z_j) e^{...} */
            cplx Ah = 0.0, Vh = 0.0;
            for (int n = 0; n < N; ++n) {
                if (n == 0) { Uf[0] = 0.0; Vf[0] = 0.0; continue; }
                if (n >= 2) {
                    double Dz = zs[n - 1] - zs[n - 2];
                    cplx e = cexp(-bl * Dz);
                    Vh = e * (Vh + Dz * Ah);
                    Ah = e * Ah;
                }
                Ah += qs[n - 1];
                double dz = zs[n] - zs[n - 1];
                cplx e = cexp(-bl * dz);
                Uf[n] = e * Ah;
                Vf[n] = e * (Vh + dz * Ah);
            }
            Ah = 0.0; Vh = 0.0;
            for (int n = N - 1; n >= 0; --n) {
                if (n == N - 1) { Ub[n] = 0.0; Vb[n] = 0.0; continue; }
                if (n <= N - 3) {
                    double Dz = zs[n + 2] - zs[n + 1];
                    cplx e = cexp(-bl * Dz);
                    Vh = e * (Vh + Dz * Ah);
                    Ah = e * Ah;
                }
                Ah += qs[n + 1];
                double dz = zs[n + 1] - zs[n];
                cplx e = cexp(-bl * dz);
                Ub[n] = e * Ah;
                Vb[n] = e * (Vh + dz * Ah);
            }
            for (int n = 0; n < N; ++n) {
                double lin_f = zs[n] * Ql[n] - Zl[n];                             /* sum_{j<n} q_j z_nj */
                double lin_b = (ztot - Zl[n] - qs[n] * zs[n]) - zs[n] * (qtot - Ql[n] - qs[n]);
                double Qf = Ql[n], Qb = qtot - Ql[n] - qs[n];
                cplx kf = w[l] / SQPI * (2.0 / s[l] * lin_f + (1.0 / alpha) * Uf[n] - 2.0 / s[l] * Vf[n]);
                cplx kb = w[l] / SQPI * (2.0 / s[l] * lin_b + (1.0 / alpha) * Ub[n] - 2.0 / s[l] * Vb[n]);
                cplx df = w[l] / SQPI * (2.0 / s[l] * Qf - (s[l] + 2.0 / s[l]) * Uf[n] + 2.0 * alpha * Vf[n]);
                cplx db = w[l] / SQPI * (2.0 / s[l] * Qb - (s[l] + 2.0 / s[l]) * Ub[n] + 2.0 * alpha * Vb[n]);
                p0[n] += creal(kf + kb);
                f0[n] += creal(df - db);
            }
        }
        for (int n = 0; n < N; ++n) {
            phs[n] += -(2.0 * PI / A2) * (p0[n] + qs[n] * K0self);
            fzs[n] += (2.0 * PI / A2) * qs[n] * f0[n];
            phs[n] += qs[n] * diag - 2.0 * alpha * qs[n] / SQPI;
        }
        free(Ql); free(Zl); free(Uf); free(Vf); free(Ub); free(Vb); free(p0); free(f0);
    }

    for (int n = 0; n < N; ++n) {
        phi[ord[n]] = phs[n];
        Fx[ord[n]] = fxs[n];
        Fy[ord[n]] = fys[n];
        Fz[ord[n]] = fzs[n];
    }
    free(ord); free(zs); free(xs); free(ys); free(qs); free(w); free(s);
    free(phs); free(fxs); free(fys); free(fzs);
    return 0;
}
