// Real-space part of the Ewald split (Sec. 2.2, eq. phi_s) with a uniform cell list:
//   phi_s,i = sum over images m and j (j != i for m = 0), |r_ij + M| <= r_c, of q_j erfc(alpha r)/r
//   F_s,i   = q_i sum q_j [erfc(alpha r)/r^2 + (2 alpha/sqrt(pi)) e^{-alpha^2 r^2}/r] (r_ij + M)/r
// With r_c <= min(Lx, Ly)/2 at most one image of a particle lies within r_c,
// so the minimum-image displacement in x and y is exact.  Cells have edge
// >= r_c; the 3 x 3 x 3 neighbourhood (periodic in x, y; not in z) is
// visited with duplicate cells removed when a direction has fewer than 3 cells.
// Arithmetic is FP64 whatever the plan precision; each cell's particles are
// ordered by index so results are deterministic.
#include "q2d_internal.h"

namespace q2d {

namespace {

struct Grid {
    int nx, ny, nz;
    double Lx, Ly, Lz, hx, hy, hz;
};

template <typename T>
__device__ inline int cell_of(const T *pos, int64_t i, const Grid &g, double &x, double &y,
                              double &z) {
    x = (double)pos[3 * i];
    y = (double)pos[3 * i + 1];
    z = (double)pos[3 * i + 2];
    x -= floor(x / g.Lx) * g.Lx;
    y -= floor(y / g.Ly) * g.Ly;
    int cx_ = min(g.nx - 1, max(0, (int)(x / g.hx)));
    int cy_ = min(g.ny - 1, max(0, (int)(y / g.hy)));
    int cz_ = min(g.nz - 1, max(0, (int)(z / g.hz)));
    return (cz_ * g.ny + cy_) * g.nx + cx_;
}

template <typename T>
__global__ void k_cell_count(const T *pos, int64_t N, Grid g, int32_t *__restrict__ cidx,
                             int32_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double x, y, z;
    const int c = cell_of(pos, i, g, x, y, z);
    cidx[i] = c;
    atomicAdd(&count[c], 1);
}

// single block exclusive scan of cell counts
__global__ __launch_bounds__(1024) void k_cell_scan(const int32_t *count, int ncell,
                                                    int32_t *start, int32_t *fill) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int per = (ncell + 1023) / 1024;
    const int b0 = min(t * per, ncell), b1 = min(b0 + per, ncell);
    int32_t s = 0;
    for (int b = b0; b < b1; ++b) s += count[b];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = t ? part[t - 1] : 0;
    for (int b = b0; b < b1; ++b) {
        start[b] = run;
        fill[b] = 0;
        run += count[b];
    }
    if (t == 1023) start[ncell] = part[1023];
}

__global__ void k_cell_fill(const int32_t *cidx, int64_t N, const int32_t *start, int32_t *fill,
                            int32_t *list) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int c = cidx[i];
    const int at = atomicAdd(&fill[c], 1);
    list[start[c] + at] = (int32_t)i;
}

// order each cell's list by particle index (insertion sort; cells are small)
__global__ void k_cell_order(const int32_t *start, int ncell, int32_t *list) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int b = start[c], e = start[c + 1];
    for (int i = b + 1; i < e; ++i) {
        const int32_t v = list[i];
        int j = i - 1;
        while (j >= b && list[j] > v) {
            list[j + 1] = list[j];
            --j;
        }
        list[j + 1] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_short(const T *__restrict__ pos, const T *__restrict__ q,
                                               int64_t N, Grid g, double alpha, double rc,
                                               const int32_t *__restrict__ start,
                                               const int32_t *__restrict__ list,
                                               T *__restrict__ phi, T *__restrict__ F,
                                               double *__restrict__ epart) {
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < N) {
        double xi, yi, zi;
        const int ci = cell_of(pos, i, g, xi, yi, zi);
        const int cxi = ci % g.nx, cyi = (ci / g.nx) % g.ny, czi = ci / (g.nx * g.ny);
        const double qi = (double)q[i];
        double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
        const double two_a_sqpi = 2.0 * alpha / sqrt(3.14159265358979323846);
        int xs[3], ys[3];
        int nxs = 0, nys = 0;
        for (int d = -1; d <= 1; ++d) {
            const int c = ((cxi + d) % g.nx + g.nx) % g.nx;
            bool dup = false;
            for (int k = 0; k < nxs; ++k) dup |= xs[k] == c;
            if (!dup) xs[nxs++] = c;
        }
        for (int d = -1; d <= 1; ++d) {
            const int c = ((cyi + d) % g.ny + g.ny) % g.ny;
            bool dup = false;
            for (int k = 0; k < nys; ++k) dup |= ys[k] == c;
            if (!dup) ys[nys++] = c;
        }
        for (int dzc = -1; dzc <= 1; ++dzc) {
            const int cz_ = czi + dzc;
            if (cz_ < 0 || cz_ >= g.nz) continue;
            for (int a = 0; a < nys; ++a)
                for (int b = 0; b < nxs; ++b) {
                    const int c = (cz_ * g.ny + ys[a]) * g.nx + xs[b];
                    for (int t = start[c]; t < start[c + 1]; ++t) {
                        const int64_t j = list[t];
                        if (j == i) continue;
                        double dx = xi - (double)pos[3 * j];
                        double dy = yi - (double)pos[3 * j + 1];
                        const double dz = zi - (double)pos[3 * j + 2];
                        dx -= rint(dx / g.Lx) * g.Lx;
                        dy -= rint(dy / g.Ly) * g.Ly;
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 > rc * rc || r2 == 0.0) continue;
                        const double r = sqrt(r2);
                        const double qj = (double)q[j];
                        const double ec = erfc(alpha * r) / r;
                        ph += qj * ec;
                        const double fm = qi * qj * (ec / r + two_a_sqpi * exp(-alpha * alpha * r2) / r) / r;
                        fx += fm * dx;
                        fy += fm * dy;
                        fz += fm * dz;
                    }
                }
        }
        if (phi) phi[i] = (T)ph;
        if (F) {
            F[3 * i] = (T)fx;
            F[3 * i + 1] = (T)fy;
            F[3 * i + 2] = (T)fz;
        }
        e = qi * ph;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) epart[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_half(const double *part, int n, double *E) {
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < n; b += 256) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) E[0] = 0.5 * red[0];
}

__global__ void k_zero_i32(int32_t *a, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

template <typename T>
q2d_status short_impl(Plan *p, const T *pos, const T *q, int64_t N, T *phi, T *F, double *E) {
    Grid g;
    g.Lx = p->Lx;
    g.Ly = p->Ly;
    g.Lz = p->Lz;
    g.nx = max(1, (int)floor(p->Lx / p->rc));
    g.ny = max(1, (int)floor(p->Ly / p->rc));
    g.nz = max(1, (int)floor(p->Lz / p->rc));
    // bound the grid so the cell arrays stay modest
    while ((int64_t)g.nx * g.ny * g.nz > (int64_t)1 << 22) {
        g.nx = max(1, g.nx / 2);
        g.ny = max(1, g.ny / 2);
        g.nz = max(1, g.nz / 2);
    }
    g.hx = p->Lx / g.nx;
    g.hy = p->Ly / g.ny;
    g.hz = p->Lz / g.nz;
    const int ncell = g.nx * g.ny * g.nz;
    q2d_status st;
    if ((st = ensure(p, p->cell_count, (size_t)ncell * sizeof(int32_t))) != Q2D_OK) return st;
    if ((st = ensure(p, p->cell_start, (size_t)(2 * ncell + 1) * sizeof(int32_t))) != Q2D_OK)
        return st;
    if ((st = ensure(p, p->cell_idx, (size_t)N * sizeof(int32_t))) != Q2D_OK) return st;
    if ((st = ensure(p, p->cell_tmp, (size_t)N * sizeof(int32_t))) != Q2D_OK) return st;
    const int nb = (int)((N + 255) / 256);
    if ((st = ensure(p, p->epart, (size_t)nb * sizeof(double))) != Q2D_OK) return st;
    int32_t *count = (int32_t *)p->cell_count.p;
    int32_t *start = (int32_t *)p->cell_start.p;
    int32_t *fill = start + ncell + 1;
    k_zero_i32<<<(ncell + 255) / 256, 256, 0, p->stream>>>(count, ncell);
    k_cell_count<T><<<nb, 256, 0, p->stream>>>(pos, N, g, (int32_t *)p->cell_idx.p, count);
    k_cell_scan<<<1, 1024, 0, p->stream>>>(count, ncell, start, fill);
    k_cell_fill<<<nb, 256, 0, p->stream>>>((const int32_t *)p->cell_idx.p, N, start, fill,
                                           (int32_t *)p->cell_tmp.p);
    k_cell_order<<<(ncell + 255) / 256, 256, 0, p->stream>>>(start, ncell, (int32_t *)p->cell_tmp.p);
    k_short<T><<<nb, 256, 0, p->stream>>>(pos, q, N, g, p->alpha, p->rc, start,
                                          (const int32_t *)p->cell_tmp.p, phi, F,
                                          (double *)p->epart.p);
    if (E) k_sum_half<<<1, 256, 0, p->stream>>>((const double *)p->epart.p, nb, E);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

}  // namespace

q2d_status short_range_run(Plan *p, const void *pos, const void *q, int64_t N, void *phi, void *F,
                           double *E) {
    if (p->fp32)
        return short_impl<float>(p, (const float *)pos, (const float *)q, N, (float *)phi,
                                 (float *)F, E);
    return short_impl<double>(p, (const double *)pos, (const double *)q, N, (double *)phi,
                              (double *)F, E);
}

}  // namespace q2d
