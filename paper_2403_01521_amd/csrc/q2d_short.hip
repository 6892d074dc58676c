// Real-space part of the Ewald split (Sec. 2.2, eq. phi_s), O(N) by a cell list:
//   phi_s,i = sum over images m and j (j != i for m = 0), |r_ij + M| < r_c, of q_j erfc(alpha r)/r
//   F_s,i   = q_i sum q_j [erfc(alpha r)/r^2 + (2 alpha/sqrt(pi)) e^{-alpha^2 r^2}/r] (r_ij + M)/r
// The real-space sum is short ranged, so only neighbours within r_c count
// (the remark after eq. rckc: cell lists make it O(N)); with alpha chosen by
// eq. 59 and r_c = s/alpha (eq. rckc) the work per particle is O(1).
//
// Layout (MI355X):
//  * cells of edge >= r_c/2 in x, y, z, keyed (cy, cx, cz) with cz fastest, so
//    a row of constant cy holds its columns in x order and each column its z
//    cells; particles are sorted by cell with the library's stable radix sort
//    and copied into one (x, y, z, q) record each, in cell order;
//  * a wave takes a tile of <= 64 consecutive targets inside one row; the
//    candidates of the tile are the 5 rows cy - 2 .. cy + 2, in each the
//    columns cx_lo - 2 .. cx_hi + 2 and the z cells within 2 of the tile's,
//    visited as contiguous index ranges with an explicit periodic image shift
//    per range.  r_c <= min(Lx, Ly)/2 (checked at plan creation) puts at most
//    one image of a pair within r_c, so ranges that repeat a column with
//    another shift add nothing twice;
//  * candidates are staged 64 at a time (one coalesced record per lane, the
//    periodic shift applied) in a per-wave LDS buffer of SR_BUF records; per
//    block of 64 staged candidates every lane builds a bit mask of those within
//    r_c of its target (broadcast LDS reads), then evaluates only those pairs,
//    one per round, reading its own candidate from LDS: the erfc work is not
//    paid for the ~80% of candidates outside the sphere;
//  * FP32 plans: erfc(x) = erfcx(x) e^{-x^2}, with erfcx as a Chebyshev series
//    of degree 9 in u = 1/(1 + x/2) on [0, alpha r_c] fitted in FP64 at each
//    call from the definition (relative error below 1e-7 for alpha r_c <= 8,
//    the size of FP32 rounding; degree 12 reached 2e-10 and cost 3 more FMAs
//    per pair) and e^{-x^2}
//    shared with the force term; FP64 plans call the library erfc.  Each
//    chunk's pair terms are summed in the plan's precision and added to FP64
//    accumulators; every target sums its pairs in a fixed order, the energy in
//    a fixed reduction order (deterministic).
#include <cmath>

#include "q2d_internal.h"

namespace q2d {

namespace {

constexpr int SR_WAVES = 4;       // independent waves per work-group
constexpr int SR_BUF = 256;       // staged candidates per wave (LDS records)
constexpr int CHEB_DEG = 9;       // degree of the erfcx series (FP32 plans)

struct Grid {
    int nx, ny, nz;
    double Lx, Ly, Lz, hx, hy, hz;
};

template <typename T>
struct alignas(4 * sizeof(T)) Rec4 {
    T x, y, z, q;
};

struct ShortArgs {
    Grid g;
    double alpha, rc;
    double u0, uscale;             // t = (u - u0) * uscale - 1 maps [u0, 1] to [-1, 1]
    double cheb[CHEB_DEG + 1];     // erfcx(x) ~ sum_k cheb[k] T_k(t), cheb[0] halved
    int ntile_max;
};

template <typename T>
__global__ __launch_bounds__(256) void k_cell_stage(const T *__restrict__ pos,
                                                    const T *__restrict__ q, int64_t N, Grid g,
                                                    uint32_t *__restrict__ keys,
                                                    int32_t *__restrict__ vals,
                                                    Rec4<T> *__restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    T x = pos[3 * i], y = pos[3 * i + 1];
    const T z = pos[3 * i + 2];
    x -= floor(x / (T)g.Lx) * (T)g.Lx;
    y -= floor(y / (T)g.Ly) * (T)g.Ly;
    const int cx = min(g.nx - 1, max(0, (int)((double)x / g.hx)));
    const int cy = min(g.ny - 1, max(0, (int)((double)y / g.hy)));
    const int cz = min(g.nz - 1, max(0, (int)((double)z / g.hz)));
    keys[i] = ((uint32_t)cy * (uint32_t)g.nx + (uint32_t)cx) * (uint32_t)g.nz + (uint32_t)cz;
    vals[i] = (int32_t)i;
    rec[i] = Rec4<T>{x, y, z, q[i]};
}

template <typename T>
__global__ __launch_bounds__(256) void k_cell_gather(const Rec4<T> *__restrict__ rec,
                                                     const int32_t *__restrict__ perm, int64_t N,
                                                     Rec4<T> *__restrict__ srec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) srec[i] = rec[perm[i]];
}

// start[c] = first sorted index with key >= c, for c in [0, ncell]
__global__ __launch_bounds__(256) void k_cell_bounds(const uint32_t *__restrict__ key, int64_t N,
                                                     uint32_t ncell, int32_t *__restrict__ start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    const uint32_t lo = i == 0 ? 0u : key[i - 1] + 1u;
    const uint32_t hi = i == N ? ncell : key[i];
    for (uint32_t c = lo; c <= hi; ++c) start[c] = (int32_t)i;
}

// tiles of <= 64 targets per row: base[r] = tiles before row r, base[ny] = total
__global__ __launch_bounds__(1024) void k_row_tiles(const int32_t *__restrict__ start, int ny,
                                                    int row_cells, int32_t *__restrict__ base) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int per = (ny + 1023) / 1024;
    const int b0 = min(t * per, ny), b1 = min(b0 + per, ny);
    int32_t s = 0;
    for (int r = b0; r < b1; ++r)
        s += (start[(r + 1) * row_cells] - start[r * row_cells] + WAVE - 1) / WAVE;
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = t ? part[t - 1] : 0;
    for (int r = b0; r < b1; ++r) {
        base[r] = run;
        run += (start[(r + 1) * row_cells] - start[r * row_cells] + WAVE - 1) / WAVE;
    }
    if (t == 1023) base[ny] = part[1023];
}


// erfc(x) and e^{-x^2} for 0 <= x <= alpha r_c
__device__ inline void erfc_gauss(const ShortArgs &a, float x, float &ec, float &g) {
    g = __builtin_amdgcn_exp2f(-1.4426950408889634f * x * x);
    const float u = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
    const float t = fmaf((float)a.uscale, u - (float)a.u0, -1.0f), t2 = 2.0f * t;
    float b1 = 0.f, b2 = 0.f;
#pragma unroll
    for (int k = CHEB_DEG; k >= 1; --k) {
        const float b0 = fmaf(t2, b1, (float)a.cheb[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    ec = fmaf(t, b1, (float)a.cheb[0] - b2) * g;
}
__device__ inline void erfc_gauss(const ShortArgs &, double x, double &ec, double &g) {
    g = exp(-x * x);
    ec = erfc(x);
}
__device__ inline float rsq(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ inline double rsq(double v) { return 1.0 / sqrt(v); }

// pair term of one candidate: accumulate q_j erfc(alpha r)/r and the force
// factor q_j [erfc/r^2 + (2 alpha/sqrt(pi)) e^{-alpha^2 r^2}/r] / r along d
template <typename T>
__device__ inline void pair_term(const ShortArgs &a, const Rec4<T> &me, const Rec4<T> &c,
                                 bool has, T alpha, T c2a, T &sp, T &sfx, T &sfy, T &sfz) {
    const T dx = me.x - c.x, dy = me.y - c.y, dz = me.z - c.z;
    T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    r2 = has ? r2 : (T)1;
    const T ri = rsq(r2);
    T ec, gs;
    erfc_gauss(a, alpha * (r2 * ri), ec, gs);
    const T qj = has ? c.q : (T)0;
    const T er = ec * ri;
    sp = fma(qj, er, sp);
    const T fm = qj * fma(c2a, gs, er) * (ri * ri);
    sfx = fma(fm, dx, sfx);
    sfy = fma(fm, dy, sfy);
    sfz = fma(fm, dz, sfz);
}

// A wave per tile of <= 64 targets (lane = target).  Candidates are staged in
// a per-wave LDS buffer of SR_BUF records with their periodic shift applied
// (coalesced loads, one record per lane); when the buffer is full (and at the
// end) it is processed block by block: every lane builds its in-range bit mask
// over 64 candidates from broadcast LDS reads, then walks its own candidates,
// one per round, reading each from LDS (no lane permutes, no readlane chains).
// Each lane sums its pairs in a fixed order (deterministic).
template <typename T>
__global__ __launch_bounds__(SR_WAVES *WAVE) void k_short_tiles(
    const ShortArgs a, const Rec4<T> *__restrict__ srec, const uint32_t *__restrict__ skey,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ start,
    const int32_t *__restrict__ row_base, T *__restrict__ phi, T *__restrict__ F,
    double *__restrict__ tile_e) {
    __shared__ Rec4<T> buf_all[SR_WAVES][SR_BUF];
    const Grid &g = a.g;
    const int lane = threadIdx.x % WAVE, wv = (int)(threadIdx.x / WAVE);
    Rec4<T> *buf = buf_all[wv];
    const int tile = blockIdx.x * SR_WAVES + wv;
    if (tile >= a.ntile_max) return;
    const int ntiles = row_base[g.ny];
    if (tile >= ntiles) {
        if (lane == 0) tile_e[tile] = 0.0;
        return;
    }
    // the tile's row: last r with row_base[r] <= tile (rows may hold no tile)
    int lo = 0, hi = g.ny - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_base[mid] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int cy = lo;
    const int row_cells = g.nx * g.nz;
    const int i0 = start[cy * row_cells] + WAVE * (tile - row_base[cy]);
    const int i1 = min(i0 + WAVE, start[(cy + 1) * row_cells]);
    const int nt = i1 - i0;  // 1..64 targets
    const bool valid = lane < nt;
    const int i = valid ? i0 + lane : i0;
    const Rec4<T> me = srec[i];
    const uint32_t key = skey[i];
    const int cx = (int)((key / (uint32_t)g.nz) % (uint32_t)g.nx), cz = (int)(key % (uint32_t)g.nz);
    // columns of the tile (targets are ordered by column) and its z cells
    const int cx_lo = __builtin_amdgcn_readlane(cx, 0);
    const int cx_hi = __builtin_amdgcn_readlane(cx, nt - 1);
    int zmn = cz, zmx = cz;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        zmn = min(zmn, __shfl_xor(zmn, o));
        zmx = max(zmx, __shfl_xor(zmx, o));
    }
    const int z0 = max(0, zmn - 2), z1 = min(g.nz - 1, zmx + 2);
    const bool zfull = z0 == 0 && z1 == g.nz - 1;
    const T rc2 = (T)(a.rc * a.rc);
    const T alpha = (T)a.alpha;
    const T c2a = (T)(2.0 * a.alpha / 1.7724538509055160273);
    double aphi = 0.0, afx = 0.0, afy = 0.0, afz = 0.0;
    int fill = 0;  // staged candidates (wave-uniform)

    // the staged candidates [0, fill), one block of 64 at a time: this lane's
    // in-range mask over the block (broadcast LDS reads), then its pairs, one
    // per round, each candidate read from LDS
    auto flush = [&]() {
        // (the wave's LDS accesses run in program order: the staged records
        // of every lane are in place for the reads below)
        __builtin_amdgcn_wave_barrier();
        T sp = 0, sfx = 0, sfy = 0, sfz = 0;
        for (int b0 = 0; b0 < fill; b0 += WAVE) {
            const Rec4<T> *blk = buf + b0;
            const int nb = min(WAVE, fill - b0);
            uint32_t mlo = 0, mhi = 0;
            for (int j = 0; j < nb; ++j) {
                const Rec4<T> c = blk[j];  // same address on every lane
                const T dx = me.x - c.x, dy = me.y - c.y, dz = me.z - c.z;
                const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                const uint32_t bit = (r2 < rc2 && r2 > (T)0) ? 1u : 0u;
                if (j < 32)
                    mlo |= bit << j;
                else
                    mhi |= bit << (j - 32);
            }
            if (!valid) mlo = mhi = 0;
            while (__any((mlo | mhi) != 0)) {
                const bool has = (mlo | mhi) != 0;
                const int j = mlo ? __builtin_ctz(mlo) : (mhi ? 32 + __builtin_ctz(mhi) : 0);
                if (mlo)
                    mlo &= mlo - 1;
                else if (mhi)
                    mhi &= mhi - 1;
                pair_term(a, me, blk[j], has, alpha, c2a, sp, sfx, sfy, sfz);
            }
        }
        aphi += (double)sp;
        afx += (double)sfx;
        afy += (double)sfy;
        afz += (double)sfz;
        fill = 0;
    };

    // stage the candidates [b, e) seen through the periodic shift (sx, sy)
    auto range = [&](int b, int e, T sx, T sy) {
        for (int c0 = b; c0 < e; c0 += WAVE) {
            const int nc = min(WAVE, e - c0);
            if (fill + nc > SR_BUF) flush();
            if (lane < nc) {
                Rec4<T> c = srec[c0 + lane];
                c.x += sx;
                c.y += sy;
                buf[fill + lane] = c;
            }
            fill += nc;
        }
    };

    for (int dy = -2; dy <= 2; ++dy) {
        const int yr = cy + dy;
        const int cyr = ((yr % g.ny) + g.ny) % g.ny;
        const T sy = (T)((double)((yr - cyr) / g.ny) * g.Ly);
        const int row0 = cyr * row_cells;
        // column runs with one shift each
        int xa = cx_lo - 2;
        const int xb = cx_hi + 2;
        while (xa <= xb) {
            const int per = xa >= 0 ? xa / g.nx : -((-xa + g.nx - 1) / g.nx);  // floor(xa / nx)
            const int run_end = min(xb, (per + 1) * g.nx - 1);
            const int ca = xa - per * g.nx, cb = run_end - per * g.nx;
            const T sx = (T)((double)per * g.Lx);
            if (zfull) {
                range(start[row0 + ca * g.nz], start[row0 + cb * g.nz + g.nz], sx, sy);
            } else {
                for (int c = ca; c <= cb; ++c)
                    range(start[row0 + c * g.nz + z0], start[row0 + c * g.nz + z1 + 1], sx, sy);
            }
            xa = run_end + 1;
        }
    }
    if (fill > 0) flush();
    if (valid) {
        const int o = perm[i];
        if (phi) phi[o] = (T)aphi;
        if (F) {
            const double qi = (double)me.q;
            F[3 * (int64_t)o] = (T)(qi * afx);
            F[3 * (int64_t)o + 1] = (T)(qi * afy);
            F[3 * (int64_t)o + 2] = (T)(qi * afz);
        }
    }
    // the tile's share of 1/2 sum q_i phi_i, reduced in a fixed order
    double e = valid ? (double)me.q * aphi : 0.0;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) e += __shfl_xor(e, o);
    if (lane == 0) tile_e[tile] = e;
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

// Chebyshev coefficients of erfcx(x) = e^{x^2} erfc(x) as a series in
// t = (u - u0) * uscale - 1, u = 1/(1 + x/2), for x in [0, X] (interpolation
// at the CHEB_DEG + 1 Chebyshev points, FP64)
void erfcx_series(double X, ShortArgs &a) {
    const double PI = 3.14159265358979323846;
    const int n = CHEB_DEG + 1;
    a.u0 = 1.0 / (1.0 + 0.5 * X);
    a.uscale = 2.0 / (1.0 - a.u0);
    double f[CHEB_DEG + 1];
    for (int k = 0; k < n; ++k) {
        const double t = std::cos(PI * (k + 0.5) / n);
        const double u = a.u0 + (t + 1.0) / a.uscale;
        const double x = 2.0 * (1.0 / u - 1.0);
        f[k] = std::exp(x * x) * std::erfc(x);
    }
    for (int j = 0; j < n; ++j) {
        double c = 0.0;
        for (int k = 0; k < n; ++k) c += f[k] * std::cos(PI * j * (k + 0.5) / n);
        a.cheb[j] = 2.0 / n * c;
    }
    a.cheb[0] *= 0.5;
}

template <typename T>
q2d_status short_impl(Plan *p, const T *pos, const T *q, int64_t N, T *phi, T *F, double *E) {
    Grid g;
    g.Lx = p->Lx;
    g.Ly = p->Ly;
    g.Lz = p->Lz;
    // cell edges >= r_c / 2 (a +-2 cell stencil covers r_c); coarser cells
    // when the grid would have far more cells than particles
    g.nx = std::max(1, (int)std::floor(2.0 * p->Lx / p->rc));
    g.ny = std::max(1, (int)std::floor(2.0 * p->Ly / p->rc));
    g.nz = std::max(1, (int)std::floor(2.0 * p->Lz / p->rc));
    const int64_t cap = std::max<int64_t>(4 * N, 4096);
    while ((int64_t)g.nx * g.ny * g.nz > cap) {
        if (g.nx >= g.ny && g.nx >= g.nz)
            g.nx = std::max(1, g.nx / 2);
        else if (g.ny >= g.nz)
            g.ny = std::max(1, g.ny / 2);
        else
            g.nz = std::max(1, g.nz / 2);
    }
    g.hx = p->Lx / g.nx;
    g.hy = p->Ly / g.ny;
    g.hz = p->Lz / g.nz;
    const uint32_t ncell = (uint32_t)g.nx * g.ny * g.nz;
    int bits = 1;
    while (bits < 32 && ((uint64_t)1 << bits) < ncell) ++bits;
    const int passes = (bits + 7) / 8;
    const int ntile_max = (int)((N + WAVE - 1) / WAVE) + g.ny;
    q2d_status st;
    if ((st = ensure(p, p->keys_a, N * sizeof(uint32_t))) != Q2D_OK ||
        (st = ensure(p, p->keys_b, N * sizeof(uint32_t))) != Q2D_OK ||
        (st = ensure(p, p->vals_a, N * sizeof(int32_t))) != Q2D_OK ||
        (st = ensure(p, p->vals_b, N * sizeof(int32_t))) != Q2D_OK ||
        (st = ensure(p, p->recs, N * sizeof(Rec4<T>))) != Q2D_OK ||
        (st = ensure(p, p->cell_rec, N * sizeof(Rec4<T>))) != Q2D_OK ||
        (st = ensure(p, p->cell_start, ((size_t)ncell + 1) * sizeof(int32_t))) != Q2D_OK ||
        (st = ensure(p, p->row_tiles, ((size_t)g.ny + 1) * sizeof(int32_t))) != Q2D_OK ||
        (st = ensure(p, p->tile_e, (size_t)ntile_max * sizeof(double))) != Q2D_OK)
        return st;
    // the long-range sort shares these buffers: its order is no longer current
    p->inv_ready = false;
    const int nb = (int)((N + 255) / 256);
    k_cell_stage<T><<<nb, 256, 0, p->stream>>>(pos, q, N, g, (uint32_t *)p->keys_a.p,
                                               (int32_t *)p->vals_a.p, (Rec4<T> *)p->recs.p);
    uint32_t *skey = nullptr;
    int32_t *perm = nullptr;
    if ((st = radix_sort_u32(p, N, passes, &skey, &perm)) != Q2D_OK) return st;
    k_cell_gather<T><<<nb, 256, 0, p->stream>>>((const Rec4<T> *)p->recs.p, perm, N,
                                                (Rec4<T> *)p->cell_rec.p);
    int32_t *start = (int32_t *)p->cell_start.p;
    k_cell_bounds<<<(int)((N + 1 + 255) / 256), 256, 0, p->stream>>>(skey, N, ncell, start);
    k_row_tiles<<<1, 1024, 0, p->stream>>>(start, g.ny, g.nx * g.nz, (int32_t *)p->row_tiles.p);
    ShortArgs a{};
    a.g = g;
    a.alpha = p->alpha;
    a.rc = p->rc;
    a.ntile_max = ntile_max;
    erfcx_series(p->alpha * p->rc, a);
    const int nblk = (ntile_max + SR_WAVES - 1) / SR_WAVES;
    k_short_tiles<T><<<nblk, SR_WAVES * WAVE, 0, p->stream>>>(
        a, (const Rec4<T> *)p->cell_rec.p, skey, perm, start, (const int32_t *)p->row_tiles.p, phi,
        F, (double *)p->tile_e.p);
    if (E) k_sum_half<<<1, 256, 0, p->stream>>>((const double *)p->tile_e.p, ntile_max, E);
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
