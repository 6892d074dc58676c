// Stable z-sort of the particles and staging of the sorted structure-of-arrays.
//
// The recursion of Sec. 3.2 needs the particles ordered by height z (i > j
// <=> z_i >= z_j) so that every exponent in the scans is non-positive (the
// stability remark after eq. 35).  Sort keys are the IEEE bit patterns of z:
// for z >= 0 they order like the numbers (z + 0 turns -0 into +0).  The order
// is that of the pairs (key, input index): equal heights keep input order.
//
// The radix sort: least-significant digit first, 8-bit digits, each pass
// stable.  One pass = (1) per-tile digit histograms, (2) per-digit exclusive
// scan over tiles, (3) a stable scatter that ranks keys inside a tile with
// wave ballots.
//
// Single systems up to ~1.2e6 particles (FP32; ~6e5 FP64) take a bucket sort
// built from the same parts: one stable scatter whose digit is the z bucket
// floor(256 z / L_z) (monotone in z), then one work-group per bucket runs the
// radix sort in LDS on the bucket's keys minus its smallest key, with only as
// many passes as that span needs, and stages its part of the sorted arrays.
// The bucket arrives in input order, so the result is the (key, index)
// order.  A bucket too large for LDS (strongly clustered heights) is sorted in
// global memory by a bitonic network.
#include "q2d_internal.h"

namespace q2d {

namespace {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;

__device__ inline uint32_t zkey(float z) { return __float_as_uint(z + 0.0f); }
__device__ inline uint64_t zkey(double z) {
    return static_cast<uint64_t>(__double_as_longlong(z + 0.0));
}

// Status bits in the device status word (bit q2d_status).
__device__ inline void set_status(int *st, int code) { atomicOr(st, 1 << code); }

// z buckets of the bucket sort: floor(z * scale) clamped to [0, nb - 1], with
// scale = nb / L_z rounded once in the keys' precision; monotone in z (a
// product by a positive constant and the floor both keep order)
constexpr int BK_NB = 256;  // buckets: one digit of the scatter below
template <typename T>
__device__ inline uint32_t zbucket(T z, T scale, uint32_t nb) {
    const T v = z * scale;
    return v >= (T)nb ? nb - 1 : (v > (T)0 ? (uint32_t)v : 0u);
}
__device__ inline float key_z(uint32_t k) { return __uint_as_float(k); }
__device__ inline double key_z(uint64_t k) { return __longlong_as_double((long long)k); }

// one particle's position and charge in one aligned record: the gather after
// the sort then reads one record per particle instead of two scattered ones
template <typename T>
struct alignas(4 * sizeof(T)) Rec {
    T x, y, z, q;
};

// One sort tile per work-group (SORT_ITEMS particles per thread, coalesced):
// keys, identity values and records in input order, plus the tile's
// histogram of the first digit, the z bucket (BUCKET) or the key's low byte,
// so the first scatter needs no histogram launch of its own.
template <typename T, typename K, bool BUCKET>
__global__ __launch_bounds__(SORT_THREADS) void k_stage(
    const T *__restrict__ pos, const T *__restrict__ q, int64_t N, K *__restrict__ keys,
    int32_t *__restrict__ vals, Rec<T> *__restrict__ rec, uint32_t *__restrict__ hist, int ntiles,
    T scale, double Lz, int validate, int *status, double *qsums) {
    __shared__ uint32_t h[256];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    double qs = 0.0, qa = 0.0;
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = base + r * SORT_THREADS + t;
        if (i < N) {
            const T z = pos[3 * i + 2];
            const K key = zkey(z);
            keys[i] = key;
            vals[i] = (int32_t)i;
            rec[i] = Rec<T>{pos[3 * i], pos[3 * i + 1], z, q[i]};
            atomicAdd(&h[BUCKET ? zbucket(key_z(key), scale, (uint32_t)BK_NB)
                                : (uint32_t)key & 255u],
                      1u);
            if (validate) {
                const T x = pos[3 * i], y = pos[3 * i + 1];
                const double qv = (double)q[i];
                qs += qv;
                qa += fabs(qv);
                const bool finite = isfinite((double)x) && isfinite((double)y) &&
                                    isfinite((double)z) && isfinite(qv);
                if (!finite || !((double)z >= 0.0 && (double)z <= Lz))
                    set_status(status, Q2D_EOUTOFBOX);
            }
        }
    }
    __syncthreads();
    hist[(int64_t)t * ntiles + blockIdx.x] = h[t];
    if (validate) {
        // block sums of q and |q| for the neutrality check (order of the final
        // atomic adds only affects a threshold test)
        __shared__ double s1[SORT_THREADS], s2[SORT_THREADS];
        s1[t] = qs;
        s2[t] = qa;
        __syncthreads();
        for (int hh = SORT_THREADS / 2; hh > 0; hh >>= 1) {
            if (t < hh) {
                s1[t] += s1[t + hh];
                s2[t] += s2[t + hh];
            }
            __syncthreads();
        }
        if (t == 0) {
            atomicAdd(&qsums[0], s1[0]);
            atomicAdd(&qsums[1], s2[0]);
        }
    }
}

__global__ void k_neutral_check(const double *qsums, int *status) {
    if (fabs(qsums[0]) > 1e-6 * qsums[1] + 1e-300) atomicOr(status, 1 << Q2D_ENONNEUTRAL);
}

__global__ void k_zero2(double *a) {
    a[0] = 0.0;
    a[1] = 0.0;
}

template <typename K>
__global__ __launch_bounds__(SORT_THREADS) void k_hist(const K *__restrict__ keys, int64_t N,
                                                       int shift, uint32_t *__restrict__ hist,
                                                       int ntiles) {
    __shared__ uint32_t h[256];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = base + r * SORT_THREADS + t;
        if (i < N) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * ntiles + blockIdx.x] = h[t];
}

// One block per digit: exclusive scan of hist[d][*] over tiles, total in tot[d].
__global__ __launch_bounds__(256) void k_scan_digit(uint32_t *__restrict__ hist, int ntiles,
                                                    uint32_t *__restrict__ tot) {
    __shared__ uint32_t part[256];
    const int d = blockIdx.x, t = threadIdx.x;
    uint32_t *row = hist + (int64_t)d * ntiles;
    const int per = (ntiles + 255) / 256;
    const int b0 = min(t * per, ntiles), b1 = min(b0 + per, ntiles);
    uint32_t s = 0;
    for (int b = b0; b < b1; ++b) s += row[b];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 256 partial sums
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t v = (t >= off) ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = (t > 0) ? part[t - 1] : 0u;
    for (int b = b0; b < b1; ++b) {
        const uint32_t c = row[b];
        row[b] = run;
        run += c;
    }
    if (t == 255) tot[d] = part[255];
}

// digit of a key: its byte at shift, or its z bucket (BUCKET; scale as in k_stage)
template <typename K, bool BUCKET>
__device__ inline uint32_t key_digit(K k, int shift, double scale) {
    if (BUCKET) {
        using Z = decltype(key_z(k));
        return zbucket(key_z(k), (Z)scale, (uint32_t)BK_NB);
    }
    return (uint32_t)(k >> shift) & 255u;
}

template <typename K, bool BUCKET = false>
__global__ __launch_bounds__(SORT_THREADS) void k_scatter(
    const K *__restrict__ kin, const int32_t *__restrict__ vin, K *__restrict__ kout,
    int32_t *__restrict__ vout, int64_t N, int shift, const uint32_t *__restrict__ hist,
    const uint32_t *__restrict__ tot, int ntiles, double scale = 0.0) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[SORT_THREADS / WAVE][256];
    const int t = threadIdx.x;
    const int wave = t / WAVE, lane = t % WAVE;
    // digit base = (keys with smaller digits) + (same digit in earlier tiles)
    base[t] = tot[t];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t v = (t >= off) ? base[t - off] : 0u;
        __syncthreads();
        base[t] += v;
        __syncthreads();
    }
    const uint32_t excl = base[t] - tot[t];
    __syncthreads();
    base[t] = excl + hist[(int64_t)t * ntiles + blockIdx.x];
    run[t] = 0;
#pragma unroll
    for (int w = 0; w < SORT_THREADS / WAVE; ++w) wc[w][t] = 0;
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile0 = (int64_t)blockIdx.x * SORT_TILE;
    // the tile's keys and values, loaded up front (one memory latency, not one per round)
    K ks[SORT_ITEMS];
    int32_t vs[SORT_ITEMS];
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = tile0 + r * SORT_THREADS + t;
        ks[r] = i < N ? kin[i] : (K)0;
        vs[r] = i < N ? vin[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = tile0 + r * SORT_THREADS + t;
        const bool valid = i < N;
        const K k = ks[r];
        const int32_t v = vs[r];
        const uint32_t d = key_digit<K, BUCKET>(k, shift, scale);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0) wc[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = base[d] + run[d] + rank;
            for (int w = 0; w < wave; ++w) off += wc[w][d];
            kout[off] = k;
            vout[off] = v;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < SORT_THREADS / WAVE; ++w) {
            add += wc[w][t];
            wc[w][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

template <typename T>
struct Fix;
template <>
struct Fix<float> {
    using U = uint32_t;
    __device__ static U frac(double v) {
        // fixed-point fraction of a turn: round(frac(v) * 2^32) mod 2^32
        double f = v - floor(v);
        return (U)(uint64_t)llrint(f * 4294967296.0);
    }
};
template <>
struct Fix<double> {
    using U = double;
    __device__ static U frac(double v) { return v - floor(v); }
};

// ---------------------------------------------------------------------------
// per-bucket sort of the bucket sort (one work-group per bucket)
// ---------------------------------------------------------------------------
constexpr int BK_THREADS = 1024;
constexpr int BK_WAVES = BK_THREADS / WAVE;
// largest bucket sorted in LDS (two key and two index buffers): 144 KB of LDS
// with 32-bit keys, 112 KB with 64-bit keys
template <typename K>
constexpr int bk_cap() {
    return sizeof(K) == 4 ? 8192 : 4096;
}

// (key, index) order: a total order, so a sorted bucket is unique
template <typename K>
__device__ inline bool bk_less(K ka, int32_t ia, K kb, int32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// Bitonic network with every comparator ascending (the first half-cleaner of a
// merge of size 2^lk pairs offsets o and 2^lk - 1 - o): it sorts any length n
// by treating the positions n .. m - 1 (m = next power of two) as +infinity,
// which never move, so comparators that reach past n are skipped.  Comparator
// c of the stage (merge 2^lk, distance 2^lj) joins positions i < p.  Used in
// global memory for buckets too large for LDS.
__device__ inline void bk_pair(int c, int lk, int lj, int &i, int &p) {
    const int j = 1 << lj;
    if (lj == lk - 1) {
        const int blk = c >> lj, o = c & (j - 1);
        i = (blk << lk) + o;
        p = (blk << lk) + (1 << lk) - 1 - o;
    } else {
        i = ((c >> lj) << (lj + 1)) + (c & (j - 1));
        p = i + j;
    }
}

template <typename K>
__device__ inline void bk_bitonic(K *key, int32_t *idx, int n) {
    int lm = 0;
    while ((1 << lm) < n) ++lm;
    const int half = (1 << lm) >> 1;
    for (int lk = 1; lk <= lm; ++lk)
        for (int lj = lk - 1; lj >= 0; --lj) {
            for (int c = threadIdx.x; c < half; c += BK_THREADS) {
                int i, p;
                bk_pair(c, lk, lj, i, p);
                if (p < n) {
                    const K ki = key[i], kp = key[p];
                    const int32_t ii = idx[i], ip = idx[p];
                    if (bk_less<K>(kp, ip, ki, ii)) {
                        key[i] = kp;
                        key[p] = ki;
                        idx[i] = ip;
                        idx[p] = ii;
                    }
                }
            }
            __syncthreads();
        }
}

// LDS of the per-bucket radix sort
template <typename K>
struct BkLds {
    static constexpr int CAP = bk_cap<K>();
    K ka[CAP], kb[CAP];
    int32_t ia[CAP], ib[CAP];
    uint32_t hw[BK_WAVES][256];   // per-wave digit counts of a pass
    uint16_t pos[BK_WAVES][256];  // next output position of (wave, digit)
    uint32_t wtot[4];
    K kred[2][BK_WAVES];
    uint32_t below[BK_WAVES];
};

// One stable LSD pass in LDS on the digit ((key - kmin) >> shift) & 255.  Wave
// w owns the contiguous slice [w0, w1) of the (index-ordered) elements: the
// per-wave counts and one prefix over (digit, wave) give every wave its
// output positions, then each wave ranks its slice in rounds of 64 with
// ballots and advances its own positions (no work-group barrier per round).
template <typename K>
__device__ inline void bk_radix_pass(const K *ks, const int32_t *is, K *kd, int32_t *id, int n,
                                     K kmin, int shift, BkLds<K> &L) {
    const int t = threadIdx.x, lane = t % WAVE, wave = t / WAVE;
    const int per = (n + BK_WAVES - 1) / BK_WAVES;
    const int w0 = min(wave * per, n), w1 = min(w0 + per, n);
    auto digit = [&](K k) { return (uint32_t)((k - kmin) >> shift) & 255u; };
    for (int d = lane; d < 256; d += WAVE) L.hw[wave][d] = 0u;
    for (int x = w0 + lane; x < w1; x += WAVE) atomicAdd(&L.hw[wave][digit(ks[x])], 1u);
    __syncthreads();
    // digit totals, their exclusive scan (4 waves of 64 digits), then the
    // (digit, wave) positions
    uint32_t td = 0, v = 0;
    if (t < 256) {
#pragma unroll
        for (int w = 0; w < BK_WAVES; ++w) td += L.hw[w][t];
        v = td;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            const uint32_t u = __shfl_up(v, off);
            if (lane >= off) v += u;
        }
        if (lane == WAVE - 1) L.wtot[wave] = v;
    }
    __syncthreads();
    if (t < 256) {
        uint32_t off = v - td;
        for (int w = 0; w < wave; ++w) off += L.wtot[w];
#pragma unroll
        for (int w = 0; w < BK_WAVES; ++w) {
            L.pos[w][t] = (uint16_t)off;
            off += L.hw[w][t];
        }
    }
    __syncthreads();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int r0 = w0; r0 < w1; r0 += WAVE) {
        const int x = r0 + lane;
        const bool valid = x < w1;
        const K k = valid ? ks[x] : kmin;
        const int32_t ix = valid ? is[x] : 0;
        const uint32_t d = digit(k);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bb = 0; bb < 8; ++bb) {
            const bool bit = (d >> bb) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        // every lane reads its digit's position before the group's first lane
        // advances it (one wave: its LDS operations complete in order)
        const uint32_t at = (uint32_t)L.pos[wave][d] + rank;
        if (valid) {
            kd[at] = k;
            id[at] = ix;
        }
        if (valid && rank == 0) L.pos[wave][d] = (uint16_t)(at + (uint32_t)__popcll(peers));
    }
    __syncthreads();
}

// One work-group per bucket: sort it by (key, index).  The bucket is the scan's
// digit total tot[b] long and starts at the sum of the totals below it; it
// holds its particles in input order (the bucket scatter is stable), so a
// stable radix sort on the keys leaves it in (key, index) order.  Only the
// bits that vary inside the bucket are sorted (keys minus the smallest).  The
// work-group then stages its bucket's part of the sorted arrays (the gather:
// one record per particle through the permutation).
template <typename T, typename K>
__global__ __launch_bounds__(BK_THREADS) void k_bsort(K *__restrict__ keys,
                                                     int32_t *__restrict__ vals,
                                                     const uint32_t *__restrict__ tot,
                                                     const Rec<T> *__restrict__ rec, double Lx,
                                                     double Ly, typename Fix<T>::U *__restrict__ ux,
                                                     typename Fix<T>::U *__restrict__ uy,
                                                     T *__restrict__ zs, T *__restrict__ qs) {
    __shared__ BkLds<K> L;
    const int b = blockIdx.x, t = threadIdx.x, lane = t % WAVE, wave = t / WAVE;
    const int n = (int)tot[b];
    if (n == 0) return;
    // start = sum of tot[0 .. b - 1] (fixed order: wave sums, then the waves)
    uint32_t v = t < b ? tot[t] : 0u;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) L.below[wave] = v;
    __syncthreads();
    int64_t base = 0;
#pragma unroll
    for (int w = 0; w < BK_WAVES; ++w) base += L.below[w];
    // sorted position x of the bucket holds input particle o
    auto gather = [&](int x, int32_t o) {
        const Rec<T> r = rec[o];
        const int64_t i = base + x;
        ux[i] = Fix<T>::frac((double)r.x / Lx);
        uy[i] = Fix<T>::frac((double)r.y / Ly);
        zs[i] = r.z + (T)0;
        qs[i] = r.q;
    };
    if (n == 1) {
        if (t == 0) gather(0, vals[base]);
        return;
    }
    if (n > BkLds<K>::CAP) {
        // strongly clustered heights: in place in the work-group's own
        // global-memory region (visible to its threads across the barriers)
        bk_bitonic<K>(keys + base, vals + base, n);
        for (int x = t; x < n; x += BK_THREADS) gather(x, vals[base + x]);
        return;
    }
    K lo = ~(K)0, hi = (K)0;
    for (int x = t; x < n; x += BK_THREADS) {
        const K k = keys[base + x];
        L.ka[x] = k;
        L.ia[x] = vals[base + x];
        lo = min(lo, k);
        hi = max(hi, k);
    }
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        lo = min(lo, (K)__shfl_xor(lo, off));
        hi = max(hi, (K)__shfl_xor(hi, off));
    }
    if (lane == 0) {
        L.kred[0][wave] = lo;
        L.kred[1][wave] = hi;
    }
    __syncthreads();
    K kmin = L.kred[0][0], kmax = L.kred[1][0];
#pragma unroll
    for (int w = 1; w < BK_WAVES; ++w) {
        kmin = min(kmin, L.kred[0][w]);
        kmax = max(kmax, L.kred[1][w]);
    }
    const K span = kmax - kmin;
    if (span == 0) {
        // one key: the bucket is in input order already
        for (int x = t; x < n; x += BK_THREADS) gather(x, L.ia[x]);
        return;
    }
    const int bits = (int)(8 * sizeof(K)) -
                     (sizeof(K) == 4 ? __clz((uint32_t)span) : __clzll((unsigned long long)span));
    const int passes = (bits + 7) / 8;
    K *sk = L.ka, *dk = L.kb;
    int32_t *si = L.ia, *di = L.ib;
    for (int p = 0; p < passes; ++p) {
        bk_radix_pass<K>(sk, si, dk, di, n, kmin, 8 * p, L);
        K *tk = sk;
        sk = dk;
        dk = tk;
        int32_t *ti = si;
        si = di;
        di = ti;
    }
    for (int x = t; x < n; x += BK_THREADS) {
        keys[base + x] = sk[x];
        vals[base + x] = si[x];
        gather(x, si[x]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(const Rec<T> *__restrict__ rec,
                                                const int32_t *__restrict__ perm, int64_t N,
                                                double Lx, double Ly,
                                                typename Fix<T>::U *__restrict__ ux,
                                                typename Fix<T>::U *__restrict__ uy,
                                                T *__restrict__ zs, T *__restrict__ qs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const Rec<T> r = rec[perm[i]];
    ux[i] = Fix<T>::frac((double)r.x / Lx);
    uy[i] = Fix<T>::frac((double)r.y / Ly);
    zs[i] = r.z + (T)0;
    qs[i] = r.q;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather1(const T *__restrict__ in,
                                                 const int32_t *__restrict__ perm, int64_t N,
                                                 T *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) out[i] = in[perm[i]];
}

template <typename T, typename K>
void sort_reqs_t(Plan *p, int64_t N, Reqs &r) {
    using U = typename Fix<T>::U;
    const int ntiles = (int)((N + SORT_TILE - 1) / SORT_TILE);
    r.add(p->keys_a, N * sizeof(K));
    r.add(p->keys_b, N * sizeof(K));
    r.add(p->vals_a, N * sizeof(int32_t));
    r.add(p->vals_b, N * sizeof(int32_t));
    r.add(p->hist, ((size_t)256 * ntiles + 256) * sizeof(uint32_t));
    r.add(p->s_ux, N * sizeof(U));
    r.add(p->s_uy, N * sizeof(U));
    r.add(p->s_z, N * sizeof(T));
    r.add(p->s_q, N * sizeof(T));
    r.add(p->recs, N * sizeof(Rec<T>));
}

template <typename T, typename K>
q2d_status sort_impl(Plan *p, const void *pos_v, const void *q_v, int64_t N) {
    const T *pos = (const T *)pos_v;
    const T *q = (const T *)q_v;
    using U = typename Fix<T>::U;
    q2d_status st;
    Reqs req;
    sort_reqs_t<T, K>(p, N, req);
    if ((st = ensure_all(p, req)) != Q2D_OK) return st;
    const int ntiles = (int)((N + SORT_TILE - 1) / SORT_TILE);
    // the bucket sort while the average bucket stays well inside the LDS sort
    // (denser layers and fluctuations then fit as well); Q2D_RADIX_SORT=1
    // takes the radix sort at any size (both give the same order)
    const bool bucket = N <= (int64_t)BK_NB * bk_cap<K>() * 6 / 10 &&
                        env_int("Q2D_RADIX_SORT", 0) == 0;
    // bucket scale BK_NB / L_z, rounded once in the keys' precision
    const double scale = (double)BK_NB / p->Lz;

    int *status = (int *)p->status.p;
    double *qsums = (double *)((char *)p->status.p + 16);
    const int nb = (int)((N + 255) / 256);
    if (p->opts.validate) k_zero2<<<1, 1, 0, p->stream>>>(qsums);
    uint32_t *hist = (uint32_t *)p->hist.p;
    uint32_t *tot = hist + (size_t)256 * ntiles;
    K *kin = (K *)p->keys_a.p, *kout = (K *)p->keys_b.p;
    int32_t *vin = (int32_t *)p->vals_a.p, *vout = (int32_t *)p->vals_b.p;
    if (bucket)
        k_stage<T, K, true><<<ntiles, SORT_THREADS, 0, p->stream>>>(
            pos, q, N, kin, vin, (Rec<T> *)p->recs.p, hist, ntiles, (T)scale, p->Lz,
            p->opts.validate, status, qsums);
    else
        k_stage<T, K, false><<<ntiles, SORT_THREADS, 0, p->stream>>>(
            pos, q, N, kin, vin, (Rec<T> *)p->recs.p, hist, ntiles, (T)scale, p->Lz,
            p->opts.validate, status, qsums);
    if (p->opts.validate) k_neutral_check<<<1, 1, 0, p->stream>>>(qsums, status);
    if (bucket) {
        // one stable scatter by bucket, then every bucket sorted by (key, index)
        k_scan_digit<<<256, 256, 0, p->stream>>>(hist, ntiles, tot);
        k_scatter<K, true><<<ntiles, SORT_THREADS, 0, p->stream>>>(kin, vin, kout, vout, N, 0,
                                                                  hist, tot, ntiles, scale);
        k_bsort<T, K><<<BK_NB, BK_THREADS, 0, p->stream>>>(
            kout, vout, tot, (const Rec<T> *)p->recs.p, p->Lx, p->Ly, (U *)p->s_ux.p,
            (U *)p->s_uy.p, (T *)p->s_z.p, (T *)p->s_q.p);
        p->perm = vout;
        return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
    } else {
        const int passes = (int)sizeof(K);
        for (int pass = 0; pass < passes; ++pass) {
            const int shift = 8 * pass;
            // (k_stage wrote the first pass's tile histograms)
            if (pass > 0)
                k_hist<K><<<ntiles, SORT_THREADS, 0, p->stream>>>(kin, N, shift, hist, ntiles);
            k_scan_digit<<<256, 256, 0, p->stream>>>(hist, ntiles, tot);
            k_scatter<K><<<ntiles, SORT_THREADS, 0, p->stream>>>(kin, vin, kout, vout, N, shift,
                                                                hist, tot, ntiles);
            std::swap(kin, kout);
            std::swap(vin, vout);
        }
        p->perm = vin;
    }
    k_gather<T><<<nb, 256, 0, p->stream>>>((const Rec<T> *)p->recs.p, p->perm, N, p->Lx, p->Ly,
                                           (U *)p->s_ux.p, (U *)p->s_uy.p, (T *)p->s_z.p,
                                           (T *)p->s_q.p);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

// ---------------------------------------------------------------------------
// replica batches: sort by (replica, z), then lay each replica out in whole
// segments of S particles; the slots after its last particle are padding
// (zero charge at the replica's top height, input index -1)
// ---------------------------------------------------------------------------
template <typename T, typename K>
__global__ __launch_bounds__(256) void k_stage_batch(const T *__restrict__ pos,
                                                     const T *__restrict__ q, int64_t N,
                                                     const int32_t *__restrict__ rep_of,
                                                     const double *__restrict__ boxes,
                                                     K *__restrict__ keys, int32_t *__restrict__ vals,
                                                     int validate, int *status,
                                                     double *__restrict__ qsums) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T z = pos[3 * i + 2];
    keys[i] = zkey(z);
    vals[i] = (int32_t)i;
    if (validate) {
        const int r = rep_of[i];
        const T x = pos[3 * i], y = pos[3 * i + 1];
        const double qv = (double)q[i];
        const bool finite = isfinite((double)x) && isfinite((double)y) && isfinite((double)z) &&
                            isfinite(qv);
        if (!finite || !((double)z >= 0.0 && (double)z <= boxes[3 * r + 2]))
            set_status(status, Q2D_EOUTOFBOX);
        atomicAdd(&qsums[2 * r], qv);
        atomicAdd(&qsums[2 * r + 1], fabs(qv));
    }
}

__global__ void k_zero_sums(double *a, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

__global__ void k_neutral_batch(const double *qsums, int R, int *status) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R && fabs(qsums[2 * r]) > 1e-6 * qsums[2 * r + 1] + 1e-300)
        atomicOr(status, 1 << Q2D_ENONNEUTRAL);
}

// second key: replica of the element now at position i (bits `shift` and up)
__global__ __launch_bounds__(256) void k_repkey(const int32_t *__restrict__ vals, int64_t N,
                                                const int32_t *__restrict__ rep_of,
                                                uint32_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) keys[i] = (uint32_t)rep_of[vals[i]];
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_batch(
    const T *__restrict__ pos, const T *__restrict__ q, const int32_t *__restrict__ perm, int64_t N,
    const int32_t *__restrict__ rep_of, const int64_t *__restrict__ off,
    const int64_t *__restrict__ poff, const double *__restrict__ boxes,
    typename Fix<T>::U *__restrict__ ux, typename Fix<T>::U *__restrict__ uy, T *__restrict__ zs,
    T *__restrict__ qs, int32_t *__restrict__ pperm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t o = perm[i];
    const int r = rep_of[o];
    const int64_t pi = poff[r] + (i - off[r]);
    ux[pi] = Fix<T>::frac((double)pos[3 * (int64_t)o] / boxes[3 * r]);
    uy[pi] = Fix<T>::frac((double)pos[3 * (int64_t)o + 1] / boxes[3 * r + 1]);
    zs[pi] = pos[3 * (int64_t)o + 2] + (T)0;
    qs[pi] = q[o];
    pperm[pi] = o;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pad_batch(int64_t Npad, int S,
                                                   const int32_t *__restrict__ seg_rep,
                                                   const int64_t *__restrict__ off,
                                                   const int64_t *__restrict__ poff,
                                                   typename Fix<T>::U *__restrict__ ux,
                                                   typename Fix<T>::U *__restrict__ uy,
                                                   T *__restrict__ zs, T *__restrict__ qs,
                                                   int32_t *__restrict__ pperm) {
    const int64_t pi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pi >= Npad) return;
    const int r = seg_rep[pi / S];
    const int64_t n = off[r + 1] - off[r];
    if (pi - poff[r] < n) return;
    // a replica with padding has at least one particle: its top height
    ux[pi] = 0;
    uy[pi] = 0;
    zs[pi] = zs[poff[r] + n - 1];
    qs[pi] = (T)0;
    pperm[pi] = -1;
}

template <typename T, typename K>
q2d_status sort_batch_impl(Plan *p, const void *pos_v, const void *q_v) {
    const T *pos = (const T *)pos_v;
    const T *q = (const T *)q_v;
    using U = typename Fix<T>::U;
    const int64_t N = p->Ntot, Npad = p->Npad;
    q2d_status st;
    if ((st = ensure(p, p->keys_a, N * sizeof(K))) != Q2D_OK) return st;
    if ((st = ensure(p, p->keys_b, N * sizeof(K))) != Q2D_OK) return st;
    if ((st = ensure(p, p->vals_a, N * sizeof(int32_t))) != Q2D_OK) return st;
    if ((st = ensure(p, p->vals_b, N * sizeof(int32_t))) != Q2D_OK) return st;
    const int ntiles = (int)((N + SORT_TILE - 1) / SORT_TILE);
    if ((st = ensure(p, p->hist, ((size_t)256 * ntiles + 256) * sizeof(uint32_t))) != Q2D_OK)
        return st;
    if ((st = ensure(p, p->s_ux, Npad * sizeof(U))) != Q2D_OK) return st;
    if ((st = ensure(p, p->s_uy, Npad * sizeof(U))) != Q2D_OK) return st;
    if ((st = ensure(p, p->s_z, Npad * sizeof(T))) != Q2D_OK) return st;
    if ((st = ensure(p, p->s_q, Npad * sizeof(T))) != Q2D_OK) return st;
    if ((st = ensure(p, p->pperm, Npad * sizeof(int32_t))) != Q2D_OK) return st;
    int *status = (int *)p->status.p;
    // per-replica sums of q and |q| follow H in the same buffer ([R] + [R][2])
    double *qsums = (double *)p->rep_H.p + p->R;
    const int nb = (int)((N + 255) / 256);
    const int32_t *rep_of = (const int32_t *)p->rep_of.p;
    const double *boxes = (const double *)p->rep_box.p;
    if (p->opts.validate)
        k_zero_sums<<<(2 * p->R + 255) / 256, 256, 0, p->stream>>>(qsums, 2 * p->R);
    if (N > 0)
        k_stage_batch<T, K><<<nb, 256, 0, p->stream>>>(pos, q, N, rep_of, boxes, (K *)p->keys_a.p,
                                                       (int32_t *)p->vals_a.p, p->opts.validate,
                                                       status, qsums);
    if (p->opts.validate)
        k_neutral_batch<<<(p->R + 255) / 256, 256, 0, p->stream>>>(qsums, p->R, status);
    uint32_t *hist = (uint32_t *)p->hist.p;
    uint32_t *tot = hist + (size_t)256 * ntiles;
    K *kin = (K *)p->keys_a.p, *kout = (K *)p->keys_b.p;
    int32_t *vin = (int32_t *)p->vals_a.p, *vout = (int32_t *)p->vals_b.p;
    if (N > 0) {
        // least significant first: z (all its bytes), then the replica index
        for (int pass = 0; pass < (int)sizeof(K); ++pass) {
            k_hist<K><<<ntiles, SORT_THREADS, 0, p->stream>>>(kin, N, 8 * pass, hist, ntiles);
            k_scan_digit<<<256, 256, 0, p->stream>>>(hist, ntiles, tot);
            k_scatter<K><<<ntiles, SORT_THREADS, 0, p->stream>>>(kin, vin, kout, vout, N, 8 * pass,
                                                                hist, tot, ntiles);
            std::swap(kin, kout);
            std::swap(vin, vout);
        }
        uint32_t *rin = (uint32_t *)kin, *rout = (uint32_t *)kout;
        k_repkey<<<nb, 256, 0, p->stream>>>(vin, N, rep_of, rin);
        const int rpasses = p->R > 256 ? 2 : 1;
        for (int pass = 0; pass < rpasses; ++pass) {
            k_hist<uint32_t><<<ntiles, SORT_THREADS, 0, p->stream>>>(rin, N, 8 * pass, hist, ntiles);
            k_scan_digit<<<256, 256, 0, p->stream>>>(hist, ntiles, tot);
            k_scatter<uint32_t><<<ntiles, SORT_THREADS, 0, p->stream>>>(rin, vin, rout, vout, N,
                                                                       8 * pass, hist, tot, ntiles);
            std::swap(rin, rout);
            std::swap(vin, vout);
        }
        p->perm = vin;
        k_gather_batch<T><<<nb, 256, 0, p->stream>>>(
            pos, q, vin, N, rep_of, (const int64_t *)p->rep_off.p, (const int64_t *)p->rep_poff.p,
            boxes, (U *)p->s_ux.p, (U *)p->s_uy.p, (T *)p->s_z.p, (T *)p->s_q.p,
            (int32_t *)p->pperm.p);
    }
    if (Npad > N)
        k_pad_batch<T><<<(int)((Npad + 255) / 256), 256, 0, p->stream>>>(
            Npad, p->S_batch, (const int32_t *)p->seg_rep.p, (const int64_t *)p->rep_off.p,
            (const int64_t *)p->rep_poff.p, (U *)p->s_ux.p, (U *)p->s_uy.p, (T *)p->s_z.p,
            (T *)p->s_q.p, (int32_t *)p->pperm.p);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

}  // namespace

q2d_status sort_and_stage_batch(Plan *p, const void *pos, const void *q) {
    p->inv_ready = false;
    tstart(p, 2);
    q2d_status st = p->fp32 ? sort_batch_impl<float, uint32_t>(p, pos, q)
                            : sort_batch_impl<double, uint64_t>(p, pos, q);
    tstop(p, 2);
    return st;
}

q2d_status gather_sources(Plan *p, const void *g, int64_t N) {
    const size_t tsz = p->fp32 ? sizeof(float) : sizeof(double);
    q2d_status st = ensure(p, p->s_g, N * tsz);
    if (st != Q2D_OK) return st;
    const int nb = (int)((N + 255) / 256);
    if (p->fp32)
        k_gather1<float><<<nb, 256, 0, p->stream>>>((const float *)g, p->perm, N,
                                                    (float *)p->s_g.p);
    else
        k_gather1<double><<<nb, 256, 0, p->stream>>>((const double *)g, p->perm, N,
                                                     (double *)p->s_g.p);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

q2d_status radix_sort_u32(Plan *p, int64_t N, int passes, uint32_t **keys_out,
                          int32_t **vals_out) {
    const int ntiles = (int)((N + SORT_TILE - 1) / SORT_TILE);
    q2d_status st = ensure(p, p->hist, ((size_t)256 * ntiles + 256) * sizeof(uint32_t));
    if (st != Q2D_OK) return st;
    uint32_t *hist = (uint32_t *)p->hist.p;
    uint32_t *tot = hist + (size_t)256 * ntiles;
    uint32_t *kin = (uint32_t *)p->keys_a.p, *kout = (uint32_t *)p->keys_b.p;
    int32_t *vin = (int32_t *)p->vals_a.p, *vout = (int32_t *)p->vals_b.p;
    for (int pass = 0; pass < passes && N > 0; ++pass) {
        k_hist<uint32_t><<<ntiles, SORT_THREADS, 0, p->stream>>>(kin, N, 8 * pass, hist, ntiles);
        k_scan_digit<<<256, 256, 0, p->stream>>>(hist, ntiles, tot);
        k_scatter<uint32_t><<<ntiles, SORT_THREADS, 0, p->stream>>>(kin, vin, kout, vout, N,
                                                                   8 * pass, hist, tot, ntiles);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    *keys_out = kin;
    *vals_out = vin;
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

void sort_reqs(Plan *p, int64_t N, Reqs &q) {
    if (p->fp32)
        sort_reqs_t<float, uint32_t>(p, N, q);
    else
        sort_reqs_t<double, uint64_t>(p, N, q);
}

q2d_status sort_and_stage(Plan *p, const void *pos, const void *q, int64_t N) {
    p->inv_ready = false;  // a new order: any earlier inverse permutation is stale
    tstart(p, 2);
    q2d_status st = p->fp32 ? sort_impl<float, uint32_t>(p, pos, q, N)
                            : sort_impl<double, uint64_t>(p, pos, q, N);
    tstop(p, 2);
    return st;
}

}  // namespace q2d
