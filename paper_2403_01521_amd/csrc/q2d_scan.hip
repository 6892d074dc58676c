// Fourier modes k != 0: batched forward/backward z-ordered prefix scans.
//
// For one mode k and one exponent beta (beta = k or beta = alpha s_l) the
// recursion of Sec. 3.2 (eq. S, eq. 35) computes, over particles sorted by z,
//   T_i = sum_{j<i} b_j e^{-beta (z_i - z_j)},   B_i = sum_{j>i} b_j e^{-beta (z_j - z_i)}
// through the bounded ratios e^{-beta (z_i - z_{i-1})}.  With real sources
// x_j = q_j cos(k.rho_j) and y_j = q_j sin(k.rho_j) and the pair kernel
// K_k(z) = sum_beta a_beta e^{-beta z} (coefficients in q2d_modes.hip):
//   X_i = sum_{j != i} x_j K_k(|z_ij|) = sum_beta Re a_beta (T^x + B^x)
//   X'_i = sum_{j != i} x_j sgn(z_i - z_j) K'_k(|z_ij|) = sum_beta Re a'_beta (T^x - B^x)
// (Y, Y' likewise), and with c_i, s_i = cos, sin(k.rho_i):
//   phi_i  += omega (c_i X_i + s_i Y_i)                  (eq. SOEphi, real part)
//   F_rho  += omega q_i k_vec (s_i X_i - c_i Y_i)         (App. E, d/d rho)
//   F_z    -= omega q_i (c_i X'_i + s_i Y'_i)             (App. E, eq. z-der)
//
// GPU layout (one wave per work-group):
//  * lanes are modes: 64 modes of a batch share each particle, so the
//    particle data and the SOE decays e^{-beta_l dz} (mode independent) are
//    computed once per 64-particle block into LDS and read as broadcasts;
//  * the particle axis is cut into segments of S consecutive sorted
//    particles; a wave sweeps one segment sequentially (the recursion) for
//    its modes in one direction (the forward and backward sweeps start from
//    their own carries, so they run in separate work-groups), after (1) an
//    aggregate pass gives every segment's total
//    contribution referenced to its end (forward) and start (backward), and
//    (2) an FP64 scan over segments turns aggregates into carry-ins.  Every
//    cross-segment factor is one exponential of a z difference, never a long
//    product of rounded ratios;
//  * the per-particle results are reduced over the 64 mode lanes through a
//    padded LDS transpose in a fixed order (deterministic).
#include <algorithm>
#include <type_traits>

#include "q2d_internal.h"

namespace q2d {

namespace {

template <typename T>
struct Tr;
template <>
struct Tr<float> {
    using U = uint32_t;  // x/Lx as a 32-bit fixed-point fraction of a turn
};
template <>
struct Tr<double> {
    using U = double;    // x/Lx as a double in [0, 1)
};

// sin, cos of 2 pi (mx ux + my uy)
// FP32: the turn count mx ux + my uy is exact modulo 2^32 in fixed point; the
// hardware sine/cosine take their argument in turns (measured on gfx950:
// absolute error 1.2e-7 on [-1/2, 1/2)).
__device__ inline void phase_sc(int mx, int my, uint32_t ux, uint32_t uy, float &s, float &c) {
    const uint32_t ph = (uint32_t)mx * ux + (uint32_t)my * uy;
    const float r = (float)(int32_t)ph * 0x1p-32f;  // turns in [-1/2, 1/2)
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
}
__device__ inline void phase_sc(int mx, int my, double ux, double uy, double &s, double &c) {
    double r = fma((double)mx, ux, (double)my * uy);
    r -= rint(r);
    sincospi(2.0 * r, &s, &c);
}

// exp(-(br + i bi) t).  The angle is reduced in turns to [-1/2, 1/2] (exact
// for |turns| < 2^23) for the hardware sine and cosine; the reduced angle
// carries the rounding of bi t / (2 pi), about 2 ulp of the unreduced turn
// count, which matters only for large gaps, where |exp| = e^{-br t} is small.
// Branch-free: a full range-reduction path here held the sweep's register
// peak (167 VGPRs against 161).
__device__ inline cx<float> cexpm(float br, float bi, float t) {
    const float m = __expf(-br * t);
    float turns = bi * t * 0.15915494309189535f;  // 1/(2 pi)
    turns -= rintf(turns);
    const float s = __builtin_amdgcn_sinf(turns), c = __builtin_amdgcn_cosf(turns);
    return {m * c, -m * s};
}
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
// small arguments r = |ar| + |ai|: Taylor polynomials with remainder
// r^{n+1}/(n+1)! < 1e-17 (degree 4 below 2^-10, degree 7 below 2^-6)
__device__ inline cx<double> cexpm(double br, double bi, double t) {
    const double ar = br * t, ai = bi * t;
    const double r = fabs(ar) + fabs(ai);
    if (r < 0x1p-10) return expm_taylor<4>(ar, ai);
    if (r < 0x1p-6) return expm_taylor<7>(ar, ai);
    const double m = exp(-ar);
    double s, c;
    sincos(ai, &s, &c);
    return {m * c, -m * s};
}
__device__ inline float expm_real(float k, float t) { return __expf(-k * t); }
__device__ inline double expm_real(double k, double t) { return exp(-k * t); }
// e^{-k t} from a coefficient scaled once: FP32 keeps kl = -k log2(e) and
// takes one hardware exp2 per use (one multiply fewer than e^{-k t}); FP64
// keeps kl = -k
__device__ inline float kpre(float k) { return -k * 1.4426950408889634f; }
__device__ inline double kpre(double k) { return -k; }
__device__ inline float exp_pre(float kl, float t) { return __builtin_amdgcn_exp2f(kl * t); }
__device__ inline double exp_pre(double kl, double t) { return exp(kl * t); }

// lane exchange inside groups of four lanes (DPP quad permutations)
__device__ inline float quad_xor1(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ inline float quad_xor2(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
}
__device__ inline double quad_xor1(double v) { return __shfl_xor(v, 1); }
__device__ inline double quad_xor2(double v) { return __shfl_xor(v, 2); }

// A launch is a list of units along the (1-D) grid.  A unit is a set of
// modes that shares one lane layout: F consecutive segments per wave and
// wb = 64 / F modes per segment group.  F = 1: whole groups of 64 modes, a
// wave loops over the unit's groups; F > 1: one band of wb < 64 modes, so a
// wave still has every lane busy.  All units use the same segments (S
// particles), hence one carry scan serves them all.
constexpr int MAX_UNITS = 32;
constexpr int SMAX = 512;  // longest segment
constexpr int SUB = 4;     // steps per unrolled round; every unit has wb >= 4
struct Unit {
    int F;      // segments per wave
    int m0;     // first mode (within the launch's mode batch)
    int nm;     // modes in the unit
    int chunk;  // output chunk
    int b0;     // first work-group of the unit
    int acc;    // add to the chunk (an earlier mode batch wrote it)
};

template <typename T>
struct KArgs {
    int64_t N;
    int S, nseg;
    const typename Tr<T>::U *ux, *uy;
    const T *z, *q;
    const int32_t *modes;
    int64_t mstride;  // my of mode m at modes[mstride + m]
    const T *coef;
    int64_t cstride;  // field f of mode m at coef[f * cstride + m]
    int64_t moff;     // first mode of the batch in the tables
    int nmodes, gpad;
    int nunits;
    Unit units[MAX_UNITS];
    // sweep: 1 if each direction runs in its own work-group (block 2 b + d
    // sweeps unit block b in direction d); the backward outputs then go to
    // chunk + bchunk
    int split, bchunk;
    // replica batches: replica of each segment, and the distance between two
    // replicas' mode and coefficient tables (null / 0 for one system)
    const int32_t *seg_rep;
    int64_t rep_mstride, rep_cstride;
    T bre[MAX_PAIRS], bim[MAX_PAIRS];
    cx<T> *agg;  // [2 dirs][nseg][MH+1 slots][2 inputs][gpad]
    T *outk;     // [chunks][N][4]
};

template <int MH>
__device__ inline int64_t agg_idx(int nseg, int gpad, int dir, int seg, int slot, int inp, int m) {
    return ((((int64_t)dir * nseg + seg) * (MH + 1) + slot) * 2 + inp) * gpad + m;
}

// This work-group's unit and lane layout.  Lane L works on segment
// (wave * F + L / wb) for modes m0 + g * wb + L % wb.  The F segments
// advance in lock step; a block of wb steps covers 64 particles (wb from
// each segment), which the lanes load cooperatively, one each: lane L loads
// step L % wb of segment L / wb into LDS entry (L % wb) * F + L / wb.
struct LaneMap {
    Unit u;
    int wb, wave;
    int f, mi, seg;
    int64_t i0;  // first particle of this lane's segment
    int n;       // its length (0 if past the last segment)
    int64_t mb, cb;  // offsets of the segment's replica in the mode / coefficient tables
};

template <typename T>
__device__ inline LaneMap lane_map(const KArgs<T> &a, int bx) {
    LaneMap r;
    int k = 0;
    for (int t = 1; t < a.nunits; ++t)
        if (bx >= a.units[t].b0) k = t;
    r.u = a.units[k];
    r.wb = WAVE / r.u.F;
    r.wave = bx - r.u.b0;
    const int lane = threadIdx.x;
    r.f = lane / r.wb;
    r.mi = lane % r.wb;
    r.seg = r.wave * r.u.F + r.f;
    r.i0 = (int64_t)r.seg * a.S;
    r.n = r.seg < a.nseg ? (int)(min(r.i0 + (int64_t)a.S, a.N) - r.i0) : 0;
    const int rep = (a.seg_rep && r.seg < a.nseg) ? a.seg_rep[r.seg] : 0;
    r.mb = (int64_t)rep * a.rep_mstride;
    r.cb = (int64_t)rep * a.rep_cstride;
    return r;
}

// ---------------------------------------------------------------------------
// pass 1: per-segment aggregates (dot products with decays to the ends)
// ---------------------------------------------------------------------------
template <typename T, int MH>
__global__ __launch_bounds__(64) void k_agg(const KArgs<T> a) {
    using U = typename Tr<T>::U;
    const int lane = threadIdx.x;
    const LaneMap lm = lane_map(a, (int)blockIdx.x);
    const int BS = lm.wb;  // steps per block; lane loads segment f = lane / BS, step lane % BS
    __shared__ U c_ux[WAVE], c_uy[WAVE];
    __shared__ T c_q[WAVE], c_zf[WAVE], c_zb[WAVE];
    __shared__ cx<T> c_ef[MH][WAVE], c_eb[MH][WAVE];
    // LDS entries are step-major (entry j * F + f): the F segment groups
    // read F adjacent entries, conflict-free
    const int js = lane % BS, wi = js * lm.u.F + lm.f;
    const T s_zf = lm.n > 0 ? a.z[lm.i0] : (T)0, s_zl = lm.n > 0 ? a.z[lm.i0 + lm.n - 1] : (T)0;
    const int nblk = a.S / BS;  // S is a multiple of 64, BS a power of two >= 4
    const int ng = (lm.u.nm + lm.wb - 1) / lm.wb;
    for (int g = 0; g < ng; ++g) {
        const int ml = g * lm.wb + lm.mi;
        const bool mv = ml < lm.u.nm;
        const int m = lm.u.m0 + ml;
        const int mx = mv ? a.modes[lm.mb + a.moff + m] : 0;
        const int my = mv ? a.modes[lm.mb + a.mstride + a.moff + m] : 0;
        const T k = mv ? a.coef[lm.cb + 2 * a.cstride + a.moff + m] : (T)0;
        cx<T> fx[MH], fy[MH], bx[MH], by[MH];
#pragma unroll
        for (int l = 0; l < MH; ++l) fx[l] = fy[l] = bx[l] = by[l] = cx<T>{0, 0};
        T fkx = 0, fky = 0, bkx = 0, bky = 0;
        for (int blk = 0; blk < nblk; ++blk) {
            __syncthreads();
            {
                // positions past the segment's end hold a zero source
                const int pos = blk * BS + js;
                U ux = 0, uy = 0;
                T qv = 0, tf = 0, tb = 0;
                if (pos < lm.n) {
                    const int64_t p = lm.i0 + pos;
                    ux = a.ux[p];
                    uy = a.uy[p];
                    qv = a.q[p];
                    const T zp = a.z[p];
                    tf = s_zl - zp;
                    tb = zp - s_zf;
                }
                c_ux[wi] = ux;
                c_uy[wi] = uy;
                c_q[wi] = qv;
                c_zf[wi] = tf;
                c_zb[wi] = tb;
#pragma unroll
                for (int l = 0; l < MH; ++l) {
                    c_ef[l][wi] = cexpm(a.bre[l], a.bim[l], tf);
                    c_eb[l][wi] = cexpm(a.bre[l], a.bim[l], tb);
                }
            }
            __syncthreads();
            for (int j0 = 0; j0 < BS; j0 += SUB) {
#pragma unroll
                for (int jr = 0; jr < SUB; ++jr) {
                    const int ci = (j0 + jr) * lm.u.F + lm.f;
                    T s, c;
                    phase_sc(mx, my, c_ux[ci], c_uy[ci], s, c);
                    const T x = c_q[ci] * c, y = c_q[ci] * s;
                    const T ef = expm_real(k, c_zf[ci]), eb = expm_real(k, c_zb[ci]);
                    fkx += x * ef;
                    fky += y * ef;
                    bkx += x * eb;
                    bky += y * eb;
#pragma unroll
                    for (int l = 0; l < MH; ++l) {
                        const cx<T> e = c_ef[l][ci];
                        fx[l].re += x * e.re;
                        fx[l].im += x * e.im;
                        fy[l].re += y * e.re;
                        fy[l].im += y * e.im;
                        const cx<T> e2 = c_eb[l][ci];
                        bx[l].re += x * e2.re;
                        bx[l].im += x * e2.im;
                        by[l].re += y * e2.re;
                        by[l].im += y * e2.im;
                    }
                }
            }
        }
        // every column below gpad is written (a padded mode's aggregates are
        // finite and meet zero coefficients in the sweep)
        if (lm.seg < a.nseg && m < a.gpad) {
            const int seg = lm.seg;
#pragma unroll
            for (int l = 0; l < MH; ++l) {
                a.agg[agg_idx<MH>(a.nseg, a.gpad, 0, seg, l, 0, m)] = fx[l];
                a.agg[agg_idx<MH>(a.nseg, a.gpad, 0, seg, l, 1, m)] = fy[l];
                a.agg[agg_idx<MH>(a.nseg, a.gpad, 1, seg, l, 0, m)] = bx[l];
                a.agg[agg_idx<MH>(a.nseg, a.gpad, 1, seg, l, 1, m)] = by[l];
            }
            a.agg[agg_idx<MH>(a.nseg, a.gpad, 0, seg, MH, 0, m)] = cx<T>{fkx, 0};
            a.agg[agg_idx<MH>(a.nseg, a.gpad, 0, seg, MH, 1, m)] = cx<T>{fky, 0};
            a.agg[agg_idx<MH>(a.nseg, a.gpad, 1, seg, MH, 0, m)] = cx<T>{bkx, 0};
            a.agg[agg_idx<MH>(a.nseg, a.gpad, 1, seg, MH, 1, m)] = cx<T>{bky, 0};
        }
    }
}

// ---------------------------------------------------------------------------
// pass 1 on the fp16 matrix cores with split operands (FP32 plans, M <= 24).
// Every FP32 operand v is carried as v_hi + v_lo with v_hi = fp16(v) (rounded
// toward zero) and v_lo = fp16(v - v_hi); the products hi*hi + hi*lo + lo*hi,
// accumulated in FP32, leave an error of about 2^-20 |v| |w| per term (the
// lo*lo term and the roundings of the lo parts), FP32-sized over a segment.  The decays
// satisfy |E| <= 1; the sources are scaled by a power of two that brings the
// segment's largest |q| below 1 (undone exactly on the result), so no fp16
// overflow can occur.  v_mfma_f32_16x16x32_f16 takes 32 particles per
// instruction: lane l supplies A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16] (e < 8) and holds D[4 (l / 16) + v][l % 16].
// ---------------------------------------------------------------------------
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <int MH>
struct alignas(16) AggLdsH {
    static constexpr int NCP = (4 * MH + 15) / 16 * 16;  // columns padded to whole tiles
    static constexpr int RP = WAVE + 8;                   // row pitch in halves (16-byte rows)
    uint32_t ux[WAVE], uy[WAVE];
    float q[WAVE], zf[WAVE], zb[WAVE];
    // decays [column][entry], hi and lo; one more tile for the powers of the
    // beta = k Taylor columns
    _Float16 eh[NCP + 16][RP], el[NCP + 16][RP];
};

// hi of two values from one instruction (rounded toward zero: |v - hi| < 2^-10 |v|),
// lo = fp16(v - hi) from that same hi.  Computing hi once matters: the
// compiler otherwise forms hi both from the exact product that produced v (a
// fused multiply) and from v (a second rounding), and the two differ by an
// fp16 ulp now and then, so hi + lo != v (measured: FP32 forces 10x less
// accurate for charges that are not powers of two).  With hi fixed, any
// evaluation of lo leaves |v - hi - lo| <= 2^-21 |v|.
__device__ inline void split_pair(float a, float b, _Float16 &ha, _Float16 &hb, _Float16 &la,
                                  _Float16 &lb) {
    const auto h = __builtin_amdgcn_cvt_pkrtz(a, b);
    ha = (_Float16)h[0];
    hb = (_Float16)h[1];
    la = (_Float16)(a - (float)ha);
    lb = (_Float16)(b - (float)hb);
}

__device__ inline void split8(const float (&v)[8], h8v &hi, h8v &lo) {
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        _Float16 ha, hb, la, lb;
        split_pair(v[e], v[e + 1], ha, hb, la, lb);
        hi[e] = ha;
        hi[e + 1] = hb;
        lo[e] = la;
        lo[e + 1] = lb;
    }
}

// One work-group per segment computes the aggregates of every mode of the
// launch (independent of the sweep's mode units): the decays of a block of 64
// particles are staged in LDS once for all its waves, and each wave takes CPW
// chunks of 16 modes (rows: the x and y sources of each chunk).  The
// beta = k term (mode-dependent decay) stays on the VALU.
constexpr int AGW_MAX = 8;  // waves per work-group at most
constexpr int AGG_CPW = 2;  // default 16-mode chunks per wave (measured best of 1, 2, 4 at
                            // the single-system bench size; replica batches tune it)

// the FP64 betas and the spans table (W, G per (segment, pair)) that the
// aggregate kernel fills for the carry scan
struct SpanArgs {
    double br[MAX_PAIRS], bi[MAX_PAIRS];
    cx<double> *spans;
};

// The beta = k term (mode-dependent decay) on the matrix cores: with
// u = t / Delta in [0, 1] (t the distance to the segment end in the direction,
// Delta the segment's z span), e^{-k t} = sum_{n <= KT_DEG} (-k Delta)^n / n! u^n
// with remainder at most (k Delta)^8 / 8! < 2e-8 for k Delta <= KT_MAX.  The
// powers u^n are mode-independent columns of the contraction (8 per
// direction, in one extra column tile); each mode combines its 8 sums with
// its own coefficients afterwards.  Segments whose span is too wide for the
// largest |k| of the launch, and tables of more than 16 terms (whose pairs
// already take three tiles), keep the per-particle exponentials on the VALU.
constexpr int KT_DEG = 7;
constexpr float KT_MAX = 0.4f;

template <int MH, int CPW>
__global__ __launch_bounds__(AGW_MAX * WAVE) void k_agg_seg(const KArgs<float> a,
                                                           const SpanArgs sp) {
    constexpr int NC = 4 * MH, NCT = AggLdsH<MH>::NCP / 16, PC0 = AggLdsH<MH>::NCP;
    __shared__ AggLdsH<MH> L;
    __shared__ float red[AGW_MAX], redk[AGW_MAX];
    __shared__ double sb[2][MH];
    const int seg = blockIdx.x, tid = threadIdx.x;
    const int AGW = (int)blockDim.x / WAVE, NT = (int)blockDim.x;
    const int lane = tid % WAVE, wv = tid / WAVE;
    const int i = lane & 15, kq = lane >> 4;
    const int64_t i0 = (int64_t)seg * a.S;
    const int n = (int)(min(i0 + (int64_t)a.S, a.N) - i0);
    const int rep = a.seg_rep ? a.seg_rep[seg] : 0;
    const int64_t mb = (int64_t)rep * a.rep_mstride, cb = (int64_t)rep * a.rep_cstride;
    for (int e = tid; e < (AggLdsH<MH>::NCP - NC) * WAVE; e += NT) {
        L.eh[NC + e / WAVE][e % WAVE] = (_Float16)0.f;
        L.el[NC + e / WAVE][e % WAVE] = (_Float16)0.f;
    }
    const float s_zf = a.z[i0], s_zl = a.z[i0 + n - 1];
    // source scale 2^-e with max |q| of the segment < 2^e; the largest |k|
    float qm = 0.f, km = 0.f;
    for (int j = tid; j < n; j += NT) qm = fmaxf(qm, fabsf(a.q[i0 + j]));
    for (int m = tid; m < a.nmodes; m += NT) km = fmaxf(km, a.coef[cb + 2 * a.cstride + a.moff + m]);
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        qm = fmaxf(qm, __shfl_xor(qm, off));
        km = fmaxf(km, __shfl_xor(km, off));
    }
    if (lane == 0) {
        red[wv] = qm;
        redk[wv] = km;
    }
    if (tid == 0) {
        // uniform indices (a lane-dependent index into the arguments would
        // compile to select chains)
        for (int l = 0; l < MH; ++l) {
            sb[0][l] = sp.br[l];
            sb[1][l] = sp.bi[l];
        }
    }
    __syncthreads();
    if (tid < 2 * MH) {
        // this segment's spans: W = e^{-beta (z_last - z_first)}, G = e^{-beta
        // (z_first(next) - z_last)} (the same values as k_spans)
        const int l = tid >> 1, wg = tid & 1;
        const double zf = (double)s_zf, zl = (double)s_zl;
        const double zn = seg + 1 < a.nseg ? (double)a.z[i0 + a.S] : zl;
        sp.spans[((int64_t)seg * MH + l) * 2 + wg] =
            span_decay(sb[0][l], sb[1][l], wg ? zn - zl : zl - zf);
    }
    for (int w = 0; w < AGW; ++w) {
        qm = fmaxf(qm, red[w]);
        km = fmaxf(km, redk[w]);
    }
    int qe = 0;
    if (qm > 0.f) (void)frexpf(qm, &qe);
    qe = min(qe, 120);
    const float qscale = ldexpf(1.f, -qe), qunscale = ldexpf(1.f, qe);
    const float span = s_zl - s_zf;
    const float rspan = span > 0.f ? 1.f / span : 0.f;
    const int nblk = (n + WAVE - 1) / WAVE;
    const int nchunk = (a.nmodes + 15) / 16;  // every column a sweep lane reads
    const int npass = (nchunk + AGW * CPW - 1) / (AGW * CPW);

    auto passes = [&](auto taylor_tag) {
        constexpr bool TAY = decltype(taylor_tag)::value;
        constexpr int NCX = TAY ? NCT + 1 : NCT;  // column tiles in the contraction
        for (int ps = 0; ps < npass; ++ps) {
            const int c0 = (ps * AGW + wv) * CPW;  // this wave's first chunk (wave-uniform)
            const bool act = c0 < nchunk;
            int pmx[CPW], pmy[CPW];
            float pk[CPW];
#pragma unroll
            for (int cc = 0; cc < CPW; ++cc) {
                const int m = 16 * (c0 + cc) + i;
                const bool mv = m < a.nmodes;
                pmx[cc] = mv ? a.modes[mb + a.moff + m] : 0;
                pmy[cc] = mv ? a.modes[mb + a.mstride + a.moff + m] : 0;
                pk[cc] = (!TAY && mv) ? kpre(a.coef[cb + 2 * a.cstride + a.moff + m]) : 0.f;
            }
            f4v acc[2 * CPW][NCX];
#pragma unroll
            for (int t = 0; t < 2 * CPW; ++t)
#pragma unroll
                for (int c = 0; c < NCX; ++c) acc[t][c] = f4v{0.f, 0.f, 0.f, 0.f};
            float fk[CPW][4];
#pragma unroll
            for (int cc = 0; cc < CPW; ++cc) fk[cc][0] = fk[cc][1] = fk[cc][2] = fk[cc][3] = 0.f;
            // this lane's particle of the next block, loaded a block ahead so
            // that the loads complete during the contraction (tables of at
            // most 16 terms: with more, the registers held across the
            // contraction would lower the occupancy)
            constexpr bool PREF = NCT <= 2;
            float nz = 0.f, nq = 0.f;
            uint32_t nux = 0, nuy = 0;
            auto fetch = [&](int blk) {
                const int pos = blk * WAVE + lane;
                nz = 0.f;
                nq = 0.f;
                nux = nuy = 0;
                if (pos < n) {
                    nz = a.z[i0 + pos];
                    if (wv == 0) {
                        nux = a.ux[i0 + pos];
                        nuy = a.uy[i0 + pos];
                        nq = a.q[i0 + pos];
                    }
                }
            };
            if (PREF) fetch(0);
            // every load so far done here (vmcnt(0)): a mode's table entries
            // would otherwise be waited for inside the block loop, whose wait
            // then also takes in the loads of the next block
            if (PREF) __builtin_amdgcn_s_waitcnt(0x0F70);
            for (int blk = 0; blk < nblk; ++blk) {
                __syncthreads();
                if (!PREF) fetch(blk);
                {
                    // particle lane of the block; wave wv stages pairs wv, wv + AGW, ...
                    const int pos = blk * WAVE + lane;
                    float tf = 0.f, tb = 0.f;
                    if (pos < n) {
                        tf = s_zl - nz;
                        tb = nz - s_zf;
                    }
                    if (wv == 0) {
                        L.ux[lane] = nux;
                        L.uy[lane] = nuy;
                        L.q[lane] = nq * qscale;
                        if (!TAY) {
                            L.zf[lane] = tf;
                            L.zb[lane] = tb;
                        }
                    }
                    for (int l = wv; l < MH; l += AGW) {
                        const cx<float> ef = cexpm(a.bre[l], a.bim[l], tf);
                        const cx<float> eb = cexpm(a.bre[l], a.bim[l], tb);
                        _Float16 h[4], lo[4];
                        split_pair(ef.re, ef.im, h[0], h[1], lo[0], lo[1]);
                        split_pair(eb.re, eb.im, h[2], h[3], lo[2], lo[3]);
                        const int cols[4] = {2 * l, 2 * l + 1, 2 * MH + 2 * l, 2 * MH + 2 * l + 1};
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            L.eh[cols[u]][lane] = h[u];
                            L.el[cols[u]][lane] = lo[u];
                        }
                    }
                    if constexpr (TAY) {
                        // columns PC0 + p (forward) and PC0 + 8 + p (backward): u^p
                        const float uf = tf * rspan, ub = tb * rspan;
                        for (int pw = wv; pw <= KT_DEG; pw += AGW) {
                            float vf = 1.f, vb = 1.f;
                            for (int t = 0; t < pw; ++t) {
                                vf *= uf;
                                vb *= ub;
                            }
                            _Float16 hf, hb, lf, lb;
                            split_pair(vf, vb, hf, hb, lf, lb);
                            L.eh[PC0 + pw][lane] = hf;
                            L.el[PC0 + pw][lane] = lf;
                            L.eh[PC0 + 8 + pw][lane] = hb;
                            L.el[PC0 + 8 + pw][lane] = lb;
                        }
                    }
                    // after the staging: its own loads (the pair exponents)
                    // wait for every load in flight
                    if (PREF && blk + 1 < nblk) fetch(blk + 1);
                }
                __syncthreads();
                if (!act) continue;
#pragma unroll 1
                for (int ks = 0; ks < 2; ++ks) {
                    const int e0 = 32 * ks + 8 * kq;  // this lane's 8 particles
                    h8v bh[NCX], bl[NCX];
#pragma unroll
                    for (int c = 0; c < NCX; ++c) {
                        bh[c] = *(const h8v *)&L.eh[16 * c + i][e0];
                        bl[c] = *(const h8v *)&L.el[16 * c + i][e0];
                    }
#pragma unroll
                    for (int cc = 0; cc < CPW; ++cc) {
                        float xs[8], ys[8];
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            float sn, cs;
                            phase_sc(pmx[cc], pmy[cc], L.ux[e0 + e], L.uy[e0 + e], sn, cs);
                            const float qv = L.q[e0 + e];
                            xs[e] = qv * cs;
                            ys[e] = qv * sn;
                            if (!TAY) {
                                const float ef = exp_pre(pk[cc], L.zf[e0 + e]);
                                const float eb = exp_pre(pk[cc], L.zb[e0 + e]);
                                fk[cc][0] = fma(xs[e], ef, fk[cc][0]);
                                fk[cc][1] = fma(ys[e], ef, fk[cc][1]);
                                fk[cc][2] = fma(xs[e], eb, fk[cc][2]);
                                fk[cc][3] = fma(ys[e], eb, fk[cc][3]);
                            }
                        }
                        h8v xh, xl, yh, yl;
                        split8(xs, xh, xl);
                        split8(ys, yh, yl);
#pragma unroll
                        for (int c = 0; c < NCX; ++c) {
                            f4v &ax = acc[cc][c], &ay = acc[CPW + cc][c];
                            ax = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, bh[c], ax, 0, 0, 0);
                            ax = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, bl[c], ax, 0, 0, 0);
                            ax = __builtin_amdgcn_mfma_f32_16x16x32_f16(xl, bh[c], ax, 0, 0, 0);
                            ay = __builtin_amdgcn_mfma_f32_16x16x32_f16(yh, bh[c], ay, 0, 0, 0);
                            ay = __builtin_amdgcn_mfma_f32_16x16x32_f16(yh, bl[c], ay, 0, 0, 0);
                            ay = __builtin_amdgcn_mfma_f32_16x16x32_f16(yl, bh[c], ay, 0, 0, 0);
                        }
                        // one chunk's work at a time (interleaving the next
                        // chunk's VALU work with these matrix instructions
                        // needs 170+ VGPRs, 2 waves per SIMD); only LDS reads
                        // (mask 0x100) may move across, so the next chunk's
                        // particle data is read while these run
                        __builtin_amdgcn_sched_barrier(0x0100);
                    }
                }
            }
            if (!act) continue;
            // tile (source inp, chunk cc), column tile c, register v -> mode
            // 16 (c0 + cc) + 4 kq + v, column 16 c + i (sources scaled back)
            float *aggf = (float *)a.agg;
#pragma unroll
            for (int cc = 0; cc < CPW; ++cc)
#pragma unroll
                for (int inp = 0; inp < 2; ++inp)
#pragma unroll
                    for (int c = 0; c < NCT; ++c) {
                        const int col = 16 * c + i;
                        if (col >= NC) continue;
                        const int dir = col / (2 * MH), slot = (col % (2 * MH)) / 2, ri = col % 2;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int m = 16 * (c0 + cc) + 4 * kq + v;
                            if (m < a.gpad)
                                aggf[2 * agg_idx<MH>(a.nseg, a.gpad, dir, seg, slot, inp, m) + ri] =
                                    acc[inp * CPW + cc][c][v] * qunscale;
                        }
                    }
            if constexpr (TAY) {
                // beta = k term: lane i of the last tile holds sum_j src_j u_j^p
                // (p = i % 8, direction i / 8) for modes 16 (c0 + cc) + 4 kq + v;
                // scale by (-k Delta)^p / p! and add the 8 powers (fixed order)
                const int pw = i & 7, dir = i >> 3;
#pragma unroll
                for (int cc = 0; cc < CPW; ++cc)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int m = 16 * (c0 + cc) + 4 * kq + v;
                        const float x =
                            m < a.nmodes ? -a.coef[cb + 2 * a.cstride + a.moff + m] * span : 0.f;
                        float cf = 1.f;
#pragma unroll
                        for (int t = 1; t <= KT_DEG; ++t)
                            cf = t <= pw ? cf * (x * (1.f / (float)t)) : cf;
#pragma unroll
                        for (int inp = 0; inp < 2; ++inp) {
                            float r = acc[inp * CPW + cc][NCT][v] * cf;
                            r += __shfl_xor(r, 1);
                            r += __shfl_xor(r, 2);
                            r += __shfl_xor(r, 4);
                            if (pw == 0 && m < a.gpad)
                                a.agg[agg_idx<MH>(a.nseg, a.gpad, dir, seg, MH, inp, m)] =
                                    cx<float>{r * qunscale, 0.f};
                        }
                    }
            } else {
                // beta = k term: add the four particle quarters (lanes i, i+16, i+32, i+48)
#pragma unroll
                for (int cc = 0; cc < CPW; ++cc)
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        float v = fk[cc][w];
                        v += __shfl_xor(v, 16);
                        v += __shfl_xor(v, 32);
                        fk[cc][w] = v * qunscale;
                    }
                if (kq == 0) {
#pragma unroll
                    for (int cc = 0; cc < CPW; ++cc) {
                        const int m = 16 * (c0 + cc) + i;
                        if (m < a.gpad) {
                            a.agg[agg_idx<MH>(a.nseg, a.gpad, 0, seg, MH, 0, m)] =
                                cx<float>{fk[cc][0], 0.f};
                            a.agg[agg_idx<MH>(a.nseg, a.gpad, 0, seg, MH, 1, m)] =
                                cx<float>{fk[cc][1], 0.f};
                            a.agg[agg_idx<MH>(a.nseg, a.gpad, 1, seg, MH, 0, m)] =
                                cx<float>{fk[cc][2], 0.f};
                            a.agg[agg_idx<MH>(a.nseg, a.gpad, 1, seg, MH, 1, m)] =
                                cx<float>{fk[cc][3], 0.f};
                        }
                    }
                }
            }
        }
    };
    // the extra column tile only while the contraction has at most two (more
    // would lower the occupancy of the whole kernel)
    if constexpr (NCT <= 2) {
        if (km * span <= KT_MAX)
            passes(std::true_type{});
        else
            passes(std::false_type{});
    } else {
        passes(std::false_type{});
    }
}

// ---------------------------------------------------------------------------
// pass 3: the sweep (recursion) through each lane's segment for its mode
// ---------------------------------------------------------------------------

// Coefficients of one mode as the sweep uses them, with the mode weight omega
// and the output signs folded in: X = Re sum_beta al_beta T_beta gives omega X
// directly, Xd the z-derivative term -omega X' (forward sign; the backward
// sweep negates ad, since T - B enters the derivative).
template <typename T, int MH>
struct SweepCoef {
    T kx, ky, k, ak, akd;  // k: the mode's |k| as kpre() scales it
    T alr[MH], ali[MH], adr[MH], adi[MH];
};

template <typename T, int MH, int DIR>
__device__ inline void sweep_dir(const KArgs<T> &a, const LaneMap &lm, int m, int mx, int my,
                                 const SweepCoef<T, MH> &cf, typename Tr<T>::U *c_ux,
                                 typename Tr<T>::U *c_uy, T *c_q, T *c_dz, cx<T> (*c_d)[WAVE],
                                 T (*red)[4][WAVE + 1], T *outc, bool store) {
    using U = typename Tr<T>::U;
    const int lane = threadIdx.x;
    const int BS = lm.wb, F = lm.u.F;
    cx<T> px[MH], py[MH];
    T pkx = 0, pky = 0;
#pragma unroll
    for (int l = 0; l < MH; ++l) px[l] = py[l] = cx<T>{0, 0};
    if (lm.n > 0 && m < a.gpad) {
#pragma unroll
        for (int l = 0; l < MH; ++l) {
            px[l] = a.agg[agg_idx<MH>(a.nseg, a.gpad, DIR, lm.seg, l, 0, m)];
            py[l] = a.agg[agg_idx<MH>(a.nseg, a.gpad, DIR, lm.seg, l, 1, m)];
        }
        pkx = a.agg[agg_idx<MH>(a.nseg, a.gpad, DIR, lm.seg, MH, 0, m)].re;
        pky = a.agg[agg_idx<MH>(a.nseg, a.gpad, DIR, lm.seg, MH, 1, m)].re;
    }
    const int js = lane % BS, wi = js * F + lm.f;  // step-major LDS entries
    const int lbs = __builtin_ctz(BS);             // BS = 64 / F, a power of two
    const int nblk = a.S / BS;                     // S is a multiple of 64
    // reduction geometry: lane reads 16 entries of row (lane >> 2)
    const int rrow = lane >> 2, rchunk = lane & 3;
    const int rr = rrow >> 2, rv = rrow & 3;
    const int c0 = rchunk * 16;
    for (int bb = 0; bb < nblk; ++bb) {
        const int blk = DIR ? (nblk - 1 - bb) : bb;
        // after the first block, the barrier that ends the previous block's
        // last round already orders its reads before this staging (one
        // barrier per block fewer: narrow bands stage every 64 / F steps)
        if (bb == 0) __syncthreads();
        {
            // positions past the segment's end hold a zero source and a unit
            // decay: the recursion passes them through unchanged and their
            // outputs are never stored
            const int pos = blk * BS + js;
            U ux = 0, uy = 0;
            T qv = 0, dz = 0;
            if (pos < lm.n) {
                const int64_t p = lm.i0 + pos;
                ux = a.ux[p];
                uy = a.uy[p];
                qv = a.q[p];
                dz = pos > 0 ? a.z[p] - a.z[p - 1] : (T)0;  // gap to the particle below
            }
            c_ux[wi] = ux;
            c_uy[wi] = uy;
            c_q[wi] = qv;
            c_dz[wi] = dz;
#pragma unroll
            for (int l = 0; l < MH; ++l) c_d[l][wi] = cexpm(a.bre[l], a.bim[l], dz);
        }
        __syncthreads();
        for (int r0 = 0; r0 < BS; r0 += SUB) {
#pragma unroll
            for (int r = 0; r < SUB; ++r) {
                const int jj = r0 + r;
                const int j = DIR ? BS - 1 - jj : jj;
                const int ci = j * F + lm.f;
                T s, c;
                phase_sc(mx, my, c_ux[ci], c_uy[ci], s, c);
                const T qj = c_q[ci];
                const T x = qj * c, y = qj * s;
                const T dk = exp_pre(cf.k, c_dz[ci]);
                // explicit FMA chains: X += Re(a T) is two FMAs, not mul+fma+add
                T X, Y, Xd, Yd;
                if (DIR == 0) {
                    // T_j = (T_{j-1} + source_{j-1}) e^{-beta dz_j}
                    const T tkx = pkx * dk, tky = pky * dk;
                    X = cf.ak * tkx;
                    Xd = cf.akd * tkx;
                    Y = cf.ak * tky;
                    Yd = cf.akd * tky;
                    pkx = tkx + x;
                    pky = tky + y;
#pragma unroll
                    for (int l = 0; l < MH; ++l) {
                        const cx<T> d = c_d[l][ci];
                        const T txr = fma(px[l].re, d.re, -px[l].im * d.im);
                        const T txi = fma(px[l].re, d.im, px[l].im * d.re);
                        const T tyr = fma(py[l].re, d.re, -py[l].im * d.im);
                        const T tyi = fma(py[l].re, d.im, py[l].im * d.re);
                        X = fma(cf.alr[l], txr, X);
                        X = fma(-cf.ali[l], txi, X);
                        Xd = fma(cf.adr[l], txr, Xd);
                        Xd = fma(-cf.adi[l], txi, Xd);
                        Y = fma(cf.alr[l], tyr, Y);
                        Y = fma(-cf.ali[l], tyi, Y);
                        Yd = fma(cf.adr[l], tyr, Yd);
                        Yd = fma(-cf.adi[l], tyi, Yd);
                        px[l].re = txr + x;
                        px[l].im = txi;
                        py[l].re = tyr + y;
                        py[l].im = tyi;
                    }
                } else {
                    // B_j is the pending state; B_{j-1} = (B_j + source_j) e^{-beta dz_j}
                    X = cf.ak * pkx;
                    Xd = -cf.akd * pkx;
                    Y = cf.ak * pky;
                    Yd = -cf.akd * pky;
                    pkx = (pkx + x) * dk;
                    pky = (pky + y) * dk;
#pragma unroll
                    for (int l = 0; l < MH; ++l) {
                        const cx<T> d = c_d[l][ci];
                        const T bxr = px[l].re, bxi = px[l].im, byr = py[l].re, byi = py[l].im;
                        X = fma(cf.alr[l], bxr, X);
                        X = fma(-cf.ali[l], bxi, X);
                        Xd = fma(-cf.adr[l], bxr, Xd);
                        Xd = fma(cf.adi[l], bxi, Xd);
                        Y = fma(cf.alr[l], byr, Y);
                        Y = fma(-cf.ali[l], byi, Y);
                        Yd = fma(-cf.adr[l], byr, Yd);
                        Yd = fma(cf.adi[l], byi, Yd);
                        const T sxr = bxr + x, syr = byr + y;
                        px[l].re = fma(sxr, d.re, -bxi * d.im);
                        px[l].im = fma(sxr, d.im, bxi * d.re);
                        py[l].re = fma(syr, d.re, -byi * d.im);
                        py[l].im = fma(syr, d.im, byi * d.re);
                    }
                }
                const T oq = s * X - c * Y;
                red[r][0][lane] = c * X + s * Y;
                red[r][1][lane] = cf.kx * oq;
                red[r][2][lane] = cf.ky * oq;
                red[r][3][lane] = c * Xd + s * Yd;
            }
            // per step and segment group: the sum of 4 outputs over its wb
            // lanes (rows padded to 65 entries: conflict-free); a lane sums
            // 16 consecutive entries of one row, then partial sums of a group
            // wider than 16 lanes are combined by quad exchanges.  The output
            // chunk of the unit (and direction) receives it: stored by the
            // first pass that writes the chunk (store), added by later ones;
            // every element has one writer per pass and passes are separated
            // by barriers.
            __syncthreads();
            {
                const int pj = r0 + rr;
                const int jp = DIR ? BS - 1 - pj : pj;
                const int loc = blk * BS + jp;
                // add a segment group's sum to its output element (BS is a
                // power of two: shifts, not divisions, pick the group)
                auto put = [&](int g, T sum) {
                    const int sf = lm.wave * F + g;
                    if (sf < a.nseg) {
                        const int64_t base = (int64_t)sf * a.S;
                        const int nf = (int)min((int64_t)a.S, a.N - base);
                        if (loc < nf) {
                            T *o = outc + (base + loc) * 4 + rv;
                            *o = store ? sum : *o + sum;
                        }
                    }
                };
                if (BS >= 16) {
                    T sum = 0;
#pragma unroll
                    for (int L = 0; L < 16; ++L) sum += red[rr][rv][c0 + L];
                    if (BS >= 32) sum += quad_xor1(sum);
                    if (BS >= 64) sum += quad_xor2(sum);
                    if ((c0 & (BS - 1)) == 0) put(c0 >> lbs, sum);
                } else {
                    // BS = 8 or 4: the 16 entries hold 2 or 4 segment groups
                    for (int t = 0; t < (16 >> lbs); ++t) {
                        T sum = 0;
                        for (int L = 0; L < BS; ++L) sum += red[rr][rv][c0 + (t << lbs) + L];
                        put((c0 >> lbs) + t, sum);
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <typename T, int MH>
__global__ __launch_bounds__(64) void k_sweep(const KArgs<T> a) {
    using U = typename Tr<T>::U;
    // dir: 0 or 1 for a one-direction work-group, -1 for both
    const int dir = a.split ? (int)(blockIdx.x & 1) : -1;
    const LaneMap lm = lane_map(a, a.split ? (int)(blockIdx.x >> 1) : (int)blockIdx.x);
    __shared__ U c_ux[WAVE], c_uy[WAVE];
    __shared__ T c_q[WAVE], c_dz[WAVE];
    __shared__ cx<T> c_d[MH][WAVE];
    __shared__ T red[SUB][4][WAVE + 1];
    // output chunk of this work-group (a backward-only one writes chunk + bchunk)
    T *outc = a.outk + (int64_t)(lm.u.chunk + (dir == 1 ? a.bchunk : 0)) * a.N * 4;
    const int ng = (lm.u.nm + lm.wb - 1) / lm.wb;
    for (int g = 0; g < ng; ++g) {
        const int ml = g * lm.wb + lm.mi;
        const bool mv = ml < lm.u.nm;
        const int m = lm.u.m0 + ml;
        auto ld = [&](int f) -> T {
            return mv ? a.coef[lm.cb + (int64_t)f * a.cstride + a.moff + m] : (T)0;
        };
        const int mx = mv ? a.modes[lm.mb + a.moff + m] : 0;
        const int my = mv ? a.modes[lm.mb + a.mstride + a.moff + m] : 0;
        const T om = ld(3);
        SweepCoef<T, MH> cf;
        cf.kx = ld(0);
        cf.ky = ld(1);
        cf.k = kpre(ld(2));
        cf.ak = om * ld(4);
        cf.akd = -om * ld(5);
#pragma unroll
        for (int l = 0; l < MH; ++l) {
            cf.alr[l] = om * ld(6 + 4 * l);
            cf.ali[l] = om * ld(7 + 4 * l);
            cf.adr[l] = -om * ld(8 + 4 * l);
            cf.adi[l] = -om * ld(9 + 4 * l);
        }
        // lanes of a padded mode read column m of the aggregates if m < gpad
        // (finite) and carry zero coefficients: their outputs vanish
        // the first group of a unit stores its chunk (unless an earlier mode
        // batch wrote it), later groups add; with both directions in one
        // work-group the backward pass adds to what the forward pass stored
        const bool first = g == 0 && !lm.u.acc;
        if (dir != 1)
            sweep_dir<T, MH, 0>(a, lm, m, mx, my, cf, c_ux, c_uy, c_q, c_dz, c_d, red, outc, first);
        if (dir != 0)
            sweep_dir<T, MH, 1>(a, lm, m, mx, my, cf, c_ux, c_uy, c_q, c_dz, c_d, red, outc,
                                dir == 1 && first);
    }
}

// ---------------------------------------------------------------------------
// pass 2: FP64 scan of the aggregates over segments -> carries (in place)
// ---------------------------------------------------------------------------
template <typename T>
struct CArgs {
    int nseg, ncols, S, mh, gpad, nmodes;
    int64_t N;
    const T *z;
    const cx<double> *spans;  // [nseg][mh][2]: W (inside), G (gap above)
    cx<T> *agg;               // [2][nseg][ncols]
    const T *coef;
    int64_t cstride, moff;
    // replica batches: replica of carry segment s is seg_rep[s / seg_div]; no
    // carry crosses from one replica to the next (null for one system)
    const int32_t *seg_rep;
    int seg_div;
    int64_t rep_cstride;
};

constexpr int CAR_L = 8;       // segments per range
constexpr int CAR_BATCH = 2;   // loads issued ahead of the dependent chain (2: 103-110
                               // VGPRs, 4 waves per SIMD; 4 and 8 took 3 and 2 and were slower)

// Compose two range transfers x -> c + D x: first (c1, D1), then (c2, D2).
__device__ inline void compose(cx<double> &c2, cx<double> &D2, cx<double> c1, cx<double> D1) {
    const cx<double> t = cmul(D2, c1);
    c2 = cx<double>{c2.re + t.re, c2.im + t.im};
    D2 = cmul(D2, D1);
}

template <typename T>
__device__ inline int carry_rep(const CArgs<T> &a, int s) {
    return a.seg_rep ? a.seg_rep[s / a.seg_div] : 0;
}

// true if segment s is the last one of its system (no gap to a next segment)
template <typename T>
__device__ inline bool carry_last(const CArgs<T> &a, int s) {
    return s + 1 >= a.nseg || (a.seg_rep && carry_rep(a, s + 1) != carry_rep(a, s));
}

// Decay factors of segment s for a column: W_s = e^{-beta (z_last - z_first)}
// inside the segment and G_s = e^{-beta (z_first(s+1) - z_last(s))} across the
// gap (0 after the last segment of a replica: its carries stop there).
template <typename T, bool KMODE>
struct Decay {
    const CArgs<T> &a;
    int slot, mode;
    bool pair;
    double kk;
    __device__ Decay(const CArgs<T> &a_, int col) : a(a_) {
        slot = col / (2 * a.gpad);
        mode = col % a.gpad;
        pair = slot < a.mh;
        kk = 0.0;
        if (KMODE && !pair && mode < a.nmodes && !a.seg_rep)
            kk = (double)a.coef[2 * a.cstride + a.moff + mode];
    }
    __device__ void get(int s, cx<double> &W, cx<double> &G) const {
        if (pair) {
            W = a.spans[((int64_t)s * a.mh + slot) * 2];
            G = a.spans[((int64_t)s * a.mh + slot) * 2 + 1];
        } else if (KMODE) {
            double k = kk;
            if (a.seg_rep && mode < a.nmodes)
                k = (double)a.coef[(int64_t)carry_rep(a, s) * a.rep_cstride + 2 * a.cstride +
                                   a.moff + mode];
            const int64_t b = (int64_t)s * a.S, e = min(b + (int64_t)a.S, a.N) - 1;
            const double zf = (double)a.z[b], zl = (double)a.z[e];
            const double zn = (s + 1 < a.nseg) ? (double)a.z[(int64_t)(s + 1) * a.S] : zl;
            W = cx<double>{exp(-k * (zl - zf)), 0.0};
            G = cx<double>{exp(-k * (zn - zl)), 0.0};
        } else {
            W = cx<double>{1.0, 0.0};
            G = cx<double>{1.0, 0.0};
        }
        if (a.seg_rep && carry_last(a, s)) G = cx<double>{0.0, 0.0};
    }
    // factors of one step in direction dir: forward (W_s, G_s); backward
    // (W_s, G_{s-1}), the gap below s (none below segment 0)
    __device__ void step(int dir, int s, cx<double> &W, cx<double> &G) const {
        get(s, W, G);
        if (dir) {
            cx<double> Wm;
            G = cx<double>{0.0, 0.0};
            if (s > 0) get(s - 1, Wm, G);
        }
    }
};

// Walk the segments of one range in the direction of propagation starting from
// carry c: forward CF_{s+1} = G_s (AF_s + W_s CF_s), backward
// CB_{s-1} = G_{s-1} (AB_s + W_s CB_s).  WRITE: store each segment's carry-in
// in place of its aggregate; otherwise also accumulate the range's total
// decay D, so that the range maps x -> c + D x.
// Both directions are walked in one loop (the forward chain upwards, the
// backward chain downwards): their loads are issued together, which doubles
// the memory-level parallelism of these latency-bound walks.  c[d], D[d]:
// carry and decay of direction d.
template <typename T, bool KMODE, bool WRITE>
__device__ inline void walk2(const CArgs<T> &a, const Decay<T, KMODE> &dc, int col, int s0,
                             int s1, cx<double> (&c)[2], cx<double> (&D)[2]) {
    cx<T> *AG[2] = {a.agg, a.agg + (int64_t)a.nseg * a.ncols};
    const int n = s1 - s0;
    for (int k0 = 0; k0 < n; k0 += CAR_BATCH) {
        cx<T> av[2][CAR_BATCH];
        cx<double> W[2][CAR_BATCH], G[2][CAR_BATCH];
#pragma unroll
        for (int u = 0; u < CAR_BATCH; ++u) {
            const int k = k0 + u;
            if (k < n) {
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    const int s = d ? s1 - 1 - k : s0 + k;
                    dc.step(d, s, W[d][u], G[d][u]);
                    av[d][u] = AG[d][(int64_t)s * a.ncols + col];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < CAR_BATCH; ++u) {
            const int k = k0 + u;
            if (k < n) {
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    if (WRITE) {
                        const int s = d ? s1 - 1 - k : s0 + k;
                        AG[d][(int64_t)s * a.ncols + col] = cx<T>{(T)c[d].re, (T)c[d].im};
                    }
                    cx<double> t = cmul(W[d][u], c[d]);
                    t.re += (double)av[d][u].re;
                    t.im += (double)av[d][u].im;
                    c[d] = cmul(G[d][u], t);
                    if (!WRITE) D[d] = cmul(G[d][u], cmul(W[d][u], D[d]));
                }
            }
        }
    }
}

// The range transfers live in two planes of [2 directions][nr ranges][ncols]
// complex values, c first, then D: the lanes of a wave (consecutive columns)
// touch consecutive addresses in all three passes.
__device__ inline int64_t rc_at(int ncols, int nr, int dir, int r, int col) {
    return ((int64_t)dir * nr + r) * ncols + col;
}

// (1) one thread per (column, range): fold the range into x -> c + D x
template <typename T, bool KMODE>
__global__ __launch_bounds__(256) void k_cfold(const CArgs<T> a, int nr, cx<double> *rc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.ncols * nr) return;
    const int col = (int)(t % a.ncols), r = (int)(t / a.ncols);
    const int s0 = r * CAR_L, s1 = min(s0 + CAR_L, a.nseg);
    const Decay<T, KMODE> dc(a, col);
    cx<double> c[2] = {{0.0, 0.0}, {0.0, 0.0}}, D[2] = {{1.0, 0.0}, {1.0, 0.0}};
    walk2<T, KMODE, false>(a, dc, col, s0, s1, c, D);
    const int64_t plane = (int64_t)2 * nr * a.ncols;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const int64_t o = rc_at(a.ncols, nr, dir, r, col);
        rc[o] = c[dir];
        rc[plane + o] = D[dir];
    }
}

// (2) one work-group per CPG adjacent columns, TPC threads per column
// (thread = position * CPG + column, so a wave reads CPG consecutive columns
// of several ranges at once): exclusive scan of the range transfers in the
// direction of propagation; leaves the carry into each range in the c plane.
// Each thread composes a run of ceil(nr / TPC) ranges serially, then the runs
// are combined by a Hillis-Steele scan in LDS and re-walked.  A run's
// transfers are loaded CSCAN_PRE at a time, every load in bounds (position
// and column clamped) and none behind a branch, so that they are in flight
// together; a run of at most CSCAN_PRE stays in registers for the re-walk.
constexpr int CSCAN_PRE = 8;

template <int CPG, int TPC>
__global__ __launch_bounds__(CPG *TPC) void k_cscan(int ncols, int nr, cx<double> *rc) {
    __shared__ cx<double> sc[TPC][CPG], sd[TPC][CPG];
    const int cl = threadIdx.x % CPG, t = threadIdx.x / CPG;
    const int col = blockIdx.x * CPG + cl;
    const bool live = col < ncols;
    const int per = (nr + TPC - 1) / TPC;
    const int64_t plane = (int64_t)2 * nr * ncols;
    for (int dir = 0; dir < 2; ++dir) {
        // thread t owns propagation positions [t*per, (t+1)*per)
        auto at = [&](int pos) { return rc_at(ncols, nr, dir, dir ? nr - 1 - pos : pos, col); };
        auto ok = [&](int k) { return live && k < per && t * per + k < nr; };
        cx<double> cr[CSCAN_PRE], Dr[CSCAN_PRE];
        auto load = [&](int k0) {
#pragma unroll
            for (int u = 0; u < CSCAN_PRE; ++u) {
                const int pos = min(t * per + k0 + u, nr - 1);
                const int64_t o =
                    rc_at(ncols, nr, dir, dir ? nr - 1 - pos : pos, live ? col : ncols - 1);
                cr[u] = rc[o];
                Dr[u] = rc[plane + o];
            }
        };
        cx<double> c{0.0, 0.0}, D{1.0, 0.0};
        for (int k0 = 0; k0 < per; k0 += CSCAN_PRE) {
            load(k0);
#pragma unroll
            for (int u = 0; u < CSCAN_PRE; ++u)
                if (ok(k0 + u)) {
                    cx<double> nc = cr[u], nD = Dr[u];
                    compose(nc, nD, c, D);
                    c = nc;
                    D = nD;
                }
        }
        sc[t][cl] = c;
        sd[t][cl] = D;
        __syncthreads();
        for (int off = 1; off < TPC; off <<= 1) {
            cx<double> pc{0.0, 0.0}, pd{1.0, 0.0};
            const bool has = t >= off;
            if (has) {
                pc = sc[t - off][cl];
                pd = sd[t - off][cl];
            }
            __syncthreads();
            if (has) compose(c, D, pc, pd);
            sc[t][cl] = c;
            sd[t][cl] = D;
            __syncthreads();
        }
        cx<double> cin = t > 0 ? sc[t - 1][cl] : cx<double>{0.0, 0.0};
        __syncthreads();
        for (int k0 = 0; k0 < per; k0 += CSCAN_PRE) {
            if (per > CSCAN_PRE) load(k0);
#pragma unroll
            for (int u = 0; u < CSCAN_PRE; ++u)
                if (ok(k0 + u)) {
                    rc[at(t * per + k0 + u)] = cin;
                    cx<double> nc = cr[u], nD = Dr[u];
                    compose(nc, nD, cin, cx<double>{0.0, 0.0});
                    cin = nc;
                }
        }
        __syncthreads();
    }
}

// (3) one thread per (column, range): re-walk the range from its carry-in,
// replacing every aggregate by the segment's carry-in
template <typename T, bool KMODE>
__global__ __launch_bounds__(256) void k_capply(const CArgs<T> a, int nr, const cx<double> *rc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.ncols * nr) return;
    const int col = (int)(t % a.ncols), r = (int)(t / a.ncols);
    const int s0 = r * CAR_L, s1 = min(s0 + CAR_L, a.nseg);
    const Decay<T, KMODE> dc(a, col);
    cx<double> c[2], D[2] = {{1.0, 0.0}, {1.0, 0.0}};
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) c[dir] = rc[rc_at(a.ncols, nr, dir, r, col)];
    walk2<T, KMODE, true>(a, dc, col, s0, s1, c, D);
}

}  // namespace

size_t carry_tmp_bytes(int64_t ncols, int nseg) {
    const int64_t nr = (nseg + CAR_L - 1) / CAR_L;
    return (size_t)2 * ncols * nr * 2 * sizeof(cx<double>);
}

namespace {

template <typename T, bool KMODE>
q2d_status carry_run(Plan *p, const CArgs<T> &ca, Buf &tmp) {
    const int nr = (ca.nseg + CAR_L - 1) / CAR_L;
    q2d_status st = ensure(p, tmp, carry_tmp_bytes(ca.ncols, ca.nseg));
    if (st != Q2D_OK) return st;
    cx<double> *rc = (cx<double> *)tmp.p;
    const int64_t nt = (int64_t)ca.ncols * nr;
    const int nb = (int)((nt + 255) / 256);
    k_cfold<T, KMODE><<<nb, 256, 0, p->stream>>>(ca, nr, rc);
    // many columns of up to 2048 ranges: 8 columns of 32 threads per
    // work-group; few columns (the k = 0 carries): one column per work-group
    // (1024-thread work-groups wait for a nearly idle CU while other passes
    // run concurrently: only for very long columns)
    if (ca.ncols >= 256 ? nr <= 2048 : nr <= 256)
        k_cscan<8, 32><<<(ca.ncols + 7) / 8, 256, 0, p->stream>>>(ca.ncols, nr, rc);
    else if (nr <= 4096)
        k_cscan<1, 256><<<ca.ncols, 256, 0, p->stream>>>(ca.ncols, nr, rc);
    else
        k_cscan<1, 1024><<<ca.ncols, 1024, 0, p->stream>>>(ca.ncols, nr, rc);
    k_capply<T, KMODE><<<nb, 256, 0, p->stream>>>(ca, nr, rc);
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

// per (segment, pair): W = e^{-beta (z_last - z_first)}, G = e^{-beta (z_next_first - z_last)}
// (the spans tables of pair slots; G of a replica's last segment is replaced
// by 0 where the carry walk reads it)
template <typename T>
__global__ __launch_bounds__(256) void k_spans(const T *__restrict__ z, int64_t N, int S, int nseg,
                                               PairParams pp, cx<double> *__restrict__ spans) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nseg * pp.mh) return;
    const int s = (int)(idx / pp.mh), l = (int)(idx % pp.mh);
    const int64_t b = (int64_t)s * S, e = min(b + (int64_t)S, N) - 1;
    const double zf = (double)z[b], zl = (double)z[e];
    const double zn = (s + 1 < nseg) ? (double)z[(int64_t)(s + 1) * S] : zl;
    const double br = pp.beta_re[l], bi = pp.beta_im[l];
    spans[idx * 2] = span_decay(br, bi, zl - zf);
    spans[idx * 2 + 1] = span_decay(br, bi, zn - zl);
}

template <typename T>
void dispatch_agg(Plan *p, const KArgs<T> &ka, dim3 grid) {
    switch (p->mh) {
#define Q2D_CASE(n)                                              \
    case n:                                                      \
        k_agg<T, n><<<grid, WAVE, 0, p->stream>>>(ka);           \
        break;
        Q2D_CASE(1) Q2D_CASE(2) Q2D_CASE(3) Q2D_CASE(4) Q2D_CASE(5) Q2D_CASE(6) Q2D_CASE(7)
        Q2D_CASE(8) Q2D_CASE(9) Q2D_CASE(10) Q2D_CASE(11) Q2D_CASE(12) Q2D_CASE(13)
        Q2D_CASE(14) Q2D_CASE(15) Q2D_CASE(16)
#undef Q2D_CASE
        default:
            break;
    }
}

template <typename T>
void dispatch_sweep(Plan *p, const KArgs<T> &ka, dim3 grid) {
    switch (p->mh) {
#define Q2D_CASE(n)                                              \
    case n:                                                      \
        k_sweep<T, n><<<grid, WAVE, 0, p->stream>>>(ka);         \
        break;
        Q2D_CASE(1) Q2D_CASE(2) Q2D_CASE(3) Q2D_CASE(4) Q2D_CASE(5) Q2D_CASE(6) Q2D_CASE(7)
        Q2D_CASE(8) Q2D_CASE(9) Q2D_CASE(10) Q2D_CASE(11) Q2D_CASE(12) Q2D_CASE(13)
        Q2D_CASE(14) Q2D_CASE(15) Q2D_CASE(16)
#undef Q2D_CASE
        default:
            break;
    }
}

void dispatch_agg_seg(Plan *p, const KArgs<float> &ka, const SpanArgs &sp) {
    // AGG_CPW chunks of 16 modes per wave, as many waves as that takes (at
    // most AGW_MAX; more chunks take several passes over the segment)
    const int cpw = p->cfg_cpw ? p->cfg_cpw : AGG_CPW;
    const int nchunk = (ka.nmodes + 15) / 16;
    const int nw = std::max(1, std::min(AGW_MAX, (nchunk + cpw - 1) / cpw));
    switch (p->mh) {
#define Q2D_CASE(n)                                                                      \
    case n:                                                                              \
        if (cpw == 1)                                                                    \
            k_agg_seg<n, 1><<<ka.nseg, nw * WAVE, 0, p->stream>>>(ka, sp);               \
        else if (cpw == 4)                                                               \
            k_agg_seg<n, 4><<<ka.nseg, nw * WAVE, 0, p->stream>>>(ka, sp);               \
        else                                                                             \
            k_agg_seg<n, 2><<<ka.nseg, nw * WAVE, 0, p->stream>>>(ka, sp);               \
        break;
        Q2D_CASE(1) Q2D_CASE(2) Q2D_CASE(3) Q2D_CASE(4) Q2D_CASE(5) Q2D_CASE(6) Q2D_CASE(7)
        Q2D_CASE(8) Q2D_CASE(9) Q2D_CASE(10) Q2D_CASE(11) Q2D_CASE(12)
#undef Q2D_CASE
        default:
            break;
    }
}

// Pass 1 for a launch.  FP32 with M <= 24: the per-segment split-fp16 matrix
// kernel over all the launch's modes; otherwise the VALU kernel over the
// launch's units.
// true if launch_agg fills the spans table itself
template <typename T>
bool agg_fills_spans(const Plan *p) {
    return std::is_same<T, float>::value && p->mh <= 12;
}

template <typename T>
void launch_agg(Plan *p, const KArgs<T> &ka, int blocks) {
    if constexpr (std::is_same<T, float>::value) {
        if (agg_fills_spans<T>(p)) {
            SpanArgs sp{};
            for (int l = 0; l < p->mh; ++l) {
                sp.br[l] = p->pp.beta_re[l];
                sp.bi[l] = p->pp.beta_im[l];
            }
            sp.spans = (cx<double> *)p->spans.p;
            dispatch_agg_seg(p, ka, sp);
            return;
        }
    }
    dispatch_agg<T>(p, ka, dim3(blocks));
}

// segment length: multiple of 64, at most SMAX, aiming at ~2048 segments
int choose_S(int64_t N) {
    int s = env_int("Q2D_SEG", 0);
    if (s <= 0) {
        const int64_t want = (N + 2047) / 2048;
        s = (int)(((want + WAVE - 1) / WAVE) * WAVE);
    }
    s = ((s + WAVE - 1) / WAVE) * WAVE;
    if (s < WAVE) s = WAVE;
    if (s > SMAX) s = SMAX;
    return s;
}

// Mode decomposition.  All units share segments of S particles (one spans
// table, one carry scan).  Whole groups of 64 modes run one mode per lane
// (F = 1), gpc groups per unit; the remaining r < 64 modes, rounded up to a
// multiple of 4, split into powers of two w >= 4 (r = 32 + 4 for P = 100),
// each a band unit with F = 64 / w segments per wave, so every lane holds a
// mode (up to 3 padded lanes in the last band) and every wave sweeps S
// particles.  Mode tables longer than MB run in batches; bands join the last.
// Output chunks: one per unit and direction when each direction has its own
// work-groups (the default), else one per unit; later mode batches add into
// the F = 1 units' chunks.
struct KLayout {
    int S, nseg;
    int64_t MB, nfull, gpad_max;
    int rem, rem4, nbatch, ngroups0, gpc, nbands, nch_full, nchunks, nout;
    bool split;
};

KLayout kmodes_layout(const Plan *p, int64_t N, int64_t nmodes) {
    KLayout L{};
    // a replica batch fixes S: its particles are laid out in whole segments
    L.S = p->R ? p->S_batch : choose_S(N);
    L.nseg = (int)((N + L.S - 1) / L.S);
    L.MB = ((int64_t)std::max(env_int("Q2D_MODE_BATCH", 1024), 1) + WAVE - 1) / WAVE * WAVE;
    L.nfull = (nmodes / WAVE) * WAVE;
    L.rem = (int)(nmodes - L.nfull);
    // a remainder of 61..63 modes rounds up to a whole group: it runs as one
    // more F = 1 group whose last lanes read the tables' zero-weight padding
    // (every table is padded to a multiple of 64 columns)
    if (L.rem > WAVE - SUB) {
        L.nfull += WAVE;
        L.rem = 0;
    }
    L.rem4 = (L.rem + 3) & ~3;  // band lanes, padded to a multiple of 4
    L.nbatch = L.nfull > 0 ? (int)((L.nfull + L.MB - 1) / L.MB) : 1;
    L.ngroups0 = (int)(std::min(L.nfull, L.MB) / WAVE);
    // groups per unit: enough waves to fill the chip, few output chunks
    L.gpc = env_int("Q2D_GPC", 0);
    if (L.gpc <= 0) {
        const int target = 2048;
        int nch = (target + L.nseg - 1) / L.nseg;
        if (nch > L.ngroups0) nch = L.ngroups0;
        if (nch < 1) nch = 1;
        L.gpc = L.ngroups0 > 0 ? (L.ngroups0 + nch - 1) / nch : 1;
    }
    L.nbands = 0;
    for (int w = WAVE / 2; w >= SUB; w >>= 1) L.nbands += (L.rem4 & w) ? 1 : 0;
    if (L.ngroups0 > 0 && (L.ngroups0 + L.gpc - 1) / L.gpc > MAX_UNITS - L.nbands)
        L.gpc = (L.ngroups0 + MAX_UNITS - L.nbands - 1) / (MAX_UNITS - L.nbands);
    L.nch_full = L.ngroups0 > 0 ? (L.ngroups0 + L.gpc - 1) / L.gpc : 0;
    L.nchunks = L.nch_full + L.nbands;
    // one work-group per direction: twice the waves at half the length, so
    // the last round of the grid and the slow narrow bands leave a shorter
    // tail (Q2D_SPLIT=0: both directions in one work-group)
    L.split = p->cfg_split ? p->cfg_split == 1 : env_int("Q2D_SPLIT", 1) != 0;
    L.nout = L.split ? 2 * L.nchunks : L.nchunks;
    L.gpad_max = std::min(L.nfull, L.MB) + L.rem;
    return L;
}

template <typename T>
void kmodes_reqs_t(Plan *p, const KLayout &L, int64_t N, Reqs &q) {
    const int mh = p->mh;
    q.add(p->spans, (size_t)L.nseg * mh * 2 * sizeof(cx<double>));
    q.add(p->agg, (size_t)2 * L.nseg * (mh + 1) * 2 * L.gpad_max * sizeof(cx<T>));
    q.add(p->outk, (size_t)L.nout * N * 4 * sizeof(T));
    // the widest mode batch's carry columns
    q.add(p->carry_tmp, carry_tmp_bytes((int64_t)(mh + 1) * 2 * L.gpad_max, L.nseg));
}

template <typename T>
q2d_status kmodes_impl(Plan *p, int64_t N, const int32_t *modes, const void *coef,
                       int64_t cstride, int64_t moff0, int64_t nmodes, int *nchunks_out) {
    using U = typename Tr<T>::U;
    *nchunks_out = 0;
    if (nmodes <= 0 || N <= 0) return Q2D_OK;
    const KLayout L = kmodes_layout(p, N, nmodes);
    const int S = L.S, nseg = L.nseg, mh = p->mh;
    const int64_t MB = L.MB, nfull = L.nfull;
    const int rem = L.rem, rem4 = L.rem4, nbatch = L.nbatch, gpc = L.gpc;
    const int nch_full = L.nch_full, nchunks = L.nchunks, nout = L.nout;
    const bool split = L.split;
    const int32_t *seg_rep = p->R ? (const int32_t *)p->seg_rep.p : nullptr;
    q2d_status st;
    Reqs req;
    kmodes_reqs_t<T>(p, L, N, req);
    if ((st = ensure_all(p, req)) != Q2D_OK) return st;
    if (!agg_fills_spans<T>(p)) {
        const int64_t n = (int64_t)nseg * mh;
        k_spans<T><<<(int)((n + 255) / 256), 256, 0, p->stream>>>((const T *)p->s_z.p, N, S, nseg,
                                                                   p->pp, (cx<double> *)p->spans.p);
    }
    KArgs<T> ka{};
    ka.N = N;
    ka.S = S;
    ka.nseg = nseg;
    ka.ux = (const U *)p->s_ux.p;
    ka.uy = (const U *)p->s_uy.p;
    ka.z = (const T *)p->s_z.p;
    ka.q = (const T *)(p->src ? p->src : p->s_q.p);
    ka.modes = modes;
    ka.mstride = cstride;
    ka.coef = (const T *)coef;
    ka.cstride = cstride;
    for (int l = 0; l < mh; ++l) {
        ka.bre[l] = (T)p->pp.beta_re[l];
        ka.bim[l] = (T)p->pp.beta_im[l];
    }
    ka.agg = (cx<T> *)p->agg.p;
    ka.outk = (T *)p->outk.p;
    ka.seg_rep = seg_rep;
    ka.rep_mstride = p->R ? p->rep_mstride : 0;
    ka.rep_cstride = p->R ? p->rep_cstride : 0;
    ka.split = split ? 1 : 0;
    ka.bchunk = split ? nchunks : 0;
    for (int bi = 0; bi < nbatch; ++bi) {
        const int64_t b0 = (int64_t)bi * MB;
        const int nbf = (int)std::max<int64_t>(0, std::min(MB, nfull - b0));
        const bool last = bi == nbatch - 1;
        const int ngroups = nbf / WAVE;
        // bands first, the narrowest first: their waves are the slowest per
        // step (a staging round every 64 / F steps), dispatched early they do
        // not form the tail
        int nu = 0, blocks = 0, nbm = nbf;
        if (last) {
            int band = 0, left = rem;
            for (int w = SUB; w <= WAVE / 2; w <<= 1)
                if (rem4 & w) {
                    const int F = WAVE / w, nm = std::min(w, left);
                    ka.units[nu++] = Unit{F, nbm, nm, nch_full + band, blocks, 0};
                    blocks += (nseg + F - 1) / F;
                    nbm += nm;
                    left -= nm;
                    ++band;
                }
        }
        for (int g = 0; g < ngroups; g += gpc) {
            const int ng = std::min(gpc, ngroups - g);
            ka.units[nu++] = Unit{1, g * WAVE, ng * WAVE, g / gpc, blocks, bi > 0 ? 1 : 0};
            blocks += nseg;
        }
        ka.nunits = nu;
        ka.moff = moff0 + b0;
        ka.nmodes = nbm;
        ka.gpad = nbm;
        tstart(p, 1);
        launch_agg<T>(p, ka, blocks);
        tstop(p, 1);
        CArgs<T> ca{};
        ca.nseg = nseg;
        ca.ncols = (mh + 1) * 2 * ka.gpad;
        ca.S = S;
        ca.mh = mh;
        ca.gpad = ka.gpad;
        ca.nmodes = nbm;
        ca.N = N;
        ca.z = ka.z;
        ca.spans = (const cx<double> *)p->spans.p;
        ca.agg = ka.agg;
        ca.coef = ka.coef;
        ca.cstride = cstride;
        ca.moff = ka.moff;
        ca.seg_rep = seg_rep;
        ca.seg_div = 1;
        ca.rep_cstride = ka.rep_cstride;
        if ((st = carry_run<T, true>(p, ca, p->carry_tmp)) != Q2D_OK) return st;
        tstart(p, 0);
        dispatch_sweep<T>(p, ka, dim3(split ? 2 * blocks : blocks));
        tstop(p, 0);
    }
    *nchunks_out = nout;
    return hipGetLastError() == hipSuccess ? Q2D_OK : Q2D_EDEVICE;
}

}  // namespace

void kmodes_reqs(Plan *p, int64_t N, int64_t n_modes, Reqs &q) {
    if (n_modes <= 0 || N <= 0) return;
    const KLayout L = kmodes_layout(p, N, n_modes);
    if (p->fp32)
        kmodes_reqs_t<float>(p, L, N, q);
    else
        kmodes_reqs_t<double>(p, L, N, q);
}

q2d_status kmodes_run(Plan *p, int64_t N, const int32_t *modes, const void *coef,
                      int64_t coef_stride, int64_t mode_off, int64_t n_modes, int *n_chunks_out) {
    return p->fp32 ? kmodes_impl<float>(p, N, modes, coef, coef_stride, mode_off, n_modes,
                                        n_chunks_out)
                   : kmodes_impl<double>(p, N, modes, coef, coef_stride, mode_off, n_modes,
                                         n_chunks_out);
}

// exported for the k = 0 pass (same carry algebra, beta = 0 last slot)
q2d_status carry_k0(Plan *p, int nseg, int S, int64_t N) {
    CArgs<double> ca{};
    ca.nseg = nseg;
    ca.ncols = (p->mh + 1) * 2;
    ca.S = S;
    ca.mh = p->mh;
    ca.gpad = 1;
    ca.nmodes = 0;
    ca.N = N;
    ca.z = nullptr;
    ca.spans = (const cx<double> *)p->spans0.p;
    ca.agg = (cx<double> *)p->agg0.p;
    ca.coef = nullptr;
    if (p->R) {
        // k = 0 segments of S particles lie inside the batch's segments
        ca.seg_rep = (const int32_t *)p->seg_rep.p;
        ca.seg_div = p->S_batch / S;
    }
    return carry_run<double, false>(p, ca, p->carry_tmp0);
}

}  // namespace q2d
