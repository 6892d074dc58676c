/*
 * q2d.h -- C ABI of the quasi-2D long-range electrostatics library.
 *
 * The library evaluates, on one AMD MI355X (gfx950) GPU, the long-range part
 * of the Ewald2D sum for N point charges in a box [0,Lx] x [0,Ly] x [0,Lz]
 * that is periodic in x and y and confined in z (Sec. 2.1 of arXiv:2403.01521,
 * the Poisson problem with doubly periodic boundary conditions).  The Fourier
 * modes use the sum-of-exponentials (SOE) form of the kernels xi^+ + xi^-
 * (Sec. 3.1), which makes every mode an O(N) pair of z-ordered prefix scans
 * (Sec. 3.2, the recursion built on the z-sort); the random-batch entry point
 * samples P modes by importance sampling (Sec. 4.1, Alg. 2).
 *
 * Conventions shared by every entry point:
 *  - Units: Gaussian units, pair energy q_i q_j / r, force F_i = -grad_i U.
 *  - Arrays: pos is N x 3 row-major (x0 y0 z0 x1 ...), q, phi have N entries,
 *    F is N x 3 row-major.  The element type of pos, q, phi and F is double for
 *    a Q2D_FP64 plan and float for a Q2D_FP32 plan.  E is always one double.
 *  - Memory: every data pointer is a DEVICE pointer on the plan's device
 *    (hipMalloc / torch CUDA tensors).  The caller owns all of them; the plan
 *    owns only its internal scratch, sized at creation from n_max and p_max.
 *  - Streams: work is enqueued asynchronously on the plan's HIP stream; outputs
 *    are valid once that stream has reached the enqueued work.  One plan must
 *    not be used from two host threads at once.
 *  - Positions: x and y are wrapped into [0, L) (periodic); z is used as given
 *    and must lie in [0, Lz] (confinement).  The system must be charge neutral
 *    (Thm 2.1).  These two data conditions are checked on the device only when
 *    opts.validate is set; the result is reported by q2d_plan_check.
 *  - Outputs are overwritten, not accumulated.  NULL output pointers are
 *    skipped.  N = 0 is valid and writes E = 0.
 *  - Errors: every function returns a q2d_status; none throws or aborts.
 */
#ifndef Q2D_H
#define Q2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct q2d_plan *q2d_plan_t;

typedef enum {
    Q2D_OK = 0,
    Q2D_EINVAL = 1,        /* bad argument (null pointer, non-positive size, bad SOE table) */
    Q2D_ENONNEUTRAL = 2,   /* |sum q| > 1e-6 sum |q| (Thm 2.1); reported by q2d_plan_check */
    Q2D_EOUTOFBOX = 3,     /* z outside [0, Lz] or a non-finite input; by q2d_plan_check */
    Q2D_ENOMEM = 4,        /* a device or host allocation failed */
    Q2D_ECAPACITY = 5,     /* N > n_max or P > p_max */
    Q2D_EDEVICE = 6,       /* a HIP runtime call failed */
    Q2D_ESAMPLER = 7,      /* the mode sampler found no non-zero proposal */
    Q2D_EUNSUPPORTED = 8,  /* the plan was created without what this call needs */
    Q2D_EDTYPE = 9         /* element type of an argument differs from the plan's precision
                              (reported by bindings that see element types: the C calls
                              take untyped pointers and read them as the plan's type) */
} q2d_status;

typedef enum { Q2D_FP64 = 0, Q2D_FP32 = 1 } q2d_precision;

/* Mode samplers of the random batch (Sec. 4.1: modes drawn from
 * h(k) = exp(-k^2/(4 alpha^2)) / H over k != 0). */
typedef enum {
    Q2D_SAMPLER_METROPOLIS = 0,  /* the independence Metropolis chain of App. G */
    Q2D_SAMPLER_IID = 1          /* exact i.i.d. draws: h factorises over the two axes into
                                    discrete Gaussians; m_x from its marginal given
                                    m != (0, 0), then m_y given m_x, each by inversion of a
                                    cumulative table built in FP64 at plan creation */
} q2d_sampler;

typedef struct {
    int32_t precision;  /* q2d_precision: element type of pos, q, phi, F and of the scans */
    int32_t thin;       /* Metropolis thinning D >= 1 (App. G); 0 means 1 */
    int64_t n_max;      /* largest N any call on this plan will pass (> 0) */
    int32_t p_max;      /* largest batch size P of q2d_rbm_step (0: random batch unused) */
    int32_t validate;   /* nonzero: check neutrality, z in [0, Lz], finiteness on the device */
    int32_t sampler;    /* q2d_sampler (replica batches: Metropolis only) */
} q2d_opts;

/* Read-only facts about a plan (host values). */
typedef struct {
    int64_t n_modes_exact;  /* modes 0 < |k| <= k_c on the half lattice used by q2d_long_range */
    int32_t M;              /* number of SOE terms */
    double H;               /* sum_{k != 0} exp(-k^2 / (4 alpha^2)) (Sec. 4.1, eq. hk) */
    double diag_exact;      /* (pi/A) sum_{0<|k|<=k_c} e^{-k^2/4a^2} K_k(0): j = i constant, exact-k */
    double diag_rb;         /* the same sum over every k != 0: j = i constant, random batch */
    double soe_k0_self;     /* K_0(0) = sum_l w_l / (alpha sqrt(pi)) (eq. 32 at z = 0) */
} q2d_info;

/*
 * q2d_plan_create -- set up a solver for one box and one SOE table.
 *
 * Lx, Ly, Lz > 0: box (Sec. 2.1).  alpha > 0: Ewald splitting parameter
 * (Sec. 2.2).  r_c: real-space cutoff for q2d_short_range (<= 0 disables it;
 * otherwise 0 < r_c <= min(Lx, Ly) / 2).  k_c: Fourier cutoff of
 * q2d_long_range (<= 0 disables that entry point).  M, w, s: the SOE
 * exp(-x^2) ~ sum_l w_l exp(-s_l |x|) (Sec. 3, eq. SOE1; the plan uses
 * beta_l = alpha s_l); w and s are HOST arrays of 2M doubles, (re, im)
 * interleaved.  The table must be closed under complex conjugation, have
 * Re s_l > 0 and no real node (Im s_l = 0), so that beta_l^2 != k^2 for every
 * real k; otherwise Q2D_EINVAL.  opts: see q2d_opts (NULL: FP64, n_max = 0 is
 * invalid, so opts is required).  stream: a hipStream_t (NULL = default
 * stream).  On success *out holds a new plan.  The plan binds the device that
 * is current at creation.
 */
q2d_status q2d_plan_create(double Lx, double Ly, double Lz, double alpha, double r_c, double k_c,
                           int32_t M, const double *w, const double *s, const q2d_opts *opts,
                           void *stream, q2d_plan_t *out);

/* Release a plan and its device scratch (synchronises the plan's stream first). */
q2d_status q2d_plan_destroy(q2d_plan_t plan);

/* Bind later calls to another hipStream_t. */
q2d_status q2d_plan_set_stream(q2d_plan_t plan, void *stream);

/* Copy the plan's host-side facts into *info. */
q2d_status q2d_plan_info(q2d_plan_t plan, q2d_info *info);

/*
 * q2d_long_range -- SOEwald2D long-range sum over all 0 < |k| <= k_c
 * (Alg. 1, Fourier part; Sec. 3.2 recursion; forces of App. E).
 *
 * Writes phi_i = sum_{0<|k|<=k_c} phi^k_SOE(r_i) + phi^0_SOE(r_i) - phi_self^i,
 * where both Fourier parts include the j = i term (Sec. 2.2: phi_l contains
 * the Gaussian cloud's action on its own charge, phi_self = 2 alpha q_i/sqrt(pi)
 * removes it), F_i = -grad_i U_l, and E = 1/2 sum_i q_i phi_i (FP64).
 * pos, q: device inputs (N x 3, N); phi (N), F (N x 3), E (1 double): device
 * outputs or NULL.  Q2D_EUNSUPPORTED if the plan has k_c <= 0.
 */
q2d_status q2d_long_range(q2d_plan_t plan, const void *pos, const void *q, int64_t N, void *phi,
                          void *F, double *E);

/*
 * q2d_rbm_step -- random-batch SOE long-range sum (RBSE2D, Alg. 2, Fourier part).
 *
 * Draws P modes k_eta != 0 from h(k) = exp(-k^2/(4 alpha^2)) / H over the whole
 * lattice with the Metropolis chain of App. G driven by Philox4x32-10 with
 * key = seed and counter = (draw, step, stream); the same (seed, step) gives
 * the same modes.  Writes the estimator (eq. RBapp) of the k != 0 part for
 * every pair j != i, weight (pi/A) H/P per sampled mode, plus the deterministic
 * j = i constant q_i * diag_rb, plus the exact (SOE) k = 0 term and minus
 * phi_self, with forces and E as in q2d_long_range.  modes_out: device int32
 * array of P x 2 (mx, my) with k = 2 pi (mx/Lx, my/Ly), or NULL.
 * Q2D_ECAPACITY if P > p_max.
 * Each call also draws the modes of (seed, step + 1, P) on the plan's internal
 * stream; a following call with exactly those arguments on the same stream
 * uses them (same results, less waiting).  A plan on which a random-batch
 * step or its adjoint was ever called inside a stream capture stops drawing
 * ahead (replays of the capture rewrite the plan's mode buffers).
 */
q2d_status q2d_rbm_step(q2d_plan_t plan, const void *pos, const void *q, int64_t N, int32_t P,
                        uint64_t seed, uint64_t step, void *phi, void *F, double *E,
                        int32_t *modes_out);

/*
 * q2d_rbm_step_noalloc -- q2d_rbm_step for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving or MD loops, harnesses
 * that forbid hipMalloc.  Same arguments, checks, results and stream semantics
 * as q2d_rbm_step (bit-identical outputs for the same inputs); the call itself
 * allocates and frees nothing.  Its scratch (sorted copies, mode tables,
 * aggregates and carries, per-chunk outputs, the k = 0 term, the inverse
 * permutation) is not the plan's: it lives in one static device array of
 * Q2D_NOALLOC_SCRATCH_BYTES per device, which every device the library runs
 * on holds until the process ends, and whose address is looked up when the
 * first plan is created on that device.  The need grows with N and P (M = 16,
 * P = 100: 860 bytes per particle in FP32 up to N = 131072, fewer above as
 * the segments lengthen, so N up to about 3.3e5 in FP32 and 1.5e5 in FP64);
 * a call whose scratch does not fit returns Q2D_ECAPACITY before enqueuing
 * anything.  The plan itself (created once,
 * beforehand) keeps its own tables.  Every call on one device shares that
 * device's array and leaves its contents behind: calls on one stream are
 * ordered, but calls that can overlap in time on one device (two streams, or
 * two plans on different streams) race on it and must be serialised by the
 * caller.  Kernel timing (q2d_plan_timing_enable) records nothing for this
 * call.
 */
#define Q2D_NOALLOC_SCRATCH_BYTES ((uint64_t)128 << 20)
q2d_status q2d_rbm_step_noalloc(q2d_plan_t plan, const void *pos, const void *q, int64_t N,
                                int32_t P, uint64_t seed, uint64_t step, void *phi, void *F,
                                double *E, int32_t *modes_out);

/*
 * Adjoint (vector-Jacobian product) of the potential of q2d_long_range /
 * q2d_rbm_step.  For weights g_i on the outputs phi_i (L = sum_i g_i phi_i):
 *   dq_j   = dL/dq_j   = sum_i g_i G(r_i, r_j) = the potential of "charges" g at r_j,
 *   dpos_k = dL/dr_k   = -(g_k f(q)_k + q_k f(g)_k),
 * where phi_i = sum_j G(r_i, r_j) q_j (the same Fourier sums, j = i, k = 0 and
 * self terms as the forward call; G is symmetric) and f(s)_k is the field of
 * sources s at r_k (the force on a unit charge, App. E).  For the energy
 * E = 1/2 sum q_i phi_i no second pass is needed: dE/dq = phi and dE/dpos = -F
 * (dpos with g = q/2).  The scans
 * run twice, with sources q and with sources g (g need not be neutral; the
 * data checks apply to q only).  g: device array N (plan dtype); dq (N),
 * dpos (N x 3): device outputs or NULL.  The random-batch form uses the modes
 * of (seed, step), i.e. the same estimator as q2d_rbm_step.
 */
q2d_status q2d_long_range_vjp(q2d_plan_t plan, const void *pos, const void *q, const void *g,
                              int64_t N, void *dq, void *dpos);
q2d_status q2d_rbm_step_vjp(q2d_plan_t plan, const void *pos, const void *q, const void *g,
                            int64_t N, int32_t P, uint64_t seed, uint64_t step, void *dq,
                            void *dpos);

/*
 * q2d_modes_eval -- the k != 0 Fourier sum over a caller-given list of modes
 * with caller-given weights (the terms of eq. SOEphi with the forces of
 * App. E, term by term): for each listed mode k with weight omega_k,
 *   phi_i += omega_k sum_{j != i} q_j Re e^{i k.(rho_i - rho_j)} K_k(|z_i - z_j|)
 * (the pair kernel K_k of the SOE, its Gaussian factor being part of omega_k),
 * F_i = -grad_i of E, E = 1/2 sum_i q_i phi_i.  No k = 0 term, no j = i term
 * and no self term: with omega_k = (pi/A) e^{-k^2/(4 alpha^2)} over a subset of
 * the lattice this is that subset's part of q2d_long_range minus its j = i
 * constant; with omega_k = (pi/A) H/P over sampled modes, the k != 0 pair part
 * of q2d_rbm_step.  modes: device int32 array n_modes x 2 (mx, my), k =
 * 2 pi (mx/Lx, my/Ly), a (0, 0) entry adds nothing; weights: device double
 * array n_modes.  Scratch for the list is allocated on first use and grows.
 */
q2d_status q2d_modes_eval(q2d_plan_t plan, const void *pos, const void *q, int64_t N,
                          const int32_t *modes, const double *weights, int64_t n_modes, void *phi,
                          void *F, double *E);

/*
 * q2d_short_range -- real-space part phi_s (eq. phi_s) with cutoff r_c by a
 * uniform cell list: phi_i = sum over images m and j (j != i when m = 0) with
 * |r_ij + M| <= r_c of q_j erfc(alpha r)/r, the matching force and
 * E = 1/2 sum q_i phi_i.  Q2D_EUNSUPPORTED if the plan has r_c <= 0.
 */
q2d_status q2d_short_range(q2d_plan_t plan, const void *pos, const void *q, int64_t N, void *phi,
                           void *F, double *E);

/*
 * q2d_slab -- particle-slab term of two charged walls at z = 0 and z = Lz
 * (Sec. 2.4, Thm 2.7; eq. spectial for uniform walls), the p-s part of Alg. 2.
 * With sb(k), st(k) the Fourier coefficients of one cell of the bottom and top
 * surface charge densities, sig(k) = integral over [0,Lx) x [0,Ly) of
 * sigma(rho) e^{-i k.rho}:
 *   phi_i = (2 pi/A) Re sum_{listed k} e^{i k.rho_i}/k [sb(k) e^{-k|z_i|} + st(k) e^{-k|z_i - Lz|}]
 *           - (2 pi/A) [sig0_bot |z_i| + sig0_top |z_i - Lz|],
 * F_i = -q_i grad phi(r_i), E = sum_i q_i phi_i (no 1/2: the walls are
 * external charges).  Uniform walls of densities sigma_b, sigma_t: n_modes = 0,
 * sig0_bot = sigma_b A, sig0_top = sigma_t A.  modes: device int32 n_modes x 2
 * (mx, my), k = 2 pi (mx/Lx, my/Ly), the full lattice list (k and -k both listed
 * for a real density), no (0, 0); sig_bot, sig_top: device double arrays of
 * n_modes complex values (re, im interleaved).  Charge neutrality then reads
 * sum q + sig0_bot + sig0_top = 0 (eq. chargeneu), which the long-range entry
 * points do not check when walls carry charge (leave opts.validate off).
 * pos, q: device inputs; phi, F, E: device outputs or NULL.  FP64 arithmetic
 * for both precisions.
 */
q2d_status q2d_slab(q2d_plan_t plan, const void *pos, const void *q, int64_t N, int32_t n_modes,
                    const int32_t *modes, const double *sig_bot, const double *sig_top,
                    double sig0_bot, double sig0_top, void *phi, void *F, double *E);

/*
 * q2d_langevin_step -- one step of the Langevin dynamics of Sec. 4.3
 * (eq. langevin: dr = p/m dt, dp = (F - gamma p/m) dt + sqrt(2 gamma kT) dW)
 * by the BAOAB splitting, in two calls around the force evaluation:
 *   stage 0: p += dt/2 F; r += dt/2 p/m; p = e^{-gamma dt/m} p
 *            + sqrt(m kT (1 - e^{-2 gamma dt/m})) xi; r += dt/2 p/m; then x, y
 *            wrap into [0, L) and z folds into [0, Lz] by specular reflection
 *            at the walls (p_z flips at each reflection);
 *   stage 1: p += dt/2 F with the forces at the new positions.
 * F = F0 + F1 + F2 (device N x 3 arrays of the plan's type; NULL ones are
 * skipped), e.g. the long-range, short-range and particle-slab forces.
 * pos (stage 0 only), mom: device N x 3, updated in place; mass: device N or
 * NULL (all 1).  xi: standard normals from Philox4x32-10 with key = seed and
 * counter (particle, step, stream 3 for x, y; stream 4 for z), Box-Muller;
 * the same (seed, step) gives the same noise.  dt > 0, gamma >= 0, kT >= 0.
 */
q2d_status q2d_langevin_step(q2d_plan_t plan, void *pos, void *mom, const void *mass, int64_t N,
                             const void *F0, const void *F1, const void *F2, double dt,
                             double gamma, double kT, uint64_t seed, uint64_t step,
                             int32_t stage);

/*
 * q2d_plan_check -- wait for the plan's stream and return the first data error
 * found by the device-side checks of the calls since the last check
 * (Q2D_ENONNEUTRAL, Q2D_EOUTOFBOX, Q2D_ESAMPLER) or Q2D_OK; clears it.
 */
q2d_status q2d_plan_check(q2d_plan_t plan);

/*
 * q2d_soe_fit -- host FP64 SOE of exp(-x^2) with M terms (M even, 2 <= M <= 64)
 * by the midpoint rule on Weideman's optimised Talbot contour applied to the
 * inverse-Laplace representation of the Gaussian (Sec. 3), with the contour
 * scale that minimises the sup-norm error.  w, s: host arrays of 2M doubles
 * (re, im interleaved) filled on success; *sup_err (may be NULL) receives
 * max |exp(-x^2) - SOE(x)| measured on a grid of [0, 200].
 */
q2d_status q2d_soe_fit(int32_t M, double *w, double *s, double *sup_err);

/*
 * q2d_soe_fit_reduced -- host FP64 SOE of exp(-x^2) with M terms (M even,
 * 2 <= M <= Q2D_SOE_REDUCED_MAX) by model reduction, the construction the
 * paper's own tables (VPMR, Sec. 3 and Sec. 5) come from: the 48-term Talbot
 * SOE, read as the impulse response of a linear system with poles -s_l, is
 * reduced by square-root balanced truncation to its M states of largest
 * Hankel singular value; the reduced poles are the exponents (conjugate
 * pairs, Re s > 0), the weights follow by least squares, and a Lawson-weighted
 * Levenberg-Marquardt polish moves the table toward the minimax one.  Sup
 * errors: about 2e-8 (M = 8), 4e-10 (M = 10), 7e-12 (M = 12), where the Talbot
 * rule needs M = 16 for 7e-10 (beyond M = 12 the discarded Hankel singular
 * values reach the FP64 rounding level of the Gramians: use q2d_soe_fit).
 * Same outputs as q2d_soe_fit; takes up to a few seconds of host time.
 * Q2D_EUNSUPPORTED if a step fails to converge.
 */
#define Q2D_SOE_REDUCED_MAX 12
q2d_status q2d_soe_fit_reduced(int32_t M, double *w, double *s, double *sup_err);

/*
 * q2d_soe_fit_eps -- the fewest terms that reach a prescribed accuracy
 * (Sec. 3: the SOE error eps of eq. SOE1 is the accuracy parameter; Sec. 4.3:
 * M is picked for a tolerance): M = 2, 4, ..., M_max is tried in turn, each
 * with the better of q2d_soe_fit_reduced (M <= Q2D_SOE_REDUCED_MAX) and
 * q2d_soe_fit, and the first with sup error <= eps is returned in *M, w, s
 * (host arrays of at least 2 M_max doubles) and *sup_err (may be NULL).
 * Q2D_ECAPACITY if no M <= M_max reaches eps (w, s, *M then hold the M_max
 * fit); Q2D_EINVAL for eps <= 0 or M_max outside [2, 64].
 */
q2d_status q2d_soe_fit_eps(double eps, int32_t M_max, int32_t *M, double *w, double *s,
                           double *sup_err);

/*
 * Kernel timing (measurement only): the plan records HIP events around the
 * launches of the selected kernel families on the stream they run on and
 * accumulates their elapsed time.  Families: 0 = k != 0 sweep (the hot
 * kernel), 1 = k != 0 aggregate pass, 2 = z-sort, 3 = k = 0 term (internal
 * stream), 4 = whole call.  mask: bit w selects family w (0 disables; 31 =
 * all).  Every recorded event can delay the next launch by a few
 * microseconds, so time only what is needed.  q2d_plan_timing_read
 * synchronises and returns total milliseconds and the number of launches
 * measured since the last reset (enable resets).
 */
q2d_status q2d_plan_timing_enable(q2d_plan_t plan, int32_t mask);
q2d_status q2d_plan_timing_read(q2d_plan_t plan, int32_t which, double *ms_total, int64_t *count);
/*
 * Record the selected families only on every n-th call of the plan's entry
 * points (n >= 1; 1, the default, records every call), so that a timed loop
 * carries fewer events.  Returns Q2D_EINVAL for n < 1.
 */
q2d_status q2d_plan_timing_stride(q2d_plan_t plan, int32_t n);

/*
 * Replica batches -- R independent systems advanced by one random-batch step
 * together (the same alpha, SOE table and P; each replica its own box
 * Lx_r x Ly_r x [0, Lz_r], particle count n_r, lattice sum H_r and j = i
 * constant).  Every kernel family runs once for all replicas.
 *
 * q2d_batch_create: boxes = host array R x 3 (Lx, Ly, Lz); n = host array R
 *   (n_r >= 0, sum <= 2^31 - 1).  opts: precision, p_max (>= 1, the largest
 *   P), thin, validate (n_max is ignored).  Q2D_EINVAL on bad arguments.
 * q2d_batch_rbm_step: pos (sum n_r x 3) and q (sum n_r): device inputs with
 *   the replicas concatenated in order; phi, F: device outputs in the same
 *   layout (or NULL); E: device array of R doubles (or NULL), E_r =
 *   1/2 sum q_i phi_i over replica r.  Replica r draws its P modes exactly as
 *   q2d_rbm_step does with seed_r = seed + r * 0x9E3779B97F4A7C15 (mod 2^64)
 *   and the same step; modes_out: device int32 array R x P x 2, or NULL.
 *   Each replica's result is the single-system q2d_rbm_step result for its
 *   box and seed_r (Alg. 2, Fourier part).
 * q2d_batch_set_segment: segment length S (multiple of 64 in [64, 512]) of
 *   the replicas' layout.
 * q2d_batch_set_config / q2d_batch_get_config: the launch shapes of a step --
 *   segment length S; split = 1 (each sweep direction in its own work-groups)
 *   or 2 (both directions in one); agg_cpw = 1, 2 or 4 (16-mode chunks per
 *   wave of the FP32 aggregate pass).  Results do not depend on them beyond
 *   rounding.  Q2D_EINVAL for other values.
 * q2d_batch_tune: picks the launch shapes by timing candidates on the
 *   caller's data (phi, F, E serve as scratch; one untimed and 3 timed steps
 *   each), by coordinate descent: S over 64, 128, 256, 512, then split, then
 *   agg_cpw, then S again; keeps the fastest, returns its S in *segment, and
 *   caches the choice for the process by (device, R, total N, P, M,
 *   precision): a later tune of the same shape applies it without timing.
 * q2d_batch_capture: runs one step eagerly (step0), then captures one step
 *   into a hipGraph on the batch's internal stream; the graph reads its step
 *   number from device memory (starting at step0) and increments it last, so
 *   q2d_batch_replay(n) enqueues n steps step0, step0 + 1, ... on the batch's
 *   stream reading pos, q and writing phi, F, E at the captured addresses
 *   (keep them alive; update pos in place between replays).  A new layout or
 *   launch shape (set_segment, set_config, tune) drops the graph (replay then
 *   returns Q2D_EUNSUPPORTED).
 * q2d_batch_info: current S, padded particle count, and host copies of H_r
 *   and the random-batch j = i constants (arrays of R, or NULL).
 * q2d_batch_check: as q2d_plan_check.
 */
typedef struct q2d_batch *q2d_batch_t;
q2d_status q2d_batch_create(int32_t R, const double *boxes, const int64_t *n, double alpha,
                            int32_t M, const double *w, const double *s, const q2d_opts *opts,
                            void *stream, q2d_batch_t *out);
q2d_status q2d_batch_destroy(q2d_batch_t batch);
q2d_status q2d_batch_set_stream(q2d_batch_t batch, void *stream);
q2d_status q2d_batch_set_segment(q2d_batch_t batch, int32_t S);
q2d_status q2d_batch_set_config(q2d_batch_t batch, int32_t S, int32_t split, int32_t agg_cpw);
q2d_status q2d_batch_get_config(q2d_batch_t batch, int32_t *S, int32_t *split, int32_t *agg_cpw);
q2d_status q2d_batch_info(q2d_batch_t batch, int32_t *segment, int64_t *n_padded, double *H,
                          double *diag_rb);
q2d_status q2d_batch_rbm_step(q2d_batch_t batch, const void *pos, const void *q, int32_t P,
                              uint64_t seed, uint64_t step, void *phi, void *F, double *E,
                              int32_t *modes_out);
q2d_status q2d_batch_tune(q2d_batch_t batch, const void *pos, const void *q, int32_t P,
                          uint64_t seed, void *phi, void *F, double *E, int32_t *segment);
q2d_status q2d_batch_capture(q2d_batch_t batch, const void *pos, const void *q, int32_t P,
                             uint64_t seed, uint64_t step0, void *phi, void *F, double *E);
q2d_status q2d_batch_replay(q2d_batch_t batch, int32_t n_steps);
q2d_status q2d_batch_check(q2d_batch_t batch);

/* Static description of a status code. */
const char *q2d_status_string(q2d_status st);

#ifdef __cplusplus
}
#endif

#endif /* Q2D_H */
