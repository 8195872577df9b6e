/*
 * hjg.h -- C interface of the HJ-Gauss Monte-Carlo Picard sweep on AMD Instinct
 * MI355X (gfx950).
 *
 * The library solves the viscous Hamilton-Jacobi(-Isaacs) problem
 *     v_t + H(x, Dv) = nu * Lap v,   v(0, x) = l(x)        (t = time-to-go)
 * pointwise at batches of evaluation states, by the frozen-coefficient
 * (Picard) quasi-linearisation of Algorithm 1 of the HJ-Gauss paper
 * (Molu, Renganathan, Cho).  In the paper's notation delta = 2 nu and the
 * heat kernel of one step is N(x, delta t I).  One step, for each state x with
 * frozen coefficient c and proposal shift theta, draws z_i ~ N(0, I_n) and
 * forms (log-sum-exp, Monte-Carlo gradient and tilted-proposal corollaries of
 * the appendix; ESS as in Section 2.4):
 *     y_i = x + theta + sigma z_i,        sigma^2 = delta t
 *     a_i = -c l(y_i) - |theta|^2/(2 sigma^2) - <z_i, theta>/sigma
 *     v   = -(1/c) log((1/N) sum_i e^{a_i})
 *     Dv  = -(theta + sigma (sum_i e^{a_i} z_i / sum_i e^{a_i} - [zbar])) / (c sigma^2)
 *     ESS = (sum_i e^{a_i})^2 / sum_i e^{2 a_i}
 * where [zbar] = (1/N) sum_i z_i is subtracted only with grad_cv (a control
 * variate with mean zero).  The coefficient is c = (2/delta) H / (|p|^2 + eta)
 * with |c| clipped to [c_min, c_max] and its sign kept, sign(0) = +1
 * (coefficient definition of Section 2.1, the regularised-coefficient lemma
 * and the remark on the coefficient's sign); for H = |p|^2/2 it is exactly
 * 1/delta.  With the tube option H is replaced by min{0, H}.  The Laplace shift is theta = -sigma^2 c p (Section 2.4).
 *
 * Conventions shared by every entry point
 *  - Arrays marked "device" are device pointers on the context's GPU, owned by
 *    the caller; "host" arrays are host memory owned by the caller.  The
 *    library owns only the context (workspace, sample-table cache, graphs).
 *  - State arrays are dimension-major ("SoA"): element (d, q) of an [n][Q]
 *    array sits at index d*Q + q.  All floating-point arrays are float32
 *    unless stated otherwise.
 *  - Calls are asynchronous on the HIP stream passed in (NULL = default
 *    stream), except those with host outputs, which synchronise that stream
 *    before returning.
 *  - Arguments are validated before anything is launched; on error nothing is
 *    written, the return value is negative and hjg_last_error() describes it.
 *  - The Gaussian draws are Philox4x32-10 (Salmon et al., SC'11) with the
 *    stream layout documented at hjg_philox4x32_10 below; they are
 *    reproducible bit for bit from (seed, problem_id, time_step, iteration,
 *    query).
 *  - Not thread-safe per context: calls that share an hjg_ctx must be
 *    serialised by the caller, and run on one stream (or be ordered between
 *    streams by the caller): they share the context's workspace.
 *  - Non-finite outputs are reported, not passed on silently: every entry
 *    point that synchronises checks its outputs and returns HJG_ENONFINITE
 *    (outputs written, but some are NaN or infinite) where one is not finite;
 *    a fully asynchronous call leaves that check to the caller.
 *  - Environment switches, read per call, select alternative paths for
 *    comparison (the defaults are the tuned ones): HJG_NO_MFMA=1,
 *    HJG_TARGET_BLOCKS=n, HJG_NO_GRAPH=1, HJG_BATCH_SPLIT=n,
 *    HJG_BATCH_PERSISTENT=0|1, HJG_BATCH_CONCURRENT=0|1, HJG_TUBE_FUSED=0,
 *    HJG_TUBE_ROWS=n, HJG_MLP_FUSED=0 (the surrogate's layer-by-layer
 *    training step instead of the fused one).  The graph, launch-mode and
 *    row-chunk switches give the same bits; the path and split switches
 *    (HJG_NO_MFMA, HJG_TARGET_BLOCKS, HJG_BATCH_SPLIT, HJG_TUBE_FUSED,
 *    HJG_MLP_FUSED) change the float32 summation order, so results move at
 *    rounding level.
 */
#ifndef HJG_H
#define HJG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum hjg_status {
  HJG_OK = 0,
  HJG_ENOTCONVERGED = 1,  /* warning: outputs valid, tolerance not reached  */
  HJG_EINVAL = -1,        /* invalid argument, nothing launched              */
  HJG_ENOMEM = -2,        /* device workspace allocation failed              */
  HJG_EHIP = -3,          /* HIP runtime error                               */
  HJG_ENONFINITE = -4,    /* a non-finite value appeared in an output        */
  HJG_EUNSUPPORTED = -5   /* valid but unsupported combination               */
};

/* Hamiltonians H(x, p) = max_u min_w <p, f(x, u, w)>. */
enum hjg_ham {
  HJG_H_QUADRATIC = 0,       /* |p|^2/2; c = 1/delta exactly                           */
  HJG_H_DUBINS_PAIRS = 1,    /* sum over stacked relative Dubins pairs (n = 3m):
                                p1 (v_p cos x3 - v_e) + s p2 v_p sin x3
                                + w |p1 x2 - p2 x1 - p3| - w |p3|;
                                ham_p = {s, v_e, v_p, w}.  s = +1 follows from the
                                relative dynamics of the Dubins game in the
                                appendix, s = -1 is the form printed there.      */
  HJG_H_ZERO = 2,            /* H = 0 (pure diffusion; c = +c_min)                     */
  HJG_H_DOUBLE_INTEGRATOR = 3,/* n = 2k, k = 1, 2, 3, x = (pos[k], vel[k]), pos' = vel,
                                vel' = u, |u| <= u_max: <p_pos, vel> + u_max |p_vel|
                                (maximising control), or <p_pos, vel> - u_max |p_vel|
                                when ham_p[1] < 0 (minimising control: at n = 2 the
                                double integral plant of the appendix, eq. dint_ham
                                with u = -sign(p2): p1 x2 - |p2|);
                                ham_p = {u_max, s}                                    */
  HJG_H_PURSUIT_EVASION = 4, /* multi-pursuer single-evader game (Section 3.2): m = n/3
                                planar agents (x, y, heading), the last the evader;
                                sum_j a_j (p_xj cos th_j + p_yj sin th_j)
                                + u_max |p_th,evader| - u_max sum_pursuers |p_th,j|;
                                ham_p = {a_evader, a_pursuer, u_max}; 2 <= m <= 16 */
  HJG_H_ROCKETS = 5,         /* two rockets on a plane (appendix, game of two rockets),
                                n = 3, x = (x, z, theta) relative: with the rows of
                                its Hamiltonian definition eq. (ham_general),
                                H = -[a p1 cos th + p2 (a + a sin th - g)
                                      + u_max |p1 x - p3| - u_max |p2 x + p3|]
                                (evader u_e maximises, pursuer u_p minimises,
                                |u| <= u_max); ham_p = {a, g, u_max}              */
  HJG_H_MURMURATION = 6      /* the individual under attack in a flock (appendix,
                                murmuration Hamiltonian, general printed form),
                                n = 4, x = (x1, x2, altitude, heading) relative:
                                p1 (v_e - v_p cos x4) - p2 v_p sin x4 - w_p |p4|
                                + w_e |p2 x1 - p1 x2 + p4| + g_lo |p3| - g_hi |p3|;
                                ham_p = {v_e, v_p, w_e, w_p, g_lo, g_hi}          */
};

/* Terminal data l(y) (signed distance: negative inside the target set). */
enum hjg_datum {
  HJG_L_HALF_SQNORM = 0,     /* |y|^2 / 2                                              */
  HJG_L_BALL = 1,            /* |y[0:k]| - r; datum_p = {k, r}                         */
  HJG_L_MIN_PAIR_DISKS = 2,  /* min_j |(y[3j], y[3j+1])| - r (union of discs, n = 3m);
                                datum_p = {r}                                         */
  HJG_L_KNN_BALLS = 3,       /* min_j |y[0:3] - nb_j(q)| - r over the query's K
                                neighbour positions; datum_p = {r, K}, K <= 8;
                                datum_aux = device [K][3][Q]                          */
  HJG_L_LINEAR = 4,          /* <a, y> + b; datum_p = {b}; datum_aux = device a[n]     */
  HJG_L_CAPTURE = 5,         /* min over pursuers j of |(y[3j], y[3j+1]) - evader
                                position| - r, the evader being the last of the
                                m = n/3 agents (capture set of the Section 3.2 game);
                                datum_p = {r}; 2 <= m <= 16                           */
  HJG_L_DISC_UNION = 6       /* min_j |(y[0], y[1]) - c_j| - r over K fixed planar
                                centres shared by every state (union of capture
                                cylinders, murmuration setup); datum_p = {r, K},
                                K <= 8; datum_aux = device [K][2]; 2 <= n <= 16  */
};

/* Where the draws come from. */
enum hjg_sample_mode {
  HJG_S_FRESH = 0,      /* fresh draws per (query, iteration), generated in registers
                           (the paper's setting); n <= 16                           */
  HJG_S_CRN_STEP = 1    /* one common table z[n][N] per (problem, time step), shared
                           by every query and every Picard iteration               */
};

typedef struct hjg_problem {
  int32_t n;               /* state dimension, 1..48                               */
  int32_t ham;             /* enum hjg_ham                                          */
  double ham_p[8];          /* Hamiltonian parameters (see hjg_ham; unused entries 0) */
  int32_t datum;           /* enum hjg_datum                                        */
  double datum_p[4];
  const float* datum_aux;  /* device; see hjg_datum, else NULL                      */
  double nu;               /* viscosity; delta = 2 nu; > 0                          */
  double eta;              /* coefficient regulariser (>= 0)                        */
  double c_min, c_max;     /* clip range of |c| (0 < c_min <= c_max)                */
  int32_t tilt;            /* 1: Laplace shift theta = -sigma^2 c p from the current
                              gradient iterate (Section 2.4); 0: theta = 0          */
  int32_t sample_mode;     /* enum hjg_sample_mode                                  */
  int32_t sample_bf16;     /* 1: draws rounded to bfloat16 (nearest, ties to even)
                              and stored as bfloat16; arithmetic stays float32     */
  int32_t grad_cv;         /* 1: subtract zbar in the gradient (control variate)    */
  uint64_t seed;           /* Philox key                                            */
  uint32_t problem_id;     /* < 65536; part of the Philox tag                       */
  int32_t tube;            /* 1: the coefficient uses min{0, H} (the tube equation
                              HJI-RCBRT-Visc, v_t + min{0,H} = (delta/2) Lap v);
                              0: H as in Algorithm 1                                */
} hjg_problem;

typedef struct hjg_ctx hjg_ctx;

/* Create a context on HIP device `device`.  Returns HJG_OK and *out, or an
 * error (HJG_EHIP if the device cannot be used). */
int hjg_ctx_create(int device, hjg_ctx** out);
/* Release a context and all its device memory.  NULL is a no-op. */
void hjg_ctx_destroy(hjg_ctx* ctx);
/* Description of the last error on the calling thread ("" if none).  Valid
 * until the next call on that thread. */
const char* hjg_last_error(void);
/* Library version string. */
const char* hjg_version(void);

/*
 * Raw Philox4x32-10 words: for g in [0, G), out[4g + j] is word j of the block
 * cipher applied to counter (g, c1, c2, c3) under key (seed mod 2^32,
 * seed div 2^32).  The library's draws use counter
 * (i div 4, d, stream, tag) for sample i in dimension d, stream = query index
 * (FRESH) or 0xFFFFFFFF (common tables), tag = problem_id<<16 | time_step<<8 |
 * iteration, and map the words (w0, w1, w2, w3) to the normals of samples
 * 4g .. 4g+3 by Box-Muller on (w0, w1) and (w2, w3):
 *   u_a = ((w >> 8) + 1) 2^-24, u_b = (w >> 8) 2^-24,
 *   (r cos 2 pi u_b, r sin 2 pi u_b), r = sqrt(-2 ln u_a).
 * out: device uint32[4G].  Exposed so the draws can be checked bit for bit.
 */
int hjg_philox4x32_10(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3,
                      int64_t G, uint32_t* out, void* hip_stream);

/*
 * The common-random-number table of (problem, time_step): z[d][i] for d < n,
 * i < N, written to out (device, [n][N]); float32, or bfloat16 bits (uint16)
 * when problem->sample_bf16.  Used internally by the CRN mode; exposed for
 * checking.
 */
int hjg_sample_table(hjg_ctx* ctx, const hjg_problem* problem, int32_t N,
                     uint32_t time_step, void* out, void* hip_stream);

/*
 * One frozen-coefficient sweep (the estimators above) at Q states.
 *   x      device [n][Q]   evaluation states
 *   t      horizon (> 0)
 *   N      samples per state (>= 1)
 *   time_step, iter        Philox tag fields (iter used in FRESH mode only)
 *   c      device [Q]      frozen coefficient per state (non-zero, finite)
 *   theta  device [n][Q]   proposal shift, or NULL for theta = 0
 *   v      device [Q]      out: value
 *   grad   device [n][Q]   out: gradient
 *   ess    device [Q]      out: effective sample size, or NULL
 * Q = 0 is a no-op.  Returns HJG_ENONFINITE if an output is not finite
 * (checked only when check_finite != 0; the check synchronises the stream).
 */
int hjg_value_grad(hjg_ctx* ctx, const hjg_problem* problem, int64_t Q,
                   const float* x, double t, int32_t N, uint32_t time_step,
                   uint32_t iter, const float* c, const float* theta,
                   float* v, float* grad, float* ess, int32_t check_finite,
                   void* hip_stream);

/*
 * hjg_value_grad for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and the same results, bit for bit, as hjg_value_grad with
 * check_finite = 0 (same sample-split plan and kernels), but the call
 * allocates nothing and never synchronises: the sweep's scratch (split
 * partial sums, the common table, its column means, the pair-coordinate
 * copy) lives in one fixed device array of HJG_NOALLOC_SCRATCH_MIB MiB per
 * GPU, part of the library's code object (each GPU the library runs on holds
 * it until the process ends); its address is taken once per device by
 * hjg_ctx_create.  The common table is generated on every call into that
 * array (the context's table cache is not used), and every byte the kernels
 * read is written earlier in the same call, so no clearing is needed.
 * Returns HJG_EINVAL, before launching anything, when the call needs more
 * scratch than the array holds (about Q * splits * (20 + 4n) bytes plus, for
 * common draws, the table: the message gives the bytes needed).  Every call
 * on one GPU shares that GPU's array and it keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other contexts on the same
 * device, other host threads) race and give wrong results; order them.
 */
#define HJG_NOALLOC_SCRATCH_MIB 128
int hjg_value_grad_noalloc(hjg_ctx* ctx, const hjg_problem* problem, int64_t Q,
                           const float* x, double t, int32_t N, uint32_t time_step,
                           uint32_t iter, const float* c, const float* theta,
                           float* v, float* grad, float* ess, void* hip_stream);

/*
 * Algorithm 1 at Q states and horizon t: v^(0) = l(x), p^(0) = D l(x) (or p0),
 * then for k = 0..K-1: c^(k) = coefficient(x, p^(k)), theta^(k) (if tilt),
 * one sweep -> v^(k+1), Dv^(k+1); p^(k+1) = Dv^(k+1).  Stops after iteration k
 * when the relative L2 change ||v^(k+1) - v^(k)|| / ||v^(k)|| over the Q states
 * (float64) is below tol (tol <= 0: run all K).  The K iterations are recorded
 * once into a HIP graph and replayed; the stop is a device-side flag.
 *   p0        device [n][Q] warm-start gradient p^(0), or NULL for D l(x)
 *   v0        device [Q] warm-start value v^(0) (the reference of the first
 *             residual), or NULL for l(x)
 *   v, grad   device out, [Q] and [n][Q]: the last executed iterate
 *   c_out     device [Q] out: coefficient frozen in the last executed iteration,
 *             or NULL
 *   ess       device [Q] out, or NULL
 *   flags     device uint8 [Q] out: 1 where the per-state relative change
 *             |dv| / max(|v^(k)|, 1e-2 sigma sqrt(n)) is not <= tol (a NaN
 *             change is flagged), or v or Dv is not finite, at the last
 *             executed iteration; or NULL
 *   resid_hist host double [K] out: relative change per iteration (entries
 *             after the stop are set to 0), or NULL
 *   iters_done host out: number of executed iterations, or NULL
 * Synchronises the stream when resid_hist or iters_done is given or tol > 0;
 * such a call returns HJG_ENONFINITE when v or Dv of some state is not finite
 * after the last executed iteration (counted on the device in the residual
 * reduction), else HJG_ENOTCONVERGED (outputs valid) when tol > 0 was not
 * reached.  A call with neither host output nor tol > 0 is fully
 * asynchronous and reports no non-finite output.
 */
int hjg_picard_sweep(hjg_ctx* ctx, const hjg_problem* problem, int64_t Q,
                     const float* x, double t, int32_t N, int32_t K, double tol,
                     uint32_t time_step, const float* p0, const float* v0,
                     float* v, float* grad, float* c_out, float* ess, uint8_t* flags,
                     double* resid_hist, int32_t* iters_done, void* hip_stream);

/*
 * Algorithm 1 for P independent problems of uneven dimension, sample count,
 * state count, viscosity and iteration count in one call.  Problem p has
 * Q_p = q_off[p+1] - q_off[p] states (q_off host [P+1], q_off[0] = 0), N[p]
 * draws from its own common table (CRN_STEP only; time step 0; distinct
 * problem_id or seed give distinct tables), K[p] iterations and horizon t[p]
 * (host arrays [P]).  States: x_all device float32, problem p's [n_p][Q_p]
 * block starts at element sum_{p'<p} n_p' Q_p'; grad_all has the same layout;
 * v_all device [sum Q_p] at q_off[p].  All problems stop on the same
 * relative-change tolerance tol (<= 0: run all K[p]).
 *
 * Problems that share a kernel specialisation share its launches: each
 * Picard level is one pair-loop launch per specialisation over a work list
 * of (problem, query block, sample split) items ordered heaviest first, one
 * finalize launch per register bucket and one residual launch, and the whole
 * loop over levels is recorded once into a HIP graph (problems with K[p] <= k
 * drop out of level k; each has its own device stop flag).  resid_hist (host
 * [P][max K], entries past K[p] zero) and iters (host [P]) are optional;
 * giving either synchronises the stream, and such a call returns
 * HJG_ENONFINITE when some state of some problem ends with a non-finite value
 * or gradient.  A call whose batch differs from the previous call's waits for
 * that call's replay (on whatever stream it ran) before it re-plans.
 */
int hjg_picard_sweep_batched(hjg_ctx* ctx, int32_t P, const hjg_problem* problems,
                             const int64_t* q_off, const int32_t* N, const int32_t* K,
                             const double* t, double tol, const float* x_all,
                             float* v_all, float* grad_all, double* resid_hist,
                             int32_t* iters, void* hip_stream);

/*
 * ------------------------------------------------------------------------
 * Flock support: k nearest other agents of every agent through a uniform
 * hash grid (topological neighbour rule of the flocking example).  Their
 * positions, written as [k][3][M], are the datum_aux of HJG_L_KNN_BALLS with
 * Q = M (each agent's target set is the union of balls about its
 * neighbours; union of signed distances is their minimum).
 *
 * pos      device float32 [3][M] agent positions (SoA), all finite.
 * box_lo/hi host float[3]: the grid covers [lo, lo + g h) per axis with
 *          g = max(1, ceil((hi - lo) / cell)) cells; agents outside are
 *          clamped into the border cells (results stay exact).
 * cell     cell edge h > 0; at most 2^20 cells per axis and fewer than 2^26
 *          in all.
 * k        neighbours, 1..8; M > k.
 * idx      device int32 [k][M] or NULL: neighbour indices ordered by
 *          (squared distance, index), squared distance computed in float32
 *          as (dx*dx + dy*dy) + dz*dz, each operation rounded; never the
 *          agent itself.
 * nbr_pos  device float32 [k][3][M] or NULL: positions of those neighbours.
 * Exact for any point distribution: shells of cells are searched until no
 * unsearched cell can hold a nearer agent.  Synchronises the stream once
 * (the finiteness check of pos) before launching the build and search.
 * Returns HJG_ENONFINITE for a non-finite position, HJG_EINVAL for bad sizes.
 */
int hjg_knn_grid(hjg_ctx* ctx, int64_t M, const float* pos, const float* box_lo,
                 const float* box_hi, float cell, int32_t k, int32_t* idx, float* nbr_pos,
                 void* hip_stream);

/*
 * Autotuner.  The pair loop cuts each state's N draws into sample splits so a
 * launch has enough blocks; the split granularity is tuned per kernel
 * specialisation and size bucket (log2 Q, log2 N).
 * hjg_autotune_sweep times hjg_value_grad (HIP events, mean of 3 after one
 * warm-up) at the given arguments for targets of 512 .. 16384 blocks and keeps
 * the fastest in the context's tuning table (used by later hjg_value_grad and
 * hjg_picard_sweep calls in the same bucket); *best_blocks and *best_ms
 * receive the choice.  hjg_autotune_batched does the same for the samples per
 * split of hjg_picard_sweep_batched (2048 .. 65536), running the given batch,
 * then, at the chosen split, for its launch mode (persistent work-queue
 * launches or one block per item; a Picard level's pair loops as parallel
 * graph branches or one chain), kept as "batch_mode" = 1 + mode bits;
 * *best_ms is the time of the chosen split and mode.
 * Both synchronise the stream.  hjg_tuning_save / hjg_tuning_load write and
 * read the table as text ("hjg-tuning gfx950 1", then "key = value" lines);
 * load replaces the table, and rejects files of another format.
 */
int hjg_autotune_sweep(hjg_ctx* ctx, const hjg_problem* problem, int64_t Q, const float* x,
                       double t, int32_t N, const float* c, const float* theta,
                       int32_t* best_blocks, double* best_ms, void* hip_stream);
int hjg_autotune_batched(hjg_ctx* ctx, int32_t P, const hjg_problem* problems,
                         const int64_t* q_off, const int32_t* N, const int32_t* K,
                         const double* t, double tol, const float* x_all, float* v_all,
                         float* grad_all, int32_t* best_split, double* best_ms,
                         void* hip_stream);
int hjg_tuning_save(const hjg_ctx* ctx, const char* path);
int hjg_tuning_load(hjg_ctx* ctx, const char* path);

/*
 * Measurement helper (not part of the method): the issue rate of independent
 * full-rate (unpacked) float32 operations with waves_per_simd (1..8) blocks
 * of 4 waves resident per compute unit, each lane running 12 independent
 * chains for iters x 8 steps.  form 0: acc = acc * s + s with scalar s
 * (three-operand FMA); 1: acc += a * b with per-lane a, b (accumulating FMA);
 * 2: acc *= a; 3: acc = acc * a + b (three-operand FMA, per-lane operands);
 * 4: acc += s * a; 5: acc += s; 6: acc = min(acc, a, b); 7: forms 0 and 1
 * on alternate chains; 8-10: fixed inline-assembly sequences alternating
 * a scalar-operand FMA (S) and a vector-register accumulating FMA (F):
 * 8 independent, 9 each F reading the S just before it, 10 each F reading
 * the S two before it; 11 and 12: forms 1 and 10 with 256 vector registers
 * allocated (at most two waves per SIMD).  Writes the wave-level VALU instructions per
 * compute-unit clock (the chip's float32 vector peak, 157.3 TFLOP/s, is 2.0 per clock)
 * and the shader clock in GHz measured by the waves (shader-clock ticks
 * against the 100 MHz real-time counter).  Allocates a small workspace,
 * synchronises the stream.  Errors: HJG_EINVAL (arguments), HJG_ENOMEM,
 * HJG_EHIP.
 */
int hjg_probe_valu_rate(int32_t waves_per_simd, int32_t iters, int32_t form,
                        double* instr_per_cu_clock, double* clock_ghz, void* hip_stream);

/*
 * ------------------------------------------------------------------------
 * Learned surrogate (x, t) -> (v, Dv).
 *
 * A multilayer perceptron with n + 1 inputs (state and horizon), `depth`
 * hidden layers of `width` units with SiLU, and n + 1 linear outputs (value
 * and gradient), on normalised inputs and outputs.  Forward and backward run
 * as bfloat16 matrix-core GEMMs with float32 accumulation; float32 master
 * weights and AdamW moments.  The loss on a batch of B rows, in normalised
 * output units, is
 *   (1/B) sum_rows [ (y_0 - T_0)^2 + (grad_weight / n) sum_{j>=1} (y_j - T_j)^2 ].
 * Trained on values and gradients produced by the Monte-Carlo sweep; used by
 * hjg_surrogate_sweep as Picard warm start and proposal shift, with the plain
 * sweep as fallback and judge.  The surrogate lives on the device that was
 * current when it was created.  Parameter exchange format (host, float32):
 * for each layer in order, W [out][in] row-major, then b [out].
 * ------------------------------------------------------------------------
 */
typedef struct hjg_surrogate hjg_surrogate;

typedef struct hjg_train_cfg {
  int32_t epochs;        /* passes over the training rows (>= 1)              */
  int32_t batch;         /* rows per step, a multiple of 32                    */
  double lr, lr_min;     /* cosine schedule from lr to lr_min over all steps   */
  double weight_decay;   /* decoupled (AdamW)                                  */
  double beta1, beta2, eps;
  double grad_weight;    /* weight of the gradient outputs in the loss         */
  uint64_t seed;         /* per-epoch shuffling                                */
} hjg_train_cfg;

/* Create a network for states of dimension n (1..96); width a multiple of 32
 * (32..1024); depth 1..16 hidden layers; weights from `seed`; identity
 * normalisation. */
int hjg_surrogate_create(hjg_ctx* ctx, int32_t n, int32_t width, int32_t depth,
                         uint64_t seed, hjg_surrogate** out);
void hjg_surrogate_destroy(hjg_surrogate* s);
/* Number of parameters in the exchange format. */
int hjg_surrogate_param_count(const hjg_surrogate* s, int64_t* count);
/* Load parameters (host, exchange format) and normalisation (host float32
 * [4][n+1]: input mean, input std, output mean, output std; std > 0); resets
 * the optimiser state.  Synchronous. */
int hjg_surrogate_set_params(hjg_surrogate* s, const float* params, const float* norm);
/* Copy parameters (and, if norm != NULL, the normalisation) to host memory.
 * Synchronous. */
int hjg_surrogate_get_params(const hjg_surrogate* s, float* params, float* norm);
/* Write the network (shape, parameters in the exchange format, normalisation)
 * to a binary file; synchronous.  HJG_EINVAL on NULL or an I/O failure. */
int hjg_surrogate_save(const hjg_surrogate* s, const char* path);
/* Create a surrogate on the context's device from a file written by
 * hjg_surrogate_save (optimiser state reset).  HJG_EINVAL on NULL, an
 * unreadable or foreign file, or sizes that disagree with its header. */
int hjg_surrogate_load(hjg_ctx* ctx, const char* path, hjg_surrogate** out);
/* Evaluate at Q states: x device [n][Q], t device [Q]; v device [Q] and grad
 * device [n][Q] out.  Asynchronous. */
int hjg_surrogate_predict(hjg_surrogate* s, int64_t Q, const float* x,
                          const float* t, float* v, float* grad, void* hip_stream);
/* One forward and backward pass on B rows (B a multiple of 32) with targets
 * (v device [B], grad device [n][B]): *loss (host) and, if grads != NULL, the
 * parameter gradient in the exchange format (host).  Synchronous; for
 * checking the kernels. */
int hjg_surrogate_loss_grad(hjg_surrogate* s, int64_t B, const float* x,
                            const float* t, const float* v, const float* grad,
                            double grad_weight, double* loss, float* grads,
                            void* hip_stream);
/* Train on M rows (x [n][M], t [M], v [M], grad [n][M], all device); sets the
 * normalisation from the data; loss_hist (host [epochs], or NULL) receives the
 * mean training loss of each epoch.  Synchronises the stream each epoch.
 * Batches of 256, 512, 1024, 2048 or 4096 rows on networks of width 64, 128
 * or 256, padded input 32 or 64 and 2 to 4 hidden layers take the fused step
 * (two kernels per step, one recorded graph per epoch); the library then
 * keeps a permuted copy of the training set, M x (2 in_p + 4 out_p) bytes, on
 * the device.  Other shapes take the layer-by-layer step.  The two give the
 * same training up to the rounding of the bfloat16 operands. */
int hjg_surrogate_train(hjg_surrogate* s, int64_t M, const float* x,
                        const float* t, const float* v, const float* grad,
                        const hjg_train_cfg* cfg, double* loss_hist,
                        void* hip_stream);
/* Surrogate-accelerated sweep at Q states and horizon t:
 *   1. (v_S, Dv_S) = surrogate(x, t);
 *   2. hjg_picard_sweep with N_s draws and K_s iterations from the warm start
 *      v^(0) = v_S, p^(0) = Dv_S (so the first coefficient and proposal shift
 *      come from the surrogate), per-state flags with tolerance tol (> 0);
 *   3. the flagged states are compacted and solved again by the plain sweep
 *      (no warm start) with N_fb draws and K_fb iterations, and scattered back.
 * v, grad device out; fell_back device uint8 [Q] out (1 where step 3 ran);
 * *n_fallback (host) the number of such states.  A state whose step-2 result
 * is not finite (a non-finite surrogate output, say) is flagged and falls
 * back.  Synchronises the stream; returns HJG_ENONFINITE if a value or
 * gradient is still not finite after step 3. */
int hjg_surrogate_sweep(hjg_ctx* ctx, hjg_surrogate* s, const hjg_problem* problem,
                        int64_t Q, const float* x, double t, int32_t N_s,
                        int32_t K_s, int32_t N_fb, int32_t K_fb, double tol,
                        uint32_t time_step, float* v, float* grad,
                        uint8_t* fell_back, int64_t* n_fallback, void* hip_stream);
/* One step of time marching, the trained surrogate serving as the datum
 * (semigroup form of the viscous equation; tube equation HJI-RCBRT-Visc when
 * problem->tube is set).  The value at t_prev + dt solves the same equation
 * over [t_prev, t_prev + dt] from v(t_prev, .), so this is Algorithm 1 with
 * the horizon dt (sigma^2 = 2 nu dt) and the datum y -> v_S(y, t_prev), the
 * surrogate's value output at the previous time:
 *   v^(0) = v_S(x, t_prev), p^(0) = Dv_S(x, t_prev) (the surrogate's gradient
 *   output); for k < K: c and theta frozen from p^(k) as in hjg_picard_sweep;
 *   y_i = x + theta + sigma z_i; l_i = v_S(y_i, t_prev) from one forward pass
 *   of the network over the rows (query, sample) of a query chunk (up to 2^21
 *   rows per pass); the estimators, residual and stop rule of
 *   hjg_picard_sweep.
 * Draws: the common table of (problem, time_step) (sample_mode must be
 * HJG_S_CRN_STEP, float32 or bfloat16); N in [1, 2^21]; K in [1, 255].
 * problem->datum and datum_p must be valid but are not used.  x device
 * [n][Q]; v [Q], grad [n][Q] device out; c_out [Q] and ess [Q] device out or
 * NULL; resid_hist host [K] or NULL (zero past the last iteration);
 * *iters_done host or NULL.  problem->n must equal the surrogate's n.
 * Synchronises the stream after every iteration (the stop test is read on the
 * host).  Errors: HJG_EINVAL (arguments), HJG_EUNSUPPORTED (fresh draws),
 * HJG_ENOMEM, HJG_EHIP, HJG_ENONFINITE (some state ends with a non-finite
 * value or gradient; outputs written). */
int hjg_surrogate_tube_step(hjg_ctx* ctx, hjg_surrogate* s, const hjg_problem* problem,
                            int64_t Q, const float* x, double t_prev, double dt,
                            int32_t N, int32_t K, double tol, uint32_t time_step,
                            float* v, float* grad, float* c_out, float* ess,
                            double* resid_hist, int32_t* iters_done, void* hip_stream);

/*
 * ------------------------------------------------------------------------
 * Reach-avoid tube (the viscous reach-avoid variational inequality
 * HJI-RCBRAT-Visc, Section "Relations to Backward Reachable Sets/Tubes" and
 * the reach-avoid tube of the appendix): states of an avoid set
 * A = {l_A <= 0} must never count as reached.  In splitting form each time
 * step is the ordinary step (Algorithm 1, or hjg_surrogate_tube_step)
 * followed by the obstacle projection
 *   v <- max(v, -l_A(x)),   grad <- -D l_A(x) where -l_A(x) > v,
 * so every state of A keeps a value >= -l_A > 0 and no time step can bring
 * it below zero.  Marching then trains the next step's datum on the projected
 * labels.
 * ------------------------------------------------------------------------
 */
/* Obstacle projection in place.  obstacle: a problem record of which only n
 * and the datum fields (datum, datum_p, datum_aux) are read and checked (the
 * other fields are ignored): l_A is that datum (same kinks and tie rules as the
 * sweep's; knn_balls aux is indexed by the state index q < Q).  x device
 * [n][Q] (dimension-major, float32); v device [Q] in/out; grad device [n][Q]
 * in/out or NULL (then only v changes); active device uint8 [Q] out or NULL:
 * 1 where the projection replaced the value (strictly -l_A(x) > v in float32;
 * a NaN value is kept).  Q = 0 is a no-op.  Asynchronous on hip_stream.
 * Errors: HJG_EINVAL (NULL pointers with Q > 0, Q < 0, problem checks). */
int hjg_avoid_project(const hjg_problem* obstacle, int64_t Q, const float* x, float* v, float* grad,
                      uint8_t* active, void* hip_stream);

/*
 * ------------------------------------------------------------------------
 * Conservative safety certification (corollary "conservative safety
 * certification" of the total-error theorem).  A state is unsafe iff its
 * value is <= 0.  With a total error budget E the estimate certifies a state
 * SAFE only if v > E and UNSAFE only if v < -E; everything else is
 * UNDETERMINED, so with the theorem's probability no unsafe state is called
 * safe and no safe state unsafe.
 * ------------------------------------------------------------------------
 */
typedef struct hjg_budget {
  double C1, rho;      /* iteration term C1 rho^K                                 */
  int32_t K;
  double C2;           /* sampling term C2 sqrt(log(1/delta_p) / N)               */
  int64_t N;
  double delta_p;      /* failure probability, in (0, 1)                          */
  double eps_ql;       /* quasi-linearisation defect                              */
  double C3, delta;    /* viscosity term C3 sqrt(delta)                           */
} hjg_budget;
/* E = C1 rho^K + C2 sqrt(log(1/delta_p)/N) + eps_ql + C3 sqrt(delta) (host
 * arithmetic; the constants are the caller's).  HJG_EINVAL on NULL or on
 * negative terms. */
int hjg_error_budget(const hjg_budget* b, double* E);
/* Per-state sampling margin of the finite-sample concentration theorem for
 * the plain (unshifted) estimator with frozen coefficient c: Z = exp(-c g)
 * lies in [alpha, beta], the smaller and larger of exp(-c g_min) and
 * exp(-c g_max) (remark on the sign of the coefficient; g_max may be
 * +infinity), and with the mean taken as mu = exp(-c v) (the estimate's own)
 *   margin = -log(1 - r)/|c|,  r = (beta - alpha)/mu sqrt(log(2/delta_p)/(2N)),
 * or +infinity where r >= 1 (no finite margin at this N).  As c -> 0 it
 * tends to Hoeffding's (g_max - g_min) sqrt(log(2/delta_p)/(2N)).  With ess
 * (device [Q], the sweep's effective sample sizes) the variance-aware
 * empirical Bernstein form replaces it (the tighter kind of bound the paper's
 * remark on Bernstein points to; Maurer and Pontil 2009, two-sided):
 *   r = sqrt(2 V L/N) + 7 (beta - alpha)/mu L/(3(N - 1)),  L = log(4/delta_p),
 *   V = N/(N-1) (N/ESS - 1) (relative sample variance of the weights).
 * v, c device [Q]; margin device [Q] out (float32, computed in float64).
 * Asynchronous.  HJG_EINVAL: N < 1 (N < 2 with ess), delta_p outside (0, 1),
 * g_min not finite or g_max < g_min. */
int hjg_mc_margin(int64_t Q, const float* v, const float* c, const float* ess,
                  int32_t N, double delta_p, double g_min, double g_max,
                  float* margin, void* hip_stream);
/* Labels: label[q] = +1 (SAFE) if v[q] > E + m[q], -1 (UNSAFE) if
 * v[q] < -(E + m[q]), 0 (UNDETERMINED) otherwise, compared in float64, with
 * m = margin (device [Q]) or 0 when margin is NULL; label device int8 [Q] out
 * or NULL; counts device int64 [3] out or NULL: the number of UNSAFE,
 * UNDETERMINED and SAFE states (population certification).  Asynchronous.
 * HJG_EINVAL: E negative or not finite, both outputs NULL. */
int hjg_certify(int64_t Q, const float* v, const float* margin, double E,
                int8_t* label, int64_t* counts, void* hip_stream);

/*
 * ------------------------------------------------------------------------
 * Topology markers of the zero-sublevel set {v <= 0} on 2D slices (appendix
 * on vacuole nucleation topology: its detection algorithm and event rules).
 * ------------------------------------------------------------------------
 */
enum { HJG_EVENT_VACUOLE = 1, HJG_EVENT_CORDON = 2, HJG_EVENT_FRAGMENTATION = 4 };
/* For B slices of ny x nx grid values (v device float32 [B][ny][nx],
 * row-major, ny nx <= 16,384): n_comp[b] = connected components of
 * {v <= 0} (4-neighbour), beta1[b] = components of {v > 0} (4-neighbour)
 * that touch no edge of the grid, chi[b] = n_comp - beta1 (device int32 [B]
 * out).  A NaN counts as v > 0.  Asynchronous.  HJG_EINVAL on bad sizes or
 * NULL, HJG_EUNSUPPORTED for larger slices. */
int hjg_topology(int32_t B, int32_t ny, int32_t nx, const float* v,
                 int32_t* n_comp, int32_t* beta1, int32_t* chi, void* hip_stream);
/* Marching-squares isocontours of v = level on B slices (v device float32
 * [B][ny][nx]): cell (x, y) has corners c0 = (x, y), c1 = (x+1, y),
 * c2 = (x+1, y+1), c3 = (x, y+1); a corner is inside when v <= level; each
 * crossed edge is cut at the linear interpolation point; a cell with two
 * crossed edges gives one segment, the two saddle cells two, joined through
 * the cell centre when the mean of the corners is inside.  Segments go to
 * seg device float32 [max_seg][4] as (x0, y0, x1, y1) in (column, row) grid
 * units, with their slice in seg_slice device int32 [max_seg] (or NULL), in
 * no particular order; count device int64 [1] receives the total found,
 * which may exceed max_seg (then only max_seg were written).  Asynchronous. */
int hjg_isocontour(int32_t B, int32_t ny, int32_t nx, const float* v, float level,
                   float* seg, int32_t* seg_slice, int64_t max_seg, int64_t* count,
                   void* hip_stream);
/* Gaussian smoothing of B slices before the markers are read (the paper
 * smooths its slices' sampling speckle): out = v convolved along rows and then
 * columns with the normalised Gaussian of standard deviation sigma cells,
 * truncated at round(4 sigma) cells, mirror extension about the outer cell
 * edges.  v, out device float32 [B][ny][nx] (distinct), ny nx <= 16,384,
 * sigma in (0, 8].  Asynchronous. */
int hjg_smooth_slices(int32_t B, int32_t ny, int32_t nx, const float* v,
                      double sigma, float* out, void* hip_stream);
/* Event bits per step from the markers of T consecutive steps (host arrays):
 * HJG_EVENT_VACUOLE where chi[t] - chi[t-1] < -0.5, HJG_EVENT_CORDON where
 * beta1[t] >= 1 and beta1[t-1] == 0, HJG_EVENT_FRAGMENTATION where
 * n_comp[t] > n_comp[t-1]; events[0] = 0.  Host arithmetic. */
int hjg_topology_events(int32_t T, const int32_t* chi, const int32_t* beta1,
                        const int32_t* n_comp, int32_t* events);

/*
 * Kernel timing (profiling hook).  With timing enabled, every launch of the
 * pair-loop kernel made by hjg_value_grad / hjg_picard_sweep is bracketed by
 * HIP events on the caller's stream; while timing is on, the Picard loop is
 * launched kernel by kernel instead of being replayed from its recorded graph
 * (events recorded as graph nodes carry no usable timestamps).  hjg_sweep_time
 * waits for the last such call and returns the summed pair-loop kernel time
 * of that call (ms) and the number of launches timed.  Results are identical
 * with timing on or off.  Returns HJG_EINVAL on NULL arguments.
 */
int hjg_set_timing(hjg_ctx* ctx, int32_t enable);
int hjg_sweep_time(hjg_ctx* ctx, double* total_ms, int32_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* HJG_H */
