/*
 * mlmc_ap.h -- C ABI of the MI355X (gfx950) library for multilevel
 * asymptotic-preserving Monte Carlo particle simulation in the diffusive
 * scaling (Mortier, Robbe, Baelmans, Samaey, "Multilevel asymptotic-
 * preserving Monte Carlo for kinetic-diffusive particle simulations of the
 * Boltzmann-BGK equation").
 *
 * Problem (the paper's statement of the estimation task, Section 4.1):
 * estimate E[Q_L] = E[x_L(T)^2] for particles of the diffusively scaled BGK
 * equation  df/dt + (v/eps) df/dx = (M rho - f)/eps^2, where x_l is the
 * position at end time T of the fixed-time-step asymptotic-preserving
 * splitting scheme with step dt_l = dt0 / M^l:
 *     x <- x + h v + s xi,          h = dt eps/(eps^2+dt),
 *                                   s = sqrt(2 dt^2/(eps^2+dt)), xi ~ N(0,1)
 *     with probability p = dt/(eps^2+dt): v <- fresh draw from the equilibrium
 * (the asymptotic-preserving scheme of Dimarco et al. that the paper cites
 * in Section 1; the equilibrium has unit variance).  Level l >= 1 simulates
 * pairs: the fine path at dt_l and a coarse path at dt_{l-1} built only from
 * the fine random numbers, mapped by the time at which they act (Section
 * 3.1) and aggregated as in Section 3.2 (eqs. nu-update, epsilon-update,
 * chi-update).  The MLMC estimator is eq. mlmc-compact, with sample numbers
 * from eqs. Nopt1/Noptj and the statistical constraint of Section 4.1.
 *
 * Random numbers: Philox4x32-10 with key = seed.  The random numbers of one
 * trajectory are the word stream of its blocks 0, 1, 2, ... with counter
 * (block, sample, level tag, stream_id); the level tag is l for a
 * fine/coarse pair and l + 64 for a single-level (plain Monte Carlo)
 * trajectory.  The initial condition takes words 0-1 (a Box-Muller pair;
 * the density 1 + cos 2 pi x also word 2, and words 3-5 are skipped); every
 * fine step takes the next three: the collision decision word, then the
 * Box-Muller radius and angle words (the +-1 velocity sign is the top bit of
 * the angle word).  The coarse path draws nothing of its own.  Results
 * therefore depend only on (problem, level, sample index range) -- never on
 * launch shape, tuning or batching with other requests.  (Splitting one
 * range into several calls changes only the rounding of the merged
 * statistics.)
 *
 * Conventions for every function:
 *   - returns an mlmc_ap_status; nothing is thrown across the ABI;
 *   - pointers named *_host are caller-owned host memory, *_dev are
 *     caller-owned device memory on the current HIP device (e.g. from
 *     PyTorch), and `stream` is a hipStream_t (NULL = default stream);
 *   - the library owns its device workspace (grown on demand, freed by
 *     mlmc_ap_release or at process exit);
 *   - calls on one device are serialised by the library; results are
 *     written before the call returns (the call synchronises `stream`).
 */
#ifndef MLMC_AP_H
#define MLMC_AP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mlmc_ap_status {
    MLMC_AP_OK = 0,
    MLMC_AP_EINVAL = -1,      /* invalid argument; mlmc_ap_last_error() says which */
    MLMC_AP_ENOMEM = -2,      /* device or pinned host allocation failed */
    MLMC_AP_EDEVICE = -3,     /* HIP runtime error; mlmc_ap_last_error() has the text */
    MLMC_AP_EBUSY = -4,       /* serving: the request can never fit the memory budget */
    MLMC_AP_ECANCELLED = -5,  /* serving: the request was cancelled */
    MLMC_AP_ENOTFOUND = -6,   /* serving: unknown ticket */
    MLMC_AP_EAGAIN = -7       /* serving: request not finished yet */
} mlmc_ap_status;

/* Initial position law. */
enum { MLMC_AP_X0_DELTA = 0,    /* x0 = x0_a */
       MLMC_AP_X0_NORMAL = 1,   /* x0 ~ N(x0_a, x0_b^2) */
       MLMC_AP_X0_COSINE = 2 }; /* density 1 + cos(2 pi x) on [0, 1] */

/* Equilibrium (initial velocity law and collision resampling law). */
enum { MLMC_AP_EQ_TWO_POINT = 0,   /* v = +1 or -1, each with probability 1/2 */
       MLMC_AP_EQ_MAXWELLIAN = 1 };/* v ~ N(0, 1) */

/* Coarse kick aggregation (eq. chi-update). */
enum { MLMC_AP_COUPLING_KICK_SUM = 0,  /* normalised sum of the M fine kick normals */
       MLMC_AP_COUPLING_AGGREGATE = 1  /* also the fine velocity normals the coarse
                                          path does not reuse, weighted by their
                                          fine transport uses; Maxwellian only */ };

/* Quantity of interest. */
enum { MLMC_AP_QOI_X2 = 0,        /* Q = x(T)^2 */
       MLMC_AP_QOI_X2_HIST = 1,   /* x(T)^2 plus a position histogram */
       MLMC_AP_QOI_X = 2 };       /* Q = x(T), the expected position of Section 5 */

/* Background of the KD scheme.  DIFFUSIVE: the diffusive scaling, collision
 * rate R = 1/eps^2 and Maxwellian N(0, 1/eps^2).  B1, B2: the test case of
 * Section 5, Maxwellian N(0, 1) (mu = 0, sigma = 1; eps is not used) and a
 * collision rate that is piecewise linear with a kink at x = 1:
 *   B1 (symmetric):  R(x) = b (a |x - 1| + 1),
 *   B2 (asymmetric): R(x) = b for x <= 1, b (a (x - 1) + 1) for x > 1,
 * parameters bg_a = a >= 0 and bg_b = b > 0 (a = 0: homogeneous, R = b).
 * Flight times solve eq. intinv exactly for the piecewise-linear rate; the
 * diffusive phase uses eqs. advection and diffusion with the collision rate
 * at the collision point (the paper's corrected a^hetero, d^hetero are not
 * stated in it); pairs follow Algorithm "Correlated KD algorithm" with the
 * general eq. epsilon-update (the rate integral along the fine flight). */
enum { MLMC_AP_BG_DIFFUSIVE = 0, MLMC_AP_BG_B1 = 1, MLMC_AP_BG_B2 = 2 };

/* Particle scheme (Section 2).  SPLITTING: the asymptotic-preserving
 * splitting scheme at fixed dt (transport-diffusion step with the
 * eps- and dt-dependent drift and Gaussian kick, then a collision with
 * probability dt/(eps^2+dt)); fine/coarse pairs as in Section 3 with the
 * fixed-step mapping.  KD: the kinetic-diffusion scheme (Algorithm "KD
 * algorithm") in a homogeneous background, collision rate R = 1/eps^2 and
 * Maxwellian velocities N(0, 1/eps^2); pairs by Algorithm "Correlated KD
 * algorithm" (eqs. nu-update, epsilon-update, chi-update with the weights
 * alpha and beta of Section 3.2).  KD needs eps > 0, the Maxwellian
 * equilibrium and fp64_state = 1 (its step decisions are taken on FP64
 * times); coupling is ignored; its collision counts are KD steps, i.e.
 * collisions before T; random numbers: Philox block 0 = initial condition,
 * block k+1 = KD step k (Box-Muller pair nu_{k+1}, chi_k and E_{k+1} =
 * -log u). */
enum { MLMC_AP_SCHEME_SPLITTING = 0,
       MLMC_AP_SCHEME_KD = 1 };

#define MLMC_AP_MAX_LEVELS 31   /* levels 0..30 */
#define MLMC_AP_MAX_BINS 1024

typedef struct mlmc_ap_problem {
    double eps;          /* diffusive scaling parameter, >= 0 (0 = diffusion limit) */
    double T;            /* end time, > 0 */
    double dt0;          /* level-0 step; T/dt0 must be a positive integer (1e-9 rel.) */
    int32_t M;           /* refinement factor dt_{l-1}/dt_l, 2..64 */
    int32_t L;           /* finest level, 0..30; n_L = (T/dt0) M^L must be < 2^31 */
    int32_t x0_kind;     /* MLMC_AP_X0_* */
    int32_t eq_kind;     /* MLMC_AP_EQ_* */
    double x0_a;         /* delta: position; normal: mean */
    double x0_b;         /* normal: standard deviation (>= 0) */
    int32_t coupling;    /* MLMC_AP_COUPLING_*; AGGREGATE needs MAXWELLIAN */
    int32_t qoi;         /* MLMC_AP_QOI_* */
    int32_t nbins;       /* histogram bins, 1..MLMC_AP_MAX_BINS (QOI_X2_HIST) */
    int32_t fp64_state;  /* 0: FP32 particle state (default), 1: FP64 state */
    double hist_lo;      /* histogram range [hist_lo, hist_hi) */
    double hist_hi;
    uint64_t seed;       /* Philox key */
    uint32_t stream_id;  /* fourth counter word (request / stream id) */
    uint32_t scheme;     /* MLMC_AP_SCHEME_* (0 = splitting) */
    uint32_t background; /* MLMC_AP_BG_* (KD scheme only; 0 = diffusive scaling) */
    double bg_a, bg_b;   /* B1/B2 parameters a >= 0, b > 0 */
} mlmc_ap_problem;

/* Per-level statistics, mergeable (Chan et al. pairwise update) in FP64.
 * dq = Q_f - Q_c (level 0 or single: dq = Q_f, Q_c = 0).  m2_* are sums of
 * squared deviations (sample variance = m2/(n-1)); c_fc is the co-moment of
 * Q_f and Q_c.  coll_* count fine and coarse collisions. */
typedef struct mlmc_ap_level_stats {
    uint64_t n;
    double mean_dq, m2_dq;
    double mean_qf, m2_qf;
    double mean_qc, m2_qc;
    double c_fc;
    uint64_t coll_f, coll_c;
} mlmc_ap_level_stats;

/* Histogram counts of one level: for bin b (0 <= b < nbins)
 *   hist[3b]   = #{x_f in bin b},
 *   hist[3b+1] = #{x_c in bin b},
 *   hist[3b+2] = #{x_f and x_c both in bin b},
 * then hist[3 nbins + 0..3] = #{x_f below}, #{x_f above}, #{x_c below},
 * #{x_c above}.  Total length 3*nbins + 4 (uint64). */

/* Constants of one level, computed on the host in FP64 (for tests and
 * tooling; no device work). */
typedef struct mlmc_ap_level_info {
    double dt, h, s, p;          /* fine step and scheme coefficients */
    double dt_c, h_c, s_c, p_c;  /* coarse (level l-1) ones; zero at level 0 */
    uint64_t n_steps;            /* fine steps n_l */
    uint64_t thr_f;              /* collide iff word < thr_f = round(p 2^32) */
    uint64_t thr_c;              /* round(p_c 2^32) (level l-1's own threshold) */
    uint64_t thr_c2;             /* coarse decision word threshold (see below) */
} mlmc_ap_level_info;

/* Tuning of the particle kernels; zero fields select the defaults (or the
 * autotuner's cached choice).  Results never depend on it: the
 * time-parallel path (one trajectory per wavefront, its fine steps spread
 * over the lanes; for few long trajectories such as a warm-up) repeats the
 * per-lane arithmetic in the same order and gives bitwise identical
 * trajectories and statistics. */
typedef struct mlmc_ap_tuning {
    int32_t block;          /* threads per block: 64, 128 or 256 */
    int32_t ppt;            /* trajectories in flight per thread: 1, 2 or 4 */
    int32_t waves_per_simd; /* persistent grid occupancy target, 1..8 (capped at
                               what the kernel's registers allow) */
    int32_t tp_max_samples; /* time-parallel path for work items of at most this
                               many samples with >= 64 fine steps (pairs: M = 2
                               or 4); 0 = 4096, < 0 = never */
} mlmc_ap_tuning;

typedef struct mlmc_ap_options {
    int32_t batched;        /* 0 (default): all levels of an iteration in one
                                  persistent launch (stage, persistent, reduce
                                  kernels) issued directly; the warm-up launch of
                                  a lone request with all levels of a fixed L
                                  takes its first top-up along, planned on the
                                  device (result.device_planned);
                               3: as 0, every launch planned by the host;
                               1: the same launches replayed from captured
                                  hipGraphs (one graph per launch shape, kept by
                                  the library), planned by the host;
                               2: as 0, with HIP events around the particle
                                  kernels, so kernel_seconds is measured;
                               -1: one plain launch per level.
                               All five give bitwise identical results. */
    int32_t max_iter;       /* MLMC top-up iterations after warm-up (0 = 10) */
    uint64_t n_warmup;      /* warm-up samples per level (0 = 1000) */
    mlmc_ap_tuning tuning;
    int32_t level_select;   /* MLMC_AP_LEVELS_ALL (0, default): levels 0..L;
                               MLMC_AP_LEVELS_HEURISTIC: the level set of
                               mlmc_ap_select_levels_heuristic from the warm-up's
                               V_l and V_{l,l-1}; the pairs of the set that are not
                               adjacent levels get a warm-up of their own, adjacent
                               ones keep their warm-up samples;
                               MLMC_AP_LEVELS_OPTIMAL: the set of
                               mlmc_ap_select_levels_optimal, with the warm-up also
                               running pilot pairs (L, i), i <= L-2: the variances of
                               the pairs (i, i-1) and (L, i) are measured, the others
                               taken from eq. V_approx with the correlations
                               rho_{L,i}; costs n_i (+ n_j);
                               MLMC_AP_LEVELS_HEURISTIC_TAU (KD scheme only): the
                               off-line part of Section 5.3, a warm-up of the
                               adjacent pairs of levels 0..tau only (tau of
                               mlmc_ap_warmup_depth, dt_tau about the mean free
                               time), the profile beyond tau from
                               mlmc_ap_extrapolate_variances, then the heuristic
                               set; warm-up pairs that stay in the set keep their
                               samples, the other items of the set get a warm-up of
                               their own.  Costs: expected KD steps
                               n_l (1 - exp(-R dt_l)) per path (R = bg_b, or 1/eps^2
                               in the diffusive scaling). */
    int32_t L_max;          /* 0: the finest level is p->L.  p->L < L_max <= 30:
                               level-adaptive finest level (eq. bias_constraint;
                               the nested level sets of Section 5.2): each time the
                               statistical constraint holds, if bias_estimate of
                               the result exceeds tol/sqrt(2) and L < L_max, L
                               grows by one, the set is chosen again for the new L
                               (LEVELS_ALL: the adjacent pair (L+1, L) is added;
                               LEVELS_HEURISTIC_TAU: the heuristic on the same
                               warm-up profile) and the estimate goes on with every
                               sample of the items that stay.  Only with
                               LEVELS_ALL or LEVELS_HEURISTIC_TAU, not with plain
                               Monte Carlo or per-level histograms. */
} mlmc_ap_options;

enum { MLMC_AP_LEVELS_ALL = 0, MLMC_AP_LEVELS_HEURISTIC = 1, MLMC_AP_LEVELS_OPTIMAL = 2,
       MLMC_AP_LEVELS_HEURISTIC_TAU = 3 };

typedef struct mlmc_ap_result {
    double estimate;         /* eq. mlmc-compact: sum_l mean(dQ_l) */
    double var_estimator;    /* sum_l V_l / N_l with sample variances V_l */
    int32_t L;
    int32_t iterations;      /* top-up iterations run */
    int32_t converged;       /* 1 if sum_l V_l/N_l <= tol^2/2 */
    int32_t status;          /* mlmc_ap_status of the request (serving) */
    uint64_t N[MLMC_AP_MAX_LEVELS];
    mlmc_ap_level_stats lv[MLMC_AP_MAX_LEVELS];
    uint64_t particle_steps; /* sum_l N_l (n_l + n_{l-1}) */
    uint64_t launches;       /* particle-kernel launches or graph replays */
    double seconds;          /* host wall clock of the call */
    double gpu_seconds;      /* device time from table upload to statistics read-back */
    double kernel_seconds;   /* device time of the particle kernels alone (plain and
                                direct persistent launches; 0 for graph replays) */
    uint64_t level_mask;     /* bit l set for every level of the hierarchy used; N[l]
                                and lv[l] of a level l_j of the set hold the samples of
                                Q_{l_j} - Q_{l_{j-1}} (of Q_{l_1} for the first) */
    double bias_estimate;    /* |E[Q_L - Q]| estimated from the finest term:
                                |mean(Q_L - Q_c)| / (M^(L-c) - 1), c the level below L
                                in the set (first-order weak convergence in dt); NaN
                                if the set is {L} alone */
    double bias_se;          /* standard error of bias_estimate:
                                sqrt(V_{L,c} / N_L) / (M^(L-c) - 1) (NaN as above) */
    int32_t tau;             /* highest level of the warm-up before the selection (p->L
                                but for LEVELS_HEURISTIC_TAU) */
    int32_t levels_added;    /* finest levels added by options.L_max (L = p->L + this) */
    int32_t device_planned;  /* top-ups whose sample numbers and work table the device
                                computed right after the warm-up (direct launch forms,
                                one request, all levels; the host checks the numbers),
                                0 or 1: the results are the same either way */
    int32_t reserved;
} mlmc_ap_result;

/* Library and device set-up.  mlmc_ap_init is optional (every entry point
 * initialises lazily); mlmc_ap_release frees the workspace of the current
 * device. */
mlmc_ap_status mlmc_ap_init(void);
mlmc_ap_status mlmc_ap_release(void);
const char* mlmc_ap_status_str(mlmc_ap_status s);
/* Text of the last error of the calling thread ("" if none). */
const char* mlmc_ap_last_error(void);
/* Library version string. */
const char* mlmc_ap_version(void);

/* Validates a problem (the EINVAL rules listed in the struct comments). */
mlmc_ap_status mlmc_ap_validate(const mlmc_ap_problem* p);

/* Level constants (host only).  thr_c2 is the threshold of the coarse
 * collision decision: the coarse path of level l collides in coarse step K
 * iff the smallest fine decision word of fine steps K*M..K*M+M-1 is below
 * thr_c2.  Those M words are independent and uniform, so the coarse
 * collision probability is 1 - (1 - thr_c2/2^32)^M, and
 * thr_c2 = round(2^32 (1 - (1 - thr_c/2^32)^(1/M))) makes it the coarse
 * level's own thr_c/2^32 within M 2^-32.  thr_c2 <= thr_f, so every coarse
 * collision reuses a fine one (the uniform analogue of reusing the fine
 * exponential number in eq. epsilon-update) and its new velocity is the fine
 * velocity drawn last in the block (eq. nu-update). */
mlmc_ap_status mlmc_ap_level_constants(const mlmc_ap_problem* p, int32_t level,
                                       mlmc_ap_level_info* out_host);

/* Eqs. Nopt1/Noptj (host only): N_j = ceil((2/tol^2) sqrt(V_j/C_j)
 * sum_i sqrt(V_i C_i)) for j < n.  V_j >= 0, C_j > 0, tol > 0. */
mlmc_ap_status mlmc_ap_optimal_samples(const double* V_host, const double* C_host, int32_t n,
                                       double tol, uint64_t* N_out_host);

/* Level selection (host only).  Heuristic of Section 5.2 (Algorithm
 * "Heuristic level selection approach"): from V_l = Var[Q_l] (l = 0..L) and
 * Vdiff_l = Var[Q_l - Q_{l-1}] (l = 1..L; Vdiff_host[0] is ignored), start
 * with the first l whose Vdiff_l <= V_l and l - 1, then add every later level
 * whose Vdiff_l is below half the last one added.  Readings: the scan starts
 * after that first pair (the printed loop from l = 0 would read Vdiff_0);
 * if no level qualifies the set is {L} (plain Monte Carlo at L); L is always
 * added (Section 4.1 restricts the sets to l_J = L, which makes the estimator
 * unbiased for E[Q_L]).  So the sets for L and L + 1 share every level below
 * L (the nesting of Section 5.2, up to the finest level).  *mask_out: bit l
 * set for each selected level. */
mlmc_ap_status mlmc_ap_select_levels_heuristic(const double* V_host, const double* Vdiff_host,
                                               int32_t L, uint64_t* mask_out);

/* eq. level_selection (host only): the set {l_1 < ... < l_J = L} that
 * minimises sqrt(V_{l_1} C_{l_1}) + sum_{j>=2} sqrt(V_{l_j,l_{j-1}} C_{l_j,l_{j-1}}),
 * found exactly as a shortest path over the levels (the problem the paper
 * writes as an integer linear programme).  V_host, C_host: L+1 values of
 * the single levels; Vpair_host, Cpair_host: (L+1) x (L+1) row-major, entry
 * [i][j] (i > j) for the pair (i, j).  All >= 0 (C > 0).  *cost_out
 * (nullable) receives the minimum. */
mlmc_ap_status mlmc_ap_select_levels_optimal(const double* V_host, const double* C_host,
                                             const double* Vpair_host, const double* Cpair_host,
                                             int32_t L, uint64_t* mask_out, double* cost_out);

/* Warm-up depth of Section 5.3 (host only): the level tau whose step
 * dt_tau = dt0 M^-tau is nearest, in log scale, to the mean free time 1/R
 * (R = bg_b in a background of Section 5, 1/eps^2 in the diffusive scaling),
 * clamped to [1, L] (0 if L = 0).  Levels 0..tau are those whose steps are
 * at least about 1/R, where the measured difference variances are needed. */
mlmc_ap_status mlmc_ap_warmup_depth(const mlmc_ap_problem* p, int32_t* tau_out);

/* Variance profile of Section 5.3 (host only): from measured V_l and
 * V_{l,l-1} of levels 0..tau (V_host, Vdiff_host: tau+1 values, Vdiff_host[0]
 * ignored), the profile of levels 0..L (V_out_host, Vdiff_out_host: L+1
 * values): the measured values up to tau, beyond it the asymptotic rate
 * V_{l,l-1} = O(dt_l^3), i.e. V_{l,l-1} = V_{tau,tau-1} / M^(3 (l - tau)), and
 * V_l = V_tau.  0 <= tau <= L <= 30, 2 <= M <= 64, values >= 0. */
mlmc_ap_status mlmc_ap_extrapolate_variances(const double* V_host, const double* Vdiff_host,
                                             int32_t tau, int32_t M, int32_t L,
                                             double* V_out_host, double* Vdiff_out_host);

/* Pairwise merge of two statistics records (host only; the same update the
 * device reductions apply): out = a (+) b.  out may alias a or b. */
mlmc_ap_status mlmc_ap_merge_stats(const mlmc_ap_level_stats* a, const mlmc_ap_level_stats* b,
                                   mlmc_ap_level_stats* out);

/* Simulates samples [sample_begin, sample_begin + n_samples) of level
 * `level` on the GPU (Section 4.1: the n-th realisation of Q_{l_1} or of the
 * difference dQ_{l_j,l_{j-1}} of eq. mlmc-compact) and returns their
 * statistics.
 *   single = 0: fine/coarse pair (level 0: the fine path alone);
 *   single = 1: one trajectory of level `level` alone (plain Monte Carlo,
 *               level tag level + 64), statistics with Q_c = 0.
 *   out_host  (required) statistics of this range only.
 *   traj_dev  (nullable) 2*n_samples values, float (fp64_state = 0) or
 *             double: x_f(T) at [i], x_c(T) at [n_samples + i], i = sample -
 *             sample_begin.
 *   coll_dev  (nullable) 2*n_samples uint32: fine collisions at [i], coarse
 *             at [n_samples + i].
 *   hist_host (nullable; required when qoi = QOI_X2_HIST) 3*nbins + 4
 *             uint64 histogram counts of this range (layout above).
 * sample_begin + n_samples must not exceed 2^32 (sample counter word). */
mlmc_ap_status mlmc_ap_simulate_level(const mlmc_ap_problem* p, int32_t level, int32_t single,
                                      uint64_t sample_begin, uint64_t n_samples,
                                      mlmc_ap_level_stats* out_host, void* traj_dev,
                                      uint32_t* coll_dev, uint64_t* hist_host, void* stream);

/* As mlmc_ap_simulate_level (single = 0) for the pair of levels
 * (level, coarse_level) of a non-contiguous hierarchy (Section 4.2): the
 * coarse path is the scheme at level coarse_level (0 <= coarse_level <
 * level), one coarse step per M^(level - coarse_level) fine steps, built from
 * the fine random numbers as for adjacent levels; coarse_level = level - 1
 * is mlmc_ap_simulate_level.  Samples use the fine level's counter tag.
 * EINVAL for coarse_level outside [0, level). */
mlmc_ap_status mlmc_ap_simulate_pair(const mlmc_ap_problem* p, int32_t level, int32_t coarse_level,
                                     uint64_t sample_begin, uint64_t n_samples,
                                     mlmc_ap_level_stats* out_host, void* traj_dev,
                                     uint32_t* coll_dev, uint64_t* hist_host, void* stream);

/* Allocation-free form of mlmc_ap_simulate_level, for callers that cannot
 * allocate device memory: code being captured into a HIP graph, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, meaning, layout and
 * results (bitwise) as mlmc_ap_simulate_level.  It calls no hipMalloc,
 * hipHostMalloc or hipFree and creates no stream or event: its descriptor,
 * tile and group records, reduction counter, statistics slot and histogram
 * counters live in a device array of the library (MLMC_AP_NOALLOC_SCRATCH_BYTES,
 * about 5 MiB, one copy on every GPU the library runs on, held until the
 * process ends); the caller still passes the outputs (out_host, and the
 * optional traj_dev, coll_dev, hist_host).  EINVAL if n_samples exceeds
 * MLMC_AP_NOALLOC_MAX_SAMPLES.  Every call on a GPU uses that GPU's one array,
 * which keeps the last call's contents: the library runs these calls one at a
 * time (each returns after `stream` has finished its work), and kernels that
 * other code enqueues on that array at the same time would race with it. */
#define MLMC_AP_NOALLOC_MAX_SAMPLES 4194304ull   /* 2^22 samples per call */
#define MLMC_AP_NOALLOC_SCRATCH_BYTES 5289216ull
mlmc_ap_status mlmc_ap_simulate_level_noalloc(const mlmc_ap_problem* p, int32_t level,
                                              int32_t single, uint64_t sample_begin,
                                              uint64_t n_samples, mlmc_ap_level_stats* out_host,
                                              void* traj_dev, uint32_t* coll_dev,
                                              uint64_t* hist_host, void* stream);

/* MLMC estimate of E[Q_L] to RMSE tolerance rmse_tol (Section 4.1): warm-up
 * samples on every level 0..L, then eqs. Nopt1/Noptj with sample variances
 * and the deterministic cost C_0 = n_0, C_l = n_l + n_{l-1} (particle steps
 * per sample; for the KD scheme the expected KD steps,
 * C = sum over the paths of n (1 - e^{-R dt}), rounded up), topped up until
 * the statistical constraint
 * sum_l V_l/N_l <= rmse_tol^2/2 holds.  Level l uses samples [0, N_l).
 * opt may be NULL (defaults).  With qoi = QOI_X2_HIST, hist_host (nullable)
 * receives (L+1) per-level histograms of 3*nbins+4 counts each. */
mlmc_ap_status mlmc_ap_estimate(const mlmc_ap_problem* p, double rmse_tol,
                                const mlmc_ap_options* opt, mlmc_ap_result* out_host,
                                uint64_t* hist_host, void* stream);

/* The epsilon-adaptive on-line phase of Section 5.3: the MLMC estimate of
 * mlmc_ap_estimate run through the decreasing tolerances
 * tol_r = rmse_tol0 / sqrt(2^r), r = 0..R (the paper takes rmse_tol0 = 1), so
 * that each stage costs about twice the previous one.  Reading of the paper's
 * "repeatedly": the stages continue one estimate.  The warm-up (and the level
 * selection of opt->level_select) happens once; stage r computes eqs.
 * Nopt1/Noptj at tol_r from the statistics so far, tops up (samples are never
 * discarded: level l keeps using samples [0, N_l)) and ends when
 * sum_l V_l/N_l <= tol_r^2/2 or after opt->max_iter top-ups.
 *   out_host  R + 1 results (caller-owned), out_host[r] the state at the end
 *             of stage r: estimate, variance, N, per-level statistics, and the
 *             work, launches and times spent since the call began.  The
 *             statistics of the finest level, lv[L].mean_dq and its sample
 *             variance, estimate the level-L correction that the paper's
 *             bias estimates rest on, with more samples at every stage.
 * Stage 0 equals mlmc_ap_estimate at rmse_tol0 (bitwise, except for times).
 * EINVAL for R outside [0, 40]; per-level histograms are not produced. */
mlmc_ap_status mlmc_ap_estimate_sequence(const mlmc_ap_problem* p, double rmse_tol0,
                                         int32_t R, const mlmc_ap_options* opt,
                                         mlmc_ap_result* out_host, void* stream);

/* Plain Monte Carlo at level L (single-level trajectories, level tag
 * L + 64): N = ceil(2 V_L / rmse_tol^2) samples after the warm-up,
 * iterated like mlmc_ap_estimate.  Reported in out_host->N[L] / lv[L]. */
mlmc_ap_status mlmc_ap_plain_mc(const mlmc_ap_problem* p, double rmse_tol,
                                const mlmc_ap_options* opt, mlmc_ap_result* out_host,
                                void* stream);

/* Several independent MLMC estimates advanced together: every top-up
 * iteration of every request is one persistent launch over a shared work
 * table (uneven N_l across requests and levels), replayed from one captured
 * hipGraph.  Each result equals what mlmc_ap_estimate returns for that
 * request alone (bitwise).  n_req >= 1. */
mlmc_ap_status mlmc_ap_estimate_batch(const mlmc_ap_problem* p, const double* rmse_tol,
                                      int32_t n_req, const mlmc_ap_options* opt,
                                      mlmc_ap_result* out_host, void* stream);

/* Autotuner: runs complete MLMC estimates of p at rmse_tol (persistent
 * launches issued directly, timed with HIP events on `stream`) for every
 * (block, ppt, waves_per_simd) candidate and returns the one with the least
 * particle-kernel time.  If cache_path is non-NULL the choice is read from /
 * written to that JSON file (keyed by the device name).  The choice becomes
 * the default tuning of the current device.  Results never depend on it. */
mlmc_ap_status mlmc_ap_autotune(const mlmc_ap_problem* p, double rmse_tol,
                                const char* cache_path, mlmc_ap_tuning* out_host, void* stream);

/* Sets the default tuning of the current device (what estimates without
 * an explicit tuning, mlmc_ap_simulate_level and new servers use); zero
 * fields keep the current value.  EINVAL for an invalid shape. */
mlmc_ap_status mlmc_ap_set_tuning(const mlmc_ap_tuning* tuning_host);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of MLMC requests.                         */
/* ---------------------------------------------------------------------- */
typedef struct mlmc_ap_server mlmc_ap_server;

typedef struct mlmc_ap_server_config {
    uint64_t hbm_budget_bytes;     /* device memory the server may use for request
                                      state and tile partials (0 = 1 GiB) */
    uint64_t max_samples_per_tick; /* per request and level per tick (0 = 2^24) */
    int32_t max_active;            /* admitted requests at once (0 = 256) */
    int32_t reserved;
    mlmc_ap_options options;       /* n_warmup, max_iter, tuning (batched is implied;
                                      level_select and L_max must be 0: the server
                                      runs every level 0..L) */
} mlmc_ap_server_config;

typedef struct mlmc_ap_server_stats {
    uint64_t submitted, admitted, completed, cancelled, rejected;
    uint64_t ticks, particle_steps;
    uint64_t bytes_reserved, bytes_peak;
    int32_t active, queued;
    double busy_seconds;          /* host time spent inside ticks */
} mlmc_ap_server_stats;

mlmc_ap_status mlmc_ap_server_create(const mlmc_ap_server_config* cfg, mlmc_ap_server** out);
mlmc_ap_status mlmc_ap_server_destroy(mlmc_ap_server* srv);
/* Queues a request (QOI_X2; either scheme, FP32 or FP64 state); it is
 * admitted at a later tick once its device memory (per-level state and
 * per-tick tile partials) fits the budget.  EBUSY if it can never fit; EINVAL
 * for an invalid problem or tolerance, or a histogram QoI. */
mlmc_ap_status mlmc_ap_server_submit(mlmc_ap_server* srv, const mlmc_ap_problem* p,
                                     double rmse_tol, uint64_t* ticket_out);
/* One tick: admit queued requests that fit, run one top-up iteration of every
 * active request in one persistent launch per particle kernel in use (FP32
 * splitting, FP64 splitting, KD; launches issued directly), update their
 * level state and complete those whose statistical constraint holds.
 * n_completed_out (nullable) receives the number completed in this tick. */
mlmc_ap_status mlmc_ap_server_step(mlmc_ap_server* srv, int32_t* n_completed_out);
/* OK with the result, EAGAIN while pending, ECANCELLED, ENOTFOUND.  A
 * finished result stays available until polled once. */
mlmc_ap_status mlmc_ap_server_poll(mlmc_ap_server* srv, uint64_t ticket, mlmc_ap_result* out_host);
mlmc_ap_status mlmc_ap_server_cancel(mlmc_ap_server* srv, uint64_t ticket);
mlmc_ap_status mlmc_ap_server_get_stats(const mlmc_ap_server* srv, mlmc_ap_server_stats* out);
/* Replays an arrival trace in real time: request i is submitted when
 * arrival_s[i] seconds (non-decreasing, from the call's start) have passed,
 * ticks run back to back while work exists, and latency_s_out[i] receives
 * completion minus arrival time.  results_out (nullable) gets every result. */
mlmc_ap_status mlmc_ap_server_run_trace(mlmc_ap_server* srv, int32_t n, const double* arrival_s,
                                        const mlmc_ap_problem* p, const double* rmse_tol,
                                        mlmc_ap_result* results_out, double* latency_s_out);

/* Consistency harness of Section 5.1: the aggregated coarse numbers of KD
 * pairs (scheme KD), for checking that they follow the laws the coarse path
 * needs (eq. null_hypothesis: nu~ ~ N(0,1), E~ ~ Exp(1), chi~ ~ N(0,1)).  The
 * fine step is dt0 / M^level and the coarse step dt0 / M^coarse_level; T/dt0
 * need not be an integer here, so the coarse step may exceed T (as in the
 * paper's table).  For pair i = sample - sample_begin:
 *   rows_dev[((i * max_rows) + k) * 4 + j], k < min(counts, max_rows): coarse KD
 *     step k's chi~ (eq. chi-update), nu~ (eq. nu-update), E~ (eq.
 *     epsilon-update) and the number of fine KD steps aggregated into it;
 *   counts_dev[i]: the pair's coarse KD steps (rows beyond max_rows are not
 *     written).
 * Both buffers are caller-owned device memory (n_samples * max_rows * 4
 * doubles, n_samples uint32).  The call synchronises `stream`. */
mlmc_ap_status mlmc_ap_kd_coarse_numbers(const mlmc_ap_problem* p, int32_t level,
                                         int32_t coarse_level, uint64_t sample_begin,
                                         uint64_t n_samples, uint32_t max_rows, double* rows_dev,
                                         uint32_t* counts_dev, void* stream);

/* ---------------------------------------------------------------------- */
/* Validation entry points (bit-exact checks of the random number path).  */
/* ---------------------------------------------------------------------- */
/* Philox4x32-10 words for counters (n, sample, tag, stream_id), key = seed:
 * out_dev[((s - sample_begin) * n_steps + n) * 4 + j] for n < n_steps. */
mlmc_ap_status mlmc_ap_philox_words(uint64_t seed, uint32_t stream_id, uint32_t tag,
                                    uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps,
                                    uint32_t* out_dev, void* stream);
/* Uniforms and Box-Muller normals of the same grid as computed by the FP32
 * (fp64 = 0, float out_dev) or FP64 (fp64 = 1, double out_dev) particle
 * path: out[((s - sample_begin) * n_steps + n) * 4 + {0,1,2,3}] =
 * (u1, u2, xi, g). */
mlmc_ap_status mlmc_ap_rng_normals(uint64_t seed, uint32_t stream_id, uint32_t tag,
                                   uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps,
                                   int32_t fp64, void* out_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MLMC_AP_H */
