/*
 * FP64 CPU oracle for the multilevel asymptotic-preserving Monte Carlo
 * particle method (Mortier, Robbe, Baelmans, Samaey, "Multilevel
 * asymptotic-preserving Monte Carlo for kinetic-diffusive particle
 * simulations of the Boltzmann-BGK equation").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * path (the HIP library) never calls it and shares no code with it.
 *
 * It is written to be slow and obviously correct: one trajectory at a time,
 * every quantity in double precision, each step in the order the method
 * states it.  Parity status of each function is given in its comment;
 * every function here is pinned by the CPU tests (Philox known-answer
 * vectors, closed-form moments, brute-force enumeration, distribution
 * tests of the coarse random numbers).
 *
 * The particle scheme (asymptotic-preserving splitting, the scheme the paper
 * cites from Dimarco et al. in its introduction) for the diffusively scaled
 * BGK equation  df/dt + (v/eps) df/dx = (M rho - f)/eps^2  with an
 * equilibrium M of unit variance, at fixed time step dt:
 *     h = dt*eps/(eps^2+dt)              drift multiplier of the velocity
 *     s = sqrt(2*dt*dt/(eps^2+dt))       standard deviation of the kick
 *     p = dt/(eps^2+dt)                  collision probability
 *   transport-diffusion:  x <- x + h*v + s*xi,  xi ~ N(0,1)
 *   collision:            with probability p, v <- fresh draw from M
 *
 * Levels: dt_l = dt0 / M^l, n_l = T/dt_l steps (Section 4.1 uses T/2^l; the
 * refinement factor M generalises the factor 2 as in Section 5.1).
 *
 * Fine/coarse correlation (Section 3): every coarse random number is built
 * from fine random numbers mapped by the time at which they act (Section
 * 3.1): coarse step K uses the fine steps K*M .. K*M+M-1.
 *   - coarse kick: normalised weighted sum of the fine kick normals and of the
 *     fine velocity normals that the coarse path does not reuse
 *     (eq. chi-update, weights after eqs. for alpha and beta);
 *   - coarse velocity: the fine velocity normal drawn last in the block
 *     (eq. nu-update);
 *   - coarse collision: decided by the fine decision words of the block:
 *     it happens iff the smallest of them is below a threshold under the
 *     fine one, so the fine words that caused fine collisions are reused
 *     (the uniform analogue of reusing the fine exponential number in eq.
 *     epsilon-update), and a coarse collision always comes with a fine one.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC 2011), key = seed.  The random
 * numbers of one trajectory are the word stream W_0, W_1, ... of its blocks
 * b = 0, 1, 2, ... with counter (b, sample, level tag, stream): W_k is word
 * k mod 4 of block k/4.  The initial condition takes W_0, W_1 (a Box-Muller
 * pair; for the density 1 + cos 2 pi x also W_2, and W_3..W_5 are skipped),
 * then every fine step takes the next three words: the collision decision
 * word and a Box-Muller pair.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10, written from the published definition.               */
/* ------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;   /* Weyl key schedule */
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform on (0,1): the odd multiple (2*(w>>9)+1) * 2^-24. */
double oracle_uniform(uint32_t w)
{
    return (2.0 * (double)(w >> 9) + 1.0) * 0x1p-24;
}

/* Box-Muller pair from two words: cosine branch and sine branch.  The
 * first word gives the radius, the second the angle. */
static void box_muller(uint32_t wa, uint32_t wb, double *c, double *s)
{
    double u1 = oracle_uniform(wa);
    double u2 = oracle_uniform(wb);
    double r = sqrt(-2.0 * log(u1));
    double theta = 2.0 * M_PI * u2;
    *c = r * cos(theta);
    *s = r * sin(theta);
}

/* Inverse CDF of the density 1 + cos(2 pi x) on [0,1]:
 * F(x) = x + sin(2 pi x)/(2 pi), solved by plain bisection. */
double oracle_cosine_icdf(double u)
{
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double F = mid + sin(2.0 * M_PI * mid) / (2.0 * M_PI);
        if (F < u) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------ */
/* Level constants.                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    double dt, h, s, p;
    uint64_t n_steps;
    uint64_t thr;        /* collide iff word < thr; thr = round(p * 2^32) */
} level_consts;

static level_consts make_level(double eps, double T, double dt0, int M, int l)
{
    level_consts c;
    c.dt = dt0 / pow((double)M, (double)l);
    double denom = eps * eps + c.dt;
    c.h = c.dt * eps / denom;
    c.s = sqrt(2.0 * c.dt * c.dt / denom);
    c.p = c.dt / denom;
    c.n_steps = (uint64_t)llround(T / dt0) * (uint64_t)llround(pow((double)M, (double)l));
    c.thr = (uint64_t)llround(c.p * 4294967296.0);
    return c;
}

/* Threshold of the coarse collision decision: the coarse path of level l
 * collides in coarse step K iff the smallest fine decision word of the fine
 * steps K*M .. K*M+M-1 is below thr_c2.  The M words are independent and
 * uniform on [0, 2^32), so
 *   P(coarse collision) = 1 - (1 - thr_c2/2^32)^M,
 * and thr_c2 = 2^32 (1 - (1 - p_c)^(1/M)) makes it the coarse level's own
 * collision probability p_c = thr_c/2^32.  Since (1-p_f)^M <= 1-p_c,
 * thr_c2 <= thr_f: a word below thr_c2 is a fine collision, so a coarse
 * collision always has a fine velocity draw in its block to take over. */
uint64_t oracle_coarse_threshold(uint64_t thr_f, uint64_t thr_c, int M)
{
    double pc = (double)thr_c / 4294967296.0;
    double t = 4294967296.0 * -expm1(log1p(-pc) / (double)M);
    uint64_t r = (uint64_t)llround(t);
    if (r > thr_f) r = thr_f;
    return r;
}

void oracle_level_consts(double eps, double T, double dt0, int M, int l,
                         double out_dhsp[4], uint64_t out_n_thr[2])
{
    level_consts c = make_level(eps, T, dt0, M, l);
    out_dhsp[0] = c.dt; out_dhsp[1] = c.h; out_dhsp[2] = c.s; out_dhsp[3] = c.p;
    out_n_thr[0] = c.n_steps; out_n_thr[1] = c.thr;
}

/* ------------------------------------------------------------------ */
/* The word stream of one trajectory.                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t key[2];
    uint32_t sample, tag, stream;
    uint32_t block;      /* next block index */
    uint32_t buf[4];
    int pos;             /* next word of buf; 4 = empty */
} words_t;

static void words_init(words_t *s, const uint32_t key[2], uint32_t sample, uint32_t tag,
                       uint32_t stream)
{
    s->key[0] = key[0]; s->key[1] = key[1];
    s->sample = sample; s->tag = tag; s->stream = stream;
    s->block = 0; s->pos = 4;
}

static uint32_t next_word(words_t *s)
{
    if (s->pos == 4) {
        uint32_t ctr[4] = {s->block, s->sample, s->tag, s->stream};
        oracle_philox4x32_10(ctr, s->key, s->buf);
        s->block++;
        s->pos = 0;
    }
    return s->buf[s->pos++];
}

/* +1 or -1 from the top bit of a word: for the angle word of a Box-Muller
 * pair this is the sign of its sine branch, and it is independent of the
 * cosine branch. */
static double sign_of(uint32_t w)
{
    return (w >> 31) ? -1.0 : 1.0;
}

/* ------------------------------------------------------------------ */
/* One fine/coarse pair (or one single-level trajectory).              */
/* ------------------------------------------------------------------ */
enum { X0_DELTA = 0, X0_NORMAL = 1, X0_COSINE = 2 };
enum { EQ_TWO_POINT = 0, EQ_MAXWELLIAN = 1 };
enum { COUPLING_KICK_SUM = 0, COUPLING_AGGREGATE = 1 };

typedef struct {
    double eps, T, dt0;
    int M, level, single;
    int coarse_level;    /* level of the coarse path of a pair (level - 1 unless set) */
    int x0_kind; double x0_a, x0_b;
    int eq_kind, coupling;
    uint32_t key[2];
    uint32_t stream;
    /* KD scheme in a homogeneous background: collision rate and Maxwellian
     * standard deviation (the diffusive scaling: 1/eps^2 and 1/eps) */
    double R, sigma;
    int pair_tag;        /* single paths under the pair's counter tag (tests) */
} problem_t;

/* Optional per-step record for tiny golden traces. */
typedef struct {
    double *rows;      /* n_rows x 16 doubles, or NULL */
    uint64_t cap, used;
} trace_t;

static void trace_row(trace_t *tr, const double v[16])
{
    if (!tr || !tr->rows || tr->used >= tr->cap) return;
    memcpy(tr->rows + 16 * tr->used, v, 16 * sizeof(double));
    tr->used++;
}

/* Simulates sample `sample` and returns x_f(T), x_c(T), fine and coarse
 * collision counts.  Level 0 (or single mode) has no coarse path. */
static void simulate_one(const problem_t *P, uint64_t sample,
                         double *xf_out, double *xc_out,
                         uint32_t *cf_out, uint32_t *cc_out, trace_t *tr)
{
    const int l = P->level;
    const int coarse = (!P->single && l >= 1);
    const uint32_t tag = (uint32_t)l + (P->single ? 64u : 0u);
    /* fine steps per coarse step: M^(l - coarse level) (M for adjacent levels) */
    const int Mb = coarse ? (int)llround(pow((double)P->M, (double)(l - P->coarse_level))) : 1;
    level_consts F = make_level(P->eps, P->T, P->dt0, P->M, l);
    level_consts C = coarse ? make_level(P->eps, P->T, P->dt0, P->M, P->coarse_level) : F;
    uint64_t thr_c2 = coarse ? oracle_coarse_threshold(F.thr, C.thr, Mb) : 0;

    words_t ws;
    words_init(&ws, P->key, (uint32_t)sample, tag, P->stream);

    /* Initial condition (shared by the fine and the coarse path). */
    uint32_t ia = next_word(&ws), ib = next_word(&ws);
    double nc, ns;
    box_muller(ia, ib, &nc, &ns);
    double x0;
    if (P->x0_kind == X0_DELTA) x0 = P->x0_a;
    else if (P->x0_kind == X0_NORMAL) x0 = P->x0_a + P->x0_b * nc;
    else {
        x0 = oracle_cosine_icdf(oracle_uniform(next_word(&ws)));
        for (int k = 0; k < 3; ++k) (void)next_word(&ws);   /* W_3..W_5 unused */
    }
    double v0 = (P->eq_kind == EQ_MAXWELLIAN) ? ns : sign_of(ib);

    double xf = x0, vf = v0, xc = x0, vc = v0;
    uint32_t cf = 0, cc = 0;

    /* Per-block coarse bookkeeping. */
    double sum_xi = 0.0;          /* sum of the fine kick normals */
    double vel_num = 0.0;         /* sum of n_j * nu_j over superseded draws */
    double vel_den = 0.0;         /* sum of n_j^2 */
    int have_draw = 0;            /* a fine velocity was drawn in this block */
    double last_nu = 0.0;         /* normal of the latest in-block draw */
    double last_uses = 0.0;       /* transport uses of that draw so far */
    uint32_t min_word = 0xFFFFFFFFu; /* smallest fine decision word of the block */

    for (uint64_t n = 0; n < F.n_steps; ++n) {
        uint32_t wd = next_word(&ws);      /* collision decision */
        uint32_t wa = next_word(&ws);      /* Box-Muller radius */
        uint32_t wb = next_word(&ws);      /* Box-Muller angle */
        double xi, g;
        box_muller(wa, wb, &xi, &g);
        double v_new = (P->eq_kind == EQ_MAXWELLIAN) ? g : sign_of(wb);

        /* transport-diffusion with the pre-collision velocity */
        xf = xf + F.h * vf + F.s * xi;
        if (have_draw) last_uses += 1.0;
        sum_xi += xi;

        /* collision */
        int hit = ((uint64_t)wd < F.thr);
        if (wd < min_word) min_word = wd;
        if (hit) {
            vf = v_new;
            cf++;
            if (have_draw) {          /* previous in-block draw is superseded */
                vel_num += last_uses * last_nu;
                vel_den += last_uses * last_uses;
            }
            have_draw = 1; last_nu = v_new; last_uses = 0.0;
        }

        double row[16] = {(double)n, (double)wd, (double)wa, (double)wb,
                          (double)(ws.block * 4u - (uint32_t)(4 - ws.pos)),
                          oracle_uniform(wa), oracle_uniform(wb), xi, g, (double)hit,
                          xf, vf, 0, 0, 0, 0};

        if (coarse && (n % (uint64_t)Mb) == (uint64_t)(Mb - 1)) {
            int chit = ((uint64_t)min_word < thr_c2);
            double kick;
            if (P->coupling == COUPLING_KICK_SUM) {
                kick = sum_xi / sqrt((double)Mb);
            } else {
                /* the last in-block draw becomes the coarse velocity when the
                 * coarse path collides; otherwise it joins the kick */
                double num = vel_num, den = vel_den;
                if (have_draw && !chit) {
                    num += last_uses * last_nu;
                    den += last_uses * last_uses;
                }
                kick = (F.s * sum_xi + F.h * num) /
                       sqrt((double)Mb * F.s * F.s + F.h * F.h * den);
            }
            xc = xc + C.h * vc + C.s * kick;
            if (chit) { vc = vf; cc++; }
            row[12] = kick; row[13] = (double)chit; row[14] = xc; row[15] = vc;
            sum_xi = 0.0; vel_num = 0.0; vel_den = 0.0;
            have_draw = 0; last_nu = 0.0; last_uses = 0.0;
            min_word = 0xFFFFFFFFu;
        }
        trace_row(tr, row);
    }
    if (!coarse) { xc = 0.0; cc = 0; }
    *xf_out = xf; *xc_out = xc; *cf_out = cf; *cc_out = cc;
}

static problem_t make_problem(double eps, double T, double dt0, int M, int level,
                              int single, int x0_kind, double x0_a, double x0_b,
                              int eq_kind, int coupling, uint64_t seed, uint32_t stream)
{
    problem_t P;
    P.eps = eps; P.T = T; P.dt0 = dt0; P.M = M; P.level = level; P.single = single;
    P.coarse_level = level - 1;
    P.x0_kind = x0_kind; P.x0_a = x0_a; P.x0_b = x0_b;
    P.eq_kind = eq_kind; P.coupling = coupling;
    P.key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    P.key[1] = (uint32_t)(seed >> 32);
    P.stream = stream;
    P.R = eps > 0.0 ? 1.0 / (eps * eps) : 0.0;
    P.sigma = eps > 0.0 ? 1.0 / eps : 0.0;
    P.pair_tag = 0;
    return P;
}

/* Simulates the listed sample indices (idx != NULL) or the contiguous range
 * [sample_begin, sample_begin + n) (idx == NULL).  Outputs are indexed by
 * position in the list.  Each sample is independent, so the threads only
 * split the list; results do not depend on the thread count. */
int oracle_simulate(double eps, double T, double dt0, int M, int level, int single,
                    int x0_kind, double x0_a, double x0_b, int eq_kind, int coupling,
                    uint64_t seed, uint32_t stream,
                    uint64_t sample_begin, const uint64_t *idx, uint64_t n,
                    double *xf, double *xc, uint32_t *cf, uint32_t *cc, int nthreads)
{
    problem_t P = make_problem(eps, T, dt0, M, level, single, x0_kind, x0_a, x0_b,
                               eq_kind, coupling, seed, stream);
    (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t s = idx ? idx[i] : sample_begin + (uint64_t)i;
        simulate_one(&P, s, &xf[i], &xc[i], &cf[i], &cc[i], NULL);
    }
    return 0;
}

/* Per-step trace of one sample: 16 doubles per fine step
 * (n, decision word, radius word, angle word, words consumed so far, u1, u2,
 * xi, g, hit, x_f, v_f, kick, coarse_hit, x_c, v_c);
 * the last four are filled on the last fine step of each block. */
uint64_t oracle_trace(double eps, double T, double dt0, int M, int level, int single,
                      int x0_kind, double x0_a, double x0_b, int eq_kind, int coupling,
                      uint64_t seed, uint32_t stream, uint64_t sample,
                      double *rows, uint64_t cap, double out_final[2])
{
    problem_t P = make_problem(eps, T, dt0, M, level, single, x0_kind, x0_a, x0_b,
                               eq_kind, coupling, seed, stream);
    trace_t tr = {rows, cap, 0};
    double xf, xc; uint32_t cf, cc;
    simulate_one(&P, sample, &xf, &xc, &cf, &cc, &tr);
    out_final[0] = xf; out_final[1] = xc;
    return tr.used;
}

/* Raw Philox words for a grid of (step, sample) counters:
 * out[((s - sample_begin) * n_steps + n) * 4 + j] for steps n < n_steps. */
void oracle_words(uint64_t seed, uint32_t stream, uint32_t tag,
                  uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps,
                  uint32_t *out)
{
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    for (uint64_t i = 0; i < n_samples; ++i) {
        for (uint32_t n = 0; n < n_steps; ++n) {
            uint32_t ctr[4] = {n, (uint32_t)(sample_begin + i), tag, stream};
            oracle_philox4x32_10(ctr, key, out + (i * n_steps + n) * 4);
        }
    }
}

/* ================================================================== */
/* Kinetic-diffusion (KD) scheme, homogeneous background              */
/* ================================================================== */
/*
 * The paper's own simulation scheme (Section 2, Algorithm "KD algorithm")
 * and its correlated fine/coarse form (Section 3, Algorithm "Correlated KD
 * algorithm"), in the diffusive scaling of the BGK equation above: constant
 * collision rate R = 1/eps^2, post-collision velocities drawn from the
 * Maxwellian with mean mu = 0 and standard deviation sigma = 1/eps.
 *
 * A KD step of a path with time step dt starts on the time grid at t with
 * velocity v and a pending collision at c = t + tau (tau = E/R, E ~ Exp(1)).
 * If c < T: the path moves kinetically to c, then diffusively to the end
 * of the grid step that contains c (length theta), with the advection a
 * (eq. advection) and diffusion d (eq. diffusion) conditioned on the next
 * velocity, and a new flight is drawn (eq. position-update, eq.
 * time-update).  Once the pending collision is at or after T the path
 * moves kinetically to T.
 *
 * Random numbers of one trajectory: Philox block 0 holds the initial
 * condition (W0, W1: Box-Muller pair, cosine branch -> x0 for the normal
 * law, sine branch -> nu_0; W2 -> E_0 = -log u; W3 -> u of the cosine
 * law); block k+1 holds the numbers of KD step k (W0, W1: Box-Muller pair,
 * cosine branch -> nu_{k+1}, sine branch -> chi_k; W2 -> E_{k+1}).
 * Counter (block, sample, level tag, stream) as for the splitting scheme.
 *
 * Correlated pair (level l >= 1): the coarse path (step dt_{l-1} = M dt_l)
 * takes its numbers from the fine path (Section 3.1 mapping by the time at
 * which they act; Section 3.2 aggregation):
 *   - its flight k uses the fine flight kappa_k: the same velocity number
 *     (eq. nu-update), and the exponential number reduced by the part of
 *     the flight the fine path has already used (eq. epsilon-update); in a
 *     homogeneous background the coarse collision therefore falls at the
 *     same time as the fine one;
 *   - its diffusive phase k aggregates, by eq. chi-update, the fine
 *     diffusive numbers chi_m and the fine velocity numbers nu_m of the
 *     fine phases that follow flight kappa_k up to the first fine flight
 *     whose collision lies after the end of the coarse grid step; the
 *     weights are alpha_m = sigma tau'_m and beta_m = the unconditioned
 *     diffusive standard deviation over theta'_m (eq. weights-beta), with
 *     the expected time zeta_m = (1 - e^{-R theta_m})/R moved from each
 *     diffusive phase to the next flight.
 *
 * PARITY: pinned by the CPU tests (the second moment of x(T), which the KD
 * construction keeps exact at every dt; the conditional moments of a
 * diffusive phase against a brute-force velocity-jump simulation; the laws
 * of the aggregated coarse numbers; the coarse path against the fine path
 * of the level below).
 */

/* Stable evaluations of three functions of y = R theta >= 0 that lose
 * all their digits to cancellation when written with exp for small y
 * (exact up to rounding; the series are their Taylor expansions):
 *   kd_h(y) = e^{-y} - 1 + y                  = sum_{m>=2} (-y)^m/m!
 *   kd_f(y) = 2(e^{-y} - 1) + y(e^{-y} + 1)   = sum_{m>=3} (-1)^{m+1} (m-2) y^m/m!
 *   kd_g(y) = 1 - 2y e^{-y} - e^{-2y}         = sum_{m>=3} (-1)^{m+1} (2^m - 2m) y^m/m!
 */
#define KD_SERIES_Y 0.05
#define KD_SERIES_TERMS 16

static double kd_h(double y)
{
    if (y >= KD_SERIES_Y) return expm1(-y) + y;
    double s = 0.0, term = 1.0;
    for (int m = 1; m <= KD_SERIES_TERMS; ++m) {
        term *= -y / (double)m;           /* (-y)^m / m! */
        if (m >= 2) s += term;
    }
    return s;
}

static double kd_f(double y)
{
    if (y >= KD_SERIES_Y) {
        double e = exp(-y);
        return 2.0 * (e - 1.0) + y * (e + 1.0);
    }
    double s = 0.0, pw = 1.0;
    for (int m = 1; m <= KD_SERIES_TERMS; ++m) {
        pw *= y / (double)m;              /* y^m / m! */
        if (m >= 3) s += ((m % 2) ? 1.0 : -1.0) * (double)(m - 2) * pw;
    }
    return s;
}

static double kd_g(double y)
{
    if (y >= KD_SERIES_Y) {
        double e = exp(-y);
        return 1.0 - 2.0 * y * e - e * e;
    }
    double s = 0.0, pw = 1.0;
    for (int m = 1; m <= KD_SERIES_TERMS; ++m) {
        pw *= y / (double)m;
        if (m >= 3) s += ((m % 2) ? 1.0 : -1.0) * (ldexp(1.0, m) - 2.0 * (double)m) * pw;
    }
    return s;
}

/* eq. advection and eq. diffusion (homogeneous background): advection a and
 * diffusion coefficient d of a diffusive phase of length theta that ends
 * with velocity vnext. */
void oracle_kd_coeffs(double theta, double R, double mu, double sigma, double vnext,
                      double out[2])
{
    double y = R * theta;
    double dv = vnext - mu;
    double a = mu * theta + dv * (-expm1(-y)) / R;
    double d2 = 2.0 * sigma * sigma / (R * R) * kd_f(y) + dv * dv / (R * R) * kd_g(y);
    out[0] = a;
    out[1] = sqrt(d2 > 0.0 ? d2 : 0.0);
}

/* Numbers of one KD step from its Philox block. */
static void kd_draws(const uint32_t w[4], double *nu_next, double *chi, double *E_next)
{
    box_muller(w[0], w[1], nu_next, chi);
    *E_next = -log(oracle_uniform(w[2]));
}

static void kd_block(const problem_t *P, uint32_t sample, uint32_t tag, uint32_t b,
                     uint32_t w[4])
{
    uint32_t ctr[4] = {b, sample, tag, P->stream};
    oracle_philox4x32_10(ctr, P->key, w);
}

/* Index of the grid step that contains time c: the step [q dt, (q+1) dt). */
static double kd_step_of(double c, double dt)
{
    return floor(c / dt);
}

/* Optional record of the coarse numbers of a pair, 4 doubles per coarse
 * step: (chi~, nu~, E~, number of fine KD steps aggregated), and of the fine
 * phases behind them, 16 doubles per fine KD step m of a pair:
 *   0 coarse step k the phase is aggregated into, 1 first phase of the
 *   window (m = kappa_k: no alpha term), 2 grid time t_m the flight starts
 *   from, 3 flight tau_m, 4 theta_m, 5 zeta_m, 6 theta'_m, 7 tau'_m (0 when
 *   first), 8 alpha_m (0 when first), 9 beta_m, 10 nu_m (velocity number of
 *   flight m), 11 chi_m, 12 a_m, 13 d_m, 14 nu_{m+1}, 15 x_f after phase m. */
typedef struct {
    double *rows;
    uint64_t cap, used;
    double *phases;
    uint64_t phase_cap, phase_used;
} kd_trace_t;

static void simulate_kd_one(const problem_t *P, uint64_t sample,
                            double *xf_out, double *xc_out,
                            uint32_t *cf_out, uint32_t *cc_out, kd_trace_t *tr)
{
    const int l = P->level;
    const int coarse = (!P->single && l >= 1);
    const uint32_t tag = (uint32_t)l + (P->single ? 64u : 0u);
    const uint32_t smp = (uint32_t)sample;
    const double R = P->R;                        /* collision rate */
    const double mu = 0.0;                        /* Maxwellian mean */
    const double sigma = P->sigma;                /* Maxwellian standard deviation */
    const double T = P->T;
    const double dtf = P->dt0 / pow((double)P->M, (double)l);
    const double dtc = coarse ? P->dt0 / pow((double)P->M, (double)P->coarse_level) : 0.0;
    const double Mb = coarse ? (double)llround(pow((double)P->M, (double)(l - P->coarse_level))) : 1.0;

    /* Initial condition, shared by both paths. */
    uint32_t w[4];
    kd_block(P, smp, tag, 0, w);
    double nc, ns;
    box_muller(w[0], w[1], &nc, &ns);
    double x0;
    if (P->x0_kind == X0_DELTA) x0 = P->x0_a;
    else if (P->x0_kind == X0_NORMAL) x0 = P->x0_a + nc * P->x0_b;
    else x0 = oracle_cosine_icdf(oracle_uniform(w[3]));
    double nu = ns;                               /* nu_0 */
    double E = -log(oracle_uniform(w[2]));        /* E_0 */

    /* Fine path: position, velocity, grid time, flight, pending collision. */
    double xf = x0, vf = mu + sigma * nu, tf = 0.0, tauf = E / R;
    double cfine = tf + tauf;
    uint32_t cf = 0, cc = 0, b = 1;

    if (!coarse) {
        /* Algorithm "KD algorithm". */
        while (cfine < T) {
            double nu_next, chi, E_next;
            kd_block(P, smp, tag, b++, w);
            kd_draws(w, &nu_next, &chi, &E_next);
            double t_next = (kd_step_of(cfine, dtf) + 1.0) * dtf;
            double theta = t_next - cfine;                /* eq. diffusive-time */
            double v_next = mu + sigma * nu_next;
            double ad[2];
            oracle_kd_coeffs(theta, R, mu, sigma, v_next, ad);
            xf = xf + vf * tauf + (ad[0] + ad[1] * chi);  /* eq. position-update */
            tf = t_next;                                  /* eq. time-update */
            tauf = E_next / R;
            cfine = tf + tauf;
            vf = v_next;
            cf++;
        }
        if (tf < T) xf = xf + vf * (T - tf);
        *xf_out = xf; *xc_out = 0.0; *cf_out = cf; *cc_out = 0;
        return;
    }

    /* Algorithm "Correlated KD algorithm".  The coarse path starts with the
     * fine path's first flight (same velocity number and exponential
     * number), so the same collision time. */
    double xc = x0, vc = vf, tc = 0.0, ccoarse = cfine;
    double nu_f = nu;   /* velocity number of the fine path's pending flight */
    while (ccoarse < T || cfine < T) {
        /* end of the coarse grid step containing the coarse collision, in
         * fine steps */
        const double end_c = kd_step_of(ccoarse, dtc) + 1.0;
        const double end_c_fine = end_c * Mb;
        double num = 0.0, den = 0.0, zeta_prev = 0.0;
        int first = 1;
        uint32_t used = 0;
        do {
            /* one fine KD step (phase m) */
            double nu_next, chi, E_next;
            kd_block(P, smp, tag, b++, w);
            kd_draws(w, &nu_next, &chi, &E_next);
            double t_next = (kd_step_of(cfine, dtf) + 1.0) * dtf;
            double theta = t_next - cfine;
            double v_next = mu + sigma * nu_next;
            double ad[2];
            oracle_kd_coeffs(theta, R, mu, sigma, v_next, ad);
            xf = xf + vf * tauf + (ad[0] + ad[1] * chi);

            /* aggregation weights of phase m (Section 3.2) */
            double y = R * theta;
            double zeta = -expm1(-y) / R;                 /* expected time of nu_{m+1} */
            double theta_p = kd_h(y) / R;                 /* theta'_m = theta_m - zeta_m */
            double beta = sqrt(2.0 * sigma * sigma / (R * R) * kd_h(R * theta_p));
            double alpha = 0.0;
            if (!first) {
                alpha = (tauf + zeta_prev) * sigma;          /* sigma tau'_m */
                num += alpha * nu_f;
                den += alpha * alpha;
            }
            num += beta * chi;
            den += beta * beta;
            if (tr && tr->phases && tr->phase_used < tr->phase_cap) {
                double *r = tr->phases + 16 * tr->phase_used++;
                r[0] = (double)cc; r[1] = (double)first; r[2] = tf; r[3] = tauf;
                r[4] = theta; r[5] = zeta; r[6] = theta_p;
                r[7] = first ? 0.0 : tauf + zeta_prev; r[8] = alpha; r[9] = beta;
                r[10] = nu_f; r[11] = chi; r[12] = ad[0]; r[13] = ad[1];
                r[14] = nu_next; r[15] = xf;
            }
            zeta_prev = zeta;
            first = 0;
            used++;

            tf = t_next;
            tauf = E_next / R;
            cfine = tf + tauf;
            vf = v_next;
            nu_f = nu_next;
            cf++;
        } while (!(kd_step_of(cfine, dtf) + 1.0 > end_c_fine));

        if (ccoarse < T) {
            double nu_c = nu_f;                               /* eq. nu-update */
            double chi_c = den > 0.0 ? num / sqrt(den) : 0.0; /* eq. chi-update */
            double t_next = end_c * dtc;
            double theta = t_next - ccoarse;
            double v_next = mu + sigma * nu_c;
            double ad[2];
            oracle_kd_coeffs(theta, R, mu, sigma, v_next, ad);
            xc = xc + vc * (ccoarse - tc) + (ad[0] + ad[1] * chi_c);
            tc = t_next;
            /* eq. epsilon-update: E~ = E_kappa - R (t_c - t_f,kappa), so the
             * coarse collision is the fine one */
            double E_c = R * (cfine - tc);
            ccoarse = cfine;
            vc = v_next;
            cc++;
            if (tr && tr->rows && tr->used < tr->cap) {
                double *r = tr->rows + 4 * tr->used++;
                r[0] = chi_c; r[1] = nu_c; r[2] = E_c; r[3] = (double)used;
            }
        }
    }
    if (tf < T) xf = xf + vf * (T - tf);
    if (tc < T) xc = xc + vc * (T - tc);
    *xf_out = xf; *xc_out = xc; *cf_out = cf; *cc_out = cc;
}

/* As oracle_simulate, for the KD scheme. */
int oracle_simulate_kd(double eps, double T, double dt0, int M, int level, int single,
                       int x0_kind, double x0_a, double x0_b, int eq_kind, int coupling,
                       uint64_t seed, uint32_t stream,
                       uint64_t sample_begin, const uint64_t *idx, uint64_t n,
                       double *xf, double *xc, uint32_t *cf, uint32_t *cc, int nthreads)
{
    problem_t P = make_problem(eps, T, dt0, M, level, single, x0_kind, x0_a, x0_b,
                               eq_kind, coupling, seed, stream);
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t s = idx ? idx[i] : sample_begin + (uint64_t)i;
        simulate_kd_one(&P, s, &xf[i], &xc[i], &cf[i], &cc[i], NULL);
    }
    return 0;
}

/* Coarse numbers of one pair (rows of 4 doubles, see kd_trace_t); returns
 * the number of rows written.  out_final = (x_f, x_c). */
uint64_t oracle_kd_coarse_numbers(double eps, double T, double dt0, int M, int level,
                                  int coarse_level, int x0_kind, double x0_a, double x0_b,
                                  uint64_t seed, uint32_t stream, uint64_t sample,
                                  double *rows, uint64_t cap, double out_final[2])
{
    problem_t P = make_problem(eps, T, dt0, M, level, 0, x0_kind, x0_a, x0_b,
                               EQ_MAXWELLIAN, 0, seed, stream);
    if (coarse_level >= 0 && coarse_level < level) P.coarse_level = coarse_level;
    kd_trace_t tr = {rows, cap, 0, NULL, 0, 0};
    double xf, xc; uint32_t cf, cc;
    simulate_kd_one(&P, sample, &xf, &xc, &cf, &cc, &tr);
    out_final[0] = xf; out_final[1] = xc;
    return tr.used;
}

/* Fine phases of one pair (rows of 16 doubles, see kd_trace_t) and its
 * coarse numbers (rows of 4); *n_coarse_out receives the coarse rows
 * written; returns the phase rows written.  out_final = (x_f, x_c). */
uint64_t oracle_kd_phases(double eps, double T, double dt0, int M, int level,
                          int coarse_level, int x0_kind, double x0_a, double x0_b,
                          uint64_t seed, uint32_t stream, uint64_t sample,
                          double *phases, uint64_t phase_cap, double *rows, uint64_t cap,
                          uint64_t *n_coarse_out, double out_final[2])
{
    problem_t P = make_problem(eps, T, dt0, M, level, 0, x0_kind, x0_a, x0_b,
                               EQ_MAXWELLIAN, 0, seed, stream);
    if (coarse_level >= 0 && coarse_level < level) P.coarse_level = coarse_level;
    kd_trace_t tr = {rows, cap, 0, phases, phase_cap, 0};
    double xf, xc; uint32_t cf, cc;
    simulate_kd_one(&P, sample, &xf, &xc, &cf, &cc, &tr);
    out_final[0] = xf; out_final[1] = xc;
    *n_coarse_out = tr.used;
    return tr.phase_used;
}

/* As oracle_simulate / oracle_simulate_kd for a pair whose coarse path is at
 * level coarse_level < level (the level pairs of a non-contiguous hierarchy,
 * Section 4.2): one coarse step per M^(level - coarse_level) fine steps. */
int oracle_simulate_pair(int kd, double eps, double T, double dt0, int M, int level,
                         int coarse_level, int x0_kind, double x0_a, double x0_b, int eq_kind,
                         int coupling, uint64_t seed, uint32_t stream,
                         uint64_t sample_begin, const uint64_t *idx, uint64_t n,
                         double *xf, double *xc, uint32_t *cf, uint32_t *cc, int nthreads)
{
    problem_t P = make_problem(eps, T, dt0, M, level, 0, x0_kind, x0_a, x0_b,
                               eq_kind, coupling, seed, stream);
    if (coarse_level < 0 || coarse_level >= level) return -1;
    P.coarse_level = coarse_level;
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t s = idx ? idx[i] : sample_begin + (uint64_t)i;
        if (kd) simulate_kd_one(&P, s, &xf[i], &xc[i], &cf[i], &cc[i], NULL);
        else simulate_one(&P, s, &xf[i], &xc[i], &cf[i], &cc[i], NULL);
    }
    return 0;
}


/* ================================================================== */
/* Kinetic-diffusion scheme in the backgrounds of Section 5            */
/* ================================================================== */
/*
 * The test case of the paper's Section 5: post-collision Maxwellian with
 * mu = 0 and sigma = 1, and a collision rate that is piecewise linear with a
 * kink at x = 1,
 *   B1 (symmetric):  R(x) = b (a |x - 1| + 1),
 *   B2 (asymmetric): R(x) = b for x <= 1, b (a (x - 1) + 1) for x > 1,
 * (a = 0: the homogeneous case R = b).
 *
 * Flight (eq. intinv): the flight time tau of a particle at x with velocity
 * v and exponential number E solves  int_0^tau R(x + v s) ds = E.  The
 * integral is exact by the trapezoid rule on each linear piece of R along the
 * flight; the root is found by bisection (R >= b, so tau <= E/b).
 *
 * Diffusive phase: eqs. advection and diffusion with the collision rate taken
 * where the phase starts, at the collision point.  READING: the corrected
 * coefficients a^hetero, d^hetero that the paper uses are not given in it
 * (they differ by evaluating the Maxwellian at a midpoint, which changes
 * nothing here since mu and sigma are constant, and by an extra advection
 * term for a strongly varying R); the local-rate form is exact for a = 0 and
 * tends to the kinetic process as dt -> 0.
 *
 * Correlated pair (Algorithm "Correlated KD algorithm", literally): the fine
 * path steps until its pending collision lies in a fine step that ends after
 * the coarse step holding the coarse collision (at least one fine step per
 * coarse step); the coarse step then takes nu~ of the pending fine flight
 * kappa (eq. nu-update), chi~ from eq. chi-update with the weights of
 * Section 3.2 (rate of each phase = its local rate), and for its next flight
 * E~ = E_kappa - int_0^{t_c - t_kappa} R(x_kappa + v_kappa s) ds (eq.
 * epsilon-update, the part of the fine flight before the coarse time), from
 * which it solves eq. intinv from its own position.  Fine KD steps taken
 * from a state whose pending collision is at or after T are used for the
 * aggregation only: the fine path ends at the first such state and flies
 * kinetically to T ("remove fine steps beyond T").
 *
 * Random numbers: as for the homogeneous KD scheme (block 0 initial
 * condition, block k+1 KD step k).
 *
 * PARITY: pinned by the CPU tests (flight times against a brute-force
 * thinning simulation of the inhomogeneous Poisson process of collisions;
 * a = 0 against the homogeneous KD path; E[x(T)] = 1 in the symmetric
 * background; the coarse path against the level below; the kinetic limit
 * against a brute-force velocity-jump simulation in the background).
 */
enum { BG_DIFFUSIVE = 0, BG_B1 = 1, BG_B2 = 2 };

typedef struct {
    int kind;
    double a, b;
} bg_t;

/* R(x) of a background */
static double bg_rate(const bg_t *g, double x)
{
    double u = x - 1.0;
    if (g->kind == BG_B1) return g->b * (g->a * fabs(u) + 1.0);
    if (u <= 0.0) return g->b;
    return g->b * (g->a * u + 1.0);
}

/* int_0^t R(x + v s) ds for t >= 0 (trapezoid rule on each linear piece of R
 * along the straight flight, exact); for t < 0 the integral over [t, 0],
 * negated. */
static double bg_rate_integral(const bg_t *g, double x, double v, double t)
{
    if (t < 0.0) return -bg_rate_integral(g, x + v * t, v, -t);
    if (t == 0.0) return 0.0;
    double xe = x + v * t;
    if ((x - 1.0) * (xe - 1.0) < 0.0) {            /* crosses the kink */
        double tk = (1.0 - x) / v;
        return 0.5 * tk * (bg_rate(g, x) + bg_rate(g, 1.0)) +
               0.5 * (t - tk) * (bg_rate(g, 1.0) + bg_rate(g, xe));
    }
    return 0.5 * t * (bg_rate(g, x) + bg_rate(g, xe));
}

/* Flight time of eq. intinv by bisection. */
static double bg_flight(const bg_t *g, double x, double v, double E)
{
    double lo = 0.0, hi = E / g->b;
    if (!(E > 0.0)) return 0.0;
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (bg_rate_integral(g, x, v, mid) < E) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double oracle_bg_rate(int kind, double a, double b, double x)
{
    bg_t g = {kind, a, b};
    return bg_rate(&g, x);
}

double oracle_bg_rate_integral(int kind, double a, double b, double x, double v, double t)
{
    bg_t g = {kind, a, b};
    return bg_rate_integral(&g, x, v, t);
}

double oracle_bg_flight(int kind, double a, double b, double x, double v, double E)
{
    bg_t g = {kind, a, b};
    return bg_flight(&g, x, v, E);
}

/* One path or one correlated pair in a background; the coarse numbers (and
 * fine phases) are recorded as for the homogeneous pair. */
static void simulate_kd_bg_one(const problem_t *P, const bg_t *g, uint64_t sample,
                               double *xf_out, double *xc_out,
                               uint32_t *cf_out, uint32_t *cc_out, kd_trace_t *tr)
{
    const int l = P->level;
    const int coarse = (!P->single && l >= 1);
    const uint32_t tag = (uint32_t)l + ((P->single && !P->pair_tag) ? 64u : 0u);
    const uint32_t smp = (uint32_t)sample;
    const double mu = 0.0, sigma = 1.0;
    const double T = P->T;
    const double dtf = P->dt0 / pow((double)P->M, (double)l);
    const double dtc = coarse ? P->dt0 / pow((double)P->M, (double)P->coarse_level) : 0.0;
    const double Mb = coarse ? (double)llround(pow((double)P->M, (double)(l - P->coarse_level))) : 1.0;
    /* a fine KD step advances at least one fine grid step; beyond T a pair's
     * fine path steps at most to the end of the last coarse step (a coarse
     * step may reach past T), one step per coarse step and one more */
    const double grid_end = coarse ? ceil(T / dtc - 1e-9) * dtc : T;
    const uint64_t guard = 2u * (uint64_t)llround(grid_end / dtf) + 4u;

    uint32_t w[4];
    kd_block(P, smp, tag, 0, w);
    double nc, ns;
    box_muller(w[0], w[1], &nc, &ns);
    double x0;
    if (P->x0_kind == X0_DELTA) x0 = P->x0_a;
    else if (P->x0_kind == X0_NORMAL) x0 = P->x0_a + nc * P->x0_b;
    else x0 = oracle_cosine_icdf(oracle_uniform(w[3]));
    double nu = ns;
    double E = -log(oracle_uniform(w[2]));

    /* fine path: position, velocity, grid time, flight, its exponential
     * number and pending collision */
    double xf = x0, vf = mu + sigma * nu, tf = 0.0;
    double Ef = E, tauf = bg_flight(g, xf, vf, Ef);
    double cfine = tf + tauf;
    uint32_t cf = 0, cc = 0, b = 1;
    uint64_t steps = 0;

    if (!coarse) {
        while (cfine < T && steps < guard) {
            double nu_next, chi, E_next;
            kd_block(P, smp, tag, b++, w);
            kd_draws(w, &nu_next, &chi, &E_next);
            double t_next = (kd_step_of(cfine, dtf) + 1.0) * dtf;
            double theta = t_next - cfine;                  /* eq. diffusive-time */
            double v_next = mu + sigma * nu_next;
            double Rloc = bg_rate(g, xf + vf * tauf);       /* rate at the collision */
            double ad[2];
            oracle_kd_coeffs(theta, Rloc, mu, sigma, v_next, ad);
            xf = xf + vf * tauf + (ad[0] + ad[1] * chi);    /* eq. position-update */
            tf = t_next;
            vf = v_next;
            Ef = E_next;
            tauf = bg_flight(g, xf, vf, Ef);
            cfine = tf + tauf;
            cf++;
            steps++;
        }
        if (tf < T) xf = xf + vf * (T - tf);
        *xf_out = xf; *xc_out = 0.0; *cf_out = cf; *cc_out = 0;
        return;
    }

    double xc = x0, vc = vf, tc = 0.0, tauc = tauf, ccoarse = tc + tauc;
    double nu_f = nu;
    int fine_done = 0;                 /* the fine path has ended */
    double xf_end = 0.0;
    uint64_t phases = 0;
    while ((ccoarse < T || cfine < T) && steps < guard) {
        const double end_c = kd_step_of(ccoarse, dtc) + 1.0;
        const double end_c_fine = end_c * Mb;
        double num = 0.0, den = 0.0, zeta_prev = 0.0;
        int first = 1;
        uint32_t used = 0;
        do {
            if (cfine >= T && !fine_done) {
                /* the first fine state whose pending collision is at or
                 * after T: the fine path flies from here to T */
                xf_end = tf < T ? xf + vf * (T - tf) : xf;
                fine_done = 1;
            }
            double nu_next, chi, E_next;
            kd_block(P, smp, tag, b++, w);
            kd_draws(w, &nu_next, &chi, &E_next);
            double t_next = (kd_step_of(cfine, dtf) + 1.0) * dtf;
            double theta = t_next - cfine;
            double v_next = mu + sigma * nu_next;
            double Rm = bg_rate(g, xf + vf * tauf);
            double ad[2];
            oracle_kd_coeffs(theta, Rm, mu, sigma, v_next, ad);
            xf = xf + vf * tauf + (ad[0] + ad[1] * chi);

            /* aggregation weights of phase m with its rate R_m (Section 3.2) */
            double y = Rm * theta;
            double zeta = -expm1(-y) / Rm;
            double theta_p = kd_h(y) / Rm;
            double beta = sqrt(2.0 * sigma * sigma / (Rm * Rm) * kd_h(Rm * theta_p));
            double alpha = 0.0;
            if (!first) {
                alpha = (tauf + zeta_prev) * sigma;
                num += alpha * nu_f;
                den += alpha * alpha;
            }
            num += beta * chi;
            den += beta * beta;
            if (tr && tr->phases && tr->phase_used < tr->phase_cap) {
                double *r = tr->phases + 16 * tr->phase_used++;
                r[0] = (double)cc; r[1] = (double)first; r[2] = tf; r[3] = tauf;
                r[4] = theta; r[5] = zeta; r[6] = theta_p;
                r[7] = first ? 0.0 : tauf + zeta_prev; r[8] = alpha; r[9] = beta;
                r[10] = nu_f; r[11] = chi; r[12] = ad[0]; r[13] = ad[1];
                r[14] = nu_next; r[15] = Rm;
            }
            zeta_prev = zeta;
            first = 0;
            used++;
            phases++;

            if (!fine_done) cf++;
            tf = t_next;
            vf = v_next;
            nu_f = nu_next;
            Ef = E_next;
            tauf = bg_flight(g, xf, vf, Ef);
            cfine = tf + tauf;
            steps++;
        } while (!(kd_step_of(cfine, dtf) + 1.0 > end_c_fine) && steps < guard);

        if (ccoarse < T) {
            double nu_c = nu_f;                               /* eq. nu-update */
            double chi_c = den > 0.0 ? num / sqrt(den) : 0.0; /* eq. chi-update */
            double t_next = end_c * dtc;
            double theta = t_next - ccoarse;
            double v_next = mu + sigma * nu_c;
            double Rc = bg_rate(g, xc + vc * tauc);
            double ad[2];
            oracle_kd_coeffs(theta, Rc, mu, sigma, v_next, ad);
            xc = xc + vc * tauc + (ad[0] + ad[1] * chi_c);
            tc = t_next;
            vc = v_next;
            /* eq. epsilon-update: the part of the pending fine flight before
             * the coarse time is used up */
            double E_c = Ef - bg_rate_integral(g, xf, vf, tc - tf);
            if (E_c < 0.0) E_c = 0.0;
            tauc = bg_flight(g, xc, vc, E_c);
            ccoarse = tc + tauc;
            cc++;
            if (tr && tr->rows && tr->used < tr->cap) {
                double *r = tr->rows + 4 * tr->used++;
                r[0] = chi_c; r[1] = nu_c; r[2] = E_c; r[3] = (double)used;
            }
        }
    }
    (void)phases;
    if (!fine_done) xf_end = tf < T ? xf + vf * (T - tf) : xf;
    if (tc < T) xc = xc + vc * (T - tc);
    *xf_out = xf_end; *xc_out = xc; *cf_out = cf; *cc_out = cc;
}

/* Paths or pairs (coarse_level < 0: level - 1) in a background; kind
 * BG_B1/BG_B2 with parameters a, b.  general = 0 routes a = 0 to the
 * homogeneous KD path with R = b, sigma = 1; general = 1 always takes the
 * background path (to compare the two). */
int oracle_simulate_kd_bg(double T, double dt0, int M, int level, int coarse_level, int single,
                          int x0_kind, double x0_a, double x0_b, int bg_kind, double bg_a,
                          double bg_b, int general, uint64_t seed, uint32_t stream,
                          uint64_t sample_begin, const uint64_t *idx, uint64_t n,
                          double *xf, double *xc, uint32_t *cf, uint32_t *cc, int nthreads)
{
    if (bg_kind != BG_B1 && bg_kind != BG_B2) return -1;
    if (!(bg_b > 0.0) || !(bg_a >= 0.0)) return -1;
    /* single = 2: single paths under the counter tag of the level's pairs */
    problem_t P = make_problem(1.0, T, dt0, M, level, single != 0, x0_kind, x0_a, x0_b,
                               EQ_MAXWELLIAN, 0, seed, stream);
    P.pair_tag = single == 2;
    if (!single && level >= 1) {
        if (coarse_level < 0) coarse_level = level - 1;
        if (coarse_level >= level) return -1;
        P.coarse_level = coarse_level;
    }
    P.R = bg_b;
    P.sigma = 1.0;
    bg_t g = {bg_kind, bg_a, bg_b};
    const int homogeneous = bg_a == 0.0 && !general;
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t s = idx ? idx[i] : sample_begin + (uint64_t)i;
        if (homogeneous) simulate_kd_one(&P, s, &xf[i], &xc[i], &cf[i], &cc[i], NULL);
        else simulate_kd_bg_one(&P, &g, s, &xf[i], &xc[i], &cf[i], &cc[i], NULL);
    }
    return 0;
}

/* Coarse numbers and fine phases of one pair in a background (as
 * oracle_kd_phases; phase column 15 holds the phase's rate R_m). */
uint64_t oracle_kd_bg_phases(double T, double dt0, int M, int level, int coarse_level,
                             int x0_kind, double x0_a, double x0_b, int bg_kind, double bg_a,
                             double bg_b, uint64_t seed, uint32_t stream, uint64_t sample,
                             double *phases, uint64_t phase_cap, double *rows, uint64_t cap,
                             uint64_t *n_coarse_out, double out_final[2])
{
    problem_t P = make_problem(1.0, T, dt0, M, level, 0, x0_kind, x0_a, x0_b,
                               EQ_MAXWELLIAN, 0, seed, stream);
    if (coarse_level >= 0 && coarse_level < level) P.coarse_level = coarse_level;
    P.R = bg_b;
    P.sigma = 1.0;
    bg_t g = {bg_kind, bg_a, bg_b};
    kd_trace_t tr = {rows, cap, 0, phases, phase_cap, 0};
    double xf, xc; uint32_t cf, cc;
    simulate_kd_bg_one(&P, &g, sample, &xf, &xc, &cf, &cc, &tr);
    out_final[0] = xf; out_final[1] = xc;
    *n_coarse_out = tr.used;
    return tr.phase_used;
}
