/*
 * oracle.c -- plain, slow, FP64 CPU oracle for Parallel-Tempering Monte Carlo of
 * the 4-body smoothed-cubic random-laser model (Benedetti & Leuzzi, arXiv 2511.13508).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this code.  It shares no source with
 * the HIP library: it has its own counter-based generator, its own graph
 * builder and its own Monte Carlo loop, each written from the paper.
 *
 * Every floating-point quantity is double precision.  Functions cite the
 * passage of the paper they follow (section / equation / table).
 *
 * Conventions (readings of the paper, listed again in the design notes):
 *  - a term is stored as (p, s, m, n): the monomial conj(a_p) conj(a_s) a_m a_n,
 *    whose frequencies satisfy |w_p + w_s - w_m - w_n| < gamma  (eq. selection-rule,
 *    eq. FMC with n = 2); the Hamiltonian H4 of eq. Hamilt2 with its "+ c.c."
 *    taken literally is  H = -sum_q J_q (X_q + conj X_q) = -2 sum_q J_q Re X_q.
 *  - the local field of mode l is F_l = sum over terms containing l of
 *    J * conj(a_x) a_y a_z, x = the mode sharing l's side of the term, (y, z)
 *    the other side; then H = -2 Re(conj(a_l) F_l) + (terms without l).
 *
 * Parity status of each function is stated in its header comment.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Counter-based generator: Philox4x64 with 10 rounds, from Salmon, Moraes,   */
/* Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).        */
/* Pinned against numpy.random.Philox, an independent implementation of the  */
/* same published generator.                                                  */
/* ------------------------------------------------------------------------- */
void or_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        __uint128_t p0 = (__uint128_t)M0 * x0;
        __uint128_t p1 = (__uint128_t)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream tags (second key word).  Any fixed distinct constants work; these
 * are shared as a specification, not as code, with the library. */
#define OR_TAG_GRAPH 0x4752415048ULL /* "GRAPH" */
#define OR_TAG_INIT  0x494E4954ULL   /* "INIT"  */
#define OR_TAG_PAIR  0x50414952ULL   /* "PAIR"  */
#define OR_TAG_MOVE  0x4D4F5645ULL   /* "MOVE"  */
#define OR_TAG_SWAP  0x53574150ULL   /* "SWAP"  */

static void draw(uint64_t seed, uint64_t tag, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                 uint64_t out[4])
{
    uint64_t ctr[4] = {c0, c1, c2, c3};
    uint64_t key[2] = {seed, tag};
    or_philox4x64(ctr, key, out);
}

/* uniform in [0, 1) from the top 53 bits */
static double u53(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

/* standard normal by the Box-Muller transform (Box & Muller 1958) */
static double gauss(uint64_t w0, uint64_t w1)
{
    double u1 = 1.0 - u53(w0); /* in (0, 1] */
    double u2 = u53(w1);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * OR_PI * u2);
}

/* index in [0, n) from the top 32 bits of w */
static int32_t pick(uint64_t w, int32_t n)
{
    return (int32_t)(((w >> 32) * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------------- */
/* Graph: quenched random frequencies (sec. II.C, "Quenched random           */
/* frequencies"), linewidth gamma = 1/(2(N-1)) (eq. gamma_scaling),           */
/* FMC filter over ordered quadruplets k1<k2<k3<k4 ("Graph generation"),      */
/* Gaussian couplings (eq. Gauss) with variance sigma^2 = N / c.             */
/* ------------------------------------------------------------------------- */
static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

void or_frequencies(int32_t N, uint64_t seed, int32_t omega_kind, double* omega)
{
    if (omega_kind == 1) { /* equispaced comb on [0, 1] */
        for (int32_t i = 0; i < N; ++i) omega[i] = (double)i / (double)(N - 1);
        return;
    }
    for (int32_t i = 0; i < N; ++i) {
        uint64_t w[4];
        draw(seed, OR_TAG_GRAPH, (uint64_t)i, 0, 0, 0, w);
        omega[i] = u53(w[0]);
    }
    qsort(omega, (size_t)N, sizeof(double), cmp_double);
}

/* Enumerate the kept terms.  For each i<j<k<l the three ways of splitting the
 * four modes into a conjugated pair and a plain pair are tested in the order
 *   A: (i,l | j,k)   B: (i,k | j,l)   C: (i,j | k,l)
 * and every split that passes the frequency-matching condition becomes its
 * own term.  pair_mask selects which splits are tested (bit0 A, bit1 B, bit2 C).
 * If quads is NULL only the count is returned.  Returns the number of terms. */
int64_t or_graph_terms(int32_t N, const double* omega, double gamma, int32_t pair_mask,
                       int16_t* quads, int64_t max_terms)
{
    int64_t c = 0;
    for (int32_t i = 0; i < N; ++i)
        for (int32_t j = i + 1; j < N; ++j)
            for (int32_t k = j + 1; k < N; ++k)
                for (int32_t l = k + 1; l < N; ++l) {
                    int32_t split[3][4] = {{i, l, j, k}, {i, k, j, l}, {i, j, k, l}};
                    for (int s = 0; s < 3; ++s) {
                        if (!(pair_mask & (1 << s))) continue;
                        int32_t p = split[s][0], q = split[s][1], m = split[s][2], n = split[s][3];
                        double mismatch = (omega[p] + omega[q]) - (omega[m] + omega[n]);
                        if (fabs(mismatch) < gamma) {
                            if (quads) {
                                if (c >= max_terms) return -1;
                                quads[4 * c + 0] = (int16_t)p;
                                quads[4 * c + 1] = (int16_t)q;
                                quads[4 * c + 2] = (int16_t)m;
                                quads[4 * c + 3] = (int16_t)n;
                            }
                            ++c;
                        }
                    }
                }
    return c;
}

double or_default_gamma(int32_t N) { return 1.0 / (2.0 * (double)(N - 1)); }

/* Sparse mode-locked graph (finite connectivity per mode, the dilution the
 * paper proposes in sec. II.D and its conclusions; the construction is this
 * library's reading): c = floor(z N / 4) terms drawn uniformly without
 * replacement from the matched terms of the complete graph, by rejection.
 * Attempt t reads Philox counter (t, 2, 0, 0): four modes (top 32 bits of
 * each word times N), a split from the low 32 bits of word 0 times 3.  The
 * attempt is kept when the four modes are distinct, the split (A, B, C on the
 * sorted modes, as above) is in pair_mask, the split is matched and the term
 * was not kept before.  Terms in acceptance order.  Returns c, or -1 when the
 * attempt budget (64 N c + 10^6) runs out. */
int64_t or_graph_terms_sparse(int32_t N, const double* omega, double gamma, int32_t pair_mask, int32_t z,
                              uint64_t seed, int16_t* quads)
{
    int64_t c = (int64_t)z * N / 4, kept = 0;
    uint64_t budget = 64ull * (uint64_t)N * (uint64_t)c + 1000000ull;
    for (uint64_t t = 0; t < budget && kept < c; ++t) {
        uint64_t w[4];
        draw(seed, OR_TAG_GRAPH, t, 2, 0, 0, w);
        int32_t v[4];
        for (int r = 0; r < 4; ++r) v[r] = pick(w[r], N);
        int split = (int)(((w[0] & 0xffffffffULL) * 3ULL) >> 32);
        /* sort the four modes (insertion sort) */
        for (int a = 1; a < 4; ++a)
            for (int b = a; b > 0 && v[b - 1] > v[b]; --b) {
                int32_t x = v[b];
                v[b] = v[b - 1];
                v[b - 1] = x;
            }
        if (v[0] == v[1] || v[1] == v[2] || v[2] == v[3]) continue;
        if (!(pair_mask & (1 << split))) continue;
        int32_t t4[3][4] = {{v[0], v[3], v[1], v[2]}, {v[0], v[2], v[1], v[3]}, {v[0], v[1], v[2], v[3]}};
        int32_t* q = t4[split];
        double mismatch = (omega[q[0]] + omega[q[1]]) - (omega[q[2]] + omega[q[3]]);
        if (!(fabs(mismatch) < gamma)) continue;
        int dup = 0;
        for (int64_t e = 0; e < kept && !dup; ++e)
            dup = quads[4 * e] == q[0] && quads[4 * e + 1] == q[1] && quads[4 * e + 2] == q[2] &&
                  quads[4 * e + 3] == q[3];
        if (dup) continue;
        for (int r = 0; r < 4; ++r) quads[4 * kept + r] = (int16_t)q[r];
        ++kept;
    }
    return kept == c ? c : -1;
}

/* J_q = sigma * g_q, g_q standard normal from counter (q, 1, 0, 0) */
void or_couplings(int32_t N, uint64_t seed, int64_t n_terms, double* J)
{
    double sigma = sqrt((double)N / (double)n_terms);
    for (int64_t q = 0; q < n_terms; ++q) {
        uint64_t w[4];
        draw(seed, OR_TAG_GRAPH, (uint64_t)q, 1, 0, 0, w);
        J[q] = sigma * gauss(w[0], w[1]);
    }
}

/* ------------------------------------------------------------------------- */
/* Energy and local fields (eq. Hamilt2 / H4 with H2 = 0, real J).           */
/* a is interleaved (re, im) of length 2N.                                    */
/* ------------------------------------------------------------------------- */

/* complex helpers written out */
typedef struct { double re, im; } cplx;
static cplx C(const double* a, int32_t k) { cplx z = {a[2 * k], a[2 * k + 1]}; return z; }
static cplx cmul(cplx x, cplx y) { cplx z = {x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re}; return z; }
static cplx cconj(cplx x) { cplx z = {x.re, -x.im}; return z; }

/* H = -2 sum_q J_q Re( conj(a_p) conj(a_s) a_m a_n ) */
double or_energy(int64_t n_terms, const int16_t* quads, const double* J, const double* a)
{
    double H = 0.0;
    for (int64_t q = 0; q < n_terms; ++q) {
        cplx x = cmul(cmul(cconj(C(a, quads[4 * q])), cconj(C(a, quads[4 * q + 1]))),
                      cmul(C(a, quads[4 * q + 2]), C(a, quads[4 * q + 3])));
        H += -2.0 * J[q] * x.re;
    }
    return H;
}

/* contribution of term q to the field of its member l (l must be in q) */
static cplx term_field(const int16_t* t, double Jq, const double* a, int32_t l)
{
    int32_t p = t[0], s = t[1], m = t[2], n = t[3];
    cplx r;
    if (l == p)      r = cmul(cconj(C(a, s)), cmul(C(a, m), C(a, n)));
    else if (l == s) r = cmul(cconj(C(a, p)), cmul(C(a, m), C(a, n)));
    else if (l == m) r = cmul(cconj(C(a, n)), cmul(C(a, p), C(a, s)));
    else             r = cmul(cconj(C(a, m)), cmul(C(a, p), C(a, s)));
    r.re *= Jq;
    r.im *= Jq;
    return r;
}

/* all N local fields by one pass over the terms; F interleaved (re, im) */
void or_fields(int32_t N, int64_t n_terms, const int16_t* quads, const double* J, const double* a,
               double* F)
{
    memset(F, 0, sizeof(double) * 2 * (size_t)N);
    for (int64_t q = 0; q < n_terms; ++q)
        for (int r = 0; r < 4; ++r) {
            int32_t l = quads[4 * q + r];
            cplx f = term_field(&quads[4 * q], J[q], a, l);
            F[2 * l] += f.re;
            F[2 * l + 1] += f.im;
        }
}

/* Energy change of the paper's two-mode update (sec. III.A, "Single Metropolis
 * update" and "Energy update parallel computation"): both fields are taken on
 * one snapshot in which a_j already holds its new value and a_k the old one.
 * Pinned by brute force H(a') - H(a) in the tests. */
double or_pair_dE(int32_t N, int64_t n_terms, const int16_t* quads, const double* J, const double* a,
                  int32_t j, int32_t k, const double* aj_new, const double* ak_new)
{
    double* b = (double*)malloc(sizeof(double) * 2 * (size_t)N);
    double* F = (double*)malloc(sizeof(double) * 2 * (size_t)N);
    memcpy(b, a, sizeof(double) * 2 * (size_t)N);
    b[2 * j] = aj_new[0];
    b[2 * j + 1] = aj_new[1];
    or_fields(N, n_terms, quads, J, b, F);
    double dj_re = aj_new[0] - a[2 * j], dj_im = aj_new[1] - a[2 * j + 1];
    double dk_re = ak_new[0] - a[2 * k], dk_im = ak_new[1] - a[2 * k + 1];
    /* Re(conj(d) F) = d.re F.re + d.im F.im */
    double dE = -2.0 * (dj_re * F[2 * j] + dj_im * F[2 * j + 1]) - 2.0 * (dk_re * F[2 * k] + dk_im * F[2 * k + 1]);
    free(b);
    free(F);
    return dE;
}

/* ------------------------------------------------------------------------- */
/* Parallel tempering (sec. III.A "Exchange Monte Carlo - parallel          */
/* Tempering", Table I layout of baths x replicas).                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t n_modes;           /* N */
    int32_t rho;               /* constraint sum |a|^rho = N, eq. SmoothedCubic: 4 (0 reads as 4) or 2 */
    int64_t n_terms;           /* c */
    const int16_t* quads;      /* [c][4] (p, s, m, n) */
    const double* J;           /* [c] */
    int32_t n_temps, n_reps;   /* baths, replicas per bath */
    const double* temps;       /* [n_temps], ascending */
    uint64_t run_seed;
    int32_t sample;            /* disorder sample index mu; copy id = mu*R + local id */
    int32_t shared_pairs;      /* 0: each copy draws its own pairs; 1: one pair sequence per sample */
    int32_t swap_interval;     /* sweeps between swap rounds (>= 1) */
    int32_t resync_interval;   /* sweeps between energy recomputations (0 = never) */
    double renorm_tol;         /* rescale a when |sum|a|^4 / N - 1| exceeds this */
    int32_t measure_start;     /* measure after completed sweep n when n > measure_start ... */
    int32_t measure_interval;  /* ... and n % measure_interval == 0 */
    int32_t n_bins;            /* overlap histogram bins on [-1, 1] */
    int32_t series_len;        /* stored measurements of E and q per temperature */
    int32_t n_threads;         /* OpenMP threads for the copy loop (<= 0: runtime default) */
    int32_t pad1;
} or_pt_params;

typedef struct {
    double* a;          /* [R][N][2], R = n_temps * n_reps, copy r*n_temps + i */
    double* E;          /* [R] running energy */
    int32_t* temp_of;   /* [R] temperature index held by each copy */
    int64_t sweeps_done;
    int64_t swaps_done;
} or_pt_state;

typedef struct {
    double* e_n;  double* e_sum;  double* e_sq;   /* [T] energy moments */
    double* y2_sum; double* y4_sum;                /* [T] IPR sums */
    double* q_n;  double* q_sum;  double* q_sq;  double* q_4; /* [T] overlap moments */
    double* hist;                                  /* [T][n_bins] overlap histogram */
    double* acc;  double* tries;                   /* [T] pair-move acceptance */
    double* swap_acc; double* swap_tries;          /* [T-1] exchange acceptance */
    double* series_e; double* series_q;            /* [T][series_len] */
    double* hist_I;                                /* [T][n_bins] total intensity I/N on [0, 1] */
    double* spectrum;                              /* [T][N] sum of |a_k|^2 over measurements and replicas */
    int64_t n_meas;
} or_pt_accum;

/* per-mode term lists, built once per run (plain CSR of term indices) */
typedef struct {
    int64_t* off;   /* [N+1] */
    int64_t* term;  /* [4c] */
} or_lists;

static void lists_build(const or_pt_params* P, or_lists* L)
{
    int32_t N = P->n_modes;
    L->off = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
    L->term = (int64_t*)malloc(sizeof(int64_t) * 4 * (size_t)(P->n_terms > 0 ? P->n_terms : 1));
    for (int64_t q = 0; q < P->n_terms; ++q)
        for (int r = 0; r < 4; ++r) L->off[P->quads[4 * q + r] + 1]++;
    for (int32_t l = 0; l < N; ++l) L->off[l + 1] += L->off[l];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    for (int32_t l = 0; l < N; ++l) fill[l] = L->off[l];
    for (int64_t q = 0; q < P->n_terms; ++q)
        for (int r = 0; r < 4; ++r) L->term[fill[P->quads[4 * q + r]]++] = q;
    free(fill);
}

static void lists_free(or_lists* L) { free(L->off); free(L->term); }

static cplx field_from_lists(const or_pt_params* P, const or_lists* L, const double* a, int32_t l)
{
    cplx F = {0.0, 0.0};
    for (int64_t e = L->off[l]; e < L->off[l + 1]; ++e) {
        int64_t q = L->term[e];
        cplx f = term_field(&P->quads[4 * q], P->J[q], a, l);
        F.re += f.re;
        F.im += f.im;
    }
    return F;
}

/* Initial configuration: an exact draw from the beta = 0 law of eq. ProbDistr
 * (flat measure on the constraint surface of eq. SmoothedCubic after the
 * rescaling of sec. II.B), phases uniform.  Counter (k, copy id, 0, 0).
 *  rho = 4: with u_k = |a_k|^2 the surface sum u^2 = N, u >= 0, is a sphere
 *    sector and the flat measure on it is uniform: u = sqrt(N) |g| / ||g||
 *    with g standard normal.
 *  rho = 2 (the spherical constraint sum |a|^2 = N of sec. II.B): the
 *    intensities I_k = |a_k|^2 of a uniform point of the complex sphere are
 *    N times a flat Dirichlet vector: I = N e / sum e with e_k ~ Exp(1). */
void or_init_copy_rho(int32_t N, uint64_t run_seed, int64_t copy_id, int32_t rho, double* a)
{
    double* g = (double*)malloc(sizeof(double) * (size_t)N);
    double* ph = (double*)malloc(sizeof(double) * (size_t)N);
    double norm = 0.0;
    for (int32_t k = 0; k < N; ++k) {
        uint64_t w[4];
        draw(run_seed, OR_TAG_INIT, (uint64_t)k, (uint64_t)copy_id, 0, 0, w);
        if (rho == 2) {
            g[k] = -log(1.0 - u53(w[0]));
            norm += g[k];
        } else {
            g[k] = gauss(w[0], w[1]);
            norm += g[k] * g[k];
        }
        ph[k] = 2.0 * OR_PI * u53(w[2]);
    }
    for (int32_t k = 0; k < N; ++k) {
        double I = rho == 2 ? (double)N * g[k] / norm : sqrt((double)N) * fabs(g[k]) / sqrt(norm);
        double A = sqrt(I);
        a[2 * k] = A * cos(ph[k]);
        a[2 * k + 1] = A * sin(ph[k]);
    }
    free(g);
    free(ph);
}

void or_init_copy(int32_t N, uint64_t run_seed, int64_t copy_id, double* a)
{
    or_init_copy_rho(N, run_seed, copy_id, 4, a);
}

static int32_t rho_of(const or_pt_params* P) { return P->rho == 2 ? 2 : 4; }

void or_pt_init(const or_pt_params* P, or_pt_state* S)
{
    int32_t N = P->n_modes, R = P->n_temps * P->n_reps;
    for (int32_t c = 0; c < R; ++c) {
        int64_t id = (int64_t)P->sample * R + c;
        or_init_copy_rho(N, P->run_seed, id, rho_of(P), &S->a[(size_t)2 * N * c]);
        S->E[c] = or_energy(P->n_terms, P->quads, P->J, &S->a[(size_t)2 * N * c]);
        S->temp_of[c] = c % P->n_temps;
    }
    S->sweeps_done = 0;
    S->swaps_done = 0;
}

/* One proposal of the two-mode move, sec. III.A "Single Metropolis update":
 * random distinct j, k; fresh phases in [0, 2 pi); new magnitudes on the
 * pair's share of the constraint, with the third uniform u:
 *  rho = 4: K^4 = |a_j|^4 + |a_k|^4, theta = (pi/2) u,
 *    A_j' = K sqrt(cos theta), A_k' = K sqrt(sin theta) (as printed);
 *  rho = 2: K^2 = |a_j|^2 + |a_k|^2, A_j' = K cos theta, A_k' = K sin theta
 *    with sin^2 theta = u uniform, i.e. A_j' = K sqrt(1 - u), A_k' = K sqrt(u).
 * In both cases the new intensities are uniform on the pair's constraint curve
 * under the flat measure, so the proposal is the reference law there and the
 * Metropolis test on the energy alone is exact.  Returns j, k and the proposed
 * values; the pair comes from the pair stream, everything else from the
 * copy's move stream. */
static void propose(int32_t N, int32_t rho, uint64_t run_seed, int64_t pair_stream, int64_t copy_id,
                    int64_t sweep, int32_t step, const double* a, int32_t* j_out, int32_t* k_out,
                    double* aj_new, double* ak_new, double* u_acc)
{
    uint64_t wp[4], wm[4];
    draw(run_seed, OR_TAG_PAIR, (uint64_t)step, (uint64_t)sweep, (uint64_t)pair_stream, 0, wp);
    draw(run_seed, OR_TAG_MOVE, (uint64_t)step, (uint64_t)sweep, (uint64_t)copy_id, 0, wm);
    int32_t j = pick(wp[0], N);
    int32_t k = pick(wp[1], N - 1);
    if (k >= j) k += 1;
    double aj2 = a[2 * j] * a[2 * j] + a[2 * j + 1] * a[2 * j + 1];
    double ak2 = a[2 * k] * a[2 * k] + a[2 * k + 1] * a[2 * k + 1];
    double phj = 2.0 * OR_PI * u53(wm[0]);
    double phk = 2.0 * OR_PI * u53(wm[1]);
    double Aj, Ak;
    if (rho == 2) {
        double K = sqrt(aj2 + ak2);
        double u = u53(wm[2]);
        Aj = K * sqrt(1.0 - u);
        Ak = K * sqrt(u);
    } else {
        double K = pow(aj2 * aj2 + ak2 * ak2, 0.25);
        double theta = 0.5 * OR_PI * u53(wm[2]);
        double cj = cos(theta), sk = sin(theta);
        Aj = K * sqrt(cj > 0.0 ? cj : 0.0);
        Ak = K * sqrt(sk > 0.0 ? sk : 0.0);
    }
    aj_new[0] = Aj * cos(phj);
    aj_new[1] = Aj * sin(phj);
    ak_new[0] = Ak * cos(phk);
    ak_new[1] = Ak * sin(phk);
    *u_acc = u53(wm[3]);
    *j_out = j;
    *k_out = k;
}

/* One sweep (N/2 two-mode updates, sec. III.A) of one copy at inverse
 * temperature beta.  Returns the number of accepted moves. */
static int32_t sweep_copy(const or_pt_params* P, const or_lists* L, double* a, double* E, double beta,
                          int64_t copy_id, int64_t sweep)
{
    int32_t N = P->n_modes, acc = 0;
    int64_t pair_stream = P->shared_pairs ? (int64_t)P->sample : copy_id;
    for (int32_t step = 0; step < N / 2; ++step) {
        int32_t j, k;
        double aj_new[2], ak_new[2], u;
        propose(N, rho_of(P), P->run_seed, pair_stream, copy_id, sweep, step, a, &j, &k, aj_new, ak_new, &u);
        double aj_old[2] = {a[2 * j], a[2 * j + 1]};
        /* snapshot: a_j replaced by its proposal, a_k old */
        a[2 * j] = aj_new[0];
        a[2 * j + 1] = aj_new[1];
        cplx Fj = field_from_lists(P, L, a, j);
        cplx Fk = field_from_lists(P, L, a, k);
        double dE = -2.0 * ((aj_new[0] - aj_old[0]) * Fj.re + (aj_new[1] - aj_old[1]) * Fj.im)
                    - 2.0 * ((ak_new[0] - a[2 * k]) * Fk.re + (ak_new[1] - a[2 * k + 1]) * Fk.im);
        int accept = (dE <= 0.0) || (u < exp(-beta * dE));
        if (accept) {
            a[2 * k] = ak_new[0];
            a[2 * k + 1] = ak_new[1];
            *E += dE;
            ++acc;
        } else {
            a[2 * j] = aj_old[0];
            a[2 * j + 1] = aj_old[1];
        }
    }
    return acc;
}

/* Swap round, sec. III.A: for every ladder (one per replica index) the pairs of
 * neighbouring temperatures are proposed in ascending order, each accepted with
 * min[1, exp((beta_i - beta_{i+1}) (H_i - H_{i+1}))]. */
static void swap_round(const or_pt_params* P, or_pt_state* S, or_pt_accum* A)
{
    int32_t T = P->n_temps;
    int32_t* at = (int32_t*)malloc(sizeof(int32_t) * (size_t)T);
    for (int32_t r = 0; r < P->n_reps; ++r) {
        for (int32_t i = 0; i < T; ++i) {
            int32_t c = r * T + i;
            at[S->temp_of[c]] = c;
        }
        int64_t ladder = (int64_t)P->sample * P->n_reps + r;
        for (int32_t i = 0; i + 1 < T; ++i) {
            uint64_t w[4];
            draw(P->run_seed, OR_TAG_SWAP, (uint64_t)i, (uint64_t)S->swaps_done, (uint64_t)ladder, 0, w);
            double bi = 1.0 / P->temps[i], bj = 1.0 / P->temps[i + 1];
            double x = (bi - bj) * (S->E[at[i]] - S->E[at[i + 1]]);
            int accept = (x >= 0.0) || (u53(w[0]) < exp(x));
            if (A) A->swap_tries[i] += 1.0;
            if (accept) {
                int32_t ci = at[i], cj = at[i + 1];
                at[i] = cj;
                at[i + 1] = ci;
                S->temp_of[ci] = i + 1;
                S->temp_of[cj] = i;
                if (A) A->swap_acc[i] += 1.0;
            }
        }
    }
    S->swaps_done += 1;
    free(at);
}

/* Recompute every energy from scratch and restore the constraint if it has
 * drifted by more than renorm_tol (H is homogeneous of degree 4, so scaling a
 * by f = (N/S)^(1/rho), S = sum |a|^rho, scales H by f^4).  Returns the
 * largest relative difference between the running and recomputed energies. */
static double resync(const or_pt_params* P, or_pt_state* S)
{
    int32_t N = P->n_modes, R = P->n_temps * P->n_reps, rho = rho_of(P);
    double worst = 0.0;
    for (int32_t c = 0; c < R; ++c) {
        double* a = &S->a[(size_t)2 * N * c];
        double H = or_energy(P->n_terms, P->quads, P->J, a);
        double Sr = 0.0;
        for (int32_t k = 0; k < N; ++k) {
            double u = a[2 * k] * a[2 * k] + a[2 * k + 1] * a[2 * k + 1];
            Sr += rho == 2 ? u : u * u;
        }
        double scale = fabs(H) > 1.0 ? fabs(H) : 1.0;
        double d = fabs(S->E[c] - H) / scale;
        if (d > worst) worst = d;
        if (fabs(Sr / N - 1.0) > P->renorm_tol) {
            double f = pow((double)N / Sr, 1.0 / rho);
            for (int32_t k = 0; k < 2 * N; ++k) a[k] *= f;
            H *= f * f * f * f;
        }
        S->E[c] = H;
    }
    return worst;
}

/* Observables of sec. IV: energy moments for the specific heat (eq.
 * SpecificHeat), the replica overlap q_cd = (1/N) Re sum conj(a^c) a^d and its
 * histogram on [-1, 1] (sec. IV "Parisi overlap distribution"), and the
 * inverse participation ratios Y_2, Y_4 (sec. IV "Inverse participation
 * ratio's"). */
static void measure(const or_pt_params* P, const or_pt_state* S, or_pt_accum* A)
{
    int32_t N = P->n_modes, T = P->n_temps, Rn = P->n_reps;
    int32_t* at = (int32_t*)malloc(sizeof(int32_t) * (size_t)T * Rn);
    for (int32_t c = 0; c < T * Rn; ++c) at[(c / T) * T + S->temp_of[c]] = c;
    for (int32_t t = 0; t < T; ++t) {
        for (int32_t r = 0; r < Rn; ++r) {
            int32_t c = at[r * T + t];
            const double* a = &S->a[(size_t)2 * N * c];
            double s1 = 0.0, s2 = 0.0, s4 = 0.0;
            for (int32_t k = 0; k < N; ++k) {
                double I = a[2 * k] * a[2 * k] + a[2 * k + 1] * a[2 * k + 1];
                s1 += I;
                s2 += I * I;
                s4 += I * I * I * I;
                /* intensity spectrum I(omega_k) = <|a_k|^2> (sec. II.C), modes in frequency order */
                A->spectrum[(size_t)t * N + k] += I;
            }
            A->e_n[t] += 1.0;
            A->e_sum[t] += S->E[c];
            A->e_sq[t] += S->E[c] * S->E[c];
            A->y2_sum[t] += s2 / (s1 * s1);
            A->y4_sum[t] += s4 / (s2 * s2);
            {   /* distribution of the total intensity I = sum |a|^2 (sec. II.B, P(I)) */
                int32_t bI = (int32_t)floor(s1 / (double)N * P->n_bins);
                if (bI < 0) bI = 0;
                if (bI >= P->n_bins) bI = P->n_bins - 1;
                A->hist_I[(size_t)t * P->n_bins + bI] += 1.0;
            }
            if (r == 0 && A->n_meas < P->series_len) A->series_e[(size_t)t * P->series_len + A->n_meas] = S->E[c];
        }
        for (int32_t r = 0; r < Rn; ++r)
            for (int32_t r2 = r + 1; r2 < Rn; ++r2) {
                const double* x = &S->a[(size_t)2 * N * at[r * T + t]];
                const double* y = &S->a[(size_t)2 * N * at[r2 * T + t]];
                double q = 0.0;
                for (int32_t k = 0; k < N; ++k) q += x[2 * k] * y[2 * k] + x[2 * k + 1] * y[2 * k + 1];
                q /= (double)N;
                A->q_n[t] += 1.0;
                A->q_sum[t] += q;
                A->q_sq[t] += q * q;
                A->q_4[t] += q * q * q * q;
                int32_t b = (int32_t)floor((q + 1.0) * 0.5 * P->n_bins);
                if (b < 0) b = 0;
                if (b >= P->n_bins) b = P->n_bins - 1;
                A->hist[(size_t)t * P->n_bins + b] += 1.0;
                if (r == 0 && r2 == 1 && A->n_meas < P->series_len)
                    A->series_q[(size_t)t * P->series_len + A->n_meas] = q;
            }
    }
    A->n_meas += 1;
    free(at);
}

/* Run n_sweeps iterations of: sweep every copy; swap round every
 * swap_interval sweeps; energy recomputation every resync_interval sweeps;
 * measurement on the schedule of the params.  Returns the largest energy drift
 * seen at a recomputation. */
double or_pt_run(const or_pt_params* P, or_pt_state* S, or_pt_accum* A, int64_t n_sweeps)
{
    int32_t N = P->n_modes, T = P->n_temps, R = P->n_temps * P->n_reps;
    or_lists L;
    lists_build(P, &L);
    int32_t* acc = (int32_t*)malloc(sizeof(int32_t) * (size_t)R);
    double worst = 0.0;
    int n_threads = 1;
#ifdef _OPENMP
    n_threads = P->n_threads > 0 ? P->n_threads : omp_get_max_threads();
#endif
    for (int64_t it = 0; it < n_sweeps; ++it) {
        int64_t w = S->sweeps_done;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
        for (int32_t c = 0; c < R; ++c) {
            double beta = 1.0 / P->temps[S->temp_of[c]];
            int64_t id = (int64_t)P->sample * R + c;
            acc[c] = sweep_copy(P, &L, &S->a[(size_t)2 * N * c], &S->E[c], beta, id, w);
        }
        for (int32_t c = 0; c < R; ++c) {
            if (A) {
                A->acc[S->temp_of[c]] += acc[c];
                A->tries[S->temp_of[c]] += N / 2;
            }
        }
        S->sweeps_done = w + 1;
        int64_t n = S->sweeps_done;
        if (P->swap_interval > 0 && n % P->swap_interval == 0 && T > 1) swap_round(P, S, A);
        if (P->resync_interval > 0 && n % P->resync_interval == 0) {
            double d = resync(P, S);
            if (d > worst) worst = d;
        }
        if (A && n > P->measure_start && P->measure_interval > 0 && n % P->measure_interval == 0) measure(P, S, A);
    }
    free(acc);
    lists_free(&L);
    return worst;
}
