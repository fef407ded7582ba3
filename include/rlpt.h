/*
 * rlpt.h -- C ABI of librlpt: parallel-tempering Monte Carlo of the 4-body
 * smoothed-cubic random-laser Hamiltonian on a mode-locked graph, for AMD
 * Instinct MI355X (gfx950).  Method: Benedetti & Leuzzi, "Smoothed-Cubic
 * Spin-Glass Model of Random Lasers", arXiv 2511.13508.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns int: RLPT_OK (0) or a negative RLPT_E_* code; the
 *    message of the last failure on the calling thread is rlpt_last_error().
 *  - Host pointers are plain caller-owned arrays.  Device memory for a context
 *    is ONE caller-owned workspace (e.g. a torch uint8 tensor), sized by
 *    rlpt_workspace_size(); the library never allocates device memory for a
 *    context and never frees the workspace.  The stream is caller-owned too.
 *  - Work submitted by rlpt_init / rlpt_sweep / rlpt_swap is asynchronous on
 *    the context's stream.  Calls that return host data synchronise the stream.
 *  - Complex amplitudes cross the boundary as interleaved (re, im) doubles.
 *  - A term (p, s, m, n) is the monomial conj(a_p) conj(a_s) a_m a_n; the
 *    Hamiltonian is H = -sum_q J_q (X_q + c.c.) = -2 sum_q J_q Re X_q
 *    (eq. H4 of the paper with H2 = 0 and real couplings, sec. II).
 *  - Copies: a context holds S disorder samples, each with n_reps ladders of
 *    n_temps baths (Table I layout).  Copy c = mu*R + r*n_temps + i with
 *    R = n_temps*n_reps; copy c starts at temperature index i of its ladder
 *    and moves between temperatures only through swaps.
 */
#ifndef RLPT_H
#define RLPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RLPT_ABI_VERSION 4

enum {
    RLPT_OK = 0,
    RLPT_E_ARG = -1,         /* invalid argument or size */
    RLPT_E_NOMEM = -2,       /* host allocation failed or workspace too small */
    RLPT_E_HIP = -3,         /* a HIP runtime call failed */
    RLPT_E_STATE = -4,       /* NaN or energy / constraint drift found at a resync */
    RLPT_E_UNSUPPORTED = -5  /* option the library does not support (e.g. learned moves in FP64) */
};

enum { RLPT_OMEGA_RANDOM = 0, RLPT_OMEGA_COMB = 1 };
enum { RLPT_SPLIT_A = 1, RLPT_SPLIT_B = 2, RLPT_SPLIT_C = 4, RLPT_SPLIT_ALL = 7 };
enum { RLPT_FP32 = 0, RLPT_FP64 = 1 };
enum { RLPT_LAYOUT_AUTO = 0, RLPT_LAYOUT_PACKED = 1, RLPT_LAYOUT_CHUNKED = 2 };
enum { RLPT_FIELDS_STREAM = 0, RLPT_FIELDS_CACHED = 1 };

/* ABI version (RLPT_ABI_VERSION of the built library). */
int rlpt_abi_version(void);

/* Message of the last failed call on this thread ("" if none).  The pointer is
 * valid until the next rlpt call on the same thread. */
const char* rlpt_last_error(void);

/* ------------------------------------------------------------------------ */
/* Graph and couplings (sec. II.C: quenched random frequencies, eq.          */
/* gamma_scaling, "Graph generation", eq. Gauss).  Host only.                */
/* ------------------------------------------------------------------------ */
typedef struct rlpt_graph rlpt_graph;

typedef struct rlpt_graph_desc {
    int32_t n_modes;     /* N, 4 <= N <= 1024 */
    int32_t omega_kind;  /* RLPT_OMEGA_RANDOM: sorted uniforms on [0,1); RLPT_OMEGA_COMB: k/(N-1) */
    uint64_t seed;       /* disorder seed: frequencies and couplings */
    int32_t split_mask;  /* which splits of each i<j<k<l are tested (RLPT_SPLIT_*) */
    int32_t mean_degree; /* 0: the complete mode-locked graph (every matched term).  z > 0: a sparse
                            mode-locked graph with finite connectivity per mode (the dilution sec. II.D
                            and the conclusions propose), c = floor(z N / 4) terms drawn uniformly
                            without replacement from the matched terms: attempt t takes Philox
                            counter (t, 2, 0, 0) -> four indices (top 32 bits of each word times N),
                            a split from the low 32 bits of word 0 times 3 (0: (a,d|b,c), 1:
                            (a,c|b,d), 2: (a,b|c,d) on the sorted indices a<b<c<d), kept if the
                            indices are distinct, the split is in split_mask, the term is matched
                            and new.  Terms in acceptance order; J as for the complete graph. */
    double gamma;        /* linewidth; <= 0 selects 1/(2(N-1)) (eq. gamma_scaling) */
} rlpt_graph_desc;

typedef struct rlpt_graph_info {
    int32_t n_modes;
    int32_t pad;
    int64_t n_terms;     /* c, number of kept terms */
    int64_t deg_min, deg_max, deg_sum; /* per-mode term counts; deg_sum = 4c */
    double gamma;
    double sigma2;       /* coupling variance N / c */
    int64_t list_entries;/* packed layout: per-mode list entries after padding to multiples of 4 */
    int64_t list_bytes;  /* packed layout: bytes of all per-mode lists in an FP32 context (8 B/entry) */
    int64_t chunk_entries;/* chunked layout (N <= 256): entries after padding each partner group to 4 */
    int64_t chunk_bytes; /* chunked layout: bytes of all lists in an FP32 context (25 B per 4 entries) */
    int64_t pair_entries;   /* cached-field mode: entries of the per-pair lists (12 c; 4 B index + J) */
    int64_t gather_entries; /* cached-field mode: padded entries of the sliced-ELL field-update blocks
                               (2 B index in the chunked layout, 4 B in the packed one, + J) */
} rlpt_graph_info;

/* Build one disorder sample: frequencies; every split of every i<j<k<l into a
 * conjugated pair (p, s) and a plain pair (m, n) with |w_p + w_s - w_m - w_n|
 * < gamma becomes a term (splits tested in the order (i,l|j,k), (i,k|j,l),
 * (i,j|k,l)); J_q ~ N(0, N/c) drawn in term order.  Generator: Philox4x64-10
 * keyed by (seed, "GRAPH").  On success *out owns host memory; free it with
 * rlpt_graph_free.  Errors: RLPT_E_ARG (N out of range, NULL), RLPT_E_NOMEM. */
int rlpt_graph_build(const rlpt_graph_desc* desc, rlpt_graph** out);
void rlpt_graph_free(rlpt_graph* g);
int rlpt_graph_info_get(const rlpt_graph* g, rlpt_graph_info* out);

/* Copy out frequencies omega[N], terms quads[c][4] (p, s, m, n) and couplings
 * J[c] (double).  Any output pointer may be NULL.  Caller-allocated. */
int rlpt_graph_export(const rlpt_graph* g, double* omega, int16_t* quads, double* J);

/* ------------------------------------------------------------------------ */
/* Parallel-tempering context (sec. III.A).                                  */
/* ------------------------------------------------------------------------ */
typedef struct rlpt_ctx rlpt_ctx;

typedef struct rlpt_config {
    int32_t n_temps;          /* baths per ladder (N_PT of Table I) */
    int32_t n_reps;           /* ladders (replicas) per sample, >= 1; overlaps need >= 2 */
    int32_t precision;        /* RLPT_FP32 (fields, dE, running energy in FP32) or RLPT_FP64 */
    int32_t shared_pairs;     /* 0: each copy draws its own pair sequence (paper);
                                 1: all copies of a sample share one pair sequence */
    int32_t swap_interval;    /* sweeps between swap rounds, >= 1 */
    int32_t resync_interval;  /* sweeps between FP64 energy recomputations (0 = never) */
    double renorm_tol;        /* rescale a copy when |sum|a|^4/N - 1| exceeds this */
    double drift_tol;         /* RLPT_E_STATE when |E_run - H|/max(|H|,1) exceeds this at a
                                 recomputation (<= 0: no check; NaN always fails) */
    int32_t measure_start;    /* measure after completed sweep n when n > measure_start */
    int32_t measure_interval; /* ... and n % measure_interval == 0 */
    int32_t n_bins;           /* overlap histogram bins on [-1, 1] */
    int32_t series_len;       /* stored measurements of E (ladder 0) and q_01 per bath */
    int32_t block_threads;    /* threads per workgroup of the sweep kernel: 0 = tuned, else 64..1024 */
    int32_t copies_per_block; /* copies per workgroup: 0 = tuned, else divides block_threads/64 */
    int32_t list_layout;      /* per-mode list layout streamed by the sweep: RLPT_LAYOUT_AUTO,
                                 RLPT_LAYOUT_PACKED (8 B/entry, any N) or RLPT_LAYOUT_CHUNKED
                                 (entries grouped by partner mode in chunks of 4 sharing one
                                 partner byte, 6.25 B/entry, N <= 256) */
    /* learned global proposal (FP32 contexts, one N for all samples); 0 nets = off */
    int32_t mlp_nets;         /* networks, one per learned temperature slot */
    int32_t mlp_hidden;       /* width of the two hidden SiLU layers (default 256) */
    int32_t mlp_components;   /* Gaussian-mixture components, 1..8 (default 4) */
    int32_t mlp_capacity;     /* training pairs stored per network (default 100000) */
    int32_t mlp_batch;        /* training minibatch (default 512) */
    int32_t field_mode;       /* RLPT_FIELDS_STREAM (default): each two-mode update streams the
                                 lists of j and k to form F_j, F_k (sec. III.A);
                                 RLPT_FIELDS_CACHED: every copy keeps all N local fields
                                 (eq. local field) in device memory; an update reads only the
                                 terms holding both j and k (12 entries per term in all) and
                                 streams the two lists only when accepted, to update the fields
                                 it changes.  Same chain, same draws; results agree with the
                                 streaming sweep up to rounding order (each target's field
                                 change is gathered in a fixed order).  Fields are recomputed
                                 from scratch at init, every recomputation, rlpt_set_state and
                                 learned rounds.
                                 Needs 12 * n_terms more list entries of 4 + 4|8 bytes and
                                 (N^2 + 1) * 4 bytes per sample. */
    int32_t rho;              /* global constraint sum_k |a_k|^rho = N (eq. SmoothedCubic): 4 (default;
                                 0 reads as 4), or 2 for the spherical constraint of fixed total
                                 intensity that sec. II.B compares with.  rho = 2 draws the new
                                 magnitudes as A_j' = K cos theta, A_k' = K sin theta with
                                 K^2 = |a_j|^2 + |a_k|^2 and sin^2 theta uniform, the flat law on the
                                 pair's circle, so the energy-only Metropolis test stays exact.
                                 Learned moves need rho = 4. */
    int32_t mlp_subset;       /* learned move kind: 0 (default) moves every mode at once (the chart of
                                 all modes); m >= 2 redraws a random subset of m modes (2 <= m <= min(N, 64))
                                 in the chart of the subset and leaves the others unchanged, its energy
                                 change summed from the m modes' lists (O(m N^2) per move) */
} rlpt_config;

/* Fill *cfg with defaults: FP32, per-copy pairs, swap every sweep, FP64
 * recomputation every 100 sweeps, renorm_tol 1e-6, drift_tol 1e-3, 100 bins. */
int rlpt_config_default(rlpt_config* cfg);

/* Device bytes needed for a context over graphs[0..n_graphs) (one per sample). */
int rlpt_workspace_size(const rlpt_config* cfg, const rlpt_graph* const* graphs, int32_t n_graphs,
                        size_t* bytes);

/* Create a context.  temps[n_temps] (strictly ascending, > 0) is the ladder of
 * every sample.  d_workspace: caller-owned device memory of at least
 * rlpt_workspace_size() bytes, 256-byte aligned, alive until rlpt_destroy.
 * hip_stream: a hipStream_t (NULL = default stream).  Uploads lists,
 * couplings and ladders (host -> device copies on the stream).  The graphs
 * may be freed after this call.  Errors: RLPT_E_ARG, RLPT_E_NOMEM, RLPT_E_HIP. */
int rlpt_create(const rlpt_config* cfg, const rlpt_graph* const* graphs, int32_t n_graphs,
                const double* temps, void* d_workspace, size_t workspace_bytes, void* hip_stream,
                rlpt_ctx** out);
int rlpt_destroy(rlpt_ctx* ctx);

/* Draw every copy from the infinite-temperature law of eq. ProbDistr (flat
 * measure on sum|a|^4 = N, eq. SmoothedCubic rescaled): |a_k|^2 =
 * sqrt(N)|g_k|/||g||, g standard normal, phases uniform; Philox keyed by
 * (run_seed, "INIT") at counter (k, copy, 0, 0).  Resets temperatures,
 * counters and accumulators; computes every energy in FP64.  Async. */
int rlpt_init(rlpt_ctx* ctx, uint64_t run_seed);

/* Advance n_sweeps sweeps.  One sweep = N/2 two-mode updates per copy (sec.
 * III.A "Single Metropolis update"): distinct j, k from the pair stream;
 * K^4 = |a_j|^4 + |a_k|^4; new phases 2 pi u; theta = (pi/2) u; |a_j'| =
 * K sqrt(cos theta), |a_k'| = K sqrt(sin theta); accept when dE <= 0 or
 * u < exp(-beta dE).  After every swap_interval sweeps a swap round, every
 * resync_interval sweeps an FP64 recomputation, and measurements on the
 * configured schedule.  Async; a drift/NaN failure is reported by the next
 * synchronising call (rlpt_check, rlpt_observables, ...). */
int rlpt_sweep(rlpt_ctx* ctx, int32_t n_sweeps);

/* One extra swap round now (sec. III.A: neighbouring baths proposed in
 * ascending order, accepted with min[1, exp((b_i - b_{i+1})(H_i - H_{i+1}))]).
 * Async. */
int rlpt_swap(rlpt_ctx* ctx);

/* Recompute every energy in FP64 now (and renormalise drifted copies);
 * synchronises; *max_drift (may be NULL) receives the largest relative
 * difference between running and recomputed energies. */
int rlpt_resync(rlpt_ctx* ctx, double* max_drift);

/* Synchronise and report any drift / NaN failure recorded so far. */
int rlpt_check(rlpt_ctx* ctx);

/* Capture the work of one segment of n_sweeps sweeps (sweeps, swaps,
 * recomputations, measurements) in a HIP graph and replay it n_segments
 * times.  n_sweeps must be a multiple of swap_interval, resync_interval and
 * measure_interval (those > 0) so that every replay performs the same work.
 * Async. */
int rlpt_run_graph(rlpt_ctx* ctx, int32_t n_sweeps, int32_t n_segments);

/* Sweep-kernel timing: while enabled, every sweep launch outside graph capture
 * is bracketed by HIP events on the context's stream.  rlpt_sweep_time_get
 * synchronises, returns the summed kernel time in ms and the number of
 * timed launches since the last reset, and resets the sums. */
int rlpt_sweep_timing(rlpt_ctx* ctx, int32_t enable);
int rlpt_sweep_time_get(rlpt_ctx* ctx, double* total_ms, int64_t* n_launches);

/* Roofline diagnostic of the streaming sweep (sec. III.A "Energy update
 * parallel computation": each two-mode update streams the lists of j and k).
 * Runs n_launches launches of a kernel with the sweep kernel's grid, items,
 * tile and LDS footprint that reads exactly the list chunks one sweep launch
 * reads (the next sweeps' pair draws, same threads, same order) and does
 * nothing else: no amplitudes, no arithmetic beyond a checksum, no
 * reductions or barriers between steps.  *ms_per_launch receives the mean
 * kernel time (HIP events on the context's stream): the time the memory
 * hierarchy needs to deliver one sweep's lists in this access pattern, the
 * ceiling of the sweep's list stream.  The chain, its counters and
 * accumulators are unchanged (the checksum goes to the context's scratch
 * buffer).  Synchronous.  FP32 contexts with chunked lists and streaming
 * fields only (RLPT_E_UNSUPPORTED otherwise); RLPT_E_STATE before rlpt_init. */
int rlpt_stream_lists(rlpt_ctx* ctx, int32_t n_launches, double* ms_per_launch);

/* ------------------------------------------------------------------------ */
/* Autotuning of the sweep kernel's launch tile (workgroup size, copies per  */
/* workgroup).  A process-wide registry holds measured times per sweep; when */
/* block_threads == 0 and copies_per_block == 0, rlpt_create takes, for the  */
/* context's mix of N, the workgroup size minimising the summed best times    */
/* and for each N the best copies per workgroup at that size (built-in       */
/* defaults for N without entries).                                          */
/* ------------------------------------------------------------------------ */
typedef struct rlpt_tile {
    int32_t n_modes;
    int32_t precision;        /* RLPT_FP32 / RLPT_FP64 */
    int32_t shared_pairs;     /* pair schedule */
    int32_t block_threads;    /* power of two in [64, 1024] */
    int32_t copies_per_block; /* 1 .. block_threads/64 */
    int32_t pad;
    double ms_per_sweep;      /* measured sweep-kernel time per sweep of the tuned context */
} rlpt_tile;

int rlpt_tune_clear(void);
int rlpt_tune_set(const rlpt_tile* tile);
/* Copy up to capacity entries to out (may be NULL); *count = entries held. */
int rlpt_tune_get(rlpt_tile* out, int32_t capacity, int32_t* count);
/* One JSON object per line, keyed by the device architecture (e.g. gfx950);
 * load skips entries recorded on another architecture. */
int rlpt_tune_save(const char* path);
int rlpt_tune_load(const char* path);

/* Measure tiles on one temporary context holding all graphs (cfg's ladder and
 * precision) in the caller's workspace (>= rlpt_workspace_size for all
 * graphs).  For each workgroup size the N classes are tuned in turn: every
 * copies-per-workgroup value of one N is timed on the whole launch (all N
 * together) with the other N at their current choice (built-in at first), and
 * the best is kept; sweeps_per_trial timed sweeps per tile after one warm-up
 * sweep; each trial is recorded in the registry under its N.
 * *n_trials (may be NULL) receives the number of tiles timed.  Synchronous. */
int rlpt_autotune(const rlpt_config* cfg, const rlpt_graph* const* graphs, int32_t n_graphs,
                  const double* temps, void* d_workspace, size_t workspace_bytes, void* hip_stream,
                  int32_t sweeps_per_trial, int32_t* n_trials);

/* The launch tile a context uses: workgroup size and, for sample mu, the
 * copies per workgroup (n_samples entries, may be NULL). */
int rlpt_tile_of(rlpt_ctx* ctx, int32_t* block_threads, int32_t* copies_per_block);

/* Counters. */
int rlpt_counters(rlpt_ctx* ctx, int64_t* sweeps_done, int64_t* swaps_done, int64_t* n_meas);

/* ------------------------------------------------------------------------ */
/* State access and test hooks (synchronous, host buffers).                  */
/* ------------------------------------------------------------------------ */

/* Amplitudes of n_copies copies starting at first_copy, each 2*N doubles
 * (interleaved re, im); all copies in the range must belong to samples of one N.
 * set_state converts to the context precision and sets every copy's running
 * energy to its FP64 recomputation (no drift check, no rescaling onto the
 * constraint: rlpt_resync does that). */
int rlpt_get_state(rlpt_ctx* ctx, int32_t first_copy, int32_t n_copies, double* a);
int rlpt_set_state(rlpt_ctx* ctx, int32_t first_copy, int32_t n_copies, const double* a);

/* Checkpoint and resume (host file I/O, synchronous).  rlpt_checkpoint_save
 * writes everything a run changes on the device: amplitudes, running and FP64
 * energies, drift, the temperature permutation of every ladder, the cached
 * fields (field_mode CACHED), all accumulators, histograms, series and
 * counters, plus the run seed and the sweep and swap counts.
 * rlpt_checkpoint_load restores them into a context created with the same
 * graphs, ladder and configuration (checked by a fingerprint; RLPT_E_ARG
 * otherwise, or for a truncated file), after which the run continues exactly
 * as the saved one would have: same draws, same decisions, same bits.  The
 * learned proposal's networks and training buffers are not included (use
 * rlpt_mlp_get_params / rlpt_mlp_set_params).  Errors: RLPT_E_ARG (I/O,
 * mismatch), RLPT_E_STATE (save before rlpt_init), RLPT_E_HIP. */
int rlpt_checkpoint_save(rlpt_ctx* ctx, const char* path);
int rlpt_checkpoint_load(rlpt_ctx* ctx, const char* path);

/* Running energies E[n_copies], temperature index of each copy temp_of[n_copies]. */
int rlpt_get_energies(rlpt_ctx* ctx, double* E, int32_t* temp_of);

/* FP64 energy of every copy (no state change). */
int rlpt_energy_fp64(rlpt_ctx* ctx, double* E);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * energy of every copy, as rlpt_energy_fp64 computes it (same kernels, same
 * summation order, the same bits), written to the caller's device array
 * d_E[n_copies], asynchronously on the context's stream, with no state
 * change.  It allocates nothing and copies nothing to or from the host: its
 * partial sums (8 per copy) live in a static device array of the library,
 * 2 MiB per GPU (at most 32768 copies; RLPT_E_ARG beyond), held until the
 * process ends.  Every call on one GPU uses that GPU's array: calls that
 * overlap on one GPU (contexts on different streams) race.  Errors: RLPT_E_ARG
 * (NULL, too many copies), RLPT_E_HIP (launch). */
int rlpt_energy_fp64_noalloc(rlpt_ctx* ctx, double* d_E);

/* Local fields F_l = sum over terms containing l of J conj(a_x) a_y a_z
 * (x: l's partner on its side of the term, (y, z): the other side) of one copy,
 * computed by the sweep kernel's own field code in the context precision.
 * F: 2*N doubles.  (Energy update of sec. III.A "Energy update parallel
 * computation".) */
int rlpt_local_fields(rlpt_ctx* ctx, int32_t copy, double* F);

/* Energy change of the two-mode update (a_j, a_k) -> (aj_new, ak_new) of one
 * copy, by the sweep kernel's code path: both fields on one snapshot holding
 * aj_new and the old a_k.  n pairs; j, k, aj_new (2n), ak_new (2n), dE (n). */
int rlpt_pair_dE(rlpt_ctx* ctx, int32_t copy, int32_t n, const int32_t* j, const int32_t* k,
                 const double* aj_new, const double* ak_new, double* dE);

/* ------------------------------------------------------------------------ */
/* Observables (sec. IV): accumulated since rlpt_init per sample mu and bath t */
/* ------------------------------------------------------------------------ */
typedef struct rlpt_obs {
    /* each array is caller-allocated; NULL skips it.  Shapes use S samples,
     * T baths, B bins, L series length. */
    double* e_n;     /* [S][T] number of energy samples (measurements x replicas) */
    double* e_sum;   /* [S][T] sum E */
    double* e_sq;    /* [S][T] sum E^2            -> C_V = (<E^2> - <E>^2)/T^2 (eq. SpecificHeat) */
    double* y2_sum;  /* [S][T] sum Y_2 ; Y_n = sum|a|^(2n) / (sum|a|^n)^2 */
    double* y4_sum;  /* [S][T] sum Y_4 */
    double* q_n;     /* [S][T] number of overlap samples (measurements x replica pairs) */
    double* q_sum;   /* [S][T] sum q ; q_cd = (1/N) Re sum conj(a^c) a^d */
    double* q_sq;    /* [S][T] */
    double* q_4;     /* [S][T] */
    double* hist;    /* [S][T][B] overlap histogram on [-1, 1] */
    double* acc;     /* [S][T] accepted two-mode moves */
    double* tries;   /* [S][T] proposed two-mode moves */
    double* swap_acc;   /* [S][T-1] accepted exchanges (summed over ladders) */
    double* swap_tries; /* [S][T-1] */
    double* series_e;   /* [S][T][L] energy of ladder 0's copy at bath t, per measurement */
    double* series_q;   /* [S][T][L] overlap of ladders 0 and 1 at bath t, per measurement */
    double* hist_I;     /* [S][T][B] total intensity I/N = sum|a|^2 / N on [0, 1] (P(I), sec. II.B) */
    double* spectrum;   /* [S][T][max N] sum over measurements and replicas of |a_k|^2, modes in   */
                        /* frequency order: divide by e_n for the intensity spectrum I(omega_k)  */
                        /* of sec. II.C (Fig. spectrum); rows of samples with smaller N are      */
                        /* zero beyond their N                                                   */
} rlpt_obs;

/* Copy the accumulators to host (synchronises).  Returns RLPT_E_STATE if a
 * drift / NaN failure was recorded. */
int rlpt_observables(rlpt_ctx* ctx, rlpt_obs* out);

/* ------------------------------------------------------------------------ */
/* Learned global proposal (not in the paper; the method's moves stay as they  */
/* are and keep running every sweep).  Coordinates on sum|a|^4 = N: w =      */
/* |a|^4/N, y = log(w_k/w_{N-1}) (k < N-1), phases psi.  A network per        */
/* temperature slot maps Re/Im of a (rotated so a_0 is real positive) through  */
/* two SiLU layers to a K-component diagonal Gaussian mixture over (dy, dpsi); */
/* widths 2*sigmoid (y) and (pi/2)*sigmoid (psi), all scaled by step_scale;    */
/* phases wrap.  Exact Metropolis-Hastings with the reference density          */
/* prod w^(1/2) in (y, psi) (the flat measure of eq. ProbDistr).  Every matrix */
/* product runs on the matrix cores with bfloat16 operands (weights; inputs   */
/* rounded to nearest even) and FP32 accumulation; FP32 master weights;       */
/* training is Adam on the mean negative log-likelihood of harvested          */
/* displacements.  The harvest runs without swaps: sweep with swaps on again  */
/* before measuring.                                                          */
/* Random numbers: Philox keyed (run_seed, "LEARN") at (i, round, copy, 0).   */
/* The chart (y, psi) covers configurations with every a_k != 0 only: a move  */
/* from a configuration with a zero (or non-finite) amplitude, or to a        */
/* proposal whose intensity underflowed to zero, is rejected (log acceptance  */
/* ratio -inf); training pairs with a zero or non-finite amplitude in either  */
/* configuration are left out of the minibatch mean.                          */
/* ------------------------------------------------------------------------ */

/* Initialise weights (seeded), Adam moments and counters; temp_index[mlp_nets]
 * gives each network's temperature slot. */
int rlpt_mlp_setup(rlpt_ctx* ctx, const int32_t* temp_index, uint64_t seed);
/* Parameters per network (W1 [2N][H], b1, W2 [H][H], b2, W3 [H][Out], b3,
 * row-major, concatenated) and outputs per configuration. */
int rlpt_mlp_n_params(rlpt_ctx* ctx, int64_t* n_params, int32_t* n_outputs);
int rlpt_mlp_set_params(rlpt_ctx* ctx, int32_t net, const float* params);
int rlpt_mlp_get_params(rlpt_ctx* ctx, int32_t net, float* params);
/* Store n explicit training pairs (interleaved complex, [n][N] each) for one network. */
int rlpt_mlp_set_pairs(rlpt_ctx* ctx, int32_t net, int32_t n, const double* before, const double* after);
/* rounds x (record the copies at each network's temperature, `lag` sweeps
 * without swaps, record the same copies again).  Async-safe: synchronises. */
int rlpt_mlp_harvest(rlpt_ctx* ctx, int32_t rounds, int32_t lag);
/* Adam steps (lr) on random minibatches; mean_loss[mlp_nets] (may be NULL)
 * receives each network's loss on the last step's minibatch, averaged over its
 * pairs inside the chart.  Synchronises.  RLPT_E_STATE when a network's last
 * loss is not finite or its last minibatch held no pair inside the chart
 * (mean_loss is filled first; NaN for the latter). */
int rlpt_mlp_train(rlpt_ctx* ctx, int32_t steps, double lr, double* mean_loss);
/* Test hooks: outputs of network `net` on the first n stored "before"
 * configurations (the training forward: three matrix-core GEMMs of n <=
 * mlp_batch rows); loss (mean over the pairs inside the chart; RLPT_E_STATE if
 * none) and gradient on the first mlp_batch stored pairs. */
int rlpt_mlp_forward(rlpt_ctx* ctx, int32_t net, int32_t n, double* out);
int rlpt_mlp_loss_grad(rlpt_ctx* ctx, int32_t net, double* loss, float* grad);
/* Test hook: the inference forward that learned rounds run (one fused launch
 * that also forms the features when samples x replicas <= 16, 2N and
 * mlp_hidden are multiples of 128 and the outputs fit 16 tiles of 256 columns;
 * the feature kernel and three GEMMs otherwise) of network `net` on
 * n <= samples x replicas caller
 * configurations states[n][N] (interleaved complex doubles, converted to
 * FP32); out[n][outputs].  Uses the network's inference buffers (outputs at
 * the current configurations of the last learned round are overwritten).
 * Synchronous.  Errors: RLPT_E_ARG, RLPT_E_STATE (no rlpt_mlp_setup). */
int rlpt_mlp_infer(rlpt_ctx* ctx, int32_t net, int32_t n, const double* states, double* out);
/* Subset move (mlp_subset = m >= 2): per move, S = m distinct modes from a
 * partial Fisher-Yates shuffle of 0..N-1 (step t swaps position t with
 * t + floor(hi32(word_t) (N - t) / 2^32)), sorted ascending; chart u_i =
 * log(w_{s_i} / w_{s_m}) (i < m) and the phases of S, the sum of w over S
 * fixed; the displacement of u_i uses the y channel of mode s_i, that of
 * psi_{s_i} its phase channel; reference ratio prod_S (w'/w)^(1/2).  Draws:
 * Philox (run_seed, "LEARN") at (i, round, copy, 1): blocks i < m Gaussians
 * (2 per block), block m the component and acceptance uniforms, blocks
 * m + 1 + t/4 word t%4 the shuffle.  Training draws the subset of minibatch
 * item b at step s from Philox (setup seed, "TRAIN") at (s, net, b, 1 + t/4)
 * word t%4 and fits the displacement in its chart. */
/* Learned rounds after every sweep (0 = off) with the given step scale in (0, 1]. */
int rlpt_mlp_enable(rlpt_ctx* ctx, int32_t moves_per_sweep, double step_scale);
/* One learned round of every network now (async). */
int rlpt_mlp_move(rlpt_ctx* ctx, double step_scale);
/* Accepted and proposed learned moves per network. */
int rlpt_mlp_stats(rlpt_ctx* ctx, double* acc, double* tries);
/* Last round of network `net`: log acceptance ratio [S*reps], copies [S*reps],
 * proposals [S*reps][N] interleaved complex (each may be NULL). */
int rlpt_mlp_last_move(rlpt_ctx* ctx, int32_t net, double* log_alpha, int32_t* copies, double* proposal);

/* ------------------------------------------------------------------------ */
/* Analysis helpers (host).                                                  */
/* ------------------------------------------------------------------------ */

/* Per-temperature disorder averages over S samples of the accumulators of
 * rlpt_observables (sec. III.B eq. DisAver; errors: jackknife over samples):
 * <E>; specific heat per spin C_V/N = avg((<E^2> - <E>^2)/T^2)/N (eq.
 * SpecificHeat); <q^2>; kurtosis K = avg<q^4>/(avg(<q^2> - <q>^2))^2 (eq. kurt,
 * with the disorder-averaged mean overlap taken as 0 by the symmetry q -> -q);
 * IPR <Y_2>, <Y_4>; pair-move acceptance per temperature and swap acceptance
 * per neighbouring pair.  Each output array has T entries (T-1 for swap_rate);
 * NULL skips it. */
typedef struct rlpt_summary {
    double *E, *E_err, *cv, *cv_err, *q2, *q2_err, *kurtosis, *kurtosis_err;
    double *y2, *y2_err, *y4, *y4_err, *acc_rate, *swap_rate;
} rlpt_summary;
int rlpt_summarize(const rlpt_obs* obs, int32_t n_samples, int32_t n_temps, int32_t n_modes, const double* temps,
                   rlpt_summary* out);

/* Temperature ladder with spacing adapted to the specific heat (App. A, eq.
 * PT_Ti): T_0 = T_min, T_i = T_{i-1} / (1 - C / sqrt(C_V(T_i))), solved for T_i
 * by fixed-point iteration with C_V linearly interpolated on (T_grid, C_grid)
 * (extensive specific heat, C_grid > C^2), while T_i < T_max.  Writes at most
 * capacity temperatures; *n_out receives the count. */
int rlpt_adaptive_ladder(const double* T_grid, const double* C_grid, int32_t n_grid, double T_min, double T_max,
                         double C, double* temps, int32_t capacity, int32_t* n_out);

/* Means of x over the doubling windows [0,1), [1,2), [2,4), [4,8), ... (clipped
 * to n), the thermalisation check of sec. III.B; starts may be NULL. */
int rlpt_window_means(const double* x, int64_t n, double* means, int64_t* starts, int32_t capacity,
                      int32_t* n_windows);

/* Integrated autocorrelation time of a series x[n] with Sokal's automatic
 * window: tau(W) = 1/2 + sum_{t=1..W} rho(t), smallest W >= c_window*tau(W).
 * *tau receives tau_int, *window the chosen W. */
int rlpt_tau_int(const double* x, int64_t n, double c_window, double* tau, int64_t* window);

#ifdef __cplusplus
}
#endif

#endif /* RLPT_H */
