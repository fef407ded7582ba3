// C-ABI runtime of librlpt: contexts over a caller-owned workspace, the
// sweep / swap / recomputation / measurement schedule of parallel tempering
// (sec. III.A and sec. III.B of Benedetti & Leuzzi, arXiv 2511.13508), HIP
// graph replay of whole segments, observables read-back and host analysis.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "context.hpp"

namespace rlpt {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

static int hip_fail(hipError_t e, const char* what) {
    return fail(RLPT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                           \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Built-in launch tile of the sweep kernel for a sample of N modes: threads
// per workgroup and copies per workgroup (each copy gets (block/64)/copies
// waves).  Entries streamed per two-mode step ~ 2 * 4c/N ~ 2N^2/3; small N
// packs several copies (one wave each) into a workgroup.
struct Tile {
    int block;
    int copies;
};

static Tile default_tile(int N) {
    if (N >= 192) return {256, 1};
    if (N >= 96) return {256, 2};
    return {256, 4};
}

// Few copies for the chip: a copy's sweep is a chain of dependent two-mode
// steps, so with fewer than two workgroups per compute unit the launch is
// bound by a step's latency. Spread the copies first (fewer per workgroup),
// then give each copy more waves (a step's list is cut into shorter pieces).
static void spread_tile(const std::map<int, int>& counts, int copies_per_sample, int block_max, int* block,
                        std::map<int, int>* copies) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    auto n_blocks = [&]() {
        int64_t n = 0;
        for (const auto& nc : counts) {
            const int cpw = std::max(1, std::min((*copies)[nc.first], *block / 64));
            n += (int64_t)nc.second * ((copies_per_sample + cpw - 1) / cpw);
        }
        return n;
    };
    while (n_blocks() < 2 * (int64_t)cus) {
        bool halved = false;
        for (auto& kv : *copies)
            if (kv.second > 1) {
                kv.second /= 2;
                halved = true;
            }
        if (!halved) break;
    }
    if (n_blocks() < 2 * (int64_t)cus && *block < block_max) *block = block_max;
}

// cached-field sweep: one copy per workgroup, two waves per 64-target slice
// (an accepted move streams its gather blocks with twice the loads in flight)
static Tile default_tile_cached(int N) {
    const int ns = (N + 63) / 64;
    return {std::min(512, 128 * ns), 1};
}

}  // namespace rlpt

using namespace rlpt;


namespace {

// byte layout of a workspace; also used to size it
struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

struct Regions {
    size_t samples, items, mode_start, idx, J, chunk_start, cx, cyz, cJ, pair_start, pidx, pJ, fields, ell_start, gidx16, gidx32, gJ, c0, quads, Jq, amp, E, E64, drift, temp_of, copy_at, beta, beta64;
    size_t acc_begin, acc, swap_acc, obs, hist, hist_I, spec, series_e, series_q, meas_cnt, counters, acc_end;
    size_t scratch, scratch_doubles, rs_part, mlp, total;
};

int check_config(const rlpt_config* cfg) {
    if (!cfg) return fail(RLPT_E_ARG, "config is NULL");
    if (cfg->n_temps < 1 || cfg->n_reps < 1) return fail(RLPT_E_ARG, "n_temps and n_reps must be >= 1");
    if (cfg->precision != RLPT_FP32 && cfg->precision != RLPT_FP64) return fail(RLPT_E_ARG, "bad precision");
    if (cfg->swap_interval < 1) return fail(RLPT_E_ARG, "swap_interval must be >= 1");
    if (cfg->resync_interval < 0 || cfg->measure_interval < 0) return fail(RLPT_E_ARG, "negative interval");
    if (cfg->n_bins < 1) return fail(RLPT_E_ARG, "n_bins must be >= 1");
    if (cfg->series_len < 0) return fail(RLPT_E_ARG, "series_len must be >= 0");
    if (cfg->block_threads != 0 && (cfg->block_threads < 64 || cfg->block_threads > 1024 ||
                                    (cfg->block_threads & (cfg->block_threads - 1))))
        return fail(RLPT_E_ARG, "block_threads must be 0 or a power of two in [64, 1024]");
    if (cfg->copies_per_block < 0) return fail(RLPT_E_ARG, "copies_per_block must be >= 0");
    if (cfg->list_layout < RLPT_LAYOUT_AUTO || cfg->list_layout > RLPT_LAYOUT_CHUNKED)
        return fail(RLPT_E_ARG, "bad list_layout");
    if (cfg->mlp_nets < 0) return fail(RLPT_E_ARG, "mlp_nets must be >= 0");
    if (cfg->field_mode != RLPT_FIELDS_STREAM && cfg->field_mode != RLPT_FIELDS_CACHED)
        return fail(RLPT_E_ARG, "bad field_mode");
    if (cfg->rho != 0 && cfg->rho != 2 && cfg->rho != 4) return fail(RLPT_E_ARG, "rho must be 4 or 2");
    if (cfg->rho == 2 && cfg->mlp_nets > 0)
        return fail(RLPT_E_UNSUPPORTED, "learned moves work on the rho = 4 constraint only");
    return RLPT_OK;
}

// list layout of a context: chunked needs N <= 256 everywhere; the automatic
// choice also avoids it for small N and sparse graphs, where padding partner
// groups to 4 entries inflates the lists
int choose_layout(const rlpt_config& cfg, const rlpt_graph* const* g, int S, int* layout) {
    int max_N = 0, min_N = 1 << 30;
    for (int i = 0; i < S; ++i) {
        max_N = std::max(max_N, g[i]->N);
        min_N = std::min(min_N, g[i]->N);
    }
    if (cfg.list_layout == RLPT_LAYOUT_PACKED) *layout = kLayoutPacked;
    else if (cfg.list_layout == RLPT_LAYOUT_CHUNKED) {
        if (max_N > kMaxChunkModes) return fail(RLPT_E_ARG, "the chunked list layout needs N <= 256");
        *layout = kLayoutChunked;
    } else {
        // chunked pays when partner groups are long: dense graphs, not sparse ones,
        // whose groups of about one entry would be padded to four
        size_t chunk_entries = 0, list_entries = 0;
        for (int i = 0; i < S; ++i) {
            chunk_entries += 4 * g[i]->cx.size();
            list_entries += g[i]->mode_start.back();
        }
        const bool dense = 4 * chunk_entries <= 5 * list_entries;
        *layout = (max_N <= kMaxChunkModes && min_N >= 32 && dense) ? kLayoutChunked : kLayoutPacked;
    }
    return RLPT_OK;
}

// cached-field tables of one sample (appended to the vectors):
//  * pair lists for the energy change: for the ordered pair (j -> k), every
//    entry of k's list whose term also holds j, tagged with the slot j takes
//    in it (0: partner x, 1: y, 2: z);
//  * the sliced-ELL gather block for the field update on acceptance.
// Returns false when an index overflows 32 bits.
bool build_cached_tables(const rlpt_graph* g, int layout, std::vector<uint32_t>* pstart, std::vector<uint32_t>* pidx,
                         std::vector<double>* pJ, std::vector<uint32_t>* estart, std::vector<uint16_t>* g16,
                         std::vector<uint32_t>* g32, std::vector<double>* gJ, std::vector<uint16_t>* c0tab) {
    const int N = g->N, ns = (N + kSlice - 1) / kSlice;
    const int64_t c = g->n_terms();
    std::vector<uint32_t> cnt, c0;
    pair_counts(g, &cnt, &c0);
    const uint64_t pbase = pidx->size();
    const uint64_t gbase = gJ->size();
    const size_t E = ell_entries(g, cnt);
    if (pbase + 12 * (uint64_t)c > 0xffffffffull || gbase + E > 0xffffffffull) return false;
    // pair lists
    std::vector<uint32_t> cur((size_t)N * N);
    const size_t s0 = pstart->size();
    pstart->resize(s0 + (size_t)N * N + 1);
    uint32_t run = (uint32_t)pbase;
    for (size_t p = 0; p < (size_t)N * N; ++p) {
        (*pstart)[s0 + p] = run;
        cur[p] = run;
        run += cnt[p];
    }
    (*pstart)[s0 + (size_t)N * N] = run;
    pidx->resize(run);
    pJ->resize(run);
    for (int64_t e = 0; e < c; ++e) {
        const int16_t* q = &g->quads[4 * e];
        for (int t = 0; t < 4; ++t) {
            int x[3];
            term_triple(q, t, x);
            const uint32_t v = (uint32_t)x[0] | (uint32_t)x[1] << 10 | (uint32_t)x[2] << 20;
            for (int r = 0; r < 3; ++r) {
                const uint32_t at = cur[(size_t)x[r] * N + q[t]]++;
                (*pidx)[at] = v | (uint32_t)r << 30;
                (*pJ)[at] = g->J[e];
            }
        }
    }
    // gather blocks: entry offsets per (j, s)
    const size_t e0 = estart->size();
    estart->resize(e0 + (size_t)N * ns + 1);
    std::vector<uint64_t> blk((size_t)N * ns);
    uint64_t off = gbase;
    for (int j = 0; j < N; ++j)
        for (int s = 0; s < ns; ++s) {
            const int w = std::min(kSlice, N - kSlice * s);
            uint32_t L = 0;
            for (int i = 0; i < w; ++i) L = std::max(L, cnt[(size_t)j * N + kSlice * s + i]);
            blk[(size_t)j * ns + s] = off;
            (*estart)[e0 + (size_t)j * ns + s] = (uint32_t)off;
            off += (uint64_t)((L + 3) / 4) * 4 * w;
        }
    (*estart)[e0 + (size_t)N * ns] = (uint32_t)off;
    const bool narrow = layout == kLayoutChunked;
    if (narrow) g16->resize(off, 0);
    else g32->resize(off, 0);
    gJ->resize(off, 0.0);
    // rank cursors: partner entries first, then the others
    std::vector<uint32_t> r0((size_t)N * N, 0), r1(c0);
    for (int64_t e = 0; e < c; ++e) {
        const int16_t* q = &g->quads[4 * e];
        for (int t = 0; t < 4; ++t) {
            const int l = q[t];
            int x[3];
            term_triple(q, t, x);
            for (int r = 0; r < 3; ++r) {
                const int j = x[r];
                // r = 0: j is l's partner, change conj(d) a_y a_z; else conj(a_x) d a_(other side)
                const int p1 = r == 0 ? x[1] : x[0];
                const int p2 = r == 0 ? x[2] : (r == 1 ? x[2] : x[1]);
                const size_t jl = (size_t)j * N + l;
                const uint32_t rank = r == 0 ? r0[jl]++ : r1[jl]++;
                const int s = l / kSlice, lane = l % kSlice, w = std::min(kSlice, N - kSlice * s);
                const uint64_t at = blk[(size_t)j * ns + s] + ((uint64_t)(rank / 4) * w + lane) * 4 + rank % 4;
                if (narrow) (*g16)[at] = (uint16_t)(p1 | p2 << 8);
                else (*g32)[at] = (uint32_t)p1 | (uint32_t)p2 << 10;
                (*gJ)[at] = g->J[e];
            }
        }
    }
    const size_t cb = c0tab->size();
    c0tab->resize(cb + (size_t)N * N);
    for (size_t p = 0; p < (size_t)N * N; ++p) (*c0tab)[cb + p] = (uint16_t)c0[p];
    return true;
}

int check_graphs(const rlpt_graph* const* g, int n) {
    if (!g || n < 1) return fail(RLPT_E_ARG, "need at least one graph");
    for (int i = 0; i < n; ++i)
        if (!g[i]) return fail(RLPT_E_ARG, "graph pointer is NULL");
    return RLPT_OK;
}

Regions plan(const rlpt_config& cfg, const rlpt_graph* const* g, int S, int layout) {
    const size_t rb = cfg.precision == RLPT_FP64 ? 8 : 4;
    const size_t T = cfg.n_temps, reps = cfg.n_reps, Rc = T * reps, copies = Rc * S;
    const bool cached = cfg.field_mode == RLPT_FIELDS_CACHED;
    size_t modes = 0, entries = 0, chunks = 0, quads = 0, amp = 0, pairs = 0, pair_entries = 0;
    size_t ell_starts = 0, ell_total = 0, c0n = 0;
    int max_N = 0;
    for (int i = 0; i < S; ++i) {
        modes += g[i]->N + 1;
        pairs += (size_t)g[i]->N * g[i]->N + 1;
        pair_entries += 12 * (size_t)g[i]->n_terms();
        if (cached) {
            std::vector<uint32_t> cnt;
            pair_counts(g[i], &cnt, nullptr);
            ell_total += ell_entries(g[i], cnt);
            ell_starts += (size_t)g[i]->N * ((g[i]->N + kSlice - 1) / kSlice) + 1;
            c0n += (size_t)g[i]->N * g[i]->N;
        }
        if (layout == kLayoutPacked) entries += g[i]->mode_start.back();
        else chunks += g[i]->cx.size();
        quads += g[i]->n_terms();
        amp += Rc * g[i]->N;
        max_N = std::max(max_N, g[i]->N);
    }
    Layout L;
    Regions r{};
    r.samples = L.take(S * sizeof(SampleDev));
    r.items = L.take(copies * sizeof(ItemDev));
    r.mode_start = L.take(modes * 4);
    r.idx = L.take(entries * 4);
    r.J = L.take(entries * rb);
    r.chunk_start = L.take(layout == kLayoutChunked ? modes * 4 : 0);
    r.cx = L.take(chunks);
    r.cyz = L.take(chunks * 8);
    r.cJ = L.take(chunks * 4 * rb);
    r.pair_start = L.take(cached ? pairs * 4 : 0);
    r.pidx = L.take(cached ? pair_entries * 4 : 0);
    r.pJ = L.take(cached ? pair_entries * rb : 0);
    r.fields = L.take(cached ? amp * 2 * rb : 0);
    r.ell_start = L.take(ell_starts * 4);
    r.gidx16 = L.take(layout == kLayoutChunked ? ell_total * 2 : 0);
    r.gidx32 = L.take(layout == kLayoutChunked ? 0 : ell_total * 4);
    r.gJ = L.take(ell_total * rb);
    r.c0 = L.take(c0n * 2);
    r.quads = L.take(quads * 8);
    r.Jq = L.take(quads * 8);
    r.amp = L.take(amp * 2 * rb);
    r.E = L.take(copies * rb);
    r.E64 = L.take(copies * 8);
    r.drift = L.take(copies * 8);
    r.temp_of = L.take(copies * 4);
    r.copy_at = L.take(S * reps * T * 4);
    r.beta = L.take(T * rb);
    r.beta64 = L.take(T * 8);
    r.acc_begin = L.off;
    r.acc = L.take(S * T * 8);
    r.swap_acc = L.take(S * reps * std::max<size_t>(T - 1, 1) * 8);
    r.obs = L.take(kNumObs * S * T * 8);
    r.hist = L.take(S * T * cfg.n_bins * 8);
    r.hist_I = L.take(S * T * cfg.n_bins * 8);
    r.spec = L.take(S * T * (size_t)max_N * 8);
    r.series_e = L.take(S * T * std::max(cfg.series_len, 1) * 8);
    r.series_q = L.take(S * T * std::max(cfg.series_len, 1) * 8);
    r.meas_cnt = L.take(S * T * 4);
    r.counters = L.take(sizeof(Counters));
    r.acc_end = L.off;
    r.scratch_doubles = std::max<size_t>(2 * amp, 8192);
    r.scratch = L.take(r.scratch_doubles * 8);
    r.rs_part = L.take(copies * kResyncParts * 8);
    r.mlp = L.off;
    L.off = mlp_layout(cfg, g[0]->N, S, nullptr, nullptr, L.off);
    r.total = L.off;
    return r;
}

template <typename R>
void fill_ptrs(DevPtrs<R>& P, unsigned char* b, const Regions& r) {
    P.samples = reinterpret_cast<const SampleDev*>(b + r.samples);
    P.items = reinterpret_cast<const ItemDev*>(b + r.items);
    P.mode_start = reinterpret_cast<const uint32_t*>(b + r.mode_start);
    P.idx = reinterpret_cast<const uint32_t*>(b + r.idx);
    P.J = reinterpret_cast<const R*>(b + r.J);
    P.chunk_start = reinterpret_cast<const uint32_t*>(b + r.chunk_start);
    P.cx = reinterpret_cast<const uint8_t*>(b + r.cx);
    P.cyz = reinterpret_cast<const uint2*>(b + r.cyz);
    P.cJ = reinterpret_cast<const R*>(b + r.cJ);
    P.pair_start = reinterpret_cast<const uint32_t*>(b + r.pair_start);
    P.pidx = reinterpret_cast<const uint32_t*>(b + r.pidx);
    P.pJ = reinterpret_cast<const R*>(b + r.pJ);
    P.fields = reinterpret_cast<R*>(b + r.fields);
    P.ell_start = reinterpret_cast<const uint32_t*>(b + r.ell_start);
    P.gidx16 = reinterpret_cast<const uint16_t*>(b + r.gidx16);
    P.gidx32 = reinterpret_cast<const uint32_t*>(b + r.gidx32);
    P.gJ = reinterpret_cast<const R*>(b + r.gJ);
    P.c0 = reinterpret_cast<const uint16_t*>(b + r.c0);
    P.quads = reinterpret_cast<const ushort4*>(b + r.quads);
    P.Jq = reinterpret_cast<const double*>(b + r.Jq);
    P.amp = reinterpret_cast<R*>(b + r.amp);
    P.E = reinterpret_cast<R*>(b + r.E);
    P.E64 = reinterpret_cast<double*>(b + r.E64);
    P.drift = reinterpret_cast<double*>(b + r.drift);
    P.temp_of = reinterpret_cast<int32_t*>(b + r.temp_of);
    P.copy_at = reinterpret_cast<int32_t*>(b + r.copy_at);
    P.beta = reinterpret_cast<const R*>(b + r.beta);
    P.beta64 = reinterpret_cast<const double*>(b + r.beta64);
    P.acc = reinterpret_cast<unsigned long long*>(b + r.acc);
    P.swap_acc = reinterpret_cast<unsigned long long*>(b + r.swap_acc);
    P.obs = reinterpret_cast<double*>(b + r.obs);
    P.hist = reinterpret_cast<double*>(b + r.hist);
    P.hist_I = reinterpret_cast<double*>(b + r.hist_I);
    P.spec = reinterpret_cast<double*>(b + r.spec);
    P.series_e = reinterpret_cast<double*>(b + r.series_e);
    P.series_q = reinterpret_cast<double*>(b + r.series_q);
    P.meas_cnt = reinterpret_cast<int32_t*>(b + r.meas_cnt);
    P.counters = reinterpret_cast<Counters*>(b + r.counters);
    P.rs_part = reinterpret_cast<double*>(b + r.rs_part);
}

template <typename T>
hipError_t upload(unsigned char* base, size_t off, const std::vector<T>& v, hipStream_t st) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

Counters* counters_of(rlpt_ctx* c) { return c->cfg.precision == RLPT_FP64 ? c->pd.counters : c->pf.counters; }

bool measuring_at(const rlpt_ctx* c, int64_t n) {
    return n > c->cfg.measure_start && c->cfg.measure_interval > 0 && n % c->cfg.measure_interval == 0;
}

// cached-field mode: recompute every copy's fields from its amplitudes
int refresh_fields(rlpt_ctx* c) {
    if (!c->sh.cached) return RLPT_OK;
    HIP_TRY(launch_fields_all(c->cfg.precision, c->ptrs(), c->sh, c->n_copies, c->stream), "fields launch");
    return RLPT_OK;
}

// enqueue n sweeps starting after `done` completed sweeps (no host mirror update)
int enqueue_sweeps(rlpt_ctx* c, int64_t done, int64_t n, int64_t* swaps_added) {
    const rlpt_config& cfg = c->cfg;
    int64_t k = 0;
    *swaps_added = 0;
    while (k < n) {
        const int64_t cur = done + k;
        // sweeps until the next event boundary
        int64_t step = n - k;
        const int iv[3] = {cfg.swap_interval, cfg.resync_interval, cfg.measure_interval};
        for (int i = 0; i < 3; ++i)
            if (iv[i] > 0) step = std::min<int64_t>(step, iv[i] - cur % iv[i]);
        if (c->mlp_moves > 0) step = 1;  // learned rounds follow every sweep
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        if (c->timing && !c->capturing) {
            if (!c->spare.empty()) {
                ev = c->spare.back();
                c->spare.pop_back();
            } else {
                HIP_TRY(hipEventCreate(&ev.first), "event create");
                HIP_TRY(hipEventCreate(&ev.second), "event create");
            }
            HIP_TRY(hipEventRecord(ev.first, c->stream), "event record");
        }
        HIP_TRY(launch_sweep(cfg.precision, c->ptrs(), c->sh, c->launch, (int)step, c->stream), "sweep launch");
        if (ev.first) {
            HIP_TRY(hipEventRecord(ev.second, c->stream), "event record");
            c->events.push_back(ev);
        }
        for (int m = 0; m < c->mlp_moves; ++m) {
            int rc = mlp_enqueue_round(c);
            if (rc) return rc;
        }
        const int64_t after = cur + step;
        const bool swap = c->T > 1 && after % cfg.swap_interval == 0;
        if (swap) HIP_TRY(launch_swap(cfg.precision, c->ptrs(), c->sh, c->stream), "swap launch");
        HIP_TRY(launch_tick(c->ptrs(), cfg.precision, step, swap ? 1 : 0, c->stream), "tick launch");
        if (swap) *swaps_added += 1;
        if (cfg.resync_interval > 0 && after % cfg.resync_interval == 0) {
            HIP_TRY(launch_resync(cfg.precision, c->ptrs(), c->sh, c->n_copies, 0, c->stream), "resync launch");
            int rc = refresh_fields(c);
            if (rc) return rc;
        }
        if (measuring_at(c, after)) HIP_TRY(launch_measure(cfg.precision, c->ptrs(), c->sh, c->stream), "measure launch");
        k += step;
    }
    return RLPT_OK;
}

int sync_and_flags(rlpt_ctx* c) {
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    Counters h{};
    HIP_TRY(hipMemcpy(&h, counters_of(c), sizeof(Counters), hipMemcpyDeviceToHost), "read counters");
    if (h.error_flags & 2) return fail(RLPT_E_STATE, "non-finite energy or amplitude found at a recomputation");
    if (h.error_flags & 1) return fail(RLPT_E_STATE, "running energy drifted beyond drift_tol");
    return RLPT_OK;
}

// work items: samples ordered by decreasing N (longest work first), copies in
// chunks of the tile's copies per workgroup; sets the launch description.
// Cached-field contexts name temperature slots instead, hottest first (the
// copies with the most accepted moves, hence field updates, start first); the
// kernel finds each slot's copy in copy_at.
int build_items(rlpt_ctx* c, int block, const std::map<int, int>& copies) {
    if (block < 64 || block > 1024 || (block & (block - 1))) return fail(RLPT_E_ARG, "bad workgroup size");
    std::vector<ItemDev> items;
    int max_cpi = 1;
    std::vector<int> order(c->S);
    for (int s = 0; s < c->S; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b2) { return c->N[a] > c->N[b2]; });
    // every copy group is sized for the largest N of the context: cap the copies
    // per workgroup so that the groups fit in 64 KiB of LDS
    const size_t per_copy = sweep_lds_bytes(c->cfg.precision, block, 1, c->max_N, c->sh.cached, c->sh.short_lists);
    const int lds_cap = (int)std::max<size_t>(1, (64 * 1024) / per_copy);
    for (int s : order) {
        auto it_c = copies.find(c->N[s]);
        int cpw = it_c == copies.end() ? 1 : it_c->second;
        cpw = std::max(1, std::min({cpw, block / 64, lds_cap}));
        if (c->sh.short_lists) cpw = std::min(block / 64, lds_cap);  // one wave per copy
        for (int first = 0; first < c->Rc; first += cpw) {
            ItemDev it{};
            it.first_copy = s * c->Rc + first;
            it.n_copies = std::min(cpw, c->Rc - first);
            it.sample = s;
            items.push_back(it);
            max_cpi = std::max(max_cpi, it.n_copies);
        }
    }
    if (c->sh.cached) {  // hottest slots first across samples (stable: sample order within a rank)
        std::stable_sort(items.begin(), items.end(), [&](const ItemDev& x, const ItemDev& y) {
            return x.first_copy - x.sample * c->Rc < y.first_copy - y.sample * c->Rc;
        });
    } else {
        // within each N class (classes stay in decreasing N), deal the samples'
        // items round robin.  Workgroups go to the eight XCDs in turn, so an XCD
        // then holds the copies of few samples and its L2 sees only their lists
        // (eight samples of one N: one sample per XCD)
        std::vector<ItemDev> rr;
        rr.reserve(items.size());
        size_t b = 0;
        while (b < items.size()) {
            const int n_cls = c->N[items[b].sample];
            size_t e = b;
            while (e < items.size() && c->N[items[e].sample] == n_cls) ++e;
            // [b, e): the class's samples in turn, each with the same item count (same N, same tile)
            std::vector<size_t> start;
            for (size_t i = b; i < e; ++i)
                if (i == b || items[i].sample != items[i - 1].sample) start.push_back(i);
            const size_t per = (e - b) / start.size();
            for (size_t k = 0; k < per; ++k)
                for (size_t st = 0; st < start.size(); ++st) rr.push_back(items[start[st] + k]);
            b = e;
        }
        items.swap(rr);
    }
    const size_t lds = sweep_lds_bytes(c->cfg.precision, block, max_cpi, c->max_N, c->sh.cached, c->sh.short_lists);
    if (lds > 64 * 1024) return fail(RLPT_E_ARG, "sweep tile needs more than 64 KiB of LDS; use fewer copies per block");
    // streaming sweep over chunked lists: hold a step's chunks in registers
    // ahead when every list of the launch fits 1, 2 or 4 chunks per thread; if
    // they still fit with each list on half of a copy's waves, split the lists
    // that way (a wave then reduces two values per step instead of four)
    int prefetch = 0, split = 0;
    if (c->sh.layout == kLayoutChunked && !c->sh.cached && !c->sh.short_lists && (block == 256 || block == 512)) {
        auto pf = [](uint32_t need) { return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 0; };
        uint32_t need = 0, need_half = 0;
        bool halves = true;
        for (const ItemDev& it : items) {
            const uint32_t wpc = (uint32_t)(block / 64 / it.n_copies), nt = wpc * 64;
            need = std::max(need, (c->max_chunks[it.sample] + nt - 1) / nt);
            if (wpc >= 2)
                need_half = std::max(need_half, (c->max_chunks[it.sample] + nt / 2 - 1) / (nt / 2));
            else
                halves = false;
        }
        if (halves && pf(need_half) > 0) {
            prefetch = pf(need_half);
            split = 1;
        } else {
            prefetch = pf(need);
        }
    }
    c->items = items;
    c->tile_copies = copies;
    c->launch.block_threads = block;
    c->launch.n_items = (int)items.size();
    c->launch.max_copies_per_item = max_cpi;
    c->launch.max_N = c->max_N;
    c->launch.prefetch = prefetch;
    c->launch.split = split;
    c->launch.lds_bytes = lds;
    c->sh.by_slot = c->sh.cached;
    return RLPT_OK;
}

int upload_items(rlpt_ctx* c) {
    ItemDev* d = const_cast<ItemDev*>(c->cfg.precision == RLPT_FP64 ? c->pd.items : c->pf.items);
    HIP_TRY(hipMemcpyAsync(d, c->items.data(), c->items.size() * sizeof(ItemDev), hipMemcpyHostToDevice, c->stream),
            "upload items");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    return RLPT_OK;
}

void drop_events(rlpt_ctx* c) {
    for (auto* v : {&c->events, &c->spare})
        for (auto& e : *v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    c->events.clear();
    c->spare.clear();
}

void drop_graph(rlpt_ctx* c) {
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    c->exec = nullptr;
    c->graph_sweeps = 0;
    c->graph_phase = -1;
}

}  // namespace

extern "C" {

int rlpt_abi_version(void) { return RLPT_ABI_VERSION; }

const char* rlpt_last_error(void) { return g_last_error.c_str(); }

int rlpt_config_default(rlpt_config* cfg) {
    if (!cfg) return fail(RLPT_E_ARG, "config is NULL");
    memset(cfg, 0, sizeof(*cfg));
    cfg->n_temps = 1;
    cfg->n_reps = 2;
    cfg->precision = RLPT_FP32;
    cfg->shared_pairs = 0;
    cfg->swap_interval = 1;
    cfg->resync_interval = 100;
    cfg->renorm_tol = 1e-6;
    cfg->drift_tol = 1e-3;
    cfg->measure_start = 0;
    cfg->measure_interval = 1;
    cfg->n_bins = 100;
    cfg->series_len = 0;
    cfg->list_layout = RLPT_LAYOUT_AUTO;
    cfg->mlp_nets = 0;
    cfg->mlp_hidden = 256;
    cfg->mlp_components = 4;
    cfg->mlp_capacity = 100000;
    cfg->mlp_batch = 512;
    cfg->field_mode = RLPT_FIELDS_STREAM;
    cfg->rho = 4;
    cfg->mlp_subset = 0;
    return RLPT_OK;
}

int rlpt_workspace_size(const rlpt_config* cfg, const rlpt_graph* const* graphs, int32_t n_graphs, size_t* bytes) {
    int rc = check_config(cfg);
    if (rc) return rc;
    if ((rc = check_graphs(graphs, n_graphs))) return rc;
    if (!bytes) return fail(RLPT_E_ARG, "bytes is NULL");
    if ((rc = mlp_check_config(*cfg, graphs, n_graphs))) return rc;
    int layout = 0;
    if ((rc = choose_layout(*cfg, graphs, n_graphs, &layout))) return rc;
    *bytes = plan(*cfg, graphs, n_graphs, layout).total;
    return RLPT_OK;
}

int rlpt_create(const rlpt_config* cfg, const rlpt_graph* const* graphs, int32_t n_graphs, const double* temps,
                void* d_workspace, size_t workspace_bytes, void* hip_stream, rlpt_ctx** out) {
    int rc = check_config(cfg);
    if (rc) return rc;
    if ((rc = check_graphs(graphs, n_graphs))) return rc;
    if (!temps || !out) return fail(RLPT_E_ARG, "temps / out is NULL");
    if (!d_workspace || ((uintptr_t)d_workspace & 255)) return fail(RLPT_E_ARG, "workspace must be 256-byte aligned");
    *out = nullptr;
    if ((rc = mlp_check_config(*cfg, graphs, n_graphs))) return rc;
    {   // set-up of rlpt_energy_fp64_noalloc: the static scratch's address on the current device, once per device
        void* p = nullptr;
        HIP_TRY(static_scratch_address(&p), "static scratch address");
    }
    for (int t = 0; t < cfg->n_temps; ++t) {
        if (!(temps[t] > 0.0) || !isfinite(temps[t])) return fail(RLPT_E_ARG, "temperatures must be finite and > 0");
        if (t > 0 && !(temps[t] > temps[t - 1])) return fail(RLPT_E_ARG, "temperatures must be strictly ascending");
    }
    int layout = 0;
    if ((rc = choose_layout(*cfg, graphs, n_graphs, &layout))) return rc;
    const Regions r = plan(*cfg, graphs, n_graphs, layout);
    if (workspace_bytes < r.total) return fail(RLPT_E_NOMEM, "workspace smaller than rlpt_workspace_size()");
    rlpt_ctx* c = new (std::nothrow) rlpt_ctx;
    if (!c) return fail(RLPT_E_NOMEM, "out of host memory");
    c->cfg = *cfg;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->S = n_graphs;
    c->T = cfg->n_temps;
    c->reps = cfg->n_reps;
    c->Rc = c->T * c->reps;
    c->n_copies = c->Rc * c->S;
    c->temps.assign(temps, temps + c->T);
    c->ws = d_workspace;
    c->ws_bytes = workspace_bytes;
    c->sh.cached = cfg->field_mode == RLPT_FIELDS_CACHED ? 1 : 0;
    c->sh.layout = layout;
    c->layout = layout;
    // everything a run changes, for checkpoints: amplitudes, energies, drift,
    // temperature permutation, cached fields, accumulators and counters
    c->state_regions = {{r.amp, r.E - r.amp}, {r.E, r.E64 - r.E}, {r.E64, r.drift - r.E64},
                        {r.drift, r.temp_of - r.drift}, {r.temp_of, r.copy_at - r.temp_of},
                        {r.copy_at, r.beta - r.copy_at}, {r.fields, r.ell_start - r.fields},
                        {r.acc_begin, r.acc_end - r.acc_begin}};
    {
        uint64_t h = 1469598103934665603ull;  // FNV-1a over the samples' shapes and the ladder
        auto mix = [&](uint64_t v) {
            for (int b = 0; b < 8; ++b) {
                h ^= (v >> (8 * b)) & 0xff;
                h *= 1099511628211ull;
            }
        };
        for (int s = 0; s < n_graphs; ++s) {
            mix((uint64_t)graphs[s]->N);
            mix((uint64_t)graphs[s]->n_terms());
            mix(graphs[s]->seed);
        }
        for (int t = 0; t < cfg->n_temps; ++t) {
            uint64_t bits;
            memcpy(&bits, &temps[t], 8);
            mix(bits);
        }
        c->fingerprint = h;
    }
    c->sh.rho = cfg->rho == 2 ? 2 : 4;
    c->cfg.rho = c->sh.rho;
    // short lists (sparse graphs): every padded list fits in one wave's registers
    if (layout == kLayoutPacked && !c->sh.cached) {
        uint32_t longest = 0;
        for (int s = 0; s < n_graphs; ++s)
            for (int l = 0; l < graphs[s]->N; ++l)
                longest = std::max(longest, graphs[s]->mode_start[l + 1] - graphs[s]->mode_start[l]);
        c->sh.short_lists = longest <= 128 ? 1 : 0;
    }
    unsigned char* b = static_cast<unsigned char*>(d_workspace);
    fill_ptrs(c->pf, b, r);
    fill_ptrs(c->pd, b, r);
    c->acc_region = b + r.acc_begin;
    c->acc_region_bytes = r.acc_end - r.acc_begin;
    c->scratch = reinterpret_cast<double*>(b + r.scratch);
    c->scratch_doubles = r.scratch_doubles;
    mlp_layout(*cfg, graphs[0]->N, n_graphs, &c->mlp, b, r.mlp);

    // host images of the device tables
    std::vector<uint32_t> ms, idx, cs;
    std::vector<float> J32, cJ32;
    std::vector<double> J64, Jq, cJ64;
    std::vector<uint8_t> cx;
    std::vector<uint16_t> cyz;
    std::vector<ushort4> quads;
    std::vector<uint32_t> pstart, pidx, estart, g32;
    std::vector<uint16_t> g16, c0tab;
    std::vector<double> pJ64, gJ64;
    int64_t amp_base = 0, quad_base = 0;
    for (int s = 0; s < c->S; ++s) {
        const rlpt_graph* g = graphs[s];
        SampleDev sd{};
        sd.N = g->N;
        sd.n_steps = g->N / 2;
        sd.mode_base = (uint32_t)(layout == kLayoutPacked ? ms.size() : cs.size());
        sd.amp_base = amp_base;
        sd.quad_base = quad_base;
        sd.n_quads = g->n_terms();
        if (layout == kLayoutPacked) {
            const uint32_t ebase = (uint32_t)idx.size();
            for (uint32_t v : g->mode_start) ms.push_back(v + ebase);
            idx.insert(idx.end(), g->idx.begin(), g->idx.end());
            if (cfg->precision == RLPT_FP64) J64.insert(J64.end(), g->Jl.begin(), g->Jl.end());
            else
                for (double v : g->Jl) J32.push_back((float)v);
        } else {
            const uint32_t cbase = (uint32_t)cx.size();
            for (uint32_t v : g->chunk_start) cs.push_back(v + cbase);
            cx.insert(cx.end(), g->cx.begin(), g->cx.end());
            cyz.insert(cyz.end(), g->cyz.begin(), g->cyz.end());
            if (cfg->precision == RLPT_FP64) cJ64.insert(cJ64.end(), g->cJ.begin(), g->cJ.end());
            else
                for (double v : g->cJ) cJ32.push_back((float)v);
        }
        for (int64_t q = 0; q < g->n_terms(); ++q) {
            ushort4 u;
            u.x = (unsigned short)g->quads[4 * q];
            u.y = (unsigned short)g->quads[4 * q + 1];
            u.z = (unsigned short)g->quads[4 * q + 2];
            u.w = (unsigned short)g->quads[4 * q + 3];
            quads.push_back(u);
        }
        Jq.insert(Jq.end(), g->J.begin(), g->J.end());
        if (c->sh.cached) {
            sd.pair_base = (int64_t)pstart.size();
            sd.ell_base = (int64_t)estart.size();
            sd.c0_base = (int64_t)c0tab.size();
            if (!build_cached_tables(g, layout, &pstart, &pidx, &pJ64, &estart, &g16, &g32, &gJ64, &c0tab)) {
                delete c;
                return fail(RLPT_E_ARG, "cached-field tables exceed 2^32 entries");
            }
        }
        amp_base += (int64_t)c->Rc * g->N;
        quad_base += g->n_terms();
        c->samples.push_back(sd);
        c->N.push_back(g->N);
        {
            uint32_t mc = 0;
            if (layout == kLayoutChunked)
                for (int l = 0; l < g->N; ++l) mc = std::max(mc, g->chunk_start[l + 1] - g->chunk_start[l]);
            c->max_chunks.push_back(mc);
        }
        c->max_N = std::max(c->max_N, g->N);
    }
    c->amp_complex = amp_base;
    // launch tile: explicit in the config, else from the tune registry, else built in
    {
        int block = 0;
        std::map<int, int> copies;
        std::map<int, int> counts;
        for (int s = 0; s < c->S; ++s) counts[c->N[s]] += 1;
        // the tune registry holds streaming-sweep timings; cached contexts use the built-in tile
        if (cfg->block_threads > 0 || cfg->copies_per_block > 0 || c->sh.cached ||
            !tune_choose(counts, cfg->precision, cfg->shared_pairs, &block, &copies)) {
            auto tile = [&](int n) { return c->sh.cached ? default_tile_cached(n) : default_tile(n); };
            block = cfg->block_threads > 0 ? cfg->block_threads : tile(c->max_N).block;
            for (const auto& nc : counts)
                copies[nc.first] = cfg->copies_per_block > 0 ? cfg->copies_per_block : tile(nc.first).copies;
            // the one-wave-per-copy path of short lists packs copies by itself
            if (cfg->block_threads <= 0 && cfg->copies_per_block <= 0 && !c->sh.cached && !c->sh.short_lists)
                spread_tile(counts, c->Rc, 512, &block, &copies);
        }
        rc = build_items(c, block, copies);
        if (rc) {
            delete c;
            return rc;
        }
    }
    c->sh.n_samples = c->S;
    c->sh.n_temps = c->T;
    c->sh.n_reps = c->reps;
    c->sh.copies_per_sample = c->Rc;
    c->sh.n_bins = cfg->n_bins;
    c->sh.spec_stride = c->max_N;
    c->sh.series_len = cfg->series_len;
    c->sh.shared_pairs = cfg->shared_pairs;
    c->sh.layout = layout;
    c->sh.renorm_tol = cfg->renorm_tol;
    c->sh.drift_tol = cfg->drift_tol;

    std::vector<float> b32(c->T);
    std::vector<double> b64(c->T);
    for (int t = 0; t < c->T; ++t) {
        b64[t] = 1.0 / temps[t];
        b32[t] = (float)b64[t];
    }
    hipError_t e = hipSuccess;
    auto up = [&](size_t off, auto& v) {
        if (e == hipSuccess) e = upload(b, off, v, c->stream);
    };
    up(r.samples, c->samples);
    up(r.items, c->items);  // sized for one item per copy (the finest tile)
    up(r.mode_start, ms);
    up(r.idx, idx);
    if (cfg->precision == RLPT_FP64) up(r.J, J64);
    else up(r.J, J32);
    up(r.chunk_start, cs);
    up(r.cx, cx);
    up(r.cyz, cyz);
    if (cfg->precision == RLPT_FP64) up(r.cJ, cJ64);
    else up(r.cJ, cJ32);
    up(r.quads, quads);
    up(r.Jq, Jq);
    up(r.pair_start, pstart);
    up(r.pidx, pidx);
    up(r.ell_start, estart);
    up(r.gidx16, g16);
    up(r.gidx32, g32);
    up(r.c0, c0tab);
    if (cfg->precision == RLPT_FP64) {
        up(r.pJ, pJ64);
        up(r.gJ, gJ64);
    } else {
        std::vector<float> f(pJ64.begin(), pJ64.end());
        up(r.pJ, f);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // f is reused below
        f.assign(gJ64.begin(), gJ64.end());
        up(r.gJ, f);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (cfg->precision == RLPT_FP64) up(r.beta, b64);
    else up(r.beta, b32);
    up(r.beta64, b64);
    if (e == hipSuccess) e = launch_zero(c->acc_region, c->acc_region_bytes, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "rlpt_create upload");
    }
    *out = c;
    return RLPT_OK;
}

int rlpt_destroy(rlpt_ctx* c) {
    if (!c) return RLPT_OK;
    (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    drop_events(c);
    delete c;
    return RLPT_OK;
}

int rlpt_init(rlpt_ctx* c, uint64_t run_seed) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    int rc;
    drop_graph(c);
    c->sh.run_seed = run_seed;
    HIP_TRY(launch_zero(c->acc_region, c->acc_region_bytes, c->stream), "zero accumulators");
    HIP_TRY(launch_init(c->cfg.precision, c->ptrs(), c->sh, c->n_copies, 256, c->stream), "init launch");
    HIP_TRY(launch_resync(c->cfg.precision, c->ptrs(), c->sh, c->n_copies, 2, c->stream), "initial energies");
    if ((rc = refresh_fields(c))) return rc;
    c->sweeps_done = 0;
    c->swaps_done = 0;
    c->inited = true;
    return RLPT_OK;
}

int rlpt_sweep(rlpt_ctx* c, int32_t n_sweeps) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    if (!c->inited) return fail(RLPT_E_STATE, "rlpt_init has not been called");
    if (n_sweeps < 0) return fail(RLPT_E_ARG, "n_sweeps must be >= 0");
    int64_t swaps = 0;
    int rc = enqueue_sweeps(c, c->sweeps_done, n_sweeps, &swaps);
    if (rc) return rc;
    c->sweeps_done += n_sweeps;
    c->swaps_done += swaps;
    return RLPT_OK;
}

int rlpt_swap(rlpt_ctx* c) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    if (!c->inited) return fail(RLPT_E_STATE, "rlpt_init has not been called");
    if (c->T < 2) return RLPT_OK;
    HIP_TRY(launch_swap(c->cfg.precision, c->ptrs(), c->sh, c->stream), "swap launch");
    HIP_TRY(launch_tick(c->ptrs(), c->cfg.precision, 0, 1, c->stream), "tick launch");
    c->swaps_done += 1;
    return RLPT_OK;
}

int rlpt_resync(rlpt_ctx* c, double* max_drift) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    if (!c->inited) return fail(RLPT_E_STATE, "rlpt_init has not been called");
    HIP_TRY(launch_resync(c->cfg.precision, c->ptrs(), c->sh, c->n_copies, 0, c->stream), "resync launch");
    int rc = refresh_fields(c);
    if (rc) return rc;
    rc = sync_and_flags(c);
    if (max_drift) {
        std::vector<double> d(c->n_copies);
        const double* dp = c->cfg.precision == RLPT_FP64 ? c->pd.drift : c->pf.drift;
        HIP_TRY(hipMemcpy(d.data(), dp, d.size() * 8, hipMemcpyDeviceToHost), "read drift");
        double m = 0.0;
        for (double v : d) m = (v > m || v != v) ? v : m;
        *max_drift = m;
    }
    return rc;
}

int rlpt_check(rlpt_ctx* c) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    return sync_and_flags(c);
}

int rlpt_run_graph(rlpt_ctx* c, int32_t n_sweeps, int32_t n_segments) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    if (!c->inited) return fail(RLPT_E_STATE, "rlpt_init has not been called");
    if (n_sweeps < 1 || n_segments < 0) return fail(RLPT_E_ARG, "n_sweeps must be >= 1 and n_segments >= 0");
    if (c->stream == nullptr) return fail(RLPT_E_ARG, "graph capture needs a context created on a non-default stream");
    const rlpt_config& cfg = c->cfg;
    const int iv[3] = {cfg.swap_interval, cfg.resync_interval, cfg.measure_interval};
    for (int i = 0; i < 3; ++i)
        if (iv[i] > 0 && n_sweeps % iv[i] != 0)
            return fail(RLPT_E_ARG, "n_sweeps must be a multiple of swap, resync and measure intervals");
    const int64_t end = c->sweeps_done + (int64_t)n_sweeps * n_segments;
    if (c->sweeps_done < cfg.measure_start && end > cfg.measure_start)
        return fail(RLPT_E_ARG, "graph segments may not straddle measure_start; advance with rlpt_sweep first");
    if (n_segments == 0) return RLPT_OK;
    const bool measuring = c->sweeps_done >= cfg.measure_start;
    const int64_t phase = c->sweeps_done % n_sweeps;
    int64_t swaps_per_segment = 0;
    if (!c->exec || c->graph_sweeps != n_sweeps || c->graph_phase != phase || c->graph_measuring != measuring) {
        drop_graph(c);
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "begin capture");
        int64_t sw = 0;
        c->capturing = true;
        int rc = enqueue_sweeps(c, c->sweeps_done, n_sweeps, &sw);
        c->capturing = false;
        hipError_t e = hipStreamEndCapture(c->stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        e = hipGraphInstantiate(&c->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            c->exec = nullptr;
            return hip_fail(e, "graph instantiate");
        }
        c->graph_sweeps = n_sweeps;
        c->graph_phase = phase;
        c->graph_measuring = measuring;
    }
    {  // swaps per segment from the schedule (same for every replay)
        for (int64_t k = 1; k <= n_sweeps; ++k)
            if (c->T > 1 && (c->sweeps_done + k) % cfg.swap_interval == 0) ++swaps_per_segment;
    }
    for (int s = 0; s < n_segments; ++s) HIP_TRY(hipGraphLaunch(c->exec, c->stream), "graph launch");
    c->sweeps_done += (int64_t)n_sweeps * n_segments;
    c->swaps_done += swaps_per_segment * n_segments;
    return RLPT_OK;
}

int rlpt_sweep_timing(rlpt_ctx* c, int32_t enable) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    c->timing = enable != 0;
    return RLPT_OK;
}

int rlpt_sweep_time_get(rlpt_ctx* c, double* total_ms, int64_t* n_launches) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    double sum = 0.0;
    for (auto& e : c->events) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second), "event elapsed");
        sum += ms;
        c->spare.push_back(e);
    }
    if (n_launches) *n_launches = (int64_t)c->events.size();
    if (total_ms) *total_ms = sum;
    c->events.clear();
    return RLPT_OK;
}

int rlpt_stream_lists(rlpt_ctx* c, int32_t n_launches, double* ms_per_launch) {
    if (!c || !ms_per_launch) return fail(RLPT_E_ARG, "NULL argument");
    if (n_launches < 1) return fail(RLPT_E_ARG, "n_launches must be >= 1");
    if (c->cfg.precision != RLPT_FP32 || c->layout != kLayoutChunked || c->sh.cached || c->sh.short_lists)
        return fail(RLPT_E_UNSUPPORTED, "the list-stream ceiling covers the FP32 streaming sweep over chunked lists");
    if (!c->inited) return fail(RLPT_E_STATE, "rlpt_init has not been called");
    const size_t sink_floats = (size_t)c->launch.n_items * (c->launch.block_threads / 64);
    if (sink_floats > 2 * c->scratch_doubles) return fail(RLPT_E_ARG, "too many workgroups for the scratch buffer");
    float* sink = reinterpret_cast<float*>(c->scratch);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0), "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RLPT_E_HIP, "event create");
    }
    double total = 0.0;
    hipError_t e = hipSuccess;
    for (int i = 0; i < n_launches && e == hipSuccess; ++i) {
        e = hipEventRecord(e0, c->stream);
        if (e == hipSuccess) e = launch_stream_lists(c->ptrs(), c->sh, c->launch, i, sink, c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        total += ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(RLPT_E_HIP, std::string("list-stream ceiling: ") + hipGetErrorString(e));
    *ms_per_launch = total / n_launches;
    return RLPT_OK;
}

int rlpt_counters(rlpt_ctx* c, int64_t* sweeps_done, int64_t* swaps_done, int64_t* n_meas) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    if (sweeps_done) *sweeps_done = c->sweeps_done;
    if (swaps_done) *swaps_done = c->swaps_done;
    if (n_meas) {
        int32_t m = 0;
        const int32_t* mp = c->cfg.precision == RLPT_FP64 ? c->pd.meas_cnt : c->pf.meas_cnt;
        HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
        HIP_TRY(hipMemcpy(&m, mp, 4, hipMemcpyDeviceToHost), "read measurement count");
        *n_meas = m;
    }
    return RLPT_OK;
}

static int copy_range(rlpt_ctx* c, int first, int n, int64_t* off, int64_t* count) {
    if (first < 0 || n < 0 || first + n > c->n_copies) return fail(RLPT_E_ARG, "copy range out of bounds");
    int64_t o = 0, k = 0;
    for (int cp = 0; cp < first + n; ++cp) {
        const int64_t Nc = c->N[cp / c->Rc];
        if (cp < first) o += Nc;
        else k += Nc;
    }
    *off = o;
    *count = k;
    if ((size_t)(2 * k) > c->scratch_doubles) return fail(RLPT_E_ARG, "copy range too large");
    return RLPT_OK;
}

int rlpt_get_state(rlpt_ctx* c, int32_t first, int32_t n, double* a) {
    if (!c || !a) return fail(RLPT_E_ARG, "NULL argument");
    int64_t off, k;
    int rc = copy_range(c, first, n, &off, &k);
    if (rc) return rc;
    unsigned char* amp = reinterpret_cast<unsigned char*>(c->cfg.precision == RLPT_FP64 ? (void*)c->pd.amp : (void*)c->pf.amp);
    HIP_TRY(launch_convert_state(c->cfg.precision, amp + off * 2 * c->real_bytes(), c->scratch, k, 0, c->stream), "convert");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY(hipMemcpy(a, c->scratch, k * 16, hipMemcpyDeviceToHost), "state read");
    return RLPT_OK;
}

int rlpt_set_state(rlpt_ctx* c, int32_t first, int32_t n, const double* a) {
    if (!c || !a) return fail(RLPT_E_ARG, "NULL argument");
    if (!c->inited) return fail(RLPT_E_STATE, "rlpt_init has not been called");
    int64_t off, k;
    int rc = copy_range(c, first, n, &off, &k);
    if (rc) return rc;
    for (int64_t i = 0; i < 2 * k; ++i)
        if (!isfinite(a[i])) return fail(RLPT_E_ARG, "state holds a non-finite value");
    unsigned char* amp = reinterpret_cast<unsigned char*>(c->cfg.precision == RLPT_FP64 ? (void*)c->pd.amp : (void*)c->pf.amp);
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY(hipMemcpy(c->scratch, a, k * 16, hipMemcpyHostToDevice), "state write");
    HIP_TRY(launch_convert_state(c->cfg.precision, amp + off * 2 * c->real_bytes(), c->scratch, k, 1, c->stream), "convert");
    // the running energies follow the new configurations (FP64, as at init; no drift check, no rescaling)
    HIP_TRY(launch_resync(c->cfg.precision, c->ptrs(), c->sh, c->n_copies, 2, c->stream), "energies");
    if ((rc = refresh_fields(c))) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    return RLPT_OK;
}

int rlpt_get_energies(rlpt_ctx* c, double* E, int32_t* temp_of) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    if (E) {
        if (c->cfg.precision == RLPT_FP64) {
            HIP_TRY(hipMemcpy(E, c->pd.E, c->n_copies * 8, hipMemcpyDeviceToHost), "read energies");
        } else {
            std::vector<float> e(c->n_copies);
            HIP_TRY(hipMemcpy(e.data(), c->pf.E, c->n_copies * 4, hipMemcpyDeviceToHost), "read energies");
            for (int i = 0; i < c->n_copies; ++i) E[i] = e[i];
        }
    }
    if (temp_of) {
        const int32_t* tp = c->cfg.precision == RLPT_FP64 ? c->pd.temp_of : c->pf.temp_of;
        HIP_TRY(hipMemcpy(temp_of, tp, c->n_copies * 4, hipMemcpyDeviceToHost), "read temperatures");
    }
    return RLPT_OK;
}

int rlpt_energy_fp64(rlpt_ctx* c, double* E) {
    if (!c || !E) return fail(RLPT_E_ARG, "NULL argument");
    HIP_TRY(launch_resync(c->cfg.precision, c->ptrs(), c->sh, c->n_copies, 1, c->stream), "energy launch");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    const double* ep = c->cfg.precision == RLPT_FP64 ? c->pd.E64 : c->pf.E64;
    HIP_TRY(hipMemcpy(E, ep, c->n_copies * 8, hipMemcpyDeviceToHost), "read energies");
    return RLPT_OK;
}

int rlpt_energy_fp64_noalloc(rlpt_ctx* c, double* d_E) {
    if (!c || !d_E) return fail(RLPT_E_ARG, "NULL argument");
    if ((size_t)c->n_copies * kResyncParts * sizeof(double) > kStaticScratchBytes)
        return fail(RLPT_E_ARG, "too many copies for the static scratch (" +
                                    std::to_string(kStaticScratchBytes / (kResyncParts * sizeof(double))) + " at most)");
    HIP_TRY(launch_energy_static(c->cfg.precision, c->ptrs(), c->sh, c->n_copies, d_E, c->stream), "energy launch");
    return RLPT_OK;
}

int rlpt_local_fields(rlpt_ctx* c, int32_t copy, double* F) {
    if (!c || !F) return fail(RLPT_E_ARG, "NULL argument");
    if (copy < 0 || copy >= c->n_copies) return fail(RLPT_E_ARG, "copy out of range");
    const int mu = copy / c->Rc, N = c->N[mu];
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY(launch_fields_sh(c->cfg.precision, c->ptrs(), c->sh, copy, mu, c->scratch, c->stream), "fields launch");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY(hipMemcpy(F, c->scratch, (size_t)N * 16, hipMemcpyDeviceToHost), "read fields");
    return RLPT_OK;
}

int rlpt_pair_dE(rlpt_ctx* c, int32_t copy, int32_t n, const int32_t* j, const int32_t* k, const double* aj_new,
                 const double* ak_new, double* dE) {
    if (!c || !j || !k || !aj_new || !ak_new || !dE) return fail(RLPT_E_ARG, "NULL argument");
    if (copy < 0 || copy >= c->n_copies) return fail(RLPT_E_ARG, "copy out of range");
    const int mu = copy / c->Rc, N = c->N[mu];
    if (n < 0 || (size_t)n * 8 > c->scratch_doubles) return fail(RLPT_E_ARG, "too many pairs");
    std::vector<int32_t> jk(2 * (size_t)n);
    std::vector<double> nw(4 * (size_t)n);
    for (int p = 0; p < n; ++p) {
        if (j[p] < 0 || j[p] >= N || k[p] < 0 || k[p] >= N || j[p] == k[p])
            return fail(RLPT_E_ARG, "pair indices must be distinct modes in [0, N)");
        jk[2 * p] = j[p];
        jk[2 * p + 1] = k[p];
        nw[4 * p] = aj_new[2 * p];
        nw[4 * p + 1] = aj_new[2 * p + 1];
        nw[4 * p + 2] = ak_new[2 * p];
        nw[4 * p + 3] = ak_new[2 * p + 1];
    }
    if (n == 0) return RLPT_OK;
    double* d_nw = c->scratch;
    double* d_dE = c->scratch + 4 * (size_t)n;
    int32_t* d_jk = reinterpret_cast<int32_t*>(c->scratch + 5 * (size_t)n);
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY(hipMemcpy(d_nw, nw.data(), nw.size() * 8, hipMemcpyHostToDevice), "write proposals");
    HIP_TRY(hipMemcpy(d_jk, jk.data(), jk.size() * 4, hipMemcpyHostToDevice), "write pairs");
    HIP_TRY(launch_pair_dE_sh(c->cfg.precision, c->ptrs(), c->sh, copy, mu, n, d_jk, d_nw, d_dE, c->stream), "pair launch");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY(hipMemcpy(dE, d_dE, (size_t)n * 8, hipMemcpyDeviceToHost), "read dE");
    return RLPT_OK;
}

int rlpt_observables(rlpt_ctx* c, rlpt_obs* o) {
    if (!c || !o) return fail(RLPT_E_ARG, "NULL argument");
    int rc = sync_and_flags(c);
    const bool f64 = c->cfg.precision == RLPT_FP64;
    const int ST = c->S * c->T, T1 = std::max(c->T - 1, 1);
    std::vector<double> obs((size_t)kNumObs * ST);
    HIP_TRY(hipMemcpy(obs.data(), f64 ? c->pd.obs : c->pf.obs, obs.size() * 8, hipMemcpyDeviceToHost), "read obs");
    double* dst[kNumObs] = {o->e_n, o->e_sum, o->e_sq, o->y2_sum, o->y4_sum, o->q_n, o->q_sum, o->q_sq, o->q_4};
    for (int f = 0; f < kNumObs; ++f)
        if (dst[f]) std::copy(obs.begin() + (size_t)f * ST, obs.begin() + (size_t)(f + 1) * ST, dst[f]);
    if (o->hist)
        HIP_TRY(hipMemcpy(o->hist, f64 ? c->pd.hist : c->pf.hist, (size_t)ST * c->cfg.n_bins * 8, hipMemcpyDeviceToHost),
                "read hist");
    if (o->hist_I)
        HIP_TRY(hipMemcpy(o->hist_I, f64 ? c->pd.hist_I : c->pf.hist_I, (size_t)ST * c->cfg.n_bins * 8,
                          hipMemcpyDeviceToHost), "read intensity hist");
    if (o->spectrum)
        HIP_TRY(hipMemcpy(o->spectrum, f64 ? c->pd.spec : c->pf.spec, (size_t)ST * c->max_N * 8,
                          hipMemcpyDeviceToHost), "read spectrum");
    if (c->cfg.series_len > 0) {
        if (o->series_e)
            HIP_TRY(hipMemcpy(o->series_e, f64 ? c->pd.series_e : c->pf.series_e, (size_t)ST * c->cfg.series_len * 8,
                              hipMemcpyDeviceToHost), "read series");
        if (o->series_q)
            HIP_TRY(hipMemcpy(o->series_q, f64 ? c->pd.series_q : c->pf.series_q, (size_t)ST * c->cfg.series_len * 8,
                              hipMemcpyDeviceToHost), "read series");
    }
    if (o->acc || o->tries) {
        std::vector<unsigned long long> a(ST);
        HIP_TRY(hipMemcpy(a.data(), f64 ? c->pd.acc : c->pf.acc, ST * 8, hipMemcpyDeviceToHost), "read acc");
        for (int i = 0; i < ST; ++i) {
            if (o->acc) o->acc[i] = (double)a[i];
            if (o->tries) o->tries[i] = (double)c->reps * (double)(c->N[i / c->T] / 2) * (double)c->sweeps_done;
        }
    }
    if (o->swap_acc || o->swap_tries) {
        std::vector<unsigned long long> a((size_t)c->S * c->reps * T1);
        HIP_TRY(hipMemcpy(a.data(), f64 ? c->pd.swap_acc : c->pf.swap_acc, a.size() * 8, hipMemcpyDeviceToHost),
                "read swap acc");
        for (int s = 0; s < c->S; ++s)
            for (int i = 0; i < T1; ++i) {
                double sum = 0;
                for (int r = 0; r < c->reps; ++r) sum += (double)a[((size_t)s * c->reps + r) * T1 + i];
                if (o->swap_acc) o->swap_acc[(size_t)s * T1 + i] = sum;
                if (o->swap_tries) o->swap_tries[(size_t)s * T1 + i] = c->T > 1 ? (double)c->reps * c->swaps_done : 0.0;
            }
    }
    return rc;
}

int rlpt_tile_of(rlpt_ctx* c, int32_t* block_threads, int32_t* copies_per_block) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    if (block_threads) *block_threads = c->launch.block_threads;
    if (copies_per_block)
        for (int s = 0; s < c->S; ++s) copies_per_block[s] = c->tile_copies.count(c->N[s]) ? c->tile_copies[c->N[s]] : 1;
    return RLPT_OK;
}

namespace {

struct CkptHeader {
    char magic[8];  // "RLPTCKP1"
    int32_t version, S, T, reps, precision, rho, field_mode, layout, shared_pairs, n_regions;
    uint64_t fingerprint, run_seed;
    int64_t sweeps_done, swaps_done;
};

void ckpt_header(const rlpt_ctx* c, CkptHeader* h) {
    memset(h, 0, sizeof(*h));
    memcpy(h->magic, "RLPTCKP1", 8);
    h->version = 1;
    h->S = c->S;
    h->T = c->T;
    h->reps = c->reps;
    h->precision = c->cfg.precision;
    h->rho = c->sh.rho;
    h->field_mode = c->cfg.field_mode;
    h->layout = c->layout;
    h->shared_pairs = c->cfg.shared_pairs;
    h->n_regions = (int32_t)c->state_regions.size();
    h->fingerprint = c->fingerprint;
    h->run_seed = c->sh.run_seed;
    h->sweeps_done = c->sweeps_done;
    h->swaps_done = c->swaps_done;
}

}  // namespace

int rlpt_checkpoint_save(rlpt_ctx* c, const char* path) {
    if (!c || !path) return fail(RLPT_E_ARG, "NULL argument");
    if (!c->inited) return fail(RLPT_E_STATE, "rlpt_init has not been called");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    CkptHeader h;
    ckpt_header(c, &h);
    FILE* f = fopen(path, "wb");
    if (!f) return fail(RLPT_E_ARG, std::string("cannot open ") + path + " for writing");
    bool ok = fwrite(&h, sizeof(h), 1, f) == 1;
    unsigned char* b = static_cast<unsigned char*>(c->ws);
    std::vector<unsigned char> buf;
    for (const auto& reg : c->state_regions) {
        const uint64_t n = reg.second;
        buf.resize(n);
        if (n && hipMemcpy(buf.data(), b + reg.first, n, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
        ok = ok && fwrite(&n, sizeof(n), 1, f) == 1 && (n == 0 || fwrite(buf.data(), 1, n, f) == n);
    }
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail(RLPT_E_ARG, std::string("writing the checkpoint ") + path + " failed");
    return RLPT_OK;
}

int rlpt_checkpoint_load(rlpt_ctx* c, const char* path) {
    if (!c || !path) return fail(RLPT_E_ARG, "NULL argument");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(RLPT_E_ARG, std::string("cannot open ") + path);
    CkptHeader h, mine;
    ckpt_header(c, &mine);
    std::vector<std::vector<unsigned char>> data;
    const char* err = nullptr;
    if (fread(&h, sizeof(h), 1, f) != 1 || memcmp(h.magic, "RLPTCKP1", 8) != 0 || h.version != 1)
        err = "not a checkpoint of this library";
    else if (h.S != mine.S || h.T != mine.T || h.reps != mine.reps || h.precision != mine.precision ||
             h.rho != mine.rho || h.field_mode != mine.field_mode || h.layout != mine.layout ||
             h.shared_pairs != mine.shared_pairs || h.n_regions != mine.n_regions ||
             h.fingerprint != mine.fingerprint)
        err = "checkpoint of a different context (samples, terms, ladder or configuration)";
    for (size_t i = 0; !err && i < c->state_regions.size(); ++i) {
        uint64_t n = 0;
        if (fread(&n, sizeof(n), 1, f) != 1 || n != c->state_regions[i].second) {
            err = "checkpoint regions do not match this context";
            break;
        }
        data.emplace_back(n);
        if (n && fread(data.back().data(), 1, n, f) != n) err = "truncated checkpoint";
    }
    fclose(f);
    if (err) return fail(RLPT_E_ARG, std::string(err) + ": " + path);
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    drop_graph(c);
    unsigned char* b = static_cast<unsigned char*>(c->ws);
    for (size_t i = 0; i < c->state_regions.size(); ++i)
        if (!data[i].empty())
            HIP_TRY(hipMemcpy(b + c->state_regions[i].first, data[i].data(), data[i].size(), hipMemcpyHostToDevice),
                    "checkpoint upload");
    c->sh.run_seed = h.run_seed;
    c->sweeps_done = h.sweeps_done;
    c->swaps_done = h.swaps_done;
    c->inited = true;
    return RLPT_OK;
}

int rlpt_autotune(const rlpt_config* cfg, const rlpt_graph* const* graphs, int32_t n_graphs, const double* temps,
                  void* d_workspace, size_t workspace_bytes, void* hip_stream, int32_t sweeps_per_trial,
                  int32_t* n_trials) {
    int rc = check_config(cfg);
    if (rc) return rc;
    if (cfg->field_mode == RLPT_FIELDS_CACHED)
        return fail(RLPT_E_UNSUPPORTED, "the autotuner times the streaming sweep; use field_mode = RLPT_FIELDS_STREAM");
    if ((rc = check_graphs(graphs, n_graphs))) return rc;
    if (sweeps_per_trial < 1) return fail(RLPT_E_ARG, "sweeps_per_trial must be >= 1");
    std::map<int, int> counts;
    for (int i = 0; i < n_graphs; ++i) counts[graphs[i]->N] += 1;
    rlpt_config c2 = *cfg;
    c2.swap_interval = 1 << 30;  // timing covers sweeps only: one launch per trial
    c2.resync_interval = 0;
    c2.measure_interval = 0;
    c2.block_threads = 256;
    c2.copies_per_block = 1;
    // every trial times the whole context's launch (all N together, as the
    // context will run): per workgroup size, the N classes are tuned one after
    // another, each over its copies per workgroup with the others at their
    // current choice (built-in first), and each trial is recorded for its N
    rlpt_ctx* c = nullptr;
    rc = rlpt_create(&c2, graphs, n_graphs, temps, d_workspace, workspace_bytes, hip_stream, &c);
    if (rc) return rc;
    rc = rlpt_init(c, 1);
    int trials = 0;
    for (int b = 64; b <= 1024 && rc == RLPT_OK; b *= 2) {
        std::map<int, int> cur;
        for (const auto& nc : counts) cur[nc.first] = std::max(1, std::min(default_tile(nc.first).copies, b / 64));
        for (const auto& nc : counts) {
            double best = -1.0;
            int best_cp = cur[nc.first];
            for (int cp = 1; cp <= b / 64 && rc == RLPT_OK; cp *= 2) {
                std::map<int, int> copies = cur;
                copies[nc.first] = cp;
                if (build_items(c, b, copies) != RLPT_OK) continue;  // LDS limit
                if ((rc = upload_items(c))) break;
                if ((rc = rlpt_sweep(c, 1))) break;
                c->timing = true;
                if ((rc = rlpt_sweep(c, sweeps_per_trial))) break;
                double ms = 0;
                int64_t n = 0;
                rc = rlpt_sweep_time_get(c, &ms, &n);
                c->timing = false;
                if (rc) break;
                rlpt_tile t{};
                t.n_modes = nc.first;
                t.precision = cfg->precision;
                t.shared_pairs = cfg->shared_pairs;
                t.block_threads = b;
                t.copies_per_block = cp;
                t.ms_per_sweep = ms / sweeps_per_trial;
                tune_record(t);
                ++trials;
                if (best < 0 || t.ms_per_sweep < best) {
                    best = t.ms_per_sweep;
                    best_cp = cp;
                }
            }
            cur[nc.first] = best_cp;
        }
    }
    int rc2 = rlpt_destroy(c);
    if (rc) return rc;
    if (rc2) return rc2;
    if (n_trials) *n_trials = trials;
    return RLPT_OK;
}

int rlpt_tau_int(const double* x, int64_t n, double c_window, double* tau, int64_t* window) {
    if (!x || !tau || n < 2) return fail(RLPT_E_ARG, "need a series of at least 2 points");
    if (!(c_window > 0)) return fail(RLPT_E_ARG, "c_window must be > 0");
    double mean = 0;
    for (int64_t i = 0; i < n; ++i) mean += x[i];
    mean /= (double)n;
    double c0 = 0;
    for (int64_t i = 0; i < n; ++i) c0 += (x[i] - mean) * (x[i] - mean);
    c0 /= (double)n;
    if (!(c0 > 0)) {
        *tau = 0.5;
        if (window) *window = 0;
        return RLPT_OK;
    }
    double t = 0.5;
    int64_t W = 0;
    for (int64_t lag = 1; lag < n; ++lag) {
        double ct = 0;
        for (int64_t i = 0; i + lag < n; ++i) ct += (x[i] - mean) * (x[i + lag] - mean);
        ct /= (double)n;
        t += ct / c0;
        W = lag;
        if ((double)lag >= c_window * t) break;
    }
    *tau = t;
    if (window) *window = W;
    return RLPT_OK;
}

}  // extern "C"
