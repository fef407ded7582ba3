// Host builder of one disorder sample: quenched random frequencies, the
// frequency-matching filter and Gaussian couplings (sec. II.C of Benedetti &
// Leuzzi, arXiv 2511.13508: "Quenched random frequencies", eq. gamma_scaling,
// "Random values of the effective coupling constants" with eq. Gauss, "Graph
// generation"), plus the per-mode lists that the sweep kernel streams.
//
// Enumeration: for each i<j<k the fourth index l of a kept term lies in a
// narrow window of sorted frequencies for each split, found by binary search
// with a safety margin; the exact test |(w_p + w_s) - (w_m + w_n)| < gamma then
// decides, so the kept set and its order (i<j<k<l lexicographic, splits
// (i,l|j,k), (i,k|j,l), (i,j|k,l)) are those of the plain four-fold loop.
#include <math.h>
#include <stdlib.h>

#include <algorithm>
#include <new>
#include <unordered_set>

#include "internal.hpp"
#include "philox.hpp"

namespace {

constexpr double kPi = 3.14159265358979323846;

double gauss_from(uint64_t w0, uint64_t w1) {
    // Box & Muller (1958)
    double u1 = 1.0 - rlpt::uniform01<double>(w0);
    double u2 = rlpt::uniform01<double>(w1);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2);
}

bool matched(const double* w, int p, int s, int m, int n, double gamma) {
    double mismatch = (w[p] + w[s]) - (w[m] + w[n]);
    return fabs(mismatch) < gamma;
}

// indices l in (k, N) with w[l] within [lo, hi]
void window(const std::vector<double>& w, int k, double lo, double hi, int* first, int* last) {
    auto b = w.begin() + (k + 1);
    *first = (int)(std::lower_bound(b, w.end(), lo) - w.begin());
    *last = (int)(std::upper_bound(b, w.end(), hi) - w.begin());
}

// Sparse mode-locked graph: c = floor(z N / 4) matched terms drawn uniformly
// without replacement (rejection sampling over random quadruplets and splits,
// in the attempt order of the Philox stream (t, 2, 0, 0)).
bool sparse_terms(rlpt_graph* g, const rlpt_graph_desc* d) {
    const int N = g->N;
    const int64_t c = (int64_t)d->mean_degree * N / 4;
    if (c < 1) return false;
    const double* w = g->omega.data();
    std::unordered_set<uint64_t> seen;
    g->quads.reserve(4 * c);
    const uint64_t cap = 64ull * (uint64_t)N * (uint64_t)c + 1000000ull;
    int64_t kept = 0;
    for (uint64_t t = 0; t < cap && kept < c; ++t) {
        const rlpt::Philox4 r = rlpt::philox4x64(t, 2, 0, 0, d->seed, rlpt::kTagGraph);
        int v[4];
        for (int i = 0; i < 4; ++i) v[i] = rlpt::index_below(r.v[i], N);
        const int split = (int)(((r.v[0] & 0xffffffffull) * 3ull) >> 32);
        std::sort(v, v + 4);
        if (v[0] == v[1] || v[1] == v[2] || v[2] == v[3]) continue;
        if (!(d->split_mask & (1 << split))) continue;
        const int t4[3][4] = {{v[0], v[3], v[1], v[2]}, {v[0], v[2], v[1], v[3]}, {v[0], v[1], v[2], v[3]}};
        const int* q = t4[split];
        if (!matched(w, q[0], q[1], q[2], q[3], g->gamma)) continue;
        const uint64_t key = (uint64_t)v[0] | (uint64_t)v[1] << 10 | (uint64_t)v[2] << 20 | (uint64_t)v[3] << 30 |
                             (uint64_t)split << 40;
        if (!seen.insert(key).second) continue;
        for (int i = 0; i < 4; ++i) g->quads.push_back((int16_t)q[i]);
        ++kept;
    }
    return kept == c;
}

}  // namespace

extern "C" int rlpt_graph_build(const rlpt_graph_desc* d, rlpt_graph** out) {
    using namespace rlpt;
    if (!d || !out) return fail(RLPT_E_ARG, "rlpt_graph_build: NULL argument");
    *out = nullptr;
    const int N = d->n_modes;
    if (N < 4 || N > kMaxModes) return fail(RLPT_E_ARG, "rlpt_graph_build: n_modes must be in [4, 1024]");
    if (d->split_mask <= 0 || d->split_mask > 7) return fail(RLPT_E_ARG, "rlpt_graph_build: bad split_mask");
    if (d->omega_kind != RLPT_OMEGA_RANDOM && d->omega_kind != RLPT_OMEGA_COMB)
        return fail(RLPT_E_ARG, "rlpt_graph_build: bad omega_kind");
    rlpt_graph* g = new (std::nothrow) rlpt_graph;
    if (!g) return fail(RLPT_E_NOMEM, "rlpt_graph_build: out of host memory");
    try {
        g->N = N;
        g->seed = d->seed;
        g->gamma = d->gamma > 0.0 ? d->gamma : 1.0 / (2.0 * (double)(N - 1));
        g->omega.resize(N);
        if (d->omega_kind == RLPT_OMEGA_COMB) {
            for (int i = 0; i < N; ++i) g->omega[i] = (double)i / (double)(N - 1);
        } else {
            for (int i = 0; i < N; ++i)
                g->omega[i] = uniform01<double>(philox4x64((uint64_t)i, 0, 0, 0, d->seed, kTagGraph).v[0]);
            std::sort(g->omega.begin(), g->omega.end());
        }
        const double* w = g->omega.data();
        const double gam = g->gamma;
        if (d->mean_degree > 0) {
            if (!sparse_terms(g, d)) {
                delete g;
                return fail(RLPT_E_ARG, "rlpt_graph_build: could not draw floor(mean_degree N / 4) distinct matched "
                                        "terms; lower mean_degree");
            }
        } else {
            const double margin = 4.0 * gam + 1e-9;
            std::vector<int> cand;
            for (int i = 0; i < N; ++i)
                for (int j = i + 1; j < N; ++j)
                    for (int k = j + 1; k < N; ++k) {
                        // A: w_l ~ w_j + w_k - w_i ; B: w_l ~ w_i + w_k - w_j ; C: w_l ~ w_i + w_j - w_k
                        const double centre[3] = {w[j] + w[k] - w[i], w[i] + w[k] - w[j], w[i] + w[j] - w[k]};
                        cand.clear();
                        for (int s = 0; s < 3; ++s) {
                            if (!(d->split_mask & (1 << s))) continue;
                            int f, l;
                            window(g->omega, k, centre[s] - margin, centre[s] + margin, &f, &l);
                            for (int x = f; x < l; ++x) cand.push_back(x);
                        }
                        if (cand.empty()) continue;
                        std::sort(cand.begin(), cand.end());
                        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
                        for (int l : cand) {
                            const int split[3][4] = {{i, l, j, k}, {i, k, j, l}, {i, j, k, l}};
                            for (int s = 0; s < 3; ++s) {
                                if (!(d->split_mask & (1 << s))) continue;
                                const int* t = split[s];
                                if (matched(w, t[0], t[1], t[2], t[3], gam))
                                    for (int r = 0; r < 4; ++r) g->quads.push_back((int16_t)t[r]);
                            }
                        }
                    }
        }
        const int64_t c = (int64_t)g->quads.size() / 4;
        if (c == 0) {
            delete g;
            return fail(RLPT_E_ARG, "rlpt_graph_build: no term passes the frequency-matching filter");
        }
        g->sigma2 = (double)N / (double)c;
        const double sigma = sqrt(g->sigma2);
        g->J.resize(c);
        for (int64_t q = 0; q < c; ++q) {
            Philox4 r = philox4x64((uint64_t)q, 1, 0, 0, d->seed, kTagGraph);
            g->J[q] = sigma * gauss_from(r.v[0], r.v[1]);
        }
        // per-mode lists: for a term conj(a_p) conj(a_s) a_m a_n the field of
        // p is J conj(a_s) a_m a_n, of s is J conj(a_p) a_m a_n, of m is
        // J conj(a_n) a_p a_s, of n is J conj(a_m) a_p a_s
        std::vector<int64_t> deg(N, 0);
        for (int64_t q = 0; q < 4 * c; ++q) deg[g->quads[q]]++;
        g->mode_start.assign(N + 1, 0);
        for (int l = 0; l < N; ++l) g->mode_start[l + 1] = g->mode_start[l] + (uint32_t)((deg[l] + 3) / 4 * 4);
        const uint32_t total = g->mode_start[N];
        g->idx.assign(total, 0);
        g->Jl.assign(total, 0.0);
        std::vector<uint32_t> fill(g->mode_start.begin(), g->mode_start.end() - 1);
        auto pack = [](int x, int y, int z) { return (uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20); };
        for (int64_t q = 0; q < c; ++q) {
            const int p = g->quads[4 * q], s = g->quads[4 * q + 1], m = g->quads[4 * q + 2], n = g->quads[4 * q + 3];
            const int role[4][4] = {{p, s, m, n}, {s, p, m, n}, {m, n, p, s}, {n, m, p, s}};
            for (int r = 0; r < 4; ++r) {
                const uint32_t e = fill[role[r][0]]++;
                g->idx[e] = pack(role[r][1], role[r][2], role[r][3]);
                g->Jl[e] = g->J[q];
            }
        }
        // chunked lists: each mode's entries grouped by partner x (term order
        // kept inside a group), every group padded to a multiple of 4 entries
        if (N <= kMaxChunkModes) {
            g->chunk_start.assign(N + 1, 0);
            std::vector<uint32_t> order;
            for (int l = 0; l < N; ++l) {
                const uint32_t b = g->mode_start[l], e = b + (uint32_t)deg[l];
                order.resize(e - b);
                for (uint32_t i = 0; i < e - b; ++i) order[i] = b + i;
                std::stable_sort(order.begin(), order.end(),
                                 [&](uint32_t u, uint32_t v) { return (g->idx[u] & 1023u) < (g->idx[v] & 1023u); });
                size_t i = 0;
                while (i < order.size()) {
                    const uint32_t x = g->idx[order[i]] & 1023u;
                    size_t end = i;
                    while (end < order.size() && (g->idx[order[end]] & 1023u) == x) ++end;
                    for (size_t c0 = i; c0 < end; c0 += 4) {
                        g->cx.push_back((uint8_t)x);
                        for (size_t k = c0; k < c0 + 4; ++k) {
                            if (k < end) {
                                const uint32_t v = g->idx[order[k]];
                                const uint32_t y = (v >> 10) & 1023u, z = v >> 20;
                                g->cyz.push_back((uint16_t)(y | (z << 8)));
                                g->cJ.push_back(g->Jl[order[k]]);
                            } else {
                                g->cyz.push_back(0);
                                g->cJ.push_back(0.0);
                            }
                        }
                    }
                    i = end;
                }
                g->chunk_start[l + 1] = (uint32_t)g->cx.size();
            }
        }
    } catch (const std::bad_alloc&) {
        delete g;
        return fail(RLPT_E_NOMEM, "rlpt_graph_build: out of host memory");
    }
    *out = g;
    return RLPT_OK;
}

extern "C" void rlpt_graph_free(rlpt_graph* g) { delete g; }

namespace rlpt {

// The three other members of term e as seen from member t: its partner on
// the same side of the term, then the two modes of the other side.
void term_triple(const int16_t* q, int t, int* x) {
    static const int kRole[4][3] = {{1, 2, 3}, {0, 2, 3}, {3, 0, 1}, {2, 0, 1}};
    for (int r = 0; r < 3; ++r) x[r] = q[kRole[t][r]];
}

// per ordered pair (j -> l): how many terms hold both, and how many of them
// have j as l's partner
void pair_counts(const rlpt_graph* g, std::vector<uint32_t>* cnt, std::vector<uint32_t>* c0) {
    const int N = g->N;
    cnt->assign((size_t)N * N, 0);
    if (c0) c0->assign((size_t)N * N, 0);
    for (int64_t e = 0; e < g->n_terms(); ++e) {
        const int16_t* q = &g->quads[4 * e];
        for (int t = 0; t < 4; ++t) {
            int x[3];
            term_triple(q, t, x);
            for (int r = 0; r < 3; ++r) {
                (*cnt)[(size_t)x[r] * N + q[t]] += 1;
                if (c0 && r == 0) (*c0)[(size_t)x[r] * N + q[t]] += 1;
            }
        }
    }
}

// padded entries of the sliced-ELL gather block of one sample: per source j
// and slice s of up to 64 targets, (max rank over the slice, rounded up to 4)
// x slice width
size_t ell_entries(const rlpt_graph* g, const std::vector<uint32_t>& cnt) {
    const int N = g->N, ns = (N + kSlice - 1) / kSlice;
    size_t total = 0;
    for (int j = 0; j < N; ++j)
        for (int s = 0; s < ns; ++s) {
            const int w = std::min(kSlice, N - kSlice * s);
            uint32_t L = 0;
            for (int i = 0; i < w; ++i) L = std::max(L, cnt[(size_t)j * N + kSlice * s + i]);
            total += (size_t)((L + 3) / 4) * 4 * w;
        }
    return total;
}

}  // namespace rlpt

extern "C" int rlpt_graph_info_get(const rlpt_graph* g, rlpt_graph_info* out) {
    using namespace rlpt;
    if (!g || !out) return fail(RLPT_E_ARG, "rlpt_graph_info_get: NULL argument");
    std::vector<int64_t> deg(g->N, 0);
    for (int16_t m : g->quads) deg[m]++;
    out->n_modes = g->N;
    out->pad = 0;
    out->n_terms = g->n_terms();
    out->deg_min = *std::min_element(deg.begin(), deg.end());
    out->deg_max = *std::max_element(deg.begin(), deg.end());
    out->deg_sum = 4 * g->n_terms();
    out->gamma = g->gamma;
    out->sigma2 = g->sigma2;
    out->list_entries = g->mode_start.back();
    out->list_bytes = (int64_t)g->mode_start.back() * (int64_t)(sizeof(uint32_t) + sizeof(float));
    out->chunk_entries = 4 * (int64_t)g->cx.size();
    out->chunk_bytes = (int64_t)g->cx.size() * 25;
    std::vector<uint32_t> cnt;
    pair_counts(g, &cnt, nullptr);
    out->pair_entries = 12 * g->n_terms();
    out->gather_entries = (int64_t)ell_entries(g, cnt);
    return RLPT_OK;
}

extern "C" int rlpt_graph_export(const rlpt_graph* g, double* omega, int16_t* quads, double* J) {
    using namespace rlpt;
    if (!g) return fail(RLPT_E_ARG, "rlpt_graph_export: NULL graph");
    if (omega) std::copy(g->omega.begin(), g->omega.end(), omega);
    if (quads) std::copy(g->quads.begin(), g->quads.end(), quads);
    if (J) std::copy(g->J.begin(), g->J.end(), J);
    return RLPT_OK;
}
