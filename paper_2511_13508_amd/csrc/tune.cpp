// Tile registry of the sweep kernel: measured time per sweep for (N,
// precision, pair schedule, threads per workgroup, copies per workgroup),
// filled by rlpt_autotune, persisted as one JSON object per line, and
// consulted by rlpt_create to choose launch tiles for a context.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rlpt {
namespace {

std::mutex g_mu;
std::vector<rlpt_tile> g_reg;

bool same_key(const rlpt_tile& a, const rlpt_tile& b) {
    return a.n_modes == b.n_modes && a.precision == b.precision && a.shared_pairs == b.shared_pairs &&
           a.block_threads == b.block_threads && a.copies_per_block == b.copies_per_block;
}

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "";
    std::string a = p.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

bool get_num(const char* line, const char* key, double* v) {
    const char* p = strstr(line, key);
    if (!p) return false;
    p = strchr(p, ':');
    if (!p) return false;
    return sscanf(p + 1, "%lf", v) == 1;
}

}  // namespace

void tune_record(const rlpt_tile& t) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& e : g_reg)
        if (same_key(e, t)) {
            e = t;
            return;
        }
    g_reg.push_back(t);
}

// For a context holding `counts[N]` samples of each N: the workgroup size that
// minimises the summed best time per sweep over the N classes, and for each N
// the copies per workgroup that are best at that size.  False when some N has
// no entry.
bool tune_choose(const std::map<int, int>& counts, int precision, int shared, int* block,
                 std::map<int, int>* copies) {
    std::lock_guard<std::mutex> lk(g_mu);
    double best_total = -1.0;
    for (int b = 64; b <= 1024; b *= 2) {
        double total = 0.0;
        std::map<int, int> pick;
        bool ok = true;
        for (const auto& nc : counts) {
            double best = -1.0;
            for (const auto& e : g_reg)
                if (e.n_modes == nc.first && e.precision == precision && e.shared_pairs == shared &&
                    e.block_threads == b && (best < 0 || e.ms_per_sweep < best)) {
                    best = e.ms_per_sweep;
                    pick[nc.first] = e.copies_per_block;
                }
            if (best < 0) {
                ok = false;
                break;
            }
            total += best;
        }
        if (ok && (best_total < 0 || total < best_total)) {
            best_total = total;
            *block = b;
            *copies = pick;
        }
    }
    return best_total >= 0;
}

}  // namespace rlpt

using namespace rlpt;

extern "C" {

int rlpt_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_reg.clear();
    return RLPT_OK;
}

int rlpt_tune_set(const rlpt_tile* t) {
    if (!t) return fail(RLPT_E_ARG, "tile is NULL");
    if (t->n_modes < 4 || t->block_threads < 64 || t->block_threads > 1024 ||
        (t->block_threads & (t->block_threads - 1)) || t->copies_per_block < 1 ||
        t->copies_per_block > t->block_threads / 64 || !(t->ms_per_sweep >= 0.0))
        return fail(RLPT_E_ARG, "invalid tile entry");
    tune_record(*t);
    return RLPT_OK;
}

int rlpt_tune_get(rlpt_tile* out, int32_t capacity, int32_t* count) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (count) *count = (int32_t)g_reg.size();
    if (out)
        for (int32_t i = 0; i < capacity && i < (int32_t)g_reg.size(); ++i) out[i] = g_reg[i];
    return RLPT_OK;
}

int rlpt_tune_save(const char* path) {
    if (!path) return fail(RLPT_E_ARG, "path is NULL");
    const std::string arch = device_arch();
    std::lock_guard<std::mutex> lk(g_mu);
    FILE* f = fopen(path, "w");
    if (!f) return fail(RLPT_E_ARG, std::string("cannot write ") + path);
    for (const auto& e : g_reg)
        fprintf(f,
                "{\"device\": \"%s\", \"n_modes\": %d, \"precision\": %d, \"shared_pairs\": %d, "
                "\"block_threads\": %d, \"copies_per_block\": %d, \"ms_per_sweep\": %.6f}\n",
                arch.c_str(), e.n_modes, e.precision, e.shared_pairs, e.block_threads, e.copies_per_block,
                e.ms_per_sweep);
    fclose(f);
    return RLPT_OK;
}

int rlpt_tune_load(const char* path) {
    if (!path) return fail(RLPT_E_ARG, "path is NULL");
    FILE* f = fopen(path, "r");
    if (!f) return fail(RLPT_E_ARG, std::string("cannot read ") + path);
    const std::string arch = device_arch();
    char line[512];
    while (fgets(line, sizeof line, f)) {
        const char* d = strstr(line, "\"device\": \"");
        if (d && !arch.empty()) {
            d += strlen("\"device\": \"");
            if (strncmp(d, arch.c_str(), arch.size()) != 0 || d[arch.size()] != '"') continue;
        }
        double n, p, s, b, c, ms;
        if (!get_num(line, "\"n_modes\"", &n) || !get_num(line, "\"precision\"", &p) ||
            !get_num(line, "\"shared_pairs\"", &s) || !get_num(line, "\"block_threads\"", &b) ||
            !get_num(line, "\"copies_per_block\"", &c) || !get_num(line, "\"ms_per_sweep\"", &ms))
            continue;
        rlpt_tile t{};
        t.n_modes = (int32_t)n;
        t.precision = (int32_t)p;
        t.shared_pairs = (int32_t)s;
        t.block_threads = (int32_t)b;
        t.copies_per_block = (int32_t)c;
        t.ms_per_sweep = ms;
        if (rlpt_tune_set(&t) != RLPT_OK) continue;
    }
    fclose(f);
    return RLPT_OK;
}

}  // extern "C"
