// Host-side context of librlpt (shared by the runtime source files).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "mlp.hpp"

using rlpt::DevPtrs;
using rlpt::ItemDev;
using rlpt::SampleDev;
using rlpt::ShapeInfo;
using rlpt::SweepLaunch;

struct rlpt_ctx {
    rlpt_config cfg{};
    hipStream_t stream = nullptr;
    int S = 0, T = 0, reps = 0, Rc = 0, n_copies = 0, max_N = 0;
    std::vector<int> N;
    std::vector<uint32_t> max_chunks;  // longest chunked list of each sample (0 in the packed layout)
    std::vector<double> temps;
    std::vector<SampleDev> samples;
    std::vector<ItemDev> items;
    ShapeInfo sh{};
    SweepLaunch launch{};
    DevPtrs<float> pf{};
    DevPtrs<double> pd{};
    // regions of the workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    unsigned char* acc_region = nullptr;  // accumulators cleared at init
    size_t acc_region_bytes = 0;
    double* scratch = nullptr;            // hook / state-transfer buffer (doubles)
    size_t scratch_doubles = 0;
    int64_t amp_complex = 0;
    std::vector<std::pair<size_t, size_t>> state_regions;  // (offset, bytes) saved by a checkpoint
    uint64_t fingerprint = 0;                               // samples, terms and ladder of the context
    int layout = 0;
    int64_t sweeps_done = 0, swaps_done = 0;
    bool inited = false;
    std::map<int, int> tile_copies;       // copies per workgroup for each N
    // cached HIP graph of one segment
    hipGraphExec_t exec = nullptr;
    int graph_sweeps = 0;
    int64_t graph_phase = -1;
    bool graph_measuring = false;
    // sweep-kernel timing
    bool timing = false;
    bool capturing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events, spare;
    // learned global proposal
    rlpt::MlpDev mlp{};
    bool mlp_setup = false;
    int mlp_moves = 0;         // learned rounds after every sweep
    double mlp_scale = 1.0;    // proposal step scale
    std::vector<int32_t> mlp_temp;
    std::vector<int64_t> mlp_count;
    int mlp_slot = 0;
    int64_t mlp_adam_t = 0;
    uint64_t mlp_seed = 0;

    const void* ptrs() const {
        return cfg.precision == RLPT_FP64 ? static_cast<const void*>(&pd) : static_cast<const void*>(&pf);
    }
    size_t real_bytes() const { return cfg.precision == RLPT_FP64 ? 8 : 4; }
};

namespace rlpt {
size_t mlp_layout(const rlpt_config& cfg, int N, int S, MlpDev* M, unsigned char* base, size_t off);
int mlp_check_config(const rlpt_config& cfg, const rlpt_graph* const* g, int S);
}  // namespace rlpt
int mlp_enqueue_round(rlpt_ctx* c);
