// Internal types shared by the host runtime (api.cpp, graph.cpp) and the
// device kernels (kernels.hip).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/rlpt.h"

// ----------------------------------------------------------------- host graph
struct rlpt_graph {
    int32_t N = 0;
    uint64_t seed = 0;
    double gamma = 0.0;
    double sigma2 = 0.0;
    std::vector<double> omega;         // [N] sorted frequencies
    std::vector<int16_t> quads;        // [c][4] (p, s, m, n)
    std::vector<double> J;             // [c]
    // per-mode lists: entries of mode l are [mode_start[l], mode_start[l+1]),
    // padded to a multiple of 4; entry = (x, y, z) packed 10 bits each, coupling
    std::vector<uint32_t> mode_start;  // [N+1]
    std::vector<uint32_t> idx;         // packed x | y << 10 | z << 20
    std::vector<double> Jl;            // coupling of each entry (0 for padding)
    // chunked lists (N <= 256): mode l owns chunks [chunk_start[l], chunk_start[l+1]);
    // a chunk is 4 entries with one partner x; (y, z) packed y | z << 8 in 16 bits
    std::vector<uint32_t> chunk_start; // [N+1]
    std::vector<uint8_t> cx;           // [chunks]
    std::vector<uint16_t> cyz;         // [4 * chunks]
    std::vector<double> cJ;            // [4 * chunks] (0 for padding)
    int64_t n_terms() const { return (int64_t)J.size(); }
};

namespace rlpt {

constexpr int kMaxModes = 1024;  // three 10-bit mode indices per packed entry
constexpr int kMaxChunkModes = 256;  // 8-bit indices in the chunked layout
enum ListLayout { kLayoutPacked = 1, kLayoutChunked = 2 };

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// cached-field tables (graph.cpp): the other members of a term seen from
// member t (its partner, then the other side); per ordered pair (j -> l) the
// number of terms holding both (and, in c0, those with j as l's partner);
// padded entries of the sliced-ELL gather blocks of one sample
constexpr int kSlice = 64;
void term_triple(const int16_t* q, int t, int* x);
void pair_counts(const rlpt_graph* g, std::vector<uint32_t>* cnt, std::vector<uint32_t>* c0);
size_t ell_entries(const rlpt_graph* g, const std::vector<uint32_t>& cnt);

void tune_record(const rlpt_tile& t);
bool tune_choose(const std::map<int, int>& counts, int precision, int shared, int* block,
                 std::map<int, int>* copies);

// ----------------------------------------------------------------- device-side descriptors
struct SampleDev {
    int32_t N;
    int32_t n_steps;       // two-mode updates per sweep, N / 2
    uint32_t mode_base;    // offset of this sample's mode_start / chunk_start block (N + 1 values)
    uint32_t pad0;
    int64_t amp_base;      // complex offset of the sample's first copy
    int64_t quad_base;     // offset into the by-term arrays
    int64_t n_quads;
    int64_t pair_base;     // offset of this sample's pair_start block (N*N + 1 values)
    int64_t ell_base;      // offset of this sample's ell_start block (N * slices + 1 values)
    int64_t c0_base;       // offset of this sample's c0 block (N*N values)
};

// a unit of work of the sweep kernel: n_copies consecutive copies of one sample
struct ItemDev {
    int32_t first_copy;
    int32_t n_copies;
    int32_t sample;
    int32_t pad;
};

struct Counters {
    int64_t sweeps_done;
    int64_t swaps_done;
    int32_t error_flags;  // bit0: drift above tolerance, bit1: NaN/Inf
    int32_t pad;
};

// pointers into the caller's workspace
template <typename R>
struct DevPtrs {
    const SampleDev* samples;
    const ItemDev* items;
    const uint32_t* mode_start;
    const uint32_t* idx;
    const R* J;               // per-mode entries, context precision
    const uint32_t* chunk_start;  // chunked layout: absolute chunk index per mode
    const uint8_t* cx;        // chunk partner
    const uint2* cyz;         // chunk (y | z << 8) x 4 as 16-bit halves
    const R* cJ;              // chunk couplings (4 per chunk)
    // cached-field mode: for the ordered pair (j -> k), the entries of k's list
    // whose term also holds j: x | y << 10 | z << 20 | (slot of j) << 30, coupling
    const uint32_t* pair_start;  // absolute entry index per ordered pair, [S][N*N + 1]
    const uint32_t* pidx;
    const R* pJ;
    // cached-field gather on acceptance: for source mode j and a slice of 64
    // target modes, entries in sliced-ELL order [rank/4][target lane][rank%4];
    // entry = the two other members (p1, p2) of a term holding j and the target,
    // c0 = how many leading ranks of (j -> l) have j as l's partner
    const uint32_t* ell_start;  // absolute entry index per (sample, source, slice), + sentinel
    const uint16_t* gidx16;     // p1 | p2 << 8 (chunked layout, N <= 256)
    const uint32_t* gidx32;     // p1 | p2 << 10 (packed layout)
    const R* gJ;
    const uint16_t* c0;         // [S][N*N]
    R* fields;                // cached local fields, interleaved complex [copy][N]
    const ushort4* quads;     // by term (p, s, m, n)
    const double* Jq;         // by term, FP64
    R* amp;                   // interleaved complex [copy][N]
    R* E;                     // running energies
    double* E64;              // last FP64 energies
    double* drift;            // per-copy relative drift at the last recomputation
    int32_t* temp_of;         // [copies]
    int32_t* copy_at;         // [S][reps][T]
    const R* beta;            // [T]
    const double* beta64;     // [T]
    unsigned long long* acc;  // [S][T]
    unsigned long long* swap_acc;  // [S][reps][T-1]
    double* obs;              // accumulators, see ObsLayout
    double* series_e;
    double* series_q;
    double* hist;
    double* hist_I;           // [S][T][bins] total intensity I/N on [0, 1]
    double* spec;             // [S][T][spec_stride] per-mode intensity |a_k|^2 summed over measurements, replicas
    int32_t* meas_cnt;        // [S][T]
    Counters* counters;
    double* rs_part;          // [copies][kResyncParts] partial FP64 energies of a recomputation
};

constexpr int kResyncParts = 8;  // term ranges of one energy recomputation (workgroups per copy group)

// offsets (in doubles) of the [S][T] accumulator blocks inside DevPtrs::obs
enum ObsField { kEN = 0, kESum, kESq, kY2, kY4, kQN, kQSum, kQSq, kQ4, kNumObs };

struct ShapeInfo {
    int32_t n_samples;
    int32_t n_temps;
    int32_t n_reps;
    int32_t copies_per_sample;  // R = n_temps * n_reps
    int32_t n_bins;
    int32_t series_len;
    int32_t shared_pairs;
    int32_t layout;             // ListLayout
    int32_t cached;             // 1: cached local fields (pair lists + updates on acceptance)
    int32_t by_slot;            // items name temperature slots (hottest first), copies found via copy_at
    int32_t rho;                // constraint sum |a|^rho = N: 4 (smoothed cubic) or 2 (spherical)
    int32_t short_lists;        // every list fits one wave's registers: the one-wave-per-copy sweep
    int32_t spec_stride;        // row length of the intensity spectrum accumulator (largest N)
    uint64_t run_seed;
    double renorm_tol;
    double drift_tol;
};

// ----------------------------------------------------------------- launchers (kernels.hip)
struct SweepLaunch {
    int block_threads;
    int n_items;
    int max_copies_per_item;
    int max_N;
    int prefetch;  // chunks per thread held ahead of their step (0: streamed in the step; 1, 2 or 4)
    int split;     // prefetch > 0: half of a copy's waves sum each mode's list
    size_t lds_bytes;
};

size_t sweep_lds_bytes(int precision, int block_threads, int max_copies_per_item, int max_N, int cached,
                       int short_lists);

hipError_t launch_init(int precision, const void* ptrs, const ShapeInfo& sh, int n_copies, int block,
                       hipStream_t st);
// list-stream ceiling of the streaming sweep (FP32, chunked lists): reads what
// one sweep launch reads, nothing else; sink holds n_items x waves floats
hipError_t launch_stream_lists(const void* ptrs, const ShapeInfo& sh, const SweepLaunch& L, int64_t sweep_offset,
                               float* sink, hipStream_t st);
hipError_t launch_sweep(int precision, const void* ptrs, const ShapeInfo& sh, const SweepLaunch& L,
                        int n_sweeps, hipStream_t st);
hipError_t launch_swap(int precision, const void* ptrs, const ShapeInfo& sh, hipStream_t st);
hipError_t launch_tick(const void* ptrs_any, int precision, int64_t d_sweeps, int64_t d_swaps,
                       hipStream_t st);
// mode 0: periodic recomputation (drift check, renormalisation, store E);
// mode 1: FP64 energies into E64 only; mode 2: store E = H without checks
// FP64 energies of every copy into E[n_copies] (device) with the partial sums
// in the library's static device scratch: no allocation, no host transfer.
// hipErrorInvalidValue when n_copies x kResyncParts partials exceed it.
constexpr size_t kStaticScratchBytes = (size_t)2 << 20;
hipError_t static_scratch_address(void** out);
hipError_t launch_energy_static(int precision, const void* ptrs, const ShapeInfo& sh, int n_copies, double* E,
                                hipStream_t st);
hipError_t launch_resync(int precision, const void* ptrs, const ShapeInfo& sh, int n_copies, int mode,
                         hipStream_t st);
hipError_t launch_measure(int precision, const void* ptrs, const ShapeInfo& sh, hipStream_t st);
// recompute the cached local fields of every copy from the per-mode lists
hipError_t launch_fields_all(int precision, const void* ptrs, const ShapeInfo& sh, int n_copies, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_fields_sh(int precision, const void* ptrs, const ShapeInfo& sh, int copy, int sample,
                            double* F_dev, hipStream_t st);
hipError_t launch_pair_dE_sh(int precision, const void* ptrs, const ShapeInfo& sh, int copy, int sample, int n,
                             const int32_t* jk_dev, const double* new_dev, double* dE_dev, hipStream_t st);
hipError_t launch_convert_state(int precision, void* amp_ctx, double* buf, int64_t n_complex, int to_ctx,
                                hipStream_t st);

}  // namespace rlpt
