// Device kernels of librlpt for CDNA4 (gfx950): initial draw, the sweep
// (local fields + two-mode Metropolis update), replica exchange, FP64 energy
// recomputation, observables, and the test hooks that reuse the sweep's field
// code.  Method: Benedetti & Leuzzi, arXiv 2511.13508, sec. III.A.
//
// Sweep kernel layout
//   * one workgroup runs an "item": n_copies copies of one disorder sample;
//     each copy is served by waves_per_copy = (block/64)/n_copies waves;
//   * a copy's amplitudes live in LDS for the whole launch;
//   * the per-mode lists (packed x|y<<10|z<<20 and J) stream from HBM with
//     16-byte loads, 4 entries per lane per load, coalesced across the wave;
//   * the state-independent parts of each step (pair, phases, sqrt(cos),
//     sqrt(sin), acceptance uniform) are drawn in parallel at the start of a
//     sweep into LDS tables;
//   * per step: barrier, both fields over the two lists on one snapshot
//     (a_j already replaced by its proposal), wave reduction by shuffles,
//     cross-wave sum in LDS, barrier, then one lane decides, updates LDS and
//     prepares the next step's snapshot.
#include <hip/hip_runtime.h>

#include <mutex>
#include <math.h>

#include "internal.hpp"
#include "philox.hpp"

namespace rlpt {
namespace {

template <typename R>
struct V2;
template <>
struct V2<float> {
    using T = float2;
};
template <>
struct V2<double> {
    using T = double2;
};
template <typename R>
using R2 = typename V2<R>::T;

template <typename R>
__device__ inline R2<R> mk2(R x, R y) {
    R2<R> v;
    v.x = x;
    v.y = y;
    return v;
}

template <typename R>
__device__ inline R pi_v() {
    return (R)3.14159265358979323846;
}

__device__ inline void sincos_r(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ inline void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }

// cross-lane moves within rows of 16 lanes (DPP: quad_perm [1,0,3,2] = 0xB1,
// [2,3,0,1] = 0x4E, row_half_mirror = 0x141, row_mirror = 0x140) and reads of
// one lane's value into every lane (v_readlane, the lane index wave-uniform)
template <int CTRL>
__device__ inline float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ inline float read_lane(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ inline double read_lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline int read_lane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline uint32_t read_lane(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }

// sum over each row of 16 lanes, in every lane of the row
template <typename R>
__device__ inline R row_sum(R v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    v += dpp_move<0x140>(v);
    return v;
}

// row broadcasts (DPP row_bcast:15 = 0x142 into rows 1 and 3, row_bcast:31 =
// 0x143 into rows 2 and 3); lanes of the other rows receive 0
template <int CTRL, int ROWS>
__device__ inline float dpp_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ inline double dpp_bcast(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// sum over the wave, the same value in every lane (all lanes active)
template <typename R>
__device__ inline R wave_sum(R v) {
    v = row_sum(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// the same sum, valid in lane 63 only, without lane reads: rows 1 and 3 add
// the totals of rows 0 and 2, then row 3 adds row 1's; (r3 + r2) + (r1 + r0)
// rounds exactly as wave_sum's (r0 + r1) + (r2 + r3)
template <typename R>
__device__ inline R wave_sum_last(R v) {
    v = row_sum(v);
    v += dpp_bcast<0x142, 0xA>(v);
    v += dpp_bcast<0x143, 0xC>(v);
    return v;
}

// contribution J conj(a_x) a_y a_z of one packed entry
template <typename R>
__device__ inline void field_term(uint32_t e, R j, const R2<R>* __restrict__ a, R& fr, R& fi) {
    const R2<R> ax = a[e & 1023u];
    const R2<R> ay = a[(e >> 10) & 1023u];
    const R2<R> az = a[e >> 20];
    const R pr = ax.x * ay.x + ax.y * ay.y;
    const R pi = ax.x * ay.y - ax.y * ay.x;
    const R qr = pr * az.x - pi * az.y;
    const R qi = pr * az.y + pi * az.x;
    fr += j * qr;
    fi += j * qi;
}

template <typename R>
struct J4;
template <>
struct J4<float> {
    using T = float4;
};
template <>
struct J4<double> {
    using T = double4;
};

// partial field of one mode's list, entries [beg, end) (multiples of 4),
// thread t of nt threads takes every nt-th group of 4 entries
template <typename R>
__device__ inline void field_partial(const uint32_t* __restrict__ idx, const R* __restrict__ J, uint32_t beg,
                                     uint32_t end, const R2<R>* __restrict__ a, int t, int nt, R& fr, R& fi) {
    using JT = typename J4<R>::T;
    const uint4* __restrict__ I4 = reinterpret_cast<const uint4*>(idx + beg);
    const JT* __restrict__ Jv = reinterpret_cast<const JT*>(J + beg);
    const int n4 = (int)((end - beg) >> 2);
    int e = t;
    for (; e + nt < n4; e += 2 * nt) {
        const uint4 i0 = I4[e];
        const JT j0 = Jv[e];
        const uint4 i1 = I4[e + nt];
        const JT j1 = Jv[e + nt];
        field_term<R>(i0.x, j0.x, a, fr, fi);
        field_term<R>(i0.y, j0.y, a, fr, fi);
        field_term<R>(i0.z, j0.z, a, fr, fi);
        field_term<R>(i0.w, j0.w, a, fr, fi);
        field_term<R>(i1.x, j1.x, a, fr, fi);
        field_term<R>(i1.y, j1.y, a, fr, fi);
        field_term<R>(i1.z, j1.z, a, fr, fi);
        field_term<R>(i1.w, j1.w, a, fr, fi);
    }
    if (e < n4) {
        const uint4 i0 = I4[e];
        const JT j0 = Jv[e];
        field_term<R>(i0.x, j0.x, a, fr, fi);
        field_term<R>(i0.y, j0.y, a, fr, fi);
        field_term<R>(i0.z, j0.z, a, fr, fi);
        field_term<R>(i0.w, j0.w, a, fr, fi);
    }
}

// chunked layout: a chunk holds 4 entries sharing the partner x; the field
// contribution is conj(a_x) * sum_i J_i a_{y_i} a_{z_i}
template <typename R>
__device__ inline void chunk_pair(uint32_t v, R j, const R2<R>* __restrict__ a, R& gr, R& gi) {
    const R2<R> ay = a[v & 0xffu];
    const R2<R> az = a[(v >> 8) & 0xffu];
    gr += j * (ay.x * az.x - ay.y * az.y);
    gi += j * (ay.x * az.y + ay.y * az.x);
}

template <typename R>
__device__ inline void chunk_term(uint32_t x, uint2 yz, typename J4<R>::T j, const R2<R>* __restrict__ a, R& fr,
                                  R& fi) {
    R gr = 0, gi = 0;
    chunk_pair<R>(yz.x & 0xffffu, j.x, a, gr, gi);
    chunk_pair<R>(yz.x >> 16, j.y, a, gr, gi);
    chunk_pair<R>(yz.y & 0xffffu, j.z, a, gr, gi);
    chunk_pair<R>(yz.y >> 16, j.w, a, gr, gi);
    const R2<R> ax = a[x];
    fr += ax.x * gr + ax.y * gi;
    fi += ax.x * gi - ax.y * gr;
}

template <typename R>
__device__ inline void field_partial_chunk(const uint8_t* __restrict__ cx, const uint2* __restrict__ cyz,
                                           const R* __restrict__ cJ, uint32_t beg, uint32_t end,
                                           const R2<R>* __restrict__ a, int t, int nt, R& fr, R& fi) {
    using JT = typename J4<R>::T;
    const JT* __restrict__ Jv = reinterpret_cast<const JT*>(cJ);
    uint32_t c = beg + t;
    for (; c + nt < end; c += 2 * nt) {
        const uint32_t x0 = cx[c], x1 = cx[c + nt];
        const uint2 y0 = cyz[c], y1 = cyz[c + nt];
        const JT j0 = Jv[c], j1 = Jv[c + nt];
        chunk_term<R>(x0, y0, j0, a, fr, fi);
        chunk_term<R>(x1, y1, j1, a, fr, fi);
    }
    if (c < end) chunk_term<R>(cx[c], cyz[c], Jv[c], a, fr, fi);
}

// partial field of mode l of sample sd in the context's list layout
template <typename R, int LAYOUT>
__device__ inline void mode_field(const DevPtrs<R>& P, const SampleDev& sd, int l, const R2<R>* __restrict__ a, int t,
                                  int nt, R& fr, R& fi) {
    if constexpr (LAYOUT == kLayoutChunked) {
        const uint32_t* cs = P.chunk_start + sd.mode_base;
        field_partial_chunk<R>(P.cx, P.cyz, P.cJ, cs[l], cs[l + 1], a, t, nt, fr, fi);
    } else {
        const uint32_t* ms = P.mode_start + sd.mode_base;
        field_partial<R>(P.idx, P.J, ms[l], ms[l + 1], a, t, nt, fr, fi);
    }
}

// the same from list bounds staged in LDS (lb[l], lb[l + 1] for mode l): the
// step's first global load is then the list itself
template <typename R, int LAYOUT>
__device__ inline void mode_field_lds(const DevPtrs<R>& P, const uint32_t* lb, int l, const R2<R>* __restrict__ a,
                                      int t, int nt, R& fr, R& fi) {
    if constexpr (LAYOUT == kLayoutChunked)
        field_partial_chunk<R>(P.cx, P.cyz, P.cJ, lb[l], lb[l + 1], a, t, nt, fr, fi);
    else
        field_partial<R>(P.idx, P.J, lb[l], lb[l + 1], a, t, nt, fr, fi);
}

// workgroup barrier that waits for LDS operations only (s_waitcnt lgkmcnt(0)
// with vmcnt and expcnt at their maxima, 0xC07F): global loads issued before
// it stay in flight.  Only for loops whose global memory traffic is loads.
__device__ inline void block_sync_lds() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// list chunks of one mode held in registers ahead of their step: thread t of a
// group of nt owns chunks beg + t + m * nt, m < PF (the host picks PF so that
// every list of the launch fits); consumed in the order the streaming loop
// of field_partial_chunk would take them
template <typename R, int PF>
struct ChunkRegs {
    uint32_t x[PF];
    uint2 yz[PF];
    typename J4<R>::T J[PF];
    uint32_t n;  // chunks of this thread
};

template <typename R, int PF>
__device__ inline void chunk_prefetch(const DevPtrs<R>& P, const uint32_t* lb, int l, int t, int nt,
                                      ChunkRegs<R, PF>& rg) {
    using JT = typename J4<R>::T;
    const uint32_t beg = lb[l], end = lb[l + 1];
    const JT* __restrict__ Jv = reinterpret_cast<const JT*>(P.cJ);
    rg.n = 0;
#pragma unroll
    for (int m = 0; m < PF; ++m) {
        const uint32_t c = beg + t + (uint32_t)m * nt;
        if (c < end) {
            rg.x[m] = P.cx[c];
            rg.yz[m] = P.cyz[c];
            rg.J[m] = Jv[c];
            rg.n = m + 1;
        }
    }
}

template <typename R, int PF>
__device__ inline void chunk_consume(const ChunkRegs<R, PF>& rg, const R2<R>* __restrict__ a, R& fr, R& fi) {
#pragma unroll
    for (int m = 0; m < PF; ++m)
        if ((uint32_t)m < rg.n) chunk_term<R>(rg.x[m], rg.yz[m], rg.J[m], a, fr, fi);
}

// energy change of the two-mode update from the two fields of one snapshot:
// dE = -2 Re(conj(aj_new - aj_old) F_j) - 2 Re(conj(ak_new - ak_old) F_k)
template <typename R>
__device__ inline R pair_delta(R2<R> ajo, R2<R> ajn, R2<R> ako, R2<R> akn, R2<R> Fj, R2<R> Fk) {
    const R djr = ajn.x - ajo.x, dji = ajn.y - ajo.y;
    const R dkr = akn.x - ako.x, dki = akn.y - ako.y;
    return (R)-2 * (djr * Fj.x + dji * Fj.y) - (R)2 * (dkr * Fk.x + dki * Fk.y);
}

// state-independent part of step s of sweep w for one copy (sec. III.A):
// distinct j, k; unit phasors of the new phases; sqrt(cos theta), sqrt(sin theta);
// acceptance uniform
template <typename R>
struct StepDraw {
    int32_t jk;  // j | k << 16
    R ejr, eji, ekr, eki, cj, sk, u;
};

template <typename R>
__device__ inline StepDraw<R> draw_step(uint64_t seed, int64_t pair_stream, int64_t copy_id, int64_t sweep,
                                        int step, int N, int rho) {
    const Philox4 wp = philox4x64((uint64_t)step, (uint64_t)sweep, (uint64_t)pair_stream, 0, seed, kTagPair);
    const Philox4 wm = philox4x64((uint64_t)step, (uint64_t)sweep, (uint64_t)copy_id, 0, seed, kTagMove);
    const int j = index_below(wp.v[0], N);
    int k = index_below(wp.v[1], N - 1);
    k += (k >= j) ? 1 : 0;
    StepDraw<R> d;
    d.jk = j | (k << 16);
    const R two_pi = (R)2 * pi_v<R>();
    R s, c;
    sincos_r(two_pi * uniform01<R>(wm.v[0]), &s, &c);
    d.ejr = c;
    d.eji = s;
    sincos_r(two_pi * uniform01<R>(wm.v[1]), &s, &c);
    d.ekr = c;
    d.eki = s;
    if (rho == 2) {  // sin^2 theta uniform: A_j' = K sqrt(1 - u), A_k' = K sqrt(u)
        const R u = uniform01<R>(wm.v[2]);
        d.cj = sqrt((R)1 - u);
        d.sk = sqrt(u);
    } else {  // theta uniform: A_j' = K sqrt(cos theta), A_k' = K sqrt(sin theta)
        sincos_r((R)0.5 * pi_v<R>() * uniform01<R>(wm.v[2]), &s, &c);
        d.cj = sqrt(c > (R)0 ? c : (R)0);
        d.sk = sqrt(s > (R)0 ? s : (R)0);
    }
    d.u = uniform01<R>(wm.v[3]);
    return d;
}

// LDS bytes of the sample's list bounds (max_N + 1 offsets), ahead of the copy groups
__host__ __device__ inline size_t bounds_bytes(int max_N) { return ((size_t)(max_N + 1) * 4 + 15) & ~(size_t)15; }

// LDS bytes of one copy group: amplitudes of max_N modes + step tables + reduction slots
template <typename R>
__host__ __device__ inline size_t group_bytes(int max_N, int waves_per_block) {
    const size_t amp = (size_t)max_N * 2 * sizeof(R);
    const size_t tab = (size_t)(max_N / 2 + 1) * sizeof(StepDraw<R>);
    const size_t red = (size_t)waves_per_block * 4 * sizeof(R);
    return (amp + tab + red + 15) & ~(size_t)15;
}

// PF > 0 (chunked lists short enough for PF chunks per thread): a step's list
// chunks are loaded into registers two steps earlier, and the step loop's
// barriers wait for LDS only, so the loads stay in flight across two steps'
// reductions, decisions and barriers.  Same chain; with SPLIT each list is
// summed by half of the copy's waves, which groups the partial sums differently
// (FP rounding of the fields, not the method, changes).
template <typename R, int BLOCK, int LAYOUT, int PF, bool SPLIT>
__global__ __launch_bounds__(BLOCK) void k_sweep(DevPtrs<R> P, ShapeInfo sh, int max_N, int n_sweeps) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kWaves = BLOCK / 64;
    const ItemDev it = P.items[blockIdx.x];
    const SampleDev sd = P.samples[it.sample];
    const int N = sd.N, steps = sd.n_steps;
    const int wpc = kWaves / it.n_copies;  // waves per copy
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = wave / wpc;              // copy group of this wave
    const bool active = g < it.n_copies;
    const int gw = wave - g * wpc;         // wave index inside the group
    const int gt = threadIdx.x - g * wpc * 64;
    const int nt = wpc * 64;
    const int gsel = active ? g : 0;
    // halves (SPLIT, with PF > 0; the host sets it only when every item has two
    // or more waves per copy): the copy's first wpc/2 waves sum mode j's list
    // and the others mode k's, so a wave holds one list's chunks and reduces two
    // values, not four; lt of lnt is the thread's place in its half
    constexpr bool halves = SPLIT && PF > 0;
    const bool on_k = halves && gw >= wpc / 2;
    const int lnt = halves ? nt / 2 : nt;
    const int lt = on_k ? gt - lnt : gt;

    uint32_t* lb = reinterpret_cast<uint32_t*>(smem);  // list bounds of the item's sample
    unsigned char* base = smem + bounds_bytes(max_N) + (size_t)gsel * group_bytes<R>(max_N, kWaves);
    R2<R>* a = reinterpret_cast<R2<R>*>(base);
    StepDraw<R>* tab = reinterpret_cast<StepDraw<R>*>(base + (size_t)max_N * 2 * sizeof(R));
    R* red = reinterpret_cast<R*>(base + (size_t)max_N * 2 * sizeof(R) + (size_t)(max_N / 2 + 1) * sizeof(StepDraw<R>));
    {
        const uint32_t* gb = (LAYOUT == kLayoutChunked ? P.chunk_start : P.mode_start) + sd.mode_base;
        for (int i = threadIdx.x; i <= N; i += BLOCK) lb[i] = gb[i];  // visible after the sweep loop's first barrier
    }

    const int c = it.first_copy + gsel;
    const int64_t local = c - (int64_t)it.sample * sh.copies_per_sample;
    R2<R>* amp_g = reinterpret_cast<R2<R>*>(P.amp) + sd.amp_base + local * N;
    if (active)
        for (int i = gt; i < N; i += nt) a[i] = amp_g[i];
    const int t_idx = P.temp_of[c];
    const R beta = P.beta[t_idx];
    R E = P.E[c];
    unsigned int n_acc = 0;
    const int64_t pair_stream = sh.shared_pairs ? (int64_t)it.sample : (int64_t)c;
    const int64_t sweep0 = P.counters->sweeps_done;

    R2<R> ajo = mk2<R>(0, 0), ajn = mk2<R>(0, 0), akn = mk2<R>(0, 0);
    // PF > 0: chunks of steps s (set A for even s, B for odd s) and s + 1 in
    // registers; step s consumes its set and refills it with step s + 2
    using Regs = ChunkRegs<R, (PF > 0 ? PF : 1)>;
    Regs pjA, pkA, pjB, pkB;
    auto run_step = [&](int s, Regs& rj, Regs& rk) {
        if constexpr (PF > 0) block_sync_lds(); else __syncthreads();
        R fjr = 0, fji = 0, fkr = 0, fki = 0;
        if (active) {
            if constexpr (PF > 0) {
                if (halves) {  // this half's list only, in rj
                    R fr = 0, fi = 0;
                    chunk_consume<R, PF>(rj, a, fr, fi);
                    if (s + 2 < steps)
                        chunk_prefetch<R, PF>(P, lb, on_k ? (tab[s + 2].jk >> 16) : (tab[s + 2].jk & 0xffff), lt,
                                              lnt, rj);
                    if (on_k) {
                        fkr = fr;
                        fki = fi;
                    } else {
                        fjr = fr;
                        fji = fi;
                    }
                } else {
                    chunk_consume<R, PF>(rj, a, fjr, fji);
                    chunk_consume<R, PF>(rk, a, fkr, fki);
                    if (s + 2 < steps) {
                        chunk_prefetch<R, PF>(P, lb, tab[s + 2].jk & 0xffff, gt, nt, rj);
                        chunk_prefetch<R, PF>(P, lb, tab[s + 2].jk >> 16, gt, nt, rk);
                    }
                }
            } else {
                const int j = tab[s].jk & 0xffff, k = tab[s].jk >> 16;
                mode_field_lds<R, LAYOUT>(P, lb, j, a, gt, nt, fjr, fji);
                mode_field_lds<R, LAYOUT>(P, lb, k, a, gt, nt, fkr, fki);
            }
        }
        if (halves) {
            const R r0 = wave_sum_last(on_k ? fkr : fjr);
            const R r1 = wave_sum_last(on_k ? fki : fji);
            if (active && lane == 63) {
                red[2 * gw + 0] = r0;
                red[2 * gw + 1] = r1;
            }
        } else {
            fjr = wave_sum_last(fjr);
            fji = wave_sum_last(fji);
            fkr = wave_sum_last(fkr);
            fki = wave_sum_last(fki);
            if (active && lane == 63) {
                red[4 * gw + 0] = fjr;
                red[4 * gw + 1] = fji;
                red[4 * gw + 2] = fkr;
                red[4 * gw + 3] = fki;
            }
        }
        if constexpr (PF > 0) block_sync_lds(); else __syncthreads();
        if (active && gt == 0) {
            R2<R> Fj = mk2<R>(0, 0), Fk = mk2<R>(0, 0);
            if (halves) {
                for (int w = 0; w < wpc / 2; ++w) {
                    Fj.x += red[2 * w + 0];
                    Fj.y += red[2 * w + 1];
                }
                for (int w = wpc / 2; w < wpc; ++w) {
                    Fk.x += red[2 * w + 0];
                    Fk.y += red[2 * w + 1];
                }
            } else {
                for (int w = 0; w < wpc; ++w) {
                    Fj.x += red[4 * w + 0];
                    Fj.y += red[4 * w + 1];
                    Fk.x += red[4 * w + 2];
                    Fk.y += red[4 * w + 3];
                }
            }
            const int j = tab[s].jk & 0xffff, k = tab[s].jk >> 16;
            const R2<R> ako = a[k];
            const R dE = pair_delta<R>(ajo, ajn, ako, akn, Fj, Fk);
            const bool accept = (dE <= (R)0) || (tab[s].u < exp(-beta * dE));
            if (accept) {
                a[k] = akn;
                E += dE;
                ++n_acc;
            } else {
                a[j] = ajo;
            }
            if (s + 1 < steps) {  // snapshot of the next step
                const StepDraw<R> d = tab[s + 1];
                const int j2 = d.jk & 0xffff, k2 = d.jk >> 16;
                ajo = a[j2];
                const R2<R> ako2 = a[k2];
                const R uj = ajo.x * ajo.x + ajo.y * ajo.y, uk = ako2.x * ako2.x + ako2.y * ako2.y;
                const R K = sh.rho == 2 ? sqrt(uj + uk) : sqrt(sqrt(uj * uj + uk * uk));
                ajn = mk2<R>(K * d.cj * d.ejr, K * d.cj * d.eji);
                akn = mk2<R>(K * d.sk * d.ekr, K * d.sk * d.eki);
                a[j2] = ajn;
            }
        }
    };
    for (int sw = 0; sw < n_sweeps; ++sw) {
        __syncthreads();
        if (active)
            for (int s = gt; s < steps; s += nt) tab[s] = draw_step<R>(sh.run_seed, pair_stream, c, sweep0 + sw, s, N, sh.rho);
        __syncthreads();
        if constexpr (PF > 0) {
            if (active && halves) {
                chunk_prefetch<R, PF>(P, lb, on_k ? (tab[0].jk >> 16) : (tab[0].jk & 0xffff), lt, lnt, pjA);
                if (steps > 1)
                    chunk_prefetch<R, PF>(P, lb, on_k ? (tab[1].jk >> 16) : (tab[1].jk & 0xffff), lt, lnt, pjB);
            } else if (active) {
                chunk_prefetch<R, PF>(P, lb, tab[0].jk & 0xffff, gt, nt, pjA);
                chunk_prefetch<R, PF>(P, lb, tab[0].jk >> 16, gt, nt, pkA);
                if (steps > 1) {
                    chunk_prefetch<R, PF>(P, lb, tab[1].jk & 0xffff, gt, nt, pjB);
                    chunk_prefetch<R, PF>(P, lb, tab[1].jk >> 16, gt, nt, pkB);
                }
            }
        }
        if (active && gt == 0) {  // snapshot of step 0
            const int j = tab[0].jk & 0xffff, k = tab[0].jk >> 16;
            ajo = a[j];
            const R2<R> ako = a[k];
            const R uj = ajo.x * ajo.x + ajo.y * ajo.y, uk = ako.x * ako.x + ako.y * ako.y;
            const R K = sh.rho == 2 ? sqrt(uj + uk) : sqrt(sqrt(uj * uj + uk * uk));
            ajn = mk2<R>(K * tab[0].cj * tab[0].ejr, K * tab[0].cj * tab[0].eji);
            akn = mk2<R>(K * tab[0].sk * tab[0].ekr, K * tab[0].sk * tab[0].eki);
            a[j] = ajn;
        }
        int s = 0;
        for (; s + 1 < steps; s += 2) {
            run_step(s, pjA, pkA);
            run_step(s + 1, pjB, pkB);
        }
        if (s < steps) run_step(s, pjA, pkA);
    }
    __syncthreads();
    if (active) {
        for (int i = gt; i < N; i += nt) amp_g[i] = a[i];
        if (gt == 0) {
            P.E[c] = E;
            atomicAdd(&P.acc[(size_t)it.sample * sh.n_temps + t_idx], (unsigned long long)n_acc);
        }
    }
}

// ---------------------------------------------------------------- list-stream ceiling
// Diagnostic for the streaming sweep's roofline: the same grid, items, tile
// and LDS footprint (so the same workgroups per CU) as k_sweep, the same pair
// draws, and every list chunk of every step read in the same order by the
// same threads, the copy's threads meeting at a barrier before each step as
// in the sweep -- but nothing else: no amplitudes, no arithmetic beyond a
// checksum, no reductions, no decision.  Its rate is what the memory
// hierarchy (L2, Infinity Cache, HBM) delivers for the sweep's access
// schedule, the ceiling its list stream can reach.  (Without the per-step
// barrier the waves of a copy drift apart and the same reads took 17 %
// longer at N = 256.)  Launch w reads the draws of sweep (sweeps done + sweep_offset + w);
// nothing of the chain is changed.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_stream_lists(DevPtrs<float> P, ShapeInfo sh, int max_N,
                                                        int64_t sweep_offset, float* sink) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kWaves = BLOCK / 64;
    const ItemDev it = P.items[blockIdx.x];
    const SampleDev sd = P.samples[it.sample];
    const int N = sd.N, steps = sd.n_steps;
    const int wpc = kWaves / it.n_copies;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = wave / wpc;
    const bool active = g < it.n_copies;
    const int gsel = active ? g : 0;
    const int gt = threadIdx.x - g * wpc * 64, nt = wpc * 64;
    uint32_t* lb = reinterpret_cast<uint32_t*>(smem);
    int32_t* tab = reinterpret_cast<int32_t*>(smem + bounds_bytes(max_N)) + (size_t)gsel * (max_N / 2 + 1);
    for (int i = threadIdx.x; i <= N; i += BLOCK) lb[i] = P.chunk_start[sd.mode_base + i];
    const int c = it.first_copy + gsel;
    const int64_t pair_stream = sh.shared_pairs ? (int64_t)it.sample : (int64_t)c;
    const int64_t sweep = P.counters->sweeps_done + sweep_offset;
    if (active)
        for (int s = gt; s < steps; s += nt) tab[s] = draw_step<float>(sh.run_seed, pair_stream, c, sweep, s, N, sh.rho).jk;
    __syncthreads();
    const float4* __restrict__ Jv = reinterpret_cast<const float4*>(P.cJ);
    float acc = 0.0f;
    uint32_t h = 0;
    for (int s = 0; s < steps; ++s) {
        __syncthreads();
        if (active) {
            const int jk = tab[s];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int l = side ? (jk >> 16) : (jk & 0xffff);
                const uint32_t end = lb[l + 1];
                uint32_t cc = lb[l] + gt;
                for (; cc + nt < end; cc += 2 * nt) {
                    const float4 j0 = Jv[cc], j1 = Jv[cc + nt];
                    const uint2 y0 = P.cyz[cc], y1 = P.cyz[cc + nt];
                    h ^= (uint32_t)P.cx[cc] ^ y0.x ^ y0.y ^ ((uint32_t)P.cx[cc + nt] << 8) ^ y1.x ^ y1.y;
                    acc += (j0.x + j0.y) + (j0.z + j0.w) + (j1.x + j1.y) + (j1.z + j1.w);
                }
                if (cc < end) {
                    const float4 j0 = Jv[cc];
                    const uint2 y0 = P.cyz[cc];
                    h ^= (uint32_t)P.cx[cc] ^ y0.x ^ y0.y;
                    acc += (j0.x + j0.y) + (j0.z + j0.w);
                }
            }
        }
    }
    acc += (float)(h & 0xffu);
    acc = wave_sum(acc);
    if (lane == 0) sink[(size_t)blockIdx.x * kWaves + wave] = acc;
}

// ---------------------------------------------------------------- short lists (sparse graphs)
// When every mode's list is short (sparse mode-locked graphs, a few dozen
// terms per mode) a step is pure latency: load two lists, reduce, decide.
// One wave runs one copy with no workgroup barrier: lanes 0-31 sum F_j, lanes
// 32-63 F_k, each from kShortSlots entries per lane held in registers and
// loaded two steps ahead; each lane keeps the draws of one step of the
// current and the next 64-step chunk in registers, and every lane reads a
// step's draws from the lane holding them.  Same chain, same draws as the
// streaming sweep.  The host takes this path only when no padded list is
// longer than 32 * kShortSlots entries.
constexpr int kShortSlots = 4;

// keep the compiler from moving LDS accesses across a write by one lane that
// all lanes then read (the hardware runs one wave's LDS accesses in order);
// emits no wait, so global loads in flight stay in flight
__device__ inline void wave_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// a step's draws plus the list bounds of its two modes
template <typename R>
struct ShortStep {
    StepDraw<R> d;
    uint32_t bj, ej, bk, ek;
};

template <typename R>
__device__ inline ShortStep<R> step_from_lane(const ShortStep<R>& x, int src) {  // src wave-uniform
    ShortStep<R> o;
    o.d.jk = read_lane(x.d.jk, src);
    o.d.ejr = read_lane(x.d.ejr, src);
    o.d.eji = read_lane(x.d.eji, src);
    o.d.ekr = read_lane(x.d.ekr, src);
    o.d.eki = read_lane(x.d.eki, src);
    o.d.cj = read_lane(x.d.cj, src);
    o.d.sk = read_lane(x.d.sk, src);
    o.d.u = read_lane(x.d.u, src);
    o.bj = read_lane(x.bj, src);
    o.ej = read_lane(x.ej, src);
    o.bk = read_lane(x.bk, src);
    o.ek = read_lane(x.ek, src);
    return o;
}

template <typename R, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_sweep_short(DevPtrs<R> P, ShapeInfo sh, int max_N, int n_sweeps) {
    extern __shared__ __align__(16) unsigned char smem[];
    const ItemDev it = P.items[blockIdx.x];
    const SampleDev sd = P.samples[it.sample];
    const int N = sd.N, steps = sd.n_steps;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave >= it.n_copies) return;  // no workgroup barrier below: idle waves may leave
    R2<R>* a = reinterpret_cast<R2<R>*>(smem) + (size_t)wave * max_N;
    const int c = it.first_copy + wave;
    const int64_t local = c - (int64_t)it.sample * sh.copies_per_sample;
    R2<R>* amp_g = reinterpret_cast<R2<R>*>(P.amp) + sd.amp_base + local * N;
    for (int i = lane; i < N; i += 64) a[i] = amp_g[i];
    wave_sync();
    const int t_idx = P.temp_of[c];
    const R beta = P.beta[t_idx];
    R E = P.E[c];
    unsigned int n_acc = 0;
    const int64_t pair_stream = sh.shared_pairs ? (int64_t)it.sample : (int64_t)c;
    const int64_t sweep0 = P.counters->sweeps_done;
    const uint32_t* ms = P.mode_start + sd.mode_base;
    const uint32_t first = ms[0];
    const int half = lane >> 5, hl = lane & 31;

    // list entries two steps ahead: even steps use buffer A, odd steps B; the
    // loads for step s + 2 go into the buffer step s has just used, so each
    // load has two steps to arrive and no register is copied
    uint32_t pvA[kShortSlots], pvB[kShortSlots];
    R pjA[kShortSlots], pjB[kShortSlots];
    uint32_t inA = 0, inB = 0;  // slots holding a real entry (bit i)
    auto load = [&](const ShortStep<R>& t, uint32_t* pv, R* pj, uint32_t& in) {  // lanes 0-31: list of j, 32-63: of k
        const uint32_t b = half ? t.bk : t.bj, e = half ? t.ek : t.ej;
        in = 0;
#pragma unroll
        for (int i = 0; i < kShortSlots; ++i) {
            // past the end: the sample's first entry (its modes are < N, so the
            // amplitudes read are this copy's), masked out where it is used, so
            // that nothing here waits for the load
            const uint32_t x = b + (uint32_t)(hl + 32 * i);
            const uint32_t xs = x < e ? x : first;
            in |= (x < e ? 1u : 0u) << i;
            pv[i] = P.idx[xs];
            pj[i] = P.J[xs];
        }
    };
    // draws of the current and the next 64-step chunk, one step per lane (a
    // lane past the last step draws the last step again: every lane loads on
    // every path, so the wait counts stay exact and nothing waits early)
    ShortStep<R> mine, mine2;
    auto draw_chunk = [&](ShortStep<R>& x, int sw, int base) {
        const int t = min(base + lane, steps - 1);
        x.d = draw_step<R>(sh.run_seed, pair_stream, c, sweep0 + sw, t, N, sh.rho);
        const int j = x.d.jk & 0xffff, k = x.d.jk >> 16;
        x.bj = ms[j];
        x.ej = ms[j + 1];
        x.bk = ms[k];
        x.ek = ms[k + 1];
    };
    R2<R> ajo = mk2<R>(0, 0), ajn = mk2<R>(0, 0), akn = mk2<R>(0, 0);
    auto snapshot = [&](const StepDraw<R>& d) {  // every lane computes it; lane 0 stores a_j'
        const int j = d.jk & 0xffff, k = d.jk >> 16;
        ajo = a[j];
        const R2<R> ako = a[k];
        const R uj = ajo.x * ajo.x + ajo.y * ajo.y, uk = ako.x * ako.x + ako.y * ako.y;
        const R K = sh.rho == 2 ? sqrt(uj + uk) : sqrt(sqrt(uj * uj + uk * uk));
        ajn = mk2<R>(K * d.cj * d.ejr, K * d.cj * d.eji);
        akn = mk2<R>(K * d.sk * d.ekr, K * d.sk * d.eki);
        wave_sync();
        if (lane == 0) a[j] = ajn;
        wave_sync();
    };
    ShortStep<R> cur, nxt;
    // one step: fields from (pv, pj), then the loads of step s + 2 into them
    auto step = [&](int s, int base, uint32_t* pv, R* pj, uint32_t& in) {
        const int j = cur.d.jk & 0xffff, k = cur.d.jk >> 16;
        // fields on the snapshot (a_j new, a_k old): lanes 0-31 F_j, 32-63 F_k
        R fr = 0, fi = 0;
#pragma unroll
        for (int i = 0; i < kShortSlots; ++i) field_term<R>(pv[i], (in >> i) & 1u ? pj[i] : (R)0, a, fr, fi);
        // step s + 2 (past the last step: the last step again, loaded harmlessly)
        const int t = min(s + 2, steps - 1);
        const ShortStep<R> nxt2 = step_from_lane(t < base + 64 ? mine : mine2, t & 63);
        load(nxt2, pv, pj, in);
        fr = row_sum(fr);
        fi = row_sum(fi);
        const R Fjr = read_lane(fr, 0) + read_lane(fr, 16), Fji = read_lane(fi, 0) + read_lane(fi, 16);
        const R Fkr = read_lane(fr, 32) + read_lane(fr, 48), Fki = read_lane(fi, 32) + read_lane(fi, 48);
        // every lane takes the same decision; lane 0 writes LDS
        const R2<R> ako = a[k];
        const R dE = pair_delta<R>(ajo, ajn, ako, akn, mk2<R>(Fjr, Fji), mk2<R>(Fkr, Fki));
        const bool accept = (dE <= (R)0) || (cur.d.u < exp(-beta * dE));
        wave_sync();
        if (lane == 0) {
            if (accept) a[k] = akn;
            else a[j] = ajo;
        }
        if (accept) {
            E += dE;
            ++n_acc;
        }
        wave_sync();
        if (s + 1 < steps) snapshot(nxt.d);
        cur = nxt;
        nxt = nxt2;
    };
    for (int sw = 0; sw < n_sweeps; ++sw) {
        draw_chunk(mine, sw, 0);
        draw_chunk(mine2, sw, 64);
        cur = step_from_lane(mine, 0);
        nxt = step_from_lane(mine, min(1, steps - 1));
        load(cur, pvA, pjA, inA);
        load(nxt, pvB, pjB, inB);
        snapshot(cur.d);
        for (int base = 0; base < steps; base += 64) {
            const int end = min(base + 64, steps);
            for (int s = base; s < end; s += 2) {  // base is even: step s uses A, s + 1 uses B
                step(s, base, pvA, pjA, inA);
                if (s + 1 < end) step(s + 1, base, pvB, pjB, inB);
            }
            mine = mine2;
            draw_chunk(mine2, sw, base + 128);
        }
    }
    wave_sync();
    for (int i = lane; i < N; i += 64) amp_g[i] = a[i];
    if (lane == 0) {
        P.E[c] = E;
        atomicAdd(&P.acc[(size_t)it.sample * sh.n_temps + t_idx], (unsigned long long)n_acc);
    }
}

// ---------------------------------------------------------------- cached local fields
// With every copy's fields kept up to date, the energy change of a two-mode
// move needs F_j, F_k and, for the one-snapshot rule, the change of F_k from
// the new a_j: a short list of the terms holding both j and k.  Only an
// accepted move touches the other fields: every mode l sharing a term with j
// or k gains the change of its field, gathered per target from the sliced-ELL
// block of j (with a_k old) and of k (with a_j new), one lane per target, so
// no two lanes ever add to the same field.  Same chain, same draws as the
// streaming sweep.

// J conj(u) v w of one pair-list entry with j's slot holding d
template <typename R>
__device__ inline void pair_term(uint32_t v, R J, const R2<R>* __restrict__ a, R2<R> d, R& cr, R& ci) {
    const uint32_t role = v >> 30;
    const R2<R> u = role == 0 ? d : a[v & 1023u];
    const R2<R> w1 = role == 1 ? d : a[(v >> 10) & 1023u];
    const R2<R> w2 = role == 2 ? d : a[(v >> 20) & 1023u];
    const R pr = u.x * w1.x + u.y * w1.y, pi = u.x * w1.y - u.y * w1.x;
    cr += J * (pr * w2.x - pi * w2.y);
    ci += J * (pr * w2.y + pi * w2.x);
}

constexpr int kPairPrefetch = 8;  // pair-list entries per lane loaded one step ahead

// groups of 4 gather entries loaded before any is used (fewer with the wider
// 32-bit indices of the packed layout, to stay within three waves per SIMD)
template <int LAYOUT>
constexpr int kGatherBatch = LAYOUT == kLayoutChunked ? 8 : 4;

template <int LAYOUT>
struct GatherIdx;
template <>
struct GatherIdx<kLayoutChunked> {
    using T = uint2;  // 4 x (p1 | p2 << 8)
    __device__ static uint32_t p1(const T& v, int i) { return (i < 2 ? v.x : v.y) >> (16 * (i & 1)) & 0xffu; }
    __device__ static uint32_t p2(const T& v, int i) { return (i < 2 ? v.x : v.y) >> (16 * (i & 1) + 8) & 0xffu; }
};
template <>
struct GatherIdx<kLayoutPacked> {
    using T = uint4;  // 4 x (p1 | p2 << 10)
    __device__ static uint32_t word(const T& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
    __device__ static uint32_t p1(const T& v, int i) { return word(v, i) & 1023u; }
    __device__ static uint32_t p2(const T& v, int i) { return word(v, i) >> 10; }
};

// change of the field of target l = 64 * slice + lane from source mode src
// moving by d: over the ranks of (src -> l), J conj(d) a_p1 a_p2 when src is
// l's partner (the first c0 ranks), else J conj(a_p1) d a_p2.  With
// P = conj(d) a_p1 the second form is conj(P) a_p2, so each entry costs one
// sign flip instead of a choice of operands.  Loads go out kGatherBatch
// groups at a time, ahead of every use.
template <typename R, int LAYOUT>
__device__ inline void gather_slice(const DevPtrs<R>& P, const SampleDev& sd, int N, int src, R2<R> d, int slice,
                                    int part, int parts, int lane, const R2<R>* __restrict__ a, R& fr, R& fi) {
    const int ns = (N + 63) >> 6;
    const int w = min(64, N - 64 * slice);
    if (lane >= w) return;
    const uint32_t* es = P.ell_start + sd.ell_base + (int64_t)src * ns + slice;
    const uint32_t nall = (es[1] - es[0]) / (4u * (uint32_t)w);
    // this part's share of the groups: [part, part + 1) * nall / parts
    const uint32_t qb = (uint32_t)part * nall / (uint32_t)parts, qe = (uint32_t)(part + 1) * nall / (uint32_t)parts;
    const uint32_t b0 = es[0] + 4u * (uint32_t)w * qb, nq = qe - qb;
    const int l = 64 * slice + lane;
    const uint32_t c0 = P.c0[sd.c0_base + (int64_t)src * N + l];
    using JT = typename J4<R>::T;
    using GI = GatherIdx<LAYOUT>;
    using IT = typename GI::T;
    const IT* ip = reinterpret_cast<const IT*>(LAYOUT == kLayoutChunked ? (const void*)P.gidx16 : (const void*)P.gidx32);
    const JT* jp = reinterpret_cast<const JT*>(P.gJ);
    const uint32_t g0 = b0 / 4u + (uint32_t)lane;  // this lane's group q sits at g0 + q * w
    if (nq == 0) return;
    for (uint32_t q0 = 0; q0 < nq; q0 += kGatherBatch<LAYOUT>) {
        IT iv[kGatherBatch<LAYOUT>];
        JT jv[kGatherBatch<LAYOUT>];
#pragma unroll
        for (int u = 0; u < kGatherBatch<LAYOUT>; ++u) {
            const uint32_t q = q0 + u < nq ? q0 + u : nq - 1;
            iv[u] = ip[g0 + q * (uint32_t)w];
            jv[u] = jp[g0 + q * (uint32_t)w];
        }
#pragma unroll
        for (int u = 0; u < kGatherBatch<LAYOUT>; ++u) {
            // past the end: the clamped group again, weighted 0 (no branch, so the
            // loads above stay ahead of every use)
            const R m = q0 + u < nq ? (R)1 : (R)0;
            const R jj[4] = {m * jv[u].x, m * jv[u].y, m * jv[u].z, m * jv[u].w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const R2<R> x1 = a[GI::p1(iv[u], i)], x2 = a[GI::p2(iv[u], i)];
                const R pr = d.x * x1.x + d.y * x1.y;
                const R pim = d.x * x1.y - d.y * x1.x;
                const R pi = 4 * (qb + q0 + u) + (uint32_t)i < c0 ? pim : -pim;
                fr += jj[i] * (pr * x2.x - pi * x2.y);
                fi += jj[i] * (pr * x2.y + pi * x2.x);
            }
        }
    }
}

// LDS bytes of one copy group of the cached sweep: the streaming group plus
// the fields, the per-step pair-list ranges, d_j, d_k and the decision flag
template <typename R>
__host__ __device__ inline size_t group_bytes_cached(int max_N, int waves_per_block) {
    // fields, d_j and d_k, per-step pair-list ranges, flags, second part's sums
    const size_t extra = (size_t)max_N * 2 * sizeof(R) + 4 * sizeof(R) + (size_t)(max_N / 2 + 1) * sizeof(uint2) + 16 +
                         (size_t)max_N * 2 * sizeof(R);
    return (group_bytes<R>(max_N, waves_per_block) + extra + 15) & ~(size_t)15;
}

template <typename R, int BLOCK, int LAYOUT>
__global__ __launch_bounds__(BLOCK) void k_sweep_cached(DevPtrs<R> P, ShapeInfo sh, int max_N, int n_sweeps) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kWaves = BLOCK / 64;
    const ItemDev it = P.items[blockIdx.x];
    const SampleDev sd = P.samples[it.sample];
    const int N = sd.N, steps = sd.n_steps;
    const int wpc = kWaves / it.n_copies;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = wave / wpc;
    const bool active = g < it.n_copies;
    const int gw = wave - g * wpc;
    const int gt = threadIdx.x - g * wpc * 64;
    const int nt = wpc * 64;
    const int gsel = active ? g : 0;
    const int ns = (N + 63) >> 6;
    // field update of an accepted move: two waves share each slice when the
    // group has the waves to spare; the second leaves its sums in LDS and the
    // first adds both in a fixed order (runs are bitwise reproducible)
    const int parts = max(1, min(2, wpc / ns));

    unsigned char* base = smem + (size_t)gsel * group_bytes_cached<R>(max_N, kWaves);
    R2<R>* a = reinterpret_cast<R2<R>*>(base);
    StepDraw<R>* tab = reinterpret_cast<StepDraw<R>*>(base + (size_t)max_N * 2 * sizeof(R));
    unsigned char* after = base + group_bytes<R>(max_N, kWaves);
    R* F = reinterpret_cast<R*>(after);
    after += (size_t)max_N * 2 * sizeof(R);
    R2<R>* snap = reinterpret_cast<R2<R>*>(after);  // [0] = d_j, [1] = d_k
    after += 4 * sizeof(R);
    uint2* pr = reinterpret_cast<uint2*>(after);  // pair-list range of each step
    after += (size_t)(max_N / 2 + 1) * sizeof(uint2);
    int* flag = reinterpret_cast<int*>(after);  // decisions of even and odd steps
    after += 16;
    R2<R>* pbuf = reinterpret_cast<R2<R>*>(after);  // second part's field changes

    int c = it.first_copy + gsel;
    if (sh.by_slot) {  // slot order within the sample: temperature descending, then ladder
        const int idx = c - it.sample * sh.copies_per_sample;
        const int t = sh.n_temps - 1 - idx / sh.n_reps, r = idx % sh.n_reps;
        c = P.copy_at[((size_t)it.sample * sh.n_reps + r) * sh.n_temps + t];
    }
    const int64_t local = c - (int64_t)it.sample * sh.copies_per_sample;
    R2<R>* amp_g = reinterpret_cast<R2<R>*>(P.amp) + sd.amp_base + local * N;
    R* fld_g = P.fields + 2 * (sd.amp_base + local * N);
    if (active)
        for (int i = gt; i < N; i += nt) {
            a[i] = amp_g[i];
            F[2 * i] = fld_g[2 * i];
            F[2 * i + 1] = fld_g[2 * i + 1];
        }
    const int t_idx = P.temp_of[c];
    const R beta = P.beta[t_idx];
    R E = P.E[c];
    unsigned int n_acc = 0;
    const int64_t pair_stream = sh.shared_pairs ? (int64_t)it.sample : (int64_t)c;
    const int64_t sweep0 = P.counters->sweeps_done;
    const uint32_t* ps = P.pair_start + sd.pair_base;
    const uint32_t pfirst = ps[0];  // the sample's first pair-list entry

    // wave 0 keeps the next step's pair-list entries in registers
    uint32_t pv[kPairPrefetch];
    R pj[kPairPrefetch];
    uint32_t pin = 0;
    auto prefetch = [&](int s) {
        const uint2 r = pr[s];
        pin = 0;
#pragma unroll
        for (int i = 0; i < kPairPrefetch; ++i) {
            // past the end: the sample's first pair-list entry (modes < N, so the
            // amplitudes read are this copy's), masked out where it is used
            // (nothing here waits for the loads)
            const uint32_t e = r.x + (uint32_t)(lane + 64 * i);
            const uint32_t es = e < r.y ? e : pfirst;
            pin |= (e < r.y ? 1u : 0u) << i;
            pv[i] = P.pidx[es];
            pj[i] = P.pJ[es];
        }
    };
    R2<R> ajo = mk2<R>(0, 0), akn = mk2<R>(0, 0);
    auto prepare = [&](int s) {  // snapshot of step s (one lane)
        const StepDraw<R> d = tab[s];
        const int j2 = d.jk & 0xffff, k2 = d.jk >> 16;
        ajo = a[j2];
        const R2<R> ako2 = a[k2];
        const R uj = ajo.x * ajo.x + ajo.y * ajo.y, uk = ako2.x * ako2.x + ako2.y * ako2.y;
        const R K = sh.rho == 2 ? sqrt(uj + uk) : sqrt(sqrt(uj * uj + uk * uk));
        const R2<R> ajn = mk2<R>(K * d.cj * d.ejr, K * d.cj * d.eji);
        akn = mk2<R>(K * d.sk * d.ekr, K * d.sk * d.eki);
        a[j2] = ajn;
        snap[0] = mk2<R>(ajn.x - ajo.x, ajn.y - ajo.y);
        snap[1] = mk2<R>(akn.x - ako2.x, akn.y - ako2.y);
    };
    // One barrier per rejected step: wave 0 decides, prepares the next
    // snapshot and decides again without waiting; the other waves only learn
    // each decision (flags alternate between two slots, so a fast wave 0
    // never overwrites one still being read).  An accepted step adds the
    // field update and one more barrier; with several copies per workgroup
    // that barrier is taken every step, keeping barriers block-uniform.
    const bool lone = it.n_copies == 1;
    for (int sw = 0; sw < n_sweeps; ++sw) {
        __syncthreads();
        if (active)
            for (int s = gt; s < steps; s += nt) {
                const StepDraw<R> d = draw_step<R>(sh.run_seed, pair_stream, c, sweep0 + sw, s, N, sh.rho);
                tab[s] = d;
                const int64_t pk = (int64_t)(d.jk & 0xffff) * N + (d.jk >> 16);
                pr[s] = make_uint2(ps[pk], ps[pk + 1]);
            }
        __syncthreads();
        if (active && gt == 0) prepare(0);
        __builtin_amdgcn_wave_barrier();
        if (active && gw == 0) prefetch(0);
        for (int s = 0; s < steps; ++s) {
            const int j = tab[s].jk & 0xffff, k = tab[s].jk >> 16;
            if (active && gw == 0) {
                const R2<R> dj = snap[0];
                R cr = 0, ci = 0;
#pragma unroll
                for (int i = 0; i < kPairPrefetch; ++i) pair_term<R>(pv[i], (pin >> i) & 1u ? pj[i] : (R)0, a, dj, cr, ci);
                const uint2 r = pr[s];
                for (uint32_t e = r.x + 64 * kPairPrefetch + lane; e < r.y; e += 64) pair_term<R>(P.pidx[e], P.pJ[e], a, dj, cr, ci);
                if (s + 1 < steps) prefetch(s + 1);
                cr = wave_sum(cr);
                ci = wave_sum(ci);
                if (lane == 0) {
                    const R2<R> dk = snap[1];
                    const R Fkr = F[2 * k] + cr, Fki = F[2 * k + 1] + ci;
                    const R dE = (R)-2 * (dj.x * F[2 * j] + dj.y * F[2 * j + 1]) - (R)2 * (dk.x * Fkr + dk.y * Fki);
                    const bool accept = (dE <= (R)0) || (tab[s].u < exp(-beta * dE));
                    flag[s & 1] = accept ? 1 : 0;
                    if (accept) {
                        E += dE;
                        ++n_acc;
                    } else {
                        a[j] = ajo;
                    }
                }
            }
            block_sync_lds();
            const bool acc_s = active && flag[s & 1];
            R acc_r = 0, acc_i = 0;
            if (acc_s) {  // a_j new, a_k old in LDS: field changes of every target
                const R2<R> dj = snap[0], dk = snap[1];
                const int part = gw / ns;
                for (int sl = gw % ns; sl < ns && part < parts; sl += parts == 1 ? wpc : ns) {
                    R fr = 0, fi = 0;
                    gather_slice<R, LAYOUT>(P, sd, N, j, dj, sl, part, parts, lane, a, fr, fi);
                    gather_slice<R, LAYOUT>(P, sd, N, k, dk, sl, part, parts, lane, a, fr, fi);
                    const int l = 64 * sl + lane;
                    if (l < N) {
                        if (parts == 1) {  // the slice's only wave: add directly
                            F[2 * l] += fr;
                            F[2 * l + 1] += fi;
                        } else if (part == 0) {  // one slice per wave when parts > 1
                            acc_r = fr;
                            acc_i = fi;
                        } else {
                            pbuf[l] = mk2<R>(fr, fi);
                        }
                    }
                }
            }
            if (!lone || acc_s) block_sync_lds();
            if (parts > 1) {  // first part adds its sums and the second's, then all wait
                if (acc_s && gw < ns) {
                    const int l = 64 * gw + lane;
                    if (l < N) {
                        const R2<R> v = pbuf[l];
                        F[2 * l] += acc_r + v.x;
                        F[2 * l + 1] += acc_i + v.y;
                    }
                }
                if (!lone || acc_s) block_sync_lds();
            }
            if (active && gt == 0) {
                if (acc_s) a[k] = akn;
                if (s + 1 < steps) prepare(s + 1);
            }
            __builtin_amdgcn_wave_barrier();  // wave 0 reads lane 0's snapshot next: keep the LDS order
        }
    }
    __syncthreads();
    if (active) {
        for (int i = gt; i < N; i += nt) {
            amp_g[i] = a[i];
            fld_g[2 * i] = F[2 * i];
            fld_g[2 * i + 1] = F[2 * i + 1];
        }
        if (gt == 0) {
            P.E[c] = E;
            atomicAdd(&P.acc[(size_t)it.sample * sh.n_temps + t_idx], (unsigned long long)n_acc);
        }
    }
}

// every field of every copy from the per-mode lists (one block per copy, a wave per mode)
template <typename R, int LAYOUT>
__global__ __launch_bounds__(256) void k_fields_all(DevPtrs<R> P, ShapeInfo sh) {
    __shared__ R2<R> a[kMaxModes];
    const int c = blockIdx.x;
    const int mu = c / sh.copies_per_sample;
    const SampleDev sd = P.samples[mu];
    const int N = sd.N;
    const int64_t local = c - (int64_t)mu * sh.copies_per_sample;
    const R2<R>* amp = reinterpret_cast<const R2<R>*>(P.amp) + sd.amp_base + local * N;
    R* F = P.fields + 2 * (sd.amp_base + local * N);
    for (int i = threadIdx.x; i < N; i += blockDim.x) a[i] = amp[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int l = wave; l < N; l += blockDim.x / 64) {
        R fr = 0, fi = 0;
        mode_field<R, LAYOUT>(P, sd, l, a, lane, 64, fr, fi);
        fr = wave_sum(fr);
        fi = wave_sum(fi);
        if (lane == 0) {
            F[2 * l] = fr;
            F[2 * l + 1] = fi;
        }
    }
}

// ---------------------------------------------------------------- initial draw
// one block per copy; exact draw from the infinite-temperature law on
// sum |a|^4 = N: |a_k|^2 = sqrt(N) |g_k| / ||g||, phases uniform
template <typename R>
__global__ __launch_bounds__(256) void k_init(DevPtrs<R> P, ShapeInfo sh) {
    __shared__ double red[4];
    const int c = blockIdx.x;
    const int mu = c / sh.copies_per_sample;
    const SampleDev sd = P.samples[mu];
    const int N = sd.N;
    const int64_t local = c - (int64_t)mu * sh.copies_per_sample;
    R* amp = P.amp + 2 * (sd.amp_base + local * N);
    // rho = 4: a normal g_k per mode, intensity sqrt(N) |g_k| / ||g||;
    // rho = 2: an exponential e_k per mode, intensity N e_k / sum e
    auto weight = [&](const Philox4& w) {
        const double u1 = 1.0 - uniform01<double>(w.v[0]);
        if (sh.rho == 2) return -log(u1);
        const double u2 = uniform01<double>(w.v[1]);
        return sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2);
    };
    double part = 0.0;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const Philox4 w = philox4x64((uint64_t)k, (uint64_t)c, 0, 0, sh.run_seed, kTagInit);
        const double gk = weight(w);
        part += sh.rho == 2 ? gk : gk * gk;
    }
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    const double norm = red[0] + red[1] + red[2] + red[3];
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const Philox4 w = philox4x64((uint64_t)k, (uint64_t)c, 0, 0, sh.run_seed, kTagInit);
        const double gk = weight(w);
        const double ph = 2.0 * 3.14159265358979323846 * uniform01<double>(w.v[2]);
        const double u = sh.rho == 2 ? (double)N * gk / norm : sqrt((double)N) * fabs(gk) / sqrt(norm);
        const double A = sqrt(u);
        amp[2 * k] = (R)(A * cos(ph));
        amp[2 * k + 1] = (R)(A * sin(ph));
    }
    if (threadIdx.x == 0) {
        P.temp_of[c] = (int32_t)(local % sh.n_temps);
        const int r = (int)(local / sh.n_temps);
        P.copy_at[((size_t)mu * sh.n_reps + r) * sh.n_temps + local % sh.n_temps] = c;
    }
}

// ---------------------------------------------------------------- FP64 recomputation
// one block per copy: H = -2 sum_q J_q Re(conj a_p conj a_s a_m a_n) and
// S = sum |a|^4 in FP64.  mode 0: drift check, renormalise when
// |S/N - 1| > renorm_tol (H scales by N/S), store E; mode 1: E64 only.
// FP64 energy recomputation in two stages.  Stage one: the copies of one
// sample in groups of up to kResyncCopies (FP64 amplitudes in LDS) and the
// sample's by-term list cut into kResyncParts ranges; a workgroup streams one
// range once for its whole group and leaves each copy's partial energy.
constexpr int kResyncCopies = 8;

__host__ __device__ inline int resync_group(int N) {
    const int fit = (48 * 1024) / (N * 16);  // FP64 complex amplitudes of the group within 48 KiB
    return fit < 1 ? 1 : (fit < kResyncCopies ? fit : kResyncCopies);
}

template <typename R>
__global__ __launch_bounds__(256) void k_resync_part(DevPtrs<R> P, ShapeInfo sh, int group, int groups) {
    extern __shared__ double2 ra[];  // [group][N]
    __shared__ double red[4][kResyncCopies];
    const int part = blockIdx.x % kResyncParts;
    const int grp = (blockIdx.x / kResyncParts) % groups;
    const int mu = blockIdx.x / (kResyncParts * groups);
    const SampleDev sd = P.samples[mu];
    const int N = sd.N;
    const int g0 = grp * group;
    const int ng = sh.copies_per_sample - g0 < group ? sh.copies_per_sample - g0 : group;
    for (int i = 0; i < ng; ++i) {
        const R* amp = P.amp + 2 * (sd.amp_base + (int64_t)(g0 + i) * N);
        for (int k = threadIdx.x; k < N; k += blockDim.x)
            ra[(size_t)i * N + k] = make_double2((double)amp[2 * k], (double)amp[2 * k + 1]);
    }
    __syncthreads();
    double H[kResyncCopies];
#pragma unroll
    for (int i = 0; i < kResyncCopies; ++i) H[i] = 0.0;
    const ushort4* Q = P.quads + sd.quad_base;
    const double* Jq = P.Jq + sd.quad_base;
    const int64_t q0 = sd.n_quads * part / kResyncParts, q1 = sd.n_quads * (part + 1) / kResyncParts;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        const ushort4 t = Q[q];
        const double J = Jq[q];
#pragma unroll
        for (int i = 0; i < kResyncCopies; ++i) {
            if (i >= ng) break;
            const double2* a = ra + (size_t)i * N;
            const double2 p = a[t.x], s = a[t.y], m = a[t.z], n = a[t.w];
            // conj(p) conj(s) = (p.x s.x - p.y s.y, -(p.x s.y + p.y s.x))
            const double cr = p.x * s.x - p.y * s.y, ci = -(p.x * s.y + p.y * s.x);
            const double dr = m.x * n.x - m.y * n.y, di = m.x * n.y + m.y * n.x;
            H[i] += -2.0 * J * (cr * dr - ci * di);
        }
    }
#pragma unroll
    for (int i = 0; i < kResyncCopies; ++i) {
        if (i >= ng) break;
        const double h = wave_sum(H[i]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][i] = h;
    }
    __syncthreads();
    if (threadIdx.x < ng) {
        const int i = threadIdx.x;
        const int64_t c = (int64_t)mu * sh.copies_per_sample + g0 + i;
        P.rs_part[c * kResyncParts + part] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    }
}

// Stage two, one wave per copy: H = the parts in order, S = sum |a|^rho; the
// drift and finiteness checks, renormalisation by (N/S)^(1/rho) when S is off
// N by more than renorm_tol (H scales with the fourth power), and the energies.
// mode 0: periodic recomputation; 1: FP64 energies into E64 only; 2: E = H.
template <typename R>
__global__ __launch_bounds__(64) void k_resync_fin(DevPtrs<R> P, ShapeInfo sh, int mode) {
    const int c = blockIdx.x, lane = threadIdx.x;
    const int mu = c / sh.copies_per_sample;
    const SampleDev sd = P.samples[mu];
    const int N = sd.N;
    const int64_t local = c - (int64_t)mu * sh.copies_per_sample;
    R* amp = P.amp + 2 * (sd.amp_base + local * N);
    double s4 = 0.0;  // sum |a|^rho
    for (int k = lane; k < N; k += 64) {
        const double x = (double)amp[2 * k], y = (double)amp[2 * k + 1];
        const double u = x * x + y * y;
        s4 += sh.rho == 2 ? u : u * u;
    }
    const double St = wave_sum(s4);
    double Ht = 0.0;
    for (int p = 0; p < kResyncParts; ++p) Ht += P.rs_part[(int64_t)c * kResyncParts + p];
    double f = 1.0;
    if (mode == 0 && fabs(St / (double)N - 1.0) > sh.renorm_tol && St > 0.0)
        f = sh.rho == 2 ? sqrt((double)N / St) : pow((double)N / St, 0.25);
    if (lane == 0) {
        if (mode == 2) P.E[c] = (R)Ht;
        if (mode == 0) {
            const double Er = (double)P.E[c];
            const double scale = fabs(Ht) > 1.0 ? fabs(Ht) : 1.0;
            const double d = fabs(Er - Ht) / scale;
            P.drift[c] = d;
            if (!isfinite(Ht) || !isfinite(St) || !isfinite(Er)) atomicOr(&P.counters->error_flags, 2);
            else if (sh.drift_tol > 0.0 && d > sh.drift_tol) atomicOr(&P.counters->error_flags, 1);
            if (f != 1.0) Ht *= f * f * f * f;  // H is homogeneous of degree 4 in a
            P.E[c] = (R)Ht;
        }
        P.E64[c] = Ht;
    }
    if (f != 1.0)
        for (int k = lane; k < N; k += 64) {
            amp[2 * k] = (R)((double)amp[2 * k] * f);
            amp[2 * k + 1] = (R)((double)amp[2 * k + 1] * f);
        }
}

// ---------------------------------------------------------------- replica exchange
// one 64-thread block per ladder (sample, replica): energies of the ladder's
// temperatures, the pairs' uniforms and the differences b_i - b_{i+1} are
// staged in LDS in parallel, then one lane proposes the neighbouring baths in
// ascending order, each accepted with min[1, exp((b_i - b_{i+1})(E_i - E_{i+1}))],
// carrying the copy that moves up in registers (no global memory access in the
// chain); the ladder and the acceptance counts are written back in parallel
template <typename R>
__global__ __launch_bounds__(64) void k_swap(DevPtrs<R> P, ShapeInfo sh) {
    extern __shared__ double sw[];  // [T] energies, [T] uniforms, [T] b_i - b_{i+1}, [T] copies, [T] accepted
    const int L = blockIdx.x;
    const int T = sh.n_temps;
    double* __restrict__ e = sw;
    double* __restrict__ u = sw + T;
    double* __restrict__ db = sw + 2 * T;
    int32_t* __restrict__ at_s = reinterpret_cast<int32_t*>(sw + 3 * T);
    int32_t* __restrict__ took = at_s + T;
    int32_t* at = P.copy_at + (size_t)L * T;
    const int64_t round = P.counters->swaps_done;
    for (int i = threadIdx.x; i < T; i += 64) {
        const int c = at[i];
        at_s[i] = c;
        e[i] = (double)P.E[c];
        const Philox4 w = philox4x64((uint64_t)i, (uint64_t)round, (uint64_t)L, 0, sh.run_seed, kTagSwap);
        u[i] = uniform01<double>(w.v[0]);
        db[i] = i + 1 < T ? P.beta64[i] - P.beta64[i + 1] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the chain in registers: (cc, ec) is the copy and energy now at bath i;
        // bath i + 1 still holds its own until pair i is decided
        int cc = at_s[0];
        double ec = e[0];
        for (int i = 0; i + 1 < T; ++i) {
            const int cn = at_s[i + 1];
            const double en = e[i + 1];
            const double x = db[i] * (ec - en);
            const bool acc = (x >= 0.0) || (u[i] < exp(x));
            took[i] = acc ? 1 : 0;
            if (acc) {
                at_s[i] = cn;
            } else {
                at_s[i] = cc;
                cc = cn;
                ec = en;
            }
        }
        at_s[T - 1] = cc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < T; i += 64) {
        at[i] = at_s[i];
        P.temp_of[at_s[i]] = i;
        if (i + 1 < T && took[i]) P.swap_acc[(size_t)L * (T - 1) + i] += 1ull;
    }
}

__global__ void k_tick(Counters* cnt, int64_t d_sweeps, int64_t d_swaps) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cnt->sweeps_done += d_sweeps;
        cnt->swaps_done += d_swaps;
    }
}

__global__ void k_zero(uint32_t* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------- observables
// one block of 64 threads per (sample, bath): energy moments, IPR Y_2 and Y_4
// of every replica, overlap of every replica pair and its histogram
template <typename R>
__global__ __launch_bounds__(64) void k_measure(DevPtrs<R> P, ShapeInfo sh) {
    const int st = blockIdx.x;  // sample * T + t
    const int mu = st / sh.n_temps, t = st % sh.n_temps;
    const SampleDev sd = P.samples[mu];
    const int N = sd.N;
    const int lane = threadIdx.x;
    const int S_T = sh.n_samples * sh.n_temps;
    const int m = P.meas_cnt[st];
    double eS = 0, eQ = 0, y2S = 0, y4S = 0, e0 = 0;
    for (int r = 0; r < sh.n_reps; ++r) {
        const int c = P.copy_at[((size_t)mu * sh.n_reps + r) * sh.n_temps + t];
        const int64_t local = c - (int64_t)mu * sh.copies_per_sample;
        const R* a = P.amp + 2 * (sd.amp_base + local * N);
        double s1 = 0, s2 = 0, s4 = 0;
        double* spec = P.spec + (size_t)st * sh.spec_stride;  // each lane owns its modes
        for (int k = lane; k < N; k += 64) {
            const double x = a[2 * k], y = a[2 * k + 1];
            const double I = x * x + y * y;
            s1 += I;
            s2 += I * I;
            s4 += (I * I) * (I * I);
            spec[k] += I;
        }
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        s4 = wave_sum(s4);
        const double E = (double)P.E[c];
        if (r == 0) e0 = E;
        eS += E;
        eQ += E * E;
        y2S += s2 / (s1 * s1);
        y4S += s4 / (s2 * s2);
        if (lane == 0) {  // distribution of the total intensity I = sum |a|^2
            int bI = (int)floor(s1 / (double)N * sh.n_bins);
            bI = bI < 0 ? 0 : (bI >= sh.n_bins ? sh.n_bins - 1 : bI);
            P.hist_I[(size_t)st * sh.n_bins + bI] += 1.0;
        }
    }
    double qS = 0, qQ = 0, q4 = 0, qn = 0, q01 = 0;
    for (int r = 0; r < sh.n_reps; ++r)
        for (int r2 = r + 1; r2 < sh.n_reps; ++r2) {
            const int c1 = P.copy_at[((size_t)mu * sh.n_reps + r) * sh.n_temps + t];
            const int c2 = P.copy_at[((size_t)mu * sh.n_reps + r2) * sh.n_temps + t];
            const R* x = P.amp + 2 * (sd.amp_base + (c1 - (int64_t)mu * sh.copies_per_sample) * N);
            const R* y = P.amp + 2 * (sd.amp_base + (c2 - (int64_t)mu * sh.copies_per_sample) * N);
            double q = 0;
            for (int k = lane; k < N; k += 64) q += (double)x[2 * k] * y[2 * k] + (double)x[2 * k + 1] * y[2 * k + 1];
            q = wave_sum(q) / (double)N;
            qS += q;
            qQ += q * q;
            q4 += (q * q) * (q * q);
            qn += 1.0;
            if (r == 0 && r2 == 1) q01 = q;
            if (lane == 0) {
                int b = (int)floor((q + 1.0) * 0.5 * sh.n_bins);
                b = b < 0 ? 0 : (b >= sh.n_bins ? sh.n_bins - 1 : b);
                P.hist[(size_t)st * sh.n_bins + b] += 1.0;
            }
        }
    if (lane == 0) {
        double* o = P.obs;
        o[kEN * S_T + st] += (double)sh.n_reps;
        o[kESum * S_T + st] += eS;
        o[kESq * S_T + st] += eQ;
        o[kY2 * S_T + st] += y2S;
        o[kY4 * S_T + st] += y4S;
        o[kQN * S_T + st] += qn;
        o[kQSum * S_T + st] += qS;
        o[kQSq * S_T + st] += qQ;
        o[kQ4 * S_T + st] += q4;
        if (m < sh.series_len) {
            P.series_e[(size_t)st * sh.series_len + m] = e0;
            if (sh.n_reps > 1) P.series_q[(size_t)st * sh.series_len + m] = q01;
        }
        P.meas_cnt[st] = m + 1;
    }
}

// ---------------------------------------------------------------- test hooks
// all N local fields of one copy with the sweep's field code (one block)
template <typename R, int LAYOUT>
__global__ __launch_bounds__(256) void k_fields(DevPtrs<R> P, ShapeInfo sh, int copy, int mu, double* F) {
    __shared__ R2<R> a[kMaxModes];
    __shared__ R red[4][2];
    const SampleDev sd = P.samples[mu];
    const int N = sd.N;
    const int64_t local = copy - (int64_t)mu * sh.copies_per_sample;
    const R2<R>* amp = reinterpret_cast<const R2<R>*>(P.amp) + sd.amp_base + local * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) a[i] = amp[i];
    __syncthreads();
    for (int l = 0; l < N; ++l) {
        R fr = 0, fi = 0;
        mode_field<R, LAYOUT>(P, sd, l, a, threadIdx.x, blockDim.x, fr, fi);
        fr = wave_sum(fr);
        fi = wave_sum(fi);
        if ((threadIdx.x & 63) == 0) {
            red[threadIdx.x >> 6][0] = fr;
            red[threadIdx.x >> 6][1] = fi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            R sr = 0, si = 0;
            for (int w = 0; w < 4; ++w) {
                sr += red[w][0];
                si += red[w][1];
            }
            F[2 * l] = (double)sr;
            F[2 * l + 1] = (double)si;
        }
        __syncthreads();
    }
}

// pair energy changes on given proposals, with the sweep's snapshot rule
template <typename R, int LAYOUT>
__global__ __launch_bounds__(256) void k_pair_dE(DevPtrs<R> P, ShapeInfo sh, int copy, int mu, int n,
                                                 const int32_t* jk, const double* nw, double* dE) {
    __shared__ R2<R> a[kMaxModes];
    __shared__ R red[4][4];
    const SampleDev sd = P.samples[mu];
    const int N = sd.N;
    const int64_t local = copy - (int64_t)mu * sh.copies_per_sample;
    const R2<R>* amp = reinterpret_cast<const R2<R>*>(P.amp) + sd.amp_base + local * N;
    for (int p = 0; p < n; ++p) {
        for (int i = threadIdx.x; i < N; i += blockDim.x) a[i] = amp[i];
        __syncthreads();
        const int j = jk[2 * p], k = jk[2 * p + 1];
        const R2<R> ajo = amp[j], ako = amp[k];
        const R2<R> ajn = mk2<R>((R)nw[4 * p], (R)nw[4 * p + 1]);
        const R2<R> akn = mk2<R>((R)nw[4 * p + 2], (R)nw[4 * p + 3]);
        if (threadIdx.x == 0) a[j] = ajn;
        __syncthreads();
        R fjr = 0, fji = 0, fkr = 0, fki = 0;
        mode_field<R, LAYOUT>(P, sd, j, a, threadIdx.x, blockDim.x, fjr, fji);
        mode_field<R, LAYOUT>(P, sd, k, a, threadIdx.x, blockDim.x, fkr, fki);
        fjr = wave_sum(fjr);
        fji = wave_sum(fji);
        fkr = wave_sum(fkr);
        fki = wave_sum(fki);
        if ((threadIdx.x & 63) == 0) {
            red[threadIdx.x >> 6][0] = fjr;
            red[threadIdx.x >> 6][1] = fji;
            red[threadIdx.x >> 6][2] = fkr;
            red[threadIdx.x >> 6][3] = fki;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            R2<R> Fj = mk2<R>(0, 0), Fk = mk2<R>(0, 0);
            for (int w = 0; w < 4; ++w) {
                Fj.x += red[w][0];
                Fj.y += red[w][1];
                Fk.x += red[w][2];
                Fk.y += red[w][3];
            }
            dE[p] = (double)pair_delta<R>(ajo, ajn, ako, akn, Fj, Fk);
        }
        __syncthreads();
    }
}

template <typename R>
__global__ void k_convert(R* amp, double* buf, int64_t n, int to_ctx) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 2 * n; i += (int64_t)gridDim.x * blockDim.x) {
        if (to_ctx) amp[i] = (R)buf[i];
        else buf[i] = (double)amp[i];
    }
}

template <typename R, int BLOCK>
hipError_t launch_sweep_t(const void* ptrs, const ShapeInfo& sh, const SweepLaunch& L, int n_sweeps,
                          hipStream_t st) {
    const DevPtrs<R>& P = *static_cast<const DevPtrs<R>*>(ptrs);
    if (sh.short_lists) {
        hipLaunchKernelGGL((k_sweep_short<R, BLOCK>), dim3(L.n_items), dim3(BLOCK), L.lds_bytes, st, P, sh, L.max_N,
                           n_sweeps);
        return hipGetLastError();
    }
    if (sh.cached) {
        if (sh.layout == kLayoutChunked)
            hipLaunchKernelGGL((k_sweep_cached<R, BLOCK, kLayoutChunked>), dim3(L.n_items), dim3(BLOCK), L.lds_bytes,
                               st, P, sh, L.max_N, n_sweeps);
        else
            hipLaunchKernelGGL((k_sweep_cached<R, BLOCK, kLayoutPacked>), dim3(L.n_items), dim3(BLOCK), L.lds_bytes,
                               st, P, sh, L.max_N, n_sweeps);
        return hipGetLastError();
    }
    if (sh.layout == kLayoutChunked) {
        if constexpr (BLOCK == 256 || BLOCK == 512) {
#define RLPT_SWEEP_PF(PFV, SPV)                                                                                   \
    hipLaunchKernelGGL((k_sweep<R, BLOCK, kLayoutChunked, PFV, SPV>), dim3(L.n_items), dim3(BLOCK), L.lds_bytes, st, \
                       P, sh, L.max_N, n_sweeps)
            switch (L.prefetch * 2 + (L.split ? 1 : 0)) {
                case 0: break;
                case 2: RLPT_SWEEP_PF(1, false); return hipGetLastError();
                case 3: RLPT_SWEEP_PF(1, true); return hipGetLastError();
                case 4: RLPT_SWEEP_PF(2, false); return hipGetLastError();
                case 5: RLPT_SWEEP_PF(2, true); return hipGetLastError();
                case 8: RLPT_SWEEP_PF(4, false); return hipGetLastError();
                case 9: RLPT_SWEEP_PF(4, true); return hipGetLastError();
                default: return hipErrorInvalidValue;
            }
#undef RLPT_SWEEP_PF
        }
        hipLaunchKernelGGL((k_sweep<R, BLOCK, kLayoutChunked, 0, false>), dim3(L.n_items), dim3(BLOCK), L.lds_bytes, st,
                           P, sh, L.max_N, n_sweeps);
    } else {
        hipLaunchKernelGGL((k_sweep<R, BLOCK, kLayoutPacked, 0, false>), dim3(L.n_items), dim3(BLOCK), L.lds_bytes, st,
                           P, sh, L.max_N, n_sweeps);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_sweep_r(const void* ptrs, const ShapeInfo& sh, const SweepLaunch& L, int n_sweeps,
                          hipStream_t st) {
    switch (L.block_threads) {
        case 64: return launch_sweep_t<R, 64>(ptrs, sh, L, n_sweeps, st);
        case 128: return launch_sweep_t<R, 128>(ptrs, sh, L, n_sweeps, st);
        case 256: return launch_sweep_t<R, 256>(ptrs, sh, L, n_sweeps, st);
        case 512: return launch_sweep_t<R, 512>(ptrs, sh, L, n_sweeps, st);
        case 1024: return launch_sweep_t<R, 1024>(ptrs, sh, L, n_sweeps, st);
        default: return hipErrorInvalidValue;
    }
}

template <int BLOCK>
hipError_t stream_lists_t(const DevPtrs<float>& P, const ShapeInfo& sh, const SweepLaunch& L, int64_t offset,
                          float* sink, hipStream_t st) {
    hipLaunchKernelGGL((k_stream_lists<BLOCK>), dim3(L.n_items), dim3(BLOCK), L.lds_bytes, st, P, sh, L.max_N, offset,
                       sink);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stream_lists(const void* ptrs, const ShapeInfo& sh, const SweepLaunch& L, int64_t sweep_offset,
                               float* sink, hipStream_t st) {
    const DevPtrs<float>& P = *static_cast<const DevPtrs<float>*>(ptrs);
    switch (L.block_threads) {
        case 64: return stream_lists_t<64>(P, sh, L, sweep_offset, sink, st);
        case 128: return stream_lists_t<128>(P, sh, L, sweep_offset, sink, st);
        case 256: return stream_lists_t<256>(P, sh, L, sweep_offset, sink, st);
        case 512: return stream_lists_t<512>(P, sh, L, sweep_offset, sink, st);
        case 1024: return stream_lists_t<1024>(P, sh, L, sweep_offset, sink, st);
        default: return hipErrorInvalidValue;
    }
}

size_t sweep_lds_bytes(int precision, int block_threads, int max_copies_per_item, int max_N, int cached,
                       int short_lists) {
    const int waves = block_threads / 64;
    if (short_lists) return (size_t)max_copies_per_item * max_N * 2 * (precision == RLPT_FP64 ? 8 : 4);
    if (cached)
        return (size_t)max_copies_per_item * (precision == RLPT_FP64 ? group_bytes_cached<double>(max_N, waves)
                                                                     : group_bytes_cached<float>(max_N, waves));
    return bounds_bytes(max_N) + (size_t)max_copies_per_item * (precision == RLPT_FP64 ? group_bytes<double>(max_N, waves)
                                                                                       : group_bytes<float>(max_N, waves));
}

template <typename R>
static hipError_t fields_all_t(const void* ptrs, const ShapeInfo& sh, int n_copies, hipStream_t st) {
    const DevPtrs<R>& P = *static_cast<const DevPtrs<R>*>(ptrs);
    if (sh.layout == kLayoutChunked)
        hipLaunchKernelGGL((k_fields_all<R, kLayoutChunked>), dim3(n_copies), dim3(256), 0, st, P, sh);
    else
        hipLaunchKernelGGL((k_fields_all<R, kLayoutPacked>), dim3(n_copies), dim3(256), 0, st, P, sh);
    return hipGetLastError();
}

hipError_t launch_fields_all(int precision, const void* ptrs, const ShapeInfo& sh, int n_copies, hipStream_t st) {
    return precision == RLPT_FP64 ? fields_all_t<double>(ptrs, sh, n_copies, st)
                                  : fields_all_t<float>(ptrs, sh, n_copies, st);
}

hipError_t launch_sweep(int precision, const void* ptrs, const ShapeInfo& sh, const SweepLaunch& L, int n_sweeps,
                        hipStream_t st) {
    return precision == RLPT_FP64 ? launch_sweep_r<double>(ptrs, sh, L, n_sweeps, st)
                                  : launch_sweep_r<float>(ptrs, sh, L, n_sweeps, st);
}

template <typename R>
static hipError_t init_t(const void* ptrs, const ShapeInfo& sh, int n_copies, hipStream_t st) {
    hipLaunchKernelGGL(k_init<R>, dim3(n_copies), dim3(256), 0, st, *static_cast<const DevPtrs<R>*>(ptrs), sh);
    return hipGetLastError();
}
hipError_t launch_init(int precision, const void* ptrs, const ShapeInfo& sh, int n_copies, int, hipStream_t st) {
    return precision == RLPT_FP64 ? init_t<double>(ptrs, sh, n_copies, st) : init_t<float>(ptrs, sh, n_copies, st);
}

template <typename R>
static hipError_t swap_t(const void* ptrs, const ShapeInfo& sh, hipStream_t st) {
    const int n = sh.n_samples * sh.n_reps;
    const size_t lds = (size_t)sh.n_temps * (3 * sizeof(double) + 2 * sizeof(int32_t)) + 16;
    hipLaunchKernelGGL(k_swap<R>, dim3(n), dim3(64), lds, st, *static_cast<const DevPtrs<R>*>(ptrs), sh);
    return hipGetLastError();
}
hipError_t launch_swap(int precision, const void* ptrs, const ShapeInfo& sh, hipStream_t st) {
    return precision == RLPT_FP64 ? swap_t<double>(ptrs, sh, st) : swap_t<float>(ptrs, sh, st);
}

hipError_t launch_tick(const void* ptrs, int precision, int64_t d_sweeps, int64_t d_swaps, hipStream_t st) {
    Counters* cnt = precision == RLPT_FP64 ? static_cast<const DevPtrs<double>*>(ptrs)->counters
                                           : static_cast<const DevPtrs<float>*>(ptrs)->counters;
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, cnt, d_sweeps, d_swaps);
    return hipGetLastError();
}

template <typename R>
static hipError_t resync_t(const void* ptrs, const ShapeInfo& sh, int n_copies, int mode, hipStream_t st) {
    const DevPtrs<R>& P = *static_cast<const DevPtrs<R>*>(ptrs);
    // copy groups sized for the largest N of the context (spec_stride); n_copies = samples x copies per sample
    const int group = resync_group(sh.spec_stride);
    const int groups = (sh.copies_per_sample + group - 1) / group;
    const int samples = n_copies / sh.copies_per_sample;
    const size_t lds = (size_t)group * sh.spec_stride * sizeof(double2);
    hipLaunchKernelGGL(k_resync_part<R>, dim3(samples * groups * kResyncParts), dim3(256), lds, st, P, sh, group,
                       groups);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_resync_fin<R>, dim3(n_copies), dim3(64), 0, st, P, sh, mode);
    return hipGetLastError();
}
hipError_t launch_resync(int precision, const void* ptrs, const ShapeInfo& sh, int n_copies, int mode, hipStream_t st) {
    return precision == RLPT_FP64 ? resync_t<double>(ptrs, sh, n_copies, mode, st)
                                  : resync_t<float>(ptrs, sh, n_copies, mode, st);
}

// ---------------------------------------------------------------- FP64 energies without allocation
// Device scratch of the energy call that allocates nothing: the partial
// energies of the FP64 recomputation's term ranges, kResyncParts per copy.
// One array per GPU for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress gives on that GPU (the array's
// name is a host-side stand-in there).  Every call on a GPU shares it.
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

template <typename R>
static hipError_t energy_static_t(const void* ptrs, const ShapeInfo& sh, int n_copies, void* scratch_ptr, double* E,
                                  hipStream_t st) {
    DevPtrs<R> P = *static_cast<const DevPtrs<R>*>(ptrs);
    P.rs_part = static_cast<double*>(scratch_ptr);  // every partial is written before it is read
    P.E64 = E;                                      // mode 1 writes E64 only
    return resync_t<R>(&P, sh, n_copies, 1, st);
}

hipError_t launch_energy_static(int precision, const void* ptrs, const ShapeInfo& sh, int n_copies, double* E,
                                hipStream_t st) {
    if ((size_t)n_copies * kResyncParts * sizeof(double) > kStaticScratchBytes) return hipErrorInvalidValue;
    void* p = nullptr;
    hipError_t e = static_scratch_address(&p);
    if (e != hipSuccess) return e;
    return precision == RLPT_FP64 ? energy_static_t<double>(ptrs, sh, n_copies, p, E, st)
                                  : energy_static_t<float>(ptrs, sh, n_copies, p, E, st);
}

template <typename R>
static hipError_t measure_t(const void* ptrs, const ShapeInfo& sh, hipStream_t st) {
    hipLaunchKernelGGL(k_measure<R>, dim3(sh.n_samples * sh.n_temps), dim3(64), 0, st,
                       *static_cast<const DevPtrs<R>*>(ptrs), sh);
    return hipGetLastError();
}
hipError_t launch_measure(int precision, const void* ptrs, const ShapeInfo& sh, hipStream_t st) {
    return precision == RLPT_FP64 ? measure_t<double>(ptrs, sh, st) : measure_t<float>(ptrs, sh, st);
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, static_cast<uint32_t*>(p), n);
    return hipGetLastError();
}

template <typename R>
static hipError_t fields_t(const void* ptrs, int copy, int mu, double* F, hipStream_t st, const ShapeInfo& sh) {
    if (sh.layout == kLayoutChunked)
        hipLaunchKernelGGL((k_fields<R, kLayoutChunked>), dim3(1), dim3(256), 0, st,
                           *static_cast<const DevPtrs<R>*>(ptrs), sh, copy, mu, F);
    else
        hipLaunchKernelGGL((k_fields<R, kLayoutPacked>), dim3(1), dim3(256), 0, st,
                           *static_cast<const DevPtrs<R>*>(ptrs), sh, copy, mu, F);
    return hipGetLastError();
}

template <typename R>
static hipError_t pair_t(const void* ptrs, int copy, int mu, int n, const int32_t* jk, const double* nw, double* dE,
                         hipStream_t st, const ShapeInfo& sh) {
    if (sh.layout == kLayoutChunked)
        hipLaunchKernelGGL((k_pair_dE<R, kLayoutChunked>), dim3(1), dim3(256), 0, st,
                           *static_cast<const DevPtrs<R>*>(ptrs), sh, copy, mu, n, jk, nw, dE);
    else
        hipLaunchKernelGGL((k_pair_dE<R, kLayoutPacked>), dim3(1), dim3(256), 0, st,
                           *static_cast<const DevPtrs<R>*>(ptrs), sh, copy, mu, n, jk, nw, dE);
    return hipGetLastError();
}

template <typename R>
static hipError_t convert_t(void* amp, double* buf, int64_t n, int to_ctx, hipStream_t st) {
    int blocks = (int)((2 * n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_convert<R>, dim3(blocks), dim3(256), 0, st, static_cast<R*>(amp), buf, n, to_ctx);
    return hipGetLastError();
}
hipError_t launch_convert_state(int precision, void* amp, double* buf, int64_t n, int to_ctx, hipStream_t st) {
    return precision == RLPT_FP64 ? convert_t<double>(amp, buf, n, to_ctx, st) : convert_t<float>(amp, buf, n, to_ctx, st);
}

// the test hooks need the shape; they are launched through these two entry points
hipError_t launch_fields_sh(int precision, const void* ptrs, const ShapeInfo& sh, int copy, int mu, double* F,
                            hipStream_t st) {
    return precision == RLPT_FP64 ? fields_t<double>(ptrs, copy, mu, F, st, sh) : fields_t<float>(ptrs, copy, mu, F, st, sh);
}
hipError_t launch_pair_dE_sh(int precision, const void* ptrs, const ShapeInfo& sh, int copy, int mu, int n,
                             const int32_t* jk, const double* nw, double* dE, hipStream_t st) {
    return precision == RLPT_FP64 ? pair_t<double>(ptrs, copy, mu, n, jk, nw, dE, st, sh)
                                  : pair_t<float>(ptrs, copy, mu, n, jk, nw, dE, st, sh);
}

}  // namespace rlpt
