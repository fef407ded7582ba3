// Kernels of the learned global proposal (see mlp.hpp): batched bfloat16
// GEMMs on the matrix cores with FP32 accumulation, SiLU, the Gaussian-mixture head and
// its gradient, Adam, and the three stages of an exact Metropolis-Hastings
// global move (propose, energy change, accept).  Every launch covers all
// networks (grid z = network).
#include <hip/hip_runtime.h>
#include <math.h>

#include "mlp.hpp"
#include "philox.hpp"

namespace rlpt {
namespace {

constexpr uint64_t kTagLearn = 0x4C4541524EULL;  // "LEARN"
constexpr uint64_t kTagTrain = 0x545241494EULL;  // "TRAIN"
constexpr float kSmaxY = 2.0f;
constexpr float kSmaxPsi = 1.57079632679489662f;
constexpr float kLog2Pi = 1.83787706640934548f;
constexpr float kPiF = 3.14159265358979324f;
constexpr int kMaxK = 8;

__device__ inline uint16_t f_to_bf16(float x) {
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ inline float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }
__device__ inline float silu(float x) { return x * sigm(x); }

__device__ inline float wsum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float wmax(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
// word i (0..3) of a Philox block, chosen without indexing (an indexed pick
// of a register array would go through scratch memory)
__device__ inline uint64_t word_of(const Philox4& w, int i) {
    return i == 0 ? w.v[0] : (i == 1 ? w.v[1] : (i == 2 ? w.v[2] : w.v[3]));
}
__device__ inline float wrapf(float x) { return x - 2.0f * kPiF * ceilf((x - kPiF) / (2.0f * kPiF)); }

// ------------------------------------------------------------------ GEMM
// C[i][j] = act(sum_k A(i,k) B(k,j) + bias[j]), A(i,k) = A[i*as0 + k*as1],
// B(k,j) = B[k*bs0 + j*bs1], on the matrix cores: both operands are rounded
// to bfloat16 (nearest even; the weights already are) and staged in LDS, the
// products accumulate in FP32 through v_mfma_f32_16x16x16_bf16.  A 256-thread
// workgroup (4 waves) computes a BM x 64 tile; K advances 64 at a time, with
// the next stage's global loads in flight while the current one is multiplied.
template <typename TB>
struct Gemm {
    const float* A;
    int64_t sA;
    int as0, as1;
    const TB* B;
    int64_t sB;
    int bs0, bs1;
    const float* bias;
    int64_t sBias;
    float* Cpre;
    float* Cact;
    int64_t sC;
    int M, N, K;
};

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGemmN = 64;             // tile columns
constexpr int kGemmK = 64;             // K per LDS stage
constexpr int kGemmLd = kGemmK + 4;    // LDS row stride in bfloat16 elements (8-byte aligned rows)

__device__ inline uint16_t bf16_bits(float x) { return f_to_bf16(x); }
__device__ inline uint16_t bf16_bits(uint16_t x) { return x; }

template <typename TB, int ACT, int BM>
__global__ __launch_bounds__(256) void k_gemm(Gemm<TB> g) {
    constexpr int GM = BM >= 32 ? BM / 32 : 1;  // waves along M
    constexpr int GN = 4 / GM;                  // waves along N
    constexpr int WM = BM / (16 * GM);          // 16 x 16 blocks per wave along M
    constexpr int WN = kGemmN / (16 * GN);      // and along N
    constexpr int AE = BM * kGemmK / 256;       // A elements per thread per stage
    constexpr int BE = kGemmN * kGemmK / 256;   // B elements per thread per stage
    __shared__ __align__(16) uint16_t As[BM][kGemmLd];      // [m][k]
    __shared__ __align__(16) uint16_t Bs[kGemmN][kGemmLd];  // [n][k]
    const int net = blockIdx.z;
    const float* A = g.A + net * g.sA;
    const TB* B = g.B + net * g.sB;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * kGemmN;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm0 = (wave / GN) * WM * 16, wn0 = (wave % GN) * WN * 16;
    const bool a_m_fast = g.as0 == 1;  // A contiguous along M (a transposed operand)
    const bool b_n_fast = g.bs1 == 1;  // B contiguous along N
    // element e of a stage -> (row, k) of the A tile and (k, column) of the B tile
    auto a_rk = [&](int e, int& r, int& kk) {
        if (a_m_fast) { r = e % BM; kk = e / BM; } else { kk = e % kGemmK; r = e / kGemmK; }
    };
    auto b_kc = [&](int e, int& kk, int& c) {
        if (b_n_fast) { c = e % kGemmN; kk = e / kGemmN; } else { kk = e % kGemmK; c = e / kGemmK; }
    };
    uint16_t ra[AE], rb[BE];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < AE; ++i) {
            int r, kk;
            a_rk(threadIdx.x + 256 * i, r, kk);
            const int gi = m0 + r, gk = k0 + kk;
            ra[i] = (gi < g.M && gk < g.K) ? bf16_bits(A[(int64_t)gi * g.as0 + (int64_t)gk * g.as1]) : (uint16_t)0;
        }
#pragma unroll
        for (int i = 0; i < BE; ++i) {
            int kk, c;
            b_kc(threadIdx.x + 256 * i, kk, c);
            const int gk = k0 + kk, gj = n0 + c;
            rb[i] = (gk < g.K && gj < g.N) ? bf16_bits(B[(int64_t)gk * g.bs0 + (int64_t)gj * g.bs1]) : (uint16_t)0;
        }
    };
    f32x4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    load(0);
    for (int k0 = 0; k0 < g.K; k0 += kGemmK) {
#pragma unroll
        for (int i = 0; i < AE; ++i) {
            int r, kk;
            a_rk(threadIdx.x + 256 * i, r, kk);
            As[r][kk] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < BE; ++i) {
            int kk, c;
            b_kc(threadIdx.x + 256 * i, kk, c);
            Bs[c][kk] = rb[i];
        }
        __syncthreads();
        if (k0 + kGemmK < g.K) load(k0 + kGemmK);
#pragma unroll
        for (int kk = 0; kk < kGemmK; kk += 16) {
            // operand layout of the 16x16x16 bf16 MFMA: lane l holds A[l % 16][4 (l / 16) + 0..3]
            // and B[4 (l / 16) + 0..3][l % 16]; the result D[4 (l / 16) + v][l % 16] in slot v
            const int q = kk + 4 * (lane >> 4), rr = lane & 15;
            bf16x4 af[WM], bfr[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) af[i] = *reinterpret_cast<const bf16x4*>(&As[wm0 + 16 * i + rr][q]);
#pragma unroll
            for (int j = 0; j < WN; ++j) bfr[j] = *reinterpret_cast<const bf16x4*>(&Bs[wn0 + 16 * j + rr][q]);
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = m0 + wm0 + 16 * i + 4 * (lane >> 4) + v;
                const int gj = n0 + wn0 + 16 * j + (lane & 15);
                if (gi >= g.M || gj >= g.N) continue;
                const float x = acc[i][j][v] + (g.bias ? g.bias[net * g.sBias + gj] : 0.0f);
                g.Cpre[net * g.sC + (int64_t)gi * g.N + gj] = x;
                if (ACT) g.Cact[net * g.sC + (int64_t)gi * g.N + gj] = silu(x);
            }
}

template <typename TB, int ACT>
hipError_t gemm(const Gemm<TB>& g, int nets, hipStream_t st) {
    if (g.M <= 16) {
        dim3 grid((g.N + kGemmN - 1) / kGemmN, (g.M + 15) / 16, nets);
        hipLaunchKernelGGL((k_gemm<TB, ACT, 16>), grid, dim3(256), 0, st, g);
    } else {
        dim3 grid((g.N + kGemmN - 1) / kGemmN, (g.M + 63) / 64, nets);
        hipLaunchKernelGGL((k_gemm<TB, ACT, 64>), grid, dim3(256), 0, st, g);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ features
// Re, Im of mode k of a rotated so that a_0 is real and positive (the
// network's input; one definition for every kernel that forms it, evaluated
// without contraction so that every caller rounds the same way)
__device__ inline void feature_of(const float* a, int k, float& fr, float& fi) {
#pragma clang fp contract(off)
    const float x0 = a[0], y0 = a[1];
    const float r = sqrtf(x0 * x0 + y0 * y0);
    const float cr = r > 0.0f ? x0 / r : 1.0f, ci = r > 0.0f ? -y0 / r : 0.0f;
    const float x = a[2 * k], y = a[2 * k + 1];
    fr = x * cr - y * ci;
    fi = x * ci + y * cr;
}

__device__ inline void write_features(const float* a, int N, float* X, int lane) {
    for (int k = lane; k < N; k += 64) {
        float fr, fi;
        feature_of(a, k, fr, fi);
        X[k] = fr;
        X[N + k] = fi;
    }
}

__device__ inline const float* copy_amp(const DevPtrs<float>& P, const ShapeInfo& sh, int N, int c) {
    return P.amp + 2 * (int64_t)c * N;  // one N for every sample: copies are contiguous
}

// ------------------------------------------------------------------ fused inference forward
// MFMA fragment order of a weight matrix W [K][n] (K % 32 == 0, columns padded
// with zeros to a multiple of 64): the B operand of v_mfma_f32_16x16x16_bf16 for column
// block nb and K step ks is W[16 ks + 4 (l / 16) + i][16 nb + l % 16] in lane l,
// slot i.  The operands of the steps 2p and 2p + 1 of a block sit together,
// lane-major, 8 values per lane (step 2p in slots 0-3, step 2p + 1 in 4-7), so
// one wave reads both steps as 1024 contiguous bytes, 16 per lane.
__host__ __device__ inline int64_t frag_at(int64_t base, int K, int k, int n) {
    const int ks = k / 16;
    return base + (((int64_t)(n / 16) * (K / 32) + ks / 2) * 64 + (n % 16) + 16 * ((k % 16) / 4)) * 8 + 4 * (ks % 2) +
           (k % 4);
}
__host__ __device__ inline int64_t frag_w2(const MlpDev& M) { return (int64_t)M.In * M.H; }
__host__ __device__ inline int64_t frag_w3(const MlpDev& M) { return (int64_t)M.In * M.H + (int64_t)M.H * M.H; }
// Inference batches of at most 16 rows in one launch instead of the feature
// kernel and three GEMMs.  Workgroup (tile, net) forms the features of its
// net's rows (from the copies at the net's temperature slot, or from the
// proposals), computes both hidden layers (every tile of a net repeats them;
// activations stay in LDS as bfloat16) and then output columns [256 tile,
// 256 tile + 256).  Each of the 16 waves owns one 16 x 16 block of a layer at
// a time (16-column block w, w + 16, ...), so a wave's chain of products is
// short; it loads the block's weight fragments straight from the
// fragment-order copy, sixteen K steps (8 loads of 16 bytes) at a time, so no
// workgroup barrier falls inside a layer.  Every block sums its MFMAs over K
// in the order k_gemm does, with the same bfloat16 operands, bias and SiLU:
// the outputs are the same bits as the feature kernel followed by the three
// GEMMs.
constexpr int kFwdRows = 16;
constexpr int kFwdWaves = 16;     // workgroup of 1024 threads
constexpr int kFwdMaxTiles = 16;  // output tiles (256 columns each) up to which the fused path is used
constexpr int kFwdPairs = 8;      // step pairs loaded together: 16 K steps, 256 inputs (a 128 tail: 4 pairs)
enum FwdSource { kFwdCurrent = 0, kFwdProposal = 1 };

typedef short bf16x8 __attribute__((ext_vector_type(8)));

__host__ __device__ inline size_t forward_small_lds(int In, int H) {
    return (size_t)kFwdRows * ((In + 4) + 2 * (H + 4)) * sizeof(uint16_t);
}
__host__ __device__ inline bool forward_small_fits(const MlpDev& M) {
    return M.Bm <= kFwdRows && M.H % 128 == 0 && M.In % 128 == 0 && (M.Out + 255) / 256 <= kFwdMaxTiles &&
           forward_small_lds(M.In, M.H) <= 64 * 1024;
}

// this lane's weight fragments of W[k0, k0 + 32 PAIRS)[16 nb ..]
template <int PAIRS>
__device__ inline void fwd_load(const uint16_t* WF, int64_t fb, int K, int nb, int k0, int lane, bf16x8 (&bw)[PAIRS]) {
#pragma unroll
    for (int p = 0; p < PAIRS; ++p)
        bw[p] = *reinterpret_cast<const bf16x8*>(&WF[fb + (((int64_t)nb * (K / 32) + k0 / 32 + p) * 64 + lane) * 8]);
}

// acc += A[rows][k0, k0 + 32 PAIRS) W[k0, k0 + 32 PAIRS)[block]; A is a
// bfloat16 tile in LDS (row stride as)
template <int PAIRS>
__device__ inline void fwd_mma(const uint16_t* A, int as, int k0, int rr, int q4, const bf16x8 (&bw)[PAIRS],
                               f32x4& acc) {
    bf16x4 af[2 * PAIRS];
#pragma unroll
    for (int t = 0; t < 2 * PAIRS; ++t) af[t] = *reinterpret_cast<const bf16x4*>(&A[rr * as + k0 + 16 * t + q4]);
#pragma unroll
    for (int p = 0; p < PAIRS; ++p) {
        const bf16x4 lo = __builtin_shufflevector(bw[p], bw[p], 0, 1, 2, 3);
        const bf16x4 hi = __builtin_shufflevector(bw[p], bw[p], 4, 5, 6, 7);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[2 * p], lo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[2 * p + 1], hi, acc, 0, 0, 0);
    }
}

template <int PAIRS>
__device__ inline void fwd_batch(const uint16_t* A, int as, const uint16_t* WF, int64_t fb, int K, int nb, int k0,
                                 int rr, int q4, int lane, f32x4& acc) {
    bf16x8 bw[PAIRS];
    fwd_load<PAIRS>(WF, fb, K, nb, k0, lane, bw);
    // every load of the batch is issued before the first product waits (the
    // scheduler would otherwise interleave them with the MFMAs, one memory
    // round trip after another)
    __builtin_amdgcn_sched_barrier(0);
    fwd_mma<PAIRS>(A, as, k0, rr, q4, bw, acc);
}

// acc += A W on the 16-column block nb of W [K][.] over inputs [k0, K)
// (fragment copy at fb; its columns are padded with zeros to a multiple of
// 64, so every block of a 256-column tile exists; K - k0 is a multiple of 128)
__device__ inline void fwd_block(const uint16_t* A, int as, const uint16_t* WF, int64_t fb, int K, int nb, int k0,
                                 int rr, int q4, int lane, f32x4& acc) {
    for (; k0 + 32 * kFwdPairs <= K; k0 += 32 * kFwdPairs)
        fwd_batch<kFwdPairs>(A, as, WF, fb, K, nb, k0, rr, q4, lane, acc);
    if (k0 < K) fwd_batch<kFwdPairs / 2>(A, as, WF, fb, K, nb, k0, rr, q4, lane, acc);
}

__global__ __launch_bounds__(1024) void k_forward_small(MlpDev M, DevPtrs<float> P, ShapeInfo sh, int src, float* O) {
    extern __shared__ __align__(16) uint16_t fsm[];
    const int N = M.N, H = M.H, In = M.In, Out = M.Out, B = M.Bm;
    const int net = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rr = lane & 15, q4 = 4 * (lane >> 4);
    const int xs = In + 4, hs = H + 4;  // LDS row strides (8-byte aligned rows)
    uint16_t* x0 = fsm;
    uint16_t* h1 = x0 + kFwdRows * xs;
    uint16_t* h2 = h1 + kFwdRows * hs;
    const uint16_t* WF = M.wbt + (int64_t)net * M.NPt;
    const float* bn = M.master + (int64_t)net * M.NP;
    // the wave's first layer-1 fragments (inputs 0..127) do not depend on the
    // features: their loads are in flight while the features are formed
    bf16x8 w1[kFwdPairs / 2];
    if (16 * wave < H) fwd_load<kFwdPairs / 2>(WF, 0, In, wave, 0, lane, w1);
    // the input tile: features of each row's configuration rounded to bfloat16, zero rows beyond the batch
    const int slot = M.temp_index[net];
    for (int i = threadIdx.x; i < kFwdRows * N; i += blockDim.x) {
        const int row = i / N, k = i - row * N;
        uint16_t re = 0, im = 0;
        if (row < B) {
            const float* a = src == kFwdCurrent ? copy_amp(P, sh, N, P.copy_at[(int64_t)row * sh.n_temps + slot])
                                                : M.ap + ((int64_t)net * B + row) * 2 * N;
            float fr, fi;
            feature_of(a, k, fr, fi);
            re = f_to_bf16(fr);
            im = f_to_bf16(fi);
        }
        x0[row * xs + k] = re;
        x0[row * xs + N + k] = im;
    }
    if (src == kFwdCurrent && blockIdx.x == 0) {
        if ((int)threadIdx.x < B) M.item_copy[(int64_t)net * B + threadIdx.x] = P.copy_at[(int64_t)threadIdx.x * sh.n_temps + slot];
        // the round's index for the move draws: the later kernels of the round read it minus one
        if (net == 0 && threadIdx.x == 0) *M.moves_done += 1;
    }
    __syncthreads();
    // dst[row][col] = bf16(SiLU(A W + b)) for the batch's rows, 0 beyond
    auto hidden = [&](const uint16_t* A, int as, int64_t fb, const float* bias, int K, uint16_t* dst, bool first) {
        for (int nb = wave; 16 * nb < H; nb += kFwdWaves) {
            f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            if (first && nb == wave) {  // the prefetched fragments, then the rest of K
                fwd_mma<kFwdPairs / 2>(A, as, 0, rr, q4, w1, acc);
                fwd_block(A, as, WF, fb, K, nb, 128, rr, q4, lane, acc);
            } else {
                fwd_block(A, as, WF, fb, K, nb, 0, rr, q4, lane, acc);
            }
            const int col = 16 * nb + rr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = q4 + v;
                dst[row * hs + col] = row < B ? f_to_bf16(silu(acc[v] + bias[col])) : (uint16_t)0;
            }
        }
        __syncthreads();
    };
    hidden(x0, xs, 0, bn + M.ob1, In, h1, true);
    hidden(h1, hs, frag_w2(M), bn + M.ob2, H, h2, false);
    const int nb = blockIdx.x * 16 + wave;  // the output block of this wave
    if (16 * nb >= Out) return;
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    fwd_block(h2, hs, WF, frag_w3(M), H, nb, 0, rr, q4, lane, acc);
    const int col = 16 * nb + rr;
    if (col >= Out) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = q4 + v;
        if (row < B) O[(int64_t)net * B * Out + (int64_t)row * Out + col] = acc[v] + bn[M.ob3 + col];
    }
}

__global__ __launch_bounds__(64) void k_feat_current(MlpDev M, DevPtrs<float> P, ShapeInfo sh) {
    const int net = blockIdx.y, b = blockIdx.x, lane = threadIdx.x;
    const int mu = b / sh.n_reps, r = b % sh.n_reps;
    const int t = M.temp_index[net];
    const int c = P.copy_at[((int64_t)mu * sh.n_reps + r) * sh.n_temps + t];
    if (lane == 0) M.item_copy[net * M.Bm + b] = c;
    write_features(copy_amp(P, sh, M.N, c), M.N, M.X + ((int64_t)net * M.Bm + b) * M.In, lane);
    // the round's index for the move draws: the later kernels of the round read it minus one
    if (net == 0 && b == 0 && lane == 0) *M.moves_done += 1;
}

// log w_k and phases of one configuration held in global memory
__device__ inline float log_w(const float* a, int k, float logN) {
    const float u = a[2 * k] * a[2 * k] + a[2 * k + 1] * a[2 * k + 1];
    return 2.0f * logf(u) - logN;
}

// true in every lane when some amplitude of the configuration is zero or not
// finite: the configuration is then on the boundary of the alr chart (or
// garbage) and has no coordinates y
__device__ inline bool off_chart(const float* a, int N, int lane) {
    int bad = 0;
    for (int k = lane; k < N; k += 64) {
        const float x = a[2 * k], y = a[2 * k + 1];
        const float u = x * x + y * y;
        bad |= !(u > 0.0f) || !isfinite(x) || !isfinite(y) || !isfinite(u);
    }
    return __any(bad);
}

// the subset of a subset move or training item: a partial Fisher-Yates
// shuffle of 0..N-1 in LDS whose step t swaps position t with
// t + index_below(word(t), N - t), then the m drawn modes in ascending order.
// Called by every thread (tid of nt) of the workgroup.
template <typename Word>
__device__ inline void draw_subset(int N, int m, Word word, int* perm, int* S, int tid, int nt) {
    __shared__ int jt[kMaxSubset];
    for (int k = tid; k < N; k += nt) perm[k] = k;
    for (int t = tid; t < m; t += nt) jt[t] = t + index_below(word(t), N - t);  // the words, in parallel
    __syncthreads();
    if (tid == 0)
        for (int t = 0; t < m; ++t) {
            const int j = jt[t];
            const int x = perm[t];
            perm[t] = perm[j];
            perm[j] = x;
        }
    __syncthreads();
    if (tid < m) {
        const int v = perm[tid];
        int r = 0;
        for (int t = 0; t < m; ++t) r += perm[t] < v ? 1 : 0;
        S[r] = v;
    }
    __syncthreads();
}

// the output channel (within a component's D values) of subset coordinate d:
// the y channel of s_d for d < m - 1, then the phase channels of s_1 .. s_m
__device__ inline int subset_channel(const int* S, int d, int m, int N) {
    return d < m - 1 ? S[d] : N - 1 + S[d - (m - 1)];
}

// true in every lane when a mode of S is zero or not finite in configuration a
__device__ inline bool subset_off_chart(const float* a, const int* S, int m, int lane) {
    int bad = 0;
    for (int i = lane; i < m; i += 64) {
        const float x = a[2 * S[i]], y = a[2 * S[i] + 1];
        const float u = x * x + y * y;
        bad |= !(u > 0.0f) || !isfinite(x) || !isfinite(y) || !isfinite(u);
    }
    return __any(bad);
}

// a training pair: features of the first configuration and the displacement
// (dy, dpsi) to the second.  A pair with either configuration off the chart is
// left out (tvalid = 0; features and displacement written as zeros so that
// nothing non-finite reaches the products)
__global__ __launch_bounds__(64) void k_feat_train(MlpDev M, uint64_t seed, int64_t step, int use_first) {
    const int net = blockIdx.y, b = blockIdx.x, lane = threadIdx.x;
    const int N = M.N;
    int idx = b;
    if (!use_first) {
        const Philox4 w = philox4x64((uint64_t)step, (uint64_t)net, (uint64_t)b, 0, seed, kTagTrain);
        const int cnt = M.count[net] < M.cap ? M.count[net] : M.cap;
        idx = index_below(w.v[0], cnt > 0 ? cnt : 1);
    }
    const float* before = M.data + (((int64_t)net * M.cap + idx) * 2 + 0) * 2 * N;
    const float* after = M.data + (((int64_t)net * M.cap + idx) * 2 + 1) * 2 * N;
    const int64_t item = (int64_t)net * M.Bt + b;
    float* dl = M.tdelta + item * M.D;
    if (M.m > 0) {  // subset move: a subset per item, the displacement in its chart
        __shared__ int perm[kMaxModes / 2];
        __shared__ int S[kMaxSubset];
        const int m = M.m;
        draw_subset(N, m, [&](int t) {
            return word_of(philox4x64((uint64_t)step, (uint64_t)net, (uint64_t)b, (uint64_t)(1 + t / 4), seed, kTagTrain),
                           t & 3);
        }, perm, S, lane, 64);
        for (int i = lane; i < m; i += 64) M.tsub[item * kMaxSubset + i] = S[i];
        const bool out = subset_off_chart(before, S, m, lane) || subset_off_chart(after, S, m, lane);
        if (lane == 0) M.tvalid[item] = out ? 0 : 1;
        if (out) {
            for (int k = lane; k < M.In; k += 64) M.tX[item * M.In + k] = 0.0f;
            for (int d = lane; d < M.D; d += 64) dl[d] = 0.0f;
            return;
        }
        write_features(before, N, M.tX + item * M.In, lane);
        const float logN = logf((float)N);
        const int sl = S[m - 1];
        const float lw0 = log_w(before, sl, logN), lw1 = log_w(after, sl, logN);
        for (int i = lane; i < m; i += 64) {
            const int k = S[i];
            if (i < m - 1) dl[i] = (log_w(after, k, logN) - lw1) - (log_w(before, k, logN) - lw0);
            const float p0 = atan2f(before[2 * k + 1], before[2 * k]);
            const float p1 = atan2f(after[2 * k + 1], after[2 * k]);
            dl[m - 1 + i] = wrapf(p1 - p0);
        }
        return;
    }
    const bool out = off_chart(before, N, lane) || off_chart(after, N, lane);
    if (lane == 0) M.tvalid[item] = out ? 0 : 1;
    if (out) {
        for (int k = lane; k < M.In; k += 64) M.tX[item * M.In + k] = 0.0f;
        for (int d = lane; d < M.D; d += 64) dl[d] = 0.0f;
        return;
    }
    write_features(before, N, M.tX + item * M.In, lane);
    const float logN = logf((float)N);
    const float lw0 = log_w(before, N - 1, logN), lw1 = log_w(after, N - 1, logN);
    for (int k = lane; k < N; k += 64) {
        if (k < N - 1) dl[k] = (log_w(after, k, logN) - lw1) - (log_w(before, k, logN) - lw0);
        const float p0 = atan2f(before[2 * k + 1], before[2 * k]);
        const float p1 = atan2f(after[2 * k + 1], after[2 * k]);
        dl[N - 1 + k] = wrapf(p1 - p0);
    }
}

// test hook: features of rows [0, n) of network net from the configurations in M.ap
__global__ __launch_bounds__(64) void k_feat_ap(MlpDev M, int net, int n) {
    const int b = blockIdx.x, lane = threadIdx.x;
    if (b >= n) return;
    const int64_t item = (int64_t)net * M.Bm + b;
    write_features(M.ap + item * 2 * M.N, M.N, M.X + item * M.In, lane);
}

// ------------------------------------------------------------------ mixture head
// log normaliser of the mixture weights: log w_c = O[c] - mix_lse(O, K)
__device__ inline float mix_lse(const float* O, int K) {
    float mx = -INFINITY;
    for (int i = 0; i < K; ++i) mx = fmaxf(mx, O[i]);
    float s = 0.0f;
    for (int i = 0; i < K; ++i) s += expf(O[i] - mx);
    return mx + logf(s);
}

struct Mix {
    float lw[kMaxK];
};

__device__ inline void mix_weights(const float* O, int K, Mix& m) {
    const float lse = mix_lse(O, K);
    for (int i = 0; i < K; ++i) m.lw[i] = O[i] - lse;
}

__device__ inline float smax_of(int d, int N) { return d < N - 1 ? kSmaxY : kSmaxPsi; }

// the component of a move: the first c with sum_{i <= c} w_i > u
__device__ inline int mix_component(const float* O, int K, double u) {
    const float lse = mix_lse(O, K);
    double cum = 0.0;
    for (int i = 0; i < K; ++i) {
        cum += (double)expf(O[i] - lse);
        if (cum > u) return i;
    }
    return K - 1;
}

// log of one coordinate's density: a Gaussian (chart coordinate) or a wrapped
// Gaussian summed over |n| <= 3 (phase)
__device__ inline float log_coord(float x, float mu, float sg, bool phase) {
    if (!phase) {
        const float z = (x - mu) / sg;
        return -logf(sg) - 0.5f * kLog2Pi - 0.5f * z * z;
    }
    const float t0 = wrapf(x - mu);
    float s = 0.0f;
#pragma unroll
    for (int n = -3; n <= 3; ++n) {
        const float t = (t0 + 2.0f * kPiF * n) / sg;
        s += expf(-0.5f * t * t);
    }
    return logf(s) - logf(sg) - 0.5f * kLog2Pi;
}

// log-sum-exp over the components, accumulated one component at a time
struct Lse {
    float best = -INFINITY, s = 0.0f;
    __device__ void add(float t) {
        if (t == -INFINITY) return;  // a component of zero density adds nothing (all of them: the value is -inf)
        if (t > best) {
            s = s * expf(best - t) + 1.0f;
            best = t;
        } else {
            s += expf(t - best);
        }
    }
    __device__ float value() const { return best + logf(s); }
};

// the term of component mc of the log density of the (signed) displacement
// under the scaled mixture: log w_mc + sum_d log N(delta_d; mu, sigma) (wave-
// cooperative, the same value in every lane)
__device__ float mix_term(const float* O, float lse, const float* delta, float sign, float scale, int N, int K, int D,
                          int mc, int lane) {
    float part = 0.0f;
    for (int d = lane; d < D; d += 64) {
        const float mu = scale * O[K + mc * D + d];
        const float sg = scale * smax_of(d, N) * sigm(O[K + K * D + mc * D + d]);
        part += log_coord(sign * delta[d], mu, sg, d >= N - 1);
    }
    return O[mc] - lse + wsum(part);
}

// the same over the coordinates of a subset S (2m - 1 values in delta)
__device__ float mix_term_subset(const float* O, float lse, const int* S, const float* delta, float sign, float scale,
                                 int N, int K, int D, int m, int mc, int lane) {
    float part = 0.0f;
    for (int d = lane; d < 2 * m - 1; d += 64) {
        const int ch = subset_channel(S, d, m, N);
        const float mu = scale * O[K + mc * D + ch];
        const float sg = scale * smax_of(ch, N) * sigm(O[K + K * D + mc * D + ch]);
        part += log_coord(sign * delta[d], mu, sg, d >= m - 1);
    }
    return O[mc] - lse + wsum(part);
}

// the log density from its component terms: waves w0, w0 + 1, ... of the
// workgroup take components w0 + i, w0 + i + nw, ... (term(mc) is wave-
// cooperative), the terms meet in LDS and are combined in component order.
// Called by every thread; ends with a barrier; the value in every thread.
template <typename Term>
__device__ float log_mix_block(int K, Term term, float* sterm, int wave, int w0, int nw, int lane) {
    if (wave >= w0 && wave < w0 + nw)
        for (int mc = wave - w0; mc < K; mc += nw) {
            const float t = term(mc);
            if (lane == 0) sterm[mc] = t;
        }
    __syncthreads();
    Lse acc;
    for (int mc = 0; mc < K; ++mc) acc.add(sterm[mc]);
    const float v = acc.value();
    __syncthreads();  // sterm may be reused
    return v;
}

// log of the uniform that decides a learned move: word 1 of the Philox block
// after the move's Gaussians (counter word 3: 0 all-mode, 1 subset)
__device__ inline double accept_log_uniform(uint64_t seed, int64_t move, int c, int nb, int subset) {
    const Philox4 wu = philox4x64((uint64_t)nb, (uint64_t)move, (uint64_t)c, (uint64_t)subset, seed, kTagLearn);
    return log(uniform01<double>(wu.v[1]));
}

// training head: mean NLL of the unwrapped mixture and its gradient w.r.t. the outputs
__global__ __launch_bounds__(64) void k_head_train(MlpDev M) {
    const int net = blockIdx.y, b = blockIdx.x, lane = threadIdx.x;
    const int N = M.N, K = M.K, D = M.D;
    const int64_t item = (int64_t)net * M.Bt + b;
    const float* O = M.tO + item * M.Out;
    const float* dl = M.tdelta + item * D;
    float* dO = M.tdO + item * M.Out;
    // the loss is the mean over the minibatch's pairs inside the chart; the others get no gradient
    int nv = 0;
    for (int i = lane; i < M.Bt; i += 64) nv += M.tvalid[(int64_t)net * M.Bt + i];
    nv = (int)wsum((float)nv);  // exact: an integer count far below 2^24
    if (!M.tvalid[item] || nv == 0) {
        for (int o = lane; o < M.Out; o += 64) dO[o] = 0.0f;
        if (lane == 0) M.tloss[item] = 0.0f;
        return;
    }
    if (M.m > 0) {  // subset move: the likelihood of the subset's coordinates only
        const int m = M.m, nd = 2 * m - 1;
        const int* S = M.tsub + item * kMaxSubset;
        for (int o = lane; o < M.Out; o += 64) dO[o] = 0.0f;
        __syncthreads();  // the zeros are written before the subset's channels
        Mix mw;
        mix_weights(O, K, mw);
        float ell[kMaxK], best = -INFINITY;
        for (int mc = 0; mc < K; ++mc) {
            float part = 0.0f;
            for (int d = lane; d < nd; d += 64) {
                const int ch = subset_channel(S, d, m, N);
                const float sg = smax_of(ch, N) * sigm(O[K + K * D + mc * D + ch]);
                const float z = (dl[d] - O[K + mc * D + ch]) / sg;
                part += logf(sg) + 0.5f * kLog2Pi + 0.5f * z * z;
            }
            ell[mc] = mw.lw[mc] - wsum(part);
            best = fmaxf(best, ell[mc]);
        }
        float se = 0.0f;
        for (int mc = 0; mc < K; ++mc) se += expf(ell[mc] - best);
        const float logp = best + logf(se);
        const float inv = 1.0f / (float)nv;
        for (int mc = 0; mc < K; ++mc) {
            const float r = expf(ell[mc] - logp);
            if (lane == 0) dO[mc] = (expf(mw.lw[mc]) - r) * inv;
            for (int d = lane; d < nd; d += 64) {
                const int ch = subset_channel(S, d, m, N);
                const float sm = smax_of(ch, N);
                const float sg = sm * sigm(O[K + K * D + mc * D + ch]);
                const float z = (dl[d] - O[K + mc * D + ch]) / sg;
                dO[K + mc * D + ch] = -r * z / sg * inv;
                dO[K + K * D + mc * D + ch] = -r * (z * z - 1.0f) * (1.0f - sg / sm) * inv;
            }
        }
        if (lane == 0) M.tloss[item] = -logp;
        return;
    }
    Mix mw;
    mix_weights(O, K, mw);
    float ell[kMaxK], best = -INFINITY;
    for (int m = 0; m < K; ++m) {
        float part = 0.0f;
        for (int d = lane; d < D; d += 64) {
            const float sg = smax_of(d, N) * sigm(O[K + K * D + m * D + d]);
            const float z = (dl[d] - O[K + m * D + d]) / sg;
            part += logf(sg) + 0.5f * kLog2Pi + 0.5f * z * z;
        }
        ell[m] = mw.lw[m] - wsum(part);
        best = fmaxf(best, ell[m]);
    }
    float s = 0.0f;
    for (int m = 0; m < K; ++m) s += expf(ell[m] - best);
    const float logp = best + logf(s);
    const float inv = 1.0f / (float)nv;
    for (int m = 0; m < K; ++m) {
        const float r = expf(ell[m] - logp);
        if (lane == 0) dO[m] = (expf(mw.lw[m]) - r) * inv;
        for (int d = lane; d < D; d += 64) {
            const float sm = smax_of(d, N);
            const float sg = sm * sigm(O[K + K * D + m * D + d]);
            const float z = (dl[d] - O[K + m * D + d]) / sg;
            dO[K + m * D + d] = -r * z / sg * inv;
            dO[K + K * D + m * D + d] = -r * (z * z - 1.0f) * (1.0f - sg / sm) * inv;
        }
    }
    if (lane == 0) M.tloss[item] = -logp;
}

__global__ void k_silu_back(const float* dH, const float* P, float* dP, int64_t n) {
    const int64_t net = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float p = P[net * n + i];
        const float s = sigm(p);
        dP[net * n + i] = dH[net * n + i] * s * (1.0f + p * (1.0f - s));
    }
}

// column sums of Y [rows][cols] (bias gradients): 64 columns per 256-thread
// block, four row slices per column summed in a fixed order
__global__ __launch_bounds__(256) void k_colsum(const float* Y, int rows, int cols, int64_t sY, float* out,
                                                int64_t sOut) {
    __shared__ float part[4][64];
    const int net = blockIdx.y;
    const int c = threadIdx.x & 63, slice = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    float s = 0.0f;
    if (j < cols) {
        const float* y = Y + net * sY + j;
#pragma unroll 8
        for (int r = slice; r < rows; r += 4) s += y[(int64_t)r * cols];
    }
    part[slice][c] = s;
    __syncthreads();
    if (slice == 0 && j < cols) out[net * sOut + j] = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
}

// where parameter p of a net sits in the fragment copy (-1: a bias)
__device__ inline int64_t fragment_at(const MlpDev& M, int64_t p) {
    if (p >= M.oW1 && p < M.ob1) {
        const int64_t q = p - M.oW1;
        return frag_at(0, M.In, (int)(q / M.H), (int)(q % M.H));
    }
    if (p >= M.oW2 && p < M.ob2) {
        const int64_t q = p - M.oW2;
        return frag_at(frag_w2(M), M.H, (int)(q / M.H), (int)(q % M.H));
    }
    if (p >= M.oW3 && p < M.ob3) {
        const int64_t q = p - M.oW3;
        return frag_at(frag_w3(M), M.H, (int)(q / M.Out), (int)(q % M.Out));
    }
    return -1;
}
__device__ inline void store_bf16(const MlpDev& M, int64_t i, float w) {  // i over nets x NP
    const uint16_t b = f_to_bf16(w);
    M.wbf[i] = b;
    if (M.In % 32 != 0 || M.H % 32 != 0) return;  // no fragment order for this shape (the fused path is off)
    const int64_t net = i / M.NP, f = fragment_at(M, i - net * M.NP);
    if (f >= 0) M.wbt[net * M.NPt + f] = b;
}

__global__ void k_adam(MlpDev M, float lr, float c1, float c2) {
    const int64_t n = (int64_t)M.nets * M.NP;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float g = M.grad[i];
        const float m = 0.9f * M.am[i] + 0.1f * g;
        const float v = 0.999f * M.av[i] + 0.001f * g * g;
        M.am[i] = m;
        M.av[i] = v;
        const float w = M.master[i] - lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
        M.master[i] = w;
        store_bf16(M, i, w);
    }
}

__global__ void k_sync_bf16(MlpDev M) {
    const int64_t n = (int64_t)M.nets * M.NP;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        store_bf16(M, i, M.master[i]);
}

// ------------------------------------------------------------------ the move
// one standard normal of the move's draw (Box-Muller in FP64 on Philox words)
__device__ inline float move_gauss(uint64_t seed, int64_t move, int c, int d) {
    const Philox4 w = philox4x64((uint64_t)(d >> 1), (uint64_t)move, (uint64_t)c, 0, seed, kTagLearn);
    const int h = d & 1;
    const double u1 = 1.0 - uniform01<double>(word_of(w, 2 * h));
    const double u2 = uniform01<double>(word_of(w, 2 * h + 1));
    return (float)(sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2));
}

// The all-mode move's proposal.  Four waves share the serial work: wave 0
// picks the component and the current chart coordinates while wave 1 draws
// the Gaussians and wave 2 the acceptance uniform; every thread forms the
// displacement; wave 0 builds the proposal; every wave then writes its
// features and sums components of the forward log density.
__global__ __launch_bounds__(256) void k_propose(MlpDev M, DevPtrs<float> P, ShapeInfo sh, float scale) {
    extern __shared__ float sO[];  // [Out] the item's network outputs, staged in one round of loads
    __shared__ float sdel[2 * kMaxModes];
    __shared__ float slw[kMaxModes / 2];
    __shared__ float2 sp[kMaxModes / 2];  // the proposal
    __shared__ float sterm[kMaxK];
    __shared__ int s_mc, s_out;
    __shared__ float s_dref;
    const int net = blockIdx.y, b = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x, wave = tid >> 6, lane = tid & 63;
    const int N = M.N, K = M.K, D = M.D;
    const int64_t item = (int64_t)net * M.Bm + b;
    const int c = M.item_copy[item];
    const int64_t move = *M.moves_done - 1;
    for (int i = tid; i < M.Out; i += nt) sO[i] = M.Of[item * M.Out + i];
    __syncthreads();
    const float* O = sO;
    const float* a = copy_amp(P, sh, N, c);
    const float logN = logf((float)N);
    const int nb = (D + 1) / 2;
    if (wave == 0) {  // the component, the current chart coordinates
        const Philox4 wu = philox4x64((uint64_t)nb, (uint64_t)move, (uint64_t)c, 0, sh.run_seed, kTagLearn);
        const int mc = mix_component(O, K, uniform01<double>(wu.v[0]));
        if (lane == 0) s_mc = mc;
        for (int k = lane; k < N; k += 64) slw[k] = log_w(a, k, logN);
    } else if (wave == 1) {  // the standard normals
        for (int d = lane; d < D; d += 64) sdel[d] = move_gauss(sh.run_seed, move, c, d);
    } else if (wave == 2 && lane == 0) {
        M.lua[item] = accept_log_uniform(sh.run_seed, move, c, nb, 0);
    }
    __syncthreads();
    const int mc = s_mc;
    for (int d = tid; d < D; d += nt) {
        const float mu = scale * O[K + mc * D + d];
        const float sg = scale * smax_of(d, N) * sigm(O[K + K * D + mc * D + d]);
        const float del = mu + sg * sdel[d];
        sdel[d] = del;
        M.delta[item * D + d] = del;
    }
    __syncthreads();
    if (wave == 0) {
        // new intensities from y' = y + dy (y'_{N-1} = 0), normalised on the simplex
        const float last = slw[N - 1];
        float mx = -INFINITY;
        for (int k = lane; k < N; k += 64) mx = fmaxf(mx, k < N - 1 ? slw[k] - last + sdel[k] : 0.0f);
        mx = wmax(mx);
        float se = 0.0f;
        for (int k = lane; k < N; k += 64) se += expf((k < N - 1 ? slw[k] - last + sdel[k] : 0.0f) - mx);
        const float lse = mx + logf(wsum(se));
        float dref = 0.0f;
        int bad = 0;
        for (int k = lane; k < N; k += 64) {
            const float lwn = (k < N - 1 ? slw[k] - last + sdel[k] : 0.0f) - lse;
            dref += 0.5f * (lwn - slw[k]);
            const float A = expf(0.25f * (logN + lwn));
            const float x = a[2 * k], y = a[2 * k + 1];
            const float ph = atan2f(y, x) + sdel[N - 1 + k];
            float sn, cs;
            sincosf(ph, &sn, &cs);
            const float2 v = make_float2(A * cs, A * sn);
            sp[k] = v;
            // a move from a configuration off the alr chart (a zero amplitude), or
            // to a proposal with an intensity that underflowed to zero, is rejected
            const float u0 = x * x + y * y, u1 = v.x * v.x + v.y * v.y;
            bad |= !(u0 > 0.0f) || !isfinite(x) || !isfinite(y) || !isfinite(u0);
            bad |= !(u1 > 0.0f) || !isfinite(v.x) || !isfinite(v.y) || !isfinite(u1);
        }
        dref = wsum(dref);
        const bool out = __any(bad);
        if (lane == 0) {
            s_out = out;
            s_dref = out ? -INFINITY : dref;
        }
    }
    __syncthreads();
    // the proposal (the current configuration when rejected: the later stages see finite values only)
    const bool out = s_out;
    float* ap = M.ap + item * 2 * N;
    for (int k = tid; k < N; k += nt) {
        const float2 v = out ? make_float2(a[2 * k], a[2 * k + 1]) : sp[k];
        if (out) sp[k] = v;
        ap[2 * k] = v.x;
        ap[2 * k + 1] = v.y;
    }
    if (out) __syncthreads();
    float* X = M.X + item * M.In;  // the network's input at the proposal
    for (int k = tid; k < N; k += nt) {
        float fr, fi;
        feature_of(reinterpret_cast<const float*>(sp), k, fr, fi);
        X[k] = fr;
        X[N + k] = fi;
    }
    const float mlse = mix_lse(O, K);
    const float lq = log_mix_block(K, [&](int m) { return mix_term(O, mlse, sdel, 1.0f, scale, N, K, D, m, lane); },
                                   sterm, wave, 0, nt >> 6, lane);
    if (tid == 0) {
        M.lqf[item] = lq;
        M.dref[item] = s_dref;
    }
}

// energy change H(a') - H(a) over the by-term list, FP32.  The learned items of
// one sample (every network's temperature x replicas) share that sample's
// list: a workgroup holds up to kEnergyItems of them (current and proposed
// amplitudes in LDS) and streams a contiguous range of terms once for all of
// them; M.eparts workgroups per item group fill the chip, and the parts
// are added in a fixed order by the accept stage.
constexpr int kEnergyItems = 8;

__global__ __launch_bounds__(256) void k_energy_change(MlpDev M, DevPtrs<float> P, ShapeInfo sh, int groups,
                                                       int gsize) {
    extern __shared__ float2 samp[];  // [ni][2][N]: current, proposed
    __shared__ float red[4][kEnergyItems];
    const int N = M.N;
    const int parts = M.eparts;
    const int part = blockIdx.x % parts;
    const int grp = (blockIdx.x / parts) % groups;
    const int mu = blockIdx.x / (parts * groups);
    const int per_sample = M.nets * sh.n_reps;
    const int j0 = grp * gsize;
    const int ni = per_sample - j0 < gsize ? per_sample - j0 : gsize;
    auto item_of = [&](int i) -> int64_t {
        const int j = j0 + i, net = j / sh.n_reps, r = j % sh.n_reps;
        return (int64_t)net * M.Bm + (int64_t)mu * sh.n_reps + r;
    };
    for (int i = 0; i < ni; ++i) {
        const int64_t item = item_of(i);
        const float* a = copy_amp(P, sh, N, M.item_copy[item]);
        const float* ap = M.ap + item * 2 * N;
        float2* s0 = samp + (size_t)(2 * i) * N;
        float2* s1 = s0 + N;
        for (int k = threadIdx.x; k < N; k += blockDim.x) {
            s0[k] = make_float2(a[2 * k], a[2 * k + 1]);
            s1[k] = make_float2(ap[2 * k], ap[2 * k + 1]);
        }
    }
    __syncthreads();
    const SampleDev sd = P.samples[mu];
    const ushort4* Q = P.quads + sd.quad_base;
    const double* Jq = P.Jq + sd.quad_base;
    const int64_t q0 = sd.n_quads * part / parts, q1 = sd.n_quads * (part + 1) / parts;
    float acc[kEnergyItems];
#pragma unroll
    for (int i = 0; i < kEnergyItems; ++i) acc[i] = 0.0f;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        const ushort4 t = Q[q];
        const float J = (float)Jq[q];
#pragma unroll
        for (int i = 0; i < kEnergyItems; ++i) {
            if (i >= ni) break;
            const float2* s0 = samp + (size_t)(2 * i) * N;
            const float2* s1 = s0 + N;
            float2 p = s0[t.x], s = s0[t.y], m = s0[t.z], n = s0[t.w];
            float cr = p.x * s.x - p.y * s.y, ci = -(p.x * s.y + p.y * s.x);
            float dr = m.x * n.x - m.y * n.y, di = m.x * n.y + m.y * n.x;
            const float x0 = cr * dr - ci * di;
            p = s1[t.x], s = s1[t.y], m = s1[t.z], n = s1[t.w];
            cr = p.x * s.x - p.y * s.y, ci = -(p.x * s.y + p.y * s.x);
            dr = m.x * n.x - m.y * n.y, di = m.x * n.y + m.y * n.x;
            const float x1 = cr * dr - ci * di;
            acc[i] += -2.0f * J * (x1 - x0);
        }
    }
#pragma unroll
    for (int i = 0; i < kEnergyItems; ++i) {
        if (i >= ni) break;
        const float v = wsum(acc[i]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < ni) {
        const int i = threadIdx.x;
        M.dEp[item_of(i) * kMaxEnergyParts + part] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    }
}

// one standard normal of a subset move's draw (Box-Muller in FP64 on Philox words)
__device__ inline float subset_gauss(uint64_t seed, int64_t move, int c, int d) {
    const Philox4 w = philox4x64((uint64_t)(d >> 1), (uint64_t)move, (uint64_t)c, 1, seed, kTagLearn);
    const int h = d & 1;
    const double u1 = 1.0 - uniform01<double>(word_of(w, 2 * h));
    const double u2 = uniform01<double>(word_of(w, 2 * h + 1));
    return (float)(sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2));
}

// subset move: the proposal and its energy change, one workgroup per item.
// The item's network outputs and configuration are staged in LDS first (one
// round of loads instead of one per dependent read).  Wave 0 draws the
// component and the displacement of the subset's chart coordinates and forms
// the proposal (other modes copied), the reference ratio, the forward log
// density and the network's input at the proposal; then every wave sums the
// energy change from the subset's lists as the mode-by-mode sum
// dE = sum_i -2 Re(conj(a'_i - a_i) F_i), F_i on a snapshot that already
// holds the proposal for the modes before s_i (exact: every term holds a mode
// at most once).
template <int BLOCK, int UNITS>
__global__ __launch_bounds__(BLOCK) void k_propose_subset(MlpDev M, DevPtrs<float> P, ShapeInfo sh, float scale) {
    extern __shared__ float dyn[];  // [N] float2 snapshot, [N] float2 proposal, [Out] outputs
    __shared__ int perm[kMaxModes / 2];
    __shared__ int S[kMaxSubset];
    __shared__ float sdel[2 * kMaxSubset];
    __shared__ float slw[kMaxSubset];
    __shared__ float2 snew[kMaxSubset];
    __shared__ float red[16][2];
    __shared__ int uoff[kMaxSubset + 1];
    __shared__ uint32_t ustart[kMaxSubset];
    __shared__ float sterm[kMaxK];
    __shared__ int s_mc;
    __shared__ float s_dref;
    const int N = M.N, K = M.K, D = M.D, m = M.m;
    float2* sa = reinterpret_cast<float2*>(dyn);
    float2* sp = sa + N;
    float* sO = dyn + 4 * N;
    const int tid = threadIdx.x, nt = blockDim.x, wave = tid >> 6, lane = tid & 63;
    const int net = blockIdx.y;
    const int64_t item = (int64_t)net * M.Bm + blockIdx.x;
    const int c = M.item_copy[item];
    const int64_t move = *M.moves_done - 1;
    const float* a = copy_amp(P, sh, N, c);
    const float* O = M.Of + item * M.Out;
    for (int k = tid; k < N; k += nt) sa[k] = sp[k] = make_float2(a[2 * k], a[2 * k + 1]);
    for (int i = tid; i < M.Out; i += nt) sO[i] = O[i];
    draw_subset(N, m, [&](int t) {
        return word_of(philox4x64((uint64_t)(m + 1 + t / 4), (uint64_t)move, (uint64_t)c, 1, sh.run_seed, kTagLearn),
                       t & 3);
    }, perm, S, tid, nt);  // ends with a barrier: the staged values are visible too
    const float logN = logf((float)N);
    auto lw_of = [&](float2 v) { return 2.0f * logf(v.x * v.x + v.y * v.y) - logN; };  // log w_k
    // wave 0: the component and the subset's chart coordinates; wave 1: the
    // standard normals; wave 2: the acceptance uniform
    if (wave == 0) {
        const Philox4 wu = philox4x64((uint64_t)m, (uint64_t)move, (uint64_t)c, 1, sh.run_seed, kTagLearn);
        const int mc = mix_component(sO, K, uniform01<double>(wu.v[0]));
        if (lane == 0) s_mc = mc;
        for (int i = lane; i < m; i += 64) {
            slw[i] = lw_of(sa[S[i]]);
            M.subset[item * kMaxSubset + i] = S[i];
        }
    } else if (wave == 1) {
        for (int d = lane; d < 2 * m - 1; d += 64) sdel[d] = subset_gauss(sh.run_seed, move, c, d);
    } else if (wave == 2 && lane == 0) {
        M.lua[item] = accept_log_uniform(sh.run_seed, move, c, m, 1);
    }
    __syncthreads();
    if (wave == 0) {
        const int mc = s_mc;
        for (int d = lane; d < 2 * m - 1; d += 64) {
            const int ch = subset_channel(S, d, m, N);
            const float mu = scale * sO[K + mc * D + ch];
            const float sg = scale * smax_of(ch, N) * sigm(sO[K + K * D + mc * D + ch]);
            const float del = mu + sg * sdel[d];
            sdel[d] = del;
            M.delta[item * D + d] = del;
        }
    }
    __syncthreads();
    if (wave == 0) {
        // u' = u + du (u'_m = 0); the subset's total intensity is kept:
        // log w'_i = v_i - logsumexp(v) + logsumexp(log w_S)
        float mx = -INFINITY, mx0 = -INFINITY;
        for (int i = lane; i < m; i += 64) {
            mx = fmaxf(mx, i < m - 1 ? slw[i] - slw[m - 1] + sdel[i] : 0.0f);
            mx0 = fmaxf(mx0, slw[i]);
        }
        mx = wmax(mx);
        mx0 = wmax(mx0);
        float se = 0.0f, se0 = 0.0f;
        for (int i = lane; i < m; i += 64) {
            se += expf((i < m - 1 ? slw[i] - slw[m - 1] + sdel[i] : 0.0f) - mx);
            se0 += expf(slw[i] - mx0);
        }
        const float lse = mx + logf(wsum(se)), ltot = mx0 + logf(wsum(se0));
        float dref = 0.0f;
        int bad = 0;
        for (int i = lane; i < m; i += 64) {
            const float2 o = sa[S[i]];
            const float lwn = (i < m - 1 ? slw[i] - slw[m - 1] + sdel[i] : 0.0f) - lse + ltot;
            dref += 0.5f * (lwn - slw[i]);
            const float A = expf(0.25f * (logN + lwn));
            const float ph = atan2f(o.y, o.x) + sdel[m - 1 + i];
            float sn, cs;
            sincosf(ph, &sn, &cs);
            const float2 v = make_float2(A * cs, A * sn);
            snew[i] = v;
            // a move touching a zero amplitude of S (now or in the proposal) is rejected
            const float u0 = o.x * o.x + o.y * o.y, u1 = v.x * v.x + v.y * v.y;
            bad |= !(u0 > 0.0f) || !isfinite(o.x) || !isfinite(o.y) || !isfinite(u0);
            bad |= !(u1 > 0.0f) || !isfinite(v.x) || !isfinite(v.y) || !isfinite(u1);
        }
        dref = wsum(dref);
        if (__any(bad)) {
            for (int i = lane; i < m; i += 64) snew[i] = sa[S[i]];
            dref = -INFINITY;
        }
        for (int i = lane; i < m; i += 64) sp[S[i]] = snew[i];
        if (lane == 0) s_dref = dref;
    }
    __syncthreads();
    {  // the forward log density, components over the waves
        const float mlse = mix_lse(sO, K);
        const float lq = log_mix_block(
            K, [&](int mc) { return mix_term_subset(sO, mlse, S, sdel, 1.0f, scale, N, K, D, m, mc, lane); }, sterm,
            wave, 0, nt >> 6, lane);
        if (tid == 0) {
            M.lqf[item] = lq;
            M.dref[item] = s_dref;
        }
    }
    // the proposal, and its features for the GEMM forward
    float* ap = M.ap + item * 2 * N;
    float* X = M.X + item * M.In;
    for (int k = tid; k < N; k += nt) {
        const float2 v = sp[k];
        ap[2 * k] = v.x;
        ap[2 * k + 1] = v.y;
        float fr, fi;
        feature_of(reinterpret_cast<const float*>(sp), k, fr, fi);
        X[k] = fr;
        X[N + k] = fi;
    }
    if (s_dref == -INFINITY) {  // rejected: no energy change is needed
        if (tid == 0) M.dE[item] = 0.0f;
        return;
    }
    // The energy change in one pass over the subset's lists.  An entry of the
    // list of s_i sees the proposal at the modes s_j, j < i, and the current
    // configuration elsewhere (the snapshot of the mode-by-mode sum), so its
    // term -2 Re(conj(a'_i - a_i) J conj(a_x) a_y a_z) needs no other entry:
    // the lists are streamed together, several units per thread in flight.
    // pos[k] = rank of mode k in S (m when k is not in S); units = chunks of 4
    // entries (chunked lists) or groups of 4 entries (packed lists).
    int* pos = perm;  // the shuffle is no longer needed
    const SampleDev sd = P.samples[c / sh.copies_per_sample];
    const bool chunked = sh.layout == kLayoutChunked;
    const uint32_t* us = chunked ? P.chunk_start + sd.mode_base : P.mode_start + sd.mode_base;
    const int ushift = chunked ? 0 : 2;  // packed lists: mode_start counts entries (a multiple of 4)
    for (int k = tid; k < N; k += nt) pos[k] = m;
    if (wave == 0) {  // unit offsets of the lists in S order: an inclusive scan over the wave
        const int l = lane < m ? S[lane] : 0;
        int len = lane < m ? (int)((us[l + 1] - us[l]) >> ushift) : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(len, o, 64);
            if (lane >= o) len += v;
        }
        if (lane < m) {
            uoff[lane + 1] = len;
            ustart[lane] = us[l] >> ushift;
        }
        if (lane == 0) uoff[0] = 0;
    }
    __syncthreads();
    for (int i = tid; i < m; i += nt) pos[S[i]] = i;
    __syncthreads();
    auto val = [&](int k, int i) { return pos[k] < i ? sp[k] : sa[k]; };
    const int total = uoff[m];
    constexpr int kU = UNITS;  // units per thread in flight
    float part = 0.0f;
    int i = 0;
    for (int g0 = tid; g0 < total; g0 += kU * nt) {
        int li[kU];
        uint32_t qi[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int g = g0 + u * nt;
            li[u] = -1;
            if (g < total) {
                while (g >= uoff[i + 1]) ++i;
                li[u] = i;
                qi[u] = ustart[i] + (uint32_t)(g - uoff[i]);
            }
        }
        if (chunked) {
            uint32_t xv[kU];
            uint2 yzv[kU];
            float4 jv[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (li[u] >= 0) {
                    xv[u] = P.cx[qi[u]];
                    yzv[u] = P.cyz[qi[u]];
                    jv[u] = reinterpret_cast<const float4*>(P.cJ)[qi[u]];
                }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (li[u] < 0) continue;
                const int ii = li[u];
                const float2 ax = val(xv[u], ii);
                const uint32_t v[4] = {yzv[u].x & 0xffffu, yzv[u].x >> 16, yzv[u].y & 0xffffu, yzv[u].y >> 16};
                const float jj[4] = {jv[u].x, jv[u].y, jv[u].z, jv[u].w};
                float gr = 0.0f, gi = 0.0f;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float2 ay = val(v[e] & 0xffu, ii), az = val((v[e] >> 8) & 0xffu, ii);
                    gr += jj[e] * (ay.x * az.x - ay.y * az.y);
                    gi += jj[e] * (ay.x * az.y + ay.y * az.x);
                }
                const float fr = ax.x * gr + ax.y * gi, fi = ax.x * gi - ax.y * gr;
                const int l = S[ii];
                part += -2.0f * ((snew[ii].x - sa[l].x) * fr + (snew[ii].y - sa[l].y) * fi);
            }
        } else {
            uint4 iv[kU];
            float4 jv[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (li[u] >= 0) {
                    iv[u] = reinterpret_cast<const uint4*>(P.idx)[qi[u]];
                    jv[u] = reinterpret_cast<const float4*>(P.J)[qi[u]];
                }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (li[u] < 0) continue;
                const int ii = li[u];
                const uint32_t ev[4] = {iv[u].x, iv[u].y, iv[u].z, iv[u].w};
                const float jj[4] = {jv[u].x, jv[u].y, jv[u].z, jv[u].w};
                float fr = 0.0f, fi = 0.0f;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float2 ax = val(ev[e] & 1023u, ii), ay = val((ev[e] >> 10) & 1023u, ii),
                                 az = val(ev[e] >> 20, ii);
                    const float pr = ax.x * ay.x + ax.y * ay.y, pi = ax.x * ay.y - ax.y * ay.x;
                    fr += jj[e] * (pr * az.x - pi * az.y);
                    fi += jj[e] * (pr * az.y + pi * az.x);
                }
                const int l = S[ii];
                part += -2.0f * ((snew[ii].x - sa[l].x) * fr + (snew[ii].y - sa[l].y) * fi);
            }
        }
    }
    part = wsum(part);
    if (lane == 0) red[wave][0] = part;
    __syncthreads();
    if (tid == 0) {
        float dE = 0.0f;
        for (int w = 0; w < (nt >> 6); ++w) dE += red[w][0];
        M.dE[item] = dE;
    }
}

// The loads of the item's data are issued together at the start (one round
// trip, then one for the inverse temperature and the running energy), the
// proposal row included: it is stored into the configuration only on
// acceptance.  The reverse log density's components are summed on the four
// waves; the uniform that decides was drawn with the proposal.
constexpr int kAcceptThreads = 256;
static_assert(kAcceptThreads >= kMaxEnergyParts, "one energy part per accept thread");
constexpr int kApPerThread = kMaxModes / kAcceptThreads;  // floats of the proposal row per thread (2N <= kMaxModes)

__global__ __launch_bounds__(kAcceptThreads) void k_accept(MlpDev M, DevPtrs<float> P, ShapeInfo sh, float scale) {
    extern __shared__ float sO[];  // [Out] the network's outputs at the proposal
    __shared__ float sdel[2 * kMaxModes];
    __shared__ int S[kMaxSubset];
    __shared__ float sterm[kMaxK];
    __shared__ int s_acc;
    const int net = blockIdx.y, b = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int N = M.N, K = M.K, D = M.D, m = M.m;
    const int64_t item = (int64_t)net * M.Bm + b;
    const int c = M.item_copy[item];
    const int slot = M.temp_index[net];
    const float dref = M.dref[item], lqf = M.lqf[item];
    const double lua = M.lua[item];
    __shared__ float s_part[kAcceptThreads / 64];
    // the all-mode move's energy change: its term-range parts, one per thread, summed in a fixed order
    float dE = m > 0 ? M.dE[item] : (tid < M.eparts ? M.dEp[item * kMaxEnergyParts + tid] : 0.0f);
    const int nd = m > 0 ? 2 * m - 1 : D;
    for (int d = tid; d < nd; d += kAcceptThreads) sdel[d] = M.delta[item * D + d];
    for (int i = tid; i < m; i += kAcceptThreads) S[i] = M.subset[item * kMaxSubset + i];
    for (int i = tid; i < M.Out; i += kAcceptThreads) sO[i] = M.Or[item * M.Out + i];
    const float* ap = M.ap + item * 2 * N;
    float apv[kApPerThread];
#pragma unroll
    for (int r = 0; r < kApPerThread; ++r)
        if (tid + kAcceptThreads * r < 2 * N) apv[r] = ap[tid + kAcceptThreads * r];
    const float beta = P.beta[slot];
    const float E0 = P.E[c];
    if (m == 0) {
        dE = wsum(dE);
        if (lane == 0) s_part[wave] = dE;
    }
    __syncthreads();
    if (m == 0) {
        dE = 0.0f;
        for (int w = 0; w < kAcceptThreads / 64; ++w) dE += s_part[w];
    }
    const float mlse = mix_lse(sO, K);
    const float lqr =
        m > 0 ? log_mix_block(
                    K, [&](int mc) { return mix_term_subset(sO, mlse, S, sdel, -1.0f, scale, N, K, D, m, mc, lane); },
                    sterm, wave, 0, kAcceptThreads / 64, lane)
              : log_mix_block(K, [&](int mc) { return mix_term(sO, mlse, sdel, -1.0f, scale, N, K, D, mc, lane); },
                              sterm, wave, 0, kAcceptThreads / 64, lane);
    const float la = dref == -INFINITY ? -INFINITY : -beta * dE + dref + lqr - lqf;
    if (tid == 0) {
        const bool accept = lua < (double)la;
        s_acc = accept;
        M.la[item] = la;
        M.dE[item] = dE;
        if (accept) {
            P.E[c] = E0 + dE;
            atomicAdd(&M.acc[net], 1ull);
        }
        atomicAdd(&M.tries[net], 1ull);
    }
    __syncthreads();
    if (s_acc) {
        float* a = P.amp + 2 * (int64_t)c * N;
#pragma unroll
        for (int r = 0; r < kApPerThread; ++r)
            if (tid + kAcceptThreads * r < 2 * N) a[tid + kAcceptThreads * r] = apv[r];
    }
}


__global__ __launch_bounds__(64) void k_harvest(MlpDev M, DevPtrs<float> P, ShapeInfo sh, int which, int slot0) {
    const int net = blockIdx.y, b = blockIdx.x, lane = threadIdx.x;
    const int64_t item = (int64_t)net * M.Bm + b;
    int c;
    if (which == 0) {
        const int mu = b / sh.n_reps, r = b % sh.n_reps;
        c = P.copy_at[((int64_t)mu * sh.n_reps + r) * sh.n_temps + M.temp_index[net]];
        if (lane == 0) M.item_copy[item] = c;
    } else {
        c = M.item_copy[item];
    }
    const int slot = (slot0 + b) % M.cap;
    const float* a = copy_amp(P, sh, M.N, c);
    float* dst = M.data + (((int64_t)net * M.cap + slot) * 2 + which) * 2 * M.N;
    for (int k = lane; k < 2 * M.N; k += 64) dst[k] = a[k];
}

}  // namespace

hipError_t mlp_features_train(const MlpDev& M, uint64_t seed, int64_t step, int use_first, hipStream_t st) {
    hipLaunchKernelGGL(k_feat_train, dim3(M.Bt, M.nets), dim3(64), 0, st, M, seed, step, use_first);
    return hipGetLastError();
}

bool mlp_fused_forward(const MlpDev& M) { return forward_small_fits(M); }

hipError_t mlp_forward_current(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, hipStream_t st) {
    if (forward_small_fits(M)) {
        hipLaunchKernelGGL(k_forward_small, dim3((M.Out + 255) / 256, M.nets), dim3(64 * kFwdWaves),
                           forward_small_lds(M.In, M.H), st, M, P, sh, (int)kFwdCurrent, M.Of);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_feat_current, dim3(M.Bm, M.nets), dim3(64), 0, st, M, P, sh);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : mlp_forward(M, 0, 0, st);
}

hipError_t mlp_forward_proposal(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float* O,
                                hipStream_t st) {
    if (forward_small_fits(M)) {
        hipLaunchKernelGGL(k_forward_small, dim3((M.Out + 255) / 256, M.nets), dim3(64 * kFwdWaves),
                           forward_small_lds(M.In, M.H), st, M, P, sh, (int)kFwdProposal, O);
        return hipGetLastError();
    }
    return mlp_forward(M, 0, O == M.Or ? 1 : 0, st);  // features in M.X (written with the proposals)
}

hipError_t mlp_forward(const MlpDev& M, int train, int into_reverse, hipStream_t st) {
    const int B = train ? M.Bt : M.Bm;
    const float* X = train ? M.tX : M.X;
    float* P1 = train ? M.tP1 : M.P1;
    float* H1 = train ? M.tH1 : M.H1;
    float* P2 = train ? M.tP2 : M.P2;
    float* H2 = train ? M.tH2 : M.H2;
    float* O = train ? M.tO : (into_reverse ? M.Or : M.Of);
    Gemm<uint16_t> g{};
    g.A = X; g.sA = (int64_t)B * M.In; g.as0 = M.In; g.as1 = 1;
    g.B = M.wbf + M.oW1; g.sB = M.NP; g.bs0 = M.H; g.bs1 = 1;
    g.bias = M.master + M.ob1; g.sBias = M.NP;
    g.Cpre = P1; g.Cact = H1; g.sC = (int64_t)B * M.H; g.M = B; g.N = M.H; g.K = M.In;
    hipError_t e = gemm<uint16_t, 1>(g, M.nets, st);
    if (e != hipSuccess) return e;
    g.A = H1; g.sA = (int64_t)B * M.H; g.as0 = M.H;
    g.B = M.wbf + M.oW2; g.bs0 = M.H;
    g.bias = M.master + M.ob2;
    g.Cpre = P2; g.Cact = H2; g.K = M.H;
    if ((e = gemm<uint16_t, 1>(g, M.nets, st)) != hipSuccess) return e;
    g.A = H2;
    g.B = M.wbf + M.oW3; g.bs0 = M.Out;
    g.bias = M.master + M.ob3;
    g.Cpre = O; g.Cact = nullptr; g.sC = (int64_t)B * M.Out; g.N = M.Out; g.K = M.H;
    return gemm<uint16_t, 0>(g, M.nets, st);
}

hipError_t mlp_backward(const MlpDev& M, hipStream_t st) {
    hipError_t e;
    const int B = M.Bt;
    hipLaunchKernelGGL(k_head_train, dim3(B, M.nets), dim3(64), 0, st, M);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    auto wgrad = [&](const float* act, int in, const float* dY, int out, int64_t off) {
        Gemm<float> g{};
        g.A = act; g.sA = (int64_t)B * in; g.as0 = 1; g.as1 = in;
        g.B = dY; g.sB = (int64_t)B * out; g.bs0 = out; g.bs1 = 1;
        g.bias = nullptr; g.Cpre = M.grad + off; g.sC = M.NP; g.M = in; g.N = out; g.K = B;
        return gemm<float, 0>(g, M.nets, st);
    };
    auto bgrad = [&](const float* dY, int out, int64_t off) {
        hipLaunchKernelGGL(k_colsum, dim3((out + 63) / 64, M.nets), dim3(256), 0, st, dY, B, out, (int64_t)B * out,
                           M.grad + off, M.NP);
        return hipGetLastError();
    };
    auto xgrad = [&](const float* dY, int out, int64_t woff, int in, float* dX) {
        Gemm<uint16_t> g{};
        g.A = dY; g.sA = (int64_t)B * out; g.as0 = out; g.as1 = 1;
        g.B = M.wbf + woff; g.sB = M.NP; g.bs0 = 1; g.bs1 = out;
        g.bias = nullptr; g.Cpre = dX; g.sC = (int64_t)B * in; g.M = B; g.N = in; g.K = out;
        return gemm<uint16_t, 0>(g, M.nets, st);
    };
    auto sback = [&](const float* dH, const float* P, float* dP) {
        const int64_t n = (int64_t)B * M.H;
        hipLaunchKernelGGL(k_silu_back, dim3((unsigned)((n + 255) / 256), M.nets), dim3(256), 0, st, dH, P, dP, n);
        return hipGetLastError();
    };
    if ((e = wgrad(M.tH2, M.H, M.tdO, M.Out, M.oW3)) != hipSuccess) return e;
    if ((e = bgrad(M.tdO, M.Out, M.ob3)) != hipSuccess) return e;
    if ((e = xgrad(M.tdO, M.Out, M.oW3, M.H, M.tdA)) != hipSuccess) return e;
    if ((e = sback(M.tdA, M.tP2, M.tdB)) != hipSuccess) return e;
    if ((e = wgrad(M.tH1, M.H, M.tdB, M.H, M.oW2)) != hipSuccess) return e;
    if ((e = bgrad(M.tdB, M.H, M.ob2)) != hipSuccess) return e;
    if ((e = xgrad(M.tdB, M.H, M.oW2, M.H, M.tdA)) != hipSuccess) return e;
    if ((e = sback(M.tdA, M.tP1, M.tdB)) != hipSuccess) return e;
    if ((e = wgrad(M.tX, M.In, M.tdB, M.H, M.oW1)) != hipSuccess) return e;
    return bgrad(M.tdB, M.H, M.ob1);
}

hipError_t mlp_adam(const MlpDev& M, float lr, int64_t t, hipStream_t st) {
    const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(1024), dim3(256), 0, st, M, lr, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_sync_bf16(const MlpDev& M, hipStream_t st) {
    hipLaunchKernelGGL(k_sync_bf16, dim3(1024), dim3(256), 0, st, M);
    return hipGetLastError();
}

hipError_t mlp_propose(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float scale, hipStream_t st) {
    hipLaunchKernelGGL(k_propose, dim3(M.Bm, M.nets), dim3(256), (size_t)M.Out * sizeof(float), st, M, P, sh, scale);
    return hipGetLastError();
}

hipError_t mlp_energy_change(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, hipStream_t st) {
    // one N for every sample (checked at creation); Bm = samples x replicas
    const int per_sample = M.nets * sh.n_reps;
    const int fit = (int)(61440 / (2 * M.N * sizeof(float2)));  // items whose amplitudes fit 60 KiB of LDS
    int gsize = kEnergyItems < fit ? kEnergyItems : fit;
    gsize = gsize < per_sample ? gsize : per_sample;
    const int groups = (per_sample + gsize - 1) / gsize;
    const int samples = M.Bm / sh.n_reps;
    const size_t lds = (size_t)gsize * 2 * M.N * sizeof(float2);
    hipLaunchKernelGGL(k_energy_change, dim3((unsigned)(samples * groups * M.eparts)), dim3(256), lds, st, M, P,
                       sh, groups, gsize);
    return hipGetLastError();
}

hipError_t mlp_propose_subset(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float scale,
                              hipStream_t st) {
    // threads per item grow with the list length (N = 256: 1024 threads, ~5 chunks each per list)
    const size_t lds = (size_t)M.N * 2 * sizeof(float2) + (size_t)M.Out * sizeof(float);
    const dim3 grid(M.Bm, M.nets);
    if (M.N >= 192)
        hipLaunchKernelGGL((k_propose_subset<1024, 4>), grid, dim3(1024), lds, st, M, P, sh, scale);
    else if (M.N >= 96)
        hipLaunchKernelGGL((k_propose_subset<512, 8>), grid, dim3(512), lds, st, M, P, sh, scale);
    else
        hipLaunchKernelGGL((k_propose_subset<256, 8>), grid, dim3(256), lds, st, M, P, sh, scale);
    return hipGetLastError();
}

hipError_t mlp_accept(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float scale, hipStream_t st) {
    hipLaunchKernelGGL(k_accept, dim3(M.Bm, M.nets), dim3(kAcceptThreads), (size_t)M.Out * sizeof(float), st, M, P, sh,
                       scale);
    return hipGetLastError();
}

hipError_t mlp_features_from_proposals(const MlpDev& M, int net, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_feat_ap, dim3((unsigned)n), dim3(64), 0, st, M, net, n);
    return hipGetLastError();
}

hipError_t mlp_harvest(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, int which, int slot0,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_harvest, dim3(M.Bm, M.nets), dim3(64), 0, st, M, P, sh, which, slot0);
    return hipGetLastError();
}

}  // namespace rlpt
