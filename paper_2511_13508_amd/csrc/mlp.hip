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

// ------------------------------------------------------------------ fused inference forward
// MFMA fragment order of a weight matrix W [K][n] (K % 16 == 0, columns padded
// to a multiple of 16): the B operand of v_mfma_f32_16x16x16_bf16 for column
// block nb and K step ks is W[16 ks + 4 (l / 16) + i][16 nb + l % 16] in lane l,
// slot i; those 64 x 4 elements are stored consecutively (lane-major), so one
// wave reads a fragment as 512 contiguous bytes
__host__ __device__ inline int64_t frag_at(int64_t base, int K, int k, int n) {
    return base + (((int64_t)(n / 16) * (K / 16) + k / 16) * 64 + (n % 16) + 16 * ((k % 16) / 4)) * 4 + (k % 4);
}
__host__ __device__ inline int64_t frag_w2(const MlpDev& M) { return (int64_t)M.In * M.H; }
__host__ __device__ inline int64_t frag_w3(const MlpDev& M) { return (int64_t)M.In * M.H + (int64_t)M.H * M.H; }
// Inference batches of at most 16 rows in one launch instead of three GEMMs.
// Workgroup (tile, net) computes both hidden layers of its net (every tile of
// a net repeats them; activations stay in LDS as bfloat16) and then output
// columns [256 tile, 256 tile + 256).  Each wave owns 64 columns of a layer
// (four 16 x 16 blocks) and loads its weight fragments straight from the
// fragment-order copy, eight K steps at a time, so no workgroup barrier falls
// inside a layer.  Every block sums its MFMAs over K in the order k_gemm does,
// with the same bfloat16 operands, bias and SiLU: the outputs are the same
// bits as the three-GEMM path.
constexpr int kFwdRows = 16;
constexpr int kFwdMaxTiles = 8;   // output tiles (256 columns each) up to which the fused path is used
constexpr int kFwdSteps = 8;      // K steps of 16 whose fragments are loaded together (K % 128 == 0)

__host__ __device__ inline size_t forward_small_lds(int H) { return (size_t)2 * kFwdRows * (H + 4) * sizeof(uint16_t); }

__global__ __launch_bounds__(256) void k_forward_small(MlpDev M, const float* X, float* O) {
    extern __shared__ __align__(16) uint16_t fsm[];
    const int H = M.H, In = M.In, Out = M.Out, B = M.Bm;
    const int net = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rr = lane & 15, q4 = 4 * (lane >> 4);
    const int hs = H + 4;  // LDS row stride of an activation tile (8-byte aligned rows)
    uint16_t* h1 = fsm;
    uint16_t* h2 = fsm + kFwdRows * hs;
    const float* Xn = X + (int64_t)net * B * In;
    const uint16_t* WF = M.wbt + (int64_t)net * M.NPt;
    const float* bn = M.master + (int64_t)net * M.NP;

    auto from_x = [&](int k) {  // row rr of the features at k .. k + 3, rounded on the way in
        bf16x4 f;
#pragma unroll
        for (int i = 0; i < 4; ++i) f[i] = (short)(rr < B ? f_to_bf16(Xn[(int64_t)rr * In + k + i]) : (uint16_t)0);
        return f;
    };
    auto from_h1 = [&](int k) { return *reinterpret_cast<const bf16x4*>(&h1[rr * hs + k]); };
    auto from_h2 = [&](int k) { return *reinterpret_cast<const bf16x4*>(&h2[rr * hs + k]); };
    // C = A W on the columns [n0, n0 + 64) of W [K][ncol] (fragment copy at fb):
    // this lane's accumulators of the four 16 x 16 blocks
    auto blocks = [&](auto afrag, int64_t fb, int K, int ncol, int n0, f32x4* acc) {
        const int nb0 = n0 / 16, nbs = (ncol + 15) / 16;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int k0 = 0; k0 < K; k0 += 16 * kFwdSteps) {  // the fragments of kFwdSteps steps in flight together
            bf16x4 af[kFwdSteps], bf[kFwdSteps][4];
#pragma unroll
            for (int t = 0; t < kFwdSteps; ++t) {
                const int ks = k0 / 16 + t;
                af[t] = afrag(16 * ks + q4);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bf[t][j] = nb0 + j < nbs
                                   ? *reinterpret_cast<const bf16x4*>(
                                         &WF[fb + (((int64_t)(nb0 + j) * (K / 16) + ks) * 64 + lane) * 4])
                                   : bf16x4{0, 0, 0, 0};
            }
#pragma unroll
            for (int t = 0; t < kFwdSteps; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[t], bf[t][j], acc[j], 0, 0, 0);
        }
    };
    // dst[row][col] = bf16(SiLU(A W + b)) for the batch's rows, 0 beyond
    auto hidden = [&](auto afrag, int64_t fb, const float* bias, int K, uint16_t* dst) {
        for (int n0 = 64 * wave; n0 < H; n0 += 256) {
            f32x4 acc[4];
            blocks(afrag, fb, K, H, n0, acc);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = n0 + 16 * j + rr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = q4 + v;
                    dst[row * hs + col] = row < B ? f_to_bf16(silu(acc[j][v] + bias[col])) : (uint16_t)0;
                }
            }
        }
        __syncthreads();
    };
    hidden(from_x, 0, bn + M.ob1, In, h1);
    hidden(from_h1, frag_w2(M), bn + M.ob2, H, h2);
    const int n0 = blockIdx.x * 256 + 64 * wave;  // output columns of this wave
    if (n0 >= Out) return;
    f32x4 acc[4];
    blocks(from_h2, frag_w3(M), H, Out, n0, acc);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = n0 + 16 * j + rr;
        if (col >= Out) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = q4 + v;
            if (row < B) O[(int64_t)net * B * Out + (int64_t)row * Out + col] = acc[j][v] + bn[M.ob3 + col];
        }
    }
}

// ------------------------------------------------------------------ features
// Re, Im of a rotated so that a_0 is real and positive
__device__ inline void write_features(const float* a, int N, float* X, int lane) {
    const float x0 = a[0], y0 = a[1];
    const float r = sqrtf(x0 * x0 + y0 * y0);
    const float cr = r > 0.0f ? x0 / r : 1.0f, ci = r > 0.0f ? -y0 / r : 0.0f;
    for (int k = lane; k < N; k += 64) {
        const float x = a[2 * k], y = a[2 * k + 1];
        X[k] = x * cr - y * ci;
        X[N + k] = x * ci + y * cr;
    }
}

__device__ inline const float* copy_amp(const DevPtrs<float>& P, const ShapeInfo& sh, int N, int c) {
    return P.amp + 2 * (int64_t)c * N;  // one N for every sample: copies are contiguous
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
// Called by every lane of a single-wave workgroup.
template <typename Word>
__device__ inline void draw_subset(int N, int m, Word word, int* perm, int* S, int lane) {
    __shared__ int jt[kMaxSubset];
    for (int k = lane; k < N; k += 64) perm[k] = k;
    for (int t = lane; t < m; t += 64) jt[t] = t + index_below(word(t), N - t);  // the words, in parallel
    __syncthreads();
    if (lane == 0)
        for (int t = 0; t < m; ++t) {
            const int j = jt[t];
            const int x = perm[t];
            perm[t] = perm[j];
            perm[j] = x;
        }
    __syncthreads();
    if (lane < m) {
        const int v = perm[lane];
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
            return philox4x64((uint64_t)step, (uint64_t)net, (uint64_t)b, (uint64_t)(1 + t / 4), seed, kTagTrain).v[t & 3];
        }, perm, S, lane);
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
struct Mix {
    float lw[kMaxK];
};

__device__ inline void mix_weights(const float* O, int K, Mix& m) {
    float mx = -INFINITY;
    for (int i = 0; i < K; ++i) mx = fmaxf(mx, O[i]);
    float s = 0.0f;
    for (int i = 0; i < K; ++i) s += expf(O[i] - mx);
    const float lse = mx + logf(s);
    for (int i = 0; i < K; ++i) m.lw[i] = O[i] - lse;
}

__device__ inline float smax_of(int d, int N) { return d < N - 1 ? kSmaxY : kSmaxPsi; }

// log density of the (signed) displacement under the scaled mixture, wave-cooperative
__device__ float log_mix(const float* O, const float* delta, float sign, float scale, int N, int K, int D, int lane) {
    Mix mw;
    mix_weights(O, K, mw);
    float best = -INFINITY, terms[kMaxK];
    for (int m = 0; m < K; ++m) {
        float part = 0.0f;
        for (int d = lane; d < D; d += 64) {
            const float mu = scale * O[K + m * D + d];
            const float sg = scale * smax_of(d, N) * sigm(O[K + K * D + m * D + d]);
            const float x = sign * delta[d];
            if (d < N - 1) {
                const float z = (x - mu) / sg;
                part += -logf(sg) - 0.5f * kLog2Pi - 0.5f * z * z;
            } else {
                const float t0 = wrapf(x - mu);
                float s = 0.0f;
#pragma unroll
                for (int n = -3; n <= 3; ++n) {
                    const float t = (t0 + 2.0f * kPiF * n) / sg;
                    s += expf(-0.5f * t * t);
                }
                part += logf(s) - logf(sg) - 0.5f * kLog2Pi;
            }
        }
        terms[m] = mw.lw[m] + wsum(part);
        best = fmaxf(best, terms[m]);
    }
    float s = 0.0f;
    for (int m = 0; m < K; ++m) s += expf(terms[m] - best);
    return best + logf(s);
}

// the same over the coordinates of a subset S (2m - 1 values in delta)
__device__ float log_mix_subset(const float* O, const int* S, const float* delta, float sign, float scale, int N,
                                int K, int D, int m, int lane) {
    Mix mw;
    mix_weights(O, K, mw);
    float best = -INFINITY, terms[kMaxK];
    for (int mc = 0; mc < K; ++mc) {
        float part = 0.0f;
        for (int d = lane; d < 2 * m - 1; d += 64) {
            const int ch = subset_channel(S, d, m, N);
            const float mu = scale * O[K + mc * D + ch];
            const float sg = scale * smax_of(ch, N) * sigm(O[K + K * D + mc * D + ch]);
            const float x = sign * delta[d];
            if (d < m - 1) {
                const float z = (x - mu) / sg;
                part += -logf(sg) - 0.5f * kLog2Pi - 0.5f * z * z;
            } else {
                const float t0 = wrapf(x - mu);
                float sw = 0.0f;
#pragma unroll
                for (int n = -3; n <= 3; ++n) {
                    const float t = (t0 + 2.0f * kPiF * n) / sg;
                    sw += expf(-0.5f * t * t);
                }
                part += logf(sw) - logf(sg) - 0.5f * kLog2Pi;
            }
        }
        terms[mc] = mw.lw[mc] + wsum(part);
        best = fmaxf(best, terms[mc]);
    }
    float se = 0.0f;
    for (int mc = 0; mc < K; ++mc) se += expf(terms[mc] - best);
    return best + logf(se);
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
    if (M.In % 16 != 0 || M.H % 16 != 0) return;  // no fragment order for this shape (the fused path is off)
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
    const double u1 = 1.0 - uniform01<double>(w.v[2 * h]);
    const double u2 = uniform01<double>(w.v[2 * h + 1]);
    return (float)(sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2));
}

__global__ __launch_bounds__(64) void k_propose(MlpDev M, DevPtrs<float> P, ShapeInfo sh, float scale) {
    __shared__ float sdel[2 * kMaxModes];
    __shared__ float slw[kMaxModes];
    const int net = blockIdx.y, b = blockIdx.x, lane = threadIdx.x;
    const int N = M.N, K = M.K, D = M.D;
    const int64_t item = (int64_t)net * M.Bm + b;
    const int c = M.item_copy[item];
    const int64_t move = *M.moves_done - 1;
    const float* O = M.Of + item * M.Out;
    const float* a = copy_amp(P, sh, N, c);
    // component
    Mix mw;
    mix_weights(O, K, mw);
    const int nb = (D + 1) / 2;
    const Philox4 wu = philox4x64((uint64_t)nb, (uint64_t)move, (uint64_t)c, 0, sh.run_seed, kTagLearn);
    const double uc = uniform01<double>(wu.v[0]);
    int m = K - 1;
    double cum = 0.0;
    for (int i = 0; i < K; ++i) {
        cum += (double)expf(mw.lw[i]);
        if (cum > uc) {
            m = i;
            break;
        }
    }
    for (int d = lane; d < D; d += 64) {
        const float mu = scale * O[K + m * D + d];
        const float sg = scale * smax_of(d, N) * sigm(O[K + K * D + m * D + d]);
        const float del = mu + sg * move_gauss(sh.run_seed, move, c, d);
        sdel[d] = del;
        M.delta[item * D + d] = del;
    }
    const float logN = logf((float)N);
    for (int k = lane; k < N; k += 64) slw[k] = log_w(a, k, logN);
    __syncthreads();
    // new intensities from y' = y + dy (y'_{N-1} = 0), normalised on the simplex
    const float last = slw[N - 1];
    float mx = -INFINITY;
    for (int k = lane; k < N; k += 64) mx = fmaxf(mx, k < N - 1 ? slw[k] - last + sdel[k] : 0.0f);
    mx = wmax(mx);
    float se = 0.0f;
    for (int k = lane; k < N; k += 64) se += expf((k < N - 1 ? slw[k] - last + sdel[k] : 0.0f) - mx);
    const float lse = mx + logf(wsum(se));
    float dref = 0.0f;
    float* ap = M.ap + item * 2 * N;
    for (int k = lane; k < N; k += 64) {
        const float lwn = (k < N - 1 ? slw[k] - last + sdel[k] : 0.0f) - lse;
        dref += 0.5f * (lwn - slw[k]);
        const float A = expf(0.25f * (logN + lwn));
        const float ph = atan2f(a[2 * k + 1], a[2 * k]) + sdel[N - 1 + k];
        float sn, cs;
        sincosf(ph, &sn, &cs);
        ap[2 * k] = A * cs;
        ap[2 * k + 1] = A * sn;
    }
    dref = wsum(dref);
    __syncthreads();  // ap complete
    // a move from a configuration off the alr chart (a zero amplitude), or to a
    // proposal with an intensity that underflowed to zero, is rejected: its
    // reference-density term is -inf, and the proposal is replaced by the
    // current configuration so that the later stages see finite values only
    const bool out = off_chart(a, N, lane) || off_chart(ap, N, lane);
    if (out) {
        for (int k = lane; k < 2 * N; k += 64) ap[k] = a[k];
        dref = -INFINITY;
    }
    __syncthreads();
    write_features(ap, N, M.X + item * M.In, lane);  // the network's input at the proposal
    const float lq = log_mix(O, sdel, 1.0f, scale, N, K, D, lane);
    if (lane == 0) {
        M.lqf[item] = lq;
        M.dref[item] = dref;
    }
}

// energy change H(a') - H(a) over the by-term list, FP32.  The learned items of
// one sample (every network's temperature x replicas) share that sample's
// list: a workgroup holds up to kEnergyItems of them (current and proposed
// amplitudes in LDS) and streams a contiguous range of terms once for all of
// them; kEnergyParts workgroups per item group fill the chip, and the parts
// are added in a fixed order by the accept stage.
constexpr int kEnergyItems = 8;

__global__ __launch_bounds__(256) void k_energy_change(MlpDev M, DevPtrs<float> P, ShapeInfo sh, int groups,
                                                       int gsize) {
    extern __shared__ float2 samp[];  // [ni][2][N]: current, proposed
    __shared__ float red[4][kEnergyItems];
    const int N = M.N;
    const int part = blockIdx.x % kEnergyParts;
    const int grp = (blockIdx.x / kEnergyParts) % groups;
    const int mu = blockIdx.x / (kEnergyParts * groups);
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
    const int64_t q0 = sd.n_quads * part / kEnergyParts, q1 = sd.n_quads * (part + 1) / kEnergyParts;
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
        M.dEp[item_of(i) * kEnergyParts + part] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    }
}

// one standard normal of a subset move's draw (Box-Muller in FP64 on Philox words)
__device__ inline float subset_gauss(uint64_t seed, int64_t move, int c, int d) {
    const Philox4 w = philox4x64((uint64_t)(d >> 1), (uint64_t)move, (uint64_t)c, 1, seed, kTagLearn);
    const int h = d & 1;
    const double u1 = 1.0 - uniform01<double>(w.v[2 * h]);
    const double u2 = uniform01<double>(w.v[2 * h + 1]);
    return (float)(sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2));
}

// subset move, stage one: the subset, the component, the displacement in the
// subset's chart, the proposal (other modes copied), the reference ratio, the
// forward log density and the network's input at the proposal
__global__ __launch_bounds__(64) void k_propose_subset(MlpDev M, DevPtrs<float> P, ShapeInfo sh, float scale) {
    __shared__ int perm[kMaxModes / 2];
    __shared__ int S[kMaxSubset];
    __shared__ float sdel[2 * kMaxSubset];
    __shared__ float slw[kMaxSubset];
    const int net = blockIdx.y, b = blockIdx.x, lane = threadIdx.x;
    const int N = M.N, K = M.K, D = M.D, m = M.m;
    const int64_t item = (int64_t)net * M.Bm + b;
    const int c = M.item_copy[item];
    const int64_t move = *M.moves_done - 1;
    const float* O = M.Of + item * M.Out;
    const float* a = copy_amp(P, sh, N, c);
    Mix mw;
    mix_weights(O, K, mw);
    const Philox4 wu = philox4x64((uint64_t)m, (uint64_t)move, (uint64_t)c, 1, sh.run_seed, kTagLearn);
    const double uc = uniform01<double>(wu.v[0]);
    int mc = K - 1;
    double cum = 0.0;
    for (int i = 0; i < K; ++i) {
        cum += (double)expf(mw.lw[i]);
        if (cum > uc) {
            mc = i;
            break;
        }
    }
    draw_subset(N, m, [&](int t) {
        return philox4x64((uint64_t)(m + 1 + t / 4), (uint64_t)move, (uint64_t)c, 1, sh.run_seed, kTagLearn).v[t & 3];
    }, perm, S, lane);
    for (int d = lane; d < 2 * m - 1; d += 64) {
        const int ch = subset_channel(S, d, m, N);
        const float mu = scale * O[K + mc * D + ch];
        const float sg = scale * smax_of(ch, N) * sigm(O[K + K * D + mc * D + ch]);
        const float del = mu + sg * subset_gauss(sh.run_seed, move, c, d);
        sdel[d] = del;
        M.delta[item * D + d] = del;
    }
    const float logN = logf((float)N);
    for (int i = lane; i < m; i += 64) {
        slw[i] = log_w(a, S[i], logN);
        M.subset[item * kMaxSubset + i] = S[i];
    }
    __syncthreads();
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
    float* ap = M.ap + item * 2 * N;
    for (int k = lane; k < 2 * N; k += 64) ap[k] = a[k];
    __syncthreads();
    float dref = 0.0f;
    for (int i = lane; i < m; i += 64) {
        const int k = S[i];
        const float lwn = (i < m - 1 ? slw[i] - slw[m - 1] + sdel[i] : 0.0f) - lse + ltot;
        dref += 0.5f * (lwn - slw[i]);
        const float A = expf(0.25f * (logN + lwn));
        const float ph = atan2f(a[2 * k + 1], a[2 * k]) + sdel[m - 1 + i];
        float sn, cs;
        sincosf(ph, &sn, &cs);
        ap[2 * k] = A * cs;
        ap[2 * k + 1] = A * sn;
    }
    dref = wsum(dref);
    __syncthreads();
    // a move touching a zero amplitude of S (now or in the proposal) is rejected
    const bool out = subset_off_chart(a, S, m, lane) || subset_off_chart(ap, S, m, lane);
    if (out) {
        for (int i = lane; i < m; i += 64) {
            ap[2 * S[i]] = a[2 * S[i]];
            ap[2 * S[i] + 1] = a[2 * S[i] + 1];
        }
        dref = -INFINITY;
    }
    __syncthreads();
    write_features(ap, N, M.X + item * M.In, lane);
    const float lq = log_mix_subset(O, S, sdel, 1.0f, scale, N, K, D, m, lane);
    if (lane == 0) {
        M.lqf[item] = lq;
        M.dref[item] = dref;
    }
}

// field F_l = sum over l's list of J conj(a_x) a_y a_z from amplitudes a in
// LDS; thread t of nt takes every nt-th chunk (chunked lists) or group of 4
// entries (packed lists)
__device__ inline void list_field(const DevPtrs<float>& P, const SampleDev& sd, int layout, int l, const float2* a,
                                  int t, int nt, float& fr, float& fi) {
    if (layout == kLayoutChunked) {
        const uint32_t* cs = P.chunk_start + sd.mode_base;
        const float4* Jv = reinterpret_cast<const float4*>(P.cJ);
        for (uint32_t q = cs[l] + t; q < cs[l + 1]; q += nt) {
            const float2 ax = a[P.cx[q]];
            const uint2 yz = P.cyz[q];
            const float4 j = Jv[q];
            const uint32_t v[4] = {yz.x & 0xffffu, yz.x >> 16, yz.y & 0xffffu, yz.y >> 16};
            const float jj[4] = {j.x, j.y, j.z, j.w};
            float gr = 0.0f, gi = 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float2 ay = a[v[i] & 0xffu], az = a[(v[i] >> 8) & 0xffu];
                gr += jj[i] * (ay.x * az.x - ay.y * az.y);
                gi += jj[i] * (ay.x * az.y + ay.y * az.x);
            }
            fr += ax.x * gr + ax.y * gi;
            fi += ax.x * gi - ax.y * gr;
        }
    } else {
        const uint32_t* ms = P.mode_start + sd.mode_base;
        for (uint32_t q = ms[l] + t; q < ms[l + 1]; q += nt) {
            const uint32_t e = P.idx[q];
            const float2 ax = a[e & 1023u], ay = a[(e >> 10) & 1023u], az = a[e >> 20];
            const float pr = ax.x * ay.x + ax.y * ay.y, pi = ax.x * ay.y - ax.y * ay.x;
            fr += P.J[q] * (pr * az.x - pi * az.y);
            fi += P.J[q] * (pr * az.y + pi * az.x);
        }
    }
}

// subset move, stage two: the energy change, mode by mode on a snapshot that
// already holds the proposal for the modes before: dE = sum_i -2 Re(conj(a'_i - a_i) F_i)
// (exact: every term holds a mode at most once).  One workgroup of up to 1024
// threads per item: the items are few, and each list is streamed by the whole
// workgroup before the next can start.
__global__ __launch_bounds__(1024) void k_energy_subset(MlpDev M, DevPtrs<float> P, ShapeInfo sh) {
    extern __shared__ float2 sa[];  // [N] the snapshot
    __shared__ float red[16][2];
    const int64_t item = blockIdx.x;
    const int N = M.N, m = M.m;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (M.dref[item] == -INFINITY) {  // rejected in stage one
        if (threadIdx.x == 0) M.dE[item] = 0.0f;
        return;
    }
    const int c = M.item_copy[item];
    const SampleDev sd = P.samples[c / sh.copies_per_sample];
    const float* a = copy_amp(P, sh, N, c);
    const float* ap = M.ap + item * 2 * N;
    const int* S = M.subset + item * kMaxSubset;
    for (int k = threadIdx.x; k < N; k += blockDim.x) sa[k] = make_float2(a[2 * k], a[2 * k + 1]);
    __syncthreads();
    float dE = 0.0f;
    for (int i = 0; i < m; ++i) {
        const int l = S[i];
        float fr = 0.0f, fi = 0.0f;
        list_field(P, sd, sh.layout, l, sa, threadIdx.x, blockDim.x, fr, fi);
        fr = wsum(fr);
        fi = wsum(fi);
        if (lane == 0) {
            red[wave][0] = fr;
            red[wave][1] = fi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            float Fr = 0.0f, Fi = 0.0f;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                Fr += red[w][0];
                Fi += red[w][1];
            }
            const float2 o = sa[l];
            const float nr = ap[2 * l], ni = ap[2 * l + 1];
            dE += -2.0f * ((nr - o.x) * Fr + (ni - o.y) * Fi);
            sa[l] = make_float2(nr, ni);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) M.dE[item] = dE;
}

__global__ __launch_bounds__(64) void k_accept(MlpDev M, DevPtrs<float> P, ShapeInfo sh, float scale) {
    __shared__ float sdel[2 * kMaxModes];
    const int net = blockIdx.y, b = blockIdx.x, lane = threadIdx.x;
    const int N = M.N, K = M.K, D = M.D;
    const int64_t item = (int64_t)net * M.Bm + b;
    const int c = M.item_copy[item];
    const int64_t move = *M.moves_done - 1;
    __shared__ int S[kMaxSubset];
    const int m = M.m;
    const int nd = m > 0 ? 2 * m - 1 : D;
    for (int d = lane; d < nd; d += 64) sdel[d] = M.delta[item * D + d];
    for (int i = lane; i < m; i += 64) S[i] = M.subset[item * kMaxSubset + i];
    __syncthreads();
    float lqr, dE = 0.0f;
    if (m > 0) {
        lqr = log_mix_subset(M.Or + item * M.Out, S, sdel, -1.0f, scale, N, K, D, m, lane);
        dE = M.dE[item];
    } else {
        lqr = log_mix(M.Or + item * M.Out, sdel, -1.0f, scale, N, K, D, lane);
        for (int p = 0; p < kEnergyParts; ++p) dE += M.dEp[item * kEnergyParts + p];  // the parts, added in order
    }
    const float beta = P.beta[M.temp_index[net]];
    const float dref = M.dref[item];
    const float la = dref == -INFINITY ? -INFINITY : -beta * dE + dref + lqr - M.lqf[item];
    // the acceptance uniform: word 1 of the block after the Gaussians (counter word 3: 0 all-mode, 1 subset)
    const int nb = m > 0 ? m : (D + 1) / 2;
    const Philox4 wu = philox4x64((uint64_t)nb, (uint64_t)move, (uint64_t)c, m > 0 ? 1 : 0, sh.run_seed, kTagLearn);
    const double ua = uniform01<double>(wu.v[1]);
    const bool accept = log(ua) < (double)la;
    if (accept) {
        float* a = P.amp + 2 * (int64_t)c * N;
        const float* ap = M.ap + item * 2 * N;
        for (int k = lane; k < 2 * N; k += 64) a[k] = ap[k];
    }
    if (lane == 0) {
        M.la[item] = la;
        M.dE[item] = dE;
        if (accept) {
            P.E[c] += dE;
            atomicAdd(&M.acc[net], 1ull);
        }
        atomicAdd(&M.tries[net], 1ull);
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

hipError_t mlp_features_current(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, hipStream_t st) {
    hipLaunchKernelGGL(k_feat_current, dim3(M.Bm, M.nets), dim3(64), 0, st, M, P, sh);
    return hipGetLastError();
}

hipError_t mlp_features_train(const MlpDev& M, uint64_t seed, int64_t step, int use_first, hipStream_t st) {
    hipLaunchKernelGGL(k_feat_train, dim3(M.Bt, M.nets), dim3(64), 0, st, M, seed, step, use_first);
    return hipGetLastError();
}

hipError_t mlp_forward(const MlpDev& M, int train, int into_reverse, hipStream_t st) {
    const int tiles = (M.Out + 255) / 256;
    if (!train && M.Bm <= kFwdRows && M.H % (16 * kFwdSteps) == 0 && M.In % (16 * kFwdSteps) == 0 &&
        tiles <= kFwdMaxTiles &&
        forward_small_lds(M.H) <= 64 * 1024) {
        hipLaunchKernelGGL(k_forward_small, dim3(tiles, M.nets), dim3(256), forward_small_lds(M.H), st, M, M.X,
                           into_reverse ? M.Or : M.Of);
        return hipGetLastError();
    }
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
    hipLaunchKernelGGL(k_propose, dim3(M.Bm, M.nets), dim3(64), 0, st, M, P, sh, scale);
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
    hipLaunchKernelGGL(k_energy_change, dim3((unsigned)(samples * groups * kEnergyParts)), dim3(256), lds, st, M, P,
                       sh, groups, gsize);
    return hipGetLastError();
}

hipError_t mlp_propose_subset(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float scale,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_propose_subset, dim3(M.Bm, M.nets), dim3(64), 0, st, M, P, sh, scale);
    return hipGetLastError();
}

hipError_t mlp_energy_subset(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, hipStream_t st) {
    // threads per item grow with the list length (N = 256: 1024 threads, ~5 chunks each per list)
    const int block = M.N >= 192 ? 1024 : (M.N >= 96 ? 512 : 256);
    hipLaunchKernelGGL(k_energy_subset, dim3((unsigned)(M.Bm * M.nets)), dim3(block), (size_t)M.N * sizeof(float2), st,
                       M, P, sh);
    return hipGetLastError();
}

hipError_t mlp_accept(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float scale, hipStream_t st) {
    hipLaunchKernelGGL(k_accept, dim3(M.Bm, M.nets), dim3(64), 0, st, M, P, sh, scale);
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
