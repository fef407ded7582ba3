// Learned global proposal: device descriptor and kernel launchers.
//
// One network per learned temperature slot: features of a configuration (Re
// and Im of a rotated so that a_0 is real positive) -> H SiLU -> H SiLU ->
// K-component diagonal Gaussian mixture over the displacement (dy, dpsi) of
// the alr intensity coordinates y_k = log(w_k / w_{N-1}), w = |a|^4 / N, and of
// the phases; exact Metropolis-Hastings with the reference density
// prod w^(1/2) in (y, psi).  Weights: FP32 master + bfloat16 copies used by
// the matrix-core GEMMs (bfloat16 operands, FP32 accumulation).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace rlpt {

constexpr int kMaxEnergyParts = 128;  // most workgroups sharing one learned move's energy change
constexpr int kMaxSubset = 64;    // largest subset of the subset move

struct MlpDev {
    int32_t nets, N, In, H, K, D, Out;
    int32_t Bm;      // inference items per net (samples x replicas)
    int32_t m;       // subset move: modes per move (0: the all-mode move)
    int32_t Bt;      // training minibatch
    int32_t eparts;  // workgroups (term ranges) per item group of the all-mode energy change
    int32_t cap;     // stored training pairs per net
    int64_t NP;      // parameters per net
    int64_t oW1, ob1, oW2, ob2, oW3, ob3;  // offsets inside a parameter vector
    float* master;   // [nets][NP]
    uint16_t* wbf;   // [nets][NP] bfloat16 copies
    uint16_t* wbt;   // [nets][NPt] bfloat16 weights in MFMA fragment order (see frag_at), zero padded
    int64_t NPt;     // per net: In H + H H + H ceil(Out / 64) 64 elements (W1, W2, W3 with padded columns)
    float* grad;     // [nets][NP]
    float* am;       // Adam first moments
    float* av;       // Adam second moments
    // inference (per learned move round)
    float* X;        // [nets][Bm][In]
    float* P1;       // [nets][Bm][H] pre-activations
    float* H1;
    float* P2;
    float* H2;
    float* Of;       // [nets][Bm][Out] at the current configuration
    float* Or;       // [nets][Bm][Out] at the proposal
    float* ap;       // [nets][Bm][2N] proposed configuration (interleaved complex)
    float* delta;    // [nets][Bm][D]
    float* lqf;      // [nets][Bm] forward log density
    float* dref;     // [nets][Bm] log reference-density ratio
    float* dE;       // [nets][Bm] energy change
    float* dEp;      // [nets][Bm][kMaxEnergyParts] partial energy changes (term ranges)
    float* la;       // [nets][Bm] log acceptance ratio
    double* lua;     // [nets][Bm] log of the uniform that decides the move (drawn with the proposal)
    int32_t* item_copy;  // [nets][Bm]
    int32_t* subset;     // [nets][Bm][kMaxSubset] the subset of the last move, ascending (subset move)
    // training
    float* tX;       // [nets][Bt][In]
    float* tP1;      // [nets][Bt][H]
    float* tH1;
    float* tP2;
    float* tH2;
    float* tO;       // [nets][Bt][Out]
    float* tdO;      // [nets][Bt][Out]
    float* tdA;      // [nets][Bt][H] backward scratch
    float* tdB;      // [nets][Bt][H]
    float* tdelta;   // [nets][Bt][D]
    float* tloss;    // [nets][Bt] per-pair loss (0 for pairs left out)
    int32_t* tvalid; // [nets][Bt] 1 when both configurations of the pair are inside the alr chart
    int32_t* tsub;   // [nets][Bt][kMaxSubset] the training item's subset (subset move)
    float* data;     // [nets][cap][2][2N] pairs (before, after), interleaved complex
    int32_t* temp_index;  // [nets]
    int32_t* count;  // [nets] stored pairs
    unsigned long long* acc;    // [nets]
    unsigned long long* tries;  // [nets]
    int64_t* moves_done;        // learned-move rounds started (RNG counter; advanced by the round's first kernel)
};

// all launchers enqueue on st and cover every net in one launch (grid z = net)
hipError_t mlp_features_train(const MlpDev& M, uint64_t seed, int64_t step, int use_first, hipStream_t st);
// forward of every net through the GEMMs: inference (train = 0, from M.X into Of or Or) or training
// (from tX into tO)
hipError_t mlp_forward(const MlpDev& M, int train, int into_reverse, hipStream_t st);
// true when inference forwards take the one-launch kernel (batch <= 16 rows, In and H multiples of 128)
bool mlp_fused_forward(const MlpDev& M);
// inference forward at the copies of every net's temperature slot into Of; also records item_copy and
// starts the round (moves_done += 1)
hipError_t mlp_forward_current(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, hipStream_t st);
// inference forward at the configurations in M.ap into O (Of or Or); the GEMM path reads their features
// from M.X, which the proposal stage writes
hipError_t mlp_forward_proposal(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float* O,
                                hipStream_t st);
hipError_t mlp_backward(const MlpDev& M, hipStream_t st);
hipError_t mlp_adam(const MlpDev& M, float lr, int64_t t, hipStream_t st);
hipError_t mlp_sync_bf16(const MlpDev& M, hipStream_t st);
hipError_t mlp_propose(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float scale, hipStream_t st);
hipError_t mlp_energy_change(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, hipStream_t st);
// subset move: the proposal and its energy change from the subset's lists (one launch)
hipError_t mlp_propose_subset(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float scale,
                              hipStream_t st);
hipError_t mlp_accept(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, float scale, hipStream_t st);
hipError_t mlp_harvest(const MlpDev& M, const DevPtrs<float>& P, const ShapeInfo& sh, int which, int slot0,
                       hipStream_t st);
// features of rows [0, n) of network net from configurations held in M.ap (test hook)
hipError_t mlp_features_from_proposals(const MlpDev& M, int net, int n, hipStream_t st);

}  // namespace rlpt
