// Host side of the learned global proposal: workspace layout, parameter
// initialisation, harvesting of training pairs from the running simulation,
// Adam training, and the learned Metropolis-Hastings rounds interleaved with
// the plain sweeps.  The method's paper is silent on learned moves; the
// construction is documented in mlp.hpp and the header.
#include <math.h>
#include <string.h>

#include <cmath>
#include <string>
#include <vector>

#include "context.hpp"
#include "philox.hpp"

namespace rlpt {

namespace {

size_t take(size_t& off, size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
}

}  // namespace

// Assign the learned-proposal regions starting at byte offset `off` of base
// (base may be NULL: sizes only).  Returns the end offset.
size_t mlp_layout(const rlpt_config& cfg, int N, int S, MlpDev* M, unsigned char* base, size_t off) {
    if (cfg.mlp_nets <= 0) return off;
    MlpDev m{};
    m.nets = cfg.mlp_nets;
    m.N = N;
    m.In = 2 * N;
    m.H = cfg.mlp_hidden;
    m.K = cfg.mlp_components;
    m.D = 2 * N - 1;
    m.Out = m.K * (2 * m.D + 1);
    m.Bm = S * cfg.n_reps;
    m.m = cfg.mlp_subset;
    m.Bt = cfg.mlp_batch;
    // term ranges per item group: enough workgroups to fill the chip several times over at N = 256
    // (each streams its range once for the group's items), fewer where the lists are short
    m.eparts = N >= 192 ? kMaxEnergyParts : 32;
    m.cap = cfg.mlp_capacity;
    m.oW1 = 0;
    m.ob1 = m.oW1 + (int64_t)m.In * m.H;
    m.oW2 = m.ob1 + m.H;
    m.ob2 = m.oW2 + (int64_t)m.H * m.H;
    m.oW3 = m.ob2 + m.H;
    m.ob3 = m.oW3 + (int64_t)m.H * m.Out;
    m.NP = m.ob3 + m.Out;
    const size_t n = (size_t)m.nets, P = (size_t)m.NP, Bm = (size_t)m.Bm, Bt = (size_t)m.Bt;
    auto f = [&](size_t count) -> float* { const size_t o = take(off, count * 4); return base ? (float*)(base + o) : nullptr; };
    m.master = f(n * P);
    {
        const size_t o = take(off, n * P * 2);
        m.wbf = base ? (uint16_t*)(base + o) : nullptr;
    }
    m.NPt = ((int64_t)m.In * m.H + (int64_t)m.H * m.H + (int64_t)m.H * ((m.Out + 63) / 64 * 64) + 7) & ~(int64_t)7;
    {
        const size_t o = take(off, n * (size_t)m.NPt * 2);
        m.wbt = base ? (uint16_t*)(base + o) : nullptr;
    }
    m.grad = f(n * P);
    m.am = f(n * P);
    m.av = f(n * P);
    m.X = f(n * Bm * m.In);
    m.P1 = f(n * Bm * m.H);
    m.H1 = f(n * Bm * m.H);
    m.P2 = f(n * Bm * m.H);
    m.H2 = f(n * Bm * m.H);
    m.Of = f(n * Bm * m.Out);
    m.Or = f(n * Bm * m.Out);
    m.ap = f(n * Bm * 2 * N);
    m.delta = f(n * Bm * m.D);
    m.lqf = f(n * Bm);
    m.dref = f(n * Bm);
    m.dE = f(n * Bm);
    m.dEp = f(n * Bm * kMaxEnergyParts);
    m.la = f(n * Bm);
    m.lua = (double*)f(2 * n * Bm);
    m.item_copy = (int32_t*)f(n * Bm);
    m.subset = (int32_t*)f(n * Bm * kMaxSubset);
    m.tX = f(n * Bt * m.In);
    m.tP1 = f(n * Bt * m.H);
    m.tH1 = f(n * Bt * m.H);
    m.tP2 = f(n * Bt * m.H);
    m.tH2 = f(n * Bt * m.H);
    m.tO = f(n * Bt * m.Out);
    m.tdO = f(n * Bt * m.Out);
    m.tdA = f(n * Bt * m.H);
    m.tdB = f(n * Bt * m.H);
    m.tdelta = f(n * Bt * m.D);
    m.tloss = f(n * Bt);
    m.tvalid = (int32_t*)f(n * Bt);
    m.tsub = (int32_t*)f(n * Bt * kMaxSubset);
    m.data = f(n * (size_t)m.cap * 2 * 2 * N);
    m.temp_index = (int32_t*)f(n);
    m.count = (int32_t*)f(n);
    m.acc = (unsigned long long*)f(2 * n);
    m.tries = (unsigned long long*)f(2 * n);
    m.moves_done = (int64_t*)f(2);
    if (M) *M = m;
    return off;
}

int mlp_check_config(const rlpt_config& cfg, const rlpt_graph* const* g, int S) {
    if (cfg.mlp_nets <= 0) return RLPT_OK;
    if (cfg.mlp_nets > cfg.n_temps) return fail(RLPT_E_ARG, "mlp_nets must be <= n_temps");
    if (cfg.mlp_hidden < 1 || cfg.mlp_hidden > 4096) return fail(RLPT_E_ARG, "mlp_hidden must be in [1, 4096]");
    if (cfg.mlp_components < 1 || cfg.mlp_components > 8) return fail(RLPT_E_ARG, "mlp_components must be in [1, 8]");
    if (cfg.mlp_capacity < 1 || cfg.mlp_batch < 1) return fail(RLPT_E_ARG, "mlp_capacity and mlp_batch must be >= 1");
    if (cfg.mlp_capacity < cfg.mlp_batch) return fail(RLPT_E_ARG, "mlp_capacity must be >= mlp_batch");
    for (int i = 1; i < S; ++i)
        if (g[i]->N != g[0]->N) return fail(RLPT_E_ARG, "learned moves need one N for every sample");
    if (g[0]->N > kMaxModes / 2) return fail(RLPT_E_ARG, "learned moves support N <= 512");
    if (cfg.mlp_subset != 0 && (cfg.mlp_subset < 2 || cfg.mlp_subset > kMaxSubset || cfg.mlp_subset > g[0]->N))
        return fail(RLPT_E_ARG, "mlp_subset must be 0 or in [2, min(N, 64)]");
    return RLPT_OK;
}

}  // namespace rlpt

using namespace rlpt;

namespace {

int mlp_ready(rlpt_ctx* c) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    if (c->cfg.mlp_nets <= 0) return fail(RLPT_E_ARG, "context was created with mlp_nets = 0");
    if (c->cfg.precision != RLPT_FP32) return fail(RLPT_E_UNSUPPORTED, "learned moves run in FP32 contexts");
    if (!c->mlp_setup) return fail(RLPT_E_STATE, "rlpt_mlp_setup has not been called");
    return RLPT_OK;
}

#define HIP_TRY2(expr, what)                                                             \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(RLPT_E_HIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

// per network, the mean loss of the last training minibatch over its pairs
// inside the chart and the number of such pairs (synchronous)
int minibatch_loss(rlpt_ctx* c, std::vector<double>* loss, std::vector<int>* used) {
    const MlpDev& M = c->mlp;
    std::vector<float> L((size_t)M.nets * M.Bt);
    std::vector<int32_t> V((size_t)M.nets * M.Bt);
    HIP_TRY2(hipMemcpy(L.data(), M.tloss, L.size() * 4, hipMemcpyDeviceToHost), "read loss");
    HIP_TRY2(hipMemcpy(V.data(), M.tvalid, V.size() * 4, hipMemcpyDeviceToHost), "read pair flags");
    loss->assign(M.nets, 0.0);
    used->assign(M.nets, 0);
    for (int n = 0; n < M.nets; ++n) {
        double t = 0;
        int u = 0;
        for (int b = 0; b < M.Bt; ++b)
            if (V[(size_t)n * M.Bt + b]) {
                t += L[(size_t)n * M.Bt + b];
                ++u;
            }
        (*loss)[n] = u ? t / u : NAN;
        (*used)[n] = u;
    }
    return RLPT_OK;
}

}  // namespace

// one learned-move round of every network (enqueued; used by the sweep schedule)
int mlp_enqueue_round(rlpt_ctx* c) {
    const MlpDev& M = c->mlp;
    const float s = (float)c->mlp_scale;
    HIP_TRY2(mlp_forward_current(M, c->pf, c->sh, c->stream), "learned forward");
    if (M.m > 0) {
        HIP_TRY2(mlp_propose_subset(M, c->pf, c->sh, s, c->stream), "learned propose");
    } else {
        HIP_TRY2(mlp_propose(M, c->pf, c->sh, s, c->stream), "learned propose");
        HIP_TRY2(mlp_energy_change(M, c->pf, c->sh, c->stream), "learned energy");
    }
    HIP_TRY2(mlp_forward_proposal(M, c->pf, c->sh, M.Or, c->stream), "learned forward");
    HIP_TRY2(mlp_accept(M, c->pf, c->sh, s, c->stream), "learned accept");
    if (c->sh.cached) HIP_TRY2(launch_fields_all(c->cfg.precision, c->ptrs(), c->sh, c->n_copies, c->stream), "fields");
    return RLPT_OK;
}

extern "C" {

int rlpt_mlp_setup(rlpt_ctx* c, const int32_t* temp_index, uint64_t seed) {
    if (!c || !temp_index) return fail(RLPT_E_ARG, "NULL argument");
    if (c->cfg.mlp_nets <= 0) return fail(RLPT_E_ARG, "context was created with mlp_nets = 0");
    if (c->cfg.precision != RLPT_FP32) return fail(RLPT_E_UNSUPPORTED, "learned moves run in FP32 contexts");
    MlpDev& M = c->mlp;
    for (int n = 0; n < M.nets; ++n)
        if (temp_index[n] < 0 || temp_index[n] >= c->T) return fail(RLPT_E_ARG, "temperature index out of range");
    // weights: N(0, 1/fan_in) for the hidden layers, 0.01/sqrt(fan_in) for the output layer, zero biases
    std::vector<float> p((size_t)M.nets * M.NP, 0.0f);
    auto fill = [&](int net, int64_t off, int64_t count, double sd) {
        for (int64_t i = 0; i < count; i += 2) {
            const Philox4 w = philox4x64((uint64_t)i, (uint64_t)off, (uint64_t)net, 0, seed, 0x4D4C50ULL);
            const double u1 = 1.0 - uniform01<double>(w.v[0]), u2 = uniform01<double>(w.v[1]);
            const double r = sqrt(-2.0 * log(u1));
            p[(size_t)net * M.NP + off + i] = (float)(sd * r * cos(2.0 * 3.14159265358979323846 * u2));
            if (i + 1 < count) p[(size_t)net * M.NP + off + i + 1] = (float)(sd * r * sin(2.0 * 3.14159265358979323846 * u2));
        }
    };
    for (int n = 0; n < M.nets; ++n) {
        fill(n, M.oW1, (int64_t)M.In * M.H, 1.0 / sqrt((double)M.In));
        fill(n, M.oW2, (int64_t)M.H * M.H, 1.0 / sqrt((double)M.H));
        fill(n, M.oW3, (int64_t)M.H * M.Out, 0.01 / sqrt((double)M.H));
    }
    const size_t bytes = p.size() * 4;
    HIP_TRY2(hipMemcpyAsync(M.master, p.data(), bytes, hipMemcpyHostToDevice, c->stream), "upload weights");
    HIP_TRY2(launch_zero(M.am, bytes, c->stream), "zero moments");
    HIP_TRY2(launch_zero(M.av, bytes, c->stream), "zero moments");
    HIP_TRY2(hipMemcpyAsync(M.temp_index, temp_index, (size_t)M.nets * 4, hipMemcpyHostToDevice, c->stream),
             "upload temperatures");
    HIP_TRY2(launch_zero(M.count, (size_t)M.nets * 4, c->stream), "zero counts");
    HIP_TRY2(launch_zero(M.acc, (size_t)M.nets * 8, c->stream), "zero counts");
    HIP_TRY2(launch_zero(M.tries, (size_t)M.nets * 8, c->stream), "zero counts");
    HIP_TRY2(launch_zero(M.moves_done, 8, c->stream), "zero counts");
    HIP_TRY2(launch_zero(M.wbt, (size_t)M.nets * M.NPt * 2, c->stream), "zero fragment copy");  // padded columns
    HIP_TRY2(mlp_sync_bf16(M, c->stream), "bf16 copies");
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    c->mlp_temp.assign(temp_index, temp_index + M.nets);
    c->mlp_count.assign(M.nets, 0);
    c->mlp_slot = 0;
    c->mlp_adam_t = 0;
    c->mlp_seed = seed;
    c->mlp_setup = true;
    return RLPT_OK;
}

int rlpt_mlp_n_params(rlpt_ctx* c, int64_t* n_params, int32_t* n_outputs) {
    if (!c) return fail(RLPT_E_ARG, "ctx is NULL");
    if (c->cfg.mlp_nets <= 0) return fail(RLPT_E_ARG, "context was created with mlp_nets = 0");
    if (n_params) *n_params = c->mlp.NP;
    if (n_outputs) *n_outputs = c->mlp.Out;
    return RLPT_OK;
}

int rlpt_mlp_set_params(rlpt_ctx* c, int32_t net, const float* params) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    if (net < 0 || net >= c->mlp.nets || !params) return fail(RLPT_E_ARG, "bad net or NULL params");
    const MlpDev& M = c->mlp;
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY2(hipMemcpy(M.master + (size_t)net * M.NP, params, (size_t)M.NP * 4, hipMemcpyHostToDevice), "upload");
    HIP_TRY2(mlp_sync_bf16(M, c->stream), "bf16 copies");
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    return RLPT_OK;
}

int rlpt_mlp_get_params(rlpt_ctx* c, int32_t net, float* params) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    if (net < 0 || net >= c->mlp.nets || !params) return fail(RLPT_E_ARG, "bad net or NULL params");
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY2(hipMemcpy(params, c->mlp.master + (size_t)net * c->mlp.NP, (size_t)c->mlp.NP * 4, hipMemcpyDeviceToHost),
             "read params");
    return RLPT_OK;
}

// store explicit training pairs (host, interleaved complex doubles) for one
// network in slots [0, n); used by tests and by callers with their own data
int rlpt_mlp_set_pairs(rlpt_ctx* c, int32_t net, int32_t n, const double* before, const double* after) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    const MlpDev& M = c->mlp;
    if (net < 0 || net >= M.nets || n < 1 || n > M.cap || !before || !after) return fail(RLPT_E_ARG, "bad pairs");
    std::vector<float> buf((size_t)n * 2 * 2 * M.N);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 2 * M.N; ++k) {
            buf[((size_t)i * 2 + 0) * 2 * M.N + k] = (float)before[(size_t)i * 2 * M.N + k];
            buf[((size_t)i * 2 + 1) * 2 * M.N + k] = (float)after[(size_t)i * 2 * M.N + k];
        }
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY2(hipMemcpy(M.data + (size_t)net * M.cap * 2 * 2 * M.N, buf.data(), buf.size() * 4, hipMemcpyHostToDevice),
             "upload pairs");
    c->mlp_count[net] = n;
    int32_t cnt = n;
    HIP_TRY2(hipMemcpy(M.count + net, &cnt, 4, hipMemcpyHostToDevice), "upload count");
    return RLPT_OK;
}

// harvest: `rounds` times, record the configurations at each network's
// temperature, run `lag` sweeps without swaps, record the same copies again
int rlpt_mlp_harvest(rlpt_ctx* c, int32_t rounds, int32_t lag) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    if (rounds < 0 || lag < 1) return fail(RLPT_E_ARG, "rounds must be >= 0 and lag >= 1");
    MlpDev& M = c->mlp;
    const int saved = c->cfg.swap_interval;
    const bool saved_on = c->mlp_moves > 0;
    const int saved_moves = c->mlp_moves;
    c->cfg.swap_interval = 1 << 30;  // no exchanges while a pair is recorded
    c->mlp_moves = 0;
    for (int r = 0; r < rounds && rc == RLPT_OK; ++r) {
        HIP_TRY2(mlp_harvest(M, c->pf, c->sh, 0, c->mlp_slot, c->stream), "harvest");
        rc = rlpt_sweep(c, lag);
        if (rc) break;
        HIP_TRY2(mlp_harvest(M, c->pf, c->sh, 1, c->mlp_slot, c->stream), "harvest");
        c->mlp_slot = (c->mlp_slot + M.Bm) % M.cap;
        for (int n = 0; n < M.nets; ++n) c->mlp_count[n] = std::min<int64_t>(c->mlp_count[n] + M.Bm, M.cap);
    }
    c->cfg.swap_interval = saved;
    c->mlp_moves = saved_on ? saved_moves : 0;
    if (rc) return rc;
    std::vector<int32_t> cnt(c->mlp_count.begin(), c->mlp_count.end());
    HIP_TRY2(hipMemcpyAsync(M.count, cnt.data(), cnt.size() * 4, hipMemcpyHostToDevice, c->stream), "upload counts");
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    return RLPT_OK;
}

int rlpt_mlp_train(rlpt_ctx* c, int32_t steps, double lr, double* mean_loss) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    MlpDev& M = c->mlp;
    for (int n = 0; n < M.nets; ++n)
        if (c->mlp_count[n] < 1) return fail(RLPT_E_STATE, "no training pairs: call rlpt_mlp_harvest first");
    if (steps < 0) return fail(RLPT_E_ARG, "steps must be >= 0");
    for (int s = 0; s < steps; ++s) {
        HIP_TRY2(mlp_features_train(M, c->mlp_seed, c->mlp_adam_t, 0, c->stream), "train features");
        HIP_TRY2(mlp_forward(M, 1, 0, c->stream), "train forward");
        HIP_TRY2(mlp_backward(M, c->stream), "train backward");
        c->mlp_adam_t += 1;
        HIP_TRY2(mlp_adam(M, (float)lr, c->mlp_adam_t, c->stream), "adam");
    }
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    if (steps == 0) {
        if (mean_loss)
            for (int n = 0; n < M.nets; ++n) mean_loss[n] = 0.0;
        return RLPT_OK;
    }
    // the last step's loss: mean over the minibatch's pairs inside the chart
    std::vector<double> loss;
    std::vector<int> used;
    rc = minibatch_loss(c, &loss, &used);
    if (rc) return rc;
    if (mean_loss)
        for (int n = 0; n < M.nets; ++n) mean_loss[n] = loss[n];
    for (int n = 0; n < M.nets; ++n) {
        if (used[n] == 0)
            return fail(RLPT_E_STATE, "network " + std::to_string(n) +
                                          ": no training pair of the last minibatch lies inside the chart");
        if (!std::isfinite(loss[n]))
            return fail(RLPT_E_STATE, "network " + std::to_string(n) + ": non-finite training loss");
    }
    return RLPT_OK;
}

// forward of every network on the first n stored pairs' "before" configurations
// (test hook): out = outputs of network `net` [n][Out]
int rlpt_mlp_forward(rlpt_ctx* c, int32_t net, int32_t n, double* out) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    const MlpDev& M = c->mlp;
    if (net < 0 || net >= M.nets || n < 1 || n > M.Bt || n > c->mlp_count[net] || !out)
        return fail(RLPT_E_ARG, "bad forward request");
    HIP_TRY2(mlp_features_train(M, c->mlp_seed, 0, 1, c->stream), "features");
    HIP_TRY2(mlp_forward(M, 1, 0, c->stream), "forward");
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    std::vector<float> o((size_t)n * M.Out);
    HIP_TRY2(hipMemcpy(o.data(), M.tO + (size_t)net * M.Bt * M.Out, o.size() * 4, hipMemcpyDeviceToHost), "read");
    for (size_t i = 0; i < o.size(); ++i) out[i] = o[i];
    return RLPT_OK;
}

// loss and gradient of network `net` on the first Bt stored pairs (test hook;
// no parameter update)
int rlpt_mlp_loss_grad(rlpt_ctx* c, int32_t net, double* loss, float* grad) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    const MlpDev& M = c->mlp;
    if (net < 0 || net >= M.nets || c->mlp_count[net] < M.Bt) return fail(RLPT_E_ARG, "need mlp_batch stored pairs");
    HIP_TRY2(mlp_features_train(M, c->mlp_seed, 0, 1, c->stream), "features");
    HIP_TRY2(mlp_forward(M, 1, 0, c->stream), "forward");
    HIP_TRY2(mlp_backward(M, c->stream), "backward");
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    if (grad)
        HIP_TRY2(hipMemcpy(grad, M.grad + (size_t)net * M.NP, (size_t)M.NP * 4, hipMemcpyDeviceToHost), "read grad");
    std::vector<double> L;
    std::vector<int> used;
    rc = minibatch_loss(c, &L, &used);
    if (rc) return rc;
    if (loss) *loss = L[net];
    if (used[net] == 0) return fail(RLPT_E_STATE, "no stored pair of the minibatch lies inside the chart");
    return RLPT_OK;
}

// inference forward of network `net` (the path learned rounds take) on n <= S*reps
// configurations given by the caller (test hook): out = outputs [n][Out]
int rlpt_mlp_infer(rlpt_ctx* c, int32_t net, int32_t n, const double* states, double* out) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    const MlpDev& M = c->mlp;
    if (net < 0 || net >= M.nets || n < 1 || n > M.Bm || !states || !out) return fail(RLPT_E_ARG, "bad inference request");
    std::vector<float> buf((size_t)n * 2 * M.N);
    for (size_t i = 0; i < buf.size(); ++i) buf[i] = (float)states[i];
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY2(hipMemcpy(M.ap + (size_t)net * M.Bm * 2 * M.N, buf.data(), buf.size() * 4, hipMemcpyHostToDevice),
             "upload states");
    if (!mlp_fused_forward(M)) HIP_TRY2(mlp_features_from_proposals(M, net, n, c->stream), "features");
    HIP_TRY2(mlp_forward_proposal(M, c->pf, c->sh, M.Of, c->stream), "forward");
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    std::vector<float> o((size_t)n * M.Out);
    HIP_TRY2(hipMemcpy(o.data(), M.Of + (size_t)net * M.Bm * M.Out, o.size() * 4, hipMemcpyDeviceToHost), "read");
    for (size_t i = 0; i < o.size(); ++i) out[i] = o[i];
    return RLPT_OK;
}

int rlpt_mlp_enable(rlpt_ctx* c, int32_t moves_per_sweep, double step_scale) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    if (moves_per_sweep < 0 || !(step_scale > 0.0) || step_scale > 1.0)
        return fail(RLPT_E_ARG, "moves_per_sweep >= 0 and 0 < step_scale <= 1");
    c->mlp_moves = moves_per_sweep;
    c->mlp_scale = step_scale;
    return RLPT_OK;
}

int rlpt_mlp_move(rlpt_ctx* c, double step_scale) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    if (!(step_scale > 0.0) || step_scale > 1.0) return fail(RLPT_E_ARG, "0 < step_scale <= 1");
    const double saved = c->mlp_scale;
    c->mlp_scale = step_scale;
    rc = mlp_enqueue_round(c);
    c->mlp_scale = saved;
    return rc;
}

int rlpt_mlp_stats(rlpt_ctx* c, double* acc, double* tries) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    const MlpDev& M = c->mlp;
    std::vector<unsigned long long> a(M.nets), t(M.nets);
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_TRY2(hipMemcpy(a.data(), M.acc, a.size() * 8, hipMemcpyDeviceToHost), "read");
    HIP_TRY2(hipMemcpy(t.data(), M.tries, t.size() * 8, hipMemcpyDeviceToHost), "read");
    for (int n = 0; n < M.nets; ++n) {
        if (acc) acc[n] = (double)a[n];
        if (tries) tries[n] = (double)t[n];
    }
    return RLPT_OK;
}

// diagnostics of the last learned round of network `net` (test hook): log
// acceptance ratio, copy and proposed configuration of each item
int rlpt_mlp_last_move(rlpt_ctx* c, int32_t net, double* log_alpha, int32_t* copies, double* proposal) {
    int rc = mlp_ready(c);
    if (rc) return rc;
    const MlpDev& M = c->mlp;
    if (net < 0 || net >= M.nets) return fail(RLPT_E_ARG, "bad net");
    HIP_TRY2(hipStreamSynchronize(c->stream), "stream synchronize");
    std::vector<float> la(M.Bm), ap((size_t)M.Bm * 2 * M.N);
    HIP_TRY2(hipMemcpy(la.data(), M.la + (size_t)net * M.Bm, la.size() * 4, hipMemcpyDeviceToHost), "read");
    HIP_TRY2(hipMemcpy(ap.data(), M.ap + (size_t)net * M.Bm * 2 * M.N, ap.size() * 4, hipMemcpyDeviceToHost), "read");
    if (copies)
        HIP_TRY2(hipMemcpy(copies, M.item_copy + (size_t)net * M.Bm, (size_t)M.Bm * 4, hipMemcpyDeviceToHost), "read");
    for (int b = 0; b < M.Bm; ++b) {
        if (log_alpha) log_alpha[b] = la[b];
    }
    if (proposal)
        for (size_t i = 0; i < ap.size(); ++i) proposal[i] = ap[i];
    return RLPT_OK;
}

}  // extern "C"
