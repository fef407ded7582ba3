// Host analysis of the accumulated observables (sec. III.B "Averages and
// errors", sec. IV, App. A of Benedetti & Leuzzi, arXiv 2511.13508):
// disorder averages with jackknife errors over samples, the overlap kurtosis,
// the specific-heat-adapted temperature ladder and doubling-window means.
#include <math.h>

#include <functional>
#include <vector>

#include "internal.hpp"

using namespace rlpt;

namespace {

// jackknife over samples of a statistic f(sample set) evaluated on
// leave-one-out sets: value on the full set and the jackknife error
void jackknife(int S, const std::function<double(const std::vector<int>&)>& f, double* value, double* err) {
    std::vector<int> all(S);
    for (int i = 0; i < S; ++i) all[i] = i;
    *value = f(all);
    if (S < 2) {
        *err = 0.0;
        return;
    }
    std::vector<double> loo(S);
    double mean = 0.0;
    for (int out = 0; out < S; ++out) {
        std::vector<int> keep;
        keep.reserve(S - 1);
        for (int i = 0; i < S; ++i)
            if (i != out) keep.push_back(i);
        loo[out] = f(keep);
        mean += loo[out];
    }
    mean /= S;
    double v = 0.0;
    for (double x : loo) v += (x - mean) * (x - mean);
    *err = sqrt((double)(S - 1) / S * v);
}

}  // namespace

extern "C" {

int rlpt_summarize(const rlpt_obs* o, int32_t S, int32_t T, int32_t N, const double* temps, rlpt_summary* out) {
    if (!o || !out || !temps || S < 1 || T < 1 || N < 1) return fail(RLPT_E_ARG, "rlpt_summarize: bad argument");
    if (!o->e_n || !o->e_sum || !o->e_sq) return fail(RLPT_E_ARG, "rlpt_summarize: energy accumulators needed");
    auto at = [&](const double* a, int mu, int t) { return a[(size_t)mu * T + t]; };
    for (int t = 0; t < T; ++t) {
        const double T2 = temps[t] * temps[t];
        auto meanE = [&](const std::vector<int>& s) {
            double v = 0;
            for (int mu : s) v += at(o->e_sum, mu, t) / at(o->e_n, mu, t);
            return v / s.size();
        };
        // specific heat per spin: disorder average of the thermal energy variance / T^2 / N (eq. SpecificHeat)
        auto cv = [&](const std::vector<int>& s) {
            double v = 0;
            for (int mu : s) {
                const double m = at(o->e_sum, mu, t) / at(o->e_n, mu, t);
                v += (at(o->e_sq, mu, t) / at(o->e_n, mu, t) - m * m) / T2;
            }
            return v / s.size() / N;
        };
        double v, e;
        jackknife(S, meanE, &v, &e);
        if (out->E) out->E[t] = v;
        if (out->E_err) out->E_err[t] = e;
        jackknife(S, cv, &v, &e);
        if (out->cv) out->cv[t] = v;
        if (out->cv_err) out->cv_err[t] = e;
        auto ratio = [&](const double* num, const double* den) {
            return [&, num, den](const std::vector<int>& s) {
                double x = 0;
                for (int mu : s) x += at(num, mu, t) / at(den, mu, t);
                return x / s.size();
            };
        };
        if (o->y2_sum) {
            jackknife(S, ratio(o->y2_sum, o->e_n), &v, &e);
            if (out->y2) out->y2[t] = v;
            if (out->y2_err) out->y2_err[t] = e;
        }
        if (o->y4_sum) {
            jackknife(S, ratio(o->y4_sum, o->e_n), &v, &e);
            if (out->y4) out->y4[t] = v;
            if (out->y4_err) out->y4_err[t] = e;
        }
        if (o->q_n && o->q_sq && o->q_sum && o->q_4 && at(o->q_n, 0, t) > 0) {
            jackknife(S, ratio(o->q_sq, o->q_n), &v, &e);
            if (out->q2) out->q2[t] = v;
            if (out->q2_err) out->q2_err[t] = e;
            // kurtosis (eq. kurt) with the disorder-averaged mean overlap taken as 0
            // (q -> -q under a -> -a): avg<q^4> / (avg(<q^2> - <q>^2))^2
            auto kurt = [&](const std::vector<int>& s) {
                double num = 0, den = 0;
                for (int mu : s) {
                    const double n = at(o->q_n, mu, t), m1 = at(o->q_sum, mu, t) / n;
                    num += at(o->q_4, mu, t) / n;
                    den += at(o->q_sq, mu, t) / n - m1 * m1;
                }
                num /= s.size();
                den /= s.size();
                return num / (den * den);
            };
            jackknife(S, kurt, &v, &e);
            if (out->kurtosis) out->kurtosis[t] = v;
            if (out->kurtosis_err) out->kurtosis_err[t] = e;
        }
        if (out->acc_rate && o->acc && o->tries) {
            double a = 0, n = 0;
            for (int mu = 0; mu < S; ++mu) {
                a += at(o->acc, mu, t);
                n += at(o->tries, mu, t);
            }
            out->acc_rate[t] = n > 0 ? a / n : 0.0;
        }
    }
    if (out->swap_rate && o->swap_acc && o->swap_tries && T > 1)
        for (int i = 0; i + 1 < T; ++i) {
            double a = 0, n = 0;
            for (int mu = 0; mu < S; ++mu) {
                a += o->swap_acc[(size_t)mu * (T - 1) + i];
                n += o->swap_tries[(size_t)mu * (T - 1) + i];
            }
            out->swap_rate[i] = n > 0 ? a / n : 0.0;
        }
    return RLPT_OK;
}

int rlpt_adaptive_ladder(const double* T_grid, const double* C_grid, int32_t n_grid, double T_min, double T_max,
                         double C, double* temps, int32_t capacity, int32_t* n_out) {
    if (!T_grid || !C_grid || !temps || !n_out || n_grid < 2 || capacity < 1 || !(C > 0) || !(T_min > 0) ||
        !(T_max > T_min))
        return fail(RLPT_E_ARG, "rlpt_adaptive_ladder: bad argument");
    for (int i = 0; i < n_grid; ++i) {
        if (i > 0 && !(T_grid[i] > T_grid[i - 1])) return fail(RLPT_E_ARG, "T grid must be strictly ascending");
        if (!(C_grid[i] > C * C)) return fail(RLPT_E_ARG, "C_V must exceed C^2 on the grid (ladder step would diverge)");
    }
    // C_V(T) by linear interpolation on the grid, constant beyond its ends
    auto cv = [&](double T) {
        if (T <= T_grid[0]) return C_grid[0];
        if (T >= T_grid[n_grid - 1]) return C_grid[n_grid - 1];
        int lo = 0, hi = n_grid - 1;
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            (T_grid[mid] <= T ? lo : hi) = mid;
        }
        const double f = (T - T_grid[lo]) / (T_grid[hi] - T_grid[lo]);
        return C_grid[lo] + f * (C_grid[hi] - C_grid[lo]);
    };
    int n = 0;
    double T = T_min;
    temps[n++] = T;
    // T_i = T_{i-1} / (1 - C / sqrt(C_V(T_i)))  (eq. PT_Ti), solved by fixed-point iteration, until T_i >= T_max
    while (n < capacity) {
        double x = T / (1.0 - C / sqrt(cv(T)));
        for (int it = 0; it < 200; ++it) {
            const double y = T / (1.0 - C / sqrt(cv(x)));
            if (fabs(y - x) <= 1e-13 * x) {
                x = y;
                break;
            }
            x = y;
        }
        if (!(x < T_max)) break;
        temps[n++] = x;
        T = x;
    }
    *n_out = n;
    return RLPT_OK;
}

int rlpt_window_means(const double* x, int64_t n, double* means, int64_t* starts, int32_t capacity, int32_t* n_windows) {
    if (!x || !means || !n_windows || n < 1 || capacity < 1) return fail(RLPT_E_ARG, "rlpt_window_means: bad argument");
    // windows [0, 1), [1, 2), [2, 4), [4, 8), ... clipped to n (sec. III.B, doubling time windows)
    int w = 0;
    int64_t b = 0, e = 1;
    while (b < n && w < capacity) {
        const int64_t hi = e < n ? e : n;
        double s = 0;
        for (int64_t i = b; i < hi; ++i) s += x[i];
        means[w] = s / (double)(hi - b);
        if (starts) starts[w] = b;
        ++w;
        b = e;
        e = 2 * e;
    }
    *n_windows = w;
    return RLPT_OK;
}

}  // extern "C"
