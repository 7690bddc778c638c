// Runtime prediction (the cost estimator's runtime part: the subsection on
// runtime prediction, Eq. (13)-(21)).  Host code only.
//
//  * Iteration number: a linear regressor from a workload's meta-features
//    to the iteration count v, used through the dummy array u (1 for the
//    first v iterations, 0 after; Eq. (13)).
//  * Per-iteration runtime: a polynomial regressor with interaction terms
//    (Eq. (14)): the feature row of iteration j is every product of at most
//    `order` distinct base features, plus an intercept, where the base
//    features are the workload's meta-features and 1 / j (the iteration's
//    position: pruning improves as the centroids settle).  A task's runtime
//    is sum_j u_j yhat_j (Eq. (15)-(16)); the coefficients solve the least
//    squares problem of Eq. (17) with a small ridge term.  Its rows there are
//    a run's u-weighted sums of iteration rows against the run's total time;
//    the measured time of every iteration is known here, so every iteration
//    of every training run is a row of its own (the same model, better
//    conditioned: the 1 / j terms are no longer summed into one number).
//  * Adjustment: g(i) = yhat_i / y_i, the ratio of predicted to measured
//    time of a finished iteration, has prior mean 1 and the asymmetric
//    kernel of Eq. (20)-(21): cov(i, i') = 0 for i' - i <= -1, else
//    exp(-h(i' - i)^2 / (2 sigma^2)) with h(x) = ln(x + 1) on (-1, 0] and x
//    above, so a finished iteration informs only itself and later ones.  The
//    posterior mean of g over the remaining iterations rescales their
//    predicted times (y = yhat / g).
#include <math.h>

#include <string>
#include <vector>

#include "ekm_internal.hpp"

struct km_predictor {
    int q = 0;          // largest iteration number
    int nf = 0;         // meta-features per workload
    int order = 2;      // largest interaction order
    double sigma = 2.0; // kernel width (iterations)
    double noise = 1e-2;
    double ridge = 1e-9;
    std::vector<std::vector<int>> terms; // base-feature subsets of the polynomial (empty: intercept)
    std::vector<std::vector<double>> run_feat, run_ms;
    std::vector<double> w_iter; // iteration-number regressor: [1, features]
    std::vector<double> b_time; // per-iteration regressor over `terms`
    bool fitted = false;
    // the task being monitored
    std::vector<double> yhat; // predicted ms of iterations 1..q
    int v = 0;                // predicted iteration number
    std::vector<int> obs_i;
    std::vector<double> obs_g;
};

namespace ekm {

// Subsets of {0..m-1} of size <= order, in order of size (then lexicographic).
static void make_terms(int m, int order, std::vector<std::vector<int>> &out)
{
    out.clear();
    out.push_back({});
    std::vector<std::vector<int>> level = {{}};
    for (int sz = 1; sz <= order && sz <= m; ++sz) {
        std::vector<std::vector<int>> next;
        for (const auto &t : level) {
            const int from = t.empty() ? 0 : t.back() + 1;
            for (int i = from; i < m; ++i) {
                auto u = t;
                u.push_back(i);
                next.push_back(u);
            }
        }
        for (const auto &t : next)
            out.push_back(t);
        level.swap(next);
    }
}

// Feature row of iteration j (1-based) of a workload with features f.
static void iter_row(const km_predictor *p, const double *f, int j, std::vector<double> &row)
{
    row.assign(p->terms.size(), 1.0);
    for (size_t t = 0; t < p->terms.size(); ++t)
        for (int i : p->terms[t])
            row[t] *= i < p->nf ? f[i] : 1.0 / (double)j;
}

// Solves (A + ridge I) x = y in place (A: n x n, row major) by Gaussian
// elimination with partial pivoting; false if singular.
static bool solve(std::vector<double> A, std::vector<double> y, int n, double ridge, std::vector<double> &x)
{
    for (int i = 0; i < n; ++i)
        A[(size_t)i * n + i] += ridge;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[(size_t)r * n + c]) > fabs(A[(size_t)piv * n + c]))
                piv = r;
        if (fabs(A[(size_t)piv * n + c]) < 1e-300)
            return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k)
                std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]);
            std::swap(y[c], y[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double m = A[(size_t)r * n + c] / A[(size_t)c * n + c];
            if (m == 0.0)
                continue;
            for (int k = c; k < n; ++k)
                A[(size_t)r * n + k] -= m * A[(size_t)c * n + k];
            y[r] -= m * y[c];
        }
    }
    x.assign(n, 0.0);
    for (int r = n - 1; r >= 0; --r) {
        double s = y[r];
        for (int k = r + 1; k < n; ++k)
            s -= A[(size_t)r * n + k] * x[k];
        x[r] = s / A[(size_t)r * n + r];
    }
    return true;
}

// Least squares: rows X (m x p), targets y -> coefficients (ridge-regularised
// normal equations, the ridge scaled by the mean diagonal).
static bool least_squares(const std::vector<std::vector<double>> &X, const std::vector<double> &y, double ridge,
                          std::vector<double> &b)
{
    const int p = (int)X[0].size();
    std::vector<double> A((size_t)p * p, 0.0), r(p, 0.0);
    for (size_t m = 0; m < X.size(); ++m)
        for (int i = 0; i < p; ++i) {
            r[i] += X[m][i] * y[m];
            for (int k = 0; k < p; ++k)
                A[(size_t)i * p + k] += X[m][i] * X[m][k];
        }
    double tr = 0.0;
    for (int i = 0; i < p; ++i)
        tr += A[(size_t)i * p + i];
    return solve(A, r, p, ridge * (tr > 0.0 ? tr / p : 1.0), b);
}

double asym_kernel(double i, double ip, double sigma)
{
    const double x = ip - i;
    if (x <= -1.0)
        return 0.0;
    const double h = x <= 0.0 ? log(x + 1.0) : x;
    return exp(-h * h / (2.0 * sigma * sigma));
}

} // namespace ekm

using namespace ekm;

extern "C" {

km_status kmeans_predictor_create(km_predictor **out, int32_t q, int32_t nfeat, int32_t order, double sigma,
                                  double noise)
{
    if (!out || q < 1 || nfeat < 0 || nfeat > 16 || order < 1 || !(sigma > 0.0) || !(noise >= 0.0)) {
        set_error("kmeans_predictor_create: need q >= 1, 0 <= nfeat <= 16, order >= 1, sigma > 0, noise >= 0");
        return KM_ERR_INVALID;
    }
    km_predictor *p = new km_predictor();
    p->q = q;
    p->nf = nfeat;
    p->order = order;
    p->sigma = sigma;
    p->noise = noise;
    make_terms(nfeat + 1, order, p->terms); // base features: the meta-features, then 1 / j
    *out = p;
    return KM_OK;
}

km_status kmeans_predictor_destroy(km_predictor *p)
{
    delete p;
    return KM_OK;
}

km_status kmeans_predictor_add_run(km_predictor *p, const double *feat, const double *iter_ms, int32_t iters)
{
    if (!p || (p->nf && !feat) || !iter_ms || iters < 1 || iters > p->q) {
        set_error("kmeans_predictor_add_run: need features, 1 <= iters <= q measured iteration times");
        return KM_ERR_INVALID;
    }
    p->run_feat.emplace_back(feat, feat + p->nf);
    p->run_ms.emplace_back(iter_ms, iter_ms + iters);
    p->fitted = false;
    return KM_OK;
}

km_status kmeans_predictor_fit(km_predictor *p)
{
    if (!p || p->run_feat.empty()) {
        set_error("kmeans_predictor_fit: no training runs");
        return KM_ERR_INVALID;
    }
    const size_t R = p->run_feat.size();
    // iteration number: v = [1, f] . w
    std::vector<std::vector<double>> X(R);
    std::vector<double> y(R);
    for (size_t r = 0; r < R; ++r) {
        X[r].assign(1, 1.0);
        X[r].insert(X[r].end(), p->run_feat[r].begin(), p->run_feat[r].end());
        y[r] = (double)p->run_ms[r].size();
    }
    if (!least_squares(X, y, p->ridge, p->w_iter)) {
        set_error("kmeans_predictor_fit: singular iteration-number system");
        return KM_ERR_INVALID;
    }
    // per-iteration time: one row per measured iteration
    X.clear();
    y.clear();
    std::vector<double> row;
    for (size_t r = 0; r < R; ++r)
        for (size_t j = 0; j < p->run_ms[r].size(); ++j) {
            iter_row(p, p->run_feat[r].data(), (int)j + 1, row);
            X.push_back(row);
            y.push_back(p->run_ms[r][j]);
        }
    if (!least_squares(X, y, p->ridge, p->b_time)) {
        set_error("kmeans_predictor_fit: singular runtime system");
        return KM_ERR_INVALID;
    }
    p->fitted = true;
    return KM_OK;
}

// Predicted iteration number and per-iteration times of a workload.
static void predict(const km_predictor *p, const double *feat, int &v, std::vector<double> &yhat)
{
    double vv = p->w_iter[0];
    for (int i = 0; i < p->nf; ++i)
        vv += p->w_iter[i + 1] * feat[i];
    v = (int)lround(vv);
    v = v < 1 ? 1 : (v > p->q ? p->q : v);
    yhat.assign(p->q, 0.0);
    std::vector<double> row;
    for (int j = 1; j <= p->q; ++j) {
        iter_row(p, feat, j, row);
        double s = 0.0;
        for (size_t t = 0; t < row.size(); ++t)
            s += row[t] * p->b_time[t];
        yhat[j - 1] = s > 0.0 ? s : 0.0;
    }
}

km_status kmeans_predictor_predict(const km_predictor *p, const double *feat, int32_t *iters_out, double *iter_ms,
                                   double *total_ms)
{
    if (!p || !p->fitted || (p->nf && !feat)) {
        set_error("kmeans_predictor_predict: predictor not fitted, or null features");
        return KM_ERR_INVALID;
    }
    int v;
    std::vector<double> yhat;
    predict(p, feat, v, yhat);
    double t = 0.0;
    for (int j = 0; j < v; ++j)
        t += yhat[j];
    if (iters_out)
        *iters_out = v;
    if (iter_ms)
        for (int j = 0; j < p->q; ++j)
            iter_ms[j] = yhat[j];
    if (total_ms)
        *total_ms = t;
    return KM_OK;
}

km_status kmeans_predictor_begin(km_predictor *p, const double *feat)
{
    if (!p || !p->fitted || (p->nf && !feat)) {
        set_error("kmeans_predictor_begin: predictor not fitted, or null features");
        return KM_ERR_INVALID;
    }
    predict(p, feat, p->v, p->yhat);
    p->obs_i.clear();
    p->obs_g.clear();
    return KM_OK;
}

km_status kmeans_predictor_observe(km_predictor *p, int32_t iter, double ms, double *remaining_ms, double *total_ms)
{
    if (!p || p->yhat.empty() || iter < 1 || iter > p->q || !(ms > 0.0) ||
        (!p->obs_i.empty() && iter <= p->obs_i.back())) {
        set_error("kmeans_predictor_observe: call begin first; iterations in increasing order, ms > 0");
        return KM_ERR_INVALID;
    }
    p->obs_i.push_back(iter);
    p->obs_g.push_back(p->yhat[iter - 1] > 0.0 ? p->yhat[iter - 1] / ms : 1.0);
    // posterior mean of g: mu(j) = 1 + sum_m alpha_m cov(i_m, j), (K + noise I) alpha = g - 1
    const int m = (int)p->obs_i.size();
    std::vector<double> K((size_t)m * m), r(m), alpha;
    for (int a = 0; a < m; ++a) {
        r[a] = p->obs_g[a] - 1.0;
        for (int b = 0; b < m; ++b)
            K[(size_t)a * m + b] = asym_kernel(p->obs_i[a], p->obs_i[b], p->sigma);
    }
    if (!solve(K, r, m, p->noise, alpha)) {
        set_error("kmeans_predictor_observe: singular kernel system");
        return KM_ERR_INVALID;
    }
    double rem = 0.0;
    const int last = iter > p->v ? iter : p->v; // the task has run at least this far
    for (int j = iter + 1; j <= last && j <= p->q; ++j) {
        double g = 1.0;
        for (int a = 0; a < m; ++a)
            g += alpha[a] * asym_kernel(p->obs_i[a], j, p->sigma);
        rem += g > 1e-3 ? p->yhat[j - 1] / g : p->yhat[j - 1] * 1e3;
    }
    if (remaining_ms)
        *remaining_ms = rem;
    if (total_ms) {
        double t = rem;
        for (int a = 0; a < m; ++a)
            t += p->yhat[p->obs_i[a] - 1] / p->obs_g[a]; // the measured times
        *total_ms = t;
    }
    return KM_OK;
}

// Meta-features of a context (the paper's n, k, d, f plus what building the
// index reveals about the data): ln n, ln k, d, ln f, ln(points per leaf),
// ln(leaves), ln(leaf groups), centroid-tree levels.
km_status kmeans_context_features(const km_ctx *ctx, double *feat, int32_t cap, int32_t *nfeat)
{
    if (!ctx || !nfeat || cap < 0 || (cap > 0 && !feat)) {
        set_error("kmeans_context_features: invalid argument");
        return KM_ERR_INVALID;
    }
    const int64_t L = ctx->L > 0 ? ctx->L : 1, G = ctx->ngroups > 0 ? ctx->ngroups : 1;
    const double v[8] = {log((double)ctx->n), log((double)ctx->k), (double)ctx->d, log((double)ctx->f),
                         log((double)ctx->n / (double)L), log((double)L), log((double)G),
                         (double)ctx->tree.nlev};
    *nfeat = 8;
    for (int i = 0; i < 8 && i < cap; ++i)
        feat[i] = v[i];
    return KM_OK;
}

} // extern "C"
