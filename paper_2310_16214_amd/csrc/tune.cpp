// Tuners over the launch-parameter space (Sec. IV of arXiv:2310.16214):
// exhaustive search, the analytical occupancy guideline (Sec. IV-A) and
// Bayesian optimisation with a Gaussian-process surrogate and Expected
// Improvement (Sec. IV-B), plus the GPU timing harness they share and the
// tune cache that makes a tuned configuration the default for later calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <random>
#include <sstream>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/ppx_tune.h"
#include "ppx_internal.h"

namespace ppx {

// ============================================================ occupancy
static int64_t roundup(int64_t v, int64_t g) { return g > 0 ? (v + g - 1) / g * g : v; }

static int occupancy_blocks(const ppx_device_model &m, const ppx_resource &r, int *waves) {
    if (waves) *waves = 0;
    if (r.threads <= 0 || m.wave_size <= 0) return 0;
    if (r.lds_bytes > m.lds_per_block) return 0;
    const int64_t wpb = (r.threads + m.wave_size - 1) / m.wave_size;
    if (wpb > m.max_waves_per_cu) return 0;
    int64_t b = std::min<int64_t>(m.max_blocks_per_cu, m.max_waves_per_cu / wpb);
    if (r.regs_per_thread > 0) {
        const int64_t per_wave = roundup((int64_t)r.regs_per_thread * m.wave_size, m.reg_granule);
        if (per_wave > m.regs_per_partition) return 0;
        const int64_t waves_per_part = m.regs_per_partition / per_wave;
        b = std::min<int64_t>(b, m.partitions * waves_per_part / wpb);
    }
    if (r.lds_bytes > 0) b = std::min<int64_t>(b, m.lds_per_cu / roundup(r.lds_bytes, m.lds_granule));
    if (b < 0) b = 0;
    if (waves) *waves = (int)(b * wpb);
    return (int)b;
}

static ppx_device_model gfx950_model() {
    ppx_device_model m{};
    m.wave_size = 64;
    m.partitions = 4;
    m.regs_per_partition = 512 * 64;
    m.reg_granule = 8 * 64;
    m.max_waves_per_cu = 32;
    m.max_blocks_per_cu = 32;
    m.lds_per_cu = 160 * 1024;
    m.lds_per_block = 160 * 1024;
    m.lds_granule = 512;
    m.num_cus = 256;
    if (const DeviceInfo *di = device_info_if_ready()) {
        m.lds_per_block = (int32_t)di->lds_per_block;
        m.lds_per_cu = (int32_t)di->lds_per_cu;
        m.max_waves_per_cu = di->max_threads_per_cu / m.wave_size;
        m.num_cus = di->cus;
    }
    return m;
}

// ============================================================ guideline
struct CandEval {
    int idx;
    int blocks, waves;
    double occ;  // warp occupancy W_SM / W^max
    bool s1;     // W_SM = W^max and B_a = B^max
    int radix, P, lds;
};

static int analytical_pick_impl(const ppx_device_model &m, const ppx_config *c,
                                const ppx_resource *res, int n, int64_t batch, int flags) {
    std::vector<CandEval> ev;
    for (int i = 0; i < n; ++i) {
        int w = 0;
        const int b = occupancy_blocks(m, res[i], &w);
        if (b <= 0) continue;
        CandEval e{i, b, w, 0.0, false, c[i].radix, c[i].elems_per_thread, res[i].lds_bytes};
        e.occ = (double)w / m.max_waves_per_cu;
        e.s1 = (w == m.max_waves_per_cu && b == m.max_blocks_per_cu);
        ev.push_back(e);
    }
    if (ev.empty()) return -1;
    if (flags & PPX_ANALYTICAL_GRID_FILL) {
        std::vector<CandEval> fill;
        for (const auto &e : ev) {
            const int64_t gb = c[e.idx].problems_per_block > 0 ? c[e.idx].problems_per_block : 1;
            const int64_t grid = (batch + gb - 1) / gb;
            if (grid >= (int64_t)e.blocks * m.num_cus) fill.push_back(e);
        }
        if (!fill.empty()) ev.swap(fill);
    }
    // the occupancy window of steps 1-2: [60%, 100%] of W^max in the paper;
    // [50%, 100%] (four waves per SIMD) with the gfx950 term
    const double lo = (flags & PPX_ANALYTICAL_WINDOW_50) ? 0.5 : 0.6;
    std::vector<CandEval> window;
    for (const auto &e : ev)
        if (e.occ >= lo - 1e-12) window.push_back(e);
    auto better_window = [](const CandEval &a, const CandEval &b) {
        // step 4: larger radix first; then steps 1-2: full occupancy with all
        // blocks, more active blocks, higher occupancy; then larger P, less LDS
        if (a.radix != b.radix) return a.radix > b.radix;
        if (a.s1 != b.s1) return a.s1;
        if (a.blocks != b.blocks) return a.blocks > b.blocks;
        if (a.occ != b.occ) return a.occ > b.occ;
        if (a.P != b.P) return a.P > b.P;
        if (a.lds != b.lds) return a.lds < b.lds;
        return a.idx < b.idx;
    };
    auto better_fallback = [](const CandEval &a, const CandEval &b) {
        // step 3: highest occupancy, ties to larger P (then radix, less LDS)
        if (a.occ != b.occ) return a.occ > b.occ;
        if (a.P != b.P) return a.P > b.P;
        if (a.radix != b.radix) return a.radix > b.radix;
        if (a.lds != b.lds) return a.lds < b.lds;
        return a.idx < b.idx;
    };
    if (!window.empty()) return std::min_element(window.begin(), window.end(), better_window)->idx;
    return std::min_element(ev.begin(), ev.end(), better_fallback)->idx;
}

// ============================================================ GP + EI
// Matern-5/2 ARD kernel.
static double matern52(const double *a, const double *b, int d, const double *ls, double sf2) {
    double r2 = 0;
    for (int k = 0; k < d; ++k) {
        const double t = (a[k] - b[k]) / ls[k];
        r2 += t * t;
    }
    const double s = std::sqrt(5.0 * r2);
    return sf2 * (1.0 + s + s * s / 3.0) * std::exp(-s);
}

// In-place Cholesky of an n x n SPD matrix (lower). false if not SPD.
static bool cholesky(std::vector<double> &A, int n) {
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0)) return false;
        const double l = std::sqrt(s);
        A[j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / l;
        }
    }
    return true;
}

static void chol_solve_lower(const std::vector<double> &L, int n, std::vector<double> &b) {
    for (int i = 0; i < n; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= L[i * n + k] * b[k];
        b[i] = t / L[i * n + i];
    }
}

static void chol_solve_upper(const std::vector<double> &L, int n, std::vector<double> &b) {
    for (int i = n - 1; i >= 0; --i) {
        double t = b[i];
        for (int k = i + 1; k < n; ++k) t -= L[k * n + i] * b[k];
        b[i] = t / L[i * n + i];
    }
}

struct GP {
    int n = 0, d = 0;
    std::vector<double> X, L, alpha, ls;
    double sf2 = 1, noise = 1e-4;

    bool fit_fixed(const std::vector<double> &Xin, const std::vector<double> &y, int n_, int d_,
                   const double *ls_, double sf2_, double noise_, double *logml) {
        n = n_;
        d = d_;
        X = Xin;
        ls.assign(ls_, ls_ + d);
        sf2 = sf2_;
        noise = noise_;
        L.assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) {
                double k = matern52(&X[i * d], &X[j * d], d, ls.data(), sf2);
                if (i == j) k += noise;
                L[i * n + j] = k;
                L[j * n + i] = k;
            }
        if (!cholesky(L, n)) return false;
        alpha = y;
        chol_solve_lower(L, n, alpha);
        double quad = 0;
        for (double v : alpha) quad += v * v;
        chol_solve_upper(L, n, alpha);
        if (logml) {
            double ld = 0;
            for (int i = 0; i < n; ++i) ld += std::log(L[i * n + i]);
            *logml = -0.5 * quad - ld - 0.5 * n * std::log(2 * M_PI);
        }
        return true;
    }

    void predict(const double *xq, double *mu, double *var) const {
        std::vector<double> k(n);
        for (int i = 0; i < n; ++i) k[i] = matern52(xq, &X[i * d], d, ls.data(), sf2);
        double m = 0;
        for (int i = 0; i < n; ++i) m += k[i] * alpha[i];
        std::vector<double> v = k;
        chol_solve_lower(L, n, v);
        double q = 0;
        for (double t : v) q += t * t;
        *mu = m;
        *var = std::max(sf2 - q, 1e-12);
    }
};

// Nelder-Mead on f over R^dim (minimisation).
template <typename F>
static std::vector<double> nelder_mead(F f, std::vector<double> x0, double step, int iters) {
    const int dim = (int)x0.size();
    std::vector<std::vector<double>> s(dim + 1, x0);
    std::vector<double> fv(dim + 1);
    for (int i = 0; i < dim; ++i) s[i + 1][i] += step;
    for (int i = 0; i <= dim; ++i) fv[i] = f(s[i]);
    for (int it = 0; it < iters; ++it) {
        std::vector<int> ord(dim + 1);
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(), [&](int a, int b) { return fv[a] < fv[b]; });
        std::vector<std::vector<double>> s2(dim + 1);
        std::vector<double> f2(dim + 1);
        for (int i = 0; i <= dim; ++i) {
            s2[i] = s[ord[i]];
            f2[i] = fv[ord[i]];
        }
        s.swap(s2);
        fv.swap(f2);
        if (std::fabs(fv[dim] - fv[0]) < 1e-9) break;
        std::vector<double> cen(dim, 0.0);
        for (int i = 0; i < dim; ++i)
            for (int k = 0; k < dim; ++k) cen[k] += s[i][k] / dim;
        auto lerp = [&](double t) {
            std::vector<double> p(dim);
            for (int k = 0; k < dim; ++k) p[k] = cen[k] + t * (s[dim][k] - cen[k]);
            return p;
        };
        std::vector<double> xr = lerp(-1.0);
        double fr = f(xr);
        if (fr < fv[0]) {
            std::vector<double> xe = lerp(-2.0);
            double fe = f(xe);
            if (fe < fr) { s[dim] = xe; fv[dim] = fe; } else { s[dim] = xr; fv[dim] = fr; }
        } else if (fr < fv[dim - 1]) {
            s[dim] = xr;
            fv[dim] = fr;
        } else {
            std::vector<double> xc = lerp(fr < fv[dim] ? -0.5 : 0.5);
            double fc = f(xc);
            if (fc < std::min(fr, fv[dim])) {
                s[dim] = xc;
                fv[dim] = fc;
            } else {
                for (int i = 1; i <= dim; ++i) {
                    for (int k = 0; k < dim; ++k) s[i][k] = s[0][k] + 0.5 * (s[i][k] - s[0][k]);
                    fv[i] = f(s[i]);
                }
            }
        }
    }
    int best = (int)(std::min_element(fv.begin(), fv.end()) - fv.begin());
    return s[best];
}

// Fits hyperparameters by maximum marginal likelihood; y already standardised.
static bool fit_gp(GP &gp, const std::vector<double> &X, const std::vector<double> &y, int n, int d) {
    // theta = (log ls[0..d), log sf2, log noise), clamped to sane boxes
    auto unpack = [&](const std::vector<double> &t, std::vector<double> &ls, double &sf2, double &nz) {
        ls.resize(d);
        for (int k = 0; k < d; ++k) ls[k] = std::exp(std::min(std::max(t[k], std::log(0.05)), std::log(20.0)));
        sf2 = std::exp(std::min(std::max(t[d], std::log(0.05)), std::log(20.0)));
        nz = std::exp(std::min(std::max(t[d + 1], std::log(1e-6)), std::log(1.0)));
    };
    auto nll = [&](const std::vector<double> &t) {
        std::vector<double> ls;
        double sf2, nz;
        unpack(t, ls, sf2, nz);
        GP g;
        double lml;
        if (!g.fit_fixed(X, y, n, d, ls.data(), sf2, nz, &lml)) return 1e30;
        return -lml;
    };
    std::vector<double> best;
    double bestv = 1e300;
    for (double l0 : {std::log(0.25), std::log(1.0), std::log(3.0)}) {
        std::vector<double> t0(d + 2, l0);
        t0[d] = 0.0;
        t0[d + 1] = std::log(1e-2);
        std::vector<double> t = nelder_mead(nll, t0, 0.7, 300);
        const double v = nll(t);
        if (v < bestv) {
            bestv = v;
            best = t;
        }
    }
    std::vector<double> ls;
    double sf2, nz;
    unpack(best, ls, sf2, nz);
    return gp.fit_fixed(X, y, n, d, ls.data(), sf2, nz, nullptr);
}

static double norm_pdf(double z) { return std::exp(-0.5 * z * z) / std::sqrt(2 * M_PI); }
static double norm_cdf(double z) { return 0.5 * std::erfc(-z / std::sqrt(2.0)); }

static double expected_improvement(double mu, double sigma, double best) {
    if (!(sigma > 0)) return std::max(best - mu, 0.0);
    const double z = (best - mu) / sigma;
    return (best - mu) * norm_cdf(z) + sigma * norm_pdf(z);
}

// GP inputs: log2 radix, log2 L, log2 G_b, and one indicator per algorithm
// variant present among the candidates (the variants are categories, not an
// ordered scale); each column scaled to [0, 1].
// Large-FFT plans are timed and searched as configurations tagged with
// kLargePlanAlgo: radix = radix_a, elems_per_thread = radix_b,
// threads_per_block = n1, problems_per_block = tile_a, lds_elems = tile_b.
// Their GP inputs are the log2 of those five values.
constexpr int kLargePlanAlgo = 0x40;
static ppx_config plan_to_config(const ppx_fft_plan &p) {
    return ppx_config{p.radix_a, p.radix_b, 1 << p.log2_n1, p.tile_a, p.tile_b, kLargePlanAlgo};
}
static ppx_fft_plan config_to_plan(const ppx_config &c) {
    return ppx_fft_plan{ilog2(c.threads_per_block), c.radix, c.elems_per_thread, c.problems_per_block,
                        c.lds_elems};
}

static void features(const ppx_config *c, int n, std::vector<double> &F, int &d) {
    if (n > 0 && c[0].algo == kLargePlanAlgo) {
        d = 5;
        F.assign((size_t)n * d, 0.0);
        for (int i = 0; i < n; ++i) {
            F[i * d + 0] = std::log2((double)c[i].radix);
            F[i * d + 1] = std::log2((double)c[i].threads_per_block);
            F[i * d + 2] = std::log2((double)c[i].elems_per_thread);
            F[i * d + 3] = std::log2((double)c[i].problems_per_block);
            F[i * d + 4] = std::log2((double)c[i].lds_elems);
        }
        for (int k = 0; k < d; ++k) {
            double lo = 1e300, hi = -1e300;
            for (int i = 0; i < n; ++i) {
                lo = std::min(lo, F[i * d + k]);
                hi = std::max(hi, F[i * d + k]);
            }
            for (int i = 0; i < n; ++i) F[i * d + k] = hi > lo ? (F[i * d + k] - lo) / (hi - lo) : 0.0;
        }
        return;
    }
    std::vector<int> algos;
    for (int i = 0; i < n; ++i)
        if (std::find(algos.begin(), algos.end(), c[i].algo) == algos.end()) algos.push_back(c[i].algo);
    std::sort(algos.begin(), algos.end());
    const int na = algos.size() > 1 ? (int)algos.size() : 0;
    d = 3 + na;
    F.assign((size_t)n * d, 0.0);
    for (int i = 0; i < n; ++i) {
        F[i * d + 0] = std::log2((double)std::max(1, c[i].radix));
        F[i * d + 1] = std::log2((double)std::max(1, c[i].threads_per_block));
        F[i * d + 2] = std::log2((double)std::max(1, c[i].problems_per_block));
        for (int a = 0; a < na; ++a) F[i * d + 3 + a] = c[i].algo == algos[a] ? 1.0 : 0.0;
    }
    for (int k = 0; k < d; ++k) {
        double lo = 1e300, hi = -1e300;
        for (int i = 0; i < n; ++i) {
            lo = std::min(lo, F[i * d + k]);
            hi = std::max(hi, F[i * d + k]);
        }
        for (int i = 0; i < n; ++i) F[i * d + k] = hi > lo ? (F[i * d + k] - lo) / (hi - lo) : 0.0;
    }
}

// The search of Sec. IV-B as an ask/tell state: ask() names the next
// candidate to time (n_init random ones, then the Expected-Improvement
// maximiser of a GP fitted to the log costs so far), tell() records its cost;
// ask() returns -1 once max_evals candidates are timed, `patience`
// evaluations pass without a relative improvement of min_rel, or no
// candidate is left.  Used synchronously by the offline tuner and one
// evaluation at a time by the online sessions of a request loop.
class BoState {
  public:
    BoState(const ppx_config *c, int n, int max_evals, int n_init, int patience, double min_rel, uint64_t seed)
        : n_(n), min_rel_(min_rel) {
        if (n_init <= 0) n_init = std::max(3, (int)std::ceil(0.05 * n));
        patience_ = patience > 0 ? patience : 5;
        max_evals_ = max_evals <= 0 || max_evals > n ? n : max_evals;
        n_init_ = std::min(n_init, max_evals_);
        features(c, n, F_, d_);
        done_.assign(n, 0);
        std::mt19937_64 rng(seed);
        perm_.resize(n);
        std::iota(perm_.begin(), perm_.end(), 0);
        std::shuffle(perm_.begin(), perm_.end(), rng);
    }

    int ask() {
        const int m = (int)ord_.size();
        if (m < n_init_) return perm_[m];
        if (m >= max_evals_) return -1;
        if (m - last_improve_ >= patience_) return -1;
        std::vector<double> X((size_t)m * d_), y(m);
        for (int k = 0; k < m; ++k) {
            std::copy(&F_[ord_[k] * d_], &F_[ord_[k] * d_] + d_, &X[k * d_]);
            y[k] = std::log(std::max(val_[k], 1e-30));
        }
        const double mean = std::accumulate(y.begin(), y.end(), 0.0) / m;
        double sd = 0;
        for (double v : y) sd += (v - mean) * (v - mean);
        sd = m > 1 ? std::sqrt(sd / (m - 1)) : 1.0;
        if (!(sd > 1e-12)) sd = 1.0;
        for (double &v : y) v = (v - mean) / sd;
        GP gp;
        const bool ok = fit_gp(gp, X, y, m, d_);
        double ybest = 1e300;
        for (double v : y) ybest = std::min(ybest, v);
        int pick = -1;
        double pv = -1;
        for (int i = 0; i < n_; ++i) {
            if (done_[i]) continue;
            double ei = 0.0;
            if (ok) {
                double mu, var;
                gp.predict(&F_[i * d_], &mu, &var);
                ei = expected_improvement(mu, std::sqrt(var), ybest);
            }
            if (ei > pv) {
                pv = ei;
                pick = i;
            }
        }
        return pick;
    }

    // Cost v of candidate i (negative or non-finite: the run failed).
    void tell(int i, double v) {
        done_[i] = 1;
        ord_.push_back(i);
        const bool bad = !(v >= 0) || !std::isfinite(v);
        failed_.push_back(bad);
        val_.push_back(bad ? -1.0 : v);
        if (!bad) worst_ = std::max(worst_, v);
        // re-penalise every failure at 10x the worst valid cost so far
        for (size_t k = 0; k < val_.size(); ++k)
            if (failed_[k]) val_[k] = worst_ > 0 ? 10.0 * worst_ : 1e9;
        if (!bad && v < best_ * (1.0 - min_rel_)) last_improve_ = (int)ord_.size();
        if (!bad && v < best_) {
            best_ = v;
            best_i_ = i;
        }
        if ((int)ord_.size() == n_init_) last_improve_ = std::max(last_improve_, n_init_);
    }

    int evals() const { return (int)ord_.size(); }
    int best_index() const { return best_i_; }
    double best_cost() const { return best_; }
    const std::vector<int> &order() const { return ord_; }
    const std::vector<double> &values() const { return val_; }

  private:
    int n_, d_ = 0, n_init_, patience_, max_evals_;
    double min_rel_;
    std::vector<double> F_;
    std::vector<char> done_, failed_;
    std::vector<int> perm_, ord_;
    std::vector<double> val_;
    double worst_ = 0, best_ = 1e300;
    int best_i_ = -1, last_improve_ = 0;
};

static int bo_search_impl(const ppx_config *c, int n, ppx_eval_fn fn, void *user, int max_evals,
                          int n_init, int patience, double min_rel, uint64_t seed, int *order,
                          double *values, int *evals_used, int *best_index) {
    if (n <= 0) return fail(PPX_EINVAL, "empty candidate list");
    BoState bo(c, n, max_evals, n_init, patience, min_rel, seed);
    for (int i = bo.ask(); i >= 0; i = bo.ask()) bo.tell(i, fn(&c[i], user));
    const auto &ord = bo.order();
    const auto &val = bo.values();
    for (size_t k = 0; k < ord.size(); ++k) {
        if (order) order[k] = ord[k];
        if (values) values[k] = val[k];
    }
    if (evals_used) *evals_used = bo.evals();
    if (best_index) *best_index = bo.best_index();
    return bo.best_index() >= 0 ? PPX_OK : fail(PPX_ETIMEOUT, "every evaluated candidate failed");
}

// ============================================================ tune cache
namespace {
std::mutex g_cache_mu;
struct CacheEntry {
    ppx_config cfg;
    double us;
    int method;
};
std::map<std::tuple<int, int, int64_t, int>, CacheEntry> g_cache;  // (op, dtype, n, algo filter)
}  // namespace

// The entry for (op, dtype, n) over every algorithm; if only per-algorithm
// (per-family) entries were tuned, the fastest of them.
bool cached_config(int op, int dtype, int64_t n, ppx_config &c) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find({op, dtype, n, -1});
    if (it != g_cache.end()) {
        c = it->second.cfg;
        return true;
    }
    const CacheEntry *best = nullptr;
    for (int a = 0; a <= kTriMaxBase; ++a) {
        auto jt = g_cache.find({op, dtype, n, a});
        if (jt != g_cache.end() && jt->second.us > 0 && (!best || jt->second.us < best->us)) best = &jt->second;
    }
    if (!best) return false;
    c = best->cfg;
    return true;
}

static void cache_put(int op, int dtype, int64_t n, int algo, const ppx_config &c, double us,
                      int method) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[{op, dtype, n, algo}] = CacheEntry{c, us, method};
}

void store_cached_config(int op, int dtype, int64_t n, const ppx_config &c) {
    cache_put(op, dtype, n, -1, c, 0.0, -1);
}

// ============================================================ resources
// VGPR counts reported by the compiler for these kernels, used only
// when no device is present to ask (CPU-side resolution of a NULL config).
static int static_vgprs(int op, int dtype, int P, int algo) {
    if (op == PPX_OP_FFT) return P <= 2 ? 16 : P <= 4 ? 29 : P <= 8 ? 55 : P <= 16 ? 107 : 200;
    if (op == PPX_OP_SCAN)
        return (dtype == PPX_F64 ? 2 : 1) * (P <= 2 ? 10 : P <= 4 ? 12 : P <= 8 ? 16 : P <= 16 ? 24 : 40);
    if (tri_in_wave(algo))
        return (dtype == PPX_F64 ? 2 : 1) *
                   (tri_base(algo) == PPX_TRI_PCR_SHFL || tri_base(algo) == PPX_TRI_PCR_REG ? 6 : 5) * P *
                   ((algo & PPX_TRI_PIPE) ? 2 : 1) + 16;
    return dtype == PPX_F64 ? (algo == PPX_TRI_PCR ? 44 : 40) : (algo == PPX_TRI_PCR ? 32 : 28);
}

static const void *kernel_for(int op, int dtype, int64_t n, const ppx_config &c) {
    switch (op) {
        case PPX_OP_FFT: return fft_kernel(c.radix, c.elems_per_thread, c.algo, ilog2(n));
        case PPX_OP_SCAN: return scan_kernel(dtype, c.elems_per_thread, c.algo);
        default: return tridiag_kernel(dtype, c.algo, c.elems_per_thread, n);
    }
}

static int64_t dyn_lds(int op, int dtype, int64_t n, const ppx_config &c) {
    switch (op) {
        case PPX_OP_FFT: return fft_lds_bytes((int)n, c.problems_per_block, c.algo, c.radix);
        case PPX_OP_SCAN: return scan_lds_bytes((int)n, c.problems_per_block, c.elems_per_thread, dtype);
        default: return tridiag_lds_bytes((int)n, c, dtype);
    }
}

static int elem_bytes(int op, int dtype) {
    if (op == PPX_OP_FFT) return 8;
    if (op == PPX_OP_SCAN) return dtype == PPX_F64 ? 8 : 4;
    return dtype == PPX_F64 ? 32 : 16;  // four coefficients per equation
}

static int resources(int op, int dtype, int64_t n, const ppx_config &c, bool have_device,
                     ppx_resource &r) {
    r.threads = c.threads_per_block;
    r.lds_bytes = (int32_t)dyn_lds(op, dtype, n, c);
    r.regs_per_thread = static_vgprs(op, dtype, c.elems_per_thread, c.algo);
    if (have_device) {
        const void *k = kernel_for(op, dtype, n, c);
        hipFuncAttributes a;
        if (!k || hipFuncGetAttributes(&a, k) != hipSuccess) return fail(PPX_EHIP, "hipFuncGetAttributes failed");
        r.regs_per_thread = a.numRegs;
        r.lds_bytes += (int32_t)a.sharedSizeBytes;
    }
    return PPX_OK;
}

// Premise (i) of the analytical model (coalesced global accesses) restated
// for these kernels on gfx950: the scan kernel gives each lane P contiguous
// elements, so a load instruction is contiguous across the wave only when
// those P elements are one 16-byte vector (P * element size <= 16); where no
// such configuration exists (large n) the smallest P comes closest.  The FFT
// and tridiagonal kernels read consecutive elements with consecutive lanes
// for every P.
static bool coalesced(int op, int dtype, const ppx_config &c) {
    return op != PPX_OP_SCAN || c.elems_per_thread * elem_bytes(op, dtype) <= 16;
}

static bool persistent(int op, int algo) {
    switch (op) {
        case PPX_OP_FFT: return (algo & PPX_FFT_LDS_PIPE) != 0;
        case PPX_OP_SCAN: return (algo & PPX_SCAN_KS_PIPE) != 0;
        default: return (algo & PPX_TRI_PIPE) != 0;
    }
}
static int persistent_flag(int op) {
    return op == PPX_OP_FFT ? PPX_FFT_LDS_PIPE : op == PPX_OP_SCAN ? PPX_SCAN_KS_PIPE : PPX_TRI_PIPE;
}

// Flags of the gfx950 analytical model: the paper's guideline plus our grid
// fill term and a 50% occupancy window.
constexpr int kGfx950Flags = PPX_ANALYTICAL_GRID_FILL | PPX_ANALYTICAL_WINDOW_50;

// The candidates the gfx950 guideline ranks:
//  * coalesced ones (above);
//  * no persistent variants: the occupancy model does not see what they
//    change; the choice is mapped to its persistent twin afterwards (see
//    analytical_select);
//  * tridiagonal: the in-wave variants whenever one is valid (the paper's
//    rule to use the warp-level exchange when a system fits one), and for
//    PCR the LDS-exchange variant rather than the shuffle one: on gfx950 a
//    shuffle moves a quarter of the bytes per instruction that a 16-byte LDS
//    access moves, and PCR exchanges six values per equation and step; with
//    no family filter, the CR family (less work).
static std::vector<ppx_config> analytical_candidates(int op, int dtype, const std::vector<ppx_config> &all) {
    std::vector<ppx_config> base;
    for (const auto &c : all)
        if (!persistent(op, c.algo)) base.push_back(c);
    if (base.empty()) base = all;
    std::vector<ppx_config> out;
    for (const auto &c : base)
        if (coalesced(op, dtype, c)) out.push_back(c);
    if (out.empty()) {  // no fully coalesced shape: the smallest P
        int pmin = 1 << 30;
        for (const auto &c : base) pmin = std::min(pmin, c.elems_per_thread);
        for (const auto &c : base)
            if (c.elems_per_thread == pmin) out.push_back(c);
    }
    if (op == PPX_OP_TRIDIAG) {
        std::vector<ppx_config> wave;
        for (const auto &c : out)
            if (tri_in_wave(c.algo) && c.algo != PPX_TRI_PCR_SHFL) wave.push_back(c);
        if (!wave.empty()) out.swap(wave);
        // with both families present (no family filter), CR: O(n) work per
        // system against PCR's O(n log n)
        std::vector<ppx_config> cr;
        for (const auto &c : out)
            if (tri_family(c.algo) == PPX_TRI_CR) cr.push_back(c);
        if (!cr.empty()) out.swap(cr);
    }
    return out;
}

// Rule (v) of the gfx950 model, after the guideline has ranked: a choice that
// keeps at most two workgroups resident per CU runs as its persistent twin
// when one exists (the resident workgroups then overlap their own loads with
// their computation instead of alternating between the two).
static int analytical_select(int op, int dtype, int64_t n, int64_t batch, const std::vector<ppx_config> &cands,
                             bool have_device, ppx_config &out);

// ============================================================ analytical config
int analytical_config(int op, int dtype, int64_t n, int64_t batch, ppx_config &c) {
    static std::mutex memo_mu;
    static std::map<std::tuple<int, int, int64_t, int64_t, bool>, ppx_config> memo;
    const bool have_device = device_info() != nullptr;
    const auto key = std::make_tuple(op, dtype, n, batch, have_device);
    {
        std::lock_guard<std::mutex> lk(memo_mu);
        auto it = memo.find(key);
        if (it != memo.end()) {
            c = it->second;
            return PPX_OK;
        }
    }
    const int total = enumerate_configs(op, dtype, n, nullptr, 0);
    if (total <= 0) return default_config(op, dtype, n, c);
    std::vector<ppx_config> all(total);
    enumerate_configs(op, dtype, n, all.data(), total);
    if (analytical_select(op, dtype, n, batch, all, have_device, c) != PPX_OK)
        return default_config(op, dtype, n, c);
    std::lock_guard<std::mutex> lk(memo_mu);
    memo[key] = c;
    fail(PPX_OK, "");
    return PPX_OK;
}

static int analytical_select(int op, int dtype, int64_t n, int64_t batch, const std::vector<ppx_config> &cands,
                             bool have_device, ppx_config &out) {
    const std::vector<ppx_config> sub = analytical_candidates(op, dtype, cands);
    const int cnt = (int)sub.size();
    if (cnt == 0) return fail(PPX_ECONFIG, "no candidate");
    std::vector<ppx_resource> res(cnt);
    int rc;
    for (int i = 0; i < cnt; ++i)
        if ((rc = resources(op, dtype, n, sub[i], have_device, res[i]))) return rc;
    const ppx_device_model m = gfx950_model();
    const int k = analytical_pick_impl(m, sub.data(), res.data(), cnt, batch, kGfx950Flags);
    if (k < 0) return fail(PPX_ECONFIG, "no candidate fits the device");
    out = sub[k];
    if (occupancy_blocks(m, res[k], nullptr) <= 2) {
        ppx_config twin = out;
        twin.algo |= persistent_flag(op);
        for (const auto &c : cands)
            if (std::memcmp(&c, &twin, sizeof twin) == 0) out = twin;
    }
    return PPX_OK;
}

// ============================================================ GPU timing
namespace {
uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
double unif(uint64_t &s) { return (splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

// Device buffers for one (op, dtype, n, batch), replicated into enough sets
// that consecutive timed launches never reuse cached data.
struct Bench {
    int op, dtype;
    int64_t n, batch;
    std::vector<std::vector<void *>> sets;  // per set: in.. out
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> ev;

    ~Bench() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (auto &s : sets)
            for (void *p : s)
                if (p) (void)hipFree(p);
        for (auto e : ev) (void)hipEventDestroy(e);
        if (stream) (void)hipStreamDestroy(stream);
    }

    int init(int reps) {
        const int64_t cnt = n * batch;
        std::vector<size_t> bytes;
        int nin;
        if (op == PPX_OP_FFT) {
            bytes = {size_t(cnt) * 8, size_t(cnt) * 8};
            nin = 1;
        } else if (op == PPX_OP_SCAN) {
            const size_t es = dtype == PPX_F64 ? 8 : 4;
            bytes = {size_t(cnt) * es, size_t(cnt) * es};
            nin = 1;
        } else {
            const size_t es = dtype == PPX_F64 ? 8 : 4;
            bytes.assign(5, size_t(cnt) * es);
            nin = 4;
        }
        size_t set_bytes = 0;
        for (size_t b : bytes) set_bytes += b;
        const size_t target = size_t(1) << 30;  // rotate through >= 1 GiB
        int nsets = (int)std::min<size_t>(16, std::max<size_t>(2, (target + set_bytes - 1) / set_bytes));
        // host copy of one input set (seeded synthetic values)
        std::vector<std::vector<char>> host(nin);
        uint64_t s = 0x5eed;
        for (int k = 0; k < nin; ++k) host[k].resize(bytes[k]);
        if (op == PPX_OP_FFT) {
            float *f = reinterpret_cast<float *>(host[0].data());
            for (int64_t i = 0; i < 2 * cnt; ++i) f[i] = (float)(2 * unif(s) - 1);
        } else if (op == PPX_OP_SCAN) {
            if (dtype == PPX_I32) {
                int *v = reinterpret_cast<int *>(host[0].data());
                for (int64_t i = 0; i < cnt; ++i) v[i] = (int)(splitmix(s) % 201) - 100;
            } else if (dtype == PPX_F64) {
                double *v = reinterpret_cast<double *>(host[0].data());
                for (int64_t i = 0; i < cnt; ++i) v[i] = unif(s);
            } else {
                float *v = reinterpret_cast<float *>(host[0].data());
                for (int64_t i = 0; i < cnt; ++i) v[i] = (float)unif(s);
            }
        } else {
            for (int64_t i = 0; i < cnt; ++i) {
                const double a = 2 * unif(s) - 1, c = 2 * unif(s) - 1;
                const double b = std::fabs(a) + std::fabs(c) + 1 + unif(s), d = 2 * unif(s) - 1;
                const double v[4] = {a, b, c, d};
                for (int k = 0; k < 4; ++k) {
                    if (dtype == PPX_F64) reinterpret_cast<double *>(host[k].data())[i] = v[k];
                    else reinterpret_cast<float *>(host[k].data())[i] = (float)v[k];
                }
            }
        }
        sets.assign(nsets, std::vector<void *>(bytes.size(), nullptr));
        for (int si = 0; si < nsets; ++si)
            for (size_t k = 0; k < bytes.size(); ++k) {
                if (hipMalloc(&sets[si][k], bytes[k]) != hipSuccess) return fail(PPX_ENOMEM, "tune: out of device memory");
                if ((int)k < nin) {
                    if (hipMemcpy(sets[si][k], host[k].data(), bytes[k], hipMemcpyHostToDevice) != hipSuccess)
                        return fail(PPX_EHIP, "tune: upload failed");
                } else if (hipMemset(sets[si][k], 0, bytes[k]) != hipSuccess) {
                    return fail(PPX_EHIP, "tune: memset failed");
                }
            }
        if (hipStreamCreate(&stream) != hipSuccess) return fail(PPX_EHIP, "tune: stream creation failed");
        ev.resize(2 * (size_t)reps);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(PPX_EHIP, "tune: event creation failed");
        return PPX_OK;
    }

    int launch(const ppx_config &c, int set) {
        auto &b = sets[set % sets.size()];
        const int ln = ilog2(n);
        if (op == PPX_OP_FFT && c.algo == kLargePlanAlgo)
            return launch_fft_large(b[0], b[1], ln, batch, config_to_plan(c), false, stream);
        if (op == PPX_OP_FFT) return launch_fft(b[0], b[1], ln, batch, c, false, stream);
        if (op == PPX_OP_SCAN) return launch_scan(b[0], b[1], ln, batch, dtype, c, stream);
        return launch_tridiag(b[0], b[1], b[2], b[3], b[4], ln, batch, dtype, c, stream);
    }

    // Median microseconds over `reps` launches (after 3 warm-ups); negative
    // on a launch failure or when the deadline passes.
    double time(const ppx_config &c, int reps, double deadline_s) {
        for (int w = 0; w < 3; ++w)
            if (launch(c, w) != PPX_OK) return -1.0;
        for (int r = 0; r < reps; ++r) {
            (void)hipEventRecord(ev[2 * r], stream);
            if (launch(c, r + 3) != PPX_OK) {
                (void)hipStreamSynchronize(stream);
                return -1.0;
            }
            (void)hipEventRecord(ev[2 * r + 1], stream);
        }
        const auto t0 = std::chrono::steady_clock::now();
        while (hipEventQuery(ev[2 * reps - 1]) == hipErrorNotReady) {
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (el > deadline_s) {
                (void)hipStreamSynchronize(stream);  // drain before reuse
                fail(PPX_ETIMEOUT, "candidate exceeded its deadline");
                return -2.0;
            }
        }
        std::vector<double> t(reps);
        for (int r = 0; r < reps; ++r) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]) != hipSuccess) return -1.0;
            t[r] = ms * 1e3;
        }
        std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
        return t[reps / 2];
    }
};

struct EvalCtx {
    Bench *b;
    int reps;
    std::vector<std::pair<ppx_config, double>> *trace;
};

double eval_gpu(const ppx_config *c, void *user) {
    auto *ctx = static_cast<EvalCtx *>(user);
    const double us = ctx->b->time(*c, ctx->reps, 60.0);
    if (ctx->trace) ctx->trace->push_back({*c, us});
    return us;
}
}  // namespace

// The valid configurations a tuner searches: every algorithm (algo < 0), one
// algorithm, or for the tridiagonal solvers one family.
static int tune_candidates(int op, int dtype, int64_t n, int algo, std::vector<ppx_config> &cands) {
    const int total = enumerate_configs(op, dtype, n, nullptr, 0);
    if (total < 0) return total;
    std::vector<ppx_config> all(total);
    enumerate_configs(op, dtype, n, all.data(), total);
    cands.clear();
    for (const auto &c : all)
        if (algo < 0 || (op == PPX_OP_TRIDIAG ? tri_family(c.algo) == tri_family(algo) : c.algo == algo))
            cands.push_back(c);
    if (cands.empty()) return fail(PPX_ECONFIG, "no valid configuration to tune");
    return PPX_OK;
}

// The configuration a call with cfg == NULL uses, restricted to one
// tridiagonal family (CR, PCR, the CR -> PCR hybrid, WM or LF): the tune cache's entry recorded for
// that family, else the entry for every algorithm if it belongs to the family,
// else the analytical model's choice among the family's configurations.
int family_config(int dtype, int64_t n, int64_t batch, int family, ppx_config &c) {
    family = tri_family(family);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find({PPX_OP_TRIDIAG, dtype, n, family});
        if (it != g_cache.end()) {
            c = it->second.cfg;
            return PPX_OK;
        }
        auto jt = g_cache.find({PPX_OP_TRIDIAG, dtype, n, -1});
        if (jt != g_cache.end() && tri_family(jt->second.cfg.algo) == family) {
            c = jt->second.cfg;
            return PPX_OK;
        }
    }
    static std::mutex memo_mu;
    static std::map<std::tuple<int, int64_t, int64_t, int, bool>, ppx_config> memo;
    const bool have_device = device_info() != nullptr;
    const auto key = std::make_tuple(dtype, n, batch, family, have_device);
    {
        std::lock_guard<std::mutex> lk(memo_mu);
        auto it = memo.find(key);
        if (it != memo.end()) {
            c = it->second;
            return PPX_OK;
        }
    }
    std::vector<ppx_config> cands;
    if (int rc = tune_candidates(PPX_OP_TRIDIAG, dtype, n, family, cands)) return rc;
    if (int rc = analytical_select(PPX_OP_TRIDIAG, dtype, n, batch, cands, have_device, c)) return rc;
    std::lock_guard<std::mutex> lk(memo_mu);
    memo[key] = c;
    fail(PPX_OK, "");
    return PPX_OK;
}

static int tune_impl(int op, int dtype, int64_t n, int64_t batch, int method, int max_evals,
                     int algo, int reps, ppx_tune_report *rep) {
    if (!rep) return fail(PPX_EINVAL, "null report");
    if (method < PPX_TUNE_EXHAUSTIVE || method > PPX_TUNE_LEARNED) return fail(PPX_EINVAL, "unknown tuning method");
    if (batch < 1) return fail(PPX_EINVAL, "batch must be >= 1");
    if (reps <= 0) reps = 100;
    std::vector<ppx_config> cands;
    int rc = tune_candidates(op, dtype, n, algo, cands);
    if (rc) return rc;
    if (!device_info()) return PPX_EDEVICE;
    Bench bench;
    bench.op = op;
    bench.dtype = dtype;
    bench.n = n;
    bench.batch = batch;
    if ((rc = bench.init(reps))) return rc;
    std::vector<std::pair<ppx_config, double>> trace;
    EvalCtx ctx{&bench, reps, &trace};
    const int nc = (int)cands.size();
    int best = -1;
    if (method == PPX_TUNE_EXHAUSTIVE) {
        double bv = 1e300;
        const int lim = max_evals > 0 ? std::min(max_evals, nc) : nc;
        for (int i = 0; i < lim; ++i) {
            const double v = eval_gpu(&cands[i], &ctx);
            if (v >= 0 && v < bv) {
                bv = v;
                best = i;
            }
        }
    } else if (method == PPX_TUNE_ANALYTICAL) {
        ppx_config pick{};
        if ((rc = analytical_select(op, dtype, n, batch, cands, true, pick))) return rc;
        for (int i = 0; i < nc; ++i)
            if (std::memcmp(&cands[i], &pick, sizeof(ppx_config)) == 0) best = i;
        if (best >= 0) eval_gpu(&cands[best], &ctx);  // timed once, for the report
    } else {
        std::vector<int> order(nc);
        std::vector<double> vals(nc);
        int used = 0;
        rc = bo_search_impl(cands.data(), nc, eval_gpu, &ctx, max_evals, 0, 5, 0.01, 0x2310'16214ULL,
                            order.data(), vals.data(), &used, &best);
        if (rc) return rc;
    }
    if (best < 0) return fail(PPX_ETIMEOUT, "no candidate ran successfully");
    double best_us = -1;
    for (auto it = trace.rbegin(); it != trace.rend(); ++it)
        if (std::memcmp(&it->first, &cands[best], sizeof(ppx_config)) == 0) {
            best_us = it->second;
            break;
        }
    rep->best = cands[best];
    rep->best_us = best_us;
    rep->evals_used = method == PPX_TUNE_ANALYTICAL ? 0 : (int)trace.size();
    rep->ncands = nc;
    if (rep->trace_cfg && rep->trace_us)
        for (int i = 0; i < (int)trace.size() && i < rep->trace_cap; ++i) {
            rep->trace_cfg[i] = trace[i].first;
            rep->trace_us[i] = trace[i].second;
        }
    cache_put(op, dtype, n, algo, cands[best], best_us, method);
    fail(PPX_OK, "");
    return PPX_OK;
}

}  // namespace ppx

using namespace ppx;

// The analytical plan: the most even split (as the default plan), and for
// each pass the (radix, tile) that the occupancy guideline picks among the
// tile kernels valid for its column length.  Premise (i), coalescing, comes
// first: the candidates are the tiles whose row runs are whole cache lines
// (16 columns or more) where any is valid, else the widest valid tile; left
// to itself the occupancy guideline prefers the narrowest tiles (more
// workgroups), whose 16-byte runs waste most of each line.
static int analytical_plan(int64_t n, int64_t batch, ppx_fft_plan &out) {
    fft_default_plan(n, out);
    if (!out.log2_n1) return fail(PPX_ECONFIG, "no valid plan");
    const ppx_device_model m = gfx950_model();
    const int ln = ilog2(n);
    for (int pass = 0; pass < 2; ++pass) {
        const int l = pass == 0 ? ln - out.log2_n1 : out.log2_n1;  // column length
        const int64_t ncols = int64_t(1) << (ln - l);
        std::vector<ppx_config> c;
        std::vector<ppx_resource> r;
        int widest = 0;
        for (int radix : {8, 16})
            for (int tile : {2, 4, 8, 16, 32, 64})
                if (fft_tile_shape_valid(radix, l, tile, pass == 0) && ncols % tile == 0) widest = std::max(widest, tile);
        const int min_tile = std::min(widest, 16);
        for (int radix : {8, 16})
            for (int tile : {2, 4, 8, 16, 32, 64}) {
                if (tile < min_tile || !fft_tile_shape_valid(radix, l, tile, pass == 0) || ncols % tile) continue;
                const int threads = tile * ((1 << l) / radix);
                hipFuncAttributes a;
                if (hipFuncGetAttributes(&a, fft_tile_kernel(radix, l, tile, pass == 0)) != hipSuccess)
                    return fail(PPX_EHIP, "hipFuncGetAttributes failed");
                // a column is a "problem" and a tile of them a workgroup: the
                // grid-fill term then sees the pass's workgroup count
                c.push_back(ppx_config{radix, radix, threads, tile, 0, 0});
                r.push_back(ppx_resource{threads, a.numRegs,
                                         (int32_t)(fft_tile_lds_bytes(radix, l, tile, pass == 0) + a.sharedSizeBytes)});
            }
        if (c.empty()) return fail(PPX_ECONFIG, "no pass kernel");
        const int k = analytical_pick_impl(m, c.data(), r.data(), (int)c.size(), batch * ncols,
                                           PPX_ANALYTICAL_GRID_FILL | PPX_ANALYTICAL_WINDOW_50);
        if (k < 0) return fail(PPX_ECONFIG, "no pass kernel fits a CU");
        const int tile = c[k].problems_per_block;
        if (pass == 0) {
            out.radix_a = c[k].radix;
            out.tile_a = tile;
        } else {
            out.radix_b = c[k].radix;
            out.tile_b = tile;
        }
    }
    return PPX_OK;
}

static int tune_large_impl(int64_t n, int64_t batch, int method, int max_evals, int reps, ppx_fft_plan *best_out,
                           double *best_us_out, int *evals_out, std::vector<std::pair<ppx_config, double>> *trace_out) {
    if (method < PPX_TUNE_EXHAUSTIVE || method > PPX_TUNE_LEARNED) return fail(PPX_EINVAL, "unknown tuning method");
    if (!is_pow2(n) || n <= PPX_MAX_N || n > PPX_MAX_N_LARGE)
        return fail(PPX_EINVAL, "large FFT: n must be a power of two in (16384, 1048576]");
    if (batch < 1) return fail(PPX_EINVAL, "batch must be >= 1");
    if (reps <= 0) reps = 100;
    std::vector<ppx_config> cands;
    for (const auto &p : fft_enumerate_plans(n)) cands.push_back(plan_to_config(p));
    if (cands.empty()) return fail(PPX_ECONFIG, "no valid plan to tune");
    if (!device_info()) return PPX_EDEVICE;
    Bench bench;
    bench.op = PPX_OP_FFT;
    bench.dtype = PPX_C64;
    bench.n = n;
    bench.batch = batch;
    int rc = bench.init(reps);
    if (rc) return rc;
    std::vector<std::pair<ppx_config, double>> trace;
    EvalCtx ctx{&bench, reps, &trace};
    const int nc = (int)cands.size();
    int best = -1;
    if (method == PPX_TUNE_EXHAUSTIVE) {
        double bv = 1e300;
        const int lim = max_evals > 0 ? std::min(max_evals, nc) : nc;
        for (int i = 0; i < lim; ++i) {
            const double v = eval_gpu(&cands[i], &ctx);
            if (v >= 0 && v < bv) {
                bv = v;
                best = i;
            }
        }
    } else if (method == PPX_TUNE_ANALYTICAL) {
        ppx_fft_plan p;
        if ((rc = analytical_plan(n, batch, p))) return rc;
        const ppx_config pc = plan_to_config(p);
        for (int i = 0; i < nc; ++i)
            if (std::memcmp(&cands[i], &pc, sizeof(ppx_config)) == 0) best = i;
        if (best >= 0) eval_gpu(&cands[best], &ctx);  // timed once, for the report
    } else {
        std::vector<int> order(nc);
        std::vector<double> vals(nc);
        int used = 0;
        rc = bo_search_impl(cands.data(), nc, eval_gpu, &ctx, max_evals, 0, 5, 0.01, 0x2310'16214ULL,
                            order.data(), vals.data(), &used, &best);
        if (rc) return rc;
    }
    if (best < 0) return fail(PPX_ETIMEOUT, "no plan ran successfully");
    double best_us = -1;
    for (auto it = trace.rbegin(); it != trace.rend(); ++it)
        if (std::memcmp(&it->first, &cands[best], sizeof(ppx_config)) == 0) {
            best_us = it->second;
            break;
        }
    *best_out = config_to_plan(cands[best]);
    if (best_us_out) *best_us_out = best_us;
    if (evals_out) *evals_out = method == PPX_TUNE_ANALYTICAL ? 0 : (int)trace.size();
    if (trace_out) *trace_out = trace;
    fft_record_plan(n, *best_out);
    fail(PPX_OK, "");
    return PPX_OK;
}

// An online tuning session (include/ppx_tune.h): the learned search over
// one (op, dtype, n, algorithm filter), one evaluation at a time.
struct ppx_online {
    int op = 0, dtype = 0, algo = -1;
    int64_t n = 0;
    std::vector<ppx_config> cands;
    std::unique_ptr<ppx::BoState> bo;
    int pending = -1;       // candidate whose cost is awaited
    bool converged = false;
    ppx_config fallback{};  // before any evaluation: the analytical choice
};

extern "C" {

int ppx_occupancy(const ppx_device_model *m, const ppx_resource *r, int32_t *blocks, int32_t *waves) {
    if (!m || !r) return fail(PPX_EINVAL, "null argument");
    int w = 0;
    const int b = occupancy_blocks(*m, *r, &w);
    if (blocks) *blocks = b;
    if (waves) *waves = w;
    return b > 0 ? PPX_OK : fail(PPX_ECONFIG, "the block cannot be resident");
}

int ppx_device_model_gfx950(ppx_device_model *out) {
    if (!out) return fail(PPX_EINVAL, "null output");
    *out = gfx950_model();
    return PPX_OK;
}

int ppx_analytical_pick(const ppx_device_model *m, const ppx_config *cands, const ppx_resource *res,
                        int ncands, int64_t batch, int flags, int *chosen) {
    if (!m || !cands || !res || !chosen || ncands <= 0) return fail(PPX_EINVAL, "bad argument");
    const int k = analytical_pick_impl(*m, cands, res, ncands, batch, flags);
    *chosen = k;
    return k >= 0 ? PPX_OK : fail(PPX_ECONFIG, "no candidate can be resident");
}

int ppx_analytical_select(int op, int dtype, int64_t n, int64_t batch, const ppx_config *cands,
                          int ncands, int *chosen) {
    if (!cands || !chosen || ncands <= 0 || batch < 1) return fail(PPX_EINVAL, "bad argument");
    std::vector<ppx_config> v(cands, cands + ncands);
    for (const auto &c : v)
        if (int rc = validate_config(op, dtype, n, c)) return rc;
    ppx_config pick{};
    if (int rc = analytical_select(op, dtype, n, batch, v, device_info_if_ready() != nullptr, pick)) return rc;
    *chosen = -1;
    for (int i = 0; i < ncands; ++i)
        if (std::memcmp(&v[i], &pick, sizeof pick) == 0) *chosen = i;
    return *chosen >= 0 ? PPX_OK : fail(PPX_ECONFIG, "analytical choice not among the candidates");
}

int ppx_bo_search(const ppx_config *cands, int ncands, ppx_eval_fn fn, void *user, int max_evals,
                  int n_init, int patience, double min_rel_improvement, uint64_t seed,
                  int *order_out, double *values_out, int *evals_used, int *best_index) {
    if (!cands || !fn) return fail(PPX_EINVAL, "bad argument");
    return bo_search_impl(cands, ncands, fn, user, max_evals, n_init, patience, min_rel_improvement,
                          seed, order_out, values_out, evals_used, best_index);
}

int ppx_gp_posterior(const double *X, const double *y, int n, int d, const double *ls,
                     double sigma_f2, double noise2, const double *Xq, int m, double *mean,
                     double *var) {
    if (!X || !y || !ls || !Xq || !mean || !var || n <= 0 || d <= 0 || m < 0)
        return fail(PPX_EINVAL, "bad argument");
    GP gp;
    std::vector<double> Xv(X, X + (size_t)n * d), yv(y, y + n);
    if (!gp.fit_fixed(Xv, yv, n, d, ls, sigma_f2, noise2, nullptr))
        return fail(PPX_EINVAL, "kernel matrix is not positive definite");
    for (int i = 0; i < m; ++i) gp.predict(Xq + (size_t)i * d, &mean[i], &var[i]);
    return PPX_OK;
}

double ppx_expected_improvement(double mu, double sigma, double best) {
    return expected_improvement(mu, sigma, best);
}

int ppx_tune_ex(int op, int dtype, int64_t n, int64_t batch, int method, int max_evals, int algo,
                int reps, ppx_tune_report *report) {
    return tune_impl(op, dtype, n, batch, method, max_evals, algo, reps, report);
}

int tune(int op, int dtype, int64_t n, int64_t batch, int method, int max_evals, ppx_config *best,
         double *best_us, int *evals_used) {
    if (!best) return fail(PPX_EINVAL, "null output");
    ppx_tune_report rep{};
    const int rc = tune_impl(op, dtype, n, batch, method, max_evals, -1, 0, &rep);
    if (rc) return rc;
    *best = rep.best;
    if (best_us) *best_us = rep.best_us;
    if (evals_used) *evals_used = rep.evals_used;
    if (const char *path = std::getenv("PPX_TUNE_CACHE")) ppx_tune_cache_save(path);
    return PPX_OK;
}

int ppx_time_config(int op, int dtype, int64_t n, int64_t batch, const ppx_config *cfg, int reps,
                    double *median_us) {
    if (!cfg || !median_us) return fail(PPX_EINVAL, "null argument");
    ppx_config c = *cfg;
    complete_config(op, dtype, n, c);
    int rc = validate_config(op, dtype, n, c);
    if (rc) return rc;
    if (batch < 1) return fail(PPX_EINVAL, "batch must be >= 1");
    if (!device_info()) return PPX_EDEVICE;
    if (reps <= 0) reps = 100;
    Bench bench;
    bench.op = op;
    bench.dtype = dtype;
    bench.n = n;
    bench.batch = batch;
    if ((rc = bench.init(reps))) return rc;
    const double us = bench.time(c, reps, 60.0);
    if (us < 0) return us < -1.5 ? PPX_ETIMEOUT : fail(PPX_EHIP, "timed launch failed");
    *median_us = us;
    return PPX_OK;
}

int ppx_kernel_resources(int op, int dtype, int64_t n, const ppx_config *cfg, ppx_resource *out) {
    if (!cfg || !out) return fail(PPX_EINVAL, "null argument");
    ppx_config c = *cfg;
    complete_config(op, dtype, n, c);
    int rc = validate_config(op, dtype, n, c);
    if (rc) return rc;
    if (!device_info()) return PPX_EDEVICE;
    return resources(op, dtype, n, c, true, *out);
}

int ppx_tune_cache_load(const char *path) {
    if (!path) return fail(PPX_EINVAL, "null path");
    std::ifstream f(path);
    if (!f) return fail(PPX_EINVAL, std::string("cannot open ") + path);
    std::string line;
    int count = 0;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string arch;
        if (line.compare(0, 12, "gfx950 plan ") == 0) {  // a tuned large-FFT plan
            std::string tag;
            int64_t n;
            ppx_fft_plan p{};
            double us;
            int method;
            if (!(is >> arch >> tag >> n >> p.log2_n1 >> p.radix_a >> p.radix_b >> p.tile_a >> p.tile_b >> us >>
                  method))
                return fail(PPX_EINVAL, "malformed tune cache line: " + line);
            if (fft_plan_check(n, p) != PPX_OK) continue;  // stale entry
            fft_record_plan(n, p);
            ++count;
            continue;
        }
        int op, dtype, algo, method;
        int64_t n;
        ppx_config c{};
        double us;
        if (!(is >> arch >> op >> dtype >> n >> algo >> c.radix >> c.elems_per_thread >>
              c.threads_per_block >> c.problems_per_block >> c.lds_elems >> c.algo >> us >> method))
            return fail(PPX_EINVAL, "malformed tune cache line: " + line);
        if (arch != "gfx950") continue;
        ppx_config v = c;
        complete_config(op, dtype, n, v);
        if (validate_config(op, dtype, n, v) != PPX_OK) continue;  // stale entry
        cache_put(op, dtype, n, algo, v, us, method);
        ++count;
    }
    fail(PPX_OK, "");
    return count;
}

int ppx_tune_cache_save(const char *path) {
    if (!path) return fail(PPX_EINVAL, "null path");
    std::ofstream f(path);
    if (!f) return fail(PPX_EINVAL, std::string("cannot write ") + path);
    f << "# arch op dtype n algo_filter radix P L G_b S algo us method\n";
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (const auto &kv : g_cache) {
        const auto &c = kv.second.cfg;
        f << "gfx950 " << std::get<0>(kv.first) << ' ' << std::get<1>(kv.first) << ' '
          << std::get<2>(kv.first) << ' ' << std::get<3>(kv.first) << ' ' << c.radix << ' '
          << c.elems_per_thread << ' ' << c.threads_per_block << ' ' << c.problems_per_block << ' '
          << c.lds_elems << ' ' << c.algo << ' ' << kv.second.us << ' ' << kv.second.method << '\n';
    }
    f << "# arch plan n log2_n1 radix_a radix_b tile_a tile_b us method (tuned large-FFT plans)\n";
    for (const auto &np : fft_recorded_plans()) {
        const ppx_fft_plan &p = np.second;
        f << "gfx950 plan " << np.first << ' ' << p.log2_n1 << ' ' << p.radix_a << ' ' << p.radix_b << ' '
          << p.tile_a << ' ' << p.tile_b << " 0 -1\n";
    }
    return f ? PPX_OK : fail(PPX_EINVAL, "write failed");
}

int ppx_tune_cache_clear(void) {
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache.clear();
    }
    fft_clear_plans();
    return PPX_OK;
}

int ppx_tuned_fft_plan(int64_t n, ppx_fft_plan *out) {
    if (!out) return fail(PPX_EINVAL, "null output");
    if (!fft_tuned_plan(n, *out)) return fail(PPX_EINVAL, "no tuned plan for this n");
    return PPX_OK;
}

int tune_fft_large(int64_t n, int64_t batch, int method, int max_evals, ppx_fft_plan *best, double *best_us,
                   int *evals_used) {
    if (!best) return fail(PPX_EINVAL, "null plan");
    return tune_large_impl(n, batch, method, max_evals, 100, best, best_us, evals_used, nullptr);
}

int ppx_tune_large_trace(int64_t n, int64_t batch, int method, int max_evals, int reps, ppx_fft_plan *best,
                         double *best_us, int *evals_used, ppx_fft_plan *trace_plan, double *trace_us, int trace_cap) {
    if (!best) return fail(PPX_EINVAL, "null plan");
    std::vector<std::pair<ppx_config, double>> trace;
    const int rc = tune_large_impl(n, batch, method, max_evals, reps, best, best_us, evals_used, &trace);
    if (rc) return rc;
    for (int i = 0; i < (int)trace.size() && i < trace_cap; ++i) {
        if (trace_plan) trace_plan[i] = config_to_plan(trace[i].first);
        if (trace_us) trace_us[i] = trace[i].second;
    }
    return (int)trace.size();
}

int ppx_tuned_config(int op, int dtype, int64_t n, int algo, ppx_config *out) {
    if (!out) return fail(PPX_EINVAL, "null output");
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find({op, dtype, n, algo});
    if (it == g_cache.end()) return fail(PPX_EINVAL, "no tuned entry");
    *out = it->second.cfg;
    return PPX_OK;
}

int ppx_online_create(int op, int dtype, int64_t n, int64_t batch, int algo, int max_evals,
                      ppx_online **out) {
    if (!out) return fail(PPX_EINVAL, "null output");
    *out = nullptr;
    if (batch < 1) return fail(PPX_EINVAL, "batch must be >= 1");
    auto o = std::make_unique<ppx_online>();
    o->op = op;
    o->dtype = dtype;
    o->n = n;
    o->algo = algo;
    if (int rc = tune_candidates(op, dtype, n, algo, o->cands)) return rc;
    if (int rc = analytical_select(op, dtype, n, batch, o->cands, device_info() != nullptr, o->fallback))
        return rc;
    o->bo = std::make_unique<BoState>(o->cands.data(), (int)o->cands.size(), max_evals, 0, 5, 0.01,
                                      0x2310'16214ULL);
    *out = o.release();
    return PPX_OK;
}

int ppx_online_next(ppx_online *o, int explore, ppx_config *cfg) {
    if (!o || !cfg) return fail(PPX_EINVAL, "null argument");
    if (explore && o->pending < 0 && !o->converged) {
        const int i = o->bo->ask();
        if (i >= 0) {
            o->pending = i;
            *cfg = o->cands[i];
            return 1;
        }
        o->converged = true;
    }
    const int b = o->bo->best_index();
    *cfg = b >= 0 ? o->cands[b] : o->fallback;
    return 0;
}

int ppx_online_report(ppx_online *o, double cost) {
    if (!o) return fail(PPX_EINVAL, "null session");
    if (o->pending < 0) return fail(PPX_EINVAL, "no candidate awaits a cost");
    o->bo->tell(o->pending, cost);
    o->pending = -1;
    return PPX_OK;
}

int ppx_online_status(const ppx_online *o, int *evals, int *converged, ppx_config *best, double *best_cost) {
    if (!o) return fail(PPX_EINVAL, "null session");
    if (evals) *evals = o->bo->evals();
    if (converged) *converged = o->converged ? 1 : 0;
    const int b = o->bo->best_index();
    if (best) *best = b >= 0 ? o->cands[b] : o->fallback;
    if (best_cost) *best_cost = b >= 0 ? o->bo->best_cost() : -1.0;
    return PPX_OK;
}

int ppx_online_destroy(ppx_online *o) {
    delete o;
    return PPX_OK;
}

}  // extern "C"
