// Host drivers of the hot path: AMG-preconditioned CG on the constant M
// (Sec. II and Sec. V of the paper; the preconditioner is built once), and
// the RKC step (Sec. II, ref. [9]) whose every stage is one fused element
// pass (Sec. III) plus one M-solve.
//
// CG keeps all scalars on the device. The host enqueues iteration k+1 before
// it waits for iteration k, and reads only a "done" flag that the
// convergence finaliser writes to pinned host memory, so the GPU never idles
// between iterations; once done, further kernels exit at entry.
#include <algorithm>
#include <cmath>
#include <functional>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "eqs_internal.h"

namespace eqs {

// Host-side ranges for tracing tools (rocprofv3 --marker-trace): an RKC step,
// each stage, each CG solve, each adaptive attempt. Without a tool attached
// a push or pop is a cheap call.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

static PcgSummary read_summary(eqs_ctx* c) {
    const volatile PcgSummary* h = c->h_sum;
    PcgSummary v;
    v.all_done = h->all_done; v.n_active = h->n_active; v.n_breakdown = h->n_breakdown; v.n_notconv = h->n_notconv;
    v.n_zero_rhs = h->n_zero_rhs; v.max_it = h->max_it; v.max_relres = h->max_relres;
    return v;
}

static void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(EQS_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

// The kernels of one CG iteration take every scalar from device memory, so a
// single captured graph replays any iteration of any solve into the same x.
// One graph holds c->graph_iters iterations (a launch runs that many; those
// past convergence change nothing, see pcg_iteration). Graphs are skipped on the null stream
// and while kernels of the iteration are being timed individually (then the
// iterations are launched one by one).
static void run_iteration(eqs_ctx* c, double* x, int prec) {
    const uint32_t iter_classes = (1u << EQS_KCLASS_SPMV_M) | (1u << EQS_KCLASS_PRESMOOTH0) |
                                  (1u << EQS_KCLASS_POSTSMOOTH0) | (1u << EQS_KCLASS_VCYCLE) |
                                  (1u << EQS_KCLASS_CG_UPDATE) | (1u << EQS_KCLASS_RESTRICT0) |
                                  (1u << EQS_KCLASS_PROLONG0) | (1u << EQS_KCLASS_VCOARSE) |
                                  (1u << EQS_KCLASS_POSTSMOOTH1) |
                                  (1u << EQS_KCLASS_FINALISE);
    const int G = c->graph_iters;
    if (!c->use_graphs || c->stream == nullptr || (c->prof_mask & iter_classes)) {
        for (int k = 0; k < G; ++k) pcg_iteration(c->stream, c, nullptr, x, prec);
        return;
    }
    if (c->iter_exec == nullptr || c->iter_x != x || c->iter_prec != prec || c->iter_g != G) {
        if (c->iter_exec) {
            (void)hipGraphExecDestroy(c->iter_exec);
            c->iter_exec = nullptr;
        }
        hipGraph_t g = nullptr;
        EQS_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < G; ++k) pcg_iteration(c->stream, c, nullptr, x, prec);
        EQS_HIP(hipStreamEndCapture(c->stream, &g));
        hipError_t e = hipGraphInstantiate(&c->iter_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) fail(EQS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        c->iter_x = x;
        c->iter_prec = prec;
        c->iter_g = G;
    }
    EQS_HIP(hipGraphLaunch(c->iter_exec, c->stream));
}

void release_graphs(eqs_ctx* c) {
    if (c->iter_exec) (void)hipGraphExecDestroy(c->iter_exec);
    c->iter_exec = nullptr;
    c->iter_x = nullptr;
    c->iter_prec = -1;
}

// Solve M y = rhs for every instance to its own rel-res rtol. The host
// enqueues iteration k+1 before it waits for iteration k (unless k is expected
// to converge) and reads only the pinned summary. When every instance has converged on
// its recursive residual, the true residuals are checked; instances that
// disagree restart from them. Aggregated stats: max iterations, worst status,
// max relres; per-instance results are in c->inst_iters / c->inst_relres.
int solve_M(eqs_ctx* c, const double* rhs, double* y, double rtol, int32_t maxit, eqs_solve_stats* st,
            const double* mx_in, double* mx_out, const std::function<void()>* before_sync) {
    const Range range("eqs: CG solve of M");
    hipStream_t s = c->stream;
    const int prec = c->amg.precision;
    pcg_init(s, c, rhs, y, maxit, rtol, c->amg.flexible, mx_in);
    pcg_zero_rhs_rows(s, c, y);  // instances with rhs = 0 get y = 0 (others untouched)
    check_launch();
    // Iterations are enqueued without waiting for the start's result: an
    // instance that is already done leaves its rows alone, and once all are
    // done an iteration changes nothing (see pcg_iteration).
    PcgSummary v{};
    int restarts = 0;
    int32_t it_before = 0;
    for (;;) {
        int64_t used0[EQS_KCLASS_COUNT];
        for (int k = 0; k < EQS_KCLASS_COUNT; ++k) used0[k] = c->prof_used[k];
        // Launch k+1 (of graph_iters iterations each) is enqueued before the
        // host waits for launch k, so the GPU does not wait for the host; only
        // when launch k is expected to converge (the last two residuals the
        // host has seen, extrapolated geometrically, reach rtol) does the host
        // wait for k first, so that no launch is queued past convergence.
        // When it waits, the host first queues the residual check, which acts
        // only if launch k completed the solve: the check then runs without a
        // host round trip in between.
        const int64_t G = c->graph_iters;
        double rel_prev = -1.0, rel_last = -1.0;
        bool checked = false;
        run_iteration(c, y, prec);
        EQS_HIP(hipEventRecord(c->ev[0], s));
        for (int64_t k = 0;; ++k) {
            const bool last = (k + 1) * G > (int64_t)maxit + 2;  // the device stops itself at maxit
            bool ahead = !last;
            if (ahead && rel_last > 0.0 && rel_prev > rel_last && rel_last * (rel_last / rel_prev) <= rtol)
                ahead = false;
            checked = false;
            if (ahead) {
                run_iteration(c, y, prec);
                EQS_HIP(hipEventRecord(c->ev[(k + 1) & 1], s));
            } else if (!last && !c->prof_mask) {
                pcg_true_residual(s, c, rhs, y, mx_out, true);
                checked = true;
            }
            EQS_HIP(hipEventSynchronize(c->ev[k & 1]));
            const volatile PcgSummary* hs = c->h_sum;
            if (hs->all_done || last) break;
            rel_prev = rel_last;
            rel_last = hs->max_relres;
            if (!ahead) {
                run_iteration(c, y, prec);
                EQS_HIP(hipEventRecord(c->ev[(k + 1) & 1], s));
            }
        }
        check_launch();
        if (c->prof_mask) {
            // the launched iterations past the last one with work returned at
            // entry: their launches are not counted in the kernel-class times
            EQS_HIP(hipStreamSynchronize(s));
            const int32_t it_now = read_summary(c).max_it;
            const int64_t worked = std::max<int64_t>(0, it_now - it_before);
            for (int k : {EQS_KCLASS_SPMV_M, EQS_KCLASS_PRESMOOTH0, EQS_KCLASS_POSTSMOOTH0, EQS_KCLASS_VCYCLE,
                          EQS_KCLASS_CG_UPDATE, EQS_KCLASS_RESTRICT0, EQS_KCLASS_PROLONG0, EQS_KCLASS_VCOARSE,
                          EQS_KCLASS_POSTSMOOTH1})
                c->prof_used[k] = std::min(c->prof_used[k], used0[k] + worked);
            // three finalisers per iteration
            c->prof_used[EQS_KCLASS_FINALISE] =
                std::min(c->prof_used[EQS_KCLASS_FINALISE], used0[EQS_KCLASS_FINALISE] + 3 * worked);
            it_before = it_now;
        }
        // every instance is done on its recursive residual (or out of iterations,
        // or broken down): check the true residuals (queued behind any iteration
        // still in flight, unless already queued above); disagreeing ones restart
        if (!checked) pcg_true_residual(s, c, rhs, y, mx_out);
        if (before_sync) {
            // the host waits for the check only; the caller's work queued behind
            // it keeps the GPU busy meanwhile
            EQS_HIP(hipEventRecord(c->ev[0], s));
            (*before_sync)();
            check_launch();
            EQS_HIP(hipEventSynchronize(c->ev[0]));
        } else {
            check_launch();
            EQS_HIP(hipStreamSynchronize(s));
        }
        v = read_summary(c);
        if (v.all_done || ++restarts > 4) break;
    }
    int status = EQS_OK;
    if (v.n_notconv > 0 || !v.all_done) status = EQS_ERR_NOT_CONVERGED;
    if (v.n_breakdown > 0) status = EQS_ERR_BREAKDOWN;
    for (int64_t i = 0; i < c->n_inst; ++i) {
        const volatile PcgScalars& x = c->h_scal[i];
        c->inst_iters[i] += x.it;
        c->inst_relres[i] = std::max(c->inst_relres[i], (double)x.relres);
    }
    if (st) *st = eqs_solve_stats{v.max_it, status, v.max_relres};
    return status;
}

void apply_preconditioner(eqs_ctx* c, const double* r, double* z) {
    if (c->amg.precision == EQS_PREC_FP32) vcycle<float>(c->stream, c, c->h32, r, z, nullptr, nullptr);
    else vcycle<double>(c->stream, c, c->h64, r, z, nullptr, nullptr);
    check_launch();
    EQS_HIP(hipStreamSynchronize(c->stream));
}

int rkc_step(eqs_ctx* c, double t, double dt, int32_t s, double* x_user, double rtol, int32_t maxit,
             eqs_step_stats* st) {
    const Range range("eqs: RKC step");
    std::vector<double> mu, nu, mut, gmt, cc;
    rkc_coefficients(s, mu, nu, mut, gmt, cc);
    hipStream_t q = c->stream;
    const int64_t NF = c->n_free;

    launch_gather(q, x_user, c->d_int_to_user, c->d_Y0, NF);
    if (!c->have_Flast) {
        launch_fill(q, c->d_F, 0.0, NF);
        c->mx_of_F = false;
    }

    std::fill(c->inst_iters.begin(), c->inst_iters.end(), 0);
    std::fill(c->inst_relres.begin(), c->inst_relres.end(), 0.0);
    c->stage_iters.clear();
    eqs_step_stats S{};
    S.stages = s;
    S.min_iters = INT32_MAX;
    int rc = EQS_OK;
    const double* Ycur = c->d_Y0;
    const double* Yprev = c->d_Y0;
    bool rhs_zeroed = false;  // the last combination cleared d_rhs for this stage's element pass
    bool rhs_ready = false;   // this stage's element pass already ran (queued behind the last solve)
    // With the plain start vector the host queues the rest of the stage (F_0
    // copy, combination) and the next stage's element pass behind the residual
    // check that ends each solve, before it waits for that check: the GPU then
    // works through the host's round trip. The combination writes a third
    // buffer (no operand is overwritten) and the next element pass writes
    // d_rhs_alt, so a restart of the solve only has to queue them again.
    const bool early = c->guess.p.kind == EQS_GUESS_PREVIOUS;
    double* const ybuf[3] = {c->d_Ya, c->d_Yb, c->d_Yc};
    for (int j = 0; j < s; ++j) {
        const Range stage("eqs: RKC stage");
        const double tj = t + cc[j] * dt;
        if (!rhs_ready) launch_kx(q, true, c, Ycur, tj, c->d_rhs, rhs_zeroed);
        check_launch();
        // start vector: F_{j-1} (held in d_F), zero, or an estimator's vector
        const int kind = c->guess.p.kind;
        if (kind == EQS_GUESS_ZERO) {
            launch_fill(q, c->d_F, 0.0, NF);
        } else if (kind == EQS_GUESS_GALERKIN || kind == EQS_GUESS_MLP || kind == EQS_GUESS_MOR) {
            const int u = guess_stage(c);
            if (u == 1) S.guess_used++;
            guess_train(c);  // MLP: overlaps the solve below
        }
        double* out = ybuf[0];
        for (double* b : ybuf)
            if (b != Ycur && b != Yprev) {
                out = b;
                break;
            }
        const bool next = j + 1 < s;
        // the rest of the stage: F_0, Y_{j+1} (clearing the next element pass's
        // output), and with `early` that pass itself
        auto rest = [&]() {
            if (j == 0) launch_copy(q, c->d_F0, c->d_F, NF);
            double* zero = next ? (early ? c->d_rhs_alt : c->d_rhs) : nullptr;
            if (j == 0) {
                launch_rkc_first(c, q, out, c->d_Y0, c->d_F0, mut[1] * dt, NF, zero);
            } else {
                const int k = j + 1;
                launch_rkc_combine(c, q, out, c->d_Y0, Ycur, Yprev, c->d_F, c->d_F0, 1.0 - mu[k] - nu[k], mu[k],
                                   nu[k], mut[k] * dt, gmt[k] * dt, NF, zero);
            }
            if (early && next) launch_kx(q, true, c, out, t + cc[j + 1] * dt, c->d_rhs_alt, true);
        };
        const std::function<void()> rest_fn = rest;
        // F_j = M^{-1} r_j. Started from F_{j-1} itself, the start residual
        // reuses M F_{j-1} from the check that ended the previous solve.
        eqs_solve_stats ss{};
        const bool reuse = kind == EQS_GUESS_PREVIOUS && c->mx_of_F;
        c->mx_of_F = false;
        const int src = solve_M(c, c->d_rhs, c->d_F, rtol, maxit, &ss, reuse ? c->d_mx : nullptr, c->d_mx,
                                early ? &rest_fn : nullptr);
        c->mx_of_F = src == EQS_OK || src == EQS_ERR_NOT_CONVERGED;
        if (kind == EQS_GUESS_GALERKIN || kind == EQS_GUESS_MLP || kind == EQS_GUESS_MOR) guess_after_solve(c, ss.iters);
        c->stage_iters.push_back(ss.iters);
        S.total_iters += ss.iters;
        S.max_iters = std::max(S.max_iters, ss.iters);
        S.min_iters = std::min(S.min_iters, ss.iters);
        S.max_relres = std::max(S.max_relres, ss.relres);
        if (src == EQS_ERR_NOT_CONVERGED) {
            S.not_converged++;
            rc = EQS_ERR_NOT_CONVERGED;
        } else if (src != EQS_OK) {
            if (st) *st = S;
            c->have_Flast = false;
            return src;
        }
        if (!early) rest();
        check_launch();
        if (early && next) std::swap(c->d_rhs, c->d_rhs_alt);  // the next stage's RHS is ready
        rhs_ready = early && next;
        rhs_zeroed = !early && next;
        Yprev = Ycur;
        Ycur = out;
    }
    launch_finish_state(c, Ycur, t + dt, x_user);
    check_launch();
    EQS_HIP(hipStreamSynchronize(q));
    c->have_Flast = true;
    if (S.min_iters == INT32_MAX) S.min_iters = 0;
    if (c->guess.p.kind == EQS_GUESS_MLP) {
        S.train_loss = guess_last_loss(c);
        int32_t kept = 0, dropped = 0;
        guess_device_stats(c, &kept, &dropped);
        S.guess_used += kept;
        S.guess_fallbacks += dropped;
    }
    if (st) *st = S;
    return rc;
}

// ------------------------------------------------------------- adaptive
// One RKC(s) attempt from Y_0 = d_Y0 with F_0 = d_F0 already known: stages
// 1..s-1 (element pass + solve each), combinations into the three Y buffers.
// Returns the buffer holding Y_s; solve statistics go to S.
static const double* rkc_attempt(eqs_ctx* c, double t, double dt, int s, double rtol, int32_t maxit,
                                 eqs_step_stats& S, int& rc) {
    const Range range("eqs: adaptive RKC attempt");
    std::vector<double> mu, nu, mut, gmt, cc;
    rkc_coefficients(s, mu, nu, mut, gmt, cc);
    hipStream_t q = c->stream;
    const int64_t NF = c->n_free;
    if (c->guess.p.kind == EQS_GUESS_ZERO) launch_fill(q, c->d_F, 0.0, NF);
    else launch_copy(q, c->d_F, c->d_F0, NF);  // the first solve starts from F_0
    c->mx_of_F = false;
    double* const ybuf[3] = {c->d_Ya, c->d_Yb, c->d_Yc};
    const double* Yprev = c->d_Y0;
    double* Ycur = ybuf[0];
    launch_rkc_first(c, q, Ycur, c->d_Y0, c->d_F0, mut[1] * dt, NF, c->d_rhs);  // also clears the next RHS
    for (int j = 1; j < s; ++j) {
        launch_kx(q, true, c, Ycur, t + cc[j] * dt, c->d_rhs, true);
        if (c->guess.p.kind == EQS_GUESS_ZERO) launch_fill(q, c->d_F, 0.0, NF);
        eqs_solve_stats ss{};
        const int src = solve_M(c, c->d_rhs, c->d_F, rtol, maxit, &ss);
        S.total_iters += ss.iters;
        S.max_relres = std::max(S.max_relres, ss.relres);
        if (src == EQS_ERR_NOT_CONVERGED) {
            S.not_converged++;
            rc = EQS_ERR_NOT_CONVERGED;
        } else if (src != EQS_OK) {
            rc = src;
            return nullptr;
        }
        double* out = ybuf[0];
        for (double* b : ybuf)
            if (b != Ycur && b != Yprev) {
                out = b;
                break;
            }
        const int k = j + 1;
        launch_rkc_combine(c, q, out, c->d_Y0, Ycur, Yprev, c->d_F, c->d_F0, 1.0 - mu[k] - nu[k], mu[k], nu[k],
                           mut[k] * dt, gmt[k] * dt, NF, k < s ? c->d_rhs : nullptr);
        check_launch();
        Yprev = Ycur;
        Ycur = out;
    }
    return Ycur;
}

// F = M^{-1}(b(t) - K(x_bar)x_bar) at (t, y) into d_F (CG from d_F's content).
static int stage_solve(eqs_ctx* c, const double* y, double t, double rtol, int32_t maxit, eqs_adapt_stats& A) {
    launch_kx(c->stream, true, c, y, t, c->d_rhs);
    if (c->guess.p.kind == EQS_GUESS_ZERO) launch_fill(c->stream, c->d_F, 0.0, c->n_free);
    eqs_solve_stats ss{};
    const int rc = solve_M(c, c->d_rhs, c->d_F, rtol, maxit, &ss);
    c->mx_of_F = false;
    A.stages++;
    A.cg_iters += ss.iters;
    if (rc == EQS_ERR_NOT_CONVERGED) A.not_converged++;
    return rc;
}

int rkc_adaptive(eqs_ctx* c, double t0, double t_end, double* x_user, double rtol, int32_t maxit,
                 const eqs_adapt_params& p, eqs_adapt_record* rec, int32_t cap, int32_t* n_rec, eqs_adapt_stats* st) {
    hipStream_t q = c->stream;
    const int64_t NF = c->n_free;
    const double tau_max = p.tau_max > 0 ? p.tau_max : t_end - t0;
    const int s_max = p.s_max > 0 ? p.s_max : 256;
    const int max_att = p.max_attempts > 0 ? p.max_attempts : 100000;
    eqs_adapt_stats A{};
    int rc = EQS_OK;
    int32_t n = 0;
    auto finish = [&](int code) {
        if (n_rec) *n_rec = n;
        if (st) *st = A;
        return code;
    };
    launch_gather(q, x_user, c->d_int_to_user, c->d_Y0, NF);
    if (!c->have_Flast) launch_fill(q, c->d_F, 0.0, NF);
    c->have_Flast = false;
    // F_0 of the first step
    int src = stage_solve(c, c->d_Y0, t0, rtol, maxit, A);
    if (src != EQS_OK && src != EQS_ERR_NOT_CONVERGED) return finish(src);
    if (src == EQS_ERR_NOT_CONVERGED) rc = src;
    launch_copy(q, c->d_F0, c->d_F, NF);
    double t = t0, tau = std::min(p.tau0, tau_max), tau_prev = -1.0, err_prev = -1.0;
    while (t < t_end) {
        if (n >= max_att) {
            set_error("eqs_rkc_adaptive: too many attempted steps");
            return finish(EQS_ERR_STATE);
        }
        bool last = tau >= t_end - t;
        if (last) tau = t_end - t;
        // stages: the smallest s >= 2 with beta(s) >= tau rho (s_max and a
        // shorter step when even that does not cover it)
        const double rho = max_rate(c, c->d_Y0, t);
        int s = 2;
        if (rho > 0.0) {
            while (s < s_max && rkc_beta(s) < tau * rho) ++s;
            if (rkc_beta(s) < tau * rho) {
                tau = rkc_beta(s) / rho;
                last = false;
            }
        }
        eqs_step_stats S{};
        const double* Ys = rkc_attempt(c, t, tau, s, rtol, maxit, S, rc);
        A.stages += s - 1;
        A.cg_iters += S.total_iters;
        A.not_converged += S.not_converged;
        if (!Ys) return finish(rc);
        const double t1 = last ? t_end : t + tau;
        src = stage_solve(c, Ys, t1, rtol, maxit, A);  // F(t + tau, y_{n+1}), from F_{s-1}
        if (src != EQS_OK && src != EQS_ERR_NOT_CONVERGED) return finish(src);
        if (src == EQS_ERR_NOT_CONVERGED) rc = src;
        const double err = error_norm(c, c->d_Y0, Ys, c->d_F0, c->d_F, tau, p.atol, p.rtol);
        const bool ok = err <= 1.0;
        if (rec && n < cap) rec[n] = eqs_adapt_record{t, tau, err, s, ok ? 1 : 0};
        ++n;
        A.max_s = std::max(A.max_s, s);
        double next;
        if (ok) {
            A.accepted++;
            launch_copy(q, c->d_Y0, Ys, NF);
            launch_copy(q, c->d_F0, c->d_F, NF);
            t = t1;
            if (err == 0.0) next = 10.0 * tau;
            else if (tau_prev < 0.0) next = tau * std::max(0.1, std::min(10.0, 0.8 / std::cbrt(err)));
            else
                next = tau * std::max(0.1, std::min(10.0, 0.8 * (tau / tau_prev) * std::cbrt(err_prev) /
                                                              std::pow(err, 2.0 / 3.0)));
            tau_prev = tau;
            err_prev = err;
        } else {
            A.rejected++;
            next = 0.8 * tau / std::cbrt(err);
        }
        if (!(next >= p.tau_min) || !std::isfinite(next)) {
            set_error("eqs_rkc_adaptive: step size below tau_min");
            return finish(EQS_ERR_STATE);
        }
        tau = std::min(next, tau_max);
    }
    A.last_tau = tau;
    launch_finish_state(c, c->d_Y0, t_end, x_user);
    check_launch();
    EQS_HIP(hipStreamSynchronize(q));
    c->have_Flast = true;  // d_F holds F(t_end, x(t_end)): the next stage solve starts there
    return finish(rc);
}

}  // namespace eqs
