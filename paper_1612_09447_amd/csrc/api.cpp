// C ABI entry points (declared in include/eqs.h). Every call validates its
// arguments, runs under a catch-all so that no exception crosses the ABI, and
// records a thread-local message on failure.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <set>

#include "eqs_internal.h"

namespace {

thread_local std::string g_last_error;

template <typename F>
int guarded(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const eqs::Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return EQS_ERR_ALLOC;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return EQS_ERR_INVALID_ARG;
    } catch (...) {
        g_last_error = "unknown failure";
        return EQS_ERR_INVALID_ARG;
    }
}

using eqs::fail;

void need(bool cond, const char* msg) {
    if (!cond) fail(EQS_ERR_INVALID_ARG, msg);
}

void bind_device(const eqs_ctx* c) { EQS_HIP(hipSetDevice(c->device)); }

void need_built(const eqs_ctx* c) {
    if (!c->built) fail(EQS_ERR_STATE, "eqs_build_preconditioner has not been called since the last set-up change");
}

int result_code(int rc, const char* what) {
    if (rc == EQS_ERR_NOT_CONVERGED) g_last_error = std::string(what) + ": iteration limit reached";
    else if (rc == EQS_ERR_BREAKDOWN) g_last_error = std::string(what) + ": CG breakdown";
    return rc;
}

}  // namespace

namespace eqs {
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace eqs

extern "C" {

const char* eqs_last_error(void) { return g_last_error.c_str(); }

int eqs_create(eqs_ctx** out, int device, void* hip_stream) {
    return guarded([&] {
        need(out != nullptr, "out is NULL");
        *out = nullptr;
        int n = 0;
        EQS_HIP(hipGetDeviceCount(&n));
        need(device >= 0 && device < n, "device id out of range");
        EQS_HIP(hipSetDevice(device));
        eqs::noalloc_scratch_init(device);  // once per device: the static scratch's address
        eqs_ctx* c = new eqs_ctx();
        c->device = device;
        c->stream = (hipStream_t)hip_stream;
        const char* g = std::getenv("EQS_USE_GRAPHS");  // "0" replays CG iterations as plain launches
        c->use_graphs = !(g && g[0] == '0');
        const char* tf = std::getenv("EQS_TUNE_FILE");  // tuning record: replayed if present, else written
        if (tf && tf[0]) {
            c->tune_file = tf;
            if (FILE* f = std::fopen(tf, "r")) {
                char buf[512];
                while (std::fgets(buf, sizeof buf, f)) {
                    std::string ln(buf);
                    while (!ln.empty() && (ln.back() == '\n' || ln.back() == '\r')) ln.pop_back();
                    const size_t tab = ln.find('\t');
                    if (tab != std::string::npos) c->tune_replay[ln.substr(0, tab)] = ln.substr(tab + 1);
                }
                std::fclose(f);
            }
        }
        const char* at = std::getenv("EQS_AUTOTUNE");  // "0" keeps the rule-based operator layouts
        c->autotune = !(at && at[0] == '0');
        const char* i16 = std::getenv("EQS_INDEX16");
        c->index16 = !(i16 && i16[0] == '0');
        const char* tv = std::getenv("EQS_TUNE_LOG");  // "all": list every layout candidate's time
        c->tune_verbose = tv && std::string(tv) == "all";
        const char* fo = std::getenv("EQS_FOLD");  // "0": the plain V-cycle (no folded operators)
        c->fold = !(fo && fo[0] == '0');
        // test knobs: "1" runs the element pass with each block's own LDS stride;
        // "1" rejects the first true-residual check of every solve (restart path)
        const char* kg = std::getenv("EQS_KX_GENERIC");
        c->kx_generic = kg && kg[0] == '1';
        const char* rj = std::getenv("EQS_TEST_REJECT_CHECK");
        c->test_reject_first = rj && rj[0] == '1';
        // "sell1", "sell2", "sell4", "sell8" or "csr": every AMG operator below
        // the finest level in that layout; "sell1s" etc. also sort the rows of
        // the operators used only in products (tests compare the layouts)
        // EQS_UNROLL (4, 8 or 16): with EQS_LAYOUT's SELL layouts, the group
        // size of every operator below the finest level
        const char* un = std::getenv("EQS_UNROLL");
        if (un && un[0]) {
            const std::string v(un);
            if (v == "4") c->force_unroll = 4;
            else if (v == "8") c->force_unroll = 8;
            else if (v == "16") c->force_unroll = 16;
            else {
                delete c;
                need(false, "EQS_UNROLL must be 4, 8 or 16");
            }
        }
        const char* lay = std::getenv("EQS_LAYOUT");
        if (lay && lay[0]) {
            const std::string v(lay);
            const bool srt = v.size() == 6 && v.compare(0, 4, "sell") == 0 && v[5] == 's';
            const std::string base = srt ? v.substr(0, 5) : v;
            c->force_sorted = srt;
            if (base == "sell1") c->force_layout = 1;
            else if (base == "sell2") c->force_layout = 2;
            else if (base == "sell4") c->force_layout = 4;
            else if (base == "sell8") c->force_layout = 8;
            else if (v == "csr") c->force_layout = 0;
            else {
                delete c;
                need(false, "EQS_LAYOUT must be sell1, sell2, sell4, sell8 (optionally with s: rows sorted) or csr");
            }
        }
        *out = c;
        return EQS_OK;
    });
}

int eqs_destroy(eqs_ctx* ctx) {
    return guarded([&] {
        if (!ctx) return EQS_OK;
        (void)hipSetDevice(ctx->device);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        else (void)hipDeviceSynchronize();
        eqs::free_device(ctx);
        eqs::prof_release(ctx);
        eqs::guess_release(ctx);
        delete ctx;
        return EQS_OK;
    });
}

static int set_mesh(eqs_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets, int npe) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        need(n_nodes >= 4 && n_nodes < INT32_MAX, "n_nodes must be in [4, 2^31)");
        need(n_tets >= 1 && n_tets < INT32_MAX, "n_tets must be in [1, 2^31)");
        need(xyz != nullptr && tets != nullptr, "xyz or tets is NULL");
        for (int64_t k = 0; k < npe * n_tets; ++k)
            need(tets[k] >= 0 && tets[k] < n_nodes, "tet node id out of range");
        bind_device(c);
        eqs::free_device(c);
        c->n_nodes = n_nodes;
        c->n_tets = n_tets;
        c->npe = npe;
        c->xyz.assign(xyz, xyz + 3 * n_nodes);
        c->tets.assign(tets, tets + npe * n_tets);
        c->have_mesh = true;
        c->inst_node_off.clear();
        c->inst_tet_off.clear();
        c->have_mat = c->have_dir = false;
        c->mats.clear();
        c->tet_mat.clear();
        c->dir_nodes.clear();
        c->dir_drive.clear();
        c->drives.clear();
        return EQS_OK;
    });
}

int eqs_set_mesh(eqs_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets) {
    return set_mesh(c, n_nodes, xyz, n_tets, tets, 4);
}

int eqs_set_mesh_p2(eqs_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets) {
    return set_mesh(c, n_nodes, xyz, n_tets, tets, 10);
}

int eqs_set_materials(eqs_ctx* c, int32_t n_mat, const eqs_material* mats, const int32_t* tet_mat) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        if (!c->have_mesh) fail(EQS_ERR_STATE, "eqs_set_mesh must come first");
        need(n_mat >= 1 && n_mat <= 65535, "n_mat must be in [1, 65535]");
        need(mats != nullptr && tet_mat != nullptr, "mats or tet_mat is NULL");
        for (int32_t m = 0; m < n_mat; ++m) {
            const eqs_material& s = mats[m];
            if (!std::isfinite(s.eps_r) || !std::isfinite(s.kappa0) || !std::isfinite(s.e_s) || !std::isfinite(s.alpha))
                fail(EQS_ERR_NONFINITE, "non-finite material parameter");
            need(s.eps_r > 0, "eps_r must be > 0");
            need(s.kappa0 >= 0, "kappa0 must be >= 0");
            if (s.nonlinear) need(s.e_s > 0 && s.alpha >= 0, "nonlinear material needs e_s > 0 and alpha >= 0");
        }
        for (int64_t e = 0; e < c->n_tets; ++e) need(tet_mat[e] >= 0 && tet_mat[e] < n_mat, "tet material id out of range");
        eqs::free_device(c);
        c->mats.assign(mats, mats + n_mat);
        c->tet_mat.assign(tet_mat, tet_mat + c->n_tets);
        c->have_mat = true;
        return EQS_OK;
    });
}

int eqs_set_dirichlet(eqs_ctx* c, int64_t n_d, const int32_t* nodes, const int32_t* drive_id, int32_t n_drive,
                      const eqs_drive* drives) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        if (!c->have_mesh) fail(EQS_ERR_STATE, "eqs_set_mesh must come first");
        need(n_d >= 1 && n_d < c->n_nodes, "need 1 <= n_d < n_nodes (at least one free node)");
        need(n_drive >= 1 && n_drive <= EQS_MAX_DRIVES, "n_drive must be in [1, EQS_MAX_DRIVES]");
        need(nodes && drive_id && drives, "NULL Dirichlet array");
        std::vector<char> seen(c->n_nodes, 0);
        for (int64_t k = 0; k < n_d; ++k) {
            need(nodes[k] >= 0 && nodes[k] < c->n_nodes, "Dirichlet node id out of range");
            need(!seen[nodes[k]], "Dirichlet node listed twice");
            seen[nodes[k]] = 1;
            need(drive_id[k] >= 0 && drive_id[k] < n_drive, "drive id out of range");
        }
        for (int32_t k = 0; k < n_drive; ++k)
            if (!std::isfinite(drives[k].amp) || !std::isfinite(drives[k].freq) || !std::isfinite(drives[k].phase))
                fail(EQS_ERR_NONFINITE, "non-finite drive parameter");
        eqs::free_device(c);
        c->dir_nodes.assign(nodes, nodes + n_d);
        c->dir_drive.assign(drive_id, drive_id + n_d);
        c->drives.assign(drives, drives + n_drive);
        c->have_dir = true;
        return EQS_OK;
    });
}

}  // extern "C"

namespace {
// Checkpoint layout: magic, version, the set-up's fingerprint, the step-level
// state (the last stage solution and its M-product), the start-vector state.
constexpr uint64_t kStateMagic = 0x3154504b43535145ull;  // "EQSCKPT1"
constexpr int32_t kStateVersion = 1;

void state_stream(eqs_ctx* c, eqs::StateWriter& w) {
    EQS_HIP(hipStreamSynchronize(c->stream));
    w.s = c->stream;
    const eqs_guess_params& g = c->guess.p;
    w.val(kStateMagic);
    w.val(kStateVersion);
    for (int64_t v : {c->n_nodes, c->n_tets, c->n_free, (int64_t)c->npe, c->nnz_M, (int64_t)c->amg.precision,
                      c->n_inst, (int64_t)g.kind, (int64_t)g.window, (int64_t)g.capacity, (int64_t)g.bf16})
        w.val(v);
    w.val((int32_t)c->have_Flast);
    w.val((int32_t)c->mx_of_F);
    w.dev(c->d_F, c->have_Flast ? (int64_t)sizeof(double) * c->n_free : 0);
    w.dev(c->d_mx, c->mx_of_F ? (int64_t)sizeof(double) * c->n_free : 0);
    eqs::guess_save_state(c, w);
}
}  // namespace

extern "C" {

int eqs_state_size(eqs_ctx* c, int64_t* bytes) {
    return guarded([&] {
        need(c != nullptr && bytes != nullptr, "NULL argument");
        need_built(c);
        bind_device(c);
        eqs::StateWriter w;  // counting only
        state_stream(c, w);
        *bytes = w.n;
        return EQS_OK;
    });
}

int eqs_state_save(eqs_ctx* c, void* buf, int64_t bytes) {
    return guarded([&] {
        need(c != nullptr && buf != nullptr, "NULL argument");
        need_built(c);
        bind_device(c);
        eqs::StateWriter w;
        w.buf = static_cast<char*>(buf);
        w.cap = bytes;
        state_stream(c, w);
        return EQS_OK;
    });
}

int eqs_state_load(eqs_ctx* c, const void* buf, int64_t bytes) {
    return guarded([&] {
        need(c != nullptr && buf != nullptr, "NULL argument");
        need_built(c);
        bind_device(c);
        EQS_HIP(hipStreamSynchronize(c->stream));
        eqs::StateReader r;
        r.buf = static_cast<const char*>(buf);
        r.cap = bytes;
        r.s = c->stream;
        const eqs_guess_params& g = c->guess.p;
        if (r.val<uint64_t>() != kStateMagic || r.val<int32_t>() != kStateVersion)
            eqs::fail(EQS_ERR_INVALID_ARG, "not a checkpoint of this library version");
        for (int64_t v : {c->n_nodes, c->n_tets, c->n_free, (int64_t)c->npe, c->nnz_M, (int64_t)c->amg.precision,
                          c->n_inst, (int64_t)g.kind, (int64_t)g.window, (int64_t)g.capacity, (int64_t)g.bf16})
            if (r.val<int64_t>() != v)
                eqs::fail(EQS_ERR_INVALID_ARG, "checkpoint of another set-up or start-vector setting");
        const bool have_F = r.val<int32_t>() != 0, have_mx = r.val<int32_t>() != 0;
        r.dev(c->d_F, have_F ? (int64_t)sizeof(double) * c->n_free : 0);
        r.dev(c->d_mx, have_mx ? (int64_t)sizeof(double) * c->n_free : 0);
        eqs::guess_load_state(c, r);
        if (r.n != bytes) eqs::fail(EQS_ERR_INVALID_ARG, "state buffer longer than its checkpoint");
        c->have_Flast = have_F;
        c->mx_of_F = have_mx;
        return EQS_OK;
    });
}

int eqs_set_deterministic(eqs_ctx* c, int32_t on) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        need(on == 0 || on == 1, "on must be 0 or 1");
        if (c->built && c->deterministic != (on != 0))
            fail(EQS_ERR_STATE, "set the deterministic element pass before eqs_build_preconditioner");
        c->deterministic = on != 0;
        return EQS_OK;
    });
}

int eqs_set_graph_iters(eqs_ctx* c, int32_t iters) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        need(iters >= 1 && iters <= EQS_MAX_GRAPH_ITERS, "iterations per graph must be in [1, EQS_MAX_GRAPH_ITERS]");
        c->graph_iters = iters;
        return EQS_OK;
    });
}

int eqs_build_preconditioner(eqs_ctx* c, const eqs_amg_params* p) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        if (!(c->have_mesh && c->have_mat && c->have_dir))
            fail(EQS_ERR_STATE, "mesh, materials and Dirichlet data must be set first");
        eqs_amg_params a{};
        if (p) a = *p;
        need(a.precision == EQS_PREC_FP64 || a.precision == EQS_PREC_FP32, "precision must be FP64 or FP32");
        if (a.coarse_max == 0) a.coarse_max = 512;
        if (a.max_levels == 0) a.max_levels = 12;
        // defaults measured on the 2.1M-DOF inclusion workload (CG iterations
        // per stage and stage rate over theta in [0.001, 0.25] and weights in [1, 1.75])
        if (a.theta == 0) a.theta = 0.02;
        if (a.jacobi_weight == 0) a.jacobi_weight = 1.5;
        if (a.smooth_weight == 0) a.smooth_weight = 4.0 / 3.0;
        need(a.flexible >= 0 && a.flexible <= 2, "flexible must be 0, 1 or 2");
        if (a.flexible == 0) a.flexible = (a.precision == EQS_PREC_FP32) ? 1 : 2;
        a.flexible = (a.flexible == 1) ? 1 : 0;  // stored as: 1 Polak-Ribiere, 0 Fletcher-Reeves
        need(a.coarse_max >= 1 && a.coarse_max <= 4096, "coarse_max must be in [1, 4096]");
        need(a.max_levels >= 1 && a.max_levels <= 16, "max_levels must be in [1, 16]");
        need(a.theta >= 0 && a.theta < 1, "theta must be in [0, 1)");
        need(a.jacobi_weight > 0 && a.jacobi_weight < 2 && a.smooth_weight > 0 && a.smooth_weight < 2,
             "weights must be in (0, 2)");
        bind_device(c);
        eqs::free_device(c);
        c->amg = a;
        eqs::validate_and_order(c);
        eqs::upload(c);
        EQS_HIP(hipDeviceSynchronize());
        c->built = true;
        return EQS_OK;
    });
}

int eqs_get_info(const eqs_ctx* c, eqs_info* info) {
    return guarded([&] {
        need(c != nullptr && info != nullptr, "NULL argument");
        eqs_info o{};
        o.n_nodes = c->n_nodes;
        o.n_tets = c->n_tets;
        o.n_free = c->built ? c->n_free : 0;
        o.nnz_M = c->nnz_M;
        o.precision = c->amg.precision;
        auto levels = [&](const auto& h) {
            o.n_levels = (int32_t)h.lv.size();
            for (size_t l = 0; l < h.lv.size() && l < 16; ++l) {
                o.level_rows[l] = h.lv[l].n;
                o.level_nnz[l] = h.lv[l].A.nnz;
                o.level_p_nnz[l] = h.lv[l].P.nnz;
                o.level_r_nnz[l] = h.lv[l].R.nnz;
            }
        };
        if (c->built) {
            if (c->amg.precision == EQS_PREC_FP32) levels(c->h32);
            else levels(c->h64);
        }
        o.device_bytes = c->device_bytes;
        o.workspace_bytes = c->ws_base ? c->ws_size : 0;
        o.workspace_used = c->ws_used;
        *info = o;
        return EQS_OK;
    });
}

int eqs_query(const eqs_ctx* c, int64_t* n_free, int64_t* ws_bytes) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        need_built(c);
        if (n_free) *n_free = c->n_free;
        if (ws_bytes) *ws_bytes = eqs::workspace_need(c);
        return EQS_OK;
    });
}

int eqs_set_workspace(eqs_ctx* c, void* dev, int64_t bytes) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        if (dev) {
            need(bytes > 0, "bytes must be > 0 with a workspace");
            need(((uintptr_t)dev & 255u) == 0, "the workspace must be 256-byte aligned");
        } else {
            need(bytes == 0, "bytes must be 0 without a workspace");
        }
        bind_device(c);
        if (dev) {
            hipPointerAttribute_t attr{};
            EQS_HIP(hipPointerGetAttributes(&attr, dev));
            need(attr.type == hipMemoryTypeDevice && attr.device == c->device,
                 "the workspace must be device memory on the context's device");
        }
        eqs::set_workspace(c, dev, bytes);
        return EQS_OK;
    });
}

int eqs_apply_K(eqs_ctx* c, double t, const double* x_dev, double* y_dev) {
    return guarded([&] {
        need(c != nullptr && x_dev != nullptr && y_dev != nullptr, "NULL argument");
        need(x_dev != y_dev, "x and y must not alias");
        need(std::isfinite(t), "t must be finite");
        need_built(c);
        bind_device(c);
        hipStream_t s = c->stream;
        eqs::launch_gather(s, x_dev, c->d_int_to_user, c->d_tmpN, c->n_free);
        eqs::launch_kx(s, false, c, c->d_tmpN, t, c->d_tmpN2);
        eqs::launch_scatter(s, c->d_tmpN2, c->d_int_to_user, y_dev, c->n_nodes);
        EQS_HIP(hipGetLastError());
        EQS_HIP(hipStreamSynchronize(s));
        return EQS_OK;
    });
}

int eqs_stage_rhs(eqs_ctx* c, double t, const double* y_free_dev, double* r_dev) {
    return guarded([&] {
        need(c != nullptr && y_free_dev != nullptr && r_dev != nullptr, "NULL argument");
        need(y_free_dev != r_dev, "y and r must not alias");
        need(std::isfinite(t), "t must be finite");
        need_built(c);
        bind_device(c);
        eqs::launch_kx(c->stream, true, c, y_free_dev, t, r_dev);
        EQS_HIP(hipGetLastError());
        EQS_HIP(hipStreamSynchronize(c->stream));
        return EQS_OK;
    });
}

int eqs_apply_M(eqs_ctx* c, const double* x_dev, double* y_dev) {
    return guarded([&] {
        need(c != nullptr && x_dev != nullptr && y_dev != nullptr, "NULL argument");
        need(x_dev != y_dev, "x and y must not alias");
        need_built(c);
        bind_device(c);
        eqs::launch_spmv64(c->stream, c->M, x_dev, y_dev);
        EQS_HIP(hipGetLastError());
        EQS_HIP(hipStreamSynchronize(c->stream));
        return EQS_OK;
    });
}

int eqs_apply_preconditioner(eqs_ctx* c, const double* r_dev, double* z_dev) {
    return guarded([&] {
        need(c != nullptr && r_dev != nullptr && z_dev != nullptr, "NULL argument");
        need(r_dev != z_dev, "r and z must not alias");
        need_built(c);
        bind_device(c);
        eqs::apply_preconditioner(c, r_dev, z_dev);
        return EQS_OK;
    });
}

int eqs_solve_M(eqs_ctx* c, const double* rhs_dev, double* y_dev, double rtol, int32_t maxit, eqs_solve_stats* st) {
    return guarded([&] {
        need(c != nullptr && rhs_dev != nullptr && y_dev != nullptr, "NULL argument");
        need(rhs_dev != y_dev, "rhs and y must not alias");
        need(std::isfinite(rtol) && rtol >= 0, "rtol must be finite and >= 0");
        need(maxit >= 0, "maxit must be >= 0");
        need_built(c);
        bind_device(c);
        std::fill(c->inst_iters.begin(), c->inst_iters.end(), 0);
        std::fill(c->inst_relres.begin(), c->inst_relres.end(), 0.0);
        return result_code(eqs::solve_M(c, rhs_dev, y_dev, rtol, maxit, st), "eqs_solve_M");
    });
}

int eqs_rkc_step(eqs_ctx* c, double t, double dt, int32_t s, double* x_dev, double rtol, int32_t maxit,
                 eqs_step_stats* st) {
    return guarded([&] {
        need(c != nullptr && x_dev != nullptr, "NULL argument");
        need(std::isfinite(t) && std::isfinite(dt) && dt > 0, "t must be finite and dt > 0");
        need(s >= 2 && s <= 256, "s must be in [2, 256]");
        need(std::isfinite(rtol) && rtol >= 0, "rtol must be finite and >= 0");
        need(maxit >= 0, "maxit must be >= 0");
        need_built(c);
        bind_device(c);
        return result_code(eqs::rkc_step(c, t, dt, s, x_dev, rtol, maxit, st), "eqs_rkc_step");
    });
}

int eqs_rkc_adaptive(eqs_ctx* c, double t0, double t_end, double* x_dev, double rtol, int32_t maxit,
                     const eqs_adapt_params* p, eqs_adapt_record* rec, int32_t cap, int32_t* n_rec,
                     eqs_adapt_stats* st) {
    return guarded([&] {
        need(c != nullptr && x_dev != nullptr && p != nullptr, "NULL argument");
        need(std::isfinite(t0) && std::isfinite(t_end) && t_end > t0, "need finite t0 < t_end");
        need(std::isfinite(rtol) && rtol >= 0, "rtol must be finite and >= 0");
        need(maxit >= 0, "maxit must be >= 0");
        need(std::isfinite(p->atol) && p->atol > 0, "atol must be > 0");
        need(std::isfinite(p->rtol) && p->rtol >= 0, "the error weight rtol must be >= 0");
        need(std::isfinite(p->tau0) && p->tau0 > 0, "tau0 must be > 0");
        need(std::isfinite(p->tau_min) && p->tau_min >= 0, "tau_min must be >= 0");
        need(std::isfinite(p->tau_max) && p->tau_max >= 0, "tau_max must be >= 0");
        need(p->s_max == 0 || (p->s_max >= 2 && p->s_max <= 256), "s_max must be 0 or in [2, 256]");
        need(p->max_attempts >= 0, "max_attempts must be >= 0");
        need(cap >= 0 && (cap == 0 || rec != nullptr), "rec must hold cap records");
        need_built(c);
        if (c->n_inst != 1) fail(EQS_ERR_STATE, "adaptive stepping needs a single instance");
        if (c->npe != 4) fail(EQS_ERR_STATE, "adaptive stepping is built for first-order tets");
        if (c->guess.p.kind != EQS_GUESS_PREVIOUS && c->guess.p.kind != EQS_GUESS_ZERO)
            fail(EQS_ERR_STATE, "adaptive stepping runs with the plain or the zero start vector");
        bind_device(c);
        return result_code(eqs::rkc_adaptive(c, t0, t_end, x_dev, rtol, maxit, *p, rec, cap, n_rec, st),
                           "eqs_rkc_adaptive");
    });
}

int eqs_set_instances(eqs_ctx* c, int32_t n_inst, const int64_t* node_off, const int64_t* tet_off) {
    return guarded([&] {
        need(c != nullptr && node_off != nullptr && tet_off != nullptr, "NULL argument");
        if (!c->have_mesh) fail(EQS_ERR_STATE, "eqs_set_mesh must come first");
        need(n_inst >= 1, "n_inst must be >= 1");
        need(node_off[0] == 0 && node_off[n_inst] == c->n_nodes, "node offsets must run from 0 to n_nodes");
        need(tet_off[0] == 0 && tet_off[n_inst] == c->n_tets, "tet offsets must run from 0 to n_tets");
        for (int32_t i = 0; i < n_inst; ++i)
            need(node_off[i + 1] > node_off[i] && tet_off[i + 1] > tet_off[i], "every instance needs nodes and tets");
        if (n_inst > 1 && c->guess.p.kind >= EQS_GUESS_GALERKIN)
            fail(EQS_ERR_STATE, "Galerkin and network start vectors need a single instance");
        bind_device(c);
        eqs::free_device(c);
        c->inst_node_off.assign(node_off, node_off + n_inst + 1);
        c->inst_tet_off.assign(tet_off, tet_off + n_inst + 1);
        return EQS_OK;
    });
}

int eqs_instance_stats(const eqs_ctx* c, int32_t n_inst, int64_t* iters, double* relres) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        if (!c->built) fail(EQS_ERR_STATE, "context not built");
        need(n_inst == (int32_t)c->n_inst, "n_inst does not match the context");
        for (int32_t i = 0; i < n_inst; ++i) {
            if (iters) iters[i] = c->inst_iters[i];
            if (relres) relres[i] = c->inst_relres[i];
        }
        return EQS_OK;
    });
}

int eqs_stage_iters(const eqs_ctx* c, int32_t* iters, int32_t cap, int32_t* n) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        need(cap >= 0, "cap must be >= 0");
        need(iters != nullptr || cap == 0, "iters is NULL");
        const int32_t m = (int32_t)c->stage_iters.size();
        for (int32_t k = 0; k < std::min(cap, m); ++k) iters[k] = c->stage_iters[k];
        if (n) *n = m;
        return EQS_OK;
    });
}

int eqs_set_guess(eqs_ctx* c, const eqs_guess_params* p) {
    return guarded([&] {
        need(c != nullptr && p != nullptr, "NULL argument");
        eqs_guess_params a = *p;
        need(a.kind >= EQS_GUESS_PREVIOUS && a.kind <= EQS_GUESS_MOR, "unknown guess kind");
        need(a.add_threshold >= 0, "add_threshold must be >= 0");
        if (a.window == 0) a.window = 16;
        if (a.capacity == 0) a.capacity = 2000;
        if (a.batch == 0) a.batch = 256;
        if (a.lr == 0) a.lr = 1e-3;
        need(a.window >= 2 && a.window <= 16, "window must be in [2, 16]");
        need(a.capacity >= 1 && a.capacity <= 100000, "capacity must be in [1, 100000]");
        need(a.warmup >= 0, "warmup must be >= 0");
        need(a.batch >= 1 && a.batch <= 256, "batch must be in [1, 256]");
        need(std::isfinite(a.lr) && a.lr > 0, "lr must be > 0");
        bind_device(c);
        c->guess.init.clear();
        if (a.kind == EQS_GUESS_MLP) {
            need(a.init != nullptr, "the MLP guess needs initial parameters");
            for (int i = 0; i < EQS_MLP_NPARAM; ++i)
                if (!std::isfinite(a.init[i])) fail(EQS_ERR_NONFINITE, "non-finite network parameter");
            c->guess.init.assign(a.init, a.init + EQS_MLP_NPARAM);
        }
        a.init = nullptr;
        if (a.kind >= EQS_GUESS_GALERKIN && c->inst_node_off.size() > 2)
            fail(EQS_ERR_STATE, "Galerkin and network start vectors need a single instance");
        eqs::guess_configure(c, a);
        return EQS_OK;
    });
}

// [a, a + na) and [b, b + nb) share an element
static bool overlaps(const double* a, int64_t na, const double* b, int64_t nb) {
    const uintptr_t a0 = (uintptr_t)a, a1 = a0 + sizeof(double) * (uintptr_t)na;
    const uintptr_t b0 = (uintptr_t)b, b1 = b0 + sizeof(double) * (uintptr_t)nb;
    return a0 < b1 && b0 < a1;
}

int eqs_galerkin_start(eqs_ctx* c, int32_t k, const double* S_dev, const double* R_dev, const double* r_dev,
                       double* x0_dev, int32_t* m_out) {
    return guarded([&] {
        need(c != nullptr && S_dev != nullptr && R_dev != nullptr && r_dev != nullptr && x0_dev != nullptr,
             "NULL argument");
        need(k >= 1 && k <= 16, "k must be in [1, 16]");
        need_built(c);
        const int64_t NF = c->n_free;
        need(NF > 0, "no free nodes");
        need(!overlaps(x0_dev, NF, S_dev, (int64_t)k * NF) && !overlaps(x0_dev, NF, R_dev, (int64_t)k * NF) &&
                 !overlaps(x0_dev, NF, r_dev, NF),
             "x0 must not overlap S, R or r");
        bind_device(c);
        const int m = eqs::guess_galerkin_explicit(c, k, S_dev, R_dev, r_dev, x0_dev);
        EQS_HIP(hipStreamSynchronize(c->stream));
        if (m_out) *m_out = m;
        return EQS_OK;
    });
}

int eqs_galerkin_start_noalloc(eqs_ctx* c, int32_t k, const double* S_dev, const double* R_dev,
                               const double* r_dev, double* x0_dev, int32_t* m_out) {
    return guarded([&] {
        need(c != nullptr && S_dev != nullptr && R_dev != nullptr && r_dev != nullptr && x0_dev != nullptr,
             "NULL argument");
        need(k >= 1 && k <= 16, "k must be in [1, 16]: the static scratch holds the dots of at most 16 columns");
        need_built(c);
        const int64_t NF = c->n_free;
        need(NF > 0, "no free nodes");
        need(!overlaps(x0_dev, NF, S_dev, (int64_t)k * NF) && !overlaps(x0_dev, NF, R_dev, (int64_t)k * NF) &&
                 !overlaps(x0_dev, NF, r_dev, NF),
             "x0 must not overlap S, R or r");
        bind_device(c);
        double* base = eqs::noalloc_scratch(c->device);
        const int m = eqs::guess_galerkin_explicit(c, k, S_dev, R_dev, r_dev, x0_dev, base,
                                                   base + eqs::kNoAllocPartDoubles);
        EQS_HIP(hipStreamSynchronize(c->stream));
        if (m_out) *m_out = m;
        return EQS_OK;
    });
}

int eqs_mlp_create(eqs_mlp** out, int device, void* hip_stream, const float* params, int32_t bf16, double lr) {
    return guarded([&] {
        need(out != nullptr && params != nullptr, "NULL argument");
        *out = nullptr;
        need(std::isfinite(lr) && lr > 0, "lr must be > 0");
        for (int i = 0; i < EQS_MLP_NPARAM; ++i)
            if (!std::isfinite(params[i])) fail(EQS_ERR_NONFINITE, "non-finite network parameter");
        int n = 0;
        EQS_HIP(hipGetDeviceCount(&n));
        need(device >= 0 && device < n, "device id out of range");
        EQS_HIP(hipSetDevice(device));
        *out = eqs::mlp_create(device, (hipStream_t)hip_stream, params, bf16, lr);
        return EQS_OK;
    });
}

int eqs_mlp_destroy(eqs_mlp* net) {
    return guarded([&] {
        eqs::mlp_destroy(net);
        return EQS_OK;
    });
}

int eqs_mlp_forward(eqs_mlp* net, const float* x_dev, float* y_dev, int32_t batch) {
    return guarded([&] {
        need(net && x_dev && y_dev, "NULL argument");
        need(batch >= 1, "batch must be >= 1");
        eqs::mlp_forward(net, x_dev, y_dev, batch);
        EQS_HIP(hipGetLastError());
        return EQS_OK;
    });
}

int eqs_mlp_train_step(eqs_mlp* net, const float* x_dev, const float* t_dev, int32_t batch, float* loss) {
    return guarded([&] {
        need(net && x_dev && t_dev, "NULL argument");
        need(batch >= 1 && batch <= 64, "batch must be in [1, 64]");
        eqs::mlp_train(net, x_dev, t_dev, batch);
        EQS_HIP(hipGetLastError());
        const float l = eqs::mlp_last_loss(net);
        if (loss) *loss = l;
        return EQS_OK;
    });
}

int eqs_mlp_get(eqs_mlp* net, float* params_host, float* grad_host) {
    return guarded([&] {
        need(net != nullptr, "NULL argument");
        eqs::mlp_get(net, params_host, grad_host);
        return EQS_OK;
    });
}

int eqs_describe(const eqs_ctx* c, char* buf, int64_t cap, int64_t* needed) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        std::string d;
        char line[200];
        std::snprintf(line, sizeof line, "nodes %lld tets %lld (%d nodes each) free %lld nnz(M) %lld precision %s built %d\n",
                      (long long)c->n_nodes, (long long)c->n_tets, c->npe, (long long)c->n_free, (long long)c->nnz_M,
                      c->amg.precision == EQS_PREC_FP32 ? "fp32" : "fp64", (int)c->built);
        d += line;
        std::snprintf(line, sizeof line,
                      "element blocks %lld of %d tets, block nodes %lld (max %d), graphs %d, autotune %d%s\n",
                      (long long)c->n_blocks, eqs::kTetBlock * c->tet_tpt, (long long)c->n_block_nodes,
                      c->max_block_nodes, (int)c->use_graphs, (int)c->autotune,
                      c->kx_generic ? ", per-block LDS stride" : c->deterministic ? ", deterministic sums" : "");
        d += line;
        d += c->tune_log;
        if (needed) *needed = (int64_t)d.size() + 1;
        if (buf && cap > 0) {
            const size_t n = std::min<size_t>((size_t)cap - 1, d.size());
            std::memcpy(buf, d.data(), n);
            buf[n] = 0;
        }
        return EQS_OK;
    });
}

int eqs_profile_enable_impl(eqs_ctx* c, uint32_t mask);
int eqs_profile_read_impl(eqs_ctx* c, int32_t cls, int64_t* launches, double* total_ms);

int eqs_profile_enable(eqs_ctx* c, uint32_t class_mask) {
    return guarded([&] {
        need(c != nullptr, "ctx is NULL");
        bind_device(c);
        return eqs_profile_enable_impl(c, class_mask);
    });
}

int eqs_profile_read(eqs_ctx* c, int32_t kclass, int64_t* launches, double* total_ms) {
    return guarded([&] {
        need(c != nullptr && launches != nullptr && total_ms != nullptr, "NULL argument");
        need(kclass >= 0 && kclass < EQS_KCLASS_COUNT, "kernel class out of range");
        bind_device(c);
        return eqs_profile_read_impl(c, kclass, launches, total_ms);
    });
}

}  // extern "C"
