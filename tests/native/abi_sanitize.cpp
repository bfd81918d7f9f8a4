// Sanitizer driver of the library: its host code runs under AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only; the device code is the same as in
// the normal build). Two modes:
//   host  the set-up algorithms that need no GPU - validation and ordering of
//         the mesh, assembly of M on the free nodes (eq. (2)), the smoothed-
//         aggregation hierarchy, the RKC coefficients (Sec. II) - and the C ABI's
//         argument checks that fail before any HIP call;
//   abi   every C ABI entry point end to end on device 0: first- and second-
//         order meshes, both precisions, stepping with every start-vector kind
//         (Sec. IV), adaptive stepping, checkpoints, workspaces, instances,
//         batches, the network, timing, and the error paths; the host arrays of
//         the set-up calls are freed as soon as each call returns (the library
//         keeps copies, never the caller's pointers).
// Prints "SANITIZE OK <mode>" and exits 0 when every check held; a check that
// fails exits 1, and a sanitizer finding aborts the process.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "eqs.h"
#include "eqs_internal.h"

namespace {

int g_checks = 0;

void check(bool ok, const char* what, int line) {
    ++g_checks;
    if (!ok) {
        std::fprintf(stderr, "check failed (line %d): %s; last error: %s\n", line, what, eqs_last_error());
        std::exit(1);
    }
}
#define CHECK(cond) check((cond), #cond, __LINE__)
#define OK(call) check((call) == EQS_OK, #call, __LINE__)
// the call fails with `code` and leaves a message
#define FAILS(call, code)                                                        \
    do {                                                                         \
        const int rc_ = (call);                                                  \
        check(rc_ == (code), #call " returns " #code, __LINE__);                 \
        check(eqs_last_error()[0] != '\0', #call " leaves a message", __LINE__); \
    } while (0)
#define HIPOK(call) check((call) == hipSuccess, #call, __LINE__)

// progress line before each part, so that the log names the part a failure is in
void part(const char* name) {
    std::printf("[sanitize] %s\n", name);
    std::fflush(stdout);
}

// ------------------------------------------------------------- inputs
// The n^3 Kuhn cube mesh of [0,1]^3: six tets per sub-cube, one per order of
// the three axis steps from its lowest to its highest corner; with p2 the
// midpoints of the edges are nodes too (the half-step lattice) and a tet lists
// its vertices, then the midpoints of (0,1), (0,2), (0,3), (1,2), (1,3), (2,3).
struct Mesh {
    int64_t n_nodes = 0, n_tets = 0;
    int npe = 4;
    std::vector<double> xyz;
    std::vector<int32_t> tets;
};

Mesh kuhn_mesh(int n, bool p2) {
    static const int orders[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int edges[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    const int q = p2 ? 2 : 1, m = q * n + 1;
    Mesh M;
    M.npe = p2 ? 10 : 4;
    M.n_nodes = (int64_t)m * m * m;
    M.n_tets = 6 * (int64_t)n * n * n;
    M.xyz.resize(3 * M.n_nodes);
    for (int k = 0; k < m; ++k)
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) {
                double* p = &M.xyz[3 * (i + (int64_t)m * (j + (int64_t)m * k))];
                p[0] = (double)i / (m - 1);
                p[1] = (double)j / (m - 1);
                p[2] = (double)k / (m - 1);
            }
    for (int ck = 0; ck < n; ++ck)
        for (int cj = 0; cj < n; ++cj)
            for (int ci = 0; ci < n; ++ci)
                for (const auto& ord : orders) {
                    int off[4][3] = {};
                    for (int v = 1; v < 4; ++v) {
                        for (int d = 0; d < 3; ++d) off[v][d] = off[v - 1][d];
                        off[v][ord[v - 1]] = 1;
                    }
                    auto id = [&](int a, int b, int c) {
                        return (int32_t)((q * ci + a) + m * ((q * cj + b) + m * (q * ck + c)));
                    };
                    for (int v = 0; v < 4; ++v) M.tets.push_back(id(q * off[v][0], q * off[v][1], q * off[v][2]));
                    if (p2)
                        for (const auto& e : edges)
                            M.tets.push_back(id(off[e[0]][0] + off[e[1]][0], off[e[0]][1] + off[e[1]][1],
                                                off[e[0]][2] + off[e[1]][2]));
                }
    return M;
}

// Two meshes side by side as one (the batched form's concatenation).
Mesh concat(const Mesh& a, const Mesh& b) {
    Mesh M = a;
    M.n_nodes += b.n_nodes;
    M.n_tets += b.n_tets;
    for (int64_t i = 0; i < b.n_nodes; ++i) {
        M.xyz.push_back(b.xyz[3 * i] + 2.0);  // shifted along x, away from the first
        M.xyz.push_back(b.xyz[3 * i + 1]);
        M.xyz.push_back(b.xyz[3 * i + 2]);
    }
    for (int32_t v : b.tets) M.tets.push_back(v + (int32_t)a.n_nodes);
    return M;
}

// The slab problem: a linear host (eps_r 4, kappa0 1e-12) with a varistor
// slab 0.4 < z < 0.6 (eps_r 12, kappa0 1e-10, e_s 0.5, alpha 10); the bottom
// face grounded, the top face driven by amp sin(2 pi 50 t).
struct Inputs {
    std::vector<eqs_material> mats;
    std::vector<int32_t> tet_mat, dir_nodes, dir_drive;
    std::vector<eqs_drive> drives;
};

Inputs slab_inputs(const Mesh& M, double amp) {
    Inputs in;
    in.mats = {{4.0, 1e-12, 1.0, 0.0, 0, 0}, {12.0, 1e-10, 0.5, 10.0, 1, 0}};
    for (int64_t e = 0; e < M.n_tets; ++e) {
        double cz = 0;
        for (int a = 0; a < 4; ++a) cz += 0.25 * M.xyz[3 * (int64_t)M.tets[M.npe * e + a] + 2];
        in.tet_mat.push_back(cz > 0.4 && cz < 0.6 ? 1 : 0);
    }
    for (int64_t i = 0; i < M.n_nodes; ++i) {
        const double z = M.xyz[3 * i + 2];
        if (z == 0.0 || z == 1.0) {
            in.dir_nodes.push_back((int32_t)i);
            in.dir_drive.push_back(z == 0.0 ? 0 : 1);
        }
    }
    in.drives = {{0.0, 0.0, 0.0}, {amp, 50.0, 0.0}};
    return in;
}

// A heap copy of a host array, released as soon as the call that reads it
// returns: the library copies host arrays, so a pointer it kept would be a
// use after free that AddressSanitizer reports.
template <typename T>
struct Transient {
    T* p;
    explicit Transient(const std::vector<T>& v) : p(new T[std::max<size_t>(v.size(), 1)]) {
        std::copy(v.begin(), v.end(), p);
    }
    ~Transient() { delete[] p; }
    Transient(const Transient&) = delete;
    Transient& operator=(const Transient&) = delete;
};

void set_inputs(eqs_ctx* c, const Mesh& M, const Inputs& in) {
    {
        Transient<double> xyz(M.xyz);
        Transient<int32_t> tets(M.tets);
        OK(M.npe == 4 ? eqs_set_mesh(c, M.n_nodes, xyz.p, M.n_tets, tets.p)
                      : eqs_set_mesh_p2(c, M.n_nodes, xyz.p, M.n_tets, tets.p));
    }
    {
        Transient<eqs_material> mats(in.mats);
        Transient<int32_t> tet_mat(in.tet_mat);
        OK(eqs_set_materials(c, (int32_t)in.mats.size(), mats.p, tet_mat.p));
    }
    Transient<int32_t> nodes(in.dir_nodes), drive(in.dir_drive);
    Transient<eqs_drive> drives(in.drives);
    OK(eqs_set_dirichlet(c, (int64_t)in.dir_nodes.size(), nodes.p, drive.p, (int32_t)in.drives.size(), drives.p));
}

// A fixed pseudo-random sequence (SplitMix64) for test vectors and weights.
struct Rng {
    uint64_t s;
    double uniform() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return (double)((z ^ (z >> 31)) >> 11) * 0x1.0p-53;
    }
};

// ---------------------------------------------------------- host mode
void run_host() {
    using namespace eqs;
    // argument checks that fail before the library touches the GPU
    eqs_ctx* none = nullptr;
    FAILS(eqs_create(nullptr, 0, nullptr), EQS_ERR_INVALID_ARG);
    OK(eqs_destroy(nullptr));
    FAILS(eqs_set_mesh(none, 4, nullptr, 1, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_set_mesh_p2(none, 4, nullptr, 1, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_set_materials(none, 1, nullptr, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_set_dirichlet(none, 1, nullptr, nullptr, 1, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_build_preconditioner(none, nullptr), EQS_ERR_INVALID_ARG);
    eqs_info info{};
    FAILS(eqs_get_info(none, &info), EQS_ERR_INVALID_ARG);
    FAILS(eqs_query(none, nullptr, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_rkc_step(none, 0.0, 1e-4, 8, nullptr, 1e-8, 10, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_solve_M(none, nullptr, nullptr, 1e-8, 10, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_set_graph_iters(none, 1), EQS_ERR_INVALID_ARG);
    FAILS(eqs_describe(none, nullptr, 0, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_stage_iters(none, nullptr, 0, nullptr), EQS_ERR_INVALID_ARG);
    OK(eqs_batch_destroy(nullptr));
    FAILS(eqs_mlp_create(nullptr, 0, nullptr, nullptr, 1, 1e-3), EQS_ERR_INVALID_ARG);

    // set-up algorithms on a context filled by hand (the C ABI's setters bind the device first)
    for (int p2 = 0; p2 < 2; ++p2) {
        const Mesh M = kuhn_mesh(p2 ? 4 : 7, p2 != 0);
        const Inputs in = slab_inputs(M, 3.0);
        eqs_ctx* c = new eqs_ctx();
        c->n_nodes = M.n_nodes;
        c->n_tets = M.n_tets;
        c->npe = M.npe;
        c->xyz = M.xyz;
        c->tets = M.tets;
        c->mats = in.mats;
        c->tet_mat = in.tet_mat;
        c->dir_nodes = in.dir_nodes;
        c->dir_drive = in.dir_drive;
        c->drives = in.drives;
        c->have_mesh = c->have_mat = c->have_dir = true;
        validate_and_order(c);
        CHECK(c->n_free == M.n_nodes - (int64_t)in.dir_nodes.size());
        CHECK(c->n_inst == 1 && c->inst_row_off[1] == c->n_free);

        const Csr<double> A = assemble_M_free(c);
        CHECK(A.n_rows == c->n_free && A.n_cols == c->n_free);
        // symmetric, positive diagonal
        double amax = 0, asym = 0;
        for (int32_t i = 0; i < A.n_rows; ++i)
            for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                const int32_t j = A.col[k];
                CHECK(j >= 0 && j < A.n_cols);
                amax = std::max(amax, std::fabs(A.val[k]));
                if (j == i) CHECK(A.val[k] > 0);
                double aji = 0;
                for (int32_t kk = A.ptr[j]; kk < A.ptr[j + 1]; ++kk)
                    if (A.col[kk] == i) aji = A.val[kk];
                asym = std::max(asym, std::fabs(A.val[k] - aji));
            }
        CHECK(asym <= 1e-14 * amax);

        eqs_amg_params p{};
        p.coarse_max = 64;  // several levels on these small meshes
        p.max_levels = 12;
        p.theta = 0.02;
        p.jacobi_weight = 1.5;
        p.smooth_weight = 4.0 / 3.0;
        const AmgHost h = build_sa_amg(A, p);
        CHECK(!h.A.empty() && h.A[0].n_rows == A.n_rows);
        for (size_t l = 0; l + 1 < h.A.size(); ++l) {
            CHECK(h.P[l].n_rows == h.A[l].n_rows && h.P[l].n_cols == h.A[l + 1].n_rows);
            CHECK(h.A[l + 1].n_rows < h.A[l].n_rows);
        }
        // the coarsest operator's dense inverse (column-major)
        const Csr<double>& C = h.A.back();
        const int32_t nc = C.n_rows;
        CHECK((int64_t)h.coarse_inv.size() == (int64_t)nc * nc);
        double worst = 0;
        for (int32_t j = 0; j < nc; ++j)
            for (int32_t i = 0; i < nc; ++i) {
                double s = 0;  // (C X)_ij
                for (int32_t k = C.ptr[i]; k < C.ptr[i + 1]; ++k) s += C.val[k] * h.coarse_inv[(int64_t)j * nc + C.col[k]];
                worst = std::max(worst, std::fabs(s - (i == j ? 1.0 : 0.0)));
            }
        CHECK(worst <= 1e-8);
        std::printf("host: %s mesh, %lld free nodes, nnz(M) %lld, %zu AMG levels, coarsest %d rows\n",
                    p2 ? "second-order" : "first-order", (long long)c->n_free, (long long)A.nnz(), h.A.size(), nc);

        // a flat tet and an instance without Dirichlet nodes are rejected
        c->xyz[3 * (int64_t)c->tets[3] + 0] = c->xyz[3 * (int64_t)c->tets[0] + 0];
        c->xyz[3 * (int64_t)c->tets[3] + 1] = c->xyz[3 * (int64_t)c->tets[0] + 1];
        c->xyz[3 * (int64_t)c->tets[3] + 2] = c->xyz[3 * (int64_t)c->tets[0] + 2];
        int code = 0;
        try {
            validate_and_order(c);
        } catch (const Error& e) {
            code = e.code;
        }
        CHECK(code == EQS_ERR_INVALID_ARG);
        c->xyz = M.xyz;
        c->dir_nodes.clear();
        c->dir_drive.clear();
        code = 0;
        try {
            validate_and_order(c);
        } catch (const Error& e) {
            code = e.code;
        }
        CHECK(code == EQS_ERR_INVALID_ARG);
        delete c;
    }

    // instances side by side: their free rows are contiguous per instance, and
    // a tet across two instances or a small instance is rejected
    {
        const Mesh A8 = kuhn_mesh(8, false), A7 = kuhn_mesh(7, false);
        const Mesh B = concat(A8, A7);
        const Inputs in = slab_inputs(B, 1.0);
        auto fill = [&](eqs_ctx* c, const Mesh& m, int64_t split_node, int64_t split_tet) {
            c->n_nodes = m.n_nodes;
            c->n_tets = m.n_tets;
            c->npe = 4;
            c->xyz = m.xyz;
            c->tets = m.tets;
            c->mats = in.mats;
            c->tet_mat.assign(m.n_tets, 0);
            c->dir_nodes = in.dir_nodes;
            c->dir_drive = in.dir_drive;
            c->drives = in.drives;
            c->inst_node_off = {0, split_node, m.n_nodes};
            c->inst_tet_off = {0, split_tet, m.n_tets};
            c->have_mesh = c->have_mat = c->have_dir = true;
        };
        auto code_of = [](eqs_ctx* c) {
            try {
                validate_and_order(c);
            } catch (const Error& e) {
                return e.code;
            }
            return 0;
        };
        eqs_ctx* c = new eqs_ctx();
        fill(c, B, A8.n_nodes, A8.n_tets);
        CHECK(code_of(c) == 0);
        CHECK(c->n_inst == 2 && c->inst_row_off[2] == c->n_free);
        const int64_t nd8 = 2 * 81;  // bottom and top faces of the 8^3 mesh
        CHECK(c->inst_row_off[1] == A8.n_nodes - nd8);
        for (int64_t k = 0; k < c->n_free; ++k) {
            const int32_t u = c->int_to_user[k];
            CHECK((k < c->inst_row_off[1]) == (u < A8.n_nodes));
            if (k > 0) CHECK(u > c->int_to_user[k - 1]);
        }
        // the hierarchy of the block-diagonal M keeps the instances apart: every
        // prolongator column and every coarse row belongs to one instance
        {
            const Csr<double> A = assemble_M_free(c);
            eqs_amg_params p{};
            p.coarse_max = 32;
            p.max_levels = 12;
            p.theta = 0.02;
            p.jacobi_weight = 1.5;
            p.smooth_weight = 4.0 / 3.0;
            const AmgHost h = build_sa_amg(A, p);
            CHECK(h.A.size() >= 3);
            std::vector<int> inst(A.n_rows);
            for (int32_t i = 0; i < A.n_rows; ++i) inst[i] = i < c->inst_row_off[1] ? 0 : 1;
            for (size_t l = 0; l + 1 < h.A.size(); ++l) {
                const Csr<double>& P = h.P[l];
                std::vector<int> next(P.n_cols, -1);
                for (int32_t i = 0; i < P.n_rows; ++i)
                    for (int32_t k = P.ptr[i]; k < P.ptr[i + 1]; ++k) {
                        int& v = next[P.col[k]];
                        CHECK(v < 0 || v == inst[i]);
                        v = inst[i];
                    }
                for (int v : next) CHECK(v >= 0);
                const Csr<double>& Ac = h.A[l + 1];
                for (int32_t i = 0; i < Ac.n_rows; ++i)
                    for (int32_t k = Ac.ptr[i]; k < Ac.ptr[i + 1]; ++k) CHECK(next[Ac.col[k]] == next[i]);
                inst = next;
            }
        }
        // the last tet of the first instance moved into the second one
        fill(c, B, A8.n_nodes, A8.n_tets - 1);
        CHECK(code_of(c) == EQS_ERR_INVALID_ARG);
        delete c;
        // fewer than 256 free nodes in an instance
        const Mesh A4 = kuhn_mesh(4, false);
        const Mesh S = concat(A8, A4);
        c = new eqs_ctx();
        fill(c, S, A8.n_nodes, A8.n_tets);
        c->dir_nodes = slab_inputs(S, 1.0).dir_nodes;
        c->dir_drive = slab_inputs(S, 1.0).dir_drive;
        c->tet_mat.assign(S.n_tets, 0);
        CHECK(code_of(c) == EQS_ERR_INVALID_ARG);
        delete c;
    }

    // RKC coefficients: the last stage ends at the step's end, and the
    // stability boundary grows with s
    double prev = 0;
    for (int s : {2, 3, 8, 16, 64, 256}) {
        std::vector<double> mu, nu, mut, gmt, cc;
        rkc_coefficients(s, mu, nu, mut, gmt, cc);
        CHECK((int)cc.size() >= s && std::fabs(cc[s] - 1.0) <= 1e-12);
        const double b = rkc_beta(s);
        CHECK(std::isfinite(b) && b > prev);
        prev = b;
    }
}

// ----------------------------------------------------------- abi mode
struct Dev {
    std::vector<void*> p;
    double* vec(int64_t n) {
        void* q = nullptr;
        HIPOK(hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(double)));
        HIPOK(hipMemset(q, 0, (size_t)std::max<int64_t>(n, 1) * sizeof(double)));
        p.push_back(q);
        return (double*)q;
    }
    ~Dev() {
        for (void* q : p) (void)hipFree(q);
    }
};

std::vector<double> to_host(const double* d, int64_t n) {
    std::vector<double> h(n);
    HIPOK(hipMemcpy(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost));
    return h;
}

bool all_finite(const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

void steps(eqs_ctx* c, double* x, int n, double t0, double tau, int s, double rtol) {
    for (int k = 0; k < n; ++k) {
        eqs_step_stats st{};
        OK(eqs_rkc_step(c, t0 + k * tau, tau, s, x, rtol, 500, &st));
        CHECK(st.stages == s && st.not_converged == 0 && st.max_relres <= 1.01 * rtol);
        // the per-stage counts, read into a buffer shorter than s first
        std::vector<int32_t> its(s, -1);
        int32_t m = -1;
        OK(eqs_stage_iters(c, its.data(), s - 1, &m));
        CHECK(m == s && its[s - 1] == -1);
        OK(eqs_stage_iters(c, its.data(), s, nullptr));
        int32_t sum = 0, mx = 0;
        for (int32_t v : its) {
            sum += v;
            mx = std::max(mx, v);
        }
        CHECK(sum == st.total_iters && mx == st.max_iters);
    }
}

void run_abi() {
    hipStream_t stream = nullptr;
    HIPOK(hipStreamCreate(&stream));
    Dev dev;
    const double tau = 1e-4, rtol = 1e-10;
    const int s = 8;

    // --- first-order slab: build, products, solve, stepping, description
    part("first-order slab: build, products, solve, steps");
    const Mesh M8 = kuhn_mesh(8, false);
    const Inputs in8 = slab_inputs(M8, 3.0);
    double* x = dev.vec(M8.n_nodes);
    double* y = dev.vec(M8.n_nodes);
    eqs_ctx* c = nullptr;
    OK(eqs_create(&c, 0, stream));
    FAILS(eqs_build_preconditioner(c, nullptr), EQS_ERR_STATE);
    set_inputs(c, M8, in8);
    FAILS(eqs_apply_K(c, 0.0, nullptr, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_apply_K(c, 0.0, x, y), EQS_ERR_STATE);
    OK(eqs_set_graph_iters(c, 2));
    FAILS(eqs_set_graph_iters(c, 0), EQS_ERR_INVALID_ARG);
    FAILS(eqs_set_graph_iters(c, EQS_MAX_GRAPH_ITERS + 1), EQS_ERR_INVALID_ARG);
    OK(eqs_build_preconditioner(c, nullptr));
    eqs_info info{};
    OK(eqs_get_info(c, &info));
    CHECK(info.n_nodes == M8.n_nodes && info.n_levels >= 1);
    const int64_t nf = info.n_free;
    int64_t need = 0, ws = 0, nf2 = 0;
    char small[16];
    OK(eqs_describe(c, small, sizeof small, &need));
    CHECK(need > (int64_t)sizeof small && std::strlen(small) == sizeof small - 1);
    std::vector<char> text(need);
    OK(eqs_describe(c, text.data(), need, nullptr));
    CHECK((int64_t)std::strlen(text.data()) == need - 1);
    OK(eqs_query(c, &nf2, &ws));
    CHECK(nf2 == nf && ws > 0);

    double* r = dev.vec(nf);
    double* z = dev.vec(nf);
    double* w = dev.vec(nf);
    steps(c, x, 3, 0.0, tau, s, rtol);
    const std::vector<double> xh = to_host(x, M8.n_nodes);
    CHECK(all_finite(xh));
    OK(eqs_apply_K(c, 3 * tau, x, y));
    CHECK(all_finite(to_host(y, M8.n_nodes)));
    std::vector<double> xf(nf);  // x on the free nodes, in increasing node id
    {
        std::vector<char> is_dir(M8.n_nodes, 0);
        for (int32_t v : in8.dir_nodes) is_dir[v] = 1;
        int64_t k = 0;
        for (int64_t i = 0; i < M8.n_nodes; ++i)
            if (!is_dir[i]) xf[k++] = xh[i];
        CHECK(k == nf);
    }
    HIPOK(hipMemcpy(w, xf.data(), nf * sizeof(double), hipMemcpyHostToDevice));
    OK(eqs_stage_rhs(c, 3 * tau, w, r));
    OK(eqs_apply_M(c, r, z));
    OK(eqs_apply_preconditioner(c, r, z));
    CHECK(all_finite(to_host(z, nf)));
    HIPOK(hipMemset(z, 0, nf * sizeof(double)));
    eqs_solve_stats ss{};
    OK(eqs_solve_M(c, r, z, rtol, 500, &ss));
    CHECK(ss.status == EQS_OK && ss.relres <= 1.01 * rtol && ss.iters > 0);
    FAILS(eqs_solve_M(c, r, z, rtol, -1, &ss), EQS_ERR_INVALID_ARG);
    FAILS(eqs_solve_M(c, r, r, rtol, 500, &ss), EQS_ERR_INVALID_ARG);
    FAILS(eqs_rkc_step(c, 0.0, tau, 1, x, rtol, 500, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_rkc_step(c, 0.0, tau, 257, x, rtol, 500, nullptr), EQS_ERR_INVALID_ARG);
    FAILS(eqs_set_deterministic(c, 1), EQS_ERR_STATE);
    {
        int32_t m = -1, one = 0;
        FAILS(eqs_stage_iters(c, nullptr, 4, &m), EQS_ERR_INVALID_ARG);
        FAILS(eqs_stage_iters(c, &one, -1, &m), EQS_ERR_INVALID_ARG);
        OK(eqs_stage_iters(c, nullptr, 0, &m));
        CHECK(m == s);  // the last step's, untouched by the rejected step calls above
    }
    int64_t its = 0;
    double rr = 0;
    OK(eqs_instance_stats(c, 1, &its, &rr));
    CHECK(its == ss.iters);

    // --- timing of every kernel class
    part("kernel timing");
    OK(eqs_profile_enable(c, (1u << EQS_KCLASS_COUNT) - 1));
    steps(c, x, 1, 3 * tau, tau, s, rtol);
    int64_t launches = 0;
    double ms = 0;
    for (int k = 0; k < EQS_KCLASS_COUNT; ++k) OK(eqs_profile_read(c, k, &launches, &ms));
    OK(eqs_profile_read(c, EQS_KCLASS_ELEMENT, &launches, &ms));
    // one element pass per stage; with the plain start vector the next stage's
    // pass is queued behind a solve's convergence check and queued again when
    // the check sends the solve back (every solve, with EQS_TEST_REJECT_CHECK=1)
    const char* rj = std::getenv("EQS_TEST_REJECT_CHECK");
    if (rj && rj[0] == '1') CHECK(launches >= s && launches <= 2 * s && ms > 0);
    else CHECK(launches == s && ms > 0);
    FAILS(eqs_profile_read(c, EQS_KCLASS_COUNT, &launches, &ms), EQS_ERR_INVALID_ARG);
    OK(eqs_profile_enable(c, 0));

    // --- checkpoint and resume with a Galerkin start vector
    part("checkpoint and resume, Galerkin start vectors");
    eqs_guess_params gp{};
    gp.kind = EQS_GUESS_GALERKIN;
    gp.window = 4;
    OK(eqs_set_guess(c, &gp));
    steps(c, x, 2, 4 * tau, tau, s, rtol);
    int64_t bytes = 0;
    OK(eqs_state_size(c, &bytes));
    std::vector<unsigned char> ckpt(bytes);
    FAILS(eqs_state_save(c, ckpt.data(), bytes - 1), EQS_ERR_INVALID_ARG);
    OK(eqs_state_save(c, ckpt.data(), bytes));
    steps(c, x, 1, 6 * tau, tau, s, rtol);
    OK(eqs_state_load(c, ckpt.data(), bytes));
    std::vector<unsigned char> junk(bytes, 0x5a);
    FAILS(eqs_state_load(c, junk.data(), bytes), EQS_ERR_INVALID_ARG);
    OK(eqs_state_load(c, ckpt.data(), bytes));
    steps(c, x, 1, 6 * tau, tau, s, rtol);

    // --- the start-vector network, the model-order-reduction and zero guesses
    part("network, reduced-basis and zero start vectors");
    Rng rng{7};
    std::vector<float> init(EQS_MLP_NPARAM);
    for (float& v : init) v = (float)(0.2 * (rng.uniform() - 0.5));
    gp = eqs_guess_params{};
    gp.kind = EQS_GUESS_MLP;
    gp.window = 8;
    gp.capacity = 64;
    gp.batch = 32;
    gp.seed = 11;
    {
        Transient<float> w(init);  // the initial weights are copied by the call
        gp.init = w.p;
        OK(eqs_set_guess(c, &gp));
    }
    gp.init = nullptr;
    steps(c, x, 3, 7 * tau, tau, s, rtol);
    OK(eqs_state_size(c, &bytes));
    ckpt.assign(bytes, 0);
    OK(eqs_state_save(c, ckpt.data(), bytes));
    OK(eqs_state_load(c, ckpt.data(), bytes));
    gp = eqs_guess_params{};
    gp.kind = EQS_GUESS_MOR;
    gp.window = 3;
    OK(eqs_set_guess(c, &gp));
    steps(c, x, 2, 10 * tau, tau, s, rtol);
    gp = eqs_guess_params{};
    gp.kind = EQS_GUESS_ZERO;
    OK(eqs_set_guess(c, &gp));
    steps(c, x, 1, 12 * tau, tau, s, rtol);
    gp.kind = 9;
    FAILS(eqs_set_guess(c, &gp), EQS_ERR_INVALID_ARG);

    // --- the Galerkin start vector on a caller's window, with and without allocation
    part("Galerkin start vector on a caller's window");
    {
        const int k = 3;
        double* S = dev.vec(k * nf);
        double* R = dev.vec(k * nf);
        double* x0 = dev.vec(nf);
        double* x1 = dev.vec(nf);
        std::vector<double> col(nf);
        for (int a = 0; a < k; ++a) {
            for (double& v : col) v = rng.uniform() - 0.5;
            HIPOK(hipMemcpy(S + a * nf, col.data(), nf * sizeof(double), hipMemcpyHostToDevice));
            OK(eqs_apply_M(c, S + a * nf, R + a * nf));
        }
        int32_t m0 = -1, m1 = -1;
        OK(eqs_galerkin_start(c, k, S, R, r, x0, &m0));
        OK(eqs_galerkin_start_noalloc(c, k, S, R, r, x1, &m1));
        CHECK(m0 == k && m1 == k);
        const std::vector<double> a0 = to_host(x0, nf), a1 = to_host(x1, nf);
        double d = 0, n0 = 0;
        for (int64_t i = 0; i < nf; ++i) {
            d = std::max(d, std::fabs(a0[i] - a1[i]));
            n0 = std::max(n0, std::fabs(a0[i]));
        }
        CHECK(d <= 1e-12 * n0);
        FAILS(eqs_galerkin_start_noalloc(c, 17, S, R, r, x1, &m1), EQS_ERR_INVALID_ARG);
        FAILS(eqs_galerkin_start(c, k, S, R, r, S, &m1), EQS_ERR_INVALID_ARG);
    }

    // --- the caller's workspace: move in, step, move out
    part("caller's workspace");
    gp = eqs_guess_params{};
    OK(eqs_set_guess(c, &gp));
    OK(eqs_query(c, nullptr, &ws));
    void* wsp = nullptr;
    HIPOK(hipMalloc(&wsp, ws));
    FAILS(eqs_set_workspace(c, wsp, ws - 256), EQS_ERR_INVALID_ARG);
    OK(eqs_set_workspace(c, wsp, ws));
    OK(eqs_get_info(c, &info));
    CHECK(info.device_bytes == 0 && info.workspace_bytes == ws);
    steps(c, x, 1, 13 * tau, tau, s, rtol);
    OK(eqs_set_workspace(c, nullptr, 0));
    HIPOK(hipFree(wsp));
    steps(c, x, 1, 14 * tau, tau, s, rtol);
    OK(eqs_destroy(c));

    // --- adaptive stepping
    part("adaptive stepping");
    OK(eqs_create(&c, 0, stream));
    set_inputs(c, M8, slab_inputs(M8, 1.0));
    OK(eqs_build_preconditioner(c, nullptr));
    HIPOK(hipMemset(x, 0, M8.n_nodes * sizeof(double)));
    eqs_adapt_params ap{};  // local error below 1e-2 (Sec. V)
    ap.atol = 1e-2;
    ap.rtol = 1e-2;
    ap.tau0 = 1e-4;
    std::vector<eqs_adapt_record> rec(8);
    int32_t n_rec = 0;
    eqs_adapt_stats as{};
    OK(eqs_rkc_adaptive(c, 0.0, 2e-3, x, 1e-8, 500, &ap, rec.data(), (int32_t)rec.size(), &n_rec, &as));
    CHECK(as.accepted >= 1 && n_rec == as.accepted + as.rejected);
    CHECK(all_finite(to_host(x, M8.n_nodes)));
    ap.atol = 0;
    FAILS(eqs_rkc_adaptive(c, 0.0, 2e-3, x, 1e-8, 500, &ap, nullptr, 0, nullptr, nullptr), EQS_ERR_INVALID_ARG);
    OK(eqs_destroy(c));

    // --- deterministic element pass with the FP32 hierarchy
    part("deterministic element pass, FP32 hierarchy");
    OK(eqs_create(&c, 0, stream));
    set_inputs(c, M8, in8);
    OK(eqs_set_deterministic(c, 1));
    eqs_amg_params p32{};
    p32.precision = EQS_PREC_FP32;
    OK(eqs_build_preconditioner(c, &p32));
    HIPOK(hipMemset(x, 0, M8.n_nodes * sizeof(double)));
    steps(c, x, 2, 0.0, tau, s, rtol);
    p32.theta = 1.5;
    FAILS(eqs_build_preconditioner(c, &p32), EQS_ERR_INVALID_ARG);
    OK(eqs_destroy(c));

    // --- second-order tets
    part("second-order tets");
    {
        const Mesh P = kuhn_mesh(4, true);
        OK(eqs_create(&c, 0, stream));
        set_inputs(c, P, slab_inputs(P, 3.0));
        FAILS(eqs_build_preconditioner(c, &p32), EQS_ERR_INVALID_ARG);  // theta 1.5 is still set
        p32.theta = 0;
        OK(eqs_build_preconditioner(c, &p32));
        double* xp = dev.vec(P.n_nodes);
        steps(c, xp, 2, 0.0, tau, s, rtol);
        CHECK(all_finite(to_host(xp, P.n_nodes)));
        OK(eqs_destroy(c));
    }

    // --- several instances in one context
    part("instances and batches");
    {
        const Mesh M7 = kuhn_mesh(7, false);
        const Mesh B = concat(M8, M7);
        Inputs in = slab_inputs(B, 3.0);
        OK(eqs_create(&c, 0, stream));
        OK(eqs_set_mesh(c, B.n_nodes, B.xyz.data(), B.n_tets, B.tets.data()));
        const int64_t node_off[3] = {0, M8.n_nodes, B.n_nodes}, tet_off[3] = {0, M8.n_tets, B.n_tets};
        {
            Transient<int64_t> no(std::vector<int64_t>(node_off, node_off + 3)), to(std::vector<int64_t>(tet_off, tet_off + 3));
            OK(eqs_set_instances(c, 2, no.p, to.p));
        }
        OK(eqs_set_materials(c, (int32_t)in.mats.size(), in.mats.data(), in.tet_mat.data()));
        OK(eqs_set_dirichlet(c, (int64_t)in.dir_nodes.size(), in.dir_nodes.data(), in.dir_drive.data(),
                             (int32_t)in.drives.size(), in.drives.data()));
        OK(eqs_build_preconditioner(c, &p32));
        double* xb = dev.vec(B.n_nodes);
        steps(c, xb, 2, 0.0, tau, s, rtol);
        int64_t it2[2] = {0, 0};
        double rr2[2] = {1, 1};
        OK(eqs_instance_stats(c, 2, it2, rr2));
        CHECK(it2[0] > 0 && it2[1] > 0 && rr2[0] <= 1.01 * rtol && rr2[1] <= 1.01 * rtol);
        gp = eqs_guess_params{};
        gp.kind = EQS_GUESS_GALERKIN;
        FAILS(eqs_set_guess(c, &gp), EQS_ERR_STATE);
        OK(eqs_destroy(c));

        // the same two problems through the batch form
        eqs_ctx* parts[2] = {nullptr, nullptr};
        OK(eqs_create(&parts[0], 0, stream));
        OK(eqs_create(&parts[1], 0, stream));
        set_inputs(parts[0], M8, in8);
        set_inputs(parts[1], M7, slab_inputs(M7, 2.0));
        eqs_batch* b = nullptr;
        OK(eqs_batch_create(&b, 2, parts, 0, stream, &p32));
        OK(eqs_destroy(parts[0]));
        OK(eqs_destroy(parts[1]));
        OK(eqs_batch_set_graph_iters(b, 3));
        double* xs[2] = {dev.vec(M8.n_nodes), dev.vec(M7.n_nodes)};
        eqs_step_stats st{};
        OK(eqs_batch_rkc_steps(b, 2, 0.0, tau, s, xs, rtol, 500, &st));
        CHECK(st.max_relres <= 1.01 * rtol);
        OK(eqs_batch_instance_stats(b, it2, rr2));
        CHECK(it2[0] > 0 && it2[1] > 0);
        OK(eqs_batch_destroy(b));
    }

    // --- the network on its own
    part("network on its own");
    {
        eqs_mlp* net = nullptr;
        FAILS(eqs_mlp_create(&net, 0, stream, nullptr, 1, 1e-3), EQS_ERR_INVALID_ARG);
        OK(eqs_mlp_create(&net, 0, stream, init.data(), 1, 1e-3));
        const int B = 64;
        std::vector<float> xin(B * 32), tgt(B * 16);
        for (float& v : xin) v = (float)(rng.uniform() - 0.5);
        for (float& v : tgt) v = (float)(rng.uniform() - 0.5);
        float *dx = nullptr, *dt = nullptr, *dy = nullptr;
        HIPOK(hipMalloc((void**)&dx, xin.size() * sizeof(float)));
        HIPOK(hipMalloc((void**)&dt, tgt.size() * sizeof(float)));
        HIPOK(hipMalloc((void**)&dy, tgt.size() * sizeof(float)));
        HIPOK(hipMemcpy(dx, xin.data(), xin.size() * sizeof(float), hipMemcpyHostToDevice));
        HIPOK(hipMemcpy(dt, tgt.data(), tgt.size() * sizeof(float), hipMemcpyHostToDevice));
        OK(eqs_mlp_forward(net, dx, dy, 17));
        float loss = -1;
        OK(eqs_mlp_train_step(net, dx, dt, B, &loss));
        CHECK(std::isfinite(loss) && loss > 0);
        FAILS(eqs_mlp_train_step(net, dx, dt, B + 1, &loss), EQS_ERR_INVALID_ARG);
        std::vector<float> params(EQS_MLP_NPARAM), grad(EQS_MLP_NPARAM);
        OK(eqs_mlp_get(net, params.data(), grad.data()));
        OK(eqs_mlp_destroy(net));
        HIPOK(hipFree(dx));
        HIPOK(hipFree(dt));
        HIPOK(hipFree(dy));
    }

    // --- input errors of the setters
    part("input errors");
    OK(eqs_create(&c, 0, stream));
    {
        Mesh bad = M8;
        bad.tets[5] = (int32_t)bad.n_nodes;
        FAILS(eqs_set_mesh(c, bad.n_nodes, bad.xyz.data(), bad.n_tets, bad.tets.data()), EQS_ERR_INVALID_ARG);
        FAILS(eqs_set_materials(c, 2, in8.mats.data(), in8.tet_mat.data()), EQS_ERR_STATE);
        OK(eqs_set_mesh(c, M8.n_nodes, M8.xyz.data(), M8.n_tets, M8.tets.data()));
        std::vector<eqs_material> mats = in8.mats;
        mats[1].e_s = NAN;
        FAILS(eqs_set_materials(c, 2, mats.data(), in8.tet_mat.data()), EQS_ERR_NONFINITE);
        std::vector<int32_t> dn = in8.dir_nodes;
        dn[1] = dn[0];
        FAILS(eqs_set_dirichlet(c, (int64_t)dn.size(), dn.data(), in8.dir_drive.data(), 2, in8.drives.data()),
              EQS_ERR_INVALID_ARG);
        // a flat tet is found by the build
        bad = M8;
        for (int d = 0; d < 3; ++d) bad.xyz[3 * (int64_t)bad.tets[3] + d] = bad.xyz[3 * (int64_t)bad.tets[0] + d];
        set_inputs(c, bad, in8);
        FAILS(eqs_build_preconditioner(c, nullptr), EQS_ERR_INVALID_ARG);
    }
    OK(eqs_destroy(c));
    HIPOK(hipStreamDestroy(stream));
}

}  // namespace

int main(int argc, char** argv) {
    const std::string mode = argc > 1 ? argv[1] : "";
    if (mode == "host") run_host();
    else if (mode == "abi") run_abi();
    else {
        std::fprintf(stderr, "usage: %s host|abi\n", argv[0]);
        return 2;
    }
    std::printf("SANITIZE OK %s (%d checks)\n", mode.c_str(), g_checks);
    return 0;
}
