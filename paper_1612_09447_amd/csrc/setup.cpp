// Host-side, once-per-context setup: input validation and node ordering,
// assembly of the constant permittivity matrix M on the free nodes (eq. (2)),
// the smoothed-aggregation AMG hierarchy that preconditions every M-solve
// (built once: Sec. II, the constant M turns the stage solves into a multiple
// right-hand-side problem), RKC coefficients (ref. [9] of the paper) and the
// upload of everything to device memory in SELL-64 form.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

#include <functional>
#include <iterator>

#include "eqs_internal.h"
#include "p2.h"

namespace eqs {

static constexpr double kEps0 = 8.8541878128e-12;  // F/m

// Edge vectors from p0 and their cross products: for a tet with edges
// e1, e2, e3 from p0, the rows of J^{-1} (J = [e1 e2 e3]) are
// (e2 x e3, e3 x e1, e1 x e2) / det with det = e1 . (e2 x e3); so the
// barycentric gradients are g_k = c_k / det and g_0 = -(g_1 + g_2 + g_3).
static double tet_cofactors(const double* p0, const double* p1, const double* p2, const double* p3,
                            double c[4][3]) {
    double e1[3], e2[3], e3[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = p1[d] - p0[d];
        e2[d] = p2[d] - p0[d];
        e3[d] = p3[d] - p0[d];
    }
    auto cross = [](const double* a, const double* b, double* o) {
        o[0] = a[1] * b[2] - a[2] * b[1];
        o[1] = a[2] * b[0] - a[0] * b[2];
        o[2] = a[0] * b[1] - a[1] * b[0];
    };
    cross(e2, e3, c[1]);
    cross(e3, e1, c[2]);
    cross(e1, e2, c[3]);
    for (int d = 0; d < 3; ++d) c[0][d] = -(c[1][d] + c[2][d] + c[3][d]);
    return e1[0] * c[1][0] + e1[1] * c[1][1] + e1[2] * c[1][2];
}

// ------------------------------------------------------------ validation
void validate_and_order(eqs_ctx* c) {
    const int64_t N = c->n_nodes;
    for (int64_t i = 0; i < 3 * N; ++i)
        if (!std::isfinite(c->xyz[i])) fail(EQS_ERR_NONFINITE, "non-finite node coordinate");
    const int npe = c->npe;
    for (int64_t e = 0; e < c->n_tets; ++e) {
        const int32_t* v = &c->tets[npe * e];
        for (int a = 0; a < npe; ++a)
            if (v[a] < 0 || v[a] >= N) fail(EQS_ERR_INVALID_ARG, "tet " + std::to_string(e) + " has a node id out of range");
        double cf[4][3];
        double det = tet_cofactors(&c->xyz[3 * (int64_t)v[0]], &c->xyz[3 * (int64_t)v[1]], &c->xyz[3 * (int64_t)v[2]],
                                   &c->xyz[3 * (int64_t)v[3]], cf);
        if (!(std::fabs(det) > 0) || !std::isfinite(det))
            fail(EQS_ERR_INVALID_ARG, "tet " + std::to_string(e) + " has zero volume");
    }
    std::vector<char> is_dir(N, 0);
    for (size_t k = 0; k < c->dir_nodes.size(); ++k) is_dir[c->dir_nodes[k]] = 1;
    c->n_dir = (int64_t)c->dir_nodes.size();
    c->n_free = N - c->n_dir;
    c->int_to_user.resize(N);
    int64_t f = 0, d = c->n_free;
    for (int64_t i = 0; i < N; ++i) {
        if (is_dir[i]) c->int_to_user[d++] = (int32_t)i;
        else c->int_to_user[f++] = (int32_t)i;
    }
    // instances: free rows of instance i are the free nodes of its node range,
    // contiguous because free nodes keep increasing user ids
    if (c->inst_node_off.empty()) {
        c->inst_node_off = {0, N};
        c->inst_tet_off = {0, c->n_tets};
    }
    c->n_inst = (int64_t)c->inst_node_off.size() - 1;
    c->inst_row_off.assign(c->n_inst + 1, 0);
    for (int64_t i = 0; i < c->n_inst; ++i) {
        int64_t nf = 0, nd = 0;
        for (int64_t v = c->inst_node_off[i]; v < c->inst_node_off[i + 1]; ++v) (is_dir[v] ? nd : nf)++;
        if (nd == 0) fail(EQS_ERR_INVALID_ARG, "instance " + std::to_string(i) + " has no Dirichlet node");
        if (nf == 0) fail(EQS_ERR_INVALID_ARG, "instance " + std::to_string(i) + " has no free node");
        if (c->n_inst > 1 && nf < 256)
            fail(EQS_ERR_INVALID_ARG, "instance " + std::to_string(i) + " has fewer than 256 free nodes");
        c->inst_row_off[i + 1] = c->inst_row_off[i] + (int32_t)nf;
    }
    for (int64_t i = 0; i < c->n_inst; ++i)
        for (int64_t e = c->inst_tet_off[i]; e < c->inst_tet_off[i + 1]; ++e)
            for (int a = 0; a < npe; ++a) {
                const int32_t v = c->tets[npe * e + a];
                if (v < c->inst_node_off[i] || v >= c->inst_node_off[i + 1])
                    fail(EQS_ERR_INVALID_ARG, "tet " + std::to_string(e) + " uses a node of another instance");
            }
    c->inst_iters.assign(c->n_inst, 0);
    c->inst_relres.assign(c->n_inst, 0.0);
}

// ----------------------------------------------------------- assembly of M
// Off-diagonal entries whose magnitude is at roundoff level against the
// diagonal, |a_ij| <= 1e-14 sqrt(a_ii a_jj), are dropped. On meshes built from
// right-angled (Kuhn) tets the P1 Laplacian has exact zeros on the face and
// body diagonals of every cube, i.e. about half of the structural entries.
static Csr<double> drop_zeros(const Csr<double>& A) {
    std::vector<double> d(A.n_rows, 0.0);
    for (int32_t i = 0; i < A.n_rows; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (A.col[k] == i) d[i] = A.val[k];
    Csr<double> B;
    B.n_rows = A.n_rows;
    B.n_cols = A.n_cols;
    B.ptr.assign(A.n_rows + 1, 0);
    B.col.reserve(A.nnz());
    B.val.reserve(A.nnz());
    for (int32_t i = 0; i < A.n_rows; ++i) {
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            const int32_t j = A.col[k];
            if (j != i && std::fabs(A.val[k]) <= 1e-14 * std::sqrt(std::fabs(d[i] * d[j]))) continue;
            B.col.push_back(j);
            B.val.push_back(A.val[k]);
        }
        B.ptr[i + 1] = (int32_t)B.col.size();
    }
    return B;
}

Csr<double> assemble_M_free(const eqs_ctx* c) {
    const int64_t N = c->n_nodes, T = c->n_tets, NF = c->n_free;
    std::vector<int32_t> u2i(N);
    for (int64_t i = 0; i < N; ++i) u2i[c->int_to_user[i]] = (int32_t)i;

    const int npe = c->npe;
    // node -> incident tets
    std::vector<int64_t> nt_ptr(N + 1, 0);
    for (int64_t e = 0; e < npe * T; ++e) nt_ptr[u2i[c->tets[e]] + 1]++;
    for (int64_t i = 0; i < N; ++i) nt_ptr[i + 1] += nt_ptr[i];
    std::vector<int32_t> nt(nt_ptr[N]);
    {
        std::vector<int64_t> fill(nt_ptr.begin(), nt_ptr.end() - 1);
        for (int64_t e = 0; e < T; ++e)
            for (int a = 0; a < npe; ++a) nt[fill[u2i[c->tets[npe * e + a]]]++] = (int32_t)e;
    }

    // row patterns: free neighbours through incident tets
    Csr<double> M;
    M.n_rows = M.n_cols = (int32_t)NF;
    M.ptr.assign(NF + 1, 0);
    std::vector<int32_t> buf;
    for (int pass = 0; pass < 2; ++pass) {
        int64_t pos = 0;
        for (int64_t i = 0; i < NF; ++i) {
            buf.clear();
            for (int64_t k = nt_ptr[i]; k < nt_ptr[i + 1]; ++k) {
                const int32_t* v = &c->tets[npe * (int64_t)nt[k]];
                for (int a = 0; a < npe; ++a) {
                    int32_t j = u2i[v[a]];
                    if (j < NF) buf.push_back(j);
                }
            }
            std::sort(buf.begin(), buf.end());
            buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
            if (pass == 0) {
                pos += (int64_t)buf.size();
                if (pos > INT32_MAX) fail(EQS_ERR_INVALID_ARG, "M has more than 2^31 nonzeros");
                M.ptr[i + 1] = (int32_t)pos;
            } else {
                std::copy(buf.begin(), buf.end(), M.col.begin() + M.ptr[i]);
            }
        }
        if (pass == 0) {
            M.col.resize(M.ptr[NF]);
            M.val.assign(M.ptr[NF], 0.0);
        }
    }

    // values: P1 element matrices eps_e |T| g_a . g_b = eps_e c_a . c_b / (6 |det|);
    // second order: eps_e sum_q G_a(q) . G_b(q) / (24 |det|) (see p2.h)
    double A[kP2Nodes][kP2Nodes];
    for (int64_t e = 0; e < T; ++e) {
        const int32_t* vu = &c->tets[npe * e];
        int32_t v[kP2Nodes];
        for (int a = 0; a < npe; ++a) v[a] = u2i[vu[a]];
        double cf[4][3];
        double det = tet_cofactors(&c->xyz[3 * (int64_t)vu[0]], &c->xyz[3 * (int64_t)vu[1]], &c->xyz[3 * (int64_t)vu[2]],
                                   &c->xyz[3 * (int64_t)vu[3]], cf);
        const double eps = kEps0 * c->mats[c->tet_mat[e]].eps_r;
        if (npe == 4) {
            const double w = eps / (6.0 * std::fabs(det));
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) A[a][b] = w * (cf[a][0] * cf[b][0] + cf[a][1] * cf[b][1] + cf[a][2] * cf[b][2]);
        } else {
            for (int a = 0; a < kP2Nodes; ++a)
                for (int b = 0; b < kP2Nodes; ++b) A[a][b] = 0.0;
            const double w = eps / (24.0 * std::fabs(det));
            for (int q = 0; q < 4; ++q) {
                double G[kP2Nodes][3];
                for (int a = 0; a < 4; ++a)
                    for (int d = 0; d < 3; ++d) G[a][d] = (4.0 * p2_lambda(q, a) - 1.0) * cf[a][d];
                for (int k = 0; k < 6; ++k) {
                    const int a = p2_edge_a(k), b = p2_edge_b(k);
                    for (int d = 0; d < 3; ++d) G[4 + k][d] = 4.0 * (p2_lambda(q, b) * cf[a][d] + p2_lambda(q, a) * cf[b][d]);
                }
                for (int a = 0; a < kP2Nodes; ++a)
                    for (int b = 0; b < kP2Nodes; ++b) A[a][b] += w * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
            }
        }
        for (int a = 0; a < npe; ++a) {
            if (v[a] >= NF) continue;
            const int32_t* cb = M.col.data() + M.ptr[v[a]];
            const int32_t* ce = M.col.data() + M.ptr[v[a] + 1];
            for (int b = 0; b < npe; ++b) {
                if (v[b] >= NF) continue;
                const int32_t* it = std::lower_bound(cb, ce, v[b]);
                M.val[it - M.col.data()] += A[a][b];
            }
        }
    }
    return drop_zeros(M);
}

// ------------------------------------------------------ sparse host algebra
static Csr<double> transpose(const Csr<double>& A) {
    Csr<double> T;
    T.n_rows = A.n_cols;
    T.n_cols = A.n_rows;
    T.ptr.assign(T.n_rows + 1, 0);
    for (int32_t k = 0; k < (int32_t)A.nnz(); ++k) T.ptr[A.col[k] + 1]++;
    for (int32_t i = 0; i < T.n_rows; ++i) T.ptr[i + 1] += T.ptr[i];
    T.col.resize(A.nnz());
    T.val.resize(A.nnz());
    std::vector<int32_t> fill(T.ptr.begin(), T.ptr.end() - 1);
    for (int32_t i = 0; i < A.n_rows; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            int32_t p = fill[A.col[k]]++;
            T.col[p] = i;
            T.val[p] = A.val[k];
        }
    return T;
}

// C = A B, row by row with a dense accumulator (columns sorted per row).
static Csr<double> spgemm(const Csr<double>& A, const Csr<double>& B) {
    Csr<double> C;
    C.n_rows = A.n_rows;
    C.n_cols = B.n_cols;
    C.ptr.assign(C.n_rows + 1, 0);
    std::vector<double> acc(B.n_cols, 0.0);
    std::vector<int32_t> mark(B.n_cols, -1), cols;
    for (int32_t i = 0; i < A.n_rows; ++i) {
        cols.clear();
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            const int32_t r = A.col[k];
            const double a = A.val[k];
            for (int32_t m = B.ptr[r]; m < B.ptr[r + 1]; ++m) {
                const int32_t j = B.col[m];
                if (mark[j] != i) {
                    mark[j] = i;
                    acc[j] = 0.0;
                    cols.push_back(j);
                }
                acc[j] += a * B.val[m];
            }
        }
        std::sort(cols.begin(), cols.end());
        if ((int64_t)C.col.size() + (int64_t)cols.size() > INT32_MAX) fail(EQS_ERR_INVALID_ARG, "AMG product too large");
        for (int32_t j : cols) {
            C.col.push_back(j);
            C.val.push_back(acc[j]);
        }
        C.ptr[i + 1] = (int32_t)C.col.size();
    }
    return C;
}

static std::vector<double> diagonal(const Csr<double>& A) {
    std::vector<double> d(A.n_rows, 0.0);
    for (int32_t i = 0; i < A.n_rows; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (A.col[k] == i) d[i] = A.val[k];
    return d;
}

// Spectral radius of D^{-1} A: power iteration (deterministic start), with a
// 5 % margin, capped by the Gershgorin bound max_i sum_j |a_ij| / a_ii.
static double spectral_radius_DinvA(const Csr<double>& A, const std::vector<double>& d) {
    const int32_t n = A.n_rows;
    double gersh = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) s += std::fabs(A.val[k]);
        gersh = std::max(gersh, s / d[i]);
    }
    std::vector<double> x(n), y(n);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    for (int32_t i = 0; i < n; ++i) {
        st ^= st << 13; st ^= st >> 7; st ^= st << 17;
        x[i] = 0.5 + (double)(st >> 11) * (1.0 / 9007199254740992.0);
    }
    double lam = 0.0;
    for (int it = 0; it < 15; ++it) {
        double nx = 0.0, ny = 0.0;
        for (int32_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) s += A.val[k] * x[A.col[k]];
            y[i] = s / d[i];
            ny += y[i] * y[i];
            nx += x[i] * x[i];
        }
        lam = std::sqrt(ny / nx);
        double inv = 1.0 / std::sqrt(ny);
        for (int32_t i = 0; i < n; ++i) x[i] = y[i] * inv;
    }
    return std::min(gersh, 1.05 * lam);
}

// Greedy aggregation on the strength graph: (1) a node whose strong
// neighbours are all unassigned seeds an aggregate with them; (2) leftover
// nodes join the seeded aggregate they are most strongly tied to; (3) what is
// still unassigned forms aggregates with its unassigned strong neighbours.
static int32_t aggregate(const Csr<double>& A, const std::vector<double>& d, double theta,
                         std::vector<int32_t>& agg) {
    const int32_t n = A.n_rows;
    std::vector<char> strong(A.nnz(), 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            int32_t j = A.col[k];
            if (j != i && std::fabs(A.val[k]) >= theta * std::sqrt(std::fabs(d[i] * d[j]))) strong[k] = 1;
        }
    agg.assign(n, -1);
    int32_t na = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (agg[i] != -1) continue;
        bool free_nbhd = true, any = false;
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (strong[k]) {
                any = true;
                if (agg[A.col[k]] != -1) { free_nbhd = false; break; }
            }
        if (!any || !free_nbhd) continue;
        agg[i] = na;
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (strong[k]) agg[A.col[k]] = na;
        ++na;
    }
    std::vector<int32_t> seeded = agg;
    for (int32_t i = 0; i < n; ++i) {
        if (agg[i] != -1) continue;
        double best = -1.0;
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (strong[k] && seeded[A.col[k]] != -1 && std::fabs(A.val[k]) > best) {
                best = std::fabs(A.val[k]);
                agg[i] = seeded[A.col[k]];
            }
    }
    for (int32_t i = 0; i < n; ++i) {
        if (agg[i] != -1) continue;
        agg[i] = na;
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (strong[k] && agg[A.col[k]] == -1) agg[A.col[k]] = na;
        ++na;
    }
    // number aggregates in the order of their first row, so coarse rows follow
    // fine rows (locality, and instances stay contiguous at every level)
    std::vector<int32_t> renum(na, -1);
    int32_t next = 0;
    for (int32_t i = 0; i < n; ++i)
        if (renum[agg[i]] < 0) renum[agg[i]] = next++;
    for (int32_t i = 0; i < n; ++i) agg[i] = renum[agg[i]];
    return na;
}

// Dense inverse of a small SPD matrix via Cholesky (column-major output).
static std::vector<double> dense_spd_inverse(const Csr<double>& A) {
    const int32_t n = A.n_rows;
    std::vector<double> L((size_t)n * n, 0.0);  // row-major lower factor
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) L[(size_t)i * n + A.col[k]] = A.val[k];
    for (int32_t j = 0; j < n; ++j) {
        double s = L[(size_t)j * n + j];
        for (int32_t k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0)) fail(EQS_ERR_INVALID_ARG, "coarsest AMG matrix is not positive definite");
        const double ljj = std::sqrt(s);
        L[(size_t)j * n + j] = ljj;
        for (int32_t i = j + 1; i < n; ++i) {
            double t = L[(size_t)i * n + j];
            for (int32_t k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
    }
    std::vector<double> inv((size_t)n * n, 0.0), col(n);
    for (int32_t c = 0; c < n; ++c) {
        // solve L y = e_c, then L^T x = y
        for (int32_t i = 0; i < n; ++i) {
            double t = (i == c) ? 1.0 : 0.0;
            for (int32_t k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * col[k];
            col[i] = t / L[(size_t)i * n + i];
        }
        for (int32_t i = n - 1; i >= 0; --i) {
            double t = col[i];
            for (int32_t k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * col[k];
            col[i] = t / L[(size_t)i * n + i];
        }
        for (int32_t i = 0; i < n; ++i) inv[(size_t)c * n + i] = col[i];
    }
    return inv;
}

AmgHost build_sa_amg(const Csr<double>& M, const eqs_amg_params& p) {
    AmgHost h;
    Csr<double> A = M;
    for (;;) {
        const int32_t n = A.n_rows;
        const bool last = n <= p.coarse_max || (int32_t)h.A.size() + 1 >= p.max_levels;
        std::vector<double> d = diagonal(A);
        for (int32_t i = 0; i < n; ++i)
            if (!(d[i] > 0)) fail(EQS_ERR_INVALID_ARG, "matrix has a non-positive diagonal entry");
        if (last) {
            if (n > 4096) fail(EQS_ERR_INVALID_ARG, "AMG coarsening stalled above 4096 unknowns");
            h.coarse_inv = dense_spd_inverse(A);
            h.omega.push_back(0.0);
            h.A.push_back(std::move(A));
            break;
        }
        const double rho = spectral_radius_DinvA(A, d);
        std::vector<int32_t> agg;
        // strength threshold halves from level to level (Vanek, Mandel, Brezina 1996)
        const double theta_l = p.theta * std::ldexp(1.0, -(int)h.A.size());
        const int32_t nc = aggregate(A, d, theta_l, agg);
        if (nc >= n) fail(EQS_ERR_INVALID_ARG, "AMG aggregation did not coarsen");

        // tentative prolongator: column per aggregate, normalised
        std::vector<int32_t> size(nc, 0);
        for (int32_t i = 0; i < n; ++i) size[agg[i]]++;
        std::vector<double> w(nc);
        for (int32_t a = 0; a < nc; ++a) w[a] = 1.0 / std::sqrt((double)size[a]);

        // P = P_tent - (smooth_weight / rho) D^{-1} A P_tent
        const double sw = p.smooth_weight / rho;
        Csr<double> P;
        P.n_rows = n;
        P.n_cols = nc;
        P.ptr.assign(n + 1, 0);
        std::vector<int32_t> cols;
        std::vector<double> acc(nc, 0.0);
        std::vector<int32_t> mark(nc, -1);
        for (int32_t i = 0; i < n; ++i) {
            cols.clear();
            auto add = [&](int32_t a, double v) {
                if (mark[a] != i) { mark[a] = i; acc[a] = 0.0; cols.push_back(a); }
                acc[a] += v;
            };
            add(agg[i], w[agg[i]]);
            for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                int32_t j = A.col[k];
                add(agg[j], -sw * A.val[k] / d[i] * w[agg[j]]);
            }
            std::sort(cols.begin(), cols.end());
            for (int32_t a : cols) {
                P.col.push_back(a);
                P.val.push_back(acc[a]);
            }
            P.ptr[i + 1] = (int32_t)P.col.size();
        }
        Csr<double> R = transpose(P);
        Csr<double> AP = spgemm(A, P);
        Csr<double> Ac = spgemm(R, AP);
        h.omega.push_back(p.jacobi_weight / rho);
        h.A.push_back(std::move(A));
        h.P.push_back(std::move(P));
        h.R.push_back(std::move(R));
        A = std::move(Ac);
    }
    return h;
}

// ---------------------------------------------------------------- RKC(s)
// Stability boundary beta(s) = (1 + w0) / w1 of RKC(s) (ref. [9]), damping 2/13.
double rkc_beta(int s) {
    const double w0 = 1.0 + (2.0 / 13.0) / ((double)s * s);
    double T0 = 1.0, T = w0, d0 = 0.0, d = 1.0, dd0 = 0.0, dd = 0.0;  // T_j, T_j', T_j'' at w0 (j = 1)
    for (int j = 2; j <= s; ++j) {
        const double Tn = 2.0 * w0 * T - T0, dn = 2.0 * T + 2.0 * w0 * d - d0, ddn = 4.0 * d + 2.0 * w0 * dd - dd0;
        T0 = T; T = Tn; d0 = d; d = dn; dd0 = dd; dd = ddn;
    }
    return (1.0 + w0) / (d / dd);
}

// Coefficients of the s-stage second-order RKC method (ref. [9]: Sommeijer,
// Shampine, Verwer), damping 2/13. Index j = 0..s; mu, nu, mut (mu~), gmt
// (gamma~) are used for j >= 2 (mut also for j = 1); c are the stage times.
void rkc_coefficients(int s, std::vector<double>& mu, std::vector<double>& nu, std::vector<double>& mut,
                      std::vector<double>& gmt, std::vector<double>& c) {
    const double w0 = 1.0 + (2.0 / 13.0) / ((double)s * s);
    std::vector<double> T(s + 1), T1(s + 1), T2(s + 1);  // Chebyshev T_j and derivatives at w0
    T[0] = 1.0; T1[0] = 0.0; T2[0] = 0.0;
    T[1] = w0;  T1[1] = 1.0; T2[1] = 0.0;
    for (int j = 2; j <= s; ++j) {
        T[j] = 2.0 * w0 * T[j - 1] - T[j - 2];
        T1[j] = 2.0 * T[j - 1] + 2.0 * w0 * T1[j - 1] - T1[j - 2];
        T2[j] = 4.0 * T1[j - 1] + 2.0 * w0 * T2[j - 1] - T2[j - 2];
    }
    const double w1 = T1[s] / T2[s];
    std::vector<double> b(s + 1), a(s + 1);
    for (int j = 2; j <= s; ++j) b[j] = T2[j] / (T1[j] * T1[j]);
    b[0] = b[1] = b[2];
    for (int j = 0; j <= s; ++j) a[j] = 1.0 - b[j] * T[j];
    mu.assign(s + 1, 0.0); nu.assign(s + 1, 0.0); mut.assign(s + 1, 0.0); gmt.assign(s + 1, 0.0); c.assign(s + 1, 0.0);
    mut[1] = b[1] * w1;
    c[1] = mut[1];
    for (int j = 2; j <= s; ++j) {
        mu[j] = 2.0 * b[j] * w0 / b[j - 1];
        nu[j] = -b[j] / b[j - 2];
        mut[j] = 2.0 * b[j] * w1 / b[j - 1];
        gmt[j] = -a[j - 1] * mut[j];
        c[j] = w1 * T2[j] / T1[j];
    }
}

// ------------------------------------------------------------------ upload
// Every device buffer of a context goes through dev_alloc: 256-byte granules,
// from hipMalloc or, when the caller gave a workspace, first fit from its free
// ranges.
static constexpr int64_t kGranule = 256;
static int64_t granules(size_t bytes) { return ((int64_t)std::max<size_t>(bytes, 1) + kGranule - 1) / kGranule * kGranule; }

static bool in_workspace(const eqs_ctx* c, const void* p) {
    return c->ws_base && (const char*)p >= c->ws_base && (const char*)p < c->ws_base + c->ws_size;
}

static void ws_reset(eqs_ctx* c) {
    c->ws_free.clear();
    c->ws_used = 0;
    if (c->ws_base && c->ws_size > 0) c->ws_free[0] = c->ws_size;
}

void* dev_alloc(eqs_ctx* c, size_t bytes) {
    const int64_t len = granules(bytes);
    void* p = nullptr;
    if (c->ws_base) {
        for (auto it = c->ws_free.begin(); it != c->ws_free.end(); ++it)
            if (it->second >= len) {
                const int64_t off = it->first, rest = it->second - len;
                c->ws_free.erase(it);
                if (rest > 0) c->ws_free[off + len] = rest;
                p = c->ws_base + off;
                break;
            }
        if (!p)
            fail(EQS_ERR_ALLOC, "workspace too small: " + std::to_string(len) + " more bytes needed with " +
                                    std::to_string(c->ws_size - c->ws_used) + " free (eqs_query gives the size)");
        c->ws_used += len;
    } else {
        hipError_t e = hipMalloc(&p, (size_t)len);
        if (e != hipSuccess) fail(EQS_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
        c->device_bytes += len;
    }
    c->allocations.push_back({p, (size_t)len});
    return p;
}

void dev_free(eqs_ctx* c, void* p) {
    if (!p) return;
    for (size_t k = 0; k < c->allocations.size(); ++k)
        if (c->allocations[k].first == p) {
            const int64_t len = (int64_t)c->allocations[k].second;
            if (in_workspace(c, p)) {
                // back to the free ranges, merged with its neighbours
                int64_t off = (char*)p - c->ws_base, n = len;
                auto nx = c->ws_free.lower_bound(off);
                if (nx != c->ws_free.end() && nx->first == off + n) {
                    n += nx->second;
                    nx = c->ws_free.erase(nx);
                }
                if (nx != c->ws_free.begin()) {
                    auto pv = std::prev(nx);
                    if (pv->first + pv->second == off) {
                        off = pv->first;
                        n += pv->second;
                        c->ws_free.erase(pv);
                    }
                }
                c->ws_free[off] = n;
                c->ws_used -= len;
            } else {
                (void)hipFree(p);
                c->device_bytes -= len;
            }
            c->allocations.erase(c->allocations.begin() + k);
            return;
        }
}

int64_t workspace_need(const eqs_ctx* c) {
    int64_t n = 0;
    for (const auto& a : c->allocations) n += (int64_t)a.second;
    return n + guess_pending_bytes(c);
}

template <typename T>
static void visit_sell(Sell<T>& S, const std::function<void(void**)>& f) {
    f((void**)&S.sptr);
    f((void**)&S.col);
    f((void**)&S.d16);
    f((void**)&S.val);
    f((void**)&S.perm);
}
template <typename T>
static void visit_spmat(SpMat<T>& A, const std::function<void(void**)>& f) {
    visit_sell(A.sell, f);
    f((void**)&A.rowptr);
    f((void**)&A.col);
    f((void**)&A.d16);
    f((void**)&A.val);
}
template <typename T>
static void visit_hierarchy(Hierarchy<T>& h, const std::function<void(void**)>& f) {
    for (Level<T>& lv : h.lv) {
        visit_spmat(lv.A, f);
        visit_spmat(lv.P, f);
        visit_spmat(lv.R, f);
        visit_spmat(lv.GQ, f);
        for (T** q : {&lv.dinv, &lv.sval, &lv.b, &lv.x, &lv.xs, &lv.res, &lv.dense_inv, &lv.coarse_R}) f((void**)q);
    }
}

void visit_device_ptrs(eqs_ctx* c, const std::function<void(void**)>& f) {
    f((void**)&c->d_tpack);
    f((void**)&c->d_kslots);
    f((void**)&c->d_kend);
    f((void**)&c->d_occ_off);
    f((void**)&c->d_occ);
    f((void**)&c->d_kx_part);
    f((void**)&c->d_bnodes);
    f((void**)&c->d_boff);
    f((void**)&c->d_cx);
    f((void**)&c->d_cy);
    f((void**)&c->d_cz);
    f((void**)&c->d_mats);
    f((void**)&c->d_ddrive);
    f((void**)&c->d_drives);
    f((void**)&c->d_int_to_user);
    visit_sell(c->M, f);
    visit_hierarchy(c->h64, f);
    visit_hierarchy(c->h32, f);
    for (double** q : {&c->d_r, &c->d_z, &c->d_p, &c->d_q, &c->d_mx, &c->d_Y0, &c->d_Ya, &c->d_Yb, &c->d_Yc, &c->d_F0,
                       &c->d_F, &c->d_rhs, &c->d_rhs_alt, &c->d_tmpN, &c->d_tmpN2, &c->d_partials})
        f((void**)q);
    f((void**)&c->d_inst_row);
    f((void**)&c->d_blk_inst);
    f((void**)&c->d_scal);
    f((void**)&c->d_sum);
    f((void**)&c->d_force);
    GuessState& g = c->guess;
    for (double** q : {&g.d_S, &g.d_rprev, &g.d_alpha, &g.d_guard, &g.d_dots, &g.d_part}) f((void**)q);
    f((void**)&g.d_gstat);
    f((void**)&g.d_bx);
    f((void**)&g.d_bt);
    mlp_visit(g.net, f);
}

// Move every device buffer into [dev, dev + bytes) (dev NULL: into buffers
// the library allocates), packed in allocation order, and remap every pointer
// that points into an old buffer (interior pointers keep their offset). A
// buffer that no visited pointer reaches stops the move before anything
// changes.
void set_workspace(eqs_ctx* c, void* dev, int64_t bytes) {
    EQS_HIP(hipStreamSynchronize(c->stream));
    if (c->guess.tstream) EQS_HIP(hipStreamSynchronize(c->guess.tstream));
    const std::vector<std::pair<void*, size_t>> old = c->allocations;
    auto owner = [&](const void* p) -> int {
        for (size_t k = 0; k < old.size(); ++k)
            if ((const char*)p >= (const char*)old[k].first && (const char*)p < (const char*)old[k].first + old[k].second)
                return (int)k;
        return -1;
    };
    std::vector<int> hits(old.size(), 0);
    visit_device_ptrs(c, [&](void** pp) {
        if (*pp) {
            const int k = owner(*pp);
            if (k >= 0) hits[k]++;
        }
    });
    for (size_t k = 0; k < old.size(); ++k)
        if (!hits[k]) fail(EQS_ERR_STATE, "internal: a device buffer of the context is not reachable for the move");
    int64_t total = 0;
    for (const auto& a : old) total += (int64_t)a.second;
    if (dev) {
        if (bytes < total)
            fail(EQS_ERR_INVALID_ARG, "workspace too small: " + std::to_string(total) + " bytes needed, " +
                                          std::to_string(bytes) + " given");
        for (const auto& a : old)
            if ((const char*)a.first < (const char*)dev + bytes && (const char*)dev < (const char*)a.first + a.second)
                fail(EQS_ERR_INVALID_ARG, "workspace overlaps the context's own device memory");
    }
    std::vector<void*> fresh(old.size(), nullptr);
    int64_t off = 0;
    try {
        for (size_t k = 0; k < old.size(); ++k) {
            if (dev) {
                fresh[k] = (char*)dev + off;
                off += (int64_t)old[k].second;
            } else {
                hipError_t e = hipMalloc(&fresh[k], old[k].second);
                if (e != hipSuccess) fail(EQS_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
            }
        }
        for (size_t k = 0; k < old.size(); ++k)
            EQS_HIP(hipMemcpyAsync(fresh[k], old[k].first, old[k].second, hipMemcpyDeviceToDevice, c->stream));
        EQS_HIP(hipStreamSynchronize(c->stream));
    } catch (...) {
        if (!dev)
            for (void* p : fresh)
                if (p) (void)hipFree(p);
        throw;
    }
    release_graphs(c);  // captured iterations hold the old addresses
    visit_device_ptrs(c, [&](void** pp) {
        if (!*pp) return;
        const int k = owner(*pp);
        if (k >= 0) *pp = (char*)fresh[k] + ((char*)*pp - (char*)old[k].first);
    });
    for (size_t k = 0; k < old.size(); ++k)
        if (!in_workspace(c, old[k].first)) (void)hipFree(old[k].first);
    c->allocations.clear();
    for (size_t k = 0; k < old.size(); ++k) c->allocations.push_back({fresh[k], old[k].second});
    c->ws_base = (char*)dev;
    c->ws_size = dev ? bytes : 0;
    c->ws_free.clear();
    c->ws_used = dev ? total : 0;
    if (dev && bytes > total) c->ws_free[total] = bytes - total;
    c->device_bytes = dev ? 0 : total;
}

template <typename T>
static T* upload_vec(eqs_ctx* c, const std::vector<T>& v) {
    T* d = (T*)dev_alloc(c, v.size() * sizeof(T));
    if (!v.empty()) EQS_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

template <typename T>
Sell<T> to_sell(eqs_ctx* c, const Csr<double>& A, int lanes, bool sorted) {
    if (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8) fail(EQS_ERR_STATE, "SELL lanes per row must be 1, 2, 4 or 8");
    const int32_t rows_per = kSlice / lanes;  // rows of one slice
    const int32_t window = 4 * rows_per;      // rows of one 256-thread window
    Sell<T> S;
    S.n_rows = A.n_rows;
    S.n_cols = A.n_cols;
    S.lanes = lanes;
    S.n_slices = (A.n_rows + rows_per - 1) / rows_per;
    // pos2row[k]: the row stored at position k (positions past n_rows are
    // phantom rows >= n_rows); sorted: longest rows first within each window
    const int32_t n_pos = S.n_slices * rows_per;
    std::vector<int32_t> pos2row((size_t)n_pos);
    for (int32_t k = 0; k < n_pos; ++k) pos2row[(size_t)k] = k;
    auto len = [&](int32_t r) { return r < A.n_rows ? A.ptr[r + 1] - A.ptr[r] : 0; };
    if (sorted)
        for (int32_t w0 = 0; w0 < n_pos; w0 += window) {
            const int32_t w1 = std::min(n_pos, w0 + window);
            std::stable_sort(pos2row.begin() + w0, pos2row.begin() + w1,
                             [&](int32_t a, int32_t b) { return len(a) > len(b); });
        }
    std::vector<int32_t> sptr(S.n_slices + 1, 0);
    for (int32_t s = 0; s < S.n_slices; ++s) {
        int32_t w = 0;  // entries per lane
        for (int32_t k = s * rows_per; k < (s + 1) * rows_per; ++k) w = std::max(w, (len(pos2row[k]) + lanes - 1) / lanes);
        int64_t next = (int64_t)sptr[s] + (int64_t)w * kSlice;
        if (next > INT32_MAX) fail(EQS_ERR_INVALID_ARG, "matrix too large for SELL offsets");
        sptr[s + 1] = (int32_t)next;
    }
    S.stored = sptr[S.n_slices];
    // lane l of slice s serves the row at position s * rows_per + l / lanes and
    // holds the row's entries l % lanes + lanes * k, k = 0 .. w-1
    std::vector<int32_t> col(S.stored, 0);
    std::vector<T> val(S.stored, T(0));
    for (int32_t s = 0; s < S.n_slices; ++s) {
        const int32_t w = (sptr[s + 1] - sptr[s]) / kSlice;
        for (int32_t l = 0; l < kSlice; ++l) {
            const int32_t r = pos2row[(size_t)(s * rows_per + l / lanes)], part = l % lanes;
            int32_t pad_col = 0;
            const int32_t n = len(r);
            if (n > 0) pad_col = A.col[A.ptr[r] + n - 1];
            for (int32_t k = 0; k < w; ++k) {
                const int64_t at = sptr[s] + (int64_t)k * kSlice + l;
                const int32_t e = k * lanes + part;
                if (e < n) {
                    col[at] = A.col[A.ptr[r] + e];
                    val[at] = (T)A.val[A.ptr[r] + e];
                } else {
                    col[at] = pad_col;
                }
            }
        }
    }
    // 16-bit offsets from offset_base(row) when every stored column allows
    // (padding of rows past n_rows points at the last column)
    bool fits = c->index16 && A.n_cols > 0;
    std::vector<int16_t> d16;
    if (fits) {
        d16.assign(S.stored, 0);
        for (int32_t s = 0; s < S.n_slices && fits; ++s) {
            const int32_t w = (sptr[s + 1] - sptr[s]) / kSlice;
            for (int32_t l = 0; l < kSlice && fits; ++l) {
                const int32_t r = pos2row[(size_t)(s * rows_per + l / lanes)];
                const int64_t base = offset_base(r, A.n_rows, A.n_cols);
                for (int32_t k = 0; k < w; ++k) {
                    const int64_t at = sptr[s] + (int64_t)k * kSlice + l;
                    const int64_t d = (r < A.n_rows ? (int64_t)col[at] : (int64_t)A.n_cols - 1) - base;
                    if (d < -32767 || d > 32767) {
                        fits = false;
                        break;
                    }
                    d16[at] = (int16_t)d;
                }
            }
        }
    }
    S.sptr = upload_vec(c, sptr);
    if (fits) S.d16 = upload_vec(c, d16);
    else S.col = upload_vec(c, col);
    S.val = upload_vec(c, val);
    if (sorted) {
        std::vector<uint8_t> perm((size_t)n_pos);
        for (int32_t k = 0; k < n_pos; ++k) perm[(size_t)k] = (uint8_t)(pos2row[(size_t)k] - (k / window) * window);
        S.perm = upload_vec(c, perm);
    }
    return S;
}

template Sell<double> to_sell<double>(eqs_ctx*, const Csr<double>&, int, bool);
template Sell<float> to_sell<float>(eqs_ctx*, const Csr<double>&, int, bool);

// CSR column ids: 16-bit offsets from offset_base(row) when every entry
// allows, else absolute.
template <typename T>
static void upload_csr_cols(eqs_ctx* c, SpMat<T>& S, const Csr<double>& A) {
    bool fits = c->index16 && A.n_cols > 0;
    std::vector<int16_t> d16;
    if (fits) {
        d16.resize(A.col.size());
        for (int32_t r = 0; r < A.n_rows && fits; ++r) {
            const int64_t base = offset_base(r, A.n_rows, A.n_cols);
            for (int32_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
                const int64_t d = (int64_t)A.col[k] - base;
                if (d < -32767 || d > 32767) {
                    fits = false;
                    break;
                }
                d16[k] = (int16_t)d;
            }
        }
    }
    if (fits) S.d16 = upload_vec(c, d16);
    else S.col = upload_vec(c, A.col);
}

// Layout choice: rows of up to 16 entries go one lane per row (SELL-64);
// longer rows get L = 2^ceil(log2(mean/2)) lanes (2 <= L <= 64), so each lane
// sums about two entries per pass and a wavefront covers 64/L rows.
// Whether storing the rows of a one-lane-per-row SELL operator longest first
// within each 256-row window (a row order) pays: when it saves a tenth of the
// stored entries. Rows of different lengths that alternate (the vertex and
// edge nodes of second-order tets: 1.57 stored entries per nonzero in the
// natural order, 1.10 sorted) gain; the nearly uniform rows of first-order
// tets (1.01) do not.
static bool row_order_pays(const Csr<double>& A) {
    const int32_t n = A.n_rows;
    if (n <= 0) return false;
    auto len = [&](int32_t r) { return r < n ? A.ptr[r + 1] - A.ptr[r] : 0; };
    const int32_t n_pos = ((n + kSlice - 1) / kSlice) * kSlice;
    int64_t plain = 0, sorted = 0;
    std::vector<int32_t> w;
    for (int32_t w0 = 0; w0 < n_pos; w0 += 4 * kSlice) {
        const int32_t w1 = std::min(n_pos, w0 + 4 * kSlice);
        w.clear();
        for (int32_t r = w0; r < w1; ++r) w.push_back(len(r));
        for (int32_t s0 = 0; s0 < (int32_t)w.size(); s0 += kSlice)
            plain += (int64_t)kSlice * *std::max_element(w.begin() + s0, w.begin() + std::min((int32_t)w.size(), s0 + kSlice));
        std::sort(w.begin(), w.end(), std::greater<int32_t>());
        for (int32_t s0 = 0; s0 < (int32_t)w.size(); s0 += kSlice) sorted += (int64_t)kSlice * w[(size_t)s0];
    }
    return sorted * 10 <= plain * 9;
}

template <typename T>
SpMat<T> to_spmat(eqs_ctx* c, const Csr<double>& A) {
    SpMat<T> S;
    S.n_rows = A.n_rows;
    S.n_cols = A.n_cols;
    S.nnz = A.nnz();
    const double mean = A.n_rows ? (double)A.nnz() / A.n_rows : 0.0;
    if (mean <= 16.0) {
        S.fmt = FMT_SELL;
        S.sell = to_sell<T>(c, A, 1);
        return S;
    }
    S.fmt = FMT_CSR;
    int L = 2;
    while (L < 64 && L < mean / 2.0) L *= 2;
    S.lanes = L;
    std::vector<T> v(A.val.size());
    for (size_t k = 0; k < v.size(); ++k) v[k] = (T)A.val[k];
    S.rowptr = upload_vec(c, A.ptr);
    upload_csr_cols(c, S, A);
    S.val = upload_vec(c, v);
    return S;
}
template SpMat<double> to_spmat<double>(eqs_ctx*, const Csr<double>&);
template SpMat<float> to_spmat<float>(eqs_ctx*, const Csr<double>&);

template <typename T>
static void free_spmat(eqs_ctx* c, SpMat<T>& S) {
    dev_free(c, S.sell.sptr);
    dev_free(c, S.sell.col);
    dev_free(c, S.sell.d16);
    dev_free(c, S.sell.val);
    dev_free(c, S.sell.perm);
    dev_free(c, S.rowptr);
    dev_free(c, S.col);
    dev_free(c, S.d16);
    dev_free(c, S.val);
    S = SpMat<T>{};
}

// Autotuner: upload the operator in every candidate layout (SELL with 1 lane
// per row, and with 2, 4, 8 while each lane keeps 1.5 entries or more, each
// also with rows sorted by length within 256-thread windows (the products and
// the smoothers write only rows of their own window);
// CSR with L = 2..64 lanes per row up to about twice the mean row length, and
// with one lane per row for rows of up to 8 entries on average), time y = A x
// with HIP events on the context's stream (median of 5 rounds of 8 back-to-back launches, after a warm-up round) and
// keep the fastest.
template <typename T>
static SpMat<T> tuned_spmat(eqs_ctx* c, const Csr<double>& A, const char* what, bool sell_only = false,
                             bool allow_sorted = false) {
    if (sell_only) {  // the finest operator: its post-smoothing kernel writes per-block CG partials
        SpMat<T> S;
        S.n_rows = A.n_rows; S.n_cols = A.n_cols; S.nnz = A.nnz();
        S.fmt = FMT_SELL;
        S.sell = to_sell<T>(c, A, 1, row_order_pays(A));
        S.sell.xcd = 1;  // the finest smoothers walk their row blocks in the XCD order (row_block in sell.h)
        c->tune_log += std::string(what) + ": sell64" + (S.sell.perm ? "s" : "") + " (finest level), " +
                       (S.sell.d16 ? "16-bit column offsets\n" : "32-bit columns\n");
        return S;
    }
    if (c->force_layout >= 0) {
        SpMat<T> S;
        if (c->force_layout == 0) {
            S = to_spmat<T>(c, A);
            if (S.fmt == FMT_SELL) {  // short rows: CSR with 2 lanes
                free_spmat(c, S);
                S.n_rows = A.n_rows; S.n_cols = A.n_cols; S.nnz = A.nnz();
                S.fmt = FMT_CSR;
                S.lanes = 2;
                std::vector<T> v(A.val.size());
                for (size_t k = 0; k < v.size(); ++k) v[k] = (T)A.val[k];
                S.rowptr = upload_vec(c, A.ptr);
                upload_csr_cols(c, S, A);
                S.val = upload_vec(c, v);
            }
        } else {
            S.n_rows = A.n_rows; S.n_cols = A.n_cols; S.nnz = A.nnz();
            S.fmt = FMT_SELL;
            S.sell = to_sell<T>(c, A, c->force_layout, c->force_sorted && allow_sorted);
            S.sell.unroll = c->force_unroll;
        }
        c->tune_log += std::string(what) + ": layout set by EQS_LAYOUT\n";
        return S;
    }
    if (!c->autotune || A.n_rows == 0) return to_spmat<T>(c, A);
    const double mean = (double)A.nnz() / A.n_rows;
    auto make_csr = [&](int L) {
        SpMat<T> S;
        S.n_rows = A.n_rows; S.n_cols = A.n_cols; S.nnz = A.nnz();
        S.fmt = FMT_CSR;
        S.lanes = L;
        std::vector<T> v(A.val.size());
        for (size_t k = 0; k < v.size(); ++k) v[k] = (T)A.val[k];
        S.rowptr = upload_vec(c, A.ptr);
        upload_csr_cols(c, S, A);
        S.val = upload_vec(c, v);
        return S;
    };
    const std::string key = std::string(what) + " " + std::to_string(A.n_rows) + "x" + std::to_string(A.n_cols) + " " +
                            std::to_string(A.nnz());
    {
        auto it = c->tune_replay.find(key);
        if (it != c->tune_replay.end()) {  // a recorded choice: rebuild it without timing
            char kind[8] = {0};
            int L = 0, sorted = 0, U = 8;
            const int n = std::sscanf(it->second.c_str(), "%7s %d %d %d", kind, &L, &sorted, &U);
            SpMat<T> S;
            if (n >= 2 && std::string(kind) == "csr" && L >= 1 && L <= 64 && (L & (L - 1)) == 0) {
                S = make_csr(L);
            } else if (n == 4 && std::string(kind) == "sell" && (L == 1 || L == 2 || L == 4 || L == 8) &&
                       (U == 4 || U == 8 || U == 16)) {
                S.n_rows = A.n_rows; S.n_cols = A.n_cols; S.nnz = A.nnz();
                S.fmt = FMT_SELL;
                S.sell = to_sell<T>(c, A, L, sorted != 0 && allow_sorted);
                S.sell.unroll = U;
            } else {
                fail(EQS_ERR_INVALID_ARG, "tuning record: bad entry for " + key + ": " + it->second);
            }
            c->tune_log += key + " -> " + it->second + " (tuning record)\n";
            return S;
        }
    }
    T* x = (T*)dev_alloc(c, sizeof(T) * std::max<int32_t>(A.n_cols, 1));
    T* y = (T*)dev_alloc(c, sizeof(T) * std::max<int32_t>(A.n_rows, 1));
    {
        std::vector<T> ones(std::max<int32_t>(A.n_cols, 1), T(1));
        EQS_HIP(hipMemcpy(x, ones.data(), sizeof(T) * ones.size(), hipMemcpyHostToDevice));
    }
    SpMat<T> best;
    double best_ms = 1e300;
    std::string best_name;
    std::string tried;
    auto consider = [&](SpMat<T> cand, const std::string& name) {
        const double ms = time_mv<T>(c, cand, x, y, 5);
        if (c->tune_verbose) {
            char t[96];
            std::snprintf(t, sizeof t, " %s %.1f", name.c_str(), ms * 1e3);
            tried += t;
        }
        if (ms < best_ms) {
            if (best.n_rows || best.nnz) free_spmat(c, best);
            best = cand;
            best_ms = ms;
            best_name = name;
        } else {
            free_spmat(c, cand);
        }
    };
    for (int L = 1; L <= 8; L *= 2) {
        if (L > 1 && mean < 1.5 * L) break;  // lanes with about one entry or less
        for (int sorted = 0; sorted <= (allow_sorted ? 1 : 0); ++sorted) {
            SpMat<T> S;
            S.n_rows = A.n_rows; S.n_cols = A.n_cols; S.nnz = A.nnz();
            S.fmt = FMT_SELL;
            S.sell = to_sell<T>(c, A, L, sorted != 0);
            // the group size, timed on the product (the coarse smoothing kernels
            // take the same; the finest level's keep 8)
            {
                const double per_lane = mean / L;
                double best_u_ms = 1e300;
                int best_u = 8;
                for (int U : {4, 8, 16}) {
                    if (U == 16 && per_lane < 6.0) continue;
                    S.sell.unroll = U;
                    const double ms = time_mv<T>(c, S, x, y, 5);
                    if (c->tune_verbose) {
                        char t[64];
                        std::snprintf(t, sizeof t, " [u%d %.1f]", U, ms * 1e3);
                        tried += t;
                    }
                    if (ms < best_u_ms) {
                        best_u_ms = ms;
                        best_u = U;
                    }
                }
                S.sell.unroll = best_u;
            }
            consider(S, std::string("sell64") + (L > 1 ? "x" + std::to_string(L) : "") + (sorted ? "s" : "") +
                            (S.sell.d16 ? "/i16" : "") + (S.sell.unroll != 8 ? "/u" + std::to_string(S.sell.unroll) : ""));
        }
    }
    for (int L = (mean <= 8.0 ? 1 : 2); L <= 64; L *= 2) {
        if (L > 2 && L / 2 > 2.0 * mean) break;
        SpMat<T> S;
        S.n_rows = A.n_rows; S.n_cols = A.n_cols; S.nnz = A.nnz();
        S.fmt = FMT_CSR;
        S.lanes = L;
        std::vector<T> v(A.val.size());
        for (size_t k = 0; k < v.size(); ++k) v[k] = (T)A.val[k];
        S.rowptr = upload_vec(c, A.ptr);
        upload_csr_cols(c, S, A);
        S.val = upload_vec(c, v);
        consider(S, std::string("csr") + std::to_string(L) + (S.d16 ? "/i16" : ""));
    }
    dev_free(c, x);
    dev_free(c, y);
    if (best.fmt == FMT_CSR)
        c->tune_record.push_back(key + "\tcsr " + std::to_string(best.lanes));
    else
        c->tune_record.push_back(key + "\tsell " + std::to_string(best.sell.lanes) + " " +
                                 std::to_string(best.sell.perm ? 1 : 0) + " " + std::to_string(best.sell.unroll));
    char line[200];
    const double fill = best.fmt == FMT_SELL && A.nnz() > 0 ? (double)best.sell.stored / (double)A.nnz() : 1.0;
    std::snprintf(line, sizeof line, "%s: %d x %d, %.1f nnz/row -> %s (%.1f us, stored/nnz %.2f)\n", what, A.n_rows,
                  A.n_cols, mean, best_name.c_str(), best_ms * 1e3, fill);
    c->tune_log += line;
    if (c->tune_verbose) c->tune_log += "  tried (us):" + tried + "\n";
    return best;
}

// Values a_ij omega / a_jj of A omega D^{-1} in the storage order of the
// uploaded layout S of A (same structure, so the same positions).
template <typename T>
static T* scaled_values(eqs_ctx* c, const SpMat<T>& S, const Csr<double>& A, const std::vector<double>& d,
                        double omega) {
    Csr<double> As = A;
    for (size_t k = 0; k < As.val.size(); ++k) As.val[k] = A.val[k] * omega / d[A.col[k]];
    if (S.fmt == FMT_SELL) {  // the same layout (the row order depends on the pattern only)
        Sell<T> t = to_sell<T>(c, As, S.sell.lanes, S.sell.perm != nullptr);
        dev_free(c, t.sptr);
        dev_free(c, t.col);
        dev_free(c, t.d16);
        dev_free(c, t.perm);
        return t.val;
    }
    std::vector<T> v(As.val.size());
    for (size_t k = 0; k < v.size(); ++k) v[k] = (T)As.val[k];
    return upload_vec(c, v);
}

template <typename T>
static void upload_coarse_tail(eqs_ctx* c, const AmgHost& ah, Hierarchy<T>& h);

// Whether the level above the coarsest is folded with it (see upload_coarse_tail).
static bool coarse_tail_applies(const eqs_ctx* c, const AmgHost& ah) {
    const size_t L = ah.A.size();
    return c->fold && L >= 3 && (int64_t)ah.A[L - 1].n_rows * ah.A[L - 2].n_rows <= kMaxCoarseR;
}

// R (I - A w D^-1) = R - w (R A) D^-1 (rows in column order): the restriction
// of a level whose pre-smoother x = w D^-1 b, res = b - A x is folded into it.
static Csr<double> fold_presmoother(const Csr<double>& R, const Csr<double>& A, const std::vector<double>& d,
                                    double w) {
    Csr<double> out;
    out.n_rows = R.n_rows;
    out.n_cols = R.n_cols;
    out.ptr.assign((size_t)R.n_rows + 1, 0);
    std::vector<double> acc((size_t)R.n_cols, 0.0);
    std::vector<char> seen((size_t)R.n_cols, 0);
    std::vector<int32_t> cols;
    auto touch = [&](int32_t j) {
        if (!seen[j]) {
            seen[j] = 1;
            cols.push_back(j);
        }
    };
    for (int32_t i = 0; i < R.n_rows; ++i) {
        cols.clear();
        for (int32_t e = R.ptr[i]; e < R.ptr[i + 1]; ++e) {
            touch(R.col[e]);
            acc[R.col[e]] += R.val[e];
        }
        for (int32_t e = R.ptr[i]; e < R.ptr[i + 1]; ++e) {
            const int32_t k = R.col[e];
            const double rk = w * R.val[e];
            for (int32_t f = A.ptr[k]; f < A.ptr[k + 1]; ++f) {
                const int32_t j = A.col[f];
                touch(j);
                acc[j] -= rk * A.val[f] / d[j];
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t j : cols) {
            out.col.push_back(j);
            out.val.push_back(acc[j]);
            acc[j] = 0.0;
            seen[j] = 0;
        }
        out.ptr[(size_t)i + 1] = (int32_t)out.col.size();
    }
    return out;
}

template <typename T>
static void upload_hierarchy(eqs_ctx* c, const AmgHost& ah, Hierarchy<T>& h, const double* level0_M_vals_hint) {
    (void)level0_M_vals_hint;
    const size_t L = ah.A.size();
    const bool tail_ok = coarse_tail_applies(c, ah);
    h.lv.resize(L);
    for (size_t l = 0; l < L; ++l) {
        Level<T>& lv = h.lv[l];
        lv.n = ah.A[l].n_rows;
        // coarse operators may take a row order too: their smoothers write only rows of their own window
        lv.A = tuned_spmat<T>(c, ah.A[l], ("A" + std::to_string(l)).c_str(), l == 0, l > 0);
        std::vector<double> d = diagonal(ah.A[l]);
        std::vector<T> dinv(lv.n);
        for (int32_t i = 0; i < lv.n; ++i) dinv[i] = (T)(1.0 / d[i]);
        lv.dinv = upload_vec(c, dinv);
        lv.omega = ah.omega[l];
        lv.b = (T*)dev_alloc(c, sizeof(T) * lv.n);
        lv.x = (T*)dev_alloc(c, sizeof(T) * lv.n);
        lv.xs = (T*)dev_alloc(c, sizeof(T) * lv.n);
        lv.res = (T*)dev_alloc(c, sizeof(T) * lv.n);
        if (l + 1 < L) {
            // levels other than the finest (whose smoothers feed CG) and the
            // folded tail restrict b through R (I - A w D^-1)
            const bool tail_level = tail_ok && l == (int)L - 2;
            lv.fold_pre = c->fold && l >= 1 && !tail_level;
            if (!lv.fold_pre) lv.sval = scaled_values<T>(c, lv.A, ah.A[l], d, lv.omega);
            lv.P = tuned_spmat<T>(c, ah.P[l], ("P" + std::to_string(l)).c_str(), false, true);
            if (lv.fold_pre)
                lv.R = tuned_spmat<T>(c, fold_presmoother(ah.R[l], ah.A[l], d, lv.omega),
                                      ("R" + std::to_string(l) + "(I-AwD^-1)").c_str(), false, true);
            else
                lv.R = tuned_spmat<T>(c, ah.R[l], ("R" + std::to_string(l)).c_str(), false, true);
        } else {
            std::vector<T> inv(ah.coarse_inv.size());
            for (size_t k = 0; k < inv.size(); ++k) inv[k] = (T)ah.coarse_inv[k];
            lv.dense_inv = upload_vec(c, inv);
        }
    }
    upload_coarse_tail<T>(c, ah, h);
}

// The two lowest levels folded into two products (formed in FP64 here). With
// t = L-2 (the level above the coarsest c = L-1), S = I - w D^-1 A_t and
// T = I - A_t w D^-1, one V(1,1) visit of t with the exact coarse solve is
//   x_c = C' b_t,            C' = A_c^-1 R_t T       (dense n_c x n_t)
//   xs_t = G b_t + Q x_c,    G = (S + I) w D^-1 (A_t's pattern), Q = S P_t
// so the pre-smoother, restriction, coarse solve, prolongation and
// post-smoother of t become one dense and one sparse product, [G Q] acting on
// the stacked vector [b_t; x_c]. Only when t is not the finest level (whose
// post-smoother produces CG partials) and C' is small; with two levels only
// the restriction is folded into the coarse solve (x_c = A_c^-1 R_0 r_0).
template <typename T>
static void upload_coarse_tail(eqs_ctx* c, const AmgHost& ah, Hierarchy<T>& h) {
    const int L = (int)h.lv.size();
    if (L < 2 || !c->fold) return;
    Level<T>& lc = h.lv[L - 1];
    const int t = L - 2;
    const Csr<double>& R = ah.R[t];
    const int64_t nc = lc.n, nt = R.n_cols;
    if (nc * nt > kMaxCoarseR) return;
    auto inv = [&](int64_t i, int64_t k) { return ah.coarse_inv[(size_t)(k * nc + i)]; };  // column-major
    // C = A_c^-1 R_t (dense, row-major nc x nt)
    std::vector<double> C((size_t)(nc * nt), 0.0);
    for (int32_t k = 0; k < R.n_rows; ++k)
        for (int32_t e = R.ptr[k]; e < R.ptr[k + 1]; ++e)
            for (int64_t i = 0; i < nc; ++i) C[(size_t)(i * nt + R.col[e])] += inv(i, k) * R.val[e];
    if (t == 0) {  // finest level above the coarsest: fold the restriction only
        std::vector<T> Ct(C.size());
        for (size_t k = 0; k < C.size(); ++k) Ct[k] = (T)C[k];
        lc.coarse_R = upload_vec(c, Ct);
        lc.coarse_R_cols = (int32_t)nt;
        return;
    }
    Level<T>& lt = h.lv[t];
    const Csr<double>& A = ah.A[t];
    const Csr<double>& P = ah.P[t];
    const std::vector<double> d = diagonal(A);
    const double w = ah.omega[t];
    // C' = C - w C A D^-1: row i of C A is sum_k C(i,k) A(k,:)
    std::vector<double> Cp = C;
    for (int32_t k = 0; k < A.n_rows; ++k)
        for (int32_t e = A.ptr[k]; e < A.ptr[k + 1]; ++e) {
            const int32_t j = A.col[e];
            const double f = w * A.val[e] / d[j];
            for (int64_t i = 0; i < nc; ++i) Cp[(size_t)(i * nt + j)] -= C[(size_t)(i * nt + k)] * f;
        }
    // [G Q]: row i holds G's entries (columns j < nt) then Q's nonzeros
    // (columns nt + k), Q = P - w D^-1 A P
    Csr<double> GQ;
    GQ.n_rows = (int32_t)nt;
    GQ.n_cols = (int32_t)(nt + nc);
    GQ.ptr.assign((size_t)nt + 1, 0);
    std::vector<double> q((size_t)nc);
    for (int32_t i = 0; i < (int32_t)nt; ++i) {
        for (int32_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
            const int32_t j = A.col[e];
            const double g = (j == i ? 2.0 * w / d[i] : 0.0) - w * w * A.val[e] / (d[i] * d[j]);
            GQ.col.push_back(j);
            GQ.val.push_back(g);
        }
        std::fill(q.begin(), q.end(), 0.0);
        for (int32_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) q[P.col[e]] += P.val[e];
        for (int32_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
            const int32_t k = A.col[e];
            const double f = w * A.val[e] / d[i];
            for (int32_t u = P.ptr[k]; u < P.ptr[k + 1]; ++u) q[P.col[u]] -= f * P.val[u];
        }
        for (int64_t k = 0; k < nc; ++k)
            if (q[(size_t)k] != 0.0) {
                GQ.col.push_back((int32_t)(nt + k));
                GQ.val.push_back(q[(size_t)k]);
            }
        GQ.ptr[(size_t)i + 1] = (int32_t)GQ.col.size();
    }
    std::vector<T> Ct(Cp.size());
    for (size_t k = 0; k < Cp.size(); ++k) Ct[k] = (T)Cp[k];
    lc.coarse_R = upload_vec(c, Ct);
    lc.coarse_R_cols = (int32_t)nt;
    lt.GQ = tuned_spmat<T>(c, GQ, ("[G Q]" + std::to_string(t)).c_str(), false, true);
    // b_t and x_c side by side: the restriction from above writes b_t, the
    // dense product writes x_c, the sparse product reads both
    T* bx = (T*)dev_alloc(c, sizeof(T) * (size_t)(nt + nc));
    dev_free(c, lt.b);  // the separate vectors they replace
    dev_free(c, lc.x);
    lt.b = bx;
    lc.x = bx + nt;
    lt.tail = true;
}

// Morton key of a point quantised to 21 bits per axis inside the box [lo, hi].
static uint64_t morton3(const double* p, const double* lo, const double* inv_ext) {
    uint64_t key = 0;
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        double f = (p[d] - lo[d]) * inv_ext[d];
        f = std::min(std::max(f, 0.0), 1.0);
        q[d] = (uint32_t)(f * 2097151.0);
    }
    for (int bit = 20; bit >= 0; --bit)
        for (int d = 0; d < 3; ++d) key = (key << 1) | ((q[d] >> bit) & 1u);
    return key;
}

// Element blocks for the fused element pass: tets sorted by instance, then by
// the Morton code of their centroid, cut into blocks of kTetBlock * tpt tets;
// per block the sorted distinct internal node ids and, per tet, a 64-bit
// record: 16-bit material, then the four 12-bit block-local vertex ids.
struct ElementBlocks {
    std::vector<uint64_t> pack;
    std::vector<int32_t> boff, bnodes;
    int32_t max_nodes = 0;
};

static std::vector<int32_t> morton_tet_order(const eqs_ctx* c) {
    const int64_t T = c->n_tets;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < c->n_nodes; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], c->xyz[3 * i + d]);
            hi[d] = std::max(hi[d], c->xyz[3 * i + d]);
        }
    double inv_ext[3];
    for (int d = 0; d < 3; ++d) inv_ext[d] = hi[d] > lo[d] ? 1.0 / (hi[d] - lo[d]) : 0.0;
    std::vector<std::pair<uint64_t, int32_t>> key(T);
    std::vector<int32_t> tinst(T, 0);
    for (int64_t i = 0; i < c->n_inst; ++i)
        for (int64_t e = c->inst_tet_off[i]; e < c->inst_tet_off[i + 1]; ++e) tinst[e] = (int32_t)i;
    for (int64_t e = 0; e < T; ++e) {
        double cen[3] = {0, 0, 0};
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 3; ++d) cen[d] += 0.25 * c->xyz[3 * (int64_t)c->tets[(int64_t)c->npe * e + a] + d];
        key[e] = {morton3(cen, lo, inv_ext), (int32_t)e};
    }
    // instance first (blocks then never mix instances, whose meshes may overlap in space)
    std::stable_sort(key.begin(), key.end(),
                     [&](const std::pair<uint64_t, int32_t>& x, const std::pair<uint64_t, int32_t>& y) {
                         if (tinst[x.second] != tinst[y.second]) return tinst[x.second] < tinst[y.second];
                         return x.first < y.first;
                     });
    std::vector<int32_t> order(T);
    for (int64_t k = 0; k < T; ++k) order[k] = key[k].second;
    return order;
}

// Second-order tets take two 64-bit words per record: 16-bit material, then
// the ten 11-bit block-local ids at bits 16 + 11 k of the 128-bit pair (low
// word first).
static ElementBlocks element_blocks(const eqs_ctx* c, const std::vector<int32_t>& u2i,
                                    const std::vector<int32_t>& order, int tpt) {
    const int64_t T = c->n_tets, per = (int64_t)kTetBlock * tpt;
    const int64_t nb = (T + per - 1) / per;
    const int npe = c->npe, words = npe == 4 ? 1 : 2;
    ElementBlocks eb;
    eb.pack.assign((size_t)(nb * per * words), ~0ull);  // whole blocks; padding records are skipped
    eb.boff.assign(nb + 1, 0);
    eb.bnodes.reserve((size_t)T);
    std::vector<int32_t> ids;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t e0 = b * per, e1 = std::min<int64_t>(T, e0 + per);
        ids.clear();
        for (int64_t k = e0; k < e1; ++k)
            for (int a = 0; a < npe; ++a) ids.push_back(u2i[c->tets[npe * (int64_t)order[k] + a]]);
        std::sort(ids.begin(), ids.end());
        ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
        if (ids.size() > (size_t)kMaxBlockNodes) {  // local ids / LDS: the caller tries a smaller block
            eb.max_nodes = INT32_MAX;
            return eb;
        }
        eb.max_nodes = std::max<int32_t>(eb.max_nodes, (int32_t)ids.size());
        for (int64_t k = e0; k < e1; ++k) {
            const int32_t e = order[k];
            uint64_t w = (uint64_t)(uint16_t)c->tet_mat[e], w2 = 0;
            for (int a = 0; a < npe; ++a) {
                const uint64_t loc =
                    (uint64_t)(std::lower_bound(ids.begin(), ids.end(), u2i[c->tets[npe * (int64_t)e + a]]) - ids.begin());
                if (npe == 4) {
                    w |= loc << (16 + 12 * a);
                } else {
                    const int pos = 16 + 11 * a;
                    if (pos < 64) w |= loc << pos;
                    if (pos + 11 > 64) w2 |= pos >= 64 ? loc << (pos - 64) : loc >> (64 - pos);
                }
            }
            eb.pack[k * words] = w;
            if (words == 2) eb.pack[k * words + 1] = w2;
        }
        eb.bnodes.insert(eb.bnodes.end(), ids.begin(), ids.end());
        if (eb.bnodes.size() > (size_t)INT32_MAX) fail(EQS_ERR_INVALID_ARG, "too many block nodes");
        eb.boff[b + 1] = (int32_t)eb.bnodes.size();
    }
    return eb;
}

// Lists of the deterministic element pass (k_kx_det, k_kx_gather) from the
// blocks: slot 4 t + a is vertex a of the block's record t; a node's slots and
// a node's block occurrences are listed in increasing order (counting sorts).
static void install_det_lists(eqs_ctx* c, const ElementBlocks& eb, int tpt) {
    const int64_t nb = c->n_blocks, per = (int64_t)kTetBlock * tpt, NB = (int64_t)eb.bnodes.size();
    std::vector<uint16_t> kslots((size_t)(nb * per * 4), 0), kend((size_t)NB, 0);
    std::vector<int32_t> pos;
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t off = eb.boff[b], nn = eb.boff[b + 1] - off;
        pos.assign((size_t)nn + 1, 0);
        for (int64_t t = 0; t < per; ++t) {
            const uint64_t w = eb.pack[(size_t)(b * per + t)];
            if (w == ~0ull) continue;
            for (int a = 0; a < 4; ++a) pos[((w >> (16 + 12 * a)) & 0xfffu) + 1]++;
        }
        for (int32_t k = 0; k < nn; ++k) {
            pos[k + 1] += pos[k];
            kend[(size_t)(off + k)] = (uint16_t)pos[k + 1];
        }
        uint16_t* sl = kslots.data() + b * per * 4;
        for (int64_t t = 0; t < per; ++t) {
            const uint64_t w = eb.pack[(size_t)(b * per + t)];
            if (w == ~0ull) continue;
            for (int a = 0; a < 4; ++a) sl[pos[(w >> (16 + 12 * a)) & 0xfffu]++] = (uint16_t)(4 * t + a);
        }
    }
    std::vector<int32_t> occ_off((size_t)c->n_nodes + 1, 0), occ((size_t)NB);
    for (int64_t p = 0; p < NB; ++p) occ_off[(size_t)eb.bnodes[p] + 1]++;
    for (int64_t i = 0; i < c->n_nodes; ++i) occ_off[i + 1] += occ_off[i];
    std::vector<int32_t> fill(occ_off.begin(), occ_off.end() - 1);
    for (int64_t p = 0; p < NB; ++p) occ[(size_t)fill[eb.bnodes[p]]++] = (int32_t)p;
    c->d_kslots = upload_vec(c, kslots);
    c->d_kend = upload_vec(c, kend);
    c->d_occ_off = upload_vec(c, occ_off);
    c->d_occ = upload_vec(c, occ);
    c->d_kx_part = (double*)dev_alloc(c, sizeof(double) * (size_t)std::max<int64_t>(NB, 1));
}

static void install_blocks(eqs_ctx* c, const ElementBlocks& eb, int tpt) {
    if (c->d_tpack) { dev_free(c, c->d_tpack); dev_free(c, c->d_bnodes); dev_free(c, c->d_boff); }
    if (c->d_kslots) {
        for (void* q : {(void*)c->d_kslots, (void*)c->d_kend, (void*)c->d_occ_off, (void*)c->d_occ, (void*)c->d_kx_part})
            dev_free(c, q);
        c->d_kslots = nullptr; c->d_kend = nullptr; c->d_occ_off = nullptr; c->d_occ = nullptr; c->d_kx_part = nullptr;
    }
    c->n_blocks = (int64_t)eb.boff.size() - 1;
    c->max_block_nodes = eb.max_nodes;
    c->n_block_nodes = (int64_t)eb.bnodes.size();
    c->tet_tpt = tpt;
    c->d_tpack = upload_vec(c, eb.pack);
    c->d_bnodes = upload_vec(c, eb.bnodes);
    c->d_boff = upload_vec(c, eb.boff);
    if (c->deterministic) {
        if (c->npe != 4) fail(EQS_ERR_INVALID_ARG, "the deterministic element pass is built for first-order tets");
        install_det_lists(c, eb, tpt);
    }
}

// Blocks of 256 tets per workgroup trade LDS reuse (each block re-reads the
// nodes it shares with its neighbours) against parallelism; with autotuning
// on, every block size that fits the local ids is timed on the RHS pass and
// the fastest kept (else 4 tets per thread).
void build_element_blocks(eqs_ctx* c, const std::vector<int32_t>& u2i, const double* yfree, double* out) {
    const std::vector<int32_t> order = morton_tet_order(c);
    const int fixed = c->npe == 4 ? 4 : 1;
    if (!c->autotune || c->n_tets < 16 * (int64_t)kTetBlock * kMaxTetsPerThread) {
        for (int tpt = fixed; tpt >= 1; tpt /= 2) {
            ElementBlocks eb = element_blocks(c, u2i, order, tpt);
            if (eb.max_nodes <= kMaxBlockNodes) {
                install_blocks(c, eb, tpt);
                c->tune_log += "element: " + std::to_string(kTetBlock * tpt) + " tets per block\n";
                return;
            }
        }
        fail(EQS_ERR_INVALID_ARG, "element block of 256 tets with more than " + std::to_string(kMaxBlockNodes) +
                                      " distinct nodes");
    }
    const std::string key = "element " + std::to_string(c->n_tets) + " " + std::to_string(c->npe);
    {
        auto it = c->tune_replay.find(key);
        if (it != c->tune_replay.end()) {  // a recorded block size
            const int tpt = std::atoi(it->second.c_str());
            if (tpt < 1 || tpt > kMaxTetsPerThread || (tpt & (tpt - 1)))
                fail(EQS_ERR_INVALID_ARG, "tuning record: bad entry for " + key + ": " + it->second);
            ElementBlocks eb = element_blocks(c, u2i, order, tpt);
            if (eb.max_nodes > kMaxBlockNodes) fail(EQS_ERR_INVALID_ARG, "tuning record: " + key + " does not fit");
            install_blocks(c, eb, tpt);
            c->tune_log += "element: " + std::to_string(kTetBlock * tpt) + " tets per block (tuning record)\n";
            return;
        }
    }
    int best_tpt = 0;
    double best = 1e300;
    std::string line = "element:";
    const int max_tpt = c->npe == 4 ? kMaxTetsPerThread : 2;  // second order: ~1.3 nodes per tet
    for (int tpt = 1; tpt <= max_tpt; tpt *= 2) {
        ElementBlocks eb = element_blocks(c, u2i, order, tpt);
        if (eb.max_nodes > kMaxBlockNodes) break;
        install_blocks(c, eb, tpt);
        const double ms = time_kx(c, yfree, out, 5);
        char buf[64];
        std::snprintf(buf, sizeof buf, " %d:%.1fus", kTetBlock * tpt, 1e3 * ms);
        line += buf;
        if (ms < best) {
            best = ms;
            best_tpt = tpt;
        }
    }
    if (best_tpt == 0)
        fail(EQS_ERR_INVALID_ARG, "element block of 256 tets with more than " + std::to_string(kMaxBlockNodes) +
                                      " distinct nodes");
    if (best_tpt != c->tet_tpt) install_blocks(c, element_blocks(c, u2i, order, best_tpt), best_tpt);
    c->tune_log += line + " -> " + std::to_string(kTetBlock * best_tpt) + " tets per block\n";
    c->tune_record.push_back(key + "\t" + std::to_string(best_tpt));
}

void upload(eqs_ctx* c) {
    const int64_t N = c->n_nodes, T = c->n_tets, NF = c->n_free;
    std::vector<int32_t> u2i(N);
    for (int64_t i = 0; i < N; ++i) u2i[c->int_to_user[i]] = (int32_t)i;

    std::vector<double> px(N), py(N), pz(N);
    for (int64_t i = 0; i < N; ++i) {
        const double* p = &c->xyz[3 * (int64_t)c->int_to_user[i]];
        px[i] = p[0];
        py[i] = p[1];
        pz[i] = p[2];
    }
    std::vector<MatDev> md(c->mats.size());
    for (size_t m = 0; m < c->mats.size(); ++m) {
        const eqs_material& s = c->mats[m];
        md[m].eps = kEps0 * s.eps_r;
        md[m].kappa0 = s.kappa0;
        md[m].inv_es = s.nonlinear ? 1.0 / s.e_s : 0.0;
        md[m].alpha = s.alpha;
        md[m].nonlinear = s.nonlinear ? 1 : 0;
        md[m].ialpha = (s.alpha == std::floor(s.alpha) && s.alpha >= 0 && s.alpha <= 64) ? (int32_t)s.alpha : -1;
    }
    std::vector<int32_t> dd(c->n_dir);
    {
        std::vector<int32_t> drive_of(N, -1);
        for (size_t k = 0; k < c->dir_nodes.size(); ++k) drive_of[c->dir_nodes[k]] = c->dir_drive[k];
        for (int64_t k = 0; k < c->n_dir; ++k) dd[k] = drive_of[c->int_to_user[NF + k]];
    }
    c->d_cx = upload_vec(c, px);
    c->d_cy = upload_vec(c, py);
    c->d_cz = upload_vec(c, pz);
    c->d_mats = upload_vec(c, md);
    c->d_ddrive = upload_vec(c, dd);
    {
        std::vector<DriveDev> dr(c->drives.size());
        for (size_t k = 0; k < dr.size(); ++k)
            dr[k] = DriveDev{2.0 * M_PI * c->drives[k].freq, c->drives[k].amp, c->drives[k].phase, 0.0};
        c->d_drives = upload_vec(c, dr);
    }
    c->d_int_to_user = upload_vec(c, c->int_to_user);

    c->tune_log.clear();
    Csr<double> M = assemble_M_free(c);
    c->nnz_M = M.nnz();
    c->M = to_sell<double>(c, M, 1, row_order_pays(M));
    c->M.xcd = 1;  // the CG SpMV walks its row blocks in the XCD order (row_block in sell.h)
    c->tune_log += std::string("M: sell64") + (c->M.perm ? "s (rows sorted within 256-row windows)" : "") + ", " +
                   (c->M.d16 ? "16-bit column offsets\n" : "32-bit columns\n");
    AmgHost ah = build_sa_amg(M, c->amg);
    if (c->amg.precision == EQS_PREC_FP32) upload_hierarchy<float>(c, ah, c->h32, nullptr);
    else upload_hierarchy<double>(c, ah, c->h64, nullptr);

    auto vec = [&](int64_t n) { return (double*)dev_alloc(c, sizeof(double) * (size_t)n); };
    c->d_r = vec(NF); c->d_z = vec(NF); c->d_p = vec(NF); c->d_q = vec(NF); c->d_mx = vec(NF);
    c->mx_of_F = false;
    c->d_Y0 = vec(NF); c->d_Ya = vec(NF); c->d_Yb = vec(NF); c->d_Yc = vec(NF); c->d_F0 = vec(NF); c->d_F = vec(NF);
    c->d_rhs = vec(NF); c->d_rhs_alt = vec(NF); c->d_tmpN = vec(N); c->d_tmpN2 = vec(N);
    c->max_blocks = (std::max<int64_t>(N, T) + kBlock - 1) / kBlock + 1;
    c->d_partials = vec(8 * c->max_blocks);
    c->d_scal = (PcgScalars*)dev_alloc(c, sizeof(PcgScalars) * (size_t)c->n_inst);
    c->d_sum = (PcgSummary*)dev_alloc(c, sizeof(PcgSummary));
    EQS_HIP(hipMemset(c->d_sum, 0, sizeof(PcgSummary)));
    c->d_force = (int32_t*)dev_alloc(c, sizeof(int32_t));
    EQS_HIP(hipMemset(c->d_force, 0, sizeof(int32_t)));
    EQS_HIP(hipHostMalloc((void**)&c->h_scal, sizeof(PcgScalars) * (size_t)c->n_inst, hipHostMallocMapped));
    EQS_HIP(hipHostGetDevicePointer((void**)&c->d_hscal, c->h_scal, 0));
    EQS_HIP(hipHostMalloc((void**)&c->h_sum, sizeof(PcgSummary), hipHostMallocMapped));
    EQS_HIP(hipHostGetDevicePointer((void**)&c->d_hsum, c->h_sum, 0));
    c->d_inst_row = upload_vec(c, c->inst_row_off);
    {
        const int64_t nb = (NF + kBlock - 1) / kBlock;
        std::vector<int32_t> bi(std::max<int64_t>(nb, 1), 0);
        int32_t i = 0;
        for (int64_t b = 0; b < nb; ++b) {
            while (i + 1 < c->n_inst && c->inst_row_off[i + 1] <= b * kBlock) ++i;
            bi[b] = i;
        }
        c->d_blk_inst = upload_vec(c, bi);
    }
    guess_alloc_scratch(c);  // eqs_galerkin_start's dot scratch
    launch_fill(c->stream, c->d_Y0, 0.0, NF);
    build_element_blocks(c, u2i, c->d_Y0, c->d_rhs);
    if (!c->tune_file.empty() && c->tune_replay.empty() && !c->tune_record.empty()) {
        FILE* f = std::fopen(c->tune_file.c_str(), "w");
        if (!f) fail(EQS_ERR_INVALID_ARG, "tuning record: cannot write " + c->tune_file);
        for (const std::string& ln : c->tune_record) std::fprintf(f, "%s\n", ln.c_str());
        std::fclose(f);
    }
    c->tune_record.clear();
    EQS_HIP(hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming));
    EQS_HIP(hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming));
    c->have_Flast = false;
}

void free_device(eqs_ctx* c) {
    if (c->guess.tstream) (void)hipStreamSynchronize(c->guess.tstream);
    release_graphs(c);
    // the network's buffers belong to this memory too
    if (c->guess.net) {
        mlp_destroy(c->guess.net);
        c->guess.net = nullptr;
    }
    for (auto& a : c->allocations)
        if (!in_workspace(c, a.first)) (void)hipFree(a.first);
    c->allocations.clear();
    c->device_bytes = 0;
    ws_reset(c);  // a workspace stays attached, empty
    if (c->h_scal) { (void)hipHostFree(c->h_scal); c->h_scal = nullptr; c->d_hscal = nullptr; }
    if (c->h_sum) { (void)hipHostFree(c->h_sum); c->h_sum = nullptr; c->d_hsum = nullptr; }
    c->d_sum = nullptr; c->d_inst_row = nullptr; c->d_blk_inst = nullptr; c->d_force = nullptr;
    for (auto& e : c->ev)
        if (e) { (void)hipEventDestroy(e); e = nullptr; }
    c->M = Sell<double>{};
    c->stage_iters.clear();
    c->h64.lv.clear();
    c->h32.lv.clear();
    c->d_tpack = nullptr; c->d_bnodes = nullptr; c->d_boff = nullptr; c->n_blocks = 0; c->max_block_nodes = 0; c->n_block_nodes = 0;
    c->d_kslots = nullptr; c->d_kend = nullptr; c->d_occ_off = nullptr; c->d_occ = nullptr; c->d_kx_part = nullptr;
    c->d_cx = c->d_cy = c->d_cz = nullptr; c->d_mats = nullptr; c->tet_tpt = 0;
    c->d_ddrive = nullptr; c->d_int_to_user = nullptr; c->d_drives = nullptr;
    c->d_r = c->d_z = c->d_p = c->d_q = c->d_mx = nullptr;
    c->mx_of_F = false;
    c->d_Y0 = c->d_Ya = c->d_Yb = c->d_Yc = c->d_F0 = c->d_F = nullptr;
    c->d_rhs = c->d_rhs_alt = c->d_tmpN = c->d_tmpN2 = nullptr;
    c->d_partials = nullptr;
    c->d_scal = nullptr;
    c->built = false;
    c->have_Flast = false;
    c->guess.dev_ready = false;
    c->guess.d_S = c->guess.d_rprev = c->guess.d_alpha = c->guess.d_dots = c->guess.d_part = nullptr;
    c->guess.d_guard = nullptr;
    c->guess.d_gstat = nullptr;
    c->guess.d_bx = c->guess.d_bt = nullptr;
    if (!c->guess.G.empty()) guess_reset(c);
}

}  // namespace eqs
