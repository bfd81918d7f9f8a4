/*
 * Plain FP64 CPU oracle for the P1 finite-element operators of the EQS
 * problem (Richter, Schoeps, Clemens: "GPU Accelerated Explicit Time
 * Integration Methods for Electro-Quasistatic Fields", Sec. II, eq. (1)-(2),
 * and Sec. III).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It is written for reading, not for speed:
 * single-threaded element loops, one tet at a time, no blocking or fusion.
 * Only the Jacobi-preconditioned CG may spread its row loops over OpenMP
 * threads, so that reference trajectories on the 2.1M-unknown mesh finish
 * in minutes.
 *
 * Model (eq. (1)): div(kappa grad phi) + div(eps grad d(phi)/dt) = 0 with
 * P1 (linear) tetrahedral elements. On element e with vertices p0..p3 the
 * barycentric functions lambda_a have constant gradients, so
 *     A_e[a][b] = |T_e| grad(lambda_a) . grad(lambda_b)
 * is the exact element stiffness for a unit coefficient, and
 *     M   = sum_e eps_e   A_e             (constant, eq. (2))
 *     K(x)x = sum_e kappa_e(|E_e|) A_e x_e  with E_e = -sum_a x_a grad(lambda_a)
 * where the field is constant on a P1 element, so kappa_e is exact there.
 * The conductivity law is kappa0 (1 + (|E|/e_s)^alpha) for nonlinear
 * materials and kappa0 otherwise (the paper gives the qualitative law in
 * Sec. I; the power law is this project's stated reading).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EPS0 8.8541878128e-12 /* vacuum permittivity, F/m (CODATA 2018) */

/* ---------------------------------------------------------------- geometry */

/* Gradients of the barycentric functions and volume of tet (p0,p1,p2,p3).
 * J has columns p1-p0, p2-p0, p3-p0; the barycentric coordinates 1..3 of a
 * point x are J^{-1}(x - p0), so grad(lambda_k) is row k-1 of J^{-1}, and
 * grad(lambda_0) = -(sum of the other three). Returns -1 for a flat tet. */
static int tet_gradients(const double p[4][3], double grad[4][3], double *vol)
{
    double J[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            J[r][c] = p[c + 1][r] - p[0][r];

    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (det == 0.0 || !isfinite(det))
        return -1;

    /* inverse = adjugate / det; adjugate[i][j] = cofactor[j][i] */
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;

    for (int d = 0; d < 3; ++d) {
        grad[1][d] = inv[0][d];
        grad[2][d] = inv[1][d];
        grad[3][d] = inv[2][d];
        grad[0][d] = -(grad[1][d] + grad[2][d] + grad[3][d]);
    }
    *vol = fabs(det) / 6.0;
    return 0;
}

static void load_tet(const double *xyz, const int32_t *tet, double p[4][3])
{
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d)
            p[a][d] = xyz[3 * (int64_t)tet[a] + d];
}

/* A_e for the unit coefficient: A[a*4+b] = vol * grad_a . grad_b. */
int orc_element_matrix(const double *p12, double *A16, double *vol_out)
{
    double p[4][3], g[4][3], vol;
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d)
            p[a][d] = p12[3 * a + d];
    if (tet_gradients(p, g, &vol))
        return -1;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            A16[4 * a + b] = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
    if (vol_out)
        *vol_out = vol;
    return 0;
}

/* Check every tet for a nonzero volume; returns the index of the first flat
 * tet, or -1 if all are proper. */
int64_t orc_first_flat_tet(const double *xyz, int64_t n_tets, const int32_t *tets)
{
    for (int64_t e = 0; e < n_tets; ++e) {
        double p[4][3], g[4][3], vol;
        load_tet(xyz, tets + 4 * e, p);
        if (tet_gradients(p, g, &vol))
            return e;
    }
    return -1;
}

/* -------------------------------------------------------------- materials */

/* Conductivity law kappa(|E|) of a material (Sec. I; power-law reading). */
static double conductivity(double emag, double kappa0, double e_s, double alpha, int nonlinear)
{
    if (!nonlinear)
        return kappa0;
    return kappa0 * (1.0 + pow(emag / e_s, alpha));
}

/* Differential conductivity d(kappa |E|)/d|E| = kappa0 (1 + (alpha+1)(|E|/e_s)^alpha).
 * With the element matrices it bounds the Jacobian of K(x)x against M. */
static double differential_conductivity(double emag, double kappa0, double e_s, double alpha, int nonlinear)
{
    if (!nonlinear)
        return kappa0;
    return kappa0 * (1.0 + (alpha + 1.0) * pow(emag / e_s, alpha));
}

/* ------------------------------------------------------------ assembly of M */

typedef struct {
    int32_t col;
    double val;
} entry_t;

static int cmp_entry(const void *a, const void *b)
{
    int32_t ca = ((const entry_t *)a)->col, cb = ((const entry_t *)b)->col;
    return (ca > cb) - (ca < cb);
}

/* Assemble the full nodal matrix sum_e w_e A_e into CSR with sorted columns.
 * w_tet[e] is the element coefficient (for M: eps0 * eps_r of the element).
 * Call first with nnz_cap = 0 to learn the number of nonzeros (returned);
 * then with arrays of that size. Returns -1 for a flat tet, -2 on allocation
 * failure, -3 if nnz_cap is too small. */
int64_t orc_assemble(int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tets,
                     const double *w_tet, int64_t nnz_cap, int64_t *rowptr, int32_t *col, double *val)
{
    /* every tet adds a 4x4 block: row v[a] receives 4 (col, value) entries */
    int64_t *start = calloc((size_t)n_nodes + 1, sizeof(int64_t));
    if (!start)
        return -2;
    for (int64_t e = 0; e < n_tets; ++e)
        for (int a = 0; a < 4; ++a)
            start[tets[4 * e + a] + 1] += 4;
    for (int64_t i = 0; i < n_nodes; ++i)
        start[i + 1] += start[i];

    entry_t *ent = malloc((size_t)start[n_nodes] * sizeof(entry_t));
    int64_t *fill = malloc((size_t)n_nodes * sizeof(int64_t));
    if (!ent || !fill) {
        free(start); free(ent); free(fill);
        return -2;
    }
    memcpy(fill, start, (size_t)n_nodes * sizeof(int64_t));

    for (int64_t e = 0; e < n_tets; ++e) {
        const int32_t *v = tets + 4 * e;
        double p[4][3], g[4][3], vol;
        load_tet(xyz, v, p);
        if (tet_gradients(p, g, &vol)) {
            free(start); free(ent); free(fill);
            return -1;
        }
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                entry_t *en = &ent[fill[v[a]]++];
                en->col = v[b];
                en->val = w_tet[e] * vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
            }
    }

    /* sort each row by column and merge duplicates (fill mode when nnz_cap > 0) */
    int fill_mode = nnz_cap > 0;
    int64_t nnz = 0;
    int overflow = 0;
    if (fill_mode)
        rowptr[0] = 0;
    for (int64_t i = 0; i < n_nodes; ++i) {
        int64_t lo = start[i], hi = start[i + 1];
        qsort(ent + lo, (size_t)(hi - lo), sizeof(entry_t), cmp_entry);
        for (int64_t k = lo; k < hi; ++k) {
            int same = (k > lo && ent[k].col == ent[k - 1].col);
            if (!same)
                ++nnz; /* a new column opens entry nnz-1 */
            if (!fill_mode)
                continue;
            if (nnz > nnz_cap) {
                overflow = 1;
                continue;
            }
            if (same) {
                val[nnz - 1] += ent[k].val;
            } else {
                col[nnz - 1] = ent[k].col;
                val[nnz - 1] = ent[k].val;
            }
        }
        if (fill_mode)
            rowptr[i + 1] = nnz;
    }
    free(start); free(ent); free(fill);
    return overflow ? -3 : nnz;
}

/* ---------------------------------------------------------------- K(x) x */

/* y = K(x)x = sum_e kappa_e(|E_e|) A_e x_e over all nodes (Sec. III: only the
 * product is needed, never the matrix). Element materials come from a table
 * indexed by tet_mat. If max_rate is not NULL it receives
 * max_e sigma_e / eps_e, with sigma the differential conductivity, which
 * bounds the generalised spectrum of the Jacobian against M. */
int orc_apply_K(int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tets,
                const int32_t *tet_mat, const double *mat_eps_r, const double *mat_kappa0,
                const double *mat_e_s, const double *mat_alpha, const int32_t *mat_nonlinear,
                const double *x, double *y, double *max_rate)
{
    for (int64_t i = 0; i < n_nodes; ++i)
        y[i] = 0.0;
    double rate = 0.0;
    for (int64_t e = 0; e < n_tets; ++e) {
        const int32_t *v = tets + 4 * e;
        double p[4][3], g[4][3], vol;
        load_tet(xyz, v, p);
        if (tet_gradients(p, g, &vol))
            return -1;
        /* constant field on the element: E = -grad(phi) = -sum_a x_a grad(lambda_a) */
        double E[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 3; ++d)
                E[d] -= x[v[a]] * g[a][d];
        double emag = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
        int m = tet_mat[e];
        double kap = conductivity(emag, mat_kappa0[m], mat_e_s[m], mat_alpha[m], mat_nonlinear[m]);
        if (max_rate) {
            double sig = differential_conductivity(emag, mat_kappa0[m], mat_e_s[m], mat_alpha[m], mat_nonlinear[m]);
            double r = sig / (ORC_EPS0 * mat_eps_r[m]);
            if (r > rate)
                rate = r;
        }
        for (int a = 0; a < 4; ++a) {
            double s = 0.0;
            for (int b = 0; b < 4; ++b)
                s += vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]) * x[v[b]];
            y[v[a]] += kap * s;
        }
    }
    if (max_rate)
        *max_rate = rate;
    return 0;
}

/* Element conductivities kappa_e(|E_e|) of the state x, for assembling the
 * frozen matrix K(x) = sum_e kappa_e A_e used by the symmetry, definiteness
 * and spectrum checks. */
int orc_element_kappa(const double *xyz, int64_t n_tets, const int32_t *tets, const int32_t *tet_mat,
                      const double *mat_kappa0, const double *mat_e_s, const double *mat_alpha,
                      const int32_t *mat_nonlinear, const double *x, double *kappa_out)
{
    for (int64_t e = 0; e < n_tets; ++e) {
        const int32_t *v = tets + 4 * e;
        double p[4][3], g[4][3], vol;
        load_tet(xyz, v, p);
        if (tet_gradients(p, g, &vol))
            return -1;
        double E[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 3; ++d)
                E[d] -= x[v[a]] * g[a][d];
        double emag = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
        int m = tet_mat[e];
        kappa_out[e] = conductivity(emag, mat_kappa0[m], mat_e_s[m], mat_alpha[m], mat_nonlinear[m]);
    }
    return 0;
}

/* ---------------------------------------------------- second-order tets */

/* Second-order (10-node) Lagrange tetrahedra, the paper's P2 elements (Sec. III
 * and Sec. V). Local nodes: 0..3 the vertices, 4..9 the midpoints of the edges
 * (0,1), (0,2), (0,3), (1,2), (1,3), (2,3). In barycentric coordinates the
 * basis is N_a = lambda_a (2 lambda_a - 1) at vertex a and N_ab = 4 lambda_a
 * lambda_b at the midpoint of edge (a,b), with gradients
 *     grad N_a  = (4 lambda_a - 1) grad(lambda_a),
 *     grad N_ab = 4 (lambda_b grad(lambda_a) + lambda_a grad(lambda_b)),
 * linear on a straight-sided element. Element integrals use the symmetric
 * 4-point rule of degree 2: barycentric points (a, b, b, b) and permutations,
 * a = (5 + 3 sqrt 5) / 20, b = (5 - sqrt 5) / 20, weight |T| / 4 each. It is
 * exact for the product of two such gradients, so M is integrated exactly; in
 * K(x)x the field E = -grad(phi) is linear on the element and kappa(|E|) is
 * taken at the four points (this project's reading of the quadrature). */

static const int P2_EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

static void p2_point(int q, double lam[4])
{
    const double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0, b = (5.0 - sqrt(5.0)) / 20.0;
    for (int k = 0; k < 4; ++k)
        lam[k] = (k == q) ? a : b;
}

/* gradients of the 10 basis functions at barycentric point lam */
static void p2_gradients(const double g[4][3], const double lam[4], double G[10][3])
{
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d)
            G[a][d] = (4.0 * lam[a] - 1.0) * g[a][d];
    for (int e = 0; e < 6; ++e) {
        int a = P2_EDGE[e][0], b = P2_EDGE[e][1];
        for (int d = 0; d < 3; ++d)
            G[4 + e][d] = 4.0 * (lam[b] * g[a][d] + lam[a] * g[b][d]);
    }
}

/* the 4 vertices of 10-node tet e */
static void load_tet10(const double *xyz, const int32_t *tet, double p[4][3])
{
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d)
            p[a][d] = xyz[3 * (int64_t)tet[a] + d];
}

/* Unit-coefficient P2 element matrix A[i*10+j] = int grad N_i . grad N_j. */
int orc_p2_element_matrix(const double *p12, double *A100, double *vol_out)
{
    double p[4][3], g[4][3], vol;
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d)
            p[a][d] = p12[3 * a + d];
    if (tet_gradients(p, g, &vol))
        return -1;
    for (int k = 0; k < 100; ++k)
        A100[k] = 0.0;
    for (int q = 0; q < 4; ++q) {
        double lam[4], G[10][3];
        p2_point(q, lam);
        p2_gradients(g, lam, G);
        for (int i = 0; i < 10; ++i)
            for (int j = 0; j < 10; ++j)
                A100[10 * i + j] += 0.25 * vol * (G[i][0] * G[j][0] + G[i][1] * G[j][1] + G[i][2] * G[j][2]);
    }
    if (vol_out)
        *vol_out = vol;
    return 0;
}

/* Full nodal matrix sum_e sum_q w[e*4+q] (|T_e|/4) grad N_i . grad N_j at the
 * quadrature points (w = eps_e at every point for M, kappa at the point for a
 * frozen K(x)), CSR with sorted columns; the two-call protocol of
 * orc_assemble. */
int64_t orc_p2_assemble(int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tets,
                        const double *w_q, int64_t nnz_cap, int64_t *rowptr, int32_t *col, double *val)
{
    int64_t *start = calloc((size_t)n_nodes + 1, sizeof(int64_t));
    if (!start)
        return -2;
    for (int64_t e = 0; e < n_tets; ++e)
        for (int a = 0; a < 10; ++a)
            start[tets[10 * e + a] + 1] += 10;
    for (int64_t i = 0; i < n_nodes; ++i)
        start[i + 1] += start[i];
    entry_t *ent = malloc((size_t)start[n_nodes] * sizeof(entry_t));
    int64_t *fill = malloc((size_t)n_nodes * sizeof(int64_t));
    if (!ent || !fill) {
        free(start); free(ent); free(fill);
        return -2;
    }
    memcpy(fill, start, (size_t)n_nodes * sizeof(int64_t));
    for (int64_t e = 0; e < n_tets; ++e) {
        const int32_t *v = tets + 10 * e;
        double p[4][3], g[4][3], vol, A[10][10];
        load_tet10(xyz, v, p);
        if (tet_gradients(p, g, &vol)) {
            free(start); free(ent); free(fill);
            return -1;
        }
        for (int i = 0; i < 10; ++i)
            for (int j = 0; j < 10; ++j)
                A[i][j] = 0.0;
        for (int q = 0; q < 4; ++q) {
            double lam[4], G[10][3];
            p2_point(q, lam);
            p2_gradients(g, lam, G);
            double wq = w_q[4 * e + q] * 0.25 * vol;
            for (int i = 0; i < 10; ++i)
                for (int j = 0; j < 10; ++j)
                    A[i][j] += wq * (G[i][0] * G[j][0] + G[i][1] * G[j][1] + G[i][2] * G[j][2]);
        }
        for (int i = 0; i < 10; ++i)
            for (int j = 0; j < 10; ++j) {
                entry_t *en = &ent[fill[v[i]]++];
                en->col = v[j];
                en->val = A[i][j];
            }
    }
    int fill_mode = nnz_cap > 0;
    int64_t nnz = 0;
    int overflow = 0;
    if (fill_mode)
        rowptr[0] = 0;
    for (int64_t i = 0; i < n_nodes; ++i) {
        int64_t lo = start[i], hi = start[i + 1];
        qsort(ent + lo, (size_t)(hi - lo), sizeof(entry_t), cmp_entry);
        for (int64_t k = lo; k < hi; ++k) {
            int same = (k > lo && ent[k].col == ent[k - 1].col);
            if (!same)
                ++nnz;
            if (!fill_mode)
                continue;
            if (nnz > nnz_cap) {
                overflow = 1;
                continue;
            }
            if (same) {
                val[nnz - 1] += ent[k].val;
            } else {
                col[nnz - 1] = ent[k].col;
                val[nnz - 1] = ent[k].val;
            }
        }
        if (fill_mode)
            rowptr[i + 1] = nnz;
    }
    free(start); free(ent); free(fill);
    return overflow ? -3 : nnz;
}

/* y = K(x)x on 10-node tets: per element and quadrature point the field
 * E_q = -sum_j x_j grad N_j(q), kappa_q = kappa(|E_q|), and
 * y_i += (|T|/4) kappa_q grad N_i(q) . (-E_q). kappa_q (n_tets x 4, may be
 * NULL) receives the point conductivities; max_rate (may be NULL) the largest
 * sigma/eps over all points (sigma the differential conductivity). */
int orc_p2_apply_K(int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tets,
                   const int32_t *tet_mat, const double *mat_eps_r, const double *mat_kappa0,
                   const double *mat_e_s, const double *mat_alpha, const int32_t *mat_nonlinear,
                   const double *x, double *y, double *kappa_q, double *max_rate)
{
    if (y)
        for (int64_t i = 0; i < n_nodes; ++i)
            y[i] = 0.0;
    double rate = 0.0;
    for (int64_t e = 0; e < n_tets; ++e) {
        const int32_t *v = tets + 10 * e;
        double p[4][3], g[4][3], vol;
        load_tet10(xyz, v, p);
        if (tet_gradients(p, g, &vol))
            return -1;
        int m = tet_mat[e];
        for (int q = 0; q < 4; ++q) {
            double lam[4], G[10][3];
            p2_point(q, lam);
            p2_gradients(g, lam, G);
            double gphi[3] = {0.0, 0.0, 0.0}; /* grad(phi) = -E at the point */
            for (int j = 0; j < 10; ++j)
                for (int d = 0; d < 3; ++d)
                    gphi[d] += x[v[j]] * G[j][d];
            double emag = sqrt(gphi[0] * gphi[0] + gphi[1] * gphi[1] + gphi[2] * gphi[2]);
            double kap = conductivity(emag, mat_kappa0[m], mat_e_s[m], mat_alpha[m], mat_nonlinear[m]);
            if (kappa_q)
                kappa_q[4 * e + q] = kap;
            if (max_rate) {
                double sig = differential_conductivity(emag, mat_kappa0[m], mat_e_s[m], mat_alpha[m],
                                                       mat_nonlinear[m]);
                double r = sig / (ORC_EPS0 * mat_eps_r[m]);
                if (r > rate)
                    rate = r;
            }
            if (y)
                for (int i = 0; i < 10; ++i)
                    y[v[i]] += 0.25 * vol * kap * (G[i][0] * gphi[0] + G[i][1] * gphi[1] + G[i][2] * gphi[2]);
        }
    }
    if (max_rate)
        *max_rate = rate;
    return 0;
}

/* ------------------------------------------------------------- CSR algebra */

/* The CSR products, dot products and vector updates below run their loops
 * over rows with OpenMP when nthreads > 1 (each row or entry computed
 * exactly as in the serial loop; only the summation order of a dot product
 * changes). nthreads <= 1 keeps them serial. */

static void csr_matvec_t(int64_t n_rows, const int64_t *rowptr, const int32_t *col, const double *val,
                         const double *x, double *y, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads) if (nthreads > 1)
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += val[k] * x[col[k]];
        y[i] = s;
    }
}

void orc_csr_matvec(int64_t n_rows, const int64_t *rowptr, const int32_t *col, const double *val,
                    const double *x, double *y)
{
    csr_matvec_t(n_rows, rowptr, col, val, x, y, 1);
}

static double dot(int64_t n, const double *a, const double *b, int nthreads)
{
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s) num_threads(nthreads) if (nthreads > 1)
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

/* z = SGS(r): symmetric Gauss-Seidel, a forward sweep from z = 0 and a
 * backward sweep; z = (D+U)^{-1} D (D+L)^{-1} r, symmetric positive definite
 * for an SPD matrix. Serial by nature. */
static void sgs_apply(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                      const double *diag, const double *r, double *z)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = r[i];
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] < i)
                s -= val[k] * z[col[k]];
        z[i] = s / diag[i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] > i)
                s += val[k] * z[col[k]];
        z[i] -= s / diag[i];
    }
}

/* z = D^{-1} r (Jacobi). */
static void jacobi_apply(int64_t n, const double *diag, const double *r, double *z, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads) if (nthreads > 1)
    for (int64_t i = 0; i < n; ++i)
        z[i] = r[i] / diag[i];
}

enum { PREC_SGS = 0, PREC_JACOBI = 1 };

/* Preconditioned CG (Saad, Iterative Methods for Sparse Linear Systems,
 * Alg. 9.1) with the symmetric Gauss-Seidel or the Jacobi preconditioner.
 * x holds the start vector on entry and the solution on exit. Stops when the
 * true relative residual |rhs - A x| / |rhs| <= rtol (the recursive residual
 * triggers the check; if the true one disagrees the recurrence restarts from
 * it). |rhs| = 0 gives x = 0 with no iterations. Returns 0 when converged,
 * 1 when maxit was reached, -1 on breakdown (p.Ap <= 0), -2 on allocation
 * failure, -3 for a non-positive diagonal entry. */
static int pcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, const double *rhs,
               double *x, double rtol, int32_t maxit, int prec, int nt, int32_t *iters_out, double *relres_out)
{
    double *diag = malloc((size_t)n * sizeof(double));
    double *r = malloc((size_t)n * sizeof(double));
    double *z = malloc((size_t)n * sizeof(double));
    double *p = malloc((size_t)n * sizeof(double));
    double *q = malloc((size_t)n * sizeof(double));
    if (!diag || !r || !z || !p || !q) {
        free(diag); free(r); free(z); free(p); free(q);
        return -2;
    }
    int status = 0;
    for (int64_t i = 0; i < n; ++i) {
        diag[i] = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i)
                diag[i] = val[k];
        if (!(diag[i] > 0.0))
            status = -3;
    }
    int32_t it = 0;
    double relres = 0.0;
    double bnorm = sqrt(dot(n, rhs, rhs, nt));
    if (status != 0) {
        /* not SPD: nothing to iterate */
    } else if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i)
            x[i] = 0.0;
    } else {
        csr_matvec_t(n, rowptr, col, val, x, q, nt);
        for (int64_t i = 0; i < n; ++i)
            r[i] = rhs[i] - q[i];
        relres = sqrt(dot(n, r, r, nt)) / bnorm;
        double rho_prev = 0.0;
        int restart = 1;
        while (relres > rtol) {
            if (it >= maxit) {
                status = 1;
                break;
            }
            if (prec == PREC_SGS)
                sgs_apply(n, rowptr, col, val, diag, r, z);
            else
                jacobi_apply(n, diag, r, z, nt);
            double rho = dot(n, r, z, nt);
            if (restart) {
                memcpy(p, z, (size_t)n * sizeof(double));
            } else {
                double beta = rho / rho_prev;
#pragma omp parallel for schedule(static) num_threads(nt) if (nt > 1)
                for (int64_t i = 0; i < n; ++i)
                    p[i] = z[i] + beta * p[i];
            }
            restart = 0;
            csr_matvec_t(n, rowptr, col, val, p, q, nt);
            double pq = dot(n, p, q, nt);
            if (!(pq > 0.0)) {
                status = -1;
                break;
            }
            double alpha = rho / pq;
#pragma omp parallel for schedule(static) num_threads(nt) if (nt > 1)
            for (int64_t i = 0; i < n; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            rho_prev = rho;
            ++it;
            relres = sqrt(dot(n, r, r, nt)) / bnorm;
            if (relres <= rtol) {
                csr_matvec_t(n, rowptr, col, val, x, q, nt);
                for (int64_t i = 0; i < n; ++i)
                    r[i] = rhs[i] - q[i];
                relres = sqrt(dot(n, r, r, nt)) / bnorm;
                restart = 1;
            }
        }
    }
    if (iters_out)
        *iters_out = it;
    if (relres_out)
        *relres_out = relres;
    free(diag); free(r); free(z); free(p); free(q);
    return status;
}

/* CG with symmetric Gauss-Seidel preconditioning, single-threaded. */
int orc_pcg_sgs(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                const double *rhs, double *x, double rtol, int32_t maxit, int32_t *iters_out,
                double *relres_out)
{
    return pcg(n, rowptr, col, val, rhs, x, rtol, maxit, PREC_SGS, 1, iters_out, relres_out);
}

/* CG with Jacobi preconditioning; products, dots and updates on nthreads
 * OpenMP threads (the reference solver for the large meshes, where the
 * serial SGS sweeps would take minutes per solve). */
int orc_pcg_jacobi(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                   const double *rhs, double *x, double rtol, int32_t maxit, int32_t nthreads,
                   int32_t *iters_out, double *relres_out)
{
    return pcg(n, rowptr, col, val, rhs, x, rtol, maxit, PREC_JACOBI, nthreads < 1 ? 1 : nthreads, iters_out,
               relres_out);
}
