// Second-order (10-node) tetrahedra, the paper's P2 elements (Sec. III, Sec. V).
//
// Local nodes: 0..3 the vertices, 4..9 the midpoints of the edges (0,1), (0,2),
// (0,3), (1,2), (1,3), (2,3). With the cofactor vectors c_a of the vertices
// (grad lambda_a = c_a / det, see tet_cofactors and kx_tets) the basis
// gradients scaled by det are
//   G_a  = (4 lambda_a - 1) c_a,   G_ab = 4 (lambda_b c_a + lambda_a c_b).
// Element integrals use the symmetric 4-point rule of degree 2: point q has
// barycentric coordinates lambda_q = kP2A and kP2B for the other three, weight
// |T| / 4; it integrates G_i . G_j exactly. So, with w = sum_i u_i G_i at a
// point (det times grad phi), the element's contribution to node i is
//   sum_q kappa_q (G_i . w_q) / (24 |det|).
#pragma once

namespace eqs {

constexpr double kP2A = 0.58541019662496845446;  // (5 + 3 sqrt 5) / 20
constexpr double kP2B = 0.13819660112501051518;  // (5 - sqrt 5) / 20
constexpr int kP2Nodes = 10;

__host__ __device__ constexpr int p2_edge_a(int e) { return e < 3 ? 0 : (e < 5 ? 1 : 2); }
__host__ __device__ constexpr int p2_edge_b(int e) { return e < 3 ? e + 1 : (e < 5 ? e - 1 : 3); }

// Barycentric coordinate a of quadrature point q.
__host__ __device__ inline double p2_lambda(int q, int a) { return a == q ? kP2A : kP2B; }

}  // namespace eqs
