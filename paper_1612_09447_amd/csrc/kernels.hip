// gfx950 kernels of the EQS explicit-RKC hot path.
//
//  * k_kx: fused element pass (Sec. III): per tetrahedron the barycentric
//    gradients are formed from the four vertex coordinates, the constant field
//    E = -grad(phi) gives kappa(|E|), and the element matrix times the local
//    potentials is added straight into the output (K(x)x, or the stage
//    right-hand side b(t) - K(x)x with b folded in element by element).
//  * SELL and CSR sparse products with fused epilogues for CG on M and for
//    the smoothed-aggregation V-cycle (damped Jacobi, restriction,
//    prolongation, dense coarsest solve), including the folded operators the
//    host forms at set-up (a restriction with the pre-smoother inside, the two
//    lowest levels as one dense and one sparse product).
//  * CG vector updates with block partial sums; one-block finalisers turn the
//    partials into the CG scalars, kept in device memory.
//  * RKC stage combination (the paper's ref. [9]).
#include <algorithm>
#include <cmath>
#include <vector>

#include <hip/hip_ext.h>

#include "eqs_internal.h"
#include "p2.h"
#include "sell.h"

namespace eqs {

// Launch `kernel`; when kernel class `cls` is being profiled the launch carries
// its own start/stop events, so the class time is the kernel's execution.
#define EQS_LAUNCH_TIMED(ctx, cls, kernel, grid, block, shmem, stream, ...)                                    \
    do {                                                                                                      \
        hipEvent_t e0_, e1_;                                                                                  \
        if (prof_pair((ctx), (cls), &e0_, &e1_))                                                              \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, e0_, e1_, 0, __VA_ARGS__);              \
        else                                                                                                  \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                              \
    } while (0)


// ----------------------------------------------------------- reductions
// Threads of a finaliser block (one block per finaliser launch).
constexpr int kFin = 1024;

// A relaxed load that stays a vector load even when its address is uniform. A
// uniform plain load becomes a scalar load, and the wait for it is then shared
// with the waits for kernel arguments that later data loads need (scalar loads
// complete out of order, so the compiler waits for all of them at once);
// vector loads complete in order, so issuing one early holds nothing back.
template <typename T>
__device__ __forceinline__ T vec_load(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------- instances (batches)
// Independent instances occupy contiguous ranges of free rows. Every
// 256-row block of the finest level holds rows of at most two instances (each
// instance has >= 256 rows when there is more than one), so a block writes a
// pair of partial sums: [2b] for the instance of its first row, [2b+1] for the
// next instance (0 if the block lies in one instance).
struct InstMap {
    const int32_t* __restrict__ row_off;   // [n_inst + 1] first row of every instance
    const int32_t* __restrict__ blk_inst;  // [blocks] instance of each block's first row
    int32_t n_inst;
    int32_t rows1;  // the row count when n_inst == 1 (no table lookups then), else -1
};

// B: the block's row-block index (its logical block, see row_block)
__device__ __forceinline__ void block_instances(const InstMap& m, int32_t& lo, int32_t& bound, int64_t B) {
    if (m.rows1 >= 0) {
        lo = 0;
        bound = m.rows1;
        return;
    }
    lo = m.blk_inst[B];
    bound = m.row_off[lo + 1];
}

// Sums over the 256-thread block of K values per thread, each in a fixed order
// (wavefront tree, then the four wavefront sums in index order), with one
// barrier for all K; valid in thread 0. sh holds 4 K doubles and is used once
// per kernel.
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* sh) {
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[4 * k + wid] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = ((sh[4 * k] + sh[4 * k + 1]) + sh[4 * k + 2]) + sh[4 * k + 3];
}

// Thread 0 stores the block's pair of sums of each v[p] into part[p] (split by
// `second`, i.e. row >= bound). A block whose rows all lie before bound (the
// common case: the block lies inside one instance) has a zero second sum and
// needs only one reduction.
constexpr int kPairSh = 16;  // doubles of shared memory store_pairs needs (NP <= 2)
template <int NP>
__device__ __forceinline__ void store_pairs(double* const (&part)[NP], const double (&v)[NP], bool second,
                                            int32_t bound, double* sh, int64_t B) {
    static_assert(NP >= 1 && NP <= 2, "at most two partial arrays");
    const bool split = (int64_t)bound < (B + 1) * (int64_t)blockDim.x;  // uniform over the block
    if (!split) {
        double a[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) a[p] = v[p];
        block_sums<NP>(a, sh);
        if (threadIdx.x == 0)
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                part[p][2 * B] = a[p];
                part[p][2 * B + 1] = 0.0;
            }
    } else {
        double a[2 * NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            a[2 * p] = second ? 0.0 : v[p];
            a[2 * p + 1] = second ? v[p] : 0.0;
        }
        block_sums<2 * NP>(a, sh);
        if (threadIdx.x == 0)
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                part[p][2 * B] = a[2 * p];
                part[p][2 * B + 1] = a[2 * p + 1];
            }
    }
}

// Blocks b0..b1 hold instance i's rows r0..r1-1. Every block after b0 starts
// inside instance i, so its first partial is i's; block b0 starts inside i
// only when r0 is a multiple of 256, else i's share is its second partial.
__device__ __forceinline__ void inst_blocks(const InstMap& m, int32_t i, int32_t& b0, int32_t& b1, int32_t& head) {
    const int32_t r0 = m.rows1 >= 0 ? 0 : m.row_off[i], r1 = m.rows1 >= 0 ? m.rows1 : m.row_off[i + 1];
    if (r1 <= r0) {
        b0 = 0;
        b1 = -1;
        head = 0;
        return;
    }
    b0 = r0 >> 8;
    b1 = (r1 - 1) >> 8;
    head = (r0 & 255) ? 1 : 0;
}

// Sums over blocks lo..hi (inclusive) of the first partial of NP arrays, by
// the 64 lanes of one wavefront (the head block b0 is added by the caller);
// valid in all lanes. Lanes take blocks lo + lane, lo + lane + 64, ... in
// chunks of U whose loads carry no branch (positions past hi re-read block hi
// and are dropped by a select), so a range of up to 64 U blocks costs one
// memory latency. The order of the additions is fixed (it does not depend on
// timing).
template <int NP>
__device__ __forceinline__ void wave_range_sums(const double* const (&parts)[NP], int32_t lo, int32_t hi,
                                                double (&out)[NP]) {
    constexpr int U = 16;
    const int lane = threadIdx.x & 63;
    double acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = 0.0;
    for (int32_t b = lo + lane; b <= hi; b += 64 * U) {  // the lane's next chunk starts in range
        double t[NP][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t bc = min(b + 64 * u, hi);
#pragma unroll
            for (int p = 0; p < NP; ++p) t[p][u] = parts[p][2 * (int64_t)bc];
        }
        // every load is issued before the first add (left alone, the scheduler starts adding after the
        // first loads, and the wait for them holds back the rest)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int p = 0; p < NP; ++p) acc[p] += (b + 64 * u <= hi) ? t[p][u] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        double v = acc[p];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        out[p] = v;
    }
}

constexpr int kFinWaves = kFin / 64;

// Per-instance sums of NP pair-partial arrays, in a fixed order (the result
// does not depend on timing). A finaliser runs one workgroup per kFinWaves
// instances (fin_grid): the instances i0 = kFinWaves * blockIdx.x onwards of
// this workgroup each get kFinWaves / count wavefronts, each summing an equal
// share of the instance's blocks, so every instance's sums are in flight at
// once. body(i, sums) runs once per instance, in thread i - i0. Must be
// reached by the whole block.
template <int NP, typename F>
__device__ __forceinline__ void for_each_instance_sum(const double* const (&parts)[NP], const InstMap& m, F body) {
    __shared__ double sh[NP][kFinWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t i0 = (int32_t)blockIdx.x * kFinWaves;
    const int32_t cnt = max(1, min(kFinWaves, m.n_inst - i0));
    const int wpi = kFinWaves / cnt;
    const int li = wave / wpi, sub = wave - li * wpi;
    double v[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) v[p] = 0.0;
    if (li < cnt && i0 + li < m.n_inst) {
        int32_t b0, b1, head;
        inst_blocks(m, i0 + li, b0, b1, head);
        if (b1 >= b0) {
            const int32_t first = b0 + 1, n = b1 - b0;  // blocks first..b1 read their first partial
            const int32_t lo = first + (int32_t)(((int64_t)n * sub) / wpi);
            const int32_t hi = first + (int32_t)(((int64_t)n * (sub + 1)) / wpi) - 1;
            // the head block's partial is loaded with the range's, not after it
            double hv[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) hv[p] = sub == 0 ? parts[p][2 * (int64_t)b0 + head] : 0.0;
            wave_range_sums<NP>(parts, lo, hi, v);
            if (sub == 0)
#pragma unroll
                for (int p = 0; p < NP; ++p) v[p] += hv[p];
        }
    }
    if (lane == 0)
#pragma unroll
        for (int p = 0; p < NP; ++p) sh[p][wave] = v[p];
    __syncthreads();
    if ((int32_t)threadIdx.x < cnt && i0 + (int32_t)threadIdx.x < m.n_inst) {
        const int32_t k = threadIdx.x;
        double sums[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            double t = 0.0;
            for (int w = k * wpi; w < (k + 1) * wpi; ++w) t += sh[p][w];
            sums[p] = t;
        }
        body(i0 + k, sums);
    }
}

// ------------------------------------------------------------- simple ops
__global__ void k_fill(double* __restrict__ p, double v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

// dst[i] = src[idx[i]]
__global__ void k_gather(const double* __restrict__ src, const int32_t* __restrict__ idx, double* __restrict__ dst,
                         int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

// dst[idx[i]] = src[i]
__global__ void k_scatter(const double* __restrict__ src, const int32_t* __restrict__ idx, double* __restrict__ dst,
                          int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = src[i];
}

// x_user = (yfree on free nodes, g(t) on Dirichlet nodes), in user order.
__global__ void k_finish_state(const double* __restrict__ yfree, const int32_t* __restrict__ int_to_user,
                               const int32_t* __restrict__ ddrive, const DriveDev* __restrict__ drives, double t,
                               double* __restrict__ x_user, int64_t n_free, int64_t n_nodes) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    double v;
    if (i < n_free) {
        v = yfree[i];
    } else {
        const DriveDev d = drives[ddrive[i - n_free]];
        v = d.amp * sin(d.w * t + d.phase);
    }
    x_user[int_to_user[i]] = v;
}

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_fill(hipStream_t s, double* p, double v, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
}
void launch_copy(hipStream_t s, double* d, const double* src, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(kBlock), 0, s, d, src, n);
}
void launch_gather(hipStream_t s, const double* src, const int32_t* idx, double* dst, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(kBlock), 0, s, src, idx, dst, n);
}
void launch_scatter(hipStream_t s, const double* src, const int32_t* idx, double* dst, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_scatter, dim3(grid_for(n)), dim3(kBlock), 0, s, src, idx, dst, n);
}
void launch_finish_state(eqs_ctx* c, const double* yfree, double t, double* x_user) {
    hipLaunchKernelGGL(k_finish_state, dim3(grid_for(c->n_nodes)), dim3(kBlock), 0, c->stream, yfree,
                       c->d_int_to_user, c->d_ddrive, c->d_drives, t, x_user, c->n_free, c->n_nodes);
}

// ------------------------------------------------------ fused element pass
__device__ __forceinline__ double ipow(double x, int n) {
    double r = 1.0;
    while (n) {
        if (n & 1) r *= x;
        x *= x;
        n >>= 1;
    }
    return r;
}

// Fused element pass over blocks of kTetBlock * TPT tets (one workgroup of
// kTetBlock threads each).
// 0. The block's packed tet records are loaded first (they do not depend on
//    the node staging, so their latency overlaps it); thread t takes TPT
//    consecutive tets.
// 1. The block's distinct nodes are staged in LDS: coordinates, potential
//    (free: y[id]; Dirichlet: g(t) of its drive) and drive rate g'(t).
// 2. Per tet: with edges e_k = p_k - p_0 and cofactor rows
//    c_1 = e2 x e3, c_2 = e3 x e1, c_3 = e1 x e2, c_0 = -(c_1 + c_2 + c_3),
//    det = e1 . c_1, the barycentric gradients are c_a / det, so
//      w = sum_k c_k (u_k - u_0) = det * grad(phi),  |E| = |w| / |det|,
//      (A_e u)_a = |T| g_a . grad(phi) = c_a . w / (6 |det|).
//    kappa(|E|) scales w; RHS mode adds eps * A_e g' (b(t) = -M_ID g'(t),
//    folded in element by element). Contributions go to an LDS accumulator.
// 3. One global atomic per block node (RHS mode: free nodes only, negated).
// Workgroups are mapped so that each XCD (workgroups are dealt to the 8 XCDs
// round-robin) walks a contiguous range of Morton-ordered blocks: nodes
// shared by neighbouring blocks then meet in the same L2.

// Stage a block's nodes in LDS (one array per quantity: 8-byte stride, so
// gathers spread over the banks). Returns whether the block touches a
// Dirichlet node (node lists are sorted and Dirichlet nodes come last in the
// internal order, so iff its last node is one).

struct KxArgs {
    int64_t n_tets, n_blocks;
    const uint64_t* __restrict__ tpack;
    const int32_t* __restrict__ boff;
    const int32_t* __restrict__ bnodes;
    const double* __restrict__ X;
    const double* __restrict__ Y;
    const double* __restrict__ Z;
    const MatDev* __restrict__ mats;
    const double* __restrict__ yfree;
    int32_t n_free;
    const int32_t* __restrict__ ddrive;
    const DriveDev* __restrict__ drives;
    double t;
    double* __restrict__ out;
};

// The six LDS arrays of a block (x, y, z, potential, rate, accumulator) are
// S doubles apart: S = STRIDE when the kernel is built for a fixed stride
// (covering every block, so each node needs one LDS address and the arrays are
// reached by immediate offsets), else the block's node count. A fixed stride
// is one more than a multiple of 64 doubles: the arrays of one node then sit
// in different LDS banks (a multiple of 64 would put all six in one bank).
template <int STRIDE>
__device__ __forceinline__ int32_t kx_stride(int32_t nn) {
    return STRIDE > 0 ? STRIDE : nn;
}

template <bool RHS, int STRIDE>
__device__ __forceinline__ bool kx_stage(const KxArgs& A, double* lds, int32_t off, int32_t nn) {
    const int32_t S = kx_stride<STRIDE>(nn);
    for (int k = threadIdx.x; k < nn; k += kTetBlock) {
        const int32_t id = A.bnodes[off + k];
        double u, rate = 0.0;
        if (id < A.n_free) {
            u = A.yfree[id];
        } else {
            const DriveDev d = A.drives[A.ddrive[id - A.n_free]];
            const double ph = d.w * A.t + d.phase;
            u = d.amp * sin(ph);
            rate = d.w * d.amp * cos(ph);
        }
        double* q = lds + k;
        q[0] = A.X[id];
        q[S] = A.Y[id];
        q[2 * S] = A.Z[id];
        q[3 * S] = u;
        q[4 * S] = rate;
        q[5 * S] = 0.0;
    }
    return RHS && nn > 0 && A.bnodes[off + nn - 1] >= A.n_free;
}

// The thread's TPT consecutive tets of block b: records with 16-byte loads
// (the record array is padded to whole blocks; padding records are ~0).
template <int TPT>
__device__ __forceinline__ void kx_records(const KxArgs& A, int64_t b, uint64_t (&rec)[TPT]) {
    const uint64_t* rp = A.tpack + b * (kTetBlock * TPT) + (int64_t)threadIdx.x * TPT;
    if (TPT == 1) {
        rec[0] = rp[0];
    } else {
#pragma unroll
        for (int q = 0; q < TPT / 2; ++q) {
            const ulonglong2 v = reinterpret_cast<const ulonglong2*>(rp)[q];
            rec[2 * q] = v.x;
            rec[2 * q + 1] = v.y;
        }
    }
}

// Element matrices of the thread's tets times the staged potentials, added
// into the LDS accumulator (see the kernel comment for the algebra). With
// contrib (the deterministic pass) the four values of the thread's tet i go
// to contrib[4 (threadIdx.x TPT + i) + a] instead, each written once.
template <bool RHS, int TPT, int STRIDE>
__device__ __forceinline__ void kx_tets(const KxArgs& A, double* lds, int32_t nn, bool has_dir,
                                        const uint64_t (&rec)[TPT], double* contrib = nullptr) {
    const int32_t S = kx_stride<STRIDE>(nn);
    const double* PX = lds;
    const double* PY = PX + S;
    const double* PZ = PY + S;
    const double* PU = PZ + S;
    const double* R = PU + S;
    double* Acc = lds + 5 * S;
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
        const uint64_t w = rec[i];
        if (w == ~0ull) continue;
        const MatDev m = A.mats[(uint32_t)(w & 0xffffu)];
        int l[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) l[a] = (int)((w >> (16 + 12 * a)) & 0xfffu);
        const double4 p0 = make_double4(PX[l[0]], PY[l[0]], PZ[l[0]], PU[l[0]]);
        const double4 p1 = make_double4(PX[l[1]], PY[l[1]], PZ[l[1]], PU[l[1]]);
        const double4 p2 = make_double4(PX[l[2]], PY[l[2]], PZ[l[2]], PU[l[2]]);
        const double4 p3 = make_double4(PX[l[3]], PY[l[3]], PZ[l[3]], PU[l[3]]);
        const double e1x = p1.x - p0.x, e1y = p1.y - p0.y, e1z = p1.z - p0.z;
        const double e2x = p2.x - p0.x, e2y = p2.y - p0.y, e2z = p2.z - p0.z;
        const double e3x = p3.x - p0.x, e3y = p3.y - p0.y, e3z = p3.z - p0.z;
        const double c1x = e2y * e3z - e2z * e3y, c1y = e2z * e3x - e2x * e3z, c1z = e2x * e3y - e2y * e3x;
        const double c2x = e3y * e1z - e3z * e1y, c2y = e3z * e1x - e3x * e1z, c2z = e3x * e1y - e3y * e1x;
        const double c3x = e1y * e2z - e1z * e2y, c3y = e1z * e2x - e1x * e2z, c3z = e1x * e2y - e1y * e2x;
        const double det = e1x * c1x + e1y * c1y + e1z * c1z;
        const double inv = 1.0 / fabs(det);  // the one division per tet

        const double d1 = p1.w - p0.w, d2 = p2.w - p0.w, d3 = p3.w - p0.w;
        double wx = c1x * d1 + c2x * d2 + c3x * d3;
        double wy = c1y * d1 + c2y * d2 + c3y * d3;
        double wz = c1z * d1 + c2z * d2 + c3z * d3;

        // (A_e u)_a = c_a . w / (6 |det|): the factor sc goes into w
        const double sc = (RHS ? -1.0 / 6.0 : 1.0 / 6.0) * inv;
        double ks = m.kappa0 * sc;
        if (m.nonlinear) {
            const double ratio = sqrt(wx * wx + wy * wy + wz * wz) * inv * m.inv_es;
            // r^alpha as exp(alpha ln r): relative error ~ ulp(alpha ln r), about
            // 1e-14 for the exponents and fields here (r = 0 gives 0)
            const double pw = (m.ialpha >= 0) ? ipow(ratio, m.ialpha) : exp(m.alpha * log(ratio));
            ks *= 1.0 + pw;
        }
        wx *= ks;
        wy *= ks;
        wz *= ks;
        if (RHS && has_dir) {
            const double r0 = R[l[0]], r1 = R[l[1]], r2 = R[l[2]], r3 = R[l[3]];
            if (r0 != 0.0 || r1 != 0.0 || r2 != 0.0 || r3 != 0.0) {
                const double q1 = r1 - r0, q2 = r2 - r0, q3 = r3 - r0;
                const double es = m.eps * sc;
                wx += es * (c1x * q1 + c2x * q2 + c3x * q3);
                wy += es * (c1y * q1 + c2y * q2 + c3y * q3);
                wz += es * (c1z * q1 + c2z * q2 + c3z * q3);
            }
        }
        const double y1 = c1x * wx + c1y * wy + c1z * wz;
        const double y2 = c2x * wx + c2y * wy + c2z * wz;
        const double y3 = c3x * wx + c3y * wy + c3z * wz;
        const double y0 = -(y1 + y2 + y3);
        if (contrib) {
            double* q = contrib + 4 * ((int64_t)threadIdx.x * TPT + i);
            q[0] = y0;
            q[1] = y1;
            q[2] = y2;
            q[3] = y3;
        } else {
            unsafeAtomicAdd(&Acc[l[0]], y0);
            unsafeAtomicAdd(&Acc[l[1]], y1);
            unsafeAtomicAdd(&Acc[l[2]], y2);
            unsafeAtomicAdd(&Acc[l[3]], y3);
        }
    }
}

// One global atomic per block node (RHS mode: free nodes only; the element
// signs already give -K(x)x + b).
template <bool RHS, int STRIDE>
__device__ __forceinline__ void kx_scatter(const KxArgs& A, const double* lds, int32_t off, int32_t nn) {
    const double* Acc = lds + 5 * kx_stride<STRIDE>(nn);
    for (int k = threadIdx.x; k < nn; k += kTetBlock) {
        const int32_t id = A.bnodes[off + k];
        if (RHS && id >= A.n_free) continue;
        unsafeAtomicAdd(&A.out[id], Acc[k]);
    }
}

// One element block per workgroup (blocks in XCD-contiguous order).
template <bool RHS, int TPT, int STRIDE>
__global__ __launch_bounds__(kTetBlock, 6) void k_kx(KxArgs A) {
    extern __shared__ double lds[];
    const int64_t b = xcd_block(blockIdx.x, A.n_blocks);
    uint64_t rec[TPT];
    kx_records<TPT>(A, b, rec);  // issued first: its latency overlaps the staging
    const int32_t off = A.boff[b];
    const int32_t nn = A.boff[b + 1] - off;
    const bool has_dir = kx_stage<RHS, STRIDE>(A, lds, off, nn);
    __syncthreads();
    kx_tets<RHS, TPT, STRIDE>(A, lds, nn, has_dir, rec);
    __syncthreads();
    kx_scatter<RHS, STRIDE>(A, lds, off, nn);
}

// Deterministic element pass (eqs_set_deterministic): the same arithmetic,
// summed in an order fixed at set-up instead of the order in which atomics
// land. Each tet writes its four contributions to its own LDS slots
// (4 t + a for block-local tet t, vertex a); each block node then sums its
// slots in increasing slot order (lists built on the host: d_kslots holds,
// block after block in the record layout, the slots of node 0, node 1, ...;
// d_kend[boff[b] + k] ends node k's list) and stores the block's partial
// without atomics; k_kx_gather sums every node's partials in block order. Run
// to run the result is the same bit for bit.
template <bool RHS, int TPT, int STRIDE>
__global__ __launch_bounds__(kTetBlock) void k_kx_det(KxArgs A, const uint16_t* __restrict__ kslots,
                                                      const uint16_t* __restrict__ kend,
                                                      double* __restrict__ part) {
    extern __shared__ double lds[];
    const int64_t b = xcd_block(blockIdx.x, A.n_blocks);
    uint64_t rec[TPT];
    kx_records<TPT>(A, b, rec);
    const int32_t off = A.boff[b];
    const int32_t nn = A.boff[b + 1] - off;
    const bool has_dir = kx_stage<RHS, STRIDE>(A, lds, off, nn);
    double* contrib = lds + 6 * kx_stride<STRIDE>(nn);
    __syncthreads();
    kx_tets<RHS, TPT, STRIDE>(A, lds, nn, has_dir, rec, contrib);
    __syncthreads();
    const uint16_t* sl = kslots + b * (int64_t)(4 * kTetBlock * TPT);
    for (int k = threadIdx.x; k < nn; k += kTetBlock) {
        const int32_t beg = k ? (int32_t)kend[off + k - 1] : 0, end = kend[off + k];
        double v = 0.0;
        for (int32_t j = beg; j < end; ++j) v += contrib[sl[j]];
        part[off + k] = v;
    }
}

// out[i] = sum of node i's block partials in block order (occ lists, built at
// set-up); RHS mode covers the free nodes only.
__global__ void k_kx_gather(const int32_t* __restrict__ occ_off, const int32_t* __restrict__ occ,
                            const double* __restrict__ part, double* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = 0.0;
    for (int32_t j = occ_off[i]; j < occ_off[i + 1]; ++j) v += part[occ[j]];
    out[i] = v;
}

// ------------------------------------------------ second-order tets (P2)
// The same block structure with ten nodes per tet (p2.h): each record is two
// 64-bit words (material, then ten 11-bit block-local ids). Per tet the four
// vertex coordinates give the cofactors c_a and det; at each of the four
// quadrature points q the scaled field w_q = sum_a s_a c_a with
//   s_a = (4 lambda_a - 1) u_a + 4 sum_{b != a} lambda_b u_ab
// (det times grad phi), |E_q| = |w_q| / |det|, kappa_q = kappa(|E_q|), and with
// d_a = c_a . (kappa_q w_q) the nodes receive
//   vertex a: (4 lambda_a - 1) d_a,   edge ab: 4 (lambda_b d_a + lambda_a d_b),
// summed over q and scaled by +-1 / (24 |det|) (RHS mode: negative, and the
// Dirichlet term eps A_e g' adds eps times the same field of the drive rates).
__device__ __forceinline__ int p2_local(uint64_t lo, uint64_t hi, int k) {
    const int pos = 16 + 11 * k;
    uint64_t v;
    if (pos >= 64) v = hi >> (pos - 64);
    else if (pos + 11 > 64) v = (lo >> pos) | (hi << (64 - pos));
    else v = lo >> pos;
    return (int)(v & 0x7ffu);
}

// s_a of one quadrature point from the ten nodal values v[]
__device__ __forceinline__ void p2_svals(const double (&v)[kP2Nodes], int q, double (&sv)[4]) {
#pragma unroll
    for (int a = 0; a < 4; ++a) sv[a] = (4.0 * p2_lambda(q, a) - 1.0) * v[a];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int a = p2_edge_a(k), b = p2_edge_b(k);
        sv[a] += 4.0 * p2_lambda(q, b) * v[4 + k];
        sv[b] += 4.0 * p2_lambda(q, a) * v[4 + k];
    }
}

template <bool RHS, int TPT, int STRIDE>
__device__ __forceinline__ void kx_p2_tets(const KxArgs& A, double* lds, int32_t nn, bool has_dir,
                                           const uint64_t (&rec)[2 * TPT]) {
    const int32_t S = kx_stride<STRIDE>(nn);
    const double* PX = lds;
    const double* PY = PX + S;
    const double* PZ = PY + S;
    const double* PU = PZ + S;
    const double* R = PU + S;
    double* Acc = lds + 5 * S;
#pragma unroll 1
    for (int i = 0; i < TPT; ++i) {
        const uint64_t lo = rec[2 * i], hi = rec[2 * i + 1];
        if (lo == ~0ull) continue;
        const MatDev m = A.mats[(uint32_t)(lo & 0xffffu)];
        int l[kP2Nodes];
#pragma unroll
        for (int k = 0; k < kP2Nodes; ++k) l[k] = p2_local(lo, hi, k);
        double u[kP2Nodes];
#pragma unroll
        for (int k = 0; k < kP2Nodes; ++k) u[k] = PU[l[k]];
        double cf[4][3];
        {
            const double x0 = PX[l[0]], y0 = PY[l[0]], z0 = PZ[l[0]];
            const double e1x = PX[l[1]] - x0, e1y = PY[l[1]] - y0, e1z = PZ[l[1]] - z0;
            const double e2x = PX[l[2]] - x0, e2y = PY[l[2]] - y0, e2z = PZ[l[2]] - z0;
            const double e3x = PX[l[3]] - x0, e3y = PY[l[3]] - y0, e3z = PZ[l[3]] - z0;
            cf[1][0] = e2y * e3z - e2z * e3y; cf[1][1] = e2z * e3x - e2x * e3z; cf[1][2] = e2x * e3y - e2y * e3x;
            cf[2][0] = e3y * e1z - e3z * e1y; cf[2][1] = e3z * e1x - e3x * e1z; cf[2][2] = e3x * e1y - e3y * e1x;
            cf[3][0] = e1y * e2z - e1z * e2y; cf[3][1] = e1z * e2x - e1x * e2z; cf[3][2] = e1x * e2y - e1y * e2x;
#pragma unroll
            for (int d = 0; d < 3; ++d) cf[0][d] = -(cf[1][d] + cf[2][d] + cf[3][d]);
        }
        const double det = (PX[l[1]] - PX[l[0]]) * cf[1][0] + (PY[l[1]] - PY[l[0]]) * cf[1][1] +
                           (PZ[l[1]] - PZ[l[0]]) * cf[1][2];
        const double inv = 1.0 / fabs(det);
        double rate[kP2Nodes];
        bool drive = false;
        if (RHS && has_dir) {
#pragma unroll
            for (int k = 0; k < kP2Nodes; ++k) {
                rate[k] = R[l[k]];
                drive = drive || rate[k] != 0.0;
            }
        }
        double acc[kP2Nodes];
#pragma unroll
        for (int k = 0; k < kP2Nodes; ++k) acc[k] = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double sv[4];
            p2_svals(u, q, sv);
            double wx = 0.0, wy = 0.0, wz = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                wx += sv[a] * cf[a][0];
                wy += sv[a] * cf[a][1];
                wz += sv[a] * cf[a][2];
            }
            double ks = m.kappa0;
            if (m.nonlinear) {
                const double ratio = sqrt(wx * wx + wy * wy + wz * wz) * inv * m.inv_es;
                const double pw = (m.ialpha >= 0) ? ipow(ratio, m.ialpha) : exp(m.alpha * log(ratio));
                ks *= 1.0 + pw;
            }
            wx *= ks;
            wy *= ks;
            wz *= ks;
            if (RHS && has_dir && drive) {
                double sr[4];
                p2_svals(rate, q, sr);
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    wx += m.eps * sr[a] * cf[a][0];
                    wy += m.eps * sr[a] * cf[a][1];
                    wz += m.eps * sr[a] * cf[a][2];
                }
            }
            double dd[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) dd[a] = cf[a][0] * wx + cf[a][1] * wy + cf[a][2] * wz;
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a] += (4.0 * p2_lambda(q, a) - 1.0) * dd[a];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const int a = p2_edge_a(k), b = p2_edge_b(k);
                acc[4 + k] += 4.0 * (p2_lambda(q, b) * dd[a] + p2_lambda(q, a) * dd[b]);
            }
        }
        const double sc = (RHS ? -1.0 / 24.0 : 1.0 / 24.0) * inv;
#pragma unroll
        for (int k = 0; k < kP2Nodes; ++k) unsafeAtomicAdd(&Acc[l[k]], sc * acc[k]);
    }
}

template <bool RHS, int TPT, int STRIDE>
__global__ __launch_bounds__(kTetBlock) void k_kx_p2(KxArgs A) {
    extern __shared__ double lds[];
    const int64_t b = xcd_block(blockIdx.x, A.n_blocks);
    uint64_t rec[2 * TPT];
    {
        const uint64_t* rp = A.tpack + 2 * (b * (kTetBlock * TPT) + (int64_t)threadIdx.x * TPT);
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
            const ulonglong2 v = reinterpret_cast<const ulonglong2*>(rp)[q];
            rec[2 * q] = v.x;
            rec[2 * q + 1] = v.y;
        }
    }
    const int32_t off = A.boff[b];
    const int32_t nn = A.boff[b + 1] - off;
    const bool has_dir = kx_stage<RHS, STRIDE>(A, lds, off, nn);
    __syncthreads();
    kx_p2_tets<RHS, TPT, STRIDE>(A, lds, nn, has_dir, rec);
    __syncthreads();
    kx_scatter<RHS, STRIDE>(A, lds, off, nn);
}

// Spectral bound of one element block for the adaptive stage choice: the
// largest sigma_e / eps_e over the block's tets, with sigma = kappa0 (1 +
// (alpha + 1)(|E|/e_s)^alpha) the differential conductivity at the element's
// field (|E| = |w| / |det| as in kx_tets); folded into *out with an atomic
// maximum on the bits of non-negative doubles (whose order is the integers').
template <int TPT, int STRIDE>
__global__ __launch_bounds__(kTetBlock, 6) void k_kx_rate(KxArgs A) {
    extern __shared__ double lds[];
    __shared__ double wmax[kTetBlock / 64];
    const int64_t b = xcd_block(blockIdx.x, A.n_blocks);
    uint64_t rec[TPT];
    kx_records<TPT>(A, b, rec);
    const int32_t off = A.boff[b];
    const int32_t nn = A.boff[b + 1] - off;
    kx_stage<false, STRIDE>(A, lds, off, nn);
    __syncthreads();
    const int32_t S = kx_stride<STRIDE>(nn);
    const double* PX = lds;
    const double* PY = PX + S;
    const double* PZ = PY + S;
    const double* PU = PZ + S;
    double best = 0.0;
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
        const uint64_t w = rec[i];
        if (w == ~0ull) continue;
        const MatDev m = A.mats[(uint32_t)(w & 0xffffu)];
        int l[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) l[a] = (int)((w >> (16 + 12 * a)) & 0xfffu);
        const double e1x = PX[l[1]] - PX[l[0]], e1y = PY[l[1]] - PY[l[0]], e1z = PZ[l[1]] - PZ[l[0]];
        const double e2x = PX[l[2]] - PX[l[0]], e2y = PY[l[2]] - PY[l[0]], e2z = PZ[l[2]] - PZ[l[0]];
        const double e3x = PX[l[3]] - PX[l[0]], e3y = PY[l[3]] - PY[l[0]], e3z = PZ[l[3]] - PZ[l[0]];
        const double c1x = e2y * e3z - e2z * e3y, c1y = e2z * e3x - e2x * e3z, c1z = e2x * e3y - e2y * e3x;
        const double c2x = e3y * e1z - e3z * e1y, c2y = e3z * e1x - e3x * e1z, c2z = e3x * e1y - e3y * e1x;
        const double c3x = e1y * e2z - e1z * e2y, c3y = e1z * e2x - e1x * e2z, c3z = e1x * e2y - e1y * e2x;
        const double det = e1x * c1x + e1y * c1y + e1z * c1z;
        const double d1 = PU[l[1]] - PU[l[0]], d2 = PU[l[2]] - PU[l[0]], d3 = PU[l[3]] - PU[l[0]];
        const double wx = c1x * d1 + c2x * d2 + c3x * d3;
        const double wy = c1y * d1 + c2y * d2 + c3y * d3;
        const double wz = c1z * d1 + c2z * d2 + c3z * d3;
        double sig = m.kappa0;
        if (m.nonlinear) {
            const double ratio = sqrt(wx * wx + wy * wy + wz * wz) / fabs(det) * m.inv_es;
            const double pw = (m.ialpha >= 0) ? ipow(ratio, m.ialpha) : exp(m.alpha * log(ratio));
            sig *= 1.0 + (m.alpha + 1.0) * pw;
        }
        best = fmax(best, sig / m.eps);
    }
    for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = wmax[0];
        for (int k = 1; k < kTetBlock / 64; ++k) v = fmax(v, wmax[k]);
        atomicMax((unsigned long long*)A.out, (unsigned long long)__double_as_longlong(v));
    }
}

// Fixed LDS stride for blocks of kTetBlock * TPT tets: above the node count of
// such blocks on tetrahedral meshes of Kuhn or similar quality (about 0.33
// nodes per tet for large blocks). Blocks with more nodes take the kernel with
// the block's own node count as stride.
constexpr int kx_fixed_stride(int tpt) { return tpt == 1 ? 129 : tpt == 2 ? 193 : tpt == 4 ? 385 : 705; }

// fixed LDS strides of second-order blocks (256 and 512 tets)
constexpr int kx_p2_fixed_stride(int tpt) { return tpt == 1 ? 705 : 1217; }

template <bool RHS>
static void launch_kx_t(hipStream_t s, eqs_ctx* c, const double* yfree, double t, double* out) {
    const KxArgs A{c->n_tets, c->n_blocks, c->d_tpack, c->d_boff, c->d_bnodes, c->d_cx, c->d_cy, c->d_cz, c->d_mats,
                   yfree, (int32_t)c->n_free, c->d_ddrive, c->d_drives, t, out};
    const dim3 b(kTetBlock), g((unsigned)c->n_blocks);
    const int tpt = c->tet_tpt;
    if (c->npe == kP2Nodes) {
        const bool fixed2 = (tpt == 1 || tpt == 2) && c->max_block_nodes <= kx_p2_fixed_stride(tpt) && !c->kx_generic;
        const size_t lds2 = sizeof(double) * 6 * (size_t)(fixed2 ? kx_p2_fixed_stride(tpt) : c->max_block_nodes);
        if (tpt == 1) {
            if (fixed2) EQS_LAUNCH_TIMED(c, EQS_KCLASS_ELEMENT, (k_kx_p2<RHS, 1, kx_p2_fixed_stride(1)>), g, b, lds2, s, A);
            else EQS_LAUNCH_TIMED(c, EQS_KCLASS_ELEMENT, (k_kx_p2<RHS, 1, 0>), g, b, lds2, s, A);
        } else if (tpt == 2) {
            if (fixed2) EQS_LAUNCH_TIMED(c, EQS_KCLASS_ELEMENT, (k_kx_p2<RHS, 2, kx_p2_fixed_stride(2)>), g, b, lds2, s, A);
            else EQS_LAUNCH_TIMED(c, EQS_KCLASS_ELEMENT, (k_kx_p2<RHS, 2, 0>), g, b, lds2, s, A);
        } else {
            fail(EQS_ERR_STATE, "second-order element blocks hold 256 or 512 tets");
        }
        return;
    }
    const bool fixed = tpt >= 1 && c->max_block_nodes <= kx_fixed_stride(tpt) && !c->kx_generic;
    const size_t lds = sizeof(double) * 6 * (size_t)(fixed ? kx_fixed_stride(tpt) : c->max_block_nodes);
    if (c->deterministic) {
        if (!c->d_kslots) fail(EQS_ERR_STATE, "deterministic element pass without its lists");
        const size_t ldsd = lds + sizeof(double) * 4 * (size_t)(kTetBlock * tpt);
#define EQS_KXD(TPT_)                                                                                            \
    do {                                                                                                         \
        if (fixed)                                                                                               \
            EQS_LAUNCH_TIMED(c, EQS_KCLASS_ELEMENT, (k_kx_det<RHS, TPT_, kx_fixed_stride(TPT_)>), g, b, ldsd, s, A, \
                             c->d_kslots, c->d_kend, c->d_kx_part);                                              \
        else                                                                                                     \
            EQS_LAUNCH_TIMED(c, EQS_KCLASS_ELEMENT, (k_kx_det<RHS, TPT_, 0>), g, b, ldsd, s, A, c->d_kslots,     \
                             c->d_kend, c->d_kx_part);                                                           \
    } while (0)
        switch (tpt) {
            case 1: EQS_KXD(1); break;
            case 2: EQS_KXD(2); break;
            case 4: EQS_KXD(4); break;
            case 8: EQS_KXD(8); break;
            default: fail(EQS_ERR_STATE, "element blocks not built");
        }
#undef EQS_KXD
        const int64_t nout = RHS ? c->n_free : c->n_nodes;
        hipLaunchKernelGGL(k_kx_gather, dim3(grid_for(nout)), dim3(kBlock), 0, s, c->d_occ_off, c->d_occ,
                           (const double*)c->d_kx_part, out, nout);
        return;
    }
#define EQS_KX(TPT_)                                                                                           \
    do {                                                                                                       \
        if (fixed) EQS_LAUNCH_TIMED(c, EQS_KCLASS_ELEMENT, (k_kx<RHS, TPT_, kx_fixed_stride(TPT_)>), g, b, lds, s, A); \
        else EQS_LAUNCH_TIMED(c, EQS_KCLASS_ELEMENT, (k_kx<RHS, TPT_, 0>), g, b, lds, s, A);                    \
    } while (0)
    switch (tpt) {
        case 1: EQS_KX(1); break;
        case 2: EQS_KX(2); break;
        case 4: EQS_KX(4); break;
        case 8: EQS_KX(8); break;
        default: fail(EQS_ERR_STATE, "element blocks not built");
    }
#undef EQS_KX
}

double max_rate(eqs_ctx* c, const double* yfree, double t) {
    if (c->npe != 4) fail(EQS_ERR_STATE, "the spectral bound is built for first-order tets");
    hipStream_t s = c->stream;
    double* slot = c->d_partials;  // free between CG solves
    launch_fill(s, slot, 0.0, 1);
    const KxArgs A{c->n_tets, c->n_blocks, c->d_tpack, c->d_boff, c->d_bnodes, c->d_cx, c->d_cy, c->d_cz, c->d_mats,
                   yfree, (int32_t)c->n_free, c->d_ddrive, c->d_drives, t, slot};
    const dim3 b(kTetBlock), g((unsigned)c->n_blocks);
    const int tpt = c->tet_tpt;
    const bool fixed = tpt >= 1 && c->max_block_nodes <= kx_fixed_stride(tpt) && !c->kx_generic;
    const size_t lds = sizeof(double) * 6 * (size_t)(fixed ? kx_fixed_stride(tpt) : c->max_block_nodes);
#define EQS_KR(TPT_)                                                                                     \
    do {                                                                                                 \
        if (fixed) hipLaunchKernelGGL((k_kx_rate<TPT_, kx_fixed_stride(TPT_)>), g, b, lds, s, A);        \
        else hipLaunchKernelGGL((k_kx_rate<TPT_, 0>), g, b, lds, s, A);                                  \
    } while (0)
    switch (tpt) {
        case 1: EQS_KR(1); break;
        case 2: EQS_KR(2); break;
        case 4: EQS_KR(4); break;
        case 8: EQS_KR(8); break;
        default: fail(EQS_ERR_STATE, "element blocks not built");
    }
#undef EQS_KR
    double v = 0.0;
    EQS_HIP(hipMemcpyAsync(&v, slot, sizeof v, hipMemcpyDeviceToHost, s));
    EQS_HIP(hipStreamSynchronize(s));
    return v;
}

// Ref. [9]'s local error estimate est = (12 (y0 - y1) + 6 tau (f0 + f1)) / 15
// in the weighted RMS norm: per-block sums of (est_i / w_i)^2 with
// w_i = atol + rtol max(|y0_i|, |y1_i|), in a fixed order.
__global__ __launch_bounds__(256) void k_err_sq(const double* __restrict__ y0, const double* __restrict__ y1,
                                                 const double* __restrict__ f0, const double* __restrict__ f1,
                                                 double tau, double atol, double rtol, int64_t n,
                                                 double* __restrict__ part) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (i < n) {
        const double a = y0[i], b = y1[i];
        const double est = (12.0 * (a - b) + 6.0 * tau * (f0[i] + f1[i])) / 15.0;
        const double q = est / (atol + rtol * fmax(fabs(a), fabs(b)));
        v[0] = q * q;
    }
    block_sums<1>(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

double error_norm(eqs_ctx* c, const double* y0, const double* y1, const double* f0, const double* f1, double tau,
                  double atol, double rtol) {
    hipStream_t s = c->stream;
    const int64_t n = c->n_free;
    const unsigned nb = grid_for(n);
    hipLaunchKernelGGL(k_err_sq, dim3(nb), dim3(kBlock), 0, s, y0, y1, f0, f1, tau, atol, rtol, n, c->d_partials);
    std::vector<double> part(nb);
    EQS_HIP(hipMemcpyAsync(part.data(), c->d_partials, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    EQS_HIP(hipStreamSynchronize(s));
    double sum = 0.0;
    for (double x : part) sum += x;
    return std::sqrt(sum / (double)n);
}

void launch_kx(hipStream_t s, bool rhs_mode, eqs_ctx* c, const double* yfree, double t, double* out, bool zeroed) {
    const int64_t nout = rhs_mode ? c->n_free : c->n_nodes;
    if (!zeroed) launch_fill(s, out, 0.0, nout);
    if (c->n_tets == 0) return;
    if (rhs_mode) launch_kx_t<true>(s, c, yfree, t, out);
    else launch_kx_t<false>(s, c, yfree, t, out);
}

double time_kx(eqs_ctx* c, const double* yfree, double* out, int reps) {
    hipEvent_t e0, e1;
    EQS_HIP(hipEventCreate(&e0));
    EQS_HIP(hipEventCreate(&e1));
    std::vector<float> ms;
    for (int r = 0; r < reps + 2; ++r) {
        EQS_HIP(hipEventRecord(e0, c->stream));
        launch_kx_t<true>(c->stream, c, yfree, 0.0, out);
        EQS_HIP(hipEventRecord(e1, c->stream));
        EQS_HIP(hipEventSynchronize(e1));
        float t = 0.0f;
        EQS_HIP(hipEventElapsedTime(&t, e0, e1));
        if (r >= 2) ms.push_back(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}

// ------------------------------------------------------------- SELL-64
// Sparse products and smoothers are memory-latency bound: they are built for
// 8 wavefronts per SIMD (at most 64 VGPRs), the most a SIMD holds.
constexpr int kSparseWaves = 8;
template <typename T>
static unsigned sell_grid(const Sell<T>& A) {
    return (unsigned)(((int64_t)A.n_slices * kSlice + kBlock - 1) / kBlock);
}

// Epilogue of a product y = A x: acc 0 stores A x, 1 adds it to y, 2 stores
// omega dinv[row] b[row] + A x (the pre-smoothed x = omega D^-1 b of a level
// whose pre-smoother is folded into its restriction, plus the prolonged
// correction).
template <typename T>
struct MvInit {
    const T* __restrict__ dinv;
    const T* __restrict__ b;
    T omega;
};
template <typename T>
__device__ __forceinline__ void mv_store(T* __restrict__ y, int32_t row, T v, int acc, const MvInit<T>& in) {
    if (acc == 2) y[row] = in.omega * in.dinv[row] * in.b[row] + v;
    else y[row] = acc ? y[row] + v : v;
}

// y = A x with the epilogue above (L lanes per row, groups of U entries). The
// epilogue's own loads are issued before the row sum, so they wait together
// with the operator's loads instead of after the gathers.
template <int L, int U, typename T>
__device__ __forceinline__ void sell_mv(const SellView<T>& A, const T* __restrict__ x, T* __restrict__ y, int acc,
                                        const MvInit<T>& in) {
    const int64_t g = row_block(A.xcd) * blockDim.x + threadIdx.x;
    if (g >= (int64_t)A.n_slices * 64) return;  // whole wavefronts leave together
    const int32_t row = sell_perm_row<L>(A.perm, g);
    const bool writer = (g & (L - 1)) == 0 && row < A.n_rows;
    T y0 = T(0), d = T(0), bb = T(0);
    if (writer) {
        if (acc == 1) y0 = y[row];
        else if (acc == 2) {
            d = in.dinv[row];
            bb = in.b[row];
        }
    }
    const T v = sell_row<L, U>(A, g, row, x);
    if (writer) {
        if (acc == 2) y[row] = in.omega * d * bb + v;
        else y[row] = acc ? y0 + v : v;
    }
}

// The same product under three names, so that traces tell the V-cycle's
// restrictions (k_restrict) and prolongations (k_prolong) from other SELL
// products (k_sell_mv). Groups of 16 entries hold their loads in up to 128
// registers (4 waves per SIMD instead of 8).
#define EQS_SELL_MV_ARGS \
    SellView<T> A, const T* __restrict__ x, T* __restrict__ y, int acc, MvInit<T> in
template <int L, int U, typename T>
__global__ __launch_bounds__(256, (U >= 16 ? 4 : kSparseWaves)) void k_sell_mv(EQS_SELL_MV_ARGS) {
    sell_mv<L, U, T>(A, x, y, acc, in);
}
template <int L, int U, typename T>
__global__ __launch_bounds__(256, (U >= 16 ? 4 : kSparseWaves)) void k_restrict(EQS_SELL_MV_ARGS) {
    sell_mv<L, U, T>(A, x, y, acc, in);
}
template <int L, int U, typename T>
__global__ __launch_bounds__(256, (U >= 16 ? 4 : kSparseWaves)) void k_prolong(EQS_SELL_MV_ARGS) {
    sell_mv<L, U, T>(A, x, y, acc, in);
}
#undef EQS_SELL_MV_ARGS

enum MvRole { MV_PLAIN = 0, MV_RESTRICT = 1, MV_PROLONG = 2 };
template <int L, int U, typename T>
using SellMvKernel = void (*)(SellView<T>, const T*, T*, int, MvInit<T>);
template <int L, int U, typename T>
static SellMvKernel<L, U, T> sell_mv_kernel(int role) {
    return role == MV_RESTRICT ? k_restrict<L, U, T> : role == MV_PROLONG ? k_prolong<L, U, T> : k_sell_mv<L, U, T>;
}

__global__ __launch_bounds__(256, kSparseWaves) void k_spmv64(SellView<double> A, const double* __restrict__ x,
                                                 double* __restrict__ y) {
    const int64_t g = row_block(A.xcd) * blockDim.x + threadIdx.x;
    if (g >= (int64_t)A.n_slices * 64) return;
    const int32_t row = sell_perm_row<1>(A.perm, g);  // M may store its rows in a row order
    const double v = sell_row<1>(A, g, row, x);
    if (row < A.n_rows) y[row] = v;
}

void launch_spmv64(hipStream_t s, const Sell<double>& A, const double* x, double* y) {
    if (A.n_rows > 0) hipLaunchKernelGGL(k_spmv64, dim3(sell_grid(A)), dim3(kBlock), 0, s, view(A), x, y);
}

// ------------------------------------------------------------ V-cycle
// Pre-smoothing from a zero guess fused with the residual:
//   x = omega D^{-1} b,   res = b - A x = b - (A omega D^{-1}) b,
// the last product with the stored pre-smoothing values a_ij omega / a_jj,
// so rows gather b only.
template <int L, typename T, typename TB, int U = 8>
__global__ __launch_bounds__(256, (U >= 16 ? 4 : kSparseWaves)) void k_presmooth_res(SellView<T> As, const T* __restrict__ dinv, T omega,
                                                        const TB* __restrict__ b, T* __restrict__ x,
                                                        T* __restrict__ res) {
    const int64_t g = row_block(As.xcd) * blockDim.x + threadIdx.x;
    if (g >= (int64_t)As.n_slices * 64) return;
    const int32_t row = sell_perm_row<L>(As.perm, g);  // the finest operator may store its rows in a row order
    const T acc = sell_row<L, U>(As, g, row, b);
    if ((g & (L - 1)) == 0 && row < As.n_rows) {
        const T bi = (T)b[row];
        x[row] = omega * dinv[row] * bi;
        res[row] = bi - acc;
    }
}

// Post-smoothing: out = x + omega D^{-1} (b - A x). At the finest level the
// output is CG's z (FP64) and the block partials of r.z and r.z_old (the
// Polak-Ribiere numerator) are produced per instance (pair layout, see
// InstMap); z_old is read before it is overwritten.
template <int L, typename T, typename TB, typename TO, bool DOT, int U = 8>
__global__ __launch_bounds__(256, (U >= 16 ? 4 : kSparseWaves)) void k_postsmooth(SellView<T> A, const T* __restrict__ dinv, T omega,
                                                     const TB* __restrict__ b, const T* __restrict__ x,
                                                     TO* __restrict__ out, InstMap m, double* __restrict__ part_rz,
                                                     double* __restrict__ part_rzold) {
    static_assert(!DOT || L == 1, "CG partials are produced by the one-lane-per-row finest level");
    __shared__ double sh[kPairSh];
    const int64_t B = row_block(A.xcd);
    const int64_t g = B * blockDim.x + threadIdx.x;
    const int32_t row = sell_perm_row<L>(A.perm, g);  // the finest operator may store its rows in a row order
    double rz = 0.0, rzo = 0.0;
    if (g < (int64_t)A.n_slices * 64) {
        const T ax = sell_row<L, U>(A, g, row, x);
        if ((g & (L - 1)) == 0 && row < A.n_rows) {
            const T v = x[row] + omega * dinv[row] * ((T)b[row] - ax);
            if (DOT) {
                const double ri = (double)b[row];
                rzo = ri * (double)out[row];
                rz = ri * (double)v;
            }
            out[row] = (TO)v;
        }
    }
    if (DOT) {
        int32_t lo, bound;
        block_instances(m, lo, bound, B);
        double* const parts[2] = {part_rz, part_rzold};
        const double vals[2] = {rz, rzo};
        store_pairs<2>(parts, vals, row >= bound, bound, sh, B);
    }
}

// ---- CSR with L lanes per row (long rows of coarse operators) ----------
template <typename T>
struct CsrView {
    const int32_t* __restrict__ rp;
    const int32_t* __restrict__ col;
    const int16_t* __restrict__ d16;  // offsets from offset_base(row) instead of col when set
    const T* __restrict__ val;
    int32_t n_rows, n_cols;
};
template <typename T>
static CsrView<T> cview(const SpMat<T>& A) {
    return CsrView<T>{A.rowptr, A.col, A.d16, A.val, A.n_rows, A.n_cols};
}

// Views of a level's operator with the pre-smoothing values a_ij omega / a_jj.
template <typename T>
static SellView<T> sview(const Level<T>& lv) {
    SellView<T> v = view(lv.A.sell);
    v.val = lv.sval;
    return v;
}
template <typename T>
static CsrView<T> scview(const Level<T>& lv) {
    CsrView<T> v = cview(lv.A);
    v.val = lv.sval;
    return v;
}

// Row sum of A (lanes of one group split the row), with x_j given by f(j).
template <int L, typename T, typename F>
__device__ __forceinline__ T csr_row(const CsrView<T>& A, int32_t row, int lane, F f) {
    // each lane takes entries lane, lane + L, ... of the row, U = 4 at a time:
    // positions past the row's end re-read its last entry and are dropped by a
    // select, so the loads carry no branch; the lane's sum runs in entry order.
    // (Groups of 16 for rows of 614 entries over 64 lanes, one round of loads
    // instead of three, measured slower: 12.0 against 11.4 us, the clamped
    // re-reads of the last group costing more than the rounds saved.)
    constexpr int U = 4;
    T acc = T(0);
    const int32_t end = A.rp[row + 1];
    const int32_t base = offset_base(row, A.n_rows, A.n_cols);
    for (int32_t k = A.rp[row] + lane; k < end; k += U * L) {
        T t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t kk = min(k + u * L, end - 1);
            const int32_t j = A.d16 ? base + (int32_t)A.d16[kk] : A.col[kk];
            t[u] = A.val[kk] * f(j);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (k + u * L < end) ? t[u] : T(0);
    }
    return group_sum<L>(acc);
}

template <int L, typename T>
__global__ __launch_bounds__(256, kSparseWaves) void k_csr_mv(CsrView<T> A, const T* __restrict__ x, T* __restrict__ y, int acc,
                                                 MvInit<T> in) {
    const int64_t g = row_block(0) * blockDim.x + threadIdx.x;
    const int32_t row = (int32_t)(g / L);
    const int lane = (int)(g % L);
    if (row >= A.n_rows) return;  // whole groups leave together
    const T v = csr_row<L>(A, row, lane, [&](int32_t j) { return x[j]; });
    if (lane == 0) mv_store(y, row, v, acc, in);
}

template <int L, typename T, typename TB>
__global__ __launch_bounds__(256, kSparseWaves) void k_csr_presmooth_res(CsrView<T> As, const T* __restrict__ dinv, T omega,
                                                            const TB* __restrict__ b, T* __restrict__ x,
                                                            T* __restrict__ res) {
    const int64_t g = row_block(0) * blockDim.x + threadIdx.x;
    const int32_t row = (int32_t)(g / L);
    const int lane = (int)(g % L);
    if (row >= As.n_rows) return;
    const T acc = csr_row<L>(As, row, lane, [&](int32_t j) { return (T)b[j]; });
    if (lane == 0) {
        const T bi = (T)b[row];
        x[row] = omega * dinv[row] * bi;
        res[row] = bi - acc;
    }
}

template <int L, typename T, typename TB, typename TO>
__global__ __launch_bounds__(256, kSparseWaves) void k_csr_postsmooth(CsrView<T> A, const T* __restrict__ dinv, T omega,
                                                         const TB* __restrict__ b, const T* __restrict__ x,
                                                         TO* __restrict__ out) {
    const int64_t g = row_block(0) * blockDim.x + threadIdx.x;
    const int32_t row = (int32_t)(g / L);
    const int lane = (int)(g % L);
    if (row >= A.n_rows) return;
    const T ax = csr_row<L>(A, row, lane, [&](int32_t j) { return x[j]; });
    if (lane == 0) out[row] = (TO)(x[row] + omega * dinv[row] * ((T)b[row] - ax));
}

template <typename T>
static unsigned csr_grid(const SpMat<T>& A) {
    return (unsigned)(((int64_t)A.n_rows * A.lanes + kBlock - 1) / kBlock);
}

#define EQS_SELL_LANES_SWITCH(Lvar, CALL)                 \
    switch (Lvar) {                                       \
        case 2: { constexpr int L_ = 2; CALL; } break;    \
        case 4: { constexpr int L_ = 4; CALL; } break;    \
        case 8: { constexpr int L_ = 8; CALL; } break;    \
        default: { constexpr int L_ = 1; CALL; } break;   \
    }

// group sizes of k_sell_mv (entries per lane in flight), nested inside EQS_SELL_LANES_SWITCH
#define EQS_UNROLL_SWITCH(Uvar, CALL)                     \
    switch (Uvar) {                                       \
        case 4: { constexpr int U_ = 4; CALL; } break;    \
        case 16: { constexpr int U_ = 16; CALL; } break;  \
        default: { constexpr int U_ = 8; CALL; } break;   \
    }

#define EQS_LANES_SWITCH(Lvar, CALL) \
    switch (Lvar) {                  \
        case 1: { constexpr int L_ = 1; CALL; } break;   \
        case 2: { constexpr int L_ = 2; CALL; } break;   \
        case 4: { constexpr int L_ = 4; CALL; } break;   \
        case 8: { constexpr int L_ = 8; CALL; } break;   \
        case 16: { constexpr int L_ = 16; CALL; } break; \
        case 32: { constexpr int L_ = 32; CALL; } break; \
        default: { constexpr int L_ = 64; CALL; } break; \
    }

template <typename T>
static void launch_mv(hipStream_t s, const SpMat<T>& A, const T* x, T* y, int acc,
                      MvInit<T> in = MvInit<T>{nullptr, nullptr, T(0)}, int role = MV_PLAIN) {
    if (A.fmt == FMT_SELL) {
        EQS_SELL_LANES_SWITCH(A.sell.lanes,
                              EQS_UNROLL_SWITCH(A.sell.unroll,
                                                hipLaunchKernelGGL((sell_mv_kernel<L_, U_, T>(role)),
                                                                   dim3(sell_grid(A.sell)), dim3(kBlock), 0, s,
                                                                   view(A.sell), x, y, acc, in)));
    } else {
        EQS_LANES_SWITCH(A.lanes, hipLaunchKernelGGL((k_csr_mv<L_, T>), dim3(csr_grid(A)), dim3(kBlock), 0, s,
                                                     cview(A), x, y, acc, in));
    }
}

// launch_mv with the launch's own events when kernel class `cls` is profiled
template <typename T>
static void launch_mv_timed(hipStream_t s, eqs_ctx* c, int cls, const SpMat<T>& A, const T* x, T* y, int acc,
                            int role) {
    const MvInit<T> in{nullptr, nullptr, T(0)};
    if (A.fmt == FMT_SELL) {
        EQS_SELL_LANES_SWITCH(A.sell.lanes,
                              EQS_UNROLL_SWITCH(A.sell.unroll,
                                                EQS_LAUNCH_TIMED(c, cls, (sell_mv_kernel<L_, U_, T>(role)),
                                                                 dim3(sell_grid(A.sell)), dim3(kBlock), 0, s,
                                                                 view(A.sell), x, y, acc, in)));
    } else {
        EQS_LANES_SWITCH(A.lanes, EQS_LAUNCH_TIMED(c, cls, (k_csr_mv<L_, T>), dim3(csr_grid(A)), dim3(kBlock), 0, s,
                                                   cview(A), x, y, acc, in));
    }
}

template <typename T, typename TB>
static void launch_presmooth(hipStream_t s, const Level<T>& lv, const TB* b) {
    if (lv.A.fmt == FMT_SELL) {
        EQS_SELL_LANES_SWITCH(lv.A.sell.lanes,
                              EQS_UNROLL_SWITCH(lv.A.sell.unroll,
                                                hipLaunchKernelGGL((k_presmooth_res<L_, T, TB, U_>),
                                                                   dim3(sell_grid(lv.A.sell)), dim3(kBlock), 0, s,
                                                                   sview(lv), (const T*)lv.dinv, (T)lv.omega, b, lv.x,
                                                                   lv.res)));
    } else {
        EQS_LANES_SWITCH(lv.A.lanes, hipLaunchKernelGGL((k_csr_presmooth_res<L_, T, TB>), dim3(csr_grid(lv.A)),
                                                        dim3(kBlock), 0, s, scview(lv), (const T*)lv.dinv,
                                                        (T)lv.omega, b, lv.x, lv.res));
    }
}

// Post-smoothing of a coarse level (no dot products), timed as kernel class
// `cls` when that class is profiled.
template <typename T>
static void launch_postsmooth(hipStream_t s, eqs_ctx* c, int cls, const Level<T>& lv, const T* b, const T* x, T* out) {
    if (lv.A.fmt == FMT_SELL) {
        EQS_SELL_LANES_SWITCH(lv.A.sell.lanes,
                              EQS_UNROLL_SWITCH(lv.A.sell.unroll,
                                                EQS_LAUNCH_TIMED(c, cls, (k_postsmooth<L_, T, T, T, false, U_>),
                                                                 dim3(sell_grid(lv.A.sell)), dim3(kBlock), 0, s,
                                                                 view(lv.A.sell), (const T*)lv.dinv, (T)lv.omega, b,
                                                                 x, out, InstMap{nullptr, nullptr, 0, -1}, nullptr,
                                                                 nullptr)));
    } else {
        EQS_LANES_SWITCH(lv.A.lanes, EQS_LAUNCH_TIMED(c, cls, (k_csr_postsmooth<L_, T, T, T>), dim3(csr_grid(lv.A)),
                                                      dim3(kBlock), 0, s, cview(lv.A), (const T*)lv.dinv,
                                                      (T)lv.omega, b, x, out));
    }
}

// Time per product y = A x (ms) for the layout tuner: the median over `reps`
// rounds (after one warm-up round) of kBatch back-to-back launches between two
// events, divided by kBatch. A single launch between events carries the
// events' own cost and jitter, which at 5-20 us per launch is as large as the
// differences between layouts; back to back, the launches also run as they
// do inside the V-cycle, one after another on the stream.
template <typename T>
double time_mv(eqs_ctx* c, const SpMat<T>& A, const T* x, T* y, int reps) {
    constexpr int kBatch = 8;
    hipEvent_t e0, e1;
    EQS_HIP(hipEventCreate(&e0));
    EQS_HIP(hipEventCreate(&e1));
    std::vector<float> ms;
    for (int r = 0; r < reps + 1; ++r) {
        EQS_HIP(hipEventRecord(e0, c->stream));
        for (int k = 0; k < kBatch; ++k) launch_mv<T>(c->stream, A, x, y, 0);
        EQS_HIP(hipEventRecord(e1, c->stream));
        EQS_HIP(hipEventSynchronize(e1));
        float t = 0.0f;
        EQS_HIP(hipEventElapsedTime(&t, e0, e1));
        if (r >= 1) ms.push_back(t / kBatch);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}
template double time_mv<double>(eqs_ctx*, const SpMat<double>&, const double*, double*, int);
template double time_mv<float>(eqs_ctx*, const SpMat<float>&, const float*, float*, int);

// Coarsest level: x = A^{-1} b with the dense inverse. The inverse is
// symmetric, so row i is stored contiguously (column i); one wavefront per row
// splits the dot product over its 64 lanes.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse(const T* __restrict__ inv, const T* __restrict__ b,
                                                 T* __restrict__ x, int32_t n) {
    const int32_t i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    T acc = T(0);
    for (int32_t k = lane; k < n; k += 64) acc += inv[(int64_t)i * n + k] * b[k];
    acc = group_sum<64>(acc);
    if (lane == 0) x[i] = acc;
}

// Coarsest level with the restriction folded in: x = (A^{-1} R) r, one
// workgroup of kCoarseThreads threads per coarse row of the dense row-major
// product matrix C. Each thread sums its columns j = t, t + kCoarseThreads, ...
// eight at a time (loads in flight together: one round covers 8192 columns),
// then the block sums in a fixed order.
constexpr int kCoarseThreads = 1024;
template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_restrict(const T* __restrict__ C, const T* __restrict__ r,
                                                                     T* __restrict__ x, int32_t n, int32_t nf) {
    __shared__ double sh[kCoarseThreads / 64];
    const int32_t i = blockIdx.x;
    const T* row = C + (int64_t)i * nf;
    T acc = T(0);
    for (int32_t j0 = threadIdx.x; j0 < nf; j0 += 8 * kCoarseThreads) {
        T t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t j = min(j0 + u * kCoarseThreads, nf - 1);
            t[u] = row[j] * r[j];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += (j0 + u * kCoarseThreads < nf) ? t[u] : T(0);
    }
    double v = (double)acc;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0 && i < n) {
        double t = 0.0;
        for (int w = 0; w < kCoarseThreads / 64; ++w) t += sh[w];
        x[i] = (T)t;
    }
}

// Single-level hierarchy: z = A^{-1} r with the same r.z partials as k_postsmooth.
template <typename T, bool DOT>
__global__ __launch_bounds__(256) void k_dense_precond(const T* __restrict__ inv, const double* __restrict__ r,
                                                        double* __restrict__ z, int32_t n, InstMap m,
                                                        double* __restrict__ part_rz, double* __restrict__ part_rzold) {
    __shared__ double sh[kPairSh];
    const int64_t B = blockIdx.x;
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0.0, rzo = 0.0;
    if (i < n) {
        T acc = T(0);
        for (int32_t k = 0; k < n; ++k) acc += inv[(int64_t)k * n + i] * (T)r[k];
        if (DOT) {
            rzo = r[i] * z[i];
            rz = r[i] * (double)acc;
        }
        z[i] = (double)acc;
    }
    if (DOT) {
        int32_t lo, bound;
        block_instances(m, lo, bound, B);
        double* const parts[2] = {part_rz, part_rzold};
        const double vals[2] = {rz, rzo};
        store_pairs<2>(parts, vals, i >= bound, bound, sh, B);
    }
}

static InstMap inst_map(const eqs_ctx* c) {
    return InstMap{c->d_inst_row, c->d_blk_inst, (int32_t)c->n_inst, c->n_inst == 1 ? (int32_t)c->n_free : -1};
}

// V(1,1) cycle z = B r. r and z are FP64 (CG's vectors); the hierarchy is T.
// With part_rz the finest post-smoothing also writes the r.z and r.z_old
// partials (pair layout). Its kernels do not test CG's stop flag: a test on a
// flag in memory makes every kernel wait for it, and for the kernel arguments
// loaded after the branch, before its first data load (together about 3 of
// 186 us per cycle at 2.1M DOF, nine kernels). A CG iteration launched
// after convergence therefore runs its V-cycle on the unchanged residual; it
// writes only the cycle's temporaries, z and the r.z partials, none of which a
// finished solve or a restart (beta = 0) reads.
template <typename T>
void vcycle(hipStream_t s, eqs_ctx* c, Hierarchy<T>& h, const double* r, double* z, double* part_rz,
            double* part_rzold) {
    const int L = (int)h.lv.size();
    dim3 b(kBlock);
    if (L == 1) {
        // the matrix is small enough for its dense inverse: z = A^{-1} r
        Level<T>& lv = h.lv[0];
        if (part_rz)
            hipLaunchKernelGGL((k_dense_precond<T, true>), dim3(grid_for(lv.n)), b, 0, s, (const T*)lv.dense_inv, r, z,
                               lv.n, inst_map(c), part_rz, part_rzold);
        else
            hipLaunchKernelGGL((k_dense_precond<T, false>), dim3(grid_for(lv.n)), b, 0, s, (const T*)lv.dense_inv, r,
                               z, lv.n, inst_map(c), part_rz, part_rzold);
        return;
    }
    // descend
    for (int l = 0; l < L - 1; ++l) {
        Level<T>& lv = h.lv[l];
        if (lv.tail) break;  // folded into the coarse product and [G Q] (the last level above the coarsest)
        if (lv.fold_pre) {  // R holds R (I - A w D^-1): restrict b itself
            launch_mv<T>(s, lv.R, (const T*)lv.b, h.lv[l + 1].b, 0, MvInit<T>{nullptr, nullptr, T(0)},
                         MV_RESTRICT);
            continue;
        }
        if (l == 0) {
            // the finest operator is always SELL-64 (see tuned_spmat)
            EQS_LAUNCH_TIMED(c, EQS_KCLASS_PRESMOOTH0, (k_presmooth_res<1, T, double>), dim3(sell_grid(lv.A.sell)), b, 0,
                             s, sview(lv), (const T*)lv.dinv, (T)lv.omega, r, lv.x, lv.res);
        } else {
            launch_presmooth<T, T>(s, lv, (const T*)lv.b);
        }
        if (l + 1 < L - 1 || !h.lv[L - 1].coarse_R) {
            if (l == 0)
                launch_mv_timed<T>(s, c, EQS_KCLASS_RESTRICT0, lv.R, (const T*)lv.res, h.lv[1].b, 0,
                                   MV_RESTRICT);
            else
                launch_mv<T>(s, lv.R, (const T*)lv.res, h.lv[l + 1].b, 0, MvInit<T>{nullptr, nullptr, T(0)},
                             MV_RESTRICT);
        }
        if (l == 0) prof_begin(c, EQS_KCLASS_VCOARSE, s);
    }
    {
        Level<T>& lc = h.lv[L - 1];
        const Level<T>& la = h.lv[L - 2];
        if (lc.coarse_R)  // restriction (and, folded, the level above's pre-smoothing) and coarse solve in one product
            hipLaunchKernelGGL(k_coarse_restrict<T>, dim3((unsigned)lc.n), dim3(kCoarseThreads), 0, s,
                               (const T*)lc.coarse_R, (const T*)(la.tail ? la.b : la.res), lc.x, lc.n,
                               lc.coarse_R_cols);
        else
            hipLaunchKernelGGL(k_coarse<T>, dim3(grid_for((int64_t)lc.n * 64)), b, 0, s, (const T*)lc.dense_inv,
                               (const T*)lc.b, lc.x, lc.n);
    }
    // ascend
    for (int l = L - 2; l >= 0; --l) {
        Level<T>& lv = h.lv[l];
        if (lv.tail) {  // xs = G b + Q x_coarse on the stacked [b; x_coarse]
            launch_mv<T>(s, lv.GQ, (const T*)lv.b, lv.xs, 0);
            continue;
        }
        const T* xc = (l + 1 == L - 1) ? h.lv[l + 1].x : h.lv[l + 1].xs;
        if (l == 0) prof_end(c, EQS_KCLASS_VCOARSE, s);
        if (lv.fold_pre)  // x = w D^-1 b (the folded pre-smoother's result) + P xc
            launch_mv<T>(s, lv.P, xc, lv.x, 2, MvInit<T>{(const T*)lv.dinv, (const T*)lv.b, (T)lv.omega},
                         MV_PROLONG);
        else if (l == 0)
            launch_mv_timed<T>(s, c, EQS_KCLASS_PROLONG0, lv.P, xc, lv.x, 1, MV_PROLONG);
        else
            launch_mv<T>(s, lv.P, xc, lv.x, 1, MvInit<T>{nullptr, nullptr, T(0)}, MV_PROLONG);
        if (l > 0) {
            launch_postsmooth<T>(s, c, l == 1 ? EQS_KCLASS_POSTSMOOTH1 : -1, lv, (const T*)lv.b, (const T*)lv.x,
                                 lv.xs);
        } else {
            // the finest operator is always SELL-64 (see tuned_spmat)
            if (part_rz)
                EQS_LAUNCH_TIMED(c, EQS_KCLASS_POSTSMOOTH0, (k_postsmooth<1, T, double, double, true>),
                                 dim3(sell_grid(lv.A.sell)), b, 0, s, view(lv.A.sell), (const T*)lv.dinv, (T)lv.omega,
                                 r, (const T*)lv.x, z, inst_map(c), part_rz, part_rzold);
            else
                EQS_LAUNCH_TIMED(c, EQS_KCLASS_POSTSMOOTH0, (k_postsmooth<1, T, double, double, false>),
                                 dim3(sell_grid(lv.A.sell)), b, 0, s, view(lv.A.sell), (const T*)lv.dinv, (T)lv.omega,
                                 r, (const T*)lv.x, z, InstMap{nullptr, nullptr, 0, -1}, nullptr, nullptr);
        }
    }
}

template void vcycle<double>(hipStream_t, eqs_ctx*, Hierarchy<double>&, const double*, double*, double*, double*);
template void vcycle<float>(hipStream_t, eqs_ctx*, Hierarchy<float>&, const double*, double*, double*, double*);

// ------------------------------------------------------------------ CG
// Every instance runs its own CG (own scalars, own convergence test); the
// sparse products and the V-cycle act on all instances at once (block-diagonal
// operators). Rows of an instance that is done are left untouched.

// r = rhs - M x; pair partials of |r|^2 and |rhs|^2. With mx_out, M x is
// also stored (the next solve that starts from this x then needs no product).
__global__ __launch_bounds__(256, kSparseWaves) void k_pcg_residual(SellView<double> M, InstMap m, const double* __restrict__ rhs,
                                                       const double* __restrict__ x, double* __restrict__ r,
                                                       double* __restrict__ part_rr, double* __restrict__ part_bb,
                                                       double* __restrict__ mx_out, const int32_t* __restrict__ when_done) {
    __shared__ double sh[kPairSh];
    if (when_done && !*when_done) return;  // queued ahead of the host's decision: only once every instance is done
    const int64_t B = row_block(M.xcd);
    const int64_t g = B * blockDim.x + threadIdx.x;
    const int32_t row = sell_perm_row<1>(M.perm, g);  // the row order, if any, stays inside the block's rows
    double rr = 0.0, bb = 0.0;
    if (g < (int64_t)M.n_slices * 64) {
        const double mx = sell_row<1>(M, g, row, x);
        if (row < M.n_rows) {
            const double bi = rhs[row];
            const double ri = bi - mx;
            r[row] = ri;
            if (mx_out) mx_out[row] = mx;
            rr = ri * ri;
            bb = bi * bi;
        }
    }
    int32_t lo, bound;
    block_instances(m, lo, bound, B);
    double* const parts[2] = {part_rr, part_bb};
    const double vals[2] = {rr, bb};
    store_pairs<2>(parts, vals, row >= bound, bound, sh, B);
}

// r = rhs - mx with mx = M x stored by the residual check that ended the
// previous solve from the same x (the same products, so the same r); pair
// partials as k_pcg_residual.
__global__ __launch_bounds__(256) void k_pcg_residual_mx(InstMap m, const double* __restrict__ rhs,
                                                          const double* __restrict__ mx, double* __restrict__ r,
                                                          int64_t n, double* __restrict__ part_rr,
                                                          double* __restrict__ part_bb) {
    __shared__ double sh[kPairSh];
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0, bb = 0.0;
    if (row < n) {
        const double bi = rhs[row];
        const double ri = bi - mx[row];
        r[row] = ri;
        rr = ri * ri;
        bb = bi * bi;
    }
    int32_t lo, bound;
    block_instances(m, lo, bound, blockIdx.x);
    double* const parts[2] = {part_rr, part_bb};
    const double vals[2] = {rr, bb};
    store_pairs<2>(parts, vals, row >= bound, bound, sh, blockIdx.x);
}

// q = M z + beta q, p = z + beta p (so q = M p without a second pass); pair partials of p.q.
// stop (may be NULL) ends the launch at entry. ONE: a single instance; nothing in it waits for the scalars
// before the row's loads are issued: they are read with vector loads issued first, and used by selects, not
// branches (a branch on a loaded flag is waited for where the compiler places it, ahead of the loads). It
// writes p and q even after the solve has converged: a finished solve, and a restart (beta = 0), read neither.
template <bool ONE>
__global__ __launch_bounds__(256, kSparseWaves) void k_pcg_spmv(SellView<double> M, InstMap m, const double* __restrict__ z,
                                                   double* __restrict__ p, double* __restrict__ q,
                                                   double* __restrict__ part_pq, const PcgScalars* __restrict__ scal,
                                                   const int32_t* __restrict__ stop) {
    __shared__ double sh[kPairSh];
    if (stop && *stop) return;
    const int64_t B = row_block(M.xcd);
    const int64_t g = B * blockDim.x + threadIdx.x;
    const int32_t row = sell_perm_row<1>(M.perm, g);  // the row order, if any, stays inside the block's rows
    double pq = 0.0;
    if constexpr (ONE) {
        const double beta = vec_load(&scal->beta);
        const int32_t fresh = vec_load(&scal->fresh);
        const int32_t bound = m.rows1;
        if (g < (int64_t)M.n_slices * 64) {
            const double mz = sell_row<1>(M, g, row, z);
            if (row < M.n_rows) {
                const double zi = z[row], po = p[row], qo = q[row];
                const double pi = fresh ? zi : zi + beta * po;
                const double qi = fresh ? mz : mz + beta * qo;
                p[row] = pi;
                q[row] = qi;
                pq = pi * qi;
            }
        }
        double* const parts[1] = {part_pq};
        const double vals[1] = {pq};
        store_pairs<1>(parts, vals, row >= bound, bound, sh, B);
    } else {
        int32_t lo, bound;
        block_instances(m, lo, bound, B);
        const bool second = row >= bound;
        const PcgScalars& S = scal[min(second ? lo + 1 : lo, m.n_inst - 1)];
        if (g < (int64_t)M.n_slices * 64) {
            const double mz = sell_row<1>(M, g, row, z);
            if (row < M.n_rows && !S.done) {
                double pi, qi;
                if (S.fresh) {
                    pi = z[row];
                    qi = mz;
                } else {
                    pi = z[row] + S.beta * p[row];
                    qi = mz + S.beta * q[row];
                }
                p[row] = pi;
                q[row] = qi;
                pq = pi * qi;
            }
        }
        double* const parts[1] = {part_pq};
        const double vals[1] = {pq};
        store_pairs<1>(parts, vals, second, bound, sh, B);
    }
}
// x += alpha p, r -= alpha q; pair partials of r.r. stop and ONE as for k_pcg_spmv: with one instance the done
// flag selects the stored values (x and r written back unchanged once the solve has converged), so the four
// streams' loads do not wait for it. xcd: M's block order, so that each workgroup reads the p and q rows the SpMV
// wrote on the same XCD.
template <bool ONE>
__global__ __launch_bounds__(256) void k_pcg_update(InstMap m, double* __restrict__ x, double* __restrict__ r,
                                                     const double* __restrict__ p, const double* __restrict__ q,
                                                     int64_t n, double* __restrict__ part_rr,
                                                     const PcgScalars* __restrict__ scal,
                                                     const int32_t* __restrict__ stop, int32_t xcd) {
    __shared__ double sh[kPairSh];
    if (stop && *stop) return;
    const int64_t B = row_block(xcd);
    const int64_t i = B * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if constexpr (ONE) {
        const double alpha = vec_load(&scal->alpha);
        const int32_t done = vec_load(&scal->done);
        const int32_t bound = m.rows1;
        if (i < n) {
            const double pi = p[i], qi = q[i], xi = x[i], ri0 = r[i];
            __builtin_amdgcn_sched_barrier(0);  // the four loads are issued before anything waits
            const double xn = xi + alpha * pi, rn = ri0 - alpha * qi;
            x[i] = done ? xi : xn;
            r[i] = done ? ri0 : rn;
            rr = done ? 0.0 : rn * rn;
        }
        double* const parts[1] = {part_rr};
        const double vals[1] = {rr};
        store_pairs<1>(parts, vals, i >= bound, bound, sh, B);
    } else {
        int32_t lo, bound;
        block_instances(m, lo, bound, B);
        const bool second = i >= bound;
        const PcgScalars& S = scal[min(second ? lo + 1 : lo, m.n_inst - 1)];
        if (i < n && !S.done) {
            const double pi = p[i], qi = q[i], xi = x[i], ri0 = r[i];
            __builtin_amdgcn_sched_barrier(0);  // the four loads are issued before anything waits
            x[i] = xi + S.alpha * pi;
            const double ri = ri0 - S.alpha * qi;
            r[i] = ri;
            rr = ri * ri;
        }
        double* const parts[1] = {part_rr};
        const double vals[1] = {rr};
        store_pairs<1>(parts, vals, second, bound, sh, B);
    }
}

// x = 0 on the rows of instances whose right-hand side is zero.
__global__ void k_zero_rhs_rows(InstMap m, double* __restrict__ x, int64_t n, const PcgScalars* __restrict__ scal) {
    int32_t lo, bound;
    block_instances(m, lo, bound, blockIdx.x);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && scal[min(i >= bound ? lo + 1 : lo, m.n_inst - 1)].bb == 0.0) x[i] = 0.0;
}

// Summary over the instances, mirrored with all scalars to the host; every
// thread of the block takes part (counts and maxima do not depend on order).
// A NaN relative residual is reported as +inf.
__device__ void summarise(const PcgScalars* __restrict__ s, int32_t n, PcgSummary* __restrict__ sum,
                          PcgSummary* __restrict__ host_sum, PcgScalars* __restrict__ host) {
    __shared__ int32_t cnt[5];  // active, breakdown, not converged, zero rhs, max it
    __shared__ unsigned long long max_rel;
    if (threadIdx.x == 0) {
        cnt[0] = cnt[1] = cnt[2] = cnt[3] = cnt[4] = 0;
        max_rel = 0ull;
    }
    __syncthreads();
    int32_t act = 0, brk = 0, nc = 0, zr = 0, mit = 0;
    double mr = 0.0;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const PcgScalars x = s[i];
        host[i] = x;
        act += x.done ? 0 : 1;
        brk += x.status == EQS_ERR_BREAKDOWN;
        nc += x.status == EQS_ERR_NOT_CONVERGED;
        zr += x.bb == 0.0;
        mit = max(mit, x.it);
        mr = fmax(mr, isnan(x.relres) ? INFINITY : x.relres);
    }
    if (act) atomicAdd(&cnt[0], act);
    if (brk) atomicAdd(&cnt[1], brk);
    if (nc) atomicAdd(&cnt[2], nc);
    if (zr) atomicAdd(&cnt[3], zr);
    if (mit) atomicMax(&cnt[4], mit);
    if (mr > 0.0) atomicMax(&max_rel, (unsigned long long)__double_as_longlong(mr));  // order of non-negative doubles
    __syncthreads();
    if (threadIdx.x == 0) {
        PcgSummary v{};
        v.all_done = cnt[0] == 0;
        v.n_active = cnt[0];
        v.n_breakdown = cnt[1];
        v.n_notconv = cnt[2];
        v.n_zero_rhs = cnt[3];
        v.max_it = cnt[4];
        v.max_relres = __longlong_as_double((long long)max_rel);
        *sum = v;
        *host_sum = v;
    }
}

// The finalisers below issue their independent loads (the stop flag, the
// instance's scalars, the partials) before any of them is waited for, and test
// the flag only where it matters: a finaliser costs about one memory latency
// plus the reduction, not one latency per dependent step. Two things keep it
// so. With one instance (the plain form) the flag and the scalars are read
// with vector loads (vec_load): being uniform, plain loads would become scalar
// loads, and the wait for the kernel argument the partials' addresses need
// would then also wait for them. With several, each thread reads only the
// scalar fields it uses and stores only those it changes (a copy of the whole
// struct, read, modified and written back, would keep the untouched fields in
// LDS, and the loads into it would be waited for before the partials' loads
// are issued).
struct FinIn {
    double rho, bb, tol2;
    int32_t it, maxit, done, fresh, flexible;
};
__device__ __forceinline__ FinIn fin_fields(const PcgScalars* __restrict__ s, int32_t i) {
    const PcgScalars* p = s + i;
    return FinIn{p->rho, p->bb, p->tol2, p->it, p->maxit, p->done, p->fresh, p->flexible};
}
// the fields of instance kFinWaves * blockIdx.x + threadIdx.x, the one this thread's body call serves
// (for_each_instance_sum)
__device__ __forceinline__ FinIn prefetch_fields(const PcgScalars* __restrict__ s, const InstMap& m) {
    FinIn x{};
    const int32_t i = (int32_t)blockIdx.x * kFinWaves + (int32_t)threadIdx.x;
    if ((int32_t)threadIdx.x < kFinWaves && i < m.n_inst) x = fin_fields(s, i);
    return x;
}

// One instance: every wavefront sums an equal share of the blocks' first
// partials (the second is 0 when there is one instance); thread 0 gets the
// totals. The order of the additions is fixed.
template <int NP>
__device__ __forceinline__ void single_instance_sums(const double* const (&parts)[NP], int32_t rows,
                                                     double (&out)[NP]) {
    __shared__ double sh[NP][kFinWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t nb = (rows + 255) >> 8;
    const int32_t lo = (int32_t)(((int64_t)nb * wave) / kFinWaves);
    const int32_t hi = (int32_t)(((int64_t)nb * (wave + 1)) / kFinWaves) - 1;
    double v[NP];
    wave_range_sums<NP>(parts, lo, hi, v);
    if (lane == 0)
#pragma unroll
        for (int p = 0; p < NP; ++p) sh[p][wave] = v[p];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        double t = 0.0;
        if (threadIdx.x == 0)
            for (int w = 0; w < kFinWaves; ++w) t += sh[p][w];
        out[p] = t;
    }
}

// CG decisions from the reduced dot products; 0 = carry on.
enum { FIN_GO = 0, FIN_CONVERGED = 1, FIN_BREAKDOWN = 2, FIN_OUT_OF_ITERS = 3 };
__device__ __forceinline__ int fin_positive(double d) { return (!(d > 0.0) || !isfinite(d)) ? FIN_BREAKDOWN : FIN_GO; }
__device__ __forceinline__ int fin_conv_decision(double rr, double tol2, int32_t it, int32_t maxit) {
    if (rr <= tol2) return FIN_CONVERGED;
    if (!isfinite(rr)) return FIN_BREAKDOWN;
    if (it >= maxit) return FIN_OUT_OF_ITERS;
    return FIN_GO;
}
__device__ __forceinline__ void set_breakdown(PcgScalars* __restrict__ p) {
    p->done = 1;
    p->status = EQS_ERR_BREAKDOWN;
}
__device__ __forceinline__ double fin_beta_of(const FinIn& x, double rz, double rzo) {
    return x.fresh ? 0.0 : (x.flexible ? (rz - rzo) / x.rho : rz / x.rho);
}

// mode 0: start of a solve (it = 0); mode 1: restart from the true residual
// (iteration count kept; broken-down instances stay so). An instance is done
// when |r| <= rtol |rhs|, rhs = 0, or its iteration budget is spent.
// force (may be NULL): a one-shot flag for tests of the restart path; when
// set, this check treats every instance as not yet converged (it then
// continues from its true residual) and clears the flag. ONE: a single
// instance (its scalars handled field by field, as in k_fin_conv).
template <bool ONE>
__global__ __launch_bounds__(kFin) void k_fin_start(PcgScalars* __restrict__ s, InstMap m, const double* __restrict__ prr,
                                                     const double* __restrict__ pbb, double rtol, int32_t maxit,
                                                     int32_t flexible, int32_t mode, PcgSummary* __restrict__ sum,
                                                     PcgSummary* __restrict__ host_sum,
                                                     PcgScalars* __restrict__ host, int32_t when_done,
                                                     int32_t* __restrict__ force) {
    const double* parts[2] = {prr, pbb};
    if constexpr (ONE) {
        // both flags are read unconditionally (a load under a branch is waited for at the branch's end)
        const int32_t all_done = vec_load(&sum->all_done);
        const int32_t force_raw = vec_load(force ? (const int32_t*)force : &sum->all_done);
        const PcgScalars* p = s;
        double rho = vec_load(&p->rho), rho_old = vec_load(&p->rho_old), alpha = vec_load(&p->alpha);
        double tol2 = vec_load(&p->tol2), rr = vec_load(&p->rr), relres = vec_load(&p->relres);
        double beta = vec_load(&p->beta), bb = vec_load(&p->bb);
        int32_t it = vec_load(&p->it), mx = vec_load(&p->maxit), done = vec_load(&p->done);
        int32_t status = vec_load(&p->status), fresh = vec_load(&p->fresh), flex = vec_load(&p->flexible);
        double v[2];
        single_instance_sums<2>(parts, m.rows1, v);
        // the flags are tested only here, so that no wait for them precedes the partials' loads
        const int32_t skip = when_done ? !all_done : 0;
        const int32_t forced = (mode == 1 && force) ? force_raw : 0;
        if (threadIdx.x != 0 || skip) return;  // skip pairs with k_pcg_residual's when_done
        if (forced) *force = 0;
        if (mode == 0) {
            rho = rho_old = alpha = 0.0;
            it = 0;
            mx = maxit;
            flex = flexible;
            tol2 = rtol * rtol * v[1];
        }
        if (mode == 0 || status != EQS_ERR_BREAKDOWN) {
            bb = v[1];
            rr = v[0];
            relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
            fresh = 1;
            beta = 0.0;
            status = EQS_OK;
            done = 0;
            if (bb == 0.0 || (rr <= tol2 && !forced)) {
                done = 1;
            } else if (!isfinite(rr) || !isfinite(bb)) {
                done = 1;
                status = EQS_ERR_BREAKDOWN;
            } else if (it >= mx) {
                done = 1;
                status = EQS_ERR_NOT_CONVERGED;
            }
        }
        PcgScalars h;
        h.bb = bb;
        h.rr = rr;
        h.rho = rho;
        h.rho_old = rho_old;
        h.beta = beta;
        h.alpha = alpha;
        h.tol2 = tol2;
        h.relres = relres;
        h.it = it;
        h.maxit = mx;
        h.done = done;
        h.status = status;
        h.fresh = fresh;
        h.flexible = flex;
        *s = h;
        *host = h;
        PcgSummary v1;
        v1.all_done = done ? 1 : 0;
        v1.n_active = done ? 0 : 1;
        v1.n_breakdown = status == EQS_ERR_BREAKDOWN;
        v1.n_notconv = status == EQS_ERR_NOT_CONVERGED;
        v1.n_zero_rhs = bb == 0.0;
        v1.max_it = max(it, 0);
        const double mr = isnan(relres) ? INFINITY : relres;
        v1.max_relres = mr > 0.0 ? mr : 0.0;
        *sum = v1;
        *host_sum = v1;
    } else {
        if (when_done && !sum->all_done) return;  // pairs with k_pcg_residual's when_done
        const int32_t forced = (mode == 1 && force) ? *force : 0;
        __syncthreads();
        // with several workgroups k_fin_summary clears the flag once every workgroup has read it
        if (forced && threadIdx.x == 0 && gridDim.x == 1) *force = 0;
        // field by field, as in the single-instance form (a copy of the whole struct would be kept in LDS)
        for_each_instance_sum<2>(parts, m, [&](int32_t i, const double* v) {
            const double rr = v[0], bb = v[1];
            PcgScalars* p = s + i;
            int32_t it, mx;
            double tol2;
            if (mode == 0) {  // a fresh solve: every field set, the others 0
                it = 0;
                mx = maxit;
                tol2 = rtol * rtol * bb;
                p->rho = 0.0;
                p->rho_old = 0.0;
                p->alpha = 0.0;
                p->it = 0;
                p->maxit = maxit;
                p->flexible = flexible;
                p->tol2 = tol2;
            } else {
                if (p->status == EQS_ERR_BREAKDOWN) return;
                it = p->it;
                mx = p->maxit;
                tol2 = p->tol2;
            }
            int32_t done = 0, status = EQS_OK;
            if (bb == 0.0 || (rr <= tol2 && !forced)) {
                done = 1;
            } else if (!isfinite(rr) || !isfinite(bb)) {
                done = 1;
                status = EQS_ERR_BREAKDOWN;
            } else if (it >= mx) {
                done = 1;
                status = EQS_ERR_NOT_CONVERGED;
            }
            p->bb = bb;
            p->rr = rr;
            p->relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
            p->fresh = 1;
            p->beta = 0.0;
            p->status = status;
            p->done = done;
        });
        if (gridDim.x > 1) return;  // k_fin_summary follows
        __syncthreads();
        summarise(s, m.n_inst, sum, host_sum, host);
    }
}

// beta from r.z (Polak-Ribiere with r.z_old when flexible). ONE: a single
// instance (InstMap::rows1 >= 0); the two forms are separate kernels so each
// gets its own register allocation.
template <bool ONE>
__global__ __launch_bounds__(kFin) void k_fin_beta(PcgScalars* __restrict__ s, InstMap m,
                                                    const double* __restrict__ prz, const double* __restrict__ przold,
                                                    const int32_t* __restrict__ stop) {
    const int32_t stopped = ONE ? vec_load(stop) : *stop;
    const double* parts[2] = {prz, przold};
    if constexpr (ONE) {
        // only the fields used: a vector load whose result is never read still holds its register
        FinIn x{};
        x.rho = vec_load(&s->rho);
        x.done = vec_load(&s->done);
        x.fresh = vec_load(&s->fresh);
        x.flexible = vec_load(&s->flexible);
        double v[2];
        single_instance_sums<2>(parts, m.rows1, v);
        if (threadIdx.x == 0 && !stopped && !x.done) {
            if (fin_positive(v[0]) != FIN_GO) {
                set_breakdown(s);
            } else {
                s->beta = fin_beta_of(x, v[0], v[1]);
                s->rho = v[0];
            }
        }
    } else {
        const FinIn pre = prefetch_fields(s, m);
        for_each_instance_sum<2>(parts, m, [&](int32_t i, const double* v) {
            if (stopped) return;
            const FinIn& x = pre;
            if (x.done) return;
            PcgScalars* p = s + i;
            if (fin_positive(v[0]) != FIN_GO) {
                set_breakdown(p);
            } else {
                p->beta = fin_beta_of(x, v[0], v[1]);
                p->rho = v[0];
            }
        });
    }
}

template <bool ONE>
__global__ __launch_bounds__(kFin) void k_fin_alpha(PcgScalars* __restrict__ s, InstMap m,
                                                     const double* __restrict__ ppq, const int32_t* __restrict__ stop) {
    const int32_t stopped = ONE ? vec_load(stop) : *stop;
    const double* parts[1] = {ppq};
    if constexpr (ONE) {
        const double rho = vec_load(&s->rho);
        const int32_t done = vec_load(&s->done);
        double v[1];
        single_instance_sums<1>(parts, m.rows1, v);
        if (threadIdx.x == 0 && !stopped && !done) {
            if (fin_positive(v[0]) != FIN_GO) {
                set_breakdown(s);
            } else {
                s->alpha = rho / v[0];
                s->fresh = 0;
            }
        }
    } else {
        const FinIn pre = prefetch_fields(s, m);
        for_each_instance_sum<1>(parts, m, [&](int32_t i, const double* v) {
            if (stopped) return;
            const FinIn& x = pre;
            if (x.done) return;
            PcgScalars* p = s + i;
            if (fin_positive(v[0]) != FIN_GO) {
                set_breakdown(p);
            } else {
                p->alpha = x.rho / v[0];
                p->fresh = 0;
            }
        });
    }
}

template <bool ONE>
__global__ __launch_bounds__(kFin) void k_fin_conv(PcgScalars* __restrict__ s, InstMap m,
                                                    const double* __restrict__ prr, PcgSummary* __restrict__ sum,
                                                    PcgSummary* __restrict__ host_sum, PcgScalars* __restrict__ host) {
    const int32_t stopped = ONE ? vec_load(&sum->all_done) : sum->all_done;
    const double* parts[1] = {prr};
    if constexpr (ONE) {
        // the instance's scalars and the summary as summarise() leaves them for one instance; the struct is
        // handled field by field (a whole-struct copy would be kept in LDS)
        const PcgScalars* p = s;
        const double bb = vec_load(&p->bb), rho = vec_load(&p->rho), rho_old = vec_load(&p->rho_old);
        const double beta = vec_load(&p->beta), alpha = vec_load(&p->alpha), tol2 = vec_load(&p->tol2);
        const double rr0 = vec_load(&p->rr), relres0 = vec_load(&p->relres);
        const int32_t it0 = vec_load(&p->it), maxit = vec_load(&p->maxit), done0 = vec_load(&p->done);
        const int32_t status0 = vec_load(&p->status), fresh = vec_load(&p->fresh), flexible = vec_load(&p->flexible);
        double v[1];
        single_instance_sums<1>(parts, m.rows1, v);
        if (threadIdx.x == 0 && !stopped) {
            double rr = rr0, relres = relres0;
            int32_t it = it0, done = done0, status = status0;
            if (!done0) {
                rr = v[0];
                relres = sqrt(rr / bb);
                it = it0 + 1;
                const int d = fin_conv_decision(rr, tol2, it, maxit);
                if (d != FIN_GO) done = 1;
                if (d == FIN_BREAKDOWN) status = EQS_ERR_BREAKDOWN;
                if (d == FIN_OUT_OF_ITERS) status = EQS_ERR_NOT_CONVERGED;
                s->rr = rr;
                s->relres = relres;
                s->it = it;
                s->done = done;
                s->status = status;
            }
            PcgScalars h;
            h.bb = bb;
            h.rr = rr;
            h.rho = rho;
            h.rho_old = rho_old;
            h.beta = beta;
            h.alpha = alpha;
            h.tol2 = tol2;
            h.relres = relres;
            h.it = it;
            h.maxit = maxit;
            h.done = done;
            h.status = status;
            h.fresh = fresh;
            h.flexible = flexible;
            *host = h;
            PcgSummary v1;
            v1.all_done = done ? 1 : 0;
            v1.n_active = done ? 0 : 1;
            v1.n_breakdown = status == EQS_ERR_BREAKDOWN;
            v1.n_notconv = status == EQS_ERR_NOT_CONVERGED;
            v1.n_zero_rhs = bb == 0.0;
            v1.max_it = max(it, 0);
            const double mr = isnan(relres) ? INFINITY : relres;
            v1.max_relres = mr > 0.0 ? mr : 0.0;
            *sum = v1;
            *host_sum = v1;
        }
    } else {
        const FinIn pre = prefetch_fields(s, m);
        for_each_instance_sum<1>(parts, m, [&](int32_t i, const double* v) {
            if (stopped) return;
            const FinIn& x = pre;
            if (x.done) return;
            const double rr = v[0];
            const int32_t it = x.it + 1;
            PcgScalars* p = s + i;
            p->rr = rr;
            p->relres = sqrt(rr / x.bb);
            p->it = it;
            const int d = fin_conv_decision(rr, x.tol2, it, x.maxit);
            if (d == FIN_CONVERGED) p->done = 1;
            else if (d == FIN_BREAKDOWN) set_breakdown(p);
            else if (d == FIN_OUT_OF_ITERS) {
                p->done = 1;
                p->status = EQS_ERR_NOT_CONVERGED;
            }
        });
        if (stopped || gridDim.x > 1) return;  // the summary already says all done, or k_fin_summary follows
        __syncthreads();
        summarise(s, m.n_inst, sum, host_sum, host);
    }
}

// The summary of every instance's CG state after a finaliser of several
// workgroups (more than kFinWaves instances), which cannot summarise itself:
// what summarise() does at the end of a one-workgroup finaliser. gate 0:
// always; 1: only while the summary does not yet say all done (after
// k_fin_conv, which then acted); 2: only once it does (after a k_fin_start
// queued with when_done). force (may be NULL): cleared here, after every
// workgroup of the k_fin_start before has read it.
__global__ __launch_bounds__(kFin) void k_fin_summary(const PcgScalars* __restrict__ s, int32_t n_inst,
                                                       PcgSummary* __restrict__ sum,
                                                       PcgSummary* __restrict__ host_sum,
                                                       PcgScalars* __restrict__ host, int32_t gate,
                                                       int32_t* __restrict__ force) {
    const int32_t all_done = sum->all_done;
    if ((gate == 1 && all_done) || (gate == 2 && !all_done)) return;
    __syncthreads();  // every thread has read the old summary before summarise() writes the new one
    if (force && threadIdx.x == 0) *force = 0;
    summarise(s, n_inst, sum, host_sum, host);
}

__global__ void k_set_flag(int32_t* __restrict__ p, int32_t v) { *p = v; }

static double* part(eqs_ctx* c, int q) { return c->d_partials + (int64_t)q * 2 * c->max_blocks; }

// Workgroups of a finaliser: one per kFinWaves instances (one with a single instance).
static unsigned fin_grid(const eqs_ctx* c) { return (unsigned)((c->n_inst + kFinWaves - 1) / kFinWaves); }

void pcg_init(hipStream_t s, eqs_ctx* c, const double* rhs, const double* x, int32_t maxit, double rtol,
              int flexible, const double* mx) {
    const int64_t nb = sell_grid(c->M);
    if (mx)
        hipLaunchKernelGGL(k_pcg_residual_mx, dim3(grid_for(c->n_free)), dim3(kBlock), 0, s, inst_map(c), rhs, mx,
                           c->d_r, c->n_free, part(c, 0), part(c, 1));
    else
        hipLaunchKernelGGL(k_pcg_residual, dim3(nb), dim3(kBlock), 0, s, view(c->M), inst_map(c), rhs, x, c->d_r,
                           part(c, 0), part(c, 1), (double*)nullptr, (const int32_t*)nullptr);
    hipLaunchKernelGGL(inst_map(c).rows1 >= 0 ? k_fin_start<true> : k_fin_start<false>, dim3(fin_grid(c)),
                       dim3(kFin), 0, s, c->d_scal, inst_map(c), part(c, 0), part(c, 1), rtol, maxit, flexible, 0,
                       c->d_sum, c->d_hsum, c->d_hscal, 0, (int32_t*)nullptr);
    if (fin_grid(c) > 1)
        hipLaunchKernelGGL(k_fin_summary, dim3(1), dim3(kFin), 0, s, c->d_scal, (int32_t)c->n_inst, c->d_sum, c->d_hsum,
                           c->d_hscal, 0, (int32_t*)nullptr);
    if (c->test_reject_first) hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, s, c->d_force, 1);
}

void pcg_true_residual(hipStream_t s, eqs_ctx* c, const double* rhs, const double* x, double* mx_out,
                       bool only_if_done) {
    const int64_t nb = sell_grid(c->M);
    const int32_t* done = only_if_done ? &c->d_sum->all_done : nullptr;
    hipLaunchKernelGGL(k_pcg_residual, dim3(nb), dim3(kBlock), 0, s, view(c->M), inst_map(c), rhs, x, c->d_r,
                       part(c, 0), part(c, 1), mx_out, done);
    int32_t* force = c->test_reject_first ? c->d_force : (int32_t*)nullptr;
    hipLaunchKernelGGL(inst_map(c).rows1 >= 0 ? k_fin_start<true> : k_fin_start<false>, dim3(fin_grid(c)),
                       dim3(kFin), 0, s, c->d_scal, inst_map(c), part(c, 0), part(c, 1), 0.0, 0, 0, 1, c->d_sum,
                       c->d_hsum, c->d_hscal, only_if_done ? 1 : 0, force);
    if (fin_grid(c) > 1)
        hipLaunchKernelGGL(k_fin_summary, dim3(1), dim3(kFin), 0, s, c->d_scal, (int32_t)c->n_inst, c->d_sum, c->d_hsum,
                           c->d_hscal, only_if_done ? 2 : 0, force);
}

void pcg_zero_rhs_rows(hipStream_t s, eqs_ctx* c, double* x) {
    hipLaunchKernelGGL(k_zero_rhs_rows, dim3(grid_for(c->n_free)), dim3(kBlock), 0, s, inst_map(c), x, c->n_free,
                       c->d_scal);
}

void pcg_iteration(hipStream_t s, eqs_ctx* c, const double* rhs, double* x, int precision) {
    (void)rhs;
    const int64_t nbM = sell_grid(c->M);
    const int64_t nbV = grid_for(c->n_free);
    const int32_t* stop = &c->d_sum->all_done;
    // With one iteration per graph the CG SpMV and update do not test the flag either (the V-cycle never does;
    // see vcycle): an iteration past convergence is rarely launched (the host waits once the residuals
    // extrapolate to rtol), and it writes only partials and p and q, guarded for x and r by the instance's done
    // flag. With several iterations per graph they test it, so that surplus iterations skip their SpMV and update.
    const int32_t* vstop = c->graph_iters > 1 ? stop : nullptr;
    // z = B r, with pair partials of r.z (part 0) and r.z_old (part 1)
    prof_begin(c, EQS_KCLASS_VCYCLE, s);
    if (precision == EQS_PREC_FP32) vcycle<float>(s, c, c->h32, c->d_r, c->d_z, part(c, 0), part(c, 1));
    else vcycle<double>(s, c, c->h64, c->d_r, c->d_z, part(c, 0), part(c, 1));
    prof_end(c, EQS_KCLASS_VCYCLE, s);
    const InstMap im = inst_map(c);
    const bool one = im.rows1 >= 0;
    const dim3 fg(fin_grid(c));
    EQS_LAUNCH_TIMED(c, EQS_KCLASS_FINALISE, one ? k_fin_beta<true> : k_fin_beta<false>, fg, dim3(kFin), 0, s,
                     c->d_scal, im, part(c, 0), part(c, 1), stop);
    EQS_LAUNCH_TIMED(c, EQS_KCLASS_SPMV_M, one ? k_pcg_spmv<true> : k_pcg_spmv<false>, dim3(nbM), dim3(kBlock), 0,
                     s, view(c->M), im, c->d_z, c->d_p, c->d_q, part(c, 2), c->d_scal, vstop);
    EQS_LAUNCH_TIMED(c, EQS_KCLASS_FINALISE, one ? k_fin_alpha<true> : k_fin_alpha<false>, fg, dim3(kFin), 0, s,
                     c->d_scal, im, part(c, 2), stop);
    EQS_LAUNCH_TIMED(c, EQS_KCLASS_CG_UPDATE, one ? k_pcg_update<true> : k_pcg_update<false>, dim3(nbV),
                     dim3(kBlock), 0, s, im, x, c->d_r, c->d_p, c->d_q, c->n_free, part(c, 3), c->d_scal, vstop,
                     c->M.xcd);
    EQS_LAUNCH_TIMED(c, EQS_KCLASS_FINALISE, one ? k_fin_conv<true> : k_fin_conv<false>, fg, dim3(kFin), 0, s,
                     c->d_scal, im, part(c, 3), c->d_sum, c->d_hsum, c->d_hscal);
    if (fg.x > 1)  // the summary of all instances (part of the finalise class's work, not timed on its own)
        hipLaunchKernelGGL(k_fin_summary, dim3(1), dim3(kFin), 0, s, c->d_scal, (int32_t)c->n_inst, c->d_sum,
                           c->d_hsum, c->d_hscal, 1, (int32_t*)nullptr);
}

// ------------------------------------------------------------------ RKC
// With `zero` (may be NULL) the combination also clears that vector (the next
// stage's element-pass output), saving a launch.
__global__ void k_rkc_first(double* __restrict__ out, const double* __restrict__ Y0, const double* __restrict__ F0,
                            double a, int64_t n, double* __restrict__ zero) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        out[i] = Y0[i] + a * F0[i];
        if (zero) zero[i] = 0.0;
    }
}

// out may alias Yjm2 (each element is read before it is written).
__global__ void k_rkc_combine(double* out, const double* __restrict__ Y0, const double* __restrict__ Yjm1,
                              const double* Yjm2, const double* __restrict__ Fjm1, const double* __restrict__ F0,
                              double c0, double c1, double c2, double c3, double c4, int64_t n,
                              double* __restrict__ zero) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        out[i] = c0 * Y0[i] + c1 * Yjm1[i] + c2 * Yjm2[i] + c3 * Fjm1[i] + c4 * F0[i];
        if (zero) zero[i] = 0.0;
    }
}

void launch_rkc_first(eqs_ctx* c, hipStream_t s, double* out, const double* Y0, const double* F0, double a,
                      int64_t n, double* zero) {
    EQS_LAUNCH_TIMED(c, EQS_KCLASS_RKC_COMBINE, k_rkc_first, dim3(grid_for(n)), dim3(kBlock), 0, s, out, Y0, F0, a,
                     n, zero);
}

void launch_rkc_combine(eqs_ctx* c, hipStream_t s, double* out, const double* Y0, const double* Yjm1,
                        const double* Yjm2, const double* Fjm1, const double* F0, double c0, double c1, double c2,
                        double c3, double c4, int64_t n, double* zero) {
    EQS_LAUNCH_TIMED(c, EQS_KCLASS_RKC_COMBINE, k_rkc_combine, dim3(grid_for(n)), dim3(kBlock), 0, s, out, Y0, Yjm1,
                     Yjm2, Fjm1, F0, c0, c1, c2, c3, c4, n, zero);
}

}  // namespace eqs
