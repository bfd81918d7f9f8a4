// Start vectors for the stage solves (Sec. IV of the paper).
//
// The solutions F_j of successive stages solve M F_j = r_j with the same M, so
// a window S of the last W stage solutions spans good start vectors. Sec. IV
// builds them by a reduced solve on a basis of S (eq. (5): x0 = V (V^T M V)^{-1}
// V^T r). The reduced matrix needs no extra products because M s_k = r_k for
// every stored solution: H = S^T M S has entries r_a . s_b. The window stays in
// FP64: successive solutions differ by little, and the projection resolves
// exactly those differences (FP32 snapshots cost 1.5-2x the CG iterations).
//
// Per stage j (after the element pass wrote r_j) one fused pass reads the
// window S, u = F_{j-1}, v = r_j and w = r_{j-1}, returns S^T u, S^T v, u.u,
// u.v, u.w and stores F_{j-1} in its slot. The host then
//   * completes the training pair of stage j-1 (target V_{j-1}^T (F_{j-1} - F_{j-2})),
//   * updates G = S^T S and H with the new solution's row,
//   * forms the POD basis V = S B from G's eigenvectors (directions with
//     singular values below 1e-7 of the largest are dropped) and then
//     GALERKIN: solves eq. (5), (B^T H B) c = V^T r_j;
//     MLP: lets the network predict the change from F_{j-1} from the
//     directions of V^T F_{j-1} and V^T (r_j - r_{j-1}) (inference on the
//     GPU, which also keeps the change only if it lowers the M-norm of the
//     error, judged in the reduced space);
//   * x0 = S alpha in one pass, written over F_{j-1} (which stays in S).
// The network then takes one Adam step on a minibatch of stored pairs, on a
// stream of its own while the stage's solve runs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "eqs_internal.h"
#include "sell.h"

namespace eqs {

constexpr int kMaxWin = 16;
constexpr int kNDots = 2 * kMaxWin + 3;
constexpr int kDotGrid = 1024;
constexpr int kGuardLen = 16 * 16 + 16 + 1;
constexpr int kMaxPairsPerStage = 256;  // minibatches of up to 64 pairs, one Adam step each
constexpr int kNoAllocScratch = kNDots * kDotGrid + 64;  // doubles of the static scratch
static_assert(kNoAllocPartDoubles == (int64_t)kNDots * kDotGrid, "static scratch layout");

// ------------------------------------------------------------- kernels
template <int NQ>
__device__ __forceinline__ void block_sums_store(double (&v)[NQ], double* __restrict__ part, int64_t stride) {
    __shared__ double sh[NQ][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[q][wid] = x;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NQ; q += blockDim.x) part[q * stride + blockIdx.x] = ((sh[q][0] + sh[q][1]) + sh[q][2]) + sh[q][3];
}

// S^T u, S^T v for the first nslot slots, and u.u, u.v, u.w;
// slot `ins` (if >= 0) then receives u (each element is read before it is
// replaced, so the dots see the old window).
__global__ __launch_bounds__(256) void k_window_dots(double* __restrict__ S, int64_t ld, int nslot, int ins,
                                                      const double* __restrict__ u, const double* __restrict__ v,
                                                      const double* __restrict__ w, int64_t n,
                                                      double* __restrict__ part) {
    double acc[kNDots];
#pragma unroll
    for (int q = 0; q < kNDots; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ui = u[i], vi = v[i], wi = w[i];
        double sk[kMaxWin];
#pragma unroll
        for (int k = 0; k < kMaxWin; ++k) sk[k] = S[(int64_t)min(k, max(nslot - 1, 0)) * ld + i];
#pragma unroll
        for (int k = 0; k < kMaxWin; ++k) {
            const double d = k < nslot ? sk[k] : 0.0;
            acc[2 * k] += d * ui;
            acc[2 * k + 1] += d * vi;
        }
        acc[2 * kMaxWin] += ui * ui;
        acc[2 * kMaxWin + 1] += ui * vi;
        acc[2 * kMaxWin + 2] += ui * wi;
        if (ins >= 0) S[(int64_t)ins * ld + i] = ui;
    }
    block_sums_store<kNDots>(acc, part, kDotGrid);
}

// out[q] = sum of part[q][0..nb) in a fixed order (one block per value).
__global__ void k_sum_rows(const double* __restrict__ part, int64_t stride, int nb, double* __restrict__ out) {
    __shared__ double sh[4];
    double x = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) x += part[blockIdx.x * stride + i];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

struct Coef16 {
    double v[kMaxWin];
};

// x0 = sum_k alpha_k S_k, alpha from the device (ad) or passed by value
__global__ __launch_bounds__(256) void k_window_prolong(const double* __restrict__ S, int64_t ld, int nslot, Coef16 ah,
                                                         const double* __restrict__ ad, double* __restrict__ x0,
                                                         int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = 0; k < nslot; ++k) acc += (ad ? ad[k] : ah.v[k]) * S[k * ld + i];
    x0[i] = acc;
}

// ---------------------------------------------------------- host algebra
// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major):
// A = Q diag(lam) Q^T; columns of Q are the eigenvectors.
static void jacobi_eigen(int n, std::vector<double> A, std::vector<double>& lam, std::vector<double>& Q) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) (i == j ? diag : off) += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = cs * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = cs * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {  // Q <- Q J
                    const double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
                    Q[(size_t)k * n + p] = cs * qkp - sn * qkq;
                    Q[(size_t)k * n + q] = sn * qkp + cs * qkq;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = A[(size_t)i * n + i];
}

// Solve the small dense system K c = b (Gaussian elimination, partial pivoting).
static bool dense_solve(int n, std::vector<double> K, std::vector<double>& b) {
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(K[(size_t)r * n + c]) > std::fabs(K[(size_t)p * n + c])) p = r;
        if (!(std::fabs(K[(size_t)p * n + c]) > 0)) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(K[(size_t)p * n + k], K[(size_t)c * n + k]);
            std::swap(b[p], b[c]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = K[(size_t)r * n + c] / K[(size_t)c * n + c];
            for (int k = c; k < n; ++k) K[(size_t)r * n + k] -= f * K[(size_t)c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= K[(size_t)r * n + k] * b[k];
        b[r] = s / K[(size_t)r * n + r];
    }
    return true;
}


// SplitMix64 (Steele, Lea, Flood 2014): minibatch indices from a counter.
static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// ------------------------------------------------------------ guess state
void guess_release(eqs_ctx* c) {
    GuessState& g = c->guess;
    if (g.tstream) (void)hipStreamSynchronize(g.tstream);
    if (g.net) mlp_destroy(g.net);
    g.net = nullptr;
    if (g.ev_inf) (void)hipEventDestroy(g.ev_inf);
    if (g.ev_train) (void)hipEventDestroy(g.ev_train);
    if (g.tstream) (void)hipStreamDestroy(g.tstream);
    g.ev_inf = g.ev_train = nullptr;
    g.tstream = nullptr;
    g.inf_recorded = g.train_pending = false;
    if (g.h_stage) (void)hipHostFree(g.h_stage);
    g.h_stage = nullptr;
    if (g.h_guard) (void)hipHostFree(g.h_guard);
    g.h_guard = nullptr;
    g.dev_ready = false;
}

void guess_reset(eqs_ctx* c) {
    GuessState& g = c->guess;
    g.count = 0;
    g.oldest = 0;
    g.have_prev = false;
    g.have_pending = false;
    g.sol_scale = 0.0;
    g.last_iters = 0;
    g.frozen = false;
    g.mor_slot.clear();
    g.mor_B.clear();
    g.mor_K.clear();
    g.mor_m = 0;
    g.rcount = 0;
    g.rhead = 0;
    g.counter = 0;
    g.last_loss = 0.0;
    std::fill(g.G.begin(), g.G.end(), 0.0);
    std::fill(g.H.begin(), g.H.end(), 0.0);
}

void guess_configure(eqs_ctx* c, const eqs_guess_params& p) {
    GuessState& g = c->guess;
    guess_release(c);
    g.p = p;
    g.G.assign(kMaxWin * kMaxWin, 0.0);
    g.H.assign(kMaxWin * kMaxWin, 0.0);
    g.rdots.assign(kMaxWin, 0.0);
    g.rx.assign((size_t)p.capacity * 32, 0.0f);
    g.rt.assign((size_t)p.capacity * 16, 0.0f);
    guess_reset(c);
    if (p.kind == EQS_GUESS_MLP) {
        EQS_HIP(hipStreamCreateWithFlags(&g.tstream, hipStreamNonBlocking));  // default priority
        EQS_HIP(hipEventCreateWithFlags(&g.ev_inf, hipEventDisableTiming));
        EQS_HIP(hipEventCreateWithFlags(&g.ev_train, hipEventDisableTiming));
        g.net = mlp_create(c->device, g.tstream, g.init.data(), p.bf16, p.lr, c);
    }
    EQS_HIP(hipHostMalloc((void**)&g.h_stage, sizeof(float) * kMaxPairsPerStage * 48, hipHostMallocDefault));
    EQS_HIP(hipHostMalloc((void**)&g.h_guard, sizeof(double) * kGuardLen, hipHostMallocDefault));
}

void guess_alloc_device(eqs_ctx* c) {
    GuessState& g = c->guess;
    const int64_t NF = c->n_free;
    // buffers of an earlier configuration of this context (eqs_set_guess again)
    // go first, and the same sizes come back in the same order (so a workspace
    // reuses the same ranges); the training stream was drained when that one
    // was released. The dot scratch was allocated with the context and stays.
    for (void* p : {(void*)g.d_S, (void*)g.d_rprev, (void*)g.d_alpha, (void*)g.d_guard, (void*)g.d_gstat,
                    (void*)g.d_bx, (void*)g.d_bt})
        dev_free(c, p);
    guess_alloc_scratch(c);
    g.d_S = (double*)dev_alloc(c, sizeof(double) * (size_t)kMaxWin * NF);
    g.d_rprev = (double*)dev_alloc(c, sizeof(double) * NF);
    g.d_alpha = (double*)dev_alloc(c, sizeof(double) * kMaxWin);
    g.d_guard = (double*)dev_alloc(c, sizeof(double) * kGuardLen);
    g.d_gstat = (int32_t*)dev_alloc(c, sizeof(int32_t) * 2);
    EQS_HIP(hipMemset(g.d_gstat, 0, sizeof(int32_t) * 2));
    g.d_bx = (float*)dev_alloc(c, sizeof(float) * kMaxPairsPerStage * 32);
    g.d_bt = (float*)dev_alloc(c, sizeof(float) * kMaxPairsPerStage * 16);
    // the network's buffers are context memory too: a rebuild released them
    if (g.p.kind == EQS_GUESS_MLP && !g.net) g.net = mlp_create(c->device, g.tstream, g.init.data(), g.p.bf16, g.p.lr, c);
    g.dev_ready = true;
}

// Bytes (rounded as dev_alloc rounds) that guess_alloc_device and the explicit
// Galerkin call still have to allocate for the present settings.
static int64_t rounded(int64_t b) { return (b + 255) / 256 * 256; }
int64_t guess_pending_bytes(const eqs_ctx* c) {
    const GuessState& g = c->guess;
    const int64_t NF = c->n_free;
    const int64_t scratch = rounded(sizeof(double) * kNDots * kDotGrid) + rounded(sizeof(double) * 64);
    const int64_t have = (g.d_part ? rounded(sizeof(double) * kNDots * kDotGrid) : 0) +
                         (g.d_dots ? rounded(sizeof(double) * 64) : 0);
    if (g.p.kind >= EQS_GUESS_GALERKIN && !g.dev_ready) {
        const int64_t full = rounded(sizeof(double) * (int64_t)kMaxWin * NF) + rounded(sizeof(double) * NF) +
                             rounded(sizeof(double) * kMaxWin) + scratch + rounded(sizeof(double) * kGuardLen) +
                             rounded(sizeof(int32_t) * 2) + rounded(sizeof(float) * kMaxPairsPerStage * 32) +
                             rounded(sizeof(float) * kMaxPairsPerStage * 16);
        const int64_t net = (g.p.kind == EQS_GUESS_MLP && !g.net) ? mlp_device_bytes() : 0;
        return full - have + net;
    }
    return scratch - have;  // the dot scratch is allocated at upload, so normally 0
}

// The dot scratch of eqs_galerkin_start, allocated with the context's other buffers.
void guess_alloc_scratch(eqs_ctx* c) {
    GuessState& g = c->guess;
    if (!g.d_part) g.d_part = (double*)dev_alloc(c, sizeof(double) * kNDots * kDotGrid);
    if (!g.d_dots) g.d_dots = (double*)dev_alloc(c, sizeof(double) * 64);
}

// Basis from the Gram matrix of the current window (slots in age order).
struct Basis {
    int m = 0;                 // kept directions
    std::vector<int> slot;     // window slots (age order, newest first)
    std::vector<double> B;     // [count x m]: V = S_slots B  (B = Q diag(1/sigma))
    std::vector<double> sigma; // kept singular values
};

static Basis window_basis(const GuessState& g) {
    Basis b;
    const int n = g.count;
    const int W = g.p.window;
    for (int k = 0; k < n; ++k) b.slot.push_back((g.oldest + n - 1 - k + W) % W);  // newest first
    std::vector<double> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = g.G[b.slot[i] * kMaxWin + b.slot[j]];
    std::vector<double> lam, Q;
    jacobi_eigen(n, A, lam, Q);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return lam[x] > lam[y]; });
    const double smax = std::sqrt(std::max(lam[order[0]], 0.0));
    for (int k = 0; k < n; ++k) {
        const double sg = std::sqrt(std::max(lam[order[k]], 0.0));
        if (!(sg > 1e-7 * smax)) break;
        b.sigma.push_back(sg);
    }
    b.m = (int)b.sigma.size();
    b.B.assign((size_t)n * b.m, 0.0);
    for (int k = 0; k < b.m; ++k) {
        // sign: the newest snapshot (row 0) has a nonnegative coordinate
        const double sgn = Q[(size_t)0 * n + order[k]] < 0 ? -1.0 : 1.0;
        for (int i = 0; i < n; ++i) b.B[(size_t)i * b.m + k] = sgn * Q[(size_t)i * n + order[k]] / b.sigma[k];
    }
    return b;
}

// V^T y for y given by its dots with the window slots (d[slot]).
static std::vector<double> project(const Basis& b, const double* dslot) {
    std::vector<double> out(b.m, 0.0);
    for (int k = 0; k < b.m; ++k)
        for (int i = 0; i < (int)b.slot.size(); ++i) out[k] += b.B[(size_t)i * b.m + k] * dslot[b.slot[i]];
    return out;
}

// V^T M V = B^T H B for V = S B (m x m, symmetrised).
static std::vector<double> reduced_matrix(const GuessState& g, const Basis& B) {
    const int n = (int)B.slot.size(), m = B.m;
    std::vector<double> HB((size_t)n * m, 0.0), K((size_t)m * m, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const double h = g.H[B.slot[i] * kMaxWin + B.slot[k]];
            for (int q = 0; q < m; ++q) HB[(size_t)i * m + q] += h * B.B[(size_t)k * m + q];
        }
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < m; ++p) {
            const double bip = B.B[(size_t)i * m + p];
            for (int q = 0; q < m; ++q) K[(size_t)p * m + q] += bip * HB[(size_t)i * m + q];
        }
    for (int p = 0; p < m; ++p)
        for (int q = p + 1; q < m; ++q)
            K[(size_t)p * m + q] = K[(size_t)q * m + p] = 0.5 * (K[(size_t)p * m + q] + K[(size_t)q * m + p]);
    return K;
}

static double norm(const std::vector<double>& v) {
    double s = 0.0;
    for (double x : v) s += x * x;
    return std::sqrt(s);
}

// Eq. (5) on the basis V = S B: solve (V^T M V) c = V^T r with V^T M V = K and
// V^T r from r's dots with the window slots (rslot), then alpha = B c on the
// slots. False (coef untouched) if no direction is kept or K is singular.
static bool galerkin_coef(const Basis& B, const std::vector<double>& K, const double* rslot, Coef16& coef) {
    const int n = (int)B.slot.size(), m = B.m;
    std::vector<double> cvec = project(B, rslot);
    if (m == 0 || !dense_solve(m, K, cvec)) return false;
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int k = 0; k < m; ++k) acc += B.B[(size_t)i * m + k] * cvec[k];
        coef.v[B.slot[i]] = acc;
    }
    return true;
}

// ------------------------------------------- scratch that needs no allocation
// The dot-product partials of eqs_galerkin_start_noalloc live in this array,
// one copy per GPU for the life of the process: kNDots x kDotGrid block
// partials, then 64 summed dots (287,232 bytes). Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kNoAllocScratch];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // per device, from hipGetSymbolAddress
}  // namespace

void noalloc_scratch_init(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (g_scratch_ptr[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the device is current (eqs_create)
    if (e != hipSuccess) fail(EQS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = (double*)p;
}

double* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= (int)g_scratch_ptr.size() || !g_scratch_ptr[device])
        fail(EQS_ERR_STATE, "the static scratch of this device was not set up");
    return g_scratch_ptr[device];
}

// Eq. (5) on a window given by the caller (k columns of S, oldest first, with
// R = M S): G = S^T S and H = S^T R from k passes of the window-dots kernel,
// S^T r from one more, then the basis, reduced matrix and coefficient solve of
// a stage's GALERKIN start vector and x0 = S alpha. Returns the number of
// directions kept (0: x0 = 0). The dot partials go to `part` (kNDots x
// kDotGrid doubles) and `dots` (64 doubles), or, when part is NULL, to the
// context's start-vector scratch (allocated on first use). Runs on c->stream.
int guess_galerkin_explicit(eqs_ctx* c, int k, const double* S, const double* R, const double* r, double* x0,
                            double* part, double* dots_dev) {
    GuessState& gs = c->guess;
    if (!part) {
        // only the dot-product scratch is needed here (not the stage window)
        guess_alloc_scratch(c);
        part = gs.d_part;
        dots_dev = gs.d_dots;
    }
    hipStream_t s = c->stream;
    const int64_t NF = c->n_free;
    GuessState g;  // window bookkeeping only: slots 0..k-1, slot 0 the oldest
    g.p.window = k;
    g.count = k;
    g.oldest = 0;
    g.G.assign(kMaxWin * kMaxWin, 0.0);
    g.H.assign(kMaxWin * kMaxWin, 0.0);
    std::vector<double> rs(kMaxWin, 0.0);
    const unsigned grid = (unsigned)std::min<int64_t>(kDotGrid, (NF + kBlock - 1) / kBlock);
    double dots[kNDots];
    for (int a = 0; a <= k; ++a) {
        // u = s_a, v = r_a (column a of G and H); the last pass u = v = r
        const double* u = a < k ? S + (int64_t)a * NF : r;
        const double* v = a < k ? R + (int64_t)a * NF : r;
        hipLaunchKernelGGL(k_window_dots, dim3(grid), dim3(kBlock), 0, s, const_cast<double*>(S), NF, k, -1, u, v, v,
                           NF, part);
        hipLaunchKernelGGL(k_sum_rows, dim3(kNDots), dim3(kBlock), 0, s, part, (int64_t)kDotGrid, (int)grid,
                           dots_dev);
        EQS_HIP(hipMemcpyAsync(dots, dots_dev, sizeof dots, hipMemcpyDeviceToHost, s));
        EQS_HIP(hipStreamSynchronize(s));
        for (int b = 0; b < k; ++b) {
            if (a < k) {
                g.G[b * kMaxWin + a] = dots[2 * b];      // s_b . s_a
                g.H[b * kMaxWin + a] = dots[2 * b + 1];  // s_b . M s_a
            } else {
                rs[b] = dots[2 * b];  // s_b . r
            }
        }
    }
    for (int a = 0; a < k; ++a)  // both are symmetric; each pair was summed twice
        for (int b = a + 1; b < k; ++b) {
            const double gv = 0.5 * (g.G[a * kMaxWin + b] + g.G[b * kMaxWin + a]);
            const double hv = 0.5 * (g.H[a * kMaxWin + b] + g.H[b * kMaxWin + a]);
            g.G[a * kMaxWin + b] = g.G[b * kMaxWin + a] = gv;
            g.H[a * kMaxWin + b] = g.H[b * kMaxWin + a] = hv;
        }
    const Basis B = window_basis(g);
    const std::vector<double> K = reduced_matrix(g, B);
    Coef16 coef{};
    const bool ok = galerkin_coef(B, K, rs.data(), coef);
    if (!ok) {  // no direction kept or a singular reduced matrix: x0 = 0 (not 0 * S, which keeps NaN)
        launch_fill(s, x0, 0.0, NF);
        EQS_HIP(hipGetLastError());
        return 0;
    }
    const unsigned pg = (unsigned)((NF + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_window_prolong, dim3(pg), dim3(kBlock), 0, s, S, NF, k, coef, nullptr, x0, NF);
    EQS_HIP(hipGetLastError());
    return B.m;
}

// One stage's start vector. Called after the element pass wrote r_j into
// c->d_rhs and before the solve; d_F holds F_{j-1} (if have_prev). On return
// d_F holds the chosen start vector. Returns 1 if the estimator's vector was
// used, 2 if the network's vector went to the device guard (its decision is
// counted there, see guess_device_stats), 0 if no estimate was available.
int guess_stage(eqs_ctx* c) {
    GuessState& g = c->guess;
    hipStream_t s = c->stream;
    const int64_t NF = c->n_free;
    if (!g.dev_ready) guess_alloc_device(c);
    int used = 0;
    if (!g.have_prev) return 0;  // nothing known yet: d_F (zero or last run's) stays

    // the slot F_{j-1} will take (the oldest one once the window is full). The
    // network always adds it; GALERKIN and MOR only if its solve took more than
    // add_threshold iterations (the first one always); a frozen MOR window
    // takes no more.
    const int W = g.p.window;  // physical slots 0..W-1 fill in order, then rotate
    const int n_old = g.count;
    const int e = (g.count < W) ? (g.oldest + g.count) % W : g.oldest;
    const bool insert = !g.frozen && (g.p.kind == EQS_GUESS_MLP || g.count == 0 || g.p.add_threshold == 0 ||
                                      g.last_iters > g.p.add_threshold);
    // fused pass over the window with u = F_{j-1}, v = r_j, w = r_{j-1}; it
    // also stores F_{j-1} in slot e
    const unsigned grid = (unsigned)std::min<int64_t>(kDotGrid, (NF + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_window_dots, dim3(grid), dim3(kBlock), 0, s, g.d_S, NF, n_old, insert ? e : -1, c->d_F,
                       c->d_rhs, g.d_rprev, NF, g.d_part);
    hipLaunchKernelGGL(k_sum_rows, dim3(kNDots), dim3(kBlock), 0, s, g.d_part, (int64_t)kDotGrid, (int)grid,
                       g.d_dots);
    double dots[kNDots];
    EQS_HIP(hipMemcpyAsync(dots, g.d_dots, sizeof dots, hipMemcpyDeviceToHost, s));
    EQS_HIP(hipStreamSynchronize(s));
    double Su[kMaxWin], Sv[kMaxWin];
    for (int k = 0; k < kMaxWin; ++k) {
        Su[k] = k < n_old ? dots[2 * k] : 0.0;
        Sv[k] = k < n_old ? dots[2 * k + 1] : 0.0;
    }
    const double uu = dots[2 * kMaxWin], uv = dots[2 * kMaxWin + 1], uw = dots[2 * kMaxWin + 2];

    // (1) training pair of the previous stage: target V_{j-1}^T (F_{j-1} - F_{j-2})
    if (g.have_pending && g.p.kind == EQS_GUESS_MLP) {
        std::vector<double> tcoef(16, 0.0);
        for (int k = 0; k < g.pend_m; ++k) {
            double a = 0.0;
            for (int i = 0; i < (int)g.pend_slot.size(); ++i) a += g.pend_B[(size_t)i * g.pend_m + k] * Su[g.pend_slot[i]];
            tcoef[k] = (a - g.pend_a[k]) / g.pend_scale;
        }
        const int slot = g.rhead;
        for (int q = 0; q < 32; ++q) g.rx[(size_t)slot * 32 + q] = g.pend_x[q];
        for (int q = 0; q < 16; ++q) g.rt[(size_t)slot * 16 + q] = (float)tcoef[q];
        g.rhead = (g.rhead + 1) % g.p.capacity;
        g.rcount = std::min(g.rcount + 1, g.p.capacity);
    }
    g.have_pending = false;

    // (2) F_{j-1} has joined the window in slot e (evicting the oldest when full)
    double rprev[kMaxWin];  // r_{j-1} against the window (for the change of the RHS)
    if (insert) {
        if (g.count < W) g.count++;
        else g.oldest = (g.oldest + 1) % W;
        // slots 0..n_old-1 are the physical slots in use before the insertion
        for (int b = 0; b < n_old; ++b) {
            if (b == e) continue;
            g.G[e * kMaxWin + b] = g.G[b * kMaxWin + e] = Su[b];
            g.H[e * kMaxWin + b] = g.H[b * kMaxWin + e] = g.rdots[b];  // r_{j-1} . s_b = s_b^T M F_{j-1}
        }
        g.G[e * kMaxWin + e] = uu;
        g.H[e * kMaxWin + e] = uw;
        for (int b = 0; b < kMaxWin; ++b) rprev[b] = (b == e) ? uw : g.rdots[b];
        // r_j against the new window, kept for the next insertion
        for (int b = 0; b < kMaxWin; ++b) g.rdots[b] = (b == e) ? uv : (b < n_old ? Sv[b] : 0.0);
        if (g.p.kind == EQS_GUESS_MOR && g.count == W) g.frozen = true;
    } else {
        for (int b = 0; b < kMaxWin; ++b) {
            rprev[b] = g.rdots[b];
            g.rdots[b] = b < n_old ? Sv[b] : 0.0;
        }
    }

    if (g.count < 2) return 0;

    // (3) coefficients of the start vector on the window
    bool have = false;
    Coef16 coef{};
    if (g.p.kind == EQS_GUESS_GALERKIN || g.p.kind == EQS_GUESS_MOR) {
        // eq. (5) on the POD basis V = S B of the window: (V^T M V) c = V^T r_j,
        // V^T M V = B^T H B (H = S^T M S has entries r_a . s_b), alpha = B c.
        // A frozen MOR window keeps its basis and reduced matrix.
        Basis B;
        std::vector<double> K;
        if (g.frozen && !g.mor_slot.empty()) {
            B.slot = g.mor_slot;
            B.B = g.mor_B;
            B.m = g.mor_m;
            K = g.mor_K;
        } else {
            B = window_basis(g);
            K = reduced_matrix(g, B);
            if (g.frozen) {
                g.mor_slot = B.slot;
                g.mor_B = B.B;
                g.mor_m = B.m;
                g.mor_K = K;
            }
        }
        have = galerkin_coef(B, K, g.rdots.data(), coef);  // r_j's dots with the slots give V^T r_j
    } else if (g.p.kind == EQS_GUESS_MLP) {
        const Basis B = window_basis(g);
        const std::vector<double> a = project(B, &g.G[e * kMaxWin]);  // V^T F_{j-1}
        const std::vector<double> bh = project(B, g.rdots.data());     // V^T r_j
        // The network predicts the change of the solution from F_{j-1} within
        // span(V), c ~ V^T (F_j - F_{j-1}), from the direction of the state
        // (V^T F_{j-1}) and of the change of the RHS (V^T (r_j - r_{j-1})).
        // Inputs are unit vectors; the output is scaled by sigma |V^T dr|,
        // sigma = |V^T F| / |V^T r| fixed at the first pair, so that targets
        // are O(1); the start vector is x0 = F_{j-1} + V c.
        const std::vector<double> bp = project(B, rprev);  // V^T r_{j-1}
        std::vector<double> d(B.m);
        for (int k = 0; k < B.m; ++k) d[k] = bh[k] - bp[k];
        const double sa = norm(a), sd = norm(d);
        if (g.sol_scale == 0.0 && sa > 0 && norm(bp) > 0) g.sol_scale = sa / norm(bp);
        const double scale = g.sol_scale * sd;
        if (sa > 0 && scale > 0 && std::isfinite(scale)) {
            float x[32];
            for (int k = 0; k < 16; ++k) {
                x[k] = k < B.m ? (float)(a[k] / sa) : 0.0f;
                x[16 + k] = k < B.m ? (float)(d[k] / sd) : 0.0f;
            }
            std::memcpy(g.pend_x, x, sizeof x);
            g.pend_scale = scale;
            for (int k = 0; k < 16; ++k) g.pend_a[k] = k < B.m ? a[k] : 0.0;
            g.pend_slot = B.slot;
            g.pend_B = B.B;
            g.pend_m = B.m;
            g.have_pending = true;
            if (g.rcount >= g.p.warmup) {
                // alpha_slot = [slot == e] + sum_k B[i][k] * scale * y_k; slots past count stay 0
                double P[16 * 16], bias[16];
                std::fill(P, P + 256, 0.0);
                std::fill(bias, bias + 16, 0.0);
                bias[e] = 1.0;
                for (int i = 0; i < (int)B.slot.size(); ++i)
                    for (int k = 0; k < B.m; ++k) P[B.slot[i] * 16 + k] = B.B[(size_t)i * B.m + k] * scale;
                const double* guard = nullptr;
                if (g.p.guard) {
                    // the device keeps the correction only if it lowers the M-norm of the error
                    const std::vector<double> K = reduced_matrix(g, B);
                    std::fill(g.h_guard, g.h_guard + kGuardLen, 0.0);
                    for (int p = 0; p < B.m; ++p) {
                        for (int q = 0; q < B.m; ++q) g.h_guard[p * 16 + q] = K[(size_t)p * B.m + q];
                        g.h_guard[256 + p] = d[p];
                    }
                    g.h_guard[272] = scale;
                    EQS_HIP(hipMemcpyAsync(g.d_guard, g.h_guard, sizeof(double) * kGuardLen, hipMemcpyHostToDevice, s));
                    guard = g.d_guard;
                }
                if (g.train_pending) EQS_HIP(hipStreamWaitEvent(s, g.ev_train, 0));
                mlp_forward_coeffs(g.net, s, x, P, bias, g.d_alpha, guard, g.d_gstat);
                EQS_HIP(hipEventRecord(g.ev_inf, s));
                g.inf_recorded = true;
                have = true;
            }
        }
    }

    if (have) {
        // x0 = S alpha goes straight into d_F; F_{j-1} stays in slot e
        const bool mlp = g.p.kind == EQS_GUESS_MLP;
        hipLaunchKernelGGL(k_window_prolong, dim3((unsigned)((NF + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g.d_S,
                           NF, g.count, coef, mlp ? (const double*)g.d_alpha : nullptr, c->d_F, NF);
        // The Galerkin vector minimises the M-norm of the error over the span
        // of the window, which holds F_{j-1}: it cannot be worse than F_{j-1}
        // in the norm CG reduces. The network's correction is checked on the
        // device in the same norm (k_mlp_alpha), its decision counted there.
        used = mlp ? 2 : 1;
    }
    return used;
}

// After the solve of stage j: remember r_j (the next pass needs it) and mark
// F_j pending.
void guess_after_solve(eqs_ctx* c, int32_t iters) {
    GuessState& g = c->guess;
    std::swap(c->d_rhs, g.d_rprev);  // r_j is kept; the next element pass writes the other buffer
    g.have_prev = true;
    g.last_iters = iters;
}

// Adam steps of the network on `batch` stored pairs (minibatches of up to 64,
// one step each), enqueued on the training stream after this stage's
// inference has read the weights, so that they run while the stage's solve
// runs; the next inference waits for them.
void guess_train(eqs_ctx* c) {
    GuessState& g = c->guess;
    if (g.p.kind != EQS_GUESS_MLP || g.rcount == 0) return;
    const int total = std::min(g.p.batch, kMaxPairsPerStage);
    if (g.train_pending) EQS_HIP(hipEventSynchronize(g.ev_train));  // the staging buffer is free again
    float* hx = g.h_stage;
    float* ht = g.h_stage + kMaxPairsPerStage * 32;
    for (int b = 0; b < total; ++b) {
        const int idx = (int)(splitmix64(g.p.seed + g.counter++) % (uint64_t)g.rcount);
        std::memcpy(hx + b * 32, &g.rx[(size_t)idx * 32], 32 * sizeof(float));
        std::memcpy(ht + b * 16, &g.rt[(size_t)idx * 16], 16 * sizeof(float));
    }
    if (g.inf_recorded) EQS_HIP(hipStreamWaitEvent(g.tstream, g.ev_inf, 0));  // weights read by this stage
    EQS_HIP(hipMemcpyAsync(g.d_bx, hx, sizeof(float) * total * 32, hipMemcpyHostToDevice, g.tstream));
    EQS_HIP(hipMemcpyAsync(g.d_bt, ht, sizeof(float) * total * 16, hipMemcpyHostToDevice, g.tstream));
    for (int b0 = 0; b0 < total; b0 += 64)
        mlp_train(g.net, g.d_bx + (size_t)b0 * 32, g.d_bt + (size_t)b0 * 16, std::min(64, total - b0));
    EQS_HIP(hipEventRecord(g.ev_train, g.tstream));
    g.train_pending = true;
    g.trained = true;
}

// Checkpoint of the start-vector state (called between steps, both streams
// idle): the window's host matrices and bookkeeping, the slots in use, r_{j-1},
// the pending training pair, the replay buffer and its sampling counter, and
// the network. Loading needs the same eqs_set_guess settings.
void guess_save_state(eqs_ctx* c, StateWriter& w) {
    GuessState& g = c->guess;
    const int64_t NF = c->n_free;
    if (g.tstream) EQS_HIP(hipStreamSynchronize(g.tstream));
    w.val((int32_t)g.dev_ready);
    if (!g.dev_ready) return;
    for (int32_t v : {g.count, g.oldest, (int32_t)g.have_prev, g.last_iters, (int32_t)g.frozen, g.mor_m,
                      (int32_t)g.have_pending, g.pend_m, g.rcount, g.rhead, (int32_t)g.trained})
        w.val(v);
    w.val(g.counter);
    w.val(g.pend_scale);
    w.val(g.sol_scale);
    w.val(g.last_loss);
    w.raw(g.pend_x, sizeof g.pend_x);
    w.raw(g.pend_a, sizeof g.pend_a);
    w.vec(g.G);
    w.vec(g.H);
    w.vec(g.rdots);
    w.vec(g.mor_slot);
    w.vec(g.mor_B);
    w.vec(g.mor_K);
    w.vec(g.pend_slot);
    w.vec(g.pend_B);
    w.vec(g.rx);
    w.vec(g.rt);
    const int used = std::min(g.count, g.p.window);  // physical slots 0..used-1
    w.dev(g.d_S, (int64_t)sizeof(double) * used * NF);
    w.dev(g.d_rprev, g.have_prev ? (int64_t)sizeof(double) * NF : 0);
    const int32_t has_net = g.net ? 1 : 0;
    w.val(has_net);
    if (g.net) {
        std::vector<char> tmp((size_t)mlp_state_bytes());
        if (w.buf) mlp_save_state(g.net, tmp.data());
        w.raw(tmp.data(), (int64_t)tmp.size());
    }
}

void guess_load_state(eqs_ctx* c, StateReader& r) {
    GuessState& g = c->guess;
    const int64_t NF = c->n_free;
    if (g.tstream) EQS_HIP(hipStreamSynchronize(g.tstream));
    if (!r.val<int32_t>()) return;  // saved before the first estimator stage
    if (!g.dev_ready) guess_alloc_device(c);
    g.count = r.val<int32_t>();
    g.oldest = r.val<int32_t>();
    g.have_prev = r.val<int32_t>() != 0;
    g.last_iters = r.val<int32_t>();
    g.frozen = r.val<int32_t>() != 0;
    g.mor_m = r.val<int32_t>();
    g.have_pending = r.val<int32_t>() != 0;
    g.pend_m = r.val<int32_t>();
    g.rcount = r.val<int32_t>();
    g.rhead = r.val<int32_t>();
    g.trained = r.val<int32_t>() != 0;
    g.counter = r.val<uint64_t>();
    g.pend_scale = r.val<double>();
    g.sol_scale = r.val<double>();
    g.last_loss = r.val<double>();
    r.raw(g.pend_x, sizeof g.pend_x);
    r.raw(g.pend_a, sizeof g.pend_a);
    r.vec(g.G, kMaxWin * kMaxWin);
    r.vec(g.H, kMaxWin * kMaxWin);
    r.vec(g.rdots, kMaxWin);
    r.vec(g.mor_slot, kMaxWin);
    r.vec(g.mor_B, kMaxWin * kMaxWin);
    r.vec(g.mor_K, kMaxWin * kMaxWin);
    r.vec(g.pend_slot, kMaxWin);
    r.vec(g.pend_B, kMaxWin * kMaxWin);
    r.vec(g.rx, (int64_t)g.p.capacity * 32);
    r.vec(g.rt, (int64_t)g.p.capacity * 16);
    if (g.count < 0 || g.count > g.p.window || g.oldest < 0 || g.oldest >= std::max(1, g.p.window) ||
        g.G.size() != (size_t)kMaxWin * kMaxWin || g.H.size() != (size_t)kMaxWin * kMaxWin ||
        g.rdots.size() != (size_t)kMaxWin || g.rx.size() != (size_t)g.p.capacity * 32 ||
        g.rt.size() != (size_t)g.p.capacity * 16 || g.rcount < 0 || g.rcount > g.p.capacity || g.rhead < 0 ||
        g.rhead >= std::max(1, g.p.capacity))
        fail(EQS_ERR_INVALID_ARG, "state buffer: start-vector state does not match the context's settings");
    const int used = std::min(g.count, g.p.window);
    r.dev(g.d_S, (int64_t)sizeof(double) * used * NF);
    r.dev(g.d_rprev, g.have_prev ? (int64_t)sizeof(double) * NF : 0);
    const int32_t has_net = r.val<int32_t>();
    if (has_net != (g.net ? 1 : 0)) fail(EQS_ERR_INVALID_ARG, "state buffer: network state does not match the settings");
    if (g.net) {
        std::vector<char> tmp((size_t)mlp_state_bytes());
        r.raw(tmp.data(), (int64_t)tmp.size());
        mlp_load_state(g.net, tmp.data());
    }
    g.inf_recorded = g.train_pending = false;
    EQS_HIP(hipMemset(g.d_gstat, 0, sizeof(int32_t) * 2));
}

// Network corrections kept / dropped by the device guard since the last call
// (the stream must be idle); the counters restart at zero.
void guess_device_stats(eqs_ctx* c, int32_t* kept, int32_t* dropped) {
    GuessState& g = c->guess;
    *kept = *dropped = 0;
    if (!g.dev_ready || !g.d_gstat) return;
    int32_t h[2];
    EQS_HIP(hipMemcpy(h, g.d_gstat, sizeof h, hipMemcpyDeviceToHost));
    EQS_HIP(hipMemset(g.d_gstat, 0, sizeof h));
    *kept = h[0];
    *dropped = h[1];
}

// Loss of the latest finished training step (a step still running on the
// training stream is not waited for: its predecessor's loss is reported).
double guess_last_loss(eqs_ctx* c) {
    GuessState& g = c->guess;
    if (!g.net || !g.trained) return 0.0;
    if (g.train_pending && hipEventQuery(g.ev_train) == hipErrorNotReady) return g.last_loss;
    g.last_loss = mlp_last_loss(g.net);
    return g.last_loss;
}

}  // namespace eqs
