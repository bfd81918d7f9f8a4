// Internal declarations of the EQS explicit-RKC library (gfx950).
//
// Layout in device memory (internal node order: the free nodes in increasing
// user id, then the Dirichlet nodes in increasing user id):
//   conn   int4   [n_tets]      internal node ids of each tet
//   tmat   uint16 [n_tets]      material id of each tet
//   xyz    double4[n_nodes]     x, y, z, 0 (one 32-byte record per node)
//   mats   MatDev [n_mat]       eps (absolute), kappa0, 1/e_s, alpha, flags
//   ddrive int32  [n_dir]       drive id of Dirichlet node n_free + k
//   M      SELL-64 FP64         M restricted to the free nodes
//   AMG    per level: SELL-64 A_l, P_l, R_l = P_l^T (FP64 or FP32), 1/diag,
//          work vectors; a dense inverse at the coarsest level
//
// SELL-64: rows are cut into slices of 64 consecutive rows (one wavefront);
// slice s stores width_s = max row length of its rows, column-major: entry k
// of row 64 s + l sits at sptr[s] + 64 k + l. Short rows are padded with a
// zero value and an in-range column.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <functional>
#include <map>
#include <vector>

#include "eqs.h"

namespace eqs {

constexpr int kSlice = 64;   // SELL slice height = wavefront size
constexpr int kTetBlock = 256;  // threads per element-pass workgroup
constexpr int kMaxTetsPerThread = 8;  // element blocks hold kTetBlock * tpt tets, tpt in {1, 2, 4, 8}
constexpr int kMaxBlockNodes = 1360;  // distinct nodes per element block: 48 B of LDS each (<= 64 KiB)
constexpr int64_t kMaxCoarseR = 4 << 20;  // entries of the fused restriction + coarse solve matrix
constexpr int kBlock = 256;  // threads per block for streaming kernels

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};
void set_error(const std::string& msg);
#define EQS_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::eqs::Error{EQS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)
[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error{code, msg}; }

// ----------------------------------------------------------- host matrices
template <typename T>
struct Csr {
    int32_t n_rows = 0, n_cols = 0;
    std::vector<int32_t> ptr, col;
    std::vector<T> val;
    int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

// --------------------------------------------------------- device matrices
template <typename T>
struct Sell {
    int32_t n_rows = 0, n_cols = 0, n_slices = 0;
    int32_t lanes = 1;          // lanes per row (a slice holds 64 / lanes rows)
    int32_t unroll = 8;         // entries per lane whose loads are in flight together (4, 8 or 16)
    int64_t stored = 0;         // padded entries
    int32_t* sptr = nullptr;    // [n_slices + 1]
    int32_t* col = nullptr;     // [stored] absolute column ids, or
    int16_t* d16 = nullptr;     // [stored] column - offset_base(row) when every entry allows
    T* val = nullptr;           // [stored]
    uint8_t* perm = nullptr;    // [n_slices * 64 / lanes] row order within 256-thread windows, or NULL
    int32_t xcd = 0;            // 1: products walk row blocks in the XCD order (row_block in sell.h)
};

// A hierarchy operator in one of two layouts, chosen per matrix by timing
// (or, without the autotuner, from its mean row length): SELL (1, 2, 4 or 8
// lanes per row, sell.lanes), or CSR with `lanes` lanes per row (a power of
// two <= 64) whose partial sums are combined by cross-lane shuffles, for the
// long rows of coarse AMG operators.
enum { FMT_SELL = 0, FMT_CSR = 1 };
// Column ids stored as 16-bit offsets are relative to this base: the row
// itself for a square operator, row * n_cols / n_rows for a rectangular one
// (transfer operators between AMG levels, whose columns follow the rows).
__host__ __device__ inline int32_t offset_base(int32_t row, int32_t n_rows, int32_t n_cols) {
    return n_rows == n_cols ? row : (int32_t)(((int64_t)row * n_cols) / n_rows);
}

template <typename T>
struct SpMat {
    int fmt = FMT_SELL;
    int lanes = 1;
    Sell<T> sell;
    int32_t n_rows = 0, n_cols = 0;
    int32_t* rowptr = nullptr;  // CSR
    int32_t* col = nullptr;     // absolute column ids, or
    int16_t* d16 = nullptr;     // offsets from offset_base(row) when every entry allows
    T* val = nullptr;
    int64_t nnz = 0;
};

struct MatDev {
    double eps;      // eps0 * eps_r
    double kappa0;
    double inv_es;   // 1 / e_s
    double alpha;
    int32_t nonlinear;
    int32_t ialpha;  // alpha as an integer in [0, 64] when exact, else -1
};

// Drive k: g_k(t) = amp sin(w t + phase), g_k'(t) = w amp cos(w t + phase),
// w = 2 pi freq; evaluated on the device at the stage time.
struct DriveDev {
    double w, amp, phase, pad;
};

// PCG scalars kept on the device so that the iteration needs no host values.
struct PcgScalars {
    double bb;       // |rhs|^2
    double rr;       // |r|^2
    double rho;      // r.z of the current iteration
    double rho_old;  // r.z of the previous iteration
    double beta;
    double alpha;
    double tol2;     // (rtol |rhs|)^2
    double relres;
    int32_t it;
    int32_t maxit;
    int32_t done;    // 1 once converged, out of iterations or broken down
    int32_t status;  // EQS_OK / EQS_ERR_NOT_CONVERGED / EQS_ERR_BREAKDOWN
    int32_t fresh;   // 1: next beta is 0 (first iteration or restart)
    int32_t flexible;
};

// Summary of all instances' CG states (written by the finalisers).
struct PcgSummary {
    int32_t all_done;
    int32_t n_active;
    int32_t n_breakdown;
    int32_t n_notconv;
    int32_t n_zero_rhs;
    int32_t max_it;
    double max_relres;
};

template <typename T>
struct Level {
    int32_t n = 0;
    SpMat<T> A, P, R;  // P, R unused on the coarsest level
    T* dinv = nullptr;
    T* sval = nullptr;  // values of A omega D^{-1} in A's storage order (pre-smoothing); not on the coarsest level
    double omega = 0;   // damped Jacobi weight
    T *b = nullptr, *x = nullptr, *xs = nullptr, *res = nullptr;
    T* dense_inv = nullptr;  // coarsest level only: n x n, column-major
    // coarsest level only, when small enough: the dense matrix that maps the
    // level above to the coarse solution in one product (n x coarse_R_cols,
    // row-major): A^{-1} R r of its residual, or, with `tail` set on the level
    // above, A^{-1} R (I - A w D^{-1}) b of its right-hand side
    T* coarse_R = nullptr;
    int32_t coarse_R_cols = 0;
    // level above the coarsest, when folded (`tail`): its V(1,1) visit is
    // xs = [G Q] [b; x_coarse] after the coarse product (b and the coarsest x
    // share one buffer)
    bool tail = false;
    SpMat<T> GQ;
    // pre-smoother folded into the restriction: R holds R (I - A w D^-1), so
    // the descent restricts b directly and the prolongation stores
    // x = w D^-1 b + P x_coarse (levels other than the finest and the tail)
    bool fold_pre = false;
};

template <typename T>
struct Hierarchy {
    std::vector<Level<T>> lv;
};

// Start-vector estimator state (guess.hip).
}  // namespace eqs
struct eqs_mlp;
namespace eqs {
struct GuessState {
    eqs_guess_params p{};
    std::vector<float> init;          // network initial parameters
    // window of stage solutions (device) and its Gram / energy matrices (host)
    double* d_S = nullptr;            // [16][n_free] window of stage solutions
    double* d_rprev = nullptr;        // r_{j-1}
    double* d_alpha = nullptr;        // [16]
    double* d_guard = nullptr;        // [16 x 16 + 16 + 1] reduced matrix, RHS change, scale (network guard)
    double* h_guard = nullptr;        // pinned staging of d_guard
    int32_t* d_gstat = nullptr;       // [2] network corrections kept / dropped on the device
    double* d_dots = nullptr;
    double* d_part = nullptr;
    float *d_bx = nullptr, *d_bt = nullptr;  // minibatch staging
    float* h_stage = nullptr;         // pinned
    bool dev_ready = false;
    int count = 0, oldest = 0;
    std::vector<double> G, H, rdots;  // 16 x 16, 16 x 16, 16
    bool have_prev = false;
    int32_t last_iters = 0;           // CG iterations of the latest stage solve
    bool frozen = false;              // MOR: the window is full and kept from now on
    std::vector<int> mor_slot;        // MOR: basis and reduced matrix of the frozen window
    std::vector<double> mor_B, mor_K;
    int mor_m = 0;
    // pending training pair of the current stage
    bool have_pending = false;
    float pend_x[32];
    double pend_scale = 1.0;
    double pend_a[16];                // V^T F_{j-1} of the pending pair (its target is the change)
    double sol_scale = 0.0;           // |V^T F| / |V^T r| of the first pair, then fixed
    std::vector<int> pend_slot;
    std::vector<double> pend_B;
    int pend_m = 0;
    // replay buffer (host) and network
    std::vector<float> rx, rt;
    int rcount = 0, rhead = 0;
    uint64_t counter = 0;
    eqs_mlp* net = nullptr;
    // the network trains on a stream of its own, overlapping the stage solve:
    // training of stage j waits for that stage's inference (ev_inf), the
    // inference of stage j+1 for that training (ev_train)
    hipStream_t tstream = nullptr;
    hipEvent_t ev_inf = nullptr, ev_train = nullptr;
    bool inf_recorded = false, train_pending = false;
    bool trained = false;
    double last_loss = 0.0;
};

// ------------------------------------------------------------------ context
}  // namespace eqs

struct eqs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;

    // inputs (host copies)
    int64_t n_nodes = 0, n_tets = 0;
    int npe = 4;  // nodes per tet: 4 (P1) or 10 (second order: vertices, then edge midpoints)
    std::vector<double> xyz;
    std::vector<int32_t> tets;  // n_tets x npe
    std::vector<eqs_material> mats;
    std::vector<int32_t> tet_mat;
    std::vector<int32_t> dir_nodes, dir_drive;
    std::vector<eqs_drive> drives;
    bool have_mesh = false, have_mat = false, have_dir = false, built = false;

    // derived ordering
    int64_t n_free = 0, n_dir = 0;
    std::vector<int32_t> int_to_user;  // [n_nodes]
    eqs_amg_params amg{};
    int64_t nnz_M = 0;

    // device: mesh + materials. Tets are processed in blocks of
    // kTetBlock * tet_tpt tets (Morton order of centroids); block b lists its
    // distinct nodes in d_bnodes[d_boff[b] .. d_boff[b+1]) and every tet packs
    // the 12-bit block-local ids of its vertices and its 16-bit material id in
    // 64 bits. Coordinates are stored per axis (d_cx, d_cy, d_cz).
    uint64_t* d_tpack = nullptr;
    int32_t* d_bnodes = nullptr;
    int32_t* d_boff = nullptr;
    int64_t n_blocks = 0;
    int32_t max_block_nodes = 0;
    int32_t tet_tpt = 0;        // tets per thread of the element pass
    // deterministic element pass (eqs_set_deterministic; see k_kx_det): per
    // block the slots of every node in slot order, the end of every block
    // node's list, every node's block-node positions in block order, and the
    // block partials
    bool deterministic = false;
    uint16_t* d_kslots = nullptr;
    uint16_t* d_kend = nullptr;
    int32_t* d_occ_off = nullptr;
    int32_t* d_occ = nullptr;
    double* d_kx_part = nullptr;
    int64_t n_block_nodes = 0;  // entries of d_bnodes (nodes shared by blocks count once per block)
    double* d_cx = nullptr;
    double* d_cy = nullptr;
    double* d_cz = nullptr;
    eqs::MatDev* d_mats = nullptr;
    int32_t* d_ddrive = nullptr;
    eqs::DriveDev* d_drives = nullptr;
    int32_t* d_int_to_user = nullptr;

    // device: M and the hierarchy
    eqs::Sell<double> M;
    eqs::Hierarchy<double> h64;
    eqs::Hierarchy<float> h32;

    // device: work vectors (n_free doubles each)
    double *d_r = nullptr, *d_z = nullptr, *d_p = nullptr, *d_q = nullptr;
    double* d_mx = nullptr;  // M F of the stage solution in d_F when mx_of_F
    bool mx_of_F = false;
    double *d_Y0 = nullptr, *d_Ya = nullptr, *d_Yb = nullptr, *d_Yc = nullptr, *d_F0 = nullptr, *d_F = nullptr;
    double *d_rhs = nullptr, *d_rhs_alt = nullptr;  // the stage RHS, and the next stage's when it is formed early
    double *d_tmpN = nullptr, *d_tmpN2 = nullptr;  // n_nodes
    bool have_Flast = false;
    double* d_partials = nullptr;  // 4 * max_blocks doubles
    int64_t max_blocks = 0;
    // independent instances (a batch): contiguous node, tet and free-row ranges
    int64_t n_inst = 1;
    std::vector<int64_t> inst_node_off, inst_tet_off;  // user-level offsets [n_inst + 1]
    std::vector<int32_t> inst_row_off;                  // free rows [n_inst + 1]
    int32_t* d_inst_row = nullptr;
    int32_t* d_blk_inst = nullptr;  // instance of the first row of every 256-row block
    std::vector<int32_t> stage_iters; // CG iterations of each stage of the last rkc_step, in stage order
    std::vector<int64_t> inst_iters;  // CG iterations per instance over the last rkc_step / solve
    std::vector<double> inst_relres;  // largest final relative residual per instance over the same

    eqs::PcgScalars* d_scal = nullptr;   // [n_inst]
    eqs::PcgSummary* d_sum = nullptr;
    eqs::PcgScalars* h_scal = nullptr;   // pinned host mirror of d_scal, written by the finalisers
    eqs::PcgScalars* d_hscal = nullptr;  // its device-side address
    eqs::PcgSummary* h_sum = nullptr;    // pinned host mirror of the summary
    eqs::PcgSummary* d_hsum = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};

    // Device memory: every buffer of the context comes from dev_alloc, either
    // allocated by the library (device_bytes counts it) or carved from the
    // caller's workspace [ws_base, ws_base + ws_size) (ws_used counts it);
    // allocations lists both, with lengths rounded to 256 bytes.
    int64_t device_bytes = 0;
    std::vector<std::pair<void*, size_t>> allocations;
    char* ws_base = nullptr;
    int64_t ws_size = 0;
    int64_t ws_used = 0;
    std::map<int64_t, int64_t> ws_free;  // free ranges of the workspace: offset -> length
    bool index16 = true;   // 16-bit column offsets for SELL operators whose entries allow them
    bool autotune = true;  // time the candidate layouts of every AMG operator at build time
    bool fold = true;       // fold pre-smoothers into restrictions and the lowest two levels into two products
    int force_layout = -1;      // >= 1: SELL with that many lanes per row, 0: CSR, for every coarse operator
    bool force_sorted = false;  // with force_layout >= 1: sorted rows where allowed
    int force_unroll = 8;       // with force_layout >= 1: group size of the coarse operators (see Sell::unroll)
    bool tune_verbose = false;  // the tuner log lists every candidate's time
    // test knobs: the element pass with each block's own LDS stride (the path
    // for blocks with more nodes than the fixed stride), and a forced restart
    // at the first true-residual check of every solve
    bool kx_generic = false;
    bool test_reject_first = false;
    int32_t* d_force = nullptr;
    std::string tune_log;  // chosen layouts, one line per operator
    // Tuning record (EQS_TUNE_FILE): choices read from an existing file are
    // replayed instead of timed; otherwise the timed choices are written there
    // at the end of the build. Keys name the operator and its size.
    std::string tune_file;
    std::map<std::string, std::string> tune_replay;
    std::vector<std::string> tune_record;

    // start vectors
    eqs::GuessState guess;

    // the CG iteration body captured once as a HIP graph (x is baked in)
    bool use_graphs = true;
    int32_t graph_iters = 1;  // CG iterations per captured graph (eqs_set_graph_iters)
    hipGraphExec_t iter_exec = nullptr;
    const double* iter_x = nullptr;
    int iter_prec = -1;
    int iter_g = 0;

    // per-kernel-class timing (HIP event pairs around launches)
    uint32_t prof_mask = 0;
    std::vector<hipEvent_t> prof_ev[EQS_KCLASS_COUNT];
    int64_t prof_used[EQS_KCLASS_COUNT] = {};
};

namespace eqs {

// ------------------------------------------------------- host-side setup
void validate_and_order(eqs_ctx* c);
Csr<double> assemble_M_free(const eqs_ctx* c);
struct AmgHost {
    std::vector<Csr<double>> A, P, R;
    std::vector<double> omega;
    std::vector<double> coarse_inv;  // dense inverse of A.back(), column-major
};
AmgHost build_sa_amg(const Csr<double>& M, const eqs_amg_params& p);
void rkc_coefficients(int s, std::vector<double>& mu, std::vector<double>& nu, std::vector<double>& mut,
                      std::vector<double>& gmt, std::vector<double>& c);
double rkc_beta(int s);
// adaptive stepping: max over elements of sigma_e / eps_e at (t, yfree), and
// ref. [9]'s weighted RMS error norm of one step (both synchronise)
double max_rate(eqs_ctx* c, const double* yfree, double t);
double error_norm(eqs_ctx* c, const double* y0, const double* y1, const double* f0, const double* f1, double tau,
                  double atol, double rtol);

// device upload
void* dev_alloc(eqs_ctx* c, size_t bytes);
void dev_free(eqs_ctx* c, void* p);
// Device bytes the context needs for its present configuration: its buffers
// plus those the start-vector settings will allocate on first use.
int64_t workspace_need(const eqs_ctx* c);
// Move every device buffer of the context into [dev, dev + bytes) (dev NULL:
// into memory the library allocates) and release the old memory.
void set_workspace(eqs_ctx* c, void* dev, int64_t bytes);
// Calls f on the address of every device-pointer field of the context (the
// visitor of set_workspace).
void visit_device_ptrs(eqs_ctx* c, const std::function<void(void**)>& f);
int64_t guess_pending_bytes(const eqs_ctx* c);
void guess_alloc_scratch(eqs_ctx* c);
void mlp_visit(eqs_mlp* n, const std::function<void(void**)>& f);
int64_t mlp_device_bytes();  // device bytes of one network (rounded as dev_alloc rounds)
template <typename T>
double time_mv(eqs_ctx* c, const SpMat<T>& A, const T* x, T* y, int reps);
void upload(eqs_ctx* c);
void build_element_blocks(eqs_ctx* c, const std::vector<int32_t>& u2i, const double* yfree, double* out);
void free_device(eqs_ctx* c);
template <typename T>
Sell<T> to_sell(eqs_ctx* c, const Csr<double>& A, int lanes, bool sorted = false);
template <typename T>
SpMat<T> to_spmat(eqs_ctx* c, const Csr<double>& A);


// -------------------------------------------------------- kernel launchers
void launch_fill(hipStream_t s, double* p, double v, int64_t n);
void launch_gather(hipStream_t s, const double* src, const int32_t* idx, double* dst, int64_t n);
void launch_scatter(hipStream_t s, const double* src, const int32_t* idx, double* dst, int64_t n);
void launch_finish_state(eqs_ctx* c, const double* yfree, double t, double* x_user);
// zeroed: `out` is already cleared (no fill launch)
void launch_kx(hipStream_t s, bool rhs_mode, eqs_ctx* c, const double* yfree, double t, double* out,
               bool zeroed = false);
double time_kx(eqs_ctx* c, const double* yfree, double* out, int reps);
void launch_copy(hipStream_t s, double* dst, const double* src, int64_t n);
// zero (may be NULL): also cleared (the next stage's element-pass output)
void launch_rkc_first(eqs_ctx* c, hipStream_t s, double* out, const double* Y0, const double* F0, double a,
                      int64_t n, double* zero = nullptr);
void launch_rkc_combine(eqs_ctx* c, hipStream_t s, double* out, const double* Y0, const double* Yjm1,
                        const double* Yjm2, const double* Fjm1, const double* F0, double c0, double c1, double c2,
                        double c3, double c4, int64_t n, double* zero = nullptr);
void launch_spmv64(hipStream_t s, const Sell<double>& A, const double* x, double* y);

// PCG pieces (all scalar state on the device, one PcgScalars per instance)
// mx (may be NULL): M x as stored by the residual check that ended a solve
// from the same x; the start residual is then rhs - mx without a product.
void pcg_init(hipStream_t s, eqs_ctx* c, const double* rhs, const double* x, int32_t maxit, double rtol,
              int flexible, const double* mx = nullptr);
void pcg_iteration(hipStream_t s, eqs_ctx* c, const double* rhs, double* x, int precision);
// only_if_done: queued before the host knows the outcome of the iteration in
// flight; the kernels act only if that iteration completed every instance
void pcg_true_residual(hipStream_t s, eqs_ctx* c, const double* rhs, const double* x, double* mx_out = nullptr,
                       bool only_if_done = false);
void pcg_zero_rhs_rows(hipStream_t s, eqs_ctx* c, double* x);

template <typename T>
void vcycle(hipStream_t s, eqs_ctx* c, Hierarchy<T>& h, const double* r, double* z, double* part_rz,
            double* part_rzold);

// start-vector network (mlp.hip)
}  // namespace eqs
struct eqs_mlp;
namespace eqs {
// owner (may be NULL): the context whose device memory (dev_alloc) holds the
// network's buffers; NULL: the network allocates its own
eqs_mlp* mlp_create(int device, hipStream_t stream, const float* params, int bf16, double lr,
                    eqs_ctx* owner = nullptr);
void mlp_destroy(eqs_mlp* n);
void mlp_forward(eqs_mlp* n, const float* x, float* y, int32_t B);
void mlp_train(eqs_mlp* n, const float* x, const float* t, int32_t B);
float mlp_last_loss(eqs_mlp* n);
void mlp_get(eqs_mlp* n, float* params, float* grad);
int64_t mlp_state_bytes();
void mlp_save_state(eqs_mlp* n, void* host);
void mlp_load_state(eqs_mlp* n, const void* host);
void mlp_forward_coeffs(eqs_mlp* n, hipStream_t s, const float* x, const double* P, const double* bias,
                        double* alpha, const double* guard, int32_t* stat);

// start vectors (guess.hip)
void guess_configure(eqs_ctx* c, const eqs_guess_params& p);
void guess_release(eqs_ctx* c);
void guess_reset(eqs_ctx* c);
int guess_stage(eqs_ctx* c);
int guess_galerkin_explicit(eqs_ctx* c, int k, const double* S, const double* R, const double* r, double* x0,
                            double* part = nullptr, double* dots_dev = nullptr);
// static device scratch of eqs_galerkin_start_noalloc: set up once per device
// (with that device current), then its address on a device
void noalloc_scratch_init(int device);
double* noalloc_scratch(int device);
constexpr int64_t kNoAllocPartDoubles = (2 * 16 + 3) * 1024;  // dot partials ahead of the 64 summed dots
void guess_after_solve(eqs_ctx* c, int32_t iters);
void guess_train(eqs_ctx* c);
double guess_last_loss(eqs_ctx* c);
void guess_device_stats(eqs_ctx* c, int32_t* kept, int32_t* dropped);

// Byte stream of a checkpoint (eqs_state_save / eqs_state_load). With a NULL
// buffer it only counts; device ranges are copied on the context's stream.
struct StateWriter {
    char* buf = nullptr;
    int64_t cap = 0, n = 0;
    hipStream_t s = nullptr;
    void raw(const void* src, int64_t b) {
        if (buf) {
            if (n + b > cap) fail(EQS_ERR_INVALID_ARG, "state buffer too small");
            if (b > 0) std::memcpy(buf + n, src, (size_t)b);  // an empty vector's data() may be NULL
        }
        n += b;
    }
    template <typename T>
    void val(const T& v) { raw(&v, sizeof v); }
    template <typename T>
    void vec(const std::vector<T>& v) {
        val((int64_t)v.size());
        raw(v.data(), (int64_t)(sizeof(T) * v.size()));
    }
    void dev(const void* d, int64_t b) {
        if (buf && b > 0) {
            if (n + b > cap) fail(EQS_ERR_INVALID_ARG, "state buffer too small");
            EQS_HIP(hipMemcpyAsync(buf + n, d, (size_t)b, hipMemcpyDeviceToHost, s));
            EQS_HIP(hipStreamSynchronize(s));
        }
        n += b;
    }
};
struct StateReader {
    const char* buf = nullptr;
    int64_t cap = 0, n = 0;
    hipStream_t s = nullptr;
    void raw(void* dst, int64_t b) {
        if (b < 0 || n + b > cap) fail(EQS_ERR_INVALID_ARG, "state buffer truncated or not a checkpoint of this set-up");
        if (b > 0) std::memcpy(dst, buf + n, (size_t)b);
        n += b;
    }
    template <typename T>
    T val() {
        T v;
        raw(&v, sizeof v);
        return v;
    }
    template <typename T>
    void vec(std::vector<T>& v, int64_t max_len) {
        const int64_t k = val<int64_t>();
        if (k < 0 || k > max_len) fail(EQS_ERR_INVALID_ARG, "state buffer: bad vector length");
        v.resize((size_t)k);
        raw(v.data(), (int64_t)(sizeof(T) * v.size()));
    }
    void dev(void* d, int64_t b) {
        if (b <= 0) return;
        if (n + b > cap) fail(EQS_ERR_INVALID_ARG, "state buffer truncated or not a checkpoint of this set-up");
        EQS_HIP(hipMemcpyAsync(d, buf + n, (size_t)b, hipMemcpyHostToDevice, s));
        EQS_HIP(hipStreamSynchronize(s));
        n += b;
    }
};
void guess_save_state(eqs_ctx* c, StateWriter& w);
void guess_load_state(eqs_ctx* c, StateReader& r);

// per-kernel timing (profile.cpp)
void prof_begin(eqs_ctx* c, int cls, hipStream_t s);
void prof_end(eqs_ctx* c, int cls, hipStream_t s);
// next start/stop pair of a profiled single-kernel class (false: not profiled)
bool prof_pair(eqs_ctx* c, int cls, hipEvent_t* e0, hipEvent_t* e1);
void prof_release(eqs_ctx* c);

// drivers (solver.cpp)
// mx_in (may be NULL): M y for the incoming y (see pcg_init); mx_out (may be
// NULL): receives M y for the returned y.
// before_sync (may be NULL): queued work the caller wants behind the residual
// check, called each time before the host waits for that check (again after a
// restart, so it acts on the final solution).
int solve_M(eqs_ctx* c, const double* rhs, double* y, double rtol, int32_t maxit, eqs_solve_stats* st,
            const double* mx_in = nullptr, double* mx_out = nullptr,
            const std::function<void()>* before_sync = nullptr);
int rkc_step(eqs_ctx* c, double t, double dt, int32_t s, double* x_user, double rtol, int32_t maxit,
             eqs_step_stats* st);
void apply_preconditioner(eqs_ctx* c, const double* r, double* z);
int rkc_adaptive(eqs_ctx* c, double t0, double t_end, double* x_user, double rtol, int32_t maxit,
                 const eqs_adapt_params& p, eqs_adapt_record* rec, int32_t cap, int32_t* n_rec, eqs_adapt_stats* st);
void release_graphs(eqs_ctx* c);

}  // namespace eqs
