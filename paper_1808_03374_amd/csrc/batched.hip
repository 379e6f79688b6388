// Batched solves: many genotype matrices (per-chromosome PCAs, say) stepped
// together by the FP64 GKL iteration of Section 3 of the paper, with full CGS2
// reorthogonalisation and optional thick restart (Section 3.2 of the paper).
//
// Device work per Lanczos step, for every still-active problem at once:
//   persistent A v_j over the tiles of all problems -> reduce (- beta u_{j-1})
//   -> CGS2 against U -> alpha_j, u_j;
//   persistent A^T u_j -> reduce (- alpha_j v_j) -> CGS2 against V -> beta_j, v_{j+1};
//   step counter += 1.
// That sequence does not depend on j (the kernels read j from device memory),
// so it is captured once in a HIP graph and each step is one graph launch.
// The host intervenes only for convergence tests (one batched Ritz launch, one
// workgroup per problem), thick restarts and the final vectors.
//
// The product geometry (K splits per problem and the persistent grid) is either
// fixed or chosen at create time by timing candidates on the actual matrices.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "engine.h"

namespace gkl {

namespace {
constexpr int64_t kTargets[] = {192, 384, 768, 1536};   // blocks per problem per launch
constexpr int kGrids[] = {512, 1024, 2048};              // persistent workgroups
constexpr int64_t kDefaultTarget = 384;
constexpr int kDefaultGrid = 1024;
}  // namespace

struct BatchProblem {
    Problem prob;
    ProductPlan plan;
    double* partial = nullptr;
    double* U = nullptr;
    double* V = nullptr;
    double* alpha = nullptr;
    double* beta = nullptr;
    double* theta = nullptr;
    double* rho = nullptr;
    double* tnpart = nullptr;
    double* h = nullptr;
    double* npart = nullptr;
    double* anorm = nullptr;
    double* tmp = nullptr;      // restart scratch, max(n, p) x keep
    RitzOut ritz{};
    int64_t cap = 0;            // min(n, p): the largest Krylov basis of this problem
    // per-solve results
    int final_m = 0;
    bool converged = false;
    bool broke = false;
    bool active = false;
    int64_t matvecs = 0;
    int64_t steps = 0;
    int64_t restarts = 0;
};

struct BatchState {
    DeviceArena arena;
    std::vector<std::unique_ptr<BatchProblem>> probs;
    int count = 0;
    int maxm = 0, keep = 0, krylov = 0;
    int hstride = 0;
    int64_t max_n = 0, max_p = 0;
    BatchDesc* d_desc = nullptr;
    int* d_tile_mv = nullptr;
    int* d_tile_rmv = nullptr;
    int* d_state = nullptr;
    int* d_active = nullptr;
    int* d_breakdown = nullptr;
    int* d_nconv = nullptr;
    BatchRitzArgs* d_rargs = nullptr;
    double* svd_scratch = nullptr;
    int64_t mv_target = kDefaultTarget, rmv_target = kDefaultTarget;
    int grid_mv = kDefaultGrid, grid_rmv = kDefaultGrid;
    double tuned_mv_ms = 0.0, tuned_rmv_ms = 0.0;
    bool limb_rmv = false;             // A^T u in int8 limbs (layout S per problem)
    int64_t max_nstX = 0;              // largest number of limb super-tiles along n
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // Leave-one-block-out batch: every problem is the shared matrix without its
    // own SNP block, and the products of all problems are block products with
    // the whole matrix on the matrix cores (split BF16 or int8 limbs).
    bool loco = false;
    Problem shared;                    // the whole matrix: statistics only
    MixedShape mshape;
    uint8_t* mI = nullptr;
    uint8_t* mS = nullptr;
    MixedWork mw;
    double* Wg = nullptr;              // p x count: v_j of every problem
    double* Yg = nullptr;              // n x count: A v_j
    double* Xg = nullptr;              // n x count: u_j
    double* Zg = nullptr;              // p x count: A^T u_j
    int64_t* d_lohi = nullptr;         // own block of each problem
    ~BatchState()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    // Plans, tile prefix sums and descriptors for the given split targets.
    void set_geometry(int64_t mvt, int64_t rmvt)
    {
        std::vector<int> t_mv(count + 1, 0), t_rmv(count + 1, 0);
        std::vector<BatchDesc> desc(count);
        for (int q = 0; q < count; ++q) {
            BatchProblem& P = *probs[q];
            P.plan = product_plan(P.prob.packed, mvt, rmvt);
            const Packed& L = P.prob.packed;
            t_mv[q + 1] = t_mv[q] + P.plan.mv_rowblocks * P.plan.mv_nsplit;
            const BfSplit lg = limb_rmv ? limb_batch_split(L.ms, rmvt) : BfSplit{};
            t_rmv[q + 1] = t_rmv[q] + (limb_rmv ? lg.nrb * lg.nsplit
                                                : P.plan.rmv_colblocks * P.plan.rmv_nsplit);
            BatchDesc& d = desc[q];
            d.T = L.T;
            d.P = L.P;
            d.n = L.n;
            d.p = L.p;
            d.nT = L.nT;
            d.Pq = L.Pq;
            d.pP = L.pP;
            d.nq = L.nq;
            d.mean = P.prob.st.mean;
            d.inv_sd = P.prob.st.inv_sd;
            d.mv_per_split = P.plan.mv_per_split;
            d.rmv_per_split = P.plan.rmv_per_split;
            d.mv_nsplit = P.plan.mv_nsplit;
            d.rmv_nsplit = P.plan.rmv_nsplit;
            d.mv_rowblocks = P.plan.mv_rowblocks;
            d.rmv_colblocks = P.plan.rmv_colblocks;
            d.partial = P.partial;
            d.U = P.U;
            d.V = P.V;
            d.alpha = P.alpha;
            d.beta = P.beta;
            d.theta = P.theta;
            d.rho = P.rho;
            d.tnpart = P.tnpart;
            d.h = P.h;
            d.npart = P.npart;
            d.anorm = P.anorm;
            d.active = d_active + q;
            d.breakdown = d_breakdown + q;
            d.S = nullptr;
            d.ldS = d.nstX = d.limb_st_per = 0;
            d.limb_nrb = 0;
            d.lfrag = nullptr;
            d.lcpart = d.lcmax = nullptr;
            if (limb_rmv) {
                const MixedShape& m = L.ms;
                d.S = L.S;
                d.ldS = m.ldS;
                d.nstX = m.nstX;
                d.pP = m.pS;
                d.rmv_nsplit = lg.nsplit;
                d.limb_st_per = lg.st_per;
                d.limb_nrb = lg.nrb;
                d.lfrag = P.prob.mvw.lfrag;
                d.lcpart = P.prob.mvw.lcpart;
                d.lcmax = P.prob.mvw.lcmax;
            }
        }
        if (t_mv[count] < 0 || t_rmv[count] < 0) fail(GKL_ERR_INVALID, "batch too large");
        GKL_HIP(hipMemcpyAsync(d_desc, desc.data(), sizeof(BatchDesc) * count,
                               hipMemcpyHostToDevice, stream));
        GKL_HIP(hipMemcpyAsync(d_tile_mv, t_mv.data(), sizeof(int) * (count + 1),
                               hipMemcpyHostToDevice, stream));
        GKL_HIP(hipMemcpyAsync(d_tile_rmv, t_rmv.data(), sizeof(int) * (count + 1),
                               hipMemcpyHostToDevice, stream));
        GKL_HIP(hipStreamSynchronize(stream));
        mv_target = mvt;
        rmv_target = rmvt;
    }

    void set_active(const std::vector<int>& a)
    {
        GKL_HIP(hipMemcpyAsync(d_active, a.data(), sizeof(int) * count, hipMemcpyHostToDevice,
                               stream));
        GKL_HIP(hipStreamSynchronize(stream));
    }

    void set_state(int j, int nlock)
    {
        const int h[2] = {j, nlock};
        GKL_HIP(hipMemcpyAsync(d_state, h, sizeof(h), hipMemcpyHostToDevice, stream));
        GKL_HIP(hipStreamSynchronize(stream));   // h lives on this stack frame
    }

    // The partials of A^T u_j of every active problem.
    void right_product(int grid)
    {
        if (limb_rmv)
            launch_blimb_rmatvec(d_desc, d_tile_rmv, count, d_state, grid, max_nstX, stream);
        else
            launch_brmatvec(d_desc, d_tile_rmv, count, d_state, grid, stream);
    }

    // One Lanczos step of every active problem (the captured sequence).
    void record_step()
    {
        if (loco) {
            launch_loco_gather(d_desc, d_state, count, 0, Wg, max_p, stream);
            launch_matmat_mixed(mshape, mI, shared.st, Wg, max_p, count, Yg, max_n, mw, stream);
            launch_loco_left(d_desc, d_state, count, Yg, max_n, stream);
            launch_bortho(d_desc, d_state, count, 0, max_n, hstride, stream);
            launch_loco_gather(d_desc, d_state, count, 1, Xg, max_n, stream);
            launch_rmatmat_mixed(mshape, mS, shared.st, Xg, max_n, count, Zg, max_p, mw, stream);
            launch_loco_right(d_desc, d_state, count, Zg, max_p, d_lohi, stream);
            launch_bortho(d_desc, d_state, count, 1, max_p, hstride, stream);
            launch_bstep(d_state, stream);
            return;
        }
        launch_bmatvec(d_desc, d_tile_mv, count, d_state, grid_mv, stream);
        launch_bmatvec_reduce(d_desc, d_state, count, max_n, stream);
        launch_bortho(d_desc, d_state, count, 0, max_n, hstride, stream);
        right_product(grid_rmv);
        launch_brmatvec_reduce(d_desc, d_state, count, max_p, stream);
        launch_bortho(d_desc, d_state, count, 1, max_p, hstride, stream);
        launch_bstep(d_state, stream);
    }

    void step()
    {
        if (!use_graph) {
            record_step();
            return;
        }
        if (!exec) {
            GKL_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
            try {
                record_step();
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            GKL_HIP(hipStreamEndCapture(stream, &graph));
            GKL_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        }
        GKL_HIP(hipGraphLaunch(exec, stream));
    }

    // Average time of `reps` product launches (left or right) with the current
    // geometry, after one untimed launch.
    double time_product(bool right, int grid, int reps)
    {
        hipEvent_t e0, e1;
        GKL_HIP(hipEventCreate(&e0));
        GKL_HIP(hipEventCreate(&e1));
        float ms = 0.f;
        try {
            for (int r = 0; r <= reps; ++r) {
                if (r == 1) GKL_HIP(hipEventRecord(e0, stream));
                if (right) right_product(grid);
                else launch_bmatvec(d_desc, d_tile_mv, count, d_state, grid, stream);
            }
            GKL_HIP(hipEventRecord(e1, stream));
            GKL_HIP(hipEventSynchronize(e1));
            GKL_HIP(hipEventElapsedTime(&ms, e0, e1));
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return ms / reps;
    }

    // Try every (split target, grid) pair for each product and keep the fastest.
    void autotune(uint64_t seed)
    {
        for (int q = 0; q < count; ++q) {
            BatchProblem& P = *probs[q];
            launch_gaussian(P.V, P.prob.p, seed, 0x7017 + q, stream);
            launch_gaussian(P.U, P.prob.n, seed, 0x9017 + q, stream);
        }
        set_active(std::vector<int>(count, 1));
        set_state(0, 0);
        double best_mv = 1e30, best_rmv = 1e30;
        int64_t bt_mv = kDefaultTarget, bt_rmv = kDefaultTarget;
        int bg_mv = kDefaultGrid, bg_rmv = kDefaultGrid;
        for (int64_t t : kTargets) {
            set_geometry(t, t);
            for (int g : kGrids) {
                const double a = time_product(false, g, 3);
                if (a < best_mv) { best_mv = a; bt_mv = t; bg_mv = g; }
                const double b = time_product(true, g, 3);
                if (b < best_rmv) { best_rmv = b; bt_rmv = t; bg_rmv = g; }
            }
        }
        grid_mv = bg_mv;
        grid_rmv = bg_rmv;
        tuned_mv_ms = best_mv;
        tuned_rmv_ms = best_rmv;
        set_geometry(bt_mv, bt_rmv);
    }
};

void destroy_batch(BatchState* b) { delete b; }

namespace {
// Krylov bases, scalars and Ritz workspace of one problem (n x p, basis m).
void alloc_problem(BatchState& B, BatchProblem& P, int64_t n, int64_t p, hipStream_t s)
{
    const int m = B.maxm;
    DeviceArena& A = P.prob.arena;
    P.U = static_cast<double*>(A.alloc(sizeof(double) * (size_t)n * m));
    P.V = static_cast<double*>(A.alloc(sizeof(double) * (size_t)p * (m + 1)));
    double* sc = static_cast<double*>(A.alloc(sizeof(double) * 4 * (size_t)(m + 2)));
    P.alpha = sc;
    P.beta = sc + (m + 2);
    P.theta = sc + 2 * (m + 2);
    P.rho = sc + 3 * (m + 2);
    const size_t ch = bortho_chunks(std::max(n, p));
    P.tnpart = static_cast<double*>(A.alloc(sizeof(double) * batch_tn_partial_elems(B.hstride)));
    P.h = static_cast<double*>(A.alloc(sizeof(double) * B.hstride));
    P.npart = static_cast<double*>(A.alloc(sizeof(double) * ch));
    P.anorm = static_cast<double*>(A.alloc(sizeof(double)));
    if (B.krylov > 0)
        P.tmp = static_cast<double*>(A.alloc(sizeof(double) * (size_t)std::max(n, p) * B.keep));
    const size_t mm = (size_t)m * m;
    P.ritz.B = static_cast<double*>(A.alloc(sizeof(double) * mm));
    P.ritz.P = static_cast<double*>(A.alloc(sizeof(double) * mm));
    P.ritz.Q = static_cast<double*>(A.alloc(sizeof(double) * mm));
    P.ritz.S = static_cast<double*>(A.alloc(sizeof(double) * m));
    P.ritz.res = static_cast<double*>(A.alloc(sizeof(double) * m));
    GKL_HIP(hipMemsetAsync(sc, 0, sizeof(double) * 4 * (size_t)(m + 2), s));
}

// Shared device state of a batch (descriptors, step state, flags, Ritz args).
void alloc_batch_state(BatchState& B, hipStream_t s)
{
    const int count = B.count, m = B.maxm;
    DeviceArena& A = B.arena;
    B.d_desc = static_cast<BatchDesc*>(A.alloc(sizeof(BatchDesc) * count));
    B.d_tile_mv = static_cast<int*>(A.alloc(sizeof(int) * (count + 1)));
    B.d_tile_rmv = static_cast<int*>(A.alloc(sizeof(int) * (count + 1)));
    B.d_state = static_cast<int*>(A.alloc(sizeof(int) * 2));
    B.d_active = static_cast<int*>(A.alloc(sizeof(int) * count));
    B.d_breakdown = static_cast<int*>(A.alloc(sizeof(int) * count));
    B.d_nconv = static_cast<int*>(A.alloc(sizeof(int) * count));
    B.d_rargs = static_cast<BatchRitzArgs*>(A.alloc(sizeof(BatchRitzArgs) * count));
    if (!svd_fits_lds(m))
        B.svd_scratch = static_cast<double*>(A.alloc(sizeof(double) * svd_scratch_elems(m) * count));
    for (int q = 0; q < count; ++q) B.probs[q]->ritz.nconv = B.d_nconv + q;
    GKL_HIP(hipMemsetAsync(B.d_breakdown, 0, sizeof(int) * count, s));
}

// Basis capacity and restart keep count shared by the batch.
void batch_basis(BatchState& B, const gkl_options* o, int k, int64_t mx)
{
    if (o->krylov_dim > 0) {
        B.krylov = o->krylov_dim;
        B.maxm = (int)std::min<int64_t>(o->krylov_dim, mx);
        B.keep = o->keep > 0 ? o->keep : k + (B.krylov - k) / 2;
        B.keep = std::min(B.keep, B.maxm - 1);
        if (B.maxm <= k) B.krylov = 0;
    } else {
        B.maxm = (int)std::min<int64_t>(o->max_steps > 0 ? o->max_steps : 512, mx);
    }
    B.hstride = B.maxm + 2;
}

// The batch's stream: the caller's, or a new non-blocking one (graph capture
// needs a stream other than the null stream, which it does not order after).
void batch_stream(BatchState& B, const gkl_options* o)
{
    if (o->stream) {
        B.stream = static_cast<hipStream_t>(o->stream);
    } else {
        GKL_HIP(hipDeviceSynchronize());
        GKL_HIP(hipStreamCreateWithFlags(&B.stream, hipStreamNonBlocking));
        B.own_stream = true;
    }
}
}  // namespace

namespace {
gkl_status batch_error(gkl_ctx* ctx, gkl_status s, const std::string& msg)
{
    if (ctx) ctx->last_error = msg;
    else set_create_error(msg);
    return s;
}

void finalize_problem(BatchProblem& P, int k, double* sigma, double* Uo, int64_t ldu, double* Vo,
                      int64_t ldv, hipStream_t s)
{
    const int m = P.final_m;
    const int kk = std::min(k, m);
    const int64_t n = P.prob.n, p = P.prob.p;
    GKL_HIP(hipMemcpyAsync(sigma, P.ritz.S, sizeof(double) * kk, hipMemcpyDeviceToDevice, s));
    launch_gemm_nn(P.U, n, m, P.ritz.P, m, Uo, ldu, n, kk, 0, s);
    launch_gemm_nn(P.V, p, m, P.ritz.Q, m, Vo, ldv, p, kk, 0, s);
    launch_sign_fix(Uo, ldu, n, Vo, ldv, p, kk, s);
}
}  // namespace

}  // namespace gkl

using namespace gkl;

extern "C" {

gkl_status gkl_create_batched(int32_t count, const uint8_t* const* G, const int64_t* n,
                              const int64_t* p, int32_t k, double tol, int32_t reorth,
                              const gkl_options* o, gkl_ctx** out)
{
    if (!out) return batch_error(nullptr, GKL_ERR_INVALID, "out is NULL");
    if (count < 1 || count > kMaxBatch)
        return batch_error(nullptr, GKL_ERR_INVALID, "count must lie in [1, 1024]");
    if (!G || !n || !p || !o) return batch_error(nullptr, GKL_ERR_INVALID, "NULL array argument");
    if (o->struct_size != sizeof(gkl_options))
        return batch_error(nullptr, GKL_ERR_INVALID, "options.struct_size mismatch (ABI version)");
    if (!(tol > 0.0) || !std::isfinite(tol))
        return batch_error(nullptr, GKL_ERR_INVALID, "tol must be > 0");
    if (reorth != GKL_REORTH_FULL && reorth != GKL_REORTH_PARTIAL && reorth != GKL_REORTH_ONESIDED)
        return batch_error(nullptr, GKL_ERR_INVALID,
                           "reorth must be GKL_REORTH_FULL, _PARTIAL or _ONESIDED");
    if (reorth != GKL_REORTH_FULL)
        return batch_error(nullptr, GKL_ERR_UNSUPPORTED,
                           "batched solves use full reorthogonalisation (GKL_REORTH_FULL)");
    if (o->precision != GKL_PREC_FP64)
        return batch_error(nullptr, GKL_ERR_UNSUPPORTED, "batched solves run in FP64");
    int64_t mn = INT64_MAX, mx = 0;
    for (int q = 0; q < count; ++q) {
        if (!G[q]) return batch_error(nullptr, GKL_ERR_INVALID, "G[q] is NULL");
        if (n[q] < 1 || p[q] < 1) return batch_error(nullptr, GKL_ERR_INVALID, "n and p must be >= 1");
        if (o->ld_bytes != 0 && o->ld_bytes < (n[q] + 3) / 4)
            return batch_error(nullptr, GKL_ERR_INVALID, "ld_bytes < ceil(n/4)");
        mn = std::min(mn, std::min(n[q], p[q]));
        mx = std::max(mx, std::min(n[q], p[q]));
    }
    if (k < 1 || (int64_t)k > mn)
        return batch_error(nullptr, GKL_ERR_INVALID, "k must lie in [1, min(n, p)] of every problem");
    if (o->krylov_dim < 0 || (o->krylov_dim > 0 && o->krylov_dim <= k))
        return batch_error(nullptr, GKL_ERR_INVALID, "krylov_dim must be 0 or > k");
    if (o->krylov_dim > kMaxSvd || o->max_steps < 0 || o->max_steps > kMaxSvd)
        return batch_error(nullptr, GKL_ERR_INVALID, "krylov_dim / max_steps too large");
    if (o->keep < 0 || (o->krylov_dim > 0 && o->keep > 0 && (o->keep < k || o->keep >= o->krylov_dim)))
        return batch_error(nullptr, GKL_ERR_INVALID, "keep must lie in [k, krylov_dim)");
    if (o->check_every < 0 || o->max_matvecs < 0)
        return batch_error(nullptr, GKL_ERR_INVALID, "bad check_every / max_matvecs");
    if (o->restart == GKL_RESTART_HARMONIC)
        return batch_error(nullptr, GKL_ERR_UNSUPPORTED,
                           "harmonic restarts are built for single problems (gkl_create_ex)");
    if (o->restart != GKL_RESTART_RITZ)
        return batch_error(nullptr, GKL_ERR_INVALID, "restart must be GKL_RESTART_RITZ or _HARMONIC");
    gkl_ctx* ctx = nullptr;
    try {
        auto t0 = std::chrono::steady_clock::now();
        ctx = new gkl_ctx();
        ctx->batched = true;
        ctx->opt = *o;
        ctx->k = k;
        ctx->tol = tol;
        ctx->reorth = reorth;
        ctx->batch = new BatchState();
        BatchState& B = *ctx->batch;
        B.count = count;
        B.use_graph = o->graph != 0;
        batch_stream(B, o);
        hipStream_t s = B.stream;
        // The basis capacity is shared (problems step together); a problem whose own
        // min(n, p) is smaller leaves the batch when its Krylov space is complete.
        batch_basis(B, o, k, mx);
        double total = 0.0;
        for (int q = 0; q < count; ++q) total += (double)n[q] * (double)p[q];
        // A^T u from the tables or in int8 limbs (A v always from the tables), as
        // options.fp64_products asks; GKL_FP64_AUTO takes the limbs from 1 GB of
        // packed genotypes in the whole batch on
        B.limb_rmv = o->fp64_products == GKL_FP64_LIMBS || o->fp64_products == GKL_FP64_LUT_LIMBS ||
                     (o->fp64_products == GKL_FP64_AUTO && total >= 4e9);
        for (int q = 0; q < count; ++q) {
            B.probs.emplace_back(new BatchProblem());
            BatchProblem& P = *B.probs.back();
            const int64_t ld = o->ld_bytes ? o->ld_bytes : (n[q] + 3) / 4;
            P.prob.setup(G[q], n[q], p[q], ld, s, B.limb_rmv ? 3 : 1);
            if (B.limb_rmv) B.max_nstX = std::max(B.max_nstX, P.prob.packed.ms.nstX);
            P.cap = std::min(n[q], p[q]);
            B.max_n = std::max(B.max_n, n[q]);
            B.max_p = std::max(B.max_p, p[q]);
            size_t pe = 0;
            for (int64_t t : kTargets)
                pe = std::max(pe, product_plan_partial_elems(P.prob.packed,
                                                             product_plan(P.prob.packed, t, t)));
            if (B.limb_rmv) {
                const MixedShape& m = P.prob.packed.ms;
                for (int64_t t : kTargets)
                    pe = std::max(pe, (size_t)limb_batch_split(m, t).nsplit * (size_t)m.pS);
            }
            P.partial = static_cast<double*>(P.prob.arena.alloc(sizeof(double) * pe));
            alloc_problem(B, P, n[q], p[q], s);
        }
        alloc_batch_state(B, s);
        B.set_geometry(kDefaultTarget, kDefaultTarget);
        if (o->autotune) B.autotune(o->seed);
        GKL_HIP(hipStreamSynchronize(s));
        ctx->create_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = ctx;
        return GKL_OK;
    } catch (const Error& e) {
        delete ctx;
        return batch_error(nullptr, e.status, e.msg);
    } catch (const std::bad_alloc&) {
        delete ctx;
        return batch_error(nullptr, GKL_ERR_NOMEM, "host allocation failed");
    } catch (...) {
        delete ctx;
        return batch_error(nullptr, GKL_ERR_INTERNAL, "unexpected exception in gkl_create_batched");
    }
}

gkl_status gkl_create_loco(const uint8_t* G, int64_t n, int64_t p, int32_t nblocks,
                           const int64_t* block_start, int32_t k, double tol,
                           const gkl_options* o, gkl_ctx** out)
{
    if (!out) return batch_error(nullptr, GKL_ERR_INVALID, "out is NULL");
    if (!G || !block_start || !o) return batch_error(nullptr, GKL_ERR_INVALID, "NULL argument");
    if (o->struct_size != sizeof(gkl_options))
        return batch_error(nullptr, GKL_ERR_INVALID, "options.struct_size mismatch (ABI version)");
    if (nblocks < 2 || nblocks > 32)
        return batch_error(nullptr, GKL_ERR_INVALID, "nblocks must lie in [2, 32]");
    if (n < 1 || p < 1) return batch_error(nullptr, GKL_ERR_INVALID, "n and p must be >= 1");
    if (block_start[0] != 0 || block_start[nblocks] != p)
        return batch_error(nullptr, GKL_ERR_INVALID, "block_start must run from 0 to p");
    int64_t max_block = 0;
    for (int q = 0; q < nblocks; ++q) {
        if (block_start[q + 1] <= block_start[q])
            return batch_error(nullptr, GKL_ERR_INVALID, "blocks must be non-empty and increasing");
        max_block = std::max(max_block, block_start[q + 1] - block_start[q]);
    }
    if (!(tol > 0.0) || !std::isfinite(tol))
        return batch_error(nullptr, GKL_ERR_INVALID, "tol must be > 0");
    const int64_t mn = std::min(n, p - max_block);
    if (k < 1 || (int64_t)k > mn)
        return batch_error(nullptr, GKL_ERR_INVALID,
                           "k must lie in [1, min(n, p - largest block)]");
    if (o->precision != GKL_PREC_MIXED && o->precision != GKL_PREC_MIXED_INT8)
        return batch_error(nullptr, GKL_ERR_UNSUPPORTED,
                           "leave-one-block-out solves use the matrix-core block products "
                           "(GKL_PREC_MIXED or GKL_PREC_MIXED_INT8)");
    if (o->ld_bytes != 0 && o->ld_bytes < (n + 3) / 4)
        return batch_error(nullptr, GKL_ERR_INVALID, "ld_bytes < ceil(n/4)");
    if (o->krylov_dim < 0 || (o->krylov_dim > 0 && o->krylov_dim <= k))
        return batch_error(nullptr, GKL_ERR_INVALID, "krylov_dim must be 0 or > k");
    if (o->krylov_dim > kMaxSvd || o->max_steps < 0 || o->max_steps > kMaxSvd)
        return batch_error(nullptr, GKL_ERR_INVALID, "krylov_dim / max_steps too large");
    if (o->keep < 0 || (o->krylov_dim > 0 && o->keep > 0 && (o->keep < k || o->keep >= o->krylov_dim)))
        return batch_error(nullptr, GKL_ERR_INVALID, "keep must lie in [k, krylov_dim)");
    if (o->check_every < 0 || o->max_matvecs < 0)
        return batch_error(nullptr, GKL_ERR_INVALID, "bad check_every / max_matvecs");
    if (o->restart == GKL_RESTART_HARMONIC)
        return batch_error(nullptr, GKL_ERR_UNSUPPORTED,
                           "harmonic restarts are built for single problems (gkl_create_ex)");
    if (o->restart != GKL_RESTART_RITZ)
        return batch_error(nullptr, GKL_ERR_INVALID, "restart must be GKL_RESTART_RITZ or _HARMONIC");
    gkl_ctx* ctx = nullptr;
    try {
        auto t0 = std::chrono::steady_clock::now();
        ctx = new gkl_ctx();
        ctx->batched = true;
        ctx->opt = *o;
        ctx->k = k;
        ctx->tol = tol;
        ctx->reorth = GKL_REORTH_FULL;
        ctx->batch = new BatchState();
        BatchState& B = *ctx->batch;
        B.count = nblocks;
        B.loco = true;
        B.use_graph = o->graph != 0;
        batch_stream(B, o);
        hipStream_t s = B.stream;
        batch_basis(B, o, k, mn);
        const int64_t ld = o->ld_bytes ? o->ld_bytes : (n + 3) / 4;
        B.shared.setup(G, n, p, ld, s, 0);
        B.max_n = n;
        B.max_p = p;
        DeviceArena& A = B.arena;
        B.mshape = mixed_shape(n, p);
        B.mshape.int8 = o->precision == GKL_PREC_MIXED_INT8;
        B.mI = static_cast<uint8_t*>(A.alloc((size_t)B.mshape.nI * B.mshape.ldI));
        B.mS = static_cast<uint8_t*>(A.alloc((size_t)B.mshape.pS * B.mshape.ldS));
        build_mixed_layouts(G, n, p, ld, B.mI, B.mS, s);
        B.mw.frag = A.alloc(mixed_frag_bytes(B.mshape));
        B.mw.partial = static_cast<double*>(A.alloc(sizeof(double) * mixed_partial_elems(B.mshape)));
        B.mw.cpart = static_cast<double*>(A.alloc(sizeof(double) * 32 * 64));
        B.mw.cmax = static_cast<double*>(A.alloc(sizeof(double) * 32 * 64));
        B.Wg = static_cast<double*>(A.alloc(sizeof(double) * (size_t)p * nblocks));
        B.Zg = static_cast<double*>(A.alloc(sizeof(double) * (size_t)p * nblocks));
        B.Yg = static_cast<double*>(A.alloc(sizeof(double) * (size_t)n * nblocks));
        B.Xg = static_cast<double*>(A.alloc(sizeof(double) * (size_t)n * nblocks));
        std::vector<int64_t> lohi(2 * (size_t)nblocks);
        for (int q = 0; q < nblocks; ++q) {
            lohi[2 * q] = block_start[q];
            lohi[2 * q + 1] = block_start[q + 1];
        }
        B.d_lohi = static_cast<int64_t*>(A.alloc(sizeof(int64_t) * lohi.size()));
        GKL_HIP(hipMemcpyAsync(B.d_lohi, lohi.data(), sizeof(int64_t) * lohi.size(),
                               hipMemcpyHostToDevice, s));
        for (int q = 0; q < nblocks; ++q) {
            B.probs.emplace_back(new BatchProblem());
            BatchProblem& P = *B.probs.back();
            // the problem's sizes and statistics are the shared matrix's; its
            // right vectors carry zeros on its own block
            P.prob.n = n;
            P.prob.p = p;
            P.prob.ld = ld;
            P.prob.G_user = G;
            P.prob.stream = s;
            P.prob.st = B.shared.st;
            layout_shape(n, p, P.prob.packed);
            P.cap = std::min(n, p - (lohi[2 * q + 1] - lohi[2 * q]));
            P.partial = nullptr;
            alloc_problem(B, P, n, p, s);
        }
        alloc_batch_state(B, s);
        B.set_geometry(kDefaultTarget, kDefaultTarget);
        GKL_HIP(hipStreamSynchronize(s));
        ctx->create_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = ctx;
        return GKL_OK;
    } catch (const Error& e) {
        delete ctx;
        return batch_error(nullptr, e.status, e.msg);
    } catch (const std::bad_alloc&) {
        delete ctx;
        return batch_error(nullptr, GKL_ERR_NOMEM, "host allocation failed");
    } catch (...) {
        delete ctx;
        return batch_error(nullptr, GKL_ERR_INTERNAL, "unexpected exception in gkl_create_loco");
    }
}

gkl_status gkl_solve_batched(gkl_ctx* ctx, double* const* sigma, double* const* Uo,
                             const int64_t* ldu, double* const* Vo, const int64_t* ldv,
                             gkl_info* infos)
{
    if (!ctx) return batch_error(nullptr, GKL_ERR_INVALID, "ctx is NULL");
    if (!ctx->batched || !ctx->batch)
        return batch_error(ctx, GKL_ERR_INVALID, "ctx was not made by gkl_create_batched");
    if (!sigma || !Uo || !ldu || !Vo || !ldv)
        return batch_error(ctx, GKL_ERR_INVALID, "NULL array argument");
    BatchState& B = *ctx->batch;
    const int count = B.count;
    for (int q = 0; q < count; ++q) {
        if (!sigma[q] || !Uo[q] || !Vo[q]) return batch_error(ctx, GKL_ERR_INVALID, "NULL output pointer");
        if (ldu[q] < B.probs[q]->prob.n || ldv[q] < B.probs[q]->prob.p)
            return batch_error(ctx, GKL_ERR_INVALID, "ldu < n or ldv < p");
    }
    try {
        auto t0 = std::chrono::steady_clock::now();
        hipStream_t s = B.stream;
        if (B.own_stream) GKL_HIP(hipDeviceSynchronize());
        const int k = ctx->k;
        const double tol = ctx->tol;
        const gkl_options& o = ctx->opt;
        // start vectors: o.v0 holds the problems' p-vectors back to back
        int64_t off = 0;
        for (int q = 0; q < count; ++q) {
            BatchProblem& P = *B.probs[q];
            const int64_t pq = P.prob.p;
            if (o.v0) GKL_HIP(hipMemcpyAsync(P.V, o.v0 + off, sizeof(double) * pq,
                                             hipMemcpyDeviceToDevice, s));
            else launch_gaussian(P.V, pq, o.seed, (uint64_t)q, s);
            off += pq;
            GKL_HIP(hipMemsetAsync(P.alpha, 0, sizeof(double) * 4 * (size_t)(B.maxm + 2), s));
            P.final_m = 0;
            P.converged = P.broke = false;
            P.active = true;
            P.matvecs = P.steps = P.restarts = 0;
        }
        GKL_HIP(hipMemsetAsync(B.d_breakdown, 0, sizeof(int) * count, s));
        std::vector<int> act(count, 1);
        B.set_active(act);
        if (B.loco) launch_loco_mask(B.d_desc, count, B.d_lohi, s);
        launch_bstart(B.d_desc, count, B.max_p, B.hstride, s);
        B.set_state(0, 0);
        const int check_every = o.check_every > 0 ? o.check_every : (B.krylov > 0 ? 0 : 5);
        int j = 0, nlock = 0, last_check = 0;
        int64_t total_steps = 0;
        int nactive = count;
        std::vector<BatchRitzArgs> rargs(count);
        std::vector<int> nconv(count), brk(count);
        while (nactive > 0) {
            B.step();
            ++j;
            ++total_steps;
            for (auto& P : B.probs)
                if (P->active) {
                    P->matvecs += 2;
                    P->steps += 1;
                }
            const bool full = j >= B.maxm;
            const bool budget = o.max_matvecs > 0 && 2 * total_steps >= o.max_matvecs;
            bool complete = false;   // some active problem has a complete Krylov space
            for (auto& P : B.probs) complete = complete || (P->active && j >= P->cap);
            const bool due = (j >= k && (full || budget || (check_every > 0 && j - last_check >= check_every))) ||
                             complete;
            if (!due) continue;
            last_check = j;
            for (int q = 0; q < count; ++q) {
                BatchProblem& P = *B.probs[q];
                rargs[q] = BatchRitzArgs{P.alpha, P.beta, P.theta, P.rho, P.ritz, P.active ? 1 : 0};
            }
            GKL_HIP(hipMemcpyAsync(B.d_rargs, rargs.data(), sizeof(BatchRitzArgs) * count,
                                   hipMemcpyHostToDevice, s));
            launch_ritz_batched(B.d_rargs, count, nlock, j, k, tol, B.svd_scratch, s);
            GKL_HIP(hipMemcpyAsync(nconv.data(), B.d_nconv, sizeof(int) * count,
                                   hipMemcpyDeviceToHost, s));
            GKL_HIP(hipMemcpyAsync(brk.data(), B.d_breakdown, sizeof(int) * count,
                                   hipMemcpyDeviceToHost, s));
            GKL_HIP(hipStreamSynchronize(s));
            bool changed = false;
            for (int q = 0; q < count; ++q) {
                BatchProblem& P = *B.probs[q];
                if (!P.active) continue;
                // a breakdown on the last vector a complete Krylov space can hold is
                // the end of that space, not a failure: its Ritz values are exact
                const bool exhausted = brk[q] && (brk[q] - 1) / 2 + 1 >= P.cap;
                if (brk[q] && !exhausted) {
                    P.broke = true;
                } else if (nconv[q] >= k) {
                    P.converged = true;
                } else if (!(budget || (full && B.krylov == 0) || j >= P.cap)) {
                    continue;
                }
                P.active = false;
                P.final_m = j;
                act[q] = 0;
                --nactive;
                changed = true;
            }
            if (changed) B.set_active(act);
            if (nactive == 0) break;
            if (full) {
                // thick restart of every remaining problem, keeping B.keep Ritz
                // vectors: V(:, 0:l) = V Q(:, 0:l), v_l = v_m, U(:, 0:l) = U P(:, 0:l)
                const int kp = B.keep;
                for (int q = 0; q < count; ++q) {
                    BatchProblem& P = *B.probs[q];
                    if (!P.active) continue;
                    const int64_t nq = P.prob.n, pq = P.prob.p;
                    launch_gemm_nn(P.V, pq, j, P.ritz.Q, j, P.tmp, pq, pq, kp, 0, s);
                    GKL_HIP(hipMemcpyAsync(P.V, P.tmp, sizeof(double) * (size_t)pq * kp,
                                           hipMemcpyDeviceToDevice, s));
                    GKL_HIP(hipMemcpyAsync(P.V + (int64_t)kp * pq, P.V + (int64_t)j * pq,
                                           sizeof(double) * (size_t)pq, hipMemcpyDeviceToDevice, s));
                    launch_gemm_nn(P.U, nq, j, P.ritz.P, j, P.tmp, nq, nq, kp, 0, s);
                    GKL_HIP(hipMemcpyAsync(P.U, P.tmp, sizeof(double) * (size_t)nq * kp,
                                           hipMemcpyDeviceToDevice, s));
                    launch_restart_scalars(P.ritz.S, P.ritz.P, j, P.beta + (j - 1), kp, P.theta,
                                           P.rho, s);
                    P.restarts += 1;
                }
                j = kp;
                nlock = kp;
                last_check = kp;
                B.set_state(j, nlock);
            }
        }
        // outputs
        bool all_conv = true, any_broke = false;
        for (int q = 0; q < count; ++q) {
            BatchProblem& P = *B.probs[q];
            if (P.final_m == 0) P.final_m = j;
            finalize_problem(P, k, sigma[q], Uo[q], ldu[q], Vo[q], ldv[q], s);
            all_conv = all_conv && P.converged;
            any_broke = any_broke || P.broke;
        }
        std::vector<double> res((size_t)count * k), s0(count);
        for (int q = 0; q < count; ++q) {
            BatchProblem& P = *B.probs[q];
            const int kk = std::min(k, P.final_m);
            GKL_HIP(hipMemcpyAsync(res.data() + (size_t)q * k, P.ritz.res, sizeof(double) * kk,
                                   hipMemcpyDeviceToHost, s));
            GKL_HIP(hipMemcpyAsync(s0.data() + q, P.ritz.S, sizeof(double), hipMemcpyDeviceToHost, s));
        }
        GKL_HIP(hipStreamSynchronize(s));
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (infos) {
            for (int q = 0; q < count; ++q) {
                BatchProblem& P = *B.probs[q];
                gkl_info& I = infos[q];
                I = gkl_info{};
                I.matvecs = P.matvecs;
                I.passes_over_G = P.matvecs;
                I.steps = P.steps;
                I.restarts = P.restarts;
                I.reorths = 2 * P.matvecs;
                I.converged = P.converged ? 1 : 0;
                I.nconv = P.converged ? k : 0;
                if (!B.loco) I.fp64_products = B.limb_rmv ? GKL_FP64_LUT_LIMBS : GKL_FP64_LUT;
                const int kk = std::min(k, P.final_m);
                double sum = 0.0, mx = 0.0;
                for (int i = 0; i < kk; ++i) {
                    const double r = res[(size_t)q * k + i];
                    sum += r;
                    mx = std::max(mx, s0[q] > 0 ? r / s0[q] : 0.0);
                }
                I.sum_residual_est = sum;
                I.max_residual_rel = mx;
                I.solve_ms = ms;
                I.create_ms = ctx->create_ms;
            }
        }
        if (any_broke) {
            ctx->last_error = "a problem of the batch broke down (no new Lanczos direction)";
            return GKL_ERR_BREAKDOWN;
        }
        if (!all_conv) {
            ctx->last_error = "tolerance not met within the step budget for some problems";
            return GKL_NOT_CONVERGED;
        }
        return GKL_OK;
    } catch (const Error& e) {
        return batch_error(ctx, e.status, e.msg);
    } catch (...) {
        return batch_error(ctx, GKL_ERR_INTERNAL, "unexpected exception in gkl_solve_batched");
    }
}

gkl_status gkl_batched_plan(const gkl_ctx* ctx, int64_t* mv_target, int64_t* rmv_target,
                            int32_t* grid_mv, int32_t* grid_rmv, double* mv_ms, double* rmv_ms)
{
    if (!ctx || !ctx->batched || !ctx->batch) return GKL_ERR_INVALID;
    const BatchState& B = *ctx->batch;
    if (mv_target) *mv_target = B.mv_target;
    if (rmv_target) *rmv_target = B.rmv_target;
    if (grid_mv) *grid_mv = B.grid_mv;
    if (grid_rmv) *grid_rmv = B.grid_rmv;
    if (mv_ms) *mv_ms = B.tuned_mv_ms;
    if (rmv_ms) *rmv_ms = B.tuned_rmv_ms;
    return GKL_OK;
}

}  // extern "C"
