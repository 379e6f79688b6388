// Host engine of the GKL solver and the C ABI (include/gkl.h).
//
// The engine owns the device state of one problem (internal copy of the packed
// matrix, column statistics, Krylov bases, projected-matrix scalars) and drives
// the kernels in the order of the Golub-Kahan-Lanczos recurrence (Section 3 of
// the paper):
//     p = A v_j - beta_{j-1} u_{j-1};  reorthogonalise;  alpha_j = ||p||; u_j = p/alpha_j
//     r = A^T u_j - alpha_j v_j;       reorthogonalise;  beta_j  = ||r||; v_{j+1} = r/beta_j
// with full CGS2 or partial reorthogonalisation, convergence tests on the SVD of
// the projected matrix, and thick restarts from the leading ordinary Ritz
// vectors.  Every numerical step runs in a kernel; the host only sequences the
// launches and reads back small control values (breakdown flags, the number of
// converged Ritz values).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"

namespace gkl {

[[noreturn]] void fail(gkl_status s, const std::string& msg) { throw Error{s, msg}; }

void check_hip(hipError_t e, const char* what)
{
    if (e == hipSuccess) return;
    const gkl_status st = (e == hipErrorOutOfMemory) ? GKL_ERR_NOMEM : GKL_ERR_DEVICE;
    fail(st, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Device memory owned by a context
// ---------------------------------------------------------------------------
void* DeviceArena::alloc(size_t bytes)
{
    if (bytes == 0) bytes = 8;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? GKL_ERR_NOMEM : GKL_ERR_DEVICE,
             "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    ptrs.push_back(p);
    total += bytes;
    return p;
}

DeviceArena::~DeviceArena()
{
    for (void* p : ptrs) (void)hipFree(p);
}

// ---------------------------------------------------------------------------
// Problem setup
// ---------------------------------------------------------------------------
void Problem::setup(const uint8_t* G, int64_t n_, int64_t p_, int64_t ld_, hipStream_t s,
                    int products)
{
    n = n_;
    p = p_;
    ld = ld_;
    G_user = G;
    stream = s;
    layout_shape(n, p, packed);
    st.count = static_cast<int64_t*>(arena.alloc(sizeof(int64_t) * p));
    st.nobs = static_cast<int64_t*>(arena.alloc(sizeof(int64_t) * p));
    st.n3 = static_cast<int64_t*>(arena.alloc(sizeof(int64_t) * p));
    st.mean = static_cast<double*>(arena.alloc(sizeof(double) * p));
    st.inv_sd = static_cast<double*>(arena.alloc(sizeof(double) * p));
    bool stats_done = false;
    if (products != 0) {
        // 1: tables for both products, 2: limbs for both, 3: tables for A v and
        // limbs for A^T u
        packed.limb_mv = products == 2;
        packed.limb_rmv = products >= 2;
        if (!packed.limb_mv) packed.T = static_cast<uint8_t*>(arena.alloc(layout_T_bytes(packed)));
        if (!packed.limb_rmv) packed.P = static_cast<uint8_t*>(arena.alloc(layout_P_bytes(packed)));
        build_layouts(G, ld, packed, s);
        if (packed.limb_mv || packed.limb_rmv) {
            packed.ms = mixed_shape(n, p);
            const MixedShape& m = packed.ms;
            uint8_t* I = packed.limb_mv
                             ? static_cast<uint8_t*>(arena.alloc((size_t)m.nI * (size_t)m.ldI))
                             : nullptr;
            uint8_t* S = packed.limb_rmv
                             ? static_cast<uint8_t*>(arena.alloc((size_t)m.pS * (size_t)m.ldS))
                             : nullptr;
            // the pass that builds S also forms the column statistics
            build_mixed_layouts(G, n, p, ld, I, S, s, S ? &st : nullptr);
            stats_done = S != nullptr;
            packed.I = I;
            packed.S = S;
            mvw.lfrag = arena.alloc(limb_frag_bytes(m));
            mvw.lcpart = static_cast<double*>(arena.alloc(sizeof(double) * 64));
            mvw.lcmax = static_cast<double*>(arena.alloc(sizeof(double) * 64));
        }
    }
    if (!stats_done) launch_colstats(G, n, p, ld, st, s);
    if (products == 0) return;
    mvw.partial_elems = matvec_partial_elems(packed);
    mvw.partial = static_cast<double*>(arena.alloc(sizeof(double) * mvw.partial_elems));
    mvw.ncounters = matvec_counters(packed);
    mvw.counters = static_cast<unsigned int*>(arena.alloc(sizeof(unsigned int) * mvw.ncounters));
    mvw.npart = static_cast<double*>(arena.alloc(sizeof(double) * matvec_norm_partials(packed)));
    GKL_HIP(hipMemsetAsync(mvw.counters, 0, sizeof(unsigned int) * mvw.ncounters, s));
}

}  // namespace gkl

using namespace gkl;

// ---------------------------------------------------------------------------
// Solver state
// ---------------------------------------------------------------------------
void gkl_ctx::allocate_solver()
{
    const int64_t n = prob.n, p = prob.p;
    DeviceArena& A = prob.arena;
    const int cols = maxm;
    U = static_cast<double*>(A.alloc(sizeof(double) * (size_t)n * cols));
    V = static_cast<double*>(A.alloc(sizeof(double) * (size_t)p * (cols + 1)));
    const bool harmonic = krylov > 0 && opt.restart == GKL_RESTART_HARMONIC;
    const int keep_alloc = std::max(keep, 1) + (harmonic ? 1 : 0);
    tmp = static_cast<double*>(A.alloc(sizeof(double) * (size_t)std::max(n, p) * keep_alloc));
    if (harmonic) {
        const size_t m1 = (size_t)cols + 1;
        head = static_cast<double*>(A.alloc(sizeof(double) * (size_t)keep * keep));
        hpad = static_cast<double*>(A.alloc(sizeof(double) * m1 * m1));
        hP = static_cast<double*>(A.alloc(sizeof(double) * m1 * m1));
        hQ = static_cast<double*>(A.alloc(sizeof(double) * m1 * m1));
        hS = static_cast<double*>(A.alloc(sizeof(double) * m1));
        hZ = static_cast<double*>(A.alloc(sizeof(double) * m1 * (keep + 1)));
        hwork = static_cast<double*>(A.alloc(sizeof(double) * (size_t)cols * (keep + 1)));
        if (!svd_fits_lds(cols + 1))
            hsvd_scratch = static_cast<double*>(A.alloc(sizeof(double) * svd_scratch_elems(cols + 1)));
    }
    kScalars = 4 * (size_t)(cols + 1) + 2;
    scal = static_cast<double*>(A.alloc(sizeof(double) * kScalars));
    alpha = scal;
    beta = alpha + (cols + 1);
    theta = beta + (cols + 1);
    rho = theta + (cols + 1);
    norm_est = rho + (cols + 1);
    flags = static_cast<int*>(A.alloc(sizeof(int) * 16));
    const size_t mm = (size_t)cols * cols;
    ritz.B = static_cast<double*>(A.alloc(sizeof(double) * mm));
    ritz.P = static_cast<double*>(A.alloc(sizeof(double) * mm));
    ritz.Q = static_cast<double*>(A.alloc(sizeof(double) * mm));
    ritz.S = static_cast<double*>(A.alloc(sizeof(double) * cols));
    ritz.res = static_cast<double*>(A.alloc(sizeof(double) * cols));
    ritz.nconv = flags + 8;
    svd_scratch = svd_fits_lds(cols)
                      ? nullptr
                      : static_cast<double*>(A.alloc(sizeof(double) * svd_scratch_elems(cols)));
    pro.mu = static_cast<double*>(A.alloc(sizeof(double) * (cols + 1)));
    pro.nu = static_cast<double*>(A.alloc(sizeof(double) * (cols + 2)));
    pro.flag_left = flags + 2;
    pro.flag_right = flags + 3;
    pro.force = flags + 4;
    const int64_t maxlen = std::max(n, p);
    ow.partial_elems = ortho_partial_elems(maxlen, cols + 1);
    ow.partial = static_cast<double*>(A.alloc(sizeof(double) * ow.partial_elems));
    ow.counters = static_cast<unsigned int*>(A.alloc(sizeof(unsigned int) * kOrthoCounters));
    ow.h = static_cast<double*>(A.alloc(sizeof(double) * (3 * (size_t)(cols + 2) + 8)));
    ow.tn_partial = static_cast<double*>(A.alloc(sizeof(double) * gemm_tn_partial_elems(maxlen, cols + 1)));
    ow.npart = static_cast<double*>(A.alloc(sizeof(double) * (ceil_div(maxlen, 256) + 1)));
    ow.cgs_partial_elems = cgs_partial_elems(maxlen, cols + 1);
    ow.cgs_partial = static_cast<double*>(A.alloc(sizeof(double) * ow.cgs_partial_elems));
    hipStream_t s = prob.stream;
    GKL_HIP(hipMemsetAsync(ow.counters, 0, sizeof(unsigned int) * kOrthoCounters, s));
    GKL_HIP(hipMemsetAsync(scal, 0, sizeof(double) * kScalars, s));
    GKL_HIP(hipMemsetAsync(flags, 0, sizeof(int) * 16, s));
}

static thread_local std::string g_create_error;

namespace gkl {
void set_create_error(const std::string& msg) { g_create_error = msg; }
}  // namespace gkl

static gkl_status set_error(gkl_ctx* ctx, gkl_status s, const std::string& msg)
{
    if (ctx) ctx->last_error = msg;
    else g_create_error = msg;
    return s;
}

void gkl_ctx::record(int step, bool restart_flag, double res_rel)
{
    if (!opt.trace) return;
    double a = 0.0, b = 0.0;
    int fl[2] = {1, 1};
    GKL_HIP(hipMemcpyAsync(&a, alpha + step, sizeof(double), hipMemcpyDeviceToHost, prob.stream));
    GKL_HIP(hipMemcpyAsync(&b, beta + step, sizeof(double), hipMemcpyDeviceToHost, prob.stream));
    if (reorth == GKL_REORTH_PARTIAL)
        GKL_HIP(hipMemcpyAsync(fl, pro.flag_left, 2 * sizeof(int), hipMemcpyDeviceToHost,
                               prob.stream));
    GKL_HIP(hipStreamSynchronize(prob.stream));
    trace.push_back({(double)step, a, b, (double)fl[0], (double)fl[1], restart_flag ? 1.0 : 0.0,
                     res_rel});
}

int gkl_ctx::read_flag(const int* dflag)
{
    int h = 0;
    GKL_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, prob.stream));
    GKL_HIP(hipStreamSynchronize(prob.stream));
    return h;
}

// Kernel timing: events are taken from a pool that grows on demand and is
// reused across solves; durations are summed after the solve.  With
// options.timing = t, the first of every t launches of each product is
// bracketed (a recorded event costs the stream a few microseconds).
int gkl_ctx::timing_slot(bool right)
{
    if (opt.timing <= 0) return -1;
    if (ev_calls[right ? 1 : 0]++ % opt.timing != 0) return -1;
    if (ev_next + 4 > (int)ev_pool.size()) {
        for (int t = 0; t < 64; ++t) {
            hipEvent_t e;
            GKL_HIP(hipEventCreate(&e));
            ev_pool.push_back(e);
        }
    }
    // four events per slot: the product (start, end) and, for products made of
    // several launches, the main kernel alone (start, end)
    const int i = ev_next;
    ev_next += 4;
    return i;
}

const hipEvent_t* gkl_ctx::timing_events(int slot)
{
    return slot < 0 ? nullptr : &ev_pool[slot];
}

void gkl_ctx::timing_note(int slot, bool right, bool core)
{
    if (slot >= 0) (right ? ev_rmv : ev_mv).push_back({slot, core ? slot + 2 : slot});
}

int gkl_ctx::timing_begin(bool right)
{
    const int i = timing_slot(right);
    if (i >= 0) GKL_HIP(hipEventRecord(ev_pool[i], prob.stream));
    return i;
}

void gkl_ctx::timing_end(int start, bool right, bool core)
{
    if (start < 0) return;
    GKL_HIP(hipEventRecord(ev_pool[start + 1], prob.stream));
    timing_note(start, right, core);
}

void gkl_ctx::timing_collect()
{
    if (!opt.timing) return;
    GKL_HIP(hipStreamSynchronize(prob.stream));
    // pr = (slot, core slot): the product spans events slot, slot + 1; its main
    // kernel spans core, core + 1 (the same pair when the product is one kernel)
    double t[2] = {0.0, 0.0}, c[2] = {0.0, 0.0};
    for (int side = 0; side < 2; ++side) {
        for (auto& pr : side ? ev_rmv : ev_mv) {
            float ms = 0.f, mc = 0.f;
            GKL_HIP(hipEventElapsedTime(&ms, ev_pool[pr.first], ev_pool[pr.first + 1]));
            GKL_HIP(hipEventElapsedTime(&mc, ev_pool[pr.second], ev_pool[pr.second + 1]));
            t[side] += ms;
            c[side] += mc;
        }
    }
    info.matvec_kernel_ms = t[0];
    info.rmatvec_kernel_ms = t[1];
    info.matvec_core_ms = c[0];
    info.rmatvec_core_ms = c[1];
    info.timed_matvecs = (int64_t)ev_mv.size();
    info.timed_rmatvecs = (int64_t)ev_rmv.size();
    ev_mv.clear();
    ev_rmv.clear();
    ev_next = 0;
    ev_calls[0] = ev_calls[1] = 0;
}

// Left half-step j: U(:, j) from v_j.  Nothing is read back: a breakdown is
// recorded on the device (first half-step index) and handled at the next
// synchronisation point.
void gkl_ctx::left_step(int j)
{
    hipStream_t s = prob.stream;
    const int64_t n = prob.n, p = prob.p;
    double* uj = U + (int64_t)j * n;
    const double* vj = V + (int64_t)j * p;
    const int ev = timing_slot(false);
    const hipEvent_t* evs = timing_events(ev);
    const bool pro_on = j > 0 && reorth == GKL_REORTH_PARTIAL;
    bool pro_done = false;
    if (j > 0 && j == nlock) {
        launch_matvec(prob.packed, prob.st, vj, uj, nullptr, nullptr, prob.mvw, s, nullptr, evs);
        launch_gemv_n_sub(U, n, n, nlock, rho, uj, s);
    } else if (j > 0) {
        // alpha_j and the PRO update come with the product
        const NormTail tail = pro_tail(alpha + j, 1, j);
        launch_matvec(prob.packed, prob.st, vj, uj, beta + (j - 1), U + (int64_t)(j - 1) * n,
                      prob.mvw, s, pro_on ? &tail : nullptr, evs);
        pro_done = pro_on;
    } else {
        launch_matvec(prob.packed, prob.st, vj, uj, nullptr, nullptr, prob.mvw, s, nullptr, evs);
    }
    timing_note(ev, false);
    info.matvecs += 1;
    info.passes_over_G += 1;
    const int* gate = nullptr;
    if (j > 0) {
        if (pro_on) {
            if (!pro_done) {
                launch_normalize_only(uj, n, alpha + j);
                launch_pro_left(pro_args(j), s);
            }
            gate = pro.flag_left;
        } else if (long_side_free(0)) {
            gate = long_side_check(U, n, j, uj, alpha + j);
        }
        launch_cgs2(U, n, n, j, uj, gate, opt.adaptive_cgs2, flags + 6, ow, s);
    }
    if (j > 0 && !opt.adaptive_cgs2)
        launch_normalize_after_cgs2(uj, n, alpha + j, norm_est, root_maxdim, flags + 0, gate, ow, s,
                                    flags + 9, 2 * j);
    else
        launch_normalize(uj, n, uj, alpha + j, norm_est, root_maxdim, flags + 0, ow, s, flags + 9,
                         2 * j);
}

// Right half-step j: V(:, j+1) from u_j.
void gkl_ctx::right_step(int j)
{
    hipStream_t s = prob.stream;
    const int64_t n = prob.n, p = prob.p;
    const double* uj = U + (int64_t)j * n;
    double* vn = V + (int64_t)(j + 1) * p;
    const int ev = timing_slot(true);
    const bool pro_on = reorth == GKL_REORTH_PARTIAL;
    const NormTail tail = pro_tail(beta + j, 2, j);   // beta_j and the PRO update
    launch_rmatvec(prob.packed, prob.st, uj, vn, alpha + j, V + (int64_t)j * p, prob.mvw, s,
                   pro_on ? &tail : nullptr, timing_events(ev));
    timing_note(ev, true);
    info.matvecs += 1;
    info.passes_over_G += 1;
    const int* gate = pro_on ? pro.flag_right : nullptr;
    if (long_side_free(1)) gate = long_side_check(V, p, j + 1, vn, beta + j);
    launch_cgs2(V, p, p, j + 1, vn, gate, opt.adaptive_cgs2, flags + 6, ow, s);
    if (!opt.adaptive_cgs2)
        launch_normalize_after_cgs2(vn, p, beta + j, norm_est, root_maxdim, flags + 1, gate, ow, s,
                                    flags + 9, 2 * j + 1);
    else
        launch_normalize(vn, p, vn, beta + j, norm_est, root_maxdim, flags + 1, ow, s, flags + 9,
                         2 * j + 1);
}

ProArgs gkl_ctx::pro_args(int j) const
{
    ProArgs a;
    a.alpha = alpha;
    a.beta = beta;
    a.theta = theta;
    a.rho = rho;
    a.nlock = nlock;
    a.j = j;
    a.omega = omega;
    a.noise_scale = noise_scale;
    a.norm_est = norm_est;
    a.st = pro;
    return a;
}

NormTail gkl_ctx::pro_tail(double* nrm_out, int side, int j) const
{
    NormTail t{};
    t.nrm_out = nrm_out;
    t.pro = side;
    t.pa = pro_args(j);
    return t;
}

// Reads the number of converged Ritz values and the first breakdown half-step
// (-1 if none) in one copy.
void gkl_ctx::sync_state(int* nconv, int* breakdown)
{
    int h[3] = {0, -1, 0};
    GKL_HIP(hipMemcpyAsync(h, flags + 8, 3 * sizeof(int), hipMemcpyDeviceToHost, prob.stream));
    GKL_HIP(hipStreamSynchronize(prob.stream));
    *nconv = h[0];
    *breakdown = h[1];
    if (reorth == GKL_REORTH_ONESIDED && h[2] && !two_sided) two_sided = true;
}

// One-sided reorthogonalisation (Section 3, "Choice of reorthogonalization
// strategy"): the longer side's Gram-Schmidt is skipped while its basis stays
// orthogonal.  True until the device's overlap flag has been read back set.
bool gkl_ctx::long_side_free(int side) const
{
    return reorth == GKL_REORTH_ONESIDED && !two_sided && side != short_side;
}

// The longer side's new (unnormalised) vector r against Q(:, 0:ncols): ||r|| into
// *nrm (what the normalisation uses when Gram-Schmidt is skipped) and the sticky
// flag set when the largest overlap exceeds onesided_tol() ||r||.  Returns the
// flag, which then gates this and every later Gram-Schmidt of that side on the
// device -- no read-back in the step.
const int* gkl_ctx::long_side_check(const double* Q, int64_t len, int ncols, const double* r,
                                    double* nrm)
{
    launch_norm(r, len, nrm, ow, prob.stream);
    launch_overlap_check(Q, len, ncols, r, onesided_tol(), nrm, flags + 10, ow, prob.stream);
    return flags + 10;
}

// A loss of orthogonality eta in the unreorthogonalised basis moves the Ritz
// values (and the norms of the Ritz vectors formed from that basis) by about
// eta relative, to first order: the threshold is the smaller of omega and the
// convergence tolerance.
double gkl_ctx::onesided_tol() const
{
    return std::min(omega, tol);
}

// ||r|| into *out without scaling (PRO needs alpha_j / beta_j before deciding).
void gkl_ctx::launch_normalize_only(double* r, int64_t len, double* out)
{
    // norm into out; flag ignored; scaling skipped because nrm_out is written
    // with the norm and the scale kernel would divide -- so use a scratch copy
    launch_norm(r, len, out, ow, prob.stream);
}

// Breakdown: the new vector has (numerically) no component outside the current
// basis.  Record a zero scalar and continue with a random direction made
// orthogonal to the basis (or stop if the basis already spans the space).
void gkl_ctx::handle_breakdown(bool left, int j)
{
    hipStream_t s = prob.stream;
    const int64_t len = left ? prob.n : prob.p;
    const int ncols = left ? j : j + 1;
    double* Q = left ? U : V;
    double* r = left ? U + (int64_t)j * prob.n : V + (int64_t)(j + 1) * prob.p;
    double* scalar = left ? alpha + j : beta + j;
    if (ncols >= len) {
        exhausted = true;
        return;
    }
    for (int attempt = 0; attempt < 3; ++attempt) {
        launch_gaussian(r, len, opt.seed ^ 0xB4EA4D0ull, (uint64_t)(breakdown_draws++), s);
        launch_cgs2(Q, len, len, ncols, r, nullptr, 0, flags + 6, ow, s);
        double* tmp_nrm = ow.h + 3 * (maxm + 2) + 4;
        launch_normalize(r, len, r, tmp_nrm, norm_est, root_maxdim, flags + 7, ow, s);
        if (!read_flag(flags + 7)) {
            GKL_HIP(hipMemsetAsync(scalar, 0, sizeof(double), s));
            info.reorths += 1;
            if (reorth == GKL_REORTH_PARTIAL) launch_pro_reset(pro, maxm, 2, s);
            return;
        }
    }
    fail(GKL_ERR_BREAKDOWN, "Lanczos breakdown: no new direction orthogonal to the basis");
}

int gkl_ctx::check_convergence(int m)
{
    launch_ritz(alpha, beta, theta, rho, nlock, m, k, tol, ritz, svd_scratch, prob.stream,
                head_dense ? head : nullptr);
    ritz_m = m;
    int nconv = 0, bd = -1;
    sync_state(&nconv, &bd);
    last_breakdown = bd;
    return nconv;
}

void gkl_ctx::restart(int m)
{
    hipStream_t s = prob.stream;
    const int64_t n = prob.n, p = prob.p;
    if (ritz_m != m) check_convergence(m);
    if (opt.restart == GKL_RESTART_HARMONIC && !zero_scalar) {
        restart_harmonic(m);
        return;
    }
    zero_scalar = false;
    head_dense = false;
    // V(:, 0:l) = V(:, 0:m) Q(:, 0:l); v_l = v_m
    launch_gemm_tall(V, p, p, m, ritz.Q, m, keep, tmp, p, s);
    GKL_HIP(hipMemcpyAsync(V, tmp, sizeof(double) * (size_t)p * keep, hipMemcpyDeviceToDevice, s));
    GKL_HIP(hipMemcpyAsync(V + (int64_t)keep * p, V + (int64_t)m * p, sizeof(double) * (size_t)p,
                           hipMemcpyDeviceToDevice, s));
    // U(:, 0:l) = U(:, 0:m) P(:, 0:l)
    launch_gemm_tall(U, n, n, m, ritz.P, m, keep, tmp, n, s);
    GKL_HIP(hipMemcpyAsync(U, tmp, sizeof(double) * (size_t)n * keep, hipMemcpyDeviceToDevice, s));
    launch_restart_scalars(ritz.S, ritz.P, m, beta + (m - 1), keep, theta, rho, s);
    nlock = keep;
    ritz_m = -1;
    info.restarts += 1;
    if (reorth == GKL_REORTH_PARTIAL) launch_pro_reset(pro, maxm, 2, s);
}

// Thick restart from harmonic Ritz vectors (the small-space plan is built in
// one workgroup from the SVD of [B_m, beta_m e_m]): V(:, 0:l+1) = V(:, 0:m+1) Z,
// U(:, 0:l) = U(:, 0:m) Ph(0:m, 0:l); the projected matrix restarts with the
// dense head and the coupling column rho.
void gkl_ctx::restart_harmonic(int m)
{
    hipStream_t s = prob.stream;
    const int64_t n = prob.n, p = prob.p;
    const int l = keep, m1 = m + 1;
    launch_harmonic_pad(ritz.B, m, beta + (m - 1), hpad, s);
    launch_dense_svd(hpad, m1, hP, hS, hQ, hsvd_scratch, s);
    launch_harmonic_plan(ritz.B, m, beta + (m - 1), hP, hQ, l, hwork, hZ, head, rho, s);
    launch_gemm_tall(V, p, p, m1, hZ, m1, l + 1, tmp, p, s);
    GKL_HIP(hipMemcpyAsync(V, tmp, sizeof(double) * (size_t)p * (l + 1), hipMemcpyDeviceToDevice, s));
    launch_gemm_tall(U, n, n, m, hP, m1, l, tmp, n, s);
    GKL_HIP(hipMemcpyAsync(U, tmp, sizeof(double) * (size_t)n * l, hipMemcpyDeviceToDevice, s));
    head_dense = true;
    nlock = l;
    ritz_m = -1;
    info.restarts += 1;
}

void gkl_ctx::finalize(int m, double* sigma, double* Uo, int64_t ldu, double* Vo, int64_t ldv)
{
    hipStream_t s = prob.stream;
    const int64_t n = prob.n, p = prob.p;
    if (ritz_m != m) check_convergence(m);
    const int kk = std::min(k, m);
    GKL_HIP(hipMemcpyAsync(sigma, ritz.S, sizeof(double) * kk, hipMemcpyDeviceToDevice, s));
    launch_gemm_tall(U, n, n, m, ritz.P, m, kk, Uo, ldu, s);
    launch_gemm_tall(V, p, p, m, ritz.Q, m, kk, Vo, ldv, s);
    if (reorth == GKL_REORTH_ONESIDED) {
        // the long side's basis was not kept orthogonal: its Ritz vectors are
        // formed from the short side's, v_i = A^T u_i / ||A^T u_i|| (or
        // u_i = A v_i / ||A v_i||); one product per vector
        double* scratch_nrm = ow.h;
        for (int i = 0; i < kk; ++i) {
            double* uo = Uo + (int64_t)i * ldu;
            double* vo = Vo + (int64_t)i * ldv;
            if (short_side == 0) {
                launch_rmatvec(prob.packed, prob.st, uo, vo, nullptr, nullptr, prob.mvw, s, nullptr,
                               nullptr);
                launch_normalize(vo, p, vo, scratch_nrm, norm_est, root_maxdim, flags + 7, ow, s);
            } else {
                launch_matvec(prob.packed, prob.st, vo, uo, nullptr, nullptr, prob.mvw, s, nullptr,
                              nullptr);
                launch_normalize(uo, n, uo, scratch_nrm, norm_est, root_maxdim, flags + 7, ow, s);
            }
            info.matvecs += 1;
            info.passes_over_G += 1;
        }
    }
    launch_sign_fix(Uo, ldu, n, Vo, ldv, p, kk, s);
    std::vector<double> res(kk), sig(1);
    GKL_HIP(hipMemcpyAsync(res.data(), ritz.res, sizeof(double) * kk, hipMemcpyDeviceToHost, s));
    GKL_HIP(hipMemcpyAsync(sig.data(), ritz.S, sizeof(double), hipMemcpyDeviceToHost, s));
    GKL_HIP(hipStreamSynchronize(s));
    double sum = 0.0, mx = 0.0;
    for (int i = 0; i < kk; ++i) {
        sum += res[i];
        mx = std::max(mx, sig[0] > 0 ? res[i] / sig[0] : 0.0);
    }
    info.sum_residual_est = sum;
    info.max_residual_rel = mx;
}

gkl_status gkl_ctx::solve_fp64(double* sigma, double* Uo, int64_t ldu, double* Vo, int64_t ldv)
{
    hipStream_t s = prob.stream;
    const int64_t p = prob.p;
    // start vector
    if (opt.v0) GKL_HIP(hipMemcpyAsync(V, opt.v0, sizeof(double) * p, hipMemcpyDeviceToDevice, s));
    else launch_gaussian(V, p, opt.seed, 0, s);
    GKL_HIP(hipMemsetAsync(scal, 0, sizeof(double) * kScalars, s));
    GKL_HIP(hipMemsetAsync(flags + 9, 0xFF, sizeof(int), s));   // first breakdown = -1
    GKL_HIP(hipMemsetAsync(flags + 10, 0, sizeof(int), s));     // long side lost orthogonality
    two_sided = false;
    launch_normalize(V, p, V, tmp, norm_est, root_maxdim, flags + 1, ow, s);
    GKL_HIP(hipMemsetAsync(norm_est, 0, sizeof(double), s));
    if (reorth == GKL_REORTH_PARTIAL) launch_pro_reset(pro, maxm, 0, s);
    nlock = 0;
    ritz_m = -1;
    head_dense = false;
    zero_scalar = false;
    exhausted = false;
    breakdown_draws = 1;
    last_breakdown = -1;
    int j = 0;
    int last_check = 0;
    int nconv = 0;
    const int64_t maxbasis = std::min(prob.n, prob.p);
    // Convergence tests: every check_every steps if given; with thick restart when
    // the basis is full; without restart every 5 steps until the basis holds 20
    // vectors, then whenever it has grown by a quarter -- the projected SVD costs
    // O(j^3), so testing at a fixed interval would make it dominate large bases
    const int check_every = opt.check_every > 0 ? opt.check_every : (krylov > 0 ? 0 : 5);
    const bool grow_checks = opt.check_every <= 0 && krylov == 0;
    bool converged = false;
    while (true) {
        left_step(j);
        right_step(j);
        ++j;
        const bool budget = opt.max_matvecs > 0 && info.matvecs >= opt.max_matvecs;
        const bool full = (j == maxm) || (j >= maxbasis);
        const int every = grow_checks ? std::max(check_every, last_check / 4) : check_every;
        const bool due = j >= k && (full || (every > 0 && j - last_check >= every));
        if (opt.trace) record(j - 1, false, NAN);
        if (!(due || budget || full)) continue;
        nconv = j >= k ? check_convergence(j) : 0;
        if (j < k) {
            int dummy = 0;
            sync_state(&dummy, &last_breakdown);
        }
        last_check = j;
        if (last_breakdown >= 0) {
            // roll back to the half-step that broke down and continue from there
            const int hb = last_breakdown;
            const int jb = hb / 2;
            GKL_HIP(hipMemsetAsync(flags + 9, 0xFF, sizeof(int), s));
            last_breakdown = -1;
            ritz_m = -1;
            zero_scalar = true;
            if (hb % 2 == 0) {
                handle_breakdown(true, jb);
                if (exhausted) { j = jb; break; }
                right_step(jb);
            } else {
                handle_breakdown(false, jb);
                if (exhausted) { j = jb + 1; break; }
            }
            j = jb + 1;
            last_check = std::min(last_check, j);
            if (opt.trace) {
                while (!trace.empty() && trace.back()[0] >= jb) trace.pop_back();
                record(jb, false, NAN);
            }
            continue;
        }
        info.nconv = nconv;
        if (opt.trace && j >= k && !trace.empty()) {
            double s0 = 0.0;
            std::vector<double> res(k);
            GKL_HIP(hipMemcpy(&s0, ritz.S, sizeof(double), hipMemcpyDeviceToHost));
            GKL_HIP(hipMemcpy(res.data(), ritz.res, sizeof(double) * k, hipMemcpyDeviceToHost));
            double r = 0.0;
            for (int i = 0; i < k; ++i) r = std::max(r, s0 > 0 ? res[i] / s0 : 0.0);
            trace.back()[6] = r;
        }
        if (nconv >= k) { converged = true; break; }
        if (budget || j >= maxbasis) break;
        if (j == maxm) {
            if (krylov > 0) {
                restart(j);
                j = nlock;
                last_check = j;
                if (opt.trace && !trace.empty()) trace.back()[5] = 1.0;
            } else {
                break;
            }
        }
    }
    info.steps = j;
    finalize(j, sigma, Uo, ldu, Vo, ldv);
    int passes = 0;
    GKL_HIP(hipMemcpy(&passes, flags + 6, sizeof(int), hipMemcpyDeviceToHost));
    info.reorths += passes;
    info.converged = converged ? 1 : 0;
    info.nconv = converged ? k : nconv;
    return converged ? GKL_OK : GKL_NOT_CONVERGED;
}

gkl_ctx::~gkl_ctx()
{
    gkl::destroy_mixed(mixed);
    gkl::destroy_batch(batch);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void gkl_options_default(gkl_options* o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(gkl_options);
    o->pro_omega = 1e-8;
    o->block_width = 0;
    o->adaptive_cgs2 = 0;
    o->graph = 1;
    o->seed = 0x5EEDull;
}

const char* gkl_status_string(gkl_status s)
{
    switch (s) {
    case GKL_OK: return "ok";
    case GKL_ERR_INVALID: return "invalid argument";
    case GKL_ERR_NOMEM: return "out of device memory";
    case GKL_ERR_DEVICE: return "device error";
    case GKL_NOT_CONVERGED: return "not converged";
    case GKL_ERR_BREAKDOWN: return "Lanczos breakdown";
    case GKL_ERR_INTERNAL: return "internal error";
    case GKL_ERR_UNSUPPORTED: return "unsupported option combination";
    }
    return "unknown status";
}

const char* gkl_last_error(const gkl_ctx* ctx)
{
    return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

gkl_status gkl_create(const uint8_t* G, int64_t n, int64_t p, int32_t k, double tol,
                      int32_t reorth, gkl_ctx** out)
{
    gkl_options o;
    gkl_options_default(&o);
    return gkl_create_ex(G, n, p, k, tol, reorth, &o, out);
}

// Product format of an FP64 context: 1 = lookup tables, 2 = int8 limbs.
static int fp64_products_for(int64_t n, int64_t p, int32_t choice)
{
    if (choice == GKL_FP64_LUT) return 1;
    if (choice == GKL_FP64_LIMBS) return 2;
    if (choice == GKL_FP64_LUT_LIMBS) return 3;
    // GKL_FP64_AUTO: from 1e9 genotypes (250 MB packed) on, both products on the
    // int8 matrix cores (50,000 x 500,000: A v 1.13 ms against 1.29 ms from the
    // tables, A^T u 1.14 ms against 2.09 ms; 10,000 x 100,000: a solve of 720
    // products 94 ms against 97 ms); below that the tables, which need no
    // quantisation kernels per product
    return (double)n * (double)p >= 1e9 ? 2 : 1;
}

static gkl_status validate(const uint8_t* G, int64_t n, int64_t p, int32_t k, double tol,
                           int32_t reorth, const gkl_options* o, gkl_ctx** out)
{
    if (!out) return set_error(nullptr, GKL_ERR_INVALID, "out is NULL");
    if (!G) return set_error(nullptr, GKL_ERR_INVALID, "G is NULL");
    if (!o) return set_error(nullptr, GKL_ERR_INVALID, "options is NULL");
    if (o->struct_size != sizeof(gkl_options))
        return set_error(nullptr, GKL_ERR_INVALID, "options.struct_size mismatch (ABI version)");
    if (n < 1 || p < 1) return set_error(nullptr, GKL_ERR_INVALID, "n and p must be >= 1");
    if (k < 1 || (int64_t)k > std::min(n, p))
        return set_error(nullptr, GKL_ERR_INVALID, "k must lie in [1, min(n, p)]");
    if (!(tol > 0.0) || !isfinite(tol)) return set_error(nullptr, GKL_ERR_INVALID, "tol must be > 0");
    if (reorth != GKL_REORTH_FULL && reorth != GKL_REORTH_PARTIAL && reorth != GKL_REORTH_ONESIDED)
        return set_error(nullptr, GKL_ERR_INVALID,
                         "reorth must be GKL_REORTH_FULL, _PARTIAL or _ONESIDED");
    if (o->krylov_dim < 0 || (o->krylov_dim > 0 && o->krylov_dim <= k))
        return set_error(nullptr, GKL_ERR_INVALID, "krylov_dim must be 0 or > k");
    if (o->krylov_dim > kMaxSvd) return set_error(nullptr, GKL_ERR_INVALID, "krylov_dim too large");
    if (o->keep < 0 || (o->krylov_dim > 0 && o->keep > 0 && (o->keep < k || o->keep >= o->krylov_dim)))
        return set_error(nullptr, GKL_ERR_INVALID, "keep must lie in [k, krylov_dim)");
    if (o->ld_bytes != 0 && o->ld_bytes < (n + 3) / 4)
        return set_error(nullptr, GKL_ERR_INVALID, "ld_bytes < ceil(n/4)");
    if (o->precision != GKL_PREC_FP64 && o->precision != GKL_PREC_MIXED &&
        o->precision != GKL_PREC_MIXED_INT8 && o->precision != GKL_PREC_BLOCK_FP64)
        return set_error(nullptr, GKL_ERR_INVALID, "unknown precision");
    if (o->block_width < 0 || o->block_width > 32)
        return set_error(nullptr, GKL_ERR_INVALID, "block_width must lie in [0, 32]");
    if (o->max_steps < 0 || o->max_steps > kMaxSvd || o->check_every < 0 || o->max_matvecs < 0)
        return set_error(nullptr, GKL_ERR_INVALID, "bad max_steps / check_every / max_matvecs");
    if (o->pro_omega < 0.0) return set_error(nullptr, GKL_ERR_INVALID, "pro_omega must be >= 0");
    if (o->fp64_products < GKL_FP64_AUTO || o->fp64_products > GKL_FP64_LUT_LIMBS)
        return set_error(nullptr, GKL_ERR_INVALID, "unknown fp64_products");
    if (reorth == GKL_REORTH_ONESIDED && o->precision != GKL_PREC_FP64)
        return set_error(nullptr, GKL_ERR_UNSUPPORTED,
                         "one-sided reorthogonalisation is built for the FP64 path only");
    if (o->restart != GKL_RESTART_RITZ && o->restart != GKL_RESTART_HARMONIC)
        return set_error(nullptr, GKL_ERR_INVALID, "restart must be GKL_RESTART_RITZ or _HARMONIC");
    if (o->restart == GKL_RESTART_HARMONIC &&
        (o->precision != GKL_PREC_FP64 || reorth != GKL_REORTH_FULL))
        return set_error(nullptr, GKL_ERR_UNSUPPORTED,
                         "harmonic restarts are built for GKL_PREC_FP64 with GKL_REORTH_FULL");
    return GKL_OK;
}

gkl_status gkl_create_ex(const uint8_t* G, int64_t n, int64_t p, int32_t k, double tol,
                         int32_t reorth, const gkl_options* o, gkl_ctx** out)
{
    gkl_status v = validate(G, n, p, k, tol, reorth, o, out);
    if (v != GKL_OK) return v;
    const bool blocked = o->precision != GKL_PREC_FP64;
    if (blocked && !gkl::mixed_supported())
        return set_error(nullptr, GKL_ERR_UNSUPPORTED, "mixed precision path not built");
    gkl_ctx* ctx = nullptr;
    try {
        auto t0 = std::chrono::steady_clock::now();
        ctx = new gkl_ctx();
        ctx->opt = *o;
        ctx->k = k;
        ctx->tol = tol;
        ctx->reorth = reorth;
        ctx->short_side = n <= p ? 0 : 1;
        ctx->omega = o->pro_omega > 0.0 ? o->pro_omega : 1e-8;
        hipStream_t s = static_cast<hipStream_t>(o->stream);
        const int64_t ld = o->ld_bytes ? o->ld_bytes : (n + 3) / 4;
        ctx->prob.setup(G, n, p, ld, s, blocked ? 0 : fp64_products_for(n, p, o->fp64_products));
        ctx->root_maxdim = sqrt((double)std::max(n, p));
        ctx->noise_scale = 2.220446049250313e-16 * ctx->root_maxdim;
        ctx->krylov = o->krylov_dim;
        const int64_t mn = std::min(n, p);
        if (ctx->krylov > 0) {
            ctx->maxm = (int)std::min<int64_t>(ctx->krylov, mn);
            ctx->keep = o->keep > 0 ? o->keep : k + (ctx->krylov - k) / 2;
            ctx->keep = std::min(ctx->keep, ctx->maxm - 1);
            if (ctx->maxm <= k) ctx->krylov = 0;   // the whole space fits: no restart needed
        } else {
            ctx->maxm = (int)std::min<int64_t>(o->max_steps > 0 ? o->max_steps : 512, mn);
            ctx->keep = 0;
        }
        if (ctx->maxm < k) fail(GKL_ERR_INVALID, "basis smaller than k");
        if (blocked) ctx->setup_mixed();
        else ctx->allocate_solver();
        GKL_HIP(hipStreamSynchronize(s));
        ctx->create_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = ctx;
        return GKL_OK;
    } catch (const Error& e) {
        delete ctx;
        return set_error(nullptr, e.status, e.msg);
    } catch (const std::bad_alloc&) {
        delete ctx;
        return set_error(nullptr, GKL_ERR_NOMEM, "host allocation failed");
    } catch (...) {
        delete ctx;
        return set_error(nullptr, GKL_ERR_INTERNAL, "unexpected exception in gkl_create");
    }
}

gkl_status gkl_solve(gkl_ctx* ctx, double* sigma, double* U, int64_t ldu, double* V, int64_t ldv,
                     gkl_info* info)
{
    if (!ctx) return set_error(nullptr, GKL_ERR_INVALID, "ctx is NULL");
    if (ctx->batched) return set_error(ctx, GKL_ERR_INVALID, "use gkl_solve_batched for this ctx");
    if (!sigma || !U || !V) return set_error(ctx, GKL_ERR_INVALID, "NULL output pointer");
    if (ldu < ctx->prob.n || ldv < ctx->prob.p)
        return set_error(ctx, GKL_ERR_INVALID, "ldu < n or ldv < p");
    try {
        auto t0 = std::chrono::steady_clock::now();
        ctx->info = gkl_info{};
        ctx->trace.clear();
        gkl_status st = ctx->opt.precision != GKL_PREC_FP64
                            ? ctx->solve_mixed(sigma, U, ldu, V, ldv)
                            : ctx->solve_fp64(sigma, U, ldu, V, ldv);
        GKL_HIP(hipStreamSynchronize(ctx->prob.stream));
        ctx->info.solve_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        ctx->info.create_ms = ctx->create_ms;
        if (ctx->opt.precision == GKL_PREC_FP64)
            ctx->info.fp64_products = ctx->prob.packed.limb_mv    ? GKL_FP64_LIMBS
                                      : ctx->prob.packed.limb_rmv ? GKL_FP64_LUT_LIMBS
                                                                  : GKL_FP64_LUT;
        ctx->timing_collect();
        if (info) *info = ctx->info;
        if (st == GKL_NOT_CONVERGED) ctx->last_error = "tolerance not met within the matvec budget";
        return st;
    } catch (const Error& e) {
        return set_error(ctx, e.status, e.msg);
    } catch (...) {
        return set_error(ctx, GKL_ERR_INTERNAL, "unexpected exception in gkl_solve");
    }
}

void gkl_destroy(gkl_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->prob.stream);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

gkl_status gkl_column_stats(gkl_ctx* ctx, int64_t* count, int64_t* nobs, double* mean,
                            double* inv_sd)
{
    if (!ctx || ctx->batched) return set_error(ctx, GKL_ERR_INVALID, "bad ctx");
    try {
        hipStream_t s = ctx->prob.stream;
        const size_t p = (size_t)ctx->prob.p;
        const ColStats& st = ctx->prob.st;
        if (count) GKL_HIP(hipMemcpyAsync(count, st.count, 8 * p, hipMemcpyDeviceToDevice, s));
        if (nobs) GKL_HIP(hipMemcpyAsync(nobs, st.nobs, 8 * p, hipMemcpyDeviceToDevice, s));
        if (mean) GKL_HIP(hipMemcpyAsync(mean, st.mean, 8 * p, hipMemcpyDeviceToDevice, s));
        if (inv_sd) GKL_HIP(hipMemcpyAsync(inv_sd, st.inv_sd, 8 * p, hipMemcpyDeviceToDevice, s));
        GKL_HIP(hipStreamSynchronize(s));
        return GKL_OK;
    } catch (const Error& e) {
        return set_error(ctx, e.status, e.msg);
    }
}

gkl_status gkl_unpack(gkl_ctx* ctx, int8_t* out)
{
    if (!ctx || ctx->batched || !out) return set_error(ctx, GKL_ERR_INVALID, "bad argument");
    try {
        hipStream_t s = ctx->prob.stream;
        launch_unpack(ctx->prob.G_user, ctx->prob.n, ctx->prob.p, ctx->prob.ld, out, s);
        GKL_HIP(hipStreamSynchronize(s));
        return GKL_OK;
    } catch (const Error& e) {
        return set_error(ctx, e.status, e.msg);
    }
}

gkl_status gkl_matvec(gkl_ctx* ctx, const double* v, double* y)
{
    if (!ctx || ctx->batched || !v || !y) return set_error(ctx, GKL_ERR_INVALID, "bad argument");
    if (ctx->opt.precision != GKL_PREC_FP64 || ctx->batched)
        return set_error(ctx, GKL_ERR_INVALID, "FP64 products need an FP64 context");
    try {
        hipStream_t s = ctx->prob.stream;
        const int ev = ctx->timing_slot(false);
        launch_matvec(ctx->prob.packed, ctx->prob.st, v, y, nullptr, nullptr, ctx->prob.mvw, s,
                      nullptr, ctx->timing_events(ev));
        ctx->timing_note(ev, false);
        GKL_HIP(hipStreamSynchronize(s));
        return GKL_OK;
    } catch (const Error& e) {
        return set_error(ctx, e.status, e.msg);
    }
}

gkl_status gkl_rmatvec(gkl_ctx* ctx, const double* u, double* z)
{
    if (!ctx || ctx->batched || !u || !z) return set_error(ctx, GKL_ERR_INVALID, "bad argument");
    if (ctx->opt.precision != GKL_PREC_FP64 || ctx->batched)
        return set_error(ctx, GKL_ERR_INVALID, "FP64 products need an FP64 context");
    try {
        hipStream_t s = ctx->prob.stream;
        const int ev = ctx->timing_slot(true);
        launch_rmatvec(ctx->prob.packed, ctx->prob.st, u, z, nullptr, nullptr, ctx->prob.mvw, s,
                       nullptr, ctx->timing_events(ev));
        ctx->timing_note(ev, true);
        GKL_HIP(hipStreamSynchronize(s));
        return GKL_OK;
    } catch (const Error& e) {
        return set_error(ctx, e.status, e.msg);
    }
}

gkl_status gkl_get_trace(gkl_ctx* ctx, double* buf, int64_t cap, int64_t* written)
{
    if (!ctx || !written || (cap > 0 && !buf)) return set_error(ctx, GKL_ERR_INVALID, "bad argument");
    const int64_t rows = std::min<int64_t>((int64_t)ctx->trace.size(), cap / GKL_TRACE_FIELDS);
    for (int64_t r = 0; r < rows; ++r)
        for (int f = 0; f < GKL_TRACE_FIELDS; ++f) buf[r * GKL_TRACE_FIELDS + f] = ctx->trace[r][f];
    *written = rows;
    return GKL_OK;
}

gkl_status gkl_dense_svd(const double* B, int32_t m, double* P, double* S, double* Q, void* stream)
{
    if (!B || !P || !S || !Q || m < 1 || m > kMaxSvd)
        return set_error(nullptr, GKL_ERR_INVALID, "bad argument to gkl_dense_svd");
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        double* gscr = nullptr;
        double* rlog = nullptr;
        if (!svd_fits_lds(m)) {
            if (svd_logged_fits_lds(m))
                GKL_HIP(hipMalloc(&rlog, sizeof(double) * svd_log_elems(m)));
            else
                GKL_HIP(hipMalloc(&gscr, sizeof(double) * svd_scratch_elems(m)));
        }
        try {
            launch_dense_svd(B, m, P, S, Q, gscr, s, rlog);
            GKL_HIP(hipStreamSynchronize(s));
        } catch (...) {
            if (gscr) (void)hipFree(gscr);
            if (rlog) (void)hipFree(rlog);
            throw;
        }
        if (gscr) GKL_HIP(hipFree(gscr));
        if (rlog) GKL_HIP(hipFree(rlog));
        return GKL_OK;
    } catch (const Error& e) {
        return set_error(nullptr, e.status, e.msg);
    }
}

// ---------------------------------------------------------------------------
// gkl_dense_svd_noalloc: the same SVD with its working memory in a file-scope
// device array instead of a hipMalloc'ed buffer.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
// Largest m taken by gkl_dense_svd_noalloc and the scratch it may need: the
// rotation log of the in-LDS path for 96 < m <= 128 (svd_log_elems(128) =
// 650,240 doubles) or the working matrices of the global path for
// 128 < m <= 256 (about 135,000 doubles); 5 MiB covers both.
constexpr int kNoAllocMaxM = GKL_DENSE_SVD_NOALLOC_MAX_M;
constexpr size_t kNoAllocScratchElems = 655360;
constexpr int kNoAllocMaxDevices = 64;
}  // namespace

// Device copy per GPU, kept until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: host code uses the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kNoAllocScratchElems];

static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[kNoAllocMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
static double* noalloc_scratch()
{
    int dev = -1;
    GKL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        fail(GKL_ERR_DEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            fail(GKL_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_noalloc_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_noalloc_ptr[dev];
}

extern "C" {

gkl_status gkl_read_rate(const void* buf, int64_t bytes, int32_t reps, void* stream,
                         double* ms_per_read)
{
    if (!buf || !ms_per_read)
        return set_error(nullptr, GKL_ERR_INVALID, "gkl_read_rate: NULL pointer argument");
    if ((reinterpret_cast<uintptr_t>(buf) & 15) != 0 || bytes < 16 || reps < 1)
        return set_error(nullptr, GKL_ERR_INVALID,
                         "gkl_read_rate: buf must be 16-byte aligned, bytes >= 16, reps >= 1");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        GKL_HIP(hipEventCreate(&e0));
        GKL_HIP(hipEventCreate(&e1));
        launch_read_rate(buf, bytes, s);
        GKL_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch_read_rate(buf, bytes, s);
        GKL_HIP(hipEventRecord(e1, s));
        GKL_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        GKL_HIP(hipEventElapsedTime(&ms, e0, e1));
        *ms_per_read = (double)ms / reps;
        GKL_HIP(hipEventDestroy(e0));
        GKL_HIP(hipEventDestroy(e1));
        return GKL_OK;
    } catch (const Error& e) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return set_error(nullptr, e.status, e.msg);
    }
}

gkl_status gkl_dense_svd_noalloc(const double* B, int32_t m, double* P, double* S, double* Q,
                                 void* stream)
{
    if (!B || !P || !S || !Q)
        return set_error(nullptr, GKL_ERR_INVALID, "gkl_dense_svd_noalloc: NULL pointer argument");
    if (m < 1 || m > kNoAllocMaxM)
        return set_error(nullptr, GKL_ERR_INVALID,
                         "gkl_dense_svd_noalloc: m must lie in [1, " + std::to_string(kNoAllocMaxM) +
                             "] (its scratch is a fixed 5 MiB device array)");
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        double* gscr = nullptr;
        double* rlog = nullptr;
        if (!svd_fits_lds(m)) {
            const bool logged = svd_logged_fits_lds(m);
            const size_t need = logged ? svd_log_elems(m) : svd_scratch_elems(m);
            if (need > kNoAllocScratchElems)
                fail(GKL_ERR_INVALID, "gkl_dense_svd_noalloc: m needs more than the fixed scratch");
            double* ptr = noalloc_scratch();
            (logged ? rlog : gscr) = ptr;
        }
        // every scratch element the kernel reads it has written earlier in the
        // same launch (the log is replayed only up to the sweeps just run, the
        // working matrices are filled from B first), so nothing is cleared
        launch_dense_svd(B, m, P, S, Q, gscr, s, rlog);
        GKL_HIP(hipStreamSynchronize(s));
        return GKL_OK;
    } catch (const Error& e) {
        return set_error(nullptr, e.status, e.msg);
    }
}

}  // extern "C"
