// Host-side solver state (internal).
#pragma once

#include <array>
#include <string>
#include <vector>

#include "kernels.h"

namespace gkl {

// Every device allocation of a context; freed together.
struct DeviceArena {
    std::vector<void*> ptrs;
    size_t total = 0;
    void* alloc(size_t bytes);
    DeviceArena() = default;
    DeviceArena(const DeviceArena&) = delete;
    DeviceArena& operator=(const DeviceArena&) = delete;
    ~DeviceArena();
};

// One packed genotype matrix with its statistics and matvec scratch.
struct Problem {
    DeviceArena arena;
    int64_t n = 0, p = 0, ld = 0;
    const uint8_t* G_user = nullptr;   // the caller's matrix (borrowed)
    hipStream_t stream = nullptr;
    Packed packed;
    ColStats st{};
    MatvecWork mvw;
    // lut_layouts: build the two lookup-table layouts of the FP64 products
    // products: 0 = none (the blocked path builds its own layouts), 1 = lookup
    // tables (layouts T and P), 2 = seven int8 limbs (layouts I and S)
    void setup(const uint8_t* G, int64_t n, int64_t p, int64_t ld, hipStream_t s, int products);
};

// ||r|| into *out (no scaling).
void launch_norm(const double* r, int64_t len, double* out, OrthoWork& w, hipStream_t s);

struct MixedState;   // blocked matrix-core solver (k_mixed / mixed.hip)
struct BatchState;   // batched persistent solver (batched.hip)
bool mixed_supported();
// Message returned by gkl_last_error(NULL) (last failed create on this thread).
void set_create_error(const std::string& msg);
void destroy_mixed(MixedState* m);
void destroy_batch(BatchState* b);

}  // namespace gkl

struct gkl_ctx {
    gkl::Problem prob;
    gkl_options opt{};
    int k = 0;
    double tol = 0.0;
    int reorth = 0;
    int short_side = 0;      // 0: U (n <= p), 1: V -- the side one-sided reorth keeps
    bool two_sided = false;  // one-sided reorth switched to both sides
    double omega = 1e-8;
    double root_maxdim = 1.0;
    double noise_scale = 0.0;
    int krylov = 0;      // 0 = no restart
    int maxm = 0;        // basis capacity (left columns)
    int keep = 0;        // Ritz vectors kept at a restart
    bool batched = false;
    std::string last_error;
    std::vector<std::array<double, GKL_TRACE_FIELDS>> trace;
    gkl_info info{};
    double create_ms = 0.0;

    // device solver state (FP64 path)
    double* U = nullptr;
    double* V = nullptr;
    double* tmp = nullptr;
    double* scal = nullptr;
    double* alpha = nullptr;
    double* beta = nullptr;
    double* theta = nullptr;
    double* rho = nullptr;
    // harmonic thick restart: dense head of the projected matrix and the
    // small-space plan's buffers ((m+1) x (m+1) SVD, Z, LU work)
    double* head = nullptr;
    double* hpad = nullptr;
    double* hP = nullptr;
    double* hS = nullptr;
    double* hQ = nullptr;
    double* hZ = nullptr;
    double* hwork = nullptr;
    double* hsvd_scratch = nullptr;
    bool head_dense = false;     // the first nlock rows hold a dense head
    bool zero_scalar = false;    // a breakdown recorded a zero scalar since the last restart
    double* norm_est = nullptr;
    int* flags = nullptr;   // [0] left breakdown [1] right breakdown [2..5] PRO
                            // [6] Gram-Schmidt passes [7] scratch flag [8] nconv
                            // [9] first breakdown half-step (-1 = none)
    gkl::RitzOut ritz{};
    double* svd_scratch = nullptr;
    gkl::ProState pro{};
    gkl::OrthoWork ow;
    static constexpr size_t kScalarsPerCol = 4;
    size_t kScalars = 0;

    // loop state
    int nlock = 0;
    int ritz_m = -1;
    bool exhausted = false;
    uint64_t breakdown_draws = 1;
    int last_breakdown = -1;
    static constexpr int kOrthoCounters = 128;

    // optional kernel timing (options.timing)
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_mv, ev_rmv;   // (product slot, main-kernel slot)
    int ev_next = 0;
    int64_t ev_calls[2] = {0, 0};   // timing_slot calls (A v, A^T u) since the last collection
    int timing_slot(bool right);
    const hipEvent_t* timing_events(int slot);
    void timing_note(int slot, bool right, bool core = false);
    int timing_begin(bool right);
    void timing_end(int start, bool right, bool core = false);
    void timing_collect();

    gkl::MixedState* mixed = nullptr;
    gkl::BatchState* batch = nullptr;

    gkl_ctx() = default;
    ~gkl_ctx();

    void allocate_solver();
    void record(int step, bool restart_flag, double res_rel);
    int read_flag(const int* dflag);
    void sync_state(int* nconv, int* breakdown);
    void left_step(int j);
    void right_step(int j);
    void launch_normalize_only(double* r, int64_t len, double* out);
    gkl::ProArgs pro_args(int j) const;
    gkl::NormTail pro_tail(double* nrm_out, int side, int j) const;
    void handle_breakdown(bool left, int j);
    bool long_side_free(int side) const;
    const int* long_side_check(const double* Q, int64_t len, int ncols, const double* r,
                               double* nrm);
    double onesided_tol() const;
    int check_convergence(int m);
    void restart(int m);
    void restart_harmonic(int m);
    void finalize(int m, double* sigma, double* Uo, int64_t ldu, double* Vo, int64_t ldv);
    gkl_status solve_fp64(double* sigma, double* Uo, int64_t ldu, double* Vo, int64_t ldv);
    void setup_mixed();
    gkl_status solve_mixed(double* sigma, double* Uo, int64_t ldu, double* Vo, int64_t ldv);
};
