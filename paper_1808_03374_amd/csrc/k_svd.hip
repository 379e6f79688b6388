// Ritz extraction for GKL (gfx950, FP64).
//
// Section 3 of the paper: the top singular triplets of A are approximated from
// the SVD of the small projected matrix B_j (upper bidiagonal, or after a thick
// restart a diagonal block -- a dense block after a harmonic restart -- with one
// spike column followed by a bidiagonal tail), and convergence is tested with
// the residual bound
//     |sigma - sigma~_i| <= beta_j |P_{j,i}|
// where P holds the left singular vectors of B_j (the Table 3 caption sums these
// bounds into ||Delta theta||_1).
//
// The SVD is a one-sided (Hestenes) Jacobi method.  Up to 96 columns one
// workgroup holds the matrix and the accumulated rotations in LDS; up to 128
// columns the matrix alone is, the rotations are logged to device memory and
// replayed onto the identity afterwards (or, when the caller needs only
// well-separated leading columns, those are formed from the rotated matrix).
// Column pairs of a round-robin tournament are rotated concurrently, 16 lanes
// per pair, with the pair's columns held in registers while they are rotated
// (rows zero-padded to a multiple of 16, so every lane's loads are
// unconditional); sweeps repeat until no pair needs rotating.  Larger matrices
// work in global scratch with each round spread over workgroups (one launch
// per round, one wave per pair).  The file also holds the small-space part of
// the harmonic thick restart.
#include <math.h>

#include "kernels.h"

namespace gkl {

namespace {
constexpr int kSvdThreads = 1024;
constexpr int kGroup = 16;                      // lanes per column pair
constexpr int kGroups = kSvdThreads / kGroup;   // pairs rotated at once
constexpr int kMaxSweeps = 40;

// One 64-bit DPP move (two 32-bit halves) with a constant lane pattern.
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffff), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), kCtrl, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 16 lanes of a group (a DPP row).  Partners are symmetric at
// every level -- lane i with i^1, i^2 (quad permutes), 7-i within each half
// row, 15-i within the row -- so every lane ends with the same bits.
__device__ __forceinline__ double group_sum(double v)
{
    static_assert(kGroup == 16, "group_sum covers one DPP row");
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);   // row_half_mirror
    v += dpp_move<0x140>(v);   // row_mirror
    return v;
}


// 1/x and 1/sqrt(x) from the hardware estimates, each refined by two Newton
// steps.
__device__ __forceinline__ double rcp_refined(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double rsq_refined(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * (x * y), y, 1.5);
    return y * fma(-0.5 * (x * y), y, 1.5);
}

// Rotation of a column pair with inner product sab and squared norms saa, sbb
// (Rutishauser's formulas): zeta = (sbb - saa) / (2 sab), t = sign(zeta) /
// (|zeta| + sqrt(1 + zeta^2)), cs = 1 / sqrt(1 + t^2), sn = cs t.  Returns
// false when the pair needs no rotation: sab is negligible against the norms
// (|sab| <= tol sqrt(saa sbb), tested squared), or zeta is so large (or not a
// number, from a vanishing sab) that the angle, about 1/(2 zeta), would not
// change either column.
__device__ __forceinline__ bool jacobi_rotation(double sab, double saa, double sbb, double tol,
                                                double& t, double& cs, double& sn)
{
    if (!(sab != 0.0 && sab * sab > (tol * tol) * (saa * sbb))) return false;
    const double z = (sbb - saa) * (0.5 * rcp_refined(sab));
    if (!(fabs(z) < 1e150)) return false;
    const double w = fma(z, z, 1.0);
    t = (z >= 0.0 ? 1.0 : -1.0) * rcp_refined(fabs(z) + w * rsq_refined(w));
    cs = rsq_refined(fma(t, t, 1.0));
    sn = cs * t;
    return true;
}

// Column stride of the working arrays: rows are padded with zeros to a
// multiple of the 16-lane group when mp <= 128 (every lane then holds exactly
// svd_elems(mp) elements of a column and loads them unconditionally), else mp.
constexpr int kMaxPadElems = 8;
__host__ __device__ inline int svd_elems(int mp) { return (mp + kGroup - 1) / kGroup; }
__host__ __device__ inline int svd_ld(int mp)
{
    return mp <= kMaxPadElems * kGroup ? kGroup * svd_elems(mp) : mp;
}

// W (ld x mp, column-major) is replaced by B Q = P S; Vr accumulates Q.  mp is
// even (a zero column pads odd m); rows past mp are zero and stay zero.  Column
// norms (dn, mp doubles) are computed once per sweep and updated after each
// rotation (d_p -= t c, d_q += t c), so a pair needs one reduction (its inner
// product).  Returns after a sweep without rotations.  kJ > 0: ld = 16 kJ and
// every lane holds kJ elements of each column of its pair in registers.
// kLog: Vr is not touched; instead every pair of every round writes its
// rotation (cs, sn), or (1, 0) when it is not rotated, to
// rlog[2 ((sweep ring + round) npairs + pair)], for replay_rotations.  Returns
// the number of sweeps that rotated at least one pair (all sweeps before the
// last when the last had no rotation).
template <int kJ, bool kLog>
__device__ __forceinline__ int jacobi_sweeps_t(double* W, double* Vr, int mp, int ld, double* dn,
                                               double* __restrict__ rlog)
{
    __shared__ int rotated;
    const int g = threadIdx.x / kGroup;
    const int gl = threadIdx.x % kGroup;
    const int npairs = mp / 2;
    const int ring = mp - 1;
    // rotation threshold sqrt(m) * eps (the usual one-sided Jacobi test)
    const double tol = 2.220446049250313e-16 * sqrt((double)mp);
    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        for (int c = g; c < mp; c += kGroups) {
            const double* wc = W + (int64_t)c * ld;
            double a = 0.0;
            for (int i = gl; i < mp; i += kGroup) a = fma(wc[i], wc[i], a);
            a = group_sum(a);
            if (gl == 0) dn[c] = a;
        }
        if (threadIdx.x == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < ring; ++r) {
            for (int k = g; k < npairs; k += kGroups) {
                // round-robin tournament: pair k of round r
                int a, b;
                if (k == 0) {
                    a = ring;
                    b = r;
                } else {
                    a = r + k;
                    if (a >= ring) a -= ring;
                    b = r - k;
                    if (b < 0) b += ring;
                }
                if (a > b) { const int tmp = a; a = b; b = tmp; }
                double* xa = W + (int64_t)a * ld;
                double* xb = W + (int64_t)b * ld;
                double* ya = kLog ? nullptr : Vr + (int64_t)a * ld;
                double* yb = kLog ? nullptr : Vr + (int64_t)b * ld;
                double* lg = kLog ? rlog + 2 * (((int64_t)sweep * ring + r) * npairs + k) : nullptr;
                const double saa = dn[a], sbb = dn[b];
                double t, cs, sn, sab = 0.0;
                if (kJ > 0) {
                    // both pairs of columns are read once, unconditionally (rows
                    // are padded); the rotation is applied from registers
                    constexpr int kE = kJ > 0 ? kJ : 1;
                    double u[kE], v[kE], pa[kE], pb[kE];
#pragma unroll
                    for (int j = 0; j < kE; ++j) {
                        const int i = gl + j * kGroup;
                        u[j] = xa[i];
                        v[j] = xb[i];
                        if (!kLog) {
                            pa[j] = ya[i];
                            pb[j] = yb[i];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < kE; ++j) sab = fma(u[j], v[j], sab);
                    sab = group_sum(sab);
                    const bool rot = jacobi_rotation(sab, saa, sbb, tol, t, cs, sn);
                    if (kLog && gl == 0) {
                        lg[0] = rot ? cs : 1.0;
                        lg[1] = rot ? sn : 0.0;
                    }
                    if (!rot) continue;
#pragma unroll
                    for (int j = 0; j < kE; ++j) {
                        const int i = gl + j * kGroup;
                        xa[i] = cs * u[j] - sn * v[j];
                        xb[i] = sn * u[j] + cs * v[j];
                        if (!kLog) {
                            ya[i] = cs * pa[j] - sn * pb[j];
                            yb[i] = sn * pa[j] + cs * pb[j];
                        }
                    }
                } else {
                    for (int i = gl; i < mp; i += kGroup) sab = fma(xa[i], xb[i], sab);
                    sab = group_sum(sab);
                    if (!jacobi_rotation(sab, saa, sbb, tol, t, cs, sn)) continue;
                    for (int i = gl; i < mp; i += kGroup) {
                        const double x = xa[i], y = xb[i];
                        xa[i] = cs * x - sn * y;
                        xb[i] = sn * x + cs * y;
                        const double p = ya[i], q = yb[i];
                        ya[i] = cs * p - sn * q;
                        yb[i] = sn * p + cs * q;
                    }
                }
                if (gl == 0) {
                    dn[a] = saa - t * sab;
                    dn[b] = sbb + t * sab;
                    rotated = 1;
                }
            }
            __syncthreads();
        }
        if (!rotated) break;
        __syncthreads();
    }
    return sweep;
}

__device__ __forceinline__ void jacobi_sweeps(double* W, double* Vr, int mp, int ld, double* dn)
{
    switch (ld == kGroup * svd_elems(mp) ? svd_elems(mp) : 0) {
    case 1: jacobi_sweeps_t<1, false>(W, Vr, mp, ld, dn, nullptr); break;
    case 2: jacobi_sweeps_t<2, false>(W, Vr, mp, ld, dn, nullptr); break;
    case 3: jacobi_sweeps_t<3, false>(W, Vr, mp, ld, dn, nullptr); break;
    case 4: jacobi_sweeps_t<4, false>(W, Vr, mp, ld, dn, nullptr); break;
    case 5: jacobi_sweeps_t<5, false>(W, Vr, mp, ld, dn, nullptr); break;
    case 6: jacobi_sweeps_t<6, false>(W, Vr, mp, ld, dn, nullptr); break;
    case 7: jacobi_sweeps_t<7, false>(W, Vr, mp, ld, dn, nullptr); break;
    case 8: jacobi_sweeps_t<8, false>(W, Vr, mp, ld, dn, nullptr); break;
    default: jacobi_sweeps_t<0, false>(W, Vr, mp, ld, dn, nullptr); break;
    }
}

// Applies the logged rotations of nsw sweeps to Vr (ld = 16 kJ, starting from
// the identity) in the order the sweeps made them, so Vr ends bit for bit as
// if it had been rotated along with W.  One 16-lane group per pair (mp <= 2 x
// the groups); each group fetches its next rotation while applying the current
// one.  Identity entries are skipped, as the sweeps skipped those pairs.
template <int kJ>
__device__ __forceinline__ void replay_rotations_t(double* Vr, int mp, int ld,
                                                   const double* __restrict__ rlog, int nsw)
{
    const int g = threadIdx.x / kGroup;
    const int gl = threadIdx.x % kGroup;
    const int npairs = mp / 2;
    const int ring = mp - 1;
    const bool act = g < npairs;
    const int total = nsw * ring;
    double ncs = 1.0, nsn = 0.0;
    if (act && total > 0) {
        ncs = rlog[2 * g];
        nsn = rlog[2 * g + 1];
    }
    for (int step = 0; step < total; ++step) {
        const double cs = ncs, sn = nsn;
        if (act && step + 1 < total) {
            const double* nx = rlog + 2 * ((int64_t)(step + 1) * npairs + g);
            ncs = nx[0];
            nsn = nx[1];
        }
        const int r = step % ring;
        if (act && !(cs == 1.0 && sn == 0.0)) {
            int a, b;
            if (g == 0) {
                a = ring;
                b = r;
            } else {
                a = r + g;
                if (a >= ring) a -= ring;
                b = r - g;
                if (b < 0) b += ring;
            }
            if (a > b) { const int tmp = a; a = b; b = tmp; }
            double* ya = Vr + (int64_t)a * ld;
            double* yb = Vr + (int64_t)b * ld;
            double pa[kJ], pb[kJ];
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                pa[j] = ya[gl + j * kGroup];
                pb[j] = yb[gl + j * kGroup];
            }
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                ya[gl + j * kGroup] = cs * pa[j] - sn * pb[j];
                yb[gl + j * kGroup] = sn * pa[j] + cs * pb[j];
            }
        }
        __syncthreads();
    }
}

// Jacobi on W alone with the rotations logged, for 96 < mp <= 128 (ld = 16 kJ).
__device__ __forceinline__ int jacobi_sweeps_logged(double* W, int mp, int ld, double* dn,
                                                    double* rlog)
{
    return svd_elems(mp) == 7 ? jacobi_sweeps_t<7, true>(W, nullptr, mp, ld, dn, rlog)
                              : jacobi_sweeps_t<8, true>(W, nullptr, mp, ld, dn, rlog);
}

__device__ __forceinline__ void replay_rotations(double* Vr, int mp, int ld, const double* rlog,
                                                 int nsw)
{
    if (svd_elems(mp) == 7) replay_rotations_t<7>(Vr, mp, ld, rlog, nsw);
    else replay_rotations_t<8>(Vr, mp, ld, rlog, nsw);
}

// After jacobi_sweeps: singular values are the column norms of W; write the
// m leading (sorted descending) triplets.  With W == NULL only Q is written
// (from Vr), using the norms and order of an earlier call; with Vr == NULL only
// P and S.
__device__ __forceinline__ void extract_sorted(const double* W, const double* Vr, int m, int mp,
                                               int ld, double* sig, int* order, double* P,
                                               int ldp_, double* S, double* Q, int ldq_)
{
    for (int c = threadIdx.x / kGroup; W && c < mp; c += kGroups) {
        const double* wc = W + (int64_t)c * ld;
        double s = 0.0;
        for (int i = threadIdx.x % kGroup; i < mp; i += kGroup) s = fma(wc[i], wc[i], s);
        s = group_sum(s);
        if (threadIdx.x % kGroup == 0) sig[c] = sqrt(s);
    }
    __syncthreads();
    // rank by value (ties broken by index) -> stable descending order.  A NaN
    // norm ranks as -1 so that the ranks stay a permutation whatever the input.
    for (int c = threadIdx.x; W && c < mp; c += blockDim.x) {
        int rank = 0;
        const double sc = isnan(sig[c]) ? -1.0 : sig[c];
        for (int d = 0; d < mp; ++d) {
            const double sd = isnan(sig[d]) ? -1.0 : sig[d];
            rank += (sd > sc) || (sd == sc && d < c);
        }
        order[rank] = c;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
        const int i = t % m, o = t / m;     // row i of output column o
        const int c = order[o];
        const double s = sig[c];
        if (W) P[(int64_t)o * ldp_ + i] = s > 0.0 ? W[(int64_t)c * ld + i] / s : (i == o ? 1.0 : 0.0);
        if (Vr) Q[(int64_t)o * ldq_ + i] = Vr[(int64_t)c * ld + i];
    }
    for (int o = threadIdx.x; W && o < m; o += blockDim.x) S[o] = sig[order[o]];
}

}  // namespace

// Projected matrices too large for LDS: the sweeps of jacobi_sweeps_t<0> --
// same tournament, pairs, rotation formula and column-norm updates -- with the
// disjoint pairs of each round spread over workgroups (one launch per round;
// one wave per pair, each lane holding up to kMwElems elements of the pair's
// four columns in registers, all loaded before the inner product so that one
// memory round trip serves the pair) instead of one workgroup taking them 64
// at a time through L2.  The column norms are refreshed by their own launch at
// the start of each sweep, which also clears the sweep's rotation flag; the
// host reads the flag after the sweep and stops after a sweep without
// rotations.  The wave-wide sums add in another order than the 16-lane groups
// of the in-LDS sweeps, so the two paths agree to rounding, not bit for bit.
constexpr int kMwElems = (kMaxSvd + 1 + kWave - 1) / kWave;   // mp <= kMaxSvd + 1

__global__ void __launch_bounds__(256)
jacobi_norms_kernel(const double* __restrict__ W, int mp, int ld, double* __restrict__ dn,
                    int* __restrict__ rotated)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *rotated = 0;
    const int c = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kGroup);
    const int gl = threadIdx.x % kGroup;
    if (c >= mp) return;                  // whole 16-lane groups leave together
    const double* wc = W + (int64_t)c * ld;
    double a = 0.0;
    for (int i = gl; i < mp; i += kGroup) a = fma(wc[i], wc[i], a);
    a = group_sum(a);
    if (gl == 0) dn[c] = a;
}

__global__ void __launch_bounds__(kWave)
jacobi_round_kernel(double* __restrict__ W, double* __restrict__ Vr, int mp, int ld,
                    double* __restrict__ dn, int r, int* __restrict__ rotated)
{
    const int ring = mp - 1;
    const int k = blockIdx.x;             // pair k of round r
    const int lane = threadIdx.x;
    const double tol = 2.220446049250313e-16 * sqrt((double)mp);
    int a, b;
    if (k == 0) {
        a = ring;
        b = r;
    } else {
        a = r + k;
        if (a >= ring) a -= ring;
        b = r - k;
        if (b < 0) b += ring;
    }
    if (a > b) { const int tmp = a; a = b; b = tmp; }
    double* xa = W + (int64_t)a * ld;
    double* xb = W + (int64_t)b * ld;
    double* ya = Vr + (int64_t)a * ld;
    double* yb = Vr + (int64_t)b * ld;
    double u[kMwElems], v[kMwElems], pa[kMwElems], pb[kMwElems];
#pragma unroll
    for (int j = 0; j < kMwElems; ++j) {
        const int i = lane + j * kWave;
        const bool in = i < mp;
        u[j] = in ? xa[i] : 0.0;
        v[j] = in ? xb[i] : 0.0;
        pa[j] = in ? ya[i] : 0.0;
        pb[j] = in ? yb[i] : 0.0;
    }
    const double saa = dn[a], sbb = dn[b];
    double sab = 0.0;
#pragma unroll
    for (int j = 0; j < kMwElems; ++j) sab = fma(u[j], v[j], sab);
    sab = wave_sum(sab);
    double t, cs, sn;
    if (!jacobi_rotation(sab, saa, sbb, tol, t, cs, sn)) return;
#pragma unroll
    for (int j = 0; j < kMwElems; ++j) {
        const int i = lane + j * kWave;
        if (i < mp) {
            xa[i] = cs * u[j] - sn * v[j];
            xb[i] = sn * u[j] + cs * v[j];
            ya[i] = cs * pa[j] - sn * pb[j];
            yb[i] = sn * pa[j] + cs * pb[j];
        }
    }
    if (lane == 0) {
        dn[a] = saa - t * sab;
        dn[b] = sbb + t * sab;
        *rotated = 1;
    }
}

// flag: one int of device memory (the spare element after the working arrays).
static void jacobi_multi_wg(double* W, double* Vr, int mp, int ld, double* dn, int* flag,
                            hipStream_t s)
{
    const int npairs = mp / 2, ring = mp - 1;
    const int nn = (int)ceil_div((int64_t)mp * kGroup, 256);
    if (mp > kMwElems * kWave) fail(GKL_ERR_INTERNAL, "Jacobi working size beyond the register tile");
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        hipLaunchKernelGGL(jacobi_norms_kernel, dim3(nn), dim3(256), 0, s, W, mp, ld, dn, flag);
        GKL_LAUNCH_CHECK("jacobi_norms_kernel");
        for (int r = 0; r < ring; ++r)
            hipLaunchKernelGGL(jacobi_round_kernel, dim3(npairs), dim3(kWave), 0, s, W, Vr, mp, ld,
                               dn, r, flag);
        GKL_LAUNCH_CHECK("jacobi_round_kernel");
        int h = 0;
        GKL_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        GKL_HIP(hipStreamSynchronize(s));
        if (!h) break;
    }
}

// Working arrays in gscratch: W, Vr (ld x mp each), sig, dn (mp each), order
// (mp ints), then the flag.
struct GlobalSvd {
    double* W;
    double* Vr;
    double* sig;
    double* dn;
    int* order;
    int* flag;
};

static GlobalSvd global_svd_arrays(double* gscratch, int m)
{
    const int mp = m + (m & 1);
    const int ld = svd_ld(mp);
    GlobalSvd g;
    g.W = gscratch;
    g.Vr = g.W + (int64_t)ld * mp;
    g.sig = g.Vr + (int64_t)ld * mp;
    g.dn = g.sig + mp;
    g.order = reinterpret_cast<int*>(g.dn + mp);
    g.flag = g.order + mp;
    return g;
}

// B (m x m) into W, the identity into Vr.
__global__ void __launch_bounds__(256)
svd_load_kernel(const double* __restrict__ B, int m, double* __restrict__ W, double* __restrict__ Vr)
{
    const int mp = m + (m & 1);
    const int ld = svd_ld(mp);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)ld * mp;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % ld), c = (int)(t / ld);
        W[t] = (i < m && c < m) ? B[(int64_t)c * m + i] : 0.0;
        Vr[t] = (i == c) ? 1.0 : 0.0;
    }
}

__global__ void __launch_bounds__(kSvdThreads)
svd_extract_kernel(int m, GlobalSvd g, double* __restrict__ P, double* __restrict__ S,
                   double* __restrict__ Q)
{
    const int mp = m + (m & 1);
    extract_sorted(g.W, g.Vr, m, mp, svd_ld(mp), g.sig, g.order, P, m, S, Q, m);
}

// kLds: the working arrays live in LDS (the compiler then emits LDS
// instructions); otherwise in gscratch.
// Leading columns of Q recovered as B^T w_c / sig_c^2 (w_c = sig_c p_c, the
// rotated column) when the last of them has sig_c >= kRecoverRatio sig_max:
// their error is then below eps / kRecoverRatio^2 (about 1e-13).
constexpr double kRecoverRatio = 0.05;

// qcols: leading columns of Q the caller reads (the logged path may then skip
// the replay; columns from qcols on are left unwritten); qcols >= m: all.
template <bool kLds>
__global__ void __launch_bounds__(kSvdThreads)
dense_svd_kernel(const double* __restrict__ B, int m, double* __restrict__ P,
                 double* __restrict__ S, double* __restrict__ Q, double* gscratch, double* rlog,
                 int qcols)
{
    extern __shared__ double lds[];
    const int mp = m + (m & 1);
    const int ld = svd_ld(mp);
    if (kLds && rlog) {
        // W alone in LDS; Vr is rebuilt in the same space from the rotation log
        double* W = lds;
        double* sig = W + ld * mp;
        double* dn = sig + mp;
        int* order = reinterpret_cast<int*>(dn + mp);
        for (int t = threadIdx.x; t < ld * mp; t += blockDim.x) {
            const int i = t % ld, c = t / ld;
            W[t] = (i < m && c < m) ? B[(int64_t)c * m + i] : 0.0;
        }
        __syncthreads();
        const int nsw = jacobi_sweeps_logged(W, mp, ld, dn, rlog);
        __syncthreads();
        extract_sorted(W, nullptr, m, mp, ld, sig, order, P, m, S, nullptr, m);
        __syncthreads();
        const double smax = sig[order[0]];
        if (qcols < m && smax > 0.0 && sig[order[qcols - 1]] >= kRecoverRatio * smax) {
            for (int t = threadIdx.x; t < m * qcols; t += blockDim.x) {
                const int i = t % m, o = t / m;      // row i of output column o
                const int c = order[o];
                const double* bi = B + (int64_t)i * m;
                const double* wc = W + (int64_t)c * ld;
                double acc = 0.0;
#pragma unroll 8
                for (int r = 0; r < m; ++r) acc = fma(bi[r], wc[r], acc);
                const double sc = sig[c];
                Q[(int64_t)o * m + i] = acc / (sc * sc);
            }
            return;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < ld * mp; t += blockDim.x) W[t] = (t % ld == t / ld) ? 1.0 : 0.0;
        __threadfence_block();
        __syncthreads();
        replay_rotations(W, mp, ld, rlog, nsw);
        __syncthreads();
        extract_sorted(nullptr, W, m, mp, ld, sig, order, nullptr, m, nullptr, Q, m);
        return;
    }
    double* W = kLds ? lds : gscratch;
    double* Vr = W + ld * mp;
    double* sig = Vr + ld * mp;
    double* dn = sig + mp;
    int* order = reinterpret_cast<int*>(dn + mp);
    for (int t = threadIdx.x; t < ld * mp; t += blockDim.x) {
        const int i = t % ld, c = t / ld;
        W[t] = (i < m && c < m) ? B[(int64_t)c * m + i] : 0.0;
        Vr[t] = (i == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_sweeps(W, Vr, mp, ld, dn);
    __syncthreads();
    extract_sorted(W, Vr, m, mp, ld, sig, order, P, m, S, Q, m);
}

// W and Vr (ld x mp each), sig and dn (mp each), order (mp ints).
static size_t svd_lds_bytes(int m)
{
    const int mp = m + (m & 1);
    return sizeof(double) * (2 * (size_t)svd_ld(mp) * mp + 2 * (size_t)mp) +
           sizeof(int) * (size_t)mp;
}

// The logged path: W (ld x mp), sig and dn (mp each), order (mp ints).
static size_t svd_logged_lds_bytes(int m)
{
    const int mp = m + (m & 1);
    return sizeof(double) * ((size_t)svd_ld(mp) * mp + 2 * (size_t)mp) + sizeof(int) * (size_t)mp;
}

size_t svd_log_elems(int m)
{
    const int mp = m + (m & 1);
    return 2 * (size_t)kMaxSweeps * (size_t)(mp - 1) * (size_t)(mp / 2);
}

size_t svd_scratch_elems(int m) { return svd_lds_bytes(m) / sizeof(double) + 1; }

static int svd_lds_limit()
{
    static int limit = -1;
    if (limit < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        limit = v;
    }
    return limit;
}

// the kernels' static LDS (flags, reduction scratch) needs room beside the arrays
bool svd_fits_lds(int m)
{
    return m <= kMaxKrylov && svd_lds_bytes(m) + 256 <= (size_t)svd_lds_limit();
}

bool svd_logged_fits_lds(int m)
{
    const int mp = m + (m & 1);
    return mp <= kMaxPadElems * kGroup && mp <= 2 * kGroups &&
           svd_logged_lds_bytes(m) + 256 <= (size_t)svd_lds_limit();
}

static void check_svd_size(int m, const double* gscratch)
{
    if (m < 1 || m > kMaxSvd) fail(GKL_ERR_INVALID, "projected matrix size out of range");
    if (!svd_fits_lds(m) && gscratch == nullptr)
        fail(GKL_ERR_INTERNAL, "large projected matrix needs a global scratch buffer");
}

void launch_dense_svd(const double* B, int m, double* P, double* S, double* Q, double* gscratch,
                      hipStream_t s, double* rlog, int qcols)
{
    if (m < 1 || m > kMaxSvd) fail(GKL_ERR_INVALID, "projected matrix size out of range");
    const int qc = qcols > 0 && qcols < m ? qcols : m;
    if (svd_fits_lds(m)) {
        hipLaunchKernelGGL(dense_svd_kernel<true>, dim3(1), dim3(kSvdThreads), svd_lds_bytes(m), s,
                           B, m, P, S, Q, nullptr, nullptr, m);
    } else if (rlog && svd_logged_fits_lds(m)) {
        hipLaunchKernelGGL(dense_svd_kernel<true>, dim3(1), dim3(kSvdThreads),
                           svd_logged_lds_bytes(m), s, B, m, P, S, Q, nullptr, rlog, qc);
    } else {
        if (!gscratch) fail(GKL_ERR_INTERNAL, "large projected matrix needs a global scratch buffer");
        const int mp = m + (m & 1);
        const GlobalSvd g = global_svd_arrays(gscratch, m);
        hipLaunchKernelGGL(svd_load_kernel, dim3((unsigned)std::min<int64_t>(
                               ceil_div((int64_t)svd_ld(mp) * mp, 256), 1024)), dim3(256), 0, s,
                           B, m, g.W, g.Vr);
        GKL_LAUNCH_CHECK("svd_load_kernel");
        jacobi_multi_wg(g.W, g.Vr, mp, svd_ld(mp), g.dn, g.flag, s);
        hipLaunchKernelGGL(svd_extract_kernel, dim3(1), dim3(kSvdThreads), 0, s, m, g, P, S, Q);
        GKL_LAUNCH_CHECK("svd_extract_kernel");
        return;
    }
    GKL_LAUNCH_CHECK("dense_svd_kernel");
}

// Projected matrix from the recurrence scalars, its SVD and the residual test
// (one workgroup; W, Vr, sig, order are the working arrays).
// head (optional): after a harmonic restart the first nlock rows hold a dense
// nlock x nlock block (column-major, ld nlock) instead of diag(theta).
__device__ __forceinline__ void ritz_assemble(const double* __restrict__ alpha,
                                              const double* __restrict__ beta,
                                              const double* __restrict__ theta,
                                              const double* __restrict__ rho, int nlock, int m,
                                              const RitzOut& out, double* W, double* Vr,
                                              const double* __restrict__ head)
{
    const int mp = m + (m & 1);
    const int ld = svd_ld(mp);
    for (int t = threadIdx.x; t < ld * mp; t += blockDim.x) {
        const int i = t % ld, c = t / ld;
        double v = 0.0;
        if (i < m && c < m) {
            if (i < nlock) {
                if (c == nlock) v = rho[i];
                else if (head) v = c < nlock ? head[(int64_t)c * nlock + i] : 0.0;
                else if (c == i) v = theta[i];
            } else {
                if (c == i) v = alpha[i];
                else if (c == i + 1) v = beta[i];
            }
        }
        W[t] = v;
        Vr[t] = (i == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) out.B[t] = W[(t / m) * ld + (t % m)];
}

__device__ __forceinline__ void ritz_finish(const double* __restrict__ beta, int m, int k,
                                            double tol, const RitzOut& out, const double* W,
                                            const double* Vr, double* sig, int* order)
{
    const int mp = m + (m & 1);
    extract_sorted(W, Vr, m, mp, svd_ld(mp), sig, order, out.P, m, out.S, out.Q, m);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double bl = beta[m - 1];
        const double s0 = out.S[0];
        int nconv = 0;
        bool run = true;
        for (int i = 0; i < m; ++i) {
            const double r = fabs(bl * out.P[(int64_t)i * m + (m - 1)]);
            out.res[i] = r;
            if (i < k && run) {
                if (r <= tol * s0) ++nconv;
                else run = false;
            }
        }
        *out.nconv = nconv;
    }
}

__device__ __forceinline__ void ritz_body(const double* __restrict__ alpha,
                                          const double* __restrict__ beta,
                                          const double* __restrict__ theta,
                                          const double* __restrict__ rho, int nlock, int m, int k,
                                          double tol, const RitzOut& out, double* W, double* Vr,
                                          double* sig, double* dn, int* order,
                                          const double* __restrict__ head = nullptr)
{
    const int mp = m + (m & 1);
    ritz_assemble(alpha, beta, theta, rho, nlock, m, out, W, Vr, head);
    jacobi_sweeps(W, Vr, mp, svd_ld(mp), dn);
    __syncthreads();
    ritz_finish(beta, m, k, tol, out, W, Vr, sig, order);
}

template <bool kLds>
__global__ void __launch_bounds__(kSvdThreads)
ritz_kernel(const double* __restrict__ alpha, const double* __restrict__ beta,
            const double* __restrict__ theta, const double* __restrict__ rho, int nlock, int m,
            int k, double tol, RitzOut out, double* gscratch, const double* __restrict__ head)
{
    extern __shared__ double lds[];
    const int mp = m + (m & 1);
    const int ld = svd_ld(mp);
    double* W = kLds ? lds : gscratch;
    double* Vr = W + ld * mp;
    double* sig = Vr + ld * mp;
    double* dn = sig + mp;
    int* order = reinterpret_cast<int*>(dn + mp);
    ritz_body(alpha, beta, theta, rho, nlock, m, k, tol, out, W, Vr, sig, dn, order, head);
}

// One workgroup per problem of a batch.
template <bool kLds>
__global__ void __launch_bounds__(kSvdThreads)
ritz_batched_kernel(const BatchRitzArgs* __restrict__ args, int nlock, int m, int k, double tol,
                    double* gscratch, int64_t gstride)
{
    extern __shared__ double lds[];
    const BatchRitzArgs& a = args[blockIdx.x];
    if (!a.run) return;
    const int mp = m + (m & 1);
    const int ld = svd_ld(mp);
    double* W = kLds ? lds : gscratch + (int64_t)blockIdx.x * gstride;
    double* Vr = W + ld * mp;
    double* sig = Vr + ld * mp;
    double* dn = sig + mp;
    int* order = reinterpret_cast<int*>(dn + mp);
    ritz_body(a.alpha, a.beta, a.theta, a.rho, nlock, m, k, tol, a.out, W, Vr, sig, dn, order);
}

__global__ void __launch_bounds__(kSvdThreads)
ritz_assemble_kernel(const double* __restrict__ alpha, const double* __restrict__ beta,
                     const double* __restrict__ theta, const double* __restrict__ rho, int nlock,
                     int m, RitzOut out, GlobalSvd g, const double* __restrict__ head)
{
    ritz_assemble(alpha, beta, theta, rho, nlock, m, out, g.W, g.Vr, head);
}

__global__ void __launch_bounds__(kSvdThreads)
ritz_finish_kernel(const double* __restrict__ beta, int m, int k, double tol, RitzOut out,
                   GlobalSvd g)
{
    ritz_finish(beta, m, k, tol, out, g.W, g.Vr, g.sig, g.order);
}

void launch_ritz(const double* alpha, const double* beta, const double* theta, const double* rho,
                 int nlock, int m, int k, double tol, const RitzOut& out, double* gscratch,
                 hipStream_t s, const double* head)
{
    check_svd_size(m, gscratch);
    if (!svd_fits_lds(m)) {
        // working arrays in gscratch; the sweeps spread over workgroups
        const int mp = m + (m & 1);
        const GlobalSvd g = global_svd_arrays(gscratch, m);
        hipLaunchKernelGGL(ritz_assemble_kernel, dim3(1), dim3(kSvdThreads), 0, s, alpha, beta,
                           theta, rho, nlock, m, out, g, head);
        GKL_LAUNCH_CHECK("ritz_assemble_kernel");
        jacobi_multi_wg(g.W, g.Vr, mp, svd_ld(mp), g.dn, g.flag, s);
        hipLaunchKernelGGL(ritz_finish_kernel, dim3(1), dim3(kSvdThreads), 0, s, beta, m, k, tol,
                           out, g);
        GKL_LAUNCH_CHECK("ritz_finish_kernel");
        return;
    }
    hipLaunchKernelGGL(ritz_kernel<true>, dim3(1), dim3(kSvdThreads), svd_lds_bytes(m), s, alpha,
                       beta, theta, rho, nlock, m, k, tol, out, nullptr, head);
    GKL_LAUNCH_CHECK("ritz_kernel");
}

void launch_ritz_batched(const BatchRitzArgs* args, int count, int nlock, int m, int k, double tol,
                         double* gscratch, hipStream_t s)
{
    check_svd_size(m, gscratch);
    const bool global = !svd_fits_lds(m);
    if (global)
        hipLaunchKernelGGL(ritz_batched_kernel<false>, dim3(count), dim3(kSvdThreads), 0, s, args,
                           nlock, m, k, tol, gscratch, (int64_t)svd_scratch_elems(m));
    else
        hipLaunchKernelGGL(ritz_batched_kernel<true>, dim3(count), dim3(kSvdThreads),
                           svd_lds_bytes(m), s, args, nlock, m, k, tol, nullptr, (int64_t)0);
    GKL_LAUNCH_CHECK("ritz_batched_kernel");
}

__global__ void restart_scalars_kernel(const double* __restrict__ S, const double* __restrict__ P,
                                       int m, const double* __restrict__ beta_last, int keep,
                                       double* __restrict__ theta, double* __restrict__ rho)
{
    const double bl = *beta_last;
    for (int i = threadIdx.x; i < keep; i += blockDim.x) {
        theta[i] = S[i];
        rho[i] = bl * P[(int64_t)i * m + (m - 1)];
    }
}

void launch_restart_scalars(const double* S, const double* P, int m, const double* beta_last,
                            int keep, double* theta, double* rho, hipStream_t s)
{
    hipLaunchKernelGGL(restart_scalars_kernel, dim3(1), dim3(256), 0, s, S, P, m, beta_last, keep,
                       theta, rho);
    GKL_LAUNCH_CHECK("restart_scalars_kernel");
}

// ---------------------------------------------------------------------------
// Thick restart from harmonic Ritz vectors (Section 3, "Thick restarting";
// Baglama & Reichel, SIAM J. Sci. Comput. 27, 2005).
//
// After m steps, A V_m = U_m B and A^T U_m = V_{m+1} Bh^T with Bh = [B, beta e_m]
// (m x (m+1)) = Ph diag(sh) Qh^T.  The harmonic Ritz values of A^T A on span(V_m)
// are sh^2, its vectors V_m B^-1 ph_j, and every harmonic residual lies along
// V_{m+1} w with w = [-beta B^-1 e_m; 1].  Bh w = 0, so w is the last right
// singular vector of Bh, and sh_j [B^-1 ph_j; 0] = qh_j - qh_j(m) w / w(m): the
// kept space is span{qh_0..qh_{l-1}, w} and the harmonic vectors are its members
// with a zero last coordinate.  Nothing here needs B^-1 (nearly singular once
// the Krylov space holds a near-null vector of A, as on a wide genotype
// matrix).  The restart keeps
//   U_new = U_m Ph(0:m, 0:l),   V_new = V_{m+1} Z,
// Z = [qh_0..qh_{l-1}, w] times one Householder reflection that zeroes the last
// coordinate of its first l columns, and the projected head and coupling
// column from their definitions: head = Ph_l^T B Z(0:m, 0:l),
// c = Ph_l^T B Z(0:m, l) + Z(m, l) beta Ph(m-1, 0:l).
// ---------------------------------------------------------------------------

// Bpad ((m+1) x (m+1)) = [B, beta e_m; 0]: the SVD kernel takes square input.
__global__ void harmonic_pad_kernel(const double* __restrict__ B, int m,
                                    const double* __restrict__ beta_last, double* __restrict__ Bp)
{
    const int m1 = m + 1;
    const double bl = *beta_last;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m1 * m1; e += gridDim.x * blockDim.x) {
        const int r = e % m1, c = e / m1;
        double v = 0.0;
        if (r < m && c < m) v = B[(int64_t)c * m + r];
        else if (r == m - 1 && c == m) v = bl;
        Bp[e] = v;
    }
}

constexpr int kPlanThreads = 1024;

// One workgroup.  B: m x m (ld m); Ph, Qh: (m+1) x (m+1) (ld m+1), sorted by
// descending singular value (the last column of Qh belongs to the zero one);
// work: >= m * (l + 1) doubles.  Writes Z ((m+1) x (l+1), ld m+1), head (l x l,
// ld l) and c (l).
__global__ void __launch_bounds__(kPlanThreads)
harmonic_plan_kernel(const double* __restrict__ B, int m, const double* __restrict__ beta_last,
                     const double* __restrict__ Ph, const double* __restrict__ Qh, int l,
                     double* __restrict__ work, double* __restrict__ Z, double* __restrict__ head,
                     double* __restrict__ c)
{
    __shared__ double red[16];
    __shared__ double hv[kMaxSvd + 1];     // Householder vector
    const int t = threadIdx.x;
    const int m1 = m + 1;
    const double bl = *beta_last;
    // Z = [qh_0 .. qh_{l-1}, qh_m]
    for (int e = t; e < m1 * (l + 1); e += kPlanThreads) {
        const int r = e % m1, j = e / m1;
        Z[e] = Qh[(int64_t)(j < l ? j : m) * m1 + r];
    }
    __syncthreads();
    // reflection v = z + sign(z_l) |z| e_l of the last row z, applied on the right
    double a = 0.0;
    for (int j = t; j <= l; j += kPlanThreads) {
        const double z = Z[(int64_t)j * m1 + m];
        hv[j] = z;
        a = fma(z, z, a);
    }
    const double nz = sqrt(block_sum(a, red));
    if (t == 0) hv[l] += copysign(nz, hv[l]);
    __syncthreads();
    a = 0.0;
    for (int j = t; j <= l; j += kPlanThreads) a = fma(hv[j], hv[j], a);
    const double vv = block_sum(a, red);
    const double f = vv > 0.0 ? 2.0 / vv : 0.0;
    for (int r = t; r < m1; r += kPlanThreads) {
        double d = 0.0;
        for (int j = 0; j <= l; ++j) d = fma(Z[(int64_t)j * m1 + r], hv[j], d);
        d *= f;
        for (int j = 0; j <= l; ++j) {
            const double z = Z[(int64_t)j * m1 + r] - d * hv[j];
            Z[(int64_t)j * m1 + r] = (r == m && j < l) ? 0.0 : z;
        }
    }
    __syncthreads();
    // work = B Z(0:m, :)  (m x (l+1))
    for (int e = t; e < m * (l + 1); e += kPlanThreads) {
        const int r = e % m, j = e / m;
        const double* z = Z + (int64_t)j * m1;
        double s = 0.0;
        for (int q = 0; q < m; ++q) s = fma(B[(int64_t)q * m + r], z[q], s);
        work[(int64_t)j * m + r] = s;
    }
    __syncthreads();
    // head(i, j) = ph_i^T (B Z_j), c_i = ph_i^T (B Z_l) + Z(m, l) beta ph_i(m-1)
    for (int e = t; e < l * (l + 1); e += kPlanThreads) {
        const int i = e % l, j = e / l;
        const double* p = Ph + (int64_t)i * m1;
        const double* w = work + (int64_t)j * m;
        double s = 0.0;
        for (int r = 0; r < m; ++r) s = fma(p[r], w[r], s);
        if (j < l) head[(int64_t)j * l + i] = s;
        else c[i] = s + Z[(int64_t)l * m1 + m] * bl * p[m - 1];
    }
}

void launch_harmonic_pad(const double* B, int m, const double* beta_last, double* Bp,
                         hipStream_t s)
{
    hipLaunchKernelGGL(harmonic_pad_kernel, dim3(ceil_div((int64_t)(m + 1) * (m + 1), 256)),
                       dim3(256), 0, s, B, m, beta_last, Bp);
    GKL_LAUNCH_CHECK("harmonic_pad_kernel");
}

void launch_harmonic_plan(const double* B, int m, const double* beta_last, const double* Ph,
                          const double* Qh, int l, double* work, double* Z, double* head, double* c,
                          hipStream_t s)
{
    if (m < 2 || m > kMaxSvd || l < 1 || l >= m)
        fail(GKL_ERR_INTERNAL, "harmonic restart plan: bad sizes");
    hipLaunchKernelGGL(harmonic_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, B, m, beta_last,
                       Ph, Qh, l, work, Z, head, c);
    GKL_LAUNCH_CHECK("harmonic_plan_kernel");
}

}  // namespace gkl
