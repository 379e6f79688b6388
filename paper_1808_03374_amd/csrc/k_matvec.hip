// FP64 products with the implicitly standardised genotype matrix (gfx950).
//
//   (A v)_i   = sum_j o_ij (g_ij - mu_j) s_j v_j
//   (A^T u)_j = s_j ( sum_i g_ij u_i - mu_j sum_i o_ij u_i )
//
// Section 3 of the paper: each Lanczos step applies A once and A^T once; these
// two products are where the iteration spends its time.  Genotypes stay 2-bit
// packed in HBM; the dense standardised matrix is never formed.
//
// Both products use lookup tables in LDS so that one byte of four packed codes
// costs one table read and one FP64 add:
//   A v   -- layout T: byte (quad J, individual i) holds the codes of SNPs
//            4J..4J+3 of individual i; for each quad J the 256-entry table
//            L_J[b] = sum_k t_{4J+k}(code_k(b)), t_j(c) = (c - mu_j) s_j v_j for
//            c < 3 and 0 for missing, is built in LDS and every lane adds
//            L_J[byte] into the accumulator of its individual.
//   A^T u -- layout P: byte (individual quad I, SNP j) holds the codes of
//            individuals 4I..4I+3 of SNP j; for each quad I one table holds
//            sum_k g(c_k) u_{4I+k} per byte value and a second, indexed by the
//            byte's missing-code bits, the sum of u over the quad's missing
//            individuals; sum_i o_ij u_i = sum_i u_i - that sum.
// Tables are filled from two 16-entry pair tables (one add per entry).  Both
// store the entry of byte b at position b ^ (b >> 4): the LDS bank of an
// 8-byte entry is set by the low four bits of its position, which for a plain
// table are the codes of the first two SNPs (A v) or individuals (A^T u) only,
// so the most frequent bytes -- those two carry code 0 -- would all fall in one
// bank and conflict; the XOR brings in the other two codes (one extra
// operation per four bytes).  The kernels are bounded by VALU issue and LDS
// reads, so one read and one add per byte beat any decode with more of either.
// Wavefronts read 512 B or 1 KB contiguous per quad row.  Partial sums of the
// K-splits go to a scratch buffer and a second kernel adds them in a fixed
// order (deterministic, no atomics).
#include "pro.h"

namespace gkl {

namespace {
constexpr int kMvThreads = 256;
constexpr int kIPT = 16;                          // A v: individuals per thread (uint4)
constexpr int kRowsPerWave = kWave * kIPT;        // 1024
constexpr int kRowsPerBlock = kMvThreads * kIPT;  // 4096
constexpr int kQCH = 16;                          // A v: SNP quads per table chunk
constexpr int kSPT = 8;                           // A^T u: SNPs per thread (uint2)
constexpr int kColsPerBlock = kMvThreads * kSPT;  // 2048: padding unit of layout P
constexpr int kRmvThreads = 512;                  // A^T u workgroup: one table build serves
constexpr int kRmvCols = kRmvThreads * kSPT;      // 4096 SNPs
constexpr int kQI = 8;                            // A^T u: individual quads per chunk
}  // namespace

int64_t layout_T_rows(int64_t n) { return ((n + kRowsPerWave - 1) / kRowsPerWave) * kRowsPerWave; }
int64_t layout_P_cols(int64_t p) { return ((p + kColsPerBlock - 1) / kColsPerBlock) * kColsPerBlock; }

// ---------------------------------------------------------------------------
// Layout builders (create time)
// ---------------------------------------------------------------------------

// T[J * nT + i] = codes of SNPs 4J..4J+3 of individual i (2 bits each, SNP 4J in
// the low bits); padding individuals and SNPs get code 3.  One thread makes the
// 4 bytes of individuals 4I..4I+3 for quad J (a 4 x 4 transpose of 2-bit fields).
__global__ void build_T_kernel(const uint8_t* __restrict__ G, int64_t n, int64_t p, int64_t ld,
                               uint8_t* __restrict__ T, int64_t nT, int64_t Pq)
{
    const int64_t nbT = nT / 4;
    const int64_t nb = (n + 3) / 4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nbT * Pq;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t J = t / nbT;
        const int64_t I = t - J * nbT;
        uint32_t in[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t j = 4 * J + k;
            uint32_t b = 0xFF;
            if (j < p && I < nb) {
                b = G[j * ld + I];
                const int64_t valid = n - 4 * I;
                if (valid < 4) b |= (0xFFu << (2 * valid)) & 0xFFu;
            }
            in[k] = b;
        }
        uint32_t out = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint32_t byte = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) byte |= ((in[k] >> (2 * r)) & 3u) << (2 * k);
            out |= byte << (8 * r);
        }
        *reinterpret_cast<uint32_t*>(T + J * nT + 4 * I) = out;
    }
}

// P[I * pP + j] = byte I of SNP j (codes of individuals 4I..4I+3); padding is
// code 3.  64 x 64 byte tiles transposed through LDS.
__global__ void build_P_kernel(const uint8_t* __restrict__ G, int64_t n, int64_t p, int64_t ld,
                               uint8_t* __restrict__ P, int64_t pP, int64_t nqP)
{
    __shared__ uint8_t tile[64][65];
    const int64_t j0 = (int64_t)blockIdx.x * 64;     // SNPs
    const int64_t I0 = (int64_t)blockIdx.y * 64;     // individual quads
    const int64_t nb = (n + 3) / 4;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4
    for (int r = ty; r < 64; r += 4) {
        const int64_t j = j0 + r, I = I0 + tx;
        uint32_t b = 0xFF;
        if (j < p && I < nb) {
            b = G[j * ld + I];
            const int64_t valid = n - 4 * I;
            if (valid < 4) b |= (0xFFu << (2 * valid)) & 0xFFu;
        }
        tile[r][tx] = (uint8_t)b;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t I = I0 + r, j = j0 + tx;
        if (I < nqP && j < pP) P[I * pP + j] = tile[tx][r];
    }
}

void layout_shape(int64_t n, int64_t p, Packed& L)
{
    L.n = n;
    L.p = p;
    L.nT = layout_T_rows(n);
    L.Pq = (p + 3) / 4;
    L.pP = layout_P_cols(p);
    L.nq = (n + 3) / 4;
    L.nqP = ((L.nq + kQI - 1) / kQI) * kQI;
}

size_t layout_T_bytes(const Packed& L) { return (size_t)L.nT * (size_t)L.Pq; }
size_t layout_P_bytes(const Packed& L) { return (size_t)L.nqP * (size_t)L.pP; }

void build_layouts(const uint8_t* G, int64_t ld, const Packed& L, hipStream_t s)
{
    const int64_t n = L.n, p = L.p;
    uint8_t* T = const_cast<uint8_t*>(L.T);
    uint8_t* P = const_cast<uint8_t*>(L.P);
    if (T) {
        const int64_t tT = (L.nT / 4) * L.Pq;
        hipLaunchKernelGGL(build_T_kernel, dim3(stride_grid(tT, 256)), dim3(256), 0, s, G, n, p, ld,
                           T, L.nT, L.Pq);
        GKL_LAUNCH_CHECK("build_T_kernel");
    }
    if (!P) return;
    int64_t done = 0;
    const int64_t ytiles = (L.nqP + 63) / 64;
    while (done < ytiles) {   // grid.y <= 65535
        const int64_t chunk = ytiles - done < 65535 ? ytiles - done : 65535;
        hipLaunchKernelGGL(build_P_kernel, dim3(ceil_div(L.pP, 64), (unsigned int)chunk),
                           dim3(256), 0, s, G + done * 64, n - done * 256, p, ld,
                           P + done * 64 * L.pP, L.pP, L.nqP - done * 64);
        GKL_LAUNCH_CHECK("build_P_kernel");
        done += chunk;
    }
}

// ---------------------------------------------------------------------------
// A v: partial[split][i] over the split's SNP quads
// ---------------------------------------------------------------------------
// One tile of A v: rows of row block bx, SNP quads of split by.  Called by the
// single-problem kernel (one tile per workgroup) and by the persistent batched
// kernel (many tiles per workgroup; every thread of the workgroup runs the same
// tiles, and a tile ends with a barrier, so the LDS tables can be reused).
__device__ __forceinline__ void matvec_tile(const uint8_t* __restrict__ T, int64_t nT, int64_t p,
                                            int64_t Pq, const double* __restrict__ mean,
                                            const double* __restrict__ inv_sd,
                                            const double* __restrict__ v, int64_t quads_per_split,
                                            double* __restrict__ partial, int64_t bx, int64_t by)
{
    __shared__ double tv[kQCH * 4 * 4];          // t value per (SNP, code)
    __shared__ double pairs[kQCH * 2 * 16];      // per quad: codes of SNPs (0,1) and (2,3)
    __shared__ double lut[kQCH * 256];           // 32 KB: L_J, entry of byte b at b ^ (b >> 4)
    const int64_t row0 = bx * kRowsPerBlock + (int64_t)threadIdx.x * kIPT;
    const bool active = row0 < nT;
    const int64_t Jb = by * quads_per_split;
    const int64_t Je = Jb + quads_per_split < Pq ? Jb + quads_per_split : Pq;
    double acc[kIPT];
#pragma unroll
    for (int r = 0; r < kIPT; ++r) acc[r] = 0.0;

    for (int64_t J0 = Jb; J0 < Je; J0 += kQCH) {
        const int nq = (int)(Je - J0 < kQCH ? Je - J0 : kQCH);
        uint4 d[kQCH];
#pragma unroll
        for (int q = 0; q < kQCH; ++q) {
            if (active && q < nq) d[q] = *reinterpret_cast<const uint4*>(T + (J0 + q) * nT + row0);
            else d[q] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
        }
        {
            const int s = threadIdx.x;               // 64 SNPs x 4 codes = 256 entries
            const int64_t j = 4 * J0 + (s >> 2);
            const int c = s & 3;
            double val = 0.0;
            if (j < p && c < 3 && (s >> 4) < nq) val = ((double)c - mean[j]) * inv_sd[j] * v[j];
            tv[s] = val;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kQCH * 32; e += kMvThreads) {
            const int q = e >> 5, h = (e >> 4) & 1, x = e & 15;
            const int sa = 4 * q + 2 * h;
            pairs[e] = tv[sa * 4 + (x & 3)] + tv[(sa + 1) * 4 + (x >> 2)];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kQCH * 256; e += kMvThreads) {
            const int q = e >> 8, x = e & 255;
            const int b = x ^ (x >> 4);     // position x holds byte b
            lut[e] = pairs[q * 32 + (b & 15)] + pairs[q * 32 + 16 + (b >> 4)];
        }
        __syncthreads();
        // nT is a multiple of the rows of a wave, so `active` is the same for
        // every lane of a wave: padding waves skip the table reads
        if (active) {
#pragma unroll
            for (int q = 0; q < kQCH; ++q) {
                const double* L = lut + q * 256;
                const uint32_t w[4] = {d[q].x, d[q].y, d[q].z, d[q].w};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint32_t wx = w[t] ^ ((w[t] >> 4) & 0x0F0F0F0Fu);   // table positions
#pragma unroll
                    for (int k = 0; k < 4; ++k) acc[4 * t + k] += L[(wx >> (8 * k)) & 0xFFu];
                }
            }
        }
        __syncthreads();
    }
    if (active) {
        double* out = partial + by * nT + row0;
#pragma unroll
        for (int r = 0; r < kIPT; r += 2)
            *reinterpret_cast<double2*>(out + r) = make_double2(acc[r], acc[r + 1]);
    }
}

__global__ void __launch_bounds__(kMvThreads)
matvec_lut_kernel(const uint8_t* __restrict__ T, int64_t nT, int64_t p, int64_t Pq,
                  const double* __restrict__ mean, const double* __restrict__ inv_sd,
                  const double* __restrict__ v, int64_t quads_per_split,
                  double* __restrict__ partial)
{
    matvec_tile(T, nT, p, Pq, mean, inv_sd, v, quads_per_split, partial, blockIdx.x, blockIdx.y);
}

// y[i] = sum over splits (fixed order within each of 8 split groups, then the
// groups in order) - beta uprev[i]; 32 rows x 8 split groups per block.
constexpr int kRedRows = 32;
constexpr int kRedGroups = 8;

__global__ void __launch_bounds__(kRedRows * kRedGroups)
matvec_reduce_kernel(const double* __restrict__ partial, int64_t nT, int nsplit, int64_t n,
                     double* __restrict__ y, const double* __restrict__ beta,
                     const double* __restrict__ uprev, double* __restrict__ npart)
{
    __shared__ double sh[kRedGroups][kRedRows];
    const int r = threadIdx.x % kRedRows, g = threadIdx.x / kRedRows;
    const int64_t i = (int64_t)blockIdx.x * kRedRows + r;
    double a = 0.0;
    if (i < n) {
        int sp = g;
        for (; sp + 3 * kRedGroups < nsplit; sp += 4 * kRedGroups) {
            const double x0 = partial[(int64_t)sp * nT + i];
            const double x1 = partial[(int64_t)(sp + kRedGroups) * nT + i];
            const double x2 = partial[(int64_t)(sp + 2 * kRedGroups) * nT + i];
            const double x3 = partial[(int64_t)(sp + 3 * kRedGroups) * nT + i];
            a += x0;
            a += x1;
            a += x2;
            a += x3;
        }
        for (; sp < nsplit; sp += kRedGroups) a += partial[(int64_t)sp * nT + i];
    }
    sh[g][r] = a;
    __syncthreads();
    double ss = 0.0;
    if (g == 0 && i < n) {
        double s = 0.0;
        for (int t = 0; t < kRedGroups; ++t) s += sh[t][r];
        if (uprev) s -= (beta ? *beta : 0.0) * uprev[i];
        y[i] = s;
        ss = s * s;
    }
    if (npart) {
        ss = block_sum(ss, sh[0]);
        if (threadIdx.x == 0) npart[blockIdx.x] = ss;
    }
}

// ---------------------------------------------------------------------------
// A^T u: partial[split][j] = sum_i g u - mu_j sum_i o u over the split's quads
// ---------------------------------------------------------------------------
// One tile of A^T u: SNP block bx, individual quads of split by (see matvec_tile).
// Per SNP j the tile forms sum_i g_ij u_i - mu_j sum_i o_ij u_i over its
// individuals.  Each byte costs one read of the quad's genotype table (indexed
// by the byte) and one read of its missing table, indexed by the byte's
// missing-code bits x = byte & (byte >> 1) & 0x55 (bit 2k set when individual k
// of the quad is missing).  x is 0 for almost every byte, so the second read is
// nearly always the same entry for all lanes.  sum_i o_ij u_i is then
// sum_i u_i - sum_i m_ij u_i, with sum_i u_i read from the all-ones entry.
// The genotype table is stored swizzled like the A v table (position
// b ^ (b >> 4)).
constexpr int kMT = 88;   // missing-table entries per quad (x <= 0x55)

// A workgroup of kRmvThreads threads covers kRmvCols SNPs, so one table build
// serves 4096 SNPs.  pP (a multiple of 2048) need not be a multiple of 4096:
// threads past pP -- whole waves, as a wave covers 512 SNPs -- only help
// build the tables.
__device__ __forceinline__ void rmatvec_tile(const uint8_t* __restrict__ P, int64_t pP, int64_t n,
                                             int64_t nq, int64_t p, const double* __restrict__ u,
                                             const double* __restrict__ mean, int64_t iq_per_split,
                                             double* __restrict__ partial, int64_t bx, int64_t by)
{
    __shared__ double uq[kQI * 4];
    __shared__ double pairs[kQI * 2 * 16];
    __shared__ double lut[kQI * 256];            // 16 KB
    __shared__ double mtab[kQI * kMT];           // 5.5 KB
    const int64_t col0 = bx * kRmvCols + (int64_t)threadIdx.x * kSPT;
    const bool live = col0 < pP;
    const int64_t Ib = by * iq_per_split;
    const int64_t Ie = Ib + iq_per_split < nq ? Ib + iq_per_split : nq;
    double sg[kSPT], sm[kSPT];
#pragma unroll
    for (int k = 0; k < kSPT; ++k) { sg[k] = 0.0; sm[k] = 0.0; }
    double su = 0.0;

    for (int64_t I0 = Ib; I0 < Ie; I0 += kQI) {
        const int nqc = (int)(Ie - I0 < kQI ? Ie - I0 : kQI);
        uint2 d[kQI];
#pragma unroll
        for (int q = 0; q < kQI; ++q) {
            if (live && q < nqc) d[q] = *reinterpret_cast<const uint2*>(P + (I0 + q) * pP + col0);
            else d[q] = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
        }
        if (threadIdx.x < kQI * 4) {
            const int64_t i = 4 * I0 + threadIdx.x;
            uq[threadIdx.x] = (i < n && (int)(threadIdx.x >> 2) < nqc) ? u[i] : 0.0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kQI * 32; e += kRmvThreads) {
            const int q = e >> 5, h = (e >> 4) & 1, x = e & 15;
            const int c0 = x & 3, c1 = x >> 2;
            const double u0 = uq[4 * q + 2 * h], u1 = uq[4 * q + 2 * h + 1];
            const double g0 = c0 == 3 ? 0.0 : (double)c0, g1 = c1 == 3 ? 0.0 : (double)c1;
            pairs[e] = g0 * u0 + g1 * u1;
        }
        for (int e = threadIdx.x; e < kQI * kMT; e += kRmvThreads) {
            const int q = e / kMT, x = e - q * kMT;
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if ((x >> (2 * k)) & 1) v += uq[4 * q + k];
            mtab[e] = v;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kQI * 256; e += kRmvThreads) {
            const int q = e >> 8, x = e & 255;
            const int b = x ^ (x >> 4);     // position x holds byte b (see above)
            lut[e] = pairs[q * 32 + (b & 15)] + pairs[q * 32 + 16 + (b >> 4)];
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int q = 0; q < kQI; ++q) {
                const double* L = lut + q * 256;
                const double* M = mtab + q * kMT;
                su += L[0x55 ^ 0x05];                // all four codes 1: the quad's sum of u
                const uint32_t w[2] = {d[q].x, d[q].y};
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const uint32_t mw = w[t] & (w[t] >> 1) & 0x55555555u;
                    const uint32_t wx = w[t] ^ ((w[t] >> 4) & 0x0F0F0F0Fu);   // table positions
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        sg[4 * t + k] += L[(wx >> (8 * k)) & 0xFFu];
                        sm[4 * t + k] += M[(mw >> (8 * k)) & 0xFFu];
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!live) return;
    double* out = partial + by * pP + col0;
#pragma unroll
    for (int k = 0; k < kSPT; k += 2) {
        const int64_t j = col0 + k;
        const double m0 = j < p ? mean[j] : 0.0;
        const double m1 = j + 1 < p ? mean[j + 1] : 0.0;
        *reinterpret_cast<double2*>(out + k) =
            make_double2(sg[k] - m0 * (su - sm[k]), sg[k + 1] - m1 * (su - sm[k + 1]));
    }
}

__global__ void __launch_bounds__(kRmvThreads)
rmatvec_lut_kernel(const uint8_t* __restrict__ P, int64_t pP, int64_t n, int64_t nq, int64_t p,
                   const double* __restrict__ u, const double* __restrict__ mean,
                   int64_t iq_per_split, double* __restrict__ partial)
{
    rmatvec_tile(P, pP, n, nq, p, u, mean, iq_per_split, partial, blockIdx.x, blockIdx.y);
}

__global__ void rmatvec_reduce_kernel(const double* __restrict__ partial, int64_t pP, int nsplit,
                                      int64_t p, const double* __restrict__ inv_sd,
                                      double* __restrict__ z,
                                      const double* __restrict__ alpha,
                                      const double* __restrict__ vprev,
                                      double* __restrict__ npart)
{
    const double a = alpha ? *alpha : 0.0;
    double ss = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double s = strided_sum(partial + j, pP, nsplit);
        double r = inv_sd[j] * s;
        if (vprev) r -= a * vprev[j];
        z[j] = r;
        ss = fma(r, r, ss);
    }
    if (npart) {
        __shared__ double red[16];
        ss = block_sum(ss, red);
        if (threadIdx.x == 0) npart[blockIdx.x] = ss;
    }
}

// The norm (and PRO update) after a reduce kernel that left sums of squares.
__global__ void __launch_bounds__(256) norm_pro_kernel(NormTail t, int nparts)
{
    norm_pro_body(t, nparts);
}

static void launch_norm_pro(const NormTail* t, const MatvecWork& w, int nparts, hipStream_t s)
{
    NormTail x = *t;
    x.npart = w.npart;
    hipLaunchKernelGGL(norm_pro_kernel, dim3(1), dim3(256), 0, s, x, nparts);
    GKL_LAUNCH_CHECK("norm_pro_kernel");
}

// ---------------------------------------------------------------------------
// Launch geometry
// ---------------------------------------------------------------------------
namespace {
struct Split {
    int64_t per_split;
    int nsplit;
};

// Split K (the contraction range, in quads) so that the grid has about `target`
// blocks without making the partial-sum traffic a large share of the stream.
Split choose_split(int64_t kquads, int64_t other_blocks, int64_t chunk, int64_t target,
                   int64_t max_split)
{
    int64_t ns = (target + other_blocks - 1) / other_blocks;
    if (ns > max_split) ns = max_split;
    const int64_t max_by_chunk = (kquads + chunk - 1) / chunk;
    if (ns > max_by_chunk) ns = max_by_chunk;
    if (ns < 1) ns = 1;
    int64_t per = (kquads + ns - 1) / ns;
    per = ((per + chunk - 1) / chunk) * chunk;
    Split s;
    s.per_split = per;
    s.nsplit = (int)((kquads + per - 1) / per);
    return s;
}

constexpr int64_t kSplitTarget = 1536;   // blocks per single-problem launch

Split mv_split(const Packed& L, int64_t target = kSplitTarget)
{
    const int64_t rowblocks = (L.nT + kRowsPerBlock - 1) / kRowsPerBlock;
    // partial traffic nsplit * nT * 8 B kept near 5% of the packed bytes
    int64_t cap = (L.Pq * 4) / 400;
    if (cap < 1) cap = 1;
    return choose_split(L.Pq, rowblocks, kQCH, target, cap);
}

Split rmv_split(const Packed& L, int64_t target = kSplitTarget)
{
    const int64_t colblocks = (L.pP + kRmvCols - 1) / kRmvCols;
    // partial traffic nsplit * pP * 8 B kept near 10% of the packed bytes (the
    // partials mostly stay in the last-level cache)
    int64_t cap = (L.nq * 4) / 320;
    if (cap < 1) cap = 1;
    return choose_split(L.nq, colblocks, kQI, target, cap);
}
}  // namespace

size_t matvec_partial_elems(const Packed& L)
{
    const size_t a = L.limb_mv ? (size_t)L.ms.limbW.nsplit * (size_t)L.ms.nI
                               : (size_t)mv_split(L).nsplit * (size_t)L.nT;
    const size_t b = L.limb_rmv ? (size_t)L.ms.limbX.nsplit * (size_t)L.ms.pS
                                : (size_t)rmv_split(L).nsplit * (size_t)L.pP;
    return a > b ? a : b;
}

size_t matvec_counters(const Packed&) { return 1; }

namespace {
constexpr int64_t kRmvReduceBlocks = 2048;
}

size_t matvec_norm_partials(const Packed& L)
{
    const int64_t a = ceil_div(L.n, kRedRows);
    int64_t b = ceil_div(L.p, 256);
    if (b > kRmvReduceBlocks) b = kRmvReduceBlocks;
    return (size_t)(a > b ? a : b);
}

void launch_matvec(const Packed& L, const ColStats& st, const double* v, double* y,
                   const double* beta, const double* uprev, MatvecWork& w, hipStream_t s,
                   const NormTail* tail, const hipEvent_t* ev)
{
    if (L.limb_mv) {
        const int nsplit = launch_matvec_limb(L.ms, L.I, st, v, w, s, ev);
        hipLaunchKernelGGL(matvec_reduce_kernel, dim3(ceil_div(L.n, kRedRows)),
                           dim3(kRedRows * kRedGroups), 0, s, w.partial, L.ms.nI, nsplit, L.n, y,
                           beta, uprev, tail ? w.npart : nullptr);
        GKL_LAUNCH_CHECK("matvec_reduce_kernel");
        if (tail) launch_norm_pro(tail, w, (int)ceil_div(L.n, kRedRows), s);
        return;
    }
    const Split sp = mv_split(L);
    dim3 grid((unsigned int)((L.nT + kRowsPerBlock - 1) / kRowsPerBlock), (unsigned int)sp.nsplit);
    if (ev) GKL_HIP(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL(matvec_lut_kernel, grid, dim3(kMvThreads), 0, s, L.T, L.nT, L.p, L.Pq,
                       st.mean, st.inv_sd, v, sp.per_split, w.partial);
    GKL_LAUNCH_CHECK("matvec_lut_kernel");
    if (ev) GKL_HIP(hipEventRecord(ev[1], s));
    hipLaunchKernelGGL(matvec_reduce_kernel, dim3(ceil_div(L.n, kRedRows)),
                       dim3(kRedRows * kRedGroups), 0, s, w.partial, L.nT, sp.nsplit, L.n, y, beta,
                       uprev, tail ? w.npart : nullptr);
    GKL_LAUNCH_CHECK("matvec_reduce_kernel");
    if (tail) launch_norm_pro(tail, w, (int)ceil_div(L.n, kRedRows), s);
}

void launch_rmatvec(const Packed& L, const ColStats& st, const double* u, double* z,
                    const double* alpha, const double* vprev, MatvecWork& w, hipStream_t s,
                    const NormTail* tail, const hipEvent_t* ev)
{
    unsigned int nb = ceil_div(L.p, 256);
    if (nb > kRmvReduceBlocks) nb = kRmvReduceBlocks;
    if (L.limb_rmv) {
        const int nsplit = launch_rmatvec_limb(L.ms, L.S, st, u, w, s, ev);
        hipLaunchKernelGGL(rmatvec_reduce_kernel, dim3(nb), dim3(256), 0, s, w.partial, L.ms.pS,
                           nsplit, L.p, st.inv_sd, z, alpha, vprev, tail ? w.npart : nullptr);
        GKL_LAUNCH_CHECK("rmatvec_reduce_kernel");
        if (tail) launch_norm_pro(tail, w, (int)nb, s);
        return;
    }
    const Split sp = rmv_split(L);
    dim3 grid((unsigned int)((L.pP + kRmvCols - 1) / kRmvCols), (unsigned int)sp.nsplit);
    if (ev) GKL_HIP(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL(rmatvec_lut_kernel, grid, dim3(kRmvThreads), 0, s, L.P, L.pP, L.n, L.nq, L.p,
                       u, st.mean, sp.per_split, w.partial);
    GKL_LAUNCH_CHECK("rmatvec_lut_kernel");
    if (ev) GKL_HIP(hipEventRecord(ev[1], s));
    hipLaunchKernelGGL(rmatvec_reduce_kernel, dim3(nb), dim3(256), 0, s, w.partial, L.pP,
                       sp.nsplit, L.p, st.inv_sd, z, alpha, vprev, tail ? w.npart : nullptr);
    GKL_LAUNCH_CHECK("rmatvec_reduce_kernel");
    if (tail) launch_norm_pro(tail, w, (int)nb, s);
}

// ---------------------------------------------------------------------------
// Batched products: one persistent launch covers the tiles of every problem
// ---------------------------------------------------------------------------
ProductPlan product_plan(const Packed& L, int64_t mv_target, int64_t rmv_target)
{
    const Split a = mv_split(L, mv_target), b = rmv_split(L, rmv_target);
    ProductPlan pl;
    pl.mv_per_split = a.per_split;
    pl.mv_nsplit = a.nsplit;
    pl.mv_rowblocks = (int)((L.nT + kRowsPerBlock - 1) / kRowsPerBlock);
    pl.rmv_per_split = b.per_split;
    pl.rmv_nsplit = b.nsplit;
    pl.rmv_colblocks = (int)((L.pP + kRmvCols - 1) / kRmvCols);
    return pl;
}

size_t product_plan_partial_elems(const Packed& L, const ProductPlan& pl)
{
    const size_t a = (size_t)pl.mv_nsplit * (size_t)L.nT;
    const size_t b = (size_t)pl.rmv_nsplit * (size_t)L.pP;
    return a > b ? a : b;
}

namespace {
// Problem owning global tile t: the last q with tile0[q] <= t.
__device__ __forceinline__ int owner(const int* tile0, int count, int t)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile0[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
}  // namespace

__global__ void __launch_bounds__(kMvThreads)
bmatvec_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ tile0, int count,
               const int* __restrict__ state)
{
    __shared__ int t0[kMaxBatch + 1];
    for (int i = threadIdx.x; i <= count; i += blockDim.x) t0[i] = tile0[i];
    __syncthreads();
    const int total = t0[count];
    const int64_t j = state[0];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int q = owner(t0, count, t);
        const BatchDesc& D = desc[q];
        if (!*D.active) continue;            // the same for the whole workgroup
        const int l = t - t0[q];
        matvec_tile(D.T, D.nT, D.p, D.Pq, D.mean, D.inv_sd, D.V + j * D.p, D.mv_per_split,
                    D.partial, l % D.mv_rowblocks, l / D.mv_rowblocks);
    }
}

__global__ void __launch_bounds__(kRmvThreads)
brmatvec_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ tile0, int count,
                const int* __restrict__ state)
{
    __shared__ int t0[kMaxBatch + 1];
    for (int i = threadIdx.x; i <= count; i += blockDim.x) t0[i] = tile0[i];
    __syncthreads();
    const int total = t0[count];
    const int64_t j = state[0];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int q = owner(t0, count, t);
        const BatchDesc& D = desc[q];
        if (!*D.active) continue;
        const int l = t - t0[q];
        rmatvec_tile(D.P, D.pP, D.n, D.nq, D.p, D.U + j * D.n, D.mean, D.rmv_per_split, D.partial,
                     l % D.rmv_colblocks, l / D.rmv_colblocks);
    }
}

// grid (row chunks of the largest n, problems); same summation order as
// matvec_reduce_kernel.
__global__ void __launch_bounds__(kRedRows * kRedGroups)
bmatvec_reduce_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state)
{
    __shared__ double sh[kRedGroups][kRedRows];
    const BatchDesc& D = desc[blockIdx.y];
    if (!*D.active || (int64_t)blockIdx.x * kRedRows >= D.n) return;   // whole workgroup
    const int r = threadIdx.x % kRedRows, g = threadIdx.x / kRedRows;
    const int64_t i = (int64_t)blockIdx.x * kRedRows + r;
    const int64_t n = D.n, nT = D.nT;
    const int nsplit = D.mv_nsplit;
    const double* partial = D.partial;
    double a = 0.0;
    if (i < n) {
        int sp = g;
        for (; sp + 3 * kRedGroups < nsplit; sp += 4 * kRedGroups) {
            const double x0 = partial[(int64_t)sp * nT + i];
            const double x1 = partial[(int64_t)(sp + kRedGroups) * nT + i];
            const double x2 = partial[(int64_t)(sp + 2 * kRedGroups) * nT + i];
            const double x3 = partial[(int64_t)(sp + 3 * kRedGroups) * nT + i];
            a += x0;
            a += x1;
            a += x2;
            a += x3;
        }
        for (; sp < nsplit; sp += kRedGroups) a += partial[(int64_t)sp * nT + i];
    }
    sh[g][r] = a;
    __syncthreads();
    if (g == 0 && i < n) {
        double s = 0.0;
        for (int t = 0; t < kRedGroups; ++t) s += sh[t][r];
        const int j = state[0], nlock = state[1];
        if (j > 0 && j == nlock) {
            for (int c = 0; c < nlock; ++c) s -= D.rho[c] * D.U[(int64_t)c * n + i];
        } else if (j > 0) {
            s -= D.beta[j - 1] * D.U[(int64_t)(j - 1) * n + i];
        }
        D.U[(int64_t)j * n + i] = s;
    }
}

__global__ void __launch_bounds__(256)
brmatvec_reduce_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state)
{
    const BatchDesc& D = desc[blockIdx.y];
    if (!*D.active) return;
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= D.p) return;
    const int j = state[0];
    const double s = strided_sum(D.partial + jj, D.pP, D.rmv_nsplit);
    double r = D.inv_sd[jj] * s;
    r -= D.alpha[j] * D.V[(int64_t)j * D.p + jj];
    D.V[(int64_t)(j + 1) * D.p + jj] = r;
}

void launch_bmatvec(const BatchDesc* d, const int* tile0, int count, const int* state, int grid,
                    hipStream_t s)
{
    hipLaunchKernelGGL(bmatvec_kernel, dim3(grid), dim3(kMvThreads), 0, s, d, tile0, count, state);
    GKL_LAUNCH_CHECK("bmatvec_kernel");
}

void launch_brmatvec(const BatchDesc* d, const int* tile0, int count, const int* state, int grid,
                     hipStream_t s)
{
    hipLaunchKernelGGL(brmatvec_kernel, dim3(grid), dim3(kRmvThreads), 0, s, d, tile0, count, state);
    GKL_LAUNCH_CHECK("brmatvec_kernel");
}

void launch_bmatvec_reduce(const BatchDesc* d, const int* state, int count, int64_t max_n,
                           hipStream_t s)
{
    hipLaunchKernelGGL(bmatvec_reduce_kernel, dim3(ceil_div(max_n, kRedRows), count),
                       dim3(kRedRows * kRedGroups), 0, s, d, state);
    GKL_LAUNCH_CHECK("bmatvec_reduce_kernel");
}

void launch_brmatvec_reduce(const BatchDesc* d, const int* state, int count, int64_t max_p,
                            hipStream_t s)
{
    hipLaunchKernelGGL(brmatvec_reduce_kernel, dim3(ceil_div(max_p, 256), count), dim3(256), 0, s,
                       d, state);
    GKL_LAUNCH_CHECK("brmatvec_reduce_kernel");
}

}  // namespace gkl
