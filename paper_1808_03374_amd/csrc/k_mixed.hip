// Blocked products A W and A^T X on MFMA with split-BF16 vector tiles (gfx950).
//
// Section 5 of the paper names block Lanczos (many vectors per pass, BLAS3) as
// the next step; with b vectors per pass the product becomes a dense contraction
// and runs on the matrix cores.
//
// Exact operands.  Genotype codes are decoded in registers to two exact BF16
// operands: g (0, 1, 2; 0 for missing) and the missing indicator m (0 or 1).
// Two codes of a 32-bit word form one pair word: a shift and a mask isolate
// them, one 24-bit multiply-add turns them into a byte selector, and v_perm_b32
// reads both BF16 values from an 8-byte table held in two constants (one table
// for g, one for m).  The vector block is split into BF16 hi + lo (hi = bf16(w),
// lo = bf16(w - hi)), accumulated in FP32 per K-chunk and in FP64 across chunks
// and splits.
//
//   A W   (contract over SNPs, layout I: row = individual):
//     sum_j A_ij W_jc = sum_j g_ij W'_jc + sum_j m_ij X'_jc - sum_j X'_jc
//     W' = s W, X' = mu s W   (o = 1 - m)
//   A^T X (contract over individuals, layout S: row = SNP):
//     sum_i A_ij X_ic = s_j ( sum_i g_ij X_ic - mu_j T_c + mu_j sum_i m_ij X_ic )
//     T_c = sum_i X_ic
//
// MFMA v_mfma_f32_16x16x32_bf16: A lane l holds row l%16, B lane l column l%16,
// both with the K slice selected by (l/16, element); C lane l element e is row
// 4*(l/16)+e, column l%16.  A lane's 16 codes of one 32-bit word feed two K
// steps; element e of K step h is code 4h + (e>>1) + 8(e&1) of that word, and the
// vector fragments are written in the same order.
#include "kernels.h"

namespace gkl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kSuper = 256;            // K per super-tile (64 bytes of codes per row)
constexpr int kKSteps = kSuper / 32;   // MFMA K steps per super-tile
constexpr int kMxWaves = 4;
constexpr int kRTw = 8;                // A W: row tiles per wave
constexpr int kRTr = 4;                // A^T X: row tiles per wave
constexpr int kFlush = 4;              // super-tiles per FP32 chunk
}  // namespace

int64_t mixed_rows_I(int64_t n) { return ((n + 511) / 512) * 512; }
int64_t mixed_ld_I(int64_t p) { return (((p + 3) / 4 + 63) / 64) * 64; }
int64_t mixed_rows_S(int64_t p) { return ((p + 255) / 256) * 256; }
int64_t mixed_ld_S(int64_t n) { return (((n + 3) / 4 + 63) / 64) * 64; }

// ---------------------------------------------------------------------------
// Layouts
// ---------------------------------------------------------------------------
// Both layouts are stored in 1 KB tiles of 16 rows x 64 bytes, tile (rt, st) at
// byte (rt * (ld / 64) + st) * 1024 and row r of the tile at + r * 64, so that one
// wave's 16-byte-per-lane load of a tile reads 1 KB of consecutive bytes and a
// wave walking along K streams through consecutive tiles.
__host__ __device__ __forceinline__ int64_t tiled_offset(int64_t row, int64_t byte, int64_t ld)
{
    return ((row >> 4) * (ld >> 6) + (byte >> 6)) * 1024 + (row & 15) * 64 + (byte & 63);
}

// I: byte J of individual i = codes of SNPs 4J..4J+3 of individual i (tiled, ld
// = ldI); padding = code 3.
__global__ void build_I_kernel(const uint8_t* __restrict__ G, int64_t n, int64_t p, int64_t ld,
                               uint8_t* __restrict__ I, int64_t nI, int64_t ldI)
{
    const int64_t nb = (n + 3) / 4;
    const int64_t nrq = nI / 4;
    // t = (SNP quad J, individual quad Iq)
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nrq * ldI;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t J = t / nrq;
        const int64_t Iq = t - J * nrq;
        uint32_t in[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t j = 4 * J + k;
            uint32_t b = 0xFF;
            if (j < p && Iq < nb) {
                b = G[j * ld + Iq];
                const int64_t valid = n - 4 * Iq;
                if (valid < 4) b |= (0xFFu << (2 * valid)) & 0xFFu;
            }
            in[k] = b;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint32_t byte = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) byte |= ((in[k] >> (2 * r)) & 3u) << (2 * k);
            I[tiled_offset(4 * Iq + r, J, ldI)] = (uint8_t)byte;
        }
    }
}

// S: byte Iq of SNP j = codes of individuals 4Iq..4Iq+3 (tiled, ld = ldS);
// padding = code 3.
__global__ void build_S_kernel(const uint8_t* __restrict__ G, int64_t n, int64_t p, int64_t ld,
                               uint8_t* __restrict__ S, int64_t pS, int64_t ldS)
{
    const int64_t nb = (n + 3) / 4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < pS * ldS;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / ldS;
        const int64_t Iq = t - j * ldS;
        uint32_t b = 0xFF;
        if (j < p && Iq < nb) {
            b = G[j * ld + Iq];
            const int64_t valid = n - 4 * Iq;
            if (valid < 4) b |= (0xFFu << (2 * valid)) & 0xFFu;
        }
        S[tiled_offset(j, Iq, ldS)] = (uint8_t)b;
    }
}

void build_mixed_layouts(const uint8_t* G, int64_t n, int64_t p, int64_t ld, uint8_t* I,
                         uint8_t* S, hipStream_t s)
{
    const int64_t nI = mixed_rows_I(n), ldI = mixed_ld_I(p);
    const int64_t pS = mixed_rows_S(p), ldS = mixed_ld_S(n);
    const int64_t tI = (nI / 4) * ldI;
    hipLaunchKernelGGL(build_I_kernel, dim3(stride_grid(tI, 256)), dim3(256), 0, s, G, n, p, ld, I,
                       nI, ldI);
    GKL_LAUNCH_CHECK("build_I_kernel");
    const int64_t tS = pS * ldS;
    hipLaunchKernelGGL(build_S_kernel, dim3(stride_grid(tS, 256)), dim3(256), 0, s, G, n, p, ld, S,
                       pS, ldS);
    GKL_LAUNCH_CHECK("build_S_kernel");
}

// ---------------------------------------------------------------------------
// Decode: 16 codes of a word -> 8 pair words of each pattern
// ---------------------------------------------------------------------------
__device__ __forceinline__ void decode16(uint32_t d, uint32_t C[8], uint32_t M[8])
{
    // table bytes {S0:S1} = [lo(c=0), hi(c=0), lo(1), hi(1), lo(2), hi(2), lo(3), hi(3)]
    constexpr uint32_t kG1 = 0x3F800000u, kG0 = 0x00004000u;   // g: 0, 1.0, 2.0, 0
    constexpr uint32_t kM1 = 0x00000000u, kM0 = 0x3F800000u;   // m: 0, 0, 0, 1.0
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t u = (d >> (2 * k)) & 0x00030003u;        // code k (byte 0), k+8 (byte 2)
        const uint32_t sel = u * 0x0202u + 0x01000100u;        // [2c, 2c+1, 2c', 2c'+1]
        C[k] = __builtin_amdgcn_perm(kG0, kG1, sel);
        M[k] = __builtin_amdgcn_perm(kM0, kM1, sel);
    }
}

__device__ __forceinline__ bf16x8 pack4(uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 v = {a, b, c, d};
    return __builtin_bit_cast(bf16x8, v);
}

// position (within the lane's 16-code word) of element e of K step h
__host__ __device__ __forceinline__ int code_pos(int h, int e) { return 4 * h + (e >> 1) + 8 * (e & 1); }

__device__ __forceinline__ __bf16 to_bf16(double v) { return (__bf16)(float)v; }

// ---------------------------------------------------------------------------
// Vector fragments
// ---------------------------------------------------------------------------
// A W operands.  kPack == false: frag[((st*8 + t)*4 + op)*64 + lane][e], ops
// 0..3 = W'hi, W'lo, X'hi, X'lo for the 16 columns starting at col0.
// kPack == true (b <= 8): two operands whose 16 columns hold the hi parts of the
// b columns in 0..7 and their lo parts in 8..15: op 0 = [W'hi | W'lo], op 1 =
// [X'hi | X'lo]; one MFMA per operand then covers both halves of the split.
template <bool kPack>
__global__ void split_W_kernel(const double* __restrict__ W, int64_t ldw, int b, int col0,
                               int64_t p, const double* __restrict__ mean,
                               const double* __restrict__ inv_sd, int64_t nst,
                               bf16x8* __restrict__ frag)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (st, ks, lane)
    if (t >= nst * kKSteps * 64) return;
    const int lane = (int)(t & 63);
    const int ks = (int)((t >> 6) % kKSteps);
    const int64_t st = t / (64 * kKSteps);
    const int g = lane >> 4;
    const int col = kPack ? (lane & 7) : col0 + (lane & 15);
    const bool hi_half = !kPack || (lane & 15) < 8;
    bf16x8 whi, wlo, zhi, zlo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t j = st * kSuper + 64 * g + 16 * (ks >> 1) + code_pos(ks & 1, e);
        double w = 0.0, z = 0.0;
        if (j < p && col < b) {
            w = inv_sd[j] * W[(int64_t)col * ldw + j];
            z = mean[j] * w;
        }
        const __bf16 h1 = to_bf16(w), h2 = to_bf16(z);
        const __bf16 l1 = to_bf16(w - (double)(float)h1), l2 = to_bf16(z - (double)(float)h2);
        whi[e] = hi_half ? h1 : l1;
        zhi[e] = hi_half ? h2 : l2;
        wlo[e] = l1;
        zlo[e] = l2;
    }
    if (kPack) {
        bf16x8* f = frag + (((st * kKSteps + ks) * 2) * 64) + lane;
        f[0 * 64] = whi;
        f[1 * 64] = zhi;
    } else {
        bf16x8* f = frag + (((st * kKSteps + ks) * 4) * 64) + lane;
        f[0 * 64] = whi;
        f[1 * 64] = wlo;
        f[2 * 64] = zhi;
        f[3 * 64] = zlo;
    }
}

// Column sums over len rows: sum_j f_j X(j, c), with f_j = mean_j inv_sd_j when
// mean != NULL (the product mean_j (inv_sd_j x) is formed in that order) and
// f_j = 1 otherwise (per column c: K2_c = sum_j mu_j s_j W_jc for A W, T_c =
// sum_i X_ic for A^T X).  grid (kCsSplit, columns): each block sums one chunk
// of rows into cpart[c * kCsSplit + chunk]; the reduce kernel that consumes the
// sums adds the chunk sums (column_sums).  No cross-block handshake: its
// device-scope fences cost more than the consumer's 64 extra reads.
constexpr int kCsSplit = 64;   // == wavefront size (the chunk sums are added by one wave)

__global__ void __launch_bounds__(256)
colsum_kernel(const double* __restrict__ X, int64_t ldx, int64_t len,
              const double* __restrict__ mean, const double* __restrict__ inv_sd,
              double* __restrict__ cpart)
{
    __shared__ double sh[16];
    const int c = blockIdx.y;
    const int64_t chunk = (len + kCsSplit - 1) / kCsSplit;
    const int64_t j0 = (int64_t)blockIdx.x * chunk;
    const int64_t j1 = j0 + chunk < len ? j0 + chunk : len;
    const double* xc = X + (int64_t)c * ldx;
    double a = 0.0;
    if (mean) {
        for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) a += mean[j] * (inv_sd[j] * xc[j]);
    } else {
        for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) a += xc[j];
    }
    a = block_sum(a, sh);
    if (threadIdx.x == 0) cpart[c * kCsSplit + blockIdx.x] = a;
}

// ks[c] for c < nb: the kCsSplit chunk sums of column c added by one wave in a
// fixed butterfly (every block of the consumer gets the same bits).  Called by
// every thread of the block.
__device__ __forceinline__ void column_sums(const double* __restrict__ cpart, int nb, double* ks)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = wave; c < nb; c += (int)(blockDim.x >> 6)) {
        const double t = wave_sum(cpart[c * kCsSplit + lane]);
        if (lane == 0) ks[c] = t;
    }
    __syncthreads();
}

// A^T X operands.  kPack == false: frag[((st*8 + t)*2 + op)*64 + lane][e], ops
// 0..1 = Xhi, Xlo.  kPack == true (b <= 8): one operand [Xhi | Xlo] (hi parts in
// columns 0..7, lo parts in 8..15), frag[(st*8 + t)*64 + lane].
template <bool kPack>
__global__ void split_X_kernel(const double* __restrict__ X, int64_t ldx, int b, int col0,
                               int64_t n, int64_t nst, bf16x8* __restrict__ frag)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nst * kKSteps * 64) return;
    const int lane = (int)(t & 63);
    const int ks = (int)((t >> 6) % kKSteps);
    const int64_t st = t / (64 * kKSteps);
    const int g = lane >> 4;
    const int col = kPack ? (lane & 7) : col0 + (lane & 15);
    const bool hi_half = !kPack || (lane & 15) < 8;
    bf16x8 xhi, xlo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t i = st * kSuper + 64 * g + 16 * (ks >> 1) + code_pos(ks & 1, e);
        double x = 0.0;
        if (i < n && col < b) x = X[(int64_t)col * ldx + i];
        const __bf16 h = to_bf16(x);
        const __bf16 l = to_bf16(x - (double)(float)h);
        xhi[e] = hi_half ? h : l;
        xlo[e] = l;
    }
    if (kPack) {
        frag[(st * kKSteps + ks) * 64 + lane] = xhi;
    } else {
        bf16x8* f = frag + (((st * kKSteps + ks) * 2) * 64) + lane;
        f[0] = xhi;
        f[64] = xlo;
    }
}

// ---------------------------------------------------------------------------
// A W main kernel: block = 4 waves x 8 row tiles x 16 rows = 512 rows, K split in
// super-tiles; partial[split][row][16] FP64.
// ---------------------------------------------------------------------------
template <bool kPack>
__global__ void __launch_bounds__(256)
matmat_bf16_kernel(const uint8_t* __restrict__ I, int64_t ldI, int64_t nI,
                   const bf16x8* __restrict__ frag, int64_t nst, int64_t st_per_split,
                   double* __restrict__ partial)
{
    constexpr int kOps = kPack ? 2 : 4;
    __shared__ bf16x8 bs[kKSteps * kOps * 64];      // one super-tile of the operands
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    const int64_t row_base = (int64_t)blockIdx.x * (kMxWaves * kRTw * 16) + wave * (kRTw * 16);
    const int64_t st0 = (int64_t)blockIdx.y * st_per_split;
    const int64_t st1 = st0 + st_per_split < nst ? st0 + st_per_split : nst;
    f32x4 acc[kRTw];
    double accd[kRTw][4];
#pragma unroll
    for (int t = 0; t < kRTw; ++t) {
        acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int e = 0; e < 4; ++e) accd[t][e] = 0.0;
    }
    int chunk = 0;
    for (int64_t st = st0; st < st1; ++st) {
        uint4 a[kRTw];
#pragma unroll
        for (int t = 0; t < kRTw; ++t)
            a[t] = *reinterpret_cast<const uint4*>(I + tiled_offset(row_base + 16 * t + r, st * 64 + 16 * g, ldI));
        const bf16x8* src = frag + st * (kKSteps * kOps * 64);
        for (int q = threadIdx.x; q < kKSteps * kOps * 64; q += 256) bs[q] = src[q];
        __syncthreads();
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            bf16x8 bw0[2], bw1[2], bz0[2], bz1[2];   // W'hi, W'lo, X'hi, X'lo (packed: 0 only)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ks = 2 * w + h;
                if (kPack) {
                    bw0[h] = bs[(ks * 2 + 0) * 64 + lane];
                    bz0[h] = bs[(ks * 2 + 1) * 64 + lane];
                } else {
                    bw0[h] = bs[(ks * 4 + 0) * 64 + lane];
                    bw1[h] = bs[(ks * 4 + 1) * 64 + lane];
                    bz0[h] = bs[(ks * 4 + 2) * 64 + lane];
                    bz1[h] = bs[(ks * 4 + 3) * 64 + lane];
                }
            }
#pragma unroll
            for (int t = 0; t < kRTw; ++t) {
                const uint32_t d = w == 0 ? a[t].x : w == 1 ? a[t].y : w == 2 ? a[t].z : a[t].w;
                uint32_t C[8], M[8];
                decode16(d, C, M);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bf16x8 ca = pack4(C[4 * h], C[4 * h + 1], C[4 * h + 2], C[4 * h + 3]);
                    const bf16x8 ma = pack4(M[4 * h], M[4 * h + 1], M[4 * h + 2], M[4 * h + 3]);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ca, bw0[h], acc[t], 0, 0, 0);
                    if (!kPack)
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ca, bw1[h], acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ma, bz0[h], acc[t], 0, 0, 0);
                    if (!kPack)
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ma, bz1[h], acc[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();
        if (++chunk == kFlush) {
            chunk = 0;
#pragma unroll
            for (int t = 0; t < kRTw; ++t) {
#pragma unroll
                for (int e = 0; e < 4; ++e) accd[t][e] += (double)acc[t][e];
                acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
        }
    }
    double* out = partial + (int64_t)blockIdx.y * nI * 16;
#pragma unroll
    for (int t = 0; t < kRTw; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t row = row_base + 16 * t + 4 * g + e;
            out[row * 16 + r] = accd[t][e] + (double)acc[t][e];
        }
    }
}

// Y[i + c*ldy] = sum_split partial - K2_c for i < n, c < nb (col0 offset); packed:
// the hi (column c) and lo (column c + 8) partials of each split are added first.
template <bool kPack>
__global__ void __launch_bounds__(256)
matmat_reduce_kernel(const double* __restrict__ partial, int nsplit, int64_t nI, int64_t n,
                     int nb, const double* __restrict__ cpart, double* __restrict__ Y,
                     int64_t ldy)
{
    __shared__ double K2[16];
    column_sums(cpart, nb, K2);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 16) return;
    const int64_t i = t >> 4;
    const int c = (int)(t & 15);
    if (c >= nb) return;
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) {
        const double* pr = partial + ((int64_t)sp * nI + i) * 16;
        s += kPack ? pr[c] + pr[c + 8] : pr[c];
    }
    Y[(int64_t)c * ldy + i] = s - K2[c];
}

// ---------------------------------------------------------------------------
// A^T X main kernel: block = 4 waves x 4 SNP tiles x 16 = 256 SNPs; K = individuals.
// partial[split][2][row][16]: sums with the code operand and the missing operand.
// ---------------------------------------------------------------------------
template <bool kPack>
__global__ void __launch_bounds__(256)
rmatmat_bf16_kernel(const uint8_t* __restrict__ S, int64_t ldS, int64_t pS,
                    const bf16x8* __restrict__ frag, int64_t nst, int64_t st_per_split,
                    double* __restrict__ partial)
{
    constexpr int kOps = kPack ? 1 : 2;
    __shared__ bf16x8 bs[kKSteps * kOps * 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    const int64_t row_base = (int64_t)blockIdx.x * (kMxWaves * kRTr * 16) + wave * (kRTr * 16);
    const int64_t st0 = (int64_t)blockIdx.y * st_per_split;
    const int64_t st1 = st0 + st_per_split < nst ? st0 + st_per_split : nst;
    f32x4 accC[kRTr], accM[kRTr];
    double dC[kRTr][4], dM[kRTr][4];
#pragma unroll
    for (int t = 0; t < kRTr; ++t) {
        accC[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        accM[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int e = 0; e < 4; ++e) { dC[t][e] = 0.0; dM[t][e] = 0.0; }
    }
    int chunk = 0;
    for (int64_t st = st0; st < st1; ++st) {
        uint4 a[kRTr];
#pragma unroll
        for (int t = 0; t < kRTr; ++t)
            a[t] = *reinterpret_cast<const uint4*>(S + tiled_offset(row_base + 16 * t + r, st * 64 + 16 * g, ldS));
        const bf16x8* src = frag + st * (kKSteps * kOps * 64);
        for (int q = threadIdx.x; q < kKSteps * kOps * 64; q += 256) bs[q] = src[q];
        __syncthreads();
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            bf16x8 x0[2], x1[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ks = 2 * w + h;
                if (kPack) {
                    x0[h] = bs[ks * 64 + lane];
                } else {
                    x0[h] = bs[(ks * 2 + 0) * 64 + lane];
                    x1[h] = bs[(ks * 2 + 1) * 64 + lane];
                }
            }
#pragma unroll
            for (int t = 0; t < kRTr; ++t) {
                const uint32_t d = w == 0 ? a[t].x : w == 1 ? a[t].y : w == 2 ? a[t].z : a[t].w;
                uint32_t C[8], M[8];
                decode16(d, C, M);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bf16x8 ca = pack4(C[4 * h], C[4 * h + 1], C[4 * h + 2], C[4 * h + 3]);
                    const bf16x8 ma = pack4(M[4 * h], M[4 * h + 1], M[4 * h + 2], M[4 * h + 3]);
                    accC[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ca, x0[h], accC[t], 0, 0, 0);
                    if (!kPack)
                        accC[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ca, x1[h], accC[t], 0, 0, 0);
                    accM[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ma, x0[h], accM[t], 0, 0, 0);
                    if (!kPack)
                        accM[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ma, x1[h], accM[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();
        if (++chunk == kFlush) {
            chunk = 0;
#pragma unroll
            for (int t = 0; t < kRTr; ++t) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    dC[t][e] += (double)accC[t][e];
                    dM[t][e] += (double)accM[t][e];
                }
                accC[t] = f32x4{0.f, 0.f, 0.f, 0.f};
                accM[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
        }
    }
    double* out = partial + (int64_t)blockIdx.y * 2 * pS * 16;
#pragma unroll
    for (int t = 0; t < kRTr; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t row = row_base + 16 * t + 4 * g + e;
            out[row * 16 + r] = dC[t][e] + (double)accC[t][e];
            out[(pS + row) * 16 + r] = dM[t][e] + (double)accM[t][e];
        }
    }
}

// Z[j + c*ldz] = s_j ( SG - mu_j T_c + mu_j SM )
template <bool kPack>
__global__ void __launch_bounds__(256)
rmatmat_reduce_kernel(const double* __restrict__ partial, int nsplit, int64_t pS, int64_t p,
                      int nb, const double* __restrict__ cpart, const double* __restrict__ mean,
                      const double* __restrict__ inv_sd, double* __restrict__ Z, int64_t ldz)
{
    __shared__ double T[16];
    column_sums(cpart, nb, T);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * 16) return;
    const int64_t j = t >> 4;
    const int c = (int)(t & 15);
    if (c >= nb) return;
    double sc = 0.0, sm = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) {
        const double* pc = partial + ((int64_t)sp * 2 * pS + j) * 16;
        const double* pm = partial + ((int64_t)sp * 2 * pS + pS + j) * 16;
        sc += kPack ? pc[c] + pc[c + 8] : pc[c];
        sm += kPack ? pm[c] + pm[c + 8] : pm[c];
    }
    const double mu = mean[j];
    Z[(int64_t)c * ldz + j] = inv_sd[j] * (sc - mu * T[c] + mu * sm);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
MixedShape mixed_shape(int64_t n, int64_t p)
{
    MixedShape m;
    m.n = n;
    m.p = p;
    m.nI = mixed_rows_I(n);
    m.ldI = mixed_ld_I(p);
    m.pS = mixed_rows_S(p);
    m.ldS = mixed_ld_S(n);
    m.nstW = m.ldI / 64;                     // super-tiles along SNPs
    m.nstX = m.ldS / 64;                     // super-tiles along individuals
    // K splits: enough blocks to fill the GPU, partial traffic bounded
    const int64_t rbW = m.nI / (kMxWaves * kRTw * 16);
    int64_t sW = (1024 + rbW - 1) / rbW;
    const int64_t capW = m.nstW / 8 > 1 ? m.nstW / 8 : 1;   // >= 2048 SNPs per split
    if (sW > capW) sW = capW;
    if (sW < 1) sW = 1;
    m.stW = (m.nstW + sW - 1) / sW;
    m.splitW = (int)((m.nstW + m.stW - 1) / m.stW);
    const int64_t rbX = m.pS / (kMxWaves * kRTr * 16);
    int64_t sX = (1024 + rbX - 1) / rbX;
    const int64_t capX = m.nstX / 8 > 1 ? m.nstX / 8 : 1;
    if (sX > capX) sX = capX;
    if (sX < 1) sX = 1;
    m.stX = (m.nstX + sX - 1) / sX;
    m.splitX = (int)((m.nstX + m.stX - 1) / m.stX);
    return m;
}

size_t mixed_frag_bytes(const MixedShape& m)
{
    const size_t a = (size_t)m.nstW * kKSteps * 4 * 64 * sizeof(bf16x8);
    const size_t b = (size_t)m.nstX * kKSteps * 2 * 64 * sizeof(bf16x8);
    return a > b ? a : b;
}

size_t mixed_partial_elems(const MixedShape& m)
{
    const size_t a = (size_t)m.splitW * (size_t)m.nI * 16;
    const size_t b = (size_t)m.splitX * 2 * (size_t)m.pS * 16;
    return a > b ? a : b;
}

void launch_matmat_mixed(const MixedShape& m, const uint8_t* I, const ColStats& st,
                         const double* W, int64_t ldw, int b, double* Y, int64_t ldy,
                         MixedWork& w, hipStream_t s)
{
    const bool pack = b <= 8;
    for (int col0 = 0; col0 < b; col0 += 16) {
        const int nb = b - col0 < 16 ? b - col0 : 16;
        const int64_t nthr = m.nstW * kKSteps * 64;
        const dim3 gsplit(ceil_div(nthr, 256));
        if (pack)
            hipLaunchKernelGGL(split_W_kernel<true>, gsplit, dim3(256), 0, s, W, ldw, b, col0, m.p,
                               st.mean, st.inv_sd, m.nstW, reinterpret_cast<bf16x8*>(w.frag));
        else
            hipLaunchKernelGGL(split_W_kernel<false>, gsplit, dim3(256), 0, s, W, ldw, b, col0, m.p,
                               st.mean, st.inv_sd, m.nstW, reinterpret_cast<bf16x8*>(w.frag));
        GKL_LAUNCH_CHECK("split_W_kernel");
        hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, nb), dim3(256), 0, s,
                           W + (int64_t)col0 * ldw, ldw, m.p, st.mean, st.inv_sd, w.cpart);
        GKL_LAUNCH_CHECK("colsum_kernel");
        dim3 grid((unsigned int)(m.nI / (kMxWaves * kRTw * 16)), (unsigned int)m.splitW);
        if (pack)
            hipLaunchKernelGGL(matmat_bf16_kernel<true>, grid, dim3(256), 0, s, I, m.ldI, m.nI,
                               reinterpret_cast<const bf16x8*>(w.frag), m.nstW, m.stW, w.partial);
        else
            hipLaunchKernelGGL(matmat_bf16_kernel<false>, grid, dim3(256), 0, s, I, m.ldI, m.nI,
                               reinterpret_cast<const bf16x8*>(w.frag), m.nstW, m.stW, w.partial);
        GKL_LAUNCH_CHECK("matmat_bf16_kernel");
        const dim3 gred(ceil_div(m.n * 16, 256));
        if (pack)
            hipLaunchKernelGGL(matmat_reduce_kernel<true>, gred, dim3(256), 0, s, w.partial,
                               m.splitW, m.nI, m.n, nb, w.cpart, Y + (int64_t)col0 * ldy, ldy);
        else
            hipLaunchKernelGGL(matmat_reduce_kernel<false>, gred, dim3(256), 0, s, w.partial,
                               m.splitW, m.nI, m.n, nb, w.cpart, Y + (int64_t)col0 * ldy, ldy);
        GKL_LAUNCH_CHECK("matmat_reduce_kernel");
    }
}

void launch_rmatmat_mixed(const MixedShape& m, const uint8_t* S, const ColStats& st,
                          const double* X, int64_t ldx, int b, double* Z, int64_t ldz,
                          MixedWork& w, hipStream_t s)
{
    const bool pack = b <= 8;
    for (int col0 = 0; col0 < b; col0 += 16) {
        const int nb = b - col0 < 16 ? b - col0 : 16;
        const int64_t nthr = m.nstX * kKSteps * 64;
        const dim3 gsplit(ceil_div(nthr, 256));
        if (pack)
            hipLaunchKernelGGL(split_X_kernel<true>, gsplit, dim3(256), 0, s, X, ldx, b, col0, m.n,
                               m.nstX, reinterpret_cast<bf16x8*>(w.frag));
        else
            hipLaunchKernelGGL(split_X_kernel<false>, gsplit, dim3(256), 0, s, X, ldx, b, col0, m.n,
                               m.nstX, reinterpret_cast<bf16x8*>(w.frag));
        GKL_LAUNCH_CHECK("split_X_kernel");
        hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, nb), dim3(256), 0, s,
                           X + (int64_t)col0 * ldx, ldx, m.n, nullptr, nullptr, w.cpart);
        GKL_LAUNCH_CHECK("colsum_kernel");
        dim3 grid((unsigned int)(m.pS / (kMxWaves * kRTr * 16)), (unsigned int)m.splitX);
        if (pack)
            hipLaunchKernelGGL(rmatmat_bf16_kernel<true>, grid, dim3(256), 0, s, S, m.ldS, m.pS,
                               reinterpret_cast<const bf16x8*>(w.frag), m.nstX, m.stX, w.partial);
        else
            hipLaunchKernelGGL(rmatmat_bf16_kernel<false>, grid, dim3(256), 0, s, S, m.ldS, m.pS,
                               reinterpret_cast<const bf16x8*>(w.frag), m.nstX, m.stX, w.partial);
        GKL_LAUNCH_CHECK("rmatmat_bf16_kernel");
        const dim3 gred(ceil_div(m.p * 16, 256));
        if (pack)
            hipLaunchKernelGGL(rmatmat_reduce_kernel<true>, gred, dim3(256), 0, s, w.partial,
                               m.splitX, m.pS, m.p, nb, w.cpart, st.mean, st.inv_sd,
                               Z + (int64_t)col0 * ldz, ldz);
        else
            hipLaunchKernelGGL(rmatmat_reduce_kernel<false>, gred, dim3(256), 0, s, w.partial,
                               m.splitX, m.pS, m.p, nb, w.cpart, st.mean, st.inv_sd,
                               Z + (int64_t)col0 * ldz, ldz);
        GKL_LAUNCH_CHECK("rmatmat_reduce_kernel");
    }
}

}  // namespace gkl
