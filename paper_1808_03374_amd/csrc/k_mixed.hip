// Blocked products A W and A^T X on the matrix cores (gfx950).
//
// Section 5 of the paper names block Lanczos (many vectors per pass, BLAS3) as
// the next step; with b vectors per pass the product becomes a dense contraction
// and runs on the matrix cores.  Two operand formats are built; both keep the
// genotypes exact and differ in how the FP64 vector block is carried.
//
//   A W   (contract over SNPs, layout I: row = individual)
//   A^T X (contract over individuals, layout S: row = SNP)
//
// Split BF16 (GKL_PREC_MIXED).  Genotype codes are decoded in registers to two
// exact BF16 operands: g (0, 1, 2; 0 for missing) and the missing indicator m
// (0 or 1).  Two codes of a 32-bit word form one pair word: a shift and a mask
// isolate them, one 24-bit multiply-add turns them into a byte selector, and
// v_perm_b32 reads both BF16 values from an 8-byte table held in two constants.
// The vector block is split into BF16 hi + lo (hi = bf16(w), lo = bf16(w - hi)),
// multiplied with v_mfma_f32_16x16x32_bf16, accumulated in FP32 per K-chunk and
// in FP64 across chunks and splits.
//     sum_j A_ij W_jc = sum_j g_ij W'_jc + sum_j m_ij X'_jc - K2_c,
//       W' = s W, X' = mu s W, K2_c = sum_j mu_j W'_jc
//     sum_i A_ij X_ic = s_j ( sum_i g_ij X_ic - mu_j T_c + mu_j sum_i m_ij X_ic )
//   MFMA layout: A lane l holds row l%16, B lane l column l%16, both with the K
//   slice selected by (l/16, element); C lane l element e is row 4*(l/16)+e,
//   column l%16.  Element e of K step h is code 4h + (e>>1) + 8(e&1) of the
//   lane's word, and the fragments are written in the same order.
//
// Int8 limbs (GKL_PREC_MIXED_INT8).  The A operand is the raw 2-bit code (0, 1,
// 2, and 3 for missing) as an int8, the second operand the missing flag;
// (w >> 2i) & 0x03030303 puts codes i, 4+i, 8+i, 12+i of a word into the bytes
// of operand dword i (no table, two operations per four codes).  The vector
// block is scaled per column by a power of two, rounded to integers q (|q| <=
// 2^22) and split into three balanced 8-bit limbs, q = l0 2^16 + l1 2^8 + l2.
// v_mfma_i32_16x16x64_i8 accumulates in int32 without rounding (|code x limb|
// + |flag x limb| <= 512 per contraction index, so a K range of up to 4 10^6
// cannot overflow), the limbs are recombined exactly and the K-split partials
// are exact integers below 2^53 in FP64: the only rounding is the per-column
// quantisation (half a unit of 2^-22 times the column's scale, which is below
// twice its largest entry) and the final scaling.  Code 3 counts as 3 in
// sum_j c_ij v_j, so the missing operand carries (mu_j - 3) instead of mu_j:
//     sum_j A_ij W_jc = sum_j c_ij W'_jc + sum_j m_ij Z'_jc - K2_c,
//       Z' = (mu - 3) s W  (W' and Z' share one scale per column)
//     sum_i A_ij X_ic = s_j ( sum_i c_ij X_ic + (mu_j - 3) sum_i m_ij X_ic - mu_j T_c )
//   MFMA layout (v_mfma_i32_16x16x64_i8, probe-confirmed): byte e of A lane l
//   pairs with byte e of B in lane group l/16; byte e of a lane's operand is
//   code 4 (e & 3) + (e >> 2) of its word.  The limbs of a column sit at the
//   same lane in different column tiles (or, for up to 8 columns, limbs 0 and 1
//   share a tile 8 lanes apart), so they recombine with no or one lane shift.
#include <algorithm>

#include "kernels.h"

namespace gkl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kKSteps = 256 / 32;      // split BF16: MFMA K steps per super-tile
constexpr int kSuper = 256;            // K per super-tile (64 bytes of codes per row)
constexpr int kWords = kSuper / 64;    // MFMA K steps per super-tile (one code word per lane)
constexpr int kQBits = 22;             // |q| <= 2^kQBits (so |l0| <= 65 fits int8)
constexpr int kMxWaves = 4;
// Row tiles per wave (A W, A^T X): fewer for three limb tiles, so that two
// waves per SIMD still fit in the register file.
template <bool kPack> constexpr int rtw() { return kPack ? 8 : 4; }
template <bool kPack> constexpr int rtr() { return kPack ? 4 : 2; }
// Column tiles of the B operand per vector: kPack (b <= 8): tile 0 holds limb 0
// of the columns in 0..7 and limb 1 in 8..15, tile 1 limb 2 in 0..7; otherwise
// tile l holds limb l.
template <bool kPack> constexpr int tiles() { return kPack ? 2 : 3; }
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

// Four bytes q..q+3 of packed column j as one little-endian word; bytes at or
// past nb (and rows past n in the last real byte) are code 3.  aligned: the
// column's bytes are 4-byte aligned, so a full word is one load.
__device__ __forceinline__ uint32_t column_word(const uint8_t* __restrict__ G, int64_t ld,
                                                int64_t j, int64_t q, int64_t n, int64_t nb,
                                                bool aligned)
{
    const uint8_t* c = G + j * ld;
    uint32_t w;
    if (aligned && q + 4 <= nb) {
        w = *reinterpret_cast<const uint32_t*>(c + q);
    } else {
        w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) w |= (q + e < nb ? (uint32_t)c[q + e] : 0xFFu) << (8 * e);
    }
    const int64_t last = nb - 1 - q;          // position of the last real byte in w
    const int64_t valid = n - 4 * (nb - 1);   // individuals in that byte (1..4)
    if (valid < 4 && last >= 0 && last < 4) w |= ((0xFFu << (2 * valid)) & 0xFFu) << (8 * last);
    return w;
}

// I: byte J of individual i = codes of SNPs 4J..4J+3 of individual i (tiled, ld
// = ldI); padding = code 3.  A workgroup takes one 64-byte tile column (SNPs
// 256 st .. 256 st + 255) of 512 individuals (bytes 128 ib .. 128 ib + 127 of
// those 256 packed columns: whole 128-byte lines) through LDS.  The codes of
// SNPs 4J..4J+3 (k) of individuals 4b..4b+3 (r) form a 4 x 4 matrix of 2-bit
// fields, field (k, r) at bit 8k + 2r of the word of the four column bytes;
// two delta swaps transpose it to bit 8r + 2k, so byte r of the result is
// byte J of individual 4b + r.  Each thread forms 16 such bytes for 4
// individuals and stores them as 4 x 16 bytes; 4 neighbouring lanes fill one
// 64-byte tile row.
constexpr int kBiCols = 256;    // SNP columns per workgroup (one tile column of I)
constexpr int kBiBytes = 128;   // packed bytes per column (512 individuals)

__global__ void __launch_bounds__(256) build_I_kernel(const uint8_t* __restrict__ G, int64_t n,
                                                      int64_t p, int64_t ld,
                                                      uint8_t* __restrict__ I, int64_t nI,
                                                      int64_t ldI)
{
    // column c at c * kBiBytes + (c / 64) * 16: the reads of the four column
    // groups fall in different banks
    __shared__ __align__(16) uint8_t col[kBiCols * kBiBytes + 4 * 16];
    const int64_t nb = (n + 3) / 4;
    const int64_t nib = nI / (4 * kBiBytes), nst = ldI / 64;
    const bool aligned = (ld & 3) == 0 && (reinterpret_cast<uintptr_t>(G) & 3) == 0;
    const int t = threadIdx.x;
    for (int64_t blk = blockIdx.x; blk < nib * nst; blk += gridDim.x) {
        const int64_t ib = blk % nib, st = blk / nib;
        const int64_t q0 = ib * kBiBytes, j0 = st * kBiCols;
        __syncthreads();   // the previous block's reads of col are done
#pragma unroll 8
        for (int k = 0; k < kBiCols / 8; ++k) {   // dword t & 31 of columns 8k + t / 32
            const int c = 8 * k + (t >> 5);
            const int64_t j = j0 + c;
            const uint32_t w = j < p ? column_word(G, ld, j, q0 + 4 * (t & 31), n, nb, aligned)
                                     : 0xFFFFFFFFu;
            *reinterpret_cast<uint32_t*>(col + c * kBiBytes + (c >> 6) * 16 + 4 * (t & 31)) = w;
        }
        __syncthreads();
        const int jq = t & 3;   // output bytes 16 jq .. 16 jq + 15 of the tile row
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int b = (t >> 2) + 64 * h;   // packed byte: individuals 4b .. 4b + 3
            uint32_t W[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const uint8_t* cp = col + (64 * jq + 4 * q) * kBiBytes + jq * 16 + b;
                uint32_t x = (uint32_t)cp[0] | (uint32_t)cp[kBiBytes] << 8 |
                             (uint32_t)cp[2 * kBiBytes] << 16 | (uint32_t)cp[3 * kBiBytes] << 24;
                uint32_t d = ((x >> 6) ^ x) & 0x00CC00CCu;
                x ^= d ^ (d << 6);
                d = ((x >> 12) ^ x) & 0x0000F0F0u;
                x ^= d ^ (d << 12);
                W[q] = x;
            }
            const int64_t row0 = 4 * kBiBytes * ib + 4 * b;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                uint32_t o[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    o[e] = ((W[4 * e] >> (8 * r)) & 0xFFu) |
                           ((W[4 * e + 1] >> (8 * r)) & 0xFFu) << 8 |
                           ((W[4 * e + 2] >> (8 * r)) & 0xFFu) << 16 |
                           ((W[4 * e + 3] >> (8 * r)) & 0xFFu) << 24;
                *reinterpret_cast<uint4*>(I + tiled_offset(row0 + r, 64 * st + 16 * jq, ldI)) =
                    make_uint4(o[0], o[1], o[2], o[3]);
            }
        }
    }
}

// S: byte Iq of SNP j = codes of individuals 4Iq..4Iq+3 (tiled, ld = ldS);
// padding = code 3.  One wave per SNP row, four bytes per lane (they stay in
// one 64-byte tile row).  With stats, the wave also counts the codes of its
// column and writes the column statistics, so no separate pass reads G.
__global__ void __launch_bounds__(256) build_S_kernel(const uint8_t* __restrict__ G, int64_t n,
                                                      int64_t p, int64_t ld,
                                                      uint8_t* __restrict__ S, int64_t pS,
                                                      int64_t ldS, ColStats st, int with_stats)
{
    const int64_t nb = (n + 3) / 4;
    const bool aligned = (ld & 3) == 0 && (reinterpret_cast<uintptr_t>(G) & 3) == 0;
    const int lane = threadIdx.x & 63;
    for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < pS;
         j += (int64_t)gridDim.x * 4) {
        int64_t c1 = 0, c2 = 0, c3 = 0;
#pragma unroll 4
        for (int64_t q = 4 * lane; q < ldS; q += 256) {
            uint32_t w = 0xFFFFFFFFu;
            if (j < p && q < nb) {
                w = column_word(G, ld, j, q, n, nb, aligned);
                if (with_stats) {
                    const int64_t valid = n - 4 * q;
                    count_word(w, valid >= 16 ? 16 : (int)valid, c1, c2, c3);
                }
            }
            *reinterpret_cast<uint32_t*>(S + tiled_offset(j, q, ldS)) = w;
        }
        if (with_stats && j < p) {
            c1 = wave_sum_i64(c1);
            c2 = wave_sum_i64(c2);
            c3 = wave_sum_i64(c3);
            if (lane == 0) store_colstats(st, j, n, c1, c2, c3);
        }
    }
}

void build_mixed_layouts(const uint8_t* G, int64_t n, int64_t p, int64_t ld, uint8_t* I,
                         uint8_t* S, hipStream_t s, const ColStats* st)
{
    const int64_t nI = mixed_rows_I(n), ldI = mixed_ld_I(p);
    const int64_t pS = mixed_rows_S(p), ldS = mixed_ld_S(n);
    if (st && !S) fail(GKL_ERR_INTERNAL, "column statistics come with layout S");
    if (I) {
        const int64_t blocks = (nI / (4 * kBiBytes)) * (ldI / 64);
        const unsigned int grid = (unsigned int)std::min<int64_t>(blocks, (int64_t)1 << 20);
        hipLaunchKernelGGL(build_I_kernel, dim3(grid), dim3(256), 0, s, G, n, p, ld, I, nI, ldI);
        GKL_LAUNCH_CHECK("build_I_kernel");
    }
    if (S) {
        const int64_t rows4 = pS / 4;
        const unsigned int grid = (unsigned int)std::min<int64_t>(rows4, (int64_t)1 << 20);
        hipLaunchKernelGGL(build_S_kernel, dim3(grid), dim3(256), 0, s, G, n, p, ld, S, pS, ldS,
                           st ? *st : ColStats{}, st ? 1 : 0);
        GKL_LAUNCH_CHECK("build_S_kernel");
    }
}

// ---------------------------------------------------------------------------
// Int8 limbs: operands
// ---------------------------------------------------------------------------
// The 16 codes of a word as int8: dword i holds codes i, 4+i, 8+i, 12+i.
__device__ __forceinline__ i32x4 raw_codes(uint32_t w)
{
    const i32x4 r = {(int)(w & 0x03030303u), (int)((w >> 2) & 0x03030303u),
                     (int)((w >> 4) & 0x03030303u), (int)((w >> 6) & 0x03030303u)};
    return r;
}

// Missing flags (code 3) of the same 16 codes, in the same positions, from the
// code bytes: each code byte (0..3) selects a byte of the constant 0x01000000
// in a byte permute (v_perm_b32), one instruction per four flags.
__device__ __forceinline__ i32x4 missing_flags(const i32x4& c)
{
    const i32x4 r = {(int)__builtin_amdgcn_perm(0u, 0x01000000u, (uint32_t)c[0]),
                     (int)__builtin_amdgcn_perm(0u, 0x01000000u, (uint32_t)c[1]),
                     (int)__builtin_amdgcn_perm(0u, 0x01000000u, (uint32_t)c[2]),
                     (int)__builtin_amdgcn_perm(0u, 0x01000000u, (uint32_t)c[3])};
    return r;
}

// position (within the lane's 16-code word) of byte e of an operand
__host__ __device__ __forceinline__ int code_of_elem(int e) { return 4 * (e & 3) + (e >> 2); }

// Smallest power of two >= m (1 for m == 0): the scale of a column.
__device__ __forceinline__ double pow2_at_least(double m)
{
    if (!(m > 0.0)) return 1.0;
    int ex = 0;
    frexp(m, &ex);   // m = f 2^ex, f in [0.5, 1)
    return ldexp(1.0, ex);
}

// q = rint(v 2^kQBits / scale) split into balanced 8-bit limbs l0, l1, l2
// (q = l0 2^16 + l1 2^8 + l2, l1 and l2 in [-128, 127], |l0| <= 65).
__device__ __forceinline__ void limbs3(double v, int ex, int& l0, int& l1, int& l2)
{
    const int q = (int)rint(ldexp(v, kQBits - ex));
    l2 = ((q + 128) & 255) - 128;
    const int q1 = (q - l2) >> 8;
    l1 = ((q1 + 128) & 255) - 128;
    l0 = (q1 - l1) >> 8;
}

__device__ __forceinline__ void put_byte(i32x4& v, int e, int x)
{
    const uint32_t u = (uint32_t)(x & 0xFF) << (8 * (e & 3));
    v[e >> 2] = (int)((uint32_t)v[e >> 2] | u);
}

__device__ __forceinline__ i32x4 mfma_i8(i32x4 a, i32x4 b, i32x4 c)
{
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Split BF16: genotype operands decoded in registers
// ---------------------------------------------------------------------------
// A lane's 32-bit word d holds 16 codes (code q at bits 2q, 2q + 1).  Pair word
// k (k = 0..7) of an operand holds code k in its low bf16 and code k + 8 in its
// high bf16; pair words 4h..4h+3 are the lane's 8 elements of MFMA K step h, so
// element e of K step h is code 4h + (e >> 1) + 8 (e & 1) (code_pos).
//
// g operand: a code's two bits become the two low bits of the bf16 exponent --
// one shift and one mask per pair word -- so codes 0, 1, 2, 3 read as 0, 1, 2
// and 4 times 2^-126, all exact.  The missing code thus counts 4 in the g sum;
// the missing operand removes it.  The vector operand carries the factor 2^126.
constexpr uint32_t kExpLow = 0x01800180u;

// The four pair words of K step h: G[i] = pair word 4h + i.
__device__ __forceinline__ void g_pairs_half(uint32_t d, int h, uint32_t G[4])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 4 * h + i;
        G[i] = (k < 4 ? d << (7 - 2 * k) : d >> (2 * k - 7)) & kExpLow;
    }
}

// Missing flags at the scale of the g operand (2^-126), used by A^T X: a code is
// missing when both its bits are set, i.e. bits 7 and 8 (23 and 24) of its g
// pair word: M = G & (G >> 1).
//
// Missing flags with no shift per pair word, used by A W: f = d & (d >> 1) holds
// the flag of code q at bit 2q.  Those of codes 4..7 and 12..15 already sit at
// bits 8 + 2i and 24 + 2i (i = k - 4), inside the bf16 exponents; those of codes
// 0..3 and 8..11 get there by one shift of f by 8.  A lone exponent bit 1 + 2i
// is the bf16 2^(2^(1 + 2i) - 127): 2^-125, 2^-119, 2^-95, 2^1 for i = 0..3
// (m_scale_exp of the element); the vector operand carries the inverse factor
// element by element.
__device__ __forceinline__ void m_pairs_scaled_half(uint32_t d, int h, uint32_t M[4])
{
    const uint32_t f = d & (d >> 1);
    const uint32_t fh = h == 0 ? f << 8 : f;
#pragma unroll
    for (int i = 0; i < 4; ++i) M[i] = fh & (0x01000100u << (2 * i));
}

// Exponent of the value a set missing flag takes in element e of a K step
// (m_pairs_scaled): element e belongs to pair word 4h + (e >> 1).
__host__ __device__ __forceinline__ int m_scale_exp(int e) { return (1 << (1 + 2 * (e >> 1))) - 127; }

__device__ __forceinline__ bf16x8 pack4(uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 v = {a, b, c, d};
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// position (within the lane's 16-code word) of element e of K step h
__host__ __device__ __forceinline__ int code_pos(int h, int e) { return 4 * h + (e >> 1) + 8 * (e & 1); }

__device__ __forceinline__ __bf16 to_bf16(double v) { return (__bf16)(float)v; }

// Products are formed at 2^-(kProdShift + ex_c): the g vector operand holds
// v 2^(126 - kProdShift - ex_c), the missing one v 2^(-m_scale_exp(e) -
// kProdShift - ex_c), with 2^ex_c >= the column's largest |v|.  Every operand then
// lies below 2^110 (bf16 and FP32 reach 2^128) and every product is a normal FP32.
constexpr int kProdShift = 16;

// Workgroup -> (K split, row block).  Workgroups are dealt to the 8 XCDs of the
// chip round robin (workgroup g runs on XCD g % 8), each XCD with its own L2.
// With xcd set (nsplit a multiple of 8) every row block of one K split runs on
// the same XCD, so the split's vector fragments come from that XCD's L2 after
// the first touch instead of from the memory-side cache.
__device__ __forceinline__ void block_coords(int g, int nsplit, int nrb, int xcd, int& split,
                                             int& rb)
{
    if (xcd) {
        const int x = g & 7, q = g >> 3;
        split = x + 8 * (q / nrb);
        rb = q % nrb;
    } else {
        split = g / nrb;
        rb = g % nrb;
    }
    (void)nsplit;
}

// ---------------------------------------------------------------------------
// Column sums and maxima
// ---------------------------------------------------------------------------
// Column sums over len rows: sum_j f_j X(j, c), with f_j = mean_j inv_sd_j when
// mean != NULL (the product mean_j (inv_sd_j x) is formed in that order) and
// f_j = 1 otherwise (per column c: K2_c = sum_j mu_j s_j W_jc for A W, T_c =
// sum_i X_ic for A^T X); with them the largest magnitude to be scaled:
// |mref - mu_j| |s_j W_jc| for A W (the missing-operand values, which bound
// |s_j W_jc| since mref - mu_j >= 1; mref = 3 for int8 limbs, 4 for split BF16),
// |X_ic| for A^T X.
// grid (kCsSplit, columns): each block writes its chunk's sum and maximum to
// cpart / cmax[c * kCsSplit + chunk]; consumers add / take the maximum of the
// chunk values themselves (no cross-block handshake: its device-scope fences
// cost more than the consumer's 64 extra reads).
constexpr int kCsSplit = 64;   // == wavefront size (the chunk values are combined by one wave)

// Chunk `chunk` of one column xc (len entries): its sum (of mean_j s_j x_j when
// mean is given) and its largest magnitude (of (mref - mu_j) s_j x_j).  Called
// by every thread of the block.
__device__ __forceinline__ void colsum_chunk(const double* __restrict__ xc, int64_t len,
                                             const double* __restrict__ mean,
                                             const double* __restrict__ inv_sd, double mref,
                                             int chunk, double* __restrict__ sum_out,
                                             double* __restrict__ max_out)
{
    __shared__ double sh[16];
    const int64_t per = (len + kCsSplit - 1) / kCsSplit;
    const int64_t j0 = (int64_t)chunk * per;
    const int64_t j1 = j0 + per < len ? j0 + per : len;
    double a = 0.0, mx = 0.0;
    if (mean) {
        for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
            const double w = inv_sd[j] * xc[j];
            a += mean[j] * w;
            mx = fmax(mx, fabs((mean[j] - mref) * w));
        }
    } else {
        for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
            a += xc[j];
            mx = fmax(mx, fabs(xc[j]));
        }
    }
    a = block_sum(a, sh);
    if (threadIdx.x == 0) *sum_out = a;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, sh[w]);
        *max_out = m;
    }
}

__global__ void __launch_bounds__(256)
colsum_kernel(const double* __restrict__ X, int64_t ldx, int64_t len,
              const double* __restrict__ mean, const double* __restrict__ inv_sd, double mref,
              double* __restrict__ cpart, double* __restrict__ cmax)
{
    const int c = blockIdx.y;
    colsum_chunk(X + (int64_t)c * ldx, len, mean, inv_sd, mref, blockIdx.x,
                 cpart + c * kCsSplit + blockIdx.x, cmax + c * kCsSplit + blockIdx.x);
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

// ex[c] for c < nb: the exponent of column c's scale (scale = 2^ex >= its
// largest magnitude).  Called by every thread of the block.
__device__ __forceinline__ void column_scales(const double* __restrict__ cmax, int nb, int* ex)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = wave; c < nb; c += (int)(blockDim.x >> 6)) {
        double m = cmax[c * kCsSplit + lane];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
        if (lane == 0) ex[c] = ilogb(pow2_at_least(m));
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Split BF16: vector fragments
// ---------------------------------------------------------------------------
// frag[((st * kKSteps + ks) * ops + op) * 64 + lane] holds the 8 elements of MFMA
// K step ks of super-tile st for operand op; element e is contraction index
// st * 256 + 64 (lane >> 4) + 16 (ks >> 1) + code_pos(ks & 1, e).
//   kPack (b <= 8): the 16 columns of an operand hold the hi parts of the b
//   columns in 0..7 and their lo parts in 8..15 (one MFMA covers both halves).
//   Otherwise column tile t (16 columns, t < kT) has its own operands.
// A W operands: kPack: op 0 = g part, op 1 = missing part; otherwise op 4t + q,
// q = g hi, g lo, missing hi, missing lo.  g part v = s_j W_jc, missing part
// z = (mu_j - 4) s_j W_jc (the g operand counts the missing code as 4).
template <bool kPack, int kT>
__global__ void __launch_bounds__(256)
split_W_bf16_kernel(const double* __restrict__ W, int64_t ldw, int nb, int64_t p,
                    const double* __restrict__ mean, const double* __restrict__ inv_sd,
                    const double* __restrict__ cmax, int64_t nst, bf16x8* __restrict__ frag)
{
    constexpr int kOps = kPack ? 2 : 4 * kT;
    constexpr int kTiles = kPack ? 1 : kT;
    __shared__ int ex[32];
    column_scales(cmax, nb, ex);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (st, ks, lane)
    if (t >= nst * kKSteps * 64) return;
    const int lane = (int)(t & 63);
    const int ks = (int)((t >> 6) % kKSteps);
    const int64_t st = t / (64 * kKSteps);
    const int g = lane >> 4, cl = lane & 15;
    bf16x8 out[kOps];
#pragma unroll
    for (int tile = 0; tile < kTiles; ++tile) {
        const int col = kPack ? (cl & 7) : 16 * tile + cl;
        const bool lo_half = kPack && cl >= 8;
        const int e_c = col < nb ? ex[col] : 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t j = st * kSuper + 64 * g + 16 * (ks >> 1) + code_pos(ks & 1, e);
            double v = 0.0, z = 0.0;
            if (j < p && col < nb) {
                v = inv_sd[j] * W[(int64_t)col * ldw + j];
                z = (mean[j] - 4.0) * v;
            }
            const double vg = ldexp(v, 126 - kProdShift - e_c);
            const double zm = ldexp(z, -m_scale_exp(e) - kProdShift - e_c);
            const __bf16 gh = to_bf16(vg), mh = to_bf16(zm);
            const __bf16 gl = to_bf16(vg - (double)(float)gh), ml = to_bf16(zm - (double)(float)mh);
            if (kPack) {
                out[0][e] = lo_half ? gl : gh;
                out[1][e] = lo_half ? ml : mh;
            } else {
                out[4 * tile + 0][e] = gh;
                out[4 * tile + 1][e] = gl;
                out[4 * tile + 2][e] = mh;
                out[4 * tile + 3][e] = ml;
            }
        }
    }
    bf16x8* f = frag + ((st * kKSteps + ks) * kOps) * 64 + lane;
#pragma unroll
    for (int op = 0; op < kOps; ++op) f[op * 64] = out[op];
}

// A^T X operands (the g and missing operands share them: both carry 2^-126):
// kPack: op 0; otherwise op 2t + q, q = hi, lo.  Element value x 2^(126 -
// kProdShift - ex_c).
template <bool kPack, int kT>
__global__ void __launch_bounds__(256)
split_X_bf16_kernel(const double* __restrict__ X, int64_t ldx, int nb, int64_t n,
                    const double* __restrict__ cmax, int64_t nst, bf16x8* __restrict__ frag)
{
    constexpr int kOps = kPack ? 1 : 2 * kT;
    constexpr int kTiles = kPack ? 1 : kT;
    __shared__ int ex[32];
    column_scales(cmax, nb, ex);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nst * kKSteps * 64) return;
    const int lane = (int)(t & 63);
    const int ks = (int)((t >> 6) % kKSteps);
    const int64_t st = t / (64 * kKSteps);
    const int g = lane >> 4, cl = lane & 15;
    bf16x8 out[kOps];
#pragma unroll
    for (int tile = 0; tile < kTiles; ++tile) {
        const int col = kPack ? (cl & 7) : 16 * tile + cl;
        const bool lo_half = kPack && cl >= 8;
        const int e_c = col < nb ? ex[col] : 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t i = st * kSuper + 64 * g + 16 * (ks >> 1) + code_pos(ks & 1, e);
            const double x = (i < n && col < nb) ? X[(int64_t)col * ldx + i] : 0.0;
            const double xs = ldexp(x, 126 - kProdShift - e_c);
            const __bf16 h = to_bf16(xs);
            const __bf16 l = to_bf16(xs - (double)(float)h);
            if (kPack) {
                out[0][e] = lo_half ? l : h;
            } else {
                out[2 * tile + 0][e] = h;
                out[2 * tile + 1][e] = l;
            }
        }
    }
    bf16x8* f = frag + ((st * kKSteps + ks) * kOps) * 64 + lane;
#pragma unroll
    for (int op = 0; op < kOps; ++op) f[op * 64] = out[op];
}

// ---------------------------------------------------------------------------
// Split BF16: A W.  Workgroup = 4 waves x kRTW row tiles x 16 individuals; one
// K split of the SNPs.  Each lane loads 16 bytes (64 codes) of its row per
// super-tile and decodes one 16-code word per two MFMA K steps; the vector
// fragments of a super-tile are staged in LDS and shared by the row tiles.
// FP32 accumulation per 1,024 K values, FP64 across those chunks.
// partial[split][row][kCS] (kCS = 8 packed, 16 kT otherwise; packed rows hold
// hi + lo already added).
// ---------------------------------------------------------------------------
// Fragments are staged in LDS in blocks of kStage K steps (half a super-tile),
// double buffered: block s + 1 is loaded straight from global memory into LDS
// (global_load_lds_dwordx4: lane l of a wave writes bytes 16 l .. 16 l + 15 of
// the wave's 1 KB) while block s is multiplied, and one barrier per block,
// after every wave's loads have landed, hands the buffers over.
constexpr int kStage = 4;

template <int kFr>
__device__ __forceinline__ void stage_to_lds(const bf16x8* __restrict__ src, bf16x8* dst)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < kFr / 256; ++k) {
        const int base = 256 * k + 64 * wave;     // wave-uniform
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src + base + lane),
                                         dst + base, 16, 0, 0);
    }
}

constexpr int kRTW = 4;       // A W: row tiles per wave
constexpr int kRTX = 2;       // A^T X: row tiles per wave
constexpr int kFlush = 4;     // super-tiles per FP32 chunk

template <bool kPack, int kT>
__global__ void __launch_bounds__(256)
matmat_bf16_kernel(const uint8_t* __restrict__ I, int64_t ldI, int64_t nI,
                   const bf16x8* __restrict__ frag, int64_t nst, int64_t st_per_split,
                   int nsplit, int nrb, int xcd, double* __restrict__ partial)
{
    constexpr int kOps = kPack ? 2 : 4 * kT;
    constexpr int kTiles = kPack ? 1 : kT;
    constexpr int kCS = kPack ? 8 : 16 * kT;
    constexpr int kFr = kStage * kOps * 64;        // fragments per staged block
    __shared__ bf16x8 bs[2][kFr];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    int split, rb;
    block_coords(blockIdx.x, nsplit, nrb, xcd, split, rb);
    const int64_t row_base = (int64_t)rb * (kMxWaves * kRTW * 16) + wave * (kRTW * 16);
    const int64_t st0 = (int64_t)split * st_per_split;
    const int64_t st1 = st0 + st_per_split < nst ? st0 + st_per_split : nst;
    f32x4 acc[kRTW][kTiles];
    double accd[kRTW][kTiles][4];
#pragma unroll
    for (int t = 0; t < kRTW; ++t)
#pragma unroll
        for (int c = 0; c < kTiles; ++c) {
            acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < 4; ++e) accd[t][c][e] = 0.0;
        }
    uint4 a[kRTW], an[kRTW];
    const int64_t nstage = 2 * (st1 - st0);
    if (nstage > 0) {
        stage_to_lds<kFr>(frag + st0 * (2 * kFr), bs[0]);
#pragma unroll
        for (int t = 0; t < kRTW; ++t)
            a[t] = *reinterpret_cast<const uint4*>(
                I + tiled_offset(row_base + 16 * t + r, st0 * 64 + 16 * g, ldI));
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int chunk = 0;
    for (int64_t sidx = 0; sidx < nstage; ++sidx) {
        const int64_t st = st0 + (sidx >> 1);
        const int half = (int)(sidx & 1);
        const int buf = (int)(sidx & 1);
        if (half == 0) {
            // the next super-tile's codes are in flight while this one is used
            const int64_t stn = st + 1 < st1 ? st + 1 : st;
#pragma unroll
            for (int t = 0; t < kRTW; ++t)
                an[t] = *reinterpret_cast<const uint4*>(
                    I + tiled_offset(row_base + 16 * t + r, stn * 64 + 16 * g, ldI));
        }
        if (sidx + 1 < nstage) stage_to_lds<kFr>(frag + st0 * (2 * kFr) + (sidx + 1) * kFr, bs[buf ^ 1]);
#pragma unroll
        for (int kk = 0; kk < kStage; ++kk) {
            const int ks = half * kStage + kk;
            const int w = ks >> 1, h = ks & 1;
            bf16x8 bo[kOps];
#pragma unroll
            for (int op = 0; op < kOps; ++op) bo[op] = bs[buf][(kk * kOps + op) * 64 + lane];
#pragma unroll
            for (int t = 0; t < kRTW; ++t) {
                const uint32_t d = w == 0 ? a[t].x : w == 1 ? a[t].y : w == 2 ? a[t].z : a[t].w;
                uint32_t G[4], M[4];
                g_pairs_half(d, h, G);
                m_pairs_scaled_half(d, h, M);
                const bf16x8 ca = pack4(G[0], G[1], G[2], G[3]);
                const bf16x8 ma = pack4(M[0], M[1], M[2], M[3]);
                if (kPack) {
                    acc[t][0] = mfma_bf16(ca, bo[0], acc[t][0]);
                    acc[t][0] = mfma_bf16(ma, bo[1], acc[t][0]);
                } else {
#pragma unroll
                    for (int c = 0; c < kT; ++c) {
                        acc[t][c] = mfma_bf16(ca, bo[4 * c + 0], acc[t][c]);
                        acc[t][c] = mfma_bf16(ca, bo[4 * c + 1], acc[t][c]);
                        acc[t][c] = mfma_bf16(ma, bo[4 * c + 2], acc[t][c]);
                        acc[t][c] = mfma_bf16(ma, bo[4 * c + 3], acc[t][c]);
                    }
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (half == 1) {
#pragma unroll
            for (int t = 0; t < kRTW; ++t) a[t] = an[t];
            if (++chunk == kFlush) {
                chunk = 0;
#pragma unroll
                for (int t = 0; t < kRTW; ++t)
#pragma unroll
                    for (int c = 0; c < kTiles; ++c) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) accd[t][c][e] += (double)acc[t][c][e];
                        acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
    }
    double* out = partial + (int64_t)split * nI * kCS;
#pragma unroll
    for (int t = 0; t < kRTW; ++t)
#pragma unroll
        for (int c = 0; c < kTiles; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = row_base + 16 * t + 4 * g + e;
                double v = accd[t][c][e] + (double)acc[t][c][e];
                if (kPack) {
                    // lane r < 8 holds the hi column r, lane r + 8 its lo column
                    v += __shfl_down(v, 8, 16);
                    if (r < 8) out[row * kCS + r] = v;
                } else {
                    out[row * kCS + 16 * c + r] = v;
                }
            }
}

// Y[i + c ldy] = 2^(kProdShift + ex_c) sum_split partial - K2_c for i < n, c < nb.
__global__ void __launch_bounds__(256)
matmat_bf16_reduce_kernel(const double* __restrict__ partial, int nsplit, int64_t nI, int64_t n,
                          int nb, int kcs, const double* __restrict__ cpart,
                          const double* __restrict__ cmax, double* __restrict__ Y, int64_t ldy)
{
    __shared__ double K2[32];
    __shared__ int ex[32];
    column_sums(cpart, nb, K2);
    column_scales(cmax, nb, ex);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * kcs) return;
    const int64_t i = t / kcs;
    const int c = (int)(t - i * kcs);
    if (c >= nb) return;
    const double s = strided_sum(partial + i * kcs + c, nI * kcs, nsplit);
    Y[(int64_t)c * ldy + i] = ldexp(s, kProdShift + ex[c]) - K2[c];
}

// ---------------------------------------------------------------------------
// Split BF16: A^T X.  Workgroup = 4 waves x kRTX SNP tiles x 16 SNPs; K =
// individuals.  The g and missing operands share the vector fragments, so each
// row tile keeps two accumulators (g sum SC, missing sum SM).
// With one K split (kFused) the kernel writes Z itself:
//   Z[j + c ldz] = s_j (2^(kProdShift + ex_c) (SC + (mu_j - 4) SM) - mu_j T_c);
// otherwise partial[split][2][row][kCS] for the reduce kernel.
// ---------------------------------------------------------------------------
template <bool kPack, int kT, bool kFused>
__global__ void __launch_bounds__(256)
rmatmat_bf16_kernel(const uint8_t* __restrict__ S, int64_t ldS, int64_t pS,
                    const bf16x8* __restrict__ frag, int64_t nst, int64_t st_per_split,
                    int nsplit, int nrb, int xcd, double* __restrict__ partial, int64_t p, int nb,
                    const double* __restrict__ cpart, const double* __restrict__ cmax,
                    const double* __restrict__ mean, const double* __restrict__ inv_sd,
                    double* __restrict__ Z, int64_t ldz)
{
    constexpr int kOps = kPack ? 1 : 2 * kT;
    constexpr int kTiles = kPack ? 1 : kT;
    constexpr int kCS = kPack ? 8 : 16 * kT;
    constexpr int kFr = kStage * kOps * 64;        // fragments per staged block
    __shared__ bf16x8 bs[2][kFr];
    __shared__ double Tc[32];
    __shared__ int ex[32];
    if (kFused) {
        column_sums(cpart, nb, Tc);
        column_scales(cmax, nb, ex);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    int split, rb;
    block_coords(blockIdx.x, nsplit, nrb, xcd, split, rb);
    const int64_t row_base = (int64_t)rb * (kMxWaves * kRTX * 16) + wave * (kRTX * 16);
    const int64_t st0 = (int64_t)split * st_per_split;
    const int64_t st1 = st0 + st_per_split < nst ? st0 + st_per_split : nst;
    f32x4 aC[kRTX][kTiles], aM[kRTX][kTiles];
    double dC[kRTX][kTiles][4], dM[kRTX][kTiles][4];
#pragma unroll
    for (int t = 0; t < kRTX; ++t)
#pragma unroll
        for (int c = 0; c < kTiles; ++c) {
            aC[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
            aM[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < 4; ++e) dC[t][c][e] = dM[t][c][e] = 0.0;
        }
    uint4 a[kRTX], an[kRTX];
    const int64_t nstage = 2 * (st1 - st0);
    if (nstage > 0) {
        stage_to_lds<kFr>(frag + st0 * (2 * kFr), bs[0]);
#pragma unroll
        for (int t = 0; t < kRTX; ++t)
            a[t] = *reinterpret_cast<const uint4*>(
                S + tiled_offset(row_base + 16 * t + r, st0 * 64 + 16 * g, ldS));
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int chunk = 0;
    for (int64_t sidx = 0; sidx < nstage; ++sidx) {
        const int64_t st = st0 + (sidx >> 1);
        const int half = (int)(sidx & 1);
        const int buf = (int)(sidx & 1);
        if (half == 0) {
            const int64_t stn = st + 1 < st1 ? st + 1 : st;
#pragma unroll
            for (int t = 0; t < kRTX; ++t)
                an[t] = *reinterpret_cast<const uint4*>(
                    S + tiled_offset(row_base + 16 * t + r, stn * 64 + 16 * g, ldS));
        }
        if (sidx + 1 < nstage) stage_to_lds<kFr>(frag + st0 * (2 * kFr) + (sidx + 1) * kFr, bs[buf ^ 1]);
#pragma unroll
        for (int kk = 0; kk < kStage; ++kk) {
            const int ks = half * kStage + kk;
            const int w = ks >> 1, h = ks & 1;
            bf16x8 bo[kOps];
#pragma unroll
            for (int op = 0; op < kOps; ++op) bo[op] = bs[buf][(kk * kOps + op) * 64 + lane];
#pragma unroll
            for (int t = 0; t < kRTX; ++t) {
                const uint32_t d = w == 0 ? a[t].x : w == 1 ? a[t].y : w == 2 ? a[t].z : a[t].w;
                uint32_t G[4], M[4];
                g_pairs_half(d, h, G);
#pragma unroll
                for (int k = 0; k < 4; ++k) M[k] = G[k] & (G[k] >> 1);
                const bf16x8 ca = pack4(G[0], G[1], G[2], G[3]);
                const bf16x8 ma = pack4(M[0], M[1], M[2], M[3]);
#pragma unroll
                for (int c = 0; c < kTiles; ++c) {
#pragma unroll
                    for (int q = 0; q < (kPack ? 1 : 2); ++q) {
                        const bf16x8 b = bo[kPack ? 0 : 2 * c + q];
                        aC[t][c] = mfma_bf16(ca, b, aC[t][c]);
                        aM[t][c] = mfma_bf16(ma, b, aM[t][c]);
                    }
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (half == 1) {
#pragma unroll
            for (int t = 0; t < kRTX; ++t) a[t] = an[t];
            if (++chunk == kFlush) {
                chunk = 0;
#pragma unroll
                for (int t = 0; t < kRTX; ++t)
#pragma unroll
                    for (int c = 0; c < kTiles; ++c) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            dC[t][c][e] += (double)aC[t][c][e];
                            dM[t][c][e] += (double)aM[t][c][e];
                        }
                        aC[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
                        aM[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kRTX; ++t)
#pragma unroll
        for (int c = 0; c < kTiles; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = row_base + 16 * t + 4 * g + e;
                double vc = dC[t][c][e] + (double)aC[t][c][e];
                double vm = dM[t][c][e] + (double)aM[t][c][e];
                if (kPack) {
                    vc += __shfl_down(vc, 8, 16);
                    vm += __shfl_down(vm, 8, 16);
                }
                const int col = kPack ? r : 16 * c + r;
                if (kPack && r >= 8) continue;
                if (kFused) {
                    if (row < p && col < nb) {
                        const double mu = mean[row];
                        const double u = ldexp(vc + (mu - 4.0) * vm, kProdShift + ex[col]);
                        Z[(int64_t)col * ldz + row] = inv_sd[row] * (u - mu * Tc[col]);
                    }
                } else {
                    double* out = partial + (int64_t)split * 2 * pS * kCS;
                    out[row * kCS + col] = vc;
                    out[(pS + row) * kCS + col] = vm;
                }
            }
}

// Z[j + c ldz] = s_j (2^(kProdShift + ex_c) (SC + (mu_j - 4) SM) - mu_j T_c)
__global__ void __launch_bounds__(256)
rmatmat_bf16_reduce_kernel(const double* __restrict__ partial, int nsplit, int64_t pS, int64_t p,
                           int nb, int kcs, const double* __restrict__ cpart,
                           const double* __restrict__ cmax, const double* __restrict__ mean,
                           const double* __restrict__ inv_sd, double* __restrict__ Z, int64_t ldz)
{
    __shared__ double T[32];
    __shared__ int ex[32];
    column_sums(cpart, nb, T);
    column_scales(cmax, nb, ex);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * kcs) return;
    const int64_t j = t / kcs;
    const int c = (int)(t - j * kcs);
    if (c >= nb) return;
    const double sc = strided_sum(partial + j * kcs + c, 2 * pS * kcs, nsplit);
    const double sm = strided_sum(partial + (pS + j) * kcs + c, 2 * pS * kcs, nsplit);
    const double mu = mean[j];
    Z[(int64_t)c * ldz + j] = inv_sd[j] * (ldexp(sc + (mu - 4.0) * sm, kProdShift + ex[c]) - mu * T[c]);
}

// ---------------------------------------------------------------------------
// Vector fragments
// ---------------------------------------------------------------------------
// Byte e of lane (g, col) in column tile `tile` of the vector operand for an
// entry whose limbs are l0, l1, l2 (see tiles()).
template <bool kPack>
__device__ __forceinline__ int limb_for(int tile, int col, int l0, int l1, int l2)
{
    if (kPack) return tile == 0 ? (col < 8 ? l0 : l1) : (col < 8 ? l2 : 0);
    return tile == 0 ? l0 : tile == 1 ? l1 : l2;
}

// A W operands: frag[((st * kWords + word) * 2T + op) * 64 + lane], op 0..T-1 =
// tiles of W', T..2T-1 = tiles of Z' (T = tiles<kPack>()), for column
// col0 + c of the block, c = lane & 15 (& 7 when packed); zero past the block.
// Byte e holds SNP st*256 + 64 (lane >> 4) + 16 word + code_of_elem(e).
template <bool kPack>
__global__ void __launch_bounds__(256)
split_W_i8_kernel(const double* __restrict__ W, int64_t ldw, int nb, int64_t p,
               const double* __restrict__ mean, const double* __restrict__ inv_sd,
               const double* __restrict__ cmax, int64_t nst, i32x4* __restrict__ frag)
{
    constexpr int T = tiles<kPack>();
    __shared__ int ex[16];
    column_scales(cmax, nb, ex);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (st, word, lane)
    if (t >= nst * kWords * 64) return;
    const int lane = (int)(t & 63);
    const int word = (int)((t >> 6) % kWords);
    const int64_t st = t / (64 * kWords);
    const int g = lane >> 4, col = lane & 15, c = kPack ? (col & 7) : col;
    const int e_c = c < nb ? ex[c] : 0;
    i32x4 fw[T], fz[T];
#pragma unroll
    for (int l = 0; l < T; ++l) { fw[l] = i32x4{0, 0, 0, 0}; fz[l] = i32x4{0, 0, 0, 0}; }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t j = st * kSuper + 64 * g + 16 * word + code_of_elem(e);
        double w = 0.0, z = 0.0;
        if (j < p && c < nb) {
            w = inv_sd[j] * W[(int64_t)c * ldw + j];
            z = (mean[j] - 3.0) * w;
        }
        int a0, a1, a2, b0, b1, b2;
        limbs3(w, e_c, a0, a1, a2);
        limbs3(z, e_c, b0, b1, b2);
#pragma unroll
        for (int l = 0; l < T; ++l) {
            put_byte(fw[l], e, limb_for<kPack>(l, col, a0, a1, a2));
            put_byte(fz[l], e, limb_for<kPack>(l, col, b0, b1, b2));
        }
    }
    i32x4* f = frag + ((st * kWords + word) * 2 * T) * 64 + lane;
#pragma unroll
    for (int l = 0; l < T; ++l) {
        f[l * 64] = fw[l];
        f[(T + l) * 64] = fz[l];
    }
}

// A^T X operands: frag[((st * kWords + word) * T + l) * 64 + lane] = tile l of
// X; byte e holds individual st*256 + 64 (lane >> 4) + 16 word + code_of_elem(e).
template <bool kPack>
__global__ void __launch_bounds__(256)
split_X_i8_kernel(const double* __restrict__ X, int64_t ldx, int nb, int64_t n,
               const double* __restrict__ cmax, int64_t nst, i32x4* __restrict__ frag)
{
    constexpr int T = tiles<kPack>();
    __shared__ int ex[16];
    column_scales(cmax, nb, ex);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nst * kWords * 64) return;
    const int lane = (int)(t & 63);
    const int word = (int)((t >> 6) % kWords);
    const int64_t st = t / (64 * kWords);
    const int g = lane >> 4, col = lane & 15, c = kPack ? (col & 7) : col;
    const int e_c = c < nb ? ex[c] : 0;
    i32x4 fx[T];
#pragma unroll
    for (int l = 0; l < T; ++l) fx[l] = i32x4{0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t i = st * kSuper + 64 * g + 16 * word + code_of_elem(e);
        const double x = (i < n && c < nb) ? X[(int64_t)c * ldx + i] : 0.0;
        int a0, a1, a2;
        limbs3(x, e_c, a0, a1, a2);
#pragma unroll
        for (int l = 0; l < T; ++l) put_byte(fx[l], e, limb_for<kPack>(l, col, a0, a1, a2));
    }
    i32x4* f = frag + ((st * kWords + word) * T) * 64 + lane;
#pragma unroll
    for (int l = 0; l < T; ++l) f[l * 64] = fx[l];
}

// Element e of the limb tiles acc[0..T-1] recombined to the exact integer sum
// of column (lane & 15) -- packed: of column (lane & 7), valid in lanes with
// (lane & 15) < 8, limb 1 taken from the lane 8 places up.  Called by every lane.
template <bool kPack>
__device__ __forceinline__ double recombine(const i32x4* acc, int e)
{
    const int64_t l0 = acc[0][e];
    const int64_t l1 = kPack ? (int64_t)__shfl_down(acc[0][e], 8, 16) : (int64_t)acc[1][e];
    const int64_t l2 = kPack ? acc[1][e] : acc[2][e];
    return (double)(l0 * 65536 + l1 * 256 + l2);
}

// ---------------------------------------------------------------------------
// A W main kernel: block = 4 waves x rtw row tiles x 16 rows, K split in
// super-tiles; partial[split][row][16]: exact integers (units of 2^-22 scale_c).
// ---------------------------------------------------------------------------
template <bool kPack>
__global__ void __launch_bounds__(256)
matmat_i8_kernel(const uint8_t* __restrict__ I, int64_t ldI, int64_t nI,
                 const i32x4* __restrict__ frag, int64_t nst, int64_t st_per_split,
                 double* __restrict__ partial)
{
    constexpr int T = tiles<kPack>();
    constexpr int kRTw = rtw<kPack>();
    constexpr int kOpsW = 2 * T;                    // operands per word: W' tiles, Z' tiles
    __shared__ i32x4 bs[kWords * kOpsW * 64];      // one super-tile of the operands
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    const int64_t row_base = (int64_t)blockIdx.x * (kMxWaves * kRTw * 16) + wave * (kRTw * 16);
    const int64_t st0 = (int64_t)blockIdx.y * st_per_split;
    const int64_t st1 = st0 + st_per_split < nst ? st0 + st_per_split : nst;
    i32x4 acc[kRTw][T];
#pragma unroll
    for (int t = 0; t < kRTw; ++t)
#pragma unroll
        for (int l = 0; l < T; ++l) acc[t][l] = i32x4{0, 0, 0, 0};
    for (int64_t st = st0; st < st1; ++st) {
        uint4 a[kRTw];
#pragma unroll
        for (int t = 0; t < kRTw; ++t)
            a[t] = *reinterpret_cast<const uint4*>(I + tiled_offset(row_base + 16 * t + r, st * 64 + 16 * g, ldI));
        const i32x4* src = frag + st * (kWords * kOpsW * 64);
        for (int q = threadIdx.x; q < kWords * kOpsW * 64; q += 256) bs[q] = src[q];
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kWords; ++w) {
            i32x4 bw[T], bz[T];
#pragma unroll
            for (int l = 0; l < T; ++l) {
                bw[l] = bs[(w * kOpsW + l) * 64 + lane];
                bz[l] = bs[(w * kOpsW + T + l) * 64 + lane];
            }
#pragma unroll
            for (int t = 0; t < kRTw; ++t) {
                const uint32_t d = w == 0 ? a[t].x : w == 1 ? a[t].y : w == 2 ? a[t].z : a[t].w;
                const i32x4 ac = raw_codes(d), am = missing_flags(ac);
#pragma unroll
                for (int l = 0; l < T; ++l) {
                    acc[t][l] = mfma_i8(ac, bw[l], acc[t][l]);
                    acc[t][l] = mfma_i8(am, bz[l], acc[t][l]);
                }
            }
        }
        __syncthreads();
    }
    double* out = partial + (int64_t)blockIdx.y * nI * 16;
#pragma unroll
    for (int t = 0; t < kRTw; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t row = row_base + 16 * t + 4 * g + e;
            const double v = recombine<kPack>(acc[t], e);
            if (!kPack || r < 8) out[row * 16 + r] = v;
        }
    }
}

// Y[i + c*ldy] = 2^(ex_c - 22) sum_split partial - K2_c for i < n, c < nb (col0
// offset).  The split sums are exact (integers below 2^53).
__global__ void __launch_bounds__(256)
matmat_i8_reduce_kernel(const double* __restrict__ partial, int nsplit, int64_t nI, int64_t n,
                     int nb, const double* __restrict__ cpart, const double* __restrict__ cmax,
                     double* __restrict__ Y, int64_t ldy)
{
    __shared__ double K2[16];
    __shared__ int ex[16];
    column_sums(cpart, nb, K2);
    column_scales(cmax, nb, ex);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 16) return;
    const int64_t i = t >> 4;
    const int c = (int)(t & 15);
    if (c >= nb) return;
    const double s = strided_sum(partial + i * 16 + c, nI * 16, nsplit);
    Y[(int64_t)c * ldy + i] = ldexp(s, ex[c] - kQBits) - K2[c];
}

// ---------------------------------------------------------------------------
// A^T X main kernel: block = 4 waves x rtr SNP tiles x 16 SNPs; K = individuals.
// partial[split][2][row][16]: sums with the code operand and the missing operand
// (exact integers, units of 2^-22 scale_c).
// ---------------------------------------------------------------------------
template <bool kPack>
__global__ void __launch_bounds__(256)
rmatmat_i8_kernel(const uint8_t* __restrict__ S, int64_t ldS, int64_t pS,
                  const i32x4* __restrict__ frag, int64_t nst, int64_t st_per_split,
                  double* __restrict__ partial)
{
    constexpr int T = tiles<kPack>();
    constexpr int kRTr = rtr<kPack>();
    __shared__ i32x4 bs[kWords * T * 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    const int64_t row_base = (int64_t)blockIdx.x * (kMxWaves * kRTr * 16) + wave * (kRTr * 16);
    const int64_t st0 = (int64_t)blockIdx.y * st_per_split;
    const int64_t st1 = st0 + st_per_split < nst ? st0 + st_per_split : nst;
    i32x4 accC[kRTr][T], accM[kRTr][T];
#pragma unroll
    for (int t = 0; t < kRTr; ++t)
#pragma unroll
        for (int l = 0; l < T; ++l) {
            accC[t][l] = i32x4{0, 0, 0, 0};
            accM[t][l] = i32x4{0, 0, 0, 0};
        }
    for (int64_t st = st0; st < st1; ++st) {
        uint4 a[kRTr];
#pragma unroll
        for (int t = 0; t < kRTr; ++t)
            a[t] = *reinterpret_cast<const uint4*>(S + tiled_offset(row_base + 16 * t + r, st * 64 + 16 * g, ldS));
        const i32x4* src = frag + st * (kWords * T * 64);
        for (int q = threadIdx.x; q < kWords * T * 64; q += 256) bs[q] = src[q];
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kWords; ++w) {
            i32x4 bx[T];
#pragma unroll
            for (int l = 0; l < T; ++l) bx[l] = bs[(w * T + l) * 64 + lane];
#pragma unroll
            for (int t = 0; t < kRTr; ++t) {
                const uint32_t d = w == 0 ? a[t].x : w == 1 ? a[t].y : w == 2 ? a[t].z : a[t].w;
                const i32x4 ac = raw_codes(d), am = missing_flags(ac);
#pragma unroll
                for (int l = 0; l < T; ++l) {
                    accC[t][l] = mfma_i8(ac, bx[l], accC[t][l]);
                    accM[t][l] = mfma_i8(am, bx[l], accM[t][l]);
                }
            }
        }
        __syncthreads();
    }
    double* out = partial + (int64_t)blockIdx.y * 2 * pS * 16;
#pragma unroll
    for (int t = 0; t < kRTr; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t row = row_base + 16 * t + 4 * g + e;
            const double vc = recombine<kPack>(accC[t], e), vm = recombine<kPack>(accM[t], e);
            if (!kPack || r < 8) {
                out[row * 16 + r] = vc;
                out[(pS + row) * 16 + r] = vm;
            }
        }
    }
}

// Z[j + c*ldz] = s_j ( 2^(ex_c - 22) (SC + (mu_j - 3) SM) - mu_j T_c )
__global__ void __launch_bounds__(256)
rmatmat_i8_reduce_kernel(const double* __restrict__ partial, int nsplit, int64_t pS, int64_t p,
                      int nb, const double* __restrict__ cpart, const double* __restrict__ cmax,
                      const double* __restrict__ mean, const double* __restrict__ inv_sd,
                      double* __restrict__ Z, int64_t ldz)
{
    __shared__ double T[16];
    __shared__ int ex[16];
    column_sums(cpart, nb, T);
    column_scales(cmax, nb, ex);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * 16) return;
    const int64_t j = t >> 4;
    const int c = (int)(t & 15);
    if (c >= nb) return;
    const double sc = strided_sum(partial + j * 16 + c, 2 * pS * 16, nsplit);
    const double sm = strided_sum(partial + (pS + j) * 16 + c, 2 * pS * 16, nsplit);
    const double mu = mean[j];
    const double u = ldexp(sc + (mu - 3.0) * sm, ex[c] - kQBits);
    Z[(int64_t)c * ldz + j] = inv_sd[j] * (u - mu * T[c]);
}

// ---------------------------------------------------------------------------
// FP64 single-vector products in seven int8 limbs
// ---------------------------------------------------------------------------
// The FP64 path's A v and A^T u on the int8 matrix cores, as the limb products
// above but with one vector carried to FP64 accuracy.  The vector is scaled by
// a power of two 2^ex at least its largest magnitude (for A v the largest of
// the missing-term vector z = (mu - 3) s v, which bounds |s v| and shares the
// scale), rounded to an integer q with |q| <= 2^52 -- the rounding is at most
// half a unit of 2^(ex - 52), the last place of a double at the scale -- and q
// is split into seven balanced 8-bit limbs, q = sum_l l_l 2^(8 (6 - l)).
// Column l < 7 of the B operand holds limb l; columns 7..15 are zero.
// v_mfma_i32_16x16x64_i8 adds every limb sum exactly (|code x limb| + |flag x
// limb| <= 512 per contraction index; a K split of at most 2^20 indices keeps
// every limb sum below 2^29), the recombination
//   S = (l0 2^24 + l1 2^16 + l2 2^8 + l3) 2^24 + (l4 2^16 + l5 2^8 + l6)
// is exact up to its last addition (both brackets are integers below 2^53), so
// each split's partial carries one FP64 rounding besides the quantisation of
// the vector: the accuracy of a plain FP64 sum.
//   (A v)_i   = 2^(ex - 52) (sum_j c_ij q(s v)_j + sum_j m_ij q(z)_j) - sum_j mu_j s_j v_j
//   (A^T u)_j = s_j ( 2^(ex - 52) (SC_j + (mu_j - 3) SM_j) - mu_j sum_i u_i ),
//               SC_j = sum_i c_ij q(u)_i, SM_j = sum_i m_ij q(u)_i
// The mean terms are added by split 0; the FP64 reduce kernels add the splits,
// scale by s_j (A^T u) and apply the Lanczos recurrence term.
constexpr int kLimbs = 7;
constexpr int kQ64 = 52;
constexpr int64_t kLimbMaxSt = ((int64_t)1 << 20) / kSuper;   // super-tiles per K split
constexpr int kRTv = 4;    // A v: row tiles per wave (256 rows per workgroup)
constexpr int kRTu = 4;    // A^T u: row tiles per wave (256 rows per workgroup)
constexpr int kDepthV = 2;  // A v: super-tiles of codes loaded ahead (2: 1.6% faster than 1)
constexpr int kDepthU = 1;  // A^T u: one (two measured no faster)

__device__ __forceinline__ int64_t quantise52(double x, int ex)
{
    return (int64_t)rint(ldexp(x, kQ64 - ex));
}

// Limb fragments of kVec vectors (kVec <= 2; kOps = 1: x; kOps = 2: w = s v and
// z = (mu - 3) w), vector c at x + c ldx with its own scale 2^ex[c].  One
// workgroup per super-tile of 256 contraction indices, one thread per index:
// the thread quantises its entries once and writes their seven limbs as bytes
// of the fragment image in LDS, which the workgroup then stores as whole
// operands.  frag[((st * kWords + word) * kOps + op) * 64 + lane]: byte e of
// lane (g, col) holds index st*256 + 64 g + 16 word + code_of_elem(e), limb
// col - 7c of vector c = col / 7 (zero for col >= 7 kVec): the seven limb
// columns of two vectors fill 14 of the 16 columns of one MFMA tile, so a pair
// costs the matrix cores what one vector does.
template <int kOps, int kVec>
__device__ __forceinline__ void limb_frag_body(const double* __restrict__ x, int64_t ldx,
                                               int64_t len, const double* __restrict__ mean,
                                               const double* __restrict__ inv_sd,
                                               const double* __restrict__ cmax,
                                               i32x4* __restrict__ frag, int64_t st)
{
    static_assert(kVec == 1 || kVec == 2, "one or two vectors per MFMA tile");
    __shared__ i32x4 img[kWords * kOps * 64];
    __shared__ int ex[kVec];
    column_scales(cmax, kVec, ex);
    for (int q = threadIdx.x; q < kWords * kOps * 64; q += 256) img[q] = i32x4{0, 0, 0, 0};
    __syncthreads();
    const int o = threadIdx.x;                       // index within the super-tile
    const int64_t j = st * kSuper + o;
    const int g = o >> 6, word = (o >> 4) & 3, c = o & 15;
    const int e = (c & 3) * 4 + (c >> 2);            // code_of_elem(e) == c
    uint8_t* bytes = reinterpret_cast<uint8_t*>(img);
#pragma unroll
    for (int vc = 0; vc < kVec; ++vc) {
        const double* xv = x + (int64_t)vc * ldx;
        double val[kOps];
        if (kOps == 2) {
            const double w = j < len ? inv_sd[j] * xv[j] : 0.0;
            val[0] = w;
            val[kOps - 1] = j < len ? (mean[j] - 3.0) * w : 0.0;
        } else {
            val[0] = j < len ? xv[j] : 0.0;
        }
#pragma unroll
        for (int op = 0; op < kOps; ++op) {
            int64_t q = quantise52(val[op], ex[vc]);
            int lim[kLimbs];
#pragma unroll
            for (int k = kLimbs - 1; k >= 1; --k) {
                lim[k] = (int)(((q + 128) & 255) - 128);
                q = (q - lim[k]) >> 8;
            }
            lim[0] = (int)q;
#pragma unroll
            for (int l = 0; l < kLimbs; ++l)
                bytes[(((word * kOps + op) * 64) + g * 16 + kLimbs * vc + l) * 16 + e] =
                    (uint8_t)(lim[l] & 0xFF);
        }
    }
    __syncthreads();
    i32x4* f = frag + st * (kWords * kOps * 64);
    for (int q = threadIdx.x; q < kWords * kOps * 64; q += 256) f[q] = img[q];
}

template <int kOps, int kVec>
__global__ void __launch_bounds__(256)
limb_frag_kernel(const double* __restrict__ x, int64_t ldx, int64_t len,
                 const double* __restrict__ mean, const double* __restrict__ inv_sd,
                 const double* __restrict__ cmax, i32x4* __restrict__ frag)
{
    limb_frag_body<kOps, kVec>(x, ldx, len, mean, inv_sd, cmax, frag, blockIdx.x);
}

// Element e of accumulator a recombined from the seven limb columns base ..
// base + 6 of the lane's 16-lane group (every lane calls it; the value is that
// of its group).
__device__ __forceinline__ double limb_sum(const i32x4& a, int e, int lane, int base = 0)
{
    int32_t l[kLimbs];
#pragma unroll
    for (int k = 0; k < kLimbs; ++k) l[k] = __shfl(a[e], (lane & 48) + base + k, 64);
    const int64_t hi = ((int64_t)l[0] << 24) + ((int64_t)l[1] << 16) + ((int64_t)l[2] << 8) + l[3];
    const int64_t lo = ((int64_t)l[4] << 16) + ((int64_t)l[5] << 8) + l[6];
    return (double)hi * 16777216.0 + (double)lo;
}

// Main kernel.  kAv: A v over layout I (rows = individuals, K = SNPs), one
// accumulator per row tile fed by the code operand with the limbs of s v and
// the missing operand with the limbs of z.  Otherwise A^T u over layout S
// (rows = SNPs, K = individuals), a code and a missing accumulator sharing the
// limbs of u.  Workgroup = 4 waves x kRT row tiles of 16 rows; the K range of
// one split is walked in super-tiles of 256, the next super-tile's codes and
// fragments loaded while the current one is multiplied (fragments double
// buffered in LDS, one barrier per super-tile).  partial[split * rows_pad +
// row] = the split's share of the product (before s_j for A^T u).
// kDepth: super-tiles of codes in flight ahead of the one being multiplied
// (the three code buffers rotate statically over an unrolled loop, so no
// register copies).
template <bool kAv, int kDepth = kAv ? kDepthV : kDepthU, int kVec = 1>
__device__ __forceinline__ void limb_product_body(const uint8_t* __restrict__ L, int64_t ldL,
                                                  int64_t rows_pad, int64_t rows,
                                                  const i32x4* __restrict__ frag, int64_t nst,
                                                  int64_t st_per, int split, int rb,
                                                  const double* __restrict__ cpart,
                                                  const double* __restrict__ cmax,
                                                  const double* __restrict__ mean,
                                                  double* __restrict__ partial)
{
    static_assert(kDepth == 1 || kDepth == 2, "code prefetch depth");
    constexpr int kRT = kAv ? kRTv : kRTu;
    constexpr int kOps = kAv ? 2 : 1;
    constexpr int kAcc = kAv ? 1 : 2;
    constexpr int kFr = kWords * kOps * 64;     // fragments per super-tile
    constexpr int kFrT = kFr / 256;             // per thread
    __shared__ i32x4 bs[2][kFr];
    __shared__ double ksum[kVec];
    __shared__ int ex[kVec];
    column_sums(cpart, kVec, ksum);
    column_scales(cmax, kVec, ex);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    const int64_t row_base = (int64_t)rb * (kMxWaves * kRT * 16) + wave * (kRT * 16);
    const int64_t st0 = (int64_t)split * st_per;
    const int64_t st1 = st0 + st_per < nst ? st0 + st_per : nst;
    i32x4 acc[kRT][kAcc];
#pragma unroll
    for (int t = 0; t < kRT; ++t)
#pragma unroll
        for (int q = 0; q < kAcc; ++q) acc[t][q] = i32x4{0, 0, 0, 0};
    auto load_codes = [&](uint4 (&dst)[kRT], int64_t st) {
        const int64_t s = st < st1 ? st : st1 - 1;   // past the end: the last one again
#pragma unroll
        for (int t = 0; t < kRT; ++t)
            dst[t] = *reinterpret_cast<const uint4*>(
                L + tiled_offset(row_base + 16 * t + r, s * 64 + 16 * g, ldL));
    };
    uint4 a0[kRT], a1[kRT], a2[kRT];
    if (st0 < st1) {
        load_codes(a0, st0);
        if (kDepth > 1) load_codes(a1, st0 + 1);
#pragma unroll
        for (int k = 0; k < kFrT; ++k) bs[0][threadIdx.x + 256 * k] = frag[st0 * kFr + threadIdx.x + 256 * k];
    }
    __syncthreads();
    int buf = 0;
    // one super-tile: codes of st + kDepth into `ahead`, fragments of st + 1 into
    // registers, the products of `cur` with the fragments in bs[buf], then the
    // fragments handed over through the other buffer
    auto step = [&](int64_t st, const uint4 (&cur)[kRT], uint4 (&ahead)[kRT]) {
        load_codes(ahead, st + kDepth);
        const int64_t stn = st + 1 < st1 ? st + 1 : st;
        i32x4 fr[kFrT];
#pragma unroll
        for (int k = 0; k < kFrT; ++k) fr[k] = frag[stn * kFr + threadIdx.x + 256 * k];
#pragma unroll
        for (int w = 0; w < kWords; ++w) {
            const i32x4 b0 = bs[buf][(w * kOps) * 64 + lane];
            const i32x4 b1 = kAv ? bs[buf][(w * kOps + 1) * 64 + lane] : b0;
#pragma unroll
            for (int t = 0; t < kRT; ++t) {
                const uint32_t d = w == 0 ? cur[t].x : w == 1 ? cur[t].y : w == 2 ? cur[t].z : cur[t].w;
                const i32x4 ac = raw_codes(d), am = missing_flags(ac);
                if (kAv) {
                    acc[t][0] = mfma_i8(ac, b0, acc[t][0]);
                    acc[t][0] = mfma_i8(am, b1, acc[t][0]);
                } else {
                    acc[t][0] = mfma_i8(ac, b0, acc[t][0]);
                    acc[t][kAcc - 1] = mfma_i8(am, b0, acc[t][kAcc - 1]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kFrT; ++k) bs[buf ^ 1][threadIdx.x + 256 * k] = fr[k];
        __syncthreads();
        buf ^= 1;
    };
    if (kDepth == 1) {
        for (int64_t st = st0; st < st1; st += 2) {
            step(st, a0, a1);
            if (st + 1 < st1) step(st + 1, a1, a0);
        }
    } else {
        for (int64_t st = st0; st < st1; st += 3) {
            step(st, a0, a2);
            if (st + 1 < st1) step(st + 1, a1, a0);
            if (st + 2 < st1) step(st + 2, a2, a1);
        }
    }
#pragma unroll
    for (int vc = 0; vc < kVec; ++vc) {
        double* out = partial + ((int64_t)split * kVec + vc) * rows_pad;
        const int e0 = ex[vc];
#pragma unroll
        for (int t = 0; t < kRT; ++t) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = row_base + 16 * t + 4 * g + e;
                double val;
                if (kAv) {
                    val = ldexp(limb_sum(acc[t][0], e, lane, kLimbs * vc), e0 - kQ64);
                    if (split == 0) val -= ksum[vc];
                } else {
                    const double sc = limb_sum(acc[t][0], e, lane, kLimbs * vc);
                    const double sm = limb_sum(acc[t][kAcc - 1], e, lane, kLimbs * vc);
                    const double mu = row < rows ? mean[row] : 0.0;
                    val = ldexp(sc + (mu - 3.0) * sm, e0 - kQ64);
                    if (split == 0) val -= mu * ksum[vc];
                }
                if (r == 0) out[row] = val;
            }
        }
    }
}

template <bool kAv, int kVec>
__global__ void __launch_bounds__(256)
limb_product_kernel(const uint8_t* __restrict__ L, int64_t ldL, int64_t rows_pad, int64_t rows,
                    const i32x4* __restrict__ frag, int64_t nst, int64_t st_per, int nsplit,
                    int nrb, int xcd, const double* __restrict__ cpart,
                    const double* __restrict__ cmax, const double* __restrict__ mean,
                    double* __restrict__ partial)
{
    int split, rb;
    block_coords(blockIdx.x, nsplit, nrb, xcd, split, rb);
    limb_product_body<kAv, kAv ? kDepthV : kDepthU, kVec>(L, ldL, rows_pad, rows, frag, nst, st_per,
                                                          split, rb, cpart, cmax, mean, partial);
}

// Batched A^T u in limbs (the batched path with the S layout per problem).
// Problem q = blockIdx.y; u_j at U + j n; inactive problems skip (whole blocks).
__global__ void __launch_bounds__(256)
blimb_colsum_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state)
{
    const BatchDesc& D = desc[blockIdx.y];
    if (!*D.active) return;
    const int64_t j = state[0];
    colsum_chunk(D.U + j * D.n, D.n, nullptr, nullptr, 0.0, blockIdx.x, D.lcpart + blockIdx.x,
                 D.lcmax + blockIdx.x);
}

__global__ void __launch_bounds__(256)
blimb_frag_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state)
{
    const BatchDesc& D = desc[blockIdx.y];
    if (!*D.active || (int64_t)blockIdx.x >= D.nstX) return;
    const int64_t j = state[0];
    limb_frag_body<1, 1>(D.U + j * D.n, D.n, D.n, nullptr, nullptr, D.lcmax,
                         static_cast<i32x4*>(D.lfrag), blockIdx.x);
}

// Persistent over the (split, row block) tiles of every active problem:
// tile0[q] is problem q's first tile; tile l of a problem is split l / nrb, row
// block l % nrb.  A barrier opens every tile, so the shared scalars and operand
// buffers of the previous tile are no longer in use.
__global__ void __launch_bounds__(256)
blimb_rmatvec_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ tile0, int count,
                     const int* __restrict__ state)
{
    __shared__ int t0[kMaxBatch + 1];
    for (int i = threadIdx.x; i <= count; i += blockDim.x) t0[i] = tile0[i];
    __syncthreads();
    const int total = t0[count];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = count - 1;          // owner: the last q with t0[q] <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (t0[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const BatchDesc& D = desc[lo];
        if (!*D.active) continue;            // the same for the whole workgroup
        const int l = t - t0[lo];
        __syncthreads();
        limb_product_body<false>(D.S, D.ldS, D.pP, D.p, static_cast<const i32x4*>(D.lfrag),
                                 D.nstX, D.limb_st_per, l / D.limb_nrb, l % D.limb_nrb, D.lcpart,
                                 D.lcmax, D.mean, D.partial);
    }
}

void launch_blimb_rmatvec(const BatchDesc* d, const int* tile0, int count, const int* state,
                          int grid, int64_t max_nst, hipStream_t s)
{
    hipLaunchKernelGGL(blimb_colsum_kernel, dim3(kCsSplit, count), dim3(256), 0, s, d, state);
    GKL_LAUNCH_CHECK("blimb_colsum_kernel");
    hipLaunchKernelGGL(blimb_frag_kernel, dim3((unsigned int)max_nst, count), dim3(256), 0, s, d,
                       state);
    GKL_LAUNCH_CHECK("blimb_frag_kernel");
    hipLaunchKernelGGL(blimb_rmatvec_kernel, dim3(grid), dim3(256), 0, s, d, tile0, count, state);
    GKL_LAUNCH_CHECK("blimb_rmatvec_kernel");
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
// K splits of a split-BF16 product over `rows` padded rows in workgroups of
// `wg_rows` rows and nst super-tiles of K: enough workgroups to cover the chip
// several times, at most max_split splits (bounds the partial-sum traffic), a
// multiple of 8 from 8 on so that each split's row blocks share one XCD.
static BfSplit bf16_split(int64_t rows, int wg_rows, int64_t nst, int64_t max_split,
                          int64_t target = 2048)
{
    BfSplit g;
    g.nrb = (int)(rows / wg_rows);
    int64_t want = (target + g.nrb - 1) / g.nrb;
    if (want > max_split) want = max_split;
    if (want > nst) want = nst;
    if (want < 1) want = 1;
    if (want >= 8) want = want / 8 * 8;
    g.st_per = (nst + want - 1) / want;
    g.nsplit = (int)((nst + g.st_per - 1) / g.st_per);
    g.xcd = g.nsplit >= 8 && g.nsplit % 8 == 0 ? 1 : 0;
    return g;
}

// The same for the FP64 limb products, with at most kLimbMaxSt super-tiles per split.
static BfSplit limb_split(int64_t rows, int wg_rows, int64_t nst, int64_t max_split,
                          int64_t target = 2048)
{
    const int64_t min_split = (nst + kLimbMaxSt - 1) / kLimbMaxSt;
    BfSplit g = bf16_split(rows, wg_rows, nst, max_split > min_split ? max_split : min_split,
                           target);
    if (g.st_per > kLimbMaxSt) {
        g.st_per = kLimbMaxSt;
        g.nsplit = (int)((nst + g.st_per - 1) / g.st_per);
        g.xcd = g.nsplit >= 8 && g.nsplit % 8 == 0 ? 1 : 0;
    }
    return g;
}

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
    const int64_t rbW = m.nI / (kMxWaves * rtw<true>() * 16);
    int64_t sW = (1024 + rbW - 1) / rbW;
    const int64_t capW = m.nstW / 8 > 1 ? m.nstW / 8 : 1;   // >= 2048 SNPs per split
    if (sW > capW) sW = capW;
    if (sW < 1) sW = 1;
    m.stW = (m.nstW + sW - 1) / sW;
    m.splitW = (int)((m.nstW + m.stW - 1) / m.stW);
    const int64_t rbX = m.pS / (kMxWaves * rtr<true>() * 16);
    int64_t sX = (1024 + rbX - 1) / rbX;
    const int64_t capX = m.nstX / 8 > 1 ? m.nstX / 8 : 1;
    if (sX > capX) sX = capX;
    if (sX < 1) sX = 1;
    m.stX = (m.nstX + sX - 1) / sX;
    m.splitX = (int)((m.nstX + m.stX - 1) / m.stX);
    // split BF16, per column class (b <= 8: 8 partial columns, <= 16: 16, <= 32: 32)
    const int64_t mbytes = m.nI * m.ldI;
    // FP64 limb products: partial traffic (8 B per row and split) at most 1/16
    // of the matrix, K splits of at most 2^20 (exact limb sums)
    // A v: about eight rounds of the 768 workgroups the chip holds at once (three
    // per CU), so that the last round is a small share, but K splits of at
    // least 12 super-tiles; measured at 10,000 x 100,000 and 50,000 x 500,000,
    // where 8 splits (two rounds and a sliver) took 10% longer than 32
    int64_t limb_capW = m.nstW / 12;
    if (limb_capW < 1) limb_capW = 1;
    if (limb_capW > mbytes / (16 * 8 * m.nI)) limb_capW = mbytes / (16 * 8 * m.nI);
    m.limbW = limb_split(m.nI, kMxWaves * kRTv * 16, m.nstW, limb_capW, 6144);
    m.limbX = limb_split(m.pS, kMxWaves * kRTu * 16, m.nstX, mbytes / (16 * 8 * m.pS));
    for (int c = 0; c < 3; ++c) {
        const int64_t kcs = c == 0 ? 8 : 16 * c;
        m.bfW[c] = bf16_split(m.nI, kMxWaves * kRTW * 16, m.nstW, mbytes / (4 * 2 * 8 * m.nI * kcs));
        m.bfX[c] = bf16_split(m.pS, kMxWaves * kRTX * 16, m.nstX, mbytes / (4 * 2 * 8 * 2 * m.pS * kcs));
    }
    return m;
}

size_t mixed_frag_bytes(const MixedShape& m)
{
    // the larger of the two formats: split BF16 (up to 8 operands per K step of 32
    // for A W, 4 for A^T X) and int8 limbs (6 operands per K step of 64)
    const size_t a = (size_t)m.nstW * kKSteps * 8 * 64 * sizeof(bf16x8);
    const size_t b = (size_t)m.nstX * kKSteps * 4 * 64 * sizeof(bf16x8);
    const size_t c = (size_t)m.nstW * kWords * 2 * tiles<false>() * 64 * sizeof(i32x4);
    const size_t d = (size_t)m.nstX * kWords * tiles<false>() * 64 * sizeof(i32x4);
    return std::max(std::max(a, b), std::max(c, d));
}

size_t mixed_partial_elems(const MixedShape& m)
{
    size_t e = std::max((size_t)m.splitW * (size_t)m.nI * 16, (size_t)m.splitX * 2 * (size_t)m.pS * 16);
    // FP64-exact pairs: two columns per split
    e = std::max(e, (size_t)m.limbW.nsplit * 2 * (size_t)m.nI);
    e = std::max(e, (size_t)m.limbX.nsplit * 2 * (size_t)m.pS);
    for (int c = 0; c < 3; ++c) {
        const size_t kcs = c == 0 ? 8 : 16 * c;
        e = std::max(e, (size_t)m.bfW[c].nsplit * (size_t)m.nI * kcs);
        if (m.bfX[c].nsplit > 1) e = std::max(e, (size_t)m.bfX[c].nsplit * 2 * (size_t)m.pS * kcs);
    }
    return e;
}

BfSplit limb_batch_split(const MixedShape& m, int64_t target)
{
    BfSplit g;
    g.nrb = (int)(m.pS / (kMxWaves * kRTu * 16));
    int64_t ns = (target + g.nrb - 1) / g.nrb;
    const int64_t lo = (m.nstX + kLimbMaxSt - 1) / kLimbMaxSt;
    if (ns > m.nstX) ns = m.nstX;
    if (ns < lo) ns = lo;
    if (ns < 1) ns = 1;
    g.st_per = (m.nstX + ns - 1) / ns;
    g.nsplit = (int)((m.nstX + g.st_per - 1) / g.st_per);
    g.xcd = 0;
    return g;
}

size_t limb_frag_bytes(const MixedShape& m)
{
    return std::max((size_t)m.nstW * kWords * 2, (size_t)m.nstX * kWords) * 64 * sizeof(i32x4);
}

size_t limb_partial_elems(const MixedShape& m)
{
    return std::max((size_t)m.limbW.nsplit * (size_t)m.nI, (size_t)m.limbX.nsplit * (size_t)m.pS);
}

int launch_matvec_limb(const MixedShape& m, const uint8_t* I, const ColStats& st, const double* v,
                       MatvecWork& w, hipStream_t s, const hipEvent_t* ev)
{
    const BfSplit& gm = m.limbW;
    i32x4* frag = reinterpret_cast<i32x4*>(w.lfrag);
    hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, 1), dim3(256), 0, s, v, m.p, m.p, st.mean,
                       st.inv_sd, 3.0, w.lcpart, w.lcmax);
    GKL_LAUNCH_CHECK("colsum_kernel");
    hipLaunchKernelGGL((limb_frag_kernel<2, 1>), dim3((unsigned int)m.nstW), dim3(256), 0, s, v, m.p,
                       m.p, st.mean, st.inv_sd, w.lcmax, frag);
    GKL_LAUNCH_CHECK("limb_frag_kernel<2>");
    if (ev) GKL_HIP(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL((limb_product_kernel<true, 1>), dim3((unsigned int)(gm.nsplit * gm.nrb)),
                       dim3(256), 0, s, I, m.ldI, m.nI, m.n, frag, m.nstW, gm.st_per, gm.nsplit,
                       gm.nrb, gm.xcd, w.lcpart, w.lcmax, st.mean, w.partial);
    GKL_LAUNCH_CHECK("limb_product_kernel<A v>");
    if (ev) GKL_HIP(hipEventRecord(ev[1], s));
    return gm.nsplit;
}

int launch_rmatvec_limb(const MixedShape& m, const uint8_t* S, const ColStats& st, const double* u,
                        MatvecWork& w, hipStream_t s, const hipEvent_t* ev)
{
    const BfSplit& gm = m.limbX;
    i32x4* frag = reinterpret_cast<i32x4*>(w.lfrag);
    hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, 1), dim3(256), 0, s, u, m.n, m.n, nullptr,
                       nullptr, 0.0, w.lcpart, w.lcmax);
    GKL_LAUNCH_CHECK("colsum_kernel");
    hipLaunchKernelGGL((limb_frag_kernel<1, 1>), dim3((unsigned int)m.nstX), dim3(256), 0, s, u, m.n,
                       m.n, nullptr, nullptr, w.lcmax, frag);
    GKL_LAUNCH_CHECK("limb_frag_kernel<1>");
    if (ev) GKL_HIP(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL((limb_product_kernel<false, 1>), dim3((unsigned int)(gm.nsplit * gm.nrb)),
                       dim3(256), 0, s, S, m.ldS, m.pS, m.p, frag, m.nstX, gm.st_per, gm.nsplit,
                       gm.nrb, gm.xcd, w.lcpart, w.lcmax, st.mean, w.partial);
    GKL_LAUNCH_CHECK("limb_product_kernel<A^T u>");
    if (ev) GKL_HIP(hipEventRecord(ev[1], s));
    return gm.nsplit;
}

template <bool kPack, int kT>
static void matmat_bf16_run(const MixedShape& m, const uint8_t* I, const ColStats& st,
                            const double* W, int64_t ldw, int b, double* Y, int64_t ldy,
                            MixedWork& w, hipStream_t s, const hipEvent_t* ev)
{
    constexpr int kcs = kPack ? 8 : 16 * kT;
    const BfSplit& gm = m.bfW[kPack ? 0 : kT];
    bf16x8* frag = reinterpret_cast<bf16x8*>(w.frag);
    hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, b), dim3(256), 0, s, W, ldw, m.p, st.mean,
                       st.inv_sd, 4.0, w.cpart, w.cmax);
    GKL_LAUNCH_CHECK("colsum_kernel");
    hipLaunchKernelGGL((split_W_bf16_kernel<kPack, kT>), dim3(ceil_div(m.nstW * kKSteps * 64, 256)),
                       dim3(256), 0, s, W, ldw, b, m.p, st.mean, st.inv_sd, w.cmax, m.nstW, frag);
    GKL_LAUNCH_CHECK("split_W_bf16_kernel");
    if (ev) GKL_HIP(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL((matmat_bf16_kernel<kPack, kT>), dim3((unsigned int)(gm.nsplit * gm.nrb)),
                       dim3(256), 0, s, I, m.ldI, m.nI, frag, m.nstW, gm.st_per, gm.nsplit, gm.nrb,
                       gm.xcd, w.partial);
    GKL_LAUNCH_CHECK("matmat_bf16_kernel");
    if (ev) GKL_HIP(hipEventRecord(ev[1], s));
    hipLaunchKernelGGL(matmat_bf16_reduce_kernel, dim3(ceil_div(m.n * kcs, 256)), dim3(256), 0, s,
                       w.partial, gm.nsplit, m.nI, m.n, b, kcs, w.cpart, w.cmax, Y, ldy);
    GKL_LAUNCH_CHECK("matmat_bf16_reduce_kernel");
}

static void matmat_bf16(const MixedShape& m, const uint8_t* I, const ColStats& st, const double* W,
                        int64_t ldw, int b, double* Y, int64_t ldy, MixedWork& w, hipStream_t s,
                        const hipEvent_t* ev)
{
    if (b <= 8) matmat_bf16_run<true, 1>(m, I, st, W, ldw, b, Y, ldy, w, s, ev);
    else if (b <= 16) matmat_bf16_run<false, 1>(m, I, st, W, ldw, b, Y, ldy, w, s, ev);
    else matmat_bf16_run<false, 2>(m, I, st, W, ldw, b, Y, ldy, w, s, ev);
}

template <bool kPack, int kT>
static void rmatmat_bf16_run(const MixedShape& m, const uint8_t* S, const ColStats& st,
                             const double* X, int64_t ldx, int b, double* Z, int64_t ldz,
                             MixedWork& w, hipStream_t s, const hipEvent_t* ev)
{
    constexpr int kcs = kPack ? 8 : 16 * kT;
    const BfSplit& gm = m.bfX[kPack ? 0 : kT];
    bf16x8* frag = reinterpret_cast<bf16x8*>(w.frag);
    hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, b), dim3(256), 0, s, X, ldx, m.n, nullptr,
                       nullptr, 0.0, w.cpart, w.cmax);
    GKL_LAUNCH_CHECK("colsum_kernel");
    hipLaunchKernelGGL((split_X_bf16_kernel<kPack, kT>), dim3(ceil_div(m.nstX * kKSteps * 64, 256)),
                       dim3(256), 0, s, X, ldx, b, m.n, w.cmax, m.nstX, frag);
    GKL_LAUNCH_CHECK("split_X_bf16_kernel");
    if (ev) GKL_HIP(hipEventRecord(ev[0], s));
    const dim3 grid((unsigned int)(gm.nsplit * gm.nrb));
    if (gm.nsplit == 1)
        hipLaunchKernelGGL((rmatmat_bf16_kernel<kPack, kT, true>), grid, dim3(256), 0, s, S, m.ldS,
                           m.pS, frag, m.nstX, gm.st_per, gm.nsplit, gm.nrb, gm.xcd, w.partial, m.p,
                           b, w.cpart, w.cmax, st.mean, st.inv_sd, Z, ldz);
    else
        hipLaunchKernelGGL((rmatmat_bf16_kernel<kPack, kT, false>), grid, dim3(256), 0, s, S, m.ldS,
                           m.pS, frag, m.nstX, gm.st_per, gm.nsplit, gm.nrb, gm.xcd, w.partial, m.p,
                           b, w.cpart, w.cmax, st.mean, st.inv_sd, Z, ldz);
    GKL_LAUNCH_CHECK("rmatmat_bf16_kernel");
    if (ev) GKL_HIP(hipEventRecord(ev[1], s));
    if (gm.nsplit > 1) {
        hipLaunchKernelGGL(rmatmat_bf16_reduce_kernel, dim3(ceil_div(m.p * kcs, 256)), dim3(256), 0, s,
                           w.partial, gm.nsplit, m.pS, m.p, b, kcs, w.cpart, w.cmax, st.mean,
                           st.inv_sd, Z, ldz);
        GKL_LAUNCH_CHECK("rmatmat_bf16_reduce_kernel");
    }
}

static void rmatmat_bf16(const MixedShape& m, const uint8_t* S, const ColStats& st, const double* X,
                         int64_t ldx, int b, double* Z, int64_t ldz, MixedWork& w, hipStream_t s,
                         const hipEvent_t* ev)
{
    if (b <= 8) rmatmat_bf16_run<true, 1>(m, S, st, X, ldx, b, Z, ldz, w, s, ev);
    else if (b <= 16) rmatmat_bf16_run<false, 1>(m, S, st, X, ldx, b, Z, ldz, w, s, ev);
    else rmatmat_bf16_run<false, 2>(m, S, st, X, ldx, b, Z, ldz, w, s, ev);
}

static void matmat_i8(const MixedShape& m, const uint8_t* I, const ColStats& st, const double* W,
                      int64_t ldw, int b, double* Y, int64_t ldy, MixedWork& w, hipStream_t s, const hipEvent_t* ev)
{
    for (int col0 = 0; col0 < b; col0 += 16) {
        const int nb = b - col0 < 16 ? b - col0 : 16;
        const double* Wc = W + (int64_t)col0 * ldw;
        hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, nb), dim3(256), 0, s, Wc, ldw, m.p,
                           st.mean, st.inv_sd, 3.0, w.cpart, w.cmax);
        GKL_LAUNCH_CHECK("colsum_kernel");
        const int64_t nthr = m.nstW * kWords * 64;
        const dim3 gsplit(ceil_div(nthr, 256));
        const unsigned int rows = (unsigned int)(nb <= 8 ? rtw<true>() : rtw<false>()) * kMxWaves * 16;
        dim3 grid((unsigned int)(m.nI / rows), (unsigned int)m.splitW);
        i32x4* frag = reinterpret_cast<i32x4*>(w.frag);
        if (nb <= 8) {
            hipLaunchKernelGGL(split_W_i8_kernel<true>, gsplit, dim3(256), 0, s, Wc, ldw, nb, m.p,
                               st.mean, st.inv_sd, w.cmax, m.nstW, frag);
            GKL_LAUNCH_CHECK("split_W_i8_kernel");
            if (ev && col0 == 0) GKL_HIP(hipEventRecord(ev[0], s));
            hipLaunchKernelGGL(matmat_i8_kernel<true>, grid, dim3(256), 0, s, I, m.ldI, m.nI, frag,
                               m.nstW, m.stW, w.partial);
        } else {
            hipLaunchKernelGGL(split_W_i8_kernel<false>, gsplit, dim3(256), 0, s, Wc, ldw, nb, m.p,
                               st.mean, st.inv_sd, w.cmax, m.nstW, frag);
            GKL_LAUNCH_CHECK("split_W_i8_kernel");
            if (ev && col0 == 0) GKL_HIP(hipEventRecord(ev[0], s));
            hipLaunchKernelGGL(matmat_i8_kernel<false>, grid, dim3(256), 0, s, I, m.ldI, m.nI, frag,
                               m.nstW, m.stW, w.partial);
        }
        GKL_LAUNCH_CHECK("matmat_i8_kernel");
        if (ev && col0 + 16 >= b) GKL_HIP(hipEventRecord(ev[1], s));
        hipLaunchKernelGGL(matmat_i8_reduce_kernel, dim3(ceil_div(m.n * 16, 256)), dim3(256), 0, s,
                           w.partial, m.splitW, m.nI, m.n, nb, w.cpart, w.cmax,
                           Y + (int64_t)col0 * ldy, ldy);
        GKL_LAUNCH_CHECK("matmat_i8_reduce_kernel");
    }
}

static void rmatmat_i8(const MixedShape& m, const uint8_t* S, const ColStats& st, const double* X,
                       int64_t ldx, int b, double* Z, int64_t ldz, MixedWork& w, hipStream_t s, const hipEvent_t* ev)
{
    for (int col0 = 0; col0 < b; col0 += 16) {
        const int nb = b - col0 < 16 ? b - col0 : 16;
        const double* Xc = X + (int64_t)col0 * ldx;
        hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, nb), dim3(256), 0, s, Xc, ldx, m.n, nullptr,
                           nullptr, 0.0, w.cpart, w.cmax);
        GKL_LAUNCH_CHECK("colsum_kernel");
        const int64_t nthr = m.nstX * kWords * 64;
        const dim3 gsplit(ceil_div(nthr, 256));
        const unsigned int rows = (unsigned int)(nb <= 8 ? rtr<true>() : rtr<false>()) * kMxWaves * 16;
        dim3 grid((unsigned int)(m.pS / rows), (unsigned int)m.splitX);
        i32x4* frag = reinterpret_cast<i32x4*>(w.frag);
        if (nb <= 8) {
            hipLaunchKernelGGL(split_X_i8_kernel<true>, gsplit, dim3(256), 0, s, Xc, ldx, nb, m.n,
                               w.cmax, m.nstX, frag);
            GKL_LAUNCH_CHECK("split_X_i8_kernel");
            if (ev && col0 == 0) GKL_HIP(hipEventRecord(ev[0], s));
            hipLaunchKernelGGL(rmatmat_i8_kernel<true>, grid, dim3(256), 0, s, S, m.ldS, m.pS, frag,
                               m.nstX, m.stX, w.partial);
        } else {
            hipLaunchKernelGGL(split_X_i8_kernel<false>, gsplit, dim3(256), 0, s, Xc, ldx, nb, m.n,
                               w.cmax, m.nstX, frag);
            GKL_LAUNCH_CHECK("split_X_i8_kernel");
            if (ev && col0 == 0) GKL_HIP(hipEventRecord(ev[0], s));
            hipLaunchKernelGGL(rmatmat_i8_kernel<false>, grid, dim3(256), 0, s, S, m.ldS, m.pS, frag,
                               m.nstX, m.stX, w.partial);
        }
        GKL_LAUNCH_CHECK("rmatmat_i8_kernel");
        if (ev && col0 + 16 >= b) GKL_HIP(hipEventRecord(ev[1], s));
        hipLaunchKernelGGL(rmatmat_i8_reduce_kernel, dim3(ceil_div(m.p * 16, 256)), dim3(256), 0, s,
                           w.partial, m.splitX, m.pS, m.p, nb, w.cpart, w.cmax, st.mean, st.inv_sd,
                           Z + (int64_t)col0 * ldz, ldz);
        GKL_LAUNCH_CHECK("rmatmat_i8_reduce_kernel");
    }
}

// FP64-exact block products (GKL_PREC_BLOCK_FP64): the single-vector limb
// kernels with two vectors per MFMA tile, one pass over the matrix per pair of
// columns.  Y[:, c] = the sum of the splits' partials in split order, times s_j
// for A^T X (inv_sd non-NULL).
__global__ void __launch_bounds__(256)
limb_pair_reduce_kernel(const double* __restrict__ partial, int nsplit, int nv, int64_t rows_pad,
                        int64_t rows, const double* __restrict__ inv_sd, double* __restrict__ Y,
                        int64_t ldy)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows * nv;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / rows);
        const int64_t row = i - (int64_t)c * rows;
        double t = 0.0;
        for (int sp = 0; sp < nsplit; ++sp) t += partial[((int64_t)sp * nv + c) * rows_pad + row];
        if (inv_sd) t *= inv_sd[row];
        Y[(int64_t)c * ldy + row] = t;
    }
}

static unsigned int pair_reduce_grid(int64_t rows, int nv)
{
    const int64_t g = ceil_div(rows * nv, 256);
    return (unsigned int)(g < 2048 ? g : 2048);
}

static void matmat_exact(const MixedShape& m, const uint8_t* I, const ColStats& st, const double* W,
                         int64_t ldw, int b, double* Y, int64_t ldy, MixedWork& w, hipStream_t s,
                         const hipEvent_t* ev)
{
    const BfSplit& gm = m.limbW;
    i32x4* frag = reinterpret_cast<i32x4*>(w.frag);
    const dim3 grid((unsigned int)(gm.nsplit * gm.nrb));
    for (int c0 = 0; c0 < b; c0 += 2) {
        const int nv = b - c0 < 2 ? b - c0 : 2;
        const double* Wc = W + (int64_t)c0 * ldw;
        hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, nv), dim3(256), 0, s, Wc, ldw, m.p, st.mean,
                           st.inv_sd, 3.0, w.cpart, w.cmax);
        GKL_LAUNCH_CHECK("colsum_kernel");
        if (nv == 2)
            hipLaunchKernelGGL((limb_frag_kernel<2, 2>), dim3((unsigned int)m.nstW), dim3(256), 0, s, Wc,
                               ldw, m.p, st.mean, st.inv_sd, w.cmax, frag);
        else
            hipLaunchKernelGGL((limb_frag_kernel<2, 1>), dim3((unsigned int)m.nstW), dim3(256), 0, s, Wc,
                               ldw, m.p, st.mean, st.inv_sd, w.cmax, frag);
        GKL_LAUNCH_CHECK("limb_frag_kernel");
        if (ev && c0 == 0) GKL_HIP(hipEventRecord(ev[0], s));
        if (nv == 2)
            hipLaunchKernelGGL((limb_product_kernel<true, 2>), grid, dim3(256), 0, s, I, m.ldI, m.nI,
                               m.n, frag, m.nstW, gm.st_per, gm.nsplit, gm.nrb, gm.xcd, w.cpart, w.cmax,
                               st.mean, w.partial);
        else
            hipLaunchKernelGGL((limb_product_kernel<true, 1>), grid, dim3(256), 0, s, I, m.ldI, m.nI,
                               m.n, frag, m.nstW, gm.st_per, gm.nsplit, gm.nrb, gm.xcd, w.cpart, w.cmax,
                               st.mean, w.partial);
        GKL_LAUNCH_CHECK("limb_product_kernel<A W>");
        if (ev && c0 + 2 >= b) GKL_HIP(hipEventRecord(ev[1], s));
        hipLaunchKernelGGL(limb_pair_reduce_kernel, dim3(pair_reduce_grid(m.n, nv)), dim3(256), 0, s,
                           w.partial, gm.nsplit, nv, m.nI, m.n, nullptr, Y + (int64_t)c0 * ldy, ldy);
        GKL_LAUNCH_CHECK("limb_pair_reduce_kernel");
    }
}

static void rmatmat_exact(const MixedShape& m, const uint8_t* S, const ColStats& st, const double* X,
                          int64_t ldx, int b, double* Z, int64_t ldz, MixedWork& w, hipStream_t s,
                          const hipEvent_t* ev)
{
    const BfSplit& gm = m.limbX;
    i32x4* frag = reinterpret_cast<i32x4*>(w.frag);
    const dim3 grid((unsigned int)(gm.nsplit * gm.nrb));
    for (int c0 = 0; c0 < b; c0 += 2) {
        const int nv = b - c0 < 2 ? b - c0 : 2;
        const double* Xc = X + (int64_t)c0 * ldx;
        hipLaunchKernelGGL(colsum_kernel, dim3(kCsSplit, nv), dim3(256), 0, s, Xc, ldx, m.n, nullptr,
                           nullptr, 0.0, w.cpart, w.cmax);
        GKL_LAUNCH_CHECK("colsum_kernel");
        if (nv == 2)
            hipLaunchKernelGGL((limb_frag_kernel<1, 2>), dim3((unsigned int)m.nstX), dim3(256), 0, s, Xc,
                               ldx, m.n, nullptr, nullptr, w.cmax, frag);
        else
            hipLaunchKernelGGL((limb_frag_kernel<1, 1>), dim3((unsigned int)m.nstX), dim3(256), 0, s, Xc,
                               ldx, m.n, nullptr, nullptr, w.cmax, frag);
        GKL_LAUNCH_CHECK("limb_frag_kernel");
        if (ev && c0 == 0) GKL_HIP(hipEventRecord(ev[0], s));
        if (nv == 2)
            hipLaunchKernelGGL((limb_product_kernel<false, 2>), grid, dim3(256), 0, s, S, m.ldS, m.pS,
                               m.p, frag, m.nstX, gm.st_per, gm.nsplit, gm.nrb, gm.xcd, w.cpart, w.cmax,
                               st.mean, w.partial);
        else
            hipLaunchKernelGGL((limb_product_kernel<false, 1>), grid, dim3(256), 0, s, S, m.ldS, m.pS,
                               m.p, frag, m.nstX, gm.st_per, gm.nsplit, gm.nrb, gm.xcd, w.cpart, w.cmax,
                               st.mean, w.partial);
        GKL_LAUNCH_CHECK("limb_product_kernel<A^T X>");
        if (ev && c0 + 2 >= b) GKL_HIP(hipEventRecord(ev[1], s));
        hipLaunchKernelGGL(limb_pair_reduce_kernel, dim3(pair_reduce_grid(m.p, nv)), dim3(256), 0, s,
                           w.partial, gm.nsplit, nv, m.pS, m.p, st.inv_sd, Z + (int64_t)c0 * ldz, ldz);
        GKL_LAUNCH_CHECK("limb_pair_reduce_kernel");
    }
}

void launch_matmat_mixed(const MixedShape& m, const uint8_t* I, const ColStats& st,
                         const double* W, int64_t ldw, int b, double* Y, int64_t ldy,
                         MixedWork& w, hipStream_t s, const hipEvent_t* core_ev)
{
    if (m.exact) matmat_exact(m, I, st, W, ldw, b, Y, ldy, w, s, core_ev);
    else if (m.int8) matmat_i8(m, I, st, W, ldw, b, Y, ldy, w, s, core_ev);
    else matmat_bf16(m, I, st, W, ldw, b, Y, ldy, w, s, core_ev);
}

void launch_rmatmat_mixed(const MixedShape& m, const uint8_t* S, const ColStats& st,
                          const double* X, int64_t ldx, int b, double* Z, int64_t ldz,
                          MixedWork& w, hipStream_t s, const hipEvent_t* core_ev)
{
    if (m.exact) rmatmat_exact(m, S, st, X, ldx, b, Z, ldz, w, s, core_ev);
    else if (m.int8) rmatmat_i8(m, S, st, X, ldx, b, Z, ldz, w, s, core_ev);
    else rmatmat_bf16(m, S, st, X, ldx, b, Z, ldz, w, s, core_ev);
}

}  // namespace gkl
