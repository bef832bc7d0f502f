// Split-BF16 grouped complex GEMM for the mixed-precision path (CDNA4 bf16 MFMA).
//
// Same contractions and offset tables as the FP64 kernel; operands are stored split
// (mixed.h): four bf16 values per complex element (re_hi, re_lo, im_hi, im_lo), where
// hi = bf16(x) and lo = bf16(x - hi), both rounded to nearest even, so hi + lo carries
// 16 significant bits (|x - hi - lo| <= 2^-17 |x|).  A real product is taken as
// hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-16 relative, is dropped), accumulated in
// FP32 by v_mfma_f32_32x32x16_bf16; a complex multiply-accumulate is four real products,
// i.e. twelve MFMAs per 32x32x16 complex tile step.  The epilogue adds alpha*acc to the
// FP64 output with FP64 arithmetic.
//
// Tile: 128 x 128 complex outputs per 256-thread workgroup (2 x 2 waves of 64 x 64 =
// 2 x 2 MFMA tiles of 32 x 32), 16 complex k per stage, LDS double buffered; global loads
// run two stages ahead through two sets of staging registers, and LDS traffic is
// interleaved with the MFMAs (see k_gemm_split).  In the fast case (aligned runs of 8 k)
// eight lanes copy one row's stage, 128 contiguous bytes of split storage, so every load
// instruction reads whole cache lines; otherwise elements are gathered one by one.
#include "common.h"
#include "mixed.h"

namespace ck {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
// 16-byte staging chunk as a native vector (a copy of HIP's uint4 struct becomes a memcpy
// that keeps a register array in memory)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ conversions
// A workgroup converts 256 chunks (2048 elements) at a time: coalesced loads of
// consecutive elements, the bf16 halves staged per plane in LDS, then one 64-byte chunk
// store per thread.
__global__ __launch_bounds__(256) void k_split(int64_t n, const cd *src, uint16_t *dst) {
    __shared__ __attribute__((aligned(16))) uint16_t S[4][2048];
    const int t = threadIdx.x;
    const int64_t nch = (n + 7) / 8;
    for (int64_t c0 = (int64_t)blockIdx.x * 256; c0 < nch; c0 += (int64_t)gridDim.x * 256) {
        const int64_t e0 = c0 * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t e = e0 + t + 256 * j;
            const cd x = e < n ? src[e] : make_double2(0.0, 0.0);
            uint16_t h0, h1, h2, h3;
            split2c(x, h0, h1, h2, h3);
            S[0][t + 256 * j] = h0;
            S[1][t + 256 * j] = h1;
            S[2][t + 256 * j] = h2;
            S[3][t + 256 * j] = h3;
        }
        __syncthreads();
        if (c0 + t < nch) {
            uint4 *o = (uint4 *)(dst + (c0 + t) * 32);
#pragma unroll
            for (int p = 0; p < 4; ++p) o[p] = *(const uint4 *)&S[p][8 * t];
        }
        __syncthreads();
    }
}

void launch_split(int64_t n, const cd *src, uint16_t *dst, hipStream_t st) {
    int64_t b = std::min<int64_t>(((n + 7) / 8 + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(k_split, dim3((unsigned)std::max<int64_t>(b, 1)), dim3(256), 0, st, n, src, dst);
    CK_CHECK(hipGetLastError());
}

// ------------------------------------------------------------------ the GEMM
// Eight consecutive k of one row of one plane, element by element (zeros out of range).
__device__ inline u32x4 gather8(const uint16_t *base, const int64_t *ktab, const uint16_t *zeros, int g, int K,
                                int64_t kld, int kb, bool rok, int64_t row, int p) {
    uint32_t v[4];
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        const int k = kb + j;
        const uint16_t *x0 =
            (rok && k < K) ? base + split_index(row + ktab[(int64_t)g * kld + min(k, K - 1)], p) : zeros;
        const uint16_t *x1 =
            (rok && k + 1 < K) ? base + split_index(row + ktab[(int64_t)g * kld + min(k + 1, K - 1)], p) : zeros;
        v[j / 2] = (uint32_t)*x0 | (uint32_t)*x1 << 16;
    }
    return u32x4{v[0], v[1], v[2], v[3]};
}

// One of the twelve MFMAs of a 32 x 32 complex tile step: A, B are the four planes
// (re_hi, re_lo, im_hi, im_lo) of the lane's fragments, NA = (-im_hi, -im_lo) of A.
// The real and imaginary chains alternate so that consecutive MFMAs are independent.
template <int k>
__device__ __forceinline__ void mfma_step(f32x16 &cr, f32x16 &ci, bf16x8 a0, bf16x8 a1, bf16x8 a2, bf16x8 a3,
                                          bf16x8 na0, bf16x8 na1, bf16x8 b0, bf16x8 b1, bf16x8 b2, bf16x8 b3) {
    // re += Ar*Br - Ai*Bi ; im += Ar*Bi + Ai*Br, each real product as hi*hi + hi*lo + lo*hi
    if constexpr (k == 0) cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, cr, 0, 0, 0);
    if constexpr (k == 1) ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b2, ci, 0, 0, 0);
    if constexpr (k == 2) cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, cr, 0, 0, 0);
    if constexpr (k == 3) ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b3, ci, 0, 0, 0);
    if constexpr (k == 4) cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, cr, 0, 0, 0);
    if constexpr (k == 5) ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b2, ci, 0, 0, 0);
    if constexpr (k == 6) cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na0, b2, cr, 0, 0, 0);
    if constexpr (k == 7) ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b0, ci, 0, 0, 0);
    if constexpr (k == 8) cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na0, b3, cr, 0, 0, 0);
    if constexpr (k == 9) ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b1, ci, 0, 0, 0);
    if constexpr (k == 10) cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na1, b2, cr, 0, 0, 0);
    if constexpr (k == 11) ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3, b0, ci, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 negate_bf16x8(bf16x8 a) {
    uint4 u = __builtin_bit_cast(uint4, a);
    u.x ^= 0x80008000u;
    u.y ^= 0x80008000u;
    u.z ^= 0x80008000u;
    u.w ^= 0x80008000u;
    return __builtin_bit_cast(bf16x8, u);
}

// Tile: 128 x 128 complex outputs per 256-thread workgroup; wave (wm, wn) owns the 64 x 64
// quadrant, i.e. 2 x 2 MFMA tiles (i, j) of 32 x 32, with fragments a_i (its rows) and b_j
// (its columns).  One k stage of 16 complex values is software pipelined so that the
// MFMA pipe of each wave never waits on memory; all four fragments of a stage are in
// registers when it starts (read during the previous stage), and its 48 MFMAs run
// round robin over the four tiles, so eight accumulator chains are in flight:
//   first half: the global loads of stage k+2 into one set of staging registers, then
//               the LDS writes of stage k+1 (loaded one stage ago, other set) into the
//               other LDS buffer;
//   barrier;
//   second half: the LDS reads of all fragments of stage k+1 into the other register set.
// Every slot is one MFMA plus at most one memory operation, fenced by sched_barrier so
// the compiler keeps this order.  The negated imaginary planes of A, first needed by the
// MFMAs of step 6, are formed in two slots of step 2, so the stage does not open with a
// wait on the LDS reads of the last fragment planes (about 2% faster on the ring family).  One barrier per stage suffices: the buffer written in
// the first half of stage k was last read in the second half of stage k-2, before the
// barrier of stage k-1, and it is read in the second half of stage k, after the barrier
// of stage k.
template <bool FAST>
__global__ __launch_bounds__(256) void k_gemm_split(SplitOps op) {
    constexpr int BM = 128, BN = 128, BK = 16;
    // LDS row: one row's stage as in split storage (two chunks of 8 k, four planes each,
    // 128 bytes) plus 16 bytes of pad, so that 16 lanes reading 16 consecutive rows hit
    // distinct banks
    constexpr int RS = 72;  // bf16 per LDS row
    __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * RS];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * RS];

    const int tid = threadIdx.x;
    const int M = op.M, N = op.N, K = op.K;
    const int64_t kld = op.kld ? op.kld : K;
    const GemmTile tile = gemm_tile((M + BM - 1) / BM, (N + BN - 1) / BN, op.G, 8);
    if (!tile.valid) return;
    const int g = tile.g;
    const int m0 = tile.mt * BM, n0 = tile.nt * BN;

    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int l32 = lane & 31, lh = lane >> 5;
    // loader: lane -> 16-byte piece lq = lane % 8 of one row's stage (chunk lc = lq / 4,
    // plane lp = lq % 4), rows lr + 8i (i = 0..3) of both A and B, so eight lanes copy one
    // row's 128 bytes.  Loads are branch free from clamped, always valid addresses
    // (out-of-range rows and k read the zero buffer), so no data-dependent select sits
    // between a load and its LDS store.
    const int lq = lane & 7, lc = lq >> 2, lp = lq & 3;
    const int lr = wave * 32 + (lane >> 3);
    const int64_t *a_rows = op.a_row + (int64_t)g * M, *b_cols = op.b_col + (int64_t)g * N;
#define CK_ROW(i)                                                                    \
    const int am##i = m0 + lr + 8 * (i), bn##i = n0 + lr + 8 * (i);                  \
    const bool aok##i = am##i < M, bok##i = bn##i < N;                               \
    const int64_t arow##i = a_rows[aok##i ? am##i : M - 1], bcol##i = b_cols[bok##i ? bn##i : N - 1]; \
    /* fast case: offsets are multiples of 8, so split_index(e, lp) = 4 e + 8 lp */            \
    const uint16_t *abase##i = op.A + arow##i * 4 + lp * 8, *bbase##i = op.B + bcol##i * 4 + lp * 8;
    CK_ROW(0)
    CK_ROW(1)
    CK_ROW(2)
    CK_ROW(3)
#undef CK_ROW
    // LDS element offsets of this lane's fragment rows (8 consecutive k of row lane % 32,
    // chunk lane / 32) and of this thread's first staging piece
    const int fa0 = (wm * 64 + l32) * RS + lh * 32, fa1 = fa0 + 32 * RS;
    const int fb0 = (wn * 64 + l32) * RS + lh * 32, fb1 = fb0 + 32 * RS;
    const int sto = lr * RS + lq * 8;

    f32x16 c00r, c00i, c01r, c01i, c10r, c10i, c11r, c11i;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        c00r[r] = c00i[r] = c01r[r] = c01i[r] = 0.f;
        c10r[r] = c10i[r] = c11r[r] = c11i[r] = 0.f;
    }
    bf16x8 FA[2][2][4], FB[2][2][4];  // [set][fragment row i / column j][plane]: current, next stage
    bf16x8 NA[2][2];                   // -A_im of the current set, per fragment row
    u32x4 sa[3][4], sb[3][4];   // staging sets: this thread's pieces of A and B of one stage
    int64_t ak_cur = 0, bk_cur = 0, ak_nxt = 0, bk_nxt = 0;
    // FAST implies K % 8 == 0 and K >= 8: clamp to the last whole 8-run so a 16-byte load
    // never leaves the operand; otherwise clamp to the last k
    const int kclamp = FAST ? K - 8 : K - 1;

#define CK_SLOT __builtin_amdgcn_sched_barrier(0)
#define CK_MF(k, CR, CI, A, NA, B) \
    mfma_step<k>(CR, CI, A[0], A[1], A[2], A[3], NA[0], NA[1], B[0], B[1], B[2], B[3])
#define CK_NEG(A, NA)                   \
    {                                   \
        NA[0] = negate_bf16x8(A[2]);    \
        NA[1] = negate_bf16x8(A[3]);    \
    }
#define CK_KOFS(k0, ak, bk)                                          \
    {                                                                \
        const int kb_ = min((k0) + lc * 8, kclamp);                  \
        ak = op.a_k[(int64_t)g * kld + kb_];                         \
        bk = op.b_k[(int64_t)g * kld + kb_];                         \
    }
    // row lr + 8i of A or B, stage k0, into staging set S.  Separate names for the A and
    // B sets (no pointer select between them) keep the staging arrays in registers.
#define CK_LOADA(k0, S, i)                                                                              \
    {                                                                                                  \
        const int kb_ = (k0) + lc * 8;                                                                 \
        if (FAST) {                                                                                    \
            const bool ok_ = kb_ < K && aok##i;                                                        \
            const uint16_t *src_ = ok_ ? abase##i + ak_cur * 4 : op.zeros;                              \
            sa[S][i] = *(const u32x4 *)src_;                                                           \
        } else {                                                                                       \
            sa[S][i] = gather8(op.A, op.a_k, op.zeros, g, K, kld, kb_, aok##i, arow##i, lp);                \
        }                                                                                              \
    }
#define CK_LOADB(k0, S, i)                                                                              \
    {                                                                                                  \
        const int kb_ = (k0) + lc * 8;                                                                 \
        if (FAST) {                                                                                    \
            const bool ok_ = kb_ < K && bok##i;                                                        \
            const uint16_t *src_ = ok_ ? bbase##i + bk_cur * 4 : op.zeros;                              \
            sb[S][i] = *(const u32x4 *)src_;                                                           \
        } else {                                                                                       \
            sb[S][i] = gather8(op.B, op.b_k, op.zeros, g, K, kld, kb_, bok##i, bcol##i, lp);                \
        }                                                                                              \
    }
#define CK_STOREA(buf, S, i) *(u32x4 *)(&As[buf][sto + (i) * 8 * RS]) = sa[S][i]
#define CK_STOREB(buf, S, i) *(u32x4 *)(&Bs[buf][sto + (i) * 8 * RS]) = sb[S][i]
#define CK_RDA(dst, buf, off, p) dst = *(const bf16x8 *)(&As[buf][(off) + (p) * 8])
#define CK_RDB(dst, buf, off, p) dst = *(const bf16x8 *)(&Bs[buf][(off) + (p) * 8])

    // one pipelined stage KT held in LDS buffer BUF (literal 0 or 1), its fragments in
    // register set BUF; staging set BUF receives stage KT+2, set BUF^1 holds stage KT+1
#define CK_STAGE(KT, BUF, LS, SS)                                                                                             \
    {                                                                                                                 \
        CK_MF(0, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_KOFS(((KT) + 4) * BK, ak_nxt, bk_nxt); CK_SLOT;       \
        CK_MF(0, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_LOADA(((KT) + 3) * BK, LS, 0); CK_SLOT;              \
        CK_MF(0, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_LOADA(((KT) + 3) * BK, LS, 1); CK_SLOT;              \
        CK_MF(0, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_LOADA(((KT) + 3) * BK, LS, 2); CK_SLOT;              \
        CK_MF(1, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_LOADA(((KT) + 3) * BK, LS, 3); CK_SLOT;              \
        CK_MF(1, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_LOADB(((KT) + 3) * BK, LS, 0); CK_SLOT;              \
        CK_MF(1, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_LOADB(((KT) + 3) * BK, LS, 1); CK_SLOT;              \
        CK_MF(1, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_LOADB(((KT) + 3) * BK, LS, 2); CK_SLOT;              \
        CK_MF(2, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_LOADB(((KT) + 3) * BK, LS, 3); CK_SLOT;              \
        CK_MF(2, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_NEG(FA[BUF][0], NA[0]); CK_SLOT;                                                 \
        CK_MF(2, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_NEG(FA[BUF][1], NA[1]); CK_SLOT;                                                 \
        CK_MF(2, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_SLOT;                                                 \
        CK_MF(3, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_SLOT;                                                 \
        CK_MF(3, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_SLOT;                                                 \
        CK_MF(3, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_SLOT;                                                 \
        CK_MF(3, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_STOREA((BUF) ^ 1, SS, 0); CK_SLOT;             \
        CK_MF(4, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_STOREA((BUF) ^ 1, SS, 1); CK_SLOT;             \
        CK_MF(4, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_STOREA((BUF) ^ 1, SS, 2); CK_SLOT;             \
        CK_MF(4, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_STOREA((BUF) ^ 1, SS, 3); CK_SLOT;             \
        CK_MF(4, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_STOREB((BUF) ^ 1, SS, 0); CK_SLOT;             \
        CK_MF(5, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_STOREB((BUF) ^ 1, SS, 1); CK_SLOT;             \
        CK_MF(5, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_STOREB((BUF) ^ 1, SS, 2); CK_SLOT;             \
        CK_MF(5, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_STOREB((BUF) ^ 1, SS, 3); CK_SLOT;             \
        CK_MF(5, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_SLOT;                                                 \
        __syncthreads();                                                                                              \
        CK_SLOT;                                                                                                      \
        CK_MF(6, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_RDA(FA[(BUF) ^ 1][0][0], (BUF) ^ 1, fa0, 0); CK_SLOT; \
        CK_MF(6, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_RDB(FB[(BUF) ^ 1][0][0], (BUF) ^ 1, fb0, 0); CK_SLOT; \
        CK_MF(6, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_RDA(FA[(BUF) ^ 1][1][0], (BUF) ^ 1, fa1, 0); CK_SLOT; \
        CK_MF(6, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_RDB(FB[(BUF) ^ 1][1][0], (BUF) ^ 1, fb1, 0); CK_SLOT; \
        CK_MF(7, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_RDA(FA[(BUF) ^ 1][0][1], (BUF) ^ 1, fa0, 1); CK_SLOT; \
        CK_MF(7, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_RDB(FB[(BUF) ^ 1][0][1], (BUF) ^ 1, fb0, 1); CK_SLOT; \
        CK_MF(7, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_RDA(FA[(BUF) ^ 1][1][1], (BUF) ^ 1, fa1, 1); CK_SLOT; \
        CK_MF(7, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_RDB(FB[(BUF) ^ 1][1][1], (BUF) ^ 1, fb1, 1); CK_SLOT; \
        CK_MF(8, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_RDA(FA[(BUF) ^ 1][0][2], (BUF) ^ 1, fa0, 2); CK_SLOT; \
        CK_MF(8, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_RDB(FB[(BUF) ^ 1][0][2], (BUF) ^ 1, fb0, 2); CK_SLOT; \
        CK_MF(8, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_RDA(FA[(BUF) ^ 1][1][2], (BUF) ^ 1, fa1, 2); CK_SLOT; \
        CK_MF(8, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_RDB(FB[(BUF) ^ 1][1][2], (BUF) ^ 1, fb1, 2); CK_SLOT; \
        CK_MF(9, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_RDA(FA[(BUF) ^ 1][0][3], (BUF) ^ 1, fa0, 3); CK_SLOT; \
        CK_MF(9, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_RDB(FB[(BUF) ^ 1][0][3], (BUF) ^ 1, fb0, 3); CK_SLOT; \
        CK_MF(9, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_RDA(FA[(BUF) ^ 1][1][3], (BUF) ^ 1, fa1, 3); CK_SLOT; \
        CK_MF(9, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_RDB(FB[(BUF) ^ 1][1][3], (BUF) ^ 1, fb1, 3); CK_SLOT; \
        CK_MF(10, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_SLOT;                                                \
        CK_MF(10, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_SLOT;                                                \
        CK_MF(10, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_SLOT;                                                \
        CK_MF(10, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_SLOT;                                                \
        CK_MF(11, c00r, c00i, FA[BUF][0], NA[0], FB[BUF][0]); CK_SLOT;                                                \
        CK_MF(11, c01r, c01i, FA[BUF][0], NA[0], FB[BUF][1]); CK_SLOT;                                                \
        CK_MF(11, c10r, c10i, FA[BUF][1], NA[1], FB[BUF][0]); CK_SLOT;                                                \
        CK_MF(11, c11r, c11i, FA[BUF][1], NA[1], FB[BUF][1]); CK_SLOT;                                                \
        ak_cur = ak_nxt;                                                                                              \
        bk_cur = bk_nxt;                                                                                              \
    }

    const int nk = (K + BK - 1) / BK;
    if (nk > 0) {
        // prologue: stage 0 into LDS buffer 0 and its a_0, b_0 into registers; stage 1 into
        // staging set 1; k offsets of stage 2 ready
        CK_KOFS(0, ak_cur, bk_cur);
        CK_LOADA(0, 0, 0); CK_LOADA(0, 0, 1); CK_LOADA(0, 0, 2); CK_LOADA(0, 0, 3);
        CK_LOADB(0, 0, 0); CK_LOADB(0, 0, 1); CK_LOADB(0, 0, 2); CK_LOADB(0, 0, 3);
        CK_STOREA(0, 0, 0); CK_STOREA(0, 0, 1); CK_STOREA(0, 0, 2); CK_STOREA(0, 0, 3);
        CK_STOREB(0, 0, 0); CK_STOREB(0, 0, 1); CK_STOREB(0, 0, 2); CK_STOREB(0, 0, 3);
        CK_KOFS(BK, ak_cur, bk_cur);
        CK_LOADA(BK, 1, 0); CK_LOADA(BK, 1, 1); CK_LOADA(BK, 1, 2); CK_LOADA(BK, 1, 3);
        CK_LOADB(BK, 1, 0); CK_LOADB(BK, 1, 1); CK_LOADB(BK, 1, 2); CK_LOADB(BK, 1, 3);
        CK_KOFS(2 * BK, ak_cur, bk_cur);
        CK_LOADA(2 * BK, 2, 0); CK_LOADA(2 * BK, 2, 1); CK_LOADA(2 * BK, 2, 2); CK_LOADA(2 * BK, 2, 3);
        CK_LOADB(2 * BK, 2, 0); CK_LOADB(2 * BK, 2, 1); CK_LOADB(2 * BK, 2, 2); CK_LOADB(2 * BK, 2, 3);
        CK_KOFS(3 * BK, ak_cur, bk_cur);
        __syncthreads();
        // (constant indices only: a loop index here would let the compiler move the
        // register arrays to LDS)
        CK_RDA(FA[0][0][0], 0, fa0, 0); CK_RDA(FA[0][0][1], 0, fa0, 1); CK_RDA(FA[0][0][2], 0, fa0, 2); CK_RDA(FA[0][0][3], 0, fa0, 3);
        CK_RDA(FA[0][1][0], 0, fa1, 0); CK_RDA(FA[0][1][1], 0, fa1, 1); CK_RDA(FA[0][1][2], 0, fa1, 2); CK_RDA(FA[0][1][3], 0, fa1, 3);
        CK_RDB(FB[0][0][0], 0, fb0, 0); CK_RDB(FB[0][0][1], 0, fb0, 1); CK_RDB(FB[0][0][2], 0, fb0, 2); CK_RDB(FB[0][0][3], 0, fb0, 3);
        CK_RDB(FB[0][1][0], 0, fb1, 0); CK_RDB(FB[0][1][1], 0, fb1, 1); CK_RDB(FB[0][1][2], 0, fb1, 2); CK_RDB(FB[0][1][3], 0, fb1, 3);
        // unrolled by six (two LDS buffers and fragment sets, three staging sets) so that
        // every register set has a fixed role in each stage; one exit, so the accumulators
        // keep their registers across the stages.  Stage t: LDS buffer t % 2, loads into
        // staging set t % 3, LDS writes from set (t + 1) % 3.
        int kt = 0;
        for (; kt + 5 < nk; kt += 6) {
            CK_STAGE(kt, 0, 0, 1);
            CK_STAGE(kt + 1, 1, 1, 2);
            CK_STAGE(kt + 2, 0, 2, 0);
            CK_STAGE(kt + 3, 1, 0, 1);
            CK_STAGE(kt + 4, 0, 1, 2);
            CK_STAGE(kt + 5, 1, 2, 0);
        }
        if (kt < nk) CK_STAGE(kt, 0, 0, 1);
        if (kt + 1 < nk) CK_STAGE(kt + 1, 1, 1, 2);
        if (kt + 2 < nk) CK_STAGE(kt + 2, 0, 2, 0);
        if (kt + 3 < nk) CK_STAGE(kt + 3, 1, 0, 1);
        if (kt + 4 < nk) CK_STAGE(kt + 4, 0, 1, 2);
    }
#undef CK_SLOT
#undef CK_MF
#undef CK_NEG
#undef CK_KOFS
#undef CK_LOADA
#undef CK_LOADB
#undef CK_STOREA
#undef CK_STOREB
#undef CK_RDA
#undef CK_RDB
#undef CK_STAGE

    f32x16 accr[2][2] = {{c00r, c01r}, {c10r, c11r}};
    f32x16 acci[2][2] = {{c00i, c01i}, {c10i, c11i}};

    // epilogue: 32x32 f32 output, register r of a lane holds row 8*(r/4) + 4*(lane/32) + r%4
    // of column lane%32.  Per fragment row i the row offsets, and (beta != 0) the old values
    // of both fragment columns, are all loaded before the first store: a store to C could
    // alias a later load as far as the compiler knows, so interleaved load / store pairs
    // would each wait a full memory latency.
    const double alpha = op.alpha, beta = op.beta;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int mb = m0 + wm * 64 + i * 32 + 4 * lh;
        int64_t crow[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = mb + 8 * (r >> 2) + (r & 3);
            crow[r] = m < M ? op.c_row[(int64_t)g * M + m] : -1;
        }
        int64_t ccol[2], cscol[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn * 64 + j * 32 + l32;
            ccol[j] = n < N ? op.c_col[(int64_t)g * N + n] : -1;  // < 0: padding column
            cscol[j] = (n < N && op.cs_col) ? op.cs_col[(int64_t)g * N + n] : ccol[j];
        }
        cd o[2][16];
        if (beta != 0.0) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    o[j][r] = crow[r] >= 0 && ccol[j] >= 0 ? op.C[crow[r] + ccol[j]] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (ccol[j] < 0) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if (crow[r] < 0) continue;
                cd v = make_double2(alpha * (double)accr[i][j][r], alpha * (double)acci[i][j][r]);
                if (beta != 0.0) {
                    v.x = fma(beta, o[j][r].x, v.x);
                    v.y = fma(beta, o[j][r].y, v.y);
                }
                if (op.Cs) {
                    const int m = mb + 8 * (r >> 2) + (r & 3);
                    const int64_t e = (op.cs_row ? op.cs_row[(int64_t)g * M + m] : crow[r]) + cscol[j];
                    uint16_t h0, h1, h2, h3;
                    split2c(v, h0, h1, h2, h3);
                    op.Cs[split_index(e, 0)] = h0;
                    op.Cs[split_index(e, 1)] = h1;
                    op.Cs[split_index(e, 2)] = h2;
                    op.Cs[split_index(e, 3)] = h3;
                } else {
                    op.C[crow[r] + ccol[j]] = v;
                }
            }
        }
    }
}

void gemm_split(const SplitOps &op, hipStream_t s) {
    if (op.G <= 0 || op.M <= 0 || op.N <= 0) return;
    const dim3 grid = gemm_tile_grid((op.M + 127) / 128, (op.N + 127) / 128, op.G);
    if (op.fast)
        hipLaunchKernelGGL(k_gemm_split<true>, grid, dim3(256), 0, s, op);
    else
        hipLaunchKernelGGL(k_gemm_split<false>, grid, dim3(256), 0, s, op);
    CK_CHECK(hipGetLastError());
}

}  // namespace ck
