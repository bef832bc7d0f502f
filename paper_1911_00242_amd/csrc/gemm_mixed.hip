// Split-BF16 grouped complex GEMM for the mixed-precision path (CDNA4 bf16 MFMA).
//
// Same contractions and offset tables as the FP64 kernel; operands are stored as four
// bf16 planes per complex element, plane-major: (re_hi, re_lo, im_hi, im_lo), where
// hi = bf16(x) and lo = bf16(x - hi), both rounded to nearest even, so hi + lo carries
// 16 significant bits (|x - hi - lo| <= 2^-17 |x|).  A real product is taken as
// hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-16 relative, is dropped), accumulated in
// FP32 by v_mfma_f32_32x32x16_bf16; a complex multiply-accumulate is four real products,
// i.e. twelve MFMAs per 32x32x16 complex tile step.  The epilogue adds alpha*acc to the
// FP64 output with FP64 arithmetic.
//
// Tile: 128 x 128 complex outputs per 256-thread workgroup (2 x 2 waves of 64 x 64 =
// 2 x 2 MFMA tiles of 32 x 32), 16 complex k per stage, LDS double buffered with
// register staging.  Global loads move 16 bytes (8 consecutive k of one plane) when the
// k offsets form aligned runs of 8 (FAST), else element by element.
#include "common.h"
#include "mixed.h"

namespace ck {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__host__ __device__ inline uint16_t bf16_rne(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

__device__ inline void split2(double x, uint16_t &hi, uint16_t &lo) {
    hi = bf16_rne((float)x);
    lo = bf16_rne((float)(x - (double)bf16_to_f(hi)));
}

// ------------------------------------------------------------------ conversions
__global__ void k_split(int64_t n, const cd *src, uint16_t *dst, int64_t plane) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        cd x = src[i];
        uint16_t a, b, c, d;
        split2(x.x, a, b);
        split2(x.y, c, d);
        dst[i] = a;
        dst[plane + i] = b;
        dst[2 * plane + i] = c;
        dst[3 * plane + i] = d;
    }
}

// per momentum block (o^2 x v^2) -> split planes of the (v^2 x o^2) transpose
__global__ void k_split_transpose(Dims d, const cd *src, uint16_t *dst, int64_t plane) {
    __shared__ cd tile[32][33];
    const int R = d.no * d.no, C = d.nv * d.nv;
    const int tr = (R + 31) / 32, tc = (C + 31) / 32;
    int64_t blk = blockIdx.x / (tr * tc);
    int t = (int)(blockIdx.x % (tr * tc));
    int r0 = (t / tc) * 32, c0 = (t % tc) * 32;
    const cd *s = src + blk * d.t2blk();
    int64_t ob = blk * d.t2blk();
    int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int y = ty; y < 32; y += 8) {
        int r = r0 + y, c = c0 + tx;
        if (r < R && c < C) tile[y][tx] = s[(int64_t)r * C + c];
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        int c = c0 + y, r = r0 + tx;
        if (r < R && c < C) {
            cd x = tile[tx][y];
            int64_t i = ob + (int64_t)c * R + r;
            uint16_t a, b, e, f;
            split2(x.x, a, b);
            split2(x.y, e, f);
            dst[i] = a;
            dst[plane + i] = b;
            dst[2 * plane + i] = e;
            dst[3 * plane + i] = f;
        }
    }
}

void launch_split(int64_t n, const cd *src, uint16_t *dst, int64_t plane, hipStream_t st) {
    int64_t b = std::min<int64_t>((n + 255) / 256, 1 << 20);
    hipLaunchKernelGGL(k_split, dim3((unsigned)std::max<int64_t>(b, 1)), dim3(256), 0, st, n, src, dst, plane);
    CK_CHECK(hipGetLastError());
}

void launch_split_transpose(const Dims &d, const cd *src, uint16_t *dst, int64_t plane, hipStream_t st) {
    int R = d.no * d.no, C = d.nv * d.nv;
    dim3 g((unsigned)((int64_t)((R + 31) / 32) * ((C + 31) / 32) * d.N * d.N * d.N));
    hipLaunchKernelGGL(k_split_transpose, g, dim3(256), 0, st, d, src, dst, plane);
    CK_CHECK(hipGetLastError());
}

// ------------------------------------------------------------------ the GEMM
// Eight consecutive k of one row of one plane, element by element (zeros out of range).
__device__ inline uint4 gather8(const uint16_t *base, const int64_t *ktab, const uint16_t *zeros, int g, int K,
                                int kb, bool rok, int64_t row, int64_t plane_off) {
    uint32_t v[4];
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        const int k = kb + j;
        const uint16_t *x0 = (rok && k < K) ? base + plane_off + row + ktab[(int64_t)g * K + min(k, K - 1)] : zeros;
        const uint16_t *x1 = (rok && k + 1 < K) ? base + plane_off + row + ktab[(int64_t)g * K + min(k + 1, K - 1)] : zeros;
        v[j / 2] = (uint32_t)*x0 | (uint32_t)*x1 << 16;
    }
    return make_uint4(v[0], v[1], v[2], v[3]);
}

template <bool FAST>
__global__ __launch_bounds__(256) void k_gemm_split(SplitOps op) {
    constexpr int BM = 128, BN = 128, BK = 16, PADK = BK + 8;
    constexpr int PLANE = 128 * PADK;  // bf16 elements per plane in one LDS buffer
    __shared__ __attribute__((aligned(16))) uint16_t As[2][4 * PLANE];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][4 * PLANE];

    const int tid = threadIdx.x;
    const int g = blockIdx.z;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int M = op.M, N = op.N, K = op.K;
    // loader: thread -> (row = tid/2, chunk of 8 k = tid%2), all four planes.  Loads are
    // branch free from clamped, always valid addresses; out-of-range rows and k are
    // zeroed when the staged registers are written to LDS, so the compiler can keep the
    // loads in flight across the MFMA work of the current stage.
    const int lrow = tid >> 1, lkc = tid & 1;
    const int am = m0 + lrow, bn = n0 + lrow;
    const bool aok = am < M, bok = bn < N;
    const int64_t arow = op.a_row[(int64_t)g * M + (aok ? am : M - 1)];
    const int64_t bcol = op.b_col[(int64_t)g * N + (bok ? bn : N - 1)];

    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int l32 = lane & 31, lh = lane >> 5;

    f32x16 accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                accr[i][j][r] = 0.f;
                acci[i][j][r] = 0.f;
            }

    // Staged chunk of the next stage (registers), and the k-table offsets of the stage
    // after it.  Every iteration loads (out-of-range chunks read the zero buffer), so no
    // data-dependent select sits between a load and its LDS store.
    uint4 sa0, sa1, sa2, sa3, sb0, sb1, sb2, sb3;
    int64_t ak_cur = 0, bk_cur = 0;
    // FAST implies K % 8 == 0 and K >= 8: clamp to the last whole 8-run so a 16-byte load
    // never leaves the operand; otherwise clamp to the last k
    const int kclamp = FAST ? K - 8 : K - 1;
#define CK_KOFS(k0, ak, bk)                                          \
    {                                                                \
        const int kb_ = min((k0) + lkc * 8, kclamp);                 \
        ak = op.a_k[(int64_t)g * K + kb_];                           \
        bk = op.b_k[(int64_t)g * K + kb_];                           \
    }
#define CK_LOAD(k0)                                                                                   \
    {                                                                                                 \
        const int kb_ = (k0) + lkc * 8;                                                               \
        if (FAST) {                                                                                   \
            const uint16_t *pa_ = (kb_ < K && aok) ? op.A + arow + ak_cur : op.zeros;                 \
            const uint16_t *pb_ = (kb_ < K && bok) ? op.B + bcol + bk_cur : op.zeros;                 \
            const int64_t sa_ = (kb_ < K && aok) ? op.a_plane : 0, sb_ = (kb_ < K && bok) ? op.b_plane : 0; \
            sa0 = *(const uint4 *)(pa_);                                                              \
            sa1 = *(const uint4 *)(pa_ + sa_);                                                        \
            sa2 = *(const uint4 *)(pa_ + 2 * sa_);                                                    \
            sa3 = *(const uint4 *)(pa_ + 3 * sa_);                                                    \
            sb0 = *(const uint4 *)(pb_);                                                              \
            sb1 = *(const uint4 *)(pb_ + sb_);                                                        \
            sb2 = *(const uint4 *)(pb_ + 2 * sb_);                                                    \
            sb3 = *(const uint4 *)(pb_ + 3 * sb_);                                                    \
        } else {                                                                                      \
            sa0 = gather8(op.A, op.a_k, op.zeros, g, K, kb_, aok, arow, 0);                            \
            sa1 = gather8(op.A, op.a_k, op.zeros, g, K, kb_, aok, arow, op.a_plane);                   \
            sa2 = gather8(op.A, op.a_k, op.zeros, g, K, kb_, aok, arow, 2 * op.a_plane);               \
            sa3 = gather8(op.A, op.a_k, op.zeros, g, K, kb_, aok, arow, 3 * op.a_plane);               \
            sb0 = gather8(op.B, op.b_k, op.zeros, g, K, kb_, bok, bcol, 0);                            \
            sb1 = gather8(op.B, op.b_k, op.zeros, g, K, kb_, bok, bcol, op.b_plane);                   \
            sb2 = gather8(op.B, op.b_k, op.zeros, g, K, kb_, bok, bcol, 2 * op.b_plane);               \
            sb3 = gather8(op.B, op.b_k, op.zeros, g, K, kb_, bok, bcol, 3 * op.b_plane);               \
        }                                                                                             \
    }
#define CK_STORE(buf)                                                     \
    {                                                                     \
        uint16_t *a_ = &As[buf][lrow * PADK + lkc * 8];                   \
        uint16_t *b_ = &Bs[buf][lrow * PADK + lkc * 8];                   \
        *(uint4 *)(a_) = sa0;                                             \
        *(uint4 *)(a_ + PLANE) = sa1;                                     \
        *(uint4 *)(a_ + 2 * PLANE) = sa2;                                 \
        *(uint4 *)(a_ + 3 * PLANE) = sa3;                                 \
        *(uint4 *)(b_) = sb0;                                             \
        *(uint4 *)(b_ + PLANE) = sb1;                                     \
        *(uint4 *)(b_ + 2 * PLANE) = sb2;                                 \
        *(uint4 *)(b_ + 3 * PLANE) = sb3;                                 \
    }

    const int nk = (K + BK - 1) / BK;
    if (K > 0) {
        CK_KOFS(0, ak_cur, bk_cur);
        CK_LOAD(0);
        CK_STORE(0);
        CK_KOFS(BK, ak_cur, bk_cur);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        int64_t ak_nxt, bk_nxt;
        // next stage's data (zeros past the end) and the k offsets of the one after it,
        // issued ahead of the MFMA work they overlap with
        CK_LOAD((kt + 1) * BK);
        CK_KOFS((kt + 2) * BK, ak_nxt, bk_nxt);
        __builtin_amdgcn_sched_barrier(0);
        // fragments: lane holds 8 consecutive k of row (lane % 32), k offset 8 * (lane / 32)
        bf16x8 a[2][4], b[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                a[i][p] = *(const bf16x8 *)(&As[buf][p * PLANE + (wm * 64 + i * 32 + l32) * PADK + lh * 8]);
                b[i][p] = *(const bf16x8 *)(&Bs[buf][p * PLANE + (wn * 64 + i * 32 + l32) * PADK + lh * 8]);
            }
        // -A_im for the real part
        bf16x8 na[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                uint4 u = __builtin_bit_cast(uint4, a[i][2 + p]);
                u.x ^= 0x80008000u;
                u.y ^= 0x80008000u;
                u.z ^= 0x80008000u;
                u.w ^= 0x80008000u;
                na[i][p] = __builtin_bit_cast(bf16x8, u);
            }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                f32x16 cr = accr[i][j], ci = acci[i][j];
                // re += Ar*Br - Ai*Bi
                cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][0], cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][1], cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], b[j][0], cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na[i][0], b[j][2], cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na[i][0], b[j][3], cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na[i][1], b[j][2], cr, 0, 0, 0);
                // im += Ar*Bi + Ai*Br
                ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][2], ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][3], ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], b[j][2], ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][2], b[j][0], ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][2], b[j][1], ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][3], b[j][0], ci, 0, 0, 0);
                accr[i][j] = cr;
                acci[i][j] = ci;
            }
        __builtin_amdgcn_sched_barrier(0);
        CK_STORE(buf ^ 1);  // buf ^ 1 was last read before the previous barrier
        ak_cur = ak_nxt;
        bk_cur = bk_nxt;
        __syncthreads();
    }
#undef CK_KOFS
#undef CK_LOAD
#undef CK_STORE

    // epilogue: 32x32 f32 output, register r of a lane holds row 8*(r/4) + 4*(lane/32) + r%4
    // of column lane%32
    const double alpha = op.alpha, beta = op.beta;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn * 64 + j * 32 + l32;
            if (n >= N) continue;
            const int64_t ccol = op.c_col[(int64_t)g * N + n];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
                if (m >= M) continue;
                cd *p = op.C + op.c_row[(int64_t)g * M + m] + ccol;
                cd v = make_double2(alpha * (double)accr[i][j][r], alpha * (double)acci[i][j][r]);
                if (beta != 0.0) {
                    cd o = *p;
                    v.x = fma(beta, o.x, v.x);
                    v.y = fma(beta, o.y, v.y);
                }
                *p = v;
            }
        }
}

void gemm_split(const SplitOps &op, hipStream_t s) {
    if (op.G <= 0 || op.M <= 0 || op.N <= 0) return;
    dim3 grid((op.N + 127) / 128, (op.M + 127) / 128, op.G);
    if (op.fast)
        hipLaunchKernelGGL(k_gemm_split<true>, grid, dim3(256), 0, s, op);
    else
        hipLaunchKernelGGL(k_gemm_split<false>, grid, dim3(256), 0, s, op);
    CK_CHECK(hipGetLastError());
}

}  // namespace ck
