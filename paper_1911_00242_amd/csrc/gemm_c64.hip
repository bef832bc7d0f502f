// Grouped complex GEMM on complex64 operands (the "c64" storage of the mixed-precision
// path), in three arithmetic forms chosen per product:
//
//   SPLIT2  each fp32 operand value x becomes two bf16 terms in registers, h = bf16(x),
//           l = bf16(x - h); a real product is h*h + h*l + l*h (three MFMAs), the same
//           arithmetic as the pre-split kernel (gemm_mixed.hip) on unsplit storage;
//   SPLIT3  three bf16 terms h = bf16(x), m = bf16(x - h), l = bf16(x - h - m); a real
//           product is h*h + h*m + m*h + h*l + m*m + l*h (six MFMAs, every term down to
//           ~2^-16 of |x||y|; the dropped ones are ~2^-24), i.e. about FP32 accuracy;
//   FP32    v_mfma_f32_32x32x2_f32 on the fp32 values themselves.
// All three accumulate in FP32 (v_mfma_f32_32x32x16_bf16 for the split forms), and add
// alpha * acc to the FP64 output with FP64 arithmetic (or write the result back in
// complex64 storage for products whose output is another product's operand).
//
// Same grouped form and offset tables as the other GEMMs (element offsets in complex
// units).  Tile: 128 x 128 complex outputs per 256-thread workgroup, 2 x 2 waves of
// 64 x 64 (2 x 2 MFMA tiles of 32 x 32 each), 16 complex k per LDS stage, double
// buffered; the global loads of stage k+1 are issued before the MFMAs of stage k.  In the
// fast case (aligned runs of 8 k, as for the pre-split kernel) eight lanes copy a row's
// stage, 128 contiguous bytes of complex64.
#include "common.h"
#include "mixed.h"
#include "gemm_tiles.h"

namespace ck {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16;
constexpr int RSF = 2 * BK + 4;  // floats per LDS row: 16 complex + 16 bytes of pad

// Split 8 fp32 values into NP bf16 terms (term t in part[t]), each rounded to nearest even
// from the remainder of the previous terms, with the packed hardware conversion.
template <int NP>
__device__ __forceinline__ void split_terms(const float (&x)[8], bf16x8 (&part)[NP]) {
    float r[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = x[q];
#pragma unroll
    for (int t = 0; t < NP; ++t) {
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t p =
                __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{r[2 * q], r[2 * q + 1]}, bf16x2));
            w[q] = p;
            if (t + 1 < NP) {
                r[2 * q] -= __builtin_bit_cast(float, p << 16);
                r[2 * q + 1] -= __builtin_bit_cast(float, p & 0xffff0000u);
            }
        }
        part[t] = __builtin_bit_cast(bf16x8, u32x4{w[0], w[1], w[2], w[3]});
    }
}

__device__ __forceinline__ bf16x8 neg8(bf16x8 a) {
    u32x4 u = __builtin_bit_cast(u32x4, a);
    u ^= 0x80008000u;
    return __builtin_bit_cast(bf16x8, u);
}

// term pairs (p, q) of a split product: p indexes the A terms, q the B terms
template <int NP>
struct Pairs;
template <>
struct Pairs<2> {
    static constexpr int n = 3;
    static constexpr int p[3] = {0, 0, 1}, q[3] = {0, 1, 0};
};
template <>
struct Pairs<3> {
    static constexpr int n = 6;
    static constexpr int p[6] = {0, 0, 1, 0, 1, 2}, q[6] = {0, 1, 0, 2, 1, 0};
};

}  // namespace

// MODE: 2 = SPLIT2, 3 = SPLIT3 (NP bf16 terms), 0 = FP32 MFMA.  BT: square tile (128: 2 x 2
// waves of 64 x 64; 64: 2 x 2 waves of 32 x 32).  CHUNKED: the k range is summed in chunks
// of chk stages, each accumulated in FP32 by the MFMAs and then added to FP64 partial sums
// held in registers (with the 64 tile, 32 doubles per lane), so FP32 accumulation spans
// one chunk while the output is read and written once.
template <int MODE, bool FAST, int BT = 128, bool CHUNKED = false>
__global__ __launch_bounds__(256) void k_gemm_c64(SplitOps op, int chk) {
    constexpr int BM = BT, BN = BT;
    constexpr int TI = BT / 64;          // 32 x 32 MFMA tiles per wave along each side
    constexpr int RPW = BT / 4, NI = RPW / 8;  // rows per wave and loader passes
    __shared__ __attribute__((aligned(16))) float As[2][BM * RSF];
    __shared__ __attribute__((aligned(16))) float Bs[2][BN * RSF];

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

    const float *Af = reinterpret_cast<const float *>(op.A);
    const float *Bf = reinterpret_cast<const float *>(op.B);
    const float *Zf = reinterpret_cast<const float *>(op.zeros);

    // loader: piece lq = lane % 8 of a row's stage (k = 2 lq, 2 lq + 1; run lc = lq / 4 of
    // eight k), rows lr + 8 i (i = 0..3) of both A and B
    const int lq = lane & 7, lc = lq >> 2;
    const int lr = wave * RPW + (lane >> 3);
    int64_t arow[NI], bcol[NI];
    bool aok[NI], bok[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int am = m0 + lr + 8 * i, bn = n0 + lr + 8 * i;
        aok[i] = am < M;
        bok[i] = bn < N;
        arow[i] = op.a_row[(int64_t)g * M + (aok[i] ? am : M - 1)];
        bcol[i] = op.b_col[(int64_t)g * N + (bok[i] ? bn : N - 1)];
    }
    const int kclamp = FAST ? K - 8 : K - 1;
    f32x4 sa[NI], sb[NI];

    auto load_stage = [&](int k0) {
        if (FAST) {
            const int kb = k0 + lc * 8;
            const bool kok = kb < K;
            const int kk = min(kb, kclamp);
            const int64_t ak = op.a_k[(int64_t)g * kld + kk] + 2 * (lq & 3);
            const int64_t bk = op.b_k[(int64_t)g * kld + kk] + 2 * (lq & 3);
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                const float *pa = (kok && aok[i]) ? Af + 2 * (arow[i] + ak) : Zf;
                const float *pb = (kok && bok[i]) ? Bf + 2 * (bcol[i] + bk) : Zf;
                sa[i] = *(const f32x4 *)pa;
                sb[i] = *(const f32x4 *)pb;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                f32x2 va[2], vb[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int k = k0 + 2 * lq + u;
                    const bool kok = k < K;
                    const int kk = min(k, K - 1);
                    const float *pa = (kok && aok[i]) ? Af + 2 * (arow[i] + op.a_k[(int64_t)g * kld + kk]) : Zf;
                    const float *pb = (kok && bok[i]) ? Bf + 2 * (bcol[i] + op.b_k[(int64_t)g * kld + kk]) : Zf;
                    va[u] = *(const f32x2 *)pa;
                    vb[u] = *(const f32x2 *)pb;
                }
                sa[i] = f32x4{va[0].x, va[0].y, va[1].x, va[1].y};
                sb[i] = f32x4{vb[0].x, vb[0].y, vb[1].x, vb[1].y};
            }
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            *(f32x4 *)&As[buf][(lr + 8 * i) * RSF + 4 * lq] = sa[i];
            *(f32x4 *)&Bs[buf][(lr + 8 * i) * RSF + 4 * lq] = sb[i];
        }
    };

    f32x16 cr[TI][TI], ci[TI][TI];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TI; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) cr[i][j][r] = ci[i][j][r] = 0.f;
    // FP64 partial sums of the finished chunks (CHUNKED only; component arrays stay in
    // registers)
    double dr[CHUNKED ? TI * TI * 16 : 1], di[CHUNKED ? TI * TI * 16 : 1];
    if constexpr (CHUNKED) {
#pragma unroll
        for (int r = 0; r < TI * TI * 16; ++r) dr[r] = di[r] = 0.0;
    }

    const int nk = (K + BK - 1) / BK;
    if (nk > 0) {
        load_stage(0);
        store_stage(0);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int buf = kt & 1;
            if (kt + 1 < nk) load_stage((kt + 1) * BK);
            const float *as = As[buf], *bs = Bs[buf];
            if constexpr (MODE == 0) {
                // FP32: eight sub-steps of two k; lane (l32, lh) holds row l32, k = 2 s + lh
#pragma unroll
                for (int s = 0; s < BK / 2; ++s) {
                    f32x2 a[TI], b[TI];
#pragma unroll
                    for (int i = 0; i < TI; ++i) {
                        a[i] = *(const f32x2 *)&as[(wm * (BT / 2) + i * 32 + l32) * RSF + 2 * (2 * s + lh)];
                        b[i] = *(const f32x2 *)&bs[(wn * (BT / 2) + i * 32 + l32) * RSF + 2 * (2 * s + lh)];
                    }
#pragma unroll
                    for (int i = 0; i < TI; ++i)
#pragma unroll
                        for (int j = 0; j < TI; ++j) {
                            cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].x, cr[i][j], 0, 0, 0);
                            ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].y, ci[i][j], 0, 0, 0);
                        }
#pragma unroll
                    for (int i = 0; i < TI; ++i)
#pragma unroll
                        for (int j = 0; j < TI; ++j) {
                            cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[i].y, b[j].y, cr[i][j], 0, 0, 0);
                            ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].x, ci[i][j], 0, 0, 0);
                        }
                }
            } else {
                constexpr int NP = MODE;
                using PP = Pairs<NP>;
                // lane (l32, lh) holds the 8 k of half lh of its row l32, in NP terms each for
                // the real and the imaginary part
                bf16x8 are[TI][NP], aim[TI][NP], anim[TI][NP], bre[TI][NP], bim[TI][NP];
#pragma unroll
                for (int i = 0; i < TI; ++i) {
                    float xr[8], xi[8], yr[8], yi[8];
                    const float *pa = &as[(wm * (BT / 2) + i * 32 + l32) * RSF + 16 * lh];
                    const float *pb = &bs[(wn * (BT / 2) + i * 32 + l32) * RSF + 16 * lh];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const f32x4 qa = *(const f32x4 *)(pa + 4 * v), qb = *(const f32x4 *)(pb + 4 * v);
                        xr[2 * v] = qa.x, xi[2 * v] = qa.y, xr[2 * v + 1] = qa.z, xi[2 * v + 1] = qa.w;
                        yr[2 * v] = qb.x, yi[2 * v] = qb.y, yr[2 * v + 1] = qb.z, yi[2 * v + 1] = qb.w;
                    }
                    split_terms<NP>(xr, are[i]);
                    split_terms<NP>(xi, aim[i]);
                    split_terms<NP>(yr, bre[i]);
                    split_terms<NP>(yi, bim[i]);
#pragma unroll
                    for (int t = 0; t < NP; ++t) anim[i][t] = neg8(aim[i][t]);
                }
                // smallest terms first, so the leading product is added last to each chain
#pragma unroll
                for (int u = PP::n - 1; u >= 0; --u) {
                    const int p = PP::p[u], q = PP::q[u];
#pragma unroll
                    for (int i = 0; i < TI; ++i)
#pragma unroll
                        for (int j = 0; j < TI; ++j) {
                            cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(are[i][p], bre[j][q], cr[i][j], 0, 0, 0);
                            ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(are[i][p], bim[j][q], ci[i][j], 0, 0, 0);
                        }
#pragma unroll
                    for (int i = 0; i < TI; ++i)
#pragma unroll
                        for (int j = 0; j < TI; ++j) {
                            cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(anim[i][p], bim[j][q], cr[i][j], 0, 0, 0);
                            ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aim[i][p], bre[j][q], ci[i][j], 0, 0, 0);
                        }
                }
            }
            if constexpr (CHUNKED) {
                if ((kt + 1) % chk == 0 || kt + 1 == nk) {  // a chunk is complete: into FP64
#pragma unroll
                    for (int i = 0; i < TI; ++i)
#pragma unroll
                        for (int j = 0; j < TI; ++j)
#pragma unroll
                            for (int r = 0; r < 16; ++r) {
                                dr[(i * TI + j) * 16 + r] += (double)cr[i][j][r];
                                di[(i * TI + j) * 16 + r] += (double)ci[i][j][r];
                                cr[i][j][r] = ci[i][j][r] = 0.f;
                            }
                }
            }
            if (kt + 1 < nk) store_stage(buf ^ 1);
            __syncthreads();
        }
    }

    // epilogue (as in gemm_mixed.hip): register r of a lane holds row 8 (r / 4) + 4 lh + r % 4
    // of column l32 of its 32 x 32 tile
    const double alpha = op.alpha, beta = op.beta;
#pragma unroll
    for (int i = 0; i < TI; ++i) {
        const int mb = m0 + wm * (BT / 2) + i * 32 + 4 * lh;
        int64_t crow[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = mb + 8 * (r >> 2) + (r & 3);
            crow[r] = m < M ? op.c_row[(int64_t)g * M + m] : -1;
        }
        int64_t ccol[TI], cscol[TI];
#pragma unroll
        for (int j = 0; j < TI; ++j) {
            const int n = n0 + wn * (BT / 2) + j * 32 + l32;
            ccol[j] = n < N ? op.c_col[(int64_t)g * N + n] : -1;
            cscol[j] = (n < N && op.cs_col) ? op.cs_col[(int64_t)g * N + n] : ccol[j];
        }
        cd o[TI][16];
        if (beta != 0.0) {
#pragma unroll
            for (int j = 0; j < TI; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    o[j][r] = crow[r] >= 0 && ccol[j] >= 0 ? op.C[crow[r] + ccol[j]] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int j = 0; j < TI; ++j) {
            if (ccol[j] < 0) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if (crow[r] < 0) continue;
                const double sr = CHUNKED ? dr[(i * TI + j) * 16 + r] : (double)cr[i][j][r];
                const double si = CHUNKED ? di[(i * TI + j) * 16 + r] : (double)ci[i][j][r];
                cd v = make_double2(alpha * sr, alpha * si);
                if (beta != 0.0) {
                    v.x = fma(beta, o[j][r].x, v.x);
                    v.y = fma(beta, o[j][r].y, v.y);
                }
                if (op.Cs) {
                    const int m = mb + 8 * (r >> 2) + (r & 3);
                    const int64_t e = (op.cs_row ? op.cs_row[(int64_t)g * M + m] : crow[r]) + cscol[j];
                    reinterpret_cast<cf *>(op.Cs)[e] = make_float2((float)v.x, (float)v.y);
                } else {
                    op.C[crow[r] + ccol[j]] = v;
                }
            }
        }
    }
}

void gemm_c64(const SplitOps &op, int arith, hipStream_t s) {
    if (op.G <= 0 || op.M <= 0 || op.N <= 0) return;
    const dim3 grid = gemm_tile_grid((op.M + 127) / 128, (op.N + 127) / 128, op.G);
#define CK_LAUNCH(MODE)                                                                 \
    if (op.fast)                                                                        \
        hipLaunchKernelGGL((k_gemm_c64<MODE, true>), grid, dim3(256), 0, s, op, 0);     \
    else                                                                                \
        hipLaunchKernelGGL((k_gemm_c64<MODE, false>), grid, dim3(256), 0, s, op, 0);
    switch (arith) {
    case ARITH_SPLIT2: CK_LAUNCH(2); break;
    case ARITH_SPLIT3: CK_LAUNCH(3); break;
    case ARITH_FP32: CK_LAUNCH(0); break;
    default: throw HipError(hipErrorInvalidValue, "gemm_c64: arithmetic form", __FILE__, __LINE__);
    }
#undef CK_LAUNCH
    CK_CHECK(hipGetLastError());
}

void gemm_c64_chunked(const SplitOps &op, int arith, int kchunk, hipStream_t s) {
    if (op.G <= 0 || op.M <= 0 || op.N <= 0) return;
    if (kchunk < BK || kchunk % BK) throw HipError(hipErrorInvalidValue, "gemm_c64_chunked: chunk", __FILE__, __LINE__);
    const int chk = kchunk / BK;
    const dim3 grid = gemm_tile_grid((op.M + 63) / 64, (op.N + 63) / 64, op.G);
#define CK_LAUNCH(MODE)                                                                         \
    if (op.fast)                                                                                \
        hipLaunchKernelGGL((k_gemm_c64<MODE, true, 64, true>), grid, dim3(256), 0, s, op, chk);  \
    else                                                                                        \
        hipLaunchKernelGGL((k_gemm_c64<MODE, false, 64, true>), grid, dim3(256), 0, s, op, chk);
    switch (arith) {
    case ARITH_SPLIT2: CK_LAUNCH(2); break;
    case ARITH_SPLIT3: CK_LAUNCH(3); break;
    case ARITH_FP32: CK_LAUNCH(0); break;
    default: throw HipError(hipErrorInvalidValue, "gemm_c64_chunked: arithmetic form", __FILE__, __LINE__);
    }
#undef CK_LAUNCH
    CK_CHECK(hipGetLastError());
}

// complex128 -> complex64 storage (round to nearest); padding to a multiple of 8 zeroed
__global__ void k_to_c64_padded(int64_t n, int64_t npad, const cd *src, cf *dst) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < npad; e += (int64_t)gridDim.x * blockDim.x) {
        const cd x = e < n ? src[e] : make_double2(0.0, 0.0);
        dst[e] = make_float2((float)x.x, (float)x.y);
    }
}

void launch_to_c64(int64_t n, const cd *src, cf *dst, hipStream_t st) {
    const int64_t npad = (n + 7) / 8 * 8;
    const int64_t b = std::min<int64_t>((npad + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(k_to_c64_padded, dim3((unsigned)std::max<int64_t>(b, 1)), dim3(256), 0, st, n, npad, src, dst);
    CK_CHECK(hipGetLastError());
}

}  // namespace ck
