// Grouped complex FP64 GEMM over momentum-conserving blocks, on CDNA4 FP64 MFMA.
//
// Every contraction of the T2 residual that carries the N_band^6 N_k^4 cost (Sec. 3.1 of
// the paper; the eight-index sums of Sec. 4.3.4) becomes, once two momenta are fixed by
// a group label (total pair momentum K for the ladders, transfer q for the ring), a dense
// complex matrix product per group.  Operands are read in place from their canonical
// block layouts through per-row / per-column / per-k offset tables (GemmOps), so one
// kernel serves all five products without relayout passes; each table lookup is done
// once per tile row/column, and the k offsets of one tile are contiguous runs of at least
// n_vir (or n_occ^2) elements, so global loads stay coalesced.
//
// Tile: BM x BN complex outputs per 256-thread workgroup (4 waves as WM x WN), BK complex
// k-values per LDS stage, double buffered.  A complex multiply-accumulate is four real
// v_mfma_f64_16x16x4 products (re*re, -im*im into the real accumulator; re*im, im*re into
// the imaginary one).
#include "common.h"

namespace ck {

typedef double v4d __attribute__((ext_vector_type(4)));

template <int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmOps<cd> op) {
    constexpr int NT = 256;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    constexpr int RA = BM * BK / NT, RB = BN * BK / NT;  // complex loads per thread
    constexpr int ROWS_PER_PASS = NT / BK;
    static_assert(WM * WN == 4, "four waves");
    static_assert(BM * BK % NT == 0 && BN * BK % NT == 0, "tile/thread mismatch");

    __shared__ cd As[2][BK][BM + 1];
    __shared__ cd Bs[2][BK][BN + 1];

    const int tid = threadIdx.x;
    const int g = blockIdx.z;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int M = op.M, N = op.N, K = op.K;
    const int kl = tid % BK;        // this thread's k lane within a stage
    const int rl = tid / BK;        // first row/col handled by this thread

    // per-thread row (A) and column (B) base offsets; -1 marks out-of-range rows
    int64_t arow[RA], bcol[RB];
#pragma unroll
    for (int i = 0; i < RA; ++i) {
        int m = m0 + rl + i * ROWS_PER_PASS;
        arow[i] = m < M ? op.a_row[(int64_t)g * M + m] : -1;
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        int n = n0 + rl + i * ROWS_PER_PASS;
        bcol[i] = n < N ? op.b_col[(int64_t)g * N + n] : -1;
    }

    cd ra[RA], rb[RB];
    auto load = [&](int k0) {
        int k = k0 + kl;
        bool kin = k < K;
        int64_t ak = kin ? op.a_k[(int64_t)g * K + k] : 0;
        int64_t bk = kin ? op.b_k[(int64_t)g * K + k] : 0;
#pragma unroll
        for (int i = 0; i < RA; ++i)
            ra[i] = (kin && arow[i] >= 0) ? op.A[arow[i] + ak] : make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < RB; ++i)
            rb[i] = (kin && bcol[i] >= 0) ? op.B[bcol[i] + bk] : make_double2(0.0, 0.0);
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < RA; ++i) As[buf][kl][rl + i * ROWS_PER_PASS] = ra[i];
#pragma unroll
        for (int i = 0; i < RB; ++i) Bs[buf][kl][rl + i * ROWS_PER_PASS] = rb[i];
    };

    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int l16 = lane & 15, lk = lane >> 4;

    v4d acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            acc_re[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
            acc_im[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        }

    const int nk = (K + BK - 1) / BK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            cd af[FM], bf[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) af[i] = As[buf][kk + lk][wm * TM + i * 16 + l16];
#pragma unroll
            for (int j = 0; j < FN; ++j) bf[j] = Bs[buf][kk + lk][wn * TN + j * 16 + l16];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].x, bf[j].x, acc_re[i][j], 0, 0, 0);
                    acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-af[i].y, bf[j].y, acc_re[i][j], 0, 0, 0);
                    acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].x, bf[j].y, acc_im[i][j], 0, 0, 0);
                    acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].y, bf[j].x, acc_im[i][j], 0, 0, 0);
                }
        }
        if (kt + 1 < nk) store(buf ^ 1);
        __syncthreads();
    }

    // epilogue: for the f64 16x16x4 MFMA, register r of a lane holds row 4*r + lane/16
    // of column lane%16 of each 16x16 tile
    const double alpha = op.alpha, beta = op.beta;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int n = n0 + wn * TN + j * 16 + l16;
            if (n >= N) continue;
            const int64_t ccol = op.c_col[(int64_t)g * N + n];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * TM + i * 16 + r * 4 + lk;
                if (m >= M) continue;
                cd *p = op.C + op.c_row[(int64_t)g * M + m] + ccol;
                cd v = make_double2(alpha * acc_re[i][j][r], alpha * acc_im[i][j][r]);
                if (beta != 0.0) {
                    cd o = *p;
                    v.x = fma(beta, o.x, v.x);
                    v.y = fma(beta, o.y, v.y);
                }
                *p = v;
            }
        }
}

// One thread per output element; for tests of the tiled kernel only.
__global__ void k_gemm_f64_reference(GemmOps<cd> op) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)op.G * op.M * op.N;
    if (idx >= total) return;
    int n = (int)(idx % op.N);
    int m = (int)((idx / op.N) % op.M);
    int g = (int)(idx / ((int64_t)op.N * op.M));
    cd acc = make_double2(0.0, 0.0);
    int64_t ar = op.a_row[(int64_t)g * op.M + m], bc = op.b_col[(int64_t)g * op.N + n];
    for (int k = 0; k < op.K; ++k)
        cfma(acc, op.A[ar + op.a_k[(int64_t)g * op.K + k]], op.B[bc + op.b_k[(int64_t)g * op.K + k]]);
    cd *p = op.C + op.c_row[(int64_t)g * op.M + m] + op.c_col[(int64_t)g * op.N + n];
    cd v = cscale(acc, op.alpha);
    if (op.beta != 0.0) v = cadd(v, cscale(*p, op.beta));
    *p = v;
}

void gemm_f64(const GemmOps<cd> &op, hipStream_t s) {
    if (op.G <= 0 || op.M <= 0 || op.N <= 0) return;
    constexpr int BM = 64, BN = 64, BK = 16;
    dim3 grid((op.N + BN - 1) / BN, (op.M + BM - 1) / BM, op.G);
    hipLaunchKernelGGL((k_gemm_f64<BM, BN, BK, 2, 2>), grid, dim3(256), 0, s, op);
    CK_CHECK(hipGetLastError());
}

void gemm_f64_reference(const GemmOps<cd> &op, hipStream_t s) {
    int64_t total = (int64_t)op.G * op.M * op.N;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_gemm_f64_reference, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, op);
    CK_CHECK(hipGetLastError());
}

}  // namespace ck
