// T1 dressing of the particle-particle integrals for the mixed-precision path: the same
// arithmetic as the FP64 kernel (FP64), written directly as split-BF16 planes that the
// particle-particle ladder streams, so no complex128 copy of the dressed block exists.
#include "common.h"
#include "mixed.h"

namespace ck {

__device__ inline uint16_t rne16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline void split_pair(double x, uint16_t &hi, uint16_t &lo) {
    hi = rne16((float)x);
    lo = rne16((float)(x - (double)__builtin_bit_cast(float, (uint32_t)hi << 16)));
}

// Vt[ka][kb][ke](a,b,e,f) = <ab||ef> + t_m^b <m kb, a ka||ef> - t_m^a <m ka, b kb||ef>
__global__ void k_vvvv_dress_split(SysDev s, const cd *t1, uint16_t *Vt, int64_t plane) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t v4 = (int64_t)nv * nv * nv * nv, ov3 = (int64_t)no * nv * nv * nv;
    const int64_t total = (int64_t)N * N * N * v4;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int f = (int)(idx % nv), e = (int)((idx / nv) % nv);
        int b = (int)((idx / ((int64_t)nv * nv)) % nv), a = (int)((idx / ((int64_t)nv * nv * nv)) % nv);
        int64_t blk = idx / v4;
        int ke = (int)(blk % N), kb = (int)((blk / N) % N), ka = (int)(blk / ((int64_t)N * N));
        cd acc = s.vvvv[idx];
        const cd *g1 = s.ovvv + (((int64_t)kb * N + ka) * N + ke) * ov3 + ((int64_t)a * nv + e) * nv + f;
        const cd *g2 = s.ovvv + (((int64_t)ka * N + kb) * N + ke) * ov3 + ((int64_t)b * nv + e) * nv + f;
        for (int m = 0; m < no; ++m) {
            cfma(acc, t1[((int64_t)kb * no + m) * nv + b], g1[(int64_t)m * nv * nv * nv]);
            acc = csub(acc, cmul(t1[((int64_t)ka * no + m) * nv + a], g2[(int64_t)m * nv * nv * nv]));
        }
        uint16_t p0, p1, p2, p3;
        split_pair(acc.x, p0, p1);
        split_pair(acc.y, p2, p3);
        Vt[idx] = p0;
        Vt[plane + idx] = p1;
        Vt[2 * plane + idx] = p2;
        Vt[3 * plane + idx] = p3;
    }
}

void launch_vvvv_dress_split(const SysDev &s, const cd *t1, uint16_t *Vt, int64_t plane, hipStream_t st) {
    const int64_t total = (int64_t)s.d.N * s.d.N * s.d.N * s.d.nv * s.d.nv * s.d.nv * s.d.nv;
    int64_t b = std::min<int64_t>((total + 255) / 256, 1 << 20);
    hipLaunchKernelGGL(k_vvvv_dress_split, dim3((unsigned)std::max<int64_t>(b, 1)), dim3(256), 0, st, s, t1, Vt,
                       plane);
    CK_CHECK(hipGetLastError());
}

}  // namespace ck
