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
// One workgroup per (ka, kb, ke, a), XCD-contiguous block order (see the FP64 kernel).
__global__ void k_vvvv_dress_split(SysDev s, const cd *t1, uint16_t *Vt, int64_t plane) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t v3 = (int64_t)nv * nv * nv, v4 = v3 * nv, ov3 = (int64_t)no * v3;
    const int64_t nblk = (int64_t)N * N * N * nv;
    const int64_t per = (nblk + 7) / 8;
    const int64_t L = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nblk) return;
    const int a = (int)(L % nv);
    const int64_t blk = L / nv;
    const int ke = (int)(blk % N), kb = (int)((blk / N) % N), ka = (int)(blk / ((int64_t)N * N));
    const cd *g1b = s.ovvv + (((int64_t)kb * N + ka) * N + ke) * ov3 + (int64_t)a * nv * nv;
    const cd *g2b = s.ovvv + (((int64_t)ka * N + kb) * N + ke) * ov3;
    for (int64_t e = threadIdx.x; e < v3; e += blockDim.x) {
        const int ef = (int)(e % (nv * nv)), b = (int)(e / (nv * nv));
        const int64_t idx = blk * v4 + (int64_t)a * v3 + e;
        cd acc = s.vvvv[idx];
        for (int m = 0; m < no; ++m) {
            cfma(acc, t1[((int64_t)kb * no + m) * nv + b], g1b[(int64_t)m * v3 + ef]);
            acc = csub(acc, cmul(t1[((int64_t)ka * no + m) * nv + a], g2b[(int64_t)m * v3 + (int64_t)b * nv * nv + ef]));
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
    const int64_t nblk = (int64_t)s.d.N * s.d.N * s.d.N * s.d.nv;
    hipLaunchKernelGGL(k_vvvv_dress_split, dim3((unsigned)(((nblk + 7) / 8) * 8)), dim3(256), 0, st, s, t1, Vt, plane);
    CK_CHECK(hipGetLastError());
}

}  // namespace ck
