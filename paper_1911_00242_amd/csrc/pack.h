// Declarations of the antisymmetric pair packing, the packed R2 assembly and the mixed-path
// DIIS extrapolation (pack.hip).
#pragma once
#include "common.h"
#include "mixed.h"

namespace ck {

// Canonical pairs of each group of total pair momentum K (pack.hip): vlist[K*PV + p] =
// (kx*nv + x)*nv + y for the p-th canonical virtual pair of group K, -1 in the padding;
// olist likewise for occupied pairs (PO); vpos[(K*N + kx)*nv*nv + x*nv + y] = p, or -1
// when (kx, x, y) is not canonical; opos likewise for occupied pairs.  PV and PO are
// multiples of 16.  dblk lists the ndblk momentum blocks (ka*N + kb)*N + ke with ka <= kb
// and ke <= kf, the only ones holding canonical (a,b) and (e,f) pairs; ablk lists the nablk
// R2 blocks (ki*N + kj)*N + ka with ki <= kj and ka <= kb, one per antisymmetry orbit.
struct PairTabs {
    const int32_t *vlist, *olist, *vpos, *opos, *dblk, *ablk;
    int PV, PO, ndblk, nablk;
};

// packed ladder operands in split storage (pack.hip), rows ld elements apart: tau rows
// [K][(ki,i,j)][PV] and its hole-hole form [K][PV][PO]; <mn||ef> as [K][PO][PV]; the
// dressed <ab||ef> as [K][PV][PV]
bool dress_pack_ok(const Dims &d);
void launch_tau_pack(const Dims &d, const int32_t *kc, const PairTabs &pt, const cd *t1, const cd *t2,
                     uint16_t *tau_pk, int64_t ld_tau, uint16_t *tauT_pk, int64_t ld_tauT, hipStream_t st);
void launch_oovv_pack(const Dims &d, const int32_t *kc, const PairTabs &pt, const cd *oovv, uint16_t *out,
                      hipStream_t st);
// DIIS extrapolation of the mixed path: t = sum_j c[j] src[j] over (t1 | t2) (m <= 16), the
// split copy of the new t2 into sp, and the energy at the new amplitudes as partial sums in
// epart (2 + 2 * lincomb_t2_blocks doubles), which launch_energy_pack reduces into out[0..1]
constexpr int LINCOMB_T2_BLOCKS = 4096;
struct LincombArgs {
    const cd *src[16];
    double c[16];
};
int lincomb_t2_blocks(const Dims &d);
void launch_lincomb_pack(const SysDev &s, const cd *const *src, const double *c, int m, cd *t, uint16_t *sp,
                         double *epart, hipStream_t st);
void launch_energy_pack(const Dims &d, const double *epart, double *out, hipStream_t st);
// r2 = <ab||ij>* + P(ij)P(ab) X + the ladders' packed result Lp expanded by antisymmetry,
// stored in complex64; npart (assemble_pack_blocks doubles) receives per-workgroup sums of
// |r2|^2 over the stored values
int64_t assemble_pack_blocks(const Dims &d, const PairTabs &pt);
void launch_assemble_r2_pack(const SysDev &s, const PairTabs &pt, const cd *X, const cd *Lp, cf *r2, double *npart,
                             hipStream_t st);
// out[0] = sum |r1|^2 + sum |r2|^2 from the assembly's partial sums (fixed order)
void launch_norm_pack(const Dims &d, const PairTabs &pt, const double *npart, const cd *r1, double *out,
                      hipStream_t st);
void launch_vvvv_dress_pack(const SysDev &s, const PairTabs &pt, const cd *t1, uint16_t *out, int64_t ld,
                            hipStream_t st);

}  // namespace ck
