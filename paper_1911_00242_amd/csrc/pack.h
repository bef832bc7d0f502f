// Declarations of the antisymmetric pair packing, the packed R2 assembly and the mixed-path
// DIIS extrapolation (pack.hip).
#pragma once
#include "common.h"
#include "mixed.h"
#include "terms.h"

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
// c64: complex64 storage instead of split storage (the ladder family's operand storage)
void launch_tau_pack(const Dims &d, const int32_t *kc, const PairTabs &pt, const cd *t1, const cd *t2,
                     uint16_t *tau_pk, int64_t ld_tau, uint16_t *tauT_pk, int64_t ld_tauT, bool c64, hipStream_t st);
void launch_oovv_pack(const Dims &d, const int32_t *kc, const PairTabs &pt, const cd *oovv, uint16_t *out, bool c64,
                      hipStream_t st);
// DIIS extrapolation argument block (m <= 16 source vectors)
struct LincombArgs {
    const cd *src[16];
};
// Packed DIIS history (both paths): vectors of packed_len elements, t1 in full then t2 on
// the orbit representatives pt.ablk (whole blocks).  The update writes hist = packed
// (t + D^-1 R) and err = packed D^-1 R (complex64 on the mixed path, whose R2 is complex64;
// complex128 on the FP64 path) and the weighted overlaps out[j] = Re <e, y_j> over the full
// vector (partials: 16 * 4096 doubles); the extrapolation t = sum_j c[j] src[j] writes t
// (full) and, on the mixed path (epart non-null), its operand copy sp in the ring family's
// storage and the energy at the new amplitudes as partial sums (2 + 2 *
// lincomb_pack_blocks doubles, reduced into out[0..1] by launch_energy_packed).
int64_t packed_len(const Dims &d, const PairTabs &pt);
int64_t lincomb_pack_blocks(const Dims &d, const PairTabs &pt);
void launch_update_diis_pack(const SysDev &s, const PairTabs &pt, const cd *t, const cd *r1, const cf *r2,
                             cf *const *err, cd *const *hist, const DiisDev &dd, Gate gate, double *partials,
                             hipStream_t st);
void launch_update_diis_pack(const SysDev &s, const PairTabs &pt, const cd *t, const cd *r1, const cd *r2,
                             cd *const *err, cd *const *hist, const DiisDev &dd, Gate gate, double *partials,
                             hipStream_t st);
void launch_lincomb_packed(const SysDev &s, const PairTabs &pt, const cd *const *src, const DiisDev &dd, Gate gate,
                           cd *t, uint16_t *sp, bool c64, double *epart, hipStream_t st);
void launch_energy_packed(const Dims &d, const PairTabs &pt, const double *epart, double *out, hipStream_t st);
// r2 = <ab||ij>* + P(ij)P(ab) X + the ladders' packed result Lp expanded by antisymmetry,
// stored in complex64; npart (assemble_pack_blocks doubles) receives per-workgroup sums of
// |r2|^2 over the stored values
int64_t assemble_pack_blocks(const Dims &d, const PairTabs &pt);
void launch_assemble_r2_pack(const SysDev &s, const PairTabs &pt, const cd *X, const cd *Lp, cf *r2, double *npart,
                             hipStream_t st);
// out[0] = sum |r1|^2 + sum |r2|^2 from the assembly's partial sums (fixed order)
void launch_norm_pack(const Dims &d, const PairTabs &pt, const double *npart, const cd *r1, double *out,
                      hipStream_t st);
void launch_vvvv_dress_pack(const SysDev &s, const PairTabs &pt, const cd *t1, uint16_t *out, int64_t ld, bool c64,
                            hipStream_t st);

}  // namespace ck
