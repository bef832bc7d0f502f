// Launchers of the residual's elementwise / small-contraction kernels and of the
// reductions, update and DIIS kernels (internal to libccsdk).
#pragma once
#include "sysdev.h"

namespace ck {

// Workgroups per momentum block of the generic (1024-thread) F and R1 block-sum kernels
// (n_occ, n_vir <= 32 outside the 8 x 16 tile): the loop over n is split into this many
// ranges, each writing its own partial sums, so that grids with few momentum blocks still
// fill the chip (about 256 workgroups, at most one range per n). 1 for every other form.
// The partial arrays hold this many N^3-block slices.
__host__ __device__ inline int fr_splits(const Dims &d) {
    if ((d.no <= 8 && d.nv <= 16) || d.no > 32 || d.nv > 32) return 1;
    const int n3 = d.N * d.N * d.N, want = (256 + n3 - 1) / n3;
    return want < d.no ? want : d.no;
}

struct FWork {
    cd *Fov, *Foo, *Fvv;  // [N][o][v], [N][o][o], [N][v][v]
    cd *Fot, *Fvt;        // [N][o][o], [N][v][v]
    cd *Poo, *Pvv;        // [splits][N][N][N][o][o], [splits][N][N][N][v][v] partial sums
};

// Register-tiled F and R1 block sums (blocksum.hip) for n_occ <= 16, n_vir <= 32 outside
// the 8 x 16 tile: the same partial arrays (fr_splits slices each) as the other forms.
bool bsum_rb_fits(const Dims &d);
void launch_f_blocks_rb(const SysDev &s, const cd *t1, const cd *t2, cd *Poo, cd *Pvv, hipStream_t st);
void launch_r1_blocks_rb(const SysDev &s, const cd *t2, cd *P1a, cd *P1b, hipStream_t st);

void launch_tau(const SysDev &s, const cd *t1, const cd *t2, cd *tau, cd *tauT, hipStream_t st);
void launch_f(const SysDev &s, const cd *t1, const cd *t2, FWork w, hipStream_t st);
// canon: only the blocks with canonical rows and columns (ki <= kj, km <= kn) are written
// (all that the packed W_mnij product reads)
void launch_wmnij_init(const SysDev &s, const cd *t1, cd *WT, bool canon, hipStream_t st);
void launch_vvvv_dress(const SysDev &s, const cd *t1, cd *Vt, hipStream_t st);
// per momentum block (o^2 x v^2) -> (v^2 x o^2)
void launch_block_transpose(const Dims &d, const cd *src, cd *dst, hipStream_t st);
// rearranged hole-hole grouping (FP64 path): Y-tilde_{mnij} in place on the W_mnij seed, and
// the single-amplitude rest of the hole-hole ladder added to r2
void launch_ytilde(const SysDev &s, const cd *t1, cd *WT, hipStream_t st);
void launch_hh_t1_rest(const SysDev &s, const cd *t1, const cd *Y, const cd *X, cd *r2, hipStream_t st);
// ring seeds: W_mbej without its t2 part (WR) and X = every non-ladder, non-driver term
// arranged for one P(ij)P(ab); needs the F combinations of w
void launch_ring_init(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, cd *scratch, cd *WR, cd *X,
                      hipStream_t st);
// the same in two independent parts, each with its own scratch (N^3 o^3 v elements): the
// W_mbej seed (WR) and the X seed (needs the F combinations of w)
void launch_ring_w(const SysDev &s, const cd *t1, cd *scratch, cd *WR, hipStream_t st);
void launch_ring_x(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, cd *scratch, cd *X,
                   hipStream_t st);
// r2 = <ab||ij> + P(ij)P(ab) X
void launch_assemble_r2(const SysDev &s, const cd *X, cd *r2, hipStream_t st);
// Relaid-out copies of the static classes, made once per set of inputs on the FP64 path:
// ovvoT, ovvvT and oovvT (the last two indices swapped).
struct StaticCopies {
    cd *ovvoT, *ovvvT, *oovvT;
};
void launch_static_copies(const SysDev &s, const StaticCopies &c, hipStream_t st);
// The mixed path keeps its integral classes in complex64 only; they are made once per set
// of inputs from complex128 values passed through a staging buffer, a range at a time:
// dst = src rounded to complex64 (round_c64: exactly n elements, no padding) or widened
// to complex128 (to_c128) over n elements; nblocks blocks of v x v with their two indices
// swapped, rounded; the whole ovvo class (staged) into the swapped complex64 copy ovvoT_c.
void launch_round_c64(int64_t n, const cd *src, cf *dst, hipStream_t st);
void launch_to_c128(int64_t n, const cf *src, cd *dst, hipStream_t st);
void launch_swap_last2_c64(int64_t nblocks, int v, const cd *src, cf *dst, hipStream_t st);
void launch_ovvo_transpose_c64(const Dims &d, const cd *ovvo, cf *ovvoT, hipStream_t st);
void launch_r1(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, cd *P1, cd *r1, hipStream_t st);
// the two halves of launch_r1: the t2 x integral partial sums (which need no intermediate),
// then R1 from t1, t2, F and those partials
void launch_r1_partials(const SysDev &s, const cd *t2, cd *P1, hipStream_t st);
void launch_r1_final(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, const cd *P1, cd *r1,
                     hipStream_t st);

// reductions (deterministic: fixed grid, fixed-order partial sums) -------------------
constexpr int RED_BLOCKS = 1024;
constexpr int UPD_BLOCKS = 4096;  // grid of the DIIS update pass (its partials: m * UPD_BLOCKS)
// out[0] = sum |r1|^2 + |r2|^2 ; partials must hold RED_BLOCKS doubles
void launch_norm2(const Dims &d, const cd *r1, const cd *r2, double *partials, double *out, hipStream_t st);
// out[0..1] = complex correlation energy; partials must hold 2*RED_BLOCKS doubles
void launch_energy(const SysDev &s, const cd *t1, const cd *t2, double *partials, double *out, hipStream_t st);
// The iteration's gate: the update kernels of a system run only while its residual norm
// of this iteration (norm2 = ||R||^2 on the device) is at or above tol, so that one
// enqueued (or graph-replayed) iteration leaves a converged system's amplitudes alone.  The
// host takes the same decision, sqrt(norm2) < tol, from the same value.
struct Gate {
    const double *norm2;
    double tol;
    __device__ bool open() const { return sqrt(*norm2) >= tol; }
};

// Device-resident DIIS state of one system: state[0] the slot the next update writes (FIFO
// head), state[1] the vectors held before it; B the m x m error overlaps (row / column of a
// slot rewritten when the slot is), bnew the overlaps of the newest error vector, coef the
// extrapolation coefficients of the held slots.
struct DiisDev {
    int32_t *state;
    double *B, *bnew, *coef;
    int m;
};

// t += r / D, and (optionally) err = r / D; r2 complex128, or complex64 (mixed path)
void launch_update(const SysDev &s, cd *t1, cd *t2, const cd *r1, const cd *r2, cd *err1, cd *err2, Gate gate,
                   hipStream_t st);
void launch_update(const SysDev &s, cd *t1, cd *t2, const cd *r1, const cf *r2, cd *err1, cd *err2, Gate gate,
                   hipStream_t st);
// the DIIS step: overlaps from nparts partial sums per held vector, B, the bordered solve,
// the coefficients and the FIFO advance (one workgroup); the update pass and the
// extrapolation on the packed history are in pack.h
void launch_diis_solve(const DiisDev &dd, Gate gate, const double *partials, int nparts, hipStream_t st);

// device synthetic inputs (same recipe as the host generator) ------------------------
void launch_synth_fock(const Mesh &m, int no, int nv, uint64_t seed, cd *fock, hipStream_t st);
void launch_synth_eri(const Mesh &m, int no, int nv, uint64_t seed, double scale, const char *cls, cd *out,
                      hipStream_t st);
// elements c0 .. c0+len-1 of class cls into out[0 .. len-1]; with blist, the class stored on
// the listed momentum blocks only (element c in block blist[c / block size])
void launch_synth_eri_range(const Mesh &m, int no, int nv, uint64_t seed, double scale, const char *cls,
                            const int32_t *blist, int64_t c0, int64_t len, cd *out, hipStream_t st);
void launch_diag(const Dims &d, const cd *fock, double *eo, double *ev, hipStream_t st);

}  // namespace ck
