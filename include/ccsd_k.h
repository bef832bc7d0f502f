/*
 * ccsd_k.h — C ABI of libccsdk: the double-excitation (T2) residual of periodic
 * (k-point) spin-orbital CCSD, and the iteration around it, on one AMD MI355X (gfx950).
 *
 * What is computed (Yamashita, Kosugi, Matsushita, Sakurai, "A Parallel Computing Method
 * for the Coupled-Cluster Singles and Doubles", arXiv:1911.00242):
 *   - R2: the right-hand side of the T2 equation (Sec. 2, eq. ori_EqDouble) with the
 *     intermediates W (hole-hole, particle-particle, ring; Sec. 2 up to eq. Def_Woovv),
 *     F (eqs. ori_F_oo, ori_F_vv, ori_F_ov) and the effective amplitudes tau, tau-tilde;
 *   - R1: the right-hand side of the T1 equation (eq. ori_EqSingle);
 *   - the update t <- t + D^-1 R and the convergence test of Sec. 4.4 (successive
 *     substitution), optionally accelerated by Pulay DIIS;
 *   - the correlation energy (not printed in the paper; the standard spin-orbital
 *     expression  E = sum f_ia t_i^a + 1/4 sum <ij||ab> t_ij^ab + 1/2 sum <ij||ab> t_i^a t_j^b).
 * Momentum conservation (Sec. 3.2.5): k_p + k_q = k_r + k_s modulo a reciprocal lattice
 * vector on a Gamma-containing regular mesh.  A k label is the C-order linear index
 * k = (k0*grid[1] + k1)*grid[2] + k2.
 *
 * Array layouts (host and device alike; complex numbers interleaved re, im; row-major):
 *   fock  [N_k][n][n]                 complex128, n = n_occ + n_vir, occupied first
 *   eri[c][kp][kq][kr][p][q][r][s]    complex128 <pq||rs>, k_s fixed by conservation,
 *                                     c = 0..5 for classes oooo, ooov, oovv, ovvo, ovvv, vvvv
 *   t1, r1 [k][i][a]                  complex128
 *   t2, r2 [ki][kj][ka][i][j][a][b]   complex128, k_b fixed by conservation; every block
 *                                     and element stored (the antisymmetric copies too)
 *
 * Ownership: host arrays are read or written only during the call that receives them.
 * The device workspace is allocated by the caller (for instance a torch uint8 tensor),
 * must stay alive until ccsd_k_free, and is owned by the context while bound.  All device
 * work is enqueued on the HIP stream given to ccsd_k_init; calls that return host results
 * synchronize that stream.
 *
 * Errors: every int function returns CCSD_K_OK (0), a positive warning, or a negative
 * error; ccsd_k_last_error() describes the last failure.  After CCSD_K_EDEVICE the
 * context refuses further work (CCSD_K_ESTATE).  No C++ exception crosses the ABI.
 * A context is not thread safe; two contexts may be used from different threads.
 */
#ifndef CCSD_K_H
#define CCSD_K_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CCSD_K_OK 0
#define CCSD_K_NOT_CONVERGED 1 /* iterate: max_iter reached before ||R|| < tol      */
#define CCSD_K_EINVAL (-1)     /* bad argument, size, pointer or index                */
#define CCSD_K_ENOMEM (-2)     /* workspace smaller than ccsd_k_workspace_bytes, or a
                                  host allocation failed                            */
#define CCSD_K_EDEVICE (-3)    /* a HIP runtime call failed                            */
#define CCSD_K_ESTATE (-4)     /* call out of order (e.g. before bind) or after EDEVICE */
#define CCSD_K_ENUMERIC (-5)   /* non-finite residual norm or energy                   */

#define CCSD_K_PREC_FP64 0  /* complex128 storage, FP64 MFMA contractions            */
#define CCSD_K_PREC_MIXED 1 /* complex64 operands of the big contractions, split-BF16
                               MFMA products accumulated in FP32; the integral classes
                               are kept in complex64 only (rounded from the complex128
                               values given or generated), R2 and the DIIS error vectors
                               are stored in complex64; FP64 master amplitudes and DIIS
                               amplitude history, denominators, F intermediates, norm and
                               energy sums                                              */

/* Grouping of the hole-hole terms of the T2 equation.  STANDARD: Sec. 2 (eq. ori_EqDouble)
 * with W_mnij built once from tau and applied once, 1/2 tau_mn^ab W_mnij.  REARRANGED (FP64
 * path): the grouping of Sec. 3.3.4 (eqs. A_3rd, def_X, and the t2 Y-tilde_{mnij} term of
 * eq. A_4th with def_Y_oo): X-tilde = t2 <mn||ef>, then 1/4 t2 X-tilde and t2 Y-tilde as
 * two separate products, tau's single-amplitude part of the hole-hole ladder as a small
 * contraction; one more N_k^4 n_occ^4 n_vir^2 product than STANDARD, same result. */
#define CCSD_K_GROUPING_STANDARD 0
#define CCSD_K_GROUPING_REARRANGED 1

typedef struct ccsd_k_ctx ccsd_k_ctx;

typedef struct {
    int32_t grid[3];    /* k mesh, each >= 1; N_k = grid[0]*grid[1]*grid[2]              */
    int32_t n_occ;      /* occupied spin orbitals per k, >= 1                           */
    int32_t n_vir;      /* virtual spin orbitals per k, >= 1                            */
    int32_t precision;  /* CCSD_K_PREC_FP64 or CCSD_K_PREC_MIXED                         */
    int32_t diis_space; /* 0: plain successive substitution; 2..16: Pulay DIIS depth     */
    int32_t synthetic;  /* 1: bind fills Fock and integrals on the device from
                           (seed, eri_scale) by the seeded recipe; 0: ccsd_k_set_inputs  */
    uint64_t seed;
    double eri_scale;   /* scale of the raw complex Gaussians of the synthetic recipe   */
    int32_t grouping;   /* CCSD_K_GROUPING_STANDARD or (FP64 path) _REARRANGED            */
} ccsd_k_system;

/* Plan n_sys independent systems (1..4096), each with N_k <= 512.  hip_stream: a
 * hipStream_t, or NULL for the default stream.  Validates sizes; allocates host memory only.  On failure *out is NULL
 * and ccsd_k_last_error(NULL) holds the reason. */
int ccsd_k_init(const ccsd_k_system *sys, int32_t n_sys, void *hip_stream, ccsd_k_ctx **out);

/* Device workspace, in bytes, that ccsd_k_bind_workspace needs. */
int ccsd_k_workspace_bytes(const ccsd_k_ctx *ctx, uint64_t *bytes);

/* Hand the context a device buffer of at least ccsd_k_workspace_bytes bytes (256-byte
 * aligned).  Uploads the momentum and contraction tables, generates synthetic inputs
 * where requested, and sets every amplitude to zero.  ENOMEM if bytes is too small. */
int ccsd_k_bind_workspace(ccsd_k_ctx *ctx, void *device_ptr, uint64_t bytes);

/* Copy one system's Fock matrix and integral classes from host memory (layouts above;
 * the mixed path rounds the classes to its complex64 copies, passing them through a
 * device staging buffer a range at a time).  EINVAL when an orbital energy (real part of a Fock diagonal element) is not finite or
 * when a T1 or T2 denominator of the update (Sec. 4.4) is zero.  Resets the system's DIIS
 * history. */
int ccsd_k_set_inputs(ccsd_k_ctx *ctx, int32_t sys, const double *fock, const double *const eri[6]);

/* One evaluation of (R1, R2) (eqs. ori_EqSingle, ori_EqDouble) for system sys.
 * t1/t2: host amplitudes to evaluate at (they become the system's current amplitudes);
 * NULL = the current device amplitudes; passing either resets the system's DIIS history.  r1/r2: host buffers for the result, or NULL to
 * keep it on the device only (complex128; on the mixed path r2 is held in complex64 and
 * widened on the copy).  t2 must be antisymmetric, t_{ij}^{ab} = -t_{ji}^{ab} =
 * -t_{ij}^{ba} (with the momenta exchanged alike), as every CCSD amplitude is: several
 * terms of the T2 equation are combined under one P(ij)P(ab) using that symmetry, so for
 * other input the result differs from the equation by terms that vanish on antisymmetric
 * amplitudes.  Amplitudes produced by ccsd_k_iterate keep the symmetry. */
int ccsd_k_residual(ccsd_k_ctx *ctx, int32_t sys, const double *t1, const double *t2, double *r1,
                    double *r2);

/* Iterate every unconverged system: each iteration evaluates R, its 2-norm over all
 * stored elements of (R1, R2) and, if the norm is >= tol, applies t <- t + D^-1 R (then
 * DIIS when diis_space > 0).  Stops when every system has ||R|| < tol or after max_iter
 * residual evaluations.  *iters: evaluations done (max over systems); *max_rnorm: largest
 * last norm.  Returns CCSD_K_NOT_CONVERGED if some system did not converge.  With more than one
 * system active, the systems run side by side on eight internal streams (default priority,
 * created on the first such call, destroyed by ccsd_k_free), ordered after the work already
 * on the context's stream and joined back into it before each host synchronization; each
 * system's results do not depend on this. */
int ccsd_k_iterate(ccsd_k_ctx *ctx, int32_t max_iter, double tol, int32_t *iters, double *max_rnorm);

/* Last residual 2-norm of system sys (after ccsd_k_residual or ccsd_k_iterate). */
int ccsd_k_residual_norm(ccsd_k_ctx *ctx, int32_t sys, double *rnorm);

/* Correlation energy (supercell total, no 1/N_k) at the current amplitudes, FP64. */
int ccsd_k_energy(ccsd_k_ctx *ctx, int32_t sys, double *e_re, double *e_im);

/* Copy the current (FP64 master) amplitudes out / in (checkpoint and restart). */
int ccsd_k_get_amplitudes(ccsd_k_ctx *ctx, int32_t sys, double *t1, double *t2);
int ccsd_k_set_amplitudes(ccsd_k_ctx *ctx, int32_t sys, const double *t1, const double *t2);

/* Algorithmic work of one residual evaluation of system sys: real flops of the five
 * grouped products (8 per complex multiply-add) and of all other terms. */
int ccsd_k_flops(const ccsd_k_ctx *ctx, int32_t sys, double *gemm_flops, double *other_flops);

/* Shape of one grouped complex product as executed for system sys: G groups of an
 * M x N x K product each (complex elements).  product: 0 particle-particle ladder,
 * 1 hole-hole ladder, 2 W_mnij build, 3 W_mbej build, 4 ring product (the numbering of
 * ccsd_k_timing_get).  In the mixed path the three ladder-family products run on
 * canonical antisymmetric pairs (M, N and K of the full form each roughly halved), so the
 * executed shape is smaller than the algorithmic one counted by ccsd_k_flops, and the
 * hole-hole ladder runs inside the particle-particle product (its k pairs appended), so
 * product 1 reports a zero shape and product 0 the combined one.  Any output pointer may
 * be NULL. */
int ccsd_k_product_shape(const ccsd_k_ctx *ctx, int32_t sys, int32_t product, int64_t *G, int64_t *M, int64_t *N,
                         int64_t *K);

/* Arithmetic forms of a grouped product of a mixed-precision system.  The operands of a
 * product are stored in 8 bytes per complex element, either split (four bf16 values, the
 * high and low halves of the real and imaginary parts) or as complex64; products accumulate
 * in FP32 and add their result to FP64 (or complex64 / split) outputs.
 *   SPLIT2_PRESPLIT  split storage, each real product hi*hi + hi*lo + lo*hi on bf16 MFMA
 *                    (about 2^-16 relative per product; the default);
 *   SPLIT2           the same arithmetic on complex64 storage, split in registers;
 *   SPLIT3           complex64 storage split into three bf16 terms, six bf16 MFMA products
 *                    per real product (every term down to 2^-16 of |x||y| kept, about FP32
 *                    accuracy);
 *   FP32             complex64 storage, FP32 MFMA.
 * The ladder family (products 0 and 2) and the ring family (products 3 and 4) each keep
 * one storage: complex64 as soon as one product of the family takes a complex64 form, and a
 * SPLIT2_PRESPLIT product of such a family runs as SPLIT2.  (The precision pattern of the
 * paper's contractions, Sec. 4.3.4, is not fixed by the paper; these forms are ours.) */
#define CCSD_K_FORM_SPLIT2_PRESPLIT 0
#define CCSD_K_FORM_SPLIT2 1
#define CCSD_K_FORM_SPLIT3 2
#define CCSD_K_FORM_FP32 3

/* Set / read the arithmetic form of product (numbering of ccsd_k_timing_get: 0 the
 * particle-particle ladder, which carries the hole-hole ladder too on this path, 2 W_mnij,
 * 3 W_mbej, 4 ring) of mixed-precision system sys.  EINVAL for an FP64 system, product 1 or
 * an unknown form.  A change of a family's storage converts its static operands again. */
int ccsd_k_set_product_form(ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t form);
int ccsd_k_get_product_form(const ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t *form);

/* Tile shapes of the FP64 products (complex outputs per 256-thread workgroup, rows x
 * columns).  Every shape takes the same k stages and the same order of MFMA operations
 * along k for each output element, so all of them give bitwise the same result; they trade
 * data reuse per workgroup against the number of workgroups. */
#define CCSD_K_TILE_32X32 0 /* the initial shape of a product with few 64 x 64 tiles */
#define CCSD_K_TILE_64X64 1 /* the initial shape otherwise */
#define CCSD_K_TILE_128X64 2
#define CCSD_K_TILE_64X128 3

/* Set / read the tile shape of product (0..4, numbering of ccsd_k_timing_get) of FP64
 * system sys.  EINVAL for a mixed-precision system (its products have one tile shape) or an
 * unknown tile.  A product starts in 32 x 32 tiles while 64 x 64 ones would give fewer than
 * 4096 workgroups, in 64 x 64 tiles otherwise.  The products of the rearranged hole-hole
 * grouping other than these five run in 64 x 64 tiles. */
int ccsd_k_set_product_tile(ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t tile);
int ccsd_k_get_product_tile(const ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t *tile);

/* Autotuner.  Mixed-precision system: choose the form of every product.  For each
 * product it measures every form's average launch time on the system's own operands and
 * tables (the workspace must be bound; the overwritten intermediates are recomputed by the
 * next residual) and every form's error, max|C_form - C_fp64| / max|C_fp64| on seeded
 * operands of the product's K (and up to 256 rows and columns) against the FP64 MFMA kernel.
 * Per family it keeps the faster of the two storages whose products all stay within budget
 * (each product of a complex64 family taking its fastest admissible form); if none does,
 * the most accurate forms.  FP64 system: choose the tile shape of every product, the one
 * with the shortest measured launch time (all shapes give the same result, so budget, which
 * must still be positive, plays no part).  cache_path (NULL: none): a text file of
 * measurements keyed by device and product shape, read before measuring and appended to
 * after.  forms[5] (optional) receives the chosen form per product (-1 for product 1), or
 * the chosen tile shape per product on an FP64 system; report (optional, 5 x 4 x 2 doubles)
 * the measured (ms, error) per product and form, or (ms, 0) per product and tile shape. */
int ccsd_k_autotune(ccsd_k_ctx *ctx, int32_t sys, double budget, const char *cache_path, int32_t *forms,
                    double *report);

/* Graph replay in ccsd_k_iterate (on by default): one iteration of every active system
 * (residual, norm, and the update gated on that norm on the device: plain substitution, or
 * the DIIS update, the DIIS step solved on the device and the extrapolation) is captured
 * once as a HIP graph and replayed, with one copy of the systems' norms to the host per
 * iteration; it is captured again when the active set, a product form or the tolerance
 * changes.  Results are bitwise those of the same work enqueued directly (enable = 0,
 * while stage timing is on, or on a context created with the null stream, which cannot be
 * captured). */
int ccsd_k_set_graphs(ccsd_k_ctx *ctx, int32_t enable);

/* Two streams in a mixed-precision residual (on by default).  When one system is iterated
 * (or evaluated by ccsd_k_residual) on the context's stream, the kernels that do not feed the
 * next grouped product (the X seed of the ring terms, the T1-dressed <ab||ef>, the T1
 * residual of eq. ori_EqSingle) run on a second stream of the library's, ordered by events,
 * beside the W_mbej, ring and ladder products.  Results are bitwise those of
 * enable = 0, under which everything runs on the context's stream in one order.  Off while
 * stage timing is on, so that each product is timed alone; systems iterated together
 * already run side by side and keep one stream each.  Returns CCSD_K_EINVAL on a null
 * context. */
int ccsd_k_set_overlap(ccsd_k_ctx *ctx, int32_t enable);

/* Precision escalation in ccsd_k_iterate (on by default): a mixed-precision system whose
 * residual norm has not halved for three iterations while above the tolerance has reached
 * the rounding floor of its products (two-term split products, FP32 accumulation); its
 * two-term products are then switched to CCSD_K_FORM_SPLIT3 and every product accumulates
 * in FP32 over chunks of 256 k only, the chunks added in FP64; a second such stall
 * shortens the chunks to 64 k.  enable = 0 keeps the forms fixed. */
int ccsd_k_set_escalation(ccsd_k_ctx *ctx, int32_t enable);

/* Per-stage device timing with HIP events on the context's stream (0 = off).  Stages:
 * 0 particle-particle ladder, 1 hole-hole ladder, 2 W_mnij build, 3 ring W build,
 * 4 ring product, 5 the whole residual evaluation (all of the above and every other term).
 * When ccsd_k_iterate runs several systems side by side the events sit on their streams
 * and each interval also counts the time of work from other systems that overlaps it. */
int ccsd_k_timing(ccsd_k_ctx *ctx, int32_t enable);
int ccsd_k_timing_get(ccsd_k_ctx *ctx, int32_t stage, double *total_ms, int64_t *launches);

/* Diagnostic: dense grouped complex product C[g] = A[g] . B[g]^T on the device with the
 * tiled FP64 MFMA kernel (reference = 0), the one-thread-per-element FP64 kernel
 * (reference = 1), the split-BF16 MFMA kernel of the mixed path on pre-split operands
 * (reference = 2), the complex64-operand kernel in one of its arithmetic forms:
 * two-term split-BF16 (3), three-term split-BF16 (4) or FP32 MFMA (5), the same three forms
 * summed over 64-k chunks in FP64 in one launch (23, 24, 25: the form escalated systems
 * use), or the tiled FP64 kernel in tile shape t (reference = 10 + t, t one of
 * CCSD_K_TILE_*).  Host arrays, complex128: A [G][M][K], B [G][N][K], C [G][M][N].
 * Allocates and frees its own device buffers; synchronizes the default stream. */
int ccsd_k_debug_zgemm(int32_t G, int32_t M, int32_t N, int32_t K, const double *A, const double *B,
                       double *C, int32_t reference);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the product of ccsd_k_debug_zgemm,
 * C[g] = A[g] . B[g]^T, on caller-owned DEVICE arrays (complex128, dense row-major:
 * A [G][M][K], B [G][N][K], C [G][M][N]), enqueued on hip_stream (NULL: the default
 * stream) without allocating, copying through the host or synchronizing.  variant: 0 the
 * tiled FP64 MFMA kernel, 2 the split-BF16 MFMA kernel (the kernels of the residual's
 * grouped products; same results as ccsd_k_debug_zgemm with reference = 0 or 2).  The
 * offset tables, a zero block and the split operands live in a fixed per-device array of
 * 64 MiB that the library holds from the first call on a device until the process ends;
 * a product needing more (8 bytes per table entry, G (2M + 2N + K) entries, plus 8 bytes
 * per operand element for variant 2) is rejected with EINVAL.  Calls on one GPU share that
 * array: calls that overlap in time (other streams or threads) race and must be ordered by
 * the caller.  Errors: EINVAL (bad or too large sizes, null pointers; reason in
 * ccsd_k_last_error(NULL)), EDEVICE (a launch failed). */
int ccsd_k_zgemm_noalloc(int32_t G, int32_t M, int32_t N, int32_t K, const double *A, const double *B,
                         double *C, int32_t variant, void *hip_stream);

/* Release host state; the caller frees the workspace afterwards. NULL is ignored. */
void ccsd_k_free(ccsd_k_ctx *ctx);

/* Description of the last failure of ctx (or of ccsd_k_init when ctx is NULL). */
const char *ccsd_k_last_error(const ccsd_k_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* CCSD_K_H */
