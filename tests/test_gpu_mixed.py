"""GPU checks of the mixed-precision path (split-BF16 products, FP32 accumulation, FP64
master amplitudes / update / energy / DIIS) against the FP64 oracle.

Error model: a split-BF16 operand carries 16 significant bits (|x - hi - lo| <= 2^-17 |x|)
and a real product drops the lo*lo term, so one product is off by at most ~3 * 2^-17 of
|x||y|; FP32 accumulation adds ~2^-24 per step.  The bound used below for a product
C = sum_k A_k B_k is 4e-5 * sum_k |A_k||B_k| (about 5 * 2^-17), elementwise.
"""
import numpy as np
import pytest

import synth
from oracle import ccsd_k as O

pytestmark = pytest.mark.gpu

ck = pytest.importorskip("paper_1911_00242_amd", reason="libccsdk.so not built")


@pytest.mark.parametrize("G,M,N,K", [(1, 32, 32, 16), (2, 128, 128, 64), (3, 37, 45, 29), (2, 130, 200, 72),
                                     (1, 256, 130, 8), (2, 5, 3, 0)])
def test_split_zgemm_error_bound(G, M, N, K):
    print(f"split zgemm G={G} M={M} N={N} K={K}", flush=True)
    rng = np.random.default_rng(G * 7 + M + N + K)
    A = rng.standard_normal((G, M, K)) + 1j * rng.standard_normal((G, M, K))
    B = rng.standard_normal((G, N, K)) + 1j * rng.standard_normal((G, N, K))
    ref = np.einsum("gmk,gnk->gmn", A, B)
    bound = np.einsum("gmk,gnk->gmn", np.abs(A), np.abs(B))
    C = ck.ccsd_k_debug_zgemm(A, B, reference=2)
    err = np.abs(C - ref)
    assert np.all(err <= 4e-5 * bound + 1e-30)
    if K:
        # not exact: the split path really ran
        assert err.max() > 0


@pytest.mark.parametrize("grid,no,nv", [((2, 1, 1), 4, 8), ((3, 1, 1), 2, 3), ((2, 2, 1), 3, 5),
                                        ((2, 2, 2), 8, 16), ((2, 1, 1), 10, 3), ((1, 1, 1), 2, 34),
                                        ((2, 1, 1), 5, 23), ((1, 1, 1), 12, 20), ((3, 1, 1), 1, 1),
                                        ((1, 1, 1), 17, 2), ((2, 1, 1), 12, 32), ((3, 1, 1), 9, 17)])
def test_mixed_residual_close_to_oracle(grid, no, nv):
    print(f"mixed residual grid={grid} no={no} nv={nv}", flush=True)
    N = int(np.prod(grid))
    kc = O.kconserv(grid)
    f, eris = synth.system(404 + N, grid, no, nv, scale=0.05 / N)
    t1, t2 = synth.test_amplitudes(31 + N, grid, no, nv, scale=0.05)
    R1, R2 = O.residual(f, eris, t1, t2, kc)
    with ck.Context([dict(grid=grid, no=no, nv=nv, precision=ck.PREC_MIXED)]) as c:
        c.set_inputs(0, f, eris)
        g1, g2 = c.residual(0, t1, t2)
    # relative to the largest residual element; every product term is O(|R|) here.  A split
    # product is exact to about 3 * 2^-17 of |x||y| per term and the terms largely cancel
    # in sign, so the residual error sits near 1e-7 of max|R| (observed 5e-8 to 3e-7)
    e2 = np.abs(g2 - R2).max() / np.abs(R2).max()
    e1 = np.abs(g1 - R1).max() / np.abs(R1).max()
    print(f"  max rel err R2 {e2:.2e} R1 {e1:.2e}")
    assert e2 <= 1e-5 and e1 <= 1e-5
    assert e2 > 0  # the bf16 path really ran


@pytest.mark.parametrize("grid,no,nv", [((3, 1, 1), 4, 8), ((2, 1, 1), 8, 16)])
def test_mixed_converged_energy_matches_fp64(grid, no, nv):
    """Converge both paths on a small system (1/N_k-scaled integrals); the mixed fixed
    point differs from the FP64 one by the product error only.  8 x 16 is the workload's
    block shape, whose DIIS update and extrapolation take their constant-shape forms."""
    N = grid[0] * grid[1] * grid[2]
    f, eris = synth.system(505, grid, no, nv, scale=0.05 / N)
    ref = O.solve(f, eris, grid, max_iter=60, tol=1e-11, diis_space=6)
    assert ref["converged"]
    out = {}
    for prec in (ck.PREC_FP64, ck.PREC_MIXED):
        with ck.Context([dict(grid=grid, no=no, nv=nv, precision=prec, diis_space=6)]) as c:
            c.set_inputs(0, f, eris)
            rc, it, rn = c.iterate(60, 1e-11 if prec == ck.PREC_FP64 else 1e-9)
            out[prec] = (rc, c.energy(0), c.get_amplitudes(0)[1])
    assert out[ck.PREC_FP64][0] == ck.OK
    assert abs(out[ck.PREC_FP64][1] - ref["energy"]) <= 1e-11
    de = abs(out[ck.PREC_MIXED][1] - ref["energy"])
    dt2 = np.abs(out[ck.PREC_MIXED][2] - ref["t2"]).max()
    print(f"mixed: |dE| = {de:.3e} Eh, max|dT2| = {dt2:.3e}, E = {ref['energy']}")
    assert de <= 1e-8  # the bar on converged mixed-precision energies, absolute
    assert dt2 <= 1e-6


def test_mixed_energy_error_split_into_storage_and_arithmetic():
    """The mixed path keeps its integral classes in complex64.  Its converged energy is
    compared twice with the FP64 path: on the original integrals (the whole error) and on
    the same integrals rounded to complex64 (the error of the split products alone); the
    difference of the two FP64 energies is the part the complex64 storage contributes."""
    grid, no, nv = (2, 1, 1), 8, 16
    N = 2
    f, eris = synth.system(515, grid, no, nv, scale=0.05 / N)
    rounded = {k: v.astype(np.complex64).astype(np.complex128) for k, v in eris.items()}
    e = {}
    for name, prec, ints, tol in (("fp64", ck.PREC_FP64, eris, 1e-11), ("fp64_c64ints", ck.PREC_FP64, rounded, 1e-11),
                                  ("mixed", ck.PREC_MIXED, eris, 1e-7)):
        with ck.Context([dict(grid=grid, no=no, nv=nv, precision=prec, diis_space=6)]) as c:
            c.set_inputs(0, f, ints)
            rc, it, rn = c.iterate(60, tol)
            assert rc == ck.OK, name
            e[name] = c.energy(0)
    whole = abs(e["mixed"] - e["fp64"])
    arith = abs(e["mixed"] - e["fp64_c64ints"])
    storage = abs(e["fp64_c64ints"] - e["fp64"])
    print(f"mixed vs FP64: {whole:.2e} Eh; vs FP64 on complex64 integrals: {arith:.2e} Eh; "
          f"storage part: {storage:.2e} Eh", flush=True)
    assert whole <= 1e-8 and arith <= 1e-8
    # rounding the integrals moves the FP64 energy by about 2^-24 of the correlation energy
    assert storage <= 1e-7 * abs(e["fp64"])


@pytest.mark.parametrize("grid,no,nv", [((2, 2, 1), 3, 5), ((2, 1, 1), 8, 16)])
def test_mixed_extrapolation_caches_match_fresh_passes(grid, no, nv):
    """The mixed DIIS extrapolation also writes the split copy of t2 and the energy partial
    sums; the residual and energy taken from them equal the ones from fresh passes over the
    same amplitudes (residual bitwise, energy to rounding)."""
    N = grid[0] * grid[1] * grid[2]
    f, eris = synth.system(606, grid, no, nv, scale=0.05 / N)
    with ck.Context([dict(grid=grid, no=no, nv=nv, precision=ck.PREC_MIXED, diis_space=4)]) as c:
        c.set_inputs(0, f, eris)
        c.iterate(5, 0.0)  # several extrapolations
        e_cached = c.energy(0)
        r1a, r2a = c.residual(0)  # split t2 from the extrapolation
        t1, t2 = c.get_amplitudes(0)
        c.set_amplitudes(0, t1, t2)  # invalidates both
        e_fresh = c.energy(0)
        r1b, r2b = c.residual(0)
    assert abs(e_cached - e_fresh) <= 1e-12 * abs(e_fresh)
    assert np.array_equal(r2a, r2b)
    assert np.array_equal(r1a, r1b)


# complex64-operand product forms: the operands are rounded to complex64 (2^-24 relative),
# then split in registers.  Two terms: as the pre-split kernel (4e-5 of sum |A||B|).  Three
# terms and FP32 MFMA: about FP32 accuracy, bound 2e-6 of sum |A||B| (storage rounding of
# both operands, the dropped 2^-24 terms, FP32 accumulation over K <= 256 steps).
@pytest.mark.parametrize("form,bound", [(3, 4e-5), (4, 2e-6), (5, 2e-6)])
@pytest.mark.parametrize("G,M,N,K", [(1, 32, 32, 16), (2, 128, 128, 64), (3, 37, 45, 29), (2, 130, 200, 72),
                                     (1, 256, 130, 8), (2, 5, 3, 0)])
def test_c64_zgemm_error_bound(form, bound, G, M, N, K):
    print(f"c64 zgemm form={form} G={G} M={M} N={N} K={K}", flush=True)
    rng = np.random.default_rng(G * 7 + M + N + K + form)
    A = rng.standard_normal((G, M, K)) + 1j * rng.standard_normal((G, M, K))
    B = rng.standard_normal((G, N, K)) + 1j * rng.standard_normal((G, N, K))
    ref = np.einsum("gmk,gnk->gmn", A, B)
    absb = np.einsum("gmk,gnk->gmn", np.abs(A), np.abs(B))
    C = ck.ccsd_k_debug_zgemm(A, B, reference=form)
    err = np.abs(C - ref)
    assert np.all(err <= bound * absb + 1e-30)
    if K:
        assert err.max() > 0


# The same forms summed over 64-k chunks in FP64 in one launch (64 x 64 tiles; the form of
# escalated systems): the same bounds, and on a long k range the chunked three-term split and
# FP32 MFMA are more accurate than the unchunked ones (FP32 accumulation spans 4 steps).
@pytest.mark.parametrize("form,bound", [(23, 4e-5), (24, 2e-6), (25, 2e-6)])
@pytest.mark.parametrize("G,M,N,K", [(1, 32, 32, 16), (2, 128, 128, 64), (3, 37, 45, 29), (2, 130, 200, 300),
                                     (1, 256, 130, 8), (1, 65, 70, 1000), (2, 5, 3, 0)])
def test_c64_chunked_zgemm_error_bound(form, bound, G, M, N, K):
    print(f"c64 chunked zgemm form={form} G={G} M={M} N={N} K={K}", flush=True)
    rng = np.random.default_rng(G * 11 + M + N + K + form)
    A = rng.standard_normal((G, M, K)) + 1j * rng.standard_normal((G, M, K))
    B = rng.standard_normal((G, N, K)) + 1j * rng.standard_normal((G, N, K))
    ref = np.einsum("gmk,gnk->gmn", A, B)
    absb = np.einsum("gmk,gnk->gmn", np.abs(A), np.abs(B))
    C = ck.ccsd_k_debug_zgemm(A, B, reference=form)
    err = np.abs(C - ref)
    assert np.all(err <= bound * absb + 1e-30)
    if K:
        assert err.max() > 0


def test_c64_chunked_beats_unchunked_on_long_k():
    rng = np.random.default_rng(5)
    K = 4096
    A = rng.standard_normal((1, 96, K)) + 1j * rng.standard_normal((1, 96, K))
    B = rng.standard_normal((1, 80, K)) + 1j * rng.standard_normal((1, 80, K))
    ref = np.einsum("gmk,gnk->gmn", A, B)
    for plain, chunked in ((4, 24), (5, 25)):
        e0 = np.abs(ck.ccsd_k_debug_zgemm(A, B, reference=plain) - ref).max()
        e1 = np.abs(ck.ccsd_k_debug_zgemm(A, B, reference=chunked) - ref).max()
        print(f"form {plain}: unchunked {e0:.2e}, chunked {e1:.2e}", flush=True)
        assert e1 < e0


def test_c64_split3_beats_split2():
    """The three-term split is far more accurate than the two-term one on the same data."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((2, 128, 256)) + 1j * rng.standard_normal((2, 128, 256))
    B = rng.standard_normal((2, 96, 256)) + 1j * rng.standard_normal((2, 96, 256))
    ref = np.einsum("gmk,gnk->gmn", A, B)
    e2 = np.abs(ck.ccsd_k_debug_zgemm(A, B, reference=3) - ref).max()
    e3 = np.abs(ck.ccsd_k_debug_zgemm(A, B, reference=4) - ref).max()
    ef = np.abs(ck.ccsd_k_debug_zgemm(A, B, reference=5) - ref).max()
    print(f"max err split2 {e2:.2e} split3 {e3:.2e} fp32 {ef:.2e}")
    # beyond the two-term split's 2^-16 products, FP32 accumulation over K = 256 steps
    # (~2^-24 sqrt(K) of the running sum) limits both exact-product forms
    assert e3 < e2 / 4 and ef < e2 / 4


# ------------------------------------------------------------------ arithmetic forms
FORM_BARS = {ck.FORM_SPLIT2: 1e-5, ck.FORM_SPLIT3: 2e-6, ck.FORM_FP32: 2e-6}
PRODUCTS = ("pp_ladder", "w_mnij", "w_mbej", "ring")


@pytest.mark.parametrize("form", [ck.FORM_SPLIT2, ck.FORM_SPLIT3, ck.FORM_FP32])
@pytest.mark.parametrize("grid,no,nv", [((2, 1, 1), 8, 16), ((3, 3, 1), 3, 5), ((2, 1, 1), 5, 23)])
def test_forms_residual_close_to_oracle(form, grid, no, nv):
    """Every product in one arithmetic form on complex64 storage: the residual against the
    oracle.  The three-term split and FP32 MFMA leave the error of the complex64 storage of
    the side terms and of R2 (about 2^-24 of each element, ~1e-7 of max|R|)."""
    print(f"forms residual form={form} grid={grid} no={no} nv={nv}", flush=True)
    N = int(np.prod(grid))
    kc = O.kconserv(grid)
    f, eris = synth.system(414 + N, grid, no, nv, scale=0.05 / N)
    t1, t2 = synth.test_amplitudes(41 + N, grid, no, nv, scale=0.05)
    R1, R2 = O.residual(f, eris, t1, t2, kc)
    with ck.Context([dict(grid=grid, no=no, nv=nv, precision=ck.PREC_MIXED)]) as c:
        c.set_inputs(0, f, eris)
        for p in PRODUCTS:
            c.set_product_form(p, form)
        assert [c.product_form(p) for p in PRODUCTS] == [form] * 4
        g1, g2 = c.residual(0, t1, t2)
    e2 = np.abs(g2 - R2).max() / np.abs(R2).max()
    e1 = np.abs(g1 - R1).max() / np.abs(R1).max()
    print(f"  max rel err R2 {e2:.2e} R1 {e1:.2e}", flush=True)
    assert e2 <= FORM_BARS[form] and e1 <= FORM_BARS[form]


def test_families_in_different_storages():
    """Ladder family on split storage, ring family on complex64 (three-term split), and the
    other way round: both match the oracle."""
    grid, no, nv = (3, 1, 1), 4, 8
    kc = O.kconserv(grid)
    f, eris = synth.system(515, grid, no, nv, scale=0.05 / 3)
    t1, t2 = synth.test_amplitudes(52, grid, no, nv, scale=0.05)
    R1, R2 = O.residual(f, eris, t1, t2, kc)
    for lad, ring in ((ck.FORM_SPLIT2_PRESPLIT, ck.FORM_SPLIT3), (ck.FORM_FP32, ck.FORM_SPLIT2_PRESPLIT)):
        with ck.Context([dict(grid=grid, no=no, nv=nv, precision=ck.PREC_MIXED)]) as c:
            c.set_inputs(0, f, eris)
            c.set_product_form("pp_ladder", lad)
            c.set_product_form("w_mnij", lad)
            c.set_product_form("w_mbej", ring)
            c.set_product_form("ring", ring)
            g1, g2 = c.residual(0, t1, t2)
        e2 = np.abs(g2 - R2).max() / np.abs(R2).max()
        print(f"ladder form {lad}, ring form {ring}: max rel err R2 {e2:.2e}", flush=True)
        assert e2 <= 1e-5


@pytest.mark.parametrize("grid,no,nv", [((2, 1, 1), 8, 16), ((3, 1, 1), 5, 7)])
def test_autotune_budgets_and_cache(tmp_path, grid, no, nv):
    """A loose budget admits the pre-split two-term form, a tight one only the three-term
    split or FP32; the second call with the same cache measures nothing new; the residual
    after tuning (whose timing runs overwrite intermediates) still matches the oracle.  On
    the 3x1x1 mesh with 5 x 7 orbitals the canonical pair counts per momentum group (35
    occupied, 70 virtual) are not multiples of 8, so the padding of the packed operands
    shares 64-byte chunks with real elements, which the timing runs of the other storage
    write."""
    kc = O.kconserv(grid)
    N = int(np.prod(grid))
    f, eris = synth.system(616, grid, no, nv, scale=0.05 / N)
    t1, t2 = synth.test_amplitudes(61, grid, no, nv, scale=0.05)
    R1, R2 = O.residual(f, eris, t1, t2, kc)
    cache = str(tmp_path / "tune.txt")
    with ck.Context([dict(grid=grid, no=no, nv=nv, precision=ck.PREC_MIXED, diis_space=4)]) as c:
        c.set_inputs(0, f, eris)
        c.residual(0, t1, t2)
        forms, rep = c.autotune(1e-2, cache)
        print("budget 1e-2:", forms, "\n", rep[[0, 2, 3, 4]], flush=True)
        assert forms[1] == -1
        for p in (0, 2, 3, 4):
            assert rep[p, :, 0].min() > 0  # every form timed
            assert rep[p, 0, 1] < 1e-3  # the two-term split: ~1e-5
            assert rep[p, 2, 1] < 1e-5 and rep[p, 3, 1] < 1e-5  # three-term / FP32: ~1e-7
        lines = open(cache).read().splitlines()
        shapes = {c.product_shape(p) for p in (0, 2, 3, 4)}
        assert len(lines) == len(shapes)  # one record per product shape
        forms_t, rep_t = c.autotune(1e-6, cache)
        print("budget 1e-6:", forms_t, flush=True)
        assert open(cache).read().splitlines() == lines  # all from the cache
        assert np.allclose(rep_t, rep, rtol=1e-5, atol=0)  # the cache keeps 6 significant digits
        for p in (0, 2, 3, 4):
            assert forms_t[p] in (ck.FORM_SPLIT3, ck.FORM_FP32)
        g1, g2 = c.residual(0, t1, t2)
        assert np.abs(g2 - R2).max() / np.abs(R2).max() <= 2e-6
        # and back to a loose budget: the chosen forms run correctly as well
        c.autotune(1e-2, cache)
        g1, g2 = c.residual(0, t1, t2)
        assert np.abs(g2 - R2).max() / np.abs(R2).max() <= 1e-5


@pytest.mark.parametrize("grid,no,nv", [((3, 1, 1), 5, 7), ((2, 1, 1), 10, 3)])
def test_storage_changes_keep_packed_padding(grid, no, nv):
    """Moving the ladder family from split to complex64 storage and back (as escalation and
    the autotuner do) leaves every residual equal to the oracle's within the mixed bar, on
    shapes whose packed padding shares 64-byte chunks with real pairs; then an iteration
    from the same amplitudes is finite."""
    kc = O.kconserv(grid)
    N = int(np.prod(grid))
    f, eris = synth.system(617, grid, no, nv, scale=0.05 / N)
    t1, t2 = synth.test_amplitudes(62, grid, no, nv, scale=0.05)
    R1, R2 = O.residual(f, eris, t1, t2, kc)
    with ck.Context([dict(grid=grid, no=no, nv=nv, precision=ck.PREC_MIXED, diis_space=4)]) as c:
        c.set_inputs(0, f, eris)
        for forms in ((0, 0), (2, 2), (0, 0), (3, 1), (0, 0)):  # (pp_ladder, w_mnij)
            c.set_product_form(0, forms[0])
            c.set_product_form(2, forms[1])
            g1, g2 = c.residual(0, t1, t2)
            e = np.abs(g2 - R2).max() / np.abs(R2).max()
            print(f"forms {forms}: max rel err R2 {e:.2e}", flush=True)
            assert np.isfinite(g2).all() and e <= 1e-5
        c.set_amplitudes(0, t1, t2)
        rc, it, rn = c.iterate(2, 0.0)
        assert np.isfinite(rn)


@pytest.mark.timeout(600)
def test_strong_coupling_converges_with_escalation():
    """A 2x2x2-mesh system with n_occ=12, n_vir=24 and integrals x 0.05/N_k, the shape whose
    mixed-precision residual stalls near 2e-7, above the mixed tolerance 1e-7 (FP32
    accumulation over up to 2304 k and the two-term split's storage error both set that
    floor; the three-term split alone does not lower it): with precision escalation
    (three-term split, FP32 accumulation over 256-k chunks
    added in FP64, floor near 6e-8) the mixed path converges to 1e-7 and its energy is within
    1e-8 Eh of the FP64 path (which matches the oracle); without escalation it stalls."""
    grid, no, nv = (2, 2, 2), 12, 24
    desc = dict(grid=grid, no=no, nv=nv, diis_space=6, synthetic=1, seed=40017, eri_scale=0.05 / 8)
    with ck.Context([dict(desc, precision=ck.PREC_FP64)]) as c:
        rc, it64, rn = c.iterate(80, 1e-11)
        assert rc == ck.OK
        e64 = c.energy(0)
    with ck.Context([dict(desc, precision=ck.PREC_MIXED)]) as c:
        rc, it, rn = c.iterate(80, 1e-7)
        e = c.energy(0)
        forms = [c.product_form(p) for p in PRODUCTS]
    print(f"FP64 {it64} evaluations, E = {e64}; mixed rc={rc} {it} evaluations |R|={rn:.2e} "
          f"|dE|={abs(e - e64):.2e} forms {forms}", flush=True)
    assert rc == ck.OK
    assert abs(e - e64) <= 1e-8
    assert forms == [ck.FORM_SPLIT3] * 4
    with ck.Context([dict(desc, precision=ck.PREC_MIXED)]) as c:
        c.set_escalation(False)
        rc, it, rn = c.iterate(40, 1e-7)
        print(f"without escalation: rc={rc} |R|={rn:.2e}", flush=True)
    assert rc == ck.NOT_CONVERGED
