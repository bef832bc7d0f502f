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
                                        ((2, 1, 1), 5, 23), ((1, 1, 1), 12, 20)])
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
