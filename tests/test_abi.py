"""Host-side checks of libccsdk that need no GPU: exported symbols, argument validation,
workspace planning and the algorithmic work count."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccsd_k.h")

ck = pytest.importorskip("paper_1911_00242_amd", reason="libccsdk.so not built")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ccsd_k_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(ck.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ck.SYMBOLS)


def test_system_struct_layout_matches_header():
    assert ctypes.sizeof(ck.ccsd_k_system) == 56
    assert ck.ccsd_k_system.seed.offset == 32
    assert ck.ccsd_k_system.eri_scale.offset == 40
    assert ck.ccsd_k_system.grouping.offset == 48


@pytest.mark.parametrize("bad", [
    dict(grid=(0, 1, 1), no=2, nv=2),
    dict(grid=(2, 1, 1), no=0, nv=2),
    dict(grid=(2, 1, 1), no=2, nv=2, precision=7),
    dict(grid=(2, 1, 1), no=2, nv=2, diis_space=1),
    dict(grid=(2, 1, 1), no=2, nv=2, synthetic=1, eri_scale=-1.0),
    dict(grid=(2, 1, 1), no=2, nv=2, grouping=2),
    dict(grid=(2, 1, 1), no=2, nv=2, grouping=1, precision=1),
])
def test_init_rejects_bad_descriptions(bad):
    with pytest.raises(ck.CcsdKError) as e:
        ck.ccsd_k_init([bad])
    assert e.value.code == ck.EINVAL
    assert ck.ccsd_k_last_error(None)


def test_calls_before_bind_are_refused():
    ctx = ck.ccsd_k_init([dict(grid=(2, 1, 1), no=2, nv=3)])
    try:
        with pytest.raises(ck.CcsdKError) as e:
            ck.ccsd_k_residual(ctx, 0)
        assert e.value.code == ck.ESTATE
        with pytest.raises(ck.CcsdKError) as e:
            ck.ccsd_k_energy(ctx, 0)
        assert e.value.code == ck.ESTATE
    finally:
        ck.ccsd_k_free(ctx)


def test_workspace_and_flops_scale_as_planned():
    sizes = []
    for N1 in (1, 2, 3):
        ctx = ck.ccsd_k_init([dict(grid=(N1, 1, 1), no=4, nv=8, diis_space=6)])
        try:
            sizes.append(ck.ccsd_k_workspace_bytes(ctx))
            g, o = ck.ccsd_k_flops(ctx, 0)
        finally:
            ck.ccsd_k_free(ctx)
        N, no, nv = N1, 4, 8
        macs = N**4 * (no**2 * nv**4 + 2 * no**4 * nv**2 + 2 * no**3 * nv**3)
        assert g == 8.0 * macs
        assert o > 0
    # at least every stored integral class and the T2-sized buffers fit
    N, no, nv = 3, 4, 8
    n = no + nv
    floor = 16 * (N**3 * (no**4 + no**3 * nv + 2 * no**2 * nv**2 + no * nv**3 + nv**4) + 4 * N**3 * no**2 * nv**2)
    assert sizes[2] >= floor
    assert sizes[0] < sizes[1] < sizes[2]


def test_batch_plan_sums_systems():
    a = ck.ccsd_k_init([dict(grid=(2, 1, 1), no=2, nv=4)])
    b = ck.ccsd_k_init([dict(grid=(3, 1, 1), no=3, nv=5)])
    ab = ck.ccsd_k_init([dict(grid=(2, 1, 1), no=2, nv=4), dict(grid=(3, 1, 1), no=3, nv=5)])
    try:
        sa, sb, sab = (ck.ccsd_k_workspace_bytes(x) for x in (a, b, ab))
        assert abs(sab - (sa + sb)) < 1 << 16
    finally:
        for x in (a, b, ab):
            ck.ccsd_k_free(x)


def _canonical_pairs(grid, w):
    """Canonical pairs (kx, x) < (ky, y), ky = K - kx, of every group K, counted directly."""
    import itertools

    import numpy as np

    from oracle import ccsd_k as O

    kc = O.kconserv(grid)
    N = int(np.prod(grid))
    counts = []
    for K in range(N):
        n = 0
        for kx in range(N):
            ky = kc[K, 0, kx]
            for x, y in itertools.product(range(w), range(w)):
                n += (kx, x) < (ky, y)
        counts.append(n)
    return counts


@pytest.mark.parametrize("grid,no,nv", [((3, 3, 3), 8, 16), ((2, 2, 2), 4, 8), ((2, 1, 1), 3, 5)])
def test_product_shapes(grid, no, nv):
    """FP64: the full grouped products; mixed: the ladder family on canonical pairs padded
    to a multiple of 16 in rows, columns and k (an eighth of the work), the two ladders as
    one product, the ring family in full."""
    N = grid[0] * grid[1] * grid[2]
    pv = -(-max(_canonical_pairs(grid, nv)) // 16) * 16
    po = -(-max(_canonical_pairs(grid, no)) // 16) * 16
    full = {0: (N, N * no * no, N * nv * nv, N * nv * nv), 1: (N, N * no * no, N * nv * nv, N * no * no),
            2: (N, N * no * no, N * no * no, N * nv * nv), 3: (N, N * no * nv, N * no * nv, N * no * nv),
            4: (N, N * no * nv, N * no * nv, N * no * nv)}
    packed = dict(full)
    packed[0] = (N, po, pv, pv + po)  # both ladders in one product
    packed[1] = (0, 0, 0, 0)
    packed[2] = (N, po, po, pv)
    for prec, want in ((ck.PREC_FP64, full), (ck.PREC_MIXED, packed)):
        ctx = ck.ccsd_k_init([dict(grid=grid, no=no, nv=nv, precision=prec)], None)
        try:
            for p in range(5):
                assert ck.ccsd_k_product_shape(ctx, 0, p) == want[p], (prec, p)
        finally:
            ck.ccsd_k_free(ctx)
