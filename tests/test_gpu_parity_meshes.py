"""GPU parity on meshes where k != -k along two or three axes, at amplitudes with t1 != 0.

On 1-D meshes of two points and on 2x2x2 meshes every k equals -k, so a sign mistake in
the momentum arithmetic of an offset or pair table is invisible there.  Here the FP64 and
the mixed-precision paths are compared with the oracle on 3x3x1 and 3x3x3 meshes (momentum
conservation of Sec. 3.2.5 with wrap-around along every axis of length 3), element by
element: R1 in full and R2 on sampled momentum blocks, which include the special cases of
the tau and F terms (k_a = k_i, k_b = k_i, k_i = k_j, the Gamma block).  The oracle side is
the block-restricted oracle (``residual_blocks``), pinned equal to the full oracle.

Bars: FP64 path max|dR| <= 1e-12 max|R|; mixed path max|dR| <= 1e-5 max|R| (one split
product is exact to about 3 * 2^-17 of |x||y|; the observed error is 1e-7 to 3e-7).
"""
import numpy as np
import pytest

import synth
from oracle import ccsd_k as O

pytestmark = pytest.mark.gpu

ck = pytest.importorskip("paper_1911_00242_amd", reason="libccsdk.so not built")

# mesh, n_occ, n_vir; 8 x 16 is the block shape of the N_k=27 workload (constant-shape
# kernels and the packed pair tables of three-point axes)
CASES = [((3, 3, 1), 8, 16), ((3, 3, 1), 3, 5), ((3, 3, 3), 2, 3), ((3, 1, 3), 4, 8)]


def sample_blocks(grid, kc, count=10, seed=5):
    N = int(np.prod(grid))
    rng = np.random.default_rng(seed)
    blocks = {(0, 0, 0), (N - 1, N - 2 if N > 1 else 0, 1 % N)}
    while len(blocks) < count:
        ki, kj, ka = (int(x) for x in rng.integers(0, N, 3))
        blocks.add((ki, kj, ka))
    # special cases: k_a = k_i, k_b = k_i, k_i = k_j
    ki, kj = 1 % N, (N // 2 + 1) % N
    blocks.add((ki, kj, ki))  # k_a = k_i
    blocks.add((ki, kj, kj))  # k_b = k_i + k_j - k_a = k_i
    blocks.add((ki, ki, (ki + 2) % N))  # k_i = k_j
    return sorted(blocks)


def _oracle(grid, no, nv, seed):
    N = int(np.prod(grid))
    kc = O.kconserv(grid)
    f, eris = synth.system(seed, grid, no, nv, scale=0.1 / N)
    t1, t2 = synth.test_amplitudes(seed + 1, grid, no, nv, scale=0.05)
    blocks = sample_blocks(grid, kc)
    R1, R2b = O.residual_blocks(f, eris, t1, t2, kc, blocks)
    return f, eris, t1, t2, kc, blocks, R1, R2b


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0][0]}x{c[0][1]}x{c[0][2]}_{c[1]}x{c[2]}")
def case(request):
    grid, no, nv = request.param
    print(f"mesh parity: oracle grid={grid} no={no} nv={nv}", flush=True)
    return (grid, no, nv) + _oracle(grid, no, nv, seed=900 + no * 10 + nv)


def _compare(case, prec, asym_tol):
    grid, no, nv, f, eris, t1, t2, kc, blocks, R1, R2b = case
    print(f"mesh parity: gpu grid={grid} no={no} nv={nv} precision={prec}", flush=True)
    with ck.Context([dict(grid=grid, no=no, nv=nv, precision=prec)]) as c:
        c.set_inputs(0, f, eris)
        g1, g2 = c.residual(0, t1, t2)
    ref2 = np.stack([R2b[b] for b in blocks])
    got2 = np.stack([g2[b] for b in blocks])
    e2 = float(np.abs(got2 - ref2).max() / np.abs(ref2).max())
    e1 = float(np.abs(g1 - R1).max() / np.abs(R1).max())
    print(f"  max rel err R2 {e2:.2e} R1 {e1:.2e} over {len(blocks)} blocks", flush=True)
    # R2 antisymmetric over the whole array: R(ij,ab) = -R(ji,ab) = -R(ij,ba)
    N = int(np.prod(grid))
    scale = np.abs(g2).max()
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                kb = kc[ki, kj, ka]
                x = g2[ki, kj, ka]
                assert np.abs(x + g2[kj, ki, ka].transpose(1, 0, 2, 3)).max() <= asym_tol * scale
                assert np.abs(x + g2[ki, kj, kb].transpose(0, 1, 3, 2)).max() <= asym_tol * scale
    return e1, e2


def test_fp64_residual_on_meshes(case):
    e1, e2 = _compare(case, ck.PREC_FP64, 1e-12)
    assert e2 <= 1e-12 and e1 <= 1e-12


def test_mixed_residual_on_meshes(case):
    e1, e2 = _compare(case, ck.PREC_MIXED, 1e-6)
    assert e2 <= 1e-5 and e1 <= 1e-5
    assert e2 > 0  # the split path really ran
