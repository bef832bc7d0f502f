"""The largest mesh one GPU holds, N_k=40 (5x4x2), n_occ=8, n_vir=16 per k, on the mixed
path (238 GB of workspace; the FP64 path would need about 450 GB), in its launch
configuration (inputs generated on the device, DIIS(6), the constant-shape kernels).  The
oracle cannot evaluate whole residuals at this size; it checks, block by block:

* the driver term of R2 and R1 at t = 0 (conj(<ij||ab>), conj(f_ia); the mixed path keeps
  its integral classes in complex64, so within their rounding), and the first-order
  amplitudes after one update, t = D^-1 R(0), block by block;
* R2 antisymmetric in (i, j) and in (a, b) on the sampled blocks at seeded amplitudes with
  t1 != 0 (a property of the packed assembly, which writes all four members of an orbit
  from one representative);
* R2 on sampled momentum blocks and R1 at a sampled momentum at those amplitudes against
  the block-restricted oracle (about a minute of host time: its F intermediates read the
  whole <oo||vv> class), within the mixed path's bar of 1e-5 of max|R|, and the energy
  there within 1e-8 Eh."""

import numpy as np
import pytest

import synth
from oracle import ccsd_k as O

ck = pytest.importorskip("paper_1911_00242_amd", reason="libccsdk.so not built")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

GRID, NO, NV, SEED = (5, 4, 2), 8, 16, 404
N = 40
SCALE = 0.05 / N
TSEED, TSCALE = 4343, 0.01  # seeded test amplitudes (t1 != 0)
# sampled momentum blocks (ki, kj, ka): corners, ki = kj, ki = ka, and blocks whose pair
# momenta differ along every axis of the mesh
BLOCKS = [(0, 0, 0), (39, 38, 37), (5, 9, 5), (21, 30, 8)]
R1_KS = [5]


def _log(msg):
    print(f"[N_k=40] {msg}", flush=True)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def run():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.empty_cache()
    out = {}
    _log("mixed path: workspace and device-generated inputs")
    desc = dict(grid=GRID, no=NO, nv=NV, precision=ck.PREC_MIXED, diis_space=6, synthetic=1, seed=SEED,
                eri_scale=SCALE)
    _log("host: seeded amplitudes")
    ta1, ta2 = synth.test_amplitudes(TSEED, GRID, NO, NV, scale=TSCALE)
    with ck.Context([desc], device="cuda:0") as c:
        r1_0, r2_0 = c.residual(0)
        out["r1_0"], out["r2_0"] = r1_0, {b: r2_0[b].copy() for b in BLOCKS}
        del r2_0
        _log("mixed path: residual at t = 0 done")
        c.iterate(1, 0.0)
        t1, t2 = c.get_amplitudes(0)
        out["t1"], out["t2"] = t1, {b: t2[b].copy() for b in BLOCKS}
        del t2
        _log("mixed path: one update done")
        g1, g2 = c.residual(0, ta1, ta2)
        out["r1"], out["r2"] = g1, {b: g2[b].copy() for b in BLOCKS}
        kc = O.kconserv(GRID)
        worst, scale = 0.0, max(np.abs(g2[b]).max() for b in BLOCKS)
        for (ki, kj, ka) in BLOCKS:
            kb = kc[ki, kj, ka]
            x = g2[ki, kj, ka]
            worst = max(worst, np.abs(x + g2[kj, ki, ka].transpose(1, 0, 2, 3)).max(),
                        np.abs(x + g2[ki, kj, kb].transpose(0, 1, 3, 2)).max())
        out["asym"] = worst / scale
        del g2
        out["e"] = c.energy(0)
        _log("mixed path: residual and energy at the seeded amplitudes done")
    torch.cuda.empty_cache()
    out["ta1"], out["ta2"] = ta1, ta2
    return out


def test_driver_term_at_zero_amplitudes(run):
    """R2 = conj(<ij||ab>) and R1 = conj(f_ia) at t = 0, <ij||ab> from its complex64 copy."""
    f = synth.fock(SEED, GRID, NO, NV)
    assert _rel(run["r1_0"], np.conj(f[:, :NO, NO:])) <= 1e-13
    for b in BLOCKS:
        ref = np.conj(synth.eri_block(SEED, GRID, NO, NV, "oovv", *b, scale=SCALE))
        assert _rel(run["r2_0"][b], ref) <= 1e-7, b


def test_first_order_amplitudes(run):
    """One update from t = 0 (Sec. 4.4): t2 = conj(<ij||ab>) / D_ij^ab, t1 = conj(f_ia) / D_i^a."""
    f = synth.fock(SEED, GRID, NO, NV)
    kc = O.kconserv(GRID)
    eo = np.real(np.einsum("kii->ki", f[:, :NO, :NO]))
    ev = np.real(np.einsum("kaa->ka", f[:, NO:, NO:]))
    assert _rel(run["t1"], np.conj(f[:, :NO, NO:]) / (eo[:, :, None] - ev[:, None, :])) <= 1e-13
    for (ki, kj, ka) in BLOCKS:
        kb = kc[ki, kj, ka]
        D = eo[ki][:, None, None, None] + eo[kj][None, :, None, None] - ev[ka][None, None, :, None] - ev[kb][None, None, None, :]
        ref = np.conj(synth.eri_block(SEED, GRID, NO, NV, "oovv", ki, kj, ka, scale=SCALE)) / D
        assert _rel(run["t2"][ki, kj, ka], ref) <= 1e-7, (ki, kj, ka)


def test_residual_antisymmetric(run):
    assert run["asym"] <= 1e-12


def test_residual_and_energy_at_t1_match_oracle(run):
    """Element by element on the sampled blocks against the block-restricted oracle (every
    term of the T2 equation, the T1 dressing and the t1 parts of the W seeds included)."""
    _log("host: generating the <oo||vv> class and the Fock matrix")
    oovv = synth.eri_class(SEED, GRID, NO, NV, "oovv", scale=SCALE)
    f = synth.fock(SEED, GRID, NO, NV)
    kc = O.kconserv(GRID)

    def provider(cls, kp, kq, kr):
        if cls == "oovv":
            return oovv[kp, kq, kr]
        return synth.eri_block(SEED, GRID, NO, NV, cls, kp, kq, kr, scale=SCALE)

    _log("oracle: R1 at the sampled momenta and the sampled R2 blocks")
    R1, R2b = O.residual_blocks(f, O.LazyClasses(provider), run["ta1"], run["ta2"], kc, BLOCKS, r1_ks=R1_KS,
                                callback=lambda step: _log(f"oracle: {step} done"))
    _log("oracle: energy")
    e = O.energy(f, {"oovv": oovv}, run["ta1"], run["ta2"], kc)
    ref = np.stack([R2b[b] for b in BLOCKS])
    got = np.stack([run["r2"][b] for b in BLOCKS])
    print(f"[N_k=40] R2 {_rel(got, ref):.2e}  R1 {_rel(run['r1'][R1_KS], R1[R1_KS]):.2e}  "
          f"|dE| {abs(run['e'] - e):.2e}", flush=True)
    assert _rel(got, ref) <= 1e-5
    assert _rel(run["r1"][R1_KS], R1[R1_KS]) <= 1e-5
    assert abs(run["e"] - e) <= 1e-8
