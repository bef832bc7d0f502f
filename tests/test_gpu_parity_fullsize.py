"""Checks at the full size of the benchmark workload, N_k=27 (3x3x3 mesh), n_occ=8,
n_vir=16 per k, in its launch configuration (inputs generated on the device from the same
seed and scale, DIIS(6), the constant-shape kernels), where the oracle cannot evaluate
whole residuals in reasonable time:

* values the oracle and the host generator reproduce: the driver term of R2 and R1 at
  t = 0 and the first-order amplitudes after one update, block by block; the correlation
  energy of those amplitudes in full (the oracle's energy over the whole <oo||vv> class);
* properties that hold at any size: R2 antisymmetric in (i, j) and in (a, b) at general
  amplitudes, and the mixed-precision path within its error model of the FP64 path at the
  same amplitudes (the FP64 path itself matches the oracle element by element at the
  smaller sizes of the other parity tests, with the same kernels)."""
import numpy as np
import pytest

import synth
from oracle import ccsd_k as O

ck = pytest.importorskip("paper_1911_00242_amd", reason="libccsdk.so not built")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

GRID, NO, NV, SEED = (3, 3, 3), 8, 16, 303
N = 27
SCALE = 0.05 / N
TSEED, TSCALE = 4242, 0.01  # seeded test amplitudes (t1 != 0)
# sampled momentum blocks (ki, kj, ka): corners, the middle, ki = ka and ki = kj cases
BLOCKS = [(0, 0, 0), (1, 2, 3), (26, 25, 24), (5, 9, 5), (13, 13, 13), (7, 20, 11), (4, 4, 17)]
R1_KS = [0, 5, 26]  # R1 momenta compared element by element (k_i of sampled blocks)


def _desc(prec):
    return dict(grid=GRID, no=NO, nv=NV, precision=prec, diis_space=6, synthetic=1, seed=SEED, eri_scale=SCALE)


def _log(msg):
    print(f"[full size] {msg}", flush=True)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def runs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.empty_cache()
    out = {}
    _log("FP64 path: workspace and device-generated inputs")
    with ck.Context([_desc(ck.PREC_FP64)], device="cuda:0") as c:
        r1_0, r2_0 = c.residual(0)
        out["r1_0"] = r1_0
        out["r2_0"] = {b: r2_0[b].copy() for b in BLOCKS}
        del r2_0
        _log("FP64 path: residual at t = 0 done")
        c.iterate(1, 0.0)
        out["t1"], out["t2"] = c.get_amplitudes(0)
        out["e"] = c.energy(0)
        out["r1"], out["r2"] = c.residual(0)
        _log("FP64 path: one update, energy and residual done")
        # seeded amplitudes with t1 != 0 (the synthetic f_ov is zero, so the iteration keeps
        # t1 = 0 and the T1 terms would multiply zeros)
        ta1, ta2 = synth.test_amplitudes(TSEED, GRID, NO, NV, scale=TSCALE)
        g1, g2 = c.residual(0, ta1, ta2)
        out["r1_t"], out["r2_t"] = g1, {b: g2[b].copy() for b in BLOCKS}
        out["r2_t_asym"] = _asym(g2)
        del g2
        out["e_t"] = c.energy(0)
        _log("FP64 path: residual and energy at seeded amplitudes with t1 != 0 done")
    torch.cuda.empty_cache()
    _log("mixed path: workspace and device-generated inputs")
    with ck.Context([_desc(ck.PREC_MIXED)], device="cuda:0") as c:
        c.set_amplitudes(0, out["t1"], out["t2"])
        out["e_mixed"] = c.energy(0)
        out["r1_mixed"], out["r2_mixed"] = c.residual(0)
        _log("mixed path: energy and residual at the same amplitudes done")
        g1, g2 = c.residual(0, ta1, ta2)
        out["r1_t_mixed"], out["r2_t_mixed"] = g1, {b: g2[b].copy() for b in BLOCKS}
        del g2
        out["e_t_mixed"] = c.energy(0)
        _log("mixed path: residual and energy at the seeded amplitudes done")
    torch.cuda.empty_cache()
    out["ta1"], out["ta2"] = ta1, ta2
    return out


def _asym(r2):
    """Largest violation of R(ij,ab) = -R(ji,ab) = -R(ij,ba) over the sampled blocks,
    relative to max|R2| there."""
    kc = O.kconserv(GRID)
    worst, scale = 0.0, max(np.abs(r2[b]).max() for b in BLOCKS)
    for (ki, kj, ka) in BLOCKS:
        kb = kc[ki, kj, ka]
        x = r2[ki, kj, ka]
        worst = max(worst, np.abs(x + r2[kj, ki, ka].transpose(1, 0, 2, 3)).max(),
                    np.abs(x + r2[ki, kj, kb].transpose(0, 1, 3, 2)).max())
    return worst / scale


@pytest.fixture(scope="module")
def oracle_t(runs):
    """The block-restricted oracle at the seeded amplitudes: R1 in full, R2 on the sampled
    blocks, and the energy; <oo||vv> as a whole class, every other class block by block."""
    _log("host: generating the <oo||vv> class (5.2 GB) and the Fock matrix")
    oovv = synth.eri_class(SEED, GRID, NO, NV, "oovv", scale=SCALE)
    f = synth.fock(SEED, GRID, NO, NV)
    kc = O.kconserv(GRID)

    def provider(cls, kp, kq, kr):
        if cls == "oovv":
            return oovv[kp, kq, kr]
        return synth.eri_block(SEED, GRID, NO, NV, cls, kp, kq, kr, scale=SCALE)

    lazy = O.LazyClasses(provider)
    _log("oracle: R1 at the momenta k_i of the sampled blocks and the sampled R2 blocks")
    R1, R2b = O.residual_blocks(f, lazy, runs["ta1"], runs["ta2"], kc, BLOCKS, r1_ks=R1_KS,
                                callback=lambda step: _log(f"oracle: {step} done"))
    _log("oracle: energy at the seeded amplitudes")
    e = O.energy(f, {"oovv": oovv}, runs["ta1"], runs["ta2"], kc)
    return dict(R1=R1, R2=R2b, e=e)


def _oovv(ki, kj, ka):
    return synth.eri_block(SEED, GRID, NO, NV, "oovv", ki, kj, ka, scale=SCALE)


def test_driver_term_at_zero_amplitudes(runs):
    """R2 = conj(<ij||ab>) and R1 = conj(f_ia) at t = 0 (the host generator reproduces the
    device's values up to the last bits of its transcendentals)."""
    f = synth.fock(SEED, GRID, NO, NV)
    assert _rel(runs["r1_0"], np.conj(f[:, :NO, NO:])) <= 1e-13
    for b in BLOCKS:
        assert _rel(runs["r2_0"][b], np.conj(_oovv(*b))) <= 1e-13, b


def test_first_order_amplitudes(runs):
    """One update from t = 0: t = D^-1 R(0) (with one held vector the DIIS extrapolation is
    a copy), D from the Fock diagonal (Sec. 4.4)."""
    f = synth.fock(SEED, GRID, NO, NV)
    kc = O.kconserv(GRID)
    eo = np.real(np.einsum("kii->ki", f[:, :NO, :NO]))
    ev = np.real(np.einsum("kaa->ka", f[:, NO:, NO:]))
    assert _rel(runs["t1"], np.conj(f[:, :NO, NO:]) / (eo[:, :, None] - ev[:, None, :])) <= 1e-13
    for (ki, kj, ka) in BLOCKS:
        kb = kc[ki, kj, ka]
        D = eo[ki][:, None, None, None] + eo[kj][None, :, None, None] - ev[ka][None, None, :, None] - ev[kb][None, None, None, :]
        assert _rel(runs["t2"][ki, kj, ka], np.conj(_oovv(ki, kj, ka)) / D) <= 1e-13, (ki, kj, ka)


def test_energy_matches_oracle_in_full(runs):
    """The oracle's correlation energy over the whole host-generated <oo||vv> class at the
    device's first-order amplitudes."""
    _log("host: generating the <oo||vv> class (5.2 GB)")
    oovv = synth.eri_class(SEED, GRID, NO, NV, "oovv", scale=SCALE)
    f = synth.fock(SEED, GRID, NO, NV)
    _log("oracle: energy")
    e = O.energy(f, {"oovv": oovv}, runs["t1"], runs["t2"], O.kconserv(GRID))
    assert abs(runs["e"] - e) <= 1e-12 * abs(e)


def test_residual_antisymmetric(runs):
    """R2(ij, ab) = -R2(ji, ab) = -R2(ij, ba) (momenta exchanged with their orbitals) at the
    first-order amplitudes."""
    r2 = runs["r2"]
    kc = O.kconserv(GRID)
    scale = np.abs(r2[0, 0, 0]).max()
    for (ki, kj, ka) in BLOCKS:
        kb = kc[ki, kj, ka]
        x = r2[ki, kj, ka]
        assert np.abs(x + r2[kj, ki, ka].transpose(1, 0, 2, 3)).max() <= 1e-12 * scale, (ki, kj, ka)
        assert np.abs(x + r2[ki, kj, kb].transpose(0, 1, 3, 2)).max() <= 1e-12 * scale, (ki, kj, ka)


def test_mixed_within_error_model_of_fp64(runs):
    """Same amplitudes on both paths: the mixed residual within the bar of its parity tests
    against the oracle (1e-5 of max|R|), the energy within 1e-8 Eh."""
    assert _rel(runs["r2_mixed"], runs["r2"]) <= 1e-5
    assert _rel(runs["r1_mixed"], runs["r1"]) <= 1e-5
    assert abs(runs["e_mixed"] - runs["e"]) <= 1e-8


def test_fp64_residual_at_t1_matches_oracle(runs, oracle_t):
    """Element by element at the full size with t1 != 0: R1 at the sampled momenta and the
    sampled R2 blocks against the block-restricted oracle (every T1 path of the residual: the T1
    dressing of <ab||ef>, the t1 parts of the W seeds, tau's t1 t1 products, the F terms)."""
    ref = np.stack([oracle_t["R2"][b] for b in BLOCKS])
    got = np.stack([runs["r2_t"][b] for b in BLOCKS])
    assert _rel(got, ref) <= 1e-12
    assert _rel(runs["r1_t"][R1_KS], oracle_t["R1"][R1_KS]) <= 1e-12
    assert runs["r2_t_asym"] <= 1e-12


def test_energy_at_t1_matches_oracle(runs, oracle_t):
    """The energy with its t1 t1 term at the seeded amplitudes."""
    assert abs(runs["e_t"] - oracle_t["e"]) <= 1e-12 * abs(oracle_t["e"])


def test_mixed_residual_at_t1_matches_oracle(runs, oracle_t):
    """The mixed path at the seeded amplitudes, element by element within 1e-5 of max|R|
    (its t1-polynomial terms pass through the packed tau, the packed dressing and the
    packed assembly), the energy within 1e-8 Eh."""
    ref = np.stack([oracle_t["R2"][b] for b in BLOCKS])
    got = np.stack([runs["r2_t_mixed"][b] for b in BLOCKS])
    assert _rel(got, ref) <= 1e-5
    assert _rel(runs["r1_t_mixed"][R1_KS], oracle_t["R1"][R1_KS]) <= 1e-5
    assert abs(runs["e_t_mixed"] - oracle_t["e"]) <= 1e-8


@pytest.mark.timeout(600)
def test_converged_mixed_energy_within_1e8_of_fp64():
    """Both paths iterated to convergence from t = 0 at the full size (FP64 to ||R|| < 1e-10,
    the mixed path to its tolerance 1e-7, DIIS(6)): the converged correlation energies agree
    within 1e-8 Eh, the bar on mixed-precision energies (observed about 6e-10)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = {}
    for prec, tol in ((ck.PREC_FP64, 1e-10), (ck.PREC_MIXED, 1e-7)):
        torch.cuda.empty_cache()
        with ck.Context([_desc(prec)], device="cuda:0") as c:
            rc, it, rn = c.iterate(40, tol)
            out[prec] = (rc, it, rn, c.energy(0))
        _log(f"{('FP64', 'mixed')[prec]} path: rc={rc} evaluations={it} |R|={rn:.2e} E={out[prec][3]}")
    torch.cuda.empty_cache()
    assert out[ck.PREC_FP64][0] == ck.OK and out[ck.PREC_MIXED][0] == ck.OK
    assert abs(out[ck.PREC_MIXED][3] - out[ck.PREC_FP64][3]) <= 1e-8
