"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* Fock-space brute force: for random amplitudes and a random Hermitian Fock matrix with
  occupied-virtual coupling, the oracle's (R1, R2, E) equal the exact projections
  <Phi_mu| exp(-T) H_N exp(T) |Phi> (the CC amplitude equations are these projections).
  Grids include a 1-D mesh with N_k = 3 and a 2x2 mesh, where k != -k, so a wrong
  momentum sign or label fails.
* Two-electron exactness: CCSD is exact for two electrons, so the converged energy equals
  the eigenvalue of H_N whose eigenvector is dominated by the reference.
* MP2 closed form: one update from T = 0 gives t2 = <ab||ij>/D and
  E = 1/4 sum |<ij||ab>|^2 / D.
* Antisymmetry and momentum conservation of R2.
* Supercell folding: a k-point system re-labelled as one k point with N_k*n_occ occupied
  and N_k*n_vir virtual orbitals (zeros where momentum is not conserved) has the same
  converged energy, which checks the k-block bookkeeping against the N_k = 1 code path.
* Mutation: planting a sign error in one oracle term makes the brute-force pin fail.
* Rearranged equations: the rearranged T1 and T2 equations of Sec. 3.3 (a second oracle,
  ``oracle.rearranged``) equal the original ones; each reading of a Sec. 3.3 misprint is
  needed for that.
* Orbital rotation: the converged energy is the same in rotated occupied and virtual
  orbitals (a Fock matrix with all couplings).
"""
import numpy as np
import pytest

import synth
from oracle import ccsd_k as O
from tests import fockspace as FS


def _random_fock(rng, N, no, nv, ov=0.05):
    n = no + nv
    f = np.zeros((N, n, n), dtype=np.complex128)
    for k in range(N):
        a = 0.03 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        h = a + a.conj().T
        h[:no, no:] *= ov / 0.03
        h[no:, :no] = h[:no, no:].conj().T
        d = np.concatenate([rng.uniform(-2, -0.5, no), rng.uniform(0.5, 3, nv)])
        f[k] = h + np.diag(d)
    return f


def _classes_from_full(full, no):
    sl = {"o": slice(0, no), "v": slice(no, None)}
    return {c: np.ascontiguousarray(full[(Ellipsis,) + tuple(sl[x] for x in c)])
            for c in O.CLASSES}


BRUTE_CASES = [
    # grid, n_occ, n_vir
    ((1, 1, 1), 2, 3),
    ((2, 1, 1), 2, 2),
    ((3, 1, 1), 1, 3),
    ((3, 1, 1), 2, 1),
    ((2, 2, 1), 1, 2),
]


@pytest.mark.parametrize("grid,no,nv", BRUTE_CASES)
def test_brute_force_residual_and_energy(grid, no, nv):
    rng = np.random.default_rng(sum(grid) * 100 + no * 10 + nv)
    N = int(np.prod(grid))
    kc = O.kconserv(grid)
    f = _random_fock(rng, N, no, nv)
    full = synth.eri_class(11 + N, grid, no, nv, "nnnn", scale=0.2)
    t1, t2 = synth.test_amplitudes(5 + N, grid, no, nv, scale=0.3)
    classes = _classes_from_full(full, no)
    R1, R2 = O.residual(f, classes, t1, t2, kc)
    E = O.energy(f, classes, t1, t2, kc)
    B1, B2, BE = FS.brute_force_residual(f, full, t1, t2, kc)
    scale = max(np.abs(B2).max(), np.abs(B1).max())
    assert np.abs(R1 - B1).max() <= 1e-12 * scale
    assert np.abs(R2 - B2).max() <= 1e-12 * scale
    assert abs(E - BE) <= 1e-12 * max(1.0, abs(BE))
    # the projections are not trivially small: every term matters at this scale
    assert np.abs(B2).max() > 1e-2 and np.abs(B1).max() > 1e-2


def test_brute_force_catches_planted_sign_error(monkeypatch):
    """Flip the sign of the t1 dressing inside W_mnij: the brute-force pin must fail."""
    grid, no, nv = (3, 1, 1), 2, 1
    rng = np.random.default_rng(7)
    N = 3
    kc = O.kconserv(grid)
    f = _random_fock(rng, N, no, nv)
    full = synth.eri_class(21, grid, no, nv, "nnnn", scale=0.2)
    t1, t2 = synth.test_amplitudes(8, grid, no, nv, scale=0.3)
    classes = _classes_from_full(full, no)
    B1, B2, _ = FS.brute_force_residual(f, full, t1, t2, kc)
    orig = O.w_mnij

    def bad_w_mnij(eris, t1_, tau, kc_):
        W = orig(eris, t1_, tau, kc_)
        W2 = orig(eris, -t1_, tau, kc_)  # only the single-t1 term changes sign
        return W2 + 0 * W

    monkeypatch.setattr(O, "w_mnij", bad_w_mnij)
    _, R2 = O.residual(f, classes, t1, t2, kc)
    assert np.abs(R2 - B2).max() > 1e-6


@pytest.mark.parametrize("grid,no,nv", [((2, 1, 1), 1, 3), ((1, 1, 1), 2, 4), ((2, 1, 1), 1, 4)])
def test_two_electron_exactness(grid, no, nv):
    """Converged CCSD energy equals the exact eigenvalue for two electrons."""
    N = int(np.prod(grid))
    assert N * no == 2
    kc = O.kconserv(grid)
    f = synth.fock(31, grid, no, nv)
    full = synth.eri_class(31, grid, no, nv, "nnnn", scale=0.05)
    classes = _classes_from_full(full, no)
    res = O.solve(f, classes, grid, max_iter=200, tol=1e-12)
    assert res["converged"]
    w, weights = FS.fci_energies(f, full, kc, no)
    e_exact = w[np.argmax(weights)]
    assert weights.max() > 0.5
    assert abs(res["energy"] - e_exact) <= 1e-10


@pytest.mark.parametrize("grid,no,nv", [((2, 1, 1), 4, 8), ((3, 1, 1), 2, 4)])
def test_mp2_first_iteration(grid, no, nv):
    f, classes = synth.system(101, grid, no, nv)
    res = O.solve(f, classes, grid, max_iter=1, tol=0.0)
    kc = O.kconserv(grid)
    N = int(np.prod(grid))
    eo = np.real(np.einsum("kii->ki", f[:, :no, :no]))
    ev = np.real(np.einsum("kaa->ka", f[:, no:, no:]))
    e_mp2 = 0.0
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                kb = kc[ki, kj, ka]
                g = classes["oovv"][ki, kj, ka]
                for i in range(no):
                    for j in range(no):
                        for a in range(nv):
                            for b in range(nv):
                                d = eo[ki, i] + eo[kj, j] - ev[ka, a] - ev[kb, b]
                                e_mp2 += abs(g[i, j, a, b]) ** 2 / d / 4
    assert e_mp2 < 0
    assert abs(res["energy"] - e_mp2) <= 1e-14 * abs(e_mp2)
    assert np.allclose(res["t1"], 0)


@pytest.mark.parametrize("grid,no,nv", [((3, 1, 1), 2, 3), ((2, 2, 1), 2, 2)])
def test_residual_antisymmetry_and_conservation(grid, no, nv):
    N = int(np.prod(grid))
    kc = O.kconserv(grid)
    f, classes = synth.system(55, grid, no, nv, scale=0.1)
    t1, t2 = synth.test_amplitudes(9, grid, no, nv, scale=0.2)
    R1, R2 = O.residual(f, classes, t1, t2, kc)
    err = 0.0
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                kb = kc[ki, kj, ka]
                r = R2[ki, kj, ka]
                err = max(err, np.abs(r + R2[kj, ki, ka].transpose(1, 0, 2, 3)).max(),
                          np.abs(r + R2[ki, kj, kb].transpose(0, 1, 3, 2)).max())
    assert err <= 1e-14 * np.abs(R2).max()
    # the exact projections onto doubles that break momentum conservation vanish, so the
    # block form (which stores only conserving blocks) drops nothing
    g2, o2, v2 = ((3, 1, 1), 1, 2) if N == 3 else ((2, 2, 1), 1, 2)
    kc2 = O.kconserv(g2)
    f2 = synth.fock(56, g2, o2, v2)
    s1, s2 = synth.test_amplitudes(10, g2, o2, v2, scale=0.3)
    worst, count = FS.nonconserving_double_projection(
        f2, synth.eri_class(56, g2, o2, v2, "nnnn", 0.2), s1, s2, kc2)
    assert count > 0 and worst <= 1e-15


def test_kconserv_properties():
    for grid in [(3, 1, 1), (2, 2, 2), (3, 3, 3), (4, 2, 1)]:
        kc = O.kconserv(grid)
        N = int(np.prod(grid))
        g = np.array(grid)
        vec = np.array(np.unravel_index(np.arange(N), grid)).T
        for kp in range(N):
            for kq in range(N):
                for kr in range(N):
                    ks = kc[kp, kq, kr]
                    assert np.all((vec[kp] + vec[kq] - vec[kr] - vec[ks]) % g == 0)
        # synth's independent implementation agrees
        assert np.array_equal(kc, synth.kconserv_table(grid))
    kc = O.kconserv((3, 1, 1))
    assert kc[1, 0, 0] == 1 and kc[0, 0, 1] == 2  # -1 == 2 on a 3-point ring, not 1


def _fold_to_one_k(f, classes, grid, no, nv):
    """Relabel a k-point system as one k point: occupied (k,i) first, then virtual (k,a)."""
    N = int(np.prod(grid))
    kc = O.kconserv(grid)
    eris = O.Eris(classes, kc)
    NO, NV = N * no, N * nv
    F = np.zeros((1, NO + NV, NO + NV), dtype=np.complex128)
    for k in range(N):
        F[0, k * no:(k + 1) * no, k * no:(k + 1) * no] = f[k, :no, :no]
        F[0, NO + k * nv:NO + (k + 1) * nv, NO + k * nv:NO + (k + 1) * nv] = f[k, no:, no:]
        F[0, k * no:(k + 1) * no, NO + k * nv:NO + (k + 1) * nv] = f[k, :no, no:]
        F[0, NO + k * nv:NO + (k + 1) * nv, k * no:(k + 1) * no] = f[k, no:, :no]
    out = {}
    dims = {"o": no, "v": nv}
    for c in O.CLASSES:
        big = np.zeros((1, 1, 1) + tuple(N * dims[x] for x in c), dtype=np.complex128)
        for kp in range(N):
            for kq in range(N):
                for kr in range(N):
                    ks = kc[kp, kq, kr]
                    ks_ = [kp, kq, kr, ks]
                    sl = tuple(slice(ks_[t] * dims[c[t]], (ks_[t] + 1) * dims[c[t]]) for t in range(4))
                    big[(0, 0, 0) + sl] = eris.block(c, kp, kq, kr)
        out[c] = big
    return F, out


def test_supercell_folding_matches_k_blocks():
    grid, no, nv = (3, 1, 1), 2, 3
    f, classes = synth.system(77, grid, no, nv)
    res_k = O.solve(f, classes, grid, max_iter=60, tol=1e-11)
    F, big = _fold_to_one_k(f, classes, grid, no, nv)
    res_1 = O.solve(F, big, (1, 1, 1), max_iter=60, tol=1e-11)
    assert res_k["converged"] and res_1["converged"]
    assert abs(res_k["energy"] - res_1["energy"]) <= 1e-11


@pytest.mark.parametrize("grid,no,nv", [((1, 1, 1), 2, 3), ((2, 1, 1), 2, 2), ((3, 1, 1), 2, 3), ((2, 2, 1), 1, 2)])
def test_rearranged_equations_match_original(grid, no, nv):
    """The rearranged equations of Sec. 3.3 (A-bar + A-check + A-tilde + A-hat and the
    rearranged T1 equation) are an exact regrouping of Sec. 2: both oracles agree on random
    antisymmetric amplitudes, random integrals and a Fock matrix with occupied-virtual
    coupling.  This pins the readings of the Sec. 3.3 misprints (module docstring of
    oracle.rearranged): reversing any of them breaks the equality."""
    from oracle import rearranged as RA

    N = int(np.prod(grid))
    kc = O.kconserv(grid)
    f, eris = synth.system(900 + N, grid, no, nv, scale=0.1)
    f = _random_fock(np.random.default_rng(N + no), N, no, nv)
    t1, t2 = synth.test_amplitudes(40 + N, grid, no, nv, scale=0.2)
    R1, R2 = O.residual(f, eris, t1, t2, kc)
    A1, A2 = RA.residual(f, eris, t1, t2, kc)
    assert np.abs(A2 - R2).max() <= 1e-12 * np.abs(R2).max()
    assert np.abs(A1 - R1).max() <= 1e-12 * np.abs(R1).max()


@pytest.mark.parametrize("key,printed", [("K_SIGN_FOO", -1), ("ZETA_BAR", "ia"), ("AHAT_PAIR", "check")])
def test_rearranged_misprint_readings_are_forced(monkeypatch, key, printed):
    """Each reading of a Sec. 3.3 misprint is needed: with the printed form instead, the
    rearranged equations no longer equal the original ones (on a 1-D N_k = 3 mesh, where
    k and -k differ)."""
    from oracle import rearranged as RA

    grid, no, nv = (3, 1, 1), 2, 2
    kc = O.kconserv(grid)
    f, eris = synth.system(77, grid, no, nv, scale=0.1)
    f = _random_fock(np.random.default_rng(5), 3, no, nv)
    t1, t2 = synth.test_amplitudes(8, grid, no, nv, scale=0.2)
    R1, R2 = O.residual(f, eris, t1, t2, kc)
    monkeypatch.setitem(RA.READINGS, key, printed)
    A1, A2 = RA.residual(f, eris, t1, t2, kc)
    bad = max(np.abs(A2 - R2).max() / np.abs(R2).max(), np.abs(A1 - R1).max() / np.abs(R1).max())
    assert bad > 1e-6


def rotate_system(f, eris, kc, no, seed, angle=0.3):
    """The same system in rotated orbitals: per k, a random unitary U_k mixing the occupied
    orbitals among themselves and the virtual ones among themselves; f_k -> U_k^H f_k U_k and
    <pq||rs> -> sum conj(U_p) conj(U_q) U_r U_s <..||..>, each factor at its own momentum.
    Returns (f', eris')."""
    N, n = f.shape[0], f.shape[1]
    rng = np.random.default_rng(seed)
    U = np.zeros((N, n, n), dtype=np.complex128)
    for k in range(N):
        for lo, hi in ((0, no), (no, n)):
            m = hi - lo
            h = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
            h = angle * (h + h.conj().T) / 2
            w, v = np.linalg.eigh(h)
            U[k, lo:hi, lo:hi] = (v * np.exp(1j * w)) @ v.conj().T
    fr = np.stack([U[k].conj().T @ f[k] @ U[k] for k in range(N)])
    E = O.Eris(eris, kc)
    sl = {"o": slice(0, no), "v": slice(no, n)}
    full = np.zeros((N, N, N, n, n, n, n), dtype=np.complex128)
    for kp in range(N):
        for kq in range(N):
            for kr in range(N):
                for a in "ov":
                    for b in "ov":
                        for c in "ov":
                            for d in "ov":
                                full[kp, kq, kr][sl[a], sl[b], sl[c], sl[d]] = E.block(a + b + c + d, kp, kq, kr)
    rot = np.zeros_like(full)
    for kp in range(N):
        for kq in range(N):
            for kr in range(N):
                ks = kc[kp, kq, kr]
                rot[kp, kq, kr] = np.einsum("ap,bq,cr,ds,abcd->pqrs", U[kp].conj(), U[kq].conj(), U[kr], U[ks],
                                            full[kp, kq, kr], optimize=True)
    return fr, _classes_from_full(rot, no)


@pytest.mark.parametrize("grid,no,nv", [((3, 1, 1), 2, 3), ((2, 2, 1), 1, 2)])
def test_energy_invariant_under_orbital_rotation(grid, no, nv):
    """The converged CCSD energy does not depend on the orbital basis within the occupied
    and within the virtual space: the same system in rotated orbitals (a Fock matrix with
    occupied-occupied and virtual-virtual off-diagonal elements) converges to the same E."""
    kc = O.kconserv(grid)
    f, eris = synth.system(31, grid, no, nv, scale=0.05)
    fr, er = rotate_system(f, eris, kc, no, seed=3)
    a = O.solve(f, eris, grid, max_iter=80, tol=1e-11, diis_space=6)
    b = O.solve(fr, er, grid, max_iter=80, tol=1e-11, diis_space=6)
    assert a["converged"] and b["converged"]
    assert abs(fr[0] - f[0]).max() > 1e-3  # the rotation really changed the Fock matrix
    assert abs(a["energy"] - b["energy"]) <= 1e-10 * max(1.0, abs(a["energy"]))


# ------------------------------------------------------------------ norm and DIIS pins
def test_residual_norm_closed_form():
    """The convergence norm (the 2-norm over every stored element of R1 and R2) on a case
    with a known answer: |3+4i| = 5 in R1 and 12 in R2 give sqrt(25 + 144) = 13.  Dropping
    either part, or taking real parts instead of moduli, gives 12, 5 or sqrt(153)."""
    R1 = np.zeros((2, 1, 2), np.complex128)
    R2 = np.zeros((2, 2, 2, 1, 1, 2, 2), np.complex128)
    R1[1, 0, 1] = 3 + 4j
    R2[0, 1, 1, 0, 0, 1, 0] = -12j
    assert O.residual_norm(R1, R2) == 13.0
    assert O.residual_norm(np.zeros_like(R1), np.zeros_like(R2)) == 0.0


def test_diis_hand_solved_two_vector_extrapolation():
    """Pulay DIIS with two held vectors minimizes |c1 e1 + c2 e2| under c1 + c2 = 1, whose
    solution is c1 = (<e2,e2> - <e1,e2>) / (<e1,e1> - 2<e1,e2> + <e2,e2>) with the real
    part of the Hermitian overlap.  e1 = (1, i), e2 = (-1, 2 + 2i): <e1,e1> = 2, <e2,e2> = 9,
    Re<e1,e2> = -1 + 2 = 1, so c1 = 8/9, c2 = 1/9.  A mis-signed overlap (-1) would give
    c1 = 10/13; an unconjugated product (Re(i (2+2i)) = -2, so -3) gives c1 = 12/17."""
    d = O.Diis(6)
    v1 = np.array([1.0 + 0j, 0.0, 5.0])
    v2 = np.array([0.0 + 0j, 3.0, -1.0])
    e1 = np.array([1.0 + 0j, 1j])
    e2 = np.array([-1.0 + 0j, 2 + 2j])
    out1 = d.update(v1, e1)
    assert np.array_equal(out1, v1)  # one held vector: no extrapolation
    out2 = d.update(v2, e2)
    c1, c2 = 8 / 9, 1 / 9
    assert np.allclose(out2, c1 * v1 + c2 * v2, rtol=0, atol=1e-15)


def test_diis_fifo_drops_the_oldest_vector():
    """With a depth of 2 the third update extrapolates from the second and third vectors
    only: orthogonal errors of norms 2 and 1 give c = (1/5, 4/5)."""
    d = O.Diis(2)
    vs = [np.array([1.0 + 0j, 2.0]), np.array([3.0 + 0j, -1.0]), np.array([-2.0 + 0j, 4.0])]
    es = [np.array([1.0 + 0j, 0.0]), np.array([2.0 + 0j, 0.0]), np.array([0.0 + 0j, 1.0])]
    for v, e in zip(vs[:2], es[:2]):
        d.update(v, e)
    out = d.update(vs[2], es[2])
    assert np.allclose(out, 0.2 * vs[1] + 0.8 * vs[2], rtol=0, atol=1e-15)


def test_block_restricted_residual_equals_full():
    """The block-restricted oracle (R2 on chosen momentum blocks, integrals served block by
    block) equals the full oracle, which the brute force pins, on a 3x3x1 mesh (k != -k
    along two axes) at amplitudes with t1 != 0."""
    grid, no, nv = (3, 3, 1), 2, 3
    kc = O.kconserv(grid)
    f, eris = synth.system(808, grid, no, nv, scale=0.1)
    t1, t2 = synth.test_amplitudes(809, grid, no, nv, scale=0.2)
    R1, R2 = O.residual(f, eris, t1, t2, kc)
    lazy = O.LazyClasses(lambda cls, kp, kq, kr: synth.eri_block(808, grid, no, nv, cls, kp, kq, kr, scale=0.1))
    blocks = [(0, 0, 0), (1, 2, 3), (8, 7, 5), (4, 4, 4), (2, 6, 2)]
    B1, B2 = O.residual_blocks(f, lazy, t1, t2, kc, blocks)
    assert np.abs(B1 - R1).max() <= 1e-15 * np.abs(R1).max()
    C1, _ = O.residual_blocks(f, lazy, t1, t2, kc, blocks[:1], r1_ks=[2, 7])
    assert np.array_equal(C1[[2, 7]], B1[[2, 7]]) and not np.any(C1[[0, 1, 3, 4, 5, 6, 8]])
    for b in blocks:
        assert np.abs(B2[b] - R2[b]).max() <= 1e-15 * np.abs(R2).max(), b
