"""Plain FP64 CPU oracle for periodic (k-point) spin-orbital CCSD.

TEST INFRASTRUCTURE ONLY.  This module exists to check the GPU library; it is imported by
``tests/``, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``
and by nothing else.  It shares no code with the GPU path.

It follows the paper's Section 2 ("Basic equations in the CCSD in a periodic system")
term by term: the T1 equation (eq. ori_EqSingle), the T2 equation (eq. ori_EqDouble), the
antisymmetrizer P_-, the intermediates W (hole-hole, particle-particle, ring: eq.
Def_Woovv and the two before it), F (eqs. ori_F_oo, ori_F_vv, ori_F_ov) and the
effective amplitudes tau-tilde and tau.  The iteration follows Sec. 4.4 (successive
substitution with D^-1 R, convergence when the residual is small); the start rule
t0 = f(0) is Sec. 3.2.2.

Readings where the paper is silent or misprinted (each is pinned by a test, see
``tests/test_oracle_pins.py``):
  * the last T2 term's integral is <r k_a b k_b || i k_i j k_j> (ovoo); the printed
    ket label "c" cannot sit in an ovoo integral;
  * in W_jn^bf the orbital r sits at k_b (fixed by t_r^b), not at its own k_r;
  * the leading T1 term f_p^g is read as f_ai = conj(f_ia);
  * the correlation energy, which the paper does not print, is the standard
    E = sum f_ia t_i^a + 1/4 sum <ij||ab> t_ij^ab + 1/2 sum <ij||ab> t_i^a t_j^b
    (whole-supercell value, no 1/N_k);
  * Pulay DIIS (not in the paper) is an optional accelerator of the same fixed point.

Storage: t1[k][i][a]; t2[ki][kj][ka][i][j][a][b] with k_b fixed by conservation;
integrals by class ``oooo, ooov, oovv, ovvo, ovvv, vvvv`` as [kp][kq][kr][p][q][r][s]
with k_s fixed.  All complex128.
"""
from __future__ import annotations

import numpy as np

CLASSES = ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")


def _con(subscripts, *ops):
    return np.einsum(subscripts, *ops, optimize=True)


# --------------------------------------------------------------------------------------
# Momentum conservation (Sec. 3.2.5): k1 + k2 = k3 + k4 + G on a Gamma-containing mesh.
# --------------------------------------------------------------------------------------
def kconserv(grid) -> np.ndarray:
    """KC[kp,kq,kr] = ks with kp + kq - kr = ks modulo the mesh (C-order k labels)."""
    g = np.array(grid, dtype=np.int64)
    N = int(np.prod(g))
    vec = np.array(np.unravel_index(np.arange(N), tuple(g))).T  # (N, 3)
    s = (vec[:, None, None, :] + vec[None, :, None, :] - vec[None, None, :, :]) % g
    return np.ravel_multi_index((s[..., 0], s[..., 1], s[..., 2]), tuple(g)).astype(np.int64)


class Eris:
    """Antisymmetrized integrals <pq||rs> from the six stored classes.

    Every other o/v class follows from the relations of Sec. 3.3: Hermiticity
    <pq||rs> = conj(<rs||pq>) and antisymmetry in (p,q) and in (r,s), with each
    momentum travelling with its orbital.
    """

    def __init__(self, classes: dict, kc: np.ndarray):
        self.c = classes
        self.kc = kc

    def block(self, cls: str, kp: int, kq: int, kr: int) -> np.ndarray:
        if cls in self.c:
            return self.c[cls][kp, kq, kr]
        ks = int(self.kc[kp, kq, kr])
        # swap the bra pair
        sw = cls[1] + cls[0] + cls[2:]
        if sw in self.c:
            return -self.c[sw][kq, kp, kr].transpose(1, 0, 2, 3)
        # swap the ket pair
        sw = cls[:2] + cls[3] + cls[2]
        if sw in self.c:
            return -self.c[sw][kp, kq, ks].transpose(0, 1, 3, 2)
        sw = cls[1] + cls[0] + cls[3] + cls[2]
        if sw in self.c:
            return self.c[sw][kq, kp, ks].transpose(1, 0, 3, 2)
        # Hermitian conjugate: <pq||rs> = conj(<rs||pq>), then the swaps above
        herm = cls[2:] + cls[:2]
        return np.conj(self.block(herm, kr, ks, kp).transpose(2, 3, 0, 1))


# --------------------------------------------------------------------------------------
# Effective amplitudes (eqs. for tau-tilde and tau at the end of Sec. 2)
# --------------------------------------------------------------------------------------
def make_tau(t1, t2, kc, fac):
    """t2 + fac * P(ab) P(ij) t_i^a t_j^b with fac = 1/2 (tau) or 1/4 (tau-tilde).

    A single amplitude t_i^a is nonzero only when k_i = k_a, so the four products of
    P(ab)P(ij) t_i^a t_j^b pair up into 2 (d(k_a,k_i) t_i^a t_j^b - d(k_b,k_i) t_i^b t_j^a).
    """
    N = t1.shape[0]
    tau = t2.copy()
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                kb = kc[ki, kj, ka]
                if ka == ki:
                    tau[ki, kj, ka] += 2 * fac * _con("ia,jb->ijab", t1[ki], t1[kj])
                if kb == ki:
                    tau[ki, kj, ka] -= 2 * fac * _con("ib,ja->ijab", t1[ki], t1[kj])
    return tau


# --------------------------------------------------------------------------------------
# F intermediates (eqs. ori_F_oo, ori_F_vv, ori_F_ov)
# --------------------------------------------------------------------------------------
def f_intermediates(f, eris: Eris, t1, t2, kc, no):
    N = t1.shape[0]
    foo, fvv, fov = f[:, :no, :no], f[:, no:, no:], f[:, :no, no:]
    taut = make_tau(t1, t2, kc, 0.25)
    Fov = fov.copy()
    Foo = foo.copy()
    Fvv = fvv.copy()
    for k in range(N):
        Foo[k] += 0.5 * _con("mc,ic->mi", fov[k], t1[k])
        Fvv[k] -= 0.5 * _con("mh,ma->ah", fov[k], t1[k])
        for kn in range(N):
            # t_n^f <m k, n kn || e k, f kn>
            Fov[k] += _con("nf,mnef->me", t1[kn], eris.block("oovv", k, kn, k))
            # t_n^e <m k, n kn || i k, e kn>
            Foo[k] += _con("ne,mnie->mi", t1[kn], eris.block("ooov", k, kn, k))
            # t_m^f <a k, m kn || e k, f kn>
            Fvv[k] += _con("mf,amef->ae", t1[kn], eris.block("vovv", k, kn, k))
            for ke in range(N):
                # 1/2 taut_{i k, n kn}^{e ke, f kf} <m k, n kn || e ke, f kf>
                Foo[k] += 0.5 * _con("inef,mnef->mi", taut[k, kn, ke], eris.block("oovv", k, kn, ke))
                # -1/2 taut_{m kn, n ke}^{a k, f kf} <m kn, n ke || e k, f kf>
                Fvv[k] -= 0.5 * _con("mnaf,mnef->ae", taut[kn, ke, k], eris.block("oovv", kn, ke, k))
    return Foo, Fvv, Fov


# --------------------------------------------------------------------------------------
# W intermediates (Sec. 2, the three definitions ending with eq. Def_Woovv)
# --------------------------------------------------------------------------------------
def w_mnij_block(eris: Eris, t1, tau, kc, km, kn, ki):
    """One block W_{m km n kn i ki j kj} (k_j by conservation):
    <mn||ij> + P(ij) t_j^c <mn||ic> + 1/4 tau_ij^ef <mn||ef>."""
    N = t1.shape[0]
    kj = kc[km, kn, ki]
    w = eris.block("oooo", km, kn, ki).copy()
    w += _con("jc,mnic->mnij", t1[kj], eris.block("ooov", km, kn, ki))
    w -= _con("ic,mnjc->mnij", t1[ki], eris.block("ooov", km, kn, kj))
    for ke in range(N):
        w += 0.25 * _con("ijef,mnef->mnij", tau[ki, kj, ke], eris.block("oovv", km, kn, ke))
    return w


def w_mnij(eris: Eris, t1, tau, kc):
    """W_{m km n kn i ki j kj}: <mn||ij> + P(ij) t_j^c <mn||ic> + 1/4 tau_ij^ef <mn||ef>."""
    N = t1.shape[0]
    no = t1.shape[1]
    W = np.zeros((N, N, N, no, no, no, no), dtype=np.complex128)
    for km in range(N):
        for kn in range(N):
            for ki in range(N):
                W[km, kn, ki] = w_mnij_block(eris, t1, tau, kc, km, kn, ki)
    return W


def w_abef_block(eris: Eris, t1, tau, kc, ka, kb, ke):
    """W^{a ka b kb e ke f kf}: <ab||ef> - P(ab) t_r^b <ar||ef> + 1/4 tau_mn^ab <mn||ef>."""
    N = t1.shape[0]
    w = eris.block("vvvv", ka, kb, ke).copy()
    # -P(ab) sum_r t_{r kb}^{b kb} <a ka, r kb || e ke, f kf>
    w -= _con("rb,aref->abef", t1[kb], eris.block("vovv", ka, kb, ke))
    w += _con("ra,bref->abef", t1[ka], eris.block("vovv", kb, ka, ke))
    for km in range(N):
        kn = kc[ka, kb, km]
        w += 0.25 * _con("mnab,mnef->abef", tau[km, kn, ka], eris.block("oovv", km, kn, ke))
    return w


def w_mbej_block(eris: Eris, t1, t2, kc, km, kb, ke):
    """One block Wr[km][kb][ke](m,b,e,j) of the ring intermediate (k_j by conservation),
    printed as W_{j kj n kn}^{b kb f kf} with n -> m, f -> e:
      <mb||ej> + t_j^f <mb||ef> - t_n^b <mn||ej> - 1/2 t_{jn}^{fb} <mn||ef> - t_j^f t_n^b <mn||ef>
    with n of the third term at k_b."""
    N = t1.shape[0]
    kj = kc[km, kb, ke]
    w = eris.block("ovvo", km, kb, ke).copy()
    w += _con("jf,mbef->mbej", t1[kj], eris.block("ovvv", km, kb, ke))
    w -= _con("nb,mnej->mbej", t1[kb], eris.block("oovo", km, kb, ke))
    w -= _con("jf,nb,mnef->mbej", t1[kj], t1[kb], eris.block("oovv", km, kb, ke))
    for kn in range(N):
        kf = kc[kj, kn, kb]
        w -= 0.5 * _con("jnfb,mnef->mbej", t2[kj, kn, kf], eris.block("oovv", km, kn, ke))
    return w


def w_mbej(eris: Eris, t1, t2, kc):
    """Ring intermediate for every block: Wr[km][kb][ke](m,b,e,j) (see w_mbej_block)."""
    N, no, nv = t1.shape
    W = np.zeros((N, N, N, no, nv, nv, no), dtype=np.complex128)
    for km in range(N):
        for kb in range(N):
            for ke in range(N):
                W[km, kb, ke] = w_mbej_block(eris, t1, t2, kc, km, kb, ke)
    return W


def ring_x_block(eris: Eris, t1, t2, kc, wr, ki, kj, ka):
    """Ring quantity X_{i ki j kj}^{a ka b kb} before P(ab)P(ij):
    sum_n t_{i n}^{a f} W_{j n}^{b f} - t_i^c t_r^a <r b||c j>; wr(kn, kb, kf) returns a
    block of the ring intermediate."""
    N = t1.shape[0]
    kb = kc[ki, kj, ka]
    x = -_con("ic,ra,rbcj->ijab", t1[ki], t1[ka], eris.block("ovvo", ka, kb, ki))
    for kn in range(N):
        kf = kc[ki, kn, ka]
        # t_{i ki n kn}^{a ka f kf} W_{j kj n kn}^{b kb f kf}
        x = x + _con("inaf,nbfj->ijab", t2[ki, kn, ka], wr(kn, kb, kf))
    return x


def r2_block_nonladder(eris: Eris, t1, t2, tau, Fvt, Fot, kc, wmn, x, ki, kj, ka):
    """Every term of the T2 equation for block (ki, kj, ka) except the particle-particle
    ladder: the driver, the F terms, 1/2 tau W_mnij, P(ab)P(ij) of the ring quantity and the
    two single-amplitude integral terms.  wmn(km, kn, ki) and x(ki, kj, ka) return blocks of
    W_mnij and of the ring quantity."""
    N = t1.shape[0]
    kb = kc[ki, kj, ka]
    r = np.conj(eris.block("oovv", ki, kj, ka))  # <ab||ij> = conj(<ij||ab>)
    # P(ab) t_ij^{af} Fvt(b,f), f at kb
    r = r + _con("ijaf,bf->ijab", t2[ki, kj, ka], Fvt[kb])
    r = r - _con("ijbf,af->ijab", t2[ki, kj, kb], Fvt[ka])
    # -P(ij) t_in^{ab} Fot(n,j), n at kj
    r = r - _con("inab,nj->ijab", t2[ki, kj, ka], Fot[kj])
    r = r + _con("jnab,ni->ijab", t2[kj, ki, ka], Fot[ki])
    # 1/2 tau_mn^ab W_mnij
    for km in range(N):
        kn = kc[ki, kj, km]
        r = r + 0.5 * _con("mnab,mnij->ijab", tau[km, kn, ka], wmn(km, kn, ki))
    # P(ab)P(ij) ring
    r = r + x(ki, kj, ka) - x(kj, ki, ka).transpose(1, 0, 2, 3)
    r = r - x(ki, kj, kb).transpose(0, 1, 3, 2) + x(kj, ki, kb).transpose(1, 0, 3, 2)
    # P(ij) <a ka b kb || c ki j kj> t_{i ki}^{c ki}
    r = r + _con("abcj,ic->ijab", eris.block("vvvo", ka, kb, ki), t1[ki])
    r = r - _con("abci,jc->ijab", eris.block("vvvo", ka, kb, kj), t1[kj])
    # -P(ab) t_{r ka}^{a ka} <r ka b kb || i ki j kj>
    r = r - _con("ra,rbij->ijab", t1[ka], eris.block("ovoo", ka, kb, ki))
    r = r + _con("rb,raij->ijab", t1[kb], eris.block("ovoo", kb, ka, ki))
    return r


def t1_residual(f, eris: Eris, t1, t2, Foo, Fvv, Fov, ks=None):
    """R1: the right-hand side of the T1 equation (eq. ori_EqSingle), at the momenta ``ks``
    (default all; the other blocks are left zero)."""
    N, no, nv = t1.shape
    R1 = np.zeros_like(t1)
    for k in (range(N) if ks is None else ks):
        r = np.conj(f[k, :no, no:])  # f_ai = conj(f_ia)
        r = r + _con("ic,ac->ia", t1[k], Fvv[k])
        r = r - _con("ra,ri->ia", t1[k], Foo[k])
        for kn in range(N):
            r = r + _con("inaf,nf->ia", t2[k, kn, k], Fov[kn])
            # t_{r kn}^{c kn} <a k, r kn || i k, c kn>
            r = r + _con("rc,aric->ia", t1[kn], eris.block("voov", k, kn, k))
            for km in range(N):
                # -1/2 t_{m km, n kn}^{a k, f kf} <m km, n kn || i k, f kf>
                r = r - 0.5 * _con("mnaf,mnif->ia", t2[km, kn, k], eris.block("ooov", km, kn, k))
                # +1/2 t_{i k, n kn}^{e km, f kf} <a k, n kn || e km, f kf>
                r = r + 0.5 * _con("inef,anef->ia", t2[k, kn, km], eris.block("vovv", k, kn, km))
        R1[k] = r
    return R1


def _f_tilde(t1, Foo, Fvv, Fov):
    """Fvt(b,f) = F^{bf} - 1/2 t_r^b F_r^f and Fot(n,j) = F_nj + 1/2 t_j^c F_n^c (one k)."""
    N = t1.shape[0]
    Fvt = np.stack([Fvv[k] - 0.5 * _con("rb,rf->bf", t1[k], Fov[k]) for k in range(N)])
    Fot = np.stack([Foo[k] + 0.5 * _con("jc,nc->nj", t1[k], Fov[k]) for k in range(N)])
    return Fvt, Fot


# --------------------------------------------------------------------------------------
# Residuals (eqs. ori_EqSingle and ori_EqDouble); R = 0 at the solution
# --------------------------------------------------------------------------------------
def residual(f, classes: dict, t1, t2, kc):
    """Return (R1, R2): the right-hand sides of the T1 and T2 equations of Sec. 2."""
    N, no, nv = t1.shape
    eris = Eris(classes, kc)
    Foo, Fvv, Fov = f_intermediates(f, eris, t1, t2, kc, no)
    tau = make_tau(t1, t2, kc, 0.5)

    # ---------------- T1 equation ----------------
    R1 = t1_residual(f, eris, t1, t2, Foo, Fvv, Fov)

    # ---------------- T2 equation ----------------
    Fvt, Fot = _f_tilde(t1, Foo, Fvv, Fov)
    Wmn = w_mnij(eris, t1, tau, kc)
    Wr = w_mbej(eris, t1, t2, kc)

    # ring quantity X_{i ki j kj}^{a ka b kb} before P(ab)P(ij)
    X = np.zeros_like(t2)
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                X[ki, kj, ka] = ring_x_block(eris, t1, t2, kc, lambda a, b, c: Wr[a, b, c], ki, kj, ka)

    R2 = np.zeros_like(t2)
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                R2[ki, kj, ka] = r2_block_nonladder(eris, t1, t2, tau, Fvt, Fot, kc,
                                                    lambda a, b, c: Wmn[a, b, c],
                                                    lambda a, b, c: X[a, b, c], ki, kj, ka)

    # particle-particle ladder 1/2 W_abef tau_ij^ef: one W^{ab ef} block at a time
    for ka in range(N):
        for kb in range(N):
            for ke in range(N):
                W = w_abef_block(eris, t1, tau, kc, ka, kb, ke)
                for ki in range(N):
                    kj = kc[ka, kb, ki]
                    R2[ki, kj, ka] += 0.5 * _con("abef,ijef->ijab", W, tau[ki, kj, ke])
    return R1, R2


class LazyClasses:
    """Integral classes served block by block: ``provider(cls, kp, kq, kr)`` returns the
    block [p][q][r][s] of a stored class; every block is kept once produced.  Lets the
    block-restricted residual run where whole classes do not fit in host memory."""

    def __init__(self, provider, stored=CLASSES):
        self.provider = provider
        self.stored = tuple(stored)
        self.cache = {}

    def __contains__(self, cls):
        return cls in self.stored

    def __getitem__(self, cls):
        outer = self

        class _View:
            def __getitem__(self, key):
                k = (cls,) + tuple(int(x) for x in key)
                if k not in outer.cache:
                    outer.cache[k] = outer.provider(cls, *k[1:])
                return outer.cache[k]

        return _View()


def residual_blocks(f, classes, t1, t2, kc, blocks, r1_ks=None, callback=None):
    """R1 (at the momenta ``r1_ks``, default all) and R2 on the listed momentum blocks
    (ki, kj, ka) only, term by term as in ``residual`` (same intermediates, same order of the
    sums), computing each intermediate block only where a listed block needs it.
    ``classes``: a dict of whole classes or a ``LazyClasses``.  ``callback(step)``, if given,
    is called after each stage (progress reporting of long runs)."""
    N, no, nv = t1.shape
    eris = Eris(classes, kc)
    Foo, Fvv, Fov = f_intermediates(f, eris, t1, t2, kc, no)
    if callback:
        callback("F intermediates")
    tau = make_tau(t1, t2, kc, 0.5)
    R1 = t1_residual(f, eris, t1, t2, Foo, Fvv, Fov, ks=r1_ks)
    if callback:
        callback("R1")
    Fvt, Fot = _f_tilde(t1, Foo, Fvv, Fov)
    memo = {}

    def cached(tag, fn, *key):
        if (tag,) + key not in memo:
            memo[(tag,) + key] = fn(*key)
        return memo[(tag,) + key]

    def wmn(km, kn, ki):
        return cached("wmn", lambda a, b, c: w_mnij_block(eris, t1, tau, kc, a, b, c), km, kn, ki)

    def wr(km, kb, ke):
        return cached("wr", lambda a, b, c: w_mbej_block(eris, t1, t2, kc, a, b, c), km, kb, ke)

    def x(ki, kj, ka):
        return cached("x", lambda a, b, c: ring_x_block(eris, t1, t2, kc, wr, a, b, c), ki, kj, ka)

    out = {}
    for (ki, kj, ka) in blocks:
        kb = kc[ki, kj, ka]
        r = r2_block_nonladder(eris, t1, t2, tau, Fvt, Fot, kc, wmn, x, ki, kj, ka)
        for ke in range(N):
            W = cached("wabef", lambda a, b, c: w_abef_block(eris, t1, tau, kc, a, b, c), ka, kb, ke)
            r += 0.5 * _con("abef,ijef->ijab", W, tau[ki, kj, ke])
        out[(ki, kj, ka)] = r
        if callback:
            callback(f"R2 block {(ki, kj, ka)}")
    return R1, out


# --------------------------------------------------------------------------------------
# Energy (not printed in the paper; standard spin-orbital CCSD expression)
# --------------------------------------------------------------------------------------
def energy(f, classes: dict, t1, t2, kc):
    N, no, nv = t1.shape
    eris = Eris(classes, kc)
    e = 0j
    for k in range(N):
        e += np.sum(f[k, :no, no:] * t1[k])
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                e += 0.25 * np.sum(eris.block("oovv", ki, kj, ka) * t2[ki, kj, ka])
            e += 0.5 * _con("ijab,ia,jb->", eris.block("oovv", ki, kj, ki), t1[ki], t1[kj])
    return complex(e)


# --------------------------------------------------------------------------------------
# Update and iteration (Sec. 4.4: D, successive substitution, convergence test)
# --------------------------------------------------------------------------------------
def denominators(f, no, kc):
    """D_i^a = f_ii - f_aa and D_ij^ab = f_ii + f_jj - f_aa - f_bb (real diagonal)."""
    N = f.shape[0]
    eo = np.real(np.einsum("kii->ki", f[:, :no, :no]))
    ev = np.real(np.einsum("kaa->ka", f[:, no:, no:]))
    D1 = eo[:, :, None] - ev[:, None, :]
    nv = ev.shape[1]
    D2 = np.zeros((N, N, N, no, no, nv, nv))
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                kb = kc[ki, kj, ka]
                D2[ki, kj, ka] = (eo[ki][:, None, None, None] + eo[kj][None, :, None, None]
                                  - ev[ka][None, None, :, None] - ev[kb][None, None, None, :])
    return D1, D2


def residual_norm(R1, R2) -> float:
    return float(np.sqrt(np.sum(np.abs(R1) ** 2) + np.sum(np.abs(R2) ** 2)))


class Diis:
    """Pulay DIIS on the flattened (t1, t2); error vector e = t_new - t = R/D.

    B_ij = Re<e_i, e_j>, real coefficients from the bordered system, FIFO of ``space``
    vectors, extrapolation once two vectors are held.
    """

    def __init__(self, space: int):
        self.space = space
        self.vecs, self.errs = [], []

    def update(self, vec: np.ndarray, err: np.ndarray) -> np.ndarray:
        self.vecs.append(vec.copy())
        self.errs.append(err.copy())
        if len(self.vecs) > self.space:
            self.vecs.pop(0)
            self.errs.pop(0)
        m = len(self.vecs)
        if m < 2:
            return vec
        B = np.zeros((m + 1, m + 1))
        for i in range(m):
            for j in range(m):
                B[i, j] = np.real(np.vdot(self.errs[i], self.errs[j]))
        B[m, :m] = B[:m, m] = 1.0
        rhs = np.zeros(m + 1)
        rhs[m] = 1.0
        c = np.linalg.solve(B, rhs)[:m]
        out = np.zeros_like(vec)
        for ci, v in zip(c, self.vecs):
            out += ci * v
        return out


def solve(f, classes: dict, grid, max_iter=50, tol=1e-10, diis_space=0, t1=None, t2=None,
          callback=None):
    """Iterate t <- t + R/D (optionally DIIS-extrapolated) from t = 0 until ||R||_2 < tol.

    Starting from t = 0, the first update gives t0 = f(0), the start the paper uses.
    Returns dict(t1, t2, energy, iterations, rnorm, converged, history).
    """
    no = f.shape[1] - classes["vvvv"].shape[-1]
    kc = kconserv(grid)
    N = f.shape[0]
    nv = f.shape[1] - no
    if t1 is None:
        t1 = np.zeros((N, no, nv), dtype=np.complex128)
    if t2 is None:
        t2 = np.zeros((N, N, N, no, no, nv, nv), dtype=np.complex128)
    D1, D2 = denominators(f, no, kc)
    diis = Diis(diis_space) if diis_space > 0 else None
    hist = []
    it = 0
    converged = False
    rn = np.inf
    while True:
        R1, R2 = residual(f, classes, t1, t2, kc)
        rn = residual_norm(R1, R2)
        e = energy(f, classes, t1, t2, kc)
        hist.append((it, rn, e))
        if callback:
            callback(it, rn, e)
        if rn < tol:
            converged = True
            break
        if it >= max_iter:
            break
        n1 = t1.size
        new1 = t1 + R1 / D1
        new2 = t2 + R2 / D2
        if diis is not None:
            vec = np.concatenate([new1.ravel(), new2.ravel()])
            err = np.concatenate([(new1 - t1).ravel(), (new2 - t2).ravel()])
            vec = diis.update(vec, err)
            new1 = vec[:n1].reshape(t1.shape)
            new2 = vec[n1:].reshape(t2.shape)
        t1, t2 = new1, new2
        it += 1
    return dict(t1=t1, t2=t2, energy=energy(f, classes, t1, t2, kc), iterations=it, rnorm=rn,
                converged=converged, history=hist)
