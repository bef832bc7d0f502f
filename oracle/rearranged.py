"""The rearranged CCSD amplitude equations of Sec. 3.3, written out as a second oracle.

TEST INFRASTRUCTURE ONLY.  Like ``oracle.ccsd_k`` this module checks the GPU library and is
used by ``tests/`` alone; it shares no code with the GPU path.  It evaluates the right-hand
sides of the T1 and T2 equations in the paper's rearranged form (Sec. 3.3, "Rearrangement
of the basic equations"): the intermediates rho-check / rho-hat (Sec. 3.3.1), the
rearranged F-tilde with K-tilde and Z-tilde (Sec. 3.3.2, eqs. def_F_oo, def_F_vv,
def_F_ov, def_Z_oo, def_Z_vv, def_K), the T1 equation with L-tilde (eq. EqSingle,
def_L_oo, def_L_vv) and the T2 equation as the sum of its four parts (eq. EqDouble:
A-bar of eq. A_1st with C-tilde, W-tilde and J-tilde; A-check of eq. A_2nd with G-check,
Y-tilde^{abef} and V-tilde^{abef}; A-tilde of eq. A_3rd with X-tilde; A-hat of eq. A_4th
with G-hat, Y-tilde_{mnij} and V-tilde_{mnij}).  Since the rearrangement is exact, both
results must equal those of the original equations of Sec. 2 (``oracle.ccsd_k``), which
is the check this module exists for.

Readings of misprints in Sec. 3.3 (each one is forced by that equality, and the test
fails if any of them is reversed):
  * eq. def_F_oo: the K-tilde term enters as + (f + K-tilde), as in def_F_vv; the tau-tilde
    part of the original F_oo gives + 1/2 t_q^c K-tilde_p^c;
  * eq. A_1st: the arguments of zeta-tilde are (k_a, k_i): r and a sit at k_a, i and c at k_i;
  * eq. A_4th: the P_-(ab) partner is G-hat (defined after it), not G-check;
  * the leading T1 term f_p^g is read as in the original equations, f_ai = conj(f_ia).
The superscripts [ov], [oo], [vv] on the integrals of Sec. 3.3 name storage forms of one
integral; here every integral is taken from the stored classes through their symmetries.

Conventions as in ``oracle.ccsd_k``: t1[k][i][a]; t2[ki][kj][ka][i][j][a][b] with k_b fixed
by conservation; f[k][p][q] = <p|f|q> with occupied orbitals first.
"""
from __future__ import annotations

import numpy as np

from oracle.ccsd_k import Eris, _con

# The three readings of misprints listed above, as switches so that a test can reverse each
# one and see the equality with the original equations fail:
#   K_SIGN_FOO   sign of K-tilde inside (f +- K-tilde) in eq. def_F_oo (printed: -1)
#   ZETA_BAR     argument order of zeta-tilde in eq. A_1st: "ak" = (k_a, k_i) (printed: (k_i, k_a))
#   AHAT_PAIR    the P_-(ab) partner in eq. A_4th: "hat" = G-hat (printed: G-check)
READINGS = {"K_SIGN_FOO": +1, "ZETA_BAR": "ak", "AHAT_PAIR": "hat"}


def _fbar(f, eris, t1, t2, kc, no):
    """F-tilde of Sec. 3.3.2 at every k: (Foo[k](p,q), Fvv[k](g,h), Fov[k](p,g))."""
    N = t1.shape[0]
    fo = [f[k][:no, :no] for k in range(N)]
    fv = [f[k][no:, no:] for k in range(N)]
    fov = [f[k][:no, no:] for k in range(N)]
    # K-tilde_x^y(kbar) = sum_{r,c,khat} t_{r khat}^{c khat} <x kbar, r khat || y kbar, c khat>
    K = []
    for kb in range(N):
        acc = 0
        for kh in range(N):
            acc = acc + _con("rc,xryc->xy", t1[kh], eris.block("oovv", kb, kh, kb))
        K.append(acc)
    Foo, Fvv, Fov = [], [], []
    for kb in range(N):
        # eq. def_F_oo (the K-tilde term with + sign, see module docstring)
        foo = fo[kb] + 0.5 * _con("qc,pc->pq", t1[kb], fov[kb] + READINGS["K_SIGN_FOO"] * K[kb])
        for kh in range(N):
            foo = foo + _con("rc,prqc->pq", t1[kh], eris.block("ooov", kb, kh, kb))
        for ke in range(N):  # Z-tilde_{pq}^{ke}
            for kn in range(N):
                foo = foo + 0.5 * _con("qnef,pnef->pq", t2[kb, kn, ke], eris.block("oovv", kb, kn, ke))
        # eq. def_F_vv
        fvv = fv[kb] - 0.5 * _con("rg,rh->gh", t1[kb], fov[kb] + K[kb])
        for kh in range(N):
            fvv = fvv + _con("rc,rgch->gh", t1[kh], eris.block("ovvv", kh, kb, kh))
        for km in range(N):  # Z-tilde_{km}^{gh}
            for kn in range(N):
                fvv = fvv - 0.5 * _con("mngf,mnhf->gh", t2[km, kn, kb], eris.block("oovv", km, kn, kb))
        # eq. def_F_ov
        Foo.append(foo)
        Fvv.append(fvv)
        Fov.append(fov[kb] + K[kb])
    return Foo, Fvv, Fov


def residual(f, classes: dict, t1, t2, kc):
    """(R1, R2) of the rearranged equations EqSingle and EqDouble of Sec. 3.3."""
    N, no, nv = t1.shape
    eris = Eris(classes, kc)
    Foo, Fvv, Fov = _fbar(f, eris, t1, t2, kc, no)

    # ---------------- eq. EqSingle ----------------
    R1 = np.zeros_like(t1)
    for k in range(N):
        r = np.conj(f[k][:no, no:])
        r = r + _con("pc,gc->pg", t1[k], Fvv[k])
        r = r - _con("rg,rp->pg", t1[k], Foo[k])
        for kh in range(N):
            r = r + _con("pngf,nf->pg", t2[k, kh, k], Fov[kh])
            r = r + _con("rc,rgcp->pg", t1[kh], eris.block("ovvo", kh, k, kh))
        for km in range(N):  # - L-tilde_{p k, km}^{g}
            for kn in range(N):
                r = r - 0.5 * _con("mngf,mnpf->pg", t2[km, kn, k], eris.block("ooov", km, kn, k))
        for ke in range(N):  # + L-tilde_p^{g ke}
            for kn in range(N):
                kf = kc[k, kn, ke]
                r = r + 0.5 * _con("pnef,ngfe->pg", t2[k, kn, ke], eris.block("ovvv", kn, k, kf))
        R1[k] = r

    # ---------------- eq. EqDouble ----------------
    def W(kj, kn, kb):
        """W-tilde_{j kj, n kn}^{b kb, f kf} (eq. rearranged_W with J-tilde, eq. def_J) as [j,n,b,f];
        k_f = k_n + k_b - k_j."""
        kf = kc[kn, kb, kj]
        w = np.zeros((no, no, nv, nv), dtype=np.complex128)
        for ky in range(N):
            kx = kc[kj, ky, kb]
            # -1/2 t_{j kj, y ky}^{x kx, b kb} <n kn, y ky || f kf, x kx>
            w = w - 0.5 * _con("jyxb,nyfx->jnbf", t2[kj, ky, kx], eris.block("oovv", kn, ky, kf))
        w = w + _con("nbfj->jnbf", eris.block("ovvo", kn, kb, kf))
        w = w + _con("jc,nbfc->jnbf", t1[kj], eris.block("ovvv", kn, kb, kf))
        w = w - _con("rb,rnjf->jnbf", t1[kb], eris.block("ooov", kb, kn, kj))
        w = w - _con("rb,jc,rncf->jnbf", t1[kb], t1[kj], eris.block("oovv", kb, kn, kj))
        return w

    def Ctil(ki, kj, ka):
        """C-tilde_{i ki, j kj}^{a ka, b kb} (eq. def_C) as [i,j,a,b]."""
        kb = kc[ki, kj, ka]
        c = np.zeros((no, no, nv, nv), dtype=np.complex128)
        for kn in range(N):
            kf = kc[ki, kn, ka]
            assert kc[kn, kb, kj] == kf  # the shared f has one momentum in both factors
            c = c + _con("inaf,jnbf->ijab", t2[ki, kn, ka], W(kj, kn, kb))
        c = c - _con("rb,jc,raci->ijab", t1[kb], t1[kj], eris.block("ovvo", kb, ka, kj))
        return c

    Cb = {}
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                Cb[ki, kj, ka] = Ctil(ki, kj, ka)

    def Vvv(ka, kb, ke):
        """V-tilde^{a ka, b kb, e ke, f kf} = sum_r t_{r kb}^{b kb} <r kb, a ka || e ke, f kf>: [a,b,e,f]."""
        return _con("rb,raef->abef", t1[kb], eris.block("ovvv", kb, ka, ke))

    def Yvv(ka, kb, ke):
        """Y-tilde^{a ka, b kb, e ke, f kf} (eq. def_Y_vv) as [a,b,e,f]."""
        y = Vvv(ka, kb, ke) - _con("baef->abef", Vvv(kb, ka, ke))
        y = y - _con("baef->abef", eris.block("vvvv", kb, ka, ke))
        y = y - _con("sb,ra,sref->abef", t1[kb], t1[ka], eris.block("oovv", kb, ka, ke))
        return 0.5 * y

    def Voo(km, kn, ki):
        """V-tilde_{m km, n kn, i ki, j kj} = sum_c t_{j kj}^{c kj} <m km, n kn || i ki, c kj>: [m,n,i,j]."""
        kj = kc[km, kn, ki]
        return _con("jc,mnic->mnij", t1[kj], eris.block("ooov", km, kn, ki))

    def Yoo(km, kn, ki):
        """Y-tilde_{m km, n kn, i ki, j kj} (eq. def_Y_oo) as [m,n,i,j]."""
        kj = kc[km, kn, ki]
        y = Voo(km, kn, ki) - _con("mnji->mnij", Voo(km, kn, kj))
        y = y + eris.block("oooo", km, kn, ki)
        y = y + _con("ic,jd,mncd->mnij", t1[ki], t1[kj], eris.block("oovv", km, kn, ki))
        return 0.5 * y

    def block_terms(ki, kj, ka):
        """Every term of A-bar, A-check, A-tilde and A-hat for one block, except the
        P_-(ij) and P_-(ab) partners, which the caller adds from the partner blocks."""
        kb = kc[ki, kj, ka]
        t = {}
        # A-bar: conj(<ij||ab>) + the t1^4 term with zeta-tilde(k_a, k_i)
        t["drv"] = np.conj(eris.block("oovv", ki, kj, ka))
        if READINGS["ZETA_BAR"] == "ak":  # zeta-tilde_{ri}^{ac}(k_a, k_i) = t_{r ka}^{a ka} t_{i ki}^{c ki}
            za, zi = t1[ka], t1[ki]
        else:  # as printed, (k_i, k_a): t_{r ki}^{a ki} t_{i ka}^{c ka}
            za, zi = t1[ki], t1[ka]
        t["t4"] = _con("ra,ic,sb,jd,rscd->ijab", za, zi, t1[kb], t1[kj], eris.block("oovv", ka, kb, ki))
        # A-check
        t["eta_oooo"] = _con("ra,sb,rsij->ijab", t1[ka], t1[kb], eris.block("oooo", ka, kb, ki))
        t["Gchk"] = _con("jc,ra,sb,rsic->ijab", t1[kj], t1[ka], t1[kb], eris.block("ooov", ka, kb, ki)) \
            + _con("jc,icab->ijab", t1[kj], np.conj(eris.block("ovvv", ki, kj, ka)))
        Fvt = Fvv[kb] - 0.5 * _con("rb,rf->bf", t1[kb], Fov[kb])
        t["Fvv"] = _con("ijaf,bf->ijab", t2[ki, kj, ka], Fvt)
        y = 0
        for ke in range(N):
            y = y + _con("ijef,abef->ijab", t2[ki, kj, ke], Yvv(ka, kb, ke))
        t["Yvv"] = y
        # A-tilde: 1/4 t_{mn}^{ab} X-tilde_{mnij}
        x = 0
        for km in range(N):
            kn = kc[ka, kb, km]
            X = 0
            for ke in range(N):
                X = X + _con("ijef,mnef->mnij", t2[ki, kj, ke], eris.block("oovv", km, kn, ke))
            x = x + 0.25 * _con("mnab,mnij->ijab", t2[km, kn, ka], X)
        t["Xt"] = x
        # A-hat
        y = 0
        for km in range(N):
            kn = kc[ka, kb, km]
            y = y + _con("mnab,mnij->ijab", t2[km, kn, ka], Yoo(km, kn, ki))
        t["Yoo"] = y
        Fot = Foo[kj] + 0.5 * _con("jc,nc->nj", t1[kj], Fov[kj])
        t["Foo"] = -_con("inab,nj->ijab", t2[ki, kj, ka], Fot)
        t["eta_vvvv"] = -_con("ic,jd,bacd->ijab", t1[ki], t1[kj], eris.block("vvvv", kb, ka, ki))
        t["Ghat"] = _con("rb,ic,jd,racd->ijab", t1[kb], t1[ki], t1[kj], eris.block("ovvv", kb, ka, ki)) \
            + _con("rb,ijra->ijab", t1[kb], np.conj(eris.block("ooov", ki, kj, kb)))
        return t

    T = {}
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                T[ki, kj, ka] = block_terms(ki, kj, ka)

    R2 = np.zeros_like(t2)
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                kb = kc[ki, kj, ka]
                t, tij, tab = T[ki, kj, ka], T[kj, ki, ka], T[ki, kj, kb]
                sw_ij = lambda x: _con("jiab->ijab", x)  # noqa: E731
                sw_ab = lambda x: _con("ijba->ijab", x)  # noqa: E731
                # A-bar = P(ij)P(ab) C-tilde + driver + t1^4 term
                c = Cb[ki, kj, ka] - sw_ij(Cb[kj, ki, ka]) - sw_ab(Cb[ki, kj, kb]) + sw_ij(sw_ab(Cb[kj, ki, kb]))
                r = c + t["drv"] + t["t4"]
                # A-check = eta <oo||oo> + P(ij) G-check + P(ab) (t2 Fvt) + t2 Y-tilde^{abef}
                r = r + t["eta_oooo"] + t["Gchk"] - sw_ij(tij["Gchk"]) + t["Fvv"] - sw_ab(tab["Fvv"]) + t["Yvv"]
                # A-tilde
                r = r + t["Xt"]
                # A-hat = t2 Y-tilde_{mnij} - P(ij) (t2 Fot) - eta <vv||vv> + P(ab) G-hat
                g = "Ghat" if READINGS["AHAT_PAIR"] == "hat" else "Gchk"
                r = r + t["Yoo"] + t["Foo"] - sw_ij(tij["Foo"]) + t["eta_vvvv"] + t[g] - sw_ab(tab[g])
                R2[ki, kj, ka] = r
    return R1, R2
