"""Brute-force second quantization on Slater determinants (test helper).

Independent of the coupled-cluster equations: it builds the Hamiltonian
H = sum h_PQ a+_P a_Q + 1/4 sum <PQ||RS> a+_P a+_Q a_S a_R and the cluster operator
T = sum t_i^a a+_a a_i + 1/4 sum t_ij^ab a+_a a+_b a_j a_i as matrices on the
fixed-particle-number determinant space, and evaluates
    R_mu = <Phi_mu| exp(-T) H_N exp(T) |Phi>,   E = <Phi| H_N exp(T) |Phi>
exactly.  A spin orbital is a (k, p) pair with global index P = k*n + p; p < n_occ is
occupied in the reference |Phi>.
"""
from __future__ import annotations

import itertools

import numpy as np


def _sign_below(det: int, pos: int) -> int:
    return -1 if bin(det & ((1 << pos) - 1)).count("1") % 2 else 1


def annihilate(det, pos):
    if not (det >> pos) & 1:
        return None, 0
    return det ^ (1 << pos), _sign_below(det, pos)


def create(det, pos):
    if (det >> pos) & 1:
        return None, 0
    return det | (1 << pos), _sign_below(det, pos)


class FockSpace:
    def __init__(self, n_orb: int, n_elec: int):
        self.M = n_orb
        self.dets = [sum(1 << p for p in c) for c in itertools.combinations(range(n_orb), n_elec)]
        self.index = {d: i for i, d in enumerate(self.dets)}
        self.D = len(self.dets)

    def one_body(self, h: np.ndarray) -> np.ndarray:
        """Matrix of sum_PQ h[P,Q] a+_P a_Q."""
        Mat = np.zeros((self.D, self.D), dtype=np.complex128)
        nz = np.argwhere(np.abs(h) > 0)
        for col, det in enumerate(self.dets):
            for P, Q in nz:
                d1, s1 = annihilate(det, Q)
                if d1 is None:
                    continue
                d2, s2 = create(d1, P)
                if d2 is None:
                    continue
                Mat[self.index[d2], col] += h[P, Q] * s1 * s2
        return Mat

    def two_body(self, g: np.ndarray) -> np.ndarray:
        """Matrix of 1/4 sum <PQ||RS> a+_P a+_Q a_S a_R = sum_{P<Q,R<S} <PQ||RS> a+_P a+_Q a_S a_R
        for antisymmetric g."""
        Mat = np.zeros((self.D, self.D), dtype=np.complex128)
        M = self.M
        for col, det in enumerate(self.dets):
            occ = [p for p in range(M) if (det >> p) & 1]
            for R, S in itertools.combinations(occ, 2):
                d1, s1 = annihilate(det, R)
                d2, s2 = annihilate(d1, S)
                emp = [p for p in range(M) if not (d2 >> p) & 1]
                for P, Q in itertools.combinations(emp, 2):
                    val = g[P, Q, R, S]
                    if val == 0:
                        continue
                    d3, s3 = create(d2, Q)
                    d4, s4 = create(d3, P)
                    Mat[self.index[d4], col] += val * s1 * s2 * s3 * s4
        return Mat

    def vector(self, det: int, sign: int = 1) -> np.ndarray:
        v = np.zeros(self.D, dtype=np.complex128)
        v[self.index[det]] = sign
        return v


def expm_nilpotent(T: np.ndarray, v: np.ndarray, sign: float = 1.0) -> np.ndarray:
    """exp(sign*T) v for nilpotent T (excitation operators), by the terminating series."""
    out = v.copy()
    term = v.copy()
    for k in range(1, 64):
        term = sign * (T @ term) / k
        if not np.any(term):
            break
        out = out + term
    return out


def dense_supercell(f, eri_full, t1, t2, kc, no):
    """Block (k-labelled) inputs -> dense arrays over global spin orbitals P = k*n + p,
    with zeros where momentum is not conserved."""
    N, n = f.shape[0], f.shape[1]
    nv = n - no
    M = N * n
    F = np.zeros((M, M), dtype=np.complex128)
    G = np.zeros((M, M, M, M), dtype=np.complex128)
    T1 = np.zeros((M, M), dtype=np.complex128)  # T1[A, I] coefficient of a+_A a_I
    T2 = np.zeros((M, M, M, M), dtype=np.complex128)  # T2[A, B, I, J] = t_IJ^AB
    for k in range(N):
        F[k * n:(k + 1) * n, k * n:(k + 1) * n] = f[k]
        for i in range(no):
            for a in range(nv):
                T1[k * n + no + a, k * n + i] = t1[k, i, a]
    for kp in range(N):
        for kq in range(N):
            for kr in range(N):
                ks = kc[kp, kq, kr]
                G[kp * n:(kp + 1) * n, kq * n:(kq + 1) * n, kr * n:(kr + 1) * n,
                  ks * n:(ks + 1) * n] = eri_full[kp, kq, kr]
                for i in range(no):
                    for j in range(no):
                        for a in range(nv):
                            for b in range(nv):
                                T2[kr * n + no + a, ks * n + no + b, kp * n + i, kq * n + j] = \
                                    t2[kp, kq, kr, i, j, a, b]
    return F, G, T1, T2


def brute_force_residual(f, eri_full, t1, t2, kc):
    """Exact (R1, R2, E) of exp(-T) H_N exp(T) projected on singles and doubles.

    ``eri_full`` holds every orbital class: [kp,kq,kr][p][q][r][s] over all n orbitals.
    The one-body part of H is h = f - sum_m <P m||Q m> (m occupied), so that the Fock
    operator built from h and the integrals equals f.
    """
    N, n = f.shape[0], f.shape[1]
    no = t1.shape[1]
    nv = n - no
    M = N * n
    F, G, T1m, T2m = dense_supercell(f, eri_full, t1, t2, kc, no)
    occ = [k * n + i for k in range(N) for i in range(no)]
    h = F - sum(G[:, m, :, m] for m in occ)
    fs = FockSpace(M, len(occ))
    H = fs.one_body(h) + fs.two_body(G)
    ref = sum(1 << p for p in occ)
    phi = fs.vector(ref)
    e_ref = np.vdot(phi, H @ phi)
    HN = H - e_ref * np.eye(fs.D)
    # cluster operator matrix
    T = fs.one_body(T1m)
    # 1/4 sum t_ij^ab a+_a a+_b a_j a_i  ==  two_body with g[a,b,i,j] = t_ij^ab
    T = T + fs.two_body(T2m)
    v = expm_nilpotent(T, phi, 1.0)
    E = np.vdot(phi, HN @ v)
    x = expm_nilpotent(T, HN @ v, -1.0)

    R1 = np.zeros_like(t1)
    for k in range(N):
        for i in range(no):
            for a in range(nv):
                I, A = k * n + i, k * n + no + a
                d1, s1 = annihilate(ref, I)
                d2, s2 = create(d1, A)
                R1[k, i, a] = s1 * s2 * x[fs.index[d2]]
    R2 = np.zeros_like(t2)
    for ki in range(N):
        for kj in range(N):
            for ka in range(N):
                kb = kc[ki, kj, ka]
                for i in range(no):
                    for j in range(no):
                        for a in range(nv):
                            for b in range(nv):
                                I, J = ki * n + i, kj * n + j
                                A, B = ka * n + no + a, kb * n + no + b
                                if I == J or A == B:
                                    continue
                                d, s = annihilate(ref, I)
                                d, s2 = annihilate(d, J)
                                d, s3 = create(d, B)
                                d, s4 = create(d, A)
                                R2[ki, kj, ka, i, j, a, b] = s * s2 * s3 * s4 * x[fs.index[d]]
    return R1, R2, complex(E)


def nonconserving_double_projection(f, eri_full, t1, t2, kc):
    """max |<Phi_ij^ab| exp(-T) H_N exp(T) |Phi>| over doubles with k_i + k_j != k_a + k_b."""
    N, n = f.shape[0], f.shape[1]
    no = t1.shape[1]
    nv = n - no
    F, G, T1m, T2m = dense_supercell(f, eri_full, t1, t2, kc, no)
    occ = [k * n + i for k in range(N) for i in range(no)]
    vir = [k * n + no + a for k in range(N) for a in range(nv)]
    h = F - sum(G[:, m, :, m] for m in occ)
    fs = FockSpace(N * n, len(occ))
    H = fs.one_body(h) + fs.two_body(G)
    ref = sum(1 << p for p in occ)
    phi = fs.vector(ref)
    HN = H - np.vdot(phi, H @ phi) * np.eye(fs.D)
    T = fs.one_body(T1m) + fs.two_body(T2m)
    x = expm_nilpotent(T, HN @ expm_nilpotent(T, phi, 1.0), -1.0)
    worst, count = 0.0, 0
    for I, J in itertools.combinations(occ, 2):
        for A, B in itertools.combinations(vir, 2):
            if kc[I // n, J // n, A // n] == B // n:
                continue
            d = ref ^ (1 << I) ^ (1 << J) | (1 << A) | (1 << B)
            worst = max(worst, abs(x[fs.index[d]]))
            count += 1
    return worst, count


def fci_energies(f, eri_full, kc, no):
    """Eigenvalues of H_N (relative to the reference energy) and the reference weights."""
    N, n = f.shape[0], f.shape[1]
    M = N * n
    zt1 = np.zeros((N, no, n - no), dtype=np.complex128)
    zt2 = np.zeros((N, N, N, no, no, n - no, n - no), dtype=np.complex128)
    F, G, _, _ = dense_supercell(f, eri_full, zt1, zt2, kc, no)
    occ = [k * n + i for k in range(N) for i in range(no)]
    h = F - sum(G[:, m, :, m] for m in occ)
    fs = FockSpace(M, len(occ))
    H = fs.one_body(h) + fs.two_body(G)
    ref = sum(1 << p for p in occ)
    phi = fs.vector(ref)
    e_ref = np.vdot(phi, H @ phi).real
    w, U = np.linalg.eigh(H)
    weights = np.abs(U[fs.index[ref], :]) ** 2
    return w - e_ref, weights
