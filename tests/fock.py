"""Brute-force second-quantised checker in the full Fock space (tiny systems only).

Used to pin the oracle: determinant states, the ab initio Hamiltonian of
Sec. II.B written literally with spin-orbital creation and annihilation
operators, and one-body exponentials, all with no reference to the oracle's
orbital-space formulas.

Spin orbitals: alpha orbital p -> index p, beta orbital p -> N + p.
Occupation-number basis state b (an integer bit mask); a+_k acting on b
sets bit k with the Jordan-Wigner sign (-1)^(number of occupied k' < k).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


class FockSpace:
    def __init__(self, N: int):
        self.N = N
        self.M = 2 * N
        self.dim = 1 << self.M
        states = np.arange(self.dim)
        self._cre = []
        for k in range(self.M):
            src = states[((states >> k) & 1) == 0]
            below = src & ((1 << k) - 1)
            parity = np.array([bin(int(b)).count("1") & 1 for b in below])
            sign = np.where(parity == 1, -1.0, 1.0)
            self._cre.append((src, src | (1 << k), sign))

    # elementary operators on state vectors -------------------------------
    def cre(self, k, v):
        src, dst, sign = self._cre[k]
        out = np.zeros_like(v)
        out[dst] = sign * v[src]
        return out

    def ann(self, k, v):
        src, dst, sign = self._cre[k]
        out = np.zeros_like(v)
        out[src] = sign * v[dst]
        return out

    def vacuum(self):
        v = np.zeros(self.dim, dtype=np.complex128)
        v[0] = 1.0
        return v

    # states ----------------------------------------------------------------
    def determinant(self, phi_a, phi_b):
        """c+_{a,1} ... c+_{a,na} c+_{b,1} ... c+_{b,nb} |0>, c+_{s,i} = sum_p phi_pi a+_{p s}.

        The rightmost operator acts first, so apply the beta orbitals in
        reverse order, then the alpha orbitals in reverse order.
        """
        v = self.vacuum()
        N = self.N
        for offset, phi in ((N, phi_b), (0, phi_a)):
            for i in reversed(range(phi.shape[1])):
                w = np.zeros_like(v)
                for p in range(N):
                    if phi[p, i] != 0:
                        w = w + phi[p, i] * self.cre(offset + p, v)
                v = w
        return v

    # operators ---------------------------------------------------------------
    def one_body(self, A, v):
        """sum_{pq, s} A_pq a+_{p s} a_{q s} |v>."""
        N = self.N
        out = np.zeros_like(v)
        for s in (0, N):
            for q in range(N):
                aq = self.ann(s + q, v)
                if not np.any(aq):
                    continue
                for p in range(N):
                    if A[p, q] != 0:
                        out = out + A[p, q] * self.cre(s + p, aq)
        return out

    def hamiltonian(self, h1, L, v):
        """H|v> with H = sum h_pq a+_p a_q + 1/2 sum (pr|qs) a+_p a+_q a_s a_r (Eq. Habinitio),
        (pr|qs) = sum_g L_g,pr L_g,qs, all spin labels summed literally."""
        N = self.N
        eri = np.einsum("gpr,gqs->prqs", L, L)
        out = self.one_body(h1, v)
        for s1 in (0, N):            # spin of p and r
            for s2 in (0, N):        # spin of q and s
                for r in range(N):
                    ar = self.ann(s1 + r, v)
                    if not np.any(ar):
                        continue
                    for s in range(N):
                        asr = self.ann(s2 + s, ar)
                        if not np.any(asr):
                            continue
                        for q in range(N):
                            aq = self.cre(s2 + q, asr)
                            if not np.any(aq):
                                continue
                            for p in range(N):
                                c = eri[p, r, q, s]
                                if c != 0:
                                    out = out + 0.5 * c * self.cre(s1 + p, aq)
        return out

    def one_body_matrix(self, A):
        """Dense Fock-space matrix of sum_{pq,s} A_pq a+_{ps} a_{qs}."""
        M = np.zeros((self.dim, self.dim), dtype=np.complex128)
        for b in range(self.dim):
            e = np.zeros(self.dim, dtype=np.complex128)
            e[b] = 1.0
            M[:, b] = self.one_body(A, e)
        return M

    def expm_one_body(self, A, v):
        return scipy.linalg.expm(self.one_body_matrix(A)) @ v


# ---------------------------------------------------------------------------
# Multi-determinant trials built from excitation operators
# ---------------------------------------------------------------------------

def _mo_cre(fs, C, off, x, v):
    """a+ of orbital x (column x of C) on the Fock vector v."""
    out = np.zeros_like(v)
    for p in range(C.shape[0]):
        if C[p, x] != 0:
            out = out + C[p, x] * fs.cre(off + p, v)
    return out


def _mo_ann(fs, C, off, x, v):
    out = np.zeros_like(v)
    for p in range(C.shape[0]):
        if C[p, x] != 0:
            out = out + C[p, x] * fs.ann(off + p, v)
    return out


def excitation_trial(fs, C, nel, coeff, exc):
    """sum_a c_a t_a |psi_0>, t_a = prod_s prod_m a+_{s,q_m} a_{s,h_m} applied in
    Fock space; psi_0 per spin is the first nel[s] columns of C[s], and exc[a]
    holds per spin the (holes, particles) orbital indices of determinant a."""
    N = fs.N
    psi0 = fs.determinant(C[0][:, :nel[0]], C[1][:, :nel[1]])
    out = np.zeros_like(psi0)
    for ca, spins in zip(coeff, exc):
        v = psi0
        for s, (holes, parts) in enumerate(spins):
            for h, q in zip(holes, parts):
                v = _mo_cre(fs, C[s], s * N, q, _mo_ann(fs, C[s], s * N, h, v))
        out = out + ca * v
    return out
