"""Exact float64 enumeration of shaken dynamics on small graphs.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything is written from the definitions of section 2 of the paper:
  * the pair Hamiltonian of Definition 2.2 in matrix form,
        H(s1, s2) = -<s1, Jo s2> - q <s1, s2> - <lam, s1> - <lam, s2>,
    with Jo[x, y] = J_xy for (x, y) in E^o (equation ham21 and the matrix form
    that follows it);
  * the Ising Hamiltonian H(s) = -sum_{edges} J s_x s_y - 2 sum_x lam_x s_x
    (equation ham1), i.e. -<(1/2) Jsym s + 2 lam, s> with Jsym = Jo + Jo^T;
  * the half-step kernels as normalised Boltzmann weights of the pair
    Hamiltonian, P^{1->2}(s, s') = exp(-b H(s, s')) / sum_z exp(-b H(s, z)) and
    P^{2->1}(s', t) = exp(-b H(t, s')) / sum_z exp(-b H(z, s'));
  * P^sh = P^{1->2} P^{2->1};
  * pi(s) = Zfwd_s / Z with Zfwd_s = sum_t exp(-b H(s, t)) (Theorem 2.3), and
    pi^b(s1, s2) = exp(-b H(s1, s2)) / Z;
  * the alternate dynamics P^alt((s1,s2),(t1,t2)) = P^{1->2}(s1,t2) P^{2->1}(t2,t1).

State index i <-> configuration with spin x = +1 iff bit x of i is set.
"""
from __future__ import annotations

import numpy as np


def states(n: int) -> np.ndarray:
    i = np.arange(2 ** n, dtype=np.int64)[:, None]
    return np.where((i >> np.arange(n)) & 1, 1.0, -1.0)


def index_of(sigma) -> int:
    s = np.asarray(sigma)
    return int(sum(1 << x for x in range(len(s)) if s[x] > 0))


class Model:
    def __init__(self, n, src, dst, J=None, lam=None, q=1.0, beta=1.0):
        self.n = int(n)
        self.src = np.asarray(src, dtype=np.int64)
        self.dst = np.asarray(dst, dtype=np.int64)
        self.J = np.ones(len(self.src)) if J is None else np.asarray(J, dtype=np.float64)
        self.lam = np.zeros(self.n) if lam is None else np.asarray(lam, dtype=np.float64)
        self.q = float(q)
        self.beta = float(beta)
        Jo = np.zeros((self.n, self.n))
        for e in range(len(self.src)):
            Jo[self.src[e], self.dst[e]] += self.J[e]
        self.Jo = Jo
        self._S = None

    @property
    def S(self) -> np.ndarray:
        """all 2^n configurations (rows), built on first use"""
        if self._S is None:
            if self.n > 16:
                raise ValueError("enumeration limited to 16 spins")
            self._S = states(self.n)
        return self._S

    def field12_of(self, s) -> np.ndarray:
        """h^{1->2}(s) for one configuration s"""
        s = np.asarray(s, dtype=np.float64)
        return self.Jo.T @ s + self.q * s + self.lam

    def field21_of(self, s) -> np.ndarray:
        """h^{2->1}(s') for one configuration s'"""
        s = np.asarray(s, dtype=np.float64)
        return self.Jo @ s + self.q * s + self.lam

    def gibbs_H_of(self, s) -> float:
        """H(s) of equation ham1 for one configuration"""
        s = np.asarray(s, dtype=np.float64)
        return float(-0.5 * s @ (self.Jo + self.Jo.T) @ s - 2.0 * self.lam @ s)

    # ---------------------------------------------------------- Hamiltonians
    def pair_H(self) -> np.ndarray:
        """Matrix of H(s1, s2) over all pairs of states (Definition 2.2)."""
        S = self.S
        lam_s = S @ self.lam
        return -(S @ self.Jo @ S.T) - self.q * (S @ S.T) - lam_s[:, None] - lam_s[None, :]

    def gibbs_H(self) -> np.ndarray:
        """H(s) of equation ham1 for every state."""
        S = self.S
        Jsym = self.Jo + self.Jo.T
        return -0.5 * np.einsum("ix,xy,iy->i", S, Jsym, S) - 2.0 * (S @ self.lam)

    # -------------------------------------------------------------- kernels
    def _boltz_rows(self, M):
        """row-normalised exp(-beta M), computed stably"""
        A = -self.beta * M
        A = A - A.max(axis=1, keepdims=True)
        W = np.exp(A)
        return W / W.sum(axis=1, keepdims=True)

    def P12(self) -> np.ndarray:
        return self._boltz_rows(self.pair_H())

    def P21(self) -> np.ndarray:
        # P^{2->1}(s', t) = exp(-b H(t, s')) / sum_z exp(-b H(z, s'))
        return self._boltz_rows(self.pair_H().T)

    def fields12(self) -> np.ndarray:
        """h^{1->2}_x(s) = (Jo^T s)_x + q s_x + lam_x for every state (rows)."""
        S = self.S
        return S @ self.Jo + self.q * S + self.lam[None, :]

    def fields21(self) -> np.ndarray:
        """h^{2->1}_x(s') = (Jo s')_x + q s'_x + lam_x for every state (rows)."""
        S = self.S
        return S @ self.Jo.T + self.q * S + self.lam[None, :]

    def product_form(self, H) -> np.ndarray:
        """prod_x exp(b h_x(s) s'_x) / (2 cosh(b h_x(s))) for fields H[s, x]."""
        b = self.beta
        # log of each factor = b h s' - log(2 cosh(b h))
        lc = np.logaddexp(b * H, -b * H)  # log(2 cosh(b h))
        logP = b * (H @ self.S.T) - lc.sum(axis=1, keepdims=True)
        return np.exp(logP)

    def Psh(self) -> np.ndarray:
        return self.P12() @ self.P21()

    # ------------------------------------------------------------- measures
    def pi(self) -> np.ndarray:
        A = -self.beta * self.pair_H()
        c = A.max()
        zf = np.exp(A - c).sum(axis=1)
        return zf / zf.sum()

    def pib(self) -> np.ndarray:
        A = -self.beta * self.pair_H()
        W = np.exp(A - A.max())
        return W / W.sum()

    def gibbs(self) -> np.ndarray:
        A = -self.beta * self.gibbs_H()
        W = np.exp(A - A.max())
        return W / W.sum()

    def Palt(self) -> np.ndarray:
        """P^alt over pair states; pair index = i1 * 2^n + i2."""
        P12 = self.P12()
        P21 = self.P21()
        N = 2 ** self.n
        # P[(s1,s2),(t1,t2)] = P12[s1,t2] * P21[t2,t1], independent of s2
        K = np.einsum("ab,bc->acb", P12, P21)  # [s1, t1, t2]
        K = K.reshape(N, N * N)
        return np.repeat(K, N, axis=0)


def torus_edges(L: int):
    """E^o of the L x L torus: (x, x_up) and (x, x_right), site = row*L + col,
    up = row+1, right = col+1 (mod L)."""
    src, dst = [], []
    for r in range(L):
        for c in range(L):
            x = r * L + c
            src.append(x); dst.append(((r + 1) % L) * L + c)
            src.append(x); dst.append(r * L + (c + 1) % L)
    return np.array(src), np.array(dst)
