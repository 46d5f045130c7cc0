"""Conventional FastMNMF (Sec. II-A), written separately in the paper's own notation.

TEST INFRASTRUCTURE.  It exists only to pin the distributed oracle: with one
subarray distributed FastMNMF is conventional FastMNMF (Sec. III-B, end), and
for any partition each subarray's IP step is the conventional IP step on that
subarray's observations while the MM steps are the conventional ones with the
block-diagonal transformation (Sec. III-B).  It deliberately shares nothing
with ``oracle/dfmnmf.py``: it keeps W_i (columns w_im), t_ikn, v_kjn and the
diagonal of Lambda_in, loops over frequency bins, and evaluates
eta_ijm = sum_{k,n} t_ikn v_kjn [Lambda_in]_mm as the double sum of eq. (5)
rather than in factorised form.  Meant for tiny inputs only.

Array conventions: x[i, j, m]; Wt[i] is the M x M matrix W_i; t[i, k, n];
v[k, j, n]; lam[i, n, m] = [Lambda_in]_mm.
"""
from __future__ import annotations

import numpy as np


class FastMNMF:
    """State and update rules of conventional FastMNMF, eqs. (4)-(10)."""

    def __init__(self, x, Wt, t, v, lam, floor=1e-6):
        self.x = np.asarray(x, dtype=np.complex128)
        self.Wt = np.array(Wt, dtype=np.complex128)
        self.t = np.array(t, dtype=np.float64)
        self.v = np.array(v, dtype=np.float64)
        self.lam = np.array(lam, dtype=np.float64)
        self.floor = floor

    @property
    def shape(self):
        I, J, M = self.x.shape
        return I, J, M, self.t.shape[2], self.t.shape[1]

    def eta(self):
        """eta_ijm = sum_{k,n} t_ikn v_kjn [Lambda_in]_mm, floored (eq. (5) definition, Sec. IV-A)."""
        I, J, M, N, K = self.shape
        e = np.zeros((I, J, M))
        for i in range(I):
            for n in range(N):
                for k in range(K):
                    e[i] += self.t[i, k, n] * np.outer(self.v[k, :, n], self.lam[i, n, :])
        return np.maximum(e, self.floor)

    def decorrelated(self):
        """y_ij = W_i^H x_ij."""
        I = self.x.shape[0]
        return np.stack([self.x[i] @ self.Wt[i].conj() for i in range(I)])

    def update_W(self):
        """IP, eqs. (5)-(7): rows m in ascending order, each using the current W_i."""
        I, J, M, _, _ = self.shape
        e = self.eta()
        for i in range(I):
            for m in range(M):
                Qim = np.zeros((M, M), dtype=np.complex128)
                for j in range(J):
                    Qim += np.outer(self.x[i, j], self.x[i, j].conj()) / e[i, j, m]
                Qim /= J
                em = np.zeros(M)
                em[m] = 1.0
                A = self.Wt[i].conj().T @ Qim
                try:
                    w = np.linalg.solve(A, em)
                except np.linalg.LinAlgError:
                    w = np.linalg.pinv(A) @ em
                nrm = max(float(np.real(w.conj() @ Qim @ w)), self.floor)
                self.Wt[i][:, m] = w / np.sqrt(nrm)

    def _ratio(self, numer, denom):
        return np.sqrt(numer / np.maximum(denom, self.floor))

    def update_t(self):
        """Eq. (8)."""
        I, J, M, N, K = self.shape
        y2 = np.abs(self.decorrelated()) ** 2
        e = self.eta()
        new = np.empty_like(self.t)
        for i in range(I):
            for k in range(K):
                for n in range(N):
                    w = np.outer(self.v[k, :, n], self.lam[i, n, :])          # [J, M]
                    new[i, k, n] = self.t[i, k, n] * self._ratio(
                        np.sum(w * y2[i] / e[i] ** 2), np.sum(w / e[i]))
        self.t = new

    def update_v(self):
        """Eq. (9)."""
        I, J, M, N, K = self.shape
        y2 = np.abs(self.decorrelated()) ** 2
        e = self.eta()
        new = np.empty_like(self.v)
        for k in range(K):
            for n in range(N):
                for j in range(J):
                    w = np.outer(self.t[:, k, n], np.ones(M)) * self.lam[:, n, :]  # [I, M]
                    new[k, j, n] = self.v[k, j, n] * self._ratio(
                        np.sum(w * y2[:, j] / e[:, j] ** 2), np.sum(w / e[:, j]))
        self.v = new

    def update_lam(self):
        """Eq. (10)."""
        I, J, M, N, K = self.shape
        y2 = np.abs(self.decorrelated()) ** 2
        e = self.eta()
        new = np.empty_like(self.lam)
        for i in range(I):
            for n in range(N):
                h = self.t[i, :, n] @ self.v[:, :, n]                          # [J]
                for m in range(M):
                    new[i, n, m] = self.lam[i, n, m] * self._ratio(
                        np.sum(h * y2[i, :, m] / e[i, :, m] ** 2), np.sum(h / e[i, :, m]))
        self.lam = new

    def iteration(self):
        """IP then eqs. (8), (9), (10), eta refreshed after each (Sec. II-A)."""
        self.update_W()
        self.update_t()
        self.update_v()
        self.update_lam()

    def cost(self):
        """Eq. (4)."""
        J = self.x.shape[1]
        e = self.eta()
        y2 = np.abs(self.decorrelated()) ** 2
        c = np.sum(y2 / e + np.log(e))
        for Wi in self.Wt:
            c -= J * np.log(np.abs(np.linalg.det(Wi)) ** 2)
        return float(c)
