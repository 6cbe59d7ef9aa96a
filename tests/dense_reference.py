"""Independent dense-matrix construction of the discrete registration operators on tiny grids.

Test infrastructure.  Shares no code with the oracle or the HIP library: every operator is an
explicit matrix built from DFT matrices and Kronecker products, and the forward map of the state
equation is the matrix power Phi(v)^{n_t} m_T with Phi = I + h L + h^2 L^2 / 2 (two-stage explicit
RK2 applied to the linear autonomous transport equation, Sec. 4).  The Jacobian of m_{n_t} with
respect to v is obtained by differentiating that product with the product rule, so the Gauss-Newton
Hessian is H = F_Nyq (beta_v A + K J^T J) F_Nyq (Sec. 3.3, Sec. 4) and the reduced gradient is
g = F_Nyq (beta_v A v - K J^T (m_R - m_{n_t})).

Flattening: scalar fields row-major (i1 * n2 + i2); vector fields [component][i1][i2].
"""
from __future__ import annotations

import numpy as np


def dft(n):
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def wav(n, zero_nyquist=True):
    k = np.array([j if j < n // 2 else j - n for j in range(n)], dtype=float)
    if zero_nyquist:
        k[n // 2] = 0.0
    return k


class Dense:
    def __init__(self, n1, n2, nt, norm="H1", constraint="divfree", beta_v=1e-2, beta_w=0.0):
        self.n1, self.n2, self.nt = n1, n2, nt
        self.N = n1 * n2
        self.h = 1.0 / nt
        self.beta_v, self.beta_w = beta_v, beta_w
        F2 = np.kron(dft(n1), dft(n2))
        F2i = np.conj(F2).T / self.N
        self.F2, self.F2i = F2, F2i
        k1 = np.repeat(wav(n1), n2)
        k2 = np.tile(wav(n2), n1)
        self.k1, self.k2 = k1, k2
        ksq = k1 ** 2 + k2 ** 2

        def mult(sym):
            m = F2i @ np.diag(sym) @ F2
            assert np.abs(m.imag).max() < 1e-10
            return m.real

        # 1D derivative matrices combined by Kronecker products (d1 acts on i1, d2 on i2)
        D1 = (np.conj(dft(n1)).T / n1) @ np.diag(1j * wav(n1)) @ dft(n1)
        D2 = (np.conj(dft(n2)).T / n2) @ np.diag(1j * wav(n2)) @ dft(n2)
        self.D1 = np.kron(D1.real, np.eye(n2))
        self.D2 = np.kron(np.eye(n1), D2.real)
        keep1 = np.array([j != n1 // 2 for j in range(n1)])
        keep2 = np.array([j != n2 // 2 for j in range(n2)])
        keep = np.kron(keep1, keep2).astype(float)
        Pn = mult(keep)
        self.Pnyq = np.block([[Pn, np.zeros_like(Pn)], [np.zeros_like(Pn), Pn]])
        Ahat = ksq if norm == "H1" else ksq ** 2
        Am = mult(Ahat)
        self.A = np.block([[Am, np.zeros_like(Am)], [np.zeros_like(Am), Am]])
        inv = np.where(ksq > 0, 1.0 / np.where(ksq > 0, ksq, 1.0), 0.0)
        if constraint == "none":
            c = np.zeros_like(ksq)
        elif constraint == "divfree":
            c = np.where(ksq > 0, 1.0, 0.0)
        else:
            Mhat = 1.0 + beta_v * Ahat / (beta_w * np.where(ksq > 0, ksq, 1.0) * (ksq + 1.0))
            c = np.where(ksq > 0, 1.0 / Mhat, 0.0)
        P11, P12, P22 = mult(c * k1 * k1 * inv), mult(c * k1 * k2 * inv), mult(c * k2 * k2 * inv)
        I = np.eye(self.N)
        self.K = np.block([[I - P11, -P12], [-P12, I - P22]])

    # transport operator L_v = -(diag(v1) D1 + diag(v2) D2) and its derivative in v
    def L(self, v):
        return -(np.diag(v[: self.N]) @ self.D1 + np.diag(v[self.N:]) @ self.D2)

    def Q(self, u):
        """dL[vt] u = Q(u) vt with Q(u) = -[diag(D1 u) | diag(D2 u)]."""
        return -np.hstack([np.diag(self.D1 @ u), np.diag(self.D2 @ u)])

    def Phi(self, v):
        L = self.L(v)
        h = self.h
        return np.eye(self.N) + h * L + 0.5 * h * h * (L @ L)

    def forward(self, v, mT):
        P = self.Phi(v)
        m = mT.copy()
        for _ in range(self.nt):
            m = P @ m
        return m

    def jacobian(self, v, mT):
        """d m_{n_t} / d v of the product Phi(v)^{n_t} m_T (product rule)."""
        L = self.L(v)
        P = self.Phi(v)
        h = self.h
        ms = [mT.copy()]
        for _ in range(self.nt):
            ms.append(P @ ms[-1])
        J = np.zeros((self.N, 2 * self.N))
        Ppow = np.eye(self.N)
        for j in range(self.nt - 1, -1, -1):
            mj = ms[j]
            dPhi = h * self.Q(mj) + 0.5 * h * h * (self.Q(L @ mj) + L @ self.Q(mj))
            J += Ppow @ dPhi
            Ppow = Ppow @ P
        return J

    def hessian_gn(self, v, mT):
        J = self.jacobian(v, mT)
        return self.Pnyq @ (self.beta_v * self.A + self.K @ (J.T @ J)) @ self.Pnyq

    def gradient(self, v, mT, mR):
        J = self.jacobian(v, mT)
        r = mR - self.forward(v, mT)
        return self.Pnyq @ (self.beta_v * self.A @ v - self.K @ (J.T @ r))
