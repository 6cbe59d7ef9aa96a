"""FP64 reference of the learned warm-start network (oracle; test infrastructure only).

The network is a Fourier neural operator (Li, Kovachki, Azizzadenesheli, Liu, Bhattacharya, Stuart
and Anandkumar, "Fourier neural operator for parametric partial differential equations", ICLR 2021)
that maps an image pair (m_T, m_R) on the periodic grid to an initial velocity for the Gauss-Newton
solve of Alg. 1.  It is not part of the paper; its sizes are fixed: 4 Fourier layers of width 32,
16 retained modes per axis, a 64-wide projection.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may import this
module.  It shares nothing with the HIP library: the flat parameter layout and the definition of the
network below are an interface that both sides implement on their own.

Network (arrays shaped (batch, channel, n1, n2); x = 2 pi i / n):
  a     = [m_T, D1 m_T, D2 m_T, (D1 m_T)^2, D1 m_T D2 m_T, (D2 m_T)^2, r, r D1 m_T, r D2 m_T]
          9 input features: D = periodic central difference (u(i+1) - u(i-1)) / (2 h), h = 2 pi / n;
          r = (m_R - m_T) / s with s = sqrt(mean((m_R - m_T)^2)) (r = 0 if s = 0).  To first order
          the velocity is linear in the misfit, so the network predicts v / s: the warm start is
          v0 = s y.  Normalising by s keeps the misfit channels at unit scale (in bfloat16 the
          difference of two nearly equal images would lose most of its digits)
  h0    = Wl a + bl                                              lifting 9 -> 32
  z_l   = W_l h_l + b_l + S_l h_l,  h_{l+1} = gelu(z_l) (l < 3), h_4 = z_3
  S_l h = real( sum over retained k of w(k2) O(k) e^{i k.x} ),  O(k)[o] = sum_c H(k)[c] R_l(k)[c, o]
          H(k) = n^-2 sum_x h(x) e^{-i k.x} (Fourier coefficient); retained k1 in {0..15, -16..-1},
          k2 in {0..15}; w(0) = 1 and only the real part of the k2 = 0 column is kept (the
          inverse real FFT convention); w(k2 > 0) = 2 (Hermitian completion)
  y     = B (Q2 gelu(Q1 h4 + q1) + q2)                          projection 32 -> 64 -> 2 + 2R, then
          the band limit B u = real( sum over retained k with |k| <= 12 of w(k2) U(k) e^{i k.x} ) (S
          with identity weights on the disc |k| <= 12 and zero weights on the corners of the
          retained square): the predicted fields have no energy where the solutions have none,
          which the H2 regulariser would weight by |k|^4
  gelu(x) = x Phi(x) (exact, with the normal CDF Phi)
Output channels: y[0:2] = v / s (the warm start); y[2 + 2k : 4 + 2k] = direction z_k, k < R = 4, a
vector field for the low-rank correction of the PCG preconditioner (``solver.SolveOpts.precond_U``).
Its training target is the k-th leading generalised eigenvector of (H, M) at the solved velocity
(``solver.ritz_directions``); only the line it spans matters, so its loss is sign- and scale-free.
Loss over a batch (Euclidean sums over points and the two components):
  L = (1/B) sum_b [ ||y_b - t_b||^2 / ||t_b||^2 over channels 0, 1
                    + (lambda / R) sum_k w_bk (1 - <t_bk, y_bk>^2 / (||t_bk||^2 max(||y_bk||^2, 1e-30))) ]
with lambda = DIR_WEIGHT and w_bk = 1 if ||t_bk|| > 0, else 0 (no target: no term).

Flat parameter vector (float), in this order:
  Wl[32][4], bl[32];  for l = 0..3: Rr_l[32][16][32][32], Ri_l[32][16][32][32], W_l[32][32], b_l[32];
  Q1[64][32], q1[64], Q2[2 + 2R][64], q2[2 + 2R]
  R index order: [k1 row j][k2][c in][c out], k1 = j for j < 16 and j - 32 otherwise.

Two formulations of the same network:
  * spectral="fft": the Fourier layer through numpy's FFTs (the definition above, FP64).
  * spectral="gemm": the Fourier layer as products with truncated DFT matrices (F2, CS, IC, G2
    below), and the complex mode mixing split into real and imaginary parts.  With bf16=True every
    matrix product takes operands first stored in float32 and then rounded to bfloat16 (round to
    nearest even), and accumulates exactly (FP64 here); all other arithmetic stays FP64.  This is
    the plain definition of the network evaluated with bfloat16 multiplicands and wide accumulation.
    The output band limit B is a fixed filter on the velocity itself and always takes exact products.
The backward pass (reverse mode, by hand) follows the gemm formulation, rounding the operands of
its products the same way when bf16=True; with bf16=False it is the exact gradient.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

WIDTH = 32
MODES = 16
LAYERS = 4
IN_CH = 9
RANK = 4                 # directions of the low-rank head
OUT_CH = 2 + 2 * RANK    # velocity (2) and RANK vector fields
DIR_WEIGHT = 0.1         # lambda: weight of the direction terms in the loss
HIDDEN = 64
OUT_RADIUS = 12


# ----------------------------------------------------------------------------------------------
# rounding
# ----------------------------------------------------------------------------------------------
def to_bf16(x):
    """Store in float32 (round to nearest), then round to bfloat16 (round to nearest even)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------------------------
# parameters
# ----------------------------------------------------------------------------------------------
def param_shapes():
    C, M = WIDTH, MODES
    shapes = [("Wl", (C, IN_CH)), ("bl", (C,))]
    for l in range(LAYERS):
        shapes += [(f"Rr{l}", (2 * M, M, C, C)), (f"Ri{l}", (2 * M, M, C, C)),
                   (f"W{l}", (C, C)), (f"b{l}", (C,))]
    shapes += [("Q1", (HIDDEN, C)), ("q1", (HIDDEN,)), ("Q2", (OUT_CH, HIDDEN)), ("q2", (OUT_CH,))]
    return shapes


def param_count():
    return sum(int(np.prod(s)) for _, s in param_shapes())


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    if theta.size != param_count():
        raise ValueError(f"expected {param_count()} parameters, got {theta.size}")
    out, off = {}, 0
    for name, shp in param_shapes():
        k = int(np.prod(shp))
        out[name] = theta[off:off + k].reshape(shp)
        off += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in param_shapes()])


# ----------------------------------------------------------------------------------------------
# pieces
# ----------------------------------------------------------------------------------------------
def misfit_scale(mT, mR):
    """s = sqrt(mean((m_R - m_T)^2))."""
    d = np.asarray(mR, dtype=np.float64) - np.asarray(mT, dtype=np.float64)
    return float(np.sqrt(np.mean(d * d)))


def features(mT, mR):
    """The 9 input channels of one pair (n1, n2) -> ((9, n1, n2), s)."""
    mT = np.asarray(mT, dtype=np.float64)
    mR = np.asarray(mR, dtype=np.float64)
    n1, n2 = mT.shape
    d1 = (np.roll(mT, -1, axis=0) - np.roll(mT, 1, axis=0)) / (2.0 * (2.0 * np.pi / n1))
    d2 = (np.roll(mT, -1, axis=1) - np.roll(mT, 1, axis=1)) / (2.0 * (2.0 * np.pi / n2))
    s = misfit_scale(mT, mR)
    r = (mR - mT) / s if s > 0.0 else np.zeros_like(mT)
    return np.stack([mT, d1, d2, d1 * d1, d1 * d2, d2 * d2, r, r * d1, r * d2]), s


def predict(theta, mT, mR, bf16=False, spectral="gemm"):
    """Warm start v0 = s y[0:2] and the RANK directions y[2:] (shaped (RANK, 2, n1, n2)) for one pair."""
    a, s = features(mT, mR)
    y, _ = forward(theta, a[None], bf16=bf16, spectral=spectral)
    n1, n2 = y.shape[-2:]
    return s * y[0, :2], y[0, 2:].reshape(RANK, 2, n1, n2)


def gelu(x):
    return x * 0.5 * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def kept_k1(n):
    """Wavenumbers of the retained rows j = 0..2M-1: 0..M-1, then -M..-1."""
    return [j if j < MODES else j - 2 * MODES for j in range(2 * MODES)]


def dft_bases(n):
    """Truncated DFT matrices for an n x n grid (square grids), entries from math.cos / math.sin.

    F2 (n, 32): columns k2 = 0..15: cos(2 pi k2 i2 / n) / n, then -sin(...) / n   (forward, axis 2)
    CS (64, n): rows j: cos(2 pi k1_j i1 / n) / n, then sin(...) / n              (forward, axis 1)
    IC (n, 64): columns j: cos(2 pi k1_j i1 / n), then sin(...)                  (inverse, axis 1)
    G2 (32, n): rows k2: w cos(2 pi k2 i2 / n), then -w sin(...), w = 1 (k2 = 0) or 2  (inverse, axis 2)
    """
    M = MODES
    F2 = np.zeros((n, 2 * M))
    G2 = np.zeros((2 * M, n))
    for i in range(n):
        for k in range(M):
            ang = 2.0 * math.pi * ((k * i) % n) / n
            w = 1.0 if k == 0 else 2.0
            F2[i, k] = math.cos(ang) / n
            F2[i, M + k] = -math.sin(ang) / n
            G2[k, i] = w * math.cos(ang)
            G2[M + k, i] = -w * math.sin(ang)
    CS = np.zeros((4 * M, n))
    IC = np.zeros((n, 4 * M))
    for j, k1 in enumerate(kept_k1(n)):
        for i in range(n):
            ang = 2.0 * math.pi * ((k1 * i) % n) / n
            CS[j, i] = math.cos(ang) / n
            CS[2 * M + j, i] = math.sin(ang) / n
            IC[i, j] = math.cos(ang)
            IC[i, 2 * M + j] = math.sin(ang)
    return {"F2": F2, "CS": CS, "IC": IC, "G2": G2}


def spectral_conv_fft(h, Rr, Ri):
    """S h through numpy's real FFTs (the definition)."""
    B, C, n1, n2 = h.shape
    H = np.fft.rfft2(h) / (n1 * n2)
    rows = np.array([k % n1 for k in kept_k1(n1)])
    Zk = H[:, :, rows, :MODES]
    O = np.einsum("bcjk,jkco->bojk", Zk, Rr + 1j * Ri)
    full = np.zeros((B, Rr.shape[-1], n1, n2 // 2 + 1), dtype=np.complex128)
    full[:, :, rows, :MODES] = O
    return np.fft.irfft2(full * (n1 * n2), s=(n1, n2))


def out_mask():
    """1 on the retained modes with |k| <= OUT_RADIUS, 0 on the rest, shaped (2M rows j, M columns k2)."""
    k1 = np.array(kept_k1(0))[:, None]
    k2 = np.arange(MODES)[None, :]
    return (k1 * k1 + k2 * k2 <= OUT_RADIUS * OUT_RADIUS).astype(np.float64)


def band_limit_fft(u):
    """B u through numpy's real FFTs: S with the identity as mode weights on the disc, per channel."""
    C = u.shape[1]
    eye = out_mask()[:, :, None, None] * np.eye(C)[None, None]
    return spectral_conv_fft(u, eye, np.zeros_like(eye))


class _Mul:
    """Products of the gemm formulation, with or without bfloat16 multiplicands."""

    def __init__(self, bf16):
        self.bf16 = bf16

    def r(self, x):
        return to_bf16(x) if self.bf16 else x

    def mm(self, A, B):
        return np.matmul(self.r(A), self.r(B))

    def ein(self, spec, A, B):
        return np.einsum(spec, self.r(A), self.r(B))


def _spectral_gemm(mul, bases, h, Rr, Ri):
    """S h through truncated DFT matrices; returns the output and the intermediates."""
    M = MODES
    Y = mul.mm(h, bases["F2"])                       # (B,C,n,32): [Re | Im] of the axis-2 DFT
    T = mul.mm(bases["CS"], Y)                       # (B,C,64,32)
    Zr = T[:, :, :2 * M, :M] + T[:, :, 2 * M:, M:]   # Re of the 2D coefficient, (B,C,32,16)
    Zi = T[:, :, :2 * M, M:] - T[:, :, 2 * M:, :M]
    Or = mul.ein("bcjk,jkco->bojk", Zr, Rr) - mul.ein("bcjk,jkco->bojk", Zi, Ri)
    Oi = mul.ein("bcjk,jkco->bojk", Zr, Ri) + mul.ein("bcjk,jkco->bojk", Zi, Rr)
    Ob = np.concatenate([np.concatenate([Or, Oi], axis=3), np.concatenate([-Oi, Or], axis=3)], axis=2)
    Yp = mul.mm(bases["IC"], Ob)                     # (B,C,n,32): [Re | Im] after the axis-1 inverse
    hp = mul.mm(Yp, bases["G2"])                     # (B,C,n,n)
    return hp, (Zr, Zi)


def _band_limit_gemm(mul, bases, u):
    """B u through the truncated DFT matrices (no mode product: the weights are the identity).
    This fixed filter acts on the velocity itself and takes exact products also when the network
    uses bfloat16 multiplicands (the GPU runs it in FP32)."""
    mul = _Mul(False)
    M = MODES
    T = mul.mm(bases["CS"], mul.mm(u, bases["F2"]))
    Zr = (T[:, :, :2 * M, :M] + T[:, :, 2 * M:, M:]) * out_mask()
    Zi = (T[:, :, :2 * M, M:] - T[:, :, 2 * M:, :M]) * out_mask()
    Ob = np.concatenate([np.concatenate([Zr, Zi], axis=3), np.concatenate([-Zi, Zr], axis=3)], axis=2)
    return mul.mm(mul.mm(bases["IC"], Ob), bases["G2"])


def _band_limit_gemm_T(mul, bases, dv):
    """Transpose of _band_limit_gemm (the products in reverse order, transposed), exact products."""
    mul = _Mul(False)
    M = MODES
    dOb = mul.mm(bases["IC"].T, mul.mm(dv, bases["G2"].T))
    dZr = (dOb[:, :, :2 * M, :M] + dOb[:, :, 2 * M:, M:]) * out_mask()
    dZi = (dOb[:, :, :2 * M, M:] - dOb[:, :, 2 * M:, :M]) * out_mask()
    dT = np.concatenate([np.concatenate([dZr, dZi], axis=3), np.concatenate([-dZi, dZr], axis=3)], axis=2)
    return mul.mm(mul.mm(bases["CS"].T, dT), bases["F2"].T)


def _pointwise(mul, W, x):
    return mul.ein("oc,bcxy->boxy", W, x)


# ----------------------------------------------------------------------------------------------
# forward / backward
# ----------------------------------------------------------------------------------------------
def forward(theta, a, bf16=False, spectral="gemm"):
    """y for inputs a (B, 4, n, n); returns (y, cache)."""
    if spectral == "fft" and bf16:
        raise ValueError("the FFT formulation has no bfloat16 variant")
    P = unpack(theta)
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[-1]
    if a.shape[-2] != n:
        raise ValueError("square grids only")
    mul = _Mul(bf16)
    bases = dft_bases(n) if spectral == "gemm" else None
    h = _pointwise(mul, P["Wl"], a) + P["bl"][None, :, None, None]
    cache = {"a": a, "h": [h], "z": [], "Z": [], "bf16": bf16, "bases": bases, "P": P}
    for l in range(LAYERS):
        if spectral == "fft":
            hp = spectral_conv_fft(h, P[f"Rr{l}"], P[f"Ri{l}"])
            Zs = None
        else:
            hp, Zs = _spectral_gemm(mul, bases, h, P[f"Rr{l}"], P[f"Ri{l}"])
        z = _pointwise(mul, P[f"W{l}"], h) + P[f"b{l}"][None, :, None, None] + hp
        cache["z"].append(z)
        cache["Z"].append(Zs)
        h = gelu(z) if l < LAYERS - 1 else z
        cache["h"].append(h)
    zq = _pointwise(mul, P["Q1"], h) + P["q1"][None, :, None, None]
    s = gelu(zq)
    u = _pointwise(mul, P["Q2"], s) + P["q2"][None, :, None, None]
    y = band_limit_fft(u) if spectral == "fft" else _band_limit_gemm(mul, bases, u)
    cache["zq"], cache["s"] = zq, s
    return y, cache


def loss(y, t):
    """The loss L of the module docstring and its gradient with respect to y.

    Velocity channels: relative squared error.  Direction k: 1 - cos^2 of the angle between y_k and
    t_k, whose gradient is -2 c t / (a b) + 2 c^2 y / (a b^2) with a = ||t||^2, b = ||y||^2,
    c = <t, y>."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B = y.shape[0]
    d = y[:, :2] - t[:, :2]
    num = (d * d).reshape(B, -1).sum(axis=1)
    den = (t[:, :2] * t[:, :2]).reshape(B, -1).sum(axis=1)
    L = float((num / den).sum() / B)
    dy = np.zeros_like(y)
    dy[:, :2] = 2.0 * d / (B * den[:, None, None, None])
    wdir = DIR_WEIGHT / RANK
    for k in range(RANK):
        ch = slice(2 + 2 * k, 4 + 2 * k)
        yk, tk = y[:, ch], t[:, ch]
        a = (tk * tk).reshape(B, -1).sum(axis=1)
        b = np.maximum((yk * yk).reshape(B, -1).sum(axis=1), 1e-30)
        c = (tk * yk).reshape(B, -1).sum(axis=1)
        w = (a > 0).astype(np.float64)
        a_ = np.where(a > 0, a, 1.0)
        L += float(wdir * (w * (1.0 - c * c / (a_ * b))).sum() / B)
        f = (w * wdir / B)[:, None, None, None]
        dy[:, ch] = f * (-2.0 * (c / (a_ * b))[:, None, None, None] * tk
                         + 2.0 * (c * c / (a_ * b * b))[:, None, None, None] * yk)
    return L, dy


def backward(cache, dy):
    """Gradient of sum(dy * y) with respect to the flat parameters (reverse mode of forward)."""
    if cache["bases"] is None:
        raise ValueError("backward follows the gemm formulation: run forward with spectral='gemm'")
    mul = _Mul(cache["bf16"])
    P, bases = cache["P"], cache["bases"]
    M = MODES
    G = {}
    sum_p = lambda x: x.sum(axis=(0, 2, 3))   # noqa: E731  (bias gradients)
    # projection
    s, zq, h4 = cache["s"], cache["zq"], cache["h"][LAYERS]
    dy = _band_limit_gemm_T(mul, bases, dy)
    G["Q2"] = mul.ein("boxy,bcxy->oc", dy, s)
    G["q2"] = sum_p(dy)
    ds = mul.ein("oc,boxy->bcxy", P["Q2"], dy)
    dzq = ds * gelu_grad(zq)
    G["Q1"] = mul.ein("boxy,bcxy->oc", dzq, h4)
    G["q1"] = sum_p(dzq)
    dh = mul.ein("oc,boxy->bcxy", P["Q1"], dzq)
    for l in reversed(range(LAYERS)):
        z, hin = cache["z"][l], cache["h"][l]
        dz = dh * gelu_grad(z) if l < LAYERS - 1 else dh
        G[f"W{l}"] = mul.ein("boxy,bcxy->oc", dz, hin)
        G[f"b{l}"] = sum_p(dz)
        dh = mul.ein("oc,boxy->bcxy", P[f"W{l}"], dz)
        # spectral branch, transposed step by step
        Zr, Zi = cache["Z"][l]
        Rr, Ri = P[f"Rr{l}"], P[f"Ri{l}"]
        dYp = mul.mm(dz, bases["G2"].T)
        dOb = mul.mm(bases["IC"].T, dYp)
        dOr = dOb[:, :, :2 * M, :M] + dOb[:, :, 2 * M:, M:]
        dOi = dOb[:, :, :2 * M, M:] - dOb[:, :, 2 * M:, :M]
        G[f"Rr{l}"] = mul.ein("bcjk,bojk->jkco", Zr, dOr) + mul.ein("bcjk,bojk->jkco", Zi, dOi)
        G[f"Ri{l}"] = mul.ein("bcjk,bojk->jkco", Zr, dOi) - mul.ein("bcjk,bojk->jkco", Zi, dOr)
        dZr = mul.ein("bojk,jkco->bcjk", dOr, Rr) + mul.ein("bojk,jkco->bcjk", dOi, Ri)
        dZi = mul.ein("bojk,jkco->bcjk", dOi, Rr) - mul.ein("bojk,jkco->bcjk", dOr, Ri)
        dT = np.concatenate([np.concatenate([dZr, dZi], axis=3), np.concatenate([-dZi, dZr], axis=3)], axis=2)
        dY = mul.mm(bases["CS"].T, dT)
        dh = dh + mul.mm(dY, bases["F2"].T)
    G["Wl"] = mul.ein("boxy,bcxy->oc", dh, cache["a"])
    G["bl"] = sum_p(dh)
    return pack(G)


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, ICLR 2015, Alg. 1) at step number `step` >= 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
