"""Seeded synthetic inputs for the 2D registration problem.

This module only *draws data*: smooth template images (periodic Gaussian blobs plus a band-limited
sinusoidal texture), random band-limited velocity fields and random search directions.  It holds
none of the registration method's arithmetic (no transport, no spectral operators, no solver) and
imports neither the CPU oracle nor the HIP library; both of those consume its arrays.

The paper's images (hand images, OASIS and NIREP brain slices, Sec. 5) are not available, so these
inputs stand in for them with the properties the paper states: intensities in [0, 1] (Sec. 4),
smooth images (Sec. 4, pre-smoothing), periodic domain (Sec. 2).

Grid convention: x = (2*pi*i1/n1, 2*pi*i2/n2), arrays shaped (n1, n2), i2 fastest; vector fields are
shaped (2, n1, n2) (component-major).  Seeds: numpy PCG64 with ``BASE_SEED + config``; pair ``p`` of
a batch uses ``seed + 1000 * p``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

BASE_SEED = 150300757


def grid_coords(n1: int, n2: int):
    x1 = 2.0 * np.pi * np.arange(n1, dtype=np.float64) / n1
    x2 = 2.0 * np.pi * np.arange(n2, dtype=np.float64) / n2
    return x1, x2


def gaussian_blobs(n1: int, n2: int, nblobs: int, rng: np.random.Generator,
                   sigma_range=(0.3, 0.8), amp_range=(0.2, 1.0)) -> np.ndarray:
    """Sum of periodised isotropic Gaussians.

    B(x) = sum_b a_b sum_{p,q in {-1,0,1}} exp(-|x - c_b - 2 pi (p,q)|^2 / (2 sigma_b^2)).
    With sigma <= 0.8 the omitted periodic images contribute below 1e-13.
    The 2D Gaussian is separable, so each blob is an outer product of two 1D profiles.
    """
    x1, x2 = grid_coords(n1, n2)
    out = np.zeros((n1, n2))
    for _ in range(nblobs):
        c = rng.uniform(0.0, 2.0 * np.pi, size=2)
        s = rng.uniform(*sigma_range)
        a = rng.uniform(*amp_range)
        g1 = sum(np.exp(-((x1 - c[0] - 2.0 * np.pi * p) ** 2) / (2.0 * s * s)) for p in (-1, 0, 1))
        g2 = sum(np.exp(-((x2 - c[1] - 2.0 * np.pi * q) ** 2) / (2.0 * s * s)) for q in (-1, 0, 1))
        out += a * np.outer(g1, g2)
    return out


def _half_plane_modes(kmax: int):
    """Integer wave vectors 0 < |k| <= kmax, one of each +-k pair."""
    ks = []
    for k1 in range(-kmax, kmax + 1):
        for k2 in range(0, kmax + 1):
            if k2 == 0 and k1 <= 0:
                continue
            if k1 * k1 + k2 * k2 <= kmax * kmax:
                ks.append((k1, k2))
    return np.array(ks, dtype=np.int64).reshape(-1, 2)


def _eval_trig(n1: int, n2: int, ks: np.ndarray, ca: np.ndarray, cb: np.ndarray,
               weight1=None, weight2=None) -> np.ndarray:
    """Evaluate sum_k w(k) [ca_k cos(k.x) + cb_k sin(k.x)] on the grid.

    Evaluated directly as exponentials: sum_k c_k e^{i k.x} = E1 C E2^T with
    E_a[i, k_a] = exp(i k_a x_a[i]); no transform library is used.
    """
    x1, x2 = grid_coords(n1, n2)
    if ks.shape[0] == 0:
        return np.zeros((n1, n2))
    w = np.ones(ks.shape[0])
    if weight1 is not None:
        w = w * weight1
    if weight2 is not None:
        w = w * weight2
    k1vals = np.unique(ks[:, 0])
    k2vals = np.unique(ks[:, 1])
    i1 = np.searchsorted(k1vals, ks[:, 0])
    i2 = np.searchsorted(k2vals, ks[:, 1])
    # ca cos(t) + cb sin(t) = Re[(ca - i cb) e^{it}]
    C = np.zeros((k1vals.size, k2vals.size), dtype=np.complex128)
    np.add.at(C, (i1, i2), w * (ca - 1j * cb))
    E1 = np.exp(1j * np.outer(x1, k1vals))
    E2 = np.exp(1j * np.outer(x2, k2vals))
    return np.real(E1 @ C @ E2.T)


def texture(n1: int, n2: int, kmax: int, rng: np.random.Generator) -> np.ndarray:
    """Random band-limited texture sum_{0<|k|<=kmax} a_k cos(k.x) + b_k sin(k.x), a,b ~ N(0,1)."""
    ks = _half_plane_modes(kmax)
    a = rng.standard_normal(ks.shape[0])
    b = rng.standard_normal(ks.shape[0])
    return _eval_trig(n1, n2, ks, a, b)


def minmax01(u: np.ndarray) -> np.ndarray:
    lo, hi = float(u.min()), float(u.max())
    return (u - lo) / (hi - lo)


def template_image(n1: int, n2: int, nblobs: int, ktex: int, rng: np.random.Generator) -> np.ndarray:
    """m_T = minmax01(B + T) with max|T| = 0.1 max B (T omitted when ktex = 0)."""
    B = gaussian_blobs(n1, n2, nblobs, rng)
    if ktex > 0:
        T = texture(n1, n2, ktex, rng)
        T *= 0.1 * B.max() / np.abs(T).max()
        B = B + T
    return minmax01(B)


def _potential_gradient(n1, n2, ks, a, b, perp: bool):
    """Analytic gradient (perp=False) or rotated gradient (-d2, d1) (perp=True) of
    psi = sum_k a_k cos(k.x) + b_k sin(k.x); d_j psi = sum_k k_j (b_k cos - a_k sin)."""
    d1 = _eval_trig(n1, n2, ks, b, -a, weight1=ks[:, 0].astype(np.float64))
    d2 = _eval_trig(n1, n2, ks, b, -a, weight1=ks[:, 1].astype(np.float64))
    if perp:
        return np.stack([-d2, d1])
    return np.stack([d1, d2])


def random_velocity(n1: int, n2: int, kmax: int, rng: np.random.Generator,
                    divfree: bool = True, compressible: bool = False) -> np.ndarray:
    """Band-limited random velocity, 0 < |k| <= kmax, N(0,1) mode coefficients.

    divfree part: rotated gradient of a stream function; compressible part: gradient of a potential.
    The result is not yet scaled (see ``scale_to_cfl`` / ``scale_to_max``).
    """
    ks = _half_plane_modes(kmax)
    v = np.zeros((2, n1, n2))
    if divfree:
        v += _potential_gradient(n1, n2, ks, rng.standard_normal(ks.shape[0]),
                                 rng.standard_normal(ks.shape[0]), perp=True)
    if compressible:
        v += _potential_gradient(n1, n2, ks, rng.standard_normal(ks.shape[0]),
                                 rng.standard_normal(ks.shape[0]), perp=False)
    return v


def cfl_number(v: np.ndarray, nt: int) -> float:
    """C(v) = h_t (max|v1| n1/2 + max|v2| n2/2): the largest |h_t k.v| over resolved modes."""
    n1, n2 = v.shape[1:]
    return (1.0 / nt) * (np.abs(v[0]).max() * (n1 / 2) + np.abs(v[1]).max() * (n2 / 2))


def scale_to_cfl(v: np.ndarray, nt: int, target: float) -> np.ndarray:
    return v * (target / cfl_number(v, nt))


def scale_to_max(v: np.ndarray, vmax: float) -> np.ndarray:
    return v * (vmax / np.sqrt((v ** 2).sum(axis=0)).max())


def unit_l2(v: np.ndarray) -> np.ndarray:
    """Normalise to <v, v> = 1 with the grid inner product h1 h2 sum v.v."""
    n1, n2 = v.shape[1:]
    h = (2.0 * np.pi / n1) * (2.0 * np.pi / n2)
    return v / math.sqrt(h * float((v * v).sum()))


# --------------------------------------------------------------------------------------------
# Workload recipes (the stand-ins for the paper's image pairs)
# --------------------------------------------------------------------------------------------

@dataclass
class Workload:
    """One registration pair plus the settings it is solved with."""
    name: str
    n1: int
    n2: int
    nt: int
    norm: str            # "H1" | "H2"
    constraint: str      # "none" | "divfree" | "mass_source"
    beta_v: float
    beta_w: float
    mT: np.ndarray
    vstar: np.ndarray
    vtilde: np.ndarray   # seeded search direction used by matvec benchmarks/tests
    seed: int
    extra: dict = field(default_factory=dict)


def _direction(n1, n2, rng, constraint, kmax=16):
    vt = random_velocity(n1, n2, min(kmax, n1 // 2 - 1, n2 // 2 - 1), rng,
                         divfree=True, compressible=(constraint != "divfree"))
    return unit_l2(vt)


def make_workload(config: int, pair: int = 0, n: int | None = None, nt: int | None = None,
                  beta_v: float | None = None) -> Workload:
    """Seeded workload for one of the five configurations.

    1: 64^2, nt=4, 8 blobs, no texture; v* divergence-free, |k|<=4, max|v*|=0.2; H1, div-free,
       beta_v=1e-2.
    2: 256^2, nt=16, 32 blobs + texture |k|<=16; v* = grad(phi) + rot-grad(psi), |k|<=8, scaled to
       CFL 0.8; H2 with mass source, beta_v=1e-3, beta_w=1e-4.
    3: 1024^2, nt=32, 32 blobs + texture |k|<=64; v* divergence-free, |k|<=8, CFL 0.8; H1, div-free,
       beta_v=1e-4.
    4: batch pair ``pair`` of 96: n in {128,256,512} (32 each), nt in {8,16,32}, beta_v
       log-uniform in [1e-4,1e-2]; H1, div-free; texture |k|<=16; v* div-free |k|<=8, CFL 0.8.
    5: config 2's generator and settings at n (128 for training pairs, 256 for test pairs), with
       the velocity amplitude of config 2 at 256^2 whatever n is.
    ``n``/``nt``/``beta_v`` override the grid size, step count and weight (for small test cases).
    """
    seed = BASE_SEED + config + 1000 * pair
    rng = np.random.Generator(np.random.PCG64(seed))
    if config == 1:
        n_ = n or 64
        nt_ = nt or 4
        mT = template_image(n_, n_, 8, 0, rng)
        vs = scale_to_max(random_velocity(n_, n_, 4, rng, divfree=True), 0.2)
        vt = _direction(n_, n_, rng, "divfree")
        return Workload("c1", n_, n_, nt_, "H1", "divfree", beta_v or 1e-2, 0.0, mT, vs, vt, seed)
    if config == 2 or config == 5:
        n_ = n or (256 if config == 2 else 128)
        nt_ = nt or 16
        mT = template_image(n_, n_, 32, min(16, n_ // 2 - 1), rng)
        # config 5 keeps the physical velocity amplitude of config 2 (CFL 0.8 on the 256^2 grid)
        # at every grid size, so training pairs at 128^2 and test pairs at 256^2 share one
        # distribution of continuous velocity fields
        cfl = 0.8 if config == 2 else 0.8 * n_ / 256.0
        vs = scale_to_cfl(random_velocity(n_, n_, 8, rng, divfree=True, compressible=True), nt_, cfl)
        vt = _direction(n_, n_, rng, "mass_source")
        return Workload(f"c{config}", n_, n_, nt_, "H2", "mass_source", beta_v or 1e-3, 1e-4,
                        mT, vs, vt, seed)
    if config == 3:
        n_ = n or 1024
        nt_ = nt or 32
        mT = template_image(n_, n_, 32, min(64, n_ // 2 - 1), rng)
        vs = scale_to_cfl(random_velocity(n_, n_, 8, rng, divfree=True), nt_, 0.8)
        vt = _direction(n_, n_, rng, "divfree")
        return Workload("c3", n_, n_, nt_, "H1", "divfree", beta_v or 1e-4, 0.0, mT, vs, vt, seed)
    if config == 4:
        sizes = (128, 256, 512)
        n_ = n or sizes[pair % 3]
        nt_ = nt or int(rng.choice([8, 16, 32]))
        bv = beta_v or float(10.0 ** rng.uniform(-4.0, -2.0))
        mT = template_image(n_, n_, 32, min(16, n_ // 2 - 1), rng)
        vs = scale_to_cfl(random_velocity(n_, n_, 8, rng, divfree=True), nt_, 0.8)
        vt = _direction(n_, n_, rng, "divfree")
        return Workload("c4", n_, n_, nt_, "H1", "divfree", bv, 0.0, mT, vs, vt, seed)
    raise ValueError(f"unknown config {config}")


def sliding_pair(n: int, nt: int, cfl: float = 0.8, seed: int = BASE_SEED + 512, sharp: float = 4.0) -> Workload:
    """A self-made sliding-interface pair in the spirit of the paper's shear experiments (Sec. 5.2, whose
    images are not specified numerically): a textured blob template and the divergence-free shear flow
    v* = (a tanh(sharp sin x2), 0), whose two bands slide past each other across smooth interfaces at
    x2 = 0 and pi; a is set for the given CFL number at n_t steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mT = template_image(n, n, 48, min(24, n // 2 - 1), rng)
    _, x2 = grid_coords(n, n)
    prof = np.tanh(sharp * np.sin(x2))
    v = np.stack([np.tile(prof[None, :], (n, 1)), np.zeros((n, n))])
    v = scale_to_cfl(v, nt, cfl)
    vt = _direction(n, n, rng, "divfree")
    return Workload("sliding", n, n, nt, "H1", "divfree", 1e-3, 0.0, mT, v, vt, seed)


def random_field(n1: int, n2: int, kmax: int, seed: int) -> np.ndarray:
    """A seeded band-limited scalar field with unit max-norm (for operator tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = texture(n1, n2, kmax, rng)
    return t / np.abs(t).max()


def reference_change(n1: int, n2: int, amp: float = 0.05, kmax: int = 32, seed: int = BASE_SEED + 91) -> np.ndarray:
    """A seeded band-limited intensity change (max |.| = amp) added to a reference image so that no
    velocity explains it (the residual stays finite at the minimiser, as with real image pairs)."""
    return amp * random_field(n1, n2, min(kmax, min(n1, n2) // 2 - 1), seed)


def random_vec(n1: int, n2: int, kmax: int, seed: int, divfree: bool = False) -> np.ndarray:
    """A seeded band-limited vector field with unit L2 norm (for operator tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return unit_l2(random_velocity(n1, n2, kmax, rng, divfree=True, compressible=not divfree))


# --------------------------------------------------------------------------------------------
# Learned warm start: seeded draws of initial network weights and of training / test pairs
# --------------------------------------------------------------------------------------------

def network_init(seed: int = BASE_SEED + 55) -> np.ndarray:
    """Initial weights of the warm-start network as one flat float32 vector, in the parameter order
    of the network's interface (lifting 9->32; four Fourier layers of width 32 with 32x16 retained
    modes; projection 32->64->10: the velocity and 4 direction fields).

    Draws only: pointwise weights and biases ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)); spectral weights
    (real and imaginary parts) ~ U(0, 1) / (32 * 32), the usual initialisation of Fourier layers.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    C, M, H = 32, 16, 64

    def uni(shape, fan_in):
        b = 1.0 / math.sqrt(fan_in)
        return rng.uniform(-b, b, size=shape)

    blocks = [uni((C, 9), 9), uni((C,), 9)]
    for _ in range(4):
        blocks += [rng.uniform(0.0, 1.0, size=(2 * M, M, C, C)) / (C * C),
                   rng.uniform(0.0, 1.0, size=(2 * M, M, C, C)) / (C * C),
                   uni((C, C), C), uni((C,), C)]
    OUT = 2 + 2 * 4
    blocks += [uni((H, C), C), uni((H,), C), uni((OUT, H), H), uni((OUT,), H)]
    return np.concatenate([b.ravel() for b in blocks]).astype(np.float32)


def warmstart_pair(pair: int, n: int) -> Workload:
    """Pair ``pair`` of the warm-start data set (config 5) at grid size n.  Training pairs use
    indices 0..4095 at n = 128; test pairs use indices from 100000 on (unseen seeds) at n = 256."""
    return make_workload(5, pair=pair, n=n)
