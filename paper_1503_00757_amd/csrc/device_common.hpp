// Device building blocks for the gfx950 registration library: complex arithmetic, the
// register-resident Stockham FFT used by every spectral pass, and wave/block reductions.
//
// The FFT computes the length-N DFT (N a power of two, 8..2048) of one complex sequence with
// N/4 cooperating threads.  Thread t holds elements t + r N/4 (r = 0..3) in registers both on entry
// (natural-order input) and on exit (natural-order output): the first radix stage reads exactly those
// elements and the last one writes exactly those, so only the intermediate stages go through LDS.
// Stages are radix-4 (Stockham autosort, decimation in time), preceded by one radix-2 stage when
// log2 N is odd.  Twiddles come from a table W[m] = exp(-2 pi i m / N) computed in double precision
// on the host (no recurrences), conjugated for the inverse transform.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mr_plan.hpp"

namespace regnk {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by the twiddle w (forward) or conj(w) (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> ctw(cpx<T> a, cpx<T> w) {
    if (INV) return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
    return cmul(a, w);
}
// multiply by -i (forward DFT4) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> cmi(cpx<T> a) {
    if (INV) return {-a.y, a.x};
    return {a.y, -a.x};
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

// LDS index padding: one pad slot every 16 complex entries breaks the power-of-two strides of the
// Stockham scatter.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8).  Column tiles that share
// a 128-byte line go to blocks on the same XCD (same L2): tile for block b of nb, `group` tiles per
// line (identity unless nb is a multiple of 8 * group).
__device__ __forceinline__ int xcd_tile(int b, int nb, int group) {
    if (group <= 1 || (nb % (8 * group)) != 0) return b;
    const int x = b & 7, l = b >> 3;
    return group * (x + 8 * (l / group)) + (l % group);
}

template <int N>
struct LdsSize {
    static constexpr int value = N + (N >> 4);
};

// One length-N FFT on registers x[4] (see file header).  lds0 / lds1 are two LDS buffers of
// LdsSize<N> entries private to this transform; `buf` selects the buffer of the next exchange and
// must be carried from one call to the next so that consecutive exchanges always alternate buffers
// (a buffer is only rewritten after the barrier of the exchange that used the other one).  Must be
// reached by every thread of the block the same number of times (it contains __syncthreads).
// SINGLE: one buffer (lds1 unused); every exchange then waits at a barrier before it writes, so that
// the previous exchange's reads are done (half the LDS, one more barrier per exchange).
template <typename T, int N, bool INV, bool SINGLE = false>
__device__ __forceinline__ void fft4(cpx<T> (&x)[4], cpx<T>* lds0, cpx<T>* lds1, int t,
                                     const cpx<T>* __restrict__ tw, int& buf) {
    constexpr int Q = N / 4;
    constexpr int LOG = ilog2(N);
    int Ns = 1;
    if constexpr (LOG & 1) {
        if constexpr (SINGLE) __syncthreads();
        cpx<T>* o = (buf && !SINGLE) ? lds1 : lds0;
        cpx<T> a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
        cpx<T> b0 = cadd(x[1], x[3]), b1 = csub(x[1], x[3]);
        o[lpad(2 * t)] = a0;
        o[lpad(2 * t + 1)] = a1;
        o[lpad(2 * t + N / 2)] = b0;
        o[lpad(2 * t + N / 2 + 1)] = b1;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = o[lpad(t + r * Q)];
        buf ^= 1;
        Ns = 2;
    }
#pragma unroll
    for (int s = 0; s < LOG / 2; ++s) {
        const int k = t & (Ns - 1);
        if (Ns > 1) {
            const int step = N / (4 * Ns);
            x[1] = ctw<T, INV>(x[1], tw[(1 * k * step) & (N - 1)]);
            x[2] = ctw<T, INV>(x[2], tw[(2 * k * step) & (N - 1)]);
            x[3] = ctw<T, INV>(x[3], tw[(3 * k * step) & (N - 1)]);
        }
        cpx<T> s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
        cpx<T> s13 = cadd(x[1], x[3]), d13 = cmi<T, INV>(csub(x[1], x[3]));
        cpx<T> y0 = cadd(s02, s13), y2 = csub(s02, s13);
        cpx<T> y1 = cadd(d02, d13), y3 = csub(d02, d13);
        if (Ns == Q) {
            x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
        } else {
            if constexpr (SINGLE) __syncthreads();
            cpx<T>* o = (buf && !SINGLE) ? lds1 : lds0;
            const int base = (t - k) * 4 + k;
            o[lpad(base)] = y0;
            o[lpad(base + Ns)] = y1;
            o[lpad(base + 2 * Ns)] = y2;
            o[lpad(base + 3 * Ns)] = y3;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = o[lpad(t + r * Q)];
            buf ^= 1;
            Ns *= 4;
        }
    }
}

// ---- mixed-radix FFT with E elements per thread ------------------------------------------------
// T = N/E threads per transform; thread t holds elements t + T m (m = 0..E-1) on entry and on exit.
// Stages have radix E while the remaining factor allows, then one stage of the remaining radix
// (2, 4 or 8).  In a stage of radix R each thread runs B = E/R butterflies j = t + T b; input r of
// butterfly j is element j + r N/R, i.e. register b + B r, so every stage reads the thread's own
// register set and only the exchanges between stages go through LDS (one barrier each).
template <int M>
struct RootTab;   // exp(-2 pi i m / M), m < M, for the internal twiddles of the radix-8/16 kernels
template <>
struct RootTab<8> {
    static constexpr double c[8] = {1.0, 0.70710678118654752440, 0.0, -0.70710678118654752440,
                                    -1.0, -0.70710678118654752440, 0.0, 0.70710678118654752440};
    static constexpr double s[8] = {0.0, -0.70710678118654752440, -1.0, -0.70710678118654752440,
                                    0.0, 0.70710678118654752440, 1.0, 0.70710678118654752440};
};
template <>
struct RootTab<16> {
    static constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                     0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                                     -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                                     0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
    static constexpr double s[16] = {0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                                     -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                                     0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                                     1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
};

template <typename T, bool INV>
__device__ __forceinline__ void dft4v(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
    const cpx<T> s02 = cadd(a0, a2), d02 = csub(a0, a2);
    const cpx<T> s13 = cadd(a1, a3), d13 = cmi<T, INV>(csub(a1, a3));
    a0 = cadd(s02, s13);
    a2 = csub(s02, s13);
    a1 = cadd(d02, d13);
    a3 = csub(d02, d13);
}

// In-place DFT of R points (forward: exp(-2 pi i n k / R); inverse: conjugate).
// R = 8 and 16 are split as R = 4 * (R/4): n = (R/4) n1 + n2, k = k1 + 4 k2,
// X[k1 + 4 k2] = sum_{n2} W_{R/4}^{n2 k2} W_R^{n2 k1} sum_{n1} W_4^{n1 k1} x[(R/4) n1 + n2].
template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(cpx<T> (&a)[R]) {
    if constexpr (R == 2) {
        const cpx<T> t0 = a[0];
        a[0] = cadd(t0, a[1]);
        a[1] = csub(t0, a[1]);
    } else if constexpr (R == 4) {
        dft4v<T, INV>(a[0], a[1], a[2], a[3]);
    } else {
        constexpr int Q2 = R / 4;
        cpx<T> y[R];
#pragma unroll
        for (int n2 = 0; n2 < Q2; ++n2) {
            cpx<T> b0 = a[n2], b1 = a[Q2 + n2], b2 = a[2 * Q2 + n2], b3 = a[3 * Q2 + n2];
            dft4v<T, INV>(b0, b1, b2, b3);
            const cpx<T> bb[4] = {b0, b1, b2, b3};
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) {
                const int m = (n2 * k1) % R;
                const cpx<T> w = {T(RootTab<R>::c[m]), T(RootTab<R>::s[m])};
                y[n2 * 4 + k1] = (m == 0) ? bb[k1] : ctw<T, INV>(bb[k1], w);
            }
        }
        // DFT of length Q2 over n2 for each k1; result index k1 + 4 k2
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            if constexpr (Q2 == 2) {
                const cpx<T> u0 = y[0 * 4 + k1], u1 = y[1 * 4 + k1];
                a[k1] = cadd(u0, u1);
                a[k1 + 4] = csub(u0, u1);
            } else {
                cpx<T> u0 = y[0 * 4 + k1], u1 = y[1 * 4 + k1], u2 = y[2 * 4 + k1], u3 = y[3 * 4 + k1];
                dft4v<T, INV>(u0, u1, u2, u3);
                a[k1] = u0;
                a[k1 + 4] = u1;
                a[k1 + 8] = u2;
                a[k1 + 12] = u3;
            }
        }
    }
}

// Twiddles of all stages are loaded into registers once (they serve the forward and the inverse
// transform): stage (R, NS) needs W_{NS R}^{r k} for r = 1..R-1 and each of the thread's B
// butterflies, k = (t + T b) mod NS; the first stage (NS = 1) needs none.
template <int N, int E, int NS>
constexpr int tw_count() {
    constexpr int REM = N / NS;
    constexpr int R = REM >= E ? E : REM;
    constexpr int here = NS > 1 ? (R - 1) * (E / R) : 0;
    if constexpr (NS * R == N) {
        return here;
    } else {
        return here + tw_count<N, E, NS * R>();
    }
}
template <int N, int E>
constexpr int tw_regs() { return tw_count<N, E, 1>() > 0 ? tw_count<N, E, 1>() : 1; }

template <typename T, int N, int E, int NS, int OFF, int NW>
__device__ __forceinline__ void load_tw(cpx<T> (&W)[NW], int t, const cpx<T>* __restrict__ tw) {
    constexpr int TT = N / E;
    constexpr int REM = N / NS;
    constexpr int R = REM >= E ? E : REM;
    constexpr int B = E / R;
    if constexpr (NS > 1) {
        constexpr int step = N / (NS * R);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int k = (t + TT * b) & (NS - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) W[OFF + b * (R - 1) + (r - 1)] = tw[(r * k * step) & (N - 1)];
        }
    }
    if constexpr (NS * R < N) {
        load_tw<T, N, E, NS * R, OFF + (NS > 1 ? (R - 1) * B : 0), NW>(W, t, tw);
    }
}

template <typename T, int N, int E, int R, int NS, bool LAST, bool INV, int OFF, int NW>
__device__ __forceinline__ void fft_stage(cpx<T> (&x)[E], cpx<T>* __restrict__ o, int t, const cpx<T> (&W)[NW]) {
    constexpr int TT = N / E, B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + TT * b;
        const int k = j & (NS - 1);
        cpx<T> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = x[b + B * r];
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) a[r] = ctw<T, INV>(a[r], W[OFF + b * (R - 1) + (r - 1)]);
        }
        dftR<T, R, INV>(a);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[b + B * r] = a[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) o[lpad(base + r * NS)] = a[r];
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = o[lpad(t + TT * m)];
    }
}

template <typename T, int N, int E, int NS, bool INV, int OFF, int NW>
__device__ __forceinline__ void fft_stages(cpx<T> (&x)[E], cpx<T>* __restrict__ lds0, cpx<T>* __restrict__ lds1,
                                           int t, const cpx<T> (&W)[NW], int& buf) {
    constexpr int REM = N / NS;
    constexpr int R = REM >= E ? E : REM;
    constexpr bool LAST = (NS * R == N);
    fft_stage<T, N, E, R, NS, LAST, INV, OFF, NW>(x, buf ? lds1 : lds0, t, W);
    if constexpr (!LAST) {
        buf ^= 1;
        fft_stages<T, N, E, NS * R, INV, OFF + (NS > 1 ? (R - 1) * (E / R) : 0), NW>(x, lds0, lds1, t, W, buf);
    }
}

// Length-N FFT, E elements per thread (E in {2, 4, 8, 16}, E <= N/2); W from load_tw<T, N, E, 1, 0>;
// see fft4 for `buf`.
template <typename T, int N, int E, bool INV, int NW>
__device__ __forceinline__ void fftE(cpx<T> (&x)[E], cpx<T>* __restrict__ lds0, cpx<T>* __restrict__ lds1, int t,
                                     const cpx<T> (&W)[NW], int& buf) {
    static_assert(E == 2 || E == 4 || E == 8 || E == 16, "E");
    static_assert(N >= 2 * E, "N >= 2E");
    fft_stages<T, N, E, 1, INV, 0, NW>(x, lds0, lds1, t, W, buf);
}

// ---- mixed-radix FFT in LDS (axis lengths 2^a 3^b 5^c that are not powers of two; plan in mr_plan.hpp) --
// In-place DFT of 3 and 5 points (forward: exp(-2 pi i n k / R); inverse: conjugate), from the
// symmetric pairs a_r +- a_{R-r}: X_k = a_0 + sum_r cos(2 pi r k / R)(a_r + a_{R-r})
//                                         -+ i sum_r sin(2 pi r k / R)(a_r - a_{R-r}).
template <typename T, bool INV>
__device__ __forceinline__ void dft3(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2) {
    const T s = INV ? T(0.86602540378443864676) : T(-0.86602540378443864676);   // Im exp(-+2 pi i / 3)
    const cpx<T> t1 = cadd(a1, a2), t2 = csub(a1, a2);
    const cpx<T> m = {a0.x - T(0.5) * t1.x, a0.y - T(0.5) * t1.y};
    const cpx<T> js = {-s * t2.y, s * t2.x};   // i s (a1 - a2)
    a0 = cadd(a0, t1);
    a1 = cadd(m, js);
    a2 = csub(m, js);
}
template <typename T, bool INV>
__device__ __forceinline__ void dft5(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3, cpx<T>& a4) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);   // cos(2 pi / 5), cos(4 pi / 5)
    const T sg = INV ? T(1) : T(-1);
    const T s1 = sg * T(0.95105651629515357212), s2 = sg * T(0.58778525229247312917);   // sin(2 pi / 5), sin(4 pi / 5)
    const cpx<T> t1 = cadd(a1, a4), t2 = cadd(a2, a3), t3 = csub(a1, a4), t4 = csub(a2, a3);
    const cpx<T> m1 = {a0.x + c1 * t1.x + c2 * t2.x, a0.y + c1 * t1.y + c2 * t2.y};
    const cpx<T> m2 = {a0.x + c2 * t1.x + c1 * t2.x, a0.y + c2 * t1.y + c1 * t2.y};
    const cpx<T> u = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};   // X1, X4: m1 +- i u
    const cpx<T> w = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};   // X2, X3: m2 +- i w
    a0 = cadd(a0, cadd(t1, t2));
    a1 = {m1.x - u.y, m1.y + u.x};
    a4 = {m1.x + u.y, m1.y - u.x};
    a2 = {m2.x - w.y, m2.y + w.x};
    a3 = {m2.x + w.y, m2.y - w.x};
}

// One Stockham stage of radix R (decimation in time): butterfly j < n/R of the stage with NS = product of
// the earlier radices reads src[j + r n/R], multiplies input r by W_{NS R}^{r k} (k = j mod NS), takes the
// R-point DFT and writes dst[(j - k) R + k + r NS].
template <typename T, int R, bool INV>
__device__ __forceinline__ void mr_stage(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst, int n, int ns_prev,
                                         const cpx<T>* __restrict__ tw, int t, int nthr) {
    const int m = n / R, step = n / (ns_prev * R);
    for (int j = t; j < m; j += nthr) {
        const int k = j % ns_prev;
        cpx<T> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = src[j + r * m];
        if (ns_prev > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) a[r] = ctw<T, INV>(a[r], tw[r * k * step]);
        }
        if constexpr (R == 3) dft3<T, INV>(a[0], a[1], a[2]);
        else if constexpr (R == 5) dft5<T, INV>(a[0], a[1], a[2], a[3], a[4]);
        else dftR<T, R, INV>(a);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[base + r * ns_prev] = a[r];
    }
}

// Length-pl.n DFT of the sequence in `a` (LDS), with `b` (LDS, same length) as the other buffer of the
// ping-pong; nthr cooperating threads (index t).  Returns the buffer that holds the result (natural
// order).  Every thread of the block must call it with the same plan (it contains __syncthreads); the
// caller synchronises before the first stage reads `a`.  tw[m] = exp(-2 pi i m / n).
// act = false: the thread only takes part in the barriers (a block may hold more threads than its
// transforms use).
template <typename T, bool INV>
__device__ cpx<T>* fft_mr(cpx<T>* a, cpx<T>* b, const MrPlan& pl, const cpx<T>* __restrict__ tw, int t, int nthr,
                          bool act = true) {
    int ns = 1;
    const int t0 = act ? t : pl.n;   // an inactive thread starts past every stage's last butterfly
    for (int s = 0; s < pl.ns; ++s) {
        const int R = pl.r[s];
        switch (R) {
            case 2: mr_stage<T, 2, INV>(a, b, pl.n, ns, tw, t0, nthr); break;
            case 3: mr_stage<T, 3, INV>(a, b, pl.n, ns, tw, t0, nthr); break;
            case 4: mr_stage<T, 4, INV>(a, b, pl.n, ns, tw, t0, nthr); break;
            case 5: mr_stage<T, 5, INV>(a, b, pl.n, ns, tw, t0, nthr); break;
            default: mr_stage<T, 8, INV>(a, b, pl.n, ns, tw, t0, nthr); break;
        }
        __syncthreads();
        cpx<T>* c = a;
        a = b;
        b = c;
        ns *= R;
    }
    return a;
}

// Signed wavenumber of DFT index e on a length-n axis (any even n), Nyquist index mapped to 0.
__device__ __forceinline__ int kwave_n(int e, int n) { return e < n / 2 ? e : (2 * e == n ? 0 : e - n); }

// Signed integer wavenumber of DFT index e on a length-N axis, with the Nyquist index mapped to 0.
template <int N>
__device__ __forceinline__ int kwave(int e) {
    return e < N / 2 ? e : (e == N / 2 ? 0 : e - N);
}

// ---- reductions -------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum (fixed shuffle tree per wave, then fixed order over waves).
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < BLOCK / 64; ++i) s += sh[i];
    }
    __syncthreads();
    return s;   // valid in thread 0 only
}

}  // namespace regnk
