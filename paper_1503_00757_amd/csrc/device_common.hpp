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
template <int N>
struct LdsSize {
    static constexpr int value = N + (N >> 4);
};

// One length-N FFT on registers x[4] (see file header).  lds0 / lds1 are two LDS buffers of
// LdsSize<N> entries private to this transform; `buf` selects the buffer of the next exchange and
// must be carried from one call to the next so that consecutive exchanges always alternate buffers
// (a buffer is only rewritten after the barrier of the exchange that used the other one).  Must be
// reached by every thread of the block the same number of times (it contains __syncthreads).
template <typename T, int N, bool INV>
__device__ __forceinline__ void fft4(cpx<T> (&x)[4], cpx<T>* __restrict__ lds0,
                                     cpx<T>* __restrict__ lds1, int t,
                                     const cpx<T>* __restrict__ tw, int& buf) {
    constexpr int Q = N / 4;
    constexpr int LOG = ilog2(N);
    int Ns = 1;
    if constexpr (LOG & 1) {
        cpx<T>* o = buf ? lds1 : lds0;
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
            cpx<T>* o = buf ? lds1 : lds0;
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
