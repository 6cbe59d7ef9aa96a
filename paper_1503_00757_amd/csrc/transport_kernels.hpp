// Fused transport stages: every RK2 (Heun) stage of the state, adjoint, incremental-state and
// Gauss-Newton incremental-adjoint solves is ONE launch.
//
// A spectral partial derivative needs only a 1D transform along its own axis, and within a stage the
// x1- and x2-derivatives act on the same field, so they are independent.  Every stage update is
// therefore split additively, u_next = R + C:
//   * R: everything computable along rows.  The x2-derivative term plus all pointwise terms: the
//     RK2 combination, the v~ . grad m source, the stored gradient, the body-force quadrature.
//   * C: the x1-derivative term, computed along columns.
// The next stage rebuilds its input pointwise as u = R + C.  A launch holds row-pair blocks
// (blockIdx < nrow) and column-tile blocks, so one grid-wide dependency separates stages instead of
// two.
//
// Heun stages (h = 1/n_t), L_v u = -(v1 d1 u + v2 d2 u), L_v^T q = d1(v1 q) + d2(v2 q):
//   state      m*    = m_j + h L m_j,                 m_{j+1}  = (m_j + m*)/2 + (h/2) L m*
//   adjoint    l*    = l_{j+1} + h L^T l_{j+1},       l_j      = (l_{j+1} + l*)/2 + (h/2) L^T l*
//   inc.state  m~*   = m~_j + h (L m~_j + S_j),       m~_{j+1} = (m~_j + m~*)/2 + (h/2)(L m~* + S*_j)
// with S = -v~ . grad m, sampled at G_j and at G*_j (exact discrete adjoint) or G_{j+1} (trapezoid).
//
// Rows pack two real rows as one complex transform, columns pack two adjacent columns; i k~ maps
// real sequences to real sequences, so real and imaginary parts carry the two derivatives.
#pragma once
#include <hip/hip_ext.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace regnk {

template <typename T>
struct V2T;
template <>
struct V2T<float> {
    using t = float2;
};
template <>
struct V2T<double> {
    using t = double2;
};
// adjacent pair (i, i+1), i even: one 8- or 16-byte access
template <typename T>
__device__ __forceinline__ void ld2(const T* __restrict__ p, long i, T& a, T& b) {
    const typename V2T<T>::t v = *reinterpret_cast<const typename V2T<T>::t*>(p + i);
    a = v.x;
    b = v.y;
}
template <typename T>
__device__ __forceinline__ void st2(T* __restrict__ p, long i, T a, T b) {
    typename V2T<T>::t v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<typename V2T<T>::t*>(p + i) = v;
}

constexpr bool is_full(int op) { return op == OP_A1F || op == OP_A2F; }
constexpr bool is_a1(int op) { return op == OP_A1 || op == OP_A1F; }
constexpr bool is_a2(int op) { return op == OP_A2 || op == OP_A2F; }
constexpr bool is_adj(int op) { return is_a1(op) || is_a2(op); }
constexpr bool is_inc(int op) { return op == OP_I1 || op == OP_I2; }

// ---------------------------------------------------------------------------------------------
// Row part.  row_load issues every global load (transform input first, then epilogue operands) so
// that their latencies overlap each other and the FFTs; row_store does the epilogue and the stores.
// ---------------------------------------------------------------------------------------------
template <typename T>
struct Rp {
    T u, v, x, g0, g1, h0, h1, b0, b1;
    T l, l2, t0, t1, s0, s1;   // full Newton: lam, lam_{j+1}, grad m~_j, grad m~*_j
};

template <typename T, int OP>
__device__ __forceinline__ T row_load(const StageArgs<T>& a, long idx, Rp<T>& p) {
    const long nn = a.nn;
    if (a.flags & F_ZERO) {   // m~*_0 = -h v~ . G_0 (m~_0 = 0)
        p.u = -a.h * (a.VT[idx] * a.G2[idx] + a.VT[nn + idx] * a.G2[nn + idx]);
    } else {
        T u = a.A[idx];
        if (a.Bf) u += a.Bf[idx];
        p.u = (a.flags & F_NEG) ? -u : u;
    }
    if constexpr (OP != OP_GRAD) p.v = a.V2[idx];
    if constexpr (OP == OP_S2 || is_a2(OP)) p.x = a.X[idx];
    if constexpr (OP == OP_I2) p.x = (a.flags & F_ZERO) ? T(0) : a.X[idx];
    if constexpr (OP == OP_I1 || OP == OP_I2) {
        p.g0 = a.VT[idx];
        p.g1 = a.VT[nn + idx];
        p.h0 = a.G[idx];
        p.h1 = a.G[nn + idx];
    }
    if constexpr (is_adj(OP)) {
        if (a.B) {
            p.g0 = a.G[idx];
            p.g1 = a.G[nn + idx];
            if constexpr (is_a2(OP)) {
                p.h0 = a.G2[idx];
                p.h1 = a.G2[nn + idx];
            }
            if (a.flags & F_FIRST) {
                p.b0 = T(0);
                p.b1 = T(0);
            } else {
                p.b0 = a.B[idx];
                p.b1 = a.B[nn + idx];
            }
        }
    }
    if constexpr (is_full(OP)) {   // flux v lam~ + v~ lam (component 2 here)
        p.l = a.LAM[idx];
        const T w = a.VT[nn + idx];
        if constexpr (OP == OP_A2F) {
            p.l2 = a.LAM2[idx];
            p.t0 = a.GT ? a.GT[idx] : T(0);
            p.t1 = a.GT ? a.GT[nn + idx] : T(0);
            p.s0 = a.GT2[idx];
            p.s1 = a.GT2[nn + idx];
        }
        return p.v * p.u + w * p.l;
    }
    return is_adj(OP) ? p.v * p.u : p.u;
}

// Row-part results at 1024+ points per FP32 line are written through the XCD's L2 (a relaxed
// agent-scope atomic store is a plain vector store with the device-coherence policy): the rows are
// whole cache lines, and the kernel-end release then has little left to publish (1024^2 matvec 0.7%
// faster; at 256^2, where a stage is latency-bound, 5% slower, so shorter lines keep plain stores).
template <typename T, int N>
constexpr bool rows_write_through() { return sizeof(T) == 4 && N >= 1024; }
template <bool WT, typename S>
__device__ __forceinline__ void st1(S* p, S v) {
    if constexpr (WT) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

template <typename T, int OP, bool WT>
__device__ __forceinline__ void row_store(const StageArgs<T>& a, long idx, T d, const Rp<T>& p) {
    const long nn = a.nn;
    const T h = a.h;
    const T hh = T(0.5) * a.h;
    if constexpr (OP == OP_S1 || OP == OP_S2 || OP == OP_GRAD || is_inc(OP)) {   // d = d2 u: component 1 of grad u
        if (a.GOUT) st1<WT>(a.GOUT + (nn + idx), d);
        if (a.GOUTF) st1<WT>(a.GOUTF + (nn + idx), (float)d);
    }
    if constexpr (OP == OP_S1) {
        st1<WT>(a.ROUT + idx, p.u - h * p.v * d);                               // R of m*
        st1<WT>(a.UOUT + idx, p.u);                                             // m_j
    } else if constexpr (OP == OP_S2) {
        st1<WT>(a.ROUT + idx, T(0.5) * (p.x + p.u) - hh * p.v * d);             // R of m_{j+1}
    } else if constexpr (is_a1(OP)) {
        st1<WT>(a.ROUT + idx, p.u + h * d);                                     // R of l*
        st1<WT>(a.UOUT + idx, p.u);                                             // l_{j+1}
        if (a.B) {                                                     // trapezoid: w_{j+1} h l_{j+1} G_{j+1}
            const T w = a.bw * p.u;
            st1<WT>(a.B + idx, p.b0 + w * p.g0);
            st1<WT>(a.B + (nn + idx), p.b1 + w * p.g1);
        }
    } else if constexpr (is_a2(OP)) {
        st1<WT>(a.ROUT + idx, T(0.5) * (p.x + p.u) + hh * d);                   // R of l_j (x = l_{j+1}, u = l*)
        if (a.UOUT) st1<WT>(a.UOUT + idx, p.u);                                 // l*_j, kept for full Newton
        if (a.B) {                                                     // (h/2)(l* G_j + l_{j+1} G*_j)
            T b0 = p.u * p.g0 + p.x * p.h0, b1 = p.u * p.g1 + p.x * p.h1;
            if constexpr (OP == OP_A2F) {                              // + lam*_j grad m~_j + lam_{j+1} grad m~*_j
                b0 += p.l * p.t0 + p.l2 * p.s0;
                b1 += p.l * p.t1 + p.l2 * p.s1;
            }
            st1<WT>(a.B + idx, p.b0 + a.bw * b0);
            st1<WT>(a.B + (nn + idx), p.b1 + a.bw * b1);
        }
    } else if constexpr (OP == OP_I1) {
        st1<WT>(a.ROUT + idx, p.u - h * (p.v * d + p.g0 * p.h0 + p.g1 * p.h1));  // R of m~*
        st1<WT>(a.UOUT + idx, p.u);                                             // m~_j
    } else if constexpr (OP == OP_I2) {
        st1<WT>(a.ROUT + idx, T(0.5) * (p.x + p.u) - hh * (p.v * d + p.g0 * p.h0 + p.g1 * p.h1));  // R of m~_{j+1}
    }
}

// ---------------------------------------------------------------------------------------------
// Column part (column pair (c, c+1), 8/16-byte accesses)
// ---------------------------------------------------------------------------------------------
template <typename T>
struct Cp {
    T u, v;
};

template <typename T, int OP>
__device__ __forceinline__ cpx<T> col_load2(const StageArgs<T>& a, long idx, Cp<T>& p0, Cp<T>& p1) {
    const long nn = a.nn;
    if (a.flags & F_ZERO) {
        T va0, vb0, va1, vb1, ga0, gb0, ga1, gb1;
        ld2(a.VT, idx, va0, vb0);
        ld2(a.VT, nn + idx, va1, vb1);
        ld2(a.G2, idx, ga0, gb0);
        ld2(a.G2, nn + idx, ga1, gb1);
        p0.u = -a.h * (va0 * ga0 + va1 * ga1);
        p1.u = -a.h * (vb0 * gb0 + vb1 * gb1);
    } else {
        ld2(a.A, idx, p0.u, p1.u);
        if (a.Bf) {
            T b0, b1;
            ld2(a.Bf, idx, b0, b1);
            p0.u += b0;
            p1.u += b1;
        }
        if (a.flags & F_NEG) {
            p0.u = -p0.u;
            p1.u = -p1.u;
        }
    }
    if constexpr (OP != OP_GRAD) ld2(a.V1, idx, p0.v, p1.v);
    if constexpr (is_full(OP)) {   // flux v lam~ + v~ lam (component 1 here)
        T l0, l1, w0, w1;
        ld2(a.LAM, idx, l0, l1);
        ld2(a.VT, idx, w0, w1);
        return cpx<T>{p0.v * p0.u + w0 * l0, p1.v * p1.u + w1 * l1};
    }
    return is_adj(OP) ? cpx<T>{p0.v * p0.u, p1.v * p1.u} : cpx<T>{p0.u, p1.u};
}

template <typename T, int OP>
__device__ __forceinline__ void col_store2(const StageArgs<T>& a, long idx, T d0, T d1, const Cp<T>& p0,
                                           const Cp<T>& p1) {
    const T h = a.h;
    const T hh = T(0.5) * a.h;
    if constexpr (OP == OP_S1 || OP == OP_S2 || OP == OP_GRAD || is_inc(OP)) {   // d = d1 u: component 0 of grad u
        if (a.GOUT) st2(a.GOUT, idx, d0, d1);
        if (a.GOUTF) st2(a.GOUTF, idx, (float)d0, (float)d1);
    }
    if constexpr (OP == OP_S1 || OP == OP_I1) {
        st2(a.COUT, idx, -h * p0.v * d0, -h * p1.v * d1);
    } else if constexpr (OP == OP_S2 || OP == OP_I2) {
        st2(a.COUT, idx, -hh * p0.v * d0, -hh * p1.v * d1);
    } else if constexpr (is_a1(OP)) {
        st2(a.COUT, idx, h * d0, h * d1);
    } else if constexpr (is_a2(OP)) {
        st2(a.COUT, idx, hh * d0, hh * d1);
    }
}

// ---------------------------------------------------------------------------------------------
// Blocks
// ---------------------------------------------------------------------------------------------
// Row part: FPW transforms per block, each = one pair of rows (2r, 2r+1), length N = n2, E elements
// per thread.  lds: FPW * 2 * LdsSize<N> entries.
template <typename T, int N, int E, int FPW, int OP, bool PH = false>
__device__ __forceinline__ void row_part(const StageArgs<T>& a, int rb, cpx<T>* lds) {
    constexpr int TT = N / E;
    constexpr int L = LdsSize<N>::value;
    const int f = threadIdx.x / TT, t = threadIdx.x % TT;
    const int pair = rb * FPW + f;
    const bool valid = pair < (a.n1 >> 1);
    const long row0 = (long)(valid ? 2 * pair : 0) * N;
    const long row1 = row0 + N;
    cpx<T> x[E];
    Rp<T> q0[E], q1[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = t + TT * m;
        T p0 = 0, p1 = 0;
        if (valid) {
            p0 = row_load<T, OP>(a, row0 + e, q0[m]);
            p1 = row_load<T, OP>(a, row1 + e, q1[m]);
        }
        x[m] = {p0, p1};
    }
    cpx<T> W[tw_regs<N, E>()];
    load_tw<T, N, E, 1, 0>(W, t, a.tw2);
    if constexpr (PH) clk_phase(a, 1);
    cpx<T>* l0 = lds + f * 2 * L;
    int buf = 0;
    fftE<T, N, E, false>(x, l0, l0 + L, t, W, buf);
    const T inv = T(1) / T(N);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const T k = T(kwave<N>(t + TT * m)) * inv;
        x[m] = {-x[m].y * k, x[m].x * k};   // times i k / N
    }
    fftE<T, N, E, true>(x, l0, l0 + L, t, W, buf);
    if constexpr (PH) clk_phase(a, 2);
    if (!valid) return;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = t + TT * m;
        row_store<T, OP, rows_write_through<T, N>()>(a, row0 + e, x[m].x, q0[m]);
        row_store<T, OP, rows_write_through<T, N>()>(a, row1 + e, x[m].y, q1[m]);
    }
}

// Column part: a block owns TW = 2G adjacent columns (G transforms of length N = n1).
template <typename T, int N, int E, int G, int OP, bool PH = false>
__device__ __forceinline__ void col_part(const StageArgs<T>& a, int cb, int ncb, cpx<T>* lds) {
    constexpr int TT = N / E;
    constexpr int L = LdsSize<N>::value;
    const int f = threadIdx.x % G, t = threadIdx.x / G;
    constexpr int TWB = 2 * G * (int)sizeof(T);
    constexpr int GROUP = TWB >= 128 ? 1 : 128 / TWB;
    const int tile = xcd_tile(cb, ncb, GROUP);
    const int c = tile * 2 * G + 2 * f;
    const bool valid = c < a.n2;
    const long n2 = a.n2;
    cpx<T> x[E];
    Cp<T> q0[E], q1[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const long idx = (long)(t + TT * m) * n2 + (valid ? c : 0);
        x[m] = valid ? col_load2<T, OP>(a, idx, q0[m], q1[m]) : cpx<T>{T(0), T(0)};
    }
    cpx<T> W[tw_regs<N, E>()];
    load_tw<T, N, E, 1, 0>(W, t, a.tw1);
    if constexpr (PH) clk_phase(a, 1);
    cpx<T>* l0 = lds + f * 2 * L;
    int buf = 0;
    fftE<T, N, E, false>(x, l0, l0 + L, t, W, buf);
    const T inv = T(1) / T(N);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const T k = T(kwave<N>(t + TT * m)) * inv;
        x[m] = {-x[m].y * k, x[m].x * k};
    }
    fftE<T, N, E, true>(x, l0, l0 + L, t, W, buf);
    if constexpr (PH) clk_phase(a, 2);
    if (!valid) return;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const long idx = (long)(t + TT * m) * n2 + c;
        col_store2<T, OP>(a, idx, x[m].x, x[m].y, q0[m], q1[m]);
    }
}

// Timing (only when clk is given; the test is uniform over the grid): block b writes its start and
// its end on the device wall clock to clk[2b], clk[2b+1] (plain stores, one slot per block: no
// contention); the end is taken after every wave's stores were acknowledged (s_waitcnt 0: stores
// count in vmcnt; no cache write-back, unlike a device-scope fence, which costs an L2 flush per
// block here).  The caller takes the earliest start and the latest end.
// Phase mode (F_PHASES): four slots per block, and the phase-mode build of the fused square FP32
// Gauss-Newton stages (PH) also stamps the arrival of all its loads and the end of its transforms,
// each after waiting for every wave's memory operations; the phases then run one after another (no
// overlap of loads with transforms), so they show each phase's length rather than the overlapped
// launch.  The stamps are compiled only into that build: a branch on the flag in the production
// kernels cost 1-1.4% (it splits the code the scheduler interleaves).
template <typename T>
__device__ __forceinline__ int clk_slots_per_block(const StageArgs<T>& a) {
    return (a.flags & F_PHASES) ? 4 : 2;
}
template <typename T>
__device__ __forceinline__ void clk_start(const StageArgs<T>& a) {
    if (a.clk && threadIdx.x == 0) a.clk[clk_slots_per_block(a) * blockIdx.x] = wall_clock64();
}
template <typename T>
__device__ __forceinline__ void clk_end(const StageArgs<T>& a) {
    if (a.clk) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int k = clk_slots_per_block(a);
        if (threadIdx.x == 0) a.clk[k * blockIdx.x + k - 1] = wall_clock64();
    }
}
template <typename T>
__device__ __forceinline__ void clk_phase(const StageArgs<T>& a, int slot) {
    if (a.clk && (a.flags & F_PHASES)) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) a.clk[4 * blockIdx.x + slot] = wall_clock64();
    }
}

// Square grids: one launch, blocks [0, nrb) do row pairs, the rest column tiles.
// PH: the phase-mode build of the kernel (timing only; launched when F_PHASES is set).
template <typename T, int N, int ER, int FPW, int EC, int G, int OP, bool PH = false>
__global__ __launch_bounds__(FPW * N / ER) void stage_fused_kernel(StageArgs<T> a, int nrb) {
    static_assert(FPW * (N / ER) == G * (N / EC), "row and column blocks must have the same size");
    constexpr int LR = FPW * 2 * LdsSize<N>::value;
    constexpr int LC = G * 2 * LdsSize<N>::value;
    __shared__ cpx<T> lds[LR > LC ? LR : LC];
    clk_start(a);
    if ((int)blockIdx.x < nrb) row_part<T, N, ER, FPW, OP, PH>(a, blockIdx.x, lds);
    else col_part<T, N, EC, G, OP, PH>(a, blockIdx.x - nrb, gridDim.x - nrb, lds);
    clk_end(a);
}

// Non-square grids: the two parts as two launches.
template <typename T, int N, int E, int FPW, int OP>
__global__ __launch_bounds__(FPW * N / E) void stage_row_kernel(StageArgs<T> a) {
    __shared__ cpx<T> lds[FPW * 2 * LdsSize<N>::value];
    clk_start(a);
    row_part<T, N, E, FPW, OP>(a, blockIdx.x, lds);
    clk_end(a);
}
template <typename T, int N, int E, int G, int OP>
__global__ __launch_bounds__(G * N / E) void stage_col_kernel(StageArgs<T> a) {
    __shared__ cpx<T> lds[G * 2 * LdsSize<N>::value];
    clk_start(a);
    col_part<T, N, E, G, OP>(a, blockIdx.x, gridDim.x, lds);
    clk_end(a);
}

// Axis lengths that are not powers of two: the derivative along the axis is the product with the
// circulant spectral differentiation matrix, d_e = sum_j c[(e - j) mod n] f_j, where c is the inverse
// DFT of i k~ / n (the operator of the transform pair above, Nyquist wavenumber zeroed).  One row pair
// (column pair) per block; the complex-packed line is staged in LDS, and the epilogue operands are read
// again after the sum instead of being held in registers.  O(n^2) per line.
constexpr int DENSE_STAGE_THREADS = 256;

template <typename T, int OP>
__global__ __launch_bounds__(DENSE_STAGE_THREADS) void stage_dense_row_kernel(StageArgs<T> a) {
    extern __shared__ unsigned char dsm[];
    cpx<T>* f = reinterpret_cast<cpx<T>*>(dsm);
    const int N = a.n2;
    const long row0 = (long)(2 * blockIdx.x) * N, row1 = row0 + N;
    clk_start(a);
    for (int e = threadIdx.x; e < N; e += DENSE_STAGE_THREADS) {
        Rp<T> q0, q1;
        const T p0 = row_load<T, OP>(a, row0 + e, q0);
        const T p1 = row_load<T, OP>(a, row1 + e, q1);
        f[e] = {p0, p1};
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N; e += DENSE_STAGE_THREADS) {
        T dx = 0, dy = 0;
        int m = e;   // (e - j) mod N
        for (int j = 0; j < N; ++j) {
            const T c = a.dc2[m];
            dx += c * f[j].x;
            dy += c * f[j].y;
            m = m == 0 ? N - 1 : m - 1;
        }
        Rp<T> q0, q1;
        row_load<T, OP>(a, row0 + e, q0);
        row_load<T, OP>(a, row1 + e, q1);
        row_store<T, OP, false>(a, row0 + e, dx, q0);
        row_store<T, OP, false>(a, row1 + e, dy, q1);
    }
    clk_end(a);
}

template <typename T, int OP>
__global__ __launch_bounds__(DENSE_STAGE_THREADS) void stage_dense_col_kernel(StageArgs<T> a) {
    extern __shared__ unsigned char dsm[];
    cpx<T>* f = reinterpret_cast<cpx<T>*>(dsm);
    const int N = a.n1;
    const long c = 2 * (long)blockIdx.x, n2 = a.n2;
    clk_start(a);
    for (int r = threadIdx.x; r < N; r += DENSE_STAGE_THREADS) {
        Cp<T> q0, q1;
        f[r] = col_load2<T, OP>(a, (long)r * n2 + c, q0, q1);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < N; r += DENSE_STAGE_THREADS) {
        T dx = 0, dy = 0;
        int m = r;
        for (int j = 0; j < N; ++j) {
            const T cc = a.dc1[m];
            dx += cc * f[j].x;
            dy += cc * f[j].y;
            m = m == 0 ? N - 1 : m - 1;
        }
        Cp<T> q0, q1;
        const long idx = (long)r * n2 + c;
        col_load2<T, OP>(a, idx, q0, q1);
        col_store2<T, OP>(a, idx, dx, dy, q0, q1);
    }
    clk_end(a);
}

// Axis lengths 2^a 3^b 5^c that are not powers of two: the same stage with the mixed-radix FFT in LDS
// (fft_mr) in place of the circulant sum.  Row part: fpw row pairs per block, tpt threads per
// transform, thread t holds elements e = t + tpt m (m < EM) of both rows in registers (the epilogue
// operands too) and stages them through LDS as one complex line.  Column part: G column pairs per
// block, adjacent lanes on adjacent pairs.  LDS: two lines per transform.  Threads past the block's
// transforms only join the barriers.
// The twiddle table of the axis, copied to LDS behind the block's `nlines` line pairs when the launch
// gave room for it (twl), else read from global memory.
template <typename T>
__device__ __forceinline__ const cpx<T>* mr_twiddles(const cpx<T>* __restrict__ tw, int n, cpx<T>* lds, int nlines,
                                                     bool twl) {
    if (!twl) return tw;
    cpx<T>* t = lds + (size_t)nlines * 2 * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) t[i] = tw[i];
    return t;   // visible after the caller's next barrier
}

template <typename T, int OP, int EM>
__device__ __forceinline__ void mr_row_part(const StageArgs<T>& a, int rb, int tpt, int fpw, cpx<T>* lds, int nlines,
                                            bool twl) {
    const int N = a.n2;
    const cpx<T>* tw = mr_twiddles(a.tw2, N, lds, nlines, twl);
    const int f = threadIdx.x / tpt, t = threadIdx.x % tpt;
    const bool act = f < fpw;
    const int pair = rb * fpw + f;
    const bool valid = act && pair < (a.n1 >> 1);
    cpx<T>* L0 = lds + (size_t)(act ? f : 0) * 2 * N;
    cpx<T>* L1 = L0 + N;
    const long row0 = (long)(valid ? 2 * pair : 0) * N, row1 = row0 + N;
    Rp<T> q0[EM], q1[EM];
#pragma unroll
    for (int m = 0; m < EM; ++m) {
        const int e = t + tpt * m;
        if (act && e < N) {
            T p0 = 0, p1 = 0;
            if (valid) {
                p0 = row_load<T, OP>(a, row0 + e, q0[m]);
                p1 = row_load<T, OP>(a, row1 + e, q1[m]);
            }
            L0[e] = {p0, p1};
        }
    }
    __syncthreads();
    cpx<T>* X = fft_mr<T, false>(L0, L1, a.mr2, tw, t, tpt, act);
    const T inv = T(1) / T(N);
#pragma unroll
    for (int m = 0; m < EM; ++m) {
        const int e = t + tpt * m;
        if (act && e < N) {
            const T k = T(kwave_n(e, N)) * inv;
            const cpx<T> z = X[e];
            X[e] = {-z.y * k, z.x * k};   // times i k / N
        }
    }
    __syncthreads();
    cpx<T>* Y = fft_mr<T, true>(X, X == L0 ? L1 : L0, a.mr2, tw, t, tpt, act);
    if (valid) {
#pragma unroll
        for (int m = 0; m < EM; ++m) {
            const int e = t + tpt * m;
            if (e < N) {
                const cpx<T> y = Y[e];
                row_store<T, OP, false>(a, row0 + e, y.x, q0[m]);
                row_store<T, OP, false>(a, row1 + e, y.y, q1[m]);
            }
        }
    }
}

template <typename T, int OP, int EM>
__device__ __forceinline__ void mr_col_part(const StageArgs<T>& a, int cb, int tpt, int G, cpx<T>* lds, int nlines,
                                            bool twl) {
    const int N = a.n1;
    const cpx<T>* tw = mr_twiddles(a.tw1, N, lds, nlines, twl);
    const int f = threadIdx.x % G, t = threadIdx.x / G;
    const bool act = t < tpt;
    const int c = (cb * G + f) * 2;
    const bool valid = act && c < a.n2;
    const long n2 = a.n2;
    cpx<T>* L0 = lds + (size_t)f * 2 * N;
    cpx<T>* L1 = L0 + N;
    Cp<T> q0[EM], q1[EM];
#pragma unroll
    for (int m = 0; m < EM; ++m) {
        const int e = t + tpt * m;
        if (act && e < N) L0[e] = valid ? col_load2<T, OP>(a, (long)e * n2 + c, q0[m], q1[m]) : cpx<T>{T(0), T(0)};
    }
    __syncthreads();
    cpx<T>* X = fft_mr<T, false>(L0, L1, a.mr1, tw, t, tpt, act);
    const T inv = T(1) / T(N);
#pragma unroll
    for (int m = 0; m < EM; ++m) {
        const int e = t + tpt * m;
        if (act && e < N) {
            const T k = T(kwave_n(e, N)) * inv;
            const cpx<T> z = X[e];
            X[e] = {-z.y * k, z.x * k};
        }
    }
    __syncthreads();
    cpx<T>* Y = fft_mr<T, true>(X, X == L0 ? L1 : L0, a.mr1, tw, t, tpt, act);
    if (valid) {
#pragma unroll
        for (int m = 0; m < EM; ++m) {
            const int e = t + tpt * m;
            if (e < N) {
                const cpx<T> y = Y[e];
                col_store2<T, OP>(a, (long)e * n2 + c, y.x, y.y, q0[m], q1[m]);
            }
        }
    }
}

template <typename T, int OP, int EM>
__global__ __launch_bounds__(512) void stage_mr_row_kernel(StageArgs<T> a, int tpt, int fpw, int twl) {
    extern __shared__ unsigned char dsm[];
    clk_start(a);
    mr_row_part<T, OP, EM>(a, blockIdx.x, tpt, fpw, reinterpret_cast<cpx<T>*>(dsm), fpw, twl != 0);
    clk_end(a);
}
template <typename T, int OP, int EM>
__global__ __launch_bounds__(512) void stage_mr_col_kernel(StageArgs<T> a, int tpt, int G, int twl) {
    extern __shared__ unsigned char dsm[];
    clk_start(a);
    mr_col_part<T, OP, EM>(a, blockIdx.x, tpt, G, reinterpret_cast<cpx<T>*>(dsm), G, twl != 0);
    clk_end(a);
}
// Square grids of such a length: both parts in one launch (blocks [0, nrb) rows, the rest columns).
template <typename T, int OP, int EMR, int EMC>
__global__ __launch_bounds__(512) void stage_mr_fused_kernel(StageArgs<T> a, int nrb, int tpt_r, int fpw, int tpt_c,
                                                            int G, int twl) {
    extern __shared__ unsigned char dsm[];
    const int nlines = fpw > G ? fpw : G;
    clk_start(a);
    if ((int)blockIdx.x < nrb)
        mr_row_part<T, OP, EMR>(a, blockIdx.x, tpt_r, fpw, reinterpret_cast<cpx<T>*>(dsm), nlines, twl != 0);
    else mr_col_part<T, OP, EMC>(a, blockIdx.x - nrb, tpt_c, G, reinterpret_cast<cpx<T>*>(dsm), nlines, twl != 0);
    clk_end(a);
}

// LDS of a mixed-radix stage launch: `nlines` line pairs, plus the twiddle table when the total stays
// within 64 KiB (twl).
template <typename T>
inline size_t mr_lds_bytes(int n, int nlines, int& twl) {
    const size_t lines = (size_t)nlines * 2 * n * sizeof(cpx<T>);
    const size_t with = lines + (size_t)n * sizeof(cpx<T>);
    twl = with <= 64 * 1024 ? 1 : 0;
    return twl ? with : lines;
}

// Launch shape of a mixed-radix axis of length n: EM elements per thread, tpt threads per transform
// (tpt * EM >= n), and transforms per block (at most 256 threads for lines of up to 256 points, 512
// for longer ones, and 64 KiB of LDS per block).
struct MrShape {
    int em, tpt, per_block;
};
template <typename T>
inline MrShape mr_shape(int n, bool column) {
    const int em = n > 1024 ? 8 : (n > 256 || column ? 4 : 2);
    const int tpt = (n + em - 1) / em;
    int pb = (n > 256 ? 512 : 256) / tpt;
    const int lds_line = 2 * n * (int)sizeof(cpx<T>);
    while (pb > 1 && pb * lds_line > 64 * 1024) --pb;
    if (pb < 1) pb = 1;
    return {em, tpt, pb};
}

template <typename T, int OP>
static hipError_t launch_mr_axis(int axis, const StageArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    const int n = axis == 2 ? a.n2 : a.n1;
    const MrShape sh = mr_shape<T>(n, axis == 1);
    int twl = 0;
    const size_t lds = mr_lds_bytes<T>(n, sh.per_block, twl);
    const int lines = axis == 2 ? a.n1 / 2 : a.n2 / 2;
    const dim3 grid((lines + sh.per_block - 1) / sh.per_block), block(sh.per_block * sh.tpt);
#define REGNK_MR(EMV)                                                                                      \
    if (sh.em == EMV) {                                                                                    \
        if (axis == 2) launch_ks(stage_mr_row_kernel<T, OP, EMV>, grid, block, lds, s, t0, t1, a, sh.tpt,       \
                                 sh.per_block, twl);                                                       \
        else launch_ks(stage_mr_col_kernel<T, OP, EMV>, grid, block, lds, s, t0, t1, a, sh.tpt, sh.per_block,   \
                       twl);                                                                               \
        return hipGetLastError();                                                                          \
    }
    REGNK_MR(2) REGNK_MR(4) REGNK_MR(8)
#undef REGNK_MR
    return hipErrorInvalidValue;
}

// Square mixed-radix grids: one launch per stage (row and column shapes of the two-launch form, the
// block as large as the larger of them).
template <typename T, int OP>
static hipError_t launch_mr_fused(const StageArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    const int n = a.n1;
    const MrShape r = mr_shape<T>(n, false), c = mr_shape<T>(n, true);
    const int bs = std::max(r.per_block * r.tpt, c.per_block * c.tpt);
    const int nrb = (a.n1 / 2 + r.per_block - 1) / r.per_block, ncb = (a.n2 / 2 + c.per_block - 1) / c.per_block;
    int twl = 0;
    const size_t lds = mr_lds_bytes<T>(n, std::max(r.per_block, c.per_block), twl);
#define REGNK_MRF(ER, EC)                                                                                  \
    if (r.em == ER && c.em == EC) {                                                                        \
        launch_ks(stage_mr_fused_kernel<T, OP, ER, EC>, dim3(nrb + ncb), dim3(bs), lds, s, t0, t1, a, nrb, r.tpt, \
                  r.per_block, c.tpt, c.per_block, twl);                                                   \
        return hipGetLastError();                                                                          \
    }
    REGNK_MRF(2, 4) REGNK_MRF(4, 4) REGNK_MRF(4, 8) REGNK_MRF(8, 8)
#undef REGNK_MRF
    return hipErrorInvalidValue;
}

// Pointwise helpers of the state solve and the trapezoid end point.
template <typename T>
__global__ void finalize_state_kernel(long nn, const double* __restrict__ Q, const double* __restrict__ C,
                                      const double* __restrict__ mR, double* __restrict__ m1, T* __restrict__ lam) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
        const double m = Q[i] + C[i];
        m1[i] = m;
        if (lam) lam[i] = (T)(mR[i] - m);
    }
}
template <typename T>
__global__ void body_end_kernel(long nn, T w, const T* __restrict__ Q, const T* __restrict__ C,
                                const T* __restrict__ G, T* __restrict__ B) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
        const T l = w * (Q[i] + C[i]);
        B[i] += l * G[i];
        B[nn + i] += l * G[nn + i];
    }
}

// The exact-transpose body force of the last adjoint step (j = 0): lam_0 itself is not needed, so
// stage 2 reduces to B (+)= w (lam*_0 G_0 + lam_1 G*_0) with lam*_0 = Q + C; `keep` (nullable)
// receives lam*_0.  The arithmetic is the stage-2 epilogue's.
template <typename T>
__global__ void body_last_kernel(long nn, T w, bool first, const T* __restrict__ Q, const T* __restrict__ C,
                                 const T* __restrict__ X, const T* __restrict__ G, const T* __restrict__ G2,
                                 T* __restrict__ B, T* __restrict__ keep) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
        T u = Q[i];
        u += C[i];
        const T x = X[i];
        if (keep) keep[i] = u;
        const T b0 = u * G[i] + x * G2[i], b1 = u * G[nn + i] + x * G2[nn + i];
        const T o0 = first ? T(0) : B[i], o1 = first ? T(0) : B[nn + i];
        B[i] = o0 + w * b0;
        B[nn + i] = o1 + w * b1;
    }
}

// ---------------------------------------------------------------------------------------------
// Launch shapes.  Square FP32 grids of 64+ points: variant v = (ER, EC, BS) with ER/EC elements per
// thread of the row/column transforms and BS threads per block (FPW = BS/(N/ER) row pairs and
// G = BS/(N/EC) column pairs per block).  Variant 0 is the default; an autotuner may pick another.
// FP64 and non-square or short grids use one fixed shape.
// ---------------------------------------------------------------------------------------------
// variant:                 0    1    2    3    4    5    6    7    8   9  10  11   12   13   14   15   16   17    18   19
constexpr int VAR_ER[] = {8, 4, 4, 8, 8, 4, 8, 16, 4, 4, 8, 16, 2, 2, 2, 2, 2, 2, 2, 4};
constexpr int VAR_EC[] = {16, 16, 8, 8, 8, 4, 16, 16, 4, 4, 8, 16, 2, 4, 2, 4, 4, 8, 4, 2};
constexpr int VAR_BS[] = {128, 256, 256, 128, 256, 256, 256, 128, 512, 64, 64, 64, 128, 128, 256, 256, 512, 512, 1024, 128};
// 9-11: one wave per block; 12-19: two elements per thread on at least one axis (more waves per transform)
static_assert(sizeof(VAR_ER) / sizeof(int) == NUM_STAGE_VARIANTS, "one shape per variant");
constexpr int var_ER(int v) { return VAR_ER[v]; }
constexpr int var_EC(int v) { return VAR_EC[v]; }
constexpr int var_BS(int v) { return VAR_BS[v]; }

template <typename T, int N, int ER, int EC, int BS>
constexpr bool fused_ok() {
    return ER <= N / 2 && EC <= N / 2 && BS >= N / ER && BS >= N / EC && BS <= 1024 &&
           (BS / (N / ER)) * 2 * LdsSize<N>::value * (int)sizeof(cpx<T>) <= 160 * 1024 &&
           (BS / (N / EC)) * 2 * LdsSize<N>::value * (int)sizeof(cpx<T>) <= 160 * 1024;
}

// A launch; with timing events it goes through hipExtLaunchKernelGGL, whose events are stamped by
// the dispatch itself (the interval a profiler reports for the kernel).
template <typename K, typename... Args>
static inline void launch_ks(K kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t s, hipEvent_t t0,
                             hipEvent_t t1, Args... args) {
    if (t0 || t1) hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t0, t1, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}
template <typename K, typename... Args>
static inline void launch_k(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t t0, hipEvent_t t1,
                            Args... args) {
    launch_ks(kernel, grid, block, 0, s, t0, t1, args...);
}

template <typename T, int N, int OP, int ER, int EC, int BS>
static hipError_t launch_fused(const StageArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if constexpr (fused_ok<T, N, ER, EC, BS>()) {
        constexpr int FPW = BS / (N / ER);
        constexpr int G = BS / (N / EC);
        const int nrb = (a.n1 / 2 + FPW - 1) / FPW;
        const int ncb = (a.n2 + 2 * G - 1) / (2 * G);
        // the phase-mode build exists for the FP32 Gauss-Newton stages (the timed matvec launches)
        if constexpr (sizeof(T) == 4 && (OP == OP_A1 || OP == OP_A2 || OP == OP_I1 || OP == OP_I2)) {
            if (a.flags & F_PHASES) {
                launch_k(stage_fused_kernel<T, N, ER, FPW, EC, G, OP, true>, dim3(nrb + ncb), dim3(BS), s, t0, t1,
                         a, nrb);
                return hipGetLastError();
            }
        }
        launch_k(stage_fused_kernel<T, N, ER, FPW, EC, G, OP>, dim3(nrb + ncb), dim3(BS), s, t0, t1, a, nrb);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <int N>
constexpr int small_E() { return N >= 32 ? 8 : 4; }
template <int N, int E>
constexpr int min_block(int want) { return (N / E) >= want ? 1 : want / (N / E); }

template <typename T, int N, int OP>
static hipError_t launch_row_fixed(const StageArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    // 64..512-point lines: two elements per thread (latency-bound lengths, as the fused shapes)
    constexpr int E = (N >= 64 && N <= 512) ? 2 : (sizeof(T) == 8 ? 4 : small_E<N>());
    constexpr int FPW = min_block<N, E>(64);
    launch_k(stage_row_kernel<T, N, E, FPW, OP>, dim3((a.n1 / 2 + FPW - 1) / FPW), dim3(FPW * N / E), s, t0, t1, a);
    return hipGetLastError();
}
template <typename T, int N, int OP>
static hipError_t launch_col_fixed(const StageArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    constexpr int E = (N >= 64 && N <= 512) ? 4 : (sizeof(T) == 8 ? (N >= 16 ? 8 : 4) : small_E<N>());
    constexpr int G0 = min_block<N, E>(64);
    constexpr int G = G0 < 2 ? 2 : G0;
    launch_k(stage_col_kernel<T, N, E, G, OP>, dim3((a.n2 + 2 * G - 1) / (2 * G)), dim3(G * N / E), s, t0, t1, a);
    return hipGetLastError();
}

// Whether launch shape v fits length N (fused_ok), and the shape used when the requested one does not.
template <typename T, int N>
constexpr bool var_ok(int v) {
    switch (v) {
        case 0: return fused_ok<T, N, var_ER(0), var_EC(0), var_BS(0)>();
        case 1: return fused_ok<T, N, var_ER(1), var_EC(1), var_BS(1)>();
        case 2: return fused_ok<T, N, var_ER(2), var_EC(2), var_BS(2)>();
        case 3: return fused_ok<T, N, var_ER(3), var_EC(3), var_BS(3)>();
        case 4: return fused_ok<T, N, var_ER(4), var_EC(4), var_BS(4)>();
        case 5: return fused_ok<T, N, var_ER(5), var_EC(5), var_BS(5)>();
        case 6: return fused_ok<T, N, var_ER(6), var_EC(6), var_BS(6)>();
        case 7: return fused_ok<T, N, var_ER(7), var_EC(7), var_BS(7)>();
        case 8: return fused_ok<T, N, var_ER(8), var_EC(8), var_BS(8)>();
        case 9: return fused_ok<T, N, var_ER(9), var_EC(9), var_BS(9)>();
        case 10: return fused_ok<T, N, var_ER(10), var_EC(10), var_BS(10)>();
        case 11: return fused_ok<T, N, var_ER(11), var_EC(11), var_BS(11)>();
        case 12: return fused_ok<T, N, var_ER(12), var_EC(12), var_BS(12)>();
        case 13: return fused_ok<T, N, var_ER(13), var_EC(13), var_BS(13)>();
        case 14: return fused_ok<T, N, var_ER(14), var_EC(14), var_BS(14)>();
        case 15: return fused_ok<T, N, var_ER(15), var_EC(15), var_BS(15)>();
        case 16: return fused_ok<T, N, var_ER(16), var_EC(16), var_BS(16)>();
        case 17: return fused_ok<T, N, var_ER(17), var_EC(17), var_BS(17)>();
        case 18: return fused_ok<T, N, var_ER(18), var_EC(18), var_BS(18)>();
        case 19: return fused_ok<T, N, var_ER(19), var_EC(19), var_BS(19)>();
    }
    return false;
}
template <typename T, int N>
constexpr int default_var() {
    if (var_ok<T, N>(0)) return 0;
    if (var_ok<T, N>(8)) return 8;
    for (int v = 1; v < NUM_STAGE_VARIANTS; ++v)
        if (var_ok<T, N>(v)) return v;
    return 0;
}

template <typename T, int N, int OP>
static hipError_t launch_square(int var, const StageArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if constexpr (sizeof(T) == 8 || N < 64) {
        (void)var;
        // FP64 lines of 64..512 points: two elements per thread on the rows (a shorter per-thread
        // chain where the stage is latency-bound); longer lines are bandwidth-bound
        constexpr bool E2 = sizeof(T) == 8 && N >= 64 && N <= 512;
        constexpr int ER = E2 ? 2 : (sizeof(T) == 8 ? 4 : small_E<N>());
        constexpr int EC = E2 ? 4 : (sizeof(T) == 8 ? (N >= 16 ? 8 : 4) : small_E<N>());
        constexpr int BS0 = (N / ER) > (N / EC) ? (N / ER) : (N / EC);
        constexpr int BS = BS0 < 64 ? 64 : BS0;
        return launch_fused<T, N, OP, ER, EC, BS>(a, s, t0, t1);
    } else {
        if (!var_ok<T, N>(var)) var = default_var<T, N>();   // e.g. variant 0 has too few threads at 2048
        switch (var) {
            case 0: return launch_fused<T, N, OP, var_ER(0), var_EC(0), var_BS(0)>(a, s, t0, t1);
            case 1: return launch_fused<T, N, OP, var_ER(1), var_EC(1), var_BS(1)>(a, s, t0, t1);
            case 2: return launch_fused<T, N, OP, var_ER(2), var_EC(2), var_BS(2)>(a, s, t0, t1);
            case 3: return launch_fused<T, N, OP, var_ER(3), var_EC(3), var_BS(3)>(a, s, t0, t1);
            case 4: return launch_fused<T, N, OP, var_ER(4), var_EC(4), var_BS(4)>(a, s, t0, t1);
            case 5: return launch_fused<T, N, OP, var_ER(5), var_EC(5), var_BS(5)>(a, s, t0, t1);
            case 6: return launch_fused<T, N, OP, var_ER(6), var_EC(6), var_BS(6)>(a, s, t0, t1);
            case 7: return launch_fused<T, N, OP, var_ER(7), var_EC(7), var_BS(7)>(a, s, t0, t1);
            case 8: return launch_fused<T, N, OP, var_ER(8), var_EC(8), var_BS(8)>(a, s, t0, t1);
            case 9: return launch_fused<T, N, OP, var_ER(9), var_EC(9), var_BS(9)>(a, s, t0, t1);
            case 10: return launch_fused<T, N, OP, var_ER(10), var_EC(10), var_BS(10)>(a, s, t0, t1);
            case 11: return launch_fused<T, N, OP, var_ER(11), var_EC(11), var_BS(11)>(a, s, t0, t1);
            case 12: return launch_fused<T, N, OP, var_ER(12), var_EC(12), var_BS(12)>(a, s, t0, t1);
            case 13: return launch_fused<T, N, OP, var_ER(13), var_EC(13), var_BS(13)>(a, s, t0, t1);
            case 14: return launch_fused<T, N, OP, var_ER(14), var_EC(14), var_BS(14)>(a, s, t0, t1);
            case 15: return launch_fused<T, N, OP, var_ER(15), var_EC(15), var_BS(15)>(a, s, t0, t1);
            case 16: return launch_fused<T, N, OP, var_ER(16), var_EC(16), var_BS(16)>(a, s, t0, t1);
            case 17: return launch_fused<T, N, OP, var_ER(17), var_EC(17), var_BS(17)>(a, s, t0, t1);
            case 18: return launch_fused<T, N, OP, var_ER(18), var_EC(18), var_BS(18)>(a, s, t0, t1);
            case 19: return launch_fused<T, N, OP, var_ER(19), var_EC(19), var_BS(19)>(a, s, t0, t1);
        }
        return hipErrorInvalidValue;
    }
}

template <typename T, int OP, int AXIS>
static hipError_t launch_axis(const StageArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    const int n = AXIS == 2 ? a.n2 : a.n1;
#define REGNK_AX(NN)                                                                         \
    case NN:                                                                                 \
        return AXIS == 2 ? launch_row_fixed<T, NN, OP>(a, s, t0, t1) : launch_col_fixed<T, NN, OP>(a, s, t0, t1);
    switch (n) {
        REGNK_AX(8) REGNK_AX(16) REGNK_AX(32) REGNK_AX(64) REGNK_AX(128) REGNK_AX(256) REGNK_AX(512)
        REGNK_AX(1024) REGNK_AX(2048)
    }
#undef REGNK_AX
    return hipErrorInvalidValue;
}

template <typename T, int OP>
static hipError_t launch_dense_axis(int axis, const StageArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if ((axis == 2 ? a.mr2.ns : a.mr1.ns) > 0) return launch_mr_axis<T, OP>(axis, a, s, t0, t1);
    if (axis == 2) {
        if (!a.dc2) return hipErrorInvalidValue;
        launch_ks(stage_dense_row_kernel<T, OP>, dim3(a.n1 / 2), dim3(DENSE_STAGE_THREADS), a.n2 * sizeof(cpx<T>), s,
                  t0, t1, a);
    } else {
        if (!a.dc1) return hipErrorInvalidValue;
        launch_ks(stage_dense_col_kernel<T, OP>, dim3(a.n2 / 2), dim3(DENSE_STAGE_THREADS), a.n1 * sizeof(cpx<T>), s,
                  t0, t1, a);
    }
    return hipGetLastError();
}

constexpr bool is_pow2_len(int n) { return (n & (n - 1)) == 0; }

template <typename T, int OP>
hipError_t launch_stage_op(int var, const StageArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if (a.n1 == a.n2 && !is_pow2_len(a.n1) && a.mr1.ns > 0 && a.mr2.ns > 0) {
        if (a.clk) {   // timing slots: both parts' blocks of the one launch
            const MrShape r = mr_shape<T>(a.n1, false), c = mr_shape<T>(a.n1, true);
            if ((a.n1 / 2 + r.per_block - 1) / r.per_block + (a.n2 / 2 + c.per_block - 1) / c.per_block >
                (a.n1 + a.n2) / 2)
                return hipErrorInvalidValue;
        }
        return launch_mr_fused<T, OP>(a, s, t0, t1);
    }
    if (a.n1 == a.n2 && is_pow2_len(a.n1)) {
        switch (a.n1) {
            case 8: return launch_square<T, 8, OP>(var, a, s, t0, t1);
            case 16: return launch_square<T, 16, OP>(var, a, s, t0, t1);
            case 32: return launch_square<T, 32, OP>(var, a, s, t0, t1);
            case 64: return launch_square<T, 64, OP>(var, a, s, t0, t1);
            case 128: return launch_square<T, 128, OP>(var, a, s, t0, t1);
            case 256: return launch_square<T, 256, OP>(var, a, s, t0, t1);
            case 512: return launch_square<T, 512, OP>(var, a, s, t0, t1);
            case 1024: return launch_square<T, 1024, OP>(var, a, s, t0, t1);
            case 2048: return launch_square<T, 2048, OP>(var, a, s, t0, t1);
        }
        return hipErrorInvalidValue;
    }
    // independent parts: two launches in stream order (a timed stage spans both; timing slots of the
    // column launch follow the at most n1/2 row blocks)
    hipError_t e = is_pow2_len(a.n2) ? launch_axis<T, OP, 2>(a, s, t0, nullptr)
                                     : launch_dense_axis<T, OP>(2, a, s, t0, nullptr);
    if (e != hipSuccess) return e;
    StageArgs<T> ac = a;
    if (ac.clk) ac.clk += ((a.flags & F_PHASES) ? 4 : 2) * (a.n1 / 2);
    return is_pow2_len(a.n1) ? launch_axis<T, OP, 1>(ac, s, nullptr, t1) : launch_dense_axis<T, OP>(1, ac, s, nullptr, t1);
}

}  // namespace regnk
