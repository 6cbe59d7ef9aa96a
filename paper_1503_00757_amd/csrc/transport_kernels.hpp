// Fused transport passes: every RK2 (Heun) stage of the state, adjoint, incremental-state and
// Gauss-Newton incremental-adjoint solves is split into a row pass (derivative along x2, the
// contiguous axis) and a column pass (derivative along x1).  A spectral partial derivative only
// needs a 1D transform along its own axis, so each pass holds whole rows or whole column tiles in
// registers/LDS, applies i k~ (Nyquist -> 0) between a forward and an inverse FFT, and finishes the
// stage in its epilogue: the transport right-hand side, the Heun update, the stored gradients of the
// state and the time quadrature of the body force.
//
// Two real lines are packed into one complex transform (z = a + i b); because i k~ maps real
// sequences to real sequences, the real and imaginary parts of the result are the derivatives of a
// and b.
//
// Heun stages (h = 1/n_t), with L_v u = -(v1 d1 u + v2 d2 u), L_v^T q = d1(v1 q) + d2(v2 q):
//   state        m*_j = m_j + h L m_j,            m_{j+1} = (m_j + m*_j)/2 + (h/2) L m*_j
//   adjoint      l*_j = l_{j+1} + h L^T l_{j+1},  l_j = (l_{j+1} + l*_j)/2 + (h/2) L^T l*_j
//   inc. state   m~* = m~_j + h (L m~_j + S_j),   m~_{j+1} = (m~_j + m~*)/2 + (h/2)(L m~* + S*_j)
//                with S = -v~ . grad m (sampled at G_j, and at G*_j or G_{j+1})
// Each stage = row pass (adds the x2 part and everything pointwise) + column pass (adds the x1 part).
#pragma once
#include "device_common.hpp"
#include "kernels.hpp"

namespace regnk {

// ---------------------------------------------------------------------------------------------
// Per point: pass_load issues every global load the pass needs -- the transform input first, then
// all epilogue operands -- so that their latencies overlap each other and the FFTs; pass_store does
// the epilogue arithmetic and the stores.  idx = i1*n2 + i2; d = the derivative.
// ---------------------------------------------------------------------------------------------
template <typename T>
struct Pt {
    T u, v, x, g0, g1, h0, h1, b0, b1, mr;
};

template <typename T, int OP, int AXIS>
__device__ __forceinline__ T pass_load(const PassArgs<T>& a, long idx, Pt<T>& p) {
    const long nn = a.nn;
    if constexpr (OP == OP_I2) {
        if (a.flags & F_ZERO) {   // m~*_0 = -h v~ . G_0 (m~_0 = 0)
            p.u = -a.h * (a.VT[idx] * a.G2[idx] + a.VT[nn + idx] * a.G2[nn + idx]);
        } else {
            p.u = a.U[idx];
        }
    } else {
        p.u = a.U[idx];
    }
    if constexpr (OP != OP_GRAD) p.v = a.V[idx];
    const T val = (OP == OP_A1 || OP == OP_A2) ? p.v * p.u : p.u;
    if constexpr (AXIS == 1) {
        if constexpr (OP != OP_GRAD) p.x = a.X[idx];
        if constexpr (OP == OP_S2) {
            if (a.OUT2 || a.OUT2F) p.mr = a.MR[idx];
        }
    } else {
        if constexpr (OP == OP_S2 || OP == OP_A2) p.x = a.X[idx];
        if constexpr (OP == OP_I2) p.x = (a.flags & F_ZERO) ? T(0) : a.X[idx];
        if constexpr (OP == OP_I1 || OP == OP_I2) {
            p.g0 = a.VT[idx];
            p.g1 = a.VT[nn + idx];
            p.h0 = a.G[idx];
            p.h1 = a.G[nn + idx];
        }
        if constexpr (OP == OP_A1 || OP == OP_A2) {
            if (a.B) {
                p.g0 = a.G[idx];
                p.g1 = a.G[nn + idx];
                if constexpr (OP == OP_A2) {
                    p.h0 = a.G2[idx];
                    p.h1 = a.G2[nn + idx];
                }
                if (!(a.flags & F_FIRST)) {
                    p.b0 = a.B[idx];
                    p.b1 = a.B[nn + idx];
                } else {
                    p.b0 = T(0);
                    p.b1 = T(0);
                }
            }
        }
    }
    return val;
}

// AXIS: 2 = row pass (d = d2, V = v2), 1 = column pass (d = d1, V = v1)
template <typename T, int OP, int AXIS>
__device__ __forceinline__ void pass_store(const PassArgs<T>& a, long idx, T d, const Pt<T>& p) {
    const long nn = a.nn;
    const T h = a.h;
    const T hh = T(0.5) * a.h;
    const int gcomp = (AXIS == 2) ? 1 : 0;   // which gradient component this axis produces
    if constexpr (OP == OP_S1 || OP == OP_S2 || OP == OP_GRAD) {
        if (a.GOUT) a.GOUT[gcomp * nn + idx] = d;
        if (a.GOUTF) a.GOUTF[gcomp * nn + idx] = (float)d;
    }
    if constexpr (OP == OP_S1) {
        if constexpr (AXIS == 2) a.OUT[idx] = p.u - h * p.v * d;         // P = m_j - h v2 d2 m_j
        else a.OUT[idx] = p.x - h * p.v * d;                             // m* = P - h v1 d1 m_j
    } else if constexpr (OP == OP_S2) {
        if constexpr (AXIS == 2) {
            a.OUT[idx] = T(0.5) * (p.x + p.u) - hh * p.v * d;           // Q
        } else {
            const T o = p.x - hh * p.v * d;                              // m_{j+1}
            a.OUT[idx] = o;
            if (a.OUT2) a.OUT2[idx] = p.mr - o;                          // lam(1) = m_R - m_1
            if (a.OUT2F) a.OUT2F[idx] = (float)(p.mr - o);
        }
    } else if constexpr (OP == OP_A1) {
        if constexpr (AXIS == 2) {
            a.OUT[idx] = p.u + h * d;                                    // P = l + h d2(v2 l)
            if (a.B) {                                                   // trapezoid: w_{j+1} h l_{j+1} G_{j+1}
                const T w = a.bw * p.u;
                a.B[idx] = p.b0 + w * p.g0;
                a.B[nn + idx] = p.b1 + w * p.g1;
            }
        } else {
            a.OUT[idx] = p.x + h * d;                                    // l* = P + h d1(v1 l)
        }
    } else if constexpr (OP == OP_A2) {
        if constexpr (AXIS == 2) {
            a.OUT[idx] = T(0.5) * (p.x + p.u) + hh * d;                  // Q  (x = l_{j+1}, u = l*_j)
            if (a.B) {                                                   // (h/2)(l*_j G_j + l_{j+1} G*_j)
                a.B[idx] = p.b0 + a.bw * (p.u * p.g0 + p.x * p.h0);
                a.B[nn + idx] = p.b1 + a.bw * (p.u * p.g1 + p.x * p.h1);
            }
        } else {
            a.OUT[idx] = p.x + hh * d;                                   // l_j = Q + (h/2) d1(v1 l*)
        }
    } else if constexpr (OP == OP_I1) {
        if constexpr (AXIS == 2) {
            const T s = p.g0 * p.h0 + p.g1 * p.h1;                       // v~ . G_j
            a.OUT[idx] = p.u - h * (p.v * d + s);                        // P = m~ - h(v2 d2 m~ + v~.G_j)
        } else {
            a.OUT[idx] = p.x - h * p.v * d;                              // m~* = P - h v1 d1 m~
        }
    } else if constexpr (OP == OP_I2) {
        if constexpr (AXIS == 2) {
            const T s = p.g0 * p.h0 + p.g1 * p.h1;
            a.OUT[idx] = T(0.5) * (p.x + p.u) - hh * (p.v * d + s);      // Q
        } else {
            const T o = p.x - hh * p.v * d;                              // m~_{j+1}
            a.OUT[idx] = (a.flags & F_NEG) ? -o : o;                     // lam~(1) = -m~(1)
        }
    }
}


// ---------------------------------------------------------------------------------------------
// Row pass: FPW transforms per block, each transform = one pair of rows (2r, 2r+1), length N = n2.
// ---------------------------------------------------------------------------------------------
template <typename T, int N, int E, int FPW, int OP>
__global__ __launch_bounds__(FPW * N / E) void row_pass_kernel(PassArgs<T> a) {
    constexpr int TT = N / E;
    constexpr int L = LdsSize<N>::value;
    __shared__ cpx<T> lds[FPW][2][L];
    const int f = threadIdx.x / TT, t = threadIdx.x % TT;
    const int pair = blockIdx.x * FPW + f;
    const bool valid = pair < (a.n1 >> 1);
    const long row0 = (long)(valid ? 2 * pair : 0) * N;
    const long row1 = row0 + N;
    cpx<T> x[E];
    Pt<T> q0[E], q1[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = t + TT * m;
        T p0 = 0, p1 = 0;
        if (valid) {
            p0 = pass_load<T, OP, 2>(a, row0 + e, q0[m]);
            p1 = pass_load<T, OP, 2>(a, row1 + e, q1[m]);
        }
        x[m] = {p0, p1};
    }
    int buf = 0;
    fftE<T, N, E, false>(x, lds[f][0], lds[f][1], t, a.tw, buf);
    const T inv = T(1) / T(N);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const T k = T(kwave<N>(t + TT * m)) * inv;
        x[m] = {-x[m].y * k, x[m].x * k};   // times i k / N
    }
    fftE<T, N, E, true>(x, lds[f][0], lds[f][1], t, a.tw, buf);
    if (!valid) return;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = t + TT * m;
        pass_store<T, OP, 2>(a, row0 + e, x[m].x, q0[m]);
        pass_store<T, OP, 2>(a, row1 + e, x[m].y, q1[m]);
    }
}

// ---------------------------------------------------------------------------------------------
// Column pass: a block owns TW = 2*NF adjacent columns (NF transforms of length N = n1, column
// pairs packed as complex).  Consecutive threads take consecutive column pairs of the same row so
// that a wave reads contiguous row segments.  Column tiles are spread over the eight XCDs so that
// the tiles sharing a 128-byte line run on the same XCD (same L2).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int b, int nb, int group) {
    // blocks are dispatched round-robin over 8 XCDs: block b runs on XCD b % 8.
    if (group <= 1 || (nb % (8 * group)) != 0) return b;
    const int x = b & 7, l = b >> 3;
    return group * (x + 8 * (l / group)) + (l % group);
}

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

// Column-pass versions of pass_load / pass_store for the column pair (c, c+1).
template <typename T, int OP>
__device__ __forceinline__ cpx<T> col_load2(const PassArgs<T>& a, long idx, Pt<T>& p0, Pt<T>& p1) {
    const long nn = a.nn;
    if constexpr (OP == OP_I2) {
        if (a.flags & F_ZERO) {   // m~*_0 = -h v~ . G_0
            T va0, vb0, va1, vb1, ga0, gb0, ga1, gb1;
            ld2(a.VT, idx, va0, vb0);
            ld2(a.VT, nn + idx, va1, vb1);
            ld2(a.G2, idx, ga0, gb0);
            ld2(a.G2, nn + idx, ga1, gb1);
            p0.u = -a.h * (va0 * ga0 + va1 * ga1);
            p1.u = -a.h * (vb0 * gb0 + vb1 * gb1);
        } else {
            ld2(a.U, idx, p0.u, p1.u);
        }
    } else {
        ld2(a.U, idx, p0.u, p1.u);
    }
    if constexpr (OP != OP_GRAD) ld2(a.V, idx, p0.v, p1.v);
    const cpx<T> val = (OP == OP_A1 || OP == OP_A2) ? cpx<T>{p0.v * p0.u, p1.v * p1.u} : cpx<T>{p0.u, p1.u};
    if constexpr (OP != OP_GRAD) ld2(a.X, idx, p0.x, p1.x);
    if constexpr (OP == OP_S2) {
        if (a.OUT2 || a.OUT2F) ld2(a.MR, idx, p0.mr, p1.mr);
    }
    return val;
}

template <typename T, int OP>
__device__ __forceinline__ void col_store2(const PassArgs<T>& a, long idx, T d0, T d1, const Pt<T>& p0,
                                           const Pt<T>& p1) {
    const T h = a.h;
    const T hh = T(0.5) * a.h;
    if constexpr (OP == OP_S1 || OP == OP_S2 || OP == OP_GRAD) {
        if (a.GOUT) st2(a.GOUT, idx, d0, d1);
        if (a.GOUTF) st2(a.GOUTF, idx, (float)d0, (float)d1);
    }
    if constexpr (OP == OP_S1 || OP == OP_I1) {
        st2(a.OUT, idx, p0.x - h * p0.v * d0, p1.x - h * p1.v * d1);      // m* / m~* = P - h v1 d1 u
    } else if constexpr (OP == OP_S2) {
        const T o0 = p0.x - hh * p0.v * d0, o1 = p1.x - hh * p1.v * d1;   // m_{j+1}
        st2(a.OUT, idx, o0, o1);
        if (a.OUT2) st2(a.OUT2, idx, p0.mr - o0, p1.mr - o1);             // lam(1) = m_R - m_1
        if (a.OUT2F) st2(a.OUT2F, idx, (float)(p0.mr - o0), (float)(p1.mr - o1));
    } else if constexpr (OP == OP_A1) {
        st2(a.OUT, idx, p0.x + h * d0, p1.x + h * d1);                    // l* = P + h d1(v1 l)
    } else if constexpr (OP == OP_A2) {
        st2(a.OUT, idx, p0.x + hh * d0, p1.x + hh * d1);                  // l_j = Q + (h/2) d1(v1 l*)
    } else if constexpr (OP == OP_I2) {
        T o0 = p0.x - hh * p0.v * d0, o1 = p1.x - hh * p1.v * d1;         // m~_{j+1}
        if (a.flags & F_NEG) {                                            // lam~(1) = -m~(1)
            o0 = -o0;
            o1 = -o1;
        }
        st2(a.OUT, idx, o0, o1);
    }
}

template <typename T, int N, int E, int NF, int OP>
__global__ __launch_bounds__(NF * N / E) void col_pass_kernel(PassArgs<T> a) {
    constexpr int TT = N / E;
    constexpr int L = LdsSize<N>::value;
    __shared__ cpx<T> lds[NF][2][L];
    const int f = threadIdx.x % NF, t = threadIdx.x / NF;
    constexpr int TWB = 2 * NF * (int)sizeof(T);
    constexpr int GROUP = TWB >= 128 ? 1 : 128 / TWB;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, GROUP);
    const int c = tile * 2 * NF + 2 * f;
    const bool valid = c < a.n2;
    const long n2 = a.n2;
    cpx<T> x[E];
    Pt<T> q0[E], q1[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const long idx = (long)(t + TT * m) * n2 + (valid ? c : 0);
        x[m] = valid ? col_load2<T, OP>(a, idx, q0[m], q1[m]) : cpx<T>{T(0), T(0)};
    }
    int buf = 0;
    fftE<T, N, E, false>(x, lds[f][0], lds[f][1], t, a.tw, buf);
    const T inv = T(1) / T(N);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const T k = T(kwave<N>(t + TT * m)) * inv;
        x[m] = {-x[m].y * k, x[m].x * k};
    }
    fftE<T, N, E, true>(x, lds[f][0], lds[f][1], t, a.tw, buf);
    if (!valid) return;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const long idx = (long)(t + TT * m) * n2 + c;
        col_store2<T, OP>(a, idx, x[m].x, x[m].y, q0[m], q1[m]);
    }
}

// Trapezoid end point b += w l_0 G_0 (paper quadrature), vector accumulate.
template <typename T>
__global__ void body_end_kernel(long nn, T w, const T* __restrict__ lam, const T* __restrict__ G,
                                T* __restrict__ B) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < nn; i += (long)gridDim.x * blockDim.x) {
        const T l = w * lam[i];
        B[i] += l * G[i];
        B[nn + i] += l * G[nn + i];
    }
}

// ---------------------------------------------------------------------------------------------
// Launch variants: (elements per thread E, transforms per block G).  G = 0 means "enough
// transforms for 64 threads".  Variant 0 of each axis is the default; an autotuner may pick another.
// ---------------------------------------------------------------------------------------------
// rows: (8, auto), (4, auto), (16, auto), (8, 2); columns: (16, 2), (16, 1), (16, 4), (8, 1), (8, 2),
// (8, 4), (4, 2)
constexpr int row_var_E(int v) { return v == 1 ? 4 : (v == 2 ? 16 : 8); }
constexpr int row_var_G(int v) { return v == 3 ? 2 : 0; }
constexpr int col_var_E(int v) { return v <= 2 ? 16 : (v <= 5 ? 8 : 4); }
constexpr int col_var_G(int v) { return v == 1 || v == 3 ? 1 : ((v == 2 || v == 5) ? 4 : 2); }

template <int N, int E, int G>
constexpr int resolve_g() {
    return G > 0 ? G : ((N / E) >= 64 || (N / E) == 0 ? 1 : 64 / (N / E));
}
template <typename T, int N, int E, int G>
constexpr bool variant_ok() {
    return E <= N / 2 && resolve_g<N, E, G>() * (N / E) <= 1024 &&
           resolve_g<N, E, G>() * 2 * LdsSize<N>::value * 2 * (int)sizeof(T) <= 160 * 1024;
}

template <typename T, int N, int OP, int V>
static hipError_t launch_row_v(const PassArgs<T>& a, hipStream_t s) {
    constexpr int E = row_var_E(V);
    constexpr int G = resolve_g<N, E, row_var_G(V)>();
    if constexpr (variant_ok<T, N, E, G>()) {
        const int pairs = a.n1 / 2;
        hipLaunchKernelGGL((row_pass_kernel<T, N, E, G, OP>), dim3((pairs + G - 1) / G), dim3(G * N / E), 0, s, a);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T, int N, int OP, int V>
static hipError_t launch_col_v(const PassArgs<T>& a, hipStream_t s) {
    constexpr int E = col_var_E(V);
    constexpr int G = resolve_g<N, E, col_var_G(V)>();
    if constexpr (variant_ok<T, N, E, G>()) {
        const int tiles = (a.n2 + 2 * G - 1) / (2 * G);
        hipLaunchKernelGGL((col_pass_kernel<T, N, E, G, OP>), dim3(tiles), dim3(G * N / E), 0, s, a);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

// FP64 passes (state solve) and short FP32 axes (< 64 points) use one fixed shape per axis.
template <typename T, int N, int AXIS>
constexpr int fixed_E() {
    return sizeof(T) == 8 ? (AXIS == 2 ? 4 : (N >= 16 ? 8 : 4)) : (N >= 32 ? 8 : 4);
}

template <typename T, int N, int OP>
static hipError_t launch_fixed(int axis, const PassArgs<T>& a, hipStream_t s) {
    if (axis == 2) {
        constexpr int E = fixed_E<T, N, 2>(), G = resolve_g<N, E, 0>();
        hipLaunchKernelGGL((row_pass_kernel<T, N, E, G, OP>), dim3((a.n1 / 2 + G - 1) / G), dim3(G * N / E), 0, s, a);
    } else {
        constexpr int E = fixed_E<T, N, 1>(), G0 = resolve_g<N, E, 0>(), G = G0 < 2 ? 2 : G0;
        hipLaunchKernelGGL((col_pass_kernel<T, N, E, G, OP>), dim3((a.n2 + 2 * G - 1) / (2 * G)), dim3(G * N / E), 0, s, a);
    }
    return hipGetLastError();
}

template <typename T, int N, int OP>
static hipError_t launch_n(int axis, int var, const PassArgs<T>& a, hipStream_t s) {
    if constexpr (sizeof(T) == 8 || N < 64) {
        (void)var;
        return launch_fixed<T, N, OP>(axis, a, s);
    } else {
        if (axis == 2) {
            switch (var) {
                case 0: return launch_row_v<T, N, OP, 0>(a, s);
                case 1: return launch_row_v<T, N, OP, 1>(a, s);
                case 2: return launch_row_v<T, N, OP, 2>(a, s);
                case 3: return launch_row_v<T, N, OP, 3>(a, s);
            }
        } else {
            switch (var) {
                case 0: return launch_col_v<T, N, OP, 0>(a, s);
                case 1: return launch_col_v<T, N, OP, 1>(a, s);
                case 2: return launch_col_v<T, N, OP, 2>(a, s);
                case 3: return launch_col_v<T, N, OP, 3>(a, s);
                case 4: return launch_col_v<T, N, OP, 4>(a, s);
                case 5: return launch_col_v<T, N, OP, 5>(a, s);
                case 6: return launch_col_v<T, N, OP, 6>(a, s);
            }
        }
        return hipErrorInvalidValue;
    }
}

template <typename T, int OP>
hipError_t launch_pass_op(int axis, int var, const PassArgs<T>& a, hipStream_t s) {
    const int n = axis == 2 ? a.n2 : a.n1;
    switch (n) {
        case 8: return launch_n<T, 8, OP>(axis, 0, a, s);
        case 16: return launch_n<T, 16, OP>(axis, 0, a, s);
        case 32: return launch_n<T, 32, OP>(axis, 0, a, s);
        case 64: return launch_n<T, 64, OP>(axis, var, a, s);
        case 128: return launch_n<T, 128, OP>(axis, var, a, s);
        case 256: return launch_n<T, 256, OP>(axis, var, a, s);
        case 512: return launch_n<T, 512, OP>(axis, var, a, s);
        case 1024: return launch_n<T, 1024, OP>(axis, var, a, s);
        case 2048: return launch_n<T, 2048, OP>(axis, var, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace regnk
