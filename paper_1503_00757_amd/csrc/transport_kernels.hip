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
#include "device_common.hpp"
#include "kernels.hpp"

namespace regnk {

// ---------------------------------------------------------------------------------------------
// Per-op value to differentiate and epilogue.  `idx` is the linear index i1*n2 + i2, d the
// derivative.  uu / vv are the loaded U and V values (kept in registers for the epilogue).
// ---------------------------------------------------------------------------------------------
template <typename T, int OP>
__device__ __forceinline__ T pass_value(const PassArgs<T>& a, long idx, T& uu, T& vv) {
    const long nn = a.nn;
    if constexpr (OP == OP_I2) {
        if (a.flags & F_ZERO) {   // m~*_0 = -h v~ . G_0 (m~_0 = 0)
            uu = -a.h * (a.VT[idx] * a.G2[idx] + a.VT[nn + idx] * a.G2[nn + idx]);
        } else {
            uu = a.U[idx];
        }
    } else {
        uu = a.U[idx];
    }
    if constexpr (OP == OP_A1 || OP == OP_A2) {
        vv = a.V[idx];
        return vv * uu;
    } else {
        return uu;
    }
}

// AXIS: 2 = row pass (d = d2, V = v2), 1 = column pass (d = d1, V = v1)
template <typename T, int OP, int AXIS>
__device__ __forceinline__ void pass_epilogue(const PassArgs<T>& a, long idx, T d, T uu, T vv) {
    const long nn = a.nn;
    const T h = a.h;
    const T hh = T(0.5) * a.h;
    const int gcomp = (AXIS == 2) ? 1 : 0;   // which gradient component this axis produces
    if constexpr (OP == OP_S1) {
        if (a.GOUT) a.GOUT[gcomp * nn + idx] = d;
        if (a.GOUTF) a.GOUTF[gcomp * nn + idx] = (float)d;
        const T v = a.V[idx];
        if constexpr (AXIS == 2) a.OUT[idx] = uu - h * v * d;          // P = m_j - h v2 d2 m_j
        else a.OUT[idx] = a.X[idx] - h * v * d;                        // m* = P - h v1 d1 m_j
    } else if constexpr (OP == OP_S2) {
        if (a.GOUT) a.GOUT[gcomp * nn + idx] = d;
        if (a.GOUTF) a.GOUTF[gcomp * nn + idx] = (float)d;
        const T v = a.V[idx];
        if constexpr (AXIS == 2) {
            a.OUT[idx] = T(0.5) * (a.X[idx] + uu) - hh * v * d;      // Q
        } else {
            const T o = a.X[idx] - hh * v * d;                         // m_{j+1}
            a.OUT[idx] = o;
            if (a.OUT2) a.OUT2[idx] = a.MR[idx] - o;                   // lam(1) = m_R - m_1
            if (a.OUT2F) a.OUT2F[idx] = (float)(a.MR[idx] - o);
        }
    } else if constexpr (OP == OP_A1) {
        if constexpr (AXIS == 2) {
            a.OUT[idx] = uu + h * d;                                   // P = l + h d2(v2 l)
            if (a.B) {                                                 // trapezoid: w_{j+1} h l_{j+1} G_{j+1}
                const T w = a.bw * uu;
                if (a.flags & F_FIRST) {
                    a.B[idx] = w * a.G[idx];
                    a.B[nn + idx] = w * a.G[nn + idx];
                } else {
                    a.B[idx] += w * a.G[idx];
                    a.B[nn + idx] += w * a.G[nn + idx];
                }
            }
        } else {
            a.OUT[idx] = a.X[idx] + h * d;                             // l* = P + h d1(v1 l)
        }
    } else if constexpr (OP == OP_A2) {
        if constexpr (AXIS == 2) {
            const T lo = a.X[idx];                                     // l_{j+1}
            a.OUT[idx] = T(0.5) * (lo + uu) + hh * d;                  // Q
            if (a.B) {                                                 // (h/2)(l*_j G_j + l_{j+1} G*_j)
                const T b0 = a.bw * (uu * a.G[idx] + lo * a.G2[idx]);
                const T b1 = a.bw * (uu * a.G[nn + idx] + lo * a.G2[nn + idx]);
                if (a.flags & F_FIRST) {
                    a.B[idx] = b0;
                    a.B[nn + idx] = b1;
                } else {
                    a.B[idx] += b0;
                    a.B[nn + idx] += b1;
                }
            }
        } else {
            a.OUT[idx] = a.X[idx] + hh * d;                            // l_j = Q + (h/2) d1(v1 l*)
        }
    } else if constexpr (OP == OP_I1) {
        const T v = a.V[idx];
        if constexpr (AXIS == 2) {
            const T s = a.VT[idx] * a.G[idx] + a.VT[nn + idx] * a.G[nn + idx];
            a.OUT[idx] = uu - h * (v * d + s);                         // P = m~ - h(v2 d2 m~ + v~.G_j)
        } else {
            a.OUT[idx] = a.X[idx] - h * v * d;                         // m~* = P - h v1 d1 m~
        }
    } else if constexpr (OP == OP_I2) {
        const T v = a.V[idx];
        if constexpr (AXIS == 2) {
            const T s = a.VT[idx] * a.G[idx] + a.VT[nn + idx] * a.G[nn + idx];
            const T mj = (a.flags & F_ZERO) ? T(0) : a.X[idx];
            a.OUT[idx] = T(0.5) * (mj + uu) - hh * (v * d + s);        // Q
        } else {
            const T o = a.X[idx] - hh * v * d;                         // m~_{j+1}
            a.OUT[idx] = (a.flags & F_NEG) ? -o : o;                   // lam~(1) = -m~(1)
        }
    } else if constexpr (OP == OP_GRAD) {
        if (a.GOUT) a.GOUT[gcomp * nn + idx] = d;
        if (a.GOUTF) a.GOUTF[gcomp * nn + idx] = (float)d;
    }
}

// ---------------------------------------------------------------------------------------------
// Row pass: FPW transforms per block, each transform = one pair of rows (2r, 2r+1), length N = n2.
// ---------------------------------------------------------------------------------------------
template <typename T, int N, int FPW, int OP>
__global__ __launch_bounds__(FPW * N / 4) void row_pass_kernel(PassArgs<T> a) {
    constexpr int Q = N / 4;
    constexpr int L = LdsSize<N>::value;
    __shared__ cpx<T> lds[FPW][2][L];
    const int f = threadIdx.x / Q, t = threadIdx.x % Q;
    const int pair = blockIdx.x * FPW + f;
    const bool valid = pair < (a.n1 >> 1);
    const long row0 = (long)(valid ? 2 * pair : 0) * N;
    const long row1 = row0 + N;
    cpx<T> x[4];
    T u0[4], u1[4], w0[4], w1[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = t + r * Q;
        T p0 = 0, p1 = 0;
        if (valid) {
            p0 = pass_value<T, OP>(a, row0 + e, u0[r], w0[r]);
            p1 = pass_value<T, OP>(a, row1 + e, u1[r], w1[r]);
        }
        x[r] = {p0, p1};
    }
    int buf = 0;
    fft4<T, N, false>(x, lds[f][0], lds[f][1], t, a.tw, buf);
    const T inv = T(1) / T(N);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const T k = T(kwave<N>(t + r * Q)) * inv;
        x[r] = {-x[r].y * k, x[r].x * k};   // times i k / N
    }
    fft4<T, N, true>(x, lds[f][0], lds[f][1], t, a.tw, buf);
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = t + r * Q;
        pass_epilogue<T, OP, 2>(a, row0 + e, x[r].x, u0[r], w0[r]);
        pass_epilogue<T, OP, 2>(a, row1 + e, x[r].y, u1[r], w1[r]);
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

template <typename T, int N, int NF, int OP>
__global__ __launch_bounds__(NF * N / 4) void col_pass_kernel(PassArgs<T> a) {
    constexpr int Q = N / 4;
    constexpr int L = LdsSize<N>::value;
    __shared__ cpx<T> lds[NF][2][L];
    const int f = threadIdx.x % NF, t = threadIdx.x / NF;
    constexpr int TWB = 2 * NF * (int)sizeof(T);
    constexpr int GROUP = TWB >= 128 ? 1 : 128 / TWB;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, GROUP);
    const int c = tile * 2 * NF + 2 * f;
    const bool valid = c < a.n2;
    const long n2 = a.n2;
    cpx<T> x[4];
    T u0[4], u1[4], w0[4], w1[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const long idx = (long)(t + r * Q) * n2 + (valid ? c : 0);
        T p0 = 0, p1 = 0;
        if (valid) {
            p0 = pass_value<T, OP>(a, idx, u0[r], w0[r]);
            p1 = pass_value<T, OP>(a, idx + 1, u1[r], w1[r]);
        }
        x[r] = {p0, p1};
    }
    int buf = 0;
    fft4<T, N, false>(x, lds[f][0], lds[f][1], t, a.tw, buf);
    const T inv = T(1) / T(N);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const T k = T(kwave<N>(t + r * Q)) * inv;
        x[r] = {-x[r].y * k, x[r].x * k};
    }
    fft4<T, N, true>(x, lds[f][0], lds[f][1], t, a.tw, buf);
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const long idx = (long)(t + r * Q) * n2 + c;
        pass_epilogue<T, OP, 1>(a, idx, x[r].x, u0[r], w0[r]);
        pass_epilogue<T, OP, 1>(a, idx + 1, x[r].y, u1[r], w1[r]);
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
// Launch geometry and dispatch
// ---------------------------------------------------------------------------------------------
template <int N>
constexpr int row_fpw() { return (N / 4) >= 64 ? 1 : 64 / (N / 4); }
template <int N>
constexpr int col_nf() { return (N / 4) >= 64 ? 2 : (64 / (N / 4) < 2 ? 2 : 64 / (N / 4)); }

template <typename T, int N, int OP>
static hipError_t launch_row_n(const PassArgs<T>& a, hipStream_t s) {
    constexpr int FPW = row_fpw<N>();
    const int pairs = a.n1 / 2;
    const int blocks = (pairs + FPW - 1) / FPW;
    hipLaunchKernelGGL((row_pass_kernel<T, N, FPW, OP>), dim3(blocks), dim3(FPW * N / 4), 0, s, a);
    return hipGetLastError();
}

template <typename T, int N, int OP>
static hipError_t launch_col_n(const PassArgs<T>& a, hipStream_t s) {
    constexpr int NF = col_nf<N>();
    const int tiles = (a.n2 + 2 * NF - 1) / (2 * NF);
    hipLaunchKernelGGL((col_pass_kernel<T, N, NF, OP>), dim3(tiles), dim3(NF * N / 4), 0, s, a);
    return hipGetLastError();
}

template <typename T, int OP>
static hipError_t launch_row_op(const PassArgs<T>& a, hipStream_t s) {
    switch (a.n2) {
        case 8: return launch_row_n<T, 8, OP>(a, s);
        case 16: return launch_row_n<T, 16, OP>(a, s);
        case 32: return launch_row_n<T, 32, OP>(a, s);
        case 64: return launch_row_n<T, 64, OP>(a, s);
        case 128: return launch_row_n<T, 128, OP>(a, s);
        case 256: return launch_row_n<T, 256, OP>(a, s);
        case 512: return launch_row_n<T, 512, OP>(a, s);
        case 1024: return launch_row_n<T, 1024, OP>(a, s);
        case 2048: return launch_row_n<T, 2048, OP>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int OP>
static hipError_t launch_col_op(const PassArgs<T>& a, hipStream_t s) {
    switch (a.n1) {
        case 8: return launch_col_n<T, 8, OP>(a, s);
        case 16: return launch_col_n<T, 16, OP>(a, s);
        case 32: return launch_col_n<T, 32, OP>(a, s);
        case 64: return launch_col_n<T, 64, OP>(a, s);
        case 128: return launch_col_n<T, 128, OP>(a, s);
        case 256: return launch_col_n<T, 256, OP>(a, s);
        case 512: return launch_col_n<T, 512, OP>(a, s);
        case 1024: return launch_col_n<T, 1024, OP>(a, s);
        case 2048: return launch_col_n<T, 2048, OP>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_pass(int op, int axis, const PassArgs<T>& a, hipStream_t s) {
    if (axis == 2) {
        switch (op) {
            case OP_S1: return launch_row_op<T, OP_S1>(a, s);
            case OP_S2: return launch_row_op<T, OP_S2>(a, s);
            case OP_A1: return launch_row_op<T, OP_A1>(a, s);
            case OP_A2: return launch_row_op<T, OP_A2>(a, s);
            case OP_I1: return launch_row_op<T, OP_I1>(a, s);
            case OP_I2: return launch_row_op<T, OP_I2>(a, s);
            case OP_GRAD: return launch_row_op<T, OP_GRAD>(a, s);
        }
    } else {
        switch (op) {
            case OP_S1: return launch_col_op<T, OP_S1>(a, s);
            case OP_S2: return launch_col_op<T, OP_S2>(a, s);
            case OP_A1: return launch_col_op<T, OP_A1>(a, s);
            case OP_A2: return launch_col_op<T, OP_A2>(a, s);
            case OP_I1: return launch_col_op<T, OP_I1>(a, s);
            case OP_I2: return launch_col_op<T, OP_I2>(a, s);
            case OP_GRAD: return launch_col_op<T, OP_GRAD>(a, s);
        }
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_body_end(long nn, T w, const T* lam, const T* G, T* B, hipStream_t s) {
    int blocks = (int)((nn + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((body_end_kernel<T>), dim3(blocks), dim3(256), 0, s, nn, w, lam, G, B);
    return hipGetLastError();
}

template hipError_t launch_pass<float>(int, int, const PassArgs<float>&, hipStream_t);
template hipError_t launch_pass<double>(int, int, const PassArgs<double>&, hipStream_t);
template hipError_t launch_body_end<float>(long, float, const float*, const float*, float*, hipStream_t);
template hipError_t launch_body_end<double>(long, double, const double*, const double*, double*, hipStream_t);

}  // namespace regnk
