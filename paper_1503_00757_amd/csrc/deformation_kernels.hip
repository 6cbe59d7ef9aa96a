// Pointwise kernels of the deformation diagnostics (appendix "Illustration of Deformation Map":
// eq. (displacement) and eq. (def-grad)).  The transport part of each Heun stage runs through the
// FP64 state-stage launches; these kernels add the sources and form det F.
#include "device_common.hpp"
#include "kernels.hpp"

namespace regnk {

// out_c += w * S_c for the six components (u_1, u_2, F_11, F_12, F_21, F_22):
//   S_{u_i} = v_i,   S_{F_ik} = dv_i0 F_0k + dv_i1 F_1k   (dv_il = d_l v_i),
// with F_lk = a[l k] (+ b[l k] when b is given: the stage value is an R + C pair).
__global__ void deform_source_kernel(long nn, double w, const double* __restrict__ v, const double* __restrict__ dv,
                                     DefPtrs p) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
        double F[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) F[c] = p.a[c][i] + (p.b[c] ? p.b[c][i] : 0.0);
        p.out[0][i] += w * v[i];
        p.out[1][i] += w * v[nn + i];
#pragma unroll
        for (int r = 0; r < 2; ++r) {          // row index i of F_ik
            const double d0 = dv[(2 * r) * nn + i], d1 = dv[(2 * r + 1) * nn + i];
#pragma unroll
            for (int k = 0; k < 2; ++k) p.out[2 + 2 * r + k][i] += w * (d0 * F[k] + d1 * F[2 + k]);
        }
    }
}

// Final values q_c = R_c + C_c of the six components; u1 (vector), F1 ([2][2] fields) nullable;
// det = F_11 F_22 - F_12 F_21.
__global__ void deform_final_kernel(long nn, DefPairs p, double* __restrict__ u1, double* __restrict__ F1,
                                    double* __restrict__ det) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
        double q[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) q[c] = p.r[c][i] + p.c[c][i];
        if (u1) {
            u1[i] = q[0];
            u1[nn + i] = q[1];
        }
        if (F1) {
#pragma unroll
            for (int c = 0; c < 4; ++c) F1[(long)c * nn + i] = q[2 + c];
        }
        det[i] = q[2] * q[5] - q[3] * q[4];
    }
}

// min, max and sum of x over n entries, deterministic (fixed per-block chunks, fixed trees).
__global__ __launch_bounds__(RED_THREADS) void minmaxsum_part_kernel(const double* __restrict__ x, long n,
                                                                    double* __restrict__ partial) {
    __shared__ double sh[3][RED_THREADS];
    const long chunk = (n + RED_BLOCKS - 1) / RED_BLOCKS;
    const long lo = (long)blockIdx.x * chunk;
    const long hi = lo + chunk < n ? lo + chunk : n;
    double mn = 1e300, mx = -1e300, s = 0.0;
    for (long i = lo + threadIdx.x; i < hi; i += RED_THREADS) {
        const double t = x[i];
        mn = fmin(mn, t);
        mx = fmax(mx, t);
        s += t;
    }
    sh[0][threadIdx.x] = mn;
    sh[1][threadIdx.x] = mx;
    sh[2][threadIdx.x] = s;
    __syncthreads();
    for (int off = RED_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + off]);
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + off]);
            sh[2][threadIdx.x] += sh[2][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = sh[0][0];
        partial[RED_BLOCKS + blockIdx.x] = sh[1][0];
        partial[2 * RED_BLOCKS + blockIdx.x] = sh[2][0];
    }
}

__global__ __launch_bounds__(RED_THREADS) void minmaxsum_final_kernel(const double* __restrict__ partial,
                                                                     double* __restrict__ out) {
    __shared__ double sh[3][RED_THREADS];
    double mn = 1e300, mx = -1e300, s = 0.0;
    for (int i = threadIdx.x; i < RED_BLOCKS; i += RED_THREADS) {
        mn = fmin(mn, partial[i]);
        mx = fmax(mx, partial[RED_BLOCKS + i]);
        s += partial[2 * RED_BLOCKS + i];
    }
    sh[0][threadIdx.x] = mn;
    sh[1][threadIdx.x] = mx;
    sh[2][threadIdx.x] = s;
    __syncthreads();
    for (int off = RED_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + off]);
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + off]);
            sh[2][threadIdx.x] += sh[2][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0][0];
        out[1] = sh[1][0];
        out[2] = sh[2][0];
    }
}

static inline int grid_for_n(long n) {
    long b = (n + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

hipError_t launch_deform_source(long nn, double w, const double* v, const double* dv, const DefPtrs& p,
                                hipStream_t s) {
    hipLaunchKernelGGL(deform_source_kernel, dim3(grid_for_n(nn)), dim3(256), 0, s, nn, w, v, dv, p);
    return hipGetLastError();
}
hipError_t launch_deform_final(long nn, const DefPairs& p, double* u1, double* F1, double* det, hipStream_t s) {
    hipLaunchKernelGGL(deform_final_kernel, dim3(grid_for_n(nn)), dim3(256), 0, s, nn, p, u1, F1, det);
    return hipGetLastError();
}
hipError_t launch_minmaxsum(const double* x, long n, double* partial, double* out3, hipStream_t s) {
    hipLaunchKernelGGL(minmaxsum_part_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, n, partial);
    hipLaunchKernelGGL(minmaxsum_final_kernel, dim3(1), dim3(RED_THREADS), 0, s, partial, out3);
    return hipGetLastError();
}

}  // namespace regnk
