// FP64 inner products, norms and vector updates for PCG (Alg. 2) and the line search (Alg. 1).
// Reductions are deterministic: block b always sums the same contiguous chunk in the same order
// (fixed shuffle tree inside a wave, fixed order over waves), and one block sums the per-block
// partials in a fixed order, so two runs give bitwise identical results.
#include "device_common.hpp"
#include "kernels.hpp"

namespace regnk {

template <typename TI>
struct DotPtrs {
    const TI* a[4];
    const TI* b[4];
};

template <typename TI>
__global__ __launch_bounds__(RED_THREADS) void dots_kernel(int nk, DotPtrs<TI> p, long n, double* __restrict__ partial) {
    __shared__ double sh[RED_THREADS / 64];
    const long chunk = (n + RED_BLOCKS - 1) / RED_BLOCKS;
    const long lo = (long)blockIdx.x * chunk;
    const long hi = lo + chunk < n ? lo + chunk : n;
    for (int k = 0; k < nk; ++k) {
        double acc = 0.0;
        const TI* __restrict__ a = p.a[k];
        const TI* __restrict__ b = p.b[k];
        for (long i = lo + threadIdx.x; i < hi; i += RED_THREADS) acc += (double)a[i] * (double)b[i];
        const double s = block_sum<RED_THREADS>(acc, sh);
        if (threadIdx.x == 0) partial[k * RED_BLOCKS + blockIdx.x] = s;
    }
}

template <typename TI>
__global__ __launch_bounds__(RED_THREADS) void sqdiff_kernel(const TI* __restrict__ x, const TI* __restrict__ y, long n,
                                                             double* __restrict__ partial) {
    __shared__ double sh[RED_THREADS / 64];
    const long chunk = (n + RED_BLOCKS - 1) / RED_BLOCKS;
    const long lo = (long)blockIdx.x * chunk;
    const long hi = lo + chunk < n ? lo + chunk : n;
    double acc = 0.0;
    for (long i = lo + threadIdx.x; i < hi; i += RED_THREADS) {
        const double d = (double)x[i] - (double)y[i];
        acc += d * d;
    }
    const double s = block_sum<RED_THREADS>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = 0.5 * s;
}

__global__ __launch_bounds__(RED_THREADS) void finalize_kernel(const double* __restrict__ partial, double* __restrict__ out) {
    __shared__ double sh[RED_THREADS / 64];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < RED_BLOCKS; i += RED_THREADS) acc += partial[k * RED_BLOCKS + i];
    const double s = block_sum<RED_THREADS>(acc, sh);
    if (threadIdx.x == 0) out[k] = s;
}

__global__ void axpby_kernel(long n, double alpha, const double* __restrict__ x, double beta, double* __restrict__ y) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = alpha * x[i] + beta * y[i];
}

__global__ void add_scaled_kernel(long n, const double* x, double alpha, const double* __restrict__ y, double* z) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        z[i] = x[i] + alpha * y[i];
}

template <typename TO>
__global__ void convert_kernel(long n, const double* __restrict__ in, TO* __restrict__ out) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = (TO)in[i];
}

template <typename TI>
__global__ void widen_kernel(long n, const TI* __restrict__ in, double* __restrict__ out) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}

__global__ void fill_kernel(long n, double v, double* __restrict__ y) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = v;
}

static inline int grid_for(long n) {
    long b = (n + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

template <typename TI>
hipError_t launch_dots(int nk, const TI* const* a, const TI* const* b, long n, double* partial, double* out,
                       hipStream_t s) {
    if (nk < 1 || nk > 4) return hipErrorInvalidValue;
    DotPtrs<TI> p{};
    for (int k = 0; k < nk; ++k) {
        p.a[k] = a[k];
        p.b[k] = b[k];
    }
    hipLaunchKernelGGL((dots_kernel<TI>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, nk, p, n, partial);
    hipLaunchKernelGGL(finalize_kernel, dim3(nk), dim3(RED_THREADS), 0, s, partial, out);
    return hipGetLastError();
}

template <typename TI>
hipError_t launch_sqdiff(const TI* x, const TI* y, long n, double* partial, double* out, hipStream_t s) {
    hipLaunchKernelGGL((sqdiff_kernel<TI>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, y, n, partial);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(RED_THREADS), 0, s, partial, out);
    return hipGetLastError();
}

hipError_t launch_axpby(long n, double alpha, const double* x, double beta, double* y, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, alpha, x, beta, y);
    return hipGetLastError();
}

hipError_t launch_add_scaled(long n, const double* x, double alpha, const double* y, double* z, hipStream_t s) {
    hipLaunchKernelGGL(add_scaled_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, x, alpha, y, z);
    return hipGetLastError();
}

template <typename TO>
hipError_t launch_convert(long n, const double* in, TO* out, hipStream_t s) {
    hipLaunchKernelGGL((convert_kernel<TO>), dim3(grid_for(n)), dim3(256), 0, s, n, in, out);
    return hipGetLastError();
}

template <typename TI>
hipError_t launch_widen(long n, const TI* in, double* out, hipStream_t s) {
    hipLaunchKernelGGL((widen_kernel<TI>), dim3(grid_for(n)), dim3(256), 0, s, n, in, out);
    return hipGetLastError();
}

hipError_t launch_fill(long n, double v, double* y, hipStream_t s) {
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, v, y);
    return hipGetLastError();
}

// The scalar recurrences of PCG (one thread).  sc is read after the caller stored fresh sums into
// it, so no pointer here is declared non-aliasing.
__device__ __forceinline__ void pcg_scalar_step(int mode, double* sc) {
    if (mode == PCG_INIT) {
        sc[S_ACTIVE] = 1.0;
        sc[S_BREAK] = 0.0;
        sc[S_ITER] = 0.0;
        sc[S_RR] = sc[S_RR0];
        sc[S_KAPPA] = 0.0;
        sc[S_MU] = 0.0;
    } else if (mode == PCG_KAPPA) {
        const double shs = sc[S_SHS];
        double kappa = 0.0;
        if (sc[S_ACTIVE] != 0.0) {
            sc[S_ITER] += 1.0;
            if (shs > 0.0 && shs < 1.0e300) {
                kappa = sc[S_RZ] / shs;
            } else {                       // non-positive curvature: stop; on the first iteration
                sc[S_ACTIVE] = 0.0;        // the step is the preconditioned steepest descent s_0
                sc[S_BREAK] = sc[S_ITER];
                kappa = sc[S_ITER] == 1.0 ? 1.0 : 0.0;
            }
        }
        sc[S_KAPPA] = kappa;
    } else {   // PCG_MU
        if (sc[S_ACTIVE] != 0.0) {
            const double rzn = sc[S_RZN];
            sc[S_MU] = rzn / sc[S_RZ];
            sc[S_RZ] = rzn;
        } else {
            sc[S_MU] = 0.0;
        }
    }
}

// The second level of launch_dots for all nk sums in one block (the same partial order and tree as
// finalize_kernel), then the PCG scalar step of `mode`: one launch instead of two.  `out` points into
// `sc` (out = sc + slot), and the scalar step reads the sums just stored through `out`, so neither
// pointer is declared non-aliasing.
__global__ __launch_bounds__(RED_THREADS) void finalize_scalar_kernel(int nk, int count,
                                                                      const double* __restrict__ partial,
                                                                      double* out, int mode, double* sc) {
    __shared__ double sh[RED_THREADS / 64];
    for (int k = 0; k < nk; ++k) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < count; i += RED_THREADS) acc += partial[(long)k * count + i];
        const double t = block_sum<RED_THREADS>(acc, sh);
        if (threadIdx.x == 0) out[k] = t;
    }
    if (threadIdx.x == 0) pcg_scalar_step(mode, sc);
}

__global__ void pcg_update_kernel(long n, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ s,
                                  const double* __restrict__ st, const double* __restrict__ sc) {
    const double kappa = sc[S_KAPPA];
    const bool upd_r = sc[S_ACTIVE] != 0.0;
    // kappa = 0 (after a breakdown) leaves x as it is, also where s is no longer finite
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        if (kappa != 0.0) x[i] += kappa * s[i];
        if (upd_r) r[i] -= kappa * st[i];
    }
}

// pcg_update_kernel with the recurrences z -= kappa pst and kr -= kappa kst, and the block partial
// sums of ||r||^2 and <r, z>_W (kr . z with the weighting, r . z without) over the updated vectors,
// in the contiguous chunks, thread order and tree of dots_kernel: the sums are those dots_kernel
// would form, one launch earlier.
__global__ __launch_bounds__(RED_THREADS) void pcg_update_z_kernel(
    long n, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ s,
    const double* __restrict__ st, double* __restrict__ z, const double* __restrict__ pst, double* __restrict__ kr,
    const double* __restrict__ kst, const double* __restrict__ sc, double* __restrict__ partial) {
    __shared__ double sh[RED_THREADS / 64];
    const double kappa = sc[S_KAPPA];
    const bool upd = sc[S_ACTIVE] != 0.0;
    const long chunk = (n + RED_BLOCKS - 1) / RED_BLOCKS;
    const long lo = (long)blockIdx.x * chunk;
    const long hi = lo + chunk < n ? lo + chunk : n;
    double rr = 0.0, rz = 0.0;
    for (long i = lo + threadIdx.x; i < hi; i += RED_THREADS) {
        if (kappa != 0.0) x[i] += kappa * s[i];
        double ri = r[i], zi = z[i];
        double wi = ri;
        if (upd) {
            ri -= kappa * st[i];
            zi -= kappa * pst[i];
            r[i] = ri;
            z[i] = zi;
            wi = ri;
        }
        if (kr) {
            wi = kr[i];
            if (upd) {
                wi -= kappa * kst[i];
                kr[i] = wi;
            }
        }
        rr += ri * ri;
        rz += wi * zi;
    }
    const double t0 = block_sum<RED_THREADS>(rr, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t0;
    const double t1 = block_sum<RED_THREADS>(rz, sh);
    if (threadIdx.x == 0) partial[RED_BLOCKS + blockIdx.x] = t1;
}

template <typename T>
__global__ void pcg_dir_copy_kernel(long n, double* __restrict__ s, T* __restrict__ sT, const double* __restrict__ z,
                                    const double* __restrict__ sc) {
    const double mu = sc ? sc[S_MU] : 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double v = sc ? z[i] + mu * s[i] : z[i];
        s[i] = v;
        sT[i] = (T)v;
    }
}

hipError_t launch_dots_scalar(int nk, const double* const* a, const double* const* b, long n, double* partial,
                              double* out, int mode, double* scal, hipStream_t s) {
    if (nk < 1 || nk > 4) return hipErrorInvalidValue;
    DotPtrs<double> p{};
    for (int k = 0; k < nk; ++k) {
        p.a[k] = a[k];
        p.b[k] = b[k];
    }
    hipLaunchKernelGGL((dots_kernel<double>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, nk, p, n, partial);
    hipLaunchKernelGGL(finalize_scalar_kernel, dim3(1), dim3(RED_THREADS), 0, s, nk, RED_BLOCKS, partial, out, mode,
                       scal);
    return hipGetLastError();
}

hipError_t launch_finalize_scalar(int nk, int count, const double* partial, double* out, int mode, double* scal,
                                  hipStream_t s) {
    if (nk < 1 || count < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(finalize_scalar_kernel, dim3(1), dim3(RED_THREADS), 0, s, nk, count, partial, out, mode, scal);
    return hipGetLastError();
}

hipError_t launch_pcg_update(long n, double* x, double* r, const double* s, const double* st, const double* scal,
                             hipStream_t stream) {
    hipLaunchKernelGGL(pcg_update_kernel, dim3(grid_for(n)), dim3(256), 0, stream, n, x, r, s, st, scal);
    return hipGetLastError();
}
hipError_t launch_pcg_update_z(long n, double* x, double* r, const double* s, const double* st, double* z,
                               const double* pst, double* kr, const double* kst, const double* scal, double* partial,
                               hipStream_t stream) {
    if ((kr == nullptr) != (kst == nullptr)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pcg_update_z_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, stream, n, x, r, s, st, z, pst,
                       kr, kst, scal, partial);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_pcg_dir_copy(long n, double* s, T* sT, const double* z, const double* scal, hipStream_t stream) {
    hipLaunchKernelGGL((pcg_dir_copy_kernel<T>), dim3(grid_for(n)), dim3(256), 0, stream, n, s, sT, z, scal);
    return hipGetLastError();
}
template hipError_t launch_pcg_dir_copy<float>(long, double*, float*, const double*, const double*, hipStream_t);
template hipError_t launch_pcg_dir_copy<double>(long, double*, double*, const double*, const double*, hipStream_t);

// ---- low-rank deflation correction -------------------------------------------------------------
// valid slots, clamped to [0, cap] (cap <= LR_MAX) so that no kernel reads past the set
__device__ __forceinline__ int lr_count(const double* cnt, int cap) {
    const double c = cnt[0];
    return c >= 0.0 ? (c < (double)cap ? (int)c : cap) : 0;
}

__global__ __launch_bounds__(RED_THREADS) void lr_dots_kernel(const double* __restrict__ x, const double* __restrict__ F,
                                                             long stride, long n, const double* __restrict__ cnt,
                                                             int cap, double* __restrict__ partial) {
    __shared__ double sh[RED_THREADS / 64];
    const int nk = lr_count(cnt, cap);
    const long chunk = (n + RED_BLOCKS - 1) / RED_BLOCKS;
    const long lo = (long)blockIdx.x * chunk;
    const long hi = lo + chunk < n ? lo + chunk : n;
    for (int k = 0; k < nk; ++k) {
        const double* __restrict__ f = F + (long)k * stride;
        double acc = 0.0;
        for (long i = lo + threadIdx.x; i < hi; i += RED_THREADS) acc += x[i] * f[i];
        const double s = block_sum<RED_THREADS>(acc, sh);
        if (threadIdx.x == 0) partial[k * RED_BLOCKS + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(RED_THREADS) void lr_final_kernel(const double* __restrict__ partial,
                                                              const double* __restrict__ cnt, int cap,
                                                              double* __restrict__ out) {
    __shared__ double sh[RED_THREADS / 64];
    const int k = blockIdx.x;
    if (k >= lr_count(cnt, cap)) return;
    double acc = 0.0;
    for (int i = threadIdx.x; i < RED_BLOCKS; i += RED_THREADS) acc += partial[k * RED_BLOCKS + i];
    const double s = block_sum<RED_THREADS>(acc, sh);
    if (threadIdx.x == 0) out[k] = s;
}

__global__ __launch_bounds__(256) void lr_combine_kernel(long n, const double* base, double* out,
                                                        const double* __restrict__ F, long stride,
                                                        const double* __restrict__ cnt, const double* __restrict__ da,
                                                        const double* __restrict__ db, const double* __restrict__ e,
                                                        double sign, int cap) {
    __shared__ double c[LR_MAX];
    const int nk = lr_count(cnt, cap);
    for (int k = threadIdx.x; k < nk; k += blockDim.x) c[k] = sign * (da[k] - (db ? db[k] : 0.0)) / e[k];
    __syncthreads();
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double acc = base[i];
        for (int k = 0; k < nk; ++k) acc += c[k] * F[(long)k * stride + i];
        out[i] = acc;
    }
}

__global__ __launch_bounds__(256) void lr_mix_kernel(long n, double* F, long stride, int rin, int rout, LrMix m) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double in[LR_MIX_MAX];
#pragma unroll
        for (int k = 0; k < LR_MIX_MAX; ++k) in[k] = k < rin ? F[(long)k * stride + i] : 0.0;
#pragma unroll
        for (int j = 0; j < LR_MIX_MAX; ++j) {
            if (j < rout) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < LR_MIX_MAX; ++k) acc += m.m[k][j] * in[k];
                F[(long)j * stride + i] = acc;
            }
        }
    }
}

hipError_t launch_lr_dots(long n, const double* x, const double* F, long stride, const double* cnt, int cap,
                          double* partial, double* out, hipStream_t s) {
    if (cap < 1 || cap > LR_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lr_dots_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, F, stride, n, cnt, cap, partial);
    hipLaunchKernelGGL(lr_final_kernel, dim3(cap), dim3(RED_THREADS), 0, s, partial, cnt, cap, out);
    return hipGetLastError();
}

hipError_t launch_lr_combine(long n, const double* base, double* out, const double* F, long stride,
                             const double* cnt, int cap, const double* da, const double* db, const double* e,
                             double sign, hipStream_t s) {
    if (cap < 0 || cap > LR_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lr_combine_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, base, out, F, stride, cnt, da, db, e,
                       sign, cap);
    return hipGetLastError();
}

hipError_t launch_lr_mix(long n, double* F, long stride, int rin, int rout, const LrMix& m, hipStream_t s) {
    if (rin < 0 || rin > LR_MIX_MAX || rout < 0 || rout > LR_MIX_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lr_mix_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, F, stride, rin, rout, m);
    return hipGetLastError();
}

template hipError_t launch_dots<double>(int, const double* const*, const double* const*, long, double*, double*,
                                        hipStream_t);
template hipError_t launch_dots<float>(int, const float* const*, const float* const*, long, double*, double*,
                                       hipStream_t);
template hipError_t launch_sqdiff<double>(const double*, const double*, long, double*, double*, hipStream_t);
template hipError_t launch_sqdiff<float>(const float*, const float*, long, double*, double*, hipStream_t);
template hipError_t launch_convert<float>(long, const double*, float*, hipStream_t);
template hipError_t launch_convert<double>(long, const double*, double*, hipStream_t);
template hipError_t launch_widen<float>(long, const float*, double*, hipStream_t);
template hipError_t launch_widen<double>(long, const double*, double*, hipStream_t);

}  // namespace regnk
