// Elementwise kernels and reductions of the warm-start network (see net_kernels.hpp for layouts).
#include <algorithm>

#include "device_common.hpp"
#include "net_kernels.hpp"

namespace regnk {

namespace {

constexpr int TB = 256;

inline int blocks_for(long n) { return (int)std::max<long>(1, std::min<long>((n + TB - 1) / TB, 16384)); }

#define GRID_STRIDE(i, n) for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

__global__ void features_kernel(int n, const double* __restrict__ mT, const double* __restrict__ mR,
                                const double* __restrict__ sq, float* __restrict__ out, long cstride) {
    const long nn = (long)n * n;
    const double inv2h = n / (4.0 * 3.14159265358979323846);   // 1 / (2 h), h = 2 pi / n
    const double sc = sqrt(2.0 * sq[0] / (double)nn);
    const double inv_s = sc > 0.0 ? 1.0 / sc : 0.0;
    GRID_STRIDE(i, nn) {
        const int i1 = (int)(i / n), i2 = (int)(i % n);
        const double t = mT[i];
        const double d1 = (mT[(long)((i1 + 1) % n) * n + i2] - mT[(long)((i1 + n - 1) % n) * n + i2]) * inv2h;
        const double d2 = (mT[(long)i1 * n + (i2 + 1) % n] - mT[(long)i1 * n + (i2 + n - 1) % n]) * inv2h;
        const double r = (mR[i] - t) * inv_s;
        out[i] = (float)t;
        out[cstride + i] = (float)d1;
        out[2 * cstride + i] = (float)d2;
        out[3 * cstride + i] = (float)(d1 * d1);
        out[4 * cstride + i] = (float)(d1 * d2);
        out[5 * cstride + i] = (float)(d2 * d2);
        out[6 * cstride + i] = (float)r;
        out[7 * cstride + i] = (float)(r * d1);
        out[8 * cstride + i] = (float)(r * d2);
    }
}

__global__ void scale_kernel(long nn, const double* __restrict__ sq, double* __restrict__ scale) {
    if (threadIdx.x == 0 && blockIdx.x == 0) scale[0] = sqrt(2.0 * sq[0] / (double)nn);
}

__global__ void target_kernel(long nn, const double* __restrict__ v, const double* __restrict__ scale,
                              const double* __restrict__ dirs, float* __restrict__ out) {
    const double sc = scale[0];
    const double inv_s = sc > 0.0 ? 1.0 / sc : 0.0;
    GRID_STRIDE(i, FNO_OUT * nn) {
        if (i < 2 * nn) out[i] = (float)(v[i] * inv_s);
        else out[i] = dirs ? (float)dirs[i - 2 * nn] : 0.0f;
    }
}

__global__ void unscale_kernel(long nn, const float* __restrict__ y, const double* __restrict__ scale,
                               double* __restrict__ v, double* __restrict__ dirs) {
    const double sc = scale[0];
    GRID_STRIDE(i, FNO_OUT * nn) {
        if (i < 2 * nn) v[i] = sc * (double)y[i];
        else if (dirs) dirs[i - 2 * nn] = (double)y[i];
    }
}

__global__ void gather_kernel(const float* __restrict__ set, long nset, int channels, int n,
                              const int32_t* __restrict__ idx, const int32_t* __restrict__ sym, ChannelKinds kinds,
                              int count, float* __restrict__ out) {
    const long nn = (long)n * n;
    const long total = (long)channels * count * nn;
    GRID_STRIDE(i, total) {
        const long p = i % nn;
        const int b = (int)((i / nn) % count);
        const int c = (int)(i / (nn * count));
        const long src = idx[b];
        if (src < 0 || src >= nset) {
            out[i] = 0.0f;
            continue;
        }
        const int code = sym ? sym[b] : 0;
        const bool swap = code & 1, f1 = (code >> 1) & 1, f2 = (code >> 2) & 1;
        const int i1 = (int)(p / n), i2 = (int)(p % n);
        const int a1 = f1 ? (n - i1) % n : i1, a2 = f2 ? (n - i2) % n : i2;
        const long q = swap ? (long)a2 * n + a1 : (long)a1 * n + a2;
        const float s1 = f1 ? -1.0f : 1.0f, s2 = f2 ? -1.0f : 1.0f;
        int cc = c;
        float sign = 1.0f;
        switch (kinds.k[c]) {
            case 1: cc = swap ? c + 1 : c; sign = s1; break;
            case 2: cc = swap ? c - 1 : c; sign = s2; break;
            case 3: cc = swap ? c + 2 : c; break;
            case 4: sign = s1 * s2; break;
            case 5: cc = swap ? c - 2 : c; break;
            default: break;
        }
        out[i] = sign * set[(src * channels + cc) * nn + q];
    }
}

__global__ void mask_disc_kernel(int S, float* __restrict__ Z, int radius) {
    const long total = (long)S * FNO_MODES;
    GRID_STRIDE(i, total) {
        const int mode = (int)(i % FNO_MODES), j = mode >> 4, k2 = mode & 15;
        const int k1 = j < FNO_M ? j : j - 2 * FNO_M;
        if (k1 * k1 + k2 * k2 > radius * radius) {
            Z[i] = 0.0f;
            Z[total + i] = 0.0f;
        }
    }
}

// one thread per (slice, j, k2): 32 x 16 entries per slice
__global__ void combine_kernel(int S, const float* __restrict__ T, float* __restrict__ Z) {
    const long total = (long)S * FNO_MODES;
    GRID_STRIDE(i, total) {
        const long s = i / FNO_MODES;
        const int mode = (int)(i % FNO_MODES), j = mode >> 4, k = mode & 15;
        const float* t = T + s * 2048;
        Z[i] = t[j * 32 + k] + t[(32 + j) * 32 + 16 + k];
        Z[total + i] = t[j * 32 + 16 + k] - t[(32 + j) * 32 + k];
    }
}

__global__ void uncombine_kernel(int S, const float* __restrict__ dZ, float* __restrict__ dT) {
    const long total = (long)S * FNO_MODES;
    GRID_STRIDE(i, total) {
        const long s = i / FNO_MODES;
        const int mode = (int)(i % FNO_MODES), j = mode >> 4, k = mode & 15;
        const float zr = dZ[i], zi = dZ[total + i];
        float* t = dT + s * 2048;
        t[j * 32 + k] = zr;
        t[(32 + j) * 32 + 16 + k] = zr;
        t[j * 32 + 16 + k] = zi;
        t[(32 + j) * 32 + k] = -zi;
    }
}

__global__ void expand_o_kernel(int S, const float* __restrict__ O, float* __restrict__ Ob) {
    const long total = (long)S * FNO_MODES;
    GRID_STRIDE(i, total) {
        const long s = i / FNO_MODES;
        const int mode = (int)(i % FNO_MODES), j = mode >> 4, k = mode & 15;
        const float orr = O[i], oi = O[total + i];
        float* t = Ob + s * 2048;
        t[j * 32 + k] = orr;
        t[j * 32 + 16 + k] = oi;
        t[(32 + j) * 32 + k] = -oi;
        t[(32 + j) * 32 + 16 + k] = orr;
    }
}

__global__ void fold_o_kernel(int S, const float* __restrict__ dOb, float* __restrict__ dO) {
    const long total = (long)S * FNO_MODES;
    GRID_STRIDE(i, total) {
        const long s = i / FNO_MODES;
        const int mode = (int)(i % FNO_MODES), j = mode >> 4, k = mode & 15;
        const float* t = dOb + s * 2048;
        dO[i] = t[j * 32 + k] + t[(32 + j) * 32 + 16 + k];
        dO[total + i] = t[j * 32 + 16 + k] - t[(32 + j) * 32 + k];
    }
}

// one thread per (layer, mode, c, o)
__global__ void expand_w_kernel(int layers, const float* __restrict__ R, long lstride, float* __restrict__ W) {
    const long per = (long)FNO_MODES * FNO_C * FNO_C;
    const long total = layers * per;
    GRID_STRIDE(i, total) {
        const long l = i / per, r = i % per;
        const long mode = r / (FNO_C * FNO_C);
        const int c = (int)((r / FNO_C) % FNO_C), o = (int)(r % FNO_C);
        const float rr = R[l * lstride + r], ri = R[l * lstride + per + r];
        float* w = W + l * per * 4 + mode * 4096;
        w[c * 64 + o] = rr;
        w[c * 64 + 32 + o] = ri;
        w[(32 + c) * 64 + o] = -ri;
        w[(32 + c) * 64 + 32 + o] = rr;
    }
}

__global__ void fold_w_kernel(const float* __restrict__ dW, float* __restrict__ gR) {
    const long per = (long)FNO_MODES * FNO_C * FNO_C;
    GRID_STRIDE(i, per) {
        const long mode = i / (FNO_C * FNO_C);
        const int c = (int)((i / FNO_C) % FNO_C), o = (int)(i % FNO_C);
        const float* w = dW + mode * 4096;
        gR[i] = w[c * 64 + o] + w[(32 + c) * 64 + 32 + o];
        gR[per + i] = w[c * 64 + 32 + o] - w[(32 + c) * 64 + o];
    }
}

// block (chunk, row): the chunk-th of RS_CHUNKS contiguous pieces of row `row`
__global__ __launch_bounds__(TB) void rowsum_part_kernel(long len, const float* __restrict__ x,
                                                         double* __restrict__ part) {
    __shared__ double sh[TB / 64];
    const long piece = (len + RS_CHUNKS - 1) / RS_CHUNKS;
    const long lo = (long)blockIdx.x * piece;
    const long hi = lo + piece < len ? lo + piece : len;
    const float* row = x + (long)blockIdx.y * len;
    double acc = 0.0;
    for (long i = lo + threadIdx.x; i < hi; i += TB) acc += (double)row[i];
    const double s = block_sum<TB>(acc, sh);
    if (threadIdx.x == 0) part[(long)blockIdx.y * RS_CHUNKS + blockIdx.x] = s;
}

__global__ void rowsum_final_kernel(int rows, const double* __restrict__ part, float* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double s = 0.0;
    for (int c = 0; c < RS_CHUNKS; ++c) s += part[(long)r * RS_CHUNKS + c];
    out[r] = (float)s;
}

// block (b, g): sample b's sums over one channel pair.  g = 0, the velocity: squared error and squared
// target; g = 1 + k, direction k: ||t||^2, ||y||^2, <t, y>.  sums[(b (1 + R) + g) 3 + 0..2].
__global__ __launch_bounds__(TB) void loss_sums_kernel(int B, long npos, const float* __restrict__ y,
                                                       const float* __restrict__ t, double* __restrict__ sums) {
    __shared__ double sh[TB / 64];
    const int g = blockIdx.y;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int c = 2 * g; c < 2 * g + 2; ++c) {
        const long base = ((long)c * B + blockIdx.x) * npos;
        for (long i = threadIdx.x; i < npos; i += TB) {
            const double tv = t[base + i], yv = y[base + i];
            if (g == 0) {
                const double d = yv - tv;
                s0 += d * d;
                s1 += tv * tv;
            } else {
                s0 += tv * tv;
                s1 += yv * yv;
                s2 += tv * yv;
            }
        }
    }
    const double r0 = block_sum<TB>(s0, sh);
    const double r1 = block_sum<TB>(s1, sh);
    const double r2 = block_sum<TB>(s2, sh);
    if (threadIdx.x == 0) {
        double* o = sums + ((long)blockIdx.x * (1 + FNO_RANK) + g) * 3;
        o[0] = r0;
        o[1] = r1;
        o[2] = r2;
    }
}

__global__ void loss_grad_kernel(int B, long npos, const float* __restrict__ y, const float* __restrict__ t,
                                 const double* __restrict__ sums, float* __restrict__ dy) {
    const long total = (long)FNO_OUT * B * npos;
    GRID_STRIDE(i, total) {
        const int b = (int)((i / npos) % B);
        const int c = (int)(i / (npos * B));
        if (c < 2) {
            const double den = sums[(long)b * (1 + FNO_RANK) * 3 + 1];
            dy[i] = den > 0.0 ? (float)(2.0 * ((double)y[i] - (double)t[i]) / (B * den)) : 0.0f;
        } else {
            const double* S = sums + ((long)b * (1 + FNO_RANK) + 1 + (c - 2) / 2) * 3;
            const double a = S[0], bb = fmax(S[1], 1e-30), cc = S[2];
            const double f = FNO_DIR_WEIGHT / ((double)B * FNO_RANK);
            dy[i] = a > 0.0 ? (float)(f * (-2.0 * cc * (double)t[i] / (a * bb) + 2.0 * cc * cc * (double)y[i] / (a * bb * bb)))
                            : 0.0f;
        }
    }
}

__global__ void loss_value_kernel(int B, const double* __restrict__ sums, double* __restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double L = 0.0;
    for (int b = 0; b < B; ++b) {
        const double* S = sums + (long)b * (1 + FNO_RANK) * 3;
        L += S[1] > 0.0 ? S[0] / S[1] : 0.0;
        for (int k = 0; k < FNO_RANK; ++k) {
            const double* D = S + 3 * (1 + k);
            if (D[0] > 0.0) L += (FNO_DIR_WEIGHT / FNO_RANK) * (1.0 - D[2] * D[2] / (D[0] * fmax(D[1], 1e-30)));
        }
    }
    *loss = L / B;
}

__global__ void adam_kernel(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    GRID_STRIDE(i, n) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

}  // namespace

hipError_t launch_fno_features(int n, const double* mT, const double* mR, const double* sq, float* out, long cstride,
                               hipStream_t s) {
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for((long)n * n)), dim3(TB), 0, s, n, mT, mR, sq, out, cstride);
    return hipGetLastError();
}

hipError_t launch_fno_scale(long nn, const double* sq, double* scale, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(64), 0, s, nn, sq, scale);
    return hipGetLastError();
}

hipError_t launch_fno_target(long nn, const double* v, const double* scale, const double* dirs, float* out,
                             hipStream_t s) {
    hipLaunchKernelGGL(target_kernel, dim3(blocks_for(FNO_OUT * nn)), dim3(TB), 0, s, nn, v, scale, dirs, out);
    return hipGetLastError();
}

hipError_t launch_fno_unscale(long nn, const float* y, const double* scale, double* v, double* dirs, hipStream_t s) {
    hipLaunchKernelGGL(unscale_kernel, dim3(blocks_for(FNO_OUT * nn)), dim3(TB), 0, s, nn, y, scale, v, dirs);
    return hipGetLastError();
}

hipError_t launch_fno_gather(const float* set, long nset, int channels, int n, const int32_t* idx,
                             const int32_t* sym, ChannelKinds kinds, int count, float* out, hipStream_t s) {
    if (channels < 1 || channels > 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for((long)channels * count * n * n)), dim3(TB), 0, s, set, nset,
                       channels, n, idx, sym, kinds, count, out);
    return hipGetLastError();
}

hipError_t launch_fno_mask_disc(int S, float* Z, int radius, hipStream_t s) {
    hipLaunchKernelGGL(mask_disc_kernel, dim3(blocks_for((long)S * FNO_MODES)), dim3(TB), 0, s, S, Z, radius);
    return hipGetLastError();
}

hipError_t launch_fno_combine(int S, const float* T, float* Z, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3(blocks_for((long)S * FNO_MODES)), dim3(TB), 0, s, S, T, Z);
    return hipGetLastError();
}

hipError_t launch_fno_uncombine(int S, const float* dZ, float* dT, hipStream_t s) {
    hipLaunchKernelGGL(uncombine_kernel, dim3(blocks_for((long)S * FNO_MODES)), dim3(TB), 0, s, S, dZ, dT);
    return hipGetLastError();
}

hipError_t launch_fno_expand_o(int S, const float* O, float* Ob, hipStream_t s) {
    hipLaunchKernelGGL(expand_o_kernel, dim3(blocks_for((long)S * FNO_MODES)), dim3(TB), 0, s, S, O, Ob);
    return hipGetLastError();
}

hipError_t launch_fno_fold_o(int S, const float* dOb, float* dO, hipStream_t s) {
    hipLaunchKernelGGL(fold_o_kernel, dim3(blocks_for((long)S * FNO_MODES)), dim3(TB), 0, s, S, dOb, dO);
    return hipGetLastError();
}

hipError_t launch_fno_expand_w(int layers, const float* R, long lstride, float* W, hipStream_t s) {
    const long total = (long)layers * FNO_MODES * FNO_C * FNO_C;
    hipLaunchKernelGGL(expand_w_kernel, dim3(blocks_for(total)), dim3(TB), 0, s, layers, R, lstride, W);
    return hipGetLastError();
}

hipError_t launch_fno_fold_w(const float* dW, float* gR, hipStream_t s) {
    hipLaunchKernelGGL(fold_w_kernel, dim3(blocks_for((long)FNO_MODES * FNO_C * FNO_C)), dim3(TB), 0, s, dW, gR);
    return hipGetLastError();
}

hipError_t launch_rowsum(int rows, long len, const float* x, double* part, float* out, hipStream_t s) {
    if (rows < 1 || rows > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rowsum_part_kernel, dim3(RS_CHUNKS, rows), dim3(TB), 0, s, len, x, part);
    hipLaunchKernelGGL(rowsum_final_kernel, dim3((rows + 63) / 64), dim3(64), 0, s, rows, part, out);
    return hipGetLastError();
}

hipError_t launch_fno_loss(int B, long npos, const float* y, const float* t, double* sums, float* dy, double* loss,
                           hipStream_t s) {
    hipLaunchKernelGGL(loss_sums_kernel, dim3(B, 1 + FNO_RANK), dim3(TB), 0, s, B, npos, y, t, sums);
    hipLaunchKernelGGL(loss_grad_kernel, dim3(blocks_for((long)FNO_OUT * B * npos)), dim3(TB), 0, s, B, npos, y, t,
                       sums, dy);
    if (loss) hipLaunchKernelGGL(loss_value_kernel, dim3(1), dim3(64), 0, s, B, sums, loss);
    return hipGetLastError();
}

hipError_t launch_adam(long n, float* p, const float* g, float* m, float* v, float lr, float beta1, float beta2,
                       float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(TB), 0, s, n, p, g, m, v, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace regnk
