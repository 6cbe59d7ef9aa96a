// Batched GEMM on the CDNA4 matrix cores: bfloat16 multiplicands, FP32 accumulation (and an FP32
// vector-ALU variant of the same tiling for fixed filters, see gemm_f32_kernel).
//
// Tile: 64 x 64 outputs per workgroup of 256 threads (4 waves, 2 x 2 arrangement, each wave 32 x 32
// = 2 x 2 MFMA blocks of 16 x 16), K step 32 = one v_mfma_f32_16x16x32_bf16 per block.  Both
// operand tiles are staged in LDS k-contiguous ([row][k], pitch 40 bf16) so that every lane fetches
// its 8 multiplicands with one 16-byte LDS read: lane l holds row l % 16, k = 8 (l / 16) .. + 7 of A
// and column l % 16, the same k, of B; the accumulator holds C rows 4 (l / 16) .. + 3 of column
// l % 16.  Global loads are coalesced along whichever operand axis is contiguous in memory (k, or
// m / n), vectorised when alignment allows, and the next K tile is fetched into registers while the
// MFMAs of the current one run.
#include <algorithm>

#include "net_kernels.hpp"

namespace regnk {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BN = 64, BK = 32, LDP = BK + 8;

enum LoadMode { LD_KCONT = 0, LD_RCONT = 1, LD_GENERIC = 2 };

__device__ __forceinline__ unsigned bf16_bits(float f) {   // round to nearest even
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;   // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// The 8 values a thread owns of a 64 (rows) x 32 (k) operand tile starting at (r0, k0); `rows` and
// `kend` bound the valid region.  KCONT / GENERIC: row = t / 4, k = 8 (t % 4) + i.  RCONT (rows
// contiguous, srow == 1): k = t / 8, row = 8 (t % 8) + i.
template <int MODE>
__device__ __forceinline__ void load_tile(const float* __restrict__ p, long srow, long sk, int rows, int kend, int r0,
                                          int k0, bool vec, float (&v)[8]) {
    const int t = threadIdx.x;
    if (MODE == LD_RCONT) {
        const int k = k0 + (t >> 3);
        const int r = r0 + (t & 7) * 8;
        if (vec && k < kend && r + 8 <= rows) {
            const float4* q = reinterpret_cast<const float4*>(p + (long)k * sk + r);
            const float4 a = q[0], b = q[1];
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = (k < kend && r + i < rows) ? p[(long)k * sk + (r + i)] : 0.0f;
        }
    } else {
        const int r = r0 + (t >> 2);
        const int k = k0 + (t & 3) * 8;
        if (MODE == LD_KCONT && vec && r < rows && k + 8 <= kend) {
            const float4* q = reinterpret_cast<const float4*>(p + (long)r * srow + k);
            const float4 a = q[0], b = q[1];
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                v[i] = (r < rows && k + i < kend) ? p[(long)r * srow + (long)(k + i) * sk] : 0.0f;
        }
    }
}

template <int MODE>
__device__ __forceinline__ void store_tile(unsigned short* __restrict__ lds, const float (&v)[8]) {
    const int t = threadIdx.x;
    if (MODE == LD_RCONT) {
        const int k = t >> 3;
        const int r = (t & 7) * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[(r + i) * LDP + k] = (unsigned short)bf16_bits(v[i]);
    } else {
        const int r = t >> 2;
        const int k = (t & 3) * 8;
        uint4 w;
        w.x = bf16_bits(v[0]) | (bf16_bits(v[1]) << 16);
        w.y = bf16_bits(v[2]) | (bf16_bits(v[3]) << 16);
        w.z = bf16_bits(v[4]) | (bf16_bits(v[5]) << 16);
        w.w = bf16_bits(v[6]) | (bf16_bits(v[7]) << 16);
        *reinterpret_cast<uint4*>(lds + r * LDP + k) = w;
    }
}

template <int AMODE, int BMODE>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) unsigned short As[BM * LDP];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[BN * LDP];
    const int n0 = blockIdx.x * BN;
    const int m0 = blockIdx.y * BM;
    const int b = blockIdx.z % g.batch;
    const int ks = blockIdx.z / g.batch;
    const int kbeg = ks * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);
    const float* __restrict__ A = g.A + (long)b * g.ab;
    const float* __restrict__ B = g.B + (long)b * g.bb;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;

    f32x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    float va[8], vb[8];
    load_tile<AMODE>(A + (long)m0 * g.am, g.am, g.ak, g.M - m0, kend, 0, kbeg, g.avec, va);
    load_tile<BMODE>(B + (long)n0 * g.bn, g.bn, g.bk, g.N - n0, kend, 0, kbeg, g.bvec, vb);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();   // the previous tile's MFMA reads are done
        store_tile<AMODE>(As, va);
        store_tile<BMODE>(Bs, vb);
        __syncthreads();
        if (k0 + BK < kend) {
            load_tile<AMODE>(A + (long)m0 * g.am, g.am, g.ak, g.M - m0, kend, 0, k0 + BK, g.avec, va);
            load_tile<BMODE>(B + (long)n0 * g.bn, g.bn, g.bk, g.N - n0, kend, 0, k0 + BK, g.bvec, vb);
        }
        bf16x8_t fa[2], fb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            fa[i] = *reinterpret_cast<const bf16x8_t*>(As + (wm + i * 16 + (lane & 15)) * LDP + (lane >> 4) * 8);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            fb[j] = *reinterpret_cast<const bf16x8_t*>(Bs + (wn + j * 16 + (lane & 15)) * LDP + (lane >> 4) * 8);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                float v = acc[i][j][r];
                if (g.part) {
                    g.part[(long)ks * g.M * g.N + (long)row * g.N + col] = v;
                    continue;
                }
                const long ci = (long)b * g.cb + (long)row * g.cm + (long)col * g.cn;
                v *= g.alpha;
                if (g.beta != 0.0f) v += g.beta * g.C[ci];
                if (g.bias) v += g.bias[row];
                if (g.add) v += g.add[(long)b * g.db + (long)row * g.dm + (long)col * g.dn];
                if (g.Z) g.Z[ci] = v;
                if (g.act == ACT_GELU) v = gelu_f(v);
                else if (g.act == ACT_GELU_BWD) v *= gelu_grad_f(g.aux[ci]);
                g.C[ci] = v;
            }
}

// FP32 path: the same tiles staged k-major in LDS as floats; thread (t % 16, t / 16) accumulates a
// 4 x 4 block (rows 4 (t / 16) .., columns 4 (t % 16) ..) with FP32 FMAs.
template <int MODE>
__device__ __forceinline__ void store_tile_f32(float (*lds)[BM + 4], const float (&v)[8]) {
    const int t = threadIdx.x;
    if (MODE == LD_RCONT) {
        const int k = t >> 3;
        const int r = (t & 7) * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[k][r + i] = v[i];
    } else {
        const int r = t >> 2;
        const int k = (t & 3) * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[k + i][r] = v[i];
    }
}

template <int AMODE, int BMODE>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) float As[BK][BM + 4];
    __shared__ __attribute__((aligned(16))) float Bs[BK][BN + 4];
    const int n0 = blockIdx.x * BN;
    const int m0 = blockIdx.y * BM;
    const int b = blockIdx.z % g.batch;
    const int ks = blockIdx.z / g.batch;
    const int kbeg = ks * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);
    const float* __restrict__ A = g.A + (long)b * g.ab;
    const float* __restrict__ B = g.B + (long)b * g.bb;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
    float va[8], vb[8];
    load_tile<AMODE>(A + (long)m0 * g.am, g.am, g.ak, g.M - m0, kend, 0, kbeg, g.avec, va);
    load_tile<BMODE>(B + (long)n0 * g.bn, g.bn, g.bk, g.N - n0, kend, 0, kbeg, g.bvec, vb);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
        store_tile_f32<AMODE>(As, va);
        store_tile_f32<BMODE>(Bs, vb);
        __syncthreads();
        if (k0 + BK < kend) {
            load_tile<AMODE>(A + (long)m0 * g.am, g.am, g.ak, g.M - m0, kend, 0, k0 + BK, g.avec, va);
            load_tile<BMODE>(B + (long)n0 * g.bn, g.bn, g.bk, g.N - n0, kend, 0, k0 + BK, g.bvec, vb);
        }
#pragma unroll 8
        for (int kk = 0; kk < BK; ++kk) {
            const float4 a = *reinterpret_cast<const float4*>(&As[kk][ty * 4]);
            const float4 c = *reinterpret_cast<const float4*>(&Bs[kk][tx * 4]);
            const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = m0 + ty * 4 + i;
            const int col = n0 + tx * 4 + j;
            if (row >= g.M || col >= g.N) continue;
            float v = acc[i][j];
            if (g.part) {
                g.part[(long)ks * g.M * g.N + (long)row * g.N + col] = v;
                continue;
            }
            const long ci = (long)b * g.cb + (long)row * g.cm + (long)col * g.cn;
            v *= g.alpha;
            if (g.beta != 0.0f) v += g.beta * g.C[ci];
            if (g.bias) v += g.bias[row];
            if (g.add) v += g.add[(long)b * g.db + (long)row * g.dm + (long)col * g.dn];
            if (g.Z) g.Z[ci] = v;
            if (g.act == ACT_GELU) v = gelu_f(v);
            else if (g.act == ACT_GELU_BWD) v *= gelu_grad_f(g.aux[ci]);
            g.C[ci] = v;
        }
}

__global__ void splitk_reduce_kernel(int ksplit, int M, int N, const float* __restrict__ part, float alpha, float beta,
                                     float* __restrict__ C, long cm, long cn) {
    const long MN = (long)M * N;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < MN; i += (long)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int k = 0; k < ksplit; ++k) s += part[k * MN + i];
        const long ci = (i / N) * cm + (i % N) * cn;
        float v = alpha * s;
        if (beta != 0.0f) v += beta * C[ci];
        C[ci] = v;
    }
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <int AMODE, int BMODE>
void launch_t(const GemmArgs& g, dim3 grid, hipStream_t s) {
    if (g.f32) hipLaunchKernelGGL((gemm_f32_kernel<AMODE, BMODE>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((gemm_bf16_kernel<AMODE, BMODE>), grid, dim3(256), 0, s, g);
}

template <int AMODE>
void launch_b(const GemmArgs& g, int bmode, dim3 grid, hipStream_t s) {
    if (bmode == LD_KCONT) launch_t<AMODE, LD_KCONT>(g, grid, s);
    else if (bmode == LD_RCONT) launch_t<AMODE, LD_RCONT>(g, grid, s);
    else launch_t<AMODE, LD_GENERIC>(g, grid, s);
}

}  // namespace

hipError_t launch_gemm(GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0) return hipErrorInvalidValue;
    if (g.ksplit < 1) g.ksplit = 1;
    if (g.ksplit > 1 && !g.part) return hipErrorInvalidValue;
    if (g.part && g.batch != 1) return hipErrorInvalidValue;
    if (!g.part && !g.C) return hipErrorInvalidValue;
    // chunk: a multiple of BK so that every chunk but the last is full
    g.kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
    g.ksplit = (g.K + g.kchunk - 1) / g.kchunk;
    const int amode = g.ak == 1 ? LD_KCONT : (g.am == 1 ? LD_RCONT : LD_GENERIC);
    const int bmode = g.bk == 1 ? LD_KCONT : (g.bn == 1 ? LD_RCONT : LD_GENERIC);
    const long a_other = amode == LD_KCONT ? g.am : g.ak;
    const long b_other = bmode == LD_KCONT ? g.bn : g.bk;
    g.avec = amode != LD_GENERIC && aligned16(g.A) && a_other % 4 == 0 && (g.batch == 1 || g.ab % 4 == 0);
    g.bvec = bmode != LD_GENERIC && aligned16(g.B) && b_other % 4 == 0 && (g.batch == 1 || g.bb % 4 == 0);
    const long gz = (long)g.batch * g.ksplit;
    const long gy = (g.M + BM - 1) / BM;
    if (gz > 65535 || gy > 65535) return hipErrorInvalidConfiguration;
    dim3 grid((g.N + BN - 1) / BN, (unsigned)gy, (unsigned)gz);
    if (amode == LD_KCONT) launch_b<LD_KCONT>(g, bmode, grid, s);
    else if (amode == LD_RCONT) launch_b<LD_RCONT>(g, bmode, grid, s);
    else launch_b<LD_GENERIC>(g, bmode, grid, s);
    return hipGetLastError();
}

hipError_t launch_splitk_reduce(int ksplit, int M, int N, const float* part, float alpha, float beta, float* C,
                                long cm, long cn, hipStream_t s) {
    const long MN = (long)M * N;
    const int blocks = (int)std::min<long>((MN + 255) / 256, 1024);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, s, ksplit, M, N, part, alpha, beta, C, cm, cn);
    return hipGetLastError();
}

}  // namespace regnk
