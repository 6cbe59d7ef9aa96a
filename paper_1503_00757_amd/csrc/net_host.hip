// Host driver of the warm-start network: workspace layout, the GEMM sequences of the forward and
// reverse passes, and the C ABI of regnet.h.
//
// One Fourier layer, forward (S = 32 B slices of n x n, P = B n^2):
//   Y  [S n][32] = h [S n][n] . F2 [n][32]             truncated DFT along i2 (Re | Im of k2 < 16)
//   T  [S][64][32] = CS [64][n] . Y[s]                  DFT along i1 of Re and Im parts
//   Z  [2][S][512] = combine(T)                          Re / Im of the 512 retained coefficients
//   O  (per mode) [B][64] = Z [B][64] . Wexp [64][64]    complex channel mixing in real block form
//   Ob [S][64][32] = [[Or, Oi], [-Oi, Or]]
//   Yp [S n][32] = IC [n][64] . Ob[s]                    inverse DFT along i1
//   hp [S n][n]  = Yp . G2 [32][n]                       inverse real DFT along i2
//   h' = gelu(W h + b + hp)                              one GEMM with the epilogue fused
// The output u of the projection is band-limited the same way with identity mode weights on the
// disc |k| <= 12 of the retained square: y = IC . expand(mask(combine(CS . (u . F2)))) . G2, so the
// predicted velocity has no energy outside that disc.  This fixed filter acts on the velocity itself and runs in FP32 (FMA path): in
// bfloat16 its data would lose 2^-9 of the velocity's precision.
// The reverse pass applies the transposes of the same products in the opposite order; weight
// gradients of the pointwise layers are long-K GEMMs split over K with a deterministic reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "host_common.hpp"
#include "kernels.hpp"
#include "net_kernels.hpp"
#include "regnet.h"

using namespace regnk;

namespace {

// flat parameter offsets (layout documented in regnet.h)
constexpr long R_BLOCK = (long)FNO_MODES * FNO_C * FNO_C;       // 524288
constexpr long OFF_WL = 0;
constexpr long OFF_BL = FNO_C * FNO_IN;
constexpr long OFF_L0 = OFF_BL + FNO_C;
constexpr long L_STRIDE = 2 * R_BLOCK + FNO_C * FNO_C + FNO_C;
constexpr long off_R(int l) { return OFF_L0 + l * L_STRIDE; }
constexpr long off_W(int l) { return off_R(l) + 2 * R_BLOCK; }
constexpr long off_B(int l) { return off_W(l) + FNO_C * FNO_C; }
constexpr long OFF_Q1 = OFF_L0 + FNO_L * L_STRIDE;
constexpr long OFF_q1 = OFF_Q1 + FNO_H * FNO_C;
constexpr long OFF_Q2 = OFF_q1 + FNO_H;
constexpr long OFF_q2 = OFF_Q2 + FNO_OUT * FNO_H;
constexpr long N_PARAMS = OFF_q2 + FNO_OUT;
static_assert(N_PARAMS == REG_FNO_PARAMS, "parameter layout");
static_assert(FNO_OUT == REG_FNO_OUT && FNO_RANK == REG_FNO_RANK, "output channels");

constexpr int KSPLIT_MAX = 1024;   // weight gradients: K = P split into chunks of >= 512
constexpr long PART_FLOATS = (long)KSPLIT_MAX * FNO_H * FNO_C;

struct NetLayout {
    size_t F2, CS, IC, G2, in, y, u, du, h[FNO_L + 1], z[FNO_L - 1], zq, s, hp, Y, Yp, T, Zs[FNO_L], O, dZ, Wexp, dWexp, dy,
        dzq, dA, dB, part, rsum, sums, loss, red, sq, scale, total;
};

NetLayout net_layout(int n, int B) {
    NetLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t P = (size_t)B * n * n, S = (size_t)FNO_C * B, f = sizeof(float);
    L.F2 = take((size_t)n * 32 * f);
    L.CS = take((size_t)64 * n * f);
    L.IC = take((size_t)n * 64 * f);
    L.G2 = take((size_t)32 * n * f);
    L.in = take(FNO_IN * P * f);
    L.y = take(FNO_OUT * P * f);
    L.u = take(FNO_OUT * P * f);
    L.du = take(FNO_OUT * P * f);
    for (auto& o : L.h) o = take(FNO_C * P * f);
    for (auto& o : L.z) o = take(FNO_C * P * f);
    L.zq = take(FNO_H * P * f);
    L.s = take(FNO_H * P * f);
    L.hp = take(FNO_C * P * f);
    L.Y = take(S * n * 32 * f);
    L.Yp = take(S * n * 32 * f);
    L.T = take(S * 2048 * f);
    for (auto& o : L.Zs) o = take(2 * S * FNO_MODES * f);
    L.O = take(2 * S * FNO_MODES * f);
    L.dZ = take(2 * S * FNO_MODES * f);
    L.Wexp = take((size_t)FNO_L * FNO_MODES * 4096 * f);
    L.dWexp = take((size_t)FNO_MODES * 4096 * f);
    L.dy = take(FNO_OUT * P * f);
    L.dzq = take(FNO_H * P * f);
    L.dA = take(FNO_C * P * f);
    L.dB = take(FNO_C * P * f);
    L.part = take(PART_FLOATS * f);
    L.rsum = take((size_t)FNO_H * RS_CHUNKS * sizeof(double));
    L.sums = take((size_t)FNO_LOSS_SUMS * B * sizeof(double));
    L.loss = take(sizeof(double));
    L.red = take(RED_BLOCKS * sizeof(double));
    L.sq = take(sizeof(double));
    L.scale = take(sizeof(double));
    L.total = off;
    return L;
}

reg_status check_sizes(int n, int B) {
    if (n < 32 || n > 1024 || (n & (n - 1)) != 0) return fail(REG_EINVAL, "network grid n=%d: power of two in [32, 1024]", n);
    if (B < 1 || B > 64) return fail(REG_EINVAL, "network batch %d out of [1, 64]", B);
    return REG_OK;
}

GemmArgs gemm0() {
    GemmArgs g{};
    g.batch = 1;
    g.alpha = 1.0f;
    g.ksplit = 1;
    return g;
}

}  // namespace

struct reg_fno {
    int n = 0, B = 0, S = 0;
    long P = 0;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    NetLayout L{};
    bool have_forward = false;
    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
    float* f(size_t off) const { return at<float>(off); }
};

namespace {

reg_status gemm(reg_fno* F, GemmArgs g) {
    CK(launch_gemm(g, F->stream));
    return REG_OK;
}

// out(m, n) = sum_p A(m, p) B(p, n) over p < P (A rows contiguous in p, B = X^T with X rows
// contiguous in p): a weight gradient, split over K, reduced in a fixed order.
reg_status wgrad(reg_fno* F, int M, int N, const float* A, const float* X, float* out, long cm) {
    GemmArgs g = gemm0();
    g.M = M; g.N = N; g.K = (int)F->P;
    g.A = A; g.am = F->P; g.ak = 1;
    g.B = X; g.bk = 1; g.bn = F->P;
    g.ksplit = (int)std::min<long>(KSPLIT_MAX, std::max<long>(1, F->P / 512));
    g.part = F->f(F->L.part);
    CK(launch_gemm(g, F->stream));
    CK(launch_splitk_reduce(g.ksplit, M, N, g.part, 1.0f, 0.0f, out, cm, 1, F->stream));
    return REG_OK;
}

// y = band limit of u (ch channels, slices s = c B + b) through the DFT matrices; Y, T, O and Yp
// are scratch.
reg_status band_limit(reg_fno* F, const float* u, float* y, int ch) {
    const int n = F->n, S2 = ch * F->B;
    const NetLayout& L = F->L;
    float *Y = F->f(L.Y), *Yp = F->f(L.Yp), *T = F->f(L.T), *O = F->f(L.O);
    {
        GemmArgs g = gemm0();
        g.f32 = 1;
        g.M = S2 * n; g.N = 32; g.K = n;
        g.A = u; g.am = n; g.ak = 1;
        g.B = F->f(L.F2); g.bk = 32; g.bn = 1;
        g.C = Y; g.cm = 32; g.cn = 1;
        CKS(gemm(F, g));
    }
    {
        GemmArgs g = gemm0();
        g.f32 = 1;
        g.M = 64; g.N = 32; g.K = n; g.batch = S2;
        g.A = F->f(L.CS); g.am = n; g.ak = 1; g.ab = 0;
        g.B = Y; g.bk = 32; g.bn = 1; g.bb = 32L * n;
        g.C = T; g.cm = 32; g.cn = 1; g.cb = 2048;
        CKS(gemm(F, g));
    }
    CK(launch_fno_combine(S2, T, O, F->stream));
    CK(launch_fno_mask_disc(S2, O, FNO_RADIUS, F->stream));
    CK(launch_fno_expand_o(S2, O, T, F->stream));
    {
        GemmArgs g = gemm0();
        g.f32 = 1;
        g.M = n; g.N = 32; g.K = 64; g.batch = S2;
        g.A = F->f(L.IC); g.am = 64; g.ak = 1; g.ab = 0;
        g.B = T; g.bk = 32; g.bn = 1; g.bb = 2048;
        g.C = Yp; g.cm = 32; g.cn = 1; g.cb = 32L * n;
        CKS(gemm(F, g));
    }
    {
        GemmArgs g = gemm0();
        g.f32 = 1;
        g.M = S2 * n; g.N = n; g.K = 32;
        g.A = Yp; g.am = 32; g.ak = 1;
        g.B = F->f(L.G2); g.bk = n; g.bn = 1;
        g.C = y; g.cm = n; g.cn = 1;
        CKS(gemm(F, g));
    }
    return REG_OK;
}

// du = (band limit)^T dy: the products of band_limit transposed, in reverse order.
reg_status band_limit_T(reg_fno* F, const float* dy, float* du, int ch) {
    const int n = F->n, S2 = ch * F->B;
    const NetLayout& L = F->L;
    float *Y = F->f(L.Y), *Yp = F->f(L.Yp), *T = F->f(L.T), *O = F->f(L.O);
    {
        GemmArgs g = gemm0();
        g.f32 = 1;
        g.M = S2 * n; g.N = 32; g.K = n;
        g.A = dy; g.am = n; g.ak = 1;
        g.B = F->f(L.G2); g.bk = 1; g.bn = n;
        g.C = Yp; g.cm = 32; g.cn = 1;
        CKS(gemm(F, g));
    }
    {
        GemmArgs g = gemm0();
        g.f32 = 1;
        g.M = 64; g.N = 32; g.K = n; g.batch = S2;
        g.A = F->f(L.IC); g.am = 1; g.ak = 64; g.ab = 0;
        g.B = Yp; g.bk = 32; g.bn = 1; g.bb = 32L * n;
        g.C = T; g.cm = 32; g.cn = 1; g.cb = 2048;
        CKS(gemm(F, g));
    }
    CK(launch_fno_fold_o(S2, T, O, F->stream));
    CK(launch_fno_mask_disc(S2, O, FNO_RADIUS, F->stream));
    CK(launch_fno_uncombine(S2, O, T, F->stream));
    {
        GemmArgs g = gemm0();
        g.f32 = 1;
        g.M = n; g.N = 32; g.K = 64; g.batch = S2;
        g.A = F->f(L.CS); g.am = 1; g.ak = n; g.ab = 0;
        g.B = T; g.bk = 32; g.bn = 1; g.bb = 2048;
        g.C = Y; g.cm = 32; g.cn = 1; g.cb = 32L * n;
        CKS(gemm(F, g));
    }
    {
        GemmArgs g = gemm0();
        g.f32 = 1;
        g.M = S2 * n; g.N = n; g.K = 32;
        g.A = Y; g.am = 32; g.ak = 1;
        g.B = F->f(L.F2); g.bk = 1; g.bn = 32;
        g.C = du; g.cm = n; g.cn = 1;
        CKS(gemm(F, g));
    }
    return REG_OK;
}

reg_status forward_impl(reg_fno* F, const float* th) {
    const int n = F->n, S = F->S, B = F->B;
    const long P = F->P;
    const NetLayout& L = F->L;
    float *Y = F->f(L.Y), *Yp = F->f(L.Yp), *T = F->f(L.T), *O = F->f(L.O), *hp = F->f(L.hp);
    CK(launch_fno_expand_w(FNO_L, th + off_R(0), L_STRIDE, F->f(L.Wexp), F->stream));
    {   // lifting
        GemmArgs g = gemm0();
        g.M = FNO_C; g.N = (int)P; g.K = FNO_IN;
        g.A = th + OFF_WL; g.am = FNO_IN; g.ak = 1;
        g.B = F->f(L.in); g.bk = P; g.bn = 1;
        g.C = F->f(L.h[0]); g.cm = P; g.cn = 1;
        g.bias = th + OFF_BL;
        CKS(gemm(F, g));
    }
    for (int l = 0; l < FNO_L; ++l) {
        const float* h = F->f(L.h[l]);
        {   // Y = h . F2
            GemmArgs g = gemm0();
            g.M = S * n; g.N = 32; g.K = n;
            g.A = h; g.am = n; g.ak = 1;
            g.B = F->f(L.F2); g.bk = 32; g.bn = 1;
            g.C = Y; g.cm = 32; g.cn = 1;
            CKS(gemm(F, g));
        }
        {   // T[s] = CS . Y[s]
            GemmArgs g = gemm0();
            g.M = 64; g.N = 32; g.K = n; g.batch = S;
            g.A = F->f(L.CS); g.am = n; g.ak = 1; g.ab = 0;
            g.B = Y; g.bk = 32; g.bn = 1; g.bb = 32L * n;
            g.C = T; g.cm = 32; g.cn = 1; g.cb = 2048;
            CKS(gemm(F, g));
        }
        CK(launch_fno_combine(S, T, F->f(L.Zs[l]), F->stream));
        {   // O = Z . Wexp, one 64 x 64 product per retained mode
            GemmArgs g = gemm0();
            g.M = B; g.N = 64; g.K = 64; g.batch = FNO_MODES;
            g.A = F->f(L.Zs[l]); g.am = FNO_MODES; g.ak = (long)B * FNO_MODES; g.ab = 1;
            g.B = F->f(L.Wexp) + (long)l * FNO_MODES * 4096; g.bk = 64; g.bn = 1; g.bb = 4096;
            g.C = O; g.cm = FNO_MODES; g.cn = (long)B * FNO_MODES; g.cb = 1;
            CKS(gemm(F, g));
        }
        CK(launch_fno_expand_o(S, O, T, F->stream));
        {   // Yp[s] = IC . Ob[s]
            GemmArgs g = gemm0();
            g.M = n; g.N = 32; g.K = 64; g.batch = S;
            g.A = F->f(L.IC); g.am = 64; g.ak = 1; g.ab = 0;
            g.B = T; g.bk = 32; g.bn = 1; g.bb = 2048;
            g.C = Yp; g.cm = 32; g.cn = 1; g.cb = 32L * n;
            CKS(gemm(F, g));
        }
        {   // hp = Yp . G2
            GemmArgs g = gemm0();
            g.M = S * n; g.N = n; g.K = 32;
            g.A = Yp; g.am = 32; g.ak = 1;
            g.B = F->f(L.G2); g.bk = n; g.bn = 1;
            g.C = hp; g.cm = n; g.cn = 1;
            CKS(gemm(F, g));
        }
        {   // h_{l+1} = act(W h + b + hp)
            GemmArgs g = gemm0();
            g.M = FNO_C; g.N = (int)P; g.K = FNO_C;
            g.A = th + off_W(l); g.am = FNO_C; g.ak = 1;
            g.B = h; g.bk = P; g.bn = 1;
            g.C = F->f(L.h[l + 1]); g.cm = P; g.cn = 1;
            g.bias = th + off_B(l);
            g.add = hp; g.dm = P; g.dn = 1;
            if (l < FNO_L - 1) {
                g.Z = F->f(L.z[l]);
                g.act = ACT_GELU;
            }
            CKS(gemm(F, g));
        }
    }
    {   // s = gelu(Q1 h4 + q1)
        GemmArgs g = gemm0();
        g.M = FNO_H; g.N = (int)P; g.K = FNO_C;
        g.A = th + OFF_Q1; g.am = FNO_C; g.ak = 1;
        g.B = F->f(L.h[FNO_L]); g.bk = P; g.bn = 1;
        g.C = F->f(L.s); g.cm = P; g.cn = 1;
        g.bias = th + OFF_q1;
        g.Z = F->f(L.zq);
        g.act = ACT_GELU;
        CKS(gemm(F, g));
    }
    {   // u = Q2 s + q2
        GemmArgs g = gemm0();
        g.M = FNO_OUT; g.N = (int)P; g.K = FNO_H;
        g.A = th + OFF_Q2; g.am = FNO_H; g.ak = 1;
        g.B = F->f(L.s); g.bk = P; g.bn = 1;
        g.C = F->f(L.u); g.cm = P; g.cn = 1;
        g.bias = th + OFF_q2;
        CKS(gemm(F, g));
    }
    CKS(band_limit(F, F->f(L.u), F->f(L.y), FNO_OUT));
    F->have_forward = true;
    return REG_OK;
}

reg_status backward_impl(reg_fno* F, const float* th, const float* target, float* grad, double* loss) {
    const int n = F->n, S = F->S, B = F->B;
    const long P = F->P;
    const NetLayout& L = F->L;
    float *Y = F->f(L.Y), *Yp = F->f(L.Yp), *T = F->f(L.T), *O = F->f(L.O), *dZ = F->f(L.dZ);
    float *dy = F->f(L.dy), *dzq = F->f(L.dzq);
    CK(launch_fno_loss(B, (long)n * n, F->f(L.y), target, F->at<double>(L.sums), dy, loss, F->stream));
    CKS(band_limit_T(F, dy, F->f(L.du), FNO_OUT));
    dy = F->f(L.du);   // from here on: the gradient with respect to u
    // projection
    CKS(wgrad(F, FNO_OUT, FNO_H, dy, F->f(L.s), grad + OFF_Q2, FNO_H));
    CK(launch_rowsum(FNO_OUT, P, dy, F->at<double>(L.rsum), grad + OFF_q2, F->stream));
    {   // dzq = (Q2^T dy) * gelu'(zq)
        GemmArgs g = gemm0();
        g.M = FNO_H; g.N = (int)P; g.K = FNO_OUT;
        g.A = th + OFF_Q2; g.am = 1; g.ak = FNO_H;
        g.B = dy; g.bk = P; g.bn = 1;
        g.C = dzq; g.cm = P; g.cn = 1;
        g.act = ACT_GELU_BWD; g.aux = F->f(L.zq);
        CKS(gemm(F, g));
    }
    CKS(wgrad(F, FNO_H, FNO_C, dzq, F->f(L.h[FNO_L]), grad + OFF_Q1, FNO_C));
    CK(launch_rowsum(FNO_H, P, dzq, F->at<double>(L.rsum), grad + OFF_q1, F->stream));
    float* cur = F->f(L.dA);
    float* nxt = F->f(L.dB);
    {   // dh4 = Q1^T dzq (the last Fourier layer has no activation: this is dz_3)
        GemmArgs g = gemm0();
        g.M = FNO_C; g.N = (int)P; g.K = FNO_H;
        g.A = th + OFF_Q1; g.am = 1; g.ak = FNO_C;
        g.B = dzq; g.bk = P; g.bn = 1;
        g.C = cur; g.cm = P; g.cn = 1;
        CKS(gemm(F, g));
    }
    for (int l = FNO_L - 1; l >= 0; --l) {
        const float* dz = cur;
        CKS(wgrad(F, FNO_C, FNO_C, dz, F->f(L.h[l]), grad + off_W(l), FNO_C));
        CK(launch_rowsum(FNO_C, P, dz, F->at<double>(L.rsum), grad + off_B(l), F->stream));
        {   // dYp = dz . G2^T
            GemmArgs g = gemm0();
            g.M = S * n; g.N = 32; g.K = n;
            g.A = dz; g.am = n; g.ak = 1;
            g.B = F->f(L.G2); g.bk = 1; g.bn = n;
            g.C = Yp; g.cm = 32; g.cn = 1;
            CKS(gemm(F, g));
        }
        {   // dOb[s] = IC^T . dYp[s]
            GemmArgs g = gemm0();
            g.M = 64; g.N = 32; g.K = n; g.batch = S;
            g.A = F->f(L.IC); g.am = 1; g.ak = 64; g.ab = 0;
            g.B = Yp; g.bk = 32; g.bn = 1; g.bb = 32L * n;
            g.C = T; g.cm = 32; g.cn = 1; g.cb = 2048;
            CKS(gemm(F, g));
        }
        CK(launch_fno_fold_o(S, T, O, F->stream));   // O now holds dO
        {   // dWexp = Z^T . dO per mode
            GemmArgs g = gemm0();
            g.M = 64; g.N = 64; g.K = B; g.batch = FNO_MODES;
            g.A = F->f(L.Zs[l]); g.am = (long)B * FNO_MODES; g.ak = FNO_MODES; g.ab = 1;
            g.B = O; g.bk = FNO_MODES; g.bn = (long)B * FNO_MODES; g.bb = 1;
            g.C = F->f(L.dWexp); g.cm = 64; g.cn = 1; g.cb = 4096;
            CKS(gemm(F, g));
        }
        CK(launch_fno_fold_w(F->f(L.dWexp), grad + off_R(l), F->stream));
        {   // dZ = dO . Wexp^T per mode
            GemmArgs g = gemm0();
            g.M = B; g.N = 64; g.K = 64; g.batch = FNO_MODES;
            g.A = O; g.am = FNO_MODES; g.ak = (long)B * FNO_MODES; g.ab = 1;
            g.B = F->f(L.Wexp) + (long)l * FNO_MODES * 4096; g.bk = 1; g.bn = 64; g.bb = 4096;
            g.C = dZ; g.cm = FNO_MODES; g.cn = (long)B * FNO_MODES; g.cb = 1;
            CKS(gemm(F, g));
        }
        CK(launch_fno_uncombine(S, dZ, T, F->stream));   // T now holds dT
        {   // dY[s] = CS^T . dT[s]
            GemmArgs g = gemm0();
            g.M = n; g.N = 32; g.K = 64; g.batch = S;
            g.A = F->f(L.CS); g.am = 1; g.ak = n; g.ab = 0;
            g.B = T; g.bk = 32; g.bn = 1; g.bb = 2048;
            g.C = Y; g.cm = 32; g.cn = 1; g.cb = 32L * n;
            CKS(gemm(F, g));
        }
        {   // nxt = W^T dz
            GemmArgs g = gemm0();
            g.M = FNO_C; g.N = (int)P; g.K = FNO_C;
            g.A = th + off_W(l); g.am = 1; g.ak = FNO_C;
            g.B = dz; g.bk = P; g.bn = 1;
            g.C = nxt; g.cm = P; g.cn = 1;
            CKS(gemm(F, g));
        }
        {   // nxt += dY . F2^T, then times gelu'(z_{l-1}) below the first layer
            GemmArgs g = gemm0();
            g.M = S * n; g.N = n; g.K = 32;
            g.A = Y; g.am = 32; g.ak = 1;
            g.B = F->f(L.F2); g.bk = 1; g.bn = 32;
            g.C = nxt; g.cm = n; g.cn = 1;
            g.beta = 1.0f;
            if (l > 0) {
                g.act = ACT_GELU_BWD;
                g.aux = F->f(L.z[l - 1]);
            }
            CKS(gemm(F, g));
        }
        std::swap(cur, nxt);
    }
    CKS(wgrad(F, FNO_C, FNO_IN, cur, F->f(L.in), grad + OFF_WL, FNO_IN));
    CK(launch_rowsum(FNO_C, P, cur, F->at<double>(L.rsum), grad + OFF_BL, F->stream));
    return REG_OK;
}

reg_status adam_impl(reg_fno* F, float* params, const float* grad, float* m, float* v, int step, float lr, float b1,
                     float b2, float eps) {
    if (step < 1) return fail(REG_EINVAL, "Adam step number must be >= 1");
    if (!(lr >= 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps >= 0.0f))
        return fail(REG_EINVAL, "Adam hyper-parameters out of range");
    const double c1 = 1.0 / (1.0 - std::pow((double)b1, step));
    const double c2 = 1.0 / (1.0 - std::pow((double)b2, step));
    CK(launch_adam(N_PARAMS, params, grad, m, v, lr, b1, b2, eps, (float)c1, (float)c2, F->stream));
    return REG_OK;
}

// Truncated DFT matrices, entries from double-precision cos / sin of 2 pi ((k i) mod n) / n.
void make_bases(int n, std::vector<float>& F2, std::vector<float>& CS, std::vector<float>& IC, std::vector<float>& G2) {
    const int M = FNO_M;
    F2.assign((size_t)n * 32, 0.f);
    G2.assign((size_t)32 * n, 0.f);
    CS.assign((size_t)64 * n, 0.f);
    IC.assign((size_t)n * 64, 0.f);
    const double twopi = 6.283185307179586476925286766559;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < M; ++k) {
            const double ang = twopi * (double)(((long)k * i) % n) / n;
            const double w = k == 0 ? 1.0 : 2.0;
            F2[(size_t)i * 32 + k] = (float)(std::cos(ang) / n);
            F2[(size_t)i * 32 + M + k] = (float)(-std::sin(ang) / n);
            G2[(size_t)k * n + i] = (float)(w * std::cos(ang));
            G2[(size_t)(M + k) * n + i] = (float)(-w * std::sin(ang));
        }
    for (int j = 0; j < 2 * M; ++j) {
        const long k1 = j < M ? j : j - 2 * M;
        for (int i = 0; i < n; ++i) {
            const long km = ((k1 * i) % n + n) % n;
            const double ang = twopi * (double)km / n;
            CS[(size_t)j * n + i] = (float)(std::cos(ang) / n);
            CS[(size_t)(2 * M + j) * n + i] = (float)(std::sin(ang) / n);
            IC[(size_t)i * 64 + j] = (float)std::cos(ang);
            IC[(size_t)i * 64 + 2 * M + j] = (float)std::sin(ang);
        }
    }
}

reg_status check_handle(reg_fno* h) {
    if (!h) return fail(REG_EINVAL, "network handle is NULL");
    return REG_OK;
}

}  // namespace

extern "C" {

reg_status reg_fno_param_count(int64_t* count) {
    if (!count) return fail(REG_EINVAL, "count is NULL");
    *count = N_PARAMS;
    return REG_OK;
}

reg_status reg_fno_workspace_bytes(int32_t n, int32_t batch, size_t* bytes) {
    CKS(check_sizes(n, batch));
    if (!bytes) return fail(REG_EINVAL, "bytes is NULL");
    *bytes = net_layout(n, batch).total;
    return REG_OK;
}

reg_status reg_fno_create(int32_t n, int32_t batch, void* workspace, size_t workspace_bytes, void* hip_stream,
                          reg_fno** out) {
    CKS(check_sizes(n, batch));
    if (!out) return fail(REG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!workspace || ((uintptr_t)workspace & 255u)) return fail(REG_EINVAL, "workspace must be 256-byte aligned");
    const NetLayout L = net_layout(n, batch);
    if (workspace_bytes < L.total)
        return fail(REG_ENOMEM, "workspace of %zu bytes < %zu needed", workspace_bytes, L.total);
    reg_fno* F = new reg_fno;
    F->n = n;
    F->B = batch;
    F->S = FNO_C * batch;
    F->P = (long)batch * n * n;
    F->stream = (hipStream_t)hip_stream;
    F->base = (char*)workspace;
    F->L = L;
    std::vector<float> F2, CS, IC, G2;
    make_bases(n, F2, CS, IC, G2);
    auto up = [&](size_t off, const std::vector<float>& v) {
        return hipMemcpyAsync(F->base + off, v.data(), v.size() * sizeof(float), hipMemcpyHostToDevice, F->stream);
    };
    hipError_t e = up(L.F2, F2);
    if (e == hipSuccess) e = up(L.CS, CS);
    if (e == hipSuccess) e = up(L.IC, IC);
    if (e == hipSuccess) e = up(L.G2, G2);
    if (e == hipSuccess) e = hipStreamSynchronize(F->stream);
    if (e != hipSuccess) {
        delete F;
        return fail(REG_EDEVICE, "uploading DFT matrices failed: %s", hipGetErrorString(e));
    }
    *out = F;
    return REG_OK;
}

reg_status reg_fno_destroy(reg_fno* h) {
    delete h;
    return REG_OK;
}

static reg_status features_impl(reg_fno* h, const double* m_T, const double* m_R, float* out) {
    const long nn = (long)h->n * h->n;
    double* sq = h->at<double>(h->L.sq);
    CK(launch_sqdiff<double>(m_T, m_R, nn, h->at<double>(h->L.red), sq, h->stream));
    CK(launch_fno_features(h->n, m_T, m_R, sq, out, nn, h->stream));
    CK(launch_fno_scale(nn, sq, h->at<double>(h->L.scale), h->stream));
    return REG_OK;
}

reg_status reg_fno_features(reg_fno* h, const double* m_T, const double* m_R, float* out, double* scale) {
    CKS(check_handle(h));
    if (!m_T || !m_R || !out) return fail(REG_EINVAL, "NULL array");
    CKS(features_impl(h, m_T, m_R, out));
    if (scale) CK(hipMemcpyAsync(scale, h->at<double>(h->L.scale), sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    return REG_OK;
}

reg_status reg_fno_target(reg_fno* h, const double* v, const double* scale, const double* dirs, float* out) {
    CKS(check_handle(h));
    if (!v || !scale || !out) return fail(REG_EINVAL, "NULL array");
    CK(launch_fno_target((long)h->n * h->n, v, scale, dirs, out, h->stream));
    return REG_OK;
}

reg_status reg_fno_gather(reg_fno* h, const float* set, int64_t nset, int32_t channels, const int32_t* idx,
                          const int32_t* sym, float* out) {
    CKS(check_handle(h));
    if (!set || !idx || !out) return fail(REG_EINVAL, "NULL array");
    if (nset < 1 || channels < 1 || channels > 16) return fail(REG_EINVAL, "data set: nset >= 1, 1 <= channels <= 16");
    ChannelKinds kinds{};   // scalars unless the channel count names a known layout
    if (channels == FNO_IN) {
        const int k[FNO_IN] = {0, 1, 2, 3, 4, 5, 0, 1, 2};   // features: m_T, grad, tensor, r, r grad
        std::memcpy(kinds.k, k, sizeof k);
    } else if (channels == FNO_OUT || channels == 2) {
        for (int c = 0; c < channels; c += 2) {   // vector fields: the velocity, then the directions
            kinds.k[c] = 1;
            kinds.k[c + 1] = 2;
        }
    } else if (sym) {
        return fail(REG_EINVAL, "symmetry transforms need the feature (9), velocity (2) or output (%d) channel layout",
                    FNO_OUT);
    }
    CK(launch_fno_gather(set, nset, channels, h->n, idx, sym, kinds, h->B, out, h->stream));
    return REG_OK;
}

reg_status reg_fno_forward(reg_fno* h, const float* params, const float* in, float* out) {
    CKS(check_handle(h));
    if (!params || !in) return fail(REG_EINVAL, "NULL array");
    float* own = h->f(h->L.in);
    if (in != own) CK(hipMemcpyAsync(own, in, FNO_IN * h->P * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    CKS(forward_impl(h, params));
    if (out) CK(hipMemcpyAsync(out, h->f(h->L.y), FNO_OUT * h->P * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return REG_OK;
}

reg_status reg_fno_backward(reg_fno* h, const float* params, const float* target, float* grad, double* loss) {
    CKS(check_handle(h));
    if (!params || !target || !grad) return fail(REG_EINVAL, "NULL array");
    if (!h->have_forward) return fail(REG_ESTATE, "reg_fno_backward needs a reg_fno_forward on this handle first");
    return backward_impl(h, params, target, grad, loss);
}

reg_status reg_fno_adam(reg_fno* h, float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                        float beta1, float beta2, float eps) {
    CKS(check_handle(h));
    if (!params || !grad || !m || !v) return fail(REG_EINVAL, "NULL array");
    return adam_impl(h, params, grad, m, v, step, lr, beta1, beta2, eps);
}

reg_status reg_fno_train_step(reg_fno* h, float* params, const float* in, const float* target, float* grad, float* m,
                              float* v, int32_t step, float lr, double* loss) {
    CKS(reg_fno_forward(h, params, in, nullptr));
    CKS(reg_fno_backward(h, params, target, grad, loss));
    return reg_fno_adam(h, params, grad, m, v, step, lr, 0.9f, 0.999f, 1e-8f);
}

reg_status reg_fno_predict(reg_fno* h, const float* params, const double* m_T, const double* m_R, double* v0,
                           double* dirs) {
    CKS(check_handle(h));
    if (h->B != 1) return fail(REG_EINVAL, "reg_fno_predict needs a handle with batch 1");
    if (!params || !m_T || !m_R || !v0) return fail(REG_EINVAL, "NULL array");
    CKS(features_impl(h, m_T, m_R, h->f(h->L.in)));
    CKS(forward_impl(h, params));
    CK(launch_fno_unscale(h->P, h->f(h->L.y), h->at<double>(h->L.scale), v0, dirs, h->stream));
    return REG_OK;
}

}  // extern "C"
