// Device kernels of the warm-start network (a Fourier neural operator): a batched bfloat16 MFMA
// GEMM with FP32 accumulation and fused epilogues, and the small elementwise kernels around it.
//
// Layouts.  Activations are channel-major over the whole batch: x[c][b][i1][i2] (P = B n^2
// positions per channel), so pointwise channel mixing is one GEMM with N = P and weight gradients
// are one long-K GEMM.  Truncated spectra of slice s = c B + b are kept in the layouts given at
// each kernel below; mode = j * 16 + k2 with k1 row j (k1 = j for j < 16, j - 32 otherwise).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace regnk {

constexpr int FNO_C = 32;        // width
constexpr int FNO_M = 16;        // retained modes per axis (k1 rows: 2M, k2 columns: M)
constexpr int FNO_MODES = 2 * FNO_M * FNO_M;   // 512 retained (k1, k2) pairs
constexpr int FNO_L = 4;         // Fourier layers
constexpr int FNO_IN = 9;
constexpr int FNO_RANK = 4;                    // direction fields of the low-rank head
constexpr int FNO_OUT = 2 + 2 * FNO_RANK;      // channels 0, 1: v / s; 2 + 2k, 3 + 2k: direction k
constexpr double FNO_DIR_WEIGHT = 0.1;         // weight of the direction terms in the loss
constexpr int FNO_H = 64;        // projection width
constexpr int FNO_RADIUS = 12;   // output band: retained modes with |k| <= 12

enum GemmAct { ACT_NONE = 0, ACT_GELU = 1, ACT_GELU_BWD = 2 };

// C[b](m, n) = epilogue(alpha * sum_k A[b](m, k) B[b](k, n)), element (m, k) of A[b] at
// A + b ab + m am + k ak (likewise B, C).  Operands are FP32 in memory, rounded to bfloat16 (nearest
// even) when staged, multiplied by MFMA with FP32 accumulation.  Epilogue, in this order:
// + beta C (if beta != 0), + bias[m] (nullable), + add[b](m, n) (nullable), Z = value (nullable,
// C's strides), then ACT_GELU: gelu(value) or ACT_GELU_BWD: value * gelu'(aux) (aux with C's
// strides), stored to C.  With f32 = 1 the operands keep FP32 and the product runs as FP32 FMAs
// (for fixed filters whose data would lose precision in bfloat16).  With part != NULL (batch must be 1) K is cut into ksplit >= 1 chunks
// whose raw sums go to part[ks][M][N] and C is not touched; launch_splitk_reduce then forms
// C = alpha sum + beta C.  ksplit > 1 requires part.
struct GemmArgs {
    int M, N, K, batch;
    const float* A;
    long am, ak, ab;
    const float* B;
    long bk, bn, bb;
    float* C;
    long cm, cn, cb;
    float alpha, beta;
    const float* bias;
    const float* add;
    long dm, dn, db;
    float* Z;
    const float* aux;
    int act;
    int ksplit;
    int kchunk;          // set by launch_gemm
    float* part;
    int avec, bvec;      // set by launch_gemm: 16-byte vector loads allowed
    int f32;             // 1: FP32 multiplicands on the vector ALUs (no bfloat16 rounding)
};

// Writes the effective ksplit (<= the requested one) back into g.
hipError_t launch_gemm(GemmArgs& g, hipStream_t s);
// C(m, n) = alpha * sum_s part[s][m][n] + beta * C(m, n), fixed summation order
hipError_t launch_splitk_reduce(int ksplit, int M, int N, const float* part, float alpha, float beta, float* C,
                                long cm, long cn, hipStream_t s);

// ---- elementwise and reductions ---------------------------------------------------------------
// 9 input channels of one pair: out[c * cstride + i] = m_T, D1 m_T, D2 m_T, (D1 m_T)^2, D1 m_T D2 m_T,
// (D2 m_T)^2, r, r D1 m_T, r D2 m_T (periodic central differences, h = 2 pi / n; r = (m_R - m_T) / s,
// s = sqrt(2 sq / n^2) from sq = 1/2 sum (m_R - m_T)^2 (device), r = 0 if s = 0)
hipError_t launch_fno_features(int n, const double* mT, const double* mR, const double* sq, float* out, long cstride,
                               hipStream_t s);
// scale[0] = s = sqrt(2 sq / nn)
hipError_t launch_fno_scale(long nn, const double* sq, double* scale, hipStream_t s);
// training target of one pair, out[FNO_OUT][nn]: channels 0, 1 = v / s (0 if s = 0); channels 2.. =
// dirs[k][2][nn] as float (zeros if dirs is NULL)
hipError_t launch_fno_target(long nn, const double* v, const double* scale, const double* dirs, float* out,
                             hipStream_t s);
// v[i] = s y[i], i < 2 nn (warm start from the normalised network output); dirs (nullable) = the
// direction channels y[2 nn ..] widened to double
hipError_t launch_fno_unscale(long nn, const float* y, const double* scale, double* v, double* dirs, hipStream_t s);
// out[c][b][p] = set[idx[b]][c'][q] for 0 <= idx[b] < nset (zeros otherwise), where sym[b] (nullable:
// identity) is a symmetry of the periodic square grid: bit 0 swaps the axes, bits 1 and 2 flip axis
// 1 and 2 (i -> (n - i) mod n); output point i reads source point P(F(i)).  kind[c] says how channel c
// transforms: 0 scalar, 1 / 2 first / second component of a vector (v' = F P v), 3 / 4 / 5 entries
// (11) / (12) / (22) of a symmetric tensor (S' = F P S P F).
struct ChannelKinds {
    int k[16];
};
hipError_t launch_fno_gather(const float* set, long nset, int channels, int n, const int32_t* idx,
                             const int32_t* sym, ChannelKinds kinds, int count, float* out, hipStream_t s);
// zero the retained coefficients outside the disc |k| <= radius (Z[2][S][mode])
hipError_t launch_fno_mask_disc(int S, float* Z, int radius, hipStream_t s);
// Z[ri][s][mode] (S slices) from T[s][64][32]: Zr = T[j][k2] + T[32+j][16+k2], Zi = T[j][16+k2] - T[32+j][k2]
hipError_t launch_fno_combine(int S, const float* T, float* Z, hipStream_t s);
// dT[s][64][32] = [[dZr, dZi], [-dZi, dZr]] (the transpose of combine)
hipError_t launch_fno_uncombine(int S, const float* dZ, float* dT, hipStream_t s);
// Ob[s][64][32] = [[Or, Oi], [-Oi, Or]] from O[ri][s][mode]
hipError_t launch_fno_expand_o(int S, const float* O, float* Ob, hipStream_t s);
// dO[ri][s][mode] from dOb[s][64][32]: dOr = dOb[j][k2] + dOb[32+j][16+k2], dOi = dOb[j][16+k2] - dOb[32+j][k2]
hipError_t launch_fno_fold_o(int S, const float* dOb, float* dO, hipStream_t s);
// W[mode][64][64] = [[Rr, Ri], [-Ri, Rr]] for `layers` consecutive parameter blocks (stride lstride)
hipError_t launch_fno_expand_w(int layers, const float* R, long lstride, float* W, hipStream_t s);
// dRr = dW[c][o] + dW[32+c][32+o], dRi = dW[c][32+o] - dW[32+c][o] into grad (Rr block then Ri block)
hipError_t launch_fno_fold_w(const float* dW, float* gR, hipStream_t s);
// out[r] = sum_i x[r * len + i]: RS_CHUNKS blocks per row write FP64 partial sums to part
// (rows * RS_CHUNKS doubles), a second pass adds them in a fixed order
constexpr int RS_CHUNKS = 64;
hipError_t launch_rowsum(int rows, long len, const float* x, double* part, float* out, hipStream_t s);
// Loss of a batch (layout [FNO_OUT][B][npos]): per sample b the relative squared error of the two
// velocity channels, num_b / den_b, plus (FNO_DIR_WEIGHT / FNO_RANK) sum_k (1 - c^2 / (a max(bb, 1e-30)))
// over the direction slots k with a = ||t_k||^2 > 0 (bb = ||y_k||^2, c = <t_k, y_k>).  sums holds
// 3 (1 + FNO_RANK) B doubles; dy = dL/dy; loss = L (device double, nullable), averaged over B.
constexpr int FNO_LOSS_SUMS = 3 * (1 + FNO_RANK);
hipError_t launch_fno_loss(int B, long npos, const float* y, const float* t, double* sums, float* dy, double* loss,
                           hipStream_t s);
// Adam with bias corrections c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t)
hipError_t launch_adam(long n, float* p, const float* g, float* m, float* v, float lr, float beta1, float beta2,
                       float eps, float c1, float c2, hipStream_t s);

}  // namespace regnk
