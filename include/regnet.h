/* regnet.h -- C ABI of the learned warm start of the gfx950 registration library (libregnk.so).
 *
 * A Fourier neural operator (Li et al., "Fourier neural operator for parametric partial
 * differential equations", ICLR 2021) maps an image pair (m_T, m_R) to a velocity field that the
 * Gauss-Newton solve of Alg. 1 takes as its initial iterate v_0 (reg_solve_opts.v0 in regnk.h), and
 * to REG_FNO_RANK direction fields for the low-rank correction of the PCG preconditioner
 * (reg_solve_opts.precond_U, an extension: the balancing correction built by Rayleigh-Ritz on their
 * span).  Their training targets are the leading generalised eigenvectors of (H, M) at the solved
 * velocity (reg_ritz_directions in regnk.h).
 * The solver always judges it: the relative gradient is measured against ||g(0)|| and a warm start
 * whose objective is not below J(0) is dropped (Sec. 4 globalisation: the line search needs descent).
 *
 * Network (fixed sizes): input features a = [m_T, D1 m_T, D2 m_T, (D1 m_T)^2, D1 m_T D2 m_T,
 * (D2 m_T)^2, r, r D1 m_T, r D2 m_T] (D = periodic central difference, h = 2 pi / n) with the
 * normalised misfit r = (m_R - m_T) / s, s = sqrt(mean((m_R - m_T)^2)) (r = 0 if s = 0).  The
 * velocity is linear in the misfit to first order, so the network predicts v / s and the warm
 * start is v0 = s y.  Lifting 9 -> 32; four Fourier layers
 * z = W h + b + S h with S h = Re( sum_k w(k2) O(k) e^{i k.x} ), O(k) = H(k) R(k) over the retained
 * wavenumbers k1 in {0..15, -16..-1}, k2 in {0..15} (H = Fourier coefficients n^-2 sum h e^{-ik.x};
 * w(0) = 1 keeping only the real part of the k2 = 0 column, w(k2 > 0) = 2), GELU (exact, erf form)
 * after the first three layers; projection 32 -> 64 (GELU) -> REG_FNO_OUT, band-limited to the retained modes
 * with |k| <= 12 (S with identity weights on that disc, zero on the corners of the square) so that
 * the velocity has no energy where the solutions have none and the H2 regulariser would weight by
 * |k|^4; this fixed filter runs in FP32.  Every other matrix product runs on
 * the matrix cores with operands rounded to bfloat16 (nearest even) and FP32 accumulation; all
 * other arithmetic is FP32.  Output channels: y[0], y[1] = v / s; y[2 + 2k], y[3 + 2k] = direction k
 * (k < REG_FNO_RANK), defined up to sign and scale.  Loss over a batch, with Euclidean sums:
 *   (1/B) sum_b [ ||y_b - t_b||^2 / ||t_b||^2 over the velocity channels
 *     + (REG_FNO_DIR_WEIGHT / REG_FNO_RANK) sum_k (1 - <t_bk, y_bk>^2 / (||t_bk||^2 max(||y_bk||^2, 1e-30))) ],
 * a direction slot whose target is zero contributing nothing.
 *
 * Parameters: one flat float array of REG_FNO_PARAMS entries, in this order:
 *   Wl[32][9], bl[32];  for each of the 4 layers: Rr[32][16][32][32], Ri[32][16][32][32], W[32][32],
 *   b[32];  Q1[64][32], q1[64], Q2[REG_FNO_OUT][64], q2[REG_FNO_OUT].
 *   R index order [k1 row j][k2][c_in][c_out], k1 = j for j < 16 and j - 32 otherwise.
 * Batched arrays are channel-major: x[c][b][i1][i2].  All arrays are device arrays owned by the
 * caller; every call enqueues on the handle's stream and returns without synchronising, except
 * where stated.  Grid sizes: n a power of two in [32, 1024]; batch in [1, 64].
 */
#ifndef REGNET_H
#define REGNET_H

#include <stddef.h>
#include <stdint.h>

#include "regnk.h"

#ifdef __cplusplus
extern "C" {
#endif

#define REG_FNO_RANK 4        /* direction fields of the low-rank head */
#define REG_FNO_OUT 10        /* output channels: 2 (velocity) + 2 REG_FNO_RANK */
#define REG_FNO_DIR_WEIGHT 0.1
#define REG_FNO_PARAMS 4201610

typedef struct reg_fno reg_fno;   /* opaque handle: one grid size and batch size */

/* *count = REG_FNO_PARAMS (host only). */
reg_status reg_fno_param_count(int64_t* count);

/* Bytes of device workspace for a handle of grid n x n and `batch` samples (host only). */
reg_status reg_fno_workspace_bytes(int32_t n, int32_t batch, size_t* bytes);

/* Create a handle in caller-owned device workspace (256-byte aligned, at least
 * reg_fno_workspace_bytes bytes, kept alive until reg_fno_destroy).  Uploads the truncated DFT
 * matrices of the grid and synchronises the stream.  The library allocates no device memory. */
reg_status reg_fno_create(int32_t n, int32_t batch, void* workspace, size_t workspace_bytes, void* hip_stream,
                          reg_fno** out);
reg_status reg_fno_destroy(reg_fno* h);

/* Input features of one pair: out[9][n][n] (float) from the FP64 fields m_T, m_R [n][n]; the misfit
 * scale s goes to *scale (device double, nullable). */
reg_status reg_fno_features(reg_fno* h, const double* m_T, const double* m_R, float* out, double* scale);

/* Training target of one pair, out[REG_FNO_OUT][n][n] (float): channels 0, 1 = v / s for a solved
 * velocity v [2][n][n] (FP64) and the pair's misfit scale s (device double from reg_fno_features;
 * zeros if s = 0); channels 2.. = dirs[REG_FNO_RANK][2][n][n] (FP64, nullable: zeros, which the loss
 * skips). */
reg_status reg_fno_target(reg_fno* h, const double* v, const double* scale, const double* dirs, float* out);

/* Gather a batch from a data set stored sample-major (set[nset][channels][n][n]) into
 * out[channels][batch][n][n]: sample b is set[idx[b]] (device int32[batch]; an index outside [0, nset)
 * yields zeros) mapped by the grid symmetry sym[b] (device int32[batch], nullable = identity): bit 0
 * swaps the axes, bit 1 / bit 2 flip axis 1 / 2 (i -> (n - i) mod n).  The discrete problem is
 * invariant under these 8 maps, so they augment the training set exactly; the 9 feature channels
 * and the velocity and direction channels transform as scalars, vectors (v' = F P v) and the
 * symmetric tensor (S' = F P S P F) they are.  With sym, channels must be 9 (features), 2 (a
 * velocity) or REG_FNO_OUT (targets). */
reg_status reg_fno_gather(reg_fno* h, const float* set, int64_t nset, int32_t channels, const int32_t* idx,
                          const int32_t* sym, float* out);

/* Network output for a batch: in[9][batch][n][n] -> out[REG_FNO_OUT][batch][n][n] (out nullable).
 * Keeps the activations for reg_fno_backward. */
reg_status reg_fno_forward(reg_fno* h, const float* params, const float* in, float* out);

/* Loss against target[REG_FNO_OUT][batch][n][n] and its gradient with respect to the parameters (grad: float
 * [REG_FNO_PARAMS], overwritten) for the batch and parameters of the last reg_fno_forward on this
 * handle (REG_ESTATE if there was none).  loss: device double, nullable. */
reg_status reg_fno_backward(reg_fno* h, const float* params, const float* target, float* grad, double* loss);

/* One Adam step (Kingma and Ba, ICLR 2015) at step number `step` >= 1 over all parameters:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
reg_status reg_fno_adam(reg_fno* h, float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                        float beta1, float beta2, float eps);

/* forward + backward + Adam on one batch (the three calls above in sequence). */
reg_status reg_fno_train_step(reg_fno* h, float* params, const float* in, const float* target, float* grad,
                              float* m, float* v, int32_t step, float lr, double* loss);

/* Warm start for one pair (a handle with batch 1): v0[2][n][n] (FP64) = s y[0:2] with
 * y = network(features(m_T, m_R)); dirs (nullable) [REG_FNO_RANK][2][n][n] (FP64) = y[2:], the
 * directions to pass as reg_solve_opts.precond_U. */
reg_status reg_fno_predict(reg_fno* h, const float* params, const double* m_T, const double* m_R, double* v0,
                           double* dirs);

#ifdef __cplusplus
}
#endif

#endif /* REGNET_H */
