// Declarations shared by the device kernels and the host driver of the registration library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mr_plan.hpp"

namespace regnk {

template <typename T>
struct cpx;

// Transport stage operations (see transport_kernels.hpp for the formulas).
// OP_A1F / OP_A2F: the incremental adjoint stages of the full-Newton Hessian (flux v lam~ + v~ lam
// and the lam grad m~ body-force terms); they take the launch shapes tuned for OP_A1 / OP_A2.
enum PassOp { OP_S1 = 0, OP_S2, OP_A1, OP_A2, OP_I1, OP_I2, OP_GRAD, OP_A1F, OP_A2F };
constexpr int NUM_TUNED_OPS = 7;
constexpr int op_base(int op) { return op == OP_A1F ? OP_A1 : (op == OP_A2F ? OP_A2 : op); }
// F_PHASES (timing only, with clk): four stamps per block instead of two (see transport_kernels.hpp).
enum PassFlags { F_ZERO = 1, F_FIRST = 2, F_NEG = 4, F_PHASES = 8 };

// One RK2 stage: input u = A + Bf (Bf nullable; negated with F_NEG; with F_ZERO u = -h v~ . G2).
// Row blocks write ROUT (and UOUT = u, gradient component 1, body force); column blocks write COUT
// (and gradient component 0).  The stage result is ROUT + COUT.
template <typename T>
struct StageArgs {
    int n1, n2;
    long nn;                 // n1 * n2
    T h;                     // time step 1/n_t
    T bw;                    // body-force quadrature weight
    int flags;
    const T* A;
    const T* Bf;
    const T* V1;             // velocity component 1 (column transforms)
    const T* V2;             // velocity component 2 (row transforms)
    const T* X;              // previous-stage field for the RK2 combination (m_j, l_{j+1}, m~_j)
    const T* VT;             // v~ (vector field)
    const T* G;              // stored gradient (vector field)
    const T* G2;             // second stored gradient (vector field)
    const T* LAM;            // full Newton: stored adjoint at the stage (lam_{j+1} in stage 1, lam*_j in 2)
    const T* LAM2;           // full Newton, stage 2: lam_{j+1}
    const T* GT;             // full Newton, stage 2: grad m~_j (vector field; nullable = 0)
    const T* GT2;            // full Newton, stage 2: grad m~*_j (vector field)
    T* ROUT;
    T* UOUT;
    T* COUT;
    T* GOUT;                 // grad of the stage input (state and incremental-state stages; vector field)
    float* GOUTF;            // same, rounded to FP32 (FP64 state solve feeding an FP32 trajectory)
    T* B;                    // body-force accumulator (vector field)
    const cpx<T>* tw1;       // twiddles of length n1 (column transforms)
    const cpx<T>* tw2;       // twiddles of length n2 (row transforms)
    const T* dc1;            // axis lengths that are not powers of two: the circulant spectral
    const T* dc2;            // derivative along x1 / x2 (length n1 / n2), else unused
    MrPlan mr1, mr2;         // mixed-radix plans of the two axis lengths (ns = 0: power of two, or a
                             // length with another prime factor, which takes the circulant)
    unsigned long long* clk; // timing (nullable): block b stores its start / end (device wall clock)
                             // to clk[2b], clk[2b+1]; a stage has at most (n1 + n2) / 2 blocks.
                             // With F_PHASES: clk[4b .. 4b+3] = start, loads arrived, transforms
                             // done, stores acknowledged (one-launch FP32 Gauss-Newton stages of
                             // square grids; the others leave the middle two at their initial values)
};
// clk[2 i] = ~0, clk[2 i + 1] = 0 for i < pairs (before timed stages)
hipError_t launch_clk_init(unsigned long long* clk, int pairs, hipStream_t s);

constexpr int NUM_STAGE_VARIANTS = 20;
// var: launch-shape variant (0 = default; see transport_kernels.hpp).  FP32 stages exist for the
// matvec ops (OP_A1, OP_A2, OP_I1, OP_I2); the state ops run in FP64.
// t0 / t1 (nullable): events stamped by the dispatch itself at the stage's start and end (timing).
template <typename T>
hipError_t launch_stage(int op, int var, const StageArgs<T>& a, hipStream_t s, hipEvent_t t0 = nullptr,
                        hipEvent_t t1 = nullptr);
// Whether FP32 launch shape `var` is a distinct, valid shape on an n1 x n2 grid (other indices fall
// back to a valid default, or the grid has one fixed shape).
bool stage_variant_fits_f32(int n1, int n2, int var);
// m1 = Q + C (FP64); lam (nullable) = m_R - m1 in precision T
template <typename T>
hipError_t launch_finalize_state(long nn, const double* Q, const double* C, const double* mR, double* m1, T* lam,
                                 hipStream_t s);
// B += w (Q + C) G (vector fields B, G)
template <typename T>
hipError_t launch_body_end(long nn, T w, const T* Q, const T* C, const T* G, T* B, hipStream_t s);
// Last Gauss-Newton adjoint step of the exact-transpose quadrature (lam_0 not formed):
// B = (first ? 0 : B) + w ((Q + C) G + X G2), keep (nullable) = Q + C
template <typename T>
hipError_t launch_body_last(long nn, T w, bool first, const T* Q, const T* C, const T* X, const T* G, const T* G2,
                            T* B, T* keep, hipStream_t s);

// ---- 2D spectral operators (FP64) -----------------------------------------------------------
// SPEC_LR: first result = admissible part of x (Leray projection for w = 0, x otherwise), second
// result = K^{-1} P^ of that part (the preconditioner operator, weighted for <., .>_W).
// SPEC_HESS_P: SPEC_HESS and the preconditioner (beta_v A)^{-1} of its result, for the PCG
// recurrence of P^{-1} r: with want2 fields 0..2 = H x, K^{-1} H x, P^{-1} H x (spec holds 6 half
// spectra), without it fields 0, 1 = H x, P^{-1} H x.  Column lengths 64..512 only
// (spec_col_hess_p_ok).
enum SpecMode { SPEC_PROJ = 0, SPEC_HESS, SPEC_PREC, SPEC_REG, SPEC_LR, SPEC_HESS_P };
inline bool spec_col_hess_p_ok(int n1, int n2) {
    return (n1 & (n1 - 1)) == 0 && n1 >= 64 && n1 <= 512 && (n2 & (n2 - 1)) == 0;
}

struct SpecParams {
    int n1, n2;
    int norm;                // 1 = H1, 2 = H2, 3 = H3, 4 = shear-control model (its regularisation
                             // term is formed in real space; the multipliers project it with K and
                             // precondition with the vector Laplacian)
    int constraint;          // 0 none, 1 divfree, 2 mass source
    double beta_v, beta_w;
    MrPlan mr1, mr2;         // mixed-radix plans of n1, n2 (used for lengths that are not powers of two)
    const double* eta_sum;   // shear-control model with a mass source: device sum of the viscosity
                             // at the point of K (its mean eta_bar = sum / (n1 n2) enters M)
};

// Forward row pass: real vector fields -> half spectra (k2 < n2/2) in spec[field][comp][n1][n2/2].
// in1 may be null (one field).  TI = float or double.
template <typename TI>
hipError_t launch_spec_row_fwd(const SpecParams& p, const TI* in0, const TI* in1, cpx<double>* spec,
                               const cpx<double>* tw2, hipStream_t s);
// The same with two input types (field 0 from in0, field 1 from in1); instantiated for
// (double, float) and through launch_spec_row_fwd for equal types.
template <typename TI0, typename TI1>
hipError_t launch_spec_row_fwd2(const SpecParams& p, const TI0* in0, const TI1* in1, cpx<double>* spec,
                                const cpx<double>* tw2, hipStream_t s);
// The last adjoint step's body-force term (see launch_body_last) deferred to the assembly: the
// body force entering the transform is (first ? 0 : B) + w ((Q + C) G + X G2) (G, G2 vector fields).
template <typename T>
struct BodyLast {
    const T *Q, *C, *X, *G, *G2;   // Q == nullptr: nothing deferred
    T w;
    int first;
};
// launch_spec_row_fwd2 with field 1 = the body force B completed by `bl` on the fly (B is read, not
// written; power-of-two n2 fuse the term into the row pass, other lengths run launch_body_last
// first and then leave the completed body force in B).
template <typename T>
hipError_t launch_spec_row_fwd_body(const SpecParams& p, const double* in0, T* B, const BodyLast<T>& bl,
                                    cpx<double>* spec, const cpx<double>* tw2, hipStream_t s);
// Column pass: forward FFT along x1 of the needed spectra, Fourier multiplier of `mode`, inverse
// FFT; in place in spec (outputs: field 0 = first result, field 1 = second result if want2).
hipError_t launch_spec_col(const SpecParams& p, int mode, bool have_y, bool want2, cpx<double>* spec,
                           const cpx<double>* tw1, hipStream_t s);
// Inverse row pass: fields 0 and 1 of spec -> real vector fields out0 and out1 (out1 nullable: field
// 0 only) in one launch.
hipError_t launch_spec_row_inv2(const SpecParams& p, const cpx<double>* spec, double* out0, double* out1,
                                const cpx<double>* tw2, hipStream_t s);
// The same pass forming partial sums of <s, out_field> (field 0: out0, 1: out1; both components)
// while it writes: partial[b] for the rows of block b, in a fixed order; *count receives the number
// of partials (0 where the pass for this length does not form them: the caller then sums itself).
struct RowDot {
    const double* s;
    int field;
    double* partial;
    int* count;
};
hipError_t launch_spec_row_inv2_dot(const SpecParams& p, const cpx<double>* spec, double* out0, double* out1,
                                    const cpx<double>* tw2, const RowDot& d, hipStream_t s);
// The inverse row pass of fields 0..nf-1 (nf <= 4) into out[0..nf-1] in one launch (power-of-two n2),
// with the partial sums of `d`.
hipError_t launch_spec_row_inv4_dot(const SpecParams& p, const cpx<double>* spec, double* const* out, int nf,
                                    const cpx<double>* tw2, const RowDot& d, hipStream_t s);

// Nyquist projection of a real vector field in real space (every mode with k1 = n1/2 or k2 = n2/2
// removed): out_d (double, nullable), out_t (TO, nullable); `in` may equal out_d.  scratch: at
// least nyquist_scratch_doubles(n1, n2) doubles.
template <typename TO>
hipError_t launch_nyquist_project(int n1, int n2, const double* in, double* out_d, TO* out_t, double* scratch,
                                  hipStream_t s);
size_t nyquist_scratch_doubles(int n1, int n2);

// ---- FP64 reductions and vector updates -------------------------------------------------------
constexpr int RED_BLOCKS = 512;
constexpr int RED_THREADS = 256;
// out[k] = sum_i a_k[i] * b_k[i] for k < nk (nk <= 4), deterministic; partial: nk * RED_BLOCKS.
template <typename TI>
hipError_t launch_dots(int nk, const TI* const* a, const TI* const* b, long n, double* partial,
                       double* out, hipStream_t s);
// out = 1/2 sum (x - y)^2 (data misfit), deterministic
template <typename TI>
hipError_t launch_sqdiff(const TI* x, const TI* y, long n, double* partial, double* out, hipStream_t s);
// y = alpha * x + beta * y   (double)
hipError_t launch_axpby(long n, double alpha, const double* x, double beta, double* y, hipStream_t s);
// z = x + alpha * y  (double), z may alias x
hipError_t launch_add_scaled(long n, const double* x, double alpha, const double* y, double* z,
                             hipStream_t s);
// out_t = (TO) in_d
template <typename TO>
hipError_t launch_convert(long n, const double* in, TO* out, hipStream_t s);
// out_d = (double) in_t
template <typename TI>
hipError_t launch_widen(long n, const TI* in, double* out, hipStream_t s);
hipError_t launch_fill(long n, double v, double* y, hipStream_t s);

// ---- low-rank deflation correction of the PCG preconditioner ------------------------------------
// A set of vector fields holds slot k at F + k * stride.  cnt points to the number of valid slots
// (a device double), so captured launch graphs stay valid while the set grows.
constexpr int LR_MAX = 64;       // most directions a correction holds
constexpr int LR_MIX_MAX = 8;    // most caller directions (Rayleigh-Ritz basis)
struct LrMix {
    double m[LR_MIX_MAX][LR_MIX_MAX];   // out_j = sum_i m[i][j] in_i
};
// out[k] = sum_i x[i] F_k[i] for k < *cnt (deterministic); partial: cap * RED_BLOCKS doubles
hipError_t launch_lr_dots(long n, const double* x, const double* F, long stride, const double* cnt, int cap,
                          double* partial, double* out, hipStream_t s);
// out = base + sign * sum_{k < *cnt} (da[k] - db[k]) / e[k] * F_k   (db nullable = 0; out may alias base)
// (*cnt is clamped to [0, cap] in both kernels)
hipError_t launch_lr_combine(long n, const double* base, double* out, const double* F, long stride,
                             const double* cnt, int cap, const double* da, const double* db, const double* e,
                             double sign, hipStream_t s);
// in place: F_j <- sum_{i < rin} m[i][j] F_i for j < rout (rin, rout <= LR_MIX_MAX)
hipError_t launch_lr_mix(long n, double* F, long stride, int rin, int rout, const LrMix& m, hipStream_t s);

// ---- nonlinear Stokes (shear-control) regularisation, FP64 ---------------------------------------
// dv: the four partials d_l v_i at (2 i + l) * nn.  sig, E: 3 fields (11, 12, 22); eta, dens: 1 field.
hipError_t launch_stokes_first(long nn, const double* dv, double nu, double eps, double* sig, double* E, double* eta,
                               double* dens, hipStream_t s);
hipError_t launch_stokes_second(long nn, const double* dvt, const double* E, const double* eta, double nu, double eps,
                                double* sig, hipStream_t s);
// out (vector) = scale * div sigma from ds = (grad s11, grad s12, grad s22)
hipError_t launch_stokes_div(long nn, const double* ds, double scale, double* out, hipStream_t s);

// ---- deformation diagnostics (eqs. (displacement), (def-grad)) -----------------------------------
// Components c = 0..5: u_1, u_2, F_11, F_12, F_21, F_22.
struct DefPtrs {
    const double* a[4];   // F_11, F_12, F_21, F_22 at the stage (first part)
    const double* b[4];   // second part of an R + C pair (nullable)
    double* out[6];       // R parts that receive w * source
};
struct DefPairs {
    const double* r[6];
    const double* c[6];
};
// out_c += w * S_c with S_{u_i} = v_i, S_{F_ik} = sum_l dv[i][l] F_lk; v: vector field, dv: 4 fields
// (dv[i][l] = d_l v_i at (2 i + l) * nn)
hipError_t launch_deform_source(long nn, double w, const double* v, const double* dv, const DefPtrs& p,
                                hipStream_t s);
// q_c = r_c + c_c; u1 = (q_0, q_1) and F1 = (q_2..q_5) (both nullable); det = q_2 q_5 - q_3 q_4
hipError_t launch_deform_final(long nn, const DefPairs& p, double* u1, double* F1, double* det, hipStream_t s);
// out3 = {min, max, sum} of x (deterministic); partial: 3 * RED_BLOCKS doubles
hipError_t launch_minmaxsum(const double* x, long n, double* partial, double* out3, hipStream_t s);

// ---- PCG with device-side scalars (Alg. 2) ----------------------------------------------------
// Slots of the FP64 scalar array shared by the PCG kernels.
enum PcgSlot {
    S_RZ = 0,    // <r, z>_W of the current iterate
    S_RR0,       // ||r_0||^2 (written next to S_RZ by the start-up dots)
    S_SHS,       // <s, H s>_W
    S_RR,        // ||r||^2 after the update
    S_RZN,       // <r, z>_W after the update (written next to S_RR)
    S_KAPPA,
    S_MU,
    S_ACTIVE,    // 1 while iterating, 0 after a breakdown (<s, H s> <= 0 or not finite)
    S_BREAK,     // iteration at which the breakdown happened (0: none)
    S_ITER,      // iterations executed
    NUM_PCG_SLOTS
};
enum PcgScalarMode { PCG_INIT = 0, PCG_KAPPA, PCG_MU };
// Second level of `nk` sums of `count` partials each (partial[k * count + i]) and the PCG scalar step
// `mode` (out = sc + slot), one block.
hipError_t launch_finalize_scalar(int nk, int count, const double* partial, double* out, int mode, double* scal,
                                  hipStream_t s);
// launch_dots (FP64) followed by the PCG scalar step `mode`, the latter fused into the second level.
hipError_t launch_dots_scalar(int nk, const double* const* a, const double* const* b, long n, double* partial,
                              double* out, int mode, double* scal, hipStream_t s);
// x += kappa s, r -= kappa s~ (kappa from scal)
hipError_t launch_pcg_update(long n, double* x, double* r, const double* s, const double* st, const double* scal,
                             hipStream_t stream);
// The same, and while the iteration is active z -= kappa pst (pst = P^{-1} s~: the preconditioned
// residual by recurrence) and kr -= kappa kst (kst = K^{-1} s~: the weighted residual; kr, kst
// nullable together); partial (2 * RED_BLOCKS) receives the block sums of ||r||^2 and <r, z>_W over
// the updated vectors, those of launch_dots with a = {r, kr or r}, b = {r, z}.
hipError_t launch_pcg_update_z(long n, double* x, double* r, const double* s, const double* st, double* z,
                               const double* pst, double* kr, const double* kst, const double* scal, double* partial,
                               hipStream_t stream);
// s = z + mu s (scal == nullptr: s = z) and its copy sT = (T) s for the next matvec
template <typename T>
hipError_t launch_pcg_dir_copy(long n, double* s, T* sT, const double* z, const double* scal, hipStream_t stream);

}  // namespace regnk
