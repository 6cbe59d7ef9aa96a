// Declarations shared by the device kernels and the host driver of the registration library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace regnk {

template <typename T>
struct cpx;

// Transport pass operations (see transport_kernels.hip for the formulas).
enum PassOp { OP_S1 = 0, OP_S2, OP_A1, OP_A2, OP_I1, OP_I2, OP_GRAD };
enum PassFlags { F_ZERO = 1, F_FIRST = 2, F_NEG = 4 };

template <typename T>
struct PassArgs {
    int n1, n2;
    long nn;                 // n1 * n2
    T h;                     // time step 1/n_t
    T bw;                    // body-force quadrature weight
    int flags;
    const T* U;              // field whose derivative the pass takes (times V for the adjoint ops)
    const T* V;              // velocity component of the pass axis (v2 rows, v1 columns)
    const T* X;              // second field (m_j, l_{j+1}, or the row-pass partial result)
    const T* VT;             // v~ (vector field)
    const T* G;              // stored gradient (vector field)
    const T* G2;             // second stored gradient (vector field)
    const T* MR;             // reference image
    T* OUT;                  // output field
    T* OUT2;                 // second output field (lam(1) = m_R - m_1)
    T* GOUT;                 // gradient output (vector field) of the state passes
    float* GOUTF;            // same, rounded to FP32 (FP64 state solve feeding an FP32 trajectory)
    float* OUT2F;            // lam(1) rounded to FP32
    T* B;                    // body-force accumulator (vector field)
    const cpx<T>* tw;        // twiddles of the pass axis length
};

constexpr int NUM_ROW_VARIANTS = 4;
constexpr int NUM_COL_VARIANTS = 7;
// var: launch-shape variant of the pass (0 = default; see transport_kernels.hpp)
template <typename T>
hipError_t launch_pass(int op, int axis, int var, const PassArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_body_end(long nn, T w, const T* lam, const T* G, T* B, hipStream_t s);

// ---- 2D spectral operators (FP64) -----------------------------------------------------------
enum SpecMode { SPEC_PROJ = 0, SPEC_HESS, SPEC_PREC, SPEC_REG };

struct SpecParams {
    int n1, n2;
    int norm;                // 1 = H1, 2 = H2
    int constraint;          // 0 none, 1 divfree, 2 mass source
    double beta_v, beta_w;
};

// Forward row pass: real vector fields -> half spectra (k2 < n2/2) in spec[field][comp][n1][n2/2].
// in1 may be null (one field).  TI = float or double.
template <typename TI>
hipError_t launch_spec_row_fwd(const SpecParams& p, const TI* in0, const TI* in1, cpx<double>* spec,
                               const cpx<double>* tw2, hipStream_t s);
// Column pass: forward FFT along x1 of the needed spectra, Fourier multiplier of `mode`, inverse
// FFT; in place in spec (outputs: field 0 = first result, field 1 = second result if want2).
hipError_t launch_spec_col(const SpecParams& p, int mode, bool have_y, bool want2, cpx<double>* spec,
                           const cpx<double>* tw1, hipStream_t s);
// Inverse row pass: spec field f -> real vector field out_d (double, nullable) and out_t
// (TO, nullable).
template <typename TO>
hipError_t launch_spec_row_inv(const SpecParams& p, int field, const cpx<double>* spec, double* out_d,
                               TO* out_t, const cpx<double>* tw2, hipStream_t s);

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

}  // namespace regnk
