// Two-dimensional Fourier multipliers in FP64: the Hessian / gradient assembly
// beta_v A v + K[b] (Sec. 3.3, eqs. (control-eq-elim), (inc-control-eq-elim)), the preconditioner
// (beta_v A)^{-1} (App. E.2), the Nyquist projection and the regularisation terms of the objective.
//
// Three passes over a half spectrum that omits the Nyquist column (it is projected out anyway):
//   row forward  : each row of a vector field, packed as comp0 + i comp1, is transformed along x2 and
//                  split into the half spectra of the two real components (k2 = 0..n2/2-1);
//   column       : per column k2, FFT along x1 of every needed component, the (2x2) multiplier of the
//                  mode, inverse FFT along x1 -- in place, each block owns whole columns;
//   row inverse  : the two half spectra of a result are recombined into one complex row, inverse
//                  transformed along x2; real part -> component 0, imaginary part -> component 1.
//
// Symbols (k~ = integer wavenumber with Nyquist -> 0, |k|^2 = k~1^2 + k~2^2):
//   A^ = |k|^2 (H1), |k|^4 (H2) or |k|^6 (H3)                      eq. (var-reg-v)
//   K^ = I - c(k) k k^T/|k|^2, c = 0 (no constraint), 1 (w = 0), 1/M^ (mass source) with
//   M^ = 1 + beta_v A^ / (beta_w |k|^2 (|k|^2 + 1))                 eq. (project-body-force)
//   K^{-1} = I + c'(k) k k^T/|k|^2, c' = 1/(M^ - 1)                   (mass source only)
//   P^ = beta_v A^, or beta_v where A^ = 0                          App. E.2
// SPEC_LR returns the admissible part of a direction and K^{-1} P^ of it (low-rank correction).
#include "device_common.hpp"
#include "kernels.hpp"

namespace regnk {

template <int N>
constexpr int spec_fpw() { return (N / 4) >= 64 ? 1 : 64 / (N / 4); }
template <int N>
constexpr int spec_nf() { return (N / 4) >= 32 ? 2 : 128 / (N / 4); }

// ---------------------------------------------------------------------------------------------
// bl.Q != nullptr (field 1 only): the body force in1 is completed by the deferred last adjoint step,
// with the arithmetic of body_last_kernel.
template <typename TI0, typename TI1, int N, int FPW>
__global__ __launch_bounds__(FPW * N / 4) void spec_row_fwd_kernel(int n1, const TI0* __restrict__ in0,
                                                                  const TI1* __restrict__ in1,
                                                                  cpx<double>* __restrict__ spec,
                                                                  const cpx<double>* __restrict__ tw,
                                                                  BodyLast<TI1> bl) {
    constexpr int Q = N / 4, H = N / 2;
    constexpr int L = LdsSize<N>::value;
    __shared__ cpx<double> lds[FPW][L];   // one buffer per transform: more resident blocks
    const int f = threadIdx.x / Q, t = threadIdx.x % Q;
    const int i1 = blockIdx.x * FPW + f;
    const bool valid = i1 < n1;
    const int field = blockIdx.y;
    const long nn = (long)n1 * N;
    const long row = (long)(valid ? i1 : 0) * N;
    cpx<double> x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const long i = row + t + r * Q;
        if (!valid) {
            x[r] = cpx<double>{0.0, 0.0};
        } else if (field && bl.Q) {
            TI1 u = bl.Q[i];
            u += bl.C[i];
            const TI1 xv = bl.X[i];
            const TI1 b0 = u * bl.G[i] + xv * bl.G2[i], b1 = u * bl.G[nn + i] + xv * bl.G2[nn + i];
            const TI1 o0 = bl.first ? TI1(0) : in1[i], o1 = bl.first ? TI1(0) : in1[nn + i];
            x[r] = cpx<double>{(double)(o0 + bl.w * b0), (double)(o1 + bl.w * b1)};
        } else if (field) {
            x[r] = cpx<double>{(double)in1[i], (double)in1[nn + i]};
        } else {
            x[r] = cpx<double>{(double)in0[i], (double)in0[nn + i]};
        }
    }
    int buf = 0;
    fft4<double, N, false, true>(x, lds[f], lds[f], t, tw, buf);
    cpx<double>* o = lds[f];
    __syncthreads();   // the transform's last exchange has been read
#pragma unroll
    for (int r = 0; r < 4; ++r) o[lpad(t + r * Q)] = x[r];
    __syncthreads();
    if (!valid) return;
    const long hn = (long)n1 * H;
    cpx<double>* s0 = spec + (long)(2 * field) * hn + (long)i1 * H;
    cpx<double>* s1 = s0 + hn;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int e = t + r * Q;   // < N/2
        const cpx<double> z = x[r];
        const cpx<double> zc = o[lpad((N - e) & (N - 1))];
        // Z_e = A_e + i B_e, conj(Z_{N-e}) = A_e - i B_e  (A, B spectra of the real components)
        const double dx = z.x - zc.x, dy = z.y + zc.y;   // Z_e - conj(Z_{N-e})
        s0[e] = {0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y)};
        s1[e] = {0.5 * dy, -0.5 * dx};
    }
}

// ---------------------------------------------------------------------------------------------
struct ModeCoef {
    double a;     // A^
    double kk;    // |k|^2
    double p11, p12, p22;   // k k^T / |k|^2
};

// The Fourier multiplier of `mode` at wavenumber (k1, k2) on the (scaled-later) spectra x, y of the
// two components: first result o, second result q (see the file header).
// Mean viscosity of the shear-control model with a mass source (0 otherwise); read once per kernel.
__device__ __forceinline__ double eta_bar_of(const SpecParams& p) {
    return (p.norm == 4 && p.constraint == 2 && p.eta_sum) ? *p.eta_sum / ((double)p.n1 * (double)p.n2) : 0.0;
}

__device__ __forceinline__ void spec_multiplier(const SpecParams& p, int mode, double k1, double k2d, cpx<double> x0,
                                                cpx<double> x1, cpx<double> y0, cpx<double> y1, cpx<double>& o0,
                                                cpx<double>& o1, cpx<double>& q0, cpx<double>& q1,
                                                double eta_bar = 0.0) {
    const double kk = k1 * k1 + k2d * k2d;
    // regulariser symbol of the assembly (none for the shear-control model, whose term arrives in
    // real space with the body force) and of the preconditioner (the vector Laplacian for it)
    const double A = (p.norm == 1) ? kk : (p.norm == 2 ? kk * kk : (p.norm == 3 ? kk * kk * kk : 0.0));
    const double Ap = p.norm == 4 ? kk : A;
    const double ik = kk > 0.0 ? 1.0 / kk : 0.0;
    const double p11 = k1 * k1 * ik, p12 = k1 * k2d * ik, p22 = k2d * k2d * ik;
    double c = 0.0, ci = 0.0;   // K = I - c P, K^{-1} = I + ci P
    if (kk > 0.0) {
        if (p.constraint == 1) {
            c = 1.0;
        } else if (p.constraint == 2) {
            // M^ - 1: beta_v A^ / (beta_w |k|^2 (|k|^2 + 1)); for the shear-control model (App. A,
            // relaxed incompressibility) 2 beta_v eta_bar / (beta_w (|k|^2 + 1))
            const double q = p.norm == 4 ? 2.0 * p.beta_v * eta_bar / (p.beta_w * (kk + 1.0))
                                         : p.beta_v * A / (p.beta_w * kk * (kk + 1.0));
            c = 1.0 / (1.0 + q);
            ci = 1.0 / q;
        }
    }
    o0 = {0, 0};
    o1 = {0, 0};
    q0 = {0, 0};
    q1 = {0, 0};
    if (mode == SPEC_PROJ) {
        o0 = x0;
        o1 = x1;
    } else if (mode == SPEC_HESS) {
        if (p.norm == 4) {   // K (x + y): x is the real-space regularisation term
            y0 = {y0.x + x0.x, y0.y + x0.y};
            y1 = {y1.x + x1.x, y1.y + x1.y};
        }
        const double ba = p.beta_v * A;
        // K y
        const cpx<double> ky0 = {y0.x - c * (p11 * y0.x + p12 * y1.x), y0.y - c * (p11 * y0.y + p12 * y1.y)};
        const cpx<double> ky1 = {y1.x - c * (p12 * y0.x + p22 * y1.x), y1.y - c * (p12 * y0.y + p22 * y1.y)};
        o0 = {ba * x0.x + ky0.x, ba * x0.y + ky0.y};
        o1 = {ba * x1.x + ky1.x, ba * x1.y + ky1.y};
        // K^{-1}(beta_v A x + K y) = beta_v A K^{-1} x + y
        const cpx<double> kx0 = {x0.x + ci * (p11 * x0.x + p12 * x1.x), x0.y + ci * (p11 * x0.y + p12 * x1.y)};
        const cpx<double> kx1 = {x1.x + ci * (p12 * x0.x + p22 * x1.x), x1.y + ci * (p12 * x0.y + p22 * x1.y)};
        q0 = {ba * kx0.x + y0.x, ba * kx0.y + y0.y};
        q1 = {ba * kx1.x + y1.x, ba * kx1.y + y1.y};
    } else if (mode == SPEC_PREC) {
        const double pinv = 1.0 / (p.beta_v * (Ap > 0.0 ? Ap : 1.0));
        o0 = {x0.x * pinv, x0.y * pinv};
        o1 = {x1.x * pinv, x1.y * pinv};
        q0 = {x0.x + ci * (p11 * x0.x + p12 * x1.x), x0.y + ci * (p11 * x0.y + p12 * x1.y)};
        q1 = {x1.x + ci * (p12 * x0.x + p22 * x1.x), x1.y + ci * (p12 * x0.y + p22 * x1.y)};
    } else if (mode == SPEC_LR) {
        const double ca = p.constraint == 1 ? c : 0.0;   // Leray projection for w = 0
        o0 = {x0.x - ca * (p11 * x0.x + p12 * x1.x), x0.y - ca * (p11 * x0.y + p12 * x1.y)};
        o1 = {x1.x - ca * (p12 * x0.x + p22 * x1.x), x1.y - ca * (p12 * x0.y + p22 * x1.y)};
        const double pm = p.beta_v * (Ap > 0.0 ? Ap : 1.0);
        q0 = {pm * (o0.x + ci * (p11 * o0.x + p12 * o1.x)), pm * (o0.y + ci * (p11 * o0.y + p12 * o1.y))};
        q1 = {pm * (o1.x + ci * (p12 * o0.x + p22 * o1.x)), pm * (o1.y + ci * (p12 * o0.y + p22 * o1.y))};
    } else {   // SPEC_REG: beta_v A v and beta_w (1 + |k|^2) k k^T v
        const double ba = p.beta_v * A;
        o0 = {ba * x0.x, ba * x0.y};
        o1 = {ba * x1.x, ba * x1.y};
        const double w = p.beta_w * (1.0 + kk) * kk;
        q0 = {w * (p11 * x0.x + p12 * x1.x), w * (p11 * x0.y + p12 * x1.y)};
        q1 = {w * (p12 * x0.x + p22 * x1.x), w * (p12 * x0.y + p22 * x1.y)};
    }
}

// 1 / P^ at (k1, k2) (App. E.2; SPEC_PREC's scale): 1 / (beta_v A^), or 1 / beta_v where A^ = 0; the
// vector Laplacian's symbol for the shear-control model.
__device__ __forceinline__ double prec_inv(const SpecParams& p, double k1, double k2d) {
    const double kk = k1 * k1 + k2d * k2d;
    const double A = (p.norm == 1) ? kk : (p.norm == 2 ? kk * kk : (p.norm == 3 ? kk * kk * kk : 0.0));
    const double Ap = p.norm == 4 ? kk : A;
    return 1.0 / (p.beta_v * (Ap > 0.0 ? Ap : 1.0));
}

template <int N, int NF>
__global__ __launch_bounds__(NF * N / 4) void spec_col_kernel(SpecParams p, int mode, int have_y, int want2,
                                                              cpx<double>* __restrict__ spec,
                                                              const cpx<double>* __restrict__ tw) {
    const double eb = eta_bar_of(p);
    constexpr int Q = N / 4;
    constexpr int L = LdsSize<N>::value;
    __shared__ cpx<double> lds[NF][2][L];
    const int f = threadIdx.x % NF, t = threadIdx.x / NF;
    const int H = p.n2 / 2;
    constexpr int GROUP = 16 * NF >= 128 ? 1 : 128 / (16 * NF);   // column tiles per 128-byte line
    const int k2 = xcd_tile(blockIdx.x, gridDim.x, GROUP) * NF + f;
    const bool valid = k2 < H;
    const long hn = (long)N * H;
    const long col = valid ? k2 : 0;
    // every load first (up to four spectra), then the transforms; results overwrite the inputs
    cpx<double> X0[4], X1[4], Y0[4], Y1[4];
    auto load = [&](int comp, cpx<double>(&x)[4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long idx = comp * hn + (long)(t + r * Q) * H + col;
            x[r] = valid ? spec[idx] : cpx<double>{0.0, 0.0};
        }
    };
    load(0, X0);
    load(1, X1);
    if (have_y) {
        load(2, Y0);
        load(3, Y1);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) Y0[r] = Y1[r] = cpx<double>{0.0, 0.0};
    }
    int buf = 0;
    fft4<double, N, false>(X0, lds[f][0], lds[f][1], t, tw, buf);
    fft4<double, N, false>(X1, lds[f][0], lds[f][1], t, tw, buf);
    if (have_y) {
        fft4<double, N, false>(Y0, lds[f][0], lds[f][1], t, tw, buf);
        fft4<double, N, false>(Y1, lds[f][0], lds[f][1], t, tw, buf);
    }
    const double scale = 1.0 / ((double)N * (double)p.n2);
    const double k2d = (double)k2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = t + r * Q;
        const double k1 = (double)kwave<N>(e);
        const bool zero = (e == N / 2);   // Nyquist row of x1: projected out
        cpx<double> o0, o1, q0, q1;
        spec_multiplier(p, mode, k1, k2d, X0[r], X1[r], Y0[r], Y1[r], o0, o1, q0, q1, eb);
        const double sc = zero ? 0.0 : scale;
        X0[r] = {o0.x * sc, o0.y * sc};
        X1[r] = {o1.x * sc, o1.y * sc};
        Y0[r] = {q0.x * sc, q0.y * sc};
        Y1[r] = {q1.x * sc, q1.y * sc};
    }
    auto ifft_store = [&](int comp, cpx<double>(&x)[4]) {
        fft4<double, N, true>(x, lds[f][0], lds[f][1], t, tw, buf);
        if (valid) {
#pragma unroll
            for (int r = 0; r < 4; ++r) spec[comp * hn + (long)(t + r * Q) * H + col] = x[r];
        }
    };
    ifft_store(0, X0);
    ifft_store(1, X1);
    if (want2) {
        ifft_store(2, Y0);
        ifft_store(3, Y1);
    }
}

// The same column pass with the four spectra in parallel: one column per block, thread group c
// (N/4 threads) transforms spectrum c, the multiplier runs once per wavenumber (one per thread) on
// the spectra exchanged through LDS, and group c inverse-transforms result c.  Four times the threads
// of spec_col_kernel at a quarter of the registers each.
template <int N>
__global__ __launch_bounds__(N) void spec_col_split_kernel(SpecParams p, int mode, int have_y, int want2,
                                                           cpx<double>* __restrict__ spec,
                                                           const cpx<double>* __restrict__ tw) {
    const double eb = eta_bar_of(p);
    constexpr int Q = N / 4;
    constexpr int L = LdsSize<N>::value;
    __shared__ cpx<double> lds[4][2][L];
    const int c = threadIdx.x / Q, t = threadIdx.x % Q;
    const int H = p.n2 / 2;
    const int k2 = xcd_tile(blockIdx.x, gridDim.x, 8);   // 8 columns of 16 bytes share a line
    const long hn = (long)N * H;
    cpx<double> x[4];
    const bool in_c = c < 2 || have_y;
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = in_c ? spec[c * hn + (long)(t + r * Q) * H + k2] : cpx<double>{0.0, 0.0};
    int buf = 0;
    fft4<double, N, false>(x, lds[c][0], lds[c][1], t, tw, buf);
    const int b = buf;
#pragma unroll
    for (int r = 0; r < 4; ++r) lds[c][b][lpad(t + r * Q)] = x[r];
    __syncthreads();
    const bool hp = mode == SPEC_HESS_P;
    cpx<double> r2[4] = {};   // SPEC_HESS_P with want2: the second pass's values of this thread's wavenumber
    {
        const int e = threadIdx.x;   // one wavenumber per thread
        const double k1 = (double)kwave<N>(e);
        cpx<double> o0, o1, q0, q1;
        spec_multiplier(p, hp ? SPEC_HESS : mode, k1, (double)k2, lds[0][b][lpad(e)], lds[1][b][lpad(e)],
                        lds[2][b][lpad(e)], lds[3][b][lpad(e)], o0, o1, q0, q1, eb);
        const double sc = (e == N / 2) ? 0.0 : 1.0 / ((double)N * (double)p.n2);   // Nyquist row projected out
        if (hp) {   // P^{-1} H x: into the second field, or with want2 into the third (second pass)
            const double pi = prec_inv(p, k1, (double)k2);
            const cpx<double> p0 = {pi * o0.x, pi * o0.y}, p1 = {pi * o1.x, pi * o1.y};
            if (want2) {
                r2[0] = p0;
                r2[1] = p1;
            } else {
                q0 = p0;
                q1 = p1;
            }
        }
        __syncthreads();
        lds[0][b][lpad(e)] = {o0.x * sc, o0.y * sc};
        lds[1][b][lpad(e)] = {o1.x * sc, o1.y * sc};
        lds[2][b][lpad(e)] = {q0.x * sc, q0.y * sc};
        lds[3][b][lpad(e)] = {q1.x * sc, q1.y * sc};
#pragma unroll
        for (int k = 0; k < 4; ++k) r2[k] = {r2[k].x * sc, r2[k].y * sc};
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = lds[c][b][lpad(t + r * Q)];
    buf = b ^ 1;   // the inverse's first exchange must not overwrite the buffer just read
    fft4<double, N, true>(x, lds[c][0], lds[c][1], t, tw, buf);
    if (c < 2 || want2 || hp) {
#pragma unroll
        for (int r = 0; r < 4; ++r) spec[c * hn + (long)(t + r * Q) * H + k2] = x[r];
    }
    if (hp && want2) {   // second pass: field 2 (half spectra 4, 5; groups 2 and 3 only join the exchanges)
        const int b2 = buf ^ 1;   // not the buffer the inverse's last exchange may still be read from
        __syncthreads();
        const int e = threadIdx.x;
#pragma unroll
        for (int k = 0; k < 4; ++k) lds[k][b2][lpad(e)] = r2[k];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = lds[c][b2][lpad(t + r * Q)];
        buf = b2 ^ 1;
        fft4<double, N, true>(x, lds[c][0], lds[c][1], t, tw, buf);
        if (c < 2) {
#pragma unroll
            for (int r = 0; r < 4; ++r) spec[(4 + c) * hn + (long)(t + r * Q) * H + k2] = x[r];
        }
    }
}

// ---------------------------------------------------------------------------------------------
template <typename TO, int N, int FPW>
// blockIdx.y = f > 0: field f of spec into out_d1..3 (no T copy).  d.s != nullptr: the blocks of
// field d.field also write partial sums of <d.s, out> (see RowDot).
__global__ __launch_bounds__(FPW * N / 4) void spec_row_inv_kernel(int n1, const cpx<double>* __restrict__ spec,
                                                                  double* __restrict__ out_d0,
                                                                  TO* __restrict__ out_t0,
                                                                  double* __restrict__ out_d1,
                                                                  const cpx<double>* __restrict__ tw, RowDot d,
                                                                  double* __restrict__ out_d2,
                                                                  double* __restrict__ out_d3) {
    constexpr int Q = N / 4, H = N / 2;
    constexpr int L = LdsSize<N>::value;
    __shared__ cpx<double> lds[FPW][L];   // one buffer per transform: more resident blocks
    const int f = threadIdx.x / Q, t = threadIdx.x % Q;
    const int i1 = blockIdx.x * FPW + f;
    const bool valid = i1 < n1;
    const long hn = (long)n1 * H;
    const int field = blockIdx.y;
    double* out_d = field == 0 ? out_d0 : (field == 1 ? out_d1 : (field == 2 ? out_d2 : out_d3));
    TO* out_t = field ? nullptr : out_t0;
    const cpx<double>* s0 = spec + (long)(2 * field) * hn + (long)(valid ? i1 : 0) * H;
    const cpx<double>* s1 = s0 + hn;
    cpx<double> x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = t + r * Q;
        cpx<double> z{0.0, 0.0};
        if (valid && e != H) {
            if (e < H) {
                const cpx<double> a = s0[e], b = s1[e];
                z = {a.x - b.y, a.y + b.x};
            } else {
                const cpx<double> a = s0[N - e], b = s1[N - e];
                z = {a.x + b.y, b.x - a.y};
            }
        }
        x[r] = z;
    }
    int buf = 0;
    fft4<double, N, true, true>(x, lds[f], lds[f], t, tw, buf);
    const long nn = (long)n1 * N;
    const long row = (long)i1 * N;
    if (d.s && field == d.field) {   // uniform over the block
        __shared__ double dsh[FPW * N / 4 / 64];
        double acc = 0.0;
        if (valid) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = t + r * Q;
                acc += d.s[row + e] * x[r].x + d.s[nn + row + e] * x[r].y;
            }
        }
        const double tot = block_sum<FPW * N / 4>(acc, dsh);
        if (threadIdx.x == 0) d.partial[blockIdx.x] = tot;
    }
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = t + r * Q;
        if (out_d) {
            out_d[row + e] = x[r].x;
            out_d[nn + row + e] = x[r].y;
        }
        if (out_t) {
            out_t[row + e] = (TO)x[r].x;
            out_t[nn + row + e] = (TO)x[r].y;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Any even length (grids that are not powers of two): the same three passes with direct DFT sums
// over the twiddle table W[m] = exp(-2 pi i m / n) (index (j k) mod n), O(n^2) per line, one line per
// block, the line staged in LDS.  Results equal the FFT passes up to rounding.
constexpr int DENSE_THREADS = 256;

// rows -> half spectra: block (i1, field, comp) writes spec[2 field + comp][i1][k], k < n2/2
template <typename TI0, typename TI1>
__global__ __launch_bounds__(DENSE_THREADS) void spec_dense_row_fwd_kernel(int n1, int n2, const TI0* __restrict__ in0,
                                                                          const TI1* __restrict__ in1,
                                                                          cpx<double>* __restrict__ spec,
                                                                          const cpx<double>* __restrict__ tw) {
    extern __shared__ double xr[];
    const int i1 = blockIdx.x, field = blockIdx.y, comp = blockIdx.z;
    const long off = (long)comp * n1 * n2 + (long)i1 * n2;
    for (int j = threadIdx.x; j < n2; j += DENSE_THREADS) xr[j] = field ? (double)in1[off + j] : (double)in0[off + j];
    __syncthreads();
    const int H = n2 / 2;
    cpx<double>* out = spec + (long)(2 * field + comp) * n1 * H + (long)i1 * H;
    for (int k = threadIdx.x; k < H; k += DENSE_THREADS) {
        double re = 0.0, im = 0.0;
        int m = 0;   // (j k) mod n2
        for (int j = 0; j < n2; ++j) {
            const cpx<double> w = tw[m];
            re += xr[j] * w.x;
            im += xr[j] * w.y;
            m += k;
            if (m >= n2) m -= n2;
        }
        out[k] = {re, im};
    }
}

// columns: per k2 < n2/2, DFT along x1 of the needed spectra, multiplier, inverse DFT, in place.  The
// components pass through LDS one at a time (n1 entries); every global read of the column precedes
// the first write back, and only this block touches column k2.
__global__ __launch_bounds__(DENSE_THREADS) void spec_dense_col_kernel(SpecParams p, int mode, int have_y, int want2,
                                                                      cpx<double>* __restrict__ spec,
                                                                      const cpx<double>* __restrict__ tw) {
    const double eb = eta_bar_of(p);
    extern __shared__ cpx<double> col[];   // one component of the column
    const int n1 = p.n1, H = p.n2 / 2, k2 = blockIdx.x;
    const long hn = (long)n1 * H;
    const int nc = have_y ? 4 : 2, no = want2 ? 4 : 2;
    constexpr int EM = 8;   // n1 <= 2048 = EM * DENSE_THREADS
    cpx<double> X[4][EM];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int m = 0; m < EM; ++m) X[c][m] = {0, 0};
        if (c >= nc) continue;
        __syncthreads();   // the previous component's sums are done with LDS
        for (int i = threadIdx.x; i < n1; i += DENSE_THREADS) col[i] = spec[c * hn + (long)i * H + k2];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < EM; ++m) {
            const int e = threadIdx.x + m * DENSE_THREADS;
            if (e < n1) {
                cpx<double> acc = {0, 0};
                int q = 0;   // (i e) mod n1
                for (int i = 0; i < n1; ++i) {
                    acc = cadd(acc, cmul(col[i], tw[q]));
                    q += e;
                    if (q >= n1) q -= n1;
                }
                X[c][m] = acc;
            }
        }
    }
    const double scale = 1.0 / ((double)n1 * (double)p.n2);
#pragma unroll
    for (int m = 0; m < EM; ++m) {
        const int e = threadIdx.x + m * DENSE_THREADS;
        if (e < n1) {
            const double k1 = (double)(e < n1 / 2 ? e : (e == n1 / 2 ? 0 : e - n1));
            cpx<double> o0, o1, q0, q1;
            spec_multiplier(p, mode, k1, (double)k2, X[0][m], X[1][m], X[2][m], X[3][m], o0, o1, q0, q1, eb);
            const double sc = (e == n1 / 2) ? 0.0 : scale;   // Nyquist row of x1: projected out
            X[0][m] = {o0.x * sc, o0.y * sc};
            X[1][m] = {o1.x * sc, o1.y * sc};
            X[2][m] = {q0.x * sc, q0.y * sc};
            X[3][m] = {q1.x * sc, q1.y * sc};
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c >= no) continue;
        __syncthreads();   // LDS free again
#pragma unroll
        for (int m = 0; m < EM; ++m) {
            const int e = threadIdx.x + m * DENSE_THREADS;
            if (e < n1) col[e] = X[c][m];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n1; i += DENSE_THREADS) {   // inverse DFT: conj(W)
            cpx<double> acc = {0, 0};
            int q = 0;
            for (int e = 0; e < n1; ++e) {
                acc = cadd(acc, ctw<double, true>(col[e], tw[q]));
                q += i;
                if (q >= n1) q -= n1;
            }
            spec[c * hn + (long)i * H + k2] = acc;
        }
    }
}

// half spectra -> real rows: x_j = Re Z_0 + 2 sum_{0<k<n2/2} Re(Z_k exp(2 pi i j k / n2)) (Nyquist 0)
template <typename TO>
__global__ __launch_bounds__(DENSE_THREADS) void spec_dense_row_inv_kernel(int n1, int n2,
                                                                          const cpx<double>* __restrict__ spec,
                                                                          double* __restrict__ out_d0,
                                                                          TO* __restrict__ out_t0,
                                                                          double* __restrict__ out_d1,
                                                                          const cpx<double>* __restrict__ tw) {
    extern __shared__ cpx<double> zr[];
    const int i1 = blockIdx.x, comp = blockIdx.y, field = blockIdx.z, H = n2 / 2;
    double* out_d = field ? out_d1 : out_d0;
    TO* out_t = field ? nullptr : out_t0;
    const cpx<double>* in = spec + (long)(2 * field + comp) * n1 * H + (long)i1 * H;
    for (int k = threadIdx.x; k < H; k += DENSE_THREADS) zr[k] = in[k];
    __syncthreads();
    const long off = (long)comp * n1 * n2 + (long)i1 * n2;
    for (int j = threadIdx.x; j < n2; j += DENSE_THREADS) {
        double acc = zr[0].x;
        int q = j;   // (j k) mod n2 for k = 1
        for (int k = 1; k < H; ++k) {
            const cpx<double> w = tw[q];   // exp(-2 pi i j k / n2); Re(Z conj(w)) = Z.x w.x + Z.y w.y
            acc += 2.0 * (zr[k].x * w.x + zr[k].y * w.y);
            q += j;
            if (q >= n2) q -= n2;
        }
        if (out_d) out_d[off + j] = acc;
        if (out_t) out_t[off + j] = (TO)acc;
    }
}

// ---------------------------------------------------------------------------------------------
// Lengths 2^a 3^b 5^c that are not powers of two: the same three passes with the mixed-radix FFT in
// LDS (fft_mr), one line per block of MR_THREADS threads (thread t holds entries t + MR_THREADS m).
constexpr int MR_THREADS = 256;
constexpr int MR_EM = 8;   // entries per thread: lengths up to 2048

// The twiddle table copied to LDS behind the line buffers when it fits (twl), else read from global
// memory; visible after the kernel's next barrier.
__device__ __forceinline__ const cpx<double>* mr_table(const cpx<double>* __restrict__ tw, int n, cpx<double>* lds,
                                                       int twl) {
    if (!twl) return tw;
    for (int i = threadIdx.x; i < n; i += MR_THREADS) lds[i] = tw[i];
    return lds;
}
// LDS bytes of a mixed-radix spectral pass over a length-n line: two line buffers, plus the twiddle
// table when the total stays within 64 KiB.
static inline size_t mr_spec_lds(int n, int& twl) {
    const size_t with = 3 * (size_t)n * sizeof(cpx<double>);
    twl = with <= 64 * 1024 ? 1 : 0;
    return twl ? with : 2 * (size_t)n * sizeof(cpx<double>);
}

// rows -> half spectra: block (i1, field); the row pair of components packed as c0 + i c1
template <typename TI0, typename TI1>
__global__ __launch_bounds__(MR_THREADS) void spec_mr_row_fwd_kernel(SpecParams p, const TI0* __restrict__ in0,
                                                                    const TI1* __restrict__ in1,
                                                                    cpx<double>* __restrict__ spec,
                                                                    const cpx<double>* __restrict__ tw_g, int twl) {
    extern __shared__ cpx<double> zl[];
    const int n1 = p.n1, N = p.n2, H = N / 2;
    const int i1 = blockIdx.x, field = blockIdx.y, t = threadIdx.x;
    const long nn = (long)n1 * N, row = (long)i1 * N;
    const cpx<double>* tw = mr_table(tw_g, N, zl + 2 * N, twl);
    for (int e = t; e < N; e += MR_THREADS)
        zl[e] = field ? cpx<double>{(double)in1[row + e], (double)in1[nn + row + e]}
                      : cpx<double>{(double)in0[row + e], (double)in0[nn + row + e]};
    __syncthreads();
    const cpx<double>* Z = fft_mr<double, false>(zl, zl + N, p.mr2, tw, t, MR_THREADS);
    const long hn = (long)n1 * H;
    cpx<double>* s0 = spec + (long)(2 * field) * hn + (long)i1 * H;
    cpx<double>* s1 = s0 + hn;
    for (int e = t; e < H; e += MR_THREADS) {
        const cpx<double> z = Z[e], zc = Z[e == 0 ? 0 : N - e];
        const double dx = z.x - zc.x, dy = z.y + zc.y;   // Z_e - conj(Z_{N-e})
        s0[e] = {0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y)};
        s1[e] = {0.5 * dy, -0.5 * dx};
    }
}

// columns: per k2 < n2/2, transform the needed spectra along x1, multiply, transform back; in place
__global__ __launch_bounds__(MR_THREADS) void spec_mr_col_kernel(SpecParams p, int mode, int have_y, int want2,
                                                                cpx<double>* __restrict__ spec,
                                                                const cpx<double>* __restrict__ tw_g, int twl) {
    const double eb = eta_bar_of(p);
    extern __shared__ cpx<double> cl[];
    const int N = p.n1, H = p.n2 / 2, k2 = blockIdx.x, t = threadIdx.x;
    const cpx<double>* tw = mr_table(tw_g, N, cl + 2 * N, twl);
    const long hn = (long)N * H;
    const int nc = have_y ? 4 : 2, no = want2 ? 4 : 2;
    cpx<double> X[4][MR_EM];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int m = 0; m < MR_EM; ++m) X[c][m] = {0.0, 0.0};
        if (c >= nc) continue;
        for (int e = t; e < N; e += MR_THREADS) cl[e] = spec[c * hn + (long)e * H + k2];
        __syncthreads();
        const cpx<double>* Z = fft_mr<double, false>(cl, cl + N, p.mr1, tw, t, MR_THREADS);
#pragma unroll
        for (int m = 0; m < MR_EM; ++m) {
            const int e = t + MR_THREADS * m;
            if (e < N) X[c][m] = Z[e];
        }
        __syncthreads();   // LDS free for the next component
    }
    const double scale = 1.0 / ((double)N * (double)p.n2);
#pragma unroll
    for (int m = 0; m < MR_EM; ++m) {
        const int e = t + MR_THREADS * m;
        if (e < N) {
            cpx<double> o0, o1, q0, q1;
            spec_multiplier(p, mode, (double)kwave_n(e, N), (double)k2, X[0][m], X[1][m], X[2][m], X[3][m], o0, o1,
                            q0, q1, eb);
            const double sc = (2 * e == N) ? 0.0 : scale;   // Nyquist row of x1: projected out
            X[0][m] = {o0.x * sc, o0.y * sc};
            X[1][m] = {o1.x * sc, o1.y * sc};
            X[2][m] = {q0.x * sc, q0.y * sc};
            X[3][m] = {q1.x * sc, q1.y * sc};
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c >= no) continue;
#pragma unroll
        for (int m = 0; m < MR_EM; ++m) {
            const int e = t + MR_THREADS * m;
            if (e < N) cl[e] = X[c][m];
        }
        __syncthreads();
        const cpx<double>* Z = fft_mr<double, true>(cl, cl + N, p.mr1, tw, t, MR_THREADS);
        for (int e = t; e < N; e += MR_THREADS) spec[c * hn + (long)e * H + k2] = Z[e];
        __syncthreads();
    }
}

// half spectra -> real rows: block (i1, field); Z_e = S0_e + i S1_e (e < n2/2, conjugate-symmetric
// continuation above, Nyquist 0), inverse transform, real part -> component 0, imaginary -> 1
template <typename TO>
__global__ __launch_bounds__(MR_THREADS) void spec_mr_row_inv_kernel(SpecParams p, const cpx<double>* __restrict__ spec,
                                                                    double* __restrict__ out_d0,
                                                                    TO* __restrict__ out_t0,
                                                                    double* __restrict__ out_d1,
                                                                    const cpx<double>* __restrict__ tw_g, int twl) {
    extern __shared__ cpx<double> zl[];
    const int n1 = p.n1, N = p.n2, H = N / 2;
    const int i1 = blockIdx.x, field = blockIdx.y, t = threadIdx.x;
    const long hn = (long)n1 * H;
    const cpx<double>* tw = mr_table(tw_g, N, zl + 2 * N, twl);
    double* out_d = field ? out_d1 : out_d0;
    TO* out_t = field ? nullptr : out_t0;
    const cpx<double>* s0 = spec + (long)(2 * field) * hn + (long)i1 * H;
    const cpx<double>* s1 = s0 + hn;
    for (int e = t; e < N; e += MR_THREADS) {
        cpx<double> z{0.0, 0.0};
        if (e < H) {
            const cpx<double> a = s0[e], b = s1[e];
            z = {a.x - b.y, a.y + b.x};
        } else if (e > H) {
            const cpx<double> a = s0[N - e], b = s1[N - e];
            z = {a.x + b.y, b.x - a.y};
        }
        zl[e] = z;
    }
    __syncthreads();
    const cpx<double>* Z = fft_mr<double, true>(zl, zl + N, p.mr2, tw, t, MR_THREADS);
    const long nn = (long)n1 * N, row = (long)i1 * N;
    for (int e = t; e < N; e += MR_THREADS) {
        const cpx<double> z = Z[e];
        if (out_d) {
            out_d[row + e] = z.x;
            out_d[nn + row + e] = z.y;
        }
        if (out_t) {
            out_t[row + e] = (TO)z.x;
            out_t[nn + row + e] = (TO)z.y;
        }
    }
}

static inline bool pow2(int n) { return (n & (n - 1)) == 0; }

// ---------------------------------------------------------------------------------------------
// bl.Q != nullptr only with a power-of-two n2 (see launch_spec_row_fwd_body)
template <typename TI0, typename TI1>
static hipError_t row_fwd(const SpecParams& p, const TI0* in0, const TI1* in1, const BodyLast<TI1>& bl,
                          cpx<double>* spec, const cpx<double>* tw2, hipStream_t s) {
    const int nf = in1 ? 2 : 1;
#define ROWF(NN)                                                                                       \
    case NN: {                                                                                         \
        constexpr int FPW = spec_fpw<NN>();                                                            \
        hipLaunchKernelGGL((spec_row_fwd_kernel<TI0, TI1, NN, FPW>), dim3((p.n1 + FPW - 1) / FPW, nf), \
                           dim3(FPW * NN / 4), 0, s, p.n1, in0, in1, spec, tw2, bl);                   \
        break;                                                                                         \
    }
    if (!pow2(p.n2) && p.mr2.ns > 0) {
        int twl = 0;
        const size_t lds = mr_spec_lds(p.n2, twl);
        hipLaunchKernelGGL((spec_mr_row_fwd_kernel<TI0, TI1>), dim3(p.n1, nf), dim3(MR_THREADS), lds, s, p, in0, in1,
                           spec, tw2, twl);
        return hipGetLastError();
    }
    if (!pow2(p.n2)) {
        hipLaunchKernelGGL((spec_dense_row_fwd_kernel<TI0, TI1>), dim3(p.n1, nf, 2), dim3(DENSE_THREADS),
                           p.n2 * sizeof(double), s, p.n1, p.n2, in0, in1, spec, tw2);
        return hipGetLastError();
    }
    switch (p.n2) {
        ROWF(8) ROWF(16) ROWF(32) ROWF(64) ROWF(128) ROWF(256) ROWF(512) ROWF(1024) ROWF(2048)
        default: return hipErrorInvalidValue;
    }
#undef ROWF
    return hipGetLastError();
}

template <typename TI0, typename TI1>
hipError_t launch_spec_row_fwd2(const SpecParams& p, const TI0* in0, const TI1* in1, cpx<double>* spec,
                                const cpx<double>* tw2, hipStream_t s) {
    return row_fwd<TI0, TI1>(p, in0, in1, BodyLast<TI1>{}, spec, tw2, s);
}

template <typename TI>
hipError_t launch_spec_row_fwd(const SpecParams& p, const TI* in0, const TI* in1, cpx<double>* spec,
                               const cpx<double>* tw2, hipStream_t s) {
    return launch_spec_row_fwd2<TI, TI>(p, in0, in1, spec, tw2, s);
}

template <typename T>
hipError_t launch_spec_row_fwd_body(const SpecParams& p, const double* in0, T* B, const BodyLast<T>& bl,
                                    cpx<double>* spec, const cpx<double>* tw2, hipStream_t s) {
    if (!bl.Q || pow2(p.n2)) return row_fwd<double, T>(p, in0, B, bl, spec, tw2, s);
    const hipError_t e = launch_body_last<T>((long)p.n1 * p.n2, bl.w, bl.first != 0, bl.Q, bl.C, bl.X, bl.G, bl.G2,
                                             B, (T*)nullptr, s);
    if (e != hipSuccess) return e;
    return row_fwd<double, T>(p, in0, B, BodyLast<T>{}, spec, tw2, s);
}

hipError_t launch_spec_col(const SpecParams& p, int mode, bool have_y, bool want2, cpx<double>* spec,
                           const cpx<double>* tw1, hipStream_t s) {
    const int H = p.n2 / 2;
    if (mode == SPEC_HESS_P && !spec_col_hess_p_ok(p.n1, p.n2)) return hipErrorInvalidValue;   // four-spectra kernel only
#define COLF(NN)                                                                                       \
    case NN: {                                                                                         \
        constexpr int NF = spec_nf<NN>();                                                              \
        hipLaunchKernelGGL((spec_col_kernel<NN, NF>), dim3((H + NF - 1) / NF), dim3(NF * NN / 4), 0,  \
                           s, p, mode, (int)have_y, (int)want2, spec, tw1);                            \
        break;                                                                                         \
    }
    if (!pow2(p.n1) && p.mr1.ns > 0) {
        if (p.n1 > MR_EM * MR_THREADS) return hipErrorInvalidValue;
        int twl = 0;
        const size_t lds = mr_spec_lds(p.n1, twl);
        hipLaunchKernelGGL(spec_mr_col_kernel, dim3(H), dim3(MR_THREADS), lds, s, p, mode, (int)have_y, (int)want2,
                           spec, tw1, twl);
        return hipGetLastError();
    }
    if (!pow2(p.n1)) {
        if (p.n1 > 8 * DENSE_THREADS) return hipErrorInvalidValue;
        hipLaunchKernelGGL(spec_dense_col_kernel, dim3(H), dim3(DENSE_THREADS), p.n1 * sizeof(cpx<double>), s, p,
                           mode, (int)have_y, (int)want2, spec, tw1);
        return hipGetLastError();
    }
#define COLS(NN)                                                                                       \
    case NN:                                                                                           \
        hipLaunchKernelGGL((spec_col_split_kernel<NN>), dim3(H), dim3(NN), 0, s, p, mode, (int)have_y,   \
                           (int)want2, spec, tw1);                                                     \
        break;
    switch (p.n1) {
        COLF(8) COLF(16) COLF(32) COLS(64) COLS(128) COLS(256) COLS(512) COLF(1024) COLF(2048)
        default: return hipErrorInvalidValue;
    }
#undef COLS
#undef COLF
    return hipGetLastError();
}

// field 0 of spec at `spec` -> out_d / out_t; with out_d1, field 1 -> out_d1 in the same launch
// out_d2 / out_d3 (fields 2, 3: power-of-two n2 only) with out_d1
template <typename TO>
static hipError_t row_inv_fields(const SpecParams& p, const cpx<double>* spec, double* out_d, TO* out_t,
                                 double* out_d1, const cpx<double>* tw2, hipStream_t s, const RowDot& d = RowDot{},
                                 double* out_d2 = nullptr, double* out_d3 = nullptr) {
    const int nf = out_d3 ? 4 : (out_d2 ? 3 : (out_d1 ? 2 : 1));
    if (d.count) *d.count = 0;
    if (out_d2 && !pow2(p.n2)) return hipErrorInvalidValue;
#define ROWI(NN)                                                                                       \
    case NN: {                                                                                         \
        constexpr int FPW = spec_fpw<NN>();                                                            \
        const int nb = (p.n1 + FPW - 1) / FPW;                                                         \
        hipLaunchKernelGGL((spec_row_inv_kernel<TO, NN, FPW>), dim3(nb, nf), dim3(FPW * NN / 4), 0, s, \
                           p.n1, spec, out_d, out_t, out_d1, tw2, d, out_d2, out_d3);                  \
        if (d.s && d.count) *d.count = nb;                                                             \
        break;                                                                                         \
    }
    if (!pow2(p.n2) && p.mr2.ns > 0) {
        int twl = 0;
        const size_t lds = mr_spec_lds(p.n2, twl);
        hipLaunchKernelGGL((spec_mr_row_inv_kernel<TO>), dim3(p.n1, nf), dim3(MR_THREADS), lds, s, p, spec, out_d,
                           out_t, out_d1, tw2, twl);
        return hipGetLastError();
    }
    if (!pow2(p.n2)) {
        hipLaunchKernelGGL((spec_dense_row_inv_kernel<TO>), dim3(p.n1, 2, nf), dim3(DENSE_THREADS),
                           (p.n2 / 2) * sizeof(cpx<double>), s, p.n1, p.n2, spec, out_d, out_t, out_d1, tw2);
        return hipGetLastError();
    }
    switch (p.n2) {
        ROWI(8) ROWI(16) ROWI(32) ROWI(64) ROWI(128) ROWI(256) ROWI(512) ROWI(1024) ROWI(2048)
        default: return hipErrorInvalidValue;
    }
#undef ROWI
    return hipGetLastError();
}

hipError_t launch_spec_row_inv2(const SpecParams& p, const cpx<double>* spec, double* out0, double* out1,
                                const cpx<double>* tw2, hipStream_t s) {
    return row_inv_fields<double>(p, spec, out0, (double*)nullptr, out1, tw2, s);
}

hipError_t launch_spec_row_inv2_dot(const SpecParams& p, const cpx<double>* spec, double* out0, double* out1,
                                    const cpx<double>* tw2, const RowDot& d, hipStream_t s) {
    if (!d.s || !d.partial || !d.count || d.field < 0 || d.field > (out1 ? 1 : 0)) return hipErrorInvalidValue;
    return row_inv_fields<double>(p, spec, out0, (double*)nullptr, out1, tw2, s, d);
}

hipError_t launch_spec_row_inv4_dot(const SpecParams& p, const cpx<double>* spec, double* const* out, int nf,
                                    const cpx<double>* tw2, const RowDot& d, hipStream_t s) {
    if (nf < 1 || nf > 4) return hipErrorInvalidValue;
    if (d.s && (!d.partial || !d.count || d.field < 0 || d.field >= nf)) return hipErrorInvalidValue;
    for (int f = 0; f < nf; ++f)
        if (!out[f]) return hipErrorInvalidValue;
    return row_inv_fields<double>(p, spec, out[0], (double*)nullptr, nf > 1 ? out[1] : nullptr, tw2, s, d,
                                  nf > 2 ? out[2] : nullptr, nf > 3 ? out[3] : nullptr);
}

// ---------------------------------------------------------------------------------------------
// Nyquist projection in real space.  The modes k2 = n2/2 of row i1 and k1 = n1/2 of column i2 are
// the alternating sums a(i1) = (1/n2) sum_i2 (-1)^i2 v and b(i2) = (1/n1) sum_i1 (-1)^i1 v, and the
// corner mode c = (1/n1) sum_i1 (-1)^i1 a(i1) is counted in both, so the projection (every mode
// with k1 = n1/2 or k2 = n2/2 removed) is
//     v - (-1)^i2 a(i1) - (-1)^i1 b(i2) + (-1)^(i1 + i2) c.
// Two reads and one write of the field; fixed summation order.
constexpr int NYQ_THREADS = 256;
constexpr int NYQ_TR = 32, NYQ_TC = 64;   // tile of the first pass: 64 columns x 4 row groups of 8 rows

// pass 1, per 32 x 64 tile: partial alternating row sums rowp[comp][cb][i1] over the tile's columns,
// partial alternating column sums colp[comp][rb][i2] over its rows, and the tile's corner sum
// cpart[comp][rb][cb].  Every load is issued before the first use; the row sums go through LDS.
__global__ __launch_bounds__(NYQ_THREADS) void nyq_tile_kernel(int n1, int n2, const double* __restrict__ in,
                                                               double* __restrict__ rowp, double* __restrict__ colp,
                                                               double* __restrict__ cpart) {
    constexpr int RG = NYQ_THREADS / NYQ_TC, K = NYQ_TR / RG;   // 4 row groups of 8 rows
    __shared__ double tile[NYQ_TR][NYQ_TC + 1];
    __shared__ double csum[RG][NYQ_TC];
    __shared__ double rsum[NYQ_TR];
    const int cb = blockIdx.x, rb = blockIdx.y, comp = blockIdx.z, ncb = gridDim.x, nrb = gridDim.y;
    const int tx = threadIdx.x % NYQ_TC, ty = threadIdx.x / NYQ_TC;
    const int j = cb * NYQ_TC + tx;
    const bool jv = j < n2;
    const double* v = in + (long)comp * n1 * n2;
    double x[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {   // clamped addresses: every load in bounds, masked below
        const int i = rb * NYQ_TR + ty + RG * k;
        x[k] = v[(long)(i < n1 ? i : 0) * n2 + (jv ? j : 0)];
    }
    double col = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = rb * NYQ_TR + ty + RG * k;
        const double y = (i < n1 && jv) ? x[k] : 0.0;
        col += (i & 1) ? -y : y;
        tile[ty + RG * k][tx] = (j & 1) ? -y : y;
    }
    csum[ty][tx] = col;
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NYQ_TC) {
        if (jv) colp[((long)comp * nrb + rb) * n2 + j] = ((csum[0][t] + csum[1][t]) + csum[2][t]) + csum[3][t];
    } else if (t < NYQ_TC + NYQ_TR) {
        const int r = t - NYQ_TC, i = rb * NYQ_TR + r;
        double acc = 0.0;
        for (int c = 0; c < NYQ_TC; ++c) acc += tile[r][c];
        rsum[r] = acc;
        if (i < n1) rowp[((long)comp * ncb + cb) * n1 + i] = acc;
    }
    __syncthreads();
    if (t == 0) {
        double acc = 0.0;
        for (int r = 0; r < NYQ_TR; ++r) acc += ((rb * NYQ_TR + r) & 1) ? -rsum[r] : rsum[r];   // rows >= n1 hold 0
        cpart[((long)comp * nrb + rb) * ncb + cb] = acc;
    }
}

// pass 2, per 32 x 64 tile: a(i1) of the tile's rows and b(i2) of its columns from the partial sums,
// c from the corner sums (every block forms them in the same fixed order, so all agree), and the
// projected tile.  The tile's loads are issued first and overlap the sums.
template <typename TO>
__global__ __launch_bounds__(NYQ_THREADS) void nyq_apply_kernel(int n1, int n2, const double* __restrict__ in,
                                                                const double* __restrict__ rowp,
                                                                const double* __restrict__ colp,
                                                                const double* __restrict__ cpart,
                                                                double* __restrict__ out_d, TO* __restrict__ out_t) {
    constexpr int RG = NYQ_THREADS / NYQ_TC, K = NYQ_TR / RG;
    __shared__ double sa[NYQ_TR], sb[NYQ_TC], sh[NYQ_THREADS / 64], sc;
    const int cb = blockIdx.x, rb = blockIdx.y, comp = blockIdx.z, ncb = gridDim.x, nrb = gridDim.y;
    const int tx = threadIdx.x % NYQ_TC, ty = threadIdx.x / NYQ_TC, t = threadIdx.x;
    const int j = cb * NYQ_TC + tx;
    const bool jv = j < n2;
    const long base = (long)comp * n1 * n2;
    double x[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {   // clamped addresses: every load in bounds, masked below
        const int i = rb * NYQ_TR + ty + RG * k;
        x[k] = in[base + (long)(i < n1 ? i : 0) * n2 + (jv ? j : 0)];
    }
    const double* cp = cpart + (long)comp * nrb * ncb;
    double acc = 0.0;
    for (int k = t; k < nrb * ncb; k += NYQ_THREADS) acc += cp[k];
    const double csum = block_sum<NYQ_THREADS>(acc, sh);
    if (t == 0) sc = csum / ((double)n1 * (double)n2);
    if (t < NYQ_TR) {
        const int i = rb * NYQ_TR + t;
        double r = 0.0;
        if (i < n1) {
            const double* rp = rowp + (long)comp * ncb * n1;
#pragma unroll 8
            for (int k = 0; k < ncb; ++k) r += rp[(long)k * n1 + i];
        }
        sa[t] = r / n2;
    } else if (t < NYQ_TR + NYQ_TC) {
        const int jj = cb * NYQ_TC + (t - NYQ_TR);
        double r = 0.0;
        if (jj < n2) {
            const double* q = colp + (long)comp * nrb * n2;
#pragma unroll 8
            for (int k = 0; k < nrb; ++k) r += q[(long)k * n2 + jj];
        }
        sb[t - NYQ_TR] = r / n1;
    }
    __syncthreads();
    if (!jv) return;
    const double sj = (j & 1) ? -1.0 : 1.0;
    const double bj = sb[tx];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int r = ty + RG * k, i = rb * NYQ_TR + r;
        if (i >= n1) continue;
        const double si = (i & 1) ? -1.0 : 1.0;
        const double y = x[k] - sj * sa[r] - si * bj + sj * (si * sc);
        const long idx = base + (long)i * n2 + j;
        if (out_d) out_d[idx] = y;
        if (out_t) out_t[idx] = (TO)y;
    }
}

template <typename TO>
hipError_t launch_nyquist_project(int n1, int n2, const double* in, double* out_d, TO* out_t, double* scratch,
                                  hipStream_t s) {
    const int ncb = (n2 + NYQ_TC - 1) / NYQ_TC, nrb = (n1 + NYQ_TR - 1) / NYQ_TR;
    double* rowp = scratch;
    double* colp = rowp + 2L * ncb * n1;
    double* cpart = colp + 2L * nrb * n2;
    hipLaunchKernelGGL(nyq_tile_kernel, dim3(ncb, nrb, 2), dim3(NYQ_THREADS), 0, s, n1, n2, in, rowp, colp, cpart);
    hipLaunchKernelGGL((nyq_apply_kernel<TO>), dim3(ncb, nrb, 2), dim3(NYQ_THREADS), 0, s, n1, n2, in, rowp, colp,
                       cpart, out_d, out_t);
    return hipGetLastError();
}

size_t nyquist_scratch_doubles(int n1, int n2) {
    const size_t ncb = (n2 + NYQ_TC - 1) / NYQ_TC, nrb = (n1 + NYQ_TR - 1) / NYQ_TR;
    return 2 * ncb * n1 + 2 * nrb * n2 + 2 * nrb * ncb;
}

template hipError_t launch_spec_row_fwd<float>(const SpecParams&, const float*, const float*, cpx<double>*,
                                               const cpx<double>*, hipStream_t);
template hipError_t launch_spec_row_fwd<double>(const SpecParams&, const double*, const double*,
                                                cpx<double>*, const cpx<double>*, hipStream_t);
template hipError_t launch_spec_row_fwd2<double, float>(const SpecParams&, const double*, const float*,
                                                        cpx<double>*, const cpx<double>*, hipStream_t);
template hipError_t launch_spec_row_fwd2<double, double>(const SpecParams&, const double*, const double*,
                                                         cpx<double>*, const cpx<double>*, hipStream_t);
template hipError_t launch_spec_row_fwd_body<float>(const SpecParams&, const double*, float*, const BodyLast<float>&,
                                                    cpx<double>*, const cpx<double>*, hipStream_t);
template hipError_t launch_spec_row_fwd_body<double>(const SpecParams&, const double*, double*,
                                                     const BodyLast<double>&, cpx<double>*, const cpx<double>*,
                                                     hipStream_t);
template hipError_t launch_nyquist_project<float>(int, int, const double*, double*, float*, double*, hipStream_t);
template hipError_t launch_nyquist_project<double>(int, int, const double*, double*, double*, double*, hipStream_t);

}  // namespace regnk
