// Pointwise kernels of the nonlinear Stokes (shear-control) regularisation, Sec. 2,
// eq. (shear-control-reg-v) with its variations eqs. (1st-var-reg-v-nls), (2nd-var-reg-v-nls), in FP64.
// Derivatives come from the FP64 gradient stage launches; these kernels work on the four partials
// dv[i][l] = d_l v_i (field 2 i + l), the strain E = (E11, E12, E22) and the viscosity
// eta = (E:E + eps)^{(1-nu)/(2nu)}, with E:E = E11^2 + 2 E12^2 + E22^2.
#include <cmath>

#include "device_common.hpp"
#include "kernels.hpp"

namespace regnk {

static inline int grid_n(long n) {
    long b = (n + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

// First variation at v: stress sigma = 2 eta E (3 fields); optionally keep E and eta (the
// linearisation point of later Hessian matvecs) and the integrand (E:E + eps)^{(1+nu)/(2nu)}.
__global__ void stokes_first_kernel(long nn, const double* __restrict__ dv, double nu, double eps,
                                    double* __restrict__ sig, double* __restrict__ E, double* __restrict__ eta,
                                    double* __restrict__ dens) {
    const double pe = (1.0 - nu) / (2.0 * nu), pd = (1.0 + nu) / (2.0 * nu);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
        const double e11 = dv[i], e22 = dv[3 * nn + i], e12 = 0.5 * (dv[nn + i] + dv[2 * nn + i]);
        const double s = e11 * e11 + 2.0 * e12 * e12 + e22 * e22 + eps;
        const double et = pow(s, pe);
        if (sig) {
            sig[i] = 2.0 * et * e11;
            sig[nn + i] = 2.0 * et * e12;
            sig[2 * nn + i] = 2.0 * et * e22;
        }
        if (E) {
            E[i] = e11;
            E[nn + i] = e12;
            E[2 * nn + i] = e22;
        }
        if (eta) eta[i] = et;
        if (dens) dens[i] = pow(s, pd);
    }
}

// Second variation at the stored point in direction v~ (partials dvt): sigma~ = 2 eta (E~ + c E) with
// c = (1-nu)/nu (E : E~) / (E:E + eps).
__global__ void stokes_second_kernel(long nn, const double* __restrict__ dvt, const double* __restrict__ E,
                                     const double* __restrict__ eta, double nu, double eps,
                                     double* __restrict__ sig) {
    const double cn = (1.0 - nu) / nu;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
        const double t11 = dvt[i], t22 = dvt[3 * nn + i], t12 = 0.5 * (dvt[nn + i] + dvt[2 * nn + i]);
        const double e11 = E[i], e12 = E[nn + i], e22 = E[2 * nn + i];
        const double ee = e11 * e11 + 2.0 * e12 * e12 + e22 * e22 + eps;
        const double c = cn * (e11 * t11 + 2.0 * e12 * t12 + e22 * t22) / ee;
        const double w = 2.0 * eta[i];
        sig[i] = w * (t11 + c * e11);
        sig[nn + i] = w * (t12 + c * e12);
        sig[2 * nn + i] = w * (t22 + c * e22);
    }
}

// out = scale * div sigma: out_1 = scale (d1 s11 + d2 s12), out_2 = scale (d1 s12 + d2 s22), from the
// gradients of the three stress fields (ds: grad s11 at 0, grad s12 at 2 nn, grad s22 at 4 nn).
__global__ void stokes_div_kernel(long nn, const double* __restrict__ ds, double scale, double* __restrict__ out) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
        out[i] = scale * (ds[i] + ds[3 * nn + i]);
        out[nn + i] = scale * (ds[2 * nn + i] + ds[5 * nn + i]);
    }
}

hipError_t launch_stokes_first(long nn, const double* dv, double nu, double eps, double* sig, double* E, double* eta,
                               double* dens, hipStream_t s) {
    hipLaunchKernelGGL(stokes_first_kernel, dim3(grid_n(nn)), dim3(256), 0, s, nn, dv, nu, eps, sig, E, eta, dens);
    return hipGetLastError();
}
hipError_t launch_stokes_second(long nn, const double* dvt, const double* E, const double* eta, double nu, double eps,
                                double* sig, hipStream_t s) {
    hipLaunchKernelGGL(stokes_second_kernel, dim3(grid_n(nn)), dim3(256), 0, s, nn, dvt, E, eta, nu, eps, sig);
    return hipGetLastError();
}
hipError_t launch_stokes_div(long nn, const double* ds, double scale, double* out, hipStream_t s) {
    hipLaunchKernelGGL(stokes_div_kernel, dim3(grid_n(nn)), dim3(256), 0, s, nn, ds, scale, out);
    return hipGetLastError();
}

}  // namespace regnk
