// The library's mixed-radix LDS FFT (device_common.hpp: mr_plan, fft_mr) compiled for the host with
// a single emulated thread, exported for a CPU test against numpy's FFT (test infrastructure only).
#include <vector>

#include "device_common.hpp"

using namespace regnk;

extern "C" {
// number of stages of the plan for length n (0: length not of the form 2^a 3^b 5^c) and its radices
int mr_plan_radices(int n, int* radices) {
    const MrPlan p = mr_plan(n);
    for (int s = 0; s < p.ns; ++s) radices[s] = p.r[s];
    return p.ns;
}
// out = DFT (inv = 0: exp(-2 pi i jk/n); inv = 1: exp(+2 pi i jk/n), unscaled) of the complex sequence
// in (interleaved re/im, n entries); tw: exp(-2 pi i m / n), m < n (interleaved).  Double or single
// precision (single: in, tw and out are rounded on entry / exit).
int mr_fft(int n, int inv, int single, const double* in, const double* tw, double* out) {
    const MrPlan p = mr_plan(n);
    if (p.ns == 0) return -1;
    if (single) {
        std::vector<cpx<float>> a(n), b(n), w(n);
        for (int i = 0; i < n; ++i) {
            a[i] = {(float)in[2 * i], (float)in[2 * i + 1]};
            w[i] = {(float)tw[2 * i], (float)tw[2 * i + 1]};
        }
        cpx<float>* r = inv ? fft_mr<float, true>(a.data(), b.data(), p, w.data(), 0, 1)
                            : fft_mr<float, false>(a.data(), b.data(), p, w.data(), 0, 1);
        for (int i = 0; i < n; ++i) { out[2 * i] = r[i].x; out[2 * i + 1] = r[i].y; }
        return 0;
    }
    std::vector<cpx<double>> a(n), b(n), w(n);
    for (int i = 0; i < n; ++i) {
        a[i] = {in[2 * i], in[2 * i + 1]};
        w[i] = {tw[2 * i], tw[2 * i + 1]};
    }
    cpx<double>* r = inv ? fft_mr<double, true>(a.data(), b.data(), p, w.data(), 0, 1)
                         : fft_mr<double, false>(a.data(), b.data(), p, w.data(), 0, 1);
    for (int i = 0; i < n; ++i) { out[2 * i] = r[i].x; out[2 * i + 1] = r[i].y; }
    return 0;
}
}
