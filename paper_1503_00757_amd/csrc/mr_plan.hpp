// Factorisation of an axis length into the radices of the mixed-radix FFT (device_common.hpp: fft_mr).
// Plain C++ (no device code), shared by the host driver and the kernels' argument structs.
#pragma once

namespace regnk {

// A plan factors the length into radices 8, 4, 2, 3 and 5 (product = n); ns = 0 means the length has
// another prime factor (those axes keep the direct circulant / DFT sums).
constexpr int MR_MAX_STAGES = 16;
struct MrPlan {
    int n;
    int ns;
    int r[MR_MAX_STAGES];
};

// Host-side planner: radices 5 and 3 first, then the power of two as 8s and at most one 4 or 2.
inline MrPlan mr_plan(int n) {
    MrPlan p{};
    p.n = n;
    int m = n, ns = 0;
    const int odd[2] = {5, 3};
    for (int q : odd)
        while (m % q == 0 && ns < MR_MAX_STAGES) {
            p.r[ns++] = q;
            m /= q;
        }
    while (m % 8 == 0 && ns < MR_MAX_STAGES) {
        p.r[ns++] = 8;
        m /= 8;
    }
    if (m == 4 || m == 2) {
        p.r[ns++] = m;
        m = 1;
    }
    p.ns = (m == 1 && n > 1) ? ns : 0;
    return p;
}

}  // namespace regnk
