// Drives every entry point of the registration library's host driver, built for the CPU with the
// range-checking launch functions of regmock_kernels.cpp, for a few grids and models.  Built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_reg_host_asan.py (test
// infrastructure only): any heap or stack misuse, leak or undefined behaviour in the host code aborts
// the run, and an out-of-range launch makes the call fail.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "regnk.h"

extern "C" {
void mock_register(const void* p, size_t bytes);
void mock_reset();
const char* mock_last_error();
}

namespace {
int failures = 0;

struct Buffers {   // 256-byte aligned host buffers standing in for device memory, registered
    std::vector<void*> all;
    ~Buffers() {
        for (void* p : all) std::free(p);
    }
    template <typename T>
    T* get(size_t n) {
        const size_t bytes = ((n * sizeof(T) + 255) / 256) * 256 + 256;
        void* p = std::aligned_alloc(256, bytes);
        std::memset(p, 0, bytes);
        mock_register(p, n * sizeof(T));
        all.push_back(p);
        return static_cast<T*>(p);
    }
};

void check(const char* what, reg_status rc, const std::vector<int>& ok = {REG_OK}) {
    const char* err = mock_last_error();
    bool good = err[0] == 0;
    bool code = false;
    for (int c : ok) code |= rc == c;
    if (!good || !code) {
        std::fprintf(stderr, "%s: status %d (%s) mock: %s\n", what, rc, reg_last_error(), err);
        ++failures;
    }
}

void run(int n1, int n2, int nt, int norm, int constraint, int precision, int lowrank, int hessian) {
    mock_reset();
    Buffers B;
    reg_params p{};
    p.n1 = n1;
    p.n2 = n2;
    p.nt = nt;
    p.norm = norm;
    p.constraint = constraint;
    p.precision = precision;
    p.adjoint = REG_ADJ_DISCRETE;
    p.hessian = hessian;
    p.lowrank_capacity = lowrank;
    p.nt_max = 2 * nt;
    p.beta_v = 1e-3;
    p.beta_w = constraint == REG_MASS_SOURCE ? 1e-4 : 0.0;
    p.stokes_nu = norm == REG_STOKES ? 1.0 : 0.0;
    p.stokes_eps = norm == REG_STOKES ? 1e-6 : 0.0;
    const size_t nn = (size_t)n1 * n2;
    size_t nb = 0;
    check("workspace_bytes", reg_workspace_bytes(&p, &nb));
    void* ws = B.get<unsigned char>(nb);
    double* mT = B.get<double>(nn);
    double* mR = B.get<double>(nn);
    for (size_t i = 0; i < nn; ++i) {
        mT[i] = 0.5 + 0.25 * std::sin(0.3 * (double)(i % n2)) * std::cos(0.2 * (double)(i / n2));
        mR[i] = mT[i];
    }
    reg_problem* h = nullptr;
    check("create", reg_create(&p, mT, mR, ws, nb, nullptr, &h));
    if (!h) return;
    double* v = B.get<double>(2 * nn);
    double* g = B.get<double>(2 * nn);
    double* vt = B.get<double>(2 * nn);
    double* Hv = B.get<double>(2 * nn);
    double* z = B.get<double>(2 * nn);
    double* x = B.get<double>(2 * nn);
    double* m1 = B.get<double>(nn);
    double J = 0, terms[3], cfl = 0, rel = 0;
    int32_t it = 0;
    check("set_images", reg_set_images(h, mT, mR));
    check("state_forward", reg_state_forward(h, v, m1));
    check("objective", reg_objective(h, v, &J, terms));
    check("gradient", reg_gradient(h, v, g, &J));
    check("matvec", reg_hessian_matvec(h, vt, Hv));
    check("matvec again", reg_hessian_matvec(h, vt, Hv));
    check("precond", reg_precond_apply(h, g, z));
    check("pcg", reg_pcg(h, g, 0.5, 4, 0, x, &it, &rel), {REG_OK, REG_ENOTCONV, REG_ENONFINITE});
    check("pcg fixed", reg_pcg(h, g, 0.5, 8, 3, x, &it, &rel), {REG_OK, REG_ENOTCONV, REG_ENONFINITE});
    check("cfl", reg_cfl(h, v, &cfl));
    const std::vector<int> gn = {hessian == REG_HESS_GN ? REG_OK : REG_EINVAL};
    for (int which = 0; which < 4; ++which) {
        double ms = 0, by = 0, ex = 0, ph[6];
        check("time_pass", reg_time_pass(h, which, 2, &ms, &by, &ex), gn);
        check("time_phases", reg_time_phases(h, which, 2, ph), gn);
    }
    char report[8192];
    check("autotune", reg_autotune(h, 1, report, sizeof report));
    const int32_t var[7] = {0, 0, 1, 2, 3, 4, 0};
    check("set_pass_variants", reg_set_pass_variants(h, var, 7));
    size_t dnb = 0;
    check("deformation_workspace_bytes", reg_deformation_workspace_bytes(&p, &dnb));
    void* dws = B.get<unsigned char>(dnb);
    double* u1 = B.get<double>(2 * nn);
    double* F1 = B.get<double>(4 * nn);
    double* det = B.get<double>(nn);
    double stats[4];
    check("deformation", reg_deformation(h, v, dws, dnb, u1, F1, det, stats));
    check("deformation_static", reg_deformation_static(h, v, u1, F1, det, stats),
          {nn <= 65536 ? REG_OK : REG_EINVAL});
    if (lowrank > 0 && norm != REG_STOKES) {
        const int rank = lowrank < 4 ? lowrank : 4;
        double* U = B.get<double>((size_t)rank * 2 * nn);
        for (size_t i = 0; i < (size_t)rank * 2 * nn; ++i) U[i] = std::sin(0.01 * (double)i);
        double theta[8];
        check("ritz_directions", reg_ritz_directions(h, U, rank, 2, theta), {REG_OK, REG_ENONFINITE});
    }
    reg_solve_opts o{};
    o.max_newton = 3;
    o.max_pcg = 5;
    o.max_backtracks = 3;
    o.gtol_rel = 1e-3;
    o.armijo_c1 = 1e-4;
    o.armijo_rho = 0.5;
    o.cfl_max = 0.5;
    o.recycle = lowrank > 0 ? 1 : 0;
    reg_step_record rec[2];
    o.steps = rec;
    o.max_steps = 2;
    reg_solve_stats st{};
    double* vout = B.get<double>(2 * nn);
    check("solve", reg_solve(h, &o, vout, &st), {REG_OK, REG_ENOTCONV, REG_ENONFINITE});
    // a batch of this handle and a second one on the same grid
    void* ws2 = B.get<unsigned char>(nb);
    reg_problem* h2 = nullptr;
    check("create 2", reg_create(&p, mT, mR, ws2, nb, nullptr, &h2));
    if (h2) {
        reg_problem* hs[2] = {h, h2};
        reg_solve_opts os[2] = {o, o};
        os[0].steps = os[1].steps = nullptr;
        os[0].max_steps = os[1].max_steps = 0;
        double* outs[2] = {vout, B.get<double>(2 * nn)};
        reg_solve_stats sts[2];
        check("batch_solve", reg_batch_solve(2, hs, os, outs, sts), {REG_OK, REG_ENOTCONV, REG_ENONFINITE});
        check("destroy 2", reg_destroy(h2));
    }
    check("destroy", reg_destroy(h));
}
}  // namespace

int main() {
    run(64, 64, 4, REG_H1, REG_DIVFREE, REG_FP32_TRANSPORT, 0, REG_HESS_GN);
    run(256, 256, 4, REG_H2, REG_MASS_SOURCE, REG_FP32_TRANSPORT, 8, REG_HESS_GN);
    run(96, 150, 3, REG_H2, REG_MASS_SOURCE, REG_FP64, 0, REG_HESS_GN);
    run(14, 22, 2, REG_H1, REG_UNCONSTRAINED, REG_FP64, 2, REG_HESS_FULL);
    run(32, 32, 2, REG_STOKES, REG_DIVFREE, REG_FP64, 0, REG_HESS_GN);
    std::printf("asan driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
