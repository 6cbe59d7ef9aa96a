// Drives every entry point of the warm-start network's host driver, built for the CPU with the
// bounds-checked kernels of netmock_kernels.cpp, at a small grid.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_reg_host_asan.py (test infrastructure only): any heap or
// stack misuse, leak or undefined behaviour in the host code aborts the run, and an out-of-range
// launch operand is counted.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "regnet.h"

extern "C" {
void mock_reset();
void mock_register(void* p, size_t bytes);
int mock_violations();
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

void check(const char* what, reg_status rc, reg_status want = REG_OK) {
    if (rc != want || mock_violations() != 0) {
        std::fprintf(stderr, "%s: status %d mock: %s\n", what, rc, mock_last_error());
        ++failures;
    }
}

void run(int n, int B) {
    mock_reset();
    Buffers M;
    const size_t nn = (size_t)n * n;
    int64_t np = 0;
    check("param_count", reg_fno_param_count(&np));
    size_t nb = 0;
    check("workspace_bytes", reg_fno_workspace_bytes(n, B, &nb));
    void* ws = M.get<unsigned char>(nb);
    reg_fno* h = nullptr;
    check("create", reg_fno_create(n, B, ws, nb, nullptr, &h));
    if (!h) return;
    float* params = M.get<float>((size_t)np);
    for (int64_t i = 0; i < np; ++i) params[i] = 0.01f * std::sin(0.37f * (float)i);
    double* mT = M.get<double>(nn);
    double* mR = M.get<double>(nn);
    for (size_t i = 0; i < nn; ++i) {
        mT[i] = 0.5 + 0.25 * std::sin(0.4 * (double)(i % n)) * std::cos(0.3 * (double)(i / n));
        mR[i] = 0.5 + 0.25 * std::sin(0.4 * (double)(i % n) + 0.2) * std::cos(0.3 * (double)(i / n));
    }
    // a set of B samples: features and targets
    float* feats = M.get<float>((size_t)B * 9 * nn);
    float* targets = M.get<float>((size_t)B * REG_FNO_OUT * nn);
    double* scale = M.get<double>(1);
    double* v = M.get<double>(2 * nn);
    double* dirs = M.get<double>((size_t)REG_FNO_RANK * 2 * nn);
    for (size_t i = 0; i < 2 * nn; ++i) v[i] = 0.1 * std::sin(0.01 * (double)i);
    for (size_t i = 0; i < (size_t)REG_FNO_RANK * 2 * nn; ++i) dirs[i] = std::cos(0.02 * (double)i);
    for (int b = 0; b < B; ++b) {
        check("features", reg_fno_features(h, mT, mR, feats + (size_t)b * 9 * nn, scale));
        check("target", reg_fno_target(h, v, scale, b ? dirs : nullptr, targets + (size_t)b * REG_FNO_OUT * nn));
    }
    int32_t* idx = M.get<int32_t>(B);
    int32_t* sym = M.get<int32_t>(B);
    for (int b = 0; b < B; ++b) {
        idx[b] = (b + 1) % (B + 1);   // the last index is outside the set: zeros
        sym[b] = (3 * b + 1) % 8;
    }
    float* in = M.get<float>((size_t)9 * B * nn);
    float* tgt = M.get<float>((size_t)REG_FNO_OUT * B * nn);
    check("gather features", reg_fno_gather(h, feats, B, 9, idx, sym, in));
    check("gather targets", reg_fno_gather(h, targets, B, REG_FNO_OUT, idx, sym, tgt));
    float* out = M.get<float>((size_t)REG_FNO_OUT * B * nn);
    float* grad = M.get<float>((size_t)np);
    float* m = M.get<float>((size_t)np);
    float* vv = M.get<float>((size_t)np);
    double* loss = M.get<double>(1);
    check("backward before forward", reg_fno_backward(h, params, tgt, grad, loss), REG_ESTATE);
    check("forward", reg_fno_forward(h, params, in, out));
    check("backward", reg_fno_backward(h, params, tgt, grad, loss));
    check("adam", reg_fno_adam(h, params, grad, m, vv, 1, 1e-3f, 0.9f, 0.999f, 1e-8f));
    check("train_step", reg_fno_train_step(h, params, in, tgt, grad, m, vv, 2, 1e-3f, loss));
    check("destroy", reg_fno_destroy(h));
    // prediction on a batch-1 handle
    size_t nb1 = 0;
    check("workspace_bytes 1", reg_fno_workspace_bytes(n, 1, &nb1));
    void* ws1 = M.get<unsigned char>(nb1);
    reg_fno* h1 = nullptr;
    check("create 1", reg_fno_create(n, 1, ws1, nb1, nullptr, &h1));
    if (!h1) return;
    double* v0 = M.get<double>(2 * nn);
    double* d0 = M.get<double>((size_t)REG_FNO_RANK * 2 * nn);
    check("predict", reg_fno_predict(h1, params, mT, mR, v0, d0));
    check("predict without directions", reg_fno_predict(h1, params, mT, mR, v0, nullptr));
    check("destroy 1", reg_fno_destroy(h1));
}
}  // namespace

int main() {
    run(32, 2);
    run(64, 3);
    std::printf("net asan driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
