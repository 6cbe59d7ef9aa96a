// Bounds-checked CPU versions of the warm-start network's device kernels, written from the
// contracts in net_kernels.hpp, so that the real host driver (net_host.hip compiled with g++) can
// run on the CPU: every operand range a launch would touch is checked against the registered
// buffers before any access (test infrastructure only).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "net_kernels.hpp"
#include "host_common.hpp"

namespace {
struct Region { const char* lo; const char* hi; };
std::vector<Region> g_regions;
std::string g_err = "no error";
int g_violations = 0;
}  // namespace

bool mock_range_ok(const void* p, size_t bytes) {
    const char* a = (const char*)p;
    for (const auto& r : g_regions)
        if (a >= r.lo && a + bytes <= r.hi) return true;
    ++g_violations;
    return false;
}

namespace regnk {
reg_status fail(reg_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}
}  // namespace regnk

extern "C" {
void mock_reset() { g_regions.clear(); g_violations = 0; }
void mock_register(void* p, size_t bytes) { g_regions.push_back({(const char*)p, (const char*)p + bytes}); }
int mock_violations() { return g_violations; }
const char* mock_last_error() { return g_err.c_str(); }
}

namespace regnk {
namespace {

// elements base[i0 + sum_d idx_d * stride_d] for idx_d < ext_d, strides >= 0
bool span_ok(const float* base, std::initializer_list<std::pair<long, long>> dims) {
    long hi = 0;
    for (auto [ext, stride] : dims) {
        if (ext <= 0) return true;
        if (stride < 0) return mock_range_ok(nullptr, 1);
        hi += (ext - 1) * stride;
    }
    return mock_range_ok(base, (size_t)(hi + 1) * sizeof(float));
}

double bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}
float gelu(float x) { return 0.5f * x * (1.0f + std::erf(x * 0.70710678118654752f)); }
float gelu_grad(float x) {
    return 0.5f * (1.0f + std::erf(x * 0.70710678118654752f)) + x * 0.39894228040143268f * std::exp(-0.5f * x * x);
}
}  // namespace

hipError_t launch_gemm(GemmArgs& g, hipStream_t) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0) return hipErrorInvalidValue;
    if (g.ksplit < 1) g.ksplit = 1;
    if (g.ksplit > 1 && !g.part) return hipErrorInvalidValue;
    if (g.part && g.batch != 1) return hipErrorInvalidValue;
    if (!g.part && !g.C) return hipErrorInvalidValue;
    g.kchunk = ((g.K + g.ksplit - 1) / g.ksplit + 31) / 32 * 32;
    g.ksplit = (g.K + g.kchunk - 1) / g.kchunk;
    bool ok = span_ok(g.A, {{g.batch, g.ab}, {g.M, g.am}, {g.K, g.ak}});
    if (!ok) fprintf(stderr, "A out of range\n");
    ok = ok && span_ok(g.B, {{g.batch, g.bb}, {g.K, g.bk}, {g.N, g.bn}});
    if (!ok) fprintf(stderr, "A or B out of range\n");
    if (g.part) ok = ok && span_ok(g.part, {{g.ksplit, (long)g.M * g.N}, {g.M, g.N}, {g.N, 1}});
    else {
        ok = ok && span_ok(g.C, {{g.batch, g.cb}, {g.M, g.cm}, {g.N, g.cn}});
        if (g.Z) ok = ok && span_ok(g.Z, {{g.batch, g.cb}, {g.M, g.cm}, {g.N, g.cn}});
        if (g.aux) ok = ok && span_ok(g.aux, {{g.batch, g.cb}, {g.M, g.cm}, {g.N, g.cn}});
        if (g.add) ok = ok && span_ok(g.add, {{g.batch, g.db}, {g.M, g.dm}, {g.N, g.dn}});
        if (g.bias) ok = ok && span_ok(g.bias, {{g.M, 1}});
    }
    if (!ok) {
        fprintf(stderr, "GEMM operand out of range: M=%d N=%d K=%d batch=%d am=%ld ak=%ld ab=%ld bk=%ld bn=%ld bb=%ld "
             "cm=%ld cn=%ld cb=%ld", g.M, g.N, g.K, g.batch, g.am, g.ak, g.ab, g.bk, g.bn, g.bb, g.cm, g.cn, g.cb);
        fprintf(stderr, " part=%p ksplit=%d Z=%p aux=%p add=%p bias=%p\n", (void*)g.part, g.ksplit, (void*)g.Z, (void*)g.aux, (void*)g.add, (void*)g.bias);
        return hipErrorInvalidValue;
    }
    for (int ks = 0; ks < g.ksplit; ++ks) {
        const int k0 = ks * g.kchunk, k1 = std::min(g.K, k0 + g.kchunk);
        for (int b = 0; b < g.batch; ++b)
            for (int m = 0; m < g.M; ++m)
                for (int n = 0; n < g.N; ++n) {
                    double acc = 0.0;
                    for (int k = k0; k < k1; ++k)
                        acc += g.f32 ? (double)g.A[b * g.ab + m * g.am + k * g.ak] * g.B[b * g.bb + k * g.bk + n * g.bn]
                                     : bf16(g.A[b * g.ab + m * g.am + k * g.ak]) * bf16(g.B[b * g.bb + k * g.bk + n * g.bn]);
                    if (g.part) {
                        g.part[(long)ks * g.M * g.N + (long)m * g.N + n] = (float)acc;
                        continue;
                    }
                    const long ci = b * g.cb + m * g.cm + n * g.cn;
                    float v = g.alpha * (float)acc;
                    if (g.beta != 0.0f) v += g.beta * g.C[ci];
                    if (g.bias) v += g.bias[m];
                    if (g.add) v += g.add[b * g.db + m * g.dm + n * g.dn];
                    if (g.Z) g.Z[ci] = v;
                    if (g.act == ACT_GELU) v = gelu(v);
                    else if (g.act == ACT_GELU_BWD) v *= gelu_grad(g.aux[ci]);
                    g.C[ci] = v;
                }
    }
    return hipSuccess;
}

hipError_t launch_splitk_reduce(int ksplit, int M, int N, const float* part, float alpha, float beta, float* C, long cm,
                                long cn, hipStream_t) {
    if (!span_ok(part, {{(long)ksplit * M * N, 1}}) || !span_ok(C, {{M, cm}, {N, cn}})) return hipErrorInvalidValue;
    for (long i = 0; i < (long)M * N; ++i) {
        float s = 0.0f;
        for (int k = 0; k < ksplit; ++k) s += part[k * (long)M * N + i];
        const long ci = (i / N) * cm + (i % N) * cn;
        float v = alpha * s;
        if (beta != 0.0f) v += beta * C[ci];
        C[ci] = v;
    }
    return hipSuccess;
}

hipError_t launch_fno_features(int n, const double* mT, const double* mR, const double* sq, float* out, long cstride,
                               hipStream_t) {
    const long nn = (long)n * n;
    if (!mock_range_ok(mT, nn * 8) || !mock_range_ok(mR, nn * 8) || !mock_range_ok(sq, 8) ||
        !span_ok(out, {{9, cstride}, {nn, 1}}))
        return hipErrorInvalidValue;
    const double inv2h = n / (4.0 * 3.14159265358979323846);
    const double sc = std::sqrt(2.0 * sq[0] / (double)nn), inv_s = sc > 0 ? 1.0 / sc : 0.0;
    for (long i = 0; i < nn; ++i) {
        const int i1 = (int)(i / n), i2 = (int)(i % n);
        const double t = mT[i];
        const double d1 = (mT[(long)((i1 + 1) % n) * n + i2] - mT[(long)((i1 + n - 1) % n) * n + i2]) * inv2h;
        const double d2 = (mT[(long)i1 * n + (i2 + 1) % n] - mT[(long)i1 * n + (i2 + n - 1) % n]) * inv2h;
        const double r = (mR[i] - t) * inv_s;
        const double ch[9] = {t, d1, d2, d1 * d1, d1 * d2, d2 * d2, r, r * d1, r * d2};
        for (int c = 0; c < 9; ++c) out[c * cstride + i] = (float)ch[c];
    }
    return hipSuccess;
}

hipError_t launch_fno_scale(long nn, const double* sq, double* scale, hipStream_t) {
    if (!mock_range_ok(sq, 8) || !mock_range_ok(scale, 8)) return hipErrorInvalidValue;
    scale[0] = std::sqrt(2.0 * sq[0] / (double)nn);
    return hipSuccess;
}

hipError_t launch_fno_target(long nn, const double* v, const double* scale, const double* dirs, float* out,
                             hipStream_t) {
    if (!mock_range_ok(v, 2 * nn * 8) || !mock_range_ok(scale, 8) || !span_ok(out, {{FNO_OUT * nn, 1}}) ||
        (dirs && !mock_range_ok(dirs, (FNO_OUT - 2) * nn * 8)))
        return hipErrorInvalidValue;
    const double inv_s = scale[0] > 0 ? 1.0 / scale[0] : 0.0;
    for (long i = 0; i < 2 * nn; ++i) out[i] = (float)(v[i] * inv_s);
    for (long i = 2 * nn; i < FNO_OUT * nn; ++i) out[i] = dirs ? (float)dirs[i - 2 * nn] : 0.0f;
    return hipSuccess;
}

hipError_t launch_fno_unscale(long nn, const float* y, const double* scale, double* v, double* dirs, hipStream_t) {
    if (!span_ok(y, {{FNO_OUT * nn, 1}}) || !mock_range_ok(scale, 8) || !mock_range_ok(v, 2 * nn * 8) ||
        (dirs && !mock_range_ok(dirs, (FNO_OUT - 2) * nn * 8)))
        return hipErrorInvalidValue;
    for (long i = 0; i < 2 * nn; ++i) v[i] = scale[0] * (double)y[i];
    if (dirs)
        for (long i = 2 * nn; i < FNO_OUT * nn; ++i) dirs[i - 2 * nn] = (double)y[i];
    return hipSuccess;
}

template <>
hipError_t launch_sqdiff<double>(const double* x, const double* y, long n, double* partial, double* out, hipStream_t) {
    if (!mock_range_ok(x, n * 8) || !mock_range_ok(y, n * 8) || !mock_range_ok(partial, RED_BLOCKS * 8) ||
        !mock_range_ok(out, 8))
        return hipErrorInvalidValue;
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += (x[i] - y[i]) * (x[i] - y[i]);
    out[0] = 0.5 * s;
    return hipSuccess;
}

hipError_t launch_fno_gather(const float* set, long nset, int channels, int n, const int32_t* idx,
                             const int32_t* sym, ChannelKinds kinds, int count, float* out, hipStream_t) {
    const long nn = (long)n * n;
    if (channels < 1 || channels > 16 || !span_ok(set, {{nset * channels * nn, 1}}) || !mock_range_ok(idx, count * 4) ||
        (sym && !mock_range_ok(sym, count * 4)) || !span_ok(out, {{(long)channels * count * nn, 1}}))
        return hipErrorInvalidValue;
    for (int c = 0; c < channels; ++c)
        for (int b = 0; b < count; ++b)
            for (long p = 0; p < nn; ++p) {
                const long o = ((long)c * count + b) * nn + p;
                const long src = idx[b];
                if (src < 0 || src >= nset) { out[o] = 0.f; continue; }
                const int code = sym ? sym[b] : 0;
                const bool sw = code & 1, f1 = (code >> 1) & 1, f2 = (code >> 2) & 1;
                const int i1 = (int)(p / n), i2 = (int)(p % n);
                const int a1 = f1 ? (n - i1) % n : i1, a2 = f2 ? (n - i2) % n : i2;
                const long q = sw ? (long)a2 * n + a1 : (long)a1 * n + a2;
                const float s1 = f1 ? -1.f : 1.f, s2 = f2 ? -1.f : 1.f;
                int cc = c;
                float sign = 1.f;
                switch (kinds.k[c]) {
                    case 1: cc = sw ? c + 1 : c; sign = s1; break;
                    case 2: cc = sw ? c - 1 : c; sign = s2; break;
                    case 3: cc = sw ? c + 2 : c; break;
                    case 4: sign = s1 * s2; break;
                    case 5: cc = sw ? c - 2 : c; break;
                    default: break;
                }
                if (cc < 0 || cc >= channels) return hipErrorInvalidValue;
                out[o] = sign * set[(src * channels + cc) * nn + q];
            }
    return hipSuccess;
}

hipError_t launch_fno_mask_disc(int S, float* Z, int radius, hipStream_t) {
    const long tot = (long)S * FNO_MODES;
    if (!span_ok(Z, {{2 * tot, 1}})) return hipErrorInvalidValue;
    for (long i = 0; i < tot; ++i) {
        const int mode = (int)(i % FNO_MODES), j = mode >> 4, k2 = mode & 15;
        const int k1 = j < FNO_M ? j : j - 2 * FNO_M;
        if (k1 * k1 + k2 * k2 > radius * radius) Z[i] = Z[tot + i] = 0.f;
    }
    return hipSuccess;
}

namespace {
bool spec_ok(int S, const float* a, long a_len, const float* b, long b_len) {
    return span_ok(a, {{a_len, 1}}) && span_ok(b, {{b_len, 1}}) && S > 0;
}
}  // namespace

hipError_t launch_fno_combine(int S, const float* T, float* Z, hipStream_t) {
    if (!spec_ok(S, T, S * 2048L, Z, 2L * S * FNO_MODES)) return hipErrorInvalidValue;
    const long tot = (long)S * FNO_MODES;
    for (long i = 0; i < tot; ++i) {
        const long s = i / FNO_MODES;
        const int j = (int)(i % FNO_MODES) >> 4, k = (int)(i % FNO_MODES) & 15;
        const float* t = T + s * 2048;
        Z[i] = t[j * 32 + k] + t[(32 + j) * 32 + 16 + k];
        Z[tot + i] = t[j * 32 + 16 + k] - t[(32 + j) * 32 + k];
    }
    return hipSuccess;
}

hipError_t launch_fno_uncombine(int S, const float* dZ, float* dT, hipStream_t) {
    if (!spec_ok(S, dZ, 2L * S * FNO_MODES, dT, S * 2048L)) return hipErrorInvalidValue;
    const long tot = (long)S * FNO_MODES;
    for (long i = 0; i < tot; ++i) {
        const long s = i / FNO_MODES;
        const int j = (int)(i % FNO_MODES) >> 4, k = (int)(i % FNO_MODES) & 15;
        float* t = dT + s * 2048;
        t[j * 32 + k] = dZ[i];
        t[(32 + j) * 32 + 16 + k] = dZ[i];
        t[j * 32 + 16 + k] = dZ[tot + i];
        t[(32 + j) * 32 + k] = -dZ[tot + i];
    }
    return hipSuccess;
}

hipError_t launch_fno_expand_o(int S, const float* O, float* Ob, hipStream_t) {
    if (!spec_ok(S, O, 2L * S * FNO_MODES, Ob, S * 2048L)) return hipErrorInvalidValue;
    const long tot = (long)S * FNO_MODES;
    for (long i = 0; i < tot; ++i) {
        const long s = i / FNO_MODES;
        const int j = (int)(i % FNO_MODES) >> 4, k = (int)(i % FNO_MODES) & 15;
        float* t = Ob + s * 2048;
        t[j * 32 + k] = O[i];
        t[j * 32 + 16 + k] = O[tot + i];
        t[(32 + j) * 32 + k] = -O[tot + i];
        t[(32 + j) * 32 + 16 + k] = O[i];
    }
    return hipSuccess;
}

hipError_t launch_fno_fold_o(int S, const float* dOb, float* dO, hipStream_t) {
    if (!spec_ok(S, dOb, S * 2048L, dO, 2L * S * FNO_MODES)) return hipErrorInvalidValue;
    const long tot = (long)S * FNO_MODES;
    for (long i = 0; i < tot; ++i) {
        const long s = i / FNO_MODES;
        const int j = (int)(i % FNO_MODES) >> 4, k = (int)(i % FNO_MODES) & 15;
        const float* t = dOb + s * 2048;
        dO[i] = t[j * 32 + k] + t[(32 + j) * 32 + 16 + k];
        dO[tot + i] = t[j * 32 + 16 + k] - t[(32 + j) * 32 + k];
    }
    return hipSuccess;
}

hipError_t launch_fno_expand_w(int layers, const float* R, long lstride, float* W, hipStream_t) {
    const long per = (long)FNO_MODES * FNO_C * FNO_C;
    if (!span_ok(R, {{layers, lstride}, {2 * per, 1}}) || !span_ok(W, {{layers * per * 4, 1}})) return hipErrorInvalidValue;
    for (long l = 0; l < layers; ++l)
        for (long r = 0; r < per; ++r) {
            const long mode = r / (FNO_C * FNO_C);
            const int c = (int)((r / FNO_C) % FNO_C), o = (int)(r % FNO_C);
            const float rr = R[l * lstride + r], ri = R[l * lstride + per + r];
            float* w = W + l * per * 4 + mode * 4096;
            w[c * 64 + o] = rr;
            w[c * 64 + 32 + o] = ri;
            w[(32 + c) * 64 + o] = -ri;
            w[(32 + c) * 64 + 32 + o] = rr;
        }
    return hipSuccess;
}

hipError_t launch_fno_fold_w(const float* dW, float* gR, hipStream_t) {
    const long per = (long)FNO_MODES * FNO_C * FNO_C;
    if (!span_ok(dW, {{per * 4, 1}}) || !span_ok(gR, {{2 * per, 1}})) return hipErrorInvalidValue;
    for (long i = 0; i < per; ++i) {
        const long mode = i / (FNO_C * FNO_C);
        const int c = (int)((i / FNO_C) % FNO_C), o = (int)(i % FNO_C);
        const float* w = dW + mode * 4096;
        gR[i] = w[c * 64 + o] + w[(32 + c) * 64 + 32 + o];
        gR[per + i] = w[c * 64 + 32 + o] - w[(32 + c) * 64 + o];
    }
    return hipSuccess;
}

hipError_t launch_rowsum(int rows, long len, const float* x, double* part, float* out, hipStream_t) {
    if (!span_ok(x, {{rows * len, 1}}) || !span_ok(out, {{rows, 1}}) ||
        !mock_range_ok(part, (size_t)rows * RS_CHUNKS * sizeof(double)))
        return hipErrorInvalidValue;
    for (int r = 0; r < rows; ++r) {
        double s = 0.0;
        for (long i = 0; i < len; ++i) s += x[r * len + i];
        out[r] = (float)s;
    }
    return hipSuccess;
}

hipError_t launch_fno_loss(int B, long npos, const float* y, const float* t, double* sums, float* dy, double* loss,
                           hipStream_t) {
    const long tot = (long)FNO_OUT * B * npos;
    const int G = 1 + FNO_RANK;
    if (!span_ok(y, {{tot, 1}}) || !span_ok(t, {{tot, 1}}) || !span_ok(dy, {{tot, 1}}) ||
        !mock_range_ok(sums, 8L * FNO_LOSS_SUMS * B) || (loss && !mock_range_ok(loss, 8)))
        return hipErrorInvalidValue;
    for (int b = 0; b < B; ++b)
        for (int g = 0; g < G; ++g) {
            double s0 = 0, s1 = 0, s2 = 0;
            for (int c = 2 * g; c < 2 * g + 2; ++c)
                for (long i = 0; i < npos; ++i) {
                    const long k = ((long)c * B + b) * npos + i;
                    const double tv = t[k], yv = y[k];
                    if (g == 0) {
                        s0 += (yv - tv) * (yv - tv);
                        s1 += tv * tv;
                    } else {
                        s0 += tv * tv;
                        s1 += yv * yv;
                        s2 += tv * yv;
                    }
                }
            double* o = sums + ((long)b * G + g) * 3;
            o[0] = s0;
            o[1] = s1;
            o[2] = s2;
        }
    const double f = FNO_DIR_WEIGHT / ((double)B * FNO_RANK);
    for (long i = 0; i < tot; ++i) {
        const int b = (int)((i / npos) % B), c = (int)(i / (npos * B));
        if (c < 2) {
            const double den = sums[(long)b * G * 3 + 1];
            dy[i] = den > 0 ? (float)(2.0 * ((double)y[i] - t[i]) / (B * den)) : 0.0f;
        } else {
            const double* S = sums + ((long)b * G + 1 + (c - 2) / 2) * 3;
            const double a = S[0], bb = std::max(S[1], 1e-30), cc = S[2];
            dy[i] = a > 0 ? (float)(f * (-2.0 * cc * t[i] / (a * bb) + 2.0 * cc * cc * y[i] / (a * bb * bb))) : 0.0f;
        }
    }
    if (loss) {
        double L = 0;
        for (int b = 0; b < B; ++b) {
            const double* S = sums + (long)b * G * 3;
            L += S[1] > 0 ? S[0] / S[1] : 0.0;
            for (int k = 0; k < FNO_RANK; ++k) {
                const double* D = S + 3 * (1 + k);
                if (D[0] > 0) L += (FNO_DIR_WEIGHT / FNO_RANK) * (1.0 - D[2] * D[2] / (D[0] * std::max(D[1], 1e-30)));
            }
        }
        *loss = L / B;
    }
    return hipSuccess;
}

hipError_t launch_adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t) {
    if (!span_ok(p, {{n, 1}}) || !span_ok(g, {{n, 1}}) || !span_ok(m, {{n, 1}}) || !span_ok(v, {{n, 1}}))
        return hipErrorInvalidValue;
    for (long i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1 - b1) * g[i];
        v[i] = b2 * v[i] + (1 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] * c1) / (std::sqrt(v[i] * c2) + eps);
    }
    return hipSuccess;
}

}  // namespace regnk
