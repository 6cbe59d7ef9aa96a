// Range-checking CPU versions of every launch function the registration library's host driver calls
// (test infrastructure only).  Each one checks that every array it would read or write lies inside
// a buffer the harness registered (the caller's workspace and arrays) or a range the library
// registered through the mock runtime (its static scratch), for the extents the device kernel would
// touch; it computes nothing except the few device scalars the driver reads back, which it fills
// with finite placeholders.  An out-of-range access is recorded and the launch fails, so the
// library call fails with REG_EDEVICE.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "kernels.hpp"

namespace {
struct Range {
    const char* b;
    size_t n;
};
std::vector<Range> g_ranges;    // the caller's buffers (cleared by mock_reset)
std::vector<Range> g_symbols;   // device symbols the library looked up (kept for the process, as on a GPU)
std::string g_err;
std::mutex g_err_mu;
std::atomic<long> g_launches{0};
std::atomic<long> g_sqdiff_calls{0};
std::atomic<long> g_pcg_update{0}, g_pcg_update_z{0};   // launches of the two PCG update forms
}  // namespace

bool mock_range_ok(const void* p, size_t bytes) {
    if (bytes == 0) return true;
    const char* c = static_cast<const char*>(p);
    for (const std::vector<Range>* v : {&g_ranges, &g_symbols})
        for (const Range& r : *v)
            if (c >= r.b && c + bytes <= r.b + r.n) return true;
    return false;
}
void mock_fail(const char* what) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    if (g_err.empty()) g_err = what;
}
void mock_register_range(const void* p, size_t bytes) { g_symbols.push_back({static_cast<const char*>(p), bytes}); }

extern "C" {
void mock_register(const void* p, size_t bytes) { g_ranges.push_back({static_cast<const char*>(p), bytes}); }
void mock_reset() {
    g_ranges.clear();
    g_err.clear();
    g_launches = 0;
    g_sqdiff_calls = 0;
    g_pcg_update = 0;
    g_pcg_update_z = 0;
}
const char* mock_last_error() { return g_err.c_str(); }
long mock_launches() { return g_launches.load(); }
// launches of launch_pcg_update (z = 0) or launch_pcg_update_z (z = 1) since mock_reset
long mock_pcg_updates(int z) { return z ? g_pcg_update_z.load() : g_pcg_update.load(); }
}

namespace regnk {
namespace {
// check [p, p + count * size) for a non-null p
template <typename T>
bool chk(const T* p, size_t count, const char* what) {
    if (!p || count == 0) return true;
    if (mock_range_ok(p, count * sizeof(T))) return true;
    char buf[160];
    snprintf(buf, sizeof buf, "%s: %zu elements of %zu bytes outside every registered buffer", what, count, sizeof(T));
    mock_fail(buf);
    return false;
}
hipError_t done(bool ok) {
    ++g_launches;
    return ok ? hipSuccess : hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_clk_init(unsigned long long* clk, int pairs, hipStream_t) {
    return done(chk(clk, 2 * (size_t)pairs, "clk_init"));
}

template <typename T>
hipError_t launch_stage(int op, int var, const StageArgs<T>& a, hipStream_t, hipEvent_t, hipEvent_t) {
    const size_t nn = (size_t)a.nn, n2 = 2 * nn;
    bool ok = a.n1 >= 8 && a.n2 >= 8 && (long)a.n1 * a.n2 == a.nn && var >= 0 && var < NUM_STAGE_VARIANTS && op >= 0 &&
              op <= OP_A2F;
    if (!ok) mock_fail("stage: bad sizes, op or launch shape");
    ok &= chk(a.A, (a.flags & F_ZERO) ? 0 : nn, "stage A");
    ok &= chk(a.Bf, nn, "stage Bf");
    ok &= chk(a.V1, nn, "stage V1") && chk(a.V2, nn, "stage V2") && chk(a.X, nn, "stage X");
    ok &= chk(a.VT, n2, "stage VT") && chk(a.G, n2, "stage G") && chk(a.G2, n2, "stage G2");
    ok &= chk(a.LAM, nn, "stage LAM") && chk(a.LAM2, nn, "stage LAM2");
    ok &= chk(a.GT, n2, "stage GT") && chk(a.GT2, n2, "stage GT2");
    ok &= chk(a.ROUT, nn, "stage ROUT") && chk(a.UOUT, nn, "stage UOUT") && chk(a.COUT, nn, "stage COUT");
    ok &= chk(a.GOUT, n2, "stage GOUT") && chk(a.GOUTF, n2, "stage GOUTF") && chk(a.B, n2, "stage B");
    ok &= chk(a.tw1, (size_t)a.n1, "stage tw1") && chk(a.tw2, (size_t)a.n2, "stage tw2");
    ok &= chk(a.dc1, (size_t)a.n1, "stage dc1") && chk(a.dc2, (size_t)a.n2, "stage dc2");
    // 2 slots per block (4 with F_PHASES), at most (n1 + n2) / 2 blocks
    ok &= chk(a.clk, (size_t)((a.flags & F_PHASES) ? 2 : 1) * (a.n1 + a.n2), "stage clk");
    return done(ok);
}
template hipError_t launch_stage<float>(int, int, const StageArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_stage<double>(int, int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);

bool stage_variant_fits_f32(int n1, int n2, int var) {
    if (n1 != n2 || (n1 & (n1 - 1)) != 0 || n1 < 64) return var == 0;
    return var >= 0 && var < NUM_STAGE_VARIANTS;
}

template <typename T>
hipError_t launch_finalize_state(long nn, const double* Q, const double* C, const double* mR, double* m1, T* lam,
                                 hipStream_t) {
    return done(chk(Q, nn, "finalize Q") && chk(C, nn, "finalize C") && chk(mR, nn, "finalize mR") &&
                chk(m1, nn, "finalize m1") && chk(lam, nn, "finalize lam"));
}
template hipError_t launch_finalize_state<float>(long, const double*, const double*, const double*, double*, float*,
                                                 hipStream_t);
template hipError_t launch_finalize_state<double>(long, const double*, const double*, const double*, double*, double*,
                                                  hipStream_t);
template <typename T>
hipError_t launch_body_end(long nn, T, const T* Q, const T* C, const T* G, T* B, hipStream_t) {
    return done(chk(Q, nn, "body_end Q") && chk(C, nn, "body_end C") && chk(G, 2 * nn, "body_end G") &&
                chk(B, 2 * nn, "body_end B"));
}
template hipError_t launch_body_end<float>(long, float, const float*, const float*, const float*, float*, hipStream_t);
template hipError_t launch_body_end<double>(long, double, const double*, const double*, const double*, double*,
                                            hipStream_t);
template <typename T>
hipError_t launch_body_last(long nn, T, bool, const T* Q, const T* C, const T* X, const T* G, const T* G2, T* B,
                            T* keep, hipStream_t) {
    return done(chk(Q, nn, "body_last Q") && chk(C, nn, "body_last C") && chk(X, nn, "body_last X") &&
                chk(G, 2 * nn, "body_last G") && chk(G2, 2 * nn, "body_last G2") && chk(B, 2 * nn, "body_last B") &&
                chk(keep, nn, "body_last keep"));
}
template hipError_t launch_body_last<float>(long, float, bool, const float*, const float*, const float*, const float*,
                                            const float*, float*, float*, hipStream_t);
template hipError_t launch_body_last<double>(long, double, bool, const double*, const double*, const double*,
                                             const double*, const double*, double*, double*, hipStream_t);

// ---- spectral passes: spec holds 4 half spectra of n1 x n2/2 complex doubles ----
namespace {
size_t half(const SpecParams& p) { return (size_t)p.n1 * (p.n2 / 2); }
bool spec_ok(const SpecParams& p, const cpx<double>* spec, int comps, const char* what) {
    return chk(spec, comps * half(p), what);
}
}  // namespace
template <typename TI0, typename TI1>
hipError_t launch_spec_row_fwd2(const SpecParams& p, const TI0* in0, const TI1* in1, cpx<double>* spec,
                                const cpx<double>* tw2, hipStream_t) {
    const size_t n2f = 2 * (size_t)p.n1 * p.n2;
    return done(chk(in0, n2f, "spec_row_fwd in0") && chk(in1, n2f, "spec_row_fwd in1") &&
                spec_ok(p, spec, in1 ? 4 : 2, "spec_row_fwd spec") && chk(tw2, (size_t)p.n2, "spec_row_fwd tw2") &&
                chk(p.eta_sum, 1, "spec eta_sum"));
}
template <typename TI>
hipError_t launch_spec_row_fwd(const SpecParams& p, const TI* in0, const TI* in1, cpx<double>* spec,
                               const cpx<double>* tw2, hipStream_t s) {
    return launch_spec_row_fwd2<TI, TI>(p, in0, in1, spec, tw2, s);
}
template hipError_t launch_spec_row_fwd<float>(const SpecParams&, const float*, const float*, cpx<double>*,
                                               const cpx<double>*, hipStream_t);
template hipError_t launch_spec_row_fwd<double>(const SpecParams&, const double*, const double*, cpx<double>*,
                                                const cpx<double>*, hipStream_t);
template hipError_t launch_spec_row_fwd2<double, float>(const SpecParams&, const double*, const float*, cpx<double>*,
                                                        const cpx<double>*, hipStream_t);
template hipError_t launch_spec_row_fwd2<double, double>(const SpecParams&, const double*, const double*,
                                                         cpx<double>*, const cpx<double>*, hipStream_t);
template <typename T>
hipError_t launch_spec_row_fwd_body(const SpecParams& p, const double* in0, T* B, const BodyLast<T>& bl,
                                    cpx<double>* spec, const cpx<double>* tw2, hipStream_t s) {
    const size_t nn = (size_t)p.n1 * p.n2;
    if (bl.Q && !(chk(bl.Q, nn, "row_fwd_body Q") && chk(bl.C, nn, "row_fwd_body C") &&
                  chk(bl.X, nn, "row_fwd_body X") && chk(bl.G, 2 * nn, "row_fwd_body G") &&
                  chk(bl.G2, 2 * nn, "row_fwd_body G2")))
        return done(false);
    if (!B) {
        mock_fail("row_fwd_body: NULL body force");
        return done(false);
    }
    return launch_spec_row_fwd2<double, T>(p, in0, B, spec, tw2, s);
}
template hipError_t launch_spec_row_fwd_body<float>(const SpecParams&, const double*, float*, const BodyLast<float>&,
                                                    cpx<double>*, const cpx<double>*, hipStream_t);
template hipError_t launch_spec_row_fwd_body<double>(const SpecParams&, const double*, double*,
                                                     const BodyLast<double>&, cpx<double>*, const cpx<double>*,
                                                     hipStream_t);
hipError_t launch_spec_col(const SpecParams& p, int mode, bool have_y, bool want2, cpx<double>* spec,
                           const cpx<double>* tw1, hipStream_t) {
    bool mode_ok = mode >= SPEC_PROJ && mode <= SPEC_HESS_P;
    if (mode == SPEC_HESS_P) mode_ok &= spec_col_hess_p_ok(p.n1, p.n2);
    if (!mode_ok) mock_fail("spec_col: bad mode (or SPEC_HESS_P on a grid without the four-spectra kernel)");
    const int slots = (mode == SPEC_HESS_P && want2) ? 6 : ((have_y || want2) ? 4 : 2);
    return done(mode_ok && spec_ok(p, spec, slots, "spec_col spec") && chk(tw1, (size_t)p.n1, "spec_col tw1") &&
                chk(p.eta_sum, 1, "spec eta_sum"));
}
hipError_t launch_spec_row_inv4_dot(const SpecParams& p, const cpx<double>* spec, double* const* out, int nf,
                                    const cpx<double>* tw2, const RowDot& d, hipStream_t) {
    const size_t n2f = 2 * (size_t)p.n1 * p.n2;
    const bool p2 = (p.n2 & (p.n2 - 1)) == 0;
    bool ok = nf >= 1 && nf <= 4 && p2 && (!d.s || (d.partial && d.count && d.field >= 0 && d.field < nf));
    if (!ok) mock_fail("spec_row_inv4: bad field count, grid or dot");
    for (int f = 0; ok && f < nf; ++f) ok &= out[f] != nullptr && chk(out[f], n2f, "spec_row_inv4 out");
    if (ok && d.s) {
        *d.count = p.n1;
        ok &= chk(d.s, n2f, "spec_row_inv4 dot s") && chk(d.partial, (size_t)p.n1, "spec_row_inv4 dot partial");
    }
    return done(ok && spec_ok(p, spec, 2 * nf, "spec_row_inv4 spec") && chk(tw2, (size_t)p.n2, "spec_row_inv4 tw2"));
}
hipError_t launch_spec_row_inv2(const SpecParams& p, const cpx<double>* spec, double* out0, double* out1,
                                const cpx<double>* tw2, hipStream_t) {
    const size_t n2f = 2 * (size_t)p.n1 * p.n2;
    return done(spec_ok(p, spec, out1 ? 4 : 2, "spec_row_inv spec") && chk(out0, n2f, "spec_row_inv out0") &&
                chk(out1, n2f, "spec_row_inv out1") && chk(tw2, (size_t)p.n2, "spec_row_inv tw2"));
}
// one partial per row at most (the real pass writes one per block of rows, only for power-of-two n2)
hipError_t launch_spec_row_inv2_dot(const SpecParams& p, const cpx<double>* spec, double* out0, double* out1,
                                    const cpx<double>* tw2, const RowDot& d, hipStream_t s) {
    const size_t n2f = 2 * (size_t)p.n1 * p.n2;
    if (!d.s || !d.partial || !d.count || d.field < 0 || d.field > (out1 ? 1 : 0)) {
        mock_fail("spec_row_inv dot: bad arguments");
        return done(false);
    }
    const bool p2 = (p.n2 & (p.n2 - 1)) == 0;
    *d.count = p2 ? p.n1 : 0;
    if (!(chk(d.s, n2f, "spec_row_inv dot s") && chk(d.partial, (size_t)*d.count, "spec_row_inv dot partial")))
        return done(false);
    return launch_spec_row_inv2(p, spec, out0, out1, tw2, s);
}

size_t nyquist_scratch_doubles(int n1, int n2) {   // the real launcher's formula (32 x 64 tiles)
    const size_t ncb = (n2 + 63) / 64, nrb = (n1 + 31) / 32;
    return 2 * ncb * n1 + 2 * nrb * n2 + 2 * nrb * ncb;
}
template <typename TO>
hipError_t launch_nyquist_project(int n1, int n2, const double* in, double* out_d, TO* out_t, double* scratch,
                                  hipStream_t) {
    const size_t n2f = 2 * (size_t)n1 * n2;
    return done(chk(in, n2f, "nyquist in") && chk(out_d, n2f, "nyquist out_d") && chk(out_t, n2f, "nyquist out_t") &&
                chk(scratch, nyquist_scratch_doubles(n1, n2), "nyquist scratch"));
}
template hipError_t launch_nyquist_project<float>(int, int, const double*, double*, float*, double*, hipStream_t);
template hipError_t launch_nyquist_project<double>(int, int, const double*, double*, double*, double*, hipStream_t);

// ---- reductions and vector updates ----
hipError_t launch_finalize_scalar(int nk, int count, const double* partial, double* out, int mode, double* scal,
                                  hipStream_t) {
    bool ok = nk >= 1 && count >= 1 && mode >= PCG_INIT && mode <= PCG_MU;
    if (!ok) mock_fail("finalize_scalar: bad counts or mode");
    ok = ok && chk(partial, (size_t)nk * count, "finalize_scalar partial") && chk(out, (size_t)nk, "finalize_scalar out") &&
         chk(scal, (size_t)NUM_PCG_SLOTS, "finalize_scalar scalars");
    if (ok) {   // the placeholders of launch_dots_scalar
        for (int k = 0; k < nk; ++k) out[k] = 1.0;
        if (mode == PCG_INIT) {
            scal[S_ACTIVE] = 1.0;
            scal[S_ITER] = 0.0;
            scal[S_BREAK] = 0.0;
        } else if (mode == PCG_KAPPA) {
            scal[S_ITER] += 1.0;
        }
    }
    return done(ok);
}
template <typename TI>
hipError_t launch_dots(int nk, const TI* const* a, const TI* const* b, long n, double* partial, double* out,
                       hipStream_t) {
    bool ok = nk >= 1 && nk <= 4;
    for (int k = 0; ok && k < nk; ++k) ok &= chk(a[k], n, "dots a") && chk(b[k], n, "dots b");
    ok &= chk(partial, (size_t)nk * RED_BLOCKS, "dots partial") && chk(out, nk, "dots out");
    if (ok)   // norms positive, cross terms (a line search's slope) negative
        for (int k = 0; k < nk; ++k) out[k] = a[k] == b[k] ? 1.0 : -1.0;
    return done(ok);
}
template hipError_t launch_dots<double>(int, const double* const*, const double* const*, long, double*, double*,
                                        hipStream_t);
template hipError_t launch_dots<float>(int, const float* const*, const float* const*, long, double*, double*,
                                       hipStream_t);
template <typename TI>
hipError_t launch_sqdiff(const TI* x, const TI* y, long n, double* partial, double* out, hipStream_t) {
    const bool ok = chk(x, n, "sqdiff x") && chk(y, n, "sqdiff y") && chk(partial, RED_BLOCKS, "sqdiff partial") &&
                    chk(out, 1, "sqdiff out");
    if (ok) out[0] = 1e6 - (double)(++g_sqdiff_calls);   // a misfit that falls call by call: line searches accept
    return done(ok);
}
template hipError_t launch_sqdiff<double>(const double*, const double*, long, double*, double*, hipStream_t);
template hipError_t launch_sqdiff<float>(const float*, const float*, long, double*, double*, hipStream_t);
hipError_t launch_axpby(long n, double, const double* x, double, double* y, hipStream_t) {
    return done(chk(x, n, "axpby x") && chk(y, n, "axpby y"));
}
hipError_t launch_add_scaled(long n, const double* x, double, const double* y, double* z, hipStream_t) {
    return done(chk(x, n, "add_scaled x") && chk(y, n, "add_scaled y") && chk(z, n, "add_scaled z"));
}
template <typename TO>
hipError_t launch_convert(long n, const double* in, TO* out, hipStream_t) {
    return done(chk(in, n, "convert in") && chk(out, n, "convert out"));
}
template hipError_t launch_convert<float>(long, const double*, float*, hipStream_t);
template hipError_t launch_convert<double>(long, const double*, double*, hipStream_t);
template <typename TI>
hipError_t launch_widen(long n, const TI* in, double* out, hipStream_t) {
    return done(chk(in, n, "widen in") && chk(out, n, "widen out"));
}
template hipError_t launch_widen<float>(long, const float*, double*, hipStream_t);
template hipError_t launch_widen<double>(long, const double*, double*, hipStream_t);
hipError_t launch_fill(long n, double v, double* y, hipStream_t) {
    const bool ok = chk(y, n, "fill y");
    if (ok && n <= 64)
        for (long i = 0; i < n; ++i) y[i] = v;   // small fills are device counters the driver relies on
    return done(ok);
}

// ---- low-rank correction ----
hipError_t launch_lr_dots(long n, const double* x, const double* F, long stride, const double* cnt, int cap,
                          double* partial, double* out, hipStream_t) {
    return done(chk(x, n, "lr_dots x") && chk(F, (size_t)(cap - 1) * stride + n, "lr_dots F") &&
                chk(cnt, 1, "lr_dots cnt") && chk(partial, (size_t)cap * RED_BLOCKS, "lr_dots partial") &&
                chk(out, cap, "lr_dots out"));
}
hipError_t launch_lr_combine(long n, const double* base, double* out, const double* F, long stride, const double* cnt,
                             int cap, const double* da, const double* db, const double* e, double, hipStream_t) {
    return done(chk(base, n, "lr_combine base") && chk(out, n, "lr_combine out") &&
                chk(F, cap > 0 ? (size_t)(cap - 1) * stride + n : 0, "lr_combine F") && chk(cnt, 1, "lr_combine cnt") &&
                chk(da, cap, "lr_combine da") && chk(db, cap, "lr_combine db") && chk(e, cap, "lr_combine e"));
}
hipError_t launch_lr_mix(long n, double* F, long stride, int rin, int rout, const LrMix&, hipStream_t) {
    const int r = rin > rout ? rin : rout;
    return done(chk(F, r > 0 ? (size_t)(r - 1) * stride + n : 0, "lr_mix F"));
}

// ---- shear-control model ----
hipError_t launch_stokes_first(long nn, const double* dv, double, double, double* sig, double* E, double* eta,
                               double* dens, hipStream_t) {
    return done(chk(dv, 4 * nn, "stokes_first dv") && chk(sig, 3 * nn, "stokes_first sig") &&
                chk(E, 3 * nn, "stokes_first E") && chk(eta, nn, "stokes_first eta") && chk(dens, nn, "stokes_first dens"));
}
hipError_t launch_stokes_second(long nn, const double* dvt, const double* E, const double* eta, double, double,
                                double* sig, hipStream_t) {
    return done(chk(dvt, 4 * nn, "stokes_second dv") && chk(E, 3 * nn, "stokes_second E") &&
                chk(eta, nn, "stokes_second eta") && chk(sig, 3 * nn, "stokes_second sig"));
}
hipError_t launch_stokes_div(long nn, const double* ds, double, double* out, hipStream_t) {
    return done(chk(ds, 6 * nn, "stokes_div ds") && chk(out, 2 * nn, "stokes_div out"));
}

// ---- deformation diagnostics ----
hipError_t launch_deform_source(long nn, double, const double* v, const double* dv, const DefPtrs& p, hipStream_t) {
    bool ok = chk(v, 2 * nn, "deform_source v") && chk(dv, 4 * nn, "deform_source dv");
    for (int c = 0; c < 4; ++c) ok &= chk(p.a[c], nn, "deform_source a") && chk(p.b[c], nn, "deform_source b");
    for (int c = 0; c < 6; ++c) ok &= chk(p.out[c], nn, "deform_source out");
    return done(ok);
}
hipError_t launch_deform_final(long nn, const DefPairs& p, double* u1, double* F1, double* det, hipStream_t) {
    bool ok = chk(u1, 2 * nn, "deform_final u1") && chk(F1, 4 * nn, "deform_final F1") && chk(det, nn, "deform_final det");
    for (int c = 0; c < 6; ++c) ok &= chk(p.r[c], nn, "deform_final r") && chk(p.c[c], nn, "deform_final c");
    return done(ok);
}
hipError_t launch_minmaxsum(const double* x, long n, double* partial, double* out3, hipStream_t) {
    const bool ok = chk(x, n, "minmaxsum x") && chk(partial, 3 * (size_t)RED_BLOCKS, "minmaxsum partial") &&
                    chk(out3, 3, "minmaxsum out");
    if (ok) {
        out3[0] = -1.0;
        out3[1] = 1.0;
        out3[2] = (double)n;
    }
    return done(ok);
}

// ---- PCG ----
hipError_t launch_dots_scalar(int nk, const double* const* a, const double* const* b, long n, double* partial,
                              double* out, int mode, double* scal, hipStream_t) {
    bool ok = nk >= 1 && nk <= 4 && mode >= PCG_INIT && mode <= PCG_MU;
    for (int k = 0; ok && k < nk; ++k) ok &= chk(a[k], n, "dots_scalar a") && chk(b[k], n, "dots_scalar b");
    ok &= chk(partial, (size_t)nk * RED_BLOCKS, "dots_scalar partial") && chk(out, nk, "dots_scalar out") &&
          chk(scal, NUM_PCG_SLOTS, "dots_scalar scal");
    if (ok) {
        for (int k = 0; k < nk; ++k) out[k] = 1.0;
        if (mode == PCG_INIT) {
            scal[S_ACTIVE] = 1.0;
            scal[S_ITER] = 0.0;
            scal[S_BREAK] = 0.0;
        } else if (mode == PCG_KAPPA) {
            scal[S_ITER] += 1.0;
        }
    }
    return done(ok);
}
hipError_t launch_pcg_update(long n, double* x, double* r, const double* s, const double* st, const double* scal,
                             hipStream_t) {
    ++g_pcg_update;
    return done(chk(x, n, "pcg_update x") && chk(r, n, "pcg_update r") && chk(s, n, "pcg_update s") &&
                chk(st, n, "pcg_update st") && chk(scal, NUM_PCG_SLOTS, "pcg_update scal"));
}
hipError_t launch_pcg_update_z(long n, double* x, double* r, const double* s, const double* st, double* z,
                               const double* pst, double* kr, const double* kst, const double* scal, double* partial,
                               hipStream_t) {
    ++g_pcg_update_z;
    const bool ok_k = (kr == nullptr) == (kst == nullptr);
    if (!ok_k) mock_fail("pcg_update_z: kr and kst must come together");
    return done(ok_k && chk(x, n, "pcg_update_z x") && chk(r, n, "pcg_update_z r") && chk(s, n, "pcg_update_z s") &&
                chk(st, n, "pcg_update_z st") && chk(z, n, "pcg_update_z z") && chk(pst, n, "pcg_update_z pst") &&
                chk(kr, n, "pcg_update_z kr") && chk(kst, n, "pcg_update_z kst") &&
                chk(scal, NUM_PCG_SLOTS, "pcg_update_z scal") &&
                chk(partial, 2 * RED_BLOCKS, "pcg_update_z partial"));
}
template <typename T>
hipError_t launch_pcg_dir_copy(long n, double* s, T* sT, const double* z, const double* scal, hipStream_t) {
    return done(chk(s, n, "dir_copy s") && chk(sT, n, "dir_copy sT") && chk(z, n, "dir_copy z") &&
                chk(scal, scal ? NUM_PCG_SLOTS : 0, "dir_copy scal"));
}
template hipError_t launch_pcg_dir_copy<float>(long, double*, float*, const double*, const double*, hipStream_t);
template hipError_t launch_pcg_dir_copy<double>(long, double*, double*, const double*, const double*, hipStream_t);

}  // namespace regnk
