// Host side of the registration library: C ABI, workspace layout, and the drivers that sequence
// the device passes into the state / adjoint / incremental solves, the Hessian matvec, the gradient,
// the objective, PCG (Alg. 2) and the Newton loop (Alg. 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "regnk.h"
#include "device_common.hpp"
#include "kernels.hpp"
#include "host_common.hpp"

using namespace regnk;

// ---------------------------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------------------------
static thread_local std::string g_err = "no error";

reg_status regnk::fail(reg_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

// ---------------------------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------------------------
namespace {

constexpr int NFIELD = 9;    // scalar scratch fields in transport precision
constexpr int NSFIELD = 8;   // FP64 state-solve scratch fields
constexpr int NPCG = 8;      // x, r, z, kr, s, st, kst, P^{-1} st
constexpr int NSCAL = 32;
constexpr int MAX_TIMED = 512;   // timed stage launches per reg_time_pass call
// shear-control model, FP64 fields: partials dv (4), stress (3), stress gradients (6), E (3) and eta (1)
// at the linearisation point, integrand (1), regularisation term (2)
// and the mass-source penalty's gradient (2)
enum { STK_DV = 0, STK_SIG = 4, STK_DS = 7, STK_E = 13, STK_ETA = 16, STK_DENS = 17, STK_R = 18, STK_PEN = 20,
       STK_FIELDS = 22 };
// device scalars: {min, max, sum} of the shear-control viscosity at the linearisation point
constexpr int SC_ETA = 28;
// scalars of the low-rank correction: valid-slot count, a spare count, e_k, <z_k, r>_W, <Hz_k, y>_W
enum { LRS_CNT = 0, LRS_CNT2 = 1, LRS_E = 8, LRS_DA = LRS_E + LR_MAX, LRS_DB = LRS_DA + LR_MAX,
       LRS_G = LRS_DB + LR_MAX, LRS_N = LRS_G + LR_MIX_MAX * LR_MIX_MAX };

struct Layout {
    size_t total = 0;
    size_t take(size_t bytes) {
        size_t off = total;
        total += (bytes + 255) & ~size_t(255);
        return off;
    }
};

struct Offsets {
    size_t mT, mR, vT, vw, vtT, traj, fld[NFIELD], B, Bt;
    size_t mT64, mR64, sfld[NSFIELD];   // FP64 state-solve buffers (FP32 transport mode only)
    size_t tw1f, tw2f, tw1d, tw2d, dc1f, dc2f, dc1d, dc2d;
    size_t v64, vtrial, g64, kg64, vt64, tmp0, tmp1, vcur, vtry, rhs, pcg[NPCG], spec, partial, scal, clk;
    size_t lr[4], lrtmp, lrsc, lrpart;   // low-rank correction: sets Z, HZ, K^-1 Z, K^-1 HZ; scratch
    size_t lamtraj, gmt;                 // full Newton: lam_{j+1}, lam*_j; grad m~_j, grad m~*_j
    size_t stk;                          // shear-control model: FP64 fields (see stokes_*)
    size_t total;
};

bool is_even_in_range(int n) { return n >= 8 && n <= 2048 && n % 2 == 0; }

reg_status check_params(const reg_params* p) {
    if (!p) return fail(REG_EINVAL, "params is NULL");
    if (!is_even_in_range(p->n1) || !is_even_in_range(p->n2))
        return fail(REG_EINVAL, "n1=%d n2=%d: grid sizes must be even and in [8, 2048]", p->n1, p->n2);
    if (p->nt < 1 || p->nt > 4096) return fail(REG_EINVAL, "nt=%d out of range [1, 4096]", p->nt);
    if (p->norm < REG_H1 || p->norm > REG_STOKES) return fail(REG_EINVAL, "norm=%d", p->norm);
    if (p->norm == REG_STOKES) {
        if (!(p->stokes_nu > 0.0 && std::isfinite(p->stokes_nu)) || !(p->stokes_eps > 0.0 && std::isfinite(p->stokes_eps)))
            return fail(REG_EINVAL, "REG_STOKES needs stokes_nu > 0 and stokes_eps > 0");
    } else if (p->stokes_nu != 0.0 || p->stokes_eps != 0.0) {
        return fail(REG_EINVAL, "stokes_nu and stokes_eps must be 0 unless norm is REG_STOKES");
    }
    if (p->constraint < REG_UNCONSTRAINED || p->constraint > REG_MASS_SOURCE)
        return fail(REG_EINVAL, "constraint=%d", p->constraint);
    if (p->precision != REG_FP64 && p->precision != REG_FP32_TRANSPORT)
        return fail(REG_EINVAL, "precision=%d", p->precision);
    if (p->adjoint != REG_ADJ_DISCRETE && p->adjoint != REG_ADJ_PAPER)
        return fail(REG_EINVAL, "adjoint=%d", p->adjoint);
    if (p->hessian != REG_HESS_GN && p->hessian != REG_HESS_FULL) return fail(REG_EINVAL, "hessian=%d", p->hessian);
    if (p->hessian == REG_HESS_FULL && p->adjoint != REG_ADJ_DISCRETE)
        return fail(REG_EINVAL, "the full-Newton Hessian needs adjoint = REG_ADJ_DISCRETE");
    if (p->nt_max != 0 && (p->nt_max < p->nt || p->nt_max > 4096))
        return fail(REG_EINVAL, "nt_max=%d: must be 0 or in [nt=%d, 4096]", p->nt_max, p->nt);
    if (p->lowrank_capacity < 0 || p->lowrank_capacity > LR_MAX)
        return fail(REG_EINVAL, "lowrank_capacity=%d out of range [0, %d]", p->lowrank_capacity, LR_MAX);
    if (!(p->beta_v > 0.0) || !std::isfinite(p->beta_v)) return fail(REG_EINVAL, "beta_v must be > 0");
    const bool ms = p->constraint == REG_MASS_SOURCE;
    if (ms && !(p->beta_w > 0.0 && std::isfinite(p->beta_w)))
        return fail(REG_EINVAL, "beta_w must be > 0 for the mass-source model");
    if (!ms && p->beta_w != 0.0) return fail(REG_EINVAL, "beta_w must be 0 unless constraint is REG_MASS_SOURCE");
    return REG_OK;
}

// timing slots per stage launch: one per block, at most (n1 + n2) / 2 blocks
size_t clk_slots(const reg_params* p) { return (size_t)(p->n1 + p->n2) / 2; }

// time steps the workspace holds: n_t, or the largest n_t the CFL adaptation may reach
int nt_capacity(const reg_params* p) { return p->nt_max > p->nt ? p->nt_max : p->nt; }

Offsets layout(const reg_params* p) {
    Offsets o{};
    Layout L;
    const size_t nn = (size_t)p->n1 * p->n2;
    const size_t ts = p->precision == REG_FP64 ? 8 : 4;
    const size_t ntc = (size_t)nt_capacity(p);
    o.mT = L.take(nn * ts);
    o.mR = L.take(nn * ts);
    o.vT = L.take(2 * nn * ts);
    o.vw = L.take(2 * nn * ts);
    o.vtT = L.take(2 * nn * ts);
    o.traj = L.take((2 * ntc + 1) * 2 * nn * ts);
    for (int i = 0; i < NFIELD; ++i) o.fld[i] = L.take(nn * ts);
    o.B = L.take(2 * nn * ts);
    o.Bt = L.take(2 * nn * ts);
    const size_t s64 = p->precision == REG_FP64 ? 0 : nn * 8;
    o.mT64 = L.take(s64);
    o.mR64 = L.take(s64);
    for (int i = 0; i < NSFIELD; ++i) o.sfld[i] = L.take(s64);
    o.tw1f = L.take(p->n1 * 8);
    o.tw2f = L.take(p->n2 * 8);
    o.tw1d = L.take(p->n1 * 16);
    o.tw2d = L.take(p->n2 * 16);
    o.dc1f = L.take(p->n1 * 4);
    o.dc2f = L.take(p->n2 * 4);
    o.dc1d = L.take(p->n1 * 8);
    o.dc2d = L.take(p->n2 * 8);
    o.v64 = L.take(2 * nn * 8);
    o.vtrial = L.take(2 * nn * 8);
    o.g64 = L.take(2 * nn * 8);
    o.kg64 = L.take(2 * nn * 8);
    o.vt64 = L.take(2 * nn * 8);
    o.tmp0 = L.take(2 * nn * 8);
    o.tmp1 = L.take(2 * nn * 8);
    o.vcur = L.take(2 * nn * 8);
    o.vtry = L.take(2 * nn * 8);
    o.rhs = L.take(2 * nn * 8);
    for (int i = 0; i < NPCG; ++i) o.pcg[i] = L.take(2 * nn * 8);
    o.spec = L.take(6 * (size_t)p->n1 * (p->n2 / 2) * 16);   // 6 half spectra (SPEC_HESS_P)
    static_assert(4 * RED_BLOCKS >= 2048, "partials: one per row of the largest grid (RowDot)");
    o.partial = L.take(4 * RED_BLOCKS * 8);
    o.scal = L.take(NSCAL * 8);
    o.clk = L.take((size_t)MAX_TIMED * 2 * clk_slots(p) * sizeof(unsigned long long));
    // low-rank correction: Z and H Z (and their K^{-1} images for the mass-source model)
    const size_t cap = (size_t)p->lowrank_capacity;
    const int sets = p->constraint == REG_MASS_SOURCE ? 4 : 2;
    for (int i = 0; i < 4; ++i) o.lr[i] = L.take(i < sets ? cap * 2 * nn * 8 : 0);
    o.lrtmp = L.take(cap ? 2 * nn * 8 : 0);
    o.lrsc = L.take(cap ? LRS_N * 8 : 0);
    o.lrpart = L.take(cap ? (size_t)LR_MAX * RED_BLOCKS * 8 : 0);
    const bool full = p->hessian == REG_HESS_FULL;
    o.lamtraj = L.take(full ? 2 * ntc * nn * ts : 0);
    o.gmt = L.take(full ? 2 * ntc * 2 * nn * ts : 0);
    o.stk = L.take(p->norm == REG_STOKES ? (size_t)STK_FIELDS * nn * 8 : 0);
    o.total = L.total;
    return o;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Problem handle
// ---------------------------------------------------------------------------------------------
struct reg_problem {
    reg_params p;
    hipStream_t stream;
    int n1, n2, nt;
    long nn;
    bool f64;
    char* ws;
    Offsets o;
    bool linearized = false;
    bool matvec_done = false;
    SpecParams sp;
    double h1h2;
    int var[NUM_TUNED_OPS] = {};   // launch-shape variant per stage op (FP32 square grids)
    // Captured Hessian-matvec launch sequences, one per (input, output, K^-1 output) pointer set.
    struct MvGraph {
        const double* in = nullptr;
        double* out = nullptr;
        double* kout = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    static constexpr int NGRAPH = 4;
    MvGraph graph[NGRAPH];
    hipGraphExec_t lr_graph[LR_MIX_MAX] = {};   // H z_k of the Rayleigh-Ritz basis slots (fixed pointers)
    int graph_next = 0;
    bool use_graphs = true;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t pcg_iter_graph = nullptr;   // one PCG iteration (matvec + scalar updates)
    hipGraphExec_t pcg_iter_graph_lr = nullptr;   // the same with the low-rank correction
    hipGraphExec_t pcg_iter_graph_ex = nullptr;   // the iteration that forms z = P^{-1} r afresh
    bool lr_active = false;   // PCG applies the low-rank correction (inside reg_solve only)
    int lr_count = 0;         // valid directions (host copy of the device count)
    // measurement hook: hipEvents around every launch of one stage op during real matvecs
    int timing_op = -1;
    int clk_used = 0;   // timed launches recorded so far (reg_time_pass)
    int clk_max = 0;    // timed launches the stamp buffer holds in the current mode
    bool clk_phases = false;   // four stamps per block (reg_time_phases)
    size_t clk_stride = 0;
    std::vector<hipEvent_t> tev;   // dispatch-stamped start / end events of the timed launches

    template <typename X>
    X* at(size_t off) const { return reinterpret_cast<X*>(ws + off); }
    double* pcg(int i) const { return at<double>(o.pcg[i]); }
    // FP64 state solve: template, reference and scratch fields (the transport buffers in FP64 mode)
    double* sT() const { return at<double>(f64 ? o.mT : o.mT64); }
    double* sR() const { return at<double>(f64 ? o.mR : o.mR64); }
    double* sF(int i) const { return at<double>(f64 ? o.fld[i] : o.sfld[i]); }
    double* scal() const { return at<double>(o.scal); }
    double* partial() const { return at<double>(o.partial); }
    double* lr_set(int set) const { return at<double>(o.lr[set]); }
    double* lr_slot(int set, int k) const { return lr_set(set) + (size_t)k * 2 * nn; }
    double* lr_sc() const { return at<double>(o.lrsc); }
    cpx<double>* spec() const { return at<cpx<double>>(o.spec); }
};

namespace {

// ---- typed views ------------------------------------------------------------------------------
template <typename T>
struct TV {
    const reg_problem* P;
    T* mT() const { return P->at<T>(P->o.mT); }
    T* mR() const { return P->at<T>(P->o.mR); }
    T* vT() const { return P->at<T>(P->o.vT); }
    T* vw() const { return P->at<T>(P->o.vw); }
    T* vtT() const { return P->at<T>(P->o.vtT); }
    T* G(int slot) const { return P->at<T>(P->o.traj) + (size_t)slot * 2 * P->nn; }
    T* F(int i) const { return P->at<T>(P->o.fld[i]); }
    T* B() const { return P->at<T>(P->o.B); }
    T* Bt() const { return P->at<T>(P->o.Bt); }
    // full Newton: lam_{j+1} at slot j, lam*_j at slot n_t + j; grad m~_j at slot j (j >= 1),
    // grad m~*_j at slot n_t + j
    T* Lam(int slot) const { return P->at<T>(P->o.lamtraj) + (size_t)slot * P->nn; }
    T* Gm(int slot) const { return P->at<T>(P->o.gmt) + (size_t)slot * 2 * P->nn; }
    const cpx<T>* tw1() const;
    const cpx<T>* tw2() const;
    const T* dc1() const { return P->at<T>(sizeof(T) == 8 ? P->o.dc1d : P->o.dc1f); }
    const T* dc2() const { return P->at<T>(sizeof(T) == 8 ? P->o.dc2d : P->o.dc2f); }
};
template <>
const cpx<float>* TV<float>::tw1() const { return P->at<cpx<float>>(P->o.tw1f); }
template <>
const cpx<float>* TV<float>::tw2() const { return P->at<cpx<float>>(P->o.tw2f); }
template <>
const cpx<double>* TV<double>::tw1() const { return P->at<cpx<double>>(P->o.tw1d); }
template <>
const cpx<double>* TV<double>::tw2() const { return P->at<cpx<double>>(P->o.tw2d); }

// Gradient-trajectory slots: G_j at slot j (j = 0..nt), G*_j at slot nt + 1 + j (j < nt).
inline int slot_G(const reg_problem* P, int j) { (void)P; return j; }
inline int slot_Gs(const reg_problem* P, int j) { return P->nt + 1 + j; }

template <typename T>
StageArgs<T> base_args(const reg_problem* P) {
    TV<T> tv{P};
    StageArgs<T> a{};
    a.n1 = P->n1;
    a.n2 = P->n2;
    a.nn = P->nn;
    a.h = T(1.0 / P->nt);
    a.tw1 = tv.tw1();
    a.tw2 = tv.tw2();
    a.dc1 = tv.dc1();
    a.dc2 = tv.dc2();
    a.mr1 = P->sp.mr1;
    a.mr2 = P->sp.mr2;
    return a;
}

template <typename T>
reg_status stage(reg_problem* P, int op, const StageArgs<T>& a) {
    const int var = P->var[op_base(op)];
    if (op == P->timing_op && P->clk_used < P->clk_max && 2 * (size_t)P->clk_used + 2 <= P->tev.size()) {
        StageArgs<T> t = a;   // the blocks stamp their own start and end; the dispatch stamps two events
        t.clk = P->at<unsigned long long>(P->o.clk) + P->clk_stride * P->clk_used;
        if (P->clk_phases) t.flags |= F_PHASES;
        CK(launch_stage<T>(op, var, t, P->stream, P->tev[2 * P->clk_used], P->tev[2 * P->clk_used + 1]));
        ++P->clk_used;
    } else {
        CK(launch_stage<T>(op, var, a, P->stream));
    }
    return REG_OK;
}

// Every stage result is kept as the pair (R, C) of its row and column parts; the next stage
// rebuilds u = R + C pointwise.  Scratch roles: (Ra, Ca) current pair, P/E stage-1 pair, U the
// materialised stage input, (Rb, Cb) next pair.
struct Pair {
    int r, c;
};

// ---- state solve forward (eq. (state-eq-elim)) ----------------------------------------------------
// Always in FP64: the stored gradients feed every later matvec, and FP32 round-off in the state is
// amplified by the spectral derivative (and by Heun's growth at high wavenumbers) into G = grad m.
// v: FP64 velocity (2 nn).  store: write G_j, G*_j (and G_nt in paper mode) to the trajectory in the
// transport precision T.  m1: FP64 output field (sF(7)).  lam1 (nullable): lam(1) = m_R - m_1 in T.
template <typename T>
void set_gout(StageArgs<double>& a, T* g) {
    if constexpr (sizeof(T) == 8) a.GOUT = reinterpret_cast<double*>(g);
    else a.GOUTF = reinterpret_cast<float*>(g);
}

template <typename T>
reg_status state_forward(reg_problem* P, const double* v, bool store, double* m1, T* lam1) {
    TV<T> tv{P};
    const long nn = P->nn;
    Pair cur{0, 1}, nxt{5, 6};
    for (int j = 0; j < P->nt; ++j) {
        T* G = store ? tv.G(slot_G(P, j)) : nullptr;
        T* Gs = store ? tv.G(slot_Gs(P, j)) : nullptr;
        StageArgs<double> s1 = base_args<double>(P);
        s1.A = j == 0 ? P->sT() : P->sF(cur.r);
        s1.Bf = j == 0 ? nullptr : P->sF(cur.c);
        s1.V1 = v; s1.V2 = v + nn;
        s1.ROUT = P->sF(2); s1.UOUT = P->sF(4); s1.COUT = P->sF(3);
        set_gout<T>(s1, G);
        CKS(stage<double>(P, OP_S1, s1));
        StageArgs<double> s2 = base_args<double>(P);
        s2.A = P->sF(2); s2.Bf = P->sF(3); s2.X = P->sF(4);
        s2.V1 = v; s2.V2 = v + nn;
        s2.ROUT = P->sF(nxt.r); s2.COUT = P->sF(nxt.c);
        set_gout<T>(s2, Gs);
        CKS(stage<double>(P, OP_S2, s2));
        std::swap(cur, nxt);
    }
    CK(launch_finalize_state<T>(nn, P->sF(cur.r), P->sF(cur.c), P->sR(), m1, lam1, P->stream));
    if (store && P->p.adjoint == REG_ADJ_PAPER) {   // G_{n_t} for the trapezoid end point
        StageArgs<double> g = base_args<double>(P);
        g.A = m1;
        set_gout<T>(g, tv.G(slot_G(P, P->nt)));
        CKS(stage<double>(P, OP_GRAD, g));
    }
    return REG_OK;
}

// ---- adjoint solve backward (eq. (adj-eq-elim)); also the GN incremental adjoint ------------------
// Terminal value lam(1) = sign (TA + TB) (TB nullable).  B: body force (vector, overwritten) in the
// selected quadrature, using the stored trajectory.  Full Newton: keep = true stores the stage values
// lam_{j+1}, lam*_j (the gradient's adjoint sweep); vt != nullptr runs the full-Newton incremental
// adjoint (stages OP_A1F / OP_A2F with the stored lam and grad m~).  defer (nullable): the last
// step's body-force term of the exact-transpose quadrature is returned there instead of launched,
// for the assembly to apply while it loads B (launch_spec_row_fwd_body).
template <typename T>
reg_status adjoint_backward(reg_problem* P, const T* v, const T* TA, const T* TB, bool negate, T* B,
                            bool keep = false, const T* vt = nullptr, BodyLast<T>* defer = nullptr) {
    TV<T> tv{P};
    const long nn = P->nn;
    const T h = T(1.0 / P->nt);
    const bool paper = P->p.adjoint == REG_ADJ_PAPER;
    // the terminal pair may live in scratch fields 0/1 or 5/6: write the first result elsewhere
    Pair nxt = (TA == tv.F(5) || TA == tv.F(6)) ? Pair{0, 1} : Pair{5, 6};
    const T* A = TA;
    const T* Bf = TB;
    for (int j = P->nt - 1; j >= 0; --j) {
        const bool first = j == P->nt - 1;
        StageArgs<T> s1 = base_args<T>(P);
        s1.A = A; s1.Bf = Bf; s1.flags = (first && negate) ? F_NEG : 0;
        s1.V1 = v; s1.V2 = v + nn;
        T* u1 = keep ? tv.Lam(j) : tv.F(4);   // lam_{j+1} (materialised by stage 1)
        s1.ROUT = tv.F(2); s1.UOUT = u1; s1.COUT = tv.F(3);
        if (paper) {
            s1.B = B; s1.G = tv.G(slot_G(P, j + 1));
            s1.bw = (j + 1 == P->nt) ? T(0.5) * h : h;
            s1.flags |= first ? F_FIRST : 0;
        }
        if (vt) { s1.VT = vt; s1.LAM = tv.Lam(j); }
        CKS(stage<T>(P, vt ? OP_A1F : OP_A1, s1));
        StageArgs<T> s2 = base_args<T>(P);
        s2.A = tv.F(2); s2.Bf = tv.F(3); s2.X = u1;
        s2.V1 = v; s2.V2 = v + nn;
        s2.ROUT = tv.F(nxt.r); s2.COUT = tv.F(nxt.c);
        if (keep) s2.UOUT = tv.Lam(P->nt + j);   // lam*_j
        if (!paper) {
            s2.B = B; s2.G = tv.G(slot_G(P, j)); s2.G2 = tv.G(slot_Gs(P, j));
            s2.bw = T(0.5) * h;
            s2.flags = first ? F_FIRST : 0;
        }
        if (vt) {
            s2.VT = vt; s2.LAM = tv.Lam(P->nt + j); s2.LAM2 = tv.Lam(j);
            s2.GT = j > 0 ? tv.Gm(j) : nullptr;   // grad m~_0 = 0
            s2.GT2 = tv.Gm(P->nt + j);
        }
        if (j == 0 && !paper && !vt && B) {   // lam_0 is not needed: body force only
            if (defer && !keep) {
                *defer = BodyLast<T>{s2.A, s2.Bf, s2.X, s2.G, s2.G2, s2.bw, first ? 1 : 0};
                return REG_OK;
            }
            CK(launch_body_last<T>(nn, s2.bw, first, s2.A, s2.Bf, s2.X, s2.G, s2.G2, B, keep ? s2.UOUT : nullptr,
                                   P->stream));
            return REG_OK;
        }
        CKS(stage<T>(P, vt ? OP_A2F : OP_A2, s2));
        A = tv.F(nxt.r);
        Bf = tv.F(nxt.c);
        nxt = (nxt.r == 0) ? Pair{5, 6} : Pair{0, 1};
    }
    if (paper) CK(launch_body_end<T>(nn, T(0.5) * h, A, Bf, tv.G(slot_G(P, 0)), B, P->stream));
    return REG_OK;
}

// ---- incremental state forward (eq. (inc-state-eq-elim)) ---------------------------------------
// Leaves m~(1) = R + C; returns the scratch indices of the pair.
// keep_grad (full Newton): store grad m~_j (j >= 1) and grad m~*_j from the stage transforms.
template <typename T>
reg_status inc_state_forward(reg_problem* P, const T* v, const T* vt, Pair* out, bool keep_grad = false) {
    TV<T> tv{P};
    const long nn = P->nn;
    const bool paper = P->p.adjoint == REG_ADJ_PAPER;
    Pair cur{0, 1}, nxt{5, 6};
    for (int j = 0; j < P->nt; ++j) {
        const T* Gsrc2 = paper ? tv.G(slot_G(P, j + 1)) : tv.G(slot_Gs(P, j));
        StageArgs<T> s2 = base_args<T>(P);
        if (j == 0) {
            // m~_0 = 0: stage 1 is m~*_0 = -h v~ . G_0, formed on the fly by both parts of stage 2
            s2.flags = F_ZERO; s2.G2 = tv.G(slot_G(P, 0));
        } else {
            StageArgs<T> s1 = base_args<T>(P);
            s1.A = tv.F(cur.r); s1.Bf = tv.F(cur.c);
            s1.V1 = v; s1.V2 = v + nn; s1.VT = vt; s1.G = tv.G(slot_G(P, j));
            s1.ROUT = tv.F(2); s1.UOUT = tv.F(4); s1.COUT = tv.F(3);
            if (keep_grad) s1.GOUT = tv.Gm(j);
            CKS(stage<T>(P, OP_I1, s1));
            s2.A = tv.F(2); s2.Bf = tv.F(3); s2.X = tv.F(4);
        }
        s2.V1 = v; s2.V2 = v + nn; s2.VT = vt; s2.G = Gsrc2;
        s2.ROUT = tv.F(nxt.r); s2.COUT = tv.F(nxt.c);
        if (keep_grad) s2.GOUT = tv.Gm(P->nt + j);
        CKS(stage<T>(P, OP_I2, s2));
        std::swap(cur, nxt);
    }
    *out = cur;
    return REG_OK;
}

// ---- spectral helpers (FP64) ------------------------------------------------------------------
template <typename TI>
reg_status spec_fwd(reg_problem* P, int field, const TI* in) {
    cpx<double>* sp = P->spec() + (size_t)(2 * field) * P->n1 * (P->n2 / 2);
    CK(launch_spec_row_fwd<TI>(P->sp, in, (const TI*)nullptr, sp, P->at<cpx<double>>(P->o.tw2d), P->stream));
    return REG_OK;
}
reg_status spec_col(reg_problem* P, int mode, bool have_y, bool want2) {
    CK(launch_spec_col(P->sp, mode, have_y, want2, P->spec(), P->at<cpx<double>>(P->o.tw1d), P->stream));
    return REG_OK;
}

// Both result fields of the last column pass (the second only with out1) in one launch.
reg_status spec_inv2(reg_problem* P, double* out0, double* out1, const RowDot* dot = nullptr) {
    if (dot) CK(launch_spec_row_inv2_dot(P->sp, P->spec(), out0, out1, P->at<cpx<double>>(P->o.tw2d), *dot, P->stream));
    else CK(launch_spec_row_inv2(P->sp, P->spec(), out0, out1, P->at<cpx<double>>(P->o.tw2d), P->stream));
    return REG_OK;
}

// Nyquist projection of a caller vector field: out_d (double, nullable), out_t (T, nullable).  In
// real space (alternating row and column sums); the spectral buffer serves as scratch.
template <typename T>
reg_status project(reg_problem* P, const double* in, double* out_d, T* out_t) {
    if (nyquist_scratch_doubles(P->n1, P->n2) > 4 * (size_t)P->n1 * (P->n2 / 2) * 2)
        return fail(REG_ENOMEM, "projection scratch exceeds the spectral buffer");
    CK(launch_nyquist_project<T>(P->n1, P->n2, in, out_d, out_t, reinterpret_cast<double*>(P->spec()), P->stream));
    return REG_OK;
}

// Host-read reductions ---------------------------------------------------------------------------
reg_status fetch(reg_problem* P, int k, double* out) {
    CK(hipMemcpyAsync(out, P->scal(), sizeof(double) * k, hipMemcpyDeviceToHost, P->stream));
    CK(hipStreamSynchronize(P->stream));
    return REG_OK;
}

reg_status dots(reg_problem* P, int k, const double* const* a, const double* const* b, double* out) {
    CK(launch_dots<double>(k, a, b, 2 * P->nn, P->partial(), P->scal(), P->stream));
    return fetch(P, k, out);
}

// Regularisation terms 1/2 beta_v <v, A v> and 1/2 beta_w <div v, (1 - Lap) div v> of a projected v.
reg_status stokes_value(reg_problem* P, const double* v64, double* out);

reg_status reg_terms(reg_problem* P, const double* v64, double* rv, double* rw) {
    const bool ms = P->p.constraint == REG_MASS_SOURCE;
    const bool st = P->p.norm == REG_STOKES;
    if (st) {
        *rw = 0.0;
        CKS(stokes_value(P, v64, rv));
        if (!ms) return REG_OK;
    }
    double* t0 = P->at<double>(P->o.tmp0);
    double* t1 = P->at<double>(P->o.tmp1);
    CKS(spec_fwd<double>(P, 0, v64));
    CKS(spec_col(P, SPEC_REG, false, ms));
    CKS(spec_inv2(P, t0, ms ? t1 : nullptr));
    const double* a[2] = {v64, v64};
    const double* b[2] = {t0, t1};
    double r[2] = {0, 0};
    CKS(dots(P, ms ? 2 : 1, a, b, r));
    if (!st) *rv = 0.5 * P->h1h2 * r[0];
    *rw = ms ? 0.5 * P->h1h2 * r[1] : 0.0;
    return REG_OK;
}

reg_status data_term(reg_problem* P, const double* m1, double* out) {
    CK(launch_sqdiff<double>(P->sR(), m1, P->nn, P->partial(), P->scal(), P->stream));
    double s = 0;
    CKS(fetch(P, 1, &s));
    *out = P->h1h2 * s;
    return REG_OK;
}

// ---- shear-control regulariser (eqs. (shear-control-reg-v), (1st-var-reg-v-nls), (2nd-var-reg-v-nls)) ---
double* stk(reg_problem* P, int f) { return P->at<double>(P->o.stk) + (size_t)f * P->nn; }

reg_status grad_fd(reg_problem* P, const double* field, double* out_vec) {   // FP64 spectral gradient
    StageArgs<double> g = base_args<double>(P);
    g.A = field;
    g.GOUT = out_vec;
    return stage<double>(P, OP_GRAD, g);
}

// partials of a vector field into STK_DV
reg_status stokes_partials(reg_problem* P, const double* w) {
    for (int i = 0; i < 2; ++i) CKS(grad_fd(P, w + (size_t)i * P->nn, stk(P, STK_DV + 2 * i)));
    return REG_OK;
}

// STK_R = scale * div(stress in STK_SIG)
reg_status stokes_divergence(reg_problem* P, double scale) {
    for (int k = 0; k < 3; ++k) CKS(grad_fd(P, stk(P, STK_SIG + k), stk(P, STK_DS + 2 * k)));
    CK(launch_stokes_div(P->nn, stk(P, STK_DS), scale, stk(P, STK_R), P->stream));
    return REG_OK;
}

// Mass-source penalty gradient -beta_w grad (1 - Lap) div x (the second result of SPEC_REG) into out.
reg_status penalty_grad(reg_problem* P, const double* x, double* out) {
    CKS(spec_fwd<double>(P, 0, x));
    CKS(spec_col(P, SPEC_REG, false, true));
    CK(launch_spec_row_inv2(P->sp, P->spec(), nullptr, out, P->at<cpx<double>>(P->o.tw2d), P->stream));
    return REG_OK;
}

// beta_v A[v] into STK_R; keeps E and eta at v (the point of later Hessian matvecs).  With a mass
// source also the sum of eta at v (its mean enters M of K_v) and the penalty gradient, added to STK_R.
reg_status stokes_first(reg_problem* P, const double* v64) {
    CKS(stokes_partials(P, v64));
    CK(launch_stokes_first(P->nn, stk(P, STK_DV), P->p.stokes_nu, P->p.stokes_eps, stk(P, STK_SIG), stk(P, STK_E),
                           stk(P, STK_ETA), nullptr, P->stream));
    CKS(stokes_divergence(P, -P->p.beta_v));
    if (P->p.constraint == REG_MASS_SOURCE) {
        CK(launch_minmaxsum(stk(P, STK_ETA), P->nn, P->partial(), P->scal() + SC_ETA, P->stream));
        CKS(penalty_grad(P, v64, stk(P, STK_PEN)));
        CK(launch_add_scaled(2 * P->nn, stk(P, STK_R), 1.0, stk(P, STK_PEN), stk(P, STK_R), P->stream));
    }
    return REG_OK;
}

// beta_v B(v)[v~] (+ the penalty's Hessian with a mass source) into STK_R at the kept point
reg_status stokes_second(reg_problem* P, const double* vt64) {
    CKS(stokes_partials(P, vt64));
    CK(launch_stokes_second(P->nn, stk(P, STK_DV), stk(P, STK_E), stk(P, STK_ETA), P->p.stokes_nu, P->p.stokes_eps,
                            stk(P, STK_SIG), P->stream));
    CKS(stokes_divergence(P, -P->p.beta_v));
    if (P->p.constraint == REG_MASS_SOURCE) {
        CKS(penalty_grad(P, vt64, stk(P, STK_PEN)));
        CK(launch_add_scaled(2 * P->nn, stk(P, STK_R), 1.0, stk(P, STK_PEN), stk(P, STK_R), P->stream));
    }
    return REG_OK;
}

// beta_v R(v) (host), without touching the kept point
reg_status stokes_value(reg_problem* P, const double* v64, double* out) {
    CKS(stokes_partials(P, v64));
    CK(launch_stokes_first(P->nn, stk(P, STK_DV), P->p.stokes_nu, P->p.stokes_eps, nullptr, nullptr, nullptr,
                           stk(P, STK_DENS), P->stream));
    double r[3];
    CK(launch_minmaxsum(stk(P, STK_DENS), P->nn, P->partial(), P->scal(), P->stream));
    CK(hipMemcpyAsync(r, P->scal(), sizeof r, hipMemcpyDeviceToHost, P->stream));
    CK(hipStreamSynchronize(P->stream));
    const double nu = P->p.stokes_nu;
    *out = P->p.beta_v * 2.0 * nu / (nu + 1.0) * P->h1h2 * r[2];
    return REG_OK;
}

// ---- objective --------------------------------------------------------------------------------
template <typename T>
reg_status objective_t(reg_problem* P, const double* v, double* J, double* terms) {
    TV<T> tv{P};
    double* vp = P->at<double>(P->o.vtrial);
    CKS(project<T>(P, v, vp, (T*)nullptr));
    CKS(state_forward<T>(P, vp, false, P->sF(7), (T*)nullptr));
    double d = 0, rv = 0, rw = 0;
    CKS(data_term(P, P->sF(7), &d));
    CKS(reg_terms(P, vp, &rv, &rw));
    *J = d + rv + rw;
    if (terms) { terms[0] = d; terms[1] = rv; terms[2] = rw; }
    if (!std::isfinite(*J)) return fail(REG_ENONFINITE, "objective is not finite");
    return REG_OK;
}

// ---- gradient (sets the linearisation point) --------------------------------------------------
// g = F_Nyq[beta_v A v + K b]; also K^{-1} g for the mass-source model (kg, nullable).
template <typename T>
reg_status gradient_t(reg_problem* P, const double* v, double* g, double* kg, double* Jout) {
    TV<T> tv{P};
    double* v64 = P->at<double>(P->o.v64);
    P->linearized = false;
    P->matvec_done = false;
    CKS(project<T>(P, v, v64, tv.vT()));
    CKS(state_forward<T>(P, v64, true, P->sF(7), tv.F(8)));
    double d = 0, rv = 0, rw = 0;
    if (Jout) {
        CKS(data_term(P, P->sF(7), &d));
        CKS(reg_terms(P, v64, &rv, &rw));
    }
    BodyLast<T> bl{};
    CKS(adjoint_backward<T>(P, tv.vT(), tv.F(8), (const T*)nullptr, false, tv.B(),
                            P->p.hessian == REG_HESS_FULL, (const T*)nullptr, &bl));
    const double* x0 = v64;
    if (P->p.norm == REG_STOKES) {   // the regularisation term is formed in real space
        CKS(stokes_first(P, v64));
        x0 = stk(P, STK_R);
    }
    CK(launch_spec_row_fwd_body<T>(P->sp, x0, tv.B(), bl, P->spec(), P->at<cpx<double>>(P->o.tw2d), P->stream));
    const bool ms = P->p.constraint == REG_MASS_SOURCE;
    CKS(spec_col(P, SPEC_HESS, true, ms && kg));
    CKS(spec_inv2(P, g, (ms && kg) ? kg : nullptr));
    if (Jout) {
        *Jout = d + rv + rw;
        if (!std::isfinite(*Jout)) return fail(REG_ENONFINITE, "objective is not finite");
    }
    P->linearized = true;
    return REG_OK;
}

// ---- GN Hessian matvec on a projected FP64 input ------------------------------------------------
// converted: the caller already wrote vt64 in T to tv.vtT().
// dot (nullable): the assembly's inverse row pass also forms the partial sums of <s, out> (RowDot).
// pout (nullable; spec_col_hess_p_ok grids): also P^{-1} out (SPEC_HESS_P).
template <typename T>
reg_status matvec_t(reg_problem* P, const double* vt64, double* out, double* kout, bool converted = false,
                    const RowDot* dot = nullptr, double* pout = nullptr) {
    TV<T> tv{P};
    if (!P->linearized) return fail(REG_ESTATE, "no linearisation point: call reg_gradient first");
    if (!converted) CK(launch_convert<T>(2 * P->nn, vt64, tv.vtT(), P->stream));
    Pair mt;
    const bool full = P->p.hessian == REG_HESS_FULL;
    CKS(inc_state_forward<T>(P, tv.vT(), tv.vtT(), &mt, full));
    // lam~(1) = -m~(1)
    BodyLast<T> bl{};
    CKS(adjoint_backward<T>(P, tv.vT(), tv.F(mt.r), tv.F(mt.c), true, tv.Bt(), false,
                            full ? (const T*)tv.vtT() : (const T*)nullptr, &bl));
    const double* x0 = vt64;
    if (P->p.norm == REG_STOKES) {
        CKS(stokes_second(P, vt64));
        x0 = stk(P, STK_R);
    }
    // both fields' row transforms in one launch, the last adjoint step's body force folded in
    CK(launch_spec_row_fwd_body<T>(P->sp, x0, tv.Bt(), bl, P->spec(), P->at<cpx<double>>(P->o.tw2d), P->stream));
    if (pout) {
        CKS(spec_col(P, SPEC_HESS_P, true, kout != nullptr));
        double* outs[4] = {out, pout, nullptr, nullptr};   // fields: H s, P^{-1} H s
        int nf = 2;
        if (kout) {   // H s, K^{-1} H s, P^{-1} H s
            outs[1] = kout;
            outs[2] = pout;
            nf = 3;
        }
        CK(launch_spec_row_inv4_dot(P->sp, P->spec(), outs, nf, P->at<cpx<double>>(P->o.tw2d),
                                    dot ? *dot : RowDot{}, P->stream));
    } else {
        CKS(spec_col(P, SPEC_HESS, true, kout != nullptr));
        CKS(spec_inv2(P, out, kout, dot));
    }
    P->matvec_done = true;
    return REG_OK;
}

void drop_graphs(reg_problem* P) {
    for (auto& g : P->graph) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = reg_problem::MvGraph{};
    }
    P->graph_next = 0;
    if (P->pcg_iter_graph) (void)hipGraphExecDestroy(P->pcg_iter_graph);
    P->pcg_iter_graph = nullptr;
    if (P->pcg_iter_graph_lr) (void)hipGraphExecDestroy(P->pcg_iter_graph_lr);
    P->pcg_iter_graph_lr = nullptr;
    if (P->pcg_iter_graph_ex) (void)hipGraphExecDestroy(P->pcg_iter_graph_ex);
    P->pcg_iter_graph_ex = nullptr;
    for (auto& g : P->lr_graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// Capture the work `enqueue` puts on the problem's stream into an executable graph (on the private
// capture stream).  Returns nullptr if capture is unavailable.
template <typename F>
hipGraphExec_t capture_graph(reg_problem* P, F enqueue) {
    if (!P->capture_stream && hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraph_t graph = nullptr;
    hipStream_t saved = P->stream;
    P->stream = P->capture_stream;
    bool ok = hipStreamBeginCapture(P->capture_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    reg_status s = ok ? enqueue() : REG_EDEVICE;
    hipError_t e = ok ? hipStreamEndCapture(P->capture_stream, &graph) : hipErrorUnknown;
    P->stream = saved;
    ok = ok && s == REG_OK && e == hipSuccess && graph;
    hipGraphExec_t exec = nullptr;
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return ok ? exec : nullptr;
}

// (reg_hessian_matvec only: vt64 comes from the projection, which also wrote its T copy.)
// The matvec is a fixed chain of 4 n_t + 1 kernels (four stage launches per time step, less the
// pointwise first and the folded last one, and three assembly passes; power-of-two grids, GN, no
// shear-control term) whose arguments depend only on workspace pointers, so it is captured once
// into a HIP graph (on a private stream) and replayed on the problem's stream; this removes the
// host launch cost per pass.  Falls back to direct launches if capture is unavailable.
template <typename T>
reg_status matvec_run(reg_problem* P, const double* vt64, double* out, double* kout) {
    if (!P->linearized) return fail(REG_ESTATE, "no linearisation point: call reg_gradient first");
    if (P->use_graphs) {
        reg_problem::MvGraph* hit = nullptr;
        for (auto& g : P->graph)
            if (g.exec && g.in == vt64 && g.out == out && g.kout == kout) hit = &g;
        if (!hit) {
            hipGraphExec_t exec = capture_graph(P, [&]() { return matvec_t<T>(P, vt64, out, kout, true); });
            if (exec) {
                reg_problem::MvGraph& slot = P->graph[P->graph_next];
                if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
                slot = reg_problem::MvGraph{vt64, out, kout, exec};
                P->graph_next = (P->graph_next + 1) % reg_problem::NGRAPH;
                hit = &slot;
            } else {
                P->use_graphs = false;
                drop_graphs(P);
            }
        }
        if (hit) {
            CK(hipGraphLaunch(hit->exec, P->stream));
            P->matvec_done = true;
            return REG_OK;
        }
    }
    return matvec_t<T>(P, vt64, out, kout, true);
}

reg_status precond_t(reg_problem* P, const double* r, double* z, double* kr) {
    CKS(spec_fwd<double>(P, 0, r));
    CKS(spec_col(P, SPEC_PREC, false, kr != nullptr));
    CKS(spec_inv2(P, z, kr));
    return REG_OK;
}

// ---- low-rank deflation correction of the preconditioner -----------------------------------------
// With directions z_k, H z_k and e_k > 0 (k < count; <z_i, H z_j>_W = e_i delta_ij for directions from
// one Rayleigh-Ritz basis or one PCG solve), the balancing preconditioner is
//     z = Pi M^{-1} Pi^* r + sum_k a_k z_k,   a_k = <z_k, r>_W / e_k,   Pi = I - sum_k z_k <H z_k, .>_W / e_k,
// evaluated as r~ = r - sum a_k H z_k, y = M^{-1} r~, b_k = <H z_k, y>_W / e_k, z = y + sum (a_k - b_k) z_k.
// It is symmetric positive definite in <., .>_W for any such set.  For the mass-source model the
// W-products use the stored K^{-1} images and K^{-1} r = K^{-1} r~ + sum a_k K^{-1} H z_k.
reg_status precond_pcg(reg_problem* P, const double* r, double* z, double* kr) {
    if (!P->lr_active || P->lr_count == 0) return precond_t(P, r, z, kr);   // no directions: the plain form
    const long n = 2 * P->nn;
    const bool ms = P->p.constraint == REG_MASS_SOURCE;
    const int cap = P->p.lowrank_capacity;
    double* sc = P->lr_sc();
    double* part = P->at<double>(P->o.lrpart);
    double* rt = P->at<double>(P->o.lrtmp);
    const double* Zw = P->lr_set(ms ? 2 : 0);
    const double* HZw = P->lr_set(ms ? 3 : 1);
    CK(launch_lr_dots(n, r, Zw, n, sc + LRS_CNT, cap, part, sc + LRS_DA, P->stream));
    CK(launch_lr_combine(n, r, rt, P->lr_set(1), n, sc + LRS_CNT, cap, sc + LRS_DA, nullptr, sc + LRS_E, -1.0,
                         P->stream));
    CKS(precond_t(P, rt, z, kr));
    CK(launch_lr_dots(n, z, HZw, n, sc + LRS_CNT, cap, part, sc + LRS_DB, P->stream));
    CK(launch_lr_combine(n, z, z, P->lr_set(0), n, sc + LRS_CNT, cap, sc + LRS_DA, sc + LRS_DB, sc + LRS_E, 1.0,
                         P->stream));
    if (kr)
        CK(launch_lr_combine(n, kr, kr, P->lr_set(3), n, sc + LRS_CNT, cap, sc + LRS_DA, nullptr, sc + LRS_E, 1.0,
                             P->stream));
    return REG_OK;
}

reg_status lr_set_count(reg_problem* P, int count) {
    CK(launch_fill(1, (double)count, P->lr_sc() + LRS_CNT, P->stream));
    P->lr_count = count;
    return REG_OK;
}

// Symmetric eigen-decomposition of a small matrix (cyclic Jacobi rotations): A = V diag(w) V^T with
// w ascending.  A (n x n, row-major) is overwritten.
void sym_eig(int n, double* A, double* w, double* V) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {   // A <- J^T A J
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - sn * akq;
                    A[k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - sn * aqk;
                    A[q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - sn * vkq;
                    V[k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[a * n + a] < A[b * n + b]; });
    std::vector<double> Vs(n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = A[idx[j] * n + idx[j]];
        for (int i = 0; i < n; ++i) Vs[i * n + j] = V[i * n + idx[j]];
    }
    for (int i = 0; i < n * n; ++i) V[i] = Vs[i];
}

// Gram matrix G_ij = sum X_i . Y_j (raw sums) of the first r slots of two sets, read back to the host.
reg_status lr_gram(reg_problem* P, int setx, int sety, int r, double* G) {
    const long n = 2 * P->nn;
    double* sc = P->lr_sc();
    CK(launch_fill(1, (double)r, sc + LRS_CNT2, P->stream));
    for (int i = 0; i < r; ++i)
        CK(launch_lr_dots(n, P->lr_slot(setx, i), P->lr_set(sety), n, sc + LRS_CNT2, P->p.lowrank_capacity,
                          P->at<double>(P->o.lrpart), sc + LRS_G + i * r, P->stream));
    CK(hipMemcpyAsync(G, sc + LRS_G, sizeof(double) * r * r, hipMemcpyDeviceToHost, P->stream));
    CK(hipStreamSynchronize(P->stream));
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < i; ++j) G[i * r + j] = G[j * r + i] = 0.5 * (G[i * r + j] + G[j * r + i]);
    return REG_OK;
}

// H z_k for Rayleigh-Ritz basis slot k (and K^{-1} H z_k for the mass-source model), replayed from a
// graph captured once per slot: the slots' pointers are fixed, like the matvec's.
template <typename T>
reg_status lr_matvec(reg_problem* P, int k) {
    const bool ms = P->p.constraint == REG_MASS_SOURCE;
    const double* in = P->lr_slot(0, k);
    double* out = P->lr_slot(1, k);
    double* kout = ms ? P->lr_slot(3, k) : nullptr;
    if (P->use_graphs) {
        hipGraphExec_t& g = P->lr_graph[k];
        if (!g) g = capture_graph(P, [&]() { return matvec_t<T>(P, in, out, kout, false); });
        if (g) {
            CK(hipGraphLaunch(g, P->stream));
            P->matvec_done = true;
            return REG_OK;
        }
        P->use_graphs = false;
        drop_graphs(P);
    }
    return matvec_t<T>(P, in, out, kout, false);
}

// Rayleigh-Ritz on the caller directions U (r <= LR_MIX_MAX) at the current linearisation point:
// admissible parts Z, orthonormalised in <., M .>_W (Gram eigenvalues <= 1e-10 of the largest
// dropped), H applied to that basis, the projected Hessian diagonalised, Ritz pairs with theta <= 0
// dropped.  Fills slots [0, kept) with Z, H Z (and K^{-1} images), e = theta.  theta_out (host,
// nullable, r entries): the kept Ritz values ascending, then zeros.
template <typename T>
reg_status lr_setup_t(reg_problem* P, const double* U, int r, double* theta_out, int* nmv) {
    const long n = 2 * P->nn;
    const bool ms = P->p.constraint == REG_MASS_SOURCE;
    for (int j = 0; j < r; ++j) {
        CKS(spec_fwd<double>(P, 0, U + (size_t)j * n));
        CKS(spec_col(P, SPEC_LR, false, true));
        CKS(spec_inv2(P, P->lr_slot(0, j), P->lr_slot(1, j)));   // and K^{-1} M z_j (scratch)
    }
    double G[LR_MIX_MAX * LR_MIX_MAX], lam[LR_MIX_MAX], E[LR_MIX_MAX * LR_MIX_MAX];
    CKS(lr_gram(P, 0, 1, r, G));
    for (int i = 0; i < r * r; ++i)
        if (!std::isfinite(G[i])) return fail(REG_ENONFINITE, "precond_U is not finite");
    sym_eig(r, G, lam, E);
    const double lmax = r > 0 ? lam[r - 1] : 0.0;
    LrMix C{};
    int r1 = 0;
    for (int j = 0; j < r; ++j) {
        if (!(lmax > 0.0) || !(lam[j] > 1e-10 * lmax)) continue;
        for (int i = 0; i < r; ++i) C.m[i][r1] = E[i * r + j] / std::sqrt(lam[j]);
        ++r1;
    }
    if (theta_out)
        for (int j = 0; j < r; ++j) theta_out[j] = 0.0;
    if (r1 == 0) return lr_set_count(P, 0);
    CK(launch_lr_mix(n, P->lr_set(0), n, r, r1, C, P->stream));
    for (int k = 0; k < r1; ++k) {
        CKS(lr_matvec<T>(P, k));
        if (nmv) ++*nmv;
    }
    double Tm[LR_MIX_MAX * LR_MIX_MAX], th[LR_MIX_MAX], V[LR_MIX_MAX * LR_MIX_MAX];
    CKS(lr_gram(P, 0, ms ? 3 : 1, r1, Tm));
    for (int i = 0; i < r1 * r1; ++i)
        if (!std::isfinite(Tm[i])) return fail(REG_ENONFINITE, "Hessian on precond_U is not finite");
    sym_eig(r1, Tm, th, V);
    LrMix R{};
    double e[LR_MIX_MAX];
    int r2 = 0;
    for (int j = 0; j < r1; ++j) {
        if (!(th[j] > 0.0) || !std::isfinite(th[j])) continue;
        for (int i = 0; i < r1; ++i) R.m[i][r2] = V[i * r1 + j];
        e[r2] = th[j];
        if (theta_out) theta_out[r2] = th[j];
        ++r2;
    }
    if (r2 == 0) return lr_set_count(P, 0);
    CK(launch_lr_mix(n, P->lr_set(0), n, r1, r2, R, P->stream));
    CK(launch_lr_mix(n, P->lr_set(1), n, r1, r2, R, P->stream));
    if (ms) {
        CK(launch_lr_mix(n, P->lr_set(3), n, r1, r2, R, P->stream));
        for (int k = 0; k < r2; ++k)
            CKS(precond_t(P, P->lr_slot(0, k), P->at<double>(P->o.lrtmp), P->lr_slot(2, k)));   // K^{-1} z_k
    }
    CK(hipMemcpyAsync(P->lr_sc() + LRS_E, e, sizeof(double) * r2, hipMemcpyHostToDevice, P->stream));
    CK(hipStreamSynchronize(P->stream));   // e is a host stack array
    return lr_set_count(P, r2);
}

// Subspace iteration for the leading generalised eigenpairs of (H, M) at the current linearisation
// point: Rayleigh-Ritz on span(U), then U <- M^{-1} H z_k, repeated `iters` times (the caller's U
// holds each new basis).  Leaves the Ritz vectors in U in descending order of theta (dropped slots
// zeroed) and the values in theta (host, descending, zeros after the kept ones).
template <typename T>
reg_status ritz_t(reg_problem* P, double* U, int rank, int iters, double* theta) {
    const long n = 2 * P->nn;
    double th[LR_MIX_MAX];
    CKS(lr_setup_t<T>(P, U, rank, th, nullptr));
    for (int it = 0; it < iters && P->lr_count > 0; ++it) {
        const int r = P->lr_count;
        for (int k = 0; k < r; ++k) CKS(precond_t(P, P->lr_slot(1, k), U + (size_t)k * n, nullptr));
        CKS(lr_setup_t<T>(P, U, r, th, nullptr));
    }
    const int kept = P->lr_count;   // lr_setup_t leaves theta ascending in th[0, kept)
    for (int k = 0; k < rank; ++k) {
        if (k < kept)
            CK(hipMemcpyAsync(U + (size_t)k * n, P->lr_slot(0, kept - 1 - k), n * 8, hipMemcpyDeviceToDevice, P->stream));
        else
            CK(launch_fill(n, 0.0, U + (size_t)k * n, P->stream));
        if (theta) theta[k] = k < kept ? th[kept - 1 - k] : 0.0;
    }
    CKS(lr_set_count(P, 0));
    CK(hipStreamSynchronize(P->stream));
    return REG_OK;
}

// ---- PCG (Alg. 2) -----------------------------------------------------------------------------
enum { PX = 0, PR, PZ, PKR, PS, PST, PKST, PPST };

// Every PCG_Z_REFRESH-th iteration forms z = P^{-1} r (and K^{-1} r) from r itself; the others
// update them by recurrence.  The recurrence carries rounding of the size of the largest z seen so
// far; once ||z|| has fallen by about the unit roundoff, <r, z>_W is that rounding and the iteration
// breaks down.  Replacing z every few iterations bounds the drift by the decrease over that many
// iterations (a factor 10 per iteration at most over 8 still leaves eight digits).
constexpr int PCG_Z_REFRESH = 8;

// One PCG iteration with device-side scalars: s~ = H s, kappa, x and r updates, z = P^{-1} r,
// the new <r, z>_W and ||r||^2, mu, s = z + mu s.  No host synchronisation inside.  rec: the
// preconditioned residual by recurrence, z -= kappa P^{-1} H s, with P^{-1} H s formed by the
// assembly's column pass (the caller checks that the grid has that pass and the low-rank extension,
// whose corrected preconditioner is applied to r, is off).
template <typename T>
reg_status pcg_iter_enqueue(reg_problem* P, bool rec) {
    const long n = 2 * P->nn;
    const bool W = P->p.constraint == REG_MASS_SOURCE;
    double *x = P->pcg(PX), *r = P->pcg(PR), *z = P->pcg(PZ), *kr = P->pcg(PKR);
    double *s = P->pcg(PS), *st = P->pcg(PST), *kst = P->pcg(PKST);
    double* sc = P->scal();
    double* pst = P->pcg(PPST);
    // <s, H s>_W: partial sums from the assembly's last pass where it forms them
    int parts = 0;
    const RowDot rd{s, W ? 1 : 0, P->partial(), &parts};
    CKS(matvec_t<T>(P, s, st, W ? kst : nullptr, true, &rd, rec ? pst : nullptr));
    if (parts > 0) {
        CK(launch_finalize_scalar(1, parts, P->partial(), sc + S_SHS, PCG_KAPPA, sc, P->stream));
    } else {
        const double* a[1] = {s};
        const double* b[1] = {W ? kst : st};
        CK(launch_dots_scalar(1, a, b, n, P->partial(), sc + S_SHS, PCG_KAPPA, sc, P->stream));
    }
    if (rec) {
        // kr = K^{-1} r (the weighted residual of <., .>_W) follows r with K^{-1} H s; the update
        // forms the partial sums of ||r||^2 and <r, z>_W as it writes them
        CK(launch_pcg_update_z(n, x, r, s, st, z, pst, W ? kr : nullptr, W ? kst : nullptr, sc, P->partial(),
                               P->stream));
        CK(launch_finalize_scalar(2, RED_BLOCKS, P->partial(), sc + S_RR, PCG_MU, sc, P->stream));
    } else {
        CK(launch_pcg_update(n, x, r, s, st, sc, P->stream));
        CKS(precond_pcg(P, r, z, W ? kr : nullptr));
        const double* a[2] = {r, W ? kr : r};
        const double* b[2] = {r, z};
        CK(launch_dots_scalar(2, a, b, n, P->partial(), sc + S_RR, PCG_MU, sc, P->stream));
    }
    CK(launch_pcg_dir_copy<T>(n, s, TV<T>{P}.vtT(), z, sc, P->stream));
    return REG_OK;
}

// Iteration l (from 0) of a PCG solve.
template <typename T>
reg_status pcg_iter_run(reg_problem* P, int l) {
    // a correction without directions yet (the first Newton step of a recycling solve) is the plain
    // preconditioner; the set does not change within one PCG solve
    const bool lr = P->lr_active && P->lr_count > 0;
    const bool can_rec = !lr && spec_col_hess_p_ok(P->n1, P->n2);
    const bool rec = can_rec && (l + 1) % PCG_Z_REFRESH != 0;
    hipGraphExec_t& graph = lr                    ? P->pcg_iter_graph_lr
                            : (can_rec && !rec) ? P->pcg_iter_graph_ex
                                                : P->pcg_iter_graph;
    if (P->use_graphs && !graph) {
        graph = capture_graph(P, [&]() { return pcg_iter_enqueue<T>(P, rec); });
        if (!graph) P->use_graphs = false;
    }
    if (graph) {
        CK(hipGraphLaunch(graph, P->stream));
        P->matvec_done = true;
        return REG_OK;
    }
    return pcg_iter_enqueue<T>(P, rec);
}

// record > 0: the first `record` search directions s_l that complete a step are copied with H s_l
// (and K^{-1} H s_l) and e_l = <s_l, H s_l>_W into the correction slots lr_count + l; *recorded
// receives how many are valid (the directions of one PCG solve are mutually H-conjugate).
template <typename T>
reg_status pcg_t(reg_problem* P, const double* rhs, double eta, int max_iters, int fixed_iters, double* xout,
                 int* iters, double* relres, int* nmv, int record = 0, int* recorded = nullptr) {
    const long n = 2 * P->nn;
    const bool W = P->p.constraint == REG_MASS_SOURCE;
    if (!P->linearized) return fail(REG_ESTATE, "no linearisation point: call reg_gradient first");
    double *x = P->pcg(PX), *r = P->pcg(PR), *z = P->pcg(PZ), *kr = P->pcg(PKR);
    double* s = P->pcg(PS);
    double* sc = P->scal();
    CK(hipMemcpyAsync(r, rhs, n * 8, hipMemcpyDeviceToDevice, P->stream));
    CK(launch_fill(n, 0.0, x, P->stream));
    CKS(precond_pcg(P, r, z, W ? kr : nullptr));
    CK(launch_pcg_dir_copy<T>(n, s, TV<T>{P}.vtT(), z, nullptr, P->stream));   // s = z
    {
        const double* a[2] = {W ? kr : r, r};
        const double* b[2] = {z, r};
        CK(launch_dots_scalar(2, a, b, n, P->partial(), sc + S_RZ, PCG_INIT, sc, P->stream));   // S_RZ, S_RR0
    }
    double h[NUM_PCG_SLOTS];
    CK(hipMemcpyAsync(h, sc, sizeof h, hipMemcpyDeviceToHost, P->stream));
    CK(hipStreamSynchronize(P->stream));
    const double r0 = std::sqrt(h[S_RR0]);
    if (!std::isfinite(r0)) return fail(REG_ENONFINITE, "PCG: right-hand side is not finite");
    const int nit = fixed_iters > 0 ? fixed_iters : max_iters;
    int l = 0;
    if (recorded) *recorded = 0;
    if (record > P->p.lowrank_capacity - P->lr_count) record = P->p.lowrank_capacity - P->lr_count;
    while (l < nit) {
        const int slot = P->lr_count + l;
        if (l < record) CK(hipMemcpyAsync(P->lr_slot(0, slot), s, n * 8, hipMemcpyDeviceToDevice, P->stream));
        CKS(pcg_iter_run<T>(P, l));
        if (l < record) {
            CK(hipMemcpyAsync(P->lr_slot(1, slot), P->pcg(PST), n * 8, hipMemcpyDeviceToDevice, P->stream));
            if (W) CK(hipMemcpyAsync(P->lr_slot(3, slot), P->pcg(PKST), n * 8, hipMemcpyDeviceToDevice, P->stream));
            CK(hipMemcpyAsync(P->lr_sc() + LRS_E + slot, sc + S_SHS, 8, hipMemcpyDeviceToDevice, P->stream));
        }
        ++l;
        if (fixed_iters > 0) continue;   // fixed schedule: no stop test, no host round trip
        CK(hipMemcpyAsync(h, sc, sizeof h, hipMemcpyDeviceToHost, P->stream));
        CK(hipStreamSynchronize(P->stream));
        if (h[S_ACTIVE] == 0.0) break;
        if (!std::isfinite(h[S_RR])) return fail(REG_ENONFINITE, "PCG: residual is not finite");
        if (std::sqrt(h[S_RR]) <= eta * r0) break;
    }
    CK(hipMemcpyAsync(h, sc, sizeof h, hipMemcpyDeviceToHost, P->stream));
    CK(hipStreamSynchronize(P->stream));
    if (!std::isfinite(h[S_RR]) || !std::isfinite(h[S_RZ])) return fail(REG_ENONFINITE, "PCG: not finite");
    const int done = (int)h[S_ITER];
    // matvecs that ran: with a fixed schedule the iterations after a breakdown still run (kappa = 0,
    // x and r stay put), so count the launched iterations rather than the completed ones
    if (nmv) *nmv += l;
    if (recorded && record > 0) {
        const int ok = h[S_BREAK] > 0 ? (int)h[S_BREAK] - 1 : done;   // steps with <s, H s>_W > 0
        *recorded = std::max(0, std::min(record, ok));
    }
    if (xout != x) CK(hipMemcpyAsync(xout, x, n * 8, hipMemcpyDeviceToDevice, P->stream));
    if (iters) *iters = done;
    if (relres) *relres = r0 > 0 ? std::sqrt(h[S_RR]) / r0 : 0.0;
    return REG_OK;
}

// ---- CFL number -------------------------------------------------------------------------------
// C(v) = h_t (max|v_1| n1/2 + max|v_2| n2/2) of a device vector field (taken as given).
reg_status cfl_t(reg_problem* P, const double* v, double* out) {
    double r[2][3];
    for (int c = 0; c < 2; ++c) {
        CK(launch_minmaxsum(v + (size_t)c * P->nn, P->nn, P->partial(), P->scal() + 3 * c, P->stream));
    }
    CK(hipMemcpyAsync(r, P->scal(), sizeof r, hipMemcpyDeviceToHost, P->stream));
    CK(hipStreamSynchronize(P->stream));
    const double a1 = std::max(-r[0][0], r[0][1]), a2 = std::max(-r[1][0], r[1][1]);
    *out = (a1 * (P->n1 / 2) + a2 * (P->n2 / 2)) / P->nt;
    if (!std::isfinite(*out)) return fail(REG_ENONFINITE, "velocity is not finite");
    return REG_OK;
}

// ---- Newton (Alg. 1) --------------------------------------------------------------------------
template <typename T>
reg_status solve_t(reg_problem* P, const reg_solve_opts* o, double* vout, reg_solve_stats* st) {
    const long n = 2 * P->nn;
    reg_solve_stats S{};
    const bool W = P->p.constraint == REG_MASS_SOURCE;
    double* v = P->at<double>(P->o.vcur);       // current iterate
    double* g = P->at<double>(P->o.g64);
    double* kg = P->at<double>(P->o.kg64);
    double* vt = P->at<double>(P->o.vt64);       // Newton step
    double* trial = P->at<double>(P->o.vtry);    // line-search trial point
    double* rhs = P->at<double>(P->o.rhs);
    double J = 0;
    // g(0) at v = 0 for the relative gradient (also with a warm start)
    CK(launch_fill(n, 0.0, v, P->stream));
    CKS(gradient_t<T>(P, v, g, W ? kg : nullptr, &J));
    S.n_pde += 2;
    double gg = 0;
    {
        const double* a[1] = {g};
        CKS(dots(P, 1, a, a, &gg));
    }
    const double g0 = std::sqrt(gg);
    S.g0_norm = g0;
    if (o->v0) {
        // The warm start is kept only if it lowers the objective below J(0) (the globalisation
        // needs a descent sequence from the plain start); otherwise the solve restarts from v = 0.
        const double J0 = J, gg0 = gg;
        CK(hipMemcpyAsync(v, o->v0, n * 8, hipMemcpyDeviceToDevice, P->stream));
        reg_status s0 = gradient_t<T>(P, v, g, W ? kg : nullptr, &J);
        S.n_pde += 2;
        if (s0 != REG_OK && s0 != REG_ENONFINITE) return s0;
        if (s0 == REG_OK) {
            const double* a[1] = {g};
            CKS(dots(P, 1, a, a, &gg));
        }
        if (s0 != REG_OK || !std::isfinite(J) || !std::isfinite(gg) || !(J < J0)) {
            S.fallback_used = 1;
            CK(launch_fill(n, 0.0, v, P->stream));
            CKS(gradient_t<T>(P, v, g, W ? kg : nullptr, &J));
            S.n_pde += 2;
            J = J0;
            gg = gg0;
        }
    }
    CK(hipMemcpyAsync(v, P->at<double>(P->o.v64), n * 8, hipMemcpyDeviceToDevice, P->stream));
    // CFL-adapted n_t (Sec. 4): raise n_t when the iterate violates the limit, then re-linearise
    const int ntc = nt_capacity(&P->p);
    auto adapt_nt = [&](bool& changed) -> reg_status {
        changed = false;
        if (!(o->cfl_max > 0.0)) return REG_OK;
        double c = 0;
        CKS(cfl_t(P, v, &c));
        if (c <= o->cfl_max || P->nt >= ntc) return REG_OK;
        const double want = std::ceil(P->nt * (c / o->cfl_max) - 1e-9);
        const int nt_new = (int)std::min((double)ntc, want);
        if (nt_new <= P->nt) return REG_OK;
        P->nt = P->p.nt = nt_new;
        drop_graphs(P);   // the captured launch sequences have n_t steps
        ++S.nt_changes;
        changed = true;
        return REG_OK;
    };
    {
        bool changed = false;
        CKS(adapt_nt(changed));
        if (changed) {
            CKS(gradient_t<T>(P, v, g, W ? kg : nullptr, &J));
            S.n_pde += 2;
            const double* a[1] = {g};
            CKS(dots(P, 1, a, a, &gg));
        }
    }
    // low-rank correction of the PCG preconditioner: Rayleigh-Ritz on the caller directions at the
    // first linearisation point, then (recycle > 0) the leading PCG directions of every Newton step
    struct LrOff {
        reg_problem* P;
        ~LrOff() { P->lr_active = false; }
    } lr_off{P};
    const bool lr = o->rank > 0 || o->recycle > 0;
    if (lr) {
        CKS(lr_set_count(P, 0));
        int nmv = 0;
        if (o->rank > 0) CKS(lr_setup_t<T>(P, o->precond_U, o->rank, o->precond_d, &nmv));
        S.n_matvec += nmv;
        S.n_pde += 2 * nmv;
        P->lr_active = true;
    }
    int k = 0;
    reg_status status = REG_OK;
    double grel = 0;
    using clock = std::chrono::steady_clock;
    // per-step record k (o->steps): the current iterate's J, ||g||_rel and C(v) after the step
    auto record = [&](int kk, int its, int nbt, double alpha, clock::time_point t0) -> reg_status {
        if (!o->steps || kk >= o->max_steps) return REG_OK;
        reg_step_record& R = o->steps[kk];
        R.ms = std::chrono::duration<double, std::milli>(clock::now() - t0).count();
        R.newton_iter = kk;
        R.pcg_iters = its;
        R.backtracks = nbt;
        R.nt = P->nt;
        R.J = J;
        R.g_rel = g0 > 0 ? std::sqrt(gg) / g0 : 0.0;
        R.alpha = alpha;
        return cfl_t(P, P->at<double>(P->o.v64), &R.cfl);   // v64: the projected iterate
    };
    while (true) {
        grel = g0 > 0 ? std::sqrt(gg) / g0 : 0.0;
        if (!std::isfinite(grel) || !std::isfinite(J)) { status = REG_ENONFINITE; break; }
        if (grel <= o->gtol_rel || k >= o->max_newton) break;
        const clock::time_point t_step = clock::now();
        const double eta = std::min(0.5, std::sqrt(grel));
        CK(launch_fill(n, 0.0, rhs, P->stream));
        CK(launch_axpby(n, -1.0, g, 0.0, rhs, P->stream));   // rhs = -g
        int its = 0;
        double rr = 0;
        int rec = 0;
        CKS(pcg_t<T>(P, rhs, eta, o->max_pcg, o->fixed_pcg_iters, vt, &its, &rr, &S.n_matvec, lr ? o->recycle : 0,
                     &rec));
        S.n_pde += 2 * its;
        S.pcg_iters += its;
        if (rec > 0) {
            if (W)
                for (int q = P->lr_count; q < P->lr_count + rec; ++q)
                    CKS(precond_t(P, P->lr_slot(0, q), P->at<double>(P->o.lrtmp), P->lr_slot(2, q)));
            CKS(lr_set_count(P, P->lr_count + rec));
        }
        double slope = 0;
        {
            const double* a[1] = {W ? kg : g};
            const double* b[1] = {vt};
            CKS(dots(P, 1, a, b, &slope));
        }
        slope *= P->h1h2;
        double alpha = 1.0;
        bool accepted = false;
        int nbt = 0;
        if (slope < 0.0) {
            for (nbt = 0; nbt <= o->max_backtracks; ++nbt) {
                CK(launch_add_scaled(n, v, alpha, vt, trial, P->stream));
                double Jt = 0;
                reg_status s = objective_t<T>(P, trial, &Jt, nullptr);
                S.n_pde += 1;
                if (s != REG_OK && s != REG_ENONFINITE) return s;
                if (s == REG_OK && Jt <= J + o->armijo_c1 * alpha * slope) { accepted = true; break; }
                alpha *= o->armijo_rho;
            }
        }
        if (nbt > o->max_backtracks) nbt = o->max_backtracks;
        S.backtracks += nbt;
        if (!accepted) {
            status = REG_ENOTCONV;
            CKS(record(k, its, nbt, 0.0, t_step));
            break;
        }
        CK(launch_add_scaled(n, v, alpha, vt, v, P->stream));
        {
            bool changed = false;
            CKS(adapt_nt(changed));
        }
        CKS(gradient_t<T>(P, v, g, W ? kg : nullptr, &J));
        S.n_pde += 2;
        {
            const double* a[1] = {g};
            CKS(dots(P, 1, a, a, &gg));
        }
        CKS(record(k, its, nbt, alpha, t_step));
        ++k;
    }
    S.newton_iters = k;
    S.lowrank_dim = lr ? P->lr_count : 0;
    CKS(cfl_t(P, P->at<double>(P->o.v64), &S.cfl));
    S.g_rel = grel;
    S.J = J;
    S.status = status;
    S.nt = P->nt;
    CK(hipMemcpyAsync(vout, P->at<double>(P->o.v64), n * 8, hipMemcpyDeviceToDevice, P->stream));
    CK(hipStreamSynchronize(P->stream));
    if (st) *st = S;
    if (status == REG_ENOTCONV) return fail(REG_ENOTCONV, "Armijo line search failed after %d backtracks", o->max_backtracks);
    if (status == REG_ENONFINITE) return fail(REG_ENONFINITE, "non-finite gradient or objective");
    return REG_OK;
}

// ---- deformation diagnostics (eqs. (displacement), (def-grad)) -----------------------------------
// FP64 fields of the caller's diagnostics workspace: v (2), dv (4), then per component c < 6 the pair
// R, C, the stage pair R*, C* and the stage input U; one more for det F.
constexpr int DEF_FIELDS = 2 + 4 + 6 * 5 + 1;

reg_status deformation_run(reg_problem* P, const double* v_in, double* ws, double* u1, double* F1, double* detF,
                           double* stats) {
    const long nn = P->nn;
    auto f = [&](int i) { return ws + (size_t)i * nn; };
    double* v = f(0);
    double* dv = f(2);
    auto R = [&](int c) { return f(6 + 5 * c); };
    auto C = [&](int c) { return f(7 + 5 * c); };
    auto Rs = [&](int c) { return f(8 + 5 * c); };
    auto Cs = [&](int c) { return f(9 + 5 * c); };
    auto U = [&](int c) { return f(10 + 5 * c); };
    double* det = f(DEF_FIELDS - 1);
    CKS(project<double>(P, v_in, v, (double*)nullptr));
    for (int i = 0; i < 2; ++i) {   // dv[i][l] = d_l v_i
        StageArgs<double> g = base_args<double>(P);
        g.A = v + (size_t)i * nn;
        g.GOUT = dv + (size_t)2 * i * nn;
        CKS(stage<double>(P, OP_GRAD, g));
    }
    for (int c = 0; c < 6; ++c) {   // u(0) = 0, F(0) = I
        CK(launch_fill(nn, (c == 2 || c == 5) ? 1.0 : 0.0, R(c), P->stream));
        CK(launch_fill(nn, 0.0, C(c), P->stream));
    }
    const double h = 1.0 / P->nt;
    for (int j = 0; j < P->nt; ++j) {
        for (int c = 0; c < 6; ++c) {
            StageArgs<double> s1 = base_args<double>(P);
            s1.A = R(c); s1.Bf = C(c);
            s1.V1 = v; s1.V2 = v + nn;
            s1.ROUT = Rs(c); s1.UOUT = U(c); s1.COUT = Cs(c);
            CKS(stage<double>(P, OP_S1, s1));
        }
        DefPtrs p1{};
        for (int c = 0; c < 4; ++c) p1.a[c] = U(2 + c);
        for (int c = 0; c < 6; ++c) p1.out[c] = Rs(c);
        CK(launch_deform_source(nn, h, v, dv, p1, P->stream));        // stage 1: + h S(q_j)
        for (int c = 0; c < 6; ++c) {
            StageArgs<double> s2 = base_args<double>(P);
            s2.A = Rs(c); s2.Bf = Cs(c); s2.X = U(c);
            s2.V1 = v; s2.V2 = v + nn;
            s2.ROUT = R(c); s2.COUT = C(c);
            CKS(stage<double>(P, OP_S2, s2));
        }
        DefPtrs p2{};
        for (int c = 0; c < 4; ++c) { p2.a[c] = Rs(2 + c); p2.b[c] = Cs(2 + c); }
        for (int c = 0; c < 6; ++c) p2.out[c] = R(c);
        CK(launch_deform_source(nn, 0.5 * h, v, dv, p2, P->stream));  // stage 2: + (h/2) S(q*)
    }
    DefPairs fin{};
    for (int c = 0; c < 6; ++c) { fin.r[c] = R(c); fin.c[c] = C(c); }
    CK(launch_deform_final(nn, fin, u1, F1, detF ? detF : det, P->stream));
    if (stats) {
        double h3[3];
        CK(launch_minmaxsum(detF ? detF : det, nn, P->partial(), P->scal(), P->stream));
        CK(hipMemcpyAsync(h3, P->scal(), sizeof h3, hipMemcpyDeviceToHost, P->stream));
        CK(hipStreamSynchronize(P->stream));
        stats[0] = h3[0];
        stats[1] = h3[1];
        stats[2] = h3[2] / (double)nn;
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(stats[k])) return fail(REG_ENONFINITE, "det F is not finite");
    }
    return REG_OK;
}

// ---- measurement hook and autotuner ------------------------------------------------------------
// The four stage launches of one matvec time step, set up on live buffers at a middle time step:
// which = 0 GN adjoint stage 2, 1 incremental state stage 2, 2 GN adjoint stage 1, 3 incremental
// state stage 1.  Outputs go to scratch fields (the body-force accumulator of adjoint stage 2 is
// updated in place; every matvec rewrites it).  `fields` = scalar fields of compulsory HBM traffic
// per launch (each operand read once, each result written once).
template <typename T>
reg_status stage_spec(reg_problem* P, int which, StageArgs<T>& a, int& op, double& fields) {
    TV<T> tv{P};
    const long nn = P->nn;
    const int j = P->nt > 1 ? P->nt / 2 : 0;
    const bool paper = P->p.adjoint == REG_ADJ_PAPER;
    if (which < 0 || which > 3) return fail(REG_EINVAL, "unknown stage %d", which);
    a = base_args<T>(P);
    a.V1 = tv.vT();
    a.V2 = tv.vT() + nn;
    switch (which) {
        case 0:   // rows: A, B, X, v2, (G, G*, b: 6) -> R, (b: 2); columns: A, B, v1 -> C
            op = OP_A2;
            a.A = tv.F(2); a.Bf = tv.F(3); a.X = tv.F(4); a.ROUT = tv.F(5); a.COUT = tv.F(6);
            if (!paper) { a.B = tv.Bt(); a.G = tv.G(slot_G(P, j)); a.G2 = tv.G(slot_Gs(P, j)); a.bw = T(0.5 / P->nt); }
            fields = (paper ? 5 : 13) + 4;
            break;
        case 1:   // rows: A, B, X, v2, v~(2), G(2) -> R; columns: A, B, v1 -> C
            op = OP_I2;
            a.A = tv.F(2); a.Bf = tv.F(3); a.X = tv.F(4); a.VT = tv.vtT();
            a.G = paper ? tv.G(slot_G(P, j + 1)) : tv.G(slot_Gs(P, j));
            a.ROUT = tv.F(5); a.COUT = tv.F(6);
            fields = 9 + 4;
            break;
        case 2:   // rows: A, B, v2 -> R, U; columns: A, B, v1 -> C
            op = OP_A1;
            a.A = tv.F(0); a.Bf = tv.F(1); a.ROUT = tv.F(2); a.UOUT = tv.F(4); a.COUT = tv.F(3);
            if (paper) { a.B = tv.Bt(); a.G = tv.G(slot_G(P, j + 1)); a.bw = T(1.0 / P->nt); }
            fields = (paper ? 11 : 5) + 4;
            break;
        default:  // rows: A, B, v2, v~(2), G(2) -> R, U; columns: A, B, v1 -> C
            op = OP_I1;
            a.A = tv.F(0); a.Bf = tv.F(1); a.VT = tv.vtT(); a.G = tv.G(slot_G(P, j));
            a.ROUT = tv.F(2); a.UOUT = tv.F(4); a.COUT = tv.F(3);
            fields = 9 + 4;
            break;
    }
    return REG_OK;
}

template <typename T>
reg_status time_launches(reg_problem* P, int op, int var, const StageArgs<T>& a, int reps, double* ms) {
    hipError_t err = launch_stage<T>(op, var, a, P->stream);   // warm-up (and validity check)
    if (err != hipSuccess) return fail(REG_EINVAL, "variant %d not available: %s", var, hipGetErrorString(err));
    // best of three timed batches (clock and power-state noise)
    double best = 1e30;
    for (int rep3 = 0; rep3 < 3; ++rep3) {
        hipEvent_t e0, e1;
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
        CK(hipEventRecord(e0, P->stream));
        for (int i = 0; i < reps; ++i) CK(launch_stage<T>(op, var, a, P->stream));
        CK(hipEventRecord(e1, P->stream));
        CK(hipEventSynchronize(e1));
        float t = 0;
        CK(hipEventElapsedTime(&t, e0, e1));
        CK(hipEventDestroy(e0));
        CK(hipEventDestroy(e1));
        if ((double)t / reps < best) best = (double)t / reps;
    }
    *ms = best;
    return REG_OK;
}

// Timed matvecs with the selected stage's launches stamped (direct launches).  phases: four stamps
// per block (F_PHASES) and at most MAX_TIMED / 2 timed launches.  Leaves the host copy of the stamps
// in h (slots per launch = stamps * (n1 + n2) / 2) and the events' mean dispatch interval in ev_ms.
template <typename T>
reg_status timed_matvecs(reg_problem* P, int which, int reps, bool phases, std::vector<unsigned long long>& h,
                         int* timed_out, double* ev_ms_out, double* fields_out, int* khz_out) {
    if (!P->matvec_done) return fail(REG_ESTATE, "run one reg_hessian_matvec before timing passes");
    if (P->p.hessian != REG_HESS_GN) return fail(REG_EINVAL, "the timing hook covers the Gauss-Newton stages");
    if (reps < 1 || reps > 1000) return fail(REG_EINVAL, "reps must be in [1, 1000]");
    const int cap = phases ? MAX_TIMED / 2 : MAX_TIMED;
    if ((long)reps * P->nt > cap)
        return fail(REG_EINVAL, "reps * nt = %ld timed launches exceed %d", (long)reps * P->nt, cap);
    StageArgs<T> a;
    int op;
    CKS(stage_spec<T>(P, which, a, op, *fields_out));
    int dev = 0, khz = 0;
    CK(hipGetDevice(&dev));
    CK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return fail(REG_EDEVICE, "device wall-clock rate unavailable");
    *khz_out = khz;
    const int stamps = phases ? 4 : 2;
    const size_t slots = clk_slots(&P->p);
    P->clk_stride = stamps * slots;
    const int launches = reps * P->nt;
    while (P->tev.size() < 2 * (size_t)launches) {
        hipEvent_t e;
        CK(hipEventCreate(&e));
        P->tev.push_back(e);
    }
    unsigned long long* clk = P->at<unsigned long long>(P->o.clk);
    CK(launch_clk_init(clk, (int)(launches * slots * stamps / 2), P->stream));
    P->timing_op = op;
    P->clk_used = 0;
    P->clk_max = cap;
    P->clk_phases = phases;
    reg_status st = REG_OK;
    for (int r = 0; r < reps && st == REG_OK; ++r)
        st = matvec_t<T>(P, P->at<double>(P->o.vt64), P->pcg(PST), nullptr);
    P->timing_op = -1;
    P->clk_phases = false;
    CKS(st);
    const int timed = P->clk_used;
    if (timed == 0) return fail(REG_EINVAL, "no launches of the selected stage");
    h.assign((size_t)timed * stamps * slots, 0);
    CK(hipMemcpyAsync(h.data(), clk, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, P->stream));
    CK(hipStreamSynchronize(P->stream));
    double ev_ms = 0;
    for (int i = 0; i < timed; ++i) {
        float t = 0;
        CK(hipEventElapsedTime(&t, P->tev[2 * i], P->tev[2 * i + 1]));
        ev_ms += t;
    }
    *timed_out = timed;
    *ev_ms_out = ev_ms / timed;
    return REG_OK;
}

// Mean device time of the selected stage's launches inside `reps` real matvecs (direct launches):
//  * ms: the dispatch interval, from start / end events that the dispatch itself stamps
//    (hipExtLaunchKernelGGL) -- what a profiler reports as the kernel's duration;
//  * exec_ms: the blocks' execution interval: every block records its start and its end after its
//    stores completed on the device wall clock; latest end minus earliest start.
// The difference is the workgroup dispatch ramp and the end-of-kernel completion.
template <typename T>
reg_status time_pass_t(reg_problem* P, int which, int reps, double* ms, double* bytes, double* exec_ms) {
    std::vector<unsigned long long> h;
    int timed = 0, khz = 0;
    double ev = 0, fields = 0;
    CKS(timed_matvecs<T>(P, which, reps, false, h, &timed, &ev, &fields, &khz));
    const size_t slots = clk_slots(&P->p);
    double ticks = 0;
    for (int i = 0; i < timed; ++i) {
        unsigned long long t0 = ~0ull, t1 = 0;
        for (size_t b = 0; b < slots; ++b) {
            const unsigned long long s0 = h[(i * slots + b) * 2], s1 = h[(i * slots + b) * 2 + 1];
            if (s0 != ~0ull) t0 = std::min(t0, s0);   // untouched slots keep the sentinels
            if (s1 != 0ull) t1 = std::max(t1, s1);
        }
        if (t0 == ~0ull || t1 < t0) return fail(REG_EDEVICE, "timed launch %d recorded no interval", i);
        ticks += (double)(t1 - t0);
    }
    *ms = ev;
    if (exec_ms) *exec_ms = ticks / timed / (double)khz;   // khz ticks per millisecond
    *bytes = fields * (double)P->nn * sizeof(T);
    return REG_OK;
}

// Phase mode (F_PHASES): us[0] dispatch interval, us[1] block execution interval, us[2] spread of
// the block starts (latest minus earliest), and the per-block means of us[3] start -> loads arrived,
// us[4] -> transforms done, us[5] -> stores acknowledged, over the blocks that stamped all four
// (the one-launch FP32 stages of square grids; 0 where none did).  Microseconds per launch.
template <typename T>
reg_status time_phases_t(reg_problem* P, int which, int reps, double* us) {
    std::vector<unsigned long long> h;
    int timed = 0, khz = 0;
    double ev = 0, fields = 0;
    CKS(timed_matvecs<T>(P, which, reps, true, h, &timed, &ev, &fields, &khz));
    const size_t slots = clk_slots(&P->p);
    double exec = 0, spread = 0, ph[3] = {0, 0, 0};
    long nb = 0;
    for (int i = 0; i < timed; ++i) {
        unsigned long long t0 = ~0ull, t1 = 0, s_last = 0;
        for (size_t b = 0; b < slots; ++b) {
            const unsigned long long* q = &h[(i * slots + b) * 4];
            if (q[0] == ~0ull) continue;   // no such block
            t0 = std::min(t0, q[0]);
            s_last = std::max(s_last, q[0]);
            t1 = std::max(t1, q[3]);
            if (q[1] != 0ull && q[2] != ~0ull && q[0] <= q[1] && q[1] <= q[2] && q[2] <= q[3]) {
                ph[0] += (double)(q[1] - q[0]);
                ph[1] += (double)(q[2] - q[1]);
                ph[2] += (double)(q[3] - q[2]);
                ++nb;
            }
        }
        if (t0 == ~0ull || t1 < t0) return fail(REG_EDEVICE, "timed launch %d recorded no interval", i);
        exec += (double)(t1 - t0);
        spread += (double)(s_last - t0);
    }
    const double us_per_tick = 1e3 / (double)khz;
    us[0] = ev * 1e3;
    us[1] = exec / timed * us_per_tick;
    us[2] = spread / timed * us_per_tick;
    for (int k = 0; k < 3; ++k) us[3 + k] = nb ? ph[k] / nb * us_per_tick : 0.0;
    return REG_OK;
}

const char* op_name(int op) {
    static const char* n[7] = {"S1", "S2", "A1", "A2", "I1", "I2", "GRAD"};
    return n[op];
}

// Best of three batches of `reps` graph-replayed matvecs on the last projected input (ms per matvec).
reg_status matvec_batch_ms(reg_problem* P, int reps, double* ms) {
    double* in = P->at<double>(P->o.vt64);
    double* out = P->pcg(PST);
    CKS(matvec_run<float>(P, in, out, nullptr));   // capture with the current shapes, warm-up
    double best = 1e30;
    for (int b = 0; b < 3; ++b) {
        hipEvent_t e0, e1;
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
        CK(hipEventRecord(e0, P->stream));
        reg_status st = REG_OK;
        for (int i = 0; i < reps && st == REG_OK; ++i) st = matvec_run<float>(P, in, out, nullptr);
        CK(hipEventRecord(e1, P->stream));
        CK(hipEventSynchronize(e1));
        float t = 0;
        CK(hipEventElapsedTime(&t, e0, e1));
        CK(hipEventDestroy(e0));
        CK(hipEventDestroy(e1));
        CKS(st);
        best = std::min(best, (double)t / reps);
    }
    *ms = best;
    return REG_OK;
}

// Two rounds: every shape that fits, timed per stage op in isolation (repeated launches of one
// stage on the same operands), then whole graph-replayed matvecs decide among the isolated sweep's
// four fastest shapes of each op, one op at a time (coordinate descent; a change is kept when it
// saves more than 0.1%).  In a matvec each step reads other trajectory fields and follows other
// stages, which the isolated timings do not see.
reg_status autotune_f32(reg_problem* P, int reps, char* report, size_t cap) {
    if (!P->matvec_done) return fail(REG_ESTATE, "run one reg_hessian_matvec before tuning");
    if (reps < 1) return fail(REG_EINVAL, "reps must be >= 1");
    std::string js = "{";
    std::vector<std::pair<double, int>> iso[4];
    int ops[4] = {};
    for (int which = 0; which < 4; ++which) {
        StageArgs<float> a;
        int op;
        double fields;
        CKS(stage_spec<float>(P, which, a, op, fields));
        int best = P->var[op];
        double best_ms = 1e30;
        char buf[96];
        snprintf(buf, sizeof buf, "%s\"%s\": [", which ? ", " : "", op_name(op));
        js += buf;
        bool firstv = true;
        for (int v = 0; v < NUM_STAGE_VARIANTS; ++v) {
            double ms = 0;
            if (!stage_variant_fits_f32(P->n1, P->n2, v)) continue;
            if (time_launches<float>(P, op, v, a, reps, &ms) != REG_OK) continue;
            snprintf(buf, sizeof buf, "%s[%d, %.3f]", firstv ? "" : ", ", v, ms * 1e3);
            js += buf;
            firstv = false;
            iso[which].push_back({ms, v});
            if (ms < best_ms) { best_ms = ms; best = v; }
        }
        js += "]";
        P->var[op] = best;
        ops[which] = op;
    }
    drop_graphs(P);
    const int mreps = P->nn >= 512L * 512 ? 3 : 10;
    double cur = 0;
    CKS(matvec_batch_ms(P, mreps, &cur));
    char buf[96];
    snprintf(buf, sizeof buf, ", \"matvec_ms_isolated_choice\": %.4f", cur);
    js += buf;
    for (int which = 0; which < 4; ++which) {
        std::sort(iso[which].begin(), iso[which].end());
        const int op = ops[which];
        for (size_t c = 0; c < iso[which].size() && c < 4; ++c) {
            const int v = iso[which][c].second;
            if (v == P->var[op]) continue;
            const int prev = P->var[op];
            P->var[op] = v;
            drop_graphs(P);
            double ms = 0;
            CKS(matvec_batch_ms(P, mreps, &ms));
            if (ms < cur * 0.999) cur = ms;
            else P->var[op] = prev;
        }
    }
    drop_graphs(P);
    snprintf(buf, sizeof buf, ", \"matvec_ms\": %.4f", cur);
    js += buf;
    js += ", \"chosen\": [";
    for (int op = 0; op < NUM_TUNED_OPS; ++op) js += std::to_string(P->var[op]) + (op < NUM_TUNED_OPS - 1 ? ", " : "");
    js += "]}";
    g_err = "no error";
    if (report && cap > 0) {
        strncpy(report, js.c_str(), cap - 1);
        report[cap - 1] = 0;
    }
    return REG_OK;
}

void twiddles(int n, std::vector<cpx<float>>& f, std::vector<cpx<double>>& d) {
    f.resize(n);
    d.resize(n);
    for (int m = 0; m < n; ++m) {
        const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
        const double c = (double)cosl(ang), s = (double)sinl(ang);
        d[m] = {c, s};
        f[m] = {(float)c, (float)s};
    }
}

// Circulant spectral derivative of length n (used for lengths that are not powers of two):
// c_m = (1/n) sum_k i k~ exp(2 pi i k m / n) = -(1/n) sum_k k~ sin(2 pi k m / n), k~ the signed
// wavenumber with the Nyquist index set to 0 (the transform pair's operator written as a convolution).
void circulant_derivative(int n, std::vector<float>& f, std::vector<double>& d) {
    f.assign(n, 0.0f);
    d.assign(n, 0.0);
    const long double pi2 = 2.0L * 3.14159265358979323846264338327950288L;
    for (int m = 0; m < n; ++m) {
        long double acc = 0.0L;
        for (int k = 0; k < n; ++k) {
            const int kt = k < n / 2 ? k : (2 * k == n ? 0 : k - n);
            if (kt == 0) continue;
            acc -= (long double)kt * sinl(pi2 * (long double)(((long)k * m) % n) / (long double)n);
        }
        d[m] = (double)(acc / n);
        f[m] = (float)d[m];
    }
}

#define DISPATCH(P, call_f, call_d) ((P)->f64 ? (call_d) : (call_f))

}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
// Copy (and convert) the two images into the workspace and check that they are finite.
static reg_status load_images(reg_problem* P, const double* m_T, const double* m_R) {
    const Offsets& o = P->o;
    if (P->f64) {
        CK(launch_convert<double>(P->nn, m_T, P->at<double>(o.mT), P->stream));
        CK(launch_convert<double>(P->nn, m_R, P->at<double>(o.mR), P->stream));
    } else {
        CK(launch_convert<float>(P->nn, m_T, P->at<float>(o.mT), P->stream));
        CK(launch_convert<float>(P->nn, m_R, P->at<float>(o.mR), P->stream));
        CK(launch_convert<double>(P->nn, m_T, P->at<double>(o.mT64), P->stream));
        CK(launch_convert<double>(P->nn, m_R, P->at<double>(o.mR64), P->stream));
    }
    const double* a[2] = {m_T, m_R};
    CK(launch_dots<double>(2, a, a, P->nn, P->partial(), P->scal(), P->stream));
    double r[2];
    CK(hipMemcpyAsync(r, P->scal(), sizeof r, hipMemcpyDeviceToHost, P->stream));
    CK(hipStreamSynchronize(P->stream));
    if (!std::isfinite(r[0]) || !std::isfinite(r[1])) return fail(REG_EINVAL, "m_T or m_R contains non-finite values");
    P->linearized = false;
    P->matvec_done = false;
    return REG_OK;
}

extern "C" {

const char* reg_last_error(void) { return g_err.c_str(); }

reg_status reg_workspace_bytes(const reg_params* params, size_t* bytes) {
    CKS(check_params(params));
    if (!bytes) return fail(REG_EINVAL, "bytes is NULL");
    *bytes = layout(params).total;
    return REG_OK;
}

reg_status reg_create(const reg_params* params, const double* m_T, const double* m_R, void* workspace,
                      size_t workspace_bytes, void* hip_stream, reg_problem** out) {
    CKS(check_params(params));
    if (!out || !m_T || !m_R || !workspace) return fail(REG_EINVAL, "NULL argument");
    if (((uintptr_t)workspace & 255) != 0) return fail(REG_EINVAL, "workspace must be 256-byte aligned");
    Offsets o = layout(params);
    if (workspace_bytes < o.total)
        return fail(REG_ENOMEM, "workspace of %zu bytes is smaller than the %zu bytes needed", workspace_bytes, o.total);
    reg_problem* P = new (std::nothrow) reg_problem();
    if (!P) return fail(REG_ENOMEM, "host allocation failed");
    P->p = *params;
    P->stream = (hipStream_t)hip_stream;
    P->n1 = params->n1;
    P->n2 = params->n2;
    P->nt = params->nt;
    P->nn = (long)params->n1 * params->n2;
    P->f64 = params->precision == REG_FP64;
    P->ws = (char*)workspace;
    P->o = o;
    P->sp = SpecParams{params->n1, params->n2, params->norm, params->constraint, params->beta_v, params->beta_w,
                       MrPlan{}, MrPlan{}};
    // mixed-radix plans for axis lengths that are not powers of two (ns = 0 otherwise)
    if ((P->n1 & (P->n1 - 1)) != 0) P->sp.mr1 = mr_plan(P->n1);
    if ((P->n2 & (P->n2 - 1)) != 0) P->sp.mr2 = mr_plan(P->n2);
    P->sp.eta_sum = P->scal() + SC_ETA + 2;
    P->h1h2 = (2.0 * M_PI / params->n1) * (2.0 * M_PI / params->n2);
    std::vector<cpx<float>> f1, f2;
    std::vector<cpx<double>> d1, d2;
    twiddles(P->n1, f1, d1);
    twiddles(P->n2, f2, d2);
    auto cleanup = [&](reg_status s) { delete P; return s; };
#define CKC(call)                                                                                       \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return cleanup(fail(REG_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)));           \
    } while (0)
    CKC(hipMemcpyAsync(P->ws + o.tw1f, f1.data(), f1.size() * sizeof(f1[0]), hipMemcpyHostToDevice, P->stream));
    CKC(hipMemcpyAsync(P->ws + o.tw2f, f2.data(), f2.size() * sizeof(f2[0]), hipMemcpyHostToDevice, P->stream));
    CKC(hipMemcpyAsync(P->ws + o.tw1d, d1.data(), d1.size() * sizeof(d1[0]), hipMemcpyHostToDevice, P->stream));
    CKC(hipMemcpyAsync(P->ws + o.tw2d, d2.data(), d2.size() * sizeof(d2[0]), hipMemcpyHostToDevice, P->stream));
    std::vector<float> c1f, c2f;
    std::vector<double> c1d, c2d;
    if ((P->n1 & (P->n1 - 1)) != 0) circulant_derivative(P->n1, c1f, c1d);
    if ((P->n2 & (P->n2 - 1)) != 0) circulant_derivative(P->n2, c2f, c2d);
    if (!c1d.empty()) {
        CKC(hipMemcpyAsync(P->ws + o.dc1f, c1f.data(), c1f.size() * sizeof(float), hipMemcpyHostToDevice, P->stream));
        CKC(hipMemcpyAsync(P->ws + o.dc1d, c1d.data(), c1d.size() * sizeof(double), hipMemcpyHostToDevice, P->stream));
    }
    if (!c2d.empty()) {
        CKC(hipMemcpyAsync(P->ws + o.dc2f, c2f.data(), c2f.size() * sizeof(float), hipMemcpyHostToDevice, P->stream));
        CKC(hipMemcpyAsync(P->ws + o.dc2d, c2d.data(), c2d.size() * sizeof(double), hipMemcpyHostToDevice, P->stream));
    }
    CKC(hipStreamSynchronize(P->stream));   // the host tables go out of scope
    {
        reg_status st = load_images(P, m_T, m_R);
        if (st != REG_OK) return cleanup(st);
    }
#undef CKC
    *out = P;
    return REG_OK;
}

reg_status reg_set_images(reg_problem* h, const double* m_T, const double* m_R) {
    if (!h || !m_T || !m_R) return fail(REG_EINVAL, "NULL argument");
    return load_images(h, m_T, m_R);
}

reg_status reg_destroy(reg_problem* h) {
    if (!h) return REG_OK;
    drop_graphs(h);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    for (hipEvent_t e : h->tev) (void)hipEventDestroy(e);
    delete h;
    return REG_OK;
}

reg_status reg_set_stream(reg_problem* h, void* hip_stream) {
    if (!h) return fail(REG_EINVAL, "NULL handle");
    h->stream = (hipStream_t)hip_stream;
    return REG_OK;
}

reg_status reg_state_forward(reg_problem* h, const double* v, double* m1) {
    if (!h || !v || !m1) return fail(REG_EINVAL, "NULL argument");
    double* vp = h->at<double>(h->o.vtrial);
    if (h->f64) {
        CKS(project<double>(h, v, vp, (double*)nullptr));
        CKS(state_forward<double>(h, vp, false, h->sF(7), (double*)nullptr));
    } else {
        CKS(project<float>(h, v, vp, (float*)nullptr));
        CKS(state_forward<float>(h, vp, false, h->sF(7), (float*)nullptr));
    }
    CK(hipMemcpyAsync(m1, h->sF(7), h->nn * 8, hipMemcpyDeviceToDevice, h->stream));
    return REG_OK;
}

reg_status reg_objective(reg_problem* h, const double* v, double* J_host, double* terms3_host) {
    if (!h || !v || !J_host) return fail(REG_EINVAL, "NULL argument");
    return DISPATCH(h, objective_t<float>(h, v, J_host, terms3_host), objective_t<double>(h, v, J_host, terms3_host));
}

reg_status reg_gradient(reg_problem* h, const double* v, double* g, double* J_host) {
    if (!h || !v || !g) return fail(REG_EINVAL, "NULL argument");
    return DISPATCH(h, gradient_t<float>(h, v, g, nullptr, J_host), gradient_t<double>(h, v, g, nullptr, J_host));
}

reg_status reg_hessian_matvec(reg_problem* h, const double* vtilde, double* Hv) {
    if (!h || !vtilde || !Hv) return fail(REG_EINVAL, "NULL argument");
    if (vtilde == Hv) return fail(REG_EINVAL, "vtilde and Hvtilde may not alias");
    if (!h->linearized) return fail(REG_ESTATE, "no linearisation point: call reg_gradient first");
    double* vt64 = h->at<double>(h->o.vt64);
    if (h->f64) {
        CKS(project<double>(h, vtilde, vt64, TV<double>{h}.vtT()));
        return matvec_run<double>(h, vt64, Hv, nullptr);
    }
    CKS(project<float>(h, vtilde, vt64, TV<float>{h}.vtT()));
    return matvec_run<float>(h, vt64, Hv, nullptr);
}

reg_status reg_precond_apply(reg_problem* h, const double* r, double* z) {
    if (!h || !r || !z) return fail(REG_EINVAL, "NULL argument");
    return precond_t(h, r, z, nullptr);
}

reg_status reg_pcg(reg_problem* h, const double* rhs, double eta, int32_t max_iters, int32_t fixed_iters,
                   double* x, int32_t* iters_host, double* relres_host) {
    if (!h || !rhs || !x) return fail(REG_EINVAL, "NULL argument");
    if (!h->linearized) return fail(REG_ESTATE, "no linearisation point: call reg_gradient first");
    if (max_iters < 0 || fixed_iters < 0 || (max_iters == 0 && fixed_iters == 0))
        return fail(REG_EINVAL, "iteration limits");
    double* r = h->at<double>(h->o.tmp1);
    CKS(project<double>(h, rhs, r, (double*)nullptr));
    int it = 0;
    double rr = 0;
    reg_status s = DISPATCH(h, pcg_t<float>(h, r, eta, max_iters, fixed_iters, x, &it, &rr, nullptr),
                            pcg_t<double>(h, r, eta, max_iters, fixed_iters, x, &it, &rr, nullptr));
    if (s != REG_OK) return s;
    CK(hipStreamSynchronize(h->stream));
    if (iters_host) *iters_host = it;
    if (relres_host) *relres_host = rr;
    return REG_OK;
}

static reg_status check_opts(const reg_problem* h, const reg_solve_opts* opts) {
    if (opts->max_newton < 0 || opts->max_pcg < 1 || opts->fixed_pcg_iters < 0 || opts->max_backtracks < 0 ||
        !(opts->armijo_rho > 0 && opts->armijo_rho < 1) || !(opts->armijo_c1 > 0 && opts->armijo_c1 < 1))
        return fail(REG_EINVAL, "bad solve options");
    const int cap = h->p.lowrank_capacity;
    if (opts->rank < 0 || opts->rank > std::min(cap, LR_MIX_MAX))
        return fail(REG_EINVAL, "rank=%d: must be in [0, min(lowrank_capacity=%d, %d)]", opts->rank, cap, LR_MIX_MAX);
    if (opts->rank > 0 && !opts->precond_U) return fail(REG_EINVAL, "rank > 0 needs precond_U");
    if (opts->recycle < 0 || (opts->recycle > 0 && cap == 0))
        return fail(REG_EINVAL, "recycle=%d needs lowrank_capacity > 0", opts->recycle);
    if (h->p.norm == REG_STOKES && h->p.constraint == REG_MASS_SOURCE && (opts->rank > 0 || opts->recycle > 0))
        return fail(REG_EINVAL, "no preconditioner correction for REG_STOKES with REG_MASS_SOURCE (its W-product "
                                "moves with the linearisation point)");
    if (!(opts->cfl_max >= 0.0) || !std::isfinite(opts->cfl_max)) return fail(REG_EINVAL, "cfl_max must be >= 0");
    if (opts->max_steps < 0 || (opts->max_steps > 0 && !opts->steps))
        return fail(REG_EINVAL, "max_steps=%d needs a record array", opts->max_steps);
    return REG_OK;
}

reg_status reg_solve(reg_problem* h, const reg_solve_opts* opts, double* v_out, reg_solve_stats* stats_host) {
    if (!h || !opts || !v_out) return fail(REG_EINVAL, "NULL argument");
    CKS(check_opts(h, opts));
    return DISPATCH(h, solve_t<float>(h, opts, v_out, stats_host), solve_t<double>(h, opts, v_out, stats_host));
}

reg_status reg_batch_solve(int32_t count, reg_problem* const* problems, const reg_solve_opts* opts,
                           double* const* v_out, reg_solve_stats* stats_host) {
    if (count < 0 || (count > 0 && (!problems || !opts || !v_out)))
        return fail(REG_EINVAL, "NULL argument or negative count");
    for (int i = 0; i < count; ++i)
        if (!problems[i] || !v_out[i]) return fail(REG_EINVAL, "problem %d or its output is NULL", i);
    for (int i = 0; i < count; ++i)
        for (int k = 0; k < i; ++k)
            if (problems[i] == problems[k]) return fail(REG_EINVAL, "problem %d appears twice", i);
    for (int i = 0; i < count; ++i) CKS(check_opts(problems[i], &opts[i]));
    // largest problems first (most work per pair), then a shared work counter
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const double wa = (double)problems[a]->nn * problems[a]->nt, wb = (double)problems[b]->nn * problems[b]->nt;
        return wa > wb;
    });
    // concurrent solves: REGNK_BATCH_WORKERS (1..32) if set, else 8.  Each worker drives its own
    // stream; how many run at once on the GPU is bounded by the process's hardware queues
    // (GPU_MAX_HW_QUEUES).
    int want = 8;
    if (const char* e = std::getenv("REGNK_BATCH_WORKERS")) {
        const int w = std::atoi(e);
        if (w >= 1 && w <= 32) want = w;
    }
    const int nworkers = std::min(count, want);
    std::atomic<int> next{0};
    std::vector<reg_status> status(count, REG_OK);
    std::vector<std::string> errs(count);
    std::vector<reg_solve_stats> stats(count);
    std::vector<hipError_t> stream_err(nworkers, hipSuccess);
    auto worker = [&](int w) {
        hipStream_t st = nullptr;
        stream_err[w] = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (stream_err[w] != hipSuccess) return;
        for (int k = next.fetch_add(1); k < count; k = next.fetch_add(1)) {
            const int i = order[k];
            reg_problem* P = problems[i];
            hipStream_t saved = P->stream;
            // the caller's stream may still hold work for this problem (its create, earlier calls)
            if (hipStreamSynchronize(saved) != hipSuccess) {
                status[i] = REG_EDEVICE;
                errs[i] = "stream synchronisation failed";
                continue;
            }
            P->stream = st;
            status[i] = P->f64 ? solve_t<double>(P, &opts[i], v_out[i], &stats[i])
                               : solve_t<float>(P, &opts[i], v_out[i], &stats[i]);
            if (status[i] != REG_OK) errs[i] = g_err;
            P->stream = saved;
        }
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    };
    std::vector<std::thread> pool;
    for (int w = 0; w < nworkers; ++w) pool.emplace_back(worker, w);
    for (auto& t : pool) t.join();
    for (int w = 0; w < nworkers; ++w)
        if (stream_err[w] != hipSuccess) return fail(REG_EDEVICE, "stream creation failed: %s", hipGetErrorString(stream_err[w]));
    if (stats_host)
        for (int i = 0; i < count; ++i) stats_host[i] = stats[i];
    for (int i = 0; i < count; ++i)
        if (status[i] != REG_OK && status[i] != REG_ENOTCONV)
            return fail(status[i], "pair %d: %s", i, errs[i].c_str());
    for (int i = 0; i < count; ++i)
        if (status[i] == REG_ENOTCONV) return fail(REG_ENOTCONV, "pair %d: %s", i, errs[i].c_str());
    return REG_OK;
}

reg_status reg_ritz_directions(reg_problem* h, double* U, int32_t rank, int32_t iters, double* theta_host) {
    if (!h || !U) return fail(REG_EINVAL, "NULL argument");
    if (!h->linearized) return fail(REG_ESTATE, "no linearisation point: call reg_gradient first");
    if (rank < 1 || rank > LR_MIX_MAX || rank > h->p.lowrank_capacity)
        return fail(REG_EINVAL, "rank=%d out of [1, min(%d, lowrank_capacity=%d)]", rank, LR_MIX_MAX,
                    h->p.lowrank_capacity);
    if (iters < 0 || iters > 100) return fail(REG_EINVAL, "iters=%d out of [0, 100]", iters);
    if (h->p.norm == REG_STOKES && h->p.constraint == REG_MASS_SOURCE)
        return fail(REG_EINVAL, "no low-rank directions for the shear-control model with a mass source");
    return DISPATCH(h, ritz_t<float>(h, U, rank, iters, theta_host), ritz_t<double>(h, U, rank, iters, theta_host));
}

reg_status reg_cfl(reg_problem* h, const double* v, double* cfl_host) {
    if (!h || !v || !cfl_host) return fail(REG_EINVAL, "NULL argument");
    double* vp = h->at<double>(h->o.vtrial);
    CKS(project<double>(h, v, vp, (double*)nullptr));
    return cfl_t(h, vp, cfl_host);
}

reg_status reg_deformation_workspace_bytes(const reg_params* params, size_t* bytes) {
    CKS(check_params(params));
    if (!bytes) return fail(REG_EINVAL, "bytes is NULL");
    *bytes = (size_t)DEF_FIELDS * params->n1 * params->n2 * sizeof(double);
    return REG_OK;
}

reg_status reg_deformation(reg_problem* h, const double* v, void* workspace, size_t workspace_bytes, double* u1,
                           double* F1, double* detF1, double* stats_host) {
    if (!h || !v || !workspace) return fail(REG_EINVAL, "NULL argument");
    const size_t need = (size_t)DEF_FIELDS * h->nn * sizeof(double);
    if (workspace_bytes < need) return fail(REG_ENOMEM, "diagnostics workspace of %zu bytes, %zu needed", workspace_bytes, need);
    if ((uintptr_t)workspace % 256 != 0) return fail(REG_EINVAL, "workspace must be 256-byte aligned");
    return deformation_run(h, v, (double*)workspace, u1, F1, detF1, stats_host);
}

// ---- allocation-free variant of reg_deformation ------------------------------------------------
// The diagnostics workspace lives in a file-scope device array (one copy per GPU, kept until the
// process ends).  In host code `scratch` only names the symbol: its device address on the current GPU
// comes from hipGetSymbolAddress, taken once per device on the first call and kept.
constexpr size_t DEF_STATIC_MAX_POINTS = 65536;   // grids up to 256 x 256 (n1 n2 <= 65536)
static __device__ __align__(256) double scratch[(size_t)DEF_FIELDS * DEF_STATIC_MAX_POINTS];

namespace {
constexpr int MAX_DEVICES = 64;
std::atomic<double*> g_scratch[MAX_DEVICES];
std::mutex g_scratch_mutex;

reg_status static_scratch(double** out) {
    int dev = -1;
    CK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(REG_EDEVICE, "device index %d out of range", dev);
    double* p = g_scratch[dev].load();
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        p = g_scratch[dev].load();
        if (!p) {
            void* addr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !addr)
                return fail(REG_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            p = static_cast<double*>(addr);
            g_scratch[dev].store(p);
        }
    }
    *out = p;
    return REG_OK;
}
}  // namespace

reg_status reg_deformation_static(reg_problem* h, const double* v, double* u1, double* F1, double* detF1,
                                  double* stats_host) {
    if (!h || !v) return fail(REG_EINVAL, "NULL argument");
    if ((size_t)h->nn > DEF_STATIC_MAX_POINTS)
        return fail(REG_EINVAL, "grid of %ld points exceeds the %zu points of the static diagnostics scratch (use "
                                "reg_deformation with a caller workspace)", h->nn, DEF_STATIC_MAX_POINTS);
    double* ws = nullptr;
    CKS(static_scratch(&ws));
    return deformation_run(h, v, ws, u1, F1, detF1, stats_host);
}

reg_status reg_time_pass(reg_problem* h, int32_t which, int32_t reps, double* ms, double* bytes, double* exec_ms) {
    if (!h || !ms || !bytes) return fail(REG_EINVAL, "NULL argument");
    return DISPATCH(h, time_pass_t<float>(h, which, reps, ms, bytes, exec_ms),
                    time_pass_t<double>(h, which, reps, ms, bytes, exec_ms));
}

reg_status reg_time_phases(reg_problem* h, int32_t which, int32_t reps, double* phase_us_host) {
    if (!h || !phase_us_host) return fail(REG_EINVAL, "NULL argument");
    return DISPATCH(h, time_phases_t<float>(h, which, reps, phase_us_host),
                    time_phases_t<double>(h, which, reps, phase_us_host));
}

reg_status reg_autotune(reg_problem* h, int32_t reps, char* report, size_t report_bytes) {
    if (!h) return fail(REG_EINVAL, "NULL handle");
    if (h->f64) {   // FP64 passes use one fixed shape
        if (report && report_bytes > 0) {
            strncpy(report, "{\"fp64\": \"fixed shapes\"}", report_bytes - 1);
            report[report_bytes - 1] = 0;
        }
        return REG_OK;
    }
    drop_graphs(h);
    return autotune_f32(h, reps, report, report_bytes);
}

reg_status reg_set_pass_variants(reg_problem* h, const int32_t* variants, int32_t count) {
    if (!h || !variants) return fail(REG_EINVAL, "NULL argument");
    if (count != 7) return fail(REG_EINVAL, "count must be 7 (one launch shape per stage op)");
    for (int op = 0; op < 7; ++op)
        if (variants[op] < 0 || variants[op] >= NUM_STAGE_VARIANTS) return fail(REG_EINVAL, "variant index out of range");
    for (int op = 0; op < NUM_TUNED_OPS; ++op) h->var[op] = variants[op];
    drop_graphs(h);
    return REG_OK;
}

}  // extern "C"
