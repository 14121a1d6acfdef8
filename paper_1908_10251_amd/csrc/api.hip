// Host orchestration and the C ABI (include/pasm.h).
//
// One pasm_iterate is one correction step (Algorithm 1) for all k eigenpairs:
//   1. f = lambda M_h u; a fixed number of V-cycles for A_h u~ = f from u
//      (Algorithm 1, step 1).  In mixed precision every V-cycle runs in FP32
//      on the FP64 residual r = f - A_h x and its result is added to x in FP64
//      (defect correction), so the FP64 fixed point is unchanged.
//   2. borders b = P^T A u~, c = P^T M u~, beta, zeta (one fine sweep plus a
//      restriction chain), p = Q^T b, q = Q^T c, the arrowhead eigensolve and
//      selection (coarse.hip), u_new = P Q y' + s u~, lambda_new = mu
//      (Algorithm 1, step 2; Section 3.1).
// Algorithm 2 with h_1 = H is pasm_setup (coarse eigenproblem, start
// u_i = P q_i, lambda_i = theta_i) followed by pasm_solve.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <random>
#include <type_traits>

#include "common.h"

namespace pasm {

long arrow_work_doubles(int N, int k);
size_t arrow_workspace_bytes(int N, int k);

Grid make_grid(int dim, int n) {
    Grid g;
    g.dim = dim;
    g.n = n;
    g.m = n - 1;
    g.pitch = ((n + 1 + ORIGIN) + 15) / 16 * 16;
    long rows = (long)(n + 1) * (dim == 3 ? (n + 1) : 1);
    long pl = rows * g.pitch;
    g.plane = (pl + 63) / 64 * 64;
    g.h = 1.0 / n;
    return g;
}

namespace {

struct Level {
    Grid g;
    bool const_coef = true;
    bool general = false;  // general 7-point stencil (potential term present)
    bool general3 = false; // 3D general 15-point stencil (tensor, kappa or potential)
    double* s64 = nullptr; // its 8 planes (FP64), and FP32 copies for mixed cycles
    float* s32 = nullptr;
    double w0 = 1.0;
    double rho = 2.0;
    // coefficient arrays: 0 wx, 1 wy, 2 wz, 3 diagonal, 4 north-east weight
    double* w64[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    float* w32[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    std::vector<Cheb> pre, post;
    // V-cycle vectors of this level (type of the V-cycle), levels below the finest
    void* X = nullptr;
    void* F = nullptr;
    void* Y = nullptr;
    // FP64 border / prolongation chain vectors
    double* B = nullptr;
    double* C = nullptr;
    // conjugate-gradient smoothing work (PASM_CG)
    CgWork cg{};
};

}  // namespace
}  // namespace pasm

namespace pasm {
namespace {
// The host state a correction step's launches depend on beyond the
// context's fixed set-up: the rotating buffers, the eigenvalue buffers and
// the flags that say which fused pass forms what.  Two steps that start from
// equal states (and the same deferral) launch the same kernels with the same
// arguments and leave equal states behind.
struct StepState {
    double *U, *F64, *Y64, *R64;
    double *lam, *lam_prev, *mu;
    const double* pend_beta;
    int border_nblk;
    bool f_ready, r32_ready, border_next, border_done, pair_next, fine_pre_done, prolong_pending, e_pending, e_split;
    bool same(const StepState& o) const { return std::memcmp(this, &o, sizeof *this) == 0; }
};
struct StepGraph {
    StepState pre, post;
    bool defer;
    hipGraph_t graph;
    hipGraphExec_t exec;
};
}  // namespace
}  // namespace pasm

using pasm::Cheb;
using pasm::Coef;
using pasm::Error;
using pasm::Grid;

struct pasm_ctx {
    int dim = 2, k = 0, L = 0, NH = 0;
    pasm_options opt{};
    hipStream_t st = nullptr;
    int device = 0;        // the GPU current at set-up (the stream's device)
    bool own_stream = false;
    bool mixed = false;
    bool fuse = true;      // temporal blocking of smoothing phases (2D)
    // The correction step's right-hand side f = lam M u is never stored: the
    // FP64 residual passes of a mixed-precision step form it from u (2D edge
    // weights, at most two V-cycles, so that u is still the step's start).
    bool f_mass = false;
    // R32 holds the first residual of the next correction step (formed by
    // the prolongation pass that produced u; f_mass contexts)
    bool r32_ready = false;
    std::vector<pasm::Level> lv;
    // finest level, FP64 (padded layout: boundary entries stay zero)
    double *U = nullptr, *F64 = nullptr, *Y64 = nullptr, *R64 = nullptr;
    // compact [k][N] staging for host transfers; never used as a padded grid
    double* stage = nullptr;
    // finest level, FP32 (mixed)
    float *E32 = nullptr, *R32 = nullptr, *Y32 = nullptr;
    // 2D mixed: the last cycle's correction while E32 still holds the one
    // before (u + E32 not stored; the border pass adds both, e_split)
    float* E2_32 = nullptr;
    // coarse space
    double *theta = nullptr, *Qcm = nullptr, *Qrm = nullptr, *Ainv64 = nullptr;
    float* Ainv32 = nullptr;
    // sine-transform tables of a constant-coefficient 2D coarse operator
    // (nullptr: the coarse solve is the dense product with A_H^{-1})
    double *dstS = nullptr, *dstInv = nullptr;
    int* group = nullptr;
    double *bz = nullptr, *partial = nullptr, *pp = nullptr, *qq = nullptr, *ycoef = nullptr;
    double *s = nullptr, *mu = nullptr, *lam = nullptr, *lam_prev = nullptr, *score = nullptr;
    int *rank = nullptr, *flags = nullptr;
    void* awork = nullptr;
    void* dmv = nullptr;   // split-K workspace of the dense coarse products
    std::vector<void*> allocs;
    std::vector<double> lam_h, lam_prev_h;
    std::vector<double> theta_h;  // the k smallest coarse Ritz values (the start), kept on the host
    // Algorithm 2, step 2(A): contexts of the intermediate levels h_2 .. h_{n-1}
    // (built on first use; they share this context's coarse space and stream),
    // and the per-element kappa of those levels (host, when kappa is given)
    std::vector<pasm_ctx*> nested;
    std::vector<std::vector<double>> level_kappa;
    std::vector<double> AH3;  // set-up only: the dense coarse operator of a 3D general problem
    bool general_coef = false;    // a potential term: the nested levels are not rediscretisations
    bool coarse_shared = false;   // theta, Q, A_H^{-1}, groups belong to another context
    double* zeros = nullptr;      // k zeros: the combination weights of a restart
    double* lam_pin = nullptr;    // pinned host copy of lambda_prev and lambda (2k)
    mutable std::string err;  // last failure (also set by the read-only queries)
    rocblas_handle blas = nullptr;
    long iters = 0;
    // learned smoother (3D): weights [2][16][27], Adam state, operand words
    // of the inference kernel, fallback bookkeeping
    bool learned = false;       // smoother is PASM_LEARNED
    bool learned_on = false;    // currently smoothing with the learned step
    std::vector<float> lw;
    std::vector<double> lm, lv2;
    int ltrain_steps = 0;
    double lloss_first = 0.0, lloss_last = 0.0, lplain_rate = 0.0, llearned_rate = 0.0;
    double lplain_ms = 0.0, llearned_ms = 0.0;
    // borders formed by the last V-cycle's fine post-smoothing (2D, FP64)
    bool border_next = false, border_done = false;
    // FP64 cycles in a row: the finest post-smoothing of a cycle followed by a
    // further cycle runs together with that cycle's pre-smoothing, which then
    // finds its work done (x pre-smoothed, the coarse right-hand side formed)
    bool pair_next = false, fine_pre_done = false;
    // steps in a row (FP64 2D): a step's prolongation u = P Q y' + s u~ and
    // the next right-hand side are left to the next step's first finest
    // pre-smoothing, which forms both in its pass (Q y' waits in lv[0].B)
    bool prolong_pending = false;
    const double* pend_beta = nullptr;  // the weights of u~ in the pending prolongation (s, or zeros after a restart)
    int border_nblk = 0;
    // F64 holds lambda M u for the current U and lam (formed by the last
    // step's prolongation); anything else that touches U, lam or F64 clears it
    bool f_ready = false;
    // mixed 2D: the last V-cycle's FP32 correction (E32) is still to be added
    // to U; the step's border pass adds it
    bool e_pending = false;
    bool e_split = false;
    std::vector<char> lstag;  // per eigenpair: the plain V-cycle stagnated too (learned fallback test)
    long lcycles_learned = 0, lcycles_fallback = 0;
    double lthreshold = 0.0;    // > 0: fallback threshold set by the caller
    std::vector<double> lratio; // residual reduction of the last V-cycles (diagnostics)
    unsigned long long* lops = nullptr;
    float* lpool = nullptr;     // training residuals [lpool_n][m^3]
    int lpool_n = 0, ltrain_level = -1;
    pasm::LearnedTrainer ltrainer;
    double* Xb = nullptr;       // finest-level backup of x for a rejected V-cycle
    double* rnpart = nullptr;   // residual-norm partials and per-rhs sums
    double* rnsum = nullptr;
    // graph replay of correction steps (pasm_use_graph): one captured graph
    // per host state a step starts from, and the states stepped once eagerly
    bool use_graph = false;
    long graph_replays = 0;
    std::vector<pasm::StepGraph> graphs;
    bool stepped = false;
    // profiling of the fine-level smoothing sweeps
    bool prof = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    std::vector<double> ev_bytes;
    long prof_launches = 0;
    double prof_ms = 0.0, prof_bytes = 0.0;

    template <typename T>
    T* alloc(size_t count) {
        void* p = nullptr;
        if (count == 0) count = 1;
        if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) throw Error(PASM_E_NOMEM, "hipMalloc failed");
        allocs.push_back(p);
        PASM_HIP(hipMemsetAsync(p, 0, count * sizeof(T), st));
        return static_cast<T*>(p);
    }
    const Grid& gf() const { return lv.back().g; }
    long sf() const { return gf().plane; }

    template <typename T>
    Coef<T> coef(int l) const;
};

template <>
Coef<double> pasm_ctx::coef<double>(int l) const {
    Coef<double> c;
    const auto& L = lv[l];
    if (L.general3) {
        c.s15 = L.s64;
        c.w0 = L.w0;
        return c;
    }
    if (!L.const_coef) {
        c.wx = L.w64[0];
        c.wy = L.w64[1];
        c.wz = L.w64[2];
        if (L.general) {
            c.d = L.w64[3];
            c.wne = L.w64[4];
        }
    }
    c.w0 = L.w0;
    return c;
}
template <>
Coef<float> pasm_ctx::coef<float>(int l) const {
    Coef<float> c;
    const auto& L = lv[l];
    if (L.general3) {
        c.s15 = L.s32;
        c.w0 = (float)L.w0;
        return c;
    }
    if (!L.const_coef) {
        c.wx = L.w32[0];
        c.wy = L.w32[1];
        c.wz = L.w32[2];
        if (L.general) {
            c.d = L.w32[3];
            c.wne = L.w32[4];
        }
    }
    c.w0 = (float)L.w0;
    return c;
}

namespace pasm {
namespace {


}  // namespace
}  // namespace pasm

// ---------------------------------------------------------------------------
// V-cycle (templated on the cycle's floating type)
// ---------------------------------------------------------------------------
namespace {

void record_start(pasm_ctx* c) {
    if (!c->prof) return;
    if (c->ev_used + 2 > c->ev.size()) {
        hipEvent_t a, b;
        // timing only: no system-scope fence (it would write back and
        // invalidate the caches around every timed launch)
        PASM_HIP(hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
        PASM_HIP(hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
        c->ev.push_back(a);
        c->ev.push_back(b);
        c->ev_bytes.push_back(0.0);
    }
    PASM_HIP(hipEventRecord(c->ev[c->ev_used], c->st));
}
void record_end(pasm_ctx* c, double bytes) {
    if (!c->prof) return;
    PASM_HIP(hipEventRecord(c->ev[c->ev_used + 1], c->st));
    c->ev_bytes[c->ev_used / 2] = bytes;
    c->ev_used += 2;
}
// Recorded launches are summed when the profile is read, or after a
// synchronisation once this many events are held (every recorded event has
// completed then), so that the timing reads stay off the path between steps.
constexpr size_t kProfileBatch = 512;
void collect_profile(pasm_ctx* c) {
    if (!c->prof) return;
    for (size_t e = 0; e < c->ev_used; e += 2) {
        float ms = 0.f;
        PASM_HIP(hipEventElapsedTime(&ms, c->ev[e], c->ev[e + 1]));
        c->prof_ms += ms;
        c->prof_bytes += c->ev_bytes[e / 2];
        c->prof_launches += 1;
    }
    c->ev_used = 0;
}

// Apply the smoothing steps of `steps` at level l: x (current) and y
// (scratch) are swapped after every step so x always holds the iterate.
template <typename T>
void smooth(pasm_ctx* c, int l, T*& x, T*& y, const T* f, const std::vector<Cheb>& steps, bool x_zero,
            int nrhs) {
    if (c->learned_on && l >= 1) {
        // one learned step per phase (3D constant-coefficient levels)
        const pasm::Level& L = c->lv[l];
        const bool fine = (l == c->L - 1);
        const double nodes = (double)L.g.interior() * nrhs;
        if (fine) record_start(c);
        pasm::launch_learned_step<T>(L.g, (T)L.w0, x, f, y, nrhs, L.g.plane, c->lops, x_zero, c->st);
        if (fine) record_end(c, (x_zero ? 2.0 : 3.0) * sizeof(T) * nodes);
        std::swap(x, y);
        return;
    }
    if (steps.empty()) return;
    const pasm::Level& L = c->lv[l];
    const Coef<T> cf = c->coef<T>(l);
    const bool fine = (l == c->L - 1);
    if (c->opt.smoother == PASM_CG) {
        // x updated in place (no swap); algorithmic bytes of the kernels:
        // start 3 words (2 from x = 0), first direction 3, later ones 4,
        // updates 6 (the last of a phase 3: x only)
        const int S = (int)steps.size();
        const double words = (x_zero ? 2.0 : 3.0) + 3.0 + 4.0 * (S - 1) + 6.0 * (S - 1) + 3.0;
        if (fine) record_start(c);
        pasm::cg_smooth<T>(L.g, cf, x, f, nrhs, S, x_zero, L.cg, c->st);
        if (fine) record_end(c, words * sizeof(T) * (double)L.g.interior() * nrhs);
        return;
    }
    const double nodes = (double)L.g.interior();
    const double coef_bytes =
        L.const_coef ? 0.0 : (double)(L.general3 ? 8 : (L.general ? 4 : L.g.dim)) * sizeof(T) * nodes;
    // tallest fused tile whose LDS fits (general stencils need four coefficient tiles)
    int rows = 0;
    for (int r : {8, 4}) {
        if (pasm::fused_lds_bytes(pasm::coef_kind(cf), sizeof(T), r) <= 65536 && 4 * r > 2 * (int)steps.size()) {
            rows = r;
            break;
        }
    }
    if (c->fuse && rows > 0 && pasm::fused_supported(L.g, (int)steps.size())) {
        pasm::SmoothSteps ss{};
        ss.s = (int)steps.size();
        for (size_t j = 0; j < steps.size(); ++j) {
            ss.a[j] = steps[j].a;
            ss.b[j] = steps[j].b;
        }
        // algorithmic bytes of the fused phase: read x_0 (unless zero) and f, write x_s
        const double bytes = (x_zero ? 2.0 : 3.0) * sizeof(T) * nodes * nrhs + coef_bytes;
        if (fine) record_start(c);
        const bool ok = pasm::launch_smooth_fused<T>(L.g, cf, x, f, y, nrhs, L.g.plane, ss, x_zero, c->st, rows);
        if (!ok) throw Error(PASM_E_INVALID, "fused smoothing shape not supported");
        if (fine) record_end(c, bytes);
        std::swap(x, y);
        return;
    }
    for (size_t j = 0; j < steps.size(); ++j) {
        // starting from x = 0: step 0 does not read x_0, step 1 does not read x_{-1} = x_0
        const bool z = x_zero && j == 0;
        const int zmode = (z ? 1 : 0) | ((x_zero && j == 1) ? 2 : 0);
        if (fine) {
            // algorithmic bytes: read x_k (unless zero), x_{k-1} (if a != 0), f; write x_{k+1};
            // plus the coefficient arrays once per launch
            const double words = 2.0 + (z ? 0.0 : 1.0) + (steps[j].a != 0.0 && !z && !(zmode & 2) ? 1.0 : 0.0);
            const double bytes = words * sizeof(T) * nodes * nrhs + coef_bytes;
            record_start(c);
            pasm::launch_smooth<T>(L.g, cf, x, y, f, y, nrhs, L.g.plane, steps[j], zmode, c->st);
            record_end(c, bytes);
        } else {
            pasm::launch_smooth<T>(L.g, cf, x, y, f, y, nrhs, L.g.plane, steps[j], zmode, c->st);
        }
        std::swap(x, y);
    }
}

template <typename T>
const T* ainv(const pasm_ctx* c);
template <>
const double* ainv<double>(const pasm_ctx* c) { return c->Ainv64; }
template <>
const float* ainv<float>(const pasm_ctx* c) { return c->Ainv32; }

pasm::SmoothSteps to_steps(const std::vector<Cheb>& v) {
    pasm::SmoothSteps ss{};
    ss.s = (int)v.size();
    for (size_t j = 0; j < v.size() && j < 8; ++j) {
        ss.a[j] = v[j].a;
        ss.b[j] = v[j].b;
    }
    return ss;
}

// Exact solve on V_H (level 0, padded fields): by the sine transform where
// the coarse operator is the constant-coefficient 2D one, else the dense
// product with A_H^{-1}.
template <typename T>
void coarse_solve(pasm_ctx* c, const T* f, T* x, int nrhs) {
    const pasm::Level& L0 = c->lv[0];
    if (c->dstS)
        pasm::launch_dst_solve<T>(L0.g, c->dstS, c->dstInv, f, L0.g.plane, x, L0.g.plane, nrhs, c->st);
    else
        pasm::launch_dense_mv<T>(ainv<T>(c), c->NH, L0.g, f, L0.g.plane, true, x, L0.g.plane, true, nrhs, c->dmv,
                                 c->st);
}

// One V-cycle at level l >= 0 on (x, f); x may start at zero.
template <typename T>
void vcycle(pasm_ctx* c, int l, T*& x, T*& y, const T* f, bool x_zero, int nrhs) {
    const pasm::Level& L = c->lv[l];
    if (l == 0) {
        coarse_solve<T>(c, f, x, nrhs);
        return;
    }
    pasm::Level& Lc = c->lv[l - 1];
    T* fc = static_cast<T*>(Lc.F);
    T* xc = static_cast<T*>(Lc.X);
    T* yc = static_cast<T*>(Lc.Y);
    const bool fine = (l == c->L - 1);
    if (c->fuse && pasm::march_supported(L.g, L.const_coef, (int)L.pre.size()) &&
        pasm::march_supported(L.g, L.const_coef, (int)L.post.size())) {
        // marching phases: pre-smoothing with the residual restriction fused,
        // post-smoothing with the prolongation fused
        const double nodes = (double)L.g.interior() * nrhs, w = sizeof(T);
        const bool pre_done = fine && c->fine_pre_done;
        if (fine) c->fine_pre_done = false;
        if (!pre_done) {
            if (fine) record_start(c);
            bool prolonged = false;
            if constexpr (std::is_same<T, double>::value) {
                if (fine && c->prolong_pending) {
                    // x holds u~; x_0 = P Q y' + s u~ and f = lambda M x_0 come
                    // from the pass (f into F64, which f points to), then PRE
                    if (f != c->F64) throw Error(PASM_E_DEVICE, "prolonging pre-smoothing: unexpected right-hand side");
                    pasm::launch_march_pre_prolong(L.g, L.w0, x, c->F64, y, Lc.g, fc, c->lv[0].g, c->lv[0].B,
                                                   c->pend_beta, c->lam, nrhs, to_steps(L.pre), c->st);
                    c->prolong_pending = false;
                    prolonged = true;
                }
            }
            if (!prolonged)
                pasm::launch_march_pre<T>(L.g, (T)L.w0, x, f, y, Lc.g, fc, nrhs, to_steps(L.pre), x_zero, c->st);
            // u~ (or x_0), f, y and the coarse right-hand side
            if (fine) record_end(c, ((x_zero ? 2.0 : 3.0) + 0.25) * w * nodes);
            std::swap(x, y);
        }
        vcycle<T>(c, l - 1, xc, yc, fc, true, nrhs);
        if (fine) record_start(c);
        bool fused_border = false;
        if constexpr (std::is_same<T, double>::value) {
            if (fine && c->pair_next &&
                pasm::march_pair_supported(L.g, L.const_coef, (int)L.post.size(), (int)L.pre.size())) {
                // this cycle's post-smoothing and the next cycle's pre-smoothing
                // in one pass: x, f, y, the coarse correction and the coarse
                // right-hand side
                pasm::launch_march_post_pre(L.g, L.w0, x, f, y, Lc.g, xc, fc, nrhs, to_steps(L.post),
                                            to_steps(L.pre), c->st);
                record_end(c, 3.5 * w * nodes);
                std::swap(x, y);
                c->fine_pre_done = true;
                return;
            }
            if (fine && c->border_next && c->dim == 2) {
                // the borders of the next step come from this post-smoothing's output
                c->border_nblk = pasm::launch_march_post_border(L.g, L.w0, x, f, y, Lc.g, xc, Lc.B, Lc.C, c->partial,
                                                                nrhs, to_steps(L.post), c->st);
                c->border_done = fused_border = true;
            }
        }
        if (!fused_border) pasm::launch_march_post<T>(L.g, (T)L.w0, x, f, y, Lc.g, xc, nrhs, to_steps(L.post), c->st);
        // x, f, y and the coarse correction; with the borders also b_c, c_c
        if (fine) record_end(c, (fused_border ? 3.75 : 3.25) * w * nodes);
        std::swap(x, y);
        return;
    }
    if constexpr (std::is_same<T, float>::value) {
        // edge-weight levels (per-element kappa) in FP32: the same marching
        // phases with the weights streamed beside x and f
        const Coef<float> cw = c->coef<float>(l);
        if (c->fuse && !L.const_coef && Lc.g.n * 2 == L.g.n && pasm::march_coef_supported(L.g, cw, (int)L.pre.size()) &&
            pasm::march_coef_supported(L.g, cw, (int)L.post.size())) {
            const double nodes = (double)L.g.interior() * nrhs, w = sizeof(T);
            // the weight planes (two, or four with the diagonal and the
            // diagonal couplings), counted once per launch (every right-hand
            // side reads them; after the first they come from the caches)
            const double cbytes = (L.general ? 4.0 : 2.0) * w * (double)L.g.interior();
            if (fine) record_start(c);
            pasm::launch_march_pre_ew(L.g, cw, x, f, y, Lc.g, fc, nrhs, to_steps(L.pre), x_zero, c->st);
            if (fine) record_end(c, ((x_zero ? 2.0 : 3.0) + 0.25) * w * nodes + cbytes);
            std::swap(x, y);
            vcycle<T>(c, l - 1, xc, yc, fc, true, nrhs);
            if (fine) record_start(c);
            pasm::launch_march_post_ew(L.g, cw, x, f, y, Lc.g, xc, nrhs, to_steps(L.post), c->st);
            if (fine) record_end(c, 3.25 * w * nodes + cbytes);
            std::swap(x, y);
            return;
        }
    }
    if (c->fuse && !c->learned_on && pasm::march3_supported(L.g, L.const_coef, (int)L.pre.size()) &&
        pasm::march3_supported(L.g, L.const_coef, (int)L.post.size())) {
        // 3D marching phases: all steps of a phase in one pass, the
        // prolongation fused into post-smoothing
        const double nodes = (double)L.g.interior() * nrhs, w = sizeof(T);
        if (fine) record_start(c);
        pasm::launch_march3_smooth<T>(L.g, (T)L.w0, x, f, y, nrhs, to_steps(L.pre), x_zero, c->st);
        if (fine) record_end(c, (x_zero ? 2.0 : 3.0) * w * nodes);
        std::swap(x, y);
        pasm::launch_resid_restrict<T>(L.g, c->coef<T>(l), x, f, Lc.g, fc, nrhs, L.g.plane, Lc.g.plane, c->st);
        vcycle<T>(c, l - 1, xc, yc, fc, true, nrhs);
        if (fine) record_start(c);
        pasm::launch_march3_post<T>(L.g, (T)L.w0, x, f, y, Lc.g, xc, nrhs, to_steps(L.post), c->st);
        if (fine) record_end(c, 3.125 * w * nodes);
        std::swap(x, y);
        return;
    }
    smooth<T>(c, l, x, y, f, L.pre, x_zero, nrhs);
    const bool zero_after_pre = x_zero && L.pre.empty();
    if (zero_after_pre) {
        // x = 0: the residual is f, restricted
        pasm::launch_restrict<T>(L.g, f, Lc.g, fc, nrhs, L.g.plane, Lc.g.plane, c->st);
    } else if (L.general3) {
        // 15-point operator: the residual into the free buffer y, then restricted
        pasm::launch_resid3g<T>(L.g, c->coef<T>(l).s15, x, f, y, nrhs, L.g.plane, c->st);
        pasm::launch_restrict<T>(L.g, y, Lc.g, fc, nrhs, L.g.plane, Lc.g.plane, c->st);
    } else {
        pasm::launch_resid_restrict<T>(L.g, c->coef<T>(l), x, f, Lc.g, fc, nrhs, L.g.plane, Lc.g.plane, c->st);
    }
    vcycle<T>(c, l - 1, xc, yc, fc, true, nrhs);
    if (zero_after_pre) {
        pasm::launch_prolong<T>(Lc.g, xc, L.g, x, nrhs, Lc.g.plane, L.g.plane, false, nullptr, c->st);
    } else {
        pasm::launch_prolong<T>(Lc.g, xc, L.g, x, nrhs, Lc.g.plane, L.g.plane, true, nullptr, c->st);
    }
    smooth<T>(c, l, x, y, f, L.post, false, nrhs);
}

// ncycles V-cycles for A x = f at the finest level; x, f are FP64 finest-level
// buffers (padded), scr an FP64 scratch buffer of the same size.
// One V-cycle for A x = f at the finest level: in place (FP64), or as
// defect correction with an FP32 cycle (mixed).
//
// Mixed: r_ready says that R32 already holds f - A x (formed by the previous
// cycle's last pass); with next set, this cycle's correction and the
// next cycle's residual are formed in one pass, x moving to scr.
// keep_sum: the next cycle is the step's last, its correction added by the
// border pass, so x + e is not stored: x stays, e stays in E32 and the next
// correction goes to E2_32 (e_split).
void one_cycle(pasm_ctx* c, double*& x, double*& scr, const double* f, int nrhs, bool* r_ready = nullptr,
               bool next = false, bool defer_add = false, const double* lam_mass = nullptr, bool keep_sum = false) {
    const int lf = c->L - 1;
    if (!c->mixed) {
        c->pair_next = next;
        vcycle<double>(c, lf, x, scr, f, false, nrhs);
        c->pair_next = false;
        return;
    }
    const Grid& g = c->gf();
    if (!(r_ready && *r_ready))
        pasm::launch_resid_cast(g, c->coef<double>(lf), x, f, c->R32, nrhs, g.plane, c->st, lam_mass);
    if (r_ready) *r_ready = false;
    float* e = c->e_split ? c->E2_32 : c->E32;
    float* ye = c->Y32;
    vcycle<float>(c, lf, e, ye, c->R32, true, nrhs);
    if (next && r_ready && keep_sum && !c->e_split) {
        pasm::launch_resid_of_sum(g, c->coef<double>(lf), x, e, f, c->R32, nrhs, g.plane, c->st, lam_mass);
        c->e_split = true;
        *r_ready = true;
        return;
    }
    if (next && r_ready && pasm::add_resid_supported(g, c->coef<double>(lf))) {
        pasm::launch_add_resid(g, c->coef<double>(lf), x, e, f, scr, c->R32, nrhs, g.plane, c->st, lam_mass);
        std::swap(x, scr);
        *r_ready = true;
        return;
    }
    if (defer_add) {
        // the last cycle of a step: x + e is formed by the border pass
        c->e_pending = true;
        return;
    }
    if (c->e_split) {
        // x + e0 first, as the stored sum would have been
        pasm::launch_add_correction(c->E32, x, g.plane * nrhs, c->st);
        c->e_split = false;
    }
    pasm::launch_add_correction(e, x, g.plane * nrhs, c->st);
}

// ||f - A x||^2 per right-hand side (finest level, FP64, 3D), to the host;
// ||f||^2 per right-hand side into *fn if given
std::vector<double> resid_norms(pasm_ctx* c, const double* x, const double* f, int nrhs,
                                std::vector<double>* fn = nullptr) {
    const Grid& g = c->gf();
    const int nb = pasm::launch_resid_norm3<double>(g, c->lv.back().w0, x, f, c->rnpart, nrhs, g.plane, c->st);
    pasm::launch_reduce_pairs(c->rnpart, nb, c->rnsum, nrhs, c->st);
    std::vector<double> out(2 * (size_t)nrhs);
    PASM_HIP(hipMemcpyAsync(out.data(), c->rnsum, out.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
    PASM_HIP(hipStreamSynchronize(c->st));
    std::vector<double> n(nrhs);
    for (int r = 0; r < nrhs; ++r) n[r] = out[2 * r];
    if (fn) {
        fn->resize(nrhs);
        for (int r = 0; r < nrhs; ++r) (*fn)[r] = out[2 * r + 1];
    }
    return n;
}

// ncycles V-cycles for A x = f at the finest level; x, f are FP64 finest-level
// buffers (padded), scr an FP64 scratch buffer of the same size.  With the
// learned smoother every cycle is checked: if it reduced the residual of some
// right-hand side by less than the plain cycle does (the rate measured at
// set-up), x is restored and the cycle is redone with the plain smoother.
void bvp_cycles(pasm_ctx* c, double*& x, double*& scr, const double* f, int nrhs, int ncycles,
                bool border = false, bool eig = false) {
    if (!c->learned_on) {
        // the first residual of a correction step may come from the
        // prolongation that formed u; any other call forms its own
        bool r_ready = eig && c->r32_ready;
        c->r32_ready = false;
        c->fine_pre_done = false;
        for (int cy = 0; cy < ncycles; ++cy) {
            // the last FP64 cycle may form the borders of the next step on its way out
            c->border_next = border && cy == ncycles - 1 && !c->mixed;
            const int kind = pasm::coef_kind(c->coef<double>(c->L - 1));
            const bool defer = cy == ncycles - 1 && c->mixed && eig &&
                               ((border && c->dim == 2 && kind <= 1) || c->lv[c->L - 1].general3 ||
                                (c->dim == 3 && kind == 0));
            // f = lam M u formed by the residual passes (the first two cycles
            // of a step start from u itself or from u + e with u still in x)
            const double* lam_mass = (eig && c->f_mass && cy < 2) ? c->lam : nullptr;
            // the next cycle deferred to a row-marching border pass: u + e not stored
            const bool keep = cy + 2 == ncycles && c->mixed && eig && border && c->E2_32 &&
                              pasm::rows_supported(c->gf(), c->coef<double>(c->L - 1));
            one_cycle(c, x, scr, f, nrhs, &r_ready, cy + 1 < ncycles, defer, lam_mass, keep);
            c->border_next = false;
        }
        if (c->fine_pre_done) throw Error(PASM_E_DEVICE, "paired smoothing phases: a cycle left unfinished");
        return;
    }
    const Grid& g = c->gf();
    const size_t bytes = (size_t)g.plane * nrhs * sizeof(double);
    std::vector<double> nf;
    std::vector<double> n0 = resid_norms(c, x, f, nrhs, &nf);
    const double thr = c->lthreshold > 0.0 ? c->lthreshold : c->lplain_rate;
    const double lim = thr * thr;
    // a residual already at the cycle's rounding level (relative to f) can
    // not shrink further under any smoother: such right-hand sides do not
    // count against the learned cycle
    // (residuals are formed in FP64 in both precisions: defect correction)
    const double floor2 = (64.0 * DBL_EPSILON) * (64.0 * DBL_EPSILON);
    for (int cy = 0; cy < ncycles; ++cy) {
        PASM_HIP(hipMemcpyAsync(c->Xb, x, bytes, hipMemcpyDeviceToDevice, c->st));
        one_cycle(c, x, scr, f, nrhs);
        std::vector<double> n1 = resid_norms(c, x, f, nrhs);
        // right-hand sides of the eigen-iteration that the plain cycle could
        // not reduce either (stagnant: at a floor of the arithmetic) only
        // must not grow
        const bool track = eig && (int)c->lstag.size() == nrhs;
        bool worse = false;
        for (int r = 0; r < nrhs; ++r) {
            const bool at_floor = n1[r] <= floor2 * nf[r];
            if (track && c->lstag[r]) worse |= !(n1[r] <= 1.21 * n0[r]);
            else worse |= !(n1[r] <= lim * n0[r]) && n0[r] > 0.0 && !at_floor;
            if (n0[r] > 0.0) c->lratio.push_back(std::sqrt(n1[r] / n0[r]));
        }
        if (c->lratio.size() > 4096) c->lratio.erase(c->lratio.begin(), c->lratio.end() - 4096);
        if (worse) {
            PASM_HIP(hipMemcpyAsync(x, c->Xb, bytes, hipMemcpyDeviceToDevice, c->st));
            c->learned_on = false;
            one_cycle(c, x, scr, f, nrhs);
            c->learned_on = true;
            n1 = resid_norms(c, x, f, nrhs);
            ++c->lcycles_fallback;
            if (track)
                for (int r = 0; r < nrhs; ++r)
                    if (!(n1[r] <= lim * n0[r]) && !(n1[r] <= floor2 * nf[r])) c->lstag[r] = 1;
        } else {
            ++c->lcycles_learned;
        }
        n0 = n1;
    }
}

thread_local std::string g_setup_error;

void set_error(const pasm_ctx* c, const std::string& m) {
    if (c) c->err = m;
}

}  // namespace

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
namespace {

struct Plan {
    int dim, nH, nh, L, NH;
    bool have_kappa, have_pot, have_tensor;
    size_t nel;
};

// Argument checks only (no device calls), so invalid input is reported the
// same way with or without a GPU.
Plan validate(const pasm_options& opt, const pasm_domain* dom, const pasm_coefficients* coef, double H, double h,
              int k) {
    Plan p{};
    if (!dom || (dom->dim != 2 && dom->dim != 3)) throw Error(PASM_E_INVALID, "domain dim must be 2 or 3");
    p.dim = dom->dim;
    if (!(H > 0.0) || !(h > 0.0) || !std::isfinite(H) || !std::isfinite(h) || h > H)
        throw Error(PASM_E_INVALID, "need 0 < h <= H");
    const double nHd = 1.0 / H, nhd = 1.0 / h;
    if (nHd > 1e6 || nhd > 1e6) throw Error(PASM_E_INVALID, "mesh too fine");
    p.nH = (int)std::lround(nHd);
    p.nh = (int)std::lround(nhd);
    if (std::fabs(nHd - p.nH) > 1e-9 * nHd || std::fabs(nhd - p.nh) > 1e-9 * nhd || p.nH < 2)
        throw Error(PASM_E_INVALID, "1/H and 1/h must be integers, 1/H >= 2");
    if (p.nh % p.nH != 0) throw Error(PASM_E_INVALID, "1/h must be a multiple of 1/H");
    int ratio = p.nh / p.nH;
    p.L = 1;
    while (ratio > 1) {
        if (ratio & 1) throw Error(PASM_E_INVALID, "H/h must be a power of two");
        ratio >>= 1;
        ++p.L;
    }
    long NH = 1;
    for (int a = 0; a < p.dim; ++a) NH *= (p.nH - 1);
    if (NH > 20000) throw Error(PASM_E_INVALID, "coarse space too large for the dense coarse eigensolve");
    p.NH = (int)NH;
    if (k < 1 || k >= NH) throw Error(PASM_E_INVALID, "need 1 <= k < N_H (dimension of V_H)");
    if (opt.vcycles < 1 || opt.nu_pre < 0 || opt.nu_post < 0 || opt.max_iter < 1 || !(opt.tol >= 0.0))
        throw Error(PASM_E_INVALID, "bad cycle options");
    if (opt.precision != PASM_FP64 && opt.precision != PASM_MIXED) throw Error(PASM_E_INVALID, "bad precision");
    if (opt.smoother != PASM_JACOBI && opt.smoother != PASM_CHEBYSHEV && opt.smoother != PASM_LEARNED &&
        opt.smoother != PASM_CG)
        throw Error(PASM_E_INVALID, "bad smoother");
    if (opt.smoother == PASM_LEARNED && (p.dim != 3 || (coef && (coef->kappa || coef->potential))))
        throw Error(PASM_E_INVALID, "the learned smoother is for 3D problems with constant coefficients");
    p.have_kappa = coef && coef->kappa;
    p.have_pot = coef && coef->potential;
    p.have_tensor = coef && coef->tensor;
    if (p.have_tensor && (p.dim != 3 || opt.smoother == PASM_LEARNED))
        throw Error(PASM_E_INVALID, "the diffusion tensor is supported in 3D (not with the learned smoother)");
    p.nel = 1;
    for (int a = 0; a < p.dim; ++a) p.nel *= (size_t)p.nh;
    p.nel *= (p.dim == 2 ? 2 : 6);
    if (p.have_kappa || p.have_pot || p.have_tensor) {
        if (coef->n_elements != p.nel) throw Error(PASM_E_INVALID, "n_elements does not match the fine mesh");
    }
    if (p.have_tensor)
        for (size_t e = 0; e < p.nel; ++e) {
            const double* t = coef->tensor + 6 * e;
            bool fin = true;
            for (int q = 0; q < 6; ++q) fin = fin && std::isfinite(t[q]);
            // symmetric positive definite: the leading minors
            const double m1 = t[0], m2 = t[0] * t[1] - t[3] * t[3];
            const double m3 = t[0] * (t[1] * t[2] - t[5] * t[5]) - t[3] * (t[3] * t[2] - t[5] * t[4]) +
                              t[4] * (t[3] * t[5] - t[1] * t[4]);
            if (!fin || !(m1 > 0.0) || !(m2 > 0.0) || !(m3 > 0.0))
                throw Error(PASM_E_INVALID, "the diffusion tensor must be finite, symmetric positive definite");
        }
    if (p.have_kappa)
        for (size_t e = 0; e < p.nel; ++e)
            if (!(coef->kappa[e] > 0.0) || !std::isfinite(coef->kappa[e]))
                throw Error(PASM_E_INVALID, "kappa must be finite and positive");
    if (p.have_pot)
        for (size_t e = 0; e < p.nel; ++e)
            if (!(coef->potential[e] >= 0.0) || !std::isfinite(coef->potential[e]))
                throw Error(PASM_E_INVALID, "potential must be finite and non-negative");
    return p;
}

// share: another context of the same problem whose coarse space (theta, Q,
// A_H^{-1}, groups, start values) is reused instead of factorising again.
void build(pasm_ctx* c, const Plan& pl, const pasm_coefficients* coef, int k, const pasm_ctx* share = nullptr) {
    const int dim = pl.dim, nH = pl.nH, L = pl.L;
    const bool have_kappa = pl.have_kappa;
    const size_t nel = pl.nel;
    c->dim = dim;
    c->k = k;
    c->L = L;
    c->NH = pl.NH;
    c->mixed = (c->opt.precision == PASM_MIXED);
    // CG smoothing has no fused (temporally blocked) form: every step needs
    // the whole level's inner products
    c->fuse = c->opt.fused_smoothing != 0 && c->opt.smoother != PASM_CG;
    const double omega = c->opt.omega > 0 ? c->opt.omega : (dim == 2 ? 0.8 : 6.0 / 7.0);
    const double alpha = c->opt.cheb_alpha > 0 ? c->opt.cheb_alpha : (dim == 2 ? 4.0 : 6.0);

    // levels, coarse (0) to fine (L-1)
    c->lv.resize(L);
    std::vector<double> kap, pot;
    if (have_kappa) kap.assign(coef->kappa, coef->kappa + nel);
    const bool general = pl.have_pot;
    if (general) pot.assign(coef->potential, coef->potential + nel);
    pasm::Stencil7 sten;   // general stencil of the level being built (host)
    // 3D with any coefficient: the general 15-point operator on every level
    const bool general3 = dim == 3 && (have_kappa || pl.have_pot || pl.have_tensor);
    pasm::Stencil15 sten3;
    std::vector<double> ten;
    if (general3 && pl.have_tensor) ten.assign(coef->tensor, coef->tensor + 6 * nel);
    auto upload = [&](pasm::Level& Lv, int a, const std::vector<double>& w) {
        Lv.w64[a] = c->alloc<double>(Lv.g.plane);
        PASM_HIP(hipMemcpyAsync(Lv.w64[a], w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
        PASM_HIP(hipStreamSynchronize(c->st));
        if (c->mixed) {
            Lv.w32[a] = c->alloc<float>(Lv.g.plane);
            pasm::launch_d2f(Lv.w64[a], Lv.w32[a], Lv.g.plane, c->st);
            PASM_CHECK_LAUNCH();
        }
    };
    for (int l = L - 1; l >= 0; --l) {
        pasm::Level& Lv = c->lv[l];
        const int n = nH << l;
        Lv.g = pasm::make_grid(dim, n);
        Lv.const_coef = !have_kappa && !general && !general3;
        Lv.general = general && !general3;
        Lv.general3 = general3;
        Lv.w0 = (dim == 2) ? 1.0 : Lv.g.h;
        if (general3) {
            // finest level assembled element by element, coarser ones Galerkin
            sten3 = (l == L - 1) ? pasm::fine_stencil_3d(Lv.g, ten, kap, pot)
                                 : pasm::galerkin_stencil_3d(c->lv[l + 1].g, sten3, Lv.g);
            Lv.rho = pasm::gershgorin_3d(Lv.g, sten3);
            const size_t P = Lv.g.plane;
            Lv.s64 = c->alloc<double>(8 * P);
            for (int a = 0; a < 8; ++a)
                PASM_HIP(hipMemcpyAsync(Lv.s64 + a * P, sten3.a[a].data(), P * sizeof(double), hipMemcpyHostToDevice,
                                        c->st));
            PASM_HIP(hipStreamSynchronize(c->st));
            if (c->mixed) {
                Lv.s32 = c->alloc<float>(8 * P);
                pasm::launch_d2f(Lv.s64, Lv.s32, (long)(8 * P), c->st);
                PASM_CHECK_LAUNCH();
            }
            if (l == 0) {
                std::vector<double> A3;
                pasm::dense_from_stencil_3d(Lv.g, sten3, A3);
                c->AH3.swap(A3);
            }
        } else if (general) {
            // finest level assembled with the potential, coarser ones Galerkin
            sten = (l == L - 1) ? pasm::fine_stencil_2d(Lv.g, kap, pot)
                                : pasm::galerkin_stencil_2d(c->lv[l + 1].g, sten, Lv.g);
            Lv.rho = pasm::gershgorin_2d(Lv.g, sten);
            upload(Lv, 0, sten.wx);
            upload(Lv, 1, sten.wy);
            upload(Lv, 3, sten.d);
            upload(Lv, 4, sten.wne);
        } else if (have_kappa) {
            std::vector<double> wx, wy;
            pasm::edge_weights_2d(Lv.g, kap, wx, wy);
            // stiffness rows sum to zero, so the Gershgorin bound of D^{-1}A is 2
            Lv.rho = 2.0;
            upload(Lv, 0, wx);
            upload(Lv, 1, wy);
            if (!share && l > 0 && l < L - 1) {
                if (c->level_kappa.size() < (size_t)L) c->level_kappa.resize(L);
                c->level_kappa[l] = kap;
            }
            if (l > 0) kap = pasm::coarsen_kappa_2d(kap, n);
        } else {
            Lv.rho = 2.0;  // constant coefficients: zero row sums, D^{-1}A Gershgorin bound 2
        }
        if (c->opt.smoother == PASM_CHEBYSHEV) {
            Lv.pre = pasm::cheb_steps(Lv.rho, alpha, c->opt.nu_pre);
            Lv.post = pasm::cheb_steps(Lv.rho, alpha, c->opt.nu_post);
        } else if (c->opt.smoother == PASM_JACOBI || c->opt.smoother == PASM_LEARNED ||
                   c->opt.smoother == PASM_CG) {
            // (CG: only the step counts are used)
            Lv.pre = pasm::jacobi_steps(omega, c->opt.nu_pre);
            Lv.post = pasm::jacobi_steps(omega, c->opt.nu_post);
        } else {
            throw Error(PASM_E_INVALID, "unknown smoother");
        }
    }

    // vectors
    for (int l = 0; l < L - 1; ++l) {
        pasm::Level& Lv = c->lv[l];
        const size_t n = (size_t)Lv.g.plane * k;
        if (c->mixed) {
            Lv.X = c->alloc<float>(n);
            Lv.F = c->alloc<float>(n);
            Lv.Y = c->alloc<float>(n);
        } else {
            Lv.X = c->alloc<double>(n);
            Lv.F = c->alloc<double>(n);
            Lv.Y = c->alloc<double>(n);
        }
        // B and C adjacent, so the two coarse products with Q^T share one pass
        Lv.B = c->alloc<double>(2 * n);
        Lv.C = Lv.B + n;
    }
    if (c->opt.smoother == PASM_CG) {
        long pmax = 1;
        for (int l = 1; l < L; ++l) pmax = std::max(pmax, pasm::cg_partials(c->lv[l].g));
        double* partial = c->alloc<double>((size_t)pmax * k);
        double* sc = c->alloc<double>(3 * (size_t)k);
        for (int l = 1; l < L; ++l) {
            pasm::Level& Lv = c->lv[l];
            const size_t n = (size_t)Lv.g.plane * k;
            void* v[4];
            for (int a = 0; a < 4; ++a)
                v[a] = c->mixed ? static_cast<void*>(c->alloc<float>(n)) : static_cast<void*>(c->alloc<double>(n));
            Lv.cg = pasm::CgWork{v[0], v[1], v[2], v[3], partial, sc, sc + k, sc + 2 * k};
        }
    }
    const size_t nf = (size_t)c->sf() * k;
    c->U = c->alloc<double>(nf);
    c->F64 = c->alloc<double>(nf);
    c->Y64 = c->alloc<double>(nf);
    c->R64 = c->alloc<double>(nf);
    c->stage = c->alloc<double>((size_t)c->gf().interior() * k);
    if (c->mixed) {
        c->E32 = c->alloc<float>(nf);
        c->R32 = c->alloc<float>(nf);
        c->Y32 = c->alloc<float>(nf);
        if (c->dim == 2) c->E2_32 = c->alloc<float>(nf);
    }
    const int N = c->NH;
    c->general_coef = general || general3;
    // (not with the learned smoother: its cycle checks read f itself)
    c->f_mass = c->mixed && c->L >= 2 && c->opt.vcycles <= 2 && c->opt.smoother != PASM_LEARNED &&
                pasm::mass_rhs_fusable(c->gf(), c->coef<double>(c->L - 1));
    if (share) {
        c->coarse_shared = true;
        c->theta = share->theta;
        c->Qcm = share->Qcm;
        c->Qrm = share->Qrm;
        c->Ainv64 = share->Ainv64;
        c->Ainv32 = share->Ainv32;
        c->dstS = share->dstS;
        c->dstInv = share->dstInv;
        c->group = share->group;
    } else {
        c->theta = c->alloc<double>(N);
        c->Qcm = c->alloc<double>((size_t)N * N);
        c->Qrm = c->alloc<double>((size_t)N * N);
        c->Ainv64 = c->alloc<double>((size_t)N * N);
        if (c->mixed) c->Ainv32 = c->alloc<float>((size_t)N * N);
        c->group = c->alloc<int>(N);
    }
    c->bz = c->alloc<double>(2 * (size_t)k);
    const Grid& gfine = c->gf();
    const long nblk = pasm::border_partial_blocks(gfine);
    c->partial = c->alloc<double>(2 * (size_t)nblk * k);
    c->pp = c->alloc<double>(2 * (size_t)N * k);
    c->qq = c->pp + (size_t)N * k;
    c->ycoef = c->alloc<double>((size_t)N * k);
    c->s = c->alloc<double>(k);
    c->mu = c->alloc<double>(k);
    c->lam = c->alloc<double>(k);
    c->lam_prev = c->alloc<double>(k);
    c->score = c->alloc<double>(k);
    c->rank = c->alloc<int>(k);
    c->flags = c->alloc<int>(k);
    c->awork = c->alloc<char>(pasm::arrow_workspace_bytes(N, k));
    c->dmv = c->alloc<char>(pasm::dense_mv_workspace_bytes(N, 2 * k));

    std::vector<double> th;
    if (share) {
        th = share->theta_h;  // the k smallest coarse Ritz values: all the start needs
    } else {
    // dense coarse pencil from the level-0 operators (Galerkin: rediscretised
    // with the coarsened coefficient, or the Galerkin general stencil)
    const pasm::Level& L0 = c->lv[0];
    const Grid& g0 = L0.g;
    std::vector<double> wx0, wy0, AHgen;
    if (L0.general) pasm::dense_from_stencil_2d(g0, sten, AHgen);
    if (!L0.const_coef && !L0.general && !L0.general3) {
        wx0.resize(g0.plane);
        wy0.resize(g0.plane);
        PASM_HIP(hipMemcpyAsync(wx0.data(), L0.w64[0], g0.plane * sizeof(double), hipMemcpyDeviceToHost, c->st));
        PASM_HIP(hipMemcpyAsync(wy0.data(), L0.w64[1], g0.plane * sizeof(double), hipMemcpyDeviceToHost, c->st));
        PASM_HIP(hipStreamSynchronize(c->st));
    }
    std::vector<double> AH((size_t)N * N, 0.0), MH((size_t)N * N, 0.0);
    const int m = g0.m;
    auto cid = [&](int i, int j, int l3) -> long {
        if (i < 1 || j < 1 || i > m || j > m) return -1;
        if (dim == 3 && (l3 < 1 || l3 > m)) return -1;
        return dim == 2 ? (long)(j - 1) * m + (i - 1) : ((long)(l3 - 1) * m + (j - 1)) * m + (i - 1);
    };
    const int nz = dim == 3 ? m : 1;
    for (int l3 = 1; l3 <= nz; ++l3)
        for (int j = 1; j <= m; ++j)
            for (int i = 1; i <= m; ++i) {
                const int zz = dim == 3 ? l3 : 0;
                const long r = cid(i, j, zz);
                if (dim == 2) {
                    if (!L0.general) {
                        const long id = g0.idx(i, j);
                        double we, ww, wn, ws;
                        if (L0.const_coef) we = ww = wn = ws = L0.w0;
                        else {
                            we = wx0[id];
                            ww = wx0[id - 1];
                            wn = wy0[id];
                            ws = wy0[id - g0.pitch];
                        }
                        AH[r * N + r] = we + ww + wn + ws;
                        const int nb[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
                        const double wv[4] = {we, ww, wn, ws};
                        for (int t = 0; t < 4; ++t) {
                            const long q = cid(i + nb[t][0], j + nb[t][1], 0);
                            if (q >= 0) AH[q * N + r] = -wv[t];
                        }
                    }
                    const double H2 = g0.h * g0.h;
                    MH[r * N + r] = 0.5 * H2;
                    const int mb[6][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}};
                    for (int t = 0; t < 6; ++t) {
                        const long q = cid(i + mb[t][0], j + mb[t][1], 0);
                        if (q >= 0) MH[q * N + r] = H2 / 12.0;
                    }
                } else {
                    const double w = L0.w0, H3 = g0.h * g0.h * g0.h;
                    AH[r * N + r] = 6.0 * w;
                    MH[r * N + r] = 0.4 * H3;
                    for (int o = 1; o < 8; ++o) {
                        const int dx = o & 1, dy = (o >> 1) & 1, dz = (o >> 2) & 1;
                        const int s = dx + dy + dz;
                        const double mv = (s == 2) ? H3 / 30.0 : H3 / 20.0;
                        for (int sg = -1; sg <= 1; sg += 2) {
                            const long q = cid(i + sg * dx, j + sg * dy, l3 + sg * dz);
                            if (q < 0) continue;
                            MH[q * N + r] = mv;
                            if (s == 1) AH[q * N + r] = -w;
                        }
                    }
                }
            }
    if (L0.general) AH.swap(AHgen);
    if (L0.general3) AH.swap(c->AH3);
    c->AH3.clear();
    c->AH3.shrink_to_fit();
    double* dA = c->Qcm;
    double* dB = c->Ainv64;  // scratch for M_H during the factorisation
    PASM_HIP(hipMemcpyAsync(dA, AH.data(), AH.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    PASM_HIP(hipMemcpyAsync(dB, MH.data(), MH.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    if (rocblas_create_handle(&c->blas) != rocblas_status_success)
        throw Error(PASM_E_DEVICE, "rocblas_create_handle failed");
    rocblas_set_stream(c->blas, c->st);
    double* dE = c->alloc<double>(N);
    int* dInfo = c->alloc<int>(1);
    if (rocsolver_dsygvd(c->blas, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper, N, dA, N, dB, N,
                         c->theta, dE, dInfo) != rocblas_status_success)
        throw Error(PASM_E_DEVICE, "rocsolver_dsygvd failed");
    int info = 0;
    PASM_HIP(hipMemcpyAsync(&info, dInfo, sizeof(int), hipMemcpyDeviceToHost, c->st));
    th.resize(N);
    PASM_HIP(hipMemcpyAsync(th.data(), c->theta, N * sizeof(double), hipMemcpyDeviceToHost, c->st));
    PASM_HIP(hipStreamSynchronize(c->st));
    if (info != 0) throw Error(PASM_E_DEVICE, "coarse generalized eigensolve did not converge");
    // Q^T (row-major Q) and A_H^{-1} = Q diag(1/theta) Q^T
    pasm::launch_transpose(c->Qcm, c->Qrm, N, c->st);
    double* QS = dB;
    pasm::launch_scale_cols(c->Qcm, c->theta, QS, N, c->st);
    double* Ainv = c->alloc<double>((size_t)N * N);
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_transpose, N, N, N, &one, QS, N, c->Qcm, N,
                      &zero, Ainv, N) != rocblas_status_success)
        throw Error(PASM_E_DEVICE, "rocblas_dgemm failed");
    c->Ainv64 = Ainv;
    if (c->mixed)
        pasm::launch_d2f(c->Ainv64, c->Ainv32, (long)N * N, c->st);
    if (dim == 2 && L0.const_coef && !L0.general && pasm::dst_solve_supported(g0)) {
        std::vector<double> S, inv;
        pasm::dst_solve_tables(g0, L0.w0, S, inv);
        c->dstS = c->alloc<double>(S.size());
        c->dstInv = c->alloc<double>(inv.size());
        PASM_HIP(hipMemcpyAsync(c->dstS, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
        PASM_HIP(hipMemcpyAsync(c->dstInv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
        PASM_HIP(hipStreamSynchronize(c->st));
    }
    // groups of equal coarse Ritz values
    std::vector<int> grp(N);
    const double gtol = 16.0 * DBL_EPSILON * std::fabs(th[N - 1]);
    for (int j = 0; j < N; ++j) grp[j] = (j > 0 && th[j] - th[j - 1] <= gtol) ? grp[j - 1] : j;
    PASM_HIP(hipMemcpyAsync(c->group, grp.data(), N * sizeof(int), hipMemcpyHostToDevice, c->st));
    }  // own coarse space

    // start: lambda_i = theta_i, u_i = P q_i
    c->lam_h.assign(th.begin(), th.begin() + k);
    c->lam_prev_h = c->lam_h;
    c->theta_h = c->lam_h;
    c->zeros = c->alloc<double>(k);
    PASM_HIP(hipHostMalloc((void**)&c->lam_pin, 2 * k * sizeof(double), hipHostMallocDefault));
    PASM_HIP(hipMemsetAsync(c->zeros, 0, k * sizeof(double), c->st));
    PASM_HIP(hipMemcpyAsync(c->lam, c->lam_h.data(), k * sizeof(double), hipMemcpyHostToDevice, c->st));
    PASM_HIP(hipMemcpyAsync(c->lam_prev, c->lam_h.data(), k * sizeof(double), hipMemcpyHostToDevice, c->st));
    pasm::launch_unit_coefs(c->ycoef, N, k, k, c->st);
    PASM_CHECK_LAUNCH();
    PASM_HIP(hipStreamSynchronize(c->st));
}

// u = P Q y' + s u  (s = nullptr: u = P Q y')
// u = P Q y' + s u~ (s == nullptr: u = P Q y'); with s given, also the next
// step's right-hand side f = lamf M u in the same pass (lamf == nullptr: the
// new eigenvalues mu).
// coarse_ready: Q y' is already in place (U when the fine level is V_H, else
// the coarse level's B).
void prolong_coefs(pasm_ctx* c, const double* s, const double* lamf = nullptr, bool coarse_ready = false) {
    const int k = c->k, N = c->NH;
    const pasm::Level& L0 = c->lv[0];
    if (c->L == 1) {
        // the fine level is V_H itself: the augmentation is always skipped (s = 0)
        if (!coarse_ready)
            pasm::launch_dense_mv<double>(c->Qcm, N, L0.g, c->ycoef, N, false, c->U, L0.g.plane, true, k, c->dmv,
                                          c->st);
        return;
    }
    if (!coarse_ready)
        pasm::launch_dense_mv<double>(c->Qcm, N, L0.g, c->ycoef, N, false, c->lv[0].B, L0.g.plane, true, k, c->dmv,
                                      c->st);
    if (s && c->dim == 2) {
        // 2D: from the coarse space straight to the finest level (P1
        // interpolation on the coarse triangles), with the next step's
        // right-hand side lambda M u from the same pass
        if (c->f_mass) {
            // and the next step's first residual lambda M u - A u, in FP32
            const pasm::Coef<double>& cf = c->coef<double>(c->L - 1);
            pasm::launch_prolong_mass(L0.g, L0.B, c->gf(), c->U, c->Y64, nullptr, k, L0.g.plane, c->sf(), s,
                                      lamf ? lamf : c->mu, c->st, cf.wx, cf.wy, c->R32);
            c->r32_ready = true;
        } else {
            pasm::launch_prolong_mass(L0.g, L0.B, c->gf(), c->U, c->Y64, c->F64, k, L0.g.plane, c->sf(), s,
                                      lamf ? lamf : c->mu, c->st);
        }
        std::swap(c->U, c->Y64);
        c->f_ready = !c->f_mass;
        return;
    }
    for (int l = 1; l < c->L - 1; ++l)
        pasm::launch_prolong<double>(c->lv[l - 1].g, c->lv[l - 1].B, c->lv[l].g, c->lv[l].B, k, c->lv[l - 1].g.plane,
                                     c->lv[l].g.plane, false, nullptr, c->st);
    const pasm::Level& Lc = c->lv[c->L - 2];
    if (s && c->f_mass && c->lv[c->L - 1].general3) {
        // no f to form (the residual passes form lambda M u): u = P q + s u~
        // node by node, in place
        pasm::launch_prolong<double>(Lc.g, Lc.B, c->gf(), c->U, k, Lc.g.plane, c->sf(), false, s, c->st);
        c->f_ready = false;
        return;
    }
    if (s && c->f_mass) {
        // no f to form (the residual passes form lambda M u): u = P q + s u~
        // into the scratch field (then swapped in), with the next step's
        // first residual lambda M u - A u in FP32 from the same pass
        pasm::launch_prolong_resid3(Lc.g, Lc.B, c->gf(), c->coef<double>(c->L - 1), c->U, c->Y64, c->R32, k,
                                    Lc.g.plane, c->sf(), s, lamf ? lamf : c->mu, c->st);
        std::swap(c->U, c->Y64);
        c->r32_ready = true;
        c->f_ready = false;
        return;
    }
    if (s) {
        // the new u into the scratch field (then swapped in), with the next
        // step's right-hand side lambda M u from the same pass
        pasm::launch_prolong_mass(Lc.g, Lc.B, c->gf(), c->U, c->Y64, c->f_mass ? nullptr : c->F64, k, Lc.g.plane,
                                  c->sf(), s, lamf ? lamf : c->mu, c->st);
        std::swap(c->U, c->Y64);
        c->f_ready = !c->f_mass;
        return;
    }
    pasm::launch_prolong<double>(Lc.g, Lc.B, c->gf(), c->U, k, Lc.g.plane, c->sf(), false, s, c->st);
}

// Whether a step's prolongation can be left to the next step's first
// pre-smoothing (FP64 2D marching finest level, at least one V-cycle).
bool prolong_deferrable(const pasm_ctx* c) {
    if (c->dim != 2 || c->mixed || c->learned_on || c->L < 2 || !c->fuse || c->opt.vcycles < 1) return false;
    const pasm::Level& L = c->lv[c->L - 1];
    return pasm::march_supported(L.g, L.const_coef, (int)L.post.size()) &&
           pasm::march_prolong_supported(L.g, L.const_coef, (int)L.pre.size(), c->lv[0].g);
}

// One correction step.  defer: another step follows at once, so the
// prolongation may be left to its first pre-smoothing.
void iterate_once(pasm_ctx* c, bool defer = false) {
    const int k = c->k, N = c->NH, lf = c->L - 1;
    const Grid& g = c->gf();
    const long sf = c->sf();
    // Algorithm 1, step 1: f = lambda M u (unless the previous step's
    // prolongation formed it), V-cycles from x = u (in place in U)
    if (!c->f_ready && !c->f_mass) pasm::launch_mass_rhs(g, c->U, c->lam, c->F64, k, sf, c->st);
    c->f_ready = false;
    c->border_done = false;
    if (c->L > 1) {
        bvp_cycles(c, c->U, c->Y64, c->F64, k, c->opt.vcycles, c->dim == 2 && c->L >= 2, true);
        if (c->prolong_pending) {
            c->prolong_pending = false;
            throw Error(PASM_E_DEVICE, "prolonging pre-smoothing: the prolongation was not consumed");
        }
    } else {
        // fine level = V_H: exact solve
        coarse_solve<double>(c, c->F64, c->U, k);
    }
    // step 2: borders, fused with the first restriction
    const double* bsrc = c->Y64;
    const double* csrc = c->R64;
    int lstart = c->L - 2;
    if (c->L >= 2 && !c->lv[lf].general3) {
        pasm::Level& Lc = c->lv[c->L - 2];
        int nblk;
        if (c->e_pending) {
            // u~ = x + e (the last correction) and the borders of u~ in one pass
            // (e_split: u~ = (x + e0) + e, e0 the cycle before's correction)
            nblk = c->dim == 2 ? pasm::launch_border_restrict_add(g, c->coef<double>(lf), c->U,
                                                                  c->e_split ? c->E2_32 : c->E32, c->Y64, Lc.g, Lc.B,
                                                                  Lc.C, c->partial, k, sf, Lc.g.plane, c->st,
                                                                  c->e_split ? c->E32 : nullptr)
                               : pasm::launch_border_restrict3(g, c->coef<double>(lf), c->U, Lc.g, Lc.B, Lc.C,
                                                               c->partial, k, sf, Lc.g.plane, c->st, c->E32, c->Y64);
            std::swap(c->U, c->Y64);
            c->e_pending = false;
            c->e_split = false;
        } else {
            nblk = c->border_done ? c->border_nblk
                   : c->dim == 2  ? pasm::launch_border_restrict(g, c->coef<double>(lf), c->U, Lc.g, Lc.B, Lc.C,
                                                                 c->partial, k, sf, Lc.g.plane, c->st)
                                  : pasm::launch_border_restrict3(g, c->coef<double>(lf), c->U, Lc.g, Lc.B, Lc.C,
                                                                  c->partial, k, sf, Lc.g.plane, c->st);
        }
        pasm::launch_reduce_pairs(c->partial, nblk, c->bz, k, c->st);
        bsrc = Lc.B;
        csrc = Lc.C;
        lstart = c->L - 3;
    } else if (c->e_pending) {
        // 15-point operator: u~ = x + e and A u~, M u~ in one pass; u~ goes to
        // the buffer of f (formed again for the next step) and is swapped in
        const int nblk = pasm::launch_border3g(g, c->coef<double>(lf).s15, c->U, c->Y64, c->R64, c->partial, k, sf,
                                               c->st, c->E32, c->F64);
        std::swap(c->U, c->F64);
        c->e_pending = false;
        pasm::launch_reduce_pairs(c->partial, nblk, c->bz, k, c->st);
    } else {
        const int nblk = pasm::launch_border(g, c->coef<double>(lf), c->U, c->Y64, c->R64, c->partial, k, sf, c->st);
        pasm::launch_reduce_pairs(c->partial, nblk, c->bz, k, c->st);
    }
    for (int l = lstart; l >= 0; --l) {
        const Grid& gfl = c->lv[l + 1].g;
        if (c->dim == 2 && l >= 2 && csrc == bsrc + (long)gfl.plane * k) {
            // three levels down in one pass (b and c together)
            pasm::launch_restrict_chain3(gfl, bsrc, c->lv[l].g, c->lv[l - 1].g, c->lv[l - 2].g, c->lv[l - 2].B, 2 * k,
                                         gfl.plane, c->lv[l - 2].g.plane, c->st);
            bsrc = c->lv[l - 2].B;
            csrc = c->lv[l - 2].C;
            l -= 2;
            continue;
        }
        if (csrc == bsrc + (long)gfl.plane * k) {  // b and c adjacent: one launch for both
            pasm::launch_restrict<double>(gfl, bsrc, c->lv[l].g, c->lv[l].B, 2 * k, gfl.plane, c->lv[l].g.plane,
                                          c->st);
        } else {
            pasm::launch_restrict<double>(gfl, bsrc, c->lv[l].g, c->lv[l].B, k, gfl.plane, c->lv[l].g.plane, c->st);
            pasm::launch_restrict<double>(gfl, csrc, c->lv[l].g, c->lv[l].C, k, gfl.plane, c->lv[l].g.plane, c->st);
        }
        bsrc = c->lv[l].B;
        csrc = c->lv[l].C;
    }
    const Grid& g0 = c->lv[0].g;
    if (csrc == bsrc + (long)g0.plane * k) {
        // p = Q^T b and q = Q^T c in one pass over Q^T (2k right-hand sides)
        pasm::launch_dense_mv<double>(c->Qrm, N, g0, bsrc, g0.plane, true, c->pp, N, false, 2 * k, c->dmv, c->st);
    } else {
        pasm::launch_dense_mv<double>(c->Qrm, N, g0, bsrc, g0.plane, true, c->pp, N, false, k, c->dmv, c->st);
        pasm::launch_dense_mv<double>(c->Qrm, N, g0, csrc, g0.plane, true, c->qq, N, false, k, c->dmv, c->st);
    }
    pasm::ArrowIn in{c->theta, c->group, c->pp, c->qq, c->bz, c->lam, N, c->opt.exhaustive_selection};
    pasm::ArrowOut out{c->ycoef, c->s, c->mu, c->rank, c->score, c->flags, static_cast<double*>(c->awork)};
    pasm::launch_arrowhead(in, out, k, c->st);
    if (defer && prolong_deferrable(c)) {
        // Q y' now; P Q y' + s u~ and f = mu M u in the next step's first pass
        pasm::launch_dense_mv<double>(c->Qcm, N, c->lv[0].g, c->ycoef, N, false, c->lv[0].B, c->lv[0].g.plane, true,
                                      k, c->dmv, c->st);
        c->prolong_pending = true;
        c->pend_beta = c->s;
        c->f_ready = true;
    } else {
        prolong_coefs(c, c->s);
    }
    // lam_prev <- lam, lam <- mu by rotating the three buffers (no copies)
    std::swap(c->lam_prev, c->lam);
    std::swap(c->lam, c->mu);
}

// Forms a prolongation left pending for the next correction step with the
// stand-alone kernel (u = P Q y' + beta u~, f = lambda M u), for every caller
// that reads u, f or the level buffers in between.
void settle_prolongation(pasm_ctx* c) {
    if (!c->prolong_pending) return;
    c->prolong_pending = false;
    const pasm::Level& L0 = c->lv[0];
    pasm::launch_prolong_mass(L0.g, L0.B, c->gf(), c->U, c->Y64, c->F64, c->k, L0.g.plane, c->sf(), c->pend_beta,
                              c->lam, c->st);
    std::swap(c->U, c->Y64);
    c->f_ready = true;
}

// Graph replay of correction steps.  A step's launches are a function of the
// state it starts from (StepState) and the deferral flag.  A step from a state
// without a graph is captured into one (which records the launches without
// running them, while the host state advances as if they had run) and then
// launched; later steps from that state replay the graph and take its
// recorded end state.  The states cycle with the rotation of the eigenvalue
// buffers (3) and of u between two buffers (2), so a run of steps needs a
// handful of graphs.  Steps that read device data on the host (the learned
// smoother's fallback test) or record profiling events always run eagerly.
constexpr size_t kMaxStepGraphs = 16;

pasm::StepState save_state(const pasm_ctx* c) {
    pasm::StepState t;
    std::memset(&t, 0, sizeof t);  // padding included: states compare bytewise
    t.U = c->U;
    t.F64 = c->F64;
    t.Y64 = c->Y64;
    t.R64 = c->R64;
    t.lam = c->lam;
    t.lam_prev = c->lam_prev;
    t.mu = c->mu;
    t.pend_beta = c->pend_beta;
    t.border_nblk = c->border_nblk;
    t.f_ready = c->f_ready;
    t.r32_ready = c->r32_ready;
    t.border_next = c->border_next;
    t.border_done = c->border_done;
    t.pair_next = c->pair_next;
    t.fine_pre_done = c->fine_pre_done;
    t.prolong_pending = c->prolong_pending;
    t.e_pending = c->e_pending;
    t.e_split = c->e_split;
    return t;
}

void load_state(pasm_ctx* c, const pasm::StepState& t) {
    c->U = t.U;
    c->F64 = t.F64;
    c->Y64 = t.Y64;
    c->R64 = t.R64;
    c->lam = t.lam;
    c->lam_prev = t.lam_prev;
    c->mu = t.mu;
    c->pend_beta = t.pend_beta;
    c->border_nblk = t.border_nblk;
    c->f_ready = t.f_ready;
    c->r32_ready = t.r32_ready;
    c->border_next = t.border_next;
    c->border_done = t.border_done;
    c->pair_next = t.pair_next;
    c->fine_pre_done = t.fine_pre_done;
    c->prolong_pending = t.prolong_pending;
    c->e_pending = t.e_pending;
    c->e_split = t.e_split;
}

void drop_graphs(pasm_ctx* c) {
    for (pasm::StepGraph& g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

void step(pasm_ctx* c, bool defer = false) {
    if (!c->use_graph || c->prof || c->learned_on) {
        iterate_once(c, defer);
        return;
    }
    const pasm::StepState pre = save_state(c);
    for (const pasm::StepGraph& g : c->graphs)
        if (g.defer == defer && g.pre.same(pre)) {
            PASM_HIP(hipGraphLaunch(g.exec, c->st));
            load_state(c, g.post);
            ++c->graph_replays;
            return;
        }
    if (!c->stepped) {
        // the first step of a context runs eagerly: the launch helpers query
        // the device (occupancy) on their first call
        c->stepped = true;
        iterate_once(c, defer);
        return;
    }
    if (c->graphs.size() >= kMaxStepGraphs) drop_graphs(c);
    pasm::StepGraph g{};
    g.pre = pre;
    g.defer = defer;
    PASM_HIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    try {
        iterate_once(c, defer);
    } catch (...) {
        // nothing ran: back to the state the step started from, and on
        // without graphs for this context
        hipGraph_t part = nullptr;
        (void)hipStreamEndCapture(c->st, &part);
        if (part) (void)hipGraphDestroy(part);
        (void)hipGetLastError();
        load_state(c, pre);
        drop_graphs(c);
        c->use_graph = false;
        iterate_once(c, defer);
        return;
    }
    PASM_HIP(hipStreamEndCapture(c->st, &g.graph));
    g.post = save_state(c);
    if (hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g.graph);
        throw Error(PASM_E_DEVICE, "hipGraphInstantiate failed for a correction step");
    }
    c->graphs.push_back(g);
    PASM_HIP(hipGraphLaunch(g.exec, c->st));
}

// ---------------------------------------------------------------------------
// learned smoother: training data, training, rates
// ---------------------------------------------------------------------------
constexpr int kLearnedBatch = 8;       // residual samples per Adam step
constexpr int kLearnedPool = 64;       // residual samples drawn from plain V-cycles
constexpr int kLearnedSetupSteps = 160;
constexpr double kLearnedLr = 2e-3;

void learned_pack(pasm_ctx* c) {
    unsigned long long ops[pasm::kLearnedStepOps];
    pasm::learned_pack_step(c->lw.data(), ops);
    PASM_HIP(hipMemcpyAsync(c->lops, ops, sizeof(ops), hipMemcpyHostToDevice, c->st));
    PASM_HIP(hipStreamSynchronize(c->st));
}

// Residuals that plain V-cycles leave: random errors x (f = 0) on the
// training level, r = -A x after 0, 1 and 2 plain cycles.
template <typename T>
void learned_pool(pasm_ctx* c) {
    const int lt = c->ltrain_level, k = c->k;
    pasm::Level& Lv = c->lv[lt];
    const Grid& g = Lv.g;
    const long vol = g.interior();
    const bool was = c->learned_on;
    c->learned_on = false;
    int have = 0;
    for (unsigned seed = 1; have < kLearnedPool; ++seed) {
        T* x = static_cast<T*>(Lv.X);
        T* y = static_cast<T*>(Lv.Y);
        T* f = static_cast<T*>(Lv.F);
        pasm::launch_fill_zero(f, (size_t)g.plane * k * sizeof(T), c->st);
        pasm::launch_fill_zero(x, (size_t)g.plane * k * sizeof(T), c->st);
        pasm::launch_fill_normal3<T>(g, x, k, g.plane, 0x5eed0000ull + seed, c->st);
        for (int round = 0; round < 3 && have < kLearnedPool; ++round) {
            const int take = std::min(k, kLearnedPool - have);
            pasm::launch_pack_negA3<T>(g, (T)Lv.w0, x, take, g.plane, c->lpool + (long)have * vol, c->st);
            have += take;
            vcycle<T>(c, lt, x, y, f, false, k);
        }
    }
    c->lpool_n = have;
    c->learned_on = was;
    PASM_HIP(hipStreamSynchronize(c->st));
}

void learned_train(pasm_ctx* c, int steps, double* hist) {
    const long vol = c->lv[c->ltrain_level].g.interior();
    std::vector<double> grad(864);
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    for (int it = 0; it < steps; ++it) {
        const int first = (c->ltrain_steps * kLearnedBatch) % (c->lpool_n - kLearnedBatch + 1);
        const double L = c->ltrainer.loss_grad(c->lpool + (long)first * vol, c->lw.data(), grad.data(), c->st);
        if (!std::isfinite(L)) throw Error(PASM_E_BREAKDOWN, "learned smoother: non-finite training loss");
        const int t = ++c->ltrain_steps;
        if (t == 1) c->lloss_first = L;
        c->lloss_last = L;
        if (hist) hist[it] = L;
        for (int j = 0; j < 864; ++j) {
            c->lm[j] = b1 * c->lm[j] + (1 - b1) * grad[j];
            c->lv2[j] = b2 * c->lv2[j] + (1 - b2) * grad[j] * grad[j];
            const double mh = c->lm[j] / (1 - std::pow(b1, t)), vh = c->lv2[j] / (1 - std::pow(b2, t));
            c->lw[j] = (float)(c->lw[j] - kLearnedLr * mh / (std::sqrt(vh) + eps));
        }
    }
    learned_pack(c);
}

// Residual reduction per V-cycle of plain and learned cycles on the start
// boundary value problems (f = lambda M u from x = u): the worst ratio over
// the right-hand sides and three consecutive cycles (the later cycles see the
// smoother residuals that dominate the rate).
void learned_rates(pasm_ctx* c) {
    const Grid& g = c->gf();
    const int k = c->k;
    const size_t bytes = (size_t)g.plane * k * sizeof(double);
    pasm::launch_mass_rhs(g, c->U, c->lam, c->F64, k, g.plane, c->st);
    double rate[2] = {0.0, 0.0}, ms[2] = {0.0, 0.0};
    hipEvent_t e0, e1;
    PASM_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    PASM_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    for (int mode = 0; mode < 2; ++mode) {
        double* x = c->R64;
        double* scr = c->Y64;
        PASM_HIP(hipMemcpyAsync(x, c->U, bytes, hipMemcpyDeviceToDevice, c->st));
        c->learned_on = mode == 1;
        std::vector<double> n0 = resid_norms(c, x, c->F64, k);
        for (int cy = 0; cy < 3; ++cy) {
            PASM_HIP(hipEventRecord(e0, c->st));
            one_cycle(c, x, scr, c->F64, k);
            PASM_HIP(hipEventRecord(e1, c->st));
            const std::vector<double> n1 = resid_norms(c, x, c->F64, k);
            float t = 0.f;
            PASM_HIP(hipEventElapsedTime(&t, e0, e1));
            if (cy > 0) ms[mode] += t / 2.0;  // the first cycle warms up
            for (int r = 0; r < k; ++r)
                if (n0[r] > 0.0) rate[mode] = std::max(rate[mode], std::sqrt(n1[r] / n0[r]));
            n0 = n1;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->lplain_rate = rate[0];
    c->llearned_rate = rate[1];
    c->lplain_ms = ms[0];
    c->llearned_ms = ms[1];
    // use the learned smoother only if it reduces the residual more per unit
    // time than the plain one on this start (log rate per millisecond)
    const double gp = std::log(std::max(rate[0], 1e-300)) / std::max(ms[0], 1e-6);
    const double gl = std::log(std::max(rate[1], 1e-300)) / std::max(ms[1], 1e-6);
    c->learned_on = rate[1] < 1.0 && gl < gp;
}

void learned_setup(pasm_ctx* c) {
    c->lstag.assign(c->k, 0);
    c->lw.assign(864, 0.f);
    c->lm.assign(864, 0.0);
    c->lv2.assign(864, 0.0);
    // start from damped Jacobi: channel 0 passes +rho, channel 1 passes -rho,
    // x + omega (h_0 - h_1) = x + omega rho; the other channels start small
    const double omega = c->opt.omega > 0 ? c->opt.omega : 6.0 / 7.0;
    std::mt19937_64 rng(12345);
    std::normal_distribution<double> nd(0.0, 0.02);
    for (int j = 0; j < 864; ++j) c->lw[j] = (float)nd(rng);
    for (int t = 0; t < 27; ++t) {
        c->lw[0 * 27 + t] = c->lw[1 * 27 + t] = 0.f;
        c->lw[16 * 27 + 0 * 27 + t] = c->lw[16 * 27 + 1 * 27 + t] = 0.f;
    }
    c->lw[0 * 27 + 13] = 1.f;
    c->lw[1 * 27 + 13] = -1.f;
    c->lw[16 * 27 + 0 * 27 + 13] = (float)omega;
    c->lw[16 * 27 + 1 * 27 + 13] = (float)-omega;
    c->lops = c->alloc<unsigned long long>(pasm::kLearnedStepOps);
    const Grid& g = c->gf();
    c->Xb = c->alloc<double>((size_t)g.plane * c->k);
    const long nb = (g.interior() + 255) / 256;
    c->rnpart = c->alloc<double>(2 * (size_t)nb * c->k);
    c->rnsum = c->alloc<double>(2 * (size_t)c->k);
    learned_pack(c);
    // training level: 32 cells per side where available, below the finest
    int lt = -1;
    for (int l = 1; l < c->L - 1; ++l)
        if (c->lv[l].g.n <= 32) lt = l;
    c->ltrain_level = lt;
    if (lt < 1) {  // no level to train on: plain smoothing throughout
        c->learned_on = false;
        return;
    }
    const Grid& gt = c->lv[lt].g;
    c->lpool = c->alloc<float>((size_t)kLearnedPool * gt.interior());
    c->ltrainer.init(gt.m, kLearnedBatch, (float)c->lv[lt].w0, [c](size_t b) { return (void*)c->alloc<char>(b); });
    if (c->mixed) learned_pool<float>(c);
    else learned_pool<double>(c);
    learned_train(c, kLearnedSetupSteps, nullptr);
    learned_rates(c);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#define PASM_TRY(ctx, ...)                                         \
    try {                                                          \
        __VA_ARGS__;                                               \
    } catch (const Error& e_) {                                    \
        set_error(ctx, e_.msg);                                    \
        return e_.status;                                          \
    } catch (const std::exception& e_) {                           \
        set_error(ctx, e_.what());                                 \
        return PASM_E_DEVICE;                                      \
    }

namespace {
void restart_ctx(pasm_ctx* c);
void restart_nested(pasm_ctx* c, int varpi);
}  // namespace

extern "C" {

PASM_API void pasm_default_options(pasm_options* o) {
    if (!o) return;
    o->precision = PASM_FP64;
    o->smoother = PASM_JACOBI;
    o->nu_pre = 2;
    o->nu_post = 2;
    o->vcycles = 2;
    o->max_iter = 50;
    o->tol = 1e-10;
    o->omega = 0.0;
    o->cheb_alpha = 0.0;
    o->stream = nullptr;
    o->fused_smoothing = 1;
    o->exhaustive_selection = 0;
}

PASM_API pasm_status pasm_destroy(pasm_ctx* c) {
    if (!c) return PASM_OK;
    if (c->st) (void)hipStreamSynchronize(c->st);
    for (pasm_ctx* ch : c->nested) pasm_destroy(ch);  // they use c's stream and coarse space
    c->nested.clear();
    drop_graphs(c);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->lam_pin) (void)hipHostFree(c->lam_pin);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->blas) rocblas_destroy_handle(c->blas);
    if (c->own_stream && c->st) (void)hipStreamDestroy(c->st);
    delete c;
    return PASM_OK;
}

PASM_API pasm_status pasm_setup(pasm_ctx** out, const pasm_domain* dom, const pasm_coefficients* coef, double H,
                                double h, int k, const pasm_options* opt) {
    if (!out) return PASM_E_INVALID;
    *out = nullptr;
    pasm_ctx* c = new (std::nothrow) pasm_ctx();
    if (!c) return PASM_E_NOMEM;
    if (opt) c->opt = *opt;
    else pasm_default_options(&c->opt);
    try {
        const Plan pl = validate(c->opt, dom, coef, H, h, k);
        PASM_HIP(hipGetDevice(&c->device));
        if (c->opt.stream) c->st = static_cast<hipStream_t>(c->opt.stream);
        else {
            PASM_HIP(hipStreamCreate(&c->st));
            c->own_stream = true;
        }
        build(c, pl, coef, k);
        prolong_coefs(c, nullptr);
        PASM_HIP(hipStreamSynchronize(c->st));
        if (c->opt.smoother == PASM_LEARNED) {
            c->learned = true;
            learned_setup(c);
        }
    } catch (const Error& e) {
        g_setup_error = e.msg;
        pasm_destroy(c);
        return e.status;
    } catch (const std::exception& e) {
        g_setup_error = e.what();
        pasm_destroy(c);
        return PASM_E_DEVICE;
    }
    *out = c;
    return PASM_OK;
}

PASM_API pasm_status pasm_iterate(pasm_ctx* c, int* converged) {
    if (!c || c->k == 0) return PASM_E_STATE;
    PASM_TRY(c, {
        step(c);
        c->lam_prev_h = c->lam_h;
        PASM_HIP(hipMemcpyAsync(c->lam_pin, c->lam, c->k * sizeof(double), hipMemcpyDeviceToHost, c->st));
        PASM_HIP(hipStreamSynchronize(c->st));
        std::copy(c->lam_pin, c->lam_pin + c->k, c->lam_h.begin());
        if (c->ev_used >= kProfileBatch) collect_profile(c);
        ++c->iters;
        double dmax = 0.0;
        bool finite = true;
        for (int i = 0; i < c->k; ++i) {
            const double l = c->lam_h[i];
            if (!std::isfinite(l)) finite = false;
            dmax = std::max(dmax, std::fabs(l - c->lam_prev_h[i]) / std::fabs(l));
        }
        if (!finite) {
            set_error(c, "non-finite eigenvalue");
            return PASM_E_BREAKDOWN;
        }
        if (converged) *converged = dmax < c->opt.tol ? 1 : 0;
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_iterate_n(pasm_ctx* c, int n, int* converged) {
    if (!c || c->k == 0) return PASM_E_STATE;
    if (n < 1) return PASM_E_INVALID;
    PASM_TRY(c, {
        for (int i = 0; i < n; ++i) step(c, i + 1 < n);
        // the eigenvalues before and after the last step, in one synchronisation
        // (pinned host memory: both copies are asynchronous)
        PASM_HIP(hipMemcpyAsync(c->lam_pin, c->lam_prev, c->k * sizeof(double), hipMemcpyDeviceToHost, c->st));
        PASM_HIP(hipMemcpyAsync(c->lam_pin + c->k, c->lam, c->k * sizeof(double), hipMemcpyDeviceToHost, c->st));
        PASM_HIP(hipStreamSynchronize(c->st));
        std::copy(c->lam_pin, c->lam_pin + c->k, c->lam_prev_h.begin());
        std::copy(c->lam_pin + c->k, c->lam_pin + 2 * c->k, c->lam_h.begin());
        if (c->ev_used >= kProfileBatch) collect_profile(c);
        c->iters += n;
        double dmax = 0.0;
        bool finite = true;
        for (int i = 0; i < c->k; ++i) {
            const double l = c->lam_h[i];
            if (!std::isfinite(l)) finite = false;
            dmax = std::max(dmax, std::fabs(l - c->lam_prev_h[i]) / std::fabs(l));
        }
        if (!finite) {
            set_error(c, "non-finite eigenvalue");
            return PASM_E_BREAKDOWN;
        }
        if (converged) *converged = dmax < c->opt.tol ? 1 : 0;
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_restart(pasm_ctx* c) {
    if (!c || c->k == 0) return PASM_E_STATE;
    PASM_TRY(c, restart_ctx(c));
    return PASM_OK;
}

PASM_API pasm_status pasm_restart_nested(pasm_ctx* c, int varpi) {
    if (!c || c->k == 0) return PASM_E_STATE;
    if (varpi < 1) return PASM_E_INVALID;
    if (c->general_coef) {
        set_error(c, "the nested schedule needs the intermediate levels as rediscretisations (no potential term)");
        return PASM_E_INVALID;
    }
    PASM_TRY(c, restart_nested(c, varpi));
    return PASM_OK;
}

}  // extern "C"

namespace {
// Return to the start of Algorithm 2 (lambda_i = theta_i, u_i = P q_i).
void restart_ctx(pasm_ctx* c) {
    c->f_ready = false;
    c->lstag.assign(c->k, 0);
    {
        const int k = c->k, N = c->NH;
        c->lam_h = c->theta_h;
        c->lam_prev_h = c->theta_h;
        // lambda = lambda_prev = theta, unit coefficients, and q_i itself as
        // the coarse vector Q e_i, in one launch
        const pasm::Level& L0 = c->lv[0];
        pasm::launch_restart_coarse(c->Qcm, N, L0.g, c->L == 1 ? c->U : L0.B, L0.g.plane, c->ycoef, k, k, 0,
                                    c->theta, 0, c->lam, c->lam_prev, c->st);
        // u_i = P q_i (weights of the old u all zero) and the first step's
        // right-hand side theta_i M u_i: left to the next step's first
        // marching pre-smoothing where it can form them in its pass (any
        // other caller forms them first), else in one pass now; in flight on
        // the context's stream either way
        c->prolong_pending = false;
        if (prolong_deferrable(c)) {
            c->prolong_pending = true;
            c->pend_beta = c->zeros;
            c->f_ready = true;
        } else {
            prolong_coefs(c, c->zeros, c->lam, true);
        }
    }
}

// Context of intermediate level l (1 <= l <= L-2) of c: the same problem
// on the mesh h_l = H / 2^l (the Galerkin operators of c's hierarchy: for
// constant coefficients and per-element kappa a rediscretisation with the
// coarsened kappa), the same k, options and stream, c's coarse space.
pasm_ctx* make_level_ctx(pasm_ctx* c, int l) {
    std::unique_ptr<pasm_ctx> ch(new pasm_ctx());
    ch->opt = c->opt;
    ch->opt.stream = c->st;
    if (ch->opt.smoother == PASM_LEARNED) ch->opt.smoother = PASM_JACOBI;
    ch->st = c->st;
    ch->own_stream = false;
    ch->device = c->device;
    const int n = c->lv[l].g.n;
    pasm_domain dom{c->dim};
    pasm_coefficients cf{nullptr, nullptr, 0};
    if ((size_t)l < c->level_kappa.size() && !c->level_kappa[l].empty()) {
        cf.kappa = c->level_kappa[l].data();
        cf.n_elements = c->level_kappa[l].size();
    }
    const double H = 1.0 / c->lv[0].g.n, h = 1.0 / n;
    const Plan pl = validate(ch->opt, &dom, &cf, H, h, c->k);
    build(ch.get(), pl, &cf, c->k, c);
    return ch.release();
}

// x_next = P x (all k vectors) between the finest levels of two contexts of
// the same problem on consecutive meshes, and lambda carried over.
void carry_to_finer(pasm_ctx* from, pasm_ctx* to) {
    const Grid& gc = from->gf();
    const Grid& gf = to->gf();
    pasm::launch_prolong<double>(gc, from->U, gf, to->U, from->k, gc.plane, gf.plane, false, nullptr, to->st);
    PASM_HIP(hipMemcpyAsync(to->lam, from->lam, from->k * sizeof(double), hipMemcpyDeviceToDevice, to->st));
    PASM_HIP(hipMemcpyAsync(to->lam_prev, from->lam, from->k * sizeof(double), hipMemcpyDeviceToDevice, to->st));
    to->f_ready = false;
    to->prolong_pending = false;
    to->lstag.assign(to->k, 0);
}

// Algorithm 2 with its step 2(A): the coarse start on V_H, then varpi
// correction steps on each intermediate level h_2, ..., h_{n-1} (each level
// starting from the previous one's result), leaving the finest level at the
// start of step 2(B).  All work is enqueued on the context's stream; one
// synchronisation at the end reads the eigenvalues.
void restart_nested(pasm_ctx* c, int varpi) {
    if (c->L <= 2) {
        restart_ctx(c);
        return;
    }
    if (c->nested.empty()) {
        settle_prolongation(c);
        for (int l = 1; l <= c->L - 2; ++l) c->nested.push_back(make_level_ctx(c, l));
    }
    c->prolong_pending = false;
    pasm_ctx* prev = nullptr;
    for (pasm_ctx* ch : c->nested) {
        if (!prev) restart_ctx(ch);
        else carry_to_finer(prev, ch);
        for (int it = 0; it < varpi; ++it) iterate_once(ch, false);
        prev = ch;
    }
    carry_to_finer(prev, c);
    PASM_HIP(hipMemcpyAsync(c->lam_pin, c->lam, c->k * sizeof(double), hipMemcpyDeviceToHost, c->st));
    PASM_HIP(hipStreamSynchronize(c->st));
    c->lam_h.assign(c->lam_pin, c->lam_pin + c->k);
    c->lam_prev_h = c->lam_h;
}
}  // namespace

extern "C" {

PASM_API pasm_status pasm_solve(pasm_ctx* c, int* iterations) {
    if (!c || c->k == 0) return PASM_E_STATE;
    int it = 0, conv = 0;
    while (it < c->opt.max_iter) {
        pasm_status s = pasm_iterate(c, &conv);
        ++it;
        if (s != PASM_OK) {
            if (iterations) *iterations = it;
            return s;
        }
        if (conv) break;
    }
    if (iterations) *iterations = it;
    return conv ? PASM_OK : PASM_E_NOTCONV;
}

PASM_API pasm_status pasm_eigenpairs(pasm_ctx* c, double* lambda, double* U, size_t ldu) {
    if (!c || c->k == 0) return PASM_E_STATE;
    const size_t N = pasm_num_dofs(c);
    if (U && ldu < N) return PASM_E_INVALID;
    PASM_TRY(c, {
        if (lambda) std::memcpy(lambda, c->lam_h.data(), c->k * sizeof(double));
        if (U) {
            // eigenvectors whose last prolongation is still pending are formed first
            settle_prolongation(c);
            pasm::launch_pack<double>(c->gf(), c->U, c->sf(), c->stage, (long)N, c->k, c->st);
            PASM_HIP(hipMemcpy2DAsync(U, ldu * sizeof(double), c->stage, N * sizeof(double), N * sizeof(double), c->k,
                                      hipMemcpyDeviceToHost, c->st));
            PASM_HIP(hipStreamSynchronize(c->st));
        }
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_eigenvectors_device(pasm_ctx* c, double* U_dev, size_t ldu) {
    if (!c || c->k == 0) return PASM_E_STATE;
    if (!U_dev || ldu < pasm_num_dofs(c)) return PASM_E_INVALID;
    PASM_TRY(c, {
        settle_prolongation(c);
        pasm::launch_pack<double>(c->gf(), c->U, c->sf(), U_dev, (long)ldu, c->k, c->st);
        PASM_HIP(hipStreamSynchronize(c->st));
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_set_state(pasm_ctx* c, const double* lambda, const double* U, size_t ldu) {
    if (!c || c->k == 0) return PASM_E_STATE;
    c->f_ready = false;
    c->lstag.assign(c->k, 0);
    const size_t N = pasm_num_dofs(c);
    if (!lambda || !U || ldu < N) return PASM_E_INVALID;
    for (int i = 0; i < c->k; ++i)
        if (!std::isfinite(lambda[i])) return PASM_E_INVALID;
    // non-finite vector entries are refused here, before any kernel sees them
    for (int i = 0; i < c->k; ++i)
        for (size_t j = 0; j < N; ++j)
            if (!std::isfinite(U[(size_t)i * ldu + j])) {
                set_error(c, "pasm_set_state: U holds a non-finite value");
                return PASM_E_INVALID;
            }
    PASM_TRY(c, {
        c->prolong_pending = false;  // the state is replaced
        c->r32_ready = false;
        c->lam_h.assign(lambda, lambda + c->k);
        c->lam_prev_h = c->lam_h;
        PASM_HIP(hipMemcpyAsync(c->lam, lambda, c->k * sizeof(double), hipMemcpyHostToDevice, c->st));
        PASM_HIP(hipMemcpyAsync(c->lam_prev, lambda, c->k * sizeof(double), hipMemcpyHostToDevice, c->st));
        PASM_HIP(hipMemcpy2DAsync(c->stage, N * sizeof(double), U, ldu * sizeof(double), N * sizeof(double), c->k,
                                  hipMemcpyHostToDevice, c->st));
        pasm::launch_unpack<double>(c->gf(), c->stage, (long)N, c->U, c->sf(), c->k, c->st);
        PASM_HIP(hipStreamSynchronize(c->st));
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_last_selection(const pasm_ctx* cc, int* rank, double* score, int* flags) {
    const pasm_ctx* c = cc;
    if (!c || c->k == 0) return PASM_E_STATE;
    PASM_TRY(c, {
        if (rank) PASM_HIP(hipMemcpyAsync(rank, c->rank, c->k * sizeof(int), hipMemcpyDeviceToHost, c->st));
        if (score) PASM_HIP(hipMemcpyAsync(score, c->score, c->k * sizeof(double), hipMemcpyDeviceToHost, c->st));
        if (flags) PASM_HIP(hipMemcpyAsync(flags, c->flags, c->k * sizeof(int), hipMemcpyDeviceToHost, c->st));
        PASM_HIP(hipStreamSynchronize(c->st));
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_coarse_eigenpairs(const pasm_ctx* cc, double* theta, double* Q) {
    const pasm_ctx* c = cc;
    if (!c || c->k == 0) return PASM_E_STATE;
    const size_t N = c->NH;
    PASM_TRY(c, {
        if (theta) PASM_HIP(hipMemcpyAsync(theta, c->theta, N * sizeof(double), hipMemcpyDeviceToHost, c->st));
        if (Q) PASM_HIP(hipMemcpyAsync(Q, c->Qcm, N * N * sizeof(double), hipMemcpyDeviceToHost, c->st));
        PASM_HIP(hipStreamSynchronize(c->st));
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_last_borders(const pasm_ctx* cc, double* beta_zeta, double* p, double* q) {
    const pasm_ctx* c = cc;
    if (!c || c->k == 0) return PASM_E_STATE;
    const size_t N = c->NH, k = c->k;
    PASM_TRY(c, {
        if (beta_zeta) PASM_HIP(hipMemcpyAsync(beta_zeta, c->bz, 2 * k * sizeof(double), hipMemcpyDeviceToHost, c->st));
        if (p) PASM_HIP(hipMemcpyAsync(p, c->pp, N * k * sizeof(double), hipMemcpyDeviceToHost, c->st));
        if (q) PASM_HIP(hipMemcpyAsync(q, c->qq, N * k * sizeof(double), hipMemcpyDeviceToHost, c->st));
        PASM_HIP(hipStreamSynchronize(c->st));
    });
    return PASM_OK;
}

PASM_API size_t pasm_num_dofs(const pasm_ctx* c) { return (c && c->L) ? (size_t)c->gf().interior() : 0; }
PASM_API size_t pasm_coarse_dofs(const pasm_ctx* c) { return c ? (size_t)c->NH : 0; }
PASM_API int pasm_num_levels(const pasm_ctx* c) { return c ? c->L : 0; }

PASM_API const char* pasm_status_string(pasm_status s) {
    switch (s) {
        case PASM_OK: return "ok";
        case PASM_E_INVALID: return "invalid argument";
        case PASM_E_NOMEM: return "out of memory";
        case PASM_E_DEVICE: return "device error";
        case PASM_E_STATE: return "invalid call order";
        case PASM_E_NOTCONV: return "not converged";
        case PASM_E_BREAKDOWN: return "breakdown (non-finite values)";
    }
    return "unknown status";
}

PASM_API const char* pasm_last_error(const pasm_ctx* c) { return c ? c->err.c_str() : g_setup_error.c_str(); }

PASM_API pasm_status pasm_apply_operator(pasm_ctx* c, int level, int op, const double* x, double* y, size_t ld,
                                         int nrhs) {
    if (!c || c->k == 0) return PASM_E_STATE;
    if (level < 0 || level >= c->L || nrhs < 1 || nrhs > c->k || !x || !y) return PASM_E_INVALID;
    if (op != PASM_OP_STIFFNESS && op != PASM_OP_MASS) return PASM_E_INVALID;
    if (op == PASM_OP_MASS && level != c->L - 1) return PASM_E_INVALID;
    const Grid& g = c->lv[level].g;
    if (ld < (size_t)g.interior()) return PASM_E_INVALID;
    PASM_TRY(c, {
        settle_prolongation(c);
        // F64 may be overwritten below: the next step forms lambda M u again
        c->f_ready = false;
        const bool fine = level == c->L - 1;
        double* tin = fine ? c->Y64 : c->lv[level].B;
        double* tout = fine ? c->R64 : c->lv[level].C;
        pasm::launch_unpack<double>(g, x, (long)ld, tin, g.plane, nrhs, c->st);
        if (op == PASM_OP_MASS) pasm::launch_apply_M(g, tin, tout, nrhs, g.plane, c->st);
        else pasm::launch_apply_A<double>(g, c->coef<double>(level), tin, tout, nrhs, g.plane, c->st);
        pasm::launch_pack<double>(g, tout, g.plane, y, (long)ld, nrhs, c->st);
        PASM_HIP(hipStreamSynchronize(c->st));
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_vcycle(pasm_ctx* c, const double* f, double* x, size_t ld, int nrhs, int ncycles) {
    if (!c || c->k == 0) return PASM_E_STATE;
    const Grid& g = c->gf();
    if (!f || !x || nrhs < 1 || nrhs > c->k || ncycles < 0 || ld < (size_t)g.interior()) return PASM_E_INVALID;
    PASM_TRY(c, {
        settle_prolongation(c);
        // F64 may be overwritten below: the next step forms lambda M u again
        c->f_ready = false;
        pasm::launch_unpack<double>(g, f, (long)ld, c->F64, g.plane, nrhs, c->st);
        pasm::launch_unpack<double>(g, x, (long)ld, c->R64, g.plane, nrhs, c->st);
        double* xb = c->R64;
        double* yb = c->Y64;
        if (c->L > 1) bvp_cycles(c, xb, yb, c->F64, nrhs, ncycles);
        else if (ncycles > 0)
            coarse_solve<double>(c, c->F64, xb, nrhs);
        pasm::launch_pack<double>(g, xb, g.plane, x, (long)ld, nrhs, c->st);
        PASM_HIP(hipStreamSynchronize(c->st));
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_learned_report(const pasm_ctx* c, pasm_learned_stats* o) {
    if (!c || c->k == 0) return PASM_E_STATE;
    if (!o) return PASM_E_INVALID;
    if (!c->learned) return PASM_E_STATE;
    o->enabled = c->learned_on ? 1 : 0;
    o->train_steps = c->ltrain_steps;
    o->loss_first = c->lloss_first;
    o->loss_last = c->lloss_last;
    o->plain_rate = c->lplain_rate;
    o->learned_rate = c->llearned_rate;
    o->plain_cycle_ms = c->lplain_ms;
    o->learned_cycle_ms = c->llearned_ms;
    o->cycles_learned = c->lcycles_learned;
    o->cycles_fallback = c->lcycles_fallback;
    return PASM_OK;
}

PASM_API int pasm_learned_ratios(const pasm_ctx* c, double* out, int max) {
    if (!c || max < 0 || (max > 0 && !out)) return -1;
    const int n = (int)std::min<size_t>(c->lratio.size(), (size_t)max);
    for (int i = 0; i < n; ++i) out[i] = c->lratio[c->lratio.size() - n + i];
    return n;
}

PASM_API pasm_status pasm_learned_weights(const pasm_ctx* c, float* w) {
    if (!c || c->k == 0 || !c->learned) return PASM_E_STATE;
    if (!w) return PASM_E_INVALID;
    std::memcpy(w, c->lw.data(), 864 * sizeof(float));
    return PASM_OK;
}

PASM_API pasm_status pasm_learned_set_weights(pasm_ctx* c, const float* w) {
    if (!c || c->k == 0 || !c->learned) return PASM_E_STATE;
    if (c) c->f_ready = false;
    if (!w) return PASM_E_INVALID;
    for (int j = 0; j < 864; ++j)
        if (!std::isfinite(w[j])) return PASM_E_INVALID;
    PASM_TRY(c, {
        c->lw.assign(w, w + 864);
        learned_pack(c);
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_learned_set_threshold(pasm_ctx* c, double rate) {
    if (!c || c->k == 0 || !c->learned) return PASM_E_STATE;
    if (c) c->f_ready = false;
    if (!std::isfinite(rate)) return PASM_E_INVALID;
    c->lthreshold = rate > 0.0 ? rate : 0.0;
    return PASM_OK;
}

PASM_API pasm_status pasm_learned_enable(pasm_ctx* c, int enable) {
    if (!c || c->k == 0 || !c->learned) return PASM_E_STATE;
    PASM_TRY(c, settle_prolongation(c));
    c->f_ready = false;
    c->learned_on = enable != 0;
    return PASM_OK;
}

PASM_API pasm_status pasm_learned_train(pasm_ctx* c, int steps, double* hist) {
    if (!c || c->k == 0 || !c->learned || c->ltrain_level < 1) return PASM_E_STATE;
    if (steps < 0) return PASM_E_INVALID;
    PASM_TRY(c, {
        settle_prolongation(c);
        // F64 may be overwritten below: the next step forms lambda M u again
        c->f_ready = false;
        learned_train(c, steps, hist);
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_learned_step(pasm_ctx* c, int level, const double* x, const double* f, double* out,
                                       size_t ld, int nrhs) {
    if (!c || c->k == 0 || !c->learned) return PASM_E_STATE;
    if (level < 1 || level >= c->L || nrhs < 1 || nrhs > c->k || !x || !f || !out) return PASM_E_INVALID;
    const pasm::Level& L = c->lv[level];
    const Grid& g = L.g;
    if (ld < (size_t)g.interior()) return PASM_E_INVALID;
    PASM_TRY(c, {
        settle_prolongation(c);
        // F64 may be overwritten below: the next step forms lambda M u again
        c->f_ready = false;
        const bool fine = level == c->L - 1;
        if (c->mixed) {
            float* xb = fine ? c->E32 : static_cast<float*>(L.X);
            float* fb = fine ? c->R32 : static_cast<float*>(L.F);
            float* ob = fine ? c->Y32 : static_cast<float*>(L.Y);
            pasm::launch_unpack<float>(g, x, (long)ld, xb, g.plane, nrhs, c->st);
            pasm::launch_unpack<float>(g, f, (long)ld, fb, g.plane, nrhs, c->st);
            pasm::launch_learned_step<float>(g, (float)L.w0, xb, fb, ob, nrhs, g.plane, c->lops, false, c->st);
            pasm::launch_pack<float>(g, ob, g.plane, out, (long)ld, nrhs, c->st);
        } else {
            double* xb = fine ? c->R64 : static_cast<double*>(L.X);
            double* fb = fine ? c->F64 : static_cast<double*>(L.F);
            double* ob = fine ? c->Y64 : static_cast<double*>(L.Y);
            pasm::launch_unpack<double>(g, x, (long)ld, xb, g.plane, nrhs, c->st);
            pasm::launch_unpack<double>(g, f, (long)ld, fb, g.plane, nrhs, c->st);
            pasm::launch_learned_step<double>(g, L.w0, xb, fb, ob, nrhs, g.plane, c->lops, false, c->st);
            pasm::launch_pack<double>(g, ob, g.plane, out, (long)ld, nrhs, c->st);
        }
        PASM_HIP(hipStreamSynchronize(c->st));
    });
    return PASM_OK;
}

namespace {
__global__ void k_compact_d2f(const double* __restrict__ a, long lda, float* __restrict__ b, long n) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t < n) b[(long)blockIdx.y * n + t] = (float)a[(long)blockIdx.y * lda + t];
}
}  // namespace

PASM_API pasm_status pasm_learned_loss_grad(pasm_ctx* c, int level, const double* r, size_t ld, int ns,
                                            double* loss, double* grad) {
    if (!c || c->k == 0 || !c->learned) return PASM_E_STATE;
    if (level < 1 || level >= c->L || ns < 1 || ns > 64 || !r || !grad) return PASM_E_INVALID;
    const Grid& g = c->lv[level].g;
    const long vol = g.interior();
    if (ld < (size_t)vol) return PASM_E_INVALID;
    PASM_TRY(c, {
        settle_prolongation(c);
        // F64 may be overwritten below: the next step forms lambda M u again
        c->f_ready = false;
        // a trainer sized for this level and sample count (not the hot path)
        std::vector<void*> mine;
        auto alloc = [&](size_t b) {
            void* p = nullptr;
            if (hipMalloc(&p, b ? b : 1) != hipSuccess) throw Error(PASM_E_NOMEM, "hipMalloc failed");
            mine.push_back(p);
            PASM_HIP(hipMemsetAsync(p, 0, b ? b : 1, c->st));
            return p;
        };
        try {
            pasm::LearnedTrainer tr;
            tr.init(g.m, ns, (float)c->lv[level].w0, alloc);
            float* rf = static_cast<float*>(alloc(sizeof(float) * vol * ns));
            hipLaunchKernelGGL(k_compact_d2f, dim3((unsigned)((vol + 255) / 256), ns), dim3(256), 0, c->st, r, (long)ld,
                               rf, vol);
            PASM_CHECK_LAUNCH();
            const double L = tr.loss_grad(rf, c->lw.data(), grad, c->st);
            if (loss) *loss = L;
        } catch (...) {
            (void)hipStreamSynchronize(c->st);
            for (void* p : mine) (void)hipFree(p);
            throw;
        }
        PASM_HIP(hipStreamSynchronize(c->st));
        for (void* p : mine) (void)hipFree(p);
    });
    return PASM_OK;
}

// ---------------------------------------------------------------------------
// pasm_learned_loss_grad_noalloc: the same loss and gradient with every
// device buffer carved out of a file-scope device array instead of hipMalloc.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

// Enough for 8 samples on the 32-cell level (the library's own training
// batch) or 63 samples on the 16-cell level.  Every GPU the library runs on
// holds one copy until the process ends.
constexpr size_t kNoAllocScratchBytes = (size_t)72 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on GPU `dev`, which must be the current
// device: taken once per device with hipGetSymbolAddress and kept.  Host
// code uses only this address (the array's own name is a host-side stand-in).
void* scratch_address(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) throw Error(PASM_E_DEVICE, "device index out of range for the scratch table");
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            throw Error(PASM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// Makes the context's device current for the duration of a call and
// restores the caller's.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        PASM_HIP(hipGetDevice(&prev));
        if (prev != dev) PASM_HIP(hipSetDevice(dev));
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

__global__ void k_zero_words(uint4* __restrict__ p, long n) {
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long)gridDim.x * 256) p[t] = z;
}

// Bytes the trainer of (m, ns) and the FP32 copy of the samples take in the
// scratch array, each buffer rounded up to 256 bytes.
size_t loss_grad_scratch_bytes(int m, int ns) {
    size_t off = 0;
    auto count = [&](size_t b) -> void* {
        off += (b + 255) / 256 * 256;
        return reinterpret_cast<void*>(static_cast<uintptr_t>(256));  // never dereferenced
    };
    pasm::LearnedTrainer dry;
    dry.init(m, ns, 1.f, count);
    count(sizeof(float) * (size_t)m * m * m * ns);
    return off;
}

}  // namespace

extern "C" {

PASM_API pasm_status pasm_learned_loss_grad_noalloc(pasm_ctx* c, int level, const double* r, size_t ld, int ns,
                                                    double* loss, double* grad) {
    if (!c || c->k == 0 || !c->learned) return PASM_E_STATE;
    if (level < 1 || level >= c->L || ns < 1 || ns > 64 || !r || !grad) return PASM_E_INVALID;
    const Grid& g = c->lv[level].g;
    const long vol = g.interior();
    if (ld < (size_t)vol) return PASM_E_INVALID;
    const size_t need = loss_grad_scratch_bytes(g.m, ns);
    if (need > kNoAllocScratchBytes) {
        set_error(c, "pasm_learned_loss_grad_noalloc: " + std::to_string(ns) + " samples on a level of " +
                         std::to_string(g.n) + " cells need " + std::to_string(need) + " bytes of scratch, more than its " +
                         std::to_string(kNoAllocScratchBytes) + " (use pasm_learned_loss_grad)");
        return PASM_E_INVALID;
    }
    PASM_TRY(c, {
        DeviceGuard dg(c->device);
        settle_prolongation(c);
        c->f_ready = false;
        unsigned char* base = static_cast<unsigned char*>(scratch_address(c->device));
        // the array keeps the previous call's contents: clear the part used
        // (a kernel, not a memset, so that the call could sit in a graph)
        const long words = (long)(need / sizeof(uint4));
        hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<long>((words + 255) / 256, 4096)), dim3(256), 0, c->st,
                           reinterpret_cast<uint4*>(base), words);
        PASM_CHECK_LAUNCH();
        size_t off = 0;
        auto carve = [&](size_t b) -> void* {
            void* p = base + off;
            off += (b + 255) / 256 * 256;
            if (off > need) throw Error(PASM_E_DEVICE, "scratch layout mismatch");
            return p;
        };
        pasm::LearnedTrainer tr;
        tr.init(g.m, ns, (float)c->lv[level].w0, carve);
        float* rf = static_cast<float*>(carve(sizeof(float) * vol * ns));
        hipLaunchKernelGGL(k_compact_d2f, dim3((unsigned)((vol + 255) / 256), ns), dim3(256), 0, c->st, r, (long)ld, rf,
                           vol);
        PASM_CHECK_LAUNCH();
        const double L = tr.loss_grad(rf, c->lw.data(), grad, c->st);
        if (loss) *loss = L;
        PASM_HIP(hipStreamSynchronize(c->st));
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_use_graph(pasm_ctx* c, int enable) {
    if (!c) return PASM_E_STATE;
    PASM_TRY(c, {
        PASM_HIP(hipStreamSynchronize(c->st));
        drop_graphs(c);
    });
    c->use_graph = enable != 0;
    return PASM_OK;
}

PASM_API pasm_status pasm_graph_stats(const pasm_ctx* c, int* enabled, int* graphs, long* replays) {
    if (!c) return PASM_E_STATE;
    if (enabled) *enabled = c->use_graph ? 1 : 0;
    if (graphs) *graphs = (int)c->graphs.size();
    if (replays) *replays = c->graph_replays;
    return PASM_OK;
}

PASM_API pasm_status pasm_profile(pasm_ctx* c, int kernel, int enable) {
    if (!c) return PASM_E_STATE;
    if (kernel != 0) return PASM_E_INVALID;
    c->prof = enable != 0;
    c->prof_launches = 0;
    c->prof_ms = 0.0;
    c->prof_bytes = 0.0;
    c->ev_used = 0;
    return PASM_OK;
}

PASM_API pasm_status pasm_profile_read(pasm_ctx* c, int kernel, long* launches, double* total_ms,
                                       double* bytes_per_launch) {
    if (!c) return PASM_E_STATE;
    if (kernel != 0) return PASM_E_INVALID;
    PASM_TRY(c, {
        PASM_HIP(hipStreamSynchronize(c->st));
        collect_profile(c);
    });
    if (launches) *launches = c->prof_launches;
    if (total_ms) *total_ms = c->prof_ms;
    if (bytes_per_launch) *bytes_per_launch = c->prof_launches ? c->prof_bytes / c->prof_launches : 0.0;
    return PASM_OK;
}

}  // extern "C"
