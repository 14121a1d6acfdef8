// Batches of problems of uneven size, advanced together (include/pasm.h,
// "Batches of problems of uneven size").
//
// The correction step of Algorithm 1 is applied to every eigenpair of every
// member independently (the eigenpairs of Algorithm 2 exchange nothing), so
// the only coupling a batch adds is sharing launches.  Storage is
// level-major: members are ordered by decreasing fine size (slot order), and
// level l of the batch holds, for the first count_l slots (the members that
// have a level l), k right-hand sides each, one padded plane apart.  A member
// whose finest level is l ("top" level) occupies slots [a, count_l) of level
// l, so one launch per level runs the smoothing, residual restriction and
// prolongation of every member that is at that level in its V-cycle.  The
// FP64 state of the members with the same top level (a "group") lives in
// group buffers; the borders' restriction chain and the prolongation of the
// new coefficients share the level-major FP64 planes B and C.
//
// Every member uses the general 7-point form (Coef, kind 2) on every level:
// its fine operator is assembled from its kappa and potential, coarser ones
// are Galerkin products; the member's own Gershgorin bound scales the
// Chebyshev b coefficients (bsc), the a coefficients do not depend on it.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>

#include "common.h"

namespace pasm {
namespace {

struct BLevel {
    Grid g;
    int count = 0;                   // members with this level: slots [0, count)
    double* c64[5] = {};             // wx, wy, -, d, wne: [count][plane]
    float* c32[5] = {};
    double* bsc64 = nullptr;         // [count] factor on b (1 / member bound, or 1)
    float* bsc32 = nullptr;
    std::vector<Cheb> pre, post;
    void* X = nullptr;               // [count * k][plane], V-cycle type
    void* Y = nullptr;
    void* F = nullptr;
    double* B = nullptr;             // [count * k][plane] FP64
    double* C = nullptr;
    int rows = 8;                    // smoothing tile (0: per step)
    double tune_ms[4] = {-1, -1, -1, -1};
};

struct BGroup {
    int top = 0;        // level index of the group's finest mesh
    int a = 0, b = 0;   // slots
    double* U = nullptr;      // [(b - a) * k][plane]
    double* F64 = nullptr;    // lambda M u
    double* partial = nullptr;
    int nblk = 0;
};

constexpr int kRowsCand[4] = {0, 2, 4, 8};

}  // namespace
}  // namespace pasm

using pasm::BGroup;
using pasm::BLevel;
using pasm::Cheb;
using pasm::Coef;
using pasm::Error;
using pasm::Grid;

struct pasm_batch {
    int n = 0, k = 0, nH = 0, NH = 0, Lmax = 0;
    pasm_options opt{};
    hipStream_t st = nullptr;
    bool own_stream = false;
    bool mixed = false;
    std::vector<int> slot_of, user_of;   // user index <-> slot
    std::vector<int> top;                // per slot: level index of the finest mesh
    std::vector<BLevel> lv;
    std::vector<BGroup> grp;
    std::vector<int> grp_of;             // per slot
    // coarse space, per slot
    double *theta = nullptr, *Qcm = nullptr, *Qrm = nullptr, *Ainv64 = nullptr;
    float* Ainv32 = nullptr;
    int* group = nullptr;
    // per eigenpair (slot-major, n * k)
    double *bz = nullptr, *pp = nullptr, *qq = nullptr, *ycoef = nullptr, *s = nullptr, *mu = nullptr;
    double *lam = nullptr, *lam_prev = nullptr, *score = nullptr, *stage = nullptr;
    int *rank = nullptr, *flags = nullptr;
    void* awork = nullptr;
    void* dmv = nullptr;
    std::vector<double> lam_h, lam_prev_h;
    std::vector<void*> allocs;
    rocblas_handle blas = nullptr;
    mutable std::string err;  // last failure (also set by read-only queries)
    // graph of one iteration's device work
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // profiling (finest batched level's smoothing phases)
    bool prof = false;
    std::vector<hipEvent_t> ev;
    std::vector<double> ev_bytes;
    size_t ev_used = 0;
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
    template <typename T>
    Coef<T> coef(int l) const;
    Coef<double> coef64_slots(int l, int a) const;
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
    }
};

template <>
Coef<double> pasm_batch::coef<double>(int l) const {
    const BLevel& L = lv[l];
    Coef<double> c;
    c.wx = L.c64[0];
    c.wy = L.c64[1];
    c.d = L.c64[3];
    c.wne = L.c64[4];
    c.ms = L.g.plane;
    c.kpm = k;
    c.bsc = L.bsc64;
    return c;
}
template <>
Coef<float> pasm_batch::coef<float>(int l) const {
    const BLevel& L = lv[l];
    Coef<float> c;
    c.wx = L.c32[0];
    c.wy = L.c32[1];
    c.d = L.c32[3];
    c.wne = L.c32[4];
    c.ms = L.g.plane;
    c.kpm = k;
    c.bsc = L.bsc32;
    return c;
}
// FP64 operator of level l for the members from slot a on
Coef<double> pasm_batch::coef64_slots(int l, int a) const {
    Coef<double> c = coef<double>(l);
    const long o = (long)a * lv[l].g.plane;
    c.wx += o;
    c.wy += o;
    c.d += o;
    c.wne += o;
    c.bsc = nullptr;
    return c;
}

namespace {

thread_local std::string g_batch_setup_error;

void brecord_start(pasm_batch* b) {
    if (!b->prof) return;
    if (b->ev_used + 2 > b->ev.size()) {
        hipEvent_t e0, e1;
        // timing only: no system-scope fence around the timed launches
        PASM_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
        PASM_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
        b->ev.push_back(e0);
        b->ev.push_back(e1);
        b->ev_bytes.push_back(0.0);
    }
    PASM_HIP(hipEventRecord(b->ev[b->ev_used], b->st));
}
void brecord_end(pasm_batch* b, double bytes) {
    if (!b->prof) return;
    PASM_HIP(hipEventRecord(b->ev[b->ev_used + 1], b->st));
    b->ev_bytes[b->ev_used / 2] = bytes;
    b->ev_used += 2;
}
void bcollect(pasm_batch* b) {
    if (!b->prof) return;
    for (size_t e = 0; e < b->ev_used; e += 2) {
        float ms = 0.f;
        PASM_HIP(hipEventElapsedTime(&ms, b->ev[e], b->ev[e + 1]));
        b->prof_ms += ms;
        b->prof_bytes += b->ev_bytes[e / 2];
        b->prof_launches += 1;
    }
    b->ev_used = 0;
}

// One smoothing phase at level l for the first nr right-hand sides; the
// iterate ends in x (x and y swap as the steps ping-pong).
template <typename T>
void bsmooth(pasm_batch* b, int l, T*& x, T*& y, const T* f, const std::vector<Cheb>& steps, bool x_zero, int nr,
             int rows) {
    if (steps.empty()) return;
    const BLevel& L = b->lv[l];
    const Coef<T> cf = b->coef<T>(l);
    const bool fine = (l == b->Lmax - 1) && b->prof;
    const double nodes = (double)L.g.interior() * nr;
    if (rows > 0) {
        pasm::SmoothSteps ss{};
        ss.s = (int)steps.size();
        for (size_t j = 0; j < steps.size(); ++j) {
            ss.a[j] = steps[j].a;
            ss.b[j] = steps[j].b;
        }
        if (fine) brecord_start(b);
        const bool ok = pasm::launch_smooth_fused<T>(L.g, cf, x, f, y, nr, L.g.plane, ss, x_zero, b->st, rows);
        if (!ok) throw Error(PASM_E_INVALID, "smoothing tile not applicable to this level");
        // read x_0 (unless zero) and f, write x_s, plus four coefficient planes per member
        if (fine) brecord_end(b, ((x_zero ? 2.0 : 3.0) * nodes + 4.0 * nodes / b->k) * sizeof(T));
        std::swap(x, y);
        return;
    }
    for (size_t j = 0; j < steps.size(); ++j) {
        const bool z = x_zero && j == 0;
        const int zmode = (z ? 1 : 0) | ((x_zero && j == 1) ? 2 : 0);
        if (fine) brecord_start(b);
        pasm::launch_smooth<T>(L.g, cf, x, y, f, y, nr, L.g.plane, steps[j], zmode, b->st);
        if (fine) {
            const double words = 2.0 + (z ? 0.0 : 1.0) + (steps[j].a != 0.0 && !z && !(zmode & 2) ? 1.0 : 0.0);
            brecord_end(b, (words * nodes + 4.0 * nodes / b->k) * sizeof(T));
        }
        std::swap(x, y);
    }
}

template <typename T>
const T* bainv(const pasm_batch* b);
template <>
const double* bainv<double>(const pasm_batch* b) { return b->Ainv64; }
template <>
const float* bainv<float>(const pasm_batch* b) { return b->Ainv32; }

// Levels of 128 cells and more in FP32 with fused smoothing march (both
// phases need at least one step): every member's right-hand sides in one
// launch per phase, the member's coefficient planes and smoothing scale
// picked per pair of right-hand sides.
template <typename T>
bool bmarch(const pasm_batch* b, int l) {
    if constexpr (!std::is_same<T, float>::value) {
        return false;
    } else {
        const BLevel& Lv = b->lv[l];
        return b->opt.fused_smoothing && b->lv[l - 1].g.n * 2 == Lv.g.n &&
               pasm::march_coef_supported(Lv.g, b->coef<float>(l), (int)Lv.pre.size()) &&
               pasm::march_coef_supported(Lv.g, b->coef<float>(l), (int)Lv.post.size());
    }
}

// Coefficient planes per member the smoothers read: the two edge-weight
// planes, or four with the diagonal and the diagonal couplings.
double bcoef_planes(const pasm_batch* b) { return b->lv.back().c64[3] ? 4.0 : 2.0; }

pasm::SmoothSteps to_steps(const std::vector<Cheb>& v) {
    pasm::SmoothSteps ss{};
    ss.s = (int)v.size();
    for (size_t j = 0; j < v.size() && j < 8; ++j) {
        ss.a[j] = v[j].a;
        ss.b[j] = v[j].b;
    }
    return ss;
}

// One V-cycle from zero for every member on the right-hand sides already in
// the levels' F planes (each member's top-level residual, written by
// bresidual); the correction ends in the returned pointer of each level.
template <typename T>
std::vector<T*> bvcycle(pasm_batch* b) {
    const int L = b->Lmax, k = b->k;
    std::vector<T*> cur(L), oth(L);
    for (int l = 0; l < L; ++l) {
        cur[l] = static_cast<T*>(b->lv[l].X);
        oth[l] = static_cast<T*>(b->lv[l].Y);
    }
    for (int l = L - 1; l >= 1; --l) {
        BLevel& Lv = b->lv[l];
        const int nr = Lv.count * k;
        const T* f = static_cast<const T*>(Lv.F);
        const BLevel& Lc = b->lv[l - 1];
        if (bmarch<T>(b, l)) {
            // marching pre-smoothing from zero with the residual restriction
            // to every member's coarse right-hand side
            const bool fine = (l == b->Lmax - 1) && b->prof;
            const double nodes = (double)Lv.g.interior() * nr;
            if (fine) brecord_start(b);
            pasm::launch_march_pre_ew(Lv.g, b->coef<float>(l), reinterpret_cast<const float*>(cur[l]),
                                      reinterpret_cast<const float*>(f), reinterpret_cast<float*>(oth[l]), Lc.g,
                                      static_cast<float*>(Lc.F), nr, to_steps(Lv.pre), true, b->st);
            if (fine) brecord_end(b, (2.25 * nodes + bcoef_planes(b) * nodes / b->k) * sizeof(T));
            std::swap(cur[l], oth[l]);
            continue;
        }
        bsmooth<T>(b, l, cur[l], oth[l], f, Lv.pre, true, nr, Lv.rows);
        if (Lv.pre.empty())
            pasm::launch_restrict<T>(Lv.g, f, Lc.g, static_cast<T*>(Lc.F), nr, Lv.g.plane, Lc.g.plane, b->st);
        else
            pasm::launch_resid_restrict<T>(Lv.g, b->coef<T>(l), cur[l], f, Lc.g, static_cast<T*>(Lc.F), nr,
                                           Lv.g.plane, Lc.g.plane, b->st);
    }
    const BLevel& L0 = b->lv[0];
    pasm::launch_dense_mv<T>(bainv<T>(b), b->NH, L0.g, static_cast<const T*>(L0.F), L0.g.plane, true, cur[0],
                             L0.g.plane, true, L0.count * k, b->dmv, b->st, k, (long)b->NH * b->NH);
    for (int l = 1; l < L; ++l) {
        BLevel& Lv = b->lv[l];
        const BLevel& Lc = b->lv[l - 1];
        const int nr = Lv.count * k;
        if (bmarch<T>(b, l)) {
            // marching post-smoothing whose x_0 = x + P e_c is formed in the pass
            const bool fine = (l == b->Lmax - 1) && b->prof;
            const double nodes = (double)Lv.g.interior() * nr;
            if (fine) brecord_start(b);
            pasm::launch_march_post_ew(Lv.g, b->coef<float>(l), reinterpret_cast<const float*>(cur[l]),
                                       static_cast<const float*>(Lv.F), reinterpret_cast<float*>(oth[l]), Lc.g,
                                       reinterpret_cast<const float*>(cur[l - 1]), nr, to_steps(Lv.post), b->st);
            if (fine) brecord_end(b, (3.25 * nodes + bcoef_planes(b) * nodes / b->k) * sizeof(T));
            std::swap(cur[l], oth[l]);
            continue;
        }
        // x = 0 after pre-smoothing only when there is none: then x = P e_c
        pasm::launch_prolong<T>(Lc.g, cur[l - 1], Lv.g, cur[l], nr, Lc.g.plane, Lv.g.plane, !Lv.pre.empty(),
                                nullptr, b->st);
        bsmooth<T>(b, l, cur[l], oth[l], static_cast<const T*>(Lv.F), Lv.post, false, nr, Lv.rows);
    }
    return cur;
}

// r = f - A u at every group's top level, into the level's F planes
template <typename T>
void bresidual(pasm_batch* b) {
    const int k = b->k;
    for (const BGroup& G : b->grp) {
        const BLevel& Lv = b->lv[G.top];
        T* f = static_cast<T*>(Lv.F) + (long)G.a * k * Lv.g.plane;
        pasm::launch_resid_to<T>(Lv.g, b->coef64_slots(G.top, G.a), G.U, G.F64, f, (G.b - G.a) * k, Lv.g.plane,
                                 b->st);
    }
}

template <typename T>
void bcorrect(pasm_batch* b, const std::vector<T*>& cur) {
    const int k = b->k;
    for (const BGroup& G : b->grp) {
        const BLevel& Lv = b->lv[G.top];
        const T* e = cur[G.top] + (long)G.a * k * Lv.g.plane;
        pasm::launch_add_correction(e, G.U, (long)(G.b - G.a) * k * Lv.g.plane, b->st);
    }
}

// u = P Q y' (+ s u when s != nullptr) for every member
// coarse_ready: Q y' is already in the coarse level's B.
void bprolong_coefs(pasm_batch* b, const double* s, bool coarse_ready = false) {
    const int k = b->k, N = b->NH, L = b->Lmax;
    const BLevel& L0 = b->lv[0];
    if (!coarse_ready)
        pasm::launch_dense_mv<double>(b->Qcm, N, L0.g, b->ycoef, N, false, L0.B, L0.g.plane, true, b->n * k, b->dmv,
                                      b->st, k, (long)N * N);
    for (int l = 1; l < L; ++l) {
        const BLevel& Lv = b->lv[l];
        const BLevel& Lc = b->lv[l - 1];
        const int deeper = (l + 1 < L) ? b->lv[l + 1].count : 0;  // members whose top is above l
        if (deeper > 0)
            pasm::launch_prolong<double>(Lc.g, Lc.B, Lv.g, Lv.B, deeper * k, Lc.g.plane, Lv.g.plane, false, nullptr,
                                         b->st);
        for (const BGroup& G : b->grp) {
            if (G.top != l) continue;
            const double* src = Lc.B + (long)G.a * k * Lc.g.plane;
            pasm::launch_prolong<double>(Lc.g, src, Lv.g, G.U, (G.b - G.a) * k, Lc.g.plane, Lv.g.plane, false,
                                         s ? s + (long)G.a * k : nullptr, b->st);
        }
    }
}

// Mixed precision with two V-cycles on 2D members with coefficient planes:
// f = lambda M u is never stored.  The first residual is formed from u, the
// first correction and the second residual in one pass (u + e into the f
// buffer, u kept), and the second correction inside the border pass, which
// writes u~ back into u.
bool bfused_defect(const pasm_batch* b) {
    if (!b->mixed || b->opt.vcycles != 2) return false;
    const int kind = pasm::coef_kind(b->coef<double>(b->Lmax - 1));
    if (kind != 1 && kind != 2) return false;
    for (const BGroup& G : b->grp)
        if (G.top < 1) return false;
    return true;
}

// The device work of one correction step for every member.
void biterate_device(pasm_batch* b) {
    const int k = b->k, N = b->NH, L = b->Lmax;
    if (bfused_defect(b)) {
        // Algorithm 1, step 1 as defect correction: r = lambda M u - A u
        for (const BGroup& G : b->grp) {
            const BLevel& Lv = b->lv[G.top];
            float* r = static_cast<float*>(Lv.F) + (long)G.a * k * Lv.g.plane;
            pasm::launch_resid_mass_members(Lv.g, b->coef64_slots(G.top, G.a), G.U, b->lam + (long)G.a * k, r,
                                            (G.b - G.a) * k, Lv.g.plane, b->st);
        }
        std::vector<float*> cur = bvcycle<float>(b);
        // x = u + e (into the f buffer) and r = lambda M u - A x
        for (const BGroup& G : b->grp) {
            const BLevel& Lv = b->lv[G.top];
            const long o = (long)G.a * k * Lv.g.plane;
            pasm::launch_add_resid_members(Lv.g, b->coef64_slots(G.top, G.a), G.U, cur[G.top] + o, G.F64,
                                           static_cast<float*>(Lv.F) + o, (G.b - G.a) * k, Lv.g.plane,
                                           b->lam + (long)G.a * k, b->st);
        }
        cur = bvcycle<float>(b);
        // step 2: u~ = x + e into u, with the borders and their first
        // restriction (P^T A u~, P^T M u~ in the B and C planes one level
        // below each group's top)
        for (const BGroup& G : b->grp) {
            const BLevel& Lv = b->lv[G.top];
            const BLevel& Lc = b->lv[G.top - 1];
            const long oc = (long)G.a * k * Lc.g.plane;
            const int nblk = pasm::launch_border_restrict_add(
                Lv.g, b->coef64_slots(G.top, G.a), G.F64, cur[G.top] + (long)G.a * k * Lv.g.plane, G.U, Lc.g,
                Lc.B + oc, Lc.C + oc, G.partial, (G.b - G.a) * k, Lv.g.plane, Lc.g.plane, b->st);
            pasm::launch_reduce_pairs(G.partial, nblk, b->bz + 2L * G.a * k, (G.b - G.a) * k, b->st);
        }
    } else {
        // Algorithm 1, step 1: f = lambda M u, V-cycles (defect correction)
        for (const BGroup& G : b->grp) {
            const Grid& g = b->lv[G.top].g;
            pasm::launch_mass_rhs(g, G.U, b->lam + (long)G.a * k, G.F64, (G.b - G.a) * k, g.plane, b->st);
        }
        for (int cy = 0; cy < b->opt.vcycles; ++cy) {
            if (b->mixed) {
                bresidual<float>(b);
                bcorrect<float>(b, bvcycle<float>(b));
            } else {
                bresidual<double>(b);
                bcorrect<double>(b, bvcycle<double>(b));
            }
        }
        // step 2: borders fused with the first restriction: P^T A u~ and
        // P^T M u~ of every group land in the B and C planes one level below
        // its top
        for (const BGroup& G : b->grp) {
            const BLevel& Lv = b->lv[G.top];
            const BLevel& Lc = b->lv[G.top - 1];
            const long o = (long)G.a * k * Lc.g.plane;
            const int nblk = pasm::launch_border_restrict(Lv.g, b->coef64_slots(G.top, G.a), G.U, Lc.g, Lc.B + o,
                                                          Lc.C + o, G.partial, (G.b - G.a) * k, Lv.g.plane,
                                                          Lc.g.plane, b->st);
            pasm::launch_reduce_pairs(G.partial, nblk, b->bz + 2L * G.a * k, (G.b - G.a) * k, b->st);
        }
    }
    // the chain continues for the members whose top is at least two levels up
    for (int l = L - 3; l >= 0; --l) {
        const BLevel& Lf = b->lv[l + 1];
        const BLevel& Lc = b->lv[l];
        const int nr = b->lv[l + 2].count * k;
        if (nr == 0) continue;
        pasm::launch_restrict<double>(Lf.g, Lf.B, Lc.g, Lc.B, nr, Lf.g.plane, Lc.g.plane, b->st);
        pasm::launch_restrict<double>(Lf.g, Lf.C, Lc.g, Lc.C, nr, Lf.g.plane, Lc.g.plane, b->st);
    }
    const BLevel& L0 = b->lv[0];
    const int nk = b->n * k;
    pasm::launch_dense_mv<double>(b->Qrm, N, L0.g, L0.B, L0.g.plane, true, b->pp, N, false, nk, b->dmv, b->st, k,
                                  (long)N * N);
    pasm::launch_dense_mv<double>(b->Qrm, N, L0.g, L0.C, L0.g.plane, true, b->qq, N, false, nk, b->dmv, b->st, k,
                                  (long)N * N);
    pasm::ArrowIn in{b->theta, b->group, b->pp, b->qq, b->bz, b->lam, N, b->opt.exhaustive_selection, k};
    pasm::ArrowOut out{b->ycoef, b->s, b->mu, b->rank, b->score, b->flags, static_cast<double*>(b->awork)};
    pasm::launch_arrowhead(in, out, nk, b->st);
    bprolong_coefs(b, b->s);
    pasm::launch_copy(b->lam, b->lam_prev, nk, b->st);
    pasm::launch_copy(b->mu, b->lam, nk, b->st);
}

// Time every applicable tile height on each level (pre-smoothing from zero
// plus post-smoothing, the same launches as in a V-cycle) and keep the
// fastest.
template <typename T>
void btune(pasm_batch* b) {
    hipEvent_t e0, e1;
    PASM_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    PASM_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    for (int l = 1; l < b->Lmax; ++l) {
        BLevel& Lv = b->lv[l];
        const int nr = Lv.count * b->k;
        double best = 1e300;
        int best_rows = 0;
        for (int ci = 0; ci < 4; ++ci) {
            const int rows = pasm::kRowsCand[ci];
            Lv.tune_ms[ci] = -1.0;
            if (rows > 0) {
                const size_t lds = pasm::fused_lds_bytes(2, sizeof(T), rows);
                const int smax = (int)std::max(Lv.pre.size(), Lv.post.size());
                if (lds > 65536 || 4 * rows - 2 * smax <= 0 || smax > 4) continue;
            }
            float ms = 0.f;
            for (int rep = 0; rep < 4; ++rep) {
                T* x = static_cast<T*>(Lv.X);
                T* y = static_cast<T*>(Lv.Y);
                if (rep == 1) PASM_HIP(hipEventRecord(e0, b->st));
                bsmooth<T>(b, l, x, y, static_cast<const T*>(Lv.F), Lv.pre, true, nr, rows);
                bsmooth<T>(b, l, x, y, static_cast<const T*>(Lv.F), Lv.post, false, nr, rows);
            }
            PASM_HIP(hipEventRecord(e1, b->st));
            PASM_HIP(hipEventSynchronize(e1));
            PASM_HIP(hipEventElapsedTime(&ms, e0, e1));
            Lv.tune_ms[ci] = ms / 3.0;
            if (Lv.tune_ms[ci] < best) {
                best = Lv.tune_ms[ci];
                best_rows = rows;
            }
        }
        Lv.rows = best_rows;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the timing runs wrote the V-cycle planes; clear them (never captured)
    for (auto& Lv : b->lv) {
        const size_t bytes = (size_t)Lv.count * b->k * Lv.g.plane * (b->mixed ? sizeof(float) : sizeof(double));
        PASM_HIP(hipMemsetAsync(Lv.X, 0, bytes, b->st));
        PASM_HIP(hipMemsetAsync(Lv.Y, 0, bytes, b->st));
    }
    PASM_HIP(hipStreamSynchronize(b->st));
}

struct BPlan {
    int nH, NH, Lmax;
    std::vector<int> nf, L;   // per user index
    size_t nel_of(int i) const { return 2 * (size_t)nf[i] * nf[i]; }
};

BPlan bvalidate(const pasm_options& opt, const pasm_domain* dom, const pasm_instance* inst, int n, double H, int k) {
    BPlan p{};
    if (!dom || dom->dim != 2) throw Error(PASM_E_INVALID, "batches are supported on the unit square (dim 2)");
    if (!inst || n < 1) throw Error(PASM_E_INVALID, "need n >= 1 instances");
    if (!(H > 0.0) || !std::isfinite(H)) throw Error(PASM_E_INVALID, "bad H");
    const double nHd = 1.0 / H;
    p.nH = (int)std::lround(nHd);
    if (std::fabs(nHd - p.nH) > 1e-9 * nHd || p.nH < 2 || p.nH > 200) throw Error(PASM_E_INVALID, "1/H must be an integer in [2, 200]");
    p.NH = (p.nH - 1) * (p.nH - 1);
    if (k < 1 || k >= p.NH) throw Error(PASM_E_INVALID, "need 1 <= k < N_H");
    if (opt.vcycles < 1 || opt.nu_pre < 0 || opt.nu_post < 0 || opt.max_iter < 1 || !(opt.tol >= 0.0))
        throw Error(PASM_E_INVALID, "bad cycle options");
    if (opt.nu_pre > 8 || opt.nu_post > 8) throw Error(PASM_E_INVALID, "at most 8 smoothing steps per phase");
    if (opt.precision != PASM_FP64 && opt.precision != PASM_MIXED) throw Error(PASM_E_INVALID, "bad precision");
    if (opt.smoother != PASM_JACOBI && opt.smoother != PASM_CHEBYSHEV) throw Error(PASM_E_INVALID, "bad smoother");
    p.Lmax = 0;
    for (int i = 0; i < n; ++i) {
        const double h = inst[i].h;
        if (!(h > 0.0) || !std::isfinite(h) || h >= H) throw Error(PASM_E_INVALID, "need 0 < h < H for every instance");
        const double nhd = 1.0 / h;
        const int nh = (int)std::lround(nhd);
        if (std::fabs(nhd - nh) > 1e-9 * nhd || nhd > 1e5) throw Error(PASM_E_INVALID, "1/h must be an integer");
        if (nh % p.nH != 0) throw Error(PASM_E_INVALID, "1/h must be a multiple of 1/H");
        int ratio = nh / p.nH, L = 1;
        while (ratio > 1) {
            if (ratio & 1) throw Error(PASM_E_INVALID, "H/h must be a power of two");
            ratio >>= 1;
            ++L;
        }
        p.nf.push_back(nh);
        p.L.push_back(L);
        p.Lmax = std::max(p.Lmax, L);
        const pasm_coefficients& c = inst[i].coef;
        const size_t nel = 2 * (size_t)nh * nh;
        if ((c.kappa || c.potential) && c.n_elements != nel)
            throw Error(PASM_E_INVALID, "n_elements does not match an instance's fine mesh");
        if (c.kappa)
            for (size_t e = 0; e < nel; ++e)
                if (!(c.kappa[e] > 0.0) || !std::isfinite(c.kappa[e]))
                    throw Error(PASM_E_INVALID, "kappa must be finite and positive");
        if (c.potential)
            for (size_t e = 0; e < nel; ++e)
                if (!(c.potential[e] >= 0.0) || !std::isfinite(c.potential[e]))
                    throw Error(PASM_E_INVALID, "potential must be finite and non-negative");
    }
    return p;
}

void bbuild(pasm_batch* b, const BPlan& pl, const pasm_instance* inst) {
    const int n = b->n, k = b->k;
    b->nH = pl.nH;
    b->NH = pl.NH;
    b->Lmax = pl.Lmax;
    b->mixed = b->opt.precision == PASM_MIXED;
    // slots: decreasing fine size, ties in user order
    b->user_of.resize(n);
    std::iota(b->user_of.begin(), b->user_of.end(), 0);
    std::stable_sort(b->user_of.begin(), b->user_of.end(), [&](int x, int y) { return pl.L[x] > pl.L[y]; });
    b->slot_of.assign(n, 0);
    for (int s = 0; s < n; ++s) b->slot_of[b->user_of[s]] = s;
    b->top.resize(n);
    for (int s = 0; s < n; ++s) b->top[s] = pl.L[b->user_of[s]] - 1;

    const double omega = b->opt.omega > 0 ? b->opt.omega : 0.8;
    const double alpha = b->opt.cheb_alpha > 0 ? b->opt.cheb_alpha : 4.0;
    const bool cheb = b->opt.smoother == PASM_CHEBYSHEV;
    const size_t tsz = b->mixed ? sizeof(float) : sizeof(double);

    b->lv.resize(b->Lmax);
    for (int l = 0; l < b->Lmax; ++l) {
        BLevel& Lv = b->lv[l];
        Lv.g = pasm::make_grid(2, b->nH << l);
        Lv.count = 0;
        for (int s = 0; s < n; ++s) Lv.count += (b->top[s] >= l) ? 1 : 0;
        const size_t planes = (size_t)Lv.count * Lv.g.plane;
        for (int a : {0, 1, 3, 4}) {
            Lv.c64[a] = b->alloc<double>(planes);
            if (b->mixed) Lv.c32[a] = b->alloc<float>(planes);
        }
        Lv.bsc64 = b->alloc<double>(Lv.count);
        if (b->mixed) Lv.bsc32 = b->alloc<float>(Lv.count);
        // Chebyshev steps for the bound 1: b_j scales as 1 / bound (a_j does not)
        Lv.pre = cheb ? pasm::cheb_steps(1.0, alpha, b->opt.nu_pre) : pasm::jacobi_steps(omega, b->opt.nu_pre);
        Lv.post = cheb ? pasm::cheb_steps(1.0, alpha, b->opt.nu_post) : pasm::jacobi_steps(omega, b->opt.nu_post);
        const size_t vec = (size_t)Lv.count * k * Lv.g.plane;
        Lv.X = b->mixed ? (void*)b->alloc<float>(vec) : (void*)b->alloc<double>(vec);
        Lv.Y = b->mixed ? (void*)b->alloc<float>(vec) : (void*)b->alloc<double>(vec);
        Lv.F = b->mixed ? (void*)b->alloc<float>(vec) : (void*)b->alloc<double>(vec);
        Lv.B = b->alloc<double>(vec);
        Lv.C = b->alloc<double>(vec);
        Lv.rows = (b->opt.fused_smoothing && pasm::fused_lds_bytes(2, tsz, 4) <= 65536) ? 4 : 0;
    }

    // per member operators on every level (host), coarse pencils
    const int N = b->NH;
    std::vector<double> AH_all((size_t)n * N * N), MH((size_t)N * N, 0.0);
    std::vector<std::vector<double>> bsc(b->Lmax, std::vector<double>());
    for (int l = 0; l < b->Lmax; ++l) bsc[l].assign(b->lv[l].count, 1.0);
    for (int s = 0; s < n; ++s) {
        const int u = b->user_of[s];
        const pasm_coefficients& c = inst[u].coef;
        const size_t nel = pl.nel_of(u);
        std::vector<double> kap, pot;
        if (c.kappa) kap.assign(c.kappa, c.kappa + nel);
        if (c.potential) pot.assign(c.potential, c.potential + nel);
        pasm::Stencil7 sten;
        for (int l = b->top[s]; l >= 0; --l) {
            BLevel& Lv = b->lv[l];
            sten = (l == b->top[s]) ? pasm::fine_stencil_2d(Lv.g, kap, pot)
                                    : pasm::galerkin_stencil_2d(b->lv[l + 1].g, sten, Lv.g);
            const long o = (long)s * Lv.g.plane;
            const std::vector<double>* arr[5] = {&sten.wx, &sten.wy, nullptr, &sten.d, &sten.wne};
            for (int a : {0, 1, 3, 4})
                PASM_HIP(hipMemcpyAsync(Lv.c64[a] + o, arr[a]->data(), Lv.g.plane * sizeof(double),
                                        hipMemcpyHostToDevice, b->st));
            PASM_HIP(hipStreamSynchronize(b->st));
            if (cheb) bsc[l][s] = 1.0 / pasm::gershgorin_2d(Lv.g, sten);
            if (l == 0) {
                std::vector<double> AH;
                pasm::dense_from_stencil_2d(Lv.g, sten, AH);
                std::copy(AH.begin(), AH.end(), AH_all.begin() + (size_t)s * N * N);
            }
        }
    }
    for (int l = 0; l < b->Lmax; ++l) {
        BLevel& Lv = b->lv[l];
        PASM_HIP(hipMemcpyAsync(Lv.bsc64, bsc[l].data(), Lv.count * sizeof(double), hipMemcpyHostToDevice, b->st));
        if (b->mixed) {
            for (int a : {0, 1, 3, 4}) pasm::launch_d2f(Lv.c64[a], Lv.c32[a], (long)Lv.count * Lv.g.plane, b->st);
            pasm::launch_d2f(Lv.bsc64, Lv.bsc32, Lv.count, b->st);
        }
    }
    // coarse mass (the same for every member): h^2 (1/2 centre, 1/12 at E, W, N, S, NE, SW)
    {
        const Grid& g0 = b->lv[0].g;
        const int m = g0.m;
        const double H2 = g0.h * g0.h;
        for (int j = 1; j <= m; ++j)
            for (int i = 1; i <= m; ++i) {
                const long r = (long)(j - 1) * m + (i - 1);
                MH[(size_t)r * N + r] = 0.5 * H2;
                const int mb[6][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}};
                for (int t = 0; t < 6; ++t) {
                    const int i2 = i + mb[t][0], j2 = j + mb[t][1];
                    if (i2 < 1 || j2 < 1 || i2 > m || j2 > m) continue;
                    MH[(size_t)((j2 - 1) * m + (i2 - 1)) * N + r] = H2 / 12.0;
                }
            }
    }
    const size_t NN = (size_t)N * N;
    b->theta = b->alloc<double>((size_t)n * N);
    b->Qcm = b->alloc<double>(n * NN);
    b->Qrm = b->alloc<double>(n * NN);
    b->Ainv64 = b->alloc<double>(n * NN);
    if (b->mixed) b->Ainv32 = b->alloc<float>(n * NN);
    b->group = b->alloc<int>((size_t)n * N);
    if (rocblas_create_handle(&b->blas) != rocblas_status_success)
        throw Error(PASM_E_DEVICE, "rocblas_create_handle failed");
    rocblas_set_stream(b->blas, b->st);
    double* dB = b->alloc<double>(NN);
    double* dE = b->alloc<double>(N);
    int* dInfo = b->alloc<int>(1);
    std::vector<double> th(N);
    std::vector<int> grp(N);
    b->lam_h.assign((size_t)n * k, 0.0);
    for (int s = 0; s < n; ++s) {
        double* dA = b->Qcm + s * NN;
        double* th_s = b->theta + (size_t)s * N;
        PASM_HIP(hipMemcpyAsync(dA, AH_all.data() + s * NN, NN * sizeof(double), hipMemcpyHostToDevice, b->st));
        PASM_HIP(hipMemcpyAsync(dB, MH.data(), NN * sizeof(double), hipMemcpyHostToDevice, b->st));
        if (rocsolver_dsygvd(b->blas, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper, N, dA, N, dB, N,
                             th_s, dE, dInfo) != rocblas_status_success)
            throw Error(PASM_E_DEVICE, "rocsolver_dsygvd failed");
        int info = 0;
        PASM_HIP(hipMemcpyAsync(&info, dInfo, sizeof(int), hipMemcpyDeviceToHost, b->st));
        PASM_HIP(hipMemcpyAsync(th.data(), th_s, N * sizeof(double), hipMemcpyDeviceToHost, b->st));
        PASM_HIP(hipStreamSynchronize(b->st));
        if (info != 0) throw Error(PASM_E_DEVICE, "coarse generalized eigensolve did not converge");
        pasm::launch_transpose(dA, b->Qrm + s * NN, N, b->st);
        pasm::launch_scale_cols(dA, th_s, dB, N, b->st);
        const double one = 1.0, zero = 0.0;
        if (rocblas_dgemm(b->blas, rocblas_operation_none, rocblas_operation_transpose, N, N, N, &one, dB, N, dA, N,
                          &zero, b->Ainv64 + s * NN, N) != rocblas_status_success)
            throw Error(PASM_E_DEVICE, "rocblas_dgemm failed");
        const double gtol = 16.0 * DBL_EPSILON * std::fabs(th[N - 1]);
        for (int j = 0; j < N; ++j) grp[j] = (j > 0 && th[j] - th[j - 1] <= gtol) ? grp[j - 1] : j;
        PASM_HIP(hipMemcpyAsync(b->group + (size_t)s * N, grp.data(), N * sizeof(int), hipMemcpyHostToDevice, b->st));
        PASM_HIP(hipStreamSynchronize(b->st));
        for (int i = 0; i < k; ++i) b->lam_h[(size_t)s * k + i] = th[i];
    }
    if (b->mixed) pasm::launch_d2f(b->Ainv64, b->Ainv32, (long)(n * NN), b->st);
    b->lam_prev_h = b->lam_h;

    // groups of equal top level (contiguous slots)
    for (int s = 0; s < n;) {
        int e = s;
        while (e < n && b->top[e] == b->top[s]) ++e;
        BGroup G;
        G.top = b->top[s];
        G.a = s;
        G.b = e;
        const Grid& g = b->lv[G.top].g;
        const size_t vec = (size_t)(e - s) * k * g.plane;
        G.U = b->alloc<double>(vec);
        G.F64 = b->alloc<double>(vec);
        G.nblk = ((g.m + 63) / 64) * ((g.m + 3) / 4);
        G.partial = b->alloc<double>(2 * (size_t)G.nblk * (e - s) * k);
        b->grp.push_back(G);
        s = e;
    }
    b->grp_of.assign(n, 0);
    for (size_t gi = 0; gi < b->grp.size(); ++gi)
        for (int s = b->grp[gi].a; s < b->grp[gi].b; ++s) b->grp_of[s] = (int)gi;

    const size_t nk = (size_t)n * k;
    b->bz = b->alloc<double>(2 * nk);
    b->pp = b->alloc<double>(nk * N);
    b->qq = b->alloc<double>(nk * N);
    b->ycoef = b->alloc<double>(nk * N);
    b->s = b->alloc<double>(nk);
    b->mu = b->alloc<double>(nk);
    b->lam = b->alloc<double>(nk);
    b->lam_prev = b->alloc<double>(nk);
    b->score = b->alloc<double>(nk);
    b->rank = b->alloc<int>(nk);
    b->flags = b->alloc<int>(nk);
    b->awork = b->alloc<char>(pasm::arrow_workspace_bytes(N, (int)nk));
    b->dmv = b->alloc<char>(pasm::dense_mv_workspace_bytes(N, (int)nk));
    size_t maxdofs = 0;
    for (int s = 0; s < n; ++s) maxdofs = std::max(maxdofs, (size_t)b->lv[b->top[s]].g.interior());
    b->stage = b->alloc<double>(maxdofs * k);
    PASM_HIP(hipStreamSynchronize(b->st));
}

void brestart(pasm_batch* b) {
    const int nk = b->n * b->k, N = b->NH;
    // lambda = lambda_prev = theta_i per member, unit coefficients, and q_i
    // itself as the coarse vector Q e_i, in one launch
    const BLevel& L0 = b->lv[0];
    pasm::launch_restart_coarse(b->Qcm, N, L0.g, L0.B, L0.g.plane, b->ycoef, nk, b->k, (long)N * N, b->theta, N,
                                b->lam, b->lam_prev, b->st);
    bprolong_coefs(b, nullptr, true);
    PASM_HIP(hipMemcpyAsync(b->lam_h.data(), b->lam, nk * sizeof(double), hipMemcpyDeviceToHost, b->st));
    PASM_HIP(hipStreamSynchronize(b->st));
    b->lam_prev_h = b->lam_h;
}

void bset_error(const pasm_batch* b, const std::string& m) {
    if (b) b->err = m;
}

}  // namespace

#define PASM_BTRY(b, ...)                                          \
    try {                                                          \
        __VA_ARGS__;                                               \
    } catch (const Error& e_) {                                    \
        bset_error(b, e_.msg);                                     \
        return e_.status;                                          \
    } catch (const std::exception& e_) {                           \
        bset_error(b, e_.what());                                  \
        return PASM_E_DEVICE;                                      \
    }

extern "C" {

PASM_API pasm_status pasm_batch_destroy(pasm_batch* b) {
    if (!b) return PASM_OK;
    if (b->st) (void)hipStreamSynchronize(b->st);
    b->drop_graph();
    for (void* p : b->allocs) (void)hipFree(p);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    if (b->blas) rocblas_destroy_handle(b->blas);
    if (b->own_stream && b->st) (void)hipStreamDestroy(b->st);
    delete b;
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_setup(pasm_batch** out, const pasm_domain* dom, const pasm_instance* inst, int n,
                                      double H, int k, const pasm_options* opt) {
    if (!out) return PASM_E_INVALID;
    *out = nullptr;
    pasm_batch* b = new (std::nothrow) pasm_batch();
    if (!b) return PASM_E_NOMEM;
    if (opt) b->opt = *opt;
    else pasm_default_options(&b->opt);
    try {
        const BPlan pl = bvalidate(b->opt, dom, inst, n, H, k);
        b->n = n;
        b->k = k;
        if (b->opt.stream) b->st = static_cast<hipStream_t>(b->opt.stream);
        else {
            PASM_HIP(hipStreamCreate(&b->st));
            b->own_stream = true;
        }
        bbuild(b, pl, inst);
        if (b->opt.fused_smoothing) {
            if (b->mixed) btune<float>(b);
            else btune<double>(b);
        }
        brestart(b);
    } catch (const Error& e) {
        g_batch_setup_error = e.msg;
        pasm_batch_destroy(b);
        return e.status;
    } catch (const std::exception& e) {
        g_batch_setup_error = e.what();
        pasm_batch_destroy(b);
        return PASM_E_DEVICE;
    }
    *out = b;
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_iterate(pasm_batch* b, int* converged) {
    if (!b || b->n == 0) return PASM_E_STATE;
    PASM_BTRY(b, {
        const int nk = b->n * b->k;
        if (b->use_graph && !b->prof) {
            if (!b->gexec) {
                PASM_HIP(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
                try {
                    biterate_device(b);
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(b->st, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                PASM_HIP(hipStreamEndCapture(b->st, &b->graph));
                PASM_HIP(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
            }
            PASM_HIP(hipGraphLaunch(b->gexec, b->st));
        } else {
            biterate_device(b);
        }
        b->lam_prev_h = b->lam_h;
        PASM_HIP(hipMemcpyAsync(b->lam_h.data(), b->lam, nk * sizeof(double), hipMemcpyDeviceToHost, b->st));
        PASM_HIP(hipStreamSynchronize(b->st));
        bcollect(b);
        double dmax = 0.0;
        bool finite = true;
        for (int i = 0; i < nk; ++i) {
            const double l = b->lam_h[i];
            if (!std::isfinite(l)) finite = false;
            dmax = std::max(dmax, std::fabs(l - b->lam_prev_h[i]) / std::fabs(l));
        }
        if (!finite) {
            bset_error(b, "non-finite eigenvalue");
            return PASM_E_BREAKDOWN;
        }
        if (converged) *converged = dmax < b->opt.tol ? 1 : 0;
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_restart(pasm_batch* b) {
    if (!b || b->n == 0) return PASM_E_STATE;
    PASM_BTRY(b, brestart(b));
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_solve(pasm_batch* b, int* iterations) {
    if (!b || b->n == 0) return PASM_E_STATE;
    int it = 0, conv = 0;
    while (it < b->opt.max_iter) {
        const pasm_status s = pasm_batch_iterate(b, &conv);
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

PASM_API size_t pasm_batch_num_dofs(const pasm_batch* b, int member) {
    if (!b || member < 0 || member >= b->n) return 0;
    return (size_t)b->lv[b->top[b->slot_of[member]]].g.interior();
}

PASM_API int pasm_batch_num_levels(const pasm_batch* b) { return b ? b->Lmax : 0; }

PASM_API pasm_status pasm_batch_eigenpairs(const pasm_batch* b, int member, double* lambda, double* U, size_t ldu) {
    if (!b || b->n == 0) return PASM_E_STATE;
    if (member < 0 || member >= b->n) return PASM_E_INVALID;
    const int s = b->slot_of[member];
    const BGroup& G = b->grp[b->grp_of[s]];
    const Grid& g = b->lv[G.top].g;
    const size_t N = (size_t)g.interior();
    if (U && ldu < N) return PASM_E_INVALID;
    PASM_BTRY(b, {
        if (lambda) std::memcpy(lambda, b->lam_h.data() + (size_t)s * b->k, b->k * sizeof(double));
        if (U) {
            const double* src = G.U + (long)(s - G.a) * b->k * g.plane;
            pasm::launch_pack<double>(g, src, g.plane, b->stage, (long)N, b->k, b->st);
            PASM_HIP(hipMemcpy2DAsync(U, ldu * sizeof(double), b->stage, N * sizeof(double), N * sizeof(double), b->k,
                                      hipMemcpyDeviceToHost, b->st));
            PASM_HIP(hipStreamSynchronize(b->st));
        }
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_set_state(pasm_batch* b, int member, const double* lambda, const double* U,
                                          size_t ldu) {
    if (!b || b->n == 0) return PASM_E_STATE;
    if (member < 0 || member >= b->n || !lambda || !U) return PASM_E_INVALID;
    const int s = b->slot_of[member];
    const BGroup& G = b->grp[b->grp_of[s]];
    const Grid& g = b->lv[G.top].g;
    const size_t N = (size_t)g.interior();
    if (ldu < N) return PASM_E_INVALID;
    for (int i = 0; i < b->k; ++i)
        if (!std::isfinite(lambda[i])) return PASM_E_INVALID;
    // non-finite vector entries are refused here, before any kernel sees them
    for (int i = 0; i < b->k; ++i)
        for (size_t j = 0; j < N; ++j)
            if (!std::isfinite(U[(size_t)i * ldu + j])) {
                bset_error(b, "pasm_batch_set_state: U holds a non-finite value");
                return PASM_E_INVALID;
            }
    PASM_BTRY(b, {
        const size_t o = (size_t)s * b->k;
        std::copy(lambda, lambda + b->k, b->lam_h.begin() + o);
        std::copy(lambda, lambda + b->k, b->lam_prev_h.begin() + o);
        PASM_HIP(hipMemcpyAsync(b->lam + o, lambda, b->k * sizeof(double), hipMemcpyHostToDevice, b->st));
        PASM_HIP(hipMemcpyAsync(b->lam_prev + o, lambda, b->k * sizeof(double), hipMemcpyHostToDevice, b->st));
        PASM_HIP(hipMemcpy2DAsync(b->stage, N * sizeof(double), U, ldu * sizeof(double), N * sizeof(double), b->k,
                                  hipMemcpyHostToDevice, b->st));
        double* dst = G.U + (long)(s - G.a) * b->k * g.plane;
        pasm::launch_unpack<double>(g, b->stage, (long)N, dst, g.plane, b->k, b->st);
        PASM_HIP(hipStreamSynchronize(b->st));
    });
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_use_graph(pasm_batch* b, int enable) {
    if (!b) return PASM_E_STATE;
    b->use_graph = enable != 0;
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_tuning(const pasm_batch* b, int* rows, double* times_ms) {
    if (!b || b->n == 0) return PASM_E_STATE;
    for (int l = 0; l < b->Lmax; ++l) {
        if (rows) rows[l] = l == 0 ? 0 : b->lv[l].rows;
        if (times_ms)
            for (int c = 0; c < 4; ++c) times_ms[4 * l + c] = l == 0 ? -1.0 : b->lv[l].tune_ms[c];
    }
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_set_tiles(pasm_batch* b, const int* rows) {
    if (!b || b->n == 0) return PASM_E_STATE;
    if (!rows) return PASM_E_INVALID;
    const size_t tsz = b->mixed ? sizeof(float) : sizeof(double);
    for (int l = 1; l < b->Lmax; ++l) {
        const int r = rows[l];
        if (r == 0) continue;
        const int smax = (int)std::max(b->lv[l].pre.size(), b->lv[l].post.size());
        if ((r != 2 && r != 4 && r != 8) || pasm::fused_lds_bytes(2, tsz, r) > 65536 || 4 * r - 2 * smax <= 0 ||
            smax > 4)
            return PASM_E_INVALID;
    }
    for (int l = 1; l < b->Lmax; ++l) b->lv[l].rows = rows[l];
    b->drop_graph();  // the recorded launches used the previous tiles
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_profile(pasm_batch* b, int kernel, int enable) {
    if (!b) return PASM_E_STATE;
    if (kernel != 0) return PASM_E_INVALID;
    b->prof = enable != 0;
    b->prof_launches = 0;
    b->prof_ms = 0.0;
    b->prof_bytes = 0.0;
    b->ev_used = 0;
    return PASM_OK;
}

PASM_API pasm_status pasm_batch_profile_read(pasm_batch* b, int kernel, long* launches, double* total_ms,
                                             double* bytes_per_launch) {
    if (!b) return PASM_E_STATE;
    if (kernel != 0) return PASM_E_INVALID;
    if (launches) *launches = b->prof_launches;
    if (total_ms) *total_ms = b->prof_ms;
    if (bytes_per_launch) *bytes_per_launch = b->prof_launches ? b->prof_bytes / b->prof_launches : 0.0;
    return PASM_OK;
}

PASM_API const char* pasm_batch_last_error(const pasm_batch* b) {
    return b ? b->err.c_str() : g_batch_setup_error.c_str();
}

}  // extern "C"
